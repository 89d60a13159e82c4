// Universal extension stencil and the per-cut-leaf pseudo-inverses.
//
// Section 3.2: the stencil of a cut square S is X = X_S u X_Sbar u G on the
// extension square Sbar (side 3h, centre of S).  The interpolation matrix of
// eq. (defA), A_{X,G} = Phi_{X,G} Phi_{G,G}^{-1}, is taken in the flat limit of
// the Gaussian basis, where it is the polynomial interpolant of total degree
// `deg` on G: A = P_X P_G^{-1} for the basis T_m(x) T_n(y), m + n <= deg.
// G is the set of Padua points of degree deg ((deg+1)(deg+2)/2 points, which
// are unisolvent for that space; 66 for deg = 10 as in the paper).
//
// Per cut leaf the least-squares operator A_{X^I,G}^+ is formed once per tree
// (the paper's "QR factorization on each cut square", Section 7) with a
// one-sided Jacobi SVD, which is accurate in relative terms even for the
// strongly ill-conditioned interior row sets that occur near the boundary.
#include <algorithm>
#include <cmath>
#include <vector>

#include "vfx_internal.h"

namespace vfx {

void padua_points(int deg, std::vector<double>& xy) {
  xy.clear();
  for (int j = 0; j <= deg; ++j)
    for (int k = 0; k <= deg + 1; ++k)
      if ((j + k) % 2 == 0) {
        xy.push_back(std::cos(j * M_PI / deg));
        xy.push_back(std::cos(k * M_PI / (deg + 1)));
      }
}

static void cheb_row(double x, int deg, double* T) {
  T[0] = 1.0;
  if (deg >= 1) T[1] = x;
  for (int m = 2; m <= deg; ++m) T[m] = 2 * x * T[m - 1] - T[m - 2];
}

// Solve M X = B (M: n x n, B: n x r, both row-major, overwritten) by LU with
// partial pivoting.  Returns false if M is singular.
static bool lu_solve(std::vector<double>& M, int n, std::vector<double>& B, int r) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(M[i * n + k]) > std::fabs(M[piv * n + k])) piv = i;
    if (M[piv * n + k] == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(M[k * n + j], M[piv * n + j]);
      for (int j = 0; j < r; ++j) std::swap(B[k * r + j], B[piv * r + j]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = M[i * n + k] / M[k * n + k];
      if (f == 0.0) continue;
      for (int j = k; j < n; ++j) M[i * n + j] -= f * M[k * n + j];
      for (int j = 0; j < r; ++j) B[i * r + j] -= f * B[k * r + j];
    }
  }
  for (int k = n - 1; k >= 0; --k)
    for (int j = 0; j < r; ++j) {
      double s = B[k * r + j];
      for (int i = k + 1; i < n; ++i) s -= M[k * n + i] * B[i * r + j];
      B[k * r + j] = s / M[k * n + k];
    }
  return true;
}

void build_stencil(Tables& T) {
  const int K = T.K, Kb = T.Kbar, deg = T.deg, nG = T.nG, nX = T.nX;
  T.stencil_xy.clear();
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) {
      T.stencil_xy.push_back(T.t[a] / 3.0);
      T.stencil_xy.push_back(T.t[b] / 3.0);
    }
  for (int a = 0; a < Kb; ++a)
    for (int b = 0; b < Kb; ++b) {
      T.stencil_xy.push_back(T.tbar[a]);
      T.stencil_xy.push_back(T.tbar[b]);
    }
  std::vector<double> G;
  padua_points(deg, G);
  T.stencil_xy.insert(T.stencil_xy.end(), G.begin(), G.end());
  // Vandermonde rows in the basis T_m(x) T_n(y), m + n <= deg
  std::vector<std::pair<int, int>> basis;
  for (int m = 0; m <= deg; ++m)
    for (int nn = 0; nn <= deg - m; ++nn) basis.push_back({m, nn});
  std::vector<double> Tx(deg + 1), Ty(deg + 1);
  auto vrow = [&](int k, double* row) {
    cheb_row(T.stencil_xy[2 * k], deg, Tx.data());
    cheb_row(T.stencil_xy[2 * k + 1], deg, Ty.data());
    for (int c = 0; c < nG; ++c) row[c] = Tx[basis[c].first] * Ty[basis[c].second];
  };
  // A P_G = P_X  <=>  P_G^T A^T = P_X^T
  std::vector<double> PGt((size_t)nG * nG), PXt((size_t)nG * nX);
  std::vector<double> row(nG);
  for (int g = 0; g < nG; ++g) {
    vrow(nX - nG + g, row.data());
    for (int c = 0; c < nG; ++c) PGt[c * nG + g] = row[c];
  }
  for (int k = 0; k < nX; ++k) {
    vrow(k, row.data());
    for (int c = 0; c < nG; ++c) PXt[(size_t)c * nX + k] = row[c];
  }
  lu_solve(PGt, nG, PXt, nX);  // PXt now holds A^T (nG x nX)
  T.A.assign((size_t)nX * nG, 0.0);
  for (int k = 0; k < nX; ++k)
    for (int c = 0; c < nG; ++c) T.A[(size_t)k * nG + c] = PXt[(size_t)c * nX + k];
  // the support rows are the identity by construction
  for (int g = 0; g < nG; ++g)
    for (int c = 0; c < nG; ++c) T.A[(size_t)(nX - nG + g) * nG + c] = (g == c) ? 1.0 : 0.0;
  T.AbarT.assign((size_t)nG * Kb * Kb, 0.0);
  for (int a = 0; a < Kb * Kb; ++a)
    for (int c = 0; c < nG; ++c) T.AbarT[(size_t)c * Kb * Kb + a] = T.A[(size_t)(T.n + a) * nG + c];
}

// One-sided Jacobi (Hestenes) SVD of a tall m x n matrix held by columns:
// U (m x n, column j at U + j*m) is orthogonalised in place, V (n x n)
// accumulates the rotations.
static void hestenes(double* U, int m, int n, double* V) {
  for (int i = 0; i < n * n; ++i) V[i] = 0.0;
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double* up = U + (size_t)p * m;
        double* uq = U + (size_t)q * m;
        double a = 0, b = 0, g = 0;
        for (int i = 0; i < m; ++i) {
          a += up[i] * up[i];
          b += uq[i] * uq[i];
          g += up[i] * uq[i];
        }
        if (g == 0.0 || std::fabs(g) <= tol * std::sqrt(a * b)) continue;
        rotated = true;
        const double zeta = (b - a) / (2 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1 + t * t), s = c * t;
        for (int i = 0; i < m; ++i) {
          const double x = up[i], y = uq[i];
          up[i] = c * x - s * y;
          uq[i] = s * x + c * y;
        }
        double* vp = V + (size_t)p * n;
        double* vq = V + (size_t)q * n;
        for (int i = 0; i < n; ++i) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
    if (!rotated) break;
  }
}

int pinv_jacobi(const double* A, int m, int n, double rel_cut, double* P) {
  // P (n x m) = pinv(A) for A (m x n) row-major.  Work on the tall
  // orientation: if m >= n use A, else use A^T and transpose at the end.
  const bool tall = m >= n;
  const int rows = tall ? m : n, cols = tall ? n : m;
  std::vector<double> U((size_t)rows * cols), V((size_t)cols * cols);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      if (tall)
        U[(size_t)j * rows + i] = A[(size_t)i * n + j];
      else
        U[(size_t)i * rows + j] = A[(size_t)i * n + j];
    }
  hestenes(U.data(), rows, cols, V.data());
  std::vector<double> sig(cols);
  double smax = 0;
  for (int j = 0; j < cols; ++j) {
    double s = 0;
    for (int i = 0; i < rows; ++i) s += U[(size_t)j * rows + i] * U[(size_t)j * rows + i];
    sig[j] = std::sqrt(s);
    smax = std::max(smax, sig[j]);
  }
  // M = pinv(M_tall) with M_tall = Utilde V^T (Utilde = U Sigma):
  // pinv = V Sigma^{-2} Utilde^T, shape cols x rows
  int rank = 0;
  std::vector<double> Q((size_t)cols * rows, 0.0);
  for (int j = 0; j < cols; ++j) {
    if (!(sig[j] > rel_cut * smax)) continue;
    ++rank;
    const double inv2 = 1.0 / (sig[j] * sig[j]);
    const double* uj = U.data() + (size_t)j * rows;
    const double* vj = V.data() + (size_t)j * cols;
    for (int r = 0; r < cols; ++r) {
      const double f = vj[r] * inv2;
      if (f == 0.0) continue;
      double* qr = Q.data() + (size_t)r * rows;
      for (int i = 0; i < rows; ++i) qr[i] += f * uj[i];
    }
  }
  // tall: P = Q (n x m).  wide: Q = pinv(A^T) (m x n), P = Q^T (n x m).
  for (int r = 0; r < n; ++r)
    for (int i = 0; i < m; ++i) P[(size_t)r * m + i] = tall ? Q[(size_t)r * rows + i] : Q[(size_t)i * rows + r];
  return rank;
}

}  // namespace vfx
