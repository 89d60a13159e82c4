// Universal tables of the volume FMM, built once per context on the host.
//
// All tables are expressed in units of the target box side h, so that a
// single table serves every level (log-kernel scaling:
// int_B log|x-y| g(y) dy = h^2 [ int_B^ log|x^-y^| g dy^ + log(h) int_B^ g dy^ ]).
//
// Near-field tables (list 1, Section 4: "computed using precomputed tables of
// integrals", limited by level restriction to 33 configurations):
//   near[c][j][i] = int_{S_c} log|x_i - y| l_j(y) dy
// for the K^2 target nodes x_i of the unit target box and the Lagrange basis
// l_j of the source box of configuration c.  The weakly singular integrals
// are computed by splitting the source square into the four triangles that
// join the target point to the square's edges (signed, so the target may lie
// outside), writing each triangle in (rho, s) coordinates - rho in [0,1] along
// the ray, s along the edge - where the area element is |d| rho drho ds and
// log|x-y| = log rho + log(d^2+s^2)/2.  The rho integral is exact for the
// polynomial part with Gauss-Legendre nodes and a log-weighted product rule;
// the s integral uses Gauss-Legendre panels graded geometrically towards the
// foot of the perpendicular (the near-singular point when d is small).
//
// Expansion operators (complex Laurent / Taylor series of the log kernel,
// the multipole and local expansions of the VFMM, with coefficients scaled
// by powers of the box side):
//   multipole of box (c, h): phi(z) = a_0 log(z-c) + sum_k a_k (h/(z-c))^k
//   local of box (c, h):     phi(z) = sum_l b_l ((z-c)/h)^l
//   V = Re(phi) / (2 pi).
#include <cmath>
#include <complex>
#include <algorithm>
#include <cstring>
#include <omp.h>

#include "vfx_internal.h"

namespace vfx {

using cplx = std::complex<double>;

void gauss_legendre(int q, double* x, double* w) {
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i < (q + 1) / 2; ++i) {
    long double z = cosl(pi * (i + 0.75L) / (q + 0.5L));
    long double dp = 1;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= q; ++k) {
        long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    long double p0 = 1, p1 = z;
    for (int k = 2; k <= q; ++k) {
      long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = q * (z * p1 - p0) / (z * z - 1);
    x[i] = (double)(-z);
    x[q - 1 - i] = (double)z;
    double ww = (double)(2.0L / ((1 - z * z) * dp * dp));
    w[i] = ww;
    w[q - 1 - i] = ww;
  }
}

// Gauss-Legendre nodes r on [0,1] with plain weights w and product weights wl
// for the weight log(r): sum_i wl_i phi(r_i) = int_0^1 log(r) phi(r) dr for
// polynomials phi of degree <= N-1.  Built from the shifted-Legendre
// expansion of phi and the moments int_0^1 log(r) P_k(2r-1) dr, which are
// -1 for k = 0 and (-1)^(k+1) / (k(k+1)) for k >= 1.
void log_product_rule(int N, double* r, double* w, double* wl) {
  std::vector<double> x(N), ww(N);
  gauss_legendre(N, x.data(), ww.data());
  std::vector<long double> P(N);
  for (int i = 0; i < N; ++i) {
    r[i] = 0.5 * (x[i] + 1.0);
    w[i] = 0.5 * ww[i];
    // Legendre P_k(x_i), k = 0..N-1 (x_i = 2 r_i - 1)
    P[0] = 1.0L;
    if (N > 1) P[1] = x[i];
    for (int k = 2; k < N; ++k) P[k] = ((2 * k - 1) * (long double)x[i] * P[k - 1] - (k - 1) * P[k - 2]) / k;
    long double acc = -1.0L;  // k = 0: (2k+1) mu_0 P_0 with mu_0 = -1
    for (int k = 1; k < N; ++k) {
      const long double mu = ((k % 2) ? 1.0L : -1.0L) / ((long double)k * (k + 1));
      acc += (2 * k + 1) * mu * P[k];
    }
    wl[i] = (double)(w[i] * acc);
  }
}

static void cheb_coef_matrix(int K, const std::vector<double>& t, std::vector<double>& C) {
  // C[a][j] = (2/K) T_a(t_j), row a = 0 halved: values -> coefficients
  C.assign(K * K, 0.0);
  for (int a = 0; a < K; ++a)
    for (int j = 0; j < K; ++j) {
      double th = std::acos(std::max(-1.0, std::min(1.0, t[j])));
      C[a * K + j] = (2.0 / K) * std::cos(a * th) * (a == 0 ? 0.5 : 1.0);
    }
}

int near_config_coarse_index(int ox2, int oy2) {
  // odd values in {-3,-1,1,3}, max(|.|) == 3
  if ((ox2 & 1) == 0 || (oy2 & 1) == 0) return -1;
  if (ox2 < -3 || ox2 > 3 || oy2 < -3 || oy2 > 3) return -1;
  if (std::abs(ox2) != 3 && std::abs(oy2) != 3) return -1;
  int a = (ox2 + 3) / 2, b = (oy2 + 3) / 2;  // 0..3
  static int map[16];
  static bool init = false;
  if (!init) {
    int k = 0;
    for (int i = 0; i < 16; ++i) {
      int aa = i / 4, bb = i % 4;
      bool inner = (aa == 1 || aa == 2) && (bb == 1 || bb == 2);
      map[i] = inner ? -1 : k++;
    }
    init = true;
  }
  return map[a * 4 + b];
}

int near_config_fine_index(int ox4, int oy4) { return near_config_coarse_index(ox4, oy4); }

void near_config_geometry(int c, double* ox, double* oy, double* side) {
  if (c < 9) {
    *ox = c / 3 - 1;
    *oy = c % 3 - 1;
    *side = 1.0;
    return;
  }
  int idx = (c < 21) ? c - 9 : c - 21;
  int k = 0;
  for (int i = 0; i < 16; ++i) {
    int aa = i / 4, bb = i % 4;
    bool inner = (aa == 1 || aa == 2) && (bb == 1 || bb == 2);
    if (inner) continue;
    if (k == idx) {
      int o1 = 2 * aa - 3, o2 = 2 * bb - 3;
      if (c < 21) {
        *ox = o1 / 2.0;
        *oy = o2 / 2.0;
        *side = 2.0;
      } else {
        *ox = o1 / 4.0;
        *oy = o2 / 4.0;
        *side = 0.5;
      }
      return;
    }
    ++k;
  }
}

namespace {

struct NearRule {
  int Nr = 0;                      // radial rule of the inside case (log product rule)
  std::vector<double> r, w, wl;
  int qs = 0;                      // Gauss-Legendre along edges
  std::vector<double> gx, gw;
  int qr = 0;                      // Gauss-Legendre per radial panel (outside case)
  std::vector<double> rx, rw;
};

inline void cheb_vals(double xi, int K, double* T) {
  T[0] = 1.0;
  if (K > 1) T[1] = xi;
  for (int a = 2; a < K; ++a) T[a] = 2.0 * xi * T[a - 1] - T[a - 2];
}

inline void accumulate(double W, const double* Ta, const double* Tb, int K, double* M) {
  for (int a = 0; a < K; ++a) {
    const double wa = W * Ta[a];
    double* Ma = M + a * K;
    for (int b = 0; b < K; ++b) Ma[b] += wa * Tb[b];
  }
}

// Target strictly inside the square: the four triangles joining the target
// to the edges cover the square exactly.
void inside_log_moments(double x, double y, double ox, double oy, double s, int K,
                        const NearRule& R, double* M) {
  for (int i = 0; i < K * K; ++i) M[i] = 0.0;
  const double hs = 0.5 * s;
  const double vx[4] = {ox - hs, ox + hs, ox + hs, ox - hs};
  const double vy[4] = {oy - hs, oy - hs, oy + hs, oy + hs};
  std::vector<double> Ta(K), Tb(K);
  std::vector<double> brk;
  brk.reserve(256);
  for (int e = 0; e < 4; ++e) {
    const double Px = vx[e], Py = vy[e];
    const double Qx = vx[(e + 1) % 4], Qy = vy[(e + 1) % 4];
    const double len = std::hypot(Qx - Px, Qy - Py);
    const double ux = (Qx - Px) / len, uy = (Qy - Py) / len;
    const double nx = uy, ny = -ux;  // outward normal (counter-clockwise edges)
    const double d = nx * (Px - x) + ny * (Py - y);
    if (std::fabs(d) < 1e-300) continue;
    const double Fx = x + d * nx, Fy = y + d * ny;  // foot of the perpendicular
    const double s0 = ux * (Px - Fx) + uy * (Py - Fy);
    const double s1 = s0 + len;
    const double ad = std::fabs(d);
    brk.clear();
    brk.push_back(s0);
    if (s0 < 0 && s1 > 0) brk.push_back(0.0);
    for (double g = ad; g < 1e3; g *= 2.0) {
      if (g > s0 && g < s1) brk.push_back(g);
      if (-g > s0 && -g < s1) brk.push_back(-g);
    }
    brk.push_back(s1);
    std::sort(brk.begin(), brk.end());
    for (size_t pnl = 0; pnl + 1 < brk.size(); ++pnl) {
      const double sa = brk[pnl], sb = brk[pnl + 1];
      if (sb - sa <= 0) continue;
      const double hm = 0.5 * (sb - sa), mm = 0.5 * (sb + sa);
      for (int k = 0; k < R.qs; ++k) {
        const double sk = mm + hm * R.gx[k];
        const double wk = hm * R.gw[k];
        const double Ls = 0.5 * std::log(d * d + sk * sk);
        const double qx = Fx + sk * ux, qy = Fy + sk * uy;
        for (int i = 0; i < R.Nr; ++i) {
          const double rho = R.r[i];
          const double W = d * wk * rho * (R.wl[i] + Ls * R.w[i]);
          const double px = x + rho * (qx - x), py = y + rho * (qy - y);
          const double xi = 2.0 * (px - ox) / s, eta = 2.0 * (py - oy) / s;
          Ta[0] = 1.0;
          Tb[0] = 1.0;
          if (K > 1) {
            Ta[1] = xi;
            Tb[1] = eta;
          }
          for (int a = 2; a < K; ++a) {
            Ta[a] = 2.0 * xi * Ta[a - 1] - Ta[a - 2];
            Tb[a] = 2.0 * eta * Tb[a - 1] - Tb[a - 2];
          }
          for (int a = 0; a < K; ++a) {
            const double wa = W * Ta[a];
            double* Ma = M + a * K;
            for (int b = 0; b < K; ++b) Ma[b] += wa * Tb[b];
          }
        }
      }
    }
  }
}

// Target outside the square, at distance delta from its nearest boundary
// point Pn: the square is the fan of triangles from Pn to the edges that do
// not contain Pn, so every quadrature point lies in the square (the source
// polynomial is never evaluated outside its box).  In each triangle
// y = Pn + rho (q(s) - Pn), s the arc length along the edge, with
// dA = d_e rho drho ds (d_e the distance from Pn to the edge line);
// log|x - y| is analytic there with complex singularities at
// |rho| ~ delta / |q(s) - Pn|, so the rho panels are graded geometrically
// from that scale up to 1, and the s panels are graded towards the foot of
// the perpendicular from Pn on the scale d_e.
void fan_log_moments(double x, double y, double ox, double oy, double s, int K, const NearRule& R,
                     double* M) {
  for (int i = 0; i < K * K; ++i) M[i] = 0.0;
  const double hs = 0.5 * s;
  const double x0 = ox - hs, x1 = ox + hs, y0 = oy - hs, y1 = oy + hs;
  const double Px = std::min(std::max(x, x0), x1), Py = std::min(std::max(y, y0), y1);
  const double delta = std::hypot(x - Px, y - Py);
  const double vx[4] = {x0, x1, x1, x0};
  const double vy[4] = {y0, y0, y1, y1};
  std::vector<double> Ta(K), Tb(K), brk;
  const double tol = 1e-14 * s;
  std::vector<double> sb;
  for (int e = 0; e < 4; ++e) {
    const double Ax = vx[e], Ay = vy[e], Bx = vx[(e + 1) % 4], By = vy[(e + 1) % 4];
    const double len = std::hypot(Bx - Ax, By - Ay);
    const double ux = (Bx - Ax) / len, uy = (By - Ay) / len;
    // distance from Pn to the edge line; skip edges that contain Pn
    const double de = std::fabs((Ax - Px) * uy - (Ay - Py) * ux);
    if (de < tol) continue;
    // arc-length position of the foot of the perpendicular from Pn; the
    // integrand varies on the scale de around it
    const double sf = (Px - Ax) * ux + (Py - Ay) * uy;
    sb.clear();
    sb.push_back(0.0);
    sb.push_back(len);
    if (sf > 0 && sf < len) sb.push_back(sf);
    for (double g = de; g < 2 * len; g *= 2.0) {
      if (sf + g > 0 && sf + g < len) sb.push_back(sf + g);
      if (sf - g > 0 && sf - g < len) sb.push_back(sf - g);
    }
    std::sort(sb.begin(), sb.end());
    for (size_t sp = 0; sp + 1 < sb.size(); ++sp) {
      const double sa = sb[sp], sbb = sb[sp + 1];
      if (sbb - sa <= 0) continue;
      const double shm = 0.5 * (sbb - sa), smm = 0.5 * (sbb + sa);
      for (int k = 0; k < R.qs; ++k) {
        const double sk = smm + shm * R.gx[k], wk = shm * R.gw[k];
        const double qx = Ax + sk * ux, qy = Ay + sk * uy;
        const double rl = std::hypot(qx - Px, qy - Py);
        brk.clear();
        brk.push_back(1.0);
        for (double g = 0.5; g > 0.25 * delta / rl && g > 1e-17; g *= 0.5) brk.push_back(g);
        brk.push_back(0.0);
        std::reverse(brk.begin(), brk.end());
        for (size_t pnl = 0; pnl + 1 < brk.size(); ++pnl) {
          const double ra = brk[pnl], rb = brk[pnl + 1];
          const double hm = 0.5 * (rb - ra), mm = 0.5 * (rb + ra);
          for (int i = 0; i < R.qr; ++i) {
            const double rho = mm + hm * R.rx[i];
            const double yx = Px + rho * (qx - Px), yy = Py + rho * (qy - Py);
            const double W =
                de * wk * hm * R.rw[i] * rho * 0.5 * std::log((x - yx) * (x - yx) + (y - yy) * (y - yy));
            cheb_vals(2.0 * (yx - ox) / s, K, Ta.data());
            cheb_vals(2.0 * (yy - oy) / s, K, Tb.data());
            accumulate(W, Ta.data(), Tb.data(), K, M);
          }
        }
      }
    }
  }
}

void square_log_moments(double x, double y, double ox, double oy, double s, int K, const NearRule& R,
                        double* M) {
  const double hs = 0.5 * s;
  if (x > ox - hs && x < ox + hs && y > oy - hs && y < oy + hs)
    inside_log_moments(x, y, ox, oy, s, K, R, M);
  else
    fan_log_moments(x, y, ox, oy, s, K, R, M);
}

}  // namespace

static void build_near(Tables& T) {
  const int K = T.K, n = T.n;
  NearRule R;
  R.Nr = 2 * K + 2;
  R.r.resize(R.Nr);
  R.w.resize(R.Nr);
  R.wl.resize(R.Nr);
  log_product_rule(R.Nr, R.r.data(), R.w.data(), R.wl.data());
  R.qs = K + 20;
  R.gx.resize(R.qs);
  R.gw.resize(R.qs);
  gauss_legendre(R.qs, R.gx.data(), R.gw.data());
  R.qr = K + 14;
  R.rx.resize(R.qr);
  R.rw.resize(R.qr);
  gauss_legendre(R.qr, R.rx.data(), R.rw.data());
  std::vector<double> C;
  cheb_coef_matrix(K, T.t, C);
  T.near.assign((size_t)kNearConfigs * n * n, 0.0);
  T.near_s2.assign(kNearConfigs, 0.0);
  for (int c = 0; c < kNearConfigs; ++c) {
    double ox, oy, s;
    near_config_geometry(c, &ox, &oy, &s);
    T.near_s2[c] = s * s;
  }
#pragma omp parallel
  {
    std::vector<double> M(K * K), tmp(K * K);
#pragma omp for schedule(dynamic, 1)
    for (int ci = 0; ci < kNearConfigs * n; ++ci) {
      const int c = ci / n, i = ci % n;
      double ox, oy, s;
      near_config_geometry(c, &ox, &oy, &s);
      const double x = 0.5 * T.t[i / K], y = 0.5 * T.t[i % K];
      square_log_moments(x, y, ox, oy, s, K, R, M.data());
      // near[c][j][i] = sum_ab M[a][b] C[a][ja] C[b][jb]
      for (int a = 0; a < K; ++a)
        for (int jb = 0; jb < K; ++jb) {
          double acc = 0;
          for (int b = 0; b < K; ++b) acc += M[a * K + b] * C[b * K + jb];
          tmp[a * K + jb] = acc;
        }
      for (int ja = 0; ja < K; ++ja)
        for (int jb = 0; jb < K; ++jb) {
          double acc = 0;
          for (int a = 0; a < K; ++a) acc += C[a * K + ja] * tmp[a * K + jb];
          T.near[((size_t)c * n + (ja * K + jb)) * n + i] = acc;
        }
    }
  }
}

// Fixed-point bf16 slices of a vector v (one row of a mixed-precision MFMA
// operand, along the contraction): with e the exponent of max |v|
// (max |v| 2^-e in [1/2, 1)), v_k = 2^e sum_{s<4} q_s[k] 2^(-8(s+1)) up to
// 2^(e-33), each q_s[k] an integer of magnitude <= 256 (exact in bf16).
// Products of two such slices and their sums over 32 terms stay integers
// below 2^24, so the bf16 matrix cores sum them exactly in FP32.
static uint16_t bf16_of_int(double q) {
  const float f = (float)q;  // |q| <= 256: exact, and exact in bf16
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (uint16_t)(u >> 16);
}
// The same cut into kF8Slices = 5 int8 slices for the int8 matrix cores:
// v_k = 2^e sum_{s<5} q_s[k] 2^(-6-7s) up to 2^(e-35), |q_s[k]| <= 64, so a
// slice product is at most 2^12 and int32 sums over the whole contraction
// stay exact.
static int f8_split(const double* v, int count, long stride, int8_t* out, long slice_stride, long out_stride) {
  double m = 0.0;
  for (int k = 0; k < count; ++k) m = std::max(m, std::fabs(v[k * stride]));
  int e = 0;
  if (m > 0.0) std::frexp(m, &e);
  for (int k = 0; k < count; ++k) {
    double r = std::ldexp(v[k * stride], 6 - e);
    for (int sl = 0; sl < kF8Slices; ++sl) {
      if (sl) r *= 128.0;
      const double q = std::nearbyint(r);
      out[sl * slice_stride + k * out_stride] = (int8_t)(int)q;
      r -= q;
    }
  }
  return e;
}
static int fx_split(const double* v, int count, long stride, uint16_t* out, long slice_stride, long out_stride) {
  double m = 0.0;
  for (int k = 0; k < count; ++k) m = std::max(m, std::fabs(v[k * stride]));
  int e = 0;
  if (m > 0.0) std::frexp(m, &e);
  for (int k = 0; k < count; ++k) {
    double r = std::ldexp(v[k * stride], -e);
    for (int sl = 0; sl < 4; ++sl) {
      r *= 256.0;
      const double q = std::nearbyint(r);
      out[sl * slice_stride + k * out_stride] = bf16_of_int(q);
      r -= q;
    }
  }
  return e;
}

// Truncated rank-revealing factorisation of the n x n near-field operator
// A (A[i][j] = near[c][j][i]): Householder QR with column pivoting, stopped
// when the largest remaining column norm falls below tol times the first
// one, so ||A - Q W||_F <= sqrt(n - r) tol ||A e_piv0||.  Q: n x r with
// orthonormal columns, W = R_r Pi^T: r x n.  Returns r, or -1 when the rank
// exceeds rmax.
static int near_rrqr(const double* near_c, int n, double tol, int rmax, std::vector<double>& Q,
                     std::vector<double>& W) {
  std::vector<double> M((size_t)n * n);  // M[i][j] = A[i][j]
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) M[(size_t)i * n + j] = near_c[(size_t)j * n + i];
  std::vector<int> perm(n);
  for (int j = 0; j < n; ++j) perm[j] = j;
  std::vector<std::vector<double>> V;
  std::vector<double> tau;
  double r00 = 0.0;
  int r = 0;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    double best = -1.0;
    for (int j = k; j < n; ++j) {
      double s2 = 0.0;
      for (int i = k; i < n; ++i) s2 += M[(size_t)i * n + j] * M[(size_t)i * n + j];
      if (s2 > best) {
        best = s2;
        piv = j;
      }
    }
    const double cn = std::sqrt(best);
    if (k == 0) r00 = cn;
    if (cn <= tol * r00 || cn == 0.0) break;
    if (k >= rmax) return -1;
    if (piv != k) {
      for (int i = 0; i < n; ++i) std::swap(M[(size_t)i * n + k], M[(size_t)i * n + piv]);
      std::swap(perm[k], perm[piv]);
    }
    std::vector<double> v(n - k);
    for (int i = k; i < n; ++i) v[i - k] = M[(size_t)i * n + k];
    const double alpha = v[0] >= 0 ? -cn : cn;
    v[0] -= alpha;
    double vn2 = 0.0;
    for (double x : v) vn2 += x * x;
    const double tk = vn2 > 0 ? 2.0 / vn2 : 0.0;
    for (int j = k; j < n; ++j) {
      double d = 0.0;
      for (int i = k; i < n; ++i) d += v[i - k] * M[(size_t)i * n + j];
      d *= tk;
      for (int i = k; i < n; ++i) M[(size_t)i * n + j] -= d * v[i - k];
    }
    V.push_back(std::move(v));
    tau.push_back(tk);
    r = k + 1;
  }
  W.assign((size_t)r * n, 0.0);
  for (int a = 0; a < r; ++a)
    for (int j = a; j < n; ++j) W[(size_t)a * n + perm[j]] = M[(size_t)a * n + j];
  // Q = H_0 ... H_{r-1} [I_r; 0]
  Q.assign((size_t)n * r, 0.0);
  for (int a = 0; a < r; ++a) Q[(size_t)a * r + a] = 1.0;
  for (int k = r - 1; k >= 0; --k) {
    const std::vector<double>& v = V[k];
    for (int a = 0; a < r; ++a) {
      double d = 0.0;
      for (int i = k; i < n; ++i) d += v[i - k] * Q[(size_t)i * r + a];
      d *= tau[k];
      for (int i = k; i < n; ++i) Q[(size_t)i * r + a] -= d * v[i - k];
    }
  }
  return r;
}

// Low-rank forms of the near-field configurations whose factorisation at
// relative tolerance kNearLrTol saves work: rank rounded up to R (a
// multiple of 16, at most 64) with 2 R <= 0.6 n.  Stored as GEMM operands:
// lr_W[c][j][a] = W[a][j] (n x 64), lr_Q[c][a][i] = Q[i][a] (64 x n), zero
// padded; lr_R[c] = R, or 0 for configurations applied densely.
static void build_near_lowrank(Tables& T) {
  const int n = T.n;
  T.lr_R.assign(kNearConfigs, 0);
  T.lr_rank.assign(kNearConfigs, 0);
  T.lr_W.assign((size_t)kNearConfigs * n * kNearLrMax, 0.0);
  T.lr_Q.assign((size_t)kNearConfigs * kNearLrMax * n, 0.0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < kNearConfigs; ++c) {
    std::vector<double> Q, W;
    const int r = near_rrqr(T.near.data() + (size_t)c * n * n, n, kNearLrTol, kNearLrMax, Q, W);
    if (r <= 0) continue;
    const int R = 16 * ((r + 15) / 16);
    if (R > kNearLrMax || 10 * 2 * R > 6 * n) continue;
    T.lr_R[c] = R;
    T.lr_rank[c] = r;
    for (int a = 0; a < r; ++a)
      for (int j = 0; j < n; ++j) {
        T.lr_W[((size_t)c * n + j) * kNearLrMax + a] = W[(size_t)a * n + j];
        T.lr_Q[((size_t)c * kNearLrMax + a) * n + j] = Q[(size_t)j * r + a];
      }
  }
  // fixed-point bf16 slices for the mixed-precision kernels (K = 16):
  // W rows (rank a, along j), Q rows (target node i, along a), self table
  // rows (target node i, along j), each with its exponent
  if (n != 256) return;
  const size_t SW = (size_t)kNearLrMax * n;  // one slice of one configuration
  T.fx_W.assign((size_t)kNearConfigs * 4 * SW, 0);
  T.fx_Q.assign((size_t)kNearConfigs * 4 * SW, 0);
  T.fx_A.assign((size_t)4 * n * n, 0);
  T.fx_Wexp.assign((size_t)kNearConfigs * kNearLrMax, 0);
  T.fx_Qexp.assign((size_t)kNearConfigs * n, 0);
  T.fx_Aexp.assign(n, 0);
  for (int c = 0; c < kNearConfigs; ++c) {
    for (int a = 0; a < kNearLrMax; ++a)  // fx_W[c][s][a][j] = W[a][j]
      T.fx_Wexp[(size_t)c * kNearLrMax + a] =
          fx_split(&T.lr_W[(size_t)c * n * kNearLrMax + a], n, kNearLrMax,
                   &T.fx_W[(size_t)c * 4 * SW + (size_t)a * n], (long)SW, 1);
    for (int i = 0; i < n; ++i)  // fx_Q[c][s][i][a] = Q[i][a]
      T.fx_Qexp[(size_t)c * n + i] =
          fx_split(&T.lr_Q[(size_t)c * kNearLrMax * n + i], kNearLrMax, n,
                   &T.fx_Q[(size_t)c * 4 * SW + (size_t)i * kNearLrMax], (long)SW, 1);
  }
  for (int i = 0; i < n; ++i)  // fx_A[s][i][j] = T_self[i][j] = near[self][j][i]
    T.fx_Aexp[i] = fx_split(&T.near[(size_t)kNearSelf * n * n + i], n, n, &T.fx_A[(size_t)i * n], (long)n * n, 1);
  // int8 slices, same layouts with kF8Slices slices
  T.f8_W.assign((size_t)kNearConfigs * kF8Slices * SW, 0);
  T.f8_Q.assign((size_t)kNearConfigs * kF8Slices * SW, 0);
  T.f8_A.assign((size_t)kF8Slices * n * n, 0);
  T.f8_Wexp.assign((size_t)kNearConfigs * kNearLrMax, 0);
  T.f8_Qexp.assign((size_t)kNearConfigs * n, 0);
  T.f8_Aexp.assign(n, 0);
  for (int c = 0; c < kNearConfigs; ++c) {
    for (int a = 0; a < kNearLrMax; ++a)
      T.f8_Wexp[(size_t)c * kNearLrMax + a] =
          f8_split(&T.lr_W[(size_t)c * n * kNearLrMax + a], n, kNearLrMax,
                   &T.f8_W[(size_t)c * kF8Slices * SW + (size_t)a * n], (long)SW, 1);
    for (int i = 0; i < n; ++i)
      T.f8_Qexp[(size_t)c * n + i] =
          f8_split(&T.lr_Q[(size_t)c * kNearLrMax * n + i], kNearLrMax, n,
                   &T.f8_Q[(size_t)c * kF8Slices * SW + (size_t)i * kNearLrMax], (long)SW, 1);
  }
  for (int i = 0; i < n; ++i)
    T.f8_Aexp[i] = f8_split(&T.near[(size_t)kNearSelf * n * n + i], n, n, &T.f8_A[(size_t)i * n], (long)n * n, 1);
}

// Symmetry classes of the near-field configurations (K = 16, low-rank
// operators built): class, D4 code and base of every configuration, the
// symmetry-folded row factors, the class column factors and the transposed
// self table (see Tables).
static void build_near_classes(Tables& T) {
  const int n = T.n, K = T.K;
  T.ts_ok = false;
  if (n != 256 || T.lr_R.empty()) return;
  // canonical base offsets (units of the target side) per class
  const double bx[kNearClasses] = {0.0, 1.0, 1.0, 1.5, 1.5, 0.75, 0.75};
  const double by[kNearClasses] = {0.0, 0.0, 1.0, 1.5, 0.5, 0.75, 0.25};
  T.near_cls.assign(kNearConfigs, -1);
  T.near_g.assign(kNearConfigs, 0);
  T.cls_base.assign(kNearClasses, -1);
  T.cls_R.assign(kNearClasses, 0);
  auto class_of = [&](int c) {
    double ox, oy, side;
    near_config_geometry(c, &ox, &oy, &side);
    if (c == kNearSelf) return 0;
    const bool corner = std::fabs(std::fabs(ox) - std::fabs(oy)) < 1e-12;
    if (side == 1.0) return corner ? 2 : 1;
    if (side == 2.0) return corner ? 3 : 4;
    return corner ? 5 : 6;
  };
  for (int c = 0; c < kNearConfigs; ++c) {
    double ox, oy, side;
    near_config_geometry(c, &ox, &oy, &side);
    const int k = class_of(c);
    T.near_cls[c] = k;
    if (ox == bx[k] && oy == by[k]) T.cls_base[k] = c;
  }
  for (int k = 0; k < kNearClasses; ++k)
    if (T.cls_base[k] < 0) return;
  for (int c = 0; c < kNearConfigs; ++c) {
    double ox, oy, side;
    near_config_geometry(c, &ox, &oy, &side);
    const int k = T.near_cls[c];
    int found = -1;
    for (int g = 0; g < 8 && found < 0; ++g) {
      double gx, gy;
      d4_point(g, bx[k], by[k], &gx, &gy);
      if (gx == ox && gy == oy) found = g;
    }
    if (found < 0) return;
    T.near_g[c] = found;
  }
  for (int k = 1; k < kNearClasses; ++k) {
    T.cls_R[k] = T.lr_R[T.cls_base[k]];
    if (T.cls_R[k] <= 0) return;  // a class base applied densely: no target-stationary path
  }
  // symmetry check against the configuration tables themselves
  double err = 0.0;
  for (int c = 0; c < kNearConfigs; ++c) {
    const int b = T.cls_base[T.near_cls[c]], g = T.near_g[c];
    const double* Tc = T.near.data() + (size_t)c * n * n;
    const double* Tb = T.near.data() + (size_t)b * n * n;
    double mx = 0.0, d = 0.0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        mx = std::max(mx, std::fabs(Tb[(size_t)j * n + i]));
        d = std::max(d, std::fabs(Tc[(size_t)d4_node(g, K, j) * n + d4_node(g, K, i)] - Tb[(size_t)j * n + i]));
      }
    err = std::max(err, d / mx);
  }
  T.ts_sym_err = err;
  T.lr_Wp.assign((size_t)kNearConfigs * n * kNearLrMax, 0.0);
  for (int c = 0; c < kNearConfigs; ++c) {
    if (c == kNearSelf) continue;
    const int b = T.cls_base[T.near_cls[c]], gi = d4_inverse(T.near_g[c]);
    for (int j = 0; j < n; ++j) {
      const int jb = d4_node(gi, K, j);
      for (int a = 0; a < kNearLrMax; ++a)
        T.lr_Wp[((size_t)c * n + j) * kNearLrMax + a] = T.lr_W[((size_t)b * n + jb) * kNearLrMax + a];
    }
  }
  T.cls_QT.assign((size_t)kNearClasses * n * kNearLrMax, 0.0);
  for (int k = 1; k < kNearClasses; ++k) {
    const int b = T.cls_base[k];
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < kNearLrMax; ++a)
        T.cls_QT[((size_t)k * n + i) * kNearLrMax + a] = T.lr_Q[((size_t)b * kNearLrMax + a) * n + i];
  }
  T.self_T.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T.self_T[(size_t)i * n + j] = T.near[((size_t)kNearSelf * n + j) * n + i];
  T.ts_ok = true;
}

// Chebyshev moments of a smooth kernel over a square by tensor Gauss-Legendre
// on npan x npan panels, for several kernel values at once.
static void build_p2l(Tables& T) {
  const int K = T.K, n = T.n, P = T.p + 1;
  std::vector<double> C;
  cheb_coef_matrix(K, T.t, C);
  const int q = 24, npan = 4;
  std::vector<double> gx(q), gw(q);
  gauss_legendre(q, gx.data(), gw.data());
  T.p2l.assign((size_t)kP2LSlots * P * n * 2, 0.0);
  T.p2l_area.assign(kP2LSlots, 0.0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int slot = 0; slot < kP2LSlots; ++slot) {
    const int ox2 = 2 * (slot / 6) - 5, oy2 = 2 * (slot % 6) - 5;
    if (std::abs(ox2) != 5 && std::abs(oy2) != 5) continue;
    T.p2l_area[slot] = 4.0;
    const double ox = ox2 / 2.0, oy = oy2 / 2.0, s = 2.0;
    // moments Mre/Mim[l][a][b]
    std::vector<cplx> M((size_t)P * K * K, cplx(0, 0));
    std::vector<double> Ta(K), Tb(K);
    std::vector<cplx> pw(P);
    for (int pa = 0; pa < npan; ++pa)
      for (int pb = 0; pb < npan; ++pb)
        for (int i = 0; i < q; ++i)
          for (int j = 0; j < q; ++j) {
            // reference coordinates on [-1,1]^2 of the source square
            const double xi = -1.0 + (pa + 0.5 * (gx[i] + 1.0)) * (2.0 / npan);
            const double eta = -1.0 + (pb + 0.5 * (gx[j] + 1.0)) * (2.0 / npan);
            const double W = gw[i] * gw[j] * (1.0 / npan) * (1.0 / npan) * (s * s / 4.0);
            const cplx v(ox + 0.5 * s * xi, oy + 0.5 * s * eta);
            Ta[0] = Tb[0] = 1.0;
            if (K > 1) {
              Ta[1] = xi;
              Tb[1] = eta;
            }
            for (int a = 2; a < K; ++a) {
              Ta[a] = 2 * xi * Ta[a - 1] - Ta[a - 2];
              Tb[a] = 2 * eta * Tb[a - 1] - Tb[a - 2];
            }
            pw[0] = cplx(std::log(std::abs(v)), 0.0);
            const cplx iv = 1.0 / v;
            cplx vk = 1.0;
            for (int l = 1; l < P; ++l) {
              vk *= iv;
              pw[l] = -vk / (double)l;
            }
            for (int l = 0; l < P; ++l) {
              const cplx wl = W * pw[l];
              cplx* Ml = &M[(size_t)l * K * K];
              for (int a = 0; a < K; ++a) {
                const cplx wa = wl * Ta[a];
                for (int b = 0; b < K; ++b) Ml[a * K + b] += wa * Tb[b];
              }
            }
          }
    for (int l = 0; l < P; ++l)
      for (int ja = 0; ja < K; ++ja)
        for (int jb = 0; jb < K; ++jb) {
          cplx acc = 0;
          for (int a = 0; a < K; ++a)
            for (int b = 0; b < K; ++b) acc += M[(size_t)l * K * K + a * K + b] * C[a * K + ja] * C[b * K + jb];
          size_t o = (((size_t)slot * P + l) * n + (ja * K + jb)) * 2;
          T.p2l[o] = acc.real();
          T.p2l[o + 1] = (l == 0) ? 0.0 : acc.imag();
        }
  }
}

static double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  long double r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return (double)r;
}

static void put(std::vector<double>& v, size_t idx, cplx z) {
  v[2 * idx] = z.real();
  v[2 * idx + 1] = z.imag();
}

static void build_expansions(Tables& T) {
  const int K = T.K, n = T.n, P = T.p + 1;
  // P2M: a_0 = int f, a_k = -(1/k) int f ((w-c)/h)^k on the unit box
  {
    const int q = K + P / 2 + 4;
    std::vector<double> gx(q), gw(q), C;
    gauss_legendre(q, gx.data(), gw.data());
    cheb_coef_matrix(K, T.t, C);
    // Lagrange basis values of the 1D grid at the GL nodes on [-1/2,1/2]
    std::vector<double> Lg((size_t)q * K);
    for (int i = 0; i < q; ++i) {
      const double xi = gx[i];  // reference [-1,1]
      std::vector<double> Tm(K);
      Tm[0] = 1;
      if (K > 1) Tm[1] = xi;
      for (int a = 2; a < K; ++a) Tm[a] = 2 * xi * Tm[a - 1] - Tm[a - 2];
      for (int j = 0; j < K; ++j) {
        double acc = 0;
        for (int a = 0; a < K; ++a) acc += C[a * K + j] * Tm[a];
        Lg[i * K + j] = acc;
      }
    }
    T.p2m.assign((size_t)P * n * 2, 0.0);
    for (int k = 0; k < P; ++k)
      for (int ja = 0; ja < K; ++ja)
        for (int jb = 0; jb < K; ++jb) {
          cplx acc = 0;
          for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j) {
              const cplx wv(0.5 * gx[i], 0.5 * gx[j]);
              cplx pk = 1.0;
              for (int m = 0; m < k; ++m) pk *= wv;
              acc += 0.25 * gw[i] * gw[j] * Lg[i * K + ja] * Lg[j * K + jb] * pk;
            }
          if (k > 0) acc *= -1.0 / k;
          put(T.p2m, (size_t)k * n + ja * K + jb, k == 0 ? cplx(acc.real(), 0) : acc);
        }
  }
  // L2P: ((z_i - c)/h)^l
  T.l2p.assign((size_t)n * P * 2, 0.0);
  for (int i = 0; i < n; ++i) {
    const cplx z(0.5 * T.t[i / K], 0.5 * T.t[i % K]);
    cplx zl = 1.0;
    for (int l = 0; l < P; ++l) {
      put(T.l2p, (size_t)i * P + l, zl);
      zl *= z;
    }
  }
  // M2M and L2L for the child in Morton position q = dx + 2 dy (child
  // (2x+dx, 2y+dy)): z0/h_parent = ((2dx-1) + i (2dy-1)) / 4
  T.m2m.assign((size_t)4 * P * P * 2, 0.0);
  T.l2l.assign((size_t)4 * P * P * 2, 0.0);
  for (int qd = 0; qd < 4; ++qd) {
    const int dx = qd % 2, dy = qd / 2;
    const cplx z0(0.25 * (2 * dx - 1), 0.25 * (2 * dy - 1));
    std::vector<cplx> zp(2 * P + 1);
    zp[0] = 1.0;
    for (int i = 1; i <= 2 * P; ++i) zp[i] = zp[i - 1] * z0;
    for (int k = 0; k < P; ++k)
      for (int l = 0; l < P; ++l) {
        cplx m = 0;
        if (k == 0) {
          m = (l == 0) ? cplx(1.0) : -zp[l] / (double)l;
        } else if (l >= k) {
          m = std::ldexp(1.0, -k) * zp[l - k] * binom(l - 1, k - 1);
        }
        put(T.m2m, ((size_t)qd * P + k) * P + l, m);
        cplx g = 0;
        if (k >= l) g = binom(k, l) * zp[k - l] * std::ldexp(1.0, -l);
        put(T.l2l, ((size_t)qd * P + k) * P + l, g);
      }
  }
  // M2L for centre offsets (dx, dy) in units h: t = 1/(dx + i dy)
  T.m2l.assign((size_t)kM2LSlots * P * P * 2, 0.0);
  for (int o = 0; o < kM2LSlots; ++o) {
    const int dx = o / 7 - 3, dy = o % 7 - 3;
    if (std::max(std::abs(dx), std::abs(dy)) < 2) continue;
    const cplx tt = 1.0 / cplx(dx, dy);
    std::vector<cplx> tp(2 * P + 1);
    tp[0] = 1.0;
    for (int i = 1; i <= 2 * P; ++i) tp[i] = tp[i - 1] * tt;
    for (int k = 0; k < P; ++k)
      for (int l = 0; l < P; ++l) {
        cplx m;
        if (k == 0)
          m = (l == 0) ? cplx(std::log(std::hypot((double)dx, (double)dy)), 0.0) : -tp[l] / (double)l;
        else
          m = ((k % 2) ? -1.0 : 1.0) * binom(k + l - 1, l) * tp[k + l];
        put(T.m2l, ((size_t)o * P + k) * P + l, m);
      }
  }
}

static void build_pascal(Tables& T) {
  const int P = T.p + 1, n = T.n;
  T.pas_m2l.assign((size_t)P * P, 0.0);
  T.pas_m2m.assign((size_t)P * P, 0.0);
  T.pas_l2l.assign((size_t)P * P, 0.0);
  for (int k = 0; k < P; ++k)
    for (int l = 0; l < P; ++l) {
      if (k >= 1) T.pas_m2l[(size_t)k * P + l] = binom(k + l - 1, l);
      if (k >= 1 && k <= l) T.pas_m2m[(size_t)k * P + l] = binom(l - 1, k - 1);
      if (k >= l) T.pas_l2l[(size_t)k * P + l] = binom(k, l);
    }
  T.pas_m2l_t.assign((size_t)P * P, 0.0);
  T.pas_m2m_t.assign((size_t)P * P, 0.0);
  T.pas_l2l_t.assign((size_t)P * P, 0.0);
  for (int k = 0; k < P; ++k)
    for (int l = 0; l < P; ++l) {
      T.pas_m2l_t[(size_t)l * P + k] = T.pas_m2l[(size_t)k * P + l];
      T.pas_m2m_t[(size_t)l * P + k] = T.pas_m2m[(size_t)k * P + l];
      T.pas_l2l_t[(size_t)l * P + k] = T.pas_l2l[(size_t)k * P + l];
    }
  T.m2l_tpow.assign((size_t)kM2LSlots * P * 2, 0.0);
  T.m2l_tneg.assign((size_t)kM2LSlots * P * 2, 0.0);
  T.m2l_logd.assign(kM2LSlots, 0.0);
  for (int o = 0; o < kM2LSlots; ++o) {
    const int dx = o / 7 - 3, dy = o % 7 - 3;
    if (std::max(std::abs(dx), std::abs(dy)) < 2) continue;
    const cplx tt = 1.0 / cplx(dx, dy);
    T.m2l_logd[o] = std::log(std::hypot((double)dx, (double)dy));
    cplx a = 1.0, b = 1.0;
    for (int l = 0; l < P; ++l) {
      put(T.m2l_tpow, (size_t)o * P + l, a);
      put(T.m2l_tneg, (size_t)o * P + l, b);
      a *= tt;
      b *= -tt;
    }
  }
  T.m2m_in.assign((size_t)4 * P * 2, 0.0);
  T.m2m_out.assign((size_t)4 * P * 2, 0.0);
  T.l2l_in.assign((size_t)4 * P * 2, 0.0);
  T.l2l_out.assign((size_t)4 * P * 2, 0.0);
  for (int qd = 0; qd < 4; ++qd) {
    const int dx = qd % 2, dy = qd / 2;
    const cplx w(0.25 * (2 * dx - 1), 0.25 * (2 * dy - 1));
    const cplx iw2 = 1.0 / (2.0 * w);
    cplx wk = 1.0, iwk = 1.0;
    for (int k = 0; k < P; ++k) {
      put(T.m2m_in, (size_t)qd * P + k, iwk);
      put(T.m2m_out, (size_t)qd * P + k, wk);
      put(T.l2l_in, (size_t)qd * P + k, wk);
      put(T.l2l_out, (size_t)qd * P + k, iwk);
      wk *= w;
      iwk *= iw2;
    }
  }
  // P2L as a real GEMM operand
  T.p2l_rows = 64 * ((2 * P + 63) / 64);
  const int R = T.p2l_rows;
  T.p2l_gemm.assign((size_t)kP2LSlots * n * R, 0.0);
  for (int s = 0; s < kP2LSlots; ++s)
    for (int l = 0; l < P; ++l)
      for (int j = 0; j < n; ++j) {
        const size_t src = 2 * (((size_t)s * P + l) * n + j);
        T.p2l_gemm[((size_t)s * n + j) * R + 2 * l] = T.p2l[src];
        T.p2l_gemm[((size_t)s * n + j) * R + 2 * l + 1] = T.p2l[src + 1];
      }
  T.p2m_gemm.assign((size_t)n * R, 0.0);
  for (int k = 0; k < P; ++k)
    for (int j = 0; j < n; ++j) {
      T.p2m_gemm[(size_t)j * R + 2 * k] = T.p2m[2 * ((size_t)k * n + j)];
      T.p2m_gemm[(size_t)j * R + 2 * k + 1] = T.p2m[2 * ((size_t)k * n + j) + 1];
    }
  // M2P (list 3) as a real GEMM operand.  A list-3 box w of a leaf b in a
  // level-restricted tree is a child of a colleague of b that does not touch
  // b: one level finer, centre offset (ox, oy) h_w/2 with odd ox, oy in
  // {-5..5} and max(|ox|,|oy|) = 5 (20 of the 36 slots of the P2L grid).
  // In units of h_w, node i of b sits at z_i = (t_a - ox/2, t_b - oy/2) from
  // the centre of w, and the scaled expansion of w gives there
  //   Re sum_{k>=1} a_k z_i^-k + a_0 log|z_i| + a_0 log h_w,
  // so column 2k of the table holds Re z^-k, column 2k+1 -Im z^-k (k >= 1),
  // column 0 log|z| (the a_0 log h_w part is added per leaf).
  // Layout [slot][k][i], k < p2l_rows (zero past 2P), i < n.
  T.m2p_gemm.assign((size_t)kP2LSlots * R * n, 0.0);
  for (int slot = 0; slot < kP2LSlots; ++slot) {
    const int ox = 2 * (slot / 6) - 5, oy = 2 * (slot % 6) - 5;
    if (std::abs(ox) != 5 && std::abs(oy) != 5) continue;
    double* Ts = &T.m2p_gemm[(size_t)slot * R * n];
    for (int i = 0; i < n; ++i) {
      const std::complex<long double> z((long double)T.t[i / T.K] - 0.5L * ox, (long double)T.t[i % T.K] - 0.5L * oy);
      const std::complex<long double> iz = 1.0L / z;
      Ts[i] = (double)std::log(std::abs(z));
      std::complex<long double> zk = 1.0L;
      for (int k = 1; k < P; ++k) {
        zk *= iz;
        Ts[(size_t)(2 * k) * n + i] = (double)zk.real();
        Ts[(size_t)(2 * k + 1) * n + i] = (double)-zk.imag();
      }
    }
  }
}

void build_tables(Tables& T) {
  T.n = T.K * T.K;
  T.nG = (T.deg + 1) * (T.deg + 2) / 2;
  T.nX = T.n + T.Kbar * T.Kbar + T.nG;
  T.t.resize(T.K);
  T.tbar.resize(T.Kbar);
  for (int a = 0; a < T.K; ++a) T.t[a] = -std::cos((2 * a + 1) * M_PI / (2 * T.K));
  for (int a = 0; a < T.Kbar; ++a) T.tbar[a] = -std::cos((2 * a + 1) * M_PI / (2 * T.Kbar));
  // unit-square weights: products of Fejer weights (sum 2 on [-1,1]) / 4
  {
    std::vector<double> C;
    cheb_coef_matrix(T.K, T.t, C);
    std::vector<double> w1(T.K, 0.0);
    for (int j = 0; j < T.K; ++j) {
      double acc = 0;
      for (int a = 0; a < T.K; a += 2) acc += C[a * T.K + j] * (2.0 / (1.0 - (double)a * a));
      w1[j] = acc;
    }
    T.w2.resize(T.n);
    for (int a = 0; a < T.K; ++a)
      for (int b = 0; b < T.K; ++b) T.w2[a * T.K + b] = 0.25 * w1[a] * w1[b];
  }
  cheb_coef_matrix(T.Kbar, T.tbar, T.cbar);
  build_stencil(T);
  build_expansions(T);
  build_near(T);
  build_near_lowrank(T);
  build_near_classes(T);
  build_p2l(T);
  build_pascal(T);
}

}  // namespace vfx
