/*
 * Oracle: direct quadrature of the log-kernel volume potential.
 * Test infrastructure only (called from oracle/volume.py).
 *
 *   V(t) = (1/2pi) sum_B  int_B log|t - y| p_B(y) dy                (1)
 *
 * (the volume potential with the free-space Green's function
 * G = (1/2pi) log|x - y|, Section 1, eqs. volpot/greenf, applied to the
 * piecewise-polynomial f^e the VFMM sees, Section 4.1 and the remark that
 * the near field is exact for that piecewise polynomial.)
 *
 * p_B(y) = sum_{a,b<K} c_B[a][b] T_a(xi) T_b(eta),  xi = 2(y1-cx)/h,
 * eta = 2(y2-cy)/h, is the tensor Chebyshev interpolant on box B.
 *
 * Quadrature (deliberately plain):
 *  - far pair (distance from t to B >= h_B): one tensor Gauss-Legendre rule
 *    with QF x QF nodes on B;
 *  - near pair: P = nearest point of B to t.  B is split at P into at most
 *    four rectangles that have P as a corner; each side of each rectangle is
 *    cut at geometric breakpoints P + s*2^-k (k = M..0) and every panel of
 *    the resulting tensor mesh gets a QN x QN Gauss-Legendre rule.  Each
 *    panel (except the one touching P) keeps the singular point at least one
 *    panel length away along each axis, so plain Gauss-Legendre converges
 *    geometrically there; the panel at P has area 4^-M relative.
 * Sums are accumulated in long double.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXQ 48
#define MAXK 32

typedef struct {
  int K;
  double cx, cy, h;
  const double *c; /* K*K coefficients, c[a*K+b] */
} box_t;

/* integral over [x0,x1]x[y0,y1] (inside box b) of log|t-y| p_b(y) dy,
 * tensor Gauss-Legendre with q x q nodes */
static long double panel(double tx, double ty, double x0, double x1, double y0, double y1,
                         int q, const double *gx, const double *gw, const box_t *b) {
  const int K = b->K;
  double Tx[MAXQ][MAXK], Ty[MAXQ][MAXK], D[MAXQ][MAXK];
  double px[MAXQ], py[MAXQ];
  const double hx = 0.5 * (x1 - x0), mx = 0.5 * (x1 + x0);
  const double hy = 0.5 * (y1 - y0), my = 0.5 * (y1 + y0);
  for (int i = 0; i < q; ++i) {
    px[i] = mx + hx * gx[i];
    py[i] = my + hy * gx[i];
    double xi = 2.0 * (px[i] - b->cx) / b->h;
    double eta = 2.0 * (py[i] - b->cy) / b->h;
    Tx[i][0] = 1.0;
    Ty[i][0] = 1.0;
    if (K > 1) { Tx[i][1] = xi; Ty[i][1] = eta; }
    for (int a = 2; a < K; ++a) {
      Tx[i][a] = 2.0 * xi * Tx[i][a - 1] - Tx[i][a - 2];
      Ty[i][a] = 2.0 * eta * Ty[i][a - 1] - Ty[i][a - 2];
    }
  }
  /* D[i][bb] = sum_a Tx[i][a] c[a][bb] */
  for (int i = 0; i < q; ++i)
    for (int bb = 0; bb < K; ++bb) {
      double s = 0.0;
      for (int a = 0; a < K; ++a) s += Tx[i][a] * b->c[a * K + bb];
      D[i][bb] = s;
    }
  long double acc = 0.0L;
  for (int i = 0; i < q; ++i) {
    long double row = 0.0L;
    const double dx = px[i] - tx;
    for (int j = 0; j < q; ++j) {
      double p = 0.0;
      for (int bb = 0; bb < K; ++bb) p += D[i][bb] * Ty[j][bb];
      const double dy = py[j] - ty;
      const double r2 = dx * dx + dy * dy;
      if (r2 > 0.0) row += (long double)gw[j] * 0.5L * logl((long double)r2) * p;
    }
    acc += (long double)gw[i] * row;
  }
  return acc * hx * hy;
}

/* breakpoints of [p, p+s] graded toward p: p, p+s*2^-M, ..., p+s/2, p+s */
static int graded(double p, double s, int M, double *out) {
  int n = 0;
  out[n++] = p;
  for (int k = M; k >= 0; --k) out[n++] = p + s * ldexp(1.0, -k);
  return n;
}

static long double near_pair(double tx, double ty, const box_t *b, int M, int q,
                             const double *gx, const double *gw) {
  const double x0 = b->cx - 0.5 * b->h, x1 = b->cx + 0.5 * b->h;
  const double y0 = b->cy - 0.5 * b->h, y1 = b->cy + 0.5 * b->h;
  const double Px = tx < x0 ? x0 : (tx > x1 ? x1 : tx);
  const double Py = ty < y0 ? y0 : (ty > y1 ? y1 : ty);
  /* sides of the split in x and y: intervals [P, end] */
  double xs[2], ys[2];
  int nx = 0, ny = 0;
  if (Px > x0) xs[nx++] = x0 - Px;
  if (Px < x1) xs[nx++] = x1 - Px;
  if (Py > y0) ys[ny++] = y0 - Py;
  if (Py < y1) ys[ny++] = y1 - Py;
  double bx[70], by[70];
  long double acc = 0.0L;
  for (int ix = 0; ix < nx; ++ix) {
    int mx = graded(Px, xs[ix], M, bx);
    for (int iy = 0; iy < ny; ++iy) {
      int my = graded(Py, ys[iy], M, by);
      for (int i = 0; i + 1 < mx; ++i) {
        double a0 = bx[i] < bx[i + 1] ? bx[i] : bx[i + 1];
        double a1 = bx[i] < bx[i + 1] ? bx[i + 1] : bx[i];
        for (int j = 0; j + 1 < my; ++j) {
          double c0 = by[j] < by[j + 1] ? by[j] : by[j + 1];
          double c1 = by[j] < by[j + 1] ? by[j + 1] : by[j];
          acc += panel(tx, ty, a0, a1, c0, c1, q, gx, gw, b);
        }
      }
    }
  }
  return acc;
}

/*
 * targets: nt points (tx, ty).  boxes: nb boxes with centres, sides and
 * coefficient blocks coef[nb][K*K].  out[t] = V(t) as in (1).
 * (gxf, gwf, qf), (gxn, gwn, qn): the far / near Gauss-Legendre rules on
 * [-1,1] (nodes and weights, computed by the caller); M: grading depth;
 * far_ratio: pairs with dist(t,B) >= far_ratio*h_B use the far rule.
 */
int oracle_volume(int nt, const double *tx, const double *ty, int nb, const double *bcx,
                  const double *bcy, const double *bh, int K, const double *coef,
                  const double *gxf, const double *gwf, int qf, const double *gxn,
                  const double *gwn, int qn, int M, double far_ratio, double *out) {
  if (K > MAXK || qf < 1 || qn < 1 || qf > MAXQ || qn > MAXQ || M > 60) return -1;
  const long double inv2pi = 1.0L / (2.0L * 3.14159265358979323846264338327950288L);
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < nt; ++t) {
    long double acc = 0.0L;
    for (int k = 0; k < nb; ++k) {
      box_t b = {K, bcx[k], bcy[k], bh[k], coef + (size_t)k * K * K};
      const double x0 = b.cx - 0.5 * b.h, x1 = b.cx + 0.5 * b.h;
      const double y0 = b.cy - 0.5 * b.h, y1 = b.cy + 0.5 * b.h;
      const double dx = tx[t] < x0 ? x0 - tx[t] : (tx[t] > x1 ? tx[t] - x1 : 0.0);
      const double dy = ty[t] < y0 ? y0 - ty[t] : (ty[t] > y1 ? ty[t] - y1 : 0.0);
      const double d = sqrt(dx * dx + dy * dy);
      if (d >= far_ratio * b.h)
        acc += panel(tx[t], ty[t], x0, x1, y0, y1, qf, gxf, gwf, &b);
      else
        acc += near_pair(tx[t], ty[t], &b, M, qn, gxn, gwn);
    }
    out[t] = (double)(acc * inv2pi);
  }
  return 0;
}
