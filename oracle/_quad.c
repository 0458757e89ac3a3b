/* Oracle quadrature core (TEST INFRASTRUCTURE ONLY; plain C, FP64, OpenMP).
 *
 * The quantity everything else is built from is the log-kernel integral of the leaf basis
 * over the reference square (Sec. 4.2, eq. (vbulk), restricted to one leaf):
 *
 *     I_k(x0) = int_{[-1,1]^2} log|x0 - eta| l_k(eta) d eta,   k = j*p + i,
 *
 * l_k(eta) = L_i(eta_1) L_j(eta_2) the tensor Lagrange basis on the leaf's Chebyshev points.
 *
 * Method (plain adaptive subdivision): a square is integrated with a tensor Gauss-Legendre
 * rule when its distance to x0 is at least its side; otherwise it is split in four. Squares
 * of half-width below H_MIN are dropped; what they carry is bounded by
 * (2 H_MIN)^2 |log(2 H_MIN)| max|l_k|, below 1e-17 for H_MIN = 2.5e-10.
 *
 * The gradient (oq_direct_grad) integrates (x0 - y)/|x0 - y|^2 against f_h with the same
 * subdivision, down to squares of half-width 1e-14 (the kernel is only O(1/r) singular).
 *
 * The direct sum (oq_direct_far) applies the same routine leaf by leaf in physical
 * coordinates:  int_{B_b} log|x - y| f_h(y) dy = s_b^2 [ log(s_b) (W . f_b) + int log|x0 - eta| f^_b(eta) d eta ],
 * x0 = (x - c_b)/s_b, f^_b the leaf interpolant on the reference square.
 *
 * Nodes, barycentric weights, tensor weights and the Gauss-Legendre rule are handed in by
 * the Python side (oracle/nodes.py and NumPy's leggauss); nothing here is shared with the
 * HIP path.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PMAX 16
#define NQMAX 32

static int P = 16, NQ = 24;
static double T[PMAX], LAM[PMAX], WT[PMAX * PMAX];
static double GX[NQMAX], GW[NQMAX];
static double H_MIN = 2.5e-10;

int oq_init(int p, const double* t, const double* lam, const double* wt, int nq, const double* gx,
            const double* gw, double hmin) {
  if (p < 1 || p > PMAX || nq < 1 || nq > NQMAX) return -1;
  P = p;
  NQ = nq;
  memcpy(T, t, sizeof(double) * p);
  memcpy(LAM, lam, sizeof(double) * p);
  memcpy(WT, wt, sizeof(double) * p * p);
  memcpy(GX, gx, sizeof(double) * nq);
  memcpy(GW, gw, sizeof(double) * nq);
  if (hmin > 0) H_MIN = hmin;
  return 0;
}

/* L[i] = L_i(x), second barycentric form. */
static void lagrange_row(double x, double* L) {
  for (int i = 0; i < P; ++i)
    if (x == T[i]) {
      for (int j = 0; j < P; ++j) L[j] = (j == i) ? 1.0 : 0.0;
      return;
    }
  double s = 0.0;
  for (int i = 0; i < P; ++i) {
    L[i] = LAM[i] / (x - T[i]);
    s += L[i];
  }
  for (int i = 0; i < P; ++i) L[i] /= s;
}

static double dist_to_square(double x0, double y0, double cx, double cy, double h) {
  double dx = fabs(x0 - cx) - h, dy = fabs(y0 - cy) - h;
  if (dx < 0) dx = 0;
  if (dy < 0) dy = 0;
  return sqrt(dx * dx + dy * dy);
}

/* acc[j*P+i] += int_{square} log|x0 - y| L_i(y1) L_j(y2) dy */
static void square_basis(double x0, double y0, double cx, double cy, double h, double* acc) {
  double Lx[NQMAX][PMAX], Ly[NQMAX][PMAX], G[NQMAX][NQMAX], C[PMAX][NQMAX];
  for (int a = 0; a < NQ; ++a) lagrange_row(cx + h * GX[a], Lx[a]);
  for (int b = 0; b < NQ; ++b) lagrange_row(cy + h * GX[b], Ly[b]);
  for (int a = 0; a < NQ; ++a) {
    double dx = cx + h * GX[a] - x0;
    for (int b = 0; b < NQ; ++b) {
      double dy = cy + h * GX[b] - y0;
      G[a][b] = 0.5 * log(dx * dx + dy * dy) * GW[a] * GW[b] * h * h;
    }
  }
  for (int i = 0; i < P; ++i)
    for (int b = 0; b < NQ; ++b) {
      double s = 0.0;
      for (int a = 0; a < NQ; ++a) s += Lx[a][i] * G[a][b];
      C[i][b] = s;
    }
  for (int j = 0; j < P; ++j)
    for (int i = 0; i < P; ++i) {
      double s = 0.0;
      for (int b = 0; b < NQ; ++b) s += C[i][b] * Ly[b][j];
      acc[j * P + i] += s;
    }
}

static void adapt_basis(double x0, double y0, double cx, double cy, double h, double* acc) {
  if (dist_to_square(x0, y0, cx, cy, h) >= 2.0 * h) {
    square_basis(x0, y0, cx, cy, h, acc);
    return;
  }
  if (h <= H_MIN) return;
  double q = 0.5 * h;
  adapt_basis(x0, y0, cx - q, cy - q, q, acc);
  adapt_basis(x0, y0, cx + q, cy - q, q, acc);
  adapt_basis(x0, y0, cx - q, cy + q, q, acc);
  adapt_basis(x0, y0, cx + q, cy + q, q, acc);
}

/* out[n][P*P] = I(x0_n) for n points x0 (n x 2). */
void oq_logint(int n, const double* x0, double* out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < n; ++t) {
    double* acc = out + (size_t)t * P * P;
    memset(acc, 0, sizeof(double) * P * P);
    adapt_basis(x0[2 * t], x0[2 * t + 1], 0.0, 0.0, 1.0, acc);
  }
}

/* int_{square} log|x0 - y| f_h(y) dy  with f_h the interpolant of F (F[j*P+i]) */
static double square_f(double x0, double y0, double cx, double cy, double h, const double* F) {
  double Lx[NQMAX][PMAX], Ly[NQMAX][PMAX], Fy[NQMAX][PMAX];
  for (int a = 0; a < NQ; ++a) lagrange_row(cx + h * GX[a], Lx[a]);
  for (int b = 0; b < NQ; ++b) lagrange_row(cy + h * GX[b], Ly[b]);
  /* Fy[b][i] = sum_j F[j][i] L_j(y_b) */
  for (int b = 0; b < NQ; ++b)
    for (int i = 0; i < P; ++i) {
      double s = 0.0;
      for (int j = 0; j < P; ++j) s += F[j * P + i] * Ly[b][j];
      Fy[b][i] = s;
    }
  double tot = 0.0;
  for (int a = 0; a < NQ; ++a) {
    double dx = cx + h * GX[a] - x0;
    for (int b = 0; b < NQ; ++b) {
      double fv = 0.0;
      for (int i = 0; i < P; ++i) fv += Fy[b][i] * Lx[a][i];
      double dy = cy + h * GX[b] - y0;
      tot += 0.5 * log(dx * dx + dy * dy) * GW[a] * GW[b] * fv;
    }
  }
  return tot * h * h;
}

static double adapt_f(double x0, double y0, double cx, double cy, double h, const double* F) {
  if (dist_to_square(x0, y0, cx, cy, h) >= 2.0 * h) return square_f(x0, y0, cx, cy, h, F);
  if (h <= H_MIN) return 0.0;
  double q = 0.5 * h;
  return adapt_f(x0, y0, cx - q, cy - q, q, F) + adapt_f(x0, y0, cx + q, cy - q, q, F) +
         adapt_f(x0, y0, cx - q, cy + q, q, F) + adapt_f(x0, y0, cx + q, cy + q, q, F);
}

/* Values of f_h at the NQ x NQ Gauss points of the whole reference square: Q[a*NQ+b]. */
static void leaf_at_gauss(const double* F, double* Q) {
  double L[NQMAX][PMAX], Fy[NQMAX][PMAX];
  for (int a = 0; a < NQ; ++a) lagrange_row(GX[a], L[a]);
  for (int b = 0; b < NQ; ++b)
    for (int i = 0; i < P; ++i) {
      double s = 0.0;
      for (int j = 0; j < P; ++j) s += F[j * P + i] * L[b][j];
      Fy[b][i] = s;
    }
  for (int a = 0; a < NQ; ++a)
    for (int b = 0; b < NQ; ++b) {
      double s = 0.0;
      for (int i = 0; i < P; ++i) s += Fy[b][i] * L[a][i];
      Q[a * NQ + b] = s;
    }
}

/* out[t] = sum over leaves b not listed in excl[t] of int_{B_b} G(x_t - y) f_h(y) dy,
 * G = -(1/2pi) log. tx: nt x 2 physical targets; excl_ptr (nt+1) / excl_idx: CSR of
 * excluded leaves per target; centres nl x 2, halfw nl, f nl x P*P. */
void oq_direct_far(int nt, const double* tx, const long long* excl_ptr, const long long* excl_idx, int nl,
                   const double* centres, const double* halfw, const double* f, double* out) {
  int nq2 = NQ * NQ;
  double* Q = (double*)malloc(sizeof(double) * (size_t)nl * nq2);
  double* mass = (double*)malloc(sizeof(double) * (size_t)nl);
#pragma omp parallel for schedule(static)
  for (int b = 0; b < nl; ++b) {
    leaf_at_gauss(f + (size_t)b * P * P, Q + (size_t)b * nq2);
    double m = 0.0;
    for (int k = 0; k < P * P; ++k) m += WT[k] * f[(size_t)b * P * P + k];
    mass[b] = m;
  }
  const double inv2pi = 1.0 / (2.0 * M_PI);
#pragma omp parallel for schedule(dynamic, 4)
  for (int t = 0; t < nt; ++t) {
    double x = tx[2 * t], y = tx[2 * t + 1];
    double tot = 0.0;
    long long e0 = excl_ptr[t], e1 = excl_ptr[t + 1];
    for (int b = 0; b < nl; ++b) {
      int skip = 0;
      for (long long e = e0; e < e1; ++e)
        if (excl_idx[e] == b) {
          skip = 1;
          break;
        }
      if (skip) continue;
      double s = halfw[b];
      double x0 = (x - centres[2 * b]) / s, y0 = (y - centres[2 * b + 1]) / s;
      double integ;
      if (dist_to_square(x0, y0, 0.0, 0.0, 1.0) >= 2.0) {
        const double* Qb = Q + (size_t)b * nq2;
        double acc = 0.0;
        for (int a = 0; a < NQ; ++a) {
          double dx = GX[a] - x0;
          for (int c = 0; c < NQ; ++c) {
            double dy = GX[c] - y0;
            acc += 0.5 * log(dx * dx + dy * dy) * GW[a] * GW[c] * Qb[a * NQ + c];
          }
        }
        integ = acc;
      } else {
        integ = adapt_f(x0, y0, 0.0, 0.0, 1.0, f + (size_t)b * P * P);
      }
      tot += s * s * (log(s) * mass[b] + integ);
    }
    out[t] = -inv2pi * tot;
  }
  free(Q);
  free(mass);
}

/* ---------------------------------------------------------------- gradient
 * (gx, gy) += int_{square} (x0 - y) / |x0 - y|^2 f_h(y) dy  (the x0-gradient of the log
 * integral), same tensor rule on a square at distance >= its side from x0. */
static void square_grad(double x0, double y0, double cx, double cy, double h, const double* F, double* gx, double* gy) {
  double Lx[NQMAX][PMAX], Ly[NQMAX][PMAX], Fy[NQMAX][PMAX];
  for (int a = 0; a < NQ; ++a) lagrange_row(cx + h * GX[a], Lx[a]);
  for (int b = 0; b < NQ; ++b) lagrange_row(cy + h * GX[b], Ly[b]);
  for (int b = 0; b < NQ; ++b)
    for (int i = 0; i < P; ++i) {
      double s = 0.0;
      for (int j = 0; j < P; ++j) s += F[j * P + i] * Ly[b][j];
      Fy[b][i] = s;
    }
  double tx = 0.0, ty = 0.0;
  for (int a = 0; a < NQ; ++a) {
    double dx = x0 - (cx + h * GX[a]);
    for (int b = 0; b < NQ; ++b) {
      double fv = 0.0;
      for (int i = 0; i < P; ++i) fv += Fy[b][i] * Lx[a][i];
      double dy = y0 - (cy + h * GX[b]);
      double w = GW[a] * GW[b] * fv / (dx * dx + dy * dy);
      tx += w * dx;
      ty += w * dy;
    }
  }
  *gx += tx * h * h;
  *gy += ty * h * h;
}

/* Squares of half-width below hmin around x0 are dropped; the kernel is O(1/r), so what they
 * carry is at most about 25 hmin max|f_h| (a disc of radius 4 hmin); hmin = 1e-14 here. */
static void adapt_grad(double x0, double y0, double cx, double cy, double h, const double* F, double hmin, double* gx,
                       double* gy) {
  if (dist_to_square(x0, y0, cx, cy, h) >= 2.0 * h) {
    square_grad(x0, y0, cx, cy, h, F, gx, gy);
    return;
  }
  if (h <= hmin) return;
  double q = 0.5 * h;
  adapt_grad(x0, y0, cx - q, cy - q, q, F, hmin, gx, gy);
  adapt_grad(x0, y0, cx + q, cy - q, q, F, hmin, gx, gy);
  adapt_grad(x0, y0, cx - q, cy + q, q, F, hmin, gx, gy);
  adapt_grad(x0, y0, cx + q, cy + q, q, F, hmin, gx, gy);
}

/* grad[2t], grad[2t+1] = gradient at x_t of sum over all leaves of int_{B_b} G(x_t - y) f_h(y) dy,
 * G = -(1/2pi) log; grad_x log|x - y| = (x - y)/|x - y|^2 and d/dx = (1/s_b) d/dx0. */
void oq_direct_grad(int nt, const double* tx, int nl, const double* centres, const double* halfw, const double* f,
                    double* grad) {
  const double inv2pi = 1.0 / (2.0 * M_PI);
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < nt; ++t) {
    double x = tx[2 * t], y = tx[2 * t + 1];
    double tgx = 0.0, tgy = 0.0;
    for (int b = 0; b < nl; ++b) {
      double s = halfw[b];
      double x0 = (x - centres[2 * b]) / s, y0 = (y - centres[2 * b + 1]) / s;
      double gx = 0.0, gy = 0.0;
      adapt_grad(x0, y0, 0.0, 0.0, 1.0, f + (size_t)b * P * P, 1e-14, &gx, &gy);
      tgx += s * gx;
      tgy += s * gy;
    }
    grad[2 * t] = -inv2pi * tgx;
    grad[2 * t + 1] = -inv2pi * tgy;
  }
}
