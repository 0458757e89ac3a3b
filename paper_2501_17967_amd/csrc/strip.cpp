// Strip solve of Sec. 4.3: multidomain spectral collocation for Lap v = f in the strip between
// the boundary Gamma and the fictitious curve Gamma~, v = 0 on both. Element k spans panel k of
// each curve; its grid is X_ij = (1 + r_i)/2 x~_j + (1 - r_i)/2 x_j (second-kind Chebyshev nodes
// across the strip, r = -1 on Gamma, and along the panels, where the panel points come from its
// Gauss-Legendre nodes by polynomial interpolation). Unknowns (i, j), j fastest. Rows: Dirichlet
// on Gamma and Gamma~; the mapped Laplacian (D_X^2 + D_Y^2, D_X = M[xi_x] D_xi + M[eta_x] D_eta)
// at interior nodes; on each element's first column the value equals the previous element's
// last column, on its last column the derivative along the interface normal equals the next
// element's (periodic around the strip).
//
// The matrix is block tridiagonal with a periodic corner. Block k couples to k - 1 only through
// the value rows (a selection of m = n_r - 2 entries) and to k + 1 only through the m derivative
// rows, so every coupling has rank m. Plan time (host): each diagonal block's inverse A_k^-1 (in
// parallel); the block elimination of the non-periodic part, D_k = A_k + P'_k M_k U~_{k-1} with
// the m x m matrix M_k = S_{k-1}^T D_{k-1}^-1 P_{k-1}, whose inverse follows from A_k^-1 by the
// Woodbury identity (sequential, O(B^2 m) per block); the periodic corner is a rank-2m term,
// removed by the Woodbury identity at the global level. Apply (GPU, strip.hip): batched block
// products and two m-dimensional recurrences (forward and backward sweeps), then the corner
// correction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <stdexcept>
#include <thread>
#include <vector>

#include "../../include/volpot.h"
#include "device.hpp"

using namespace vp;

namespace {

using Mat = std::vector<double>;  // row-major

std::vector<double> cheb2(int n) {
  std::vector<double> x(static_cast<size_t>(n));
  for (int j = 0; j < n; ++j) x[size_t(j)] = -std::cos(M_PI * j / (n - 1));
  return x;
}

std::vector<double> bary(const std::vector<double>& x) {
  std::vector<double> w(x.size(), 1.0);
  for (size_t j = 0; j < x.size(); ++j)
    for (size_t k = 0; k < x.size(); ++k)
      if (k != j) w[j] /= (x[j] - x[k]);
  return w;
}

Mat diff_matrix(const std::vector<double>& x) {
  const size_t n = x.size();
  const auto w = bary(x);
  Mat D(n * n, 0.0);
  for (size_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (size_t j = 0; j < n; ++j)
      if (i != j) { D[i * n + j] = (w[j] / w[i]) / (x[i] - x[j]); s += D[i * n + j]; }
    D[i * n + i] = -s;
  }
  return D;
}

void gauss_legendre(int n, std::vector<double>& x) {
  x.assign(size_t(n), 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = n * (z * p1 - p0) / (z * z - 1.0), dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    x[size_t(n - 1 - i)] = z;
  }
}

// inverse of an n x n matrix by LU with partial pivoting (throws if singular)
Mat inverse(Mat A, int n) {
  std::vector<int> piv(static_cast<size_t>(n));
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[size_t(r) * n + c]) > std::fabs(A[size_t(p) * n + c])) p = r;
    if (A[size_t(p) * n + c] == 0.0) throw std::runtime_error("singular block");
    piv[size_t(c)] = p;
    if (p != c)
      for (int j = 0; j < n; ++j) std::swap(A[size_t(c) * n + j], A[size_t(p) * n + j]);
    const double inv = 1.0 / A[size_t(c) * n + c];
    for (int r = c + 1; r < n; ++r) {
      const double l = A[size_t(r) * n + c] * inv;
      A[size_t(r) * n + c] = l;
      if (l != 0.0)
        for (int j = c + 1; j < n; ++j) A[size_t(r) * n + j] -= l * A[size_t(c) * n + j];
    }
  }
  Mat X(size_t(n) * n, 0.0);
  std::vector<double> col(static_cast<size_t>(n));
  for (int e = 0; e < n; ++e) {
    std::fill(col.begin(), col.end(), 0.0);
    col[size_t(e)] = 1.0;
    for (int c = 0; c < n; ++c)  // apply the row swaps
      if (piv[size_t(c)] != c) std::swap(col[size_t(c)], col[size_t(piv[size_t(c)])]);
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < r; ++c) col[size_t(r)] -= A[size_t(r) * n + c] * col[size_t(c)];
    for (int r = n - 1; r >= 0; --r) {
      for (int c = r + 1; c < n; ++c) col[size_t(r)] -= A[size_t(r) * n + c] * col[size_t(c)];
      col[size_t(r)] /= A[size_t(r) * n + r];
    }
    for (int r = 0; r < n; ++r) X[size_t(r) * n + e] = col[size_t(r)];
  }
  return X;
}

struct StripHost {
  int n = 0, q = 0, nr = 0, B = 0, m = 0;
  std::vector<double> X;     // n * B * 2 node coordinates
  std::vector<int8_t> pde;   // B: PDE row flags (same in every element)
  std::vector<Mat> A;        // diagonal blocks (B x B)
  std::vector<Mat> Ut;       // m x B: derivative rows of block k acting on block k+1
  std::vector<int> Prow, Pvrow, Scol, Lcol;  // m each: derivative rows, value rows, last column, first column
  std::vector<Mat> E;        // D_k^-1 (B x B)
  std::vector<double> rs;    // n * B row scales of the PDE rows (1 elsewhere)
};

void build_blocks(StripHost& S, const double* gamma, const double* gamma_t, int n_gl) {
  const int n = S.n, q = S.q, nr = S.nr, B = S.B;
  std::vector<double> sg;
  gauss_legendre(n_gl, sg);
  const auto tq = cheb2(q), tr = cheb2(nr);
  const auto wg = bary(sg);
  // interpolation from the Gauss-Legendre nodes to the Chebyshev nodes along a panel
  Mat Ei(size_t(q) * n_gl, 0.0);
  for (int a = 0; a < q; ++a) {
    double s = 0.0;
    int hit = -1;
    for (int b = 0; b < n_gl; ++b)
      if (tq[size_t(a)] == sg[size_t(b)]) hit = b;
    for (int b = 0; b < n_gl; ++b) {
      Ei[size_t(a) * n_gl + b] = hit >= 0 ? (b == hit) : wg[size_t(b)] / (tq[size_t(a)] - sg[size_t(b)]);
      s += Ei[size_t(a) * n_gl + b];
    }
    for (int b = 0; b < n_gl; ++b) Ei[size_t(a) * n_gl + b] /= s;
  }
  S.X.assign(size_t(n) * B * 2, 0.0);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < q; ++j) {
      double x = 0, y = 0, xt = 0, yt = 0;
      for (int b = 0; b < n_gl; ++b) {
        const double e = Ei[size_t(j) * n_gl + b];
        x += e * gamma[(size_t(k) * n_gl + b) * 2];
        y += e * gamma[(size_t(k) * n_gl + b) * 2 + 1];
        xt += e * gamma_t[(size_t(k) * n_gl + b) * 2];
        yt += e * gamma_t[(size_t(k) * n_gl + b) * 2 + 1];
      }
      for (int i = 0; i < nr; ++i) {
        const double a = 0.5 * (1 + tr[size_t(i)]), c = 0.5 * (1 - tr[size_t(i)]);
        S.X[((size_t(k) * B) + size_t(i) * q + j) * 2] = a * xt + c * x;
        S.X[((size_t(k) * B) + size_t(i) * q + j) * 2 + 1] = a * yt + c * y;
      }
    }
  const Mat Dq = diff_matrix(tq), Dr = diff_matrix(tr);
  S.pde.assign(size_t(B), 0);
  S.m = nr - 2;
  S.Prow.clear(); S.Pvrow.clear(); S.Scol.clear(); S.Lcol.clear();
  for (int i = 1; i < nr - 1; ++i) {
    S.Pvrow.push_back(i * q);             // value rows (first column)
    S.Prow.push_back(i * q + q - 1);      // derivative rows (last column)
    S.Scol.push_back(i * q + q - 1);      // last-column unknowns (read by the next element's value rows)
    S.Lcol.push_back(i * q);              // first-column unknowns (read by the previous element's derivative rows)
    for (int j = 1; j < q - 1; ++j) S.pde[size_t(i) * q + j] = 1;
  }
  // per element: DX, DY as sparse rows (nonzeros in the same grid row and column)
  struct Ops { Mat DX, DY; std::vector<double> xxi, yxi; };
  std::vector<Ops> ops(static_cast<size_t>(n));
  auto make_ops = [&](int k) {
    Ops o;
    o.DX.assign(size_t(B) * B, 0.0);
    o.DY.assign(size_t(B) * B, 0.0);
    o.xxi.assign(size_t(B), 0.0);
    o.yxi.assign(size_t(B), 0.0);
    const double* Xk = S.X.data() + size_t(k) * B * 2;
    for (int i = 0; i < nr; ++i)
      for (int j = 0; j < q; ++j) {
        double xxi = 0, yxi = 0, xeta = 0, yeta = 0;
        for (int c = 0; c < q; ++c) {
          xxi += Dq[size_t(j) * q + c] * Xk[(size_t(i) * q + c) * 2];
          yxi += Dq[size_t(j) * q + c] * Xk[(size_t(i) * q + c) * 2 + 1];
        }
        for (int c = 0; c < nr; ++c) {
          xeta += Dr[size_t(i) * nr + c] * Xk[(size_t(c) * q + j) * 2];
          yeta += Dr[size_t(i) * nr + c] * Xk[(size_t(c) * q + j) * 2 + 1];
        }
        const double J = xxi * yeta - xeta * yxi;
        const double xi_x = yeta / J, xi_y = -xeta / J, eta_x = -yxi / J, eta_y = xxi / J;
        const int row = i * q + j;
        o.xxi[size_t(row)] = xxi;
        o.yxi[size_t(row)] = yxi;
        for (int c = 0; c < q; ++c) {
          o.DX[size_t(row) * B + i * q + c] += xi_x * Dq[size_t(j) * q + c];
          o.DY[size_t(row) * B + i * q + c] += xi_y * Dq[size_t(j) * q + c];
        }
        for (int c = 0; c < nr; ++c) {
          o.DX[size_t(row) * B + c * q + j] += eta_x * Dr[size_t(i) * nr + c];
          o.DY[size_t(row) * B + c * q + j] += eta_y * Dr[size_t(i) * nr + c];
        }
      }
    ops[size_t(k)] = std::move(o);
  };
  for (int k = 0; k < n; ++k) make_ops(k);
  S.A.assign(size_t(n), Mat());
  S.Ut.assign(size_t(n), Mat());
  S.rs.assign(size_t(n) * B, 1.0);
  for (int k = 0; k < n; ++k) {
    const Ops& o = ops[size_t(k)];
    const Ops& on = ops[size_t((k + 1) % n)];
    Mat A(size_t(B) * B, 0.0);
    // interface normal between element k and k + 1: the segment from Gamma's to Gamma~'s shared point
    const double* Xk = S.X.data() + size_t(k) * B * 2;
    const double px = Xk[size_t(q - 1) * 2], py = Xk[size_t(q - 1) * 2 + 1];
    const double ptx = Xk[(size_t(nr - 1) * q + q - 1) * 2], pty = Xk[(size_t(nr - 1) * q + q - 1) * 2 + 1];
    const double len = std::hypot(ptx - px, pty - py);
    double nx = (pty - py) / len, ny = -(ptx - px) / len;
    Mat Ut(size_t(S.m) * B, 0.0);
    for (int i = 0; i < nr; ++i)
      for (int j = 0; j < q; ++j) {
        const int row = i * q + j;
        if (i == 0 || i == nr - 1 || j == 0) {
          A[size_t(row) * B + row] = 1.0;  // Dirichlet, or the value row (its coupling is a selection)
        } else if (j == q - 1) {
          double sx = nx, sy = ny;
          if (sx * o.xxi[size_t(row)] + sy * o.yxi[size_t(row)] < 0) { sx = -sx; sy = -sy; }
          for (int c = 0; c < B; ++c) A[size_t(row) * B + c] = sx * o.DX[size_t(row) * B + c] + sy * o.DY[size_t(row) * B + c];
          const int nrow = i * q;  // the next element's first-column node on this interface
          for (int c = 0; c < B; ++c)
            Ut[size_t(i - 1) * B + c] = -(sx * on.DX[size_t(nrow) * B + c] + sy * on.DY[size_t(nrow) * B + c]);
        } else {  // Laplacian row: (DX DX + DY DY)[row], through the sparse rows of DX, DY
          for (int c = 0; c < B; ++c) {
            const double ax = o.DX[size_t(row) * B + c], ay = o.DY[size_t(row) * B + c];
            if (ax == 0.0 && ay == 0.0) continue;
            for (int d = 0; d < B; ++d)
              A[size_t(row) * B + d] += ax * o.DX[size_t(c) * B + d] + ay * o.DY[size_t(c) * B + d];
          }
        }
      }
    // Row equilibration: the Laplacian rows have 1-norms up to ~1e7 (spectral second derivatives
    // on thin elements), the Dirichlet and value rows 1 or 2. Scaling the PDE and derivative rows
    // to unit 1-norm (the derivative rows together with their coupling to element k + 1) leaves
    // the solution unchanged and keeps the block inverses and the recurrences well conditioned.
    // The value rows keep their unit coefficients (norm 2), so the coupling to k - 1 stays a
    // selection; the right-hand side of a PDE row is scaled with it (rs, applied on the GPU).
    for (int i = 1; i < nr - 1; ++i)
      for (int j = 1; j < q; ++j) {
        const int row = i * q + j;
        double nrm = 0.0;
        for (int c = 0; c < B; ++c) nrm += std::fabs(A[size_t(row) * B + c]);
        if (j == q - 1)
          for (int c = 0; c < B; ++c) nrm += std::fabs(Ut[size_t(i - 1) * B + c]);
        const double sc = 1.0 / nrm;
        for (int c = 0; c < B; ++c) A[size_t(row) * B + c] *= sc;
        if (j == q - 1)
          for (int c = 0; c < B; ++c) Ut[size_t(i - 1) * B + c] *= sc;
        else
          S.rs[size_t(k) * B + row] = sc;
      }
    S.A[size_t(k)] = std::move(A);
    S.Ut[size_t(k)] = std::move(Ut);
  }
}

// E_k = D_k^-1 for the non-periodic block-tridiagonal part, from A_k^-1 (parallel) and the
// rank-m chain M_k = S^T E_{k-1} P (sequential).
void factor(StripHost& S) {
  const int n = S.n, B = S.B, m = S.m;
  std::vector<Mat> Ainv(static_cast<size_t>(n));
  std::atomic<int> next(0);
  std::vector<std::exception_ptr> err(static_cast<size_t>(n));
  auto work = [&]() {
    for (int k; (k = next.fetch_add(1)) < n;) {
      try {
        Ainv[size_t(k)] = inverse(S.A[size_t(k)], B);
      } catch (...) {
        err[size_t(k)] = std::current_exception();
      }
    }
  };
  const unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned i = 1; i < nt; ++i) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  S.E.assign(size_t(n), Mat());
  S.E[0] = Ainv[0];
  for (int k = 1; k < n; ++k) {
    const Mat& Ep = S.E[size_t(k - 1)];
    const Mat& Ai = Ainv[size_t(k)];
    const Mat& Up = S.Ut[size_t(k - 1)];  // m x B, acting on block k
    // M = S^T E_{k-1} P: E_{k-1}[last-column node, derivative row]   (m x m)
    Mat M(size_t(m) * m);
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) M[size_t(a) * m + b] = Ep[size_t(S.Scol[size_t(a)]) * B + S.Prow[size_t(b)]];
    // D_k = A_k + P'_k M U~_{k-1}; D_k^-1 = Ai - C M G^-1 R, C = Ai P' (B x m), R = U~ Ai (m x B),
    // G = I + (R P') M
    Mat C(size_t(B) * m), R(size_t(m) * B, 0.0);
    for (int r = 0; r < B; ++r)
      for (int b = 0; b < m; ++b) C[size_t(r) * m + b] = Ai[size_t(r) * B + S.Pvrow[size_t(b)]];
    for (int a = 0; a < m; ++a)
      for (int c = 0; c < B; ++c) {
        const double u = Up[size_t(a) * B + c];
        if (u == 0.0) continue;
        for (int d = 0; d < B; ++d) R[size_t(a) * B + d] += u * Ai[size_t(c) * B + d];
      }
    Mat G(size_t(m) * m, 0.0);
    for (int a = 0; a < m; ++a) {
      G[size_t(a) * m + a] = 1.0;
      for (int b = 0; b < m; ++b) {
        double s = 0.0;
        for (int c = 0; c < m; ++c) s += R[size_t(a) * B + S.Pvrow[size_t(c)]] * M[size_t(c) * m + b];
        G[size_t(a) * m + b] += s;
      }
    }
    const Mat Gi = inverse(G, m);
    Mat MG(size_t(m) * m, 0.0);  // M G^-1
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) {
        double s = 0.0;
        for (int c = 0; c < m; ++c) s += M[size_t(a) * m + c] * Gi[size_t(c) * m + b];
        MG[size_t(a) * m + b] = s;
      }
    Mat CMG(size_t(B) * m, 0.0);
    for (int r = 0; r < B; ++r)
      for (int b = 0; b < m; ++b) {
        double s = 0.0;
        for (int c = 0; c < m; ++c) s += C[size_t(r) * m + c] * MG[size_t(c) * m + b];
        CMG[size_t(r) * m + b] = s;
      }
    Mat Ek = Ai;
    for (int r = 0; r < B; ++r)
      for (int b = 0; b < m; ++b) {
        const double cmg = CMG[size_t(r) * m + b];
        for (int d = 0; d < B; ++d) Ek[size_t(r) * B + d] -= cmg * R[size_t(b) * B + d];
      }
    S.E[size_t(k)] = std::move(Ek);
  }
}

// x = T^-1 b for the non-periodic part on the host (plan time: the corner columns)
void host_tsolve(const StripHost& S, const double* b, double* x) {
  const int n = S.n, B = S.B, m = S.m;
  std::vector<double> y(static_cast<size_t>(n) * B), rhs(static_cast<size_t>(B));
  for (int k = 0; k < n; ++k) {
    for (int r = 0; r < B; ++r) rhs[size_t(r)] = b[size_t(k) * B + r];
    if (k > 0)  // b_k - L_k y_{k-1}: the value rows add the previous element's last column
      for (int a = 0; a < m; ++a) rhs[size_t(S.Pvrow[size_t(a)])] += y[size_t(k - 1) * B + S.Scol[size_t(a)]];
    for (int r = 0; r < B; ++r) {
      double s = 0.0;
      for (int c = 0; c < B; ++c) s += S.E[size_t(k)][size_t(r) * B + c] * rhs[size_t(c)];
      y[size_t(k) * B + r] = s;
    }
  }
  for (int r = 0; r < B; ++r) x[size_t(n - 1) * B + r] = y[size_t(n - 1) * B + r];
  for (int k = n - 2; k >= 0; --k) {
    std::vector<double> t(size_t(m), 0.0);  // U~_k x_{k+1}
    for (int a = 0; a < m; ++a)
      for (int c = 0; c < B; ++c) t[size_t(a)] += S.Ut[size_t(k)][size_t(a) * B + c] * x[size_t(k + 1) * B + c];
    for (int r = 0; r < B; ++r) {
      double s = 0.0;  // E_k P t
      for (int a = 0; a < m; ++a) s += S.E[size_t(k)][size_t(r) * B + S.Prow[size_t(a)]] * t[size_t(a)];
      x[size_t(k) * B + r] = y[size_t(k) * B + r] - s;
    }
  }
}

// Arrays of the three-launch apply. With Bi = m q the interior rows (1 <= i <= n_r - 2, a
// contiguous range q .. B - q - 1 of each element), the Dirichlet rows of D_k are identity rows,
// so x is zero there and only the interior block of E_k = D_k^-1 is ever applied.
//   rhs pass:  s_k = E_k[S, :] b_k,  w_k = U~_{k-1} E_k b_k         (W_k, 2m x Bi; U~_{-1} = U~_{n-1})
//   sweep:     z_0 = 0, z_{k+1} = s_k + F_k z_k;  g_k = w_k + G_k z_k;
//              t_n = 0, t_k = g_k - H_k t_{k+1} (k = n-1 .. 1);
//              h = K [z_n; w_0 - H_0 t_1]                          (the periodic corner, Woodbury)
//   solution:  z*_k = z_k + Pz_k h_lo,  t*_{k+1} = t_{k+1} + Pt_{k+1} h,
//              x_k = E_k (b_k + P' z*_k - P t*_{k+1})             (interior block, Bi x Bi)
// The corrected solution T^-1 (b - U_c h) is the non-periodic sweep started from z_0 = h_lo and
// t_n = h_hi (U_c injects exactly there), and the sweep is linear in those two boundary values:
// Pz_k, Pt_k are its responses, precomputed here.
struct StripArrays {
  int n = 0, q = 0, B = 0, m = 0, Bi = 0;
  std::vector<double> EiT, W, F, G, Hm, Pz, Pt, K, rs;
};

template <class Fn>
void parallel_for(int n, Fn fn) {
  std::atomic<int> next(0);
  auto work = [&]() {
    for (int k; (k = next.fetch_add(1)) < n;) fn(k);
  };
  const unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned i = 1; i < nt && i < unsigned(n); ++i) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
}

void apply_arrays(const StripHost& H, StripArrays& R) {
  const int n = H.n, B = H.B, m = H.m, q = H.q, Bi = B - 2 * q;
  R.n = n; R.q = q; R.B = B; R.m = m; R.Bi = Bi;
  const size_t mm = size_t(m) * m;
  R.EiT.assign(size_t(n) * Bi * Bi, 0.0);
  R.W.assign(size_t(n) * 2 * m * Bi, 0.0);
  R.F.assign(size_t(n) * mm, 0.0);
  R.G.assign(size_t(n) * mm, 0.0);
  R.Hm.assign(size_t(n) * mm, 0.0);
  parallel_for(n, [&](int k) {
    const Mat& E = H.E[size_t(k)];
    const Mat& U = H.Ut[size_t((k + n - 1) % n)];  // derivative rows of element k - 1 acting on k
    for (int c = 0; c < Bi; ++c)
      for (int p = 0; p < Bi; ++p) R.EiT[(size_t(k) * Bi + c) * Bi + p] = E[size_t(q + p) * B + q + c];
    std::vector<double> UE(size_t(m) * B, 0.0);  // U~ E_k (m x B)
    for (int a = 0; a < m; ++a)
      for (int r = 0; r < B; ++r) {
        const double u = U[size_t(a) * B + r];
        if (u == 0.0) continue;
        for (int c = 0; c < B; ++c) UE[size_t(a) * B + c] += u * E[size_t(r) * B + c];
      }
    double* W = R.W.data() + size_t(k) * 2 * m * Bi;
    for (int a = 0; a < m; ++a)
      for (int c = 0; c < Bi; ++c) {
        W[size_t(a) * Bi + c] = E[size_t(H.Scol[size_t(a)]) * B + q + c];
        W[size_t(m + a) * Bi + c] = UE[size_t(a) * B + q + c];
      }
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) {
        R.F[size_t(k) * mm + size_t(a) * m + b] = E[size_t(H.Scol[size_t(a)]) * B + H.Pvrow[size_t(b)]];
        R.G[size_t(k) * mm + size_t(a) * m + b] = UE[size_t(a) * B + H.Pvrow[size_t(b)]];
        R.Hm[size_t(k) * mm + size_t(a) * m + b] = UE[size_t(a) * B + H.Prow[size_t(b)]];
      }
  });
  // responses of the sweep to its boundary values
  const int m2 = 2 * m;
  R.Pz.assign(size_t(n) * mm, 0.0);
  for (int a = 0; a < m; ++a) R.Pz[size_t(a) * m + a] = 1.0;
  for (int k = 0; k + 1 < n; ++k)
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) {
        double acc = 0.0;
        for (int c = 0; c < m; ++c) acc += R.F[size_t(k) * mm + size_t(a) * m + c] * R.Pz[size_t(k) * mm + size_t(c) * m + b];
        R.Pz[size_t(k + 1) * mm + size_t(a) * m + b] = acc;
      }
  R.Pt.assign(size_t(n + 1) * m * m2, 0.0);
  for (int a = 0; a < m; ++a) R.Pt[size_t(n) * m * m2 + size_t(a) * m2 + m + a] = 1.0;
  for (int k = n - 1; k >= 1; --k)
    for (int a = 0; a < m; ++a)
      for (int j = 0; j < m2; ++j) {
        double acc = 0.0;
        if (j < m)
          for (int c = 0; c < m; ++c) acc += R.G[size_t(k) * mm + size_t(a) * m + c] * R.Pz[size_t(k) * mm + size_t(c) * m + j];
        for (int c = 0; c < m; ++c)
          acc -= R.Hm[size_t(k) * mm + size_t(a) * m + c] * R.Pt[size_t(k + 1) * m * m2 + size_t(c) * m2 + j];
        R.Pt[size_t(k) * m * m2 + size_t(a) * m2 + j] = acc;
      }
  // the corner: Z = T^-1 U_c (columns -e at element 0's value rows, +e at element n-1's
  // derivative rows), K = (I + V^T Z)^-1 with V^T = [element n-1's last column; U~_{n-1} on element 0]
  const size_t N = size_t(n) * B;
  std::vector<double> Z(N * m2);
  parallel_for(m2, [&](int j) {
    std::vector<double> col(N, 0.0), sol(N);
    if (j < m) col[size_t(H.Pvrow[size_t(j)])] = -1.0;
    else col[size_t(n - 1) * B + H.Prow[size_t(j - m)]] = 1.0;
    host_tsolve(H, col.data(), sol.data());
    for (size_t r = 0; r < N; ++r) Z[r * m2 + j] = sol[r];
  });
  Mat Gc(size_t(m2) * m2, 0.0);
  for (int a = 0; a < m2; ++a) {
    Gc[size_t(a) * m2 + a] = 1.0;
    for (int j = 0; j < m2; ++j) {
      double v;
      if (a < m) {
        v = Z[(size_t(n - 1) * B + H.Scol[size_t(a)]) * m2 + j];
      } else {
        v = 0.0;
        for (int r = 0; r < B; ++r) v += H.Ut[size_t(n - 1)][size_t(a - m) * B + r] * Z[size_t(r) * m2 + j];
      }
      Gc[size_t(a) * m2 + j] += v;
    }
  }
  R.K = inverse(Gc, m2);  // throws on a singular corner system
  R.rs = H.rs;
}

}  // namespace

struct volpot_strip_s {
  StripHost H;
  int device = -1;
  StripDevice d{};
  char* block = nullptr;
};

// Device copy of everything the apply reads, and its work vectors, in one allocation.
static int strip_upload(volpot_strip_s* s, const StripArrays& R) {
  const int n = R.n, m = R.m;
  const size_t N = size_t(n) * R.B;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const std::vector<double>* in[] = {&R.EiT, &R.W, &R.F, &R.G, &R.Hm, &R.Pz, &R.Pt, &R.K, &R.rs};
  size_t off[9], o = 0;
  for (int i = 0; i < 9; ++i) { off[i] = o; o += al(in[i]->size() * 8); }
  const size_t os = o; o += al(size_t(n) * m * 8);
  const size_t ow = o; o += al(size_t(n) * m * 8);
  const size_t oz = o; o += al(size_t(n + 1) * m * 8);
  const size_t ot = o; o += al(size_t(n + 1) * m * 8);
  const size_t oh = o; o += al(size_t(2 * m) * 8);
  (void)N;
  if (hipGetDevice(&s->device) != hipSuccess) return VOLPOT_ERR_HIP;
  if (hipMalloc(&s->block, o) != hipSuccess) { s->block = nullptr; return VOLPOT_ERR_OOM; }
  char* b = s->block;
  for (int i = 0; i < 9; ++i)
    if (hipMemcpy(b + off[i], in[i]->data(), in[i]->size() * 8, hipMemcpyHostToDevice) != hipSuccess) return VOLPOT_ERR_HIP;
  StripDevice& d = s->d;
  d.n = n; d.q = R.q; d.B = R.B; d.m = m; d.Bi = R.Bi;
  auto cd = [&](int i) { return reinterpret_cast<const double*>(b + off[i]); };
  d.EiT = cd(0); d.W = cd(1); d.F = cd(2); d.G = cd(3); d.H = cd(4); d.Pz = cd(5); d.Pt = cd(6); d.K = cd(7); d.rs = cd(8);
  d.s = reinterpret_cast<double*>(b + os);
  d.w = reinterpret_cast<double*>(b + ow);
  d.z = reinterpret_cast<double*>(b + oz);
  d.t = reinterpret_cast<double*>(b + ot);
  d.h = reinterpret_cast<double*>(b + oh);
  d.chunk = std::max(1, 3072 / (m * m + m));  // two buffers of at most 24 KiB
  return VOLPOT_OK;
}

extern "C" {

int volpot_strip_nodes(volpot_strip_t s, double* xy) {
  if (!s || !xy) return VOLPOT_ERR_ARG;
  std::memcpy(xy, s->H.X.data(), s->H.X.size() * sizeof(double));
  return VOLPOT_OK;
}

int volpot_strip_apply(volpot_strip_t s, const double* f_dev, double* v_dev, void* hip_stream) {
  if (!s || !f_dev || !v_dev || f_dev == v_dev) return VOLPOT_ERR_ARG;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (s->device != prev) (void)hipSetDevice(s->device);
  const hipError_t e = launch_strip_solve(s->d, f_dev, v_dev, reinterpret_cast<hipStream_t>(hip_stream));
  if (s->device != prev && prev >= 0) (void)hipSetDevice(prev);
  return e == hipSuccess ? VOLPOT_OK : VOLPOT_ERR_HIP;
}

void volpot_strip_destroy(volpot_strip_t s) {
  if (!s) return;
  if (s->block) {
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (s->device >= 0 && s->device != prev) (void)hipSetDevice(s->device);
    (void)hipFree(s->block);
    if (s->device >= 0 && s->device != prev && prev >= 0) (void)hipSetDevice(prev);
  }
  delete s;
}

int volpot_strip_plan(int32_t n_panel, int32_t n_gl, const double* gamma, const double* gamma_t, int32_t q, int32_t n_r,
                      volpot_strip_t* out) {
  if (!out || !gamma || !gamma_t || n_panel < 3 || n_gl < 2 || n_gl > 64 || q < 4 || n_r < 4 || q > 32 || n_r > 32 ||
      q * n_r > 1024)
    return VOLPOT_ERR_ARG;
  for (int64_t i = 0; i < int64_t(n_panel) * n_gl * 2; ++i)
    if (!std::isfinite(gamma[i]) || !std::isfinite(gamma_t[i])) return VOLPOT_ERR_ARG;
  auto* s = new (std::nothrow) volpot_strip_s();
  if (!s) return VOLPOT_ERR_OOM;
  StripHost& H = s->H;
  H.n = n_panel; H.q = q; H.nr = n_r; H.B = q * n_r;
  try {
    build_blocks(H, gamma, gamma_t, n_gl);
    factor(H);
  } catch (const std::bad_alloc&) {
    delete s;
    return VOLPOT_ERR_OOM;
  } catch (...) {
    delete s;
    return VOLPOT_ERR_ARG;  // a singular block: degenerate element geometry
  }
  StripArrays R;
  try {
    apply_arrays(H, R);
  } catch (const std::bad_alloc&) {
    delete s;
    return VOLPOT_ERR_OOM;
  } catch (...) {
    delete s;
    return VOLPOT_ERR_ARG;  // a singular corner system
  }
  std::vector<Mat>().swap(H.A);  // the host blocks are no longer needed
  std::vector<Mat>().swap(H.E);
  std::vector<Mat>().swap(H.Ut);
  int rc = strip_upload(s, R);
  if (rc != VOLPOT_OK) { volpot_strip_destroy(s); return rc; }
  *out = s;
  return VOLPOT_OK;
}

}  // extern "C"
