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
// rows, so every coupling has rank m. The Dirichlet unknowns are zero, so only the interior rows
// and columns of a block (Bi = m q of them, a contiguous range) enter. The factorization:
//   host   nodes, differentiation matrices, inverse-map factors and interface normals
//   GPU    assembly of the interior blocks A_k (row-equilibrated), the couplings U~_k and the
//          row scales; A_k^-1 for all elements (batched blocked Gauss-Jordan on FP64 MFMA) and
//          R_k = U~_{k-1} A_k^-1 (strip_factor.hip)
//   host   the block elimination of the non-periodic part on m x m pieces only:
//          D_k = A_k + P'_k M_k U~_{k-1}, M_k = E_{k-1}[S, P], E_k = D_k^-1 = A_k^-1 - C_k MG_k R_k
//          (Woodbury, MG_k = M_k (I + R_k[:, V] M_k)^-1, C_k = A_k^-1[:, V]); the sweep matrices
//          F, G, H, their responses to the corner values, and the corner's capacitance matrix
//   GPU    E_k on the interior (the apply's blocks) and the right-hand-side functionals W_k
// Apply (GPU, strip.hip): per-element functionals, the two m-dimensional sweeps, the per-element
// solution product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <exception>
#include <memory>
#include <new>
#include <stdexcept>
#include <thread>
#include <vector>

#include "../../include/volpot.h"
#include "strip.hpp"

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

template <class Fn>
void parallel_for(int n, Fn fn) {  // rethrows the first exception a task threw
  std::atomic<int> next(0);
  std::vector<std::exception_ptr> err(static_cast<size_t>(n));
  auto work = [&]() {
    for (int k; (k = next.fetch_add(1)) < n;) {
      try {
        fn(k);
      } catch (...) {
        err[size_t(k)] = std::current_exception();
      }
    }
  };
  const unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned i = 1; i < nt && i < unsigned(n); ++i) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

struct StripHost {
  int n = 0, q = 0, nr = 0, B = 0, m = 0, Bi = 0, N = 0;  // N: Bi rounded up to a multiple of 16
  std::vector<double> X;    // n * B * 2 node coordinates
  std::vector<double> met;  // n * 6 * B: xi_x, xi_y, eta_x, eta_y, x_xi, y_xi per node
  std::vector<double> nrm;  // n * 2: unit normal of the interface between element k and k + 1
  std::vector<double> Dq, Dr;  // differentiation along the panels (q x q) and across (nr x nr)
};

// Nodes, differentiation matrices, the inverse-map factors of every node and the interface
// normals; the blocks themselves are assembled on the GPU from these (strip_factor.hip).
void assemble(StripHost& S, const double* gamma, const double* gamma_t, int n_gl) {
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
  S.Dq = diff_matrix(tq);
  S.Dr = diff_matrix(tr);
  const Mat& Dq = S.Dq;
  const Mat& Dr = S.Dr;
  // per element and node: the inverse-map factors of D_X = M[xi_x] D_xi + M[eta_x] D_eta (and
  // D_Y), and x_xi, y_xi (the orientation of the interface normal)
  S.met.assign(size_t(n) * 6 * B, 0.0);
  S.nrm.assign(size_t(n) * 2, 0.0);
  parallel_for(n, [&](int k) {
    double* o = S.met.data() + size_t(k) * 6 * B;
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
        if (!(std::fabs(J) > 0.0) || !std::isfinite(J)) throw std::invalid_argument("degenerate element map");
        const size_t r = size_t(i) * q + j;
        o[r] = yeta / J;
        o[B + r] = -xeta / J;
        o[2 * B + r] = -yxi / J;
        o[3 * B + r] = xxi / J;
        o[4 * B + r] = xxi;
        o[5 * B + r] = yxi;
      }
    // interface normal between element k and k + 1: the segment from Gamma's to Gamma~'s shared point
    const double px = Xk[size_t(q - 1) * 2], py = Xk[size_t(q - 1) * 2 + 1];
    const double ptx = Xk[(size_t(nr - 1) * q + q - 1) * 2], pty = Xk[(size_t(nr - 1) * q + q - 1) * 2 + 1];
    const double len = std::hypot(ptx - px, pty - py);
    if (!(len > 0.0) || !std::isfinite(len)) throw std::invalid_argument("degenerate interface");
    S.nrm[size_t(k) * 2] = (pty - py) / len;
    S.nrm[size_t(k) * 2 + 1] = -(ptx - px) / len;
  });
}

// The chain on m x m pieces (row-major), after the GPU has formed A_k^-1 and R_k.
struct Chain {
  std::vector<double> MG, F, G, H, Pz, Pt, K;
};

Mat mul(const Mat& X, const Mat& Y, int r, int s, int t) {  // (r x s)(s x t)
  Mat Z(size_t(r) * t, 0.0);
  for (int i = 0; i < r; ++i)
    for (int l = 0; l < s; ++l) {
      const double x = X[size_t(i) * s + l];
      for (int j = 0; j < t; ++j) Z[size_t(i) * t + j] += x * Y[size_t(l) * t + j];
    }
  return Z;
}

void chain(int n, int m, const std::vector<double>& pieces, Chain& C) {
  const size_t mm = size_t(m) * m;
  auto piece = [&](int k, int which) {
    return Mat(pieces.begin() + long(size_t(k) * 4 * mm + which * mm), pieces.begin() + long(size_t(k) * 4 * mm + (which + 1) * mm));
  };
  Mat I(mm, 0.0);
  for (int a = 0; a < m; ++a) I[size_t(a) * m + a] = 1.0;
  C.MG.assign(size_t(n) * mm, 0.0);
  C.F.assign(size_t(n) * mm, 0.0);
  C.G.assign(size_t(n) * mm, 0.0);
  C.H.assign(size_t(n) * mm, 0.0);
  auto put = [&](std::vector<double>& dst, int k, const Mat& v) { std::copy(v.begin(), v.end(), dst.begin() + long(size_t(k) * mm)); };
  // element 0: E_0 = A_0^-1 (no elimination yet); G_0, H_0 use U~_{n-1} (the corner's terms)
  Mat ESP = piece(0, 0);
  put(C.F, 0, piece(0, 1));
  put(C.G, 0, piece(0, 3));
  put(C.H, 0, piece(0, 2));
  for (int k = 1; k < n; ++k) {
    const Mat aSP = piece(k, 0), aSV = piece(k, 1), rP = piece(k, 2), rV = piece(k, 3);
    Mat Gm = mul(rV, ESP, m, m, m);
    for (size_t e = 0; e < mm; ++e) Gm[e] += I[e];
    const Mat MG = mul(ESP, inverse(Gm, m), m, m, m);
    const Mat T1 = mul(aSV, MG, m, m, m);
    const Mat T1P = mul(T1, rP, m, m, m), T1V = mul(T1, rV, m, m, m);
    Mat Y = mul(rV, MG, m, m, m);
    for (size_t e = 0; e < mm; ++e) Y[e] = I[e] - Y[e];
    Mat Fk(mm);
    for (size_t e = 0; e < mm; ++e) {
      ESP[e] = aSP[e] - T1P[e];
      Fk[e] = aSV[e] - T1V[e];
    }
    put(C.MG, k, MG);
    put(C.F, k, Fk);
    put(C.G, k, mul(Y, rV, m, m, m));
    put(C.H, k, mul(Y, rP, m, m, m));
  }
  // ESP = E_{n-1}[S, P]
  const int m2 = 2 * m;
  // responses of the sweep to its boundary values z_0 = h_lo, t_n = h_hi
  C.Pz.assign(size_t(n) * mm, 0.0);
  for (int a = 0; a < m; ++a) C.Pz[size_t(a) * m + a] = 1.0;
  for (int k = 0; k + 1 < n; ++k) {
    const Mat Fk(C.F.begin() + long(size_t(k) * mm), C.F.begin() + long(size_t(k + 1) * mm));
    const Mat Pk(C.Pz.begin() + long(size_t(k) * mm), C.Pz.begin() + long(size_t(k + 1) * mm));
    put(C.Pz, k + 1, mul(Fk, Pk, m, m, m));
  }
  C.Pt.assign(size_t(n + 1) * m * m2, 0.0);
  for (int a = 0; a < m; ++a) C.Pt[size_t(n) * m * m2 + size_t(a) * m2 + m + a] = 1.0;
  for (int k = n - 1; k >= 1; --k)
    for (int a = 0; a < m; ++a)
      for (int j = 0; j < m2; ++j) {
        double acc = 0.0;
        if (j < m)
          for (int c = 0; c < m; ++c) acc += C.G[size_t(k) * mm + size_t(a) * m + c] * C.Pz[size_t(k) * mm + size_t(c) * m + j];
        for (int c = 0; c < m; ++c)
          acc -= C.H[size_t(k) * mm + size_t(a) * m + c] * C.Pt[size_t(k + 1) * m * m2 + size_t(c) * m2 + j];
        C.Pt[size_t(k) * m * m2 + size_t(a) * m2 + j] = acc;
      }
  // the corner: K = (I + V^T Z)^-1, Z = T^-1 U_c. A column of U_c enters the sweep as a boundary
  // value (-e_j at z_0, or -e_j at t_n), so V^T Z follows from the responses:
  //   j < m:  [-(F_{n-1} Pz_{n-1})[:, j];  -G_0[:, j] + (H_0 Pt_1)[:, j]]
  //   j >= m: [E_{n-1}[S, P][:, j - m];    (H_0 Pt_1)[:, j]]
  const Mat Fl(C.F.begin() + long(size_t(n - 1) * mm), C.F.end());
  const Mat Pl(C.Pz.begin() + long(size_t(n - 1) * mm), C.Pz.end());
  const Mat FP = mul(Fl, Pl, m, m, m);
  const Mat H0(C.H.begin(), C.H.begin() + long(mm));
  const Mat Pt1(C.Pt.begin() + long(size_t(m) * m2), C.Pt.begin() + long(size_t(2) * m * m2));
  const Mat HP = mul(H0, Pt1, m, m, m2);
  Mat Gc(size_t(m2) * m2, 0.0);
  for (int a = 0; a < m; ++a)
    for (int j = 0; j < m2; ++j) {
      Gc[size_t(a) * m2 + j] = j < m ? -FP[size_t(a) * m + j] : ESP[size_t(a) * m + (j - m)];
      Gc[size_t(m + a) * m2 + j] = (j < m ? -C.G[size_t(a) * m + j] : 0.0) + HP[size_t(a) * m2 + j];
    }
  for (int a = 0; a < m2; ++a) Gc[size_t(a) * m2 + a] += 1.0;
  C.K = inverse(Gc, m2);  // throws on a singular corner system
}

}  // namespace

struct volpot_strip_s {
  int n = 0, q = 0, nr = 0;
  std::vector<double> X;  // node coordinates
  int device = -1;
  StripDevice d{};
  char* block = nullptr;
};

namespace {

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// The factorization: host geometry, GPU assembly and inverses, host chain, GPU blocks; the
// apply's arrays in one allocation (s->block).
int strip_factor(volpot_strip_s* s, StripHost& H) {
  const int n = H.n, m = H.m, Bi = H.Bi, N = H.N, B = H.B, q = H.q;
  const size_t mm = size_t(m) * m, m2 = size_t(2) * m;
  if (hipGetDevice(&s->device) != hipSuccess) return VOLPOT_ERR_HIP;
  // the apply's block
  const size_t nEiT = size_t(n) * Bi * Bi, nW = size_t(n) * m2 * Bi, nmm = size_t(n) * mm;
  size_t o = 0;
  const size_t oEiT = o; o += al256(nEiT * 8);
  const size_t oW = o; o += al256(nW * 8);
  const size_t oF = o; o += al256(nmm * 8);
  const size_t oG = o; o += al256(nmm * 8);
  const size_t oH = o; o += al256(nmm * 8);
  const size_t oPz = o; o += al256(nmm * 8);
  const size_t oPt = o; o += al256(size_t(n + 1) * m * m2 * 8);
  const size_t oK = o; o += al256(m2 * m2 * 8);
  const size_t oR = o; o += al256(size_t(n) * B * 8);
  const size_t os = o; o += al256(size_t(n) * m * 8);
  const size_t ow = o; o += al256(size_t(n) * m * 8);
  const size_t oz = o; o += al256(size_t(n + 1) * m * 8);
  const size_t ot = o; o += al256(size_t(n + 1) * m * 8);
  const size_t oh = o; o += al256(m2 * 8);
  if (hipMalloc(&s->block, o) != hipSuccess) { s->block = nullptr; return VOLPOT_ERR_OOM; }
  char* b = s->block;
  // plan-time work memory
  size_t w = 0;
  const size_t wA = w; w += al256(size_t(n) * N * N * 8);
  const size_t wAi = w; w += al256(size_t(n) * N * N * 8);
  const size_t wPv = w; w += al256(size_t(n) * N * 4);
  const size_t wPm = w; w += al256(size_t(n) * kPermInts * 4);
  const size_t wFl = w; w += al256(size_t(n) * 4);
  const size_t wMt = w; w += al256(H.met.size() * 8);
  const size_t wNm = w; w += al256(H.nrm.size() * 8);
  const size_t wDq = w; w += al256(H.Dq.size() * 8);
  const size_t wDr = w; w += al256(H.Dr.size() * 8);
  const size_t wSc = w; w += al256(size_t(n) * Bi * 8);
  const size_t wU = w; w += al256(size_t(n) * m * Bi * 8);
  const size_t wRm = w; w += al256(size_t(n) * m * Bi * 8);
  const size_t wPc = w; w += al256(size_t(n) * 4 * mm * 8);
  const size_t wMG = w; w += al256(nmm * 8);
  const size_t wQ = w; w += al256(size_t(n) * m * Bi * 8);
  char* work = nullptr;
  if (hipMalloc(&work, w) != hipSuccess) return VOLPOT_ERR_OOM;
  int rc = VOLPOT_OK;
  auto fail = [&](int e) { rc = e; return e; };
  do {
    StripFactorDevice f{};
    f.n = n; f.N = N; f.Bi = Bi; f.m = m; f.q = q;
    f.A = reinterpret_cast<double*>(work + wA);
    f.Ainv = reinterpret_cast<double*>(work + wAi);
    f.nr = H.nr; f.B = B;
    f.met = reinterpret_cast<const double*>(work + wMt);
    f.nrm = reinterpret_cast<const double*>(work + wNm);
    f.Dq = reinterpret_cast<const double*>(work + wDq);
    f.Dr = reinterpret_cast<const double*>(work + wDr);
    f.rowsc = reinterpret_cast<double*>(work + wSc);
    f.rs = reinterpret_cast<double*>(b + oR);
    f.piv = reinterpret_cast<int32_t*>(work + wPv);
    f.perm = reinterpret_cast<int32_t*>(work + wPm);
    f.flag = reinterpret_cast<int32_t*>(work + wFl);
    f.U = reinterpret_cast<double*>(work + wU);
    f.R = reinterpret_cast<double*>(work + wRm);
    f.pieces = reinterpret_cast<double*>(work + wPc);
    f.MG = reinterpret_cast<const double*>(work + wMG);
    f.Q = reinterpret_cast<double*>(work + wQ);
    f.W = reinterpret_cast<double*>(b + oW);
    f.EiT = reinterpret_cast<double*>(b + oEiT);
    if (hipMemcpy(work + wMt, H.met.data(), H.met.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(work + wNm, H.nrm.data(), H.nrm.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(work + wDq, H.Dq.data(), H.Dq.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(work + wDr, H.Dr.data(), H.Dr.size() * 8, hipMemcpyHostToDevice) != hipSuccess) { fail(VOLPOT_ERR_HIP); break; }
    if (launch_strip_factor(f, 0, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) { fail(VOLPOT_ERR_HIP); break; }
    std::vector<int32_t> flag(static_cast<size_t>(n));
    std::vector<double> pieces(size_t(n) * 4 * mm);
    if (hipMemcpy(flag.data(), f.flag, size_t(n) * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(pieces.data(), f.pieces, pieces.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) { fail(VOLPOT_ERR_HIP); break; }
    if (std::any_of(flag.begin(), flag.end(), [](int32_t v) { return v != 0; })) { fail(VOLPOT_ERR_ARG); break; }
    Chain C;
    try {
      chain(n, m, pieces, C);
    } catch (const std::bad_alloc&) {
      fail(VOLPOT_ERR_OOM);
      break;
    } catch (...) {
      fail(VOLPOT_ERR_ARG);  // a singular m x m system: degenerate geometry
      break;
    }
    if (hipMemcpy(work + wMG, C.MG.data(), nmm * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b + oF, C.F.data(), nmm * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b + oG, C.G.data(), nmm * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b + oH, C.H.data(), nmm * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b + oPz, C.Pz.data(), nmm * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b + oPt, C.Pt.data(), C.Pt.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b + oK, C.K.data(), C.K.size() * 8, hipMemcpyHostToDevice) != hipSuccess) { fail(VOLPOT_ERR_HIP); break; }
    if (launch_strip_factor(f, 1, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) { fail(VOLPOT_ERR_HIP); break; }
  } while (false);
  (void)hipFree(work);
  if (rc != VOLPOT_OK) return rc;
  StripDevice& d = s->d;
  d.n = n; d.q = q; d.B = B; d.m = m; d.Bi = Bi;
  auto cd = [&](size_t off) { return reinterpret_cast<const double*>(b + off); };
  d.EiT = cd(oEiT); d.W = cd(oW); d.F = cd(oF); d.G = cd(oG); d.H = cd(oH); d.Pz = cd(oPz); d.Pt = cd(oPt);
  d.K = cd(oK); d.rs = cd(oR);
  d.s = reinterpret_cast<double*>(b + os);
  d.w = reinterpret_cast<double*>(b + ow);
  d.z = reinterpret_cast<double*>(b + oz);
  d.t = reinterpret_cast<double*>(b + ot);
  d.h = reinterpret_cast<double*>(b + oh);
  d.chunk = std::max(1, 3072 / (m * m + m));  // two buffers of at most 24 KiB
  return VOLPOT_OK;
}

}  // namespace

extern "C" {

int volpot_strip_nodes(volpot_strip_t s, double* xy) {
  if (!s || !xy) return VOLPOT_ERR_ARG;
  std::memcpy(xy, s->X.data(), s->X.size() * sizeof(double));
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

int volpot_strip_apply_noalloc(volpot_strip_t s, const double* f_dev, double* v_dev, void* hip_stream) {
  if (!s || !f_dev || !v_dev || f_dev == v_dev) return VOLPOT_ERR_ARG;
  const int64_t n = s->d.n, m = s->d.m;
  if ((4 * n + 4) * m > kStripScratchDoubles) return VOLPOT_ERR_ARG;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (s->device != prev) (void)hipSetDevice(s->device);
  double* base = nullptr;
  hipError_t e = strip_scratch(&base);
  if (e == hipSuccess) {
    // every element of the work vectors is written before it is read within one apply, so the
    // previous call's contents need no clearing
    StripDevice d = s->d;
    d.s = base;
    d.w = d.s + n * m;
    d.z = d.w + n * m;
    d.t = d.z + (n + 1) * m;
    d.h = d.t + (n + 1) * m;
    e = launch_strip_solve(d, f_dev, v_dev, reinterpret_cast<hipStream_t>(hip_stream));
  }
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
  s->n = n_panel; s->q = q; s->nr = n_r;
  StripHost H;
  H.n = n_panel; H.q = q; H.nr = n_r; H.B = q * n_r; H.m = n_r - 2; H.Bi = H.m * q; H.N = (H.Bi + 15) / 16 * 16;
  try {
    assemble(H, gamma, gamma_t, n_gl);
  } catch (const std::bad_alloc&) {
    delete s;
    return VOLPOT_ERR_OOM;
  } catch (...) {
    delete s;
    return VOLPOT_ERR_ARG;  // degenerate geometry (a zero-length interface or a singular element map)
  }
  s->X = H.X;
  const int rc = strip_factor(s, H);
  if (rc != VOLPOT_OK) { volpot_strip_destroy(s); return rc; }
  *out = s;
  return VOLPOT_OK;
}

}  // extern "C"
