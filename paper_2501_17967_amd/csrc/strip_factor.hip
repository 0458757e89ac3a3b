// HIP kernels of the strip factorization (plan time; the host side is strip.cpp).
//
//   strip_rows_kernel     the row scales (unit 1-norm of each PDE and derivative row) and the
//                         couplings U~_k, one wave per interior row.
//   strip_fill_kernel     the row-equilibrated interior blocks A_k, column-major, one thread per
//                         row of a 16-column tile (the entries of the mapped Laplacian and of the
//                         normal derivative written out from the inverse-map factors).
// The inverse of every interior block A_k (N x N, column-major, N a multiple of 16, identity
// padding) by blocked Gauss-Jordan elimination with partial pivoting, in 16-column panels, each
// panel as two launches over all elements so that the whole device takes part:
//   strip_panel_kernel    one workgroup per element: the panel's elimination with its rows held
//                         in registers (pivot by a block-wide argmax, row exchange and broadcast
//                         through LDS); the panel then holds T's columns (T the panel's
//                         transformation), and the panel's row exchanges are stored as one net
//                         permutation of at most 32 rows.
//   strip_update_kernel   one workgroup per (element, other 16-column tile): that tile's rows
//                         permuted and updated as A[:, c] += (T - I_panel) A_old[panel rows, c],
//                         a rank-16 product on FP64 MFMA (v_mfma_f64_16x16x4f64).
//   strip_gather_kernel   the columns of the result gathered through the inverse of the row
//                         exchanges (in-place Gauss-Jordan yields (PA)^-1 = A^-1 P^-1).
//   strip_couple_kernel   R_k = U~_{k-1} A_k^-1 (m x Bi), one wave per column.
//   strip_pieces_kernel   the m x m pieces the host chain needs: A^-1[S, P], A^-1[S, V],
//                         R[:, P], R[:, V].
//   strip_q_kernel        Q_k = MG_k R_k, and the lower half of W_k, (I - R[:, V] MG_k) R_k.
//   strip_e_kernel        E_k = A_k^-1 - A_k^-1[:, V] Q_k written column-major on the interior
//                         (the solution kernel's layout), and the upper half of W_k, E_k[S, :].
// S = P: the derivative rows / last-column unknowns (interior index a q + q - 1), V: the value
// rows (a q), a = 0 .. m - 1.
#include <hip/hip_runtime.h>

#include "strip.hpp"

namespace vp {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kInvThreads = 512;  // panel workgroup: 8 waves
constexpr int kNb = 16;           // panel width (one MFMA tile)
constexpr int kRpt = 2;           // panel rows per thread: N <= 1024
constexpr int kUpdThreads = 256;  // update workgroup: 4 waves, one 16-row tile each at a time

__device__ __forceinline__ bool better(double v, int i, double bv, int bi) { return v > bv || (v == bv && i < bi); }

// Panel j0 .. j0 + 15 of element blockIdx.x. perm[k] receives the net row permutation of the
// panel's exchanges: count, then rows (destinations) and the old rows that end up there.
__global__ void __launch_bounds__(kInvThreads) strip_panel_kernel(StripFactorDevice f, int j0) {
  const int N = f.N, k = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* a = f.A + size_t(k) * N * N;
  __shared__ double prow[kNb], xrow[kNb];
  __shared__ double redv[kInvThreads / 64];
  __shared__ int redi[kInvThreads / 64];
  __shared__ int pivs[kNb];
  if (tid == 0 && j0 == 0) f.flag[k] = 0;
  // panel rows tid + 512 r in registers
  double pv[kRpt][kNb];
#pragma unroll
  for (int r = 0; r < kRpt; ++r) {
    const int row = tid + kInvThreads * r;
#pragma unroll
    for (int c = 0; c < kNb; ++c) pv[r][c] = row < N ? a[size_t(j0 + c) * N + row] : 0.0;
  }
#pragma unroll
  for (int jj = 0; jj < kNb; ++jj) {
    const int j = j0 + jj;
    double bv = -1.0;
    int bi = N;
#pragma unroll
    for (int r = 0; r < kRpt; ++r) {
      const int row = tid + kInvThreads * r;
      if (row >= j && row < N && better(fabs(pv[r][jj]), row, bv, bi)) {
        bv = fabs(pv[r][jj]);
        bi = row;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { redv[wave] = bv; redi[wave] = bi; }
    __syncthreads();
    bv = redv[0];
    bi = redi[0];
#pragma unroll
    for (int w = 1; w < kInvThreads / 64; ++w)
      if (better(redv[w], redi[w], bv, bi)) { bv = redv[w]; bi = redi[w]; }
    // the pivot row (the same in every thread); no usable candidate (a zero or non-finite
    // column): no exchange, and the block is reported singular
    const int pr = bi < N ? bi : j;
    if (tid == 0) {
      pivs[jj] = pr;
      f.piv[size_t(k) * N + j] = pr;
      if (!(bv > 0.0)) f.flag[k] = 1;
    }
    // exchange rows j and pr of the panel; prow = the new row j (unscaled)
#pragma unroll
    for (int r = 0; r < kRpt; ++r) {
      const int row = tid + kInvThreads * r;
      if (row == pr)
#pragma unroll
        for (int c = 0; c < kNb; ++c) prow[c] = pv[r][c];
      if (row == j && pr != j)
#pragma unroll
        for (int c = 0; c < kNb; ++c) xrow[c] = pv[r][c];
    }
    __syncthreads();
    double pj[kNb];
#pragma unroll
    for (int c = 0; c < kNb; ++c) pj[c] = prow[c];
    const double ip = 1.0 / (bv > 0.0 ? pj[jj] : 1.0);
#pragma unroll
    for (int c = 0; c < kNb; ++c) pj[c] *= ip;  // the scaled pivot row
#pragma unroll
    for (int r = 0; r < kRpt; ++r) {
      const int row = tid + kInvThreads * r;
      if (row == pr && pr != j)
#pragma unroll
        for (int c = 0; c < kNb; ++c) pv[r][c] = xrow[c];
      if (row == j) {
#pragma unroll
        for (int c = 0; c < kNb; ++c) pv[r][c] = c == jj ? ip : pj[c];
      } else {
        const double fm = pv[r][jj];
#pragma unroll
        for (int c = 0; c < kNb; ++c) pv[r][c] = c == jj ? -fm * ip : fma(-fm, pj[c], pv[r][c]);
      }
    }
  }
  // the panel now holds T's columns j0 .. j0 + 15
#pragma unroll
  for (int r = 0; r < kRpt; ++r) {
    const int row = tid + kInvThreads * r;
    if (row < N)
#pragma unroll
      for (int c = 0; c < kNb; ++c) a[size_t(j0 + c) * N + row] = pv[r][c];
  }
  // net permutation of the rows the exchanges touched: entries 0 .. 15 are rows j0 .. j0 + 15
  if (tid == 0) {
    int pdst[2 * kNb], psrc[2 * kNb];
    int cnt = kNb;
    for (int e = 0; e < kNb; ++e) { pdst[e] = j0 + e; psrc[e] = j0 + e; }
    for (int jj = 0; jj < kNb; ++jj) {
      const int pr = pivs[jj];
      int ep = -1;
      for (int e = 0; e < cnt; ++e)
        if (pdst[e] == pr) ep = e;
      if (ep < 0) { pdst[cnt] = pr; psrc[cnt] = pr; ep = cnt++; }
      const int t = psrc[jj];
      psrc[jj] = psrc[ep];
      psrc[ep] = t;
    }
    int32_t* pm = f.perm + size_t(k) * kPermInts;
    pm[0] = cnt;
    for (int e = 0; e < cnt; ++e) { pm[1 + e] = pdst[e]; pm[1 + 2 * kNb + e] = psrc[e]; }
  }
}

// Column tile ct (!= the panel's) of element blockIdx.x after panel j0: rows permuted by the
// panel's exchanges and updated by the rank-16 product. The rows the permutation touches are
// read (old values) into LDS before any is written, so the in-place update has no order
// hazard; every other row is read and written by the one wave that owns its tile.
__global__ void __launch_bounds__(kUpdThreads) strip_update_kernel(StripFactorDevice f, int j0) {
  const int N = f.N, k = blockIdx.x, ct = blockIdx.y, pt = j0 / 16;
  if (ct == pt) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, ntile = N / 16;
  double* a = f.A + size_t(k) * N * N;
  __shared__ int np, pdst[2 * kNb], psrc[2 * kNb];
  __shared__ int rowmap[1024];        // row -> its entry in the permutation, -1 if untouched
  __shared__ double xr[2 * kNb][16];  // old values of the touched source rows, this tile's columns
  const int32_t* pm = f.perm + size_t(k) * kPermInts;
  if (tid == 0) np = pm[0];
  if (tid < 2 * kNb) { pdst[tid] = pm[1 + tid]; psrc[tid] = pm[1 + 2 * kNb + tid]; }
  for (int r = tid; r < N; r += kUpdThreads) rowmap[r] = -1;
  __syncthreads();
  const int n_e = np;
  if (tid < n_e) rowmap[pdst[tid]] = tid;
  for (int i = tid; i < n_e * 16; i += kUpdThreads) {
    const int e = i >> 4, c = i & 15;
    xr[e][c] = a[size_t(ct * 16 + c) * N + psrc[e]];
  }
  __syncthreads();
  // B operand: the exchanged panel rows j0 + e (entries e < 16), this tile's columns
  double bv[4];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) bv[kb] = xr[4 * kb + (lane >> 4)][lane & 15];
  const int col = ct * 16 + (lane & 15);
  for (int rt = wave; rt < ntile; rt += kUpdThreads / 64) {
    const int arow = rt * 16 + (lane & 15);
    double av[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const int kc = 4 * kb + (lane >> 4);
      av[kb] = a[size_t(j0 + kc) * N + arow] - (arow == j0 + kc ? 1.0 : 0.0);
    }
    double* cp = a + size_t(col) * N + rt * 16 + (lane >> 4);
    d4 acc;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = rt * 16 + 4 * i + (lane >> 4);
      const int e = rowmap[row];
      acc[i] = e >= 0 ? xr[e][lane & 15] : cp[4 * i];
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kb], bv[kb], acc, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) cp[4 * i] = acc[i];
  }
}

// A^-1[:, c] = X[:, idx[c]], idx the row exchanges undone in reverse order; block (element, 16
// columns)
__global__ void __launch_bounds__(256) strip_gather_kernel(StripFactorDevice f) {
  const int N = f.N, k = blockIdx.x, c0 = blockIdx.y * 16, tid = threadIdx.x;
  __shared__ int idx[1024], piv[1024];
  for (int c = tid; c < N; c += 256) {
    idx[c] = c;
    piv[c] = f.piv[size_t(k) * N + c];
  }
  __syncthreads();
  if (tid == 0)
    for (int j = N - 1; j >= 0; --j) {
      const int p = piv[j], t = idx[j];
      idx[j] = idx[p];
      idx[p] = t;
    }
  __syncthreads();
  const double* a = f.A + size_t(k) * N * N;
  double* out = f.Ainv + size_t(k) * N * N;
  for (int c = c0; c < c0 + 16; ++c) {
    const double* src = a + size_t(idx[c]) * N;
    for (int r = tid; r < N; r += 256) out[size_t(c) * N + r] = src[r];
  }
}

__device__ __forceinline__ double wave_total(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---- assembly of the row-equilibrated interior blocks (Sec. 4.3's collocation rows)
// The inverse-map factors of one element's nodes: D_X = M[xi_x] D_xi + M[eta_x] D_eta, D_Y with
// xi_y, eta_y; D_xi acts along the panel (Dq, index j), D_eta across the strip (Dr, index i).
struct ElemGeo {
  const double *ax, *ay, *ex, *ey, *xxi, *yxi;
};

// The factors ax, ay, ex, ey of element k staged in LDS (4 B doubles at dst), with Dq and Dr
// (q^2 + nr^2 doubles after them): every entry reads several of these
constexpr int kGeoLds = 4 * 1024 + 32 * 32 + 32 * 32;  // doubles, for B <= 1024, q, nr <= 32
__device__ void stage_geo(const StripFactorDevice& f, int k, double* dst, double** Dq, double** Dr) {
  const double* o = f.met + size_t(k) * 6 * f.B;
  for (int t = threadIdx.x; t < 4 * f.B; t += blockDim.x) dst[t] = o[t];
  double* q2 = dst + 4 * f.B;
  double* r2 = q2 + f.q * f.q;
  for (int t = threadIdx.x; t < f.q * f.q; t += blockDim.x) q2[t] = f.Dq[t];
  for (int t = threadIdx.x; t < f.nr * f.nr; t += blockDim.x) r2[t] = f.Dr[t];
  *Dq = q2;
  *Dr = r2;
}

// (sx D_X + sy D_Y)[(i, j)][(ii, jj)]: nonzero on grid row i and grid column j only
__device__ double grad_entry(const ElemGeo& g, const double* Dq, const double* Dr, int q, int nr, int i, int j, int ii,
                             int jj, double sx, double sy) {
  const int r = i * q + j;
  double v = 0.0;
  if (ii == i) v += (sx * g.ax[r] + sy * g.ay[r]) * Dq[j * q + jj];
  if (jj == j) v += (sx * g.ex[r] + sy * g.ey[r]) * Dr[i * nr + ii];
  return v;
}

// (D_X D_X + D_Y D_Y)[(i, j)][(ii, jj)], the product of the two first-derivative operators
// written out: with a = the D_xi factor and e = the D_eta factor of each direction,
//   delta(ii, i) a(i, j) sum_j' Dq[j][j'] a(i, j') Dq[j'][jj]    (along, then along)
// + a(i, j) Dq[j][jj] e(i, jj) Dr[i][ii]                         (along, then across)
// + e(i, j) Dr[i][ii] a(ii, j) Dq[j][jj]                         (across, then along)
// + delta(jj, j) e(i, j) sum_i' Dr[i][i'] e(i', j) Dr[i'][ii]    (across, then across)
__device__ double lap_entry(const ElemGeo& g, const double* Dq, const double* Dr, int q, int nr, int i, int j, int ii,
                            int jj) {
  const int r = i * q + j;
  double v = 0.0;
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const double* A = d ? g.ay : g.ax;
    const double* E = d ? g.ey : g.ex;
    const double a = A[r], e = E[r];
    if (ii == i) {
      double s = 0.0;
      for (int jp = 0; jp < q; ++jp) s += Dq[j * q + jp] * A[i * q + jp] * Dq[jp * q + jj];
      v += a * s;
    }
    v += a * Dq[j * q + jj] * E[i * q + jj] * Dr[i * nr + ii];
    v += e * Dr[i * nr + ii] * A[ii * q + j] * Dq[j * q + jj];
    if (jj == j) {
      double s = 0.0;
      for (int ip = 0; ip < nr; ++ip) s += Dr[i * nr + ip] * E[ip * q + j] * Dr[ip * nr + ii];
      v += e * s;
    }
  }
  return v;
}

// The interface normal of derivative row `row` of element k, oriented along increasing j
__device__ __forceinline__ void row_normal(const ElemGeo& g, const StripFactorDevice& f, int k, int row, double& sx,
                                           double& sy) {
  sx = f.nrm[2 * k];
  sy = f.nrm[2 * k + 1];
  if (sx * g.xxi[row] + sy * g.yxi[row] < 0) {
    sx = -sx;
    sy = -sy;
  }
}

// Row scales, block (element, 16 interior rows), one wave per row. The PDE rows and the
// derivative rows (with their coupling to element k + 1) are scaled to unit 1-norm over all B
// columns (the Dirichlet columns included), the value rows not; the PDE rows' right-hand side
// takes the same scale (rs). The derivative rows' couplings U~_k are written here.
__global__ void __launch_bounds__(1024) strip_rows_kernel(StripFactorDevice f) {
  const int k = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = f.q, nr = f.nr, B = f.B, m = f.m, Bi = f.Bi;
  __shared__ double geo[kGeoLds], geon[4 * 1024];
  double *Dq, *Dr;
  stage_geo(f, k, geo, &Dq, &Dr);
  const double* on = f.met + size_t((k + 1) % f.n) * 6 * B;  // the next element's factors
  for (int t = threadIdx.x; t < 4 * B; t += blockDim.x) geon[t] = on[t];
  if (blockIdx.y == 0)  // the rows on Gamma and Gamma~ keep their right-hand side
    for (int t = threadIdx.x; t < 2 * q; t += blockDim.x) f.rs[size_t(k) * B + (t < q ? t : (nr - 1) * q + t - q)] = 1.0;
  __syncthreads();
  const int p = blockIdx.y * 16 + wave;
  if (p >= Bi) return;
  const int row = p + q, i = row / q, j = row % q;
  const double* xo = f.met + size_t(k) * 6 * B;
  const ElemGeo g{geo, geo + B, geo + 2 * B, geo + 3 * B, xo + 4 * B, xo + 5 * B};
  double sc = 1.0;
  if (j == q - 1) {
    double sx, sy;
    row_normal(g, f, k, row, sx, sy);
    const ElemGeo gn{geon, geon + B, geon + 2 * B, geon + 3 * B, nullptr, nullptr};  // node (i, 0) of element k + 1
    double s = 0.0;
    for (int t = lane; t < B; t += 64)
      s += fabs(grad_entry(g, Dq, Dr, q, nr, i, j, t / q, t % q, sx, sy)) +
           fabs(grad_entry(gn, Dq, Dr, q, nr, i, 0, t / q, t % q, -sx, -sy));
    sc = 1.0 / wave_total(s);
    for (int c = lane; c < Bi; c += 64)
      f.U[(size_t(k) * m + (i - 1)) * Bi + c] = sc * grad_entry(gn, Dq, Dr, q, nr, i, 0, (c + q) / q, (c + q) % q, -sx, -sy);
  } else if (j != 0) {
    double s = 0.0;
    for (int t = lane; t < B; t += 64) s += fabs(lap_entry(g, Dq, Dr, q, nr, i, j, t / q, t % q));
    sc = 1.0 / wave_total(s);
  }
  if (lane == 0) {
    f.rowsc[size_t(k) * Bi + p] = sc;
    f.rs[size_t(k) * B + row] = (j == 0 || j == q - 1) ? 1.0 : sc;
  }
}

// A_k (column-major, interior rows and columns, identity padding up to N), block (element, 16
// columns): value rows (j = 0) have a unit diagonal, PDE and derivative rows their scaled
// operator entries.
__global__ void __launch_bounds__(256) strip_fill_kernel(StripFactorDevice f) {
  const int k = blockIdx.x, c0 = blockIdx.y * 16, q = f.q, nr = f.nr, N = f.N, Bi = f.Bi, B = f.B;
  __shared__ double geo[kGeoLds];
  double *Dq, *Dr;
  stage_geo(f, k, geo, &Dq, &Dr);
  __syncthreads();
  const double* xo = f.met + size_t(k) * 6 * B;
  const ElemGeo g{geo, geo + B, geo + 2 * B, geo + 3 * B, xo + 4 * B, xo + 5 * B};
  double* Ak = f.A + size_t(k) * N * N;
  for (int p = threadIdx.x; p < N; p += 256) {
    const int row = p + q, i = row / q, j = row % q;
    double sc = 1.0, sx = 0.0, sy = 0.0;
    if (p < Bi) {
      sc = f.rowsc[size_t(k) * Bi + p];
      if (j == q - 1) row_normal(g, f, k, row, sx, sy);
    }
    for (int c = c0; c < c0 + 16; ++c) {
      double v;
      if (p >= Bi || c >= Bi || j == 0) {
        v = p == c ? 1.0 : 0.0;
      } else {
        const int ii = (c + q) / q, jj = (c + q) % q;
        v = sc * (j == q - 1 ? grad_entry(g, Dq, Dr, q, nr, i, j, ii, jj, sx, sy) : lap_entry(g, Dq, Dr, q, nr, i, j, ii, jj));
      }
      Ak[size_t(c) * N + p] = v;
    }
  }
}

// R_k[a][c] = sum_r U~_{k-1}[a][r] A_k^-1[r][c]: block (k, 4 columns), a wave per column
__global__ void __launch_bounds__(256) strip_couple_kernel(StripFactorDevice f) {
  const int k = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.y * 4 + wave, N = f.N, Bi = f.Bi, m = f.m;
  if (c >= Bi) return;
  const double* col = f.Ainv + (size_t(k) * N + c) * N;
  const double* U = f.U + size_t((k + f.n - 1) % f.n) * m * Bi;
  double x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = lane + 64 * i < Bi ? col[lane + 64 * i] : 0.0;
  for (int aa = 0; aa < m; ++aa) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (lane + 64 * i < Bi) s = fma(U[size_t(aa) * Bi + lane + 64 * i], x[i], s);
    s = wave_total(s);
    if (lane == 0) f.R[(size_t(k) * m + aa) * Bi + c] = s;
  }
}

// pieces[k] = [A^-1[S, P], A^-1[S, V], R[:, P], R[:, V]], each m x m row-major
__global__ void strip_pieces_kernel(StripFactorDevice f) {
  const int k = blockIdx.x, m = f.m, q = f.q, N = f.N, Bi = f.Bi, mm = m * m;
  for (int e = threadIdx.x; e < 4 * mm; e += blockDim.x) {
    const int which = e / mm, i = (e % mm) / m, j = e % m;
    const int S = i * q + q - 1, P = j * q + q - 1, V = j * q;
    double v;
    if (which == 0) v = f.Ainv[(size_t(k) * N + P) * N + S];
    else if (which == 1) v = f.Ainv[(size_t(k) * N + V) * N + S];
    else if (which == 2) v = f.R[(size_t(k) * m + i) * Bi + P];
    else v = f.R[(size_t(k) * m + i) * Bi + V];
    f.pieces[size_t(k) * 4 * mm + e] = v;
  }
}

// Q_k[b][c] = sum_a MG_k[b][a] R_k[a][c]; W_k[m + a][c] = R_k[a][c] - sum_b R_k[a][V_b] Q_k[b][c]
__global__ void __launch_bounds__(256) strip_q_kernel(StripFactorDevice f) {
  const int k = blockIdx.x, c = blockIdx.y * 256 + threadIdx.x, m = f.m, q = f.q, Bi = f.Bi;
  if (c >= Bi) return;
  const double* R = f.R + size_t(k) * m * Bi;
  const double* MG = f.MG + size_t(k) * m * m;
  double r[30], qv[30];
#pragma unroll
  for (int aa = 0; aa < 30; ++aa)
    if (aa < m) r[aa] = R[size_t(aa) * Bi + c];
#pragma unroll
  for (int b = 0; b < 30; ++b)
    if (b < m) {
      double s = 0.0;
#pragma unroll
      for (int aa = 0; aa < 30; ++aa)
        if (aa < m) s = fma(MG[b * m + aa], r[aa], s);
      qv[b] = s;
      f.Q[(size_t(k) * m + b) * Bi + c] = s;
    }
  double* W = f.W + size_t(k) * 2 * m * Bi;
#pragma unroll
  for (int aa = 0; aa < 30; ++aa)
    if (aa < m) {
      double s = r[aa];
#pragma unroll
      for (int b = 0; b < 30; ++b)
        if (b < m) s = fma(-R[size_t(aa) * Bi + b * q], qv[b], s);
      W[size_t(m + aa) * Bi + c] = s;
    }
}

// EiT[c][p] = E_k[p][c] = A^-1[p][c] - sum_b A^-1[p][V_b] Q[b][c]; block (k, 64 rows), 4 waves
// splitting the columns; rows S also go to W_k[0 .. m)
__global__ void __launch_bounds__(256) strip_e_kernel(StripFactorDevice f) {
  const int k = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = f.m, q = f.q, N = f.N, Bi = f.Bi;
  const int p = blockIdx.y * 64 + lane;
  const bool on = p < Bi;
  const int pc = on ? p : 0;
  const double* Ai = f.Ainv + size_t(k) * N * N;
  const double* Q = f.Q + size_t(k) * m * Bi;
  double cv[30];
#pragma unroll
  for (int b = 0; b < 30; ++b)
    if (b < m) cv[b] = Ai[size_t(b * q) * N + pc];
  const bool srow = on && (p % q) == q - 1;  // a derivative row: S_a with a = p / q
  double* EiT = f.EiT + size_t(k) * Bi * Bi;
  double* W = f.W + size_t(k) * 2 * m * Bi;
  for (int c = wave; c < Bi; c += 4) {
    double e = Ai[size_t(c) * N + pc];
#pragma unroll
    for (int b = 0; b < 30; ++b)
      if (b < m) e = fma(-cv[b], Q[size_t(b) * Bi + c], e);
    if (on) EiT[size_t(c) * Bi + p] = e;
    if (srow) W[size_t(p / q) * Bi + c] = e;
  }
}

}  // namespace

hipError_t launch_strip_factor(const StripFactorDevice& f, int stage, hipStream_t stream) {
  if (f.N % 16 != 0 || f.N > 1024 || f.m < 1 || f.m > 30) return hipErrorInvalidValue;
  if (stage == 0) {
    hipLaunchKernelGGL(strip_rows_kernel, dim3(unsigned(f.n), unsigned((f.Bi + 15) / 16)), dim3(1024), 0, stream, f);
    hipLaunchKernelGGL(strip_fill_kernel, dim3(unsigned(f.n), unsigned(f.N / 16)), dim3(256), 0, stream, f);
    for (int j0 = 0; j0 < f.N; j0 += kNb) {
      hipLaunchKernelGGL(strip_panel_kernel, dim3(unsigned(f.n)), dim3(kInvThreads), 0, stream, f, j0);
      hipLaunchKernelGGL(strip_update_kernel, dim3(unsigned(f.n), unsigned(f.N / 16)), dim3(kUpdThreads), 0, stream,
                         f, j0);
    }
    hipLaunchKernelGGL(strip_gather_kernel, dim3(unsigned(f.n), unsigned(f.N / 16)), dim3(256), 0, stream, f);
    hipLaunchKernelGGL(strip_couple_kernel, dim3(unsigned(f.n), unsigned((f.Bi + 3) / 4)), dim3(256), 0, stream, f);
    hipLaunchKernelGGL(strip_pieces_kernel, dim3(unsigned(f.n)), dim3(256), 0, stream, f);
  } else {
    hipLaunchKernelGGL(strip_q_kernel, dim3(unsigned(f.n), unsigned((f.Bi + 255) / 256)), dim3(256), 0, stream, f);
    hipLaunchKernelGGL(strip_e_kernel, dim3(unsigned(f.n), unsigned((f.Bi + 63) / 64)), dim3(256), 0, stream, f);
  }
  return hipGetLastError();
}

}  // namespace vp
