// HIP kernels of the strip factorization (plan time; the host side is strip.cpp).
//
//   strip_invert_kernel   one workgroup per element: the inverse of the interior block A_k
//                         (N x N, column-major, N a multiple of 16, identity padding) by blocked
//                         Gauss-Jordan elimination with partial pivoting. Per panel of 16
//                         columns: the panel's elimination with its rows held in registers
//                         (pivot by a block-wide argmax, row exchange and broadcast through
//                         LDS); the panel's row exchanges applied to the other columns as one
//                         net permutation; then the other columns updated as
//                         A[:, c] += (T - I_panel) A_old[panel rows, c], a rank-16 product on
//                         FP64 MFMA (v_mfma_f64_16x16x4f64), T the panel's transformation. The
//                         columns of the result are finally gathered through the inverse of the
//                         row exchanges (in-place Gauss-Jordan yields (PA)^-1 = A^-1 P^-1).
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

constexpr int kInvThreads = 512;  // 8 waves
constexpr int kNb = 16;           // panel width (one MFMA tile)
constexpr int kRpt = 2;           // panel rows per thread: N <= 1024

__device__ __forceinline__ bool better(double v, int i, double bv, int bi) { return v > bv || (v == bv && i < bi); }

__global__ void __launch_bounds__(kInvThreads)
    strip_invert_kernel(int N, double* __restrict__ Aall, double* __restrict__ Rball, int32_t* __restrict__ flag,
                        double* __restrict__ Ainv) {
  const int k = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* a = Aall + size_t(k) * N * N;
  double* rb = Rball + size_t(k) * kNb * N;
  __shared__ double prow[kNb], xrow[kNb];
  __shared__ double redv[kInvThreads / 64];
  __shared__ int redi[kInvThreads / 64];
  __shared__ int pivs[kNb];
  __shared__ int pdst[2 * kNb], psrc[2 * kNb];
  __shared__ int npair;
  __shared__ int pivall[1024];
  __shared__ int singular;
  if (tid == 0) singular = 0;
  const int ntile = N / 16;

  for (int j0 = 0; j0 < N; j0 += kNb) {
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
        pivall[j] = pr;
        if (!(bv > 0.0)) singular = 1;
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
          const double f = pv[r][jj];
#pragma unroll
          for (int c = 0; c < kNb; ++c) pv[r][c] = c == jj ? -f * ip : fma(-f, pj[c], pv[r][c]);
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
    if (tid == 0) {  // pdst: the rows, psrc: which old row ends up there (LDS, indexed at run time)
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
      npair = cnt;
    }
    __syncthreads();
    const int np = npair;
    for (int c = tid; c < N; c += kInvThreads) {
      if (c >= j0 && c < j0 + kNb) continue;
      double* col = a + size_t(c) * N;
      double v[2 * kNb];
#pragma unroll
      for (int e = 0; e < 2 * kNb; ++e)
        if (e < np) v[e] = col[psrc[e]];
#pragma unroll
      for (int e = 0; e < 2 * kNb; ++e)
        if (e < np && pdst[e] != psrc[e]) col[pdst[e]] = v[e];
#pragma unroll
      for (int e = 0; e < kNb; ++e) rb[size_t(e) * N + c] = v[e];  // the exchanged rows j0 .. j0 + 15
    }
    __syncthreads();
    // A[:, c] += (T - I_panel) rb[:, c] for the other column tiles, 16 x 16 tiles on MFMA
    const int pt = j0 / 16;
    for (int rt = wave; rt < ntile; rt += kInvThreads / 64) {
      const int row = rt * 16 + (lane & 15);
      double av[4];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const int kc = 4 * kb + (lane >> 4);
        av[kb] = a[size_t(j0 + kc) * N + row] - (row == j0 + kc ? 1.0 : 0.0);
      }
      for (int ct = 0; ct < ntile; ++ct) {
        if (ct == pt) continue;
        const int col = ct * 16 + (lane & 15);
        double* cp = a + size_t(col) * N + rt * 16 + (lane >> 4);
        d4 acc = {cp[0], cp[4], cp[8], cp[12]};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          const double bvk = rb[size_t(4 * kb + (lane >> 4)) * N + col];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kb], bvk, acc, 0, 0, 0);
        }
        cp[0] = acc[0];
        cp[4] = acc[1];
        cp[8] = acc[2];
        cp[12] = acc[3];
      }
    }
    __syncthreads();
  }
  // column gather: A^-1[:, c] = X[:, idx[c]], idx the row exchanges undone in reverse order
  __shared__ int idx[1024];
  for (int c = tid; c < N; c += kInvThreads) idx[c] = c;
  __syncthreads();
  if (tid == 0) {
    for (int j = N - 1; j >= 0; --j) {
      const int p = pivall[j], t = idx[j];
      idx[j] = idx[p];
      idx[p] = t;
    }
    flag[k] = singular;
  }
  __syncthreads();
  double* out = Ainv + size_t(k) * N * N;
  for (int c = 0; c < N; ++c) {
    const double* src = a + size_t(idx[c]) * N;
    for (int r = tid; r < N; r += kInvThreads) out[size_t(c) * N + r] = src[r];
  }
}

__device__ __forceinline__ double wave_total(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
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
    hipLaunchKernelGGL(strip_invert_kernel, dim3(unsigned(f.n)), dim3(kInvThreads), 0, stream, f.N, f.A, f.Rb,
                       f.flag, f.Ainv);
    hipLaunchKernelGGL(strip_couple_kernel, dim3(unsigned(f.n), unsigned((f.Bi + 3) / 4)), dim3(256), 0, stream, f);
    hipLaunchKernelGGL(strip_pieces_kernel, dim3(unsigned(f.n)), dim3(256), 0, stream, f);
  } else {
    hipLaunchKernelGGL(strip_q_kernel, dim3(unsigned(f.n), unsigned((f.Bi + 255) / 256)), dim3(256), 0, stream, f);
    hipLaunchKernelGGL(strip_e_kernel, dim3(unsigned(f.n), unsigned((f.Bi + 63) / 64)), dim3(256), 0, stream, f);
  }
  return hipGetLastError();
}

}  // namespace vp
