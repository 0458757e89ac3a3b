// HIP kernels of the strip solve (the factored system of strip.cpp). One apply:
//   c_k = E_k b_k                      b = f * rs at the PDE rows, else 0   (per element)
//   z_{k+1} = c_k[S] + F_k z_k         forward recurrence, m values         (one workgroup)
//   y_k = c_k + E_k[:, value rows] z_k                                      (per element)
//   g_k = U~_{k-1} y_k                                                       (per element)
//   t_k = g_k - H_k t_{k+1}            backward recurrence                  (one workgroup)
//   x_k = y_k - E_k[:, derivative rows] t_{k+1}                              (per element)
//   x -= Z K [x_{n-1}[S]; U~_{n-1} x_0]  the periodic corner (Woodbury)
// Per-element kernels run one thread per unknown; sums have a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace vp {

namespace {

__device__ __forceinline__ double block_sum(double v, double* red) {
  // sum over the block (blockDim.x a multiple of 64, at most 1024); every thread gets the result
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

__global__ void strip_c_kernel(StripDevice d, const double* __restrict__ f) {
  extern __shared__ double b[];
  const int k = blockIdx.x, r = threadIdx.x, B = d.B;
  if (r < B) b[r] = d.pde[r] ? f[size_t(k) * B + r] * d.rs[size_t(k) * B + r] : 0.0;
  __syncthreads();
  if (r >= B) return;
  const double* E = d.Et + size_t(k) * B * B;
  double s = 0.0;
  for (int c = 0; c < B; ++c) s = fma(E[size_t(c) * B + r], b[c], s);
  d.c[size_t(k) * B + r] = s;
}

__global__ void strip_forward_kernel(StripDevice d) {
  __shared__ double z[64];
  const int a = threadIdx.x, m = d.m;
  if (a < m) { z[a] = 0.0; d.z[a] = 0.0; }
  __syncthreads();
  for (int k = 0; k < d.n; ++k) {
    double v = 0.0;
    if (a < m) {
      v = d.c[size_t(k) * d.B + d.scol[a]];
      const double* F = d.F + size_t(k) * m * m;
      for (int b = 0; b < m; ++b) v = fma(F[a * m + b], z[b], v);
    }
    __syncthreads();
    if (a < m) { z[a] = v; d.z[size_t(k + 1) * m + a] = v; }
    __syncthreads();
  }
}

__global__ void strip_y_kernel(StripDevice d) {
  __shared__ double red[16];
  const int k = blockIdx.x, r = threadIdx.x, B = d.B, m = d.m;
  const double* E = d.Et + size_t(k) * B * B;
  double y = 0.0;
  if (r < B) {
    y = d.c[size_t(k) * B + r];
    for (int b = 0; b < m; ++b) y = fma(E[size_t(d.pvrow[b]) * B + r], d.z[size_t(k) * m + b], y);
    d.y[size_t(k) * B + r] = y;
  }
  if (k == 0) return;  // g_k = U~_{k-1} y_k for k >= 1 (block-uniform branch)
  const double* U = d.Ut + size_t(k - 1) * m * B;
  for (int a = 0; a < m; ++a) {
    const double s = block_sum(r < B ? U[size_t(a) * B + r] * y : 0.0, red);
    if (r == 0) d.g[size_t(k) * m + a] = s;
  }
}

__global__ void strip_backward_kernel(StripDevice d) {
  __shared__ double t[64];
  const int a = threadIdx.x, m = d.m, n = d.n;
  if (a < m) { t[a] = 0.0; d.t[size_t(n) * m + a] = 0.0; d.t[size_t(n - 1) * m + a] = 0.0; }
  // t_{n-1} (x_{n-1} = y_{n-1}, no element after it in the non-periodic part) = g_{n-1}
  __syncthreads();
  if (a < m) t[a] = d.g[size_t(n - 1) * m + a];
  __syncthreads();
  if (a < m) d.t[size_t(n - 1) * m + a] = t[a];
  for (int k = n - 2; k >= 1; --k) {
    double v = 0.0;
    if (a < m) {
      v = d.g[size_t(k) * m + a];
      const double* H = d.H + size_t(k) * m * m;
      for (int b = 0; b < m; ++b) v = fma(-H[a * m + b], t[b], v);
    }
    __syncthreads();
    if (a < m) { t[a] = v; d.t[size_t(k) * m + a] = v; }
    __syncthreads();
  }
}

__global__ void strip_x_kernel(StripDevice d, double* __restrict__ x) {
  const int k = blockIdx.x, r = threadIdx.x, B = d.B, m = d.m;
  if (r >= B) return;
  const double* E = d.Et + size_t(k) * B * B;
  double v = d.y[size_t(k) * B + r];
  if (k + 1 < d.n)
    for (int a = 0; a < m; ++a) v = fma(-E[size_t(d.prow[a]) * B + r], d.t[size_t(k + 1) * m + a], v);
  x[size_t(k) * B + r] = v;
}

__global__ void strip_corner_kernel(StripDevice d, const double* __restrict__ x) {
  __shared__ double red[16];
  __shared__ double gv[128];
  const int r = threadIdx.x, B = d.B, m = d.m, n = d.n;
  const double* U = d.Ut + size_t(n - 1) * m * B;  // acting on element 0
  if (r < m) gv[r] = x[size_t(n - 1) * B + d.scol[r]];
  for (int a = 0; a < m; ++a) {
    const double s = block_sum(r < B ? U[size_t(a) * B + r] * x[r] : 0.0, red);
    if (r == 0) gv[m + a] = s;
  }
  __syncthreads();
  if (r < 2 * m) {
    double s = 0.0;
    for (int b = 0; b < 2 * m; ++b) s = fma(d.K[r * 2 * m + b], gv[b], s);
    d.h[r] = s;
  }
}

__global__ void strip_fix_kernel(StripDevice d, double* __restrict__ x) {
  const int k = blockIdx.x, r = threadIdx.x, B = d.B, m2 = 2 * d.m;
  if (r >= B) return;
  const size_t row = size_t(k) * B + r;
  double v = x[row];
  for (int j = 0; j < m2; ++j) v = fma(-d.Z[row * m2 + j], d.h[j], v);
  x[row] = v;
}

}  // namespace

hipError_t launch_strip_solve(const StripDevice& d, const double* f, double* v, hipStream_t stream) {
  const unsigned threads = unsigned((d.B + 63) / 64 * 64);
  hipLaunchKernelGGL(strip_c_kernel, dim3(unsigned(d.n)), dim3(threads), size_t(d.B) * sizeof(double), stream, d, f);
  hipLaunchKernelGGL(strip_forward_kernel, dim3(1), dim3(64), 0, stream, d);
  hipLaunchKernelGGL(strip_y_kernel, dim3(unsigned(d.n)), dim3(threads), 0, stream, d);
  hipLaunchKernelGGL(strip_backward_kernel, dim3(1), dim3(64), 0, stream, d);
  hipLaunchKernelGGL(strip_x_kernel, dim3(unsigned(d.n)), dim3(threads), 0, stream, d, v);
  hipLaunchKernelGGL(strip_corner_kernel, dim3(1), dim3(threads), 0, stream, d, (const double*)v);
  hipLaunchKernelGGL(strip_fix_kernel, dim3(unsigned(d.n)), dim3(threads), 0, stream, d, v);
  return hipGetLastError();
}

}  // namespace vp
