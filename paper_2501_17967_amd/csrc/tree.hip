// HIP kernels of the adaptive quadtree construction (Sec. 4.2.1, Alg. 2): the node
// coordinates of the boxes to be sampled, and each sampled box's Chebyshev tail
//     max { |c_nm| : n >= p - 2 or m >= p - 2 },  c = D V D^T,
// V[j][i] the samples (x fastest), D[m][i] = (2 - delta_m0)/p T_m(t_i) the transform from values
// at the first-kind points to Chebyshev coefficients. One wave per box; the maximum is exact,
// so the tail does not depend on the reduction order.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace vp {

namespace {

__global__ void __launch_bounds__(256) tree_nodes_kernel(const int64_t* __restrict__ keys, TreeRule r,
                                                         double* __restrict__ nodes) {
  const int64_t b = blockIdx.x;
  const int m = threadIdx.x;
  const int64_t k = keys[b];
  const int l = int(k >> 58);
  const int64_t ix = (k >> 29) & ((int64_t(1) << 29) - 1), iy = k & ((int64_t(1) << 29) - 1);
  const double s = ldexp(1.0, -l);
  const double cx = -1.0 + (2.0 * double(ix) + 1.0) * s, cy = -1.0 + (2.0 * double(iy) + 1.0) * s;
  nodes[(b * 256 + m) * 2] = cx + s * r.t[m & 15];
  nodes[(b * 256 + m) * 2 + 1] = cy + s * r.t[m >> 4];
}

__global__ void __launch_bounds__(64) tree_tail_kernel(const double* __restrict__ values, TreeRule r,
                                                       double* __restrict__ tails) {
  __shared__ double V[256], A[256];
  const int64_t b = blockIdx.x;
  const int l = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 4; ++q) V[l + 64 * q] = values[b * 256 + l + 64 * q];
  __syncthreads();
  // A[n][i] = sum_j D[n][j] V[j][i]
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = l + 64 * q, n = e >> 4, i = e & 15;
    double s = 0.0;
    for (int j = 0; j < 16; ++j) s = fma(r.D[n * 16 + j], V[j * 16 + i], s);
    A[e] = s;
  }
  __syncthreads();
  // c[n][m] = sum_i A[n][i] D[m][i]; tail over n >= 14 or m >= 14
  double mx = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = l + 64 * q, n = e >> 4, m = e & 15;
    if (n < 14 && m < 14) continue;
    double s = 0.0;
    for (int i = 0; i < 16; ++i) s = fma(A[n * 16 + i], r.D[m * 16 + i], s);
    mx = fmax(mx, fabs(s));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if (l == 0) tails[b] = mx;
}

}  // namespace

hipError_t launch_tree_nodes(const int64_t* keys, int64_t n, const TreeRule& r, double* nodes, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(tree_nodes_kernel, dim3(unsigned(n)), dim3(256), 0, stream, keys, r, nodes);
  return hipGetLastError();
}

hipError_t launch_tree_tail(const double* values, int64_t n, const TreeRule& r, double* tails, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(tree_tail_kernel, dim3(unsigned(n)), dim3(64), 0, stream, values, r, tails);
  return hipGetLastError();
}

}  // namespace vp
