// The measured companion of the published FP64 matrix peak: a kernel that issues nothing but
// v_mfma_f64_16x16x4f64 on register operands, eight independent accumulator chains per wave (as
// many as a near-field wave keeps), so that its rate is what the matrix cores sustain on this
// device and clock.
#include <hip/hip_runtime.h>

#include "../../include/volpot.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// Lane l holds A[l % 16][l / 16] = 1 + (l % 16 + 16 (l / 16)) / 1024 and B[l / 16][l % 16] =
// 1 - (16 (l / 16) + l % 16) / 1024 of every product; every chain adds A B to its accumulator
// iters times. Each thread writes the sum of its 32 accumulator values (the 8 chains agree).
__global__ void __launch_bounds__(256) mfma_peak_kernel(int iters, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const double a = 1.0 + double(lane) / 1024.0, b = 1.0 - double(lane) / 1024.0;
  d4 acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[size_t(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" int volpot_peak_mfma(int32_t blocks, int32_t iters, double* out_dev, void* hip_stream) {
  if (blocks <= 0 || iters <= 0 || !out_dev) return VOLPOT_ERR_ARG;
  hipLaunchKernelGGL(mfma_peak_kernel, dim3(unsigned(blocks)), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     iters, out_dev);
  return hipGetLastError() == hipSuccess ? VOLPOT_OK : VOLPOT_ERR_HIP;
}
