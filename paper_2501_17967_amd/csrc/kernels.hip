// HIP kernels of the box code for gfx950 (CDNA4), FP64 throughout.
//
// One kernel template serves every stage: a grouped-relation GEMM. A workgroup owns a tile of
// NT output vectors ("slots") of M rows each and loops over the relations present in the tile
// (sorted by relation id). For relation r it stages the NT source vectors (gathered by index,
// optionally scaled by s^2 of the source leaf) in LDS in k-chunks of 64 and accumulates
//     C[:, slot] += A_r[:, k-chunk] * B[k-chunk, slot]
// with v_mfma_f64_16x16x4f64. A_r is streamed from global memory (L2-resident tables) in a
// fragment-major layout so every fragment load is one contiguous 512-byte wave access.
// Each output vector has exactly one owner and a fixed relation order: no atomics, bitwise
// deterministic, identical whether a tree is applied alone or inside a forest.
//
// MFMA f64 16x16x4 operand layout (lane l, checked on gfx950):
//   A: A[l % 16][l / 16]   B: B[l / 16][l % 16]   D (4 regs r): D[4 r + l / 16][l % 16]
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace vp {

typedef double d4 __attribute__((ext_vector_type(4)));

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous range of
// tiles so neighbouring tiles (which share source leaves) share an L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
  const int q = G >> 3, r = G & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

template <int MT, int NTT, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) grg_kernel(const GrgParams p) {
  constexpr int M = 16 * MT * WM;
  constexpr int NT = 16 * NTT * WN;
  constexpr int NTHR = 64 * WM * WN;
  constexpr int KC = 64;
  constexpr int LDB = KC + 2;
  __shared__ double Bs[NT * LDB];
  __shared__ double r1s[NT];

  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;

  d4 acc[MT][NTT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NTT; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int s0 = p.tile_seg_ptr[tile], s1 = p.tile_seg_ptr[tile + 1];
  for (int s = s0; s < s1; ++s) {
    const RelDesc rd = p.rels[p.seg_rel[s]];
    const int fam = p.seg_fam[s];
    const double* __restrict__ base = p.fam_base[fam];
    const int stride = p.fam_stride[fam];
    const bool scaled = p.fam_scaled[fam] != 0;
    const int32_t* __restrict__ src = p.seg_src + (size_t)s * NT;
    for (int k0 = 0; k0 < rd.K; k0 += KC) {
      const int kc = min(KC, rd.K - k0);
      const int half = kc >> 1;
      __syncthreads();
      for (int idx = tid; idx < NT * half; idx += NTHR) {
        const int t = idx / half, kp = idx - t * half;
        const int si = src[t];
        double2 v = make_double2(0.0, 0.0);
        if (si >= 0) {
          v = *reinterpret_cast<const double2*>(base + (size_t)si * stride + k0 + 2 * kp);
          if (scaled) {
            const double sc = p.leaf_s2[si];
            v.x *= sc;
            v.y *= sc;
          }
        }
        Bs[t * LDB + 2 * kp] = v.x;
        Bs[t * LDB + 2 * kp + 1] = v.y;
      }
      __syncthreads();
      const int nk = kc >> 2;
      const double* __restrict__ Ab = rd.A + (size_t)(k0 >> 2) * (M / 16) * 64 + (size_t)(wm * MT) * 64 + lane;
      const double* __restrict__ Bw = Bs + ((wn * NTT) * 16 + (lane & 15)) * LDB + (lane >> 4);
      for (int kk = 0; kk < nk; ++kk) {
        double a[MT], b[NTT];
#pragma unroll
        for (int i = 0; i < MT; ++i) a[i] = Ab[((size_t)kk * (M / 16) + i) * 64];
#pragma unroll
        for (int j = 0; j < NTT; ++j) b[j] = Bw[j * 16 * LDB + kk * 4];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
          for (int j = 0; j < NTT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
  }

  // rank-one log-scale terms, one scalar per slot
  __syncthreads();
  for (int t = tid; t < NT; t += NTHR) {
    const int ti = tile * NT + t;
    double c = 0.0;
    for (int e = p.r1_ptr[ti]; e < p.r1_ptr[ti + 1]; ++e) {
      const int f = p.r1_fam[e];
      c += p.r1_coef[e] * p.r1_base[f][(size_t)p.r1_idx[e] * p.r1_stride[f]];
    }
    r1s[t] = c;
  }
  __syncthreads();

#pragma unroll
  for (int j = 0; j < NTT; ++j) {
    const int slot = (wn * NTT + j) * 16 + (lane & 15);
    const int tgt = p.tile_tgt[tile * NT + slot];
    if (tgt < 0) continue;
    const double sc = p.out_scaled ? p.leaf_s2[tgt] : 1.0;
    const double r1 = r1s[slot];
    double* __restrict__ o = p.out + (size_t)tgt * p.out_stride;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (wm * MT + i) * 16 + 4 * r + (lane >> 4);
        double v = acc[i][j][r];
        if (p.r1_all_rows || row == 0) v += r1;
        o[row] = v * sc;
      }
  }
}

__global__ void rowsum_kernel(const double* __restrict__ x, double* __restrict__ out, int64_t n) {
  const int64_t leaf = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (leaf >= n) return;
  const double* xl = x + leaf * 256;
  double s = xl[lane] + xl[lane + 64] + xl[lane + 128] + xl[lane + 192];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) out[leaf] = s;
}

hipError_t launch_grg(int M, int NT, const GrgParams& p, hipStream_t stream) {
  if (p.n_tiles <= 0) return hipSuccess;
  dim3 grid(p.n_tiles);
  if (M == 256 && NT == 64) {
    hipLaunchKernelGGL((grg_kernel<4, 4, 4, 1>), grid, dim3(256), 0, stream, p);
  } else if (M == 256 && NT == 32) {
    hipLaunchKernelGGL((grg_kernel<4, 2, 4, 1>), grid, dim3(256), 0, stream, p);
  } else if (M == 80 && NT == 64) {
    hipLaunchKernelGGL((grg_kernel<5, 1, 1, 4>), grid, dim3(256), 0, stream, p);
  } else if (M == 80 && NT == 32) {
    hipLaunchKernelGGL((grg_kernel<5, 1, 1, 2>), grid, dim3(128), 0, stream, p);
  } else if (M == 80 && NT == 16) {
    hipLaunchKernelGGL((grg_kernel<5, 1, 1, 1>), grid, dim3(64), 0, stream, p);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rowsum(const double* x, double* usum, int64_t n_leaves, hipStream_t stream) {
  if (n_leaves <= 0) return hipSuccess;
  dim3 grid((unsigned)((n_leaves + 3) / 4));
  hipLaunchKernelGGL(rowsum_kernel, grid, dim3(256), 0, stream, x, usum, n_leaves);
  return hipGetLastError();
}

}  // namespace vp
