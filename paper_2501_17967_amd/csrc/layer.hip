// HIP kernels of the layer-potential evaluation (Sec. 4.4: v_glue = S[sigma] - D[tau] on the
// fictitious curve, evaluated at every quadtree node with the FMM), FP64 throughout.
//
// With z = x + i y, node positions zeta_j, charges q_j = w_j sigma_j and complex dipoles
// mu_j = w_j tau_j (n_x + i n_y), the potential is
//     V(z) = -(1/2pi) Re sum_j [ q_j log(z - zeta_j) + mu_j / (z - zeta_j) ],
// the same kernel as the volume code, so its multipoles, locals and translation tables serve
// unchanged. These kernels add what depends on the node positions:
//   P2M  multipole of a leaf (centre c, half-width s, eta = (zeta - c) / s):
//        a_0 = sum q,  a_n = sum [ -(q / n) eta^n + (mu / s) eta^(n-1) ]           (n >= 1)
//   P2L  local expansion of a box from the nodes of its X-list leaves (w = (zeta - c) / s):
//        b_0 = sum [ q log|zeta - c| - (mu / s) / w ],
//        b_l = sum [ -(q / l) w^-l - (mu / s) w^-(l+1) ]                           (l >= 1)
//        (only real parts reach V, so the log keeps its modulus only)
//   P2P  direct sum at the 256 nodes of a leaf over the curve nodes in its adjacent leaves.
// Each output has one owner and a fixed summation order: deterministic, no atomics.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace vp {

namespace {

constexpr int kTerms = 40;
constexpr int kReals = 80;
constexpr double kInv2Pi = 0.15915494309189533576888376337251436;

// (x + i y)^k by repeated squaring
__device__ __forceinline__ void cpow(double x, double y, int k, double& pr, double& pi) {
  double rr = 1.0, ri = 0.0, br = x, bi = y;
  while (k > 0) {
    if (k & 1) {
      const double t = rr * br - ri * bi;
      ri = rr * bi + ri * br;
      rr = t;
    }
    k >>= 1;
    if (k > 0) {
      const double t = br * br - bi * bi;
      bi = 2.0 * br * bi;
      br = t;
    }
  }
  pr = rr;
  pi = ri;
}

__global__ void layer_prep_kernel(int64_t n, const int32_t* __restrict__ order, const double* __restrict__ w,
                                  const double* __restrict__ nrm, const double* __restrict__ sigma,
                                  const double* __restrict__ tau, double* __restrict__ q, double* __restrict__ mu) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int32_t o = order[j];
  const double wj = w[j];
  q[j] = wj * sigma[o];
  const double d = wj * tau[o];
  mu[2 * j] = d * nrm[2 * j];
  mu[2 * j + 1] = d * nrm[2 * j + 1];
}

// one wave per target leaf box; lane n < 40 owns term n
__global__ void __launch_bounds__(64) p2m_kernel(const int32_t* __restrict__ tgt, const int32_t* __restrict__ bptr,
                                                 const double* __restrict__ geo, const double* __restrict__ sxy,
                                                 const double* __restrict__ q, const double* __restrict__ mu,
                                                 double* __restrict__ mp) {
  const int32_t b = tgt[blockIdx.x];
  const int n = threadIdx.x;
  if (n >= kTerms) return;
  const double cx = geo[4 * size_t(b)], cy = geo[4 * size_t(b) + 1], is = 1.0 / geo[4 * size_t(b) + 2];
  const double inv_n = n > 0 ? 1.0 / double(n) : 0.0;
  double ar = 0.0, ai = 0.0;
  const int32_t j1 = bptr[b + 1];
  for (int32_t j = bptr[b]; j < j1; ++j) {
    const double qj = q[j];
    if (n == 0) {
      ar += qj;
      continue;
    }
    const double ex = (sxy[2 * size_t(j)] - cx) * is, ey = (sxy[2 * size_t(j) + 1] - cy) * is;
    double pr, pi;
    cpow(ex, ey, n - 1, pr, pi);
    // eta^(n-1) [ -(q/n) eta + mu/s ]
    const double cr = -qj * inv_n * ex + mu[2 * size_t(j)] * is;
    const double ci = -qj * inv_n * ey + mu[2 * size_t(j) + 1] * is;
    ar += pr * cr - pi * ci;
    ai += pr * ci + pi * cr;
  }
  mp[size_t(b) * kReals + 2 * n] = ar;
  mp[size_t(b) * kReals + 2 * n + 1] = ai;
}

// one wave per target box; lane l < 40 owns term l; adds onto the far part written by M2L
__global__ void __launch_bounds__(64) p2l_kernel(const int32_t* __restrict__ tgt, const int32_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ idx, const int32_t* __restrict__ bptr,
                                                 const double* __restrict__ geo, const double* __restrict__ sxy,
                                                 const double* __restrict__ q, const double* __restrict__ mu,
                                                 double* __restrict__ far) {
  const int i = blockIdx.x;
  const int32_t b = tgt[i];
  const int l = threadIdx.x;
  if (l >= kTerms) return;
  const double cx = geo[4 * size_t(b)], cy = geo[4 * size_t(b) + 1], s = geo[4 * size_t(b) + 2], is = 1.0 / s;
  const double log_s = log(s);
  const double inv_l = l > 0 ? 1.0 / double(l) : 0.0;
  double br = 0.0, bi = 0.0;
  const int32_t e1 = ptr[i + 1];
  for (int32_t e = ptr[i]; e < e1; ++e) {
    const int32_t lb = idx[e];
    const int32_t j1 = bptr[lb + 1];
    for (int32_t j = bptr[lb]; j < j1; ++j) {
      const double wx = (sxy[2 * size_t(j)] - cx) * is, wy = (sxy[2 * size_t(j) + 1] - cy) * is;
      const double d = wx * wx + wy * wy;
      const double vx = wx / d, vy = -wy / d;  // 1 / w
      const double qj = q[j];
      const double mx = mu[2 * size_t(j)] * is, my = mu[2 * size_t(j) + 1] * is;
      const double mvx = mx * vx - my * vy, mvy = mx * vy + my * vx;  // (mu / s) / w
      if (l == 0) {
        br += qj * (0.5 * log(d) + log_s) - mvx;
        bi -= mvy;
      } else {
        double pr, pi;
        cpow(vx, vy, l, pr, pi);
        // w^-l [ -(q/l) - (mu/s) / w ]
        const double cr = -qj * inv_l - mvx, ci = -mvy;
        br += pr * cr - pi * ci;
        bi += pr * ci + pi * cr;
      }
    }
  }
  far[size_t(b) * kReals + 2 * l] += br;
  far[size_t(b) * kReals + 2 * l + 1] += bi;
}

// one block per target leaf, one thread per node; the curve nodes of each adjacent leaf pass
// through LDS in chunks of 256
__global__ void __launch_bounds__(256) p2p_kernel(const int32_t* __restrict__ tgt, const int32_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ idx, const int32_t* __restrict__ leaf_box,
                                                  const int32_t* __restrict__ bptr, const double* __restrict__ geo,
                                                  const double* __restrict__ sxy, const double* __restrict__ q,
                                                  const double* __restrict__ mu, LeafNodes nodes, double* __restrict__ u) {
  __shared__ double sx[256], sy[256], sq[256], smx[256], smy[256];
  const int i = blockIdx.x;
  const int32_t a = tgt[i];
  const int m = threadIdx.x;
  const int32_t b = leaf_box[a];
  const double s = geo[4 * size_t(b) + 2];
  const double x = geo[4 * size_t(b)] + s * nodes.t[m & 15];
  const double y = geo[4 * size_t(b) + 1] + s * nodes.t[m >> 4];
  double vs = 0.0, vd = 0.0;
  const int32_t e1 = ptr[i + 1];
  for (int32_t e = ptr[i]; e < e1; ++e) {
    const int32_t lb = idx[e];
    const int32_t j0 = bptr[lb], j1 = bptr[lb + 1];
    for (int32_t c = j0; c < j1; c += 256) {
      const int nn = min(256, j1 - c);
      __syncthreads();  // the previous chunk is no longer read
      if (m < nn) {
        const size_t j = size_t(c + m);
        sx[m] = sxy[2 * j];
        sy[m] = sxy[2 * j + 1];
        sq[m] = q[j];
        smx[m] = mu[2 * j];
        smy[m] = mu[2 * j + 1];
      }
      __syncthreads();
      for (int k = 0; k < nn; ++k) {
        const double dx = x - sx[k], dy = y - sy[k];
        const double r2 = dx * dx + dy * dy;
        vs += sq[k] * log(r2);
        vd += (smx[k] * dx + smy[k] * dy) / r2;
      }
    }
  }
  u[size_t(a) * 256 + m] = -kInv2Pi * (0.5 * vs + vd);
}

}  // namespace

hipError_t launch_layer_prep(int64_t n, const int32_t* order, const double* w, const double* nrm, const double* sigma,
                             const double* tau, double* q, double* mu, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(layer_prep_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream, n, order, w, nrm, sigma,
                     tau, q, mu);
  return hipGetLastError();
}

hipError_t launch_p2m(int32_t n_tgt, const int32_t* tgt, const int32_t* bptr, const double* geo, const double* sxy,
                      const double* q, const double* mu, double* mp, hipStream_t stream) {
  if (n_tgt <= 0) return hipSuccess;
  hipLaunchKernelGGL(p2m_kernel, dim3(unsigned(n_tgt)), dim3(64), 0, stream, tgt, bptr, geo, sxy, q, mu, mp);
  return hipGetLastError();
}

hipError_t launch_p2l(int32_t n_tgt, const int32_t* tgt, const int32_t* ptr, const int32_t* idx, const int32_t* bptr,
                      const double* geo, const double* sxy, const double* q, const double* mu, double* far,
                      hipStream_t stream) {
  if (n_tgt <= 0) return hipSuccess;
  hipLaunchKernelGGL(p2l_kernel, dim3(unsigned(n_tgt)), dim3(64), 0, stream, tgt, ptr, idx, bptr, geo, sxy, q, mu, far);
  return hipGetLastError();
}

hipError_t launch_p2p(int32_t n_tgt, const int32_t* tgt, const int32_t* ptr, const int32_t* idx, const int32_t* leaf_box,
                      const int32_t* bptr, const double* geo, const double* sxy, const double* q, const double* mu,
                      const LeafNodes& nodes, double* u, hipStream_t stream) {
  if (n_tgt <= 0) return hipSuccess;
  hipLaunchKernelGGL(p2p_kernel, dim3(unsigned(n_tgt)), dim3(256), 0, stream, tgt, ptr, idx, leaf_box, bptr, geo, sxy,
                     q, mu, nodes, u);
  return hipGetLastError();
}

}  // namespace vp
