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
//   P2P  direct sum at the 256 nodes of a leaf over the curve nodes in its adjacent leaves,
//        added onto the far field (only leaves with curve nodes nearby are launched).
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

// The curve nodes a target reads: the sorted nodes of the leaf boxes idx[e0 .. e1) (at most
// kMaxRanges of them; the plan checks), numbered 0 .. total-1 in list order; list_node() maps a
// position of that numbering to its sorted node. Kernels stage CH of them at a time in LDS.
constexpr int kMaxRanges = 64;
constexpr int CH = 256;

struct NodeList {
  int32_t start[kMaxRanges];  // first sorted node of each range
  int32_t pre[kMaxRanges + 1];  // prefix of the range lengths
  int n_ranges;
};

__device__ __forceinline__ int list_init(NodeList& L, const int32_t* __restrict__ idx, int32_t e0, int32_t e1,
                                         const int32_t* __restrict__ bptr, int tid) {
  const int nr = e1 - e0;
  if (tid < nr) {
    const int32_t b = idx[e0 + tid];
    L.start[tid] = bptr[b];
    L.pre[tid + 1] = bptr[b + 1] - bptr[b];
  }
  __syncthreads();
  if (tid == 0) {
    L.pre[0] = 0;
    for (int r = 0; r < nr; ++r) L.pre[r + 1] += L.pre[r];
    L.n_ranges = nr;
  }
  __syncthreads();
  return L.pre[nr];
}

// sorted node index of list position k < total
__device__ __forceinline__ int32_t list_node(const NodeList& L, int k) {
  int r = 0;
  while (k >= L.pre[r + 1]) ++r;
  return L.start[r] + (k - L.pre[r]);
}

// Multipole / local expansion of one target from its nodes: thread t < 240 owns term l = t % 40
// and the nodes k = g (mod 6) of each staged chunk, g = t / 40; the six partial sums of a term
// are added in g order at the end (fixed order: deterministic).
constexpr int kGroups = 6;

// P2M (local == false): terms of eta = (zeta - c) / s; P2L (local == true): terms of 1 / w,
// w = (zeta - c) / s, added onto the output.
template <bool local>
__device__ __forceinline__ void expand(int32_t b, const NodeList& L, int total, const double* __restrict__ geo,
                                       const double* __restrict__ sxy, const double* __restrict__ q,
                                       const double* __restrict__ mu, double* __restrict__ out, int tid) {
  __shared__ double zr[CH], zi[CH], cq[CH], dr[CH], di[CH], lg[CH];
  __shared__ double red[kGroups][2 * kTerms];
  const double cx = geo[4 * size_t(b)], cy = geo[4 * size_t(b) + 1], s = geo[4 * size_t(b) + 2], is = 1.0 / s;
  const int l = tid % kTerms, g = tid / kTerms;
  const double inv_l = l > 0 ? 1.0 / double(l) : 0.0;
  double br = 0.0, bi = 0.0;
  for (int c0 = 0; c0 < total; c0 += CH) {
    const int nn = min(CH, total - c0);
    __syncthreads();  // the previous chunk is no longer read
    if (tid < nn) {
      const size_t j = size_t(list_node(L, c0 + tid));
      const double wx = (sxy[2 * j] - cx) * is, wy = (sxy[2 * j + 1] - cy) * is;
      const double mx = mu[2 * j] * is, my = mu[2 * j + 1] * is;  // mu / s
      cq[tid] = q[j];
      if (local) {
        const double d = wx * wx + wy * wy;
        const double vx = wx / d, vy = -wy / d;  // 1 / w
        zr[tid] = vx;
        zi[tid] = vy;
        dr[tid] = mx * vx - my * vy;  // (mu / s) / w
        di[tid] = mx * vy + my * vx;
        lg[tid] = q[j] * (0.5 * log(d) + log(s));  // q log|zeta - c|
      } else {
        zr[tid] = wx;
        zi[tid] = wy;
        dr[tid] = mx;
        di[tid] = my;
      }
    }
    __syncthreads();
    if (g < kGroups) {
      for (int k = g; k < nn; k += kGroups) {
        const double qk = cq[k];
        if (local) {
          // b_0 += q log|zeta - c| - (mu/s)/w;  b_l += w^-l [ -(q/l) - (mu/s)/w ]
          if (l == 0) {
            br += lg[k] - dr[k];
            bi -= di[k];
          } else {
            double pr, pi;
            cpow(zr[k], zi[k], l, pr, pi);
            const double cr = -qk * inv_l - dr[k], ci = -di[k];
            br += pr * cr - pi * ci;
            bi += pr * ci + pi * cr;
          }
        } else {
          // a_0 += q;  a_n += eta^(n-1) [ -(q/n) eta + mu/s ]
          if (l == 0) {
            br += qk;
          } else {
            double pr, pi;
            cpow(zr[k], zi[k], l - 1, pr, pi);
            const double cr = -qk * inv_l * zr[k] + dr[k], ci = -qk * inv_l * zi[k] + di[k];
            br += pr * cr - pi * ci;
            bi += pr * ci + pi * cr;
          }
        }
      }
      red[g][2 * l] = br;
      red[g][2 * l + 1] = bi;
    }
    br = bi = 0.0;
    __syncthreads();
    if (tid < 2 * kTerms) {  // add this chunk's group sums in group order
      double v = 0.0;
      for (int gg = 0; gg < kGroups; ++gg) v += red[gg][tid];
      double* o = out + size_t(b) * kReals + tid;
      *o = (local || c0 > 0) ? *o + v : v;
    }
  }
}

__global__ void __launch_bounds__(256) p2m_kernel(const int32_t* __restrict__ tgt, const int32_t* __restrict__ bptr,
                                                  const double* __restrict__ geo, const double* __restrict__ sxy,
                                                  const double* __restrict__ q, const double* __restrict__ mu,
                                                  double* __restrict__ mp) {
  __shared__ NodeList L;
  const int32_t b = tgt[blockIdx.x];
  const int total = list_init(L, tgt, blockIdx.x, blockIdx.x + 1, bptr, threadIdx.x);
  expand<false>(b, L, total, geo, sxy, q, mu, mp, threadIdx.x);
}

__global__ void __launch_bounds__(256) p2l_kernel(const int32_t* __restrict__ tgt, const int32_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ idx, const int32_t* __restrict__ bptr,
                                                  const double* __restrict__ geo, const double* __restrict__ sxy,
                                                  const double* __restrict__ q, const double* __restrict__ mu,
                                                  double* __restrict__ far) {
  __shared__ NodeList L;
  const int i = blockIdx.x;
  const int total = list_init(L, idx, ptr[i], ptr[i + 1], bptr, threadIdx.x);
  expand<true>(tgt[i], L, total, geo, sxy, q, mu, far, threadIdx.x);
}

// log x for finite x >= 0 (log 0 = -inf), table-driven after P. T. P. Tang (ACM TOMS 16, 1990): x = 2^e m with
// m in [1, 2); c = m with all but its 7 leading fraction bits cleared (so m - c is exact and
// 0 <= r = (m - c) / c < 2^-7); log x = e log 2 + log c + log1p(r), the last by its Taylor
// series to r^8 (truncation below 2^-60 relative). lc[i] = log(1 + i/128) and ic[i] = 1 / (1 + i/128)
// come from the block's table. The absolute error is a few units in the last place of
// max(|e log 2|, 1); just below x = 1 the two leading terms cancel and the relative error of the
// (small) result grows, which a weighted sum of logarithms does not notice.
__device__ __forceinline__ double table_log(double x, const double* __restrict__ lc, const double* __restrict__ ic) {
  int e;
  double m = frexp(x, &e);  // m in [0.5, 1)
  m *= 2.0;
  e -= 1;
  const unsigned long long bits = __double_as_longlong(m);
  const int i = int((bits >> 45) & 127);
  const double c = __longlong_as_double(bits & ~((1ull << 45) - 1));
  const double r = (m - c) * ic[i];
  // log1p(r) = r - r^2/2 + r^3/3 - ... + (-1)^7 r^8/8  (Horner)
  double p = -1.0 / 8.0;
  p = fma(p, r, 1.0 / 7.0);
  p = fma(p, r, -1.0 / 6.0);
  p = fma(p, r, 1.0 / 5.0);
  p = fma(p, r, -1.0 / 4.0);
  p = fma(p, r, 1.0 / 3.0);
  p = fma(p, r, -0.5);
  p = fma(p, r * r, r);
  const double v = fma(double(e), 0.69314718055994530941723212145817657, lc[i] + p);
  return x == 0.0 ? -__builtin_inf() : v;  // frexp(0) gives m = 0, which the table would map to -log 2
}

// 1 / x for finite x > 0: the hardware estimate refined by two Newton-Raphson steps
// (y <- y + y (1 - x y)), each of which squares the relative error.
__device__ __forceinline__ double recip(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double t = fma(-x, y, 1.0);
  y = fma(y, t, y);
  t = fma(-x, y, 1.0);
  return fma(y, t, y);
}

// one block per target leaf, one thread per node; u += direct sum over the curve nodes of its
// adjacent leaves, staged through LDS 256 at a time
__global__ void __launch_bounds__(256) p2p_kernel(const int32_t* __restrict__ tgt, const int32_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ idx, const int32_t* __restrict__ leaf_box,
                                                  const int32_t* __restrict__ bptr, const double* __restrict__ geo,
                                                  const double* __restrict__ sxy, const double* __restrict__ q,
                                                  const double* __restrict__ mu, LeafNodes nodes, double* __restrict__ u) {
  __shared__ double sx[CH], sy[CH], sq[CH], smx[CH], smy[CH];
  __shared__ double lc[128], ic[128];
  __shared__ NodeList L;
  const int i = blockIdx.x;
  const int32_t a = tgt[i];
  const int m = threadIdx.x;
  if (m < 128) {  // the logarithm's table (list_init's barrier publishes it)
    const double c = 1.0 + double(m) / 128.0;
    lc[m] = log(c);
    ic[m] = 1.0 / c;
  }
  const int total = list_init(L, idx, ptr[i], ptr[i + 1], bptr, m);
  const int32_t b = leaf_box[a];
  const double s = geo[4 * size_t(b) + 2];
  const double x = geo[4 * size_t(b)] + s * nodes.t[m & 15];
  const double y = geo[4 * size_t(b) + 1] + s * nodes.t[m >> 4];
  double vs = 0.0, vd = 0.0;
  for (int c0 = 0; c0 < total; c0 += CH) {
    const int nn = min(CH, total - c0);
    __syncthreads();  // the previous chunk is no longer read
    if (m < nn) {
      const size_t j = size_t(list_node(L, c0 + m));
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
      vs = fma(sq[k], table_log(r2, lc, ic), vs);
      vd = fma(smx[k] * dx + smy[k] * dy, recip(r2), vd);
    }
  }
  u[size_t(a) * 256 + m] += -kInv2Pi * (0.5 * vs + vd);
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
  hipLaunchKernelGGL(p2m_kernel, dim3(unsigned(n_tgt)), dim3(256), 0, stream, tgt, bptr, geo, sxy, q, mu, mp);
  return hipGetLastError();
}

hipError_t launch_p2l(int32_t n_tgt, const int32_t* tgt, const int32_t* ptr, const int32_t* idx, const int32_t* bptr,
                      const double* geo, const double* sxy, const double* q, const double* mu, double* far,
                      hipStream_t stream) {
  if (n_tgt <= 0) return hipSuccess;
  hipLaunchKernelGGL(p2l_kernel, dim3(unsigned(n_tgt)), dim3(256), 0, stream, tgt, ptr, idx, bptr, geo, sxy, q, mu, far);
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
