// HIP kernel of the evaluation of the volume potential and its gradient at arbitrary points
// (v_bulk and its normal derivative on the fictitious curve feed the glue step, Alg. 1 and
// Sec. 4.4), FP64. It runs after a forward apply, whose expansions it reads:
//   u(x) = -(1/2pi) Re psi_a(x)                          local expansion of the point's leaf a
//        + sum_{c in W(a)} -(1/2pi) Re phi_c(x)          multipoles of a's W list
//        + sum_{b in U(a)} m_b(x) . f_b                   adjacent leaves: plan-time moments
// with psi_a = sum_l b_l w^l, w = (z - c_a) / s_a, and phi_c = a_0 log|z - c_c| + sum_k a_k
// (s_c / (z - c_c))^k. Gradients: d/dx Re F = Re F', d/dy Re F = -Im F' for analytic F.
// One wave per point; the lanes split the moment dot products and the expansion terms, and a
// fixed butterfly adds them (deterministic).
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace vp {

namespace {

constexpr int kTerms = 40;
constexpr int kReals = 80;
constexpr double kInv2Pi = 0.15915494309189533576888376337251436;

__device__ __forceinline__ void cpow_(double x, double y, int k, double& pr, double& pi) {
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(64) points_kernel(PointParams p) {
  const int i = blockIdx.x;
  const int l = threadIdx.x;
  const double x = p.xy[2 * size_t(i)], y = p.xy[2 * size_t(i) + 1];
  double u = 0.0, gx = 0.0, gy = 0.0;
  // adjacent leaves: moment dot products (lane l takes values l, l+64, l+128, l+192)
  for (int32_t e = p.near_ptr[i]; e < p.near_ptr[i + 1]; ++e) {
    const double* __restrict__ m = p.mom + size_t(e) * 768;
    const double* __restrict__ f = p.f + size_t(p.near_leaf[e]) * 256;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = l + 64 * q;
      const double fk = f[k];
      u = fma(m[k], fk, u);
      gx = fma(m[256 + k], fk, gx);
      gy = fma(m[512 + k], fk, gy);
    }
  }
  double pr = 0.0, pi = 0.0, dr = 0.0, di = 0.0;  // sum of expansion terms F and of F'
  // local expansion of the point's leaf
  const int32_t a = p.loc_box[i];
  if (a >= 0 && l < kTerms) {
    const double* g = p.geo + 4 * size_t(a);
    const double is = 1.0 / g[2];
    const double wx = (x - g[0]) * is, wy = (y - g[1]) * is;
    const double br = p.loc[size_t(a) * kReals + 2 * l], bi = p.loc[size_t(a) * kReals + 2 * l + 1];
    double tr, ti;
    cpow_(wx, wy, l, tr, ti);  // w^l
    pr += br * tr - bi * ti;
    pi += br * ti + bi * tr;
    if (l > 0) {  // l b_l w^(l-1) / s
      double sr, si;
      cpow_(wx, wy, l - 1, sr, si);
      const double c = double(l) * is;
      dr += c * (br * sr - bi * si);
      di += c * (br * si + bi * sr);
    }
  }
  // multipoles of the W list
  for (int32_t e = p.w_ptr[i]; e < p.w_ptr[i + 1]; ++e) {
    if (l >= kTerms) break;
    const int32_t c = p.w_box[e];
    const double* g = p.geo + 4 * size_t(c);
    const double s = g[2];
    const double zx = x - g[0], zy = y - g[1];
    const double d2 = zx * zx + zy * zy;
    const double vx = zx / d2, vy = -zy / d2;  // 1 / (z - c)
    const double ar = p.mp[size_t(c) * kReals + 2 * l], ai = p.mp[size_t(c) * kReals + 2 * l + 1];
    if (l == 0) {  // a_0 log|z - c| and a_0 / (z - c)
      pr += ar * 0.5 * log(d2);
      dr += ar * vx - ai * vy;
      di += ar * vy + ai * vx;
    } else {  // a_k (s / (z - c))^k and -k a_k (s / (z - c))^k / (z - c)
      double tr, ti;
      cpow_(s * vx, s * vy, l, tr, ti);
      const double qr = ar * tr - ai * ti, qi = ar * ti + ai * tr;
      pr += qr;
      pi += qi;
      dr -= double(l) * (qr * vx - qi * vy);
      di -= double(l) * (qr * vy + qi * vx);
    }
  }
  u += -kInv2Pi * pr;
  gx += -kInv2Pi * dr;
  gy += kInv2Pi * di;
  u = wave_sum(u);
  gx = wave_sum(gx);
  gy = wave_sum(gy);
  if (l == 0) {
    p.u[i] = u;
    if (p.grad) {
      p.grad[2 * size_t(i)] = gx;
      p.grad[2 * size_t(i) + 1] = gy;
    }
  }
}

}  // namespace

hipError_t launch_points(const PointParams& p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(points_kernel, dim3(unsigned(n)), dim3(64), 0, stream, p);
  return hipGetLastError();
}

}  // namespace vp
