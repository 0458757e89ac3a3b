// HIP kernels of the strip solve (the factored system built in strip.cpp). One apply is three
// launches:
//   strip_rhs_kernel       per element and 4 rows: s_k = E_k[S, :] b_k and w_k = U~_{k-1} E_k b_k,
//                          b_k = f * rs at the PDE rows (2m dot products of length Bi, a wave each)
//   strip_sweep_kernel     one workgroup: the forward sweep z_{k+1} = s_k + F_k z_k, then
//                          g_k = w_k + G_k z_k and the backward sweep t_k = g_k - H_k t_{k+1},
//                          then the periodic corner h = K [z_n; w_0 - H_0 t_1]
//   strip_solution_kernel  per element and 64-row tile: z*_k = z_k + Pz_k h_lo,
//                          t*_{k+1} = t_{k+1} + Pt_{k+1} h, x_k = E_k (b_k + P' z*_k - P t*_{k+1})
//                          on the interior rows; the Dirichlet rows are zero
// In the sweep, wave 0 runs the recurrence with lane a holding component a of the vector (each
// step writes the vector to a wave-private LDS slot and reads it back as a broadcast), reading
// its m x m matrices from LDS, while waves 1-3 stage the next chunk of matrices (double buffer,
// one barrier per chunk). All sums have a fixed order, so repeated applies are bitwise identical.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "strip.hpp"

namespace vp {

namespace {

constexpr int kStripThreads = 256;
constexpr int kSolThreads = 512;  // solution kernel: 8 waves split the columns of a 64-row tile
constexpr int kMaxM = 30;  // n_r <= 32

__device__ __forceinline__ double lane_value(double v, int lane) {
  // the value held by `lane` (wave-uniform) of this wavefront
  const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffull), lane));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u >> 32), lane));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

__device__ __forceinline__ double wave_total(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(kStripThreads) strip_rhs_kernel(StripDevice d, const double* __restrict__ f) {
  // block (k, y): rows a = 4y .. 4y + 3 of the 2m rows of W_k, one wave each
  extern __shared__ double b[];  // Bi
  const int k = blockIdx.x, q = d.q, Bi = d.Bi, m = d.m;
  const size_t base = size_t(k) * d.B + q;
  for (int c = threadIdx.x; c < Bi; c += kStripThreads) {
    const int j = c % q;
    b[c] = (j != 0 && j != q - 1) ? f[base + c] * d.rs[base + c] : 0.0;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, a = blockIdx.y * (kStripThreads / 64) + wave;
  if (a >= 2 * m) return;
  const double* row = d.W + (size_t(k) * 2 * m + a) * Bi;
  double acc = 0.0;
#pragma unroll 4
  for (int c = lane; c < Bi; c += 64) acc = fma(row[c], b[c], acc);
  acc = wave_total(acc);
  if (lane == 0) (a < m ? d.s : d.w)[size_t(k) * m + (a < m ? a : a - m)] = acc;
}

// One step of a sweep in wave 0: v_a = c_a + sgn * sum_b A[a][b] x_b for lanes a < m, x
// distributed over lanes (load_row, then apply_row). Lanes >= m work on row m - 1 and their value
// is discarded, so every read stays inside A. m is a compile-time constant: straight-line code.
template <int m>
__device__ __forceinline__ void load_row(const double* A, int lane, double (&row)[m]) {
  const int a = lane < m ? lane : m - 1;
#pragma unroll
  for (int b = 0; b < m; ++b) row[b] = A[a * m + b];
}

__device__ __forceinline__ void wave_sync() {
  // orders this wavefront's LDS accesses around the point (the LDS executes a wave's accesses in
  // issue order; the fences keep the compiler from moving them across)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// As apply_row, with x broadcast through a wave-private LDS vector xb (m doubles, 16-byte
// aligned): one write and m/2 broadcast reads instead of 2m lane reads.
template <int m>
__device__ __forceinline__ double apply_row_lds(const double (&row)[m], double c, double x, double sgn, double* xb,
                                                int lane) {
  if (lane < m) xb[lane] = x;
  wave_sync();
  double xv[m];
#pragma unroll
  for (int b = 0; b < m; ++b) xv[b] = xb[b];
  wave_sync();
  double v0 = c, v1 = 0.0;
#pragma unroll
  for (int b = 0; b < m; b += 2) {
    v0 = fma(sgn * row[b], xv[b], v0);
    if (b + 1 < m) v1 = fma(sgn * row[b + 1], xv[b + 1], v1);
  }
  return v0 + v1;
}

template <int m>
__device__ __forceinline__ double apply_row(const double (&row)[m], double c, double x, double sgn) {
  double v0 = c, v1 = 0.0;
#pragma unroll
  for (int b = 0; b < m; b += 2) {
    v0 = fma(sgn * row[b], lane_value(x, b), v0);
    if (b + 1 < m) v1 = fma(sgn * row[b + 1], lane_value(x, b + 1), v1);
  }
  return v0 + v1;
}

// Loader waves copy n_el consecutive doubles from src to dst, 16 loads in flight per thread.
__device__ __forceinline__ void stage(double* dst, const double* __restrict__ src, int n_el, int loader, int nload) {
  constexpr int kU = 16;
  for (int e0 = loader; e0 < n_el; e0 += kU * nload) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + u * nload;
      v[u] = src[e < n_el ? e : n_el - 1];  // clamped: every read inside src
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + u * nload;
      if (e < n_el) dst[e] = v[u];
    }
  }
}

template <int m>
__global__ void __launch_bounds__(kStripThreads) strip_sweep_kernel(StripDevice d) {
  extern __shared__ double sm[];
  // a chunk buffer holds C matrices (m x m each) followed by C vectors (m each)
  const int n = d.n, C = d.chunk, mm = m * m, st = mm + m;
  // buffer i of the double buffer, computed from the LDS base so that the accesses stay LDS
  // accesses (a pointer taken through a private array would become a generic one)
  auto buf = [&](int i) { return sm + size_t(i & 1) * C * st; };
  double* xb = sm + size_t(2) * C * st;  // wave 0's broadcast vector (32 doubles)
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int loader = tid - 64, nload = kStripThreads - 64;
  const int nfc = (n + C - 1) / C;        // forward chunks: buffers 0 .. nfc - 1
  const int nb = n - 1, nbc = (nb + C - 1) / C;  // backward chunks: buffers nfc .. nfc + nbc - 1

  // forward sweep, steps k = 0 .. n - 1: [F_k] [s_k]
  auto load_fwd = [&](int ci, double* dst) {
    const int k0 = ci * C, ns = min(C, n - k0);
    stage(dst, d.F + size_t(k0) * mm, ns * mm, loader, nload);
    stage(dst + size_t(C) * mm, d.s + size_t(k0) * m, ns * m, loader, nload);
  };
  // backward sweep, steps k = n - 1 .. 1 (u = n - 1 - k): the chunk's H_k are one contiguous
  // range, stored ascending in k ([H_klo .. H_khi]); then g_k = w_k + G_k z_k, stored by u
  auto load_bwd_h = [&](int ci, double* dst) {
    const int u0 = ci * C, ns = min(C, nb - u0), klo = n - u0 - ns;
    stage(dst, d.H + size_t(klo) * mm, ns * mm, loader, nload);
  };
  auto load_bwd_g = [&](int ci, double* dst) {
    const int u0 = ci * C, ns = min(C, nb - u0);
    for (int e = loader; e < ns * m; e += nload) {
      const int uu = e / m, a = e - uu * m, k = n - 1 - (u0 + uu);
      const double* Gk = d.G + size_t(k) * mm + size_t(a) * m;
      const double* zk = d.z + size_t(k) * m;
      double gv[m], zv[m];
#pragma unroll
      for (int b = 0; b < m; ++b) { gv[b] = Gk[b]; zv[b] = zk[b]; }
      double g = d.w[size_t(k) * m + a];
#pragma unroll
      for (int b = 0; b < m; ++b) g = fma(gv[b], zv[b], g);
      dst[size_t(C) * mm + e] = g;
    }
  };

  if (wave > 0) load_fwd(0, buf(0));
  if (wave == 0 && lane < m) d.z[lane] = 0.0;
  double z = 0.0;
  __syncthreads();
  for (int ci = 0; ci < nfc; ++ci) {
    if (wave == 0) {
      const double* cb = buf(ci);
      const int k0 = ci * C, ns = min(C, n - k0), ml = min(lane, m - 1);
      for (int kk = 0; kk < ns; ++kk) {
        double row[m];
        load_row<m>(cb + size_t(kk) * mm, lane, row);
        z = apply_row_lds<m>(row, cb[size_t(C) * mm + size_t(kk) * m + ml], z, 1.0, xb, lane);
        if (lane < m) d.z[size_t(k0 + kk + 1) * m + lane] = z;
      }
    } else if (ci + 1 < nfc) {
      load_fwd(ci + 1, buf(ci + 1));
    } else {
      load_bwd_h(0, buf(nfc));  // H of the first backward chunk does not wait for z
    }
    __syncthreads();
  }
  const double zn = z;

  if (wave > 0) load_bwd_g(0, buf(nfc));
  if (wave == 0 && lane < m) d.t[size_t(n) * m + lane] = 0.0;
  double t = 0.0;
  __syncthreads();
  for (int ci = 0; ci < nbc; ++ci) {
    if (wave == 0) {
      const double* cb = buf(nfc + ci);
      const int u0 = ci * C, ns = min(C, nb - u0), ml = min(lane, m - 1);
      // step uu works on k = n - 1 - (u0 + uu); the chunk stores its H_k ascending in k, so H_k
      // is the chunk's matrix ns - 1 - uu
      for (int uu = 0; uu < ns; ++uu) {
        double row[m];
        load_row<m>(cb + size_t(ns - 1 - uu) * mm, lane, row);
        t = apply_row_lds<m>(row, cb[size_t(C) * mm + size_t(uu) * m + ml], t, -1.0, xb, lane);
        if (lane < m) d.t[size_t(n - 1 - (u0 + uu)) * m + lane] = t;
      }
    } else if (ci + 1 < nbc) {
      load_bwd_h(ci + 1, buf(nfc + ci + 1));
      load_bwd_g(ci + 1, buf(nfc + ci + 1));
    }
    __syncthreads();
  }

  // periodic corner: h = K [z_n; w_0 - H_0 t_1] (t holds t_1)
  if (wave == 0) {
    const int m2 = 2 * m, ak = lane < m2 ? lane : m2 - 1;
    double h0row[m];
    load_row<m>(d.H, lane, h0row);
    const double g2 = apply_row<m>(h0row, d.w[min(lane, m - 1)], t, -1.0);
    double h = 0.0;
#pragma unroll
    for (int j = 0; j < m; ++j)
      h = fma(d.K[ak * m2 + m + j], lane_value(g2, j), fma(d.K[ak * m2 + j], lane_value(zn, j), h));
    if (lane < m2) d.h[lane] = h;
  }
}

__global__ void __launch_bounds__(kSolThreads)
    strip_solution_kernel(StripDevice d, const double* __restrict__ f, double* __restrict__ x) {
  extern __shared__ double sm[];  // r (Bi), z* (m), t* (m), partial sums (kSolThreads)
  const int k = blockIdx.x, tile = blockIdx.y, q = d.q, Bi = d.Bi, m = d.m, B = d.B;
  double* r = sm;
  double* zs = r + Bi;
  double* ts = zs + m;
  double* red = ts + m;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid < m) {
    const double* P = d.Pz + size_t(k) * m * m + size_t(tid) * m;
    double v = d.z[size_t(k) * m + tid];
    for (int b = 0; b < m; ++b) v = fma(P[b], d.h[b], v);
    zs[tid] = v;
  } else if (tid >= 64 && tid < 64 + m) {
    const int a = tid - 64, m2 = 2 * m;
    const double* P = d.Pt + size_t(k + 1) * m * m2 + size_t(a) * m2;
    double v = d.t[size_t(k + 1) * m + a];
    for (int j = 0; j < m2; ++j) v = fma(P[j], d.h[j], v);
    ts[a] = v;
  }
  __syncthreads();
  const size_t base = size_t(k) * B + q;
  for (int c = tid; c < Bi; c += kSolThreads) {
    const int j = c % q, a = c / q;
    r[c] = j == 0 ? zs[a] : (j == q - 1 ? -ts[a] : f[base + c] * d.rs[base + c]);
  }
  __syncthreads();
  constexpr int kWaves = kSolThreads / 64;
  const int p = tile * 64 + lane, per = (Bi + kWaves - 1) / kWaves, c0 = wave * per, c1 = min(Bi, c0 + per);
  double acc = 0.0;
  if (p < Bi) {
    const double* E = d.EiT + size_t(k) * Bi * Bi + p;
#pragma unroll 8
    for (int c = c0; c < c1; ++c) acc = fma(E[size_t(c) * Bi], r[c], acc);
  }
  red[tid] = acc;
  __syncthreads();
  if (wave == 0 && p < Bi) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) v += red[w * 64 + lane];
    x[base + p] = v;
  }
  if (tile == 0 && tid < 2 * q) x[size_t(k) * B + (tid < q ? tid : B - 2 * q + tid)] = 0.0;
}

// Work vectors of the apply (s, w, z, t, h) for callers that cannot allocate: one static array
// per device, held until the process ends. Host code reaches it only through the address
// hipGetSymbolAddress returns on each device (strip_scratch); the array's name is not a device
// address on the host.
static __device__ __align__(256) double scratch[kStripScratchDoubles];

}  // namespace

hipError_t strip_scratch(double** out) {
  static std::mutex mu;
  static std::vector<double*> per_device;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if (per_device.size() <= size_t(dev)) per_device.resize(size_t(dev) + 1, nullptr);
  if (!per_device[size_t(dev)]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    per_device[size_t(dev)] = static_cast<double*>(p);
  }
  *out = per_device[size_t(dev)];
  return hipSuccess;
}

hipError_t launch_strip_solve(const StripDevice& d, const double* f, double* v, hipStream_t stream) {
  if (d.m < 2 || d.m > kMaxM) return hipErrorInvalidValue;  // the plan keeps 4 <= n_r <= 32
  const size_t lds_sweep = (size_t(2) * d.chunk * (d.m * d.m + d.m) + 32) * sizeof(double);
  hipLaunchKernelGGL(strip_rhs_kernel, dim3(unsigned(d.n), unsigned((2 * d.m + 3) / 4)), dim3(kStripThreads),
                     size_t(d.Bi) * sizeof(double), stream, d, f);
  using Sweep = void (*)(StripDevice);
  static const Sweep sweeps[kMaxM + 1] = {
      nullptr, nullptr, strip_sweep_kernel<2>, strip_sweep_kernel<3>, strip_sweep_kernel<4>, strip_sweep_kernel<5>,
      strip_sweep_kernel<6>, strip_sweep_kernel<7>, strip_sweep_kernel<8>, strip_sweep_kernel<9>, strip_sweep_kernel<10>,
      strip_sweep_kernel<11>, strip_sweep_kernel<12>, strip_sweep_kernel<13>, strip_sweep_kernel<14>,
      strip_sweep_kernel<15>, strip_sweep_kernel<16>, strip_sweep_kernel<17>, strip_sweep_kernel<18>,
      strip_sweep_kernel<19>, strip_sweep_kernel<20>, strip_sweep_kernel<21>, strip_sweep_kernel<22>,
      strip_sweep_kernel<23>, strip_sweep_kernel<24>, strip_sweep_kernel<25>, strip_sweep_kernel<26>,
      strip_sweep_kernel<27>, strip_sweep_kernel<28>, strip_sweep_kernel<29>, strip_sweep_kernel<30>};
  hipLaunchKernelGGL(sweeps[d.m], dim3(1), dim3(kStripThreads), lds_sweep, stream, d);
  hipLaunchKernelGGL(strip_solution_kernel, dim3(unsigned(d.n), unsigned((d.Bi + 63) / 64)), dim3(kSolThreads),
                     size_t(d.Bi + 2 * d.m + kSolThreads) * sizeof(double), stream, d, f, v);
  return hipGetLastError();
}

}  // namespace vp
