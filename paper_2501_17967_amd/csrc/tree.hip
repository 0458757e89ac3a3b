// HIP kernels of the adaptive quadtree construction (Sec. 4.2.1, Alg. 2): the node
// coordinates of the boxes to be sampled, and each sampled box's Chebyshev tail
//     max { |c_nm| : n >= p - 2 or m >= p - 2 },  c = D V D^T,
// V[j][i] the samples (x fastest), D[m][i] = (2 - delta_m0)/p T_m(t_i) the transform from values
// at the first-kind points to Chebyshev coefficients. One wave per box; the maximum is exact,
// so the tail does not depend on the reduction order.
//
// The bookkeeping stays on the device as well: each round's split decisions and the
// compaction of the split boxes' children and of the new leaves (prefix sums), and the 2:1
// balance over edges and corners. The balance works on the sorted leaf keys and the sorted keys
// of all their proper ancestors (the internal boxes): a neighbour box q (same level, one of the
// eight around a leaf) is fine when q is a leaf, an internal box, or a child of a leaf;
// otherwise the leaf covering q is two or more levels coarser, found by binary searches at the
// coarser levels, and is split. Rounds of this run until no leaf is split; the result is the
// coarsest balanced refinement, which is unique, so it does not depend on the order of splits.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

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

constexpr uint64_t kMask29 = (uint64_t(1) << 29) - 1;
__device__ __forceinline__ int key_lv(uint64_t k) { return int(k >> 58); }
__device__ __forceinline__ uint64_t key_ix(uint64_t k) { return (k >> 29) & kMask29; }
__device__ __forceinline__ uint64_t key_iy(uint64_t k) { return k & kMask29; }
__device__ __forceinline__ uint64_t key_of(int l, uint64_t x, uint64_t y) { return (uint64_t(l) << 58) | (x << 29) | y; }

// position of k in the ascending array a[0..n), or -1
__device__ __forceinline__ int64_t find_key(const uint64_t* __restrict__ a, int64_t n, uint64_t k) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && a[lo] == k) ? lo : -1;
}

__global__ void decide_kernel(const uint64_t* __restrict__ keys, const double* __restrict__ tails, int64_t n,
                              double tol, int max_level, int32_t* __restrict__ split) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // a non-finite tail is not <= tol: the box is split (down to max_level)
  split[i] = (key_lv(keys[i]) < max_level && !(tails[i] <= tol)) ? 1 : 0;
}

// children of split boxes to next[4 pos[i] ..], the others to leaves[n_leaves + i - pos[i]]
__global__ void emit_kernel(const uint64_t* __restrict__ keys, const int32_t* __restrict__ split,
                            const int32_t* __restrict__ pos, int64_t n, uint64_t* __restrict__ next,
                            uint64_t* __restrict__ leaves, int64_t n_leaves) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = keys[i];
  if (split[i]) {
    const int l = key_lv(k) + 1;
    const uint64_t x = 2 * key_ix(k), y = 2 * key_iy(k);
    uint64_t* o = next + 4 * int64_t(pos[i]);
    o[0] = key_of(l, x, y);
    o[1] = key_of(l, x + 1, y);
    o[2] = key_of(l, x, y + 1);
    o[3] = key_of(l, x + 1, y + 1);
  } else {
    leaves[n_leaves + i - pos[i]] = k;
  }
}

// proper ancestors of each leaf at anc[off[i] ..], off = exclusive sum of the levels
__global__ void ancestors_kernel(const uint64_t* __restrict__ leaves, const int32_t* __restrict__ off, int64_t n,
                                 uint64_t* __restrict__ anc) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = leaves[i];
  const int l = key_lv(k);
  uint64_t x = key_ix(k), y = key_iy(k);
  uint64_t* o = anc + off[i];
  for (int a = l - 1; a >= 0; --a) {
    x >>= 1;
    y >>= 1;
    o[l - 1 - a] = key_of(a, x, y);
  }
}

__global__ void level_kernel(const uint64_t* __restrict__ leaves, int64_t n, int32_t* __restrict__ lv) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) lv[i] = key_lv(leaves[i]);
}

// one thread per (leaf, neighbour direction): flag[j] = 1 for the leaf j (position in the sorted
// leaves) that covers a same-level neighbour of leaf i from two or more levels up
__global__ void balance_check_kernel(const uint64_t* __restrict__ leaves, int64_t n, const uint64_t* __restrict__ inner,
                                     int64_t n_inner, int32_t* __restrict__ flag) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= 8 * n) return;
  const int64_t i = t >> 3;
  const int d = int(t & 7), dd = d < 4 ? d : d + 1;  // the 8 of the 3 x 3 offsets, centre skipped
  const int dx = dd % 3 - 1, dy = dd / 3 - 1;
  const uint64_t k = leaves[i];
  const int l = key_lv(k);
  const int64_t qx = int64_t(key_ix(k)) + dx, qy = int64_t(key_iy(k)) + dy, lim = int64_t(1) << l;
  if (qx < 0 || qy < 0 || qx >= lim || qy >= lim) return;
  const uint64_t q = key_of(l, uint64_t(qx), uint64_t(qy));
  if (find_key(leaves, n, q) >= 0 || find_key(inner, n_inner, q) >= 0) return;
  if (l > 0 && find_key(leaves, n, key_of(l - 1, uint64_t(qx) >> 1, uint64_t(qy) >> 1)) >= 0) return;
  for (int c = l - 2; c >= 0; --c) {
    const int sh = l - c;
    const int64_t j = find_key(leaves, n, key_of(c, uint64_t(qx) >> sh, uint64_t(qy) >> sh));
    if (j >= 0) {
      flag[j] = 1;  // every writer stores the same value
      return;
    }
  }
}

// leaves kept at out[j - pos[j]], a flagged leaf's four children at out[n - n_flag + 4 pos[j] ..]
__global__ void balance_split_kernel(const uint64_t* __restrict__ leaves, const int32_t* __restrict__ flag,
                                     const int32_t* __restrict__ pos, int64_t n, int64_t n_keep,
                                     uint64_t* __restrict__ out) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint64_t k = leaves[j];
  if (!flag[j]) {
    out[j - pos[j]] = k;
    return;
  }
  const int l = key_lv(k) + 1;
  const uint64_t x = 2 * key_ix(k), y = 2 * key_iy(k);
  uint64_t* o = out + n_keep + 4 * int64_t(pos[j]);
  o[0] = key_of(l, x, y);
  o[1] = key_of(l, x + 1, y);
  o[2] = key_of(l, x, y + 1);
  o[3] = key_of(l, x + 1, y + 1);
}

__global__ void zero_kernel(int32_t* __restrict__ a, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

// (level, x, y) keys to (level, y, x) keys, whose ascending order is by level, then y, then x
__global__ void swap_xy_kernel(uint64_t* __restrict__ keys, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = keys[i];
  keys[i] = key_of(key_lv(k), key_iy(k), key_ix(k));
}

constexpr int kThreads = 256;
inline unsigned blocks_for(int64_t n) { return unsigned((n + kThreads - 1) / kThreads); }

template <class T>
hipError_t grow(T*& p, size_t& cap, size_t need) {
  if (need <= cap) return hipSuccess;
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
  const size_t c = std::max<size_t>(need, 1024);
  hipError_t e = hipMalloc(&p, c * sizeof(T));
  if (e == hipSuccess) cap = c;
  return e;
}

hipError_t grow_scratch(TreeWork& w, size_t bytes) {
  if (bytes <= w.scratch_bytes) return hipSuccess;
  if (w.scratch) (void)hipFree(w.scratch);
  w.scratch = nullptr;
  w.scratch_bytes = 0;
  hipError_t e = hipMalloc(&w.scratch, bytes);
  if (e == hipSuccess) w.scratch_bytes = bytes;
  return e;
}

// pos = exclusive sum of flag[0..n); returns the total in *total (read back: synchronises)
hipError_t exclusive_count(TreeWork& w, const int32_t* flag, int32_t* pos, int64_t n, int64_t* total,
                           hipStream_t stream) {
  size_t bytes = 0;
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, flag, pos, int(n), stream);
  if (e == hipSuccess) e = grow_scratch(w, bytes);
  if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(w.scratch, bytes, flag, pos, int(n), stream);
  int32_t last[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(&last[0], pos + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&last[1], flag + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  *total = int64_t(last[0]) + last[1];
  return e;
}

hipError_t sort_keys(TreeWork& w, const uint64_t* in, uint64_t* out, int64_t n, hipStream_t stream) {
  size_t bytes = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, in, out, int(n), 0, 64, stream);
  if (e == hipSuccess) e = grow_scratch(w, bytes);
  if (e == hipSuccess) e = hipcub::DeviceRadixSort::SortKeys(w.scratch, bytes, in, out, int(n), 0, 64, stream);
  return e;
}

}  // namespace

hipError_t tree_upload_pending(TreeWork& w, const uint64_t* keys, int64_t n, hipStream_t stream) {
  hipError_t e = grow(w.pend, w.cap_pend, size_t(n));
  if (e == hipSuccess && n > 0) e = hipMemcpyAsync(w.pend, keys, size_t(n) * sizeof(uint64_t), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e == hipSuccess) w.n_pend = n;
  return e;
}

hipError_t tree_round(TreeWork& w, const double* values, const TreeRule& r, double tol, int max_level,
                      hipStream_t stream) {
  const int64_t n = w.n_pend;
  if (n <= 0) return hipSuccess;
  if (n > (int64_t(1) << 29)) return hipErrorInvalidValue;
  hipError_t e = grow(w.tails, w.cap_tails, size_t(n));
  if (e == hipSuccess) e = grow(w.flag, w.cap_flag, size_t(n));
  if (e == hipSuccess) e = grow(w.pos, w.cap_pos, size_t(n));
  if (e == hipSuccess) e = launch_tree_tail(values, n, r, w.tails, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(decide_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, stream, w.pend, w.tails, n, tol,
                     max_level, w.flag);
  int64_t n_split = 0;
  e = exclusive_count(w, w.flag, w.pos, n, &n_split, stream);
  if (e == hipSuccess) e = grow(w.next, w.cap_next, size_t(4 * n_split));
  if (e == hipSuccess && size_t(w.n_leaves + n - n_split) > w.cap_leaves) {
    // a larger leaf array that keeps the leaves found so far
    uint64_t* nl = nullptr;
    const size_t c = std::max<size_t>(size_t(2 * (w.n_leaves + n)), 1024);
    e = hipMalloc(&nl, c * sizeof(uint64_t));
    if (e == hipSuccess && w.n_leaves > 0)
      e = hipMemcpyAsync(nl, w.leaves, size_t(w.n_leaves) * sizeof(uint64_t), hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess) {
      if (w.leaves) (void)hipFree(w.leaves);
      w.leaves = nl;
      w.cap_leaves = c;
    } else if (nl) {
      (void)hipFree(nl);
    }
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(emit_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, stream, w.pend, w.flag, w.pos, n, w.next,
                     w.leaves, w.n_leaves);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return e;
  std::swap(w.pend, w.next);
  std::swap(w.cap_pend, w.cap_next);
  w.n_leaves += n - n_split;
  w.n_pend = 4 * n_split;
  return hipSuccess;
}

hipError_t tree_balance(TreeWork& w, hipStream_t stream) {
  for (;;) {
    const int64_t n = w.n_leaves;
    if (n <= 0) return hipSuccess;
    if (n > (int64_t(1) << 26)) return hipErrorInvalidValue;  // 29 ancestors per leaf stay below 2^31
    // sorted leaves in tmp
    hipError_t e = grow(w.tmp, w.cap_tmp, size_t(n));
    if (e == hipSuccess) e = sort_keys(w, w.leaves, w.tmp, n, stream);
    // the internal boxes: every proper ancestor, sorted, duplicates kept (searches do not mind)
    if (e == hipSuccess) e = grow(w.flag, w.cap_flag, size_t(n));
    if (e == hipSuccess) e = grow(w.pos, w.cap_pos, size_t(n));
    int64_t n_anc = 0;
    if (e == hipSuccess) {
      hipLaunchKernelGGL(level_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, stream, w.tmp, n, w.flag);
      e = exclusive_count(w, w.flag, w.pos, n, &n_anc, stream);
    }
    if (e == hipSuccess) e = grow(w.anc, w.cap_anc, size_t(2 * std::max<int64_t>(n_anc, 1)));
    if (e == hipSuccess && n_anc > 0) {
      hipLaunchKernelGGL(ancestors_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, stream, w.tmp, w.pos, n,
                         w.anc + n_anc);
      e = sort_keys(w, w.anc + n_anc, w.anc, n_anc, stream);
    }
    // flags of the leaves to split
    if (e == hipSuccess) {
      hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, stream, w.flag, n);
      hipLaunchKernelGGL(balance_check_kernel, dim3(blocks_for(8 * n)), dim3(kThreads), 0, stream, w.tmp, n, w.anc,
                         n_anc, w.flag);
      e = hipGetLastError();
    }
    int64_t n_flag = 0;
    if (e == hipSuccess) e = exclusive_count(w, w.flag, w.pos, n, &n_flag, stream);
    if (e != hipSuccess) return e;
    if (n_flag == 0) {  // balanced: sort by level, y, x into leaves
      hipLaunchKernelGGL(swap_xy_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, stream, w.tmp, n);
      e = sort_keys(w, w.tmp, w.leaves, n, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      return e;
    }
    const int64_t n_new = n + 3 * n_flag;
    if (size_t(n_new) > w.cap_leaves) {
      if (w.leaves) (void)hipFree(w.leaves);
      w.leaves = nullptr;
      w.cap_leaves = 0;
      e = grow(w.leaves, w.cap_leaves, size_t(2 * n_new));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(balance_split_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, stream, w.tmp, w.flag, w.pos, n,
                       n - n_flag, w.leaves);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    w.n_leaves = n_new;
  }
}

void tree_free(TreeWork& w) {
  for (void* p : {static_cast<void*>(w.pend), static_cast<void*>(w.next), static_cast<void*>(w.leaves),
                  static_cast<void*>(w.tmp), static_cast<void*>(w.anc), static_cast<void*>(w.tails),
                  static_cast<void*>(w.flag), static_cast<void*>(w.pos), w.scratch})
    if (p) (void)hipFree(p);
  w = TreeWork();
}

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
