// Adaptive quadtree construction on the GPU (Sec. 4.2.1, Alg. 2, the function-resolution
// criterion) and the 2:1 balance over edges and corners. The caller samples f at the nodes
// the builder hands out; the builder computes each box's Chebyshev tail on the GPU and splits
// the boxes whose tail exceeds eps * scale, one level per round; boxes above min_level are split
// without samples and boxes at max_level are leaves. The balance then splits any leaf that a
// leaf two or more levels finer touches, until none does (host; hash set of packed keys).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <unordered_set>
#include <vector>

#include "../../include/volpot.h"
#include "device.hpp"

using namespace vp;

namespace {
constexpr int kMaxTreeLevel = 29;
inline uint64_t tkey(int l, int64_t x, int64_t y) { return (uint64_t(l) << 58) | (uint64_t(x) << 29) | uint64_t(y); }
inline int tl(uint64_t k) { return int(k >> 58); }
inline int64_t tx(uint64_t k) { return int64_t((k >> 29) & ((1ull << 29) - 1)); }
inline int64_t ty(uint64_t k) { return int64_t(k & ((1ull << 29) - 1)); }
}  // namespace

struct volpot_tree_s {
  double tol = 0.0;
  int min_level = 0, max_level = 0, device = -1;
  TreeRule rule{};
  std::vector<uint64_t> pending, leaves;
  bool balanced = false;
  int64_t cap = 0;  // boxes the device buffers hold
  int64_t* d_keys = nullptr;
  double* d_tails = nullptr;
  std::vector<double> tails;
};

namespace {

struct TreeDevice {  // makes the builder's device current for the call
  int prev = -1;
  explicit TreeDevice(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (dev >= 0 && dev != prev) (void)hipSetDevice(dev);
  }
  ~TreeDevice() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

void free_tree(volpot_tree_s* t) {
  if (!t) return;
  if (t->d_keys) (void)hipFree(t->d_keys);
  if (t->d_tails) (void)hipFree(t->d_tails);
  delete t;
}

int ensure_capacity(volpot_tree_s* t, int64_t n) {
  if (n <= t->cap) return VOLPOT_OK;
  // the previous round's work on these buffers has completed: submit synchronised its stream
  if (t->d_keys) (void)hipFree(t->d_keys);
  if (t->d_tails) (void)hipFree(t->d_tails);
  t->d_keys = nullptr; t->d_tails = nullptr; t->cap = 0;
  const int64_t c = std::max<int64_t>(n, 1024);
  if (hipMalloc(&t->d_keys, size_t(c) * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&t->d_tails, size_t(c) * sizeof(double)) != hipSuccess)
    return VOLPOT_ERR_OOM;
  t->cap = c;
  return VOLPOT_OK;
}

void split_into(std::vector<uint64_t>& out, uint64_t k) {
  const int l = tl(k);
  const int64_t x = tx(k), y = ty(k);
  for (int b = 0; b < 2; ++b)
    for (int a = 0; a < 2; ++a) out.push_back(tkey(l + 1, 2 * x + a, 2 * y + b));
}

void balance(std::vector<uint64_t>& leaves) {
  std::unordered_set<uint64_t> L(leaves.begin(), leaves.end());
  bool changed = true;
  while (changed) {
    changed = false;
    std::vector<uint64_t> order(L.begin(), L.end());
    std::sort(order.begin(), order.end(), [](uint64_t a, uint64_t b) { return tl(a) > tl(b) || (tl(a) == tl(b) && a < b); });
    for (uint64_t k : order) {
      if (!L.count(k)) continue;
      const int l = tl(k);
      const int64_t n = int64_t(1) << l;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (!(dx || dy)) continue;
          int64_t cx = tx(k) + dx, cy = ty(k) + dy;
          if (cx < 0 || cy < 0 || cx >= n || cy >= n) continue;
          int cl = l;
          while (cl >= 0 && !L.count(tkey(cl, cx, cy))) { --cl; cx >>= 1; cy >>= 1; }
          if (cl >= 0 && cl <= l - 2) {
            const uint64_t c = tkey(cl, cx, cy);
            L.erase(c);
            std::vector<uint64_t> kids;
            split_into(kids, c);
            L.insert(kids.begin(), kids.end());
            changed = true;
          }
        }
    }
  }
  leaves.assign(L.begin(), L.end());
  std::sort(leaves.begin(), leaves.end(), [](uint64_t a, uint64_t b) {
    if (tl(a) != tl(b)) return tl(a) < tl(b);
    if (ty(a) != ty(b)) return ty(a) < ty(b);
    return tx(a) < tx(b);
  });
}

}  // namespace

extern "C" {

int volpot_tree_create(int32_t p, double eps, double scale, int32_t min_level, int32_t max_level, volpot_tree_t* out) {
  if (!out || !(eps > 0.0) || !(scale >= 0.0) || !std::isfinite(eps * scale) || min_level < 0 || max_level < min_level)
    return VOLPOT_ERR_ARG;
  if (p != 16 || max_level > kMaxTreeLevel) return VOLPOT_ERR_UNSUPPORTED;
  auto* t = new (std::nothrow) volpot_tree_s();
  if (!t) return VOLPOT_ERR_OOM;
  t->tol = eps * scale;
  t->min_level = min_level;
  t->max_level = max_level;
  double w[16];
  volpot_nodes(16, t->rule.t, w);
  for (int m = 0; m < 16; ++m)
    for (int i = 0; i < 16; ++i)
      t->rule.D[m * 16 + i] = (m == 0 ? 1.0 : 2.0) / 16.0 * std::cos(m * std::acos(t->rule.t[i]));
  // boxes above min_level are split without samples
  if (min_level > 12) { delete t; return VOLPOT_ERR_UNSUPPORTED; }  // 4^12 first-round boxes at most
  const int64_t n = int64_t(1) << min_level;
  for (int64_t y = 0; y < n; ++y)
    for (int64_t x = 0; x < n; ++x) t->pending.push_back(tkey(min_level, x, y));
  *out = t;
  return VOLPOT_OK;
}

int volpot_tree_pending(volpot_tree_t t, int64_t* n) {
  if (!t || !n) return VOLPOT_ERR_ARG;
  *n = int64_t(t->pending.size());
  return VOLPOT_OK;
}

int volpot_tree_nodes(volpot_tree_t t, double* nodes_dev, void* hip_stream) {
  if (!t || (!t->pending.empty() && !nodes_dev)) return VOLPOT_ERR_ARG;
  if (t->pending.empty()) return VOLPOT_OK;
  if (t->device < 0 && hipGetDevice(&t->device) != hipSuccess) return VOLPOT_ERR_HIP;  // the first device call
  TreeDevice dg(t->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const int64_t n = int64_t(t->pending.size());
  int rc = ensure_capacity(t, n);
  if (rc != VOLPOT_OK) return rc;
  if (hipMemcpyAsync(t->d_keys, t->pending.data(), t->pending.size() * sizeof(int64_t), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      launch_tree_nodes(t->d_keys, n, t->rule, nodes_dev, s) != hipSuccess)
    return VOLPOT_ERR_HIP;
  return VOLPOT_OK;
}

int volpot_tree_submit(volpot_tree_t t, const double* values_dev, void* hip_stream) {
  if (!t || (!t->pending.empty() && !values_dev)) return VOLPOT_ERR_ARG;
  if (t->pending.empty()) return VOLPOT_OK;
  if (t->device < 0 && hipGetDevice(&t->device) != hipSuccess) return VOLPOT_ERR_HIP;
  TreeDevice dg(t->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  int rc = ensure_capacity(t, int64_t(t->pending.size()));
  if (rc != VOLPOT_OK) return rc;
  const int64_t n = int64_t(t->pending.size());
  t->tails.resize(size_t(n));
  if (launch_tree_tail(values_dev, n, t->rule, t->d_tails, s) != hipSuccess ||
      hipMemcpyAsync(t->tails.data(), t->d_tails, size_t(n) * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return VOLPOT_ERR_HIP;
  std::vector<uint64_t> next;
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t k = t->pending[size_t(i)];
    // a non-finite sample gives a non-finite tail, which does not pass the test
    if (tl(k) < t->max_level && !(t->tails[size_t(i)] <= t->tol)) split_into(next, k);
    else t->leaves.push_back(k);
  }
  t->pending.swap(next);
  t->balanced = false;
  return VOLPOT_OK;
}

int volpot_tree_leaves(volpot_tree_t t, int64_t* n, double* centres, int32_t* levels) {
  if (!t || !n) return VOLPOT_ERR_ARG;
  if (!t->pending.empty()) return VOLPOT_ERR_STATE;
  if (!t->balanced) {
    try {
      balance(t->leaves);
    } catch (const std::bad_alloc&) {
      return VOLPOT_ERR_OOM;
    }
    t->balanced = true;
  }
  *n = int64_t(t->leaves.size());
  for (size_t i = 0; i < t->leaves.size(); ++i) {
    const uint64_t k = t->leaves[i];
    const double s = std::ldexp(1.0, -tl(k));
    if (centres) {
      centres[2 * i] = -1.0 + (2.0 * double(tx(k)) + 1.0) * s;
      centres[2 * i + 1] = -1.0 + (2.0 * double(ty(k)) + 1.0) * s;
    }
    if (levels) levels[i] = tl(k);
  }
  return VOLPOT_OK;
}

void volpot_tree_destroy(volpot_tree_t t) {
  if (!t) return;
  TreeDevice dg(t->device);
  free_tree(t);
}

}  // extern "C"
