// Adaptive quadtree construction on the GPU (Sec. 4.2.1, Alg. 2, the function-resolution
// criterion) and the 2:1 balance over edges and corners. The caller samples f at the nodes
// the builder hands out; the builder computes each box's Chebyshev tail on the GPU and splits
// the boxes whose tail exceeds eps * scale, one level per round; boxes above min_level are split
// without samples and boxes at max_level are leaves. The pending boxes, the split decisions, the
// leaves and the balance all live on the device (tree.hip); the host holds only counts, and the
// balanced leaves once they are asked for.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/volpot.h"
#include "device.hpp"

using namespace vp;

namespace {
constexpr int kMaxTreeLevel = 29;
inline uint64_t tkey(int l, int64_t x, int64_t y) { return (uint64_t(l) << 58) | (uint64_t(x) << 29) | uint64_t(y); }
}  // namespace

struct volpot_tree_s {
  double tol = 0.0;
  int min_level = 0, max_level = 0, device = -1;
  TreeRule rule{};
  std::vector<uint64_t> first;  // the first round's boxes, until they are uploaded
  bool uploaded = false, balanced = false;
  TreeWork w;
  std::vector<uint64_t> leaves;  // balanced leaves (level, iy, ix keys), once read back
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

// the first device call of a builder: its device, and the first round's keys on it
int ensure_uploaded(volpot_tree_s* t, hipStream_t s) {
  if (t->uploaded) return VOLPOT_OK;
  const hipError_t e = tree_upload_pending(t->w, t->first.data(), int64_t(t->first.size()), s);
  if (e == hipErrorOutOfMemory) return VOLPOT_ERR_OOM;
  if (e != hipSuccess) return VOLPOT_ERR_HIP;
  std::vector<uint64_t>().swap(t->first);
  t->uploaded = true;
  return VOLPOT_OK;
}

int64_t pending_of(const volpot_tree_s* t) { return t->uploaded ? t->w.n_pend : int64_t(t->first.size()); }

}  // namespace

extern "C" {

int volpot_tree_create(int32_t p, double eps, double scale, int32_t min_level, int32_t max_level, volpot_tree_t* out) {
  if (!out || !(eps > 0.0) || !(scale >= 0.0) || !std::isfinite(eps * scale) || min_level < 0 || max_level < min_level)
    return VOLPOT_ERR_ARG;
  if (p != 16 || max_level > kMaxTreeLevel) return VOLPOT_ERR_UNSUPPORTED;
  // boxes above min_level are split without samples
  if (min_level > 12) return VOLPOT_ERR_UNSUPPORTED;  // 4^12 first-round boxes at most
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
  const int64_t n = int64_t(1) << min_level;
  try {
    t->first.reserve(size_t(n * n));
    for (int64_t y = 0; y < n; ++y)
      for (int64_t x = 0; x < n; ++x) t->first.push_back(tkey(min_level, x, y));
  } catch (const std::bad_alloc&) {
    delete t;
    return VOLPOT_ERR_OOM;
  }
  *out = t;
  return VOLPOT_OK;
}

int volpot_tree_pending(volpot_tree_t t, int64_t* n) {
  if (!t || !n) return VOLPOT_ERR_ARG;
  *n = pending_of(t);
  return VOLPOT_OK;
}

int volpot_tree_nodes(volpot_tree_t t, double* nodes_dev, void* hip_stream) {
  if (!t || (pending_of(t) > 0 && !nodes_dev)) return VOLPOT_ERR_ARG;
  if (pending_of(t) == 0) return VOLPOT_OK;
  if (t->device < 0 && hipGetDevice(&t->device) != hipSuccess) return VOLPOT_ERR_HIP;  // the first device call
  TreeDevice dg(t->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  int rc = ensure_uploaded(t, s);
  if (rc != VOLPOT_OK) return rc;
  if (launch_tree_nodes(reinterpret_cast<const int64_t*>(t->w.pend), t->w.n_pend, t->rule, nodes_dev, s) != hipSuccess)
    return VOLPOT_ERR_HIP;
  return VOLPOT_OK;
}

int volpot_tree_submit(volpot_tree_t t, const double* values_dev, void* hip_stream) {
  if (!t || (pending_of(t) > 0 && !values_dev)) return VOLPOT_ERR_ARG;
  if (pending_of(t) == 0) return VOLPOT_OK;
  if (t->device < 0 && hipGetDevice(&t->device) != hipSuccess) return VOLPOT_ERR_HIP;
  TreeDevice dg(t->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  int rc = ensure_uploaded(t, s);
  if (rc != VOLPOT_OK) return rc;
  const hipError_t e = tree_round(t->w, values_dev, t->rule, t->tol, t->max_level, s);
  if (e == hipErrorOutOfMemory) return VOLPOT_ERR_OOM;
  if (e != hipSuccess) return VOLPOT_ERR_HIP;
  t->balanced = false;
  return VOLPOT_OK;
}

int volpot_tree_leaves(volpot_tree_t t, int64_t* n, double* centres, int32_t* levels) {
  if (!t || !n) return VOLPOT_ERR_ARG;
  if (pending_of(t) > 0) return VOLPOT_ERR_STATE;
  if (!t->balanced) {
    if (t->device < 0 && hipGetDevice(&t->device) != hipSuccess) return VOLPOT_ERR_HIP;
    TreeDevice dg(t->device);
    hipError_t e = tree_balance(t->w, nullptr);
    try {
      if (e == hipSuccess) t->leaves.resize(size_t(t->w.n_leaves));
    } catch (const std::bad_alloc&) {
      return VOLPOT_ERR_OOM;
    }
    if (e == hipSuccess && t->w.n_leaves > 0)
      e = hipMemcpy(t->leaves.data(), t->w.leaves, size_t(t->w.n_leaves) * sizeof(uint64_t), hipMemcpyDeviceToHost);
    if (e == hipErrorOutOfMemory) return VOLPOT_ERR_OOM;
    if (e != hipSuccess) return VOLPOT_ERR_HIP;
    t->balanced = true;
  }
  *n = int64_t(t->leaves.size());
  for (size_t i = 0; i < t->leaves.size(); ++i) {
    const uint64_t k = t->leaves[i];  // level << 58 | iy << 29 | ix
    const int l = int(k >> 58);
    const double s = std::ldexp(1.0, -l);
    const double ix = double(k & ((1ull << 29) - 1)), iy = double((k >> 29) & ((1ull << 29) - 1));
    if (centres) {
      centres[2 * i] = -1.0 + (2.0 * ix + 1.0) * s;
      centres[2 * i + 1] = -1.0 + (2.0 * iy + 1.0) * s;
    }
    if (levels) levels[i] = l;
  }
  return VOLPOT_OK;
}

void volpot_tree_destroy(volpot_tree_t t) {
  if (!t) return;
  TreeDevice dg(t->device);
  tree_free(t->w);
  delete t;
}

}  // extern "C"
