// Host plan: tree validation, integer box keys, adaptive-FMM interaction lists, and the
// stage/tile schedules consumed by the grouped-relation kernels (plan.hpp).
//
// Lists (geometric definitions of the adaptive FMM; the box code of Sec. 4.2 is one):
//   U(a)  leaves adjacent to leaf a, a included   -> near tables (33 relations)
//   V(b)  same-level children of the colleagues of b's parent, not adjacent to b -> M2L
//   W(a)  children of leaf a's colleagues, not adjacent to a                    -> M2T
//   X(b)  leaves c with b in W(c)                                               -> S2L
// 2:1 balance over edges and corners (Sec. 4.2.1) bounds adjacent levels to l-1..l+1, which
// is what makes the 33 near relations and the 20 W / X offsets exhaustive.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <exception>
#include <functional>
#include <map>
#include <stdexcept>
#include <thread>

#include "../../include/volpot.h"
#include "plan.hpp"

namespace vp {

// ---------------------------------------------------------------- offsets
static std::vector<Offset> make_near() {
  std::vector<Offset> v;
  v.push_back({0, 0, 1});
  for (int dy = -2; dy <= 2; dy += 2)
    for (int dx = -2; dx <= 2; dx += 2)
      if (dx || dy) v.push_back({double(dx), double(dy), 1.0});
  for (double a : {-1.5, -0.5, 0.5, 1.5})
    for (double b : {-1.5, -0.5, 0.5, 1.5})
      if (std::fabs(a) == 1.5 || std::fabs(b) == 1.5) v.push_back({a, b, 0.5});
  for (double a : {-3.0, -1.0, 1.0, 3.0})
    for (double b : {-3.0, -1.0, 1.0, 3.0})
      if (std::fabs(a) == 3.0 || std::fabs(b) == 3.0) v.push_back({a, b, 2.0});
  return v;
}
static std::vector<Offset> make_v() {
  std::vector<Offset> v;
  for (int j = -3; j <= 3; ++j)
    for (int i = -3; i <= 3; ++i)
      if (std::max(std::abs(i), std::abs(j)) >= 2) v.push_back({2.0 * i, 2.0 * j, 1.0});
  return v;
}
static std::vector<Offset> make_w() {
  std::vector<Offset> v;
  for (double a : {-2.5, -1.5, -0.5, 0.5, 1.5, 2.5})
    for (double b : {-2.5, -1.5, -0.5, 0.5, 1.5, 2.5})
      if (std::fabs(a) == 2.5 || std::fabs(b) == 2.5) v.push_back({a, b, 0.5});
  return v;
}
static std::vector<Offset> make_x() {
  std::vector<Offset> v;
  for (double a : {-5.0, -3.0, -1.0, 1.0, 3.0, 5.0})
    for (double b : {-5.0, -3.0, -1.0, 1.0, 3.0, 5.0})
      if (std::fabs(a) == 5.0 || std::fabs(b) == 5.0) v.push_back({a, b, 2.0});
  return v;
}
const std::vector<Offset>& near_offsets() { static const auto v = make_near(); return v; }
const std::vector<Offset>& v_offsets() { static const auto v = make_v(); return v; }
const std::vector<Offset>& w_offsets() { static const auto v = make_w(); return v; }
const std::vector<Offset>& x_offsets() { static const auto v = make_x(); return v; }

int find_offset(const std::vector<Offset>& v, double dx, double dy, double rho) {
  for (size_t i = 0; i < v.size(); ++i)
    if (std::fabs(v[i].dx - dx) < 1e-9 && std::fabs(v[i].dy - dy) < 1e-9 && std::fabs(v[i].rho - rho) < 1e-12)
      return int(i);
  return -1;
}

// ---------------------------------------------------------------- keys
static inline uint64_t pack(int l, int64_t x, int64_t y) {
  return (uint64_t(l) << 58) | (uint64_t(x) << 29) | uint64_t(y);
}
static inline int key_l(uint64_t k) { return int(k >> 58); }
static inline int64_t key_x(uint64_t k) { return int64_t((k >> 29) & ((1ull << 29) - 1)); }
static inline int64_t key_y(uint64_t k) { return int64_t(k & ((1ull << 29) - 1)); }
static inline uint64_t parent_key(uint64_t k) {
  return pack(key_l(k) - 1, key_x(k) >> 1, key_y(k) >> 1);
}
static inline uint64_t child_key(uint64_t k, int q) {
  return pack(key_l(k) + 1, 2 * key_x(k) + (q & 1), 2 * key_y(k) + (q >> 1));
}
static inline bool touch(uint64_t a, uint64_t b) {
  int la = key_l(a), lb = key_l(b), L = std::max(la, lb);
  int64_t ax0 = key_x(a) << (L - la), ax1 = (key_x(a) + 1) << (L - la);
  int64_t bx0 = key_x(b) << (L - lb), bx1 = (key_x(b) + 1) << (L - lb);
  int64_t ay0 = key_y(a) << (L - la), ay1 = (key_y(a) + 1) << (L - la);
  int64_t by0 = key_y(b) << (L - lb), by1 = (key_y(b) + 1) << (L - lb);
  return std::max(ax0, bx0) <= std::min(ax1, bx1) && std::max(ay0, by0) <= std::min(ay1, by1);
}
static inline uint64_t morton(int64_t x, int64_t y) {
  uint64_t m = 0;
  for (int b = 0; b < 29; ++b) m |= ((uint64_t(x) >> b) & 1) << (2 * b) | ((uint64_t(y) >> b) & 1) << (2 * b + 1);
  return m;
}
static inline double centre_of(int64_t i, int l) { return -1.0 + (2.0 * double(i) + 1.0) * std::ldexp(1.0, -l); }

struct TreeBoxes {
  std::unordered_map<uint64_t, int64_t> leaf;  // key -> caller leaf index
  std::unordered_map<uint64_t, int32_t> box;   // key -> global box id (filled later)
};

// Validate one tree; fill the leaf map and the set of boxes (ids assigned later).
static int validate_tree(int64_t off, int64_t n, const double* centres, const int32_t* levels,
                         TreeBoxes& tb, std::vector<uint64_t>& keys, int64_t* bad) {
  keys.resize(n);
  int L = 0;
  for (int64_t i = 0; i < n; ++i) {
    int l = levels[off + i];
    if (l < 0 || l > kMaxLevel) { if (bad) *bad = off + i; return l < 0 ? VOLPOT_ERR_TREE : VOLPOT_ERR_UNSUPPORTED; }
    double s = std::ldexp(1.0, -l);
    double fx = (centres[2 * (off + i)] + 1.0) / (2.0 * s) - 0.5;
    double fy = (centres[2 * (off + i) + 1] + 1.0) / (2.0 * s) - 0.5;
    double rx = std::nearbyint(fx), ry = std::nearbyint(fy);
    double lim = std::ldexp(1.0, l);
    if (!(std::fabs(fx - rx) < 1e-6) || !(std::fabs(fy - ry) < 1e-6) || !(rx >= 0 && rx < lim) || !(ry >= 0 && ry < lim)) {
      if (bad) *bad = off + i;
      return VOLPOT_ERR_TREE;
    }
    keys[i] = pack(l, int64_t(rx), int64_t(ry));
    if (!tb.leaf.emplace(keys[i], off + i).second) { if (bad) *bad = off + i; return VOLPOT_ERR_TREE; }
    L = std::max(L, l);
  }
  unsigned __int128 area = 0;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t k = keys[i];
    area += (unsigned __int128)1 << (2 * (L - key_l(k)));
    while (key_l(k) > 0) {
      k = parent_key(k);
      if (tb.leaf.count(k)) { if (bad) *bad = off + i; return VOLPOT_ERR_TREE; }
      if (!tb.box.emplace(k, -1).second) break;  // ancestors above are present already
    }
  }
  if (area != ((unsigned __int128)1 << (2 * L))) { if (bad) *bad = off; return VOLPOT_ERR_TREE; }
  for (int64_t i = 0; i < n; ++i) tb.box.emplace(keys[i], -1);
  // 2:1 balance over edges and corners
  for (int64_t i = 0; i < n; ++i) {
    uint64_t k = keys[i];
    int l = key_l(k);
    int64_t nmax = int64_t(1) << l;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (!dx && !dy) continue;
        int64_t qx = key_x(k) + dx, qy = key_y(k) + dy;
        if (qx < 0 || qy < 0 || qx >= nmax || qy >= nmax) continue;
        uint64_t q = pack(l, qx, qy);
        if (tb.box.count(q)) {
          if (tb.leaf.count(q)) continue;
          for (int c = 0; c < 4; ++c) {
            uint64_t ch = child_key(q, c);
            if (touch(ch, k) && !tb.leaf.count(ch)) { if (bad) *bad = off + i; return VOLPOT_ERR_UNBALANCED; }
          }
        } else {
          uint64_t c = q;
          while (!tb.leaf.count(c)) c = parent_key(c);
          if (key_l(c) < l - 1) { if (bad) *bad = off + i; return VOLPOT_ERR_UNBALANCED; }
        }
      }
  }
  return VOLPOT_OK;
}

int validate_forest(int32_t n_trees, const int64_t* offsets, const double* centres, const int32_t* levels,
                    int64_t* bad) {
  for (int t = 0; t < n_trees; ++t) {
    int64_t n = offsets[t + 1] - offsets[t];
    if (n <= 0) { if (bad) *bad = offsets[t]; return VOLPOT_ERR_TREE; }
    TreeBoxes tb;
    std::vector<uint64_t> keys;
    int rc = validate_tree(offsets[t], n, centres, levels, tb, keys, bad);
    if (rc != VOLPOT_OK) return rc;
  }
  return VOLPOT_OK;
}

struct Entry { int32_t rel; int8_t fam; int32_t src; };
struct R1 { int8_t fam; int32_t idx; double coef; };

// Interaction lists in compressed rows: row i holds (relation, index) pairs.
using RelIdx = std::pair<int32_t, int32_t>;
struct Lists {
  std::vector<int64_t> ptr{0};
  std::vector<RelIdx> e;
  struct Row {
    const RelIdx *b, *e;
    const RelIdx* begin() const { return b; }
    const RelIdx* end() const { return e; }
    size_t size() const { return size_t(e - b); }
    bool empty() const { return b == e; }
  };
  Row operator[](size_t i) const { return {e.data() + ptr[i], e.data() + ptr[i + 1]}; }
  size_t rows() const { return ptr.size() - 1; }
};

// f(i) for i in [0, n) on up to 16 host threads, in chunks of `grain`; the first exception
// thrown by any call is rethrown.
template <class F>
static void par_for(int64_t n, const F& f, int64_t grain = 2048) {
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const unsigned nt = unsigned(std::min<int64_t>(hw, (n + grain - 1) / grain));
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next(0);
  std::exception_ptr err;
  std::atomic<bool> failed(false);
  auto work = [&]() {
    try {
      for (int64_t i0; !failed.load() && (i0 = next.fetch_add(grain)) < n;)
        for (int64_t i = i0; i < std::min(n, i0 + grain); ++i) f(i);
    } catch (...) {
      if (!failed.exchange(true)) err = std::current_exception();
    }
  };
  std::vector<std::thread> pool;
  for (unsigned t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
  if (err) std::rethrow_exception(err);
}

// Rows of `n_out` lists for items [0, n): row(i, outs) appends item i's entries to outs[k] for
// list k. Contiguous chunks of items are filled concurrently and concatenated in item order.
template <class F>
static void build_rows(int64_t n, std::vector<Lists*> lists, const F& row) {
  const int64_t chunk = 4096, nc = (n + chunk - 1) / chunk;
  const size_t K = lists.size();
  auto ent = std::vector<std::vector<std::vector<RelIdx>>>(static_cast<size_t>(nc), std::vector<std::vector<RelIdx>>(K));
  auto cnt = std::vector<std::vector<std::vector<int64_t>>>(static_cast<size_t>(nc), std::vector<std::vector<int64_t>>(K));
  par_for(nc, [&](int64_t c) {
    std::vector<std::vector<RelIdx>*> outs(K);
    for (size_t k = 0; k < K; ++k) outs[k] = &ent[size_t(c)][k];
    for (int64_t i = c * chunk; i < std::min(n, (c + 1) * chunk); ++i) {
      std::vector<size_t> before(K);
      for (size_t k = 0; k < K; ++k) before[k] = outs[k]->size();
      row(i, outs);
      for (size_t k = 0; k < K; ++k) cnt[size_t(c)][k].push_back(int64_t(outs[k]->size() - before[k]));
    }
  }, 1);
  for (size_t k = 0; k < K; ++k) {
    Lists& L = *lists[k];
    L.ptr.assign(1, 0);
    L.ptr.reserve(size_t(n) + 1);
    size_t total = 0;
    for (int64_t c = 0; c < nc; ++c) total += ent[size_t(c)][k].size();
    L.e.clear();
    L.e.reserve(total);
    for (int64_t c = 0; c < nc; ++c) {
      for (int64_t m : cnt[size_t(c)][k]) L.ptr.push_back(L.ptr.back() + m);
      L.e.insert(L.e.end(), ent[size_t(c)][k].begin(), ent[size_t(c)][k].end());
    }
  }
}

// The transpose of list A (rows over [0, n_rows_a)) into rows over [0, n_rows_t): row t holds
// (relation, a) for every entry (relation, t) of row a, in increasing a.
static Lists transpose_rows(const Lists& A, int64_t n_rows_t) {
  Lists T;
  T.ptr.assign(size_t(n_rows_t) + 1, 0);
  for (const RelIdx& x : A.e) T.ptr[size_t(x.second) + 1]++;
  for (int64_t t = 0; t < n_rows_t; ++t) T.ptr[size_t(t) + 1] += T.ptr[size_t(t)];
  T.e.resize(A.e.size());
  std::vector<int64_t> pos(T.ptr.begin(), T.ptr.end() - 1);
  for (size_t a = 0; a < A.rows(); ++a)
    for (const RelIdx& x : A[a]) T.e[size_t(pos[size_t(x.second)]++)] = {x.first, int32_t(a)};
  return T;
}

static void make_tiles_ordered(Stage& st, const std::vector<int32_t>& targets,
                               const std::vector<std::vector<Entry>>& entries,
                               const std::vector<std::vector<R1>>& r1, const std::vector<int32_t>& ord,
                               const Matrices& mats);

// Targets grouped by the set of relations they take, classes in lexicographic order of their
// sorted relation lists (neighbouring classes share most relations), the given order within a
// class. Every segment of a tile costs the same whatever its occupancy, so a tile should hold
// targets that take the same relations: in adaptive trees, targets near refinement boundaries
// take neighbours in many patterns. Classes are found by hashing each target's sorted keys
// (equal hashes are compared key by key), so that the cost is linear in the entries.
static void make_tiles(Stage& st, const std::vector<int32_t>& targets, const std::vector<std::vector<Entry>>& entries,
                       const std::vector<std::vector<R1>>& r1, const Matrices& mats) {
  const size_t n = targets.size();
  std::vector<int64_t> kp(n + 1, 0);  // sorted keys of target i: keys[kp[i] .. kp[i + 1])
  for (size_t i = 0; i < n; ++i) kp[i + 1] = kp[i] + int64_t(entries[i].size());
  std::vector<int32_t> keys(static_cast<size_t>(kp[n]));
  std::vector<std::pair<uint64_t, int32_t>> hs(n);
  for (size_t i = 0; i < n; ++i) {
    int32_t* k = keys.data() + kp[i];
    for (size_t e = 0; e < entries[i].size(); ++e) k[e] = entries[i][e].rel * 16 + entries[i][e].fam;
    std::sort(k, k + entries[i].size());
    uint64_t h = 1469598103934665603ull ^ uint64_t(entries[i].size());
    for (size_t e = 0; e < entries[i].size(); ++e) h = (h ^ uint64_t(uint32_t(k[e]))) * 1099511628211ull;
    hs[i] = {h, int32_t(i)};
  }
  auto same = [&](int32_t a, int32_t b) {
    return kp[a + 1] - kp[a] == kp[b + 1] - kp[b] &&
           std::equal(keys.begin() + kp[a], keys.begin() + kp[a + 1], keys.begin() + kp[b]);
  };
  auto less = [&](int32_t a, int32_t b) {
    return std::lexicographical_compare(keys.begin() + kp[a], keys.begin() + kp[a + 1], keys.begin() + kp[b],
                                        keys.begin() + kp[b + 1]);
  };
  std::sort(hs.begin(), hs.end());
  // class of each target; rep: one target of each class
  std::vector<int32_t> c(n), rep;
  for (size_t g = 0; g < n;) {
    size_t g1 = g;
    while (g1 < n && hs[g1].first == hs[g].first) ++g1;
    const size_t c0 = rep.size();
    for (size_t q = g; q < g1; ++q) {  // equal hashes: compare with the group's classes so far
      const int32_t i = hs[q].second;
      size_t r = c0;
      while (r < rep.size() && !same(rep[r], i)) ++r;
      if (r == rep.size()) rep.push_back(i);
      c[size_t(i)] = int32_t(r);
    }
    g = g1;
  }
  std::vector<int32_t> byk(rep.size()), rank(rep.size());
  for (size_t r = 0; r < rep.size(); ++r) byk[r] = int32_t(r);
  std::sort(byk.begin(), byk.end(), [&](int32_t x, int32_t y) { return less(rep[size_t(x)], rep[size_t(y)]); });
  for (size_t r = 0; r < byk.size(); ++r) rank[size_t(byk[r])] = int32_t(r);
  // stable counting sort by class rank
  std::vector<int64_t> start(rep.size() + 1, 0);
  for (size_t i = 0; i < n; ++i) start[size_t(rank[size_t(c[i])]) + 1]++;
  for (size_t r = 0; r < rep.size(); ++r) start[r + 1] += start[r];
  std::vector<int32_t> ord(n);
  for (size_t i = 0; i < n; ++i) ord[size_t(start[size_t(rank[size_t(c[i])])]++)] = int32_t(i);
  make_tiles_ordered(st, targets, entries, r1, ord, mats);
}

static void make_tiles_ordered(Stage& st, const std::vector<int32_t>& targets,
                               const std::vector<std::vector<Entry>>& entries,
                               const std::vector<std::vector<R1>>& r1, const std::vector<int32_t>& ord,
                               const Matrices& mats) {
  // slot ti of the tiled order holds target ord[ti]
  auto at = [&](size_t ti) { return size_t(ord[ti]); };
  const int NT = st.NT;
  st.n_tiles = int((targets.size() + NT - 1) / NT);
  st.tile_tgt.assign(size_t(st.n_tiles) * NT, -1);
  st.tile_seg_ptr.assign(st.n_tiles + 1, 0);
  st.r1_ptr.assign(size_t(st.n_tiles) * NT + 1, 0);
  st.seg_rel.clear(); st.seg_k.clear(); st.seg_fam.clear(); st.seg_src.clear();
  st.r1_idx.clear(); st.r1_fam.clear(); st.r1_coef.clear();
  st.flops = 0; st.n_pairs = 0; st.flops_issued = 0;
  std::vector<int32_t> seg_of(size_t(kNumRel) * 16, -1), used;
  // a factored stage multiplies every segment by its core (cx_rel) and reads 2 K reals per source
  const bool cx = st.cx_rel >= 0;
  auto table = [&](int rel) { return cx ? st.cx_rel : rel; };
  auto src_len = [&](int rel) { return cx ? 2 * mats.K[size_t(st.cx_rel)] : mats.K[size_t(rel)]; };
  if (cx && (st.cx_rel >= kNumRel || st.KC != mats.K[size_t(st.cx_rel)])) throw std::runtime_error("bad factored stage");
  for (int t = 0; t < st.n_tiles; ++t) {
    // segments keyed by (relation, source family), ordered by relation then family
    used.clear();
    for (int s = 0; s < NT; ++s) {
      size_t ti = size_t(t) * NT + s;
      if (ti >= targets.size()) break;
      st.tile_tgt[ti] = targets[at(ti)];
      for (const Entry& e : entries[at(ti)]) {
        if (e.rel < 0 || e.rel >= kNumRel || e.fam < 0 || e.fam >= 4) throw std::runtime_error("bad entry");
        const int32_t key = e.rel * 16 + e.fam;
        if (seg_of[size_t(key)] < 0) {
          seg_of[size_t(key)] = 0;
          used.push_back(key);
        }
      }
    }
    std::sort(used.begin(), used.end());
    for (int32_t key : used) {  // each (relation, family) of the tile, checked once
      const int rel = key / 16, fam = key % 16;
      // the kernel reads M x K of the relation's table and K values of each source
      if (cx && mats.w_in[size_t(rel)].empty()) throw std::runtime_error("relation has no factored form");
      if (mats.M[table(rel)] != st.M) throw std::runtime_error("relation rows differ from stage rows");
      if (st.fam[fam].stride < mats.koff[size_t(table(rel))] + src_len(rel))
        throw std::runtime_error("source shorter than relation");
      // the kernel walks K in full chunks of KC
      if (mats.K[table(rel)] % st.KC != 0) throw std::runtime_error("relation K not a multiple of the stage k-chunk");
    }
    for (int32_t key : used) {
      seg_of[size_t(key)] = int32_t(st.seg_rel.size());
      st.seg_rel.push_back(key / 16);
      st.seg_k.push_back(mats.K[table(key / 16)]);
      st.seg_fam.push_back(int8_t(key % 16));
      st.flops_issued += 2.0 * st.M * mats.K[table(key / 16)] * NT * (cx ? 2 : 1);
    }
    st.seg_src.resize(st.seg_rel.size() * NT, -1);
    for (int s = 0; s < NT; ++s) {
      size_t ti = size_t(t) * NT + s;
      if (ti >= targets.size()) break;
      for (const Entry& e : entries[at(ti)]) {
        int32_t& slot = st.seg_src[size_t(seg_of[size_t(e.rel * 16 + e.fam)]) * NT + s];
        if (slot != -1) throw std::runtime_error("duplicate relation for one target");
        slot = e.src;
        // factored: the core on both parts, then the two complex diagonals (6 and 8 flops a term)
        st.flops += cx ? 4.0 * mats.nnz[size_t(st.cx_rel)] + 14.0 * mats.K[size_t(st.cx_rel)] : 2.0 * mats.nnz[e.rel];
        st.n_pairs += 1;
      }
    }
    for (int32_t key : used) seg_of[size_t(key)] = -1;
    st.tile_seg_ptr[t + 1] = int32_t(st.seg_rel.size());
  }
  for (size_t ti = 0; ti < st.tile_tgt.size(); ++ti) {
    if (ti < targets.size())
      for (const R1& e : r1[at(ti)]) {
        st.r1_idx.push_back(e.idx);
        st.r1_fam.push_back(e.fam);
        st.r1_coef.push_back(e.coef);
        st.flops += st.r1_all_rows ? 2.0 * st.M : 2.0;
      }
    st.r1_ptr[ti + 1] = int32_t(st.r1_idx.size());
  }
}

// Launch order and stream flags. Built order: [S2M] [M2M chain] [FARV] [FARX] [L2L chain]
// [NEARC NEARC48] [NEAR or NEAR_A NEAR_B] [LOCT] (adjoint: [AL2T] [AL2L chain] [AFARV] [AFARW]
// [AM2M chain] [ANEARC...] [ANEAR...] [ALOCT]). Launch order of the dense near field:
//   S2M, M2M chain (helper), NEAR_A, FARV (join), FARX + L2L chain (helper), NEAR_B, LOCT (join)
// so that, with the overlap option, each latency-bound chain runs beside half of the near
// field, which does not depend on the far field. The low-rank near field, folded with the leaf
// stage into one stage that needs the far field, puts its pair stages there instead:
//   S2M, M2M chain (helper), NEARC, FARV (join), FARX, L2L chain (helper), NEARC48, NEAR+LOCT (join)
// Without overlap everything runs in this order on one stream, which is also a valid order. A
// layer plan has P2M in S2M's place, P2L in FARX's, and its direct sum P2P, which adds onto
// LOCT's output, last.
static void arrange_stages(std::vector<Stage>& v, bool adjoint) {
  const int k_up = adjoint ? K_AUP : K_UP, k_down = adjoint ? K_ADOWN : K_DOWN;
  const int k_near = adjoint ? K_ANEAR : K_NEAR, k_loct = adjoint ? K_ALOCT : K_LOCT;
  std::vector<Stage> head, up_chain, far, down_chain, pre, near, tail;
  for (Stage& s : v) {
    s.helper = s.join_before = s.fork_before = s.concurrent = 0;
    if (s.pre_near) pre.push_back(std::move(s));                            // NEARC / ANEARC
    else if (s.after_far) tail.push_back(std::move(s));                     // NEAR+LOCT / ANEAR+ALOCT
    else if (s.kind == k_up && s.level < 0) head.push_back(std::move(s));   // S2M / AL2T
    else if (s.kind == k_up) up_chain.push_back(std::move(s));              // M2M[l] / AL2L[l]
    else if (s.kind == k_down && s.level < 0) far.push_back(std::move(s));  // FARV, FARX / AFARV, AFARW
    else if (s.kind == k_down) down_chain.push_back(std::move(s));          // L2L[l] / AM2M[l]
    else if (s.kind == k_near) near.push_back(std::move(s));
    else if (s.kind == k_loct) tail.push_back(std::move(s));
    else throw std::runtime_error("unexpected stage kind");
  }
  v.clear();
  auto chain = [&](std::vector<Stage>& c) {
    for (size_t i = 0; i < c.size(); ++i) {
      c[i].helper = 1;
      c[i].fork_before = i == 0;
      v.push_back(std::move(c[i]));
    }
  };
  auto put_near = [&](size_t i) {
    if (i < near.size()) {
      near[i].concurrent = 1;
      v.push_back(std::move(near[i]));
    }
  };
  // layer plans: the direct sum (P2P) adds onto LOCT's output, so it runs last
  std::vector<Stage> last;
  if (near.size() == 1 && near[0].custom == C_P2P) last.push_back(std::move(near[0])), near.clear();
  const bool folded = near.empty() && !tail.empty() && tail[0].after_far;
  auto put_pre = [&](size_t i0, size_t i1) {  // the low-rank near field's pair stages [i0, i1)
    for (size_t i = i0; i < std::min(i1, pre.size()); ++i) {
      pre[i].concurrent = 1;
      v.push_back(std::move(pre[i]));
    }
  };
  for (Stage& s : head) v.push_back(std::move(s));
  chain(up_chain);
  put_pre(0, folded ? 1 : pre.size());
  put_near(0);
  // M2L (FARV / AFARV) on the caller's stream. The S2L / M2T^T stage (FARX / AFARW), which only
  // the downward chain reads, opens that chain on the helper stream beside the dense near
  // field's second half; beside the folded near field's second pair stage it stays on the
  // caller's stream (it is as large as the pair stage)
  std::vector<Stage> down;
  for (size_t i = 0; i < far.size(); ++i) {
    if (i == 0) far[i].join_before = 1;
    if (i == 0 || folded) v.push_back(std::move(far[i]));
    else down.push_back(std::move(far[i]));
  }
  for (Stage& s : down_chain) down.push_back(std::move(s));
  chain(down);
  put_pre(1, pre.size());
  put_near(1);
  for (size_t i = 0; i < tail.size(); ++i) {
    tail[i].join_before = i == 0;
    v.push_back(std::move(tail[i]));
  }
  for (Stage& s : last) v.push_back(std::move(s));
}

void build_schedule(Stage& st, int max_blocks, int min_units, int tile_cost) {
  const int T = st.n_tiles;
  st.pieces.clear();
  st.blk_ptr.assign(1, 0);
  st.n_blocks = 0;
  st.n_slots = 0;
  if (T <= 0) return;
  auto chunks = [&](int32_t seg) { return int64_t(st.seg_k[size_t(seg)] / st.KC); };
  // Work units: a tile's k-chunks, then tile_cost more for its fixed cost (index loads, rank-one
  // terms, the output pass), which only the block that ends the tile pays. A tile without
  // segments still has one unit.
  std::vector<int64_t> tu(T + 1, 0), tc(T, 0);  // first unit, chunk units of each tile
  for (int t = 0; t < T; ++t) {
    int64_t n = 0;
    for (int32_t g = st.tile_seg_ptr[t]; g < st.tile_seg_ptr[t + 1]; ++g) n += chunks(g);
    tc[t] = std::max<int64_t>(n, 1);
    tu[t + 1] = tu[t] + tc[t] + std::max(0, tile_cost);
  }
  const int64_t U = tu[T];
  // min_units < 0: one block per tile, no tile cut
  const bool whole = min_units < 0;
  const int64_t mu = std::max(1, min_units);
  const int64_t G = whole ? T : std::max<int64_t>(1, std::min<int64_t>(std::max(1, max_blocks), (U + mu - 1) / mu));
  // first unit of block b; a boundary inside a tile's fixed-cost units moves to the tile's end
  auto first = [&](int64_t b) {
    if (whole) return tu[b];
    const int64_t u = b * U / G;
    const int64_t t = std::upper_bound(tu.begin(), tu.end(), u) - tu.begin() - 1;
    return (t < T && u - tu[size_t(t)] >= tc[size_t(t)]) ? tu[size_t(t) + 1] : u;
  };
  // pass 1: pieces per tile
  std::vector<int32_t> npc(T, 0);
  for (int64_t b = 0, t = 0; b < G; ++b)
    for (int64_t u = first(b), ue = first(b + 1); u < ue;) {
      while (tu[t + 1] <= u) ++t;
      npc[t]++;
      u = std::min(ue, tu[t + 1]);
    }
  std::vector<int32_t> slot0(T, -1), seen(T, 0);
  for (int t = 0; t < T; ++t)
    if (npc[t] > 1) { slot0[t] = st.n_slots; st.n_slots += npc[t]; }
  // pass 2: the pieces, block by block
  for (int64_t b = 0, t = 0; b < G; ++b) {
    for (int64_t u = first(b), ue = first(b + 1); u < ue;) {
      while (tu[t + 1] <= u) ++t;
      const int64_t end = std::min(ue, tu[t + 1]);
      Piece pc{};
      pc.tile = int32_t(t);
      pc.n_pieces = npc[t];
      pc.slot0 = slot0[t];
      pc.slot = npc[t] > 1 ? slot0[t] + seen[t] : -1;
      seen[t]++;
      const int32_t g0 = st.tile_seg_ptr[t], g1 = st.tile_seg_ptr[t + 1];
      pc.seg = g0;
      pc.k0 = 0;
      pc.n_chunks = 0;
      if (g1 > g0) {
        int64_t o = u - tu[t];
        int32_t g = g0;
        while (o >= chunks(g)) { o -= chunks(g); ++g; }
        pc.seg = g;
        pc.k0 = int32_t(o * st.KC);
        pc.n_chunks = int32_t(std::min(end, tu[t] + tc[t]) - u);
      }
      st.pieces.push_back(pc);
      u = end;
    }
    st.blk_ptr.push_back(int32_t(st.pieces.size()));
  }
  st.n_blocks = int(G);
  // the kernel trusts these: every chunk of every tile exactly once, in order, within its tile
  std::vector<int64_t> got(T, 0);
  for (const Piece& pc : st.pieces) {
    if (pc.tile < 0 || pc.tile >= T) throw std::runtime_error("schedule: bad tile");
    if (pc.n_chunks > 0) {
      int64_t o = 0;
      for (int32_t g = st.tile_seg_ptr[pc.tile]; g < pc.seg; ++g) o += chunks(g);
      if (pc.seg < st.tile_seg_ptr[pc.tile] || pc.seg >= st.tile_seg_ptr[pc.tile + 1] || pc.k0 % st.KC)
        throw std::runtime_error("schedule: bad segment");
      if (o + pc.k0 / st.KC != got[pc.tile]) throw std::runtime_error("schedule: chunks out of order");
      if (got[pc.tile] + pc.n_chunks > tc[pc.tile]) throw std::runtime_error("schedule: overrun");
      got[pc.tile] += pc.n_chunks;
    } else {
      if (st.tile_seg_ptr[pc.tile + 1] != st.tile_seg_ptr[pc.tile] || pc.n_pieces != 1)
        throw std::runtime_error("schedule: empty piece");
    }
    if ((pc.slot < 0) != (pc.n_pieces == 1) || (pc.slot >= 0 && (pc.slot < pc.slot0 || pc.slot >= pc.slot0 + pc.n_pieces)))
      throw std::runtime_error("schedule: bad slot");
  }
  for (int t = 0; t < T; ++t)
    if (st.tile_seg_ptr[t + 1] > st.tile_seg_ptr[t] && got[t] != tc[t])
      throw std::runtime_error("schedule: tile not covered");
}

int build_plan(int32_t n_trees, const int64_t* offsets, const double* centres, const int32_t* levels,
               int tile_leaf, int tile_box, int overlap, Plan& P, int64_t* bad, const LayerSources* layer,
               const PointTargets* points, const RootBox& root, int tile_leaf_exp, int ne, int kchunk_leaf,
               bool dense_m2l, bool dense_near) {
  if (!(ne == 32 || ne == 48 || ne == 64 || ne == 80)) return VOLPOT_ERR_UNSUPPORTED;
  if ((layer || points) && ne != kNE) return VOLPOT_ERR_UNSUPPORTED;  // their kernels take 40 terms
  const int kNE = ne;  // reals per expansion of this plan (the namespace constant is the default)
  if (layer && (n_trees != 1 || layer->n < 0 || (layer->n > 0 && (!layer->xy || !layer->weights || !layer->normals))))
    return VOLPOT_ERR_ARG;
  if (points && (layer || n_trees != 1 || points->n < 0 || (points->n > 0 && !points->xy))) return VOLPOT_ERR_ARG;
  const double kLn2 = std::log(2.0);
  const double kInv2Pi = 1.0 / (2.0 * M_PI);
  P = Plan();
  P.ne = ne;
  P.n_trees = n_trees;
  P.n_leaves = offsets[n_trees];
  std::vector<TreeBoxes> trees(n_trees);
  std::vector<std::vector<uint64_t>> tkeys(n_trees);
  for (int t = 0; t < n_trees; ++t) {
    int64_t n = offsets[t + 1] - offsets[t];
    if (n <= 0) { if (bad) *bad = offsets[t]; return VOLPOT_ERR_TREE; }
    int rc = validate_tree(offsets[t], n, centres, levels, trees[t], tkeys[t], bad);
    if (rc != VOLPOT_OK) return rc;
  }
  // global box numbering: by (level, tree, morton)
  struct BK { int l; int32_t tree; uint64_t m; uint64_t key; };
  std::vector<BK> all;
  for (int t = 0; t < n_trees; ++t)
    for (auto& kv : trees[t].box) all.push_back({key_l(kv.first), t, morton(key_x(kv.first), key_y(kv.first)), kv.first});
  std::sort(all.begin(), all.end(), [](const BK& a, const BK& b) {
    if (a.l != b.l) return a.l < b.l;
    if (a.tree != b.tree) return a.tree < b.tree;
    return a.m < b.m;
  });
  P.n_boxes = int64_t(all.size());
  P.box_level.resize(all.size()); P.box_tree.resize(all.size()); P.box_parent.assign(all.size(), -1);
  P.box_leaf.assign(all.size(), -1); P.box_x.resize(all.size()); P.box_y.resize(all.size());
  P.box_child.assign(all.size(), {-1, -1, -1, -1});
  P.leaf_box.assign(P.n_leaves, -1);
  for (size_t i = 0; i < all.size(); ++i) {
    trees[all[i].tree].box[all[i].key] = int32_t(i);
    P.box_level[i] = all[i].l; P.box_tree[i] = all[i].tree;
    P.box_x[i] = key_x(all[i].key); P.box_y[i] = key_y(all[i].key);
    P.max_level = std::max(P.max_level, all[i].l);
  }
  for (size_t i = 0; i < all.size(); ++i) {
    TreeBoxes& tb = trees[all[i].tree];
    uint64_t k = all[i].key;
    auto lf = tb.leaf.find(k);
    if (lf != tb.leaf.end()) { P.box_leaf[i] = int32_t(lf->second); P.leaf_box[lf->second] = int32_t(i); }
    if (key_l(k) > 0) {
      int32_t p = tb.box.at(parent_key(k));
      P.box_parent[i] = p;
      int q = int(key_x(k) & 1) + 2 * int(key_y(k) & 1);
      P.box_child[p][q] = int32_t(i);
    }
  }
  // physical half-width of a level-l box: h 2^-l
  const double lnH = std::log(root.h);
  P.leaf_s2.resize(P.n_leaves); P.leaf_kappa.resize(P.n_leaves);
  for (int64_t a = 0; a < P.n_leaves; ++a) {
    int l = levels[a];
    P.leaf_s2[a] = root.h * root.h * std::ldexp(1.0, -2 * l);
    P.leaf_kappa[a] = (l * kLn2 - lnH) * kInv2Pi;  // -(1/2pi) ln s
  }
  auto key_of = [&](int32_t b) { return pack(P.box_level[b], P.box_x[b], P.box_y[b]); };
  auto find_box = [&](int32_t tree, uint64_t k) -> int32_t {
    auto it = trees[tree].box.find(k);
    return it == trees[tree].box.end() ? -1 : it->second;
  };
  auto cx = [&](int32_t b) { return centre_of(P.box_x[b], P.box_level[b]); };
  auto cy = [&](int32_t b) { return centre_of(P.box_y[b], P.box_level[b]); };
  auto hw = [&](int32_t b) { return std::ldexp(1.0, -P.box_level[b]); };
  // the box geometry the layer and point kernels read: physical centre and half-width
  auto set_geo = [&]() {
    P.box_geo.assign(size_t(P.n_boxes) * 4, 0.0);
    for (int32_t b = 0; b < P.n_boxes; ++b) {
      P.box_geo[4 * size_t(b)] = root.cx + root.h * cx(b);
      P.box_geo[4 * size_t(b) + 1] = root.cy + root.h * cy(b);
      P.box_geo[4 * size_t(b) + 2] = root.h * hw(b);
    }
  };

  // ---------------------------------------------------------------- lists
  const int64_t NB = P.n_boxes;
  Lists Ulist;  // per leaf: (near rel, src leaf)
  Lists Wlist;  // per leaf: (w rel, src box)
  Lists Vlist;  // per box: (v rel, src box)
  Lists Xlist;  // per box: (x rel, src leaf)
  const auto& NO = near_offsets();
  const auto& VO = v_offsets();
  const auto& WO = w_offsets();
  const auto& XO = x_offsets();
  build_rows(P.n_leaves, {&Ulist, &Wlist}, [&](int64_t a, std::vector<std::vector<RelIdx>*>& out) {
    int32_t ba = P.leaf_box[a];
    int32_t tr = P.box_tree[ba];
    uint64_t k = key_of(ba);
    int l = key_l(k);
    int64_t nmax = int64_t(1) << l;
    double sa = hw(ba);
    int32_t adj[32];
    int na = 0;
    adj[na++] = ba;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (!dx && !dy) continue;
        int64_t qx = key_x(k) + dx, qy = key_y(k) + dy;
        if (qx < 0 || qy < 0 || qx >= nmax || qy >= nmax) continue;
        uint64_t q = pack(l, qx, qy);
        int32_t bq = find_box(tr, q);
        if (bq >= 0) {
          if (P.box_leaf[bq] >= 0) { adj[na++] = bq; continue; }
          for (int c = 0; c < 4; ++c) {
            int32_t ch = P.box_child[bq][c];
            if (touch(key_of(ch), k)) {
              adj[na++] = ch;  // leaves by 2:1 balance
            } else {
              int r = find_offset(WO, (cx(ch) - cx(ba)) / sa, (cy(ch) - cy(ba)) / sa, 0.5);
              if (r < 0) throw std::runtime_error("W relation not found");
              out[1]->push_back({r, ch});
            }
          }
        } else {
          uint64_t c = q;
          while (find_box(tr, c) < 0 || P.box_leaf[find_box(tr, c)] < 0) c = parent_key(c);
          adj[na++] = find_box(tr, c);
        }
      }
    std::sort(adj, adj + na);
    na = int(std::unique(adj, adj + na) - adj);
    for (int i = 0; i < na; ++i) {
      const int32_t bb = adj[i];
      int r = find_offset(NO, (cx(bb) - cx(ba)) / sa, (cy(bb) - cy(ba)) / sa, hw(bb) / sa);
      if (r < 0) throw std::runtime_error("near relation not found");
      out[0]->push_back({r, P.box_leaf[bb]});
    }
  });
  build_rows(NB, {&Vlist}, [&](int64_t bi, std::vector<std::vector<RelIdx>*>& out) {
    const int32_t b = int32_t(bi);
    int l = P.box_level[b];
    if (l < 2) return;
    int32_t tr = P.box_tree[b];
    uint64_t k = key_of(b);
    int32_t par = P.box_parent[b];
    uint64_t pk = key_of(par);
    int64_t nmax = int64_t(1) << (l - 1);
    double s = hw(b);
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (!dx && !dy) continue;
        int64_t qx = key_x(pk) + dx, qy = key_y(pk) + dy;
        if (qx < 0 || qy < 0 || qx >= nmax || qy >= nmax) continue;
        int32_t pc = find_box(tr, pack(l - 1, qx, qy));
        if (pc < 0 || P.box_leaf[pc] >= 0) continue;
        for (int c = 0; c < 4; ++c) {
          int32_t ch = P.box_child[pc][c];
          if (touch(key_of(ch), k)) continue;
          int r = find_offset(VO, (cx(ch) - cx(b)) / s, (cy(ch) - cy(b)) / s, 1.0);
          if (r < 0) throw std::runtime_error("V relation not found");
          out[0]->push_back({r, ch});
        }
      }
  });
  {  // X: the dual of W, with its own offsets (from the source box's point of view)
    Xlist = transpose_rows(Wlist, NB);
    std::atomic<bool> bad_x(false);
    par_for(NB, [&](int64_t c) {
      const double s = hw(int32_t(c));
      for (int64_t e = Xlist.ptr[size_t(c)]; e < Xlist.ptr[size_t(c) + 1]; ++e) {
        RelIdx& x = Xlist.e[size_t(e)];
        const int32_t ba = P.leaf_box[x.second];
        x.first = find_offset(XO, (cx(ba) - cx(int32_t(c))) / s, (cy(ba) - cy(int32_t(c))) / s, 2.0);
        if (x.first < 0) bad_x = true;
      }
    });
    if (bad_x) throw std::runtime_error("X relation not found");
  }

  // ---------------------------------------------------------------- layer sources
  // Each curve node belongs to the leaf that holds it (a node on an edge between boxes goes to
  // the box on its right / upper side, one on the root's right or top edge to the box inside);
  // nodes are sorted by that leaf's box. A box is active when its subtree holds nodes: only
  // active boxes have multipoles, and only they are sources of M2M, M2L and M2T.
  std::vector<char> active;
  if (layer) {
    const int64_t n = layer->n;
    P.layer = true;
    P.n_src = n;
    set_geo();
    const int32_t root_box = find_box(0, pack(0, 0, 0));
    std::vector<int32_t> src_box(static_cast<size_t>(n));
    for (int64_t j = 0; j < n; ++j) {
      const double x = (layer->xy[2 * j] - root.cx) / root.h, y = (layer->xy[2 * j + 1] - root.cy) / root.h;
      const double nx = layer->normals[2 * j], ny = layer->normals[2 * j + 1];
      if (!(x >= -1.0 && x <= 1.0 && y >= -1.0 && y <= 1.0) || !std::isfinite(layer->weights[j]) || !std::isfinite(nx) ||
          !std::isfinite(ny)) {
        if (bad) *bad = j;
        return VOLPOT_ERR_ARG;
      }
      int32_t b = root_box;
      while (P.box_leaf[b] < 0) b = P.box_child[b][int(x >= cx(b)) + 2 * int(y >= cy(b))];
      src_box[size_t(j)] = b;
    }
    P.src_order.resize(size_t(n));
    for (int64_t j = 0; j < n; ++j) P.src_order[size_t(j)] = int32_t(j);
    std::stable_sort(P.src_order.begin(), P.src_order.end(),
                     [&](int32_t a, int32_t b) { return src_box[size_t(a)] < src_box[size_t(b)]; });
    P.src_xy.resize(size_t(2 * n)); P.src_w.resize(size_t(n)); P.src_n.resize(size_t(2 * n));
    for (int64_t i = 0; i < n; ++i) {
      const int64_t j = P.src_order[size_t(i)];
      P.src_xy[2 * i] = layer->xy[2 * j]; P.src_xy[2 * i + 1] = layer->xy[2 * j + 1];
      P.src_w[i] = layer->weights[j];
      P.src_n[2 * i] = layer->normals[2 * j]; P.src_n[2 * i + 1] = layer->normals[2 * j + 1];
    }
    std::vector<int64_t> cnt(size_t(NB), 0);
    for (int64_t j = 0; j < n; ++j) cnt[size_t(src_box[size_t(j)])]++;
    P.box_src_ptr.assign(size_t(NB) + 1, 0);
    for (int32_t b = 0; b < NB; ++b) P.box_src_ptr[size_t(b) + 1] = P.box_src_ptr[size_t(b)] + int32_t(cnt[size_t(b)]);
    for (int32_t b = 0; b < NB; ++b) P.n_src_leaves += (P.box_leaf[b] >= 0 && cnt[size_t(b)] > 0);
    for (int32_t b = int32_t(NB) - 1; b >= 0; --b)  // children follow their parents in box order
      if (P.box_parent[b] >= 0) cnt[size_t(P.box_parent[b])] += cnt[size_t(b)];
    active.resize(size_t(NB));
    for (int32_t b = 0; b < NB; ++b) { active[size_t(b)] = cnt[size_t(b)] > 0; P.n_active += active[size_t(b)]; }
  }
  auto use = [&](int32_t b) { return !layer || active[size_t(b)]; };

  // ---------------------------------------------------------------- evaluation points
  // Each point belongs to a leaf a (the rule of the layer nodes). At the point, u is a's local
  // expansion (level >= 2), the multipoles of a's W list, and the integrals over a's U list,
  // which take precomputed moment vectors: for leaf b with half-width s and reference point
  // xi = (x - c_b) / s, int_{B_b} G(x - y) l_k dy = s^2 (-1/2pi) (log s W_k + I_k(xi)) and its
  // x-gradient s (-1/2pi) grad I_k(xi). The plan keeps (xi, s) per pair; the moments are computed
  // on the device when the plan is uploaded (moments.hip).
  if (points) {
    const int64_t n = points->n;
    P.n_pts = n;
    set_geo();
    const int32_t root_box = find_box(0, pack(0, 0, 0));
    P.pt_xy.assign(points->xy, points->xy + 2 * n);  // physical, as the kernel evaluates
    std::vector<double> ref(size_t(2 * n));          // in the reference square
    for (int64_t j = 0; j < n; ++j) {
      ref[size_t(2 * j)] = (points->xy[2 * j] - root.cx) / root.h;
      ref[size_t(2 * j + 1)] = (points->xy[2 * j + 1] - root.cy) / root.h;
    }
    P.pt_box.resize(size_t(n));
    P.pt_loc.resize(size_t(n));
    P.pt_near_ptr.assign(1, 0);
    P.pt_w_ptr.assign(1, 0);
    for (int64_t j = 0; j < n; ++j) {
      const double x = ref[size_t(2 * j)], y = ref[size_t(2 * j + 1)];
      if (!(x >= -1.0 && x <= 1.0 && y >= -1.0 && y <= 1.0)) {
        if (bad) *bad = j;
        return VOLPOT_ERR_ARG;
      }
      int32_t b = root_box;
      while (P.box_leaf[b] < 0) b = P.box_child[b][int(x >= cx(b)) + 2 * int(y >= cy(b))];
      const int32_t a = P.box_leaf[b];
      P.pt_box[size_t(j)] = b;
      P.pt_loc[size_t(j)] = levels[a] >= 2 ? b : -1;
      for (auto& e : Ulist[size_t(a)]) P.pt_near_leaf.push_back(e.second);
      P.pt_near_ptr.push_back(int32_t(P.pt_near_leaf.size()));
      for (auto& e : Wlist[size_t(a)]) P.pt_w_box.push_back(e.second);
      P.pt_w_ptr.push_back(int32_t(P.pt_w_box.size()));
    }
    const size_t n_pairs = P.pt_near_leaf.size();
    P.pt_xi.assign(n_pairs * 3, 0.0);
    for (int64_t j = 0; j < n; ++j)
      for (int32_t e = P.pt_near_ptr[size_t(j)]; e < P.pt_near_ptr[size_t(j) + 1]; ++e) {
        const int32_t bb = P.leaf_box[P.pt_near_leaf[size_t(e)]];
        const double s = hw(bb);
        P.pt_xi[3 * size_t(e)] = (ref[2 * size_t(j)] - cx(bb)) / s;
        P.pt_xi[3 * size_t(e) + 1] = (ref[2 * size_t(j) + 1] - cy(bb)) / s;
        P.pt_xi[3 * size_t(e) + 2] = root.h * s;  // physical half-width
      }
  }

  // ---------------------------------------------------------------- stages
  const Matrices& mats = matrices(ne / 2);
  const int NTL = (tile_leaf == 32 || tile_leaf == 64) ? tile_leaf : 32;
  // k-chunk of the near-field stages; the low-rank form's segments (K = 48 or 64) take 16
  const bool lr = !layer && !dense_near;
  const int KCL = (lr || kchunk_leaf == 16) ? 16 : 32;
  const int NTB = (tile_box == 16 || tile_box == 32 || tile_box == 64) ? tile_box : 32;
  // the expansion-row stages that read or write leaf data (K or M = 256: S2M, S2L and their
  // transposes, and the pair stages of the low-rank near field) take kLeafDataTile slots
  // The leaf stages with K = 80 (L2T, M2T and their transposes' counterparts S2M^T, S2L^T) do
  // little work per tile: on small trees 16-slot tiles give more independent workgroups to hide
  // the latency of their few dependent k-chunks; on large trees and forests wider tiles read
  // each 256 x 80 table once for more slots.
  const int kNTK80 = (tile_leaf_exp == 32 || tile_leaf_exp == 64) ? tile_leaf_exp : 16;
  auto quadrant = [&](int32_t b) { return int(P.box_x[b] & 1) + 2 * int(P.box_y[b] & 1); };
  std::vector<std::vector<int32_t>> boxes_at(P.max_level + 1);
  for (int32_t b = 0; b < NB; ++b) boxes_at[P.box_level[b]].push_back(b);
  auto lnS = [&](int l) { return lnH - double(l) * kLn2; };
  std::vector<int32_t> leaf_order(P.n_leaves);
  for (int64_t a = 0; a < P.n_leaves; ++a) leaf_order[a] = int32_t(a);
  std::sort(leaf_order.begin(), leaf_order.end(), [&](int32_t x, int32_t y) { return P.leaf_box[x] < P.leaf_box[y]; });

  // inverse lists for the adjoint
  const Lists Uinv = transpose_rows(Ulist, P.n_leaves), Winv = transpose_rows(Wlist, NB),
              Vinv = transpose_rows(Vlist, NB), Xinv = transpose_rows(Xlist, P.n_leaves);
  P.pairs_near = int64_t(Ulist.e.size());
  P.pairs_w = int64_t(Wlist.e.size());
  P.pairs_v = int64_t(Vlist.e.size());
  P.pairs_x = int64_t(Xlist.e.size());

  // K: the inner dimension shared by every relation of the stage; it fixes the k-chunk
  auto init_stage = [](Stage& st, int kind, const std::string& name, int level, int M, int K, int NT, int8_t out,
                       int32_t ostride) {
    st.kind = kind; st.name = name; st.level = level; st.M = M; st.NT = NT; st.out_arr = out; st.out_stride = ostride;
    st.K = K;
    st.KC = (K == kNP) ? 32 : (M == kNP ? 16 : (K == 80 ? 40 : 16));
    for (auto& f : st.fam) f = {A_NONE, 0, 0};
    for (auto& f : st.r1fam) f = {A_NONE, 0, 0};
  };
  // the factored M2L: rows of the padded core, K and the k-chunk in complex terms (one chunk a
  // segment); the output keeps its 2q reals per box. At q = 32 the default 32-slot tiles become
  // 64-slot ones (waves of 16 rows and 32 slots); 16 slots, which small trees tune to, stay
  auto m2l_factored = [&](Stage& st, bool adj) {
    st.cx_rel = kRelH + (adj ? kNumFwd : 0);
    st.M = mats.M[size_t(st.cx_rel)];
    st.K = st.KC = mats.K[size_t(st.cx_rel)];
    if (st.KC == 32 && st.NT == 32) st.NT = 64;
  };
  // boxes at levels >= 2 ordered by (level, quadrant, tree, morton): targets of one tile then
  // share their V-list offset pattern
  std::vector<int32_t> deep_by_quadrant;
  for (int l = 2; l <= P.max_level; ++l) {
    std::vector<int32_t> tg = boxes_at[l];
    std::stable_sort(tg.begin(), tg.end(), [&](int32_t x, int32_t y) { return quadrant(x) < quadrant(y); });
    deep_by_quadrant.insert(deep_by_quadrant.end(), tg.begin(), tg.end());
  }

  // Tiling (make_tiles) is the costly part of a stage; the stages are tiled concurrently once
  // all have been described, and kept in the order they were described.
  struct Job {
    Stage st;
    std::vector<int32_t> tg;
    std::vector<std::vector<Entry>> E;
    std::vector<std::vector<R1>> R;
    bool adj;
  };
  std::vector<Job> jobs;
  auto defer = [&](Stage&& st, const std::vector<int32_t>& tg, std::vector<std::vector<Entry>>&& E,
                   std::vector<std::vector<R1>>&& R, bool adj) {
    jobs.push_back(Job{std::move(st), tg, std::move(E), std::move(R), adj});
  };

  // ================================================================ forward
  if (layer) {  // P2M: multipoles of the leaves that hold curve nodes
    Stage st; init_stage(st, K_UP, "P2M", -1, kNE, kNE, 1, A_MP, kNE);
    st.custom = C_P2M;
    for (int32_t b = 0; b < NB; ++b)
      if (P.box_leaf[b] >= 0 && P.box_src_ptr[size_t(b) + 1] > P.box_src_ptr[size_t(b)]) st.c_tgt.push_back(b);
    st.n_tiles = int(st.c_tgt.size());
    defer(std::move(st), {}, {}, {}, false);
  }
  if (!layer) {  // S2M: every leaf's multipole
    std::vector<int32_t> tg;
    for (int32_t b = 0; b < NB; ++b) if (P.box_leaf[b] >= 0) tg.push_back(b);
    Stage st; init_stage(st, K_UP, "S2M", -1, kNE, kNP, kLeafDataTile, A_MP, kNE);
    st.fam[0] = {A_INS, kNP, 0};
    std::vector<std::vector<Entry>> E(tg.size());
    std::vector<std::vector<R1>> R(tg.size());
    for (size_t i = 0; i < tg.size(); ++i) { E[i].push_back({kRelS2M, 0, P.box_leaf[tg[i]]}); P.n_s2m++; }
    defer(std::move(st), tg, std::move(E), std::move(R), false);
  }
  // Upward chain, two levels per launch: boxes of level l from their children (level l + 1,
  // complete), boxes of level l - 1 from their leaf children (level l) and, through the
  // composite M2M_qc M2M_qg, from their grandchildren (level l + 1): the launch reads nothing
  // it writes.
  auto up_pairs = [&](bool adj) {
    const int rel1 = adj ? kRelL2L + kNumFwd : kRelM2M, rel2 = adj ? kRelL2L2 + kNumFwd : kRelM2M2;
    const int8_t arr = adj ? A_LB : A_MP;
    for (int l = P.max_level - 1; l >= 2; l -= 2) {
      std::vector<int32_t> tg;
      std::vector<std::vector<Entry>> E;
      for (int32_t b : boxes_at[l]) {
        if (P.box_leaf[b] >= 0 || !use(b)) continue;
        tg.push_back(b);
        E.emplace_back();
        for (int q = 0; q < 4; ++q)
          if (use(P.box_child[b][q])) { E.back().push_back({rel1 + q, 0, P.box_child[b][q]}); P.n_m2m += !adj; }
      }
      if (l - 1 >= 2)
        for (int32_t a : boxes_at[l - 1]) {
          if (P.box_leaf[a] >= 0 || !use(a)) continue;
          tg.push_back(a);
          E.emplace_back();
          for (int qc = 0; qc < 4; ++qc) {
            const int32_t c = P.box_child[a][qc];
            if (!use(c)) continue;
            if (P.box_leaf[c] >= 0) { E.back().push_back({rel1 + qc, 0, c}); P.n_m2m += !adj; continue; }
            for (int qg = 0; qg < 4; ++qg)
              if (use(P.box_child[c][qg])) {
                E.back().push_back({rel2 + 4 * qc + qg, 0, P.box_child[c][qg]});
                P.n_m2m += !adj;
              }
          }
        }
      if (tg.empty()) continue;
      std::string name = std::string(adj ? "AL2L[" : "M2M[") + std::to_string(l) +
                         (l - 1 >= 2 ? "," + std::to_string(l - 1) : std::string()) + "]";
      Stage st; init_stage(st, adj ? K_AUP : K_UP, name, l, kNE, kNE, NTB, arr, kNE);
      st.fam[0] = {arr, kNE, 0};
      std::vector<std::vector<R1>> R(tg.size());
      defer(std::move(st), tg, std::move(E), std::move(R), adj);
    }
  };
  // Downward chain, two levels per launch, out-of-place: total = far part (acc_arr) + the
  // parent's translated total. Boxes of level l take L2L_qc of their parent's total (level
  // l - 1, complete; at level 2 the total is the far part); boxes of level l + 1 take L2L_qg of
  // their parent's far part plus the composite L2L_qg L2L_qc of their grandparent's total. The
  // first launch also copies the far part of leaves at level <= copy_level (their total).
  auto down_pairs = [&](bool adj) {
    const int rel1 = adj ? kRelM2M + kNumFwd : kRelL2L, rel2 = adj ? kRelM2M2 + kNumFwd : kRelL2L2;
    const int8_t tot = adj ? A_AB : A_LOC, farp = adj ? A_AFAR : A_FAR;
    const int copy_level = adj ? 2 : 2;
    auto parent_fam = [&](int level) -> int8_t { return level <= 2 ? 1 : 0; };  // fam 0 totals, 1 far parts
    bool first = true;
    for (int l = 3;; l += 2) {
      std::vector<int32_t> tg;
      std::vector<std::vector<Entry>> E;
      if (first)
        for (int lc = adj ? 0 : 2; lc <= std::min(copy_level, P.max_level); ++lc)
          for (int32_t b : boxes_at[lc])
            if (P.box_leaf[b] >= 0) { tg.push_back(b); E.emplace_back(); }
      if (l <= P.max_level)
        for (int32_t c : boxes_at[l]) {
          tg.push_back(c);
          E.emplace_back();
          E.back().push_back({rel1 + quadrant(c), parent_fam(l - 1), P.box_parent[c]});
          P.n_l2l += !adj;
        }
      if (l + 1 <= P.max_level)
        for (int32_t g : boxes_at[l + 1]) {
          const int32_t c = P.box_parent[g];
          tg.push_back(g);
          E.emplace_back();
          E.back().push_back({rel1 + quadrant(g), 1, c});
          E.back().push_back({rel2 + 4 * quadrant(c) + quadrant(g), parent_fam(l - 1), P.box_parent[c]});
          P.n_l2l += !adj;
        }
      first = false;
      if (!tg.empty()) {
        std::string name = std::string(adj ? "AM2M[" : "L2L[") + std::to_string(l) +
                           (l + 1 <= P.max_level ? "," + std::to_string(l + 1) : std::string()) + "]";
        Stage st; init_stage(st, adj ? K_ADOWN : K_DOWN, name, l, kNE, kNE, NTB, tot, kNE);
        st.accumulate = 1;
        st.acc_arr = farp;
        st.fam[0] = {tot, kNE, 0}; st.fam[1] = {farp, kNE, 0};
        std::vector<std::vector<R1>> R(tg.size());
        defer(std::move(st), tg, std::move(E), std::move(R), adj);
      }
      if (l + 1 >= P.max_level) break;
    }
  };
  up_pairs(false);
  if (!deep_by_quadrant.empty()) {  // FARV: M2L for every box of every level >= 2, plus all log terms
    std::vector<int32_t> tg = deep_by_quadrant;
    if (layer) {  // most boxes have few active sources: group boxes with the same V relations
      std::map<std::vector<int32_t>, int32_t> cls;
      std::vector<std::vector<int32_t>> sig(static_cast<size_t>(NB));
      for (int32_t b : tg) {
        for (auto& e : Vlist[b]) if (use(e.second)) sig[size_t(b)].push_back(e.first);
        std::sort(sig[size_t(b)].begin(), sig[size_t(b)].end());
        cls.emplace(sig[size_t(b)], 0);
      }
      int32_t rank = 0;
      for (auto& kv : cls) kv.second = rank++;
      std::stable_sort(tg.begin(), tg.end(), [&](int32_t x, int32_t y) { return cls[sig[size_t(x)]] < cls[sig[size_t(y)]]; });
    }
    Stage st; init_stage(st, K_DOWN, "FARV", -1, kNE, kNE, NTB, A_FAR, kNE);
    if (!dense_m2l) m2l_factored(st, false);
    st.fam[0] = {A_MP, kNE, 0};
    st.r1fam[0] = {A_MP, kNE, 0};
    std::vector<std::vector<Entry>> E(tg.size());
    std::vector<std::vector<R1>> R(tg.size());
    par_for(int64_t(tg.size()), [&](int64_t i) {
      int32_t b = tg[size_t(i)];
      double ls = lnS(P.box_level[b]);
      // the factored form leaves the ln|d| a_0 term of each pair to the rank-one terms
      for (auto& e : Vlist[b])
        if (use(e.second)) {
          E[size_t(i)].push_back({kRelM2L + e.first, 0, e.second});
          R[size_t(i)].push_back({0, e.second, ls + (dense_m2l ? 0.0 : mats.lnd[size_t(kRelM2L + e.first)])});
        }
      if (!layer)
        for (auto& e : Xlist[b]) R[size_t(i)].push_back({0, P.leaf_box[e.second], ls});
    });
    defer(std::move(st), tg, std::move(E), std::move(R), false);
  }
  if (layer) {  // P2L: the nodes of X-list leaves, added onto FARV
    Stage st; init_stage(st, K_DOWN, "P2L", -1, kNE, kNE, 1, A_FAR, kNE);
    st.custom = C_P2L;
    st.c_ptr.push_back(0);
    for (int32_t b : deep_by_quadrant) {
      bool any = false;
      for (auto& e : Xlist[b]) {
        const int32_t lb = P.leaf_box[e.second];
        const int32_t ns = P.box_src_ptr[size_t(lb) + 1] - P.box_src_ptr[size_t(lb)];
        if (ns == 0) continue;
        st.c_idx.push_back(lb);
        P.pairs_p2l += ns;
        any = true;
      }
      if (any) { st.c_tgt.push_back(b); st.c_ptr.push_back(int32_t(st.c_idx.size())); }
    }
    st.n_tiles = int(st.c_tgt.size());
    defer(std::move(st), {}, {}, {}, false);
  }
  if (!layer) {  // FARX: S2L, added onto FARV for the boxes that have an X list
    std::vector<int32_t> tg;
    for (int32_t b : deep_by_quadrant) if (!Xlist[b].empty()) tg.push_back(b);
    if (!tg.empty()) {
      Stage st; init_stage(st, K_DOWN, "FARX", -1, kNE, kNP, kLeafDataTile, A_FAR, kNE);
        st.accumulate = 1;
      st.fam[0] = {A_INS, kNP, 0};
      std::vector<std::vector<Entry>> E(tg.size());
      std::vector<std::vector<R1>> R(tg.size());
      par_for(int64_t(tg.size()), [&](int64_t i) {
        for (auto& e : Xlist[tg[size_t(i)]]) E[size_t(i)].push_back({kRelS2L + e.first, 0, e.second});
      });
      defer(std::move(st), tg, std::move(E), std::move(R), false);
    }
  }
  down_pairs(false);
  // Near-field targets grouped by the set of relations they take (in an adaptive tree, leaves at
  // a refinement boundary take fine or coarse neighbours in many patterns; interior leaves all
  // take the same nine), classes in lexicographic order of their relation lists (neighbouring
  // classes share most relations), box order within a class. A tile then holds
  // few relations whose slots are mostly empty: each segment costs the same whatever its
  // occupancy.
  auto by_signature = [&](const Lists& lists) {
    // a leaf's signature as a bit set of its near relations (33 < 64; one source per relation)
    std::vector<uint64_t> sig(size_t(P.n_leaves), 0);
    par_for(P.n_leaves, [&](int64_t a) {
      for (auto& e : lists[size_t(a)]) sig[size_t(a)] |= uint64_t(1) << e.first;
    });
    std::vector<uint64_t> cls(sig);
    std::sort(cls.begin(), cls.end());
    cls.erase(std::unique(cls.begin(), cls.end()), cls.end());
    // lexicographic order of the sorted relation lists: compare the lowest differing relation
    auto lex_less = [](uint64_t x, uint64_t y) {
      while (x && y) {
        const int bx = __builtin_ctzll(x), by = __builtin_ctzll(y);
        if (bx != by) return bx < by;
        x &= x - 1;
        y &= y - 1;
      }
      return x == 0 && y != 0;  // a proper prefix comes first
    };
    std::sort(cls.begin(), cls.end(), lex_less);
    std::vector<int32_t> c(size_t(P.n_leaves));
    par_for(P.n_leaves, [&](int64_t a) {
      c[size_t(a)] = int32_t(std::lower_bound(cls.begin(), cls.end(), sig[size_t(a)], lex_less) - cls.begin());
    });
    std::vector<int32_t> o(leaf_order);
    std::stable_sort(o.begin(), o.end(), [&](int32_t x, int32_t y) { return c[size_t(x)] < c[size_t(y)]; });
    return o;
  };
  const std::vector<int32_t> near_order = by_signature(Ulist), anear_order = by_signature(Uinv);
  // with overlap the dense near field's targets are cut in two parts (at a tile boundary): it
  // then runs as two launches, each beside one far-field chain. The downward chain is the
  // longer one (the S2L stage opens it), so the first part takes 45% of the leaves; on the
  // size-matched 20-Gaussian tree that gave 1.55 ms per forward + adjoint step, against 1.57 ms
  // at 50% and 1.59 ms at 55%.
  std::vector<std::pair<size_t, size_t>> halves;
  if (overlap > 0 && leaf_order.size() > size_t(NTL) && !lr) {
    const size_t cut = (leaf_order.size() * 9 / 20 + NTL - 1) / NTL * NTL;
    halves = {{0, cut}, {cut, leaf_order.size()}};
  } else {
    halves = {{0, leaf_order.size()}};
  }
  if (layer) {  // P2P: the leaves with curve nodes in an adjacent leaf (itself included), added onto LOCT
    Stage st; init_stage(st, K_NEAR, "P2P", -1, kNP, kNE, 1, A_OUT, kNP);
    st.custom = C_P2P;
    st.c_ptr.push_back(0);
    for (int32_t a : leaf_order) {
      bool any = false;
      for (auto& e : Ulist[size_t(a)]) {
        const int32_t lb = P.leaf_box[e.second];
        const int32_t ns = P.box_src_ptr[size_t(lb) + 1] - P.box_src_ptr[size_t(lb)];
        if (ns == 0) continue;
        st.c_idx.push_back(lb);
        P.pairs_p2p += int64_t(ns) * kNP;
        any = true;
      }
      if (any) { st.c_tgt.push_back(a); st.c_ptr.push_back(int32_t(st.c_idx.size())); }
    }
    st.n_tiles = int(st.c_tgt.size());
    defer(std::move(st), {}, {}, {}, false);
  }
  if (layer) halves.clear();
  // Low-rank near field (volume plans unless dense_near): every adjacent-leaf pair other than a
  // leaf with itself gets a row of A_NW holding V_r f~ of its source (stages NEARC, one per rank
  // k_r, with k_r rows), and the near field proper applies U_r to those rows and the self table,
  // in four 64-column slices, to the leaf's own f~. lr_idx: the row of each entry of Ulist (-1
  // for the self entry).
  std::vector<int64_t> lr_idx;
  auto near_rank = [&](int r) { return mats.M[size_t(kRelNV + r - 1)]; };
  // one pair stage per rank: rows of the pairs whose relation has that rank, as (row, entry)
  auto pair_stage = [&](int kind, const char* name, int rank, int8_t out, bool adj,
                        const std::function<Entry(int64_t g, int64_t a)>& entry) {
    // rows in leaf order: count each leaf's pairs of this rank, then fill concurrently
    std::vector<int64_t> at(size_t(P.n_leaves) + 1, 0);
    auto take = [&](int64_t g) { return lr_idx[size_t(g)] >= 0 && near_rank(Ulist.e[size_t(g)].first) == rank; };
    par_for(P.n_leaves, [&](int64_t a) {
      for (int64_t g = Ulist.ptr[size_t(a)]; g < Ulist.ptr[size_t(a) + 1]; ++g) at[size_t(a) + 1] += take(g);
    });
    for (int64_t a = 0; a < P.n_leaves; ++a) at[size_t(a) + 1] += at[size_t(a)];
    if (at[size_t(P.n_leaves)] == 0) return;
    std::vector<int32_t> tg(static_cast<size_t>(at[size_t(P.n_leaves)]));
    std::vector<std::vector<Entry>> E(tg.size());
    par_for(P.n_leaves, [&](int64_t a) {
      int64_t i = at[size_t(a)];
      for (int64_t g = Ulist.ptr[size_t(a)]; g < Ulist.ptr[size_t(a) + 1]; ++g)
        if (take(g)) {
          tg[size_t(i)] = int32_t(lr_idx[size_t(g)]);
          E[size_t(i++)] = {entry(g, a)};
        }
    });
    Stage st; init_stage(st, kind, name, -1, rank, kNP, kLeafDataTile, out, kNearRank);
    st.pre_near = 1;
    st.fam[0] = {adj ? A_IN : A_INS, kNP, 0};
    std::vector<std::vector<R1>> R(tg.size());
    defer(std::move(st), tg, std::move(E), std::move(R), adj);
  };
  if (lr) {
    lr_idx.assign(Ulist.e.size(), -1);
    int64_t n = 0;
    for (size_t g = 0; g < Ulist.e.size(); ++g)
      if (Ulist.e[g].first != 0) lr_idx[g] = n++;
    if (n >= (int64_t(1) << 31)) throw std::runtime_error("too many adjacent-leaf pairs");
    P.pairs_lr = n;
    for (int rank : {kNearRank, kNearRankLow})
      pair_stage(K_NEARC, rank == kNearRank ? "NEARC" : "NEARC48", rank, A_NW, false, [&](int64_t g, int64_t) {
        return Entry{kRelNV + Ulist.e[size_t(g)].first - 1, 0, Ulist.e[size_t(g)].second};
      });
  }
  // The low-rank near field is one launch into which the leaf stage (LOCT: L2T, M2T and the log
  // terms, and its adjoint ALOCT) folds: the same targets, 256 rows and k-chunk 16, its
  // segments read families 2 and 3. The folded stage runs after the far field, in LOCT's place,
  // and writes the output once instead of the near field writing it and LOCT adding on; with
  // overlap its pair stages run beside the chains.
  const bool fold = lr;
  // LOCT's segments and log terms of leaf a (families f0, f0 + 1: multipoles, locals)
  auto loct_terms = [&](int32_t a, std::vector<Entry>& E, std::vector<R1>& R, int8_t f0) {
    const double kap = P.leaf_kappa[a];
    for (auto& e : Ulist[size_t(a)]) R.push_back({0, P.leaf_box[e.second], kap});
    for (auto& e : Wlist[size_t(a)]) { E.push_back({kRelM2T + e.first, f0, e.second}); R.push_back({0, e.second, kap}); }
    if (levels[a] >= 2) E.push_back({kRelL2T, int8_t(f0 + 1), P.leaf_box[a]});
  };
  for (size_t h = 0; h < halves.size(); ++h) {  // NEAR: the adjacent-leaf tables
    const std::vector<int32_t> part(near_order.begin() + long(halves[h].first), near_order.begin() + long(halves[h].second));
    Stage st; init_stage(st, K_NEAR, halves.size() > 1 ? (h ? "NEAR_B" : "NEAR_A") : (fold ? "NEAR+LOCT" : "NEAR"), -1,
                         kNP, lr ? 64 : kNP, NTL, A_OUT, kNP);
    st.KC = KCL;
    st.fam[0] = {A_INS, kNP, 0};
    if (lr) st.fam[1] = {A_NW, kNearRank, 0};
    if (fold) {
      st.after_far = 1;
      st.r1_all_rows = 1;
      st.fam[2] = {A_MP, kNE, 0}; st.fam[3] = {A_LOC, kNE, 0};
      st.r1fam[0] = {A_MP, kNE, 0};
    }
    std::vector<std::vector<Entry>> E(part.size());
    std::vector<std::vector<R1>> R(part.size());
    par_for(int64_t(part.size()), [&](int64_t i) {
      const int32_t a = part[size_t(i)];
      if (!lr) {
        for (auto& e : Ulist[size_t(a)]) E[size_t(i)].push_back({kRelNear + e.first, 0, e.second});
        return;
      }
      for (int q = 0; q < 4; ++q) E[size_t(i)].push_back({kRelNSF + q, 0, a});
      for (int64_t g = Ulist.ptr[size_t(a)]; g < Ulist.ptr[size_t(a) + 1]; ++g)
        if (lr_idx[size_t(g)] >= 0)
          E[size_t(i)].push_back({kRelNU + Ulist.e[size_t(g)].first - 1, 1, int32_t(lr_idx[size_t(g)])});
      if (fold) loct_terms(a, E[size_t(i)], R[size_t(i)], 2);
    });
    if (fold)
      for (int32_t a : part) P.n_l2t += levels[a] >= 2;
    defer(std::move(st), part, std::move(E), std::move(R), false);
  }
  if (layer) {  // LOCT: L2T + M2T of active W boxes and their kappa(s_a) * mass terms (P2P adds on)
    Stage st; init_stage(st, K_LOCT, "LOCT", -1, kNP, kNE, kNTK80, A_OUT, kNP);
    st.r1_all_rows = 1;
    st.fam[0] = {A_MP, kNE, 0}; st.fam[1] = {A_LOC, kNE, 0};
    st.r1fam[0] = {A_MP, kNE, 0};
    std::vector<std::vector<Entry>> E(P.n_leaves);
    std::vector<std::vector<R1>> R(P.n_leaves);
    par_for(int64_t(leaf_order.size()), [&](int64_t i) {
      int32_t a = leaf_order[size_t(i)];
      double kap = P.leaf_kappa[a];
      for (auto& e : Wlist[a])
        if (use(e.second)) { E[size_t(i)].push_back({kRelM2T + e.first, 0, e.second}); R[size_t(i)].push_back({0, e.second, kap}); }
      if (levels[a] >= 2) E[size_t(i)].push_back({kRelL2T, 1, P.leaf_box[a]});
    });
    for (int32_t a : leaf_order) P.n_l2t += levels[a] >= 2;
    defer(std::move(st), leaf_order, std::move(E), std::move(R), false);
  }
  if (!layer && !fold) {  // LOCT: L2T + M2T + every kappa(s_a) * mass term, added onto NEAR
    Stage st; init_stage(st, K_LOCT, "LOCT", -1, kNP, kNE, kNTK80, A_OUT, kNP);
    st.accumulate = 1;
    st.r1_all_rows = 1;
    st.fam[0] = {A_MP, kNE, 0}; st.fam[1] = {A_LOC, kNE, 0};
    st.r1fam[0] = {A_MP, kNE, 0};
    std::vector<std::vector<Entry>> E(P.n_leaves);
    std::vector<std::vector<R1>> R(P.n_leaves);
    par_for(int64_t(leaf_order.size()), [&](int64_t i) {
      loct_terms(leaf_order[size_t(i)], E[size_t(i)], R[size_t(i)], 0);
    });
    for (int32_t a : leaf_order) P.n_l2t += levels[a] >= 2;
    defer(std::move(st), leaf_order, std::move(E), std::move(R), false);
  }

  // ================================================================ adjoint
  if (!layer) {
  {  // AL2T: lbar of leaves at level >= 2
    std::vector<int32_t> tg;
    for (int32_t b = 0; b < NB; ++b) if (P.box_leaf[b] >= 0 && P.box_level[b] >= 2) tg.push_back(b);
    if (!tg.empty()) {
      Stage st; init_stage(st, K_AUP, "AL2T", -1, kNE, kNP, kLeafDataTile, A_LB, kNE);
        st.fam[0] = {A_IN, kNP, 0};
      std::vector<std::vector<Entry>> E(tg.size());
      std::vector<std::vector<R1>> R(tg.size());
      for (size_t i = 0; i < tg.size(); ++i) E[i].push_back({kRelL2T + kNumFwd, 0, P.box_leaf[tg[i]]});
      defer(std::move(st), tg, std::move(E), std::move(R), true);
    }
  }
  up_pairs(true);
  // abar is needed for every box whose multipole is used: all leaves and boxes of level >= 2
  std::vector<int32_t> afar_tg;
  for (int l = 0; l < 2 && l <= P.max_level; ++l)
    for (int32_t b : boxes_at[l]) if (P.box_leaf[b] >= 0) afar_tg.push_back(b);
  afar_tg.insert(afar_tg.end(), deep_by_quadrant.begin(), deep_by_quadrant.end());
  // The log term of leaf a's cotangent: kappa(s_a) times the sum of ubar over a's nodes. For a
  // leaf at level >= 2 that sum is already in its lbar: L2T's first column is -1/(2 pi) at every
  // node, so AL2T leaves -(1/2 pi) sum(ubar) in row 0. Leaves above level 2 (no L2T) read the
  // leaf sums of a separate pass.
  auto usum_term = [&](int32_t a) -> R1 {
    if (levels[a] >= 2) return {0, P.leaf_box[a], -2.0 * M_PI * P.leaf_kappa[a]};
    return {1, a, P.leaf_kappa[a]};
  };
  for (int64_t a = 0; a < P.n_leaves && !P.adj_leaf_sums; ++a) P.adj_leaf_sums = levels[a] < 2;
  {  // AFARV: M2L^T plus every log term
    const auto& tg = afar_tg;
    Stage st; init_stage(st, K_ADOWN, "AFARV", -1, kNE, kNE, NTB, A_AFAR, kNE);
    if (!dense_m2l) m2l_factored(st, true);
    st.fam[0] = {A_LB, kNE, 0};
    st.r1fam[0] = {A_LB, kNE, 0}; st.r1fam[1] = {A_USUM, 1, 0};
    std::vector<std::vector<Entry>> E(tg.size());
    std::vector<std::vector<R1>> R(tg.size());
    par_for(int64_t(tg.size()), [&](int64_t ii) {
      const size_t i = size_t(ii);
      int32_t b = tg[i];
      double ls = lnS(P.box_level[b]);
      for (auto& e : Vinv[b]) {
        E[i].push_back({kRelM2L + e.first + kNumFwd, 0, e.second});
        R[i].push_back({0, e.second, ls + (dense_m2l ? 0.0 : mats.lnd[size_t(kRelM2L + e.first)])});
      }
      for (auto& e : Winv[b]) R[i].push_back(usum_term(e.second));
      int32_t leaf = P.box_leaf[b];
      if (leaf >= 0) {
        for (auto& e : Uinv[leaf]) R[i].push_back(usum_term(e.second));
        for (auto& e : Xinv[leaf]) R[i].push_back({0, e.second, lnS(P.box_level[e.second])});
      }
    });
    defer(std::move(st), tg, std::move(E), std::move(R), true);
  }
  {  // AFARW: M2T^T, added onto AFARV for the boxes that have a W^-1 list
    std::vector<int32_t> tg;
    for (int32_t b : afar_tg) if (!Winv[b].empty()) tg.push_back(b);
    if (!tg.empty()) {
      Stage st; init_stage(st, K_ADOWN, "AFARW", -1, kNE, kNP, kLeafDataTile, A_AFAR, kNE);
        st.accumulate = 1;
      st.fam[0] = {A_IN, kNP, 0};
      std::vector<std::vector<Entry>> E(tg.size());
      std::vector<std::vector<R1>> R(tg.size());
      par_for(int64_t(tg.size()), [&](int64_t i) {
        for (auto& e : Winv[tg[size_t(i)]]) E[size_t(i)].push_back({kRelM2T + e.first + kNumFwd, 0, e.second});
      });
      defer(std::move(st), tg, std::move(E), std::move(R), true);
    }
  }
  down_pairs(true);
  // the row of pair (target a, relation r != 0) in A_NW / A_NWA
  auto pair_row = [&](int32_t a, int32_t r) -> int32_t {
    for (int64_t g = Ulist.ptr[size_t(a)]; g < Ulist.ptr[size_t(a) + 1]; ++g)
      if (Ulist.e[size_t(g)].first == r) return int32_t(lr_idx[size_t(g)]);
    throw std::runtime_error("adjacent-leaf pair not found");
  };
  // ALOCT's segments of leaf b (families f0, f0 + 1: multipole and local cotangents)
  auto aloct_terms = [&](int32_t b, std::vector<Entry>& E, int8_t f0) {
    E.push_back({kRelS2M + kNumFwd, f0, P.leaf_box[b]});
    for (auto& e : Xinv[size_t(b)]) E.push_back({kRelS2L + e.first + kNumFwd, int8_t(f0 + 1), e.second});
  };
  if (lr)  // ANEARC: U_r^T ubar of the target of every pair, one stage per rank
    for (int rank : {kNearRank, kNearRankLow})
      pair_stage(K_ANEARC, rank == kNearRank ? "ANEARC" : "ANEARC48", rank, A_NWA, true, [&](int64_t g, int64_t a) {
        return Entry{kRelNU + Ulist.e[size_t(g)].first - 1 + kNumFwd, 0, int32_t(a)};
      });
  for (size_t h = 0; h < halves.size(); ++h) {  // ANEAR: transposed near tables
    const std::vector<int32_t> part(anear_order.begin() + long(halves[h].first), anear_order.begin() + long(halves[h].second));
    Stage st; init_stage(st, K_ANEAR, halves.size() > 1 ? (h ? "ANEAR_B" : "ANEAR_A") : (fold ? "ANEAR+ALOCT" : "ANEAR"),
                         -1, kNP, lr ? 64 : kNP, NTL, A_OUT, kNP);
    st.KC = KCL;
    st.out_scaled = 1;
    st.fam[0] = {A_IN, kNP, 0};
    if (lr) st.fam[1] = {A_NWA, kNearRank, 0};
    if (fold) {
      st.after_far = 1;
      st.fam[2] = {A_AB, kNE, 0}; st.fam[3] = {A_LB, kNE, 0};
    }
    std::vector<std::vector<Entry>> E(part.size());
    std::vector<std::vector<R1>> R(part.size());
    par_for(int64_t(part.size()), [&](int64_t i) {
      const int32_t b = part[size_t(i)];
      if (!lr) {
        for (auto& e : Uinv[size_t(b)]) E[size_t(i)].push_back({kRelNear + e.first + kNumFwd, 0, e.second});
        return;
      }
      for (int q = 0; q < 4; ++q) E[size_t(i)].push_back({kRelNSA + q, 0, b});
      for (auto& e : Uinv[size_t(b)])
        if (e.first != 0) E[size_t(i)].push_back({kRelNV + e.first - 1 + kNumFwd, 1, pair_row(e.second, e.first)});
      if (fold) aloct_terms(b, E[size_t(i)], 2);
    });
    defer(std::move(st), part, std::move(E), std::move(R), true);
  }
  if (!fold) {  // ALOCT: S2M^T + S2L^T, added onto ANEAR
    Stage st; init_stage(st, K_ALOCT, "ALOCT", -1, kNP, kNE, kNTK80, A_OUT, kNP);
    st.accumulate = 1;
    st.out_scaled = 1;
    st.fam[0] = {A_AB, kNE, 0}; st.fam[1] = {A_LB, kNE, 0};
    std::vector<std::vector<Entry>> E(P.n_leaves);
    std::vector<std::vector<R1>> R(P.n_leaves);
    par_for(int64_t(leaf_order.size()), [&](int64_t i) {
      aloct_terms(leaf_order[size_t(i)], E[size_t(i)], 0);
    });
    defer(std::move(st), leaf_order, std::move(E), std::move(R), true);
  }
  }  // adjoint
  {
    std::vector<std::exception_ptr> err(jobs.size());
    std::atomic<size_t> next(0);
    auto work = [&]() {
      for (size_t j; (j = next.fetch_add(1)) < jobs.size();) {
        try {
          if (jobs[j].st.custom == C_NONE) make_tiles(jobs[j].st, jobs[j].tg, jobs[j].E, jobs[j].R, mats);
        } catch (...) {
          err[j] = std::current_exception();
        }
        // the descriptions are not needed once tiled
        std::vector<std::vector<Entry>>().swap(jobs[j].E);
        std::vector<std::vector<R1>>().swap(jobs[j].R);
      }
    };
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned i = 1; i < nt; ++i) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
    for (auto& e : err)
      if (e) std::rethrow_exception(e);
    for (Job& j : jobs) {
      for (size_t i = 0; i + 1 < j.st.c_ptr.size(); ++i)  // the layer kernels stage at most 64 leaves per target
        if (j.st.c_ptr[i + 1] - j.st.c_ptr[i] > 64) throw std::runtime_error("layer list longer than 64 leaves");
      (j.adj ? P.adj : P.fwd).push_back(std::move(j.st));
    }
  }
  arrange_stages(P.fwd, false);
  arrange_stages(P.adj, true);
  return VOLPOT_OK;
}

}  // namespace vp
