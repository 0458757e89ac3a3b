// C ABI of the box code (declared in include/volpot.h): plan lifecycle, device upload of the
// shared tables and per-plan schedules, and the stage launch sequence of apply / adjoint.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <vector>

#include "../../include/volpot.h"
#include "device.hpp"
#include "moments.hpp"
#include "plan.hpp"

using namespace vp;

namespace {

// ---------------------------------------------------------------- shared device tables
struct DeviceTables {
  int device = -1, q = kTerms;  // device and expansion terms
  double* buf = nullptr;
  RelDesc* d_rels = nullptr;
  std::vector<RelDesc> rels;  // host copy (device pointers)
  size_t bytes = 0;
  int refs = 0;
};
std::mutex g_mu;
std::map<std::pair<int, int>, DeviceTables*> g_tables;  // per (device, expansion terms)

int acquire_tables(int device, int q, DeviceTables** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tables.find({device, q});
  if (it != g_tables.end()) {
    it->second->refs++;
    *out = it->second;
    return VOLPOT_OK;
  }
  const Matrices& M = matrices(q);
  std::vector<size_t> off(kNumRel), woff(kNumRel);
  size_t total = 0;
  for (int r = 0; r < kNumRel; ++r) {
    off[r] = total;
    total += size_t(M.M[r]) * M.K[r];
  }
  for (int r = 0; r < kNumRel; ++r) {  // the factored relations' diagonals after the tables
    woff[r] = total;
    total += M.w_in[r].size() + M.w_out[r].size();
  }
  std::vector<double> host(total);
  for (int r = 0; r < kNumRel; ++r) {
    std::copy(M.w_in[r].begin(), M.w_in[r].end(), host.begin() + std::ptrdiff_t(woff[r]));
    std::copy(M.w_out[r].begin(), M.w_out[r].end(), host.begin() + std::ptrdiff_t(woff[r] + M.w_in[r].size()));
  }
  for (int r = 0; r < kNumRel; ++r) {
    const int rows = M.M[r], cols = M.K[r], nt = rows / 16;
    const double* a = M.a[r].data();
    double* f = host.data() + off[r];
    for (int kk = 0; kk < cols / 4; ++kk)
      for (int i = 0; i < nt; ++i)
        for (int l = 0; l < 64; ++l) f[(size_t(kk) * nt + i) * 64 + l] = a[size_t(16 * i + (l & 15)) * cols + 4 * kk + (l >> 4)];
  }
  auto* T = new (std::nothrow) DeviceTables();
  if (!T) return VOLPOT_ERR_OOM;
  T->device = device;
  T->q = q;
  T->bytes = total * sizeof(double) + kNumRel * sizeof(RelDesc);
  if (hipMalloc(&T->buf, total * sizeof(double)) != hipSuccess) { delete T; return VOLPOT_ERR_OOM; }
  if (hipMalloc(&T->d_rels, kNumRel * sizeof(RelDesc)) != hipSuccess) { (void)hipFree(T->buf); delete T; return VOLPOT_ERR_OOM; }
  std::vector<RelDesc> rd(kNumRel);
  for (int r = 0; r < kNumRel; ++r) {
    const bool w = !M.w_in[r].empty();
    rd[r] = {T->buf + off[r], M.M[r], M.K[r], w ? T->buf + woff[r] : nullptr,
             w ? T->buf + woff[r] + M.w_in[r].size() : nullptr, M.koff[r]};
  }
  T->rels = rd;
  if (hipMemcpy(T->buf, host.data(), total * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T->d_rels, rd.data(), kNumRel * sizeof(RelDesc), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(T->buf); (void)hipFree(T->d_rels); delete T;
    return VOLPOT_ERR_HIP;
  }
  T->refs = 1;
  g_tables[{device, q}] = T;
  *out = T;
  return VOLPOT_OK;
}

void release_tables(DeviceTables* T) {
  if (!T) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (--T->refs == 0) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(T->device);
    (void)hipFree(T->buf);
    (void)hipFree(T->d_rels);
    (void)hipSetDevice(prev);
    g_tables.erase({T->device, T->q});
    delete T;
  }
}

struct DevStage {
  const Stage* st = nullptr;
  int32_t *tile_tgt = nullptr, *tile_seg_ptr = nullptr, *seg_src = nullptr;
  SegDesc* segs = nullptr;
  int32_t *r1_ptr = nullptr, *r1_idx = nullptr;
  int8_t* r1_fam = nullptr;
  double* r1_coef = nullptr;
  PieceDesc* pieces = nullptr;
  int32_t *blk_ptr = nullptr, *tile_count = nullptr;
  int32_t *c_tgt = nullptr, *c_ptr = nullptr, *c_idx = nullptr;  // custom (layer) stages
};

struct GraphEntry {
  const void* in;
  const void* in2;
  void* out;
  bool adjoint;
  hipGraphExec_t exec;
};

struct Pending { int kind; hipEvent_t a, b; };

}  // namespace

struct volpot_plan_s {
  Plan host;
  bool host_only = false;
  bool use_graph = false;
  int device = -1;
  DeviceTables* tables = nullptr;
  char* d_block = nullptr;
  double *d_mp = nullptr, *d_loc = nullptr, *d_lb = nullptr, *d_ab = nullptr, *d_usum = nullptr, *d_leaf_s2 = nullptr;
  double *d_far = nullptr, *d_afar = nullptr;  // far-field parts before the downward chains
  double *d_nw = nullptr, *d_nwa = nullptr;    // low-rank near field: per pair V_r f~, U_r^T ubar
  double* d_fs = nullptr;  // prescaled input s^2 f
  double* d_part[2] = {nullptr, nullptr};  // partial sums of split tiles: helper-stream, caller-stream stages
  int split_min = 0;
  int overlap = 0;  // compute units left to the helper stream during the near field (0: one stream)
  std::vector<DevStage> dfwd, dadj;
  int64_t device_bytes = 0;
  int32_t timing = 0;  // bit k: time the launches of stage kind k
  std::vector<hipEvent_t> ev_free;
  std::vector<Pending> pending;
  double ms[K_NUM] = {0};
  int64_t cnt[K_NUM] = {0};
  hipStream_t cap_stream = nullptr;
  std::vector<GraphEntry> graphs;
  hipStream_t helper = nullptr;  // far-field chain runs here, forked from the caller's stream
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // layer potentials: sorted curve nodes and their per-apply charges / dipoles
  int32_t *d_order = nullptr, *d_bptr = nullptr, *d_leaf_box = nullptr;
  double *d_sxy = nullptr, *d_sw = nullptr, *d_sn = nullptr, *d_geo = nullptr, *d_sq = nullptr, *d_smu = nullptr;
  LeafNodes nodes{};
  // evaluation points (volpot_plan_points)
  PointParams pts{};
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (dev >= 0 && dev != prev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

template <class T>
size_t add_bytes(size_t& total, const std::vector<T>& v) {
  size_t o = (total + 255) & ~size_t(255);
  total = o + std::max<size_t>(v.size(), 1) * sizeof(T);
  return o;
}

// Balanced schedules for every stage of the plan on the current device: each launch has as
// many blocks as fit on the device at once (fewer for small stages), each given an equal
// share of the stage's k-chunks. nominal > 0 replaces the device query (host-only plans).
int schedule_all(volpot_plan_s* p, int nominal) {
  std::map<std::array<int, 4>, int> resident;
  int cus = 256;
  if (nominal <= 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return VOLPOT_ERR_HIP;
  }
  try {
    for (auto* v : {&p->host.fwd, &p->host.adj})
      for (Stage& s : *v) {
        if (s.custom != C_NONE) continue;  // own kernels, one block per target
        auto key = std::array<int, 4>{s.M, s.NT, s.KC, s.cx_rel >= 0};
        auto it = resident.find(key);
        if (it == resident.end())
          it = resident.emplace(key, nominal > 0 ? nominal : grg_resident_blocks(s.M, s.NT, s.KC, s.cx_rel >= 0)).first;
        if (it->second <= 0) return VOLPOT_ERR_HIP;
        // a stage that runs beside the helper stream leaves `overlap` compute units' share free
        // (helper-stream stages get that share only)
        int blocks = it->second;
        const int per_cu = blocks / std::max(cus, 1);
        if (p->overlap > 0 && s.concurrent) blocks = std::max(1, blocks - per_cu * p->overlap);
        if (p->overlap > 0 && s.helper) blocks = std::max(1, std::min(blocks, per_cu * p->overlap));
        // default: a block gets at least one whole segment (K / KC chunks). A tile's fixed cost
        // (index loads, rank-one terms, the output pass) is weighted as one segment: without it,
        // blocks whose share is many one-segment tiles ran about twice as long as the others
        // in the leaf stages
        build_schedule(s, blocks, p->split_min != 0 ? p->split_min : s.K / s.KC, s.K / s.KC);
      }
  } catch (const std::bad_alloc&) {
    return VOLPOT_ERR_OOM;
  } catch (...) {
    return VOLPOT_ERR_ARG;
  }
  return VOLPOT_OK;
}

int upload(volpot_plan_s* p) {
  Plan& P = p->host;
  int rc = schedule_all(p, 0);
  if (rc != VOLPOT_OK) return rc;
  size_t total = 0;
  const size_t nb = size_t(P.n_boxes) * P.ne * sizeof(double);
  struct Off { size_t tt, tsp, sd, ss, rp, ri, rf, rc, pc, bp, tc, ct, cp, ci; };
  std::vector<std::vector<int32_t>> zeros;  // arrival counters start at zero
  std::vector<std::vector<SegDesc>> segd;   // segment descriptors (table pointers of this device)
  auto plan_stage = [&](const Stage& s) {
    Off o;
    segd.emplace_back(s.seg_rel.size());
    for (size_t i = 0; i < s.seg_rel.size(); ++i) {
      const RelDesc& rd = p->tables->rels[size_t(s.seg_rel[i])];
      const RelDesc& ra = s.cx_rel >= 0 ? p->tables->rels[size_t(s.cx_rel)] : rd;  // factored: the core
      segd.back()[i] = {ra.A, ra.K, int32_t(s.seg_fam[i]), rd.w_in, rd.w_out, rd.koff};
    }
    o.tt = add_bytes(total, s.tile_tgt); o.tsp = add_bytes(total, s.tile_seg_ptr); o.sd = add_bytes(total, segd.back());
    o.ss = add_bytes(total, s.seg_src); o.rp = add_bytes(total, s.r1_ptr);
    o.ri = add_bytes(total, s.r1_idx); o.rf = add_bytes(total, s.r1_fam); o.rc = add_bytes(total, s.r1_coef);
    o.pc = add_bytes(total, s.pieces); o.bp = add_bytes(total, s.blk_ptr);
    zeros.emplace_back(size_t(std::max(s.n_tiles, 1)), 0);
    o.tc = add_bytes(total, zeros.back());
    o.ct = add_bytes(total, s.c_tgt); o.cp = add_bytes(total, s.c_ptr); o.ci = add_bytes(total, s.c_idx);
    return o;
  };
  std::vector<Off> ofw, oad;
  for (auto& s : P.fwd) ofw.push_back(plan_stage(s));
  for (auto& s : P.adj) oad.push_back(plan_stage(s));
  const bool vol = !P.layer;  // the adjoint's and the prescaled input's arrays are for volume plans only
  size_t o_mp = (total + 255) & ~size_t(255); total = o_mp + nb;
  size_t o_loc = (total + 255) & ~size_t(255); total = o_loc + nb;
  size_t o_lb = (total + 255) & ~size_t(255); total = o_lb + (vol ? nb : 0);
  size_t o_ab = (total + 255) & ~size_t(255); total = o_ab + (vol ? nb : 0);
  size_t o_far = (total + 255) & ~size_t(255); total = o_far + nb;
  size_t o_afar = (total + 255) & ~size_t(255); total = o_afar + (vol ? nb : 0);
  const size_t nlr = size_t(P.pairs_lr) * kNearRank * sizeof(double);
  size_t o_nw = (total + 255) & ~size_t(255); total = o_nw + nlr;
  size_t o_nwa = (total + 255) & ~size_t(255); total = o_nwa + (vol ? nlr : 0);
  size_t o_us = (total + 255) & ~size_t(255); total = o_us + (vol ? size_t(P.n_leaves) * sizeof(double) : 0);
  size_t o_fs = (total + 255) & ~size_t(255); total = o_fs + (vol ? size_t(P.n_leaves) * kNP * sizeof(double) : 0);
  std::vector<double> s2(P.leaf_s2);
  size_t o_s2 = add_bytes(total, s2);
  std::vector<int32_t> leaf_box(P.layer ? P.leaf_box : std::vector<int32_t>());
  size_t o_order = add_bytes(total, P.src_order), o_sxy = add_bytes(total, P.src_xy), o_sw = add_bytes(total, P.src_w);
  size_t o_sn = add_bytes(total, P.src_n), o_bptr = add_bytes(total, P.box_src_ptr), o_geo = add_bytes(total, P.box_geo);
  size_t o_lbox = add_bytes(total, leaf_box);
  size_t o_pxy = add_bytes(total, P.pt_xy), o_ploc = add_bytes(total, P.pt_loc), o_pnp = add_bytes(total, P.pt_near_ptr);
  const size_t n_pairs = P.pt_xi.size() / 3;
  size_t o_pnl = add_bytes(total, P.pt_near_leaf), o_pwp = add_bytes(total, P.pt_w_ptr);
  size_t o_pmom = (total + 255) & ~size_t(255); total = o_pmom + n_pairs * 3 * kNP * sizeof(double);
  size_t o_pxi = add_bytes(total, P.pt_xi);
  size_t o_pwb = add_bytes(total, P.pt_w_box);
  size_t o_sq = (total + 255) & ~size_t(255); total = o_sq + std::max<size_t>(size_t(P.n_src), 1) * sizeof(double);
  size_t o_smu = (total + 255) & ~size_t(255); total = o_smu + std::max<size_t>(size_t(P.n_src), 1) * 2 * sizeof(double);
  std::vector<char> host(total, 0);
  auto put = [&](size_t o, const auto& v) {
    if (!v.empty()) std::memcpy(host.data() + o, v.data(), v.size() * sizeof(v[0]));
  };
  size_t si_ = 0;
  auto put_stage = [&](const Stage& s, const Off& o) {
    put(o.tt, s.tile_tgt); put(o.tsp, s.tile_seg_ptr); put(o.sd, segd[si_++]); put(o.ss, s.seg_src);
    put(o.rp, s.r1_ptr); put(o.ri, s.r1_idx); put(o.rf, s.r1_fam); put(o.rc, s.r1_coef);
    put(o.pc, s.pieces); put(o.bp, s.blk_ptr);
    put(o.ct, s.c_tgt); put(o.cp, s.c_ptr); put(o.ci, s.c_idx);
  };
  for (size_t i = 0; i < P.fwd.size(); ++i) put_stage(P.fwd[i], ofw[i]);
  for (size_t i = 0; i < P.adj.size(); ++i) put_stage(P.adj[i], oad[i]);
  static_assert(sizeof(Piece) == sizeof(PieceDesc), "piece layouts differ");
  put(o_s2, s2);
  put(o_order, P.src_order); put(o_sxy, P.src_xy); put(o_sw, P.src_w); put(o_sn, P.src_n);
  put(o_bptr, P.box_src_ptr); put(o_geo, P.box_geo); put(o_lbox, leaf_box);
  put(o_pxy, P.pt_xy); put(o_ploc, P.pt_loc); put(o_pnp, P.pt_near_ptr); put(o_pnl, P.pt_near_leaf);
  put(o_pxi, P.pt_xi); put(o_pwp, P.pt_w_ptr); put(o_pwb, P.pt_w_box);
  if (hipMalloc(&p->d_block, total) != hipSuccess) return VOLPOT_ERR_OOM;
  p->device_bytes = int64_t(total);
  if (hipMemcpy(p->d_block, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) return VOLPOT_ERR_HIP;
  char* b = p->d_block;
  auto mk = [&](const Stage& s, const Off& o) {
    DevStage d;
    d.st = &s;
    d.tile_tgt = reinterpret_cast<int32_t*>(b + o.tt); d.tile_seg_ptr = reinterpret_cast<int32_t*>(b + o.tsp);
    d.segs = reinterpret_cast<SegDesc*>(b + o.sd);
    d.seg_src = reinterpret_cast<int32_t*>(b + o.ss); d.r1_ptr = reinterpret_cast<int32_t*>(b + o.rp);
    d.r1_idx = reinterpret_cast<int32_t*>(b + o.ri); d.r1_fam = reinterpret_cast<int8_t*>(b + o.rf);
    d.r1_coef = reinterpret_cast<double*>(b + o.rc);
    d.pieces = reinterpret_cast<PieceDesc*>(b + o.pc); d.blk_ptr = reinterpret_cast<int32_t*>(b + o.bp);
    d.tile_count = reinterpret_cast<int32_t*>(b + o.tc);
    d.c_tgt = reinterpret_cast<int32_t*>(b + o.ct); d.c_ptr = reinterpret_cast<int32_t*>(b + o.cp);
    d.c_idx = reinterpret_cast<int32_t*>(b + o.ci);
    return d;
  };
  for (size_t i = 0; i < P.fwd.size(); ++i) p->dfwd.push_back(mk(P.fwd[i], ofw[i]));
  for (size_t i = 0; i < P.adj.size(); ++i) p->dadj.push_back(mk(P.adj[i], oad[i]));
  p->d_mp = reinterpret_cast<double*>(b + o_mp);
  p->d_loc = reinterpret_cast<double*>(b + o_loc);
  p->d_lb = reinterpret_cast<double*>(b + o_lb);
  p->d_ab = reinterpret_cast<double*>(b + o_ab);
  p->d_far = reinterpret_cast<double*>(b + o_far);
  p->d_afar = reinterpret_cast<double*>(b + o_afar);
  p->d_nw = reinterpret_cast<double*>(b + o_nw);
  p->d_nwa = reinterpret_cast<double*>(b + o_nwa);
  p->d_usum = reinterpret_cast<double*>(b + o_us);
  p->d_fs = reinterpret_cast<double*>(b + o_fs);
  p->d_leaf_s2 = reinterpret_cast<double*>(b + o_s2);
  p->d_order = reinterpret_cast<int32_t*>(b + o_order);
  p->d_sxy = reinterpret_cast<double*>(b + o_sxy);
  p->d_sw = reinterpret_cast<double*>(b + o_sw);
  p->d_sn = reinterpret_cast<double*>(b + o_sn);
  p->d_bptr = reinterpret_cast<int32_t*>(b + o_bptr);
  p->d_geo = reinterpret_cast<double*>(b + o_geo);
  p->d_leaf_box = reinterpret_cast<int32_t*>(b + o_lbox);
  p->d_sq = reinterpret_cast<double*>(b + o_sq);
  p->d_smu = reinterpret_cast<double*>(b + o_smu);
  p->pts.xy = reinterpret_cast<const double*>(b + o_pxy);
  p->pts.loc_box = reinterpret_cast<const int32_t*>(b + o_ploc);
  p->pts.near_ptr = reinterpret_cast<const int32_t*>(b + o_pnp);
  p->pts.near_leaf = reinterpret_cast<const int32_t*>(b + o_pnl);
  p->pts.mom = reinterpret_cast<const double*>(b + o_pmom);
  if (n_pairs > 0) {  // the near moments of the points' adjacent leaves, on the device
    MomentRules R;
    moment_rules(&R);
    int32_t* d_flag = nullptr;
    if (hipMalloc(&d_flag, n_pairs * sizeof(int32_t)) != hipSuccess) return VOLPOT_ERR_OOM;
    std::vector<int32_t> flag(n_pairs);
    const bool ok = launch_point_moments(R, int64_t(n_pairs), reinterpret_cast<const double*>(b + o_pxi),
                                         reinterpret_cast<double*>(b + o_pmom), d_flag, nullptr) == hipSuccess &&
                    hipDeviceSynchronize() == hipSuccess &&
                    hipMemcpy(flag.data(), d_flag, n_pairs * sizeof(int32_t), hipMemcpyDeviceToHost) == hipSuccess;
    (void)hipFree(d_flag);
    if (!ok) return VOLPOT_ERR_HIP;
    // the kernel's lists are sized so that no pair can outgrow them (bounds in moments.hip);
    // a flagged pair would mean truncated moments, so the plan fails instead
    for (size_t e = 0; e < n_pairs; ++e)
      if (flag[e]) return VOLPOT_ERR_UNSUPPORTED;
  }
  p->pts.w_ptr = reinterpret_cast<const int32_t*>(b + o_pwp);
  p->pts.w_box = reinterpret_cast<const int32_t*>(b + o_pwb);
  p->pts.geo = p->d_geo;
  p->pts.loc = p->d_loc;
  p->pts.mp = p->d_mp;
  {
    double w[kP];
    volpot_nodes(kP, p->nodes.t, w);
  }
  // partial-sum buffers, one per stream (stages on one stream run one after another)
  size_t part[2] = {0, 0};
  for (auto* v : {&P.fwd, &P.adj})
    for (const Stage& s : *v) {
      size_t need = size_t(s.n_slots) * s.M * s.NT * (s.cx_rel >= 0 ? 2 : 1) * sizeof(double);
      part[s.helper ? 0 : 1] = std::max(part[s.helper ? 0 : 1], need);
    }
  for (int i = 0; i < 2; ++i)
    if (part[i]) {
      if (hipMalloc(&p->d_part[i], part[i]) != hipSuccess) return VOLPOT_ERR_OOM;
      p->device_bytes += int64_t(part[i]);
    }
  if (hipStreamCreateWithFlags(&p->helper, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess)
    return VOLPOT_ERR_HIP;
  return VOLPOT_OK;
}

const double* arr_ptr(volpot_plan_s* p, int8_t a, const double* in, double* out) {
  switch (a) {
    case A_IN: return in;
    case A_INS: return p->d_fs;
    case A_OUT: return out;
    case A_MP: return p->d_mp;
    case A_LOC: return p->d_loc;
    case A_LB: return p->d_lb;
    case A_AB: return p->d_ab;
    case A_USUM: return p->d_usum;
    case A_FAR: return p->d_far;
    case A_AFAR: return p->d_afar;
    case A_NW: return p->d_nw;
    case A_NWA: return p->d_nwa;
    default: return nullptr;
  }
}

hipEvent_t take_event(volpot_plan_s* p) {
  if (!p->ev_free.empty()) {
    hipEvent_t e = p->ev_free.back();
    p->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void timed_begin(volpot_plan_s* p, int32_t timing, int kind, hipStream_t st, hipEvent_t* ea, hipEvent_t* eb) {
  *ea = *eb = nullptr;
  if (!(timing >> kind & 1)) return;
  *ea = take_event(p);
  *eb = take_event(p);
  if (*ea) (void)hipEventRecord(*ea, st);
}
void timed_end(volpot_plan_s* p, int kind, hipStream_t st, hipEvent_t ea, hipEvent_t eb) {
  if (ea && eb) {
    (void)hipEventRecord(eb, st);
    p->pending.push_back({kind, ea, eb});
  }
}

// The whole apply: every stage in plan order on the caller's stream. With the overlap option,
// a stage marked fork_before makes the plan's helper stream wait for the caller's stream, the
// stages marked helper then run on it (the far-field chains) while the caller's stream goes on
// (the near field), and a stage marked join_before, and the end of the apply, make the
// caller's stream wait for the helper's work, so that the caller's stream orders everything.
int run(volpot_plan_s* p, bool adjoint, const double* in, const double* in2, double* out, hipStream_t main,
        int32_t timing) {
  std::vector<DevStage>& stages = adjoint ? p->dadj : p->dfwd;
  const bool two = p->overlap > 0;
  bool forked = false;  // the helper stream holds work not yet joined
  auto fork = [&]() {
    if (hipEventRecord(p->ev_fork, main) != hipSuccess || hipStreamWaitEvent(p->helper, p->ev_fork, 0) != hipSuccess)
      return false;
    forked = true;
    return true;
  };
  auto join = [&]() {
    if (!forked) return true;
    if (hipEventRecord(p->ev_join, p->helper) != hipSuccess || hipStreamWaitEvent(main, p->ev_join, 0) != hipSuccess)
      return false;
    forked = false;
    return true;
  };
  {
    hipEvent_t ea, eb;
    if (p->host.layer) {  // charges and dipoles of the sorted curve nodes
      timed_begin(p, timing, K_UP, main, &ea, &eb);
      if (launch_layer_prep(p->host.n_src, p->d_order, p->d_sw, p->d_sn, in, in2, p->d_sq, p->d_smu, main) != hipSuccess)
        return VOLPOT_ERR_HIP;
      timed_end(p, K_UP, main, ea, eb);
    } else if (!adjoint) {  // every forward source read uses s^2 f: scale once
      timed_begin(p, timing, K_UP, main, &ea, &eb);
      if (launch_prescale(in, p->d_leaf_s2, p->d_fs, p->host.n_leaves, main) != hipSuccess) return VOLPOT_ERR_HIP;
      timed_end(p, K_UP, main, ea, eb);
    } else if (p->host.adj_leaf_sums) {  // leaf sums of the cotangent, for log terms of leaves above level 2
      timed_begin(p, timing, K_ASUM, main, &ea, &eb);
      if (launch_rowsum(in, p->d_usum, p->host.n_leaves, main) != hipSuccess) return VOLPOT_ERR_HIP;
      timed_end(p, K_ASUM, main, ea, eb);
    }
  }
  for (DevStage& d : stages) {
    const Stage& s = *d.st;
    if (two && s.fork_before && !fork()) return VOLPOT_ERR_HIP;
    if (two && s.join_before && !join()) return VOLPOT_ERR_HIP;
    if (s.n_tiles == 0) continue;
    hipStream_t st = (two && s.helper && forked) ? p->helper : main;
    if (s.custom != C_NONE) {
      hipEvent_t ea, eb;
      timed_begin(p, timing, s.kind, st, &ea, &eb);
      roctxRangePushA(s.name.c_str());
      hipError_t e = hipSuccess;
      if (s.custom == C_P2M)
        e = launch_p2m(s.n_tiles, d.c_tgt, p->d_bptr, p->d_geo, p->d_sxy, p->d_sq, p->d_smu, p->d_mp, st);
      else if (s.custom == C_P2L)
        e = launch_p2l(s.n_tiles, d.c_tgt, d.c_ptr, d.c_idx, p->d_bptr, p->d_geo, p->d_sxy, p->d_sq, p->d_smu, p->d_far, st);
      else
        e = launch_p2p(s.n_tiles, d.c_tgt, d.c_ptr, d.c_idx, p->d_leaf_box, p->d_bptr, p->d_geo, p->d_sxy, p->d_sq,
                       p->d_smu, p->nodes, out, st);
      roctxRangePop();
      timed_end(p, s.kind, st, ea, eb);
      if (e != hipSuccess) return VOLPOT_ERR_HIP;
      continue;
    }
    GrgParams g;
    std::memset(&g, 0, sizeof(g));
    g.tile_tgt = d.tile_tgt; g.tile_seg_ptr = d.tile_seg_ptr; g.segs = d.segs; g.seg_src = d.seg_src;
    for (int f = 0; f < 4; ++f) {
      g.fam_base[f] = arr_ptr(p, s.fam[f].arr, in, out);
      g.fam_stride[f] = s.fam[f].stride;
    }
    g.leaf_s2 = p->d_leaf_s2;
    g.r1_ptr = d.r1_ptr; g.r1_idx = d.r1_idx; g.r1_fam = d.r1_fam; g.r1_coef = d.r1_coef;
    for (int f = 0; f < 3; ++f) {
      g.r1_base[f] = arr_ptr(p, s.r1fam[f].arr, in, out);
      g.r1_stride[f] = s.r1fam[f].stride;
    }
    g.out = const_cast<double*>(arr_ptr(p, s.out_arr, in, out));
    g.out_stride = s.out_stride;
    g.out_scaled = s.out_scaled;
    g.r1_all_rows = s.r1_all_rows;
    g.accumulate = s.accumulate;
    g.acc_src = s.acc_arr == A_NONE ? nullptr : arr_ptr(p, s.acc_arr, in, out);
    g.pieces = d.pieces; g.blk_ptr = d.blk_ptr; g.tile_count = d.tile_count;
    g.partial = p->d_part[s.helper ? 0 : 1];  // helper-marked stages never share a buffer with the others
    g.n_blocks = s.n_blocks;
    g.cx_core = s.cx_rel >= 0 ? p->tables->rels[size_t(s.cx_rel)].A : nullptr;
    hipEvent_t ea, eb;
    timed_begin(p, timing, s.kind, st, &ea, &eb);
    roctxRangePushA(s.name.c_str());  // a host range per stage, named as in volpot_plan_stage
    hipError_t e = launch_grg(s.M, s.NT, s.KC, s.cx_rel >= 0, g, st);
    roctxRangePop();
    timed_end(p, s.kind, st, ea, eb);
    if (e != hipSuccess) return VOLPOT_ERR_HIP;
  }
  if (two && !join()) return VOLPOT_ERR_HIP;
  return VOLPOT_OK;
}

int run_graph(volpot_plan_s* p, bool adjoint, const double* in, const double* in2, double* out, hipStream_t stream) {
  for (auto& g : p->graphs)
    if (g.in == in && g.in2 == in2 && g.out == out && g.adjoint == adjoint)
      return hipGraphLaunch(g.exec, stream) == hipSuccess ? VOLPOT_OK : VOLPOT_ERR_HIP;
  if (!p->cap_stream && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) return VOLPOT_ERR_HIP;
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return VOLPOT_ERR_HIP;
  int rc = run(p, adjoint, in, in2, out, p->cap_stream, 0);
  hipError_t ec = hipStreamEndCapture(p->cap_stream, &graph);
  if (rc != VOLPOT_OK || ec != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return VOLPOT_ERR_HIP;
  }
  hipGraphExec_t exec = nullptr;
  ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ec != hipSuccess) return VOLPOT_ERR_HIP;
  p->graphs.push_back({in, in2, out, adjoint, exec});
  return hipGraphLaunch(exec, stream) == hipSuccess ? VOLPOT_OK : VOLPOT_ERR_HIP;
}

void free_plan(volpot_plan_s* p) {
  if (!p) return;
  if (p->device >= 0) {
    DeviceGuard dg(p->device);
    for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->helper) (void)hipStreamDestroy(p->helper);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    for (auto& e : p->pending) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    for (auto e : p->ev_free) (void)hipEventDestroy(e);
    if (p->d_block) (void)hipFree(p->d_block);
    for (double* d : p->d_part)
      if (d) (void)hipFree(d);
    release_tables(p->tables);
  }
  delete p;
}

int make_plan(int32_t n_trees, const int64_t* offsets, const double* centres, const int32_t* levels, int32_t p,
              const volpot_options* opt, volpot_plan_t* out, const LayerSources* layer = nullptr,
              const PointTargets* points = nullptr) {
  if (!out || !offsets || !centres || !levels || n_trees <= 0) return VOLPOT_ERR_ARG;
  if (p != kP) return VOLPOT_ERR_UNSUPPORTED;
  if (offsets[0] != 0) return VOLPOT_ERR_ARG;
  for (int t = 0; t < n_trees; ++t)
    if (offsets[t + 1] <= offsets[t]) return VOLPOT_ERR_ARG;
  if (offsets[n_trees] > (int64_t(1) << 31) - 1) return VOLPOT_ERR_UNSUPPORTED;
  volpot_options o;
  std::memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  if (o.table_cache) set_table_cache_dir(o.table_cache);
  // expansion order from the far-field tolerance (0: the default 1e-13)
  const double eps = o.eps == 0.0 ? kDefaultEps : o.eps;
  if (!(eps > 0.0)) return VOLPOT_ERR_ARG;
  const int ne = reals_for_eps(eps);
  if (ne == 0) return VOLPOT_ERR_UNSUPPORTED;
  RootBox root;
  if (o.root_halfwidth != 0.0) {
    root = RootBox{o.root_centre[0], o.root_centre[1], o.root_halfwidth};
    if (!(root.h > 0.0) || !std::isfinite(root.h) || !std::isfinite(root.cx) || !std::isfinite(root.cy))
      return VOLPOT_ERR_ARG;
  } else if (o.root_centre[0] != 0.0 || o.root_centre[1] != 0.0) {
    root.cx = o.root_centre[0];
    root.cy = o.root_centre[1];
    if (!std::isfinite(root.cx) || !std::isfinite(root.cy)) return VOLPOT_ERR_ARG;
  }
  // leaf centres in the reference square [-1,1]^2, where keys and lists are built
  std::vector<double> ref;
  const double* cref = centres;
  if (root.h != 1.0 || root.cx != 0.0 || root.cy != 0.0) {
    try {
      ref.resize(size_t(2 * offsets[n_trees]));
    } catch (const std::bad_alloc&) {
      return VOLPOT_ERR_OOM;
    }
    for (int64_t i = 0; i < offsets[n_trees]; ++i) {
      ref[size_t(2 * i)] = (centres[2 * i] - root.cx) / root.h;
      ref[size_t(2 * i + 1)] = (centres[2 * i + 1] - root.cy) / root.h;
    }
    cref = ref.data();
  }
  auto* plan = new (std::nothrow) volpot_plan_s();
  if (!plan) return VOLPOT_ERR_OOM;
  int rc;
  try {
    rc = build_plan(n_trees, offsets, cref, levels, o.tile_leaf, o.tile_box, std::max(0, o.overlap), plan->host,
                    nullptr, layer, points, root, o.tile_leaf_exp, ne, o.kchunk_leaf, o.dense_m2l != 0,
                    o.dense_near != 0);
  } catch (const std::bad_alloc&) {
    rc = VOLPOT_ERR_OOM;
  } catch (...) {
    rc = VOLPOT_ERR_TREE;
  }
  if (rc != VOLPOT_OK) { delete plan; return rc; }
  plan->host_only = o.host_only != 0;
  plan->use_graph = o.use_graph != 0;
  plan->split_min = o.deterministic ? -1 : o.split_min;  // no cut tiles: no arrival counters
  plan->overlap = std::max(0, o.overlap);
  if (plan->host_only) {  // schedules for a nominal device, so that they can be inspected
    rc = schedule_all(plan, 1024);
    if (rc != VOLPOT_OK) { delete plan; return rc; }
  } else {
    if (hipGetDevice(&plan->device) != hipSuccess) { delete plan; return VOLPOT_ERR_HIP; }
    rc = acquire_tables(plan->device, plan->host.ne / 2, &plan->tables);
    if (rc == VOLPOT_OK) rc = upload(plan);
    if (rc != VOLPOT_OK) { free_plan(plan); return rc; }
  }
  *out = plan;
  return VOLPOT_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

namespace vp {
// Reals per expansion for a far-field tolerance: the smallest order among 15, 23, 31 and 39 whose
// error bound lies below eps, 0 when none does. The bounds are about ten times the largest
// relative max-norm error of u against the oracle over adaptive trees at each order (2.3e-8 at
// 15, 2.7e-11 at 23; at 31 and 39 the truncation lies under the rounding of the sums, about
// 1e-14); the truncation part decays like 0.547^P, the rate of the V-list translations.
int reals_for_eps(double eps) {
  static const struct { double bound; int ne; } kOrders[] = {{3e-7, 32}, {3e-10, 48}, {1e-12, 64}, {1e-13, 80}};
  for (const auto& o : kOrders)
    if (eps >= o.bound) return o.ne;
  return 0;
}
}  // namespace vp

namespace {

}  // namespace

extern "C" {

int volpot_plan(const double* centres, const int32_t* levels, int64_t n_leaves, int32_t p, const volpot_options* opt,
                volpot_plan_t* out) {
  if (n_leaves <= 0) return VOLPOT_ERR_ARG;
  int64_t off[2] = {0, n_leaves};
  return make_plan(1, off, centres, levels, p, opt, out);
}

int volpot_plan_forest(int32_t n_trees, const int64_t* tree_offsets, const double* centres, const int32_t* levels,
                       int32_t p, const volpot_options* opt, volpot_plan_t* out) {
  return make_plan(n_trees, tree_offsets, centres, levels, p, opt, out);
}

int volpot_apply(volpot_plan_t plan, const double* f_dev, double* u_dev, void* hip_stream) {
  if (!plan || !f_dev || !u_dev || !aligned16(f_dev) || !aligned16(u_dev) || f_dev == u_dev) return VOLPOT_ERR_ARG;
  if (plan->host_only || plan->host.layer) return VOLPOT_ERR_STATE;
  DeviceGuard dg(plan->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  if (plan->use_graph) return run_graph(plan, false, f_dev, nullptr, u_dev, s);
  return run(plan, false, f_dev, nullptr, u_dev, s, plan->timing);
}

int volpot_apply_adjoint(volpot_plan_t plan, const double* ubar_dev, double* fbar_dev, void* hip_stream) {
  if (!plan || !ubar_dev || !fbar_dev || !aligned16(ubar_dev) || !aligned16(fbar_dev) || ubar_dev == fbar_dev)
    return VOLPOT_ERR_ARG;
  if (plan->host_only || plan->host.layer) return VOLPOT_ERR_STATE;
  DeviceGuard dg(plan->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  if (plan->use_graph) return run_graph(plan, true, ubar_dev, nullptr, fbar_dev, s);
  return run(plan, true, ubar_dev, nullptr, fbar_dev, s, plan->timing);
}

int volpot_plan_points(const double* centres, const int32_t* levels, int64_t n_leaves, int32_t p, int64_t n_points,
                       const double* points, const volpot_options* opt, volpot_plan_t* out) {
  if (n_leaves <= 0 || n_points < 0 || n_points > (int64_t(1) << 31) - 1 || (n_points > 0 && !points))
    return VOLPOT_ERR_ARG;
  int64_t off[2] = {0, n_leaves};
  PointTargets pt{n_points, points};
  return make_plan(1, off, centres, levels, p, opt, out, nullptr, &pt);
}

int volpot_apply_points(volpot_plan_t plan, const double* f_dev, double* u_dev, double* u_pts_dev, double* grad_pts_dev,
                        void* hip_stream) {
  if (!plan || !f_dev || !u_dev || !aligned16(f_dev) || !aligned16(u_dev) || f_dev == u_dev) return VOLPOT_ERR_ARG;
  if (plan->host.n_pts > 0 && !u_pts_dev) return VOLPOT_ERR_ARG;
  if (plan->host_only || plan->host.layer) return VOLPOT_ERR_STATE;
  DeviceGuard dg(plan->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  int rc = plan->use_graph ? run_graph(plan, false, f_dev, nullptr, u_dev, s)
                           : run(plan, false, f_dev, nullptr, u_dev, s, plan->timing);
  if (rc != VOLPOT_OK) return rc;
  PointParams pp = plan->pts;
  pp.f = f_dev;
  pp.u = u_pts_dev;
  pp.grad = grad_pts_dev;
  hipEvent_t ea, eb;
  timed_begin(plan, plan->timing, K_LOCT, s, &ea, &eb);
  hipError_t e = launch_points(pp, plan->host.n_pts, s);
  timed_end(plan, K_LOCT, s, ea, eb);
  return e == hipSuccess ? VOLPOT_OK : VOLPOT_ERR_HIP;
}

int volpot_layer_plan(const double* centres, const int32_t* levels, int64_t n_leaves, int32_t p, int64_t n_nodes,
                      const double* nodes, const double* weights, const double* normals, const volpot_options* opt,
                      volpot_plan_t* out) {
  if (n_leaves <= 0 || n_nodes < 0 || n_nodes > (int64_t(1) << 31) - 1) return VOLPOT_ERR_ARG;
  if (n_nodes > 0 && (!nodes || !weights || !normals)) return VOLPOT_ERR_ARG;
  int64_t off[2] = {0, n_leaves};
  LayerSources ls{n_nodes, nodes, weights, normals};
  return make_plan(1, off, centres, levels, p, opt, out, &ls);
}

int volpot_layer_apply(volpot_plan_t plan, const double* sigma_dev, const double* tau_dev, double* u_dev,
                       void* hip_stream) {
  if (!plan || !u_dev || !aligned16(u_dev)) return VOLPOT_ERR_ARG;
  if (plan->host.n_src > 0 && (!sigma_dev || !tau_dev)) return VOLPOT_ERR_ARG;
  if (plan->host_only || !plan->host.layer) return VOLPOT_ERR_STATE;
  DeviceGuard dg(plan->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  if (plan->use_graph) return run_graph(plan, false, sigma_dev, tau_dev, u_dev, s);
  return run(plan, false, sigma_dev, tau_dev, u_dev, s, plan->timing);
}

int volpot_plan_info(volpot_plan_t plan, volpot_info* out) {
  if (!plan || !out) return VOLPOT_ERR_ARG;
  const Plan& P = plan->host;
  std::memset(out, 0, sizeof(*out));
  out->n_leaves = P.n_leaves;
  out->n_boxes = P.n_boxes;
  out->n_trees = P.n_trees;
  out->max_level = P.max_level;
  out->order = plan->host.ne / 2 - 1;
  out->n_reals = plan->host.ne;
  out->n_stages = int32_t(P.fwd.size() + P.adj.size());
  out->pairs_near = P.pairs_near; out->pairs_v = P.pairs_v; out->pairs_w = P.pairs_w; out->pairs_x = P.pairs_x;
  out->n_m2m = P.n_m2m; out->n_l2l = P.n_l2l; out->n_s2m = P.n_s2m; out->n_l2t = P.n_l2t;
  for (const Stage& s : P.fwd) {
    out->flops_total += s.flops;
    out->flops_kind[s.kind] += s.flops;
    out->flops_issued_kind[s.kind] += s.flops_issued;
    out->launches_kind[s.kind] += s.n_tiles > 0;
  }
  for (const Stage& s : P.adj) {
    out->flops_adjoint += s.flops;
    out->flops_kind[s.kind] += s.flops;
    out->flops_issued_kind[s.kind] += s.flops_issued;
    out->launches_kind[s.kind] += s.n_tiles > 0;
  }
  if (P.adj_leaf_sums) {  // the leaf-sum pass runs only for plans with leaves above level 2
    out->flops_kind[K_ASUM] = double(P.n_leaves) * kNP;  // one add per value
    out->flops_adjoint += out->flops_kind[K_ASUM];
    out->launches_kind[K_ASUM] = 1;
  }
  out->bytes_min = 16.0 * double(P.n_leaves) * kNP;
  if (P.layer) {
    out->flops_kind[K_ASUM] = 0.0;
    out->launches_kind[K_ASUM] = 0;
    out->flops_adjoint = 0.0;
    out->bytes_min = 8.0 * double(P.n_leaves) * kNP + 16.0 * double(P.n_src);
  }
  out->n_layer_nodes = P.n_src;
  out->n_source_leaves = P.n_src_leaves;
  out->n_active_boxes = P.n_active;
  out->pairs_p2p = P.pairs_p2p;
  out->pairs_p2l = P.pairs_p2l;
  out->n_points = P.n_pts;
  out->pairs_points = int64_t(P.pt_near_leaf.size());
  out->pairs_lowrank = P.pairs_lr;
  out->device_bytes = plan->device_bytes + (plan->tables ? int64_t(plan->tables->bytes) : 0);
  return VOLPOT_OK;
}

int volpot_plan_n_stages(volpot_plan_t plan, int32_t adjoint, int32_t* n) {
  if (!plan || !n) return VOLPOT_ERR_ARG;
  *n = int32_t((adjoint ? plan->host.adj : plan->host.fwd).size());
  return VOLPOT_OK;
}

int volpot_plan_stage(volpot_plan_t plan, int32_t adjoint, int32_t index, volpot_stage_info* out) {
  if (!plan || !out) return VOLPOT_ERR_ARG;
  const auto& v = adjoint ? plan->host.adj : plan->host.fwd;
  if (index < 0 || size_t(index) >= v.size()) return VOLPOT_ERR_ARG;
  const Stage& s = v[size_t(index)];
  std::memset(out, 0, sizeof(*out));
  std::strncpy(out->name, s.name.c_str(), sizeof(out->name) - 1);
  out->kind = s.kind;
  out->rows = s.M;
  out->tile = s.NT;
  out->kchunk = s.KC;
  out->helper = s.helper;
  out->n_tiles = s.n_tiles;
  out->n_segments = int64_t(s.seg_rel.size());
  out->n_blocks = s.n_blocks;
  std::vector<int32_t> pieces(size_t(std::max(s.n_tiles, 0)), 0);
  for (const Piece& pc : s.pieces) pieces[size_t(pc.tile)]++;
  for (int32_t c : pieces) out->n_split_tiles += c > 1;
  out->flops = s.flops;
  out->flops_issued = s.flops_issued;
  out->inner = s.K;
  out->factored = s.cx_rel >= 0;
  for (int32_t k : s.seg_k) out->n_chunks += k / s.KC;
  return VOLPOT_OK;
}

int volpot_validate_tree(const double* centres, const int32_t* levels, int64_t n_leaves, int32_t p, int64_t* bad_index) {
  if (!centres || !levels || n_leaves <= 0) return VOLPOT_ERR_ARG;
  if (p != kP) return VOLPOT_ERR_UNSUPPORTED;
  int64_t off[2] = {0, n_leaves};
  try {
    return validate_forest(1, off, centres, levels, bad_index);
  } catch (const std::bad_alloc&) {
    return VOLPOT_ERR_OOM;
  } catch (...) {
    return VOLPOT_ERR_TREE;
  }
}

int volpot_nodes(int32_t p, double* t, double* w) {
  if (p < 1 || p > 64 || !t || !w) return VOLPOT_ERR_ARG;
  for (int i = 0; i < p; ++i) {
    double th = (2.0 * i + 1.0) * M_PI / (2.0 * p);
    t[i] = -std::cos(th);
    double s = 0.0;
    for (int j = 1; j <= p / 2; ++j) s += std::cos(2.0 * j * th) / (4.0 * j * j - 1.0);
    w[i] = (2.0 / p) * (1.0 - 2.0 * s);
  }
  return VOLPOT_OK;
}

void volpot_plan_destroy(volpot_plan_t plan) { free_plan(plan); }

const char* volpot_status_string(int status) {
  switch (status) {
    case VOLPOT_OK: return "ok";
    case VOLPOT_ERR_ARG: return "invalid argument";
    case VOLPOT_ERR_TREE: return "leaves do not form a tiling of the root on the level grid";
    case VOLPOT_ERR_UNBALANCED: return "tree is not 2:1 balanced over edges and corners";
    case VOLPOT_ERR_UNSUPPORTED: return "unsupported order or level";
    case VOLPOT_ERR_HIP: return "HIP runtime error";
    case VOLPOT_ERR_OOM: return "out of memory";
    case VOLPOT_ERR_STATE: return "plan has no device state (host-only or destroyed)";
    default: return "unknown status";
  }
}

int volpot_set_timing(volpot_plan_t plan, int32_t enable) {
  if (!plan) return VOLPOT_ERR_ARG;
  if (plan->use_graph && enable) return VOLPOT_ERR_STATE;
  if (enable != 0 && enable != 1 && (enable < 256 || (enable >> 8) >= (1 << K_NUM))) return VOLPOT_ERR_ARG;
  plan->timing = enable == 1 ? (1 << K_NUM) - 1 : (enable >> 8);
  return VOLPOT_OK;
}

int volpot_stage_times(volpot_plan_t plan, double* ms, int64_t* launches, int32_t n_kinds) {
  if (!plan || !ms || !launches || n_kinds < 1) return VOLPOT_ERR_ARG;
  if (plan->device >= 0) {
    DeviceGuard dg(plan->device);
    for (auto& e : plan->pending) {
      float t = 0.0f;
      if (hipEventSynchronize(e.b) != hipSuccess || hipEventElapsedTime(&t, e.a, e.b) != hipSuccess) return VOLPOT_ERR_HIP;
      plan->ms[e.kind] += t;
      plan->cnt[e.kind] += 1;
      plan->ev_free.push_back(e.a);
      plan->ev_free.push_back(e.b);
    }
    plan->pending.clear();
  }
  for (int k = 0; k < n_kinds; ++k) {
    ms[k] = k < K_NUM ? plan->ms[k] : 0.0;
    launches[k] = k < K_NUM ? plan->cnt[k] : 0;
  }
  for (int k = 0; k < K_NUM; ++k) { plan->ms[k] = 0.0; plan->cnt[k] = 0; }
  return VOLPOT_OK;
}

int volpot_plan_table(volpot_plan_t plan, int32_t kind, int32_t index, double* out, int64_t n) {
  if (!plan || !out) return VOLPOT_ERR_ARG;
  const Matrices& M = matrices(plan->host.ne / 2);
  int id;
  if (kind == 0 && index >= 0 && index < 33) id = kRelNear + index;
  else if (kind == 1 && index == 0) id = kRelS2M;
  else if (kind == 2 && index == 0) id = kRelL2T;
  else if ((kind == 3 || kind == 4) && index >= 1 && index < 33) {  // zero-padded to rank 64
    id = (kind == 3 ? kRelNU : kRelNV) + index - 1;
    const int rows = kind == 3 ? kNP : kNearRank, cols = kind == 3 ? kNearRank : kNP;
    if (n < int64_t(rows) * cols) return VOLPOT_ERR_ARG;
    const int m = M.M[size_t(id)], k = M.K[size_t(id)];
    for (int i = 0; i < rows; ++i)
      for (int c = 0; c < cols; ++c) out[size_t(i) * cols + c] = (i < m && c < k) ? M.a[size_t(id)][size_t(i) * k + c] : 0.0;
    return VOLPOT_OK;
  } else {
    return VOLPOT_ERR_ARG;
  }
  if (n < int64_t(M.a[id].size())) return VOLPOT_ERR_ARG;
  std::memcpy(out, M.a[id].data(), M.a[id].size() * sizeof(double));
  return VOLPOT_OK;
}

int volpot_near_relation(int32_t r, double* dx, double* dy, double* rho) {
  if (r < 0 || r >= 33 || !dx || !dy || !rho) return VOLPOT_ERR_ARG;
  const Offset& o = near_offsets()[r];
  *dx = o.dx; *dy = o.dy; *rho = o.rho;
  return VOLPOT_OK;
}

}  // extern "C"
