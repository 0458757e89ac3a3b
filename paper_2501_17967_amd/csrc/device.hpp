// Device-side interface between the C ABI (api.cpp) and the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vp {

// Work of one block: n_chunks k-chunks of one tile (mirrors the host plan's Piece)
struct PieceDesc {
  int32_t tile, seg, k0, n_chunks, slot, slot0, n_pieces, pad;
};

// One segment of a tile: its relation table (fragment-major), inner dimension and source family;
// in a factored stage also the relation's complex diagonals (interleaved Re, Im): w_in scales
// the K source terms before the table, w_out the table's rows after it
struct SegDesc {
  const double* A;
  int32_t K;
  int32_t fam;
  const double* w_in;
  const double* w_out;
  int32_t k_off;  // the relation reads its K source values from this offset on (self-table slices)
  int32_t pad;
};

struct RelDesc {
  const double* A;  // fragment-major: frag[(kk * (M/16) + row_tile) * 64 + lane] = A[16 row_tile + lane%16][4 kk + lane/16]
  int32_t M, K;
  const double* w_in;   // factored M2L relations only, else null
  const double* w_out;
  int32_t koff;         // offset into the source vector (self-table slices), else 0
};

// Arguments of one stage launch (grouped-relation GEMM). Passed by value.
struct GrgParams {
  const int32_t* tile_tgt;      // n_tiles * NT, -1 = empty slot
  const int32_t* tile_seg_ptr;  // n_tiles + 1
  const SegDesc* segs;          // per segment
  const int32_t* seg_src;       // n_seg * NT source index, -1 = none
  const double* fam_base[4];
  int32_t fam_stride[4];
  const double* leaf_s2;        // s^2 per leaf (output scaling of the adjoint leaf stages)
  const int32_t* r1_ptr;        // n_tiles * NT + 1
  const int32_t* r1_idx;
  const int8_t* r1_fam;
  const double* r1_coef;
  const double* r1_base[3];
  int32_t r1_stride[3];
  double* out;
  int32_t out_stride;
  int32_t out_scaled;           // 1: multiply the output of target t by leaf_s2[t]
  int32_t r1_all_rows;          // 1: rank-one term on every row, else on row 0 only
  int32_t accumulate;           // 1: add to the existing output (or to acc_src), else overwrite
  const double* acc_src;        // with accumulate: add this array's values (output layout) instead of the output's
  const PieceDesc* pieces;      // balanced schedule: block b runs pieces [blk_ptr[b], blk_ptr[b+1])
  const int32_t* blk_ptr;       // n_blocks + 1
  int32_t* tile_count;          // n_tiles arrival counters of split tiles, zero between launches
  double* partial;              // partial sums of split tiles, M x NT doubles per slot (2 NT factored)
  int32_t n_blocks;
  const double* cx_core;        // factored stages: the core table (fragment-major, M x K)
};

// Blocks of the grouped-product kernel for (M, NT, KC, factored) that fit on the current device
// at once (0 on error).
int grg_resident_blocks(int M, int NT, int KC, bool factored = false);

// Launch one stage: M rows, NT slots per tile, k-chunk KC; factored (the M2L core between two
// complex diagonals): M = the padded core rows, KC = the complex terms q, 2 NT columns.
// hipErrorInvalidValue for a shape without an instantiation.
hipError_t launch_grg(int M, int NT, int KC, bool factored, const GrgParams& p, hipStream_t stream);
// out = s2[leaf] * x  (n_leaves x 256)
hipError_t launch_prescale(const double* x, const double* s2, double* out, int64_t n_leaves, hipStream_t stream);
// usum[a] = sum of the 256 values of leaf a
hipError_t launch_rowsum(const double* x, double* usum, int64_t n_leaves, hipStream_t stream);

// ---------------------------------------------------------------- layer potentials (layer.hip)
// Nodes of a leaf on [-1,1] (first-kind Chebyshev, ascending); passed by value.
struct LeafNodes {
  double t[16];
};
// Sorted curve nodes j: q[j] = w[j] sigma[order[j]], mu[j] = w[j] tau[order[j]] n[j] (complex).
hipError_t launch_layer_prep(int64_t n, const int32_t* order, const double* w, const double* nrm, const double* sigma,
                             const double* tau, double* q, double* mu, hipStream_t stream);
// Multipoles (80 reals) of the leaf boxes tgt[0 .. n_tgt) from their sorted nodes bptr[b] .. bptr[b+1].
hipError_t launch_p2m(int32_t n_tgt, const int32_t* tgt, const int32_t* bptr, const double* geo, const double* sxy,
                      const double* q, const double* mu, double* mp, hipStream_t stream);
// far[tgt[i]] += local expansion of the nodes of the leaf boxes idx[ptr[i] .. ptr[i+1]).
hipError_t launch_p2l(int32_t n_tgt, const int32_t* tgt, const int32_t* ptr, const int32_t* idx, const int32_t* bptr,
                      const double* geo, const double* sxy, const double* q, const double* mu, double* far,
                      hipStream_t stream);
// u[tgt[i]] (256 values) = direct sum over the nodes of the leaf boxes idx[ptr[i] .. ptr[i+1]).
hipError_t launch_p2p(int32_t n_tgt, const int32_t* tgt, const int32_t* ptr, const int32_t* idx, const int32_t* leaf_box,
                      const int32_t* bptr, const double* geo, const double* sxy, const double* q, const double* mu,
                      const LeafNodes& nodes, double* u, hipStream_t stream);

// ---------------------------------------------------------------- evaluation points (points.hip)
struct PointParams {
  const double* xy;         // n x 2
  const int32_t* loc_box;   // box whose local expansion applies, -1 for leaves above level 2
  const int32_t* near_ptr;  // n + 1
  const int32_t* near_leaf;
  const double* mom;        // per pair 3 x 256
  const int32_t* w_ptr;     // n + 1
  const int32_t* w_box;
  const double* geo;        // per box: centre x, centre y, half-width, 0
  const double* f;          // the apply's input, [n_leaves][256]
  const double* loc;        // local expansions, [n_boxes][80]
  const double* mp;         // multipoles, [n_boxes][80]
  double* u;                // n
  double* grad;             // n x 2, or null
};
// u (and grad) at the n points, after a forward apply that filled loc and mp
hipError_t launch_points(const PointParams& p, int64_t n, hipStream_t stream);

// ---------------------------------------------------------------- quadtree construction (tree.hip)
// First-kind points t (ascending) and the values-to-coefficients transform D[m][i]; by value.
struct TreeRule {
  double t[16];
  double D[256];
};
// Node coordinates [n][256][2] of the boxes with packed keys (level << 58 | ix << 29 | iy).
hipError_t launch_tree_nodes(const int64_t* keys, int64_t n, const TreeRule& r, double* nodes, hipStream_t stream);
// Chebyshev tail of each box's 256 samples.
hipError_t launch_tree_tail(const double* values, int64_t n, const TreeRule& r, double* tails, hipStream_t stream);

// Device work of the builder (tree.hip). Keys are packed (level << 58 | ix << 29 | iy).
struct TreeWork {
  // growable device buffers (element capacities alongside), owned by the builder
  uint64_t *pend = nullptr, *next = nullptr, *leaves = nullptr, *tmp = nullptr, *anc = nullptr;
  double* tails = nullptr;
  int32_t *flag = nullptr, *pos = nullptr;
  void* scratch = nullptr;
  size_t cap_pend = 0, cap_next = 0, cap_leaves = 0, cap_tmp = 0, cap_anc = 0, cap_tails = 0, cap_flag = 0,
         cap_pos = 0, scratch_bytes = 0;
  int64_t n_pend = 0, n_leaves = 0;  // pending boxes (keys in pend) and leaves so far (in leaves)
};
// Device copy of the first round's keys (host, n): pend and n_pend.
hipError_t tree_upload_pending(TreeWork& w, const uint64_t* keys, int64_t n, hipStream_t stream);
// One round: tails of the pending boxes from their samples, the split decision (level below
// max_level and tail not <= tol), the split boxes' children as the next pending boxes and the
// others appended to the leaves; n_pend and n_leaves are updated (synchronises the stream).
hipError_t tree_round(TreeWork& w, const double* values, const TreeRule& r, double tol, int max_level,
                      hipStream_t stream);
// The 2:1 balance of the leaves over edges and corners (split every leaf that a leaf two or more
// levels finer touches, to a fixpoint); leaves then holds n_leaves keys (level << 58 | iy << 29 |
// ix), ascending: by level, then y, then x (synchronises).
hipError_t tree_balance(TreeWork& w, hipStream_t stream);
void tree_free(TreeWork& w);

}  // namespace vp
