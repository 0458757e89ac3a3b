// Host-side plan of the box code: tree, interaction lists, stage schedules, tables.
//
// The box code (Sec. 4.2 evaluates eq. (vbulk) with one) is organised here as a short
// sequence of "stages". Each stage writes (or adds to) one output array in a single launch.
// Within a stage every output vector (a "target") is owned by exactly one slot of one tile
// and receives a sum of small dense products A_r * source, grouped by relation r:
//
//   forward   S2M      mp  = S2M f                       all leaves        (helper stream)
//             M2M[l]   mp  = sum_q M2M_q mp[child q]     per level, up     (helper)
//             FARV     loc = sum_V M2L_r mp              levels >= 2       (helper)
//             FARX     loc += sum_X S2L_r f              boxes with X list (helper)
//             L2L[l]   loc += L2L_q loc[parent]          per level, down   (helper)
//             NEAR     u   = sum_U T_r f                 all leaves        (main, concurrent)
//             LOCT     u  += L2T loc + sum_W M2T_r mp    all leaves        (main, after join)
//   adjoint   ASUM     usum = row sums of ubar                             (helper)
//             AL2T     lbar = L2T^T ubar                 leaves            (helper)
//             AL2L[l]  lbar = sum_q L2L_q^T lbar[child q]   per level, up  (helper)
//             AFARV    abar = sum_V M2L_r^T lbar                           (helper)
//             AFARW    abar += sum_W M2T_r^T ubar       boxes with W list  (helper)
//             AM2M[l]  abar += M2M_q^T abar[parent]      per level, down   (helper)
//             ANEAR    fbar = s^2 sum_U T_r^T ubar                         (main, concurrent)
//             ALOCT    fbar += s^2 [S2M^T abar + sum_X S2L_r^T lbar]       (main, after join)
//
// All relations of one stage share the inner dimension K (80 for expansions, 256 for leaf
// values), which the k-chunk KC of the stage's kernel divides, so the kernel's chunks are
// always full. Rank-one log-scale terms (ln s_l times a box mass) are folded into the
// epilogues of FARV, LOCT and AFARV. Stages run in this order on the caller's stream; with the
// overlap option, the stages marked (helper) run on a plan-owned helper stream instead,
// concurrently with the near field, which depends on nothing but f, and LOCT waits for both.
// Owner-computes with a fixed relation order gives bitwise-deterministic results.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

namespace vp {

constexpr int kP = 16;         // nodes per dimension
constexpr int kNP = 256;       // nodes per leaf
constexpr int kTerms = 40;     // complex expansion terms (order 39)
constexpr int kNE = 80;        // reals per expansion (Re, Im interleaved), at the default order
constexpr double kDefaultEps = 1e-13;  // far-field tolerance when the options leave it at 0
int reals_for_eps(double eps);  // 32, 48, 64 or 80 reals (orders 15, 23, 31, 39); 0: eps too small
constexpr int kMaxLevel = 29;

// ---------------------------------------------------------------- relations (matrix ids)
// Forward families occupy ids [0, kNumFwd); the adjoint uses id + kNumFwd for the transpose.
constexpr int kRelS2M = 0;
constexpr int kRelM2M = 1;    // +q, q = quadrant 0..3 (child dx, dy = -/+ 1/2: q = (dy>0)*2 + (dx>0))
constexpr int kRelL2L = 5;    // +q
constexpr int kRelM2L = 9;    // +40 offsets
constexpr int kRelS2L = 49;   // +20 offsets
constexpr int kRelNear = 69;  // +33 relations
constexpr int kRelM2T = 102;  // +20 offsets
constexpr int kRelL2T = 122;
constexpr int kRelM2M2 = 123; // +4 qc + qg: M2M_qc M2M_qg, grandchild (quadrant qg of child qc) to box
constexpr int kRelL2L2 = 139; // +4 qc + qg: L2L_qg L2L_qc, box to grandchild
// The core of the factored M2L: K_r = diag(d^-l) H diag((-1)^k d^-k) + ln|d| e0 e0^T, with H the
// real, offset-free matrix H[0][0] = 0, H[0][k] = 1, H[l][0] = -1/l, H[l][k] = C(k+l-1, l),
// acting on the real and imaginary parts alike. Stored with its q rows padded to a multiple of
// 16 (zero rows), q columns; the adjoint id holds H^T padded the same way.
constexpr int kRelH = 155;
// The adjacent-leaf tables of the 32 relations other than a leaf with itself (near relation
// r = 1..32 at index r - 1) in low-rank form T_r = U_r V_r (U_r 256 x k_r, V_r k_r x 256,
// Householder QR with column pivoting truncated after k_r columns). k_r is 48 where that
// truncation is exact to rounding (corner neighbours and every coarser neighbour), else 64; the
// rows of a pair's intermediate V_r f are kNearRank apart whatever k_r. The self table (relation
// 0) as four 64-column slices for the forward (T[:, 64q .. 64q + 63], read at offset 64q of the
// source leaf) and four for the adjoint ((T[64q .. 64q + 63, :])^T, read at offset 64q of the
// cotangent).
constexpr int kNearRank = 64;
constexpr int kNearRankLow = 48;
// slots per tile of the expansion-row stages whose other side is leaf data (K or M = 256):
// S2M, S2L, their transposes and the pair stages (V_r f, U_r^T u). 64 slots make four waves
// of 16 slots each, which the kernel holds to four blocks per compute unit.
constexpr int kLeafDataTile = 64;
constexpr int kRelNU = 156;   // +32: U_r
constexpr int kRelNV = 188;   // +32: V_r
constexpr int kRelNSF = 220;  // +4: forward self slices
constexpr int kRelNSA = 224;  // +4: adjoint self slices
constexpr int kNumFwd = 228;
constexpr int kNumRel = 2 * kNumFwd;

struct Offset { double dx, dy, rho; };
const std::vector<Offset>& near_offsets();  // 33, in target half-widths
const std::vector<Offset>& v_offsets();     // 40, in half-widths (rho 1)
const std::vector<Offset>& w_offsets();     // 20 (rho 1/2)
const std::vector<Offset>& x_offsets();     // 20 (rho 2)
int find_offset(const std::vector<Offset>& v, double dx, double dy, double rho);

// ---------------------------------------------------------------- matrices
struct Matrices {
  // row-major real matrices, indexed by relation id (forward and transposed)
  std::vector<int> M, K;
  std::vector<std::vector<double>> a;
  std::vector<double> nnz;  // non-zero count of each
  // M2L relations (forward and adjoint ids) in factored form: the complex diagonals applied to
  // the source before kRelH (w_in, q values) and to the product after it (w_out, q values and
  // zeros up to the padded row count), interleaved (Re, Im); ln|d| of the offset (lnd).
  // The adjoint takes the conjugates, in swapped roles.
  std::vector<std::vector<double>> w_in, w_out;
  std::vector<double> lnd;
  // offset (in doubles) into each source vector at which a relation reads its K values (the
  // self-table slices; 0 for every other relation)
  std::vector<int> koff;
};
constexpr int pad16(int n) { return (n + 15) / 16 * 16; }
// The relation matrices for expansions of q complex terms (order q - 1; q = 16, 24, 32 or 40),
// built once per process and q; the near tables (polar quadrature) are the same for every q.
const Matrices& matrices(int q = kTerms);
// The quadrature rules of the point-moment kernel (moments.hip): leaf nodes and barycentric
// weights, the 24-point tensor rule, the 12-point edge rule and the 16-point log-product rule.
struct MomentRules;
void moment_rules(MomentRules* R);
void set_table_cache_dir(const char* dir);

// ---------------------------------------------------------------- plan
// A_INS: the input with each leaf scaled by its s^2 (forward only; written by a prescale pass)
// A_FAR / A_AFAR: the far-field parts (M2L + S2L, and their transposes) before the downward
// chains add the parents' contributions into A_LOC / A_AB
// A_NW / A_NWA: per adjacent-leaf pair (other than a leaf with itself) the 64 values V_r f of the
// low-rank near field, and U_r^T ubar of its transpose
enum Arr : int8_t { A_IN = 0, A_INS, A_OUT, A_MP, A_LOC, A_LB, A_AB, A_USUM, A_FAR, A_AFAR, A_NW, A_NWA, A_NONE };
// timing / accounting kinds: 0 upward (S2M, M2M), 1 downward (FARV/X, L2L), 2 NEAR, 3 LOCT,
// 4 adjoint upward (AL2T, AL2L), 5 adjoint downward (AFARV/W, AM2M), 6 ANEAR, 7 ALOCT,
// 8 adjoint row sums, 9 NEARC (the low-rank near field's V_r f per pair), 10 ANEARC (U_r^T ubar)
enum StageKind : int { K_UP = 0, K_DOWN, K_NEAR, K_LOCT, K_AUP, K_ADOWN, K_ANEAR, K_ALOCT, K_ASUM, K_NEARC, K_ANEARC,
                       K_NUM };

struct FamDesc { int8_t arr; int32_t stride; int8_t unused; };

// Stages of the layer-potential evaluation that are not grouped products: per-point
// expansions and direct sums over the curve's quadrature nodes (their own kernels).
enum Custom : int8_t { C_NONE = 0, C_P2M, C_P2L, C_P2P };

// One piece of a stage's work as run by one block: n_chunks consecutive k-chunks of one tile,
// starting at chunk k0 / KC of segment seg. A tile cut over several blocks ("split") has its
// pieces' partial sums added, in piece order, by whichever of those blocks finishes last.
struct Piece {
  int32_t tile;
  int32_t seg;       // first segment (index into seg_rel / seg_src)
  int32_t k0;        // first k within that segment
  int32_t n_chunks;  // 0 only for a tile without segments
  int32_t slot;      // partial-sum slot of this piece; -1 when the piece is the whole tile
  int32_t slot0;     // first slot of the tile's pieces
  int32_t n_pieces;  // pieces of the tile
  int32_t pad;
};

struct Stage {
  int kind = 0, level = 0;
  int M = 0;       // output rows (80 or 256)
  int NT = 0;      // slots per tile
  int K = 0;       // inner dimension shared by every relation of the stage
  int KC = 0;      // k-chunk of the kernel instantiation
  // >= 0: factored M2L (kRelH or its adjoint id): every segment multiplies by this core, between
  // the complex diagonals of its own relation; K is then in complex terms, one chunk per
  // segment, and the tile's columns are the real and imaginary parts of its slots
  int cx_rel = -1;
  int8_t pre_near = 0;     // runs right before the near field (its compression stage)
  int8_t after_far = 0;    // a near field with the leaf stage folded in: runs in the leaf stage's place
  double flops_issued = 0;  // MFMA work of the tiles, empty slots included
  int n_tiles = 0;
  int8_t out_arr = A_NONE;
  int32_t out_stride = 0;
  int8_t out_scaled = 0;   // multiply output by s^2 of the target leaf
  int8_t r1_all_rows = 0;  // rank-one term added to all rows (else row 0 only)
  int8_t accumulate = 0;   // add to the output (else overwrite)
  int8_t acc_arr = A_NONE; // with accumulate: add the values of this array (same layout) instead of the output's
  int8_t helper = 0;       // runs on the helper stream (far-field chain)
  int8_t join_before = 0;  // waits for the helper stream's work before launching
  int8_t fork_before = 0;  // the helper stream waits for the caller's stream before this stage
  int8_t concurrent = 0;   // runs while helper-stream stages may run: leaves compute units free
  int8_t custom = C_NONE;  // not a grouped product: c_tgt / c_ptr / c_idx describe the work
  std::string name;        // stage name for reports, e.g. NEAR or M2M[5]
  FamDesc fam[4];
  FamDesc r1fam[3];
  std::vector<int32_t> tile_tgt;      // n_tiles * NT, -1 = empty slot
  std::vector<int32_t> tile_seg_ptr;  // n_tiles + 1
  std::vector<int32_t> seg_rel;       // relation id
  std::vector<int32_t> seg_k;         // its K (a multiple of KC)
  std::vector<int8_t> seg_fam;        // index into fam[]
  std::vector<int32_t> seg_src;       // n_seg * NT source index, -1 = none
  std::vector<int32_t> r1_ptr;        // n_tiles * NT + 1
  std::vector<int32_t> r1_idx;
  std::vector<int8_t> r1_fam;
  std::vector<double> r1_coef;
  // custom stages: target c_tgt[i] takes the source leaves (boxes) c_idx[c_ptr[i] .. c_ptr[i+1])
  std::vector<int32_t> c_tgt, c_ptr, c_idx;
  double flops = 0.0;
  int64_t n_pairs = 0;
  // balanced schedule (build_schedule): block b runs pieces [blk_ptr[b], blk_ptr[b+1])
  std::vector<Piece> pieces;
  std::vector<int32_t> blk_ptr;
  int n_blocks = 0;
  int n_slots = 0;  // partial-sum slots (M x NT doubles each)
};

struct Plan {
  int ne = kNE;  // reals per expansion (2 x terms)
  int64_t n_leaves = 0, n_boxes = 0;
  int32_t n_trees = 0, max_level = 0;
  // boxes sorted by (level, tree, morton)
  std::vector<int32_t> box_level, box_tree, box_parent, box_leaf;  // box_leaf: caller leaf or -1
  std::vector<int64_t> box_x, box_y;
  std::vector<std::array<int32_t, 4>> box_child;
  std::vector<int32_t> leaf_box;     // caller leaf -> box
  std::vector<double> leaf_s2;       // s^2 per caller leaf
  std::vector<double> leaf_kappa;    // -(1/2pi) ln s per caller leaf
  std::vector<Stage> fwd, adj;
  // pair counts
  int64_t pairs_near = 0, pairs_v = 0, pairs_w = 0, pairs_x = 0, n_m2m = 0, n_l2l = 0, n_s2m = 0,
          n_l2t = 0;
  int64_t pairs_lr = 0;  // adjacent-leaf pairs in low-rank form (rows of A_NW / A_NWA), 0 if dense
  bool adj_leaf_sums = false;  // the adjoint reads leaf sums of ubar (a leaf above level 2)
  // layer potentials (point sources on a curve; empty for the volume potential)
  bool layer = false;
  int64_t n_src = 0, n_src_leaves = 0, n_active = 0, pairs_p2p = 0, pairs_p2l = 0;
  std::vector<int32_t> src_order;    // sorted position -> caller node index (sorted by leaf box)
  std::vector<double> src_xy, src_w, src_n;  // sorted positions (x, y), weights, normals (x, y)
  std::vector<int32_t> box_src_ptr;  // n_boxes + 1: the sorted nodes inside each leaf box
  std::vector<double> box_geo;       // per box: centre x, centre y, half-width, 0
  // evaluation points (volume plans with points; empty otherwise)
  int64_t n_pts = 0;
  std::vector<double> pt_xy;            // n_pts x 2
  std::vector<int32_t> pt_box;          // box of the leaf holding each point
  std::vector<int32_t> pt_loc;          // that box if its level >= 2 (it has a local expansion), else -1
  std::vector<int32_t> pt_near_ptr;     // n_pts + 1: pairs (point, adjacent leaf)
  std::vector<int32_t> pt_near_leaf;    // caller leaf of each pair
  std::vector<double> pt_xi;            // per pair: the point in that leaf's reference square (2), its half-width
                                        // (the device computes the pair's 3 x 256 moments from these)
  std::vector<int32_t> pt_w_ptr;        // n_pts + 1
  std::vector<int32_t> pt_w_box;        // W-list boxes of each point's leaf
};

// Points at which a volume plan also evaluates u and its gradient (host, caller order).
struct PointTargets {
  int64_t n;
  const double* xy;  // n x 2
};

// Quadrature nodes of a curve carrying the layer densities (host arrays, caller order).
struct LayerSources {
  int64_t n;
  const double* xy;       // n x 2
  const double* weights;  // n
  const double* normals;  // n x 2, unit
};

// Validates trees only (tiling, level grid, 2:1 balance); no tables are built.
int validate_forest(int32_t n_trees, const int64_t* offsets, const double* centres, const int32_t* levels,
                    int64_t* bad_leaf);

// Validates and builds the host plan. Returns a VOLPOT_* status; bad_leaf gets the first
// offending caller leaf index on tree errors.
// Cut a stage's work (units: one k-chunk of one segment; a tile without segments is one unit;
// tile_cost more per tile for its fixed cost, which is never cut) into at most max_blocks
// contiguous, equal ranges of at least min_units units each.
// min_units < 0 gives one block per tile instead (no tile is cut).
void build_schedule(Stage& st, int max_blocks, int min_units, int tile_cost = 0);

// overlap > 0: near field split in two launches, each concurrent with one chain of the far
// field on the helper stream (stage order and flags below); 0: one stream, plan order.
// layer != nullptr: plan the evaluation of the layer potentials of those nodes at every leaf
// node of one tree instead (no adjoint stages). points != nullptr (one tree): also prepare the
// evaluation of u and its gradient at those points (near-field moments, lists).
// The root box in the caller's coordinates: centre (cx, cy) and half-width h. Keys, lists and
// tables live in the reference square [-1,1]^2 (centres arrive mapped there); every absolute
// size the kernels see is physical: the leaves' s^2 and -(1/2pi) ln s terms, the ln s terms of
// the far field, and the box geometry, curve nodes and points of layer and point plans.
struct RootBox {
  double cx = 0.0, cy = 0.0, h = 1.0;
};

int build_plan(int32_t n_trees, const int64_t* offsets, const double* centres,
               const int32_t* levels, int tile_leaf, int tile_box, int overlap, Plan& plan, int64_t* bad_leaf,
               const LayerSources* layer = nullptr, const PointTargets* points = nullptr,
               const RootBox& root = RootBox(), int tile_leaf_exp = 16, int ne = kNE, int kchunk_leaf = 32,
               bool dense_m2l = false, bool dense_near = false);

}  // namespace vp
