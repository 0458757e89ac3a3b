/* volpot.h -- C ABI of the MI355X machine code for the 2D Laplace volume potential.
 *
 * What is computed (Sec. 4.2, eq. (vbulk) of Fortunato, Stein & Barnett, "A fully adaptive,
 * high-order, fast Poisson solver for complex two-dimensional geometries"): the volume
 * potential of leaf data on an adaptive, 2:1-balanced quadtree,
 *
 *     u(x) = int_{Omega_B} G(x - y) f_h(y) dy,      G(r) = -(1/2 pi) log |r|,
 *
 * evaluated at every leaf node. Omega_B is the union of the leaves; on each leaf f_h is the
 * order-p tensor Chebyshev interpolant of the nodal values the caller supplies (Sec. 4.2.1,
 * "Constructing a quadtree approximation to f"). The sign is chosen so that -Lap u = f; the
 * paper's v_bulk equals -u.
 *
 * Conventions
 *   root box      [-1,1]^2 at level 0 by default (volpot_options.root_centre / root_halfwidth
 *                 move and scale it); a level-l box has half-width s_l = h 2^-l; levels 0..29.
 *   leaf nodes    p = 16 first-kind Chebyshev points per dimension,
 *                 t_i = -cos((2i-1) pi / (2p)), i = 1..p (ascending); see volpot_nodes.
 *   leaf data     FP64, contiguous [n_leaves][p][p]: leaf in the caller's order, then the y
 *                 index j, then the x index i (x fastest). Same layout for f, u, their
 *                 cotangents, and for every tree of a forest (trees concatenated).
 *   balance       neighbouring leaves (sharing an edge or a corner) differ by at most one level
 *                 (the 2:1 balance the paper applies after building the tree, Sec. 4.2.1).
 *
 * Ownership and streams
 *   A plan owns every device table, list and workspace it needs; they are allocated by
 *   volpot_plan / volpot_plan_forest, so volpot_apply and volpot_apply_adjoint allocate
 *   nothing. The caller owns f, u and the stream. Both apply calls are asynchronous on the
 *   given hipStream_t (NULL = the default stream) and do not synchronise the host. One plan
 *   serves one stream at a time (its workspace is shared); destroy a plan only after work
 *   queued on it has completed. Input and output arrays must not alias.
 *
 * Errors
 *   Every call returns a status code (VOLPOT_OK = 0, negative on error) and never throws.
 *   Invalid trees are rejected at plan time; volpot_validate_tree reports the first offending
 *   leaf. NaN/Inf in the data are not checked and propagate.
 */
#ifndef VOLPOT_H
#define VOLPOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct volpot_plan_s* volpot_plan_t;

enum {
  VOLPOT_OK = 0,
  VOLPOT_ERR_ARG = -1,         /* null pointer, bad size or option */
  VOLPOT_ERR_TREE = -2,        /* leaves do not tile the root, overlap, or are off the level grid */
  VOLPOT_ERR_UNBALANCED = -3,  /* two adjacent leaves differ by more than one level */
  VOLPOT_ERR_UNSUPPORTED = -4, /* p other than 16, level above 29 */
  VOLPOT_ERR_HIP = -5,         /* a HIP runtime call failed */
  VOLPOT_ERR_OOM = -6,         /* device or host allocation failed */
  VOLPOT_ERR_STATE = -7        /* plan built host-only, or destroyed */
};

typedef struct {
  int32_t host_only;       /* 1: build lists and tables on the host only (no device memory;
                              apply calls return VOLPOT_ERR_STATE). Default 0. */
  int32_t use_graph;       /* 1: capture each apply once per (input, output) pointer pair into
                              a hipGraph and replay it. Default 0. */
  int32_t tile_leaf;       /* slots per tile of the near-field stages (256 rows): 32 or 64;
                              0 = default (32). The 256-row stages with K = 80 take
                              tile_leaf_exp. */
  int32_t tile_box;        /* slots per tile of the expansion translation stages (M2M, L2L
                              chains, M2L): 16, 32 or 64; 0 = default (32). The expansion
                              stages whose other side is leaf data (S2M, S2L, their transposes,
                              the low-rank near field's pair stages) take 64, and so does the
                              factored M2L at expansion order 31 in place of 32. */
  const char* table_cache; /* directory for the host table cache; NULL = keep tables in memory */
  int32_t split_min;       /* each stage is cut into as many equal shares of its k-chunks as the
                              device runs blocks at once; a share has at least this many chunks
                              (0 = default: one relation's worth, K / chunk; -1 = no cut:
                              one block per tile) */
  int32_t overlap;         /* 0 (default): every stage on the caller's stream, in plan order.
                              n > 0: the near field runs as two launches that leave n compute
                              units' share of blocks free, each beside one latency-bound chain
                              of the far field (upward, downward) on a plan-owned helper
                              stream forked from and joined back into the caller's stream */
  double root_centre[2];   /* centre (x, y) of the root box in the caller's coordinates
                              (default 0, 0) */
  double root_halfwidth;   /* half-width h > 0 of the root box; 0 = default 1. The root box
                              B_0 = centre + [-h, h]^2 must hold the domain (Sec. 4.2.1); a
                              level-l leaf has half-width h 2^-l, and every coordinate the plan
                              takes (leaf centres, curve nodes, evaluation points) and every
                              output is in the caller's coordinates: u is the potential of the
                              caller's box sizes, including the log kernel's ln h term. */
  int32_t tile_leaf_exp;   /* slots per tile of the leaf stages whose sources are expansions
                              (L2T + M2T, and S2M^T + S2L^T in the adjoint; K = 80): 16, 32 or
                              64; 0 = default (16) */
  double eps;              /* far-field tolerance (Sec. 4.2.1: the user gives p and epsilon):
                              a bound on the relative max-norm error of u from truncating the
                              expansions. It selects the expansion order P, the smallest of 15,
                              23, 31, 39 whose bound is below eps (bounds 3e-7, 3e-10, 1e-12,
                              1e-13: about ten times the largest error measured against the CPU
                              oracle at that order). 0 = default 1e-13 (P = 39).
                              VOLPOT_ERR_UNSUPPORTED below 1e-13, and for layer-potential and
                              point plans at any P other than 39. */
  int32_t kchunk_leaf;     /* k-chunk of the dense near-field stages (dense_near = 1, layer
                              plans): 32 (default; 0) or 16 (shorter chunks, less LDS and fewer
                              registers: three blocks per compute unit instead of two). The
                              low-rank near field always takes 16. */
  int32_t dense_m2l;       /* 0 (default): the M2L stages (FARV and its transpose) apply each
                              translation in factored form, diag(d^-l) H diag((-1)^k d^-k)
                              with one real, offset-free core H shared by all 40 V-list offsets
                              (the translation formula of Sec. 4.2's box code, split), half the
                              matrix-core work of the dense form; the ln|d| a_0 term joins the
                              rank-one ln s terms. 1: dense 2q x 2q real matrices per offset.
                              Both agree to rounding (the tests compare them). */
  int32_t deterministic;   /* results are bitwise repeatable in every mode: each output has one
                              owner and a fixed summation order (the partial sums of a tile cut
                              between blocks are added in piece order). 0 (default): tiles may be
                              cut; the block that finishes a cut tile last, found by an atomic
                              arrival counter, adds its pieces. 1: no atomic operations at all:
                              every tile belongs to one block (split_min is taken as -1). The
                              two modes sum in different orders and agree to rounding. */
  int32_t dense_near;      /* 0 (default, volume plans): the adjacent-leaf tables other than a
                              leaf's own apply in low-rank form T_r = U_r V_r (Householder QR
                              with column pivoting of each 256 x 256 table, stopped after k_r =
                              64 columns, or 48 where that loses only rounding-level terms: the
                              corner and coarser neighbours): stages NEARC / NEARC48 form V_r f
                              for every such pair (64 values a pair in plan memory), the near
                              field then applies U_r to those and the self table to the leaf's
                              own data, about half the dense matrix-core work. 1: the dense
                              tables. The two agree to rounding (the tests compare them). */
} volpot_options;

/* Algorithmic work of one apply, from the plan's exact pair counts. Flops are 2 x the
 * non-zeros of every applied real matrix (zero padding of MFMA tiles not counted). */
typedef struct {
  int64_t n_leaves, n_boxes, n_trees;
  int32_t max_level, order, n_reals, n_stages;  /* order: the expansion order P; n_reals = 2 (P + 1) */
  int64_t pairs_near, pairs_v, pairs_w, pairs_x, n_m2m, n_l2l, n_s2m, n_l2t;
  double flops_total;       /* forward apply */
  double flops_adjoint;     /* adjoint apply (the same pairs, transposed) */
  double flops_kind[11];    /* per stage kind: 0 upward (S2M, M2M chain), 1 downward (M2L + S2L
                               for all levels, L2L chain), 2 near field, 3 L2T + M2T + log terms,
                               4 adjoint upward (L2T^T, L2L^T chain), 5 adjoint downward (M2L^T,
                               M2T^T, M2M^T chain), 6 adjoint near field, 7 S2M^T + S2L^T,
                               8 adjoint row sums (plans with leaves above level 2 only),
                               9 the low-rank near field's first stage (V_r f per pair), 10 its
                               transpose's (U_r^T ubar per pair). The low-rank near field folds
                               kinds 3 and 7 into kinds 2 and 6 (stages NEAR+LOCT, ANEAR+ALOCT). */
  int64_t launches_kind[11]; /* kernel launches per apply of each stage kind */
  double bytes_min;         /* mandatory HBM traffic: 16 B per unknown (f in, u out) */
  int64_t device_bytes;     /* device memory the plan holds (tables shared per device) */
  double flops_issued_kind[11]; /* matrix-core work the kernels issue per stage kind: every tile
                                  multiplies each of its relation tables by all of its slots,
                                  occupied or not (>= flops_kind) */
  /* layer-potential plans (volpot_layer_plan; zero otherwise) */
  int64_t n_layer_nodes;    /* curve quadrature nodes */
  int64_t n_source_leaves;  /* leaves holding at least one node */
  int64_t n_active_boxes;   /* boxes whose subtree holds nodes (the only multipole sources) */
  int64_t pairs_p2p;        /* (leaf node, curve node) pairs summed directly */
  int64_t pairs_p2l;        /* (box, curve node) pairs expanded directly into local expansions */
  /* plans with evaluation points (volpot_plan_points; zero otherwise) */
  int64_t n_points;         /* evaluation points */
  int64_t pairs_points;     /* (point, adjacent leaf) pairs, each a precomputed 3 x 256 moment block */
  int64_t pairs_lowrank;    /* adjacent-leaf pairs in low-rank form (0 with dense_near) */
} volpot_info;

/* Build a plan for one tree (Sec. 4.2.1: boxes {B_k}, order p; here p = 16 only).
 *   centres  host, n_leaves x 2 (x, y) leaf centres; must sit on their level's grid (of the
 *            root box the options give; a centre may be off it by 1e-6 of its box's width)
 *   levels   host, n_leaves leaf levels (0..29)
 *   opt      nullable; defaults as documented in volpot_options
 *   out      receives the plan; untouched on error
 * Returns VOLPOT_ERR_TREE / _UNBALANCED for invalid trees, _UNSUPPORTED for p != 16. */
int volpot_plan(const double* centres, const int32_t* levels, int64_t n_leaves, int32_t p,
                const volpot_options* opt, volpot_plan_t* out);

/* Plan for n_trees independent trees applied together (one launch per stage for all trees).
 *   tree_offsets  host, n_trees + 1 ascending offsets into centres/levels (first 0)
 * Each tree has its own root box (all of them the one the options give); data of tree t occupy leaves
 * [tree_offsets[t], tree_offsets[t+1]) of f and u. */
int volpot_plan_forest(int32_t n_trees, const int64_t* tree_offsets, const double* centres,
                       const int32_t* levels, int32_t p, const volpot_options* opt,
                       volpot_plan_t* out);

/* u = A f: the volume potential of the leaf data at all leaf nodes (eq. (vbulk) with the
 * sign -Lap u = f). f_dev, u_dev: device FP64 arrays [n_leaves][16][16]. */
int volpot_apply(volpot_plan_t plan, const double* f_dev, double* u_dev, void* hip_stream);

/* fbar = A^T ubar: the exact transpose of the discrete operator applied by volpot_apply
 * (the gradient of <ubar, A f> with respect to f). Same layout and stream rules. */
int volpot_apply_adjoint(volpot_plan_t plan, const double* ubar_dev, double* fbar_dev,
                         void* hip_stream);

/* Off-grid evaluation (the glue step of Sec. 4.4 needs v_bulk and its normal derivative on the
 * fictitious curve, away from the leaf nodes): a volume plan that can also evaluate
 *     u(x) = int_{Omega_B} G(x - y) f_h(y) dy  and  grad u(x)
 * at n_points fixed points x (host, n_points x 2, inside the root box [-1,1]^2). The box code's
 * own decomposition is used at each point: the local expansion of the leaf holding it, the
 * multipoles of that leaf's W list, and the integrals over its adjacent leaves, whose moments
 * against the leaf basis are computed at plan time (adaptive quadrature, a few milliseconds
 * per point on the host). A point on an edge between leaves belongs to the leaf on its
 * right / upper side. Returns VOLPOT_ERR_ARG for a point outside the root box; the tree errors
 * of volpot_plan otherwise. The plan is a full volume plan (volpot_apply and the adjoint work). */
int volpot_plan_points(const double* centres, const int32_t* levels, int64_t n_leaves, int32_t p,
                       int64_t n_points, const double* points, const volpot_options* opt, volpot_plan_t* out);

/* One forward apply (as volpot_apply: u_dev at the leaf nodes) that also writes u at the plan's
 * points to u_pts_dev (device, n_points) and, when grad_pts_dev is not NULL, its gradient
 * (device, n_points x 2: d/dx, d/dy). Asynchronous on the stream. */
int volpot_apply_points(volpot_plan_t plan, const double* f_dev, double* u_dev, double* u_pts_dev,
                        double* grad_pts_dev, void* hip_stream);

/* Glue layer potentials (Sec. 4.4): a plan that evaluates
 *
 *     V(x) = S[sigma](x) - D[tau](x)
 *          = -(1/2 pi) sum_j w_j [ sigma_j log|x - y_j| + tau_j n_j . (x - y_j) / |x - y_j|^2 ]
 *
 * (S, D the single- and double-layer potentials of the fundamental solution of -Lap on the
 * fictitious curve, discretised by quadrature nodes y_j with weights w_j and unit normals n_j)
 * at every leaf node of one tree, with the box code's far-field machinery: multipoles of the
 * leaves holding nodes, the same M2M / M2L / L2L / L2T / M2T translations, local expansions
 * from the nodes of X-list leaves, and direct sums over the nodes of adjacent leaves.
 *   centres, levels, n_leaves, p   the tree, as volpot_plan
 *   nodes    host, n_nodes x 2; every node must lie in the root box [-1,1]^2
 *   weights  host, n_nodes quadrature weights (arc length included)
 *   normals  host, n_nodes x 2 unit normals
 *   opt      nullable; host_only, use_graph, tile_box, split_min, table_cache and overlap apply
 * The plan copies the node geometry. Returns VOLPOT_ERR_ARG for a node outside the root box or
 * non-finite node data, the tree errors of volpot_plan otherwise. n_nodes may be 0 (V = 0).
 * volpot_apply and volpot_apply_adjoint reject a layer plan (VOLPOT_ERR_STATE); every other
 * call taking a plan works on it. */
int volpot_layer_plan(const double* centres, const int32_t* levels, int64_t n_leaves, int32_t p,
                      int64_t n_nodes, const double* nodes, const double* weights, const double* normals,
                      const volpot_options* opt, volpot_plan_t* out);

/* u = V at every leaf node, [n_leaves][16][16] as volpot_apply's output (overwritten).
 * sigma_dev, tau_dev: device FP64 densities at the nodes, in the order given to the plan.
 * A leaf node that coincides with a curve node gets a non-finite value. Asynchronous on the
 * stream; returns VOLPOT_ERR_STATE for a volume plan. */
int volpot_layer_apply(volpot_plan_t plan, const double* sigma_dev, const double* tau_dev, double* u_dev,
                       void* hip_stream);

/* Adaptive quadtree construction (Sec. 4.2.1, Alg. 2: the function-resolution criterion)
 * followed by the 2:1 balance over edges and corners, with the per-box work on the GPU. The
 * library hands out the nodes of the boxes to test; the caller samples f there (any way it
 * likes, e.g. a kernel of its own) and submits the samples; the library computes each box's
 * Chebyshev coefficients c_nm (n in y, m in x) and splits the boxes whose tail
 * max { |c_nm| : n >= p-2 or m >= p-2 } exceeds eps * scale; one level per round.
 *   p           16 only (VOLPOT_ERR_UNSUPPORTED otherwise)
 *   eps, scale  tolerance (> 0) and a global magnitude of f (>= 0), e.g. its maximum
 *   min_level   boxes above this level are split without samples (0..12)
 *   max_level   boxes at this level are leaves (min_level..29)
 * The builder allocates device memory for the round's nodes and tails (not for use inside
 * graph capture). */
typedef struct volpot_tree_s* volpot_tree_t;
int volpot_tree_create(int32_t p, double eps, double scale, int32_t min_level, int32_t max_level,
                       volpot_tree_t* out);
/* Number of boxes in the round (0 when the construction is finished). */
int volpot_tree_pending(volpot_tree_t tree, int64_t* n);
/* Writes the round's node coordinates to nodes_dev (device, caller-owned, [n][16][16][2] as
 * (x, y), the leaf-data layout) asynchronously on hip_stream. */
int volpot_tree_nodes(volpot_tree_t tree, double* nodes_dev, void* hip_stream);
/* values_dev: device [n][16][16] samples of f at the round's nodes (same stream). Decides every
 * box of the round (synchronises the stream). A non-finite sample splits its box (down to
 * max_level). */
int volpot_tree_submit(volpot_tree_t tree, const double* values_dev, void* hip_stream);
/* After the last round: the balanced leaves, ordered by level, then y, then x. *n receives their
 * number; centres (n x 2) and levels (n) are host arrays, each nullable (ask for n first).
 * VOLPOT_ERR_STATE while boxes are pending. The result is a valid input of volpot_plan. */
int volpot_tree_leaves(volpot_tree_t tree, int64_t* n, double* centres, int32_t* levels);
void volpot_tree_destroy(volpot_tree_t tree);

/* Strip solve (Sec. 4.3): Lap v = f in the strip between the boundary Gamma and the fictitious
 * curve Gamma~, v = 0 on both, by multidomain spectral collocation. Element k spans panel k of
 * Gamma and panel k of Gamma~ (the panels correspond one to one, in the same direction around the
 * closed curves); its nodes are the curvilinear tensor grid of second-kind Chebyshev points,
 * q along the panel (the panel's points interpolated from its Gauss-Legendre nodes) and n_r
 * across the strip (r = -1 on Gamma). The plan assembles the block-tridiagonal periodic system
 * on the host, inverts every element's block on the current device (batched, one launch), and
 * eliminates the rank-(n_r - 2) couplings and the periodic corner (Woodbury) on m x m pieces;
 * it synchronises the device and keeps the factors in device memory until destroy. The apply
 * solves on the GPU.
 *   n_panel        panels per curve (>= 3)
 *   n_gl           Gauss-Legendre nodes per panel (2..64)
 *   gamma, gamma_t host, n_panel x n_gl x 2: the nodes of each panel, in the panel's direction
 *   q, n_r         4..32 each, q * n_r <= 1024
 * Node order: element, then radial index i (0 on Gamma), then along-panel index j (fastest).
 * Returns VOLPOT_ERR_ARG for bad sizes, non-finite nodes, degenerate geometry (a zero-length
 * element edge between the curves, a singular element map) or a singular block;
 * VOLPOT_ERR_OOM / VOLPOT_ERR_HIP when device memory or a HIP call fails. */
typedef struct volpot_strip_s* volpot_strip_t;
int volpot_strip_plan(int32_t n_panel, int32_t n_gl, const double* gamma, const double* gamma_t, int32_t q,
                      int32_t n_r, volpot_strip_t* out);
/* The element nodes (host, n_panel x n_r x q x 2), where the caller samples f. */
int volpot_strip_nodes(volpot_strip_t strip, double* xy);
/* v_dev (device, n_panel x n_r x q) from f_dev (device, f at the nodes; values at the nodes on
 * Gamma, Gamma~ and the element edges are ignored). Asynchronous on the stream; one solve at a
 * time per plan (shared workspace). */
int volpot_strip_apply(volpot_strip_t strip, const double* f_dev, double* v_dev, void* hip_stream);
/* As volpot_strip_apply, for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the apply's work vectors live in a
 * static 1 MiB array of each device the library runs on (held until the process ends) instead of
 * the plan's memory, and the call allocates nothing. The plan must satisfy
 * (4 n_panel + 4) (n_r - 2) <= 131072 (e.g. 1,091 panels at n_r = 32); VOLPOT_ERR_ARG otherwise.
 * All calls on one device share that device's array: calls whose work overlaps on one device
 * (different streams, or threads) race and give wrong results; serialise them. Same results as
 * volpot_strip_apply, bit for bit. */
int volpot_strip_apply_noalloc(volpot_strip_t strip, const double* f_dev, double* v_dev, void* hip_stream);
void volpot_strip_destroy(volpot_strip_t strip);

/* Sizes and algorithmic flop/byte counts of the plan. */
int volpot_plan_info(volpot_plan_t plan, volpot_info* out);

/* Host-only check of a tree (tiling of the root, level grid, 2:1 balance over edges and
 * corners). On error *bad_index (nullable) receives the first offending leaf. */
int volpot_validate_tree(const double* centres, const int32_t* levels, int64_t n_leaves,
                         int32_t p, int64_t* bad_index);

/* The node convention: t[i] (p ascending first-kind Chebyshev points) and w[i], the weights
 * of the interpolatory rule on them (w_i = integral over [-1,1] of the i-th Lagrange basis). */
int volpot_nodes(int32_t p, double* t, double* w);

/* Release a plan (NULL is ignored). Work queued on it must have completed. */
void volpot_plan_destroy(volpot_plan_t plan);

/* Static text for a status code. */
const char* volpot_status_string(int status);

/* Timing hooks for measurement. enable: 0 off, 1 every stage kind, or bit (8 + k) set for each
 * stage kind k (numbered as in volpot_info.flops_kind) to be timed. Apply calls then record a
 * HIP event pair around every launch of those kinds on the stream that launch uses (the
 * caller's; with the overlap option the far-field chain's stream is the plan's helper stream);
 * volpot_stage_times synchronises those events and returns, per stage kind k, the summed
 * milliseconds ms[k] and launch counts n[k] since the last reset, then resets. Disabled by
 * default; not available with use_graph. */
int volpot_set_timing(volpot_plan_t plan, int32_t enable);
int volpot_stage_times(volpot_plan_t plan, double* ms, int64_t* launches, int32_t n_kinds);

/* Inspection: copy a host-side table of the plan (row-major) into out (n doubles).
 *   kind 0: near table of relation index (0..32, see volpot_near_relation), 256 x 256
 *   kind 1: S2M (2q x 256);   kind 2: L2T (256 x 2q), q = P + 1 of the plan's order
 *   kind 3: U_r (256 x 64) and kind 4: V_r (64 x 256) of relation index 1..32, the factors
 *           the low-rank near field applies (T_r ~ U_r V_r); a relation of rank 48 comes
 *           zero-padded (columns 48..63 of U_r, rows 48..63 of V_r)
 * Returns VOLPOT_ERR_ARG for an unknown kind/index or n too small. */
int volpot_plan_table(volpot_plan_t plan, int32_t kind, int32_t index, double* out, int64_t n);

/* Autotuner (for callers that apply one tree shape many times, e.g. batched forests): searches
 * the launch shapes tile_box 16|32|64, tile_leaf 32|64, kchunk_leaf 32|16 and tile_leaf_exp
 * 16|32|64 (these two with dense_near only), split_min 0|1|-1 and overlap 0|16|24|32|48 one knob
 * at a time from the defaults (the other fields, eps among them, are taken from base,
 * nullable), building a plan for each candidate (the defaults' and the current choice's are
 * kept for timing again) and timing one forward plus one adjoint apply on internal device
 * buffers after a warm-up (HIP events, private stream, best of 5); writes the fastest options
 * to *best and their time in milliseconds to *best_ms (nullable). A candidate must beat the
 * current choice by more than 1.5%, and the result must beat the defaults by as much when both
 * are timed again, so that differences within timing noise keep the defaults. With cache_path
 * (nullable) the result is looked up in, and appended to, that text file, keyed by a signature
 * of the trees' level histogram and sizes, of the expansion order that base's eps selects, of
 * base's dense_m2l and dense_near and of the device, so that a shape is timed once.
 * VOLPOT_ERR_UNSUPPORTED for an eps no order meets. Allocates (up to three plans at once) and
 * synchronises; not for use inside a timed region.
 * Arguments as volpot_plan_forest (a single tree: n_trees = 1, offsets {0, n_leaves}). */
int volpot_autotune(int32_t n_trees, const int64_t* tree_offsets, const double* centres,
                    const int32_t* levels, int32_t p, const volpot_options* base,
                    const char* cache_path, volpot_options* best, double* best_ms);

/* Measurement: the FP64 matrix-core rate this device sustains, the measured companion of the
 * published 78.6 TFLOP/s in roofline reports. Launches `blocks` workgroups of 256 threads on the
 * stream; every wave runs `iters` rounds of 8 independent v_mfma_f64_16x16x4f64 (2,048 flops
 * each) on register operands, so one launch does blocks * 4 * iters * 8 * 2048 flops; time it
 * with events on the same stream. Thread t of block k writes out_dev[256 k + t], the sum of its
 * accumulators: iters * 8 * sum over its 4 output rows i of sum_{c<4} A[i][c] B[c][j], with
 * lane l = 16 c + m holding A[m][c] = 1 + l / 1024 and B[c][m] = 1 - l / 1024 (out_dev holds
 * 256 blocks doubles, caller-owned). VOLPOT_ERR_ARG for blocks or iters <= 0 or a null out_dev. */
int volpot_peak_mfma(int32_t blocks, int32_t iters, double* out_dev, void* hip_stream);

/* One stage (one kernel launch) of an apply, for inspection and tuning. */
typedef struct {
  char name[24];           /* e.g. "NEAR", "M2M[5]", "AFARV" */
  int32_t kind;            /* stage kind, numbered as in volpot_info.flops_kind */
  int32_t rows, tile, kchunk; /* output rows per slot (2q or 256; the padded core's rows when
                              factored), slots per tile, k-chunk */
  int32_t helper;          /* 1: runs on the plan's helper stream */
  int64_t n_tiles, n_segments, n_blocks, n_split_tiles;
  double flops, flops_issued;
  int32_t inner;           /* inner dimension K of the stage's products (reals; complex terms
                              when factored); the largest one where segments differ (the
                              low-rank near field's K = 48 and 64) */
  int32_t factored;        /* 1: the factored M2L form (see volpot_options.dense_m2l) */
  int64_t n_chunks;        /* k-chunks over all segments (each segment's K / kchunk) */
} volpot_stage_info;

/* Number of stages of the forward (adjoint = 0) or adjoint (1) apply, in launch order. */
int volpot_plan_n_stages(volpot_plan_t plan, int32_t adjoint, int32_t* n);
/* Stage index (0 .. n-1) of the forward or adjoint apply. */
int volpot_plan_stage(volpot_plan_t plan, int32_t adjoint, int32_t index, volpot_stage_info* out);

/* Geometry of near relation r (0..32): offset (dx, dy) of the source leaf centre from the
 * target leaf centre in target half-widths, and rho = source / target half-width. */
int volpot_near_relation(int32_t r, double* dx, double* dy, double* rho);

#ifdef __cplusplus
}
#endif

#endif /* VOLPOT_H */
