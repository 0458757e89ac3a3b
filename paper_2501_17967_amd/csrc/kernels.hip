// HIP kernels of the box code for gfx950 (CDNA4), FP64 throughout.
//
// One kernel template serves every stage: a grouped-relation GEMM. A workgroup owns a tile of
// NT output vectors ("slots") of M rows each and walks the relation segments present in the
// tile (sorted by relation id). For relation r it accumulates
//     C[:, slot] += A_r[:, k-chunk] * B[k-chunk, slot]
// with v_mfma_f64_16x16x4f64, where B gathers the NT source vectors by index. Both operands are
// staged through LDS in k-chunks of KC; the global loads of chunk c+1 are issued into registers
// before chunk c is multiplied, so memory latency overlaps the MFMA work. A_r is stored
// fragment-major, which makes every chunk of A one contiguous block (a straight coalesced
// copy) and every LDS fragment read a contiguous 512-byte wave access. A segment's metadata
// (table pointer, source family, this thread's source indices) is fetched once per segment.
//
// Each output vector has exactly one owner and a fixed relation order: no atomics, bitwise
// deterministic, identical whether a tree is applied alone or inside a forest.
//
// MFMA f64 16x16x4 operand layout (lane l, checked on gfx950):
//   A: A[l % 16][l / 16]   B: B[l / 16][l % 16]   D (4 regs r): D[4 r + l / 16][l % 16]
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace vp {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));  // native vector: keeps staging arrays in registers

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous range of
// tiles so neighbouring tiles (which share source leaves) share an L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
  const int q = G >> 3, r = G & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// Kernel-argument arrays indexed with a runtime value would be copied to scratch; pick with
// constant indices instead.
template <typename T>
__device__ __forceinline__ T pick4(const T (&a)[4], int i) {
  return i == 0 ? a[0] : (i == 1 ? a[1] : (i == 2 ? a[2] : a[3]));
}
template <typename T>
__device__ __forceinline__ T pick3(const T (&a)[3], int i) {
  return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]);
}

// Global-memory pointers: loads through them compile to global_load (vmcnt only), not flat
// loads, which would also count against the LDS wait counter and serialise the pipeline.
#define GLOBAL __attribute__((address_space(1)))
typedef const GLOBAL double* gdp;
typedef const GLOBAL d2* gd2p;
typedef const GLOBAL int32_t* gip;

// The loading side of a tile's walk over (segment, k-chunk) steps. Every relation of a stage has
// the same K, a multiple of KC, so every chunk is full. Thread tid owns the A pairs
// tid + q NTHR of each chunk and the B pairs idx = tid + q NTHR, i.e. slot t = idx / (KC/2) and
// k pair kp = idx % (KC/2); the source indices of a segment are fetched once per segment.
template <int M, int NT, int NTHR, int KC>
struct Loader {
  static constexpr int A_V2 = M * KC / 2;
  static constexpr int A_PER = (A_V2 + NTHR - 1) / NTHR;
  static constexpr int B_V2 = NT * KC / 2;
  static constexpr int B_PER = (B_V2 + NTHR - 1) / NTHR;
  static constexpr int HALF = KC / 2;
  int s, k0;              // step being loaded
  gdp A;                  // table of segment s
  int K;
  gdp base;               // source family of segment s
  int stride;
  int si[B_PER];          // this thread's source index per B pair (-1: none)
  d2 ra[A_PER], rb[B_PER];

  __device__ __forceinline__ void segment(const GrgParams& p, int tid) {
    gip src = (gip)(p.seg_src + (size_t)s * NT);
#pragma unroll
    for (int q = 0; q < B_PER; ++q) {
      const int t = (tid + q * NTHR) / HALF;
      si[q] = t < NT ? src[t] : -1;
    }
    const SegDesc sd = p.segs[s];
    A = (gdp)sd.A;
    K = sd.K;
    base = (gdp)pick4(p.fam_base, sd.fam) + sd.k_off;
    stride = pick4(p.fam_stride, sd.fam);
  }
  __device__ __forceinline__ void load(int tid) {
    gd2p A2 = (gd2p)(A + (size_t)k0 * M);
#pragma unroll
    for (int q = 0; q < A_PER; ++q) {
      const int idx = tid + q * NTHR;
      ra[q] = A2[(A_V2 % NTHR == 0 || idx < A_V2) ? idx : 0];
    }
#pragma unroll
    for (int q = 0; q < B_PER; ++q) {
      const int kp = (tid + q * NTHR) % HALF;
      const bool ok = si[q] >= 0;
      const d2 v = *(gd2p)(base + (size_t)(ok ? si[q] : 0) * stride + k0 + 2 * kp);
      rb[q] = ok ? v : d2{0.0, 0.0};
    }
  }
  template <int LDB>
  __device__ __forceinline__ void store(int tid, double* As, double* Bs) const {
    d2* As2 = reinterpret_cast<d2*>(As);
#pragma unroll
    for (int q = 0; q < A_PER; ++q) {
      const int idx = tid + q * NTHR;
      if (A_V2 % NTHR == 0 || idx < A_V2) As2[idx] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < B_PER; ++q) {
      const int idx = tid + q * NTHR;
      const int t = idx / HALF, kp = idx % HALF;
      if (B_V2 % NTHR == 0 || t < NT) {
        Bs[t * LDB + 2 * kp] = rb[q].x;
        Bs[t * LDB + 2 * kp + 1] = rb[q].y;
      }
    }
  }
  // advance to the next k-chunk (the schedule guarantees it exists)
  __device__ __forceinline__ void advance(const GrgParams& p, int tid) {
    k0 += KC;
    if (k0 >= K) {
      ++s;
      k0 = 0;
      segment(p, tid);
    }
  }
};

// Column of part h (0 real, 1 imaginary) of slot t in a factored tile: each group of 16 slots
// takes 32 columns, the real parts first, so that one wave's two column fragments hold both
// parts of the same 16 slots in the same lanes.
__device__ __forceinline__ int cx_col(int t, int h) { return (t >> 4) * 32 + h * 16 + (t & 15); }

// The loading side of a factored M2L stage: one chunk is one whole segment, the Q complex terms
// of NT sources. Thread tid owns term k = tid % Q of the slots t = tid / Q + G q (G = NTHR / Q
// thread groups; threads past G Q idle here), so it needs one input weight w_in[k] per segment.
// Each source term is scaled by its complex weight on the way into LDS, its parts to columns
// cx_col(t, 0) and cx_col(t, 1); thread tid < MP also stages the output weight w_out[tid] of
// the segment.
template <int NT, int NTHR, int Q, int MP>
struct LoaderCX {
  static constexpr int G = NTHR / Q;
  static constexpr int B_PER = (NT + G - 1) / G;
  static_assert(G >= 1 && NTHR >= MP, "factored loader needs a thread per term and per output row");
  int s;
  gdp base;
  int stride;
  int si[B_PER];  // source index per owned slot (-1: none)
  d2 rb[B_PER], rw, ro;

  __device__ __forceinline__ void segment(const GrgParams& p, int tid) {
    gip src = (gip)(p.seg_src + (size_t)s * NT);
    const int g = tid / Q;
#pragma unroll
    for (int q = 0; q < B_PER; ++q) {
      const int t = g + G * q;
      si[q] = (g < G && t < NT) ? src[t] : -1;
    }
    const SegDesc sd = p.segs[s];
    base = (gdp)pick4(p.fam_base, sd.fam);
    stride = pick4(p.fam_stride, sd.fam);
    const int k = tid % Q;
    rw = ((gd2p)sd.w_in)[k];
    ro = ((gd2p)sd.w_out)[tid < MP ? tid : 0];
  }
  __device__ __forceinline__ void load(int tid) {
    const int k = tid % Q;
#pragma unroll
    for (int q = 0; q < B_PER; ++q) {
      const bool ok = si[q] >= 0;
      const d2 v = *(gd2p)(base + (size_t)(ok ? si[q] : 0) * stride + 2 * k);
      rb[q] = ok ? v : d2{0.0, 0.0};
    }
  }
  template <int LDB>
  __device__ __forceinline__ void store(int tid, double* Bs, double* Ws) const {
    const int k = tid % Q, g = tid / Q;
    if (g < G) {
#pragma unroll
      for (int q = 0; q < B_PER; ++q) {
        const int t = g + G * q;
        if (NT % G == 0 || t < NT) {
          const d2 v = rb[q];
          Bs[cx_col(t, 0) * LDB + k] = v.x * rw.x - v.y * rw.y;
          Bs[cx_col(t, 1) * LDB + k] = v.x * rw.y + v.y * rw.x;
        }
      }
    }
    if (tid < MP) reinterpret_cast<d2*>(Ws)[tid] = ro;
  }
  __device__ __forceinline__ void advance(const GrgParams& p, int tid) {
    ++s;
    segment(p, tid);
  }
};

// One k-step (4 values of k) of the tile product for one wave: MT x NTT MFMA fragments.
template <int MT, int NTT, int M, int LDB>
__device__ __forceinline__ void mfma_step(const double* __restrict__ Aw, const double* __restrict__ Bw, int kk,
                                          d4 (&acc)[MT][NTT]) {
  double a[MT], b[NTT];
#pragma unroll
  for (int i = 0; i < MT; ++i) a[i] = Aw[(kk * (M / 16) + i) * 64];
#pragma unroll
  for (int j = 0; j < NTT; ++j) b[j] = Bw[j * 16 * LDB + kk * 4];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NTT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
}

// One k-chunk of the tile product for one wave, with the operands of k-step kk + 1 read from
// LDS before the products of step kk issue, so that the LDS latency hides behind them. The
// scheduling barriers keep that order (left to itself, the compiler sinks the reads below the
// products to reuse the operand registers, and each step then waits for its reads).
template <int MT, int NTT, int M, int LDB, int KC>
__device__ __forceinline__ void mfma_chunk(const double* __restrict__ Aw, const double* __restrict__ Bw,
                                           d4 (&acc)[MT][NTT]) {
  constexpr int NK = KC / 4;
  double a[2][MT], b[2][NTT];
#pragma unroll
  for (int i = 0; i < MT; ++i) a[0][i] = Aw[i * 64];
#pragma unroll
  for (int j = 0; j < NTT; ++j) b[0][j] = Bw[j * 16 * LDB];
#pragma unroll
  for (int kk = 0; kk < NK; ++kk) {
    const int cur = kk & 1;
    if (kk + 1 < NK) {
#pragma unroll
      for (int i = 0; i < MT; ++i) a[cur ^ 1][i] = Aw[((kk + 1) * (M / 16) + i) * 64];
#pragma unroll
      for (int j = 0; j < NTT; ++j) b[cur ^ 1][j] = Bw[j * 16 * LDB + (kk + 1) * 4];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NTT; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cur][i], b[cur][j], acc[i][j], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Output of one tile: rank-one terms, optional s^2 scaling, overwrite or accumulate.
// The rank-one sum of each slot is spread over NTHR / NT threads, each taking every
// (NTHR / NT)-th entry four at a time (independent loads in flight), and the per-thread sums
// are added in thread order: a fixed order, so the result is repeatable.
// Indices the epilogue of a tile needs, loaded when its piece starts so that their latency
// hides behind the piece's products.
// In a factored stage column c of the tile is part (c / 16) % 2 (real, imaginary) of slot
// (c / 32) 16 + c % 16 (the inverse of cx_col).
__device__ __forceinline__ int cx_slot(int col) { return (col >> 5) * 16 + (col & 15); }

template <int NTT, int NT, int NTHR, bool CX>
struct EpiIdx {
  int tgt[NTT];
  double sc[NTT];
  int e0, e1;
  __device__ __forceinline__ void load(const GrgParams& p, int tile, int tid, int lane, int wn) {
#pragma unroll
    for (int j = 0; j < NTT; ++j) {
      const int col = (wn * NTT + j) * 16 + (lane & 15);
      tgt[j] = p.tile_tgt[tile * NT + (CX ? cx_slot(col) : col)];
    }
    const int ti = tile * NT + tid / (NTHR / NT);
    e0 = p.r1_ptr[ti];
    e1 = p.r1_ptr[ti + 1];
#pragma unroll
    for (int j = 0; j < NTT; ++j) sc[j] = (p.out_scaled && tgt[j] >= 0) ? p.leaf_s2[tgt[j]] : 1.0;
  }
};

// Factored stages (CX) have NT slots in 2 NT columns and write only the QV complex rows of
// the padded core: reals 2 l and 2 l + 1 of each slot's expansion.
template <int MT, int NTT, int WM, int NT, int NTHR, bool CX, int QV>
__device__ __forceinline__ void tile_epilogue(const GrgParams& p, const EpiIdx<NTT, NT, NTHR, CX>& ix,
                                              const d4 (&acc)[MT][NTT], double* r1s, double* r1p, int tid, int lane,
                                              int wm, int wn) {
  constexpr int TPS = NTHR / NT;
  static_assert(TPS >= 1 && NTHR % NT == 0, "threads per slot");
  {
    const int e1 = ix.e1;
    double c = 0.0;
    for (int e = ix.e0 + tid % TPS; e < e1; e += 4 * TPS) {
      int idx[4], fm[4];
      double cf[4], v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int eq = e + q * TPS < e1 ? e + q * TPS : e;
        idx[q] = p.r1_idx[eq];
        fm[q] = p.r1_fam[eq];
        cf[q] = e + q * TPS < e1 ? p.r1_coef[eq] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = ((gdp)pick3(p.r1_base, fm[q]))[(size_t)idx[q] * pick3(p.r1_stride, fm[q])];
#pragma unroll
      for (int q = 0; q < 4; ++q) c += cf[q] * v[q];
    }
    r1p[tid] = c;
  }
  __syncthreads();
  if (tid < NT) {
    double c = r1p[tid * TPS];
    for (int q = 1; q < TPS; ++q) c += r1p[tid * TPS + q];
    r1s[tid] = c;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NTT; ++j) {
    const int col = (wn * NTT + j) * 16 + (lane & 15);
    const int slot = CX ? cx_slot(col) : col;
    const int part = CX ? (col >> 4) & 1 : 0;
    const int tgt = ix.tgt[j];
    if (tgt < 0) continue;
    const double sc = ix.sc[j];
    const double r1 = r1s[slot];
    double* __restrict__ o = p.out + (size_t)tgt * p.out_stride;
    // output index of accumulator row `row` (-1: a padding row of a factored stage)
    auto index = [&](int row) { return CX ? (row < QV ? 2 * row + part : -1) : row; };
    double prev[MT][4];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) prev[i][r] = 0.0;
    if (p.accumulate) {
      const double* __restrict__ a = (p.acc_src ? p.acc_src : p.out) + (size_t)tgt * p.out_stride;
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int x = index((wm * MT + i) * 16 + 4 * r + (lane >> 4));
          if (x >= 0) prev[i][r] = a[x];
        }
    }
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = index((wm * MT + i) * 16 + 4 * r + (lane >> 4));
        if (x < 0) continue;
        double v = acc[i][j][r];
        if (p.r1_all_rows || x == 0) v += r1;
        o[x] = v * sc + prev[i][r];
      }
  }
}

// Persistent, balanced launch: block b runs the pieces the plan gave it. A piece that is a
// whole tile writes the tile's output directly. A piece of a split tile stores its partial sum,
// then counts itself in on the tile's counter; the block that arrives last adds the partials
// in piece order (so the result does not depend on arrival order), writes the output and
// re-arms the counter. No block ever waits for another.
// The near-field instantiation (256 rows, 32 slots, 4 waves) is held to two blocks per compute
// unit (256 registers per lane): the other block works while this one waits at a barrier or
// for memory. Its k-chunk-16 form, which also runs the leaf stages that read expansions
// (K = 64 or 80), is held to three (168 registers): those stages are latency-bound, and the
// third block took 7% off them. The expansion-row instantiations of four 16-slot waves (up to
// 64 rows) are held to four blocks (128 registers, no spills): their tiles are short (one
// segment of K = 256 in eight chunks), and the compiler's own choice, three blocks with the
// accumulators in extra registers, left the pair stages 15% slower. The other
// instantiations keep the compiler's own choice.
// The factored M2L instantiations ask for three waves per SIMD (two for q = 40, whose
// accumulators are half as large again); the one with waves of 32 slots is held to three
// blocks (164 registers, no spills; the compiler's choice, 176, left two).
template <int MT, int NTT, int WM, int WN, int KC, bool CX>
constexpr int min_blocks() {
  if (!CX && WM == 1 && WN == 4 && NTT == 1 && MT <= 4) return 4;
  if (CX && NTT == 4) return 3;
  return (!CX && MT == 4 && NTT == 2 && WM == 4 && WN == 1) ? (KC == 32 ? 2 : KC == 16 ? 3 : 1) : 1;
}
template <int KC, bool CX>
constexpr int waves_per_simd() { return CX ? (KC == 40 ? 2 : 3) : 1; }

// Factored M2L (CX): the tile's columns are the real and imaginary parts of NT = NCOL / 2 slots,
// the table is the offset-free core (M padded rows, K = KC complex terms), held in LDS for the
// whole launch. Each chunk is one whole segment (one offset): its sources are scaled by the
// offset's input diagonal while staged, multiplied by the core into a fresh accumulator, and the
// product is scaled by the offset's output diagonal (a complex multiply across each lane pair)
// as it is added to the tile's sum.
template <int MT, int NTT, int WM, int WN, int KC, bool CX>
__global__ void __launch_bounds__(64 * WM * WN, (min_blocks<MT, NTT, WM, WN, KC, CX>()))
__attribute__((amdgpu_waves_per_eu(waves_per_simd<KC, CX>()))) grg_kernel(const GrgParams p) {
  constexpr int M = 16 * MT * WM;
  constexpr int NCOL = 16 * NTT * WN;
  constexpr int NT = CX ? NCOL / 2 : NCOL;  // slots
  constexpr int NTHR = 64 * WM * WN;
  constexpr int LDB = KC + 1;  // odd row stride: conflict-free B fragment reads
  constexpr int WPART = MT * NTT * 256;  // partial-sum doubles per wave
  __shared__ double As[M * KC];
  __shared__ double Bs[NCOL * LDB];
  __shared__ double Ws[CX ? 2 * M : 2];
  __shared__ double r1s[NT];
  __shared__ double r1p[NTHR];
  __shared__ int last_s;

  const int blk = xcd_tile(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const double* __restrict__ Aw = As + (wm * MT) * 64 + lane;
  const double* __restrict__ Bw = Bs + ((wn * NTT) * 16 + (lane & 15)) * LDB + (lane >> 4);

  const int pc0 = p.blk_ptr[blk], pc1 = p.blk_ptr[blk + 1];
  if (CX && pc0 < pc1) {  // the core, once (made visible by the first piece's barrier)
    gd2p A2 = (gd2p)p.cx_core;
    d2* As2 = reinterpret_cast<d2*>(As);
    for (int i = tid; i < M * KC / 2; i += NTHR) As2[i] = A2[i];
  }
  for (int pc = pc0; pc < pc1; ++pc) {
    const PieceDesc P = p.pieces[pc];
    EpiIdx<NTT, NT, NTHR, CX> ix;
    ix.load(p, P.tile, tid, lane, wn);
    d4 acc[MT][NTT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NTT; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();  // the previous piece no longer reads LDS

    if constexpr (CX) {
     if (P.n_chunks > 0) {
      LoaderCX<NT, NTHR, KC, M> L;
      L.s = P.seg;
      L.segment(p, tid);
      L.load(tid);
      L.template store<LDB>(tid, Bs, Ws);
      __syncthreads();
      const d2* __restrict__ W2 = reinterpret_cast<const d2*>(Ws);
      static_assert(!CX || NTT % 2 == 0, "a factored wave holds both parts of its slots");
      for (int left = P.n_chunks;;) {
        const bool more = --left > 0;
        if (more) {  // next segment in flight while this one is multiplied
          L.advance(p, tid);
          L.load(tid);
        }
        d4 part[MT][NTT];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
          for (int j = 0; j < NTT; ++j) part[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        mfma_chunk<MT, NTT, M, LDB, KC>(Aw, Bw, part);
        // acc += w_out[l] * part, complex: fragments 2j and 2j + 1 hold the real and the
        // imaginary part of (l, slot) in the same lane
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const d2 w = W2[(wm * MT + i) * 16 + 4 * r + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < NTT; j += 2) {
              const double re = part[i][j][r], im = part[i][j + 1][r];
              acc[i][j][r] = fma(w.x, re, fma(-w.y, im, acc[i][j][r]));
              acc[i][j + 1][r] = fma(w.x, im, fma(w.y, re, acc[i][j + 1][r]));
            }
          }
        if (!more) break;
        __syncthreads();  // every wave is done reading the segment and its weights
        L.template store<LDB>(tid, Bs, Ws);
        __syncthreads();  // the next segment is visible
      }
     }
    } else if (P.n_chunks > 0) {
      Loader<M, NT, NTHR, KC> L;
      L.s = P.seg;
      L.k0 = P.k0;
      L.segment(p, tid);
      L.load(tid);
      L.template store<LDB>(tid, As, Bs);
      __syncthreads();
      for (int left = P.n_chunks;;) {
        const bool more = --left > 0;
        if (more) {  // next chunk in flight while this one is multiplied
          L.advance(p, tid);
          L.load(tid);
        }
        mfma_chunk<MT, NTT, M, LDB, KC>(Aw, Bw, acc);
        if (!more) break;
        __syncthreads();  // every wave is done reading the chunk
        L.template store<LDB>(tid, As, Bs);
        __syncthreads();  // the next chunk is visible
      }
    }

    if (P.slot >= 0) {  // a piece of a split tile
      // Partial sums go through device-coherent stores and loads (agent scope), so the hand-off
      // needs no device-wide cache write-back or invalidate, which would also evict every other
      // block's table lines: the stores are complete (waitcnt) before the block counts itself
      // in, and the last block reads the partial sums only after its count has returned. The
      // ordering is kept by the hardware's in-order completion at these points (waitcnt, then
      // the barrier); compiler-only fences keep the compiler from moving any of the atomics
      // across them. An agent-scope acquire on the counter would invalidate the L2 of the block's
      // XCD (every other block's table lines with it).
      double* __restrict__ mine = p.partial + (size_t)P.slot * (M * NCOL) + wave * WPART + lane;
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NTT; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            __hip_atomic_store(mine + ((i * NTT + j) * 4 + r) * 64, acc[i][j][r], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (tid == 0)
        last_s = __hip_atomic_fetch_add(p.tile_count + P.tile, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                 P.n_pieces - 1;
      __syncthreads();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (!last_s) continue;
      for (int q = 0; q < P.n_pieces; ++q) {
        const double* __restrict__ part = p.partial + (size_t)(P.slot0 + q) * (M * NCOL) + wave * WPART + lane;
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
          for (int j = 0; j < NTT; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const double v = __hip_atomic_load(part + ((i * NTT + j) * 4 + r) * 64, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
              acc[i][j][r] = q == 0 ? v : acc[i][j][r] + v;
            }
      }
      if (tid == 0) __hip_atomic_store(p.tile_count + P.tile, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    tile_epilogue<MT, NTT, WM, NT, NTHR, CX, KC>(p, ix, acc, r1s, r1p, tid, lane, wm, wn);
  }
}

// out[leaf][k] = s2[leaf] * x[leaf][k]  (the s^2 Jacobian of each source leaf, applied once)
__global__ void prescale_kernel(const double* __restrict__ x, const double* __restrict__ s2, double* __restrict__ out,
                                int64_t n_leaves) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one double pair per thread
  if (i >= n_leaves * 128) return;
  const d2 v = reinterpret_cast<const d2*>(x)[i];
  const double s = s2[i >> 7];
  reinterpret_cast<d2*>(out)[i] = v * s;
}

__global__ void rowsum_kernel(const double* __restrict__ x, double* __restrict__ out, int64_t n) {
  const int64_t leaf = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (leaf >= n) return;
  const double* xl = x + leaf * 256;
  double s = xl[lane] + xl[lane + 64] + xl[lane + 128] + xl[lane + 192];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) out[leaf] = s;
}

// Every (M, NT, KC) instantiation: MT, NTT, WM, WN, KC, threads
#define VP_CONFIGS(X)                                                                            \
  X(256, 32, 32, 4, 2, 4, 1, 256) X(256, 64, 32, 4, 2, 4, 2, 512) X(256, 16, 16, 4, 1, 4, 1, 256) \
  X(256, 32, 16, 4, 2, 4, 1, 256) X(256, 64, 16, 4, 2, 4, 2, 512)                                 \
  X(80, 64, 40, 5, 1, 1, 4, 256) X(80, 32, 40, 5, 1, 1, 2, 128) X(80, 16, 40, 5, 1, 1, 1, 64)     \
  X(80, 64, 32, 5, 1, 1, 4, 256) X(80, 32, 32, 5, 1, 1, 2, 128) X(80, 16, 32, 5, 1, 1, 1, 64)     \
  X(64, 64, 16, 4, 1, 1, 4, 256) X(64, 32, 16, 4, 1, 1, 2, 128) X(64, 16, 16, 4, 1, 1, 1, 64)     \
  X(64, 64, 32, 4, 1, 1, 4, 256) X(64, 32, 32, 4, 1, 1, 2, 128) X(64, 16, 32, 4, 1, 1, 1, 64)     \
  X(48, 64, 16, 3, 1, 1, 4, 256) X(48, 32, 16, 3, 1, 1, 2, 128) X(48, 16, 16, 3, 1, 1, 1, 64)     \
  X(48, 64, 32, 3, 1, 1, 4, 256) X(48, 32, 32, 3, 1, 1, 2, 128) X(48, 16, 32, 3, 1, 1, 1, 64)     \
  X(32, 64, 16, 2, 1, 1, 4, 256) X(32, 32, 16, 2, 1, 1, 2, 128) X(32, 16, 16, 2, 1, 1, 1, 64)     \
  X(32, 64, 32, 2, 1, 1, 4, 256) X(32, 32, 32, 2, 1, 1, 2, 128) X(32, 16, 32, 2, 1, 1, 1, 64)

// Factored M2L instantiations: padded core rows, slots, complex terms q (= k-chunk); MT, NTT, WM,
// WN, threads (2 NT columns in 16-wide fragments, an even number per wave). At q = 32 the rows
// split over two waves (16 rows each): with 32 slots (one real and one imaginary fragment per
// wave, 114 registers, four blocks per compute unit) the order-31 M2L of the 256-tree forest
// took 3% less time than with 32-row waves (192 registers, two blocks); with 64 slots (waves of
// 32 slots, four fragments, three blocks) 3% less again, which the plan uses at q = 32.
#define VP_CONFIGS_CX(X)                                                                          \
  X(48, 16, 40, 3, 2, 1, 1, 64) X(48, 32, 40, 3, 2, 1, 2, 128) X(48, 64, 40, 3, 2, 1, 4, 256)     \
  X(32, 16, 32, 2, 2, 1, 1, 64) X(32, 32, 32, 1, 2, 2, 2, 256) X(32, 64, 32, 1, 4, 2, 2, 256)     \
  X(32, 16, 24, 2, 2, 1, 1, 64) X(32, 32, 24, 2, 2, 1, 2, 128) X(32, 64, 24, 2, 2, 1, 4, 256)     \
  X(16, 16, 16, 1, 2, 1, 1, 64) X(16, 32, 16, 1, 2, 1, 2, 128) X(16, 64, 16, 1, 2, 1, 4, 256)

hipError_t launch_grg(int M, int NT, int KC, bool factored, const GrgParams& p, hipStream_t stream) {
  if (p.n_blocks <= 0) return hipSuccess;
  dim3 grid(p.n_blocks);
#define VP_LAUNCH(m, nt, kc, MT, NTT, WM, WN, THR)                                                  \
  if (!factored && M == m && NT == nt && KC == kc) {                                              \
    hipLaunchKernelGGL((grg_kernel<MT, NTT, WM, WN, kc, false>), grid, dim3(THR), 0, stream, p);   \
    return hipGetLastError();                                                                     \
  }
  VP_CONFIGS(VP_LAUNCH)
#undef VP_LAUNCH
#define VP_LAUNCH_CX(m, nt, kc, MT, NTT, WM, WN, THR)                                               \
  if (factored && M == m && NT == nt && KC == kc) {                                               \
    hipLaunchKernelGGL((grg_kernel<MT, NTT, WM, WN, kc, true>), grid, dim3(THR), 0, stream, p);    \
    return hipGetLastError();                                                                     \
  }
  VP_CONFIGS_CX(VP_LAUNCH_CX)
#undef VP_LAUNCH_CX
  return hipErrorInvalidValue;
}

int grg_resident_blocks(int M, int NT, int KC, bool factored) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
#define VP_OCC(m, nt, kc, MT, NTT, WM, WN, THR, CXV)                                                \
  if (factored == CXV && M == m && NT == nt && KC == kc) {                                        \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(                                             \
            &per_cu, reinterpret_cast<const void*>(&grg_kernel<MT, NTT, WM, WN, kc, CXV>), THR, 0) != \
        hipSuccess)                                                                               \
      return 0;                                                                                   \
    return per_cu * cus;                                                                          \
  }
#define VP_OCC_D(m, nt, kc, MT, NTT, WM, WN, THR) VP_OCC(m, nt, kc, MT, NTT, WM, WN, THR, false)
#define VP_OCC_C(m, nt, kc, MT, NTT, WM, WN, THR) VP_OCC(m, nt, kc, MT, NTT, WM, WN, THR, true)
  VP_CONFIGS(VP_OCC_D)
  VP_CONFIGS_CX(VP_OCC_C)
#undef VP_OCC_C
#undef VP_OCC_D
#undef VP_OCC
  return 0;
}

hipError_t launch_prescale(const double* x, const double* s2, double* out, int64_t n_leaves, hipStream_t stream) {
  if (n_leaves <= 0) return hipSuccess;
  const int64_t n = n_leaves * 128;
  dim3 grid((unsigned)((n + 255) / 256));
  hipLaunchKernelGGL(prescale_kernel, grid, dim3(256), 0, stream, x, s2, out, n_leaves);
  return hipGetLastError();
}

hipError_t launch_rowsum(const double* x, double* usum, int64_t n_leaves, hipStream_t stream) {
  if (n_leaves <= 0) return hipSuccess;
  dim3 grid((unsigned)((n_leaves + 3) / 4));
  hipLaunchKernelGGL(rowsum_kernel, grid, dim3(256), 0, stream, x, usum, n_leaves);
  return hipGetLastError();
}

}  // namespace vp
