// Device interface of the strip solve (strip.cpp, strip.hip, strip_factor.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace vp {

// Device data of the factored strip system (strip.cpp): n elements of B = q n_r unknowns,
// m = n_r - 2 interface rows per side.
struct StripDevice {
  int32_t n, q, B, m, Bi, chunk;  // elements, nodes along, nodes per element, m = n_r - 2, Bi = m q
  const double* EiT;  // n x Bi x Bi: interior block of E_k = D_k^-1, column c contiguous
  const double* W;    // n x 2m x Bi: [E_k[last column, :]; U~_{k-1} E_k] on the interior columns
  const double* F;    // n x m x m: E_k[last column, value rows]
  const double* G;    // n x m x m: U~_{k-1} E_k[:, value rows]
  const double* H;    // n x m x m: U~_{k-1} E_k[:, derivative rows] (k = 0: the corner term)
  const double* Pz;   // n x m x m: response of z_k to the corner values h_lo
  const double* Pt;   // (n + 1) x m x 2m: response of t_k to h
  const double* K;    // 2m x 2m: the Woodbury capacitance inverse of the periodic corner
  const double* rs;   // n x B: row scale of each PDE row (the right-hand side is f * rs)
  double* s;          // n x m work: E_k[last column, :] b_k
  double* w;          // n x m work: U~_{k-1} E_k b_k
  double* z;          // (n + 1) x m work: forward sweep
  double* t;          // (n + 1) x m work: backward sweep
  double* h;          // 2m work: corner values
};
// v (n x B) from the node samples f (n x B): Lap v = f inside, the boundary and interface rows zero
hipError_t launch_strip_solve(const StripDevice& d, const double* f, double* v, hipStream_t stream);

// Static work memory of the apply without allocation: (4 n + 4) m doubles are needed (s, w: n m;
// z, t: (n + 1) m; h: 2 m). strip_scratch gives its address on the current device (looked up once
// per device).
constexpr int64_t kStripScratchDoubles = int64_t(1) << 17;  // 1 MiB per device
hipError_t strip_scratch(double** out);

// Plan-time factorization on the GPU (strip_factor.hip).
constexpr int kPermInts = 72;  // count, 32 destination rows, 32 source rows (padded)
struct StripFactorDevice {
  int32_t n, N, Bi, m, q;  // elements, padded interior size (multiple of 16), Bi = m q, m, q
  int32_t nr, B;           // nodes across the strip, B = nr q nodes per element
  const double* met;       // n x 6 x B: xi_x, xi_y, eta_x, eta_y, x_xi, y_xi per node
  const double* nrm;       // n x 2: normal of the interface between element k and k + 1
  const double* Dq;        // q x q, row-major: differentiation along the panels
  const double* Dr;        // nr x nr: across the strip
  double* rowsc;           // n x Bi: scale of each interior row (1 for the value rows)
  double* rs;              // n x B: scale of the right-hand side of each row (the plan's)
  double* A;               // n x N x N: interior blocks, column-major (destroyed)
  int32_t* piv;            // n x N: the pivot row of each column
  int32_t* perm;           // n x kPermInts: the last panel's net row permutation
  int32_t* flag;           // n: 1 where a block is singular
  double* Ainv;            // n x N x N: the inverses, column-major
  double* U;               // n x m x Bi: U~_k (element k's derivative rows on element k + 1)
  double* R;               // n x m x Bi: R_k = U~_{k-1} A_k^-1
  double* pieces;          // n x 4 x m x m: A^-1[S, P], A^-1[S, V], R[:, P], R[:, V]
  const double* MG;        // n x m x m: the chain's M_k G_k^-1 (host)
  double* Q;               // n x m x Bi: MG_k R_k
  double* W;               // n x 2m x Bi: the apply's right-hand-side functionals
  double* EiT;             // n x Bi x Bi: the apply's interior blocks of E_k, column c contiguous
};
// stage 0: assembly, inverses, R and the pieces; stage 1 (after the host chain): Q, W and EiT
hipError_t launch_strip_factor(const StripFactorDevice& f, int stage, hipStream_t stream);

}  // namespace vp
