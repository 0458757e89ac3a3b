// HIP kernel of the point moments: for an off-grid point x and an adjacent leaf b (half-width s,
// x at xi = (x - c_b) / s in b's reference square), the weights of the leaf's 256 values in
// int_{B_b} G(x - y) f(y) dy and in its gradient. With G = -(1/2pi) ln|x - y|:
//   int_{B_b} G(x - y) l_k((y - c_b) / s) dy = s^2 (-1/2pi) (ln s W_k + I_k(xi)),
//   I_k(xi) = int_{[-1,1]^2} ln|xi - eta| l_k(eta) d eta,   gradient s (-1/2pi) grad_xi I_k.
// One workgroup per pair, thread t = 16 j + i for the basis function l_k = l_i(eta_1) l_j(eta_2).
// The reference square is refined towards xi as a quadtree, level by level: a square at
// distance >= its side from xi is accepted and takes a 24 x 24 tensor Gauss rule (the kernels
// are analytic on it); a square of half-width <= 1/32 whose closure holds xi is split into four
// polar-Duffy triangles with apex xi (a 16-point rule with a logarithmic weight in the radial
// variable; 12-point panels along the far edge, bisected until the edge parameter of xi's
// projection is far enough in the Bernstein-ellipse sense). Thread 0 sorts each level's squares;
// the threads contract the accepted ones with the basis in LDS as each level is sorted, then the
// triangles, in a fixed order. The flag of a pair is set only if a list capacity were exceeded.
#include <hip/hip_runtime.h>

#include "moments.hpp"

namespace vp {

namespace {

constexpr int kMT = 256;
constexpr int kNQ = 24;
// List capacities. None can be reached, so the flag the kernel writes stays 0:
//  * a square is refined only while its distance to xi is below its side 2h, so the refined
//    squares of one level lie in the disc of radius (2 + sqrt 2) h about xi and number at most
//    pi (3.42 h)^2 / (2h)^2 < 10 (18 for a loose count): a level has at most 4 * 18 = 72 squares,
//    of which at most 72 are accepted;
//  * at most 4 squares of one level hold xi (xi at their shared corner), and holding squares are
//    not refined further;
//  * the panel bisection of a triangle edge stops at half-length 1e-12 (depth <= 39); on each
//    depth at most 3 panels lie within 2.125 half-lengths of xi's projection (the rho = 4
//    Bernstein ellipse), so at most 6 are examined and 3 refined per depth: <= 3 * 39 + 6 panels,
//    and the depth-first stack holds at most depth + 2 entries.
constexpr int kMaxAcc = 256;   // accepted squares of one level
constexpr int kMaxLvl = 256;   // squares refined on one level
constexpr int kMaxHold = 16;   // squares of half-width <= 1/32 holding xi
constexpr int kMaxPanel = 160; // panels of one Duffy triangle
constexpr double kInv2Pi = 0.15915494309189533576888376337251436;

// barycentric Lagrange values of the 16 leaf nodes at x
__device__ void lagrange16(const MomentRules& R, double x, double* L) {
  int hit = -1;
  for (int a = 0; a < 16; ++a)
    if (x == R.t[a]) hit = a;
  if (hit >= 0) {
    for (int a = 0; a < 16; ++a) L[a] = a == hit ? 1.0 : 0.0;
    return;
  }
  double s = 0.0;
  for (int a = 0; a < 16; ++a) {
    L[a] = R.lam[a] / (x - R.t[a]);
    s += L[a];
  }
  const double inv = 1.0 / s;
  for (int a = 0; a < 16; ++a) L[a] *= inv;
}

// principal square root of a + i b
__device__ __forceinline__ void csqrt_(double a, double b, double& re, double& im) {
  const double r = hypot(a, b);
  re = sqrt(0.5 * (r + a));
  im = copysign(sqrt(0.5 * fmax(r - a, 0.0)), b);
}

// the parameter of the Bernstein ellipse of [c - hl, c + hl] through the complex point z
__device__ double bernstein_rho(double zr, double zi, double c, double hl) {
  const double wr = (zr - c) / hl, wi = zi / hl;
  double ar, ai, br, bi;
  csqrt_(wr - 1.0, wi, ar, ai);
  csqrt_(wr + 1.0, wi, br, bi);
  const double sr = ar * br - ai * bi, si = ar * bi + ai * br;
  return fmax(hypot(wr + sr, wi + si), hypot(wr - sr, wi - si));
}

__global__ void __launch_bounds__(kMT)
    point_moments_kernel(MomentRules R, const double* __restrict__ pairs, double* __restrict__ mom,
                         int32_t* __restrict__ flag) {
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x, ii = tid & 15, jj = tid >> 4;
  const double x0 = pairs[3 * e], y0 = pairs[3 * e + 1], s = pairs[3 * e + 2];
  __shared__ double sq[kMaxAcc][2];
  __shared__ double hold[kMaxHold][3];
  __shared__ double lvl[2][kMaxLvl][2];
  __shared__ double pan[kMaxPanel][2];
  __shared__ double pst[64][2];  // bisection stack of the panels
  __shared__ int nsq, nnext, nhold, npan, bad;
  // work area: tensor squares use Lx[24][16], Ly[24][16], G[3][24][24], C[3][16][24];
  // triangles use Lx[64][16], Ly[64][16], wts[3][64]
  __shared__ double work[2 * kNQ * 16 + 3 * kNQ * kNQ + 3 * 16 * kNQ];
  if (tid == 0) {
    nhold = 0;
    bad = 0;
    lvl[0][0][0] = 0.0;
    lvl[0][0][1] = 0.0;
  }
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;

  // level by level: thread 0 sorts the level's squares into accepted ones (tensor rule, contracted
  // right away by all threads), ones holding xi (triangles, after the loop) and ones to refine
  int cur = 0, ncur = 1;  // ncur: thread 0 only
  double h = 1.0;
  for (;;) {
    if (tid == 0) {
      int nn = 0, na = 0;
      for (int c = 0; c < ncur; ++c) {
        const double cx = lvl[cur][c][0], cy = lvl[cur][c][1];
        const double ddx = fmax(fabs(x0 - cx) - h, 0.0), ddy = fmax(fabs(y0 - cy) - h, 0.0);
        if (hypot(ddx, ddy) >= 2.0 * h) {
          if (na < kMaxAcc) {
            sq[na][0] = cx; sq[na][1] = cy;
            ++na;
          } else {
            bad = 1;
          }
          continue;
        }
        const bool holds = fabs(x0 - cx) <= h && fabs(y0 - cy) <= h;
        if (holds && h <= 1.0 / 32.0) {
          if (nhold < kMaxHold) {
            hold[nhold][0] = cx; hold[nhold][1] = cy; hold[nhold][2] = h;
            ++nhold;
          } else {
            bad = 1;
          }
          continue;
        }
        if (h < 1e-15) continue;  // only beside xi, within 2e-15: below the rounding of the sums
        if (nn + 4 > kMaxLvl) { bad = 1; continue; }
        const double q = 0.5 * h;
        const double cxs[4] = {cx - q, cx + q, cx - q, cx + q}, cys[4] = {cy - q, cy - q, cy + q, cy + q};
        for (int k = 0; k < 4; ++k) {
          lvl[1 - cur][nn][0] = cxs[k];
          lvl[1 - cur][nn][1] = cys[k];
          ++nn;
        }
      }
      nsq = na;
      nnext = nn;
      ncur = nn;
    }
    __syncthreads();
    // accepted squares of this level: tensor rule, contracted in two stages
    {
      double* Lx = work;                 // [24][16]
      double* Ly = Lx + kNQ * 16;        // [24][16]
      double* G = Ly + kNQ * 16;         // [3][24][24]
      double* C = G + 3 * kNQ * kNQ;     // [3][16][24]
      const int n_sq = nsq;
      for (int q = 0; q < n_sq; ++q) {
        const double cx = sq[q][0], cy = sq[q][1];
        if (tid < kNQ) lagrange16(R, cx + h * R.gx[tid], Lx + tid * 16);
        else if (tid >= 32 && tid < 32 + kNQ) lagrange16(R, cy + h * R.gx[tid - 32], Ly + (tid - 32) * 16);
        for (int o = tid; o < kNQ * kNQ; o += kMT) {
          const int a = o / kNQ, b = o % kNQ;
          const double dx = x0 - (cx + h * R.gx[a]), dy = y0 - (cy + h * R.gx[b]);
          const double r2 = dx * dx + dy * dy, wq = R.gw[a] * R.gw[b] * h * h;
          G[o] = 0.5 * log(r2) * wq;
          G[kNQ * kNQ + o] = dx / r2 * wq;
          G[2 * kNQ * kNQ + o] = dy / r2 * wq;
        }
        __syncthreads();
        for (int o = tid; o < 3 * 16 * kNQ; o += kMT) {  // C[k][i][b] = sum_a Lx[a][i] G[k][a][b]
          const int k = o / (16 * kNQ), i = (o / kNQ) % 16, b = o % kNQ;
          const double* g = G + k * kNQ * kNQ + b;
          double v = 0.0;
          for (int a = 0; a < kNQ; ++a) v = fma(Lx[a * 16 + i], g[a * kNQ], v);
          C[o] = v;
        }
        __syncthreads();
        for (int b = 0; b < kNQ; ++b) {
          const double l = Ly[b * 16 + jj];
          acc0 = fma(C[(0 * 16 + ii) * kNQ + b], l, acc0);
          acc1 = fma(C[(1 * 16 + ii) * kNQ + b], l, acc1);
          acc2 = fma(C[(2 * 16 + ii) * kNQ + b], l, acc2);
        }
        __syncthreads();
      }
    }
    const int more = nnext;
    __syncthreads();  // every thread has read nsq and nnext before thread 0 writes the next level's
    if (more == 0) break;
    cur = 1 - cur;
    h *= 0.5;
  }

  // squares holding xi: four polar-Duffy triangles each
  {
    double* Lx = work;           // [64][16]
    double* Ly = Lx + 64 * 16;   // [64][16]
    double* wt = Ly + 64 * 16;   // [3][64]
    const int n_hold = nhold;
    for (int hq = 0; hq < n_hold; ++hq) {
      const double cx = hold[hq][0], cy = hold[hq][1], h = hold[hq][2];
      for (int ed = 0; ed < 4; ++ed) {
        // the edge from corner ed to corner ed + 1, corners counter-clockwise from (-h, -h)
        const int ea = ed, eb = (ed + 1) & 3;
        const double ax = cx + ((ea == 1 || ea == 2) ? h : -h), ay = cy + (ea >= 2 ? h : -h);
        const double bx = cx + ((eb == 1 || eb == 2) ? h : -h), by = cy + (eb >= 2 ? h : -h);
        const double e0x = ax - x0, e0y = ay - y0;
        const double dx = bx - ax, dy = by - ay;
        const double twoA = fabs(e0x * dy - e0y * dx);
        if (twoA < 1e-300) continue;  // xi on this edge's line: the triangle is empty
        const double L2 = dx * dx + dy * dy;
        const double vf = -(e0x * dx + e0y * dy) / L2, hv = twoA / L2;
        if (tid == 0) {  // panels of [0, 1] by bisection (a small stack in the panel list's tail)
          int np = 0, top = 0;
          pst[top][0] = 0.0;
          pst[top][1] = 1.0;
          ++top;
          while (top > 0) {
            --top;
            const double a = pst[top][0], b = pst[top][1];
            const double c = 0.5 * (a + b), hl = 0.5 * (b - a);
            const bool done = bernstein_rho(vf, hv, c, hl) >= 4.0 || hl < 1e-12;
            if (done || top + 2 > 64) {
              if (!done) bad = 1;  // the stack is full (cannot happen, see the capacities above)
              if (np < kMaxPanel) {
                pan[np][0] = c;
                pan[np][1] = hl;
                ++np;
              } else {
                bad = 1;
              }
            } else {
              pst[top][0] = a; pst[top][1] = c; ++top;
              pst[top][0] = c; pst[top][1] = b; ++top;
            }
          }
          npan = np;
        }
        __syncthreads();
        const int n_pan = npan;
        const int n_nodes = n_pan * 12 * 16;
        for (int n0 = 0; n0 < n_nodes; n0 += 64) {
          // node (panel p, edge point qv, radial point ju); threads 0..63 the x rows and weights,
          // threads 64..127 the y rows
          if (tid < 128) {
            const int nq = n0 + (tid & 63);
            const bool live = nq < n_nodes;
            const int nqc = live ? nq : 0;
            const int p = nqc / 192, qv = (nqc / 16) % 12, ju = nqc % 16;
            const double c = pan[p][0], hl = pan[p][1];
            const double v = c + hl * R.px[qv], wv = hl * R.pw[qv];
            const double ex = e0x + v * dx, ey = e0y + v * dy;
            const double u = R.u[ju];
            if (tid < 64) {
              lagrange16(R, x0 + u * ex, Lx + tid * 16);
              const double e2 = ex * ex + ey * ey, lnE = 0.5 * log(e2);
              wt[tid] = live ? twoA * wv * u * (R.ul[ju] + lnE * R.uw[ju]) : 0.0;
              wt[64 + tid] = live ? -twoA * wv * ex / e2 * R.uw[ju] : 0.0;
              wt[128 + tid] = live ? -twoA * wv * ey / e2 * R.uw[ju] : 0.0;
            } else {
              lagrange16(R, y0 + u * ey, Ly + (tid - 64) * 16);
            }
          }
          __syncthreads();
          for (int q = 0; q < 64; ++q) {
            const double l = Lx[q * 16 + ii] * Ly[q * 16 + jj];
            acc0 = fma(wt[q], l, acc0);
            acc1 = fma(wt[64 + q], l, acc1);
            acc2 = fma(wt[128 + q], l, acc2);
          }
          __syncthreads();
        }
      }
    }
  }
  const double ls = log(s), Wk = R.w[ii] * R.w[jj];
  double* m = mom + e * 768;
  m[tid] = -kInv2Pi * s * s * (ls * Wk + acc0);
  m[256 + tid] = -kInv2Pi * s * acc1;
  m[512 + tid] = -kInv2Pi * s * acc2;
  if (tid == 0) flag[e] = bad;
}

}  // namespace

hipError_t launch_point_moments(const MomentRules& R, int64_t n, const double* pairs, double* mom, int32_t* flag,
                                hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (n > int64_t(0x7fffffff)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(point_moments_kernel, dim3(unsigned(n)), dim3(kMT), 0, stream, R, pairs, mom, flag);
  return hipGetLastError();
}

}  // namespace vp
