// Device interface of the point moments (moments.hip): the near-field weights of an off-grid
// point on an adjacent leaf.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace vp {

// The quadrature rules, by value (about 1.2 KB).
struct MomentRules {
  double t[16], lam[16], w[16];  // leaf nodes (first-kind Chebyshev), barycentric weights, node weights
  double gx[24], gw[24];         // Gauss rule of the accepted squares (per direction)
  double px[12], pw[12];         // Gauss rule of the panels along a Duffy triangle's far edge
  double u[16], uw[16], ul[16];  // radial rule: nodes, weights of int_0^1 f, weights of int_0^1 f ln u
};

// pairs: n x 3 (xi_x, xi_y, s): the point in leaf b's reference square and b's half-width.
// mom: n x 3 x 256: s^2 (-1/2pi) (ln s W_k + I_k(xi)), s (-1/2pi) dI_k/dxi_x, s (-1/2pi) dI_k/dxi_y
// with I_k(xi) = int over [-1,1]^2 of ln|xi - eta| l_k(eta) d eta. flag[e] = 1 where pair e's
// refinement outgrew the kernel's fixed lists (its moments must then come from elsewhere).
hipError_t launch_point_moments(const MomentRules& R, int64_t n, const double* pairs, double* mom, int32_t* flag,
                                hipStream_t stream);

}  // namespace vp
