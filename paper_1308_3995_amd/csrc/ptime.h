// Backward-Euler pseudo-time step of the Newton iteration (Sec. 3.3), shared by the Euler
// and Navier-Stokes condensation kernels.
//
// The time derivative adds the element mass matrix over a local step dt_K to the w-w block
// of the element Jacobian. With the orthonormal basis the mass matrix of element K is
// det J times the identity, so the shift is a scalar on that block's diagonal:
//   sigma_K = det J / dt_K,  dt_K = CFL |K| / (lambda_c + 4 lambda_v),
//   lambda_c = sum_e (|v.n| + c) |e|,  lambda_v = (mu gamma / (rho Pr)) sum_e |e|^2 / |K|,
// both at the element-mean state (the constant mode of w_h times the constant basis value).
#pragma once

#include "hdg_internal.h"

namespace hdg {

// wbar: element-mean conserved state; visc = mu gamma / Pr (0 for the Euler equations).
// Returns 0 when cfl == 0 (a pure Newton step).
__device__ __forceinline__ double pseudo_time_shift(const ElemInfo* E, const double* wbar, double cfl,
                                                    double gamma, double visc) {
    if (!(cfl > 0.0)) return 0.0;
    const double rho = wbar[0], u = wbar[1] / rho, v = wbar[2] / rho;
    const double p = (gamma - 1.0) * (wbar[3] - 0.5 * rho * (u * u + v * v));
    const double c = sqrt(gamma * p / rho);
    const double area = 2.0 * E->detj;
    double lc = 0.0, l2 = 0.0;
#pragma unroll
    for (int lf = 0; lf < 3; ++lf) {
        lc += (fabs(u * E->nrm[lf][0] + v * E->nrm[lf][1]) + c) * E->len[lf];
        l2 += E->len[lf] * E->len[lf];
    }
    const double lv = visc / rho * l2 / area;
    const double dt = cfl * area / (lc + 4.0 * lv);
    return E->detj / dt;
}

}  // namespace hdg
