// One 1D V-tensor row evaluated on the device in FP64 (paper Sec. 4,
// eq. CartesianVector in the monomial form of eq. Ccoefficients):
//   V(q) = exp(-q^2 / (4p)) * exp(i q P) * sum_u e_u (i q)^u ,
// with every q-independent factor of the primitive pair folded into e_u.
// The phase q P is reduced to revolutions in [-1/2, 1/2] before the sine
// and cosine.  Shared by the 1D-table, points and separable kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "engine.h"

namespace scff {

__device__ __forceinline__ double2 eval_row_fp64(const VRowDev& r, double q) {
    const double rev = q * r.P * 0.15915494309189535;   // 1/(2 pi)
    const double red = rev - rint(rev);
    double s, c;
    sincospi(2.0 * red, &s, &c);
    const double q2 = q * q;
    const double g = exp(-q2 * r.inv4p);
    // sum_u e_u (i q)^u = (e0 - e2 q^2 + e4 q^4) + i q (e1 - e3 q^2)
    const double pr = fma(fma(r.e[4], q2, -r.e[2]), q2, r.e[0]);
    const double pi = q * fma(-r.e[3], q2, r.e[1]);
    return make_double2(g * (c * pr - s * pi), g * (c * pi + s * pr));
}

}  // namespace scff
