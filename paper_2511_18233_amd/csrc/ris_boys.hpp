// Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt on the device, FP64.
//
// T < 40: F_M(T) from a table on the grid T_k = k/16 by a Taylor expansion in
// (T - T_k), using dF_m/dT = -F_{m+1}:
//     F_M(T) = sum_j F_{M+j}(T_k) (T_k - T)^j / j!,  |T - T_k| <= 1/32,
// eight terms (truncation below 1e-16 relative), then the downward recursion
// F_m = (2T F_{m+1} + e^{-T}) / (2m+1), which is stable.
// T >= 40: F_0 = (1/2) sqrt(pi/T) (erf(sqrt 40) rounds to 1 in FP64) and the
// upward recursion F_{m+1} = ((2m+1) F_m - e^{-T}) / (2T), stable for T > m.
#pragma once

#include "ris_common.hpp"

namespace ris {

template <int M>
__device__ __forceinline__ void boys_eval(double T, const double *__restrict__ tab, double (&F)[M + 1])
{
    static_assert(M <= kBoysMaxM, "Boys order beyond the table");
    const double et = exp(-T);
    if (T < kBoysTMax) {
        const int k = __double2int_rn(T * kBoysInvStep);
        const double d = (double)k * (1.0 / kBoysInvStep) - T;  // T_k - T
        const double *row = tab + (size_t)k * kBoysCols + M;
        // Horner form of sum_j row[j] d^j / j!
        double s = row[kBoysTaylor - 1];
#pragma unroll
        for (int j = kBoysTaylor - 1; j >= 1; --j) s = row[j - 1] + s * d * (1.0 / j);
        F[M] = s;
        const double t2 = 2.0 * T;
#pragma unroll
        for (int m = M - 1; m >= 0; --m) F[m] = (t2 * F[m + 1] + et) * (1.0 / (2 * m + 1));
    } else {
        F[0] = 0.5 * sqrt(3.14159265358979323846 / T);
        const double inv2t = 0.5 / T;
#pragma unroll
        for (int m = 0; m < M; ++m) F[m + 1] = ((2 * m + 1) * F[m] - et) * inv2t;
    }
}

}  // namespace ris
