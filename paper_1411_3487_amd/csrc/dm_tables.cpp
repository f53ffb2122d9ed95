// dm_tables.cpp -- host FP64 mode tables for one chain length (K0).
//
// Rouse modes phi_{n,p} = sqrt(2/M) cos(p (n+1/2) pi/M), phi_{n,0} = 1/sqrt(M)
// (Eq. c8; the p = 0 normalisation is the one that makes phi orthogonal,
// Eq. c2).  Rates in their cancellation-free forms, with s_p = sin(p pi/2M):
//   zeta^l_p = 4 s_p^2 (1 - 2 nu cos(p pi/M))          (Eq. c9)
//   zeta_p   = zeta^l_p - (1-2nu) 4 s_p^2 = 16 nu s_p^4 (Eq. e9)
// and the per-step coefficients
//   E_p = exp(-zeta_p dtau)                              (Eq. d3)
//   C_p = [exp(-zeta_p dtau) - exp(-zeta^l_p dtau)] / (zeta^l_p - zeta_p)
//       = -E_p expm1(-(1-2nu) 4 s_p^2 dtau) / ((1-2nu) 4 s_p^2)  (Eq. f2)
//   W_p = sqrt(T* [1 - exp(-2 zeta_p dtau)] / zeta_p)    (Eq. d6)
// with the zeta -> 0 limits W = sqrt(2 T* dtau) and C = dtau E.
#include "dm_tables.h"

#include <cmath>

namespace dm {

void rouse_matrix(int M, std::vector<double> &phi)
{
    phi.assign((size_t)M * M, 0.0);
    const double pi = 3.141592653589793238462643383279502884;
    const double c0 = std::sqrt(1.0 / M), c1 = std::sqrt(2.0 / M);
    for (int n = 0; n < M; ++n)
        for (int p = 0; p < M; ++p)
            phi[(size_t)n * M + p] =
                (p == 0) ? c0 : c1 * std::cos(pi * (double)p * (n + 0.5) / M);
}

void mode_coefficients(int M, double nu, double T_star, double dtau, ModeCoefs &out)
{
    const double pi = 3.141592653589793238462643383279502884;
    out.zeta_l.assign(M, 0.0);
    out.zeta.assign(M, 0.0);
    out.E.assign(M, 1.0);
    out.C.assign(M, dtau);
    out.W.assign(M, std::sqrt(2.0 * T_star * dtau));
    const double lin = 1.0 - 2.0 * nu;
    for (int p = 1; p < M; ++p) {
        const double s = std::sin(pi * p / (2.0 * M));
        const double s2 = s * s;
        const double zl = 4.0 * s2 * (1.0 - 2.0 * nu * std::cos(pi * p / M));
        const double z = 16.0 * nu * s2 * s2;
        const double dz = lin * 4.0 * s2;
        const double E = std::exp(-z * dtau);
        out.zeta_l[p] = zl;
        out.zeta[p] = z;
        out.E[p] = E;
        out.C[p] = dz > 0.0 ? -E * std::expm1(-dz * dtau) / dz : dtau * E;
        out.W[p] = z > 0.0 ? std::sqrt(-T_star * std::expm1(-2.0 * z * dtau) / z)
                           : std::sqrt(2.0 * T_star * dtau);
    }
}

}  // namespace dm
