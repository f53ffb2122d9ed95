// dm_tables.h -- host FP64 mode tables (see dm_tables.cpp).
#pragma once
#include <vector>

namespace dm {

struct ModeCoefs {
    std::vector<double> zeta_l, zeta, E, C, W;  // index p = 0..M-1
};

// phi[n*M + p] = phi_{n,p} of Eq. (c8) (orthonormal, Eq. c2).
void rouse_matrix(int M, std::vector<double> &phi);

// Rates and one-step coefficients of the mode update for step dtau.
void mode_coefficients(int M, double nu, double T_star, double dtau, ModeCoefs &out);

}  // namespace dm
