// dm_fused.h -- reduced-precision fused mode stepper (dm_fused.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "dm_tables.h"

namespace dm {

// Device state and tables of one length bucket on the fused path.
struct FusedBucket {
    int bf16 = 0;            // 1: split-BF16 transforms, 0: FP32 MFMA
    int RT = 0;              // 16-row tiles per half: Hp = 16 RT >= M/2
    int ntiles = 0;          // chain tiles of 5 chains
    void *d_X = nullptr;     // bond-mode transform fragments (see dm_fused.hip)
    float *d_R = nullptr;    // internal mode amplitudes, fragment order
    double *d_R0 = nullptr;  // centre-of-mass mode, ntiles * 16 doubles
    float *d_coef = nullptr; // per-slot update coefficients (see dm_fused.hip)
    double *d_sig = nullptr; // sigma_p of the even modes, by half-mode slot
    int JC = 0;              // coupling row tiles with non-negligible C_p
    int resident = 0;        // tables held in LDS for the whole launch
    double W0 = 0.0, gdt = 0.0;
    float lin = 0.0f;
    std::vector<double> Xo, Se, sig;  // host FP64 half tables (the coupling
                                      // table is rebuilt when dtau changes)
};

bool fused_supports(int M);
hipError_t fused_alloc(FusedBucket &f, int M, int n, bool bf16);
void fused_free(FusedBucket &f);
hipError_t fused_pack_modes(FusedBucket &f, const double *R64, int M, int n, hipStream_t st);
hipError_t fused_unpack_modes(const FusedBucket &f, double *R64, int M, int n, hipStream_t st);
hipError_t fused_set_coefs(FusedBucket &f, const ModeCoefs &mc, int M, double lin, double gdt,
                           hipStream_t st);
hipError_t fused_step(FusedBucket &f, const int32_t *ids, int M, int n, uint64_t seed,
                      int64_t step0, int n_steps, int nonlinear, hipStream_t st);
hipError_t fused_check_finite(const FusedBucket &f, int M, int n, int *flag, hipStream_t st);

}  // namespace dm
