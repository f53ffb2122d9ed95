// dm_internal.h -- launchers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dnamodes.h"

namespace dm {

// Doubles of one chain's accumulators: head, |R_p|^2 sums, tumbling bins.
__host__ __device__ inline int acc_width(int M)
{
    return DM_NACC_HEAD + M + DM_NTUMBLE_BINS + 4 * DM_NCORR;
}

// Time correlations at one sample of one chain: v = (L, u_m, d), 9 doubles;
// ring holds the chain's last R = 2^(K-1) samples (K >= 1 lags), count the
// samples written so far; the lag blocks of the chain's accumulators start
// at corr.  Lag j compares with the sample l_j = (j ? 2^(j-1) : 0) back.
__device__ inline void corr_update(double *ring, double *count, double *corr, const double v[9],
                                   int K)
{
    const long R = 1L << (K - 1);
    const long i = (long)*count;
    double *slot = ring + (i & (R - 1)) * 9;
    for (int q = 0; q < 9; ++q) slot[q] = v[q];
    for (int j = 0; j < K; ++j) {
        const long l = j ? (1L << (j - 1)) : 0;
        if (l > i) break;
        const double *w = ring + ((i - l) & (R - 1)) * 9;
        double *cj = corr + 4 * j;
        cj[DM_CORR_L] += v[0] * w[0] + v[1] * w[1] + v[2] * w[2];
        cj[DM_CORR_UMID] += v[3] * w[3] + v[4] * w[4] + v[5] * w[5];
        const double dx = v[6] - w[6], dy = v[7] - w[7], dz = v[8] - w[8];
        cj[DM_CORR_MSD] += dx * dx + dy * dy + dz * dz;
        cj[DM_CORR_COUNT] += 1.0;
    }
    *count = (double)(i + 1);
}

// Message that dm_last_error(NULL) returns (errors of calls without a
// context), dm_api.hip.
void set_ctxless_error(const char *msg);

// Plain-form (FP64) kernels, dm_plain.hip.  Every launcher only enqueues on
// `st` and returns the launch status.

// Y[c][i] = sum_k A[i*M + k] X[c*M + k] for c < ncol, i, k < M (FP64 MFMA).
hipError_t launch_gemm_f64(const double *A, const double *X, double *Y, int M,
                           int ncol, hipStream_t st);

// Bead forces of the nonlinear bond term from internal positions r:
// g_n = u_n (1/|u_n| - lin), F_n = g_n - g_{n+1} (Eqs. e4, e11).
hipError_t launch_stencil_f64(const double *r, double *F, int M, int nch,
                              double lin, hipStream_t st);

// R_p <- E_p R_p + C_p dH_p + W_p eta_p, then R^x_p += gdt E_p R^y_p(old);
// p = 0 takes no coupling.  Philox step index = (*step_dev) + step_off
// (step_dev may be null).
hipError_t launch_mode_update_f64(double *R, const double *dH, const double *E,
                                  const double *C, const double *W,
                                  const int32_t *ids, int M, int nch,
                                  uint64_t seed, const int64_t *step_dev,
                                  int64_t step_off, double gdt, int nonlinear,
                                  hipStream_t st);

// n_steps bead-space Euler steps on positions pos (SoA), one block per chain.
hipError_t launch_euler_f64(double *pos, const int32_t *ids, int M, int nch,
                            double nu, double dtau, double T_star, double gdt,
                            uint64_t seed, int64_t step0, int n_steps,
                            hipStream_t st);

// n_steps of the inextensible limit (Eqs. y2-y14) on positions pos (SoA,
// nch chains of M beads with unit bonds): one wavefront per chain with the
// chain in registers up to M = 64 and in LDS up to M = 341, else one thread
// per chain with its state in
// scr, which holds wlc_scratch_doubles(M, nch) doubles (0 when the chain fits
// the LDS; scr may then be null).  The tension cycle runs at most iters
// times and, with tol > 0, stops after a cycle that moves no bond component
// by more than tol.  midpoint != 0: forces and tensions act along the
// midpoint bonds (u_n + u'_n)/|u_n + u'_n|; 0: along the bonds u_n of the
// start of the step.
size_t wlc_scratch_doubles(int M, int nch);
hipError_t launch_wlc(double *pos, double *scr, const int32_t *ids, int M, int nch, double T_bar,
                      double dt, int iters, double tol, int midpoint, uint64_t seed,
                      int64_t step0, int n_steps, hipStream_t st);

// n_sweeps Metropolis sweeps of the FP64 amplitudes R (nch chains of 3*M),
// with chiT[p*(M-1) + n-1] = chi_{n,p} and step half-widths sstep[p]; the
// accepted proposals of chain c go to accepted[c].
hipError_t launch_mc(double *R, const double *chiT, const double *sstep, const int32_t *ids,
                     int M, int nch, double nu, double T_star, uint64_t seed, int64_t step0,
                     int n_sweeps, int64_t *accepted, hipStream_t st);

// Per-chain observables from positions and modes; writes obs[c*16 + .] and
// m2[c*M + p] = |R_p|^2, and adds into the per-chain accumulators
// acc[c*acc_width(M) + .] when accumulate != 0, advancing the tumbling state
// (tstate[c] = -1, 0, +1; tlast[c] = step of the last tumble + 1, or 0) with
// the current step *step_dev.
// With K > 0 lags also the time correlations (corr_update) with the ring
// ring[c*R*9] and the sample counts ccount[c].
hipError_t launch_chain_obs(const double *pos, const double *R, double *obs,
                            double *m2, double *acc, const double *cm0,
                            double *tstate, double *tlast,
                            const int64_t *step_dev, double *ring, double *ccount,
                            int K, int M, int nch, int accumulate, hipStream_t st);

// out[j] = sum_c acc[c*width + j], summed over chains in order.
hipError_t launch_reduce_chains(const double *acc, double *out, int width,
                                int nch, hipStream_t st);

// *flag |= 1 if any of x[0..n) is NaN or Inf (flag is not cleared).
hipError_t launch_check_finite_f64(const double *x, size_t n, int *flag,
                                   hipStream_t st);
hipError_t launch_check_finite_f32(const float *x, size_t n, int *flag,
                                   hipStream_t st);

// dst[off[c] + i] = src[c*len + i] for i < len (bucket -> caller order).
hipError_t launch_scatter_chains(const double *src, double *dst,
                                 const int64_t *off, int len, int nch,
                                 hipStream_t st);

}  // namespace dm
