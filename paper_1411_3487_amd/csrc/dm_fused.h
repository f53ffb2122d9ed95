// dm_fused.h -- reduced-precision fused mode stepper (dm_fused.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
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
    float *d_P = nullptr;    // FP32 position tables of the observables
    float *d_Rs = nullptr;   // snapshot of d_R / d_R0 for deferred observables
    double *d_R0s = nullptr;
    int JC = 0;              // coupling row tiles with non-negligible C_p
    int resident = 0;        // tables held in LDS for the whole launch
    int tpw = 4;             // tiles per workgroup (1..4; 4 when streamed, 1 split)
    int split = 0;           // 1: one tile per workgroup, its rows and modes
                             // divided among 4 wavefronts; 2: among 8
                             // (split-BF16, RT = 8 and 16, a kernel of its own)
    double item_us = 0.0;    // measured time of one workgroup-step (0: model)
    int n = 0;               // chains
    const int32_t *ids = nullptr;  // device: global chain index per local chain
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

// One launch over all buckets: a list of workgroup items, longest first.
struct FusedPlan {
    int bf16 = 0, nitems = 0, nbuckets = 0;
    int nwide = 0;  // the last nwide items run on 8-wavefront split tiles
    void *d_buckets = nullptr, *d_items = nullptr;
};
// Build the launch for the buckets (all of one precision) with their current
// tile shapes; max_items > 0 keeps only the first items (timing).
hipError_t fused_plan(FusedPlan &p, const std::vector<const FusedBucket *> &bs, int max_items,
                      hipStream_t st);
void fused_plan_free(FusedPlan &p);
// n_steps mode steps of every bucket of the plan; the Philox step of the
// first step is *d_step when d_step is non-null (read on the device, for
// replayed graphs), else step0.
hipError_t fused_launch(const FusedPlan &p, uint64_t seed, int64_t step0, const int64_t *d_step,
                        int n_steps, int nonlinear, hipStream_t st);
// Time every tile shape of every bucket on a scratch copy of its state and
// keep the combination with the shortest list-schedule makespan.  One line
// per candidate goes to report.
hipError_t fused_autotune(std::vector<FusedBucket *> &bs, uint64_t seed, int steps,
                          hipStream_t st, std::string &report);
// Time of one workgroup item of the bucket for one step, in microseconds:
// measured by the autotuner, else the cost model.
double fused_item_us(const FusedBucket &f);
// Force a tile shape where it exists: table_mode 1 resident, 2 streamed,
// 3 split over 4 wavefronts, 4 split over 8 (0 keeps the current); tpw 1..4
// where resident (0 keeps the current).
void fused_force_shape(FusedBucket &f, int table_mode, int tpw);
// Device step counter of replayed graphs: *d_step = value, *d_step += n.
hipError_t fused_set_step(int64_t *d_step, int64_t value, hipStream_t st);
hipError_t fused_advance_step(int64_t *d_step, int64_t n, hipStream_t st);
// Per-chain observables, |R_p|^2 and (accumulate != 0) the FP64 accumulators
// and tumbling state of the bucket, in the layout of launch_chain_obs, from
// the fused state directly (positions in FP32 MFMA, sums in FP64).
// from_snapshot: read the state saved by fused_snapshot instead of the live
// one; max_wg > 0 caps the grid (each workgroup then loops over tiles).
hipError_t fused_observe(const FusedBucket &f, int M, double *obs, double *m2, double *acc,
                         const double *cm0, double *tstate, double *tlast,
                         const int64_t *d_step, double *ring, double *ccount, int K,
                         int accumulate, hipStream_t st, bool from_snapshot = false,
                         int max_wg = 0);
// Copy of the state (d_R, d_R0 -> d_Rs, d_R0s) for observables taken while
// the next steps already run; fused_snapshot_alloc allocates it (not inside a
// graph capture).
hipError_t fused_snapshot_alloc(FusedBucket &f);
hipError_t fused_snapshot(const FusedBucket &f, hipStream_t st);
hipError_t fused_check_finite(const FusedBucket &f, int M, int n, int *flag, hipStream_t st);

}  // namespace dm
