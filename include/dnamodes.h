/*
 * dnamodes.h -- C ABI of the MI355X (gfx950) library for the mode-amplitude
 * Langevin dynamics of semiflexible chains of Panja, Barkema & van Leeuwen,
 * "Efficient simulation of semiflexible polymers" (arXiv:1411.3487).
 *
 * Model (Sec. II, Eqs. a1-a3): a chain of M = N+1 beads r_0..r_N with bonds
 * u_n = r_n - r_{n-1}, Hamiltonian
 *     H = lambda/2 sum_n (|u_n| - d)^2 - kappa sum_n u_n . u_{n+1},
 * reduced by nu = kappa/lambda and T* = kT/(lambda d^2); lengths in units of
 * d, time in units of xi/lambda (Sec. III, Eqs. b3-b5).  Overdamped Langevin
 * dynamics with friction xi and thermal noise of variance 2 T*.
 *
 * Method (Secs. III.A–IV.B): positions are expanded in Rouse modes
 * phi_{n,p} = sqrt(2/M) cos(p (n + 1/2) pi / M) (phi_{n,0} = 1/sqrt(M)),
 * Eqs. (c1), (c8); each amplitude R_p obeys Eq. (e10),
 *     dR_p/dtau = -zeta_p R_p + Delta H_p + G_p,
 * and is advanced by the integrating factor of Eq. (d3) with the noise
 * variance of Eq. (d6) and the coupling integral approximated by Eq. (f2):
 *     R_p <- E_p R_p + C_p Delta H_p + W_p eta_p.
 * The bead-space Euler scheme of Eqs. (b3)-(b5) is provided as the plain
 * baseline.  Simple shear (Eq. btum) adds gamma_dot * y along x.
 *
 * Conventions for every function below:
 *  - Return value: DM_OK (0) on success, a negative DM_E* code on failure;
 *    dm_last_error() then gives a message.  A failed call leaves the
 *    simulation state unchanged unless stated otherwise.
 *  - Pointers marked "host" are read or written during the call only and
 *    stay owned by the caller.  The context owns all device memory it
 *    allocates (freed by dm_destroy).
 *  - Work is enqueued on the HIP stream given to dm_init_chains and runs
 *    asynchronously; calls that return host data synchronise that stream.
 *  - A context is not thread-safe; separate contexts are independent.
 *  - Array layout ("SoA"): one chain is 3*M doubles, component-major:
 *    x_0..x_{M-1}, y_0.., z_0..; chains follow each other in chain order.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 *    (seed lo, seed hi) and counter (index/4, chain, step lo,
 *    (step hi << 8) | (component << 4) | tag); the four outputs give two
 *    Box-Muller pairs, normal j of the block belongs to index 4*(index/4)+j.
 *    tag 0 = mode step (index = mode p), 1 = Euler step (index = bead n),
 *    2 = Monte Carlo sweep (index = mode p, see dm_step_mc),
 *    3 = inextensible limit (index = bead n, see dm_step_wlc),
 *    4 and 5 = initial state of a context created without positions
 *    (see dm_init_chains).
 *    Results are therefore independent of how chains are batched.
 */
#ifndef DNAMODES_H
#define DNAMODES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define DM_OK          0
#define DM_EINVAL     -1   /* invalid argument */
#define DM_ENOMEM     -2   /* device or host allocation failed */
#define DM_EHIP       -3   /* a HIP runtime call failed */
#define DM_ENONFINITE -4   /* the state became NaN or Inf */
#define DM_ESTATE     -5   /* call out of order (e.g. stepping before set_params) */

/* Arithmetic of the mode step. */
#define DM_FP64    0  /* plain form: dense phi products on FP64 MFMA, separate
                         force-stencil and mode-update kernels, FP64 state */
#define DM_FP32    1  /* fused persistent kernel, FP32 MFMA transforms, FP32
                         internal modes, FP64 centre of mass */
#define DM_BF16X3  2  /* fused persistent kernel, transforms as three BF16 MFMA
                         products (hi*hi + hi*lo + lo*hi) accumulated in FP32,
                         FP32 internal modes, FP64 centre of mass */

/* dm_observables() selection bits. */
#define DM_OBS_CHAIN  1  /* per chain, current state, DM_NCHAIN_OBS doubles */
#define DM_OBS_MODES  2  /* per chain, current |R_p|^2, p = 0..M_c-1 */
#define DM_OBS_ACCUM  4  /* per length bucket, sums since the last reset */
#define DM_OBS_RESET  8  /* zero the accumulators after copying them out */

/* Per-chain observables (Sec. V.B): index into the DM_OBS_CHAIN block. */
#define DM_NCHAIN_OBS   16
#define DM_CO_BOND       0  /* mean bond length (1/N) sum_n |u_n| */
#define DM_CO_L2         1  /* |L|^2, end-to-end vector L = r_N - r_0 */
#define DM_CO_LX         2  /* L_x, L_y, L_z at 2, 3, 4 */
#define DM_CO_CM         5  /* centre of mass r_cm = R_0 / sqrt(M), 5..7 */
#define DM_CO_UMID       8  /* middle bond u_{M/2}, 8..10 */
#define DM_CO_DMID      11  /* r_{(M-1)/2} - r_cm, 11..13 */
#define DM_CO_XSPAN     14  /* max_n x_n - min_n x_n */
#define DM_CO_BOND2     15  /* mean squared bond length (1/N) sum_n |u_n|^2 */

/* Accumulator block of one length bucket: DM_NACC_HEAD doubles, then the
   sum over samples and chains of |R_p|^2 for p = 0..M-1, then
   DM_NTUMBLE_BINS counts of tumbling times: bin k counts intervals tau
   (in steps) with 2^k <= tau < 2^(k+1) (the last bin also everything
   longer).  Tumbling (Sec. VIII, simple shear): the in-plane end-to-end
   vector (L_x, L_y) is "along +x" once L_x > |(L_x, L_y)|/2 and "along -x"
   once L_x < -|(L_x, L_y)|/2 (hysteresis: in between the previous state is
   kept); each change between the two states at a sample is one tumble, and
   a tumbling time is the interval between two tumbles of a chain.
   Then DM_NCORR blocks of 4 doubles, one per lag l_j (l_0 = 0,
   l_j = 2^(j-1) samples), for the time correlations of Sec. V.B (measured
   for j < corr_lags, zero otherwise): sum of L(t).L(t - l_j) (end-to-end
   vector), of u_m(t).u_m(t - l_j) (middle bond u_{M/2}), of
   |d(t) - d(t - l_j)|^2 with d = r_{(M-1)/2} - r_cm (msd of the middle bead
   about the centre of mass), and the number of pairs summed. */
#define DM_NACC_HEAD    13
#define DM_ACC_M         0  /* beads per chain in this bucket */
#define DM_ACC_NCHAINS   1
#define DM_ACC_NSAMPLES  2  /* number of sampling events */
#define DM_ACC_BOND      3  /* sum of DM_CO_BOND over chains and samples */
#define DM_ACC_BOND2     4  /* sum of DM_CO_BOND2 */
#define DM_ACC_L2        5  /* sum of DM_CO_L2 */
#define DM_ACC_MSDCM     6  /* sum of |r_cm - r_cm at the last reset|^2 */
#define DM_ACC_DMID2     7  /* sum of |r_mid - r_cm|^2 */
#define DM_ACC_XSPAN     8  /* sum of DM_CO_XSPAN (extension along the flow) */
#define DM_ACC_TUMBLES   9  /* number of tumbles */
#define DM_ACC_TAU      10  /* sum of tumbling times (steps) */
#define DM_ACC_TAU2     11  /* sum of squared tumbling times (steps^2) */
#define DM_ACC_NTAU     12  /* number of tumbling times */
#define DM_NTUMBLE_BINS 32
#define DM_NCORR        16
#define DM_CORR_L        0  /* offsets inside one lag block */
#define DM_CORR_UMID     1
#define DM_CORR_MSD      2
#define DM_CORR_COUNT    3

/* dm_get_tiling(): DM_NTILING doubles per length bucket. */
#define DM_NTILING       9
#define DM_TI_M          0  /* beads per chain */
#define DM_TI_NCHAINS    1
#define DM_TI_RT         2  /* 16-row tiles per half transform (fused) */
#define DM_TI_JC         3  /* coupling row tiles kept (modes p <= 32 JC) */
#define DM_TI_RESIDENT   4  /* 1: tables held in LDS for a whole launch */
#define DM_TI_TPW        5  /* tiles of 5 chains per workgroup */
#define DM_TI_ITEMS      6  /* workgroups of this bucket per launch */
#define DM_TI_ITEM_US    7  /* measured us per workgroup-step (autotune), or 0 */
#define DM_TI_SPLIT      8  /* 1: one tile per workgroup, its bond rows and
                               mode tiles divided among 4 wavefronts; 2: among
                               8 (two per SIMD; split-BF16, RT = 8 and 16) */

typedef struct dm_ctx dm_ctx;

/* Model, time step and run parameters.
   Physical units when lambda > 0 (pN/nm for lambda and kappa, pN nm for kT,
   nm for a, pN ps/nm for xi, ps for dt, 1/ps for gamma_dot): then
   nu = kappa/lambda, b = 1/(1-2nu), d = a/b, T* = kT/(lambda d^2) (Eqs. a2,
   a3) and dtau = dt lambda/xi (Sec. III).  Reduced units when lambda == 0:
   T_star, nu, dt (= dtau) and gamma_dot are used as given. */
typedef struct {
    double lambda, kappa, kT, a, xi;
    double T_star, nu;
    double gamma_dot;        /* shear rate of Eq. (btum); 0 = no flow */
    int32_t nonlinear;       /* 1: coupling Delta H_p of Eq. (e11) on;
                                0: free Ornstein-Uhlenbeck modes (test mode) */
    int32_t n_lengths;       /* entries in lengths[] / dt[] */
    const int32_t *lengths;  /* host: chain lengths (beads) */
    const double *dt;        /* host: time step for each length */
    int32_t sample_every;    /* accumulate observables every this many
                                mode steps (0 = never) */
    int32_t check_finite;    /* 1: after each dm_step_* call check the state
                                for NaN/Inf and return DM_ENONFINITE */
    int32_t autotune;        /* fused paths, 1: dm_set_params times every tile
                                shape of every length bucket on a scratch
                                copy of the state and keeps the combination
                                with the shortest schedule (see
                                dm_get_tiling); 0: fixed shapes */
    int32_t use_graphs;      /* sample_every > 0 (at most 256 on DM_FP64), 1:
                                whole sampling blocks (the fused launch, or
                                the FP64 plain form's four launches per step
                                and length, the step counter and the
                                observables) are captured once as a HIP graph
                                and replayed.  On the fused paths, when the
                                launch leaves compute units idle, runs of
                                several blocks take each block's sample from
                                a snapshot of its state on a second stream
                                while the next block runs (same results) */
    int32_t tiles_per_wg;    /* fused paths: 0 = automatic; 1..4 = tiles of 5
                                chains per workgroup where the tables are
                                resident (streamed tables always take 4) */
    int32_t table_mode;      /* fused paths: 0 = automatic, 1 = tables
                                resident in LDS, 2 = streamed from L2,
                                3 = split tiles (one tile of 5 chains per
                                workgroup, its bond rows and mode tiles
                                divided among 4 wavefronts: for launches
                                with fewer tiles than SIMDs; lengths with
                                RT = 4, 8, 12, 16, i.e. 65..128, 193..256,
                                321..384, 449..512 beads), 4 = split tiles
                                over 8 wavefronts (split-BF16, RT = 8 and
                                16), each where that form exists for the
                                length (it overrides the autotuner).
                                Automatic without autotune: split tiles
                                where they exist when the launch has no
                                more tiles than compute units (of 8
                                wavefronts when every length has that
                                form), else resident tables where they
                                fit.  Results do not depend on the tile
                                shape */
    int32_t corr_lags;       /* 0..14: number of lags of the time
                                correlations in the accumulators (a ring of
                                2^(corr_lags-1) past samples per chain is
                                kept on the device; 0 = off).  The ring
                                restarts at dm_set_params and dm_load_state */
} dm_params;

/* Create a context for n_chains chains; beads[c] >= 2 is the number of beads
   of chain c (host array, at most 2048).  pos0 (host, SoA, sum_c 3*beads[c] doubles, in
   units of d) is the initial conformation; it is transformed to mode
   amplitudes in FP64, Eq. (c1).  pos0 may be NULL: the first dm_set_params
   then builds the initial state of the batched workloads (the paper
   prescribes none): chain c straight with bond length b = 1/(1 - 2 nu) along
   a direction uniform on the unit sphere (Philox tag 5, index 0, step 0:
   cos(theta) = 2 U0 - 1, phi = 2 pi U1 from words 0 and 1), every coordinate
   jittered by 0.01 b times a normal (tag 4, index bead n, component a, step
   0); until then every call that reads or advances the state returns
   DM_ESTATE (dm_load_state supplies a state instead).  Chains are grouped into buckets of equal
   length internally; chain c keeps Philox chain index c.  precision is one
   of DM_FP64, DM_FP32, DM_BF16X3 (the fused paths need an even number of
   beads, at most 512).  hip_stream is a hipStream_t (NULL = the null stream).
   On success *out owns the context.  Errors: DM_EINVAL, DM_ENOMEM, DM_EHIP. */
int dm_init_chains(dm_ctx **out, int32_t n_chains, const int32_t *beads,
                   const double *pos0, uint64_t seed, int32_t precision,
                   void *hip_stream);

/* Set model parameters and time steps (Secs. II, III, VII.B); builds the mode
   tables of Eqs. (c8), (c9), (e9), (d3), (d6), (f2) in FP64 on the host for
   every chain length and uploads them.  May be called again to change
   parameters.  Errors: DM_EINVAL for nu outside [0, 1/2) (stability of
   Eq. a2), T* <= 0, dt <= 0, or a chain length missing from lengths[]. */
int dm_set_params(dm_ctx *ctx, const dm_params *p);

/* Advance every chain by n_steps mode steps (Sec. IV, Eqs. e10, d3, d6, f2):
   inverse transform of the internal modes to bond vectors, the nonlinear
   bond force g_n = u_n (1/|u_n| - (1-2nu)) (Eqs. e4, e11), forward
   transform to Delta H_p, and the per-mode update with Philox noise; the
   centre-of-mass mode R_0 is a free random walk (FP64).  Asynchronous.
   Errors: DM_ESTATE before dm_set_params, DM_ENONFINITE (check_finite). */
int dm_step_modes(dm_ctx *ctx, int64_t n_steps);

/* Advance every chain by n_steps bead-space Euler steps of reduced length
   dtau (Eqs. b3-b5): r_n += dtau (h_{n+1} - h_n) + sqrt(2 T* dtau) eta_n with
   h_n = (|u_n| - 1) u_n/|u_n| - nu (u_{n-1} + u_{n+1}), in FP64.  The
   state is converted from and back to mode amplitudes once per call.
   The scheme is unstable for dtau above about 0.3 (Sec. III.A).
   Errors: DM_ESTATE, DM_EINVAL (dtau <= 0), DM_ENONFINITE (check_finite). */
int dm_step_euler(dm_ctx *ctx, int64_t n_steps, double dtau);

/* The nu -> 0 limit (Sec. VI.A, Eqs. y2-y14): the inextensible wormlike chain
   in the bending units tau-bar = nu tau, T-bar = T* / nu, Hamiltonian
   -sum_n u_n . u_{n+1} with bonds of unit length held by tensions f_n.  The
   bonds of every chain are first scaled to unit length (positions then in
   units of the bond length); each step moves bead n by
   (-f_n u^m_n + f_{n+1} u^m_{n+1} + h_{n+1} - h_n) dt_bar
   + sqrt(2 T_bar dt_bar) eta_n with the bending gradient
   h_n = -(u^m_{n-1} + u^m_{n+1}) and the tensions from the tridiagonal
   system (u_n + u'_n) . du_n = 0, all at the midpoint bonds
   u^m_n = (u_n + u'_n)/|u_n + u'_n| (Eq. y14).  The cycle starts from
   u' = u and is repeated until it converges: at most iters times, and with
   tol > 0 it stops after the first cycle that changes no component of any
   u'_n by more than tol (tol = 0: exactly iters cycles; 8 cycles hold the
   bonds at unit length to ~1e-12 per step at dt_bar = 1e-3).  FP64: one
   wavefront per chain with the chain in registers up to M = 64 and in LDS
   up to M = 341 (tensions by cyclic reduction), one thread per chain beyond
   (Thomas sweep, global scratch allocated on first use); noise tag 3
   (index = bead).  midpoint != 0: forces and tensions at the midpoint
   bonds u^m_n as above (Eq. y14, the time-symmetric form); midpoint == 0:
   at the bonds u_n of the start of the step, the constraint rows still
   (u_n + u'_n) . du_n = 0 (the cycle of Eqs. y9-y13 as first written).
   The state is converted from and back to mode amplitudes once per call.
   Without metric pseudo-forces the scheme samples the constrained ensemble
   exp(-H/T_bar) sqrt(det G), G the constraint metric.  Errors: DM_EINVAL
   (n_steps < 0, dt_bar or T_bar <= 0, iters outside 1..64, tol < 0 or not
   finite), DM_ENONFINITE. */
int dm_step_wlc(dm_ctx *ctx, int64_t n_steps, double dt_bar, double T_bar,
                int32_t iters, double tol, int32_t midpoint);

/* Metropolis Monte Carlo in the mode representation, the paper's benchmark
   for equilibrium values (Sec. V.B: large steps in the slow modes, small in
   the fast ones).  One sweep proposes, for p = 1..M-1 and component
   a = x, y, z in order, R_p^a += delta, delta uniform on (-s_p, s_p) with
   s_p = step_scale * sqrt(T* / zeta^l_p) (the width of mode p under the
   harmonic Hamiltonian, Eqs. c6, c9), accepted with probability
   min(1, exp(-dH'/T*)) for the reduced Hamiltonian H' of Eq. (b3); the
   centre of mass is unchanged.  Philox counter (p, chain, sweep, a, tag 2):
   word 0 gives delta = s_p (2 U0 - 1), word 1 the uniform U1 of the test
   U1 < exp(-dH'/T*), U = (x + 1/2) 2^-32.  FP64 on every precision (the
   fused state is converted in and out).  Sweeps advance the step counter;
   observables are accumulated every sample_every sweeps as after mode
   steps.  step_scale = 3 accepts about 56 % of the proposals.  *accepted
   (host, may be NULL) receives the accepted proposals of the call, summed
   over chains.  Synchronises the stream.  Errors: DM_ESTATE, DM_EINVAL
   (n_sweeps < 0, step_scale < 0, M > 1365), DM_ENONFINITE (check_finite). */
int dm_step_mc(dm_ctx *ctx, int64_t n_sweeps, double step_scale,
               int64_t *accepted);

/* Observables of Sec. V.B.  which = OR of DM_OBS_* bits; the selected blocks
   are written to out_host in the order CHAIN, MODES, ACCUM (see the layout
   macros above).  out_len is the capacity in doubles; dm_observables_size()
   gives the length needed.  Synchronises the stream.
   Errors: DM_EINVAL if out_len is too small. */
int dm_observables(dm_ctx *ctx, int32_t which, double *out_host,
                   size_t out_len);
int dm_observables_size(const dm_ctx *ctx, int32_t which, size_t *len);

/* Bead positions (SoA, all chains, units of d) from the current mode
   amplitudes, Eq. (c1), in FP64.  dst is a host pointer, or a device pointer
   when dst_on_device != 0.  Synchronises the stream. */
int dm_get_positions(dm_ctx *ctx, double *dst, int32_t dst_on_device);

/* Mode amplitudes R_p (SoA, all chains, p = 0..M_c-1) in FP64.  Host dst. */
int dm_get_modes(dm_ctx *ctx, double *dst_host);

/* Serialise / restore the full state (mode amplitudes, step counters,
   accumulators).  Philox is counter based, so a restored run continues
   bit-identically.  dm_save_state with buf == NULL returns the size in *len. */
int dm_save_state(dm_ctx *ctx, void *buf, size_t *len);
int dm_load_state(dm_ctx *ctx, const void *buf, size_t len);

/* Global step counter (mode and Euler steps share it: it is the Philox
   step index). */
int dm_get_step(const dm_ctx *ctx, int64_t *step);

/* Tile shapes of the fused launch (all zero except M and chains for
   DM_FP64).  Every length bucket advances in the same kernel launch: one
   workgroup item per tpw tiles of 5 chains, items ordered by decreasing cost
   so that in-order dispatch to free CUs is a longest-first schedule.  With
   out == NULL only *n_buckets is set.  Errors: DM_EINVAL if len is below
   DM_NTILING * n_buckets. */
int dm_get_tiling(const dm_ctx *ctx, double *out, size_t len, int32_t *n_buckets);

/* Text of the last autotuning (one line per timed tile shape), or "". */
const char *dm_tuning_report(const dm_ctx *ctx);

/* Model parameters of a coarse-grained chain (Sec. VI): one bead per k
   basepairs, on the force-extension curve of Eq. (x1) with r = l_p / a and
   y = l_p K_0 / kT (Eq. x2).  With r_k = r / k and y unchanged, Eq. (x4):
       T*_k = (2 r^2 + k^2 y) r / (k^3 y^2),  nu_k = r^2 / (2 r^2 + k^2 y)
   (k = 1 is the fit of Eq. x3).  The bond rest length of the reduced model
   is b_k = 1/(1 - 2 nu_k) in units of d_k = k a / b_k.  Host only, no
   context.  Errors: DM_EINVAL for r <= 0, y <= 0, k < 1 or NULL outputs. */
int dm_coarse_grain(double r, double y, int32_t k, double *T_star_k, double *nu_k);

/* Time unit of that coarse-grained chain (Sec. VII.B, Eq. g2 with a_k = k a and
   the friction of k basepairs, xi_k = k xi): real time t = c_k tau_k with
       c_k = k^3 T*_k (1 - 2 nu_k)^2   [in units of a^2 xi / kT],
   a the basepair spacing and xi the friction per basepair.  Host only.
   Errors: as dm_coarse_grain. */
int dm_coarse_grain_time(double r, double y, int32_t k, double *c_k);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
   plain-form mode step of dm_step_modes for one chain length, without a
   context.  R_dev (device, caller-owned, 16-byte aligned) holds n_chains
   chains of M mode amplitudes R_p in the SoA layout (3*M doubles per
   chain, p = 0..M-1) and is advanced in place by n_steps steps at Philox
   steps step0 .. step0 + n_steps - 1; chain j draws its noise as chain index
   chain0 + j, so a call reproduces dm_step_modes on those chains of a
   context.  Reduced units: T_star, nu, dtau (= Delta tau), gamma_dot; tables
   and coefficients are built on the device at every call.  No allocation:
   the tables, the chain indices and the two work buffers live in one fixed
   device array of DM_STATIC_SCRATCH_BYTES per GPU, held from the first use
   until the process ends; it needs 8 (2 M^2 + 3 M + 6 M n_chains) +
   4 n_chains bytes (each part rounded up to 256), e.g. 4096 chains of 256
   beads.  Calls that overlap on one GPU share that array and race; calls on
   one stream are ordered.  Asynchronous on hip_stream.  Errors (message in
   dm_last_error(NULL)): DM_EINVAL for a size beyond the array, M outside
   2..2048, n_chains < 1, nu outside [0, 1/2), T* or dtau not positive,
   n_steps or step0 < 0, a misaligned or NULL R_dev; DM_EHIP. */
#define DM_STATIC_SCRATCH_BYTES (64u << 20)
int dm_step_modes_f64_static(double *R_dev, int32_t n_chains, int32_t M,
                             double T_star, double nu, double dtau,
                             double gamma_dot, int32_t nonlinear, uint64_t seed,
                             uint32_t chain0, int64_t step0, int64_t n_steps,
                             void *hip_stream);

/* Synchronise the context's stream. */
int dm_sync(dm_ctx *ctx);

int dm_destroy(dm_ctx *ctx);

/* Message of the last error on this context (ctx may be NULL for errors of
   dm_init_chains).  Valid until the next call on the context. */
const char *dm_last_error(const dm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* DNAMODES_H */
