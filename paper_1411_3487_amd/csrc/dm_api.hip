// dm_api.hip -- context, buckets and the C ABI of libdnamodes (dnamodes.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/dnamodes.h"
#include "dm_fused.h"
#include "dm_internal.h"
#include "dm_rng.h"
#include "dm_tables.h"

namespace {

thread_local std::string g_init_error;

// Longest sampling block the FP64 plain form replays as a graph (it holds
// four kernel nodes per step and length bucket).
constexpr int kMaxPlainGraphSteps = 256;

struct Bucket {
    int M = 0;
    int n = 0;                       // chains
    std::vector<int32_t> ids;        // caller chain index of each local chain
    std::vector<int64_t> user_off;   // SoA offset (doubles) of each chain in caller order
    double dtau = 0.0;
    // device
    int32_t *d_ids = nullptr;
    int64_t *d_off = nullptr;
    double *d_Ainv = nullptr;        // phi with column p = 0 zeroed (inverse, internal)
    double *d_Apos = nullptr;        // phi (inverse, all modes)
    double *d_Afwd = nullptr;        // phi^T (forward)
    double *d_E = nullptr, *d_C = nullptr, *d_W = nullptr;
    double *d_R64 = nullptr;         // n*3*M full mode amplitudes (FP64 state / scratch)
    double *d_r = nullptr;           // n*3*M positions / workspace
    double *d_F = nullptr;           // n*3*M forces
    double *d_dH = nullptr;          // n*3*M coupling
    double *d_obs = nullptr;         // n*16
    double *d_m2 = nullptr;          // n*M
    double *d_acc = nullptr;         // n*acc_width(M)
    double *d_accsum = nullptr;      // acc_width(M)
    double *d_tumble = nullptr;      // 2n: tumbling state, step of the last tumble + 1
    double *d_ring = nullptr;        // n * 2^(K-1) * 9: past (L, u_m, d) for the correlations
    double *d_ccount = nullptr;      // n: samples written to the ring
    // Metropolis sampler (allocated on first use)
    double *d_chiT = nullptr;        // chi_{n,p} at [p][n-1], M x (M-1)
    double *d_mcstep = nullptr;      // proposal half-widths s_p
    int64_t *d_mcacc = nullptr;      // accepted proposals per chain
    double *d_wlc = nullptr;         // scratch of the inextensible limit
    std::vector<double> zeta_l;      // host zeta^l_p of the current parameters
    std::vector<double> mcstep_h;    // host copy of s_p (kept alive for the upload)
    double *d_cm0 = nullptr;         // n*3
    dm::FusedBucket fused;           // reduced-precision state and tables
};

}  // namespace

namespace dm {
void set_ctxless_error(const char *msg) { g_init_error = msg; }
}  // namespace dm

struct dm_ctx {
    int nchains = 0;
    int precision = DM_FP64;
    uint64_t seed = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<int32_t> beads;
    std::vector<int64_t> offset;     // SoA offset of chain c (doubles)
    size_t total = 0;                // sum of 3*beads
    std::vector<Bucket> buckets;
    bool have_params = false;
    bool pending_init = false;       // created without positions: state built at set_params
    double T_star = 0, nu = 0, gamma_dot = 0;
    int nonlinear = 1, sample_every = 0, check_finite = 0;
    int64_t step = 0;
    int *d_flag = nullptr;
    // fused paths: one launch over all buckets, and the captured graph of
    // one sampling block (fused launch, step-counter advance, observables)
    dm::FusedPlan plan;
    int use_graphs = 0, autotune = 0, corr_lags = 0;
    int64_t *d_step = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_steps = 0;
    // deferred observables: runs of several sampling blocks replay "first"
    // (launch, snapshot of the state, counter advance) and then "steady",
    // where the observables of the previous block's snapshot run on a second
    // stream beside the launch, on the compute units the launch leaves idle
    hipStream_t cap_stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraph_t g_first = nullptr, g_steady = nullptr;
    hipGraphExec_t x_first = nullptr, x_steady = nullptr;
    int overlap_steps = 0;
    int ncu = 0;
    int obs_wg = 0;      // grid cap of the deferred observation kernels
    int ov_se = 0;       // sampling interval the overlap decision was taken for
    bool ov_use = false; // that decision
    std::string tune_report;
    std::string err;
};

namespace {

int fail(dm_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_init_error = buf;
    return code;
}

#define DM_HIP(ctx, expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), DM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

template <typename T>
int dalloc(dm_ctx *ctx, T **p, size_t count)
{
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * count);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(ctx, DM_ENOMEM, "hipMalloc of %zu bytes failed: %s", sizeof(T) * count,
                    hipGetErrorString(e));
    }
    return DM_OK;
}

void free_bucket(Bucket &b)
{
    void *ptrs[] = {b.d_ids, b.d_off,  b.d_Ainv, b.d_Apos, b.d_Afwd, b.d_E,   b.d_C,
                    b.d_W,   b.d_R64, b.d_r,    b.d_F,    b.d_dH,   b.d_obs, b.d_m2,
                    b.d_acc, b.d_accsum, b.d_cm0, b.d_tumble, b.d_chiT, b.d_mcstep,
                    b.d_mcacc, b.d_ring, b.d_ccount, b.d_wlc};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    dm::fused_free(b.fused);
}

bool fused_precision(int p) { return p == DM_FP32 || p == DM_BF16X3; }

// Positions of all chains of a bucket (FP64, bucket order) into b.d_r.
int bucket_positions(dm_ctx *ctx, Bucket &b, hipStream_t st)
{
    if (fused_precision(ctx->precision))
        DM_HIP(ctx, dm::fused_unpack_modes(b.fused, b.d_R64, b.M, b.n, st));
    DM_HIP(ctx, dm::launch_gemm_f64(b.d_Apos, b.d_R64, b.d_r, b.M, 3 * b.n, st));
    return DM_OK;
}

// Observables of the current state; with accumulate != 0 also the sums and
// the tumbling state, at the step held in ctx->d_step (set here unless the
// call is being captured, where the block's own counter kernel keeps it).
int observe(dm_ctx *ctx, int accumulate, hipStream_t st, bool captured = false,
            bool from_snapshot = false, int max_wg = 0)
{
    if (accumulate && !captured) DM_HIP(ctx, dm::fused_set_step(ctx->d_step, ctx->step, st));
    for (Bucket &b : ctx->buckets) {
        if (fused_precision(ctx->precision)) {
            DM_HIP(ctx, dm::fused_observe(b.fused, b.M, b.d_obs, b.d_m2, b.d_acc, b.d_cm0,
                                          b.d_tumble, b.d_tumble + b.n, ctx->d_step, b.d_ring,
                                          b.d_ccount, ctx->corr_lags, accumulate, st,
                                          from_snapshot, max_wg));
            continue;
        }
        int rc = bucket_positions(ctx, b, st);
        if (rc) return rc;
        DM_HIP(ctx, dm::launch_chain_obs(b.d_r, b.d_R64, b.d_obs, b.d_m2, b.d_acc, b.d_cm0,
                                         b.d_tumble, b.d_tumble + b.n, ctx->d_step, b.d_ring,
                                         b.d_ccount, ctx->corr_lags, b.M, b.n, accumulate, st));
    }
    return DM_OK;
}

void drop_block_graph(dm_ctx *ctx)
{
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_steps = 0;
}

void drop_overlap_graphs(dm_ctx *ctx)
{
    for (hipGraphExec_t *x : {&ctx->x_first, &ctx->x_steady})
        if (*x) (void)hipGraphExecDestroy(*x), *x = nullptr;
    for (hipGraph_t *g : {&ctx->g_first, &ctx->g_steady})
        if (*g) (void)hipGraphDestroy(*g), *g = nullptr;
    ctx->overlap_steps = 0;
}

void drop_graph(dm_ctx *ctx)
{
    drop_block_graph(ctx);
    drop_overlap_graphs(ctx);
    ctx->ov_se = 0;  // the overlap decision depends on the plan
}

// Deferred observables pay off when the launch leaves compute units idle
// (one workgroup item per compute unit, all in flight at once, at least 16
// units to spare: the observation kernels are capped to the spare units
// less 3, so the launch's items never wait for them) and when the capped
// observation is not slower than the block it hides behind: it is timed
// once per sampling interval on the live state without accumulating (that
// rewrites only the current-state observables, with the same values), and
// compared with the block's estimated time (the longest item's step time,
// measured by the autotuner or modelled, times the steps per block).
int overlap_pays(dm_ctx *ctx, int se, bool *use)
{
    if (ctx->ov_se == se) {
        *use = ctx->ov_use;
        return DM_OK;
    }
    const int spare = ctx->ncu - ctx->plan.nitems - 3;
    ctx->ov_se = se;
    ctx->ov_use = false;
    if (ctx->ncu > 0 && spare >= 16) {
        ctx->obs_wg = spare;
        double step_us = 0.0;
        for (Bucket &b : ctx->buckets) step_us = std::max(step_us, dm::fused_item_us(b.fused));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        DM_HIP(ctx, hipEventCreate(&e0));
        hipError_t e = hipEventCreate(&e1);
        int rc = DM_OK;
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
        if (e == hipSuccess) rc = observe(ctx, 0, ctx->stream, false, false, ctx->obs_wg);
        if (e == hipSuccess && rc == DM_OK) e = hipEventRecord(e1, ctx->stream);
        if (e == hipSuccess && rc == DM_OK) e = hipEventSynchronize(e1);
        if (e == hipSuccess && rc == DM_OK) e = hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (rc != DM_OK) return rc;
        if (e != hipSuccess)
            return fail(ctx, DM_EHIP, "timing the observables failed: %s", hipGetErrorString(e));
        ctx->ov_use = 1e3 * ms <= step_us * se;
    }
    *use = ctx->ov_use;
    return DM_OK;
}

// Capture the two graphs of deferred observables (see dm_ctx).
int capture_overlap(dm_ctx *ctx, int steps)
{
    drop_overlap_graphs(ctx);
    for (Bucket &b : ctx->buckets) DM_HIP(ctx, dm::fused_snapshot_alloc(b.fused));
    if (!ctx->cap_stream)
        DM_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    if (!ctx->cap_stream2)
        DM_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream2, hipStreamNonBlocking));
    if (!ctx->ev_fork) DM_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    if (!ctx->ev_join) DM_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    hipStream_t s1 = ctx->cap_stream, s2 = ctx->cap_stream2;
    for (int which = 0; which < 2; ++which) {
        DM_HIP(ctx, hipStreamBeginCapture(s1, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        int rc = DM_OK;
        if (which == 1) {  // the previous block's sample beside this block's launch
            e = hipEventRecord(ctx->ev_fork, s1);
            if (e == hipSuccess) e = hipStreamWaitEvent(s2, ctx->ev_fork, 0);
            if (e == hipSuccess) rc = observe(ctx, 1, s2, true, true, ctx->obs_wg);
        }
        if (e == hipSuccess && rc == DM_OK)
            e = dm::fused_launch(ctx->plan, ctx->seed, 0, ctx->d_step, steps, ctx->nonlinear, s1);
        if (which == 1) {
            const hipError_t e1 = hipEventRecord(ctx->ev_join, s2);
            const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(s1, ctx->ev_join, 0) : e1;
            if (e == hipSuccess) e = e2;
        }
        for (Bucket &b : ctx->buckets)
            if (e == hipSuccess) e = dm::fused_snapshot(b.fused, s1);
        if (e == hipSuccess) e = dm::fused_advance_step(ctx->d_step, steps, s1);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(s1, &g);
        if (e != hipSuccess || rc != DM_OK || ec != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            drop_overlap_graphs(ctx);
            if (rc != DM_OK) return rc;
            return fail(ctx, DM_EHIP, "graph capture failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : ec));
        }
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            drop_overlap_graphs(ctx);
            return fail(ctx, DM_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
        }
        (which ? ctx->g_steady : ctx->g_first) = g;
        (which ? ctx->x_steady : ctx->x_first) = x;
    }
    ctx->overlap_steps = steps;
    return DM_OK;
}

// One FP64 plain-form mode step of one bucket on stream st at Philox step
// k, or (step_dev non-null, inside a captured block) *step_dev + k.
int plain_step(dm_ctx *ctx, Bucket &b, int64_t k, hipStream_t st,
               const int64_t *step_dev = nullptr)
{
    const int ncol = 3 * b.n;
    if (ctx->nonlinear) {
        DM_HIP(ctx, dm::launch_gemm_f64(b.d_Ainv, b.d_R64, b.d_r, b.M, ncol, st));
        DM_HIP(ctx, dm::launch_stencil_f64(b.d_r, b.d_F, b.M, b.n, 1.0 - 2.0 * ctx->nu, st));
        DM_HIP(ctx, dm::launch_gemm_f64(b.d_Afwd, b.d_F, b.d_dH, b.M, ncol, st));
    }
    DM_HIP(ctx, dm::launch_mode_update_f64(b.d_R64, b.d_dH, b.d_E, b.d_C, b.d_W, b.d_ids, b.M,
                                           b.n, ctx->seed, step_dev, k,
                                           ctx->gamma_dot * b.dtau, ctx->nonlinear, st));
    return DM_OK;
}

// Capture one sampling block of `steps` fused steps: the launch reads its
// Philox step from ctx->d_step, a one-thread kernel advances it, then the
// observables are accumulated.  No memset nodes (plain kernels only).
int capture_block(dm_ctx *ctx, int steps)
{
    drop_block_graph(ctx);
    if (!ctx->cap_stream)
        DM_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    DM_HIP(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    int rc = DM_OK;
    if (fused_precision(ctx->precision)) {
        e = dm::fused_launch(ctx->plan, ctx->seed, 0, ctx->d_step, steps, ctx->nonlinear,
                             ctx->cap_stream);
    } else {
        // the plain form's four launches per step and bucket, each update
        // reading its Philox step from the device counter
        for (int s = 0; s < steps && rc == DM_OK; ++s)
            for (Bucket &b : ctx->buckets)
                if (rc == DM_OK) rc = plain_step(ctx, b, s, ctx->cap_stream, ctx->d_step);
    }
    if (e == hipSuccess && rc == DM_OK)
        e = dm::fused_advance_step(ctx->d_step, steps, ctx->cap_stream);
    if (e == hipSuccess && rc == DM_OK) rc = observe(ctx, 1, ctx->cap_stream, true);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &g);
    if (e != hipSuccess || rc != DM_OK || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (rc != DM_OK) return rc;
        return fail(ctx, DM_EHIP, "graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : ec));
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(ctx, DM_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    ctx->graph = g;
    ctx->graph_exec = x;
    ctx->graph_steps = steps;
    return DM_OK;
}

int build_plan(dm_ctx *ctx)
{
    std::vector<const dm::FusedBucket *> fb;
    for (Bucket &b : ctx->buckets) fb.push_back(&b.fused);
    DM_HIP(ctx, dm::fused_plan(ctx->plan, fb, 0, ctx->stream));
    return DM_OK;
}

int check_state(dm_ctx *ctx)
{
    DM_HIP(ctx, hipMemsetAsync(ctx->d_flag, 0, sizeof(int), ctx->stream));
    for (Bucket &b : ctx->buckets) {
        if (fused_precision(ctx->precision))
            DM_HIP(ctx, dm::fused_check_finite(b.fused, b.M, b.n, ctx->d_flag, ctx->stream));
        else
            DM_HIP(ctx, dm::launch_check_finite_f64(b.d_R64, (size_t)3 * b.M * b.n, ctx->d_flag,
                                                    ctx->stream));
    }
    int flag = 0;
    DM_HIP(ctx, hipMemcpyAsync(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost,
                               ctx->stream));
    DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (flag) return fail(ctx, DM_ENONFINITE, "state is not finite after step %lld",
                          (long long)ctx->step);
    return DM_OK;
}

// Centre of mass of each of n chains of M beads (SoA positions).
void centres(const std::vector<double> &pos, int M, int n, std::vector<double> &cm)
{
    for (int j = 0; j < n; ++j)
        for (int a = 0; a < 3; ++a) {
            double s = 0.0;
            for (int i = 0; i < M; ++i) s += pos[(size_t)3 * M * j + (size_t)a * M + i];
            cm[3 * j + a] = s / M;
        }
}

// The initial state of a context created without positions (the batched
// workloads' recipe; the paper prescribes none): chain c straight with bond
// length bl = 1/(1 - 2 nu) along a direction uniform on the unit sphere
// (Philox tag kTagOrient, block 0: cos(theta) = 2 U0 - 1, phi = 2 pi U1),
// every coordinate jittered by 0.01 bl times a normal (tag kTagInit, index
// bead n, component a), all at step 0.  Built on the host in FP64, then
// transformed to mode amplitudes as an initial conformation given by the
// caller would be.
int config_state(dm_ctx *ctx, double nu)
{
    const double bl = 1.0 / (1.0 - 2.0 * nu), scale = 2.3283064365386962890625e-10;
    const double two_pi = 6.283185307179586476925286766559;
    for (Bucket &b : ctx->buckets) {
        const int M = b.M;
        std::vector<double> pos((size_t)3 * M * b.n), cm0((size_t)3 * b.n);
        for (int j = 0; j < b.n; ++j) {
            const uint32_t chain = (uint32_t)b.ids[j];
            const dm::Block4 o = dm::noise_bits(ctx->seed, 0u, chain, 0, 0u, dm::kTagOrient);
            const double u0 = ((double)o.v[0] + 0.5) * scale, u1 = ((double)o.v[1] + 0.5) * scale;
            const double ct = 2.0 * u0 - 1.0, st = std::sqrt(1.0 - ct * ct), ph = two_pi * u1;
            const double e[3] = {st * std::cos(ph), st * std::sin(ph), ct};
            double *r = &pos[(size_t)3 * M * j];
            for (int a = 0; a < 3; ++a)
                for (int q = 0; 4 * q < M; ++q) {
                    double z[4];
                    dm::normals4_f64(dm::noise_bits(ctx->seed, (uint32_t)q, chain, 0, (uint32_t)a,
                                                    dm::kTagInit),
                                     z);
                    for (int i = 4 * q; i < M && i < 4 * q + 4; ++i)
                        r[(size_t)a * M + i] = i * bl * e[a] + 0.01 * bl * z[i - 4 * q];
                }
        }
        centres(pos, M, b.n, cm0);
        DM_HIP(ctx, hipMemcpyAsync(b.d_r, pos.data(), sizeof(double) * pos.size(),
                                   hipMemcpyHostToDevice, ctx->stream));
        DM_HIP(ctx, hipMemcpyAsync(b.d_cm0, cm0.data(), sizeof(double) * cm0.size(),
                                   hipMemcpyHostToDevice, ctx->stream));
        DM_HIP(ctx, dm::launch_gemm_f64(b.d_Afwd, b.d_r, b.d_R64, M, 3 * b.n, ctx->stream));
        if (fused_precision(ctx->precision))
            DM_HIP(ctx, dm::fused_pack_modes(b.fused, b.d_R64, M, b.n, ctx->stream));
        DM_HIP(ctx, hipStreamSynchronize(ctx->stream));  // the host arrays die here
    }
    ctx->pending_init = false;
    return DM_OK;
}

}  // namespace

extern "C" {

int dm_init_chains(dm_ctx **out, int32_t n_chains, const int32_t *beads, const double *pos0,
                   uint64_t seed, int32_t precision, void *hip_stream)
{
    g_init_error.clear();
    if (!out) return fail(nullptr, DM_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_chains <= 0) return fail(nullptr, DM_EINVAL, "n_chains must be positive");
    if (!beads) return fail(nullptr, DM_EINVAL, "beads must be non-NULL");
    if (precision != DM_FP64 && !fused_precision(precision))
        return fail(nullptr, DM_EINVAL, "unknown precision %d", precision);
    for (int c = 0; c < n_chains; ++c) {
        const int M = beads[c];
        if (M < 2) return fail(nullptr, DM_EINVAL, "chain %d has %d beads (need >= 2)", c, M);
        if (M > 2048)
            return fail(nullptr, DM_EINVAL, "chain %d has %d beads (at most 2048)", c, M);
        if (fused_precision(precision) && !dm::fused_supports(M))
            return fail(nullptr, DM_EINVAL,
                        "chain %d: %d beads not supported by the fused path (even, 4..512)",
                        c, M);
    }
    dm_ctx *ctx = new dm_ctx();
    ctx->nchains = n_chains;
    ctx->pending_init = pos0 == nullptr;
    ctx->precision = precision;
    ctx->seed = seed;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return fail(nullptr, DM_EHIP, "no HIP device");
    }
    if (hipDeviceGetAttribute(&ctx->ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) !=
        hipSuccess)
        ctx->ncu = 0;  // deferred observables off
    ctx->beads.assign(beads, beads + n_chains);
    ctx->offset.resize(n_chains);
    int64_t off = 0;
    std::map<int, int> bucket_of;
    for (int c = 0; c < n_chains; ++c) {
        ctx->offset[c] = off;
        off += 3 * (int64_t)beads[c];
        bucket_of[beads[c]] = 0;
    }
    ctx->total = (size_t)off;
    int nb = 0;
    for (auto &kv : bucket_of) kv.second = nb++;
    ctx->buckets.resize(nb);
    for (auto &kv : bucket_of) ctx->buckets[kv.second].M = kv.first;
    for (int c = 0; c < n_chains; ++c) {
        Bucket &b = ctx->buckets[bucket_of[beads[c]]];
        b.ids.push_back(c);
        b.user_off.push_back(ctx->offset[c]);
        b.n++;
    }
    int rc = DM_OK;
    auto bail = [&](int code) {
        std::string msg = ctx->err;
        for (Bucket &b : ctx->buckets) free_bucket(b);
        if (ctx->d_flag) (void)hipFree(ctx->d_flag);
        if (ctx->d_step) (void)hipFree(ctx->d_step);
        delete ctx;
        g_init_error = msg;
        return code;
    };
    if ((rc = dalloc(ctx, &ctx->d_flag, 1))) return bail(rc);
    if ((rc = dalloc(ctx, &ctx->d_step, 1))) return bail(rc);
    std::vector<double> phi, tmp;
    for (Bucket &b : ctx->buckets) {
        const size_t MM = (size_t)b.M * b.M, S = (size_t)3 * b.M * b.n;
        if ((rc = dalloc(ctx, &b.d_ids, b.n)) || (rc = dalloc(ctx, &b.d_off, b.n)) ||
            (rc = dalloc(ctx, &b.d_Ainv, MM)) || (rc = dalloc(ctx, &b.d_Apos, MM)) ||
            (rc = dalloc(ctx, &b.d_Afwd, MM)) || (rc = dalloc(ctx, &b.d_E, b.M)) ||
            (rc = dalloc(ctx, &b.d_C, b.M)) || (rc = dalloc(ctx, &b.d_W, b.M)) ||
            (rc = dalloc(ctx, &b.d_R64, S)) || (rc = dalloc(ctx, &b.d_r, S)) ||
            (rc = dalloc(ctx, &b.d_F, S)) || (rc = dalloc(ctx, &b.d_dH, S)) ||
            (rc = dalloc(ctx, &b.d_obs, (size_t)16 * b.n)) ||
            (rc = dalloc(ctx, &b.d_m2, (size_t)b.M * b.n)) ||
            (rc = dalloc(ctx, &b.d_acc, (size_t)dm::acc_width(b.M) * b.n)) ||
            (rc = dalloc(ctx, &b.d_accsum, (size_t)dm::acc_width(b.M))) ||
            (rc = dalloc(ctx, &b.d_tumble, (size_t)2 * b.n)) ||
            (rc = dalloc(ctx, &b.d_cm0, (size_t)3 * b.n)))
            return bail(rc);
        dm::rouse_matrix(b.M, phi);
        std::vector<double> ainv(phi), afwd(MM);
        for (int n = 0; n < b.M; ++n) {
            ainv[(size_t)n * b.M] = 0.0;
            for (int p = 0; p < b.M; ++p) afwd[(size_t)p * b.M + n] = phi[(size_t)n * b.M + p];
        }
        std::vector<double> pos, cm0((size_t)3 * b.n, 0.0);
        if (pos0) {
            pos.resize(S);
            for (int j = 0; j < b.n; ++j)
                std::memcpy(&pos[(size_t)3 * b.M * j], pos0 + b.user_off[j],
                            sizeof(double) * 3 * b.M);
            centres(pos, b.M, b.n, cm0);
        }
        hipError_t e = hipSuccess;
        auto up = [&](void *d, const void *h, size_t bytes) {
            if (e == hipSuccess)
                e = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, ctx->stream);
        };
        up(b.d_ids, b.ids.data(), sizeof(int32_t) * b.n);
        up(b.d_off, b.user_off.data(), sizeof(int64_t) * b.n);
        up(b.d_Ainv, ainv.data(), sizeof(double) * MM);
        up(b.d_Apos, phi.data(), sizeof(double) * MM);
        up(b.d_Afwd, afwd.data(), sizeof(double) * MM);
        if (pos0) up(b.d_r, pos.data(), sizeof(double) * S);
        up(b.d_cm0, cm0.data(), sizeof(double) * 3 * b.n);
        if (e == hipSuccess)
            e = hipMemsetAsync(b.d_acc, 0, sizeof(double) * dm::acc_width(b.M) * b.n,
                               ctx->stream);
        if (e == hipSuccess)
            e = hipMemsetAsync(b.d_tumble, 0, sizeof(double) * 2 * b.n, ctx->stream);
        if (e == hipSuccess && pos0)
            e = dm::launch_gemm_f64(b.d_Afwd, b.d_r, b.d_R64, b.M, 3 * b.n, ctx->stream);
        if (e == hipSuccess && fused_precision(precision)) {
            e = dm::fused_alloc(b.fused, b.M, b.n, precision == DM_BF16X3);
            b.fused.ids = b.d_ids;
            if (e == hipSuccess && pos0)
                e = dm::fused_pack_modes(b.fused, b.d_R64, b.M, b.n, ctx->stream);
        }
        // the host staging buffers die with this scope: finish the uploads first
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            fail(ctx, DM_EHIP, "init upload failed: %s", hipGetErrorString(e));
            return bail(DM_EHIP);
        }
    }
    *out = ctx;
    return DM_OK;
}

int dm_set_params(dm_ctx *ctx, const dm_params *p)
{
    if (!ctx) return DM_EINVAL;
    if (!p) return fail(ctx, DM_EINVAL, "params is NULL");
    double T_star, nu, tunit = 1.0;
    if (p->lambda > 0.0) {
        if (!(p->kappa >= 0.0) || !(p->kT > 0.0) || !(p->a > 0.0) || !(p->xi > 0.0))
            return fail(ctx, DM_EINVAL, "physical parameters must be positive");
        nu = p->kappa / p->lambda;
        const double b = 1.0 / (1.0 - 2.0 * nu), d = p->a / b;
        T_star = p->kT / (p->lambda * d * d);
        tunit = p->xi / p->lambda;  // ps per reduced time unit
    } else {
        T_star = p->T_star;
        nu = p->nu;
    }
    if (!(nu >= 0.0 && nu < 0.5))
        return fail(ctx, DM_EINVAL, "nu = %g outside [0, 1/2)", nu);
    if (!(T_star > 0.0) || !std::isfinite(T_star))
        return fail(ctx, DM_EINVAL, "T* = %g must be positive", T_star);
    if (p->n_lengths <= 0 || !p->lengths || !p->dt)
        return fail(ctx, DM_EINVAL, "lengths / dt tables are empty");
    if (p->sample_every < 0) return fail(ctx, DM_EINVAL, "sample_every must be >= 0");
    if (p->tiles_per_wg < 0 || p->tiles_per_wg > 4 || p->table_mode < 0 || p->table_mode > 4)
        return fail(ctx, DM_EINVAL, "tiles_per_wg must be 0..4 and table_mode 0..4");
    if (p->corr_lags < 0 || p->corr_lags > 14)
        return fail(ctx, DM_EINVAL, "corr_lags must be 0..14");
    std::vector<double> dtau(ctx->buckets.size());
    for (size_t i = 0; i < ctx->buckets.size(); ++i) {
        int found = -1;
        for (int j = 0; j < p->n_lengths; ++j)
            if (p->lengths[j] == ctx->buckets[i].M) found = j;
        if (found < 0)
            return fail(ctx, DM_EINVAL, "no time step for chain length %d",
                        ctx->buckets[i].M);
        dtau[i] = p->dt[found] / tunit;
        if (!(dtau[i] > 0.0) || !std::isfinite(dtau[i]))
            return fail(ctx, DM_EINVAL, "time step for length %d must be positive",
                        ctx->buckets[i].M);
    }
    const double gdot = p->gamma_dot * tunit;
    if (!std::isfinite(gdot)) return fail(ctx, DM_EINVAL, "gamma_dot is not finite");
    if (ctx->pending_init) {
        int rc = config_state(ctx, nu);
        if (rc) return rc;
    }
    for (size_t i = 0; i < ctx->buckets.size(); ++i) {
        Bucket &b = ctx->buckets[i];
        dm::ModeCoefs mc;
        dm::mode_coefficients(b.M, nu, T_star, dtau[i], mc);
        DM_HIP(ctx, hipMemcpyAsync(b.d_E, mc.E.data(), sizeof(double) * b.M,
                                   hipMemcpyHostToDevice, ctx->stream));
        DM_HIP(ctx, hipMemcpyAsync(b.d_C, mc.C.data(), sizeof(double) * b.M,
                                   hipMemcpyHostToDevice, ctx->stream));
        DM_HIP(ctx, hipMemcpyAsync(b.d_W, mc.W.data(), sizeof(double) * b.M,
                                   hipMemcpyHostToDevice, ctx->stream));
        if (fused_precision(ctx->precision))
            DM_HIP(ctx, dm::fused_set_coefs(b.fused, mc, b.M, 1.0 - 2.0 * nu, gdot * dtau[i],
                                            ctx->stream));
        DM_HIP(ctx, hipStreamSynchronize(ctx->stream));  // host tables go out of scope
        b.dtau = dtau[i];
        b.zeta_l = mc.zeta_l;
    }
    ctx->T_star = T_star;
    ctx->nu = nu;
    ctx->gamma_dot = gdot;
    ctx->nonlinear = p->nonlinear ? 1 : 0;
    ctx->sample_every = p->sample_every;
    ctx->check_finite = p->check_finite ? 1 : 0;
    ctx->use_graphs = p->use_graphs ? 1 : 0;
    {   // correlation rings: (re)allocate for the lag count, restart
        const int K = p->corr_lags;
        for (Bucket &b : ctx->buckets) {
            if (b.d_ring) (void)hipFree(b.d_ring);
            b.d_ring = nullptr;
            if (!b.d_ccount) {
                int rc = dalloc(ctx, &b.d_ccount, b.n);
                if (rc) return rc;
            }
            DM_HIP(ctx, hipMemsetAsync(b.d_ccount, 0, sizeof(double) * b.n, ctx->stream));
            if (K > 0) {
                int rc = dalloc(ctx, &b.d_ring, (size_t)b.n * 9 * ((size_t)1 << (K - 1)));
                if (rc) return rc;
            }
        }
        ctx->corr_lags = K;
    }
    ctx->autotune = p->autotune ? 1 : 0;
    drop_graph(ctx);  // captured launches hold the old tables and plan
    if (fused_precision(ctx->precision)) {
        ctx->tune_report.clear();
        if (ctx->autotune) {
            std::vector<dm::FusedBucket *> fb;
            for (Bucket &b : ctx->buckets) fb.push_back(&b.fused);
            DM_HIP(ctx, dm::fused_autotune(fb, ctx->seed, 64, ctx->stream, ctx->tune_report));
        } else if (!p->table_mode) {
            // untimed: split tiles when a wavefront per tile would leave
            // compute units idle; of 8 wavefronts when every bucket has that
            // form (one launch of their kernel), else of 4
            size_t tiles = 0;
            for (const Bucket &b : ctx->buckets) tiles += (size_t)b.fused.ntiles;
            if (ctx->ncu > 0 && tiles <= (size_t)ctx->ncu) {
                bool wide = true;
                for (Bucket &b : ctx->buckets) {
                    dm::fused_force_shape(b.fused, 4, 0);
                    wide = wide && b.fused.split == 2;
                }
                if (!wide)
                    for (Bucket &b : ctx->buckets) dm::fused_force_shape(b.fused, 3, 0);
            }
        }
        if (p->tiles_per_wg || p->table_mode)
            for (Bucket &b : ctx->buckets)
                dm::fused_force_shape(b.fused, p->table_mode, p->tiles_per_wg);
        int rc = build_plan(ctx);
        if (rc) return rc;
    }
    ctx->have_params = true;
    return DM_OK;
}

int dm_step_modes(dm_ctx *ctx, int64_t n_steps)
{
    if (!ctx) return DM_EINVAL;
    if (!ctx->have_params) return fail(ctx, DM_ESTATE, "dm_set_params has not been called");
    if (n_steps < 0) return fail(ctx, DM_EINVAL, "n_steps must be >= 0");
    int64_t done = 0;
    const bool fused = fused_precision(ctx->precision);
    // the plain form captures its launches one by one: blocks of at most
    // kMaxPlainGraphSteps steps
    const bool graphs = ctx->use_graphs && ctx->sample_every > 0 &&
                        (fused || ctx->sample_every <= kMaxPlainGraphSteps);
    while (done < n_steps) {
        const int se = ctx->sample_every;
        if (graphs && ctx->step % se == 0 && n_steps - done >= se) {
            const int64_t blocks = (n_steps - done) / se;
            bool overlap = false;
            if (blocks >= 2 && fused) {
                int rc = overlap_pays(ctx, se, &overlap);
                if (rc) return rc;
            }
            if (overlap) {
                // deferred observables: each block's sample is taken from its
                // snapshot during the next block; the last one right after
                if (!ctx->x_steady || ctx->overlap_steps != se) {
                    int rc = capture_overlap(ctx, se);
                    if (rc) return rc;
                }
                DM_HIP(ctx, dm::fused_set_step(ctx->d_step, ctx->step, ctx->stream));
                DM_HIP(ctx, hipGraphLaunch(ctx->x_first, ctx->stream));
                for (int64_t i = 1; i < blocks; ++i)
                    DM_HIP(ctx, hipGraphLaunch(ctx->x_steady, ctx->stream));
                ctx->step += blocks * se;
                done += blocks * se;
                int rc = observe(ctx, 1, ctx->stream, false, true);
                if (rc) return rc;
                continue;
            }
            // whole sampling blocks: replay the captured block
            if (!ctx->graph_exec || ctx->graph_steps != se) {
                int rc = capture_block(ctx, se);
                if (rc) return rc;
            }
            DM_HIP(ctx, dm::fused_set_step(ctx->d_step, ctx->step, ctx->stream));
            for (int64_t i = 0; i < blocks; ++i)
                DM_HIP(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
            ctx->step += blocks * se;
            done += blocks * se;
            continue;
        }
        // steps until the next sampling point (or the end of the request)
        int64_t chunk = n_steps - done;
        if (ctx->sample_every > 0) {
            const int64_t to_sample = ctx->sample_every - (ctx->step % ctx->sample_every);
            chunk = std::min(chunk, to_sample);
        }
        if (fused_precision(ctx->precision)) {
            chunk = std::min<int64_t>(chunk, 1 << 30);
            DM_HIP(ctx, dm::fused_launch(ctx->plan, ctx->seed, ctx->step, nullptr, (int)chunk,
                                         ctx->nonlinear, ctx->stream));
        } else {
            for (int64_t s = 0; s < chunk; ++s)
                for (Bucket &b : ctx->buckets) {
                    int rc = plain_step(ctx, b, ctx->step + s, ctx->stream);
                    if (rc) return rc;
                }
        }
        ctx->step += chunk;
        done += chunk;
        if (ctx->sample_every > 0 && ctx->step % ctx->sample_every == 0) {
            int rc = observe(ctx, 1, ctx->stream);
            if (rc) return rc;
        }
    }
    if (ctx->check_finite) return check_state(ctx);
    return DM_OK;
}

int dm_step_euler(dm_ctx *ctx, int64_t n_steps, double dtau)
{
    if (!ctx) return DM_EINVAL;
    if (!ctx->have_params) return fail(ctx, DM_ESTATE, "dm_set_params has not been called");
    if (!(dtau > 0.0) || !std::isfinite(dtau)) return fail(ctx, DM_EINVAL, "dtau must be > 0");
    if (n_steps < 0 || n_steps > (1 << 30)) return fail(ctx, DM_EINVAL, "bad n_steps");
    if (n_steps == 0) return DM_OK;
    const double gdt = ctx->gamma_dot * dtau;
    for (Bucket &b : ctx->buckets) {
        int rc = bucket_positions(ctx, b, ctx->stream);  // b.d_r = phi R (all modes, FP64)
        if (rc) return rc;
        DM_HIP(ctx, dm::launch_euler_f64(b.d_r, b.d_ids, b.M, b.n, ctx->nu, dtau, ctx->T_star,
                                         gdt, ctx->seed, ctx->step, (int)n_steps, ctx->stream));
        DM_HIP(ctx, dm::launch_gemm_f64(b.d_Afwd, b.d_r, b.d_R64, b.M, 3 * b.n, ctx->stream));
        if (fused_precision(ctx->precision))
            DM_HIP(ctx, dm::fused_pack_modes(b.fused, b.d_R64, b.M, b.n, ctx->stream));
    }
    ctx->step += n_steps;
    if (ctx->check_finite) return check_state(ctx);
    return DM_OK;
}

int dm_step_wlc(dm_ctx *ctx, int64_t n_steps, double dt_bar, double T_bar, int32_t iters,
                double tol, int32_t midpoint)
{
    if (!ctx) return DM_EINVAL;
    if (n_steps < 0 || n_steps > (1 << 30)) return fail(ctx, DM_EINVAL, "bad n_steps");
    if (!(dt_bar > 0.0) || !std::isfinite(dt_bar) || !(T_bar > 0.0) || !std::isfinite(T_bar))
        return fail(ctx, DM_EINVAL, "dt_bar and T_bar must be positive");
    if (iters < 1 || iters > 64) return fail(ctx, DM_EINVAL, "iters must be 1..64");
    if (ctx->pending_init)
        return fail(ctx, DM_ESTATE, "no state yet: the initial state is built by dm_set_params");
    if (!(tol >= 0.0) || !std::isfinite(tol))
        return fail(ctx, DM_EINVAL, "tol must be finite and >= 0");
    if (n_steps == 0) return DM_OK;
    for (Bucket &b : ctx->buckets) {
        const size_t scratch = dm::wlc_scratch_doubles(b.M, b.n);
        if (scratch && !b.d_wlc) {
            int rc = dalloc(ctx, &b.d_wlc, scratch);
            if (rc) return rc;
        }
        int rc = bucket_positions(ctx, b, ctx->stream);  // b.d_r = phi R (FP64)
        if (rc) return rc;
        DM_HIP(ctx, dm::launch_wlc(b.d_r, b.d_wlc, b.d_ids, b.M, b.n, T_bar, dt_bar, iters, tol,
                                   midpoint ? 1 : 0,
                                   ctx->seed, ctx->step, (int)n_steps, ctx->stream));
        DM_HIP(ctx, dm::launch_gemm_f64(b.d_Afwd, b.d_r, b.d_R64, b.M, 3 * b.n, ctx->stream));
        if (fused_precision(ctx->precision))
            DM_HIP(ctx, dm::fused_pack_modes(b.fused, b.d_R64, b.M, b.n, ctx->stream));
    }
    ctx->step += n_steps;
    if (ctx->check_finite) return check_state(ctx);
    return DM_OK;
}

int dm_step_mc(dm_ctx *ctx, int64_t n_sweeps, double step_scale, int64_t *accepted)
{
    if (!ctx) return DM_EINVAL;
    if (!ctx->have_params) return fail(ctx, DM_ESTATE, "dm_set_params has not been called");
    if (n_sweeps < 0 || n_sweeps > (1 << 30)) return fail(ctx, DM_EINVAL, "bad n_sweeps");
    if (!(step_scale >= 0.0) || !std::isfinite(step_scale))
        return fail(ctx, DM_EINVAL, "step_scale must be finite and >= 0");
    for (Bucket &b : ctx->buckets)
        if (48 * (size_t)b.M > 64 * 1024)
            return fail(ctx, DM_EINVAL, "Monte Carlo needs M <= 1365 (LDS), got %d", b.M);
    if (accepted) *accepted = 0;
    if (n_sweeps == 0) return DM_OK;
    const bool fused = fused_precision(ctx->precision);
    for (Bucket &b : ctx->buckets) {
        const int M = b.M, NB = M - 1;
        if (!b.d_chiT) {
            std::vector<double> phi, chiT((size_t)M * NB, 0.0);
            dm::rouse_matrix(M, phi);
            for (int p = 1; p < M; ++p)
                for (int n = 1; n < M; ++n)
                    chiT[(size_t)p * NB + n - 1] = phi[(size_t)n * M + p] - phi[(size_t)(n - 1) * M + p];
            int rc;
            if ((rc = dalloc(ctx, &b.d_chiT, chiT.size())) || (rc = dalloc(ctx, &b.d_mcstep, M)) ||
                (rc = dalloc(ctx, &b.d_mcacc, b.n)))
                return rc;
            DM_HIP(ctx, hipMemcpy(b.d_chiT, chiT.data(), sizeof(double) * chiT.size(),
                                  hipMemcpyHostToDevice));
        }
        b.mcstep_h.assign(M, 0.0);
        for (int p = 1; p < M; ++p)
            b.mcstep_h[p] = step_scale * std::sqrt(ctx->T_star / b.zeta_l[p]);
        DM_HIP(ctx, hipMemcpyAsync(b.d_mcstep, b.mcstep_h.data(), sizeof(double) * M,
                                   hipMemcpyHostToDevice, ctx->stream));
        if (fused) DM_HIP(ctx, dm::fused_unpack_modes(b.fused, b.d_R64, b.M, b.n, ctx->stream));
    }
    int64_t done = 0, total = 0;
    std::vector<int64_t> h;
    while (done < n_sweeps) {
        int64_t chunk = n_sweeps - done;
        if (ctx->sample_every > 0)
            chunk = std::min<int64_t>(chunk, ctx->sample_every - ctx->step % ctx->sample_every);
        for (Bucket &b : ctx->buckets) {
            DM_HIP(ctx, dm::launch_mc(b.d_R64, b.d_chiT, b.d_mcstep, b.d_ids, b.M, b.n, ctx->nu,
                                      ctx->T_star, ctx->seed, ctx->step, (int)chunk, b.d_mcacc,
                                      ctx->stream));
            if (fused) DM_HIP(ctx, dm::fused_pack_modes(b.fused, b.d_R64, b.M, b.n, ctx->stream));
            h.resize(b.n);
            DM_HIP(ctx, hipMemcpyAsync(h.data(), b.d_mcacc, sizeof(int64_t) * b.n,
                                       hipMemcpyDeviceToHost, ctx->stream));
            DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
            for (int64_t v : h) total += v;
        }
        ctx->step += chunk;
        done += chunk;
        if (ctx->sample_every > 0 && ctx->step % ctx->sample_every == 0) {
            int rc = observe(ctx, 1, ctx->stream);
            if (rc) return rc;
        }
    }
    if (accepted) *accepted = total;
    if (ctx->check_finite) return check_state(ctx);
    return DM_OK;
}

int dm_observables_size(const dm_ctx *ctx, int32_t which, size_t *len)
{
    if (!ctx || !len) return DM_EINVAL;
    size_t n = 0;
    if (which & DM_OBS_CHAIN) n += (size_t)DM_NCHAIN_OBS * ctx->nchains;
    if (which & DM_OBS_MODES) n += ctx->total / 3;
    if (which & DM_OBS_ACCUM)
        for (const Bucket &b : ctx->buckets) n += dm::acc_width(b.M);
    *len = n;
    return DM_OK;
}

int dm_observables(dm_ctx *ctx, int32_t which, double *out_host, size_t out_len)
{
    if (!ctx) return DM_EINVAL;
    size_t need = 0;
    dm_observables_size(ctx, which, &need);
    if (out_len < need || (need && !out_host))
        return fail(ctx, DM_EINVAL, "output needs %zu doubles, got %zu", need, out_len);
    if (ctx->pending_init)
        return fail(ctx, DM_ESTATE, "no state yet: the initial state is built by dm_set_params");
    double *o = out_host;
    if (which & (DM_OBS_CHAIN | DM_OBS_MODES)) {
        int rc = observe(ctx, 0, ctx->stream);
        if (rc) return rc;
        DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (which & DM_OBS_CHAIN) {
        for (Bucket &b : ctx->buckets) {
            std::vector<double> h((size_t)16 * b.n);
            DM_HIP(ctx, hipMemcpy(h.data(), b.d_obs, sizeof(double) * h.size(),
                                  hipMemcpyDeviceToHost));
            for (int j = 0; j < b.n; ++j)
                std::memcpy(o + (size_t)DM_NCHAIN_OBS * b.ids[j], &h[(size_t)16 * j],
                            sizeof(double) * 16);
        }
        o += (size_t)DM_NCHAIN_OBS * ctx->nchains;
    }
    if (which & DM_OBS_MODES) {
        for (Bucket &b : ctx->buckets) {
            std::vector<double> h((size_t)b.M * b.n);
            DM_HIP(ctx, hipMemcpy(h.data(), b.d_m2, sizeof(double) * h.size(),
                                  hipMemcpyDeviceToHost));
            for (int j = 0; j < b.n; ++j)
                std::memcpy(o + ctx->offset[b.ids[j]] / 3, &h[(size_t)b.M * j],
                            sizeof(double) * b.M);
        }
        o += ctx->total / 3;
    }
    if (which & DM_OBS_ACCUM) {
        for (Bucket &b : ctx->buckets) {
            const int w = dm::acc_width(b.M);
            DM_HIP(ctx, dm::launch_reduce_chains(b.d_acc, b.d_accsum, w, b.n, ctx->stream));
            DM_HIP(ctx, hipMemcpyAsync(o, b.d_accsum, sizeof(double) * w, hipMemcpyDeviceToHost,
                                       ctx->stream));
            DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
            o[DM_ACC_M] = b.M;
            o[DM_ACC_NCHAINS] = b.n;
            o[DM_ACC_NSAMPLES] = b.n ? o[DM_ACC_NSAMPLES] / b.n : 0.0;
            o += w;
        }
    }
    if (which & DM_OBS_RESET) {
        // the MSD reference becomes the current centre of mass
        int rc = observe(ctx, 0, ctx->stream);
        if (rc) return rc;
        for (Bucket &b : ctx->buckets) {
            DM_HIP(ctx, hipMemsetAsync(b.d_acc, 0, sizeof(double) * dm::acc_width(b.M) * b.n,
                                       ctx->stream));
            // tumbling times restart; the orientation state is kept
            DM_HIP(ctx, hipMemsetAsync(b.d_tumble + b.n, 0, sizeof(double) * b.n, ctx->stream));
            DM_HIP(ctx, hipMemcpy2DAsync(b.d_cm0, 3 * sizeof(double), b.d_obs + DM_CO_CM,
                                         16 * sizeof(double), 3 * sizeof(double), b.n,
                                         hipMemcpyDeviceToDevice, ctx->stream));
        }
        DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    return DM_OK;
}

int dm_get_positions(dm_ctx *ctx, double *dst, int32_t dst_on_device)
{
    if (!ctx || !dst) return ctx ? fail(ctx, DM_EINVAL, "dst is NULL") : DM_EINVAL;
    if (ctx->pending_init)
        return fail(ctx, DM_ESTATE, "no state yet: the initial state is built by dm_set_params");
    for (Bucket &b : ctx->buckets) {
        int rc = bucket_positions(ctx, b, ctx->stream);
        if (rc) return rc;
        if (dst_on_device) {
            DM_HIP(ctx, dm::launch_scatter_chains(b.d_r, dst, b.d_off, 3 * b.M, b.n,
                                                  ctx->stream));
        } else {
            std::vector<double> h((size_t)3 * b.M * b.n);
            DM_HIP(ctx, hipMemcpyAsync(h.data(), b.d_r, sizeof(double) * h.size(),
                                       hipMemcpyDeviceToHost, ctx->stream));
            DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
            for (int j = 0; j < b.n; ++j)
                std::memcpy(dst + b.user_off[j], &h[(size_t)3 * b.M * j],
                            sizeof(double) * 3 * b.M);
        }
    }
    DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return DM_OK;
}

int dm_get_modes(dm_ctx *ctx, double *dst)
{
    if (!ctx || !dst) return ctx ? fail(ctx, DM_EINVAL, "dst is NULL") : DM_EINVAL;
    if (ctx->pending_init)
        return fail(ctx, DM_ESTATE, "no state yet: the initial state is built by dm_set_params");
    for (Bucket &b : ctx->buckets) {
        if (fused_precision(ctx->precision))
            DM_HIP(ctx, dm::fused_unpack_modes(b.fused, b.d_R64, b.M, b.n, ctx->stream));
        std::vector<double> h((size_t)3 * b.M * b.n);
        DM_HIP(ctx, hipMemcpyAsync(h.data(), b.d_R64, sizeof(double) * h.size(),
                                   hipMemcpyDeviceToHost, ctx->stream));
        DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
        for (int j = 0; j < b.n; ++j)
            std::memcpy(dst + b.user_off[j], &h[(size_t)3 * b.M * j], sizeof(double) * 3 * b.M);
    }
    return DM_OK;
}

// State blob: header, then per bucket the FP64 modes (n*3*M), the centre of
// mass reference (n*3), the per-chain accumulators (n*acc_width(M)) and the
// tumbling state (2n).
struct StateHeader {
    uint64_t magic;
    int64_t step;
    int32_t nchains, precision, nbuckets, pad;
};
static const uint64_t kStateMagic = 0x324d4f444d4e4144ull;  // "DANMDOM2"

static size_t state_size(const dm_ctx *ctx)
{
    size_t s = sizeof(StateHeader);
    for (const Bucket &b : ctx->buckets)
        s += sizeof(int32_t) * 2 + sizeof(double) * ((size_t)3 * b.M * b.n + 3 * (size_t)b.n +
                                                     (size_t)dm::acc_width(b.M) * b.n +
                                                     2 * (size_t)b.n);
    return s;
}

int dm_save_state(dm_ctx *ctx, void *buf, size_t *len)
{
    if (!ctx || !len) return DM_EINVAL;
    const size_t need = state_size(ctx);
    if (!buf) {
        *len = need;
        return DM_OK;
    }
    if (*len < need) return fail(ctx, DM_EINVAL, "state buffer needs %zu bytes", need);
    if (ctx->pending_init)
        return fail(ctx, DM_ESTATE, "no state yet: the initial state is built by dm_set_params");
    char *p = (char *)buf;
    StateHeader h{kStateMagic, ctx->step, ctx->nchains, ctx->precision,
                  (int32_t)ctx->buckets.size(), 0};
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    for (Bucket &b : ctx->buckets) {
        int32_t mn[2] = {b.M, b.n};
        std::memcpy(p, mn, sizeof mn);
        p += sizeof mn;
        if (fused_precision(ctx->precision))
            DM_HIP(ctx, dm::fused_unpack_modes(b.fused, b.d_R64, b.M, b.n, ctx->stream));
        const size_t s1 = sizeof(double) * 3 * b.M * b.n, s2 = sizeof(double) * 3 * b.n,
                     s3 = sizeof(double) * dm::acc_width(b.M) * b.n,
                     s4 = sizeof(double) * 2 * b.n;
        DM_HIP(ctx, hipMemcpyAsync(p, b.d_R64, s1, hipMemcpyDeviceToHost, ctx->stream));
        DM_HIP(ctx, hipMemcpyAsync(p + s1, b.d_cm0, s2, hipMemcpyDeviceToHost, ctx->stream));
        DM_HIP(ctx, hipMemcpyAsync(p + s1 + s2, b.d_acc, s3, hipMemcpyDeviceToHost, ctx->stream));
        DM_HIP(ctx, hipMemcpyAsync(p + s1 + s2 + s3, b.d_tumble, s4, hipMemcpyDeviceToHost,
                                   ctx->stream));
        p += s1 + s2 + s3 + s4;
    }
    DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *len = need;
    return DM_OK;
}

int dm_load_state(dm_ctx *ctx, const void *buf, size_t len)
{
    if (!ctx || !buf) return DM_EINVAL;
    if (len < state_size(ctx)) return fail(ctx, DM_EINVAL, "state blob too short");
    const char *p = (const char *)buf;
    StateHeader h;
    std::memcpy(&h, p, sizeof h);
    p += sizeof h;
    if (h.magic != kStateMagic || h.nchains != ctx->nchains || h.precision != ctx->precision ||
        h.nbuckets != (int32_t)ctx->buckets.size())
        return fail(ctx, DM_EINVAL, "state blob does not match this context");
    const char *q = p;
    for (Bucket &b : ctx->buckets) {  // validate before touching the state
        int32_t mn[2];
        std::memcpy(mn, q, sizeof mn);
        if (mn[0] != b.M || mn[1] != b.n)
            return fail(ctx, DM_EINVAL, "state blob bucket mismatch");
        q += sizeof mn + sizeof(double) * ((size_t)3 * b.M * b.n + 3 * (size_t)b.n +
                                           (size_t)dm::acc_width(b.M) * b.n + 2 * (size_t)b.n);
    }
    for (Bucket &b : ctx->buckets) {
        p += 2 * sizeof(int32_t);
        const size_t s1 = sizeof(double) * 3 * b.M * b.n, s2 = sizeof(double) * 3 * b.n,
                     s3 = sizeof(double) * dm::acc_width(b.M) * b.n,
                     s4 = sizeof(double) * 2 * b.n;
        DM_HIP(ctx, hipMemcpyAsync(b.d_R64, p, s1, hipMemcpyHostToDevice, ctx->stream));
        DM_HIP(ctx, hipMemcpyAsync(b.d_cm0, p + s1, s2, hipMemcpyHostToDevice, ctx->stream));
        DM_HIP(ctx, hipMemcpyAsync(b.d_acc, p + s1 + s2, s3, hipMemcpyHostToDevice, ctx->stream));
        DM_HIP(ctx, hipMemcpyAsync(b.d_tumble, p + s1 + s2 + s3, s4, hipMemcpyHostToDevice,
                                   ctx->stream));
        if (fused_precision(ctx->precision))
            DM_HIP(ctx, dm::fused_pack_modes(b.fused, b.d_R64, b.M, b.n, ctx->stream));
        p += s1 + s2 + s3 + s4;
    }
    for (Bucket &b : ctx->buckets)  // the correlation rings restart
        if (b.d_ccount)
            DM_HIP(ctx, hipMemsetAsync(b.d_ccount, 0, sizeof(double) * b.n, ctx->stream));
    DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->step = h.step;
    ctx->pending_init = false;
    return DM_OK;
}

int dm_get_step(const dm_ctx *ctx, int64_t *step)
{
    if (!ctx || !step) return DM_EINVAL;
    *step = ctx->step;
    return DM_OK;
}

int dm_sync(dm_ctx *ctx)
{
    if (!ctx) return DM_EINVAL;
    DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return DM_OK;
}

int dm_destroy(dm_ctx *ctx)
{
    if (!ctx) return DM_EINVAL;
    (void)hipStreamSynchronize(ctx->stream);
    drop_graph(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->cap_stream2) (void)hipStreamDestroy(ctx->cap_stream2);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    dm::fused_plan_free(ctx->plan);
    for (Bucket &b : ctx->buckets) free_bucket(b);
    if (ctx->d_flag) (void)hipFree(ctx->d_flag);
    if (ctx->d_step) (void)hipFree(ctx->d_step);
    delete ctx;
    return DM_OK;
}

int dm_get_tiling(const dm_ctx *ctx, double *out, size_t len, int32_t *n_buckets)
{
    if (!ctx || !n_buckets) return DM_EINVAL;
    *n_buckets = (int32_t)ctx->buckets.size();
    if (!out) return DM_OK;
    if (len < (size_t)DM_NTILING * ctx->buckets.size())
        return fail(const_cast<dm_ctx *>(ctx), DM_EINVAL, "tiling needs %zu doubles",
                    (size_t)DM_NTILING * ctx->buckets.size());
    const bool fused = fused_precision(ctx->precision);
    for (size_t i = 0; i < ctx->buckets.size(); ++i) {
        const Bucket &b = ctx->buckets[i];
        const dm::FusedBucket &f = b.fused;
        double *o = out + DM_NTILING * i;
        o[DM_TI_M] = b.M;
        o[DM_TI_NCHAINS] = b.n;
        o[DM_TI_RT] = fused ? f.RT : 0;
        o[DM_TI_JC] = fused ? f.JC : 0;
        o[DM_TI_RESIDENT] = fused ? f.resident : 0;
        o[DM_TI_TPW] = fused ? f.tpw : 0;
        o[DM_TI_ITEMS] = fused ? (f.ntiles + f.tpw - 1) / f.tpw : 0;
        o[DM_TI_ITEM_US] = fused ? f.item_us : 0;
        o[DM_TI_SPLIT] = fused ? f.split : 0;
    }
    return DM_OK;
}

const char *dm_tuning_report(const dm_ctx *ctx) { return ctx ? ctx->tune_report.c_str() : ""; }

int dm_coarse_grain(double r, double y, int32_t k, double *T_star_k, double *nu_k)
{
    if (!(r > 0.0) || !(y > 0.0) || k < 1 || !T_star_k || !nu_k || !std::isfinite(r) ||
        !std::isfinite(y))
        return fail(nullptr, DM_EINVAL, "coarse graining needs r > 0, y > 0, k >= 1");
    const double kk = (double)k, a = 2.0 * r * r + kk * kk * y;
    *T_star_k = a * r / (kk * kk * kk * y * y);
    *nu_k = r * r / a;
    return DM_OK;
}

int dm_coarse_grain_time(double r, double y, int32_t k, double *c_k)
{
    double T = 0.0, nu = 0.0;
    if (!c_k) return fail(nullptr, DM_EINVAL, "coarse graining needs an output");
    const int rc = dm_coarse_grain(r, y, k, &T, &nu);
    if (rc) return rc;
    const double kk = (double)k, s = 1.0 - 2.0 * nu;
    *c_k = kk * kk * kk * T * s * s;
    return DM_OK;
}

const char *dm_last_error(const dm_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

}  // extern "C"
