// dm_plain.hip -- the plain FP64 form of the mode step and the bead-space
// Euler baseline, as separate kernels (gfx950).
//
// Data layout in HBM: a bucket of nch chains of M beads stores positions,
// forces and mode amplitudes as nch*3 columns of M doubles (SoA, column
// (chain, component) contiguous in the bead or mode index).  A transform is
// then one GEMM Y = A X^T with a square M x M table A and 3*nch columns:
//   inverse  r_n  = sum_{p>=1} phi_{n,p} R_p     (Eq. c1, internal coords)
//   forward  dH_p = sum_n phi_{n,p} F_n          (Eqs. c5, e11)
#include "dm_internal.h"
#include "dm_rng.h"

namespace dm {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// --------------------------------------------------------------------------
// GEMM on FP64 MFMA (v_mfma_f64_16x16x4f64).  Workgroup tile 64 rows x 64
// columns, 4 waves of 32 x 32 (2 x 2 MFMA tiles), K staged through LDS in
// chunks of 16.  MFMA operand layout per lane l: A[i = l%16][k = l/16],
// B[k = l/16][j = l%16]; result D[i = l/16 + 4r][j = l%16], r = 0..3 (the
// FP64 instruction interleaves its four result rows across the lane groups).
// --------------------------------------------------------------------------
constexpr int kGemmBM = 64, kGemmBN = 64, kGemmBK = 16;

__global__ __launch_bounds__(256) void gemm_f64_kernel(const double *__restrict__ A,
                                                       const double *__restrict__ X,
                                                       double *__restrict__ Y, int M,
                                                       int ncol)
{
    __shared__ double As[kGemmBM][kGemmBK + 1];
    __shared__ double Xs[kGemmBN][kGemmBK + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    const int i0 = blockIdx.x * kGemmBM;
    const int c0 = blockIdx.y * kGemmBN;
    f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < M; k0 += kGemmBK) {
#pragma unroll
        for (int e = 0; e < (kGemmBM * kGemmBK) / 256; ++e) {
            const int idx = tid + 256 * e;
            const int row = idx / kGemmBK, kk = idx % kGemmBK;
            const int gk = k0 + kk;
            const int gi = i0 + row, gc = c0 + row;
            As[row][kk] = (gi < M && gk < M) ? A[(size_t)gi * M + gk] : 0.0;
            Xs[row][kk] = (gc < ncol && gk < M) ? X[(size_t)gc * M + gk] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kGemmBK; ks += 4) {
            double a[2], b[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                a[t] = As[32 * wi + 16 * t + (lane & 15)][ks + (lane >> 4)];
                b[t] = Xs[32 * wj + 16 * t + (lane & 15)][ks + (lane >> 4)];
            }
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj)
                    acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj],
                                                                      acc[ti][tj], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
            const int c = c0 + 32 * wj + 16 * tj + (lane & 15);
            const int ib = i0 + 32 * wi + 16 * ti + (lane >> 4);
            if (c >= ncol) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (ib + 4 * r < M) Y[(size_t)c * M + ib + 4 * r] = acc[ti][tj][r];
        }
}

// The same product when M is a multiple of 16 (every chain length the
// method runs in practice): 16-byte loads of A and X, and a software
// pipeline over the K chunks -- the next chunk is loaded into registers while
// the current one is multiplied from the other of two LDS buffers, one
// barrier per chunk.  The MFMA sequence of every accumulator is the one of
// the kernel above, so both give the same bits.  BN = 64 or 32 columns per
// workgroup tile (each wavefront 32 rows x BN/2 columns): the narrower tile
// doubles the workgroups of small launches (1024 chains of 128 beads make 96
// tiles of 64 x 64 for 256 CUs) and leaves every accumulator's sequence as it
// is.
typedef double f64x2 __attribute__((ext_vector_type(2)));

// Workgroups of a launch are dispatched round-robin over the GPU's 8 XCDs
// (workgroup w to XCD w % 8), each with its own L2.  This maps the
// dispatch index w of n workgroups to a logical index such that every XCD
// takes one contiguous range of logical indices (a bijection on [0, n)).
__device__ __forceinline__ int xcd_local_index(int w, int n)
{
    constexpr int kXcd = 8;
    const int q = n / kXcd, r = n % kXcd, x = w % kXcd, s = w / kXcd;
    return x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

template <int BN>
__global__ __launch_bounds__(256) void gemm_f64_pipe_kernel(const double *__restrict__ A,
                                                            const double *__restrict__ X,
                                                            double *__restrict__ Y, int M,
                                                            int ncol)
{
    static_assert(BN == 64 || BN == 32, "column tile");
    constexpr int TJ = BN / 32;  // 16-column MFMA tiles per wavefront
    __shared__ double As[2][kGemmBM][kGemmBK + 1];
    __shared__ double Xs[2][BN][kGemmBK + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    // one-dimensional grid, row tiles fastest in the XCD-local order: the
    // row tiles that read the same column block of X run on one XCD and
    // share its L2, so each X block crosses HBM about once
    const int nrt = (M + kGemmBM - 1) / kGemmBM;
    const int L = xcd_local_index((int)blockIdx.x, (int)gridDim.x);
    const int i0 = (L % nrt) * kGemmBM;
    const int c0 = (L / nrt) * BN;
    // each thread moves 4 consecutive k of one row of A and (lr < BN) of one
    // column of X
    const int lr = tid >> 2, lk = (tid & 3) * 4;
    const bool xown = lr < BN;
    const bool arow = i0 + lr < M, xrow = xown && c0 + lr < ncol;
    const f64x2 *pa = reinterpret_cast<const f64x2 *>(A + (size_t)(arow ? i0 + lr : 0) * M + lk);
    const f64x2 *px = reinterpret_cast<const f64x2 *>(X + (size_t)(xrow ? c0 + lr : 0) * M + lk);
    f64x2 ra0, ra1, rx0, rx1;
    auto load = [&](int k0) {
        const f64x2 z = {0.0, 0.0};
        ra0 = arow ? pa[k0 / 2] : z;
        ra1 = arow ? pa[k0 / 2 + 1] : z;
        rx0 = xrow ? px[k0 / 2] : z;
        rx1 = xrow ? px[k0 / 2 + 1] : z;
    };
    auto store = [&](int b) {
        As[b][lr][lk] = ra0[0];
        As[b][lr][lk + 1] = ra0[1];
        As[b][lr][lk + 2] = ra1[0];
        As[b][lr][lk + 3] = ra1[1];
        if (xown) {
            Xs[b][lr][lk] = rx0[0];
            Xs[b][lr][lk + 1] = rx0[1];
            Xs[b][lr][lk + 2] = rx1[0];
            Xs[b][lr][lk + 3] = rx1[1];
        }
    };
    f64x4 acc[2][TJ];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < TJ; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

    const int nk = M / kGemmBK;
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int b = kt & 1;
        if (kt + 1 < nk) load((kt + 1) * kGemmBK);
#pragma unroll
        for (int ks = 0; ks < kGemmBK; ks += 4) {
            double a[2], x[TJ];
#pragma unroll
            for (int t = 0; t < 2; ++t)
                a[t] = As[b][32 * wi + 16 * t + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
            for (int t = 0; t < TJ; ++t)
                x[t] = Xs[b][(BN / 2) * wj + 16 * t + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < TJ; ++tj)
                    acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], x[tj],
                                                                      acc[ti][tj], 0, 0, 0);
        }
        if (kt + 1 < nk) store(b ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) {
            const int c = c0 + (BN / 2) * wj + 16 * tj + (lane & 15);
            const int ib = i0 + 32 * wi + 16 * ti + (lane >> 4);
            if (c >= ncol) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (ib + 4 * r < M) Y[(size_t)c * M + ib + 4 * r] = acc[ti][tj][r];
        }
}

// --------------------------------------------------------------------------
// Force stencil, one thread per (chain, bead).  Bonds u_n = r_n - r_{n-1}
// (n = 1..M-1), g_n = u_n (1/|u_n| - lin) with lin = 1 - 2 nu (Eq. e4),
// F_n = g_n - g_{n+1} with g_0 = g_M = 0.
// --------------------------------------------------------------------------
__device__ __forceinline__ void bond_g(const double *__restrict__ x, int M, int m,
                                       double lin, double g[3])
{
    const double ux = x[m] - x[m - 1];
    const double uy = x[M + m] - x[M + m - 1];
    const double uz = x[2 * M + m] - x[2 * M + m - 1];
    const double l = sqrt(ux * ux + uy * uy + uz * uz);
    const double f = 1.0 / l - lin;
    g[0] = ux * f;
    g[1] = uy * f;
    g[2] = uz * f;
}

__global__ __launch_bounds__(256) void stencil_f64_kernel(const double *__restrict__ r,
                                                          double *__restrict__ F, int M,
                                                          int nch, double lin)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nch * M) return;
    const int c = (int)(idx / M), n = (int)(idx % M);
    const double *x = r + (size_t)c * 3 * M;
    double g0[3] = {0.0, 0.0, 0.0}, g1[3] = {0.0, 0.0, 0.0};
    if (n >= 1) bond_g(x, M, n, lin, g0);
    if (n + 1 <= M - 1) bond_g(x, M, n + 1, lin, g1);
    double *f = F + (size_t)c * 3 * M;
    f[n] = g0[0] - g1[0];
    f[M + n] = g0[1] - g1[1];
    f[2 * M + n] = g0[2] - g1[2];
}

// --------------------------------------------------------------------------
// Mode update (Eqs. d3, d6, f2, btum), one thread per (chain, 4 modes): its
// three Philox blocks (one per component) give all twelve normals, and for
// even M each row's quad moves as two 16-byte pieces, so the lanes of a
// wavefront read and write contiguous runs and the shear drift is folded
// into the one store.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mode_update_f64_kernel(
    double *__restrict__ R, const double *__restrict__ dH, const double *__restrict__ E,
    const double *__restrict__ C, const double *__restrict__ W,
    const int32_t *__restrict__ ids, int M, int nch, uint64_t seed,
    const int64_t *__restrict__ step_dev, int64_t step_off, double gdt, int nonlinear)
{
    const int nq = (M + 3) / 4;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nch * nq) return;
    const int c = (int)(idx / nq), q = (int)(idx % nq);
    const int64_t k = (step_dev ? *step_dev : 0) + step_off;
    const uint32_t chain = (uint32_t)ids[c];
    double z[3][4];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        normals4_f64(noise_bits(seed, (uint32_t)q, chain, k, (uint32_t)a, kTagMode), z[a]);
    double *Rc = R + (size_t)c * 3 * M;
    const double *dHc = dH + (size_t)c * 3 * M;
    // a whole quad of an even-length chain moves as two 16-byte pieces per row
    const bool vec = (M % 2 == 0) && (4 * q + 3 < M);
    double r[3][4], d[3][4], e[4], w[4], cc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int p = min(4 * q + j, M - 1);
        e[j] = E[p];
        w[j] = W[p];
        cc[j] = C[p];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (vec) {
            const f64x2 *src = reinterpret_cast<const f64x2 *>(Rc + a * M + 4 * q);
            const f64x2 lo = src[0], hi = src[1];
            r[a][0] = lo[0], r[a][1] = lo[1], r[a][2] = hi[0], r[a][3] = hi[1];
            if (nonlinear) {
                const f64x2 *hs = reinterpret_cast<const f64x2 *>(dHc + a * M + 4 * q);
                const f64x2 dl = hs[0], dh = hs[1];
                d[a][0] = dl[0], d[a][1] = dl[1], d[a][2] = dh[0], d[a][3] = dh[1];
            } else {
                d[a][0] = d[a][1] = d[a][2] = d[a][3] = 0.0;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int p = min(4 * q + j, M - 1);
                r[a][j] = Rc[a * M + p];
                d[a][j] = nonlinear ? dHc[a * M + p] : 0.0;
            }
        }
    }
    double v[3][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int p = 4 * q + j;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a][j] = e[j] * r[a][j] + w[j] * z[a][j];
            if (nonlinear && p > 0) v[a][j] += cc[j] * d[a][j];
        }
        v[0][j] += gdt * e[j] * r[1][j];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (vec) {
            f64x2 *dst = reinterpret_cast<f64x2 *>(Rc + a * M + 4 * q);
            dst[0] = f64x2{v[a][0], v[a][1]};
            dst[1] = f64x2{v[a][2], v[a][3]};
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (4 * q + j < M) Rc[a * M + 4 * q + j] = v[a][j];
        }
    }
}

// --------------------------------------------------------------------------
// Bead-space Euler (Eqs. b3-b5, btum).  One block per chain, positions held
// in LDS across all steps; thread t owns beads 4t..4t+3.
//   u_m = x_m - x_{m-1} for 1 <= m <= M-1, else 0;
//   h_m = (|u_m| - 1) u_m/|u_m| - nu (u_{m-1} + u_{m+1}) for 1 <= m <= M-1;
//   x_n += dtau (h_{n+1} - h_n) + sqrt(2 T* dtau) eta_n;  x_n += gdt y_n(old).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void euler_f64_kernel(double *__restrict__ pos,
                                                         const int32_t *__restrict__ ids,
                                                         int M, double nu, double dtau,
                                                         double amp, double gdt,
                                                         uint64_t seed, int64_t step0,
                                                         int n_steps)
{
    extern __shared__ double xs[];  // 3*M
    const int c = blockIdx.x, tid = threadIdx.x;
    double *P = pos + (size_t)c * 3 * M;
    for (int i = tid; i < 3 * M; i += blockDim.x) xs[i] = P[i];
    __syncthreads();
    const int nq = (M + 3) / 4;
    const bool active = tid < nq;
    const int n0 = 4 * tid;
    const uint32_t chain = (uint32_t)ids[c];
    for (int s = 0; s < n_steps; ++s) {
        double nx[3][4];
        if (active) {
            const int64_t k = step0 + s;
            double z[3][4];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                normals4_f64(noise_bits(seed, (uint32_t)tid, chain, k, (uint32_t)a, kTagEuler),
                             z[a]);
            // bonds m = n0-1 .. n0+5  -> u[0..6]
            double u[3][7];
#pragma unroll
            for (int j = 0; j < 7; ++j) {
                const int m = n0 - 1 + j;
                const bool ok = (m >= 1) && (m <= M - 1);
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    u[a][j] = ok ? xs[a * M + m] - xs[a * M + m - 1] : 0.0;
            }
            // h_m for m = n0 .. n0+4 -> h[0..4] (u index j = m - n0 + 1)
            double h[3][5];
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                const int m = n0 + j;
                const bool ok = (m >= 1) && (m <= M - 1);
                const double l = sqrt(u[0][j + 1] * u[0][j + 1] + u[1][j + 1] * u[1][j + 1] +
                                      u[2][j + 1] * u[2][j + 1]);
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    h[a][j] = ok ? (l - 1.0) * u[a][j + 1] / l - nu * (u[a][j] + u[a][j + 2])
                                 : 0.0;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n = n0 + j;
                if (n >= M) break;
                const double y_old = xs[M + n];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    nx[a][j] = xs[a * M + n] + (dtau * (h[a][j + 1] - h[a][j]) + amp * z[a][j]);
                nx[0][j] += gdt * y_old;
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n = n0 + j;
                if (n >= M) break;
#pragma unroll
                for (int a = 0; a < 3; ++a) xs[a * M + n] = nx[a][j];
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < 3 * M; i += blockDim.x) P[i] = xs[i];
}

// --------------------------------------------------------------------------
// Observables (Sec. V.B): one wave per chain, FP64 wavefront reductions.
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ __launch_bounds__(64) void chain_obs_kernel(const double *__restrict__ pos,
                                                       const double *__restrict__ R,
                                                       double *__restrict__ obs,
                                                       double *__restrict__ m2,
                                                       double *__restrict__ acc,
                                                       const double *__restrict__ cm0,
                                                       double *__restrict__ tstate,
                                                       double *__restrict__ tlast,
                                                       const int64_t *__restrict__ step_dev,
                                                       double *__restrict__ ring,
                                                       double *__restrict__ ccount, int K,
                                                       int M, int accumulate)
{
    const int c = blockIdx.x, lane = threadIdx.x;
    const double *x = pos + (size_t)c * 3 * M;
    double ls = 0.0, l2s = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    double xmin = x[0], xmax = x[0];
    for (int n = lane; n < M; n += 64) {
        sx += x[n];
        sy += x[M + n];
        sz += x[2 * M + n];
        xmin = fmin(xmin, x[n]);
        xmax = fmax(xmax, x[n]);
        if (n >= 1) {
            const double ux = x[n] - x[n - 1], uy = x[M + n] - x[M + n - 1],
                         uz = x[2 * M + n] - x[2 * M + n - 1];
            const double q = ux * ux + uy * uy + uz * uz;
            ls += sqrt(q);
            l2s += q;
        }
    }
    ls = wave_sum(ls);
    l2s = wave_sum(l2s);
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    sz = wave_sum(sz);
    xmin = wave_min(xmin);
    xmax = wave_max(xmax);
    const double *Rc = R + (size_t)c * 3 * M;
    double *accc = acc + (size_t)c * acc_width(M);
    for (int p = lane; p < M; p += 64) {
        const double v = Rc[p] * Rc[p] + Rc[M + p] * Rc[M + p] + Rc[2 * M + p] * Rc[2 * M + p];
        m2[(size_t)c * M + p] = v;
        if (accumulate) accc[DM_NACC_HEAD + p] += v;
    }
    if (lane == 0) {
        double o[16];
        o[0] = ls / (M - 1);
        const double Lx = x[M - 1] - x[0], Ly = x[2 * M - 1] - x[M],
                     Lz = x[3 * M - 1] - x[2 * M];
        o[1] = Lx * Lx + Ly * Ly + Lz * Lz;
        o[2] = Lx;
        o[3] = Ly;
        o[4] = Lz;
        o[5] = sx / M;
        o[6] = sy / M;
        o[7] = sz / M;
        const int m = M / 2, mid = (M - 1) / 2;
        for (int a = 0; a < 3; ++a) {
            o[8 + a] = x[a * M + m] - x[a * M + m - 1];
            o[11 + a] = x[a * M + mid] - o[5 + a];
        }
        o[14] = xmax - xmin;
        o[15] = l2s / (M - 1);
        for (int j = 0; j < 16; ++j) obs[(size_t)c * 16 + j] = o[j];
        if (accumulate) {
            const double dx = o[5] - cm0[3 * c], dy = o[6] - cm0[3 * c + 1],
                         dz = o[7] - cm0[3 * c + 2];
            accc[DM_ACC_NSAMPLES] += 1.0;
            accc[DM_ACC_BOND] += o[0];
            accc[DM_ACC_BOND2] += o[15];
            accc[DM_ACC_L2] += o[1];
            accc[DM_ACC_MSDCM] += dx * dx + dy * dy + dz * dz;
            accc[DM_ACC_DMID2] += o[11] * o[11] + o[12] * o[12] + o[13] * o[13];
            accc[DM_ACC_XSPAN] += o[14];
            // tumbling in the flow plane, with hysteresis (see dnamodes.h)
            const double rho = sqrt(Lx * Lx + Ly * Ly);
            const double s0 = tstate[c];
            const double s1 = Lx > 0.5 * rho ? 1.0 : (Lx < -0.5 * rho ? -1.0 : s0);
            if (s0 != 0.0 && s1 != s0) {
                const double k = (double)*step_dev;
                accc[DM_ACC_TUMBLES] += 1.0;
                if (tlast[c] > 0.0) {
                    const double tau = k - (tlast[c] - 1.0);
                    accc[DM_ACC_TAU] += tau;
                    accc[DM_ACC_TAU2] += tau * tau;
                    accc[DM_ACC_NTAU] += 1.0;
                    const int bin = min(DM_NTUMBLE_BINS - 1, max(0, ilogb(tau)));
                    accc[DM_NACC_HEAD + M + bin] += 1.0;
                }
                tlast[c] = k + 1.0;
            }
            tstate[c] = s1;
            if (K > 0) {
                const double v[9] = {Lx, Ly, Lz, o[8], o[9], o[10], o[11], o[12], o[13]};
                corr_update(ring + (size_t)c * ((size_t)9 << (K - 1)), ccount + c,
                            accc + DM_NACC_HEAD + M + DM_NTUMBLE_BINS, v, K);
            }
        }
    }
}

// Metropolis Monte Carlo in the mode representation, one wavefront per
// chain (the paper's equilibrium benchmark, Sec. V.B).  A sweep proposes, for
// p = 1..M-1 and component a = x, y, z in order, R_p^a += delta with delta
// uniform on (-s_p, s_p), and accepts with probability
// min(1, exp(-dH'/T*)) for the reduced Hamiltonian of Eq. (b3).  The bond
// vectors u_n (n = 1..M-1) live in LDS; a move shifts every bond by
// chi_{n,p} delta along a, so dH' is a sum over bonds of the change of
// (|u_n| - 1)^2 / 2 and of -nu u_n . u_{n+1}, reduced over the wavefront
// (every lane ends with the same sum, hence the same decision).  Random
// numbers: Philox block (p, chain, sweep, a, tag 2), word 0 for delta, word 1
// for the acceptance test.
__global__ __launch_bounds__(64) void mc_kernel(double *__restrict__ R,
                                                const double *__restrict__ chiT,
                                                const double *__restrict__ sstep,
                                                const int32_t *__restrict__ ids, int M,
                                                double nu, double T_star, uint64_t seed,
                                                int64_t step0, int n_sweeps,
                                                int64_t *__restrict__ accepted)
{
    extern __shared__ double mcl[];  // u[3][M-1], then the amplitudes R[3][M]
    const int c = blockIdx.x, lane = threadIdx.x, NB = M - 1;
    double *u = mcl, *Rl = mcl + 3 * NB;
    double *Rc = R + (size_t)c * 3 * M;
    const uint32_t chain = (uint32_t)ids[c];
    for (int i = lane; i < 3 * M; i += 64) Rl[i] = Rc[i];
    __syncthreads();
    // u_n = sum_{p >= 1} chi_{n,p} R_p
    for (int n = lane; n < NB; n += 64)
        for (int a = 0; a < 3; ++a) {
            double s = 0.0;
            for (int p = 1; p < M; ++p) s += chiT[(size_t)p * NB + n] * Rl[a * M + p];
            u[a * NB + n] = s;
        }
    __syncthreads();
    int64_t acc = 0;
    const double two_m32 = 2.3283064365386962890625e-10;
    for (int s = 0; s < n_sweeps; ++s) {
        const int64_t k = step0 + s;
        for (int p = 1; p < M; ++p) {
            const double sp = sstep[p];
            const double *chi = chiT + (size_t)p * NB;
            for (int a = 0; a < 3; ++a) {
                const Block4 x = noise_bits(seed, (uint32_t)p, chain, k, (uint32_t)a, kTagMC);
                const double u0 = ((double)x.v[0] + 0.5) * two_m32;
                const double u1 = ((double)x.v[1] + 0.5) * two_m32;
                const double delta = sp * (2.0 * u0 - 1.0);
                double d = 0.0;
                for (int n = lane; n < NB; n += 64) {
                    const double ch = chi[n], ua = u[a * NB + n];
                    const double ux = u[n], uy = u[NB + n], uz = u[2 * NB + n];
                    const double l2 = ux * ux + uy * uy + uz * uz;
                    const double l2n = l2 + ch * delta * (2.0 * ua + ch * delta);
                    const double lo = sqrt(l2) - 1.0, ln = sqrt(l2n) - 1.0;
                    d += 0.5 * (ln * ln - lo * lo);
                    if (n + 1 < NB) {
                        const double ch1 = chi[n + 1], ua1 = u[a * NB + n + 1];
                        d -= nu * (delta * (ch * ua1 + ch1 * ua) + delta * delta * ch * ch1);
                    }
                }
                d = wave_sum(d);
                if (u1 < exp(-d / T_star)) {
                    __syncthreads();  // every lane has read the old bonds
                    for (int n = lane; n < NB; n += 64) u[a * NB + n] += chi[n] * delta;
                    if (lane == 0) Rl[a * M + p] += delta;
                    ++acc;
                    __syncthreads();
                }
            }
        }
    }
    for (int i = lane; i < 3 * M; i += 64) Rc[i] = Rl[i];
    if (lane == 0) accepted[c] = acc;
}

// The nu -> 0 limit (Sec. VI.A, Eqs. y2-y14), one thread per chain, FP64: the
// inextensible chain in bending units (tau-bar, T-bar), bonds of unit
// length held by tensions.  A step moves bead n by
//   dr_n = (-f_n u^m_n + f_{n+1} u^m_{n+1} + h_{n+1} - h_n) dt + sqrt(2 T-bar dt) eta_n,
// h_n = -(u^m_{n-1} + u^m_{n+1}) the bending gradient, u^m_n = (u_n + u'_n) /
// |u_n + u'_n| the midpoint bonds (Eq. y14); the tensions f_n solve the
// tridiagonal system (u_n + u'_n) . du_n = 0 (Eqs. y11-y13) by the Thomas
// algorithm, and the cycle (midpoint, tensions, u') is repeated from u' = u
// until it converges: at most `iters` times, fewer when tol > 0 and a cycle
// moves no component of u' by more than tol.  Scratch, chain-fastest ([index][chain], coalesced):
// u, u', u^m (3 (N+2) each, bonds 0 and N+1 zero), noise (3 (N+1)), the
// Thomas coefficients c', d' (N each) and f (N+2).  Noise: the bead index
// with tag 3.  The bonds are scaled to unit length on entry.
__global__ __launch_bounds__(64) void wlc_kernel(double *__restrict__ pos,
                                                 double *__restrict__ scr,
                                                 const int32_t *__restrict__ ids, int M, int nch,
                                                 double T_bar, double dt, int iters, double tol,
                                                 int midpoint, uint64_t seed, int64_t step0,
                                                 int n_steps)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nch) return;
    const int N = M - 1;
    const size_t S = (size_t)nch;
    double *U = scr, *UN = U + 3 * (size_t)(N + 2) * S, *UM = UN + 3 * (size_t)(N + 2) * S;
    double *NZ = UM + 3 * (size_t)(N + 2) * S, *CP = NZ + 3 * (size_t)(N + 1) * S;
    double *DP = CP + (size_t)N * S, *F = DP + (size_t)N * S;
#define V3(A, n, a) A[((size_t)3 * (n) + (a)) * S + c]
    double *x = pos + (size_t)c * 3 * M;
    const uint32_t chain = (uint32_t)ids[c];
    const double amp = sqrt(2.0 * T_bar * dt);
    for (int a = 0; a < 3; ++a) {
        V3(U, 0, a) = V3(U, N + 1, a) = 0.0;
        V3(UN, 0, a) = V3(UN, N + 1, a) = 0.0;
        V3(UM, 0, a) = V3(UM, N + 1, a) = 0.0;
    }
    for (int n = 1; n <= N; ++n) {  // bonds, scaled to unit length
        double u[3], s2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            u[a] = x[a * M + n] - x[a * M + n - 1];
            s2 += u[a] * u[a];
        }
        const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
        for (int a = 0; a < 3; ++a) V3(U, n, a) = u[a] * inv;
    }
    F[0 * S + c] = 0.0;
    F[(size_t)(N + 1) * S + c] = 0.0;
    double r0[3] = {x[0], x[M], x[2 * M]};
    // regular displacement of bead n (bending at the midpoint bonds + noise)
    auto drr = [&](int n, int a) {
        const double hn = n >= 1 ? -(V3(UM, n - 1, a) + V3(UM, n + 1, a)) : 0.0;
        const double hn1 = n + 1 <= N ? -(V3(UM, n, a) + V3(UM, n + 2 <= N + 1 ? n + 2 : N + 1, a))
                                      : 0.0;
        return (hn1 - hn) * dt + V3(NZ, n, a);
    };
    for (int s = 0; s < n_steps; ++s) {
        const int64_t k = step0 + s;
        for (int a = 0; a < 3; ++a)
            for (int q = 0; q <= N / 4; ++q) {
                double z[4];
                normals4_f64(noise_bits(seed, (uint32_t)q, chain, k, (uint32_t)a, kTagWLC), z);
                for (int e = 0; e < 4 && 4 * q + e <= N; ++e) V3(NZ, 4 * q + e, a) = amp * z[e];
            }
        for (int n = 1; n <= N; ++n)
            for (int a = 0; a < 3; ++a) V3(UN, n, a) = V3(U, n, a);
        for (int it = 0; it < iters; ++it) {
            for (int n = 1; n <= N; ++n) {
                double w[3], s2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    w[a] = V3(U, n, a) + V3(UN, n, a);
                    s2 += w[a] * w[a];
                }
                const double inv = 1.0 / sqrt(s2);
                for (int a = 0; a < 3; ++a) V3(UM, n, a) = midpoint ? w[a] * inv : V3(U, n, a);
            }
            // Thomas forward sweep: a f_{n-1} + b f_n + c f_{n+1} = r
            double cp = 0.0, dp = 0.0;
            for (int n = 1; n <= N; ++n) {
                double wl = 0.0, wm = 0.0, wr = 0.0, wd = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double w = V3(U, n, a) + V3(UN, n, a);
                    wl += w * V3(UM, n - 1, a);
                    wm += w * V3(UM, n, a);
                    wr += w * V3(UM, n + 1, a);
                    wd += w * (drr(n, a) - drr(n - 1, a));
                }
                const double ca = wl * dt, cb = -2.0 * wm * dt, cc = wr * dt, rr = -wd;
                const double m = n == 1 ? cb : cb - ca * cp;
                cp = cc / m;
                dp = (n == 1 ? rr : rr - ca * dp) / m;
                CP[(size_t)(n - 1) * S + c] = cp;
                DP[(size_t)(n - 1) * S + c] = dp;
            }
            double fn = DP[(size_t)(N - 1) * S + c];
            F[(size_t)N * S + c] = fn;
            for (int n = N - 1; n >= 1; --n) {
                fn = DP[(size_t)(n - 1) * S + c] - CP[(size_t)(n - 1) * S + c] * fn;
                F[(size_t)n * S + c] = fn;
            }
            double change = 0.0;
            for (int n = 1; n <= N; ++n) {
                const double fl = F[(size_t)(n - 1) * S + c], fm = F[(size_t)n * S + c],
                             fr = F[(size_t)(n + 1) * S + c];
                for (int a = 0; a < 3; ++a) {
                    const double v = V3(U, n, a) + (drr(n, a) - drr(n - 1, a)) +
                                     (fl * V3(UM, n - 1, a) - 2.0 * fm * V3(UM, n, a) +
                                      fr * V3(UM, n + 1, a)) * dt;
                    change = fmax(change, fabs(v - V3(UN, n, a)));
                    V3(UN, n, a) = v;
                }
            }
            if (tol > 0.0 && change <= tol) break;
        }
        for (int a = 0; a < 3; ++a) r0[a] += drr(0, a) + F[(size_t)1 * S + c] * V3(UM, 1, a) * dt;
        for (int n = 1; n <= N; ++n)
            for (int a = 0; a < 3; ++a) V3(U, n, a) = V3(UN, n, a);
    }
    for (int a = 0; a < 3; ++a) {
        x[a * M] = r0[a];
        for (int n = 1; n <= N; ++n) x[a * M + n] = x[a * M + n - 1] + V3(U, n, a);
    }
#undef V3
}

// The same step with one wavefront per chain and the chain in LDS: bonds and
// beads are spread over the lanes, and the tension system is solved by
// parallel cyclic reduction (each of ceil(log2 N) rounds eliminates the
// couplings to the rows s apart, s = 1, 2, 4, ...) instead of the serial
// Thomas sweep.  LDS, doubles ([axis][index]): u, u', u^m (3 (N+2) each),
// noise and the regular displacements (3 (N+1) each), two sets of the
// tridiagonal rows a, b, c, r (4 N each) and f (N+2): wlc_lds_doubles(M).
constexpr size_t kWlcMaxLds = 64 * 1024;  // the wave kernel's LDS limit

__host__ __device__ inline size_t wlc_lds_doubles(int M)
{
    const size_t N = (size_t)M - 1;
    return 9 * (N + 2) + 6 * (N + 1) + 8 * N + (N + 2);
}

__global__ __launch_bounds__(64) void wlc_wave_kernel(double *__restrict__ pos,
                                                      const int32_t *__restrict__ ids, int M,
                                                      double T_bar, double dt, int iters,
                                                      double tol, int midpoint, uint64_t seed,
                                                      int64_t step0, int n_steps)
{
    extern __shared__ double lds[];
    const int c = blockIdx.x, t = threadIdx.x;
    const int N = M - 1, P = N + 2, Q = N + 1;
    double *U = lds, *UN = U + 3 * P, *UM = UN + 3 * P;
    double *NZ = UM + 3 * P, *D = NZ + 3 * Q;
    double *const rows = D + 3 * Q;  // set h: a, b, c, r at rows + (4 h + 0..3) N
    double *F = rows + 8 * (size_t)N;
    double *x = pos + (size_t)c * 3 * M;
    const uint32_t chain = (uint32_t)ids[c];
    const double amp = sqrt(2.0 * T_bar * dt);
    for (int i = t; i < 3 * P; i += 64) U[i] = UN[i] = UM[i] = 0.0;
    for (int i = t; i < P; i += 64) F[i] = 0.0;
    __syncthreads();
    for (int n = 1 + t; n <= N; n += 64) {  // bonds, scaled to unit length
        double u[3], s2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            u[a] = x[a * M + n] - x[a * M + n - 1];
            s2 += u[a] * u[a];
        }
        const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
        for (int a = 0; a < 3; ++a) U[a * P + n] = u[a] * inv;
    }
    double r0 = t < 3 ? x[t * M] : 0.0;
    const int nq = N / 4 + 1;
    __syncthreads();
    for (int s = 0; s < n_steps; ++s) {
        const int64_t k = step0 + s;
        for (int i = t; i < 3 * nq; i += 64) {
            const int a = i / nq, q = i - a * nq;
            double z[4];
            normals4_f64(noise_bits(seed, (uint32_t)q, chain, k, (uint32_t)a, kTagWLC), z);
            for (int e = 0; e < 4 && 4 * q + e <= N; ++e) NZ[a * Q + 4 * q + e] = amp * z[e];
        }
        for (int n = 1 + t; n <= N; n += 64)
            for (int a = 0; a < 3; ++a) UN[a * P + n] = U[a * P + n];
        __syncthreads();
        for (int it = 0; it < iters; ++it) {
            for (int n = 1 + t; n <= N; n += 64) {  // midpoint bonds
                double w[3], s2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    w[a] = U[a * P + n] + UN[a * P + n];
                    s2 += w[a] * w[a];
                }
                const double inv = 1.0 / sqrt(s2);
                for (int a = 0; a < 3; ++a) UM[a * P + n] = midpoint ? w[a] * inv : U[a * P + n];
            }
            __syncthreads();
            for (int n = t; n <= N; n += 64)  // regular displacements of the beads
                for (int a = 0; a < 3; ++a) {
                    const double *um = UM + a * P;
                    const double hn = n >= 1 ? -(um[n - 1] + um[n + 1]) : 0.0;
                    const double hn1 = n + 1 <= N ? -(um[n] + um[n + 2]) : 0.0;
                    D[a * Q + n] = (hn1 - hn) * dt + NZ[a * Q + n];
                }
            __syncthreads();
            for (int n = 1 + t; n <= N; n += 64) {  // row n: a f_{n-1} + b f_n + c f_{n+1} = r
                double wl = 0.0, wm = 0.0, wr = 0.0, wd = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double w = U[a * P + n] + UN[a * P + n];
                    wl += w * UM[a * P + n - 1];
                    wm += w * UM[a * P + n];
                    wr += w * UM[a * P + n + 1];
                    wd += w * (D[a * Q + n] - D[a * Q + n - 1]);
                }
                rows[n - 1] = wl * dt;
                rows[N + n - 1] = -2.0 * wm * dt;
                rows[2 * N + n - 1] = wr * dt;
                rows[3 * N + n - 1] = -wd;
            }
            __syncthreads();
            int h = 0;
            for (int sd = 1; sd < N; sd *= 2, h ^= 1) {
                const double *ra = rows + (size_t)(4 * h) * N, *rb = ra + N, *rc = rb + N,
                             *rr = rc + N;
                double *oa = rows + (size_t)(4 * (h ^ 1)) * N, *ob = oa + N, *oc = ob + N,
                       *od = oc + N;
                for (int j = t; j < N; j += 64) {
                    double an = 0.0, cn = 0.0, bn = rb[j], dn = rr[j];
                    if (j - sd >= 0) {
                        const double al = -ra[j] / rb[j - sd];
                        an = al * ra[j - sd];
                        bn += al * rc[j - sd];
                        dn += al * rr[j - sd];
                    }
                    if (j + sd < N) {
                        const double ga = -rc[j] / rb[j + sd];
                        cn = ga * rc[j + sd];
                        bn += ga * ra[j + sd];
                        dn += ga * rr[j + sd];
                    }
                    oa[j] = an;
                    ob[j] = bn;
                    oc[j] = cn;
                    od[j] = dn;
                }
                __syncthreads();
            }
            for (int j = t; j < N; j += 64)
                F[j + 1] = rows[(size_t)(4 * h + 3) * N + j] / rows[(size_t)(4 * h + 1) * N + j];
            __syncthreads();
            double change = 0.0;
            for (int n = 1 + t; n <= N; n += 64) {  // bond update
                const double fl = F[n - 1], fm = F[n], fr = F[n + 1];
                for (int a = 0; a < 3; ++a) {
                    const double v = U[a * P + n] + (D[a * Q + n] - D[a * Q + n - 1]) +
                                     (fl * UM[a * P + n - 1] - 2.0 * fm * UM[a * P + n] +
                                      fr * UM[a * P + n + 1]) * dt;
                    change = fmax(change, fabs(v - UN[a * P + n]));
                    UN[a * P + n] = v;
                }
            }
            __syncthreads();
            if (tol > 0.0) {  // the same maximum in every lane: a uniform exit
                for (int o = 32; o >= 1; o >>= 1) change = fmax(change, __shfl_xor(change, o));
                if (change <= tol) break;
            }
        }
        if (t < 3) r0 += D[t * Q] + F[1] * UM[t * P + 1] * dt;
        for (int n = 1 + t; n <= N; n += 64)
            for (int a = 0; a < 3; ++a) U[a * P + n] = UN[a * P + n];
        __syncthreads();
    }
    if (t < 3) {
        double v = r0;
        x[t * M] = v;
        for (int n = 1; n <= N; ++n) {
            v += U[t * P + n];
            x[t * M + n] = v;
        }
    }
}

// Chains of up to 64 beads: one wavefront per chain with bond n and bead n
// in lane n and the whole chain in registers -- neighbours by cross-lane
// reads (executed by every lane, then masked), the tension system by the
// same cyclic reduction with identity rows in the lanes that hold no bond.
// The noise blocks are drawn one per lane and handed to the beads that use
// them.  Four chains per workgroup, one per wavefront, no LDS and no
// barrier; the positions are rebuilt at the end in the serial order of the
// other kernels.
constexpr int kWlcRegMaxM = 64;

__device__ __forceinline__ double lane_read(double v, int src)
{
    return __shfl(v, src < 0 ? 0 : (src > 63 ? 63 : src), 64);
}

// The value of lane - 1 (lane 0 gets 0) or of lane + 1 (lane 63 gets 0): DPP
// whole-wavefront shifts, two 32-bit moves per double, no LDS crossbar.
template <int CTRL>
__device__ __forceinline__ double wave_shift(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF,
                                                              true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL,
                                                              0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
constexpr int kWaveShr1 = 0x138, kWaveShl1 = 0x130;
__device__ __forceinline__ double from_prev(double v) { return wave_shift<kWaveShr1>(v); }
__device__ __forceinline__ double from_next(double v) { return wave_shift<kWaveShl1>(v); }

__global__ __launch_bounds__(256) void wlc_reg_kernel(double *__restrict__ pos,
                                                      const int32_t *__restrict__ ids, int M,
                                                      int nch, double T_bar, double dt, int iters,
                                                      double tol, int midpoint, uint64_t seed,
                                                      int64_t step0, int n_steps)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = blockIdx.x * 4 + wv;
    if (c >= nch) return;  // a whole wavefront
    const int N = M - 1, nq = N / 4 + 1;
    const bool bond = lane >= 1 && lane <= N;  // this lane's bond n = lane exists
    const bool bead = lane <= N;
    double *x = pos + (size_t)c * 3 * M;
    const uint32_t chain = (uint32_t)ids[c];
    const double amp = sqrt(2.0 * T_bar * dt);
    double U[3] = {0.0, 0.0, 0.0};
    if (bond) {  // bonds, scaled to unit length
        double u[3], s2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            u[a] = x[a * M + lane] - x[a * M + lane - 1];
            s2 += u[a] * u[a];
        }
        const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
        for (int a = 0; a < 3; ++a) U[a] = u[a] * inv;
    }
    double r0[3] = {x[0], x[M], x[2 * M]};  // used in lane 0
    for (int s = 0; s < n_steps; ++s) {
        const int64_t k = step0 + s;
        // noise: lane a nq + q draws block q of component a; bead n takes
        // element n % 4 of block n / 4
        double zb[4] = {0.0, 0.0, 0.0, 0.0};
        if (lane < 3 * nq) {
            const int a = lane / nq, q = lane - a * nq;
            normals4_f64(noise_bits(seed, (uint32_t)q, chain, k, (uint32_t)a, kTagWLC), zb);
        }
        double NZ[3];
        for (int a = 0; a < 3; ++a) {
            const int src = a * nq + (lane >> 2);
            const double z0 = lane_read(zb[0], src), z1 = lane_read(zb[1], src),
                         z2 = lane_read(zb[2], src), z3 = lane_read(zb[3], src);
            const int e = lane & 3;
            const double z = e == 0 ? z0 : (e == 1 ? z1 : (e == 2 ? z2 : z3));
            NZ[a] = bead ? amp * z : 0.0;
        }
        double UN[3] = {U[0], U[1], U[2]};
        double D[3], UM[3], UMl[3], UMr[3], F = 0.0;
        for (int it = 0; it < iters; ++it) {
            double w[3];
            {  // midpoint bonds
                double s2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    w[a] = U[a] + UN[a];
                    s2 += w[a] * w[a];
                }
                const double inv = bond ? 1.0 / sqrt(s2) : 0.0;
                for (int a = 0; a < 3; ++a) UM[a] = bond ? (midpoint ? w[a] * inv : U[a]) : 0.0;
            }
            double Dl[3];
            for (int a = 0; a < 3; ++a) {  // bending gradients and bead displacements
                UMl[a] = from_prev(UM[a]);
                UMr[a] = from_next(UM[a]);
                if (lane == 0) UMl[a] = 0.0;
                if (lane == 63) UMr[a] = 0.0;
                const double h = bond ? -(UMl[a] + UMr[a]) : 0.0;
                const double h1 = from_next(h);
                const double hn1 = lane + 1 <= N ? h1 : 0.0;
                D[a] = bead ? (hn1 - h) * dt + NZ[a] : 0.0;
                const double dprev = from_prev(D[a]);
                Dl[a] = lane >= 1 ? dprev : 0.0;
            }
            // row n - 1 of the tension system in lane n; identity elsewhere
            double ra = 0.0, rb = 1.0, rc = 0.0, rr = 0.0;
            if (bond) {
                double wl = 0.0, wm = 0.0, wr = 0.0, wd = 0.0;
                for (int a = 0; a < 3; ++a) {
                    wl += w[a] * UMl[a];
                    wm += w[a] * UM[a];
                    wr += w[a] * UMr[a];
                    wd += w[a] * (D[a] - Dl[a]);
                }
                ra = wl * dt;
                rb = -2.0 * wm * dt;
                rc = wr * dt;
                rr = -wd;
            }
            for (int sd = 1; sd < N; sd *= 2) {
                const bool hasl = lane - sd >= 1, hasr = lane + sd <= N;
                double la, lb, lc, lr, qa, qb, qc, qr;
                if (sd == 1) {  // neighbours by DPP shifts
                    la = from_prev(ra), lb = from_prev(rb), lc = from_prev(rc), lr = from_prev(rr);
                    qa = from_next(ra), qb = from_next(rb), qc = from_next(rc), qr = from_next(rr);
                } else {
                    la = lane_read(ra, lane - sd), lb = lane_read(rb, lane - sd);
                    lc = lane_read(rc, lane - sd), lr = lane_read(rr, lane - sd);
                    qa = lane_read(ra, lane + sd), qb = lane_read(rb, lane + sd);
                    qc = lane_read(rc, lane + sd), qr = lane_read(rr, lane + sd);
                }
                double an = 0.0, cn = 0.0, bn = rb, dn = rr;
                if (hasl) {
                    const double al = -ra / lb;
                    an = al * la;
                    bn += al * lc;
                    dn += al * lr;
                }
                if (hasr) {
                    const double ga = -rc / qb;
                    cn = ga * qc;
                    bn += ga * qa;
                    dn += ga * qr;
                }
                if (bond) {
                    ra = an;
                    rb = bn;
                    rc = cn;
                    rr = dn;
                }
            }
            F = bond ? rr / rb : 0.0;
            const double fl = from_prev(F), fr = from_next(F);
            double change = 0.0;
            if (bond) {  // bond update
                for (int a = 0; a < 3; ++a) {
                    const double v = U[a] + (D[a] - Dl[a]) +
                                     ((lane >= 2 ? fl : 0.0) * UMl[a] - 2.0 * F * UM[a] +
                                      (lane + 1 <= N ? fr : 0.0) * UMr[a]) * dt;
                    change = fmax(change, fabs(v - UN[a]));
                    UN[a] = v;
                }
            }
            if (tol > 0.0) {  // the same maximum in every lane: a uniform exit
                for (int o = 32; o >= 1; o >>= 1) change = fmax(change, __shfl_xor(change, o));
                if (change <= tol) break;
            }
        }
        {  // bead 0 moves with its own tension, bending and noise
            const double F1 = lane_read(F, 1);
            for (int a = 0; a < 3; ++a) {
                const double um1 = lane_read(UM[a], 1);
                if (lane == 0) r0[a] += D[a] + F1 * um1 * dt;
            }
        }
        for (int a = 0; a < 3; ++a) U[a] = UN[a];
    }
    // positions: every lane forms the same serial sums, lane 0 stores them
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = __shfl(r0[a], 0, 64);
    if (lane == 0)
        for (int a = 0; a < 3; ++a) x[a * M] = v[a];
    for (int n = 1; n <= N; ++n)
        for (int a = 0; a < 3; ++a) {
            v[a] += __shfl(U[a], n, 64);
            if (lane == 0) x[a * M + n] = v[a];
        }
}

__global__ void reduce_chains_kernel(const double *__restrict__ acc, double *__restrict__ out,
                                     int width, int nch)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= width) return;
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += acc[(size_t)c * width + j];
    out[j] = s;
}

template <typename T>
__global__ void check_finite_kernel(const T *__restrict__ x, size_t n, int *flag)
{
    int bad = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        bad |= !isfinite(x[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

__global__ void scatter_chains_kernel(const double *__restrict__ src, double *__restrict__ dst,
                                      const int64_t *__restrict__ off, int len, int nch)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nch * len) return;
    const int c = (int)(idx / len), i = (int)(idx % len);
    dst[off[c] + i] = src[idx];
}

inline unsigned blocks_for(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_gemm_f64(const double *A, const double *X, double *Y, int M, int ncol,
                           hipStream_t st)
{
    if (M <= 0 || ncol <= 0) return hipSuccess;
    dim3 grid((M + kGemmBM - 1) / kGemmBM, (ncol + kGemmBN - 1) / kGemmBN);
    if (M % kGemmBK == 0) {
        // narrower column tiles while 64 x 64 tiles would not give every CU
        // of the GPU two workgroups
        if (grid.x * grid.y < 512) {
            const dim3 g1(grid.x * ((ncol + 31) / 32));
            hipLaunchKernelGGL(gemm_f64_pipe_kernel<32>, g1, dim3(256), 0, st, A, X, Y, M,
                               ncol);
        } else {
            const dim3 g1(grid.x * grid.y);
            hipLaunchKernelGGL(gemm_f64_pipe_kernel<64>, g1, dim3(256), 0, st, A, X, Y, M,
                               ncol);
        }
    } else {
        hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, st, A, X, Y, M, ncol);
    }
    return hipGetLastError();
}

hipError_t launch_stencil_f64(const double *r, double *F, int M, int nch, double lin,
                              hipStream_t st)
{
    const size_t n = (size_t)nch * M;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(stencil_f64_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, r, F, M,
                       nch, lin);
    return hipGetLastError();
}

hipError_t launch_mode_update_f64(double *R, const double *dH, const double *E, const double *C,
                                  const double *W, const int32_t *ids, int M, int nch,
                                  uint64_t seed, const int64_t *step_dev, int64_t step_off,
                                  double gdt, int nonlinear, hipStream_t st)
{
    const size_t n = (size_t)nch * ((M + 3) / 4);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(mode_update_f64_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, R,
                       dH, E, C, W, ids, M, nch, seed, step_dev, step_off, gdt, nonlinear);
    return hipGetLastError();
}

hipError_t launch_euler_f64(double *pos, const int32_t *ids, int M, int nch, double nu,
                            double dtau, double T_star, double gdt, uint64_t seed, int64_t step0,
                            int n_steps, hipStream_t st)
{
    if (nch == 0 || n_steps == 0) return hipSuccess;
    const int nq = (M + 3) / 4;
    if (nq > 1024) return hipErrorInvalidValue;
    const int threads = ((nq + 63) / 64) * 64;
    const size_t lds = sizeof(double) * 3 * (size_t)M;
    if (lds > 64 * 1024) return hipErrorInvalidValue;  // positions must fit the LDS
    hipLaunchKernelGGL(euler_f64_kernel, dim3(nch), dim3(threads), lds, st, pos, ids, M, nu,
                       dtau, sqrt(2.0 * T_star * dtau), gdt, seed, step0, n_steps);
    return hipGetLastError();
}

size_t wlc_scratch_doubles(int M, int nch)
{
    if (sizeof(double) * wlc_lds_doubles(M) <= kWlcMaxLds) return 0;  // chain held in LDS
    const size_t N = (size_t)M - 1;
    return (9 * (N + 2) + 3 * (N + 1) + 2 * N + (N + 2)) * (size_t)nch;
}

hipError_t launch_wlc(double *pos, double *scr, const int32_t *ids, int M, int nch, double T_bar,
                      double dt, int iters, double tol, int midpoint, uint64_t seed,
                      int64_t step0, int n_steps, hipStream_t st)
{
    if (nch == 0 || n_steps == 0) return hipSuccess;
    if (M < 2 || iters < 1) return hipErrorInvalidValue;
    if (M <= kWlcRegMaxM) {
        hipLaunchKernelGGL(wlc_reg_kernel, dim3((nch + 3) / 4), dim3(256), 0, st, pos, ids, M, nch,
                           T_bar, dt, iters, tol, midpoint, seed, step0, n_steps);
        return hipGetLastError();
    }
    const size_t lds = sizeof(double) * wlc_lds_doubles(M);
    if (lds <= kWlcMaxLds) {
        hipLaunchKernelGGL(wlc_wave_kernel, dim3(nch), dim3(64), lds, st, pos, ids, M, T_bar, dt,
                           iters, tol, midpoint, seed, step0, n_steps);
        return hipGetLastError();
    }
    if (!scr) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wlc_kernel, dim3((nch + 63) / 64), dim3(64), 0, st, pos, scr, ids, M, nch,
                       T_bar, dt, iters, tol, midpoint, seed, step0, n_steps);
    return hipGetLastError();
}

hipError_t launch_mc(double *R, const double *chiT, const double *sstep, const int32_t *ids,
                     int M, int nch, double nu, double T_star, uint64_t seed, int64_t step0,
                     int n_sweeps, int64_t *accepted, hipStream_t st)
{
    if (nch == 0 || n_sweeps == 0) return hipSuccess;
    const size_t lds = sizeof(double) * (3 * (size_t)(M - 1) + 3 * (size_t)M);
    if (M < 2 || lds > 64 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mc_kernel, dim3(nch), dim3(64), lds, st, R, chiT, sstep, ids, M, nu,
                       T_star, seed, step0, n_sweeps, accepted);
    return hipGetLastError();
}

hipError_t launch_chain_obs(const double *pos, const double *R, double *obs, double *m2,
                            double *acc, const double *cm0, double *tstate, double *tlast,
                            const int64_t *step_dev, double *ring, double *ccount, int K, int M,
                            int nch, int accumulate, hipStream_t st)
{
    if (nch == 0) return hipSuccess;
    hipLaunchKernelGGL(chain_obs_kernel, dim3(nch), dim3(64), 0, st, pos, R, obs, m2, acc, cm0,
                       tstate, tlast, step_dev, ring, ccount, K, M, accumulate);
    return hipGetLastError();
}

hipError_t launch_reduce_chains(const double *acc, double *out, int width, int nch,
                                hipStream_t st)
{
    hipLaunchKernelGGL(reduce_chains_kernel, dim3(blocks_for(width, 256)), dim3(256), 0, st, acc,
                       out, width, nch);
    return hipGetLastError();
}

hipError_t launch_check_finite_f64(const double *x, size_t n, int *flag, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    unsigned b = blocks_for(n, 256);
    if (b > 2048) b = 2048;
    hipLaunchKernelGGL(check_finite_kernel<double>, dim3(b), dim3(256), 0, st, x, n, flag);
    return hipGetLastError();
}

hipError_t launch_check_finite_f32(const float *x, size_t n, int *flag, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    unsigned b = blocks_for(n, 256);
    if (b > 2048) b = 2048;
    hipLaunchKernelGGL(check_finite_kernel<float>, dim3(b), dim3(256), 0, st, x, n, flag);
    return hipGetLastError();
}

hipError_t launch_scatter_chains(const double *src, double *dst, const int64_t *off, int len,
                                 int nch, hipStream_t st)
{
    const size_t n = (size_t)nch * len;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_chains_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, src,
                       dst, off, len, nch);
    return hipGetLastError();
}

}  // namespace dm
