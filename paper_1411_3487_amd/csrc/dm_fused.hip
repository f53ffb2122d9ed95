// dm_fused.hip -- fused multi-step mode stepper in reduced precision (gfx950).
//
// One wavefront owns a tile of 5 chains and keeps their internal mode
// amplitudes in registers for a whole block of steps.  Each step runs
//   u = chi R            bond vectors from modes          (Eq. e5)
//   g_n = u_n (1/|u_n| - (1-2nu))                          (Eqs. e4, e11)
//   Delta H = chi^T g                                      (Eq. e11)
//   R <- E R + C Delta H + W eta (+ shear)                 (Eqs. d3, d6, f2, btum)
// with chi_{n,p} = phi_{n,p} - phi_{n-1,p} (Eq. e3, computed as the
// difference).  Applying the bond difference inside the transform keeps the
// O(|u|) bond vectors free of the O(M |u|) positions, which is what lets the
// transforms run in FP32 or split BF16.
//
// Mirror symmetry (Sec. 5a: phi_{N-n,p} = (-1)^p phi_{n,p}) gives
// chi_{M-n,p} = (-1)^{p+1} chi_{n,p}: for half-bond rows i = 1..H (H = M/2)
//   S_i = sum_{p odd} chi_{i,p} R_p,  A_i = sum_{p even} chi_{i,p} R_p,
//   u_i = S_i + A_i,  u_{M-i} = S_i - A_i,
//   Delta H_{p odd}  = sum_i chi_{i,p} (g_i + g_{M-i}),
//   Delta H_{p even} = sum_i chi_{i,p} (g_i - g_{M-i}),
// (the middle bond i = H counted once), so each transform is two H x H
// products instead of one M x M product: half the MFMA work.
//
// MFMA layout.  Columns of every product are the 15 (chain, component)
// pairs of the tile plus one unused column; col = 3 * chain + component.
// A 16x16 result tile puts column l%16 and rows 4(l/16)+r (r = 0..3) in lane
// l, which is the lane/K layout the next product needs for its B operand, so
// results chain into the next MFMA without data movement; the transform
// tables are stored pre-permuted to the same K order ("fragment order").
//   FP32 path : v_mfma_f32_16x16x4_f32, one K = 4 slab per (tile, r).
//   BF16X3    : v_mfma_f32_16x16x32_bf16 over K = 32 slabs (two row tiles);
//               x = x_hi + x_lo for both operands, products
//               hi*hi + hi*lo + lo*hi accumulated in FP32.
// The centre-of-mass mode R_0 (p = 0) is kept in FP64 in lanes 0..14.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "dm_fused.h"
#include "dm_rng.h"

namespace dm {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kChainsPerTile = 5;

struct FusedArgs {
    const void *X;
    float *R;
    double *R0;
    const float *coef;
    const int32_t *ids;
    int M, H, n, ntiles;
    uint64_t seed;
    int64_t step0;
    int n_steps, nonlinear;
    float lin;
    double W0, gdt;
};

// Sum of v over the three component lanes of this lane's chain
// (columns 3c, 3c+1, 3c+2 of a 16-lane row); alpha = column % 3.
__device__ __forceinline__ float comp_sum(float v, int lane, int alpha)
{
    const float a = __shfl(v, (lane + 1) & 63, 64);
    const float b = __shfl(v, (lane + 2) & 63, 64);
    const float s = v + a + b;  // complete in the alpha == 0 lane
    return __shfl(s, lane - alpha, 64);
}

// The transform tables do not change between steps; without this the
// compiler hoists every table load out of the step loop into registers and
// spills.  Adding an opaque zero at each use site keeps the loads in place
// (and in the global address space).
template <typename T>
__device__ __forceinline__ const T *opaque(const T *p)
{
    int zero = 0;
    asm volatile("" : "+s"(zero));
    return p + zero;
}

__device__ __forceinline__ void split_bf16(const f32x4 lo4, const f32x4 hi4, bf16x8 &h, bf16x8 &l)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float v = e < 4 ? lo4[e] : hi4[e - 4];
        const __bf16 vh = (__bf16)v;
        h[e] = vh;
        l[e] = (__bf16)(v - (float)vh);
    }
}

template <int RT, bool BF16>
__global__ __launch_bounds__(256) void fused_kernel(FusedArgs a)
{
    __shared__ float cf[4 * 32 * RT];  // E, C, W, gdt*E per mode slot
    for (int i = threadIdx.x; i < 4 * 32 * RT; i += blockDim.x) cf[i] = a.coef[i];
    __syncthreads();
    const float *cE = cf, *cC = cf + 32 * RT, *cW = cf + 64 * RT, *cS = cf + 96 * RT;

    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= a.ntiles) return;
    const int col = lane & 15, g = lane >> 4;
    const int cl = col / 3, alpha = col - 3 * cl;
    const int nvalid = min(kChainsPerTile, a.n - kChainsPerTile * tile);
    const bool valid = (col < 15) && (cl < nvalid);
    const uint32_t chain = valid ? (uint32_t)a.ids[kChainsPerTile * tile + cl] : 0u;
    const float vmask = valid ? 1.0f : 0.0f;

    f32x4 Ro[RT], Re[RT];
    const f32x4 *Rt = reinterpret_cast<const f32x4 *>(a.R) + (size_t)tile * 2 * RT * 64;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        Ro[t] = Rt[(0 * RT + t) * 64 + lane];
        Re[t] = Rt[(1 * RT + t) * 64 + lane];
    }
    const bool com_lane = valid && g == 0;
    double r0 = com_lane ? a.R0[(size_t)tile * 16 + col] : 0.0;

    for (int s = 0; s < a.n_steps; ++s) {
        const int64_t k = a.step0 + s;
        // ---------------- bond forces: G+ / G- over half-bond rows
        f32x4 Gp[RT], Gm[RT];
        if (a.nonlinear) {
            if constexpr (BF16) {
                constexpr int KS = RT / 2, TS = RT * KS * 64;
                bf16x8 Boh[KS], Bol[KS], Beh[KS], Bel[KS];
#pragma unroll
                for (int q = 0; q < KS; ++q) {
                    split_bf16(Ro[2 * q], Ro[2 * q + 1], Boh[q], Bol[q]);
                    split_bf16(Re[2 * q], Re[2 * q + 1], Beh[q], Bel[q]);
                }
#pragma unroll
                for (int I = 0; I < RT; ++I) {
                    const bf16x8 *X1 = opaque(reinterpret_cast<const bf16x8 *>(a.X));
                    f32x4 aS = {0.f, 0.f, 0.f, 0.f}, aA = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int q = 0; q < KS; ++q) {
                        const int off = (I * KS + q) * 64 + lane;
                        const bf16x8 xoh = X1[0 * TS + off], xol = X1[1 * TS + off];
                        const bf16x8 xeh = X1[2 * TS + off], xel = X1[3 * TS + off];
                        aS = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xoh, Boh[q], aS, 0, 0, 0);
                        aA = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xeh, Beh[q], aA, 0, 0, 0);
                        aS = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xoh, Bol[q], aS, 0, 0, 0);
                        aA = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xeh, Bel[q], aA, 0, 0, 0);
                        aS = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xol, Boh[q], aS, 0, 0, 0);
                        aA = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xel, Beh[q], aA, 0, 0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 16 * I + 4 * g + r;
                        const float up = aS[r] + aA[r], um = aS[r] - aA[r];
                        const float sp = comp_sum(up * up, lane, alpha);
                        const float sm = comp_sum(um * um, lane, alpha);
                        const float gp = up * (__builtin_amdgcn_rsqf(sp) - a.lin);
                        const float gm = um * (__builtin_amdgcn_rsqf(sm) - a.lin);
                        const bool ok = valid && i < a.H;
                        const bool mid = (i == a.H - 1);
                        Gp[I][r] = ok ? (mid ? gp : gp + gm) : 0.0f;
                        Gm[I][r] = (ok && !mid) ? gp - gm : 0.0f;
                    }
                }
            } else {
                constexpr int TS = RT * RT * 64;
#pragma unroll
                for (int I = 0; I < RT; ++I) {
                    const f32x4 *X1 = opaque(reinterpret_cast<const f32x4 *>(a.X));
                    f32x4 aS = {0.f, 0.f, 0.f, 0.f}, aA = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
                        const int off = (I * RT + t) * 64 + lane;
                        const f32x4 xo = X1[0 * TS + off], xe = X1[1 * TS + off];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            aS = __builtin_amdgcn_mfma_f32_16x16x4f32(xo[r], Ro[t][r], aS, 0, 0, 0);
                            aA = __builtin_amdgcn_mfma_f32_16x16x4f32(xe[r], Re[t][r], aA, 0, 0, 0);
                        }
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 16 * I + 4 * g + r;
                        const float up = aS[r] + aA[r], um = aS[r] - aA[r];
                        const float sp = comp_sum(up * up, lane, alpha);
                        const float sm = comp_sum(um * um, lane, alpha);
                        const float gp = up * (__builtin_amdgcn_rsqf(sp) - a.lin);
                        const float gm = um * (__builtin_amdgcn_rsqf(sm) - a.lin);
                        const bool ok = valid && i < a.H;
                        const bool mid = (i == a.H - 1);
                        Gp[I][r] = ok ? (mid ? gp : gp + gm) : 0.0f;
                        Gm[I][r] = (ok && !mid) ? gp - gm : 0.0f;
                    }
                }
            }
        }
        // ---------------- coupling per mode tile J, then the mode update
        [[maybe_unused]] bf16x8 Gph[RT / 2], Gpl[RT / 2], Gmh[RT / 2], Gml[RT / 2];
        if constexpr (BF16) {
            if (a.nonlinear) {
#pragma unroll
                for (int q = 0; q < RT / 2; ++q) {
                    split_bf16(Gp[2 * q], Gp[2 * q + 1], Gph[q], Gpl[q]);
                    split_bf16(Gm[2 * q], Gm[2 * q + 1], Gmh[q], Gml[q]);
                }
            }
        }
#pragma unroll
        for (int J = 0; J < RT; ++J) {
            f32x4 dO = {0.f, 0.f, 0.f, 0.f}, dE = {0.f, 0.f, 0.f, 0.f};
            if (a.nonlinear) {
                if constexpr (BF16) {
                    constexpr int KS = RT / 2, TS = RT * KS * 64;
                    const bf16x8 *X2 = opaque(reinterpret_cast<const bf16x8 *>(a.X)) + 4 * TS;
#pragma unroll
                    for (int q = 0; q < KS; ++q) {
                        const int off = (J * KS + q) * 64 + lane;
                        const bf16x8 xoh = X2[0 * TS + off], xol = X2[1 * TS + off];
                        const bf16x8 xeh = X2[2 * TS + off], xel = X2[3 * TS + off];
                        dO = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xoh, Gph[q], dO, 0, 0, 0);
                        dE = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xeh, Gmh[q], dE, 0, 0, 0);
                        dO = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xoh, Gpl[q], dO, 0, 0, 0);
                        dE = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xeh, Gml[q], dE, 0, 0, 0);
                        dO = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xol, Gph[q], dO, 0, 0, 0);
                        dE = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xel, Gmh[q], dE, 0, 0, 0);
                    }
                } else {
                    constexpr int TS = RT * RT * 64;
                    const f32x4 *X2 = opaque(reinterpret_cast<const f32x4 *>(a.X)) + 2 * TS;
#pragma unroll
                    for (int I = 0; I < RT; ++I) {
                        const int off = (J * RT + I) * 64 + lane;
                        const f32x4 xo = X2[0 * TS + off], xe = X2[1 * TS + off];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            dO = __builtin_amdgcn_mfma_f32_16x16x4f32(xo[r], Gp[I][r], dO, 0, 0, 0);
                            dE = __builtin_amdgcn_mfma_f32_16x16x4f32(xe[r], Gm[I][r], dE, 0, 0, 0);
                        }
                    }
                }
            }
            // modes of this lane: p = 32J + 8g + m, m = 0..7; even p = .. + 2r
            // sits in Re[J][r], odd p = .. + 2r + 1 in Ro[J][r]
            float z[8];
            normals4_f32(noise_bits(a.seed, (uint32_t)(8 * J + 2 * g), chain, k, (uint32_t)alpha,
                                    kTagMode),
                         z);
            normals4_f32(noise_bits(a.seed, (uint32_t)(8 * J + 2 * g + 1), chain, k,
                                    (uint32_t)alpha, kTagMode),
                         z + 4);
            // opaque zero: keeps the coefficient reads inside the step loop
            int cb = (J * 4 + g) * 8;
            asm volatile("" : "+v"(cb));
            f32x4 ye = {0.f, 0.f, 0.f, 0.f}, yo = {0.f, 0.f, 0.f, 0.f};
            if (a.gdt != 0.0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    ye[r] = __shfl(Re[J][r], (lane + 1) & 63, 64);
                    yo[r] = __shfl(Ro[J][r], (lane + 1) & 63, 64);
                }
            }
            const float shear = alpha == 0 ? 1.0f : 0.0f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int me = cb + 2 * r, mo = me + 1;
                float ve = cE[me] * Re[J][r] + cW[me] * z[2 * r];
                float vo = cE[mo] * Ro[J][r] + cW[mo] * z[2 * r + 1];
                ve += cC[me] * dE[r];
                vo += cC[mo] * dO[r];
                ve += shear * cS[me] * ye[r];
                vo += shear * cS[mo] * yo[r];
                Re[J][r] = vmask * ve;
                Ro[J][r] = vmask * vo;
            }
            if (J == 0) {
                // centre of mass (p = 0, slot m = 0 of the g = 0 lanes): free
                // random walk in FP64, shear drift from R_0^y
                const double r0y = __shfl(r0, (lane + 1) & 63, 64);
                double nr0 = r0 + a.W0 * (double)z[0];
                if (alpha == 0) nr0 += a.gdt * r0y;
                r0 = com_lane ? nr0 : 0.0;
            }
        }
    }
    f32x4 *Rw = reinterpret_cast<f32x4 *>(a.R) + (size_t)tile * 2 * RT * 64;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        Rw[(0 * RT + t) * 64 + lane] = Ro[t];
        Rw[(1 * RT + t) * 64 + lane] = Re[t];
    }
    if (com_lane) a.R0[(size_t)tile * 16 + col] = r0;
}

// Slot of mode p >= 1 of (local chain j, component alpha) in the state.
__device__ __forceinline__ size_t state_slot(int j, int alpha, int p, int RT)
{
    const int T = j / kChainsPerTile, cl = j % kChainsPerTile, col = 3 * cl + alpha;
    const int set = (p & 1) ? 0 : 1;
    const int jj = (p & 1) ? (p - 1) / 2 : p / 2;
    const int t = jj / 16, rho = jj % 16;
    const int lane = 16 * (rho / 4) + col;
    return (((size_t)T * 2 + set) * RT + t) * 256 + (size_t)lane * 4 + (rho % 4);
}

__global__ void pack_kernel(const double *__restrict__ R64, float *__restrict__ R,
                            double *__restrict__ R0, int M, int n, int RT)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n * 3 * M) return;
    const int p = (int)(idx % M);
    const int alpha = (int)((idx / M) % 3);
    const int j = (int)(idx / ((size_t)3 * M));
    const double v = R64[idx];
    if (p == 0) {
        R0[(size_t)(j / kChainsPerTile) * 16 + 3 * (j % kChainsPerTile) + alpha] = v;
    } else {
        R[state_slot(j, alpha, p, RT)] = (float)v;
    }
}

__global__ void unpack_kernel(const float *__restrict__ R, const double *__restrict__ R0,
                              double *__restrict__ R64, int M, int n, int RT)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n * 3 * M) return;
    const int p = (int)(idx % M);
    const int alpha = (int)((idx / M) % 3);
    const int j = (int)(idx / ((size_t)3 * M));
    R64[idx] = (p == 0)
                   ? R0[(size_t)(j / kChainsPerTile) * 16 + 3 * (j % kChainsPerTile) + alpha]
                   : (double)R[state_slot(j, alpha, p, RT)];
}

template <typename T>
__global__ void finite_kernel(const T *__restrict__ x, size_t n, int *flag)
{
    int bad = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        bad |= !isfinite(x[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

int tiles_of(int n) { return (n + kChainsPerTile - 1) / kChainsPerTile; }
int rt_of(int M)
{
    const int H = M / 2;
    return ((H + 31) / 32) * 2;
}
size_t state_floats(int RT, int ntiles) { return (size_t)ntiles * 2 * RT * 256; }
size_t x_bytes(int RT, bool bf16)
{
    // 4 products (GEMM1 odd/even, GEMM2 odd/even) of RT x RT tiles of 256 values
    return (size_t)4 * RT * RT * 256 * (bf16 ? 2 * sizeof(__bf16) : sizeof(float));
}

// K index of slot e in lane group gq of K-slab q (BF16, K = 32 per slab).
inline int kslab_index(int q, int gq, int e)
{
    return 32 * q + (e < 4 ? 4 * gq + e : 16 + 4 * gq + (e - 4));
}

unsigned nblocks(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

bool fused_supports(int M) { return M >= 2 && M <= 512 && (M % 2) == 0; }

hipError_t fused_alloc(FusedBucket &f, int M, int n, bool bf16, const std::vector<double> &phi)
{
    f.bf16 = bf16 ? 1 : 0;
    f.RT = rt_of(M);
    f.ntiles = tiles_of(n);
    const int RT = f.RT, H = M / 2, Hp = 16 * RT;
    // half-bond x half-mode tables: Xo[i][j] = chi_{i+1, 2j+1}, Xe[i][j] = chi_{i+1, 2j}
    std::vector<double> Xo((size_t)Hp * Hp, 0.0), Xe((size_t)Hp * Hp, 0.0);
    auto chi = [&](int bond, int p) {
        return phi[(size_t)bond * M + p] - phi[(size_t)(bond - 1) * M + p];
    };
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < H; ++j) {
            Xo[(size_t)i * Hp + j] = chi(i + 1, 2 * j + 1);
            // the middle bond has no antisymmetric part: chi_{H, even} = 0 exactly
            Xe[(size_t)i * Hp + j] = (j == 0 || i == H - 1) ? 0.0 : chi(i + 1, 2 * j);
        }
    const size_t xb = x_bytes(RT, bf16);
    hipError_t e;
    if ((e = hipMalloc(&f.d_X, xb)) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&f.d_R, sizeof(float) * state_floats(RT, f.ntiles))) != hipSuccess)
        return e;
    if ((e = hipMalloc((void **)&f.d_R0, sizeof(double) * 16 * (size_t)f.ntiles)) != hipSuccess)
        return e;
    if ((e = hipMalloc((void **)&f.d_coef, sizeof(float) * 128 * (size_t)RT)) != hipSuccess)
        return e;
    const double *src[2] = {Xo.data(), Xe.data()};
    if (!bf16) {
        // GEMM1 (I, t, lane, r): X[16I + lane%16][16t + 4(lane/16) + r]
        // GEMM2 (J, I, lane, r): X[16I + 4(lane/16) + r][16J + lane%16]
        std::vector<float> h((size_t)4 * RT * RT * 256);
        const size_t TS = (size_t)RT * RT * 256;
        for (int kind = 0; kind < 2; ++kind)
            for (int A = 0; A < RT; ++A)
                for (int B = 0; B < RT; ++B)
                    for (int l = 0; l < 64; ++l)
                        for (int r = 0; r < 4; ++r) {
                            const size_t o = (((size_t)A * RT + B) * 64 + l) * 4 + r;
                            const int lo = l % 16, hi = 4 * (l / 16) + r;
                            h[kind * TS + o] = (float)src[kind][(size_t)(16 * A + lo) * Hp + 16 * B + hi];
                            h[(2 + kind) * TS + o] =
                                (float)src[kind][(size_t)(16 * B + hi) * Hp + 16 * A + lo];
                        }
        e = hipMemcpy(f.d_X, h.data(), xb, hipMemcpyHostToDevice);
    } else {
        // slabs of K = 32: GEMM1 (I, q, lane, e): X[16I + lane%16][k(q, lane/16, e)]
        //                  GEMM2 (J, q, lane, e): X[k(q, lane/16, e)][16J + lane%16]
        // tables in the order [GEMM1 o hi, o lo, e hi, e lo, GEMM2 o hi, o lo, e hi, e lo]
        const int KS = RT / 2;
        const size_t TS = (size_t)RT * KS * 512;
        std::vector<__bf16> h(8 * TS);
        for (int kind = 0; kind < 2; ++kind)
            for (int A = 0; A < RT; ++A)
                for (int q = 0; q < KS; ++q)
                    for (int l = 0; l < 64; ++l)
                        for (int el = 0; el < 8; ++el) {
                            const size_t o = (((size_t)A * KS + q) * 64 + l) * 8 + el;
                            const int kk = kslab_index(q, l / 16, el), lo = l % 16;
                            const double v1 = src[kind][(size_t)(16 * A + lo) * Hp + kk];
                            const double v2 = src[kind][(size_t)kk * Hp + 16 * A + lo];
                            const __bf16 h1 = (__bf16)(float)v1, h2 = (__bf16)(float)v2;
                            h[(2 * kind + 0) * TS + o] = h1;
                            h[(2 * kind + 1) * TS + o] = (__bf16)(float)(v1 - (double)(float)h1);
                            h[(4 + 2 * kind + 0) * TS + o] = h2;
                            h[(4 + 2 * kind + 1) * TS + o] = (__bf16)(float)(v2 - (double)(float)h2);
                        }
        e = hipMemcpy(f.d_X, h.data(), xb, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return e;
    return hipMemset(f.d_R, 0, sizeof(float) * state_floats(RT, f.ntiles));
}

void fused_free(FusedBucket &f)
{
    if (f.d_X) (void)hipFree(f.d_X);
    if (f.d_R) (void)hipFree(f.d_R);
    if (f.d_R0) (void)hipFree(f.d_R0);
    if (f.d_coef) (void)hipFree(f.d_coef);
    f = FusedBucket();
}

hipError_t fused_pack_modes(FusedBucket &f, const double *R64, int M, int n, hipStream_t st)
{
    const size_t N = (size_t)n * 3 * M;
    hipLaunchKernelGGL(pack_kernel, dim3(nblocks(N, 256)), dim3(256), 0, st, R64, f.d_R, f.d_R0,
                       M, n, f.RT);
    return hipGetLastError();
}

hipError_t fused_unpack_modes(const FusedBucket &f, double *R64, int M, int n, hipStream_t st)
{
    const size_t N = (size_t)n * 3 * M;
    hipLaunchKernelGGL(unpack_kernel, dim3(nblocks(N, 256)), dim3(256), 0, st, f.d_R, f.d_R0,
                       R64, M, n, f.RT);
    return hipGetLastError();
}

hipError_t fused_set_coefs(FusedBucket &f, const ModeCoefs &mc, int M, double lin, double gdt,
                           hipStream_t st)
{
    const int RT = f.RT;
    std::vector<float> h((size_t)128 * RT, 0.0f);
    // slot (J, g, m) <-> mode p = 32J + 8g + m; p = 0 (centre of mass) and
    // padding p >= M stay zero
    for (int slot = 0; slot < 32 * RT; ++slot) {
        const int p = slot;
        if (p == 0 || p >= M) continue;
        h[slot] = (float)mc.E[p];
        h[32 * RT + slot] = (float)mc.C[p];
        h[64 * RT + slot] = (float)mc.W[p];
        h[96 * RT + slot] = (float)(gdt * mc.E[p]);
    }
    f.W0 = mc.W[0];
    f.gdt = gdt;
    f.lin = (float)lin;
    hipError_t e = hipMemcpyAsync(f.d_coef, h.data(), sizeof(float) * h.size(),
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

template <int RT>
static hipError_t launch_rt(const FusedBucket &f, const FusedArgs &a, hipStream_t st)
{
    const dim3 grid(nblocks(f.ntiles, 4)), block(256);
    if (f.bf16)
        hipLaunchKernelGGL((fused_kernel<RT, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((fused_kernel<RT, false>), grid, block, 0, st, a);
    return hipGetLastError();
}

hipError_t fused_step(FusedBucket &f, const int32_t *ids, int M, int n, uint64_t seed,
                      int64_t step0, int n_steps, int nonlinear, hipStream_t st)
{
    if (n_steps <= 0 || n <= 0) return hipSuccess;
    FusedArgs a;
    a.X = f.d_X;
    a.R = f.d_R;
    a.R0 = f.d_R0;
    a.coef = f.d_coef;
    a.ids = ids;
    a.M = M;
    a.H = M / 2;
    a.n = n;
    a.ntiles = f.ntiles;
    a.seed = seed;
    a.step0 = step0;
    a.n_steps = n_steps;
    a.nonlinear = nonlinear;
    a.lin = f.lin;
    a.W0 = f.W0;
    a.gdt = f.gdt;
    switch (f.RT) {
    case 2: return launch_rt<2>(f, a, st);
    case 4: return launch_rt<4>(f, a, st);
    case 6: return launch_rt<6>(f, a, st);
    case 8: return launch_rt<8>(f, a, st);
    case 10: return launch_rt<10>(f, a, st);
    case 12: return launch_rt<12>(f, a, st);
    case 14: return launch_rt<14>(f, a, st);
    case 16: return launch_rt<16>(f, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t fused_check_finite(const FusedBucket &f, int M, int n, int *flag, hipStream_t st)
{
    (void)M;
    (void)n;
    const size_t nf = state_floats(f.RT, f.ntiles), nd = (size_t)16 * f.ntiles;
    unsigned b = nblocks(nf, 256);
    if (b > 2048) b = 2048;
    hipLaunchKernelGGL(finite_kernel<float>, dim3(b), dim3(256), 0, st, f.d_R, nf, flag);
    hipLaunchKernelGGL(finite_kernel<double>, dim3(nblocks(nd, 256)), dim3(256), 0, st, f.d_R0,
                       nd, flag);
    return hipGetLastError();
}

}  // namespace dm
