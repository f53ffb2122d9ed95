// dm_fused.hip -- fused multi-step mode stepper in reduced precision (gfx950).
//
// One wavefront owns a tile of 5 chains and keeps their internal mode
// amplitudes in registers for a whole block of steps.  Each step runs
//   u = chi R            bond vectors from modes          (Eq. e5)
//   g_n = u_n (1/|u_n| - (1-2nu))                          (Eqs. e4, e11)
//   Delta H = chi^T g                                      (Eq. e11)
//   R <- E R + C Delta H + W eta (+ shear)                 (Eqs. d3, d6, f2, btum)
// with chi_{n,p} = phi_{n,p} - phi_{n-1,p} = sigma_p sin(p n pi/M),
// sigma_p = -2 sqrt(2/M) sin(p pi/2M) (the difference of two modes of
// Eq. c8; Eq. e3 prints the opposite sign).  Applying the bond difference
// inside the transform keeps the O(|u|) bond vectors free of the O(M |u|)
// positions, which is what lets the transforms run in FP32 or split BF16.
//
// Mirror symmetry (Sec. V.A: phi_{N-n,p} = (-1)^p phi_{n,p}) gives
// chi_{M-n,p} = (-1)^{p+1} chi_{n,p}: for half-bond rows i = 1..H (H = M/2)
//   S_i = sum_{p odd} chi_{i,p} R_p,  A_i = sum_{p even} chi_{i,p} R_p,
//   u_i = S_i + A_i,  u_{M-i} = S_i - A_i,
//   Delta H_{p odd}  = sum_i chi_{i,p} (g_i + g_{M-i}),
//   Delta H_{p even} = sum_i chi_{i,p} (g_i - g_{M-i}),
// (the middle bond i = H counted once), so each transform is two H x H
// products instead of one M x M product: half the MFMA work.
//
// Even modes.  Slot j of the even half holds p = 2j + 2 (the p = 0 centre of
// mass is kept apart, in FP64) scaled as Rt_p = sigma_p R_p.  With bond row
// i <-> bond i + 1 the even-mode table is then
//   S_{ij} = sin((i+1)(j+1) pi / H),
// which is symmetric, so the coupling product Delta H_even = sigma S G- reads
// the very fragments of u = chi R: in LDS the tables take the u = chi R
// product plus the odd-mode coupling rows only.  The update of a scaled
// amplitude is Rt <- E Rt + sigma^2 C (S G-) + sigma W eta.
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

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>
#include <string>
#include <vector>

#include "dm_fused.h"
#include "dm_internal.h"
#include "dm_rng.h"

namespace dm {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kChainsPerTile = 5;

// Per-slot coefficients of the update, [kind][16 RT half-mode slots]: odd
// mode E, W, gdt E; even mode E, sigma W, gdt E, sigma^2 C.
enum { kEo, kWo, kGo, kEe, kWe, kGe, kCe, kKinds };

// One length bucket as the kernel sees it (read from device memory).
struct BucketArgs {
    const void *X;        // transform tables, fragment order
    float *R;             // internal mode amplitudes, fragment order
    double *R0;           // centre-of-mass mode, 16 doubles per tile
    const float *coef;    // [kind][16 RT] update coefficients
    const int32_t *ids;   // global chain index of each local chain
    int n, ntiles, x_bytes, jc, variant, tpw;
    float lin;
    double W0, gdt;
};

// One workgroup of a launch: tiles tile0 .. tile0 + tpw - 1 of one bucket.
struct Item {
    int bucket, tile0;
};

struct LaunchArgs {
    const BucketArgs *buckets;
    const Item *items;
    const int64_t *step;  // Philox step of the first step, or null: step0
    int64_t step0;
    uint64_t seed;
    int n_steps, nonlinear;
};

// DPP lane moves inside a 16-lane row (out-of-row sources read 0):
// row_shl:n gives lane i the value of lane i+n, row_shr:n that of lane i-n.
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
constexpr int kRowShl1 = 0x101, kRowShl2 = 0x102, kRowShr1 = 0x111, kRowShr2 = 0x112;

// Sum of v over the three component lanes of this lane's chain (columns 3c,
// 3c+1, 3c+2 of a 16-lane row); alpha = column % 3.
__device__ __forceinline__ float comp_sum(float v, int alpha)
{
    const float s = v + dpp<kRowShl1>(v) + dpp<kRowShl2>(v);  // complete at alpha == 0
    const float s1 = dpp<kRowShr1>(s), s2 = dpp<kRowShr2>(s);
    return alpha == 0 ? s : (alpha == 1 ? s1 : s2);
}

// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (round to nearest
// even), two values per conversion: hi of a pair is one v_cvt_pk_bf16_f32,
// its two halves widen back to FP32 by a shift and a mask.
__device__ __forceinline__ void split2(float a, float b, bf16x2 &h, bf16x2 &l)
{
    h = __builtin_convertvector(f32x2{a, b}, bf16x2);
    const uint32_t u = __builtin_bit_cast(uint32_t, h);
    const float ha = __uint_as_float(u << 16), hb = __uint_as_float(u & 0xffff0000u);
    l = __builtin_convertvector(f32x2{a - ha, b - hb}, bf16x2);
}

// The split of the 8 K-slots of a slab made of two 16-row result tiles.
__device__ __forceinline__ void split_bf16(const f32x4 lo4, const f32x4 hi4, bf16x8 &h, bf16x8 &l)
{
    bf16x2 h0, h1, h2, h3, l0, l1, l2, l3;
    split2(lo4[0], lo4[1], h0, l0);
    split2(lo4[2], lo4[3], h1, l1);
    split2(hi4[0], hi4[1], h2, l2);
    split2(hi4[2], hi4[3], h3, l3);
    h = bf16x8{h0[0], h0[1], h1[0], h1[1], h2[0], h2[1], h3[0], h3[1]};
    l = bf16x8{l0[0], l0[1], l1[0], l1[1], l2[0], l2[1], l3[0], l3[1]};
}

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Bond force of the half-bond rows of one 16-row tile: G+ = g_i + g_{M-i},
// G- = g_i - g_{M-i}, g = u (1/|u| - lin).  No masks are needed: padding rows,
// padding columns and the antisymmetric part of the middle bond are exactly
// zero (u = 0 gives g = 0 thanks to a tiny offset under the rsqrt), and the
// middle bond, which enters G+ twice, has its coupling column halved in the
// table.
__device__ __forceinline__ void bond_forces(const f32x4 aS, const f32x4 aA, int alpha, float lin,
                                            f32x4 &Gp, f32x4 &Gm)
{
    // each component lane adds a third of the offset to its square, so the
    // sum over the chain's three lanes carries it once
    constexpr float kTiny3 = 1e-30f / 3.0f;
    // level by level over the 8 independent sums, so that every lane move
    // reads a value written several instructions earlier (a DPP read right
    // after the write of its source costs wait states)
    float up[4], um[4], vp[4], vm[4], sp[4], sm[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        up[r] = aS[r] + aA[r];
        um[r] = aS[r] - aA[r];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        vp[r] = __builtin_fmaf(up[r], up[r], kTiny3);
        vm[r] = __builtin_fmaf(um[r], um[r], kTiny3);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        sp[r] = vp[r] + dpp<kRowShl1>(vp[r]);
        sm[r] = vm[r] + dpp<kRowShl1>(vm[r]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        sp[r] = sp[r] + dpp<kRowShl2>(vp[r]);  // complete at alpha == 0
        sm[r] = sm[r] + dpp<kRowShl2>(vm[r]);
    }
    // kept at the x lanes only, then spread to the two lanes after each (the
    // two lanes before an x lane hold zero, so the sums are exact)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        sp[r] = alpha == 0 ? sp[r] : 0.0f;
        sm[r] = alpha == 0 ? sm[r] : 0.0f;
    }
    float bp[4], bm[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        bp[r] = sp[r] + dpp<kRowShr1>(sp[r]);
        bm[r] = sm[r] + dpp<kRowShr1>(sm[r]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        bp[r] = bp[r] + dpp<kRowShr2>(sp[r]);
        bm[r] = bm[r] + dpp<kRowShr2>(sm[r]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float tp = __builtin_amdgcn_rsqf(bp[r]) - lin;
        const float gm = um[r] * (__builtin_amdgcn_rsqf(bm[r]) - lin);
        Gp[r] = __builtin_fmaf(up[r], tp, gm);
        Gm[r] = __builtin_fmaf(up[r], tp, -gm);
    }
}

// Copy fragments first .. first + NFRAG - 1 of the transform tables (1 KB
// each) to LDS: the whole workgroup issues buffer loads that write LDS
// directly (16 bytes per lane, no register staging).  All address
// arithmetic is scalar: one buffer descriptor, the byte offsets in SGPRs, the
// lane offset in one VGPR.
template <int NFRAG>
__device__ __forceinline__ void stage(__amdgpu_buffer_rsrc_t rs, int first, f32x4 *dst, int wave,
                                      int lane_bytes)
{
    static_assert(NFRAG % 4 == 0, "fragments are split over 4 wavefronts");
#pragma unroll
    for (int f = 0; f < NFRAG / 4; ++f) {
        const int fr = 4 * f + wave;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (__attribute__((address_space(3))) void *)(dst + fr * 64), 16, lane_bytes,
            (first + fr) * 1024, 0, 0);
    }
}

// The same for a run-time fragment count (one-off loads at launch start).
__device__ __forceinline__ void copy_frags(__amdgpu_buffer_rsrc_t rs, int first, f32x4 *dst, int n,
                                           int wave, int lane_bytes)
{
    for (int fr = wave; fr < n; fr += 4)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (__attribute__((address_space(3))) void *)(dst + fr * 64), 16, lane_bytes,
            (first + fr) * 1024, 0, 0);
}

// s_waitcnt vmcnt(N) alone (gfx9 encoding: vmcnt in bits 3:0 and 15:14,
// expcnt 6:4 and lgkmcnt 11:8 left at their no-wait maximum).  Vector memory
// loads retire in order, so this waits for all but the N most recent.
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt is six bits");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Value of x that the compiler must treat as depending on d: used to keep
// the noise generation of a mode tile after the work it would otherwise be
// hoisted above (which would keep all normals of a step live at once).
__device__ __forceinline__ uint32_t after(uint32_t x, float d)
{
    asm("" : "+v"(x) : "v"(d));
    return x;
}

// Fused stepper.  Workgroup = 4 wavefronts = 4 tiles of 5 chains sharing the
// transform tables in LDS.  In HBM the tables are a linear sequence of
// 2 RT stages of 2 RT fragments (1 KB each, 16 bytes per lane):
//   stage t <  RT : u = chi R, K slab q = t/2, row tiles I of half t%2, [I][f]
//                   BF16 f = (odd hi, odd lo, even hi, even lo) of a K = 32
//                   slab; FP32 f = (odd t=2q, odd 2q+1, even 2q, even 2q+1),
//                   four K = 4 slices each
//   stage RT + J  : coupling rows of mode row tile J, [parity][q][hi, lo]
//                   (FP32: [parity][q][K slice 2q, 2q+1]); the odd rows carry
//                   C_p (Eq. f2) and the middle bond's column halved, the
//                   even rows are S itself.
// Only the first a.jc coupling row tiles are used: beyond them C_p is below
// FP32 resolution of the update (Eq. f4).  RESIDENT: the u = chi R stages and
// the odd coupling rows of tiles J < a.jc are loaded into LDS once per launch
// and the even coupling rows are read from the u = chi R fragments (S is
// symmetric).  Otherwise the RT + a.jc stages of a step stream from L2
// through NB stage buffers with a prefetch distance of NB - 1 stages (L2
// latency is only covered with ~100 KB in flight), and each table byte
// crosses L2 once per workgroup and step.  The odd accumulators start from
// E_p R_p + W_p eta_p (+ shear), so their coupling product is the new
// amplitude; the even ones add sigma^2 C times their product.
constexpr int kTableFrags = 152;  // LDS for transform tables, in 1 KB fragments

// u = chi R and the bond forces of a tile whose tables are resident in LDS
// (split BF16), row tile by row tile: the 24 products of half-bond row tile I
// run over the K slabs in order, so every accumulator sees the products in
// the order of the stage-by-stage form (same bits); the fragments of row
// tile I are read from LDS two K slabs ahead, and the bond forces of row
// tile I - 1 (and the split of a finished pair) are computed between its
// products, where the VALU work issues beside the matrix cores.
template <int RT>
__device__ __forceinline__ void chi_forces_resident(const f32x4 *xb, int lane, const f32x4 (&Ro)[RT],
                                                    const f32x4 (&Re)[RT], int alpha, float lin,
                                                    f32x4 (&Gp)[RT], f32x4 (&Gm)[RT],
                                                    bf16x8 (&gph)[RT / 2], bf16x8 (&gpl)[RT / 2],
                                                    bf16x8 (&gmh)[RT / 2], bf16x8 (&gml)[RT / 2])
{
    constexpr int KS = RT / 2, HALF = RT / 2, SF = 2 * RT;
    bf16x8 boh[KS], bol[KS], beh[KS], bel[KS];
#pragma unroll
    for (int q = 0; q < KS; ++q) {
        split_bf16(Ro[2 * q], Ro[2 * q + 1], boh[q], bol[q]);
        split_bf16(Re[2 * q], Re[2 * q + 1], beh[q], bel[q]);
    }
    // fragment f (odd hi, odd lo, even hi, even lo) of row tile I in K slab q:
    // stage 2q + I / HALF, position I % HALF of that stage.  Slab u = I KS + q
    // of the sequence is read D slabs ahead into ring buffer u % (D + 1).
    constexpr int D = 2, NU = RT * KS;
    bf16x8 x[D + 1][4];
    auto load = [&](int u) {
        const int I = u / KS, q = u % KS;
#pragma unroll
        for (int f = 0; f < 4; ++f)
            x[u % (D + 1)][f] = __builtin_bit_cast(
                bf16x8, xb[((2 * q + I / HALF) * SF + (I % HALF) * 4 + f) * 64 + lane]);
    };
#pragma unroll
    for (int u = 0; u < D; ++u) load(u);
    f32x4 aS[2], aA[2];
#pragma unroll
    for (int I = 0; I <= RT; ++I) {
        if (I < RT) {
            f32x4 s = f32x4{0.f, 0.f, 0.f, 0.f}, t = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < KS; ++q) {
                const int u = I * KS + q;
                if (u + D < NU) load(u + D);
                const bf16x8 *xf = x[u % (D + 1)];
                s = mfma_bf16(xf[0], boh[q], s);
                t = mfma_bf16(xf[2], beh[q], t);
                s = mfma_bf16(xf[0], bol[q], s);
                t = mfma_bf16(xf[2], bel[q], t);
                s = mfma_bf16(xf[1], boh[q], s);
                t = mfma_bf16(xf[3], beh[q], t);
            }
            aS[I & 1] = s;
            aA[I & 1] = t;
        }
        if (I >= 1) {
            const int P = I - 1;
            bond_forces(aS[P & 1], aA[P & 1], alpha, lin, Gp[P], Gm[P]);
            if (P & 1) {
                split_bf16(Gp[P - 1], Gp[P], gph[P / 2], gpl[P / 2]);
                split_bf16(Gm[P - 1], Gm[P], gmh[P / 2], gml[P / 2]);
            }
        }
        // one scheduling region per row tile: the compiler interleaves the
        // products, the reads and the forces inside it (measured faster than
        // a prescribed interleave by group barriers)
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int RT, bool BF16, bool RESIDENT>
__device__ __forceinline__ void fused_tiles(const BucketArgs &a, const LaunchArgs &la, int tile0,
                                            int64_t step0, f32x4 *cf, f32x4 *xb)
{
    constexpr int KS = RT / 2;
    constexpr int SF = 2 * RT;    // fragments per stage
    constexpr int HALF = RT / 2;  // row tiles per half slab
    constexpr int G1 = RT * SF;   // fragments of u = chi R
    constexpr int NB = kTableFrags / SF;
    constexpr int DIST = RESIDENT ? 0 : NB - 1;  // prefetch distance when streaming
    static_assert(!RESIDENT || G1 + RT <= kTableFrags, "resident tables exceed LDS");
    static_assert(RESIDENT || (NB >= 3 && (DIST - 1) * (SF / 4) < 64), "stream buffers");
    const int NS = RT + a.jc;  // stages per step when streaming
    // cf: [kind][J][g], four slots r each; xb: table fragments
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    {
        const f32x4 *c4 = reinterpret_cast<const f32x4 *>(a.coef);
        for (int i = threadIdx.x; i < kKinds * RT * 4; i += blockDim.x) cf[i] = c4[i];
    }

    const int tile = tile0 + wave;
    // idle waves still stage (and, when streaming, synchronise)
    const bool has_tile = wave < a.tpw && tile < a.ntiles;
    const int col = lane & 15, g = lane >> 4;
    const int cl = col / 3, alpha = col - 3 * cl;
    const int nvalid = has_tile ? min(kChainsPerTile, a.n - kChainsPerTile * tile) : 0;
    const bool valid = (col < 15) && (cl < nvalid);
    const uint32_t chain = valid ? (uint32_t)a.ids[kChainsPerTile * tile + cl] : 0u;
    const __amdgpu_buffer_rsrc_t xrs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(a.X), 0, a.x_bytes, 0x00020000);
    const int lane_bytes = lane * 16;

    f32x4 Ro[RT], Re[RT];
    const f32x4 *Rt = reinterpret_cast<const f32x4 *>(a.R) + (size_t)tile * 2 * RT * 64;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        Ro[t] = has_tile ? Rt[(0 * RT + t) * 64 + lane] : f32x4{0.f, 0.f, 0.f, 0.f};
        Re[t] = has_tile ? Rt[(1 * RT + t) * 64 + lane] : f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const bool com_lane = valid && g == 0;
    const float xlane = alpha == 0 ? 1.0f : 0.0f;  // lanes holding x components
    double r0 = com_lane ? a.R0[(size_t)tile * 16 + col] : 0.0;

    // streaming: stage t of any step lives in buffer (b0 + t) % NB; b0
    // advances by NS per step
    int b0 = 0;
    if (la.nonlinear) {
        if constexpr (RESIDENT) {
            copy_frags(xrs, 0, xb, G1, wave, lane_bytes);
            for (int J = 0; J < a.jc; ++J)  // odd halves of the coupling stages
                copy_frags(xrs, G1 + J * SF, xb + (G1 + J * RT) * 64, RT, wave, lane_bytes);
            wait_vmcnt<0>();
        } else {
            // the first DIST stages (wrapping into the next steps when a step
            // has fewer stages than the prefetch distance)
            int issued = 0;
            for (int t = 0; t < DIST; ++t)
                if (t / NS < la.n_steps) {
                    stage<SF>(xrs, (t % NS) * SF, xb + (t % NB) * SF * 64, wave, lane_bytes);
                    ++issued;
                }
            if (issued == DIST)
                wait_vmcnt<(DIST - 1) * (SF / 4)>();  // stage 0 landed (own loads)
            else
                wait_vmcnt<0>();
        }
    }
    __syncthreads();
    if constexpr (RESIDENT) {
        if (!has_tile) return;  // no barrier follows
    }

    // Streaming: issue the copy of stage t + DIST (of this step or, wrapping,
    // of the next) and, after the compute of stage t, wait until stage t + 1
    // has landed (loads retire in order).  The tests below read ns, which
    // the step loop makes opaque at every step: otherwise the compiler
    // hoists one test per stage out of the loop, the longest shapes spill
    // them, and each reload from scratch (a vector memory load, counted with
    // the copies in flight) waits for all the prefetched stages.
    int ns = NS;
    auto prefetch = [&](int t, int s) {
        if constexpr (!RESIDENT) {
            // stage t + DIST counted from the start of this step, as (step
            // ahead, stage of that step); nothing beyond the last step.
            // DIST <= RT <= NS, so it is at most one step ahead (a compare,
            // not a scalar division by the run-time NS).
            static_assert(RESIDENT || DIST <= RT, "prefetch reaches two steps ahead");
            const int tn = t + DIST;
            const bool ahead = tn >= ns;
            if (s + (ahead ? 1 : 0) < la.n_steps)
                stage<SF>(xrs, (ahead ? tn - ns : tn) * SF, xb + ((b0 + tn) % NB) * SF * 64, wave,
                          lane_bytes);
        }
    };
    // outstanding loads of this wave after stage t: stages t+1 .. t+DIST that
    // were issued; all but stage t+1 may stay in flight
    auto finish = [&](int t, int s) {
        if constexpr (!RESIDENT) {
            // last stage issued so far, counted from the start of this step
            const int last = min(t + DIST, (la.n_steps - s) * ns - 1);
            const int ahead = last - (t + 1);  // issued beyond t+1
            if (ahead >= DIST - 1)
                wait_vmcnt<(DIST - 1) * (SF / 4)>();
            else
                wait_vmcnt<0>();
            // A bare barrier: __syncthreads() would add a workgroup release
            // fence, i.e. a wait for ALL outstanding loads (vmcnt(0)), which
            // drains the prefetch pipeline at every stage.  The explicit wait
            // above has made this wave's copies of stage t+1 land in LDS; the
            // barrier makes that true for every wave.  The buffer the next
            // prefetch overwrites held stage t-1, whose LDS reads every wave
            // consumed (its products need them) before reaching this point.
            // The signal fences keep the compiler from moving LDS accesses
            // across the barrier; they emit no instruction.
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_s_barrier();
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
    };
    auto stage_at = [&](int t) -> const f32x4 * {
        if constexpr (RESIDENT)
            return xb + t * SF * 64;
        else
            return xb + ((b0 + t) % NB) * SF * 64;
    };
    for (int s = 0; s < la.n_steps; ++s) {
        const int64_t k = step0 + s;
        if constexpr (!RESIDENT) {
            ns = NS;
            asm volatile("" : "+s"(ns));
        }
        f32x4 Gp[RT], Gm[RT];
        [[maybe_unused]] bf16x8 gph[KS], gpl[KS], gmh[KS], gml[KS];
        if constexpr (RESIDENT && BF16) {
            if (la.nonlinear)
                chi_forces_resident<RT>(xb, lane, Ro, Re, alpha, a.lin, Gp, Gm, gph, gpl, gmh, gml);
        } else if (la.nonlinear) {
            // ---- u = chi R: half-bond rows I, K over mode slabs q
            f32x4 aS[RT], aA[RT];
#pragma unroll
            for (int I = 0; I < RT; ++I) {
                aS[I] = f32x4{0.f, 0.f, 0.f, 0.f};
                aA[I] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
            [[maybe_unused]] bf16x8 boh, bol, beh, bel;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int q = t / 2, h = t % 2;
                prefetch(t, s);
                const f32x4 *xs = stage_at(t);
                if constexpr (BF16) {
                    if (h == 0) {
                        split_bf16(Ro[2 * q], Ro[2 * q + 1], boh, bol);
                        split_bf16(Re[2 * q], Re[2 * q + 1], beh, bel);
                    }
                    // the fragments of FB row tiles first, then each product over
                    // them: FB independent accumulator pairs between two MFMAs
                    // into the same accumulator (FB = HALF up to RT = 12; the
                    // longest shapes take 4 at a time, whose 64 registers instead
                    // of 4 HALF keep them free of scratch spills -- a spill
                    // reload waits for every copy in flight, as they share the
                    // vector memory counter)
                    constexpr int FB = RT >= 14 ? 4 : HALF;
#pragma unroll
                    for (int i0 = 0; i0 < HALF; i0 += FB) {
                        bf16x8 xoh[FB], xol[FB], xeh[FB], xel[FB];
#pragma unroll
                        for (int ii = 0; ii < FB; ++ii) {
                            const f32x4 *fr = xs + ((i0 + ii) * 4) * 64 + lane;
                            xoh[ii] = __builtin_bit_cast(bf16x8, fr[0]);
                            xol[ii] = __builtin_bit_cast(bf16x8, fr[64]);
                            xeh[ii] = __builtin_bit_cast(bf16x8, fr[128]);
                            xel[ii] = __builtin_bit_cast(bf16x8, fr[192]);
                        }
                        const int I0 = h * HALF + i0;
#pragma unroll
                        for (int ii = 0; ii < FB; ++ii) {
                            aS[I0 + ii] = mfma_bf16(xoh[ii], boh, aS[I0 + ii]);
                            aA[I0 + ii] = mfma_bf16(xeh[ii], beh, aA[I0 + ii]);
                        }
#pragma unroll
                        for (int ii = 0; ii < FB; ++ii) {
                            aS[I0 + ii] = mfma_bf16(xoh[ii], bol, aS[I0 + ii]);
                            aA[I0 + ii] = mfma_bf16(xeh[ii], bel, aA[I0 + ii]);
                        }
#pragma unroll
                        for (int ii = 0; ii < FB; ++ii) {
                            aS[I0 + ii] = mfma_bf16(xol[ii], boh, aS[I0 + ii]);
                            aA[I0 + ii] = mfma_bf16(xel[ii], beh, aA[I0 + ii]);
                        }
                    }
                } else {
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh) {
                        // fragments first, then K slice r over the HALF row tiles
                        f32x4 xo[HALF], xe[HALF];
#pragma unroll
                        for (int ii = 0; ii < HALF; ++ii) {
                            xo[ii] = xs[(ii * 4 + hh) * 64 + lane];
                            xe[ii] = xs[(ii * 4 + 2 + hh) * 64 + lane];
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int ii = 0; ii < HALF; ++ii) {
                                const int I = h * HALF + ii;
                                aS[I] = mfma_f32(xo[ii][r], Ro[2 * q + hh][r], aS[I]);
                                aA[I] = mfma_f32(xe[ii][r], Re[2 * q + hh][r], aA[I]);
                            }
                    }
                }
                finish(t, s);
            }
            // ---- bond forces (and their BF16 split for the coupling product;
            // the longest shapes go slab by slab, so the FP32 forces and the
            // accumulators die early, the others keep the order that
            // schedules best for them: all forces, then all splits)
            if constexpr (RT >= 14) {
#pragma unroll
                for (int q = 0; q < KS; ++q) {
                    bond_forces(aS[2 * q], aA[2 * q], alpha, a.lin, Gp[2 * q], Gm[2 * q]);
                    bond_forces(aS[2 * q + 1], aA[2 * q + 1], alpha, a.lin, Gp[2 * q + 1],
                                Gm[2 * q + 1]);
                    if constexpr (BF16) {
                        split_bf16(Gp[2 * q], Gp[2 * q + 1], gph[q], gpl[q]);
                        split_bf16(Gm[2 * q], Gm[2 * q + 1], gmh[q], gml[q]);
                    }
                }
            } else {
#pragma unroll
                for (int I = 0; I < RT; ++I)
                    bond_forces(aS[I], aA[I], alpha, a.lin, Gp[I], Gm[I]);
                if constexpr (BF16) {
#pragma unroll
                    for (int q = 0; q < KS; ++q) {
                        split_bf16(Gp[2 * q], Gp[2 * q + 1], gph[q], gpl[q]);
                        split_bf16(Gm[2 * q], Gm[2 * q + 1], gmh[q], gml[q]);
                    }
                }
            }
        }
        // ---- per mode tile J: E R + W eta (+ shear) and the coupling, with
        // every multiply-add written as an explicit fma, so that the
        // rounding does not depend on which products the compiler fuses in
        // each tile shape (all shapes give the same bits).  Lane
        // holds half-mode slots j = 16J + 4g + r: odd p = 2j + 1 in Ro[J][r],
        // even p = 2j + 2 (scaled) in Re[J][r].  Normal p of the step is
        // element p % 4 of Philox block p / 4, so a lane group draws normals
        // 32J + 8g .. + 7 and takes normal 32J + 8g + 8 (its even slot r = 3)
        // from the next lane group; lane group 3 gets it one tile later.
        float wcarry = 0.0f;  // W of the even slot r = 3 of the previous tile
#pragma unroll
        for (int J = 0; J < RT; ++J) {
            const int t = RT + J;
            const bool couple = la.nonlinear && J < a.jc;
            if (couple) prefetch(t, s);
            // coefficients first, so their LDS reads are in flight during the
            // noise, and the cross-lane read of normal 0 between the two blocks
            const f32x4 Eo = cf[(kEo * RT + J) * 4 + g], Wo = cf[(kWo * RT + J) * 4 + g];
            const f32x4 Ee = cf[(kEe * RT + J) * 4 + g], We = cf[(kWe * RT + J) * 4 + g];
            const uint32_t ch =
                after(chain, J ? Ro[J - 1][3] : (la.nonlinear ? Gm[0][0] : Re[0][0]));
            float z[8];
            scaled_normals4_f32(noise_bits(la.seed, (uint32_t)(8 * J + 2 * g), ch, k, (uint32_t)alpha,
                                    kTagMode),
                         z);
            const float zn = __shfl(z[0], (lane + 16) & 63, 64);
            scaled_normals4_f32(noise_bits(la.seed, (uint32_t)(8 * J + 2 * g + 1), ch, k,
                                    (uint32_t)alpha, kTagMode),
                         z + 4);
            if (J > 0) Re[J - 1][3] = __builtin_fmaf(g == 3 ? wcarry : 0.0f, zn, Re[J - 1][3]);
            f32x4 ao, ae;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float ze = r < 3 ? z[2 * r + 2] : (g < 3 ? zn : 0.0f);
                ao[r] = __builtin_fmaf(Eo[r], Ro[J][r], Wo[r] * z[2 * r + 1]);
                ae[r] = __builtin_fmaf(Ee[r], Re[J][r], We[r] * ze);
            }
            wcarry = We[3];
            if (a.gdt != 0.0) {
                const f32x4 Go = cf[(kGo * RT + J) * 4 + g], Ge = cf[(kGe * RT + J) * 4 + g];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // R^y of the same chain, for the x lanes only.  The lane
                    // move runs with every lane active (a DPP read from a lane
                    // masked off by a branch returns 0), then is masked.
                    ao[r] = __builtin_fmaf(Go[r], xlane * dpp<kRowShl1>(Ro[J][r]), ao[r]);
                    ae[r] = __builtin_fmaf(Ge[r], xlane * dpp<kRowShl1>(Re[J][r]), ae[r]);
                }
            }
            if (J == 0) {
                // centre of mass (p = 0, normal 0 of the g = 0 lanes): free
                // random walk in FP64, shear drift from R_0^y
                const double r0y = __shfl(r0, (lane + 1) & 63, 64);
                double nr0 = __builtin_fma(a.W0, (double)z[0], r0);
                if (alpha == 0) nr0 = __builtin_fma(a.gdt, r0y, nr0);
                r0 = com_lane ? nr0 : 0.0;
            }
            if (couple) {
                // odd rows at xo2 + 2q (+1 for lo / the second K slice); even
                // rows at xe2 + ES q (+1)
                const f32x4 *xo2, *xe2;
                constexpr int ES = RESIDENT ? 2 * SF : 2;
                if constexpr (RESIDENT) {
                    xo2 = xb + (G1 + J * RT) * 64 + lane;
                    xe2 = xb + ((J / HALF) * SF + (J % HALF) * 4 + 2) * 64 + lane;
                } else {
                    xo2 = stage_at(t) + lane;
                    xe2 = xo2 + RT * 64;
                }
                f32x4 ce = f32x4{0.f, 0.f, 0.f, 0.f};
                if constexpr (BF16) {
                    // alternate slabs go to a second accumulator pair, so two
                    // MFMA chains are in flight
                    f32x4 ao2 = f32x4{0.f, 0.f, 0.f, 0.f}, ce2 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int q = 0; q < KS; ++q) {
                        const bf16x8 xoh = __builtin_bit_cast(bf16x8, xo2[(2 * q) * 64]);
                        const bf16x8 xol = __builtin_bit_cast(bf16x8, xo2[(2 * q + 1) * 64]);
                        const bf16x8 xeh = __builtin_bit_cast(bf16x8, xe2[(ES * q) * 64]);
                        const bf16x8 xel = __builtin_bit_cast(bf16x8, xe2[(ES * q + 1) * 64]);
                        f32x4 &A = (q & 1) ? ao2 : ao;
                        f32x4 &C = (q & 1) ? ce2 : ce;
                        A = mfma_bf16(xoh, gph[q], A);
                        C = mfma_bf16(xeh, gmh[q], C);
                        A = mfma_bf16(xoh, gpl[q], A);
                        C = mfma_bf16(xeh, gml[q], C);
                        A = mfma_bf16(xol, gph[q], A);
                        C = mfma_bf16(xel, gmh[q], C);
                    }
                    ao += ao2;
                    ce += ce2;
                } else {
#pragma unroll
                    for (int q = 0; q < KS; ++q) {
#pragma unroll
                        for (int hh = 0; hh < 2; ++hh) {
                            const f32x4 xo = xo2[(2 * q + hh) * 64], xe = xe2[(ES * q + hh) * 64];
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                ao = mfma_f32(xo[r], Gp[2 * q + hh][r], ao);
                                ce = mfma_f32(xe[r], Gm[2 * q + hh][r], ce);
                            }
                        }
                    }
                }
                const f32x4 Ce = cf[(kCe * RT + J) * 4 + g];
#pragma unroll
                for (int r = 0; r < 4; ++r) ae[r] = __builtin_fmaf(Ce[r], ce[r], ae[r]);
                finish(t, s);
            }
            Ro[J] = ao;
            Re[J] = ae;
        }
        if constexpr (!RESIDENT) b0 = (b0 + NS) % NB;
    }
    if (!has_tile) return;
    f32x4 *Rw = reinterpret_cast<f32x4 *>(a.R) + (size_t)tile * 2 * RT * 64;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        Rw[(0 * RT + t) * 64 + lane] = Ro[t];
        Rw[(1 * RT + t) * 64 + lane] = Re[t];
    }
    if (com_lane) a.R0[(size_t)tile * 16 + col] = r0;
}

// ---- Split tile: one tile of 5 chains per workgroup, its work divided
// among P = 4 (or 8) wavefronts, for launches with fewer tiles than the GPU
// has SIMDs (with one wavefront per tile, 1024 chains make 205 wavefronts).
// Wavefront w owns the mode tiles J = w, w + P, ... (their amplitudes, noise
// and update) and the half-bond row tiles I = w, w + P, ... (their rows of
// u = chi R and their bond forces); the round-robin spreads the few coupled
// mode tiles J < jc over the wavefronts.  With 8 wavefronts (split-BF16, RT
// = 8 and 16, a kernel of its own with at most 256 registers per lane) each
// SIMD runs two of the tile's wavefronts, whose waits and matrix products
// overlap the other's vector work.  Each step they exchange through LDS
// what their products take from the others:
//   Rb  the amplitudes (split BF16 or FP32), the B operand of u = chi R;
//   Gb  the bond forces G+ and G- (split or FP32), the B operand of the
//       coupling product;
//   cz  normal 0 of lane group 0 of each mode tile, which lane group 3 of the
//       previous tile takes for its even slot r = 3.
// Three barriers a step: forces written (B), normals written (C), amplitudes
// written (A).  Each accumulator sees the same products in the same order as
// in fused_tiles, and every update the same operations, so the states are
// bit-identical to the other tile shapes.  The table fragments a wavefront
// reads (its own bond rows, its own coupling rows) are read by no other
// wavefront, so they go from L2 straight to registers: up to RT = 12 the
// u = chi R fragments of the own rows stay in registers for the whole
// launch, and at RT = 16 a ring keeps DU = 4 K slabs of them in flight (the
// first ones of the next step issued after the update, when the coupling
// registers are free); a mode tile's first DC K slabs of coupling rows are
// loaded before its noise is drawn.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// s_waitcnt lgkmcnt(0) alone: this wavefront's LDS accesses have completed.
__device__ __forceinline__ void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Workgroup barrier for the LDS exchanges that leaves the table loads in
// flight (__syncthreads() would also wait for every outstanding vector
// memory load).  Each wavefront's LDS accesses complete before it arrives;
// the signal fences keep the compiler from moving LDS accesses across.
__device__ __forceinline__ void lds_barrier()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    wait_lgkm0();
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// hi/lo BF16 of one 16-row result tile: its 4 K slots of a K = 32 slab (the
// first or second half of what split_bf16 makes of two tiles).
__device__ __forceinline__ void split_half(const f32x4 v, bf16x4 &h, bf16x4 &l)
{
    bf16x2 h0, h1, l0, l1;
    split2(v[0], v[1], h0, l0);
    split2(v[2], v[3], h1, l1);
    h = bf16x4{h0[0], h0[1], h1[0], h1[1]};
    l = bf16x4{l0[0], l0[1], l1[0], l1[1]};
}

// BF16 exchange buffers: [K slab q][kind k][lane] bf16x8; 16-row tile T
// fills half T % 2 of slab T / 2.  (In both precisions the four 16-byte
// B operands of K slab q sit at [4 q + k][lane].)
__device__ __forceinline__ void put_half(f32x4 *buf, int T, int k, int lane, bf16x4 v)
{
    reinterpret_cast<bf16x4 *>(buf + ((T >> 1) * 4 + k) * 64 + lane)[T & 1] = v;
}
__device__ __forceinline__ void slab4(const f32x4 *buf, int q, f32x4 *dst, int lane)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[k] = buf[(4 * q + k) * 64 + lane];
}

template <int RT, bool BF16, int P = 4>  // P: wavefronts of the workgroup
__device__ __forceinline__ void split_tile(const BucketArgs &a, const LaunchArgs &la, int tile,
                                           int64_t step0, f32x4 *cf, f32x4 *xb)
{
    constexpr int NJ = RT / P;    // mode tiles and row tiles of each
    constexpr int KS = RT / 2;    // K slabs
    constexpr int SF = 2 * RT;    // fragments per table stage
    constexpr int FU = 4 * NJ;    // u = chi R fragments of one K slab for the own rows
    // K slabs in registers: all u = chi R ones up to RT = 12 (loaded once
    // per launch), 4 at RT = 16; the coupling ring holds the whole tile up
    // to RT = 8, else 2 (RT = 12, beside the resident u = chi R fragments)
    // or 4 (RT = 16, whose u = chi R ring is free during the update)
    constexpr int DU = RT <= 12 ? KS : 4;
    constexpr int DC = RT <= 8 ? KS : (RT == 12 ? 2 : 4);
    static_assert(RT % P == 0 && KS % DU == 0, "split tile shape");
    static_assert(4 * RT * 64 + 4 * RT <= kTableFrags * 64, "split tile exchange buffers");
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    {
        const f32x4 *c4 = reinterpret_cast<const f32x4 *>(a.coef);
        for (int i = threadIdx.x; i < kKinds * RT * 4; i += blockDim.x) cf[i] = c4[i];
    }
    // Rb and Gb: 2 RT fragments each ([q][k] BF16, [T][parity] FP32); cz: [J][16]
    f32x4 *Rb = xb, *Gb = xb + 2 * RT * 64;
    float *cz = reinterpret_cast<float *>(xb + 4 * RT * 64);

    const int col = lane & 15, g = lane >> 4;
    const int cl = col / 3, alpha = col - 3 * cl;
    const int nvalid = min(kChainsPerTile, a.n - kChainsPerTile * tile);
    const bool valid = (col < 15) && (cl < nvalid);
    const uint32_t chain = valid ? (uint32_t)a.ids[kChainsPerTile * tile + cl] : 0u;
    const float xlane = alpha == 0 ? 1.0f : 0.0f;
    // table fragment F (1 KB): a buffer load at a scalar offset, so no
    // per-lane 64-bit addresses are kept and only vmcnt counts it
    const __amdgpu_buffer_rsrc_t xrs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(a.X), 0, a.x_bytes, 0x00020000);
    const int lane_bytes = lane * 16;
    auto frag = [&](int F) {
        return __builtin_bit_cast(f32x4,
                                  __builtin_amdgcn_raw_buffer_load_b128(xrs, lane_bytes, F * 1024, 0));
    };

    f32x4 Ro[NJ], Re[NJ];
    const f32x4 *Rt = reinterpret_cast<const f32x4 *>(a.R) + (size_t)tile * 2 * RT * 64;
#pragma unroll
    for (int ii = 0; ii < NJ; ++ii) {
        const int J = wave + P * ii;
        Ro[ii] = Rt[J * 64 + lane];
        Re[ii] = Rt[(RT + J) * 64 + lane];
    }
    const bool com_lane = valid && g == 0 && wave == 0;
    double r0 = com_lane ? a.R0[(size_t)tile * 16 + col] : 0.0;

    auto put_state = [&](int ii) {
        const int J = wave + P * ii;
        if constexpr (BF16) {
            bf16x4 h, l;
            split_half(Ro[ii], h, l);
            put_half(Rb, J, 0, lane, h);
            put_half(Rb, J, 1, lane, l);
            split_half(Re[ii], h, l);
            put_half(Rb, J, 2, lane, h);
            put_half(Rb, J, 3, lane, l);
        } else {
            Rb[(2 * J) * 64 + lane] = Ro[ii];
            Rb[(2 * J + 1) * 64 + lane] = Re[ii];
        }
    };
    // u = chi R fragments of K slab q for the own rows, [row tile][f]
    f32x4 xu[DU][FU];
    auto load_u = [&](int q, f32x4 *dst) {
#pragma unroll
        for (int ii = 0; ii < NJ; ++ii)
#pragma unroll
            for (int f = 0; f < 4; ++f)
                dst[4 * ii + f] = frag((q * RT + wave + P * ii) * 4 + f);
    };
    // Split BF16 runs u = chi R own row tile by own row tile (see the step
    // loop); at RT = 16 its fragments stream through a ring of RL entries
    // (own row tile ii, K slab q) in that order instead of the slab ring.
    constexpr bool ROWS = BF16;
    constexpr bool RING = ROWS && DU < KS;
    constexpr int RL = 4;
    [[maybe_unused]] f32x4 xr[RL][4];
    auto load_r = [&](int u) {
        const int ii = u / KS, q = u % KS;
#pragma unroll
        for (int f = 0; f < 4; ++f) xr[u % RL][f] = frag((q * RT + wave + P * ii) * 4 + f);
    };
    if (la.nonlinear) {
#pragma unroll
        for (int ii = 0; ii < NJ; ++ii) put_state(ii);
    }
    __syncthreads();  // coefficients and amplitudes in LDS
    if (la.nonlinear) {
        if constexpr (RING) {
#pragma unroll
            for (int u = 0; u < RL; ++u) load_r(u);
        } else {
#pragma unroll
            for (int q = 0; q < DU; ++q) load_u(q, xu[q]);
        }
    }

    for (int s = 0; s < la.n_steps; ++s) {
        const int64_t k = step0 + s;
        float gdep = 0.0f;  // last force written: keeps the noise below the forces
        if (ROWS && la.nonlinear) {
            // ---- u = chi R own row tile by own row tile: the 24 products of
            // row tile ii over the K slabs in order (each accumulator sees the
            // products of the slab-by-slab form in the same order: same bits),
            // the B operands read from LDS one slab ahead, and the bond forces
            // of row tile ii - 1 (split and written to LDS) computed between
            // the products, where the VALU work issues beside the matrix cores
            constexpr int NU = NJ * KS;
            f32x4 pS[2], pA[2];
            f32x4 bn[4];
            slab4(Rb, 0, bn, lane);
#pragma unroll
            for (int ii = 0; ii <= NJ; ++ii) {
                if (ii < NJ) {
                    f32x4 sacc = f32x4{0.f, 0.f, 0.f, 0.f}, tacc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int q = 0; q < KS; ++q) {
                        const int u = ii * KS + q;
                        f32x4 bc[4];
#pragma unroll
                        for (int k2 = 0; k2 < 4; ++k2) bc[k2] = bn[k2];
                        if (u + 1 < NU) slab4(Rb, (q + 1) % KS, bn, lane);
                        f32x4 xf[4];
#pragma unroll
                        for (int f = 0; f < 4; ++f) {
                            if constexpr (RING)
                                xf[f] = xr[u % RL][f];
                            else
                                xf[f] = xu[q][4 * ii + f];
                        }
                        if constexpr (RING) {
                            if (u + RL < NU) load_r(u + RL);
                        }
                        const bf16x8 boh = __builtin_bit_cast(bf16x8, bc[0]);
                        const bf16x8 bol = __builtin_bit_cast(bf16x8, bc[1]);
                        const bf16x8 beh = __builtin_bit_cast(bf16x8, bc[2]);
                        const bf16x8 bel = __builtin_bit_cast(bf16x8, bc[3]);
                        sacc = mfma_bf16(__builtin_bit_cast(bf16x8, xf[0]), boh, sacc);
                        tacc = mfma_bf16(__builtin_bit_cast(bf16x8, xf[2]), beh, tacc);
                        sacc = mfma_bf16(__builtin_bit_cast(bf16x8, xf[0]), bol, sacc);
                        tacc = mfma_bf16(__builtin_bit_cast(bf16x8, xf[2]), bel, tacc);
                        sacc = mfma_bf16(__builtin_bit_cast(bf16x8, xf[1]), boh, sacc);
                        tacc = mfma_bf16(__builtin_bit_cast(bf16x8, xf[3]), beh, tacc);
                        // streamed fragments: each slab its own region, so the
                        // ring's loads are not hoisted ahead of their slot
                        if constexpr (RING) __builtin_amdgcn_sched_barrier(0);
                    }
                    pS[ii & 1] = sacc;
                    pA[ii & 1] = tacc;
                }
                if (ii >= 1) {
                    const int pi = ii - 1, I = wave + P * pi;
                    f32x4 Gp, Gm;
                    bond_forces(pS[pi & 1], pA[pi & 1], alpha, a.lin, Gp, Gm);
                    bf16x4 h, l;
                    split_half(Gp, h, l);
                    put_half(Gb, I, 0, lane, h);
                    put_half(Gb, I, 1, lane, l);
                    split_half(Gm, h, l);
                    put_half(Gb, I, 2, lane, h);
                    put_half(Gb, I, 3, lane, l);
                    gdep = Gm[0];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            lds_barrier();  // B
        } else if (la.nonlinear) {
            // ---- u = chi R for the own half-bond row tiles
            f32x4 aS[NJ], aA[NJ];
#pragma unroll
            for (int ii = 0; ii < NJ; ++ii) {
                aS[ii] = f32x4{0.f, 0.f, 0.f, 0.f};
                aA[ii] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
            // B operands of slab q + 1 are read from LDS during slab q
            f32x4 bn[4];
            slab4(Rb, 0, bn, lane);
#pragma unroll
            for (int q = 0; q < KS; ++q) {
                const f32x4 *xs = xu[q % DU];
                f32x4 bc[4];
#pragma unroll
                for (int k2 = 0; k2 < 4; ++k2) bc[k2] = bn[k2];
                if (q + 1 < KS) slab4(Rb, q + 1, bn, lane);
                if constexpr (BF16) {
                    const bf16x8 boh = __builtin_bit_cast(bf16x8, bc[0]);
                    const bf16x8 bol = __builtin_bit_cast(bf16x8, bc[1]);
                    const bf16x8 beh = __builtin_bit_cast(bf16x8, bc[2]);
                    const bf16x8 bel = __builtin_bit_cast(bf16x8, bc[3]);
#pragma unroll
                    for (int ii = 0; ii < NJ; ++ii) {
                        aS[ii] = mfma_bf16(__builtin_bit_cast(bf16x8, xs[4 * ii]), boh, aS[ii]);
                        aA[ii] = mfma_bf16(__builtin_bit_cast(bf16x8, xs[4 * ii + 2]), beh, aA[ii]);
                    }
#pragma unroll
                    for (int ii = 0; ii < NJ; ++ii) {
                        aS[ii] = mfma_bf16(__builtin_bit_cast(bf16x8, xs[4 * ii]), bol, aS[ii]);
                        aA[ii] = mfma_bf16(__builtin_bit_cast(bf16x8, xs[4 * ii + 2]), bel, aA[ii]);
                    }
#pragma unroll
                    for (int ii = 0; ii < NJ; ++ii) {
                        aS[ii] = mfma_bf16(__builtin_bit_cast(bf16x8, xs[4 * ii + 1]), boh, aS[ii]);
                        aA[ii] = mfma_bf16(__builtin_bit_cast(bf16x8, xs[4 * ii + 3]), beh, aA[ii]);
                    }
                } else {
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh) {
                        const f32x4 bo = bc[2 * hh], be = bc[2 * hh + 1];
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int ii = 0; ii < NJ; ++ii) {
                                aS[ii] = mfma_f32(xs[4 * ii + hh][r], bo[r], aS[ii]);
                                aA[ii] = mfma_f32(xs[4 * ii + 2 + hh][r], be[r], aA[ii]);
                            }
                    }
                }
                if constexpr (DU < KS) {
                    // the next loads stay in this slab: the scheduler would
                    // otherwise hoist them all to the top, past the registers
                    if (q + DU < KS) load_u(q + DU, xu[q % DU]);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // ---- bond forces of the own rows, to LDS
#pragma unroll
            for (int ii = 0; ii < NJ; ++ii) {
                const int I = wave + P * ii;
                f32x4 Gp, Gm;
                bond_forces(aS[ii], aA[ii], alpha, a.lin, Gp, Gm);
                if constexpr (BF16) {
                    bf16x4 h, l;
                    split_half(Gp, h, l);
                    put_half(Gb, I, 0, lane, h);
                    put_half(Gb, I, 1, lane, l);
                    split_half(Gm, h, l);
                    put_half(Gb, I, 2, lane, h);
                    put_half(Gb, I, 3, lane, l);
                } else {
                    Gb[(2 * I) * 64 + lane] = Gp;
                    Gb[(2 * I + 1) * 64 + lane] = Gm;
                }
                gdep = Gm[0];
            }
            lds_barrier();  // B
        }
        // ---- own mode tiles: E R + W eta (+ shear) and the coupling
#pragma unroll
        for (int ii = 0; ii < NJ; ++ii) {
            const int J = wave + P * ii;
            const bool couple = la.nonlinear && J < a.jc;
            // coupling rows of tile J, K slab q in xc[q % DC]: [odd hi, odd lo,
            // even hi, even lo] (FP32: [odd 2q, 2q+1, even 2q, 2q+1]); the
            // first DC slabs are in flight during the noise
            f32x4 xc[DC][4];
            auto load_c = [&](int q) {
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    xc[q % DC][f] = frag((RT + J) * SF + (f >> 1) * RT + 2 * q + (f & 1));
            };
            if (couple) {
#pragma unroll
                for (int q = 0; q < DC; ++q) load_c(q);
            }
            // coefficients first and the cross-lane read between the two
            // blocks, as in the one-wavefront tiles
            const f32x4 Eo = cf[(kEo * RT + J) * 4 + g], Wo = cf[(kWo * RT + J) * 4 + g];
            const f32x4 Ee = cf[(kEe * RT + J) * 4 + g], We = cf[(kWe * RT + J) * 4 + g];
            const uint32_t ch = after(chain, ii ? Ro[ii - 1][3] : (la.nonlinear ? gdep : Re[0][0]));
            float z[8];
            scaled_normals4_f32(noise_bits(la.seed, (uint32_t)(8 * J + 2 * g), ch, k, (uint32_t)alpha,
                                    kTagMode),
                         z);
            const float zn = __shfl(z[0], (lane + 16) & 63, 64);
            if (lane < 16) cz[J * 16 + lane] = z[0];
            scaled_normals4_f32(noise_bits(la.seed, (uint32_t)(8 * J + 2 * g + 1), ch, k,
                                    (uint32_t)alpha, kTagMode),
                         z + 4);
            f32x4 ao, ae;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float ze = r < 3 ? z[2 * r + 2] : (g < 3 ? zn : 0.0f);
                ao[r] = __builtin_fmaf(Eo[r], Ro[ii][r], Wo[r] * z[2 * r + 1]);
                ae[r] = __builtin_fmaf(Ee[r], Re[ii][r], We[r] * ze);
            }
            if (a.gdt != 0.0) {
                const f32x4 Go = cf[(kGo * RT + J) * 4 + g], Ge = cf[(kGe * RT + J) * 4 + g];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    ao[r] = __builtin_fmaf(Go[r], xlane * dpp<kRowShl1>(Ro[ii][r]), ao[r]);
                    ae[r] = __builtin_fmaf(Ge[r], xlane * dpp<kRowShl1>(Re[ii][r]), ae[r]);
                }
            }
            if (J == 0) {
                const double r0y = __shfl(r0, (lane + 1) & 63, 64);
                double nr0 = __builtin_fma(a.W0, (double)z[0], r0);
                if (alpha == 0) nr0 = __builtin_fma(a.gdt, r0y, nr0);
                r0 = com_lane ? nr0 : 0.0;
            }
            if (couple) {
                f32x4 ce = f32x4{0.f, 0.f, 0.f, 0.f};
                f32x4 gn[4];  // forces of slab q + 1, read during slab q
                slab4(Gb, 0, gn, lane);
                if constexpr (BF16) {
                    f32x4 ao2 = f32x4{0.f, 0.f, 0.f, 0.f}, ce2 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int q = 0; q < KS; ++q) {
                        const bf16x8 xoh = __builtin_bit_cast(bf16x8, xc[q % DC][0]);
                        const bf16x8 xol = __builtin_bit_cast(bf16x8, xc[q % DC][1]);
                        const bf16x8 xeh = __builtin_bit_cast(bf16x8, xc[q % DC][2]);
                        const bf16x8 xel = __builtin_bit_cast(bf16x8, xc[q % DC][3]);
                        const bf16x8 gph = __builtin_bit_cast(bf16x8, gn[0]);
                        const bf16x8 gpl = __builtin_bit_cast(bf16x8, gn[1]);
                        const bf16x8 gmh = __builtin_bit_cast(bf16x8, gn[2]);
                        const bf16x8 gml = __builtin_bit_cast(bf16x8, gn[3]);
                        if (q + 1 < KS) slab4(Gb, q + 1, gn, lane);
                        f32x4 &A = (q & 1) ? ao2 : ao;
                        f32x4 &C = (q & 1) ? ce2 : ce;
                        A = mfma_bf16(xoh, gph, A);
                        C = mfma_bf16(xeh, gmh, C);
                        A = mfma_bf16(xoh, gpl, A);
                        C = mfma_bf16(xeh, gml, C);
                        A = mfma_bf16(xol, gph, A);
                        C = mfma_bf16(xel, gmh, C);
                        if constexpr (DC < KS) {
                            if (q + DC < KS) load_c(q + DC);
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                    ao += ao2;
                    ce += ce2;
                } else {
#pragma unroll
                    for (int q = 0; q < KS; ++q) {
                        f32x4 gc[4];
#pragma unroll
                        for (int k2 = 0; k2 < 4; ++k2) gc[k2] = gn[k2];
                        if (q + 1 < KS) slab4(Gb, q + 1, gn, lane);
#pragma unroll
                        for (int hh = 0; hh < 2; ++hh) {
                            const f32x4 gp = gc[2 * hh], gm = gc[2 * hh + 1];
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                ao = mfma_f32(xc[q % DC][hh][r], gp[r], ao);
                                ce = mfma_f32(xc[q % DC][2 + hh][r], gm[r], ce);
                            }
                        }
                        if constexpr (DC < KS) {
                            if (q + DC < KS) load_c(q + DC);
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                }
                const f32x4 Ce = cf[(kCe * RT + J) * 4 + g];
#pragma unroll
                for (int r = 0; r < 4; ++r) ae[r] = __builtin_fmaf(Ce[r], ce[r], ae[r]);
            }
            Ro[ii] = ao;
            Re[ii] = ae;
        }
        if constexpr (DU < KS) {
            if (la.nonlinear) {
                if constexpr (RING) {
#pragma unroll
                    for (int u = 0; u < RL; ++u) load_r(u);
                } else {
#pragma unroll
                    for (int q = 0; q < DU; ++q) load_u(q, xu[q]);
                }
            }
        }
        lds_barrier();  // C
        // lane group 3's even slot r = 3 takes normal 0 of the next tile
#pragma unroll
        for (int ii = 0; ii < NJ; ++ii) {
            const int J = wave + P * ii;
            if (J + 1 < RT) {
                const float w3 = cf[(kWe * RT + J) * 4 + g][3];
                const float zc = cz[(J + 1) * 16 + (lane & 15)];
                Re[ii][3] = __builtin_fmaf(g == 3 ? w3 : 0.0f, zc, Re[ii][3]);
            }
        }
        if (la.nonlinear) {
#pragma unroll
            for (int ii = 0; ii < NJ; ++ii) put_state(ii);
        }
        lds_barrier();  // A (also orders this step's reads of cz before the next writes)
    }
    f32x4 *Rw = reinterpret_cast<f32x4 *>(a.R) + (size_t)tile * 2 * RT * 64;
#pragma unroll
    for (int ii = 0; ii < NJ; ++ii) {
        const int J = wave + P * ii;
        Rw[J * 64 + lane] = Ro[ii];
        Rw[(RT + J) * 64 + lane] = Re[ii];
    }
    if (com_lane) a.R0[(size_t)tile * 16 + col] = r0;
}

constexpr int kCoefF4 = kKinds * 16 * 4;  // coefficients of the largest tiles

// The launch: each workgroup runs one item, on the tile shape of its bucket.
// Items are ordered longest first, so the hardware's in-order dispatch of
// workgroups to free CUs is a longest-processing-time schedule.
template <bool BF16>
__global__ __launch_bounds__(256) void fused_kernel(LaunchArgs la)
{
    __shared__ f32x4 lds[kCoefF4 + kTableFrags * 64];
    const Item it = la.items[blockIdx.x];
    const BucketArgs a = la.buckets[it.bucket];
    const int64_t step0 = la.step ? *la.step : la.step0;
    f32x4 *cf = lds, *xb = lds + kCoefF4;
    switch (a.variant) {
    case 0: fused_tiles<2, BF16, true>(a, la, it.tile0, step0, cf, xb); break;
    case 1: fused_tiles<4, BF16, true>(a, la, it.tile0, step0, cf, xb); break;
    case 2: fused_tiles<6, BF16, true>(a, la, it.tile0, step0, cf, xb); break;
    case 3: fused_tiles<8, BF16, true>(a, la, it.tile0, step0, cf, xb); break;
    case 4: fused_tiles<8, BF16, false>(a, la, it.tile0, step0, cf, xb); break;
    case 5: fused_tiles<10, BF16, false>(a, la, it.tile0, step0, cf, xb); break;
    case 6: fused_tiles<12, BF16, false>(a, la, it.tile0, step0, cf, xb); break;
    case 7: fused_tiles<14, BF16, false>(a, la, it.tile0, step0, cf, xb); break;
    case 8: fused_tiles<16, BF16, false>(a, la, it.tile0, step0, cf, xb); break;
    case 9: split_tile<4, BF16>(a, la, it.tile0, step0, cf, xb); break;
    case 10: split_tile<8, BF16>(a, la, it.tile0, step0, cf, xb); break;
    case 11: split_tile<12, BF16>(a, la, it.tile0, step0, cf, xb); break;
    case 12: split_tile<16, BF16>(a, la, it.tile0, step0, cf, xb); break;
    default: break;
    }
}

// Split tiles of 8 wavefronts (split-BF16): two wavefronts of the tile per
// SIMD, so at most 256 registers per lane; the exchange buffers of the
// largest tile (RT = 16) in LDS.
constexpr int kWideLds = kKinds * 16 * 4 + 4 * 16 * 64 + 4 * 16;  // f32x4
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void split_wide_kernel(LaunchArgs la)
{
    __shared__ f32x4 lds[kWideLds];
    const Item it = la.items[blockIdx.x];
    const BucketArgs a = la.buckets[it.bucket];
    const int64_t step0 = la.step ? *la.step : la.step0;
    switch (a.variant) {
    case 13: split_tile<8, true, 8>(a, la, it.tile0, step0, lds, lds + kKinds * 8 * 4); break;
    case 14: split_tile<16, true, 8>(a, la, it.tile0, step0, lds, lds + kKinds * 16 * 4); break;
    default: break;
    }
}

// Kernel variant of a tile shape: resident tables exist for RT <= 8,
// streamed ones for RT >= 8, split tiles for RT = 4, 8, 12, 16, and split
// tiles of 8 wavefronts for RT = 8, 16 in split-BF16.
int variant_of(int RT, bool resident) { return resident ? RT / 2 - 1 : 4 + (RT - 8) / 2; }
bool has_variant(int RT, bool resident) { return resident ? RT <= 8 : RT >= 8; }
int split_variant(int RT, int waves) { return waves == 8 ? 12 + RT / 8 : 8 + RT / 4; }
bool has_split(int RT, int waves, bool bf16)
{
    return waves == 8 ? bf16 && (RT == 8 || RT == 16) : RT >= 4 && RT <= 16 && RT % 4 == 0;
}
// Wavefronts of a bucket's split tiles (split = 1: 4, split = 2: 8).
static int split_waves(const FusedBucket &f) { return f.split == 2 ? 8 : 4; }

// Slot of mode p >= 1 of (local chain j, component alpha) in the state:
// odd p at half-mode slot (p - 1)/2, even p at p/2 - 1.
__device__ __forceinline__ size_t state_slot(int j, int alpha, int p, int RT)
{
    const int T = j / kChainsPerTile, cl = j % kChainsPerTile, col = 3 * cl + alpha;
    const int set = (p & 1) ? 0 : 1;
    const int jj = (p & 1) ? (p - 1) / 2 : p / 2 - 1;
    const int t = jj / 16, rho = jj % 16;
    const int lane = 16 * (rho / 4) + col;
    return (((size_t)T * 2 + set) * RT + t) * 256 + (size_t)lane * 4 + (rho % 4);
}

// Observables of the fused state, one workgroup of 4 wavefronts per tile.  Positions
// relative to the centre of mass, r_n - r_cm = sum_{p >= 1} phi_{n,p} R_p
// (Eq. c1; the internal modes sum to zero over the beads), in the mirror
// halves of Sec. V.A (the 4 wavefronts share the row tiles): for beads n < H
//   O_n = sum_{p odd} phi_{n,p} R_p,  E_n = sum_{p even} phi_{n,p} R_p,
//   r_n = E_n + O_n,  r_{M-1-n} = E_n - O_n,
// as FP32 MFMA products with the tables P (odd: phi_{n,2j+1}; even:
// phi_{n,2j+2} / sigma_{2j+2}, undoing the scaling of the stored even
// amplitudes), fragment (I, t, kind) holding rows 16 I + l%16 and K slots
// 16 t + 4 (l/16) + r.  The positions go to LDS; then 8 lanes per chain
// reduce bond lengths, end-to-end vector and extent in FP64, and the
// per-chain outputs and accumulators follow the FP64 path's layout.
struct ObsArgs {
    const float *R;
    const double *R0;
    const float *P;
    const double *sig;
    double *obs, *m2, *acc;
    const double *cm0;
    double *tstate, *tlast;
    const int64_t *step;
    double *ring, *ccount;
    int K, M, n, ntiles, accumulate;
};

// Observables of one tile.  LDS: pos [16][M] floats (positions about the
// centre of mass, column = 3 chain + component), then msq [5][M] floats
// (|R_p|^2 of each chain).
template <int RT>
__device__ __forceinline__ void obs_tile(const ObsArgs &a, int tile, float *pos)
{
    const int M = a.M, H = M / 2;
    float *msq = pos + 16 * M;
    const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cl = col / 3, alpha = col - 3 * cl;
    const int nvalid = min(kChainsPerTile, a.n - kChainsPerTile * tile);
    const size_t c0 = (size_t)kChainsPerTile * tile;
    f32x4 Ro[RT], Re[RT];
    const f32x4 *Rt = reinterpret_cast<const f32x4 *>(a.R) + (size_t)tile * 2 * RT * 64;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        Ro[t] = Rt[(0 * RT + t) * 64 + lane];
        Re[t] = Rt[(1 * RT + t) * 64 + lane];
    }
    const f32x4 *P = reinterpret_cast<const f32x4 *>(a.P);
    for (int I = wave; I < RT; I += 4) {
        f32x4 o = f32x4{0.f, 0.f, 0.f, 0.f}, e = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const f32x4 po = P[((I * RT + t) * 2) * 64 + lane];
            const f32x4 pe = P[((I * RT + t) * 2 + 1) * 64 + lane];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                o = mfma_f32(po[r], Ro[t][r], o);
                e = mfma_f32(pe[r], Re[t][r], e);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int nb = 16 * I + 4 * g + r;
            if (nb < H) {
                pos[col * M + nb] = e[r] + o[r];
                pos[col * M + M - 1 - nb] = e[r] - o[r];
            }
        }
    }
    // |R_p|^2 of p >= 1, summed over the chain's three component lanes: the
    // mode tiles spread over the wavefronts, staged in LDS
    for (int t = wave; t < RT; t += 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = 16 * t + 4 * g + r;
            const float vo = Ro[t][r];
            const float ve = j < H - 1 ? (float)((double)Re[t][r] / a.sig[j]) : 0.0f;
            const float so = comp_sum(vo * vo, alpha), se = comp_sum(ve * ve, alpha);
            if (alpha == 0 && col < 15) {
                const int po = 2 * j + 1, pe = 2 * j + 2;
                if (po < M) msq[cl * M + po] = so;
                if (pe < M) msq[cl * M + pe] = se;
            }
        }
    }
    __syncthreads();
    // written out chain by chain, consecutive modes in consecutive threads
    const int W = acc_width(M);
    for (int i = threadIdx.x; i < nvalid * M; i += blockDim.x) {
        const int c = i / M, p = i - c * M;
        if (p == 0) continue;  // the centre of mass, below
        const float v = msq[c * M + p];
        a.m2[(c0 + c) * M + p] = v;
        if (a.accumulate) a.acc[(c0 + c) * W + DM_NACC_HEAD + p] += v;
    }
    // 32 lanes per chain (chains 0..4 in threads 0..159): bond lengths and the
    // x extent
    const int c8 = threadIdx.x >> 5, part = threadIdx.x & 31;
    const bool cv = c8 < nvalid;
    if (c8 >= kChainsPerTile) return;
    const float *px = pos + 3 * (cv ? c8 : 0) * M, *py = px + M, *pz = py + M;
    double ls = 0.0, l2s = 0.0, xmin = 1e300, xmax = -1e300;
    if (cv) {
        for (int nb = part; nb < M; nb += 32) {
            const double x = px[nb];
            xmin = fmin(xmin, x);
            xmax = fmax(xmax, x);
            if (nb >= 1) {
                const double ux = x - px[nb - 1], uy = (double)py[nb] - py[nb - 1],
                             uz = (double)pz[nb] - pz[nb - 1];
                const double q = ux * ux + uy * uy + uz * uz;
                ls += sqrt(q);
                l2s += q;
            }
        }
    }
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
        ls += __shfl_xor(ls, off, 64);
        l2s += __shfl_xor(l2s, off, 64);
        xmin = fmin(xmin, __shfl_xor(xmin, off, 64));
        xmax = fmax(xmax, __shfl_xor(xmax, off, 64));
    }
    if (!cv || part != 0) return;
    const size_t c = c0 + c8;
    const double *r0 = a.R0 + (size_t)tile * 16 + 3 * c8;
    const double rs = 1.0 / sqrt((double)M);
    double o[DM_NCHAIN_OBS];
    o[DM_CO_BOND] = ls / (M - 1);
    const double Lx = (double)px[M - 1] - px[0], Ly = (double)py[M - 1] - py[0],
                 Lz = (double)pz[M - 1] - pz[0];
    o[DM_CO_L2] = Lx * Lx + Ly * Ly + Lz * Lz;
    o[DM_CO_LX] = Lx;
    o[DM_CO_LX + 1] = Ly;
    o[DM_CO_LX + 2] = Lz;
    const int m = M / 2, mid = (M - 1) / 2;
    const float *pc[3] = {px, py, pz};
    for (int k = 0; k < 3; ++k) {
        o[DM_CO_CM + k] = r0[k] * rs;
        o[DM_CO_UMID + k] = (double)pc[k][m] - pc[k][m - 1];
        o[DM_CO_DMID + k] = pc[k][mid];
    }
    o[DM_CO_XSPAN] = xmax - xmin;
    o[DM_CO_BOND2] = l2s / (M - 1);
    for (int k = 0; k < DM_NCHAIN_OBS; ++k) a.obs[c * DM_NCHAIN_OBS + k] = o[k];
    const double m20 = r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2];
    a.m2[c * M] = m20;
    if (!a.accumulate) return;
    double *ac = a.acc + c * W;
    const double dx = o[DM_CO_CM] - a.cm0[3 * c], dy = o[DM_CO_CM + 1] - a.cm0[3 * c + 1],
                 dz = o[DM_CO_CM + 2] - a.cm0[3 * c + 2];
    ac[DM_NACC_HEAD] += m20;
    ac[DM_ACC_NSAMPLES] += 1.0;
    ac[DM_ACC_BOND] += o[DM_CO_BOND];
    ac[DM_ACC_BOND2] += o[DM_CO_BOND2];
    ac[DM_ACC_L2] += o[DM_CO_L2];
    ac[DM_ACC_MSDCM] += dx * dx + dy * dy + dz * dz;
    ac[DM_ACC_DMID2] += o[DM_CO_DMID] * o[DM_CO_DMID] + o[DM_CO_DMID + 1] * o[DM_CO_DMID + 1] +
                        o[DM_CO_DMID + 2] * o[DM_CO_DMID + 2];
    ac[DM_ACC_XSPAN] += o[DM_CO_XSPAN];
    // tumbling in the flow plane, with hysteresis (as the FP64 path)
    const double rho = sqrt(Lx * Lx + Ly * Ly);
    const double s0 = a.tstate[c];
    const double s1 = Lx > 0.5 * rho ? 1.0 : (Lx < -0.5 * rho ? -1.0 : s0);
    if (s0 != 0.0 && s1 != s0) {
        const double k = (double)*a.step;
        ac[DM_ACC_TUMBLES] += 1.0;
        if (a.tlast[c] > 0.0) {
            const double tau = k - (a.tlast[c] - 1.0);
            ac[DM_ACC_TAU] += tau;
            ac[DM_ACC_TAU2] += tau * tau;
            ac[DM_ACC_NTAU] += 1.0;
            ac[DM_NACC_HEAD + M + min(DM_NTUMBLE_BINS - 1, max(0, ilogb(tau)))] += 1.0;
        }
        a.tlast[c] = k + 1.0;
    }
    a.tstate[c] = s1;
    if (a.K > 0) {
        const double v[9] = {Lx, Ly, Lz, o[DM_CO_UMID], o[DM_CO_UMID + 1], o[DM_CO_UMID + 2],
                             o[DM_CO_DMID], o[DM_CO_DMID + 1], o[DM_CO_DMID + 2]};
        corr_update(a.ring + c * ((size_t)9 << (a.K - 1)), a.ccount + c,
                    ac + DM_NACC_HEAD + M + DM_NTUMBLE_BINS, v, a.K);
    }
}

// One workgroup per tile, or a smaller grid looping over the tiles (to leave
// most compute units to a fused launch running at the same time).
template <int RT>
__global__ __launch_bounds__(256) void fused_obs_kernel(ObsArgs a)
{
    extern __shared__ float pos[];  // [16][M]
    for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        obs_tile<RT>(a, tile, pos);
        __syncthreads();  // pos is rewritten for the next tile
    }
}

__global__ void snapshot_kernel(const f32x4 *__restrict__ R, f32x4 *__restrict__ Rs, size_t n4,
                                const double *__restrict__ R0, double *__restrict__ R0s,
                                size_t n0)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        Rs[i] = R[i];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n0; i += stride)
        R0s[i] = R0[i];
}

// FP64 amplitudes [chain][component][p] -> fused state (even modes scaled
// by sigma_p, sig[p/2 - 1]) and back.
__global__ void pack_kernel(const double *__restrict__ R64, const double *__restrict__ sig,
                            float *__restrict__ R, double *__restrict__ R0, int M, int n, int RT)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n * 3 * M) return;
    const int p = (int)(idx % M);
    const int alpha = (int)((idx / M) % 3);
    const int j = (int)(idx / ((size_t)3 * M));
    const double v = R64[idx];
    if (p == 0)
        R0[(size_t)(j / kChainsPerTile) * 16 + 3 * (j % kChainsPerTile) + alpha] = v;
    else
        R[state_slot(j, alpha, p, RT)] = (float)((p & 1) ? v : v * sig[p / 2 - 1]);
}

__global__ void unpack_kernel(const float *__restrict__ R, const double *__restrict__ R0,
                              const double *__restrict__ sig, double *__restrict__ R64, int M,
                              int n, int RT)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n * 3 * M) return;
    const int p = (int)(idx % M);
    const int alpha = (int)((idx / M) % 3);
    const int j = (int)(idx / ((size_t)3 * M));
    if (p == 0) {
        R64[idx] = R0[(size_t)(j / kChainsPerTile) * 16 + 3 * (j % kChainsPerTile) + alpha];
    } else {
        const double v = (double)R[state_slot(j, alpha, p, RT)];
        R64[idx] = (p & 1) ? v : v / sig[p / 2 - 1];
    }
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
int table_frags(int RT) { return 4 * RT * RT; }  // both products, all coupling rows
size_t x_bytes(int RT) { return (size_t)table_frags(RT) * 1024; }
// LDS fragments of the resident tables with jc coupling row tiles
bool fits_resident(int RT, int jc) { return 2 * RT * RT + jc * RT <= kTableFrags; }

// K index of slot e in lane group gq of K-slab q (BF16, K = 32 per slab).
inline int kslab_index(int q, int gq, int e)
{
    return 32 * q + (e < 4 ? 4 * gq + e : 16 + 4 * gq + (e - 4));
}

unsigned nblocks(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

const double kPi = 3.141592653589793238462643383279502884;

// sin(pi m / d) for integers m, d > 0, with exact zeros at multiples of d.
double sin_pi_frac(long m, long d)
{
    m %= 2 * d;
    if (m == 0 || m == d) return 0.0;
    return std::sin(kPi * (double)m / (double)d);
}

}  // namespace

bool fused_supports(int M) { return M >= 2 && M <= 512 && (M % 2) == 0; }

hipError_t fused_alloc(FusedBucket &f, int M, int n, bool bf16)
{
    f.bf16 = bf16 ? 1 : 0;
    f.RT = rt_of(M);
    f.ntiles = tiles_of(n);
    f.n = n;
    const int RT = f.RT, H = M / 2, Hp = 16 * RT;
    // half-bond x half-mode tables, bond row i <-> bond i + 1:
    //   Xo[i][j] = chi_{i+1, 2j+1} = sigma_{2j+1} sin((i+1)(2j+1) pi/M)
    //   Se[i][j] = sin((i+1)(j+1) pi/H) for i, j < H - 1 (the even modes
    //              p = 2j + 2 < M, the bonds off the middle one), else 0
    f.Xo.assign((size_t)Hp * Hp, 0.0);
    f.Se.assign((size_t)Hp * Hp, 0.0);
    std::vector<double> sig((size_t)Hp, 0.0);  // sigma_{2j+2}
    auto sigma = [&](int p) { return -2.0 * std::sqrt(2.0 / M) * sin_pi_frac(p, 2L * M); };
    for (int j = 0; j + 1 < H; ++j) sig[j] = sigma(2 * j + 2);
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < H; ++j) {
            f.Xo[(size_t)i * Hp + j] = sigma(2 * j + 1) * sin_pi_frac((long)(i + 1) * (2 * j + 1), M);
            if (i + 1 < H && j + 1 < H)
                f.Se[(size_t)i * Hp + j] = sin_pi_frac((long)(i + 1) * (j + 1), H);
        }
    f.sig = sig;
    const size_t xb = x_bytes(RT);
    hipError_t e;
    if ((e = hipMalloc(&f.d_X, xb)) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&f.d_R, sizeof(float) * state_floats(RT, f.ntiles))) != hipSuccess)
        return e;
    if ((e = hipMalloc((void **)&f.d_R0, sizeof(double) * 16 * (size_t)f.ntiles)) != hipSuccess)
        return e;
    if ((e = hipMalloc((void **)&f.d_coef, sizeof(float) * kKinds * 16 * (size_t)RT)) !=
        hipSuccess)
        return e;
    if ((e = hipMalloc((void **)&f.d_sig, sizeof(double) * Hp)) != hipSuccess) return e;
    if ((e = hipMemcpy(f.d_sig, sig.data(), sizeof(double) * Hp, hipMemcpyHostToDevice)) !=
        hipSuccess)
        return e;
    if ((e = hipMemset(f.d_X, 0, xb)) != hipSuccess) return e;
    if ((e = hipMemset(f.d_R, 0, sizeof(float) * state_floats(RT, f.ntiles))) != hipSuccess)
        return e;
    // observation tables: rows n (bead), K slot j; fragment (I, t, kind)
    const double c1 = std::sqrt(2.0 / M);
    std::vector<float> P((size_t)2 * RT * RT * 256, 0.0f);
    for (int I = 0; I < RT; ++I)
        for (int t = 0; t < RT; ++t)
            for (int kind = 0; kind < 2; ++kind)
                for (int l = 0; l < 64; ++l)
                    for (int r = 0; r < 4; ++r) {
                        const int nb = 16 * I + l % 16, j = 16 * t + 4 * (l / 16) + r;
                        const int p = kind == 0 ? 2 * j + 1 : 2 * j + 2;
                        double v = 0.0;
                        if (nb < H && p < M) {
                            // cos(p (n + 1/2) pi / M) = cos(pi p (2n + 1) / 2M)
                            v = c1 * std::cos(kPi * (double)((long)p * (2 * nb + 1) % (4L * M)) /
                                              (2.0 * M));
                            if (kind == 1) v /= sig[j];
                        }
                        P[((((size_t)I * RT + t) * 2 + kind) * 64 + l) * 4 + r] = (float)v;
                    }
    if ((e = hipMalloc((void **)&f.d_P, sizeof(float) * P.size())) != hipSuccess) return e;
    return hipMemcpy(f.d_P, P.data(), sizeof(float) * P.size(), hipMemcpyHostToDevice);
}

// Write both products' fragments (layout at fused_kernel) for step
// coefficients C and upload them.
static hipError_t upload_tables(const FusedBucket &f, int M, const double *C, hipStream_t st)
{
    const int RT = f.RT, KS = RT / 2, H = M / 2, Hp = 16 * RT, G1 = 2 * RT * RT;
    // u = chi R: row i, K index kk (mode slot), kind 0 odd / 1 even
    auto v1 = [&](int kind, int i, int kk) {
        return (kind == 0 ? f.Xo : f.Se)[(size_t)i * Hp + kk];
    };
    // coupling: row j (mode slot), K index kk (bond row)
    auto v2 = [&](int kind, int j, int kk) {
        if (kind == 1) return f.Se[(size_t)kk * Hp + j];
        const int p = 2 * j + 1;
        if (p >= M) return 0.0;
        double v = f.Xo[(size_t)kk * Hp + j] * C[p];
        if (kk == H - 1) v *= 0.5;  // the middle bond enters G+ twice
        return v;
    };
    const size_t nfr = (size_t)table_frags(RT);
    std::vector<unsigned char> h(nfr * 1024);
    for (size_t F = 0; F < nfr; ++F) {
        // decode fragment F
        int prod, kind, A, q, sub;  // sub: hi/lo (BF16) or K slice (FP32)
        if ((int)F < G1) {
            prod = 0;
            const int fr = (int)F % 4;
            A = ((int)F / 4) % RT;
            q = (int)F / 4 / RT;
            kind = fr / 2;
            sub = fr % 2;
        } else {
            prod = 1;
            const int G = (int)F - G1;
            sub = G % 2;
            q = (G / 2) % KS;
            kind = (G / 2 / KS) % 2;
            A = G / 2 / KS / 2;
        }
        for (int l = 0; l < 64; ++l) {
            const int row = 16 * A + l % 16;
            if (f.bf16) {
                __bf16 *o = reinterpret_cast<__bf16 *>(h.data() + F * 1024) + l * 8;
                for (int el = 0; el < 8; ++el) {
                    const int kk = kslab_index(q, l / 16, el);
                    const double v = prod == 0 ? v1(kind, row, kk) : v2(kind, row, kk);
                    const __bf16 vh = (__bf16)(float)v;
                    o[el] = sub == 0 ? vh : (__bf16)(float)(v - (double)(float)vh);
                }
            } else {
                float *o = reinterpret_cast<float *>(h.data() + F * 1024) + l * 4;
                for (int r = 0; r < 4; ++r) {
                    const int kk = 16 * (2 * q + sub) + 4 * (l / 16) + r;
                    o[r] = (float)(prod == 0 ? v1(kind, row, kk) : v2(kind, row, kk));
                }
            }
        }
    }
    hipError_t e = hipMemcpyAsync(f.d_X, h.data(), h.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

void fused_free(FusedBucket &f)
{
    if (f.d_X) (void)hipFree(f.d_X);
    if (f.d_R) (void)hipFree(f.d_R);
    if (f.d_R0) (void)hipFree(f.d_R0);
    if (f.d_coef) (void)hipFree(f.d_coef);
    if (f.d_sig) (void)hipFree(f.d_sig);
    if (f.d_P) (void)hipFree(f.d_P);
    if (f.d_Rs) (void)hipFree(f.d_Rs);
    if (f.d_R0s) (void)hipFree(f.d_R0s);
    f = FusedBucket();
}

hipError_t fused_pack_modes(FusedBucket &f, const double *R64, int M, int n, hipStream_t st)
{
    const size_t N = (size_t)n * 3 * M;
    hipLaunchKernelGGL(pack_kernel, dim3(nblocks(N, 256)), dim3(256), 0, st, R64, f.d_sig, f.d_R,
                       f.d_R0, M, n, f.RT);
    return hipGetLastError();
}

hipError_t fused_unpack_modes(const FusedBucket &f, double *R64, int M, int n, hipStream_t st)
{
    const size_t N = (size_t)n * 3 * M;
    hipLaunchKernelGGL(unpack_kernel, dim3(nblocks(N, 256)), dim3(256), 0, st, f.d_R, f.d_R0,
                       f.d_sig, R64, M, n, f.RT);
    return hipGetLastError();
}

hipError_t fused_set_coefs(FusedBucket &f, const ModeCoefs &mc, int M, double lin, double gdt,
                           hipStream_t st)
{
    const int RT = f.RT, Hp = 16 * RT;
    // [kind][slot j]: odd p = 2j + 1, even p = 2j + 2 (scaled by sigma_p);
    // padding p >= M stays zero.  C of the odd modes goes into the table.
    // W (and W0) carry kNormalScale: the kernels' normals come divided by it.
    std::vector<float> h((size_t)kKinds * Hp, 0.0f);
    for (int j = 0; j < Hp; ++j) {
        const int po = 2 * j + 1, pe = 2 * j + 2;
        if (po < M) {
            h[kEo * Hp + j] = (float)mc.E[po];
            h[kWo * Hp + j] = (float)(kNormalScale * mc.W[po]);
            h[kGo * Hp + j] = (float)(gdt * mc.E[po]);
        }
        if (pe < M) {
            const double sg = f.sig[j];
            h[kEe * Hp + j] = (float)mc.E[pe];
            h[kWe * Hp + j] = (float)(kNormalScale * sg * mc.W[pe]);
            h[kGe * Hp + j] = (float)(gdt * mc.E[pe]);
            h[kCe * Hp + j] = (float)(sg * sg * mc.C[pe]);
        }
    }
    f.W0 = kNormalScale * mc.W[0];
    f.gdt = gdt;
    f.lin = (float)lin;
    // Coupling rows whose kick is below FP32 resolution of the update are
    // skipped (Eq. f4: for modes equilibrated within a step the coupling is
    // exponentially small).  |Delta H_p| <= |chi_p| |g| <= 2 s_p * 3 sqrt(M)
    // (column norm 2 s_p from Eq. e6; |g_n| = |1 - (1-2nu) l_n| <= 3 for
    // bonds shorter than four rest lengths); row tile J (modes 32J + 1 ..
    // 32J + 32) is kept if any of its modes has C_p * 6 s_p sqrt(M) >=
    // 2^-30 W_p.
    int pmax = 0;
    for (int p = 1; p < M; ++p) {
        const double sp = sin_pi_frac(p, 2L * M);
        if (mc.C[p] * 6.0 * sp * std::sqrt((double)M) >= std::ldexp(mc.W[p], -30)) pmax = p;
    }
    f.JC = pmax > 0 ? std::min(RT, (pmax - 1) / 32 + 1) : 0;
    f.resident = fits_resident(RT, f.JC) ? 1 : 0;
    f.tpw = 4;  // default shape; timings of other coefficients are stale
    f.split = 0;
    f.item_us = 0.0;
    hipError_t e;
    if ((e = upload_tables(f, M, mc.C.data(), st)) != hipSuccess) return e;
    e = hipMemcpyAsync(f.d_coef, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

static BucketArgs bucket_args(const FusedBucket &f)
{
    BucketArgs a;
    a.X = f.d_X;
    a.R = f.d_R;
    a.R0 = f.d_R0;
    a.coef = f.d_coef;
    a.ids = f.ids;
    a.n = f.n;
    a.ntiles = f.ntiles;
    a.x_bytes = (int)x_bytes(f.RT);
    a.jc = f.JC;
    a.variant = f.split ? split_variant(f.RT, split_waves(f)) : variant_of(f.RT, f.resident != 0);
    a.tpw = f.tpw;
    a.lin = f.lin;
    a.W0 = f.W0;
    a.gdt = f.gdt;
    return a;
}

// Cost model of one workgroup-step when nothing was measured: the MFMA and
// table work grow as RT^2, the noise and forces as RT; a split tile takes
// about a third of a wavefront's time for one tile (a quarter on 8
// wavefronts).
static double model_us(const FusedBucket &f)
{
    const double rt = f.RT;
    const double us = 0.12 * rt * rt + 0.3 * rt + (f.resident ? 0.0 : 0.02 * rt * rt);
    return f.split == 2 ? us / 4.0 : f.split ? us / 3.0 : us;
}

double fused_item_us(const FusedBucket &f) { return f.item_us > 0.0 ? f.item_us : model_us(f); }

// Items of the given buckets, longest first (ties in bucket, tile order).
static std::vector<Item> ordered_items(const std::vector<const FusedBucket *> &bs,
                                       std::vector<double> *cost = nullptr)
{
    std::vector<std::pair<double, Item>> v;
    for (size_t b = 0; b < bs.size(); ++b) {
        const FusedBucket &f = *bs[b];
        const double c = f.item_us > 0.0 ? f.item_us : model_us(f);
        for (int t = 0; t < f.ntiles; t += f.tpw) v.push_back({c, Item{(int)b, t}});
    }
    std::stable_sort(v.begin(), v.end(),
                     [](const std::pair<double, Item> &x, const std::pair<double, Item> &y) {
                         return x.first > y.first;
                     });
    std::vector<Item> out;
    out.reserve(v.size());
    if (cost) cost->clear();
    for (auto &e : v) {
        out.push_back(e.second);
        if (cost) cost->push_back(e.first);
    }
    return out;
}

void fused_plan_free(FusedPlan &p)
{
    if (p.d_buckets) (void)hipFree(p.d_buckets);
    if (p.d_items) (void)hipFree(p.d_items);
    p = FusedPlan();
}

// The bodies of all tile shapes are inlined into the launch kernels, whose
// private (spill) segment must stay within the HIP runtime's default
// per-thread stack of 1 KB: a larger segment is refused here rather than
// launched.
constexpr size_t kMaxPrivateBytes = 1024;
static hipError_t check_private_segment(const void *fn)
{
    hipFuncAttributes at;
    hipError_t e = hipFuncGetAttributes(&at, fn);
    if (e != hipSuccess) return e;
    return at.localSizeBytes <= kMaxPrivateBytes ? hipSuccess : hipErrorInvalidConfiguration;
}

hipError_t fused_plan(FusedPlan &p, const std::vector<const FusedBucket *> &bs, int max_items,
                      hipStream_t st)
{
    fused_plan_free(p);
    if (bs.empty()) return hipSuccess;
    p.bf16 = bs[0]->bf16;
    hipError_t e = check_private_segment(p.bf16 ? reinterpret_cast<const void *>(&fused_kernel<true>)
                                                : reinterpret_cast<const void *>(&fused_kernel<false>));
    if (e != hipSuccess) return e;
    std::vector<BucketArgs> ba;
    bool wide = false;
    for (const FusedBucket *f : bs) {
        if (f->bf16 != p.bf16) return hipErrorInvalidValue;
        const bool ok = f->split ? f->split <= 2 && has_split(f->RT, split_waves(*f), f->bf16 != 0) &&
                                       f->tpw == 1 && !f->resident
                                 : has_variant(f->RT, f->resident != 0) && f->tpw >= 1 &&
                                       f->tpw <= 4 && (f->resident || f->tpw == 4);
        if (!ok) return hipErrorInvalidValue;
        wide = wide || f->split == 2;
        ba.push_back(bucket_args(*f));
    }
    if (wide && (e = check_private_segment(reinterpret_cast<const void *>(&split_wide_kernel))) !=
                    hipSuccess)
        return e;
    std::vector<Item> items = ordered_items(bs);
    if (max_items > 0 && (int)items.size() > max_items) items.resize(max_items);
    // the items of 8-wavefront split tiles go to their own kernel, after the
    // others (each part keeps its longest-first order)
    std::stable_partition(items.begin(), items.end(),
                          [&](const Item &it) { return bs[it.bucket]->split != 2; });
    p.nitems = (int)items.size();
    p.nwide = (int)std::count_if(items.begin(), items.end(),
                                 [&](const Item &it) { return bs[it.bucket]->split == 2; });
    p.nbuckets = (int)bs.size();
    if ((e = hipMalloc(&p.d_buckets, sizeof(BucketArgs) * ba.size())) != hipSuccess) return e;
    if ((e = hipMalloc(&p.d_items, sizeof(Item) * std::max<size_t>(1, items.size()))) !=
        hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(p.d_buckets, ba.data(), sizeof(BucketArgs) * ba.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(p.d_items, items.data(), sizeof(Item) * items.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
    return hipStreamSynchronize(st);  // the host vectors die here
}

hipError_t fused_launch(const FusedPlan &p, uint64_t seed, int64_t step0, const int64_t *d_step,
                        int n_steps, int nonlinear, hipStream_t st)
{
    if (n_steps <= 0 || p.nitems == 0) return hipSuccess;
    LaunchArgs la;
    la.buckets = static_cast<const BucketArgs *>(p.d_buckets);
    la.items = static_cast<const Item *>(p.d_items);
    la.step = d_step;
    la.step0 = step0;
    la.seed = seed;
    la.n_steps = n_steps;
    la.nonlinear = nonlinear;
    const int nmain = p.nitems - p.nwide;
    if (nmain > 0) {
        if (p.bf16)
            hipLaunchKernelGGL(fused_kernel<true>, dim3(nmain), dim3(256), 0, st, la);
        else
            hipLaunchKernelGGL(fused_kernel<false>, dim3(nmain), dim3(256), 0, st, la);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (p.nwide > 0) {
        la.items += nmain;
        hipLaunchKernelGGL(split_wide_kernel, dim3(p.nwide), dim3(512), 0, st, la);
    }
    return hipGetLastError();
}

// Makespan of a longest-first list schedule of the items on ncu CUs (one
// workgroup per CU: the tables take the LDS).
static double makespan(const std::vector<double> &cost, int ncu)
{
    std::vector<double> load((size_t)std::max(1, ncu), 0.0);
    double m = 0.0;
    for (double c : cost) {  // cost is sorted longest first
        auto it = std::min_element(load.begin(), load.end());
        *it += c;
        m = std::max(m, *it);
    }
    return m;
}

hipError_t fused_autotune(std::vector<FusedBucket *> &bs, uint64_t seed, int steps,
                          hipStream_t st, std::string &report)
{
    int dev = 0, ncu = 256;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) !=
        hipSuccess)
        return e;
    if (steps < 1) steps = 64;
    struct Cand {
        int resident, tpw, split;
        double us;  // per workgroup-step
    };
    std::vector<std::vector<Cand>> cands(bs.size());
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) return e;
    for (size_t b = 0; b < bs.size() && e == hipSuccess; ++b) {
        FusedBucket &f = *bs[b];
        // time each shape on a scratch copy of the state (the tables and
        // coefficients are shared, the state is not touched)
        FusedBucket t = f;
        t.d_R = nullptr;
        t.d_R0 = nullptr;
        const size_t nR = sizeof(float) * state_floats(f.RT, f.ntiles);
        const size_t nR0 = sizeof(double) * 16 * (size_t)f.ntiles;
        if ((e = hipMalloc((void **)&t.d_R, nR)) != hipSuccess) break;
        if ((e = hipMalloc((void **)&t.d_R0, nR0)) != hipSuccess) {
            (void)hipFree(t.d_R);
            break;
        }
        e = hipMemcpyAsync(t.d_R, f.d_R, nR, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(t.d_R0, f.d_R0, nR0, hipMemcpyDeviceToDevice, st);
        std::vector<Cand> list;
        for (int res = 1; res >= 0; --res) {
            if (!has_variant(f.RT, res) || (res && !fits_resident(f.RT, f.JC))) continue;
            for (int tpw : {4, 2, 1}) {
                if (!res && tpw != 4) continue;
                list.push_back({res, tpw, 0, 0.0});
            }
        }
        if (has_split(f.RT, 4, f.bf16 != 0)) list.push_back({0, 1, 1, 0.0});
        if (has_split(f.RT, 8, f.bf16 != 0)) list.push_back({0, 1, 2, 0.0});
        for (Cand &c : list) {
            if (e != hipSuccess) break;
            t.resident = c.resident;
            t.tpw = c.tpw;
            t.split = c.split;
            t.item_us = 0.0;
            FusedPlan p;
            // at most one workgroup per CU: the time of one item
            e = fused_plan(p, {&t}, ncu, st);
            double best = 1e30;
            for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
                e = hipEventRecord(e0, st);
                if (e == hipSuccess) e = fused_launch(p, seed, 0, nullptr, steps, 1, st);
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                best = std::min(best, 1e3 * (double)ms / steps);
            }
            fused_plan_free(p);
            c.us = best;
        }
        (void)hipFree(t.d_R);
        (void)hipFree(t.d_R0);
        cands[b] = list;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    // choose one shape per bucket: exhaustive over small products, otherwise
    // each bucket's cheapest shape per tile
    size_t combos = 1;
    for (auto &l : cands) combos = std::min<size_t>(combos * std::max<size_t>(1, l.size()), 1 << 20);
    std::vector<int> pick(bs.size(), 0), cur(bs.size(), 0);
    // the 8-wavefront split tiles run in a kernel of their own after the
    // others: the two makespans add
    auto evaluate = [&](const std::vector<int> &sel) {
        std::vector<double> cost, wcost;
        for (size_t b = 0; b < bs.size(); ++b) {
            const Cand &c = cands[b][sel[b]];
            const int ni = (bs[b]->ntiles + c.tpw - 1) / c.tpw;
            std::vector<double> &v = c.split == 2 ? wcost : cost;
            v.insert(v.end(), (size_t)ni, c.us);
        }
        std::sort(cost.begin(), cost.end(), std::greater<double>());
        std::sort(wcost.begin(), wcost.end(), std::greater<double>());
        return makespan(cost, ncu) + makespan(wcost, ncu);
    };
    if (combos <= 4096) {
        double best = 1e300;
        for (size_t k = 0; k < combos; ++k) {
            size_t r = k;
            for (size_t b = 0; b < bs.size(); ++b) {
                cur[b] = (int)(r % cands[b].size());
                r /= cands[b].size();
            }
            const double m = evaluate(cur);
            if (m < best) {
                best = m;
                pick = cur;
            }
        }
    } else {
        // from each bucket's cheapest shape per tile, change one bucket at a
        // time while the makespan shrinks
        for (size_t b = 0; b < bs.size(); ++b) {
            double best = 1e300;
            for (size_t c = 0; c < cands[b].size(); ++c) {
                const double per_tile = cands[b][c].us / cands[b][c].tpw;
                if (per_tile < best) {
                    best = per_tile;
                    pick[b] = (int)c;
                }
            }
        }
        double cur_m = evaluate(pick);
        for (int pass = 0; pass < 8; ++pass) {
            bool improved = false;
            for (size_t b = 0; b < bs.size(); ++b)
                for (size_t c = 0; c < cands[b].size(); ++c) {
                    if ((int)c == pick[b]) continue;
                    std::vector<int> trial = pick;
                    trial[b] = (int)c;
                    const double m = evaluate(trial);
                    if (m < cur_m) {
                        cur_m = m;
                        pick = trial;
                        improved = true;
                    }
                }
            if (!improved) break;
        }
    }
    char line[256];
    report.clear();
    for (size_t b = 0; b < bs.size(); ++b) {
        FusedBucket &f = *bs[b];
        const Cand &c = cands[b][pick[b]];
        f.resident = c.resident;
        f.tpw = c.tpw;
        f.split = c.split;
        f.item_us = c.us;
        for (size_t k = 0; k < cands[b].size(); ++k) {
            const Cand &ck = cands[b][k];
            const char *shape = ck.split == 2 ? "split8"
                                : ck.split    ? "split"
                                : ck.resident ? "resident"
                                              : "streamed";
            snprintf(line, sizeof line, "RT=%d %s tpw=%d: %.2f us/step%s\n", f.RT, shape, ck.tpw,
                     ck.us,
                     (int)k == pick[b] ? "  <- chosen" : "");
            report += line;
        }
    }
    return hipSuccess;
}

void fused_force_shape(FusedBucket &f, int table_mode, int tpw)
{
    if (table_mode == 1 && has_variant(f.RT, true) && fits_resident(f.RT, f.JC)) {
        f.resident = 1;
        f.split = 0;
        f.item_us = 0.0;
    } else if (table_mode == 2 && has_variant(f.RT, false)) {
        f.resident = 0;
        f.split = 0;
        f.tpw = 4;
        f.item_us = 0.0;
    } else if ((table_mode == 3 || table_mode == 4) &&
               has_split(f.RT, table_mode == 4 ? 8 : 4, f.bf16 != 0)) {
        f.resident = 0;
        f.split = table_mode == 4 ? 2 : 1;
        f.tpw = 1;
        f.item_us = 0.0;
    }
    if (tpw >= 1 && tpw <= 4 && f.resident) {
        f.tpw = tpw;
        f.item_us = 0.0;
    }
}

__global__ void set_step_kernel(int64_t *d_step, int64_t value, int64_t add)
{
    if (threadIdx.x == 0) *d_step = add ? *d_step + add : value;
}

hipError_t fused_set_step(int64_t *d_step, int64_t value, hipStream_t st)
{
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, st, d_step, value, (int64_t)0);
    return hipGetLastError();
}

hipError_t fused_advance_step(int64_t *d_step, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, st, d_step, (int64_t)0, n);
    return hipGetLastError();
}

template <int RT>
static void launch_obs(const ObsArgs &a, int nwg, hipStream_t st)
{
    hipLaunchKernelGGL(fused_obs_kernel<RT>, dim3(nwg), dim3(256),
                       sizeof(float) * (16 + kChainsPerTile) * (size_t)a.M, st, a);
}

hipError_t fused_snapshot_alloc(FusedBucket &f)
{
    hipError_t e = hipSuccess;
    if (!f.d_Rs) e = hipMalloc((void **)&f.d_Rs, sizeof(float) * state_floats(f.RT, f.ntiles));
    if (e == hipSuccess && !f.d_R0s)
        e = hipMalloc((void **)&f.d_R0s, sizeof(double) * 16 * (size_t)f.ntiles);
    return e;
}

hipError_t fused_snapshot(const FusedBucket &f, hipStream_t st)
{
    if (f.n <= 0) return hipSuccess;
    if (!f.d_Rs || !f.d_R0s) return hipErrorInvalidValue;
    const size_t n4 = state_floats(f.RT, f.ntiles) / 4, n0 = (size_t)16 * f.ntiles;
    unsigned b = nblocks(n4, 256);
    if (b > 1024) b = 1024;
    hipLaunchKernelGGL(snapshot_kernel, dim3(b), dim3(256), 0, st,
                       reinterpret_cast<const f32x4 *>(f.d_R), reinterpret_cast<f32x4 *>(f.d_Rs),
                       n4, f.d_R0, f.d_R0s, n0);
    return hipGetLastError();
}

hipError_t fused_observe(const FusedBucket &f, int M, double *obs, double *m2, double *acc,
                         const double *cm0, double *tstate, double *tlast,
                         const int64_t *d_step, double *ring, double *ccount, int K,
                         int accumulate, hipStream_t st, bool from_snapshot, int max_wg)
{
    if (f.n <= 0) return hipSuccess;
    if (from_snapshot && (!f.d_Rs || !f.d_R0s)) return hipErrorInvalidValue;
    ObsArgs a;
    a.R = from_snapshot ? f.d_Rs : f.d_R;
    a.R0 = from_snapshot ? f.d_R0s : f.d_R0;
    a.P = f.d_P;
    a.sig = f.d_sig;
    a.obs = obs;
    a.m2 = m2;
    a.acc = acc;
    a.cm0 = cm0;
    a.tstate = tstate;
    a.tlast = tlast;
    a.step = d_step;
    a.ring = ring;
    a.ccount = ccount;
    a.K = K;
    a.M = M;
    a.n = f.n;
    a.ntiles = f.ntiles;
    a.accumulate = accumulate;
    const int nwg = max_wg > 0 ? std::min(f.ntiles, max_wg) : f.ntiles;
    switch (f.RT) {
    case 2: launch_obs<2>(a, nwg, st); break;
    case 4: launch_obs<4>(a, nwg, st); break;
    case 6: launch_obs<6>(a, nwg, st); break;
    case 8: launch_obs<8>(a, nwg, st); break;
    case 10: launch_obs<10>(a, nwg, st); break;
    case 12: launch_obs<12>(a, nwg, st); break;
    case 14: launch_obs<14>(a, nwg, st); break;
    case 16: launch_obs<16>(a, nwg, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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
