// dm_rng.h -- counter-based Gaussian noise for the Langevin steps.
//
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies and xors
// on a 128-bit counter, key schedule by the Weyl constants.  Box-Muller
// (1958) turns the four 32-bit outputs into four standard normals.
//
// Counter convention (shared with the C ABI documentation):
//   key     = (seed lo, seed hi)
//   counter = (index / 4, chain, step lo, (step hi << 8) | (comp << 4) | tag)
// and normal j of a block belongs to index 4 * (index / 4) + j.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dm {

enum : uint32_t {
    kTagMode = 0u,
    kTagEuler = 1u,
    kTagMC = 2u,
    kTagWLC = 3u,
    kTagInit = 4u,    // jitter of the initial state (index = bead)
    kTagOrient = 5u,  // direction of an initial chain (index 0)
};

struct Block4 {
    uint32_t v[4];
};

// x ^ y ^ k in one VALU op on gfx950 (v_bitop3_b32, truth table 0x96).
__host__ __device__ __forceinline__ uint32_t xor3(uint32_t x, uint32_t y, uint32_t k)
{
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(x), "v"(y), "s"(k));
    return r;
#else
    return x ^ y ^ k;
#endif
}

__host__ __device__ __forceinline__ Block4 philox4x32_10(uint32_t c0, uint32_t c1,
                                                         uint32_t c2, uint32_t c3,
                                                         uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // full 32x32->64 products (one v_mad_u64_u32 each)
        const uint64_t pa = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t pb = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t a_lo = (uint32_t)pa, a_hi = (uint32_t)(pa >> 32);
        const uint32_t b_lo = (uint32_t)pb, b_hi = (uint32_t)(pb >> 32);
        const uint32_t n0 = xor3(b_hi, c1, k0);
        const uint32_t n2 = xor3(a_hi, c3, k1);
        c0 = n0;
        c1 = b_lo;
        c2 = n2;
        c3 = a_lo;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Block4 out;
    out.v[0] = c0;
    out.v[1] = c1;
    out.v[2] = c2;
    out.v[3] = c3;
    return out;
}

__host__ __device__ __forceinline__ Block4 noise_bits(uint64_t seed, uint32_t block,
                                                      uint32_t chain, int64_t step,
                                                      uint32_t comp, uint32_t tag)
{
    const uint64_t k = (uint64_t)step;
    return philox4x32_10(block, chain, (uint32_t)k,
                         ((uint32_t)(k >> 32) << 8) | (comp << 4) | tag,
                         (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Box-Muller pair `second` (0: words 0, 1; 1: words 2, 3) of a block in
// FP64: uniforms (x + 1/2) 2^-32, z = sqrt(-2 ln u_a) (cos, sin)(2 pi u_b).
__host__ __device__ __forceinline__ void normal_pair_f64(const Block4 &b, int second, double z[2])
{
    const double scale = 2.3283064365386962890625e-10;  // 2^-32
    const double two_pi = 6.283185307179586476925286766559;
    const double ua = ((double)b.v[2 * second] + 0.5) * scale;
    const double ub = ((double)b.v[2 * second + 1] + 0.5) * scale;
    const double ra = sqrt(-2.0 * log(ua));
    z[0] = ra * cos(two_pi * ub);
    z[1] = ra * sin(two_pi * ub);
}

// Four N(0,1) in FP64: the block's two Box-Muller pairs.
__host__ __device__ __forceinline__ void normals4_f64(const Block4 &b, double z[4])
{
    normal_pair_f64(b, 0, z);
    normal_pair_f64(b, 1, z + 2);
}

// Box-Muller radius factor that the FP32 form leaves to its callers:
// sqrt(-2 ln u) = sqrt(2 ln 2) sqrt(-log2 u).
constexpr double kNormalScale = 1.1774100225154747;  // sqrt(2 ln 2)

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)
// Four N(0,1) in FP32 from the same bits, divided by kNormalScale (the caller
// folds the factor into the coefficient it multiplies them by), with the
// hardware transcendentals.  Radius: the uniform (x + 1/2) 2^-32 as in FP64,
// from x rounded to 24 significant bits (never 0; 1 where x rounds to 2^32,
// which gives the normal 0), v_log_f32 (log2) and v_sqrt_f32 of its
// negation.  Angle: v_sin/v_cos_f32 take their argument in revolutions and
// are periodic in it, so the uniform enters as 1 + (x >> 9) 2^-23 in [1, 2),
// its 23 leading bits placed in a mantissa by one bit alignment (an angle
// within 2^-23 of a revolution of the FP64 one).
__device__ __forceinline__ void scaled_normals4_f32(const Block4 &b, float z[4])
{
    const float s32 = 2.3283064365386962890625e-10f;  // 2^-32
    const float u0 = __builtin_fmaf((float)b.v[0], s32, 0.5f * s32);
    const float u2 = __builtin_fmaf((float)b.v[2], s32, 0.5f * s32);
    // {0x7f, x} >> 9: the exponent of 1.0 above the top 23 bits of x
    const float u1 = __uint_as_float(__builtin_amdgcn_alignbit(0x7fu, b.v[1], 9u));
    const float u3 = __uint_as_float(__builtin_amdgcn_alignbit(0x7fu, b.v[3], 9u));
    const float ra = __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(u0));
    const float rb = __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(u2));
    z[0] = ra * __builtin_amdgcn_cosf(u1);
    z[1] = ra * __builtin_amdgcn_sinf(u1);
    z[2] = rb * __builtin_amdgcn_cosf(u3);
    z[3] = rb * __builtin_amdgcn_sinf(u3);
}
#endif

}  // namespace dm
