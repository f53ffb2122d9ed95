// Independent Philox4x32-10 for pinning the oracle: calls AMD's open-source
// rocRAND engine (header-only, host-callable).  With offset 4k and
// subsequence s, rocRAND's first block is Philox(counter = (k lo, k hi,
// s lo, s hi), key = (seed lo, seed hi)).
#include <rocrand/rocrand_philox4x32_10.h>
#include <stdint.h>

extern "C" void rr_philox_block(uint64_t seed, uint64_t k, uint64_t s, uint32_t out[4])
{
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, s, 4ull * k, &st);
    uint4 v = rocrand4(&st);
    out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
}
