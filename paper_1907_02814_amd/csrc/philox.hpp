// philox.hpp -- Philox4x32-10 counter-based generator (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) and the
// draws of the step.  Counter = (x, cell, step low word, tag<<24 | step bits
// 32..55), key = (seed low, seed high): every random number of the method
// is a pure function of where it is used, so results do not depend on the
// launch schedule.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmc {

struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64-bit multiply gives both halves of each product
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// tags of the counter's last word
enum : uint32_t {
    kTagKeyE = 0x01, kTagKeyIE = 0x02, kTagKeyG = 0x03, kTagKeyIG = 0x04,
    kTagAccBr = 0x11, kTagSmpBr = 0x12, kTagHiBr = 0x13,
    kTagAccTr = 0x21, kTagSmpTr = 0x22, kTagHiTr = 0x23,
    kTagAccBh = 0x31, kTagSmpBh = 0x32, kTagHiBh = 0x33
};

struct Rng {
    uint32_t k0, k1, step_lo, step_hi;
    __device__ __forceinline__ U4 draw(uint32_t x, uint32_t cell, uint32_t tag) const {
        // The round keys are derived from (k0, k1) inside each draw: hoisted
        // out of a loop of draws they would be twenty live scalar registers,
        // more than a kernel with other uniform state keeps.
        uint32_t a = k0, b = k1;
        asm volatile("" : "+s"(a), "+s"(b));
        return philox4x32_10(x, cell, step_lo, (tag << 24) | (step_hi & 0xFFFFFFu), a, b);
    }
};

// uniform double in [0, 1) with 53 random bits
__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// The acceptance test of the pair whose numbers are keyed by x (eq:proba3):
// the upper 32 of U1's 53 bits are word (x >> 8) & 3 of the draw with the
// process's hi tag keyed by hi_group(x), which four pairs share; the lower
// 21 are the top bits of word 0 of the pair's own draw (acceptance tag),
// whose words 2 and 3 give U2.  A bound test needs only the shared word.
__device__ __forceinline__ uint32_t hi_group(uint32_t x) { return ((x >> 10) << 8) | (x & 255u); }

__device__ __forceinline__ uint32_t hi_word(const U4& h, uint32_t w) {
    return w == 0u ? h.x : (w == 1u ? h.y : (w == 2u ? h.z : h.w));
}

__device__ __forceinline__ void accept_uniforms(const Rng& rng, uint32_t x, uint32_t cell, uint32_t tag,
                                                uint32_t tag_hi, double& U1, double& U2) {
    const U4 h = rng.draw(hi_group(x), cell, tag_hi);
    const U4 r = rng.draw(x, cell, tag);
    U1 = ((double)hi_word(h, (x >> 8) & 3u) * 2097152.0 + (double)(r.x >> 11)) * (1.0 / 9007199254740992.0);
    U2 = u53(r.z, r.w);
}

}  // namespace cmc
