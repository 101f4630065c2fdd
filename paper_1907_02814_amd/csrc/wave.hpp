// wave.hpp -- sums over the 64 lanes of a wavefront with DPP row moves and
// lane reads (no LDS), the same value in every lane.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmc {

// A lane's value after a DPP move of the wavefront (both halves of a double)
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), kCtrl, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double lane_f64(double v, int lane) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wavefront (all active), the same value in every
// lane: a butterfly over lane distances 1, 2, 4, 8 inside each row of 16
// lanes (DPP quad permutations and mirrors, each lane adding its partner's
// partial, which a commutative add makes equal on both sides), then the four
// row sums as (r0 + r1) + (r2 + r3).
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);   // row_half_mirror: the other quad of 8
    v += dpp_f64<0x140>(v);   // row_mirror: the other 8 of 16
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// The same for 32-bit integers (exact in any order)
__device__ __forceinline__ int wave_sum_i32(int v) {
    v += __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
    v += __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
    v += __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);
    v += __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false);
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
           __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

}  // namespace cmc
