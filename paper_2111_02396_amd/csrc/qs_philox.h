// Counter-based generator used by the host planner and the sampling kernels:
// Philox4x32 with ten rounds (Salmon, Moraes, Dror, Shaw, SC'11).  A round
// forms the two 32x32->64-bit products of counter words 0 and 2 with the
// multipliers below, then builds the next counter from the high halves
// xor-ed with words 1/3 and the round key, and the low halves; the key is
// bumped by the two Weyl increments before every round after the first.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qs {

struct PhiloxWords {
    uint32_t w[4];
};

__host__ __device__ __forceinline__ void philox_mul(uint32_t a, uint32_t b, uint32_t &hi,
                                                    uint32_t &lo) {
    const uint64_t prod = static_cast<uint64_t>(a) * static_cast<uint64_t>(b);
    hi = static_cast<uint32_t>(prod >> 32);
    lo = static_cast<uint32_t>(prod);
}

__host__ __device__ __forceinline__ PhiloxWords philox4x32_10(uint32_t c0, uint32_t c1,
                                                              uint32_t c2, uint32_t c3,
                                                              uint32_t key0, uint32_t key1) {
    constexpr uint32_t kMulA = 0xD2511F53u;
    constexpr uint32_t kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u;
    constexpr uint32_t kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hiA, loA, hiB, loB;
        philox_mul(kMulA, c0, hiA, loA);
        philox_mul(kMulB, c2, hiB, loB);
        const uint32_t n0 = hiB ^ c1 ^ key0;
        const uint32_t n2 = hiA ^ c3 ^ key1;
        c0 = n0;
        c1 = loB;
        c2 = n2;
        c3 = loA;
        key0 += kWeylA;
        key1 += kWeylB;
    }
    PhiloxWords out;
    out.w[0] = c0;
    out.w[1] = c1;
    out.w[2] = c2;
    out.w[3] = c3;
    return out;
}

// 53-bit uniform in [0, 1) from output words 1 (high) and 0 (low).
__host__ __device__ __forceinline__ double unit_double(uint32_t lo, uint32_t hi) {
    const uint64_t bits = (static_cast<uint64_t>(hi) << 21) | (static_cast<uint64_t>(lo) >> 11);
    return static_cast<double>(bits) * 0x1.0p-53;
}

enum : uint32_t { kStreamChannel = 0, kStreamMeasure = 1, kStreamReadout = 2 };

__host__ __device__ __forceinline__ double philox_uniform(uint64_t seed, uint32_t index,
                                                          uint32_t traj, uint32_t circ,
                                                          uint32_t stream) {
    const PhiloxWords o = philox4x32_10(index, traj, circ, stream,
                                        static_cast<uint32_t>(seed),
                                        static_cast<uint32_t>(seed >> 32));
    return unit_double(o.w[0], o.w[1]);
}

}  // namespace qs
