// dq_fastdiv.hpp - unsigned 32-bit division by a divisor fixed for a launch.
//
// A multiply-high and two shifts (the round-up method of Granlund and
// Montgomery, "Division by invariant integers using multiplication", 1994).
// With l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1 (which fits in
// 32 bits),
//     n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0),  t = mulhi(m, n),
// exactly, for every 32-bit n and every divisor d >= 1. The divisor's
// constants are made on the host; the division runs on either side.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dq {

struct FastDiv {
    uint32_t d, m, s1, s2;
    __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
        const uint32_t t = (uint32_t)(((uint64_t)m * n) >> 32);
        return (t + ((n - t) >> s1)) >> s2;
    }
};

inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < (unsigned long long)d) ++l;
    FastDiv f;
    f.d = d;
    f.m = (uint32_t)((((unsigned __int128)1 << 32) * ((1ull << l) - d)) / d + 1);
    f.s1 = l < 1 ? l : 1u;
    f.s2 = l > 1 ? l - 1 : 0u;
    return f;
}

}  // namespace dq
