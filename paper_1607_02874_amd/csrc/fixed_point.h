// Fixed-point terms of the In(k) sums of the sputtering boundary, and the
// bits that drive the stochastic rounding of 16-bit stores.  Plain C++ that
// compiles for the GPU (included by the kernels) and for the host (so the
// encoders can be checked on a CPU).
//
// In(k) = sum_j f*_j(k - c_j) over the active links of interface node k
// (first line of the sputtering equations) is summed by the sweep with
// 64-bit integer atomics: each term x is rounded to a multiple of 2^-S and
// added as an integer, so the sum is the same in any order.  The rounding
// adds 1.5 * 2^52 to x * 2^S in one fused operation: for |x * 2^S| < 2^51
// the result's low mantissa bits hold round-to-nearest(x * 2^S), so its bit
// pattern is MAGIC_BITS + that integer and the reader subtracts b(k) *
// MAGIC_BITS from a sum of b(k) patterns.  A term outside that window (or not
// finite) becomes POISON instead, and any sum that holds 1 to 18 poisoned
// terms lies beyond +-2^55 once the magic patterns are removed, where the
// reader reports it as non-finite (checked for every count on the host).
#pragma once

#include <cmath>
#include <cstdint>
#include <cstring>

#if defined(__HIPCC__)
#define LBM_HD __host__ __device__ __forceinline__
#else
#define LBM_HD inline
#endif

namespace lbmfx {

constexpr double MAGIC = 6755399441055744.0;  // 1.5 * 2^52
constexpr unsigned long long MAGIC_BITS = 0x4338000000000000ull;
constexpr double TERM_LIMIT = 2251799813685248.0;  // 2^51
constexpr unsigned long long POISON = 0x7ff8000000000000ull;  // quiet-NaN bits
constexpr long long SUM_LIMIT = 1ll << 55;

LBM_HD unsigned long long dbits(double v) {
    unsigned long long u;
    std::memcpy(&u, &v, sizeof u);
    return u;
}

// Pattern of one term x at scale 2^S (scale = 2^S exactly).
LBM_HD unsigned long long term(double x, double scale) {
    return std::fabs(x * scale) < TERM_LIMIT ? dbits(std::fma(x, scale, MAGIC)) : POISON;
}

// A sum of patterns with the magic offsets removed, read back as 2^S times
// the sum of the terms; false when a poisoned term (or an overflow) put it
// out of range.
LBM_HD bool sum_in_range(long long fixed) { return fixed <= SUM_LIMIT && fixed >= -SUM_LIMIT; }

// ---------------------------------------------------- stochastic rounding --
// gfx950's stochastic-rounding conversions (FP32 -> FP16 / BF16) add the top
// bits of a 32-bit word to the discarded mantissa bits (13 for FP16, 16 for
// BF16) and truncate, rounding the magnitude; the word 0x80000000 therefore
// rounds to nearest (ties away from zero), and a uniformly random word rounds
// up with probability equal to the discarded fraction (unbiased).
constexpr uint32_t ROUND_NEAREST_BITS = 0x80000000u;
constexpr uint32_t WEYL = 0x9e3779b9u;  // odd step between the words of one node

// 32-bit integer hash of the xorshift-multiply family (constants from
// C. Wellons' hash-prospector search, "lowbias32").
LBM_HD uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Per-step key of the rounding words: a function of the step and the seed,
// so runs are reproducible and no two steps share words.  `salt` separates
// the population stores (0) from the emission stores (1).
LBM_HD uint32_t round_key(uint32_t step, uint64_t seed, uint32_t salt) {
    return mix32(mix32(step * WEYL + salt) ^ uint32_t(seed)) ^ uint32_t(seed >> 32);
}

// The words of one node (or interface node) n: word t of the node is
// base + t * step, base = mix32(n ^ key).  With step = 0 and base =
// ROUND_NEAREST_BITS every word rounds to nearest.
struct RoundWords {
    uint32_t base, step;
    LBM_HD uint32_t at(int t) const { return base + uint32_t(t) * step; }
};
LBM_HD RoundWords round_words(bool stochastic, uint32_t key, uint32_t n) {
    RoundWords r;
    r.base = stochastic ? mix32(n ^ key) : ROUND_NEAREST_BITS;
    r.step = stochastic ? WEYL : 0u;
    return r;
}

}  // namespace lbmfx
