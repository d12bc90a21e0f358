// device_math.h -- counter-based random numbers and the logarithm used by the
// SSA kernels.  Device code for gfx950; compiled with -ffp-contract=off so
// every floating-point operation below is exactly one IEEE binary64 rounding.
#pragma once
#include "device_types.h"

namespace siminf {

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of
//   (x0, x1, x2, x3) -> (hi(B*x2) ^ x1 ^ k0, lo(B*x2), hi(A*x0) ^ x3 ^ k1, lo(A*x0))
// with A = 0xD2511F53, B = 0xCD9E8D57 and the key advanced by the Weyl
// increments (0x9E3779B9, 0xBB67AE85) before every round but the first.
struct Block4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ Block4 philox10(uint32_t k0, uint32_t k1, uint32_t x0, uint32_t x1,
                                           uint32_t x2, uint32_t x3) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)0xD2511F53u * x0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)pb;
        x3 = (uint32_t)pa;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {x0, x1, x2, x3};
}

// (0,1) uniform from 52 random bits k (hi word's 32 bits above lo word's top
// 20), centred in its cell: (k + 1/2) 2^-52, exact, never 0 or 1.  Computed
// as the double with exponent 0 and fraction k, 1 + k 2^-52, minus the
// largest double below 1, 1 - 2^-53: by Sterbenz's lemma the difference is
// exact, so this is the value above without an integer conversion.
__device__ __forceinline__ double open_uniform(uint32_t hi, uint32_t lo) {
    const uint32_t frac_lo = (hi << 20) | (lo >> 12);
    const uint32_t frac_hi = (hi >> 12) | 0x3ff00000u;
    const double one_plus = __longlong_as_double((long long)(((uint64_t)frac_hi << 32) | frac_lo));
    return one_plus - 0x1.fffffffffffffp-1;
}

// A constant for the addend of a fused multiply-add, in a scalar register
// pair at its point of use: otherwise the compiler keeps the series'
// coefficients in vector registers across the draw loop (20 of them) and adds
// a vector move before every multiply-add.  The empty statement emits no
// instruction.
__device__ __forceinline__ double in_sgpr(double c) {
    asm volatile("" : "+s"(c));
    return c;
}

// Natural log of a normal x in (0, 1]: x = m 2^e with m in (sqrt(1/2), sqrt(2)],
// ln m = 2 atanh(s), s = (m-1)/(m+1), as s * (2 + 2z/3 + ... + 2z^11/23),
// z = s^2, by Horner with one fused multiply-add (one rounding) per step;
// ln x = e ln2_hi + (e ln2_lo + ln m), both as fused multiply-adds (the
// first product is exact: ln2_hi has 32 trailing zero bits).
__device__ __forceinline__ double series_log(double x) {
    const uint64_t ix = (uint64_t)__double_as_longlong(x);
    int ex = (int)((ix >> 52) & 0x7ff) - 1023;
    double m = __longlong_as_double((long long)((ix & 0x000fffffffffffffull) | 0x3ff0000000000000ull));
    if (m > 0x1.6a09e667f3bcdp+0) {  // sqrt(2) rounded to binary64
        m = m * 0.5;
        ex = ex + 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    // coefficients 1/(2k+1), k = 11 .. 0, each the correctly rounded quotient
    double h = 1.0 / 23.0;
    h = __builtin_fma(h, z, in_sgpr(1.0 / 21.0));
    h = __builtin_fma(h, z, in_sgpr(1.0 / 19.0));
    h = __builtin_fma(h, z, in_sgpr(1.0 / 17.0));
    h = __builtin_fma(h, z, in_sgpr(1.0 / 15.0));
    h = __builtin_fma(h, z, in_sgpr(1.0 / 13.0));
    h = __builtin_fma(h, z, in_sgpr(1.0 / 11.0));
    h = __builtin_fma(h, z, in_sgpr(1.0 / 9.0));
    h = __builtin_fma(h, z, in_sgpr(1.0 / 7.0));
    h = __builtin_fma(h, z, in_sgpr(1.0 / 5.0));
    h = __builtin_fma(h, z, in_sgpr(1.0 / 3.0));
    h = __builtin_fma(h, z, 1.0);
    const double lnm = (s + s) * h;
    const double fe = (double)ex;
    return __builtin_fma(fe, 0x1.62e42feep-1, __builtin_fma(fe, 0x1.a39ef35793c76p-33, lnm));
}

// Sequential 32-bit words of the Philox blocks (b, 0, id, stream | 1<<24),
// b = 0, 1, ..., used to sample the individuals of one scheduled event.
struct EventWords {
    uint32_t k0, k1, id, tag, blk;
    Block4 cur;
    int left;
    __device__ __forceinline__ EventWords(uint64_t seed, uint32_t stream, uint32_t event_id)
        : k0((uint32_t)seed), k1((uint32_t)(seed >> 32)), id(event_id),
          tag((stream & 0xFFFFFFu) | (1u << 24)), blk(0), cur{0, 0, 0, 0}, left(0) {}
    __device__ __forceinline__ uint32_t next() {
        if (left == 0) {
            cur = philox10(k0, k1, blk, 0u, id, tag);
            blk += 1;
            left = 4;
        }
        const int used = 4 - left;
        left -= 1;
        return used == 0 ? cur.x : used == 1 ? cur.y : used == 2 ? cur.z : cur.w;
    }
    // uniform integer in [0, range), range >= 1 (Lemire, ACM TOMACS 2019):
    // take the high word of word*range, rejecting the biased low-word region.
    __device__ __forceinline__ uint32_t below(uint32_t range) {
        uint64_t prod = (uint64_t)next() * range;
        uint32_t low = (uint32_t)prod;
        if (low < range) {
            const uint32_t thresh = (0u - range) % range;
            while (low < thresh) {
                prod = (uint64_t)next() * range;
                low = (uint32_t)prod;
            }
        }
        return (uint32_t)(prod >> 32);
    }
};

}  // namespace siminf
