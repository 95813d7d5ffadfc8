// Order-independent accumulation for the deterministic mode: each value is added as a
// signed 128-bit fixed-point number (64 integer and 64 fraction bits, in units of a power
// of two `scale` chosen by the host above any single term), held in two 64-bit words per
// entry (low word at 2 i, high word at 2 i + 1).  Integer addition is associative, so the
// total does not depend on the order in which lanes, waves or workgroups add: the low
// word wraps floor(sum of low parts / 2^64) times whatever the order, and each wrap is
// carried into the high word by the adder that caused it.  A term is truncated to
// 2^-64 scale (about 5e-20 of the largest charge weight); the read-out rounds once.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fepic {

__device__ __forceinline__ void fix_add(unsigned long long* __restrict__ acc, int64_t i, double v, double inv_scale) {
    if (v == 0.0) return;
    const double x = v * inv_scale;   // exact: inv_scale is a power of two
    const double f = floor(x);
    const unsigned long long hi = (unsigned long long)(long long)f;
    const unsigned long long lo = (unsigned long long)((x - f) * 18446744073709551616.0);   // x - f in [0, 1)
    unsigned long long* p = acc + 2 * i;
    const unsigned long long old = atomicAdd(p, lo);
    atomicAdd(p + 1, hi + ((old + lo < old) ? 1ull : 0ull));
}

// The accumulated value times scale, rounded once: the magnitude of the 128-bit number
// converted, then the sign applied (so small negative totals keep their digits).
__device__ __forceinline__ double fix_value(unsigned long long lo, unsigned long long hi, double scale) {
    const bool neg = (long long)hi < 0;
    if (neg) {   // two's complement negation of (hi, lo)
        lo = ~lo + 1ull;
        hi = ~hi + (lo == 0ull ? 1ull : 0ull);
    }
    const double m = ((double)hi + (double)lo * 5.421010862427522e-20) * scale;   // 2^-64
    return neg ? -m : m;
}

}  // namespace fepic
