// exact_acc.h -- exact summation of binary64 terms on the device.
//
// Every coupling, field and effective field of an instance is an integer
// multiple of 2^b0, where b0 is the lowest set bit over all nonzero inputs
// (effective fields are correctly rounded sums of such terms, so they are too).
// A sum of up to 2^40 such terms, each below 2^top, is therefore an integer
// that fits 256 bits once top - b0 + 41 <= 255.  Terms are added exactly into
// two unsigned 256-bit magnitudes (positive and negative parts); the exact
// result is rounded once to binary64, round to nearest even.  Results do not
// depend on the order of the additions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hqa {

struct Acc256 {
    uint64_t p[4];
    uint64_t n[4];
};

__device__ __forceinline__ void acc_zero(Acc256 &a) {
#pragma unroll
    for (int k = 0; k < 4; k++) { a.p[k] = 0; a.n[k] = 0; }
}

__device__ __forceinline__ void add256(uint64_t *a, const uint64_t *b) {
    uint64_t c = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        uint64_t t = a[k] + b[k];
        uint64_t c1 = t < a[k];
        uint64_t t2 = t + c;
        uint64_t c2 = t2 < t;
        a[k] = t2;
        c = c1 | c2;
    }
}

// Add the binary64 value t (a multiple of 2^b0, |t| < 2^(b0+210)) exactly.
__device__ __forceinline__ void acc_add(Acc256 &a, double t, int b0) {
    if (t == 0.0) return;
    uint64_t bits = (uint64_t)__double_as_longlong(t);
    int E = (int)((bits >> 52) & 0x7ff);
    uint64_t m = bits & 0xfffffffffffffull;
    int e2;  // t = +-m * 2^e2
    if (E == 0) e2 = -1074;
    else { m |= 1ull << 52; e2 = E - 1075; }
    // drop trailing zero bits so that e2 is the exponent of the lowest set bit (>= b0)
    int tz = __ffsll((long long)m) - 1;
    m >>= tz;
    e2 += tz;
    const int s = e2 - b0;
    // limb k holds bits [64 k, 64 k + 64) of m << s; each limb is formed from its own
    // shift (no store at a run-time index, which would put the array in memory)
    uint64_t add[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int sh = s - 64 * k;
        add[k] = (sh >= 0 && sh < 64) ? (m << sh) : (sh < 0 && sh > -64) ? (m >> -sh) : 0ull;
    }
    // both magnitudes take an add, one of them of zeros: no branch for the compiler to
    // merge into an array chosen at run time, so both stay in registers
    const uint64_t neg = 0ull - (bits >> 63);
    uint64_t ap[4], an[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        ap[k] = add[k] & ~neg;
        an[k] = add[k] & neg;
    }
    add256(a.p, ap);
    add256(a.n, an);
}

__device__ __forceinline__ void acc_merge(Acc256 &a, const Acc256 &b) {
    add256(a.p, b.p);
    add256(a.n, b.n);
}

// Wavefront-wide merge by butterfly shuffles; every lane ends with the total.
__device__ __forceinline__ void acc_wave_allreduce(Acc256 &a) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        Acc256 b;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            b.p[k] = (uint64_t)__shfl_xor((long long)a.p[k], off, 64);
            b.n[k] = (uint64_t)__shfl_xor((long long)a.n[k], off, 64);
        }
        acc_merge(a, b);
    }
}

// Correctly rounded binary64 value of (p - n) * 2^b0.
__device__ __forceinline__ double acc_round(const Acc256 &a, int b0) {
    uint64_t d[4];
    int neg = 0;
    // compare magnitudes from the top limb
    int cmp = 0;
    for (int k = 3; k >= 0 && cmp == 0; k--) {
        if (a.p[k] > a.n[k]) cmp = 1;
        else if (a.p[k] < a.n[k]) cmp = -1;
    }
    if (cmp == 0) return 0.0;
    const uint64_t *x = a.p, *y = a.n;
    if (cmp < 0) { x = a.n; y = a.p; neg = 1; }
    uint64_t br = 0;
    for (int k = 0; k < 4; k++) {
        uint64_t t = x[k] - y[k];
        uint64_t b1 = x[k] < y[k];
        uint64_t t2 = t - br;
        uint64_t b2 = t < br;
        d[k] = t2;
        br = b1 | b2;
    }
    int top = -1;
    for (int k = 3; k >= 0; k--)
        if (d[k]) { top = 64 * k + 63 - __clzll((long long)d[k]); break; }
    double r;
    if (top <= 52) {
        r = ldexp((double)d[0], b0);
    } else {
        int sh = top - 52;  // drop sh low bits
        // mantissa = bits [sh, sh+52]
        int L = sh >> 6, o = sh & 63;
        uint64_t mant = d[L] >> o;
        if (o && L + 1 < 4) mant |= d[L + 1] << (64 - o);
        mant &= (1ull << 53) - 1;
        // round bit = bit sh-1, sticky = any bit below sh-1
        int rb = sh - 1;
        uint64_t round = (d[rb >> 6] >> (rb & 63)) & 1ull;
        uint64_t sticky = 0;
        for (int k = 0; k < (rb >> 6); k++) sticky |= d[k];
        sticky |= d[rb >> 6] & ((1ull << (rb & 63)) - 1ull);
        if (round && (sticky || (mant & 1ull))) {
            mant += 1;
            if (mant == (1ull << 53)) { mant >>= 1; sh += 1; }
        }
        r = ldexp((double)mant, b0 + sh);
    }
    return neg ? -r : r;
}

}  // namespace hqa
