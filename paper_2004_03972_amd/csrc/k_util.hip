// k_util.hip -- schedule table, instance ingest (validation, storage conversion),
// initial state and state import/export.
#include <math.h>

#include <algorithm>

#include "hqa_internal.h"

namespace hqa {

// ---------------------------------------------------------------------------
// Schedule (Methods, "Scheduling functions for MD"), tabulated on the half-step
// grid tau_k = k/(2T) so that integer step m sits at k = 2m and m+1/2 at 2m+1.
// binary64 with the operation order
//   alpha = a_f * ((tau + rho1*(1-tau)) + rho2*(tau*(tau-1))),
// and a binary32 copy for the FP32 paths.
// ---------------------------------------------------------------------------
__global__ void k_schedule(Schedule64 s, double *a64, double *b64, float *a32, float *b32) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > 2 * s.T) return;
    double tau = s.frozen ? s.tau_frozen : (double)k / (double)(2 * s.T);
    double om = 1.0 - tau;
    double q = tau * (tau - 1.0);
    double a = s.prm[0] * ((tau + s.prm[1] * om) + s.prm[2] * q);
    double b = s.prm[3] * ((tau + s.prm[4] * om) + s.prm[5] * q);
    a64[k] = a;
    b64[k] = b;
    a32[k] = (float)a;
    b32[k] = (float)b;
}

hipError_t launch_schedule(const Schedule64 &s, double *a64, double *b64, float *a32, float *b32,
                           hipStream_t st) {
    int64_t n = 2 * s.T + 1;
    k_schedule<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(s, a64, b64, a32, b32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ingest checks.  stats[0] = lowest set-bit exponent, stats[1] = highest bit
// exponent over nonzero |J|, |h|; stats[2] = 1 while every value is an integer.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void value_stats(double v, int &lsb, int &msb, int &integral) {
    if (v == 0.0) return;
    uint64_t bits = (uint64_t)__double_as_longlong(v);
    int E = (int)((bits >> 52) & 0x7ff);
    uint64_t m = bits & 0xfffffffffffffull;
    int e2;
    if (E == 0) e2 = -1074;
    else { m |= 1ull << 52; e2 = E - 1075; }
    int lo = e2 + __ffsll((long long)m) - 1;
    int hi = e2 + 63 - __clzll((long long)m);
    lsb = min(lsb, lo);
    msb = max(msb, hi);
    if (v != floor(v)) integral = 0;
}

__device__ __forceinline__ void stats_flush(int lsb, int msb, int integral, int32_t *stats) {
    for (int off = 32; off >= 1; off >>= 1) {
        lsb = min(lsb, __shfl_xor(lsb, off, 64));
        msb = max(msb, __shfl_xor(msb, off, 64));
        integral &= __shfl_xor(integral, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&stats[0], lsb);
        atomicMax(&stats[1], msb);
        if (!integral) atomicAnd(&stats[2], 0);
    }
}

__global__ void k_validate_dense(const double *J, const double *h, int N, int32_t *err,
                                 int32_t *stats) {
    int lsb = 1 << 20, msb = -(1 << 20), integral = 1, e = 0;
    int64_t total = (int64_t)N * N;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(t / N), j = (int)(t % N);
        double v = J[t];
        if (!isfinite(v)) e |= ERR_NOTFINITE_IN;
        if (i == j && v != 0.0) e |= ERR_DIAG;
        if (j > i && v != J[(int64_t)j * N + i]) e |= ERR_ASYM;
        value_stats(v, lsb, msb, integral);
    }
    if (h) {
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N;
             t += (int64_t)gridDim.x * blockDim.x) {
            if (!isfinite(h[t])) e |= ERR_NOTFINITE_IN;
            value_stats(h[t], lsb, msb, integral);
        }
    }
    if (e) atomicOr(err, e);
    stats_flush(lsb, msb, integral, stats);
}

hipError_t launch_validate_dense(const double *J, const double *h, int N, int32_t *err,
                                 int32_t *stats, hipStream_t st) {
    int64_t total = (int64_t)N * N;
    int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    k_validate_dense<<<blocks, 256, 0, st>>>(J, h, N, err, stats);
    return hipGetLastError();
}

__device__ __forceinline__ int csr_find(const int32_t *rp, const int32_t *ci, int row, int col) {
    int lo = rp[row], hi = rp[row + 1];
    while (lo < hi) {
        int mid = lo + ((hi - lo) >> 1);
        if (ci[mid] < col) lo = mid + 1;
        else hi = mid;
    }
    return (lo < rp[row + 1] && ci[lo] == col) ? lo : -1;
}

// One thread per row: ordering, range, diagonal, symmetry (binary search for the
// transposed entry), finiteness, exponent statistics.
__global__ void k_validate_csr(const int32_t *rp, const int32_t *ci, const double *v,
                               const double *h, int N, int32_t *err, int32_t *stats) {
    int lsb = 1 << 20, msb = -(1 << 20), integral = 1, e = 0;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        int b = rp[i], en = rp[i + 1];
        if (b > en) e |= ERR_CSR_ORDER;
        int prev = -1;
        for (int k = b; k < en && !(e & ERR_CSR_ORDER); k++) {
            int j = ci[k];
            if (j <= prev || j < 0 || j >= N) { e |= ERR_CSR_ORDER; break; }
            prev = j;
            double x = v[k];
            if (!isfinite(x)) e |= ERR_NOTFINITE_IN;
            if (j == i && x != 0.0) e |= ERR_DIAG;
            int t = csr_find(rp, ci, j, i);
            if (t < 0 ? x != 0.0 : v[t] != x) e |= ERR_ASYM;
            value_stats(x, lsb, msb, integral);
        }
        if (h) {
            if (!isfinite(h[i])) e |= ERR_NOTFINITE_IN;
            value_stats(h[i], lsb, msb, integral);
        }
    }
    if (e) atomicOr(err, e);
    stats_flush(lsb, msb, integral, stats);
}

hipError_t launch_validate_csr(const int32_t *rp, const int32_t *ci, const double *v,
                               const double *h, int N, int32_t *err, int32_t *stats,
                               hipStream_t st) {
    k_validate_csr<<<(N + 255) / 256, 256, 0, st>>>(rp, ci, v, h, N, err, stats);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Storage conversion for the fast paths.
// ---------------------------------------------------------------------------
// binary64 -> bfloat16, round to nearest even: round to odd into binary32 first
// (24 >= 8 + 2 bits, so the second rounding is then correct), then RNE to 16 bits.
__device__ __forceinline__ uint16_t to_bf16_bits(double v) {
    float f = (float)v;
    if (fabs((double)f) > fabs(v)) f = nextafterf(f, 0.0f);
    uint32_t u = __float_as_uint(f);
    if ((double)f != v) u |= 1u;
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

__device__ __forceinline__ double from_bf16_bits(uint16_t b) {
    return (double)__uint_as_float((uint32_t)b << 16);
}

// binary64 -> FP8 e4m3 (OCP: bias 7, no infinities, max 448), round to nearest even,
// saturating.  Subnormal codes encode m * 2^-9.
__device__ __forceinline__ uint8_t to_e4m3(double v) {
    uint8_t s = signbit(v) ? 0x80 : 0;
    double a = fabs(v);
    if (a == 0.0) return s;
    if (a >= 464.0) return s | 0x7e;
    int e = ilogb(a);
    if (e < -6) {
        double m = rint(ldexp(a, 9));
        return s | (uint8_t)m;           // m == 8 is the smallest normal code 0x08
    }
    double mi = rint((ldexp(a, -e) - 1.0) * 8.0);
    if (mi == 8.0) { mi = 0.0; e += 1; }
    if (e > 8) return s | 0x7e;
    return s | (uint8_t)(((e + 7) << 3) | (int)mi);
}

__device__ __forceinline__ double from_e4m3(uint8_t c) {
    int eb = (c >> 3) & 15, m = c & 7;
    double a = eb == 0 ? ldexp((double)m, -9) : ldexp(1.0 + m / 8.0, eb - 7);
    return (c & 0x80) ? -a : a;
}

__global__ void k_convert_dense(const double *J, int N, int Np, int jt, void *out, int32_t *err) {
    int64_t total = (int64_t)Np * Np;
    int e = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(t / Np), j = (int)(t % Np);
        double v = (i < N && j < N) ? J[(int64_t)i * N + j] : 0.0;
        if (jt == JT_F32) {
            float f = (float)v;
            ((float *)out)[t] = f;
            if ((double)f != v) e |= ERR_INEXACT;
        } else if (jt == JT_BF16) {
            uint16_t b = to_bf16_bits(v);
            ((uint16_t *)out)[t] = b;
            if (from_bf16_bits(b) != v) e |= ERR_INEXACT;
        } else {
            uint8_t c = to_e4m3(v);
            ((uint8_t *)out)[t] = c;
            if (from_e4m3(c) != v) e |= ERR_INEXACT;
        }
    }
    if (e) atomicOr(err, e);
}

hipError_t launch_convert_dense(const double *J, int N, int Np, JType jt, void *out,
                                int32_t *err, hipStream_t st) {
    int64_t total = (int64_t)Np * Np;
    int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
    k_convert_dense<<<blocks, 256, 0, st>>>(J, N, Np, (int)jt, out, err);
    return hipGetLastError();
}

__global__ void k_convert_csr(const double *v, int64_t nnz, float *out, int32_t *err) {
    int e = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnz;
         t += (int64_t)gridDim.x * blockDim.x) {
        float f = (float)v[t];
        out[t] = f;
        if ((double)f != v[t]) e |= ERR_INEXACT;
    }
    if (e) atomicOr(err, e);
}

hipError_t launch_convert_csr(const double *v, int64_t nnz, float *out, int32_t *err,
                              hipStream_t st) {
    int blocks = (int)std::min<int64_t>((nnz + 255) / 256, 8192);
    if (blocks < 1) blocks = 1;
    k_convert_csr<<<blocks, 256, 0, st>>>(v, nnz, out, err);
    return hipGetLastError();
}

__global__ void k_convert_h(const double *h, int N, float *out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) out[i] = (float)h[i];
}

hipError_t launch_convert_h(const double *h, int N, float *out, hipStream_t st) {
    k_convert_h<<<(N + 255) / 256, 256, 0, st>>>(h, N, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Initial state (Results, "Molecular dynamics for flux variables"): phi(0) = 0,
// p(0) = +-1 from the SplitMix64 output function (Steele, Lea, Flood 2014) at
// counter z = seed + (r*N + i + 1) * 0x9E3779B97F4A7C15, top bit set = -1;
// explicit arrays (binary64, [R][N]) override either.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t ctr) {
    uint64_t z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct InitArgs {
    int N, R, ld;
    int smaj, f64;
    uint64_t seed;
    const double *p0, *phi0;
    double *phi64, *p64, *S64;
    float *phi32, *p32, *S32;
    bf16 *phib;
};

__global__ void k_init_state(InitArgs a) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.N * a.R) return;
    int r = (int)(t / a.N), i = (int)(t % a.N);
    double p = a.p0 ? a.p0[t] : ((splitmix64_at(a.seed, (uint64_t)t) >> 63) ? -1.0 : 1.0);
    double x = a.phi0 ? a.phi0[t] : 0.0;
    if (a.f64) {
        a.phi64[t] = x;
        a.p64[t] = p;
        a.S64[t] = 0.0;
    } else {
        int64_t k = a.smaj ? (int64_t)i * a.ld + r : (int64_t)r * a.ld + i;
        a.phi32[k] = (float)x;
        a.p32[k] = (float)p;
        a.S32[k] = 0.0f;
        if (a.phib) a.phib[k] = (bf16)(float)x;
    }
}

hipError_t launch_init_state(const Instance &I, int R, int prec, uint64_t seed,
                             const double *p0, const double *phi0, hipStream_t st) {
    InitArgs a;
    a.N = I.N; a.R = R; a.ld = I.ld; a.smaj = I.smaj; a.f64 = prec == HQA_PREC_F64_REF;
    a.seed = seed; a.p0 = p0; a.phi0 = phi0;
    a.phi64 = I.phi64[I.cur]; a.p64 = I.p64; a.S64 = I.S64;
    a.phi32 = I.phi32[I.cur]; a.p32 = I.p32; a.S32 = I.S32;
    a.phib = I.phib[I.cur];
    int64_t n = (int64_t)I.N * R;
    k_init_state<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// State export / import, always as binary64 [R][N].
// ---------------------------------------------------------------------------
struct XArgs {
    int N, R, ld, smaj, f64, what, import, W;
    double *x64;
    float *x32;
    bf16 *xb;
    double *dst;
};

__global__ void k_export(XArgs a) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.N * a.R) return;
    int r = (int)(t / a.N), i = (int)(t % a.N);
    if (a.f64) {
        if (a.import) a.x64[t] = a.dst[t];
        else a.dst[t] = a.what == HQA_STATE_PHIBAR ? a.x64[t] / (double)a.W : a.x64[t];
    } else {
        int64_t k = a.smaj ? (int64_t)i * a.ld + r : (int64_t)r * a.ld + i;
        if (a.import) {
            float f = (float)a.dst[t];
            a.x32[k] = f;
            if (a.xb) a.xb[k] = (bf16)f;
        } else {
            a.dst[t] = a.what == HQA_STATE_PHIBAR ? (double)(a.x32[k] / (float)a.W)
                                                  : (double)a.x32[k];
        }
    }
}

hipError_t launch_export(const Instance &I, int R, int prec, int what, double *dst, int import,
                         int W, hipStream_t st) {
    XArgs a;
    a.N = I.N; a.R = R; a.ld = I.ld; a.smaj = I.smaj; a.f64 = prec == HQA_PREC_F64_REF;
    a.what = what; a.import = import; a.dst = dst; a.W = W;
    a.xb = nullptr;
    if (what == HQA_STATE_PHI) {
        a.x64 = I.phi64[I.cur]; a.x32 = I.phi32[I.cur]; a.xb = I.phib[I.cur];
    } else if (what == HQA_STATE_P) {
        a.x64 = I.p64; a.x32 = I.p32;
    } else {
        a.x64 = I.S64; a.x32 = I.S32;
    }
    int64_t n = (int64_t)I.N * R;
    k_export<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace hqa

namespace hqa {

__global__ void k_layout_to_f64(int N, int R, int ld, int smaj, const float *src, double *dst) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)N * R) return;
    int r = (int)(t / N), i = (int)(t % N);
    dst[t] = (double)src[smaj ? (int64_t)i * ld + r : (int64_t)r * ld + i];
}

hipError_t launch_layout_to_f64(int N, int R, int ld, int smaj, const float *src, double *dst,
                                hipStream_t st) {
    int64_t n = (int64_t)N * R;
    k_layout_to_f64<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(N, R, ld, smaj, src, dst);
    return hipGetLastError();
}

}  // namespace hqa
