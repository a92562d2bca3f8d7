// k_readout.hip -- frozen/ambivalent sort, reduced problem, exact enumeration,
// merge and exact Ising energies.
#include <math.h>

#include "exact_acc.h"
#include <cstring>
#include <vector>

#include "hqa_internal.h"

namespace hqa {

// Position of spin i of replica r in the state arrays.
__device__ __forceinline__ int64_t sidx(int smaj, int ld, int r, int i) {
    return smaj ? (int64_t)i * ld + r : (int64_t)r * ld + i;
}

// ---------------------------------------------------------------------------
// Sort (Results, "Sorting frozen and ambivalent variables"): per replica the n
// spins with the smallest |phibar| (ties: lower index) are ambivalent, listed in
// ascending index; s_i = sgn(phibar_i), sgn(0) = +1.  phibar = S / W in the
// state's precision.  One workgroup (256 threads) per replica: an MSD radix
// select over the bit patterns of |phibar| (non-negative floats order as their
// bit patterns) finds the n-th smallest key K*, then an index-ordered scan takes
// every key < K* and the lowest-index keys == K* up to n.
// ---------------------------------------------------------------------------
struct SelArgs {
    int N, R, ld, smaj, f64, W, n;
    const double *S64;
    const float *S32;
    int32_t *amb;
    int8_t *spins;
    const float *keys;   // if set: keys [R][N] (non-negative) and spins already written
};

__device__ __forceinline__ uint64_t sel_key(const SelArgs &a, int r, int i, int8_t *sgn) {
    if (a.keys) return (uint64_t)__float_as_uint(a.keys[(int64_t)r * a.N + i]);
    if (a.f64) {
        double pb = a.S64[(int64_t)r * a.N + i] / (double)a.W;
        if (sgn) *sgn = pb < 0.0 ? -1 : 1;
        return (uint64_t)__double_as_longlong(fabs(pb));
    }
    float pb = a.S32[sidx(a.smaj, a.ld, r, i)] / (float)a.W;
    if (sgn) *sgn = pb < 0.0f ? -1 : 1;
    return (uint64_t)__float_as_uint(fabsf(pb));
}

__device__ __forceinline__ void select_body(const SelArgs &a, const int bx_) {
    __shared__ uint32_t hist[256];
    __shared__ uint64_t s_prefix;
    __shared__ int s_k;
    __shared__ int wsum[2][4];
    const int r = bx_, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // spins
    for (int i = tid; i < a.N && !a.keys; i += 256) {
        int8_t s;
        sel_key(a, r, i, &s);
        a.spins[(int64_t)r * a.N + i] = s;
    }
    if (a.n == 0) return;
    uint64_t prefix = 0, pmask = 0;
    if (tid == 0) s_k = a.n;
    const int passes = a.f64 ? 8 : 4;
    for (int ps = passes - 1; ps >= 0; ps--) {
        hist[tid] = 0;
        __syncthreads();
        for (int i = tid; i < a.N; i += 256) {
            uint64_t k = sel_key(a, r, i, nullptr);
            if ((k & pmask) == prefix) atomicAdd(&hist[(k >> (8 * ps)) & 255], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            int k = s_k;
            int b = 0;
            while (b < 255 && (int)hist[b] < k) { k -= hist[b]; b++; }
            s_k = k;
            s_prefix = prefix | ((uint64_t)b << (8 * ps));
        }
        __syncthreads();
        prefix = s_prefix;
        pmask |= (uint64_t)255 << (8 * ps);
    }
    const uint64_t kstar = prefix;
    const int m = s_k;  // how many keys equal to K* are taken
    int eq_run = 0, out_run = 0;
    for (int c0 = 0; c0 < a.N; c0 += 256) {
        int i = c0 + tid;
        uint64_t k = i < a.N ? sel_key(a, r, i, nullptr) : ~0ull;
        bool eq = i < a.N && k == kstar;
        bool lt = i < a.N && k < kstar;
        uint64_t beq = __ballot(eq);
        uint64_t lanemask = lane ? (~0ull >> (64 - lane)) : 0ull;
        int eq_before_w = __popcll(beq & lanemask);
        if (lane == 0) wsum[0][w] = __popcll(beq);
        __syncthreads();
        int eq_before = eq_run + eq_before_w;
        for (int v = 0; v < w; v++) eq_before += wsum[0][v];
        bool sel = lt || (eq && eq_before < m);
        uint64_t bsel = __ballot(sel);
        if (lane == 0) wsum[1][w] = __popcll(bsel);
        __syncthreads();
        int pos = out_run + __popcll(bsel & lanemask);
        for (int v = 0; v < w; v++) pos += wsum[1][v];
        if (sel && pos < a.n) a.amb[(int64_t)r * a.n + pos] = i;
        for (int v = 0; v < 4; v++) { eq_run += wsum[0][v]; out_run += wsum[1][v]; }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_select(SelArgs a) { select_body(a, blockIdx.x); }

// Many instances in one launch: instance blockIdx.y, its own block count nb[y].
__global__ __launch_bounds__(256) void k_select_many(const SelArgs *as, const int *nb) {
    const int k = blockIdx.y;
    if ((int)blockIdx.x >= nb[k]) return;
    const SelArgs a = as[k];
    select_body(a, blockIdx.x);
}

hipError_t launch_select(const Instance &I, int R, int prec, int W, int n, int32_t *amb,
                         int8_t *spins, hipStream_t st) {
    SelArgs a;
    a.N = I.N; a.R = R; a.ld = I.ld; a.smaj = I.smaj; a.f64 = prec == HQA_PREC_F64_REF;
    a.W = W; a.n = n; a.S64 = I.S64; a.S32 = I.S32; a.amb = amb; a.spins = spins;
    a.keys = nullptr;
    k_select<<<R, 256, 0, st>>>(a);
    return hipGetLastError();
}

// Selection on explicit keys (ascending, ties to the lower index); spins untouched.
hipError_t launch_select_keys(int N, int R, const float *keys, int n, int32_t *amb,
                              int8_t *spins, hipStream_t st) {
    SelArgs a;
    a.N = N; a.R = R; a.ld = N; a.smaj = 0; a.f64 = 0; a.W = 1; a.n = n;
    a.S64 = nullptr; a.S32 = nullptr; a.amb = amb; a.spins = spins; a.keys = keys;
    k_select<<<R, 256, 0, st>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reduced problem (HQA section, effective couplings): J_eff = J[A, A] and
// h_eff_a = h_a + sum_{k not in A} J_ak s_k, each h_eff the correctly rounded
// exact sum.  One wavefront per (replica, ambivalent spin).
// ---------------------------------------------------------------------------
struct RedArgs {
    int N, R, n, csr, b0;
    const double *J;
    const int32_t *rp, *ci;
    const double *h;
    const int32_t *amb;
    const int8_t *spins;
    double *h_eff, *J_eff;
};

__device__ __forceinline__ bool in_sorted(const int32_t *A, int n, int k) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (A[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo < n && A[lo] == k;
}

__device__ __forceinline__ double jlookup(const RedArgs &a, int i, int j) {
    if (!a.csr) return a.J[(int64_t)i * a.N + j];
    int lo = a.rp[i], hi = a.rp[i + 1];
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a.ci[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < a.rp[i + 1] && a.ci[lo] == j) ? a.J[lo] : 0.0;
}

__device__ __forceinline__ void reduce_body(const RedArgs &a, const int bx_) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = ((int64_t)bx_ * blockDim.x + threadIdx.x) >> 6;
    if (wid >= (int64_t)a.R * a.n) return;
    const int r = (int)(wid / a.n), ai = (int)(wid % a.n);
    const int32_t *A = a.amb + (int64_t)r * a.n;
    const int8_t *s = a.spins + (int64_t)r * a.N;
    const int row = A[ai];
    if (row < 0 || row >= a.N) return;
    Acc256 acc;
    acc_zero(acc);
    if (lane == 0) acc_add(acc, a.h[row], a.b0);
    if (!a.csr) {
        const double *Jr = a.J + (int64_t)row * a.N;
        for (int k = lane; k < a.N; k += 64)
            if (!in_sorted(A, a.n, k)) acc_add(acc, Jr[k] * (double)s[k], a.b0);
    } else {
        for (int e = a.rp[row] + lane; e < a.rp[row + 1]; e += 64) {
            int k = a.ci[e];
            if (!in_sorted(A, a.n, k)) acc_add(acc, a.J[e] * (double)s[k], a.b0);
        }
    }
    acc_wave_allreduce(acc);
    if (lane == 0) a.h_eff[(int64_t)r * a.n + ai] = acc_round(acc, a.b0);
    if (a.J_eff)   // optional: the tabu search reads J[A, A] from the instance itself
        for (int b = lane; b < a.n; b += 64)
            a.J_eff[((int64_t)r * a.n + ai) * a.n + b] = jlookup(a, row, A[b]);
}

__global__ __launch_bounds__(256) void k_reduce(RedArgs a) { reduce_body(a, blockIdx.x); }

__global__ __launch_bounds__(256) void k_reduce_many(const RedArgs *as, const int *nb) {
    const int k = blockIdx.y;
    if ((int)blockIdx.x >= nb[k]) return;
    const RedArgs a = as[k];
    reduce_body(a, blockIdx.x);
}

hipError_t launch_reduce(const Instance &I, int R, int n, const int32_t *amb,
                         const int8_t *spins, double *h_eff, double *J_eff, hipStream_t st) {
    RedArgs a;
    a.N = I.N; a.R = R; a.n = n; a.csr = I.layout == HQA_CSR; a.b0 = I.es.lsb;
    a.J = I.J64; a.rp = I.rp; a.ci = I.ci; a.h = I.h64;
    a.amb = amb; a.spins = spins; a.h_eff = h_eff; a.J_eff = J_eff;
    int64_t waves = (int64_t)R * n;
    if (waves == 0) return hipSuccess;
    k_reduce<<<(unsigned)((waves + 3) / 4), 256, 0, st>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exact minimum of the reduced energy E'(c) = sum_{a<b} J_ab x_a x_b + sum_a h_a x_a
// over all codes c (bit a set: x_a = -1), ties to the smallest code.  Thread t
// fixes the top bits of the code to t and walks the low bits in Gray-code order
// (one workgroup per replica for integer couplings, several for real ones; see
// k_enumerate_int and k_enum_real), updating E' and the local fields
// f_a = h_a + sum_{b != a} J_ab x_b by one flip per code (dE = -2 x_a f_a).
// Integer instances run in int64 (exact).  Otherwise pass 1 walks in binary64
// and pass 2 re-walks, rescoring exactly (fixed-point accumulator, rounded once)
// every code whose binary64 energy lies within a rigorous error bound of the
// pass-1 minimum.
// ---------------------------------------------------------------------------
#define ENUM_MAXN 24
#define ENERGY_MAXN_LDS 16384
#define ENUM_MAXLOW 16

template <typename T>
struct EnumState {
    T E;
    int64_t code;
};

__device__ __forceinline__ bool better_i(int64_t e1, int64_t c1, int64_t e2, int64_t c2) {
    return e1 < e2 || (e1 == e2 && c1 < c2);
}
__device__ __forceinline__ bool better_d(double e1, int64_t c1, double e2, int64_t c2) {
    return e1 < e2 || (e1 == e2 && c1 < c2);
}

struct EnumArgs {
    int n, R, b0, integral;
    const double *J_eff, *h_eff;
    int64_t *code;
    double *e_red;
};

template <typename T>
__device__ __forceinline__ T energy_from_scratch(const T *J, const T *h, int n, uint32_t code) {
    T E = 0;
    for (int a = 0; a < n; a++) {
        T xa = ((code >> a) & 1) ? (T)-1 : (T)1;
        T acc = 0;
        for (int b = a + 1; b < n; b++) {
            T xb = ((code >> b) & 1) ? (T)-1 : (T)1;
            acc = acc + J[a * n + b] * xb;
        }
        E = E + xa * (acc + h[a]);
    }
    return E;
}

__device__ __forceinline__ double energy_exact(const double *J, const double *h, int n,
                                               uint32_t code, int b0) {
    Acc256 acc;
    acc_zero(acc);
    for (int a = 0; a < n; a++) {
        double xa = ((code >> a) & 1) ? -1.0 : 1.0;
        for (int b = a + 1; b < n; b++) {
            double xb = ((code >> b) & 1) ? -1.0 : 1.0;
            acc_add(acc, J[a * n + b] * (xa * xb), b0);
        }
        acc_add(acc, h[a] * xa, b0);
    }
    return acc_round(acc, b0);
}

// Gray walk over the low `nl` bits with the top bits fixed to `top`.  The visitor
// sees (energy, code) for every code of the chunk.
template <typename T, typename Visit>
__device__ __forceinline__ void gray_walk(const T *J, const T *h, int n, int nl, uint32_t top,
                                          T *f, Visit visit) {
    uint32_t code = top << nl;
    T E = energy_from_scratch<T>(J, h, n, code);
    for (int a = 0; a < nl; a++) {
        T acc = h[a];
        for (int b = 0; b < n; b++)
            if (b != a) acc = acc + J[a * n + b] * (((code >> b) & 1) ? (T)-1 : (T)1);
        f[a] = acc;
    }
    visit(E, code);
    const uint32_t cnt = 1u << nl;
    for (uint32_t k = 1; k < cnt; k++) {
        int a = __ffs(k) - 1;
        T xa = ((code >> a) & 1) ? (T)-1 : (T)1;
        E = E - (T)2 * xa * f[a];
        for (int b = 0; b < nl; b++)
            if (b != a) f[b] = f[b] - (T)2 * J[a * n + b] * xa;
        code ^= 1u << a;
        visit(E, code);
    }
}

// Real couplings, many codes: the code space of each replica is split over P
// workgroups of 256 threads; thread t of workgroup p fixes the top pt = n - NL bits of
// the code to p * 256 + t and walks the NL low bits in Gray-code order.  Every code
// sees the operations of gray_walk above in the same order (E and the local fields
// from scratch at the start, then E - 2 x_a f_a and f_b - 2 J_ab x_a per flip, each
// product exact, one rounding per update; the products are formed inside fma, which
// rounds once like the two-step form), so the pass-1 minimum obeys the same error
// bound with K = 2^NL codes per walk.  The local fields sit in registers: within a
// block of 16 codes the flipped bit is a compile-time ruler index (with 2 J_ab of
// those bits in registers), and the flip between blocks picks its field by selects.
//   k_enum_real<NL>(pass 1): each workgroup's binary64 minimum (E, code) -> part;
//   k_enum_real_mid: per replica, the minimum over the workgroups and the rescoring
//     threshold E_min + 2 delta + 4 u S (the bound of k_enumerate);
//   k_enum_real<NL>(pass 2): every code at or below the threshold is rescored exactly
//     (fixed-point accumulator, rounded once); each workgroup's exact minimum -> part;
//   k_enum_real_fin: per replica, the exact minimum over the workgroups, ties to the
//     smallest code.
// ---------------------------------------------------------------------------
#define ENUM_PT_REAL 12

struct EnumRealArgs {
    int n, R, P, b0;
    const double *J_eff, *h_eff;
    double *partE;        // [R][P]
    int64_t *partC;       // [R][P]
    double *thresh;       // [R]
    int64_t *code;
    double *e_red;
};

template <int NL>
__device__ __forceinline__ void enum_real_body(const EnumRealArgs &a, int pass, const int bx_) {
    __shared__ double Jd[ENUM_MAXN * ENUM_MAXN], J2[ENUM_MAXN * ENUM_MAXN], hd[ENUM_MAXN];
    __shared__ double sE[256];
    __shared__ int64_t sC[256];
    const int r = bx_ / a.P, p = bx_ % a.P, tid = threadIdx.x, n = a.n;
    for (int k = tid; k < n * n; k += 256) {
        const double v = a.J_eff[(int64_t)r * n * n + k];
        Jd[k] = v;
        J2[k] = 2.0 * v;
    }
    for (int k = tid; k < n; k += 256) hd[k] = a.h_eff[(int64_t)r * n + k];
    __syncthreads();
    const uint32_t top = (uint32_t)(p * 256 + tid);
    const bool active = top < (1u << (n - NL));
    const double thr = pass == 2 ? a.thresh[r] : 0.0;
    double bestE = INFINITY;
    int64_t bestC = INT64_MAX;
    auto visit = [&](double E, uint32_t c) {
        if (pass == 1) {
            if (better_d(E, c, bestE, bestC)) { bestE = E; bestC = c; }
        } else if (E <= thr) {
            const double ex = energy_exact(Jd, hd, n, c, a.b0);
            if (better_d(ex, c, bestE, bestC)) { bestE = ex; bestC = c; }
        }
    };
    if (active) {
        uint32_t code = top << NL;
        double E = energy_from_scratch<double>(Jd, hd, n, code);
        visit(E, code);
        if constexpr (NL > 0) {
            double f[NL];
#pragma unroll
            for (int aa = 0; aa < NL; aa++) {
                double acc = hd[aa];
                for (int b = 0; b < n; b++)
                    if (b != aa) acc = acc + Jd[aa * n + b] * (((code >> b) & 1) ? -1.0 : 1.0);
                f[aa] = acc;
            }
            constexpr int NA = NL < 4 ? NL : 4;        // bits flipped inside a block of 16
            double D[NA][NL];
#pragma unroll
            for (int aa = 0; aa < NA; aa++)
#pragma unroll
                for (int b = 0; b < NL; b++) D[aa][b] = J2[aa * n + b];
            constexpr int NBLK = NL >= 4 ? 1 << (NL - 4) : 1;
            for (int m = 0; m < NBLK; m++) {
#pragma unroll
                for (int j = 1; j < 16; j++) {
                    if (j >= (1 << NL)) break;
                    const int aa = __builtin_ctz(j);
                    const double xa = ((code >> aa) & 1u) ? -1.0 : 1.0;
                    E = __builtin_fma(-2.0 * xa, f[aa], E);
#pragma unroll
                    for (int b = 0; b < NL; b++)
                        if (b != aa) f[b] = __builtin_fma(-xa, D[aa][b], f[b]);
                    code ^= 1u << aa;
                    visit(E, code);
                }
                if (m + 1 < NBLK) {                       // flip of bit 4 + ctz(m + 1)
                    const int aa = 4 + __builtin_ctz(m + 1);
                    const double xa = ((code >> aa) & 1u) ? -1.0 : 1.0;
                    double fa = f[0];
#pragma unroll
                    for (int b = 1; b < NL; b++) fa = b == aa ? f[b] : fa;
                    E = __builtin_fma(-2.0 * xa, fa, E);
#pragma unroll
                    for (int b = 0; b < NL; b++)
                        if (b != aa) f[b] = __builtin_fma(-xa, J2[aa * n + b], f[b]);
                    code ^= 1u << aa;
                    visit(E, code);
                }
            }
        }
    }
    sE[tid] = bestE;
    sC[tid] = bestC;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (tid < s2 && better_d(sE[tid + s2], sC[tid + s2], sE[tid], sC[tid])) {
            sE[tid] = sE[tid + s2];
            sC[tid] = sC[tid + s2];
        }
        __syncthreads();
    }
    if (tid == 0) {
        a.partE[(int64_t)r * a.P + p] = sE[0];
        a.partC[(int64_t)r * a.P + p] = sC[0];
    }
}

template <int NL>
__global__ __launch_bounds__(256) void k_enum_real(EnumRealArgs a, int pass) {
    enum_real_body<NL>(a, pass, blockIdx.x);
}

template <int NL>
__global__ __launch_bounds__(256) void k_enum_real_many(const EnumRealArgs *as, const int *nb,
                                                        int pass) {
    const int k = blockIdx.y;
    if ((int)blockIdx.x >= nb[k]) return;
    const EnumRealArgs a = as[k];
    enum_real_body<NL>(a, pass, blockIdx.x);
}

// One wavefront per replica: minimum over the P workgroup results; after pass 1 the
// rescoring threshold, after pass 2 the result.
__device__ __forceinline__ void enum_real_mid_body(const EnumRealArgs &a, int pass, const int bx_) {
    const int r = bx_, lane = threadIdx.x, n = a.n;
    double E = INFINITY;
    int64_t C = INT64_MAX;
    for (int p = lane; p < a.P; p += 64) {
        const double e2 = a.partE[(int64_t)r * a.P + p];
        const int64_t c2 = a.partC[(int64_t)r * a.P + p];
        if (better_d(e2, c2, E, C)) { E = e2; C = c2; }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double e2 = __shfl_xor(E, off);
        const int64_t c2 = __shfl_xor(C, off);
        if (better_d(e2, c2, E, C)) { E = e2; C = c2; }
    }
    if (pass == 2) {
        if (lane == 0) {
            a.code[r] = C;
            a.e_red[r] = E;
        }
        return;
    }
    // rigorous bound on |E_binary64 - E_exact| along a walk of K = 2^NL codes:
    // u S (m + K (2n + 1) + K^2) with S = sum |J_ab| (a < b) + sum |h_a|, m the term
    // count, u = 2^-53; doubled (the minimum's own error and a candidate's), plus the
    // rounding of the exact values themselves
    double Ssum = 0.0;
    const double *J = a.J_eff + (int64_t)r * n * n, *h = a.h_eff + (int64_t)r * n;
    for (int k = lane; k < n * n; k += 64)
        if (k % n > k / n) Ssum += fabs(J[k]);
    for (int k = lane; k < n; k += 64) Ssum += fabs(h[k]);
    for (int off = 32; off > 0; off >>= 1) Ssum += __shfl_xor(Ssum, off);
    if (lane == 0) {
        const int nl = n > ENUM_PT_REAL ? n - ENUM_PT_REAL : 0;
        const double S = Ssum * (1.0 + 1e-12);
        const double K = (double)(1u << nl);
        const double mterms = (double)(n * (n - 1) / 2 + n);
        const double u = 1.1102230246251565e-16;
        const double delta = u * S * (mterms + K * (2.0 * n + 1.0) + K * K);
        a.thresh[r] = E + 2.0 * delta + 4.0 * u * S;
    }
}

__global__ __launch_bounds__(64) void k_enum_real_mid(EnumRealArgs a, int pass) {
    enum_real_mid_body(a, pass, blockIdx.x);
}

__global__ __launch_bounds__(64) void k_enum_real_mid_many(const EnumRealArgs *as, const int *nb,
                                                          int pass) {
    const int k = blockIdx.y;
    if ((int)blockIdx.x >= nb[k]) return;
    const EnumRealArgs a = as[k];
    enum_real_mid_body(a, pass, blockIdx.x);
}

template <int NL>
static void launch_enum_real(const EnumRealArgs &a, hipStream_t st) {
    k_enum_real<NL><<<a.R * a.P, 256, 0, st>>>(a, 1);
    k_enum_real_mid<<<a.R, 64, 0, st>>>(a, 1);
    k_enum_real<NL><<<a.R * a.P, 256, 0, st>>>(a, 2);
    k_enum_real_mid<<<a.R, 64, 0, st>>>(a, 2);
}

size_t enum_scratch_bytes(int n, int R) {
    const int pt = n < ENUM_PT_REAL ? n : ENUM_PT_REAL;
    const int P = ((1 << pt) + 255) / 256;
    return (size_t)R * P * 16 + (size_t)R * 8 + 64;
}

// Integer instances with small sums: 1024 threads per replica, thread t fixes the
// top pt = n - NL <= 10 bits of the code to t and walks the NL low bits in Gray-code
// order in int32.  The low bits of every thread follow the same sequence, so the
// flipped bit a and the sign x_a before the flip are the same for all lanes: 15 of
// every 16 flips have a compile-time a (the ruler sequence of the block), the local
// fields sit in registers and each update f_b += (-x_a) 2 J_ab is one 24-bit
// multiply-add with a wavefront-uniform factor.  The walk keeps the minimum of the
// key (E' + S) << NL | low code, so equal energies resolve to the smallest code.
// Requires every |J_ab|, |h_a| integral with S = sum_{a<b} |J_ab| + sum_a |h_a| below
// 2^22 and 2 S < 2^(31 - NL) (all terms then fit the 24-bit products and the key);
// other integer replicas take the int64 walk.
#define ENUM_PT 10

__device__ __forceinline__ int32_t mad24(int32_t x, int32_t y, int32_t z) {
    return __mul24(x, y) + z;
}

template <int NL>
__device__ __forceinline__ void walk_i32(const int32_t *Jv, const int32_t *J2, const int32_t *hv,
                                         int n, uint32_t top, int32_t S, int64_t &bestE,
                                         int64_t &bestC) {
    // start: low bits all 0 (x = +1), top bits from `top`
    auto xof = [&](int c) -> int32_t {
        return c < NL ? 1 : (((top >> (c - NL)) & 1u) ? -1 : 1);
    };
    int32_t E = S;
    for (int aa = 0; aa < n; aa++) {
        int32_t acc = hv[aa];
        for (int bb = aa + 1; bb < n; bb++) acc += Jv[aa * n + bb] * xof(bb);
        E += xof(aa) * acc;
    }
    uint32_t key = (uint32_t)E << NL;
    if constexpr (NL > 0) {
        int32_t f[NL];
#pragma unroll
        for (int b = 0; b < NL; b++) {
            int32_t acc = hv[b];
            for (int c = 0; c < n; c++) acc += Jv[b * n + c] * xof(c);   // J_bb = 0
            f[b] = acc;
        }
        constexpr int NA = NL < 4 ? NL : 4;           // bits flipped inside a block of 16
        int32_t D[NA][NL];
#pragma unroll
        for (int aa = 0; aa < NA; aa++)
#pragma unroll
            for (int b = 0; b < NL; b++) D[aa][b] = J2[aa * n + b];
        uint32_t g = 0;                                // low code (uniform)
        constexpr int NBLK = NL >= 4 ? 1 << (NL - 4) : 1;
        for (int m = 0; m < NBLK; m++) {
#pragma unroll
            for (int j = 1; j < 16; j++) {
                if (j >= (1 << NL)) break;
                constexpr int dummy = 0;
                (void)dummy;
                const int aa = __builtin_ctz(j);
                const int32_t sgn = ((g >> aa) & 1u) ? 1 : -1;   // -x_a before the flip
                E = mad24(f[aa], 2 * sgn, E);
#pragma unroll
                for (int b = 0; b < NL; b++)
                    if (b != aa) f[b] = mad24(D[aa][b], sgn, f[b]);
                g ^= 1u << aa;
                key = min(key, ((uint32_t)E << NL) | g);
            }
            if (m + 1 < NBLK) {                        // flip of bit 4 + ctz(m + 1)
                const int aa = 4 + __builtin_ctz(m + 1);
                const int32_t sgn = ((g >> aa) & 1u) ? 1 : -1;
                int32_t fa = f[0];
#pragma unroll
                for (int b = 1; b < NL; b++) fa = b == aa ? f[b] : fa;
                E = mad24(fa, 2 * sgn, E);
#pragma unroll
                for (int b = 0; b < NL; b++) f[b] = mad24(J2[aa * n + b], sgn, f[b]);   // J_aa = 0
                g ^= 1u << aa;
                key = min(key, ((uint32_t)E << NL) | g);
            }
        }
    }
    bestE = (int64_t)(key >> NL) - S;
    bestC = ((int64_t)top << NL) | (key & ((1u << NL) - 1u));
}

template <int NL>
__device__ __forceinline__ void enumerate_int_body(const EnumArgs &a, const int bx_) {
    __shared__ int32_t Jv[ENUM_MAXN * ENUM_MAXN], J2[ENUM_MAXN * ENUM_MAXN], hv[ENUM_MAXN];
    __shared__ int64_t Jl[ENUM_MAXN * ENUM_MAXN], hl[ENUM_MAXN];
    __shared__ int64_t sEi[1024], sC[1024];
    __shared__ unsigned long long sS;
    const int r = bx_, tid = threadIdx.x, n = a.n;
    if (tid == 0) sS = 0;
    __syncthreads();
    for (int k = tid; k < n * n; k += 1024) {
        const int64_t v = (int64_t)a.J_eff[(int64_t)r * n * n + k];
        Jl[k] = v;
        if (k / n < k % n) atomicAdd(&sS, (unsigned long long)(v < 0 ? -v : v));
    }
    for (int k = tid; k < n; k += 1024) {
        const int64_t v = (int64_t)a.h_eff[(int64_t)r * n + k];
        hl[k] = v;
        atomicAdd(&sS, (unsigned long long)(v < 0 ? -v : v));
    }
    __syncthreads();
    const unsigned long long S = sS;
    const bool fast = S < (1ull << 22) && 2 * S < (1ull << (31 - NL));   // uniform
    if (fast) {
        for (int k = tid; k < n * n; k += 1024) {
            Jv[k] = (int32_t)Jl[k];
            J2[k] = 2 * (int32_t)Jl[k];
        }
        for (int k = tid; k < n; k += 1024) hv[k] = (int32_t)hl[k];
        __syncthreads();
    }
    const bool active = tid < (1 << (n - NL));
    int64_t bestE = INT64_MAX, bestC = INT64_MAX;
    if (active) {
        if (fast) {
            walk_i32<NL>(Jv, J2, hv, n, (uint32_t)tid, (int32_t)S, bestE, bestC);
        } else {
            int64_t f[ENUM_MAXLOW];
            gray_walk<int64_t>(Jl, hl, n, NL, (uint32_t)tid, f, [&](int64_t E, uint32_t c) {
                if (better_i(E, c, bestE, bestC)) { bestE = E; bestC = c; }
            });
        }
    }
    // argmin over the workgroup, ties to the smaller code
    sEi[tid] = bestE;
    sC[tid] = bestC;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (tid < st && better_i(sEi[tid + st], sC[tid + st], sEi[tid], sC[tid])) {
            sEi[tid] = sEi[tid + st];
            sC[tid] = sC[tid + st];
        }
        __syncthreads();
    }
    if (tid == 0) {
        a.code[r] = sC[0];
        a.e_red[r] = (double)sEi[0];
    }
}

template <int NL>
__global__ __launch_bounds__(1024) void k_enumerate_int(EnumArgs a) {
    enumerate_int_body<NL>(a, blockIdx.x);
}

template <int NL>
__global__ __launch_bounds__(1024) void k_enumerate_int_many(const EnumArgs *as, const int *nb) {
    const int k = blockIdx.y;
    if ((int)blockIdx.x >= nb[k]) return;
    const EnumArgs a = as[k];
    enumerate_int_body<NL>(a, blockIdx.x);
}

template <int NL>
static void launch_enum_int(const EnumArgs &a, hipStream_t st) {
    k_enumerate_int<NL><<<a.R, 1024, 0, st>>>(a);
}

hipError_t launch_enumerate(int n, int R, const double *J_eff, const double *h_eff, int b0,
                            int integral, int64_t *code, double *e_red, void *scratch,
                            hipStream_t st) {
    EnumArgs a;
    a.n = n; a.R = R; a.b0 = b0; a.integral = integral;
    a.J_eff = J_eff; a.h_eff = h_eff; a.code = code; a.e_red = e_red;
    if (R == 0) return hipSuccess;
    if (!integral) {
        EnumRealArgs b;
        const int pt = n < ENUM_PT_REAL ? n : ENUM_PT_REAL;
        b.n = n; b.R = R; b.P = ((1 << pt) + 255) / 256; b.b0 = b0;
        b.J_eff = J_eff; b.h_eff = h_eff; b.code = code; b.e_red = e_red;
        b.partE = (double *)scratch;
        b.partC = (int64_t *)((char *)scratch + (size_t)R * b.P * 8);
        b.thresh = (double *)((char *)scratch + (size_t)R * b.P * 16);
        switch (n - pt) {
            case 0: launch_enum_real<0>(b, st); break;
            case 1: launch_enum_real<1>(b, st); break;
            case 2: launch_enum_real<2>(b, st); break;
            case 3: launch_enum_real<3>(b, st); break;
            case 4: launch_enum_real<4>(b, st); break;
            case 5: launch_enum_real<5>(b, st); break;
            case 6: launch_enum_real<6>(b, st); break;
            case 7: launch_enum_real<7>(b, st); break;
            case 8: launch_enum_real<8>(b, st); break;
            case 9: launch_enum_real<9>(b, st); break;
            case 10: launch_enum_real<10>(b, st); break;
            case 11: launch_enum_real<11>(b, st); break;
            default: launch_enum_real<12>(b, st); break;
        }
        return hipGetLastError();
    }
    switch (n > ENUM_PT ? n - ENUM_PT : 0) {   // low bits walked per thread
        case 0: launch_enum_int<0>(a, st); break;
        case 1: launch_enum_int<1>(a, st); break;
        case 2: launch_enum_int<2>(a, st); break;
        case 3: launch_enum_int<3>(a, st); break;
        case 4: launch_enum_int<4>(a, st); break;
        case 5: launch_enum_int<5>(a, st); break;
        case 6: launch_enum_int<6>(a, st); break;
        case 7: launch_enum_int<7>(a, st); break;
        case 8: launch_enum_int<8>(a, st); break;
        case 9: launch_enum_int<9>(a, st); break;
        case 10: launch_enum_int<10>(a, st); break;
        case 11: launch_enum_int<11>(a, st); break;
        case 12: launch_enum_int<12>(a, st); break;
        case 13: launch_enum_int<13>(a, st); break;
        default: launch_enum_int<14>(a, st); break;
    }
    return hipGetLastError();
}

struct MergeArgs {
    int N, R, n;
    const int32_t *amb;
    const int64_t *code;
    int8_t *spins;
};

__device__ __forceinline__ void merge_body(int N, int R, int n, const int32_t *amb,
                                           const int64_t *code, int8_t *spins, const int bx_) {
    int64_t t = (int64_t)bx_ * blockDim.x + threadIdx.x;
    if (t >= (int64_t)R * n) return;
    int r = (int)(t / n), ai = (int)(t % n);
    int i = amb[t];
    if (i < 0 || i >= N) return;
    spins[(int64_t)r * N + i] = ((code[r] >> ai) & 1) ? -1 : 1;
}

__global__ void k_merge(int N, int R, int n, const int32_t *amb, const int64_t *code,
                        int8_t *spins) {
    merge_body(N, R, n, amb, code, spins, blockIdx.x);
}

__global__ void k_merge_many(const MergeArgs *as, const int *nb) {
    const int k = blockIdx.y;
    if ((int)blockIdx.x >= nb[k]) return;
    const MergeArgs a = as[k];
    merge_body(a.N, a.R, a.n, a.amb, a.code, a.spins, blockIdx.x);
}

hipError_t launch_merge(int N, int R, int n, const int32_t *amb, const int64_t *code,
                        int8_t *spins, hipStream_t st) {
    int64_t t = (int64_t)R * n;
    if (t == 0) return hipSuccess;
    k_merge<<<(unsigned)((t + 255) / 256), 256, 0, st>>>(N, R, n, amb, code, spins);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exact Ising energy (Eq. 1) and cut (Methods, MAX-CUT with w = J).
//
// Dense instances (k_energy_mv): over the upper triangle, with s_i s_j = 1 - 2 [s_i != s_j]
// and s_i = 1 - 2 [s_i = -1],
//   C = sum_{i<j, s_i != s_j} J_ij,   S = sum_{i<j} J_ij,
//   H = sum_i h_i s_i = Ht - 2 Hn,    Ht = sum_i h_i,   Hn = sum_{i: s_i = -1} h_i,
//   E = sum_{i<j} J_ij s_i s_j + H = S - 2 C + Ht - 2 Hn.
// The spins of 64 vectors are packed into one 64-bit word per spin (bit v: vector v has
// s = -1), so one pass over the upper triangle serves every vector of a group: for the
// pair (i, j) the word m_i ^ m_j marks the vectors the pair cuts.
//
// Exactness by level sums: every J and h is a multiple of 2^b0 below 2^(msb + 1).  With
// lg = ceil(log2(N^2 + N)) and w = 51 - lg, the levels sigma_k = b0 + k w (k < L) cover
// the bits [b0, msb] when L w >= msb + 1 - b0.  A term is cut into parts t_k, multiples of
// 2^sigma_k below 2^(sigma_(k+1)) (top level: 2^(sigma_L + 1)), by rounding to a multiple
// of 2^sigma_k from the top level down ((r + K_k) - K_k with K_k = 1.5 2^(sigma_k + 52),
// exact for |r| <= 2^(sigma_k + 51)) and keeping the exact remainder; the lowest part is
// the last remainder.  Any sum of at most 2^lg parts of one level is then a multiple of
// 2^sigma_k below 2^(sigma_k + 53): binary64 adds them exactly, in any order and any
// grouping (lanes, wavefronts, workgroups, slices).  The merge adds the level totals
// into the fixed-point accumulator and rounds once.  L = 1 is a plain binary64 sum.
//
// CSR instances, and dense ones whose bits need more than four levels (k_energy), keep
// one workgroup per (vector, slice): the sum over ordered pairs i != j counts each pair
// twice, so 2E = sum_{i!=j} J s s + 2 sum h s and 2C = sum_{i!=j, s_i != s_j} J are
// accumulated exactly (binary64 when the fast condition holds, else the fixed-point
// accumulator per term) and rounded with the scale halved.
// ---------------------------------------------------------------------------
struct EnArgs {
    int N, V, P, csr, b0;
    int fast;          // plain binary64 sums are exact (see launch_energy)
    const double *J;
    const int32_t *rp, *ci;
    const double *h;
    const int8_t *spins;
    void *part;        // [V][P] partials: two doubles (fast) or two Acc256
    double *E, *cut;
};

__device__ void block_acc_reduce(Acc256 &acc, Acc256 *sh) {
    acc_wave_allreduce(acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int v = 1; v < (int)(blockDim.x >> 6); v++) acc_merge(acc, sh[v]);
    __syncthreads();
}

// Sum of a binary64 value over the workgroup (exact when every partial sum is).
__device__ double block_sum(double x, double *sh) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = x;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int v = 0; v < (int)(blockDim.x >> 6); v++) t += sh[v];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(256) void k_energy(EnArgs a) {
    __shared__ Acc256 sh[4];
    __shared__ double shd[4];
    __shared__ int8_t sv[ENERGY_MAXN_LDS];
    const int v = blockIdx.x / a.P, p = blockIdx.x % a.P, tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int8_t *s = a.spins + (int64_t)v * a.N;
    const bool lds = a.N <= ENERGY_MAXN_LDS;
    if (lds)
        for (int i = tid; i < a.N; i += 256) sv[i] = s[i];
    __syncthreads();
    const int8_t *ss = lds ? sv : s;
    const int b0 = a.b0;
    const int64_t slot = (int64_t)v * a.P + p;
    if (a.fast) {
        // every partial sum is a multiple of 2^b0 below 2^(53 + b0): binary64 is exact
        double ae = 0.0, ac = 0.0;
        if (!a.csr) {
            for (int i = 4 * p + w; i < a.N; i += 4 * a.P) {
                const double *Jr = a.J + (int64_t)i * a.N;
                const int si = ss[i];
                for (int j = lane; j < a.N; j += 64) {
                    const double J = Jr[j];
                    const bool same = si == ss[j];
                    ae += same ? J : -J;
                    ac += same ? 0.0 : J;
                }
            }
        } else {
            for (int i = 256 * p + tid; i < a.N; i += 256 * a.P) {
                const int si = ss[i];
                for (int e = a.rp[i]; e < a.rp[i + 1]; e++) {
                    const double J = a.J[e];
                    const bool same = si == ss[a.ci[e]];
                    ae += same ? J : -J;
                    ac += same ? 0.0 : J;
                }
            }
        }
        for (int i = 256 * p + tid; i < a.N; i += 256 * a.P)
            ae += ss[i] > 0 ? 2.0 * a.h[i] : -2.0 * a.h[i];
        ae = block_sum(ae, shd);
        ac = block_sum(ac, shd);
        if (tid == 0) {
            double *o = (double *)a.part + 2 * slot;
            o[0] = ae;
            o[1] = ac;
        }
        return;
    }
    Acc256 ae, ac;
    acc_zero(ae);
    acc_zero(ac);
    if (!a.csr) {
        for (int i = 4 * p + w; i < a.N; i += 4 * a.P) {
            const double *Jr = a.J + (int64_t)i * a.N;
            const int si = ss[i];
            for (int j = lane; j < a.N; j += 64) {
                const double J = Jr[j];
                if (J == 0.0) continue;
                const int sj = ss[j];
                acc_add(ae, si == sj ? J : -J, b0);
                if (si != sj) acc_add(ac, J, b0);
            }
        }
    } else {
        for (int i = 256 * p + tid; i < a.N; i += 256 * a.P) {
            int si = ss[i];
            for (int e = a.rp[i]; e < a.rp[i + 1]; e++) {
                double J = a.J[e];
                int sj = ss[a.ci[e]];
                acc_add(ae, si == sj ? J : -J, b0);
                if (si != sj) acc_add(ac, J, b0);
            }
        }
    }
    for (int i = 256 * p + tid; i < a.N; i += 256 * a.P) {
        double hh = a.h[i];
        if (hh != 0.0) acc_add(ae, ss[i] > 0 ? 2.0 * hh : -2.0 * hh, b0);
    }
    block_acc_reduce(ae, sh);
    block_acc_reduce(ac, sh);
    if (tid == 0) {
        Acc256 *o = (Acc256 *)a.part + 2 * slot;
        o[0] = ae;
        o[1] = ac;
    }
}

// Totals of the P slices of each vector (a thread per vector), rounded once.
__global__ __launch_bounds__(64) void k_energy_merge(EnArgs a) {
    const int v = blockIdx.x * 64 + threadIdx.x;
    if (v >= a.V) return;
    const int64_t s0 = (int64_t)v * a.P;
    if (a.fast) {
        const double *o = (const double *)a.part;
        double ae = 0.0, ac = 0.0;
        for (int p = 0; p < a.P; p++) {
            ae += o[2 * (s0 + p)];
            ac += o[2 * (s0 + p) + 1];
        }
        if (a.E) a.E[v] = 0.5 * ae;
        if (a.cut) a.cut[v] = 0.5 * ac;
        return;
    }
    const Acc256 *o = (const Acc256 *)a.part;
    Acc256 ae = o[2 * s0], ac = o[2 * s0 + 1];
    for (int p = 1; p < a.P; p++) {
        acc_merge(ae, o[2 * (s0 + p)]);
        acc_merge(ac, o[2 * (s0 + p) + 1]);
    }
    if (a.E) a.E[v] = acc_round(ae, a.b0 - 1);
    if (a.cut) a.cut[v] = acc_round(ac, a.b0 - 1);
}

// ----- dense: many vectors per pass, level sums -----
struct EnMvArgs {
    int N, V, P, b0;
    int jt;            // type of Js (JT_F32, JT_BF16, JT_FP8), -1 to read J
    int ldj;           // row pitch of Js
    const void *Js;    // the exact storage copy of J (or NULL)
    const double *J;
    const double *h;   // NULL: no field
    const int8_t *spins;
    uint64_t *masks;   // [ceil(V / 64)][N]
    double *part;      // see energy_mv_layout
    double K[4];       // rounding constants of levels 1 .. L - 1
    double *E, *cut;
};

// Offsets (in doubles) of the partial sums of a launch with P slices, V vectors, L
// levels: C and Hn per (slice, vector, level), then S and Ht per (slice, level).
struct EnMvLayout {
    int64_t c, hn, s, ht, total;
};
static __host__ __device__ EnMvLayout energy_mv_layout(int P, int V, int L) {
    EnMvLayout o;
    o.c = 0;
    o.hn = (int64_t)P * V * L;
    o.s = 2 * o.hn;
    o.ht = o.s + (int64_t)P * L;
    o.total = o.ht + (int64_t)P * L;
    return o;
}

// Packed spins: word b of spin j has bit v set when vector 64 b + v has s_j = -1.  A
// thread per (word, spin): its 64 loads (rows clamped to the last vector, bits past it
// cleared) are independent, so they are all in flight at once, and consecutive threads
// read consecutive bytes of a row.
struct PackArgs {
    int N, V;
    const int8_t *spins;
    uint64_t *masks;
};

__device__ __forceinline__ void pack_masks_body(int N, int V, const int8_t *spins,
                                                uint64_t *masks, const int bx_) {
    const int64_t t = (int64_t)bx_ * blockDim.x + threadIdx.x;
    const int nw = (V + 63) / 64;
    if (t >= (int64_t)nw * N) return;
    const int b = (int)(t / N), j = (int)(t % N);
    int8_t x[64];
#pragma unroll
    for (int v = 0; v < 64; v++) x[v] = spins[(int64_t)min(64 * b + v, V - 1) * N + j];
    uint64_t m = 0;
#pragma unroll
    for (int v = 0; v < 64; v++) m |= (uint64_t)(x[v] < 0) << v;
    const int have = V - 64 * b;                     // vectors in this word
    if (have < 64) m &= (1ull << have) - 1ull;
    masks[t] = m;
}

__global__ __launch_bounds__(256) void k_pack_masks(int N, int V, const int8_t *spins,
                                                    uint64_t *masks) {
    pack_masks_body(N, V, spins, masks, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_pack_masks_many(const PackArgs *as, const int *nb) {
    const int k = blockIdx.y;
    if ((int)blockIdx.x >= nb[k]) return;
    const PackArgs a = as[k];
    pack_masks_body(a.N, a.V, a.spins, a.masks, blockIdx.x);
}

__device__ __forceinline__ double mv_coupling(const EnMvArgs &a, int i, int j) {
    if (a.jt < 0) return a.J[(int64_t)i * a.N + j];
    const int64_t t = (int64_t)i * a.ldj + j;
    if (a.jt == JT_FP8) {
        // OCP e4m3: sign, 4 exponent bits (bias 7), 3 mantissa bits; exponent 0 is
        // subnormal (m 2^-9).  The couplings are finite, so 0x7f / 0xff do not occur.
        const uint32_t b = ((const uint8_t *)a.Js)[t];
        const uint32_t e = (b >> 3) & 15u, m = b & 7u;
        const double mag = e ? (double)(8u + m) * (double)__uint_as_float((e + 117u) << 23)
                             : (double)m * 0x1p-9;
        return (b & 0x80u) ? -mag : mag;
    }
    if (a.jt == JT_BF16) {
        const uint32_t b = ((const uint16_t *)a.Js)[t];
        return (double)__uint_as_float(b << 16);
    }
    return (double)((const float *)a.Js)[t];
}

// The parts of a term on levels 0 .. L - 1 (see above).
template <int L>
__device__ __forceinline__ void mv_split(const EnMvArgs &a, double r, double (&t)[L]) {
#pragma unroll
    for (int k = L - 1; k >= 1; k--) {
        const double hi = (r + a.K[k]) - a.K[k];
        r -= hi;
        t[k] = hi;
    }
    t[0] = r;
}

// Workgroup (p, g): vectors g G .. g G + G - 1 (G divides 64, so one mask word), rows
// 4 p + w, 4 p + w + 4 P, ... (wavefront w), lanes along the columns j > i.  Lane x holds
// the column sums of C for every vector of the group and, for vector g G + x, the sum
// Hn; group 0 also sums S and Ht.
template <int G, int L>
__device__ __forceinline__ void energy_mv_body(const EnMvArgs &a, const int bx_, const int by_) {
    __shared__ double red[4][G + 2][L];
    const int p = bx_, g = by_, tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int v0 = g * G, word = v0 >> 6, sh = v0 & 63;
    const bool first = g == 0;
    const uint64_t *M = a.masks + (int64_t)word * a.N;
    double c[G][L], hn[L], s[L], ht[L];
#pragma unroll
    for (int k = 0; k < L; k++) {
        hn[k] = 0.0; s[k] = 0.0; ht[k] = 0.0;
#pragma unroll
        for (int v = 0; v < G; v++) c[v][k] = 0.0;
    }
    for (int i = 4 * p + w; i < a.N; i += 4 * a.P) {
        const uint64_t mi = M[i];
        if (a.h) {
            double t[L];
            mv_split<L>(a, a.h[i], t);
            // lanes x < G read bit sh + x <= 63 of the word; the others are not used
            const double bit = (double)(uint32_t)((mi >> ((sh + lane) & 63)) & 1ull);
            if (lane < G) {
#pragma unroll
                for (int k = 0; k < L; k++) hn[k] = fma(t[k], bit, hn[k]);
            }
            if (first && lane == 0) {
#pragma unroll
                for (int k = 0; k < L; k++) ht[k] += t[k];
            }
        }
        for (int j = i + 1 + lane; j < a.N; j += 64) {
            double t[L];
            mv_split<L>(a, mv_coupling(a, i, j), t);
            if (first) {
#pragma unroll
                for (int k = 0; k < L; k++) s[k] += t[k];
            }
            const uint64_t d = (mi ^ M[j]) >> sh;
#pragma unroll
            for (int v = 0; v < G; v++) {
                const double bit = (double)(uint32_t)((d >> v) & 1ull);
#pragma unroll
                for (int k = 0; k < L; k++) c[v][k] = fma(t[k], bit, c[v][k]);
            }
        }
    }
    // column sums over the lanes, then over the wavefronts
#pragma unroll
    for (int v = 0; v < G; v++)
#pragma unroll
        for (int k = 0; k < L; k++) {
            double x = c[v][k];
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
            if (lane == 0) red[w][v][k] = x;
        }
#pragma unroll
    for (int k = 0; k < L; k++) {
        double x = s[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) {
            red[w][G][k] = x;
            red[w][G + 1][k] = ht[k];
        }
    }
    __syncthreads();
    const EnMvLayout lay = energy_mv_layout(a.P, a.V, L);
    for (int e = tid; e < G * L; e += 256) {
        const int v = e / L, k = e % L;
        if (v0 + v < a.V)
            a.part[lay.c + ((int64_t)p * a.V + v0 + v) * L + k] =
                red[0][v][k] + red[1][v][k] + red[2][v][k] + red[3][v][k];
    }
    __syncthreads();
    // Hn: lane x of each wavefront holds vector v0 + x
    if (lane < G) {
#pragma unroll
        for (int k = 0; k < L; k++) red[w][lane][k] = hn[k];
    }
    __syncthreads();
    for (int e = tid; e < G * L; e += 256) {
        const int v = e / L, k = e % L;
        if (v0 + v < a.V)
            a.part[lay.hn + ((int64_t)p * a.V + v0 + v) * L + k] =
                red[0][v][k] + red[1][v][k] + red[2][v][k] + red[3][v][k];
    }
    if (first && tid < L) {
        a.part[lay.s + (int64_t)p * L + tid] =
            red[0][G][tid] + red[1][G][tid] + red[2][G][tid] + red[3][G][tid];
        a.part[lay.ht + (int64_t)p * L + tid] =
            red[0][G + 1][tid] + red[1][G + 1][tid] + red[2][G + 1][tid] + red[3][G + 1][tid];
    }
}

template <int G, int L>
__global__ __launch_bounds__(256) void k_energy_mv(EnMvArgs a) {
    energy_mv_body<G, L>(a, blockIdx.x, blockIdx.y);
}

// Many instances: instance blockIdx.z, its own slice count nb[z] (= its a.P).
template <int G, int L>
__global__ __launch_bounds__(256) void k_energy_mv_many(const EnMvArgs *as, const int *nb) {
    const int k = blockIdx.z;
    if ((int)blockIdx.x >= nb[k]) return;
    const EnMvArgs a = as[k];
    energy_mv_body<G, L>(a, blockIdx.x, blockIdx.y);
}

// Per vector (one wavefront, lanes over the slices): level totals over the slices (exact
// binary64 in any grouping), then E = S - 2 C + Ht - 2 Hn and C in the fixed-point
// accumulator, each rounded once.
template <int L>
__device__ __forceinline__ void energy_mv_merge_body(const EnMvArgs &a, const int bx_) {
    const int v = bx_ * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (v >= a.V) return;
    const EnMvLayout lay = energy_mv_layout(a.P, a.V, L);
    double C[L], Hn[L], S[L], Ht[L];
#pragma unroll
    for (int k = 0; k < L; k++) {
        C[k] = 0.0; Hn[k] = 0.0; S[k] = 0.0; Ht[k] = 0.0;
    }
    for (int p = lane; p < a.P; p += 64) {
#pragma unroll
        for (int k = 0; k < L; k++) {
            C[k] += a.part[lay.c + ((int64_t)p * a.V + v) * L + k];
            Hn[k] += a.part[lay.hn + ((int64_t)p * a.V + v) * L + k];
            S[k] += a.part[lay.s + (int64_t)p * L + k];
            Ht[k] += a.part[lay.ht + (int64_t)p * L + k];
        }
    }
#pragma unroll
    for (int k = 0; k < L; k++)
        for (int o = 32; o > 0; o >>= 1) {
            C[k] += __shfl_xor(C[k], o);
            Hn[k] += __shfl_xor(Hn[k], o);
            S[k] += __shfl_xor(S[k], o);
            Ht[k] += __shfl_xor(Ht[k], o);
        }
    if (lane) return;
    Acc256 ae, ac;
    acc_zero(ae);
    acc_zero(ac);
#pragma unroll
    for (int k = 0; k < L; k++) {
        acc_add(ac, C[k], a.b0);
        acc_add(ae, S[k], a.b0);
        acc_add(ae, Ht[k], a.b0);
        acc_add(ae, -2.0 * C[k], a.b0);
        acc_add(ae, -2.0 * Hn[k], a.b0);
    }
    if (a.E) a.E[v] = acc_round(ae, a.b0);
    if (a.cut) a.cut[v] = acc_round(ac, a.b0);
}

template <int L>
__global__ __launch_bounds__(256) void k_energy_mv_merge(EnMvArgs a) {
    energy_mv_merge_body<L>(a, blockIdx.x);
}

template <int L>
__global__ __launch_bounds__(256) void k_energy_mv_merge_many(const EnMvArgs *as, const int *nb) {
    const int k = blockIdx.y;
    if ((int)blockIdx.x >= nb[k]) return;
    const EnMvArgs a = as[k];
    energy_mv_merge_body<L>(a, blockIdx.x);
}

int energy_slices(int N, int V) {
    if (V <= 0) return 1;
    const int want = (512 + V - 1) / V;          // at least 512 workgroups in all
    const int most = (N + 63) / 64;              // at least 64 rows per slice
    return std::max(1, std::min(want, most));
}

// Slices of the many-vector kernel: about 1024 workgroups over the vector groups, each
// slice at least 16 rows.
static int energy_mv_slices(int N, int groups) {
    const int want = (1024 + groups - 1) / groups;
    const int most = (N + 15) / 16;
    return std::max(1, std::min(want, most));
}

static int energy_mv_group(int L) { return L == 1 ? 64 : L == 2 ? 32 : 16; }

size_t energy_part_bytes(int N, int V) {
    V = std::max(V, 1);
    const size_t old = (size_t)V * energy_slices(N, V) * 2 * sizeof(Acc256);
    size_t mv = 0;
    for (int L = 1; L <= 4; L++) {
        const int G = energy_mv_group(L);
        const int P = energy_mv_slices(N, (V + G - 1) / G);
        const size_t b = (size_t)((V + 63) / 64) * N * 8 +
                         (size_t)energy_mv_layout(P, V, L).total * 8 + 256;
        mv = std::max(mv, b);
    }
    return std::max(old, mv);
}

// Levels of the many-vector kernel for instance I (0: it does not apply).
static int energy_levels(const Instance &I, double *K) {
    for (int k = 0; k < 4; k++) K[k] = 0.0;
    if (I.layout != HQA_DENSE || I.es.lsb == INT32_MIN) return 0;
    const double terms = (double)I.N * I.N + I.N;
    int lg = 0;
    while (lg < 64 && std::ldexp(1.0, lg) < terms) lg++;
    const int w = 51 - lg;
    if (w < 8) return 0;
    const int span = I.es.msb + 1 - I.es.lsb;
    const int L = std::max(1, (span + w - 1) / w);
    // the rounding constants stay normal binary64 numbers
    if (L > 4 || I.es.lsb + 52 < -1022 || I.es.lsb + (L - 1) * w + 52 > 1000) return 0;
    for (int k = 1; k < L; k++) K[k] = std::ldexp(1.5, I.es.lsb + k * w + 52);
    return L;
}

template <int L>
static void launch_mv(EnMvArgs &a, hipStream_t st) {
    constexpr int G = L == 1 ? 64 : L == 2 ? 32 : 16;
    const int groups = (a.V + G - 1) / G;
    a.P = energy_mv_slices(a.N, groups);
    k_energy_mv<G, L><<<dim3(a.P, groups), 256, 0, st>>>(a);
    k_energy_mv_merge<L><<<(a.V + 3) / 4, 256, 0, st>>>(a);
}

hipError_t launch_energy(const Instance &I, int V, const int8_t *spins, double *E, double *cut,
                         void *part, hipStream_t st) {
    if (V == 0) return hipSuccess;
    EnMvArgs m;
    const int L = energy_levels(I, m.K);
    if (L) {
        m.N = I.N; m.V = V; m.b0 = I.es.lsb;
        m.J = I.J64; m.h = I.h64; m.spins = spins; m.E = E; m.cut = cut;
        // the compact storage copy when it holds every coupling exactly
        m.jt = -1; m.ldj = 0; m.Js = nullptr;
        if (I.js_exact && I.Js) {
            m.jt = (int)I.jt; m.ldj = I.Np; m.Js = I.Js;
        }
        m.masks = (uint64_t *)part;
        const size_t mw = (size_t)((V + 63) / 64) * I.N;
        m.part = (double *)((uint8_t *)part + ((mw * 8 + 255) & ~(size_t)255));
        k_pack_masks<<<(unsigned)((mw + 255) / 256), 256, 0, st>>>(I.N, V, spins, m.masks);
        if (L == 1) launch_mv<1>(m, st);
        else if (L == 2) launch_mv<2>(m, st);
        else if (L == 3) launch_mv<3>(m, st);
        else launch_mv<4>(m, st);
        return hipGetLastError();
    }
    EnArgs a;
    a.N = I.N; a.V = V; a.P = energy_slices(I.N, V); a.csr = I.layout == HQA_CSR; a.b0 = I.es.lsb;
    // Every J and h is a multiple of 2^lsb below 2^(msb + 1); the sums take at most
    // N^2 + N terms of magnitude below 2^(msb + 2) (2h).  When those fit 53 bits above
    // 2^lsb, every partial binary64 sum is exact, whatever the order.
    {
        const double terms = (double)I.N * I.N + I.N;
        int lg = 0;
        while (lg < 64 && std::ldexp(1.0, lg) < terms) lg++;
        a.fast = I.es.lsb != INT32_MIN && (I.es.msb + 2 - I.es.lsb) + lg <= 52;
    }
    a.J = I.J64; a.rp = I.rp; a.ci = I.ci; a.h = I.h64; a.spins = spins; a.part = part;
    a.E = E; a.cut = cut;
    k_energy<<<V * a.P, 256, 0, st>>>(a);
    k_energy_merge<<<(V + 63) / 64, 64, 0, st>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The read-out of many instances (same R, n and solve) in one launch per stage: every
// stage's kernel runs for all instances at once (instance = the last grid dimension,
// each with its own block count), in the order select, reduce, enumerate, merge,
// energy, so the many small grids of one instance no longer leave the device idle.
// Each stage computes exactly what the per-instance launches compute.
// ---------------------------------------------------------------------------
namespace {
struct Blob {
    std::vector<uint8_t> h;
    size_t put(const void *p, size_t n) {
        const size_t off = (h.size() + 255) & ~(size_t)255;
        h.resize(off + n);
        memcpy(h.data() + off, p, n);
        return off;
    }
};
template <class T>
size_t put_vec(Blob &b, const std::vector<T> &v) { return b.put(v.data(), v.size() * sizeof(T)); }
}  // namespace

size_t readout_batch_arg_bytes(int count) {
    // the argument arrays and their block counts, each rounded to 256 bytes
    const size_t per = sizeof(EnMvArgs) + sizeof(EnumRealArgs) + sizeof(EnumArgs) + sizeof(SelArgs) +
                       sizeof(RedArgs) + sizeof(MergeArgs) + sizeof(PackArgs) + 24 * sizeof(int);
    return (size_t)count * per + 40 * 256;
}

hipError_t launch_readout_batch(const std::vector<ReadoutJob> &jobs, int R, int n, int solve,
                                void *argbuf, size_t argcap, hipStream_t st, int mode) {
    const int count = (int)jobs.size();
    if (count == 0) return hipSuccess;
    Blob b;
    // select
    std::vector<SelArgs> sel(count);
    std::vector<int> nsel(count, R);
    for (int c = 0; c < count; c++) {
        const ReadoutJob &j = jobs[c];
        SelArgs &a = sel[c];
        a.N = j.I->N; a.R = R; a.ld = j.I->ld; a.smaj = j.I->smaj; a.f64 = j.prec == HQA_PREC_F64_REF;
        a.W = j.W; a.n = n; a.S64 = j.I->S64; a.S32 = j.I->S32; a.amb = j.amb; a.spins = j.spins;
        a.keys = nullptr;
    }
    const size_t o_sel = put_vec(b, sel), o_nsel = put_vec(b, nsel);
    // reduce, enumerate, merge (exact solution of the reduced problems)
    const bool solving = solve && n > 0;
    std::vector<RedArgs> red;
    std::vector<EnumRealArgs> er;
    std::vector<EnumArgs> ei;
    std::vector<MergeArgs> mg;
    std::vector<int> nred, ner, nmid, nei, nmg;
    const int pt = n < ENUM_PT_REAL ? n : ENUM_PT_REAL;
    const int Pe = ((1 << pt) + 255) / 256;
    if (solving) {
        for (int c = 0; c < count; c++) {
            const ReadoutJob &j = jobs[c];
            const Instance &I = *j.I;
            RedArgs a;
            a.N = I.N; a.R = R; a.n = n; a.csr = I.layout == HQA_CSR; a.b0 = I.es.lsb;
            a.J = I.J64; a.rp = I.rp; a.ci = I.ci; a.h = I.h64;
            a.amb = j.amb; a.spins = j.spins; a.h_eff = j.h_eff; a.J_eff = j.J_eff;
            red.push_back(a);
            nred.push_back((R * n + 3) / 4);
            if (!I.j_integral) {
                EnumRealArgs e;
                e.n = n; e.R = R; e.P = Pe; e.b0 = I.es.lsb;
                e.J_eff = j.J_eff; e.h_eff = j.h_eff; e.code = j.code; e.e_red = j.e_red;
                e.partE = (double *)j.escr;
                e.partC = (int64_t *)((char *)j.escr + (size_t)R * e.P * 8);
                e.thresh = (double *)((char *)j.escr + (size_t)R * e.P * 16);
                er.push_back(e);
                ner.push_back(R * Pe);
                nmid.push_back(R);
            } else {
                EnumArgs e;
                e.n = n; e.R = R; e.b0 = I.es.lsb; e.integral = 1;
                e.J_eff = j.J_eff; e.h_eff = j.h_eff; e.code = j.code; e.e_red = j.e_red;
                ei.push_back(e);
                nei.push_back(R);
            }
            MergeArgs m;
            m.N = I.N; m.R = R; m.n = n; m.amb = j.amb; m.code = j.code; m.spins = j.spins;
            mg.push_back(m);
            nmg.push_back((R * n + 255) / 256);
        }
    }
    const size_t o_red = put_vec(b, red), o_nred = put_vec(b, nred);
    const size_t o_er = put_vec(b, er), o_ner = put_vec(b, ner), o_nmid = put_vec(b, nmid);
    const size_t o_ei = put_vec(b, ei), o_nei = put_vec(b, nei);
    const size_t o_mg = put_vec(b, mg), o_nmg = put_vec(b, nmg);
    // energy: the many-vector kernel by level count; others one instance at a time
    std::vector<PackArgs> pk;
    std::vector<int> npk;
    std::vector<EnMvArgs> mv[5];
    std::vector<int> nmv[5], nmm[5];   // slices of the sums, blocks of the merge
    std::vector<int> fallback;
    for (int c = 0; c < count; c++) {
        const ReadoutJob &j = jobs[c];
        const Instance &I = *j.I;
        EnMvArgs m;
        const int L = energy_levels(I, m.K);
        if (!L) {
            fallback.push_back(c);
            continue;
        }
        m.N = I.N; m.V = R; m.b0 = I.es.lsb;
        m.J = I.J64; m.h = I.h64; m.spins = j.spins; m.E = j.E; m.cut = j.C;
        m.jt = -1; m.ldj = 0; m.Js = nullptr;
        if (I.js_exact && I.Js) {
            m.jt = (int)I.jt; m.ldj = I.Np; m.Js = I.Js;
        }
        m.masks = (uint64_t *)j.part;
        const size_t mw = (size_t)((R + 63) / 64) * I.N;
        m.part = (double *)((uint8_t *)j.part + ((mw * 8 + 255) & ~(size_t)255));
        const int G = energy_mv_group(L);
        m.P = energy_mv_slices(I.N, (R + G - 1) / G);
        PackArgs q;
        q.N = I.N; q.V = R; q.spins = j.spins; q.masks = m.masks;
        pk.push_back(q);
        npk.push_back((int)((mw + 255) / 256));
        mv[L].push_back(m);
        nmv[L].push_back(m.P);
        nmm[L].push_back((R + 3) / 4);
    }
    const size_t o_pk = put_vec(b, pk), o_npk = put_vec(b, npk);
    size_t o_mv[5] = {}, o_nmv[5] = {}, o_nmm[5] = {};
    for (int L = 1; L <= 4; L++) {
        o_mv[L] = put_vec(b, mv[L]);
        o_nmv[L] = put_vec(b, nmv[L]);
        o_nmm[L] = put_vec(b, nmm[L]);
    }
    if (b.h.size() > argcap) return hipErrorInvalidValue;
    // the host copy of the arguments lives only in this call: wait for the upload
    hipError_t e = hipSuccess;
    if (mode != READOUT_LAUNCH) {
        e = hipMemcpyAsync(argbuf, b.h.data(), b.h.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess || mode == READOUT_UPLOAD) return e;
    }
    uint8_t *d = (uint8_t *)argbuf;
    auto mx = [](const std::vector<int> &v) { int m = 0; for (int x : v) m = std::max(m, x); return m; };
    k_select_many<<<dim3(R, count), 256, 0, st>>>((const SelArgs *)(d + o_sel), (const int *)(d + o_nsel));
    if (solving) {
        k_reduce_many<<<dim3(mx(nred), count), 256, 0, st>>>((const RedArgs *)(d + o_red),
                                                            (const int *)(d + o_nred));
        if (!er.empty()) {
            const EnumRealArgs *as = (const EnumRealArgs *)(d + o_er);
            const int *nr = (const int *)(d + o_ner), *nm = (const int *)(d + o_nmid);
            const int ce = (int)er.size();
            for (int pass = 1; pass <= 2; pass++) {
                switch (n - pt) {
#define HQA_ER(NL) case NL: k_enum_real_many<NL><<<dim3(R * Pe, ce), 256, 0, st>>>(as, nr, pass); break;
                    HQA_ER(0) HQA_ER(1) HQA_ER(2) HQA_ER(3) HQA_ER(4) HQA_ER(5) HQA_ER(6)
                    HQA_ER(7) HQA_ER(8) HQA_ER(9) HQA_ER(10) HQA_ER(11)
                    default: k_enum_real_many<12><<<dim3(R * Pe, ce), 256, 0, st>>>(as, nr, pass); break;
#undef HQA_ER
                }
                k_enum_real_mid_many<<<dim3(R, ce), 64, 0, st>>>(as, nm, pass);
            }
        }
        if (!ei.empty()) {
            const EnumArgs *as = (const EnumArgs *)(d + o_ei);
            const int *ni = (const int *)(d + o_nei);
            const int ci = (int)ei.size();
            switch (n > ENUM_PT ? n - ENUM_PT : 0) {
#define HQA_EI(NL) case NL: k_enumerate_int_many<NL><<<dim3(R, ci), 1024, 0, st>>>(as, ni); break;
                HQA_EI(0) HQA_EI(1) HQA_EI(2) HQA_EI(3) HQA_EI(4) HQA_EI(5) HQA_EI(6) HQA_EI(7)
                HQA_EI(8) HQA_EI(9) HQA_EI(10) HQA_EI(11) HQA_EI(12) HQA_EI(13)
                default: k_enumerate_int_many<14><<<dim3(R, ci), 1024, 0, st>>>(as, ni); break;
#undef HQA_EI
            }
        }
        k_merge_many<<<dim3(mx(nmg), count), 256, 0, st>>>((const MergeArgs *)(d + o_mg),
                                                          (const int *)(d + o_nmg));
    }
    if (!pk.empty())
        k_pack_masks_many<<<dim3(mx(npk), (int)pk.size()), 256, 0, st>>>(
            (const PackArgs *)(d + o_pk), (const int *)(d + o_npk));
    for (int L = 1; L <= 4; L++) {
        if (mv[L].empty()) continue;
        const int G = energy_mv_group(L), groups = (R + G - 1) / G, cl = (int)mv[L].size();
        const EnMvArgs *as = (const EnMvArgs *)(d + o_mv[L]);
        const int *np = (const int *)(d + o_nmv[L]), *nq = (const int *)(d + o_nmm[L]);
        const dim3 g1(mx(nmv[L]), groups, cl), g2((R + 3) / 4, cl);
        if (L == 1) { k_energy_mv_many<64, 1><<<g1, 256, 0, st>>>(as, np); k_energy_mv_merge_many<1><<<g2, 256, 0, st>>>(as, nq); }
        if (L == 2) { k_energy_mv_many<32, 2><<<g1, 256, 0, st>>>(as, np); k_energy_mv_merge_many<2><<<g2, 256, 0, st>>>(as, nq); }
        if (L == 3) { k_energy_mv_many<16, 3><<<g1, 256, 0, st>>>(as, np); k_energy_mv_merge_many<3><<<g2, 256, 0, st>>>(as, nq); }
        if (L == 4) { k_energy_mv_many<16, 4><<<g1, 256, 0, st>>>(as, np); k_energy_mv_merge_many<4><<<g2, 256, 0, st>>>(as, nq); }
    }
    for (int c : fallback) {
        const ReadoutJob &j = jobs[c];
        e = launch_energy(*j.I, R, j.spins, j.E, j.C, j.part, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Single-flip tabu search on each replica's reduced problem, for n beyond exact
// enumeration (the paper hands n = 1000 ambivalent spins to a tabu search in its
// K2000 experiment; the search itself is this library's reading):
//   x = the read-out of the ambivalent spins; f_a = h_eff_a + sum_{b != a} J_ab x_b
//   (b ascending); D = 0, D_best = 0; for t = 1 .. iters: d_a = -2 x_a f_a; a move is
//   allowed when tabu_until[a] < t or D + d_a < D_best; a* = the allowed a with the
//   smallest d_a (ties: smallest a); D += d_a*; f_b -= 2 J_a*b x_a* (old value) for
//   b != a*; x_a* = -x_a*; tabu_until[a*] = t + tenure; if D < D_best keep x.
// One workgroup of 1024 threads per replica, up to TABU_SPT spins per thread; J_ab is
// read from the instance's binary64 couplings at the ambivalent indices.  The
// operations are those of the definition in binary64 without contraction, so the
// trajectory is the same whatever the launch shape.  Each move costs one workgroup
// barrier (the wavefronts' candidates go to LDS slots double-buffered by parity).
// ---------------------------------------------------------------------------
#define TABU_SPT 4
struct TabuArgs {
    int N, R, n, csr, tenure;
    int64_t iters;
    const double *J;
    const int32_t *rp, *ci;
    const int32_t *amb;
    const int8_t *spins;
    const double *h_eff;
    int8_t *spins_out;    // read-out with the best configuration merged in
    double *d_best;
};

__device__ __forceinline__ double tabu_j(const TabuArgs &a, int i, int j) {
    if (!a.csr) return a.J[(int64_t)i * a.N + j];
    int lo = a.rp[i], hi = a.rp[i + 1];
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a.ci[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < a.rp[i + 1] && a.ci[lo] == j) ? a.J[lo] : 0.0;
}

// The better of two candidates (gain d, key 2 index + [old spin > 0]): smaller d, ties
// to the smaller index.  Indices are distinct, so this is a total order and any
// reduction tree picks the same candidate.
__device__ __forceinline__ void tabu_better(double &d, int &key, double d2, int key2) {
    if (d2 < d || (d2 == d && key2 < key)) { d = d2; key = key2; }
}

// One reduction level between lane pairs given by a DPP pattern inside 16-lane rows
// (quad permutations, half-row and row mirrors): register moves, no LDS.
template <int CTRL>
__device__ __forceinline__ void tabu_dpp(double &d, int &key) {
    const int lo = __double2loint(d), hi = __double2hiint(d);
    const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
    const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
    const int k2 = __builtin_amdgcn_update_dpp(key, key, CTRL, 0xF, 0xF, false);
    tabu_better(d, key, __hiloint2double(hi2, lo2), k2);
}

// The level between lane l and l ^ 16 (ROW32 = false) or l ^ 32: the permlane swaps
// hand every lane both members of its pair, and both take the better one.
template <bool ROW32>
__device__ __forceinline__ void tabu_swap(double &d, int &key) {
    const unsigned lo = (unsigned)__double2loint(d), hi = (unsigned)__double2hiint(d);
    const auto l = ROW32 ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                         : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = ROW32 ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                         : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const auto k = ROW32 ? __builtin_amdgcn_permlane32_swap((unsigned)key, (unsigned)key, false, false)
                         : __builtin_amdgcn_permlane16_swap((unsigned)key, (unsigned)key, false, false);
    d = __hiloint2double((int)h[0], (int)l[0]);
    key = (int)k[0];
    tabu_better(d, key, __hiloint2double((int)h[1], (int)l[1]), (int)k[1]);
}

// Best candidate of the 16 lanes of each row: quad xor 1 and 2, then the half-row
// mirror (lane i with 7 - i) and the row mirror (i with 15 - i).
__device__ __forceinline__ void tabu_row_min(double &d, int &key) {
    tabu_dpp<0xB1>(d, key);    // quad_perm [1, 0, 3, 2]
    tabu_dpp<0x4E>(d, key);    // quad_perm [2, 3, 0, 1]
    tabu_dpp<0x141>(d, key);   // row_half_mirror
    tabu_dpp<0x140>(d, key);   // row_mirror
}

__global__ __launch_bounds__(1024) void k_tabu(TabuArgs a) {
    __shared__ int8_t sx[TABU_SPT * 1024];      // starting spins of the ambivalent set
    __shared__ int32_t sA[TABU_SPT * 1024];     // their indices (a move reads one)
    __shared__ double sd[2][16];
    __shared__ int sk[2][16];
    const int r = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int n = a.n, N = a.N;
    const int32_t *A = a.amb + (int64_t)r * n;
    const int8_t *s0 = a.spins + (int64_t)r * N;
    for (int b = tid; b < n; b += 1024) {
        const int i = A[b];
        sA[b] = i;
        sx[b] = s0[i];
    }
    __syncthreads();
    double f[TABU_SPT];
    int x[TABU_SPT], xb[TABU_SPT], Ai[TABU_SPT];
    int64_t until[TABU_SPT];
#pragma unroll
    for (int k = 0; k < TABU_SPT; k++) {
        const int ai = tid + 1024 * k;
        f[k] = 0.0; x[k] = 1; xb[k] = 1; Ai[k] = 0; until[k] = 0;
        if (ai < n) {
            Ai[k] = sA[ai];
            x[k] = xb[k] = sx[ai];
            double acc = a.h_eff[(int64_t)r * n + ai];
            if (!a.csr) {
                // the loads of a row are independent, so several are in flight; the
                // sum itself keeps the order b = 0, 1, ...
                const double *Jr = a.J + (int64_t)Ai[k] * N;
#pragma unroll 8
                for (int b = 0; b < n; b++) {
                    const double J = Jr[sA[b]];
                    if (b != ai) acc = acc + J * (double)sx[b];
                }
            } else {
                for (int b = 0; b < n; b++)
                    if (b != ai) acc = acc + tabu_j(a, Ai[k], sA[b]) * (double)sx[b];
            }
            f[k] = acc;
        }
    }
    const int tenure = min(a.tenure, n - 1);
    double D = 0.0, Db = 0.0;
    for (int64_t t = 1; t <= a.iters; t++) {
        const int par = (int)(t & 1);
        double bd = INFINITY;
        int bk = INT_MAX;
#pragma unroll
        for (int k = 0; k < TABU_SPT; k++) {
            const int ai = tid + 1024 * k;
            if (ai >= n) continue;
            const double d = x[k] > 0 ? -2.0 * f[k] : 2.0 * f[k];
            if (until[k] < t || D + d < Db) tabu_better(bd, bk, d, 2 * ai + (x[k] > 0));
        }
        tabu_row_min(bd, bk);
        tabu_swap<false>(bd, bk);
        tabu_swap<true>(bd, bk);
        if (lane == 0) { sd[par][w] = bd; sk[par][w] = bk; }
        __syncthreads();
        // each wavefront combines the 16 slots: lane v takes slot v mod 16
        bd = sd[par][lane & 15];
        bk = sk[par][lane & 15];
        tabu_row_min(bd, bk);
        const int bi = bk >> 1, bo = (bk & 1) ? 1 : -1;
        // At most tenure < n spins are tabu, so some move is allowed; only gains that
        // are all NaN (fields overflowed) leave none.  bi is the same in every thread.
        if (bk == INT_MAX) break;
        D = D + bd;
        const int rowj = sA[bi];
#pragma unroll
        for (int k = 0; k < TABU_SPT; k++) {
            const int ai = tid + 1024 * k;
            if (ai >= n) continue;
            if (ai == bi) {
                x[k] = -x[k];
                until[k] = t + tenure;
            } else {
                const double J = tabu_j(a, rowj, Ai[k]);
                f[k] = f[k] - (bo > 0 ? 2.0 * J : -2.0 * J);
            }
        }
        if (D < Db) {   // uniform
            Db = D;
#pragma unroll
            for (int k = 0; k < TABU_SPT; k++) xb[k] = x[k];
        }
    }
    int8_t *so_r = a.spins_out + (int64_t)r * N;
#pragma unroll
    for (int k = 0; k < TABU_SPT; k++) {
        const int ai = tid + 1024 * k;
        if (ai < n) so_r[Ai[k]] = (int8_t)xb[k];
    }
    if (tid == 0) a.d_best[r] = Db;
}

hipError_t launch_tabu(const Instance &I, int R, int n, const int32_t *amb, const int8_t *spins,
                       const double *h_eff, int64_t iters, int tenure, int8_t *spins_out,
                       double *d_best, hipStream_t st) {
    TabuArgs a;
    a.N = I.N; a.R = R; a.n = n; a.csr = I.layout == HQA_CSR; a.tenure = tenure; a.iters = iters;
    a.J = I.J64; a.rp = I.rp; a.ci = I.ci; a.amb = amb; a.spins = spins; a.h_eff = h_eff;
    a.spins_out = spins_out; a.d_best = d_best;
    if (R == 0 || n == 0) return hipSuccess;
    k_tabu<<<R, 1024, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace hqa
