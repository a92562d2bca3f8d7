// k_md_batch.hip -- one MD step of many dense instances in one launch.
//
// A batch of uneven instances (sizes N_k, one shared schedule and replica count)
// advances step by step; each step is one launch over a tile table of (instance, 128
// rows, 64 replicas) tiles, whatever the storage type (FP32, BF16, FP8), so with 64
// replicas each J row block is read once per step.  An FP8 instance whose couplings are
// all 0 or 1 (unit-weight MAX-CUT) is streamed from a copy with one bit per coupling,
// expanded in registers to the same BF16 operands.  The tiles of an instance share
// one XCD, and instances are placed longest-first (LPT by padded size), so the largest
// instances start first and the short tiles fill the tail of the step.  The field
// uses the chunk-to-chain decomposition of the other dense kernels, and the update
// the same binary32 sequence, so a batched instance evolves bit-identically to the
// same instance run alone.
#include <algorithm>
#include <type_traits>

#include "hqa_internal.h"
#include "md_epilogue.h"

namespace hqa {

typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2_b;

__device__ __forceinline__ bf16x8 cvt_fp8x8_b(uint2 raw) {
    bf16x2_b a = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.x, 1.0f, false);
    bf16x2_b b = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.x, 1.0f, true);
    bf16x2_b c = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.y, 1.0f, false);
    bf16x2_b d = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.y, 1.0f, true);
    bf16x8 o;
    o[0] = a[0]; o[1] = a[1]; o[2] = b[0]; o[3] = b[1];
    o[4] = c[0]; o[5] = c[1]; o[6] = d[0]; o[7] = d[1];
    return o;
}

struct BatchInst {
    int N, Np, ld, jt;
    const void *J;
    const void *Jt;       // MFMA-tiled copy of J (BF16 / FP8 storage, or bits for JT_BIT)
    int nrounds;          // 128-column groups per row (Np / 128)
    const float *h;
    float *phi[2];
    bf16 *xb[2];
    float *p, *S;
};

struct BatchTile {
    int inst, i0, r0, pad;
};

struct BatchArgs {
    const BatchInst *inst;
    const BatchTile *tiles;
    int ntiles, R, M, W, cur;
    int64_t T;
    float rg;
    const float *a32, *b32;
    int32_t *err;
};

// BF16 / FP8 storage: tiles of 128 rows x 64 replicas, eight wavefronts, wavefront w
// owning row tile i0 + 16 w and all four replica tiles.  Per 128-column group the
// flux operand block (64 replicas x 128 columns, BF16) is staged once into LDS by
// the whole workgroup with full-line loads and shared by the eight row tiles, so it
// is read from L2 once per 128 rows instead of once per 32; the J fragments come
// from the MFMA-tiled copy, one group ahead in registers; the LDS block is double-
// buffered with one barrier per group.  Chains, operands and epilogue are those of
// the other dense kernels (bit-identical results).  Wavefronts whose rows are all
// padding compute on a real row tile, store nothing, and take part in the staging and
// the barriers.  The kernel is held to 128 VGPRs so that two workgroups share a
// compute unit: each covers the other's memory waits, tile prologue and epilogue.  On
// the 512-instance batch that beat one workgroup per CU with a three-deep register
// prefetch and the epilogue's loads issued early (220 VGPRs) by 4%.
//
// Every global access goes through global-address-space pointers.  The buffers come
// from a table in memory, so plain pointers would be generic (flat) ones, and a flat
// load counts against the LDS counter as well: the wait for the B fragments' LDS reads
// would then also wait for the next group's prefetch, and every group would pay the
// whole memory latency.  Global loads count only against the vector-memory counter,
// so the prefetch stays in flight across the group's MFMAs and its barrier.
constexpr int BL_ROWS = 128, BL_REPS = 64, BL_LDB = 128 + 8;   // LDS row: 272 bytes

template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gld(const void *p) {
    return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gst(void *p) {
    return (__attribute__((address_space(1))) T *)p;
}

typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4_b;

// The four K chunks of one 128-column group as BF16 operands: from four 16-byte words
// (BF16 storage) or from the eight FP8 bytes of each chunk in two words (FP8 storage).
// Eight couplings of value 0 or 1 (bit e = element e) as eight BF16 operands: each pair
// of bits t becomes the word t0 * 0x3F80 + t1 * 0x3F800000 (BF16 1.0 = 0x3F80).
__device__ __forceinline__ bf16x8 bits_to_bf16x8(uint32_t byte) {
    u32x4_b o;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const uint32_t t = (byte >> (2 * i)) & 3u;
        const uint32_t m = (t * 0x8001u) & 0x10001u;   // bit 0 -> bit 0, bit 1 -> bit 16
        o[i] = m * 0x3F80u;
    }
    return __builtin_bit_cast(bf16x8, o);
}

template <int JT, typename W>
__device__ __forceinline__ bf16x8 a_chunk(const W *g, int j) {
    if constexpr (JT == JT_BIT) {
        return bits_to_bf16x8((g[0] >> (8 * j)) & 0xFFu);
    } else if constexpr (JT == JT_BF16) {
        return __builtin_bit_cast(bf16x8, g[j]);
    } else {
        const u32x4_b w = g[j >> 1];
        return (j & 1) ? cvt_fp8x8_b(make_uint2(w[2], w[3])) : cvt_fp8x8_b(make_uint2(w[0], w[1]));
    }
}

template <int JT>
__device__ __forceinline__ void batch_lds_tile(const BatchArgs &a, int64_t q, const BatchTile &tl,
                                               const BatchInst &I,
                                               bf16 (&Bs)[2][BL_REPS][BL_LDB]) {
    const int tid = threadIdx.x, lane = tid & 63, kg = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i0 = tl.i0 + 16 * w;
    const int r0 = tl.r0;
    // buffers of the current parity, chosen without run-time indexing of the table
    const bool odd = a.cur != 0;
    const float *phi_in = odd ? I.phi[1] : I.phi[0];
    const bf16 *xb_in = odd ? I.xb[1] : I.xb[0];
    float *phi_out = odd ? I.phi[0] : I.phi[1];
    bf16 *xb_out = odd ? I.xb[0] : I.xb[1];
    const int ngroups = I.Np / 128;
    // words of J per lane and group: 16-byte words of BF16 or FP8, or one 32-bit word of
    // bits (four chunks of eight couplings)
    using JW = typename std::conditional<JT == JT_BIT, uint32_t, u32x4_b>::type;
    constexpr int NA = JT == JT_BF16 ? 4 : JT == JT_FP8 ? 2 : 1;
    // the tiled copy holds ceil(N / 16) row tiles: a wavefront whose rows are all
    // padding reads the last real row tile instead (its results are never stored)
    // (wavefront-uniform bases and 32-bit per-lane offsets: the offsets take one register
    // each where a per-lane pointer takes two)
    const int jtile = min(i0, I.N - 1) / 16;
    const auto *Jt = gld<JW>((const uint8_t *)I.Jt + (int64_t)jtile * I.nrounds * 64 * (int)sizeof(JW) * NA);
    const int jl = lane * NA;
    // staging: thread -> (replica row, 16-column segment) of the 64 x 128 block
    const int srow = tid >> 3, sseg = tid & 7;
    const auto *Bsrc = gld<u32x4_b>(xb_in + (int64_t)r0 * I.ld);
    const int sl = ((min(r0 + srow, a.R - 1) - r0) * I.ld + 16 * sseg) / 8;
    u32x4_b *Bdst0 = (u32x4_b *)&Bs[0][srow][16 * sseg];
    u32x4_b *Bdst1 = (u32x4_b *)&Bs[1][srow][16 * sseg];

    f32x4 acc[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; rt++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[rt][j] = (f32x4){0.f, 0.f, 0.f, 0.f};

    // Two register sets for the couplings, one for the fluxes: the couplings and the
    // fluxes of group g + 1 are requested when group g begins (the loop is unrolled by
    // two, so no set is copied into the other).  The fluxes are requested first: loads
    // complete in order, so the wait that lets them go to LDS at the end of group g
    // leaves the couplings in flight across the barrier.  At 128 VGPRs two workgroups
    // share a CU, and each covers the other's waits, prologue and epilogue.
    JW A0[NA], A1[NA];
    u32x4_b S0a, S0b;
#define HQA_LOAD_J(g, A)                                                              \
    do {                                                                              \
        _Pragma("unroll") for (int j = 0; j < NA; j++) A[j] = Jt[(g) * 64 * NA + jl + j]; \
    } while (0)
#define HQA_LOAD_S(g, Sa, Sb)                                                         \
    do {                                                                              \
        Sa = Bsrc[sl + 16 * (g)];                                                     \
        Sb = Bsrc[sl + 16 * (g) + 1];                                                 \
    } while (0)
#define HQA_MFMA_GROUP(buf, A)                                                        \
    do {                                                                              \
        _Pragma("unroll") for (int j = 0; j < 4; j++) {                              \
            const bf16x8 av = a_chunk<JT>(A, j);                                      \
            _Pragma("unroll") for (int rt = 0; rt < 4; rt++) {                       \
                const bf16x8 bv = *(const bf16x8 *)&Bs[buf][16 * rt + (lane & 15)][32 * j + 8 * kg]; \
                acc[rt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[rt][j], 0, 0, 0); \
            }                                                                         \
        }                                                                             \
    } while (0)
    const int gl = ngroups - 1;
    if constexpr (JT == JT_BIT) {
        // bit tiles hold two flux register sets (their couplings take one register per
        // set): the fluxes of group g + 2 are requested when group g begins
        u32x4_b S1a, S1b;
        HQA_LOAD_S(0, S0a, S0b);
        HQA_LOAD_J(0, A0);
        Bdst0[0] = S0a;
        Bdst0[1] = S0b;
        __syncthreads();
        HQA_LOAD_S(min(1, gl), S0a, S0b);
        for (int gi = 0; gi < ngroups; gi += 2) {
            HQA_LOAD_S(min(gi + 2, gl), S1a, S1b);
            HQA_LOAD_J(min(gi + 1, gl), A1);
            __builtin_amdgcn_sched_barrier(0);
            HQA_MFMA_GROUP(0, A0);
            Bdst1[0] = S0a;
            Bdst1[1] = S0b;
            __syncthreads();
            if (gi + 1 >= ngroups) break;
            HQA_LOAD_S(min(gi + 3, gl), S0a, S0b);
            HQA_LOAD_J(min(gi + 2, gl), A0);
            __builtin_amdgcn_sched_barrier(0);
            HQA_MFMA_GROUP(1, A1);
            Bdst0[0] = S1a;
            Bdst0[1] = S1b;
            __syncthreads();
        }
    } else {
        HQA_LOAD_S(0, S0a, S0b);
        HQA_LOAD_J(0, A0);
        Bdst0[0] = S0a;
        Bdst0[1] = S0b;
        __syncthreads();
        // even groups compute from A0 and LDS buffer 0, odd ones from A1 and buffer 1
        for (int gi = 0; gi < ngroups; gi += 2) {
            HQA_LOAD_S(min(gi + 1, gl), S0a, S0b);
            HQA_LOAD_J(min(gi + 1, gl), A1);
            __builtin_amdgcn_sched_barrier(0);
            HQA_MFMA_GROUP(0, A0);
            Bdst1[0] = S0a;
            Bdst1[1] = S0b;
            __syncthreads();
            if (gi + 1 >= ngroups) break;
            HQA_LOAD_S(min(gi + 2, gl), S0a, S0b);
            HQA_LOAD_J(min(gi + 2, gl), A0);
            __builtin_amdgcn_sched_barrier(0);
            HQA_MFMA_GROUP(1, A1);
            Bdst0[0] = S0a;
            Bdst0[1] = S0b;
            __syncthreads();
        }
    }
#undef HQA_LOAD_J
#undef HQA_LOAD_S
#undef HQA_MFMA_GROUP

    // Epilogue with full-line accesses: the fields pass through LDS (the flux stages
    // are free after the last barrier), and thread (replica t / 8, j = t % 8) updates
    // rows 32 v + 4 j .. 32 v + 4 j + 3 for v = 0..3, so the eight threads of a replica
    // read and write one whole 128-byte line of fluxes and momenta per instruction.
    {
        float *U = (float *)&Bs[0][0][0];                  // [64 replicas][136]
        constexpr int UL = 136;
#pragma unroll
        for (int rt = 0; rt < 4; rt++) {
            const f32x4 parts[4] = {acc[rt][0], acc[rt][1], acc[rt][2], acc[rt][3]};
            const f32x4 u = combine4(parts);
            *(f32x4 *)&U[(16 * rt + (lane & 15)) * UL + 16 * w + 4 * kg] = u;
        }
        // the fluxes and momenta are requested before the barrier (the couplings'
        // registers are free by now), so their latency overlaps the exchange
        const int rep = tid >> 3, j8 = tid & 7;
        const int col = r0 + rep;
        f32x4 xv[4], pv[4];
        if (col < a.R) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int ib = tl.i0 + 32 * v + 4 * j8;
                if (ib >= I.N) continue;
                const int64_t base = (int64_t)col * I.ld + ib;
                xv[v] = *gld<f32x4>(phi_in + base);
                pv[v] = *gld<f32x4>(I.p + base);
            }
        }
        __syncthreads();
        const StepCoef cf = step_coef(a.a32, a.b32, q, a.rg, a.M);
        const bool win = q + 1 >= a.T - a.W + 1;
        bool bad = false;
        const auto *hg = gld<float>(I.h);
        if (col < a.R) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int loc = 32 * v + 4 * j8;
                const int ib = tl.i0 + loc;
                if (ib >= I.N) continue;
                const f32x4 u = *(const f32x4 *)&U[rep * UL + loc];
                const int64_t base = (int64_t)col * I.ld + ib;
                const f32x4 x = xv[v];
                const f32x4 p = pv[v];
                float xs[4] = {x[0], x[1], x[2], x[3]}, ps[4] = {p[0], p[1], p[2], p[3]}, xn[4];
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    if (ib + e < I.N) {
                        leapfrog(cf, xs[e], u[e], hg[ib + e], ps[e], xn[e]);
                        bad |= !isfinite(xn[e]) || !isfinite(ps[e]);
                    } else {
                        xn[e] = 0.0f;
                        ps[e] = 0.0f;
                    }
                }
                *gst<f32x4>(phi_out + base) = (f32x4){xn[0], xn[1], xn[2], xn[3]};
                *gst<f32x4>(I.p + base) = (f32x4){ps[0], ps[1], ps[2], ps[3]};
                typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
                bf16x4 b = {(bf16)xn[0], (bf16)xn[1], (bf16)xn[2], (bf16)xn[3]};
                *gst<bf16x4>(xb_out + base) = b;
                if (win) {
                    f32x4 s = *gld<f32x4>(I.S + base);
                    s[0] = s[0] + xn[0]; s[1] = s[1] + xn[1]; s[2] = s[2] + xn[2]; s[3] = s[3] + xn[3];
                    *gst<f32x4>(I.S + base) = s;
                }
            }
        }
        if (bad) atomicOr(a.err, ERR_NONFINITE);
    }
}

// FP32 storage: the same tiles, staging, prefetch and epilogue as batch_lds_tile, with
// FP32 couplings read row-major (four 16-byte words per lane per group of 64 columns),
// the FP32 flux block staged in LDS (64 replicas x 64 columns), and 16x16x4 FP32 MFMAs:
// chunk j of 16 columns feeds chain j, its four MFMAs taking columns 4 kg + e, e = 0..3,
// in that order -- the operand order of every FP32 dense plan (bit-identical results).
__device__ __forceinline__ void batch_f32_tile(const BatchArgs &a, int64_t q, const BatchTile &tl,
                                               const BatchInst &I,
                                               bf16 (&Bsh)[2][BL_REPS][BL_LDB]) {
    typedef float BsRow[BL_LDB / 2];
    BsRow *Bs0 = (BsRow *)&Bsh[0][0][0];
    BsRow *Bs1 = (BsRow *)&Bsh[1][0][0];
    const int tid = threadIdx.x, lane = tid & 63, kg = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i0 = tl.i0 + 16 * w;
    const int r0 = tl.r0;
    // buffers of the current parity, chosen without run-time indexing of the table
    const bool odd = a.cur != 0;
    const float *phi_in = odd ? I.phi[1] : I.phi[0];
    float *phi_out = odd ? I.phi[0] : I.phi[1];
    bf16 *xb_out = odd ? I.xb[0] : I.xb[1];
    const int ngroups = I.Np / 64;
    constexpr int NA = 4;                              // 16-byte words of J per lane and group
    // row-major FP32 couplings with pitch Np: rows up to Np - 1 exist (zero padding), so
    // a wavefront whose rows are all padding reads zeros (its results are never stored)
    const auto *Jt = gld<u32x4_b>((const float *)I.J + (int64_t)(i0 + (lane & 15)) * I.Np + 4 * kg);
    // staging: thread -> (replica row, 8-column segment) of the 64 x 64 FP32 block
    const int srow = tid >> 3, sseg = tid & 7;
    const auto *Bsrc = gld<u32x4_b>(phi_in + (int64_t)min(r0 + srow, a.R - 1) * I.ld + 8 * sseg);
    u32x4_b *Bdst0 = (u32x4_b *)&Bs0[srow][8 * sseg];
    u32x4_b *Bdst1 = (u32x4_b *)&Bs1[srow][8 * sseg];

    f32x4 acc[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; rt++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[rt][j] = (f32x4){0.f, 0.f, 0.f, 0.f};

    // Two register sets for the couplings, one for the fluxes, as in batch_lds_tile.
    u32x4_b A0[NA], A1[NA];
    u32x4_b S0a, S0b;
#define HQA_LOAD_J(g, A)                                                              \
    do {                                                                              \
        _Pragma("unroll") for (int j = 0; j < NA; j++) A[j] = Jt[(int64_t)(g) * 16 + 4 * j]; \
    } while (0)
#define HQA_LOAD_S(g, Sa, Sb)                                                         \
    do {                                                                              \
        Sa = Bsrc[16 * (g)];                                                          \
        Sb = Bsrc[16 * (g) + 1];                                                      \
    } while (0)
#define HQA_MFMA_GROUP(buf, A)                                                        \
    do {                                                                              \
        _Pragma("unroll") for (int j = 0; j < 4; j++) {                              \
            const f32x4 av = __builtin_bit_cast(f32x4, A[j]);                         \
            _Pragma("unroll") for (int rt = 0; rt < 4; rt++) {                       \
                const f32x4 bv = *(const f32x4 *)&((buf) ? Bs1 : Bs0)[16 * rt + (lane & 15)][16 * j + 4 * kg]; \
                _Pragma("unroll") for (int e = 0; e < 4; e++)                        \
                    acc[rt][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[e], bv[e], acc[rt][j], 0, 0, 0); \
            }                                                                         \
        }                                                                             \
    } while (0)
    const int gl = ngroups - 1;
    HQA_LOAD_S(0, S0a, S0b);
    HQA_LOAD_J(0, A0);
    Bdst0[0] = S0a;
    Bdst0[1] = S0b;
    __syncthreads();
    for (int gi = 0; gi < ngroups; gi += 2) {
        HQA_LOAD_S(min(gi + 1, gl), S0a, S0b);
        HQA_LOAD_J(min(gi + 1, gl), A1);
        __builtin_amdgcn_sched_barrier(0);
        HQA_MFMA_GROUP(0, A0);
        Bdst1[0] = S0a;
        Bdst1[1] = S0b;
        __syncthreads();
        if (gi + 1 >= ngroups) break;
        HQA_LOAD_S(min(gi + 2, gl), S0a, S0b);
        HQA_LOAD_J(min(gi + 2, gl), A0);
        __builtin_amdgcn_sched_barrier(0);
        HQA_MFMA_GROUP(1, A1);
        Bdst0[0] = S0a;
        Bdst0[1] = S0b;
        __syncthreads();
    }
#undef HQA_LOAD_J
#undef HQA_LOAD_S
#undef HQA_MFMA_GROUP

    // Epilogue with full-line accesses: the fields pass through LDS (the flux stages
    // are free after the last barrier), and thread (replica t / 8, j = t % 8) updates
    // rows 32 v + 4 j .. 32 v + 4 j + 3 for v = 0..3, so the eight threads of a replica
    // read and write one whole 128-byte line of fluxes and momenta per instruction.
    {
        float *U = (float *)&Bsh[0][0][0];                 // [64 replicas][136]
        constexpr int UL = 136;
#pragma unroll
        for (int rt = 0; rt < 4; rt++) {
            const f32x4 parts[4] = {acc[rt][0], acc[rt][1], acc[rt][2], acc[rt][3]};
            const f32x4 u = combine4(parts);
            *(f32x4 *)&U[(16 * rt + (lane & 15)) * UL + 16 * w + 4 * kg] = u;
        }
        // the fluxes and momenta are requested before the barrier (the couplings'
        // registers are free by now), so their latency overlaps the exchange
        const int rep = tid >> 3, j8 = tid & 7;
        const int col = r0 + rep;
        f32x4 xv[4], pv[4];
        if (col < a.R) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int ib = tl.i0 + 32 * v + 4 * j8;
                if (ib >= I.N) continue;
                const int64_t base = (int64_t)col * I.ld + ib;
                xv[v] = *gld<f32x4>(phi_in + base);
                pv[v] = *gld<f32x4>(I.p + base);
            }
        }
        __syncthreads();
        const StepCoef cf = step_coef(a.a32, a.b32, q, a.rg, a.M);
        const bool win = q + 1 >= a.T - a.W + 1;
        bool bad = false;
        const auto *hg = gld<float>(I.h);
        if (col < a.R) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int loc = 32 * v + 4 * j8;
                const int ib = tl.i0 + loc;
                if (ib >= I.N) continue;
                const f32x4 u = *(const f32x4 *)&U[rep * UL + loc];
                const int64_t base = (int64_t)col * I.ld + ib;
                const f32x4 x = xv[v];
                const f32x4 p = pv[v];
                float xs[4] = {x[0], x[1], x[2], x[3]}, ps[4] = {p[0], p[1], p[2], p[3]}, xn[4];
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    if (ib + e < I.N) {
                        leapfrog(cf, xs[e], u[e], hg[ib + e], ps[e], xn[e]);
                        bad |= !isfinite(xn[e]) || !isfinite(ps[e]);
                    } else {
                        xn[e] = 0.0f;
                        ps[e] = 0.0f;
                    }
                }
                *gst<f32x4>(phi_out + base) = (f32x4){xn[0], xn[1], xn[2], xn[3]};
                *gst<f32x4>(I.p + base) = (f32x4){ps[0], ps[1], ps[2], ps[3]};
                if (xb_out) {   // an operand copy exists only when a BF16 plan may read it
                    typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
                    bf16x4 b = {(bf16)xn[0], (bf16)xn[1], (bf16)xn[2], (bf16)xn[3]};
                    *gst<bf16x4>(xb_out + base) = b;
                }
                if (win) {
                    f32x4 s = *gld<f32x4>(I.S + base);
                    s[0] = s[0] + xn[0]; s[1] = s[1] + xn[1]; s[2] = s[2] + xn[2]; s[3] = s[3] + xn[3];
                    *gst<f32x4>(I.S + base) = s;
                }
            }
        }
        if (bad) atomicOr(a.err, ERR_NONFINITE);
    }
}

// One launch per MD step for every BF16 and FP8 instance of the batch: the storage
// type is uniform per tile.  A tile with instance index -1 is a placeholder of the
// XCD placement and does nothing.
__global__ __launch_bounds__(512, 4) void k_step_batch_lds(BatchArgs a, int64_t q) {
    __shared__ __align__(16) bf16 Bs[2][BL_REPS][BL_LDB];
    const BatchTile tl = a.tiles[blockIdx.x];
    if (tl.inst < 0) return;
    const BatchInst I = a.inst[tl.inst];
    if (I.jt == JT_FP8) batch_lds_tile<JT_FP8>(a, q, tl, I, Bs);
    else if (I.jt == JT_BIT) batch_lds_tile<JT_BIT>(a, q, tl, I, Bs);
    else batch_lds_tile<JT_BF16>(a, q, tl, I, Bs);
}

// The same for the FP32 instances of the batch (their own tile table and launch).
__global__ __launch_bounds__(512, 4) void k_step_batch_f32(BatchArgs a, int64_t q) {
    __shared__ __align__(16) bf16 Bs[2][BL_REPS][BL_LDB];
    const BatchTile tl = a.tiles[blockIdx.x];
    if (tl.inst < 0) return;
    const BatchInst I = a.inst[tl.inst];
    batch_f32_tile(a, q, tl, I, Bs);
}

// Device tables of a batch, built once per handle: instance descriptors and the
// tile lists (FP32 storage; BF16 and FP8 storage together).
// A captured run of steps [q0, q1) that starts on flux buffer `cur`: replaying it
// launches the same kernels with the same arguments as the eager path.
struct BatchGraph {
    int64_t q0, q1;
    int cur;
    hipGraphExec_t exec;
};
constexpr size_t BATCH_MAX_GRAPHS = 8;

struct BatchPlan {
    BatchInst *dinst = nullptr;
    BatchTile *dtiles[3] = {nullptr, nullptr, nullptr};
    int ntiles[3] = {0, 0, 0};
    std::vector<BatchGraph> graphs;     // most recently used last
    hipStream_t cap = nullptr;          // capture-only stream (no work runs on it)
};

void free_batch_plan(void *p) {
    BatchPlan *bp = (BatchPlan *)p;
    if (!bp) return;
    for (auto &g : bp->graphs) (void)hipGraphExecDestroy(g.exec);
    if (bp->cap) (void)hipStreamDestroy(bp->cap);
    if (bp->dinst) (void)hipFree(bp->dinst);
    for (int t = 0; t < 3; t++)
        if (bp->dtiles[t]) (void)hipFree(bp->dtiles[t]);
    delete bp;
}

static hipError_t build_plan(hqa_md *md, BatchPlan *&out) {
    BatchPlan *bp = new BatchPlan();
    std::vector<BatchInst> hi;
    std::vector<int> dense;
    for (size_t k = 0; k < md->inst.size(); k++) {
        Instance &I = md->inst[k];
        BatchInst b;
        b.N = I.N; b.Np = I.Np; b.ld = I.ld; b.jt = I.jt;
        b.J = I.Js; b.h = I.h32;
        b.Jt = nullptr;
        b.nrounds = I.Np / 128;
        if (I.layout == HQA_DENSE && (I.jt == JT_BF16 || I.jt == JT_FP8)) {
            // FP8 with every coupling 0 or 1: the 1-bit copy; otherwise (BF16, other FP8)
            // the MFMA-tiled copy of the storage
            hipError_t e = I.jt == JT_FP8 ? ensure_tiled_bits(I, md->stream) : hipSuccess;
            if (e == hipSuccess && I.jbits <= 0) e = ensure_tiled_j(I, md->stream);
            if (e != hipSuccess) {
                delete bp;
                return e;
            }
            if (I.jbits > 0) {
                b.jt = JT_BIT;
                b.Jt = I.Jbits;
            } else {
                b.Jt = I.Jt;
            }
            if (!b.Jt) {   // every streamed form needs its copy
                delete bp;
                return hipErrorInvalidValue;
            }
        }
        b.phi[0] = I.phi32[0]; b.phi[1] = I.phi32[1];
        b.xb[0] = I.phib[0]; b.xb[1] = I.phib[1];
        b.p = I.p32; b.S = I.S32;
        hi.push_back(b);
        if (I.layout == HQA_DENSE) dense.push_back((int)k);
    }
    // longest processing time first: larger padded size first, then instance index
    // (every tile of an instance costs the same, so the order by size is the order by
    // tile work within a storage form)
    std::stable_sort(dense.begin(), dense.end(), [&](int x, int y) {
        return md->inst[x].Np > md->inst[y].Np;
    });
    std::vector<BatchTile> ht[3];
    // Every tile of an instance on one XCD (workgroup b of a launch runs on XCD b mod 8),
    // so the instance's flux operand is fetched into one L2; instances go to the
    // least-loaded XCD, largest first (LPT on the tile count, i.e. on N^2 R work); the
    // per-XCD lists are interleaved into the launch order and padded with placeholder
    // tiles.  An instance with at
    // least an eighth of all the work is split instead: its row blocks are cut into
    // eight contiguous ranges, one per XCD, each with all replica tiles, so every XCD
    // reads an eighth of J and the 64-replica tiles of a row block share its J lines in
    // one L2.
    // one launch for the FP32 instances, one for the BF16 and FP8 ones
    for (int fam = 0; fam < 2; fam++) {
        auto member = [&](const Instance &I) { return (I.jt == JT_F32) == (fam == 0); };
        constexpr int NX = 8;
        std::vector<BatchTile> xl[NX];
        int64_t load[NX] = {0};
        int64_t total = 0;
        // work of a tile: the bytes it streams (its couplings and the staged flux
        // block) plus a fixed cost of its first loads and epilogue (about the time of
        // 256 KB)
        auto tile_work = [&](const Instance &I) -> int64_t {
            const int64_t jb = I.jt == JT_F32 ? 512 : I.jt == JT_BF16 ? 256 : I.jbits > 0 ? 16 : 128;
            return (jb + 128) * (int64_t)I.Np + 262144;
        };
        for (int k : dense) {
            const Instance &I = md->inst[k];
            if (!member(I)) continue;
            total += (int64_t)((I.N + BL_ROWS - 1) / BL_ROWS) * ((md->R + 63) / 64) * tile_work(I);
        }
        for (int k : dense) {
            const Instance &I = md->inst[k];
            if (!member(I)) continue;
            const int nrb = (I.N + BL_ROWS - 1) / BL_ROWS;
            const int64_t tw = tile_work(I);
            const int64_t work = (int64_t)nrb * ((md->R + 63) / 64) * tw;
            if (nrb >= NX && NX * work >= total) {
                for (int x = 0; x < NX; x++) {
                    for (int rb = x * nrb / NX; rb < (x + 1) * nrb / NX; rb++)
                        for (int r0 = 0; r0 < md->R; r0 += 64) {
                            xl[x].push_back({k, rb * BL_ROWS, r0, 0});
                            load[x] += tw;
                        }
                }
                continue;
            }
            int x = 0;
            for (int y = 1; y < NX; y++)
                if (load[y] < load[x]) x = y;
            for (int i0 = 0; i0 < I.N; i0 += BL_ROWS)
                for (int r0 = 0; r0 < md->R; r0 += 64) {
                    xl[x].push_back({k, i0, r0, 0});
                    load[x] += tw;
                }
        }
        size_t longest = 0;
        for (int x = 0; x < NX; x++) longest = std::max(longest, xl[x].size());
        std::vector<BatchTile> &dst = ht[fam == 0 ? JT_F32 : JT_BF16];
        for (size_t j = 0; j < longest; j++)
            for (int x = 0; x < NX; x++)
                dst.push_back(j < xl[x].size() ? xl[x][j] : BatchTile{-1, 0, 0, 0});
    }
    hipError_t e = dev_malloc((void **)&bp->dinst, sizeof(BatchInst) * hi.size());
    if (e == hipSuccess)
        e = hipMemcpy(bp->dinst, hi.data(), sizeof(BatchInst) * hi.size(), hipMemcpyHostToDevice);
    for (int t = 0; t < 3 && e == hipSuccess; t++) {
        bp->ntiles[t] = (int)ht[t].size();
        if (!bp->ntiles[t]) continue;
        e = dev_malloc((void **)&bp->dtiles[t], sizeof(BatchTile) * ht[t].size());
        if (e == hipSuccess)
            e = hipMemcpy(bp->dtiles[t], ht[t].data(), sizeof(BatchTile) * ht[t].size(),
                          hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        free_batch_plan(bp);
        return e;
    }
    out = bp;
    return hipSuccess;
}

// Advance every dense instance of the handle from q0 to q1, one launch per step
// and storage type.  Instances advance in lockstep, so one parity serves all.
// The launches of steps [q0, q1) from flux buffer `cur`, in order, on stream `st`.
static void enqueue_steps(hqa_md *md, const BatchPlan *bp, int64_t q0, int64_t q1, int cur,
                          hipStream_t st) {
    BatchArgs a;
    a.inst = bp->dinst; a.R = md->R; a.M = md->sch.M; a.W = md->sch.W; a.T = md->sch.T;
    a.rg = (float)md->sch.r_g; a.a32 = md->a32; a.b32 = md->b32; a.err = md->err;
    for (int64_t q = q0; q < q1; q++) {
        a.cur = cur;
        for (int t = 0; t < 3; t++) {
            if (!bp->ntiles[t]) continue;
            a.tiles = bp->dtiles[t];
            a.ntiles = bp->ntiles[t];
            if (t == JT_F32) k_step_batch_f32<<<a.ntiles, 512, 0, st>>>(a, q);
            else k_step_batch_lds<<<a.ntiles, 512, 0, st>>>(a, q);   // BF16 and FP8
        }
        cur ^= 1;
    }
}

// The graph of steps [q0, q1) from buffer `cur`: from the cache, else captured on the
// plan's own stream (a capture records the launches without running them, so the
// caller's stream may be any stream, the null stream included) and instantiated.
static hipError_t batch_graph(hqa_md *md, BatchPlan *bp, int64_t q0, int64_t q1, int cur,
                              hipGraphExec_t *out) {
    for (size_t k = 0; k < bp->graphs.size(); k++) {
        const BatchGraph g = bp->graphs[k];
        if (g.q0 == q0 && g.q1 == q1 && g.cur == cur) {
            bp->graphs.erase(bp->graphs.begin() + k);
            bp->graphs.push_back(g);
            *out = g.exec;
            return hipSuccess;
        }
    }
    hipError_t e = hipSuccess;
    if (!bp->cap) e = hipStreamCreateWithFlags(&bp->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(bp->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    enqueue_steps(md, bp, q0, q1, cur, bp->cap);
    hipError_t le = hipGetLastError();
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(bp->cap, &graph);
    if (e == hipSuccess) e = le;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    if (bp->graphs.size() >= BATCH_MAX_GRAPHS) {
        // the least recently used graph; a replay of it already enqueued keeps its own
        // reference in the runtime until it has run
        (void)hipGraphExecDestroy(bp->graphs.front().exec);
        bp->graphs.erase(bp->graphs.begin());
    }
    bp->graphs.push_back({q0, q1, cur, exec});
    *out = exec;
    return hipSuccess;
}

// The storage form the batch plan streams for an instance (JT_F32, JT_BF16, JT_FP8 or
// JT_BIT), or -1 when the plan is not built or the instance is not dense.
int batch_form(const hqa_md *md, int instance) {
    const Instance &I = md->inst[instance];
    if (!md->batch || I.layout != HQA_DENSE) return -1;
    if (I.jt == JT_FP8 && I.jbits > 0) return JT_BIT;
    return I.jt;
}

// 1-bit MFMA-tiled copy of an FP8 storage whose every byte is 0 or 0x38 (1.0): word
// (t, m, lane) holds, at bit 8 k + e, J[16 t + (lane & 15)][128 m + 32 k + 8 (lane >> 4)
// + e] for k = 0..3, e = 0..7 (the A-operand fragments of chunks 4m..4m+3 of row tile t,
// in the order of the FP8 tiled copy).  Any other byte sets *bad.
__global__ void k_tile_bits(const uint8_t *__restrict__ J, int Np, int ntile, int nrounds,
                            uint32_t *__restrict__ out, int32_t *bad) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (t, m, lane)
    const int64_t n = (int64_t)ntile * nrounds * 64;
    if (g >= n) return;
    const int lane = (int)(g & 63);
    const int64_t tm = g >> 6;
    const int m = (int)(tm % nrounds), t = (int)(tm / nrounds);
    const int row = 16 * t + (lane & 15);
    uint32_t w = 0;
    bool odd = false;
    for (int k = 0; k < 4; k++) {
        const uint8_t *src = J + (int64_t)row * Np + 128 * m + 32 * k + 8 * (lane >> 4);
        for (int e = 0; e < 8; e++) {
            const uint8_t v = src[e];
            odd |= v != 0 && v != 0x38;
            w |= (uint32_t)(v == 0x38) << (8 * k + e);
        }
    }
    out[g] = w;
    if (odd) atomicOr(bad, 1);
}

// Builds the 1-bit copy of an FP8 instance once, or marks the instance as not {0, 1}.
// Synchronises the stream (once per instance, when the batch plan is built).
hipError_t ensure_tiled_bits(Instance &I, hipStream_t st) {
    if (I.jbits != 0) return hipSuccess;
    if (I.jt != JT_FP8 || !I.Js) {
        I.jbits = -1;
        return hipSuccess;
    }
    const int ntile = (I.N + 15) / 16, nrounds = I.Np / 128;
    const int64_t n = (int64_t)ntile * nrounds * 64;
    int32_t *dbad = nullptr;
    hipError_t e = dev_malloc((void **)&dbad, sizeof(int32_t));
    if (e == hipSuccess) e = dev_malloc(&I.Jbits, n * 4);
    if (e == hipSuccess) e = hipMemsetAsync(dbad, 0, sizeof(int32_t), st);
    if (e == hipSuccess) {
        k_tile_bits<<<(unsigned)((n + 255) / 256), 256, 0, st>>>((const uint8_t *)I.Js, I.Np, ntile,
                                                               nrounds, (uint32_t *)I.Jbits, dbad);
        e = hipGetLastError();
    }
    int32_t bad = 1;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, dbad, sizeof bad, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (dbad) (void)hipFree(dbad);
    if (e != hipSuccess || bad) {
        if (I.Jbits) (void)hipFree(I.Jbits);
        I.Jbits = nullptr;
    }
    if (e != hipSuccess) return e;
    I.jbits = bad ? -1 : 1;
    return hipSuccess;
}

hipError_t launch_md_steps_batch(hqa_md *md, int64_t q0, int64_t q1, bool graph) {
    if (!md->batch) {
        BatchPlan *bp = nullptr;
        hipError_t e = build_plan(md, bp);
        if (e != hipSuccess) return e;
        md->batch = bp;
    }
    BatchPlan *bp = (BatchPlan *)md->batch;
    int cur = -1;
    for (auto &I : md->inst)
        if (I.layout == HQA_DENSE) { cur = I.cur; break; }
    if (cur < 0) return hipSuccess;
    if (graph && q1 > q0) {
        hipGraphExec_t exec = nullptr;
        hipError_t e = batch_graph(md, bp, q0, q1, cur, &exec);
        if (e != hipSuccess) return e;
        e = hipGraphLaunch(exec, md->stream);
        if (e != hipSuccess) return e;
    } else {
        enqueue_steps(md, bp, q0, q1, cur, md->stream);
    }
    if ((q1 - q0) & 1) cur ^= 1;
    for (auto &I : md->inst)
        if (I.layout == HQA_DENSE) I.cur = cur;
    return hipGetLastError();
}

}  // namespace hqa
