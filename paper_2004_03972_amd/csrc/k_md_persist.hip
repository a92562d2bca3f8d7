// k_md_persist.hip -- all MD steps of a dense instance in one persistent launch.
//
// Replicas are independent, so the work splits into clusters: cluster c owns the
// 16 replicas [16c, 16c+16) and G workgroups; workgroup g owns the rows
// [g NB, g NB + NB), NB = 64 * TRW (TRW row tiles of 16 per wavefront).  For the
// whole run a workgroup keeps
//   - its J row block in LDS (stored type; rows padded by 16 bytes against bank
//     conflicts), or reads it from L2 when the block does not fit,
//   - the binary32 flux, momentum and window sum of its rows x 16 replicas in
//     registers (four consecutive rows of one replica per lane: the MFMA
//     accumulator layout).
// Step q needs the fluxes phi^(q) of all N spins of the cluster's replicas, which
// the other workgroups of the cluster produce.  They travel through an exchange
// buffer of tagged entries, each flux stored together with a step tag.  At the
// start of a step the workgroup reads the cluster's whole flux block, all loads
// in flight together; a thread that finds an entry whose tag is not yet the
// step's reads its part again, and the values are staged in LDS, from which every
// wavefront reads its MFMA operands.  Each entry validates itself, so no flag,
// fence, grid barrier or L2 write-back is needed.  Two exchange buffers (by step
// parity) cannot be overwritten early: a producer writes step q+2 into the buffer
// of step q only after it has gathered step q+1, which every consumer produced
// after finishing its gather of step q.  Tags run 1..65535 within a launch and the
// buffers are cleared before it, so stale entries never match.
//
// The members of a cluster share one XCD (workgroup b runs on XCD b mod 8), and
// the L2 of an XCD is the coherence point of its CUs.  So a flux only has to
// reach that L2: producers write it with ordinary stores (the vector L1 writes
// through, and the line stays in the L2 without a write-back to memory), and
// consumers read it with agent-scope loads, which miss in the L1 and are served
// by the L2.  Agent-scope stores would also write every entry through to memory,
// which the exchange does not need.  Each workgroup checks at start that it runs
// on the XCD its cluster assumes and otherwise aborts the launch (ERR_PLACEMENT);
// an agent-scope acquire at start drops any copy of the cleared buffer that the
// L2 may hold from an earlier launch.
//
// The binary32 update applies the same operation sequence as the per-step
// kernel, so both paths give identical states.  Every wait is bounded: past the
// bound a workgroup raises an abort flag that all other waiters observe, and
// the whole grid leaves the kernel.
//
// For BF16 / FP8 storage with Np <= 2048 a second kernel (k_persist_rj) keeps each
// wavefront's 16 rows of J in registers instead of LDS, so that the staged flux
// block is the only LDS operand of a step.
#include <type_traits>

#include "hqa_internal.h"
#include "md_epilogue.h"

namespace hqa {

typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2_t;

// Buffers of one instance; a register-J launch may serve several instances of one
// size (cluster c belongs to instance c / C1).
#define PERSIST_MAXK 8
struct PersistInst {
    const void *J;
    const float *h, *phi_in;
    float *phi_out;
    bf16 *xb_out;
    float *p, *S;
    uint64_t *xch;
};

struct PersistArgs {
    int N, Np, R, ld, M, G, C;
    int K, C1;               // instances in the launch, clusters per instance (C = K C1)
    PersistInst ins[PERSIST_MAXK];
    int64_t T, q0, q1;
    int W;
    float rg;
    const void *J;
    const float *h;
    const float *a32, *b32;
    const float *phi_in;     // phi^(q0), binary32 state layout
    float *phi_out;          // receives phi^(q1)
    bf16 *xb_out;            // BF16 operand copy of phi^(q1) (per-step kernels read it)
    float *p, *S;
    uint64_t *xch;           // [2][Rp][Np] tagged entries: u32 (bf16|tag<<16) or u64 (f32|tag<<32)
    int64_t xch_half;        // entries per parity buffer
    int32_t *abort_flag;
    int32_t *err;
    int jstride;             // LDS row stride of the J block (bytes)
    int jbytes;              // LDS bytes of the J block (0 when J is read from L2)
    int pstride;             // LDS row stride of the staged flux block (bytes)
    int64_t spin_limit;
};

__device__ __forceinline__ bf16x8 cvt_fp8x8(uint2 raw) {
    bf16x2_t a = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.x, 1.0f, false);
    bf16x2_t b = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.x, 1.0f, true);
    bf16x2_t c = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.y, 1.0f, false);
    bf16x2_t d = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.y, 1.0f, true);
    bf16x8 o;
    o[0] = a[0]; o[1] = a[1]; o[2] = b[0]; o[3] = b[1];
    o[4] = c[0]; o[5] = c[1]; o[6] = d[0]; o[7] = d[1];
    return o;
}

typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// An ordinary 64-bit store (single-copy atomic): it reaches the XCD's L2.  The
// compiler barrier keeps it ahead of the waits that follow.
__device__ __forceinline__ void st_l2(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Four BF16 entries (flux | tag << 16, one 32-bit word each) in one 16-byte store.
__device__ __forceinline__ void st4_l2(uint32_t *p, u32x4 v) {
    *(u32x4 *)p = v;
}
// 16 bytes of a raw buffer at byte offset off, loaded at agent scope (sc1: misses
// in the L1, served by the L2); offsets past the buffer's size read zeros.
__device__ __forceinline__ u32x4 ld16_agent(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 16);
}

// Aborts the launch unless the workgroup runs on XCD `xcd`; then drops stale L2
// copies of the exchange buffer.  Returns false when the workgroup must leave.
__device__ __forceinline__ bool check_placement(int32_t *abort_flag, int32_t *err, int xcd) {
    uint32_t xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
    if ((int)(xcc & 0xfu) != xcd) {   // uniform over the workgroup
        if (threadIdx.x == 0) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicOr(err, ERR_PLACEMENT);
        }
        return false;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// Polls a wait may make before it gives up: 2^22 (seconds of waiting), or
// HQA_SPIN_LIMIT=k (k >= 0) read at each launch, for tests of the abort path.
static int64_t spin_limit() {
    const char *v = getenv("HQA_SPIN_LIMIT");
    if (v && *v) {
        char *end = nullptr;
        const long long k = strtoll(v, &end, 10);
        if (end && *end == 0 && k >= 0) return (int64_t)k;
    }
    return (int64_t)1 << 22;
}

struct Waiter {
    int64_t spins;
    bool dead;
};

__device__ __forceinline__ bool keep_waiting(const PersistArgs &a, Waiter &wt) {
    if (++wt.spins > a.spin_limit) {
        __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicOr(a.err, ERR_BARRIER);
        wt.dead = true;
        return false;
    }
    if ((wt.spins & 63) == 0 &&
        __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        wt.dead = true;
        return false;
    }
    __builtin_amdgcn_s_sleep(1);
    return true;
}

// Gather the cluster's flux block of one step into LDS.  The
// block is [ld / 4 units of four rows][16 replicas][4 entries]: unit idx holds
// rows 4 (idx >> 4) .. +3 of replica idx & 15.
//  - FP32: 64-bit entries, four 64-bit atomic loads per unit, one 16-byte LDS
//    store; batches of 256 units (4 ld is a multiple of 512, so every batch is
//    whole and its guard uniform).
//  - BF16: 32-bit entries, one 16-byte load per unit.  A thread takes two units
//    of one replica with adjacent row groups, idx and idx + 16, and stores their
//    eight bf16 values to LDS with one 16-byte store (the row stride of the staged
//    block is 4 dwords modulo 64 banks, so a quarter-wavefront's stores cover the
//    banks once); batches of 512 units.  NBC > 0: the batch count ld / 128 known at
//    compile time (no guards; at most 16).
// A thread that gives up waiting sets *dead; the caller synchronises and leaves.
template <int JT, int NBC = 0>
__device__ __forceinline__ void gather(const PersistArgs &a, int par, int r0, uint32_t tag,
                                       uint8_t *phis, Waiter &wt) {
    const int tid = threadIdx.x;
    const int rr = tid & 15;                          // replica of this thread's units
    if constexpr (JT == JT_F32) {
        constexpr int GB = 8;                         // units per thread in flight
        const int nb = 4 * a.ld / 256;
        const uint64_t *src = a.xch + par * a.xch_half + (int64_t)r0 * a.ld;
        const uint64_t tg = (uint64_t)tag << 32;
        for (int b0 = 0; b0 < nb; b0 += GB) {
            uint64_t v[GB][4];
            while (true) {
                uint64_t bad = 0;
#pragma unroll
                for (int m = 0; m < GB; m++) {
                    const uint64_t *u = src + ((b0 + m) * 256 + tid) * 4;
                    if (b0 + m < nb) {
#pragma unroll
                        for (int e = 0; e < 4; e++) v[m][e] = ld_relaxed(u + e);
                    }
                }
#pragma unroll
                for (int m = 0; m < GB; m++) {
                    if (b0 + m < nb) {
#pragma unroll
                        for (int e = 0; e < 4; e++) bad |= v[m][e] ^ tg;
                    }
                }
                if ((bad >> 32) == 0 || !keep_waiting(a, wt)) break;
            }
#pragma unroll
            for (int m = 0; m < GB; m++) {
                const int kk = (((b0 + m) * 256 + tid) >> 4) * 4;
                if (b0 + m < nb)
                    *(uint4 *)(phis + (size_t)rr * a.pstride + kk * 4) =
                        make_uint4((uint32_t)v[m][0], (uint32_t)v[m][1], (uint32_t)v[m][2], (uint32_t)v[m][3]);
            }
        }
    } else {
        constexpr int GB = NBC > 0 ? NBC : 8;         // unit pairs per thread in flight
        const int nb = NBC > 0 ? NBC : a.ld / 128;
        const uint32_t *src = (const uint32_t *)a.xch + par * a.xch_half + (int64_t)r0 * a.ld;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void *)src, (short)0, 64 * a.ld, 0x00020000);
        const uint32_t tg = tag << 16;
        const int u0 = (tid >> 4) * 32 + rr;          // first unit of the pair in a batch
        for (int b0 = 0; b0 < nb; b0 += GB) {
            u32x4 v[GB][2];
            while (true) {
                uint32_t bad = 0;
#pragma unroll
                for (int m = 0; m < GB; m++)
                    if (b0 + m < nb) {
                        v[m][0] = ld16_agent(rs, ((b0 + m) * 512 + u0) * 16);
                        v[m][1] = ld16_agent(rs, ((b0 + m) * 512 + u0 + 16) * 16);
                    }
#pragma unroll
                for (int m = 0; m < GB; m++)
                    if (b0 + m < nb)
#pragma unroll
                        for (int h = 0; h < 2; h++)
                            bad |= (v[m][h][0] ^ tg) | (v[m][h][1] ^ tg) | (v[m][h][2] ^ tg) |
                                   (v[m][h][3] ^ tg);
                if ((bad >> 16) == 0 || !keep_waiting(a, wt)) break;
                asm volatile("" ::: "memory");   // the re-loads must read memory again
            }
#pragma unroll
            for (int m = 0; m < GB; m++) {
                if (b0 + m < nb) {
                    const int ku = (b0 + m) * 32 + (tid >> 4) * 2;   // row group of the pair
                    uint4 o;
                    o.x = __builtin_amdgcn_perm(v[m][0][1], v[m][0][0], 0x05040100u);
                    o.y = __builtin_amdgcn_perm(v[m][0][3], v[m][0][2], 0x05040100u);
                    o.z = __builtin_amdgcn_perm(v[m][1][1], v[m][1][0], 0x05040100u);
                    o.w = __builtin_amdgcn_perm(v[m][1][3], v[m][1][2], 0x05040100u);
                    *(uint4 *)(phis + (size_t)rr * a.pstride + ku * 8) = o;
                }
            }
        }
    }
}

__device__ __forceinline__ uint64_t bf16_word(float x, uint32_t tag) {
    bf16 b = (bf16)x;
    return (uint64_t)(__builtin_bit_cast(uint16_t, b)) | ((uint64_t)tag << 16);
}

// Publish four consecutive rows of one replica for step tag `tag`.
template <int JT>
__device__ __forceinline__ void publish(const PersistArgs &a, int par, int col, int ib,
                                        const float *xn, uint32_t tag) {
    if constexpr (JT == JT_F32) {
        uint64_t *dst = a.xch + par * a.xch_half + (int64_t)(col & ~15) * a.ld +
                        ((ib >> 2) * 16 + (col & 15)) * 4;
#pragma unroll
        for (int v = 0; v < 4; v++)
            st_l2(dst + v, (uint64_t)__float_as_uint(xn[v]) | ((uint64_t)tag << 32));
    } else {
        // [ld / 4][16][4] block of the cluster of replica col (see gather): a
        // wavefront's 16 replicas x 16 rows are one contiguous kilobyte
        uint32_t *dst = (uint32_t *)a.xch + par * a.xch_half + (int64_t)(col & ~15) * a.ld +
                        ((ib >> 2) * 16 + (col & 15)) * 4;
        st4_l2(dst, (u32x4){(uint32_t)bf16_word(xn[0], tag), (uint32_t)bf16_word(xn[1], tag),
                            (uint32_t)bf16_word(xn[2], tag), (uint32_t)bf16_word(xn[3], tag)});
    }
    asm volatile("" ::: "memory");   // issued before the next gather's waits
}

template <int JT, int TRW, bool JLDS>
__global__ __launch_bounds__(256) void k_persist(PersistArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    // block -> (xcd, slot) -> (cluster, rank): cluster members share an XCD
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int cl_in_xcd = slot / a.G, g = slot % a.G;
    const int c = cl_in_xcd * 8 + xcd;
    if (c >= a.C) return;
    if (!check_placement(a.abort_flag, a.err, xcd)) return;
    __shared__ int s_dead;   // a thread gave up waiting
    if (threadIdx.x == 0) s_dead = 0;
    __syncthreads();
    const int NB = 64 * TRW;
    const int row0 = g * NB;
    if (row0 >= a.Np) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = 16 * c;
    const int esz = JT == JT_F32 ? 4 : JT == JT_BF16 ? 2 : 1;
    uint8_t *phis = lds + a.jbytes;   // staged flux block [16][pstride]

    if constexpr (JLDS) {
        const int rows = min(NB, a.Np - row0);
        const int per_row = a.Np * esz / 16;
        for (int t = threadIdx.x; t < rows * per_row; t += 256) {
            int rr = t / per_row, cc = t % per_row;
            const uint4 *src = (const uint4 *)((const uint8_t *)a.J +
                                               ((int64_t)(row0 + rr) * a.Np) * esz) + cc;
            *(uint4 *)(lds + (size_t)rr * a.jstride + cc * 16) = *src;
        }
    }

    const int col = r0 + (lane & 15);
    const int kg = lane >> 4;
    const bool rvalid = col < a.R;
    float xs[TRW][4], ps[TRW][4], ss[TRW][4], hs[TRW][4];
    bool tile_ok[TRW];
#pragma unroll
    for (int t = 0; t < TRW; t++) {
        tile_ok[t] = row0 + 16 * (w * TRW + t) < a.Np;
        const int ib = row0 + 16 * (w * TRW + t) + 4 * kg;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int i = ib + v;
            const bool ok = rvalid && i < a.N;
            const int64_t k = (int64_t)col * a.ld + i;
            xs[t][v] = ok ? a.phi_in[k] : 0.f;
            ps[t][v] = ok ? a.p[k] : 0.f;
            ss[t][v] = ok ? a.S[k] : 0.f;
            hs[t][v] = (i < a.N) ? a.h[i] : 0.f;
        }
        if (tile_ok[t]) publish<JT>(a, 0, col, ib, xs[t], 1u);
    }
    Waiter wt{0, false};
    bool bad = false;
    const int nsteps = (int)(a.q1 - a.q0);
    // schedule values are loaded one step ahead, so their latency is never waited for
    CoefRaw cfn = load_coef(a.a32, a.b32, a.q0);
    for (int s = 0; s < nsteps; s++) {
        const int64_t q = a.q0 + s;
        const int par = s & 1;
        const StepCoef cf = make_coef(cfn, q, a.rg, a.M);
        if (s + 1 < nsteps) cfn = load_coef(a.a32, a.b32, q + 1);
        gather<JT>(a, par, r0, (uint32_t)(s % 65535) + 1u, phis, wt);
        if (wt.dead) s_dead = 1;
        __syncthreads();
        if (s_dead) return;   // aborted: the workgroup leaves
        // field in the four chains of combine4 (chunk c -> chain c mod 4)
        f32x4 acc[TRW][4];
#pragma unroll
        for (int t = 0; t < TRW; t++)
#pragma unroll
            for (int j = 0; j < 4; j++) acc[t][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
        const uint8_t *Xb = phis + (size_t)(lane & 15) * a.pstride;
        // Np is a multiple of 128: whole groups of four chunks, the next group's
        // operands are loaded while the current group's MFMAs run.
        if constexpr (JT == JT_F32) {
            const int ngroups = a.Np / 64;
            float4 A[TRW][4], B[4], An[TRW][4], Bn[4];
            auto load = [&](int gi, float4 (&Ag)[TRW][4], float4 (&Bg)[4]) {
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int kk = gi * 64 + 16 * j + 4 * kg;
                    Bg[j] = *(const float4 *)(Xb + kk * 4);
#pragma unroll
                    for (int t = 0; t < TRW; t++) {
                        const int rr = 16 * (w * TRW + t) + (lane & 15);
                        if (!tile_ok[t]) { Ag[t][j] = make_float4(0.f, 0.f, 0.f, 0.f); continue; }
                        if constexpr (JLDS) Ag[t][j] = *(const float4 *)(lds + (size_t)rr * a.jstride + kk * 4);
                        else Ag[t][j] = *(const float4 *)((const float *)a.J + (int64_t)(row0 + rr) * a.Np + kk);
                    }
                }
            };
            load(0, A, B);
            for (int gi = 0; gi < ngroups; gi++) {
                if (gi + 1 < ngroups) load(gi + 1, An, Bn);
#pragma unroll
                for (int j = 0; j < 4; j++)
#pragma unroll
                    for (int t = 0; t < TRW; t++) {
                        acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[t][j].x, B[j].x, acc[t][j], 0, 0, 0);
                        acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[t][j].y, B[j].y, acc[t][j], 0, 0, 0);
                        acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[t][j].z, B[j].z, acc[t][j], 0, 0, 0);
                        acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[t][j].w, B[j].w, acc[t][j], 0, 0, 0);
                    }
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    B[j] = Bn[j];
#pragma unroll
                    for (int t = 0; t < TRW; t++) A[t][j] = An[t][j];
                }
            }
        } else {
            typedef typename std::conditional<JT == JT_BF16, bf16x8, uint2>::type AT;
            const int ngroups = a.Np / 128;
            AT A[TRW][4], An[TRW][4];
            bf16x8 B[4], Bn[4];
            auto load = [&](int gi, AT (&Ag)[TRW][4], bf16x8 (&Bg)[4]) {
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int kk = gi * 128 + 32 * j + 8 * kg;
                    Bg[j] = *(const bf16x8 *)(Xb + kk * 2);
#pragma unroll
                    for (int t = 0; t < TRW; t++) {
                        const int rr = 16 * (w * TRW + t) + (lane & 15);
                        if (!tile_ok[t]) { Ag[t][j] = AT{}; continue; }
                        if constexpr (JT == JT_BF16) {
                            if constexpr (JLDS) Ag[t][j] = *(const bf16x8 *)(lds + (size_t)rr * a.jstride + kk * 2);
                            else Ag[t][j] = *(const bf16x8 *)((const bf16 *)a.J + (int64_t)(row0 + rr) * a.Np + kk);
                        } else {
                            if constexpr (JLDS) Ag[t][j] = *(const uint2 *)(lds + (size_t)rr * a.jstride + kk);
                            else Ag[t][j] = *(const uint2 *)((const uint8_t *)a.J + (int64_t)(row0 + rr) * a.Np + kk);
                        }
                    }
                }
            };
            load(0, A, B);
            for (int gi = 0; gi < ngroups; gi++) {
                if (gi + 1 < ngroups) load(gi + 1, An, Bn);
#pragma unroll
                for (int j = 0; j < 4; j++)
#pragma unroll
                    for (int t = 0; t < TRW; t++) {
                        bf16x8 av;
                        if constexpr (JT == JT_BF16) av = A[t][j];
                        else av = cvt_fp8x8(A[t][j]);
                        acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, B[j], acc[t][j], 0, 0, 0);
                    }
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    B[j] = Bn[j];
#pragma unroll
                    for (int t = 0; t < TRW; t++) A[t][j] = An[t][j];
                }
            }
        }
        const bool win = q + 1 >= a.T - a.W + 1;
        const uint32_t ntag = (uint32_t)((s + 1) % 65535) + 1u;
#pragma unroll
        for (int t = 0; t < TRW; t++) {
            if (!tile_ok[t]) continue;
            const int ib = row0 + 16 * (w * TRW + t) + 4 * kg;
            const f32x4 u = combine4(acc[t]);
            float xn[4];
#pragma unroll
            for (int v = 0; v < 4; v++) {
                if (rvalid && ib + v < a.N) {
                    leapfrog(cf, xs[t][v], u[v], hs[t][v], ps[t][v], xn[v]);
                    bad |= !isfinite(xn[v]) || !isfinite(ps[t][v]);
                    if (win) ss[t][v] = ss[t][v] + xn[v];
                } else {
                    xn[v] = 0.f;
                }
                xs[t][v] = xn[v];
            }
            if (s + 1 < nsteps) publish<JT>(a, par ^ 1, col, ib, xn, ntag);
        }
        __syncthreads();   // the staged block is rewritten by the next gather
    }
#pragma unroll
    for (int t = 0; t < TRW; t++) {
        if (!tile_ok[t] || !rvalid) continue;
        const int ib = row0 + 16 * (w * TRW + t) + 4 * kg;
        const int64_t base = (int64_t)col * a.ld + ib;
        *(float4 *)(a.phi_out + base) = make_float4(xs[t][0], xs[t][1], xs[t][2], xs[t][3]);
        *(float4 *)(a.p + base) = make_float4(ps[t][0], ps[t][1], ps[t][2], ps[t][3]);
        *(float4 *)(a.S + base) = make_float4(ss[t][0], ss[t][1], ss[t][2], ss[t][3]);
        if (a.xb_out) {
            typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
            bf16x4 b = {(bf16)xs[t][0], (bf16)xs[t][1], (bf16)xs[t][2], (bf16)xs[t][3]};
            *(bf16x4 *)(a.xb_out + base) = b;
        }
    }
    if (bad) atomicOr(a.err, ERR_NONFINITE);
}

// Register-resident J (BF16 / FP8 storage, Np <= 2048): workgroups of 64 rows (four
// row tiles of 16); the cluster has Np / 64 members.  Wavefront w computes
// accumulation chain w -- chunks 4 gi + w (gi < NG = Np / 128) of all four row tiles --
// and holds those J fragments in registers for the whole run.  It reads its MFMA B
// fragments (16 replicas x 32 columns per chunk, two exchange units per lane) straight
// from the cluster's exchange block, so nothing is staged and a wavefront starts its
// MFMAs as soon as its own chunks have arrived.  The four chains of a tile meet in LDS
// (double-buffered by step parity, so one workgroup barrier per step suffices: a
// wavefront rewrites a parity's partials only after the next step's barrier, which
// every wavefront passes after reading them), and wavefront w combines tile w as
// (a0 + a1) + (a2 + a3), updates it and publishes it.  The MFMAs, their operands and
// their order per chain are those of every other dense kernel, so the trajectories
// are identical.  Past NG = 8 the fragments no longer fit the 256 architectural
// registers and the compiler keeps part of them in the accumulation registers.
// The launch arguments with instance k's buffers in place of instance 0's (k is
// wavefront-uniform; the selection runs over compile-time indices, so the argument
// block is never indexed at run time).
__device__ __forceinline__ PersistArgs for_instance(const PersistArgs &a0, int k) {
    PersistArgs a = a0;
#pragma unroll
    for (int kk = 1; kk < PERSIST_MAXK; kk++) {
        if (kk == k) {
            const PersistInst &q = a0.ins[kk];
            a.J = q.J; a.h = q.h; a.phi_in = q.phi_in; a.phi_out = q.phi_out;
            a.xb_out = q.xb_out; a.p = q.p; a.S = q.S; a.xch = q.xch;
        }
    }
    return a;
}

template <int JT, int NG, int MP>
__global__ __launch_bounds__(256) void k_persist_rj(PersistArgs a0) {
    __shared__ f32x4 part[2][4][4][64];   // [step parity][chain][row tile][lane]
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int cl_in_xcd = slot / a0.G, g = slot % a0.G;
    const int cg = cl_in_xcd * 8 + xcd;   // cluster of the launch
    if (cg >= a0.C) return;
    const int k = cg / a0.C1, c = cg - k * a0.C1;   // instance, cluster within it
    const PersistArgs a = for_instance(a0, k);
    if (!check_placement(a.abort_flag, a.err, xcd)) return;
    __shared__ int s_dead[2];   // a thread gave up waiting (by step parity, like the partials)
    if (threadIdx.x < 2) s_dead[threadIdx.x] = 0;
    __syncthreads();
    const int row0 = g * 64;          // G = Np / 64: every member's rows lie below Np
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = 16 * c;
    const int kg = lane >> 4;

    typedef typename std::conditional<JT == JT_BF16, bf16x8, uint2>::type AT;
    constexpr int esz = JT == JT_BF16 ? 2 : 1;
    AT A[NG][4];                      // [gi][row tile]: chunk 4 gi + w
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const uint8_t *Jr = (const uint8_t *)a.J + (int64_t)(row0 + 16 * t + (lane & 15)) * a.Np * esz;
#pragma unroll
        for (int gi = 0; gi < NG; gi++)
            A[gi][t] = *(const AT *)(Jr + (32 * (4 * gi + w) + 8 * kg) * esz);
    }

    // the update and publication of row tile w
    const int col = r0 + (lane & 15);
    const bool rvalid = col < a.R;
    const int ib = row0 + 16 * w + 4 * kg;
    float xs[4], ps[4], ss[4], hs[4];
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int i = ib + v;
        const bool ok = rvalid && i < a.N;
        const int64_t k = (int64_t)col * a.ld + i;
        xs[v] = ok ? a.phi_in[k] : 0.f;
        ps[v] = ok ? a.p[k] : 0.f;
        ss[v] = ok ? a.S[k] : 0.f;
        hs[v] = (i < a.N) ? a.h[i] : 0.f;
    }
    publish<JT>(a, 0, col, ib, xs, 1u);

    // exchange units of this lane's B fragments: the block is [ld / 4][16][4] entries,
    // chunk 4 gi + w needs units (8 (4 gi + w) + 2 kg) * 16 + (lane & 15) and the next
    // row group (16 units on)
    __amdgpu_buffer_rsrc_t rs[2];
#pragma unroll
    for (int pr = 0; pr < 2; pr++)
        rs[pr] = __builtin_amdgcn_make_buffer_rsrc(
            (void *)((const uint32_t *)a.xch + pr * a.xch_half + (int64_t)r0 * a.ld), (short)0,
            64 * a.ld, 0x00020000);
    const int uoff = ((8 * w + 2 * kg) * 16 + (lane & 15)) * 16;   // bytes, chunk gi adds 32 * 16 * 16 gi

    Waiter wt{0, false};
    bool bad = false;
    const int nsteps = (int)(a.q1 - a.q0);
    // schedule values are loaded one step ahead, so their latency is never waited for
    CoefRaw cfn = load_coef(a.a32, a.b32, a.q0);
    for (int s = 0; s < nsteps; s++) {
        const int64_t q = a.q0 + s;
        const int par = s & 1;
        const StepCoef cf = make_coef(cfn, q, a.rg, a.M);
        if (s + 1 < nsteps) cfn = load_coef(a.a32, a.b32, q + 1);
        const uint32_t tg = ((uint32_t)(s % 65535) + 1u) << 16;
        // All of this lane's units are requested at once and chunk gi is fed to the
        // MFMAs as soon as its two units are in, while later chunks are still on their
        // way (straight-line code, so each chunk waits only for its own loads).  The
        // tags are folded into one word on the way; if any unit of the wavefront was
        // stale (its producer had not stored the step yet) the wavefront reads its units
        // again (all of them, or past eight chunk groups only the stale ones) and redoes
        // the chain from zero, so the order within the chain never changes.
        u32x4 bx[NG][2];
        f32x4 acc[4];
        auto load_units = [&]() {
#pragma unroll
            for (int gi = 0; gi < NG; gi++) {
                bx[gi][0] = ld16_agent(rs[par], uoff + gi * 8192);
                bx[gi][1] = ld16_agent(rs[par], uoff + gi * 8192 + 256);
            }
        };
        // a lane reads again only those of its units that are stale: for large blocks
        // this saves L2 traffic (at Np = 2048 each member reads 128 KB per step); for
        // small ones the per-unit branches cost more than reading everything again
        auto reload_stale = [&]() {
#pragma unroll
            for (int gi = 0; gi < NG; gi++) {
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const uint32_t x = (bx[gi][h][0] ^ tg) | (bx[gi][h][1] ^ tg) |
                                       (bx[gi][h][2] ^ tg) | (bx[gi][h][3] ^ tg);
                    if (x >> 16) bx[gi][h] = ld16_agent(rs[par], uoff + gi * 8192 + 256 * h);
                }
            }
        };
        auto chain = [&]() -> uint32_t {
            uint32_t stale = 0;
#pragma unroll
            for (int t = 0; t < 4; t++) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int gi = 0; gi < NG; gi++) {
#pragma unroll
                for (int h = 0; h < 2; h++)
                    stale |= (bx[gi][h][0] ^ tg) | (bx[gi][h][1] ^ tg) | (bx[gi][h][2] ^ tg) |
                             (bx[gi][h][3] ^ tg);
                typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t w4;
                const w4 o = {__builtin_amdgcn_perm(bx[gi][0][1], bx[gi][0][0], 0x05040100u),
                              __builtin_amdgcn_perm(bx[gi][0][3], bx[gi][0][2], 0x05040100u),
                              __builtin_amdgcn_perm(bx[gi][1][1], bx[gi][1][0], 0x05040100u),
                              __builtin_amdgcn_perm(bx[gi][1][3], bx[gi][1][2], 0x05040100u)};
                const bf16x8 bv = __builtin_bit_cast(bf16x8, o);
                // chain w of the four row tiles
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    bf16x8 av;
                    if constexpr (JT == JT_BF16) av = A[gi][t];
                    else av = cvt_fp8x8(A[gi][t]);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t], 0, 0, 0);
                }
            }
            return stale >> 16;
        };
        load_units();
        // the decision to read again is taken for the whole wavefront: an MFMA is a
        // wavefront-wide operation and must run with every lane active
        if (__any(chain() != 0)) {
            while (true) {
                if (__any(!keep_waiting(a, wt))) break;   // giving up: the launch aborts
                asm volatile("" ::: "memory");   // the re-loads must read memory again
                if constexpr (NG > 8) reload_stale();
                else load_units();
                if (!__any(chain() != 0)) break;
            }
        }
#pragma unroll
        for (int t = 0; t < 4; t++) part[par][w][t][lane] = acc[t];
        if (wt.dead) s_dead[par] = 1;
        __syncthreads();
        if (s_dead[par]) return;   // aborted: the workgroup leaves
        const f32x4 chains[4] = {part[par][0][w][lane], part[par][1][w][lane],
                                 part[par][2][w][lane], part[par][3][w][lane]};
        const bool win = q + 1 >= a.T - a.W + 1;
        const f32x4 u = combine4(chains);
        float xn[4];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            // padding rows and replicas hold zero state and a zero field; their update
            // is computed and discarded, so the lanes do not branch
            const bool ok = rvalid && ib + v < a.N;
            float pv = ps[v], x1;
            if constexpr (MP == 6) leapfrog_m<6>(cf, xs[v], u[v], hs[v], pv, x1);
            else leapfrog(cf, xs[v], u[v], hs[v], pv, x1);
            xn[v] = ok ? x1 : 0.f;
            ps[v] = ok ? pv : ps[v];
            bad |= !isfinite(xn[v]) || !isfinite(ps[v]);
            ss[v] = win && ok ? ss[v] + xn[v] : ss[v];
            xs[v] = xn[v];
        }
        if (s + 1 < nsteps) publish<JT>(a, par ^ 1, col, ib, xn, (uint32_t)((s + 1) % 65535) + 1u);
    }
    if (rvalid) {
        const int64_t base = (int64_t)col * a.ld + ib;
        *(float4 *)(a.phi_out + base) = make_float4(xs[0], xs[1], xs[2], xs[3]);
        *(float4 *)(a.p + base) = make_float4(ps[0], ps[1], ps[2], ps[3]);
        *(float4 *)(a.S + base) = make_float4(ss[0], ss[1], ss[2], ss[3]);
        if (a.xb_out) {
            typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
            bf16x4 b = {(bf16)xs[0], (bf16)xs[1], (bf16)xs[2], (bf16)xs[3]};
            *(bf16x4 *)(a.xb_out + base) = b;
        }
    }
    if (bad) atomicOr(a.err, ERR_NONFINITE);
}

// Plan of a persistent launch for one dense instance.
struct PersistPlan {
    int TRW, G, C, C1, grid, jlds, jstride, jbytes, pstride;
    int rj;          // J fragments in registers (k_persist_rj)
    size_t lds;
};

// K > 1: K instances of this size in one register-J launch (no other kernel takes
// several instances).
static bool plan_persist(const Instance &I, int R, JType jt, int max_wg, PersistPlan &p,
                         int K = 1) {
    const int esz = jt == JT_F32 ? 4 : jt == JT_BF16 ? 2 : 1;
    const int eb = jt == JT_F32 ? 4 : 2;               // staged flux element bytes
    const size_t lds_cap = 156 * 1024;
    p.C1 = (R + 15) / 16;
    p.C = K * p.C1;
    p.pstride = I.Np * eb + 16;
    const size_t stage = (size_t)16 * p.pstride;
    if (stage > lds_cap) return false;
    p.rj = 0;
    // first choice: J in registers (BF16 / FP8, at most sixteen 128-column groups)
    if (jt != JT_F32 && I.Np <= 2048) {
        const int G = I.Np / 64;
        const int need_xcd_slots = (p.C + 7) / 8;
        if (G <= 32 && need_xcd_slots <= 32 / G && 8 * need_xcd_slots * G <= max_wg) {
            p.rj = 1;
            p.TRW = 1;
            p.G = G;
            p.jlds = 0;
            p.jstride = 0;
            p.jbytes = 0;
            p.lds = 0;                                 // static LDS only (chain partials)
            p.grid = 8 * need_xcd_slots * G;
            return true;
        }
    }
    if (K > 1) return false;
    // then a J block resident in LDS, then two row tiles per wavefront
    for (int want_lds : {1, 0}) {
        for (int trw : {2, 1}) {
            int NB = 64 * trw;
            int G = (I.Np + NB - 1) / NB;
            if (G > 32) continue;                     // a cluster must fit one XCD (32 CUs)
            int per_xcd = 32 / G;                     // clusters per XCD
            int need_xcd_slots = (p.C + 7) / 8;
            if (need_xcd_slots > per_xcd) continue;
            size_t stride = (size_t)I.Np * esz + 16;
            size_t jb = (size_t)NB * stride;
            if (want_lds && jb + stage > lds_cap) continue;
            p.TRW = trw;
            p.G = G;
            p.jlds = want_lds;
            p.jstride = (int)stride;
            p.jbytes = want_lds ? (int)jb : 0;
            p.lds = (size_t)p.jbytes + stage;
            p.grid = 8 * need_xcd_slots * G;
            if (p.grid > max_wg) continue;
            return true;
        }
    }
    return false;
}

template <int JT, int TRW, bool JLDS>
static hipError_t launch_p(const PersistArgs &a, const PersistPlan &pl, hipStream_t st) {
    void *args[] = {(void *)&a};
    return hipLaunchCooperativeKernel((const void *)k_persist<JT, TRW, JLDS>, dim3(pl.grid),
                                      dim3(256), args, (unsigned)pl.lds, st);
}

// MP: the potential exponent when it is the paper's M = 6 (power unrolled), else 0.
template <int JT, int NG>
static hipError_t launch_rj(const PersistArgs &a, const PersistPlan &pl, hipStream_t st) {
    void *args[] = {(void *)&a};
    const void *k = a.M == 6 ? (const void *)k_persist_rj<JT, NG, 6> : (const void *)k_persist_rj<JT, NG, 0>;
    return hipLaunchCooperativeKernel(k, dim3(pl.grid), dim3(256), args, (unsigned)pl.lds, st);
}

template <int JT>
static hipError_t launch_rj_ng(const PersistArgs &a, const PersistPlan &pl, hipStream_t st) {
    switch (a.Np / 128) {
        case 1: return launch_rj<JT, 1>(a, pl, st);
        case 2: return launch_rj<JT, 2>(a, pl, st);
        case 3: return launch_rj<JT, 3>(a, pl, st);
        case 4: return launch_rj<JT, 4>(a, pl, st);
        case 5: return launch_rj<JT, 5>(a, pl, st);
        case 6: return launch_rj<JT, 6>(a, pl, st);
        case 7: return launch_rj<JT, 7>(a, pl, st);
        case 8: return launch_rj<JT, 8>(a, pl, st);
        case 9: return launch_rj<JT, 9>(a, pl, st);
        case 10: return launch_rj<JT, 10>(a, pl, st);
        case 11: return launch_rj<JT, 11>(a, pl, st);
        case 12: return launch_rj<JT, 12>(a, pl, st);
        case 13: return launch_rj<JT, 13>(a, pl, st);
        case 14: return launch_rj<JT, 14>(a, pl, st);
        case 15: return launch_rj<JT, 15>(a, pl, st);
        case 16: return launch_rj<JT, 16>(a, pl, st);
        default: return hipErrorNotSupported;
    }
}

template <int JT>
static hipError_t launch_jt(const PersistArgs &a, const PersistPlan &pl, hipStream_t st) {
    if constexpr (JT != JT_F32)
        if (pl.rj) return launch_rj_ng<JT>(a, pl, st);
    if (pl.TRW == 2) return pl.jlds ? launch_p<JT, 2, true>(a, pl, st) : launch_p<JT, 2, false>(a, pl, st);
    return pl.jlds ? launch_p<JT, 1, true>(a, pl, st) : launch_p<JT, 1, false>(a, pl, st);
}

// Returns hipErrorNotSupported when the instances have no persistent plan (the caller
// then runs one launch per step).  Several instances share a launch only when they
// have one size and one storage type and the register-J kernel fits them all.
hipError_t launch_md_persist_set(hqa_md *md, Instance *const *set, int K, int64_t q0,
                                 int64_t q1) {
    static int max_wg = -1;
    if (max_wg < 0) {
        int dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        max_wg = cus;   // one 256-thread workgroup per CU is always co-resident
    }
    if (K < 1 || K > PERSIST_MAXK) return hipErrorNotSupported;
    Instance &I0 = *set[0];
    for (int k = 1; k < K; k++)
        if (set[k]->Np != I0.Np || set[k]->N != I0.N || set[k]->jt != I0.jt ||
            set[k]->ld != I0.ld || set[k]->Rp != I0.Rp)
            return hipErrorNotSupported;
    PersistPlan pl;
    if (!plan_persist(I0, md->R, I0.jt, max_wg, pl, K)) return hipErrorNotSupported;
    const size_t esz = I0.jt == JT_F32 ? 8 : 4;
    const int64_t half = (int64_t)I0.Rp * I0.ld;
    const size_t bytes = 2 * (size_t)half * esz;
    for (int k = 0; k < K; k++) {
        Instance &I = *set[k];
        if (!I.xch || I.xch_bytes < bytes) {
            if (I.xch) (void)hipFree(I.xch);
            I.xch = nullptr;
            I.xch_bytes = 0;
            hipError_t e = dev_malloc(&I.xch, bytes);
            if (e != hipSuccess) return e;
            I.xch_bytes = bytes;
        }
    }
    if (!md->bar) {
        hipError_t e = dev_malloc((void **)&md->bar, sizeof(int32_t) * 64);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMemsetAsync(md->bar, 0, sizeof(int32_t) * 64, md->stream);
    for (int k = 0; k < K && e == hipSuccess; k++) e = hipMemsetAsync(set[k]->xch, 0, bytes, md->stream);
    if (e != hipSuccess) return e;
    PersistArgs a;
    a.N = I0.N; a.Np = I0.Np; a.R = md->R; a.ld = I0.ld; a.M = md->sch.M; a.G = pl.G; a.C = pl.C;
    a.K = K; a.C1 = pl.C1;
    a.T = md->sch.T; a.q0 = q0; a.q1 = q1; a.W = md->sch.W;
    a.rg = (float)md->sch.r_g;
    a.a32 = md->a32; a.b32 = md->b32;
    const int par = (int)((q1 - q0) & 1);
    for (int k = 0; k < PERSIST_MAXK; k++) {
        Instance &I = *set[k < K ? k : 0];
        PersistInst &q = a.ins[k];
        q.J = I.Js; q.h = I.h32;
        q.phi_in = I.phi32[I.cur];
        q.phi_out = I.phi32[I.cur ^ par];
        q.xb_out = I.phib[I.cur ^ par];
        q.p = I.p32; q.S = I.S32;
        q.xch = (uint64_t *)I.xch;
    }
    a.J = a.ins[0].J; a.h = a.ins[0].h; a.phi_in = a.ins[0].phi_in; a.phi_out = a.ins[0].phi_out;
    a.xb_out = a.ins[0].xb_out; a.p = a.ins[0].p; a.S = a.ins[0].S; a.xch = a.ins[0].xch;
    a.xch_half = half;
    a.abort_flag = md->bar + 63; a.err = md->err;
    a.jstride = pl.jstride;
    a.jbytes = pl.jbytes;
    a.pstride = pl.pstride;
    a.spin_limit = spin_limit();
    switch (I0.jt) {
        case JT_F32: e = launch_jt<JT_F32>(a, pl, md->stream); break;
        case JT_BF16: e = launch_jt<JT_BF16>(a, pl, md->stream); break;
        default: e = launch_jt<JT_FP8>(a, pl, md->stream); break;
    }
    if (e == hipSuccess)
        for (int k = 0; k < K; k++) set[k]->cur ^= par;
    return e;
}

hipError_t launch_md_persist(hqa_md *md, Instance &I, int64_t q0, int64_t q1) {
    Instance *one = &I;
    return launch_md_persist_set(md, &one, 1, q0, q1);
}

}  // namespace hqa
