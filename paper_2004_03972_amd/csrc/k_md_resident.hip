// k_md_resident.hip -- replica-resident dense anneal: the whole run of a group
// of 16 replicas in one workgroup, one launch for all steps.
//
// Replicas never interact (Results, "Molecular dynamics for flux variables":
// each initial momentum draw is an independent trajectory), so a workgroup that
// owns 16 replicas needs no communication with any other workgroup: its fluxes
// (binary32), momenta, the BF16 operand copy of the fluxes (double-buffered) and
// the field h stay in LDS from the first step to the last, and the only memory
// traffic per step is J, streamed from L2 (every workgroup reads the same J, so
// it is fetched from HBM once and then served by each XCD's L2).  With no
// kernel boundary and no grid-wide barrier between steps, the step costs the J
// stream and the MFMA work of one workgroup (measured per-CU L2 read rate about
// 135 GB/s, so about 5 us per step for N = 800 with FP8 J), instead of a launch.
//
// Arithmetic is that of the per-step kernel: chunk c of 32 columns feeds
// accumulation chain c mod 4 in ascending order, the field is (a0 + a1) + (a2 +
// a3), the same MFMA instruction sees the same operand fragments, and the
// leapfrog is the shared binary32 sequence, so the two give bit-identical
// trajectories.  (Chunks made only of padding columns are skipped here: adding
// a product of zeros to an accumulator that started at +0 leaves it unchanged.)
//
// Wavefront w owns row tiles [tb, te) (16 rows each), processed in groups of
// four; a round is four chunks (one per chain) of one group.  The J fragments of
// the next PF rounds are in flight in registers at all times, across group and
// step boundaries (J is constant, so the stream is periodic), and the only
// barrier is the one that separates consecutive steps.
#include <algorithm>
#include <type_traits>

#include "hqa_internal.h"
#include "md_epilogue.h"

namespace hqa {

typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2_r;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4_r;

struct ResArgs {
    int N, Np, R, M, ld;
    int nck, ntile, nrounds;   // chunks of 32 columns, tiles of 16 rows, rounds per group
    int ldb, ldf;              // LDS row strides (BF16 / binary32 elements)
    int jbytes;                // bytes of the stored J (Np * Np * element size)
    int64_t T, q0, q1;
    int W;
    float rg;
    const void *J;
    const float *h, *a32, *b32;
    const float *phi_in;
    const bf16 *xb_in;
    float *phi_out, *p, *S;
    bf16 *xb_out;
    int32_t *err;
};

__device__ __forceinline__ bf16x8 res_fp8x8(uint2 raw) {
    bf16x2_r a = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.x, 1.0f, false);
    bf16x2_r b = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.x, 1.0f, true);
    bf16x2_r c = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.y, 1.0f, false);
    bf16x2_r d = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.y, 1.0f, true);
    bf16x8 o;
    o[0] = a[0]; o[1] = a[1]; o[2] = b[0]; o[3] = b[1];
    o[4] = c[0]; o[5] = c[1]; o[6] = d[0]; o[7] = d[1];
    return o;
}

size_t resident_lds_bytes(int N) {
    const int nk = (N + 31) / 32 * 32;
    const size_t ldb = nk + 8, ldf = nk + 4;
    return 2 * 16 * ldb * 2 + 2 * 16 * ldf * 4 + ldf * 4;
}

// Schedule coefficients of step q through the scalar cache: q is uniform, and a
// scalar load keeps them out of the vector-memory counter that orders the J stream.
__device__ __forceinline__ StepCoef res_coef(const ResArgs &a, int64_t q) {
    typedef const __attribute__((address_space(4))) float cfloat;
    cfloat *al = (cfloat *)a.a32, *be = (cfloat *)a.b32;
    StepCoef c;
    c.al = al[2 * q];
    c.be = be[2 * q];
    c.ad = al[2 * q + 1];
    if (a.rg != 1.0f) c.ad = a.rg * c.ad;
    c.rg = a.rg;
    c.kick = q == 0 ? 0.5f : 1.0f;
    c.M = a.M;
    return c;
}

// WIN: every step of the launch adds phi' to the window sum (the host splits a run
// at the start of the averaging window, so the loop of the other launch carries no
// global-memory access besides the J stream).
template <int JT, int PF, bool WIN, int MP>
__global__ __launch_bounds__(256) void k_md_resident(ResArgs a) {
    typedef typename std::conditional<JT == JT_BF16, bf16x8, uint2>::type AT;
    constexpr int esz = JT == JT_BF16 ? 2 : 1;
    extern __shared__ __align__(16) unsigned char lds[];
    bf16 *xbl = (bf16 *)lds;                                    // [2][16][ldb]
    float *x32 = (float *)(lds + (size_t)2 * 16 * a.ldb * 2);   // [16][ldf]
    float *p32 = x32 + 16 * a.ldf;                              // [16][ldf]
    float *hl = p32 + 16 * a.ldf;                               // [ldf]

    // the wavefront index is made scalar so every tile / chunk guard is a uniform branch
    const int tid = threadIdx.x, lane = tid & 63, kg = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r0 = blockIdx.x * 16;
    const int nk = a.nck * 32;

    // ---- state in: rows r0 .. r0+15 of the replica-major arrays, columns < nk
    for (int e = tid; e < 16 * nk; e += 256) {
        const int rl = e / nk, k = e - rl * nk;
        const int64_t g = (int64_t)(r0 + rl) * a.ld + k;
        xbl[rl * a.ldb + k] = a.xb_in[g];
        xbl[(16 + rl) * a.ldb + k] = (bf16)0.0f;
        x32[rl * a.ldf + k] = a.phi_in[g];
        p32[rl * a.ldf + k] = a.p[g];
    }
    for (int k = tid; k < nk; k += 256) hl[k] = k < a.N ? a.h[k] : 0.0f;
    __syncthreads();

    // ---- this wavefront's row tiles and its periodic round sequence
    const int tb = w * a.ntile / 4, te = (w + 1) * a.ntile / 4;
    const int ngw = (te - tb + 3) / 4;
    const int64_t total = (a.q1 - a.q0) * (int64_t)ngw * a.nrounds;
    // J comes from its MFMA-tiled copy (see k_tile_j): the operand bytes of lane l
    // for the four chunks of round m of row tile t are contiguous, so one round of
    // one tile is 64 lanes x 32 B (FP8) or 64 B (BF16) of consecutive memory and
    // every 16-byte load fills whole cache lines.  Loads go through a bounds-checked
    // buffer resource: a slot outside the wavefront's tiles (or past the end of the
    // stream) gets an offset beyond the resource, which reads zero without touching
    // memory, so every round issues the same loads and the wait before each use
    // counts exactly the loads issued after it.
    const __amdgpu_buffer_rsrc_t jr =
        __builtin_amdgcn_make_buffer_rsrc((void *)a.J, (short)0, a.jbytes, 0x00020000);
    const int oob = a.jbytes;
    constexpr int lane_bytes = 4 * 8 * esz;   // four chunks of eight elements

    AT A[PF][4][4];
    int gl = 0, ml = 0;          // next round to load (group, round)
    int64_t issued = 0;
    auto load_round = [&](AT (&dst)[4][4]) {
#pragma unroll
        for (int tm = 0; tm < 4; tm++) {
            const int t = tb + 4 * gl + tm;
            const int off = (t < te && issued < total)
                                ? ((t * a.nrounds + ml) * 64 + lane) * lane_bytes
                                : oob;
            if constexpr (JT == JT_BF16) {
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    auto v = __builtin_amdgcn_raw_buffer_load_b128(jr, off + 16 * k, 0, 0);
                    dst[k][tm] = __builtin_bit_cast(bf16x8, v);
                }
            } else {
                auto lo = __builtin_amdgcn_raw_buffer_load_b128(jr, off, 0, 0);
                auto hi = __builtin_amdgcn_raw_buffer_load_b128(jr, off + 16, 0, 0);
                dst[0][tm] = make_uint2(lo[0], lo[1]);
                dst[1][tm] = make_uint2(lo[2], lo[3]);
                dst[2][tm] = make_uint2(hi[0], hi[1]);
                dst[3][tm] = make_uint2(hi[2], hi[3]);
            }
        }
        if (++ml == a.nrounds) {
            ml = 0;
            if (++gl == ngw) gl = 0;
        }
        issued++;
    };
#pragma unroll
    for (int j = 0; j < PF; j++) load_round(A[j]);

    int gc = 0, mc = 0, cur = 0;
    int64_t q = a.q0;
    StepCoef cf = res_coef(a, q);
    bool bad = false;
    f32x4 acc[4][4];
#pragma unroll
    for (int tm = 0; tm < 4; tm++)
#pragma unroll
        for (int k = 0; k < 4; k++) acc[tm][k] = (f32x4){0.f, 0.f, 0.f, 0.f};
    // one round: four chunks of the current group, the refill of its register slot,
    // and at the end of a group its epilogue (and at the end of a step the barrier)
    auto round = [&](AT (&Aj)[4][4]) {
        // Every MFMA of the round is issued: a slot outside this wavefront's tiles
        // holds zeros (out-of-range load), a chunk past the last one holds the zero
        // padding of J, and its B fragment is read from a valid chunk, so the
        // products are exact zeros and leave the accumulator (which starts at +0
        // and so is never -0) bit-unchanged.  No branch separates the MFMAs, which
        // keeps the accumulators in place across the round.
        const bf16 *xin = xbl + cur * 16 * a.ldb + (lane & 15) * a.ldb + 8 * kg;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int c = min(4 * mc + k, a.nck - 1);
            const bf16x8 B = *(const bf16x8 *)(xin + 32 * c);
#pragma unroll
            for (int tm = 0; tm < 4; tm++) {
                bf16x8 av;
                if constexpr (JT == JT_BF16) av = Aj[k][tm];
                else av = res_fp8x8(Aj[k][tm]);
                acc[tm][k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, B, acc[tm][k], 0, 0, 0);
            }
        }
        load_round(Aj);   // past the end of the stream it reads zeros
        if (mc == a.nrounds - 1) {
            // epilogue of the group: leapfrog of its rows for this wavefront's lanes
            const int rl = lane & 15;
#pragma unroll
            for (int tm = 0; tm < 4; tm++) {
                const int t = tb + 4 * gc + tm;
                if (t >= te || r0 + rl >= a.R) continue;
                const f32x4 parts[4] = {acc[tm][0], acc[tm][1], acc[tm][2], acc[tm][3]};
                const f32x4 u = combine4(parts);
                const int ib = 16 * t + 4 * kg;
                float4 x = *(const float4 *)(x32 + rl * a.ldf + ib);
                float4 pp = *(const float4 *)(p32 + rl * a.ldf + ib);
                float xs[4] = {x.x, x.y, x.z, x.w}, ps[4] = {pp.x, pp.y, pp.z, pp.w}, xn[4];
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    if (ib + v < a.N) {
                        if constexpr (MP == 6) leapfrog_m<6>(cf, xs[v], u[v], hl[ib + v], ps[v], xn[v]);
                        else leapfrog(cf, xs[v], u[v], hl[ib + v], ps[v], xn[v]);
                        bad |= !isfinite(xn[v]) || !isfinite(ps[v]);
                    } else {
                        xn[v] = 0.0f;
                        ps[v] = 0.0f;
                    }
                }
                *(float4 *)(x32 + rl * a.ldf + ib) = make_float4(xn[0], xn[1], xn[2], xn[3]);
                *(float4 *)(p32 + rl * a.ldf + ib) = make_float4(ps[0], ps[1], ps[2], ps[3]);
                bf16x4_r b = {(bf16)xn[0], (bf16)xn[1], (bf16)xn[2], (bf16)xn[3]};
                *(bf16x4_r *)(xbl + (cur ^ 1) * 16 * a.ldb + rl * a.ldb + ib) = b;
                if constexpr (WIN) {   // every step of this launch is inside the window
                    float4 *sp = (float4 *)(a.S + (int64_t)(r0 + rl) * a.ld + ib);
                    float4 s = *sp;
                    s.x = s.x + xn[0]; s.y = s.y + xn[1]; s.z = s.z + xn[2]; s.w = s.w + xn[3];
                    *sp = s;
                }
            }
#pragma unroll
            for (int tm = 0; tm < 4; tm++)
#pragma unroll
                for (int k = 0; k < 4; k++) acc[tm][k] = (f32x4){0.f, 0.f, 0.f, 0.f};
        }
        if (++mc == a.nrounds) {
            mc = 0;
            if (++gc == ngw) {
                // end of this wavefront's step: every wavefront arrives here once per step
                gc = 0;
                __syncthreads();
                cur ^= 1;
                q++;
                if (q < a.q1) cf = res_coef(a, q);
            }
        }
    };
    int64_t s0 = 0;
    for (; s0 + PF <= total; s0 += PF) {
#pragma unroll
        for (int j = 0; j < PF; j++) round(A[j]);
    }
#pragma unroll
    for (int j = 0; j < PF; j++)
        if (s0 + j < total) round(A[j]);
    if (bad) atomicOr(a.err, ERR_NONFINITE);

    // ---- state out: full padded rows (zeros beyond the held columns)
    for (int e = tid; e < 16 * a.ld; e += 256) {
        const int rl = e / a.ld, k = e - rl * a.ld;
        const int64_t g = (int64_t)(r0 + rl) * a.ld + k;
        const bool in = k < nk;
        a.phi_out[g] = in ? x32[rl * a.ldf + k] : 0.0f;
        a.p[g] = in ? p32[rl * a.ldf + k] : 0.0f;
        a.xb_out[g] = in ? xbl[cur * 16 * a.ldb + rl * a.ldb + k] : (bf16)0.0f;
    }
}

// MFMA-tiled copy of the stored J for the resident plan: block (t, m) holds, for
// lanes l = 0..63 in order, the elements J[16 t + (l & 15)][128 m + 32 k + 8 (l >> 4)
// + 0..7] for k = 0..3 (the A-operand fragments of chunks 4m..4m+3 of row tile t).
// Rows up to 16 ntile and columns up to 128 nrounds lie inside the padded Np x Np
// storage, whose padding is zero.
__global__ void k_tile_j(const uint8_t *__restrict__ J, int Np, int ntile, int nrounds, int esz,
                         uint8_t *__restrict__ out) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (t, m, lane, k)
    const int64_t n = (int64_t)ntile * nrounds * 64 * 4;
    if (g >= n) return;
    const int k = (int)(g & 3), lane = (int)((g >> 2) & 63);
    const int64_t tm = g >> 8;
    const int m = (int)(tm % nrounds), t = (int)(tm / nrounds);
    const int row = 16 * t + (lane & 15), col = 128 * m + 32 * k + 8 * (lane >> 4);
    const uint8_t *src = J + ((int64_t)row * Np + col) * esz;
    uint8_t *dst = out + g * 8 * esz;
    for (int b = 0; b < 8 * esz; b++) dst[b] = src[b];
}

int64_t resident_tile_bytes(const Instance &I) {
    const int ntile = (I.N + 15) / 16, nrounds = ((I.N + 31) / 32 + 3) / 4;
    return (int64_t)ntile * nrounds * 64 * 32 * (I.jt == JT_BF16 ? 2 : 1);
}

// Whether the resident plan applies: BF16 or FP8 J, every wavefront owns at
// least one row tile, and the LDS footprint fits the device.
bool resident_fits(const Instance &I, int max_lds) {
    if (I.layout != HQA_DENSE || (I.jt != JT_BF16 && I.jt != JT_FP8)) return false;
    if ((I.N + 15) / 16 < 4) return false;
    return resident_lds_bytes(I.N) <= (size_t)max_lds;
}

template <int JT, int PF, bool WIN, int MP>
static hipError_t launch_resm(const ResArgs &a, int grid, size_t lds, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)k_md_resident<JT, PF, WIN, MP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    k_md_resident<JT, PF, WIN, MP><<<grid, 256, lds, st>>>(a);
    return hipGetLastError();
}

// MP: the potential exponent when it is the paper's M = 6 (power loop unrolled), else 0.
template <int JT, int PF, bool WIN>
static hipError_t launch_res(const ResArgs &a, int grid, size_t lds, hipStream_t st) {
    return a.M == 6 ? launch_resm<JT, PF, WIN, 6>(a, grid, lds, st)
                    : launch_resm<JT, PF, WIN, 0>(a, grid, lds, st);
}

// Steps [q0, q1) in at most two launches: the part before the averaging window
// and the part inside it.
// Build the MFMA-tiled copy of a BF16 or FP8 J once per instance (on first use).
hipError_t ensure_tiled_j(Instance &I, hipStream_t st) {
    if (I.Jt) return hipSuccess;
    if (I.jt != JT_BF16 && I.jt != JT_FP8) return hipErrorNotSupported;
    const int esz = I.jt == JT_BF16 ? 2 : 1;
    const int64_t tb = resident_tile_bytes(I);
    hipError_t e = dev_malloc(&I.Jt, tb);
    if (e != hipSuccess) {
        I.Jt = nullptr;
        return e;
    }
    const int64_t n = tb / (8 * esz);
    k_tile_j<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
        (const uint8_t *)I.Js, I.Np, (I.N + 15) / 16, ((I.N + 31) / 32 + 3) / 4, esz,
        (uint8_t *)I.Jt);
    return hipGetLastError();
}

hipError_t launch_md_resident(hqa_md *md, Instance &I, int64_t q0, int64_t q1) {
    const int64_t tb = resident_tile_bytes(I);
    hipError_t et = ensure_tiled_j(I, md->stream);
    if (et != hipSuccess) return et;
    const int64_t qw = md->sch.T - md->sch.W;   // first step whose phi' enters the window
    const size_t lds = resident_lds_bytes(I.N);
    const int grid = I.Rp / 16;
    for (int part = 0; part < 2; part++) {
        const int64_t a0 = part == 0 ? q0 : std::max(q0, qw);
        const int64_t a1 = part == 0 ? std::min(q1, qw) : q1;
        if (a1 <= a0) continue;
        ResArgs a;
        a.N = I.N; a.Np = I.Np; a.R = md->R; a.M = md->sch.M; a.ld = I.ld;
        a.nck = (I.N + 31) / 32;
        a.ntile = (I.N + 15) / 16;
        a.nrounds = (a.nck + 3) / 4;
        const int nk = a.nck * 32;
        a.ldb = nk + 8; a.ldf = nk + 4;
        a.T = md->sch.T; a.q0 = a0; a.q1 = a1; a.W = md->sch.W; a.rg = (float)md->sch.r_g;
        a.J = I.Jt; a.h = I.h32; a.a32 = md->a32; a.b32 = md->b32;
        a.jbytes = (int)tb;
        a.phi_in = I.phi32[I.cur]; a.xb_in = I.phib[I.cur];
        a.phi_out = I.phi32[I.cur ^ 1]; a.xb_out = I.phib[I.cur ^ 1];
        a.p = I.p32; a.S = I.S32; a.err = md->err;
        hipError_t e;
        if (I.jt == JT_FP8)
            e = part ? launch_res<JT_FP8, 2, true>(a, grid, lds, md->stream)
                     : launch_res<JT_FP8, 2, false>(a, grid, lds, md->stream);
        else
            e = part ? launch_res<JT_BF16, 1, true>(a, grid, lds, md->stream)
                     : launch_res<JT_BF16, 1, false>(a, grid, lds, md->stream);
        if (e != hipSuccess) return e;
        I.cur ^= 1;
    }
    return hipSuccess;
}

}  // namespace hqa
