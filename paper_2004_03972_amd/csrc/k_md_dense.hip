// k_md_dense.hip -- dense field U = J Phi on MFMA with the leapfrog fused into
// the epilogue, one launch per MD step.
//
// Layout: J is stored Np x Np (N padded to a multiple of 128, zeros outside),
// row-major, as FP32, BF16 or FP8 e4m3.  The state is replica-major [Rp][ld]
// (ld = Np): row r of the binary32 fluxes / momenta / window sum and of the
// BF16 operand copy is one replica.  With U[i][r] = sum_k J[i][k] Phi[r][k],
// the A operand (16 rows i x K) and the B operand (K x 16 replicas r) are both
// read as 16-byte runs along k, and each lane's accumulator holds four
// consecutive rows of one replica, so the epilogue reads and writes 16-byte
// vectors of the state.
//
// Workgroup: a block of TM x TN output tiles (16 TM rows x 16 TN replicas; the
// tuner picks TM in {1, 2} and TN in {1, 2, 4}, by default 2 x the widest TN that
// divides the padded replica count), K split over the four wavefronts by
// accumulation chain.  The dense field is accumulated in four chains (K chunk c
// of 32 columns for BF16 operands, 16 for FP32, feeds chain c mod 4; see
// combine4), and wavefront w computes chain w of every tile of the block:
// chunks w, w+4, w+8, ... in ascending order, four chunks' loads in flight
// together, each loaded fragment feeding several MFMAs.  The partial tiles meet
// in LDS; the combine (a0 + a1) + (a2 + a3) and the leapfrog are shared out over
// the wavefronts.  The result is bit-identical to the batched and persistent
// kernels, which accumulate the same chains.
#include <type_traits>

#include "hqa_internal.h"
#include "md_epilogue.h"

namespace hqa {

typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;

struct DenseArgs {
    int N, Np, R, Rp, ld, M;
    int64_t T;
    int W;
    float rg;
    const void *J;
    const float *h;
    const float *a32, *b32;
    const float *phi_in;
    const bf16 *xb_in;
    float *phi_out, *p, *S;
    bf16 *xb_out;
    float *u_out;       // field-only mode: U written here ([R][ld]), no update
    int jt;             // storage type of J (host-side dispatch)
    float *st;          // early-stop statistics (9 x state size) or null
    int64_t sst;
    const float *inv_n2;
    int32_t *err;
    const void *Jt;     // MFMA-tiled copy of a BF16 / FP8 J (tiled plans), else null
    int ntile, nrounds; // its row tiles (of 16) and 128-column groups
};

// Eight FP8 e4m3 codes to eight BF16 values (exact: e4m3 embeds in bf16).
__device__ __forceinline__ bf16x8 fp8x8_to_bf16(uint2 raw) {
    bf16x2 a = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.x, 1.0f, false);
    bf16x2 b = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.x, 1.0f, true);
    bf16x2 c = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.y, 1.0f, false);
    bf16x2 d = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(raw.y, 1.0f, true);
    bf16x8 o;
    o[0] = a[0]; o[1] = a[1]; o[2] = b[0]; o[3] = b[1];
    o[4] = c[0]; o[5] = c[1]; o[6] = d[0]; o[7] = d[1];
    return o;
}

// Chain w of a block of TM x TN output tiles (rows i0 + 16 tm, replicas r0 + 16 tn):
// per chunk the wavefront loads TM A fragments and TN B fragments and issues
// TM * TN MFMAs, so each fragment is reused across the block.  TJ: the A fragments
// come from the MFMA-tiled copy of J (a 16-row x 128-column group is one contiguous
// block whose four chunks the four wavefronts read together) instead of from the
// row-major storage (16 rows of 64 or 32 bytes per load); same fragments.
template <int JT, int TM, int TN, int CB, bool TJ = false>
__device__ __forceinline__ void chain_block(const DenseArgs &a, int i0, int r0, int lane, int w,
                                            f32x4 (&acc)[TM][TN]) {
    const int kg = lane >> 4;
#pragma unroll
    for (int tm = 0; tm < TM; tm++)
#pragma unroll
        for (int tn = 0; tn < TN; tn++) acc[tm][tn] = (f32x4){0.f, 0.f, 0.f, 0.f};
    if constexpr (JT == JT_F32) {
        const int nch = a.Np / 64;
        for (int m0 = 0; m0 < nch; m0 += CB) {
            float4 A[CB][TM], B[CB][TN];
#pragma unroll
            for (int m = 0; m < CB; m++) {
                if (m0 + m >= nch) continue;
                const int kk = 16 * (w + 4 * (m0 + m)) + 4 * kg;
#pragma unroll
                for (int tm = 0; tm < TM; tm++)
                    A[m][tm] = *(const float4 *)((const float *)a.J +
                                                 (int64_t)(i0 + 16 * tm + (lane & 15)) * a.Np + kk);
#pragma unroll
                for (int tn = 0; tn < TN; tn++)
                    B[m][tn] = *(const float4 *)(a.phi_in +
                                                 (int64_t)(r0 + 16 * tn + (lane & 15)) * a.ld + kk);
            }
#pragma unroll
            for (int m = 0; m < CB; m++) {
                if (m0 + m >= nch) continue;
#pragma unroll
                for (int tm = 0; tm < TM; tm++)
#pragma unroll
                    for (int tn = 0; tn < TN; tn++) {
                        f32x4 &c = acc[tm][tn];
                        c = __builtin_amdgcn_mfma_f32_16x16x4f32(A[m][tm].x, B[m][tn].x, c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x4f32(A[m][tm].y, B[m][tn].y, c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x4f32(A[m][tm].z, B[m][tn].z, c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x4f32(A[m][tm].w, B[m][tn].w, c, 0, 0, 0);
                    }
            }
        }
    } else {
        typedef typename std::conditional<JT == JT_BF16, bf16x8, uint2>::type AT;
        constexpr int esz = JT == JT_BF16 ? 2 : 1;
        const int nch = a.Np / 128;
        for (int m0 = 0; m0 < nch; m0 += CB) {
            AT A[CB][TM];
            bf16x8 B[CB][TN];
#pragma unroll
            for (int m = 0; m < CB; m++) {
                if (m0 + m >= nch) continue;
                const int kk = 32 * (w + 4 * (m0 + m)) + 8 * kg;
#pragma unroll
                for (int tm = 0; tm < TM; tm++) {
                    if constexpr (TJ) {
                        const int t = i0 / 16 + tm;   // row tiles past the copy are padding
                        A[m][tm] = t < a.ntile
                                       ? *(const AT *)((const uint8_t *)a.Jt +
                                                       ((((int64_t)t * a.nrounds + m0 + m) * 64 + lane) * 4 + w) *
                                                           8 * esz)
                                       : AT{};
                    } else {
                        A[m][tm] = *(const AT *)((const uint8_t *)a.J +
                                                 ((int64_t)(i0 + 16 * tm + (lane & 15)) * a.Np + kk) * esz);
                    }
                }
#pragma unroll
                for (int tn = 0; tn < TN; tn++)
                    B[m][tn] = *(const bf16x8 *)(a.xb_in + (int64_t)(r0 + 16 * tn + (lane & 15)) * a.ld + kk);
            }
#pragma unroll
            for (int m = 0; m < CB; m++) {
                if (m0 + m >= nch) continue;
#pragma unroll
                for (int tm = 0; tm < TM; tm++) {
                    bf16x8 av;
                    if constexpr (JT == JT_BF16) av = A[m][tm];
                    else av = fp8x8_to_bf16(A[m][tm]);
#pragma unroll
                    for (int tn = 0; tn < TN; tn++)
                        acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, B[m][tn], acc[tm][tn], 0, 0, 0);
                }
            }
        }
    }
}

// State of four consecutive rows (ib..ib+3) of one replica that the update reads,
// loaded before the field so that its latency overlaps the field's loads.
struct TileState {
    float4 x, p, s;
    float h[4];
};

__device__ __forceinline__ void load_tile_state(const DenseArgs &a, int64_t q, int col, int ib,
                                                TileState &ts) {
    const int64_t base = (int64_t)col * a.ld + ib;
    ts.x = *(const float4 *)(a.phi_in + base);
    ts.p = *(const float4 *)(a.p + base);
    ts.s = q + 1 >= a.T - a.W + 1 ? *(const float4 *)(a.S + base) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int v = 0; v < 4; v++) ts.h[v] = ib + v < a.N ? a.h[ib + v] : 0.f;
}

// Leapfrog of four consecutive rows (ib..ib+3) of replica col with field u.
__device__ __forceinline__ void dense_update(const DenseArgs &a, int64_t q, int col, int ib,
                                             const f32x4 &u, const StepCoef &c, const TileState &ts) {
    const int64_t base = (int64_t)col * a.ld + ib;
    float xs[4] = {ts.x.x, ts.x.y, ts.x.z, ts.x.w}, ps[4] = {ts.p.x, ts.p.y, ts.p.z, ts.p.w}, xn[4];
    bool bad = false;
#pragma unroll
    for (int v = 0; v < 4; v++) {
        if (ib + v < a.N) {
            leapfrog(c, xs[v], u[v], ts.h[v], ps[v], xn[v]);
            if (a.st) es_accumulate(a.st, a.sst, base + v, xs[v], xn[v], u[v], ps[v],
                                    a.inv_n2[ib + v]);
            bad |= !isfinite(xn[v]) || !isfinite(ps[v]);
        } else {
            xn[v] = 0.0f;
            ps[v] = 0.0f;
        }
    }
    *(float4 *)(a.phi_out + base) = make_float4(xn[0], xn[1], xn[2], xn[3]);
    *(float4 *)(a.p + base) = make_float4(ps[0], ps[1], ps[2], ps[3]);
    if (a.xb_out) {
        typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
        bf16x4 b = {(bf16)xn[0], (bf16)xn[1], (bf16)xn[2], (bf16)xn[3]};
        *(bf16x4 *)(a.xb_out + base) = b;
    }
    if (q + 1 >= a.T - a.W + 1) {
        float4 s = ts.s;
        s.x = s.x + xn[0]; s.y = s.y + xn[1]; s.z = s.z + xn[2]; s.w = s.w + xn[3];
        *(float4 *)(a.S + base) = s;
    }
    if (bad) atomicOr(a.err, ERR_NONFINITE);
}

// Block of TM x TN output tiles (32 rows x 16 TN replicas for TM = 2): each
// wavefront accumulates one chain of every tile; the partial tiles meet in LDS
// and wavefront w combines and updates tiles w, w + 4, ... in chain order.  The
// state these updates read is loaded first, together with the field operands.
template <int JT, int TM, int TN, bool FIELD_ONLY, int CB = 4, bool TJ = false>
__global__ __launch_bounds__(256) void k_step_block(DenseArgs a, int64_t q) {
    constexpr int NT = (TM * TN + 3) / 4;   // tiles updated per wavefront
    __shared__ f32x4 part[4][TM * TN][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i0 = blockIdx.x * 16 * TM, r0 = blockIdx.y * 16 * TN;
    StepCoef cf;
    TileState ts[NT];
    if constexpr (!FIELD_ONLY) {
        cf = step_coef(a.a32, a.b32, q, a.rg, a.M);
#pragma unroll
        for (int k = 0; k < NT; k++) {
            const int t = w + 4 * k;
            const int tm = t / TN, tn = t % TN;
            const int col = r0 + 16 * tn + (lane & 15);
            const int ib = i0 + 16 * tm + 4 * (lane >> 4);
            if (t < TM * TN && col < a.R && ib < a.N) load_tile_state(a, q, col, ib, ts[k]);
        }
    }
    f32x4 acc[TM][TN];
    chain_block<JT, TM, TN, CB, TJ>(a, i0, r0, lane, w, acc);
#pragma unroll
    for (int tm = 0; tm < TM; tm++)
#pragma unroll
        for (int tn = 0; tn < TN; tn++) part[w][tm * TN + tn][lane] = acc[tm][tn];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NT; k++) {
        const int t = w + 4 * k;
        if (t >= TM * TN) continue;
        const int tm = t / TN, tn = t % TN;
        const int col = r0 + 16 * tn + (lane & 15);
        const int ib = i0 + 16 * tm + 4 * (lane >> 4);
        if (col >= a.R || ib >= a.N) continue;
        const f32x4 parts[4] = {part[0][t][lane], part[1][t][lane], part[2][t][lane],
                                part[3][t][lane]};
        const f32x4 u = combine4(parts);
        if constexpr (FIELD_ONLY) {
            *(float4 *)(a.u_out + (int64_t)col * a.ld + ib) = make_float4(u[0], u[1], u[2], u[3]);
        } else {
            dense_update(a, q, col, ib, u, cf, ts[k]);
        }
    }
}

static DenseArgs dense_args(hqa_md *md, Instance &I) {
    DenseArgs a;
    a.N = I.N; a.Np = I.Np; a.R = md->R; a.Rp = I.Rp; a.ld = I.ld; a.M = md->sch.M;
    a.T = md->sch.T; a.W = md->sch.W; a.rg = (float)md->sch.r_g;
    a.J = I.Js; a.h = I.h32; a.a32 = md->a32; a.b32 = md->b32;
    a.phi_in = I.phi32[I.cur]; a.xb_in = I.phib[I.cur];
    a.phi_out = I.phi32[I.cur ^ 1]; a.xb_out = I.phib[I.cur ^ 1];
    a.p = I.p32; a.S = I.S32; a.u_out = nullptr; a.err = md->err; a.jt = I.jt;
    a.st = nullptr; a.sst = (int64_t)I.Rp * I.ld; a.inv_n2 = I.inv_n2;
    a.Jt = nullptr; a.ntile = (I.N + 15) / 16; a.nrounds = I.Np / 128;
    return a;
}

// Replica tiles per block: 4 (64 replicas) when they divide Rp, else 2, else 1.
static int block_tn(int Rp) { return Rp % 64 == 0 ? 4 : Rp % 32 == 0 ? 2 : 1; }

// Blocks of tm x tn output tiles: 16 tm rows x 16 tn replicas per workgroup; cb
// chunks of each chain's loads in flight together (8: a chain of up to eight chunks
// costs one round trip to L2).
template <int JT, bool FO, int CB, bool TJ>
static void launch_cb(const DenseArgs &a, int tm, int tn, int64_t q, hipStream_t st) {
    dim3 grid(a.Np / (16 * tm), a.Rp / (16 * tn));
    if (tm == 2) {
        if (tn == 4) k_step_block<JT, 2, 4, FO, CB, TJ><<<grid, 256, 0, st>>>(a, q);
        else if (tn == 2) k_step_block<JT, 2, 2, FO, CB, TJ><<<grid, 256, 0, st>>>(a, q);
        else k_step_block<JT, 2, 1, FO, CB, TJ><<<grid, 256, 0, st>>>(a, q);
    } else {
        if (tn == 4) k_step_block<JT, 1, 4, FO, CB, TJ><<<grid, 256, 0, st>>>(a, q);
        else if (tn == 2) k_step_block<JT, 1, 2, FO, CB, TJ><<<grid, 256, 0, st>>>(a, q);
        else k_step_block<JT, 1, 1, FO, CB, TJ><<<grid, 256, 0, st>>>(a, q);
    }
}

template <int JT, bool FO>
static void launch_jt(const DenseArgs &a, int tm, int tn, int cb, int64_t q, hipStream_t st) {
    if constexpr (JT != JT_F32 && !FO) {
        if (a.Jt) {
            if (cb == 8) launch_cb<JT, FO, 8, true>(a, tm, tn, q, st);
            else launch_cb<JT, FO, 4, true>(a, tm, tn, q, st);
            return;
        }
    }
    if (cb == 8) launch_cb<JT, FO, 8, false>(a, tm, tn, q, st);
    else launch_cb<JT, FO, 4, false>(a, tm, tn, q, st);
}

template <bool FO>
static void launch_one(const DenseArgs &a, int tm, int tn, int cb, int64_t q, hipStream_t st) {
    switch (a.jt) {
        case JT_F32: launch_jt<JT_F32, FO>(a, tm, tn, cb, q, st); break;
        case JT_BF16: launch_jt<JT_BF16, FO>(a, tm, tn, cb, q, st); break;
        default: launch_jt<JT_FP8, FO>(a, tm, tn, cb, q, st); break;
    }
}

hipError_t launch_md_steps_dense(hqa_md *md, Instance &I, int64_t q0, int64_t q1) {
    // tile width: the tuner's choice when it divides the padded replica count
    const int tn = (I.step_tn == 1 || I.step_tn == 2 || I.step_tn == 4) &&
                           I.Rp % (16 * I.step_tn) == 0
                       ? I.step_tn
                       : block_tn(I.Rp);
    const int tm = I.step_tm == 1 ? 1 : 2;   // Np is a multiple of 128: both divide it
    const int cb = I.step_cb == 8 ? 8 : 4;
    if (I.step_tj) {
        hipError_t e = ensure_tiled_j(I, md->stream);
        if (e != hipSuccess) return e;
    }
    for (int64_t q = q0; q < q1; q++) {
        DenseArgs a = dense_args(md, I);
        if (I.step_tj) a.Jt = I.Jt;
        if (I.st && stats_step(md, q)) a.st = I.st;
        launch_one<false>(a, tm, tn, cb, q, md->stream);
        I.cur ^= 1;
    }
    return hipGetLastError();
}

hipError_t launch_field_dense(hqa_md *md, Instance &I, float *u, hipStream_t st) {
    DenseArgs a = dense_args(md, I);
    a.u_out = u;
    launch_one<true>(a, 2, block_tn(a.Rp), 4, 0, st);
    return hipGetLastError();
}

}  // namespace hqa
