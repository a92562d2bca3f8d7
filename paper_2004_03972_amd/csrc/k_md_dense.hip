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
// Workgroup tile: 32 rows x 32 replicas, one 16 x 16 MFMA tile per wavefront.
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

// Accumulate one 16x16 tile U[i0..i0+16)[r0..r0+16) over the full K = Np in the
// four chains of combine4 (chunk c -> chain c mod 4).
template <int JT>
__device__ __forceinline__ f32x4 tile_field(const DenseArgs &a, int i0, int r0, int lane) {
    const int row = i0 + (lane & 15), col = r0 + (lane & 15), kg = lane >> 4;
    f32x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; j++) acc[j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    // Np is a multiple of 128: whole groups of four chunks; the next group's
    // operands are loaded while the current group's MFMAs run.
    if constexpr (JT == JT_F32) {
        const float *Ja = (const float *)a.J + (int64_t)row * a.Np + 4 * kg;
        const float *Xb = a.phi_in + (int64_t)col * a.ld + 4 * kg;
        const int ngroups = a.Np / 64;
        float4 A[4], B[4], An[4], Bn[4];
#pragma unroll
        for (int j = 0; j < 4; j++) { A[j] = *(const float4 *)(Ja + 16 * j); B[j] = *(const float4 *)(Xb + 16 * j); }
        for (int gi = 0; gi < ngroups; gi++) {
            if (gi + 1 < ngroups) {
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    An[j] = *(const float4 *)(Ja + (gi + 1) * 64 + 16 * j);
                    Bn[j] = *(const float4 *)(Xb + (gi + 1) * 64 + 16 * j);
                }
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[j].x, B[j].x, acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[j].y, B[j].y, acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[j].z, B[j].z, acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[j].w, B[j].w, acc[j], 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < 4; j++) { A[j] = An[j]; B[j] = Bn[j]; }
        }
    } else {
        typedef typename std::conditional<JT == JT_BF16, bf16x8, uint2>::type AT;
        const uint8_t *Ja = (const uint8_t *)a.J + ((int64_t)row * a.Np + 8 * kg) * (JT == JT_BF16 ? 2 : 1);
        const bf16 *Xb = a.xb_in + (int64_t)col * a.ld + 8 * kg;
        const int ngroups = a.Np / 128;
        AT A[4], An[4];
        bf16x8 B[4], Bn[4];
        auto load = [&](int gi, AT (&Ag)[4], bf16x8 (&Bg)[4]) {
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int kk = gi * 128 + 32 * j;
                Ag[j] = *(const AT *)(Ja + kk * (JT == JT_BF16 ? 2 : 1));
                Bg[j] = *(const bf16x8 *)(Xb + kk);
            }
        };
        load(0, A, B);
        for (int gi = 0; gi < ngroups; gi++) {
            if (gi + 1 < ngroups) load(gi + 1, An, Bn);
#pragma unroll
            for (int j = 0; j < 4; j++) {
                bf16x8 av;
                if constexpr (JT == JT_BF16) av = A[j];
                else av = fp8x8_to_bf16(A[j]);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, B[j], acc[j], 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < 4; j++) { A[j] = An[j]; B[j] = Bn[j]; }
        }
    }
    return combine4(acc);
}

template <int JT, bool FIELD_ONLY>
__global__ __launch_bounds__(256) void k_step_dense(DenseArgs a, int64_t q) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i0 = blockIdx.x * 32 + 16 * (w & 1);
    const int r0 = blockIdx.y * 32 + 16 * (w >> 1);
    if (r0 >= a.Rp || i0 >= a.Np) return;
    f32x4 acc = tile_field<JT>(a, i0, r0, lane);
    const int col = r0 + (lane & 15);
    const int ib = i0 + 4 * (lane >> 4);
    if (col >= a.R || ib >= a.N) return;
    const int64_t base = (int64_t)col * a.ld + ib;
    if constexpr (FIELD_ONLY) {
        *(float4 *)(a.u_out + base) = make_float4(acc[0], acc[1], acc[2], acc[3]);
        return;
    } else {
        const StepCoef c = step_coef(a.a32, a.b32, q, a.rg, a.M);
        float4 x = *(const float4 *)(a.phi_in + base);
        float4 p = *(const float4 *)(a.p + base);
        float xs[4] = {x.x, x.y, x.z, x.w}, ps[4] = {p.x, p.y, p.z, p.w}, xn[4];
        bool bad = false;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            if (ib + v < a.N) {
                leapfrog(c, xs[v], acc[v], a.h[ib + v], ps[v], xn[v]);
                if (a.st) es_accumulate(a.st, a.sst, base + v, xs[v], xn[v], acc[v], ps[v],
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
            float4 s = *(const float4 *)(a.S + base);
            s.x = s.x + xn[0]; s.y = s.y + xn[1]; s.z = s.z + xn[2]; s.w = s.w + xn[3];
            *(float4 *)(a.S + base) = s;
        }
        if (bad) atomicOr(a.err, ERR_NONFINITE);
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
    return a;
}

template <bool FO>
static void launch_one(hqa_md *md, const DenseArgs &a, dim3 grid, int64_t q, hipStream_t st) {
    switch (a.jt) {
        case JT_F32: k_step_dense<JT_F32, FO><<<grid, 256, 0, st>>>(a, q); break;
        case JT_BF16: k_step_dense<JT_BF16, FO><<<grid, 256, 0, st>>>(a, q); break;
        default: k_step_dense<JT_FP8, FO><<<grid, 256, 0, st>>>(a, q); break;
    }
}

hipError_t launch_md_steps_dense(hqa_md *md, Instance &I, int64_t q0, int64_t q1) {
    dim3 grid(I.Np / 32, (I.Rp + 31) / 32);
    for (int64_t q = q0; q < q1; q++) {
        DenseArgs a = dense_args(md, I);
        if (I.st && q >= md->stats_k0 && q < md->stats_k1) a.st = I.st;
        launch_one<false>(md, a, grid, q, md->stream);
        I.cur ^= 1;
    }
    return hipGetLastError();
}

hipError_t launch_field_dense(hqa_md *md, Instance &I, float *u, hipStream_t st) {
    dim3 grid(I.Np / 32, (I.Rp + 31) / 32);
    DenseArgs a = dense_args(md, I);
    a.u_out = u;
    launch_one<true>(md, a, grid, 0, st);
    return hipGetLastError();
}

}  // namespace hqa
