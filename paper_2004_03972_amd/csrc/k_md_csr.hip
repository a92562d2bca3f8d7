// k_md_csr.hip -- sparse field (CSR SpMM over replica-contiguous fluxes) with the
// leapfrog fused, one launch per MD step.
//
// Layout: the binary32 state is spin-major [N][Rp] (Rp = R padded to a multiple
// of 4): row i holds spin i of every replica, so a neighbour's fluxes are one
// contiguous run.  Each thread owns four consecutive replicas of one spin and
// walks that spin's couplings in ascending column order; the column indices
// and values are uniform across the threads of a row (scalar broadcasts) and
// every flux gather is a coalesced 16-byte-per-lane read.  Per spin update the
// kernel moves 16 bytes of state (read phi, read and write p, write phi').
#include "hqa_internal.h"
#include "md_epilogue.h"

namespace hqa {

struct CsrArgs {
    int N, R, Rq, M;     // Rq = Rp / 4 threads per row
    int64_t T;
    int W;
    float rg;
    const int32_t *rp, *ci;
    const float *v;
    const float *h;
    const float *a32, *b32;
    const float *phi_in;
    float *phi_out, *p, *S;
    float *u_out;
    int32_t *err;
    float *st;             // early-stop statistics (9 x state size) or null
    int64_t sst;           // stride between the nine statistics arrays
    const float *inv_n2;   // 1 / ||J_i||_2
};

// Workgroup b of a launch runs on XCD b mod 8, each XCD with its own L2.  The
// remap gives XCD x the contiguous block range [x nb/8, (x+1) nb/8) (the last
// nb mod 8 blocks keep their index), so rows whose neighbours are nearby in index
// (lattices, banded graphs) find those neighbours' fluxes in their own L2 instead
// of fetching them into a second and third one.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t per = nb / 8;
    return b < per * 8 ? (b % 8) * per + b / 8 : b;
}

template <bool FIELD_ONLY>
__global__ __launch_bounds__(256) void k_step_csr(CsrArgs a, int64_t q) {
    int64_t t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.N * a.Rq) return;
    const int i = (int)(t / a.Rq), c4 = (int)(t % a.Rq);
    const int Rp = a.Rq * 4;
    const float4 *X = (const float4 *)a.phi_in;
    float4 u = make_float4(0.f, 0.f, 0.f, 0.f);
    const int e0 = a.rp[i], e1 = a.rp[i + 1];
    for (int e = e0; e < e1; e++) {
        const int j = a.ci[e];
        const float w = a.v[e];
        const float4 xj = X[(int64_t)j * a.Rq + c4];
        u.x = fmaf(w, xj.x, u.x);
        u.y = fmaf(w, xj.y, u.y);
        u.z = fmaf(w, xj.z, u.z);
        u.w = fmaf(w, xj.w, u.w);
    }
    const int64_t base = (int64_t)i * Rp + 4 * c4;
    if constexpr (FIELD_ONLY) {
        *(float4 *)(a.u_out + base) = u;
        return;
    } else {
        const StepCoef c = step_coef(a.a32, a.b32, q, a.rg, a.M);
        const float hi = a.h[i];
        float4 x = X[(int64_t)i * a.Rq + c4];
        float4 p = *(const float4 *)(a.p + base);
        float4 xn;
        leapfrog(c, x.x, u.x, hi, p.x, xn.x);
        leapfrog(c, x.y, u.y, hi, p.y, xn.y);
        leapfrog(c, x.z, u.z, hi, p.z, xn.z);
        leapfrog(c, x.w, u.w, hi, p.w, xn.w);
        if (a.st) {
            const float in2 = a.inv_n2[i];
            es_accumulate(a.st, a.sst, base + 0, x.x, xn.x, u.x, p.x, in2);
            es_accumulate(a.st, a.sst, base + 1, x.y, xn.y, u.y, p.y, in2);
            es_accumulate(a.st, a.sst, base + 2, x.z, xn.z, u.z, p.z, in2);
            es_accumulate(a.st, a.sst, base + 3, x.w, xn.w, u.w, p.w, in2);
        }
        *(float4 *)(a.phi_out + base) = xn;
        *(float4 *)(a.p + base) = p;
        if (q + 1 >= a.T - a.W + 1) {
            float4 s = *(const float4 *)(a.S + base);
            s.x = s.x + xn.x; s.y = s.y + xn.y; s.z = s.z + xn.z; s.w = s.w + xn.w;
            *(float4 *)(a.S + base) = s;
        }
        bool bad = !isfinite(xn.x) || !isfinite(xn.y) || !isfinite(xn.z) || !isfinite(xn.w) ||
                   !isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z) || !isfinite(p.w);
        if (bad) atomicOr(a.err, ERR_NONFINITE);
    }
}

static CsrArgs csr_args(hqa_md *md, Instance &I) {
    CsrArgs a;
    a.N = I.N; a.R = md->R; a.Rq = I.Rp / 4; a.M = md->sch.M;
    a.T = md->sch.T; a.W = md->sch.W; a.rg = (float)md->sch.r_g;
    a.rp = I.rp; a.ci = I.ci; a.v = I.v32; a.h = I.h32; a.a32 = md->a32; a.b32 = md->b32;
    a.phi_in = I.phi32[I.cur]; a.phi_out = I.phi32[I.cur ^ 1];
    a.p = I.p32; a.S = I.S32; a.u_out = nullptr; a.err = md->err;
    a.st = nullptr; a.sst = (int64_t)I.N * I.ld; a.inv_n2 = I.inv_n2;
    return a;
}

hipError_t launch_md_steps_csr(hqa_md *md, Instance &I, int64_t q0, int64_t q1) {
    int64_t n = (int64_t)I.N * (I.Rp / 4);
    unsigned blocks = (unsigned)((n + 255) / 256);
    for (int64_t q = q0; q < q1; q++) {
        CsrArgs a = csr_args(md, I);
        if (I.st && stats_step(md, q)) a.st = I.st;
        k_step_csr<false><<<blocks, 256, 0, md->stream>>>(a, q);
        I.cur ^= 1;
    }
    return hipGetLastError();
}

hipError_t launch_field_csr(hqa_md *md, Instance &I, float *u, hipStream_t st) {
    int64_t n = (int64_t)I.N * (I.Rp / 4);
    CsrArgs a = csr_args(md, I);
    a.u_out = u;
    k_step_csr<true><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a, 0);
    return hipGetLastError();
}

}  // namespace hqa
