// k_csr_resident.hip -- replica-resident sparse anneal: the whole run of a group
// of four replicas in one workgroup, one launch for all steps.
//
// Replicas are independent trajectories, so a workgroup that owns four replicas
// of a sparse instance needs nothing from any other workgroup.  For a bounded-
// degree graph (every row at most DMAX couplings; lattices have six) the whole
// per-step working set stays on chip for the entire anneal:
//   * the fluxes of the four replicas, double-buffered, in LDS ([N] x float4 each);
//   * the field h in LDS;
//   * each thread's spins' couplings (column, value) in registers, loaded once;
//   * each thread's momenta and window sums in registers.
// A step then reads no global memory at all: six LDS gathers of 16 bytes and the
// fused leapfrog per spin and replica, and one barrier.  1024 threads (four spins
// each at N = 4096) keep four wavefronts per SIMD to hide the LDS latency.  The
// arithmetic is the streamed CSR kernel's (field accumulated with fmaf in ascending column order
// from +0, the shared binary32 leapfrog, the window sum), so both give
// bit-identical trajectories.
#include "hqa_internal.h"
#include "md_epilogue.h"

namespace hqa {

constexpr int CSR_RES_THREADS = 1024;
constexpr int CSR_RES_DMAX = 8;    // couplings per row held in registers
constexpr int CSR_RES_RG = 4;      // replicas per workgroup

struct CsrResArgs {
    int N, M, ld;                  // ld: padded replica count (row length of the state)
    int64_t T, q0, q1;
    int W;
    float rg;
    const int32_t *rp, *ci;
    const float *v, *h, *a32, *b32;
    const float *phi_in;
    float *phi_out, *p, *S;
    int32_t *err;
};

size_t csr_resident_lds_bytes(int N) { return (size_t)N * (2 * CSR_RES_RG * 4 + 4); }

__device__ __forceinline__ StepCoef csr_res_coef(const CsrResArgs &a, int64_t q) {
    typedef const __attribute__((address_space(4))) float cfloat;   // scalar loads: q is uniform
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

// SPT spins per thread: spin i = tid + CSR_RES_THREADS k, k < SPT.  MP: the potential
// exponent when it is 6 (the paper's), else 0 for any even M.
template <int SPT, int MP>
__global__ __launch_bounds__(CSR_RES_THREADS) void k_csr_resident(CsrResArgs a) {
    extern __shared__ __align__(16) float lds_c[];
    float4 *ph0 = (float4 *)lds_c, *ph1 = ph0 + a.N;
    float *hl = (float *)(ph1 + a.N);
    const int tid = threadIdx.x;
    const int g0 = blockIdx.x * CSR_RES_RG;

    for (int i = tid; i < a.N; i += CSR_RES_THREADS) {
        ph0[i] = *(const float4 *)(a.phi_in + (int64_t)i * a.ld + g0);
        hl[i] = a.h[i];
    }
    int deg[SPT], col[SPT][CSR_RES_DMAX];
    float val[SPT][CSR_RES_DMAX];
    float4 p[SPT], S[SPT];
#pragma unroll
    for (int k = 0; k < SPT; k++) {
        const int i = tid + CSR_RES_THREADS * k;
        deg[k] = 0;
        p[k] = S[k] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int d = 0; d < CSR_RES_DMAX; d++) {
            col[k][d] = 0;
            val[k][d] = 0.0f;
        }
        if (i < a.N) {
            const int e0 = a.rp[i];
            deg[k] = a.rp[i + 1] - e0;   // the host checked deg <= CSR_RES_DMAX
#pragma unroll
            for (int d = 0; d < CSR_RES_DMAX; d++) {
                if (d < deg[k]) {
                    col[k][d] = a.ci[e0 + d];
                    val[k][d] = a.v[e0 + d];
                }
            }
            const int64_t base = (int64_t)i * a.ld + g0;
            p[k] = *(const float4 *)(a.p + base);
            S[k] = *(const float4 *)(a.S + base);
        }
    }
    __syncthreads();

    int cur = 0;
    for (int64_t q = a.q0; q < a.q1; q++) {
        const StepCoef c = csr_res_coef(a, q);
        const bool win = q + 1 >= a.T - a.W + 1;
        const float4 *X = cur ? ph1 : ph0;
        float4 *Y = cur ? ph0 : ph1;
#pragma unroll
        for (int k = 0; k < SPT; k++) {
            const int i = tid + CSR_RES_THREADS * k;
            if (i < a.N) {
                float4 u = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int d = 0; d < CSR_RES_DMAX; d++) {
                    if (d < deg[k]) {
                        const float w = val[k][d];
                        const float4 xj = X[col[k][d]];
                        u.x = fmaf(w, xj.x, u.x);
                        u.y = fmaf(w, xj.y, u.y);
                        u.z = fmaf(w, xj.z, u.z);
                        u.w = fmaf(w, xj.w, u.w);
                    }
                }
                const float hi = hl[i];
                const float4 x = X[i];
                float4 xn;
                if constexpr (MP == 6) {
                    leapfrog_m<6>(c, x.x, u.x, hi, p[k].x, xn.x);
                    leapfrog_m<6>(c, x.y, u.y, hi, p[k].y, xn.y);
                    leapfrog_m<6>(c, x.z, u.z, hi, p[k].z, xn.z);
                    leapfrog_m<6>(c, x.w, u.w, hi, p[k].w, xn.w);
                } else {
                    leapfrog(c, x.x, u.x, hi, p[k].x, xn.x);
                    leapfrog(c, x.y, u.y, hi, p[k].y, xn.y);
                    leapfrog(c, x.z, u.z, hi, p[k].z, xn.z);
                    leapfrog(c, x.w, u.w, hi, p[k].w, xn.w);
                }
                Y[i] = xn;
                if (win) {
                    S[k].x = S[k].x + xn.x; S[k].y = S[k].y + xn.y;
                    S[k].z = S[k].z + xn.z; S[k].w = S[k].w + xn.w;
                }
            }
        }
        __syncthreads();
        cur ^= 1;
    }

    // A non-finite flux or momentum never becomes finite again under the leapfrog (and
    // spreads to the neighbours through the field), so checking the final state raises
    // the same flag as checking every step.
    const float4 *X = cur ? ph1 : ph0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < SPT; k++) {
        const int i = tid + CSR_RES_THREADS * k;
        if (i < a.N) {
            const int64_t base = (int64_t)i * a.ld + g0;
            const float4 xf = X[i];
            bad |= !isfinite(xf.x) || !isfinite(xf.y) || !isfinite(xf.z) || !isfinite(xf.w) ||
                   !isfinite(p[k].x) || !isfinite(p[k].y) || !isfinite(p[k].z) ||
                   !isfinite(p[k].w);
            *(float4 *)(a.phi_out + base) = xf;
            *(float4 *)(a.p + base) = p[k];
            *(float4 *)(a.S + base) = S[k];
        }
    }
    if (bad) atomicOr(a.err, ERR_NONFINITE);
}

bool csr_resident_fits(hqa_md *md, Instance &I) {
    if (I.layout != HQA_CSR || !I.smaj || I.Rp % CSR_RES_RG != 0) return false;
    if (I.N > 4 * CSR_RES_THREADS) return false;
    if (csr_resident_lds_bytes(I.N) > (size_t)md->max_lds) return false;
    return I.max_deg >= 0 && I.max_deg <= CSR_RES_DMAX;   // max_deg: set at ingest
}

template <int SPT, int MP>
static hipError_t launch_crm(const CsrResArgs &a, int grid, size_t lds, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)k_csr_resident<SPT, MP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    k_csr_resident<SPT, MP><<<grid, CSR_RES_THREADS, lds, st>>>(a);
    return hipGetLastError();
}

template <int SPT>
static hipError_t launch_cr(const CsrResArgs &a, int grid, size_t lds, hipStream_t st) {
    return a.M == 6 ? launch_crm<SPT, 6>(a, grid, lds, st) : launch_crm<SPT, 0>(a, grid, lds, st);
}

hipError_t launch_md_csr_resident(hqa_md *md, Instance &I, int64_t q0, int64_t q1) {
    CsrResArgs a;
    a.N = I.N; a.M = md->sch.M; a.ld = I.ld;
    a.T = md->sch.T; a.q0 = q0; a.q1 = q1; a.W = md->sch.W; a.rg = (float)md->sch.r_g;
    a.rp = I.rp; a.ci = I.ci; a.v = I.v32; a.h = I.h32; a.a32 = md->a32; a.b32 = md->b32;
    a.phi_in = I.phi32[I.cur]; a.phi_out = I.phi32[I.cur ^ 1];
    a.p = I.p32; a.S = I.S32; a.err = md->err;
    const size_t lds = csr_resident_lds_bytes(I.N);
    const int grid = I.Rp / CSR_RES_RG;
    const int spt = (I.N + CSR_RES_THREADS - 1) / CSR_RES_THREADS;
    hipError_t e;
    if (spt <= 1) e = launch_cr<1>(a, grid, lds, md->stream);
    else if (spt <= 2) e = launch_cr<2>(a, grid, lds, md->stream);
    else e = launch_cr<4>(a, grid, lds, md->stream);
    if (e == hipSuccess) I.cur ^= 1;
    return e;
}

}  // namespace hqa
