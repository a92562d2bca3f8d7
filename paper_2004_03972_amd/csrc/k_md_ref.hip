// k_md_ref.hip -- binary64 reference MD step, field and MD Hamiltonian.
//
// The step uses a fixed operation order (built with -ffp-contract=off):
//   u   = fma chain over the stored couplings of row i in ascending column order
//   v   = phi^(M-1) by M-2 successive multiplications
//   g   = u + (2 h) |phi|
//   F   = (alpha (M v)) + (beta g),  F = r_g F when r_g != 1
//   p   = p - F/2 at q = 0 (initial half step), p - F afterwards
//   phi = phi + (alpha_(2q+1) p)      (alpha_(2q+1) scaled by r_g when r_g != 1)
// following the leapfrog of Methods ("Leapfrog algorithm") on Eq. 3.
#include "hqa_internal.h"

namespace hqa {

struct RefArgs {
    int N, R, M, csr;
    int64_t T;
    int W;
    double r_g;
    const double *J;
    const int32_t *rp, *ci;
    const double *h;
    const double *a64, *b64;
    const double *phi_in;
    double *phi_out, *p, *S;
    int32_t *err;
};

__device__ __forceinline__ double ref_field(const RefArgs &a, int i, const double *x) {
    double u = 0.0;
    if (!a.csr) {
        const double *Ji = a.J + (int64_t)i * a.N;
        for (int j = 0; j < a.N; j++) u = fma(Ji[j], x[j], u);
    } else {
        for (int e = a.rp[i]; e < a.rp[i + 1]; e++) u = fma(a.J[e], x[a.ci[e]], u);
    }
    return u;
}

__device__ __forceinline__ double ref_force(const RefArgs &a, int i, const double *x, double al,
                                            double be) {
    double xi = x[i];
    double u = ref_field(a, i, x);
    double v = xi;
    for (int k = 0; k < a.M - 2; k++) v = v * xi;
    double g = u + (2.0 * a.h[i]) * fabs(xi);
    double F = (al * ((double)a.M * v)) + (be * g);
    if (a.r_g != 1.0) F = a.r_g * F;
    return F;
}

__global__ void k_step_f64(RefArgs a, int64_t q) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.N * a.R) return;
    int r = (int)(t / a.N), i = (int)(t % a.N);
    const double *x = a.phi_in + (int64_t)r * a.N;
    double F = ref_force(a, i, x, a.a64[2 * q], a.b64[2 * q]);
    double p = a.p[t];
    p = (q == 0) ? p - 0.5 * F : p - F;
    double ad = a.a64[2 * q + 1];
    if (a.r_g != 1.0) ad = a.r_g * ad;
    double xn = x[i] + (ad * p);
    a.p[t] = p;
    a.phi_out[t] = xn;
    if (q + 1 >= a.T - a.W + 1) a.S[t] = a.S[t] + xn;
    if (!isfinite(xn) || !isfinite(p)) atomicOr(a.err, ERR_NONFINITE);
}

static RefArgs ref_args(hqa_md *md, Instance &I) {
    RefArgs a;
    a.N = I.N; a.R = md->R; a.M = md->sch.M; a.csr = I.layout == HQA_CSR;
    a.T = md->sch.T; a.W = md->sch.W; a.r_g = md->sch.r_g;
    a.J = I.J64; a.rp = I.rp; a.ci = I.ci; a.h = I.h64;
    a.a64 = md->a64; a.b64 = md->b64;
    a.phi_in = nullptr; a.phi_out = nullptr; a.p = I.p64; a.S = I.S64; a.err = md->err;
    return a;
}

hipError_t launch_md_steps_f64(hqa_md *md, Instance &I, int64_t q0, int64_t q1) {
    RefArgs a = ref_args(md, I);
    int64_t n = (int64_t)I.N * md->R;
    unsigned blocks = (unsigned)((n + 255) / 256);
    for (int64_t q = q0; q < q1; q++) {
        a.phi_in = I.phi64[I.cur];
        a.phi_out = I.phi64[I.cur ^ 1];
        k_step_f64<<<blocks, 256, 0, md->stream>>>(a, q);
        I.cur ^= 1;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// binary64 field u = J phi from the binary64 couplings, for any state precision.
// ---------------------------------------------------------------------------
struct F64View {
    int N, R, ld, smaj, f64;
    const double *x64;
    const float *x32;
};

__device__ __forceinline__ double view_get(const F64View &v, int r, int i) {
    if (v.f64) return v.x64[(int64_t)r * v.N + i];
    int64_t k = v.smaj ? (int64_t)i * v.ld + r : (int64_t)r * v.ld + i;
    return (double)v.x32[k];
}

static F64View make_view(hqa_md *md, Instance &I, bool phi) {
    F64View v;
    v.N = I.N; v.R = md->R; v.ld = I.ld; v.smaj = I.smaj; v.f64 = md->prec == HQA_PREC_F64_REF;
    v.x64 = phi ? I.phi64[I.cur] : I.p64;
    v.x32 = phi ? I.phi32[I.cur] : I.p32;
    return v;
}

// One workgroup per replica: the replica's fluxes are staged in LDS in binary64.
__global__ void k_field_f64(RefArgs a, F64View xv, double *u) {
    extern __shared__ double xs[];
    int r = blockIdx.x;
    for (int i = threadIdx.x; i < a.N; i += blockDim.x) xs[i] = view_get(xv, r, i);
    __syncthreads();
    for (int i = threadIdx.x; i < a.N; i += blockDim.x) u[(int64_t)r * a.N + i] = ref_field(a, i, xs);
}

hipError_t launch_field_f64(hqa_md *md, Instance &I, double *u, hipStream_t st) {
    RefArgs a = ref_args(md, I);
    F64View xv = make_view(md, I, true);
    const size_t lds = (size_t)I.N * sizeof(double);   // one replica's fluxes in binary64
    hipError_t e = hipFuncSetAttribute((const void *)k_field_f64,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    k_field_f64<<<md->R, 256, lds, st>>>(a, xv, u);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MD Hamiltonian (Eq. 3) at integer step q, binary64, one workgroup per replica.
// The momentum at integer time is p^(q) = p^(q-1/2) - F(phi^(q))/2 (q >= 1).
// ---------------------------------------------------------------------------
__global__ void k_hamiltonian(RefArgs a, F64View xv, F64View pv, int64_t q, double *H) {
    extern __shared__ double xs[];
    __shared__ double red[3][256];
    int r = blockIdx.x;
    for (int i = threadIdx.x; i < a.N; i += blockDim.x) xs[i] = view_get(xv, r, i);
    __syncthreads();
    double al = a.a64[2 * q], be = a.b64[2 * q];
    double kin = 0.0, cpl = 0.0, fld = 0.0;
    for (int i = threadIdx.x; i < a.N; i += blockDim.x) {
        double x = xs[i];
        double p = view_get(pv, r, i);
        if (q > 0) p = p - 0.5 * ref_force(a, i, xs, al, be);
        double xm = x;
        for (int k = 0; k < a.M - 1; k++) xm = xm * x;
        kin += 0.5 * p * p + xm;
        cpl += x * ref_field(a, i, xs);
        fld += a.h[i] * fabs(x) * x;
    }
    red[0][threadIdx.x] = kin; red[1][threadIdx.x] = cpl; red[2][threadIdx.x] = fld;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 3; c++) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) H[r] = al * red[0][0] + be * (0.5 * red[1][0] + red[2][0]);
}

hipError_t launch_hamiltonian(hqa_md *md, Instance &I, double *H, hipStream_t st) {
    RefArgs a = ref_args(md, I);
    F64View xv = make_view(md, I, true), pv = make_view(md, I, false);
    const size_t lds = (size_t)I.N * sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void *)k_hamiltonian,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    k_hamiltonian<<<md->R, 256, lds, st>>>(a, xv, pv, md->q, H);
    return hipGetLastError();
}

}  // namespace hqa
