// md_epilogue.h -- the fused leapfrog update of the binary32 paths.
//
// Given the local field u = sum_j J_ij phi_j of one (spin, replica) the force of
// Eq. 3 is F = alpha M phi^(M-1) + beta (u + 2 h |phi|) (times r_g), the kick is
// p -= F (F/2 on the initial half step, q = 0) and the drift is
// phi' = phi + alpha_(q+1/2) p (Methods, "Leapfrog algorithm").  The operation
// order is the same in every binary32 kernel (the library is built without fp
// contraction), so per-step and persistent launches give identical results.
#pragma once
#include <hip/hip_runtime.h>

namespace hqa {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_e;

// The dense field is accumulated in four independent MFMA chains: K chunk c
// (32 columns for BF16 operands, 16 for FP32) feeds chain c mod 4, and the field
// is (a0 + a1) + (a2 + a3).  Every dense kernel uses this decomposition, so the
// per-step and persistent launches produce identical fields, and the four chains
// keep the MFMA pipeline busy instead of waiting on one accumulator.
__device__ __forceinline__ f32x4_e combine4(const f32x4_e *a) {
    f32x4_e s01 = a[0] + a[1];
    f32x4_e s23 = a[2] + a[3];
    return s01 + s23;
}

struct StepCoef {
    float al, be;     // alpha, beta at tau = q/T
    float ad;         // alpha at tau = (q + 1/2)/T, times r_g
    float rg;
    float kick;       // 0.5 at q = 0, else 1
    int M;
};

__device__ __forceinline__ void leapfrog(const StepCoef &c, float x, float u, float h, float &p,
                                         float &xn) {
    float v = x;
    for (int k = 0; k < c.M - 2; k++) v = v * x;
    float g = u + (2.0f * h) * fabsf(x);
    float F = (c.al * ((float)c.M * v)) + (c.be * g);
    if (c.rg != 1.0f) F = c.rg * F;
    p = p - c.kick * F;
    xn = x + c.ad * p;
}

// The same sequence with the potential exponent fixed at compile time (the power
// loop unrolled; identical operations).
template <int M>
__device__ __forceinline__ void leapfrog_m(const StepCoef &c, float x, float u, float h, float &p,
                                           float &xn) {
    float v = x;
#pragma unroll
    for (int k = 0; k < M - 2; k++) v = v * x;
    float g = u + (2.0f * h) * fabsf(x);
    float F = (c.al * ((float)M * v)) + (c.be * g);
    if (c.rg != 1.0f) F = c.rg * F;
    p = p - c.kick * F;
    xn = x + c.ad * p;
}

// Statistics of the learned early stop for one (spin, replica) and one step:
// old flux xo = phi^(q), new flux xn = phi^(q+1), field u at phi^(q), momentum
// p = p^(q+1/2), nu = u / ||J_i||_2 (inv_n2 = 1/||J_i||_2, 0 for an empty row).
// Nine running sums, stored as st[j * stride + k]; sgn(0) = +1.
__device__ __forceinline__ void es_accumulate(float *st, int64_t stride, int64_t k, float xo,
                                              float xn, float u, float p, float inv_n2) {
    const float nu = u * inv_n2;
    const float so = xo < 0.0f ? -1.0f : 1.0f;
    st[0 * stride + k] += xn;
    st[1 * stride + k] += xn * xn;
    st[2 * stride + k] += fabsf(xn);
    st[3 * stride + k] += xn > 0.0f ? 1.0f : 0.0f;
    st[4 * stride + k] += ((xn < 0.0f) != (xo < 0.0f)) ? 1.0f : 0.0f;
    st[5 * stride + k] += nu;
    st[6 * stride + k] += nu * nu;
    st[7 * stride + k] += -so * nu;
    st[8 * stride + k] += p * p;
}

// The schedule values of step q as stored, and the coefficients built from them (the
// same operations as step_coef).  Persistent kernels load the next step's values a
// step ahead and build them when the step begins, so the load's latency is hidden.
struct CoefRaw {
    float al, be, ad;
};

// The tables are read-only for the whole launch and q is uniform, so the values are
// read through the constant address space (scalar loads, which do not share the
// vector memory counter with the kernel's stores).
__device__ __forceinline__ CoefRaw load_coef(const float *a32, const float *b32, int64_t q) {
    typedef const __attribute__((address_space(4))) float cfloat;
    const cfloat *A = (const cfloat *)a32;
    const cfloat *B = (const cfloat *)b32;
    return CoefRaw{A[2 * q], B[2 * q], A[2 * q + 1]};
}

__device__ __forceinline__ StepCoef make_coef(const CoefRaw &r, int64_t q, float rg, int M) {
    StepCoef c;
    c.al = r.al;
    c.be = r.be;
    c.ad = r.ad;
    if (rg != 1.0f) c.ad = rg * c.ad;
    c.rg = rg;
    c.kick = q == 0 ? 0.5f : 1.0f;
    c.M = M;
    return c;
}

__device__ __forceinline__ StepCoef step_coef(const float *a32, const float *b32, int64_t q,
                                              float rg, int M) {
    StepCoef c;
    c.al = a32[2 * q];
    c.be = b32[2 * q];
    c.ad = a32[2 * q + 1];
    if (rg != 1.0f) c.ad = rg * c.ad;
    c.rg = rg;
    c.kick = q == 0 ? 0.5f : 1.0f;
    c.M = M;
    return c;
}

}  // namespace hqa
