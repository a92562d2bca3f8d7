// k_es.hip -- learned early stop: per-spin features from the MD statistics, a
// 12-64-64-3 GELU perceptron (forward, class-weighted cross-entropy gradient,
// Adam), and the spin read-out driven by predicted labels.
//
// The paper defines no learned component; the definitions are the library's:
// statistics over a window of steps [K0, K1) (nine running sums per spin and
// replica, accumulated in the MD step epilogue), twelve features at the
// checkpoint normalised per replica, three classes {frozen +, frozen -,
// ambivalent}.  Parameter vector (5187 binary32): W1[64][12], b1[64],
// W2[64][64], b2[64], W3[3][64], b3[3], weights row-major [out][in].
#include <math.h>

#include "hqa_internal.h"

namespace hqa {

enum { NF = 12, H1 = 64, H2 = 64, NC = 3 };
enum { OFF_W1 = 0, OFF_B1 = OFF_W1 + H1 * NF, OFF_W2 = OFF_B1 + H1, OFF_B2 = OFF_W2 + H2 * H1,
       OFF_W3 = OFF_B2 + H2, OFF_B3 = OFF_W3 + NC * H2, NPARAM = OFF_B3 + NC };

// ---------------------------------------------------------------- row norms
__global__ void k_row_norms(const double *J, const int32_t *rp, const int32_t *ci, int N, int csr,
                            float *n1, float *inv_n2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double a = 0.0, b = 0.0;
    if (!csr) {
        for (int j = 0; j < N; j++) {
            double v = J[(int64_t)i * N + j];
            a += fabs(v);
            b += v * v;
        }
    } else {
        for (int e = rp[i]; e < rp[i + 1]; e++) {
            a += fabs(J[e]);
            b += J[e] * J[e];
        }
    }
    n1[i] = (float)a;
    inv_n2[i] = b > 0.0 ? (float)(1.0 / sqrt(b)) : 0.0f;
}

hipError_t launch_row_norms(const Instance &I, float *n1, float *inv_n2, hipStream_t st) {
    k_row_norms<<<(I.N + 255) / 256, 256, 0, st>>>(I.J64, I.rp, I.ci, I.N, I.layout == HQA_CSR,
                                                   n1, inv_n2);
    return hipGetLastError();
}

// ------------------------------------------------------------------ features
struct FeatArgs {
    int N, R, ld, smaj;
    int64_t sst;
    float K, tau, mean_n1;
    const float *phi, *st, *n1;
    float *feat;
};

__device__ __forceinline__ int64_t fidx(const FeatArgs &a, int r, int i) {
    return a.smaj ? (int64_t)i * a.ld + r : (int64_t)r * a.ld + i;
}

__global__ __launch_bounds__(256) void k_features(FeatArgs a) {
    __shared__ float red[2][256];
    const int r = blockIdx.x, tid = threadIdx.x;
    float s2 = 0.f, pm = 0.f;
    for (int i = tid; i < a.N; i += 256) {
        const int64_t k = fidx(a, r, i);
        const float x = a.phi[k];
        s2 += x * x;
        pm += a.st[8 * a.sst + k] / a.K;
    }
    red[0][tid] = s2;
    red[1][tid] = pm;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            red[0][tid] += red[0][tid + s];
            red[1][tid] += red[1][tid + s];
        }
        __syncthreads();
    }
    float sig = sqrtf(red[0][0] / (float)a.N);
    if (sig == 0.f) sig = 1.f;
    float pmean = red[1][0] / (float)a.N;
    if (pmean == 0.f) pmean = 1.f;
    for (int i = tid; i < a.N; i += 256) {
        const int64_t k = fidx(a, r, i);
        const float *S = a.st + k;
        const float m0 = S[0] / a.K, m5 = S[5 * a.sst] / a.K;
        float *f = a.feat + ((int64_t)r * a.N + i) * NF;
        f[0] = m0 / sig;
        f[1] = sqrtf(fmaxf(S[1 * a.sst] / a.K - m0 * m0, 0.f)) / sig;
        f[2] = (S[2 * a.sst] / a.K) / sig;
        f[3] = a.phi[k] / sig;
        f[4] = fabsf(2.f * S[3 * a.sst] / a.K - 1.f);
        f[5] = S[4 * a.sst] / a.K;
        f[6] = m5 / sig;
        f[7] = sqrtf(fmaxf(S[6 * a.sst] / a.K - m5 * m5, 0.f)) / sig;
        f[8] = (S[7 * a.sst] / a.K) / sig;
        f[9] = (S[8 * a.sst] / a.K) / pmean;
        f[10] = a.mean_n1 > 0.f ? a.n1[i] / a.mean_n1 : 0.f;
        f[11] = a.tau;
    }
}

hipError_t launch_features(const Instance &I, int R, int64_t K, float tau, float mean_n1,
                           float *feat, hipStream_t st) {
    FeatArgs a;
    a.N = I.N; a.R = R; a.ld = I.ld; a.smaj = I.smaj;
    a.sst = I.smaj ? (int64_t)I.N * I.ld : (int64_t)I.Rp * I.ld;
    a.K = (float)K; a.tau = tau; a.mean_n1 = mean_n1;
    a.phi = I.phi32[I.cur]; a.st = I.st; a.n1 = I.n1; a.feat = feat;
    k_features<<<R, 256, 0, st>>>(a);
    return hipGetLastError();
}

// -------------------------------------------------------------------- MLP
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}
__device__ __forceinline__ float rbf(float x, bool on) { return on ? (float)(bf16)x : x; }

__device__ __forceinline__ uint64_t mix64(uint64_t seed, uint64_t ctr) {
    uint64_t z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Weights uniform in [-1/sqrt(fan_in), 1/sqrt(fan_in)] from the counter hash, biases 0.
__global__ void k_mlp_init(float *P, uint64_t seed) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NPARAM) return;
    int fan = 0;
    if (k < OFF_B1) fan = NF;
    else if (k >= OFF_W2 && k < OFF_B2) fan = H1;
    else if (k >= OFF_W3 && k < OFF_B3) fan = H2;
    if (!fan) { P[k] = 0.f; return; }
    double u = (double)(mix64(seed, (uint64_t)k) >> 11) * (1.0 / 9007199254740992.0);
    P[k] = (float)((2.0 * u - 1.0) / sqrt((double)fan));
}

hipError_t launch_mlp_init(float *P, uint64_t seed, hipStream_t st) {
    k_mlp_init<<<(NPARAM + 255) / 256, 256, 0, st>>>(P, seed);
    return hipGetLastError();
}

// Forward of one sample; h1/h2/z1/z2 optional outputs.  bf: BF16 inference
// (weights and layer inputs rounded to bfloat16, binary32 accumulation).
__device__ __forceinline__ void mlp_fwd1(const float *P, const float *x, bool bf, float *z1,
                                         float *h1, float *z2, float *h2, float *prob) {
    float xi[NF];
#pragma unroll
    for (int i = 0; i < NF; i++) xi[i] = rbf(x[i], bf);
    for (int o = 0; o < H1; o++) {
        float s = P[OFF_B1 + o];
#pragma unroll
        for (int i = 0; i < NF; i++) s = fmaf(rbf(P[OFF_W1 + o * NF + i], bf), xi[i], s);
        z1[o] = s;
        h1[o] = rbf(gelu(s), bf);
    }
    for (int o = 0; o < H2; o++) {
        float s = P[OFF_B2 + o];
        for (int i = 0; i < H1; i++) s = fmaf(rbf(P[OFF_W2 + o * H1 + i], bf), h1[i], s);
        z2[o] = s;
        h2[o] = rbf(gelu(s), bf);
    }
    float z3[NC], mx = -INFINITY;
#pragma unroll
    for (int o = 0; o < NC; o++) {
        float s = P[OFF_B3 + o];
        for (int i = 0; i < H2; i++) s = fmaf(rbf(P[OFF_W3 + o * H2 + i], bf), h2[i], s);
        z3[o] = s;
        mx = fmaxf(mx, s);
    }
    float den = 0.f, e[NC];
#pragma unroll
    for (int o = 0; o < NC; o++) { e[o] = expf(z3[o] - mx); den += e[o]; }
#pragma unroll
    for (int o = 0; o < NC; o++) prob[o] = e[o] / den;
}

__global__ __launch_bounds__(256) void k_mlp_predict(const float *P, int64_t B, const float *x,
                                                     float *prob, int bf) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    float z1[H1], h1[H1], z2[H2], h2[H2];
    mlp_fwd1(P, x + s * NF, bf != 0, z1, h1, z2, h2, prob + s * NC);
}

hipError_t launch_mlp_predict(const float *P, int64_t B, const float *x, float *prob, int bf,
                              hipStream_t st) {
    if (B == 0) return hipSuccess;
    k_mlp_predict<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(P, B, x, prob, bf);
    return hipGetLastError();
}

// Gradient of sum_s w_{y_s} * (-log prob_s[y_s]) (unnormalised; acc[0] += sum of the
// weighted losses, acc[1] += sum of the weights).  A workgroup of 64 threads takes
// sub-batches of 64 samples: each thread runs its sample forward and backward and
// leaves its layer vectors in LDS, then the threads accumulate the parameter
// gradients over the sub-batch into an LDS copy, flushed by atomics at the end.
__global__ __launch_bounds__(64) void k_mlp_grad(const float *P, int64_t B, const float *x,
                                                 const int32_t *y, const float *cw, float *grad,
                                                 float *acc) {
    extern __shared__ float sm[];
    float *X = sm;                     // [64][NF]
    float *Hh1 = X + 64 * NF;          // [64][H1]
    float *D1 = Hh1 + 64 * H1;         // [64][H1]
    float *Hh2 = D1 + 64 * H1;         // [64][H2]
    float *D2 = Hh2 + 64 * H2;         // [64][H2]
    float *D3 = D2 + 64 * H2;          // [64][NC]
    float *G = D3 + 64 * NC;           // [NPARAM]
    const int t = threadIdx.x;
    for (int k = t; k < NPARAM; k += 64) G[k] = 0.f;
    float lsum = 0.f, wsum = 0.f;
    for (int64_t s0 = (int64_t)blockIdx.x * 64; s0 < B; s0 += (int64_t)gridDim.x * 64) {
        const int64_t s = s0 + t;
        const bool live = s < B;
        float z1[H1], h1[H1], z2[H2], h2[H2], pr[NC];
        float xs[NF];
#pragma unroll
        for (int i = 0; i < NF; i++) xs[i] = live ? x[s * NF + i] : 0.f;
        mlp_fwd1(P, xs, false, z1, h1, z2, h2, pr);
        const int yy = live ? y[s] : 0;
        const float w = live ? cw[yy] : 0.f;
        if (live) { lsum += -w * logf(pr[yy]); wsum += w; }
        float d3[NC];
#pragma unroll
        for (int o = 0; o < NC; o++) d3[o] = w * (pr[o] - (o == yy ? 1.f : 0.f));
        float d2[H2];
        for (int i = 0; i < H2; i++) {
            float a = 0.f;
#pragma unroll
            for (int o = 0; o < NC; o++) a = fmaf(P[OFF_W3 + o * H2 + i], d3[o], a);
            d2[i] = a * gelu_d(z2[i]);
        }
        for (int i = 0; i < H1; i++) {
            float a = 0.f;
            for (int o = 0; o < H2; o++) a = fmaf(P[OFF_W2 + o * H1 + i], d2[o], a);
            D1[t * H1 + i] = a * gelu_d(z1[i]);
            Hh1[t * H1 + i] = h1[i];
        }
        for (int i = 0; i < H2; i++) { D2[t * H2 + i] = d2[i]; Hh2[t * H2 + i] = h2[i]; }
#pragma unroll
        for (int o = 0; o < NC; o++) D3[t * NC + o] = d3[o];
#pragma unroll
        for (int i = 0; i < NF; i++) X[t * NF + i] = xs[i];
        __syncthreads();
        // parameter gradients of this sub-batch: thread t owns entries k = t, t+64, ...
        for (int k = t; k < NPARAM; k += 64) {
            float g = 0.f;
            if (k < OFF_B1) {
                const int o = k / NF, i = k % NF;
                for (int q = 0; q < 64; q++) g = fmaf(D1[q * H1 + o], X[q * NF + i], g);
            } else if (k < OFF_W2) {
                const int o = k - OFF_B1;
                for (int q = 0; q < 64; q++) g += D1[q * H1 + o];
            } else if (k < OFF_B2) {
                const int o = (k - OFF_W2) / H1, i = (k - OFF_W2) % H1;
                for (int q = 0; q < 64; q++) g = fmaf(D2[q * H2 + o], Hh1[q * H1 + i], g);
            } else if (k < OFF_W3) {
                const int o = k - OFF_B2;
                for (int q = 0; q < 64; q++) g += D2[q * H2 + o];
            } else if (k < OFF_B3) {
                const int o = (k - OFF_W3) / H2, i = (k - OFF_W3) % H2;
                for (int q = 0; q < 64; q++) g = fmaf(D3[q * NC + o], Hh2[q * H2 + i], g);
            } else {
                const int o = k - OFF_B3;
                for (int q = 0; q < 64; q++) g += D3[q * NC + o];
            }
            G[k] += g;
        }
        __syncthreads();
    }
    for (int k = t; k < NPARAM; k += 64) atomicAdd(&grad[k], G[k]);
    for (int off = 32; off > 0; off >>= 1) {
        lsum += __shfl_xor(lsum, off, 64);
        wsum += __shfl_xor(wsum, off, 64);
    }
    if (t == 0) {
        atomicAdd(&acc[0], lsum);
        atomicAdd(&acc[1], wsum);
    }
}

__global__ void k_grad_finalize(float *grad, float *acc) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    float W = acc[1];
    if (k < NPARAM) grad[k] = W > 0.f ? grad[k] / W : 0.f;
    if (k == 0) acc[2] = W > 0.f ? acc[0] / W : 0.f;   // mean weighted loss
}

hipError_t launch_mlp_grad(const float *P, int64_t B, const float *x, const int32_t *y,
                           const float *cw, float *grad, float *acc, hipStream_t st) {
    hipError_t e = hipMemsetAsync(grad, 0, sizeof(float) * NPARAM, st);
    if (e == hipSuccess) e = hipMemsetAsync(acc, 0, sizeof(float) * 4, st);
    if (e != hipSuccess) return e;
    if (B > 0) {
        const size_t lds = sizeof(float) * (64 * NF + 4 * 64 * 64 + 64 * NC + NPARAM);
        int64_t nb = (B + 63) / 64;
        unsigned grid = (unsigned)(nb < 512 ? nb : 512);
        k_mlp_grad<<<grid, 64, lds, st>>>(P, B, x, y, cw, grad, acc);
    }
    k_grad_finalize<<<(NPARAM + 255) / 256, 256, 0, st>>>(grad, acc);
    return hipGetLastError();
}

// Adam (Kingma & Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// P -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void k_adam(float *P, const float *g, float *m, float *v, int64_t t, float lr, float b1,
                       float b2, float eps) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NPARAM) return;
    float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    m[k] = b1 * m[k] + (1.f - b1) * g[k];
    v[k] = b2 * v[k] + (1.f - b2) * g[k] * g[k];
    P[k] -= lr * (m[k] / c1) / (sqrtf(v[k] / c2) + eps);
}

hipError_t launch_adam(float *P, const float *g, float *m, float *v, int64_t t, float lr,
                       hipStream_t st) {
    k_adam<<<(NPARAM + 255) / 256, 256, 0, st>>>(P, g, m, v, t, lr, 0.9f, 0.999f, 1e-8f);
    return hipGetLastError();
}

// ------------------------------------------------- read-out from predictions
// spins: +1 if P(frozen +) >= P(frozen -) else -1; selection key 1 - P(ambivalent)
// as non-negative binary32 (smallest key = most ambivalent).
__global__ void k_probs_to_keys(int64_t n, const float *prob, int8_t *spins, float *key) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float *p = prob + t * NC;
    spins[t] = p[0] >= p[1] ? 1 : -1;
    key[t] = 1.0f - p[2];
}

hipError_t launch_probs_to_keys(int64_t n, const float *prob, int8_t *spins, float *key,
                                hipStream_t st) {
    k_probs_to_keys<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, prob, spins, key);
    return hipGetLastError();
}

}  // namespace hqa
