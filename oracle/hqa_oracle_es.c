/*
 * hqa_oracle_es.c -- FP64 oracle of the learned early stop (TEST INFRASTRUCTURE
 * ONLY: used by the tests and the benchmark's CPU baseline, never by the product).
 *
 * The paper gives no learned component; this is the library's own design, kept
 * here in plain form so the GPU kernels can be checked:
 *  - per (spin, replica) statistics over a window of MD steps [K0, K1), taken
 *    from the leapfrog of the paper (Methods): old flux x = phi^(q), new flux
 *    x' = phi^(q+1), local field u = sum_j J_ij phi^(q)_j, momentum p^(q+1/2);
 *  - twelve features per spin at the checkpoint q = K1, normalised per replica;
 *  - a 12-64-64-3 perceptron with GELU (x (1 + erf(x / sqrt 2)) / 2), softmax
 *    output over {frozen +, frozen -, ambivalent}, class-weighted cross entropy,
 *    its analytic gradient, and one Adam step (Kingma & Ba 2015).
 * Parameter vector (5187 values): W1[64][12], b1[64], W2[64][64], b2[64],
 * W3[3][64], b3[3], each weight matrix row-major [out][in].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t N;
    const double *J;
    const int32_t *rp;
    const int32_t *ci;
    const double *jv;
    const double *h;
} or_problem;

typedef struct {
    int32_t M;
    double r_g;
    int64_t T;
    int32_t W;
    const double *alpha;
    const double *beta;
} or_md_params;

enum { NF = 12, H1 = 64, H2 = 64, NC = 3 };
enum { OFF_W1 = 0, OFF_B1 = OFF_W1 + H1 * NF, OFF_W2 = OFF_B1 + H1, OFF_B2 = OFF_W2 + H2 * H1,
       OFF_W3 = OFF_B2 + H2, OFF_B3 = OFF_W3 + NC * H2, NPARAM = OFF_B3 + NC };

static double row_field(const or_problem *pb, int64_t i, const double *x) {
    double u = 0.0;
    if (pb->J) {
        for (int64_t j = 0; j < pb->N; j++) u = fma(pb->J[i * pb->N + j], x[j], u);
    } else {
        for (int32_t e = pb->rp[i]; e < pb->rp[i + 1]; e++) u = fma(pb->jv[e], x[pb->ci[e]], u);
    }
    return u;
}

static void row_norms(const or_problem *pb, double *n1, double *n2) {
    for (int64_t i = 0; i < pb->N; i++) {
        double a = 0.0, b = 0.0;
        if (pb->J) {
            for (int64_t j = 0; j < pb->N; j++) {
                double v = pb->J[i * pb->N + j];
                a += fabs(v);
                b += v * v;
            }
        } else {
            for (int32_t e = pb->rp[i]; e < pb->rp[i + 1]; e++) {
                a += fabs(pb->jv[e]);
                b += pb->jv[e] * pb->jv[e];
            }
        }
        n1[i] = a;
        n2[i] = sqrt(b);
    }
}

/* Run R replicas from (phi0, p0) to step K1 with the leapfrog of Methods, collect
 * the statistics over [K0, K1) and write the features [R][N][12] at q = K1.
 * phi_out / p_out receive phi^(K1), p^(K1-1/2). */
int or_es_features(const or_problem *pb, const or_md_params *mp, int32_t R, const double *phi0,
                   const double *p0, int64_t K0, int64_t K1, int64_t every, double *feat,
                   double *phi_out, double *p_out) {
    const int64_t N = pb->N;
    if (K0 < 0 || K1 <= K0 || K1 > mp->T || every < 1) return -1;
    double *x = malloc(sizeof(double) * N), *xn = malloc(sizeof(double) * N);
    double *p = malloc(sizeof(double) * N), *u = malloc(sizeof(double) * N);
    double *A = calloc((size_t)9 * N, sizeof(double));
    double *n1 = malloc(sizeof(double) * N), *n2 = malloc(sizeof(double) * N);
    if (!x || !xn || !p || !u || !A || !n1 || !n2) return -2;
    row_norms(pb, n1, n2);
    double mean_n1 = 0.0;
    for (int64_t i = 0; i < N; i++) mean_n1 += n1[i];
    mean_n1 /= (double)N;
    for (int32_t r = 0; r < R; r++) {
        memcpy(x, phi0 + (int64_t)r * N, sizeof(double) * N);
        memcpy(p, p0 + (int64_t)r * N, sizeof(double) * N);
        memset(A, 0, sizeof(double) * 9 * N);
        for (int64_t q = 0; q < K1; q++) {
            double a = mp->alpha[2 * q], b = mp->beta[2 * q];
            double ad = mp->alpha[2 * q + 1];
            if (mp->r_g != 1.0) ad = mp->r_g * ad;
            for (int64_t i = 0; i < N; i++) {
                double xi = x[i];
                u[i] = row_field(pb, i, x);
                double v = xi;
                for (int32_t k = 0; k < mp->M - 2; k++) v = v * xi;
                double hi = pb->h ? pb->h[i] : 0.0;
                double g = u[i] + (2.0 * hi) * fabs(xi);
                double F = (a * ((double)mp->M * v)) + (b * g);
                if (mp->r_g != 1.0) F = mp->r_g * F;
                p[i] = q == 0 ? p[i] - 0.5 * F : p[i] - F;
                xn[i] = xi + (ad * p[i]);
            }
            if (q >= K0 && (q - K0) % every == 0) {   /* every-th step of the window */
                for (int64_t i = 0; i < N; i++) {
                    double nu = n2[i] > 0.0 ? u[i] / n2[i] : 0.0;
                    double so = x[i] < 0.0 ? -1.0 : 1.0;
                    A[0 * N + i] += xn[i];
                    A[1 * N + i] += xn[i] * xn[i];
                    A[2 * N + i] += fabs(xn[i]);
                    A[3 * N + i] += xn[i] > 0.0 ? 1.0 : 0.0;
                    A[4 * N + i] += ((xn[i] < 0.0) != (x[i] < 0.0)) ? 1.0 : 0.0;
                    A[5 * N + i] += nu;
                    A[6 * N + i] += nu * nu;
                    A[7 * N + i] += -so * nu;
                    A[8 * N + i] += p[i] * p[i];
                }
            }
            memcpy(x, xn, sizeof(double) * N);
        }
        const double K = (double)((K1 - K0 + every - 1) / every);   /* sampled steps */
        double s2 = 0.0, pm = 0.0;
        for (int64_t i = 0; i < N; i++) {
            s2 += x[i] * x[i];
            pm += A[8 * N + i] / K;
        }
        double sig = sqrt(s2 / (double)N);
        if (sig == 0.0) sig = 1.0;
        pm /= (double)N;
        if (pm == 0.0) pm = 1.0;
        for (int64_t i = 0; i < N; i++) {
            double *f = feat + ((int64_t)r * N + i) * NF;
            double m0 = A[0 * N + i] / K, m5 = A[5 * N + i] / K;
            f[0] = m0 / sig;
            f[1] = sqrt(fmax(A[1 * N + i] / K - m0 * m0, 0.0)) / sig;
            f[2] = (A[2 * N + i] / K) / sig;
            f[3] = x[i] / sig;
            f[4] = fabs(2.0 * A[3 * N + i] / K - 1.0);
            f[5] = A[4 * N + i] / K;
            f[6] = m5 / sig;
            f[7] = sqrt(fmax(A[6 * N + i] / K - m5 * m5, 0.0)) / sig;
            f[8] = (A[7 * N + i] / K) / sig;
            f[9] = (A[8 * N + i] / K) / pm;
            f[10] = mean_n1 > 0.0 ? n1[i] / mean_n1 : 0.0;
            f[11] = (double)K1 / (double)mp->T;
        }
        if (phi_out) memcpy(phi_out + (int64_t)r * N, x, sizeof(double) * N);
        if (p_out) memcpy(p_out + (int64_t)r * N, p, sizeof(double) * N);
    }
    free(x); free(xn); free(p); free(u); free(A); free(n1); free(n2);
    return 0;
}

double or_gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }

static double gelu_d(double z) {
    const double two_pi = 6.283185307179586;
    return 0.5 * (1.0 + erf(z / sqrt(2.0))) + z * exp(-0.5 * z * z) / sqrt(two_pi);
}

/* Forward pass of one sample: z1, h1, z2, h2, logits and softmax probabilities. */
static void fwd1(const double *P, const double *x, double *z1, double *h1, double *z2,
                 double *h2, double *z3, double *prob) {
    for (int o = 0; o < H1; o++) {
        double s = P[OFF_B1 + o];
        for (int i = 0; i < NF; i++) s += P[OFF_W1 + o * NF + i] * x[i];
        z1[o] = s;
        h1[o] = or_gelu(s);
    }
    for (int o = 0; o < H2; o++) {
        double s = P[OFF_B2 + o];
        for (int i = 0; i < H1; i++) s += P[OFF_W2 + o * H1 + i] * h1[i];
        z2[o] = s;
        h2[o] = or_gelu(s);
    }
    double mx = -INFINITY;
    for (int o = 0; o < NC; o++) {
        double s = P[OFF_B3 + o];
        for (int i = 0; i < H2; i++) s += P[OFF_W3 + o * H2 + i] * h2[i];
        z3[o] = s;
        if (s > mx) mx = s;
    }
    double den = 0.0;
    for (int o = 0; o < NC; o++) den += exp(z3[o] - mx);
    for (int o = 0; o < NC; o++) prob[o] = exp(z3[o] - mx) / den;
}

void or_mlp_forward(const double *P, int64_t B, const double *x, double *prob) {
    double z1[H1], h1[H1], z2[H2], h2[H2], z3[NC];
    for (int64_t s = 0; s < B; s++) fwd1(P, x + s * NF, z1, h1, z2, h2, z3, prob + s * NC);
}

/* Weighted cross entropy L = -sum_s w_{y_s} log prob_s[y_s] / sum_s w_{y_s} and its
 * gradient with respect to every parameter (grad[NPARAM], overwritten). */
double or_mlp_loss_grad(const double *P, int64_t B, const double *x, const int32_t *y,
                        const double *cw, double *grad) {
    double z1[H1], h1[H1], z2[H2], h2[H2], z3[NC], pr[NC];
    double d3[NC], dh2[H2], d2[H2], dh1[H1], d1[H1];
    memset(grad, 0, sizeof(double) * NPARAM);
    double wsum = 0.0, loss = 0.0;
    for (int64_t s = 0; s < B; s++) wsum += cw[y[s]];
    for (int64_t s = 0; s < B; s++) {
        const double *xs = x + s * NF;
        fwd1(P, xs, z1, h1, z2, h2, z3, pr);
        double w = cw[y[s]] / wsum;
        loss -= w * log(pr[y[s]]);
        for (int o = 0; o < NC; o++) d3[o] = w * (pr[o] - (o == y[s] ? 1.0 : 0.0));
        for (int i = 0; i < H2; i++) {
            double a = 0.0;
            for (int o = 0; o < NC; o++) a += P[OFF_W3 + o * H2 + i] * d3[o];
            dh2[i] = a;
            d2[i] = a * gelu_d(z2[i]);
        }
        for (int i = 0; i < H1; i++) {
            double a = 0.0;
            for (int o = 0; o < H2; o++) a += P[OFF_W2 + o * H1 + i] * d2[o];
            dh1[i] = a;
            d1[i] = a * gelu_d(z1[i]);
        }
        for (int o = 0; o < NC; o++) {
            grad[OFF_B3 + o] += d3[o];
            for (int i = 0; i < H2; i++) grad[OFF_W3 + o * H2 + i] += d3[o] * h2[i];
        }
        for (int o = 0; o < H2; o++) {
            grad[OFF_B2 + o] += d2[o];
            for (int i = 0; i < H1; i++) grad[OFF_W2 + o * H1 + i] += d2[o] * h1[i];
        }
        for (int o = 0; o < H1; o++) {
            grad[OFF_B1 + o] += d1[o];
            for (int i = 0; i < NF; i++) grad[OFF_W1 + o * NF + i] += d1[o] * xs[i];
        }
    }
    return loss;
}

/* One Adam step (Kingma & Ba 2015, Algorithm 1) at step count t >= 1:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, P -= lr mhat / (sqrt(vhat) + eps). */
void or_adam_step(double *P, const double *g, double *m, double *v, int64_t n, int64_t t,
                  double lr, double b1, double b2, double eps) {
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t k = 0; k < n; k++) {
        m[k] = b1 * m[k] + (1.0 - b1) * g[k];
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
        P[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
    }
}
