/*
 * hqa_oracle.c -- slow, plain FP64 CPU oracle for HQA-MD.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg do.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * Method: Irie, Liang, Doi, Gongyo, Hatsuda, "Hybrid Quantum Annealing via
 * Molecular Dynamics" (arXiv:2004.03972).  Every routine names the passage
 * it follows.  All floating point is IEEE binary64, round to nearest even,
 * built with -ffp-contract=off; fma() appears only in the field sum.
 *
 * Layout: every per-replica array is replica-major, x[r*N + i].
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ENONFINITE (-5)

/* An Ising instance (Results, Eq. 1): symmetric J with zero diagonal, field h.
 * Either dense J (row-major N*N) or CSR (row_ptr, col, val; columns ascending). */
typedef struct {
    int32_t N;
    const double *J;       /* dense, or NULL */
    const int32_t *rp;     /* CSR row pointer [N+1], or NULL */
    const int32_t *ci;     /* CSR column indices */
    const double *jv;      /* CSR values */
    const double *h;       /* [N] or NULL (zero field) */
} or_problem;

/* MD run parameters (Methods: scheduling functions, leapfrog). */
typedef struct {
    int32_t M;             /* potential V = phi^M */
    double r_g;            /* delta-tau / g; the paper identifies g with delta-tau, r_g = 1 */
    int64_t T;             /* number of steps, delta-tau = 1/T */
    int32_t W;             /* averaging window in steps, delta = W * delta-tau */
    const double *alpha;   /* [2T+1] schedule on the half-integer grid tau_k = k/(2T) */
    const double *beta;    /* [2T+1] */
} or_md_params;

/* ------------------------------------------------------------------------ */
/* Correctly rounded sum of doubles.                                        */
/* Shewchuk's exact non-overlapping expansion (J. R. Shewchuk, "Adaptive    */
/* Precision Floating-Point Arithmetic and Fast Robust Geometric            */
/* Predicates", 1997): each new term is merged into the partials by         */
/* error-free two-sums; the expansion is then collapsed from the top with   */
/* the round-half-even correction for the case where the discarded tail    */
/* would otherwise be lost.                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *p;
    int64_t n, cap;
} or_xsum;

static void xs_init(or_xsum *a) { a->p = NULL; a->n = 0; a->cap = 0; }
static void xs_free(or_xsum *a) { free(a->p); a->p = NULL; a->n = a->cap = 0; }

static int xs_add(or_xsum *a, double x) {
    int64_t i = 0;
    for (int64_t j = 0; j < a->n; j++) {
        double y = a->p[j];
        if (fabs(x) < fabs(y)) { double t = x; x = y; y = t; }
        double hi = x + y;
        double lo = y - (hi - x);
        if (lo != 0.0) a->p[i++] = lo;
        x = hi;
    }
    if (i >= a->cap) {
        int64_t nc = a->cap ? 2 * a->cap : 32;
        double *np = (double *)realloc(a->p, (size_t)nc * sizeof(double));
        if (!np) return OR_ENOMEM;
        a->p = np; a->cap = nc;
    }
    a->p[i++] = x;
    a->n = i;
    return OR_OK;
}

static double xs_round(const or_xsum *a) {
    int64_t n = a->n;
    if (n == 0) return 0.0;
    double hi = a->p[--n], lo = 0.0;
    while (n > 0) {
        double x = hi, y = a->p[--n];
        hi = x + y;
        double yr = hi - x;
        lo = y - yr;
        if (lo != 0.0) break;
    }
    if (n > 0 && ((lo < 0.0 && a->p[n - 1] < 0.0) || (lo > 0.0 && a->p[n - 1] > 0.0))) {
        double y = lo * 2.0;
        double x = hi + y;
        double yr = x - hi;
        if (y == yr) hi = x;
    }
    return hi;
}

double or_exact_sum(const double *x, int64_t n) {
    or_xsum a; xs_init(&a);
    for (int64_t k = 0; k < n; k++) xs_add(&a, x[k]);
    double s = xs_round(&a);
    xs_free(&a);
    return s;
}

static int is_int53(double v) { return v == floor(v) && fabs(v) < 9007199254740992.0; }

/* ------------------------------------------------------------------------ */
/* Schedule (Methods, "Scheduling functions for MD").                       */
/* alpha(tau) = a_f (tau + rho1 (1-tau) + rho2 tau (tau-1)),                */
/* beta(tau)  = b_f (tau + kap1 (1-tau) + kap2 tau (tau-1)),                */
/* tabulated on tau_k = k/(2T), k = 0..2T, so that integer steps m sit at    */
/* k = 2m and half steps m+1/2 at k = 2m+1 (Methods, leapfrog notation).     */
/* prm = {a_f, rho1, rho2, b_f, kap1, kap2}.  A frozen schedule holds both   */
/* at tau_fix (used only by the conservation and reversibility checks).     */
/* ------------------------------------------------------------------------ */
void or_schedule(const double *prm, int64_t T, int32_t frozen, double tau_fix,
                 double *alpha, double *beta) {
    for (int64_t k = 0; k <= 2 * T; k++) {
        double tau = frozen ? tau_fix : (double)k / (double)(2 * T);
        double om = 1.0 - tau;
        double q = tau * (tau - 1.0);
        alpha[k] = prm[0] * ((tau + prm[1] * om) + prm[2] * q);
        beta[k] = prm[3] * ((tau + prm[4] * om) + prm[5] * q);
    }
}

/* ------------------------------------------------------------------------ */
/* Initial momenta (Results, "Molecular dynamics for flux variables"): each */
/* p_i(0) is +1 or -1 at random.  The coin is the SplitMix64 output         */
/* function (Steele, Lea, Flood, OOPSLA 2014) at counter                    */
/* z = seed + (r*N + i + 1) * 0x9E3779B97F4A7C15; top bit set means -1.      */
/* ------------------------------------------------------------------------ */
uint64_t or_splitmix64_at(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void or_init_p0(uint64_t seed, int32_t N, int32_t R, double *p0) {
    for (int64_t r = 0; r < R; r++)
        for (int64_t i = 0; i < N; i++) {
            uint64_t z = or_splitmix64_at(seed, (uint64_t)(r * N + i));
            p0[r * N + i] = (z >> 63) ? -1.0 : 1.0;
        }
}

/* ------------------------------------------------------------------------ */
/* Local field u_i = sum_j J_ij phi_j (the coupling part of the force in the */
/* leapfrog kick), summed over j in ascending order as a chain of fma.      */
/* ------------------------------------------------------------------------ */
static double field_row(const or_problem *pb, int64_t i, const double *phi) {
    double u = 0.0;
    if (pb->J) {
        const double *Ji = pb->J + i * pb->N;
        for (int64_t j = 0; j < pb->N; j++) u = fma(Ji[j], phi[j], u);
    } else {
        for (int32_t e = pb->rp[i]; e < pb->rp[i + 1]; e++) u = fma(pb->jv[e], phi[pb->ci[e]], u);
    }
    return u;
}

/* phi^(M-1) by repeated multiplication. */
static double pow_m1(double x, int32_t M) {
    double v = x;
    for (int32_t k = 0; k < M - 2; k++) v = v * x;
    return v;
}

/* Force F_i = d H_MD / d phi_i at one step (Eq. 3 and the leapfrog kick):
 * alpha * M phi^(M-1) + beta * (u_i + 2 h_i |phi_i|), times r_g. */
static double force_i(const or_problem *pb, const or_md_params *mp, int64_t i,
                      const double *phi, double a, double b) {
    double x = phi[i];
    double u = field_row(pb, i, phi);
    double hi = pb->h ? pb->h[i] : 0.0;
    double v = pow_m1(x, mp->M);
    double g = u + (2.0 * hi) * fabs(x);
    double F = (a * ((double)mp->M * v)) + (b * g);
    if (mp->r_g != 1.0) F = mp->r_g * F;
    return F;
}

/* Local fields u_i = sum_j J_ij phi_j of R replicas [R][N] (the field term of the */
/* force, Eq. 3), exported for the field parity checks of the binary32 forms.    */
void or_field(const or_problem *pb, int32_t R, const double *phi, double *u) {
    for (int32_t r = 0; r < R; r++)
        for (int64_t i = 0; i < pb->N; i++)
            u[(int64_t)r * pb->N + i] = field_row(pb, i, phi + (int64_t)r * pb->N);
}

/* Force at phi for one replica, exposed for the gradient checks. */
void or_force(const or_problem *pb, const or_md_params *mp, int64_t q,
              const double *phi, double *F) {
    double a = mp->alpha[2 * q], b = mp->beta[2 * q];
    for (int64_t i = 0; i < pb->N; i++) F[i] = force_i(pb, mp, i, phi, a, b);
}

/* ------------------------------------------------------------------------ */
/* Leapfrog (Methods, "Leapfrog algorithm"), one replica.                    */
/* State on entry: phi = phi^(q_from), p = p^(q_from - 1/2) (or p^(0) when    */
/* q_from = 0).  Step q computes F at phi^(q) with alpha_(2q), beta_(2q),     */
/* kicks p by F (by F/2 for the initial half step q = 0), then drifts        */
/* phi^(q+1) = phi^(q) + alpha_(2q+1) p.  Fluxes phi^(q+1) with               */
/* q+1 >= T-W+1 are added to the window sum S (time average, Results,        */
/* "Sorting frozen and ambivalent variables").  Fields are all taken from    */
/* the same phi^(q) (two buffers).                                          */
/* ------------------------------------------------------------------------ */
static int md_replica(const or_problem *pb, const or_md_params *mp, double *phi, double *p,
                      double *S, int64_t q_from, int64_t q_to, double *F) {
    const int64_t N = pb->N;
    for (int64_t q = q_from; q < q_to; q++) {
        double a = mp->alpha[2 * q], b = mp->beta[2 * q];
        for (int64_t i = 0; i < N; i++) F[i] = force_i(pb, mp, i, phi, a, b);
        double ad = mp->alpha[2 * q + 1];
        if (mp->r_g != 1.0) ad = mp->r_g * ad;
        int in_window = (q + 1) >= (mp->T - mp->W + 1);
        for (int64_t i = 0; i < N; i++) {
            if (q == 0) p[i] = p[i] - 0.5 * F[i];
            else p[i] = p[i] - F[i];
            phi[i] = phi[i] + (ad * p[i]);
            if (in_window && S) S[i] = S[i] + phi[i];
        }
    }
    for (int64_t i = 0; i < N; i++)
        if (!isfinite(phi[i]) || !isfinite(p[i])) return OR_ENONFINITE;
    return OR_OK;
}

typedef struct {
    const or_problem *pb;
    const or_md_params *mp;
    double *phi, *p, *S;
    int64_t q_from, q_to;
    int32_t r0, r1;
    int status;
} md_job;

static void *md_worker(void *arg) {
    md_job *jb = (md_job *)arg;
    const int64_t N = jb->pb->N;
    double *F = (double *)malloc((size_t)N * sizeof(double));
    if (!F) { jb->status = OR_ENOMEM; return NULL; }
    jb->status = OR_OK;
    for (int32_t r = jb->r0; r < jb->r1; r++) {
        int st = md_replica(jb->pb, jb->mp, jb->phi + (int64_t)r * N, jb->p + (int64_t)r * N,
                            jb->S ? jb->S + (int64_t)r * N : NULL, jb->q_from, jb->q_to, F);
        if (st != OR_OK) jb->status = st;
    }
    free(F);
    return NULL;
}

/* Advance R independent replicas from q_from to q_to, threads over replicas. */
int or_md_advance(const or_problem *pb, const or_md_params *mp, int32_t R,
                  double *phi, double *p, double *S, int64_t q_from, int64_t q_to,
                  int32_t nthreads) {
    if (q_from < 0 || q_to > mp->T || q_from > q_to || mp->W < 1 || mp->W > mp->T) return OR_EINVAL;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > R) nthreads = R;
    md_job *jobs = (md_job *)calloc((size_t)nthreads, sizeof(md_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return OR_ENOMEM; }
    for (int32_t t = 0; t < nthreads; t++) {
        jobs[t] = (md_job){pb, mp, phi, p, S, q_from, q_to,
                           (int32_t)((int64_t)R * t / nthreads),
                           (int32_t)((int64_t)R * (t + 1) / nthreads), OR_OK};
        if (nthreads == 1) md_worker(&jobs[t]);
        else pthread_create(&th[t], NULL, md_worker, &jobs[t]);
    }
    int st = OR_OK;
    for (int32_t t = 0; t < nthreads; t++) {
        if (nthreads > 1) pthread_join(th[t], NULL);
        if (jobs[t].status != OR_OK) st = jobs[t].status;
    }
    free(jobs); free(th);
    return st;
}

/* Full run: phi^(0), p^(0) in; phibar = S / W, phi^(T), p^(T-1/2) out. */
int or_md_run(const or_problem *pb, const or_md_params *mp, int32_t R,
              const double *phi0, const double *p0, double *phibar, double *phiT,
              double *pT, int32_t nthreads) {
    const int64_t n = (int64_t)R * pb->N;
    double *S = (double *)calloc((size_t)n, sizeof(double));
    if (!S) return OR_ENOMEM;
    memcpy(phiT, phi0, (size_t)n * sizeof(double));
    memcpy(pT, p0, (size_t)n * sizeof(double));
    int st = or_md_advance(pb, mp, R, phiT, pT, S, 0, mp->T, nthreads);
    for (int64_t k = 0; k < n; k++) phibar[k] = S[k] / (double)mp->W;
    free(S);
    return st;
}

/* ------------------------------------------------------------------------ */
/* MD Hamiltonian (Eq. 3) at integer step q, per replica:                    */
/* H = alpha_(2q) sum(p^2/2 + phi^M) + beta_(2q) (1/2 sum phi_i u_i          */
/*     + sum h_i |phi_i| phi_i),                                             */
/* with p given at integer time.  or_integer_p turns the stored half-step   */
/* momentum p^(q-1/2) into p^(q) = p^(q-1/2) - F(phi^(q))/2.                  */
/* ------------------------------------------------------------------------ */
void or_hmd(const or_problem *pb, const or_md_params *mp, int32_t R, int64_t q,
            const double *phi, const double *p_int, double *H) {
    const int64_t N = pb->N;
    double a = mp->alpha[2 * q], b = mp->beta[2 * q];
    for (int32_t r = 0; r < R; r++) {
        const double *x = phi + (int64_t)r * N, *pp = p_int + (int64_t)r * N;
        double kin = 0.0, cpl = 0.0, fld = 0.0;
        for (int64_t i = 0; i < N; i++) {
            double xm = pow_m1(x[i], mp->M) * x[i];
            kin = kin + ((pp[i] * pp[i]) * 0.5 + xm);
            cpl = cpl + x[i] * field_row(pb, i, x);
            if (pb->h) fld = fld + (pb->h[i] * fabs(x[i])) * x[i];
        }
        H[r] = a * kin + b * (0.5 * cpl + fld);
    }
}

void or_integer_p(const or_problem *pb, const or_md_params *mp, int32_t R, int64_t q,
                  const double *phi, const double *p_half, double *p_int) {
    const int64_t N = pb->N;
    double a = mp->alpha[2 * q], b = mp->beta[2 * q];
    for (int32_t r = 0; r < R; r++)
        for (int64_t i = 0; i < N; i++)
            p_int[(int64_t)r * N + i] = p_half[(int64_t)r * N + i] -
                0.5 * force_i(pb, mp, i, phi + (int64_t)r * N, a, b);
}

/* ------------------------------------------------------------------------ */
/* Sort into ambivalent and frozen (Results, "Sorting ..."; HQA section):   */
/* order spins by (|phibar_i|, i) ascending; the first n are ambivalent,     */
/* listed back in ascending spin index.  Every spin gets s = sgn(phibar)     */
/* with sgn(0) = +1 (frozen projection; the MD-alone read-out).             */
/* ------------------------------------------------------------------------ */
typedef struct { double key; int32_t idx; } kv;

static int kv_cmp(const void *a, const void *b) {
    const kv *x = (const kv *)a, *y = (const kv *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static int i32_cmp(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int or_classify(int32_t N, int32_t R, const double *phibar, int32_t n,
                int32_t *amb_idx, int8_t *spins) {
    if (n < 0 || n > N) return OR_EINVAL;
    kv *buf = (kv *)malloc((size_t)N * sizeof(kv));
    if (!buf) return OR_ENOMEM;
    for (int32_t r = 0; r < R; r++) {
        const double *pb = phibar + (int64_t)r * N;
        for (int32_t i = 0; i < N; i++) {
            buf[i].key = fabs(pb[i]);
            buf[i].idx = i;
            spins[(int64_t)r * N + i] = pb[i] > 0.0 ? 1 : (pb[i] < 0.0 ? -1 : 1);
        }
        qsort(buf, (size_t)N, sizeof(kv), kv_cmp);
        int32_t *A = amb_idx + (int64_t)r * n;
        for (int32_t a = 0; a < n; a++) A[a] = buf[a].idx;
        qsort(A, (size_t)n, sizeof(int32_t), i32_cmp);
    }
    free(buf);
    return OR_OK;
}

/* J_ij lookup for dense or CSR storage. */
static double jget(const or_problem *pb, int32_t i, int32_t j) {
    if (pb->J) return pb->J[(int64_t)i * pb->N + j];
    int32_t lo = pb->rp[i], hi = pb->rp[i + 1];
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (pb->ci[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < pb->rp[i + 1] && pb->ci[lo] == j) ? pb->jv[lo] : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Reduced subproblem (HQA section, effective couplings):                    */
/* J_eff = J[A,A], h_eff_a = h_a + sum_{k not in A} J_ak s_k, each h_eff the  */
/* correctly rounded exact sum of its terms.                                 */
/* ------------------------------------------------------------------------ */
int or_reduce(const or_problem *pb, int32_t R, int32_t n, const int32_t *amb_idx,
              const int8_t *spins, double *h_eff, double *J_eff) {
    const int32_t N = pb->N;
    uint8_t *inA = (uint8_t *)calloc((size_t)N, 1);
    if (!inA) return OR_ENOMEM;
    for (int32_t r = 0; r < R; r++) {
        const int32_t *A = amb_idx + (int64_t)r * n;
        const int8_t *s = spins + (int64_t)r * N;
        memset(inA, 0, (size_t)N);
        for (int32_t a = 0; a < n; a++) inA[A[a]] = 1;
        for (int32_t a = 0; a < n; a++) {
            or_xsum acc; xs_init(&acc);
            xs_add(&acc, pb->h ? pb->h[A[a]] : 0.0);
            if (pb->J) {
                for (int32_t k = 0; k < N; k++)
                    if (!inA[k]) xs_add(&acc, pb->J[(int64_t)A[a] * N + k] * (double)s[k]);
            } else {
                for (int32_t e = pb->rp[A[a]]; e < pb->rp[A[a] + 1]; e++)
                    if (!inA[pb->ci[e]]) xs_add(&acc, pb->jv[e] * (double)s[pb->ci[e]]);
            }
            h_eff[(int64_t)r * n + a] = xs_round(&acc);
            xs_free(&acc);
            for (int32_t b = 0; b < n; b++)
                J_eff[((int64_t)r * n + a) * n + b] = jget(pb, A[a], A[b]);
        }
    }
    free(inA);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact solution of the reduced problem by enumeration: every code c in    */
/* 0..2^n-1, x_a = -1 when bit a of c is set, else +1; E'(c) is the          */
/* correctly rounded exact sum of {J_ab x_a x_b : a<b} and {h_a x_a}; the    */
/* minimum wins, ties to the smallest code.  Each code is scored from        */
/* scratch (no incremental update).                                          */
/* ------------------------------------------------------------------------ */
/* The scan over codes c0 <= c < c1 of one reduced problem (first code with the   */
/* smallest E' in that range).  The minimum over all codes with ties to the        */
/* smallest code is unique, so a caller may split 0..2^n-1 into ascending blocks   */
/* and keep the first block whose minimum is strictly smallest.                    */
static void enum_range(int32_t n, const double *Je, const double *he, int64_t c0, int64_t c1,
                       int64_t *best_code, double *best_E) {
    {
        int integral = 1;
        for (int32_t a = 0; a < n && integral; a++) {
            if (!is_int53(he[a])) integral = 0;
            for (int32_t b = 0; b < n; b++)
                if (!is_int53(Je[a * n + b])) integral = 0;
        }
        int64_t bc = c0;
        double bE = INFINITY;
        int64_t bEi = INT64_MAX;
        for (int64_t c = c0; c < c1; c++) {
            if (integral) {
                int64_t E = 0;
                for (int32_t a = 0; a < n; a++) {
                    int64_t xa = ((c >> a) & 1) ? -1 : 1;
                    for (int32_t b = a + 1; b < n; b++) {
                        int64_t xb = ((c >> b) & 1) ? -1 : 1;
                        E += (int64_t)Je[a * n + b] * xa * xb;
                    }
                    E += (int64_t)he[a] * xa;
                }
                if (E < bEi) { bEi = E; bc = c; }
            } else {
                or_xsum acc; xs_init(&acc);
                for (int32_t a = 0; a < n; a++) {
                    double xa = ((c >> a) & 1) ? -1.0 : 1.0;
                    for (int32_t b = a + 1; b < n; b++) {
                        double xb = ((c >> b) & 1) ? -1.0 : 1.0;
                        xs_add(&acc, Je[a * n + b] * (xa * xb));
                    }
                    xs_add(&acc, he[a] * xa);
                }
                double E = xs_round(&acc);
                xs_free(&acc);
                if (E < bE) { bE = E; bc = c; }
            }
        }
        *best_code = bc;
        *best_E = integral ? (double)bEi : bE;
    }
}

int or_enumerate(int32_t n, int32_t R, const double *J_eff, const double *h_eff,
                 int64_t *best_code, double *best_E) {
    if (n < 0 || n > 30) return OR_EINVAL;
    for (int32_t r = 0; r < R; r++)
        enum_range(n, J_eff + (int64_t)r * n * n, h_eff + (int64_t)r * n, 0, (int64_t)1 << n,
                   &best_code[r], &best_E[r]);
    return OR_OK;
}

/* One block of codes [c0, c1) of one reduced problem (see enum_range). */
int or_enumerate_range(int32_t n, const double *J_eff, const double *h_eff, int64_t c0,
                       int64_t c1, int64_t *best_code, double *best_E) {
    if (n < 0 || n > 30 || c0 < 0 || c1 > ((int64_t)1 << n) || c0 >= c1) return OR_EINVAL;
    enum_range(n, J_eff, h_eff, c0, c1, best_code, best_E);
    return OR_OK;
}

/* Merge: frozen spins keep sgn(phibar); ambivalent spin A[a] takes x_a of the code. */
/* Tabu search on the reduced problem of every replica.  The paper sends the n
 * ambivalent spins, with the frozen ones fixed, to a quantum annealer or, for
 * n = 1000, to a tabu search (Results, the K2000 MAX-CUT experiment: HQA(TS1000)).
 * That tabu search is an external solver the paper does not specify; this is a
 * plain single-flip tabu search (this library's reading), in binary64:
 *   x = x0 (the MD read-out of the n spins); f_a = h_a + sum_{b != a} J_ab x_b with
 *   b ascending, one rounding per addition; D = 0 (energy change from x0),
 *   D_best = 0, x_best = x0; then for t = 1 .. iters:
 *     d_a = -2 x_a f_a (exact) for every a;
 *     move a is allowed when tabu_until[a] < t, or when D + d_a < D_best (aspiration);
 *     a* = the allowed a with the smallest d_a, ties to the smallest a;
 *     D = D + d_a*;  f_b = f_b - 2 J_a*b x_a* (x_a* before the flip) for b != a*;
 *     x_a* = -x_a*;  tabu_until[a*] = t + tenure;
 *     if D < D_best: D_best = D, x_best = x.
 * tenure is clamped to n - 1, so at least one move is always allowed.  Outputs the
 * best configuration and D_best = E'(x_best) - E'(x0) as accumulated (exact when J
 * and h are integers).  J_eff is [R][n][n] with a zero diagonal, h_eff [R][n], x0 and
 * x_best [R][n] of +-1. */
int or_tabu(int32_t n, int32_t R, const double *J_eff, const double *h_eff, const int8_t *x0,
            int64_t iters, int32_t tenure, int8_t *x_best, double *d_best) {
    if (n < 0 || R < 0 || iters < 0 || tenure < 0) return OR_EINVAL;
    if (n == 0) {
        for (int32_t r = 0; r < R; r++) d_best[r] = 0.0;
        return OR_OK;
    }
    if (tenure > n - 1) tenure = n - 1;
    double *f = malloc(sizeof(double) * (size_t)n);
    int8_t *x = malloc((size_t)n);
    int64_t *until = malloc(sizeof(int64_t) * (size_t)n);
    if (!f || !x || !until) { free(f); free(x); free(until); return OR_ENOMEM; }
    for (int32_t r = 0; r < R; r++) {
        const double *J = J_eff + (int64_t)r * n * n, *h = h_eff + (int64_t)r * n;
        int8_t *xb = x_best + (int64_t)r * n;
        memcpy(x, x0 + (int64_t)r * n, (size_t)n);
        memcpy(xb, x, (size_t)n);
        for (int32_t a = 0; a < n; a++) {
            double acc = h[a];
            for (int32_t b = 0; b < n; b++)
                if (b != a) acc = acc + J[(int64_t)a * n + b] * (double)x[b];
            f[a] = acc;
            until[a] = 0;
        }
        double D = 0.0, Db = 0.0;
        for (int64_t t = 1; t <= iters; t++) {
            int32_t best = -1;
            double bd = 0.0;
            for (int32_t a = 0; a < n; a++) {
                const double d = x[a] > 0 ? -2.0 * f[a] : 2.0 * f[a];
                const int allowed = until[a] < t || D + d < Db;
                if (allowed && (best < 0 || d < bd)) { best = a; bd = d; }
            }
            D = D + bd;
            const int8_t xo = x[best];
            const double *Jr = J + (int64_t)best * n;
            for (int32_t b = 0; b < n; b++)
                if (b != best) f[b] = f[b] - (xo > 0 ? 2.0 * Jr[b] : -2.0 * Jr[b]);
            x[best] = (int8_t)-xo;
            until[best] = t + tenure;
            if (D < Db) {
                Db = D;
                memcpy(xb, x, (size_t)n);
            }
        }
        d_best[r] = Db;
    }
    free(f); free(x); free(until);
    return OR_OK;
}

void or_merge(int32_t N, int32_t R, int32_t n, const int32_t *amb_idx, const int64_t *code,
              int8_t *spins) {
    for (int32_t r = 0; r < R; r++)
        for (int32_t a = 0; a < n; a++)
            spins[(int64_t)r * N + amb_idx[(int64_t)r * n + a]] = ((code[r] >> a) & 1) ? -1 : 1;
}

/* ------------------------------------------------------------------------ */
/* Ising energy (Eq. 1) H(s) = sum_{i<j} J_ij s_i s_j + sum_i h_i s_i, as a   */
/* correctly rounded exact sum, and the cut (Methods, MAX-CUT) with w = J:   */
/* C(s) = sum over i<j with s_i != s_j of J_ij, also exact.                  */
/* ------------------------------------------------------------------------ */
int or_energy(const or_problem *pb, int32_t V, const int8_t *spins, double *E, double *cut) {
    const int32_t N = pb->N;
    for (int32_t v = 0; v < V; v++) {
        const int8_t *s = spins + (int64_t)v * N;
        or_xsum ae, ac; xs_init(&ae); xs_init(&ac);
        for (int32_t i = 0; i < N; i++) {
            if (pb->J) {
                for (int32_t j = i + 1; j < N; j++) {
                    double Jij = pb->J[(int64_t)i * N + j];
                    if (Jij == 0.0) continue;
                    xs_add(&ae, Jij * (double)(s[i] * s[j]));
                    if (s[i] != s[j]) xs_add(&ac, Jij);
                }
            } else {
                for (int32_t e = pb->rp[i]; e < pb->rp[i + 1]; e++) {
                    int32_t j = pb->ci[e];
                    if (j <= i) continue;
                    xs_add(&ae, pb->jv[e] * (double)(s[i] * s[j]));
                    if (s[i] != s[j]) xs_add(&ac, pb->jv[e]);
                }
            }
            if (pb->h) xs_add(&ae, pb->h[i] * (double)s[i]);
        }
        E[v] = xs_round(&ae);
        if (cut) cut[v] = xs_round(&ac);
        xs_free(&ae); xs_free(&ac);
    }
    return OR_OK;
}
