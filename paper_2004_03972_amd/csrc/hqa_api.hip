#include <atomic>
#include <mutex>
// hqa_api.hip -- the C ABI of include/hqa.h: argument checks, device buffers,
// dispatch of the MD step kernels and of the read-out chain.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "hqa_internal.h"

using namespace hqa;

namespace hqa {
hipError_t launch_md_steps_f64(hqa_md *md, Instance &I, int64_t q0, int64_t q1);
hipError_t launch_md_steps_dense(hqa_md *md, Instance &I, int64_t q0, int64_t q1);
hipError_t launch_md_steps_csr(hqa_md *md, Instance &I, int64_t q0, int64_t q1);
hipError_t launch_md_persist(hqa_md *md, Instance &I, int64_t q0, int64_t q1);
hipError_t launch_md_persist_set(hqa_md *md, Instance *const *set, int K, int64_t q0,
                                 int64_t q1);
hipError_t launch_md_steps_batch(hqa_md *md, int64_t q0, int64_t q1, bool graph = false);
void free_batch_plan(void *p);
hipError_t launch_field_f64(hqa_md *md, Instance &I, double *u, hipStream_t st);
hipError_t launch_field_dense(hqa_md *md, Instance &I, float *u, hipStream_t st);
hipError_t launch_field_csr(hqa_md *md, Instance &I, float *u, hipStream_t st);
hipError_t launch_layout_to_f64(int N, int R, int ld, int smaj, const float *src, double *dst,
                                hipStream_t st);
}  // namespace hqa

static thread_local std::string g_err;

static hqa_status fail(hqa_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(e_ == hipErrorOutOfMemory ? HQA_ENOMEM : HQA_EDEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                 \
    } while (0)

namespace hqa {
static std::atomic<int64_t> g_alloc_count{0}, g_alloc_fail{0};

void fault_alloc_arm() {
    const char *v = getenv("HQA_FAULT_ALLOC");
    g_alloc_fail = v ? atoll(v) : 0;
    g_alloc_count = 0;
}

hipError_t dev_malloc(void **p, size_t bytes) {
    *p = nullptr;
    const int64_t k = ++g_alloc_count;
    const int64_t f = g_alloc_fail.load();
    if (f > 0 && k == f) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
}
}  // namespace hqa

// The status of a failed HIP call: an allocation that failed is HQA_ENOMEM.
static hqa_status dev_status(hipError_t e) {
    return e == hipErrorOutOfMemory ? HQA_ENOMEM : HQA_EDEVICE;
}

template <typename T>
static hipError_t dalloc(T **p, size_t count) {
    if (count == 0) count = 1;
    return dev_malloc((void **)p, count * sizeof(T));
}

// HQA_TIMING=1 (any value but 0): hqa_md_run and the read-outs time their device work
// with HIP events on their stream, synchronise, and print one line to stderr.
static bool timing_on() {
    const char *v = getenv("HQA_TIMING");
    return v && *v && strcmp(v, "0") != 0;
}

struct CallTimer {
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool on = false;
    explicit CallTimer(hipStream_t s) : st(s), on(timing_on()) {
        if (on && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
                   hipEventRecord(e0, st) != hipSuccess))
            on = false;
    }
    // milliseconds since construction, or -1 when timing is off or failed
    double stop() {
        float ms = -1.0f;
        if (on && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess)
            (void)hipEventElapsedTime(&ms, e0, e1);
        on = false;
        return ms;
    }
    ~CallTimer() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

static void dfree(void *p) {
    if (p) (void)hipFree(p);
}

static void free_instance(Instance &I) {
    dfree(I.J64); dfree(I.rp); dfree(I.ci); dfree(I.h64); dfree(I.h32); dfree(I.Js); dfree(I.v32);
    for (int k = 0; k < 2; k++) { dfree(I.phi64[k]); dfree(I.phi32[k]); dfree(I.phib[k]); }
    dfree(I.p64); dfree(I.S64); dfree(I.p32); dfree(I.S32); dfree(I.xch); dfree(I.Jt);
    dfree(I.Jbits);
    dfree(I.st); dfree(I.n1); dfree(I.inv_n2);
    I = Instance();
}

static hipMemcpyKind kind_in(int mem) { return mem == HQA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
static hipMemcpyKind kind_out(int mem) { return mem == HQA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

static std::string err_text(int e) {
    std::string s;
    if (e & ERR_ASYM) s += " J is not symmetric;";
    if (e & ERR_DIAG) s += " J has a nonzero diagonal entry;";
    if (e & ERR_NOTFINITE_IN) s += " J or h holds a non-finite value;";
    if (e & ERR_CSR_ORDER) s += " CSR columns not strictly ascending or out of range;";
    if (e & ERR_INEXACT) s += " J does not convert exactly to the storage type;";
    if (e & ERR_NONFINITE) s += " a flux or momentum became non-finite;";
    if (e & ERR_BARRIER) s += " a persistent-kernel barrier wait exceeded its bound;";
    if (e & ERR_PLACEMENT) s += " a persistent-kernel workgroup ran outside its cluster's XCD;";
    return s;
}

// Host-side checks of a problem descriptor that need no device work.
static hqa_status check_problem(const hqa_problem &P, int k) {
    if (P.n < 1) return fail(HQA_EINVAL, "instance %d: n must be >= 1", k);
    if (P.layout != HQA_DENSE && P.layout != HQA_CSR)
        return fail(HQA_EINVAL, "instance %d: unknown layout", k);
    if (P.mem != HQA_HOST && P.mem != HQA_DEVICE) return fail(HQA_EINVAL, "instance %d: bad mem", k);
    if (!P.j) return fail(HQA_EINVAL, "instance %d: j is NULL", k);
    if (P.layout == HQA_CSR) {
        if (!P.row_ptr || !P.col) return fail(HQA_EINVAL, "instance %d: CSR arrays missing", k);
        if (P.nnz < 0) return fail(HQA_EINVAL, "instance %d: nnz < 0", k);
    }
    return HQA_OK;
}

// Upload binary64 couplings and field, validate on the device, gather exponent
// statistics.  Leaves I.J64 / rp / ci / h64 filled.
static hqa_status ingest(const hqa_problem &P, int k, hipStream_t st, int32_t *derr,
                         int32_t *dstats, Instance &I) {
    I.N = P.n;
    I.layout = P.layout;
    I.has_h = P.h != nullptr;
    const int N = P.n;
    if (P.layout == HQA_DENSE) {
        I.nnz = (int64_t)N * N;
        HIPCHK(dalloc(&I.J64, (size_t)N * N));
        HIPCHK(hipMemcpyAsync(I.J64, P.j, sizeof(double) * N * N, kind_in(P.mem), st));
    } else {
        // the row pointer is needed on the host to size the arrays
        std::vector<int32_t> rp(N + 1);
        HIPCHK(hipMemcpyAsync(rp.data(), P.row_ptr, sizeof(int32_t) * (N + 1),
                              P.mem == HQA_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (rp[0] != 0 || rp[N] != P.nnz)
            return fail(HQA_EINVAL, "instance %d: row_ptr[0] must be 0 and row_ptr[n] = nnz", k);
        int max_deg = 0;
        for (int i = 0; i < N; i++) {
            if (rp[i + 1] < rp[i]) return fail(HQA_EINVAL, "instance %d: row_ptr decreases", k);
            max_deg = std::max(max_deg, rp[i + 1] - rp[i]);
        }
        I.max_deg = max_deg;
        I.nnz = P.nnz;
        HIPCHK(dalloc(&I.J64, (size_t)P.nnz));
        HIPCHK(dalloc(&I.rp, (size_t)N + 1));
        HIPCHK(dalloc(&I.ci, (size_t)P.nnz));
        HIPCHK(hipMemcpyAsync(I.rp, rp.data(), sizeof(int32_t) * (N + 1), hipMemcpyHostToDevice, st));
        if (P.nnz) {
            HIPCHK(hipMemcpyAsync(I.ci, P.col, sizeof(int32_t) * P.nnz, kind_in(P.mem), st));
            HIPCHK(hipMemcpyAsync(I.J64, P.j, sizeof(double) * P.nnz, kind_in(P.mem), st));
        }
    }
    HIPCHK(dalloc(&I.h64, (size_t)N));
    if (P.h) HIPCHK(hipMemcpyAsync(I.h64, P.h, sizeof(double) * N, kind_in(P.mem), st));
    else HIPCHK(hipMemsetAsync(I.h64, 0, sizeof(double) * N, st));
    int32_t init[4] = {1 << 20, -(1 << 20), 1, 0};
    HIPCHK(hipMemcpyAsync(dstats, init, sizeof init, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(derr, 0, sizeof(int32_t), st));
    if (P.layout == HQA_DENSE) HIPCHK(launch_validate_dense(I.J64, I.h64, N, derr, dstats, st));
    else HIPCHK(launch_validate_csr(I.rp, I.ci, I.J64, I.h64, N, derr, dstats, st));
    int32_t stats[4], e = 0;
    HIPCHK(hipMemcpyAsync(stats, dstats, sizeof stats, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&e, derr, sizeof e, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (e) return fail(HQA_EINVAL, "instance %d:%s", k, err_text(e).c_str());
    if (stats[1] < stats[0]) { stats[0] = 0; stats[1] = 0; }   // all zero
    I.es.lsb = stats[0];
    I.es.msb = stats[1];
    I.j_integral = stats[2] != 0;
    if (I.es.msb - I.es.lsb > 150 || I.es.lsb < -1022 + 53)
        I.es.lsb = INT32_MIN;  // exact read-out unavailable for this instance
    return HQA_OK;
}

static bool exact_ok(const Instance &I) { return I.es.lsb != INT32_MIN; }

// Scoped device buffers for the read-out.
struct DevBufs {
    std::vector<void *> v;
    template <typename T>
    hipError_t get(T **p, size_t n) {
        hipError_t e = dalloc(p, n);
        if (e == hipSuccess) v.push_back(*p);
        return e;
    }
    ~DevBufs() {
        for (void *p : v) dfree(p);
    }
};


// Per-block maxima of |a - b| and |b| over n values (finished on the host).
__global__ void k_maxdiff(const double *a, const double *b, int64_t n, double *out) {
    __shared__ double m0[256], m1[256];
    double d = 0.0, r = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        d = fmax(d, fabs(a[i] - b[i]));
        r = fmax(r, fabs(b[i]));
    }
    m0[threadIdx.x] = d;
    m1[threadIdx.x] = r;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            m0[threadIdx.x] = fmax(m0[threadIdx.x], m0[threadIdx.x + s]);
            m1[threadIdx.x] = fmax(m1[threadIdx.x], m1[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = m0[0];
        out[2 * blockIdx.x + 1] = m1[0];
    }
}

// Per-block sums over rows of max(p0, p1, p2) (finished on the host).
__global__ void k_sum_maxprob(const float *p, int64_t n, double *out) {
    __shared__ double sm[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        acc += (double)fmaxf(fmaxf(p[3 * i], p[3 * i + 1]), p[3 * i + 2]);
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

extern "C" {

int32_t hqa_abi_version(void) { return HQA_ABI_VERSION; }

const char *hqa_last_error(void) { return g_err.c_str(); }

void hqa_schedule_default(hqa_schedule *s) {
    if (!s) return;
    memset(s, 0, sizeof *s);
    s->alpha_f = 0.008; s->rho1 = 4.0; s->rho2 = 3.0;
    s->beta_f = 0.12; s->kappa1 = 0.05; s->kappa2 = 1.0;
    s->T = 50000; s->M = 6; s->W = 100; s->r_g = 1.0;
    s->frozen = 0; s->tau_frozen = 0.0;
}

void hqa_md_opts_default(hqa_md_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->replicas = 1;
    o->precision = HQA_PREC_F32;
    o->plan = HQA_PLAN_AUTO;
}

static void free_pass(void *p);

void hqa_md_destroy(hqa_md *md) {
    if (!md) return;
    if (md->stream || true) (void)hipStreamSynchronize(md->stream);
    for (auto &I : md->inst) free_instance(I);
    dfree(md->a64); dfree(md->b64); dfree(md->a32); dfree(md->b32);
    dfree(md->err); dfree(md->scratch_i); dfree(md->bar);
    free_batch_plan(md->batch);
    free_pass(md->pass);
    delete md;
}

hqa_status hqa_md_init(const hqa_problem *probs, int32_t count, const hqa_schedule *sched,
                       const hqa_md_opts *opts, void *hip_stream, hqa_md **out) {
    g_err.clear();
    fault_alloc_arm();
    if (!out) return fail(HQA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!probs || count < 1) return fail(HQA_EINVAL, "need at least one problem");
    if (!sched || !opts) return fail(HQA_EINVAL, "schedule and options are required");
    if (sched->T < 1) return fail(HQA_EINVAL, "T must be >= 1");
    if (sched->W < 1 || sched->W > sched->T) return fail(HQA_EINVAL, "W must satisfy 1 <= W <= T");
    if (sched->M < 2 || (sched->M & 1)) return fail(HQA_EINVAL, "M must be even and >= 2");
    if (!(sched->r_g > 0.0) || !isfinite(sched->r_g)) return fail(HQA_EINVAL, "r_g must be > 0");
    if (opts->replicas < 1) return fail(HQA_EINVAL, "replicas must be >= 1");
    if (opts->precision < HQA_PREC_F64_REF || opts->precision > HQA_PREC_FP8J_BF16)
        return fail(HQA_EINVAL, "unknown precision");
    if ((opts->p0 || opts->phi0) && opts->init_mem != HQA_HOST && opts->init_mem != HQA_DEVICE)
        return fail(HQA_EINVAL, "bad init_mem");
    if (opts->plan < HQA_PLAN_AUTO || opts->plan > HQA_PLAN_BATCH)
        return fail(HQA_EINVAL, "unknown plan %d", opts->plan);
    if (opts->flags & ~HQA_MD_GRAPH) return fail(HQA_EINVAL, "unknown flags 0x%x", opts->flags);
    for (int k = 0; k < count; k++) {
        hqa_status s = check_problem(probs[k], k);
        if (s != HQA_OK) return s;
        if (probs[k].layout == HQA_CSR && opts->precision >= HQA_PREC_BF16)
            return fail(HQA_EUNSUPPORTED, "instance %d: BF16/FP8 storage is for dense J only", k);
        const int sto = probs[k].storage;
        if (sto != 0) {
            if (sto != HQA_PREC_F32 && sto != HQA_PREC_BF16 && sto != HQA_PREC_FP8J_BF16)
                return fail(HQA_EINVAL, "instance %d: unknown storage %d", k, sto);
            if (probs[k].layout == HQA_CSR || opts->precision == HQA_PREC_F64_REF)
                return fail(HQA_EUNSUPPORTED,
                            "instance %d: a storage override needs a dense instance in a "
                            "non-reference handle", k);
        }
    }
    hipStream_t st = (hipStream_t)hip_stream;
    hqa_md *md = new hqa_md();
    md->stream = st;
    md->R = opts->replicas;
    md->prec = opts->precision;
    md->plan = opts->plan;
    md->flags = opts->flags;
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            lds > 0)
            md->max_lds = lds;
    }
    md->jt = opts->precision == HQA_PREC_BF16 ? JT_BF16
             : opts->precision == HQA_PREC_FP8J_BF16 ? JT_FP8 : JT_F32;
    Schedule64 &S = md->sch;
    S.prm[0] = sched->alpha_f; S.prm[1] = sched->rho1; S.prm[2] = sched->rho2;
    S.prm[3] = sched->beta_f; S.prm[4] = sched->kappa1; S.prm[5] = sched->kappa2;
    S.T = sched->T; S.M = sched->M; S.W = sched->W; S.r_g = sched->r_g;
    S.frozen = sched->frozen; S.tau_frozen = sched->tau_frozen;
    md->inst.resize(count);
    auto bail = [&](hqa_status s) { hqa_md_destroy(md); return s; };
#define CK(expr)                                 \
    do {                                         \
        hqa_status s_ = (expr);                  \
        if (s_ != HQA_OK) return bail(s_);       \
    } while (0)
#define HK(expr)                                                                            \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return bail(fail(e_ == hipErrorOutOfMemory ? HQA_ENOMEM : HQA_EDEVICE, "%s: %s", \
                             #expr, hipGetErrorString(e_)));                                \
    } while (0)
    HK(dalloc(&md->err, 1));
    HK(dalloc(&md->scratch_i, 16));
    HK(hipMemsetAsync(md->err, 0, sizeof(int32_t), st));
    const int64_t nk = 2 * S.T + 1;
    HK(dalloc(&md->a64, nk)); HK(dalloc(&md->b64, nk));
    HK(dalloc(&md->a32, nk)); HK(dalloc(&md->b32, nk));
    HK(launch_schedule(S, md->a64, md->b64, md->a32, md->b32, st));
    const int R = md->R;
    const bool f64 = md->prec == HQA_PREC_F64_REF;
    int64_t off = 0;
    for (int k = 0; k < count; k++) {
        Instance &I = md->inst[k];
        const hqa_problem &P = probs[k];
        CK(ingest(P, k, st, md->err, md->scratch_i, I));
        const int N = I.N;
        if (f64) {
            I.ld = N;
            size_t n = (size_t)N * R;
            HK(dalloc(&I.phi64[0], n)); HK(dalloc(&I.phi64[1], n));
            HK(dalloc(&I.p64, n)); HK(dalloc(&I.S64, n));
        } else {
            HK(dalloc(&I.h32, (size_t)N));
            HK(launch_convert_h(I.h64, N, I.h32, st));
            HK(hipMemsetAsync(md->err, 0, sizeof(int32_t), st));
            if (P.layout == HQA_DENSE) {
                I.smaj = false;
                I.Np = (N + 127) / 128 * 128;
                I.Rp = (R + 15) / 16 * 16;
                I.ld = I.Np;
                I.jt = md->jt;
                if (P.storage == HQA_PREC_F32) I.jt = JT_F32;
                else if (P.storage == HQA_PREC_BF16) I.jt = JT_BF16;
                else if (P.storage == HQA_PREC_FP8J_BF16) I.jt = JT_FP8;
                size_t esz = I.jt == JT_F32 ? 4 : I.jt == JT_BF16 ? 2 : 1;
                HK(dev_malloc(&I.Js, (size_t)I.Np * I.Np * esz));
                HK(launch_convert_dense(I.J64, N, I.Np, I.jt, I.Js, md->err, st));
                size_t n = (size_t)I.Rp * I.ld;
                for (int b = 0; b < 2; b++) {
                    HK(dalloc(&I.phi32[b], n));
                    HK(hipMemsetAsync(I.phi32[b], 0, n * 4, st));
                    if (I.jt != JT_F32) {
                        HK(dalloc(&I.phib[b], n));
                        HK(hipMemsetAsync(I.phib[b], 0, n * 2, st));
                    }
                }
                HK(dalloc(&I.p32, n)); HK(hipMemsetAsync(I.p32, 0, n * 4, st));
                HK(dalloc(&I.S32, n)); HK(hipMemsetAsync(I.S32, 0, n * 4, st));
            } else {
                I.smaj = true;
                I.Rp = (R + 3) / 4 * 4;
                I.ld = I.Rp;
                HK(dalloc(&I.v32, (size_t)I.nnz));
                if (I.nnz) HK(launch_convert_csr(I.J64, I.nnz, I.v32, md->err, st));
                size_t n = (size_t)N * I.Rp;
                for (int b = 0; b < 2; b++) {
                    HK(dalloc(&I.phi32[b], n));
                    HK(hipMemsetAsync(I.phi32[b], 0, n * 4, st));
                }
                HK(dalloc(&I.p32, n)); HK(hipMemsetAsync(I.p32, 0, n * 4, st));
                HK(dalloc(&I.S32, n)); HK(hipMemsetAsync(I.S32, 0, n * 4, st));
            }
            int32_t e = 0;
            HK(hipMemcpyAsync(&e, md->err, sizeof e, hipMemcpyDeviceToHost, st));
            HK(hipStreamSynchronize(st));
            if ((e & ERR_INEXACT) && opts->require_exact)
                return bail(fail(HQA_EUNSUPPORTED,
                                 "instance %d: J is not exactly representable in the storage "
                                 "type of the requested precision", k));
            I.js_exact = P.layout == HQA_DENSE && !(e & ERR_INEXACT);
            HK(hipMemsetAsync(md->err, 0, sizeof(int32_t), st));
        }
        const double *p0 = opts->p0 ? opts->p0 + off : nullptr;
        const double *phi0 = opts->phi0 ? opts->phi0 + off : nullptr;
        double *dp0 = nullptr, *dphi0 = nullptr;
        if (opts->init_mem == HQA_HOST && (p0 || phi0)) {
            size_t n = (size_t)N * R;
            if (p0) {
                HK(dalloc(&dp0, n));
                HK(hipMemcpyAsync(dp0, p0, n * 8, hipMemcpyHostToDevice, st));
            }
            if (phi0) {
                HK(dalloc(&dphi0, n));
                HK(hipMemcpyAsync(dphi0, phi0, n * 8, hipMemcpyHostToDevice, st));
            }
            p0 = dp0;
            phi0 = dphi0;
        }
        hipError_t le = launch_init_state(I, R, md->prec, opts->seed, p0, phi0, st);
        if (dp0 || dphi0) {
            (void)hipStreamSynchronize(st);
            dfree(dp0);
            dfree(dphi0);
        }
        HK(le);
        off += (int64_t)N * R;
    }
    HK(hipStreamSynchronize(st));
#undef CK
#undef HK
    *out = md;
    return HQA_OK;
}

int64_t hqa_md_step_index(const hqa_md *md) { return md ? md->q : -1; }

int32_t hqa_md_batch_form(const hqa_md *md, int32_t instance) {
    if (!md || instance < 0 || instance >= (int32_t)md->inst.size()) return -1;
    return batch_form(md, instance);
}

int32_t hqa_md_last_plan(const hqa_md *md) { return md ? md->last_plan : 0; }

hqa_status hqa_md_set_step(hqa_md *md, int64_t q) {
    if (!md) return fail(HQA_EINVAL, "null handle");
    if (q < 0 || q > md->sch.T) return fail(HQA_EINVAL, "step %lld outside [0, T]", (long long)q);
    md->q = q;
    return HQA_OK;
}

// Steps [q0, q1) of one dense binary32 instance under `plan`; a plan that does not
// apply (or whose launch is refused) falls back to one launch per step.
// The batched kernel as the plan of a single instance: the handle's only dense
// instance, with BF16 or FP8 storage (tiles of 128 rows x 64 replicas spread over
// the XCDs).
static bool batch_alone(const hqa_md *md, const Instance &I) {
    int ndense = 0;
    for (const auto &J : md->inst) ndense += J.layout == HQA_DENSE;
    return ndense == 1 && I.layout == HQA_DENSE && (I.jt == JT_BF16 || I.jt == JT_FP8);
}

static hipError_t run_dense(hqa_md *md, Instance &I, int64_t q0, int64_t q1, bool stats_live,
                            int plan, int *used) {
    if (plan == HQA_PLAN_AUTO) plan = I.tuned_plan ? I.tuned_plan : HQA_PLAN_STEP;
    if (!stats_live && plan == HQA_PLAN_RESIDENT && resident_fits(I, md->max_lds)) {
        hipError_t e = launch_md_resident(md, I, q0, q1);
        if (e == hipSuccess) {
            *used = HQA_PLAN_RESIDENT;
            return e;
        }
        (void)hipGetLastError();
    }
    if (!stats_live && plan == HQA_PLAN_BATCH && batch_alone(md, I)) {
        hipError_t e = launch_md_steps_batch(md, q0, q1, md->flags & HQA_MD_GRAPH);
        if (e == hipSuccess) {
            *used = HQA_PLAN_BATCH;
            return e;
        }
        (void)hipGetLastError();
    }
    if (!stats_live && plan == HQA_PLAN_CLUSTER) {
        hipError_t e = launch_md_persist(md, I, q0, q1);
        if (e == hipSuccess) {
            *used = HQA_PLAN_CLUSTER;
            return e;
        }
        (void)hipGetLastError();
    }
    *used = HQA_PLAN_STEP;
    return launch_md_steps_dense(md, I, q0, q1);
}

// The cluster plan over several dense instances: runs of consecutive instances of one
// size and storage share a register-J launch (the largest run the device fits, at
// most 8), so that instances whose clusters fill only part of the device advance
// together, each cluster on its own XCD.  An instance no launch takes runs alone.
static hipError_t run_dense_clusters(hqa_md *md, int64_t q0, int64_t q1, int *used) {
    std::vector<Instance *> d;
    for (auto &I : md->inst)
        if (I.layout == HQA_DENSE) d.push_back(&I);
    size_t i = 0;
    while (i < d.size()) {
        int k = 1;
        while (i + k < d.size() && k < 8 && d[i + k]->N == d[i]->N && d[i + k]->jt == d[i]->jt) k++;
        hipError_t e = hipErrorNotSupported;
        for (; k > 1; k--) {
            e = launch_md_persist_set(md, &d[i], k, q0, q1);
            if (e != hipErrorNotSupported) break;
        }
        if (e == hipErrorNotSupported) {
            k = 1;
            e = run_dense(md, *d[i], q0, q1, false, HQA_PLAN_CLUSTER, used);
        } else {
            *used = HQA_PLAN_CLUSTER;
        }
        if (e != hipSuccess) return e;
        i += k;
    }
    return hipSuccess;
}

// Steps [q0, q1) of one sparse binary32 instance under `plan` (RESIDENT or STEP).
static hipError_t run_csr(hqa_md *md, Instance &I, int64_t q0, int64_t q1, bool stats_live,
                          int plan, int *used) {
    if (plan == HQA_PLAN_AUTO) plan = I.tuned_plan ? I.tuned_plan : HQA_PLAN_STEP;
    if (!stats_live && plan == HQA_PLAN_RESIDENT && csr_resident_fits(md, I)) {
        hipError_t e = launch_md_csr_resident(md, I, q0, q1);
        if (e == hipSuccess) {
            *used = HQA_PLAN_RESIDENT;
            return e;
        }
        (void)hipGetLastError();
    }
    *used = HQA_PLAN_STEP;
    return launch_md_steps_csr(md, I, q0, q1);
}

// Which way several dense instances advance (the batch plan, or clusters).
static void multi_ways(const hqa_md *md, int64_t q1, bool *batched, bool *clustered) {
    int ndense = 0;
    for (auto &I : md->inst) ndense += I.layout == HQA_DENSE;
    // steps inside an early-stop statistics window run on the per-step kernels,
    // whose epilogues accumulate the statistics
    const bool stats_live = md->stats_k1 > md->q && md->stats_k0 < q1;
    // several dense instances under AUTO: the tuner's choice (batch when untuned)
    const bool multi = md->prec != HQA_PREC_F64_REF && ndense > 1 && !stats_live;
    const int mp = md->plan == HQA_PLAN_AUTO ? (md->multi_plan ? md->multi_plan : HQA_PLAN_BATCH)
                                             : md->plan;
    *batched = multi && md->plan == HQA_PLAN_AUTO && mp == HQA_PLAN_BATCH;
    *clustered = multi && mp == HQA_PLAN_CLUSTER;
}

// The steps md->q -> q1 on md->stream; `graph` lets the batch plan replay its cached
// step graphs.
static hqa_status run_core(hqa_md *md, int64_t q1, bool graph) {
    md->last_plan = 0;
    const bool stats_live = md->stats_k1 > md->q && md->stats_k0 < q1;
    bool batched = false, clustered = false;
    multi_ways(md, q1, &batched, &clustered);
    if (batched) {
        hipError_t e = launch_md_steps_batch(md, md->q, q1, graph);
        if (e != hipSuccess) return fail(dev_status(e), "batch step launch: %s", hipGetErrorString(e));
        md->last_plan = HQA_PLAN_BATCH;
    }
    if (clustered) {
        hipError_t e = run_dense_clusters(md, md->q, q1, &md->last_plan);
        if (e != hipSuccess) return fail(dev_status(e), "cluster launch: %s", hipGetErrorString(e));
    }
    for (auto &I : md->inst) {
        hipError_t e;
        if (md->prec == HQA_PREC_F64_REF) e = launch_md_steps_f64(md, I, md->q, q1);
        else if (I.layout == HQA_DENSE && (batched || clustered)) e = hipSuccess;
        else if (I.layout == HQA_DENSE) e = run_dense(md, I, md->q, q1, stats_live, md->plan, &md->last_plan);
        else e = run_csr(md, I, md->q, q1, stats_live, md->plan, &md->last_plan);
        if (e != hipSuccess) return fail(dev_status(e), "step launch: %s", hipGetErrorString(e));
    }
    md->q = q1;
    return HQA_OK;
}

hqa_status hqa_md_run(hqa_md *md, int64_t until_step) {
    if (!md) return fail(HQA_EINVAL, "null handle");
    int64_t q1 = until_step < 0 ? md->sch.T : until_step;
    if (q1 > md->sch.T) return fail(HQA_EINVAL, "until_step beyond T");
    if (q1 < md->q) return fail(HQA_ESTATE, "until_step %lld is before the current step %lld",
                                (long long)q1, (long long)md->q);
    if (q1 == md->q) return HQA_OK;
    CallTimer tm(md->stream);
    const int64_t q0 = md->q;
    const hqa_status rs = run_core(md, q1, md->flags & HQA_MD_GRAPH);
    if (rs != HQA_OK) return rs;
    const double ms = tm.stop();
    if (ms >= 0.0) {
        static const char *names[] = {"none", "step", "cluster", "resident", "batch"};
        const int lp = md->last_plan >= 0 && md->last_plan <= 4 ? md->last_plan : 0;
        fprintf(stderr, "hqa timing: hqa_md_run steps %lld..%lld, %zu instances, plan %s: "
                "%.3f ms, %.3f us per step\n", (long long)q0, (long long)q1, md->inst.size(),
                names[lp], ms, 1e3 * ms / (double)(q1 - q0));
    }
    return HQA_OK;
}

// Zeroes n 32-bit words with a kernel rather than a memset, so that a reset can be
// recorded into a HIP graph.
__global__ void k_zero_u32(uint32_t *p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

static hipError_t zero_u32(void *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    k_zero_u32<<<(unsigned)blocks, 256, 0, st>>>((uint32_t *)p, n);
    return hipGetLastError();
}

// The reset's device work on md->stream: no memset, no synchronisation.
static hipError_t reset_core(hqa_md *md, uint64_t seed) {
    hipError_t e = zero_u32(md->err, 1, md->stream);
    for (auto &I : md->inst) {
        if (e == hipSuccess && md->prec != HQA_PREC_F64_REF) {
            // padded rows / replicas of both flux buffers must stay zero
            size_t n = I.smaj ? (size_t)I.N * I.ld : (size_t)I.Rp * I.ld;
            e = zero_u32(I.phi32[I.cur ^ 1], (int64_t)n, md->stream);
        }
        if (e == hipSuccess) e = launch_init_state(I, md->R, md->prec, seed, nullptr, nullptr, md->stream);
    }
    md->q = 0;
    return e;
}

hqa_status hqa_md_reset(hqa_md *md, uint64_t seed) {
    if (!md) return fail(HQA_EINVAL, "null handle");
    HIPCHK(reset_core(md, seed));
    return HQA_OK;
}

// ---------------------------------------------------------------------------
// Autotuner of the dense binary32 step.  Every candidate computes the same
// binary32 operations in the same order, so the tuner may pick by time alone:
// it snapshots the state, times `steps` steps of each candidate from it with
// HIP events, restores it after each, and keeps the fastest for HQA_PLAN_AUTO.
// ---------------------------------------------------------------------------
struct TuneCand {
    int plan, tm, tn, cb, tj;
};

// Persisted tuner choices (HQA_TUNE_CACHE=path): one line per tuned case,
//   <key> | <plan> <tm> <tn> <cb> <tj>
// the last line for a key winning.  The key names the device (architecture and compute
// units), the case (one instance: layout, N, nonzeros, R, storage type, precision, LDS per
// workgroup; several dense instances: R, precision and every dense instance's N and
// storage type) and the tuning length.  Every plan gives bit-identical trajectories, so a
// stale entry can cost speed but never change a result; an entry naming a plan that does
// not apply falls back to STEP at run time like any other choice.
struct TuneCache {
    bool on = false;
    std::string path, device;
    std::map<std::string, TuneCand> m;

    explicit TuneCache(hqa_md *md) {
        const char *v = getenv("HQA_TUNE_CACHE");
        if (!v || !*v) return;
        path = v;
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return;
        char b[320];
        snprintf(b, sizeof b, "%s/%dcu/lds%d", prop.gcnArchName, prop.multiProcessorCount,
                 md->max_lds);
        device = b;
        on = true;
        FILE *f = fopen(path.c_str(), "r");
        if (!f) return;
        char line[4096];
        while (fgets(line, sizeof line, f)) {
            char *bar = strchr(line, '|');
            if (!bar) continue;
            TuneCand c;
            if (sscanf(bar + 1, "%d %d %d %d %d", &c.plan, &c.tm, &c.tn, &c.cb, &c.tj) != 5) continue;
            if (c.plan < HQA_PLAN_STEP || c.plan > HQA_PLAN_BATCH) continue;
            std::string k(line, bar - line);
            while (!k.empty() && k.back() == ' ') k.pop_back();
            m[k] = c;
        }
        fclose(f);
    }
    std::string instance_key(const hqa_md *md, const Instance &I, int steps) const {
        char b[256];
        snprintf(b, sizeof b, "%s one %s N=%d nnz=%lld R=%d jt=%d prec=%d steps=%d", device.c_str(),
                 I.layout == HQA_DENSE ? "dense" : "csr", I.N, (long long)I.nnz, md->R, (int)I.jt,
                 md->prec, steps);
        return b;
    }
    std::string multi_key(const hqa_md *md, int steps) const {
        std::string k = device + " several R=" + std::to_string(md->R) +
                        " prec=" + std::to_string(md->prec) + " steps=" + std::to_string(steps) + " N:jt=";
        for (const auto &I : md->inst)
            if (I.layout == HQA_DENSE) k += std::to_string(I.N) + ":" + std::to_string((int)I.jt) + ",";
        return k;
    }
    bool find(const std::string &k, TuneCand &c) const {
        if (!on) return false;
        auto it = m.find(k);
        if (it == m.end()) return false;
        c = it->second;
        return true;
    }
    // An entry is used only if it is a choice the tuner itself could make for I (the file
    // is input like any other: tile shapes must fit, as hqa_md_set_step_tiles checks).
    static bool fits(const Instance &I, const TuneCand &c) {
        const bool none = c.tm == 0 && c.tn == 0 && c.cb == 0 && c.tj == 0;
        if (I.layout != HQA_DENSE)
            return none && (c.plan == HQA_PLAN_STEP || c.plan == HQA_PLAN_RESIDENT);
        if (c.plan != HQA_PLAN_STEP) return none && c.plan >= HQA_PLAN_CLUSTER && c.plan <= HQA_PLAN_BATCH;
        if (none) return true;
        const bool lowp = I.jt == JT_BF16 || I.jt == JT_FP8;
        return (c.tm == 1 || c.tm == 2) && (c.tn == 1 || c.tn == 2 || c.tn == 4) &&
               I.Rp % (16 * c.tn) == 0 && (c.cb == 4 || c.cb == 8) && (c.tj == 0 || c.tj == 1) &&
               (!c.tj || lowp);
    }
    void store(const std::string &k, const TuneCand &c) {
        if (!on) return;
        m[k] = c;
        FILE *f = fopen(path.c_str(), "a");
        if (!f) return;
        fprintf(f, "%s | %d %d %d %d %d\n", k.c_str(), c.plan, c.tm, c.tn, c.cb, c.tj);
        fclose(f);
    }
};

// Several dense instances: time the batched kernel, the same-size cluster launches and
// each instance on its own tuned plan, over all dense instances together (snapshot,
// `steps` and 2 `steps` steps, restore, as for one instance), and keep the fastest in
// md->multi_plan for AUTO.  A candidate that raises the error word is disqualified.
static hqa_status tune_multi(hqa_md *md, int32_t steps, hipEvent_t e0, hipEvent_t e1,
                             TuneCache &cache) {
    std::vector<Instance *> d;
    for (auto &I : md->inst)
        if (I.layout == HQA_DENSE) d.push_back(&I);
    md->multi_plan = 0;
    if (d.size() < 2) return HQA_OK;
    const std::string key = cache.multi_key(md, steps);
    TuneCand cached;
    if (cache.find(key, cached) && (cached.plan == HQA_PLAN_BATCH || cached.plan == HQA_PLAN_CLUSTER ||
                                    cached.plan == HQA_PLAN_STEP)) {
        md->multi_plan = cached.plan;
        return HQA_OK;
    }
    struct Snap { float *x, *p, *S; bf16 *b; size_t n; int cur; };
    std::vector<Snap> sn(d.size(), Snap{nullptr, nullptr, nullptr, nullptr, 0, 0});
    hipError_t he = hipSuccess;
    for (size_t k = 0; k < d.size() && he == hipSuccess; k++) {
        sn[k].n = (size_t)d[k]->Rp * d[k]->ld;
        sn[k].cur = d[k]->cur;
        he = dalloc(&sn[k].x, sn[k].n);
        if (he == hipSuccess) he = dalloc(&sn[k].p, sn[k].n);
        if (he == hipSuccess) he = dalloc(&sn[k].S, sn[k].n);
        if (he == hipSuccess) he = dalloc(&sn[k].b, sn[k].n);
    }
    if (he != hipSuccess) {
        for (auto &x : sn) { dfree(x.x); dfree(x.p); dfree(x.S); dfree(x.b); }
        return fail(HQA_ENOMEM, "tuner snapshot of %zu instances", d.size());
    }
    auto copy = [&](bool save) -> hipError_t {
        hipError_t e = hipSuccess;
        for (size_t k = 0; k < d.size(); k++) {
            Instance &I = *d[k];
            auto cp = [&](void *a, void *b, size_t bytes) {
                if (e == hipSuccess)
                    e = hipMemcpyAsync(save ? b : a, save ? a : b, bytes, hipMemcpyDeviceToDevice,
                                       md->stream);
            };
            cp(I.phi32[sn[k].cur], sn[k].x, sn[k].n * 4);
            cp(I.p32, sn[k].p, sn[k].n * 4);
            cp(I.S32, sn[k].S, sn[k].n * 4);
            if (I.phib[sn[k].cur]) cp(I.phib[sn[k].cur], sn[k].b, sn[k].n * 2);
            I.cur = sn[k].cur;
        }
        return e;
    };
    int32_t err0 = 0;
    if (he == hipSuccess) he = copy(true);
    if (he == hipSuccess)
        he = hipMemcpyAsync(&err0, md->err, sizeof err0, hipMemcpyDeviceToHost, md->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(md->stream);
    float best = 1e30f;
    int pick = HQA_PLAN_BATCH;
    for (int cand : {HQA_PLAN_BATCH, HQA_PLAN_CLUSTER, HQA_PLAN_STEP}) {
        float t[3] = {0.f, 0.f, 0.f};
        for (int pass = 0; pass < 3 && he == hipSuccess; pass++) {
            const int64_t q1 = md->q + (pass == 2 ? 2 * (int64_t)steps : steps);
            int used = 0;
            he = hipEventRecord(e0, md->stream);
            if (he == hipSuccess) {
                if (cand == HQA_PLAN_BATCH) {
                    he = launch_md_steps_batch(md, md->q, q1);
                } else if (cand == HQA_PLAN_CLUSTER) {
                    he = run_dense_clusters(md, md->q, q1, &used);
                } else {
                    for (Instance *I : d)
                        if (he == hipSuccess)
                            he = run_dense(md, *I, md->q, q1, false, HQA_PLAN_AUTO, &used);
                }
            }
            if (he == hipSuccess) he = hipEventRecord(e1, md->stream);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            if (he == hipSuccess) he = hipEventElapsedTime(&t[pass], e0, e1);
            if (he == hipSuccess) he = copy(false);
        }
        float ms = std::max(t[2] - t[1], 0.0f);
        int32_t errc = err0;
        if (he == hipSuccess)
            he = hipMemcpyAsync(&errc, md->err, sizeof errc, hipMemcpyDeviceToHost, md->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(md->stream);
        if (he == hipSuccess && errc != err0) {
            ms = 1e30f;
            he = hipMemcpyAsync(md->err, &err0, sizeof err0, hipMemcpyHostToDevice, md->stream);
            if (he == hipSuccess) he = hipStreamSynchronize(md->stream);
        }
        if (he == hipSuccess && ms < best) {
            best = ms;
            pick = cand;
        }
    }
    if (he == hipSuccess) he = hipStreamSynchronize(md->stream);
    for (auto &x : sn) { dfree(x.x); dfree(x.p); dfree(x.S); dfree(x.b); }
    if (he != hipSuccess) return fail(dev_status(he), "tuning several instances: %s", hipGetErrorString(he));
    md->multi_plan = pick;
    cache.store(key, TuneCand{pick, 0, 0, 0, 0});
    return HQA_OK;
}

hqa_status hqa_md_tune(hqa_md *md, int32_t steps) {
    if (!md) return fail(HQA_EINVAL, "null handle");
    if (steps < 1) return fail(HQA_EINVAL, "steps must be >= 1");
    if (md->q + 2 * (int64_t)steps > md->sch.T)
        return fail(HQA_ESTATE, "fewer than %d steps remain before T", 2 * steps);
    if (md->prec == HQA_PREC_F64_REF) return HQA_OK;
    HIPCHK(hipStreamSynchronize(md->stream));
    const int64_t k0 = md->stats_k0, k1 = md->stats_k1;
    md->stats_k0 = md->stats_k1 = 0;   // candidates accumulate no statistics
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hqa_status rs = HQA_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rs = fail(HQA_EDEVICE, "event creation failed");
    TuneCache cache(md);
    for (auto &I : md->inst) {
        if (rs != HQA_OK) break;
        const bool dense = I.layout == HQA_DENSE;
        const std::string key = cache.instance_key(md, I, steps);
        TuneCand cached;
        if (cache.find(key, cached) && TuneCache::fits(I, cached)) {
            I.tuned_plan = cached.plan;
            I.step_tm = cached.tm;
            I.step_tn = cached.tn;
            I.step_cb = cached.cb;
            I.step_tj = cached.tj;
            continue;
        }
        const size_t n = I.smaj ? (size_t)I.N * I.ld : (size_t)I.Rp * I.ld;
        float *sx = nullptr, *sp = nullptr, *sS = nullptr;
        bf16 *sb = nullptr;
        if (dalloc(&sx, n) != hipSuccess || dalloc(&sp, n) != hipSuccess ||
            dalloc(&sS, n) != hipSuccess || dalloc(&sb, n) != hipSuccess) {
            dfree(sx); dfree(sp); dfree(sS); dfree(sb);
            rs = fail(HQA_ENOMEM, "tuner snapshot");
            break;
        }
        const int cur0 = I.cur;
        auto copy = [&](bool save) -> hipError_t {
            hipError_t e = hipSuccess;
            auto cp = [&](void *a, void *b, size_t bytes) {
                if (e == hipSuccess)
                    e = hipMemcpyAsync(save ? b : a, save ? a : b, bytes, hipMemcpyDeviceToDevice,
                                       md->stream);
            };
            cp(I.phi32[cur0], sx, n * 4);
            cp(I.p32, sp, n * 4);
            cp(I.S32, sS, n * 4);
            if (I.phib[cur0]) cp(I.phib[cur0], sb, n * 2);   // BF16 operand copy, if kept
            I.cur = cur0;
            return e;
        };
        std::vector<TuneCand> cands;
        if (dense) {
            const bool lowp = I.jt == JT_BF16 || I.jt == JT_FP8;
            for (int tj : {0, 1}) {
                if (tj && !lowp) continue;
                for (int cb : {4, 8})
                    for (int tm : {2, 1})
                        for (int tn : {4, 2, 1})
                            if (I.Rp % (16 * tn) == 0) cands.push_back({HQA_PLAN_STEP, tm, tn, cb, tj});
            }
            cands.push_back({HQA_PLAN_CLUSTER, 0, 0, 0, 0});
            if (resident_fits(I, md->max_lds)) cands.push_back({HQA_PLAN_RESIDENT, 0, 0, 0, 0});
            if (batch_alone(md, I)) cands.push_back({HQA_PLAN_BATCH, 0, 0, 0, 0});
        } else {
            cands.push_back({HQA_PLAN_STEP, 0, 0, 0, 0});
            if (csr_resident_fits(md, I)) cands.push_back({HQA_PLAN_RESIDENT, 0, 0, 0, 0});
        }
        float best = 1e30f;
        TuneCand pick{HQA_PLAN_STEP, 0, 0, 0, 0};
        const int tn0 = I.step_tn, tm0 = I.step_tm, cb0 = I.step_cb, tj0 = I.step_tj;
        const char *stage = "snapshot";
        hipError_t he = copy(true);
        // the error word as the caller left it: a candidate that raises a flag is
        // disqualified and the word is put back, so timing never leaks a status
        int32_t err0 = 0;
        if (he == hipSuccess)
            he = hipMemcpyAsync(&err0, md->err, sizeof err0, hipMemcpyDeviceToHost, md->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(md->stream);
        TuneCand failed{0, 0, 0, 0, 0};
        for (const TuneCand &c : cands) {
            if (he != hipSuccess) break;
            failed = c;
            I.step_tn = c.tn;
            I.step_tm = c.tm;
            I.step_cb = c.cb;
            I.step_tj = c.tj;
            // pass 0 warms up; passes 1 and 2 run `steps` and 2 `steps` steps, and the
            // difference is the cost of `steps` steps without the plan's fixed per-run
            // cost (state staging of the one-launch plans, first-use set-up)
            float ms = 0.f, t[3] = {0.f, 0.f, 0.f};
            for (int pass = 0; pass < 3 && he == hipSuccess; pass++) {
                const int64_t len = pass == 2 ? 2 * (int64_t)steps : steps;
                int used = 0;
                stage = "event record";
                he = hipEventRecord(e0, md->stream);
                if (he == hipSuccess) {
                    stage = "run";
                    he = dense ? run_dense(md, I, md->q, md->q + len, false, c.plan, &used)
                               : run_csr(md, I, md->q, md->q + len, false, c.plan, &used);
                }
                if (he == hipSuccess) {
                    stage = "event record";
                    he = hipEventRecord(e1, md->stream);
                }
                if (he == hipSuccess) {
                    stage = "event synchronize";
                    he = hipEventSynchronize(e1);
                }
                if (he == hipSuccess) {
                    stage = "elapsed time";
                    he = hipEventElapsedTime(&t[pass], e0, e1);
                }
                if (he == hipSuccess) {
                    stage = "restore";
                    he = copy(false);
                }
                if (he == hipSuccess && used != c.plan) t[pass] = 1e30f;   // not applicable
            }
            ms = t[2] >= 1e30f || t[1] >= 1e30f ? 1e30f : std::max(t[2] - t[1], 0.0f);
            int32_t errc = err0;
            if (he == hipSuccess) {
                stage = "error word";
                he = hipMemcpyAsync(&errc, md->err, sizeof errc, hipMemcpyDeviceToHost, md->stream);
                if (he == hipSuccess) he = hipStreamSynchronize(md->stream);
            }
            if (he == hipSuccess && errc != err0) {
                ms = 1e30f;
                he = hipMemcpyAsync(md->err, &err0, sizeof err0, hipMemcpyHostToDevice, md->stream);
                if (he == hipSuccess) he = hipStreamSynchronize(md->stream);
            }
            if (he == hipSuccess && ms < best) {
                best = ms;
                pick = c;
            }
        }
        I.step_tn = tn0;
        I.step_tm = tm0;
        I.step_cb = cb0;
        I.step_tj = tj0;
        if (he == hipSuccess) he = hipStreamSynchronize(md->stream);
        dfree(sx); dfree(sp); dfree(sS); dfree(sb);
        if (he != hipSuccess) {
            rs = fail(dev_status(he), "tuning (plan %d, tiles %d x %d, %s): %s", failed.plan, failed.tm,
                      failed.tn, stage, hipGetErrorString(he));
            break;
        }
        I.tuned_plan = pick.plan;
        I.step_tn = pick.tn;
        I.step_tm = pick.tm;
        I.step_cb = pick.cb;
        I.step_tj = pick.tj;
        cache.store(key, pick);
    }
    if (rs == HQA_OK) rs = tune_multi(md, steps, e0, e1, cache);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    md->stats_k0 = k0;
    md->stats_k1 = k1;
    return rs;
}

hqa_status hqa_md_set_step_tiles(hqa_md *md, int32_t k, int32_t tm, int32_t tn, int32_t cb,
                                 int32_t tiled) {
    if (!md) return fail(HQA_EINVAL, "null handle");
    if (k < 0 || k >= (int32_t)md->inst.size()) return fail(HQA_EINVAL, "instance %d out of range", k);
    Instance &I = md->inst[k];
    if (I.layout != HQA_DENSE) return fail(HQA_EINVAL, "instance %d is not dense", k);
    if ((tm != 1 && tm != 2) || (tn != 1 && tn != 2 && tn != 4) || I.Rp % (16 * tn) != 0)
        return fail(HQA_EINVAL, "block of %d x %d tiles does not fit (padded replicas %d)", tm, tn, I.Rp);
    if (cb != 4 && cb != 8) return fail(HQA_EINVAL, "chunks in flight must be 4 or 8");
    if (tiled != 0 && tiled != 1) return fail(HQA_EINVAL, "tiled must be 0 or 1");
    if (tiled && I.jt != JT_BF16 && I.jt != JT_FP8)
        return fail(HQA_EINVAL, "the tiled copy of J exists for BF16 and FP8 storage only");
    I.step_tm = tm;
    I.step_tn = tn;
    I.step_cb = cb;
    I.step_tj = tiled;
    I.tuned_plan = HQA_PLAN_STEP;
    return HQA_OK;
}

int32_t hqa_md_tuned_plan(const hqa_md *md, int32_t k, int32_t *tm, int32_t *tn, int32_t *cb,
                          int32_t *tiled) {
    if (!md || k < 0 || k >= (int32_t)md->inst.size()) return -1;
    if (tm) *tm = md->inst[k].step_tm;
    if (tn) *tn = md->inst[k].step_tn;
    if (cb) *cb = md->inst[k].step_cb;
    if (tiled) *tiled = md->inst[k].step_tj;
    return md->inst[k].tuned_plan;
}

hqa_status hqa_md_sync(hqa_md *md) {
    if (!md) return fail(HQA_EINVAL, "null handle");
    int32_t e = 0;
    HIPCHK(hipMemcpyAsync(&e, md->err, sizeof e, hipMemcpyDeviceToHost, md->stream));
    HIPCHK(hipStreamSynchronize(md->stream));
    if (e & ERR_NONFINITE) return fail(HQA_ENONFINITE, "a flux or momentum became non-finite");
    if (e) return fail(HQA_EDEVICE, "device error:%s", err_text(e).c_str());
    return HQA_OK;
}

static hqa_status check_instance(hqa_md *md, int32_t k) {
    if (!md) return fail(HQA_EINVAL, "null handle");
    if (k < 0 || k >= (int32_t)md->inst.size()) return fail(HQA_EINVAL, "instance %d out of range", k);
    return HQA_OK;
}

__global__ void k_scale_f64(double *x, int64_t n, double s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = x[i] * s;
}

hqa_status hqa_md_state(hqa_md *md, int32_t instance, int32_t what, void *dst, int32_t dst_mem,
                        int32_t import) {
    hqa_status s = check_instance(md, instance);
    if (s != HQA_OK) return s;
    if (!dst) return fail(HQA_EINVAL, "dst is NULL");
    if (what < HQA_STATE_PHI || what > HQA_STATE_STATMEAN) return fail(HQA_EINVAL, "unknown state");
    if (import && (what == HQA_STATE_PHIBAR || what == HQA_STATE_STATMEAN))
        return fail(HQA_EINVAL, "this state cannot be imported");
    Instance &I = md->inst[instance];
    int64_t nstat = 0;
    if (what == HQA_STATE_STATMEAN) {
        if (md->prec == HQA_PREC_F64_REF || !I.st)
            return fail(HQA_ESTATE, "no statistics window has been set");
        nstat = stats_count(md);
        if (nstat < 1) return fail(HQA_ESTATE, "no step of the statistics window has run");
    }
    const size_t n = (size_t)I.N * md->R;
    double *buf = (double *)dst;
    if (dst_mem == HQA_HOST) HIPCHK(dalloc(&buf, n));
    if (import && dst_mem == HQA_HOST)
        HIPCHK(hipMemcpyAsync(buf, dst, n * 8, hipMemcpyHostToDevice, md->stream));
    if (what == HQA_STATE_STATMEAN) {
        // the first statistics array is the running sum of phi^(q+1)
        HIPCHK(launch_layout_to_f64(I.N, md->R, I.ld, I.smaj, I.st, buf, md->stream));
        k_scale_f64<<<(unsigned)((n + 255) / 256), 256, 0, md->stream>>>(buf, (int64_t)n,
                                                                       1.0 / (double)nstat);
        HIPCHK(hipGetLastError());
    } else {
        HIPCHK(launch_export(I, md->R, md->prec, what, buf, import, md->sch.W, md->stream));
    }
    if (!import && dst_mem == HQA_HOST)
        HIPCHK(hipMemcpyAsync(dst, buf, n * 8, hipMemcpyDeviceToHost, md->stream));
    HIPCHK(hipStreamSynchronize(md->stream));
    if (dst_mem == HQA_HOST) dfree(buf);
    return HQA_OK;
}

hqa_status hqa_md_field_error(hqa_md *md, int32_t instance, double *max_abs_err,
                              double *max_abs_field) {
    hqa_status s = check_instance(md, instance);
    if (s != HQA_OK) return s;
    if (!max_abs_err || !max_abs_field) return fail(HQA_EINVAL, "null output");
    if (md->prec == HQA_PREC_F64_REF) return fail(HQA_EUNSUPPORTED, "the reference mode is binary64");
    Instance &I = md->inst[instance];
    if ((size_t)I.N * 8 + 8192 > (size_t)md->max_lds)
        return fail(HQA_EUNSUPPORTED, "binary64 field: N = %d exceeds the LDS capacity", I.N);
    const size_t n = (size_t)I.N * md->R;
    const size_t m = I.smaj ? (size_t)I.N * I.ld : (size_t)I.Rp * I.ld;
    DevBufs bufs;
    double *u, *u64, *part;
    float *u32;
    const int blocks = 256;
    HIPCHK(bufs.get(&u, n));
    HIPCHK(bufs.get(&u64, n));
    HIPCHK(bufs.get(&part, 2 * blocks));
    HIPCHK(bufs.get(&u32, m));
    if (I.layout == HQA_DENSE) HIPCHK(launch_field_dense(md, I, u32, md->stream));
    else HIPCHK(launch_field_csr(md, I, u32, md->stream));
    HIPCHK(launch_layout_to_f64(I.N, md->R, I.ld, I.smaj, u32, u, md->stream));
    HIPCHK(launch_field_f64(md, I, u64, md->stream));
    k_maxdiff<<<blocks, 256, 0, md->stream>>>(u, u64, (int64_t)n, part);
    HIPCHK(hipGetLastError());
    std::vector<double> h(2 * blocks);
    HIPCHK(hipMemcpyAsync(h.data(), part, sizeof(double) * 2 * blocks, hipMemcpyDeviceToHost,
                          md->stream));
    HIPCHK(hipStreamSynchronize(md->stream));
    double e = 0.0, r = 0.0;
    for (int b = 0; b < blocks; b++) {
        e = std::max(e, h[2 * b]);
        r = std::max(r, h[2 * b + 1]);
    }
    *max_abs_err = e;
    *max_abs_field = r;
    return HQA_OK;
}

hqa_status hqa_md_field(hqa_md *md, int32_t instance, double *u, int32_t dst_mem) {
    hqa_status s = check_instance(md, instance);
    if (s != HQA_OK) return s;
    if (!u) return fail(HQA_EINVAL, "u is NULL");
    Instance &I = md->inst[instance];
    const size_t n = (size_t)I.N * md->R;
    double *buf = u;
    if (dst_mem == HQA_HOST) HIPCHK(dalloc(&buf, n));
    if (md->prec == HQA_PREC_F64_REF) {
        if ((size_t)I.N * 8 + 8192 > (size_t)md->max_lds)
        return fail(HQA_EUNSUPPORTED, "binary64 field: N = %d exceeds the LDS capacity", I.N);
        HIPCHK(launch_field_f64(md, I, buf, md->stream));
    } else {
        float *u32;
        size_t m = I.smaj ? (size_t)I.N * I.ld : (size_t)I.Rp * I.ld;
        HIPCHK(dalloc(&u32, m));
        if (I.layout == HQA_DENSE) HIPCHK(launch_field_dense(md, I, u32, md->stream));
        else HIPCHK(launch_field_csr(md, I, u32, md->stream));
        HIPCHK(launch_layout_to_f64(I.N, md->R, I.ld, I.smaj, u32, buf, md->stream));
        HIPCHK(hipStreamSynchronize(md->stream));
        dfree(u32);
    }
    if (dst_mem == HQA_HOST) HIPCHK(hipMemcpyAsync(u, buf, n * 8, hipMemcpyDeviceToHost, md->stream));
    HIPCHK(hipStreamSynchronize(md->stream));
    if (dst_mem == HQA_HOST) dfree(buf);
    return HQA_OK;
}

hqa_status hqa_md_hamiltonian(hqa_md *md, int32_t instance, double *H, int32_t dst_mem) {
    hqa_status s = check_instance(md, instance);
    if (s != HQA_OK) return s;
    if (!H) return fail(HQA_EINVAL, "H is NULL");
    Instance &I = md->inst[instance];
    if ((size_t)I.N * 8 + 8192 > (size_t)md->max_lds)
        return fail(HQA_EUNSUPPORTED, "binary64 Hamiltonian: N = %d exceeds the LDS capacity", I.N);
    double *buf = H;
    if (dst_mem == HQA_HOST) HIPCHK(dalloc(&buf, (size_t)md->R));
    HIPCHK(launch_hamiltonian(md, I, buf, md->stream));
    if (dst_mem == HQA_HOST)
        HIPCHK(hipMemcpyAsync(H, buf, (size_t)md->R * 8, hipMemcpyDeviceToHost, md->stream));
    HIPCHK(hipStreamSynchronize(md->stream));
    if (dst_mem == HQA_HOST) dfree(buf);
    return HQA_OK;
}

// Read-out shared by hqa_classify (sort by |phibar|), hqa_classify_probs (predicted
// labels) and hqa_classify_tabu: selection, optional reduced problem solved exactly
// (solve = 1) or by the tabu search (solve = 2), merge, energies.
static hqa_status classify_checks(hqa_md *md, int32_t instance, int32_t n_amb, int32_t solve,
                                  const hqa_classify_out *out, const float *prob,
                                  bool need_spins = true, bool need_T = true) {
    hqa_status s = check_instance(md, instance);
    if (s != HQA_OK) return s;
    if (!out || (need_spins && !out->spins)) return fail(HQA_EINVAL, "out->spins is required");
    Instance &I = md->inst[instance];
    const int N = I.N;
    if (n_amb < 0 || n_amb > N) return fail(HQA_EINVAL, "n_amb must lie in [0, N]");
    if (solve == 1 && n_amb > 24)
        return fail(HQA_EUNSUPPORTED, "exact enumeration limited to n <= 24");
    if (!prob && need_T && md->q != md->sch.T)
        return fail(HQA_ESTATE, "classify needs the run to reach step T");
    if ((solve || out->energy || out->cut || out->h_eff) && !exact_ok(I))
        return fail(HQA_EUNSUPPORTED, "coupling exponents span too many binades for exact sums");
    if (solve == 2 && I.es.lsb != INT32_MIN) {
        // |f_a| <= 2 (N + 1) max(|J|, |h|) and |D| <= 2 (N + 1)^2 max(|J|, |h|): both stay
        // finite, so every gain is a number and the search follows its definition
        int lg = 0;
        while (lg < 62 && ((int64_t)1 << lg) < (int64_t)N + 1) lg++;
        if (I.es.msb + 2 * lg + 4 > 1023)
            return fail(HQA_EUNSUPPORTED, "couplings too large for finite tabu-search fields");
    }
    if (solve == 1 && I.j_integral && I.es.msb + 2 * 16 + 8 > 62)
        return fail(HQA_EUNSUPPORTED, "integer couplings too large for int64 enumeration");
    return HQA_OK;
}

// The read-out after classify_checks; device scratch comes from B (DevBufs allocates,
// ScratchArena carves a fixed array).
extern "C++" {
template <class Bufs>
static hqa_status classify_core(hqa_md *md, int32_t instance, int32_t n_amb, int32_t solve,
                                const hqa_classify_out *out, int32_t out_mem, const float *prob,
                                int32_t prob_mem, int64_t tabu_iters, int32_t tenure, Bufs &B,
                                bool sync = true, hipStream_t side = nullptr) {
    Instance &I = md->inst[instance];
    const int R = md->R, N = I.N;
    if (sync) {
        hqa_status s = hqa_md_sync(md);
        if (s != HQA_OK) return s;
    }
    // the handle's stream, or (side != NULL, no sync) a stream of the caller's that has
    // been ordered after it
    hipStream_t st = side ? side : md->stream;
    int32_t *amb;
    int8_t *spins;
    HIPCHK(B.get(&amb, (size_t)R * (n_amb ? n_amb : 1)));
    HIPCHK(B.get(&spins, (size_t)R * N));
    if (!prob) {
        HIPCHK(launch_select(I, R, md->prec, md->sch.W, n_amb, amb, spins, st));
    } else {
        const float *dprob = prob;
        float *tmp = nullptr, *keys = nullptr;
        if (prob_mem == HQA_HOST) {
            HIPCHK(B.get(&tmp, (size_t)R * N * 3));
            HIPCHK(hipMemcpyAsync(tmp, prob, sizeof(float) * R * N * 3, hipMemcpyHostToDevice, st));
            dprob = tmp;
        }
        HIPCHK(B.get(&keys, (size_t)R * N));
        HIPCHK(launch_probs_to_keys((int64_t)R * N, dprob, spins, keys, st));
        HIPCHK(launch_select_keys(N, R, keys, n_amb, amb, spins, st));
    }
    double *h_eff = nullptr, *J_eff = nullptr, *e_red = nullptr;
    int64_t *code = nullptr;
    if (solve == 2 && n_amb > 0) {
        int8_t *merged;
        HIPCHK(B.get(&h_eff, (size_t)R * n_amb));
        HIPCHK(B.get(&e_red, (size_t)R));
        HIPCHK(B.get(&merged, (size_t)R * N));
        HIPCHK(launch_reduce(I, R, n_amb, amb, spins, h_eff, nullptr, st));
        HIPCHK(hipMemcpyAsync(merged, spins, (size_t)R * N, hipMemcpyDeviceToDevice, st));
        HIPCHK(launch_tabu(I, R, n_amb, amb, spins, h_eff, tabu_iters, tenure, merged, e_red, st));
        spins = merged;
    } else if (solve == 2) {   // nothing to search: D_best = 0
        HIPCHK(B.get(&e_red, (size_t)R));
        HIPCHK(hipMemsetAsync(e_red, 0, sizeof(double) * R, st));
    } else if (solve && n_amb > 0) {
        HIPCHK(B.get(&h_eff, (size_t)R * n_amb));
        HIPCHK(B.get(&J_eff, (size_t)R * n_amb * n_amb));
        HIPCHK(B.get(&code, (size_t)R));
        HIPCHK(B.get(&e_red, (size_t)R));
        HIPCHK(launch_reduce(I, R, n_amb, amb, spins, h_eff, J_eff, st));
        uint8_t *escr;
        HIPCHK(B.get(&escr, enum_scratch_bytes(n_amb, R)));
        HIPCHK(launch_enumerate(n_amb, R, J_eff, h_eff, I.es.lsb, I.j_integral ? 1 : 0, code,
                                e_red, escr, st));
        HIPCHK(launch_merge(N, R, n_amb, amb, code, spins, st));
    } else if (out->h_eff && n_amb > 0) {
        HIPCHK(B.get(&h_eff, (size_t)R * n_amb));
        HIPCHK(B.get(&J_eff, (size_t)R * n_amb * n_amb));
        HIPCHK(launch_reduce(I, R, n_amb, amb, spins, h_eff, J_eff, st));
    }
    double *E = nullptr, *C = nullptr;
    if (out->energy || out->cut) {
        HIPCHK(B.get(&E, (size_t)R));
        HIPCHK(B.get(&C, (size_t)R));
        uint8_t *part;
        HIPCHK(B.get(&part, energy_part_bytes(N, R)));
        HIPCHK(launch_energy(I, R, spins, E, C, part, st));
    }
    hipMemcpyKind kd = kind_out(out_mem);
    if (out->spins) HIPCHK(hipMemcpyAsync(out->spins, spins, (size_t)R * N, kd, st));
    if (out->amb_idx && n_amb) HIPCHK(hipMemcpyAsync(out->amb_idx, amb, (size_t)R * n_amb * 4, kd, st));
    if (out->energy) HIPCHK(hipMemcpyAsync(out->energy, E, (size_t)R * 8, kd, st));
    if (out->cut) HIPCHK(hipMemcpyAsync(out->cut, C, (size_t)R * 8, kd, st));
    if (out->h_eff && h_eff) HIPCHK(hipMemcpyAsync(out->h_eff, h_eff, (size_t)R * n_amb * 8, kd, st));
    if (out->code && code) HIPCHK(hipMemcpyAsync(out->code, code, (size_t)R * 8, kd, st));
    if (out->e_reduced && e_red) HIPCHK(hipMemcpyAsync(out->e_reduced, e_red, (size_t)R * 8, kd, st));
    if (sync) HIPCHK(hipStreamSynchronize(st));
    return HQA_OK;
}
}  // extern "C++"

static hqa_status classify_impl(hqa_md *md, int32_t instance, int32_t n_amb, int32_t solve,
                                const hqa_classify_out *out, int32_t out_mem, const float *prob,
                                int32_t prob_mem, int64_t tabu_iters = 0, int32_t tenure = 0) {
    hqa_status s = classify_checks(md, instance, n_amb, solve, out, prob);
    if (s != HQA_OK) return s;
    DevBufs B;
    CallTimer tm(md->stream);
    s = classify_core(md, instance, n_amb, solve, out, out_mem, prob, prob_mem, tabu_iters,
                      tenure, B);
    const double ms = tm.stop();
    if (s == HQA_OK && ms >= 0.0)
        fprintf(stderr, "hqa timing: read-out of instance %d (N = %d, R = %d, n = %d, solve %d): "
                "%.3f ms\n", instance, md->inst[instance].N, md->R, n_amb, solve, ms);
    return s;
}

hqa_status hqa_classify(hqa_md *md, int32_t instance, int32_t n_amb, int32_t solve,
                        const hqa_classify_out *out, int32_t out_mem) {
    // the tabu mode (2) is reachable only through hqa_classify_tabu, which checks its limits
    if (solve != 0 && solve != 1) return fail(HQA_EINVAL, "solve must be 0 or 1");
    return classify_impl(md, instance, n_amb, solve, out, out_mem, nullptr, HQA_HOST);
}

// ---------------------------------------------------------------------------
// Read-out without device allocation.  Its scratch is one fixed device array per GPU;
// host code never passes the array's name to a kernel (in host code that name is a
// stand-in, not a device address): the address comes from hipGetSymbolAddress, once
// per device, and only that pointer is used.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[HQA_NOALLOC_SCRATCH_BYTES];

#define HQA_MAX_DEVICES 64
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[HQA_MAX_DEVICES] = {};

// The current device's address of `scratch` (looked up at the first call on a device).
static hqa_status noalloc_scratch(void **ptr) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= HQA_MAX_DEVICES)
        return fail(HQA_EUNSUPPORTED, "device %d beyond the %d the library tracks", dev,
                    HQA_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HQA_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return HQA_OK;
}

// Bump allocation from a fixed region, 256-byte aligned, in the same order and sizes
// as DevBufs::get calls of classify_core.
extern "C++" {
struct ScratchArena {
    uint8_t *base = nullptr;
    size_t cap = 0, used = 0;
    static size_t round(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
    template <typename T>
    hipError_t get(T **p, size_t n) {
        const size_t b = round(n * sizeof(T));
        if (used + b > cap) return hipErrorOutOfMemory;
        *p = (T *)(base + used);
        used += b;
        return hipSuccess;
    }
};
}  // extern "C++"

// Bytes classify_core takes from its provider for solve in {0, 1} and phibar input.
static size_t classify_scratch_bytes(int R, int N, int n, int solve, const hqa_classify_out *out) {
    auto r = ScratchArena::round;
    size_t b = r((size_t)R * (n ? n : 1) * 4) + r((size_t)R * N);
    if (solve && n > 0)
        b += r((size_t)R * n * 8) + r((size_t)R * n * n * 8) + r((size_t)R * 8) + r((size_t)R * 8) +
             r(enum_scratch_bytes(n, R));
    else if (out->h_eff && n > 0)
        b += r((size_t)R * n * 8) + r((size_t)R * n * n * 8);
    if (out->energy || out->cut) b += 2 * r((size_t)R * 8) + r(energy_part_bytes(N, R));
    return b;
}

hqa_status hqa_classify_noalloc(hqa_md *md, int32_t instance, int32_t n_amb, int32_t solve,
                                const hqa_classify_out *out, int32_t out_mem) {
    if (solve != 0 && solve != 1) return fail(HQA_EINVAL, "solve must be 0 or 1");
    hqa_status s = classify_checks(md, instance, n_amb, solve, out, nullptr);
    if (s != HQA_OK) return s;
    const size_t need = classify_scratch_bytes(md->R, md->inst[instance].N, n_amb, solve, out);
    if (need > (size_t)HQA_NOALLOC_SCRATCH_BYTES)
        return fail(HQA_EUNSUPPORTED, "read-out needs %zu bytes of scratch, above the %zu of the "
                    "fixed array", need, (size_t)HQA_NOALLOC_SCRATCH_BYTES);
    void *base = nullptr;
    if ((s = noalloc_scratch(&base)) != HQA_OK) return s;
    ScratchArena A;
    A.base = (uint8_t *)base;
    A.cap = HQA_NOALLOC_SCRATCH_BYTES;
    return classify_core(md, instance, n_amb, solve, out, out_mem, nullptr, HQA_HOST, 0, 0, A);
}

hqa_status hqa_classify_many(hqa_md *md, const int32_t *instances, int32_t count,
                             int32_t n_amb, int32_t solve, double *energy, double *cut,
                             int32_t out_mem) {
    if (!md) return fail(HQA_EINVAL, "null handle");
    if (!instances || count < 1) return fail(HQA_EINVAL, "need a list of at least one instance");
    if (!energy && !cut) return fail(HQA_EINVAL, "energy and cut are both NULL");
    if (solve != 0 && solve != 1) return fail(HQA_EINVAL, "solve must be 0 or 1");
    if (out_mem != HQA_HOST && out_mem != HQA_DEVICE) return fail(HQA_EINVAL, "bad out_mem");
    const int R = md->R;
    hqa_classify_out o{};
    o.energy = energy;          // only their presence matters to the checks and the sizing
    o.cut = cut;
    size_t need = 0;
    for (int32_t c = 0; c < count; c++) {
        hqa_status s = classify_checks(md, instances[c], n_amb, solve, &o, nullptr, false);
        if (s != HQA_OK) return s;
        need = std::max(need, classify_scratch_bytes(R, md->inst[instances[c]].N, n_amb, solve,
                                                     &o));
    }
    hqa_status s = hqa_md_sync(md);
    if (s != HQA_OK) return s;
    CallTimer tm(md->stream);
    // One launch per stage for all listed instances (select, reduce, enumerate, merge,
    // energy), each instance with a scratch region sized for the largest; the energies
    // and cuts go straight to the device outputs (or to staging for host outputs).
    const size_t res = ScratchArena::round((size_t)count * R * 8);
    const size_t argb = ScratchArena::round(readout_batch_arg_bytes(count));
    uint8_t *base = nullptr;
    HIPCHK(dev_malloc((void **)&base, (size_t)count * need + 2 * res + argb));
    double *dE = energy, *dC = cut;
    if (out_mem == HQA_HOST) {
        dE = energy ? (double *)(base + (size_t)count * need) : nullptr;
        dC = cut ? (double *)(base + (size_t)count * need + res) : nullptr;
    }
    uint8_t *argbuf = base + (size_t)count * need + 2 * res;
    std::vector<ReadoutJob> jobs(count);
    hipError_t e = hipSuccess;
    for (int32_t c = 0; c < count && e == hipSuccess; c++) {
        Instance &I = md->inst[instances[c]];
        ScratchArena A;
        A.base = base + (size_t)c * need;
        A.cap = need;
        ReadoutJob &jb = jobs[c];
        jb.I = &I;
        jb.prec = md->prec;
        jb.W = md->sch.W;
        jb.h_eff = jb.J_eff = jb.e_red = nullptr;
        jb.code = nullptr;
        jb.escr = nullptr;
        // the same carving as the one-instance read-out
        e = A.get(&jb.amb, (size_t)R * (n_amb ? n_amb : 1));
        if (e == hipSuccess) e = A.get(&jb.spins, (size_t)R * I.N);
        if (e == hipSuccess && solve && n_amb > 0) {
            e = A.get(&jb.h_eff, (size_t)R * n_amb);
            if (e == hipSuccess) e = A.get(&jb.J_eff, (size_t)R * n_amb * n_amb);
            if (e == hipSuccess) e = A.get(&jb.code, (size_t)R);
            if (e == hipSuccess) e = A.get(&jb.e_red, (size_t)R);
            uint8_t *escr = nullptr;
            if (e == hipSuccess) e = A.get(&escr, enum_scratch_bytes(n_amb, R));
            jb.escr = escr;
        }
        double *E = nullptr, *C = nullptr;
        uint8_t *part = nullptr;
        if (e == hipSuccess) e = A.get(&E, (size_t)R);
        if (e == hipSuccess) e = A.get(&C, (size_t)R);
        if (e == hipSuccess) e = A.get(&part, energy_part_bytes(I.N, R));
        jb.E = dE ? dE + (size_t)c * R : E;
        jb.C = dC ? dC + (size_t)c * R : C;
        jb.part = part;
    }
    if (e == hipSuccess)
        e = launch_readout_batch(jobs, R, n_amb, solve, argbuf, argb, md->stream);
    if (e == hipSuccess && out_mem == HQA_HOST) {
        if (energy) e = hipMemcpyAsync(energy, dE, (size_t)count * R * 8, hipMemcpyDeviceToHost,
                                       md->stream);
        if (e == hipSuccess && cut)
            e = hipMemcpyAsync(cut, dC, (size_t)count * R * 8, hipMemcpyDeviceToHost, md->stream);
    }
    // whatever happened above, the stream is drained before its memory is released
    hipError_t e2 = hipStreamSynchronize(md->stream);
    (void)hipFree(base);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return fail(dev_status(e), "read-out: %s", hipGetErrorString(e));
    const double ms = tm.stop();
    if (ms >= 0.0)
        fprintf(stderr, "hqa timing: read-out of %d instances (R = %d, n = %d, solve %d, one "
                "launch per stage): %.3f ms\n", count, R, n_amb, solve, ms);
    return HQA_OK;
}

hqa_status hqa_classify_tabu(hqa_md *md, int32_t instance, int32_t n_amb, int64_t iters,
                             int32_t tenure, const hqa_classify_out *out, int32_t out_mem) {
    if (iters < 0 || tenure < 0) return fail(HQA_EINVAL, "iters and tenure must be >= 0");
    if (n_amb > 4096) return fail(HQA_EUNSUPPORTED, "tabu search limited to n <= 4096");
    return classify_impl(md, instance, n_amb, 2, out, out_mem, nullptr, HQA_HOST, iters, tenure);
}

hqa_status hqa_classify_probs(hqa_md *md, int32_t instance, const float *prob, int32_t prob_mem,
                              int32_t n_amb, int32_t solve, const hqa_classify_out *out,
                              int32_t out_mem) {
    if (!prob) return fail(HQA_EINVAL, "prob is NULL");
    if (prob_mem != HQA_HOST && prob_mem != HQA_DEVICE) return fail(HQA_EINVAL, "bad prob_mem");
    if (solve != 0 && solve != 1) return fail(HQA_EINVAL, "solve must be 0 or 1");
    return classify_impl(md, instance, n_amb, solve, out, out_mem, prob, prob_mem);
}

hqa_status hqa_md_stats_window(hqa_md *md, int64_t k0, int64_t k1, int64_t every) {
    if (!md) return fail(HQA_EINVAL, "null handle");
    if (md->prec == HQA_PREC_F64_REF)
        return fail(HQA_EUNSUPPORTED, "early-stop statistics run on the binary32 paths");
    if (k0 < 0 || k1 <= k0 || k1 > md->sch.T) return fail(HQA_EINVAL, "need 0 <= k0 < k1 <= T");
    if (every < 1) return fail(HQA_EINVAL, "every must be >= 1");
    md->stats_every = every;
    for (auto &I : md->inst) {
        const size_t n = I.smaj ? (size_t)I.N * I.ld : (size_t)I.Rp * I.ld;
        if (!I.st) {
            HIPCHK(dalloc(&I.st, 9 * n));
            HIPCHK(dalloc(&I.n1, (size_t)I.N));
            HIPCHK(dalloc(&I.inv_n2, (size_t)I.N));
            HIPCHK(launch_row_norms(I, I.n1, I.inv_n2, md->stream));
            std::vector<float> h(I.N);
            HIPCHK(hipMemcpyAsync(h.data(), I.n1, sizeof(float) * I.N, hipMemcpyDeviceToHost,
                                  md->stream));
            HIPCHK(hipStreamSynchronize(md->stream));
            double s = 0.0;
            for (float v : h) s += v;
            I.mean_n1 = (float)(s / I.N);
        }
        HIPCHK(hipMemsetAsync(I.st, 0, sizeof(float) * 9 * n, md->stream));
    }
    md->stats_k0 = k0;
    md->stats_k1 = k1;
    return HQA_OK;
}

hqa_status hqa_md_features(hqa_md *md, int32_t instance, float *feat, int32_t dst_mem) {
    hqa_status s = check_instance(md, instance);
    if (s != HQA_OK) return s;
    if (!feat) return fail(HQA_EINVAL, "feat is NULL");
    Instance &I = md->inst[instance];
    if (!I.st) return fail(HQA_ESTATE, "no statistics window set");
    const int64_t K = stats_count(md);
    if (K < 1) return fail(HQA_ESTATE, "no step of the statistics window has run");
    const size_t n = (size_t)md->R * I.N * 12;
    float *buf = feat;
    if (dst_mem == HQA_HOST) HIPCHK(dalloc(&buf, n));
    HIPCHK(launch_features(I, md->R, K, (float)((double)md->q / (double)md->sch.T), I.mean_n1,
                           buf, md->stream));
    if (dst_mem == HQA_HOST)
        HIPCHK(hipMemcpyAsync(feat, buf, n * 4, hipMemcpyDeviceToHost, md->stream));
    HIPCHK(hipStreamSynchronize(md->stream));
    if (dst_mem == HQA_HOST) dfree(buf);
    return HQA_OK;
}

// ------------------------------------------------------------- MLP model
struct hqa_es {
    hipStream_t stream = nullptr;
    float *P = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *acc = nullptr;
    int64_t t = 0;
};

void hqa_es_destroy(hqa_es *es) {
    if (!es) return;
    (void)hipStreamSynchronize(es->stream);
    dfree(es->P); dfree(es->m); dfree(es->v); dfree(es->g); dfree(es->acc);
    delete es;
}

hqa_status hqa_es_create(uint64_t seed, void *hip_stream, hqa_es **out) {
    g_err.clear();
    if (!out) return fail(HQA_EINVAL, "out is NULL");
    *out = nullptr;
    hqa_es *es = new hqa_es();
    es->stream = (hipStream_t)hip_stream;
    hipError_t e = dalloc(&es->P, HQA_ES_NPARAM);
    if (e == hipSuccess) e = dalloc(&es->m, HQA_ES_NPARAM);
    if (e == hipSuccess) e = dalloc(&es->v, HQA_ES_NPARAM);
    if (e == hipSuccess) e = dalloc(&es->g, HQA_ES_NPARAM);
    if (e == hipSuccess) e = dalloc(&es->acc, 4);
    if (e == hipSuccess) e = hipMemsetAsync(es->m, 0, sizeof(float) * HQA_ES_NPARAM, es->stream);
    if (e == hipSuccess) e = hipMemsetAsync(es->v, 0, sizeof(float) * HQA_ES_NPARAM, es->stream);
    if (e == hipSuccess) e = launch_mlp_init(es->P, seed, es->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(es->stream);
    if (e != hipSuccess) {
        hqa_es_destroy(es);
        return fail(e == hipErrorOutOfMemory ? HQA_ENOMEM : HQA_EDEVICE, "es create: %s",
                    hipGetErrorString(e));
    }
    *out = es;
    return HQA_OK;
}

hqa_status hqa_es_params(hqa_es *es, float *params, int32_t mem, int32_t import) {
    if (!es || !params) return fail(HQA_EINVAL, "bad arguments");
    const size_t nb = sizeof(float) * HQA_ES_NPARAM;
    if (import) {
        HIPCHK(hipMemcpyAsync(es->P, params, nb, kind_in(mem), es->stream));
        HIPCHK(hipMemsetAsync(es->m, 0, nb, es->stream));
        HIPCHK(hipMemsetAsync(es->v, 0, nb, es->stream));
        es->t = 0;
    } else {
        HIPCHK(hipMemcpyAsync(params, es->P, nb, kind_out(mem), es->stream));
    }
    HIPCHK(hipStreamSynchronize(es->stream));
    return HQA_OK;
}

// Device copies of host minibatch inputs.
static hqa_status es_inputs(hqa_es *es, DevBufs &B, const float *x, const int32_t *y,
                            const float *cw, int64_t n, int32_t mem, const float **dx,
                            const int32_t **dy, const float **dcw) {
    *dx = x; *dy = y; *dcw = cw;
    if (mem == HQA_DEVICE) return HQA_OK;
    float *tx = nullptr, *tcw = nullptr;
    int32_t *ty = nullptr;
    HIPCHK(B.get(&tx, (size_t)n * 12));
    HIPCHK(hipMemcpyAsync(tx, x, sizeof(float) * n * 12, hipMemcpyHostToDevice, es->stream));
    *dx = tx;
    if (y) {
        HIPCHK(B.get(&ty, (size_t)n));
        HIPCHK(hipMemcpyAsync(ty, y, sizeof(int32_t) * n, hipMemcpyHostToDevice, es->stream));
        *dy = ty;
    }
    if (cw) {
        HIPCHK(B.get(&tcw, 3));
        HIPCHK(hipMemcpyAsync(tcw, cw, sizeof(float) * 3, hipMemcpyHostToDevice, es->stream));
        *dcw = tcw;
    }
    return HQA_OK;
}

hqa_status hqa_es_grad(hqa_es *es, const float *x, const int32_t *y, int64_t n, const float *cw,
                       float *grad, float *loss, int32_t mem) {
    if (!es || !x || !y || !cw || n < 1) return fail(HQA_EINVAL, "bad arguments");
    DevBufs B;
    const float *dx, *dcw;
    const int32_t *dy;
    hqa_status s = es_inputs(es, B, x, y, cw, n, mem, &dx, &dy, &dcw);
    if (s != HQA_OK) return s;
    HIPCHK(launch_mlp_grad(es->P, n, dx, dy, dcw, es->g, es->acc, es->stream));
    if (grad) HIPCHK(hipMemcpyAsync(grad, es->g, sizeof(float) * HQA_ES_NPARAM, kind_out(mem), es->stream));
    if (loss) HIPCHK(hipMemcpyAsync(loss, es->acc + 2, sizeof(float), kind_out(mem), es->stream));
    HIPCHK(hipStreamSynchronize(es->stream));
    return HQA_OK;
}

hqa_status hqa_es_train_step(hqa_es *es, const float *x, const int32_t *y, int64_t n,
                             const float *cw, float lr, float *loss, int32_t mem) {
    if (!es || !x || !y || !cw || n < 1 || !(lr > 0.f)) return fail(HQA_EINVAL, "bad arguments");
    DevBufs B;
    const float *dx, *dcw;
    const int32_t *dy;
    hqa_status s = es_inputs(es, B, x, y, cw, n, mem, &dx, &dy, &dcw);
    if (s != HQA_OK) return s;
    HIPCHK(launch_mlp_grad(es->P, n, dx, dy, dcw, es->g, es->acc, es->stream));
    es->t += 1;
    HIPCHK(launch_adam(es->P, es->g, es->m, es->v, es->t, lr, es->stream));
    if (loss) HIPCHK(hipMemcpyAsync(loss, es->acc + 2, sizeof(float), kind_out(mem), es->stream));
    if (mem == HQA_HOST || loss) HIPCHK(hipStreamSynchronize(es->stream));
    return HQA_OK;
}

hqa_status hqa_es_predict(hqa_es *es, const float *x, int64_t n, float *prob, int32_t bf16_infer,
                          int32_t mem) {
    if (!es || !x || !prob || n < 0) return fail(HQA_EINVAL, "bad arguments");
    DevBufs B;
    const float *dx, *dcw;
    const int32_t *dy;
    hqa_status s = es_inputs(es, B, x, nullptr, nullptr, n, mem, &dx, &dy, &dcw);
    if (s != HQA_OK) return s;
    float *dp = prob;
    if (mem == HQA_HOST) HIPCHK(B.get(&dp, (size_t)n * 3));
    HIPCHK(launch_mlp_predict(es->P, n, dx, dp, bf16_infer ? 1 : 0, es->stream));
    if (mem == HQA_HOST)
        HIPCHK(hipMemcpyAsync(prob, dp, sizeof(float) * n * 3, hipMemcpyDeviceToHost, es->stream));
    HIPCHK(hipStreamSynchronize(es->stream));
    return HQA_OK;
}

hqa_status hqa_es_confidence(hqa_es *es, const float *prob, int64_t n, int32_t mem,
                             double *mean_max) {
    if (!es || !prob || !mean_max || n < 1) return fail(HQA_EINVAL, "bad arguments");
    if (mem != HQA_HOST && mem != HQA_DEVICE) return fail(HQA_EINVAL, "bad mem");
    DevBufs B;
    const float *dp = prob;
    if (mem == HQA_HOST) {
        float *t;
        HIPCHK(B.get(&t, (size_t)n * 3));
        HIPCHK(hipMemcpyAsync(t, prob, sizeof(float) * n * 3, hipMemcpyHostToDevice, es->stream));
        dp = t;
    }
    const int blocks = 256;
    double *part;
    HIPCHK(B.get(&part, blocks));
    k_sum_maxprob<<<blocks, 256, 0, es->stream>>>(dp, n, part);
    HIPCHK(hipGetLastError());
    std::vector<double> h(blocks);
    HIPCHK(hipMemcpyAsync(h.data(), part, sizeof(double) * blocks, hipMemcpyDeviceToHost, es->stream));
    HIPCHK(hipStreamSynchronize(es->stream));
    double t = 0.0;
    for (double v : h) t += v;
    *mean_max = t / (double)n;
    return HQA_OK;
}

hqa_status hqa_md_run_es(hqa_md *md, int32_t instance, hqa_es *es, int64_t K, int64_t Ks,
                         int64_t stride, double threshold, int32_t bf16_infer, float *prob,
                         int32_t prob_mem, int64_t *stop_step, double *confidence) {
    hqa_status s = check_instance(md, instance);
    if (s != HQA_OK) return s;
    if (!es) return fail(HQA_EINVAL, "es is NULL");
    if (K < 1 || Ks < 1 || Ks > K || stride < 1)
        return fail(HQA_EINVAL, "need K >= 1, 1 <= Ks <= K and stride >= 1");
    if (prob && prob_mem != HQA_HOST && prob_mem != HQA_DEVICE) return fail(HQA_EINVAL, "bad prob_mem");
    if (md->prec == HQA_PREC_F64_REF)
        return fail(HQA_EUNSUPPORTED, "early-stop statistics run on the binary32 paths");
    if (md->q >= md->sch.T) return fail(HQA_ESTATE, "the run has already reached step T");
    const Instance &I = md->inst[instance];
    const int64_t n = (int64_t)md->R * I.N;
    DevBufs B;
    float *feat, *pd;
    HIPCHK(B.get(&feat, (size_t)n * HQA_ES_NFEAT));
    HIPCHK(B.get(&pd, (size_t)n * 3));
    const int64_t T = md->sch.T;
    int64_t q = md->q;
    double conf = 0.0;
    for (;;) {
        const int64_t nxt = std::min(q + K, T);
        const int64_t k0 = std::max(q, nxt - Ks);
        if ((s = hqa_md_run(md, k0)) != HQA_OK) return s;
        if ((s = hqa_md_stats_window(md, k0, nxt, stride)) != HQA_OK) return s;
        if ((s = hqa_md_run(md, nxt)) != HQA_OK) return s;
        q = nxt;
        if ((s = hqa_md_features(md, instance, feat, HQA_DEVICE)) != HQA_OK) return s;
        if ((s = hqa_es_predict(es, feat, n, pd, bf16_infer, HQA_DEVICE)) != HQA_OK) return s;
        if ((s = hqa_es_confidence(es, pd, n, HQA_DEVICE, &conf)) != HQA_OK) return s;
        if (conf >= threshold || q >= T) break;
    }
    if (prob)
        HIPCHK(hipMemcpy(prob, pd, sizeof(float) * n * 3,
                         prob_mem == HQA_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice));
    if (stop_step) *stop_step = q;
    if (confidence) *confidence = conf;
    return HQA_OK;
}

hqa_status hqa_ising_energy(const hqa_problem *prob, const int8_t *spins, int32_t n_vectors,
                            double *energy, double *cut, int32_t mem, void *hip_stream) {
    g_err.clear();
    if (!prob || !spins || n_vectors < 0) return fail(HQA_EINVAL, "bad arguments");
    if (mem != HQA_HOST && mem != HQA_DEVICE) return fail(HQA_EINVAL, "bad mem");
    hqa_status s = check_problem(*prob, 0);
    if (s != HQA_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    DevBufs B;
    int32_t *derr, *dstats;
    HIPCHK(B.get(&derr, 1));
    HIPCHK(B.get(&dstats, 4));
    Instance I;
    s = ingest(*prob, 0, st, derr, dstats, I);
    if (s == HQA_OK && !exact_ok(I))
        s = fail(HQA_EUNSUPPORTED, "coupling exponents span too many binades for exact sums");
    if (s != HQA_OK) { free_instance(I); return s; }
    const size_t V = (size_t)n_vectors, N = (size_t)I.N;
    int8_t *dsp = (int8_t *)spins;
    double *dE = energy, *dC = cut;
    hipError_t e = hipSuccess;
    if (mem == HQA_HOST) {
        if (e == hipSuccess) e = B.get(&dsp, V * N);
        if (e == hipSuccess) e = hipMemcpyAsync(dsp, spins, V * N, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && energy) e = B.get(&dE, V);
        if (e == hipSuccess && cut) e = B.get(&dC, V);
    }
    uint8_t *part = nullptr;
    if (e == hipSuccess) e = B.get(&part, energy_part_bytes(I.N, n_vectors));
    if (e == hipSuccess) e = launch_energy(I, n_vectors, dsp, dE, dC, part, st);
    if (e == hipSuccess && mem == HQA_HOST && energy)
        e = hipMemcpyAsync(energy, dE, V * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && mem == HQA_HOST && cut)
        e = hipMemcpyAsync(cut, dC, V * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    free_instance(I);
    if (e != hipSuccess) return fail(dev_status(e), "energy: %s", hipGetErrorString(e));
    return HQA_OK;
}

// ---------------------------------------------------------------------------
// One whole pass (reset, every step, the read-out of every instance) as one unit of
// stream work, optionally captured into a HIP graph and replayed.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t PASS_MAX_GRAPHS = 4;

struct PassGraph {
    uint64_t seed;
    int32_t n_amb, solve;
    double *E, *C;
    std::vector<int> cur0, cur1;      // flux-buffer parities before and after the pass
    hipGraphExec_t exec;
};

struct PassRes {
    uint8_t *scratch = nullptr;
    size_t cap = 0;                   // bytes per instance
    uint8_t *args = nullptr;          // the read-out's stage arguments (uploaded once per key)
    size_t argcap = 0;
    bool table = false;               // args hold the table of (tn, tsolve, tE, tC)
    int32_t tn = 0, tsolve = 0;
    double *tE = nullptr, *tC = nullptr;
    hipStream_t cap_stream = nullptr; // capture stream (the handle's stream may be the null stream)
    std::vector<PassGraph> graphs;    // least recently used first
};
}  // namespace

static void drop_pass_graphs(PassRes *pr) {
    for (auto &g : pr->graphs) (void)hipGraphExecDestroy(g.exec);
    pr->graphs.clear();
}

static void free_pass(void *p) {
    PassRes *pr = (PassRes *)p;
    if (!pr) return;
    drop_pass_graphs(pr);
    if (pr->cap_stream) (void)hipStreamDestroy(pr->cap_stream);
    dfree(pr->scratch);
    dfree(pr->args);
    delete pr;
}

// The read-out jobs of a pass: instance c's buffers carved from its scratch region in
// the order of the one-instance read-out; energies and cuts go to E, C (device).
static hipError_t pass_jobs(hqa_md *md, PassRes *pr, int32_t n_amb, int32_t solve, double *E,
                            double *C, std::vector<ReadoutJob> &jobs) {
    const int32_t count = (int32_t)md->inst.size();
    const int R = md->R;
    jobs.assign(count, ReadoutJob{});
    hipError_t e = hipSuccess;
    for (int32_t c = 0; c < count && e == hipSuccess; c++) {
        Instance &I = md->inst[c];
        ScratchArena A;
        A.base = pr->scratch + (size_t)c * pr->cap;
        A.cap = pr->cap;
        ReadoutJob &jb = jobs[c];
        jb.I = &I;
        jb.prec = md->prec;
        jb.W = md->sch.W;
        e = A.get(&jb.amb, (size_t)R * (n_amb ? n_amb : 1));
        if (e == hipSuccess) e = A.get(&jb.spins, (size_t)R * I.N);
        if (e == hipSuccess && solve && n_amb > 0) {
            e = A.get(&jb.h_eff, (size_t)R * n_amb);
            if (e == hipSuccess) e = A.get(&jb.J_eff, (size_t)R * n_amb * n_amb);
            if (e == hipSuccess) e = A.get(&jb.code, (size_t)R);
            if (e == hipSuccess) e = A.get(&jb.e_red, (size_t)R);
            uint8_t *escr = nullptr;
            if (e == hipSuccess) e = A.get(&escr, enum_scratch_bytes(n_amb, R));
            jb.escr = escr;
        }
        double *Es = nullptr, *Cs = nullptr;
        uint8_t *part = nullptr;
        if (e == hipSuccess) e = A.get(&Es, (size_t)R);
        if (e == hipSuccess) e = A.get(&Cs, (size_t)R);
        if (e == hipSuccess) e = A.get(&part, energy_part_bytes(I.N, R));
        jb.E = E ? E + (size_t)c * R : Es;
        jb.C = C ? C + (size_t)c * R : Cs;
        jb.part = part;
    }
    return e;
}

// The pass's device work on md->stream: no allocation, no memset, no synchronisation
// (the read-out's stage arguments were uploaded before).
static hqa_status enqueue_pass(hqa_md *md, PassRes *pr, uint64_t seed, int32_t n_amb,
                               int32_t solve, double *E, double *C) {
    HIPCHK(reset_core(md, seed));
    hqa_status s = run_core(md, md->sch.T, false);
    if (s != HQA_OK) return s;
    std::vector<ReadoutJob> jobs;
    HIPCHK(pass_jobs(md, pr, n_amb, solve, E, C, jobs));
    HIPCHK(launch_readout_batch(jobs, md->R, n_amb, solve, pr->args, pr->argcap, md->stream,
                                READOUT_LAUNCH));
    return HQA_OK;
}

hqa_status hqa_md_pass(hqa_md *md, uint64_t seed, int32_t n_amb, int32_t solve, double *energy,
                       double *cut, int32_t flags) {
    if (!md) return fail(HQA_EINVAL, "null handle");
    if (!energy && !cut) return fail(HQA_EINVAL, "energy and cut are both NULL");
    if (solve != 0 && solve != 1) return fail(HQA_EINVAL, "solve must be 0 or 1");
    if (flags & ~HQA_MD_GRAPH) return fail(HQA_EINVAL, "unknown flags 0x%x", flags);
    const bool graph = flags & HQA_MD_GRAPH;
    const int32_t count = (int32_t)md->inst.size();
    hqa_classify_out o{};
    o.energy = energy;
    o.cut = cut;
    size_t need = 0;
    for (int32_t c = 0; c < count; c++) {
        hqa_status s = classify_checks(md, c, n_amb, solve, &o, nullptr, false, false);
        if (s != HQA_OK) return s;
        need = std::max(need, classify_scratch_bytes(md->R, md->inst[c].N, n_amb, solve, &o));
    }
    if (graph) {
        bool batched = false, clustered = false;
        const int64_t q_saved = md->q;
        md->q = 0;
        multi_ways(md, md->sch.T, &batched, &clustered);
        md->q = q_saved;
        for (auto &I : md->inst) batched = batched && I.layout == HQA_DENSE;
        if (!batched)
            return fail(HQA_EUNSUPPORTED, "a captured pass needs every instance on the batch plan");
    }
    PassRes *pr = (PassRes *)md->pass;
    if (!pr) {
        pr = new PassRes();
        md->pass = pr;
        hipError_t e = hipStreamCreateWithFlags(&pr->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(dev_status(e), "pass stream: %s", hipGetErrorString(e));
    }
    if (need > pr->cap || !pr->args) {
        // earlier passes may still use the old buffers, and captured graphs name them
        HIPCHK(hipStreamSynchronize(md->stream));
        drop_pass_graphs(pr);
        pr->table = false;
        dfree(pr->scratch);
        pr->scratch = nullptr;
        pr->cap = 0;
        HIPCHK(dev_malloc((void **)&pr->scratch, (size_t)count * need));
        pr->cap = need;
        if (!pr->args) {
            pr->argcap = readout_batch_arg_bytes(count);
            HIPCHK(dev_malloc((void **)&pr->args, pr->argcap));
        }
    }
    if (!pr->table || pr->tn != n_amb || pr->tsolve != solve || pr->tE != energy ||
        pr->tC != cut) {
        // a new argument table: graphs captured with the old one would read it
        HIPCHK(hipStreamSynchronize(md->stream));
        drop_pass_graphs(pr);
        std::vector<ReadoutJob> jobs;
        HIPCHK(pass_jobs(md, pr, n_amb, solve, energy, cut, jobs));
        HIPCHK(launch_readout_batch(jobs, md->R, n_amb, solve, pr->args, pr->argcap, md->stream,
                                    READOUT_UPLOAD));
        pr->table = true;
        pr->tn = n_amb; pr->tsolve = solve; pr->tE = energy; pr->tC = cut;
    }
    if (!graph) return enqueue_pass(md, pr, seed, n_amb, solve, energy, cut);

    // the batch plan's tables are built (allocated and uploaded) before any capture
    hipError_t pe = launch_md_steps_batch(md, md->q, md->q, false);
    if (pe != hipSuccess) return fail(dev_status(pe), "batch plan: %s", hipGetErrorString(pe));
    std::vector<int> cur0;
    for (auto &I : md->inst) cur0.push_back(I.cur);
    for (size_t k = 0; k < pr->graphs.size(); k++) {
        PassGraph g = pr->graphs[k];
        if (g.seed == seed && g.n_amb == n_amb && g.solve == solve && g.E == energy &&
            g.C == cut && g.cur0 == cur0) {
            pr->graphs.erase(pr->graphs.begin() + k);
            pr->graphs.push_back(g);
            HIPCHK(hipGraphLaunch(g.exec, md->stream));
            for (size_t i = 0; i < md->inst.size(); i++) md->inst[i].cur = g.cur1[i];
            md->q = md->sch.T;
            return HQA_OK;
        }
    }
    // capture on the pass's own stream, with the handle pointed at it meanwhile; the
    // capture records the work without running it
    hipStream_t own = md->stream;
    const int64_t q_before = md->q;
    hipError_t e = hipStreamBeginCapture(pr->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(dev_status(e), "begin capture: %s", hipGetErrorString(e));
    md->stream = pr->cap_stream;
    hqa_status s = enqueue_pass(md, pr, seed, n_amb, solve, energy, cut);
    md->stream = own;
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(pr->cap_stream, &gr);
    hipGraphExec_t exec = nullptr;
    if (s == HQA_OK && e == hipSuccess) e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
    if (gr) (void)hipGraphDestroy(gr);
    std::vector<int> cur1;
    for (auto &I : md->inst) cur1.push_back(I.cur);
    // the capture ran nothing: the handle's host state goes back to before the pass
    for (size_t i = 0; i < md->inst.size(); i++) md->inst[i].cur = cur0[i];
    md->q = q_before;
    if (s != HQA_OK) {
        if (exec) (void)hipGraphExecDestroy(exec);
        return s;
    }
    if (e != hipSuccess) return fail(dev_status(e), "pass capture: %s", hipGetErrorString(e));
    if (pr->graphs.size() >= PASS_MAX_GRAPHS) {
        (void)hipGraphExecDestroy(pr->graphs.front().exec);
        pr->graphs.erase(pr->graphs.begin());
    }
    pr->graphs.push_back(PassGraph{seed, n_amb, solve, energy, cut, cur0, cur1, exec});
    HIPCHK(hipGraphLaunch(exec, md->stream));
    for (size_t i = 0; i < md->inst.size(); i++) md->inst[i].cur = cur1[i];
    md->q = md->sch.T;
    return HQA_OK;
}

}  // extern "C"
