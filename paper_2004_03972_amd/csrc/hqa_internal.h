// hqa_internal.h -- device buffers, kernel argument blocks and launchers shared
// by the HIP translation units of libhqa.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/hqa.h"

namespace hqa {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// Storage type of J for the fast paths.
// JT_BIT: couplings that are all 0 or 1, streamed by the batch plan as one bit each
// (its MFMA operands are the FP8 path's, so results are identical)
enum JType { JT_F32 = 0, JT_BF16 = 1, JT_FP8 = 2, JT_BIT = 3 };

// Error bits raised by kernels into a device word.
enum {
    ERR_NONFINITE = 1,      // flux or momentum became NaN/Inf
    ERR_ASYM = 2,           // J not symmetric
    ERR_DIAG = 4,           // nonzero diagonal
    ERR_NOTFINITE_IN = 8,   // non-finite coupling or field
    ERR_INEXACT = 16,       // J does not convert exactly to the storage type
    ERR_CSR_ORDER = 32,     // CSR columns not strictly ascending / out of range
    ERR_FP8_SUBNORMAL = 64, // J value whose e4m3 code would be subnormal
    ERR_BARRIER = 128,      // persistent-kernel barrier wait exceeded its bound
    ERR_PLACEMENT = 256,    // persistent-kernel workgroup not on the XCD its cluster assumes
};

// Exponent statistics of an instance for the exact accumulator:
// lsb = lowest set-bit exponent over nonzero inputs, msb = highest bit exponent.
struct ExpStats {
    int lsb;
    int msb;
};

struct Instance {
    int32_t N = 0;
    int32_t layout = HQA_DENSE;
    int64_t nnz = 0;
    int32_t Np = 0;           // dense fast paths: N padded to a multiple of 128
    int32_t Rp = 0;           // replicas padded to a multiple of 16
    bool smaj = false;        // state layout [N][R] (CSR fast path) else [R][ld]
    int32_t ld = 0;           // leading dimension of replica-major state
    bool has_h = false;

    // binary64 copies of the input (every precision keeps them: reduce, energy,
    // drift check and the reference mode read them)
    double *J64 = nullptr;    // dense N*N or CSR values
    int32_t *rp = nullptr, *ci = nullptr;
    double *h64 = nullptr;    // N (zeros when no field)
    float *h32 = nullptr;     // N (or Np)

    JType jt = JT_F32;        // storage type of Js
    void *Js = nullptr;       // dense storage for the fast paths, Np*Np of JType
    void *Jt = nullptr;       // MFMA-tiled copy of Js for the resident plan (built on first use)
    void *Jbits = nullptr;    // 1-bit tiled copy when every coupling is 0 or 1 (batch plan)
    int jbits = 0;            // 0 not checked, 1 Jbits built, -1 some coupling is not 0 or 1
    float *v32 = nullptr;     // CSR FP32 values

    // state
    double *phi64[2] = {nullptr, nullptr};
    double *p64 = nullptr, *S64 = nullptr;
    float *phi32[2] = {nullptr, nullptr};
    float *p32 = nullptr, *S32 = nullptr;
    bf16 *phib[2] = {nullptr, nullptr};
    int cur = 0;              // phi[cur] holds phi^(q)
    void *xch = nullptr;      // persistent-kernel exchange buffers (tagged words)
    size_t xch_bytes = 0;
    // learned early stop: nine statistics arrays (state layout), row norms
    float *st = nullptr;
    float *n1 = nullptr, *inv_n2 = nullptr;
    float mean_n1 = 0.f;

    ExpStats es{0, 0};
    bool j_integral = false;  // every J and h is an integer
    bool js_exact = false;    // dense: Js holds every coupling exactly
    // dense binary32 plan chosen by the tuner (0: not tuned) and its per-step tile width
    int32_t tuned_plan = 0;
    int32_t step_tn = 0;      // replica tiles of 16 per per-step block (0: widest that divides Rp)
    int32_t step_tm = 0;      // row tiles of 16 per per-step block (0: 2)
    int32_t step_cb = 0;      // chunks per chain loaded together (0: 4)
    int32_t step_tj = 0;      // per-step A fragments from the MFMA-tiled J (BF16 / FP8)
    int32_t max_deg = -1;     // CSR: largest row degree (computed on first need)
};

struct Schedule64 {
    double prm[6];
    int64_t T;
    int32_t M, W;
    double r_g;
    int32_t frozen;
    double tau_frozen;
};

}  // namespace hqa

struct hqa_md {
    hipStream_t stream = nullptr;
    int32_t R = 1;
    int32_t prec = HQA_PREC_F32;
    int32_t plan = HQA_PLAN_AUTO;            // requested plan of the dense binary32 step
    int32_t max_lds = 65536;                 // LDS bytes per workgroup on the device
    hqa::Schedule64 sch{};
    int64_t q = 0;
    std::vector<hqa::Instance> inst;
    double *a64 = nullptr, *b64 = nullptr;   // schedule tables [2T+1]
    float *a32 = nullptr, *b32 = nullptr;
    int32_t *err = nullptr;                  // device error word
    int32_t *scratch_i = nullptr;            // small device scratch (ints)
    int32_t *bar = nullptr;                  // persistent-launch barrier counters + abort flag
    hqa::JType jt = hqa::JT_F32;
    int last_plan = 0;                       // plan the last run used (HQA_PLAN_*)
    int multi_plan = 0;                      // tuned way to run several dense instances:
                                             // BATCH, CLUSTER, or STEP (each on its own plan)
    void *batch = nullptr;                   // device tile tables of a multi-instance batch
                                             // and its captured step graphs
    int32_t flags = 0;                       // HQA_MD_* run flags
    void *pass = nullptr;                    // read-out scratch, side streams and captured
                                             // graphs of hqa_md_pass
    int64_t stats_k0 = 0, stats_k1 = 0;      // early-stop statistics window [k0, k1)
    int64_t stats_every = 1;                 // ... sampling steps k0, k0 + every, ...
};

namespace hqa {

// ---- kernel launchers (each returns hipGetLastError of the launch) ----------
hipError_t launch_schedule(const Schedule64 &s, double *a64, double *b64, float *a32, float *b32,
                           hipStream_t st);
hipError_t launch_validate_dense(const double *J, const double *h, int N, int32_t *err,
                                 int32_t *stats, hipStream_t st);
hipError_t launch_validate_csr(const int32_t *rp, const int32_t *ci, const double *v,
                               const double *h, int N, int32_t *err, int32_t *stats,
                               hipStream_t st);
hipError_t launch_convert_dense(const double *J, int N, int Np, JType jt, void *out,
                                int32_t *err, hipStream_t st);
hipError_t launch_convert_csr(const double *v, int64_t nnz, float *out, int32_t *err,
                              hipStream_t st);
hipError_t launch_convert_h(const double *h, int N, float *out, hipStream_t st);
hipError_t launch_init_state(const Instance &I, int R, int prec, uint64_t seed,
                             const double *p0, const double *phi0, hipStream_t st);
hipError_t launch_export(const Instance &I, int R, int prec, int what, double *dst,
                         int import, int W, hipStream_t st);

// MD steps: advance from step q to q + nsteps
hipError_t launch_md_steps(hqa_md *md, Instance &I, int64_t q0, int64_t q1);
size_t resident_lds_bytes(int N);
bool resident_fits(const Instance &I, int max_lds);
hipError_t launch_md_resident(hqa_md *md, Instance &I, int64_t q0, int64_t q1);
hipError_t ensure_tiled_j(Instance &I, hipStream_t st);
hipError_t ensure_tiled_bits(Instance &I, hipStream_t st);
int batch_form(const hqa_md *md, int instance);
bool csr_resident_fits(hqa_md *md, Instance &I);
hipError_t launch_md_csr_resident(hqa_md *md, Instance &I, int64_t q0, int64_t q1);
hipError_t launch_field(hqa_md *md, Instance &I, double *u, hipStream_t st);
hipError_t launch_hamiltonian(hqa_md *md, Instance &I, double *H, hipStream_t st);

// read-out
hipError_t launch_select(const Instance &I, int R, int prec, int W, int n, int32_t *amb,
                         int8_t *spins, hipStream_t st);
hipError_t launch_reduce(const Instance &I, int R, int n, const int32_t *amb,
                         const int8_t *spins, double *h_eff, double *J_eff, hipStream_t st);
hipError_t launch_tabu(const Instance &I, int R, int n, const int32_t *amb, const int8_t *spins,
                       const double *h_eff, int64_t iters, int tenure, int8_t *spins_out,
                       double *d_best, hipStream_t st);
hipError_t launch_enumerate(int n, int R, const double *J_eff, const double *h_eff, int b0,
                            int integral, int64_t *code, double *e_red, void *scratch,
                            hipStream_t st);
size_t enum_scratch_bytes(int n, int R);
hipError_t launch_merge(int N, int R, int n, const int32_t *amb, const int64_t *code,
                        int8_t *spins, hipStream_t st);
// Every device allocation of the library goes through dev_malloc.  With HQA_FAULT_ALLOC=k
// in the environment, the k-th allocation counted from the start of the latest
// hqa_md_init (from 1) fails as out of memory (tests of the error paths).
hipError_t dev_malloc(void **p, size_t bytes);
void fault_alloc_arm();

// Exact energies and cuts of V spin vectors; `part` holds energy_part_bytes(N, V)
// bytes of device scratch for the per-slice partial sums.
int energy_slices(int N, int V);
size_t energy_part_bytes(int N, int V);
// One instance's part of a batched read-out: its buffers in device scratch.
struct ReadoutJob {
    const Instance *I;
    int prec, W;
    int32_t *amb;
    int8_t *spins;
    double *h_eff, *J_eff;
    int64_t *code;
    double *e_red;
    void *escr;
    double *E, *C;
    void *part;
};
size_t readout_batch_arg_bytes(int count);
// mode: READOUT_ALL uploads the stage arguments (and waits for the upload) and launches;
// READOUT_UPLOAD only uploads; READOUT_LAUNCH only launches, from a table an earlier call
// with the same jobs uploaded (no copy, no wait: such a launch may be recorded in a graph)
enum { READOUT_ALL = 0, READOUT_UPLOAD = 1, READOUT_LAUNCH = 2 };
hipError_t launch_readout_batch(const std::vector<ReadoutJob> &jobs, int R, int n, int solve,
                                void *argbuf, size_t argcap, hipStream_t st, int mode = READOUT_ALL);
hipError_t launch_energy(const Instance &I, int V, const int8_t *spins, double *E, double *cut,
                         void *part, hipStream_t st);
hipError_t launch_select_keys(int N, int R, const float *keys, int n, int32_t *amb,
                              int8_t *spins, hipStream_t st);

// learned early stop
hipError_t launch_row_norms(const Instance &I, float *n1, float *inv_n2, hipStream_t st);
hipError_t launch_features(const Instance &I, int R, int64_t K, float tau, float mean_n1,
                           float *feat, hipStream_t st);
hipError_t launch_mlp_init(float *P, uint64_t seed, hipStream_t st);
hipError_t launch_mlp_predict(const float *P, int64_t B, const float *x, float *prob, int bf,
                              hipStream_t st);
hipError_t launch_mlp_grad(const float *P, int64_t B, const float *x, const int32_t *y,
                           const float *cw, float *grad, float *acc, hipStream_t st);
hipError_t launch_adam(float *P, const float *g, float *m, float *v, int64_t t, float lr,
                       hipStream_t st);
hipError_t launch_probs_to_keys(int64_t n, const float *prob, int8_t *spins, float *key,
                                hipStream_t st);

}  // namespace hqa

// Whether MD step q accumulates early-stop statistics.
inline bool stats_step(const hqa_md *md, int64_t q) {
    return q >= md->stats_k0 && q < md->stats_k1 && (q - md->stats_k0) % md->stats_every == 0;
}

// Number of statistics samples taken by the steps run so far.
inline int64_t stats_count(const hqa_md *md) {
    const int64_t m = std::min(md->q, md->stats_k1) - md->stats_k0;
    return m <= 0 ? 0 : (m + md->stats_every - 1) / md->stats_every;
}
