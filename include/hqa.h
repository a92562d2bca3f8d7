/*
 * hqa.h -- C ABI of the HQA-MD hot path on MI355X (gfx950).
 *
 * Method: H. Irie, H. Liang, T. Doi, S. Gongyo, T. Hatsuda, "Hybrid Quantum
 * Annealing via Molecular Dynamics", arXiv:2004.03972.  The library runs the
 * classical flux dynamics of the paper (Eq. 3, the Hamilton equations and
 * the leapfrog of Methods) for many independent replicas, sorts the spins
 * into frozen and ambivalent sets by the time-averaged flux (Results,
 * "Sorting frozen and ambivalent variables"), solves the reduced n-spin
 * problem (HQA section, effective couplings) exactly by enumeration for
 * n <= 24, and scores spin vectors exactly (Eq. 1, Methods "MAX-CUT").
 *
 * Conventions
 *  - Plain C types only.  Every call returns an hqa_status; on failure the
 *    thread-local hqa_last_error() names the cause, and a handle stays usable.
 *  - Pointers tagged by a *_mem field are host (HQA_HOST) or device
 *    (HQA_DEVICE, e.g. a torch tensor's data_ptr()) memory.  Inputs are
 *    borrowed for the duration of the call; J, h, p0 and phi0 are copied at
 *    init, and the library keeps no caller pointer.  Outputs are caller-owned.
 *  - The handle owns every device buffer it allocates.  All device work is
 *    ordered on the HIP stream given at init (NULL = the null stream).
 *    hqa_md_run is asynchronous; calls that write host outputs synchronise.
 *  - Replica-indexed arrays are replica-major: x[r * N + i].
 *
 * Environment
 *  - HQA_TIMING=1 (any value but 0): hqa_md_run, hqa_classify and
 *    hqa_classify_many time their device work with HIP events on their stream,
 *    synchronise, and print one line per call to stderr ("hqa timing: ...").
 *    hqa_md_run is then synchronous.
 *  - HQA_FAULT_ALLOC=k (k >= 1): the k-th device allocation counted from the
 *    start of the latest hqa_md_init fails as out of memory, so the caller sees
 *    HQA_ENOMEM from whichever call made it (tests of the error paths; a handle
 *    that init returned stays usable after a later call fails this way).
 *  - HQA_TUNE_CACHE=path: hqa_md_tune keeps its choices in that text file, one
 *    line per tuned case (device, instance shape and storage, R, precision,
 *    tuning length), and takes a stored choice instead of timing the candidates
 *    when the case comes again.  Every plan gives bit-identical trajectories, so
 *    the file affects speed only; entries that do not fit the instance are
 *    ignored.
 *  - HQA_SPIN_LIMIT=k (k >= 0): every bounded wait of the CLUSTER plan's
 *    persistent kernels gives up after k polls instead of 2^22, read at each
 *    launch (tests of the abort path).  A wait that gives up raises the launch's
 *    abort flag, every workgroup leaves, the launch ends normally and
 *    hqa_md_sync reports HQA_EDEVICE; hqa_md_reset makes the handle usable again.
 */
#ifndef HQA_H
#define HQA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HQA_ABI_VERSION 10

typedef enum {
    HQA_OK = 0,
    HQA_EINVAL = -1,       /* bad argument; detected before any device work */
    HQA_ENOMEM = -2,       /* device or host allocation failed */
    HQA_EDEVICE = -3,      /* a HIP call failed */
    HQA_EUNSUPPORTED = -4, /* valid request outside what this build supports */
    HQA_ENONFINITE = -5,   /* a flux or momentum became NaN/Inf during the run */
    HQA_ESTATE = -6        /* call not valid in the handle's current state */
} hqa_status;

enum { HQA_DENSE = 0, HQA_CSR = 1 };
enum { HQA_HOST = 0, HQA_DEVICE = 1 };

/* Arithmetic of the MD step (field contraction + leapfrog update).
 * F64_REF  : binary64 VALU in a fixed operation order (field as an fma chain over
 *            ascending column index); bit-reproducible against any FP64 code that
 *            uses the same order.
 * F32      : J, fluxes, momenta and accumulation in binary32 (dense: FP32 MFMA).
 * BF16     : J stored in bfloat16, fluxes rounded to bfloat16 as the MFMA operand,
 *            FP32 accumulation; FP32 fluxes, momenta and update.  Dense only.
 * FP8J_BF16: J stored in FP8 e4m3 (OCP), widened to bfloat16 in registers, else as
 *            BF16.  Dense only. */
typedef enum {
    HQA_PREC_F64_REF = 0,
    HQA_PREC_F32 = 1,
    HQA_PREC_BF16 = 2,
    HQA_PREC_FP8J_BF16 = 3
} hqa_precision;

/* An Ising instance (Results, Eq. 1): H(s) = 1/2 sum_{i!=j} J_ij s_i s_j + sum_i h_i s_i.
 * J must be symmetric with a zero diagonal, all values finite.
 * Dense: j holds n*n values, row-major.  CSR: row_ptr[n+1], col[nnz] strictly
 * ascending within each row, j[nnz]; the pattern and values must be symmetric.
 * h may be NULL (no field).  A MAX-CUT graph with weights w maps to J = w, h = 0
 * (Methods, "MAX-CUT and Ising spin-glass"). */
typedef struct hqa_problem {
    int32_t n;
    int32_t layout;          /* HQA_DENSE or HQA_CSR */
    int32_t mem;             /* where j, row_ptr, col and h live */
    int32_t storage;         /* 0: J stored as the handle's precision; HQA_PREC_F32,
                                HQA_PREC_BF16 or HQA_PREC_FP8J_BF16: this dense instance's
                                own storage in a non-reference handle (a batch may mix
                                BF16 and FP8 instances) */
    const double *j;
    const int32_t *row_ptr;
    const int32_t *col;
    int64_t nnz;
    const double *h;
} hqa_problem;

/* Annealing schedule and integrator settings (Methods, "Scheduling functions for MD"
 * and "Leapfrog algorithm"):
 *   alpha(tau) = alpha_f (tau + rho1 (1-tau) + rho2 tau (tau-1)),
 *   beta(tau)  = beta_f  (tau + kappa1 (1-tau) + kappa2 tau (tau-1)),
 * tabulated at tau_k = k/(2T), k = 0..2T (integer step m at k = 2m).  T steps of
 * size 1/T; the paper identifies g with the step (r_g = delta-tau/g = 1).  V = phi^M.
 * The time average phibar takes the last W fluxes phi^(T-W+1..T) (delta = W/T).
 * frozen != 0 holds alpha, beta at tau_frozen (conservation checks only). */
typedef struct hqa_schedule {
    double alpha_f, rho1, rho2;
    double beta_f, kappa1, kappa2;
    int64_t T;
    int32_t M;               /* even, >= 2 */
    int32_t W;               /* 1 <= W <= T */
    double r_g;
    int32_t frozen;
    int32_t reserved;
    double tau_frozen;
} hqa_schedule;

/* Run options.  Initial condition (Results, "Molecular dynamics for flux variables"):
 * phi(0) = 0 and p(0) = +-1 at random, the coin for (replica r, spin i) of instance k
 * being the top bit of the SplitMix64 output function (Steele, Lea, Flood 2014) at
 * counter z = seed + (r*N + i + 1) * 0x9E3779B97F4A7C15, set = -1.  p0 / phi0, when
 * not NULL, override this: concatenated over instances, each [R][N_k] binary64. */
typedef struct hqa_md_opts {
    int32_t replicas;        /* R >= 1 */
    int32_t precision;       /* hqa_precision */
    uint64_t seed;
    const double *p0;
    const double *phi0;
    int32_t init_mem;        /* where p0 / phi0 live */
    int32_t require_exact;   /* 1: fail with HQA_EUNSUPPORTED unless every J_ij converts
                                exactly to the storage type of the precision */
    int32_t plan;            /* hqa_plan for the dense binary32 instances (below);
                                every plan gives bit-identical trajectories */
    int32_t flags;           /* 0 or HQA_MD_GRAPH (below); other bits: HQA_EINVAL */
} hqa_md_opts;

/* HQA_MD_GRAPH: hqa_md_run enqueues the BATCH plan's launches of steps [q, until_step)
 * as one HIP graph launch on the handle's stream.  The graph is captured on first use
 * (on a stream of the handle's own, so the handle's stream may be the null stream)
 * and kept per (first step, last step, flux-buffer parity), up to 8 graphs per handle,
 * least recently used dropped first; a replay runs the same kernels with the same
 * arguments as the eager launches, so trajectories are bit-identical.  It saves the
 * host the cost of one launch per step when the steps are short (small instances).
 * Other plans, and steps inside an early-stop statistics window, launch eagerly.  A
 * capture or instantiation failure is returned as HQA_EDEVICE by hqa_md_run. */
#define HQA_MD_GRAPH 1

/* Execution plans of the dense binary32 step.  All of them compute the same
 * binary32 operations in the same order (K chunk c of 32 columns feeds MFMA
 * accumulation chain c mod 4, field (a0 + a1) + (a2 + a3), then the fused
 * leapfrog), so they differ only in speed.
 *   HQA_PLAN_AUTO      the tuned plan of the instance if hqa_md_tune has run, else
 *                      STEP (BATCH for several dense instances).
 *   HQA_PLAN_STEP      one launch per MD step (any size).
 *   HQA_PLAN_CLUSTER   all steps in one cooperative launch; the workgroups of a
 *                      16-replica cluster own row blocks of J and exchange fluxes
 *                      every step through the L2 of the XCD they share (workgroup b
 *                      is assumed to run on XCD b mod 8, the dispatch order of a
 *                      single-partition MI355X).  A workgroup found on another XCD
 *                      aborts the launch, and the run (or hqa_md_sync) returns
 *                      HQA_EDEVICE naming the placement; the tuner then skips the
 *                      plan.  Every wait inside the launch is bounded.  With several
 *                      dense instances (BF16/FP8, N <= 2048), runs of up to 8
 *                      consecutive instances of one size share a launch, each cluster
 *                      on its own XCD; an instance no launch takes runs alone.
 *                      Under AUTO, a handle with several dense instances runs them as
 *                      hqa_md_tune found fastest: BATCH, these CLUSTER launches, or
 *                      each instance on its own tuned plan (BATCH until tuned).
 *   HQA_PLAN_RESIDENT  all steps in one launch; one workgroup per 16 replicas keeps
 *                      their whole state in LDS and streams J from L2 (BF16/FP8 J,
 *                      N up to 800 on a device with 160 KB of LDS per workgroup).
 *   HQA_PLAN_BATCH     one launch per MD step over tiles of 128 rows x 64 replicas
 *                      with the flux operand staged in LDS: AUTO's plan for several
 *                      dense instances; selectable for a handle whose only dense
 *                      instance has BF16 or FP8 storage (row blocks of a large
 *                      instance spread over all XCDs).
 * Sparse (CSR) binary32 instances have two plans: STEP (one launch per step) and
 * RESIDENT (all steps in one launch; one workgroup per 4 replicas keeps their fluxes
 * in LDS and each thread's couplings, momenta and window sums in registers; for
 * N <= 4096 and at most 8 couplings per row).  Both give bit-identical trajectories.
 * A plan that does not apply to an instance (too large, FP32 J, statistics window
 * live) falls back to STEP for that run; hqa_md_last_plan reports what ran. */
enum {
    HQA_PLAN_AUTO = 0,
    HQA_PLAN_STEP = 1,
    HQA_PLAN_CLUSTER = 2,
    HQA_PLAN_RESIDENT = 3,
    HQA_PLAN_BATCH = 4
};

typedef struct hqa_md hqa_md;

/* Version of this ABI (HQA_ABI_VERSION). */
int32_t hqa_abi_version(void);

/* Thread-local description of the last failure on this thread ("" if none). */
const char *hqa_last_error(void);

/* Paper defaults: (alpha_f, rho1, rho2) = (0.008, 4, 3), (beta_f, kappa1, kappa2) =
 * (0.12, 0.05, 1), M = 6, W = 100, r_g = 1, T = 50000, not frozen. */
void hqa_schedule_default(hqa_schedule *s);

/* R = 1, F32, seed 0, random p0, phi0 = 0, plan HQA_PLAN_AUTO. */
void hqa_md_opts_default(hqa_md_opts *o);

/* Validate and upload `count` instances (symmetry, zero diagonal, finite values,
 * CSR ordering, W <= T, M even, exactness when requested), build the schedule table
 * and the initial state on the device.  All instances share the schedule, R and the
 * precision.  Errors: HQA_EINVAL (bad argument or instance; nothing allocated),
 * HQA_EUNSUPPORTED (precision not available for the layout, or inexact conversion
 * under require_exact), HQA_ENOMEM, HQA_EDEVICE.  *out is NULL on failure. */
hqa_status hqa_md_init(const hqa_problem *probs, int32_t count, const hqa_schedule *sched,
                       const hqa_md_opts *opts, void *hip_stream, hqa_md **out);

/* Advance every instance to step until_step (T when negative), asynchronously: the
 * leapfrog integration of the Hamilton equations of Eq. (3) (Methods, "Leapfrog
 * algorithm", with the schedule of "Scheduling functions for MD").
 * Step q evaluates the force at phi^(q) with alpha/beta at tau = q/T, kicks p (half a
 * kick at q = 0), then drifts phi^(q+1) = phi^(q) + alpha(tau=(q+1/2)/T) p, adding
 * phi^(q+1) to the window sum when q+1 >= T-W+1.  HQA_ESTATE if until_step is before
 * the current step. */
hqa_status hqa_md_run(hqa_md *md, int64_t until_step);

/* Restart every instance from tau = 0 without re-uploading J: phi(0) = 0, p(0) = +-1
 * from the counter hash with the given seed (as at init), window sums cleared, the
 * step index set to 0 and the non-finite flag cleared.  Asynchronous; kernels only (no
 * memset), so the call may be recorded into a HIP graph. */
hqa_status hqa_md_reset(hqa_md *md, uint64_t seed);

/* Wait for queued work; HQA_ENONFINITE if any flux or momentum became non-finite. */
hqa_status hqa_md_sync(hqa_md *md);

/* Storage form the BATCH plan streams for a dense instance once the plan is built (by
 * the first batched hqa_md_run or hqa_md_pass): 0 FP32, 1 BF16, 2 FP8 e4m3, 3 one bit
 * per coupling (an FP8 instance whose couplings are all 0 or 1, such as unit-weight
 * MAX-CUT: the bits expand in registers to the FP8 path's BF16 operands, so the
 * results are the same bit for bit, from 1/8 of the coupling bytes); -1 before the plan
 * is built, for a CSR instance, a bad index or a NULL handle. */
int32_t hqa_md_batch_form(const hqa_md *md, int32_t instance);

/* The plan the last hqa_md_run used for the binary32 instances (HQA_PLAN_STEP,
 * _CLUSTER, _RESIDENT or _BATCH; the last instance's when they differ), 0 if it
 * advanced none (binary64 reference mode). */
int32_t hqa_md_last_plan(const hqa_md *md);

/* Autotuner: for every binary32 instance, time each applicable plan and tile
 * shape (dense: per-step blocks of 16 or 32 rows x 16, 32 or 64 replicas with 4 or 8
 * chunks of loads in flight, cluster, resident; sparse: per step, resident) from the
 * current state with HIP events on the handle's stream: runs of `steps` and 2 `steps`
 * MD steps, whose difference is the per-step cost without a plan's fixed per-run
 * cost.  The state is restored after each run, and the fastest is kept for
 * HQA_PLAN_AUTO.  Because the plans are bit-identical the choice never changes
 * results.  Synchronises.  HQA_EINVAL for steps < 1; HQA_ESTATE if fewer than
 * 2 `steps` steps remain before T. */
hqa_status hqa_md_tune(hqa_md *md, int32_t steps);

/* Error of the binary32 field of instance k against the binary64 field on the same
 * fluxes (the current phi^(q), widened exactly): the field the instance's precision
 * form computes (FP32, or BF16 operands with FP32 accumulation, J in its storage type)
 * against sum_j J_ij phi_j in binary64 with the input J (Results, Eq. (3) force term).
 * Writes max |u32 - u64| and max |u64| over all spins and replicas.  HQA_EUNSUPPORTED
 * for the reference mode and when one replica's binary64 fluxes (8 N bytes) do not fit
 * the workgroup LDS (N above about 19,000 with 160 KB).  Synchronises. */
hqa_status hqa_md_field_error(hqa_md *md, int32_t instance, double *max_abs_err,
                              double *max_abs_field);

/* The tuned plan of dense instance k (0 if not tuned, -1 for a bad argument); *tm, *tn
 * and *cb, if not NULL, receive the per-step block shape in row and replica tiles of
 * 16 and the K chunks per accumulation chain loaded together (0 = default); *tiled
 * receives 1 when the per-step kernel reads J from its MFMA-tiled copy. */
int32_t hqa_md_tuned_plan(const hqa_md *md, int32_t k, int32_t *tm, int32_t *tn, int32_t *cb,
                          int32_t *tiled);

/* Pin dense instance k to the per-step plan with blocks of tm row tiles (1 or 2) by
 * tn replica tiles (1, 2 or 4; 16 tn must divide the replica count padded to a
 * multiple of 16), loading cb (4 or 8) K chunks of each chain together, with the A
 * operand read from the row-major J (tiled = 0) or from an MFMA-tiled copy of it
 * (tiled = 1, BF16 and FP8 storage; the copy, N^2 storage bytes, is built on first
 * use and kept with the instance), as if the tuner had chosen it.  Same results
 * either way.  HQA_EINVAL otherwise. */
hqa_status hqa_md_set_step_tiles(hqa_md *md, int32_t k, int32_t tm, int32_t tn, int32_t cb,
                                 int32_t tiled);

/* Current step index q (fluxes are phi^(q), momenta p^(q-1/2), or p^(0) at q = 0). */
int64_t hqa_md_step_index(const hqa_md *md);

enum {
    HQA_STATE_PHI = 0,       /* phi^(q)               [R][N] */
    HQA_STATE_P = 1,         /* p^(q-1/2) (p^(0) at q = 0) */
    HQA_STATE_PHIBAR = 2,    /* window mean S/W (defined at q = T) */
    HQA_STATE_WSUM = 3,      /* window sum S */
    HQA_STATE_STATMEAN = 4   /* mean of phi^(q+1) over the steps of the statistics window
                                run so far (export only; needs hqa_md_stats_window) */
};

/* Copy state `what` of instance k out to dst ([R][N] binary64, dst_mem), or, with
 * import != 0, overwrite it from dst (checkpoint/resume; the BF16 operand copy
 * follows phi).  Synchronises. */
hqa_status hqa_md_state(hqa_md *md, int32_t instance, int32_t what, void *dst,
                        int32_t dst_mem, int32_t import);

/* Set the step index (with hqa_md_state import, resumes a checkpoint). */
hqa_status hqa_md_set_step(hqa_md *md, int64_t q);

/* Local fields u = J phi^(q) of instance k, computed by the same contraction and
 * storage precision as the MD step, written as binary64 [R][N].  Synchronises. */
hqa_status hqa_md_field(hqa_md *md, int32_t instance, double *u, int32_t dst_mem);

/* MD Hamiltonian (Eq. 3) at the current integer step q in binary64 on the GPU:
 * alpha(q) sum(p^2/2 + phi^M) + beta(q) (1/2 sum phi_i u_i + sum h_i |phi_i| phi_i),
 * with the integer-time momentum p^(q) = p^(q-1/2) - F(phi^(q))/2 and u = J phi in
 * binary64 from the binary64 couplings.  H[R].  For the drift check.  Synchronises. */
hqa_status hqa_md_hamiltonian(hqa_md *md, int32_t instance, double *H, int32_t dst_mem);

/* Read-out outputs of hqa_classify; every pointer except spins may be NULL. */
typedef struct hqa_classify_out {
    int8_t *spins;           /* [R][N] read-out spins (+1/-1) */
    int32_t *amb_idx;        /* [R][n] ambivalent spins, ascending index */
    double *energy;          /* [R] exact Ising energy of spins (correctly rounded) */
    double *cut;             /* [R] cut value sum_{i<j, s_i != s_j} J_ij, exact */
    double *h_eff;           /* [R][n] effective fields of the reduced problem */
    int64_t *code;           /* [R] winning code (bit a set: ambivalent spin a is -1) */
    double *e_reduced;       /* [R] reduced energy H'(code), correctly rounded */
} hqa_classify_out;

/* Frozen/ambivalent sort and read-out at q = T (Results, "Sorting ..."; HQA section):
 * per replica the n_amb spins with the smallest |phibar| (ties: lower index) are
 * ambivalent; every spin gets s = sgn(phibar), sgn(0) = +1 (solve = 0: the MD-alone
 * read-out).  solve = 1 also forms h_eff_a = h_a + sum_{k not in A} J_ak s_k (exact)
 * and J_eff = J[A, A], finds the exact minimum of the reduced energy over all 2^n
 * codes (ties: smallest code) and writes the merged spins.  Energies and cuts are
 * exact sums of the binary64 couplings, correctly rounded.  HQA_ESTATE before q = T,
 * HQA_EINVAL for n_amb outside [0, N] or solve outside {0, 1}, HQA_EUNSUPPORTED for
 * solve = 1 with n_amb > 24.
 * Synchronises. */
hqa_status hqa_classify(hqa_md *md, int32_t instance, int32_t n_amb, int32_t solve,
                        const hqa_classify_out *out, int32_t out_mem);

/* The read-out of hqa_classify for several instances of a handle in one call (Results,
 * "Sorting ..."; HQA section): instance instances[c], c < count, gets the operations of
 * hqa_classify with the same n_amb and solve, and its R exact energies and cuts go to
 * energy[c R .. c R + R) and cut[c R .. c R + R) (either may be NULL, not both; host or
 * device memory per out_mem).  Spins and the other outputs are not returned (hqa_classify
 * gives them per instance).  Results equal those of hqa_classify bit for bit.  Each
 * stage of the read-out (selection, reduction, enumeration, merge, energy) is one
 * launch for all listed instances, each with a scratch region sized for the largest
 * listed instance, so the small grids of single instances no longer leave the device
 * idle; the call synchronises on the handle's stream, once after uploading the stage
 * arguments and once at its end.  Errors as
 * hqa_classify, checked for every listed instance before any device work; HQA_EINVAL for
 * count < 1, a NULL list or both outputs NULL. */
hqa_status hqa_classify_many(hqa_md *md, const int32_t *instances, int32_t count,
                             int32_t n_amb, int32_t solve, double *energy, double *cut,
                             int32_t out_mem);

/* One whole pass of the method over every instance of the handle (Methods, molecular
 * dynamics from tau = 0 to 1, then the read-out of the HQA section): hqa_md_reset(seed),
 * the steps from 0 to T as hqa_md_run, then for every instance c the read-out of
 * hqa_classify_many (n_amb, solve 0 or 1) with its R exact energies and cuts written to
 * the DEVICE arrays energy[c R .. c R + R) and cut[c R .. c R + R) (either may be NULL,
 * not both).  Results equal those of that sequence of calls bit for bit.  All of it is
 * enqueued on the handle's stream (the read-out as one launch per stage for all
 * instances): nothing is synchronised and nothing is allocated, except that the first
 * call, and a call whose n_amb, solve or output arrays differ from the previous call's,
 * waits once for the handle's stream while it uploads the read-out's stage arguments
 * (the scratch, argument table and capture stream stay with the handle until
 * hqa_md_destroy; a larger read-out reallocates them).  The caller synchronises (hqa_md_sync reports a non-finite state)
 * before reading the outputs.  With flags = HQA_MD_GRAPH the pass is captured into one
 * HIP graph on its first call with these arguments (seed, n_amb, solve, energy, cut and
 * the flux-buffer parity, which an odd T flips) and replayed by later calls: a replay
 * reruns every kernel of the pass.  Up to 4 such graphs per handle, least recently used
 * dropped first.  Graph mode needs every instance dense and on the batch plan (several
 * dense instances, plan AUTO untuned or tuned to BATCH, no statistics window), else
 * HQA_EUNSUPPORTED; flags = 0 runs any handle.  Errors as hqa_classify_many, checked for
 * every instance before any device work; HQA_EINVAL for solve outside {0, 1}, unknown
 * flags or both outputs NULL. */
hqa_status hqa_md_pass(hqa_md *md, uint64_t seed, int32_t n_amb, int32_t solve, double *energy,
                       double *cut, int32_t flags);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hqa_classify with the same
 * arguments, outputs and errors, but no device allocation or release.  Its scratch
 * (ambivalent indices, read-out spins, reduced problem, enumeration and energy partial
 * results) lives in one fixed device array of HQA_NOALLOC_SCRATCH_BYTES bytes that each
 * GPU the library runs on holds until the process ends; its address is looked up at
 * the first call on a device.  A read-out that needs more (about R (N + 8 n^2) bytes)
 * returns HQA_EUNSUPPORTED before any device work.  Every call on one GPU uses that
 * GPU's array, whose contents the last call leaves behind: calls that overlap in time
 * on one GPU (other host threads, other streams) race, so serialise them.  Outputs may
 * be host or device memory (out_mem); host outputs are copied synchronously.
 * Synchronises. */
#define HQA_NOALLOC_SCRATCH_BYTES (16u << 20)
hqa_status hqa_classify_noalloc(hqa_md *md, int32_t instance, int32_t n_amb, int32_t solve,
                                const hqa_classify_out *out, int32_t out_mem);

/* Read-out at q = T as hqa_classify, with the reduced problem of the n_amb
 * ambivalent spins (HQA section: past exact enumeration the paper passes the
 * reduced problem to a tabu search) solved by a deterministic single-flip tabu
 * search that starts from the MD read-out x of those spins:
 *   f_a = h_eff_a + sum_{b != a} J_ab x_b (b ascending); D = D_best = 0;
 *   for t = 1 .. iters: d_a = -2 x_a f_a; a is allowed when tabu_until[a] < t or
 *   D + d_a < D_best; flip the allowed a* with the smallest d_a (ties: smallest a),
 *   D += d_a*, f_b -= 2 J_a*b x_a* (before the flip) for b != a*,
 *   tabu_until[a*] = t + min(tenure, n - 1); keep x whenever D < D_best.
 * Every operation is binary64 in that order (no contraction), so the result does
 * not depend on the launch.  J_ab are the instance's binary64 couplings.  The best
 * configuration is merged into spins; e_reduced receives D_best (<= 0; 0 for
 * n_amb = 0), the change of the Ising energy from the MD read-out; code is not
 * written; h_eff as hqa_classify.  HQA_EINVAL for iters or tenure < 0 or n_amb
 * outside [0, N], HQA_EUNSUPPORTED for n_amb > 4096 or for couplings and fields so
 * large (max |J|, |h| >= 2^(1020 - 2 ceil(log2(N + 1)))) that a local field or the
 * energy change could overflow binary64, HQA_ESTATE before q = T.  Synchronises. */
hqa_status hqa_classify_tabu(hqa_md *md, int32_t instance, int32_t n_amb, int64_t iters,
                             int32_t tenure, const hqa_classify_out *out, int32_t out_mem);

/* Exact Ising energy (Eq. 1) and cut (w = J) of n_vectors spin vectors [V][N] (int8,
 * +1/-1) for one instance.  energy / cut [V] (either may be NULL).  Input and outputs
 * in `mem`.  HQA_EUNSUPPORTED if the exponent spread of J and h is too wide for the
 * exact fixed-point accumulator (more than 170 binades).  Synchronises. */
hqa_status hqa_ising_energy(const hqa_problem *prob, const int8_t *spins, int32_t n_vectors,
                            double *energy, double *cut, int32_t mem, void *hip_stream);

/* Release every device buffer of the handle (NULL is accepted). */
void hqa_md_destroy(hqa_md *md);

/* ---------------------------------------------------------------------------
 * Learned early stop.  The paper has no learned component; this is the
 * library's extension: a small per-spin classifier, trained on trajectories of
 * the method itself, predicts from the first steps which spins end frozen
 * (and with which sign) and which end ambivalent, so that a run can stop early
 * and hand the predicted ambivalent spins to the exact solver.
 *
 * Statistics: for every step q in a window [k0, k1) the step epilogue adds, per
 * spin i and replica, with x = phi^(q), x' = phi^(q+1), u = (J phi^(q))_i,
 * p = p^(q+1/2), nu = u / ||J_i||_2 and sgn(0) = +1:
 *   x', x'^2, |x'|, [x' > 0], [sgn x' != sgn x], nu, nu^2, -sgn(x) nu, p^2.
 * Features at the current step q (K = min(q, k1) - k0 window steps), per replica
 * with sigma = rms_i phi^(q)_i and P = mean_i (sum p^2 / K):
 *   0 mean x'/sigma, 1 std x'/sigma, 2 mean |x'|/sigma, 3 phi^(q)/sigma,
 *   4 |2 mean[x'>0] - 1|, 5 sign-change rate, 6 mean nu/sigma, 7 std nu/sigma,
 *   8 mean(-sgn x nu)/sigma, 9 mean p^2 / P, 10 ||J_i||_1 / mean_k ||J_k||_1, 11 q/T.
 * Classifier: 12-64-64-3 perceptron with GELU x(1 + erf(x/sqrt 2))/2 and softmax
 * over {0: frozen +, 1: frozen -, 2: ambivalent}; HQA_ES_NPARAM binary32
 * parameters W1[64][12], b1[64], W2[64][64], b2[64], W3[3][64], b3[3] (row-major
 * [out][in]).  Training minimises the class-weighted cross entropy
 * sum_s w_{y_s} (-log prob_s[y_s]) / sum_s w_{y_s} with Adam (Kingma & Ba 2015;
 * b1 = 0.9, b2 = 0.999, eps = 1e-8).
 * ------------------------------------------------------------------------- */
#define HQA_ES_NFEAT 12
#define HQA_ES_NPARAM 5187

/* Collect the statistics over the steps k0, k0 + every, k0 + 2 every, ... below k1 of
 * the following runs (cleared now); the features are means over those samples.  Steps
 * of the window run on the per-step kernels.  HQA_EUNSUPPORTED for the binary64
 * reference precision; HQA_EINVAL unless 0 <= k0 < k1 <= T and every >= 1. */
hqa_status hqa_md_stats_window(hqa_md *md, int64_t k0, int64_t k1, int64_t every);

/* Features [R][N][12] (binary32) of instance k at the current step.  HQA_ESTATE if
 * no window step has run.  Synchronises. */
hqa_status hqa_md_features(hqa_md *md, int32_t instance, float *feat, int32_t dst_mem);

/* Read-out from predicted class probabilities prob [R][N][3] instead of phibar
 * (any step): s = +1 if P(frozen +) >= P(frozen -) else -1; the n_amb spins with
 * the largest P(ambivalent) (ties: lower index; compared as 1 - P in binary32) are
 * ambivalent; solve, outputs and errors as hqa_classify. */
hqa_status hqa_classify_probs(hqa_md *md, int32_t instance, const float *prob, int32_t prob_mem,
                              int32_t n_amb, int32_t solve, const hqa_classify_out *out,
                              int32_t out_mem);

typedef struct hqa_es hqa_es;

/* New classifier: weights uniform in +-1/sqrt(fan_in) from the counter hash of the
 * seed, biases 0, Adam moments 0.  All work on the given stream. */
hqa_status hqa_es_create(uint64_t seed, void *hip_stream, hqa_es **out);

/* Copy the HQA_ES_NPARAM parameters out, or in with import != 0 (which also resets
 * the Adam state).  Synchronises. */
hqa_status hqa_es_params(hqa_es *es, float *params, int32_t mem, int32_t import);

/* Gradient (HQA_ES_NPARAM) and loss of the weighted cross entropy on n samples
 * x [n][12], labels y [n] in {0,1,2}, class weights cw [3]; grad or loss may be
 * NULL.  Inputs and outputs in `mem`.  Synchronises. */
hqa_status hqa_es_grad(hqa_es *es, const float *x, const int32_t *y, int64_t n, const float *cw,
                       float *grad, float *loss, int32_t mem);

/* One Adam step on the minibatch (gradient as hqa_es_grad, learning rate lr);
 * loss (may be NULL) receives the minibatch loss before the step. */
hqa_status hqa_es_train_step(hqa_es *es, const float *x, const int32_t *y, int64_t n,
                             const float *cw, float lr, float *loss, int32_t mem);

/* Class probabilities prob [n][3] of x [n][12]; bf16_infer != 0 rounds weights and
 * layer inputs to bfloat16 (binary32 accumulation).  Synchronises. */
hqa_status hqa_es_predict(hqa_es *es, const float *x, int64_t n, float *prob, int32_t bf16_infer,
                          int32_t mem);

/* Stop-rule confidence of a prediction: the mean over the n rows of prob [n][3] of the
 * largest class probability, summed in binary64.  prob is in host or device memory
 * (mem); only the scalar comes back, so a checkpoint evaluated on device data moves
 * one number to the host.  Synchronises the handle's stream. */
hqa_status hqa_es_confidence(hqa_es *es, const float *prob, int64_t n, int32_t mem,
                             double *mean_max);

/* The stop rule of the learned early stop, run inside the library: from the current
 * step, advance every instance in checkpoints of K steps (the last one ending at T);
 * before each checkpoint collect the statistics over its last Ks steps, sampling every
 * stride-th step (hqa_md_stats_window), form the features of instance `instance`
 * (hqa_md_features), predict its class probabilities with es (BF16 inference when
 * bf16_infer != 0, hqa_es_predict) and compute their confidence (hqa_es_confidence);
 * stop at the first checkpoint whose confidence reaches `threshold`, or at T (the
 * fallback: the full run).  The last checkpoint's probabilities [R][N][3] go to prob
 * (prob_mem; may be NULL) for hqa_classify_probs; *stop_step receives the step reached
 * and *confidence its confidence (either may be NULL).  Only one number per
 * checkpoint reaches the host.  HQA_EINVAL unless K >= 1, 1 <= Ks <= K and stride >= 1;
 * HQA_EUNSUPPORTED for the binary64 reference precision; HQA_ESTATE if the run has
 * already reached T; errors of the calls above are passed on.  Synchronises. */
hqa_status hqa_md_run_es(hqa_md *md, int32_t instance, hqa_es *es, int64_t K, int64_t Ks,
                         int64_t stride, double threshold, int32_t bf16_infer, float *prob,
                         int32_t prob_mem, int64_t *stop_step, double *confidence);

void hqa_es_destroy(hqa_es *es);

#ifdef __cplusplus
}
#endif

#endif /* HQA_H */
