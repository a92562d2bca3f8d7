"""Thin ctypes binding of ``include/hqa.h`` (libhqa.so).

The functions carry the C names and only marshal arguments: every step of the
method runs in the HIP library.  There is no fallback: if ``libhqa.so`` is not
built, :func:`lib` raises.  Arrays may be numpy (host memory, ``mem=HQA_HOST``)
or torch CUDA tensors (device memory via ``data_ptr()``, ``mem=HQA_DEVICE``).
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

HQA_OK, HQA_EINVAL, HQA_ENOMEM, HQA_EDEVICE = 0, -1, -2, -3
HQA_EUNSUPPORTED, HQA_ENONFINITE, HQA_ESTATE = -4, -5, -6
HQA_DENSE, HQA_CSR = 0, 1
HQA_HOST, HQA_DEVICE = 0, 1
HQA_PREC_F64_REF, HQA_PREC_F32, HQA_PREC_BF16, HQA_PREC_FP8J_BF16 = 0, 1, 2, 3
HQA_STATE_PHI, HQA_STATE_P, HQA_STATE_PHIBAR, HQA_STATE_WSUM, HQA_STATE_STATMEAN = 0, 1, 2, 3, 4
PRECISIONS = {"f64": HQA_PREC_F64_REF, "f32": HQA_PREC_F32, "bf16": HQA_PREC_BF16,
              "fp8": HQA_PREC_FP8J_BF16}

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhqa.so")
EXPORTED = ("hqa_abi_version", "hqa_last_error", "hqa_schedule_default", "hqa_md_opts_default",
            "hqa_md_init", "hqa_md_run", "hqa_md_reset", "hqa_md_sync", "hqa_md_step_index", "hqa_md_state",
            "hqa_md_set_step", "hqa_md_field", "hqa_md_hamiltonian", "hqa_classify",
            "hqa_ising_energy", "hqa_md_destroy", "hqa_md_last_plan", "hqa_md_tune",
            "hqa_md_tuned_plan", "hqa_md_set_step_tiles", "hqa_md_field_error",
            "hqa_md_stats_window", "hqa_md_features", "hqa_classify_probs", "hqa_es_create",
            "hqa_es_params", "hqa_es_grad", "hqa_es_train_step", "hqa_es_predict",
            "hqa_es_confidence", "hqa_es_destroy", "hqa_classify_tabu", "hqa_md_run_es",
            "hqa_classify_noalloc", "hqa_classify_many", "hqa_md_pass", "hqa_md_batch_form")
HQA_ES_NFEAT, HQA_ES_NPARAM = 12, 5187
HQA_NOALLOC_SCRATCH_BYTES = 16 << 20
ABI_VERSION = 10
HQA_PLAN_AUTO, HQA_PLAN_STEP, HQA_PLAN_CLUSTER, HQA_PLAN_RESIDENT, HQA_PLAN_BATCH = 0, 1, 2, 3, 4
HQA_MD_GRAPH = 1
PLANS = {"auto": HQA_PLAN_AUTO, "step": HQA_PLAN_STEP, "cluster": HQA_PLAN_CLUSTER,
         "resident": HQA_PLAN_RESIDENT, "batch": HQA_PLAN_BATCH}
PLAN_NAMES = {0: None, 1: "step", 2: "cluster", 3: "resident", 4: "batch"}


class HQAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hqa status {status}: {msg}")
        self.status = status


class hqa_problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("layout", C.c_int32), ("mem", C.c_int32),
                ("storage", C.c_int32), ("j", C.c_void_p), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("nnz", C.c_int64), ("h", C.c_void_p)]


class hqa_schedule(C.Structure):
    _fields_ = [("alpha_f", C.c_double), ("rho1", C.c_double), ("rho2", C.c_double),
                ("beta_f", C.c_double), ("kappa1", C.c_double), ("kappa2", C.c_double),
                ("T", C.c_int64), ("M", C.c_int32), ("W", C.c_int32), ("r_g", C.c_double),
                ("frozen", C.c_int32), ("reserved", C.c_int32), ("tau_frozen", C.c_double)]


class hqa_md_opts(C.Structure):
    _fields_ = [("replicas", C.c_int32), ("precision", C.c_int32), ("seed", C.c_uint64),
                ("p0", C.c_void_p), ("phi0", C.c_void_p), ("init_mem", C.c_int32),
                ("require_exact", C.c_int32), ("plan", C.c_int32),
                ("flags", C.c_int32)]


class hqa_classify_out(C.Structure):
    _fields_ = [("spins", C.c_void_p), ("amb_idx", C.c_void_p), ("energy", C.c_void_p),
                ("cut", C.c_void_p), ("h_eff", C.c_void_p), ("code", C.c_void_p),
                ("e_reduced", C.c_void_p)]


_lib = None


def lib():
    """Load libhqa.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(_LIB_PATH)
        P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.hqa_abi_version.restype = i32
        L.hqa_last_error.restype = C.c_char_p
        L.hqa_schedule_default.argtypes = [P]
        L.hqa_md_opts_default.argtypes = [P]
        L.hqa_md_init.argtypes = [P, i32, P, P, P, P]
        L.hqa_md_run.argtypes = [P, i64]
        L.hqa_md_sync.argtypes = [P]
        L.hqa_md_reset.argtypes = [P, C.c_uint64]
        L.hqa_md_step_index.argtypes = [P]
        L.hqa_md_step_index.restype = i64
        L.hqa_md_batch_form.argtypes = [P, i32]
        L.hqa_md_batch_form.restype = i32
        L.hqa_md_last_plan.argtypes = [P]
        L.hqa_md_last_plan.restype = i32
        L.hqa_md_tune.argtypes = [P, i32]
        L.hqa_md_tuned_plan.argtypes = [P, i32, P, P, P, P]
        L.hqa_md_tuned_plan.restype = i32
        L.hqa_md_set_step_tiles.argtypes = [P, i32, i32, i32, i32, i32]
        L.hqa_md_field_error.argtypes = [P, i32, P, P]
        L.hqa_es_confidence.argtypes = [P, P, i64, i32, P]
        L.hqa_md_run_es.argtypes = [P, i32, P, i64, i64, i64, C.c_double, i32, P, i32, P, P]
        L.hqa_md_state.argtypes = [P, i32, i32, P, i32, i32]
        L.hqa_md_set_step.argtypes = [P, i64]
        L.hqa_md_field.argtypes = [P, i32, P, i32]
        L.hqa_md_hamiltonian.argtypes = [P, i32, P, i32]
        L.hqa_classify.argtypes = [P, i32, i32, i32, P, i32]
        L.hqa_classify_noalloc.argtypes = [P, i32, i32, i32, P, i32]
        L.hqa_classify_many.argtypes = [P, P, i32, i32, i32, P, P, i32]
        L.hqa_md_pass.argtypes = [P, C.c_uint64, i32, i32, P, P, i32]
        L.hqa_ising_energy.argtypes = [P, P, i32, P, P, i32, P]
        L.hqa_md_destroy.argtypes = [P]
        L.hqa_md_stats_window.argtypes = [P, i64, i64, i64]
        L.hqa_md_features.argtypes = [P, i32, P, i32]
        L.hqa_classify_probs.argtypes = [P, i32, P, i32, i32, i32, P, i32]
        L.hqa_classify_tabu.argtypes = [P, i32, i32, i64, i32, P, i32]
        L.hqa_es_create.argtypes = [C.c_uint64, P, P]
        L.hqa_es_params.argtypes = [P, P, i32, i32]
        L.hqa_es_grad.argtypes = [P, P, P, i64, P, P, P, i32]
        L.hqa_es_train_step.argtypes = [P, P, P, i64, P, C.c_float, P, i32]
        L.hqa_es_predict.argtypes = [P, P, i64, P, i32, i32]
        L.hqa_es_destroy.argtypes = [P]
        for f in ("hqa_md_init", "hqa_md_run", "hqa_md_reset", "hqa_md_sync", "hqa_md_state", "hqa_md_set_step",
                  "hqa_md_field", "hqa_md_hamiltonian", "hqa_classify", "hqa_ising_energy",
                  "hqa_md_stats_window", "hqa_md_features", "hqa_classify_probs", "hqa_es_create",
                  "hqa_es_params", "hqa_es_grad", "hqa_es_train_step", "hqa_es_predict",
                  "hqa_md_tune", "hqa_md_set_step_tiles", "hqa_md_field_error",
                  "hqa_es_confidence", "hqa_classify_tabu"):
            getattr(L, f).restype = C.c_int
        if L.hqa_abi_version() != ABI_VERSION:
            raise ImportError("libhqa ABI version mismatch")
        _lib = L
    return _lib


def _check(status: int):
    if status != HQA_OK:
        raise HQAError(status, lib().hqa_last_error().decode())


def _addr(a):
    """(address, keepalive) of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None, None
    if isinstance(a, np.ndarray):
        return a.ctypes.data, a
    return a.data_ptr(), a


# ---------------------------------------------------------------- C-named calls
def hqa_abi_version() -> int:
    return lib().hqa_abi_version()


def hqa_last_error() -> str:
    return lib().hqa_last_error().decode()


def hqa_schedule_default() -> hqa_schedule:
    s = hqa_schedule()
    lib().hqa_schedule_default(C.byref(s))
    return s


def hqa_md_opts_default() -> hqa_md_opts:
    o = hqa_md_opts()
    lib().hqa_md_opts_default(C.byref(o))
    return o


def hqa_md_init(probs, sched: hqa_schedule, opts: hqa_md_opts, stream: int = 0):
    arr = (hqa_problem * len(probs))(*probs)
    h = C.c_void_p()
    _check(lib().hqa_md_init(arr, len(probs), C.byref(sched), C.byref(opts), stream or None,
                             C.byref(h)))
    return h


def hqa_md_run(md, until_step: int = -1):
    _check(lib().hqa_md_run(md, until_step))


def hqa_md_sync(md):
    _check(lib().hqa_md_sync(md))


def hqa_md_reset(md, seed: int):
    _check(lib().hqa_md_reset(md, seed))


def hqa_md_step_index(md) -> int:
    return lib().hqa_md_step_index(md)


BATCH_FORMS = {0: "f32", 1: "bf16", 2: "fp8", 3: "bit"}


def hqa_md_batch_form(md, instance: int) -> int:
    return lib().hqa_md_batch_form(md, instance)


def hqa_md_last_plan(md) -> int:
    return lib().hqa_md_last_plan(md)


def hqa_md_tune(md, steps: int):
    _check(lib().hqa_md_tune(md, steps))


def hqa_es_confidence(es, prob, n: int, mem: int) -> float:
    out = C.c_double(0.0)
    pa, _ = _addr(prob)
    _check(lib().hqa_es_confidence(es, pa, n, mem, C.byref(out)))
    return out.value


def hqa_md_run_es(md, instance: int, es, K: int, Ks: int, stride: int, threshold: float,
                  bf16_infer: int, prob, prob_mem: int) -> tuple[int, float]:
    stop, conf = C.c_int64(0), C.c_double(0.0)
    pp, _k = _addr(prob)
    _check(lib().hqa_md_run_es(md, instance, es, K, Ks, stride, threshold, bf16_infer, pp,
                               prob_mem, C.byref(stop), C.byref(conf)))
    return stop.value, conf.value


def hqa_md_field_error(md, k: int = 0) -> tuple[float, float]:
    e, r = C.c_double(0.0), C.c_double(0.0)
    _check(lib().hqa_md_field_error(md, k, C.byref(e), C.byref(r)))
    return e.value, r.value


def hqa_md_set_step_tiles(md, k: int, tm: int, tn: int, cb: int = 4, tiled: int = 0):
    _check(lib().hqa_md_set_step_tiles(md, k, tm, tn, cb, int(tiled)))


def hqa_md_tuned_plan(md, k: int = 0) -> tuple[int, int, int, int, int]:
    tm, tn, cb, tj = C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_int32(0)
    p = lib().hqa_md_tuned_plan(md, k, C.byref(tm), C.byref(tn), C.byref(cb), C.byref(tj))
    return p, tm.value, tn.value, cb.value, tj.value


def hqa_md_set_step(md, q: int):
    _check(lib().hqa_md_set_step(md, q))


def hqa_md_state(md, instance: int, what: int, dst, dst_mem: int, import_: int = 0):
    p, _k = _addr(dst)
    _check(lib().hqa_md_state(md, instance, what, p, dst_mem, import_))


def hqa_md_field(md, instance: int, u, dst_mem: int):
    p, _k = _addr(u)
    _check(lib().hqa_md_field(md, instance, p, dst_mem))


def hqa_md_hamiltonian(md, instance: int, H, dst_mem: int):
    p, _k = _addr(H)
    _check(lib().hqa_md_hamiltonian(md, instance, p, dst_mem))


def hqa_classify(md, instance: int, n_amb: int, solve: int, out: hqa_classify_out, out_mem: int):
    _check(lib().hqa_classify(md, instance, n_amb, solve, C.byref(out), out_mem))


def hqa_classify_noalloc(md, instance: int, n_amb: int, solve: int, out: hqa_classify_out,
                         out_mem: int):
    _check(lib().hqa_classify_noalloc(md, instance, n_amb, solve, C.byref(out), out_mem))


def hqa_classify_many(md, instances, count: int, n_amb: int, solve: int, energy, cut,
                      out_mem: int):
    ks, _k = _addr(instances)
    e, _e = _addr(energy)
    c, _c = _addr(cut)
    _check(lib().hqa_classify_many(md, ks, count, n_amb, solve, e, c, out_mem))


def hqa_md_pass(md, seed: int, n_amb: int, solve: int, energy, cut, flags: int):
    e, _e = _addr(energy)
    c, _c = _addr(cut)
    _check(lib().hqa_md_pass(md, seed, n_amb, solve, e, c, flags))


def hqa_classify_tabu(md, instance: int, n_amb: int, iters: int, tenure: int,
                      out: hqa_classify_out, out_mem: int):
    _check(lib().hqa_classify_tabu(md, instance, n_amb, iters, tenure, C.byref(out), out_mem))


def hqa_ising_energy(prob: hqa_problem, spins, n_vectors: int, energy, cut, mem: int,
                     stream: int = 0):
    sp, _a = _addr(spins)
    ep, _b = _addr(energy)
    cp, _c = _addr(cut)
    _check(lib().hqa_ising_energy(C.byref(prob), sp, n_vectors, ep, cp, mem, stream or None))


def hqa_md_destroy(md):
    lib().hqa_md_destroy(md)


def hqa_md_stats_window(md, k0: int, k1: int, every: int = 1):
    _check(lib().hqa_md_stats_window(md, k0, k1, every))


def hqa_md_features(md, instance: int, feat, dst_mem: int):
    p, _k = _addr(feat)
    _check(lib().hqa_md_features(md, instance, p, dst_mem))


def hqa_classify_probs(md, instance: int, prob, prob_mem: int, n_amb: int, solve: int,
                       out: hqa_classify_out, out_mem: int):
    pp, _k = _addr(prob)
    _check(lib().hqa_classify_probs(md, instance, pp, prob_mem, n_amb, solve, C.byref(out),
                                    out_mem))


def hqa_es_create(seed: int, stream: int = 0):
    h = C.c_void_p()
    _check(lib().hqa_es_create(seed, stream or None, C.byref(h)))
    return h


def hqa_es_params(es, params, mem: int, import_: int = 0):
    p, _k = _addr(params)
    _check(lib().hqa_es_params(es, p, mem, import_))


def hqa_es_grad(es, x, y, n: int, cw, grad, loss, mem: int):
    a = [_addr(v) for v in (x, y, cw, grad, loss)]
    _check(lib().hqa_es_grad(es, a[0][0], a[1][0], n, a[2][0], a[3][0], a[4][0], mem))


def hqa_es_train_step(es, x, y, n: int, cw, lr: float, loss, mem: int):
    a = [_addr(v) for v in (x, y, cw, loss)]
    _check(lib().hqa_es_train_step(es, a[0][0], a[1][0], n, a[2][0], lr, a[3][0], mem))


def hqa_es_predict(es, x, n: int, prob, bf16_infer: int, mem: int):
    a = [_addr(v) for v in (x, prob)]
    _check(lib().hqa_es_predict(es, a[0][0], n, a[1][0], bf16_infer, mem))


def hqa_es_destroy(es):
    lib().hqa_es_destroy(es)


class ES:
    """The early-stop classifier with numpy in/out (host memory)."""

    def __init__(self, seed: int = 0, stream: int = 0):
        self.h = hqa_es_create(seed, stream)

    def close(self):
        if self.h:
            hqa_es_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # a handle still open at interpreter shutdown is left to the process exit: the HIP
        # runtime may already be torn down, so no device call is made from here then
        # (the check is bound at definition: module globals are gone by that time)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    @property
    def params(self) -> np.ndarray:
        out = np.empty(HQA_ES_NPARAM, dtype=np.float32)
        hqa_es_params(self.h, out, HQA_HOST)
        return out

    @params.setter
    def params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        hqa_es_params(self.h, p, HQA_HOST, 1)

    @staticmethod
    def _xy(x, y=None, cw=None):
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, HQA_ES_NFEAT)
        y = None if y is None else np.ascontiguousarray(y, dtype=np.int32)
        cw = None if cw is None else np.ascontiguousarray(cw, dtype=np.float32)
        return x, y, cw

    def grad(self, x, y, cw):
        x, y, cw = self._xy(x, y, cw)
        g = np.empty(HQA_ES_NPARAM, dtype=np.float32)
        loss = np.empty(1, dtype=np.float32)
        hqa_es_grad(self.h, x, y, x.shape[0], cw, g, loss, HQA_HOST)
        return float(loss[0]), g

    def train_step(self, x, y, cw, lr: float) -> float:
        x, y, cw = self._xy(x, y, cw)
        loss = np.empty(1, dtype=np.float32)
        hqa_es_train_step(self.h, x, y, x.shape[0], cw, lr, loss, HQA_HOST)
        return float(loss[0])

    def predict(self, x, bf16: bool = False, out=None):
        """Class probabilities [n][3].  With a device tensor x (float32, contiguous [n][12])
        and a device tensor out ([n][3]) the call stays on the device."""
        if out is not None:
            hqa_es_predict(self.h, x, x.shape[0], out, int(bf16), HQA_DEVICE)
            return out
        x, _, _ = self._xy(x)
        prob = np.empty((x.shape[0], 3), dtype=np.float32)
        hqa_es_predict(self.h, x, x.shape[0], prob, int(bf16), HQA_HOST)
        return prob

    def confidence(self, prob) -> float:
        """Mean over rows of the largest class probability (host array or device tensor)."""
        dev = not isinstance(prob, np.ndarray)
        if not dev:
            prob = np.ascontiguousarray(prob, dtype=np.float32).reshape(-1, 3)
        return hqa_es_confidence(self.h, prob, prob.shape[0] if not dev else prob.numel() // 3,
                                 HQA_DEVICE if dev else HQA_HOST)


# ------------------------------------------------------ marshalling conveniences
class Problem:
    """Owns host copies of an instance and its hqa_problem descriptor (host memory)."""

    def __init__(self, J=None, h=None, row_ptr=None, col=None, val=None, n=None, storage=0):
        storage = PRECISIONS.get(storage, storage) if storage else 0
        if J is not None:
            self.J = np.ascontiguousarray(J, dtype=np.float64)
            N = self.J.shape[0]
            self.c = hqa_problem(N, HQA_DENSE, HQA_HOST, storage, self.J.ctypes.data, None, None,
                                 N * N, None)
        else:
            self.rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
            self.col = np.ascontiguousarray(col, dtype=np.int32)
            self.val = np.ascontiguousarray(val, dtype=np.float64)
            N = len(self.rp) - 1 if n is None else n
            self.c = hqa_problem(N, HQA_CSR, HQA_HOST, 0, self.val.ctypes.data,
                                 self.rp.ctypes.data, self.col.ctypes.data, self.val.size, None)
        self.h = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
        if self.h is not None:
            self.c.h = self.h.ctypes.data
        self.n = N


def make_schedule(T: int, W: int = 100, M: int = 6, r_g: float = 1.0, params=None,
                  frozen: bool = False, tau_frozen: float = 0.0) -> hqa_schedule:
    s = hqa_schedule_default()
    if params is not None:
        (s.alpha_f, s.rho1, s.rho2, s.beta_f, s.kappa1, s.kappa2) = params
    s.T, s.W, s.M, s.r_g, s.frozen, s.tau_frozen = T, W, M, r_g, int(frozen), tau_frozen
    return s


class MD:
    """A handle over hqa_md_* calls with numpy in/out (host memory)."""

    def __init__(self, problems, sched: hqa_schedule, replicas: int, precision="f32", seed=0,
                 p0=None, phi0=None, require_exact=False, plan="auto", stream: int = 0,
                 graph: bool = False):
        self.problems = problems if isinstance(problems, (list, tuple)) else [problems]
        o = hqa_md_opts_default()
        o.replicas = replicas
        o.precision = PRECISIONS.get(precision, precision)
        o.seed = seed
        o.require_exact = int(require_exact)
        o.plan = PLANS[plan] if isinstance(plan, str) else int(plan)
        o.flags = HQA_MD_GRAPH if graph else 0
        self._p0 = None if p0 is None else np.ascontiguousarray(p0, dtype=np.float64)
        self._phi0 = None if phi0 is None else np.ascontiguousarray(phi0, dtype=np.float64)
        o.p0 = None if self._p0 is None else self._p0.ctypes.data
        o.phi0 = None if self._phi0 is None else self._phi0.ctypes.data
        o.init_mem = HQA_HOST
        self.R = replicas
        self.T = sched.T
        self.h = hqa_md_init([p.c for p in self.problems], sched, o, stream)

    def close(self):
        if self.h:
            hqa_md_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # a handle still open at interpreter shutdown is left to the process exit: the HIP
        # runtime may already be torn down, so no device call is made from here then
        # (the check is bound at definition: module globals are gone by that time)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def run(self, until=-1):
        hqa_md_run(self.h, until)

    def sync(self):
        hqa_md_sync(self.h)

    def reset(self, seed: int):
        hqa_md_reset(self.h, seed)

    @property
    def step(self) -> int:
        return hqa_md_step_index(self.h)

    def batch_form(self, k: int = 0):
        """Storage form the batch plan streams for instance k ("f32", "bf16", "fp8" or
        "bit"), or None before the plan is built."""
        return BATCH_FORMS.get(hqa_md_batch_form(self.h, k))

    @property
    def last_plan(self):
        """'step', 'cluster', 'resident' or 'batch' (None if no dense binary32 instance ran)."""
        return PLAN_NAMES[hqa_md_last_plan(self.h)]

    def tune(self, steps: int = 20):
        """Time every bit-identical plan from the current state and keep the fastest."""
        hqa_md_tune(self.h, steps)

    def run_es(self, es, K: int, Ks: int, stride: int, threshold: float, k: int = 0,
               bf16: bool = True, prob=None) -> tuple[int, float]:
        """The learned early stop's checkpoint loop (hqa_md_run_es): returns (stop step,
        confidence); the last checkpoint's probabilities go to `prob` (a device tensor
        [R*N][3] or a host array [R][N][3]) when given."""
        mem = HQA_HOST if prob is None or isinstance(prob, np.ndarray) else HQA_DEVICE
        return hqa_md_run_es(self.h, k, es.h, K, Ks, stride, threshold, int(bf16), prob, mem)

    def field_error(self, k: int = 0) -> tuple[float, float]:
        """(max |u32 - u64|, max |u64|) of instance k's field on the current fluxes."""
        return hqa_md_field_error(self.h, k)

    def set_step_tiles(self, tm: int, tn: int, cb: int = 4, k: int = 0, tiled: bool = False):
        """Pin instance k to per-step blocks of tm x tn tiles of 16 (rows x replicas)
        with cb chunks of each accumulation chain loaded together, J read from its
        MFMA-tiled copy when tiled (BF16 / FP8 storage)."""
        hqa_md_set_step_tiles(self.h, k, tm, tn, cb, tiled)

    def tuned_plan(self, k: int = 0):
        """(plan, row tiles, replica tiles, chunks in flight, tiled J) chosen by tune() for k."""
        p, tm, tn, cb, tj = hqa_md_tuned_plan(self.h, k)
        return PLAN_NAMES.get(p), tm, tn, cb, tj

    def state(self, what: int, k: int = 0) -> np.ndarray:
        out = np.empty((self.R, self.problems[k].n))
        hqa_md_state(self.h, k, what, out, HQA_HOST)
        return out

    def set_state(self, what: int, x, k: int = 0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        hqa_md_state(self.h, k, what, x, HQA_HOST, 1)

    def field(self, k: int = 0) -> np.ndarray:
        out = np.empty((self.R, self.problems[k].n))
        hqa_md_field(self.h, k, out, HQA_HOST)
        return out

    def hamiltonian(self, k: int = 0) -> np.ndarray:
        out = np.empty(self.R)
        hqa_md_hamiltonian(self.h, k, out, HQA_HOST)
        return out

    def stats_window(self, k0: int, k1: int, every: int = 1):
        """Statistics over the steps k0, k0 + every, ... below k1 of the following runs."""
        hqa_md_stats_window(self.h, k0, k1, every)

    def features(self, k: int = 0, out=None):
        """Features [R][N][12]; into a device tensor `out` when given (no host copy)."""
        if out is not None:
            hqa_md_features(self.h, k, out, HQA_DEVICE)
            return out
        out = np.empty((self.R, self.problems[k].n, HQA_ES_NFEAT), dtype=np.float32)
        hqa_md_features(self.h, k, out, HQA_HOST)
        return out

    def _classify_out(self, n_amb: int, k: int):
        N, R = self.problems[k].n, self.R
        res = dict(spins=np.empty((R, N), dtype=np.int8),
                   amb_idx=np.empty((R, max(n_amb, 1)), dtype=np.int32),
                   energy=np.empty(R), cut=np.empty(R),
                   h_eff=np.empty((R, max(n_amb, 1))), code=np.full(R, -1, dtype=np.int64),
                   e_reduced=np.full(R, np.nan))
        o = hqa_classify_out(*(res[f].ctypes.data for f in
                               ("spins", "amb_idx", "energy", "cut", "h_eff", "code", "e_reduced")))
        return res, o

    def classify_tabu(self, n_amb: int, iters: int, tenure: int, k: int = 0) -> dict:
        """Read-out with the reduced problem solved by the tabu search; e_reduced holds
        the best energy change D_best relative to the MD read-out."""
        res, o = self._classify_out(n_amb, k)
        hqa_classify_tabu(self.h, k, n_amb, iters, tenure, o, HQA_HOST)
        res["amb_idx"] = res["amb_idx"][:, :n_amb]
        res["h_eff"] = res["h_eff"][:, :n_amb]
        return res

    def classify(self, n_amb: int, solve: bool = False, k: int = 0, prob=None) -> dict:
        res, o = self._classify_out(n_amb, k)
        if prob is None:
            hqa_classify(self.h, k, n_amb, int(solve), o, HQA_HOST)
        elif not isinstance(prob, np.ndarray) and hasattr(prob, "data_ptr"):
            hqa_classify_probs(self.h, k, prob, HQA_DEVICE, n_amb, int(solve), o, HQA_HOST)
        else:
            prob = np.ascontiguousarray(prob, dtype=np.float32)
            hqa_classify_probs(self.h, k, prob, HQA_HOST, n_amb, int(solve), o, HQA_HOST)
        res["amb_idx"] = res["amb_idx"][:, :n_amb]
        res["h_eff"] = res["h_eff"][:, :n_amb]
        return res


    def run_pass(self, seed: int, n_amb: int, solve: bool = True, graph: bool = True,
                 energy=None, cut=None):
        """One whole pass (reset with `seed`, every MD step, the read-out of every instance)
        enqueued on the handle's stream (hqa_md_pass), replayed from a captured HIP graph
        when `graph`.  Returns the device tensors (energy, cut) [count][R] float64, filled
        once the stream has reached them (call sync() before reading)."""
        import torch
        shape = (len(self.problems), self.R)
        if energy is None:
            energy = torch.empty(shape, dtype=torch.float64, device="cuda")
        if cut is None:
            cut = torch.empty(shape, dtype=torch.float64, device="cuda")
        hqa_md_pass(self.h, seed, n_amb, int(solve), energy, cut, HQA_MD_GRAPH if graph else 0)
        return energy, cut

    def classify_many(self, n_amb: int, solve: bool = True, instances=None):
        """Exact energies and cuts [count][R] of the read-out of several instances
        (default: all) in one call (hqa_classify_many)."""
        ks = np.arange(len(self.problems), dtype=np.int32) if instances is None else \
            np.ascontiguousarray(instances, dtype=np.int32)
        E = np.empty((ks.size, self.R))
        Cc = np.empty((ks.size, self.R))
        hqa_classify_many(self.h, ks, ks.size, n_amb, int(solve), E, Cc, HQA_HOST)
        return E, Cc


def ising_energy(problem: Problem, spins) -> tuple[np.ndarray, np.ndarray]:
    spins = np.ascontiguousarray(np.atleast_2d(spins), dtype=np.int8)
    V = spins.shape[0]
    E, cut = np.empty(V), np.empty(V)
    hqa_ising_energy(problem.c, spins, V, E, cut, HQA_HOST)
    return E, cut
