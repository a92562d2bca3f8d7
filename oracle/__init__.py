"""FP64 CPU oracle for HQA-MD -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or executes anything in here, and
this package imports nothing from the product.

The arithmetic lives in ``hqa_oracle.c`` (plain C, binary64, built with
``-ffp-contract=off``); this module only marshals numpy arrays through ctypes.
Method: Irie et al., "Hybrid Quantum Annealing via Molecular Dynamics",
arXiv:2004.03972.  Arrays indexed by replica are replica-major, ``x[r, i]``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "hqa_oracle.c"), os.path.join(_HERE, "hqa_oracle_es.c")]
NFEAT, NPARAM = 12, 5187

# Schedule constants of the paper (Methods, "Scheduling functions for MD"):
# (alpha_f, rho1, rho2) = (0.008, 4, 3), (beta_f, kappa1, kappa2) = (0.12, 0.05, 1).
PAPER_SCHEDULE = (0.008, 4.0, 3.0, 0.12, 0.05, 1.0)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no fast-math, no fp contraction)."""
    if force or not os.path.exists(_SO) or any(
        os.path.getmtime(s) > os.path.getmtime(_SO) for s in _SRC
    ):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-pthread", "-o", tmp] + _SRC + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = C.CDLL(_SO)
        _declare(_lib)
    return _lib


class _Problem(C.Structure):
    _fields_ = [("N", C.c_int32), ("J", C.c_void_p), ("rp", C.c_void_p), ("ci", C.c_void_p),
                ("jv", C.c_void_p), ("h", C.c_void_p)]


class _MDParams(C.Structure):
    _fields_ = [("M", C.c_int32), ("r_g", C.c_double), ("T", C.c_int64), ("W", C.c_int32),
                ("alpha", C.c_void_p), ("beta", C.c_void_p)]


def _declare(L):
    P, V, i32, i64, u64, d = C.c_void_p, None, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    sigs = {
        "or_exact_sum": (d, [P, i64]),
        "or_schedule": (V, [P, i64, i32, d, P, P]),
        "or_splitmix64_at": (u64, [u64, u64]),
        "or_init_p0": (V, [u64, i32, i32, P]),
        "or_force": (V, [P, P, i64, P, P]),
        "or_md_advance": (C.c_int, [P, P, i32, P, P, P, i64, i64, i32]),
        "or_md_run": (C.c_int, [P, P, i32, P, P, P, P, P, i32]),
        "or_hmd": (V, [P, P, i32, i64, P, P, P]),
        "or_integer_p": (V, [P, P, i32, i64, P, P, P]),
        "or_classify": (C.c_int, [i32, i32, P, i32, P, P]),
        "or_enumerate_range": (C.c_int, [i32, P, P, i64, i64, P, P]),
        "or_field": (V, [P, i32, P, P]),
        "or_reduce": (C.c_int, [P, i32, i32, P, P, P, P]),
        "or_enumerate": (C.c_int, [i32, i32, P, P, P, P]),
        "or_merge": (V, [i32, i32, i32, P, P, P]),
        "or_tabu": (C.c_int, [i32, i32, P, P, P, C.c_int64, i32, P, P]),
        "or_energy": (C.c_int, [P, i32, P, P, P]),
        "or_es_features": (C.c_int, [P, P, i32, P, P, i64, i64, i64, P, P, P]),
        "or_gelu": (d, [d]),
        "or_mlp_forward": (V, [P, i64, P, P]),
        "or_mlp_loss_grad": (d, [P, i64, P, P, P, P]),
        "or_adam_step": (V, [P, P, P, P, i64, i64, d, d, d, d]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Problem:
    """Ising instance: dense J (N x N) or CSR (row_ptr, col, val), field h (or None)."""
    N: int
    J: np.ndarray | None = None
    row_ptr: np.ndarray | None = None
    col: np.ndarray | None = None
    val: np.ndarray | None = None
    h: np.ndarray | None = None

    def __post_init__(self):
        self.J = _f64(self.J)
        self.h = _f64(self.h)
        if self.row_ptr is not None:
            self.row_ptr = np.ascontiguousarray(self.row_ptr, dtype=np.int32)
            self.col = np.ascontiguousarray(self.col, dtype=np.int32)
            self.val = _f64(self.val)
        self._c = _Problem(self.N, _ptr(self.J), _ptr(self.row_ptr), _ptr(self.col),
                           _ptr(self.val), _ptr(self.h))

    @property
    def c(self):
        return C.byref(self._c)


@dataclass
class MDParams:
    T: int
    W: int = 100
    M: int = 6
    r_g: float = 1.0
    schedule: tuple = PAPER_SCHEDULE
    frozen: bool = False
    tau_fix: float = 0.0

    def __post_init__(self):
        self.alpha, self.beta = schedule(self.T, self.schedule, self.frozen, self.tau_fix)
        self._c = _MDParams(self.M, self.r_g, self.T, self.W, _ptr(self.alpha), _ptr(self.beta))

    @property
    def c(self):
        return C.byref(self._c)


def exact_sum(x) -> float:
    x = _f64(np.ravel(x))
    return lib().or_exact_sum(_ptr(x), x.size)


def schedule(T: int, prm=PAPER_SCHEDULE, frozen=False, tau_fix=0.0):
    a = np.empty(2 * T + 1)
    b = np.empty(2 * T + 1)
    p = np.asarray(prm, dtype=np.float64)
    lib().or_schedule(_ptr(p), T, int(frozen), float(tau_fix), _ptr(a), _ptr(b))
    return a, b


def splitmix64_at(seed: int, counter: int) -> int:
    return lib().or_splitmix64_at(seed, counter)


def init_p0(seed: int, N: int, R: int) -> np.ndarray:
    p = np.empty((R, N))
    lib().or_init_p0(seed, N, R, _ptr(p))
    return p


def force(pb: Problem, mp: MDParams, q: int, phi) -> np.ndarray:
    phi = _f64(phi)
    F = np.empty(pb.N)
    lib().or_force(pb.c, mp.c, q, _ptr(phi), _ptr(F))
    return F


def field(pb: Problem, phi) -> np.ndarray:
    """Local fields u = J phi [R, N] of fluxes phi [R, N] (fma chain over ascending j)."""
    phi = _f64(np.atleast_2d(phi))
    u = np.empty_like(phi)
    lib().or_field(pb.c, phi.shape[0], _ptr(phi), _ptr(u))
    return u


def md_run(pb: Problem, mp: MDParams, phi0, p0, nthreads: int = 1):
    """Returns (phibar, phi^(T), p^(T-1/2)), each [R, N]."""
    phi0, p0 = _f64(phi0), _f64(p0)
    R = phi0.shape[0]
    phibar, phiT, pT = np.empty_like(phi0), np.empty_like(phi0), np.empty_like(phi0)
    st = lib().or_md_run(pb.c, mp.c, R, _ptr(phi0), _ptr(p0), _ptr(phibar), _ptr(phiT),
                         _ptr(pT), nthreads)
    if st != 0:
        raise FloatingPointError(f"oracle MD status {st}")
    return phibar, phiT, pT


def md_advance(pb: Problem, mp: MDParams, phi, p, S, q_from: int, q_to: int, nthreads: int = 1):
    """In-place advance of (phi, p, S) arrays [R, N] from step q_from to q_to."""
    for a in (phi, p) + ((S,) if S is not None else ()):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    st = lib().or_md_advance(pb.c, mp.c, phi.shape[0], _ptr(phi), _ptr(p), _ptr(S), q_from,
                             q_to, nthreads)
    if st != 0:
        raise FloatingPointError(f"oracle MD status {st}")


def integer_p(pb: Problem, mp: MDParams, q: int, phi, p_half) -> np.ndarray:
    phi, p_half = _f64(phi), _f64(p_half)
    out = np.empty_like(phi)
    lib().or_integer_p(pb.c, mp.c, phi.shape[0], q, _ptr(phi), _ptr(p_half), _ptr(out))
    return out


def hmd(pb: Problem, mp: MDParams, q: int, phi, p_int) -> np.ndarray:
    phi, p_int = _f64(phi), _f64(p_int)
    H = np.empty(phi.shape[0])
    lib().or_hmd(pb.c, mp.c, phi.shape[0], q, _ptr(phi), _ptr(p_int), _ptr(H))
    return H


def classify(phibar, n: int):
    """Returns (amb_idx [R, n] ascending, spins int8 [R, N])."""
    phibar = _f64(phibar)
    R, N = phibar.shape
    A = np.empty((R, n), dtype=np.int32)
    s = np.empty((R, N), dtype=np.int8)
    if lib().or_classify(N, R, _ptr(phibar), n, _ptr(A), _ptr(s)) != 0:
        raise ValueError("bad n")
    return A, s


def reduce(pb: Problem, amb_idx, spins):
    amb_idx = np.ascontiguousarray(amb_idx, dtype=np.int32)
    spins = np.ascontiguousarray(spins, dtype=np.int8)
    R, n = amb_idx.shape
    he = np.empty((R, n))
    Je = np.empty((R, n, n))
    lib().or_reduce(pb.c, R, n, _ptr(amb_idx), _ptr(spins), _ptr(he), _ptr(Je))
    return he, Je


def enumerate_exact(J_eff, h_eff):
    J_eff, h_eff = _f64(J_eff), _f64(h_eff)
    R, n = h_eff.shape
    code = np.empty(R, dtype=np.int64)
    E = np.empty(R)
    if lib().or_enumerate(n, R, _ptr(J_eff), _ptr(h_eff), _ptr(code), _ptr(E)) != 0:
        raise ValueError("bad n")
    return code, E


def enumerate_exact_blocks(J_eff, h_eff, nthreads: int = 8):
    """enumerate_exact with each replica's codes split into ascending blocks scanned on
    host threads (ctypes releases the GIL).  The minimum of E' with ties to the smallest
    code is unique, so the first block holding the strictly smallest block minimum
    gives the same code and energy as one scan over all codes."""
    from concurrent.futures import ThreadPoolExecutor
    J_eff, h_eff = _f64(J_eff), _f64(h_eff)
    R, n = h_eff.shape
    total = 1 << n
    nb = max(1, min(int(nthreads) * 4, total))
    bounds = [(total * b // nb, total * (b + 1) // nb) for b in range(nb)]
    code = np.empty(R, dtype=np.int64)
    E = np.empty(R)
    for r in range(R):
        Jr, hr = np.ascontiguousarray(J_eff[r]), np.ascontiguousarray(h_eff[r])

        def scan(bd):
            c, e = np.zeros(1, np.int64), np.zeros(1)
            if lib().or_enumerate_range(n, _ptr(Jr), _ptr(hr), bd[0], bd[1], _ptr(c),
                                        _ptr(e)) != 0:
                raise ValueError("bad block")
            return int(c[0]), float(e[0])
        with ThreadPoolExecutor(max_workers=max(1, int(nthreads))) as ex:
            res = list(ex.map(scan, [b for b in bounds if b[0] < b[1]]))
        bc, be = res[0]
        for c, e in res[1:]:
            if e < be:
                bc, be = c, e
        code[r], E[r] = bc, be
    return code, E


def tabu(J_eff, h_eff, x0, iters: int, tenure: int):
    """Single-flip tabu search on each replica's reduced problem (hqa_oracle.c
    or_tabu): returns (x_best int8 [R, n], D_best [R] = E'(x_best) - E'(x0))."""
    J_eff, h_eff = _f64(J_eff), _f64(h_eff)
    R, n = h_eff.shape
    x0 = np.ascontiguousarray(x0, dtype=np.int8).reshape(R, n)
    xb = np.empty((R, n), dtype=np.int8)
    db = np.empty(R)
    if lib().or_tabu(n, R, _ptr(J_eff), _ptr(h_eff), _ptr(x0), int(iters), int(tenure),
                     _ptr(xb), _ptr(db)) != 0:
        raise ValueError("bad arguments")
    return xb, db


def merge_x(spins, amb_idx, x):
    """Write the +-1 values x [R, n] into the spins at the ambivalent positions."""
    spins = np.array(spins, dtype=np.int8, order="C")
    amb_idx = np.asarray(amb_idx)
    for r in range(spins.shape[0]):
        spins[r, amb_idx[r]] = x[r]
    return spins


def merge(spins, amb_idx, code):
    spins = np.array(spins, dtype=np.int8, order="C")
    amb_idx = np.ascontiguousarray(amb_idx, dtype=np.int32)
    code = np.ascontiguousarray(code, dtype=np.int64)
    R, N = spins.shape
    lib().or_merge(N, R, amb_idx.shape[1], _ptr(amb_idx), _ptr(code), _ptr(spins))
    return spins


def energy(pb: Problem, spins):
    """Exact (correctly rounded) Ising energy and cut value of each spin vector."""
    spins = np.ascontiguousarray(np.atleast_2d(spins), dtype=np.int8)
    V = spins.shape[0]
    E, cut = np.empty(V), np.empty(V)
    lib().or_energy(pb.c, V, _ptr(spins), _ptr(E), _ptr(cut))
    return E, cut


def hqa(pb: Problem, mp: MDParams, p0, n: int, phi0=None, nthreads: int = 1):
    """The whole method (Fig. 5 flowchart): MD, sort, reduce, exact solve, merge, score."""
    p0 = _f64(p0)
    phi0 = np.zeros_like(p0) if phi0 is None else _f64(phi0)
    phibar, phiT, pT = md_run(pb, mp, phi0, p0, nthreads)
    A, s_md = classify(phibar, n)
    he, Je = reduce(pb, A, s_md)
    code, Ered = enumerate_exact(Je, he)
    s_hqa = merge(s_md, A, code)
    E_md, C_md = energy(pb, s_md)
    E_hqa, C_hqa = energy(pb, s_hqa)
    return dict(phibar=phibar, phiT=phiT, pT=pT, amb_idx=A, spins_md=s_md, h_eff=he,
                J_eff=Je, code=code, E_reduced=Ered, spins_hqa=s_hqa, E_md=E_md, cut_md=C_md,
                E_hqa=E_hqa, cut_hqa=C_hqa)


# ----------------------------------------------------------- learned early stop
def es_features(pb: Problem, mp: MDParams, phi0, p0, K0: int, K1: int, every: int = 1):
    """Features [R, N, 12] at step K1 from statistics over the steps K0, K0 + every, ...
    below K1; also returns phi^(K1) and p^(K1-1/2)."""
    phi0, p0 = _f64(phi0), _f64(p0)
    R, N = phi0.shape
    feat = np.empty((R, N, NFEAT))
    phi, p = np.empty_like(phi0), np.empty_like(phi0)
    st = lib().or_es_features(pb.c, mp.c, R, _ptr(phi0), _ptr(p0), K0, K1, every, _ptr(feat),
                              _ptr(phi), _ptr(p))
    if st != 0:
        raise ValueError(f"or_es_features status {st}")
    return feat, phi, p


def gelu(z: float) -> float:
    return lib().or_gelu(z)


def mlp_forward(params, x):
    params, x = _f64(params), _f64(np.atleast_2d(x))
    prob = np.empty((x.shape[0], 3))
    lib().or_mlp_forward(_ptr(params), x.shape[0], _ptr(x), _ptr(prob))
    return prob


def mlp_loss_grad(params, x, y, class_w):
    params, x, cw = _f64(params), _f64(np.atleast_2d(x)), _f64(class_w)
    y = np.ascontiguousarray(y, dtype=np.int32)
    g = np.empty(NPARAM)
    loss = lib().or_mlp_loss_grad(_ptr(params), x.shape[0], _ptr(x), _ptr(y), _ptr(cw), _ptr(g))
    return loss, g


def adam_step(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update of (params, m, v) at step count t >= 1."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(grad)
    lib().or_adam_step(_ptr(params), _ptr(g), _ptr(m), _ptr(v), params.size, t, lr, b1, b2, eps)
