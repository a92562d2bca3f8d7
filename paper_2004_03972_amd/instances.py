"""Seeded synthetic Ising instances.

This module holds only random-instance recipes (no step of the method); the
tests feed the same arrays to the HIP library and to the CPU oracle.  Every
generator is deterministic in its seed (numpy PCG64 via default_rng).

Recipes follow the workloads the method is run on: Sherrington-Kirkpatrick
glasses, Erdos-Renyi MAX-CUT graphs with unit weights mapped to J = +w
(Methods, "MAX-CUT and Ising spin-glass": J_ij = w_ij, h = 0), the 3D +-J
Edwards-Anderson lattice, K_N with +-1 weights (the K2000 benchmark) and the
uniform glass J ~ U[-1,1], h ~ U[-2,2] (spin-glass benchmark section).
"""
from __future__ import annotations

import numpy as np


def _symmetrize_upper(U: np.ndarray) -> np.ndarray:
    J = np.triu(U, 1)
    return J + J.T


def sk(N: int, seed: int, std: float | None = None) -> np.ndarray:
    """Dense SK couplings, J_ij ~ Normal(0, std^2) for i<j (default std = 1/sqrt(N))."""
    rng = np.random.default_rng(seed)
    s = 1.0 / np.sqrt(N) if std is None else std
    return _symmetrize_upper(rng.standard_normal((N, N)) * s)


def er_maxcut(N: int, p: float, seed: int) -> np.ndarray:
    """Dense J of an Erdos-Renyi G(N, p) graph with unit weights, J = +w."""
    rng = np.random.default_rng(seed)
    return _symmetrize_upper((rng.random((N, N)) < p).astype(np.float64))


def pm_complete(N: int, seed: int) -> np.ndarray:
    """K_N with independent +-1 weights (the K2000 MAX-CUT benchmark for N = 2000)."""
    rng = np.random.default_rng(seed)
    return _symmetrize_upper(rng.choice(np.array([-1.0, 1.0]), size=(N, N)))


def uniform_glass(N: int, seed: int):
    """J_ij ~ U[-1, 1], h_i ~ U[-2, 2] (the spin-glass benchmark's ensemble)."""
    rng = np.random.default_rng(seed)
    J = _symmetrize_upper(rng.uniform(-1.0, 1.0, size=(N, N)))
    h = rng.uniform(-2.0, 2.0, size=N)
    return J, h


def small_int(N: int, seed: int, lo: int = -3, hi: int = 3, density: float = 1.0) -> np.ndarray:
    """Dense small-integer couplings (exact in FP8 e4m3 for |J| <= 16)."""
    rng = np.random.default_rng(seed)
    U = rng.integers(lo, hi + 1, size=(N, N)).astype(np.float64)
    U *= rng.random((N, N)) < density
    return _symmetrize_upper(U)


def ea3d(L: int, seed: int):
    """3D +-J Edwards-Anderson glass on a periodic L^3 lattice, CSR with ascending columns.

    Site i = x + L*y + L*L*z, six neighbours, one +-1 draw (p = 1/2) per bond.
    Returns (row_ptr, col, val) as int32, int32, float64.
    """
    rng = np.random.default_rng(seed)
    N = L * L * L
    idx = np.arange(N)
    x, y, z = idx % L, (idx // L) % L, idx // (L * L)
    rows, cols, vals = [], [], []
    for dx, dy, dz in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        j = ((x + dx) % L) + L * ((y + dy) % L) + L * L * ((z + dz) % L)
        v = rng.choice(np.array([-1.0, 1.0]), size=N)
        rows += [idx, j]
        cols += [j, idx]
        vals += [v, v]
    return coo_to_csr(N, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def er_sparse(N: int, d: float, seed: int):
    """Sparse ER MAX-CUT graph with mean degree d, unit weights, CSR (J = +w)."""
    rng = np.random.default_rng(seed)
    p = d / (N - 1)
    m = rng.binomial(N * (N - 1) // 2, p)
    i = rng.integers(0, N, size=int(m * 1.2) + 16)
    j = rng.integers(0, N, size=i.size)
    keep = i < j
    key = np.unique(i[keep].astype(np.int64) * N + j[keep])
    rng.shuffle(key)
    key = key[:m]
    ii, jj = key // N, key % N
    v = np.ones(ii.size)
    return coo_to_csr(N, np.concatenate([ii, jj]), np.concatenate([jj, ii]), np.concatenate([v, v]))


def coo_to_csr(N: int, rows, cols, vals):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], np.asarray(vals, dtype=np.float64)[order]
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr).astype(np.int32), cols.astype(np.int32), vals


def dense_to_csr(J: np.ndarray):
    r, c = np.nonzero(J)
    return coo_to_csr(J.shape[0], r, c, J[r, c])


def csr_to_dense(N: int, row_ptr, col, val) -> np.ndarray:
    J = np.zeros((N, N))
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    J[rows, col] = val
    return J


def random_pm1(shape, seed: int) -> np.ndarray:
    """Random +-1 array (float64), e.g. explicit initial momenta or spin vectors."""
    rng = np.random.default_rng(seed)
    return rng.choice(np.array([-1.0, 1.0]), size=shape)


def uneven_batch_specs(count: int = 512, seed: int = 4):
    """Sizes of the uneven batch: the first half Sherrington-Kirkpatrick glasses with
    N ~ U{100..2000} (couplings stored in BF16), the second half Erdos-Renyi MAX-CUT
    graphs with N ~ U{500..5000} and edge probability ~ U[0.01, 0.1] (unit weights,
    stored exactly in FP8 e4m3).  Returns [(family, N, p, instance seed)]; the
    couplings come from uneven_batch_instance."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        if k < count // 2:
            out.append(("sk", int(rng.integers(100, 2001)), 0.0, 4000 + k))
        else:
            N = int(rng.integers(500, 5001))
            out.append(("er", N, float(rng.uniform(0.01, 0.1)), 4000 + k))
    return out


def uneven_batch_instance(spec) -> np.ndarray:
    family, N, p, s = spec
    return sk(N, s) if family == "sk" else er_maxcut(N, p, s)


def stratified(specs, per_family: int = 8):
    """Indices of per_family instances of each family spread evenly over its size range
    (ranks 0, ..., count - 1 of the sizes, evenly spaced)."""
    out = []
    for fam in ("sk", "er"):
        idx = [k for k, s in enumerate(specs) if s[0] == fam]
        idx.sort(key=lambda k: (specs[k][1], k))
        m = len(idx)
        out += [idx[round(j * (m - 1) / max(1, per_family - 1))] for j in range(min(per_family, m))]
    return out
