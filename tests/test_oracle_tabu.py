"""Pins of the oracle's single-flip tabu search (oracle or_tabu), the subproblem
solver for n beyond exact enumeration (the paper's HQA(TS1000) hands the n = 1000
ambivalent spins to a tabu search, Results, K2000 MAX-CUT).  The search is this
library's reading; what pins it is independent of its code: a hand-traced example,
exact energies of the returned configuration, 1-flip local optimality, and brute-force
optima on small instances (reached only by moves the tabu rule forces past local
minima)."""
import itertools
import os

import numpy as np
import pytest

import oracle as orc

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tabu_hand_trace.txt")


def _energy(J, h, x):
    """E'(x) = sum_{a<b} J_ab x_a x_b + sum_a h_a x_a, in exact integer arithmetic."""
    Ji = np.rint(J).astype(np.int64)
    xi = x.astype(np.int64)
    return int(np.triu(Ji, 1).dot(xi).dot(xi) + np.rint(h).astype(np.int64).dot(xi))


def _instance(n, seed, lo=-2, hi=2):
    rng = np.random.default_rng(seed)
    J = rng.integers(lo, hi + 1, (n, n)).astype(np.float64)
    J = np.triu(J, 1)
    J = J + J.T
    h = rng.integers(-3, 4, n).astype(np.float64)
    x0 = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    return J, h, x0


def test_tabu_hand_trace():
    J = np.array([[0, 1, -1], [1, 0, 2], [-1, 2, 0]], dtype=np.float64)
    h = np.array([1.0, 0.0, -1.0])
    x0 = np.ones((1, 3), dtype=np.int8)
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert rows
    for row in rows:
        iters, xb, db = int(row[0]), [int(v) for v in row[1:4]], float(row[4])
        x, d = orc.tabu(J[None], h[None], x0, iters, 1)
        assert x[0].tolist() == xb and d[0] == db
    # the brute-force minimum of this instance is the value reached
    best = min(_energy(J, h, np.array(c)) for c in itertools.product((1, -1), repeat=3))
    assert _energy(J, h, np.array([1, -1, 1])) == best == 2 - 6


@pytest.mark.parametrize("n,seed", [(5, 1), (9, 2), (16, 3), (31, 4), (64, 5)])
def test_tabu_energy_bookkeeping_and_local_optimality(n, seed):
    J, h, x0 = _instance(n, seed)
    iters = 60 * n
    x, d = orc.tabu(J[None], h[None], x0[None], iters, max(1, n // 4))
    e0, eb = _energy(J, h, x0), _energy(J, h, x[0])
    assert d[0] == eb - e0 <= 0                      # the running energy is exact
    for a in range(n):                               # no single flip improves x_best
        y = x[0].copy()
        y[a] = -y[a]
        assert _energy(J, h, y) >= eb


def _pm1_instance(n, seed):
    """Frustrated +-1 couplings (SK-like), no field, random start."""
    rng = np.random.default_rng(seed)
    J = np.where(rng.random((n, n)) < 0.5, 1.0, -1.0)
    J = np.triu(J, 1)
    J = J + J.T
    return J, np.zeros(n), np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)


@pytest.mark.parametrize("n,seed", [(10, 105), (10, 107), (12, 103), (12, 107), (14, 101),
                                    (14, 102)])
def test_tabu_reaches_brute_force_minimum(n, seed):
    """On these frustrated instances steepest descent from the same start stops in a
    local minimum above the brute-force one (tenure 0: a move back is always allowed,
    so the search cycles there); the tabu rule carries it to the minimum."""
    J, h, x0 = _pm1_instance(n, seed)
    best = min(_energy(J, h, np.array(c)) for c in itertools.product((1, -1), repeat=n))
    xs, _ = orc.tabu(J[None], h[None], x0[None], 200 * n, 0)
    assert _energy(J, h, xs[0]) > best
    x, d = orc.tabu(J[None], h[None], x0[None], 200 * n, max(2, n // 3))
    assert _energy(J, h, x[0]) == best


def test_tabu_edge_cases():
    J, h, x0 = _instance(4, 21)
    x, d = orc.tabu(J[None], h[None], x0[None], 0, 2)          # no move: the start
    assert x[0].tolist() == x0.tolist() and d[0] == 0.0
    x, d = orc.tabu(J[None], h[None], x0[None], 40, 99)        # tenure clamped to n - 1
    assert d[0] == _energy(J, h, x[0]) - _energy(J, h, x0)
    x, d = orc.tabu(np.zeros((1, 1, 1)), np.array([[2.0]]), np.ones((1, 1), dtype=np.int8), 3, 0)
    assert x[0].tolist() == [-1] and d[0] == -4.0                # one spin: flip to -sgn h
