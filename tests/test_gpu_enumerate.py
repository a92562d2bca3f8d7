"""Exact solution of the reduced n-spin problem (Results, "Hybrid Quantum Annealing via
Molecular Dynamics": the ambivalent spins are solved with the frozen ones fixed) on
integer instances, through hqa_classify: every launch shape of the integer kernel
(low bits walked per thread NL = n - 10 for n > 10, else 0, up to n = 24), small-integer
couplings with many equal energies, a guaranteed tie (all spins ambivalent and h = 0,
so a configuration and its mirror are both optimal: the smaller code must win), and
sums too large for the int32 walk (the int64 walk).  The minimising code and the
reduced energy must equal the oracle's brute force over all 2^n codes."""
import numpy as np
import pytest

import oracle as orc
from paper_2004_03972_amd import instances as inst

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    from paper_2004_03972_amd import hqa
    hqa.lib()
    return hqa


def _solve(H, J, n, R, seed, h=None):
    """Classify a chosen mean flux (imported as the window sum) and solve exactly."""
    N = J.shape[0]
    T, W = 200, 50
    md = H.MD(H.Problem(J, h=h), H.make_schedule(T, W), R, "f32", seed=1)
    rng = np.random.default_rng(seed)
    md.set_state(H.HQA_STATE_WSUM, rng.standard_normal((R, N)) * W)
    H.hqa_md_set_step(md.h, T)
    g = md.classify(n, solve=True)
    bar = md.state(H.HQA_STATE_PHIBAR)
    md.close()
    pb = orc.Problem(N, J=J, h=h)
    A, s = orc.classify(bar, n)
    he, Je = orc.reduce(pb, A, s)
    code, Ered = orc.enumerate_exact(Je, he)
    assert np.array_equal(g["amb_idx"], A) and np.array_equal(g["h_eff"], he)
    assert np.array_equal(g["code"], code), (g["code"], code)
    assert np.array_equal(g["e_reduced"], Ered)
    assert np.array_equal(g["spins"], orc.merge(s, A, code))
    return code


@pytest.mark.parametrize("n,R", [(1, 8), (3, 8), (7, 8), (10, 8), (11, 8), (12, 6), (13, 6),
                                 (14, 4), (15, 4), (16, 3), (17, 2), (18, 2), (19, 2), (20, 2),
                                 (21, 1), (22, 1), (23, 1), (24, 1)])
def test_integer_enumeration_matches_brute_force(H, n, R):
    print("enumerate n", n, "R", R, flush=True)
    J = inst.small_int(48, 1000 + n, -2, 2, density=0.5)
    h = np.random.default_rng(n).integers(-3, 4, 48).astype(np.float64)
    _solve(H, J, n, R, seed=n, h=h)


@pytest.mark.parametrize("n", [6, 12, 20])
def test_integer_enumeration_tie_takes_smaller_code(H, n):
    print("tie n", n, flush=True)
    J = inst.small_int(n, 2000 + n, -1, 1, density=0.7)   # h = 0, every spin ambivalent
    code = _solve(H, J, n, 2, seed=3)
    assert np.all(code < (1 << (n - 1)))   # of the two mirror codes, the one without bit n-1


def test_integer_enumeration_large_sums_take_int64_walk(H):
    n = 14
    J = inst.small_int(40, 3000, -3, 3, density=0.6) * float(1 << 21)
    print("large sums n", n, flush=True)
    _solve(H, J, n, 3, seed=5)


def _solve_real(H, J, n, R, seed, h=None):
    """As _solve, for couplings that are not integers: the binary64 Gray walk with the
    exact rescoring of near-ties.  The oracle scores every code from scratch with a
    correctly rounded sum (its code range split over host threads)."""
    N = J.shape[0]
    T, W = 200, 50
    md = H.MD(H.Problem(J, h=h), H.make_schedule(T, W), R, "f32", seed=1)
    rng = np.random.default_rng(seed)
    md.set_state(H.HQA_STATE_WSUM, rng.standard_normal((R, N)) * W)
    H.hqa_md_set_step(md.h, T)
    g = md.classify(n, solve=True)
    bar = md.state(H.HQA_STATE_PHIBAR)
    md.close()
    pb = orc.Problem(N, J=J, h=h)
    A, s = orc.classify(bar, n)
    he, Je = orc.reduce(pb, A, s)
    code, Ered = orc.enumerate_exact_blocks(Je, he, nthreads=16)
    assert np.array_equal(g["amb_idx"], A) and np.array_equal(g["h_eff"], he)
    assert np.array_equal(g["code"], code), (g["code"], code)
    assert np.array_equal(g["e_reduced"], Ered), (g["e_reduced"] - Ered)
    assert np.array_equal(g["spins"], orc.merge(s, A, code))


# Real couplings at the walk widths where the low walk carries 6, 10 and 14 bits and the
# K^2 term of the rescoring bound sets the window: the path SK reduced problems take.
@pytest.mark.parametrize("n,R", [(16, 3), (20, 2), (24, 1)])
def test_real_enumeration_sk_matches_oracle(H, n, R):
    print("real enumerate SK n", n, "R", R, flush=True)
    _solve_real(H, inst.sk(64, 5000 + n), n, R, seed=100 + n)


@pytest.mark.parametrize("n,R", [(16, 3), (20, 2), (24, 1)])
def test_real_enumeration_glass_with_field_matches_oracle(H, n, R):
    print("real enumerate glass n", n, "R", R, flush=True)
    J, h = inst.uniform_glass(64, 6000 + n)
    _solve_real(H, J, n, R, seed=200 + n, h=h)


def test_real_enumeration_near_ties(H):
    # couplings on a coarse binary grid plus one tiny offset: many codes tie in binary64
    # sums up to the offset, so the exact rescoring decides; n = 20 with a field
    n = 20
    rng = np.random.default_rng(77)
    N = 48
    J = np.triu(rng.integers(-4, 5, (N, N)) * 0.25, 1)
    J[0, 1] += 2.0 ** -40
    J = J + J.T
    h = rng.integers(-2, 3, N) * 0.5
    print("real enumerate near ties n", n, flush=True)
    _solve_real(H, J, n, 2, seed=9, h=h)
