"""Parity at the benchmark's full size, in the launch configuration the benchmark
times (ER MAX-CUT G(800, 0.06), J = +w stored exactly in FP8, R = 256, T = 5000,
tuned plan, n = 20 solved exactly).  The oracle cannot afford the trajectories, so
this checks what it can compute one output at a time:

* the ambivalent sets of all replicas equal the oracle's sort of the exported phibar,
  and the frozen spins its signs;
* the exact energies and cuts of all 256 read-out spin vectors equal the oracle's,
  and satisfy C = C0 - E/2;
* for sampled replicas the reduced problem, the exact enumeration and the merged
  spins equal the oracle's.
"""
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


def test_bench_configuration_readout(H):
    N, R, T, n = 800, 256, 5000, 20
    J = inst.er_maxcut(N, 0.06, 201)
    md = H.MD(H.Problem(J), H.make_schedule(T, 100), R, "fp8", seed=2, require_exact=True)
    md.tune(20)
    print("tuned plan", md.tuned_plan(), flush=True)
    md.run()
    md.sync()
    g = md.classify(n, solve=True)
    bar = md.state(H.HQA_STATE_PHIBAR)
    pb = orc.Problem(N, J=J)
    A, s = orc.classify(bar, n)
    assert np.array_equal(g["amb_idx"], A)
    frozen = np.ones((R, N), dtype=bool)
    frozen[np.repeat(np.arange(R), n), A.ravel()] = False
    assert np.array_equal(g["spins"][frozen], s[frozen])
    E, C = orc.energy(pb, g["spins"])
    assert np.array_equal(g["energy"], E) and np.array_equal(g["cut"], C)
    C0 = np.triu(J, 1).sum() / 2.0          # E = sum(uncut w) - sum(cut w): C = C0 - E / 2
    assert np.array_equal(C, C0 - E / 2)
    rows = np.array([0, 85, 170, 255])
    he, Je = orc.reduce(pb, A[rows], s[rows])
    code, Ered = orc.enumerate_exact(Je, he)
    assert np.array_equal(g["h_eff"][rows], he)
    assert np.array_equal(g["code"][rows], code) and np.array_equal(g["e_reduced"][rows], Ered)
    assert np.array_equal(g["spins"][rows], orc.merge(s[rows], A[rows], code))
    print("best cut", C.max(), "mean", C.mean(), flush=True)
    md.close()
