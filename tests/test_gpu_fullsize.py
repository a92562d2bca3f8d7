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


def test_batch_bench_configuration(H):
    """The uneven batch at the bench line's full size and launch configuration: 512
    instances (256 SK N~U{100..2000} in BF16, 256 ER N~U{500..5000} in exact FP8), R = 64,
    T = 5000, the batch kernel, n = 20 exact.  Checked one output at a time where the
    oracle can follow:
    * for the smallest and largest instance of each family, the ambivalent sets and the
      frozen signs equal the oracle's sort of the exported phibar, the exact energies and
      cuts of all 64 read-out vectors equal the oracle's, ER cuts satisfy C = C0 - E/2,
      and for two replicas
      the reduced problem, the exact enumeration and the merged spins equal the oracle's;
    * the largest instance of each family, run alone with the same initial momenta,
      gives the same phibar bit for bit as inside the batch."""
    specs = inst.uneven_batch_specs(512)
    Js = [inst.uneven_batch_instance(s) for s in specs]
    probs = [H.Problem(J, storage="bf16" if s[0] == "sk" else "fp8") for J, s in zip(Js, specs)]
    R, T, W, n = 64, 5000, 100, 20
    md = H.MD(probs, H.make_schedule(T, W), R, "bf16", seed=4)
    md.run()
    md.sync()
    assert md.last_plan == "batch"
    pick = inst.stratified(specs, 2)        # smallest and largest SK, smallest and largest ER
    print("sampled instances", [(k, specs[k][0], specs[k][1]) for k in pick], flush=True)
    bars = {}
    for k in pick:
        fam, N = specs[k][0], specs[k][1]
        g = md.classify(n, solve=True, k=k)
        bar = md.state(H.HQA_STATE_PHIBAR, k)
        bars[k] = bar
        pb = orc.Problem(N, J=Js[k])
        A, s = orc.classify(bar, n)
        assert np.array_equal(g["amb_idx"], A)
        frozen = np.ones((R, N), dtype=bool)
        frozen[np.repeat(np.arange(R), n), A.ravel()] = False
        assert np.array_equal(g["spins"][frozen], s[frozen])
        E, C = orc.energy(pb, g["spins"])
        assert np.array_equal(g["energy"], E) and np.array_equal(g["cut"], C)
        if fam == "er":
            C0 = np.triu(Js[k], 1).sum() / 2.0
            assert np.array_equal(g["cut"], C0 - g["energy"] / 2)
        two = np.array([0, 63])
        he, Je = orc.reduce(pb, A[two], s[two])
        code, Ered = orc.enumerate_exact_blocks(Je, he, nthreads=16)
        assert np.array_equal(g["h_eff"][two], he)
        assert np.array_equal(g["code"][two], code) and np.array_equal(g["e_reduced"][two], Ered)
        assert np.array_equal(g["spins"][two], orc.merge(s[two], A[two], code))
        print(fam, N, "best cut", g["cut"].max(), flush=True)
    md.close()
    for k in (pick[1], pick[3]):
        alone = H.MD(probs[k], H.make_schedule(T, W), R, "bf16", seed=4)
        alone.run()
        assert np.array_equal(alone.state(H.HQA_STATE_PHIBAR), bars[k])
        alone.close()
