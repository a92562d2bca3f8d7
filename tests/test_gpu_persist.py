"""The cluster plan (all steps in one cooperative launch, cluster barriers) must give
bit-identical states to one launch per step: both apply the same binary32
operation sequence.  Shapes cover LDS-resident and L2-streamed J blocks, ragged
row and replica tails, the small-SK/large-ER sizes and the bench shape."""
import numpy as np
import pytest

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


def _states(H, md):
    return [md.state(w) for w in (H.HQA_STATE_PHI, H.HQA_STATE_P, H.HQA_STATE_WSUM)]


@pytest.mark.parametrize("prec", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("N,R,T", [(300, 40, 250), (64, 16, 120), (800, 256, 400),
                                   (1300, 64, 150), (2100, 32, 60)])
def test_persistent_equals_per_step(H, prec, N, R, T):
    print("persist", prec, N, R, T, flush=True)
    J = inst.er_maxcut(N, 0.05, N)
    out = []
    for pers in (True, False):
        plan = "cluster" if pers else "step"
        md = H.MD(H.Problem(J), H.make_schedule(T, 30), R, prec, seed=7, plan=plan)
        md.run()
        md.sync()
        assert md.last_plan == plan
        out.append(_states(H, md))
        md.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_persistent_in_pieces_and_single_step(H, prec):
    N, R, T = 500, 48, 300
    J, h = inst.uniform_glass(N, 3)
    J *= 0.05
    a = H.MD(H.Problem(J, h=h), H.make_schedule(T, 40), R, prec, seed=1, plan="step")
    a.run()
    b = H.MD(H.Problem(J, h=h), H.make_schedule(T, 40), R, prec, seed=1, plan="cluster")
    for q in (1, 2, 101, 257, T):
        b.run(q)
        assert b.last_plan == "cluster"
    for x, y in zip(_states(H, a), _states(H, b)):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("N,R", [(150, 24), (500, 48), (600, 16), (700, 40), (1000, 80),
                                 (1100, 20), (1250, 40), (1500, 36), (1650, 16), (1900, 40),
                                 (2000, 16)])
def test_register_j_kernel_every_group_count(H, prec, N, R):
    """The register-J cluster kernel is instantiated per 128-column group count
    NG = Np / 128 (Np = N padded to 128); NG from 2 to 16 (past 8 part of the J
    fragments live in accumulation registers; 2000 x 16 is the K2000 shape), ragged
    replica clusters, against one launch per step."""
    print("persist rj", prec, N, R, flush=True)
    J = inst.er_maxcut(N, 0.04, N + 1)
    out = []
    for plan in ("cluster", "step"):
        md = H.MD(H.Problem(J), H.make_schedule(90, 20), R, prec, seed=3, plan=plan)
        md.run()
        md.sync()
        assert md.last_plan == plan
        out.append(_states(H, md))
        md.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("R", [16, 40])
def test_cluster_launch_over_several_instances(H, prec, R):
    """Consecutive instances of one size share a register-J launch (cluster c serves
    instance c / C1, each cluster on its own XCD): five of 600 spins, two of 300 and
    three of 2000 (at R = 40 only two of those fit one launch and the third runs
    alone).  Every instance follows the trajectory it has alone."""
    print("cluster set", prec, R, flush=True)
    sizes = [600, 600, 600, 600, 600, 300, 300, 2000, 2000, 2000]
    Js = [inst.er_maxcut(n, 0.05, 40 + k) for k, n in enumerate(sizes)]
    T = 90
    b = H.MD([H.Problem(J) for J in Js], H.make_schedule(T, 20), R, prec, seed=5, plan="cluster")
    b.run()
    b.sync()
    assert b.last_plan == "cluster"
    for k, J in enumerate(Js):
        a = H.MD(H.Problem(J), H.make_schedule(T, 20), R, prec, seed=5, plan="step")
        a.run()
        for w in (H.HQA_STATE_PHI, H.HQA_STATE_P, H.HQA_STATE_WSUM):
            assert np.array_equal(a.state(w), b.state(w, k)), (k, w)
        a.close()


def test_tuned_auto_over_several_instances(H):
    """The tuner times the batched kernel, the same-size cluster launches and each
    instance on its own plan for a handle of several dense instances; whichever AUTO
    then takes, every instance follows the trajectory it has alone."""
    sizes = [700, 700, 700, 700, 700]
    Js = [inst.er_maxcut(n, 0.05, 60 + k) for k, n in enumerate(sizes)]
    T, R = 200, 16
    b = H.MD([H.Problem(J) for J in Js], H.make_schedule(T, 20), R, "fp8", seed=9)
    b.tune(20)
    b.run()
    b.sync()
    print("tuned plan for five instances:", b.last_plan, flush=True)
    assert b.last_plan in ("batch", "cluster", "step", "resident")
    for k, J in enumerate(Js):
        a = H.MD(H.Problem(J), H.make_schedule(T, 20), R, "fp8", seed=9, plan="step")
        a.run()
        for w in (H.HQA_STATE_PHI, H.HQA_STATE_P, H.HQA_STATE_WSUM):
            assert np.array_equal(a.state(w), b.state(w, k)), (k, w)
        a.close()
