"""The replica-resident plan (one workgroup per 16 replicas, whole anneal in one
launch, state in LDS) must give bit-identical states to one launch per step: both
apply the same binary32 operation sequence.  Shapes cover the smallest size the
plan takes (4 row tiles), ragged row and replica tails, a field h, runs split at
arbitrary steps (including the half kick at q = 0 and a split inside the averaging
window), the bench shape, and the fallback for sizes whose state does not fit LDS.
The tuner must pick a plan without changing any result."""
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


def _pair(H, prob, T, W, R, prec, seed, cuts=(None,)):
    out = []
    for plan in ("resident", "step"):
        md = H.MD(prob, H.make_schedule(T, W), R, prec, seed=seed, plan=plan)
        for q in cuts:
            md.run(-1 if q is None else q)
            assert md.last_plan == plan
        md.sync()
        out.append(_states(H, md))
        md.close()
    return out


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("N,R,T", [(64, 16, 150), (300, 40, 250), (333, 17, 120),
                                   (800, 256, 300), (790, 48, 90)])
def test_resident_equals_per_step(H, prec, N, R, T):
    print("resident", prec, N, R, T, flush=True)
    J = inst.er_maxcut(N, 0.06, N)
    a, b = _pair(H, H.Problem(J), T, 30, R, prec, seed=7)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert np.all(np.isfinite(a[0])) and np.abs(a[0]).max() > 0


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_resident_with_field_and_pieces(H, prec):
    N, R, T, W = 257, 33, 300, 40
    J = inst.small_int(N, 5, -2, 2, density=0.2).astype(np.float64)
    h = np.random.default_rng(2).integers(-2, 3, size=N).astype(np.float64)
    a, b = _pair(H, H.Problem(J * 0.25, h=h * 0.25), T, W, R, prec, seed=3,
                 cuts=(1, 2, 100, 270, T))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_resident_classify_matches_per_step(H):
    N, R, T, n = 400, 32, 400, 12
    J = inst.er_maxcut(N, 0.06, 9)
    g = []
    for plan in ("resident", "step"):
        md = H.MD(H.Problem(J), H.make_schedule(T, 50), R, "fp8", seed=4, plan=plan)
        md.run()
        g.append(md.classify(n, solve=True))
        md.close()
    for k in ("spins", "amb_idx", "energy", "cut", "code"):
        assert np.array_equal(g[0][k], g[1][k])


def test_resident_falls_back_when_too_large(H):
    J = inst.er_maxcut(1100, 0.02, 3)
    md = H.MD(H.Problem(J), H.make_schedule(20, 5), 16, "fp8", seed=1, plan="resident")
    md.run()
    md.sync()
    assert md.last_plan == "step"
    md.close()
    md = H.MD(H.Problem(J), H.make_schedule(20, 5), 16, "f32", seed=1, plan="resident")
    md.run()
    assert md.last_plan == "step"        # FP32 J has no resident plan
    md.close()


def test_auto_plan_and_tuner_keep_results(H):
    N, R, T = 600, 64, 200
    J = inst.er_maxcut(N, 0.06, 11)
    ref = H.MD(H.Problem(J), H.make_schedule(T, 30), R, "bf16", seed=5, plan="step")
    ref.run()
    want = _states(H, ref)
    md = H.MD(H.Problem(J), H.make_schedule(T, 30), R, "bf16", seed=5)
    md.run(37)
    assert md.last_plan == "step"            # the untuned default
    md.tune(20)
    plan, tm, tn, cb, tj = md.tuned_plan()
    print("tuned plan", plan, tm, tn, cb, tj, flush=True)
    assert plan in ("step", "cluster", "resident", "batch")
    assert md.step == 37
    md.run()
    assert md.last_plan == plan
    for x, y in zip(want, _states(H, md)):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", ["f32", "fp8"])
def test_tuner_at_bench_shape(H, prec):
    """The tuner on the bench shape, on a non-default stream, in every binary32 precision
    (F32 keeps no BF16 operand copy and has no resident plan)."""
    import torch
    J = inst.er_maxcut(800, 0.06, 201)
    st = torch.cuda.Stream()
    ref = H.MD(H.Problem(J), H.make_schedule(200, 20), 256, prec, seed=2, plan="step",
               stream=st.cuda_stream)
    ref.run()
    want = _states(H, ref)
    md = H.MD(H.Problem(J), H.make_schedule(200, 20), 256, prec, seed=2, stream=st.cuda_stream)
    md.tune(10)
    plan, tm, tn, cb, tj = md.tuned_plan()
    print(prec, "tuned", plan, tm, tn, cb, tj, flush=True)
    md.run()
    for x, y in zip(want, _states(H, md)):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", ["f32", "bf16", "fp8"])
def test_every_step_block_shape_is_bit_identical(H, prec):
    """Per-step blocks of 16/32 rows x 16/32/64 replicas, with 4 or 8 chunks of loads in
    flight and (BF16 / FP8) J read row-major or from its MFMA-tiled copy, accumulate the
    same chains.  N = 333 leaves padding row tiles past the tiled copy."""
    N, R, T = 333, 64, 60
    J = inst.er_maxcut(N, 0.06, 3)
    out = {}
    for tj in ((0, 1) if prec != "f32" else (0,)):
        for cb in (4, 8):
            for tm in (1, 2):
                for tn in (1, 2, 4):
                    md = H.MD(H.Problem(J), H.make_schedule(T, 20), R, prec, seed=9)
                    md.set_step_tiles(tm, tn, cb, tiled=bool(tj))
                    md.run()
                    assert md.last_plan == "step"
                    out[(tm, tn, cb, tj)] = _states(H, md)
                    md.close()
    ref = out[(2, 4, 4, 0)]
    for key, st in out.items():
        for x, y in zip(ref, st):
            assert np.array_equal(x, y), key



def _csr_pair(H, prob, T, W, R, seed, cuts=(None,)):
    out = []
    for plan in ("resident", "step"):
        md = H.MD(prob, H.make_schedule(T, W), R, "f32", seed=seed, plan=plan)
        for q in cuts:
            md.run(-1 if q is None else q)
            assert md.last_plan == plan
        md.sync()
        out.append(_states(H, md))
        md.close()
    return out


@pytest.mark.parametrize("L,R,T", [(8, 4, 200), (8, 13, 150), (16, 64, 120), (16, 1024, 60)])
def test_csr_resident_equals_per_step(H, L, R, T):
    """Sparse replica-resident plan on the 3D +-J lattice: bit-identical to per step."""
    print("csr resident", L, R, T, flush=True)
    rp, ci, v = inst.ea3d(L, 300 + L)
    a, b = _csr_pair(H, H.Problem(row_ptr=rp, col=ci, val=v), T, 25, R, seed=3)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert np.abs(a[0]).max() > 0


def test_csr_resident_field_ragged_rows_and_pieces(H):
    """Rows of different degree (0..8), a field h, and runs split at arbitrary steps."""
    N, R, T = 700, 9, 300
    rng = np.random.default_rng(4)
    rows, cols, vals = [], [], []
    for i in range(N):
        for j in rng.choice(N, size=int(rng.integers(0, 5)), replace=False):
            if i != j:
                rows += [i, j]
                cols += [j, i]
                w = float(rng.choice([-1.0, 1.0, 0.5]))
                vals += [w, w]
    J = np.zeros((N, N))
    J[rows, cols] = vals                       # duplicates collapse to one symmetric value
    deg = (J != 0).sum(1)
    keep = deg <= 8
    J = J * keep[:, None] * keep[None, :]
    rp, ci, v = inst.dense_to_csr(J)
    h = rng.uniform(-0.5, 0.5, size=N)
    a, b = _csr_pair(H, H.Problem(row_ptr=rp, col=ci, val=v, h=h), T, 40, R, seed=6,
                     cuts=(1, 2, 100, 270, T))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_csr_resident_falls_back_and_tuner(H):
    rp, ci, v = inst.er_sparse(500, 20, 7)            # degrees above 8: no resident plan
    md = H.MD(H.Problem(row_ptr=rp, col=ci, val=v), H.make_schedule(50, 10), 8, "f32", seed=1,
              plan="resident")
    md.run()
    assert md.last_plan == "step"
    md.close()
    rp, ci, v = inst.ea3d(16, 301)
    prob = H.Problem(row_ptr=rp, col=ci, val=v)
    ref = H.MD(prob, H.make_schedule(200, 20), 256, "f32", seed=2, plan="step")
    ref.run()
    want = _states(H, ref)
    md = H.MD(prob, H.make_schedule(200, 20), 256, "f32", seed=2)
    md.tune(20)
    plan = md.tuned_plan()[0]
    print("csr tuned plan", plan, flush=True)
    assert plan in ("step", "resident")
    md.run()
    assert md.last_plan == plan
    for x, y in zip(want, _states(H, md)):
        assert np.array_equal(x, y)
