"""Learned early stop on the GPU against the FP64 oracle.

- statistics/features of a binary32 run (dense and CSR) against the oracle's FP64
  features of the same initial state (short window: the trajectories agree to
  ~1e-5, the features to 1e-3);
- the GPU gradient of the weighted cross entropy against the oracle's analytic
  FP64 gradient (relative 2-norm error <= 1e-4), one Adam step against the
  oracle's step, binary32 and BF16 inference against the FP64 forward;
- the read-out from predicted probabilities against a lexicographic sort.
"""
import numpy as np
import pytest

import oracle as orc
from f32_bound import f32_bound
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


@pytest.mark.parametrize("layout,every", [("dense", 1), ("csr", 1), ("dense", 3), ("csr", 7)])
def test_features_match_oracle(H, layout, every):
    N, R, T, K0, K1 = 300, 6, 2000, 60, 260
    if layout == "dense":
        J = inst.er_maxcut(N, 0.05, 31)
        P, pb = H.Problem(J), orc.Problem(N, J=J)
    else:
        rp, ci, v = inst.er_sparse(N, 12, 31)
        P, pb = H.Problem(row_ptr=rp, col=ci, val=v), orc.Problem(N, row_ptr=rp, col=ci, val=v)
    md = H.MD(P, H.make_schedule(T, 100), R, "f32", seed=5)
    # the trajectory: within the derived binary32 error bound after 30 steps
    e, phis = f32_bound(orc, pb, orc.MDParams(T=T, W=100), np.zeros((R, N)),
                        orc.init_p0(5, N, R), 30)
    md.run(30)
    assert np.max(np.abs(md.state(H.HQA_STATE_PHI) - phis[30])) <= e[30]
    md.stats_window(K0, K1, every)
    md.run(K1)
    f = md.features()
    fo, phi, _ = orc.es_features(pb, orc.MDParams(T=T, W=100), np.zeros((R, N)),
                                 orc.init_p0(5, N, R), K0, K1, every)
    print(layout, "max |phi32 - phi64| at the checkpoint (observed)",
          np.max(np.abs(md.state(H.HQA_STATE_PHI) - phi)), flush=True)
    # features: statistics of two trajectories that differ by the divergence above;
    # the sign-based features are not continuous in the fluxes, so this bar is the
    # observed agreement, not a derived bound
    err = np.max(np.abs(f - fo), axis=(0, 1))
    print(layout, "max |feature err| per feature", err, flush=True)
    assert np.all(err < 2e-3)
    # features at a later checkpoint with a new window (continuing the same run)
    md.stats_window(K1, K1 + 150)
    md.run(K1 + 150)
    assert md.features().shape == (R, N, 12)


def _rand_params(seed, scale=0.25):
    return np.random.default_rng(seed).normal(0, scale, size=5187)


def test_gradient_loss_and_adam_match_oracle(H):
    rng = np.random.default_rng(3)
    n = 1000
    x = rng.normal(size=(n, 12))
    y = rng.integers(0, 3, size=n).astype(np.int32)
    cw = np.array([1.0, 1.5, 6.0])
    P = _rand_params(4)
    es = H.ES(seed=1)
    es.params = P
    Pf = es.params.astype(np.float64)                # binary32 parameters as used on the GPU
    xf = x.astype(np.float32).astype(np.float64)
    loss, g = es.grad(x, y, cw)
    lo, go = orc.mlp_loss_grad(Pf, xf, y, cw)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    print("grad rel err", rel, "loss", loss, lo, flush=True)
    assert rel <= 1e-4 and loss == pytest.approx(lo, rel=1e-5)
    # one Adam step from zero moments
    l2 = es.train_step(x, y, cw, 1e-3)
    assert l2 == pytest.approx(lo, rel=1e-5)
    Q, m, v = Pf.copy(), np.zeros(5187), np.zeros(5187)
    orc.adam_step(Q, go, m, v, 1, lr=1e-3)
    assert np.max(np.abs(es.params - Q)) < 5e-6
    # inference
    pr = es.predict(x)
    po = orc.mlp_forward(es.params.astype(np.float64), xf)
    assert np.max(np.abs(pr - po)) < 1e-5
    pb = es.predict(x, bf16=True)
    assert np.max(np.abs(pb - po)) < 5e-2
    print("bf16 inference max |dp|", np.max(np.abs(pb - po)), flush=True)


def test_training_reduces_loss(H):
    rng = np.random.default_rng(8)
    n = 4096
    x = rng.normal(size=(n, 12))
    y = np.where(x[:, 0] > 0.5, 0, np.where(x[:, 0] < -0.5, 1, 2)).astype(np.int32)
    cw = np.ones(3)
    es = H.ES(seed=2)
    first = es.train_step(x, y, cw, 3e-3)
    for _ in range(300):
        last = es.train_step(x, y, cw, 3e-3)
    acc = np.mean(np.argmax(es.predict(x), 1) == y)
    print("loss", first, "->", last, "acc", acc, flush=True)
    assert last < 0.5 * first and acc > 0.9


def test_classify_from_probabilities(H):
    N, R, n = 250, 5, 12
    J = inst.small_int(N, 41, -2, 2, density=0.3)
    md = H.MD(H.Problem(J), H.make_schedule(50, 10), R, "f32", seed=1)
    md.run(20)                                      # any step: the read-out does not need T
    rng = np.random.default_rng(9)
    prob = rng.dirichlet(np.ones(3), size=(R, N)).astype(np.float32)
    prob[0, :6] = prob[0, 6]                         # ties in P(ambivalent)
    g = md.classify(n, solve=True, prob=prob)
    key = (np.float32(1.0) - prob[..., 2]).astype(np.float32)
    s = np.where(prob[..., 0] >= prob[..., 1], 1, -1).astype(np.int8)
    A = np.stack([np.sort(np.lexsort((np.arange(N), key[r]))[:n]) for r in range(R)]).astype(np.int32)
    assert np.array_equal(g["amb_idx"], A)
    pb = orc.Problem(N, J=J)
    he, Je = orc.reduce(pb, A, s)
    code, Ered = orc.enumerate_exact(Je, he)
    sh = orc.merge(s, A, code)
    assert np.array_equal(g["spins"], sh) and np.array_equal(g["code"], code)
    E, C = orc.energy(pb, sh)
    assert np.array_equal(g["energy"], E)


def test_run_es_equals_checkpoint_loop(H):
    """hqa_md_run_es (the stop loop inside the library) against the same calls made one
    by one: the same stop step, and bit-identical probabilities and confidence."""
    import torch
    N, R, T, K, Ks, stride = 300, 4, 2000, 400, 100, 2
    J = inst.er_maxcut(N, 0.05, 41)
    es = H.ES(seed=3)
    md = H.MD(H.Problem(J), H.make_schedule(T, 100), R, "f32", seed=6)
    feat = torch.empty((R * N, 12), dtype=torch.float32, device="cuda")
    probs, confs, q = [], [], 0
    while q < T:
        nxt = min(q + K, T)
        md.run(max(q, nxt - Ks))
        md.stats_window(max(q, nxt - Ks), nxt, stride)
        md.run(nxt)
        q = nxt
        md.features(out=feat)
        pd = torch.empty((R * N, 3), dtype=torch.float32, device="cuda")
        es.predict(feat, bf16=True, out=pd)
        probs.append(pd.cpu().numpy())
        confs.append(es.confidence(pd))
    md.close()
    thr = confs[2]
    want = next(j for j, c in enumerate(confs) if c >= thr)
    md = H.MD(H.Problem(J), H.make_schedule(T, 100), R, "f32", seed=6)
    out = np.empty((R, N, 3), dtype=np.float32)
    stop, conf = md.run_es(es, K, Ks, stride, thr, prob=out)
    print("confidences", confs, "stop", stop, flush=True)
    assert stop == (want + 1) * K and conf == confs[want]
    assert np.array_equal(out.reshape(-1, 3), probs[want])
    md.close()
    # a threshold never reached runs to T (the fallback)
    md = H.MD(H.Problem(J), H.make_schedule(T, 100), R, "f32", seed=6)
    stop, conf = md.run_es(es, K, Ks, stride, 2.0)
    assert stop == T and conf == confs[-1]
    with pytest.raises(H.HQAError) as e:
        md.run_es(es, K, Ks, stride, 0.5)            # already at T
    assert e.value.status == H.HQA_ESTATE
    md.close()
    md = H.MD(H.Problem(J), H.make_schedule(T, 100), R, "f32", seed=6)
    for bad in ((0, 1, 1), (100, 200, 1), (100, 50, 0)):
        with pytest.raises(H.HQAError) as e:
            md.run_es(es, *bad, 0.5)
        assert e.value.status == H.HQA_EINVAL
    md.close()
    es.close()
