"""Learned early stop end to end on the GPU, at a reduced scale.

Sparse Erdos-Renyi MAX-CUT instances (N 300..600, mean degree 10..40, unit weights,
J = +w), 16 replicas, T = 4000 MD steps, statistics windows of K = T/16 steps.
Training data are runs of the method itself: features at every checkpoint, labels
from the full-length run of the same initial momenta (the 5% smallest |phibar| per
replica ambivalent, the others frozen with their sign).  The 12-64-64-3 network is
trained by the library's own forward/backward/Adam kernels.

Checked:
* training lowers the loss;
* the gain over the method without the network: on held-out instances, at the same
  checkpoint, the labels the network implies (n highest P(ambivalent), sign from
  P(+) vs P(-)) disagree with the full run's labels less often than the truncation
  read-out's (sign of the trailing-window mean, n smallest |mean|);
* the stop rule with a threshold calibrated on validation runs (by the mislabel rate,
  or by the cut the read-out loses at the stop): the read-out at the stop step (frozen
  spins from the network, n <= 24 ambivalent spins solved exactly) loses at most 0.2%
  of the full run's best cut, and never stops after T.

The network's quality is not fixed by the paper (it has no learned part): the full
run is the reference.  The printed lines give the mislabel curves, the threshold, the
stop step and the cuts.
"""
import numpy as np
import pytest

from paper_2004_03972_amd import instances as inst

pytestmark = pytest.mark.gpu

T, R = 4000, 16
K = T // 16
NCK = 15


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    from paper_2004_03972_amd import hqa
    hqa.lib()
    return hqa


@pytest.fixture(scope="module")
def trained(H):
    from paper_2004_03972_amd import early_stop as E
    rng = np.random.default_rng(5)
    sched = H.make_schedule(T, 100)
    recs = []
    for k in range(24):
        N = int(rng.integers(300, 601))
        d = float(rng.uniform(10, 40))
        rp, ci, v = inst.er_sparse(N, d, 5_000_000 + k)
        P = H.Problem(row_ptr=rp, col=ci, val=v)
        n_lab = max(1, round(0.05 * N))
        rec = E.record_run(P, sched, R, K, NCK, seed=100 + k, n_amb=n_lab, solve_n=min(20, n_lab))
        if not 16 <= k < 20:
            rec.md.close()            # the validation handles serve the cut calibration
        recs.append((N, n_lab, P, rec))
    train, val, test = recs[:16], recs[16:20], recs[20:]
    X, y = E.dataset([r for *_, r in train])
    es = H.ES(seed=1)
    losses = E.train(es, X, y, epochs=6, batch=8192, lr=3e-3)
    print("training samples", X.shape[0], "class counts", np.bincount(y), flush=True)
    yield E, es, losses, sched, val, test
    for *_, r in val:
        r.md.close()


def test_training_lowers_loss(trained):
    E, es, losses, *_ = trained
    per_epoch = len(losses) // 6
    first, last = np.mean(losses[:per_epoch]), np.mean(losses[-per_epoch:])
    print("loss first epoch", first, "last epoch", last, flush=True)
    assert last < first


def test_network_beats_truncation_at_the_same_step(trained):
    E, es, _, _, _, test = trained
    gains, wins = [], []
    for N, n_lab, _, r in test:
        curve = []
        for j, f in enumerate(r.feats):
            if not (T // 4 <= r.steps[j] <= 7 * T // 8):
                continue
            pr = es.predict(f.reshape(-1, 12), bf16=True).reshape(R, N, 3)
            m_net = float(np.mean(E.labels_from_probs(pr, n_lab) != r.labels))
            m_tr = float(np.mean(E.labels_from_probs(E.truncation_probs(r.means[j]), n_lab)
                                 != r.labels))
            curve.append((r.steps[j], round(m_net, 4), round(m_tr, 4)))
            gains.append(m_tr - m_net)
            wins.append(m_net < m_tr)
        print(f"N={N} (step, network, truncation) mislabel:", curve, flush=True)
    print("mean gain", np.mean(gains), "win fraction", np.mean(wins), flush=True)
    assert np.mean(gains) > 0.005
    assert np.mean(wins) >= 0.75


@pytest.mark.parametrize("by", ["mislabel", "cut"])
def test_stop_rule_keeps_the_cut(trained, by):
    """Both calibrations: a 3% mislabel rate, or 0.1% of the best cut lost, at the stop
    on the validation runs."""
    E, es, _, sched, val, test = trained
    if by == "mislabel":
        thr = E.calibrate(es, [r for *_, r in val], target_mislabel=0.03)
    else:
        thr = E.calibrate_cut(es, [r for *_, r in val], target_loss=1e-3)
    if not np.isfinite(thr):
        thr = 1.1                      # never confident: every run is the full run
    print("calibrated by", by, "threshold", thr, flush=True)
    for k, (N, n_lab, P, r) in enumerate(test):
        res = E.run_with_early_stop(es, P, sched, R, K, thr, n_amb=min(20, n_lab),
                                    seed=120 + k, labels=r.labels, n_label=n_lab)
        full = float(r.full["cut"].max())
        early = float(res.readout["cut"].max())
        trunc = float(res.ablation["cut"].max())
        print(f"N={N} stop {res.stop_step}/{T} (speedup {T / res.stop_step:.2f}) mislabel "
              f"network {res.mislabel:.4f} truncation {res.mislabel_ablation:.4f}; best cut "
              f"early {early:.0f} truncation {trunc:.0f} full {full:.0f}", flush=True)
        assert res.stop_step <= T
        assert early >= (1.0 - 0.002) * full
        assert res.readout["spins"].shape == (R, N)
