"""Learned early stop: the workflow around the library's statistics, features,
classifier kernels and read-out (every numerical step runs in libhqa).

The paper has no learned component; this is the library's extension.  A run
with statistics windows [(j-1)K, jK) yields per-spin features at checkpoints
jK; labels come from the full-length run of the same initial state (the
n_amb smallest |phibar(T)| per replica are ambivalent, the others
frozen with the sign of phibar(T)); the 12-64-64-3 classifier is trained on
the GPU by the library's own forward/backward/Adam kernels.  At inference the
run stops at the first checkpoint whose mean max-probability reaches a
threshold calibrated on validation runs; frozen spins take their predicted
sign and the n most-ambivalent spins go to the exact solver.  The full run is
both the fallback (no stop before T) and the reference (mislabel rate, cut loss).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import hqa


@dataclass
class RunRecord:
    feats: list        # per checkpoint: [R, N, 12] float32
    steps: list        # checkpoint steps
    labels: np.ndarray  # [R, N] int32 from the full run
    full: dict         # full-run read-out (classify with solve) at T
    md: object
    means: list        # per checkpoint: trailing-window mean flux [R, N] (truncation read-out)


def labels_from_full(md, n_amb: int) -> tuple[np.ndarray, dict]:
    """Labels of the full run: 2 = ambivalent (n_amb smallest |phibar|), else 0/1 by sign."""
    g = md.classify(n_amb, solve=False)
    lab = np.where(g["spins"] > 0, 0, 1).astype(np.int32)
    R = lab.shape[0]
    lab[np.repeat(np.arange(R), g["amb_idx"].shape[1]), g["amb_idx"].ravel()] = 2
    return lab, g


def record_run(problem, sched, R: int, K: int, n_ckpt: int, seed: int, n_amb: int,
               precision="f32", solve_n: int = 0, every: int = 1, Ks: int | None = None,
               stride: int = 1, keep: float = 1.0, keep_seed: int = 0,
               means: bool = True) -> RunRecord:
    """Run to T with statistics windows of the last Ks steps (default K; sampling every
    stride-th step) before every every-th checkpoint among K, 2K, ..., n_ckpt K; return
    the features and the trailing-window mean flux at those checkpoints and the labels
    from the full run.  With keep < 1 only a random fraction `keep` of the (replica,
    spin) samples of each checkpoint is returned, as rows [n, 12] with their labels in
    record.labels (large training sets)."""
    Ks = K if Ks is None else Ks
    md = hqa.MD(problem, sched, R, precision, seed=seed)
    feats, steps, mlist = [], [], []
    for j in range(every, n_ckpt + 1, every):
        md.run(j * K - Ks)
        md.stats_window(j * K - Ks, j * K, stride)
        md.run(j * K)
        feats.append(md.features())
        if means:
            mlist.append(md.state(hqa.HQA_STATE_STATMEAN))
        steps.append(j * K)
    md.run()
    lab, g = labels_from_full(md, n_amb)
    full = md.classify(solve_n, solve=solve_n > 0) if solve_n else g
    if keep < 1.0:
        rng = np.random.default_rng(keep_seed)
        sel = [rng.random(lab.size) < keep for _ in feats]
        feats = [f.reshape(-1, hqa.HQA_ES_NFEAT)[m] for f, m in zip(feats, sel)]
        lab = [lab.ravel()[m] for m in sel]
    return RunRecord(feats, steps, lab, full, md, mlist)


def dataset(records) -> tuple[np.ndarray, np.ndarray]:
    X, y = [], []
    for rec in records:
        for c, f in enumerate(rec.feats):
            X.append(f.reshape(-1, hqa.HQA_ES_NFEAT))
            # subsampled records keep one label vector per checkpoint
            y.append(rec.labels[c] if isinstance(rec.labels, list) else rec.labels.ravel())
    return np.concatenate(X), np.concatenate(y)


def class_weights(y: np.ndarray) -> np.ndarray:
    cnt = np.bincount(y, minlength=3).astype(np.float64)
    w = cnt.sum() / np.maximum(cnt, 1.0) / 3.0
    return w.astype(np.float32)


def train(es, X, y, epochs: int = 4, batch: int = 8192, lr: float = 3e-3, seed: int = 0,
          log=None) -> list:
    rng = np.random.default_rng(seed)
    cw = class_weights(y)
    losses = []
    n = X.shape[0]
    for ep in range(epochs):
        perm = rng.permutation(n)
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            losses.append(es.train_step(X[idx], y[idx], cw, lr))
        if log:
            log(f"epoch {ep}: loss {np.mean(losses[-max(1, n // batch):]):.4f}")
    return losses


def labels_from_probs(prob: np.ndarray, n_amb: int) -> np.ndarray:
    """Labels implied by a read-out: per replica the n_amb highest P(ambivalent) are
    ambivalent (ties: lower index), the others frozen + if P(+) >= P(-) else frozen -."""
    R, N, _ = prob.shape
    lab = np.where(prob[..., 0] >= prob[..., 1], 0, 1).astype(np.int32)
    key = (np.float32(1.0) - prob[..., 2].astype(np.float32))
    for r in range(R):
        lab[r, np.lexsort((np.arange(N), key[r]))[:n_amb]] = 2
    return lab


def confidence(prob: np.ndarray) -> float:
    """Mean over spins and replicas of the largest class probability."""
    return float(prob.reshape(-1, 3).max(axis=1).mean())


def pick_threshold(per, target: float, cands=None) -> float:
    """Smallest threshold c such that, for every validation run, stopping at the first
    checkpoint whose confidence is >= c costs at most `target`.  per[run] lists
    (confidence, cost) per checkpoint in step order; a run with no such checkpoint runs
    to T, which costs 0.  inf if no candidate meets the target."""
    cands = np.linspace(0.50, 0.999, 200) if cands is None else cands
    for c in cands:
        worst = 0.0
        for rows in per:
            hit = [cost for conf, cost in rows if conf >= c]
            worst = max(worst, hit[0] if hit else 0.0)
        if worst <= target:
            return float(c)
    return float("inf")


def calibrate(es, records, target_mislabel: float = 0.02, bf16: bool = True) -> float:
    """Smallest threshold c such that, on validation runs, stopping at the first
    checkpoint with confidence >= c gives a mislabel rate <= target (inf if none).
    Each record's labels fix its number of ambivalent spins per replica."""
    per = []
    for rec in records:
        n_lab = int(np.sum(rec.labels[0] == 2))
        rows = []
        for f in rec.feats:
            pr = es.predict(f.reshape(-1, 12), bf16=bf16).reshape(f.shape[0], f.shape[1], 3)
            mis = float(np.mean(labels_from_probs(pr, n_lab) != rec.labels))
            rows.append((confidence(pr), mis))
        per.append(rows)
    return pick_threshold(per, target_mislabel)


def calibrate_cut(es, records, target_loss: float = 1e-3, n_amb: int | None = None,
                  bf16: bool = True) -> float:
    """Smallest threshold c such that, on validation runs, the read-out at the first
    checkpoint with confidence >= c (frozen spins from the predicted signs, the n_amb
    most ambivalent solved exactly) loses at most target_loss of the full run's best cut
    (inf if none).  The records' handles must still be open (the read-out uses their
    couplings) and their `full` read-outs must have solved spins exactly (n_amb defaults
    to the number they solved)."""
    per = []
    for rec in records:
        best = float(rec.full["cut"].max())
        n = rec.full["amb_idx"].shape[1] if n_amb is None else n_amb
        rows = []
        for f in rec.feats:
            pr = es.predict(f.reshape(-1, 12), bf16=bf16).reshape(f.shape[0], f.shape[1], 3)
            cut = float(rec.md.classify(n, solve=True, prob=pr)["cut"].max())
            rows.append((confidence(pr), max(0.0, (best - cut) / abs(best)) if best else 0.0))
        per.append(rows)
    return pick_threshold(per, target_loss)


def truncation_probs(m: np.ndarray) -> np.ndarray:
    """The method without the network, at the same step: sign and ambivalence from the
    trailing-window mean flux m [R, N] alone: P(+) = [m >= 0], P(-) = [m < 0],
    P(amb) = 1 - |m| / max |m| (so the smallest |m| are the most ambivalent)."""
    a = np.abs(m)
    mx = a.max(axis=1, keepdims=True) + 1e-30
    P = np.zeros(m.shape + (3,), dtype=np.float32)
    P[..., 0] = m >= 0
    P[..., 1] = m < 0
    P[..., 2] = 1.0 - a / mx
    return P


@dataclass
class StopResult:
    stop_step: int
    stopped: bool
    prob: np.ndarray
    readout: dict
    ablation: dict
    mislabel: float
    mislabel_ablation: float
    wall_ms: float = float("nan")   # the method alone: checkpointed MD to the stop + read-out


def run_with_early_stop(es, problem, sched, R: int, K: int, threshold: float, n_amb: int,
                        seed: int, labels=None, n_label: int | None = None,
                        bf16: bool = True, Ks: int | None = None, stride: int = 1) -> StopResult:
    """Run checkpoint by checkpoint (statistics over the last Ks steps before each); stop
    at the first confident checkpoint (or T).  n_amb spins go to the exact solver; mislabel rates (when the full run's labels are
    given) count n_label ambivalent spins per replica (default n_amb)."""
    import time
    import torch   # device memory for the checkpoint evaluation (the arithmetic is libhqa's)
    n_label = n_amb if n_label is None else n_label
    md = hqa.MD(problem, sched, R, "f32", seed=seed)
    T, N = sched.T, problem.n
    # features and probabilities stay on the device; each checkpoint returns one number
    pdev = torch.empty((R * N, 3), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ks = K if Ks is None else Ks
    # the checkpoint loop and the stop rule run in the library (hqa_md_run_es)
    q, _conf = md.run_es(es, K, Ks, stride, threshold, bf16=bf16, prob=pdev)
    stopped = q < T
    out = md.classify(n_amb, solve=True, prob=pdev)   # host outputs: synchronises
    wall_ms = (time.perf_counter() - t0) * 1e3
    # evaluation only (not part of the method's time): the truncation ablation and the
    # mislabel rates
    tp = truncation_probs(md.state(hqa.HQA_STATE_STATMEAN))
    prob = pdev.cpu().numpy().reshape(R, N, 3)
    abl = md.classify(n_amb, solve=True, prob=tp)
    mis = mis_a = float("nan")
    if labels is not None:
        mis = float(np.mean(labels_from_probs(prob, n_label) != labels))
        mis_a = float(np.mean(labels_from_probs(tp, n_label) != labels))
    md.close()
    return StopResult(q, stopped, prob, out, abl, mis, mis_a, wall_ms)
