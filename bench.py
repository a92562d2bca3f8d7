"""HQA-MD throughput on one MI355X: MD spin-updates/s, plain FP32 vs the chosen form.

Workload: MAX-CUT on an Erdos-Renyi graph G(800, 0.06) with unit weights mapped to
J = +w, 256 replicas, 5000 MD steps (paper schedule, M = 6, W = 100), n = 20
ambivalent spins solved exactly.  One bench step is one pass of the whole hot
path on the resident instance: reset of the initial state, T MD steps (field +
fused leapfrog), the frozen/ambivalent sort, the reduced problem, exact
enumeration, merge and exact energies/cuts.  value = N * R * T * steps / time of
the chosen form (FP8 e4m3 J widened to BF16, BF16 flux operand, FP32 accumulate).
The same steps run in plain FP32 (FP32 J and fluxes on FP32 MFMA) with the same
initial momenta; the chosen form's best cut must be within 0.1% of FP32's.

  python bench.py [--steps K] [--warmup W] [--no-cpu] [--prec fp8|bf16|f32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, P_EDGE, R, T, W, N_AMB = 800, 0.06, 256, 5000, 100, 20
INSTANCE_SEED, RUN_SEED = 201, 2
PEAK = {"bf16": 2.5e15, "fp8": 2.5e15, "f32": 157.3e12}   # dense MFMA FLOP/s (fp8 J runs bf16 MFMA)
HBM_PEAK = 8.0e12


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(hqa, torch, prob, prec, steps, warmup):
    stream = torch.cuda.current_stream()
    md = hqa.MD(prob, hqa.make_schedule(T, W), R, prec, seed=RUN_SEED, require_exact=True,
                stream=stream.cuda_stream)
    best_cut, best_cut_md, md_ms = [], [], []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for k in range(warmup):
        md.reset(RUN_SEED + 1000 + k)
        md.run()
        md.classify(N_AMB, solve=True)
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(steps):
        md.reset(RUN_SEED + k)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        md.run()
        e1.record(stream)
        g = md.classify(N_AMB, solve=True)          # synchronises
        md_ms.append(e0.elapsed_time(e1))
        best_cut.append(float(g["cut"].max()))
        g0 = md.classify(N_AMB, solve=False) if k == 0 else None
        if g0 is not None:
            best_cut_md.append(float(g0["cut"].max()))
            frozen_amb = dict(n_frozen=N - N_AMB, n_ambivalent=N_AMB)
    ev[1].record(stream)
    torch.cuda.synchronize()
    total_ms = ev[0].elapsed_time(ev[1])
    md.close()
    return dict(total_ms=total_ms, md_ms=md_ms, best_cut=best_cut, best_cut_md=best_cut_md,
                split=frozen_amb)


def cpu_baseline():
    """The FP64 oracle on a bounded sample: 16 replicas x 5000 steps of the same instance."""
    import oracle as orc
    from paper_2004_03972_amd import instances as inst
    threads = max(1, min(16, os.cpu_count() or 1))
    Rs = 16
    J = inst.er_maxcut(N, P_EDGE, INSTANCE_SEED)
    pb = orc.Problem(N, J=J)
    mp = orc.MDParams(T=T, W=W)
    p0 = orc.init_p0(RUN_SEED, N, Rs)
    t0 = time.perf_counter()
    orc.md_run(pb, mp, np.zeros_like(p0), p0, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": N * Rs * T / dt, "unit": "spin-updates/s", "cores": min(threads, Rs),
            "kind": "oracle",
            "sample": f"MD only: {Rs} replicas x {T} steps of the ER N={N} instance, FP64, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="fp8", choices=["fp8", "bf16", "f32"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this build runs on one GPU only: the method's replicas shard trivially, but no "
              "multi-GPU path is built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2004_03972_amd import hqa, instances as inst
    hqa.lib()
    torch.cuda.set_device(0)
    J = inst.er_maxcut(N, P_EDGE, INSTANCE_SEED)
    prob = hqa.Problem(J)
    _log(f"bench: ER N={N} p={P_EDGE} R={R} T={T}; chosen={args.prec}")
    chosen = run_form(hqa, torch, prob, args.prec, args.steps, args.warmup)
    _log("chosen done", chosen["total_ms"], "ms")
    ref = None
    if not args.no_fp32 and args.prec != "f32":
        ref = run_form(hqa, torch, prob, "f32", args.steps, args.warmup)
        _log("fp32 done", ref["total_ms"], "ms")
    upd = N * R * T
    value = upd * args.steps / (chosen["total_ms"] / 1e3)
    md_ms = float(np.mean(chosen["md_ms"]))
    flop_per_launch = 2.0 * N * N * R                  # field contraction of one MD step
    launch_s = md_ms / 1e3 / T                         # one launch per MD step
    achieved = flop_per_launch / launch_s
    peak = PEAK[args.prec]
    out = {
        "metric": "MD spin-updates/s (N×replicas×steps) at matched best cut; "
                  "plain FP32 vs chosen",
        "value": value, "unit": "spin-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": chosen["total_ms"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if args.prec != "f32" else "f32", "data": "synthetic",
        "config": {"workload": f"ER MAX-CUT G({N},{P_EDGE}) w=+1 -> J=+w, R={R}, T={T}, "
                               f"W={W}, n={N_AMB} exact; J {args.prec}",
                   "N": N, "replicas": R, "md_steps": T, "n_amb": N_AMB,
                   "precision": args.prec, "parallelism": "none (1 GPU)"},
        "md_only_spin_updates_per_s": upd / (md_ms / 1e3),
        "best_cut": {"chosen_hqa": chosen["best_cut"], "chosen_md_alone": chosen["best_cut_md"]},
        "split": chosen["split"],
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "kernel": "k_step_dense (field + leapfrog)",
                     "flop_per_launch": flop_per_launch, "launch_ms": launch_s * 1e3},
    }
    if ref is not None:
        rv = upd * args.steps / (ref["total_ms"] / 1e3)
        ratio = [c / f for c, f in zip(chosen["best_cut"], ref["best_cut"])]
        out["fp32"] = {"value": rv, "ms_per_step": ref["total_ms"] / args.steps,
                       "md_only_spin_updates_per_s": upd / (np.mean(ref["md_ms"]) / 1e3),
                       "best_cut_hqa": ref["best_cut"]}
        out["speedup_vs_fp32"] = value / rv
        out["matched_cut"] = {"min_ratio": min(ratio), "bar": 0.999, "ok": min(ratio) >= 0.999}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
