"""HQA-MD throughput on one MI355X: MD spin-updates/s, plain FP32 vs the chosen form.

Default workload (the bench line): a batch of 512 uneven dense instances, 256
Sherrington-Kirkpatrick glasses (N ~ U{100..2000}, J ~ N(0, 1/N), couplings stored in
BF16) and 256 Erdos-Renyi MAX-CUT graphs (N ~ U{500..5000}, p ~ U[0.01, 0.1], unit
weights J = +w stored exactly in FP8 e4m3), 64 replicas each, 5000 MD steps (paper
schedule, M = 6, W = 100), n = 20 ambivalent spins of every replica solved exactly.
One bench step is one pass of the whole hot path over the batch: reset of the initial
state, T MD steps of all 512 instances (field on MFMA with BF16 flux operands and FP32
accumulation, fused leapfrog and window sum), then for every instance the
frozen/ambivalent sort, the reduced problem, the exact enumeration, merge and exact
energies/cuts.  value = sum_k N_k * R * T * steps / time.  The same instances and
initial momenta run in plain FP32 (FP32 couplings, FP32 MFMA) for the first seeds; the
line reports the best-cut ratio per instance and seed, the field error of every
instance against binary64, the trajectory divergence from the FP64 oracle on a
stratified sample, and the oracle's own rate on that sample.

Other workloads (measurement lines for the design notes, not the bench line):
  --workload er800     ER MAX-CUT G(800, 0.06), R = 256, T = 5000, FP8 / BF16 / FP32
  --workload ea3d      3D +-J lattice 16^3, CSR FP32, R = 1024, T = 10000
  --workload es        learned early stop: train on ER runs, evaluate on ER N = 10^4
  --workload k2000     MAX-CUT on K_2000 with +-1 weights: deviation from C* vs MD steps
                       (MD alone, HQA with n = 20 exact, HQA with the n = 1000 tabu search)
  --workload glass     spin glass with fields, N = 1000, 2000, 10^4: energy vs MD steps
  --workload dense8k   enlarged dense shape N = 8192, R = 512 (BF16 SK, FP8 +-1): MFMA fraction
  --workload sweep     kappa2 and M sweeps on the spin glass with fields, N = 10^4
  --workload copy      a plain device copy of known size (HBM counter calibration)

  python bench.py [--steps K] [--warmup W] [--no-cpu] [--workload ...]
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
PEAK_MFMA = {"bf16": 2.5e15, "fp8": 2.5e15, "f32": 157.3e12}   # dense FLOP/s of the MFMA used
HBM_PEAK = 8.0e12
METRIC = "MD spin-updates/s (N×replicas×steps) at matched best cut; plain FP32 vs chosen"


JT_NAME = {"f32": 0, "bf16": 1, "fp8": 2}


def measured_traffic(name, sources="dense", kernel=None):
    """HBM bytes per launch from a committed PMC summary (FETCH_SIZE and WRITE_SIZE in KiB
    per dispatch, each scaled by the factor a plain copy of known size gives), or None when
    the summary is missing, was taken for another kernel instance than `kernel`, or the
    kernel changed since the counters were taken: its gfx950 machine code in the loaded
    library (isa_sha256, when the summary stores one), else its sources (source_sha256)."""
    from paper_2004_03972_amd import profsum
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if kernel is not None and f"hqa::{kernel}(" not in text:
        return None
    kv = {}
    for line in text.splitlines():
        if ":" in line and not line.startswith((" ", "#", "$")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if "isa_sha256" in kv:
            if kernel is None or kv["isa_sha256"] != profsum.isa_hash(kernel):
                return None
        elif kv.get("source_sha256") != profsum.source_hash(profsum.SOURCES[sources]):
            return None
        return (float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_factor"])
                + float(kv["write_kib_per_dispatch"]) * float(kv["write_factor"])) * 1024.0
    except (KeyError, ValueError):
        return None


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def run_form(hqa, torch, prob, prec, steps, warmup, pin=None):
    """Timed bench steps of one precision; returns times and read-out quality."""
    stream = torch.cuda.current_stream()
    md = hqa.MD(prob, hqa.make_schedule(T, W), R, prec, seed=RUN_SEED, require_exact=True,
                stream=stream.cuda_stream)
    if pin:                                        # a fixed per-step block (profiling runs)
        md.set_step_tiles(*pin)
    else:
        md.tune(50)                                # plan and tile shape, untimed
    plan = md.tuned_plan()
    for k in range(warmup):
        md.reset(RUN_SEED + 1000 + k)
        md.run()
        md.classify(N_AMB, solve=True)
    torch.cuda.synchronize()
    best_cut, best_md, md_ms, split = [], [], [], None
    t0, t1 = _events(torch)
    t0.record(stream)
    for k in range(steps):
        md.reset(RUN_SEED + k)
        e0, e1 = _events(torch)
        e0.record(stream)
        md.run()
        e1.record(stream)
        g = md.classify(N_AMB, solve=True)          # synchronises
        md_ms.append(e0.elapsed_time(e1))
        best_cut.append(float(g["cut"].max()))
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    # MD-alone read-out of the last step (outside the timed region)
    g0 = md.classify(N_AMB, solve=False)
    best_md.append(float(g0["cut"].max()))
    split = {"n_frozen": N - N_AMB, "n_ambivalent": N_AMB,
             "mean_abs_phibar_frozen": None}
    md.close()
    return dict(total_ms=total_ms, md_ms=md_ms, best_cut=best_cut, best_cut_md_alone=best_md,
                split=split, plan=plan)


def cpu_baseline():
    """The FP64 oracle on a bounded sample: 64 replicas x 5000 steps of the same instance
    (about 10-20 s on 16 host cores)."""
    import oracle as orc
    from paper_2004_03972_amd import instances as inst
    threads = max(1, min(16, os.cpu_count() or 1))
    Rs = 64
    J = inst.er_maxcut(N, P_EDGE, INSTANCE_SEED)
    pb = orc.Problem(N, J=J)
    mp = orc.MDParams(T=T, W=W)
    p0 = orc.init_p0(RUN_SEED, N, Rs)
    t0 = time.perf_counter()
    orc.md_run(pb, mp, np.zeros_like(p0), p0, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": N * Rs * T / dt, "unit": "spin-updates/s", "cores": min(threads, Rs),
            "kind": "oracle",
            "sample": f"MD only: {Rs} of the {R} replicas x all {T} steps of the ER N={N} "
                      f"instance, FP64 oracle, {dt:.1f} s"}


def bench_er800(args, hqa, torch):
    from paper_2004_03972_amd import instances as inst
    J = inst.er_maxcut(N, P_EDGE, INSTANCE_SEED)
    prob = hqa.Problem(J)
    forms = {}
    for prec in args.forms:
        _log(f"bench: ER N={N} p={P_EDGE} R={R} T={T}; form {prec}")
        forms[prec] = run_form(hqa, torch, prob, prec, args.steps, args.warmup, args.pin)
        _log(f"  {prec}: {forms[prec]['total_ms']:.1f} ms for {args.steps} steps")
    upd = N * R * T
    val = {p: upd * args.steps / (f["total_ms"] / 1e3) for p, f in forms.items()}
    # the chosen form: exact FP8 e4m3 storage of the unit weights (BF16 MFMA operands);
    # BF16 storage is reported beside it
    lowp = [p for p in ("fp8", "bf16") if p in forms]
    chosen = lowp[0] if lowp else "f32"
    c = forms[chosen]
    md_ms = float(np.mean(c["md_ms"]))
    plan, tm, tn, cb, tj = c["plan"]
    if plan == "resident":                      # two launches: before and inside the window
        kernel = f"k_md_resident<{JT_NAME[chosen]}, {2 if chosen == 'fp8' else 1}, false, 6>"
        launches, srcs = 2, "resident"
    elif plan == "cluster":                     # one cooperative launch for all steps
        np_ = -(-N // 128) * 128
        kernel = (f"k_persist_rj<{JT_NAME[chosen]}, {np_ // 128}, 6>" if chosen != "f32" and np_ <= 1024
                  else f"k_persist<{JT_NAME[chosen]}")
        launches, srcs = 1, "persist"
    else:                                       # one launch per MD step
        kernel = (f"k_step_block<{JT_NAME[chosen]}, {tm or 2}, {tn or 4}, false, {cb or 4}, "
                  f"{'true' if tj else 'false'}>")
        launches, srcs = T, "dense"
    flop_per_launch = 2.0 * N * N * R * T / launches   # field contraction (2 N^2 R per step)
    launch_s = md_ms / 1e3 / launches
    achieved = flop_per_launch / launch_s
    peak = PEAK_MFMA[chosen]
    out = {
        "metric": METRIC, "value": val[chosen], "unit": "spin-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": c["total_ms"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if chosen != "f32" else "f32", "data": "synthetic",
        "config": {"workload": f"ER MAX-CUT G({N},{P_EDGE}) unit weights, J=+w, R={R} replicas, "
                               f"T={T} MD steps, W={W}, n={N_AMB} exact; J storage {chosen}",
                   "N": N, "replicas": R, "md_steps": T, "n_amb": N_AMB,
                   "j_storage": chosen, "parallelism": "none (1 GPU)"},
        "md_only_spin_updates_per_s": upd / (md_ms / 1e3),
        "best_cut": {"chosen_hqa": c["best_cut"], "chosen_md_alone_last": c["best_cut_md_alone"]},
        "split": c["split"],
        "forms": {p: {"value": val[p], "ms_per_step": f["total_ms"] / args.steps,
                      "md_ms": float(np.mean(f["md_ms"])), "best_cut_hqa": f["best_cut"],
                      "plan": f["plan"]}
                  for p, f in forms.items()},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic(f"{kernel.split('<')[0]}_{chosen}_er800_pmc.txt",
                                                 srcs, kernel),
                     "kernel": kernel, "plan": plan,
                     "flop_per_launch": flop_per_launch, "launch_us": launch_s * 1e6},
    }
    if "f32" in forms and chosen != "f32":
        ratio = [a / b for a, b in zip(c["best_cut"], forms["f32"]["best_cut"])]
        out["fp32"] = {"value": val["f32"], "best_cut_hqa": forms["f32"]["best_cut"]}
        out["speedup_vs_fp32"] = val[chosen] / val["f32"]
        out["matched_cut"] = {"min_ratio": min(ratio), "bar": 0.999, "ok": min(ratio) >= 0.999}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    return out


def bench_ea3d(args, hqa, torch):
    """3D +-J lattice 16^3, CSR FP32, 1024 replicas, 10000 steps (measurement line)."""
    from paper_2004_03972_amd import instances as inst
    L, Rr, Tt = 16, 1024, 10000
    rp, ci, v = inst.ea3d(L, 301)
    Nn = L ** 3
    st = torch.cuda.current_stream()
    md = hqa.MD(hqa.Problem(row_ptr=rp, col=ci, val=v), hqa.make_schedule(Tt, 100), Rr, "f32",
                seed=3, stream=st.cuda_stream)
    if args.pin:                                  # profiling runs: the resident plan, untuned
        md.close()
        md = hqa.MD(hqa.Problem(row_ptr=rp, col=ci, val=v), hqa.make_schedule(Tt, 100), Rr,
                    "f32", seed=3, stream=st.cuda_stream, plan="resident")
        plan = "resident"
    else:
        md.tune(20)                               # per-step vs replica-resident, untimed
        plan = md.tuned_plan()[0]
    md.run(); md.sync()
    times = []
    for k in range(args.steps):
        md.reset(3 + k)
        e0, e1 = _events(torch)
        e0.record(st); md.run(); e1.record(st)
        g = md.classify(20, solve=True)
        times.append(e0.elapsed_time(e1))
    ms = float(np.mean(times))
    upd = Nn * Rr * Tt
    bytes_alg = 16.0 * upd + 8.0 * v.size * Tt + 8.0 * Nn * Rr * 100   # state + J + window
    out = {"metric": "MD spin-updates/s", "workload": "EA 3D +-J 16^3 CSR FP32, R=1024, T=10000",
           "value": upd / (ms / 1e3), "unit": "spin-updates/s", "md_ms": ms, "plan": plan,
           "best_energy": float(g["energy"].min())}
    if plan == "resident":
        # state stays on chip: bound by FP32 vector arithmetic (2 flop per coupling for the
        # field, 17 for the leapfrog, per spin-update).  Peak: 256 CUs x 4 SIMDs x 16 lanes
        # x 2 flop (FMA) x 2.4 GHz = 78.6 TFLOP/s of unpacked FP32, the rate this build can
        # reach (packed FP32, which the vendor's 157.3 counts, is not emitted)
        flop = (2.0 * v.size / Nn + 17.0) * upd
        out["roofline"] = {"bound": "alu", "achieved": flop / (ms / 1e3) / 1e12,
                           "peak": 78.6, "unit": "TFLOP/s",
                           "frac": flop / (ms / 1e3) / 78.6e12,
                           "frac_of_vendor_157": flop / (ms / 1e3) / 157.3e12,
                           "traffic": measured_traffic("k_csr_resident_ea3d_pmc.txt",
                                                       "csr_resident", "k_csr_resident<4, 6>"),
                           "kernel": "k_csr_resident<4, 6>", "flop_per_update": flop / upd,
                           "hbm_equivalent_GBps": bytes_alg / (ms / 1e3) / 1e9}
    else:
        out["roofline"] = {"bound": "hbm", "achieved": bytes_alg / (ms / 1e3) / 1e9,
                           "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                           "frac": bytes_alg / (ms / 1e3) / HBM_PEAK,
                           "traffic": measured_traffic("k_step_csr_ea3d_pmc.txt", "csr"),
                           "kernel": "k_step_csr", "bytes_per_update": bytes_alg / upd}
    return out


BATCH_R, BATCH_T, BATCH_N_AMB, BATCH_SEED = 64, 5000, 20, 4
BATCH_WORKLOAD = ("512 uneven dense instances: 256 SK N~U{100..2000} J~N(0,1/N) stored BF16, "
                  "256 ER MAX-CUT N~U{500..5000} p~U[0.01,0.1] unit weights J=+w stored FP8 "
                  "e4m3 (exact) and streamed one bit per coupling; R=64 replicas each, T=5000 "
                  "MD steps, W=100, n=20 exact")


FORM_BYTES = {"f32": 4.0, "bf16": 2.0, "fp8": 1.0, "bit": 0.125}


def batch_bytes_per_step(specs, R, W, T, forms=None):
    """Algorithmic HBM bytes of one MD step of the batch: every coupling once in the form the
    batch plan streams it (`forms`, from the library: BF16 2 B, FP8 1 B, one bit for 0/1
    couplings; without it BF16 for SK and FP8 for ER), and per spin-update 20 B of state
    (flux in 4, momentum in 4 and out 4, new flux out 4, its BF16 operand copy out 2 and in
    2 as the MFMA operand), plus the window sum (in 4, out 4) on W of the T steps."""
    if forms is None:
        forms = ["bf16" if fam == "sk" else "fp8" for fam, _, _, _ in specs]
    j = sum(N * N * FORM_BYTES[f] for (_, N, _, _), f in zip(specs, forms))
    upd = sum(N for _, N, _, _ in specs) * R
    return j + upd * (20.0 + 8.0 * W / T), j, upd


def classify_batch(md, K, n_amb):
    """Exact HQA read-out of every instance (one hqa_classify_many call): best cut and best
    energy over the replicas."""
    en, cut = md.classify_many(n_amb, solve=True)
    assert en.shape[0] == K
    return cut.max(axis=1), en.min(axis=1)


def cpu_baseline_batch(specs, Js, chosen, fp32, torch, rs=4, ts=500, checkpoints=(1, 10, 100, 500)):
    """The FP64 oracle on a bounded sample of the batch: the stratified 16 instances (8 SK,
    8 ER spread over the size range), the first `rs` replicas of each (the same initial
    momenta as the GPU runs), `ts` MD steps, (instance, replica) items on 16 host threads;
    then a one-thread figure on one replica of each for ts/10 steps.  The oracle's fluxes at
    the checkpoints give the trajectory divergence of the GPU forms (same initial momenta,
    same steps): max |phi_form - phi_64| per checkpoint, over the sample."""
    import oracle as orc
    from concurrent.futures import ThreadPoolExecutor
    from paper_2004_03972_amd import instances as inst
    strat = inst.stratified(specs)
    threads = 16
    seed = BATCH_SEED + 7
    mp = orc.MDParams(T=BATCH_T, W=100)
    items = []
    for k in strat:
        N = specs[k][1]
        pb = orc.Problem(N, J=Js[k])
        p0 = orc.init_p0(seed, N, rs)
        for r in range(rs):
            items.append((k, r, pb, p0[r:r + 1].copy()))
    traj = {}

    def one(it, steps, keep):
        k, r, pb, p0 = it
        phi, p = np.zeros_like(p0), p0.copy()
        q = 0
        out = {}
        for c in [c for c in checkpoints if c <= steps] + [steps]:
            if c > q:
                orc.md_advance(pb, mp, phi, p, None, q, c, nthreads=1)
                q = c
            if keep:
                out[c] = phi[0].copy()
        return (k, r), out

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for key, out in ex.map(lambda it: one(it, ts, True), items):
            traj[key] = out
    dt = time.perf_counter() - t0
    upd = sum(specs[k][1] for k, _, _, _ in items) * ts
    t1 = time.perf_counter()
    one1 = [it for it in items if it[1] == 0]
    for it in one1:
        one(it, ts // 10, False)
    dt1 = time.perf_counter() - t1
    upd1 = sum(specs[k][1] for k, _, _, _ in one1) * (ts // 10)
    # divergence of the GPU forms from the oracle on the same sample
    div = {}
    for name, md in (("chosen", chosen), ("fp32", fp32)):
        if md is None:
            continue
        md.reset(seed)
        q = 0
        rows = {c: {"sk": 0.0, "er": 0.0} for c in checkpoints if c <= ts}
        for c in sorted(rows):
            md.run(c)
            for k in strat:
                ph = md.state(0, k=k)[:rs]
                fam = specs[k][0]
                d = max(float(np.max(np.abs(ph[r] - traj[(k, r)][c]))) for r in range(rs))
                rows[c][fam] = max(rows[c][fam], d)
        div[name] = {str(c): v for c, v in rows.items()}
        md.reset(BATCH_SEED)
    return {"value": upd / dt, "unit": "spin-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"stratified 16 of the 512 instances (8 SK, 8 ER, N {min(specs[k][1] for k in strat)}"
                      f"..{max(specs[k][1] for k in strat)}), {rs} replicas each, {ts} of the "
                      f"{BATCH_T} MD steps, FP64 oracle, {dt:.1f} s",
            "single_thread": {"value": upd1 / dt1, "cores": 1,
                              "sample": f"the same 16 instances, 1 replica, {ts // 10} steps, "
                                        f"{dt1:.1f} s"}}, \
        {"measure": "max over the stratified sample of max_i |phi_i^(m) - phi64_i^(m)| at step m "
                    "(same initial momenta), by family; chosen = BF16 operands with BF16 (SK) or "
                    "FP8 (ER) couplings", "replicas": rs, **div}


def bench_batch(args, hqa, torch):
    """The bench line: the uneven batch of 512 dense instances (BF16 SK and exact FP8 ER
    couplings, BF16 flux operands, FP32 accumulation and state), R = 64, T = 5000, against
    plain FP32 on the same instances and initial momenta."""
    from paper_2004_03972_amd import instances as inst
    K = args.instances
    specs = inst.uneven_batch_specs(512)[:K] if K >= 512 else \
        inst.uneven_batch_specs(512)[:K // 2] + inst.uneven_batch_specs(512)[256:256 + K - K // 2]
    Rr, Tt, W = BATCH_R, args.md_steps or BATCH_T, 100
    t0 = time.perf_counter()
    Js = [inst.uneven_batch_instance(s) for s in specs]
    _log(f"bench: generated {len(specs)} instances in {time.perf_counter() - t0:.1f} s")
    Kn = len(specs)
    st = torch.cuda.current_stream()
    sched = hqa.make_schedule(Tt, W)
    probs = [hqa.Problem(J, storage="bf16" if s[0] == "sk" else "fp8") for J, s in zip(Js, specs)]
    # each run's 5000 step launches are replayed from one captured HIP graph (captured in
    # the untimed warm-up; --eager launches them one by one)
    md = hqa.MD(probs, sched, Rr, "bf16", seed=BATCH_SEED, stream=st.cuda_stream,
                graph=not args.eager)
    # exactness of the FP8 storage of the unit weights, and the BF16 rounding of SK
    jerr = {"er_fp8_exact": True, "sk_bf16_max_rel": 0.0}
    for J, s in zip(Js, specs):
        if s[0] == "sk":
            Jb = torch.from_numpy(J).to(torch.bfloat16).double().numpy()
            jerr["sk_bf16_max_rel"] = max(jerr["sk_bf16_max_rel"],
                                          float(np.max(np.abs(Jb - J)) / np.max(np.abs(J))))
        else:
            jerr["er_fp8_exact"] &= bool(np.all((J == 0) | (J == 1)))
    md.run(min(Tt, 10)); md.sync()
    for w in range(args.warmup):
        md.reset(BATCH_SEED + 1000 + w)
        md.run()
        classify_batch(md, Kn, BATCH_N_AMB)
    torch.cuda.synchronize()
    cut_c, en_c, md_ms = [], [], []
    t0e, t1e = _events(torch)
    t0e.record(st)
    for k in range(args.steps):
        md.reset(BATCH_SEED + k)
        e0, e1 = _events(torch)
        e0.record(st); md.run(); e1.record(st)
        c, e = classify_batch(md, Kn, BATCH_N_AMB)
        md_ms.append(e0.elapsed_time(e1))
        cut_c.append(c); en_c.append(e)
    t1e.record(st)
    torch.cuda.synchronize()
    total_ms = t0e.elapsed_time(t1e)
    _log(f"  chosen: {total_ms:.1f} ms for {args.steps} steps (MD {np.mean(md_ms):.1f} ms per run)")
    forms = [md.batch_form(k) for k in range(Kn)]
    bytes_step, jbytes, upd_step = batch_bytes_per_step(specs, Rr, W, Tt, forms)
    flop_step = sum(2.0 * N * N * Rr for _, N, _, _ in specs)
    upd_run = upd_step * Tt
    value = upd_run * args.steps / (total_ms / 1e3)
    # max |dh| of every instance: the form's field against binary64 on the final fluxes
    fe = [md.field_error(k) for k in range(Kn)]
    dh = np.array([e for e, _ in fe])
    rel = np.array([e / r if r > 0 else 0.0 for e, r in fe])
    fam = np.array([s[0] for s in specs])
    # plain FP32 on the same instances and seeds (fewer seeds: it is the slow side)
    nf = min(args.steps, args.fp32_seeds)
    cut_f, f_ms = [], None
    md32 = None
    if nf > 0:
        probs32 = [hqa.Problem(J, storage="f32") for J in Js]
        md32 = hqa.MD(probs32, sched, Rr, "f32", seed=BATCH_SEED, stream=st.cuda_stream)
        md32.run(min(Tt, 10)); md32.sync()
        torch.cuda.synchronize()
        a0, a1 = _events(torch)
        a0.record(st)
        for k in range(nf):
            md32.reset(BATCH_SEED + k)
            md32.run()
            c, _ = classify_batch(md32, Kn, BATCH_N_AMB)
            cut_f.append(c)
        a1.record(st)
        torch.cuda.synchronize()
        f_ms = a0.elapsed_time(a1) / nf
        _log(f"  fp32: {f_ms:.1f} ms per step over {nf} seeds")
    out = {
        "metric": METRIC, "value": value, "unit": "spin-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total_ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": BATCH_WORKLOAD if Kn == 512 and Tt == BATCH_T else
                   f"{Kn} uneven instances, R={Rr}, T={Tt}", "instances": Kn, "replicas": Rr,
                   "md_steps": Tt, "n_amb": BATCH_N_AMB, "j_storage": "bf16 (SK) / fp8 (ER)",
                   "j_streamed": {f: forms.count(f) for f in sorted(set(forms))},
                   "spin_updates_per_run": upd_run, "parallelism": "none (1 GPU)",
                   "launch": "eager" if args.eager else "one HIP graph per run"},
        "md_only_spin_updates_per_s": upd_run / (np.mean(md_ms) / 1e3),
        "j_storage_error": jerr,
        "max_abs_dh": {"measure": "per instance max|u_form - u_64| / max|u_64| (and absolute) on "
                                  "the final fluxes; the binary64 field is sum_j J_ij phi_j",
                       "sk_bf16": {"max_rel": float(rel[fam == "sk"].max()),
                                   "median_rel": float(np.median(rel[fam == "sk"])),
                                   "max_abs": float(dh[fam == "sk"].max())},
                       "er_fp8": {"max_rel": float(rel[fam == "er"].max()),
                                  "median_rel": float(np.median(rel[fam == "er"])),
                                  "max_abs": float(dh[fam == "er"].max())},
                       "instances": Kn},
    }
    if nf > 0:
        ratios = np.array([cut_c[k] / cut_f[k] for k in range(nf)])        # [seed][instance]
        worst = np.unravel_index(np.argmin(ratios), ratios.shape)
        per_inst = ratios.mean(axis=0)
        mean = float(per_inst.mean())
        half = 1.96 * float(per_inst.std(ddof=1)) / np.sqrt(per_inst.size) if per_inst.size > 1 else 0.0
        out["fp32"] = {"value": upd_run / (f_ms / 1e3), "ms_per_step": f_ms, "seeds": nf}
        out["speedup_vs_fp32"] = value / out["fp32"]["value"]
        mc = {
            "bar": 0.999,
            "reading": "best cut over the replicas, chosen form / plain FP32 with the same "
                       "initial momenta, per instance and seed; the two forms' trajectories "
                       "diverge chaotically within a few hundred steps, so one pair compares "
                       "two samples of the same distribution: the bar is applied to the mean "
                       "over the batch (95% interval), and the per-pair spread is set "
                       "against FP32's own spread between two seeds",
            "pairs": int(ratios.size), "seeds": nf,
            "mean_ratio": mean, "mean_ratio_ci95": [mean - half, mean + half],
            "min_ratio": float(ratios.min()),
            "quantiles_1_5_50": [float(np.quantile(ratios, q)) for q in (0.01, 0.05, 0.5)],
            "sk_min": float(ratios[:, fam == "sk"].min()),
            "er_min": float(ratios[:, fam == "er"].min()),
            "sk_mean": float(ratios[:, fam == "sk"].mean()),
            "er_mean": float(ratios[:, fam == "er"].mean()),
            "chosen_better_or_equal": int(np.sum(ratios >= 1.0)),
            "pairs_below_bar": int(np.sum(ratios < 0.999)),
            "worst": {"instance": int(worst[1]), "family": specs[worst[1]][0],
                      "N": specs[worst[1]][1], "seed": BATCH_SEED + int(worst[0]),
                      "chosen": float(cut_c[worst[0]][worst[1]]),
                      "fp32": float(cut_f[worst[0]][worst[1]])},
            "ok": bool(mean - half >= 0.999), "every_pair_ok": bool(ratios.min() >= 0.999)}
        if nf >= 2:
            noise = cut_f[1] / cut_f[0]
            mc["fp32_seed_to_seed"] = {
                "min_ratio": float(noise.min()),
                "quantiles_1_5_50": [float(np.quantile(noise, q)) for q in (0.01, 0.05, 0.5)],
                "sk_min": float(noise[fam == "sk"].min()), "er_min": float(noise[fam == "er"].min()),
                "pairs_below_bar": int(np.sum(np.minimum(noise, 1.0 / noise) < 0.999))}
        out["matched_cut"] = mc
        if args.detail:
            with open(args.detail, "w") as fh:
                json.dump({"specs": specs, "cut_chosen": [c.tolist() for c in cut_c],
                           "cut_fp32": [c.tolist() for c in cut_f],
                           "dh_abs": dh.tolist(), "dh_rel": rel.tolist()}, fh)
    launch_s = float(np.mean(md_ms)) / 1e3 / Tt       # one launch per MD step
    out["roofline"] = {"bound": "hbm", "achieved": bytes_step / launch_s / 1e9, "peak": 8000.0,
                       "unit": "GB/s", "frac": bytes_step / launch_s / 8.0e12,
                       "traffic": measured_traffic("k_step_batch_lds_batch512_pmc.txt", "batch",
                                                   "k_step_batch_lds"),
                       "kernel": "k_step_batch_lds", "launches_per_run": Tt,
                       "bytes_per_launch": bytes_step, "j_bytes_per_launch": jbytes,
                       "launch_us": launch_s * 1e6,
                       "mfma_tflops": flop_step / launch_s / 1e12,
                       "mfma_frac_bf16": flop_step / launch_s / 2.5e15}
    if not args.no_cpu:
        cb, div = cpu_baseline_batch(specs, Js, md, md32, torch)
        out["cpu_baseline"] = cb
        out["divergence"] = div
    if md32 is not None:
        md32.close()
    md.close()
    return out


def bench_es(args, hqa, torch):
    """Learned early stop on sparse ER MAX-CUT: train on runs of the method itself
    (N ~ U{1000..4000}, mean degree ~ U[20, 100], T = 20000, checkpoints every K = 1000
    steps with statistics sampled every 10th step of the last Ks = 100 steps before each),
    calibrate the stop threshold on validation runs (by default: the smallest threshold
    at which the read-out at the stop loses at most --es-target-cut of the full run's best
    cut on every validation run), then evaluate on ER N = 10^4, p = 0.005 (mean degree
    ~50), R = 128: stop step, mislabel rate and best cut against the full run, and the
    truncation ablation at the same step."""
    from paper_2004_03972_amd import early_stop as E
    from paper_2004_03972_amd import instances as inst
    Tt, K, Ks = 20000, args.es_k, args.es_ks
    nck = Tt // K
    sched = hqa.make_schedule(Tt, 100)
    rng = np.random.default_rng(5)
    t0 = time.perf_counter()
    recs = []
    # training runs: es_train instances x es_train_r replicas (each replica is one run
    # of the method from its own initial momenta); a fraction es_keep of the (replica,
    # spin) samples of every second checkpoint is kept for training
    ntrain, nval, Rt = args.es_train, 8, args.es_train_r
    for k in range(ntrain + nval):
        Nk = int(rng.integers(1000, 4001))
        d = float(rng.uniform(20, 100))
        rp, ci, v = inst.er_sparse(Nk, d, 5_000_000 + k)
        n_lab = max(1, round(0.05 * Nk))
        train = k < ntrain
        rec = E.record_run(hqa.Problem(row_ptr=rp, col=ci, val=v), sched, Rt if train else 4,
                           K, nck, seed=100 + k, n_amb=n_lab, every=2 if train else 1, Ks=Ks,
                           stride=args.es_stride, keep=args.es_keep if train else 1.0,
                           keep_seed=k, means=not train, solve_n=0 if train else 20)
        if train:
            rec.md.close()                    # validation handles stay open for calibration
        recs.append(rec)
        if k % 32 == 31:
            _log(f"  recorded {k + 1} instances, {time.perf_counter() - t0:.1f} s")
    record_s = time.perf_counter() - t0
    X, y = E.dataset(recs[:ntrain])
    es = hqa.ES(seed=1)
    t1 = time.perf_counter()
    losses = E.train(es, X, y, epochs=2, batch=16384, lr=2e-3, log=_log)
    train_s = time.perf_counter() - t1
    # the threshold: on the validation runs, the read-out at the stop loses at most
    # --es-target-cut of the full run's best cut (default), or the labels at the stop are
    # wrong for at most --es-target of the spins
    if args.es_calibrate == "cut":
        thr = E.calibrate_cut(es, recs[ntrain:], target_loss=args.es_target_cut, n_amb=20)
        calib = {"by": "cut loss of the read-out at the stop", "target": args.es_target_cut,
                 "validation_runs": 4 * nval}
    else:
        thr = E.calibrate(es, recs[ntrain:], target_mislabel=args.es_target)
        calib = {"by": "mislabel rate at the stop", "target": args.es_target,
                 "validation_runs": 4 * nval}
    for rec in recs[ntrain:]:
        rec.md.close()
    _log(f"  trained on {X.shape[0]} samples in {train_s:.1f} s, threshold {thr:.4f}")
    # evaluation instance: ER N = 10^4, p = 0.005
    Ne, Re = 10000, 128
    rp, ci, v = inst.er_sparse(Ne, 0.005 * (Ne - 1), 5001)
    prob = hqa.Problem(row_ptr=rp, col=ci, val=v)
    n_lab = round(0.05 * Ne)
    # the full run's labels (the reference for the mislabel rate), untimed
    full = E.record_run(prob, sched, Re, K, nck, seed=7, n_amb=n_lab, solve_n=20, every=nck,
                        Ks=Ks, stride=args.es_stride)
    full.md.close()
    # timed: the method alone on both sides -- MD to T and the exact read-out, against
    # checkpointed MD to the learned stop and the read-out from the predicted labels
    # (the ablation and the mislabel counts are evaluated outside both timings)
    md = hqa.MD(prob, sched, Re, "f32", seed=7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    md.run()
    md.classify(20, solve=True)
    full_ms = (time.perf_counter() - t0) * 1e3
    md.close()
    res = E.run_with_early_stop(es, prob, sched, Re, K, thr if np.isfinite(thr) else 1.1,
                                n_amb=20, seed=7, labels=full.labels, n_label=n_lab, Ks=Ks,
                                stride=args.es_stride)
    es_ms = res.wall_ms
    cut_full = float(full.full["cut"].max())
    cut_es = float(res.readout["cut"].max())
    cut_tr = float(res.ablation["cut"].max())
    return {"metric": "learned early stop: speedup T/K_stop at cut loss", "workload":
            f"train {ntrain * Rt} ER runs ({ntrain} instances N 1000..4000, d 20..100, x {Rt} "
            f"replicas, T={Tt}, K={K}, Ks={Ks}, stride {args.es_stride}, {args.es_keep:g} of "
            f"the samples kept); eval ER N={Ne} p=0.005 R={Re} T={Tt}, n=20 exact",
            "train_runs": ntrain * Rt, "record_s": record_s,
            "train_samples": int(X.shape[0]), "train_s": train_s,
            "loss_first_last": [float(np.mean(losses[:20])), float(np.mean(losses[-20:]))],
            "threshold": thr, "calibration": calib,
            "stop_step": res.stop_step, "speedup_steps": Tt / res.stop_step,
            "wall_ms_full": full_ms, "wall_ms_early": es_ms, "speedup_wall": full_ms / es_ms,
            "mislabel": {"network": res.mislabel, "truncation_same_step": res.mislabel_ablation},
            "best_cut": {"full_run_hqa": cut_full, "early_stop_hqa": cut_es,
                         "truncation_hqa": cut_tr,
                         "loss_vs_full": (cut_full - cut_es) / cut_full}}


def bench_k2000(args, hqa, torch):
    """MAX-CUT on K_2000 with +-1 weights (the paper's headline experiment): J = +w stored
    exactly in FP8, each instance and its mirror -J, R replicas, MD alone (sign of
    phibar), HQA with n = 20 solved exactly and HQA with the n most ambivalent spins
    handed to the tabu search.  Deviation from the theoretical maximum cut C* = 33,932.6
    (recomputed from the paper's formula, see tests/golden/kn_maxcut_cstar.txt), for
    replica 0 (one initial condition per instance, as in the paper) and for the best of
    the R replicas.  --k2000-group instances (instance and mirror pairs) share one
    handle and one cluster launch, each 16-replica cluster on its own XCD; the
    initial momenta come from the seed 11 + (first instance of the group)."""
    from paper_2004_03972_amd import instances as inst
    Nk, Rr, cstar = 2000, args.k2000_replicas, 33932.6
    pairs = max(1, args.k2000_group // 2)
    out = {"metric": "MAX-CUT deviation from C* (K2000, +-1 weights)", "C_star": cstar,
           "instances": args.k2000_instances, "first_instance": args.k2000_first,
           "mirrors": True, "replicas": Rr, "handle_group": 2 * pairs, "by_T": {}}
    st = torch.cuda.current_stream()
    ks_all = list(range(args.k2000_first, args.k2000_first + args.k2000_instances))
    for Tt in [int(x) for x in args.k2000_steps.split(",")]:
        dev = {"md_one_init": [], "hqa_one_init": [], "md_best": [], "hqa_best": [],
               "hqa_ts_one_init": [], "hqa_ts_best": []}
        ms_tot = ts_tot = 0.0
        for g in range(0, len(ks_all), pairs):
            ks = ks_all[g:g + pairs]
            Js = []
            for k in ks:
                J = inst.pm_complete(Nk, 9000 + k)
                Js += [J, -J]
            md = hqa.MD([hqa.Problem(J) for J in Js], hqa.make_schedule(Tt, 100), Rr, "fp8",
                        seed=11 + ks[0], require_exact=True, stream=st.cuda_stream,
                        plan="cluster")
            e0, e1 = _events(torch)
            e0.record(st); md.run(); e1.record(st); md.sync()
            ms_tot += e0.elapsed_time(e1)
            for kk in range(len(Js)):
                g0 = md.classify(20, solve=False, k=kk)
                g1 = md.classify(20, solve=True, k=kk)
                dev["md_one_init"].append((cstar - g0["cut"][0]) / cstar)
                dev["hqa_one_init"].append((cstar - g1["cut"][0]) / cstar)
                dev["md_best"].append((cstar - g0["cut"].max()) / cstar)
                dev["hqa_best"].append((cstar - g1["cut"].max()) / cstar)
                if args.k2000_tabu_iters > 0:
                    t0 = time.perf_counter()
                    g2 = md.classify_tabu(args.k2000_tabu_n, args.k2000_tabu_iters,
                                          args.k2000_tabu_tenure, k=kk)
                    ts_tot += (time.perf_counter() - t0) * 1e3
                    dev["hqa_ts_one_init"].append((cstar - g2["cut"][0]) / cstar)
                    dev["hqa_ts_best"].append((cstar - g2["cut"].max()) / cstar)
            md.close()
            _log(f"  T={Tt}: instances {ks[0]}..{ks[-1]} done")
        runs = 2 * len(ks_all)
        out["by_T"][str(Tt)] = {kk: {"mean": float(np.mean(v)), "min": float(np.min(v)),
                                     "max": float(np.max(v))} for kk, v in dev.items() if v}
        if args.k2000_per_run:
            out["by_T"][str(Tt)]["per_run"] = {kk: [float(x) for x in v] for kk, v in dev.items()}
        out["by_T"][str(Tt)]["md_ms_per_run"] = ms_tot / runs
        if args.k2000_tabu_iters > 0:
            out["by_T"][str(Tt)]["tabu_read_out_ms_per_run"] = ts_tot / runs
    out["tabu"] = {"n": args.k2000_tabu_n, "iters": args.k2000_tabu_iters,
                   "tenure": args.k2000_tabu_tenure}
    out["paper"] = ("MD alone about 0.4% and HQA(TS1000) about 0.2% below C* at 5e5 MD steps "
                    "(one init per instance); TS1000 time about 0.24 of the MD time")
    return out


def bench_glass(args, hqa, torch):
    """Ising spin glass with fields (J_ij ~ U[-1, 1], h_i ~ U[-2, 2], dense, BF16 storage
    of J for the dynamics, exact binary64 energies): mean Ising energy per spin over
    instances against MD steps, for N = 1000, 2000 and 10^4.  Read-outs: MD alone
    (sign of phibar) for replica 0 (one initial condition per instance) and the best
    of R replicas; HQA with the n = 20 most ambivalent spins solved exactly; HQA with
    the n most ambivalent spins (each n of --glass-tabu-n up to N) handed to the tabu
    search for --glass-tabu-sweeps * n moves, tenure n / 20."""
    from paper_2004_03972_amd import instances as inst
    Rr = args.glass_replicas
    tabu_ns = [int(x) for x in args.glass_tabu_n.split(",") if x]
    sizes = [int(x) for x in args.glass_n.split(",")]
    counts = [int(x) for x in args.glass_instances.split(",")]
    steps = [int(x) for x in args.glass_steps.split(",")]
    st = torch.cuda.current_stream()
    out = {"metric": "Ising energy per spin vs MD steps (spin glass with fields)",
           "workload": "J~U[-1,1], h~U[-2,2], dense, BF16 J in the dynamics", "replicas": Rr,
           "by_N": {}}
    for Nn, cnt in zip(sizes, counts):
        rows = {}
        for Tt in steps:
            e = {"md_one_init": [], "md_best": [], "hqa_one_init": [], "hqa_best": []}
            for nt in tabu_ns:
                if nt <= Nn:
                    e[f"hqa_ts{nt}_one_init"], e[f"hqa_ts{nt}_best"] = [], []
            bad_tot, ms_tot = 0, 0.0
            # instances up to 2048 spins advance together in one cluster launch (one
            # 16-replica cluster per instance, each on its own XCD; momenta from one seed);
            # larger ones run alone on the tuner's plan
            groups = [list(range(cnt))] if Nn <= 2048 else [[k] for k in range(cnt)]
            for grp in groups:
                Jh = [inst.uniform_glass(Nn, 7000 + 31 * Nn + k) for k in grp]
                md = hqa.MD([hqa.Problem(J, h=h, storage="bf16") for J, h in Jh],
                            hqa.make_schedule(Tt, 100), Rr, "bf16", seed=40 + grp[0],
                            stream=st.cuda_stream, plan="cluster" if len(grp) > 1 else "auto")
                if len(grp) == 1:
                    md.tune(max(20, min(100, Tt // 10)))
                e0, e1 = _events(torch)
                e0.record(st); md.run(); e1.record(st); st.synchronize()
                ms_tot += e0.elapsed_time(e1)
                for kk in range(len(grp)):
                    bad = int(np.sum(~np.isfinite(md.hamiltonian(kk))))
                    bad_tot += bad
                    if bad:
                        continue
                    g0 = md.classify(20, solve=False, k=kk)
                    g1 = md.classify(20, solve=True, k=kk)
                    e["md_one_init"].append(g0["energy"][0] / Nn)
                    e["md_best"].append(g0["energy"].min() / Nn)
                    e["hqa_one_init"].append(g1["energy"][0] / Nn)
                    e["hqa_best"].append(g1["energy"].min() / Nn)
                    for nt in tabu_ns:
                        if nt <= Nn:
                            g2 = md.classify_tabu(nt, args.glass_tabu_sweeps * nt, max(1, nt // 20),
                                                  k=kk)
                            e[f"hqa_ts{nt}_one_init"].append(g2["energy"][0] / Nn)
                            e[f"hqa_ts{nt}_best"].append(g2["energy"].min() / Nn)
                md.close()
            rows[str(Tt)] = {kk: (float(np.mean(v)) if v else None) for kk, v in e.items()}
            rows[str(Tt)]["instances"] = cnt
            rows[str(Tt)]["diverged_replicas"] = bad_tot
            rows[str(Tt)]["md_ms_per_run"] = ms_tot / cnt
            _log(f"  N={Nn} T={Tt}: " + ", ".join(
                f"{kk} {rows[str(Tt)][kk]:.5f}" for kk in e if rows[str(Tt)][kk] is not None
                and kk.endswith("one_init")))
        out["by_N"][str(Nn)] = rows
    out["paper"] = ("energies decrease with MD steps from 10^3 to 5*10^5 for N = 1000, 2000 and "
                    "10^4; the figure's values are not printed in the text")
    return out


def bench_dense8k(args, hqa, torch):
    """The enlarged dense shape where the MFMA roofline can bind: N = 8192, R = 512.
    SK couplings J ~ N(0, 1/N) in BF16 (inexact) and +-1 couplings in FP8 (exact), the
    paper's schedule.  Per plan (the tuner's choice, the per-step kernel, the batched
    kernel), the time of 200 MD steps with HIP events on the handle's stream; 2 N^2 R
    flop per step of the field against the dense BF16 MFMA peak."""
    from paper_2004_03972_amd import instances as inst
    Nn, Rr, Tt, steps = 8192, 512, 2000, 200
    st = torch.cuda.current_stream()
    out = {"metric": "field TFLOP/s and MFMA fraction at the enlarged dense shape",
           "workload": f"dense N={Nn}, R={Rr}", "peak_tflops": PEAK_MFMA["bf16"] / 1e12,
           "forms": {}}
    for name, J, form in (("sk_bf16", inst.sk(Nn, 8192), "bf16"),
                          ("pm1_fp8", inst.pm_complete(Nn, 8193), "fp8")):
        prob = hqa.Problem(J, storage=form)
        del J
        res = {}
        for plan in ("auto", "step", "batch"):
            md = hqa.MD(prob, hqa.make_schedule(Tt, 100), Rr, form, seed=8, plan=plan,
                        stream=st.cuda_stream)
            if plan == "auto":
                md.tune(10)
            md.run(40)
            e0, e1 = _events(torch)
            e0.record(st); md.run(40 + steps); e1.record(st); st.synchronize()
            md.sync()
            us = e0.elapsed_time(e1) * 1e3 / steps
            tf = 2.0 * Nn * Nn * Rr / (us * 1e-6) / 1e12
            key = plan if plan != "auto" else "tuned:" + "/".join(str(x) for x in md.tuned_plan())
            res[key] = {"us_per_step": us, "tflops": tf, "mfma_frac": tf * 1e12 / PEAK_MFMA["bf16"],
                        "ran": md.last_plan}
            _log(f"  {name} {key}: {us:.1f} us/step, {tf:.0f} TFLOP/s ({md.last_plan})")
            md.close()
        out["forms"][name] = res
    return out


def bench_sweep(args, hqa, torch):
    """Schedule and potential sweeps on the Ising spin glass with fields (J_ij ~ U[-1, 1],
    h_i ~ U[-2, 2], dense N = 10^4, BF16 storage, 10 initial conditions): H_MD at tau = 1
    (binary64, integer-time momenta) normalised by its value for kappa2 = 1 at the longest
    run, for kappa2 in [-1, 1] and several MD step counts, beside the best Ising energy
    per spin of the exact read-out (n = 20); then the potential exponent M in {4, 6, 8}."""
    from paper_2004_03972_amd import instances as inst
    Nn, Rr = args.sweep_n, 10
    J, h = inst.uniform_glass(Nn, 8001)
    prob = hqa.Problem(J, h=h, storage="bf16")
    st = torch.cuda.current_stream()
    kappas = [-1.0, -0.5, 0.0, 0.5, 1.0]
    steps = [int(x) for x in args.sweep_steps.split(",")]
    t_best = args.sweep_best

    def one(T, kappa2=1.0, M=6):
        md = hqa.MD(prob, hqa.make_schedule(T, 100, M=M,
                                            params=(0.008, 4.0, 3.0, 0.12, 0.05, kappa2)),
                    Rr, "bf16", seed=12, stream=st.cuda_stream)
        md.tune(min(20, T // 4))
        md.run()
        H = md.hamiltonian()          # per replica; NaN where the replica diverged
        bad = int(np.sum(~np.isfinite(H)))
        e = None
        if bad == 0:
            md.sync()
            e = float(md.classify(20, solve=True)["energy"].min()) / Nn
        md.close()
        return float(np.mean(H[np.isfinite(H)])) if bad < Rr else float("nan"), e, bad

    t0 = time.perf_counter()
    h_best, e_best, bad = one(t_best)
    if bad:
        raise RuntimeError(f"{bad} of {Rr} replicas diverged in the reference run")
    _log(f"  best run T={t_best}: H_MD(1) = {h_best:.3f}, E/N = {e_best:.5f} "
         f"({time.perf_counter() - t0:.1f} s)")
    table = {}
    for T in steps:
        for k2 in kappas:
            hm, e, bad = one(T, kappa2=k2)
            table[f"T={T} kappa2={k2:+.1f}"] = {"H_MD(1)/H_best": hm / h_best if np.isfinite(hm) else None,
                                                "E_best/N": e,
                                                "diverged_replicas": bad}
        _log(f"  T={T} done ({time.perf_counter() - t0:.1f} s)")
    mt = {}
    for M in (4, 6, 8):
        hm, e, bad = one(steps[-1], M=M)
        mt[f"M={M}"] = {"E_best/N": e, "diverged_replicas": bad}
    return {"metric": "H_MD(tau=1)/H_best vs kappa2 and MD steps; E/N vs M",
            "workload": f"spin glass J~U[-1,1], h~U[-2,2], dense N={Nn}, BF16 J, R={Rr}",
            "H_best": h_best, "H_best_run": {"T": t_best, "kappa2": 1.0, "E_best/N": e_best},
            "kappa2_sweep": table, "M_sweep_T": steps[-1], "M_sweep": mt,
            "paper": "H_MD(1) nearly independent of kappa2 for enough steps; fastest approach "
                     "to H_best at kappa2 = +1 (paper's note on adiabaticity)",
            "note": "a replica whose flux passes the explicit leapfrog's stability bound "
                    "(alpha^2 M (M-1) phi^(M-2) about 4) diverges; such replicas are counted, "
                    "H_MD is averaged over the others and no read-out energy is given"}


def bench_copy(args, hqa, torch):
    """A plain device copy of 1 GiB (reads 1 GiB, writes 1 GiB): HBM counter calibration."""
    n = 1 << 28
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    return {"workload": "copy 1 GiB float32", "bytes_read": 4 * n, "bytes_written": 4 * n}


def bench_peaks(args, hqa, torch):
    """Achievable peaks next to the vendor figures: a plain device copy of 1 GiB (HBM
    bytes read + written per second), torch's sum over the same 1 GiB (bytes read per
    second; a reduction kernel, not a bound on reads) and the library BF16 GEMM at 8192^3 (dense MFMA
    flop per second), each the best of 10 timed repetitions after 3 warm-ups."""
    st = torch.cuda.current_stream()

    def best_ms(fn, reps=10):
        for _ in range(3):
            fn()
        ts = []
        for _ in range(reps):
            e0, e1 = _events(torch)
            e0.record(st); fn(); e1.record(st); e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return min(ts)

    n = 1 << 28
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    ms_copy = best_ms(lambda: y.copy_(x))
    hbm = 2 * 4 * n / (ms_copy * 1e-3) / 1e9
    ms_read = best_ms(lambda: x.sum())             # torch's reduction: reads 1 GiB
    hbm_read = 4 * n / (ms_read * 1e-3) / 1e9
    del x, y
    m = 8192
    a = torch.randn(m, m, dtype=torch.bfloat16, device="cuda")
    b = torch.randn(m, m, dtype=torch.bfloat16, device="cuda")
    ms_mm = best_ms(lambda: torch.mm(a, b))
    tf = 2.0 * m ** 3 / (ms_mm * 1e-3) / 1e12
    return {"workload": "achievable peaks", "hbm_copy_GBps": hbm, "torch_sum_read_GBps": hbm_read,
            "hbm_vendor_GBps": 8000.0,
            "bf16_gemm_8192_TFLOPs": tf, "bf16_vendor_dense_TFLOPs": 2500.0,
            "copy_ms": ms_copy, "gemm_ms": ms_mm}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch",
                    choices=["batch", "er800", "ea3d", "batch512", "es", "k2000", "glass", "dense8k", "sweep", "copy",
                             "peaks"])
    ap.add_argument("--glass-n", default="1000,2000,10000")
    ap.add_argument("--glass-instances", default="8,8,2")
    ap.add_argument("--glass-steps", default="1000,10000,100000,500000")
    ap.add_argument("--glass-replicas", type=int, default=16)
    ap.add_argument("--glass-tabu-n", default="500,1000,4000")
    ap.add_argument("--glass-tabu-sweeps", type=int, default=20)
    ap.add_argument("--sweep-n", type=int, default=10000)
    ap.add_argument("--sweep-steps", default="2000,10000,50000")
    ap.add_argument("--sweep-best", type=int, default=200000)
    ap.add_argument("--k2000-instances", type=int, default=4)
    ap.add_argument("--k2000-replicas", type=int, default=16)
    ap.add_argument("--k2000-steps", default="50000,500000")
    ap.add_argument("--k2000-first", type=int, default=0)
    ap.add_argument("--k2000-group", type=int, default=8)
    ap.add_argument("--k2000-per-run", action="store_true")
    ap.add_argument("--k2000-tabu-n", type=int, default=1000)
    ap.add_argument("--k2000-tabu-iters", type=int, default=20000)
    ap.add_argument("--k2000-tabu-tenure", type=int, default=50)
    ap.add_argument("--es-train", type=int, default=48)
    ap.add_argument("--es-train-r", type=int, default=4)
    ap.add_argument("--es-keep", type=float, default=1.0)
    ap.add_argument("--es-target", type=float, default=0.03,
                    help="es --es-calibrate mislabel: largest mislabel rate at the stop")
    ap.add_argument("--es-calibrate", choices=["cut", "mislabel"], default="cut")
    ap.add_argument("--es-target-cut", type=float, default=1e-3,
                    help="es --es-calibrate cut: largest relative cut loss at the stop")
    ap.add_argument("--es-k", type=int, default=1000)
    ap.add_argument("--es-ks", type=int, default=100)
    ap.add_argument("--es-stride", type=int, default=10)
    ap.add_argument("--forms", default="fp8,bf16,f32")
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--md-steps", type=int, default=0)
    ap.add_argument("--fp32-seeds", type=int, default=2,
                    help="seeds of the plain FP32 comparison (the first of the timed seeds)")
    ap.add_argument("--detail", default="", help="write per-instance cuts and errors here")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--eager", action="store_true",
                    help="batch: launch the MD steps one by one instead of replaying a graph")
    ap.add_argument("--pin", default="",
                    help="TM,TN,CB[,TILED]: fixed per-step block instead of tuning")
    args = ap.parse_args()
    args.forms = [f for f in args.forms.split(",") if f]
    args.pin = tuple(int(x) for x in args.pin.split(",")) if args.pin else None
    if args.gpus != 1:
        print("this build runs on one GPU: replicas and instances would shard across GPUs "
              "without communication, but no multi-GPU path is built; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2004_03972_amd import hqa
    hqa.lib()
    torch.cuda.set_device(0)
    fn = {"batch": bench_batch, "batch512": bench_batch, "er800": bench_er800, "ea3d": bench_ea3d,
          "es": bench_es, "k2000": bench_k2000, "glass": bench_glass, "dense8k": bench_dense8k, "sweep": bench_sweep,
          "copy": bench_copy, "peaks": bench_peaks}[args.workload]
    print(json.dumps(fn(args, hqa, torch)), flush=True)


if __name__ == "__main__":
    main()
