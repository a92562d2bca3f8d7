"""The library's environment switches on the GPU: allocation-failure injection
(HQA_FAULT_ALLOC) through every device allocation that init, a batched run and a
read-out make, the per-call timing lines (HQA_TIMING), the persisted tuner choices
(HQA_TUNE_CACHE) and the abort path of the persistent kernels' bounded waits
(HQA_SPIN_LIMIT)."""
import os

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


def _problems(H):
    return [H.Problem(inst.sk(150, 1), storage="bf16"),
            H.Problem(inst.er_maxcut(300, 0.05, 2), storage="fp8")]


def _session(H, probs):
    """Init, a batched run, the read-out of both instances; returns the energies."""
    md = H.MD(probs, H.make_schedule(40, 10), 16, "bf16", seed=2)   # init may fail: nothing to close
    try:
        md.run()
        E, C = md.classify_many(6)
        g = md.classify(6, solve=True, k=1)
        return np.concatenate([E.ravel(), C.ravel(), g["energy"]])
    finally:
        md.close()


def test_fault_alloc_every_allocation(H, monkeypatch):
    """HQA_FAULT_ALLOC=k for k = 1, 2, ...: the k-th device allocation fails, the call
    that made it returns HQA_ENOMEM naming the allocation, the partial handle is released,
    and the next session without the switch gives the reference results; k past the last
    allocation changes nothing."""
    probs = _problems(H)
    monkeypatch.delenv("HQA_FAULT_ALLOC", raising=False)
    ref = _session(H, probs)
    failed = 0
    for k in range(1, 200):
        monkeypatch.setenv("HQA_FAULT_ALLOC", str(k))
        try:
            out = _session(H, probs)
        except H.HQAError as e:
            assert e.status == H.HQA_ENOMEM, (k, str(e))
            failed += 1
            monkeypatch.delenv("HQA_FAULT_ALLOC")
            assert np.array_equal(_session(H, probs), ref), k
            continue
        assert np.array_equal(out, ref)
        break
    print("allocations that failed one by one:", failed, flush=True)
    assert failed >= 10
    # disarm (init re-reads the switch) before other tests allocate
    monkeypatch.delenv("HQA_FAULT_ALLOC")
    assert np.array_equal(_session(H, probs), ref)


def test_timing_lines(H, monkeypatch, capfd):
    probs = _problems(H)
    monkeypatch.setenv("HQA_TIMING", "1")
    md = H.MD(probs, H.make_schedule(40, 10), 16, "bf16", seed=2)
    md.run(20)
    md.run()
    md.classify_many(6)
    md.classify(6, solve=True, k=0)
    md.close()
    monkeypatch.setenv("HQA_TIMING", "0")
    err = capfd.readouterr().err
    lines = [ln for ln in err.splitlines() if ln.startswith("hqa timing:")]
    print("\n".join(lines))
    assert sum("hqa_md_run steps 0..20" in ln for ln in lines) == 1
    assert sum("hqa_md_run steps 20..40" in ln and "plan batch" in ln for ln in lines) == 1
    assert sum("read-out of 2 instances" in ln for ln in lines) == 1
    assert sum("read-out of instance 0" in ln for ln in lines) == 1


def test_tune_cache(H, monkeypatch, tmp_path):
    """HQA_TUNE_CACHE: hqa_md_tune writes one line per tuned case; a later tune of the
    same case takes the stored choice without timing (forced here to a different valid
    STEP block to see it taken); an entry that does not fit the instance is ignored;
    every choice gives the same trajectory."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("HQA_TUNE_CACHE", str(path))
    J = inst.er_maxcut(400, 0.05, 3)
    prob = H.Problem(J, storage="fp8")
    sched = H.make_schedule(200, 20)

    def run(expect=None):
        md = H.MD(prob, sched, 32, "fp8", seed=4)
        md.tune(10)
        plan = md.tuned_plan()
        if expect is not None:
            assert plan == expect, plan
        md.run()
        out = md.state(H.HQA_STATE_PHIBAR)
        md.close()
        return plan, out

    plan0, ref = run()
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and " one dense N=400 " in lines[0] and " R=32 " in lines[0]
    key = lines[0].split("|")[0].rstrip()
    # a different valid per-step block for the same case
    forced = ("step", 1, 1, 4, 0) if plan0 != ("step", 1, 1, 4, 0) else ("step", 2, 2, 8, 1)
    P = {"step": H.HQA_PLAN_STEP}
    path.write_text(lines[0] + "\n" + f"{key} | {P['step']} {forced[1]} {forced[2]} {forced[3]} {forced[4]}\n")
    plan1, out1 = run(expect=forced)
    assert np.array_equal(out1, ref)
    assert len(path.read_text().splitlines()) == 2          # a hit writes nothing
    # an entry that does not fit (4 replica tiles need R divisible by 64): tuned again
    path.write_text(f"{key} | {P['step']} 1 4 4 0\n")
    plan2, out2 = run()
    assert plan2 != ("step", 1, 4, 4, 0)
    assert np.array_equal(out2, ref)
    assert len(path.read_text().splitlines()) == 2
    # several dense instances: one more line for the joint choice
    path.write_text("")
    md = H.MD([prob, H.Problem(inst.sk(300, 5), storage="bf16")], sched, 32, "bf16", seed=4)
    md.tune(10)
    md.close()
    keys = [ln.split("|")[0] for ln in path.read_text().splitlines()]
    assert sum(" one " in k for k in keys) == 2 and sum(" several " in k for k in keys) == 1


def test_spin_limit_aborts_cleanly(H, monkeypatch):
    """HQA_SPIN_LIMIT=0: every wait of the CLUSTER plan's persistent kernel gives up at its
    first poll that finds a flux not yet published.  The launch still ends (the abort flag
    sends every workgroup home), hqa_md_sync reports HQA_EDEVICE naming the barrier bound,
    and after hqa_md_reset without the limit the handle's trajectory equals a fresh
    handle's bit for bit."""
    prob = H.Problem(inst.er_maxcut(400, 0.05, 9), storage="fp8")
    T, R = 60, 64
    ws = (H.HQA_STATE_PHI, H.HQA_STATE_P, H.HQA_STATE_WSUM)
    ref = H.MD(prob, H.make_schedule(T, 10), R, "fp8", seed=4, plan="cluster")
    ref.run()
    ref.sync()
    assert ref.last_plan == "cluster"
    want = [ref.state(w) for w in ws]
    ref.close()
    md = H.MD(prob, H.make_schedule(T, 10), R, "fp8", seed=4, plan="cluster")
    aborted = 0
    for rnd in range(3):
        print("spin-limit round", rnd, flush=True)
        monkeypatch.setenv("HQA_SPIN_LIMIT", "0")
        md.reset(4)
        md.run()
        try:
            md.sync()
        except H.HQAError as e:
            assert e.status == H.HQA_EDEVICE and "barrier" in str(e), str(e)
            aborted += 1
        monkeypatch.delenv("HQA_SPIN_LIMIT")
        md.reset(4)
        md.run()
        md.sync()
        assert md.last_plan == "cluster"
        for w, x in zip(ws, want):
            assert np.array_equal(md.state(w), x), (rnd, w)
    md.close()
    assert aborted >= 1
