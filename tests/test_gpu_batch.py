"""Batched uneven instances (one launch per step over an LPT tile table).

- a batched instance evolves bit-identically to the same instance run alone,
  with SK (BF16, inexact) and ER (FP8 e4m3, exact) instances mixed in one batch;
- fields of every instance of a batch on a shared flux: FP8/BF16 storage equals
  J . bf16(phi) (with J rounded to its storage) within 1e-5 relative;
- a short FP32 batched run tracks the FP64 oracle (same step semantics).
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


def bf16_nearest(x):
    """Nearest bfloat16 (ties to even) of binary64 values, chosen between the two
    bfloat16 neighbours by exact binary64 distance (no double rounding)."""
    x = np.asarray(x, dtype=np.float64)
    f = x.astype(np.float32).view(np.uint32)
    lo = (f & np.uint32(0xFFFF0000))
    hi = lo + np.uint32(0x10000)
    clo = lo.view(np.float32).astype(np.float64)
    chi = hi.view(np.float32).astype(np.float64)
    dlo, dhi = np.abs(x - clo), np.abs(x - chi)
    even_lo = ((lo >> 16) & 1) == 0
    pick_lo = (dlo < dhi) | ((dlo == dhi) & even_lo)
    return np.where(pick_lo, clo, chi)


def _mixed_batch(H, sizes_sk, sizes_er, seed0):
    probs, Js = [], []
    for k, N in enumerate(sizes_sk):
        J = inst.sk(N, seed0 + k)
        probs.append(H.Problem(J, storage="bf16"))
        Js.append(("sk", J))
    for k, N in enumerate(sizes_er):
        J = inst.er_maxcut(N, 0.05, seed0 + 100 + k)
        probs.append(H.Problem(J, storage="fp8"))
        Js.append(("er", J))
    return probs, Js


@pytest.mark.parametrize("R", [64, 40])
def test_batch_equals_individual_runs(H, R):
    """Every instance of an uneven batch (SK in BF16; unit-weight ER MAX-CUT, which the
    batch plan streams one bit per coupling) evolves bit-identically to the same instance
    run alone on its own plan (FP8 storage for ER)."""
    probs, Js = _mixed_batch(H, [100, 333, 517], [700, 1200], 10)
    T = 160
    b = H.MD(probs, H.make_schedule(T, 30), R, "bf16", seed=3)
    b.run()
    b.sync()
    assert [b.batch_form(k) for k in range(len(probs))] == ["bf16"] * 3 + ["bit"] * 2
    for k, p in enumerate(probs):
        a = H.MD(p, H.make_schedule(T, 30), R, "bf16", seed=3)
        a.run()
        for w in (H.HQA_STATE_PHI, H.HQA_STATE_P, H.HQA_STATE_WSUM):
            assert np.array_equal(a.state(w), b.state(w, k)), (k, w)
        a.close()


def test_bit_form_only_for_zero_one_couplings(H):
    """The one-bit form is taken only when every coupling is 0 or 1: FP8 instances with
    +-1 couplings or small integers stay FP8 in the batch, unit weights go to bits (also
    with ragged sizes N = 130, 129 + 128 k), and every instance still equals its lone run
    bit for bit; the per-step plan ignores the form."""
    Js = [inst.pm_complete(200, 3), inst.small_int(257, 4, 0, 2, density=0.3),
          inst.er_maxcut(130, 0.2, 5), inst.er_maxcut(385, 0.1, 6)]
    probs = [H.Problem(J, storage="fp8") for J in Js]
    T, R = 120, 64
    b = H.MD(probs, H.make_schedule(T, 30), R, "bf16", seed=8)
    assert b.batch_form(0) is None
    b.run()
    b.sync()
    assert b.last_plan == "batch"
    assert [b.batch_form(k) for k in range(len(probs))] == ["fp8", "fp8", "bit", "bit"]
    for k, p in enumerate(probs):
        a = H.MD(p, H.make_schedule(T, 30), R, "bf16", seed=8, plan="step")
        a.run()
        for w in (H.HQA_STATE_PHI, H.HQA_STATE_P, H.HQA_STATE_WSUM):
            assert np.array_equal(a.state(w), b.state(w, k)), (k, w)
        a.close()
    b.close()


@pytest.mark.parametrize("R", [64, 24])
def test_f32_batch_equals_individual_runs(H, R):
    """FP32 storage in the batch kernel (128-row tiles, FP32 flux block in LDS, 16x16x4
    FP32 MFMAs): every instance of an uneven FP32 batch evolves bit-identically to the
    same instance run alone on the per-step plan, with ragged row blocks and replica
    tiles."""
    sizes = [100, 333, 517, 130]
    probs = []
    for k, N in enumerate(sizes):
        J, h = inst.uniform_glass(N, 600 + k)
        probs.append(H.Problem(J * 0.1, h=h))
    T = 150
    b = H.MD(probs, H.make_schedule(T, 30), R, "f32", seed=6)
    b.run()
    b.sync()
    assert b.last_plan == "batch"
    for k, p in enumerate(probs):
        a = H.MD(p, H.make_schedule(T, 30), R, "f32", seed=6, plan="step")
        a.run()
        for w in (H.HQA_STATE_PHI, H.HQA_STATE_P, H.HQA_STATE_WSUM):
            assert np.array_equal(a.state(w), b.state(w, k)), (k, w)
        a.close()
    b.close()


def test_batch_fields_all_instances(H):
    import torch
    rng = np.random.default_rng(77)
    sizes_sk = list(rng.integers(100, 700, size=6))
    sizes_er = list(rng.integers(300, 1500, size=6))
    probs, Js = _mixed_batch(H, sizes_sk, sizes_er, 40)
    R = 64
    b = H.MD(probs, H.make_schedule(10, 5), R, "bf16")
    worst = 0.0
    for k, (kind, J) in enumerate(Js):
        N = J.shape[0]
        phi = rng.uniform(-1.2, 1.2, size=(R, N))
        b.set_state(H.HQA_STATE_PHI, phi, k)
        u = b.field(k)
        # the flux operand is rounded from its binary32 copy, J from binary64
        phib = bf16_nearest(phi.astype(np.float32).astype(np.float64))
        Jst = bf16_nearest(J)
        u64 = orc.field(orc.Problem(N, J=Jst), phib)
        rel = np.max(np.abs(u - u64)) / np.max(np.abs(u64))
        worst = max(worst, rel)
        dh = np.max(np.abs(u - orc.field(orc.Problem(N, J=J), phi)))
        print(kind, N, "rel vs J.bf16(phi)", rel, "max |dh| vs FP64", dh, flush=True)
    assert worst <= 1e-5


def test_batch_f32_tracks_oracle(H):
    sizes = [64, 150, 233, 97]
    probs, Js = [], []
    for k, N in enumerate(sizes):
        J, h = inst.uniform_glass(N, 500 + k)
        J *= 0.1
        probs.append(H.Problem(J, h=h))
        Js.append((J, h))
    R, T, W = 8, 120, 20
    b = H.MD(probs, H.make_schedule(T, W), R, "f32", seed=9)
    # the binary32 fluxes after 10, 20 and 30 steps lie within the first-order forward
    # error bound of the binary32 arithmetic against the oracle's binary64 trajectory
    # (tests/f32_bound.py); past a few dozen steps that worst-case bound grows faster
    # than the trajectories diverge, so the check stops there
    bounds = []
    for k, (J, h) in enumerate(Js):
        N = J.shape[0]
        e, phis = f32_bound(orc, orc.Problem(N, J=J, h=h), orc.MDParams(T=T, W=W),
                            np.zeros((R, N)), orc.init_p0(9, N, R), 30)
        bounds.append((e, phis))
    for q in (10, 20, 30):
        b.run(q)
        for k in range(len(Js)):
            e, phis = bounds[k]
            err = np.max(np.abs(b.state(H.HQA_STATE_PHI, k) - phis[q]))
            print("instance", k, "step", q, "max |phi32 - phi64|", err, "bound", e[q], flush=True)
            assert err <= e[q]
    b.run()
    for k, (J, h) in enumerate(Js):
        N = J.shape[0]
        bar, phiT, _ = orc.md_run(orc.Problem(N, J=J, h=h), orc.MDParams(T=T, W=W),
                                  np.zeros((R, N)), orc.init_p0(9, N, R))
        print("instance", k, "step", T, "max |phi32 - phi64| (observed)",
              np.max(np.abs(b.state(H.HQA_STATE_PHI, k) - phiT)), flush=True)


def test_field_error_against_binary64(H):
    """hqa_md_field_error: binary32 field of each instance's precision form against the
    binary64 field on the same fluxes; the reference magnitude is checked against
    the oracle's field."""
    R = 32
    Js = [inst.sk(300, 11), inst.er_maxcut(500, 0.05, 12), inst.sk(200, 13)]
    probs = [H.Problem(Js[0], storage="bf16"), H.Problem(Js[1], storage="fp8"),
             H.Problem(Js[2], storage="f32")]
    md = H.MD(probs, H.make_schedule(200, 20), R, "bf16", seed=3)
    md.run(120)
    for k, (J, bar) in enumerate(zip(Js, (2e-2, 2e-2, 1e-5))):
        err, ref = md.field_error(k)
        phi = md.state(H.HQA_STATE_PHI, k)
        want = np.abs(orc.field(orc.Problem(J.shape[0], J=J), phi)).max()
        print("instance", k, "max|du|", err, "max|u|", ref, "relative", err / ref, flush=True)
        assert ref == pytest.approx(want, rel=1e-12)
        assert err / ref <= bar
        if k < 2:
            assert err > 0.0                  # BF16 flux operand: a rounding error exists


@pytest.mark.parametrize("kind,N,R", [("glass", 1100, 72), ("pm", 1030, 64), ("glass", 300, 16)])
def test_single_instance_batch_plan_equals_step(H, kind, N, R):
    """The batched kernel as the plan of a lone dense instance (row blocks spread over
    the XCDs when the instance has at least eight of them) gives the per-step plan's
    trajectory bit for bit, with fields, ragged replica tiles and a padded last row block."""
    print("single batch", kind, N, R, flush=True)
    if kind == "glass":
        J, h = inst.uniform_glass(N, 21)
        prob, prec = H.Problem(J, h=h, storage="bf16"), "bf16"
    else:
        J, h = inst.pm_complete(N, 22), None
        prob, prec = H.Problem(J, storage="fp8"), "fp8"
    T = 140
    out = []
    for plan in ("batch", "step"):
        md = H.MD(prob, H.make_schedule(T, 30), R, prec, seed=5, plan=plan)
        md.run(T // 2)
        md.run()
        md.sync()
        assert md.last_plan == plan
        out.append([md.state(w) for w in (H.HQA_STATE_PHI, H.HQA_STATE_P, H.HQA_STATE_WSUM)])
        md.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_graph_replay_equals_eager(H):
    """HQA_MD_GRAPH: the batch plan's steps replayed from captured HIP graphs give the
    eager launches' trajectories bit for bit, over several replays of each graph with
    eager work and synchronisations between them, split runs (two graphs per run) and
    an odd step count (so the flux-buffer parity, part of a graph's key, alternates
    between rounds); a single instance on the BATCH plan replays as well."""
    probs, Js = _mixed_batch(H, [100, 333], [700], 60)
    T, R = 161, 64
    ws = (H.HQA_STATE_PHI, H.HQA_STATE_P, H.HQA_STATE_WSUM)
    eager = H.MD(probs, H.make_schedule(T, 30), R, "bf16", seed=3)
    graph = H.MD(probs, H.make_schedule(T, 30), R, "bf16", seed=3, graph=True)
    for rnd in range(4):
        print("graph replay round", rnd, flush=True)
        for md in (eager, graph):
            md.reset(10 + rnd)
            md.run(T // 2)
            md.run()
            md.sync()
            assert md.last_plan == "batch"
        for k in range(len(probs)):
            for w in ws:
                assert np.array_equal(eager.state(w, k), graph.state(w, k)), (rnd, k, w)
    eager.close()
    graph.close()
    # a lone dense instance on the BATCH plan
    out = []
    for g in (False, True):
        md = H.MD(probs[2], H.make_schedule(T, 30), R, "fp8", seed=7, plan="batch", graph=g)
        for rnd in range(3):
            md.reset(7 + rnd)
            md.run()
            md.sync()
        assert md.last_plan == "batch"
        out.append([md.state(w) for w in ws])
        md.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("T", [160, 161])
def test_pass_equals_separate_calls(H, T):
    """hqa_md_pass: a whole pass (reset, every step, the read-out of every instance)
    equals hqa_md_reset + hqa_md_run + hqa_classify_many bit for bit, in energies, cuts
    and the final state; replayed from its captured HIP graph several times with other
    eager work and synchronisations between the replays (an odd T flips the flux-buffer
    parity, so two graphs alternate), and run eagerly.  A handle that is not on the
    batch plan refuses graph mode but runs the pass eagerly."""
    import torch
    probs, Js = _mixed_batch(H, [100, 333], [517, 700], 90)
    R, n = 64, 12
    ws = (H.HQA_STATE_PHI, H.HQA_STATE_P, H.HQA_STATE_WSUM)
    md = H.MD(probs, H.make_schedule(T, 30), R, "bf16", seed=3)
    md.reset(21)
    md.run()
    E0, C0 = md.classify_many(n, True)
    S0 = [[md.state(w, k) for w in ws] for k in range(len(probs))]
    E = torch.full((len(probs), R), float("nan"), dtype=torch.float64, device="cuda")
    C = torch.full((len(probs), R), float("nan"), dtype=torch.float64, device="cuda")
    for rnd in range(4):
        print("pass replay round", rnd, flush=True)
        E.fill_(float("nan"))
        C.fill_(float("nan"))
        md.run_pass(21, n, True, graph=rnd < 3, energy=E, cut=C)
        md.sync()
        assert md.step == T
        assert np.array_equal(E.cpu().numpy(), E0) and np.array_equal(C.cpu().numpy(), C0), rnd
        for k in range(len(probs)):
            for w, ref in zip(ws, S0[k]):
                assert np.array_equal(md.state(w, k), ref), (rnd, k, w)
        # other eager work between the replays: another seed through the separate calls
        md.reset(40 + rnd)
        md.run()
        md.classify_many(n, False)
        torch.cuda.synchronize()
    md.close()
    # one dense instance under AUTO runs on the per-step plan: graph mode is refused
    one = H.MD(probs[2], H.make_schedule(T, 30), R, "fp8", seed=5)
    e1 = torch.empty((1, R), dtype=torch.float64, device="cuda")
    with pytest.raises(H.HQAError) as ex:
        one.run_pass(8, n, True, graph=True, energy=e1, cut=None)
    assert ex.value.status == H.HQA_EUNSUPPORTED
    one.run_pass(8, n, True, graph=False, energy=e1, cut=None)
    one.sync()
    one.reset(8)
    one.run()
    Er, _ = one.classify_many(n, True)
    assert np.array_equal(e1.cpu().numpy(), Er)
    one.close()


def test_classify_many_equals_per_instance(H):
    """hqa_classify_many: the energies and cuts of every listed instance equal
    hqa_classify's bit for bit (exact enumeration at n = 12 and the MD-alone read-out),
    for all instances, for a subset with a repeat, and with device outputs; bad lists
    are refused before any device work."""
    import torch
    probs, Js = _mixed_batch(H, [100, 333, 517], [700, 1200], 80)
    R, T = 40, 120
    md = H.MD(probs, H.make_schedule(T, 30), R, "bf16", seed=5)
    md.run()
    for solve, n in ((True, 12), (False, 7)):
        E, Cc = md.classify_many(n, solve=solve)
        for k in range(len(probs)):
            g = md.classify(n, solve=solve, k=k)
            assert np.array_equal(E[k], g["energy"]) and np.array_equal(Cc[k], g["cut"]), (solve, k)
    ks = np.array([4, 0, 4], dtype=np.int32)
    E2, C2 = md.classify_many(12, instances=ks)
    E, Cc = md.classify_many(12)
    assert np.array_equal(E2, E[ks]) and np.array_equal(C2, Cc[ks])
    dE = torch.empty((3, R), dtype=torch.float64, device="cuda")
    H.hqa_classify_many(md.h, ks, 3, 12, 1, dE, None, H.HQA_DEVICE)
    assert np.array_equal(dE.cpu().numpy(), E[ks])
    for bad in (np.array([5], np.int32), np.array([-1], np.int32)):
        with pytest.raises(H.HQAError) as e:
            md.classify_many(12, instances=bad)
        assert e.value.status == H.HQA_EINVAL
    with pytest.raises(H.HQAError) as e:
        H.hqa_classify_many(md.h, ks, 0, 12, 1, dE, None, H.HQA_DEVICE)
    assert e.value.status == H.HQA_EINVAL
    with pytest.raises(H.HQAError) as e:
        md.classify_many(25)                      # exact enumeration limited to n <= 24
    assert e.value.status == H.HQA_EUNSUPPORTED
    md.close()
