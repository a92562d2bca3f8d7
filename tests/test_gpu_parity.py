"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars: bit-exact for the binary64 reference mode (fluxes, window means, sort,
effective fields, enumeration, energies) and for every integer/index output;
binary32 fields within 1e-5 of the FP64 field relative to its largest magnitude
(max |u32 - u64| / max |u64|) for the same fluxes; read-out of a binary32 run
compared with the oracle's read-out of the same exported window means.
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


def _say(*a):
    print(*a, flush=True)


LINEAR = (0.008, 4.0, 0.0, 0.12, 0.05, 0.0)


def _oracle_run(pb, T, W, sched, p0, phi0=None, M=6, r_g=1.0):
    mp = orc.MDParams(T=T, W=W, M=M, r_g=r_g, schedule=sched)
    phi0 = np.zeros_like(p0) if phi0 is None else phi0
    return orc.md_run(pb, mp, phi0, p0, nthreads=8), mp


# ------------------------------------------------------------ binary64 reference
@pytest.mark.parametrize("sched", ["linear", "paper"])
def test_f64_ref_sk64_bit_exact(H, sched):
    # SK, N = 64, J ~ N(0, 1/N), 8 replicas, 2000 steps, n = 12 (small SK case)
    N, R, T, W, n = 64, 8, 2000, 100, 12
    prm = LINEAR if sched == "linear" else orc.PAPER_SCHEDULE
    J = inst.sk(N, 101)
    _say("f64 ref SK64", sched)
    md = H.MD(H.Problem(J), H.make_schedule(T, W, params=prm), R, "f64", seed=1)
    md.run()
    md.sync()
    p0 = orc.init_p0(1, N, R)
    (bar, phiT, pT), mp = _oracle_run(orc.Problem(N, J=J), T, W, prm, p0)
    assert np.array_equal(md.state(H.HQA_STATE_PHI), phiT)
    assert np.array_equal(md.state(H.HQA_STATE_P), pT)
    assert np.array_equal(md.state(H.HQA_STATE_PHIBAR), bar)
    g = md.classify(n, solve=True)
    A, s_md = orc.classify(bar, n)
    he, Je = orc.reduce(orc.Problem(N, J=J), A, s_md)
    code, Ered = orc.enumerate_exact(Je, he)
    s_hqa = orc.merge(s_md, A, code)
    E, C = orc.energy(orc.Problem(N, J=J), s_hqa)
    assert np.array_equal(g["amb_idx"], A)
    assert np.array_equal(g["h_eff"], he)
    assert np.array_equal(g["code"], code)
    assert np.array_equal(g["e_reduced"], Ered)
    assert np.array_equal(g["spins"], s_hqa)
    assert np.array_equal(g["energy"], E) and np.array_equal(g["cut"], C)
    g0 = md.classify(n, solve=False)
    E0, C0 = orc.energy(orc.Problem(N, J=J), s_md)
    assert np.array_equal(g0["spins"], s_md)
    assert np.array_equal(g0["energy"], E0) and np.array_equal(g0["cut"], C0)
    assert np.all(g["energy"] <= g0["energy"])
    md.close()


def test_f64_ref_csr_field_and_explicit_init(H):
    # EA +-J lattice (CSR) and the uniform glass with a field (dense), explicit
    # phi0 != 0 and p0, r_g != 1, M = 4: every branch of the reference step.
    rp, ci, v = inst.ea3d(4, 7)
    N, R, T, W = 64, 3, 300, 40
    rng = np.random.default_rng(3)
    p0 = inst.random_pm1((R, N), 5)
    phi0 = rng.uniform(-0.2, 0.2, size=(R, N))
    md = H.MD(H.Problem(row_ptr=rp, col=ci, val=v), H.make_schedule(T, W, M=4, r_g=0.7), R,
              "f64", p0=p0, phi0=phi0)
    md.run()
    (bar, phiT, pT), _ = _oracle_run(orc.Problem(N, row_ptr=rp, col=ci, val=v), T, W,
                                     orc.PAPER_SCHEDULE, p0, phi0, M=4, r_g=0.7)
    assert np.array_equal(md.state(H.HQA_STATE_PHI), phiT)
    assert np.array_equal(md.state(H.HQA_STATE_PHIBAR), bar)
    J, h = inst.uniform_glass(50, 9)
    md = H.MD(H.Problem(J, h=h), H.make_schedule(T, W), 5, "f64", seed=77)
    md.run()
    (bar, phiT, pT), _ = _oracle_run(orc.Problem(50, J=J, h=h), T, W, orc.PAPER_SCHEDULE,
                                     orc.init_p0(77, 50, 5))
    assert np.array_equal(md.state(H.HQA_STATE_PHI), phiT)
    assert np.array_equal(md.state(H.HQA_STATE_P), pT)
    g = md.classify(10, solve=True)
    A, s = orc.classify(bar, 10)
    he, Je = orc.reduce(orc.Problem(50, J=J, h=h), A, s)
    code, Ered = orc.enumerate_exact(Je, he)
    assert np.array_equal(g["h_eff"], he) and np.array_equal(g["code"], code)
    assert np.array_equal(g["e_reduced"], Ered)
    E, C = orc.energy(orc.Problem(50, J=J, h=h), orc.merge(s, A, code))
    assert np.array_equal(g["energy"], E)


def test_f64_hamiltonian_matches_oracle(H):
    N, R, T = 40, 4, 200
    J, h = inst.uniform_glass(N, 13)
    prm = (0.03, 0.0, 0.0, 0.05, 0.0, 0.0)
    s = H.make_schedule(T, 1, params=prm, frozen=True, tau_frozen=1.0)
    md = H.MD(H.Problem(J, h=h), s, R, "f64", seed=4)
    mp = orc.MDParams(T=T, W=1, schedule=prm, frozen=True, tau_fix=1.0)
    pb = orc.Problem(N, J=J, h=h)
    phi, p = np.zeros((R, N)), orc.init_p0(4, N, R)
    Hg0 = md.hamiltonian()
    assert np.allclose(Hg0, orc.hmd(pb, mp, 0, phi, p), rtol=1e-13, atol=1e-15)
    md.run(150)
    orc.md_advance(pb, mp, phi, p, None, 0, 150)
    Ho = orc.hmd(pb, mp, 150, phi, orc.integer_p(pb, mp, 150, phi, p))
    Hg = md.hamiltonian()
    assert np.allclose(Hg, Ho, rtol=1e-12, atol=1e-14)
    assert np.max(np.abs(Hg - Hg0)) < 5e-2 * np.max(np.abs(Hg0))   # bounded drift


# ------------------------------------------------------------- binary32 fields
def _shared_phi(R, N, seed):
    return np.random.default_rng(seed).uniform(-1.2, 1.2, size=(R, N))


@pytest.mark.parametrize("N,R", [(200, 40), (64, 16), (800, 256), (1000, 64)])
def test_f32_dense_field_within_1e5(H, N, R):
    J = inst.sk(N, 300 + N)
    md = H.MD(H.Problem(J), H.make_schedule(10, 5), R, "f32")
    phi = _shared_phi(R, N, N).astype(np.float32).astype(np.float64)
    md.set_state(H.HQA_STATE_PHI, phi)
    u = md.field()
    u64 = orc.field(orc.Problem(N, J=J), phi)
    rel = np.max(np.abs(u - u64)) / np.max(np.abs(u64))
    _say("dense f32 field rel err", N, R, rel)
    assert rel <= 1e-5


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_lowp_dense_field(H, prec):
    # BF16 operand: the GPU field equals J . bf16(phi) up to FP32 accumulation.
    N, R = 520, 48
    J = inst.small_int(N, 400, -2, 2, density=0.3)
    md = H.MD(H.Problem(J), H.make_schedule(10, 5), R, prec, require_exact=True)
    phi = _shared_phi(R, N, 401)
    md.set_state(H.HQA_STATE_PHI, phi)
    u = md.field()
    import torch
    phib = torch.tensor(phi, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    pb = orc.Problem(N, J=J)
    u64 = orc.field(pb, phib)
    assert np.max(np.abs(u - u64)) / np.max(np.abs(u64)) <= 1e-5
    uf = orc.field(pb, phi)
    _say(prec, "max |dh| vs fp64 phi", np.max(np.abs(u - uf)))


def test_csr_f32_field_within_1e5(H):
    rp, ci, v = inst.ea3d(16, 301)
    N, R = 4096, 100
    md = H.MD(H.Problem(row_ptr=rp, col=ci, val=v), H.make_schedule(10, 5), R, "f32")
    phi = _shared_phi(R, N, 5).astype(np.float32).astype(np.float64)
    md.set_state(H.HQA_STATE_PHI, phi)
    u = md.field()
    u64 = orc.field(orc.Problem(N, row_ptr=rp, col=ci, val=v), phi)
    assert np.max(np.abs(u - u64)) / np.max(np.abs(u64)) <= 1e-5


def test_bf16_and_fp8_storage_give_identical_runs(H):
    # +-1 / 0 couplings are exact in both BF16 and FP8 e4m3, so the two storage
    # forms must give bit-identical trajectories.
    N, R, T = 300, 32, 400
    J = inst.er_maxcut(N, 0.06, 500)
    out = []
    for prec in ("bf16", "fp8"):
        md = H.MD(H.Problem(J), H.make_schedule(T, 50), R, prec, seed=3, require_exact=True)
        md.run()
        md.sync()
        out.append((md.state(H.HQA_STATE_PHI), md.state(H.HQA_STATE_PHIBAR)))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("prec", ["f32", "bf16", "fp8"])
def test_z2_symmetry_all_precisions(H, prec):
    # h = 0: p0 -> -p0 gives phi -> -phi exactly (round-to-nearest-even is odd).
    N, R, T = 96, 16, 300
    J = inst.er_maxcut(N, 0.1, 600)
    p0 = orc.init_p0(9, N, R)
    res = []
    for sgn in (1, -1):
        md = H.MD(H.Problem(J), H.make_schedule(T, 30), R, prec, p0=sgn * p0)
        md.run()
        res.append(md.state(H.HQA_STATE_PHI))
    assert np.array_equal(res[0], -res[1])


# ------------------------------------------------------- read-out of FP32 runs
@pytest.mark.parametrize("layout", ["dense", "csr"])
def test_f32_readout_matches_oracle_on_same_phibar(H, layout):
    N, R, T, n = 180, 20, 600, 14
    J = inst.er_maxcut(N, 0.08, 700)
    if layout == "dense":
        P, pb = H.Problem(J), orc.Problem(N, J=J)
    else:
        rp, ci, v = inst.dense_to_csr(J)
        P, pb = H.Problem(row_ptr=rp, col=ci, val=v), orc.Problem(N, row_ptr=rp, col=ci, val=v)
    md = H.MD(P, H.make_schedule(T, 60), R, "f32", seed=11)
    md.run()
    g = md.classify(n, solve=True)
    bar = md.state(H.HQA_STATE_PHIBAR)
    A, s = orc.classify(bar, n)
    he, Je = orc.reduce(pb, A, s)
    code, Ered = orc.enumerate_exact(Je, he)
    sh = orc.merge(s, A, code)
    E, C = orc.energy(pb, sh)
    assert np.array_equal(g["amb_idx"], A) and np.array_equal(g["h_eff"], he)
    assert np.array_equal(g["code"], code) and np.array_equal(g["e_reduced"], Ered)
    assert np.array_equal(g["spins"], sh)
    assert np.array_equal(g["energy"], E) and np.array_equal(g["cut"], C)


# --------------------------------------------------------------- exact energies
@pytest.mark.parametrize("kind", ["sk", "int", "glass", "csr", "csr_int", "int_h"])
def test_ising_energy_exact(H, kind):
    """Exact energies and cuts: the binary64 fast path (integer J and h: every partial
    sum exact) and the fixed-point accumulator (real J), dense and CSR; 7 vectors of
    333 spins, each split into 6 row slices whose partial sums are added exactly."""
    N = 333
    h = None
    if kind == "sk":
        J = inst.sk(N, 800)
    elif kind in ("int", "csr_int"):
        J = inst.small_int(N, 801, -5, 5, density=0.5)
    elif kind == "int_h":
        J = inst.small_int(N, 804, -3, 3, density=0.3)
        h = np.random.default_rng(805).integers(-4, 5, N).astype(np.float64)
    else:
        J, h = inst.uniform_glass(N, 802)
    spins = inst.random_pm1((7, N), 803).astype(np.int8)
    if kind in ("csr", "csr_int"):
        rp, ci, v = inst.dense_to_csr(J)
        P = H.Problem(row_ptr=rp, col=ci, val=v, h=h)
        pb = orc.Problem(N, row_ptr=rp, col=ci, val=v, h=h)
    else:
        P, pb = H.Problem(J, h=h), orc.Problem(N, J=J, h=h)
    E, C = H.ising_energy(P, spins)
    Eo, Co = orc.energy(pb, spins)
    assert np.array_equal(E, Eo) and np.array_equal(C, Co)


@pytest.mark.parametrize("kind,N,V", [("glass", 3000, 1), ("int", 3000, 1), ("glass", 2000, 3),
                                      ("csr", 2500, 2), ("int", 100, 600)])
def test_ising_energy_exact_slices(H, kind, N, V):
    """One vector split into up to 47 row slices (few vectors fill the device), and 600
    vectors of one slice each: the same exact energies and cuts as the oracle."""
    _say("energy slices", kind, N, V)
    h = None
    if kind == "int":
        J = inst.small_int(N, 811, -4, 4, density=0.4)
        h = np.random.default_rng(812).integers(-3, 4, N).astype(np.float64)
    else:
        J, h = inst.uniform_glass(N, 813)
    spins = inst.random_pm1((V, N), 814).astype(np.int8)
    if kind == "csr":
        keep = np.triu(inst.random_pm1((N, N), 815) > 0, 1)   # half the couplings, symmetric
        rp, ci, v = inst.dense_to_csr(J * (keep | keep.T))
        P = H.Problem(row_ptr=rp, col=ci, val=v, h=h)
        pb = orc.Problem(N, row_ptr=rp, col=ci, val=v, h=h)
    else:
        P, pb = H.Problem(J, h=h), orc.Problem(N, J=J, h=h)
    E, C = H.ising_energy(P, spins)
    Eo, Co = orc.energy(pb, spins)
    assert np.array_equal(E, Eo) and np.array_equal(C, Co)


def _spanned(N, span, seed, top=-3):
    """Symmetric J (zero diagonal) and h whose nonzero values carry full 53-bit mantissas
    and exponents spread so that the bits of the set run from 2^top down to about
    2^(top - span + 1); an eighth of the mantissas are all ones and a few values sit at
    the largest magnitude."""
    rng = np.random.default_rng(seed)
    b = min(span, 53)                      # mantissa bits; the exponents spread the rest
    m = rng.integers(2**(b - 1), 2**b, size=(N, N), dtype=np.uint64).astype(np.float64)
    m[rng.random((N, N)) < 0.125] = float(2**b - 1)
    e = rng.integers(top - span + b, top + 1, size=(N, N))
    J = np.ldexp(m, e - (b - 1)) * np.where(rng.random((N, N)) < 0.5, -1.0, 1.0)
    J[rng.random((N, N)) < 0.02] = np.ldexp(float(2**b - 1), top - (b - 1))
    J = np.triu(J, 1)
    J = J + J.T
    h = np.ldexp(rng.integers(2**(b - 1), 2**b, size=N).astype(np.float64),
                 rng.integers(top - span + b, top + 1, size=N) - (b - 1))
    return J, h


@pytest.mark.parametrize("span", [60, 100, 130, 145])
def test_ising_energy_exact_level_sums(H, span):
    """Exact energies and cuts of real couplings whose bits span 60, 100 and 130 binades
    (two, three and four binary64 level sums at N = 300, 34 bits each) and 145 (beyond
    four levels: the fixed-point accumulator per term; the library refuses exact sums
    past 151): the oracle's values bit for bit."""
    N, V = 300, 9
    J, h = _spanned(N, span, 900 + span)
    spins = inst.random_pm1((V, N), 901).astype(np.int8)
    E, C = H.ising_energy(H.Problem(J, h=h), spins)
    Eo, Co = orc.energy(orc.Problem(N, J=J, h=h), spins)
    assert np.array_equal(E, Eo) and np.array_equal(C, Co)


@pytest.mark.parametrize("storage,prec", [("fp8", "fp8"), ("bf16", "bf16"), ("f32", "f32")])
def test_readout_energy_from_storage_copy(H, storage, prec):
    """Read-out energies on a handle whose stored couplings hold J exactly (small
    integers): the energy kernel reads the 1-, 2- or 4-byte copy instead of binary64.
    R = 70 (a full and a partial group of 64 vectors); energies and cuts equal the
    oracle's for the returned spins."""
    N, R = 403, 70
    J = inst.small_int(N, 831, -3, 3, density=0.4)
    h = np.random.default_rng(832).integers(-2, 3, N).astype(np.float64)
    md = H.MD(H.Problem(J, h=h, storage=storage), H.make_schedule(60, 10), R, prec, seed=3,
              require_exact=True)
    md.run()
    g = md.classify(9, solve=True)
    E, C = orc.energy(orc.Problem(N, J=J, h=h), g["spins"])
    assert np.array_equal(g["energy"], E) and np.array_equal(g["cut"], C)
    md.close()


@pytest.mark.parametrize("N,V,span", [(2, 1, 20), (3, 65, 20), (130, 129, 60), (257, 64, 100),
                                      (64, 200, 130)])
def test_ising_energy_vector_groups(H, N, V, span):
    """Tiny and ragged shapes of the many-vector energy kernel: one or two spins, vector
    counts just past a group of 64 (and of 32 and 16 on the multi-level paths): the
    oracle's energies and cuts bit for bit."""
    J, h = _spanned(N, span, 840 + N)
    spins = inst.random_pm1((V, N), 841).astype(np.int8)
    E, C = H.ising_energy(H.Problem(J, h=h), spins)
    Eo, Co = orc.energy(orc.Problem(N, J=J, h=h), spins)
    assert np.array_equal(E, Eo) and np.array_equal(C, Co)


# ------------------------------------------------------ determinism and resume
def test_checkpoint_resume_bit_identical(H):
    N, R, T = 160, 24, 500
    J = inst.sk(N, 900)
    for prec in ("f64", "f32", "bf16"):
        a = H.MD(H.Problem(J), H.make_schedule(T, 100), R, prec, seed=5)
        a.run()
        b = H.MD(H.Problem(J), H.make_schedule(T, 100), R, prec, seed=5)
        b.run(T // 2 + 37)
        ck = {w: b.state(w) for w in (H.HQA_STATE_PHI, H.HQA_STATE_P, H.HQA_STATE_WSUM)}
        c = H.MD(H.Problem(J), H.make_schedule(T, 100), R, prec, seed=99)
        for w, x in ck.items():
            c.set_state(w, x)
        H.hqa_md_set_step(c.h, T // 2 + 37)
        c.run()
        assert np.array_equal(a.state(H.HQA_STATE_PHIBAR), c.state(H.HQA_STATE_PHIBAR)), prec
        assert np.array_equal(a.state(H.HQA_STATE_PHI), c.state(H.HQA_STATE_PHI)), prec


# ------------------------------------------------------------------ error paths
def test_error_paths(H):
    N = 30
    J = inst.sk(N, 1000)
    bad = J.copy(); bad[0, 1] += 1.0
    with pytest.raises(H.HQAError) as e:
        H.MD(H.Problem(bad), H.make_schedule(10, 5), 2, "f32")
    assert e.value.status == H.HQA_EINVAL
    bad = J.copy(); bad[3, 3] = 1.0
    with pytest.raises(H.HQAError) as e:
        H.MD(H.Problem(bad), H.make_schedule(10, 5), 2, "f32")
    assert e.value.status == H.HQA_EINVAL
    with pytest.raises(H.HQAError) as e:
        H.MD(H.Problem(J), H.make_schedule(10, 5), 2, "fp8", require_exact=True)
    assert e.value.status == H.HQA_EUNSUPPORTED
    md = H.MD(H.Problem(J), H.make_schedule(10, 5), 2, "f32")
    with pytest.raises(H.HQAError) as e:
        md.classify(3)
    assert e.value.status == H.HQA_ESTATE
    md.run()
    with pytest.raises(H.HQAError) as e:
        md.classify(25, solve=True)
    assert e.value.status == H.HQA_EUNSUPPORTED
    with pytest.raises(H.HQAError) as e:
        md.classify(N + 1)
    assert e.value.status == H.HQA_EINVAL
    # solve outside {0, 1} is refused on the host (the tabu mode has its own entry point),
    # by hqa_classify and by hqa_classify_probs alike; no kernel is launched
    out = H.hqa_classify_out()
    spins = np.zeros((2, N), np.int8)
    out.spins = spins.ctypes.data
    prob = np.full((2, N, 3), 1.0 / 3.0, np.float32)
    for solve in (2, 3, -1):
        with pytest.raises(H.HQAError) as e:
            H.hqa_classify(md.h, 0, 3, solve, out, H.HQA_HOST)
        assert e.value.status == H.HQA_EINVAL
        with pytest.raises(H.HQAError) as e:
            H.hqa_classify_probs(md.h, 0, prob, H.HQA_HOST, 3, solve, out, H.HQA_HOST)
        assert e.value.status == H.HQA_EINVAL
    # a flux poisoned from the host overflows phi^5 -> non-finite flag at sync
    md = H.MD(H.Problem(J), H.make_schedule(10, 5), 2, "f32")
    md.set_state(H.HQA_STATE_PHI, np.full((2, N), 1e30))
    md.run()
    with pytest.raises(H.HQAError) as e:
        md.sync()
    assert e.value.status == H.HQA_ENONFINITE


@pytest.mark.parametrize("prec", ["fp8", "bf16"])
def test_lowp_trajectory_within_bound(H, prec):
    """The chosen forms against the oracle's binary64 trajectory over the first steps:
    within the derived forward error bound (tests/f32_bound.py) with the couplings
    rounded to their storage (exact for unit weights in FP8, 2^-8 relative in BF16) and
    the flux operand rounded to BF16 (2^-8 relative), FP32 accumulation (the matrix
    core's summation allowed twice the round-to-nearest error)."""
    from f32_bound import f32_bound
    R, T = 8, 2000
    if prec == "fp8":
        N = 300
        J = inst.er_maxcut(N, 0.05, 81)
        uJ = 0.0
    else:
        N = 200
        J = inst.sk(N, 82)
        uJ = 2.0 ** -8
    md = H.MD(H.Problem(J), H.make_schedule(T, 100), R, prec, seed=3,
              require_exact=(prec == "fp8"))
    e, phis = f32_bound(orc, orc.Problem(N, J=J), orc.MDParams(T=T, W=100), np.zeros((R, N)),
                        orc.init_p0(3, N, R), 30, uJ=uJ, uB=2.0 ** -8, gam_factor=2.0)
    for q in (1, 5, 10, 20, 30):
        md.run(q)
        err = np.max(np.abs(md.state(H.HQA_STATE_PHI) - phis[q]))
        _say(prec, "step", q, "max |phi - phi64|", err, "bound", e[q])
        assert err <= e[q]
    md.close()
