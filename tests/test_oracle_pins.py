"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: printed
constants, closed-form solutions of special cases, an independent ODE solver,
library routines (math.fsum, numpy lexsort), brute force on tiny inputs and
exact invariants.  Method: arXiv:2004.03972.
"""
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2004_03972_amd import instances as inst

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- exact sums
def test_exact_sum_matches_fsum(orc):
    rng = np.random.default_rng(7)
    for trial in range(50):
        n = int(rng.integers(1, 400))
        x = rng.standard_normal(n) * 10.0 ** rng.integers(-20, 20, size=n)
        # add cancellation: large terms and their negatives
        x = np.concatenate([x, -x[: n // 2] * (1 + 2.0 ** -52), [1e100, 1.0, -1e100]])
        rng.shuffle(x)
        assert orc.exact_sum(x) == math.fsum(x)
    # round-half-even tie: 1 + 2^-53 rounds to 1, (1+2^-52) + 2^-53 to 1 + 2^-51
    assert orc.exact_sum([1.0, 2.0 ** -53]) == math.fsum([1.0, 2.0 ** -53]) == 1.0
    x = [1.0 + 2.0 ** -52, 2.0 ** -53, 2.0 ** -110]
    assert orc.exact_sum(x) == math.fsum(x)


# -------------------------------------------------------- published constants
def test_splitmix64_published_vector(orc):
    # SplitMix64 started from state 0: the first outputs are the published test
    # vector of the generator (golden file cites the source).
    for row in _golden("splitmix64_state0.txt"):
        k, val = int(row[0]), int(row[1], 16)
        assert orc.splitmix64_at(0, k) == val


def test_schedule_printed_constants(orc):
    # Methods, "Scheduling functions for MD": values at tau = 0, 1/2, 1 for the
    # printed constants (alpha_f,rho1,rho2) = (0.008,4,3), (beta_f,k1,k2) = (0.12,0.05,1),
    # and for the linear reading rho2 = kappa2 = 0.
    for row in _golden("schedule_points.txt"):
        kind, tau2, a_exp, b_exp = row[0], int(row[1]), float(row[2]), float(row[3])
        prm = orc.PAPER_SCHEDULE if kind == "paper" else (0.008, 4.0, 0.0, 0.12, 0.05, 0.0)
        a, b = orc.schedule(1, prm)  # T = 1: grid tau_k = k/2
        assert a[tau2] == pytest.approx(a_exp, rel=1e-14)
        assert b[tau2] == pytest.approx(b_exp, rel=1e-14)


def test_c_star_from_printed_formula():
    # Methods, "MAX-CUT and Ising spin-glass": E*/N^(3/2) -> e0 + A N^(-omega),
    # C* = -E*/2 = 33933(4) for N = 2000.
    row = _golden("kn_maxcut_cstar.txt")[0]
    e0, A, omega, N, cstar, tol = map(float, row)
    E = (e0 + A * N ** (-omega)) * N ** 1.5
    assert abs(-E / 2 - cstar) <= tol


# ------------------------------------------------------- integrator closed forms
def _frozen(orc, T, M, alpha, beta, r_g=1.0, W=1):
    # Frozen schedule: alpha(tau) = alpha, beta(tau) = beta.
    prm = (alpha, 0.0, 0.0, beta, 0.0, 0.0)
    return orc.MDParams(T=T, W=W, M=M, r_g=r_g, schedule=prm, frozen=True, tau_fix=1.0)


def _run_traj(orc, pb, mp, phi0, p0):
    """phi^(q) for q = 0..T of each replica, stepping the oracle one step at a time."""
    phi, p = np.array(phi0, dtype=np.float64), np.array(p0, dtype=np.float64)
    out = [phi.copy()]
    for q in range(mp.T):
        orc.md_advance(pb, mp, phi, p, None, q, q + 1)
        out.append(phi.copy())
    return np.array(out), p


def test_harmonic_closed_form(orc):
    # M = 2, J = 0, h = 0, frozen alpha: phi^(m+2) = 2(1-alpha^2) phi^(m+1) - phi^(m),
    # so phi^(m) = alpha p0 sin(m theta)/sin(theta) with cos(theta) = 1 - alpha^2
    # (leapfrog of Methods on V = phi^2, textbook Stormer-Verlet).
    N, alpha, T = 5, 0.3, 400
    pb = orc.Problem(N, J=np.zeros((N, N)))
    mp = _frozen(orc, T, 2, alpha, 0.7)
    p0 = inst.random_pm1((1, N), 3)
    traj, _ = _run_traj(orc, pb, mp, np.zeros((1, N)), p0)
    th = math.acos(1 - alpha ** 2)
    m = np.arange(T + 1)[:, None, None]
    exact = alpha * p0[None] * np.sin(m * th) / math.sin(th)
    assert np.max(np.abs(traj - exact)) < 1e-12


def test_two_spin_normal_modes(orc):
    # M = 2, two spins coupled by J12, frozen (alpha, beta): the modes phi1 +- phi2
    # obey cos(theta_pm) = 1 - alpha (2 alpha +- beta J12) / 2.
    alpha, beta, J12, T = 0.2, 0.5, 0.6, 300
    J = np.array([[0.0, J12], [J12, 0.0]])
    pb = orc.Problem(2, J=J)
    mp = _frozen(orc, T, 2, alpha, beta)
    p0 = np.array([[1.0, -1.0], [1.0, 1.0]])
    traj, _ = _run_traj(orc, pb, mp, np.zeros((2, 2)), p0)
    m = np.arange(T + 1)
    for sgn in (+1, -1):
        th = math.acos(1 - alpha * (2 * alpha + sgn * beta * J12) / 2)
        mode = traj[:, :, 0] + sgn * traj[:, :, 1]          # [T+1, R]
        amp = alpha * (p0[:, 0] + sgn * p0[:, 1])            # drift of the first step
        exact = amp[None, :] * np.sin(m[:, None] * th) / math.sin(th)
        assert np.max(np.abs(mode - exact)) < 1e-12


def _hmd_numpy_grad(J, h, M, a, b, phi):
    # gradient of Eq. 3 in phi, written from the Hamiltonian: a M phi^(M-1) + b (J phi + 2 h |phi|)
    return a * M * phi ** (M - 1) + b * (J @ phi + 2 * h * np.abs(phi))


def test_force_is_gradient_of_hmd(orc):
    # The kick's force must be d H_MD / d phi (Hamilton equations) -- checked by central
    # finite differences of the oracle's own H_MD evaluator, which is Eq. 3 term by term.
    N = 6
    J, h = inst.uniform_glass(N, 11)
    pb = orc.Problem(N, J=J, h=h)
    mp = orc.MDParams(T=10, W=1, M=6)
    rng = np.random.default_rng(5)
    phi = rng.uniform(-1.2, 1.2, size=N)
    q = 3
    F = orc.force(pb, mp, q, phi)
    eps = 1e-6
    fd = np.empty(N)
    for i in range(N):
        e = np.zeros(N); e[i] = eps
        Hp = orc.hmd(pb, mp, q, (phi + e)[None], np.zeros((1, N)))[0]
        Hm = orc.hmd(pb, mp, q, (phi - e)[None], np.zeros((1, N)))[0]
        fd[i] = (Hp - Hm) / (2 * eps)
    assert np.max(np.abs(F - fd)) < 1e-7 * max(1.0, np.max(np.abs(F)))
    # and the kinetic part: dH/dp = alpha p
    p = rng.uniform(-1, 1, size=N)
    i = 2
    e = np.zeros(N); e[i] = eps
    dHdp = (orc.hmd(pb, mp, q, phi[None], (p + e)[None])[0] - orc.hmd(pb, mp, q, phi[None], (p - e)[None])[0]) / (2 * eps)
    assert dHdp == pytest.approx(mp.alpha[2 * q] * p[i], rel=1e-7)


def _ode_reference(orc, J, h, M, T0, phi0, p0):
    # Hamilton equations g dphi/dtau = dH/dp, g dp/dtau = -dH/dphi (Eq. 3, 4) with the
    # paper's time-dependent schedule and a fixed g = 1/T0, solved by an independent
    # adaptive integrator.
    N = J.shape[0]
    af, r1, r2, bf, k1, k2 = orc.PAPER_SCHEDULE
    g = 1.0 / T0

    def rhs(tau, y):
        phi, p = y[:N], y[N:]
        a = af * (tau + r1 * (1 - tau) + r2 * tau * (tau - 1))
        b = bf * (tau + k1 * (1 - tau) + k2 * tau * (tau - 1))
        return np.concatenate([a * p / g, -_hmd_numpy_grad(J, h, M, a, b, phi) / g])

    sol = solve_ivp(rhs, (0, 1), np.concatenate([phi0[0], p0[0]]), method="DOP853",
                    rtol=1e-13, atol=1e-13)
    return sol.y[:N, -1]


def _leapfrog_errors(orc, J, h, M, T0, phi0, p0, rs):
    ref = _ode_reference(orc, J, h, M, T0, phi0, p0)
    pb = orc.Problem(J.shape[0], J=J, h=h)
    errs = []
    for r in rs:
        mp = orc.MDParams(T=int(round(T0 / r)), W=1, M=M, r_g=r)
        _, phiT, _ = orc.md_run(pb, mp, phi0, p0)
        errs.append(np.max(np.abs(phiT[0] - ref)))
    return errs


def test_leapfrog_second_order_against_ode_solver(orc):
    # Steps delta-tau = r g.  The leapfrog with kicks at integer times, drifts at half
    # times and the initial half step converges as r^2 to the ODE solution (Methods:
    # O(delta-tau^2) error).  A kick or drift taken at the wrong grid point of the
    # schedule, or a missing initial half step, drops the order to 1 (ratio 2).
    N, T0, M = 4, 60, 6
    J, _ = inst.uniform_glass(N, 21)
    J *= 0.5
    p0 = inst.random_pm1((1, N), 4)
    phi0 = np.random.default_rng(8).uniform(-0.3, 0.3, size=(1, N))
    errs = _leapfrog_errors(orc, J, np.zeros(N), M, T0, phi0, p0, (1.0, 0.5, 0.25, 0.125))
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    assert all(3.9 < x < 4.1 for x in ratios), (errs, ratios)
    # With a field the force has a kink at phi = 0 (h |phi| phi); the scheme still
    # converges to the ODE solution, which pins the field term's sign and factor 2.
    _, h = inst.uniform_glass(N, 21)
    errs = _leapfrog_errors(orc, J, h, M, T0, phi0, p0, (1.0, 0.125))
    assert errs[1] < 3e-6 and errs[0] / errs[1] > 25, errs


def test_time_reversibility(orc):
    # Frozen schedule: K steps forward, negate the integer-time momentum, K steps again
    # recovers phi^(0) and -p^(0) (Methods: time reversibility without explicit tau).
    N, K = 12, 300
    J, h = inst.uniform_glass(N, 31)
    pb = orc.Problem(N, J=J * 0.3, h=h * 0.3)
    mp = _frozen(orc, 2 * K, 6, 0.02, 0.05, W=1)
    rng = np.random.default_rng(9)
    phi0 = rng.uniform(-0.5, 0.5, size=(2, N))
    p0 = inst.random_pm1((2, N), 10)
    phi, p = phi0.copy(), p0.copy()
    orc.md_advance(pb, mp, phi, p, None, 0, K)
    p_int = orc.integer_p(pb, mp, K, phi, p)
    phi2, p2 = phi.copy(), -p_int
    orc.md_advance(pb, mp, phi2, p2, None, 0, K)
    p2_int = orc.integer_p(pb, mp, K, phi2, p2)
    assert np.max(np.abs(phi2 - phi0)) < 1e-12
    assert np.max(np.abs(p2_int + p0)) < 1e-12


def test_energy_drift_second_order(orc):
    # Frozen schedule: H_MD is conserved by the exact flow; the leapfrog error stays
    # bounded and its maximum scales as r^2 over a fixed physical time.
    N = 10
    J = inst.sk(N, 41, std=0.5)
    pb = orc.Problem(N, J=J)
    p0 = inst.random_pm1((1, N), 12)
    phi0 = np.random.default_rng(13).uniform(-0.4, 0.4, size=(1, N))
    maxerr = []
    for r in (1.0, 0.5, 0.25):
        K = int(round(400 / r))
        mp = _frozen(orc, K, 6, 0.05, 0.08, r_g=r)
        phi, p = phi0.copy(), p0.copy()
        H0 = orc.hmd(pb, mp, 0, phi, p)[0]
        dev = 0.0
        for q in range(K):
            orc.md_advance(pb, mp, phi, p, None, q, q + 1)
            Hq = orc.hmd(pb, mp, q + 1, phi, orc.integer_p(pb, mp, q + 1, phi, p))[0]
            dev = max(dev, abs(Hq - H0))
        maxerr.append(dev)
    r1, r2 = maxerr[0] / maxerr[1], maxerr[1] / maxerr[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, maxerr


# ------------------------------------------------------------- exact invariants
def test_sign_and_gauge_symmetry(orc):
    # h = 0: p0 -> -p0 gives phi -> -phi exactly; a gauge G = diag(g), g in {+-1}^N,
    # applied as (J, h, p0) -> (GJG, Gh, Gp0) gives phi -> G phi exactly.
    N, T = 24, 300
    J = inst.sk(N, 51)
    pb = orc.Problem(N, J=J)
    mp = orc.MDParams(T=T, W=50)
    p0 = orc.init_p0(5, N, 3)
    z = np.zeros_like(p0)
    bar, phiT, _ = orc.md_run(pb, mp, z, p0)
    bar2, phiT2, _ = orc.md_run(pb, mp, z, -p0)
    assert np.array_equal(phiT2, -phiT) and np.array_equal(bar2, -bar)
    Jh, h = inst.uniform_glass(N, 52)
    G = inst.random_pm1(N, 53)
    pbh = orc.Problem(N, J=Jh, h=h)
    pbg = orc.Problem(N, J=G[:, None] * Jh * G[None, :], h=G * h)
    _, a, _ = orc.md_run(pbh, mp, z, p0)
    _, b, _ = orc.md_run(pbg, mp, z, p0 * G[None, :])
    assert np.array_equal(b, a * G[None, :])


def test_dense_and_csr_agree_bitwise(orc):
    N = 40
    J = inst.small_int(N, 61, density=0.2)
    rp, ci, v = inst.dense_to_csr(J)
    mp = orc.MDParams(T=200, W=20)
    p0 = orc.init_p0(1, N, 4)
    z = np.zeros_like(p0)
    a = orc.md_run(orc.Problem(N, J=J), mp, z, p0)
    b = orc.md_run(orc.Problem(N, row_ptr=rp, col=ci, val=v), mp, z, p0)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_window_is_mean_of_last_w_fluxes(orc):
    N, T, W = 16, 120, 25
    J = inst.sk(N, 71)
    pb = orc.Problem(N, J=J)
    mp = orc.MDParams(T=T, W=W)
    p0 = orc.init_p0(2, N, 2)
    traj, _ = _run_traj(orc, pb, mp, np.zeros_like(p0), p0)
    bar, phiT, _ = orc.md_run(pb, mp, np.zeros_like(p0), p0)
    assert np.array_equal(phiT, traj[-1])
    expect = np.array([[math.fsum(traj[T - W + 1:, r, i]) / W for i in range(N)] for r in range(2)])
    assert np.max(np.abs(bar - expect)) <= 1e-15 * W


# ------------------------------------------------------ classify / reduce / solve
def test_classify_matches_lexsort(orc):
    rng = np.random.default_rng(81)
    R, N, n = 5, 300, 37
    bar = rng.standard_normal((R, N))
    bar[:, ::7] = np.round(bar[:, ::7], 1)          # many ties in |phibar|
    bar[0, :5] = 0.0                                 # sgn(0) = +1
    A, s = orc.classify(bar, n)
    for r in range(R):
        order = np.lexsort((np.arange(N), np.abs(bar[r])))
        assert np.array_equal(A[r], np.sort(order[:n]))
    assert np.array_equal(s, np.where(bar < 0, -1, 1).astype(np.int8))


def _brute_energies(J, h):
    # energies of all 2^n states, bit a set means x_a = -1; exact via fsum per state
    n = J.shape[0]
    codes = np.arange(1 << n)
    X = 1 - 2 * ((codes[:, None] >> np.arange(n)[None, :]) & 1)
    iu = np.triu_indices(n, 1)
    out = np.empty(codes.size)
    for c in codes:
        x = X[c]
        out[c] = math.fsum(list(J[iu] * x[iu[0]] * x[iu[1]]) + list(h * x))
    return out


@pytest.mark.parametrize("kind", ["int", "real"])
def test_enumeration_matches_brute_force(orc, kind):
    rng = np.random.default_rng(91 if kind == "int" else 92)
    R, n = 3, 10
    if kind == "int":
        Je = np.stack([inst.small_int(n, 100 + r, -2, 2) for r in range(R)])
        he = rng.integers(-3, 4, size=(R, n)).astype(float)
    else:
        Je = np.stack([inst.sk(n, 200 + r) for r in range(R)])
        he = rng.standard_normal((R, n))
    code, E = orc.enumerate_exact(Je, he)
    for r in range(R):
        e = _brute_energies(Je[r], he[r])
        assert E[r] == e.min()
        assert code[r] == int(np.flatnonzero(e == e.min())[0])   # ties -> smallest code


def test_energy_and_cut_exact(orc):
    N = 60
    J, h = inst.uniform_glass(N, 111)
    s = inst.random_pm1((4, N), 112).astype(np.int8)
    E, cut = orc.energy(orc.Problem(N, J=J, h=h), s)
    iu = np.triu_indices(N, 1)
    for v in range(4):
        x = s[v].astype(float)
        assert E[v] == math.fsum(list(J[iu] * x[iu[0]] * x[iu[1]]) + list(h * x))
        assert cut[v] == math.fsum(J[iu][x[iu[0]] != x[iu[1]]])
    # MAX-CUT mapping (Methods): J = w, h = 0 gives C(s) = C0 - H(s)/2, C0 = sum_{i<j} w / 2
    W = inst.er_maxcut(N, 0.3, 113)
    E, cut = orc.energy(orc.Problem(N, J=W), s)
    C0 = W[iu].sum() / 2
    assert np.all(cut == C0 - E / 2)
    x = s.astype(float)
    assert np.all(cut == [0.5 * np.sum(W[iu] * (1 - x[v][iu[0]] * x[v][iu[1]])) for v in range(4)])


def test_reduced_hamiltonian_identity(orc):
    # HQA section: H(s) = H'(s_A) + const with the frozen spins fixed.
    N, n = 30, 8
    J = inst.small_int(N, 121, -4, 4)
    h = np.random.default_rng(122).integers(-5, 6, size=N).astype(float)
    pb = orc.Problem(N, J=J, h=h)
    rng = np.random.default_rng(123)
    bar = rng.standard_normal((1, N))
    A, s = orc.classify(bar, n)
    he, Je = orc.reduce(pb, A, s)
    iu = np.triu_indices(n, 1)
    diffs = []
    for c in range(1 << n):
        full = orc.merge(s, A, np.array([c]))
        x = 1 - 2 * ((c >> np.arange(n)) & 1)
        Hp = np.sum(Je[0][iu] * x[iu[0]] * x[iu[1]]) + np.sum(he[0] * x)
        diffs.append(orc.energy(pb, full)[0][0] - Hp)
    assert len(set(diffs)) == 1


def test_hqa_full_subproblem_is_ground_state(orc):
    # With n = N the reduced problem is the whole instance: HQA must return the brute-force
    # ground energy; for any n, HQA is never worse than the MD-alone read-out.
    for seed, kind in ((131, "sk"), (132, "er"), (133, "glass")):
        N = 12
        h = None
        if kind == "sk":
            J = inst.sk(N, seed)
        elif kind == "er":
            J = inst.er_maxcut(N, 0.5, seed)
        else:
            J, h = inst.uniform_glass(N, seed)
        pb = orc.Problem(N, J=J, h=h)
        mp = orc.MDParams(T=300, W=30)
        p0 = orc.init_p0(seed, N, 3)
        out = orc.hqa(pb, mp, p0, n=N)
        gs = _brute_energies(J, np.zeros(N) if h is None else h).min()
        assert np.all(out["E_hqa"] == gs)
        out = orc.hqa(pb, mp, p0, n=5)
        assert np.all(out["E_hqa"] <= out["E_md"])


def test_enumeration_blocks_equal_one_scan(orc):
    # splitting the code range into ascending blocks leaves the minimiser unchanged,
    # ties included (h = 0 mirror pairs; small-integer couplings with many equal sums)
    from paper_2004_03972_amd import instances as inst
    for n in (1, 2, 5, 9, 13):
        rng = np.random.default_rng(n)
        Jr = np.triu(rng.standard_normal((n, n)), 1)
        Jr = Jr + Jr.T
        Ji = inst.small_int(n, 40 + n, -1, 1, density=0.8) if n > 1 else np.zeros((1, 1))
        for J, h in ((Jr, rng.standard_normal(n)), (Ji, np.zeros(n)),
                     (Ji, rng.integers(-1, 2, n).astype(float))):
            a = orc.enumerate_exact(J[None], h[None])
            for th in (1, 3, 8):
                b = orc.enumerate_exact_blocks(J[None], h[None], nthreads=th)
                assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_field_export_exact_on_dyadic_inputs(orc):
    # u_i = sum_j J_ij phi_j (the field term of Eq. 3).  With integer couplings and
    # fluxes k / 1024 every product and partial sum is exact in binary64, so the
    # oracle's field must equal the integer result exactly.  J is not symmetric here,
    # so a transposed operand fails; three replicas with different fluxes catch a
    # replica-indexing slip; the CSR form of the same matrix must agree.
    from paper_2004_03972_amd import instances as inst
    rng = np.random.default_rng(11)
    N, R = 37, 3
    Ji = rng.integers(-3, 4, (N, N)) * (rng.random((N, N)) < 0.6)
    np.fill_diagonal(Ji, 0)
    k = rng.integers(-2000, 2001, (R, N))
    exact = np.array([[sum(int(Ji[i, j]) * int(k[r, j]) for j in range(N)) for i in range(N)]
                      for r in range(R)])
    u = orc.field(orc.Problem(N, J=Ji.astype(float)), k / 1024.0)
    assert np.array_equal(u * 1024.0, exact.astype(float))
    rp, ci, v = inst.dense_to_csr(Ji.astype(float))
    u2 = orc.field(orc.Problem(N, row_ptr=rp, col=ci, val=v), k / 1024.0)
    assert np.array_equal(u2, u)
    assert not np.array_equal(orc.field(orc.Problem(N, J=Ji.T.astype(float)), k / 1024.0), u)


def test_divergence_follows_leapfrog_stability_bound(orc):
    """Why some runs diverge (schedule sweeps with kappa2 < 0): the leapfrog of the
    Methods, linearised about phi for the potential alone, reads
    phi_(m+1) - 2 phi_m + phi_(m-1) = -k phi_m with k = alpha^2 M (M-1) phi^(M-2), and is
    stable only for 0 < k < 4.  On the spin glass with fields at the field scale of
    N = 10^4 (J ~ U[-1, 1] scaled by sqrt(10^4 / N), h ~ U[-2, 2]), the binary64 oracle
    run with kappa2 = -1 blows up (|phi| > 10^3 or non-finite) only after
    k = alpha^2 M (M-1) max|phi|^(M-2) has passed 4, shortly before; with kappa2 = +1
    and the same instance and initial momenta, k stays below 4 and the run stays
    finite."""
    from paper_2004_03972_amd import instances as inst
    N, M, T = 200, 6, 2000
    J, h = inst.uniform_glass(N, 4)
    pb = orc.Problem(N, J=J * np.sqrt(1e4 / N), h=h)
    p0 = orc.init_p0(1, N, 32)[3:4]

    def trace(kappa2):
        mp = orc.MDParams(T=T, W=100, M=M, schedule=(0.008, 4.0, 3.0, 0.12, 0.05, kappa2))
        phi, p = np.zeros((1, N)), p0.copy()
        first_k4, kmax = None, 0.0
        for q in range(T):
            a = mp.alpha[2 * q]
            k = a * a * M * (M - 1) * np.max(np.abs(phi)) ** (M - 2)
            if first_k4 is None and k > 4.0:
                first_k4 = q
            kmax = max(kmax, k)
            try:
                orc.md_advance(pb, mp, phi, p, None, q, q + 1)
            except FloatingPointError:
                return first_k4, q, kmax
            if np.max(np.abs(phi)) > 1e3:
                return first_k4, q, kmax
        return first_k4, None, kmax

    first, blow, _ = trace(-1.0)
    assert blow is not None and first is not None
    assert first < blow <= first + 100
    first, blow, kmax = trace(1.0)
    assert blow is None and first is None and kmax < 4.0
