"""Pins of the FP64 oracle of the learned early stop (features, MLP, Adam).

The paper has no learned component; the definitions are this library's.  The pins
check the oracle against mathematics it must satisfy: GELU identities and the
normal CDF (scipy), softmax invariances, a hidden-unit permutation (catches
transposed weight indices), finite differences of the loss, the closed form of
Adam's first step, and features of a harmonic trajectory known in closed form.
"""
import math

import numpy as np
import pytest
from scipy.stats import norm

from paper_2004_03972_amd import instances as inst

NF, H1, H2, NC = 12, 64, 64, 3
OFF = dict(W1=0, b1=H1 * NF, W2=H1 * NF + H1, b2=H1 * NF + H1 + H2 * H1,
           W3=H1 * NF + H1 + H2 * H1 + H2, b3=H1 * NF + H1 + H2 * H1 + H2 + NC * H2)


def _rand_params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, size=5187)


def test_gelu_identities(orc):
    assert orc.gelu(0.0) == 0.0
    for x in (0.3, 1.0, 2.5, -1.7):
        assert orc.gelu(x) - orc.gelu(-x) == pytest.approx(x, abs=1e-15)
        assert orc.gelu(x) == pytest.approx(x * norm.cdf(x), rel=1e-14, abs=1e-16)
    assert orc.gelu(1.0) == pytest.approx(0.841344746, abs=1e-9)   # Phi(1), normal tables
    assert orc.gelu(40.0) == 40.0


def test_softmax_and_bias_invariances(orc):
    P = _rand_params(1)
    x = np.random.default_rng(2).normal(size=(7, NF))
    pr = orc.mlp_forward(P, x)
    assert np.allclose(pr.sum(1), 1.0, atol=1e-15)
    Q = P.copy()
    Q[OFF["b3"]:OFF["b3"] + 3] += 5.0               # common shift of the logits
    assert np.allclose(orc.mlp_forward(Q, x), pr, atol=1e-14)
    Z = P.copy()
    Z[OFF["W3"]:OFF["W3"] + NC * H2] = 0.0           # no hidden signal: softmax(b3)
    b3 = Z[OFF["b3"]:OFF["b3"] + 3]
    e = np.exp(b3 - b3.max())
    assert np.allclose(orc.mlp_forward(Z, x), np.tile(e / e.sum(), (7, 1)), atol=1e-15)


def test_hidden_permutation_invariance(orc):
    P = _rand_params(3)
    x = np.random.default_rng(4).normal(size=(5, NF))
    rng = np.random.default_rng(5)
    p1, p2 = rng.permutation(H1), rng.permutation(H2)
    W1 = P[OFF["W1"]:OFF["b1"]].reshape(H1, NF)
    b1 = P[OFF["b1"]:OFF["W2"]]
    W2 = P[OFF["W2"]:OFF["b2"]].reshape(H2, H1)
    b2 = P[OFF["b2"]:OFF["W3"]]
    W3 = P[OFF["W3"]:OFF["b3"]].reshape(NC, H2)
    Q = np.concatenate([W1[p1].ravel(), b1[p1], W2[p2][:, p1].ravel(), b2[p2],
                        W3[:, p2].ravel(), P[OFF["b3"]:]])
    assert np.allclose(orc.mlp_forward(Q, x), orc.mlp_forward(P, x), atol=1e-14)
    # a transposed W2 (a plausible indexing slip) changes the output
    Qt = np.concatenate([W1.ravel(), b1, W2.T.ravel(), b2, W3.ravel(), P[OFF["b3"]:]])
    assert not np.allclose(orc.mlp_forward(Qt, x), orc.mlp_forward(P, x), atol=1e-6)


def _loss(orc, P, x, y, cw):
    pr = orc.mlp_forward(P, x)
    w = cw[y]
    return -np.sum(w * np.log(pr[np.arange(len(y)), y])) / w.sum()


def test_gradient_matches_finite_differences(orc):
    P = _rand_params(6)
    rng = np.random.default_rng(7)
    x = rng.normal(size=(9, NF))
    y = rng.integers(0, 3, size=9).astype(np.int32)
    cw = np.array([1.0, 2.5, 7.0])
    L, g = orc.mlp_loss_grad(P, x, y, cw)
    assert L == pytest.approx(_loss(orc, P, x, y, cw), rel=1e-13)
    idx = np.concatenate([rng.choice(np.arange(OFF[k], OFF[k] + 40), 6, replace=False)
                          for k in ("W1", "b1", "W2", "b2", "W3")] + [np.arange(OFF["b3"], OFF["b3"] + 3)])
    eps = 1e-6
    for k in idx:
        e = np.zeros_like(P); e[k] = eps
        fd = (_loss(orc, P + e, x, y, cw) - _loss(orc, P - e, x, y, cw)) / (2 * eps)
        assert g[k] == pytest.approx(fd, rel=2e-6, abs=1e-9), k


def test_adam_first_steps_closed_form(orc):
    rng = np.random.default_rng(8)
    P0 = rng.normal(size=50)
    g = rng.normal(size=50)
    P, m, v = P0.copy(), np.zeros(50), np.zeros(50)
    lr, eps = 1e-2, 1e-8
    orc.adam_step(P, g, m, v, 1, lr=lr, eps=eps)
    # t = 1: bias-corrected moments are g and g^2, the step is lr g / (|g| + eps)
    assert np.allclose(P, P0 - lr * g / (np.abs(g) + eps), rtol=1e-14, atol=1e-15)
    orc.adam_step(P, g, m, v, 2, lr=lr, eps=eps)
    assert np.allclose(P, P0 - 2 * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("every", [1, 3])
def test_features_of_harmonic_trajectory(orc, every):
    # J = 0, h = 0, M = 2, frozen alpha: phi^(q) = alpha p0 sin(q th)/sin th, cos th = 1 - alpha^2,
    # p^(q+1/2) = (phi^(q+1) - phi^(q)) / alpha; the field and the row norms vanish.  With
    # every > 1 the window statistics sample the steps K0, K0 + every, ... below K1.
    N, R, T, alpha = 6, 2, 60, 0.35
    K0, K1 = 10, 47
    pb = orc.Problem(N, J=np.zeros((N, N)))
    mp = orc.MDParams(T=T, W=1, M=2, schedule=(alpha, 0, 0, 0.5, 0, 0), frozen=True, tau_fix=1.0)
    p0 = inst.random_pm1((R, N), 11)
    feat, phiK, _ = orc.es_features(pb, mp, np.zeros((R, N)), p0, K0, K1, every)
    th = math.acos(1 - alpha ** 2)
    q = np.arange(T + 1)[:, None, None]
    phi = alpha * p0[None] * np.sin(q * th) / math.sin(th)            # [T+1, R, N]
    steps = np.arange(K0, K1, every)
    new = phi[steps + 1]
    old = phi[steps]
    p = (new - old) / alpha
    sig = np.sqrt(np.mean(phi[K1] ** 2, axis=1))[:, None]
    pm = np.mean(np.mean(p ** 2, axis=0), axis=1)[:, None]
    m0 = new.mean(0)
    want = np.stack([m0 / sig, np.sqrt(np.maximum((new ** 2).mean(0) - m0 ** 2, 0)) / sig,
                     np.abs(new).mean(0) / sig, phi[K1] / sig,
                     np.abs(2 * (new > 0).mean(0) - 1), ((new < 0) != (old < 0)).mean(0),
                     np.zeros((R, N)), np.zeros((R, N)), np.zeros((R, N)),
                     (p ** 2).mean(0) / pm, np.zeros((R, N)), np.full((R, N), K1 / T)], axis=-1)
    assert np.allclose(phiK, phi[K1], atol=1e-13)
    assert np.allclose(feat, want, atol=1e-10)


def test_features_sign_symmetry_and_trajectory(orc):
    # h = 0: p0 -> -p0 flips phi, u and nu; features 0, 3, 6 change sign, the rest stay.
    N, R, T = 30, 3, 400
    J = inst.er_maxcut(N, 0.3, 12)
    pb = orc.Problem(N, J=J)
    mp = orc.MDParams(T=T, W=10)
    p0 = orc.init_p0(3, N, R)
    z = np.zeros((R, N))
    f, phi, p = orc.es_features(pb, mp, z, p0, 100, 250)
    g, phi2, _ = orc.es_features(pb, mp, z, -p0, 100, 250)
    flip = np.ones(NF); flip[[0, 3, 6]] = -1
    assert np.allclose(g, f * flip, atol=1e-12)
    ref = z.copy(); pr = p0.copy()
    orc.md_advance(pb, mp, ref, pr, None, 0, 250)
    assert np.array_equal(phi, ref) and np.array_equal(p, pr)
    assert np.all(np.abs(f[..., 4]) <= 1) and np.all((f[..., 5] >= 0) & (f[..., 5] <= 1))
