"""First-order forward error bound of a binary32 MD trajectory against the binary64
oracle's, for the parity tests of the binary32 forms.

Both runs start from the same fluxes and momenta and take the same leapfrog steps
(Methods, "Leapfrog algorithm"; force of Eq. 3).  The binary32 run differs by
  - the schedule values rounded to binary32 (relative error <= u),
  - the couplings rounded to the storage type (relative error <= uJ per coupling), and
    for the low-precision forms the flux operand rounded to BF16 (relative error <= uB),
  - the field accumulated in binary32 (any order: error <= gamma_(N+2) sum_j |J_ij phi_j|,
    gamma_k = k u / (1 - k u)),
  - one rounding (<= u relative) per operation of the update,
with u = 2^-24.  With e_phi, e_p the largest errors of the fluxes phi^(q) and momenta
p^(q-1/2) so far, the errors after step q are bounded to first order by
  |du|   <= sum_j |J_ij| e_phi + (uJ + uB + uJ uB + gamma) sum_j |J_ij| |phi_j|
  |dv|   <= (M-1) |phi|^(M-2) e_phi + (M-2) u |phi|^(M-1)           (v = phi^(M-1))
  |dg|   <= |du| + 2 |h| e_phi + u (|u| + 4 |h| |phi|)              (g = u + 2 h |phi|)
  |dF|   <= u a M |v| + a M |dv| + u b |g| + b |dg| + u (2 a M |v| + b |g| + |F|)
  e_p'   <= e_p + kick |dF| + u |p'|
  e_phi' <= e_phi + u a_h |p'| + a_h e_p' + u (a_h |p'| + |phi'|),
(gam_factor > 1 widens gamma for summation whose roundings are not to nearest, such as
a matrix core's internal accumulation), each magnitude taken from the binary64
trajectory plus its error bound (so the power's
mean-value bound and the rounding terms hold as written).  The products of two small
error terms that the list omits (a rounded schedule value times an error, say) are
below u times the terms kept; they are covered by a factor 1.01 per step."""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24


def f32_bound(orc, pb, mp, phi0, p0, steps, uJ=U32, u=U32, uB=0.0, gam_factor=1.0):
    """Per-step bounds (e_phi, e_p) for `steps` steps from (phi0, p0), together with the
    binary64 trajectory's fluxes at every step: returns (e_phi[steps+1], phi64 list)."""
    N = pb.N
    J = pb.J if pb.J is not None else _dense(pb)
    h = np.zeros(N) if pb.h is None else pb.h
    aJ = np.abs(J)
    gam = gam_factor * (N + 2) * u / (1 - gam_factor * (N + 2) * u)
    M = mp.M
    phi, p = np.array(phi0, dtype=np.float64, copy=True), np.array(p0, dtype=np.float64, copy=True)
    ephi, ep = 0.0, 0.0
    out_e, out_phi = [0.0], [phi.copy()]
    for q in range(steps):
        a, b, ah = mp.alpha[2 * q], mp.beta[2 * q], mp.alpha[2 * q + 1]
        kick = 0.5 if q == 0 else 1.0
        ph = np.abs(phi) + ephi
        uu = phi @ J.T
        du = ephi * aJ.sum(axis=1)[None, :] + (uJ + uB + uJ * uB + gam) * (ph @ aJ.T)
        v = np.abs(phi) ** (M - 1) + 0.0
        dv = (M - 1) * ph ** (M - 2) * ephi + (M - 2) * u * ph ** (M - 1)
        g = np.abs(uu) + np.abs(du) + 2 * np.abs(h)[None, :] * ph
        dg = du + 2 * np.abs(h)[None, :] * ephi + u * (g + 4 * np.abs(h)[None, :] * ph)
        vb = ph ** (M - 1)
        F = a * M * vb + b * g
        dF = u * a * M * vb + a * M * dv + u * b * g + b * dg + u * (2 * a * M * vb + b * g + F)
        orc.md_advance(pb, mp, phi, p, None, q, q + 1)
        pm = np.abs(p) + ep + kick * np.max(dF)
        ep_new = ep + kick * np.max(dF) + u * np.max(pm)
        ephi_new = (ephi + u * ah * np.max(pm) + ah * ep_new
                    + u * (ah * np.max(pm) + np.max(np.abs(phi)) + ephi))
        ephi, ep = 1.01 * ephi_new, 1.01 * ep_new
        out_e.append(ephi)
        out_phi.append(phi.copy())
    return np.array(out_e), out_phi


def _dense(pb):
    J = np.zeros((pb.N, pb.N))
    for i in range(pb.N):
        for e in range(pb.row_ptr[i], pb.row_ptr[i + 1]):
            J[i, pb.col[e]] = pb.val[e]
    return J
