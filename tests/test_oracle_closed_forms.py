"""Closed-form pins of the oracle's pair arithmetic and global totals.

The quantities are recomputed here from the definitions of Sec. 2.2 with
ingredients obtained by a different route than the oracle's own code:

* the kernel gradient grad_i W_ij by fourth-order central differences of the
  kernel value W (itself pinned by its unit integral and lattice sum), never
  by the oracle's closed-form gradient factor;
* the sound speed c_k = sqrt(dp/drho) at rho_k by central differences of the
  Tait pressure (pinned by p(rho0) = 0 and the hydrostatic closed form);
* the artificial viscosity isolated as the part of the acceleration that is
  linear in alpha (two oracle runs, alpha and 0).

Each case is built so that a plausible slip changes the result by far more
than the tolerance: separations and velocities are fully 3-D (a transposed
or dropped component shows), the pair approaches (the viscous branch is
live), rho_i != rho_j and both differ from rho0 (c_bar vs c0, rho_bar vs rho_i
differ), eta^2 = 0.01 h^2 is much smaller than r^2 (eta vs eta^2 differ by a
large factor), and h != 1 (a dropped h shows).
"""
import math

import numpy as np
import pytest

from paper_1210_1017_amd import cases



def _params(dp=0.01, alpha=0.01, g=(0.0, 0.0, 0.0)):
    p = cases.base_params(dp, alpha=alpha)
    p["g"] = tuple(g)
    cases.set_grid(p, (-0.2, -0.2, -0.2), (0.6, 0.6, 0.6))
    return p


def _state(pos, vel, rho, typ=None):
    pos = np.asarray(pos, dtype=np.float64)
    n = len(pos)
    typ = np.zeros(n, dtype=np.uint8) if typ is None else np.asarray(typ, dtype=np.uint8)
    st = cases._make_state(pos, typ, np.asarray(rho, dtype=np.float64),
                           np.asarray(vel, dtype=np.float64))
    # the oracle takes FP64 states: keep the exact FP64 values given here
    out = {k: np.asarray(v, dtype=np.float64) for k, v in st.items()
           if k not in ("type", "id")}
    out["x"], out["y"], out["z"] = pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy()
    vel = np.asarray(vel, dtype=np.float64)
    for a, k in enumerate(("vx", "vy", "vz")):
        out[k] = vel[:, a].copy()
        out[k + "p"] = vel[:, a].copy()
    out["rho"] = np.asarray(rho, dtype=np.float64).copy()
    out["rhop"] = out["rho"].copy()
    out["type"], out["id"] = st["type"], st["id"]
    return out


def _by_id(orc, p, st):
    """Interaction of a state, results indexed by particle id."""
    srt = orc.sort_state(p, st)
    acc = orc.interact(p, srt)
    ids = srt["state"]["id"][: len(acc["ax"])]
    order = np.argsort(ids)
    return {k: v[order] for k, v in acc.items()}, srt, acc


def _grad_w_fd(orc, rij, h):
    """grad_i W(|r_i - r_j|) by fourth-order central differences of W in r_i."""
    d = 1e-4 * h
    g = np.zeros(3)
    for a in range(3):
        def w(s):
            r = np.array(rij, dtype=np.float64)
            r[a] += s
            return orc.kernel_w(float(np.linalg.norm(r)), h)
        g[a] = (-w(2 * d) + 8 * w(d) - 8 * w(-d) + w(-2 * d)) / (12 * d)
    return g


def _sound_speed_fd(orc, p, rho):
    d = 1e-3
    dpdr = (orc.eos(p, rho + d)[0] - orc.eos(p, rho - d)[0]) / (2 * d)
    return math.sqrt(dpdr)


# Two fluid particles, fully 3-D separation, approaching, rho_i != rho_j != rho0.
RI = np.array([0.1, 0.2, 0.3])
SEP = np.array([0.0061, -0.0043, 0.0087])      # r_i - r_j, |SEP| = 0.01146 < 2h = 0.026
VI = np.array([0.31, -0.12, -0.44])
VJ = np.array([-0.05, 0.20, 0.10])
RHO_I, RHO_J = 1012.0, 994.0


def _pair(orc, alpha):
    p = _params(alpha=alpha)
    st = _state([RI, RI - SEP], [VI, VJ], [RHO_I, RHO_J])
    acc, _, _ = _by_id(orc, p, st)
    return p, acc


def _expected_pair_terms(orc, p):
    h, m = p["h"], p["mass"]
    r2 = float(SEP @ SEP)
    vij = VI - VJ
    vr = float(vij @ SEP)
    eta = 0.1 * h
    mu = h * vr / (r2 + eta * eta)                      # Sec. 2.2, artificial viscosity
    ci, cj = _sound_speed_fd(orc, p, RHO_I), _sound_speed_fd(orc, p, RHO_J)
    cbar, rhobar = 0.5 * (ci + cj), 0.5 * (RHO_I + RHO_J)
    Pi = -p["alpha"] * cbar * mu / rhobar if vr < 0 else 0.0
    gW = _grad_w_fd(orc, SEP, h)
    return dict(mu=mu, Pi=Pi, ci=ci, cj=cj, gW=gW, vr=vr, vij=vij, m=m, h=h)


def test_pair_setup_is_non_degenerate(orc):
    """The case exercises what the pins below claim: approaching pair inside the
    support, eta^2 << r^2, densities on both sides of rho0."""
    p = _params()
    h = p["h"]
    r = float(np.linalg.norm(SEP))
    assert 0.3 * h < r < 2 * h
    assert float((VI - VJ) @ SEP) < 0
    assert (0.1 * h) ** 2 < 0.02 * r * r
    assert RHO_J < p["rho0"] < RHO_I


def test_viscous_acceleration_two_particles(orc):
    """The part of a_i linear in alpha is -m Pi_ij grad_i W_ij with
    Pi_ij = -alpha cbar mu / rhobar, mu = h v_ij.r_ij / (r^2 + eta^2) (Sec. 2.2).
    Catches: a dropped h in mu, eta in place of eta^2, c0 in place of cbar,
    rho_i in place of rhobar, a wrong sign, a missing mass factor."""
    alpha = 0.7  # large, so the viscous part is not a rounding-level difference
    p, a1 = _pair(orc, alpha)
    _, a0 = _pair(orc, 0.0)
    e = _expected_pair_terms(orc, p)
    visc_i = np.array([a1[k][0] - a0[k][0] for k in ("ax", "ay", "az")])
    visc_j = np.array([a1[k][1] - a0[k][1] for k in ("ax", "ay", "az")])
    want_i = -e["m"] * e["Pi"] * e["gW"]
    assert e["Pi"] > 0  # approaching: a repulsive viscous pressure
    np.testing.assert_allclose(visc_i, want_i, rtol=1e-7, atol=0)
    # grad_j W_ji = -grad_i W_ij and Pi_ji = Pi_ij: equal and opposite
    np.testing.assert_allclose(visc_j, -want_i, rtol=1e-7, atol=0)
    # linear in alpha: half the coefficient gives half the viscous part
    _, ah = _pair(orc, alpha / 2)
    visc_h = np.array([ah[k][0] - a0[k][0] for k in ("ax", "ay", "az")])
    np.testing.assert_allclose(visc_h, want_i / 2, rtol=1e-7, atol=0)


def test_full_momentum_two_particles(orc):
    """a_i = -m (p_i/rho_i^2 + p_j/rho_j^2 + Pi_ij) grad_i W_ij + g at the
    workload's alpha, with gravity switched on (Sec. 2.2, symmetric form)."""
    g = (0.0, 0.0, -9.81)
    p = _params(g=g)
    st = _state([RI, RI - SEP], [VI, VJ], [RHO_I, RHO_J])
    acc, _, _ = _by_id(orc, p, st)
    e = _expected_pair_terms(orc, p)
    Pi_i = orc.eos(p, RHO_I)[0] / RHO_I ** 2
    Pj = orc.eos(p, RHO_J)[0] / RHO_J ** 2
    want = -e["m"] * (Pi_i + Pj + e["Pi"]) * e["gW"] + np.array(g)
    got = np.array([acc[k][0] for k in ("ax", "ay", "az")])
    np.testing.assert_allclose(got - np.array(g), want - np.array(g), rtol=1e-7, atol=0)


def test_continuity_rate_two_particles(orc):
    """D_i = m v_ij . grad_i W_ij (Sec. 2.2) and D_j = D_i (v_ji = -v_ij,
    grad_j W_ji = -grad_i W_ij). Catches a dropped mass, v_i in place of v_ij,
    a sign slip or a transposed component."""
    p, acc = _pair(orc, 0.01)
    e = _expected_pair_terms(orc, p)
    want = e["m"] * float(e["vij"] @ e["gW"])
    assert want > 0  # approaching particles compress
    assert acc["drho"][0] == pytest.approx(want, rel=1e-7, abs=0)
    assert acc["drho"][1] == pytest.approx(want, rel=1e-7, abs=0)
    # a rigid translation of both particles changes nothing
    st = _state([RI, RI - SEP], [VI + 0.25, VJ + 0.25], [RHO_I, RHO_J])
    moved, _, _ = _by_id(orc, _params(), st)
    assert moved["drho"][0] == pytest.approx(acc["drho"][0], rel=1e-12, abs=0)


def test_continuity_rate_three_particles_sums(orc):
    """With two neighbours the rate is the sum of both pair terms."""
    p = _params()
    h = p["h"]
    s2 = np.array([-0.0052, 0.0091, 0.0033])
    v2 = np.array([0.15, -0.33, 0.27])
    st = _state([RI, RI - SEP, RI - s2], [VI, VJ, v2], [RHO_I, RHO_J, 1003.0])
    acc, _, _ = _by_id(orc, p, st)
    m = p["mass"]
    want = (m * float((VI - VJ) @ _grad_w_fd(orc, SEP, h))
            + m * float((VI - v2) @ _grad_w_fd(orc, s2, h)))
    assert np.linalg.norm(s2) < 2 * h
    assert acc["drho"][0] == pytest.approx(want, rel=1e-7, abs=0)


def test_nu_is_max_of_mu(orc):
    """nu_i = max_j |mu_ij| (not a sum): particle 0 sees one approaching and one
    separating neighbour with different |mu|."""
    p = _params()
    h = p["h"]
    eta2 = (0.1 * h) ** 2
    s1, s2 = SEP, np.array([-0.0052, 0.0091, 0.0033])
    v1, v2 = VJ, np.array([0.9, -0.8, 0.4])
    st = _state([RI, RI - s1, RI - s2], [VI, v1, v2], [RHO_I, RHO_J, 1003.0])
    acc, _, _ = _by_id(orc, p, st)
    mu1 = h * float((VI - v1) @ s1) / (float(s1 @ s1) + eta2)
    mu2 = h * float((VI - v2) @ s2) / (float(s2 @ s2) + eta2)
    assert mu1 < 0 < mu2 and abs(mu1) != abs(mu2)
    assert acc["nu"][0] == pytest.approx(max(abs(mu1), abs(mu2)), rel=1e-13, abs=0)


def test_acoustic_time_step_two_particles(orc):
    """dt = CFL min(min_fluid sqrt(h/|a|), min h/(c_k + nu_k)) (Sec. 3.3 CFL
    condition): for this slow pair the acoustic limit of the denser particle
    decides, with c_k = c0 (rho_k/rho0)^3 from the Tait law and nu_k = |mu|."""
    p, acc = _pair(orc, 0.01)
    e = _expected_pair_terms(orc, p)
    h, nu = e["h"], abs(e["mu"])
    lim_ac = min(h / (e["ci"] + nu), h / (e["cj"] + nu))
    amag = [math.sqrt(sum(acc[k][i] ** 2 for k in ("ax", "ay", "az"))) for i in (0, 1)]
    lim_f = min(math.sqrt(h / a) for a in amag)
    assert lim_ac < lim_f  # the acoustic limit decides here
    srt = orc.sort_state(p, _state([RI, RI - SEP], [VI, VJ], [RHO_I, RHO_J]))
    dt = orc.dt(p, srt, orc.interact(p, srt))
    assert dt == pytest.approx(p["cfl"] * lim_ac, rel=1e-9, abs=0)
    # nu matters at this precision: without it the limit moves by far more
    assert abs(h / e["ci"] - h / (e["ci"] + nu)) > 1e-4 * h / e["ci"]


def test_totals_hand_sums(orc):
    """orc_totals on a four-particle state (one ghost, excluded): mass, the
    three momentum components, kinetic energy 1/2 m |v|^2, potential energy
    -m g.r, internal energy m e(rho) with e from quadrature of p/rho^2, count."""
    from scipy.integrate import quad
    p = _params(g=(0.3, -0.2, -9.81))
    pos = [[0.01, 0.02, 0.03], [0.05, 0.04, 0.02], [0.11, 0.0, 0.07], [0.2, 0.2, 0.2]]
    vel = [[0.5, -1.0, 2.0], [-0.25, 0.75, 0.0], [0.0, 0.0, -3.0], [9.0, 9.0, 9.0]]
    rho = [1010.0, 992.0, 1000.0, 1050.0]
    st = _state(pos, vel, rho, typ=[0, 1, 0, 2])
    t = orc.totals(p, st)
    m = p["mass"]
    # hand sums over particles 0, 1, 2 (particle 3 is a ghost)
    assert t[0] == pytest.approx(3 * m, rel=1e-15)
    assert t[1] == pytest.approx(m * (0.5 - 0.25 + 0.0), rel=1e-15)
    assert t[2] == pytest.approx(m * (-1.0 + 0.75 + 0.0), rel=1e-15)
    assert t[3] == pytest.approx(m * (2.0 + 0.0 - 3.0), rel=1e-15)
    ke = 0.5 * m * ((0.25 + 1.0 + 4.0) + (0.0625 + 0.5625) + 9.0)
    assert t[4] == pytest.approx(ke, rel=1e-15)
    pe = -m * sum(0.3 * x - 0.2 * y - 9.81 * z for x, y, z in pos[:3])
    assert t[5] == pytest.approx(pe, rel=1e-13)
    e = [quad(lambda r: orc.eos(p, r)[0] / (r * r), p["rho0"], rr, epsabs=0,
              epsrel=1e-13)[0] for rr in rho[:3]]
    assert t[6] == pytest.approx(m * sum(e), rel=1e-9)
    assert t[7] == 3.0


def test_support_edge_is_strict_and_three_dimensional(orc):
    """The neighbour test of Sec. 2.2 (|r_ij| < 2h, strict) at its edge, on
    separations whose FP32 arithmetic is exact: h = 1.5 s with s = 2^-7, so
    4h^2 = 9 s^2, and r_ij = (s, 2s, 2s + d) has |r_ij|^2 = 4h^2 exactly for
    d = 0. A pair at exactly 2h is no neighbour, one 2^-20 m closer is, one
    2^-20 m farther is not; every component counts (dropping dz or dy, or
    flipping the comparison, changes a count)."""
    s = 2.0 ** -7
    p = _params()
    p["h"] = 1.5 * s
    cases.set_grid(p, (-0.2, -0.2, -0.2), (0.6, 0.6, 0.6))
    ri = np.array([0.25, 0.25, 0.25])
    eps = 2.0 ** -20
    for d, want in ((0.0, 0), (-eps, 1), (eps, 0)):
        for perm in ((0, 1, 2), (2, 0, 1), (1, 2, 0)):
            sep = np.array([s, 2 * s, 2 * s + d])[list(perm)]
            st = _state([ri, ri - sep], [[0.0] * 3] * 2, [1000.0, 1000.0])
            acc, _, _ = _by_id(orc, p, st)
            assert acc["npair"].tolist() == [want, want], (d, perm)


def test_isolated_cluster_neighbour_counts(orc):
    """Clusters of k = 1..12 particles far apart: the oracle's neighbour count
    of every particle is the number of others within 2h by brute force over
    the FP64 positions, k - 1 here (a wrong cell offset, a dropped z-run or a
    counted self pair breaks it)."""
    case = cases.isolated_clusters(23)
    p, st, n = case.params, case.state, case.n
    pos = case.pos64
    d2 = ((pos[:, None, :] - pos[None, :, :]) ** 2).sum(-1)
    brute = (d2 < (2.0 * p["h"]) ** 2).sum(1) - 1
    assert np.array_equal(np.bincount(brute, minlength=12), 8 * np.arange(1, 13))
    srt = orc.sort_state(p, st)
    acc = orc.interact(p, srt)
    ids = srt["state"]["id"][:n]
    assert np.array_equal(acc["npair"].astype(np.int64), brute[ids])
