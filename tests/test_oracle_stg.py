"""Pins of the oracle's synthetic turbulence generator.

Checks against published generator vectors, the geometry the paper states
for d^n and sigma^n, closed-form properties of the spectrum, exact
expectations of the mode sum over seeds and over time, the frozen-convection
form of the pseudo-position, and library routines for special cases.
"""

import math
import os

import numpy as np
import pytest
from scipy import stats as sps

from oracle import splitmix, stg
from oracle.channel import OracleChannel
from oracle import units
from workloads import channel_config, channel_rans_profile

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vectors():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "splitmix64_vectors.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 8
    for seed, idx, hexval in rows:
        seed, idx = int(seed), int(idx)
        assert splitmix.output(seed, idx) == int(hexval, 16)
        assert splitmix.stream(seed, idx)[-1] == int(hexval, 16)
    u = [splitmix.uniform(7, m) for m in range(1, 2001)]
    assert 0.0 <= min(u) and max(u) < 1.0
    assert sps.kstest(u, "uniform").pvalue > 1e-3


def test_mode_geometry():
    """|d| = |sigma| = 1, sigma . d = 0, d uniform on the sphere (eq. dn)."""
    d, sigma, phase = stg.draw_modes(11, 4000)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(np.linalg.norm(sigma, axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(np.einsum("na,na->n", d, sigma), 0.0, atol=1e-15)
    assert ((phase >= 0) & (phase < 2 * np.pi)).all()
    # uniform on the sphere: each Cartesian component is uniform on [-1, 1]
    for a in range(3):
        assert sps.kstest((d[:, a] + 1) / 2, "uniform").pvalue > 1e-3
    np.testing.assert_allclose(d.T @ d / len(d), np.eye(3) / 3, atol=0.03)
    np.testing.assert_allclose(sigma.T @ sigma / len(d), np.eye(3) / 3, atol=0.03)
    assert sps.kstest(phase / (2 * np.pi), "uniform").pvalue > 1e-3


def test_cholesky_factor():
    """a a^T = R with a lower-triangular, positive diagonal (eq. cholesky)."""
    y = np.linspace(0.01, 1.99, 41)
    R6 = channel_rans_profile(y, 395.0)["R6"]
    a, clamps = stg.cholesky_factor(R6)
    assert clamps == 0
    for j in range(len(y)):
        R11, R22, R33, R12, R13, R23 = R6[j]
        R = np.array([[R11, R12, R13], [R12, R22, R23], [R13, R23, R33]])
        np.testing.assert_allclose(a[j] @ a[j].T, R, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(a[j], np.linalg.cholesky(R), rtol=1e-12, atol=1e-15)
    # a full, non-diagonal SPD tensor
    A = np.array([[2.0, 0.3, -0.4], [0.3, 1.5, 0.2], [-0.4, 0.2, 1.1]])
    a1, _ = stg.cholesky_factor([[A[0, 0], A[1, 1], A[2, 2], A[0, 1], A[0, 2], A[1, 2]]])
    np.testing.assert_allclose(a1[0], np.linalg.cholesky(A), rtol=1e-14)
    # a non-realizable tensor is clamped and counted
    _, c = stg.cholesky_factor([[1.0, 0.1, 1.0, 0.9, 0.0, 0.0]])
    assert c == 1


def test_interpolation():
    """Identity at the RANS points, exact on linear data, zero at the walls."""
    yc = np.array([0.1, 0.4, 0.9, 1.3, 1.8])
    rans = {"y": yc, "U3": np.stack([2 + 3 * yc, -yc, 0.5 * yc], 1), "k": 1 + yc,
            "omega": 10 + yc, "R6": np.stack([yc * (c + 1) for c in range(6)], 1)}
    out = stg.interpolate_rans(rans, yc, 1.0)
    np.testing.assert_array_equal(out["U3"], rans["U3"])
    np.testing.assert_array_equal(out["omega"], rans["omega"])
    yi = np.array([0.25, 0.7, 1.55])
    out = stg.interpolate_rans(rans, yi, 1.0)
    np.testing.assert_allclose(out["U3"][:, 0], 2 + 3 * yi, rtol=1e-15)
    np.testing.assert_allclose(out["k"], 1 + yi, rtol=1e-15)
    yw = np.array([0.05, 1.9])
    out = stg.interpolate_rans(rans, yw, 1.0)
    np.testing.assert_allclose(out["U3"][:, 0], [(2 + 0.3) * 0.5, (2 + 5.4) * 0.5], rtol=1e-14)
    np.testing.assert_allclose(out["omega"], [10.1, 11.8], rtol=1e-15)


def test_length_scales_and_cutoff():
    k = np.array([1e-4, 0.5, 1.0])
    om = np.array([100.0, 5.0, 0.1])
    dw = np.array([0.01, 0.5, 1.0])
    l_t, l_e = stg.length_scales(k, om, dw, 3.0, 0.09)
    np.testing.assert_allclose(l_t, np.sqrt(k) / (0.09 * om))
    np.testing.assert_allclose(l_e, np.minimum(2 * dw, 3 * l_t))
    # eq. lcut: 2 min(max(d_x, d_y, 0.3 d_max) + 0.1 d_w, d_max)
    assert stg.cutoff_length(1.0, 2.0, 3.0, 5.0) == pytest.approx(5.0)
    assert stg.cutoff_length(1.0, 2.0, 3.0, 0.0) == pytest.approx(4.0)
    np.testing.assert_allclose(stg.cutoff_length(0.1, 0.1, 0.1, np.array([0.0, 1.0])), [0.2, 0.2])


def test_length_scales_log_layer():
    """The RANS length scale against the log law (l_t of the STG section).

    In the log layer production balances dissipation, eps = u_tau^3/(kappa y), and
    the eddy viscosity is the mixing-length one, nu_t = kappa y u_tau; the k-omega
    model's log-layer solution is k = u_tau^2/sqrt(C_mu), omega = k/nu_t (Wilcox).
    The integral length k^(3/2)/eps of that flow is kappa y C_mu^(-3/4), and l_t
    must equal it; l_e is then 2 d_w, since C_l l_t = 7.5 y exceeds 2 y there.
    """
    kappa, C_mu, u_tau = 0.41, 0.09, 0.7
    y = np.array([0.02, 0.05, 0.1, 0.2])
    k = np.full_like(y, u_tau ** 2 / math.sqrt(C_mu))
    omega = k / (kappa * y * u_tau)
    l_t, l_e = stg.length_scales(k, omega, y, 3.0, C_mu)
    eps = u_tau ** 3 / (kappa * y)
    np.testing.assert_allclose(l_t, k ** 1.5 / eps, rtol=1e-14)
    np.testing.assert_allclose(l_t, kappa * y * C_mu ** -0.75, rtol=1e-14)
    np.testing.assert_allclose(l_e, 2.0 * y, rtol=1e-15)


def test_mode_count_and_wavenumbers():
    assert stg.mode_count(100.0, 1.0, 0.01) == 464        # ceil(462.8 + 1)
    kn, a = stg.wavenumbers(2.0, 300.0, 600, 0.0)
    assert kn[0] == 2.0 and kn[-1] == pytest.approx(300.0, rel=1e-12)
    np.testing.assert_allclose(kn[1:] / kn[:-1], 1 + a, rtol=1e-13)
    kn, a = stg.wavenumbers(2.0, 300.0, 50, 0.05)
    assert a == 0.05 and kn[-1] == pytest.approx(2.0 * 1.05 ** 49)


def test_von_karman_shape():
    """Peak at k = k_e, k^4 at low k, k^(-5/3) inertial range, both damping factors."""
    ke = 3.0
    inf = 1e300
    E = lambda k: stg.von_karman_modified(k, ke, inf, inf)
    # d ln E/d ln k = 4 - (17/3) 2.4 r^2/(1 + 2.4 r^2) vanishes at r = 1
    assert E(ke) > E(ke * (1 + 1e-4)) and E(ke) > E(ke * (1 - 1e-4))
    slope = lambda k1, k2: math.log(E(k2) / E(k1)) / math.log(k2 / k1)
    assert slope(1e-4 * ke, 2e-4 * ke) == pytest.approx(4.0, abs=1e-6)
    assert slope(1e5 * ke, 2e5 * ke) == pytest.approx(-5.0 / 3.0, abs=1e-6)
    r = 1e6
    assert E(r * ke) == pytest.approx(2.4 ** (-17 / 6) * r ** (-5 / 3), rel=1e-5)
    # Kolmogorov and grid cut-off factors
    k_eta, k_cut = 1200.0, 50.0
    f = lambda k: stg.von_karman_modified(k, ke, k_eta, k_cut) / stg.von_karman_modified(k, ke, inf, inf)
    assert f(k_eta / 12) * 1.0 == pytest.approx(math.exp(-1.0) * math.exp(-((4 * (k_eta / 12 - 45) / 50) ** 3)), rel=1e-12)
    assert f(0.9 * k_cut) == pytest.approx(math.exp(-(12 * 45 / 1200) ** 2), rel=1e-12)
    assert f(1.15 * k_cut) == pytest.approx(math.exp(-1.0) * math.exp(-(12 * 57.5 / 1200) ** 2), rel=1e-12)


def test_spectrum_weights():
    """sum_n q^n = 1 and q^n / q^m = E(k^n) k^n / (E(k^m) k^m) (eq. qn)."""
    kn, a = stg.wavenumbers(1.5, 200.0, 80, 0.0)
    l_e = np.array([0.1, 0.5, 2.0])
    k = np.array([0.5, 2.0, 1.0])
    om = np.array([500.0, 50.0, 5.0])
    kc = np.full(3, 150.0)
    q = stg.spectrum_weights(kn, a, l_e, k, om, 1 / 180, kc)
    np.testing.assert_allclose(q.sum(1), 1.0, rtol=1e-14)
    eps = 0.09 * k * om
    k_eta = 2 * np.pi / (1 / 180 ** 3 / eps) ** 0.25
    for j in range(3):
        E = stg.von_karman_modified(kn, 2 * np.pi / l_e[j], k_eta[j], 150.0)
        np.testing.assert_allclose(q[j] / q[j, 0], E * kn / (E[0] * kn[0]), rtol=1e-12)


def _fixed_geometry():
    kn, _ = stg.wavenumbers(1.6, 75.0, 50, 0.05)
    q = np.linspace(1.0, 3.0, 50) * np.exp(-np.arange(50) / 20)
    q /= q.sum()
    return kn, np.sqrt(q)[None, :], q


def test_stg_ensemble_moments():
    """Over seeds, E[v'] = 0 and E[v' v'^T] = I; hence E[u' u'^T] = a a^T = R.

    6 sum_n q^n E[sigma sigma^T] E[cos^2] = 6 * 1 * I/3 * 1/2 = I.
    """
    kn, sq, _ = _fixed_geometry()
    S = 3000
    v = np.zeros((S, 3))
    y, z = np.array([0.3]), np.array([0.7])
    for s in range(S):
        d, sigma, ph = stg.draw_modes(10_000 + s, 50)
        v[s] = stg.auxiliary_field(0.37, 0.0, y, z, kn, d, sigma, ph, sq, 1.9, 15.5)[0, 0]
    se = math.sqrt(2.0 / S)
    np.testing.assert_allclose(v.mean(0), 0.0, atol=5 * math.sqrt(1.0 / S))
    np.testing.assert_allclose(v.T @ v / S, np.eye(3), atol=5 * se)
    R6 = channel_rans_profile(np.array([0.3]), 180.0)["R6"]
    a, _ = stg.cholesky_factor(R6)
    u = v @ a[0].T
    R = np.array([[R6[0, 0], R6[0, 3], 0], [R6[0, 3], R6[0, 1], 0], [0, 0, R6[0, 2]]])
    np.testing.assert_allclose(u.T @ u / S, R, atol=5 * se * R6[0, 0])


def test_stg_time_average_of_one_draw():
    """For one draw the long-time covariance at a point tends to 3 sum_n q^n sigma^n sigma^n^T.

    Each mode oscillates at its own frequency 2 pi d_x^n U_b / L_e (eq. psu),
    so cross terms average out and cos^2 averages to 1/2.
    """
    kn, sq, q = _fixed_geometry()
    d, sigma, ph = stg.draw_modes(5, 50)
    L_e, U_b = 1.9, 15.5
    rng = np.random.default_rng(0)
    ts = rng.uniform(0.0, 1e7 * L_e / U_b, 20000)
    y, z = np.array([0.8]), np.array([0.2])
    v = np.array([stg.auxiliary_field(t, 0.0, y, z, kn, d, sigma, ph, sq, L_e, U_b)[0, 0] for t in ts])
    expect = 3.0 * np.einsum("n,na,nb->ab", q, sigma, sigma)
    np.testing.assert_allclose(v.T @ v / len(ts), expect, atol=0.04)
    np.testing.assert_allclose(v.mean(0), 0.0, atol=0.04)


def test_pseudo_position_is_frozen_convection():
    """v'(x, t) depends on x - U_b t only (eq. psu): the inlet pattern convects at U_b."""
    kn, sq, _ = _fixed_geometry()
    d, sigma, ph = stg.draw_modes(3, 50)
    y = np.linspace(0.05, 1.95, 7)
    z = np.linspace(0.0, 1.5, 5)
    L_e, U_b, dt = 1.9, 15.5, 0.0123
    v0 = stg.auxiliary_field(0.0, 0.0, y, z, kn, d, sigma, ph, np.repeat(sq, 7, 0), L_e, U_b)
    v1 = stg.auxiliary_field(dt, U_b * dt, y, z, kn, d, sigma, ph, np.repeat(sq, 7, 0), L_e, U_b)
    np.testing.assert_allclose(v1, v0, atol=1e-12)
    v2 = stg.auxiliary_field(dt, 0.0, y, z, kn, d, sigma, ph, np.repeat(sq, 7, 0), L_e, U_b)
    assert np.abs(v2 - v0).max() > 1e-3


@pytest.mark.parametrize("cfg_index", [0, 1])
def test_inlet_plane_guard_and_units(cfg_index):
    """|u_bc . n| < 0.3 c_s (eq. density_bc); the plane mean is the converted RANS mean."""
    cfg = channel_config(cfg_index)
    ch = OracleChannel.from_config(cfg)
    gen = ch.inlet
    for t in (1, 777, 20_000):
        pl = gen.plane(t)
        assert pl.shape == (cfg["ny"], cfg["nz"], 3)
        assert np.abs(pl[:, :, 0]).max() < 0.3 * units.CS
    # mean over many spanwise nodes and times approaches U_int c_t / c_x
    mean = np.mean([gen.plane(t)[:, :, 0].mean() for t in range(1, 4000, 400)])
    expect = gen.U_int[:, 0].mean() * gen.c_t / gen.c_x
    assert mean == pytest.approx(expect, rel=0.05)
    assert expect == pytest.approx(cfg["u_b_lb"], rel=0.02 if cfg_index == 0 else 0.05)


def _seed_fields(S, positions, seed0):
    """v' of the fixed-geometry generator for S seeds, evaluated by `positions(seed index, draw)`."""
    kn, sq, q = _fixed_geometry()
    out = []
    for s in range(S):
        d, sigma, ph = stg.draw_modes(seed0 + s, kn.size)
        out.append(positions(kn, sq, d, sigma, ph))
    return kn, q, np.array(out)


def _within(est, se, expect, k=5.0):
    return np.all(np.abs(est - expect) <= k * se)


def test_stg_spanwise_two_point_correlation():
    """Ensemble spanwise correlation of v' (eqs. aux_vec, psu) against its closed form.

    With phases uniform and independent, E[cos(A + phi) cos(B + phi)] = cos(A - B)/2
    and the modes decorrelate, so for a spanwise separation r
        tr E[v'(z) v'(z + r)] = 3 sum_n q^n E[cos(k^n d_z r)] = 3 sum_n q^n sin(k^n r)/(k^n r),
    since d_z is uniform on [-1, 1] for directions uniform on the sphere.  For the
    spanwise component, E[sigma_z^2 | d] = (1 - d_z^2)/2 (sigma uniform on the circle
    normal to d), giving E[w'(z) w'(z + r)] = 3 sum_n q^n (sin b - b cos b)/b^3, b = k^n r.
    A wavenumber scaled by 2 pi (or its inverse) in the spatial part of the phase, or
    sigma not normal to d, moves these curves by many standard errors (checked below).
    """
    r = np.array([0.0, 0.05, 0.1, 0.2, 0.35, 0.6, 1.0])
    z0 = np.linspace(0.0, 70.0, 8)          # base points far apart (several correlation lengths)
    z = (z0[:, None] + r[None, :]).ravel()
    y = np.array([0.45])
    L_e, U_b, t = 1.9, 15.5, 0.21

    def field(kn, sq, d, sigma, ph):
        v = stg.auxiliary_field(t, 0.0, y, z, kn, d, sigma, ph, sq, L_e, U_b)[0].reshape(len(z0), len(r), 3)
        tr = np.einsum("pa,pra->pr", v[:, 0, :], v).mean(0)
        ww = (v[:, 0, 2][:, None] * v[:, :, 2]).mean(0)
        return np.concatenate([tr, ww])

    S = 1500
    kn, q, X = _seed_fields(S, field, 50_000)
    est, se = X.mean(0), X.std(0, ddof=1) / math.sqrt(S)
    b = np.outer(r, kn)
    with np.errstate(invalid="ignore", divide="ignore"):
        sinc = np.where(b > 0, np.sin(b) / b, 1.0)
        g = np.where(b > 0, (np.sin(b) - b * np.cos(b)) / b ** 3, 1.0 / 3.0)
    tr_expect = 3.0 * sinc @ q
    ww_expect = 3.0 * g @ q
    n = len(r)
    assert tr_expect[0] == pytest.approx(3.0) and ww_expect[0] == pytest.approx(1.0)
    assert _within(est[:n], se[:n], tr_expect), (est[:n], tr_expect, se[:n])
    assert _within(est[n:], se[n:], ww_expect), (est[n:], ww_expect, se[n:])
    # the test separates plausible mistakes in the wavenumber scaling
    for wrong in (2.0 * np.pi, 1.0 / (2.0 * np.pi)):
        bw = b * wrong
        with np.errstate(invalid="ignore", divide="ignore"):
            alt = 3.0 * np.where(bw > 0, np.sin(bw) / bw, 1.0) @ q
        assert not _within(est[:n], se[:n], alt)
    # ... and sigma taken along d instead of normal to it: E[w'w'] -> 3 sum q E[d_z^2 cos]
    with np.errstate(invalid="ignore", divide="ignore"):
        alt_ww = 3.0 * np.where(b > 0, sinc - 2.0 * g, 1.0 / 3.0) @ q
    assert not _within(est[n:], se[n:], alt_ww)


def test_stg_temporal_two_point_correlation():
    """Ensemble correlation of v' at one point over a time lag s (eq. psu).

    The pseudo-position scales the streamwise phase so that every mode advances by
    2 pi d_x U_b s / max(l_e) over a lag s, whatever its wavenumber; with d_x uniform
    on [-1, 1] and sum_n q^n = 1 this gives tr E[v'(t) v'(t + s)] = 3 sin(a)/a with
    a = 2 pi U_b s / max(l_e).  A pseudo-position without the 2 pi/(k^n max l_e)
    factor would give 3 sum_n q^n sin(k^n U_b s)/(k^n U_b s) instead (checked below).
    """
    L_e, U_b = 1.9, 15.5
    a = np.array([0.0, 0.4, 1.0, 2.0, 3.2, 4.5, 6.0])
    s_lag = a * L_e / (2.0 * np.pi * U_b)
    t0 = 3.7
    y, z = np.array([0.8]), np.linspace(0.35, 70.35, 6)     # base points far apart in z

    def field(kn, sq, d, sigma, ph):
        v = [stg.auxiliary_field(t0 + s, 0.0, y, z, kn, d, sigma, ph, sq, L_e, U_b)[0] for s in s_lag]
        return np.array([np.einsum("pa,pa->p", v[0], vs).mean() for vs in v])

    S = 1200
    kn, q, X = _seed_fields(S, field, 90_000)
    est, se = X.mean(0), X.std(0, ddof=1) / math.sqrt(S)
    with np.errstate(invalid="ignore", divide="ignore"):
        expect = 3.0 * np.where(a > 0, np.sin(a) / a, 1.0)
    assert _within(est, se, expect), (est, expect, se)
    bw = np.outer(s_lag * U_b, kn)
    with np.errstate(invalid="ignore", divide="ignore"):
        alt = 3.0 * np.where(bw > 0, np.sin(bw) / bw, 1.0) @ q
    assert not _within(est, se, alt)
