"""The seeded inputs: RANS stand-in profiles, FV grids, configurations, job mixes."""

import math

import numpy as np
import pytest

import workloads as wl
from workloads.configs import small_channel, perturbed_state


def test_reichardt_wall_and_log_law():
    assert wl.reichardt_uplus(0.0) == 0.0
    assert wl.reichardt_duplus(0.0) == pytest.approx(1.0, abs=1e-15)
    yp = np.array([0.5, 3.0, 20.0, 150.0])
    h = 1e-6
    fd = (wl.reichardt_uplus(yp + h) - wl.reichardt_uplus(yp - h)) / (2 * h)
    np.testing.assert_allclose(wl.reichardt_duplus(yp), fd, rtol=1e-7)
    # log law: U+ - ln(y+)/kappa -> ln(kappa)/kappa + C at large y+
    big = 1e8
    assert wl.reichardt_uplus(big) - math.log(big) / wl.KAPPA == pytest.approx(
        math.log(wl.KAPPA) / wl.KAPPA + 7.8, abs=1e-6)


def test_fv_grid_matches_paper_description():
    """96 cells, first centre y+ ~ 0.6, 4 % stretching, Delta y+ ~ 8 at the centre (Numerical setup)."""
    yc, w = wl.stretched_fv_grid(96, 1.04, 1.0)
    assert len(yc) == 96 and w.sum() == pytest.approx(2.0)
    assert np.all(np.diff(yc) > 0)
    assert yc[0] * 180 == pytest.approx(0.6, abs=0.1)
    assert w[47] * 180 == pytest.approx(8.0, abs=0.5)
    np.testing.assert_allclose(w[1:48] / w[:47], 1.04, rtol=1e-12)
    np.testing.assert_allclose(yc, 2.0 - yc[::-1], atol=1e-14)


def test_profile_realizable_and_bulk_velocity():
    for re_tau, ncell in ((180.0, 96), (550.0, 160)):
        yc, w = wl.stretched_fv_grid(ncell, 1.04, 1.0)
        p = wl.channel_rans_profile(yc, re_tau)
        R11, R22, R12 = p["R6"][:, 0], p["R6"][:, 1], p["R6"][:, 3]
        assert np.all(R12 ** 2 < R11 * R22)
        assert np.all(p["k"] > 0) and np.all(p["omega"] > 0)
        # R12 antisymmetric about the centre line
        np.testing.assert_allclose(R12, -R12[::-1], rtol=1e-12)
    yc, w = wl.stretched_fv_grid(96, 1.04, 1.0)
    p = wl.channel_rans_profile(yc, 180.0)
    # the paper's k-omega RANS gives U_b = 15.37 m/s
    assert wl.bulk_velocity_fv(p["U3"][:, 0], w) == pytest.approx(15.37, rel=0.015)


def test_configs():
    for i in range(4):
        c = wl.channel_config(i)
        assert c["cells"] == c["nx"] * c["ny"] * c["nz"]
        assert c["rans"]["y"].min() > 0 and c["rans"]["y"].max() < 2.0
    assert wl.channel_config(0)["sponge_cells"] == 6
    assert wl.channel_config(1)["sponge_cells"] == 26
    assert wl.channel_config(3)["sponge_cells"] == 51
    c = small_channel(16, 8, 4)
    assert c["rans"]["y"].size == 8
    g = perturbed_state(4, 3, 2, seed=1)
    assert g.shape == (19, 2, 3, 4)
    np.testing.assert_array_equal(g, perturbed_state(4, 3, 2, seed=1))


def test_serving_jobs_seeded():
    a = wl.serving_jobs(64, seed=4)
    b = wl.serving_jobs(64, seed=4)
    assert a == b and len(a) == 64
    arr = np.array([j["arrival_s"] for j in a])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    assert np.mean(np.diff(arr)) == pytest.approx(0.5, rel=0.3)
    assert {j["store"] for j in a} <= {"f32", "f16"}
    assert all(1000 <= j["steps"] <= 20000 for j in a)


def test_periodic_channel_config():
    from workloads import periodic_channel
    a = periodic_channel(24, 16, 8, seed=3)
    b = periodic_channel(24, 16, 8, seed=3)
    assert a["periodic_x"] and a["sponge_cells"] == 0
    assert a["force_phys"] == (1.0, 0.0, 0.0)            # u_tau^2 / delta with u_tau = delta = 1
    u = a["start_velocity_phys"]
    assert u.shape == (3, 8, 16, 24)
    np.testing.assert_array_equal(u, b["start_velocity_phys"])
    U_b = a["rans"]["U_b"]
    pert = u.copy()
    pert[0] -= a["rans"]["U3"][:, 0][None, :, None]
    assert np.abs(pert).max() <= 0.1 * U_b
    assert np.abs(pert).max() > 0.09 * U_b
    assert a["rans"]["U3"].shape[0] == 16
