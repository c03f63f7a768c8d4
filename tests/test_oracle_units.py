"""Pins of the unit conversion against the paper's worked example."""

import json
import math
import os

import pytest

from oracle import units

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_units_example.json")


def _sig(x, digits):
    return float(f"{x:.{digits - 1}e}")


def test_paper_worked_example():
    ex = json.load(open(GOLDEN))
    p = ex["printed"]
    c_t = units.time_step_from_tau(ex["tau"], ex["c_x"], ex["nu_phys"])
    assert _sig(c_t, p["c_t_digits"]) == p["c_t"]
    ma = units.mach(units.velocity_to_lattice(ex["U_max"], c_t, ex["c_x"]))
    assert _sig(ma, p["mach_digits"]) == p["mach"]
    f_lb = units.acceleration_to_lattice(ex["force_phys"], c_t, ex["c_x"])
    assert _sig(f_lb, p["force_lb_digits"]) == p["force_lb"]
    # the lattice resolves L_x x L_y x L_z = 19.2 x 2 x 1.6 m at c_x = 1/90 m
    lat = ex["lattice"]
    assert (round(19.2 / ex["c_x"]), round(2.0 / ex["c_x"]), round(1.6 / ex["c_x"])) == (lat["nx"], lat["ny"], lat["nz"])
    # Re_tau = u_tau delta / nu with u_tau = 1 m/s, delta = 1 m, converted to lattice units
    nu_lb = units.nu_lattice(ex["nu_phys"], c_t, ex["c_x"])
    u_tau_lb = units.velocity_to_lattice(1.0, c_t, ex["c_x"])
    assert u_tau_lb * (1.0 / ex["c_x"]) / nu_lb == pytest.approx(lat["re_tau"], rel=1e-12)
    assert units.tau_from_nu(nu_lb) == pytest.approx(ex["tau"], rel=1e-14)


def test_channel_units_roundtrip():
    c_x, c_t, nu_lb, tau0 = units.channel_units(1.0, 32, 0.05, 15.5, 1 / 180)
    assert c_x == 1 / 16
    assert units.velocity_to_lattice(15.5, c_t, c_x) == pytest.approx(0.05, rel=1e-15)
    assert nu_lb == pytest.approx((tau0 - 0.5) / 3, rel=1e-12)
    assert units.time_step_from_tau(tau0, c_x, 1 / 180) == pytest.approx(c_t, rel=1e-10)
    assert units.CS == pytest.approx(1 / math.sqrt(3))
