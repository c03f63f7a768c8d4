"""Oracle pins for the velocity-set and collision variants (D3Q15, D3Q19,
D3Q27; regularized or plain BGK bulk): lattice isotropy, equilibrium moments,
conservation, the exact Poiseuille solution, pull = push streaming, and the
boundary rebuilds."""

import itertools
import math

import numpy as np
import pytest

from oracle import lattice as L
from oracle.channel import OracleChannel

SETS = (15, 19, 27)


@pytest.mark.parametrize("q", SETS)
def test_isotropy_to_fourth_order(q):
    vs = L.velocity_set(q)
    C = vs.C.astype(float)
    assert vs.Q == q and len({tuple(c) for c in vs.C}) == q
    assert vs.W.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia->a", vs.W, C), 0.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", vs.W, C, C), np.eye(3) / 3.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", vs.W, C, C, C), 0.0, atol=1e-16)
    d = np.eye(3)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", vs.W, C, C, C, C), iso4, atol=1e-16)
    for i in range(q):
        assert (vs.C[vs.OPP[i]] == -vs.C[i]).all()
    # D3Q27 contains D3Q19 in the same order; D3Q15 = axes + corners
    if q == 27:
        np.testing.assert_array_equal(vs.C[:19], L.D3Q19.C)
    if q == 15:
        assert all(abs(c).sum() in (0, 1, 3) for c in vs.C)


@pytest.mark.parametrize("q", SETS)
def test_equilibrium_moments(q):
    rng = np.random.default_rng(q)
    rho = 1.0 + 0.1 * rng.uniform(-1, 1, (3, 4))
    u = 0.1 * rng.uniform(-1, 1, (3, 3, 4))
    feq = L.equilibrium(rho, u, q)
    C = L.velocity_set(q).C.astype(float)
    np.testing.assert_allclose(feq.sum(axis=0), rho, rtol=1e-14)
    np.testing.assert_allclose(np.einsum("ia,i...->a...", C, feq), rho * u, atol=1e-15)
    pi = np.einsum("ia,ib,i...->ab...", C, C, feq)
    ref = rho * (np.eye(3)[:, :, None, None] / 3.0 + np.einsum("a...,b...->ab...", u, u))
    np.testing.assert_allclose(pi, ref, atol=1e-15)


@pytest.mark.parametrize("q,operator", itertools.product(SETS, ("regularized", "bgk")))
def test_collision_conservation(q, operator):
    vs = L.velocity_set(q)
    rng = np.random.default_rng(3)
    shape = (2, 3, 4)
    f = vs.W.reshape((q, 1, 1, 1)) * (1.0 + 0.05 * rng.uniform(-1, 1, (q,) + shape))
    force = (2e-5, -1e-5, 3e-6)
    fp, rho, u = L.collide(f, 0.6, 0.1, force, np.ones(shape[-1]), operator)
    C = vs.C.astype(float)
    np.testing.assert_allclose(fp.sum(axis=0), f.sum(axis=0), rtol=1e-14)
    np.testing.assert_allclose(np.einsum("ia,i...->a...", C, fp),
                               np.einsum("ia,i...->a...", C, f) + np.array(force)[:, None, None, None], atol=1e-15)


@pytest.mark.parametrize("q,operator,tau", [(q, "regularized", 0.875) for q in SETS] +
                         [(q, "bgk", 0.5 + math.sqrt(3) / 4) for q in SETS])
def test_poiseuille_exact_at_special_tau(q, operator, tau):
    """Halfway bounce-back + Guo force: exact parabola at Lambda = 3/16 for every set."""
    ny, F = 8, 1e-6
    nu = (tau - 0.5) / 3
    ch = OracleChannel(1, ny, 1, nu_lb=nu, cs_smag=0.0, force=(F, 0, 0), periodic_x=True, operator=operator,
                       velocity_set=q)
    ch.step(int(4 * ny * ny / nu))
    eta = np.arange(ny) + 0.5
    exact = F / (2 * nu) * eta * (ny - eta)
    np.testing.assert_allclose(ch.last_u[0, 0, :, 0], exact, rtol=1e-9)
    np.testing.assert_allclose(ch.last_u[1:], 0.0, atol=1e-14)


@pytest.mark.parametrize("q", (15, 27))
def test_stream_matches_push_bruteforce(q):
    vs = L.velocity_set(q)
    rng = np.random.default_rng(4)
    nz, ny, nx = 3, 4, 5
    fpost = rng.uniform(0.0, 1.0, (q, nz, ny, nx))
    push = np.full_like(fpost, np.nan)
    for i, z, y, x in itertools.product(range(q), range(nz), range(ny), range(nx)):
        cx, cy, cz = vs.C[i]
        yd = y + cy
        if yd < 0 or yd >= ny:
            push[vs.OPP[i], z, y, x] = fpost[i, z, y, x]
        else:
            push[i, (z + cz) % nz, yd, (x + cx) % nx] = fpost[i, z, y, x]
    np.testing.assert_array_equal(L.stream(fpost, periodic_x=True), push)


@pytest.mark.parametrize("q", (15, 27))
def test_boundary_rebuilds_reproduce_moments(q):
    vs = L.velocity_set(q)
    rng = np.random.default_rng(6)
    shape = (3, 2)
    f = vs.W.reshape((q, 1, 1)) * (1.0 + 0.02 * rng.uniform(-1, 1, (q,) + shape))
    u_bc = np.stack([0.04 + 0.01 * rng.uniform(-1, 1, shape), 0.01 * rng.uniform(-1, 1, shape),
                     0.01 * rng.uniform(-1, 1, shape)])
    ft = f.copy()
    ft[vs.INLET_UNKNOWN] = np.nan
    rho_bc = L.inlet_density(ft, u_bc[0])
    fb = L.regularized_rebuild(ft, rho_bc, u_bc, vs.INLET_UNKNOWN)
    C = vs.C.astype(float)
    np.testing.assert_allclose(fb.sum(axis=0), rho_bc, rtol=1e-14)
    np.testing.assert_allclose(np.einsum("ia,i...->a...", C, fb), rho_bc * u_bc, atol=1e-15)
    ft = f.copy()
    ft[vs.OUTLET_UNKNOWN] = np.nan
    u = L.outlet_velocity(ft, 1.0)
    fb = L.regularized_rebuild(ft, np.ones(shape), u, vs.OUTLET_UNKNOWN)
    np.testing.assert_allclose(fb.sum(axis=0), 1.0, rtol=1e-14)
    np.testing.assert_allclose(np.einsum("ia,i...->a...", C, fb), u, atol=1e-15)


@pytest.mark.parametrize("q", (15, 27))
def test_channel_runs_and_conserves_mass_with_walls(q):
    """Periodic box with walls: mass is constant over steps for the variant sets."""
    ch = OracleChannel(6, 5, 4, nu_lb=0.02, cs_smag=0.1, periodic_x=True, velocity_set=q)
    rng = np.random.default_rng(9)
    ch.set_f(ch.f * (1.0 + 0.01 * rng.uniform(-1, 1, ch.f.shape)))
    m0 = ch.f.sum()
    ch.step(20)
    assert ch.f.sum() == pytest.approx(m0, rel=1e-13)
    assert ch.f.shape[0] == q
