"""Pins of the oracle's lattice-Boltzmann part against closed forms and invariants.

Every test checks the oracle against something other than itself: moment
identities of the D3Q19 set, the exact laminar Poiseuille solution,
the viscous decay of a shear wave, a brute-force push-streaming loop, exact
conservation laws and boundary-rebuild identities.
"""

import itertools
import math

import numpy as np
import pytest

from oracle import lattice as L
from oracle.channel import OracleChannel

RNG = np.random.default_rng(1234)


def _random_state(shape, amp=1e-2, seed=0):
    rng = np.random.default_rng(seed)
    return L.W.reshape((19,) + (1,) * len(shape)) * (1.0 + amp * rng.uniform(-1, 1, (19,) + shape))


def test_velocity_set_isotropy():
    """D3Q19 weights give the isotropic moments the equilibrium relies on."""
    C = L.C.astype(float)
    assert L.W.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia->a", L.W, C), 0.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", L.W, C, C), np.eye(3) / 3.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", L.W, C, C, C), 0.0, atol=1e-16)
    d = np.eye(3)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9.0
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", L.W, C, C, C, C), iso4, atol=1e-16)
    for i in range(19):
        assert (L.C[L.OPP[i]] == -L.C[i]).all()
    assert len({tuple(c) for c in L.C}) == 19


def test_equilibrium_moments():
    """sum f_eq = rho, sum c f_eq = rho u, sum cc f_eq = rho (c_s^2 I + u u) (eq. local_eq)."""
    rho = RNG.uniform(0.8, 1.2, size=(5, 4))
    u = RNG.uniform(-0.1, 0.1, size=(3, 5, 4))
    feq = L.equilibrium(rho, u)
    np.testing.assert_allclose(feq.sum(0), rho, rtol=1e-15)
    np.testing.assert_allclose(np.einsum("ia,i...->a...", L.C.astype(float), feq), rho * u, atol=1e-16)
    pi = L.second_moment(feq)
    expect = rho[None, None] * (np.eye(3)[:, :, None, None] / 3.0 + np.einsum("a...,b...->ab...", u, u))
    np.testing.assert_allclose(pi, expect, atol=1e-15)


def test_hermite_projection_factor():
    """The rebuilt non-equilibrium part carries exactly Pi_neq (factor w_i/(2 c_s^4)).

    With the factor printed in eq. f_i_neq (w_i/c_s^4) the second moment would
    be 2 Pi_neq; the test documents that reading.
    """
    rng = np.random.default_rng(77)   # own stream: the draws do not depend on which tests ran first
    A = rng.normal(size=(3, 3, 7))
    pi = 0.5 * (A + A.transpose(1, 0, 2)) * 1e-3
    h = L.hermite_part(pi)
    # entries of h are ~1e-4; a 19-term FP64 sum of them rounds at ~1e-19 each,
    # a wrong factor or sign would leave O(1e-4)
    np.testing.assert_allclose(h.sum(0), 0.0, atol=1e-17)
    np.testing.assert_allclose(np.einsum("ia,i...->a...", L.C.astype(float), h), 0.0, atol=1e-17)
    np.testing.assert_allclose(L.second_moment(h), pi, atol=1e-17)
    np.testing.assert_allclose(L.second_moment(2.0 * h), 2.0 * pi, atol=1e-17)
    j = rng.normal(size=(3, 7)) * 1e-3
    h1 = L.first_order_part(j)
    np.testing.assert_allclose(np.einsum("ia,i...->a...", L.C.astype(float), h1), j, atol=1e-17)
    np.testing.assert_allclose(h1.sum(0), 0.0, atol=1e-17)
    np.testing.assert_allclose(L.second_moment(h1), 0.0, atol=1e-17)


@pytest.mark.parametrize("force", [(0.0, 0.0, 0.0), (2e-5, -1e-5, 3e-6)])
def test_collision_conservation_and_stress(force):
    """Mass kept, momentum gains F, stress relaxes as BGK+Guo (eqs. lbe, bodyforce)."""
    nz, ny, nx = 3, 4, 5
    f = _random_state((nz, ny, nx), seed=3)
    tau0, cs = 0.52, 0.1
    sponge = L.sponge_factor(nx, 3, 1000.0, 3.0)
    fp, rho, u = L.collide(f, tau0, cs, force, sponge)
    Cf = L.C.astype(float)
    np.testing.assert_allclose(fp.sum(0), f.sum(0), rtol=1e-14)
    mom = np.einsum("ia,i...->a...", Cf, fp)
    mom0 = np.einsum("ia,i...->a...", Cf, f)
    np.testing.assert_allclose(mom, mom0 + np.array(force)[:, None, None, None], atol=1e-16)
    # second moment: Pi_eq + (1 - 1/tau) Pi_neq + (1 - 1/(2 tau)) (u F + F u)
    feq = L.equilibrium(rho, u)
    pi_neq = L.second_moment(f - feq)
    qh = np.sqrt(np.einsum("ab...,ab...->...", pi_neq, pi_neq))
    tau = 0.5 * (tau0 + np.sqrt(tau0 ** 2 + 18 * math.sqrt(2) * cs ** 2 * qh / rho))
    tau = 0.5 + (tau - 0.5) * sponge
    F = np.array(force)[:, None, None, None]
    uF = np.einsum("a...,b...->ab...", u, F * np.ones_like(u))
    expect = (L.second_moment(feq) + (1 - 1 / tau) * pi_neq + (1 - 0.5 / tau) * (uF + uF.transpose(1, 0, 2, 3, 4)))
    np.testing.assert_allclose(L.second_moment(fp), expect, atol=1e-16)


def test_tau_eff_closed_form():
    """tau(tau - tau0) = (9/sqrt 2) C Q^1/2 / rho, tau(0) = tau0, tau = tau0 + 3 C |S| (eqs. strain, tau_eff)."""
    tau0, cs = 0.5009, 0.1
    qh = np.array([0.0, 1e-6, 1e-4, 1e-2])
    rho = np.array([1.0, 0.97, 1.05, 1.2])
    tau = L.tau_effective(tau0, cs, qh, rho)
    assert tau[0] == tau0
    # tau - tau0 cancels for small Q, so compare at 1e-8
    np.testing.assert_allclose(tau * (tau - tau0), 9 / math.sqrt(2) * cs ** 2 * qh / rho, rtol=1e-8, atol=1e-18)
    S = L.smagorinsky_strain(tau0, cs, qh[1:], rho[1:])
    # nu_eff = nu0 + C |S| and nu = c_s^2 (tau - 1/2)
    np.testing.assert_allclose(tau[1:], tau0 + 3 * cs ** 2 * S, rtol=1e-12)


def test_shear_wave_viscous_decay():
    """u_x = U0 sin(2 pi y/L) decays as exp(-nu k^2 t), nu = c_s^2 (tau - 1/2) (eq. lbe-nu).

    The lattice decay rate approaches the viscous one at second order in k.
    """
    tau, U0 = 0.8, 1e-4
    nu = (tau - 0.5) / 3
    errs = []
    for ny in (32, 64):
        k = 2 * np.pi / ny
        T = int(round(1.0 / (nu * k * k)))
        ch = OracleChannel(1, ny, 1, nu_lb=nu, cs_smag=0.0, periodic_x=True, periodic_y=True)
        y = np.arange(ny)
        u = np.zeros((3, 1, ny, 1))
        u[0, 0, :, 0] = U0 * np.sin(2 * np.pi * y / ny)
        ch.set_f(L.equilibrium(np.ones((1, ny, 1)), u))
        ch.step(T)
        amp = 2.0 / ny * np.sum(ch.last_u[0, 0, :, 0] * np.sin(2 * np.pi * y / ny))
        errs.append(amp / U0 / math.exp(-nu * k * k * T) - 1.0)
    assert abs(errs[1]) < 1e-3
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)


@pytest.mark.parametrize("operator,tau", [("regularized", 0.875), ("bgk", 0.5 + math.sqrt(3) / 4)])
def test_poiseuille_exact_at_special_tau(operator, tau):
    """Halfway bounce-back + Guo force give the exact parabola u = F/(2 nu) eta (H - eta).

    eta = y + 1/2 is the distance from the wall at y = -1/2, H = NY.  The
    scheme is exact when Lambda = (tau+ - 1/2)(tau- - 1/2) = 3/16 (Ginzburg &
    d'Humieres): for BGK tau+ = tau- = tau; the regularized operator returns
    the odd (third-order) non-equilibrium moments to zero, i.e. tau- = 1.
    """
    ny, F = 8, 1e-6
    nu = (tau - 0.5) / 3
    ch = OracleChannel(1, ny, 1, nu_lb=nu, cs_smag=0.0, force=(F, 0, 0), periodic_x=True, operator=operator)
    ch.step(int(4 * ny * ny / nu))
    eta = np.arange(ny) + 0.5
    exact = F / (2 * nu) * eta * (ny - eta)
    np.testing.assert_allclose(ch.last_u[0, 0, :, 0], exact, rtol=1e-9)
    np.testing.assert_allclose(ch.last_u[1:], 0.0, atol=1e-14)


def test_poiseuille_second_order():
    """Away from the special tau the wall error converges at second order in NY."""
    tau, F = 0.7, 1e-7
    nu = (tau - 0.5) / 3
    errs = []
    for ny in (8, 16):
        ch = OracleChannel(1, ny, 1, nu_lb=nu, cs_smag=0.0, force=(F, 0, 0), periodic_x=True)
        ch.step(int(4 * ny * ny / nu))
        eta = np.arange(ny) + 0.5
        exact = F / (2 * nu) * eta * (ny - eta)
        errs.append(np.abs(ch.last_u[0, 0, :, 0] - exact).max() / exact.max())
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)


def _smagorinsky_poiseuille(eta, H, nu0, cs, F):
    """Steady laminar channel with the Smagorinsky viscosity, in closed form.

    The momentum balance of a forced channel (walls at eta = 0 and H) fixes the
    shear stress, nu_eff U' = F (H/2 - eta).  In simple shear |S| = sqrt(2 S:S)
    = |U'|, so with nu_eff = nu0 + C |S| (filter width = lattice spacing,
    C = Cs^2) the balance (nu0 + C U') U' = F (H/2 - eta) is a quadratic in U'
    for eta < H/2.  With g = F (H/2 - eta),
        U' = (sqrt(nu0^2 + 4 C g) - nu0) / (2 C),
    and since dg = -F d(eta), U(eta) = (G(F H/2) - G(g(eta))) / F with
        G(g) = ((nu0^2 + 4 C g)^(3/2) / (6 C) - nu0 g) / (2 C).
    The profile is symmetric about H/2.
    """
    c = cs * cs

    def G(g):
        return ((nu0 ** 2 + 4.0 * c * g) ** 1.5 / (6.0 * c) - nu0 * g) / (2.0 * c)

    e = np.minimum(eta, H - eta)
    return (G(F * H / 2.0) - G(F * (H / 2.0 - e))) / F


def test_smagorinsky_poiseuille_second_order():
    """The Smagorinsky chain (Pi_neq -> Q^1/2 -> tau_eff, eqs. tensor, strain, tau_eff)
    against the closed-form Smagorinsky-Poiseuille profile, converging at second order.

    The resolutions are related by diffusive scaling with a fixed filter width in
    physical units: tau0 fixed, F ~ NY^-3 and Cs ~ NY, so every NY solves the same
    problem (Smagorinsky viscosity about a quarter of nu0 at the walls; the profile
    differs from the Cs = 0 parabola by 15 % of its maximum).  The run starts from
    f_eq of the closed form and steps until the transient is well below the
    discretisation error.  A wrong factor anywhere in the chain (the sqrt 2, C versus
    Cs, the Frobenius norm, rho) gives another steady profile, and the error would
    then stop falling with NY.
    """
    nu0 = 0.2
    errs = []
    for ny, cs in ((16, 2.1), (32, 4.2), (64, 8.4)):
        F = 3.125e-4 * (16.0 / ny) ** 3
        ch = OracleChannel(1, ny, 1, nu_lb=nu0, cs_smag=cs, force=(F, 0.0, 0.0), periodic_x=True)
        eta = np.arange(ny) + 0.5
        exact = _smagorinsky_poiseuille(eta, ny, nu0, cs, F)
        u0 = np.zeros((3, 1, ny, 1))
        u0[0, 0, :, 0] = exact
        ch.set_f(L.equilibrium(np.ones((1, ny, 1)), u0))
        ch.step(int(0.6 * ny * ny / nu0))
        errs.append(np.abs(ch.last_u[0, 0, :, 0] - exact).max() / exact.max())
        parabola = F / (2.0 * nu0) * eta * (ny - eta)
        assert np.abs(parabola - exact).max() / exact.max() > 0.15       # the model term matters
        np.testing.assert_allclose(ch.last_u[1:], 0.0, atol=1e-14)
    assert errs[2] < 4e-4
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.03)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.03)


def test_q_half_of_simple_shear():
    """Q^1/2 = sqrt(Pi:Pi): sqrt(2) |s| for a simple shear Pi_xy = Pi_yx = s, and the
    norm of a rotated tensor is unchanged (the Frobenius norm is rotation invariant)."""
    s = np.array([3e-4, -2e-3])
    pi = np.zeros((3, 3, 2))
    pi[0, 1] = pi[1, 0] = s
    np.testing.assert_allclose(L.q_half(pi), math.sqrt(2.0) * np.abs(s), rtol=1e-15)
    # the non-equilibrium of f_eq + Hermite part carries Pi exactly, so Q^1/2 follows
    f = L.equilibrium(np.ones(2), np.zeros((3, 2))) + L.hermite_part(pi)
    pi_back = L.second_moment(f - L.equilibrium(L.density(f), L.velocity(f, L.density(f), (0, 0, 0))))
    np.testing.assert_allclose(L.q_half(pi_back), math.sqrt(2.0) * np.abs(s), rtol=1e-12)
    rng = np.random.default_rng(5)
    A = rng.normal(size=(3, 3))
    A = A + A.T
    Rm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    B = Rm @ A @ Rm.T
    assert L.q_half(A[:, :, None])[0] == pytest.approx(np.sqrt((np.linalg.eigvalsh(A) ** 2).sum()), rel=1e-13)
    assert L.q_half(B[:, :, None])[0] == pytest.approx(L.q_half(A[:, :, None])[0], rel=1e-13)


def test_stream_matches_push_bruteforce():
    """Pull streaming with halfway bounce-back equals an explicit push loop."""
    nz, ny, nx = 3, 4, 5
    fpost = RNG.uniform(0, 1, (19, nz, ny, nx))
    for periodic_x in (True, False):
        ft = L.stream(fpost, periodic_x)
        push = np.full_like(fpost, np.nan)
        for i, z, y, x in itertools.product(range(19), range(nz), range(ny), range(nx)):
            cx, cy, cz = L.C[i]
            xt, yt, zt = x + cx, y + cy, (z + cz) % nz
            if periodic_x:
                xt %= nx
            if yt < 0 or yt >= ny:          # reflected at the wall back into this node
                push[L.OPP[i], z, y, x] = fpost[i, z, y, x]
            elif 0 <= xt < nx:
                push[i, zt, yt, xt] = fpost[i, z, y, x]
        if not periodic_x:
            # reading: every c_x = +1 population at the inlet (and c_x = -1 at the
            # outlet) is rebuilt, also where the wall bounce-back supplied one
            push[L.C[:, 0] == 1, :, :, 0] = np.nan
            push[L.C[:, 0] == -1, :, :, nx - 1] = np.nan
        np.testing.assert_array_equal(np.isnan(ft), np.isnan(push))
        ok = ~np.isnan(push)
        np.testing.assert_array_equal(ft[ok], push[ok])
        if not periodic_x:
            assert np.isnan(ft[L.C[:, 0] == 1][:, :, :, 0]).all()
            assert np.isnan(ft[L.C[:, 0] == -1][:, :, :, nx - 1]).all()


def test_global_mass_conserved_with_walls():
    """Periodic x, walls in y, Smagorinsky: total mass constant to round-off."""
    nz, ny, nx = 4, 6, 5
    ch = OracleChannel(nx, ny, nz, nu_lb=1e-3, cs_smag=0.1, periodic_x=True)
    ch.set_f(_random_state((nz, ny, nx), amp=0.05, seed=5))
    m0 = ch.f.sum()
    ch.step(40)
    assert abs(ch.f.sum() - m0) / m0 < 1e-13


def _regularized_state(rho, u, pi):
    return L.equilibrium(rho, u) + L.hermite_part(pi)


def test_zou_he_density_identity():
    """(sum_{c_x=0} f + 2 sum_{c_x=-1} f) = rho (1 - u_x) for any f with moments rho, rho u."""
    f = _random_state((4, 3), amp=0.1, seed=9)
    rho = f.sum(0)
    ux = np.einsum("i,i...->...", L.C[:, 0].astype(float), f) / rho
    np.testing.assert_allclose(L.inlet_density(f, ux), rho, rtol=1e-14)


def test_inlet_rebuild_moments_and_identity():
    """After the rebuild sum f = rho_bc, sum c f = rho_bc u_bc; a regularized state is a fixed point."""
    shape = (4, 3)
    ft = _random_state(shape, amp=0.05, seed=11)
    ft[L.INLET_UNKNOWN] = np.nan
    u_bc = RNG.uniform(-0.02, 0.08, (3,) + shape)
    rho_bc = L.inlet_density(ft, u_bc[0])
    fb = L.regularized_rebuild(ft, rho_bc, u_bc, L.INLET_UNKNOWN)
    assert np.isfinite(fb).all()
    np.testing.assert_allclose(fb.sum(0), rho_bc, rtol=1e-14)
    np.testing.assert_allclose(np.einsum("ia,i...->a...", L.C.astype(float), fb), rho_bc * u_bc, atol=1e-16)
    # identity on a regularized state with the same velocity
    rho = RNG.uniform(0.95, 1.05, shape)
    A = RNG.normal(size=(3, 3) + shape) * 1e-4
    pi = 0.5 * (A + A.transpose(1, 0, 2, 3))
    fr = _regularized_state(rho, u_bc, pi)
    fr_known = fr.copy()
    fr_known[L.INLET_UNKNOWN] = np.nan
    np.testing.assert_allclose(L.inlet_density(fr_known, u_bc[0]), rho, rtol=1e-14)
    fb2 = L.regularized_rebuild(fr_known, L.inlet_density(fr_known, u_bc[0]), u_bc, L.INLET_UNKNOWN)
    np.testing.assert_allclose(fb2, fr, rtol=1e-13)


def test_outlet_rebuild():
    """Outlet: rho = rho_out, tangential velocity 0, regularized states with u = (u_x,0,0) unchanged."""
    shape = (4, 3)
    ft = _random_state(shape, amp=0.05, seed=13)
    ft[L.OUTLET_UNKNOWN] = np.nan
    rho_out = 1.0
    u = L.outlet_velocity(ft, rho_out)
    fb = L.regularized_rebuild(ft, np.full(shape, rho_out), u, L.OUTLET_UNKNOWN)
    np.testing.assert_allclose(fb.sum(0), rho_out, rtol=1e-14)
    mom = np.einsum("ia,i...->a...", L.C.astype(float), fb)
    np.testing.assert_allclose(mom[1:], 0.0, atol=1e-16)
    np.testing.assert_allclose(mom[0], u[0], atol=1e-16)
    ux = RNG.uniform(0.0, 0.06, shape)
    uu = np.zeros((3,) + shape)
    uu[0] = ux
    A = RNG.normal(size=(3, 3) + shape) * 1e-4
    fr = _regularized_state(np.full(shape, rho_out), uu, 0.5 * (A + A.transpose(1, 0, 2, 3)))
    fk = fr.copy()
    fk[L.OUTLET_UNKNOWN] = np.nan
    np.testing.assert_allclose(L.outlet_velocity(fk, rho_out)[0], ux, atol=1e-16)
    fb2 = L.regularized_rebuild(fk, np.full(shape, rho_out), L.outlet_velocity(fk, rho_out), L.OUTLET_UNKNOWN)
    np.testing.assert_allclose(fb2, fr, rtol=1e-13)


def test_sponge_factor():
    """nu_sponge = nu_eff (K s^p + 1): 1 at the sponge start, K+1 at the outlet (eq. sponge_visco)."""
    nx, Ls, K, p = 40, 8, 1000.0, 3.0
    fac = L.sponge_factor(nx, Ls, K, p)
    xs = nx - 1 - Ls
    np.testing.assert_array_equal(fac[: xs + 1], 1.0)
    assert fac[-1] == K + 1.0
    assert fac[xs + Ls // 2] == pytest.approx(1.0 + K * 0.5 ** 3)
    assert np.all(np.diff(fac) >= 0)
    np.testing.assert_array_equal(L.sponge_factor(nx, 0, K, p), 1.0)


def test_stats_bins_bruteforce():
    """Per-(x, y) sums over z of the nine velocity moments (eq. v_rms inputs)."""
    u = RNG.normal(size=(3, 3, 4, 5))
    s = L.stats_bins(u)
    assert s.shape == (5, 4, 9)
    for x in range(5):
        for y in range(4):
            a, b, c = (u[k, :, y, x] for k in range(3))
            ref = [a.sum(), b.sum(), c.sum(), (a * a).sum(), (b * b).sum(), (c * c).sum(),
                   (a * b).sum(), (a * c).sum(), (b * c).sum()]
            np.testing.assert_allclose(s[x, y], ref, rtol=1e-14)


def test_rest_is_fixed_point():
    ch = OracleChannel(4, 5, 3, nu_lb=1e-3, periodic_x=True)
    f0 = ch.f.copy()
    ch.step(3)
    np.testing.assert_allclose(ch.f, f0, rtol=1e-14)


def test_laminar_inlet_outlet_steady_mass_flux():
    """Steady laminar inflow (no fluctuations, a = 0): equal mass flux through every x-face.

    The flux through the face x + 1/2 counts the c_x = +1 populations leaving
    plane x and the c_x = -1 populations leaving plane x+1, excluding those the
    walls reflect back into their own plane.
    """
    from oracle.stg import InletGenerator  # noqa: F401  (constructed by set_rans_inlet)
    from workloads.configs import small_channel

    nx, ny, nz = 24, 8, 2
    rans = dict(small_channel(nx, ny, nz)["rans"])
    rans["R6"] = np.zeros_like(rans["R6"])
    ch = OracleChannel(nx, ny, nz, nu_lb=0.1, cs_smag=0.0, sponge_cells=0)
    c_x = 2.0 / ny
    ch.set_rans_inlet(rans, 1.0, c_x, 0.05 * c_x / rans["U_b"], 1 / 180, rans["U_b"], 20, 0.05, 0)
    ch.step(2000)

    def crossing(f, sgn):
        tot = np.zeros(nx)
        for i in range(19):
            cx, cy, _ = L.C[i]
            if cx != sgn:
                continue
            g = f[i].copy()
            if cy == 1:
                g[:, ny - 1, :] = 0.0
            elif cy == -1:
                g[:, 0, :] = 0.0
            tot += g.sum(axis=(0, 1))
        return tot

    phi = crossing(ch.f, 1)[:-1] - crossing(ch.f, -1)[1:]
    assert phi.mean() > 0
    assert np.ptp(phi) / phi.mean() < 1e-5
    # the outlet keeps its density and no tangential velocity
    np.testing.assert_allclose(ch.last_rho[:, :, -1], 1.0, rtol=1e-13)
    np.testing.assert_allclose(ch.last_u[1:, :, :, -1], 0.0, atol=1e-15)


def test_periodic_reference_start_state():
    """The periodic reference channel starts from f_eq(1, u0): its moments return
    rho = 1 and u0 exactly (equilibrium moments), u0 = (RANS U(y) + perturbation) c_t/c_x,
    and the body force is a c_t^2/c_x for a = 1 m/s^2 (eq. of the unit conversion)."""
    from workloads import periodic_channel
    from oracle import units
    cfg = periodic_channel(12, 8, 4, seed=1)
    ch = OracleChannel.periodic_from_config(cfg)
    rho = L.density(ch.f)
    u = np.einsum("ia,i...->a...", L.C.astype(np.float64), ch.f) / rho
    c_x, c_t, _, _ = units.channel_units(cfg["delta"], cfg["ny"], cfg["u_b_lb"], cfg["rans"]["U_b"], cfg["nu_phys"])
    u0 = cfg["start_velocity_phys"] * c_t / c_x
    # the perturbation is relative to the bulk velocity: U_b c_t/c_x is the lattice bulk velocity
    pert = u0.copy()
    pert[0] -= (cfg["rans"]["U3"][:, 0] * c_t / c_x)[None, :, None]
    assert np.abs(pert).max() <= 0.1 * cfg["u_b_lb"] * (1 + 1e-12)
    np.testing.assert_allclose(rho, 1.0, atol=1e-14)
    np.testing.assert_allclose(u, u0, atol=1e-15)
    assert ch.force[0] == pytest.approx(c_t ** 2 / c_x, rel=1e-15)
    assert ch.periodic_x
    m0 = ch.f.sum()
    ch.step(5)
    assert ch.f.sum() == pytest.approx(m0, rel=1e-13)
