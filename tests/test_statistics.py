"""Post-processing of the FP64 statistics and probe series (CPU): profiles,
friction velocity (eq. u_shear), adaptation length, autocorrelation B_uu and
the integral time scale (eq. time-integral), against closed forms and brute
force."""

import numpy as np
import pytest

from paper_2205_02774_amd import statistics as S


def _sums(u, v, w):
    """Statistics sums of velocity samples of shape (T, NZ, NY, NX) -> (NX, NY, 9)."""
    q = [u, v, w, u * u, v * v, w * w, u * v, u * w, v * w]
    return np.stack([a.sum(axis=(0, 1)).T for a in q], axis=-1)


def test_profiles_recover_means_and_stresses():
    rng = np.random.default_rng(0)
    T, nz, ny, nx = 400, 6, 5, 4
    U = np.linspace(0.1, 0.5, ny)
    u = U[None, None, :, None] + 0.02 * rng.standard_normal((T, nz, ny, nx))
    v = 0.01 * rng.standard_normal((T, nz, ny, nx)) - 0.3 * (u - U[None, None, :, None])
    w = 0.015 * rng.standard_normal((T, nz, ny, nx))
    st = _sums(u, v, w)
    P = S.profiles(st, T, nz, 1, 3)
    sel = (slice(None), slice(None), slice(None), slice(1, 3))
    for key, a, b in (("urms", u, u), ("vrms", v, v), ("wrms", w, w), ("uv", u, v)):
        ref = []
        for x in (1, 2):
            aa, bb = a[..., x], b[..., x]
            cov = (aa * bb).mean(axis=(0, 1)) - aa.mean(axis=(0, 1)) * bb.mean(axis=(0, 1))
            ref.append(np.sqrt(cov) if key != "uv" else cov)
        np.testing.assert_allclose(P[key], np.mean(ref, axis=0), rtol=1e-10, atol=1e-15)
    np.testing.assert_allclose(P["U"], u[sel].mean(axis=(0, 1, 3)), rtol=1e-12)
    assert S.profile_errors(P, P) == {k: 0.0 for k in P}


def test_friction_velocity_linear_wall_layer():
    """U = G eta near both walls (eta = distance from the halfway wall) gives u_tau = sqrt(nu G)."""
    nx, ny, nz, n, nu, G = 7, 10, 3, 5, 2e-3, 0.04
    eta = np.minimum(np.arange(ny) + 0.5, ny - 0.5 - np.arange(ny))
    st = np.zeros((nx, ny, 9))
    st[..., 0] = (G * eta)[None, :] * n * nz
    np.testing.assert_allclose(S.friction_velocity(st, n, nz, nu), np.sqrt(nu * G), rtol=1e-14)


def test_adaptation_length():
    x = np.linspace(0.0, 10.0, 101)
    r = 1.0 + 0.2 * np.exp(-3.0 * x)                 # decays into the +-3 % band at x = ln(0.2/0.03)/3
    L = S.adaptation_length(r, x)
    assert L == pytest.approx(np.ceil(10 * np.log(0.2 / 0.03) / 3) / 10, abs=1e-12)
    # a dip after the sponge start does not count; one inside the range does
    r2 = r.copy()
    r2[x > 9] = 0.5
    assert S.adaptation_length(r2, x, x_stop=9.0) == L
    assert S.adaptation_length(r2, x) is None


def test_autocorrelation_matches_direct_sum():
    rng = np.random.default_rng(2)
    u = np.cumsum(rng.standard_normal(300)) * 0.1 + rng.standard_normal(300)
    B = S.autocorrelation(u)
    up = u - u.mean()
    direct = np.array([np.dot(up[: len(up) - k], up[k:]) for k in range(len(up))]) / np.dot(up, up)
    np.testing.assert_allclose(B, direct, atol=1e-12)
    assert B[0] == pytest.approx(1.0)


def test_integral_time_closed_forms():
    # B = cos(omega t): first zero at pi / (2 omega), integral 1 / omega
    omega, dt = 0.37, 1e-3
    t = np.arange(0, 20.0, dt)
    assert S.integral_time(np.cos(omega * t), dt) == pytest.approx(1.0 / omega, rel=1e-6)
    # no zero crossing: the whole record, T (1 - exp(-L / T))
    T = 2.5
    B = np.exp(-t / T)
    assert S.integral_time(B, dt) == pytest.approx(T * (1.0 - np.exp(-t[-1] / T)), rel=1e-6)
    # exponentially correlated process (AR(1), phi = exp(-dt / T)): estimate near T
    rng = np.random.default_rng(5)
    dt, T, n = 0.05, 1.0, 400_000
    phi = np.exp(-dt / T)
    e = rng.standard_normal(n) * np.sqrt(1 - phi * phi)
    x = np.empty(n)
    x[0] = 0.0
    for k in range(1, n):
        x[k] = phi * x[k - 1] + e[k]
    assert S.integral_time(S.autocorrelation(x), dt) == pytest.approx(T, rel=0.15)


def test_window_means():
    u = np.arange(10.0)
    np.testing.assert_allclose(S.window_means(u, 3), [1.0, 4.0, 7.0])
