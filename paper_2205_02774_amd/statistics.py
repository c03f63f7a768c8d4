"""Flow profiles from the FP64 statistics sums returned by `Lattice.get_stats`.

The sums are per (x, y) bin over z and the sampled steps: u, v, w, uu, vv,
ww, uv, uw, vw (in that order).  Dividing by n_samples * NZ gives the means;
the Reynolds stresses are <u_a u_b> - U_a U_b per bin, then averaged over an x
range.
"""

import numpy as np


def profiles(stats, n_samples, nz, x0, x1, u_tau=1.0):
    """Mean U, u_rms, v_rms, w_rms and uv over x0 <= x < x1, as functions of y (in units of u_tau)."""
    s = np.asarray(stats)[x0:x1] / (n_samples * nz)
    U, V, W = s[..., 0], s[..., 1], s[..., 2]
    out = {
        "U": U / u_tau,
        "urms": np.sqrt(np.maximum(s[..., 3] - U * U, 0.0)) / u_tau,
        "vrms": np.sqrt(np.maximum(s[..., 4] - V * V, 0.0)) / u_tau,
        "wrms": np.sqrt(np.maximum(s[..., 5] - W * W, 0.0)) / u_tau,
        "uv": (s[..., 6] - U * V) / u_tau ** 2,
    }
    return {k: v.mean(axis=0) for k, v in out.items()}


def profile_errors(p, ref):
    """Largest deviation over y of each profile, relative to the reference profile's largest magnitude."""
    return {k: float(np.abs(p[k] - ref[k]).max() / np.abs(ref[k]).max()) for k in ref}


def friction_velocity(stats, n_samples, nz, nu_lb):
    """u_tau(x) in lattice units from the mean streamwise velocity at the first
    row next to each wall (eq. u_shear: u_tau = sqrt(nu dU/dy), first-order
    gradient).  The first rows sit half a cell from the halfway bounce-back
    walls, so dU/dy = U / (1/2) there; both walls are averaged."""
    U = np.asarray(stats)[..., 0] / (n_samples * nz)           # (NX, NY)
    grad = 0.5 * (U[:, 0] + U[:, -1]) / 0.5
    return np.sqrt(nu_lb * np.maximum(grad, 0.0))


def adaptation_length(ratio, x_over_delta, band=0.03, x_stop=None):
    """Smallest x/delta from which u_tau / u_theory stays within 1 +- band up to x_stop
    (the start of the sponge, if given); None if it never settles."""
    r = np.asarray(ratio)
    x = np.asarray(x_over_delta)
    keep = np.ones_like(x, dtype=bool) if x_stop is None else x < x_stop
    ok = (np.abs(r - 1.0) <= band) | ~keep
    bad = np.nonzero(~ok)[0]
    if len(bad) == 0:
        return float(x[0])
    last_bad = bad[-1]
    if last_bad + 1 >= len(x) or not keep[last_bad + 1]:
        return None
    return float(x[last_bad + 1])


def autocorrelation(series):
    """Normalised temporal autocorrelation B_uu(k) = <u'(t) u'(t + k)> / <u'^2> of a
    sampled signal (biased estimator: sums over the overlap divided by the full length)."""
    u = np.asarray(series, dtype=np.float64)
    up = u - u.mean()
    n = len(up)
    spec = np.fft.rfft(up, 2 * n)
    acf = np.fft.irfft(spec * np.conj(spec))[:n] / n
    return acf / acf[0]


def integral_time(B, dt):
    """Integral time scale T_t = integral of B_uu from 0 to its first zero (eq. time-integral),
    trapezoidal rule on the samples, the last interval cut at the linearly interpolated zero."""
    B = np.asarray(B, dtype=np.float64)
    neg = np.nonzero(B <= 0.0)[0]
    if len(neg) == 0:
        return float(np.trapezoid(B, dx=dt))
    k = neg[0]
    total = float(np.trapezoid(B[:k], dx=dt)) if k > 1 else 0.0
    frac = B[k - 1] / (B[k - 1] - B[k])                           # zero between samples k-1 and k
    return total + 0.5 * B[k - 1] * frac * dt


def window_means(series, window):
    """Means of consecutive windows of `window` samples (ensemble means per window, e.g. 1T windows)."""
    u = np.asarray(series, dtype=np.float64)
    m = len(u) // window
    return u[: m * window].reshape(m, window, *u.shape[1:]).mean(axis=1)
