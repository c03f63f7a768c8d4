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
