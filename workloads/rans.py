"""Synthetic RANS channel profiles (stand-in for the paper's k-omega FV solution).

The paper obtains U, k, omega and the Reynolds stresses R from a Wilcox
k-omega finite-volume channel computation (Numerical setup section: 96 cells
in y, first centre at y+ = 0.6, 4 % stretching) and that output is not
available.  These closed forms reproduce the *shape* of such a solution so the
method has realistic inputs; they are inputs, not part of the method:

* mean velocity: Reichardt's law of the wall,
      U+ = ln(1 + kappa y+)/kappa + C (1 - exp(-y+/chi) - (y+/chi) exp(-y+/3)),
  kappa = 0.41, C = 7.8, chi = 11;
* turbulent kinetic energy, a wall-damped form with k+ ~ y+^2 at the wall:
      k+ = 0.13 y+^2 exp(-y+/7.5) + 0.8 (1 - exp(-(y+/10)^2));
* specific dissipation blending Wilcox's viscous-sublayer value
  6 nu/(beta_1 y^2) (beta_1 = 0.075) and the log-layer value
  u_tau/(sqrt(beta*) kappa y) (beta* = 0.09):
      omega+ = sqrt((6/(0.075 y+^2))^2 + (1/(0.3 kappa y+))^2);
* Reynolds stresses from the Boussinesq hypothesis with nu_t = k/omega:
      R11 = R22 = R33 = 2k/3,  R12 = -nu_t dU/dy,  R13 = R23 = 0.

Physical units follow the paper's channel: half-height delta = 1 m, friction
velocity u_tau = 1 m/s, nu = u_tau delta / Re_tau.
"""

import numpy as np

KAPPA = 0.41
REICHARDT_C = 7.8
REICHARDT_CHI = 11.0


def reichardt_uplus(yp):
    yp = np.asarray(yp, dtype=np.float64)
    chi = REICHARDT_CHI
    return (np.log1p(KAPPA * yp) / KAPPA
            + REICHARDT_C * (1.0 - np.exp(-yp / chi) - (yp / chi) * np.exp(-yp / 3.0)))


def reichardt_duplus(yp):
    """dU+/dy+ of Reichardt's law (analytic)."""
    yp = np.asarray(yp, dtype=np.float64)
    chi = REICHARDT_CHI
    return (1.0 / (1.0 + KAPPA * yp)
            + REICHARDT_C * (np.exp(-yp / chi) / chi
                             - np.exp(-yp / 3.0) / chi
                             + (yp / (3.0 * chi)) * np.exp(-yp / 3.0)))


def k_plus(yp):
    yp = np.asarray(yp, dtype=np.float64)
    return 0.13 * yp ** 2 * np.exp(-yp / 7.5) + 0.8 * (1.0 - np.exp(-(yp / 10.0) ** 2))


def omega_plus(yp):
    yp = np.asarray(yp, dtype=np.float64)
    return np.sqrt((6.0 / (0.075 * yp ** 2)) ** 2 + (1.0 / (0.3 * KAPPA * yp)) ** 2)


def stretched_fv_grid(n_cells, ratio, delta=1.0):
    """Cell centres and widths of a wall-clustered finite-volume y-grid.

    n_cells/2 cells per half channel, widths growing geometrically by
    `ratio` from each wall, the first width chosen so each half spans delta.
    Returns (centres, widths), centres ascending in (0, 2 delta).
    """
    if n_cells % 2:
        raise ValueError("n_cells must be even")
    half = n_cells // 2
    h1 = delta * (ratio - 1.0) / (ratio ** half - 1.0)
    widths_lo = h1 * ratio ** np.arange(half)
    faces_lo = np.concatenate([[0.0], np.cumsum(widths_lo)])
    faces_lo[-1] = delta
    faces = np.concatenate([faces_lo, 2.0 * delta - faces_lo[-2::-1]])
    centres = 0.5 * (faces[1:] + faces[:-1])
    widths = faces[1:] - faces[:-1]
    return centres, widths


def channel_rans_profile(y, re_tau, delta=1.0, u_tau=1.0):
    """Synthetic RANS fields at heights y (m) of a channel of half-height delta.

    Returns a dict with y (n,), U3 (n,3) in m/s, k (n,) in m^2/s^2,
    omega (n,) in 1/s and R6 (n,6) = (R11, R22, R33, R12, R13, R23) in m^2/s^2.
    """
    y = np.asarray(y, dtype=np.float64)
    nu = u_tau * delta / re_tau
    d_w = np.minimum(y, 2.0 * delta - y)
    if np.any(d_w <= 0.0):
        raise ValueError("profile points must lie strictly inside the channel")
    yp = d_w * u_tau / nu
    U = u_tau * reichardt_uplus(yp)
    sign = np.where(y <= delta, 1.0, -1.0)       # dU/dy flips in the upper half
    dUdy = sign * reichardt_duplus(yp) * u_tau ** 2 / nu
    k = u_tau ** 2 * k_plus(yp)
    omega = u_tau ** 2 / nu * omega_plus(yp)
    nu_t = k / omega
    n = y.size
    U3 = np.zeros((n, 3))
    U3[:, 0] = U
    R6 = np.zeros((n, 6))
    R6[:, 0] = R6[:, 1] = R6[:, 2] = 2.0 * k / 3.0
    R6[:, 3] = -nu_t * dUdy
    return {"y": y.copy(), "U3": U3, "k": k, "omega": omega, "R6": R6}


def bulk_velocity_fv(U, widths, delta=1.0):
    """Finite-volume bulk velocity sum(U_c dy_c) / (2 delta) (the RANS side's U_b)."""
    return float(np.sum(np.asarray(U) * np.asarray(widths)) / (2.0 * delta))
