"""Synthetic turbulence generator at the RANS/LES-LBM interface, FP64.

Follows the section "Synthetic turbulence generator in the Lattice Boltzmann
framework" and Algorithm 1 (LBM section, steps 1-8) in the paper's order:
interpolate the RANS fields to the lattice rows, Cholesky-factor the Reynolds
stress (eq. cholesky), form the length scales l_t, l_e, the cut-off l_cut
(eq. lcut) and the wavenumber range, weight the modes with the modified
von Karman spectrum (eq. qn), draw the random directions, normal vectors
and phases (eq. dn and the two lines after it), sum the Fourier modes at the
pseudo-position (eqs. aux_vec, psu), scale by the Cholesky factor (eq.
v_fluc), add the RANS mean (eqs. u_couple, u_phys) and convert to lattice
units (eq. u_transfer).  All lengths are physical (m), times in s.

Readings where the paper is silent or garbled:

* Interpolation (not specified): piecewise linear in y through the RANS cell
  centres plus the two wall points, where U = k = R = 0 and omega takes the
  value of the nearest centre (the k-omega wall value is singular).
* Lattice rows sit at y_j = (j + 1/2) c_x (halfway walls); the wall distance
  is d_w = min(y_j, 2 delta - y_j); spanwise nodes at z_k = k c_x; the inlet
  plane at x = 0.
* Theta = arccos(1 - 2 gamma) with gamma uniform in [0, 1): the printed range
  [0, 2 pi) would put the arccos argument outside [-1, 1]; this reading makes
  d^n uniform on the sphere as the text requires.
* The modified von Karman spectrum E(k) is cited, not printed.  The form of
  Shur et al. (2014) is used:
      E(k) = (k/k_e)^4 / (1 + 2.4 (k/k_e)^2)^(17/6) f_eta f_cut,
      f_eta = exp(-(12 k/k_eta)^2),
      f_cut = exp(-(4 max(k - 0.9 k_cut, 0)/k_cut)^3),
  k_e = 2 pi/l_e, k_eta = 2 pi/eta, eta = (nu^3/eps)^(1/4), eps = C_mu k omega,
  k_cut = 2 pi/l_cut.  Parity unpinned for the constants 2.4, 17/6, 12, 0.9,
  4 and 3 (the paper does not print them); the shape is pinned by its
  asymptotes.
* Wavenumbers k^n = k_min (1 + alpha)^(n-1), n = 1..N, with Delta k^n
  proportional to k^n (any such choice cancels in q^n).  N comes from the
  configuration; alpha is given, or chosen so that k^N = k_max.
* The grid sizes in eq. lcut are those of the uniform LES lattice,
  d_x = d_y = d_z = c_x.
* A negative radicand in the Cholesky factor is clamped to 0 and counted.
* U_b in eq. psu is the RANS bulk velocity (Algorithm 1, RANS step 2).
"""

import math

import numpy as np

from . import splitmix


def interpolate_rans(rans, y_rows, delta):
    """Linear interpolation of U, k, omega, R from the RANS grid to lattice rows."""
    y = np.asarray(rans["y"], dtype=np.float64)
    yy = np.concatenate([[0.0], y, [2.0 * delta]])

    def wall_zero(v):
        return np.concatenate([[0.0], v, [0.0]])

    out = {}
    out["U3"] = np.stack([np.interp(y_rows, yy, wall_zero(rans["U3"][:, c])) for c in range(3)], axis=1)
    out["k"] = np.interp(y_rows, yy, wall_zero(rans["k"]))
    om = rans["omega"]
    out["omega"] = np.interp(y_rows, yy, np.concatenate([[om[0]], om, [om[-1]]]))
    out["R6"] = np.stack([np.interp(y_rows, yy, wall_zero(rans["R6"][:, c])) for c in range(6)], axis=1)
    return out


def cholesky_factor(R6):
    """Lower-triangular a with a a^T = R (eq. cholesky), per row.

    R6 columns: R11, R22, R33, R12, R13, R23.  Returns (a (n,3,3), clamps).
    """
    R6 = np.atleast_2d(R6)
    n = R6.shape[0]
    a = np.zeros((n, 3, 3))
    clamps = 0
    for j in range(n):
        R11, R22, R33, R12, R13, R23 = R6[j]
        r = R11
        if r < 0.0:
            clamps += 1
            r = 0.0
        a11 = math.sqrt(r)
        a21 = R12 / a11 if a11 > 0.0 else 0.0
        a31 = R13 / a11 if a11 > 0.0 else 0.0
        r = R22 - a21 ** 2
        if r < 0.0:
            clamps += 1
            r = 0.0
        a22 = math.sqrt(r)
        a32 = (R23 - a21 * a31) / a22 if a22 > 0.0 else 0.0
        r = R33 - a31 ** 2 - a32 ** 2
        if r < 0.0:
            clamps += 1
            r = 0.0
        a33 = math.sqrt(r)
        a[j] = [[a11, 0.0, 0.0], [a21, a22, 0.0], [a31, a32, a33]]
    return a, clamps


def length_scales(k, omega, d_w, C_l=3.0, C_mu=0.09):
    """l_t = sqrt(k)/(C_mu omega) and l_e = min(2 d_w, C_l l_t)."""
    l_t = np.sqrt(k) / (C_mu * omega)
    l_e = np.minimum(2.0 * d_w, C_l * l_t)
    return l_t, l_e


def cutoff_length(d_x, d_y, d_z, d_w):
    """l_cut = 2 min(max(d_x, d_y, 0.3 d_max) + 0.1 d_w, d_max) (eq. lcut)."""
    d_max = max(d_x, d_y, d_z)
    return 2.0 * np.minimum(max(d_x, d_y, 0.3 * d_max) + 0.1 * np.asarray(d_w), d_max)


def mode_count(k_max, k_min, alpha=0.01):
    """N = ceil(ln(k_max/k_min)/ln(1 + alpha) + 1) (eq. Nmode)."""
    return int(math.ceil(math.log(k_max / k_min) / math.log(1.0 + alpha) + 1.0))


def wavenumbers(k_min, k_max, n_modes, alpha):
    """k^n = k_min (1 + alpha)^(n-1), n = 1..N; alpha <= 0 spans [k_min, k_max]."""
    if alpha <= 0.0:
        alpha = (k_max / k_min) ** (1.0 / (n_modes - 1)) - 1.0
    n = np.arange(n_modes, dtype=np.float64)
    return k_min * (1.0 + alpha) ** n, alpha


def von_karman_modified(k, k_e, k_eta, k_cut):
    """Modified von Karman spectrum (form of Shur et al. 2014, see header)."""
    k = np.asarray(k, dtype=np.float64)
    r = k / k_e
    f_eta = np.exp(-((12.0 * k / k_eta) ** 2))
    f_cut = np.exp(-((4.0 * np.maximum(k - 0.9 * k_cut, 0.0) / k_cut) ** 3))
    return r ** 4 / (1.0 + 2.4 * r ** 2) ** (17.0 / 6.0) * f_eta * f_cut


def spectrum_weights(k_n, alpha, l_e, k, omega, nu, k_cut, C_mu=0.09):
    """q^n per lattice row (eq. qn): (NY, N), each row summing to 1."""
    eps = C_mu * k * omega
    eta = (nu ** 3 / eps) ** 0.25
    k_eta = 2.0 * np.pi / eta
    k_e = 2.0 * np.pi / l_e
    dk = alpha * k_n
    E = von_karman_modified(k_n[None, :], k_e[:, None], k_eta[:, None], np.asarray(k_cut)[:, None] * np.ones_like(k_n)[None, :])
    Edk = E * dk[None, :]
    return Edk / Edk.sum(axis=1, keepdims=True)


def draw_modes(seed, n_modes):
    """Random directions d^n, normals sigma^n and phases phi^n (eq. dn).

    Uniforms from SplitMix64(seed), four per mode in the order
    Phi, gamma, eta, phi: outputs 4n+1 .. 4n+4 for mode n = 0..N-1.
    """
    d = np.zeros((n_modes, 3))
    sigma = np.zeros((n_modes, 3))
    phase = np.zeros(n_modes)
    for n in range(n_modes):
        u1, u2, u3, u4 = (splitmix.uniform(seed, 4 * n + m) for m in (1, 2, 3, 4))
        Phi = 2.0 * math.pi * u1
        Theta = math.acos(1.0 - 2.0 * u2)
        eta = 2.0 * math.pi * u3
        d[n] = [math.sin(Theta) * math.cos(Phi), math.sin(Theta) * math.sin(Phi), math.cos(Theta)]
        sigma[n] = [math.cos(Phi) * math.cos(Theta) * math.cos(eta) - math.sin(Phi) * math.sin(eta),
                    math.sin(Phi) * math.cos(Theta) * math.cos(eta) + math.cos(Phi) * math.sin(eta),
                    -math.sin(Theta) * math.cos(eta)]
        phase[n] = 2.0 * math.pi * u4
    return d, sigma, phase


def auxiliary_field(t, x, y, z, k_n, d, sigma, phase, sqrt_q, L_e, U_b):
    """v'(x, t) = sqrt(6) sum_n sqrt(q^n) sigma^n cos(k^n d^n . x' + phi^n) (eqs. aux_vec, psu).

    y: (NY,), z: (NZ,) physical node coordinates; x scalar (the inlet plane);
    sqrt_q: (NY, N).  Returns v' of shape (NY, NZ, 3).
    """
    ny, nz = y.size, z.size
    v = np.zeros((ny, nz, 3))
    for n in range(k_n.size):
        x_pseudo = 2.0 * np.pi / (k_n[n] * L_e) * (x - U_b * t)
        arg = k_n[n] * (d[n, 0] * x_pseudo + d[n, 1] * y[:, None] + d[n, 2] * z[None, :]) + phase[n]
        amp = sqrt_q[:, n][:, None] * np.cos(arg)
        v += amp[:, :, None] * sigma[n][None, None, :]
    return math.sqrt(6.0) * v


class InletGenerator:
    """Per-row precompute (Algorithm 1, LBM steps 1-4) and the plane (steps 5-8)."""

    def __init__(self, rans, ny, nz, delta, c_x, c_t, nu_phys, U_b, n_modes, alpha, seed,
                 C_l=3.0, C_mu=0.09):
        self.ny, self.nz = ny, nz
        self.c_x, self.c_t = c_x, c_t
        self.U_b = U_b
        self.y = (np.arange(ny) + 0.5) * c_x
        self.z = np.arange(nz) * c_x
        self.d_w = np.minimum(self.y, 2.0 * delta - self.y)
        it = interpolate_rans(rans, self.y, delta)
        self.U_int = it["U3"]
        self.k, self.omega, self.R6 = it["k"], it["omega"], it["R6"]
        self.a, self.clamps = cholesky_factor(self.R6)
        self.l_t, self.l_e = length_scales(self.k, self.omega, self.d_w, C_l, C_mu)
        self.L_e = float(self.l_e.max())
        self.l_cut = cutoff_length(c_x, c_x, c_x, self.d_w)
        self.k_cut = 2.0 * np.pi / self.l_cut
        self.k_min = np.pi / self.L_e
        self.k_max = 1.5 * float(self.k_cut.max())
        self.k_n, self.alpha = wavenumbers(self.k_min, self.k_max, n_modes, alpha)
        self.q = spectrum_weights(self.k_n, self.alpha, self.l_e, self.k, self.omega, nu_phys,
                                  self.k_cut, C_mu)
        self.d, self.sigma, self.phase = draw_modes(seed, n_modes)

    def fluctuation(self, t_step):
        """u'(t) = a v' (eq. v_fluc) in m/s, shape (NY, NZ, 3)."""
        t = t_step * self.c_t
        v = auxiliary_field(t, 0.0, self.y, self.z, self.k_n, self.d, self.sigma, self.phase,
                            np.sqrt(self.q), self.L_e, self.U_b)
        return np.einsum("jab,jzb->jza", self.a, v)

    def plane(self, t_step):
        """u_bc in lattice units at step index t_step (eqs. u_phys, u_transfer): (NY, NZ, 3)."""
        u_phys = self.U_int[:, None, :] + self.fluctuation(t_step)
        return u_phys * self.c_t / self.c_x

    def modes_table(self):
        """(N, 8): k^n, d^n (3), sigma^n (3), phi^n."""
        return np.concatenate([self.k_n[:, None], self.d, self.sigma, self.phase[:, None]], axis=1)
