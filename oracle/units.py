"""Lattice <-> physical unit conversion (Numerical setup section), FP64.

c_x = L_phys / L_LB and c_t = t_phys / t_LB (eq. c_factor); velocities
convert as u_LB = u_phys c_t / c_x (eq. u_transfer); viscosities as
nu_LB = nu_phys c_t / c_x^2, with nu_LB = c_s^2 (tau - 1/2) (eq. lbe-nu);
the Mach number is u_LB / c_s (eq. ma-eq); an acceleration converts as
a_LB = a_phys c_t^2 / c_x.
"""

import math

CS = 1.0 / math.sqrt(3.0)


def lattice_spacing(delta, ny):
    """c_x for a channel of height 2 delta resolved by NY lattice rows."""
    return 2.0 * delta / ny


def time_step_from_bulk(u_b_lb, c_x, U_b_phys):
    """c_t that maps the RANS bulk velocity U_b onto the lattice bulk velocity u_b_lb."""
    return u_b_lb * c_x / U_b_phys


def time_step_from_tau(tau, c_x, nu_phys):
    """c_t = nu_LB / nu_phys c_x^2 with nu_LB = c_s^2 (tau - 1/2) (paper's worked example)."""
    return CS ** 2 * (tau - 0.5) / nu_phys * c_x ** 2


def nu_lattice(nu_phys, c_t, c_x):
    return nu_phys * c_t / c_x ** 2


def tau_from_nu(nu_lb):
    return nu_lb / CS ** 2 + 0.5


def velocity_to_lattice(u_phys, c_t, c_x):
    return u_phys * c_t / c_x


def mach(u_lb):
    return u_lb / CS


def acceleration_to_lattice(a_phys, c_t, c_x):
    return a_phys * c_t ** 2 / c_x


def channel_units(delta, ny, u_b_lb, U_b_phys, nu_phys):
    """(c_x, c_t, nu_LB, tau0) of a channel run at lattice bulk velocity u_b_lb."""
    c_x = lattice_spacing(delta, ny)
    c_t = time_step_from_bulk(u_b_lb, c_x, U_b_phys)
    nu_lb = nu_lattice(nu_phys, c_t, c_x)
    return c_x, c_t, nu_lb, tau_from_nu(nu_lb)
