"""D3Q19 lattice-Boltzmann LES, FP64 (test infrastructure, see package header).

Every function also runs on the D3Q15 and D3Q27 sets: the set is taken from
the leading dimension of the distribution array (or a q argument).

Arrays of distributions are indexed f[i, z, y, x]: population i, spanwise
z, wall-normal y, streamwise x.  All functions work on whole arrays with
NumPy broadcasting; nothing is blocked, fused or reordered beyond the
equations cited.

Readings adopted where the paper is silent or garbled:

* COLLISION_SIGN: the lbe equation prints "+Omega[f - f_eq]" with
  Omega = dt/tau; relaxation toward equilibrium needs -1/tau(f - f_eq).
* The bulk collision is the regularized BGK operator: the non-equilibrium part
  is replaced by its Hermite projection of order <= 2,
  w_i [c_i . J_neq / c_s^2 + Q_i:Pi_neq / (2 c_s^4)], before relaxing; the
  second-order part is the operator the method uses to rebuild boundary
  populations.  J_neq = sum_i c_i (f_i - f_eq_i) is -F/2 under the momentum
  definition of eq. momentum; keeping it makes the Guo force of eq.
  bodyforce add exactly F of momentum per step, as it does for plain BGK.
  Plain BGK (eq. lbe as printed, with the sign read as relaxation) is kept as
  an oracle-only option for the Poiseuille self-test.
* REG_FACTOR: eq. f_i_neq prints w_i/c_s^4 Q_i:Pi_neq; with that factor the
  second moment of the rebuilt part is 2 Pi_neq, so the factor is
  w_i/(2 c_s^4) (pinned by the Hermite-projection test).
* tau_eff: eq. tau_eff drops a factor rho inside the root relative to eq.
  strain; the strain-consistent form with dx = dt = filter width = 1 is
  tau = (tau0 + sqrt(tau0^2 + 18 sqrt(2) C Q^{1/2}/rho))/2, C = Cs^2.
* Pi_neq in the bulk is sum_i c_i c_i (f_i - f_eq_i) without a forcing
  correction.
* Walls: halfway (link) bounce-back, walls at y = -1/2 and y = NY - 1/2.
* Zou-He density: eq. density_bc_sub swaps the two index sets and leaves out
  the rest population; the text's definition is used: populations pointing
  toward the boundary count twice, those tangential to it (rest included)
  once.
* Inlet unknowns are always the c_x = +1 populations, outlet unknowns the
  c_x = -1 populations; wall bounce-back is applied before the boundary
  rebuild.
* Outlet: density fixed at rho_out, normal velocity from the same Zou-He mass
  identity, tangential velocity zero, then the same regularized rebuild.
* Sponge (eq. sponge_visco): nu is multiplied by (1 + K s^p) with
  s = (x - x_start)/(x_end - x_start), x_end = NX - 1, x_start = x_end - L_s.
"""

import numpy as np

CS2 = 1.0 / 3.0          # c_s^2 (Methodology: c_s = 1/sqrt(3)); the same for D3Q15, D3Q19 and D3Q27
CS4 = CS2 * CS2

_AXES = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
_FACES = [(1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
          (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
          (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
_CORNERS = [(1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
            (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1)]


class VelocitySet:
    """A cubic velocity set: rest, then opposite directions as neighbours (i, i+1) for odd i.

    D3Q19 is the method's set (Methodology); D3Q15 and D3Q27 are the variants
    the method's boundary treatment carries over to (Numerical method, the
    remark on other velocity sets).  Weights are the standard ones that make
    the moments isotropic up to fourth order with c_s^2 = 1/3.
    """

    def __init__(self, name, dirs, weights):
        self.name = name
        self.C = np.array([(0, 0, 0)] + dirs, dtype=np.int64)
        self.Q = len(self.C)
        self.W = np.array(weights, dtype=np.float64)
        self.OPP = np.array([0] + [i + 1 if i % 2 == 1 else i - 1 for i in range(1, self.Q)], dtype=np.int64)
        # Q_i = c_i c_i - c_s^2 I (eq. f_i_neq), shape (Q, 3, 3)
        self.QT = np.einsum("ia,ib->iab", self.C, self.C).astype(np.float64) - CS2 * np.eye(3)[None]
        self.INLET_UNKNOWN = self.C[:, 0] == 1
        self.OUTLET_UNKNOWN = self.C[:, 0] == -1


D3Q19 = VelocitySet("D3Q19", _AXES + _FACES, [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
D3Q15 = VelocitySet("D3Q15", _AXES + _CORNERS, [2 / 9] + [1 / 9] * 6 + [1 / 72] * 8)
D3Q27 = VelocitySet("D3Q27", _AXES + _FACES + _CORNERS,
                    [8 / 27] + [2 / 27] * 6 + [1 / 54] * 12 + [1 / 216] * 8)
VELOCITY_SETS = {15: D3Q15, 19: D3Q19, 27: D3Q27}


def velocity_set(q):
    """The velocity set with q populations (15, 19 or 27)."""
    return VELOCITY_SETS[int(q)]


# The method's set, under the names the rest of the oracle and its pins use.
Q, C, W, OPP, QT = D3Q19.Q, D3Q19.C, D3Q19.W, D3Q19.OPP, D3Q19.QT


def _bc(v, nd):
    """Broadcast a (Q,) table against a field with nd trailing dims."""
    return v.reshape((len(v),) + (1,) * nd)


def density(f):
    """rho = sum_i f_i (eq. density)."""
    return f.sum(axis=0)


def velocity(f, rho, force):
    """u from rho u = sum_i f_i c_i + F dt/2 (eq. momentum), dt = 1."""
    vs = velocity_set(f.shape[0])
    nd = f.ndim - 1
    u = np.empty((3,) + f.shape[1:])
    for a in range(3):
        u[a] = ((f * _bc(vs.C[:, a].astype(np.float64), nd)).sum(axis=0) + 0.5 * force[a]) / rho
    return u


def equilibrium(rho, u, q=19):
    """Second-order equilibrium f_eq_i(rho, u) (eq. local_eq), shape (q, ...)."""
    vs = velocity_set(q)
    nd = rho.ndim
    cu = np.einsum("ia,a...->i...", vs.C.astype(np.float64), u)
    uu = (u * u).sum(axis=0)
    return _bc(vs.W, nd) * rho[None] * (1.0 + cu / CS2 + cu ** 2 / (2.0 * CS4) - uu[None] / (2.0 * CS2))


def second_moment(h):
    """sum_i c_i c_i h_i as a (3, 3, ...) tensor (eq. tensor)."""
    Cf = velocity_set(h.shape[0]).C.astype(np.float64)
    return np.einsum("ia,ib,i...->ab...", Cf, Cf, h)


def hermite_part(pi_neq, q=19):
    """w_i/(2 c_s^4) Q_i : Pi_neq (eq. f_i_neq with the factor 1/2, see header)."""
    vs = velocity_set(q)
    nd = pi_neq.ndim - 2
    qp = np.einsum("iab,ab...->i...", vs.QT, pi_neq)
    return _bc(vs.W, nd) / (2.0 * CS4) * qp


def first_order_part(j_neq, q=19):
    """w_i c_i . J_neq / c_s^2: first-order Hermite projection of a non-equilibrium part."""
    vs = velocity_set(q)
    nd = j_neq.ndim - 1
    cj = np.einsum("ia,a...->i...", vs.C.astype(np.float64), j_neq)
    return _bc(vs.W, nd) * cj / CS2


def q_half(pi_neq):
    """Q^{1/2} = sqrt(Pi_neq : Pi_neq) (Smagorinsky section)."""
    return np.sqrt(np.einsum("ab...,ab...->...", pi_neq, pi_neq))


def tau_effective(tau0, cs_smag, qh, rho):
    """Effective relaxation time of the Smagorinsky model, dx = dt = 1.

    From eq. strain and nu_eff = nu_0 + C delta^2 |S| = c_s^2 (tau_eff - 1/2)
    with C = Cs^2: tau_eff = (tau0 + sqrt(tau0^2 + 18 sqrt(2) C Q^{1/2}/rho))/2.
    """
    c = cs_smag ** 2
    return 0.5 * (tau0 + np.sqrt(tau0 ** 2 + 18.0 * np.sqrt(2.0) * c * qh / rho))


def smagorinsky_strain(tau0, cs_smag, qh, rho):
    """|S| of eq. strain with dx = dt = c = delta = 1 (used by the pins)."""
    c = cs_smag ** 2
    return (-tau0 * rho + np.sqrt((tau0 * rho) ** 2 + 18.0 * np.sqrt(2.0) * rho * c * qh)) / (6.0 * rho * c)


def sponge_factor(nx, sponge_cells, K, p):
    """Per-x viscosity multiplier 1 + K s^p of eq. sponge_visco (1 outside)."""
    fac = np.ones(nx)
    if sponge_cells > 0:
        x_end = nx - 1
        x_start = x_end - sponge_cells
        x = np.arange(nx, dtype=np.float64)
        s = (x - x_start) / (x_end - x_start)
        inside = x >= x_start
        fac[inside] = K * s[inside] ** p + 1.0
    return fac


def guo_source(u, tau, force, q=19):
    """Guo forcing F_i (eq. bodyforce) for acceleration F, shape (q, ...)."""
    vs = velocity_set(q)
    nd = u.ndim - 1
    Cf = vs.C.astype(np.float64)
    out = np.zeros((vs.Q,) + u.shape[1:])
    cu = np.einsum("ia,a...->i...", Cf, u)
    for a in range(3):
        if force[a] == 0.0:
            continue
        term = (_bc(Cf[:, a], nd) - u[a][None]) / CS2 + cu / CS4 * _bc(Cf[:, a], nd)
        out += term * force[a]
    return (1.0 - 1.0 / (2.0 * tau))[None] * _bc(vs.W, nd) * out


def collide(f, tau0, cs_smag, force, sponge, operator="regularized"):
    """BGK-type collision with Smagorinsky tau_eff, sponge and Guo force.

    f: post-streaming populations (after any boundary rebuild), (Q, NZ, NY, NX)
    for any of the velocity sets.  sponge: (NX,) viscosity multipliers.
    operator="regularized" relaxes the Hermite projection of f - f_eq (orders 1
    and 2, see header); operator="bgk" relaxes the full f - f_eq (eq. lbe, the
    paper's plain BGK bulk).  Returns (f_post, rho, u).
    """
    q = f.shape[0]
    rho = density(f)
    u = velocity(f, rho, force)
    feq = equilibrium(rho, u, q)
    fneq = f - feq
    pi_neq = second_moment(fneq)
    tau = tau_effective(tau0, cs_smag, q_half(pi_neq), rho)
    tau = 0.5 + (tau - 0.5) * sponge[None, None, :]
    if operator == "bgk":
        reg = fneq
    else:
        j_neq = np.einsum("ia,i...->a...", velocity_set(q).C.astype(np.float64), fneq)
        reg = first_order_part(j_neq, q) + hermite_part(pi_neq, q)
    f_post = feq + (1.0 - 1.0 / tau)[None] * reg
    if any(fc != 0.0 for fc in force):
        f_post = f_post + guo_source(u, tau, force, q)
    return f_post, rho, u


def stream(f_post, periodic_x, periodic_y=False):
    """Pull streaming f~_i(x) = f*_i(x - c_i) with the domain's boundaries.

    z is periodic; y has halfway bounce-back walls, f~_i = f*_opp(i) at the
    same node when x - c_i lies behind a wall.  x is periodic when periodic_x,
    otherwise populations entering through the inlet (x = 0, c_x = +1) or the
    outlet (x = NX-1, c_x = -1) are unknown and set to NaN here, so that any
    use of them before the boundary rebuild shows up.  periodic_y replaces the
    walls by wrap-around (oracle-only, for the shear-wave self-test).
    """
    vs = velocity_set(f_post.shape[0])
    _, nz, ny, nx = f_post.shape
    ft = np.empty_like(f_post)
    for i in range(vs.Q):
        cx, cy, cz = (int(v) for v in vs.C[i])
        ft[i] = np.roll(f_post[i], shift=(cz, cy, cx), axis=(0, 1, 2))
        if periodic_y:
            pass
        elif cy == 1:
            ft[i][:, 0, :] = f_post[vs.OPP[i]][:, 0, :]
        elif cy == -1:
            ft[i][:, ny - 1, :] = f_post[vs.OPP[i]][:, ny - 1, :]
        if not periodic_x:
            if cx == 1:
                ft[i][:, :, 0] = np.nan
            elif cx == -1:
                ft[i][:, :, nx - 1] = np.nan
    return ft


def regularized_rebuild(f_plane, rho_bc, u_bc, unknown):
    """Regularized reconstruction of a boundary node (eqs. f_i .. bc_eq).

    f_plane: (19, ...) post-stream populations, entries of `unknown` unused.
    rho_bc (...), u_bc (3, ...): boundary density and velocity.
    unknown: boolean (19,) mask of the populations entering the domain.
    f_neq = f - f_eq(rho_bc, u_bc) on the known set, f_neq_i = f_neq_opp(i) on
    the unknown set (eq. unknown_neq), Pi_neq = sum_i Q_i f_neq_i (eq. pi_neq),
    f_i = f_eq_i + w_i/(2 c_s^4) Q_i:Pi_neq for every i.
    """
    vs = velocity_set(f_plane.shape[0])
    feq = equilibrium(rho_bc, u_bc, vs.Q)
    fneq = f_plane - feq
    for i in range(vs.Q):
        if unknown[i]:
            fneq[i] = fneq[vs.OPP[i]]
    pi_neq = np.einsum("iab,i...->ab...", vs.QT, fneq)
    return feq + hermite_part(pi_neq, vs.Q)


def inlet_density(f_plane, u_bc_x):
    """Zou-He density at the x = 0 plane (eq. density_bc, outward n = -x).

    rho_bc = (sum_{c_x = 0} f + 2 sum_{c_x = -1} f) / (1 + u.n), u.n = -u_x.
    """
    Cs = velocity_set(f_plane.shape[0]).C
    tang = f_plane[Cs[:, 0] == 0].sum(axis=0)
    toward = f_plane[Cs[:, 0] == -1].sum(axis=0)
    return (2.0 * toward + tang) / (1.0 - u_bc_x)


def outlet_velocity(f_plane, rho_out):
    """Normal velocity at the x = NX-1 plane from the Zou-He mass identity.

    rho_out (1 + u_x) = sum_{c_x = 0} f + 2 sum_{c_x = +1} f; tangential
    velocity zero (reading of the regularized pressure outlet).
    """
    Cs = velocity_set(f_plane.shape[0]).C
    tang = f_plane[Cs[:, 0] == 0].sum(axis=0)
    toward = f_plane[Cs[:, 0] == 1].sum(axis=0)
    ux = (tang + 2.0 * toward) / rho_out - 1.0
    u = np.zeros((3,) + ux.shape)
    u[0] = ux
    return u


INLET_UNKNOWN = D3Q19.INLET_UNKNOWN
OUTLET_UNKNOWN = D3Q19.OUTLET_UNKNOWN


def apply_inlet(ft, u_bc_zy):
    """Rebuild the x = 0 plane from the inlet velocity u_bc (3, NZ, NY)."""
    plane = ft[:, :, :, 0]
    rho_bc = inlet_density(plane, u_bc_zy[0])
    ft[:, :, :, 0] = regularized_rebuild(plane, rho_bc, u_bc_zy, velocity_set(ft.shape[0]).INLET_UNKNOWN)


def apply_outlet(ft, rho_out):
    """Rebuild the x = NX-1 plane with fixed density rho_out."""
    plane = ft[:, :, :, -1]
    u = outlet_velocity(plane, rho_out)
    rho = np.full(plane.shape[1:], float(rho_out))
    ft[:, :, :, -1] = regularized_rebuild(plane, rho, u, velocity_set(ft.shape[0]).OUTLET_UNKNOWN)


def lattice_step(f_post, *, tau0, cs_smag, force, sponge, periodic_x, u_bc_zy=None, rho_out=1.0,
                 periodic_y=False, operator="regularized"):
    """One time step n -> n+1 (Algorithm 1, steps 9-12 for every cell).

    Returns (f_post_new, rho, u) where rho, u are the moments the collision
    used (the values the flow statistics sample).
    """
    ft = stream(f_post, periodic_x, periodic_y)
    if not periodic_x:
        apply_inlet(ft, u_bc_zy)
        apply_outlet(ft, rho_out)
    return collide(ft, tau0, cs_smag, force, sponge, operator)


def stats_bins(u):
    """Per-(x, y) sums over z of u, v, w, uu, vv, ww, uv, uw, vw; shape (NX, NY, 9)."""
    ux, uy, uz = u
    comps = (ux, uy, uz, ux * ux, uy * uy, uz * uz, ux * uy, ux * uz, uy * uz)
    return np.stack([c.sum(axis=0).T for c in comps], axis=-1)
