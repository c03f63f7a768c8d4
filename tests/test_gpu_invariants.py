"""Properties of the HIP path that hold whatever the size: a steady laminar
inlet/outlet channel carries the same mass flux through every x-face, and the
outlet holds its density; the oracle pins the same property in FP64."""

import numpy as np
import pytest

from oracle.lattice import C
from workloads.configs import small_channel

pytestmark = pytest.mark.gpu


def _face_flux(f, nx, ny):
    """Mass crossing each face x + 1/2 per step: c_x = +1 populations leaving
    plane x minus c_x = -1 populations leaving plane x + 1, without those the
    walls reflect back into their own plane."""
    def crossing(sgn):
        tot = np.zeros(nx)
        for i in range(19):
            cx, cy, _ = C[i]
            if cx != sgn:
                continue
            g = f[i].copy()
            if cy == 1:
                g[:, ny - 1, :] = 0.0
            elif cy == -1:
                g[:, 0, :] = 0.0
            tot += g.sum(axis=(0, 1))
        return tot
    return crossing(1)[:-1] - crossing(-1)[1:]


@pytest.mark.parametrize("shape", [(24, 8, 2), (130, 12, 3)])
def test_laminar_inlet_outlet_mass_flux(shape):
    """No fluctuations (R = 0, so the Cholesky factor and u' vanish): after the
    transient the flux is equal on every face to FP32 rounding."""
    from paper_2205_02774_amd import Lattice
    nx, ny, nz = shape
    rans = dict(small_channel(nx, ny, nz)["rans"])
    rans["R6"] = np.zeros_like(rans["R6"])
    print(f"[gpu] laminar mass flux {shape}", flush=True)
    lat = Lattice(nx, ny, nz, device="cuda:0", nu_lb=0.1, cs_smag=0.0, sponge_cells=0,
                  max_modes=20, max_rans=len(rans["y"]))
    c_x = 2.0 / ny
    lat.set_rans_inlet(rans, delta=1.0, nu_phys=1 / 180, c_x=c_x, c_t=0.05 * c_x / rans["U_b"], U_b=rans["U_b"],
                       n_modes=20, alpha=0.05, seed=0)
    lat.step(4000)
    f = lat.get_f()
    lat.close()
    phi = _face_flux(f, nx, ny)
    spread = np.ptp(phi) / phi.mean()
    print(f"[gpu] laminar mass flux {shape}: mean {phi.mean():.6e}, spread {spread:.2e}", flush=True)
    assert phi.mean() > 0
    # FP32 state: each f carries ~6e-8 relative rounding and a face sum adds NY NZ 5 of them
    assert spread < 1e-5
    # pressure outlet: rho = rho_out on the last plane (after its rebuild and collision, which conserves mass)
    rho_out = f[:, :, :, -1].sum(axis=0)
    assert np.abs(rho_out - 1.0).max() < 1e-5
