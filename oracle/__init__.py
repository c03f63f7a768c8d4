"""FP64 CPU oracle of the STG-LBM hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct NumPy implementation of what the method
computes, written from the paper (Xue, Yao & Davidson, "Synthetic turbulence
generator for lattice Boltzmann method at the interface between RANS and
LES"), section by section:

* ``lattice``  -- D3Q19 (and D3Q15, D3Q27) lattice BGK, regularized or
  plain, with Guo forcing (Methodology, eqs.
  density/momentum/tensor, lbe, local_eq, lbe-nu, bodyforce), Smagorinsky
  effective relaxation (eqs. smogrinsky_model, strain, tau_eff), regularized
  boundary reconstruction (eqs. f_i .. bc_eq), halfway bounce-back walls,
  periodic span, the regularized pressure outlet and the sponge (eq.
  sponge_visco), on-device-style flow statistics (eq. v_rms).
* ``stg``      -- the synthetic turbulence generator (eqs. u_couple .. lcut):
  RANS-to-lattice interpolation, Cholesky factor, length scales, modified
  von Karman spectrum weights, random Fourier modes, pseudo-position and the
  inlet velocity plane (eqs. u_phys, u_transfer).
* ``units``    -- lattice/physical conversion (eqs. c_factor, lbe-nu, ma-eq).
* ``splitmix`` -- SplitMix64, the counter-based generator both sides use for
  the random mode draws.
* ``channel``  -- Algorithm 1 (STG-LBM) driven step by step.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import or run anything in this package.  The GPU library shares no
code with it: the two meet only in the seeded inputs of ``workloads``.

Readings of passages where the paper is silent, garbled or inconsistent are
named constants or flags here and are listed with each function.

Parity status: every function is pinned by a test in ``tests/test_oracle_*``
against closed forms, invariants, textbook special cases or the paper's
worked example, except where a docstring says "parity unpinned".
"""

from . import lattice, stg, units, splitmix, channel  # noqa: F401
from .channel import OracleChannel  # noqa: F401
