"""Minimum of the UCCSD energy over its parameters (oracle, test only).

Paper: Sec. II-A -- VQE hands the energy E(theta) of the ansatz state (Eq. 2
with the state of Eq. 3-4) to a classical optimizer, which updates theta until
E stops decreasing; the paper does not name the optimizer.  What the outer
loop computes is therefore a local minimum of E(theta): a point where the
gradient vanishes, and its energy.  That value, not the path to it, is the
result; several optimizers reach the same minimum from the same start.

The oracle reaches it with scipy's L-BFGS-B (a library minimiser used as one
step) on the dense state-vector energy and its exact adjoint gradient, with
tolerances far below what a caller asks of the GPU loop, so the returned
energy is the minimum's value to rounding.

Pins (tests/test_oracle_minimize.py): for two electrons UCCSD spans the whole
fixed-electron sector, so the minimum equals the lowest eigenvalue of the
determinant-space Hamiltonian of ``fockspace`` (no Pauli algebra); for more
electrons the minimum lies above that eigenvalue (variational bound); the
returned point is stationary by central differences of ``fockspace``'s UCCSD
energy.
"""
from __future__ import annotations

import numpy as np
import scipy.optimize

from . import statevector as sv


def uccsd_minimum(n: int, n_elec: int, c_id, terms, rots, theta0, gtol: float = 1e-11):
    """Local minimum of E(theta) reached from theta0: (theta*, E*, n_iter).
    E excludes the constant energy shift, like ``statevector.vqe_energy``."""
    pa = sv.PauliApplier(n)

    def fg(th):
        g, _, e = sv.grad_adjoint(n, n_elec, c_id, terms, rots, th, pa)
        return e, g

    res = scipy.optimize.minimize(fg, np.asarray(theta0, dtype=float), jac=True, method="L-BFGS-B",
                                  options={"gtol": gtol, "ftol": 1e-16, "maxiter": 5000})
    return res.x, float(res.fun), int(res.nit)
