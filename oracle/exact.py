"""Brute-force ground-state energy of a qubit Hamiltonian (oracle, test only).

Used for the variational bound E(theta, D) >= E_0: any normalised state,
including a truncated MPS, has energy at least the lowest eigenvalue of H over
the full 2^N space.  Dense diagonalisation (numpy eigvalsh), N <= 12.
"""
from __future__ import annotations

import numpy as np

from .statevector import PauliApplier


def hamiltonian_matrix(n: int, c_id: float, terms) -> np.ndarray:
    if n > 12:
        raise ValueError("brute force limited to 12 qubits")
    pa = PauliApplier(n)
    dim = 1 << n
    H = np.zeros((dim, dim), dtype=complex)
    H[np.arange(dim), np.arange(dim)] += c_id
    cols = np.arange(dim)
    for x, z, c in terms:
        dest, coef = pa.parts(x, z)
        # P|b> = coef[b] |dest[b]>  ->  H[dest[b], b] += c coef[b]
        H[dest, cols] += c * coef
    return H


def ground_energy(n: int, c_id: float, terms) -> float:
    return float(np.linalg.eigvalsh(hamiltonian_matrix(n, c_id, terms))[0])
