"""Pins of the oracle's UCCSD minimum (the VQE outer loop's result), checked
against constructions that share no code with it: the determinant-space
Hamiltonian and UCCSD state of ``oracle.fockspace`` (no Pauli algebra, no
state-vector code) and brute-force diagonalisation."""
import numpy as np
import pytest

from oracle import exact, fermion, fockspace, minimize, uccsd
from workloads import n_uccsd_params, random_integrals


def _problem(n_orb, n_elec, seed):
    I = random_integrals(n_orb, n_elec, seed)
    c_id, terms = fermion.hamiltonian_terms(fermion.jw_hamiltonian(I.h1, I.eri))
    n = 2 * n_orb
    return I, n, c_id, terms, uccsd.rotations(n, n_elec)


@pytest.mark.parametrize("n_orb,seed", [(2, 11), (2, 13), (3, 14)])
def test_two_electrons_reach_the_sector_ground_state(n_orb, seed):
    """With two electrons the UCCSD product reaches every state of the
    two-electron sector, so its minimum is that sector's lowest eigenvalue."""
    I, n, c_id, terms, rots = _problem(n_orb, 2, seed)
    th0 = np.zeros(n_uccsd_params(n_orb, 2))
    _, e, _ = minimize.uccsd_minimum(n, 2, c_id, terms, rots, th0)
    sec = fockspace.Sector(n, 2)
    e0 = np.linalg.eigvalsh(fockspace.hamiltonian(sec, I.h1, I.eri))[0]
    assert abs(e - e0) < 1e-10, (e, e0)


def test_eight_qubit_minimum_is_variational_and_stationary():
    """8 qubits (4 orbitals, 4 electrons, integral seed 1001): the minimum from
    theta = 0 lies above the four-electron sector's ground state (UCCSD is not
    exact here) and above the whole space's; its energy is the determinant-space
    UCCSD energy at the returned point; and every central difference of that
    energy vanishes there."""
    I, n, c_id, terms, rots = _problem(4, 4, 1001)
    th, e, _ = minimize.uccsd_minimum(n, 4, c_id, terms, rots, np.zeros(n_uccsd_params(4, 4)))
    sec = fockspace.Sector(n, 4)
    H = fockspace.hamiltonian(sec, I.h1, I.eri)
    e_sec = np.linalg.eigvalsh(H)[0]
    assert e_sec + 1e-5 < e < e_sec + 1e-2
    assert e >= exact.ground_energy(n, c_id, terms) - 1e-12
    assert abs(fockspace.uccsd_energy(sec, H, th) - e) < 1e-12
    h = 1e-4
    for k in range(len(th)):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (fockspace.uccsd_energy(sec, H, tp) - fockspace.uccsd_energy(sec, H, tm)) / (2 * h)
        assert abs(fd) < 1e-6, (k, fd)
