"""Pins for the oracle's Pauli algebra and Jordan-Wigner Hamiltonian.

Each check is independent of the code it tests: dense 2x2 Kronecker products,
canonical anticommutation relations, a Pauli-basis trace decomposition of the
Hamiltonian built in determinant space (no Pauli algebra), structural
invariants of real Hamiltonians, and the count the paper prints for H2.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import fermion, fockspace
from oracle.statevector import PauliApplier
from workloads import h2_like_integrals, random_integrals

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_pauli_product_matches_dense_matrices():
    n = 3
    rng = np.random.default_rng(0)
    for _ in range(200):
        x1, z1, x2, z2 = (int(v) for v in rng.integers(0, 1 << n, size=4))
        ph, x3, z3 = fermion.pauli_mul(x1, z1, x2, z2)
        lhs = fermion.pauli_dense(x1, z1, n) @ fermion.pauli_dense(x2, z2, n)
        rhs = ph * fermion.pauli_dense(x3, z3, n)
        assert np.allclose(lhs, rhs, atol=1e-14)


def test_statevector_pauli_application_matches_dense():
    n = 4
    pa = PauliApplier(n)
    rng = np.random.default_rng(1)
    psi = rng.normal(size=16) + 1j * rng.normal(size=16)
    for x in range(16):
        for z in range(16):
            assert np.allclose(pa.apply(x, z, psi), fermion.pauli_dense(x, z, n) @ psi, atol=1e-13)


def test_jordan_wigner_anticommutation():
    n = 4
    a = [fermion.paulisum_dense(fermion.jw_annihilate(P), n) for P in range(n)]
    ad = [fermion.paulisum_dense(fermion.jw_create(P), n) for P in range(n)]
    eye = np.eye(1 << n)
    for P, Q in itertools.product(range(n), repeat=2):
        assert np.allclose(a[P] @ ad[Q] + ad[Q] @ a[P], eye * (P == Q), atol=1e-14)
        assert np.allclose(a[P] @ a[Q] + a[Q] @ a[P], 0, atol=1e-14)
        assert np.allclose(ad[P], a[P].conj().T)
    # |1> = occupied: n_P = a+_P a_P is diagonal with 1 where qubit P is 1
    for P in range(n):
        num = ad[P] @ a[P]
        bits = [(b >> (n - 1 - P)) & 1 for b in range(1 << n)]
        assert np.allclose(num, np.diag(bits))


@pytest.mark.parametrize("n_orb,seed", [(2, 3), (3, 4)])
def test_jw_coefficients_equal_trace_decomposition_of_fock_hamiltonian(n_orb, seed):
    """c_P = Tr(P H) / 2^N with H built from fermionic sign rules only."""
    I = random_integrals(n_orb, n_orb, seed)
    n = 2 * n_orb
    sec = fockspace.Sector(n, None)
    Hq = fockspace.to_qubit_basis(sec, fockspace.hamiltonian(sec, I.h1, I.eri, 0.37))
    jw = fermion.jw_hamiltonian(I.h1, I.eri, 0.37)
    pa = PauliApplier(n)
    cols = np.arange(1 << n)
    found = {}
    for x in range(1 << n):
        for z in range(1 << n):
            dest, coef = pa.parts(x, z)
            # Tr(P H) = sum_b <b|P H|b> = sum_b conj(coef[b]) H[dest[b], b]
            tr = np.sum(np.conj(coef) * Hq[dest, cols]) / (1 << n)
            if abs(tr) > 1e-12:
                found[(x, z)] = tr
    assert set(found) == set(jw.terms)
    for k, v in found.items():
        assert abs(jw.terms[k] - v) < 1e-12


def test_h2_string_count_matches_paper():
    with open(os.path.join(GOLDEN, "h2_paper_counts.json")) as f:
        g = json.load(f)
    I = h2_like_integrals()
    H = fermion.jw_hamiltonian(I.h1, I.eri)
    c_id, terms = fermion.hamiltonian_terms(H)
    assert len(terms) + 1 == g["pauli_strings_including_identity"]


@pytest.mark.parametrize("n_orb,seed", [(2, 5), (3, 6), (4, 7)])
def test_hamiltonian_invariants(n_orb, seed):
    """Real integrals give a real Hermitian operator: real coefficients, an
    even number of Y per string; number and S_z conservation give an even
    X/Y count on alpha (even) qubits and on beta (odd) qubits."""
    I = random_integrals(n_orb, n_orb, seed)
    H = fermion.jw_hamiltonian(I.h1, I.eri)
    n = 2 * n_orb
    alpha = sum(1 << q for q in range(0, n, 2))
    beta = sum(1 << q for q in range(1, n, 2))
    for (x, z), c in H.terms.items():
        assert abs(c.imag) < 1e-12
        assert fermion.popcount(x & z) % 2 == 0
        assert fermion.popcount(x & alpha) % 2 == 0
        assert fermion.popcount(x & beta) % 2 == 0


@pytest.mark.parametrize("n_orb,seed", [(2, 8), (4, 9)])
def test_diagonal_equals_determinant_energies(n_orb, seed):
    """<n| sum_j c_j P_j |n> = <n|H|n> from determinant space, for every
    computational basis state of every electron number."""
    I = random_integrals(n_orb, n_orb, seed)
    n = 2 * n_orb
    c_id, terms = fermion.hamiltonian_terms(fermion.jw_hamiltonian(I.h1, I.eri))
    for ne in range(n + 1):
        sec = fockspace.Sector(n, ne)
        Hd = fockspace.hamiltonian(sec, I.h1, I.eri)
        for j, det in enumerate(sec.dets):
            diag = c_id
            for x, z, c in terms:
                if x == 0:
                    diag += c * (1 - 2 * (fermion.popcount(z & det) & 1))
            assert abs(diag - Hd[j, j]) < 1e-12
