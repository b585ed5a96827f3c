"""Pins for the CPU MPS oracle: at full bond dimension it must reproduce the
state vector amplitude by amplitude; the update must keep right-canonical
form and unit norm; truncated states must obey the variational bound; the
environment-based expectations must match dense expectations."""
import numpy as np
import pytest

from oracle import exact, fermion, mps as om, statevector as sv, uccsd
from workloads import random_integrals, random_theta


def _setup(n_orb, n_elec, seed, amp=0.3):
    I = random_integrals(n_orb, n_elec, seed)
    c_id, terms = fermion.hamiltonian_terms(fermion.jw_hamiltonian(I.h1, I.eri))
    n = 2 * n_orb
    rots, gates = uccsd.compile_fused(n, n_elec)
    th = random_theta(len(uccsd.excitations(n, n_elec)), seed + 1, amp=amp)
    return n, c_id, terms, rots, gates, uccsd.rotation_angles(rots, th)


@pytest.mark.parametrize("n_orb,n_elec,seed", [(2, 2, 81), (3, 4, 82), (4, 4, 83)])
def test_full_bond_mps_equals_statevector(n_orb, n_elec, seed):
    n, c_id, terms, rots, gates, phis = _setup(n_orb, n_elec, seed)
    occ = uccsd.hf_occupation(n, n_elec)
    m = om.MPS(occ, 1 << (n // 2))
    for g in gates:
        m.apply_gate(g.site, g.matrix(phis))
        assert abs(np.sum(m.lam[g.site] ** 2) - 1) < 1e-13
    assert m.discarded < 1e-20
    psi = sv.evolve(n, occ, rots, phis)
    assert np.max(np.abs(m.to_statevector() - psi)) < 1e-12
    assert m.right_canonical_error() < 1e-12
    e_mps, imag = om.energy(m, c_id, terms)
    assert abs(e_mps - sv.energy(sv.PauliApplier(n), c_id, terms, psi)) < 1e-12
    assert imag < 1e-12


def test_right_canonical_after_every_gate():
    n, c_id, terms, rots, gates, phis = _setup(3, 2, 91)
    m = om.MPS(uccsd.hf_occupation(n, 2), 8)
    for g in gates:
        m.apply_gate(g.site, g.matrix(phis))
        for s in (g.site, g.site + 1):
            if s == 0:
                continue
            B = m.B[s]
            G = sum(B[:, i, :] @ B[:, i, :].conj().T for i in range(2))
            assert np.max(np.abs(G - np.eye(G.shape[0]))) < 1e-12
        assert abs(m.norm2() - 1) < 1e-12


def test_expectations_match_dense_on_random_mps():
    """Environment sweeps vs <psi|P|psi> on the contracted vector, for every
    Pauli string on 5 qubits, on a random (non-canonical) MPS."""
    rng = np.random.default_rng(3)
    n = 5
    m = om.MPS([0] * n, 4)
    dims = [1, 2, 4, 4, 2, 1]
    m.B = [rng.normal(size=(dims[k], 2, dims[k + 1])) + 1j * rng.normal(size=(dims[k], 2, dims[k + 1]))
           for k in range(n)]
    psi = m.to_statevector()
    strings = [(x, z) for x in range(1 << n) for z in range(1 << n)]
    ev = om.pauli_expectations(m, strings)
    nrm = np.vdot(psi, psi).real
    for (x, z), e in zip(strings, ev):
        want = np.vdot(psi, fermion.pauli_dense(x, z, n) @ psi) / nrm
        assert abs(e - want) < 1e-12


@pytest.mark.parametrize("D", [2, 3, 4, 6])
def test_truncated_mps_is_variational(D):
    n, c_id, terms, rots, gates, phis = _setup(4, 4, 101, amp=0.5)
    e0 = exact.ground_energy(n, c_id, terms)
    m = om.run_circuit(n, uccsd.hf_occupation(n, 4), gates, phis, D)
    assert m.max_chi <= D
    assert m.discarded > 0
    e, _ = om.energy(m, c_id, terms)
    assert e >= e0 - 1e-12


def test_hartree_fock_at_any_bond_dimension():
    """At theta = 0 every ladder intermediate has Schmidt rank <= 2, so even
    D = 2 reproduces E_HF exactly."""
    n, c_id, terms, rots, gates, _ = _setup(4, 4, 111)
    phis = np.zeros(len(rots))
    m = om.run_circuit(n, uccsd.hf_occupation(n, 4), gates, phis, 2)
    e, _ = om.energy(m, c_id, terms)
    psi = sv.basis_state(n, uccsd.hf_occupation(n, 4))
    assert abs(e - sv.energy(sv.PauliApplier(n), c_id, terms, psi)) < 1e-12
    assert m.discarded < 1e-20
