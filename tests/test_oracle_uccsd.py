"""Pins for the oracle's UCCSD excitations, rotations and gate compile."""
import json
import math
import os

import numpy as np
import pytest

from oracle import fermion, statevector as sv, uccsd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _closed_form_counts(n_orb, n_elec):
    """Counts from combinatorics over spatial orbitals and spin-orbital
    indices alone (no operator algebra)."""
    oa = n_elec // 2
    va = n_orb - oa
    singles = 2 * oa * va
    doubles = 2 * math.comb(oa, 2) * math.comb(va, 2) + oa * oa * va * va
    nq = 2 * n_orb
    occ = range(n_elec)
    vir = range(n_elec, nq)
    gates = 0
    for i in occ:
        for a in vir:
            if i % 2 == a % 2:
                gates += 2 * (2 * (a - i) - 1)  # 2 strings, support i..a
    for i in occ:
        for j in occ:
            if j <= i:
                continue
            for a in vir:
                for b in vir:
                    if b <= a or (i % 2) + (j % 2) != (a % 2) + (b % 2):
                        continue
                    gates += 8 * (2 * (b - i) - 1)  # 8 strings, support i..b
    return singles, doubles, 2 * singles + 8 * doubles, gates


@pytest.mark.parametrize("n_orb", [2, 3, 4, 5, 6, 8])
def test_counts_match_closed_forms(n_orb):
    n_elec = n_orb
    s, d, nrot, ngates = _closed_form_counts(n_orb, n_elec)
    exc = uccsd.excitations(2 * n_orb, n_elec)
    assert sum(e.kind == "s" for e in exc) == s
    assert sum(e.kind == "d" for e in exc) == d
    if n_orb <= 6:
        rots, gates = uccsd.compile_fused(2 * n_orb, n_elec)
        assert len(rots) == nrot
        assert len(gates) == ngates


def test_h2_ansatz_gate_count_matches_paper():
    with open(os.path.join(GOLDEN, "h2_paper_counts.json")) as f:
        g = json.load(f)
    rots, native = uccsd.compile_native(g["n_qubits"], g["n_elec"])
    exc = uccsd.excitations(g["n_qubits"], g["n_elec"])
    # The paper's H2 ansatz keeps the one double excitation (its singles
    # vanish by symmetry).
    dbl = [k for k, e in enumerate(exc) if e.kind == "d"]
    assert len(dbl) == 1
    n_native = sum(len(uccsd.native_rotation_gates(r, m)) for m, r in enumerate(rots)
                   if r.param == dbl[0])
    assert n_native == g["ansatz_native_gates"]
    assert sum(uccsd.hf_occupation(4, 2)) == g["hf_x_gates"]


@pytest.mark.parametrize("n_orb", [2, 3, 4])
def test_generators_are_commuting_real_pauli_sums(n_orb):
    n = 2 * n_orb
    for e in uccsd.excitations(n, n_orb):
        strings = uccsd.generator_strings(e)
        want = 0.5 if e.kind == "s" else 0.125
        assert len(strings) == (2 if e.kind == "s" else 8)
        for x, z, c in strings:
            assert abs(abs(c) - want) < 1e-15
        for x1, z1, _ in strings:
            for x2, z2, _ in strings:
                ph, _, _ = fermion.pauli_mul(x1, z1, x2, z2)
                ph2, _, _ = fermion.pauli_mul(x2, z2, x1, z1)
                assert ph == ph2


def _random_state(n, seed):
    rng = np.random.default_rng(seed)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return psi / np.linalg.norm(psi)


@pytest.mark.parametrize("n_orb", [2, 3])
def test_native_and_fused_compiles_reproduce_rotations(n_orb):
    """Each compiled rotation, applied gate by gate, equals
    cos(phi/2) - i sin(phi/2) P on an arbitrary state."""
    n = 2 * n_orb
    rots = uccsd.rotations(n, n_orb)
    pa = sv.PauliApplier(n)
    rng = np.random.default_rng(2)
    for m, r in enumerate(rots):
        phi = rng.uniform(-3, 3)
        phis = np.zeros(len(rots))
        phis[m] = phi
        psi0 = _random_state(n, m)
        want = sv.apply_rotation(pa, r, phi, psi0)
        psi = psi0
        for g in uccsd.native_rotation_gates(r, m):
            mat = uccsd.rz(phi) if g.name == "RZ" else g.matrix
            if len(g.qubits) == 1:
                psi = sv.apply_one_site(psi, n, g.qubits[0], mat)
            else:
                psi = sv.apply_two_site(psi, n, g.qubits[0], mat)
        assert np.allclose(psi, want, atol=1e-13)
        fused = uccsd.fused_rotation_gates(r, m)
        lo, hi = r.support()
        assert len(fused) == 2 * (hi - lo) - 1
        psi = psi0
        for g in fused:
            assert lo <= g.site < hi
            psi = sv.apply_two_site(psi, n, g.site, g.matrix(phis))
        assert np.allclose(psi, want, atol=1e-13)


def test_fused_gates_are_unitary():
    rots, gates = uccsd.compile_fused(8, 4)
    phis = np.linspace(-1, 1, len(rots))
    for g in gates:
        u = g.matrix(phis)
        assert np.allclose(u @ u.conj().T, np.eye(4), atol=1e-14)
