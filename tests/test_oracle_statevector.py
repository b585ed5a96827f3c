"""Pins for the state-vector oracle: determinant-space equality (no Pauli
code on that side), textbook closed forms, gradient identities, norm and the
variational bound."""
import numpy as np
import pytest

from oracle import exact, fermion, fockspace, statevector as sv, uccsd
from workloads import h2_like_integrals, random_integrals, random_theta


def _problem(n_orb, n_elec, seed):
    I = random_integrals(n_orb, n_elec, seed)
    c_id, terms = fermion.hamiltonian_terms(fermion.jw_hamiltonian(I.h1, I.eri))
    rots = uccsd.rotations(2 * n_orb, n_elec)
    return I, c_id, terms, rots


@pytest.mark.parametrize("n_orb,n_elec,seed", [(2, 2, 21), (3, 2, 22), (3, 4, 23), (4, 4, 24), (5, 4, 25)])
def test_energy_equals_determinant_space(n_orb, n_elec, seed):
    I, c_id, terms, rots = _problem(n_orb, n_elec, seed)
    n = 2 * n_orb
    th = random_theta(len(uccsd.excitations(n, n_elec)), seed + 100, amp=0.4)
    e_sv = sv.vqe_energy(n, n_elec, c_id, terms, rots, th)
    sec = fockspace.Sector(n, n_elec)
    e_fs = fockspace.uccsd_energy(sec, fockspace.hamiltonian(sec, I.h1, I.eri), th)
    assert abs(e_sv - e_fs) < 1e-12


@pytest.mark.parametrize("n_orb,n_elec,seed", [(2, 2, 31), (4, 4, 32), (6, 6, 33)])
def test_theta_zero_is_hartree_fock_closed_form(n_orb, n_elec, seed):
    I, c_id, terms, rots = _problem(n_orb, n_elec, seed)
    n = 2 * n_orb
    th = np.zeros(len(uccsd.excitations(n, n_elec)))
    e = sv.vqe_energy(n, n_elec, c_id, terms, rots, th)
    assert abs(e - fockspace.hf_energy_closed_form(I.h1, I.eri, n_elec)) < 1e-12


@pytest.mark.parametrize("th2", [0.3, -0.7, 1.1])
def test_two_level_closed_form(th2):
    """Two orbitals, two electrons, singles at zero: the state stays in
    span{HF, doubly excited} and
    E = cos^2 H00 + sin^2 HDD - sin(2 theta) K01."""
    I = h2_like_integrals()
    c_id, terms = fermion.hamiltonian_terms(fermion.jw_hamiltonian(I.h1, I.eri))
    rots = uccsd.rotations(4, 2)
    e = sv.vqe_energy(4, 2, c_id, terms, rots, np.array([0.0, 0.0, th2]))
    H00 = 2 * I.h1[0, 0] + I.eri[0, 0, 0, 0]
    HDD = 2 * I.h1[1, 1] + I.eri[1, 1, 1, 1]
    K = I.eri[0, 1, 0, 1]
    want = np.cos(th2) ** 2 * H00 + np.sin(th2) ** 2 * HDD - np.sin(2 * th2) * K
    assert abs(e - want) < 1e-12
    # its minimum over theta is the lowest eigenvalue of the 2x2 CI matrix
    grid = np.linspace(-np.pi / 2, np.pi / 2, 20001)
    emin = np.min(np.cos(grid) ** 2 * H00 + np.sin(grid) ** 2 * HDD - np.sin(2 * grid) * K)
    lam = np.linalg.eigvalsh(np.array([[H00, K], [K, HDD]]))[0]
    assert abs(emin - lam) < 1e-6


@pytest.mark.parametrize("n_orb,n_elec,seed", [(2, 2, 41), (3, 2, 42), (4, 4, 43)])
def test_gradient_at_zero_closed_form(n_orb, n_elec, seed):
    I, c_id, terms, rots = _problem(n_orb, n_elec, seed)
    n = 2 * n_orb
    th = np.zeros(len(uccsd.excitations(n, n_elec)))
    g, _, _ = sv.grad_adjoint(n, n_elec, c_id, terms, rots, th)
    g_cf = fockspace.hf_gradient_closed_form(I.h1, I.eri, n, n_elec)
    assert np.max(np.abs(g - g_cf)) < 1e-10


def test_gradient_rules_agree():
    """Per-rotation two-term shift == adjoint (exact) and == central finite
    difference of the energy (h = 1e-5)."""
    I, c_id, terms, rots = _problem(3, 4, 51)
    n = 6
    npar = len(uccsd.excitations(n, 4))
    th = random_theta(npar, 52, amp=0.3)
    g_ad, dphi_ad, _ = sv.grad_adjoint(n, 4, c_id, terms, rots, th)
    g_ps, dphi_ps = sv.grad_paramshift(n, 4, c_id, terms, rots, th)
    assert np.max(np.abs(dphi_ad - dphi_ps)) < 1e-12
    assert np.max(np.abs(g_ad - g_ps)) < 1e-12
    h = 1e-5
    for k in range(npar):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (sv.vqe_energy(n, 4, c_id, terms, rots, tp) - sv.vqe_energy(n, 4, c_id, terms, rots, tm)) / (2 * h)
        assert abs(fd - g_ad[k]) < 1e-7


@pytest.mark.parametrize("n_orb,n_elec", [(2, 2), (3, 2), (3, 4), (4, 4)])
def test_excitation_generators_have_spectrum_0_pm1(n_orb, n_elec):
    """G_k = sum_m c_m P_m of every UCCSD parameter (its rotations combined)
    has eigenvalues in {0, +-1}: built densely from Kronecker products of the
    Pauli matrices, not through the oracle's Pauli code."""
    n = 2 * n_orb
    P = {(0, 0): np.eye(2), (1, 0): np.array([[0, 1], [1, 0]]), (1, 1): np.array([[0, -1j], [1j, 0]]),
         (0, 1): np.diag([1.0, -1.0])}
    rots = uccsd.rotations(n, n_elec)
    for k in range(len(uccsd.excitations(n, n_elec))):
        G = np.zeros((1 << n, 1 << n), dtype=complex)
        for r in rots:
            if r.param != k:
                continue
            M = np.ones((1, 1))
            for q in reversed(range(n)):  # qubit 0 is the least significant bit of the index
                M = np.kron(M, P[((r.x >> q) & 1, (r.z >> q) & 1)])
            G += r.c * M
        ev = np.linalg.eigvalsh(G)
        assert np.all(np.min(np.abs(ev[:, None] - np.array([-1.0, 0.0, 1.0])[None, :]), axis=1) < 1e-12), k


def test_fourterm_rule_equals_adjoint():
    """The per-parameter four-term shift rule equals the exact gradient."""
    for n_orb, n_elec, seed in ((2, 2, 71), (3, 4, 72)):
        I, c_id, terms, rots = _problem(n_orb, n_elec, seed)
        n = 2 * n_orb
        th = random_theta(len(uccsd.excitations(n, n_elec)), seed + 1, amp=0.4)
        g_ad, _, _ = sv.grad_adjoint(n, n_elec, c_id, terms, rots, th)
        g_4 = sv.grad_fourterm(n, n_elec, c_id, terms, rots, th)
        assert np.max(np.abs(g_ad - g_4)) < 1e-11


@pytest.mark.parametrize("n_orb,seed", [(2, 61), (3, 62), (4, 63)])
def test_norm_and_variational_bound(n_orb, seed):
    I, c_id, terms, rots = _problem(n_orb, n_orb, seed)
    n = 2 * n_orb
    e0 = exact.ground_energy(n, c_id, terms)
    rng = np.random.default_rng(seed)
    for _ in range(3):
        th = rng.uniform(-1, 1, len(uccsd.excitations(n, n_orb)))
        phis = uccsd.rotation_angles(rots, th)
        psi = sv.evolve(n, uccsd.hf_occupation(n, n_orb), rots, phis)
        assert abs(np.linalg.norm(psi) - 1) < 1e-13
        assert sv.energy(sv.PauliApplier(n), c_id, terms, psi) >= e0 - 1e-12


def test_brute_force_matches_determinant_space_spectrum():
    """The full-space ground energy is the minimum over all electron-number
    sectors of the determinant-space Hamiltonian."""
    I, c_id, terms, _ = _problem(2, 2, 71)
    e0 = exact.ground_energy(4, c_id, terms)
    best = min(np.linalg.eigvalsh(fockspace.hamiltonian(fockspace.Sector(4, ne), I.h1, I.eri))[0]
               for ne in range(5))
    assert abs(e0 - best) < 1e-12
