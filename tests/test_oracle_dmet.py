"""Pins of the oracle's DMET chemical-potential loop (no GPU): DMET is exact
without interaction, particle-hole symmetry fixes mu at half filling, the
embedding space holds the mean-field electrons exactly, and two-electron
fragments make the UCCSD solver exact."""
import numpy as np
import pytest

from oracle import dmet
from workloads import random_lattice


@pytest.mark.parametrize("k,solver", [(1, "fci"), (2, "fci"), (1, "uccsd")])
def test_no_interaction_is_exact(k, solver):
    """U = 0: the embedded ground state is the projected mean-field
    determinant, so at mu = 0 every fragment holds its mean-field electrons
    and the loop stops at mu = 0."""
    lat = random_lattice(8, k, 8, 5, U=0.0)
    r = dmet.dmet(lat, solver)
    assert r.status == 1 and abs(r.mu) < 1e-6
    occ = 2.0 * np.diag(dmet.mean_field_density(lat))
    want = occ.reshape(lat.n_frags, k).sum(axis=1)
    assert np.max(np.abs(r.n_frag - want)) < 1e-6


@pytest.mark.parametrize("n_sites,ring", [(8, False), (6, True)])
def test_half_filling_particle_hole_symmetry(n_sites, ring):
    """Uniform bipartite chain or ring (6 sites: its Fermi level has a gap) at
    half filling: particle-hole symmetry maps the embedded problem at mu to
    the one at U - mu, so mu* = U/2 and every fragment holds k electrons."""
    lat = random_lattice(n_sites, 2, n_sites, 1, eps_amp=0.0, U=4.0, ring=ring)
    r = dmet.dmet(lat, "fci", mu_lo=0.0, mu_hi=4.0)
    assert r.status == 1 and abs(r.mu - 2.0) < 1e-6
    assert np.max(np.abs(r.n_frag - 2.0)) < 1e-6


@pytest.mark.parametrize("k", [1, 2, 4])
def test_embedding_space_holds_the_mean_field_electrons(k):
    """The embedding orbitals are orthonormal, contain the fragment sites, and
    the mean-field density restricted to them is diag(1 x k, 0 x k)."""
    lat = random_lattice(8, k, 8, 3)
    D = dmet.mean_field_density(lat)
    for f in range(lat.n_frags):
        N = dmet.embedding_basis(lat, D, f)
        assert np.max(np.abs(N.T @ N - np.eye(2 * k))) < 1e-12
        assert np.max(np.abs(N.T @ D @ N - np.diag([1.0] * k + [0.0] * k))) < 1e-12
        F = slice(f * k, (f + 1) * k)
        P = N @ N.T
        assert np.max(np.abs(P[F, F] - np.eye(k))) < 1e-12


def test_two_electron_fragments_uccsd_equals_exact():
    """Fragments of one site embed two electrons in two orbitals, where UCCSD
    is exact: the UCCSD loop reaches the exact-solver loop's mu and energies."""
    lat = random_lattice(8, 1, 8, 5, U=4.0)
    ru = dmet.dmet(lat, "uccsd", mu_lo=0.0, mu_hi=4.0)
    rf = dmet.dmet(lat, "fci", mu_lo=0.0, mu_hi=4.0)
    assert ru.status == rf.status == 1
    assert abs(ru.mu - rf.mu) < 1e-6
    assert abs(ru.e_frag.sum() - rf.e_frag.sum()) < 1e-6


def test_degenerate_fermi_level_is_an_error():
    """The uniform 8-site ring at half filling has two orbitals at the Fermi
    level: no unique mean-field determinant."""
    with pytest.raises(ValueError):
        dmet.mean_field_density(random_lattice(8, 2, 8, 1, eps_amp=0.0, ring=True))


@pytest.mark.parametrize("k,solver", [(1, "fci"), (2, "fci"), (2, "uccsd")])
def test_fragment_energies_add_up_to_the_mean_field_energy(k, solver):
    """U = 0, mu = 0: the embedded ground state is the projected mean-field
    determinant, so the fragment energies (democratic partitioning of the
    one-body energy) add up to the mean-field energy 2 Tr(h D)."""
    lat = random_lattice(8, k, 8, 5, U=0.0)
    D = dmet.mean_field_density(lat)
    total = 0.0
    for f in range(lat.n_frags):
        N = dmet.embedding_basis(lat, D, f)
        _, ef, _ = dmet.solve_fragment(lat, dmet.embedded_problem(lat, N, f, 0.0), solver)
        total += ef
    assert abs(total - 2.0 * np.trace(lat.h @ D)) < 1e-12
