"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays them out: it holds none of the
method's arithmetic (no fermion algebra, no Pauli strings, no gates, no MPS).
Both the CPU oracle and the GPU path take their inputs from here, and nothing
else is shared between them.

Stand-in for the paper's molecules (H chains, H2, LiH, H2O, (H2)3, C18; Sec. IV)
whose integrals are not available: real symmetric one-electron integrals and
real two-electron integrals with the 8-fold permutation symmetry of real
orbitals, in chemist notation (pq|rs), which is the form the second-quantised
Hamiltonian of Eq. (1) consumes.

Draw recipe (numpy ``Generator(PCG64(seed))``):
  1. h: upper triangle row-major (p <= q), each N(0, sd=0.5), mirrored.
  2. h[p, p] += linspace(-2, 0, n_orb)[p]  (aufbau order = index order).
  3. eri: one N(0, sd=0.1) value per canonical quadruple in the nested loop
     p >= q, r >= s, pair(p,q) >= pair(r,s) with pair(p,q) = p(p+1)/2 + q,
     written to all 8 symmetric index permutations.
  4. theta: a separate generator, U[-0.1, 0.1] per UCCSD parameter.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "Integrals",
    "random_integrals",
    "random_theta",
    "CONFIGS",
    "WorkloadConfig",
    "h2_like_integrals",
    "serving_stream",
    "ServingRequest",
    "n_uccsd_params",
    "Lattice",
    "random_lattice",
]


@dataclasses.dataclass(frozen=True)
class Integrals:
    """Molecular-orbital integrals of a closed-shell problem."""

    n_orb: int
    n_elec: int
    h1: np.ndarray  # (n_orb, n_orb) float64, symmetric
    eri: np.ndarray  # (n_orb,)*4 float64, chemist notation (pq|rs), 8-fold symmetric
    e_const: float = 0.0

    @property
    def n_qubits(self) -> int:
        return 2 * self.n_orb


def _pair(p: int, q: int) -> int:
    return p * (p + 1) // 2 + q


def _fill8(eri: np.ndarray, p: int, q: int, r: int, s: int, v: float) -> None:
    for a, b, c, d in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                       (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
        eri[a, b, c, d] = v


def random_integrals(n_orb: int, n_elec: int, seed: int,
                     h_sd: float = 0.5, eri_sd: float = 0.1,
                     mu: float = 0.0, n_frag_orb: int = 0) -> Integrals:
    """Draw the synthetic integrals described in the module docstring.

    ``mu`` and ``n_frag_orb`` add a DMET-style chemical-potential shift
    ``-mu`` to the diagonal of the first ``n_frag_orb`` (fragment) orbitals.
    """
    if n_orb < 1 or n_elec < 0 or n_elec > 2 * n_orb:
        raise ValueError("bad orbital/electron counts")
    rng = np.random.Generator(np.random.PCG64(seed))
    h = np.zeros((n_orb, n_orb))
    for p in range(n_orb):
        for q in range(p, n_orb):
            v = rng.normal(0.0, h_sd)
            h[p, q] = v
            h[q, p] = v
    h[np.diag_indices(n_orb)] += np.linspace(-2.0, 0.0, n_orb)
    if n_frag_orb:
        for p in range(min(n_frag_orb, n_orb)):
            h[p, p] -= mu
    eri = np.zeros((n_orb,) * 4)
    for p in range(n_orb):
        for q in range(p + 1):
            for r in range(n_orb):
                for s in range(r + 1):
                    if _pair(p, q) >= _pair(r, s):
                        _fill8(eri, p, q, r, s, rng.normal(0.0, eri_sd))
    return Integrals(n_orb, n_elec, h, eri, 0.0)


def h2_like_integrals(seed: int = 7) -> Integrals:
    """Two-orbital, two-electron integrals with the zero pattern of H2 in a
    minimal basis (D-infinity-h symmetry: the bonding and antibonding orbitals
    belong to different irreps).  Only h00, h11, (00|00), (11|11), (00|11) and
    (01|01) with their symmetric copies are nonzero.  Values are random."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = np.zeros((2, 2))
    h[0, 0] = -1.25 + 0.1 * rng.normal()
    h[1, 1] = -0.47 + 0.1 * rng.normal()
    eri = np.zeros((2, 2, 2, 2))
    _fill8(eri, 0, 0, 0, 0, 0.67 + 0.05 * rng.normal())
    _fill8(eri, 1, 1, 1, 1, 0.70 + 0.05 * rng.normal())
    _fill8(eri, 0, 0, 1, 1, 0.66 + 0.05 * rng.normal())
    _fill8(eri, 0, 1, 0, 1, 0.18 + 0.02 * rng.normal())
    return Integrals(2, 2, h, eri, 0.0)


def n_uccsd_params(n_orb: int, n_elec: int) -> int:
    """Number of spin-conserving singles plus doubles over interleaved
    spin-orbitals (counting only; used to size theta)."""
    nq = 2 * n_orb
    occ = list(range(n_elec))
    vir = list(range(n_elec, nq))
    ns = sum(1 for i in occ for a in vir if i % 2 == a % 2)
    nd = 0
    for ii, i in enumerate(occ):
        for j in occ[ii + 1:]:
            for ia, a in enumerate(vir):
                for b in vir[ia + 1:]:
                    if (i % 2) + (j % 2) == (a % 2) + (b % 2):
                        nd += 1
    return ns + nd


def random_theta(n_params: int, seed: int, amp: float = 0.1) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-amp, amp, size=n_params)


@dataclasses.dataclass(frozen=True)
class WorkloadConfig:
    name: str
    n_orb: int
    n_elec: int
    int_seed: int
    theta_seed: int
    max_bond: int

    def integrals(self) -> Integrals:
        return random_integrals(self.n_orb, self.n_elec, self.int_seed)

    def theta(self) -> np.ndarray:
        return random_theta(n_uccsd_params(self.n_orb, self.n_elec), self.theta_seed)


CONFIGS = {
    "q8_d16": WorkloadConfig("q8_d16", 4, 4, 1001, 1002, 16),
    "q16_d64": WorkloadConfig("q16_d64", 8, 8, 2001, 2002, 64),
    "q24_d128": WorkloadConfig("q24_d128", 12, 12, 3001, 3002, 128),
    "q24_d256": WorkloadConfig("q24_d256", 12, 12, 3001, 3002, 256),
}


@dataclasses.dataclass(frozen=True)
class ServingRequest:
    index: int
    n_frag_orb: int  # k: fragment orbitals; embedded problem has 2k orbitals
    max_bond: int
    mu: float
    arrival_gap: float  # exponential inter-arrival in units of 1/rate

    @property
    def n_orb(self) -> int:
        return 2 * self.n_frag_orb

    @property
    def n_elec(self) -> int:
        return 2 * self.n_frag_orb

    def integrals(self) -> Integrals:
        return random_integrals(self.n_orb, self.n_elec, 500000 + self.index,
                                mu=self.mu, n_frag_orb=self.n_frag_orb)

    def theta(self) -> np.ndarray:
        return random_theta(n_uccsd_params(self.n_orb, self.n_elec), 600000 + self.index)


def serving_stream(n: int, seed: int = 5000, k_range=(2, 8),
                   bonds=(32, 64, 128, 256)) -> list[ServingRequest]:
    """DMET-style fragment solve requests: fragment size k ~ U{k_range},
    D ~ U{bonds}, mu ~ U[-0.5, 0.5] (its own generator per request), and
    unit-rate exponential inter-arrival gaps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for r in range(n):
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        d = int(bonds[int(rng.integers(0, len(bonds)))])
        gap = float(rng.exponential(1.0))
        mu = float(np.random.Generator(np.random.PCG64(700000 + r)).uniform(-0.5, 0.5))
        out.append(ServingRequest(r, k, d, mu, gap))
    return out


@dataclasses.dataclass(frozen=True)
class Lattice:
    """A one-dimensional Hubbard-type lattice split into fragments: one-body
    matrix h (hopping -t between neighbouring sites, on-site energies on the
    diagonal), on-site repulsion U, n_elec electrons (even), fragments of
    frag_size consecutive sites.  Stand-in for the lattice one-body models
    around a DMET fragment (Sec. III-B); the paper's molecules are not
    available."""

    n_sites: int
    frag_size: int
    n_elec: int
    h: np.ndarray  # (n_sites, n_sites) float64, symmetric
    U: float

    @property
    def n_frags(self) -> int:
        return self.n_sites // self.frag_size


def random_lattice(n_sites: int, frag_size: int, n_elec: int, seed: int, t: float = 1.0,
                   eps_amp: float = 0.5, U: float = 4.0, ring: bool = False) -> Lattice:
    """On-site energies U[-eps_amp, eps_amp] (numpy PCG64(seed)), hopping -t on
    the chain (and between the ends when ring)."""
    if n_sites % frag_size or n_elec % 2 or not 0 < n_elec < 2 * n_sites:
        raise ValueError("bad lattice shape")
    rng = np.random.Generator(np.random.PCG64(seed))
    h = np.diag(rng.uniform(-eps_amp, eps_amp, n_sites)) if eps_amp > 0 else np.zeros((n_sites, n_sites))
    for i in range(n_sites - 1):
        h[i, i + 1] = h[i + 1, i] = -t
    if ring and n_sites > 2:
        h[0, n_sites - 1] = h[n_sites - 1, 0] = -t
    return Lattice(n_sites, frag_size, n_elec, h, float(U))
