"""Determinant-space (occupation-number) oracle (test only).

Paper: Eq. (1) and Eq. (3)-(4), evaluated without any qubit mapping.  This
module uses only the definition of fermionic operators on occupation-number
states, so it pins the Jordan-Wigner signs of ``fermion.py`` independently:

  |n> = (a+_0)^{n_0} (a+_1)^{n_1} ... |vac>      (lowest index leftmost)
  a_P  |n> = (-1)^{sum_{Q<P} n_Q} |n - e_P>      if n_P = 1, else 0
  a+_P |n> = (-1)^{sum_{Q<P} n_Q} |n + e_P>      if n_P = 0, else 0

Determinants are integers with bit P = occupation of spin-orbital P; the
Hamiltonian is built as a dense matrix on the fixed-electron-number sector.
The UCCSD state is prod_{k=K..1} expm(theta_k (tau_k - tau_k^T)) |HF>.

Closed forms (textbook Slater-Condon rules for a closed-shell determinant,
spatial orbitals, chemist notation):
  E_HF = 2 sum_i h_ii + sum_{ij} [2 (ii|jj) - (ij|ji)] + E_const
  <HF|H a+_a a_i|HF>           = F_ia = h_ia + sum_j [2 (ia|jj) - (ij|ja)]
  <HF|H a+_a a+_b a_i a_j|HF>  = -<ij||ab>,  <ij||ab> = <ij|ab> - <ij|ba>,
                                  <pq|rs> = (pr|qs) delta_spin(p,r) delta_spin(q,s)
(the minus sign: a_i a_j = -a_j a_i and the standard doubly-excited
determinant is a+_a a+_b a_j a_i |HF>).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg

from .uccsd import Excitation, excitations


def _sign_below(n: int, P: int) -> int:
    return -1 if bin(n & ((1 << P) - 1)).count("1") & 1 else 1


def annihilate(P: int, det: int):
    if not (det >> P) & 1:
        return None
    return _sign_below(det, P), det & ~(1 << P)


def create(P: int, det: int):
    if (det >> P) & 1:
        return None
    return _sign_below(det, P), det | (1 << P)


def apply_ops(ops, det: int):
    """ops = [("+"|"-", P), ...] written left-to-right as in the operator
    product; applied right-to-left.  Returns (sign, det) or None."""
    sign = 1
    for kind, P in reversed(ops):
        r = create(P, det) if kind == "+" else annihilate(P, det)
        if r is None:
            return None
        s, det = r
        sign *= s
    return sign, det


class Sector:
    """All determinants of n_qubits spin-orbitals with n_elec electrons
    (``n_elec=None``: every occupation pattern, i.e. the whole Fock space)."""

    def __init__(self, n_qubits: int, n_elec: int | None):
        self.n = n_qubits
        self.ne = n_elec
        if n_elec is None:
            self.dets = list(range(1 << n_qubits))
        else:
            self.dets = []
            for occ in itertools.combinations(range(n_qubits), n_elec):
                d = 0
                for P in occ:
                    d |= 1 << P
                self.dets.append(d)
        self.dets.sort()
        self.index = {d: i for i, d in enumerate(self.dets)}

    @property
    def dim(self) -> int:
        return len(self.dets)

    def hf(self) -> np.ndarray:
        v = np.zeros(self.dim)
        v[self.index[(1 << self.ne) - 1]] = 1.0
        return v

    def operator(self, terms) -> np.ndarray:
        """Dense matrix of sum_t coef_t * (product of ops_t)."""
        m = np.zeros((self.dim, self.dim))
        for j, d in enumerate(self.dets):
            for coef, ops in terms:
                r = apply_ops(ops, d)
                if r is None:
                    continue
                s, d2 = r
                i = self.index.get(d2)
                if i is not None:
                    m[i, j] += s * coef
        return m


def hamiltonian_terms(h1: np.ndarray, eri: np.ndarray):
    n = h1.shape[0]
    terms = []
    for p in range(n):
        for q in range(n):
            if h1[p, q] != 0.0:
                for s in range(2):
                    terms.append((h1[p, q], [("+", 2 * p + s), ("-", 2 * q + s)]))
    for p, q, r, s_ in itertools.product(range(n), repeat=4):
        g = eri[p, q, r, s_]
        if g == 0.0:
            continue
        for s in range(2):
            for t in range(2):
                terms.append((0.5 * g, [("+", 2 * p + s), ("+", 2 * r + t),
                                        ("-", 2 * s_ + t), ("-", 2 * q + s)]))
    return terms


def hamiltonian(sector: Sector, h1, eri, e_const: float = 0.0) -> np.ndarray:
    H = sector.operator(hamiltonian_terms(h1, eri))
    return H + e_const * np.eye(sector.dim)


def excitation_ops(e: Excitation):
    if e.kind == "s":
        return [("+", e.vir[0]), ("-", e.occ[0])]
    return [("+", e.vir[0]), ("+", e.vir[1]), ("-", e.occ[0]), ("-", e.occ[1])]


def uccsd_state(sector: Sector, theta) -> np.ndarray:
    exc = excitations(sector.n, sector.ne)
    psi = sector.hf()
    for k, e in enumerate(exc):
        if theta[k] == 0.0:
            continue
        tau = sector.operator([(1.0, excitation_ops(e))])
        psi = scipy.linalg.expm(theta[k] * (tau - tau.T)) @ psi
    return psi


def uccsd_energy(sector: Sector, H: np.ndarray, theta) -> float:
    psi = uccsd_state(sector, theta)
    return float(psi @ H @ psi)


# ----------------------------------------------------------- closed forms ---

def hf_energy_closed_form(h1, eri, n_elec: int, e_const: float = 0.0) -> float:
    occ = range(n_elec // 2)
    e = e_const + 2.0 * sum(h1[i, i] for i in occ)
    for i in occ:
        for j in occ:
            e += 2.0 * eri[i, i, j, j] - eri[i, j, j, i]
    return float(e)


def fock_closed_form(h1, eri, n_elec: int, i: int, a: int) -> float:
    """Closed-shell Fock matrix element over spatial orbitals i, a."""
    f = h1[i, a]
    for j in range(n_elec // 2):
        f += 2.0 * eri[i, a, j, j] - eri[i, j, j, a]
    return float(f)


def _phys(eri, p: int, q: int, r: int, s: int) -> float:
    """<pq|rs> over spin-orbitals (interleaved)."""
    if p % 2 != r % 2 or q % 2 != s % 2:
        return 0.0
    return float(eri[p // 2, r // 2, q // 2, s // 2])


def hf_gradient_closed_form(h1, eri, n_qubits: int, n_elec: int) -> np.ndarray:
    """dE/dtheta_k at theta = 0, i.e. 2 <HF|H tau_k|HF>, from the closed forms."""
    out = []
    for e in excitations(n_qubits, n_elec):
        if e.kind == "s":
            out.append(2.0 * fock_closed_form(h1, eri, n_elec, e.occ[0] // 2, e.vir[0] // 2))
        else:
            (i, j), (a, b) = e.occ, e.vir
            anti = _phys(eri, i, j, a, b) - _phys(eri, i, j, b, a)
            out.append(-2.0 * anti)
    return np.array(out)


def to_qubit_basis(sector: Sector, m: np.ndarray) -> np.ndarray:
    """Embed a sector matrix in the 2^N qubit space: spin-orbital P is qubit P,
    qubit 0 the most significant bit of the basis index."""
    n = sector.n
    dim = 1 << n

    def qidx(det):
        b = 0
        for P in range(n):
            if (det >> P) & 1:
                b |= 1 << (n - 1 - P)
        return b

    idx = np.array([qidx(d) for d in sector.dets])
    out = np.zeros((dim, dim), dtype=m.dtype)
    out[np.ix_(idx, idx)] = m
    return out
