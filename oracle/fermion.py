"""Pauli-string algebra and the Jordan-Wigner Hamiltonian (oracle, test only).

Paper: Sec. II-A, Eq. (1) (second-quantised electronic Hamiltonian) and
Eq. (2) (energy as a weighted sum of Pauli-string expectations after the
Jordan-Wigner or Bravyi-Kitaev map; Jordan-Wigner is the one used, Sec. III-C).

Conventions
-----------
* A Pauli string on N qubits is a pair of bit masks (x, z); bit k refers to
  qubit k.  Qubit k carries X if only x_k is set, Z if only z_k is set, Y if
  both are set, identity otherwise.
* With that labelling, sigma(x, z) = i^{|x & z|} X^x Z^z per qubit, because
  Y = i X Z.  Moving Z^{z1} to the right of X^{x2} costs (-1)^{|z1 & x2|},
  hence
      sigma(x1,z1) sigma(x2,z2)
          = i^{|x1&z1| + |x2&z2| + 2|z1&x2| - |x3&z3|} sigma(x3, z3),
  with x3 = x1 ^ x2, z3 = z1 ^ z2 (exponent taken mod 4).
* Jordan-Wigner: spin-orbital P maps to qubit P; |1> = occupied;
      a_P^dag = (prod_{Q<P} Z_Q) (X_P - i Y_P)/2,
      a_P     = (prod_{Q<P} Z_Q) (X_P + i Y_P)/2.
* Spin-orbitals are interleaved: P = 2p + sigma (sigma = 0 alpha, 1 beta).
* Hamiltonian (chemist notation, the textbook form of Eq. 1):
      H = E_const + sum_{pq,s} h_pq a+_{ps} a_{qs}
          + 1/2 sum_{pqrs,s,t} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

_I_POW = (1.0 + 0.0j, 1.0j, -1.0 + 0.0j, -1.0j)

DROP_TOL = 1e-12


def popcount(v: int) -> int:
    return bin(v).count("1")


def pauli_mul(x1: int, z1: int, x2: int, z2: int):
    """Product of two Pauli strings: returns (phase, x3, z3)."""
    x3 = x1 ^ x2
    z3 = z1 ^ z2
    e = popcount(x1 & z1) + popcount(x2 & z2) + 2 * popcount(z1 & x2) - popcount(x3 & z3)
    return _I_POW[e % 4], x3, z3


class PauliSum:
    """A linear combination of Pauli strings: {(x, z): complex coefficient}."""

    __slots__ = ("terms",)

    def __init__(self, terms=None):
        self.terms = defaultdict(complex)
        if terms:
            for k, v in terms.items():
                self.terms[k] += v

    def copy(self) -> "PauliSum":
        return PauliSum(dict(self.terms))

    def __add__(self, other: "PauliSum") -> "PauliSum":
        out = self.copy()
        for k, v in other.terms.items():
            out.terms[k] += v
        return out

    def __sub__(self, other: "PauliSum") -> "PauliSum":
        return self + other.scale(-1.0)

    def scale(self, c: complex) -> "PauliSum":
        return PauliSum({k: c * v for k, v in self.terms.items()})

    def __mul__(self, other: "PauliSum") -> "PauliSum":
        out = PauliSum()
        acc = out.terms
        for (x1, z1), c1 in self.terms.items():
            for (x2, z2), c2 in other.terms.items():
                ph, x3, z3 = pauli_mul(x1, z1, x2, z2)
                acc[(x3, z3)] += ph * c1 * c2
        return out

    def dagger(self) -> "PauliSum":
        # Every Pauli string is Hermitian, so only the coefficients conjugate.
        return PauliSum({k: np.conj(v) for k, v in self.terms.items()})

    def pruned(self, tol: float = DROP_TOL) -> "PauliSum":
        return PauliSum({k: v for k, v in self.terms.items() if abs(v) >= tol})


def jw_create(P: int) -> PauliSum:
    zmask = (1 << P) - 1
    b = 1 << P
    return PauliSum({(b, zmask): 0.5, (b, zmask | b): -0.5j})


def jw_annihilate(P: int) -> PauliSum:
    zmask = (1 << P) - 1
    b = 1 << P
    return PauliSum({(b, zmask): 0.5, (b, zmask | b): 0.5j})


def spin_orbital(p: int, sigma: int) -> int:
    return 2 * p + sigma


def jw_hamiltonian(h1: np.ndarray, eri: np.ndarray, e_const: float = 0.0) -> PauliSum:
    """Jordan-Wigner image of the chemist-notation Hamiltonian (Eq. 1)."""
    n = h1.shape[0]
    nq = 2 * n
    cre = [jw_create(P) for P in range(nq)]
    ann = [jw_annihilate(P) for P in range(nq)]
    H = PauliSum({(0, 0): complex(e_const)})
    acc = H.terms
    # one-body part
    for p in range(n):
        for q in range(n):
            if h1[p, q] == 0.0:
                continue
            for s in range(2):
                term = cre[spin_orbital(p, s)] * ann[spin_orbital(q, s)]
                for k, v in term.terms.items():
                    acc[k] += h1[p, q] * v
    # two-body part: 1/2 (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}
    pair_cre = {}
    pair_ann = {}
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for s_ in range(n):
                    g = eri[p, q, r, s_]
                    if g == 0.0:
                        continue
                    for s in range(2):
                        for t in range(2):
                            P, Q = spin_orbital(p, s), spin_orbital(q, s)
                            R, S = spin_orbital(r, t), spin_orbital(s_, t)
                            if P == R or Q == S:
                                continue  # a+_P a+_P = 0, a_S a_S = 0
                            kc = (P, R)
                            if kc not in pair_cre:
                                pair_cre[kc] = cre[P] * cre[R]
                            ka = (S, Q)
                            if ka not in pair_ann:
                                pair_ann[ka] = ann[S] * ann[Q]
                            term = pair_cre[kc] * pair_ann[ka]
                            for k, v in term.terms.items():
                                acc[k] += 0.5 * g * v
    return H.pruned()


def hamiltonian_terms(H: PauliSum):
    """Split a Hermitian PauliSum into (identity coefficient, sorted list of
    (x, z, c)) with real c, ascending by (x, z).  Raises if a coefficient has
    an imaginary part above the drop tolerance."""
    c_id = 0.0
    out = []
    for (x, z), c in H.terms.items():
        if abs(c.imag) > DROP_TOL:
            raise ValueError(f"non-real Pauli coefficient {c} on {(x, z)}")
        if (x, z) == (0, 0):
            c_id = c.real
        elif abs(c.real) >= DROP_TOL:
            out.append((x, z, c.real))
    out.sort(key=lambda t: (t[0], t[1]))
    return c_id, out


def pauli_label(x: int, z: int, n: int) -> str:
    """Qubit 0 first."""
    s = []
    for k in range(n):
        b = ((x >> k) & 1, (z >> k) & 1)
        s.append({(0, 0): "I", (1, 0): "X", (0, 1): "Z", (1, 1): "Y"}[b])
    return "".join(s)


# --- dense matrices (small N only): an independent check of the algebra ----

_PAULI_2x2 = {
    "I": np.eye(2, dtype=complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.array([[1, 0], [0, -1]], dtype=complex),
}


def pauli_dense(x: int, z: int, n: int) -> np.ndarray:
    """Kronecker product with qubit 0 as the most significant factor."""
    m = np.ones((1, 1), dtype=complex)
    for ch in pauli_label(x, z, n):
        m = np.kron(m, _PAULI_2x2[ch])
    return m


def paulisum_dense(H: PauliSum, n: int) -> np.ndarray:
    m = np.zeros((1 << n, 1 << n), dtype=complex)
    for (x, z), c in H.terms.items():
        m += c * pauli_dense(x, z, n)
    return m
