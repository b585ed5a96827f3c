"""UCCSD ansatz as Pauli rotations and its nearest-neighbour gate compile
(oracle, test only).

Paper: Eq. (3) (UCC unitary exp(T - T^dag) on a Slater determinant),
Eq. (4) (singles a+_a a_i and doubles a+_a a+_b a_i a_j), Sec. III-D (the
ansatz is a first-order Trotter product with the variational parameters in RZ
gates; the Hartree-Fock reference is prepared by X gates), Sec. III-A (gates
act on neighbouring qubits; single-qubit gates are absorbed into two-qubit
gates by gate fusion).

Definitions used (one reading of the paper, listed in the design notes):
* Occupied spin-orbitals are 0..n_e-1 (Hartree-Fock), virtual n_e..N-1.
* Singles tau = a+_a a_i (i occupied, a virtual, same spin), sorted by (i, a).
  Doubles tau = a+_a a+_b a_i a_j (i<j occupied, a<b virtual, S_z conserved),
  sorted by (i, j, a, b).  Singles come first.  One parameter per excitation.
* U(theta) = prod_{k=K..1} exp(theta_k (tau_k - tau_k^dag)): parameter 1 acts
  first.
* tau - tau^dag = i sum_m c_m P_m with mutually commuting Pauli strings, so
  exp(theta (tau - tau^dag)) = prod_m R_{P_m}(phi_m),
  R_P(phi) = exp(-i phi P / 2), phi_m = -2 c_m theta.  Within one excitation
  the strings are applied in ascending (x, z) order.
* Nearest-neighbour compile of R_P(phi) with support lo..hi:
  basis change on each X/Y qubit (X: H, Y: H S^dag, i.e. S^dag first), a
  parity ladder up the support (CNOT(k, k+1) if qubit k+1 is in the support,
  SWAP(k, k+1) across identity qubits), RZ(phi) on qubit hi, the mirrored
  ladder down, and the basis changes undone.  Each single-qubit gate is fused
  into the first (before) or last (after) two-qubit gate that touches its
  qubit; the two ladder gates on bond (hi-1, hi) and the RZ between them form
  one gate.  That gives 2(hi-lo)-1 two-qubit gates per rotation.
* Two-qubit gate matrices are 4x4 with basis index 2*i_n + i_{n+1}, i.e.
  kron(A_n, B_{n+1}).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .fermion import DROP_TOL, PauliSum, jw_annihilate, jw_create


@dataclasses.dataclass(frozen=True)
class Excitation:
    kind: str  # "s" or "d"
    occ: tuple  # (i,) or (i, j)
    vir: tuple  # (a,) or (a, b)


def excitations(n_qubits: int, n_elec: int) -> list[Excitation]:
    occ = list(range(n_elec))
    vir = list(range(n_elec, n_qubits))
    singles = [Excitation("s", (i,), (a,)) for i in occ for a in vir if i % 2 == a % 2]
    doubles = []
    for x, i in enumerate(occ):
        for j in occ[x + 1:]:
            for y, a in enumerate(vir):
                for b in vir[y + 1:]:
                    if (i % 2) + (j % 2) == (a % 2) + (b % 2):
                        doubles.append(Excitation("d", (i, j), (a, b)))
    singles.sort(key=lambda e: (e.occ, e.vir))
    doubles.sort(key=lambda e: (e.occ, e.vir))
    return singles + doubles


def excitation_operator(e: Excitation) -> PauliSum:
    """tau as a PauliSum (literal operator order of Eq. 4)."""
    if e.kind == "s":
        (i,), (a,) = e.occ, e.vir
        return jw_create(a) * jw_annihilate(i)
    (i, j), (a, b) = e.occ, e.vir
    return jw_create(a) * jw_create(b) * jw_annihilate(i) * jw_annihilate(j)


def generator_strings(e: Excitation):
    """tau - tau^dag = i sum_m c_m P_m; returns [(x, z, c_m)] ascending (x, z)."""
    tau = excitation_operator(e)
    g = (tau - tau.dagger()).pruned()
    out = []
    for (x, z), v in g.terms.items():
        c = v / 1j
        if abs(c.imag) > DROP_TOL:
            raise ValueError("generator is not i times a real Pauli sum")
        out.append((x, z, c.real))
    out.sort(key=lambda t: (t[0], t[1]))
    return out


@dataclasses.dataclass(frozen=True)
class Rotation:
    x: int
    z: int
    c: float  # phi = -2 c theta[param]
    param: int

    def support(self) -> tuple[int, int]:
        m = self.x | self.z
        lo = (m & -m).bit_length() - 1
        hi = m.bit_length() - 1
        return lo, hi


def rotations(n_qubits: int, n_elec: int) -> list[Rotation]:
    out = []
    for k, e in enumerate(excitations(n_qubits, n_elec)):
        for x, z, c in generator_strings(e):
            out.append(Rotation(x, z, c, k))
    return out


def rotation_angles(rots: list[Rotation], theta: np.ndarray) -> np.ndarray:
    return np.array([-2.0 * r.c * theta[r.param] for r in rots])


# ----------------------------------------------------------------- gates ---

_SQ2 = 1.0 / np.sqrt(2.0)
GATE_H = np.array([[_SQ2, _SQ2], [_SQ2, -_SQ2]], dtype=complex)
GATE_SDAG = np.array([[1, 0], [0, -1j]], dtype=complex)
GATE_I = np.eye(2, dtype=complex)
GATE_CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
GATE_SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=complex)


def rz(phi: float) -> np.ndarray:
    return np.diag([np.exp(-0.5j * phi), np.exp(0.5j * phi)])


def basis_change(p: str) -> np.ndarray:
    """V with V^dag Z V = P (applied before the Z-parity rotation)."""
    if p == "X":
        return GATE_H
    if p == "Y":
        return GATE_H @ GATE_SDAG
    return GATE_I


def _qubit_pauli(rot: Rotation, q: int) -> str:
    b = ((rot.x >> q) & 1, (rot.z >> q) & 1)
    return {(0, 0): "I", (1, 0): "X", (0, 1): "Z", (1, 1): "Y"}[b]


@dataclasses.dataclass
class NativeGate:
    """One unfused gate.  qubits=(q,) for single-qubit, (k, k+1) for two-qubit.
    ``rot`` is the rotation index when the matrix depends on the angle (RZ)."""

    name: str
    qubits: tuple
    matrix: np.ndarray | None
    rot: int = -1


def native_rotation_gates(rot: Rotation, rot_index: int) -> list[NativeGate]:
    lo, hi = rot.support()
    supp = [q for q in range(lo, hi + 1) if _qubit_pauli(rot, q) != "I"]
    gates = []
    for q in supp:
        p = _qubit_pauli(rot, q)
        if p in "XY":
            gates.append(NativeGate("V" + p, (q,), basis_change(p)))
    ladder = []
    for k in range(lo, hi):
        if _qubit_pauli(rot, k + 1) != "I":
            ladder.append(NativeGate("CNOT", (k, k + 1), GATE_CNOT))
        else:
            ladder.append(NativeGate("SWAP", (k, k + 1), GATE_SWAP))
    gates += ladder
    gates.append(NativeGate("RZ", (hi,), None, rot_index))
    gates += [NativeGate(g.name, g.qubits, g.matrix) for g in reversed(ladder)]
    for q in supp:
        p = _qubit_pauli(rot, q)
        if p in "XY":
            gates.append(NativeGate("V" + p + "dag", (q,), basis_change(p).conj().T))
    return gates


@dataclasses.dataclass
class FusedGate:
    """Nearest-neighbour two-qubit gate on (site, site+1).

    Constant gate: ``rot == -1`` and the 4x4 is ``mat``.
    Angle gate (apex): 4x4 = post @ kron(I, RZ(phi_rot)) @ pre.
    """

    site: int
    rot: int
    mat: np.ndarray | None = None
    pre: np.ndarray | None = None
    post: np.ndarray | None = None

    def matrix(self, phis: np.ndarray) -> np.ndarray:
        if self.rot < 0:
            return self.mat
        return self.post @ np.kron(GATE_I, rz(phis[self.rot])) @ self.pre


def fused_rotation_gates(rot: Rotation, rot_index: int) -> list[FusedGate]:
    lo, hi = rot.support()
    L = hi - lo
    V = [basis_change(_qubit_pauli(rot, q)) if _qubit_pauli(rot, q) in "XY" else GATE_I
         for q in range(lo, hi + 1)]  # V[q - lo]

    def ladder(k):
        return GATE_CNOT if _qubit_pauli(rot, k + 1) != "I" else GATE_SWAP

    out = []
    # up ladder except its top gate; each fuses the basis change of the qubit
    # it touches first (both qubits for the bottom gate).
    for j in range(L - 1):
        k = lo + j
        pre = np.kron(V[0] if j == 0 else GATE_I, V[j + 1])
        out.append(FusedGate(k, -1, mat=ladder(k) @ pre))
    # apex on bond (hi-1, hi)
    k = hi - 1
    pre_v = np.kron(V[0] if L == 1 else GATE_I, V[L])
    post_v = pre_v.conj().T
    out.append(FusedGate(k, rot_index, pre=ladder(k) @ pre_v, post=post_v @ ladder(k)))
    # down ladder except its top gate; each fuses the undo of the basis change
    # of the qubit it touches last.
    for j in reversed(range(L - 1)):
        k = lo + j
        post = np.kron(V[0] if j == 0 else GATE_I, V[j + 1]).conj().T
        out.append(FusedGate(k, -1, mat=post @ ladder(k)))
    return out


def compile_fused(n_qubits: int, n_elec: int):
    """(rotations, fused nearest-neighbour gate list)."""
    rots = rotations(n_qubits, n_elec)
    gates = []
    for m, r in enumerate(rots):
        gates += fused_rotation_gates(r, m)
    return rots, gates


def compile_native(n_qubits: int, n_elec: int):
    rots = rotations(n_qubits, n_elec)
    gates = []
    for m, r in enumerate(rots):
        gates += native_rotation_gates(r, m)
    return rots, gates


def hf_occupation(n_qubits: int, n_elec: int) -> list[int]:
    return [1 if q < n_elec else 0 for q in range(n_qubits)]
