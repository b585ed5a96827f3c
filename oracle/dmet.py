"""DMET chemical-potential loop around a fragment solver (oracle, test only).

Paper: Sec. III-B (the DMET-MPS-VQE procedure).  A low-level (mean-field)
calculation of the whole system; fragments of consecutive sites; for each
fragment a bath from the Schmidt decomposition of the mean-field state and the
Hamiltonian projected onto fragment + bath; the fragment problem solved by VQE,
its electron count read from the one-particle density matrix; a global
chemical potential mu changed until the fragments' counts add up to the
system's electron number.  The paper does not fix the details; the readings
taken here:

* Low level: the restricted determinant of the one-body lattice matrix h
  (U = 0), n_elec / 2 lowest orbitals doubly occupied; its per-spin density
  matrix D = C_occ C_occ^T.  A degenerate Fermi level (no unique
  determinant) is an error.
* Bath: the fragment's environment rows of D, D[E, F] = U s V^T; the k left
  singular vectors with s > 1e-10 span the bath (k = fragment size; fewer is
  an error).  Fragment + bath hold exactly k electrons per spin.
* Embedding basis: the natural orbitals of D inside fragment + bath
  (eigenvalue 1 first, then 0), each block rotated to diagonalise h within
  it, each orbital's sign fixed so its largest-magnitude site coefficient is
  positive.  The UCCSD reference (first n_elec/2 orbitals occupied) is then
  the mean-field determinant.
* Embedded Hamiltonian: one-body N^T h N - mu N^T P_F N (P_F: projector on the
  fragment sites), two-body U on the fragment sites only (interacting
  fragment, non-interacting bath), (pq|rs) = U sum_{i in F} N_ip N_iq N_ir N_is.
* Fragment electrons: <sum_sigma sum_pq (N^T P_F N)_pq a+_p a_q>; fragment
  energy (democratic partitioning): the one-body part 1/2 (P_F h + h P_F)
  projected, plus the whole on-site interaction (all its indices are fragment
  indices); the DMET energy is the sum over fragments.
* mu: Illinois regula falsi on f(mu) = sum N_frag(mu) - n_elec over a bracket
  [mu_lo, mu_hi] with f(mu_lo) <= 0 <= f(mu_hi) (N_frag grows with mu);
  stop when |f| <= n_tol.
* Solvers: the UCCSD VQE minimum from theta = 0 (``minimize.uccsd_minimum``,
  the GPU loop's counterpart), or exact diagonalisation of the embedded
  Hamiltonian in its electron sector (for the pins).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import fermion, fockspace, minimize, uccsd
from . import statevector as sv


def mean_field_density(lat) -> np.ndarray:
    w, C = np.linalg.eigh(lat.h)
    no = lat.n_elec // 2
    if no < lat.n_sites and abs(w[no] - w[no - 1]) < 1e-10:
        raise ValueError("the mean-field determinant is degenerate (no gap at the Fermi level)")
    occ = C[:, :no]
    return occ @ occ.T


def _fix_signs(V: np.ndarray) -> np.ndarray:
    V = V.copy()
    for j in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, j])))
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return V


def embedding_basis(lat, D: np.ndarray, frag: int) -> np.ndarray:
    """Orthonormal embedding orbitals (n_sites x 2k) of fragment `frag`:
    occupied natural orbitals first, each block canonical in h."""
    k, L = lat.frag_size, lat.n_sites
    F = list(range(frag * k, (frag + 1) * k))
    E = [i for i in range(L) if i not in F]
    Ub, s, _ = np.linalg.svd(D[np.ix_(E, F)], full_matrices=False)
    if np.sum(s > 1e-10) != k:
        raise ValueError("the fragment's bath has fewer than k orbitals")
    W = np.zeros((L, 2 * k))
    W[F, np.arange(k)] = 1.0
    W[E, k:] = Ub[:, :k]
    w, V = np.linalg.eigh(W.T @ D @ W)
    order = np.argsort(-w, kind="stable")
    V = V[:, order]
    blocks = []
    for blk in (V[:, :k], V[:, k:]):
        hb = blk.T @ W.T @ lat.h @ W @ blk
        _, R = np.linalg.eigh(hb)
        blocks.append(blk @ R)
    return _fix_signs(W @ np.hstack(blocks))


@dataclasses.dataclass
class Embedded:
    h1: np.ndarray      # one-body matrix including -mu P_F
    eri: np.ndarray     # (pq|rs)
    nop: np.ndarray     # one-body matrix of the fragment electron count
    efrag_h1: np.ndarray  # one-body part of the fragment energy


def embedded_problem(lat, N: np.ndarray, frag: int, mu: float) -> Embedded:
    k = lat.frag_size
    PF = np.zeros(lat.n_sites)
    PF[frag * k:(frag + 1) * k] = 1.0
    nop = N.T @ (PF[:, None] * N)
    h1 = N.T @ lat.h @ N - mu * nop
    NF = N[frag * k:(frag + 1) * k, :]
    eri = lat.U * np.einsum("ip,iq,ir,is->pqrs", NF, NF, NF, NF)
    hp = PF[:, None] * lat.h
    efrag_h1 = N.T @ (0.5 * (hp + hp.T)) @ N
    return Embedded(h1, eri, nop, efrag_h1)


def _jw(h1, eri):
    return fermion.hamiltonian_terms(fermion.jw_hamiltonian(h1, eri))


def solve_fragment(lat, emb: Embedded, solver: str = "uccsd"):
    """(N_frag, E_frag, E_emb) of one embedded problem: 2k orbitals, 2k electrons."""
    k = lat.frag_size
    n, ne = 4 * k, 2 * k
    zero = np.zeros((2 * k,) * 4)
    if solver == "uccsd":
        c_id, terms = _jw(emb.h1, emb.eri)
        rots = uccsd.rotations(n, ne)
        th, e, _ = minimize.uccsd_minimum(n, ne, c_id, terms, rots, np.zeros(len({r.param for r in rots})))
        pa = sv.PauliApplier(n)
        nf = sv.vqe_energy(n, ne, *_jw(emb.nop, zero), rots, th, pa)
        ef = sv.vqe_energy(n, ne, *_jw(emb.efrag_h1, emb.eri), rots, th, pa)
        return nf, ef, e
    sec = fockspace.Sector(n, ne)
    H = fockspace.hamiltonian(sec, emb.h1, emb.eri)
    w, V = np.linalg.eigh(H)
    psi = V[:, 0]
    nf = float(psi @ fockspace.hamiltonian(sec, emb.nop, zero) @ psi)
    ef = float(psi @ fockspace.hamiltonian(sec, emb.efrag_h1, emb.eri) @ psi)
    return nf, ef, float(w[0])


@dataclasses.dataclass
class DmetResult:
    mu: float
    n_frag: np.ndarray
    e_frag: np.ndarray
    e_emb: np.ndarray
    iterations: int
    status: int  # 1 converged, 0 iteration limit, 3 bracket holds no sign change
    mu_trace: list


def dmet(lat, solver: str = "uccsd", mu_lo: float = -2.0, mu_hi: float = 2.0, n_tol: float = 1e-6,
         max_iter: int = 40) -> DmetResult:
    D = mean_field_density(lat)
    bases = [embedding_basis(lat, D, f) for f in range(lat.n_frags)]
    trace = []

    def evaluate(mu):
        out = [solve_fragment(lat, embedded_problem(lat, bases[f], f, mu), solver) for f in range(lat.n_frags)]
        nf, ef, ee = (np.array(x) for x in zip(*out))
        trace.append(mu)
        return float(np.sum(nf)) - lat.n_elec, nf, ef, ee

    a, b = mu_lo, mu_hi
    fa, *ra = evaluate(a)
    fb, *rb = evaluate(b)
    if abs(fa) <= n_tol:
        return DmetResult(a, *ra, 0, 1, trace)
    if abs(fb) <= n_tol:
        return DmetResult(b, *rb, 0, 1, trace)
    if fa > 0 or fb < 0:
        return DmetResult(a, *ra, 0, 3, trace)
    side = 0
    c, rc = a, ra
    for it in range(1, max_iter + 1):
        c = (a * fb - b * fa) / (fb - fa)
        fc, *rc = evaluate(c)
        if abs(fc) <= n_tol:
            return DmetResult(c, *rc, it, 1, trace)
        if fc < 0:
            a, fa = c, fc
            if side == -1:
                fb *= 0.5
            side = -1
        else:
            b, fb = c, fc
            if side == 1:
                fa *= 0.5
            side = 1
    return DmetResult(c, *rc, max_iter, 0, trace)
