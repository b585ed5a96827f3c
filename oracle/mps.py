"""CPU matrix-product-state oracle (test only).

Paper: Sec. III-A.  Eq. (6) (MPS with bond dimension D, right-canonical
gauge), Eq. (7) (two-site contraction with the gate), Eq. (8) (scaling by the
Schmidt values of the left bond), Eq. (9) (SVD and truncation to the D
largest Schmidt values), Eq. (10) (the update that keeps right-canonical form
without dividing by Schmidt values), Eq. (11) and Eq. (2) (expectations).

Per gate O on sites (n, n+1), with lambda_{-1} = [1]:
  1. Theta[a,i,j,c] = sum_m B_n[a,i,m] B_{n+1}[m,j,c]
  2. M[a,i,j,c]     = sum_{i'j'} O[2i+j, 2i'+j'] Theta[a,i',j',c]
  3. M'             = lambda_{n-1}[a] * M
  4. M' (as (2 chi_l) x (2 chi_r)) = U S W^H   (LAPACK, S descending)
  5. chi' = min(D, #{s_k > 1e-12 s_1})
  6. lambda_n = S[:chi'] / ||S[:chi']||
  7. B_{n+1} = W^H[:chi']
  8. B_n     = M W[:, :chi'] / ||S[:chi']||
  9. discarded weight += sum_{k >= chi'} s_k^2 / sum_k s_k^2
Expectations are exact contractions of the stored MPS divided by its norm:
identity environments from both ends, a transfer sweep with the Pauli
operator over the string's support, and a closing trace.  This equals the
paper's lambda^2 form (Eq. 11) and its Hadamard-test form when the state is
exactly right-canonical, and stays variational when it is truncated.
"""
from __future__ import annotations

import numpy as np

from .statevector import neumaier_sum

SV_CUTOFF_REL = 1e-12


def _svd_gesdd(mat):
    return np.linalg.svd(mat, full_matrices=False)


def _svd_gesvd(mat):
    import scipy.linalg

    return scipy.linalg.svd(mat, full_matrices=False, lapack_driver="gesvd")


SVD_DRIVERS = {"gesdd": _svd_gesdd, "gesvd": _svd_gesvd}


class MPS:
    """``svd`` selects the LAPACK driver (divide-and-conquer ``gesdd`` or
    QR-iteration ``gesvd``); both are backward-stable, and comparing them
    measures how far rounding alone moves a truncated trajectory."""

    def __init__(self, occ, max_bond: int, svd: str = "gesdd"):
        self.n = len(occ)
        self.D = max_bond
        self._svd = SVD_DRIVERS[svd]
        self.B = []
        for o in occ:
            t = np.zeros((1, 2, 1), dtype=complex)
            t[0, 1 if o else 0, 0] = 1.0
            self.B.append(t)
        self.lam = [np.ones(1) for _ in range(self.n - 1)]  # bond b between b, b+1
        self.discarded = 0.0
        self.max_discarded = 0.0
        self.max_chi = 1
        self.min_gap_rel = np.inf  # smallest (s_D - s_{D+1}) / s_1 at a cut

    def lam_left(self, n: int) -> np.ndarray:
        return np.ones(1) if n == 0 else self.lam[n - 1]

    def chi(self, b: int) -> int:
        return self.B[b].shape[2]

    def apply_gate(self, n: int, O: np.ndarray) -> float:
        Bn, Bn1 = self.B[n], self.B[n + 1]
        chil, chir = Bn.shape[0], Bn1.shape[2]
        theta = np.tensordot(Bn, Bn1, axes=([2], [0]))  # a i j c
        O4 = O.reshape(2, 2, 2, 2)
        M = np.einsum("ijkl,aklc->aijc", O4, theta)
        Mp = self.lam_left(n)[:, None, None, None] * M
        mat = Mp.reshape(2 * chil, 2 * chir)
        _, S, Wh = self._svd(mat)
        nz = int(np.count_nonzero(S > SV_CUTOFF_REL * S[0]))
        keep = min(self.D, nz)
        if keep < nz:
            self.min_gap_rel = min(self.min_gap_rel, (S[keep - 1] - S[keep]) / S[0])
        tot = float(np.sum(S * S))
        norm = float(np.sqrt(np.sum(S[:keep] ** 2)))
        d = float(np.sum(S[keep:] ** 2)) / tot
        self.lam[n] = S[:keep] / norm
        W = Wh[:keep].conj().T
        self.B[n + 1] = Wh[:keep].reshape(keep, 2, chir)
        self.B[n] = (M.reshape(2 * chil, 2 * chir) @ W / norm).reshape(chil, 2, keep)
        self.discarded += d
        self.max_discarded = max(self.max_discarded, d)
        self.max_chi = max(self.max_chi, keep)
        return d

    # ---------------------------------------------------------- readouts ---

    def to_statevector(self) -> np.ndarray:
        psi = self.B[0].reshape(2, -1)
        for n in range(1, self.n):
            Bn = self.B[n]
            psi = (psi @ Bn.reshape(Bn.shape[0], -1)).reshape(-1, Bn.shape[2])
        return psi.reshape(-1)

    def left_envs(self):
        L = [np.ones((1, 1), dtype=complex)]
        for n in range(self.n):
            B = self.B[n]
            T = sum(B[:, i, :].conj().T @ L[-1] @ B[:, i, :] for i in range(2))
            L.append(T)
        return L  # L[k]: environment to the left of site k

    def right_envs(self):
        R = [None] * (self.n + 1)
        R[self.n] = np.ones((1, 1), dtype=complex)
        for n in reversed(range(self.n)):
            B = self.B[n]
            R[n] = sum(B[:, i, :].conj() @ R[n + 1] @ B[:, i, :].T for i in range(2))
        return R  # R[k]: environment to the right of site k-1 (indices of bond k-1)

    def norm2(self) -> float:
        return float(self.left_envs()[-1][0, 0].real)

    def right_canonical_error(self) -> float:
        err = 0.0
        for n in range(1, self.n):
            B = self.B[n]
            G = sum(B[:, i, :] @ B[:, i, :].conj().T for i in range(2))
            err = max(err, float(np.max(np.abs(G - np.eye(G.shape[0])))))
        return err


_PAULI = {
    (0, 0): np.eye(2, dtype=complex),
    (1, 0): np.array([[0, 1], [1, 0]], dtype=complex),
    (0, 1): np.array([[1, 0], [0, -1]], dtype=complex),
    (1, 1): np.array([[0, -1j], [1j, 0]], dtype=complex),
}


def pauli_expectations(mps: MPS, strings, L=None, R=None) -> np.ndarray:
    """<P>/<psi|psi> for each (x, z[, c]) string (complex)."""
    L = L or mps.left_envs()
    R = R or mps.right_envs()
    nrm = L[-1][0, 0].real
    out = np.empty(len(strings), dtype=complex)
    for t, s in enumerate(strings):
        x, z = s[0], s[1]
        m = x | z
        if m == 0:
            out[t] = 1.0
            continue
        lo = (m & -m).bit_length() - 1
        hi = m.bit_length() - 1
        T = L[lo]
        for k in range(lo, hi + 1):
            sig = _PAULI[((x >> k) & 1, (z >> k) & 1)]
            B = mps.B[k]
            Tn = 0
            for i in range(2):
                for ip in range(2):
                    if sig[i, ip] != 0:
                        Tn = Tn + sig[i, ip] * (B[:, i, :].conj().T @ T @ B[:, ip, :])
            T = Tn
        out[t] = np.sum(T * R[hi + 1]) / nrm
    return out


def energy(mps: MPS, c_id: float, terms) -> tuple[float, float]:
    """(E, max |Im <P>|) with the Neumaier sum in term order, c_id last."""
    ev = pauli_expectations(mps, terms)
    vals = [c * e.real for (_, _, c), e in zip(terms, ev)]
    return neumaier_sum(vals + [c_id]), float(np.max(np.abs(ev.imag))) if len(ev) else 0.0


def run_circuit(n: int, occ, gates, phis, max_bond: int, progress=None, svd: str = "gesdd") -> MPS:
    mps = MPS(occ, max_bond, svd)
    for g_i, g in enumerate(gates):
        mps.apply_gate(g.site, g.matrix(phis))
        if progress and g_i % 5000 == 0:
            progress(g_i)
    return mps
