"""Dense state-vector oracle (test only).

Paper: Eq. (2) (E = sum_i a_i <P_i>), Eq. (3)-(4) with the first-order Trotter
product of Sec. III-D.  The state is a 2^N complex128 vector with qubit 0 the
most significant bit of the basis index (the same order as the MPS sites).

* A Pauli string sigma(x, z) = i^{|x&z|} X^x Z^z maps basis state |b> to
  i^{|x&z|} (-1)^{|z & b|} |b xor x>  (masks in basis-index bit positions).
* R_P(phi) psi = cos(phi/2) psi - i sin(phi/2) P psi.
* E = sum_j c_j Re<psi|P_j|psi>, Neumaier-compensated, ascending term order,
  identity coefficient and constant added last.
* Gradients: exact adjoint sweep, and the two-term shift
  dE/dphi = (E(phi + pi/2) - E(phi - pi/2)) / 2 per rotation, chained to the
  excitation parameters by dphi_m/dtheta_k = -2 c_m.
"""
from __future__ import annotations

import numpy as np

from .uccsd import Rotation, rotation_angles

_I_POW = (1.0 + 0.0j, 1.0j, -1.0 + 0.0j, -1.0j)


def _to_index_mask(mask: int, n: int) -> int:
    """Qubit-k bit -> basis-index bit (n-1-k)."""
    out = 0
    for k in range(n):
        if (mask >> k) & 1:
            out |= 1 << (n - 1 - k)
    return out


def _parity(v: np.ndarray) -> np.ndarray:
    v = v.copy()
    p = np.zeros_like(v)
    while np.any(v):
        p ^= v & 1
        v >>= 1
    return p


class PauliApplier:
    """Caches index permutations and sign vectors for Pauli strings."""

    def __init__(self, n: int):
        self.n = n
        self.idx = np.arange(1 << n, dtype=np.int64)
        self._cache = {}

    def parts(self, x: int, z: int):
        key = (x, z)
        if key not in self._cache:
            xb = _to_index_mask(x, self.n)
            zb = _to_index_mask(z, self.n)
            ph = _I_POW[bin(x & z).count("1") % 4]
            sign = 1.0 - 2.0 * _parity(self.idx & zb)
            self._cache[key] = (self.idx ^ xb, ph * sign)
            if len(self._cache) > 20000:
                self._cache.clear()
        return self._cache[key]

    def apply(self, x: int, z: int, psi: np.ndarray) -> np.ndarray:
        dest, coef = self.parts(x, z)
        out = np.empty_like(psi)
        out[dest] = coef * psi
        return out


def basis_state(n: int, occ) -> np.ndarray:
    b = 0
    for k, o in enumerate(occ):
        if o:
            b |= 1 << (n - 1 - k)
    psi = np.zeros(1 << n, dtype=complex)
    psi[b] = 1.0
    return psi


def apply_rotation(pa: PauliApplier, rot: Rotation, phi: float, psi: np.ndarray) -> np.ndarray:
    return np.cos(0.5 * phi) * psi - 1j * np.sin(0.5 * phi) * pa.apply(rot.x, rot.z, psi)


def evolve(n: int, occ, rots, phis, pa: PauliApplier | None = None) -> np.ndarray:
    pa = pa or PauliApplier(n)
    psi = basis_state(n, occ)
    for r, phi in zip(rots, phis):
        psi = apply_rotation(pa, r, phi, psi)
    return psi


def neumaier_sum(values) -> float:
    s = 0.0
    comp = 0.0
    for v in values:
        t = s + v
        if abs(s) >= abs(v):
            comp += (s - t) + v
        else:
            comp += (v - t) + s
        s = t
    return s + comp


def expectations(pa: PauliApplier, terms, psi: np.ndarray) -> np.ndarray:
    """<psi|P|psi> for each (x, z, c) term (complex; imaginary part ~ 0)."""
    out = np.empty(len(terms), dtype=complex)
    for t, (x, z, _) in enumerate(terms):
        out[t] = np.vdot(psi, pa.apply(x, z, psi))
    return out


def energy(pa: PauliApplier, c_id: float, terms, psi: np.ndarray, e_const: float = 0.0) -> float:
    """Energy of a normalised state (the constant is normally folded into
    c_id already; kept separate for callers that split it)."""
    ev = expectations(pa, terms, psi)
    vals = [c * e.real for (_, _, c), e in zip(terms, ev)]
    return neumaier_sum(vals + [c_id, e_const])


def apply_hamiltonian(pa: PauliApplier, c_id: float, terms, psi: np.ndarray) -> np.ndarray:
    out = c_id * psi
    for x, z, c in terms:
        out = out + c * pa.apply(x, z, psi)
    return out


def vqe_energy(n: int, n_elec: int, c_id, terms, rots, theta, pa=None) -> float:
    pa = pa or PauliApplier(n)
    occ = [1 if q < n_elec else 0 for q in range(n)]
    psi = evolve(n, occ, rots, rotation_angles(rots, theta), pa)
    return energy(pa, c_id, terms, psi)


def grad_adjoint(n: int, n_elec: int, c_id, terms, rots, theta, pa=None):
    """Exact dE/dtheta by one reverse sweep; returns (grad, dE/dphi, E)."""
    pa = pa or PauliApplier(n)
    occ = [1 if q < n_elec else 0 for q in range(n)]
    phis = rotation_angles(rots, theta)
    psi = evolve(n, occ, rots, phis, pa)
    lam = apply_hamiltonian(pa, c_id, terms, psi)
    e = float(np.vdot(psi, lam).real)
    dphi = np.zeros(len(rots))
    for m in reversed(range(len(rots))):
        r = rots[m]
        # dE/dphi_m = 2 Re <lam| (-i/2) P_m |psi> = Im <lam|P_m|psi>
        dphi[m] = np.vdot(lam, pa.apply(r.x, r.z, psi)).imag
        psi = apply_rotation(pa, r, -phis[m], psi)
        lam = apply_rotation(pa, r, -phis[m], lam)
    grad = np.zeros(len(theta))
    for m, r in enumerate(rots):
        grad[r.param] += -2.0 * r.c * dphi[m]
    return grad, dphi, e


def grad_paramshift(n: int, n_elec: int, c_id, terms, rots, theta, pa=None,
                     rot_subset=None):
    """Two-term shift per rotation angle; returns (grad, dE/dphi)."""
    pa = pa or PauliApplier(n)
    occ = [1 if q < n_elec else 0 for q in range(n)]
    phis = rotation_angles(rots, theta)
    sel = range(len(rots)) if rot_subset is None else rot_subset
    dphi = np.zeros(len(rots))
    for m in sel:
        vals = []
        for sh in (0.5 * np.pi, -0.5 * np.pi):
            p2 = phis.copy()
            p2[m] += sh
            psi = evolve(n, occ, rots, p2, pa)
            vals.append(energy(pa, c_id, terms, psi))
        dphi[m] = 0.5 * (vals[0] - vals[1])
    grad = np.zeros(len(theta))
    for m, r in enumerate(rots):
        grad[r.param] += -2.0 * r.c * dphi[m]
    return grad, dphi


def grad_fourterm(n: int, n_elec: int, c_id, terms, rots, theta, pa=None):
    """Four-term shift per UCCSD parameter.  The rotations of one excitation
    commute, so together they are exp(i theta_k G_k) with G_k = sum_m c_m P_m;
    when G_k has eigenvalues in {0, +-1} (one-excitation rotations between two
    determinants), E(theta_k) holds only the frequencies 1 and 2 and
    dE/dtheta_k = D(pi/4) + (1 - sqrt 2) / 2 D(pi/2) exactly, with
    D(s) = E(theta_k + s) - E(theta_k - s) (the general parameter-shift rule
    for two frequencies)."""
    pa = pa or PauliApplier(n)
    theta = np.asarray(theta, dtype=float)
    grad = np.zeros(len(theta))

    def e_at(k, s):
        th = theta.copy()
        th[k] += s
        return vqe_energy(n, n_elec, c_id, terms, rots, th, pa)

    for k in range(len(theta)):
        d1 = e_at(k, 0.5 * np.pi) - e_at(k, -0.5 * np.pi)
        d2 = e_at(k, 0.25 * np.pi) - e_at(k, -0.25 * np.pi)
        grad[k] = d2 + 0.5 * (1.0 - np.sqrt(2.0)) * d1
    return grad


def apply_two_site(psi: np.ndarray, n: int, site: int, g: np.ndarray) -> np.ndarray:
    """Apply a 4x4 gate (basis 2*i_site + i_{site+1}) to a dense state."""
    t = psi.reshape((1 << site, 4, 1 << (n - site - 2)))
    return np.einsum("ij,ajb->aib", g, t).reshape(-1)


def apply_one_site(psi: np.ndarray, n: int, q: int, g: np.ndarray) -> np.ndarray:
    t = psi.reshape((1 << q, 2, 1 << (n - q - 1)))
    return np.einsum("ij,ajb->aib", g, t).reshape(-1)
