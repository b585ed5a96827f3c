"""Host-side checks of libq2c that need no GPU: exported symbols, the C++
problem compiler against the independently written oracle, and the error
conventions of the C ABI."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import fermion, uccsd
from workloads import CONFIGS, h2_like_integrals, random_integrals

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "q2c.h")

q2c = pytest.importorskip("paper_2207_03711_amd.q2c", reason="libq2c.so not built")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_0-9]+)\s*\(", src)) - {"sizeof"})


def test_header_symbols_are_exported_and_bound():
    names = _declared_functions()
    assert "vqe_energy" in names and "mps_apply_gate" in names
    lib = C.CDLL(q2c.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
        assert n in q2c.SIGNATURES, n


def _host_problem(I):
    return q2c.vqe_problem_create(None, I.n_orb, I.n_elec, I.h1, I.eri, I.e_const)


@pytest.mark.parametrize("which", ["h2", "q8", "q12"])
def test_pauli_list_matches_oracle(which):
    if which == "h2":
        I = h2_like_integrals()
    elif which == "q8":
        I = CONFIGS["q8_d16"].integrals()
    else:
        I = random_integrals(6, 6, 77)
    p = _host_problem(I)
    try:
        info = q2c.vqe_problem_info(p)
        x, z, c = q2c.vqe_problem_paulis(p)
        cid_o, terms_o = fermion.hamiltonian_terms(fermion.jw_hamiltonian(I.h1, I.eri, I.e_const))
        assert info["n_strings"] == len(terms_o)
        assert abs(info["identity_coeff"] - cid_o) < 1e-12
        assert [(int(a), int(b)) for a, b in zip(x, z)] == [(t[0], t[1]) for t in terms_o]
        assert np.max(np.abs(c - np.array([t[2] for t in terms_o]))) < 1e-12
    finally:
        q2c.vqe_problem_destroy(p)


@pytest.mark.parametrize("n_orb,n_elec", [(2, 2), (3, 2), (4, 4)])
def test_rotations_and_gates_match_oracle(n_orb, n_elec):
    I = random_integrals(n_orb, n_elec, 5)
    p = _host_problem(I)
    try:
        n = 2 * n_orb
        info = q2c.vqe_problem_info(p)
        rots_o, gates_o = uccsd.compile_fused(n, n_elec)
        assert info["n_params"] == len(uccsd.excitations(n, n_elec))
        assert info["n_rotations"] == len(rots_o)
        assert info["n_gates"] == len(gates_o)
        x, z, c, par = q2c.vqe_problem_rotations(p)
        for m, r in enumerate(rots_o):
            assert (int(x[m]), int(z[m]), int(par[m])) == (r.x, r.z, r.param)
            assert abs(c[m] - r.c) < 1e-15
        site, rot, pre, post = q2c.vqe_problem_gates(p)
        for g, go in enumerate(gates_o):
            assert site[g] == go.site and rot[g] == go.rot
            if go.rot < 0:
                assert np.max(np.abs(pre[g] - go.mat)) < 1e-14
                assert np.max(np.abs(post[g] - np.eye(4))) < 1e-15
            else:
                assert np.max(np.abs(pre[g] - go.pre)) < 1e-14
                assert np.max(np.abs(post[g] - go.post)) < 1e-14
    finally:
        q2c.vqe_problem_destroy(p)


def test_counts_at_16_qubits():
    I = CONFIGS["q16_d64"].integrals()
    p = _host_problem(I)
    try:
        info = q2c.vqe_problem_info(p)
        assert (info["n_params"], info["n_rotations"], info["n_gates"]) == (360, 2688, 55424)
        cid_o, terms_o = fermion.hamiltonian_terms(fermion.jw_hamiltonian(I.h1, I.eri))
        assert info["n_strings"] == len(terms_o)
    finally:
        q2c.vqe_problem_destroy(p)


def _expect_error(fn, code):
    with pytest.raises(q2c.Q2CError) as ei:
        fn()
    assert ei.value.code == code
    assert q2c.last_error()


def test_argument_errors():
    I = random_integrals(2, 2, 1)
    _expect_error(lambda: q2c.vqe_problem_create(None, 0, 0, I.h1, I.eri), q2c.Q2C_ERR_ARG)
    _expect_error(lambda: q2c.vqe_problem_create(None, 2, 3, I.h1, I.eri), q2c.Q2C_ERR_ARG)
    _expect_error(lambda: q2c.vqe_problem_create(None, 2, 6, I.h1, I.eri), q2c.Q2C_ERR_ARG)
    bad = I.eri.copy()
    bad[0, 1, 0, 1] = np.nan
    _expect_error(lambda: q2c.vqe_problem_create(None, 2, 2, I.h1, bad), q2c.Q2C_ERR_ARG)
    badh = I.h1.copy()
    badh[1, 1] = np.inf
    _expect_error(lambda: q2c.vqe_problem_create(None, 2, 2, badh, I.eri), q2c.Q2C_ERR_ARG)
    # NULL handles
    assert q2c.lib.vqe_problem_destroy(None) == q2c.Q2C_ERR_ARG
    assert q2c.lib.mps_destroy(None) == q2c.Q2C_ERR_ARG
    assert q2c.lib.q2c_ctx_destroy(None) == q2c.Q2C_ERR_ARG
    assert q2c.lib.mps_apply_gate(None, 0, None, None) == q2c.Q2C_ERR_ARG
    # a host-only problem cannot be evaluated
    p = _host_problem(I)
    try:
        th = np.zeros(q2c.vqe_problem_info(p)["n_params"])
        _expect_error(lambda: q2c.vqe_energy(p, th, 4), q2c.Q2C_ERR_ARG)
        # the VQE loop checks its own arguments, then passes the inner error through
        _expect_error(lambda: q2c.vqe_minimize(p, th[:-1], 4), q2c.Q2C_ERR_ARG)
        assert "n_theta" in q2c.last_error()
        _expect_error(lambda: q2c.vqe_minimize(p, th, 4, n_trial=65), q2c.Q2C_ERR_ARG)
        _expect_error(lambda: q2c.vqe_minimize(p, th, 4, gtol=-1.0), q2c.Q2C_ERR_ARG)
        bad_th = th.copy()
        bad_th[0] = np.nan
        _expect_error(lambda: q2c.vqe_minimize(p, bad_th, 4), q2c.Q2C_ERR_ARG)
        _expect_error(lambda: q2c.vqe_minimize(p, th, 4), q2c.Q2C_ERR_ARG)
        assert q2c.vqe_problem_electrons(p) == (2, 2)
        _expect_error(lambda: q2c.vqe_energy_hadamard(None, p, th, 4), q2c.Q2C_ERR_ARG)
    finally:
        q2c.vqe_problem_destroy(p)
    assert q2c.lib.vqe_minimize(None, None, 0, 4, 0, None, None, None, None, None) == q2c.Q2C_ERR_ARG


def test_context_without_gpu_reports_device_error():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    _expect_error(lambda: q2c.q2c_ctx_create(0), q2c.Q2C_ERR_DEVICE)


def _letters(x, z, lo, hi):
    return tuple(((x >> k) & 1) | (((z >> k) & 1) << 1) for k in range(lo, hi + 1))


def _support(x, z):
    m = x | z
    if m == 0:
        return None
    return (m & -m).bit_length() - 1, m.bit_length() - 1


@pytest.mark.parametrize("which", ["q8", "q16", "random"])
def test_pauli_prefix_order(which):
    """The prefix order is a permutation sorted by (lowest qubit, letters);
    each share is the common leading run with the previous sorted string;
    and the transfer steps it leaves equal the node count of the prefix
    trie, counted here from the set of distinct (lowest qubit, prefix)."""
    if which == "random":
        rng = np.random.default_rng(11)
        n = 300
        x = rng.integers(0, 1 << 12, n, dtype=np.uint64) & rng.integers(0, 1 << 12, n, dtype=np.uint64)
        z = rng.integers(0, 1 << 12, n, dtype=np.uint64) & rng.integers(0, 1 << 12, n, dtype=np.uint64)
        x[:3] = 0
        z[:3] = 0  # identity strings, repeated
        x[3:6] = x[6]
        z[3:6] = z[6]  # repeated strings
    else:
        I = CONFIGS["q8_d16" if which == "q8" else "q16_d64"].integrals()
        _, terms = fermion.hamiltonian_terms(fermion.jw_hamiltonian(I.h1, I.eri, I.e_const))
        x = np.array([t[0] for t in terms], dtype=np.uint64)
        z = np.array([t[1] for t in terms], dtype=np.uint64)
    order, share, (plain, shared) = q2c.pauli_prefix_order(x, z)
    n = len(x)
    assert sorted(order.tolist()) == list(range(n))
    xs = [int(v) for v in x]
    zs = [int(v) for v in z]

    def key(s):
        sp = _support(xs[s], zs[s])
        return (-1, ()) if sp is None else (sp[0], _letters(xs[s], zs[s], sp[0], 63))

    keys = [key(int(s)) for s in order]
    assert keys == sorted(keys)
    nodes, total = set(), 0
    for t, s in enumerate(order):
        s = int(s)
        sp = _support(xs[s], zs[s])
        want = 0
        if sp is not None:
            lo, hi = sp
            L = _letters(xs[s], zs[s], lo, hi)
            total += len(L)
            for d in range(1, len(L) + 1):
                nodes.add((lo, L[:d]))
            if t > 0:
                p = int(order[t - 1])
                spp = _support(xs[p], zs[p])
                if spp is not None and spp[0] == lo:
                    Lp = _letters(xs[p], zs[p], lo, spp[1])
                    while want < min(len(L), len(Lp)) and L[want] == Lp[want]:
                        want += 1
        assert share[t] == want, (t, s)
    assert plain == total
    assert shared == len(nodes)
    if which == "q16":
        assert shared < plain / 3.5


@pytest.mark.parametrize("n_sites,k,seed", [(8, 1, 5), (8, 2, 3), (12, 3, 4), (12, 4, 6)])
def test_dmet_embedding_matches_oracle(n_sites, k, seed):
    """The C++ embedding (mean field, bath, natural orbitals, projected
    integrals; its own Jacobi eigensolver) equals the oracle's (LAPACK) for
    every fragment."""
    from oracle import dmet
    from workloads import random_lattice

    lat = random_lattice(n_sites, k, n_sites, seed, U=3.0)
    D = dmet.mean_field_density(lat)
    for f in range(lat.n_frags):
        N = dmet.embedding_basis(lat, D, f)
        ref = dmet.embedded_problem(lat, N, f, 0.7)
        got = q2c.dmet_embedding(n_sites, k, n_sites, lat.h, lat.U, f, 0.7)
        assert np.max(np.abs(got["orbitals"] - N)) < 1e-10, f
        for name in ("h1", "eri", "nop", "efrag_h1"):
            assert np.max(np.abs(got[name] - getattr(ref, name))) < 1e-10, (f, name)


def test_dmet_argument_errors():
    from workloads import random_lattice

    lat = random_lattice(8, 2, 8, 1)
    _expect_error(lambda: q2c.dmet_embedding(8, 3, 8, lat.h, 1.0, 0), q2c.Q2C_ERR_ARG)  # k does not divide L
    _expect_error(lambda: q2c.dmet_embedding(8, 2, 7, lat.h, 1.0, 0), q2c.Q2C_ERR_ARG)  # odd electrons
    _expect_error(lambda: q2c.dmet_embedding(8, 2, 8, lat.h, 1.0, 4), q2c.Q2C_ERR_ARG)  # fragment index
    bad = lat.h.copy()
    bad[0, 1] += 1e-3
    _expect_error(lambda: q2c.dmet_embedding(8, 2, 8, bad, 1.0, 0), q2c.Q2C_ERR_ARG)  # not symmetric
    ring = random_lattice(8, 2, 8, 1, eps_amp=0.0, ring=True)
    _expect_error(lambda: q2c.dmet_embedding(8, 2, 8, ring.h, 1.0, 0), q2c.Q2C_ERR_ARG)  # degenerate Fermi level
    assert "degenerate" in q2c.last_error()
    assert q2c.lib.dmet_solve(None, None, None, None, None, None, None, None) == q2c.Q2C_ERR_ARG
