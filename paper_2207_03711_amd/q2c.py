"""ctypes binding of libq2c (the C ABI declared in include/q2c.h).

Argument marshalling only: every step of the energy path runs in the HIP
library.  The library must have been built (``python -m
paper_2207_03711_amd.build``); importing this module fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libq2c.so")

Q2C_OK = 0
Q2C_ERR_ARG = -1
Q2C_ERR_OOM = -2
Q2C_ERR_DEVICE = -3
Q2C_ERR_NOCONV = -4
Q2C_ERR_NUMERIC = -5
Q2C_ERR_BUSY = -6
Q2C_FP64 = 0
Q2C_MIXED = 1

_ERR_NAMES = {
    Q2C_ERR_ARG: "ARG", Q2C_ERR_OOM: "OOM", Q2C_ERR_DEVICE: "DEVICE",
    Q2C_ERR_NOCONV: "NOCONV", Q2C_ERR_NUMERIC: "NUMERIC", Q2C_ERR_BUSY: "BUSY",
}


class Q2CError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"q2c error {_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class q2c_opts(C.Structure):
    _fields_ = [
        ("max_sweeps", C.c_int),
        ("sv_cutoff_rel", C.c_double),
        ("svd_tol", C.c_double),
        ("slots", C.c_int),
        ("hbm_budget_bytes", C.c_size_t),
        ("svd_algorithm", C.c_int),
        ("shift_from_start", C.c_int),
        ("eager_batches", C.c_int),
        ("no_autotune", C.c_int),
        ("autotune_cache", C.c_char_p),
        ("grad_rule", C.c_int),
    ]


class q2c_stats(C.Structure):
    _fields_ = [
        ("discarded_weight_sum", C.c_double),
        ("max_discarded", C.c_double),
        ("max_abs_imag", C.c_double),
        ("norm", C.c_double),
        ("max_chi", C.c_int),
        ("max_sweeps_used", C.c_int),
        ("seconds", C.c_double),
        ("gate_flops", C.c_double),
        ("jacobi_sweeps", C.c_double),
        ("gate_ms", C.c_double),
        ("env_ms", C.c_double),
        ("pauli_ms", C.c_double),
        ("reduce_ms", C.c_double),
        ("gate_launches", C.c_int),
        ("n_circuits", C.c_int),
        ("cycles", C.c_double * 6),
        ("svd_bisect_gates", C.c_double),
        ("svd_fallbacks", C.c_double),
        ("graph_ms", C.c_double),
        ("graph_launches", C.c_int),
        ("pauli_tile", C.c_int),
        ("pauli_wg", C.c_int),
        ("tune_ms", C.c_double),
    ]

    PHASES = ("contract", "reduce", "values", "vectors", "back", "update")

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "cycles"}
        d["cycles"] = dict(zip(self.PHASES, list(self.cycles)))
        return d


class q2c_min_opts(C.Structure):
    _fields_ = [
        ("max_iter", C.c_int),
        ("history", C.c_int),
        ("n_trial", C.c_int),
        ("gtol", C.c_double),
        ("ftol", C.c_double),
        ("max_step", C.c_double),
        ("no_speculation", C.c_int),
    ]


class q2c_min_report(C.Structure):
    _fields_ = [
        ("iterations", C.c_int),
        ("grad_evals", C.c_int),
        ("energy_evals", C.c_int),
        ("status", C.c_int),
        ("grad_max", C.c_double),
        ("seconds", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class q2c_lattice(C.Structure):
    _fields_ = [
        ("n_sites", C.c_int),
        ("frag_size", C.c_int),
        ("n_elec", C.c_int),
        ("h", C.POINTER(C.c_double)),
        ("U", C.c_double),
    ]


class q2c_dmet_opts(C.Structure):
    _fields_ = [
        ("mu_lo", C.c_double),
        ("mu_hi", C.c_double),
        ("n_tol", C.c_double),
        ("max_iter", C.c_int),
        ("max_bond", C.c_int),
        ("precision", C.c_int),
        ("vqe", q2c_min_opts),
        ("workers", C.c_int),
    ]


class q2c_dmet_report(C.Structure):
    _fields_ = [
        ("mu", C.c_double),
        ("e_dmet", C.c_double),
        ("iterations", C.c_int),
        ("status", C.c_int),
        ("vqe_runs", C.c_int),
        ("seconds", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class q2c_server_opts(C.Structure):
    _fields_ = [("slots_per_class", C.c_int), ("gates_per_step", C.c_int)]


class q2c_result(C.Structure):
    _fields_ = [
        ("tag", C.c_uint64),
        ("status", C.c_int),
        ("n_qubits", C.c_int),
        ("max_bond", C.c_int),
        ("precision", C.c_int),
        ("energy", C.c_double),
        ("n_frag", C.c_double),
        ("submit_s", C.c_double),
        ("admit_s", C.c_double),
        ("done_s", C.c_double),
        ("discarded_weight_sum", C.c_double),
        ("max_chi", C.c_int),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2207_03711_amd.build`")
    # One HIP runtime per process: load PyTorch's first so libq2c binds to it.
    import torch

    hip_rt = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
    if os.path.exists(hip_rt):
        C.CDLL(hip_rt, mode=C.RTLD_GLOBAL)
    return C.CDLL(LIB_PATH)


lib = _load()

_vp = C.c_void_p
_pvp = C.POINTER(C.c_void_p)
_pd = C.POINTER(C.c_double)
_pi = C.POINTER(C.c_int)
_pu64 = C.POINTER(C.c_uint64)
_pu8 = C.POINTER(C.c_uint8)

# name -> (restype, argtypes); every symbol declared in include/q2c.h
SIGNATURES = {
    "q2c_ctx_create": (C.c_int, [C.c_int, _vp, C.POINTER(q2c_opts), _pvp]),
    "q2c_ctx_destroy": (C.c_int, [_vp]),
    "q2c_ctx_memory": (C.c_int, [_vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "mps_create": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, _pu8, _pvp]),
    "mps_destroy": (C.c_int, [_vp]),
    "mps_apply_gate": (C.c_int, [_vp, C.c_int, _pd, _pd]),
    "mps_expect_pauli_batch": (C.c_int, [_vp, C.c_int, C.c_int, _pu64, _pu64, _pd, _pd]),
    "q2c_pauli_prefix_order": (C.c_int, [C.c_int, _pu64, _pu64, _pi, _pi, C.POINTER(C.c_int64)]),
    "mps_export": (C.c_int, [_vp, _pi, _pd, _pd]),
    "mps_get_stats": (C.c_int, [_vp, C.POINTER(q2c_stats)]),
    "vqe_problem_create": (C.c_int, [_vp, C.c_int, C.c_int, _pd, _pd, C.c_double, _pvp]),
    "vqe_problem_destroy": (C.c_int, [_vp]),
    "vqe_problem_info": (C.c_int, [_vp, _pi, _pi, _pi, _pi, _pi, _pd]),
    "vqe_problem_paulis": (C.c_int, [_vp, _pu64, _pu64, _pd]),
    "vqe_problem_rotations": (C.c_int, [_vp, _pu64, _pu64, _pd, _pi]),
    "vqe_problem_gates": (C.c_int, [_vp, _pi, _pi, _pd, _pd]),
    "vqe_energy": (C.c_int, [_vp, _pd, C.c_int, C.c_int, C.c_int, _pd, C.POINTER(q2c_stats)]),
    "vqe_energy_batch": (C.c_int, [_vp, _pd, C.c_int, C.c_int, C.c_int, C.c_int, _pd, C.POINTER(q2c_stats)]),
    "vqe_grad_paramshift": (C.c_int, [_vp, _pd, C.c_int, C.c_int, C.c_int, _pd, _pd, C.POINTER(q2c_stats)]),
    "vqe_shift_energies": (C.c_int, [_vp, _pd, C.c_int, _pi, C.c_int, C.c_int, C.c_int, _pd, _pd,
                                     C.POINTER(q2c_stats)]),
    "vqe_minimize": (C.c_int, [_vp, _pd, C.c_int, C.c_int, C.c_int, C.POINTER(q2c_min_opts), _pd, _pd, _pd,
                               C.POINTER(q2c_min_report)]),
    "mps_copy": (C.c_int, [_vp, _vp]),
    "vqe_problem_electrons": (C.c_int, [_vp, _pi, _pi]),
    "vqe_energy_hadamard": (C.c_int, [_vp, _vp, _pd, C.c_int, C.c_int, C.c_int, C.c_int, _pi, C.c_int, _pd, _pd,
                                      _pd]),
    "dmet_solve": (C.c_int, [_vp, C.POINTER(q2c_lattice), C.POINTER(q2c_dmet_opts), _pd, _pd, _pd, _pd,
                             C.POINTER(q2c_dmet_report)]),
    "dmet_embedding": (C.c_int, [C.POINTER(q2c_lattice), C.c_int, C.c_double, _pd, _pd, _pd, _pd, _pd]),
    "q2c_server_create": (C.c_int, [_vp, C.POINTER(q2c_server_opts), _pvp]),
    "q2c_server_destroy": (C.c_int, [_vp]),
    "q2c_server_submit": (C.c_int, [_vp, C.c_uint64, C.c_int, C.c_int, _pd, _pd, C.c_double, _pd, C.c_int, C.c_int,
                                    C.c_int, C.c_int]),
    "q2c_server_step": (C.c_int, [_vp, _pi, _pi, _pi]),
    "q2c_server_poll": (C.c_int, [_vp, C.POINTER(q2c_result), C.c_int, _pi]),
    "q2c_last_error": (C.c_char_p, []),
    "q2c_version": (C.c_char_p, []),
}

for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def last_error() -> str:
    return lib.q2c_last_error().decode()


def version() -> str:
    return lib.q2c_version().decode()


def _check(rc: int) -> None:
    if rc != Q2C_OK:
        raise Q2CError(rc, last_error())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_pd)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------- C entry points


def q2c_ctx_create(device: int = 0, hip_stream: int | None = None, opts: q2c_opts | None = None):
    h = C.c_void_p()
    _check(lib.q2c_ctx_create(device, hip_stream, C.byref(opts) if opts else None, C.byref(h)))
    return h


def q2c_ctx_destroy(ctx) -> None:
    _check(lib.q2c_ctx_destroy(ctx))


def q2c_ctx_memory(ctx):
    """(bytes in use, budget) of a context."""
    used, budget = C.c_size_t(), C.c_size_t()
    _check(lib.q2c_ctx_memory(ctx, C.byref(used), C.byref(budget)))
    return used.value, budget.value


def mps_create(ctx, n_qubits: int, max_bond: int, precision: int, occ):
    o = np.ascontiguousarray(occ, dtype=np.uint8)
    h = C.c_void_p()
    _check(lib.mps_create(ctx, n_qubits, max_bond, precision, o.ctypes.data_as(_pu8), C.byref(h)))
    return h


def mps_destroy(s) -> None:
    _check(lib.mps_destroy(s))


def mps_apply_gate(s, site: int, gate: np.ndarray) -> float:
    g = np.ascontiguousarray(np.asarray(gate, dtype=np.complex128).reshape(4, 4)).view(np.float64).reshape(-1)
    d = C.c_double()
    _check(lib.mps_apply_gate(s, site, _dp(g), C.byref(d)))
    return d.value


def mps_expect_pauli_batch(s, x_masks, z_masks, n_qubits: int):
    x = np.ascontiguousarray(x_masks, dtype=np.uint64)
    z = np.ascontiguousarray(z_masks, dtype=np.uint64)
    n = len(x)
    re = np.zeros(n)
    im = np.zeros(n)
    nw = (n_qubits + 63) // 64
    _check(lib.mps_expect_pauli_batch(s, n, nw, x.ctypes.data_as(_pu64), z.ctypes.data_as(_pu64), _dp(re), _dp(im)))
    return re, im


def pauli_prefix_order(x_masks, z_masks):
    """Prefix order of Pauli strings: (order, share, (steps_plain, steps_shared))."""
    x = np.ascontiguousarray(x_masks, dtype=np.uint64)
    z = np.ascontiguousarray(z_masks, dtype=np.uint64)
    n = len(x)
    order = np.zeros(n, dtype=np.int32)
    share = np.zeros(n, dtype=np.int32)
    steps = np.zeros(2, dtype=np.int64)
    _check(lib.q2c_pauli_prefix_order(n, x.ctypes.data_as(_pu64), z.ctypes.data_as(_pu64),
                                      order.ctypes.data_as(_pi), share.ctypes.data_as(_pi),
                                      steps.ctypes.data_as(C.POINTER(C.c_int64))))
    return order, share, (int(steps[0]), int(steps[1]))


def mps_export(s, n_qubits: int):
    chi = np.zeros(n_qubits + 1, dtype=np.int32)
    _check(lib.mps_export(s, chi.ctypes.data_as(_pi), None, None))
    size = sum(int(chi[n]) * 2 * int(chi[n + 1]) for n in range(n_qubits))
    t = np.zeros(2 * size)
    lam = np.zeros(max(1, sum(int(chi[b + 1]) for b in range(n_qubits - 1))))
    _check(lib.mps_export(s, chi.ctypes.data_as(_pi), _dp(t), _dp(lam)))
    tc = t.view(np.complex128)
    sites, o = [], 0
    for n in range(n_qubits):
        cl, cr = int(chi[n]), int(chi[n + 1])
        sites.append(tc[o:o + cl * 2 * cr].reshape(cl, 2, cr).copy())
        o += cl * 2 * cr
    lams, o = [], 0
    for b in range(n_qubits - 1):
        lams.append(lam[o:o + int(chi[b + 1])].copy())
        o += int(chi[b + 1])
    return chi, sites, lams


def mps_get_stats(s) -> dict:
    st = q2c_stats()
    _check(lib.mps_get_stats(s, C.byref(st)))
    return st.as_dict()


def vqe_problem_create(ctx, n_orb: int, n_elec: int, h1, eri, e_const: float = 0.0):
    h = _f64(h1).reshape(-1)
    e = _f64(eri).reshape(-1)
    p = C.c_void_p()
    _check(lib.vqe_problem_create(ctx, n_orb, n_elec, _dp(h), _dp(e), float(e_const), C.byref(p)))
    return p


def vqe_problem_destroy(p) -> None:
    _check(lib.vqe_problem_destroy(p))


def vqe_problem_info(p) -> dict:
    v = [C.c_int() for _ in range(5)]
    cid = C.c_double()
    _check(lib.vqe_problem_info(p, *[C.byref(x) for x in v], C.byref(cid)))
    keys = ["n_qubits", "n_params", "n_strings", "n_rotations", "n_gates"]
    out = {k: x.value for k, x in zip(keys, v)}
    out["identity_coeff"] = cid.value
    return out


def vqe_problem_paulis(p):
    n = vqe_problem_info(p)["n_strings"]
    x = np.zeros(n, dtype=np.uint64)
    z = np.zeros(n, dtype=np.uint64)
    c = np.zeros(n)
    _check(lib.vqe_problem_paulis(p, x.ctypes.data_as(_pu64), z.ctypes.data_as(_pu64), _dp(c)))
    return x, z, c


def vqe_problem_rotations(p):
    n = vqe_problem_info(p)["n_rotations"]
    x = np.zeros(n, dtype=np.uint64)
    z = np.zeros(n, dtype=np.uint64)
    c = np.zeros(n)
    par = np.zeros(n, dtype=np.int32)
    _check(lib.vqe_problem_rotations(p, x.ctypes.data_as(_pu64), z.ctypes.data_as(_pu64), _dp(c),
                                     par.ctypes.data_as(_pi)))
    return x, z, c, par


def vqe_problem_gates(p):
    n = vqe_problem_info(p)["n_gates"]
    site = np.zeros(n, dtype=np.int32)
    rot = np.zeros(n, dtype=np.int32)
    pre = np.zeros(n * 32)
    post = np.zeros(n * 32)
    _check(lib.vqe_problem_gates(p, site.ctypes.data_as(_pi), rot.ctypes.data_as(_pi), _dp(pre), _dp(post)))
    return site, rot, pre.view(np.complex128).reshape(n, 4, 4), post.view(np.complex128).reshape(n, 4, 4)


def vqe_energy(p, theta, max_bond: int, precision: int = Q2C_FP64):
    t = _f64(theta)
    e = C.c_double()
    st = q2c_stats()
    _check(lib.vqe_energy(p, _dp(t), len(t), max_bond, precision, C.byref(e), C.byref(st)))
    return e.value, st.as_dict()


def vqe_energy_batch(p, thetas, max_bond: int, precision: int = Q2C_FP64):
    t = _f64(thetas)
    nb, nt = t.shape
    out = np.zeros(nb)
    st = q2c_stats()
    _check(lib.vqe_energy_batch(p, _dp(t), nb, nt, max_bond, precision, _dp(out), C.byref(st)))
    return out, st.as_dict()


def vqe_grad_paramshift(p, theta, max_bond: int, precision: int = Q2C_FP64):
    t = _f64(theta)
    g = np.zeros(len(t))
    e = C.c_double()
    st = q2c_stats()
    _check(lib.vqe_grad_paramshift(p, _dp(t), len(t), max_bond, precision, _dp(g), C.byref(e), C.byref(st)))
    return g, e.value, st.as_dict()


def vqe_shift_energies(p, theta, rot_idx, max_bond: int, precision: int = Q2C_FP64):
    t = _f64(theta)
    r = np.ascontiguousarray(rot_idx, dtype=np.int32)
    ep = np.zeros(len(r))
    em = np.zeros(len(r))
    st = q2c_stats()
    _check(lib.vqe_shift_energies(p, _dp(t), len(t), r.ctypes.data_as(_pi), len(r), max_bond, precision,
                                  _dp(ep), _dp(em), C.byref(st)))
    return ep, em, st.as_dict()


def vqe_minimize(p, theta0, max_bond: int, precision: int = Q2C_FP64, **opts):
    """L-BFGS minimisation of E(theta) on the device: (theta, energy,
    energy_trace, report dict).  opts: fields of q2c_min_opts."""
    t = _f64(theta0)
    o = q2c_min_opts()
    for k, v in opts.items():
        setattr(o, k, v)
    n_tr = (o.max_iter if o.max_iter > 0 else 100) + 1
    out = np.zeros(len(t))
    trace = np.zeros(n_tr)
    e = C.c_double()
    rep = q2c_min_report()
    _check(lib.vqe_minimize(p, _dp(t), len(t), max_bond, precision, C.byref(o), _dp(out), C.byref(e), _dp(trace),
                            C.byref(rep)))
    return out, e.value, trace[: rep.iterations + 1].copy(), rep.as_dict()


def vqe_energy_hadamard(ctx, p, theta, max_bond: int, precision: int = Q2C_FP64, shared_state: bool = True,
                        string_idx=None):
    """Hadamard-test measurement, one circuit per string: (energy or None,
    expectations, seconds)."""
    t = _f64(theta)
    n_strings = vqe_problem_info(p)["n_strings"]
    idx = None if string_idx is None else np.ascontiguousarray(string_idx, dtype=np.int32)
    ev = np.zeros(n_strings if idx is None else len(idx))
    e = C.c_double(np.nan)
    sec = C.c_double()
    _check(lib.vqe_energy_hadamard(ctx, p, _dp(t), len(t), max_bond, precision, int(shared_state),
                                   None if idx is None else idx.ctypes.data_as(_pi), 0 if idx is None else len(idx),
                                   C.byref(e), _dp(ev), C.byref(sec)))
    return (e.value if idx is None else None), ev, sec.value


def mps_copy(src, dst) -> None:
    _check(lib.mps_copy(src, dst))


def vqe_problem_electrons(p):
    no, ne = C.c_int(), C.c_int()
    _check(lib.vqe_problem_electrons(p, C.byref(no), C.byref(ne)))
    return no.value, ne.value


def _lattice(n_sites: int, frag_size: int, n_elec: int, h, U: float):
    hh = _f64(h).reshape(-1)
    if hh.size != n_sites * n_sites:
        raise ValueError("h must be n_sites x n_sites")
    return q2c_lattice(n_sites, frag_size, n_elec, _dp(hh), float(U)), hh


def dmet_embedding(n_sites: int, frag_size: int, n_elec: int, h, U: float, frag: int, mu: float = 0.0):
    """Host-side embedded problem of one fragment: dict of orbitals (L x 2k),
    h1, eri, nop, efrag_h1."""
    lat, keep = _lattice(n_sites, frag_size, n_elec, h, U)
    m = 2 * frag_size
    out = {"orbitals": np.zeros((n_sites, m)), "h1": np.zeros((m, m)), "eri": np.zeros((m,) * 4),
           "nop": np.zeros((m, m)), "efrag_h1": np.zeros((m, m))}
    _check(lib.dmet_embedding(C.byref(lat), frag, float(mu), _dp(out["orbitals"]), _dp(out["h1"]), _dp(out["eri"]),
                              _dp(out["nop"]), _dp(out["efrag_h1"])))
    del keep
    return out


def dmet_solve(ctx, n_sites: int, frag_size: int, n_elec: int, h, U: float, mu_lo: float = 0.0, mu_hi: float = 0.0,
               n_tol: float = 0.0, max_iter: int = 0, max_bond: int = 0, precision: int = Q2C_FP64, workers: int = 0,
               **vqe_opts):
    """DMET chemical-potential loop on the device: dict with n_frag, e_frag,
    e_emb (per fragment), mu_trace and the report fields."""
    lat, keep = _lattice(n_sites, frag_size, n_elec, h, U)
    o = q2c_dmet_opts()
    o.mu_lo, o.mu_hi, o.n_tol, o.max_iter, o.max_bond, o.precision = mu_lo, mu_hi, n_tol, max_iter, max_bond, precision
    o.workers = workers
    for k, v in vqe_opts.items():
        setattr(o.vqe, k, v)
    nf = n_sites // frag_size
    res = {"n_frag": np.zeros(nf), "e_frag": np.zeros(nf), "e_emb": np.zeros(nf)}
    trace = np.full((max_iter if max_iter > 0 else 40) + 2, np.nan)
    rep = q2c_dmet_report()
    _check(lib.dmet_solve(ctx, C.byref(lat), C.byref(o), _dp(res["n_frag"]), _dp(res["e_frag"]), _dp(res["e_emb"]),
                          _dp(trace), C.byref(rep)))
    del keep
    res["mu_trace"] = trace[~np.isnan(trace)]
    res.update(rep.as_dict())
    return res


# ------------------------------------------------------------- handle classes


class Context:
    def __init__(self, device: int = 0, hip_stream: int | None = None, **opts):
        o = q2c_opts()
        for k, v in opts.items():
            if isinstance(v, str):
                v = v.encode()  # the library copies the string during the call
            setattr(o, k, v)
        self.h = q2c_ctx_create(device, hip_stream, o)

    def close(self):
        if self.h:
            q2c_ctx_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Problem:
    def __init__(self, ctx: Context | None, n_orb: int, n_elec: int, h1, eri, e_const: float = 0.0):
        self.ctx = ctx
        self.h = vqe_problem_create(ctx.h if ctx else None, n_orb, n_elec, h1, eri, e_const)
        self.info = vqe_problem_info(self.h)

    def close(self):
        if self.h:
            vqe_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def energy(self, theta, max_bond: int, precision: int = Q2C_FP64):
        return vqe_energy(self.h, theta, max_bond, precision)

    def energy_batch(self, thetas, max_bond: int, precision: int = Q2C_FP64):
        return vqe_energy_batch(self.h, thetas, max_bond, precision)

    def grad(self, theta, max_bond: int, precision: int = Q2C_FP64):
        return vqe_grad_paramshift(self.h, theta, max_bond, precision)

    def shift_energies(self, theta, rot_idx, max_bond: int, precision: int = Q2C_FP64):
        return vqe_shift_energies(self.h, theta, rot_idx, max_bond, precision)

    def minimize(self, theta0, max_bond: int, precision: int = Q2C_FP64, **opts):
        return vqe_minimize(self.h, theta0, max_bond, precision, **opts)


class MPS:
    def __init__(self, ctx: Context, occ, max_bond: int, precision: int = Q2C_FP64):
        self.n = len(occ)
        self.h = mps_create(ctx.h, self.n, max_bond, precision, occ)

    def close(self):
        if self.h:
            mps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_gate(self, site: int, gate) -> float:
        return mps_apply_gate(self.h, site, gate)

    def expect(self, x_masks, z_masks):
        return mps_expect_pauli_batch(self.h, x_masks, z_masks, self.n)

    def export(self):
        return mps_export(self.h, self.n)

    def stats(self) -> dict:
        return mps_get_stats(self.h)


# ------------------------------------------------------------------- serving


def q2c_server_create(ctx, opts=None):
    h = _vp()
    _check(lib.q2c_server_create(ctx, C.byref(opts) if opts is not None else None, C.byref(h)))
    return h


def q2c_server_destroy(srv):
    _check(lib.q2c_server_destroy(srv))


def q2c_server_submit(srv, tag: int, n_orb: int, n_elec: int, h1, eri, e_const: float, theta, max_bond: int,
                      precision: int = Q2C_FP64, n_frag_orb: int = 0):
    h = _f64(h1)
    e = _f64(eri)
    t = _f64(theta)
    _check(lib.q2c_server_submit(srv, tag, n_orb, n_elec, _dp(h), _dp(e), e_const, _dp(t), len(t), max_bond,
                                 precision, n_frag_orb))


def q2c_server_step(srv):
    q, a, r = C.c_int(), C.c_int(), C.c_int()
    _check(lib.q2c_server_step(srv, C.byref(q), C.byref(a), C.byref(r)))
    return q.value, a.value, r.value


def q2c_server_poll(srv, max_out: int = 256):
    buf = (q2c_result * max_out)()
    n = C.c_int()
    _check(lib.q2c_server_poll(srv, buf, max_out, C.byref(n)))
    return [buf[i].as_dict() for i in range(n.value)]


class Server:
    """Continuous-batching request server (argument marshalling only)."""

    def __init__(self, ctx: Context, slots_per_class: int = 64, gates_per_step: int = 1024):
        o = q2c_server_opts(slots_per_class, gates_per_step)
        self.h = q2c_server_create(ctx.h, o)

    def submit(self, tag, n_orb, n_elec, h1, eri, e_const, theta, max_bond, precision=Q2C_FP64, n_frag_orb=0):
        q2c_server_submit(self.h, tag, n_orb, n_elec, h1, eri, e_const, theta, max_bond, precision, n_frag_orb)

    def step(self):
        return q2c_server_step(self.h)

    def poll(self, max_out: int = 256):
        return q2c_server_poll(self.h, max_out)

    def close(self):
        if self.h:
            q2c_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
