"""GPU: the request server (continuous batching of fragment solves).

Requests of several classes (qubit count, D, precision) are submitted in two
waves -- the second while the first is on the device -- into classes with
fewer slots than requests, so slots are reused.  Every served energy must be
bit-for-bit the energy of the same problem run alone through vqe_energy, and
at full bond dimension the energy and the fragment occupation must match the
state-vector oracle.
"""
import time

import numpy as np
import pytest

from oracle import fermion, statevector as sv, uccsd
from workloads import serving_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q2c():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_03711_amd import q2c as mod

    return mod


def _oracle(I, th, k):
    n = 2 * I.n_orb
    c_id, terms = fermion.hamiltonian_terms(fermion.jw_hamiltonian(I.h1, I.eri, I.e_const))
    rots = uccsd.rotations(n, I.n_elec)
    pa = sv.PauliApplier(n)
    psi = sv.evolve(n, uccsd.hf_occupation(n, I.n_elec), rots, uccsd.rotation_angles(rots, th), pa)
    e = sv.energy(pa, c_id, terms, psi)
    nf = sum(0.5 * (1.0 - sv.energy(pa, 0.0, [(0, 1 << q, 1.0)], psi)) for q in range(2 * k))
    return e, nf


def test_served_results_equal_alone(q2c):
    reqs = serving_stream(12, seed=77, k_range=(1, 2), bonds=(2, 4, 16))
    jobs = [(r.index, r, q2c.Q2C_FP64) for r in reqs] + [(100 + r.index, r, q2c.Q2C_MIXED) for r in reqs[:3]]
    ctx = q2c.Context(0)
    srv = q2c.Server(ctx, slots_per_class=3, gates_per_step=64)

    def submit(tag, r, prec):
        I = r.integrals()
        srv.submit(tag, I.n_orb, I.n_elec, I.h1, I.eri, I.e_const, r.theta(), r.max_bond, prec, r.n_frag_orb)

    for j in jobs[:7]:
        submit(*j)
    results, steps, t0 = {}, 0, time.time()
    while len(results) < len(jobs):
        q, a, n = srv.step()
        steps += 1
        if steps == 3:
            assert a > 0  # the second wave joins while the first is running
            for j in jobs[7:]:
                submit(*j)
        for res in srv.poll():
            results[res["tag"]] = res
        assert time.time() - t0 < 300
    srv.close()

    for tag, r, prec in jobs:
        res = results[tag]
        assert res["status"] == 0
        assert res["submit_s"] <= res["admit_s"] <= res["done_s"]
        I, th = r.integrals(), r.theta()
        p = q2c.Problem(ctx, I.n_orb, I.n_elec, I.h1, I.eri, I.e_const)
        e_alone, _ = p.energy(th, r.max_bond, precision=prec)
        p.close()
        assert abs(res["energy"] - e_alone) <= 1e-13, (tag, res["energy"], e_alone)
        n = 2 * I.n_orb
        if r.max_bond >= 2 ** (n // 2) and prec == q2c.Q2C_FP64:
            e_ref, nf_ref = _oracle(I, th, r.n_frag_orb)
            assert abs(res["energy"] - e_ref) < 1e-10
            assert abs(res["n_frag"] - nf_ref) < 1e-10
    ctx.close()


def test_server_rejects_bad_requests(q2c):
    ctx = q2c.Context(0)
    srv = q2c.Server(ctx)
    r = serving_stream(1, seed=3, k_range=(1, 1), bonds=(4,))[0]
    I = r.integrals()
    with pytest.raises(q2c.Q2CError):
        srv.submit(0, I.n_orb, I.n_elec, I.h1, I.eri, I.e_const, r.theta()[:-1], 4)  # wrong theta length
    with pytest.raises(q2c.Q2CError):
        srv.submit(0, I.n_orb, I.n_elec, I.h1, I.eri, I.e_const, r.theta(), 0)  # bad D
    with pytest.raises(q2c.Q2CError):
        srv.submit(0, I.n_orb, I.n_elec, I.h1, I.eri, I.e_const, r.theta(), 4, n_frag_orb=I.n_orb + 1)
    assert srv.step() == (0, 0, 0)
    srv.close()
    ctx.close()


def test_idle_classes_evicted_under_budget(q2c):
    """Idle request classes stay allocated for later requests of their shape;
    a new class that does not fit the context's HBM budget evicts idle
    classes, least recently used first.  The peak memory of one class (4
    qubits, D = 4) is measured; under a budget of 1.3 times that, requests of
    D = 4, 3 and 2 served one after another all complete (the second needs
    the first class evicted), within the budget, and each result equals the
    same problem run alone."""
    from workloads import ServingRequest

    reqs = [ServingRequest(i, 1, D, 0.2, 0.0) for i, D in enumerate((4, 3, 2))]

    def serve(ctx, srv, r, watch=None):
        I = r.integrals()
        srv.submit(r.index, I.n_orb, I.n_elec, I.h1, I.eri, I.e_const, r.theta(), r.max_bond, q2c.Q2C_FP64,
                   r.n_frag_orb)
        t0 = time.time()
        while True:
            srv.step()
            if watch is not None:
                watch.append(q2c.q2c_ctx_memory(ctx.h)[0])
            out = srv.poll()
            if out:
                return out[0]
            assert time.time() - t0 < 60, "request never admitted"

    ctx0 = q2c.Context(0)
    srv0 = q2c.Server(ctx0, slots_per_class=2, gates_per_step=64)
    base = q2c.q2c_ctx_memory(ctx0.h)[0]
    seen = []
    serve(ctx0, srv0, reqs[0], seen)
    peak = max(seen) - base
    srv0.close()
    ctx0.close()
    assert peak > 0

    budget = base + int(1.3 * peak)
    ctx = q2c.Context(0, hbm_budget_bytes=budget)
    ctx_alone = q2c.Context(0)  # reference runs outside the budget
    srv = q2c.Server(ctx, slots_per_class=2, gates_per_step=64)
    used = []
    for r in reqs:
        res = serve(ctx, srv, r, used)
        assert res["status"] == 0
        I = r.integrals()
        p = q2c.Problem(ctx_alone, I.n_orb, I.n_elec, I.h1, I.eri, I.e_const)
        e_alone, _ = p.energy(r.theta(), r.max_bond)
        p.close()
        assert res["energy"] == e_alone, r.max_bond
    assert max(used) <= budget
    srv.close()
    ctx.close()
    ctx_alone.close()
