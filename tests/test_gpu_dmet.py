"""GPU: the DMET chemical-potential loop (dmet_solve: host embedding, device
VQE fragment solves) against the oracle's loop with the state-vector UCCSD
solver.  Fragment minima agree to the VQE tolerance, so the chemical
potential, the fragments' electrons and energies agree to about 1e-6."""
import numpy as np
import pytest

from oracle import dmet
from workloads import random_lattice

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q2c():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_03711_amd import q2c as mod

    return mod


def _gpu(q2c, lat, **kw):
    ctx = q2c.Context(0, slots=128, grad_rule=1)
    try:
        r = q2c.dmet_solve(ctx.h, lat.n_sites, lat.frag_size, lat.n_elec, lat.h, lat.U, gtol=1e-8, **kw)
    finally:
        ctx.close()
    print(f"dmet L={lat.n_sites} k={lat.frag_size} U={lat.U}: mu {r['mu']:.9f} status {r['status']} "
          f"steps {r['iterations']} vqe runs {r['vqe_runs']} {r['seconds']:.1f}s", flush=True)
    return r


@pytest.mark.parametrize("n_sites,k,seed", [(8, 1, 5), (4, 2, 9)])
def test_dmet_matches_oracle(q2c, n_sites, k, seed):
    lat = random_lattice(n_sites, k, n_sites, seed, U=4.0)
    r = _gpu(q2c, lat, mu_lo=0.0, mu_hi=4.0)
    ref = dmet.dmet(lat, "uccsd", mu_lo=0.0, mu_hi=4.0)
    assert r["status"] == ref.status == 1
    assert abs(r["mu"] - ref.mu) < 1e-5
    assert np.max(np.abs(r["n_frag"] - ref.n_frag)) < 1e-5
    assert abs(r["n_frag"].sum() - lat.n_elec) < 1e-6
    assert np.max(np.abs(r["e_frag"] - ref.e_frag)) < 1e-5
    assert abs(r["e_dmet"] - ref.e_frag.sum()) < 1e-5
    assert np.max(np.abs(r["e_emb"] - ref.e_emb)) < 1e-5
    assert r["mu_trace"][0] == 0.0 and r["mu_trace"][1] == 4.0


def test_dmet_workers_do_not_change_results(q2c):
    """Fragments solved one at a time and eight at a time (each worker on a
    context of its own) give the same results bit for bit."""
    lat = random_lattice(8, 1, 8, 5, U=4.0)
    r1 = _gpu(q2c, lat, mu_lo=0.0, mu_hi=4.0, workers=1)
    r8 = _gpu(q2c, lat, mu_lo=0.0, mu_hi=4.0)
    assert r1["mu"] == r8["mu"] and r1["iterations"] == r8["iterations"]
    for k in ("n_frag", "e_frag", "e_emb", "mu_trace"):
        assert np.array_equal(r1[k], r8[k]), k


def test_dmet_without_interaction_is_exact(q2c):
    """U = 0: the loop stops at mu = 0 with the mean-field fragment electrons."""
    lat = random_lattice(8, 1, 8, 5, U=0.0)
    r = _gpu(q2c, lat)
    assert r["status"] == 1 and abs(r["mu"]) < 1e-5
    occ = 2.0 * np.diag(dmet.mean_field_density(lat))
    assert np.max(np.abs(r["n_frag"] - occ)) < 1e-5
