"""Write tests/golden/reference_energies.json from the CPU oracle only.

Run from the repository root:  python tests/golden/make_reference.py [names...]
Each entry records the oracle's MPS energy at the stated bond dimension (and
the state-vector energy where it is affordable), the truncation statistics,
and -- for truncated runs -- the energy obtained with a second LAPACK SVD
driver, whose difference bounds what rounding alone does to the trajectory.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fermion, mps as om, statevector as sv, uccsd  # noqa: E402
from workloads import random_integrals, random_theta, n_uccsd_params  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "reference_energies.json")

# name: (n_orb, n_elec, int_seed, theta_seed, D, statevector?, second driver?)
CASES = {
    "q8_d16": (4, 4, 1001, 1002, 16, True, False),
    "q8_d4": (4, 4, 1001, 1002, 4, False, True),
    "q12_d16": (6, 6, 1201, 1202, 16, True, True),
    "q16_d64": (8, 8, 2001, 2002, 64, False, True),
}


def statevector_energy(name):
    n_orb, n_elec, si, st, D, _, _ = CASES[name]
    I = random_integrals(n_orb, n_elec, si)
    th = random_theta(n_uccsd_params(n_orb, n_elec), st)
    n = 2 * n_orb
    c_id, terms = fermion.hamiltonian_terms(fermion.jw_hamiltonian(I.h1, I.eri))
    rots = uccsd.rotations(n, n_elec)
    phis = uccsd.rotation_angles(rots, th)
    pa = sv.PauliApplier(n)
    psi = sv.evolve(n, uccsd.hf_occupation(n, n_elec), rots, phis, pa)
    return sv.energy(pa, c_id, terms, psi)


def run(name):
    n_orb, n_elec, si, st, D, do_sv, second = CASES[name]
    I = random_integrals(n_orb, n_elec, si)
    th = random_theta(n_uccsd_params(n_orb, n_elec), st)
    n = 2 * n_orb
    c_id, terms = fermion.hamiltonian_terms(fermion.jw_hamiltonian(I.h1, I.eri))
    rots, gates = uccsd.compile_fused(n, n_elec)
    phis = uccsd.rotation_angles(rots, th)
    occ = uccsd.hf_occupation(n, n_elec)
    t0 = time.time()
    m = om.run_circuit(n, occ, gates, phis, D)
    e, imag = om.energy(m, c_id, terms)
    rec = {
        "n_orb": n_orb, "n_elec": n_elec, "int_seed": si, "theta_seed": st, "max_bond": D,
        "n_strings": len(terms), "n_gates": len(gates),
        "energy_mps": e, "max_abs_imag": imag,
        "discarded_weight_sum": m.discarded, "max_discarded": m.max_discarded,
        "min_cut_gap_rel": None if not np.isfinite(m.min_gap_rel) else m.min_gap_rel,
        "chi": [m.chi(b) for b in range(n - 1)],
        "oracle_seconds": time.time() - t0,
    }
    if second:
        m2 = om.run_circuit(n, occ, gates, phis, D, svd="gesvd")
        e2, _ = om.energy(m2, c_id, terms)
        rec["energy_mps_gesvd"] = e2
    if do_sv:
        psi = sv.evolve(n, occ, rots, phis)
        rec["energy_statevector"] = sv.energy(sv.PauliApplier(n), c_id, terms, psi)
    return rec


if __name__ == "__main__":
    args = sys.argv[1:]
    sv_only = "--statevector-only" in args
    names = [a for a in args if not a.startswith("--")] or list(CASES)
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data["_source"] = "written by tests/golden/make_reference.py from oracle/ only"
    for nm in names:
        print("running", nm, flush=True)
        if sv_only:
            data.setdefault(nm, {})["energy_statevector"] = statevector_energy(nm)
        else:
            data[nm] = run(nm)
        print(json.dumps(data[nm]), flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
