"""CPU oracle for the MPS-VQE energy path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct CPU implementations (numpy, complex128/float64)
of what the GPU library computes, written from the paper's definitions:

  fermion.py     Pauli-string algebra and the Jordan-Wigner transform of the
                 second-quantised Hamiltonian (Eq. 1 -> Eq. 2).
  uccsd.py       UCCSD excitations (Eq. 3-4), their first-order Trotter
                 product of Pauli rotations, and the nearest-neighbour gate
                 compile with single-qubit gates fused into two-qubit gates.
  statevector.py Dense 2^N state: rotations, energy, adjoint and
                 parameter-shift gradients.
  fockspace.py   Determinant-space (occupation-number) Hamiltonian and UCCSD,
                 written with fermionic sign rules only -- no Pauli algebra --
                 used to pin the Jordan-Wigner signs.
  mps.py         Right-canonical MPS with the two-site update of Eq. 7-10
                 (LAPACK SVD, truncation to D) and exact environment-based
                 Pauli expectations.
  exact.py       Brute-force ground-state energy (variational bound).
  minimize.py    Local minimum of the UCCSD energy (the VQE outer loop's
                 result) by a library minimiser on the exact gradient.
  dmet.py        DMET chemical-potential loop (mean-field bath, embedded
                 Hamiltonian, fragment electrons) around a UCCSD or exact
                 fragment solver.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  The product library never calls it, and it
imports nothing from the product package: the two share only the seeded input
generators in ``workloads``.

Parity status: every function here is pinned by an independent check in
``tests/test_oracle_*.py`` (closed forms, a second independent construction,
brute force on small inputs, or counts the paper prints).  The energy of an
MPS truncated below full bond dimension has no closed form: it is pinned only
through the pinned pieces it is built from (the full-D equality with the
statevector, canonical-form and norm invariants, the variational bound).
"""
