// Host-side problem compiler: integrals -> Jordan-Wigner Pauli strings,
// UCCSD excitations -> Pauli rotations -> fused nearest-neighbour gates.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace q2c {

using cplx = std::complex<double>;

struct PauliTerm {
  uint64_t x = 0, z = 0;  // bit k = qubit k
  double c = 0.0;
};

struct Rotation {
  uint64_t x = 0, z = 0;
  double c = 0.0;  // phi = -2 c theta[param]
  int param = 0;
  int lo = 0, hi = 0;  // support
};

// A two-qubit gate on (site, site+1).  rot < 0: constant, matrix = pre.
// rot >= 0: matrix = post * kron(I, RZ(phi[rot])) * pre.  Row-major 4x4,
// basis index 2*i_site + i_{site+1}.
struct Gate {
  int site = 0;
  int rot = -1;
  cplx pre[16];
  cplx post[16];
};

struct Problem {
  int n_orb = 0, n_elec = 0, n_qubits = 0;
  double e_const = 0.0;
  double c_identity = 0.0;  // coefficient of the identity string, e_const included
  std::vector<PauliTerm> terms;  // ascending (x, z), identity excluded
  int n_params = 0;
  std::vector<Rotation> rotations;
  std::vector<Gate> gates;
};

// Throws std::invalid_argument on bad input.
Problem compile_problem(int n_orb, int n_elec, const double* h1, const double* eri, double e_const);

// Prefix order of Pauli strings for the transfer sweeps: strings sorted by
// their lowest non-identity site, then by their letters site by site upward
// (the identity string first).  share[t] = number of leading transfer steps
// (sites from that lowest site on) that sorted string t has in common with
// sorted string t - 1; 0 for t = 0, for a different lowest site and for
// either string being the identity.  Never more than the length of either.
struct PrefixOrder {
  std::vector<int> order;  // sorted position -> input index
  std::vector<int> share;  // per sorted position
  long steps_plain = 0;    // transfer steps without reuse
  long steps_shared = 0;   // with reuse along the whole order
};
PrefixOrder pauli_prefix_order(const uint64_t* x, const uint64_t* z, int n);

}  // namespace q2c
