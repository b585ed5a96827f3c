// The paper's own measurement of the energy (Sec. III-A after Eq. 11, and
// Sec. III-D with the H2 circuits): one circuit per Pauli string -- the
// Hartree-Fock preparation, the UCCSD ansatz, then a Hadamard test on one
// ancillary qubit placed after the last qubit: the ancilla in |+>, the string
// applied under the ancilla's control, and <X> of the ancilla, which equals
// Re <psi|P|psi>.  It is kept as the baseline the transfer-matrix sweeps
// replace, and as a cross-check of their values.
//
// On the MPS the ancilla is the extra site n.  It travels down to the
// string's first qubit lo by nearest-neighbour gates: the gate on (j, j+1),
// j = n-1 .. lo, applies the letter of qubit j controlled by the ancilla on
// site j+1, then swaps the two sites (a plain swap for identity letters), so
// a string costs n - lo two-site updates and leaves the ancilla on site lo.
// The bond dimension must hold the ancilla's two branches (up to twice that
// of the ansatz state) for the test to be exact.
//
// shared_state = 0 runs every string's whole circuit, as the paper's
// simulator does (its memory-efficient scheme shares the ansatz circuit, not
// the state); shared_state = 1 prepares the ansatz state once and copies it
// on the device for each string.  Both give the same values bit for bit.
// Everything goes through the public calls of this library.
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "runtime.hpp"

using namespace q2c_rt;

namespace {

void call(int rc) {
  if (rc != Q2C_OK) throw StatusError(rc, g_last_error);
}

using C = std::complex<double>;

struct Mps {
  mps_state* s = nullptr;
  Mps() = default;
  Mps(const Mps&) = delete;
  Mps& operator=(const Mps&) = delete;
  ~Mps() {
    if (s) mps_destroy(s);
  }
};

// 4x4 complex gate as the 32 interleaved doubles mps_apply_gate takes
std::vector<double> pack(const C (&g)[4][4]) {
  std::vector<double> v(32);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      v[2 * (4 * i + j)] = g[i][j].real();
      v[2 * (4 * i + j) + 1] = g[i][j].imag();
    }
  return v;
}

// Gate on (data qubit j, ancilla on j+1): controlled letter, then swap.
// Basis index 2 i_j + i_{j+1}; letter 0 I, 1 X, 2 Z, 3 Y.
std::vector<double> ctrl_swap(int letter) {
  C s[2][2] = {{1, 0}, {0, 1}};
  if (letter == 1) {
    s[0][0] = 0; s[0][1] = 1; s[1][0] = 1; s[1][1] = 0;
  } else if (letter == 2) {
    s[1][1] = -1;
  } else if (letter == 3) {
    s[0][0] = 0; s[0][1] = C(0, -1); s[1][0] = C(0, 1); s[1][1] = 0;
  }
  C cg[4][4] = {};
  for (int d = 0; d < 2; ++d)
    for (int dp = 0; dp < 2; ++dp) {
      cg[2 * dp][2 * d] = d == dp ? 1.0 : 0.0;  // ancilla 0: identity on the data qubit
      cg[2 * dp + 1][2 * d + 1] = s[dp][d];      // ancilla 1: the letter
    }
  C g[4][4] = {};
  for (int r = 0; r < 4; ++r)  // swap: row (d', a') <- (a', d')
    for (int c = 0; c < 4; ++c) g[r][c] = cg[2 * (r & 1) + (r >> 1)][c];
  return pack(g);
}

}  // namespace

extern "C" {

int vqe_energy_hadamard(q2c_ctx* ctx, vqe_problem* p, const double* theta, int n_theta, int max_bond,
                        int precision, int shared_state, const int* string_idx, int n_idx, double* energy,
                        double* expect, double* seconds) {
  return guarded([&] {
    if (!ctx || !p || !theta) throw ArgError("ctx, problem or theta is NULL");
    int nq = 0, np = 0, ns = 0, nr = 0, ng = 0;
    double cid = 0.0;
    call(vqe_problem_info(p, &nq, &np, &ns, &nr, &ng, &cid));
    if (n_theta != np) throw ArgError("n_theta does not match the problem's parameter count");
    if (nq + 1 > 64) throw ArgError("the ancilla needs n_qubits <= 63");
    for (int k = 0; k < np; ++k)
      if (!std::isfinite(theta[k])) throw ArgError("theta holds a non-finite value");
    std::vector<int> idx;
    if (string_idx) {
      if (n_idx < 1) throw ArgError("n_idx must be >= 1");
      for (int i = 0; i < n_idx; ++i) {
        if (string_idx[i] < 0 || string_idx[i] >= ns) throw ArgError("string index out of range");
        idx.push_back(string_idx[i]);
      }
    } else {
      for (int i = 0; i < ns; ++i) idx.push_back(i);
    }
    const auto t0 = std::chrono::steady_clock::now();
    // compiled problem: strings, rotations, gates
    std::vector<uint64_t> x(ns), z(ns), rx(nr), rz(nr);
    std::vector<double> coef(ns), rc(nr), pre(size_t(ng) * 32), post(size_t(ng) * 32);
    std::vector<int> rpar(nr), gsite(ng), grot(ng);
    call(vqe_problem_paulis(p, x.data(), z.data(), coef.data()));
    call(vqe_problem_rotations(p, rx.data(), rz.data(), rc.data(), rpar.data()));
    call(vqe_problem_gates(p, gsite.data(), grot.data(), pre.data(), post.data()));
    std::vector<std::vector<double>> ansatz(ng, std::vector<double>(32));
    for (int g = 0; g < ng; ++g) {
      if (grot[g] < 0) {
        std::copy(pre.begin() + size_t(g) * 32, pre.begin() + size_t(g) * 32 + 32, ansatz[g].begin());
        continue;
      }
      // the apex gate: post (I x RZ(phi)) pre, phi = -2 c theta_k
      const int m = grot[g];
      const double phi = -2.0 * rc[m] * theta[rpar[m]];
      const C dm(std::cos(0.5 * phi), -std::sin(0.5 * phi)), dp(std::cos(0.5 * phi), std::sin(0.5 * phi));
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          C s = 0.0;
          for (int k = 0; k < 4; ++k) {
            const C po(post[size_t(g) * 32 + 2 * (4 * i + k)], post[size_t(g) * 32 + 2 * (4 * i + k) + 1]);
            const C pr(pre[size_t(g) * 32 + 2 * (4 * k + j)], pre[size_t(g) * 32 + 2 * (4 * k + j) + 1]);
            s += po * ((k & 1) ? dp : dm) * pr;
          }
          ansatz[g][2 * (4 * i + j)] = s.real();
          ansatz[g][2 * (4 * i + j) + 1] = s.imag();
        }
    }
    int ne = 0;
    call(vqe_problem_electrons(p, nullptr, &ne));
    const int n = nq + 1;  // data qubits 0 .. nq-1, ancilla on site nq
    std::vector<uint8_t> occ(n, 0);
    for (int q = 0; q < ne; ++q) occ[q] = 1;
    // ancilla |0> -> |+>: identity on qubit nq-1, Hadamard on the ancilla
    std::vector<double> hgate(32, 0.0);
    {
      const double r = 1.0 / std::sqrt(2.0);
      const double hm[2][2] = {{r, r}, {r, -r}};
      for (int d = 0; d < 2; ++d)
        for (int a = 0; a < 2; ++a)
          for (int ap = 0; ap < 2; ++ap) hgate[2 * (4 * (2 * d + ap) + (2 * d + a))] = hm[ap][a];
    }
    std::vector<std::vector<double>> cs(4);
    for (int l = 0; l < 4; ++l) cs[l] = ctrl_swap(l);
    Mps base, work;
    auto prepare = [&](mps_state* s) {
      call(mps_apply_gate(s, nq - 1, hgate.data(), nullptr));
      for (int g = 0; g < ng; ++g) call(mps_apply_gate(s, gsite[g], ansatz[g].data(), nullptr));
    };
    call(mps_create(ctx, n, max_bond, precision, occ.data(), &work.s));
    if (shared_state) {
      call(mps_create(ctx, n, max_bond, precision, occ.data(), &base.s));
      prepare(base.s);
    }
    std::vector<double> ev(idx.size());
    for (size_t t = 0; t < idx.size(); ++t) {
      const int i = idx[t];
      if (shared_state) {
        call(mps_copy(base.s, work.s));
      } else {
        Mps fresh;
        call(mps_create(ctx, n, max_bond, precision, occ.data(), &fresh.s));
        prepare(fresh.s);
        call(mps_copy(fresh.s, work.s));
      }
      const uint64_t sup = x[i] | z[i];
      int lo = 0;
      while (lo < nq && !((sup >> lo) & 1)) ++lo;
      for (int j = nq - 1; j >= lo; --j) {
        const int letter = int((x[i] >> j) & 1) | (int((z[i] >> j) & 1) << 1);  // 0 I, 1 X, 2 Z, 3 Y
        call(mps_apply_gate(work.s, j, cs[letter].data(), nullptr));
      }
      const uint64_t ax = uint64_t(1) << lo, az = 0;
      double re = 0.0;
      call(mps_expect_pauli_batch(work.s, 1, 1, &ax, &az, &re, nullptr));
      ev[t] = re;
    }
    if (!string_idx && energy) {
      // Neumaier sum in the strings' order, the identity coefficient last
      double sum = 0.0, comp = 0.0;
      auto add = [&](double v) {
        const double t2 = sum + v;
        comp += std::fabs(sum) >= std::fabs(v) ? (sum - t2) + v : (v - t2) + sum;
        sum = t2;
      };
      for (int t = 0; t < ns; ++t) add(coef[t] * ev[t]);
      add(cid);
      *energy = sum + comp;
    }
    if (expect) std::copy(ev.begin(), ev.end(), expect);
    if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  });
}

}  // extern "C"
