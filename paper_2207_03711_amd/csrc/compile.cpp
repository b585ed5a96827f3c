// Host problem compiler.
//
// * Hamiltonian (Eq. 1, chemist notation) -> Jordan-Wigner Pauli strings
//   (Eq. 2).  Each fermionic monomial is mapped qubit by qubit: ladder
//   operator a(+)_P is Z on every qubit below P, sigma(+/-) on qubit P and
//   the identity above, so the monomial's factor on qubit k is the ordered
//   product of 2x2 matrices contributed by each operator; that 2x2 is then
//   expanded in {I, X, Y, Z} and the tensor product of the expansions gives
//   the Pauli strings.
// * UCCSD (Eq. 3-4): singles a+_a a_i and doubles a+_a a+_b a_i a_j over
//   interleaved spin-orbitals, one parameter each, in (i, a) then (i, j, a, b)
//   order; tau - tau^dag = i sum_m c_m P_m and every P_m becomes the rotation
//   exp(-i phi_m P_m / 2) with phi_m = -2 c_m theta (first-order Trotter, the
//   first parameter acting first).
// * Nearest-neighbour compile (Sec. III-A gate fusion): basis changes (X: H,
//   Y: H S^dag), a CNOT ladder up the support with SWAPs across identity
//   qubits, RZ on the top qubit, the mirrored ladder and the undo; each
//   single-qubit gate fused into the first/last two-qubit gate touching its
//   qubit; the top ladder gates and the RZ fused into one angle-dependent
//   gate.  2(hi-lo)-1 gates per rotation.
#include "compile.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <unordered_map>

namespace q2c {
namespace {

struct Key {
  uint64_t x, z;
  bool operator==(const Key& o) const { return x == o.x && z == o.z; }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = k.x * 0x9E3779B97F4A7C15ull ^ (k.z + 0x632BE59BD9B4E019ull + (k.x << 6) + (k.x >> 2));
    return static_cast<size_t>(h ^ (h >> 31));
  }
};
using PauliMap = std::unordered_map<Key, cplx, KeyHash>;

struct M2 {
  cplx a[2][2];
};
M2 m2_identity() { return M2{{{1.0, 0.0}, {0.0, 1.0}}}; }
M2 m2_mul(const M2& p, const M2& q) {
  M2 r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r.a[i][j] = p.a[i][0] * q.a[0][j] + p.a[i][1] * q.a[1][j];
  return r;
}
const M2 kZ{{{1.0, 0.0}, {0.0, -1.0}}};
const M2 kRaise{{{0.0, 0.0}, {1.0, 0.0}}};  // |1><0|: creates an electron
const M2 kLower{{{0.0, 1.0}, {0.0, 0.0}}};  // |0><1|

struct Ladder {
  bool create;
  int P;
};

// Adds coef * (JW image of the ordered monomial) to out.
void add_monomial(const std::vector<Ladder>& ops, cplx coef, PauliMap& out) {
  int top = 0;
  for (const auto& o : ops) top = std::max(top, o.P);
  // per-qubit Pauli expansion: up to 4 (pauli, coefficient) entries
  struct Comp {
    int x, z;
    cplx c;
  };
  std::vector<std::vector<Comp>> qcomp(top + 1);
  for (int k = 0; k <= top; ++k) {
    M2 m = m2_identity();
    for (const auto& o : ops) {
      if (k < o.P)
        m = m2_mul(m, kZ);
      else if (k == o.P)
        m = m2_mul(m, o.create ? kRaise : kLower);
    }
    const cplx cI = 0.5 * (m.a[0][0] + m.a[1][1]);
    const cplx cZ = 0.5 * (m.a[0][0] - m.a[1][1]);
    const cplx cX = 0.5 * (m.a[0][1] + m.a[1][0]);
    const cplx cY = cplx(0.0, 0.5) * (m.a[0][1] - m.a[1][0]);
    auto& v = qcomp[k];
    if (std::abs(cI) > 0) v.push_back({0, 0, cI});
    if (std::abs(cX) > 0) v.push_back({1, 0, cX});
    if (std::abs(cY) > 0) v.push_back({1, 1, cY});
    if (std::abs(cZ) > 0) v.push_back({0, 1, cZ});
    if (v.empty()) return;  // the monomial vanishes (e.g. a_P a_P)
  }
  // tensor-product expansion
  struct Partial {
    uint64_t x, z;
    cplx c;
  };
  std::vector<Partial> acc{{0, 0, coef}}, nxt;
  for (int k = 0; k <= top; ++k) {
    nxt.clear();
    for (const auto& p : acc)
      for (const auto& q : qcomp[k])
        nxt.push_back({p.x | (uint64_t(q.x) << k), p.z | (uint64_t(q.z) << k), p.c * q.c});
    acc.swap(nxt);
  }
  for (const auto& p : acc) out[Key{p.x, p.z}] += p.c;
}

constexpr double kDrop = 1e-12;

// --- 4x4 gate algebra -------------------------------------------------------
struct M4 {
  cplx a[16];
};
M4 m4_mul(const M4& p, const M4& q) {
  M4 r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx s = 0;
      for (int k = 0; k < 4; ++k) s += p.a[i * 4 + k] * q.a[k * 4 + j];
      r.a[i * 4 + j] = s;
    }
  return r;
}
M4 m4_dag(const M4& p) {
  M4 r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) r.a[i * 4 + j] = std::conj(p.a[j * 4 + i]);
  return r;
}
M4 kron(const M2& A, const M2& B) {  // index 2*i_A + i_B
  M4 r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 2; ++l) r.a[(2 * i + k) * 4 + (2 * j + l)] = A.a[i][j] * B.a[k][l];
  return r;
}
M4 cnot() {
  M4 r{};
  r.a[0 * 4 + 0] = r.a[1 * 4 + 1] = r.a[2 * 4 + 3] = r.a[3 * 4 + 2] = 1.0;
  return r;
}
M4 swapg() {
  M4 r{};
  r.a[0 * 4 + 0] = r.a[1 * 4 + 2] = r.a[2 * 4 + 1] = r.a[3 * 4 + 3] = 1.0;
  return r;
}

// Basis change V with V^dag Z V = P for the Pauli on one qubit.
M2 basis_change(int xb, int zb) {
  const double h = 1.0 / std::sqrt(2.0);
  M2 Hm;
  Hm.a[0][0] = h;
  Hm.a[0][1] = h;
  Hm.a[1][0] = h;
  Hm.a[1][1] = -h;
  if (xb && !zb) return Hm;  // X
  if (xb && zb) {            // Y: S^dag first, then H
    M2 Sd{{{1.0, 0.0}, {0.0, cplx(0.0, -1.0)}}};
    return m2_mul(Hm, Sd);
  }
  return m2_identity();
}

void compile_rotation(const Rotation& r, int rot_index, std::vector<Gate>& out) {
  const int lo = r.lo, hi = r.hi, L = hi - lo;
  auto bitx = [&](int q) { return int((r.x >> q) & 1); };
  auto bitz = [&](int q) { return int((r.z >> q) & 1); };
  auto in_support = [&](int q) { return bitx(q) || bitz(q); };
  std::vector<M2> V(L + 1);
  for (int q = lo; q <= hi; ++q) V[q - lo] = basis_change(bitx(q), bitz(q));
  auto ladder = [&](int k) { return in_support(k + 1) ? cnot() : swapg(); };
  const M2 I2 = m2_identity();
  auto emit_const = [&](int site, const M4& m) {
    Gate g;
    g.site = site;
    g.rot = -1;
    for (int i = 0; i < 16; ++i) {
      g.pre[i] = m.a[i];
      g.post[i] = (i % 5 == 0) ? 1.0 : 0.0;
    }
    out.push_back(g);
  };
  for (int j = 0; j + 1 < L; ++j) {
    const int k = lo + j;
    emit_const(k, m4_mul(ladder(k), kron(j == 0 ? V[0] : I2, V[j + 1])));
  }
  {
    const int k = hi - 1;
    const M4 pv = kron(L == 1 ? V[0] : I2, V[L]);
    Gate g;
    g.site = k;
    g.rot = rot_index;
    const M4 pre = m4_mul(ladder(k), pv);
    const M4 post = m4_mul(m4_dag(pv), ladder(k));
    for (int i = 0; i < 16; ++i) {
      g.pre[i] = pre.a[i];
      g.post[i] = post.a[i];
    }
    out.push_back(g);
  }
  for (int j = L - 2; j >= 0; --j) {
    const int k = lo + j;
    emit_const(k, m4_mul(m4_dag(kron(j == 0 ? V[0] : I2, V[j + 1])), ladder(k)));
  }
}

}  // namespace

Problem compile_problem(int n_orb, int n_elec, const double* h1, const double* eri, double e_const) {
  if (n_orb < 1 || n_orb > 32) throw std::invalid_argument("n_orb must be in 1..32");
  if (n_elec < 0 || n_elec > 2 * n_orb || (n_elec & 1))
    throw std::invalid_argument("n_elec must be even and in 0..2*n_orb");
  if (!h1 || !eri) throw std::invalid_argument("NULL integrals");
  if (!std::isfinite(e_const)) throw std::invalid_argument("non-finite e_const");
  const size_t n2 = size_t(n_orb) * n_orb, n4 = n2 * n2;
  for (size_t i = 0; i < n2; ++i)
    if (!std::isfinite(h1[i])) throw std::invalid_argument("non-finite h1 entry");
  for (size_t i = 0; i < n4; ++i)
    if (!std::isfinite(eri[i])) throw std::invalid_argument("non-finite eri entry");

  Problem P;
  P.n_orb = n_orb;
  P.n_elec = n_elec;
  P.n_qubits = 2 * n_orb;
  P.e_const = e_const;
  const int n = n_orb;
  auto so = [](int p, int s) { return 2 * p + s; };

  PauliMap H;
  H[Key{0, 0}] += e_const;
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      const double v = h1[p * n + q];
      if (v == 0.0) continue;
      for (int s = 0; s < 2; ++s) add_monomial({{true, so(p, s)}, {false, so(q, s)}}, v, H);
    }
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q)
      for (int r = 0; r < n; ++r)
        for (int t = 0; t < n; ++t) {
          const double g = eri[((size_t(p) * n + q) * n + r) * n + t];
          if (g == 0.0) continue;
          for (int s1 = 0; s1 < 2; ++s1)
            for (int s2 = 0; s2 < 2; ++s2)
              add_monomial({{true, so(p, s1)}, {true, so(r, s2)}, {false, so(t, s2)}, {false, so(q, s1)}},
                           0.5 * g, H);
        }
  for (const auto& kv : H) {
    const cplx c = kv.second;
    if (std::abs(c.imag()) > kDrop) throw std::runtime_error("Hamiltonian has a non-real Pauli coefficient");
    if (kv.first.x == 0 && kv.first.z == 0) {
      P.c_identity = c.real();
    } else if (std::abs(c.real()) >= kDrop) {
      P.terms.push_back(PauliTerm{kv.first.x, kv.first.z, c.real()});
    }
  }
  std::sort(P.terms.begin(), P.terms.end(), [](const PauliTerm& a, const PauliTerm& b) {
    return a.x != b.x ? a.x < b.x : a.z < b.z;
  });

  // UCCSD excitations
  const int nq = P.n_qubits;
  struct Exc {
    std::vector<Ladder> tau;
  };
  std::vector<Exc> exc;
  for (int i = 0; i < n_elec; ++i)
    for (int a = n_elec; a < nq; ++a)
      if ((i & 1) == (a & 1)) exc.push_back({{{true, a}, {false, i}}});
  for (int i = 0; i < n_elec; ++i)
    for (int j = i + 1; j < n_elec; ++j)
      for (int a = n_elec; a < nq; ++a)
        for (int b = a + 1; b < nq; ++b)
          if ((i & 1) + (j & 1) == (a & 1) + (b & 1)) exc.push_back({{{true, a}, {true, b}, {false, i}, {false, j}}});
  P.n_params = int(exc.size());
  for (int k = 0; k < P.n_params; ++k) {
    PauliMap G;
    add_monomial(exc[k].tau, 1.0, G);
    std::vector<Ladder> dag;
    for (auto it = exc[k].tau.rbegin(); it != exc[k].tau.rend(); ++it) dag.push_back({!it->create, it->P});
    add_monomial(dag, -1.0, G);
    std::vector<Rotation> rs;
    for (const auto& kv : G) {
      const cplx v = kv.second;
      if (std::abs(v) < kDrop) continue;
      if (std::abs(v.real()) > kDrop) throw std::runtime_error("UCCSD generator is not anti-Hermitian");
      Rotation r;
      r.x = kv.first.x;
      r.z = kv.first.z;
      r.c = v.imag();  // v = i c
      r.param = k;
      const uint64_t m = r.x | r.z;
      r.lo = __builtin_ctzll(m);
      r.hi = 63 - __builtin_clzll(m);
      rs.push_back(r);
    }
    std::sort(rs.begin(), rs.end(), [](const Rotation& a, const Rotation& b) {
      return a.x != b.x ? a.x < b.x : a.z < b.z;
    });
    for (auto& r : rs) P.rotations.push_back(r);
  }
  for (size_t m = 0; m < P.rotations.size(); ++m) compile_rotation(P.rotations[m], int(m), P.gates);
  return P;
}

PrefixOrder pauli_prefix_order(const uint64_t* x, const uint64_t* z, int n) {
  PrefixOrder po;
  po.order.resize(n);
  po.share.assign(n, 0);
  auto lo_of = [&](int s) { return (x[s] | z[s]) ? __builtin_ctzll(x[s] | z[s]) : -1; };
  auto len_of = [&](int s) {
    const uint64_t m = x[s] | z[s];
    return m ? 64 - __builtin_clzll(m) - __builtin_ctzll(m) : 0;
  };
  auto letter = [&](int s, int k) { return int((x[s] >> k) & 1) | int((z[s] >> k) & 1) << 1; };
  for (int i = 0; i < n; ++i) po.order[i] = i;
  std::stable_sort(po.order.begin(), po.order.end(), [&](int a, int b) {
    const int la = lo_of(a), lb = lo_of(b);
    if (la != lb) return la < lb;
    if (la < 0) return false;
    for (int k = la; k < 64; ++k) {
      const int ca = letter(a, k), cb = letter(b, k);
      if (ca != cb) return ca < cb;
    }
    return false;
  });
  for (int t = 0; t < n; ++t) {
    const int s = po.order[t];
    const int len = len_of(s);
    po.steps_plain += len;
    int sh = 0;
    if (t > 0) {
      const int p = po.order[t - 1];
      const int lo = lo_of(s);
      if (lo >= 0 && lo == lo_of(p)) {
        const int cap = std::min(len, len_of(p));
        while (sh < cap && letter(s, lo + sh) == letter(p, lo + sh)) ++sh;
      }
    }
    po.share[t] = sh;
    po.steps_shared += len - sh;
  }
  return po;
}

}  // namespace q2c
