// DMET chemical-potential loop (Sec. III-B) around the device fragment
// solver.  Host steps: the restricted mean-field determinant of the lattice
// one-body matrix (the low-level calculation), for each fragment the bath
// from the Schmidt decomposition of that determinant, and the Hamiltonian
// projected onto fragment + bath; device steps: the UCCSD fragment problem
// minimised by vqe_minimize, then its electron count and energy as
// expectation values at the minimum (vqe_energy of one-body and two-body
// operators built on the same embedding orbitals).  The global chemical
// potential moves by regula falsi with the Illinois modification until the
// fragments' electrons add up to the lattice's.
//
// Embedding orbitals: the natural orbitals of the mean-field density inside
// fragment + bath, occupied (eigenvalue 1) first, each block rotated to
// diagonalise h within it, each orbital's sign fixed by its largest-magnitude
// site coefficient; the UCCSD reference (first k orbitals doubly occupied) is
// then the mean-field determinant.  Interaction U on the fragment sites only.
#include <chrono>
#include <cmath>
#include <exception>
#include <numeric>
#include <thread>
#include <vector>

#include "runtime.hpp"

using namespace q2c_rt;

namespace {

void call(int rc) {
  if (rc != Q2C_OK) throw StatusError(rc, g_last_error);
}

using Mat = std::vector<double>;  // row-major

// Symmetric eigenproblem by the cyclic Jacobi method (Golub & Van Loan,
// Matrix Computations, 4th ed., Sec. 8.5.2): eigenvalues ascending in w,
// eigenvectors as the columns of V (n x n, row-major).
void sym_eig(int n, Mat a, std::vector<double>& w, Mat& V) {
  Mat U(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) U[size_t(i) * n + i] = 1.0;
  bool converged = false;
  for (int sweep = 0; sweep <= 64; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double v = a[size_t(i) * n + j] * a[size_t(i) * n + j];
        tot += v;
        if (i != j) off += v;
      }
    if (!std::isfinite(tot)) break;
    // off-diagonal norm <= n 1e-15 of the whole: above what rounding leaves
    if (!(off > (1e-30 * n * n) * tot)) {
      converged = true;
      break;
    }
    if (sweep == 64) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[size_t(p) * n + q];
        if (apq == 0.0) continue;
        const double tau = (a[size_t(q) * n + q] - a[size_t(p) * n + p]) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // A J
          const double x = a[size_t(k) * n + p], y = a[size_t(k) * n + q];
          a[size_t(k) * n + p] = c * x - s * y;
          a[size_t(k) * n + q] = s * x + c * y;
        }
        for (int k = 0; k < n; ++k) {  // J^T (A J)
          const double x = a[size_t(p) * n + k], y = a[size_t(q) * n + k];
          a[size_t(p) * n + k] = c * x - s * y;
          a[size_t(q) * n + k] = s * x + c * y;
        }
        for (int k = 0; k < n; ++k) {  // U J
          const double x = U[size_t(k) * n + p], y = U[size_t(k) * n + q];
          U[size_t(k) * n + p] = c * x - s * y;
          U[size_t(k) * n + q] = s * x + c * y;
        }
      }
  }
  if (!converged) throw StatusError(Q2C_ERR_NUMERIC, "symmetric eigensolver did not converge in 64 Jacobi sweeps");
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int i, int j) { return a[size_t(i) * n + i] < a[size_t(j) * n + j]; });
  w.assign(n, 0.0);
  V.assign(size_t(n) * n, 0.0);
  for (int c = 0; c < n; ++c) {
    w[c] = a[size_t(ord[c]) * n + ord[c]];
    for (int r = 0; r < n; ++r) V[size_t(r) * n + c] = U[size_t(r) * n + ord[c]];
  }
}

// C = A^T B (A: r x m, B: r x n, C: m x n)
Mat atb(int r, int m, int n, const Mat& A, const Mat& B) {
  Mat C(size_t(m) * n, 0.0);
  for (int i = 0; i < r; ++i)
    for (int a = 0; a < m; ++a) {
      const double x = A[size_t(i) * m + a];
      if (x == 0.0) continue;
      for (int b = 0; b < n; ++b) C[size_t(a) * n + b] += x * B[size_t(i) * n + b];
    }
  return C;
}

// C = A B (A: m x r, B: r x n)
Mat ab(int m, int r, int n, const Mat& A, const Mat& B) {
  Mat C(size_t(m) * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < r; ++j) {
      const double x = A[size_t(i) * r + j];
      if (x == 0.0) continue;
      for (int b = 0; b < n; ++b) C[size_t(i) * n + b] += x * B[size_t(j) * n + b];
    }
  return C;
}

struct Lat {
  int L, k, ne;
  Mat h;
  double U;
};

// Per-spin density matrix of the n_elec / 2 lowest orbitals of h.
Mat mean_field_density(const Lat& lat) {
  std::vector<double> w;
  Mat C;
  sym_eig(lat.L, lat.h, w, C);
  const int no = lat.ne / 2;
  if (no < lat.L && std::fabs(w[no] - w[no - 1]) < 1e-10)
    throw ArgError("the mean-field determinant is degenerate (no gap at the Fermi level)");
  Mat D(size_t(lat.L) * lat.L, 0.0);
  for (int i = 0; i < lat.L; ++i)
    for (int j = 0; j < lat.L; ++j) {
      double s = 0.0;
      for (int o = 0; o < no; ++o) s += C[size_t(i) * lat.L + o] * C[size_t(j) * lat.L + o];
      D[size_t(i) * lat.L + j] = s;
    }
  return D;
}

// Embedding orbitals of fragment f as the columns of N (L x 2k).
Mat embedding_basis(const Lat& lat, const Mat& D, int f) {
  const int L = lat.L, k = lat.k, ne = L - k, m = 2 * k;
  std::vector<int> F, E;
  for (int i = 0; i < L; ++i) (i / k == f ? F : E).push_back(i);
  // B = D[E, F]; bath = left singular vectors of B, from the eigenvectors of B^T B
  Mat B(size_t(ne) * k);
  for (int a = 0; a < ne; ++a)
    for (int b = 0; b < k; ++b) B[size_t(a) * k + b] = D[size_t(E[a]) * L + F[b]];
  std::vector<double> s2;
  Mat Vb;
  sym_eig(k, atb(ne, k, k, B, B), s2, Vb);
  Mat W(size_t(L) * m, 0.0);
  for (int b = 0; b < k; ++b) W[size_t(F[b]) * m + b] = 1.0;
  for (int j = 0; j < k; ++j) {
    if (!(s2[j] > 1e-20)) throw ArgError("a fragment's bath has fewer orbitals than the fragment has sites");
    const double inv = 1.0 / std::sqrt(s2[j]);
    for (int a = 0; a < ne; ++a) {
      double v = 0.0;
      for (int b = 0; b < k; ++b) v += B[size_t(a) * k + b] * Vb[size_t(b) * k + j];
      W[size_t(E[a]) * m + k + j] = v * inv;
    }
  }
  // natural orbitals of D in span(W): occupied (eigenvalue 1) first
  std::vector<double> wd;
  Mat Vd;
  sym_eig(m, atb(L, m, m, W, ab(L, L, m, D, W)), wd, Vd);
  const Mat hW = atb(L, m, m, W, ab(L, L, m, lat.h, W));  // W^T h W
  Mat T(size_t(m) * m, 0.0);                              // columns: orbitals in the W basis
  for (int blk = 0; blk < 2; ++blk) {
    // block 0: the k largest eigenvalues (occupied), block 1: the k smallest
    Mat Q(size_t(m) * k);
    for (int c = 0; c < k; ++c) {
      const int src = blk == 0 ? m - 1 - c : c;
      for (int r = 0; r < m; ++r) Q[size_t(r) * k + c] = Vd[size_t(r) * m + src];
    }
    std::vector<double> we;
    Mat R;
    sym_eig(k, atb(m, k, k, Q, ab(m, m, k, hW, Q)), we, R);
    const Mat QR = ab(m, k, k, Q, R);
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < k; ++c) T[size_t(r) * m + blk * k + c] = QR[size_t(r) * k + c];
  }
  Mat N = ab(L, m, m, W, T);
  for (int c = 0; c < m; ++c) {
    int best = 0;
    for (int i = 1; i < L; ++i)
      if (std::fabs(N[size_t(i) * m + c]) > std::fabs(N[size_t(best) * m + c])) best = i;
    if (N[size_t(best) * m + c] < 0.0)
      for (int i = 0; i < L; ++i) N[size_t(i) * m + c] = -N[size_t(i) * m + c];
  }
  return N;
}

struct Embedded {
  Mat hbase, nop, efrag, eri;  // 2k x 2k, 2k x 2k, 2k x 2k, (2k)^4
};

Embedded embed(const Lat& lat, const Mat& N, int f) {
  const int L = lat.L, k = lat.k, m = 2 * k;
  Embedded e;
  e.hbase = atb(L, m, m, N, ab(L, L, m, lat.h, N));
  Mat PN(size_t(L) * m, 0.0), Ph(size_t(L) * L, 0.0);
  for (int i = f * k; i < (f + 1) * k; ++i)
    for (int c = 0; c < m; ++c) PN[size_t(i) * m + c] = N[size_t(i) * m + c];
  e.nop = atb(L, m, m, N, PN);
  // 1/2 (P_F h + h P_F)
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < L; ++j) {
      const bool fi = i / k == f, fj = j / k == f;
      Ph[size_t(i) * L + j] = 0.5 * ((fi ? 1.0 : 0.0) + (fj ? 1.0 : 0.0)) * lat.h[size_t(i) * L + j];
    }
  e.efrag = atb(L, m, m, N, ab(L, L, m, Ph, N));
  e.eri.assign(size_t(m) * m * m * m, 0.0);
  for (int i = f * k; i < (f + 1) * k; ++i) {
    const double* n = &N[size_t(i) * m];
    for (int p = 0; p < m; ++p)
      for (int q = 0; q < m; ++q)
        for (int r = 0; r < m; ++r)
          for (int s = 0; s < m; ++s)
            e.eri[((size_t(p) * m + q) * m + r) * m + s] += lat.U * n[p] * n[q] * n[r] * n[s];
  }
  return e;
}

constexpr int kDmetWorkers = 8;  // concurrent fragment solves

struct Ctx {
  q2c_ctx* c = nullptr;
  Ctx() = default;
  Ctx(const Ctx&) = delete;
  Ctx& operator=(const Ctx&) = delete;
  ~Ctx() {
    if (c) q2c_ctx_destroy(c);
  }
};

struct Problem {
  vqe_problem* p = nullptr;
  Problem() = default;
  Problem(const Problem&) = delete;
  Problem& operator=(const Problem&) = delete;
  ~Problem() {
    if (p) vqe_problem_destroy(p);
  }
};

}  // namespace

namespace {

Lat check_lattice(const q2c_lattice* lat_in) {
  if (!lat_in || !lat_in->h) throw ArgError("lattice or lattice->h is NULL");
  Lat lat{lat_in->n_sites, lat_in->frag_size, lat_in->n_elec, {}, lat_in->U};
  if (lat.L < 2 || lat.L > 64 || lat.k < 1 || lat.k > 4 || lat.L % lat.k || lat.k >= lat.L)
    throw ArgError("need 2 <= n_sites <= 64 and 1 <= frag_size <= 4 dividing n_sites, frag_size < n_sites");
  if (lat.ne < 2 || lat.ne % 2 || lat.ne >= 2 * lat.L) throw ArgError("n_elec must be even and in 2 .. 2 n_sites - 2");
  if (!std::isfinite(lat.U)) throw ArgError("U is not finite");
  lat.h.assign(lat_in->h, lat_in->h + size_t(lat.L) * lat.L);
  for (int i = 0; i < lat.L; ++i)
    for (int j = 0; j < lat.L; ++j) {
      const double a = lat.h[size_t(i) * lat.L + j], b = lat.h[size_t(j) * lat.L + i];
      if (!std::isfinite(a) || a != b) throw ArgError("h must be finite and symmetric");
    }
  return lat;
}

}  // namespace

extern "C" {

int dmet_embedding(const q2c_lattice* lattice, int frag, double mu, double* orbitals, double* h1, double* eri,
                   double* nop, double* efrag_h1) {
  return guarded([&] {
    const Lat lat = check_lattice(lattice);
    if (frag < 0 || frag >= lat.L / lat.k) throw ArgError("fragment index out of range");
    if (!std::isfinite(mu)) throw ArgError("mu is not finite");
    const Mat N = embedding_basis(lat, mean_field_density(lat), frag);
    const Embedded e = embed(lat, N, frag);
    if (orbitals) std::copy(N.begin(), N.end(), orbitals);
    if (h1)
      for (size_t i = 0; i < e.hbase.size(); ++i) h1[i] = e.hbase[i] - mu * e.nop[i];
    if (eri) std::copy(e.eri.begin(), e.eri.end(), eri);
    if (nop) std::copy(e.nop.begin(), e.nop.end(), nop);
    if (efrag_h1) std::copy(e.efrag.begin(), e.efrag.end(), efrag_h1);
  });
}

int dmet_solve(q2c_ctx* ctx, const q2c_lattice* lat_in, const q2c_dmet_opts* opts, double* n_frag, double* e_frag,
               double* e_emb, double* mu_trace, q2c_dmet_report* report) {
  return guarded([&] {
    if (!ctx) throw ArgError("ctx is NULL");
    const Lat lat = check_lattice(lat_in);
    q2c_dmet_opts o{};
    if (opts) o = *opts;
    const double mu_lo = (o.mu_lo == 0.0 && o.mu_hi == 0.0) ? -2.0 : o.mu_lo;
    const double mu_hi = (o.mu_lo == 0.0 && o.mu_hi == 0.0) ? 2.0 : o.mu_hi;
    const double n_tol = o.n_tol > 0.0 ? o.n_tol : 1e-6;
    const int max_iter = o.max_iter > 0 ? o.max_iter : 40;
    const int m = 2 * lat.k;
    const int D = o.max_bond > 0 ? o.max_bond : (1 << m);
    if (!(mu_lo < mu_hi) || !std::isfinite(mu_lo) || !std::isfinite(mu_hi)) throw ArgError("need mu_lo < mu_hi");
    if (o.max_iter < 0 || !(o.n_tol >= 0.0) || D > 256) throw ArgError("bad DMET option");
    const auto t0 = std::chrono::steady_clock::now();

    const int nf = lat.L / lat.k;
    const Mat Dm = mean_field_density(lat);
    // fragments are independent (the paper's first level of parallelism):
    // W worker threads, each with a context (stream) of its own on the same
    // device, solve fragments f = w, w + W, ... concurrently; each fragment's
    // arithmetic is the same as alone, so the results do not depend on W
    if (o.workers < 0) throw ArgError("workers must be >= 0");
    const int W = std::min(nf, o.workers > 0 ? o.workers : kDmetWorkers);
    std::vector<Ctx> workers(W);
    {
      q2c_opts wo = ctx->opts;
      wo.autotune_cache = nullptr;
      for (int w = 0; w < W; ++w) call(q2c_ctx_create(ctx->device, nullptr, &wo, &workers[w].c));
    }
    std::vector<Embedded> emb;
    std::vector<Problem> pn(nf), pe(nf);
    const std::vector<double> zero(size_t(m) * m * m * m, 0.0);
    for (int f = 0; f < nf; ++f) {
      emb.push_back(embed(lat, embedding_basis(lat, Dm, f), f));
      q2c_ctx* c = workers[f % W].c;
      call(vqe_problem_create(c, m, m, emb[f].nop.data(), zero.data(), 0.0, &pn[f].p));
      call(vqe_problem_create(c, m, m, emb[f].efrag.data(), emb[f].eri.data(), 0.0, &pe[f].p));
    }
    int np = 0;
    call(vqe_problem_info(pn[0].p, nullptr, &np, nullptr, nullptr, nullptr, nullptr));
    q2c_dmet_report rep{};
    std::vector<double> trace;
    struct Eval {
      double f;
      std::vector<double> nfrag, efrag, eemb;
    };
    auto evaluate = [&](double mu) {
      Eval ev{0.0, std::vector<double>(nf), std::vector<double>(nf), std::vector<double>(nf)};
      std::vector<std::exception_ptr> err(W);
      auto work = [&](int w) {
        try {
          q2c_ctx* c = workers[w].c;
          const std::vector<double> th0(np, 0.0);
          std::vector<double> th(np);
          for (int f = w; f < nf; f += W) {
            Mat h1 = emb[f].hbase;
            for (size_t i = 0; i < h1.size(); ++i) h1[i] -= mu * emb[f].nop[i];
            Problem ph;
            call(vqe_problem_create(c, m, m, h1.data(), emb[f].eri.data(), 0.0, &ph.p));
            call(vqe_minimize(ph.p, th0.data(), np, D, o.precision, &o.vqe, th.data(), &ev.eemb[f], nullptr,
                              nullptr));
            call(vqe_energy(pn[f].p, th.data(), np, D, o.precision, &ev.nfrag[f], nullptr));
            call(vqe_energy(pe[f].p, th.data(), np, D, o.precision, &ev.efrag[f], nullptr));
          }
        } catch (...) {
          err[w] = std::current_exception();
        }
      };
      std::vector<std::thread> threads;
      {
        // joins every started worker on every path (also when starting one throws)
        struct Joiner {
          std::vector<std::thread>& t;
          ~Joiner() {
            for (auto& x : t)
              if (x.joinable()) x.join();
          }
        } joiner{threads};
        for (int w = 1; w < W; ++w) threads.emplace_back(work, w);
        work(0);
      }
      for (auto& e : err)
        if (e) std::rethrow_exception(e);
      double total = 0.0;
      for (int f = 0; f < nf; ++f) total += ev.nfrag[f];
      rep.vqe_runs += nf;
      ev.f = total - lat.ne;
      trace.push_back(mu);
      return ev;
    };
    double a = mu_lo, b = mu_hi, c = a;
    Eval ea = evaluate(a), eb = evaluate(b), ec = ea;
    int status = 0, it = 0;
    if (std::fabs(ea.f) <= n_tol) {
      status = 1;
    } else if (std::fabs(eb.f) <= n_tol) {
      status = 1;
      c = b;
      ec = eb;
    } else if (ea.f > 0.0 || eb.f < 0.0) {
      status = 3;
    } else {
      double fa = ea.f, fb = eb.f;
      int side = 0;
      for (it = 1; it <= max_iter; ++it) {
        c = (a * fb - b * fa) / (fb - fa);
        ec = evaluate(c);
        if (std::fabs(ec.f) <= n_tol) {
          status = 1;
          break;
        }
        if (ec.f < 0.0) {
          a = c;
          fa = ec.f;
          if (side == -1) fb *= 0.5;
          side = -1;
        } else {
          b = c;
          fb = ec.f;
          if (side == 1) fa *= 0.5;
          side = 1;
        }
      }
      if (status == 0) it = max_iter;
    }
    rep.mu = c;
    rep.iterations = it;
    rep.status = status;
    rep.e_dmet = 0.0;
    for (int f = 0; f < nf; ++f) rep.e_dmet += ec.efrag[f];
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (n_frag) std::copy(ec.nfrag.begin(), ec.nfrag.end(), n_frag);
    if (e_frag) std::copy(ec.efrag.begin(), ec.efrag.end(), e_frag);
    if (e_emb) std::copy(ec.eemb.begin(), ec.eemb.end(), e_emb);
    if (mu_trace) std::copy(trace.begin(), trace.end(), mu_trace);
    if (report) *report = rep;
  });
}

}  // extern "C"
