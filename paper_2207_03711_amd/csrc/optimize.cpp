// VQE outer loop: minimise E(theta) over the UCCSD parameters with L-BFGS
// (Nocedal & Wright, Numerical Optimization, 2nd ed., Alg. 7.4 two-loop
// recursion and Alg. 7.5), every energy and gradient evaluated on the device
// through vqe_energy_batch and vqe_grad_paramshift.  The paper's VQE hands
// E(theta) to a classical optimizer (Sec. II-A); it does not name one.
//
// Per iteration: direction d = -H g from the last `history` curvature pairs
// (H_0 = (s^T y / y^T y) I; before the first pair a steepest-descent step
// whose largest component is max_step); backtracking on the Armijo condition
// E(theta + a d) <= E + 1e-4 a g^T d with a = 1, 1/2, 1/4, ..., n_trial step
// lengths evaluated at once as one batch of circuits and the largest
// acceptable one taken; then the gradient at the new point.  By default step
// length 1 is tried first through the gradient call at x + d, whose
// unshifted circuit gives E(x + d) bit for bit as a batch would: an accepted
// unit step then costs one call instead of a batch and a call, and a rejected
// one continues the same sequence 1/2, 1/4, ... in batches, so the accepted
// steps are the same.  A pair (s, y)
// enters the memory only when s^T y > 1e-12 |s| |y| (Armijo alone does not
// guarantee positive curvature); a non-descent direction clears the memory.
#include <chrono>
#include <cmath>
#include <vector>

#include "runtime.hpp"

using namespace q2c_rt;

namespace {

void call(int rc) {
  if (rc != Q2C_OK) throw StatusError(rc, g_last_error);
}

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

double max_abs(const std::vector<double>& a) {
  double m = 0.0;
  for (double v : a) m = std::max(m, std::fabs(v));
  return m;
}

}  // namespace

extern "C" {

int vqe_minimize(vqe_problem* p, const double* theta0, int n_theta, int max_bond, int precision,
                 const q2c_min_opts* opts, double* theta_out, double* energy, double* energy_trace,
                 q2c_min_report* report) {
  return guarded([&] {
    if (!p) throw ArgError("problem is NULL");
    if (!theta0 || !theta_out) throw ArgError("theta0 / theta_out is NULL");
    int nq = 0, np = 0, ns = 0, nr = 0, ng = 0;
    double cid = 0.0;
    call(vqe_problem_info(p, &nq, &np, &ns, &nr, &ng, &cid));
    if (n_theta != np) throw ArgError("n_theta does not match the problem's parameter count");
    for (int k = 0; k < n_theta; ++k)
      if (!std::isfinite(theta0[k])) throw ArgError("theta0 holds a non-finite value");
    q2c_min_opts o{};
    if (opts) o = *opts;
    const int max_iter = o.max_iter > 0 ? o.max_iter : 100;
    const int hist = o.history > 0 ? o.history : 8;
    const int n_trial = o.n_trial > 0 ? o.n_trial : 4;
    const double gtol = o.gtol > 0.0 ? o.gtol : 1e-6;
    const double ftol = o.ftol > 0.0 ? o.ftol : 1e-13;
    const double max_step = o.max_step > 0.0 ? o.max_step : 0.1;
    if (o.max_iter < 0 || o.history < 0 || o.n_trial < 0 || o.n_trial > 64 || !(o.gtol >= 0.0) ||
        !(o.ftol >= 0.0) || !(o.max_step >= 0.0))
      throw ArgError("negative or out-of-range optimizer option");
    constexpr double kArmijo = 1e-4;
    constexpr int kRounds = 6;  // line-search batches before giving up: a >= 2^-(6 n_trial)
    const auto t0 = std::chrono::steady_clock::now();

    std::vector<double> x(theta0, theta0 + n_theta), g(n_theta), xn(n_theta), gn(n_theta), d(n_theta);
    std::vector<std::vector<double>> S, Y;
    std::vector<double> trace;
    double E = 0.0;
    q2c_min_report rep{};
    call(vqe_grad_paramshift(p, x.data(), n_theta, max_bond, precision, g.data(), &E, nullptr));
    rep.grad_evals = 1;
    trace.push_back(E);
    int status = 0;
    std::vector<double> trial(size_t(n_trial) * n_theta), et(n_trial);
    while (true) {
      if (max_abs(g) <= gtol) {
        status = 1;
        break;
      }
      if (rep.iterations >= max_iter) {
        status = 0;
        break;
      }
      // two-loop recursion: d = -H g
      std::vector<double> q = g, alpha(S.size());
      for (int i = int(S.size()) - 1; i >= 0; --i) {
        alpha[i] = dot(S[i], q) / dot(Y[i], S[i]);
        for (int k = 0; k < n_theta; ++k) q[k] -= alpha[i] * Y[i][k];
      }
      double gamma;
      if (S.empty())
        gamma = max_step / max_abs(g);
      else
        gamma = dot(S.back(), Y.back()) / dot(Y.back(), Y.back());
      for (int k = 0; k < n_theta; ++k) q[k] *= gamma;
      for (size_t i = 0; i < S.size(); ++i) {
        const double b = dot(Y[i], q) / dot(Y[i], S[i]);
        for (int k = 0; k < n_theta; ++k) q[k] += S[i][k] * (alpha[i] - b);
      }
      for (int k = 0; k < n_theta; ++k) d[k] = -q[k];
      double slope = dot(g, d);
      if (!(slope < 0.0)) {  // not a descent direction: forget the curvature pairs
        S.clear();
        Y.clear();
        const double s0 = max_step / max_abs(g);
        for (int k = 0; k < n_theta; ++k) d[k] = -s0 * g[k];
        slope = dot(g, d);
      }
      // backtracking, n_trial step lengths per batch
      double a0 = 1.0, acc = 0.0, e_acc = 0.0, En = 0.0;
      bool have_grad = false;
      if (!o.no_speculation) {
        for (int k = 0; k < n_theta; ++k) xn[k] = x[k] + d[k];
        call(vqe_grad_paramshift(p, xn.data(), n_theta, max_bond, precision, gn.data(), &En, nullptr));
        rep.grad_evals += 1;
        if (En <= E + kArmijo * slope) {
          acc = 1.0;
          e_acc = En;
          have_grad = true;
        } else {
          a0 = 0.5;
        }
      }
      for (int round = 0; round < kRounds && acc == 0.0; ++round) {
        for (int j = 0; j < n_trial; ++j) {
          const double a = a0 * std::ldexp(1.0, -j);
          for (int k = 0; k < n_theta; ++k) trial[size_t(j) * n_theta + k] = x[k] + a * d[k];
        }
        call(vqe_energy_batch(p, trial.data(), n_trial, n_theta, max_bond, precision, et.data(), nullptr));
        rep.energy_evals += n_trial;
        for (int j = 0; j < n_trial; ++j) {
          const double a = a0 * std::ldexp(1.0, -j);
          if (et[j] <= E + kArmijo * a * slope) {
            acc = a;
            e_acc = et[j];
            break;
          }
        }
        a0 = std::ldexp(a0, -n_trial);
      }
      if (acc == 0.0) {  // no decrease found: at the resolution of E
        status = 3;
        break;
      }
      if (!have_grad) {
        for (int k = 0; k < n_theta; ++k) xn[k] = x[k] + acc * d[k];
        call(vqe_grad_paramshift(p, xn.data(), n_theta, max_bond, precision, gn.data(), &En, nullptr));
        rep.grad_evals += 1;
      }
      (void)e_acc;  // the gradient call evaluates the same circuit; En is that energy
      rep.iterations += 1;
      trace.push_back(En);
      std::vector<double> s(n_theta), y(n_theta);
      for (int k = 0; k < n_theta; ++k) {
        s[k] = xn[k] - x[k];
        y[k] = gn[k] - g[k];
      }
      const double sy = dot(s, y);
      if (sy > 1e-12 * std::sqrt(dot(s, s) * dot(y, y))) {
        S.push_back(s);
        Y.push_back(y);
        if (int(S.size()) > hist) {
          S.erase(S.begin());
          Y.erase(Y.begin());
        }
      }
      const double drop = E - En;
      x.swap(xn);
      g.swap(gn);
      E = En;
      if (drop <= ftol * std::max(1.0, std::fabs(E))) {
        status = max_abs(g) <= gtol ? 1 : 2;
        break;
      }
    }
    rep.status = status;
    rep.grad_max = max_abs(g);
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::copy(x.begin(), x.end(), theta_out);
    if (energy) *energy = E;
    if (energy_trace) std::copy(trace.begin(), trace.end(), energy_trace);
    if (report) *report = rep;
  });
}

}  // extern "C"
