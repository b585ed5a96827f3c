// Request server: continuous batching of independent energy evaluations
// (fragment solves of the DMET embedding, Sec. III-B/III-C).  See q2c.h.
#include <chrono>
#include <deque>
#include <map>
#include <tuple>

#include "compile.hpp"
#include "runtime.hpp"

using namespace q2c_rt;

namespace {

using Clock = std::chrono::steady_clock;

struct SrvRequest {
  uint64_t tag = 0;
  int n_frag_orb = 0, D = 0, precision = 0;
  q2c::Problem prob;  // strings of this request; gates and rotations as its class's
  std::vector<double> theta;
  double t_submit = 0.0, t_admit = -1.0;
  DBuf sx, sz, sc;    // Hamiltonian strings, then 2 n_frag_orb single-Z strings (coefficient 0)
  DBuf sord, sshr;    // their prefix order
  int n_str = 0;
};

// Requests that share the UCCSD circuit structure and the MPS layout.
struct SrvClass {
  int n_qubits = 0, n_elec = 0, D = 0, precision = 0;
  std::unique_ptr<Batch> batch;
  q2c::DevProblem dev;
  DBuf gsite, grot, gpre, gpost, rc, rparam, occ, cursor, theta1, phi, ev_re, ev_im, energy, scratch;
  size_t ev_cap = 0;
  int n_wg = 32;
  std::vector<std::unique_ptr<SrvRequest>> slot_req;  // request per slot, null when free
  std::vector<int> cursor_host;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool in_flight = false;
  uint64_t last_use = 0;  // server step of the last admission or launch (eviction order)

  ~SrvClass() {
    if (stream) {
      (void)hipStreamSynchronize(stream);
      (void)hipStreamDestroy(stream);
    }
    if (done) (void)hipEventDestroy(done);
  }
  int active() const {
    int a = 0;
    for (const auto& r : slot_req) a += r ? 1 : 0;
    return a;
  }
  int free_slot() const {
    for (size_t i = 0; i < slot_req.size(); ++i)
      if (!slot_req[i]) return int(i);
    return -1;
  }
};

using ClassKey = std::tuple<int, int, int, int>;  // qubits, electrons, D, precision

}  // namespace

struct q2c_server {
  q2c_ctx* ctx = nullptr;
  q2c_server_opts opts{};
  Clock::time_point t0;
  std::map<ClassKey, std::unique_ptr<SrvClass>> classes;
  std::deque<std::unique_ptr<SrvRequest>> queue;
  std::deque<q2c_result> ready;
  uint64_t steps = 0;  // completed q2c_server_step calls

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

// Whether a queued request waits for the class `key`.
bool class_queued(const q2c_server* srv, const ClassKey& key) {
  for (const auto& r : srv->queue)
    if (ClassKey{r->prob.n_qubits, r->prob.n_elec, r->D, r->precision} == key) return true;
  return false;
}

template <class T>
void upload(q2c_ctx* ctx, DBuf& buf, const std::vector<T>& v, hipStream_t st) {
  buf = DBuf(ctx, std::max<size_t>(sizeof(T) * v.size(), 16));
  if (!v.empty()) hip_check(hipMemcpyAsync(buf.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st), "upload");
}

// A class for the structure of request r: device gate list, rotations and a
// slot batch, charged to the context's budget (OomError when it does not fit).
std::unique_ptr<SrvClass> make_class(q2c_server* s, const SrvRequest& r) {
  q2c_ctx* ctx = s->ctx;
  const auto& H = r.prob;
  auto c = std::make_unique<SrvClass>();
  c->n_qubits = H.n_qubits;
  c->n_elec = H.n_elec;
  c->D = r.D;
  c->precision = r.precision;
  hip_check(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "hipStreamCreate");
  hip_check(hipEventCreateWithFlags(&c->done, hipEventDisableTiming), "hipEventCreate");
  const int S = std::max(1, s->opts.slots_per_class);
  c->batch = std::make_unique<Batch>(ctx, H.n_qubits, r.D, S, r.precision);
  auto& d = c->dev;
  d.n_qubits = H.n_qubits;
  d.n_gates = int(H.gates.size());
  d.n_rot = int(H.rotations.size());
  std::vector<int> site(d.n_gates), rot(d.n_gates), rparam(d.n_rot);
  std::vector<double2> pre(size_t(d.n_gates) * 16), post(size_t(d.n_gates) * 16);
  std::vector<double> rc(d.n_rot);
  for (int g = 0; g < d.n_gates; ++g) {
    site[g] = H.gates[g].site;
    rot[g] = H.gates[g].rot;
    for (int i = 0; i < 16; ++i) {
      pre[size_t(g) * 16 + i] = make_double2(H.gates[g].pre[i].real(), H.gates[g].pre[i].imag());
      post[size_t(g) * 16 + i] = make_double2(H.gates[g].post[i].real(), H.gates[g].post[i].imag());
    }
  }
  for (int m = 0; m < d.n_rot; ++m) {
    rc[m] = H.rotations[m].c;
    rparam[m] = H.rotations[m].param;
  }
  std::vector<uint8_t> occ(H.n_qubits);
  for (int q = 0; q < H.n_qubits; ++q) occ[q] = q < H.n_elec ? 1 : 0;
  upload(ctx, c->gsite, site, c->stream);
  upload(ctx, c->grot, rot, c->stream);
  upload(ctx, c->gpre, pre, c->stream);
  upload(ctx, c->gpost, post, c->stream);
  upload(ctx, c->rc, rc, c->stream);
  upload(ctx, c->rparam, rparam, c->stream);
  upload(ctx, c->occ, occ, c->stream);
  d.gate_site = c->gsite.as<int>();
  d.gate_rot = c->grot.as<int>();
  d.gate_pre = c->gpre.as<double2>();
  d.gate_post = c->gpost.as<double2>();
  d.rot_c = c->rc.as<double>();
  d.rot_param = c->rparam.as<int>();
  c->cursor_host.assign(S, d.n_gates);  // every slot idle
  upload(ctx, c->cursor, c->cursor_host, c->stream);
  c->theta1 = DBuf(ctx, sizeof(double) * std::max(1, H.n_params));
  c->phi = DBuf(ctx, sizeof(double) * std::max(1, S * d.n_rot));
  c->energy = DBuf(ctx, sizeof(double));
  const int cm = c->batch->cm;
  c->scratch = DBuf(ctx, size_t(c->n_wg) * q2c::pauli_scratch_mats(c->n_qubits) * cm * cm * sizeof(double2));
  c->batch->d.phi = c->phi.as<double>();
  c->batch->d.cursor = c->cursor.as<int>();
  c->batch->d.n_gates = d.n_gates;
  c->slot_req.resize(S);
  hip_check(hipStreamSynchronize(c->stream), "sync");
  return c;
}

q2c::DevBatch one_slot(const SrvClass& c, int slot) {
  q2c::DevBatch b = c.batch->d;
  b.slot0 = slot;
  b.n_slots = 1;
  return b;
}

// Places request r in a free slot of class c (which is not running).
void admit(q2c_server* s, SrvClass& c, int slot, std::unique_ptr<SrvRequest> r) {
  q2c_ctx* ctx = s->ctx;
  hipStream_t st = c.stream;
  const auto& H = r->prob;
  // strings: the Hamiltonian, then Z on each fragment spin-orbital
  std::vector<uint64_t> sx, sz;
  std::vector<double> sc;
  for (const auto& t : H.terms) {
    sx.push_back(t.x);
    sz.push_back(t.z);
    sc.push_back(t.c);
  }
  for (int q = 0; q < 2 * r->n_frag_orb; ++q) {
    sx.push_back(0);
    sz.push_back(uint64_t(1) << q);
    sc.push_back(0.0);
  }
  r->n_str = int(sx.size());
  upload(ctx, r->sx, sx, st);
  upload(ctx, r->sz, sz, st);
  upload(ctx, r->sc, sc, st);
  const q2c::PrefixOrder po = q2c::pauli_prefix_order(sx.data(), sz.data(), r->n_str);
  upload(ctx, r->sord, po.order, st);
  upload(ctx, r->sshr, po.share, st);
  if (!r->theta.empty())
    hip_check(hipMemcpyAsync(c.theta1.p, r->theta.data(), sizeof(double) * r->theta.size(), hipMemcpyHostToDevice, st),
              "copy theta");
  const q2c::DevBatch b = one_slot(c, slot);
  hip_check(q2c::launch_init_product(b, c.occ.as<uint8_t>(), st), "init");
  hip_check(q2c::launch_angles(b, c.dev, c.theta1.as<double>(), H.n_params, nullptr, nullptr, st), "angles");
  const int zero = 0;
  hip_check(hipMemcpyAsync(c.cursor.as<int>() + slot, &zero, sizeof(int), hipMemcpyHostToDevice, st), "cursor");
  hip_check(hipStreamSynchronize(st), "sync");  // the host copies above are from stack memory
  c.cursor_host[slot] = 0;
  r->t_admit = s->now();
  c.slot_req[slot] = std::move(r);
}

// Environments, Pauli sweeps and the energy of a slot whose gates are done.
void finish(q2c_server* s, SrvClass& c, int slot) {
  q2c_ctx* ctx = s->ctx;
  hipStream_t st = c.stream;
  SrvRequest& r = *c.slot_req[slot];
  const q2c::DevBatch b = one_slot(c, slot);
  const int ns = r.n_str;
  const size_t evb = sizeof(double) * std::max(1, ns);
  if (c.ev_cap < evb) {
    c.ev_re = DBuf(ctx, evb);
    c.ev_im = DBuf(ctx, evb);
    c.ev_cap = evb;
  }
  q2c_result res{};
  res.tag = r.tag;
  res.n_qubits = c.n_qubits;
  res.max_bond = c.D;
  res.precision = c.precision;
  res.submit_s = r.t_submit;
  res.admit_s = r.t_admit;
  hip_check(q2c::launch_envs(b, st), "envs");
  const int n_wg = std::min(c.n_wg, pauli_workgroups(ns, 1));
  hip_check(q2c::launch_pauli(b, r.sx.as<uint64_t>(), r.sz.as<uint64_t>(), ns, r.sord.as<int>(), r.sshr.as<int>(),
                              c.scratch.as<double2>(), n_wg, c.batch->cm, c.ev_re.as<double>(), c.ev_im.as<double>(),
                              0, st),
            "pauli");
  hip_check(q2c::launch_energy_reduce(b, r.sc.as<double>(), c.ev_re.as<double>(), c.ev_im.as<double>(), ns,
                                      r.prob.c_identity, c.energy.as<double>(), st),
            "reduce");
  double e = 0.0;
  int flag = 0;
  std::vector<double> st_slot(q2c::kNStats), zf(2 * r.n_frag_orb);
  hip_check(hipMemcpyAsync(&e, c.energy.p, sizeof(double), hipMemcpyDeviceToHost, st), "copy E");
  hip_check(hipMemcpyAsync(&flag, b.flags + slot, sizeof(int), hipMemcpyDeviceToHost, st), "copy flag");
  hip_check(hipMemcpyAsync(st_slot.data(), b.stats + size_t(slot) * q2c::kNStats, sizeof(double) * q2c::kNStats,
                           hipMemcpyDeviceToHost, st),
            "copy stats");
  if (!zf.empty())
    hip_check(hipMemcpyAsync(zf.data(), c.ev_re.as<double>() + (ns - zf.size()), sizeof(double) * zf.size(),
                             hipMemcpyDeviceToHost, st),
              "copy Z");
  hip_check(hipStreamSynchronize(st), "sync");
  res.energy = e;
  double nf = 0.0;
  for (double z : zf) nf += 0.5 * (1.0 - z);
  res.n_frag = nf;
  res.discarded_weight_sum = st_slot[q2c::kStatDisc];
  res.max_chi = int(st_slot[q2c::kStatMaxChi]);
  res.status = Q2C_OK;
  if (flag & q2c::kFlagNumeric) res.status = Q2C_ERR_NUMERIC;
  else if (flag & q2c::kFlagNoConv) res.status = Q2C_ERR_NOCONV;
  else if (!std::isfinite(e)) res.status = Q2C_ERR_NUMERIC;
  res.done_s = s->now();
  s->ready.push_back(res);
  c.slot_req[slot].reset();
  c.cursor_host[slot] = c.dev.n_gates;
}

}  // namespace

extern "C" {

int q2c_server_create(q2c_ctx* ctx, const q2c_server_opts* opts, q2c_server** out) {
  return guarded([&] {
    require(ctx && out, "NULL argument");
    auto s = std::make_unique<q2c_server>();
    s->ctx = ctx;
    if (opts) s->opts = *opts;
    if (s->opts.slots_per_class <= 0) s->opts.slots_per_class = 64;
    if (s->opts.gates_per_step <= 0) s->opts.gates_per_step = 1024;
    require(s->opts.slots_per_class <= 4096, "slots_per_class must be <= 4096");
    s->t0 = Clock::now();
    *out = s.release();
  });
}

int q2c_server_destroy(q2c_server* srv) {
  return guarded([&] {
    if (!srv) return;
    srv->ctx->activate();
    delete srv;
  });
}

int q2c_server_submit(q2c_server* srv, uint64_t tag, int n_orb, int n_elec, const double* h1, const double* eri,
                      double e_const, const double* theta, int n_theta, int max_bond, int precision, int n_frag_orb) {
  return guarded([&] {
    require(srv != nullptr, "srv is NULL");
    require(max_bond >= 1 && max_bond <= 256, "max_bond must be in 1..256");
    require(precision == Q2C_FP64 || precision == Q2C_MIXED, "unknown precision");
    require(n_frag_orb >= 0 && n_frag_orb <= n_orb, "n_frag_orb must be in 0..n_orb");
    auto r = std::make_unique<SrvRequest>();
    r->t_submit = srv->now();
    r->prob = q2c::compile_problem(n_orb, n_elec, h1, eri, e_const);
    require(n_theta == r->prob.n_params, "theta length does not match the number of UCCSD parameters");
    require(n_theta == 0 || theta != nullptr, "theta is NULL");
    for (int i = 0; i < n_theta; ++i) require(std::isfinite(theta[i]), "theta has a non-finite entry");
    r->theta.assign(theta, theta + n_theta);
    r->tag = tag;
    r->D = max_bond;
    r->precision = precision;
    r->n_frag_orb = n_frag_orb;
    srv->queue.push_back(std::move(r));
  });
}

int q2c_server_step(q2c_server* srv, int* n_queued, int* n_active, int* n_ready) {
  return guarded([&] {
    require(srv != nullptr, "srv is NULL");
    q2c_ctx* ctx = srv->ctx;
    ctx->activate();
    // 1. classes whose launch has completed: retire finished slots
    for (auto& kv : srv->classes) {
      SrvClass& c = *kv.second;
      if (!c.in_flight) continue;
      const hipError_t q = hipEventQuery(c.done);
      if (q == hipErrorNotReady) continue;
      hip_check(q, "hipEventQuery");
      c.in_flight = false;
      hip_check(hipMemcpyAsync(c.cursor_host.data(), c.cursor.p, sizeof(int) * c.cursor_host.size(),
                               hipMemcpyDeviceToHost, c.stream),
                "copy cursors");
      hip_check(hipStreamSynchronize(c.stream), "sync");
      for (size_t i = 0; i < c.slot_req.size(); ++i)
        if (c.slot_req[i] && c.cursor_host[i] >= c.dev.n_gates) finish(srv, c, int(i));
    }
    // 2. admission into free slots of idle classes (new classes while the budget allows)
    for (auto it = srv->queue.begin(); it != srv->queue.end();) {
      SrvRequest& r = **it;
      const ClassKey key{r.prob.n_qubits, r.prob.n_elec, r.D, r.precision};
      auto ci = srv->classes.find(key);
      if (ci == srv->classes.end()) {
        // a new class; when it does not fit the budget, idle classes (nothing
        // queued for them, nothing running) give their memory back, least
        // recently used first
        std::unique_ptr<SrvClass> made;
        while (!made) {
          try {
            made = make_class(srv, r);
          } catch (const OomError&) {
            auto victim = srv->classes.end();
            for (auto vi = srv->classes.begin(); vi != srv->classes.end(); ++vi) {
              const SrvClass& v = *vi->second;
              if (v.in_flight || v.active() > 0 || class_queued(srv, vi->first)) continue;
              if (victim == srv->classes.end() || v.last_use < victim->second->last_use) victim = vi;
            }
            if (victim == srv->classes.end()) break;
            srv->classes.erase(victim);
          }
        }
        if (!made) {
          ++it;  // waits until memory frees up
          continue;
        }
        ci = srv->classes.emplace(key, std::move(made)).first;
      }
      SrvClass& c = *ci->second;
      const int slot = c.in_flight ? -1 : c.free_slot();
      if (slot < 0) {
        ++it;
        continue;
      }
      c.last_use = srv->steps;
      std::unique_ptr<SrvRequest> req = std::move(*it);
      it = srv->queue.erase(it);
      try {
        admit(srv, c, slot, std::move(req));
      } catch (const OomError&) {
        // strings did not fit: give up on this request
        q2c_result res{};
        res.status = Q2C_ERR_OOM;
        res.done_s = srv->now();
        srv->ready.push_back(res);
      }
    }
    // 3. next gate chunk of every idle class with work; classes run on their own streams
    const q2c::SvdParams sp = svd_params(ctx);
    for (auto& kv : srv->classes) {
      SrvClass& c = *kv.second;
      if (c.in_flight || c.active() == 0) continue;
      hip_check(q2c::launch_gates(c.batch->d, c.dev.gate_site, c.dev.gate_rot, c.dev.gate_pre, c.dev.gate_post, 0,
                                  srv->opts.gates_per_step, c.dev.n_rot, sp, c.stream),
                "gates");
      hip_check(hipEventRecord(c.done, c.stream), "event");
      c.in_flight = true;
      c.last_use = srv->steps;
    }
    // idle classes keep their slots and compiled gate list for the next
    // request of their shape; they are evicted only when a new class needs
    // the memory (step 2)
    ++srv->steps;
    int act = 0;
    for (auto& kv : srv->classes) act += kv.second->active();
    if (n_queued) *n_queued = int(srv->queue.size());
    if (n_active) *n_active = act;
    if (n_ready) *n_ready = int(srv->ready.size());
  });
}

int q2c_server_poll(q2c_server* srv, q2c_result* out, int max_out, int* n_out) {
  return guarded([&] {
    require(srv && n_out, "NULL argument");
    require(max_out >= 0 && (max_out == 0 || out), "out is NULL");
    int n = 0;
    while (n < max_out && !srv->ready.empty()) {
      out[n++] = srv->ready.front();
      srv->ready.pop_front();
    }
    *n_out = n;
  });
}

}  // extern "C"
