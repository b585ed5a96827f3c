// C ABI of libq2c: argument checking, device memory, launch sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <tuple>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/q2c.h"
#include "compile.hpp"
#include "engine.hpp"

#include "runtime.hpp"

namespace q2c_rt {
thread_local std::string g_last_error;
}  // namespace q2c_rt

using namespace q2c_rt;


// ------------------------------------------------------------------- handles --

struct mps_state {
  q2c_ctx* ctx = nullptr;
  int n = 0, D = 0, precision = 0;
  std::unique_ptr<Batch> batch;
  DBuf occ, gsite, grot, gmat, scratch, ev_re, ev_im, sx, sz, sord, sshr;
  int scratch_wg = 0;
};

// Pinned host memory (hipHostMalloc), the staging area of graph inputs and
// outputs.
struct HostBuf {
  void* p = nullptr;
  explicit HostBuf(size_t bytes) { hip_check(hipHostMalloc(&p, std::max<size_t>(bytes, 16), 0), "hipHostMalloc"); }
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// One batch shape captured as a HIP graph: the inputs copied from pinned
// host memory, the angles, the initial states (the Hartree-Fock product, or
// copies of snapshot slots that start at per-slot fork gates), every gate
// launch over per-slot gate cursors, the environments, the Pauli sweep, the
// reduction, and energies, flags and statistics copied back to pinned host
// memory.  Every buffer the graph touches is its own or lives as long as the
// problem, so a replay needs only new inputs in the staging area.
struct BatchGraph {
  int nb = 0;
  bool fork = false;
  bool tuned = false;
  int launches = 0;  // gate-kernel launches per replay
  PauliCfg cfg;
  std::unique_ptr<HostBuf> h_theta, h_srot, h_sval, h_cursor, h_pairs, h_energy, h_flags, h_stats;
  DBuf theta, srot, sval, cursor, pairs, phi, ev_re, ev_im, scratch, energy;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void release_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~BatchGraph() { release_graph(); }
};

struct vqe_problem {
  q2c_ctx* ctx = nullptr;
  q2c::Problem host;
  q2c::DevProblem dev;
  DBuf gsite, grot, gpre, gpost, rc, rparam, sx, sz, sc, sord, sshr, occ;
  std::map<std::tuple<int, int, int>, std::unique_ptr<Batch>> batches;  // (D, slots, precision)
  // (D, precision): the one-slot batch of the unshifted circuit in forked
  // parameter shifts, apart from `batches` so that a one-circuit batch of
  // shifted circuits never shares its slot
  std::map<std::tuple<int, int>, std::unique_ptr<Batch>> base_batches;
  DBuf theta, shift_rot, shift_val, ev_re, ev_im, energies, scratch, phi, cursor, pairs;
  size_t theta_cap = 0, srot_cap = 0, sval_cap = 0, evr_cap = 0, evi_cap = 0, en_cap = 0, scratch_cap = 0,
         phi_cap = 0, cursor_cap = 0, pairs_cap = 0;
  std::vector<int> fork_gate;   // per rotation: its first gate whose matrix depends on the rotation's angle
  std::vector<int> param_fork;  // per parameter: the first fork gate of its rotations
  std::map<std::tuple<int, int, int>, std::unique_ptr<SlotStore>> snaps;  // (D, precision, 0/1): fork snapshots
  // (D, slots, precision, kind): kind 0 from the Hartree-Fock state, 1 / 2 from snapshot store 0 / 1
  std::map<std::tuple<int, int, int, int>, std::unique_ptr<BatchGraph>> graphs;
};

namespace {

void ensure(q2c_ctx* ctx, DBuf& buf, size_t& cap, size_t bytes) {
  if (cap >= bytes && buf.p) return;
  buf = DBuf(ctx, bytes);
  cap = bytes;
}

Batch& batch_for(vqe_problem* p, int D, int n_slots, int precision) {
  auto key = std::make_tuple(D, n_slots, precision);
  if (!p->batches.count(key))
    p->batches[key] = std::make_unique<Batch>(p->ctx, p->host.n_qubits, D, n_slots, precision);
  return *p->batches[key];
}

Batch& base_batch_for(vqe_problem* p, int D, int precision) {
  auto key = std::make_tuple(D, precision);
  if (!p->base_batches.count(key))
    p->base_batches[key] = std::make_unique<Batch>(p->ctx, p->host.n_qubits, D, 1, precision);
  return *p->base_batches[key];
}

bool progress_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("Q2C_PROGRESS");
    return e && *e && *e != '0';
  }();
  return on;
}

// Gates [g0, g1) of every slot of db, in launches of up to kGateChunk gates.
// With db.cursor set, each launch instead runs up to kGateChunk gates of each
// slot from its cursor, and the launches cover g1 - g0 gates per slot.
int run_gates(vqe_problem* p, const q2c::DevBatch& db, int g0, int g1, hipStream_t st) {
  const q2c::SvdParams sp = svd_params(p->ctx);
  const auto tp0 = std::chrono::steady_clock::now();
  int launches = 0;
  for (int c0 = g0; c0 < g1; c0 += kGateChunk) {
    const int c1 = std::min(g1, c0 + kGateChunk);
    hip_check(q2c::launch_gates(db, p->dev.gate_site, p->dev.gate_rot, p->dev.gate_pre, p->dev.gate_post,
                                db.cursor ? 0 : c0, db.cursor ? c1 - c0 : c1, p->dev.n_rot, sp, st),
              "gates");
    ++launches;
    if (progress_enabled() && g1 - g0 > kGateChunk) {  // runs of more than one launch
      hip_check(hipStreamSynchronize(st), "sync");
      std::fprintf(stderr, "[q2c] %d circuit(s): gates %d/%d done, %.1f s\n", db.n_slots, c1, g1,
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - tp0).count());
      std::fflush(stderr);
    }
  }
  return launches;
}

Tuner::Key pauli_key(const vqe_problem* p, const q2c::DevBatch& db, int n_slots) {
  return Tuner::Key{p->host.n_qubits, db.max_bond, n_slots, db.mixed ? Q2C_MIXED : Q2C_FP64, p->dev.n_strings};
}

size_t pauli_scratch_bytes(const vqe_problem* p, const Batch& B, int n_slots, int n_wg) {
  return size_t(n_slots) * n_wg * q2c::pauli_scratch_mats(p->host.n_qubits) * size_t(B.cm) * B.cm *
         sizeof(double2);
}

// Tuning is skipped (the default is kept and recorded) when one default
// sweep takes longer than this: there the sweep is a small part of a batch
// whose gates take seconds, and timing every candidate would cost more than
// it could save.
constexpr double kTuneMaxMs = 50.0;

// Times every candidate launch of the Pauli sweep (each tile, with half,
// once and twice the default workgroups per circuit) on the environments
// already in db, after one untimed launch, and stores the fastest in the
// context's table.  Outputs go to ev_re / ev_im and are overwritten by the
// caller's own launch.  Adds the time spent to *tune_ms.
PauliCfg tune_pauli(vqe_problem* p, const Batch& B, const q2c::DevBatch& db, int n_slots, double* ev_re,
                    double* ev_im, hipStream_t st, double* tune_ms) {
  const auto t0 = std::chrono::steady_clock::now();
  struct AddTime {
    std::chrono::steady_clock::time_point t0;
    double* out;
    ~AddTime() { *out += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count(); }
  } add_time{t0, tune_ms};
  q2c_ctx* ctx = p->ctx;
  const int ns = p->dev.n_strings;
  const int base = pauli_workgroups(ns, n_slots);
  std::vector<int> wgs;
  for (int w : {base / 2, base, 2 * base}) {
    w = std::max(1, std::min(w, ns));
    if (std::find(wgs.begin(), wgs.end(), w) == wgs.end()) wgs.push_back(w);
  }
  DBuf scr(ctx, pauli_scratch_bytes(p, B, n_slots, *std::max_element(wgs.begin(), wgs.end())));
  auto launch = [&](int tile, int w) {
    hip_check(q2c::launch_pauli(db, p->dev.str_x, p->dev.str_z, ns, p->dev.str_order, p->dev.str_share,
                                scr.as<double2>(), w, B.cm, ev_re, ev_im, tile, st),
              "pauli (tuning)");
  };
  Events ev;
  hip_check(hipEventRecord(ev.e[0], st), "event");
  launch(0, base);
  hip_check(hipEventRecord(ev.e[1], st), "event");
  hip_check(hipEventSynchronize(ev.e[1]), "sync");
  PauliCfg best{0, base, ev.ms(0, 1)};
  if (best.ms > kTuneMaxMs) {
    p->ctx->tuner.store(pauli_key(p, db, n_slots), best);
    return best;
  }
  best.ms = 1e300;
  for (int tile = 0; tile < q2c::kPauliTiles; ++tile)
    for (int w : wgs) {
      hip_check(hipEventRecord(ev.e[0], st), "event");
      launch(tile, w);
      hip_check(hipEventRecord(ev.e[1], st), "event");
      hip_check(hipEventSynchronize(ev.e[1]), "sync");
      const double ms = ev.ms(0, 1);
      if (ms < best.ms) best = PauliCfg{tile, w, ms};
    }
  ctx->tuner.store(pauli_key(p, db, n_slots), best);
  return best;
}

// The Pauli-sweep choice for a batch shape: tuned, or the default when
// tuning is off; *need_tuning tells whether the shape is still untuned.
PauliCfg pauli_choice(const vqe_problem* p, const q2c::DevBatch& db, int n_slots, bool* need_tuning) {
  const PauliCfg* t = p->ctx->tuner.find(pauli_key(p, db, n_slots));
  *need_tuning = !t && !p->ctx->opts.no_autotune;
  if (t) return *t;
  return PauliCfg{0, pauli_workgroups(p->dev.n_strings, n_slots), 0.0};
}

// Energies of slots 0 .. n_slots-1 of db, whose gates have all run:
// environments, Pauli sweeps, reduction; reads back energies, flags and
// statistics and synchronises the stream.
void finish_circuits(vqe_problem* p, const Batch& B, const q2c::DevBatch& db, int n_slots, double* energies,
                     std::vector<double>& stats_out, PhaseTimes& pt) {
  Events ev;
  q2c_ctx* ctx = p->ctx;
  hipStream_t st = ctx->stream;
  const auto& H = p->host;
  hip_check(hipEventRecord(ev.e[0], st), "event");
  hip_check(q2c::launch_envs(db, st), "envs");
  hip_check(hipEventRecord(ev.e[1], st), "event");
  const int ns = p->dev.n_strings;
  ensure(ctx, p->ev_re, p->evr_cap, sizeof(double) * std::max<size_t>(1, size_t(n_slots) * ns));
  ensure(ctx, p->ev_im, p->evi_cap, sizeof(double) * std::max<size_t>(1, size_t(n_slots) * ns));
  bool need_tuning = false;
  PauliCfg cfg = pauli_choice(p, db, n_slots, &need_tuning);
  if (need_tuning)
    cfg = tune_pauli(p, B, db, n_slots, p->ev_re.as<double>(), p->ev_im.as<double>(), st, &pt.tune_ms);
  pt.pauli = cfg;
  ensure(ctx, p->scratch, p->scratch_cap, pauli_scratch_bytes(p, B, n_slots, cfg.n_wg));
  hip_check(hipEventRecord(ev.e[2], st), "event");
  hip_check(q2c::launch_pauli(db, p->dev.str_x, p->dev.str_z, ns, p->dev.str_order, p->dev.str_share,
                              p->scratch.as<double2>(), cfg.n_wg, B.cm, p->ev_re.as<double>(), p->ev_im.as<double>(),
                              cfg.tile, st),
            "pauli");
  hip_check(hipEventRecord(ev.e[3], st), "event");
  ensure(ctx, p->energies, p->en_cap, sizeof(double) * n_slots);
  hip_check(q2c::launch_energy_reduce(db, p->dev.str_c, p->ev_re.as<double>(), p->ev_im.as<double>(), ns,
                                      H.c_identity, p->energies.as<double>(), st),
            "reduce");
  hip_check(hipEventRecord(ev.e[4], st), "event");
  std::vector<int> flags(n_slots);
  stats_out.assign(size_t(n_slots) * q2c::kNStats, 0.0);
  hip_check(hipMemcpyAsync(energies, p->energies.p, sizeof(double) * n_slots, hipMemcpyDeviceToHost, st), "copy E");
  hip_check(hipMemcpyAsync(flags.data(), db.flags + db.slot0, sizeof(int) * n_slots, hipMemcpyDeviceToHost, st),
            "copy flags");
  hip_check(hipMemcpyAsync(stats_out.data(), db.stats + size_t(db.slot0) * q2c::kNStats,
                           sizeof(double) * n_slots * q2c::kNStats, hipMemcpyDeviceToHost, st),
            "copy stats");
  hip_check(hipStreamSynchronize(st), "sync");
  pt.env_ms += ev.ms(0, 1);
  pt.pauli_ms += ev.ms(2, 3);
  pt.reduce_ms += ev.ms(3, 4);
  pt.circuits += n_slots;
  check_flags(flags);
  for (int i = 0; i < n_slots; ++i)
    if (!std::isfinite(energies[i])) throw StatusError(Q2C_ERR_NUMERIC, "non-finite energy");
}

// Runs n_slots circuits of problem p with theta (n_slots x n_params) and
// optional per-slot shifts; writes per-slot energies.
void run_circuits(vqe_problem* p, int D, int precision, const double* theta, int n_slots, const int* shift_rot,
                  const double* shift_val, double* energies, std::vector<double>& stats_out, PhaseTimes& pt) {
  Events ev;
  q2c_ctx* ctx = p->ctx;
  ctx->activate();
  hipStream_t st = ctx->stream;
  const int np = p->host.n_params;
  Batch& B = batch_for(p, D, n_slots, precision);
  q2c::DevBatch db = B.d;

  ensure(ctx, p->theta, p->theta_cap, sizeof(double) * std::max(1, n_slots * np));
  if (np) hip_check(hipMemcpyAsync(p->theta.p, theta, sizeof(double) * n_slots * np, hipMemcpyHostToDevice, st), "copy theta");
  const int* d_shift_rot = nullptr;
  const double* d_shift_val = nullptr;
  if (shift_rot) {
    ensure(ctx, p->shift_rot, p->srot_cap, sizeof(int) * n_slots);
    ensure(ctx, p->shift_val, p->sval_cap, sizeof(double) * n_slots);
    hip_check(hipMemcpyAsync(p->shift_rot.p, shift_rot, sizeof(int) * n_slots, hipMemcpyHostToDevice, st), "copy shifts");
    hip_check(hipMemcpyAsync(p->shift_val.p, shift_val, sizeof(double) * n_slots, hipMemcpyHostToDevice, st), "copy shifts");
    d_shift_rot = p->shift_rot.as<int>();
    d_shift_val = p->shift_val.as<double>();
  }
  const int nr = std::max(1, p->dev.n_rot);
  ensure(ctx, p->phi, p->phi_cap, sizeof(double) * size_t(n_slots) * nr);
  db.phi = p->phi.as<double>();

  hip_check(q2c::launch_init_product(db, p->occ.as<uint8_t>(), st), "init");
  hip_check(q2c::launch_angles(db, p->dev, p->theta.as<double>(), np, d_shift_rot, d_shift_val, st), "angles");
  hip_check(hipEventRecord(ev.e[0], st), "event");
  pt.gate_launches += run_gates(p, db, 0, p->dev.n_gates, st);
  hip_check(hipEventRecord(ev.e[1], st), "event");
  finish_circuits(p, B, db, n_slots, energies, stats_out, pt);
  pt.gate_ms += ev.ms(0, 1);
}

// Snapshot store idx (0 or 1) of shape (D, precision); fork graphs of kind
// idx + 1 read it.
SlotStore& snap_store(vqe_problem* p, int D, int precision, int slots, int idx) {
  auto key = std::make_tuple(D, precision, idx);
  auto& ss = p->snaps[key];
  if (!ss || ss->d.n_slots < slots) {
    for (auto it = p->graphs.begin(); it != p->graphs.end();)  // fork graphs read the old store
      it = (std::get<0>(it->first) == D && std::get<2>(it->first) == precision && std::get<3>(it->first) == idx + 1)
               ? p->graphs.erase(it)
               : std::next(it);
    ss.reset();
    ss = std::make_unique<SlotStore>(p->ctx, batch_for(p, D, 1, precision).d, slots);
  }
  return *ss;
}

// Enqueues one batch of G on stream cs (the capture stream).
void enqueue_batch(vqe_problem* p, const Batch& B, BatchGraph& G, const SlotStore* snaps, hipStream_t cs) {
  const auto& H = p->host;
  const int nb = G.nb, np = H.n_params, ns = p->dev.n_strings;
  auto h2d = [&](DBuf& dst, const HostBuf& src, size_t bytes) {
    hip_check(hipMemcpyAsync(dst.p, src.p, bytes, hipMemcpyHostToDevice, cs), "graph input");
  };
  if (np) h2d(G.theta, *G.h_theta, sizeof(double) * size_t(nb) * np);
  h2d(G.srot, *G.h_srot, sizeof(int) * nb);
  h2d(G.sval, *G.h_sval, sizeof(double) * nb);
  h2d(G.cursor, *G.h_cursor, sizeof(int) * nb);
  if (G.fork) h2d(G.pairs, *G.h_pairs, sizeof(int2) * nb);
  q2c::DevBatch db = B.d;
  db.phi = G.phi.as<double>();
  db.cursor = G.cursor.as<int>();
  db.n_gates = p->dev.n_gates;
  hip_check(q2c::launch_angles(db, p->dev, G.theta.as<double>(), np, G.srot.as<int>(), G.sval.as<double>(), cs),
            "angles");
  if (G.fork)
    hip_check(q2c::launch_copy_slots(snaps->d, db, G.pairs.as<int2>(), nb, make_int2(0, 0), true, cs), "restore");
  else
    hip_check(q2c::launch_init_product(db, p->occ.as<uint8_t>(), cs), "init");
  const q2c::SvdParams sp = svd_params(p->ctx);
  G.launches = 0;
  for (int c0 = 0; c0 < p->dev.n_gates; c0 += kGateChunk, ++G.launches)
    hip_check(q2c::launch_gates(db, p->dev.gate_site, p->dev.gate_rot, p->dev.gate_pre, p->dev.gate_post, 0,
                                kGateChunk, p->dev.n_rot, sp, cs),
              "gates");
  hip_check(q2c::launch_envs(db, cs), "envs");
  hip_check(q2c::launch_pauli(db, p->dev.str_x, p->dev.str_z, ns, p->dev.str_order, p->dev.str_share,
                              G.scratch.as<double2>(), G.cfg.n_wg, B.cm, G.ev_re.as<double>(), G.ev_im.as<double>(),
                              G.cfg.tile, cs),
            "pauli");
  hip_check(q2c::launch_energy_reduce(db, p->dev.str_c, G.ev_re.as<double>(), G.ev_im.as<double>(), ns, H.c_identity,
                                      G.energy.as<double>(), cs),
            "reduce");
  hip_check(hipMemcpyAsync(G.h_energy->p, G.energy.p, sizeof(double) * nb, hipMemcpyDeviceToHost, cs), "graph output");
  hip_check(hipMemcpyAsync(G.h_flags->p, db.flags, sizeof(int) * nb, hipMemcpyDeviceToHost, cs), "graph output");
  hip_check(hipMemcpyAsync(G.h_stats->p, db.stats, sizeof(double) * nb * q2c::kNStats, hipMemcpyDeviceToHost, cs),
            "graph output");
}

// (Re)captures G with its current Pauli choice on a private stream.
void capture_graph(vqe_problem* p, const Batch& B, BatchGraph& G, const SlotStore* snaps) {
  q2c_ctx* ctx = p->ctx;
  G.release_graph();
  G.scratch = DBuf(ctx, pauli_scratch_bytes(p, B, G.nb, G.cfg.n_wg));
  hipStream_t cs = nullptr;
  hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } guard{cs};
  hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  try {
    enqueue_batch(p, B, G, snaps, cs);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(cs, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hip_check(hipStreamEndCapture(cs, &G.graph), "hipStreamEndCapture");
  hip_check(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
}

// Runs nb circuits through the batch graph of their shape (captured on first
// use): theta nb x n_params; per slot a shift target (see launch_angles) and
// shift, a first gate (0, or the fork gate) and, for fork kinds 1 / 2, the
// slot of snapshot store 0 / 1 to start from.  Writes energies and per-slot
// statistics.  After the first replay of an untuned shape the Pauli sweep is
// tuned on the live state and the graph re-captured if the choice changed.
void run_graph(vqe_problem* p, int D, int precision, int nb, int fork_kind, const double* theta, const int* srot,
               const double* sval, const int* first_gate, const int* snap_slot, const SlotStore* snaps,
               double* energies, std::vector<double>& stats_out, PhaseTimes& pt) {
  const bool fork = fork_kind != 0;
  q2c_ctx* ctx = p->ctx;
  ctx->activate();
  hipStream_t st = ctx->stream;
  const auto& H = p->host;
  const int np = H.n_params, ns = p->dev.n_strings;
  Batch& B = batch_for(p, D, nb, precision);
  auto key = std::make_tuple(D, nb, precision, fork_kind);
  auto& gp = p->graphs[key];
  if (!gp) {
    auto G = std::make_unique<BatchGraph>();
    G->nb = nb;
    G->fork = fork;
    bool need = false;
    G->cfg = pauli_choice(p, B.d, nb, &need);
    G->tuned = !need;
    G->h_theta = std::make_unique<HostBuf>(sizeof(double) * size_t(nb) * std::max(1, np));
    G->h_srot = std::make_unique<HostBuf>(sizeof(int) * nb);
    G->h_sval = std::make_unique<HostBuf>(sizeof(double) * nb);
    G->h_cursor = std::make_unique<HostBuf>(sizeof(int) * nb);
    G->h_pairs = std::make_unique<HostBuf>(sizeof(int2) * nb);
    G->h_energy = std::make_unique<HostBuf>(sizeof(double) * nb);
    G->h_flags = std::make_unique<HostBuf>(sizeof(int) * nb);
    G->h_stats = std::make_unique<HostBuf>(sizeof(double) * nb * q2c::kNStats);
    G->theta = DBuf(ctx, sizeof(double) * size_t(nb) * std::max(1, np));
    G->srot = DBuf(ctx, sizeof(int) * nb);
    G->sval = DBuf(ctx, sizeof(double) * nb);
    G->cursor = DBuf(ctx, sizeof(int) * nb);
    G->pairs = DBuf(ctx, sizeof(int2) * nb);
    G->phi = DBuf(ctx, sizeof(double) * size_t(nb) * std::max(1, p->dev.n_rot));
    G->ev_re = DBuf(ctx, sizeof(double) * std::max<size_t>(1, size_t(nb) * ns));
    G->ev_im = DBuf(ctx, sizeof(double) * std::max<size_t>(1, size_t(nb) * ns));
    G->energy = DBuf(ctx, sizeof(double) * nb);
    capture_graph(p, B, *G, snaps);
    gp = std::move(G);
  }
  BatchGraph& G = *gp;
  // inputs (the previous replay on this stream has completed: every call synchronises)
  if (np) std::memcpy(G.h_theta->p, theta, sizeof(double) * size_t(nb) * np);
  for (int i = 0; i < nb; ++i) {
    G.h_srot->as<int>()[i] = srot ? srot[i] : -1;
    G.h_sval->as<double>()[i] = sval ? sval[i] : 0.0;
    G.h_cursor->as<int>()[i] = first_gate ? first_gate[i] : 0;
    G.h_pairs->as<int2>()[i] = make_int2(snap_slot ? snap_slot[i] : 0, i);
  }
  Events ev;
  hip_check(hipEventRecord(ev.e[0], st), "event");
  hip_check(hipGraphLaunch(G.exec, st), "hipGraphLaunch");
  hip_check(hipEventRecord(ev.e[1], st), "event");
  hip_check(hipStreamSynchronize(st), "sync");
  pt.graph_ms += ev.ms(0, 1);
  pt.graph_launches += 1;
  pt.gate_launches += G.launches;
  pt.circuits += nb;
  pt.pauli = G.cfg;
  std::memcpy(energies, G.h_energy->p, sizeof(double) * nb);
  std::vector<int> flags(G.h_flags->as<int>(), G.h_flags->as<int>() + nb);
  stats_out.assign(G.h_stats->as<double>(), G.h_stats->as<double>() + size_t(nb) * q2c::kNStats);
  if (progress_enabled() && ev.ms(0, 1) >= 1000.0) {  // long batches only
    std::fprintf(stderr, "[q2c] %d circuit(s): batch graph replayed, %.1f s\n", nb, ev.ms(0, 1) / 1e3);
    std::fflush(stderr);
  }
  check_flags(flags);
  for (int i = 0; i < nb; ++i)
    if (!std::isfinite(energies[i])) throw StatusError(Q2C_ERR_NUMERIC, "non-finite energy");
  if (!G.tuned) {
    q2c::DevBatch db = B.d;
    const PauliCfg best = tune_pauli(p, B, db, nb, G.ev_re.as<double>(), G.ev_im.as<double>(), st, &pt.tune_ms);
    G.tuned = true;
    if (best.tile != G.cfg.tile || best.n_wg != G.cfg.n_wg) {
      G.cfg = best;
      capture_graph(p, B, G, snaps);
    } else {
      G.cfg = best;
    }
  }
}

bool use_graphs(const vqe_problem* p) { return !p->ctx->opts.eager_batches; }

void check_theta(const vqe_problem* p, const double* theta, int n_theta, int count) {
  require(theta != nullptr || p->host.n_params == 0, "theta is NULL");
  if (n_theta != p->host.n_params)
    throw ArgError("n_theta (" + std::to_string(n_theta) + ") != number of UCCSD parameters (" +
                   std::to_string(p->host.n_params) + ")");
  for (long i = 0; i < long(count) * n_theta; ++i)
    if (!std::isfinite(theta[i])) throw ArgError("non-finite theta");
}

void check_eval(const vqe_problem* p, int max_bond, int precision) {
  require(p != nullptr, "NULL problem");
  if (!p->ctx) throw ArgError("problem was compiled without a context (host-only)");
  require(max_bond >= 1 && max_bond <= 256, "max_bond must be in 1..256");
  require(precision == Q2C_FP64 || precision == Q2C_MIXED, "unknown precision");
}

int chunk_slots(const vqe_problem* p) { return std::max(1, p->ctx->opts.slots); }

}  // namespace

// ------------------------------------------------------------------ exports --

extern "C" {

const char* q2c_last_error(void) { return g_last_error.c_str(); }
const char* q2c_version(void) { return "q2c 0.1 (gfx950, FP64)"; }

int q2c_ctx_create(int device, void* hip_stream, const q2c_opts* opts, q2c_ctx** out) {
  return guarded([&] {
    require(out != nullptr, "out is NULL");
    int ndev = 0;
    const hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0)
      throw DeviceError(std::string("no HIP device available (") + hipGetErrorString(e) +
                        "); a second HIP runtime loaded in this process also causes this");
    require(device >= 0 && device < ndev, "device ordinal out of range");
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      throw DeviceError(std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    auto c = std::make_unique<q2c_ctx>();
    c->device = device;
    c->activate();
    q2c_opts o{};
    if (opts) o = *opts;
    if (o.max_sweeps <= 0) o.max_sweeps = 60;
    if (!(o.sv_cutoff_rel > 0)) o.sv_cutoff_rel = 1e-12;
    if (!(o.svd_tol > 0)) o.svd_tol = 1e-15;
    if (o.slots <= 0) o.slots = 256;
    if (o.hbm_budget_bytes == 0) o.hbm_budget_bytes = size_t(64) << 30;
    require(o.sv_cutoff_rel < 1.0 && o.svd_tol < 1e-3, "bad tolerances");
    require(o.svd_algorithm == 0 || o.svd_algorithm == 1, "svd_algorithm must be 0 or 1");
    require(o.shift_from_start == 0 || o.shift_from_start == 1, "shift_from_start must be 0 or 1");
    require(o.eager_batches == 0 || o.eager_batches == 1, "eager_batches must be 0 or 1");
    require(o.no_autotune == 0 || o.no_autotune == 1, "no_autotune must be 0 or 1");
    require(o.grad_rule == 0 || o.grad_rule == 1, "grad_rule must be 0 or 1");
    c->tuner.load(o.autotune_cache);
    o.autotune_cache = nullptr;  // the caller's string is not kept
    c->opts = o;
    if (hip_stream) {
      c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      hip_check(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "hipStreamCreate");
      c->own_stream = true;
    }
    *out = c.release();
  });
}

int q2c_ctx_memory(const q2c_ctx* ctx, size_t* bytes_in_use, size_t* budget_bytes) {
  return guarded([&] {
    require(ctx != nullptr, "NULL context");
    if (bytes_in_use) *bytes_in_use = ctx->bytes_in_use;
    if (budget_bytes) *budget_bytes = ctx->opts.hbm_budget_bytes;
  });
}

int q2c_ctx_destroy(q2c_ctx* ctx) {
  return guarded([&] {
    require(ctx != nullptr, "NULL context");
    ctx->activate();
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->aux) {
      (void)hipStreamSynchronize(ctx->aux);
      (void)hipStreamDestroy(ctx->aux);
    }
    delete ctx;
  });
}

int mps_create(q2c_ctx* ctx, int n_qubits, int max_bond, int precision, const uint8_t* occ, mps_state** out) {
  return guarded([&] {
    require(ctx && out && occ, "NULL argument");
    require(n_qubits >= 2 && n_qubits <= q2c::kMaxQubits, "n_qubits must be in 2..64");
    require(max_bond >= 1 && max_bond <= 256, "max_bond must be in 1..256");
    require(precision == Q2C_FP64 || precision == Q2C_MIXED, "unknown precision");
      for (int i = 0; i < n_qubits; ++i) require(occ[i] <= 1, "occ entries must be 0 or 1");
    ctx->activate();
    auto s = std::make_unique<mps_state>();
    s->ctx = ctx;
    s->n = n_qubits;
    s->D = max_bond;
    s->precision = precision;
    s->batch = std::make_unique<Batch>(ctx, n_qubits, max_bond, 1, precision);
    s->occ = DBuf(ctx, n_qubits);
    s->gsite = DBuf(ctx, sizeof(int));
    s->grot = DBuf(ctx, sizeof(int));
    s->gmat = DBuf(ctx, 32 * sizeof(double));
    hip_check(hipMemcpyAsync(s->occ.p, occ, n_qubits, hipMemcpyHostToDevice, ctx->stream), "copy occ");
    const int m1 = -1;
    hip_check(hipMemcpyAsync(s->grot.p, &m1, sizeof(int), hipMemcpyHostToDevice, ctx->stream), "copy");
    hip_check(q2c::launch_init_product(s->batch->d, s->occ.as<uint8_t>(), ctx->stream), "init");
    hip_check(hipStreamSynchronize(ctx->stream), "sync");
    *out = s.release();
  });
}

int mps_destroy(mps_state* s) {
  return guarded([&] {
    require(s != nullptr, "NULL state");
    s->ctx->activate();
    (void)hipStreamSynchronize(s->ctx->stream);
    delete s;
  });
}

int mps_copy(mps_state* src, mps_state* dst) {
  return guarded([&] {
    require(src && dst, "NULL state");
    require(src != dst, "src and dst are the same state");
    require(src->ctx == dst->ctx, "src and dst belong to different contexts");
    require(src->n == dst->n && src->D == dst->D && src->precision == dst->precision,
            "src and dst differ in qubits, max_bond or precision");
    q2c_ctx* ctx = src->ctx;
    ctx->activate();
    hip_check(q2c::launch_copy_slots(src->batch->d, dst->batch->d, nullptr, 1, make_int2(0, 0), false, ctx->stream),
              "copy");
    hip_check(hipStreamSynchronize(ctx->stream), "sync");
  });
}

int mps_apply_gate(mps_state* s, int site, const double* gate, double* discarded_weight) {
  return guarded([&] {
    require(s && gate, "NULL argument");
    require(site >= 0 && site <= s->n - 2, "site must be in 0..n_qubits-2");
    for (int i = 0; i < 32; ++i) require(std::isfinite(gate[i]), "non-finite gate entry");
    q2c_ctx* ctx = s->ctx;
    ctx->activate();
    hipStream_t st = ctx->stream;
    std::vector<double> before(q2c::kNStats), after(q2c::kNStats);
    q2c::DevBatch& db = s->batch->d;
    hip_check(hipMemcpyAsync(s->gsite.p, &site, sizeof(int), hipMemcpyHostToDevice, st), "copy");
    hip_check(hipMemcpyAsync(s->gmat.p, gate, 32 * sizeof(double), hipMemcpyHostToDevice, st), "copy");
    hip_check(hipMemcpyAsync(before.data(), db.stats, sizeof(double) * q2c::kNStats, hipMemcpyDeviceToHost, st), "copy");
    hip_check(q2c::launch_gates(db, s->gsite.as<int>(), s->grot.as<int>(), s->gmat.as<double2>(),
                                s->gmat.as<double2>(), 0, 1, 0, svd_params(ctx), st),
              "gate");
    int flag = 0;
    hip_check(hipMemcpyAsync(&flag, db.flags, sizeof(int), hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipMemcpyAsync(after.data(), db.stats, sizeof(double) * q2c::kNStats, hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipStreamSynchronize(st), "sync");
    check_flags({flag});
    if (discarded_weight) *discarded_weight = after[q2c::kStatDisc] - before[q2c::kStatDisc];
  });
}

int mps_expect_pauli_batch(mps_state* s, int n_strings, int n_words, const uint64_t* x_masks,
                           const uint64_t* z_masks, double* out_re, double* out_im) {
  return guarded([&] {
    require(s && out_re, "NULL argument");
    require(n_strings >= 0, "n_strings < 0");
    require(n_words == (s->n + 63) / 64, "n_words must be ceil(n_qubits/64)");
    if (n_strings == 0) return;
    require(x_masks && z_masks, "NULL masks");
    const uint64_t valid = s->n == 64 ? ~0ull : ((1ull << s->n) - 1);
    for (int i = 0; i < n_strings; ++i)
      require(((x_masks[i] | z_masks[i]) & ~valid) == 0, "mask bits beyond n_qubits");
    q2c_ctx* ctx = s->ctx;
    ctx->activate();
    hipStream_t st = ctx->stream;
    Batch& B = *s->batch;
    s->sx = DBuf(ctx, sizeof(uint64_t) * n_strings);
    s->sz = DBuf(ctx, sizeof(uint64_t) * n_strings);
    s->ev_re = DBuf(ctx, sizeof(double) * n_strings);
    s->ev_im = DBuf(ctx, sizeof(double) * n_strings);
    hip_check(hipMemcpyAsync(s->sx.p, x_masks, sizeof(uint64_t) * n_strings, hipMemcpyHostToDevice, st), "copy");
    hip_check(hipMemcpyAsync(s->sz.p, z_masks, sizeof(uint64_t) * n_strings, hipMemcpyHostToDevice, st), "copy");
    const q2c::PrefixOrder po = q2c::pauli_prefix_order(x_masks, z_masks, n_strings);
    s->sord = DBuf(ctx, sizeof(int) * n_strings);
    s->sshr = DBuf(ctx, sizeof(int) * n_strings);
    hip_check(hipMemcpyAsync(s->sord.p, po.order.data(), sizeof(int) * n_strings, hipMemcpyHostToDevice, st), "copy");
    hip_check(hipMemcpyAsync(s->sshr.p, po.share.data(), sizeof(int) * n_strings, hipMemcpyHostToDevice, st), "copy");
    const int n_wg = pauli_workgroups(n_strings, 1);
    if (s->scratch_wg < n_wg) {
      s->scratch = DBuf(ctx, size_t(n_wg) * q2c::pauli_scratch_mats(s->n) * B.cm * B.cm * sizeof(double2));
      s->scratch_wg = n_wg;
    }
    hip_check(q2c::launch_envs(B.d, st), "envs");
    hip_check(q2c::launch_pauli(B.d, s->sx.as<uint64_t>(), s->sz.as<uint64_t>(), n_strings, s->sord.as<int>(),
                                s->sshr.as<int>(), s->scratch.as<double2>(), n_wg, B.cm, s->ev_re.as<double>(),
                                s->ev_im.as<double>(), 0, st),
              "pauli");
    hip_check(hipMemcpyAsync(out_re, s->ev_re.p, sizeof(double) * n_strings, hipMemcpyDeviceToHost, st), "copy");
    if (out_im) hip_check(hipMemcpyAsync(out_im, s->ev_im.p, sizeof(double) * n_strings, hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipStreamSynchronize(st), "sync");
  });
}

int q2c_pauli_prefix_order(int n_strings, const uint64_t* x_masks, const uint64_t* z_masks, int* order, int* share,
                           int64_t* steps) {
  return guarded([&] {
    require(n_strings >= 0, "n_strings < 0");
    if (n_strings == 0) return;
    require(x_masks && z_masks && order && share, "NULL argument");
    const q2c::PrefixOrder po = q2c::pauli_prefix_order(x_masks, z_masks, n_strings);
    std::copy(po.order.begin(), po.order.end(), order);
    std::copy(po.share.begin(), po.share.end(), share);
    if (steps) {
      steps[0] = po.steps_plain;
      steps[1] = po.steps_shared;
    }
  });
}

int mps_export(mps_state* s, int* chi_out, double* tensors, double* lambdas) {
  return guarded([&] {
    require(s && chi_out, "NULL argument");
    q2c_ctx* ctx = s->ctx;
    ctx->activate();
    hipStream_t st = ctx->stream;
    const q2c::DevBatch& b = s->batch->d;
    const int N = s->n;
    std::vector<double2> sites(b.site_stride);
    std::vector<float2> sites32(b.mixed ? b.site_stride : 0);
    std::vector<double> lam(b.lam_stride);
    hip_check(hipMemcpyAsync(chi_out, b.chi, sizeof(int) * (N + 1), hipMemcpyDeviceToHost, st), "copy");
    if (b.mixed)
      hip_check(hipMemcpyAsync(sites32.data(), b.sites, sizeof(float2) * b.site_stride, hipMemcpyDeviceToHost, st),
                "copy");
    else
      hip_check(hipMemcpyAsync(sites.data(), b.sites, sizeof(double2) * b.site_stride, hipMemcpyDeviceToHost, st),
                "copy");
    hip_check(hipMemcpyAsync(lam.data(), b.lam, sizeof(double) * b.lam_stride, hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipStreamSynchronize(st), "sync");
    if (b.mixed)
      for (long i = 0; i < b.site_stride; ++i) sites[i] = make_double2(sites32[i].x, sites32[i].y);
    if (tensors) {
      size_t o = 0;
      for (int n = 0; n < N; ++n) {
        const int cl = chi_out[n], cr = chi_out[n + 1], capr = b.cap[n + 1];
        for (int a = 0; a < cl; ++a)
          for (int i = 0; i < 2; ++i)
            for (int c = 0; c < cr; ++c) {
              const double2 v = sites[b.site_off[n] + (long(2 * a + i)) * capr + c];
              tensors[o++] = v.x;
              tensors[o++] = v.y;
            }
      }
    }
    if (lambdas) {
      size_t o = 0;
      for (int bb = 0; bb < N - 1; ++bb)
        for (int k = 0; k < chi_out[bb + 1]; ++k) lambdas[o++] = lam[b.lam_off[bb] + k];
    }
  });
}

int mps_get_stats(mps_state* s, q2c_stats* stats) {
  return guarded([&] {
    require(s && stats, "NULL argument");
    s->ctx->activate();
    std::vector<double> st(q2c::kNStats);
    hip_check(hipMemcpy(st.data(), s->batch->d.stats, sizeof(double) * q2c::kNStats, hipMemcpyDeviceToHost), "copy");
    fill_stats(stats, st, 1, 0.0);
  });
}

int vqe_problem_create(q2c_ctx* ctx, int n_orb, int n_elec, const double* h1, const double* eri, double e_const,
                       vqe_problem** out) {
  return guarded([&] {
    require(out != nullptr, "out is NULL");
    auto p = std::make_unique<vqe_problem>();
    p->host = q2c::compile_problem(n_orb, n_elec, h1, eri, e_const);
    p->ctx = ctx;
    if (ctx) {
      ctx->activate();
      hipStream_t st = ctx->stream;
      const auto& H = p->host;
      auto& d = p->dev;
      d.n_qubits = H.n_qubits;
      d.n_gates = int(H.gates.size());
      d.n_rot = int(H.rotations.size());
      d.n_strings = int(H.terms.size());
      std::vector<int> site(d.n_gates), rot(d.n_gates);
      std::vector<double2> pre(size_t(d.n_gates) * 16), post(size_t(d.n_gates) * 16);
      for (int g = 0; g < d.n_gates; ++g) {
        site[g] = H.gates[g].site;
        rot[g] = H.gates[g].rot;
        for (int i = 0; i < 16; ++i) {
          pre[size_t(g) * 16 + i] = make_double2(H.gates[g].pre[i].real(), H.gates[g].pre[i].imag());
          post[size_t(g) * 16 + i] = make_double2(H.gates[g].post[i].real(), H.gates[g].post[i].imag());
        }
      }
      std::vector<double> rc(d.n_rot), sc(d.n_strings);
      std::vector<int> rparam(d.n_rot);
      std::vector<uint64_t> sx(d.n_strings), sz(d.n_strings);
      for (int m = 0; m < d.n_rot; ++m) {
        rc[m] = H.rotations[m].c;
        rparam[m] = H.rotations[m].param;
      }
      for (int s = 0; s < d.n_strings; ++s) {
        sx[s] = H.terms[s].x;
        sz[s] = H.terms[s].z;
        sc[s] = H.terms[s].c;
      }
      std::vector<uint8_t> occ(H.n_qubits);
      for (int q = 0; q < H.n_qubits; ++q) occ[q] = q < H.n_elec ? 1 : 0;
      auto up = [&](DBuf& buf, const void* src, size_t bytes) {
        buf = DBuf(ctx, std::max<size_t>(bytes, 16));
        if (bytes) hip_check(hipMemcpyAsync(buf.p, src, bytes, hipMemcpyHostToDevice, st), "upload");
      };
      up(p->gsite, site.data(), sizeof(int) * site.size());
      up(p->grot, rot.data(), sizeof(int) * rot.size());
      up(p->gpre, pre.data(), sizeof(double2) * pre.size());
      up(p->gpost, post.data(), sizeof(double2) * post.size());
      up(p->rc, rc.data(), sizeof(double) * rc.size());
      up(p->rparam, rparam.data(), sizeof(int) * rparam.size());
      up(p->sx, sx.data(), sizeof(uint64_t) * sx.size());
      up(p->sz, sz.data(), sizeof(uint64_t) * sz.size());
      up(p->sc, sc.data(), sizeof(double) * sc.size());
      const q2c::PrefixOrder po = q2c::pauli_prefix_order(sx.data(), sz.data(), d.n_strings);
      up(p->sord, po.order.data(), sizeof(int) * po.order.size());
      up(p->sshr, po.share.data(), sizeof(int) * po.share.size());
      up(p->occ, occ.data(), occ.size());
      d.gate_site = p->gsite.as<int>();
      d.gate_rot = p->grot.as<int>();
      d.gate_pre = p->gpre.as<double2>();
      d.gate_post = p->gpost.as<double2>();
      d.rot_c = p->rc.as<double>();
      d.rot_param = p->rparam.as<int>();
      d.str_x = p->sx.as<uint64_t>();
      d.str_z = p->sz.as<uint64_t>();
      d.str_c = p->sc.as<double>();
      d.str_order = p->sord.as<int>();
      p->fork_gate.assign(H.rotations.size(), -1);
      for (size_t g = 0; g < H.gates.size(); ++g) {
        const int r = H.gates[g].rot;
        if (r >= 0 && p->fork_gate[r] < 0) p->fork_gate[r] = int(g);
      }
      for (int f : p->fork_gate)
        if (f < 0) throw std::logic_error("rotation without an angle-dependent gate");
      p->param_fork.assign(std::max(1, H.n_params), std::numeric_limits<int>::max());
      for (size_t m = 0; m < H.rotations.size(); ++m) {
        int& pf = p->param_fork[H.rotations[m].param];
        pf = std::min(pf, p->fork_gate[m]);
      }
      d.str_share = p->sshr.as<int>();
      hip_check(hipStreamSynchronize(st), "sync");
    }
    *out = p.release();
  });
}

int vqe_problem_destroy(vqe_problem* p) {
  return guarded([&] {
    require(p != nullptr, "NULL problem");
    if (p->ctx) {
      p->ctx->activate();
      (void)hipStreamSynchronize(p->ctx->stream);
    }
    delete p;
  });
}

int vqe_problem_info(const vqe_problem* p, int* n_qubits, int* n_params, int* n_strings, int* n_rotations,
                     int* n_gates, double* identity_coeff) {
  return guarded([&] {
    require(p != nullptr, "NULL problem");
    if (n_qubits) *n_qubits = p->host.n_qubits;
    if (n_params) *n_params = p->host.n_params;
    if (n_strings) *n_strings = int(p->host.terms.size());
    if (n_rotations) *n_rotations = int(p->host.rotations.size());
    if (n_gates) *n_gates = int(p->host.gates.size());
    if (identity_coeff) *identity_coeff = p->host.c_identity;
  });
}

int vqe_problem_electrons(const vqe_problem* p, int* n_orb, int* n_elec) {
  return guarded([&] {
    require(p != nullptr, "NULL problem");
    if (n_orb) *n_orb = p->host.n_orb;
    if (n_elec) *n_elec = p->host.n_elec;
  });
}

int vqe_problem_paulis(const vqe_problem* p, uint64_t* x, uint64_t* z, double* coeff) {
  return guarded([&] {
    require(p != nullptr, "NULL problem");
    const auto& t = p->host.terms;
    for (size_t i = 0; i < t.size(); ++i) {
      if (x) x[i] = t[i].x;
      if (z) z[i] = t[i].z;
      if (coeff) coeff[i] = t[i].c;
    }
  });
}

int vqe_problem_rotations(const vqe_problem* p, uint64_t* x, uint64_t* z, double* c, int* param) {
  return guarded([&] {
    require(p != nullptr, "NULL problem");
    const auto& r = p->host.rotations;
    for (size_t i = 0; i < r.size(); ++i) {
      if (x) x[i] = r[i].x;
      if (z) z[i] = r[i].z;
      if (c) c[i] = r[i].c;
      if (param) param[i] = r[i].param;
    }
  });
}

int vqe_problem_gates(const vqe_problem* p, int* site, int* rot, double* pre, double* post) {
  return guarded([&] {
    require(p != nullptr, "NULL problem");
    const auto& g = p->host.gates;
    for (size_t i = 0; i < g.size(); ++i) {
      if (site) site[i] = g[i].site;
      if (rot) rot[i] = g[i].rot;
      for (int k = 0; k < 16; ++k) {
        if (pre) {
          pre[i * 32 + 2 * k] = g[i].pre[k].real();
          pre[i * 32 + 2 * k + 1] = g[i].pre[k].imag();
        }
        if (post) {
          post[i * 32 + 2 * k] = g[i].post[k].real();
          post[i * 32 + 2 * k + 1] = g[i].post[k].imag();
        }
      }
    }
  });
}

int vqe_energy(vqe_problem* p, const double* theta, int n_theta, int max_bond, int precision, double* energy,
               q2c_stats* stats) {
  return guarded([&] {
    check_eval(p, max_bond, precision);
    require(energy != nullptr, "energy is NULL");
    check_theta(p, theta, n_theta, 1);
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<double> st;
    PhaseTimes pt;
    double e = 0.0;
    run_circuits(p, max_bond, precision, theta, 1, nullptr, nullptr, &e, st, pt);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *energy = e;
    fill_stats(stats, st, 1, secs, pt);
  });
}

int vqe_energy_batch(vqe_problem* p, const double* theta, int n_batch, int n_theta, int max_bond, int precision,
                     double* energies, q2c_stats* stats) {
  return guarded([&] {
    check_eval(p, max_bond, precision);
    require(energies != nullptr, "energies is NULL");
    require(n_batch >= 1, "n_batch must be >= 1");
    check_theta(p, theta, n_theta, n_batch);
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<double> out(n_batch), all_st, st;
    PhaseTimes pt;
    const int chunk = chunk_slots(p);
    for (int b0 = 0; b0 < n_batch; b0 += chunk) {
      const int nb = std::min(chunk, n_batch - b0);
      if (use_graphs(p))
        run_graph(p, max_bond, precision, nb, 0, theta + size_t(b0) * n_theta, nullptr, nullptr, nullptr, nullptr,
                  nullptr, out.data() + b0, st, pt);
      else
        run_circuits(p, max_bond, precision, theta + size_t(b0) * n_theta, nb, nullptr, nullptr, out.data() + b0, st,
                     pt);
      all_st.insert(all_st.end(), st.begin(), st.end());
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::copy(out.begin(), out.end(), energies);
    fill_stats(stats, all_st, n_batch, secs, pt);
  });
}

namespace {
// A shifted circuit: target t >= 0 shifts rotation angle phi_t, t = -2 - k
// shifts parameter theta_k (every rotation of it); see launch_angles.
struct ShiftCircuit {
  int target;
  double shift;
};

int fork_of(const vqe_problem* p, int target) {
  return target >= 0 ? p->fork_gate[target] : p->param_fork[-2 - target];
}

// Energies of the shifted circuits, each run from the first gate, then of the
// unshifted circuit if requested, in batches of the context's slot count.
void shift_energies_from_start(vqe_problem* p, const double* theta, const std::vector<ShiftCircuit>& cs, int max_bond,
                               int precision, std::vector<double>& en, bool want_base, std::vector<double>& all_st,
                               PhaseTimes& pt) {
  const int np = p->host.n_params;
  std::vector<int> srot;
  std::vector<double> sval;
  for (const auto& c : cs) {
    srot.push_back(c.target);
    sval.push_back(c.shift);
  }
  if (want_base) {
    srot.push_back(-1);
    sval.push_back(0.0);
  }
  const int total = int(srot.size());
  en.assign(total, 0.0);
  std::vector<double> st;
  const int chunk = chunk_slots(p);
  std::vector<double> th(size_t(chunk) * np);
  for (int b0 = 0; b0 < total; b0 += chunk) {
    const int nb = std::min(chunk, total - b0);
    for (int i = 0; i < nb; ++i) std::copy(theta, theta + np, th.begin() + size_t(i) * np);
    if (use_graphs(p))
      run_graph(p, max_bond, precision, nb, 0, th.data(), srot.data() + b0, sval.data() + b0, nullptr, nullptr,
                nullptr, en.data() + b0, st, pt);
    else
      run_circuits(p, max_bond, precision, th.data(), nb, srot.data() + b0, sval.data() + b0, en.data() + b0, st,
                   pt);
    all_st.insert(all_st.end(), st.begin(), st.end());
  }
}

// The same energies with the shared prefixes run once.  A shifted circuit
// agrees with the unshifted one up to the first gate that depends on its
// shifted angle (rotation) or angles (parameter), its fork gate.  One base
// slot runs the unshifted circuit and its state is copied at each fork gate;
// the shifted circuits start from that copy at their fork gate.  Circuits are
// taken in fork order, a batch of up to slots - 4 circuits with at most
// slots/2 distinct fork gates at a time, so the circuits of one batch have
// about the same number of gates left; every gate runs as in a run from the
// start, so the energies are the same bit for bit.  The base slot runs on the
// context's second stream one batch ahead, into the other of two snapshot
// stores, so its gates overlap the previous batch (the batch leaves a few
// compute units free for its workgroup); events order the two streams.
void shift_energies_forked(vqe_problem* p, const double* theta, const std::vector<ShiftCircuit>& cs, int max_bond,
                           int precision, std::vector<double>& en, bool want_base, std::vector<double>& all_st,
                           PhaseTimes& pt) {
  q2c_ctx* ctx = p->ctx;
  ctx->activate();
  hipStream_t st = ctx->stream, sb = ctx->aux_stream();
  const auto& H = p->host;
  const int np = H.n_params, n_gates = p->dev.n_gates;
  const int nc = int(cs.size());
  en.assign(nc + (want_base ? 1 : 0), 0.0);
  std::vector<int> ord(nc);
  for (int i = 0; i < nc; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int a, int b) { return fork_of(p, cs[a].target) < fork_of(p, cs[b].target); });
  const int C = chunk_slots(p);
  const int W = std::max(1, C / 2), Cb = std::max(1, C > 8 ? C - 4 : C);
  // batches: circuits ord[lo .. hi), their distinct fork gates and each circuit's snapshot slot
  struct Window {
    int lo, hi;
    std::vector<int> forks, snap_slot;
  };
  std::vector<Window> win;
  for (int i0 = 0; i0 < nc;) {
    Window w{i0, i0, {}, {}};
    while (w.hi < nc && w.hi - i0 < Cb) {
      const int f = fork_of(p, cs[ord[w.hi]].target);
      if (w.forks.empty() || f != w.forks.back()) {
        if (int(w.forks.size()) == W) break;
        w.forks.push_back(f);
      }
      w.snap_slot.push_back(int(w.forks.size()) - 1);
      ++w.hi;
    }
    i0 = w.hi;
    win.push_back(std::move(w));
  }
  // base slot: the unshifted circuit, on the second stream, in a batch of its own
  Batch& base = base_batch_for(p, max_bond, precision);
  SlotStore* store[2] = {&snap_store(p, max_bond, precision, W, 0), &snap_store(p, max_bond, precision, W, 1)};
  ensure(ctx, p->theta, p->theta_cap, sizeof(double) * size_t(std::max(1, C) * np));
  ensure(ctx, p->phi, p->phi_cap, sizeof(double) * size_t(C) * std::max(1, p->dev.n_rot));
  DBuf base_phi(ctx, sizeof(double) * std::max(1, p->dev.n_rot));
  DBuf base_theta(ctx, sizeof(double) * std::max(1, np));
  q2c::DevBatch bd = base.d;
  bd.phi = base_phi.as<double>();
  if (np) hip_check(hipMemcpyAsync(base_theta.p, theta, sizeof(double) * np, hipMemcpyHostToDevice, sb), "copy theta");
  hip_check(q2c::launch_init_product(bd, p->occ.as<uint8_t>(), sb), "init");
  hip_check(q2c::launch_angles(bd, p->dev, base_theta.as<double>(), np, nullptr, nullptr, sb), "angles");
  Events evb;  // base segments: e[0] .. e[1] around each; e[2]: base ready; e[3]: a batch done
  int cur = 0;
  double base_ms = 0.0;
  auto base_segment = [&](const Window& w, int idx) {
    hip_check(hipEventRecord(evb.e[0], sb), "event");
    for (size_t s = 0; s < w.forks.size(); ++s) {
      pt.gate_launches += run_gates(p, bd, cur, w.forks[s], sb);
      cur = std::max(cur, w.forks[s]);
      hip_check(q2c::launch_copy_slots(bd, store[idx]->d, nullptr, 1, make_int2(0, int(s)), false, sb), "snapshot");
    }
    hip_check(hipEventRecord(evb.e[1], sb), "event");
    hip_check(hipEventRecord(evb.e[2], sb), "event");
  };
  std::vector<double> st_batch, e_batch;
  if (!win.empty()) base_segment(win[0], 0);
  for (size_t wi = 0; wi < win.size(); ++wi) {
    const Window& w = win[wi];
    const int idx = int(wi & 1), nb = w.hi - w.lo;
    // this batch waits for its snapshots
    hip_check(hipStreamWaitEvent(st, evb.e[2], 0), "wait");
    hip_check(hipEventSynchronize(evb.e[1]), "sync");
    base_ms += evb.ms(0, 1);
    // the base slot runs ahead into the other store (free: the batch that read it has finished)
    if (wi + 1 < win.size()) base_segment(win[wi + 1], 1 - idx);
    std::vector<double> th(size_t(nb) * np), sval(nb);
    std::vector<int> srot(nb), cursor(nb);
    std::vector<int2> pairs(nb);
    for (int j = 0; j < nb; ++j) {
      const ShiftCircuit& c = cs[ord[w.lo + j]];
      std::copy(theta, theta + np, th.begin() + size_t(j) * np);
      srot[j] = c.target;
      sval[j] = c.shift;
      cursor[j] = fork_of(p, c.target);
      pairs[j] = make_int2(w.snap_slot[j], j);
    }
    e_batch.resize(nb);
    if (use_graphs(p)) {
      run_graph(p, max_bond, precision, nb, 1 + idx, th.data(), srot.data(), sval.data(), cursor.data(),
                w.snap_slot.data(), store[idx], e_batch.data(), st_batch, pt);
    } else {
      Events ev;
      Batch& B = batch_for(p, max_bond, nb, precision);
      q2c::DevBatch db = B.d;
      ensure(ctx, p->shift_rot, p->srot_cap, sizeof(int) * nb);
      ensure(ctx, p->shift_val, p->sval_cap, sizeof(double) * nb);
      ensure(ctx, p->cursor, p->cursor_cap, sizeof(int) * nb);
      ensure(ctx, p->pairs, p->pairs_cap, sizeof(int2) * nb);
      if (np)
        hip_check(hipMemcpyAsync(p->theta.p, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice, st),
                  "copy theta");
      hip_check(hipMemcpyAsync(p->shift_rot.p, srot.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st), "copy shifts");
      hip_check(hipMemcpyAsync(p->shift_val.p, sval.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st),
                "copy shifts");
      hip_check(hipMemcpyAsync(p->cursor.p, cursor.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st), "copy cursor");
      hip_check(hipMemcpyAsync(p->pairs.p, pairs.data(), sizeof(int2) * nb, hipMemcpyHostToDevice, st), "copy pairs");
      db.phi = p->phi.as<double>();
      hip_check(q2c::launch_angles(db, p->dev, p->theta.as<double>(), np, p->shift_rot.as<int>(),
                                   p->shift_val.as<double>(), st),
                "angles");
      hip_check(q2c::launch_copy_slots(store[idx]->d, db, p->pairs.as<int2>(), nb, make_int2(0, 0), true, st),
                "restore");
      db.cursor = p->cursor.as<int>();
      db.n_gates = n_gates;
      hip_check(hipEventRecord(ev.e[0], st), "event");
      pt.gate_launches += run_gates(p, db, 0, n_gates - w.forks.front(), st);
      hip_check(hipEventRecord(ev.e[1], st), "event");
      finish_circuits(p, B, db, nb, e_batch.data(), st_batch, pt);
      pt.gate_ms += ev.ms(0, 1);
    }
    // the segment for window wi + 2 refills store idx: it waits until this
    // batch (and its restore from that store) is done; the base tail does not
    if (wi + 2 < win.size()) {
      hip_check(hipEventRecord(evb.e[3], st), "event");
      hip_check(hipStreamWaitEvent(sb, evb.e[3], 0), "wait");
    }
    for (int j = 0; j < nb; ++j) en[ord[w.lo + j]] = e_batch[j];
    all_st.insert(all_st.end(), st_batch.begin(), st_batch.end());
  }
  // the base slot's own energy, or only its statistics (its gates count once)
  std::vector<double> st_base(q2c::kNStats);
  hip_check(hipEventRecord(evb.e[0], sb), "event");
  if (want_base) pt.gate_launches += run_gates(p, bd, cur, n_gates, sb);
  hip_check(hipEventRecord(evb.e[1], sb), "event");
  hip_check(hipEventSynchronize(evb.e[1]), "sync");
  base_ms += evb.ms(0, 1);
  pt.gate_ms += base_ms;
  if (want_base) {
    finish_circuits(p, base, bd, 1, &en[nc], st_base, pt);
  } else {
    std::vector<int> flag(1);
    hip_check(hipMemcpyAsync(st_base.data(), bd.stats, sizeof(double) * q2c::kNStats, hipMemcpyDeviceToHost, st),
              "copy stats");
    hip_check(hipMemcpyAsync(flag.data(), bd.flags, sizeof(int), hipMemcpyDeviceToHost, st), "copy flags");
    hip_check(hipStreamSynchronize(st), "sync");
    check_flags(flag);
    // physics statistics of a circuit that was not evaluated are not reported
    for (int k : {q2c::kStatNorm, q2c::kStatMaxImag}) st_base[k] = 0.0;
  }
  all_st.insert(all_st.end(), st_base.begin(), st_base.end());
}

// Energies of the shifted circuits cs (in order), then the unshifted one if
// base is given.
void shift_energies(vqe_problem* p, const double* theta, const std::vector<ShiftCircuit>& cs, int max_bond,
                    int precision, std::vector<double>& en, double* base, std::vector<double>& all_st,
                    PhaseTimes& pt) {
  if (p->ctx->opts.shift_from_start)
    shift_energies_from_start(p, theta, cs, max_bond, precision, en, base != nullptr, all_st, pt);
  else
    shift_energies_forked(p, theta, cs, max_bond, precision, en, base != nullptr, all_st, pt);
  if (base) *base = en[cs.size()];
}
}  // namespace

int vqe_grad_paramshift(vqe_problem* p, const double* theta, int n_theta, int max_bond, int precision, double* grad,
                        double* energy, q2c_stats* stats) {
  return guarded([&] {
    check_eval(p, max_bond, precision);
    require(grad != nullptr, "grad is NULL");
    check_theta(p, theta, n_theta, 1);
    const auto t0 = std::chrono::steady_clock::now();
    const auto& R = p->host.rotations;
    std::vector<ShiftCircuit> cs;
    std::vector<double> en, all_st;
    PhaseTimes pt;
    double base = 0.0;
    std::vector<double> g(n_theta, 0.0);
    if (p->ctx->opts.grad_rule == 0) {
      // two-term shift of every rotation angle: dE/dphi_m = (E(phi_m + pi/2) - E(phi_m - pi/2)) / 2
      for (size_t m = 0; m < R.size(); ++m) {
        cs.push_back({int(m), 0.5 * M_PI});
        cs.push_back({int(m), -0.5 * M_PI});
      }
      shift_energies(p, theta, cs, max_bond, precision, en, energy ? &base : nullptr, all_st, pt);
      for (size_t m = 0; m < R.size(); ++m) g[R[m].param] += -2.0 * R[m].c * 0.5 * (en[2 * m] - en[2 * m + 1]);
    } else {
      // four-term shift of every parameter (its rotations commute and their
      // generator has eigenvalues 0, +-1, so E(theta_k) has the frequencies 1
      // and 2): dE/dtheta_k = D(pi/4) + (1 - sqrt 2) / 2 D(pi/2),
      // D(s) = E(theta_k + s) - E(theta_k - s)
      for (int k = 0; k < n_theta; ++k)
        for (double sh : {0.5 * M_PI, -0.5 * M_PI, 0.25 * M_PI, -0.25 * M_PI}) cs.push_back({-2 - k, sh});
      shift_energies(p, theta, cs, max_bond, precision, en, energy ? &base : nullptr, all_st, pt);
      for (int k = 0; k < n_theta; ++k) {
        const double d1 = en[4 * k] - en[4 * k + 1], d2 = en[4 * k + 2] - en[4 * k + 3];
        g[k] = d2 + 0.5 * (1.0 - std::sqrt(2.0)) * d1;
      }
    }
    std::copy(g.begin(), g.end(), grad);
    if (energy) *energy = base;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(stats, all_st, int(all_st.size() / q2c::kNStats), secs, pt);
  });
}

int vqe_shift_energies(vqe_problem* p, const double* theta, int n_theta, const int* rot_idx, int n_rot, int max_bond,
                       int precision, double* e_plus, double* e_minus, q2c_stats* stats) {
  return guarded([&] {
    check_eval(p, max_bond, precision);
    require(rot_idx && e_plus && e_minus, "NULL argument");
    require(n_rot >= 1, "n_rot must be >= 1");
    check_theta(p, theta, n_theta, 1);
    std::vector<ShiftCircuit> cs;
    for (int i = 0; i < n_rot; ++i) {
      const int m = rot_idx[i];
      require(m >= 0 && m < int(p->host.rotations.size()), "rotation index out of range");
      cs.push_back({m, 0.5 * M_PI});
      cs.push_back({m, -0.5 * M_PI});
    }
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<double> en, all_st;
    PhaseTimes pt;
    shift_energies(p, theta, cs, max_bond, precision, en, nullptr, all_st, pt);
    for (int i = 0; i < n_rot; ++i) {
      e_plus[i] = en[2 * i];
      e_minus[i] = en[2 * i + 1];
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(stats, all_st, int(all_st.size() / q2c::kNStats), secs, pt);
  });
}

}  // extern "C"
