// Host runtime shared by the C ABI and the request server (internal to libq2c):
// error mapping, context, budgeted device buffers, slot batches, timing.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/q2c.h"
#include "compile.hpp"
#include "engine.hpp"

using q2c::cplx;

namespace q2c_rt {

extern thread_local std::string g_last_error;

struct ArgError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct DeviceError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct OomError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct StatusError : std::runtime_error {
  int code;
  StatusError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) throw OomError(std::string(what) + ": " + hipGetErrorString(e));
    throw DeviceError(std::string(what) + ": " + hipGetErrorString(e));
  }
}

template <class F>
inline int guarded(F&& f) {
  try {
    f();
    return Q2C_OK;
  } catch (const ArgError& e) {
    g_last_error = e.what();
    return Q2C_ERR_ARG;
  } catch (const std::invalid_argument& e) {
    g_last_error = e.what();
    return Q2C_ERR_ARG;
  } catch (const OomError& e) {
    g_last_error = e.what();
    return Q2C_ERR_OOM;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return Q2C_ERR_OOM;
  } catch (const StatusError& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const DeviceError& e) {
    g_last_error = e.what();
    return Q2C_ERR_DEVICE;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return Q2C_ERR_DEVICE;
  } catch (...) {
    g_last_error = "unknown error";
    return Q2C_ERR_DEVICE;
  }
}

inline void require(bool ok, const char* msg) {
  if (!ok) throw ArgError(msg);
}

}  // namespace

// ------------------------------------------------------------------ context --

using q2c_rt::hip_check;
using q2c_rt::OomError;

namespace q2c_rt {

// Launch choice of the Pauli sweep for one batch shape.
struct PauliCfg {
  int tile = 0;    // launch_pauli tile index
  int n_wg = 1;    // workgroups per circuit
  double ms = 0.0; // time measured when tuned (0: default, not measured)
};

// Tuned launch choices by batch shape (qubits, D, circuits, precision,
// strings), filled by timing every candidate on live data the first time a
// shape is seen; the choice never changes results, only time.  Entries can
// be read from and appended to a text file, one per line:
//   pauli n_qubits max_bond slots precision n_strings tile n_wg ms
struct Tuner {
  using Key = std::array<int, 5>;
  std::map<Key, PauliCfg> pauli;
  std::string path;

  void load(const char* file) {
    if (!file || !*file) return;
    path = file;
    std::FILE* f = std::fopen(file, "r");
    if (!f) return;  // created on the first store
    char kind[16];
    int k[5], tile, wg;
    double ms;
    while (std::fscanf(f, "%15s %d %d %d %d %d %d %d %lf", kind, &k[0], &k[1], &k[2], &k[3], &k[4], &tile, &wg,
                       &ms) == 9) {
      if (std::strcmp(kind, "pauli") == 0 && tile >= 0 && tile < q2c::kPauliTiles && wg >= 1 && wg <= k[4])
        pauli[Key{k[0], k[1], k[2], k[3], k[4]}] = PauliCfg{tile, wg, ms};
    }
    std::fclose(f);
  }
  const PauliCfg* find(const Key& k) const {
    auto it = pauli.find(k);
    return it == pauli.end() ? nullptr : &it->second;
  }
  void store(const Key& k, const PauliCfg& c) {
    pauli[k] = c;
    if (path.empty()) return;
    if (std::FILE* f = std::fopen(path.c_str(), "a")) {
      std::fprintf(f, "pauli %d %d %d %d %d %d %d %.6f\n", k[0], k[1], k[2], k[3], k[4], c.tile, c.n_wg, c.ms);
      std::fclose(f);
    }
  }
};

}  // namespace q2c_rt

struct q2c_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t aux = nullptr;  // second stream of the library's own (default priority), created on first use
  q2c_opts opts{};
  size_t bytes_in_use = 0;
  q2c_rt::Tuner tuner;

  void activate() const { hip_check(hipSetDevice(device), "hipSetDevice"); }
  hipStream_t aux_stream() {
    if (!aux) hip_check(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking), "hipStreamCreate");
    return aux;
  }

  void* dalloc(size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (bytes_in_use + bytes > opts.hbm_budget_bytes)
      throw OomError("context HBM budget exceeded (" + std::to_string(bytes_in_use + bytes) + " > " +
                     std::to_string(opts.hbm_budget_bytes) + " bytes)");
    void* p = nullptr;
    hip_check(hipMalloc(&p, bytes), "hipMalloc");
    bytes_in_use += bytes;
    return p;
  }
  void dfree(void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    bytes_in_use -= std::min(bytes_in_use, bytes == 0 ? size_t(16) : bytes);
  }
};

namespace q2c_rt {

// RAII device buffer charged to a context.
struct DBuf {
  q2c_ctx* ctx = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(q2c_ctx* c, size_t n) : ctx(c), p(c->dalloc(n)), bytes(n) {}
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : ctx(o.ctx), p(o.p), bytes(o.bytes) { o.p = nullptr; }
  DBuf& operator=(DBuf&& o) noexcept {
    release();
    ctx = o.ctx;
    p = o.p;
    bytes = o.bytes;
    o.p = nullptr;
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p && ctx) ctx->dfree(p, bytes);
    p = nullptr;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

inline long bond_cap(int N, int b, int D) {
  // capacity of bond b (between sites b and b+1), b in -1..N-1
  if (b < 0 || b >= N - 1) return 1;
  long left = (b + 1 >= 40) ? (1L << 40) : (1L << (b + 1));
  long right = (N - b - 1 >= 40) ? (1L << 40) : (1L << (N - b - 1));
  return std::min<long>(std::min(left, right), D);
}

// Owns the device arrays of a batch of MPS slots.
struct Batch {
  q2c::DevBatch d;
  int cm = 1;  // largest bond cap
  std::vector<DBuf> bufs;

  Batch(q2c_ctx* ctx, int N, int D, int slots, int precision) {
    auto& b = d;
    b.mixed = precision == Q2C_MIXED ? 1 : 0;
    b.n_qubits = N;
    b.max_bond = D;
    b.n_slots = slots;
    for (int i = 0; i <= N; ++i) b.cap[i] = int(bond_cap(N, i - 1, D));
    cm = 1;
    for (int i = 0; i <= N; ++i) cm = std::max(cm, b.cap[i]);
    b.ws = 2 * cm;
    long off = 0;
    for (int n = 0; n < N; ++n) {
      b.site_off[n] = off;
      off += long(b.cap[n]) * 2 * b.cap[n + 1];
    }
    b.site_off[N] = off;
    b.site_stride = (off + 31) & ~31L;
    off = 0;
    for (int bb = 0; bb < N - 1; ++bb) {
      b.lam_off[bb] = off;
      off += b.cap[bb + 1];
    }
    b.lam_off[N - 1] = off;
    b.lam_stride = std::max<long>(32, (off + 31) & ~31L);
    off = 0;
    for (int k = 0; k <= N; ++k) {
      b.env_off[k] = off;
      off += long(b.cap[k]) * b.cap[k];
    }
    b.env_off[N + 1] = off;
    b.env_stride = (off + 31) & ~31L;
    b.ws_stride = long(b.ws) * b.ws;
    auto alloc = [&](size_t bytes) -> void* {
      bufs.emplace_back(ctx, bytes);
      return bufs.back().p;
    };
    const size_t S = size_t(slots);
    b.sites = static_cast<double2*>(alloc(S * b.site_stride * sizeof(double2)));
    b.lam = static_cast<double*>(alloc(S * b.lam_stride * sizeof(double)));
    b.chi = static_cast<int*>(alloc(S * (N + 1) * sizeof(int)));
    b.wsM = static_cast<double2*>(alloc(S * b.ws_stride * sizeof(double2)));
    b.wsA = static_cast<double2*>(alloc(S * b.ws_stride * sizeof(double2)));
    b.wsH = static_cast<double2*>(alloc(S * b.ws_stride * sizeof(double2)));
    b.wsW = static_cast<double2*>(alloc(S * b.ws_stride * sizeof(double2)));
    b.wsV = static_cast<double2*>(alloc(S * 4 * b.ws_stride * sizeof(double2)));
    b.wsS = static_cast<double*>(alloc(S * 2 * b.ws * sizeof(double)));
    b.wsP = static_cast<int*>(alloc(S * b.ws * sizeof(int)));
    b.envL = static_cast<double2*>(alloc(S * b.env_stride * sizeof(double2)));
    b.envR = static_cast<double2*>(alloc(S * b.env_stride * sizeof(double2)));
    b.stats = static_cast<double*>(alloc(S * q2c::kNStats * sizeof(double)));
    b.flags = static_cast<int*>(alloc(S * sizeof(int)));
    b.phi = nullptr;
  }
};

// Slot states without workspaces (snapshots of a batch's slots): the site
// tensors, Schmidt values, bond dimensions, statistics and flags of `slots`
// slots in the layout of the batch `shape`.
struct SlotStore {
  q2c::DevBatch d;
  std::vector<DBuf> bufs;
  SlotStore(q2c_ctx* ctx, const q2c::DevBatch& shape, int slots) {
    const int N = shape.n_qubits;
    q2c::DevBatch b{};
    b.n_qubits = N;
    b.max_bond = shape.max_bond;
    b.n_slots = slots;
    b.ws = shape.ws;
    b.mixed = shape.mixed;
    for (int i = 0; i <= q2c::kMaxQubits; ++i) {
      b.cap[i] = shape.cap[i];
      b.site_off[i] = shape.site_off[i];
      b.lam_off[i] = shape.lam_off[i];
    }
    b.site_stride = shape.site_stride;
    b.lam_stride = shape.lam_stride;
    auto alloc = [&](size_t bytes) -> void* {
      bufs.emplace_back(ctx, bytes);
      return bufs.back().p;
    };
    const size_t S = size_t(slots);
    b.sites = static_cast<double2*>(alloc(S * b.site_stride * sizeof(double2)));
    b.lam = static_cast<double*>(alloc(S * b.lam_stride * sizeof(double)));
    b.chi = static_cast<int*>(alloc(S * (N + 1) * sizeof(int)));
    b.stats = static_cast<double*>(alloc(S * q2c::kNStats * sizeof(double)));
    b.flags = static_cast<int*>(alloc(S * sizeof(int)));
    d = b;
  }
};

inline q2c::SvdParams svd_params(const q2c_ctx* ctx) {
  q2c::SvdParams sp;
  sp.max_sweeps = ctx->opts.max_sweeps;
  sp.tol = ctx->opts.svd_tol;
  sp.cutoff_rel = ctx->opts.sv_cutoff_rel;
  sp.algo = ctx->opts.svd_algorithm;
  return sp;
}

// HIP-event times and launch counts of the device phases of a call.
struct PhaseTimes {
  double gate_ms = 0, env_ms = 0, pauli_ms = 0, reduce_ms = 0, graph_ms = 0, tune_ms = 0;
  int gate_launches = 0, circuits = 0, graph_launches = 0;
  PauliCfg pauli;
};

struct Events {
  hipEvent_t e[5] = {};
  Events() {
    for (auto& x : e) hip_check(hipEventCreate(&x), "hipEventCreate");
  }
  ~Events() {
    for (auto& x : e) (void)hipEventDestroy(x);
  }
  double ms(int a, int b) const {
    float t = 0.f;
    hip_check(hipEventElapsedTime(&t, e[a], e[b]), "hipEventElapsedTime");
    return double(t);
  }
};

inline void fill_stats(q2c_stats* out, const std::vector<double>& st, int slots, double seconds,
                const PhaseTimes& pt = PhaseTimes()) {
  if (!out) return;
  q2c_stats s{};
  for (int i = 0; i < slots; ++i) {
    const double* p = &st[size_t(i) * q2c::kNStats];
    s.discarded_weight_sum = std::max(s.discarded_weight_sum, p[q2c::kStatDisc]);
    s.max_discarded = std::max(s.max_discarded, p[q2c::kStatMaxDisc]);
    s.max_chi = std::max(s.max_chi, int(p[q2c::kStatMaxChi]));
    s.max_sweeps_used = std::max(s.max_sweeps_used, int(p[q2c::kStatSweeps]));
    s.max_abs_imag = std::max(s.max_abs_imag, p[q2c::kStatMaxImag]);
    s.gate_flops += p[q2c::kStatFlops];
    s.jacobi_sweeps += p[q2c::kStatSweepSum];
    for (int c = 0; c < 6; ++c) s.cycles[c] += p[q2c::kStatCycContract + c];
    s.svd_bisect_gates += p[q2c::kStatBisect];
    s.svd_fallbacks += p[q2c::kStatFallbacks];
    if (i == 0) s.norm = p[q2c::kStatNorm];
  }
  s.seconds = seconds;
  s.gate_ms = pt.gate_ms;
  s.env_ms = pt.env_ms;
  s.pauli_ms = pt.pauli_ms;
  s.reduce_ms = pt.reduce_ms;
  s.gate_launches = pt.gate_launches;
  s.n_circuits = pt.circuits;
  s.graph_ms = pt.graph_ms;
  s.graph_launches = pt.graph_launches;
  s.pauli_tile = pt.pauli.tile;
  s.pauli_wg = pt.pauli.n_wg;
  s.tune_ms = pt.tune_ms;
  *out = s;
}

inline void check_flags(const std::vector<int>& flags) {
  int f = 0;
  for (int v : flags) f |= v;
  if (f & q2c::kFlagNumeric) throw StatusError(Q2C_ERR_NUMERIC, "non-finite or zero Schmidt values on the device");
  if (f & q2c::kFlagNoConv) throw StatusError(Q2C_ERR_NOCONV, "Jacobi SVD reached max_sweeps without converging");
}

constexpr int kGateChunk = 8192;  // gates per launch of the gate kernel

// Workgroups per slot of the Pauli sweep: about 1024 workgroups in all to
// fill the chip, but runs of at least kPauliRun sorted strings each, so that
// a workgroup reuses the shared prefixes of its run.
constexpr int kPauliRun = 32;
inline int pauli_workgroups(int n_strings, int n_slots) {
  int n_wg = std::max(1, 1024 / std::max(1, n_slots));
  n_wg = std::min(n_wg, (n_strings + kPauliRun - 1) / kPauliRun);
  return std::max(1, std::min(n_wg, n_strings));
}

}  // namespace
