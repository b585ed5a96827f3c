// Device-side data layout and kernel launchers (internal to libq2c).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace q2c {

constexpr int kBlock = 512;        // threads per workgroup for the slot kernels
constexpr int kMaxQubits = 64;

// Compiled problem resident on the device.
struct DevProblem {
  int n_qubits = 0;
  int n_gates = 0;
  int n_rot = 0;
  int n_strings = 0;
  int* gate_site = nullptr;     // [n_gates]
  int* gate_rot = nullptr;      // [n_gates], -1 for constant gates
  double2* gate_pre = nullptr;  // [n_gates][16]
  double2* gate_post = nullptr; // [n_gates][16]
  double* rot_c = nullptr;      // [n_rot]
  int* rot_param = nullptr;     // [n_rot]
  uint64_t* str_x = nullptr;    // [n_strings]
  uint64_t* str_z = nullptr;    // [n_strings]
  double* str_c = nullptr;      // [n_strings]
  int* str_order = nullptr;     // [n_strings] prefix order of the strings (sorted position -> index)
  int* str_share = nullptr;     // [n_strings] transfer steps shared with the previous sorted string
};

// A batch of MPS "slots" with a common shape (qubits, bond cap).  Every
// per-slot array is slot-major with the stride given.
struct DevBatch {
  int n_qubits = 0;
  int max_bond = 0;
  int n_slots = 0;
  int ws = 0;                 // workspace matrix dimension: 2 * largest bond cap
  int mixed = 0;              // 1: site tensors, contractions and sweeps in complex64
  int slot0 = 0;              // first slot of a launch (launches cover slots slot0 .. slot0 + n_slots - 1)
  int* cursor = nullptr;      // optional per-slot next gate: the gate kernel then runs up to
  int n_gates = 0;            //   g1 - g0 gates from cursor[slot] (capped at n_gates) and advances it
  int cap[kMaxQubits + 1];    // cap[b+1] = capacity of bond b, b = -1..N-1
  long site_off[kMaxQubits + 1];  // offsets (in double2) of site tensors; [N] = total
  long lam_off[kMaxQubits + 1];   // offsets (in doubles) of bond b at lam_off[b]; [N-1] = total
  long env_off[kMaxQubits + 2];   // offsets of environment k (cap[k]^2 each); [N+1] = total
  long site_stride = 0, lam_stride = 0, env_stride = 0, ws_stride = 0;

  double2* sites = nullptr;   // [slot][site_stride]
  double* lam = nullptr;      // [slot][lam_stride]
  int* chi = nullptr;         // [slot][N+1]: chi[b+1] = dimension of bond b
  double* phi = nullptr;      // [slot][n_rot] rotation angles
  double2* wsM = nullptr;     // [slot][ws*ws] two-site tensor M
  double2* wsA = nullptr;     // [slot][ws*ws] M' -> Jacobi rows
  double2* wsH = nullptr;     // [slot][ws*ws] LQ reflectors
  double2* wsW = nullptr;     // [slot][ws*ws] sorted normalised rows (W^H)
  double2* wsV = nullptr;     // [slot][4*ws*ws] vector scratch of the bisection SVD
  double* wsS = nullptr;      // [slot][2*ws] row norms
  int* wsP = nullptr;         // [slot][ws] sort permutation
  double2* envL = nullptr;    // [slot][env_stride]
  double2* envR = nullptr;    // [slot][env_stride] (transposed right environments)
  double* stats = nullptr;    // [slot][8]: 0 disc sum, 1 max disc, 2 max chi, 3 max sweeps, 4 norm
  int* flags = nullptr;       // [slot]: bit0 NOCONV, bit1 NUMERIC
};

enum {
  kStatDisc = 0,
  kStatMaxDisc = 1,
  kStatMaxChi = 2,
  kStatSweeps = 3,
  kStatNorm = 4,
  kStatMaxImag = 5,
  kStatFlops = 6,
  kStatSweepSum = 7,
  // device cycle counters per phase of the gate update (thread 0, summed)
  kStatCycContract = 8,
  kStatCycLQ = 9,
  kStatCycQR = 10,
  kStatCycJacobi = 11,
  kStatCycBack = 12,
  kStatCycUpdate = 13,
  kStatFallbacks = 14,  // bisection SVDs that fell back to Jacobi
  kStatBisect = 15,     // gates whose SVD used bisection
  kNStats = 16
};
enum { kFlagNoConv = 1, kFlagNumeric = 2 };

struct SvdParams {
  int max_sweeps;
  double tol;
  double cutoff_rel;
  int algo;  // 0: bidiagonal bisection with Jacobi fallback; 1: Jacobi only
};

// Launchers (stream-ordered, asynchronous).
hipError_t launch_init_product(const DevBatch& b, const uint8_t* d_occ, hipStream_t st);
// phi[slot][m] = -2 c_m theta[slot][param_m] + (m == shift_rot[slot] ? shift_val[slot] : 0)
// Copies slot states src -> dst (same shape): pairs[i] = (src slot, dst
// slot), or the single pair `one` when d_pairs is null.
hipError_t launch_copy_slots(const DevBatch& src, const DevBatch& dst, const int2* d_pairs, int n_pairs, int2 one,
                             bool clear_work, hipStream_t st);
// phi_m = -2 c_m theta[param(m)] per slot; optional per-slot shift: target
// t >= 0 adds the shift to phi_t, t = -2 - k adds it to theta_k (all rotations
// of parameter k), t = -1 none.
hipError_t launch_angles(const DevBatch& b, const DevProblem& p, const double* d_theta, int n_theta,
                         const int* d_shift_rot, const double* d_shift_val, hipStream_t st);
hipError_t launch_gates(const DevBatch& b, const int* d_site, const int* d_rot, const double2* d_pre,
                        const double2* d_post, int g0, int g1, int n_rot, SvdParams sp, hipStream_t st);
hipError_t launch_envs(const DevBatch& b, hipStream_t st);
// d_order / d_share: prefix order (nullable: input order, no reuse).  Each
// workgroup takes a contiguous run of ceil(n_strings / n_wg) sorted strings.
// d_scratch: n_slots * n_wg * pauli_scratch_mats(N) * cm * cm double2,
// cm = largest bond cap.
// tile: 0 .. kPauliTiles-1, the GEMM tile of the transfers (64x64x8,
// 64x64x16, 32x32x16); every tile gives the same results bit for bit.
constexpr int kPauliTiles = 3;
hipError_t launch_pauli(const DevBatch& b, const uint64_t* d_x, const uint64_t* d_z, int n_strings,
                        const int* d_order, const int* d_share, double2* d_scratch, int n_wg, int cm,
                        double* d_ev_re, double* d_ev_im, int tile, hipStream_t st);
inline int pauli_scratch_mats(int n_qubits) { return n_qubits + 2; }
hipError_t launch_energy_reduce(const DevBatch& b, const double* d_coeff, const double* d_ev_re,
                                const double* d_ev_im, int n_strings, double c_identity,
                                double* d_energy, hipStream_t st);

}  // namespace q2c
