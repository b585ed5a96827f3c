/*
 * q2c.h -- C ABI of the MI355X MPS-VQE energy library (libq2c.so).
 *
 * The library evaluates the UCCSD energy E(theta) = <psi(theta)|H|psi(theta)>
 * of a Jordan-Wigner Pauli-string Hamiltonian on a matrix product state, the
 * hot path of the MPS-VQE simulator in "Large-Scale Simulation of Quantum
 * Computational Chemistry on a New Sunway Supercomputer" (Sec. II-A, III-A,
 * III-D).  Everything that scales with the state runs in HIP kernels on one
 * gfx950 GPU; the host only validates arguments, compiles the problem once
 * and launches.
 *
 * Conventions shared by every call
 * --------------------------------
 * Qubits / sites / spin-orbitals: qubit n = MPS site n = spin-orbital n,
 *   interleaved spins (2p = p-alpha, 2p+1 = p-beta).  |1> = occupied.
 * Two-qubit gates act on (site, site+1); the 4x4 matrix is row-major with
 *   basis index 2*i_site + i_{site+1}, complex values stored as interleaved
 *   (re, im) doubles: 32 doubles per gate.
 * Pauli strings: bit b of word w of a mask refers to qubit 64*w + b.
 *   A qubit carries X if only its x bit is set, Z if only its z bit is set,
 *   Y if both are set.  n_words = ceil(n_qubits / 64).
 * Ownership: every pointer argument is a HOST pointer owned by the caller and
 *   only read (or, for outputs, written) during the call; the library copies
 *   what it keeps.  Device memory belongs to the library.  Handles are opaque
 *   and freed by the matching *_destroy.
 * Synchronisation: a call returns after its device work has finished and its
 *   host outputs are valid.  Calls on one context must not overlap (one host
 *   thread per context at a time); different contexts are independent.
 * Errors: every entry point returns Q2C_OK (0) or a negative Q2C_ERR_* code.
 *   On error no output is written and q2c_last_error() returns a message
 *   (thread-local, valid until the next call on that thread).  No C++
 *   exception crosses this boundary.
 * Environment: Q2C_PROGRESS=1 prints a progress line to stderr after each
 *   launch of gate runs longer than one launch (8,192 gates) and after each
 *   batch graph that ran for at least a second.
 */
#ifndef Q2C_H
#define Q2C_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  Q2C_OK = 0,
  Q2C_ERR_ARG = -1,     /* bad size, index, NULL, NaN/Inf input, theta length mismatch */
  Q2C_ERR_OOM = -2,     /* device allocation or the context's HBM budget failed          */
  Q2C_ERR_DEVICE = -3,  /* a HIP call failed, or no usable gfx950 device                   */
  Q2C_ERR_NOCONV = -4,  /* Jacobi SVD reached max_sweeps without converging               */
  Q2C_ERR_NUMERIC = -5, /* non-finite values appeared on the device                         */
  Q2C_ERR_BUSY = -6     /* the handle is in use by an unfinished operation                  */
};

/* Precision of an MPS or an energy evaluation.
 *   Q2C_FP64   complex128 throughout.
 *   Q2C_MIXED  site tensors, the two-site contraction, the update B_n = M W and
 *              the transfer sweeps in complex64 with FP32 accumulation; the SVD,
 *              the renormalisation, the Schmidt values and the energy sum in FP64
 *              (Sec. IV-B splits the time between the SVD and the contractions). */
enum { Q2C_FP64 = 0, Q2C_MIXED = 1 };

typedef struct q2c_ctx q2c_ctx;
typedef struct mps_state mps_state;
typedef struct vqe_problem vqe_problem;

/* Options of a context.  Zero-initialised fields take the defaults noted. */
typedef struct {
  int max_sweeps;           /* Jacobi sweep limit per SVD (0 -> 60)                      */
  double sv_cutoff_rel;     /* keep s_k > sv_cutoff_rel * s_1 (0 -> 1e-12)               */
  double svd_tol;           /* rotate a row pair while |<r_p,r_q>| > svd_tol*|r_p||r_q|
                               (0 -> 1e-15)                                               */
  int slots;                /* max circuits resident at once in batched calls (0 -> 256)  */
  size_t hbm_budget_bytes;  /* device memory the context may hold (0 -> 64 GiB)           */
  int svd_algorithm;        /* 0: Golub-Kahan bidiagonalisation, bisection for the kept
                               singular values, twisted-factorisation vectors (D <= 64;
                               falls back to 1 when the vectors cannot be certified);
                               1: LQ+QR-preconditioned one-sided Jacobi                    */
  int shift_from_start;     /* parameter-shift circuits: 0 -> each shifted circuit starts
                               from a copy of the unshifted circuit's state at its first
                               angle-dependent gate (same energies, about half the gates);
                               1 -> every circuit runs from the first gate                 */
  int eager_batches;        /* batched calls (energy batches, parameter shifts): 0 -> each
                               batch shape is captured once as a HIP graph (inputs, every
                               kernel, outputs) and replayed; 1 -> launched one by one     */
  int no_autotune;          /* 0 -> the Pauli sweep's GEMM tile and workgroups per circuit
                               are chosen by timing the candidates on the first batch of
                               each shape (results do not depend on the choice);
                               1 -> fixed defaults                                         */
  const char* autotune_cache; /* nullable: text file of tuned choices, read at context
                               creation and appended to; the string is copied            */
  int grad_rule;            /* vqe_grad_paramshift: 0 -> two-term shift of every rotation
                               angle (2 circuits per rotation); 1 -> four-term shift of
                               every UCCSD parameter (4 circuits per parameter; exact
                               because the rotations of one excitation commute and their
                               generator has eigenvalues 0, +-1)                          */
} q2c_opts;

/* Statistics of the last state evolution (all over the gates applied). */
typedef struct {
  double discarded_weight_sum; /* sum over gates of sum_{k>chi'} s_k^2 / sum_k s_k^2     */
  double max_discarded;        /* largest single-gate discarded weight                    */
  double max_abs_imag;         /* max |Im <P>| over the strings evaluated                 */
  double norm;                 /* <psi|psi> of the stored MPS before division            */
  int max_chi;                 /* largest bond dimension reached                          */
  int max_sweeps_used;         /* most Jacobi sweeps any SVD needed                       */
  double seconds;              /* wall time of the call                                   */
  /* Device-side accounting, summed over every circuit of the call:                         */
  double gate_flops;           /* algorithmic FLOPs of the gate updates at the realised
                                  bond dimensions: per gate 32 cl cm cr + 128 cl cr
                                  (contraction), 4 (4 m n^2 + 8 n^3) with m >= n the sides
                                  of the 2cl x 2cr matrix (SVD, singular values and right
                                  vectors), 8 (2cl)(2cr) chi' (update)                     */
  double jacobi_sweeps;        /* Jacobi sweeps executed                                  */
  double gate_ms;              /* HIP-event time of the gate-kernel launches              */
  double env_ms;               /* HIP-event time of the environment kernel                */
  double pauli_ms;             /* HIP-event time of the Pauli-sweep kernel                */
  double reduce_ms;            /* HIP-event time of the energy reduction                  */
  int gate_launches;           /* gate-kernel launches                                    */
  int n_circuits;              /* circuits (MPS evolutions) run                           */
  /* Shader-clock cycles spent by the gate kernel in each phase of the update,
   * summed over gates and circuits: [0] contraction + gate + scaling,
   * [1] reduction (bidiagonalisation, or LQ + QR), [2] singular values
   * (bisection, or Jacobi sweeps), [3] vectors (twisted factorisations +
   * CholQR2, or row back-transformation), [4] back-transformation of the
   * kept vectors (or sorting), [5] truncation + update.                      */
  double cycles[6];
  double svd_bisect_gates;     /* gate SVDs done by bisection                               */
  double svd_fallbacks;        /* bisection SVDs that fell back to Jacobi                   */
  double graph_ms;             /* HIP-event time of replayed batch graphs (whole batches:
                                  gates, environments, sweeps, reduction, copies)         */
  int graph_launches;          /* batch graphs replayed                                    */
  int pauli_tile;              /* Pauli-sweep tile of the last batch (0: 64x64x8,
                                  1: 64x64x16, 2: 32x32x16)                               */
  int pauli_wg;                /* Pauli-sweep workgroups per circuit of the last batch     */
  double tune_ms;              /* wall time spent autotuning during the call (first use of
                                  a batch shape; candidates are timed only when one sweep
                                  takes at most 50 ms)                                     */
} q2c_stats;

/* Context: one device, one HIP stream.
 *   device      HIP device ordinal.
 *   hip_stream  hipStream_t to launch on, or NULL for a stream the context
 *               creates (default priority).  A caller-provided stream stays
 *               owned by the caller.
 *   opts        may be NULL for defaults.
 * Returns Q2C_ERR_DEVICE if the device is absent or is not gfx950. */
int q2c_ctx_create(int device, void* hip_stream, const q2c_opts* opts, q2c_ctx** out);
int q2c_ctx_destroy(q2c_ctx* ctx);
/* Device memory the library holds for ctx (problems, MPS, batches, server
 * classes, scratch) and the budget it may not exceed (q2c_opts
 * hbm_budget_bytes); either pointer may be NULL. */
int q2c_ctx_memory(const q2c_ctx* ctx, size_t* bytes_in_use, size_t* budget_bytes);

/* Matrix product state in a product state (Eq. 6 with every bond of
 * dimension 1, e.g. the Hartree-Fock reference of Sec. III-D prepared by X
 * gates).  Bond n (between sites n and n+1) may grow to
 * min(2^(n+1), 2^(N-n-1), max_bond).
 *   n_qubits  2..64.
 *   max_bond  1..256 (D).
 *   precision Q2C_FP64 or Q2C_MIXED (see the enum above).
 *   occ       n_qubits bytes, 0 or 1 (site n starts in |occ[n]>). */
int mps_create(q2c_ctx* ctx, int n_qubits, int max_bond, int precision,
               const uint8_t* occ, mps_state** out);
int mps_destroy(mps_state* s);

/* Apply one two-qubit gate to sites (site, site+1) and restore the MPS form
 * (Sec. III-A, Eq. 7-10): contract the gate with the two site tensors, scale
 * by the left bond's Schmidt values, take the SVD in FP64, keep the
 * min(D, #{s_k > cutoff * s_1}) largest Schmidt values (renormalised), set
 * site+1 to the kept right singular vectors and site to M W / ||S_kept||.
 *   site   0..n_qubits-2.
 *   gate   32 doubles (4x4 complex, row-major, interleaved re/im); need not
 *          be unitary, but must be finite.
 *   discarded_weight  nullable; receives sum_{k>chi'} s_k^2 / sum_k s_k^2. */
int mps_apply_gate(mps_state* s, int site, const double* gate, double* discarded_weight);

/* Copy the state of src into dst on the device (site tensors, Schmidt
 * values, bond dimensions, statistics).  Both must belong to one context and
 * have the same qubits, max_bond and precision. */
int mps_copy(mps_state* src, mps_state* dst);

/* Expectation values <psi|P|psi> / <psi|psi> of Hermitian Pauli strings by
 * exact transfer-matrix contraction of the stored MPS (Eq. 2, Eq. 11).
 *   x_masks, z_masks  n_strings * n_words uint64 each, string-major.
 *   out_re            n_strings doubles.
 *   out_im            nullable; n_strings doubles (zero up to rounding). */
int mps_expect_pauli_batch(mps_state* s, int n_strings, int n_words,
                           const uint64_t* x_masks, const uint64_t* z_masks,
                           double* out_re, double* out_im);

/* Host only (no device call): the order in which the transfer sweeps visit
 * Pauli strings so that strings with a common leading part share its
 * transfer steps (Sec. III-B, prefix sharing of the strings of Eq. 2).
 * Strings are sorted by lowest non-identity qubit, then by their letters
 * qubit by qubit upward, the identity first.
 *   x_masks, z_masks  n_strings uint64 each (n_qubits <= 64).
 *   order  out, n_strings: sorted position -> input index.
 *   share  out, n_strings: transfer steps sorted string t has in common with
 *          sorted string t-1 (0 for t = 0 or a different lowest qubit).
 *   steps  nullable out, 2 int64: transfer steps without and with sharing
 *          along the whole order (the second = nodes of the prefix trie). */
int q2c_pauli_prefix_order(int n_strings, const uint64_t* x_masks, const uint64_t* z_masks,
                           int* order, int* share, int64_t* steps);

/* Copy the site tensors and Schmidt values to the host (debugging, checks).
 *   chi_out   n_qubits+1 ints: chi_out[0] = 1, chi_out[n+1] = right bond of
 *             site n, chi_out[N] = 1.
 *   tensors   nullable; receives site after site, each chi_l x 2 x chi_r
 *             complex (interleaved doubles) row-major; size from chi_out.
 *   lambdas   nullable; receives bond after bond (n_qubits-1 bonds). */
int mps_export(mps_state* s, int* chi_out, double* tensors, double* lambdas);
int mps_get_stats(mps_state* s, q2c_stats* stats);

/* Problem: integrals (Eq. 1) -> Jordan-Wigner Pauli strings (Eq. 2) and the
 * UCCSD ansatz (Eq. 3-4) as a first-order Trotter product of Pauli
 * rotations, compiled to nearest-neighbour two-qubit gates with the
 * single-qubit gates fused in (Sec. III-A, III-D).
 *   ctx     may be NULL: the problem is then compiled on the host only and
 *           can be inspected with vqe_problem_info / _paulis / _gates, but
 *           not evaluated.
 *   n_orb   1..32 spatial orbitals (2*n_orb qubits).
 *   n_elec  even, 0..2*n_orb; Hartree-Fock occupies spin-orbitals 0..n_elec-1.
 *   h1      n_orb^2 doubles, symmetric.
 *   eri     n_orb^4 doubles, chemist notation (pq|rs), row-major [p][q][r][s].
 *   e_const constant added to the energy. */
int vqe_problem_create(q2c_ctx* ctx, int n_orb, int n_elec, const double* h1,
                       const double* eri, double e_const, vqe_problem** out);
int vqe_problem_destroy(vqe_problem* p);

/* Sizes of a compiled problem (any pointer may be NULL). */
int vqe_problem_info(const vqe_problem* p, int* n_qubits, int* n_params, int* n_strings,
                     int* n_rotations, int* n_gates, double* identity_coeff);
/* Spatial orbitals and electrons the problem was created with (any pointer
 * may be NULL); the Hartree-Fock state occupies qubits 0 .. n_elec-1. */
int vqe_problem_electrons(const vqe_problem* p, int* n_orb, int* n_elec);
/* Pauli strings in the order they are summed (ascending (x, z)), excluding
 * the identity; x, z: n_strings * n_words each; coeff: n_strings. */
int vqe_problem_paulis(const vqe_problem* p, uint64_t* x, uint64_t* z, double* coeff);
/* Rotations: x, z masks, coefficient c (phi = -2 c theta[param]), param. */
int vqe_problem_rotations(const vqe_problem* p, uint64_t* x, uint64_t* z, double* c,
                          int* param);
/* Gates in application order: site, rotation index (-1 if constant), and
 * pre/post 4x4 complex (32 doubles each).  A constant gate is `pre` (post is
 * the identity); an angle gate is post * kron(I, RZ(phi)) * pre. */
int vqe_problem_gates(const vqe_problem* p, int* site, int* rot, double* pre, double* post);

/* E(theta) = E_const + c_I + sum_P c_P <P>, from the Hartree-Fock product
 * state through every compiled gate at bond dimension max_bond, then the
 * Pauli sum (FP64, compensated, fixed order).
 *   theta  n_theta doubles; n_theta must equal the problem's n_params.
 *   stats  nullable. */
int vqe_energy(vqe_problem* p, const double* theta, int n_theta, int max_bond, int precision,
               double* energy, q2c_stats* stats);

/* Energies of n_batch independent parameter vectors (theta is n_batch x
 * n_theta, row-major), run as concurrent circuits on the device.
 *   energies  n_batch doubles. */
int vqe_energy_batch(vqe_problem* p, const double* theta, int n_batch, int n_theta,
                     int max_bond, int precision, double* energies, q2c_stats* stats);

/* Gradient by parameter shifts.  q2c_opts.grad_rule = 0: the two-term shift
 * of every rotation angle,
 * dE/dtheta_k = sum_{m in k} (-2 c_m) (E(phi_m + pi/2) - E(phi_m - pi/2)) / 2;
 * grad_rule = 1: the four-term shift of every parameter,
 * dE/dtheta_k = D(pi/4) + (1 - sqrt 2) / 2 D(pi/2), D(s) = E(theta_k + s) -
 * E(theta_k - s).  Both are exact for the compiled circuit at full bond
 * dimension.
 * All shifted circuits and the unshifted one run as batches of concurrent
 * circuits; by default (q2c_opts.shift_from_start = 0) each shifted circuit
 * starts from the unshifted circuit's state at its first gate that depends
 * on a shifted angle, which leaves every energy unchanged.
 * stats->gate_flops then counts every gate that ran once.
 *   grad    n_theta doubles.
 *   energy  nullable; E(theta). */
int vqe_grad_paramshift(vqe_problem* p, const double* theta, int n_theta, int max_bond,
                        int precision, double* grad, double* energy, q2c_stats* stats);

/* Shifted-circuit energies for a chosen subset of rotations (for sampling
 * and tests): for each listed rotation m, e_plus[i] = E(phi_m + pi/2) and
 * e_minus[i] = E(phi_m - pi/2). */
int vqe_shift_energies(vqe_problem* p, const double* theta, int n_theta, const int* rot_idx,
                       int n_rot, int max_bond, int precision, double* e_plus, double* e_minus,
                       q2c_stats* stats);

/* The paper's own measurement, kept as the baseline the transfer sweeps
 * replace (Sec. III-A after Eq. 11; the per-string circuits of Sec. III-D):
 * for every Pauli string a Hadamard test on an ancillary qubit after the
 * last qubit (site n_qubits of an (n_qubits + 1)-site MPS at max_bond, on
 * ctx): Hartree-Fock state, ansatz gates, ancilla in |+>, the string applied
 * under the ancilla's control as the ancilla moves down to the string's
 * first qubit lo (n_qubits - lo gates, each a controlled letter and a swap),
 * <X> of the ancilla = Re <psi|P|psi>.  Exact when max_bond holds the
 * (n_qubits + 1)-site state (twice the ansatz state's bonds suffice).
 *   p             any problem, also one created without a context (only its
 *                 compiled strings, rotations and gates are read).
 *   shared_state  0: every string's circuit runs the ansatz again (the
 *                 paper's scheme); 1: the ansatz state is prepared once and
 *                 copied on the device per string.  Same values bit for bit.
 *   string_idx    nullable: the strings to measure (n_idx of them); NULL
 *                 measures all and also writes energy (identity coefficient
 *                 included, compensated sum in string order).
 *   expect        nullable: one value per measured string.
 *   seconds       nullable: wall time. */
int vqe_energy_hadamard(q2c_ctx* ctx, vqe_problem* p, const double* theta, int n_theta, int max_bond,
                        int precision, int shared_state, const int* string_idx, int n_idx, double* energy,
                        double* expect, double* seconds);

/* ---------------------------------------------------------------- VQE loop
 * The variational outer loop (Sec. II-A: the energy of the ansatz state is
 * handed to a classical optimizer that updates theta; the paper names none):
 * L-BFGS (Nocedal & Wright, Alg. 7.4/7.5) with Armijo backtracking.  Every
 * gradient is vqe_grad_paramshift (rule from q2c_opts.grad_rule) and the
 * trial step lengths of one backtracking round are one vqe_energy_batch, so
 * all circuits run on the device; the host only forms the search direction
 * from n_theta-long vectors.  Zero fields take the defaults in brackets. */
typedef struct {
  int max_iter;     /* accepted steps at most                                   [100]  */
  int history;      /* curvature pairs kept                                     [8]    */
  int n_trial;      /* step lengths 1, 1/2, 1/4, ... per backtracking batch (<= 64) [4] */
  double gtol;      /* converged when max_k |dE/dtheta_k| <= gtol                [1e-6] */
  double ftol;      /* stop when a step lowers E by <= ftol max(1, |E|)         [1e-13] */
  double max_step;  /* largest component of a steepest-descent step (radians)   [0.1]  */
  int no_speculation; /* 0: step length 1 is tried through the gradient call at the
                       trial point (its unshifted circuit gives E there; accepted
                       steps then cost one call, rejected ones continue with
                       1/2, 1/4, ... in batches); 1: step length 1 is the first
                       entry of the first batch.  The same steps either way.    */
} q2c_min_opts;

typedef struct {
  int iterations;   /* accepted steps                                                   */
  int grad_evals;   /* gradient calls (iterations + 1, plus rejected trials of step
                       length 1 when speculating)                                        */
  int energy_evals; /* line-search circuits                                             */
  int status;       /* 1: gtol met; 2: ftol met; 0: max_iter reached; 3: no step of
                       length >= 2^-(6 n_trial) (2^-(6 n_trial + 1) when speculating)
                       lowered E (the energy's resolution)                              */
  double grad_max;  /* max_k |dE/dtheta_k| at theta_out                                  */
  double seconds;   /* wall time                                                        */
} q2c_min_report;

/* Minimise E(theta) from theta0 at bond dimension max_bond.
 *   theta0        n_theta starting parameters (n_theta = the problem's n_params).
 *   opts          nullable (all defaults).
 *   theta_out     n_theta doubles: the last accepted point (may equal theta0).
 *   energy        nullable; E(theta_out).
 *   energy_trace  nullable; room for max_iter + 1 doubles: E(theta0), then E
 *                 after each accepted step (report->iterations + 1 written).
 *   report        nullable.
 * Non-convergence (status 0 or 3) is not an error.  Errors of the inner
 * evaluations are returned unchanged, with nothing written. */
int vqe_minimize(vqe_problem* p, const double* theta0, int n_theta, int max_bond, int precision,
                 const q2c_min_opts* opts, double* theta_out, double* energy, double* energy_trace,
                 q2c_min_report* report);

/* ---------------------------------------------------------------- DMET loop
 * The DMET procedure around the fragment solver (Sec. III-B): a low-level
 * (restricted mean-field, U = 0) calculation of the whole lattice; for each
 * fragment, bath orbitals from the Schmidt decomposition of that determinant
 * and the Hamiltonian projected onto fragment + bath (2k orbitals, 2k
 * electrons); the fragment problem minimised by vqe_minimize from theta = 0;
 * the fragment's electron count from its one-particle density matrix at the
 * minimum; the global chemical potential mu (entering as -mu times the
 * fragment electron count) moved by regula falsi (Illinois) until the
 * fragments' electrons add up to n_elec.  Fragment energy: the fragment's
 * share of the one-body energy, 1/2 (P_F h + h P_F), plus its on-site
 * interaction; the DMET energy is their sum.  Embedding orbitals: mean-field
 * natural orbitals in fragment + bath, occupied first, each block
 * diagonalising h, signs fixed by the largest site coefficient; U acts on
 * the fragment sites only (non-interacting bath).  All circuits run on the
 * device; the host does the n_sites-sized linear algebra.  Fragments are
 * independent and are solved concurrently on worker contexts created on
 * ctx's device with ctx's options. */
typedef struct {
  int n_sites;      /* L, 2 .. 64                                                */
  int frag_size;    /* k, 1 .. 4, dividing L: fragments of k consecutive sites   */
  int n_elec;       /* even, 2 .. 2L - 2                                         */
  const double* h;  /* L x L row-major one-body matrix (symmetric, finite)       */
  double U;         /* on-site repulsion U n_up n_down on every site             */
} q2c_lattice;

typedef struct {
  double mu_lo, mu_hi; /* bracket with sum N_frag - n_elec <= 0 at mu_lo and >= 0
                          at mu_hi; both 0 -> [-2, 2]                           */
  double n_tol;        /* stop when |sum N_frag - n_elec| <= n_tol       [1e-6] */
  int max_iter;        /* regula-falsi steps after the two bracket ends   [40]   */
  int max_bond;        /* fragment MPS bond dimension [2^(2k): exact], <= 256    */
  int precision;       /* Q2C_FP64 or Q2C_MIXED for the fragment circuits         */
  q2c_min_opts vqe;    /* fragment VQE options (zero fields: defaults)           */
  int workers;         /* fragments solved at once, each on a context (stream) of
                          its own on ctx's device; results do not depend on it
                          [min(8, fragments)]                                      */
} q2c_dmet_opts;

typedef struct {
  double mu;        /* chemical potential of the returned fragment results        */
  double e_dmet;    /* sum of the fragment energies at mu                         */
  int iterations;   /* regula-falsi steps                                          */
  int status;       /* 1: converged; 0: max_iter reached; 3: the bracket ends
                       have the same sign (results are those of mu_lo)            */
  int vqe_runs;     /* fragment minimisations                                      */
  double seconds;
} q2c_dmet_report;

/* Outputs (all nullable): n_frag, e_frag, e_emb with L/k doubles each (the
 * fragments' electrons, fragment energies and embedded ground-state energies
 * at the returned mu); mu_trace with room for max_iter + 2 doubles (every mu
 * evaluated, bracket ends first).  Errors: Q2C_ERR_ARG for bad shapes or a
 * degenerate mean field (no gap at the Fermi level, or a bath with fewer
 * than k orbitals); inner errors are returned unchanged. */
int dmet_solve(q2c_ctx* ctx, const q2c_lattice* lattice, const q2c_dmet_opts* opts, double* n_frag,
               double* e_frag, double* e_emb, double* mu_trace, q2c_dmet_report* report);

/* The embedded problem of fragment frag at chemical potential mu, as
 * dmet_solve builds it (host only, no device): orbitals (L x 2k, row-major:
 * site coefficients of the embedding orbitals), h1 ((2k)^2, including
 * -mu times the fragment count), eri ((2k)^4, chemist (pq|rs)), nop ((2k)^2,
 * one-body matrix of the fragment electron count), efrag_h1 ((2k)^2, one-body
 * part of the fragment energy).  Every output is nullable. */
int dmet_embedding(const q2c_lattice* lattice, int frag, double mu, double* orbitals, double* h1,
                   double* eri, double* nop, double* efrag_h1);

/* ---------------------------------------------------------------- serving
 * A request server for independent fragment solves (the per-fragment VQE of
 * the DMET embedding, Sec. III-B; fragments are independent, Sec. III-C).
 * Requests with the same (qubits, electrons, D, precision) form a class: one
 * slot batch on the device sharing the UCCSD gate list; every slot carries
 * its own Hamiltonian, parameters and gate cursor.  q2c_server_step()
 * retires finished slots, admits queued requests into free slots (creating a
 * class when the context's HBM budget allows; idle classes stay allocated for
 * later requests of their shape and are evicted, least recently used first,
 * only when a new class does not fit) and launches the next gate
 * chunk of every class on that class's own stream, so classes overlap on the
 * device and requests join while others run (continuous batching).  Each
 * result depends only on its own request: served alone or in any mix it is
 * bit-for-bit the same as vqe_energy() of the same problem.  Not thread-safe;
 * one thread drives a server. */
typedef struct q2c_server q2c_server;

typedef struct {
  int slots_per_class;  /* slots of each class; default 64                      */
  int gates_per_step;   /* gates a slot advances per launch; default 1024       */
} q2c_server_opts;

typedef struct {
  uint64_t tag;         /* the caller's tag from q2c_server_submit              */
  int status;           /* Q2C_OK, or the error code that ended the request     */
  int n_qubits, max_bond, precision;
  double energy;        /* <psi|H|psi> / <psi|psi> (Eq. 2)                       */
  double n_frag;        /* sum of <n_p> over the first 2 n_frag_orb spin-orbitals */
  double submit_s, admit_s, done_s;  /* seconds since the server was created */
  double discarded_weight_sum;
  int max_chi;
} q2c_result;

/* opts nullable (defaults).  The server uses the context's device, budget and
 * SVD options; it creates one stream per class. */
int q2c_server_create(q2c_ctx* ctx, const q2c_server_opts* opts, q2c_server** out);
int q2c_server_destroy(q2c_server* srv);

/* Queue one energy evaluation.  Integrals as for vqe_problem_create (the
 * problem is compiled here, which counts toward the request's latency);
 * theta as for vqe_energy; n_frag_orb in 0..n_orb selects the spatial
 * orbitals whose occupation is returned in n_frag.  Copies every input. */
int q2c_server_submit(q2c_server* srv, uint64_t tag, int n_orb, int n_elec, const double* h1,
                      const double* eri, double e_const, const double* theta, int n_theta,
                      int max_bond, int precision, int n_frag_orb);

/* One scheduling round (does not wait for running launches).  Outputs
 * nullable: requests still queued, requests on the device, results ready. */
int q2c_server_step(q2c_server* srv, int* n_queued, int* n_active, int* n_ready);

/* Move up to max_out finished results into out (completion order). */
int q2c_server_poll(q2c_server* srv, q2c_result* out, int max_out, int* n_out);

/* Thread-local message for the last non-OK return on this thread. */
const char* q2c_last_error(void);

/* Library version string. */
const char* q2c_version(void);

#ifdef __cplusplus
}
#endif

#endif /* Q2C_H */
