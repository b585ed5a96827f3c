// HIP kernels for gfx950: MPS gate application (contraction, FP64 SVD,
// truncation, update), identity environments, Pauli transfer sweeps and the
// compensated energy sum.  One workgroup owns one MPS slot, so a batch of
// independent circuits runs as a grid of workgroups.
#include <hip/hip_runtime.h>

#include <cmath>

#include "engine.hpp"

namespace q2c {

// ------------------------------------------------------------ helpers ----

__device__ __forceinline__ double2 cmk(double r, double i) { return make_double2(r, i); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return cmk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return cmk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return cmk(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return cmk(a.x * s, a.y * s); }
// acc += a * b
__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ double cabs2(double2 a) { return fma(a.x, a.x, a.y * a.y); }

// complex64 counterparts (mixed-precision path: site tensors, contractions and
// transfer sweeps in FP32 with FP32 accumulation)
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ void cfma(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
}
template <typename T>
__device__ __forceinline__ T cval(double r, double i);
template <>
__device__ __forceinline__ double2 cval<double2>(double r, double i) { return make_double2(r, i); }
template <>
__device__ __forceinline__ float2 cval<float2>(double r, double i) { return make_float2(float(r), float(i)); }
template <typename T>
__device__ __forceinline__ T cfrom(double2 a) { return cval<T>(a.x, a.y); }
__device__ __forceinline__ double2 c64(double2 a) { return a; }
__device__ __forceinline__ double2 c64(float2 a) { return make_double2(double(a.x), double(a.y)); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the block (deterministic order); red needs kBlock/64 doubles.
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// Block-level complex GEMM with a chosen tile: C = alpha * op(A) * op(B)
// (+ C if accumulate), operands as in bgemm below.
// 512 threads as 16 x 32; tile BM x BN (BM = 32 RM, BN = 16 RN) over K in
// steps of BK, staged in lds: (BM + BN) * BK elements.  Every output is
// summed over k in ascending order, whatever the tile, so all tiles give the
// same result bit for bit.  All threads of the block must call it.
template <bool TA, bool TB, typename T, int BM, int BN, int BK>
__device__ void bgemm_tiled(int M, int N, int K, const T* __restrict__ A, int lda, const T* __restrict__ B, int ldb,
                            T* __restrict__ C, int ldc, T alpha, bool accumulate, T* lds) {
  static_assert(BM % 32 == 0 && BN % 16 == 0, "tile must cover the 16 x 32 thread grid");
  constexpr int RM = BM / 32, RN = BN / 16;
  T* As = lds;
  T* Bs = lds + BK * BM;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;  // 16 x 32 threads
  __syncthreads();
  for (int i0 = 0; i0 < M; i0 += BM) {
    for (int j0 = 0; j0 < N; j0 += BN) {
      T acc[RM][RN];
#pragma unroll
      for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int q = 0; q < RN; ++q) acc[r][q] = cval<T>(0.0, 0.0);
      for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (unsigned e = tid; e < unsigned(BM * BK); e += 512) {
          const int r = int(e / BK), k = int(e % BK);
          const int gi = i0 + r, gk = k0 + k;
          T v = cval<T>(0.0, 0.0);
          if (gi < M && gk < K) v = TA ? cconj(A[(long)gk * lda + gi]) : A[(long)gi * lda + gk];
          As[k * BM + r] = v;
        }
#pragma unroll
        for (unsigned e = tid; e < unsigned(BK * BN); e += 512) {
          const int k = int(e / BN), c = int(e % BN);
          const int gk = k0 + k, gj = j0 + c;
          T v = cval<T>(0.0, 0.0);
          if (gk < K && gj < N) v = TB ? cconj(B[(long)gj * ldb + gk]) : B[(long)gk * ldb + gj];
          Bs[k * BN + c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BK; ++k) {
          T a[RM];
#pragma unroll
          for (int r = 0; r < RM; ++r) a[r] = As[k * BM + ty * RM + r];
#pragma unroll
          for (int q = 0; q < RN; ++q) {
            const T bv = Bs[k * BN + tx * RN + q];
#pragma unroll
            for (int r = 0; r < RM; ++r) cfma(acc[r][q], a[r], bv);
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int q = 0; q < RN; ++q) {
          const int gi = i0 + ty * RM + r, gj = j0 + tx * RN + q;
          if (gi < M && gj < N) {
            T v = cmul(alpha, acc[r][q]);
            T* dst = &C[(long)gi * ldc + gj];
            *dst = accumulate ? cadd(*dst, v) : v;
          }
        }
    }
  }
  __syncthreads();
}

// Block-level complex GEMM: C = alpha * op(A) * op(B) (+ C if accumulate).
// op(A)[i][k] = TA ? conj(A[k*lda+i]) : A[i*lda+k]
// op(B)[k][j] = TB ? conj(B[j*ldb+k]) : B[k*ldb+j]
// lds: 2*64*8 double2.  All threads of the block must call it.
template <bool TA, bool TB, typename T>
__device__ void bgemm(int M, int N, int K, const T* __restrict__ A, int lda, const T* __restrict__ B, int ldb,
                      T* __restrict__ C, int ldc, T alpha, bool accumulate, T* lds) {
  constexpr int BM = 64, BN = 64, BK = 8;
  T* As = lds;
  T* Bs = lds + BK * BM;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;  // 16 x 32 threads
  __syncthreads();
  for (int i0 = 0; i0 < M; i0 += BM) {
    for (int j0 = 0; j0 < N; j0 += BN) {
      T acc[2][4];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = cval<T>(0.0, 0.0);
      for (int k0 = 0; k0 < K; k0 += BK) {
        {
          const int r = tid >> 3, k = tid & 7;
          const int gi = i0 + r, gk = k0 + k;
          T v = cval<T>(0.0, 0.0);
          if (gi < M && gk < K) v = TA ? cconj(A[(long)gk * lda + gi]) : A[(long)gi * lda + gk];
          As[k * BM + r] = v;
        }
        {
          const int k = tid >> 6, c = tid & 63;
          const int gk = k0 + k, gj = j0 + c;
          T v = cval<T>(0.0, 0.0);
          if (gk < K && gj < N) v = TB ? cconj(B[(long)gj * ldb + gk]) : B[(long)gk * ldb + gj];
          Bs[k * BN + c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BK; ++k) {
          const T a0 = As[k * BM + ty * 2], a1 = As[k * BM + ty * 2 + 1];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const T bv = Bs[k * BN + tx * 4 + q];
            cfma(acc[0][q], a0, bv);
            cfma(acc[1][q], a1, bv);
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int gi = i0 + ty * 2 + r, gj = j0 + tx * 4 + q;
          if (gi < M && gj < N) {
            T v = cmul(alpha, acc[r][q]);
            T* dst = &C[(long)gi * ldc + gj];
            *dst = accumulate ? cadd(*dst, v) : v;
          }
        }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------- MFMA complex GEMM --
// C[M x N] = alpha * op(A) * op(B) (+ C if accumulate) on the matrix cores,
// operands as in bgemm, read straight from memory (L2/L1-resident slot
// workspace).  Each wave computes 16 x 16 NT strips of C, strips dealt out
// round-robin over the waves; K advances 4 at a time (one 16x16x4 MFMA per
// real product: Re += ar br - ai bi, Im += ar bi + ai br) with the next
// operands loaded while the current ones multiply.  FP64 operands use
// v_mfma_f64_16x16x4 (output row of lane l, register r: l / 16 + 4 r), FP32
// operands v_mfma_f32_16x16x4 (output row 4 (l / 16) + r).  All threads of
// the block must call it; it begins and ends with a block barrier.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaOps;
template <>
struct MfmaOps<double2> {
  using R = double;
  using Acc = mfma_d4;
  static __device__ __forceinline__ Acc mma(R a, R b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct MfmaOps<float2> {
  using R = float;
  using Acc = mfma_f4;
  static __device__ __forceinline__ Acc mma(R a, R b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

template <bool TA, bool TB, typename T, int NT>
__device__ __noinline__ void zgemm_mfma(int M, int N, int K, const T* __restrict__ A, int lda, const T* __restrict__ B,
                                        int ldb, T* __restrict__ C, int ldc, T alpha, bool accumulate) {
  using Op = MfmaOps<T>;
  using Acc = typename Op::Acc;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tm = (M + 15) >> 4, tn = (N + 16 * NT - 1) / (16 * NT);
  for (int t = wave; t < tm * tn; t += nw) {
    const int i0 = (t / tn) * 16, j0 = (t % tn) * (16 * NT);
    const int ia = i0 + li;
    auto ldA = [&](int k) -> T {
      if (ia >= M || k >= K) return cval<T>(0.0, 0.0);
      return TA ? cconj(A[(long)k * lda + ia]) : A[(long)ia * lda + k];
    };
    auto ldB = [&](int k, int j) -> T {
      if (j >= N || k >= K) return cval<T>(0.0, 0.0);
      return TB ? cconj(B[(long)j * ldb + k]) : B[(long)k * ldb + j];
    };
    Acc cr[NT], ci[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      cr[q] = Acc{0, 0, 0, 0};
      ci[q] = Acc{0, 0, 0, 0};
    }
    T a = ldA(lk), bb[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) bb[q] = ldB(lk, j0 + 16 * q + li);
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int kn = k0 + 4 + lk;
      const T an = ldA(kn);
      T bn[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) bn[q] = ldB(kn, j0 + 16 * q + li);
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        cr[q] = Op::mma(a.x, bb[q].x, cr[q]);
        cr[q] = Op::mma(-a.y, bb[q].y, cr[q]);
        ci[q] = Op::mma(a.x, bb[q].y, ci[q]);
        ci[q] = Op::mma(a.y, bb[q].x, ci[q]);
      }
      a = an;
#pragma unroll
      for (int q = 0; q < NT; ++q) bb[q] = bn[q];
    }
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + Op::row(lk, r), col = j0 + 16 * q + li;
        if (row < M && col < N) {
          T v;
          v.x = cr[q][r];
          v.y = ci[q][r];
          v = cmul(alpha, v);
          T* dst = &C[(long)row * ldc + col];
          *dst = accumulate ? cadd(*dst, v) : v;
        }
      }
  }
  __syncthreads();
}

// Householder vector for a row (conj=true: reflector applied from the
// right to rows, built from conj(x)) or a column (conj=false).
// Given x (len L) returns u with H = I - u u^H mapping x -> -ph*|x| e_0 and
// writes beta = -ph*|x| (the new leading entry; for rows the entry stored in
// the row is beta as well).  Executed by one wave; u written to dst.
__device__ void wave_householder(const double2* x, int L, bool rowform, double2* dst, double2* beta_out,
                                 bool* zero_out) {
  const int lane = threadIdx.x & 63;
  double nrm2 = 0.0;
  for (int j = lane; j < L; j += 64) nrm2 += cabs2(x[j]);
  nrm2 = wave_sum(nrm2);
  const double nx = sqrt(nrm2);
  const double2 x0 = x[0];
  const double ax = sqrt(cabs2(x0));
  const double2 ph = ax > 0.0 ? cscale(x0, 1.0 / ax) : cmk(1.0, 0.0);
  if (nx == 0.0) {
    for (int j = lane; j < L; j += 64) dst[j] = cmk(0.0, 0.0);
    if (lane == 0) {
      *beta_out = cmk(0.0, 0.0);
      *zero_out = true;
    }
    return;
  }
  const double inv = 1.0 / sqrt(nx * (nx + ax));
  for (int j = lane; j < L; j += 64) {
    double2 v = x[j];
    if (j == 0) v = cscale(ph, ax + nx);
    if (rowform) v = cconj(v);
    dst[j] = cscale(v, inv);
  }
  if (lane == 0) {
    *beta_out = cscale(ph, -nx);
    *zero_out = false;
  }
}

// ---------------------------------------------------------- init / angles --

template <typename S>
__global__ void k_init_product(DevBatch b, const uint8_t* occ) {
  const int slot = b.slot0 + blockIdx.x;
  const int N = b.n_qubits;
  S* sites = reinterpret_cast<S*>(b.sites + slot * b.site_stride);  // slot bases as in slot_view
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    S* B = sites + b.site_off[n];
    const int o = occ[n] ? 1 : 0;
    // chi_l = chi_r = 1: element [0][i][0] at i * cap_r
    B[0] = cval<S>(o == 0 ? 1.0 : 0.0, 0.0);
    B[b.cap[n + 1]] = cval<S>(o == 1 ? 1.0 : 0.0, 0.0);
  }
  for (int i = threadIdx.x; i <= N; i += blockDim.x) b.chi[slot * (N + 1) + i] = 1;
  for (int n = threadIdx.x; n < N - 1; n += blockDim.x) b.lam[slot * b.lam_stride + b.lam_off[n]] = 1.0;
  for (int i = threadIdx.x; i < kNStats; i += blockDim.x) b.stats[slot * kNStats + i] = 0.0;
  if (threadIdx.x == 0) {
    b.stats[slot * kNStats + kStatMaxChi] = 1.0;
    b.flags[slot] = 0;
  }
}

// State copy between slots of two batches of one shape: the site tensors,
// Schmidt values, bond dimensions, statistics and flags of slot pr.x of src
// go to slot pr.y of dst, pr = pairs[blockIdx.x] (pairs null: the one pair
// given).  With clear_work the copy's executed-work counters (FLOPs, sweeps,
// cycles, SVD path counts) start from zero, so that summing them over slots
// counts every gate that ran once.
__global__ void k_copy_slots(DevBatch src, DevBatch dst, const int2* pairs, int2 one, int clear_work) {
  const int2 pr = pairs ? pairs[blockIdx.x] : one;
  const int N = src.n_qubits;
  const long n16 = (src.site_off[N] * (src.mixed ? 8 : 16) + 15) / 16;
  const uint4* s4 = reinterpret_cast<const uint4*>(src.sites + pr.x * src.site_stride);
  uint4* d4 = reinterpret_cast<uint4*>(dst.sites + pr.y * dst.site_stride);
  for (long i = threadIdx.x; i < n16; i += blockDim.x) d4[i] = s4[i];
  for (long i = threadIdx.x; i < src.lam_off[N - 1]; i += blockDim.x)
    dst.lam[pr.y * dst.lam_stride + i] = src.lam[pr.x * src.lam_stride + i];
  for (int i = threadIdx.x; i <= N; i += blockDim.x) dst.chi[pr.y * (N + 1) + i] = src.chi[pr.x * (N + 1) + i];
  for (int i = threadIdx.x; i < kNStats; i += blockDim.x) {
    const bool work = i == kStatFlops || i == kStatSweepSum || (i >= kStatCycContract && i <= kStatCycUpdate) ||
                      i == kStatFallbacks || i == kStatBisect;
    dst.stats[pr.y * kNStats + i] = (clear_work && work) ? 0.0 : src.stats[pr.x * kNStats + i];
  }
  if (threadIdx.x == 0) dst.flags[pr.y] = src.flags[pr.x];
}

// phi of slots slot0 + y (theta and the shifts are indexed from the launch's first slot)
__global__ void k_angles(double* phi, int n_rot, const double* rot_c, const int* rot_param,
                         const double* theta, int n_theta, const int* shift_rot, const double* shift_val,
                         int slot0) {
  const int r = blockIdx.y, slot = slot0 + r;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_rot) return;
  const int k = rot_param[m];
  double th = theta[(long)r * n_theta + k];
  double add = 0.0;
  if (shift_rot) {
    // shift target: rotation t >= 0 (phi_t += shift), or parameter -2 - t
    // (theta_k += shift for every rotation of that parameter); -1: none
    const int t = shift_rot[r];
    if (t == m) add = shift_val[r];
    if (t == -2 - k) th += shift_val[r];
  }
  phi[(long)slot * n_rot + m] = -2.0 * rot_c[m] * th + add;
}

// ----------------------------------------------------------- gate kernel --

struct SlotView {
  double2* sites;
  double* lam;
  int* chi;
  double2 *M, *A, *H, *W;
  double* V;  // inverse-iteration scratch and real vectors (8 ws^2 doubles)
  double* S;
  int* P;
  double* stats;
  int* flags;
};

__device__ SlotView slot_view(const DevBatch& b, int slot) {
  SlotView v;
  v.sites = b.sites + slot * b.site_stride;
  v.lam = b.lam + slot * b.lam_stride;
  v.chi = b.chi + slot * (b.n_qubits + 1);
  v.M = b.wsM + slot * b.ws_stride;
  v.A = b.wsA + slot * b.ws_stride;
  v.H = b.wsH + slot * b.ws_stride;
  v.W = b.wsW + slot * b.ws_stride;
  v.V = reinterpret_cast<double*>(b.wsV + slot * 4 * b.ws_stride);
  v.S = b.wsS + slot * 2 * b.ws;
  v.P = b.wsP + slot * b.ws;
  v.stats = b.stats + slot * kNStats;
  v.flags = b.flags + slot;
  return v;
}

// Circle-method round-robin: position -> row in round t (P even).
__device__ __forceinline__ int rr_row(int pos, int t, int P) {
  return pos == 0 ? 0 : 1 + ((pos - 1 + t) % (P - 1));
}


constexpr int kQB = 128;      // bisection path: q = min(m, n) <= kQB
constexpr int kKB = 64;       // bisection path: kept vectors <= kKB
constexpr int kZS = kKB + 1;  // row stride (doubles) of the vector work array

// Static LDS of the gate kernel (about 150 KB of the 160 KB per CU).
struct GateLds {
  double2 O[16];
  double2 dc[kQB], ec[kQB], pa[kQB], pb[kQB];  // bidiagonal and its phases
  double t[2 * kQB], t2[2 * kQB + 16];         // Golub-Kahan tridiagonal (t2 zero-padded)
  double sig[512];                             // kept singular values, descending
  double ldiag[kKB];                           // reciprocal Cholesky diagonal
  int blo[2 * kQB], bhi[2 * kQB];              // blocks of the split tridiagonal
  double red[16];
  double2 sbeta;
  int szero, srot, sabort, skeep, sfail, snblk;
  double sdisc, stot, snorm, sgersh, stmax;
  union {
    double2 gemm[2 * 64 * 8];  // block-GEMM tiles
    struct {
      double2 uq[512], wq[512], vq[512], zq[512];  // Jacobi-path work vectors
    };
    struct {
      double2 rowb[2][kQB], w[kQB];
      double2 part[8][kQB];
    } bd;                      // exchange area of the bidiagonalisation
    double Z[2 * kQB * kZS];   // twisted factorisations, kept vectors, Gram; later reflectors
  };
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---- cross-lane sums without the LDS pipe (DPP row ops and gfx950 lane swaps).
// Every lane of the wave must execute them.
template <int kCtrl>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), kCtrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// Sum over the 16 lanes of a row; every lane of the row gets the same value.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_mov<0x128>(v);  // row_ror:8
  v += dpp_mov<0x124>(v);  // row_ror:4
  v += dpp_mov<0x4E>(v);   // quad_perm 2,3,0,1
  v += dpp_mov<0xB1>(v);   // quad_perm 1,0,3,2
  return v;
}
// Sum over the four lanes of a quad.
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0xB1>(v);
  return v;
}
// Lanes below 32 return a(l) + a(l + 32); the others b(l - 32) + b(l).
__device__ __forceinline__ double pair_sum32(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
// Lanes in even 16-lane rows return a(l) + a(l + 16); odd rows b(l - 16) + b(l).
__device__ __forceinline__ double pair_sum16(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double2 pair_sum32(double2 a, double2 b) {
  return cmk(pair_sum32(a.x, b.x), pair_sum32(a.y, b.y));
}
__device__ __forceinline__ double2 pair_sum16(double2 a, double2 b) {
  return cmk(pair_sum16(a.x, b.x), pair_sum16(a.y, b.y));
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Number of eigenvalues below x of the symmetric tridiagonal with zero diagonal
// whose squared off-diagonals are t2[0 .. n-2]: the sign changes along the
// leading minors p_0 = 1, p_1 = -x, p_{i+1} = -x p_i - t2[i-1] p_{i-1}.  A zero
// off-diagonal needs no special case (minors of a block-diagonal matrix
// factorise).  With |t| <= 1 and 0 < x <= 1 the values grow by less than 2^12
// over sixteen steps; off-diagonals below 1e-15 of the largest are split off,
// so t2 >= 1e-30 and a pair of minors shrinks by at most 2^-800 over sixteen
// steps.  A power-of-two renormalisation whenever the larger exponent leaves
// [-200, 200], checked every sixteen steps, keeps them in range.
// Division-free.  t2 must be readable up to index n + 14 (zero padding).
__device__ int sturm_count(const double* __restrict__ t2, int n, double x) {
  const double nx = -x;
  double pm = 1.0, pc = nx;
  unsigned last = (unsigned)__double2hiint(pc) >> 31;  // sign bit of p_1
  int c = (int)last;                                   // p_0 = 1 > 0
  int i = 1;
  // t2 is read one chunk of sixteen ahead
  double tt[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) tt[u] = t2[u];
  for (; i + 16 <= n; i += 16) {
    double tn[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) tn[u] = t2[i + 15 + u];
    // shift register of sign bits: bit 16 holds the sign of p_i, bit 0 that of p_{i+16}
    unsigned w = last;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const double pn = fma(nx, pc, -tt[u] * pm);
      pm = pc;
      pc = pn;
      w = __builtin_amdgcn_alignbit(w, (unsigned)__double2hiint(pn), 31u);
    }
    c += __builtin_popcount((w ^ (w >> 1)) & 0xFFFFu);
    last = w & 1u;
    const int e = max(__builtin_amdgcn_frexp_exp(pc), __builtin_amdgcn_frexp_exp(pm));
    if (e > 200 || e < -200) {
      pc = ldexp(pc, -e);
      pm = ldexp(pm, -e);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) tt[u] = tn[u];
  }
  for (; i < n; ++i) {
    const double pn = fma(nx, pc, -t2[i - 1] * pm);
    const unsigned sg = (unsigned)__double2hiint(pn) >> 31;
    c += (int)(sg ^ last);
    last = sg;
    pm = pc;
    pc = pn;
  }
  return c;
}

// 1/d to full double precision: hardware estimate and two Newton steps.
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// 1/sqrt(x) for normal x > 0: hardware estimate and two Newton steps.
__device__ __forceinline__ double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = fma(-h * r, r, 0.5);
  r = fma(r, e, r);
  e = fma(-h * r, r, 0.5);
  return fma(r, e, r);
}

// x -= a * b and x -= a * conj(b), four fused multiply-adds each
__device__ __forceinline__ void cfms(double2& x, double2 a, double2 b) {
  x.x = fma(-a.x, b.x, x.x);
  x.x = fma(a.y, b.y, x.x);
  x.y = fma(-a.x, b.y, x.y);
  x.y = fma(-a.y, b.x, x.y);
}
// y - conj(a) b
__device__ __forceinline__ double2 cfms_conj_val(double2 y, double2 a, double2 b) {
  y.x = fma(-a.x, b.x, y.x);
  y.x = fma(-a.y, b.y, y.x);
  y.y = fma(-a.x, b.y, y.y);
  y.y = fma(a.y, b.x, y.y);
  return y;
}
__device__ __forceinline__ void cfms_conj(double2& x, double2 a, double2 b) {
  x.x = fma(-a.x, b.x, x.x);
  x.x = fma(-a.y, b.y, x.x);
  x.y = fma(a.x, b.y, x.y);
  x.y = fma(-a.y, b.x, x.y);
}

// Householder scalars for a vector with squared norm n2 and leading entry x0:
// H = I - u u^H maps x to beta e_0 with beta = -ph |x|, ph = x0 / |x0| (1 if
// x0 = 0); u = x * inv except u_0 = ph (|x0| + |x|) inv.  Norms below 1e-280
// count as zero (no reflection).
struct HhScalars {
  double2 ph, beta;
  double inv, head;  // u_0 = ph * head
  bool zero;
};
__device__ __forceinline__ HhScalars hh_scalars(double n2, double2 x0) {
  HhScalars h;
  h.zero = !(n2 > 1e-280);
  const double nx = h.zero ? 0.0 : n2 * rsq_nr(n2);
  const double ax2 = cabs2(x0);
  const double ra = ax2 > 1e-280 ? rsq_nr(ax2) : 0.0;
  const double ax = ax2 * ra;
  h.ph = ax2 > 1e-280 ? cscale(x0, ra) : cmk(1.0, 0.0);
  h.inv = h.zero ? 0.0 : rsq_nr(nx * (nx + ax));
  h.head = (ax + nx) * h.inv;
  h.beta = h.zero ? cmk(0.0, 0.0) : cscale(h.ph, -nx);
  return h;
}

// ---- Phase A: Theta = B_n B_{n+1}, gate mixing (Eq. 7), lambda scaling (Eq. 8)
// S = double2 (FP64 path) or float2 (mixed path: Theta and M in complex64; M'
// for the SVD always in FP64).
template <typename S>
__device__ void gate_contract(const DevBatch& b, SlotView& v, GateLds& L, int n, int chil, int chim, int chir) {
  const int tid = threadIdx.x;
  const int nn = 2 * chir, m = 2 * chil;
  const int capl_r = b.cap[n + 1], capr_r = b.cap[n + 2];
  const S* sites = reinterpret_cast<const S*>(v.sites);
  const S* Bn = sites + b.site_off[n];
  const S* Bn1 = sites + b.site_off[n + 1];
  S* Mw = reinterpret_cast<S*>(v.M);
  for (int j = 0; j < 2; ++j)
    zgemm_mfma<false, false, S, 4>(m, chir, chim, Bn, capl_r, Bn1 + j * capr_r, 2 * capr_r, Mw + j * chir, nn,
                                   cval<S>(1.0, 0.0), false);
  double part = 0.0;
  for (int idx = tid; idx < chil * chir; idx += blockDim.x) {
    const int a = idx / chir, c = idx - a * chir;
    S t[4];
#pragma unroll
    for (int ip = 0; ip < 2; ++ip)
#pragma unroll
      for (int jp = 0; jp < 2; ++jp) t[2 * ip + jp] = Mw[(long)(2 * a + ip) * nn + jp * chir + c];
    const double la = n == 0 ? 1.0 : v.lam[b.lam_off[n - 1] + a];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        S s = cval<S>(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < 4; ++q) cfma(s, cfrom<S>(L.O[(2 * i + jj) * 4 + q]), t[q]);
        const long off = (long)(2 * a + i) * nn + jj * chir + c;
        Mw[off] = s;
        const double2 sp = cscale(c64(s), la);
        v.A[off] = sp;
        part += cabs2(sp);
      }
  }
  const double tot = block_sum(part, L.red);
  if (tid == 0) L.stot = tot;
  __syncthreads();
}

// M' = lambda * M again (before the Jacobi fallback).
template <typename S>
__device__ void restore_mprime(const DevBatch& b, SlotView& v, int n, int chil, int chir) {
  const int nn = 2 * chir;
  const S* Mw = reinterpret_cast<const S*>(v.M);
  for (int idx = threadIdx.x; idx < 2 * chil * nn; idx += blockDim.x) {
    const int row = idx / nn;
    const double la = n == 0 ? 1.0 : v.lam[b.lam_off[n - 1] + (row >> 1)];
    v.A[idx] = cscale(c64(Mw[idx]), la);
  }
  __syncthreads();
}

// Values that are the same in every lane, moved to scalar registers so that
// conditions on them compile to uniform branches (function arguments arrive in
// vector registers and would otherwise count as divergent).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ double uni(double x) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x)),
                          __builtin_amdgcn_readfirstlane(__double2loint(x)));
}

// ---- Phase B (default), step 1: Golub-Kahan bidiagonalisation of the p x q
// matrix X (p >= q <= 128) held in registers.  Thread (r0, c0), r0 = 4 wave +
// lane / 16, c0 = lane % 16, owns X[r0 + 32 rs][c0 + 16 cs] for rs < 4, cs < 8,
// so that a wave holds whole rows and the rows and columns still active at
// step k are spread evenly over all waves.  Step k (in phase KS = k / 16,
// which fixes the register slot of column k and of row k at compile time)
// applies H_k from the left to zero column k below the diagonal and G_k from
// the right to zero row k right of the superdiagonal.  The reflectors needed
// for the back-transformation go to global memory: G_k (stored conjugated, as
// applied to columns) when X = M', H_k when X = M'^H.
struct BdArgs {
  double2* Hg;
  int ldh, p, q, r0, c0, lane, wave;
  bool trans;
};

template <int KS>
__device__ __forceinline__ void bd_step(double2 (&X)[4][8], const int k, const BdArgs& a, GateLds& L) {
  constexpr int RSK = KS / 2, CSK = KS;
  const int tid = threadIdx.x;
  double2* rowb = L.bd.rowb[k & 1];  // row k before H_k (double-buffered: a wave may run one step ahead)
  // ---- A: x = column k (rows k .. p-1) from the lane that holds it in this
  // thread's 16-lane row group; partial y_j = sum_i conj(x_i) X_ij over this
  // thread's rows (y_k = |x|^2), reduced over the four lanes sharing c0.
  double2 x[4];
  {
    const int src = (a.lane & 0x30) | (k & 15);
#pragma unroll
    for (int rs = 0; rs < 4; ++rs) {
      double2 xv = cmk(0.0, 0.0);
      if (rs >= RSK) {
        xv.x = __shfl(X[rs][CSK].x, src, 64);
        xv.y = __shfl(X[rs][CSK].y, src, 64);
        // rows in slots above RSK are all below row k; only slot RSK is masked
        if (rs == RSK && a.r0 + 32 * rs < k) xv = cmk(0.0, 0.0);
      }
      x[rs] = xv;
    }
    double2 wp[8];
#pragma unroll
    for (int cs = 0; cs < 8; ++cs) {
      double2 acc = cmk(0.0, 0.0);
      if (cs >= CSK) {
#pragma unroll
        for (int rs = RSK; rs < 4; ++rs) {
          const double2 uc = x[rs], xv = X[rs][cs];
          acc.x = fma(uc.x, xv.x, acc.x);
          acc.x = fma(uc.y, xv.y, acc.x);
          acc.y = fma(uc.x, xv.y, acc.y);
          acc.y = fma(-uc.y, xv.x, acc.y);
        }
      }
      wp[cs] = acc;
    }
    // reduce-scatter over the four lanes sharing c0: lane bits (5, 4) = (b5, b4)
    // keep column slots 4 b5 + 2 b4 + {0, 1}
    double2 h[4], g[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) h[i] = pair_sum32(wp[i], wp[4 + i]);
#pragma unroll
    for (int i = 0; i < 2; ++i) g[i] = pair_sum16(h[i], h[2 + i]);
    const int sb = 4 * ((a.lane >> 5) & 1) + 2 * ((a.lane >> 4) & 1);
    L.bd.part[a.wave][a.c0 + 16 * sb] = g[0];
    L.bd.part[a.wave][a.c0 + 16 * (sb + 1)] = g[1];
    if (a.r0 == (k & 31)) {
#pragma unroll
      for (int cs = CSK; cs < 8; ++cs) rowb[a.c0 + 16 * cs] = X[RSK][cs];
    }
  }
  __syncthreads();
  // ---- B: y_j = sum over the waves (j >= k)
  if (tid < kQB) {
    double2 sy = cmk(0.0, 0.0);
    if (tid >= k) {
#pragma unroll
      for (int w = 0; w < 8; ++w) sy = cadd(sy, L.bd.part[w][tid]);
    }
    L.bd.w[tid] = sy;
  }
  __syncthreads();
  // ---- C: H_k = I - u u^H from |x|^2 = Re y_k and the pivot X_kk; with
  // u = inv (x - alpha e_k), w_j = sum_i conj(u_i) X_ij = inv (y_j - conj(alpha) X_kj)
  // every input of the reflector scalars is the same in all lanes; taken from
  // lane 0 they are wave-uniform, so the branches on them are scalar
  const HhScalars h = hh_scalars(uni(L.bd.w[k].x), cmk(uni(rowb[k].x), uni(rowb[k].y)));
  if (tid == 0) L.dc[k] = h.beta;
  const double2 uk = cscale(h.ph, h.head);
  double2 wj[8], rj[8];  // w_j and row k before H_k, own columns (zero for j <= k)
#pragma unroll
  for (int cs = 0; cs < 8; ++cs) {
    const int j = a.c0 + 16 * cs;
    // columns in slots above CSK are all right of column k; only slot CSK is masked
    rj[cs] = (cs > CSK || (cs == CSK && j > k)) ? rowb[j] : cmk(0.0, 0.0);
    wj[cs] = cmk(0.0, 0.0);
  }
  if (!h.zero) {  // uniform; one branch around the whole block
#pragma unroll
    for (int cs = CSK; cs < 8; ++cs) {
      const int j = a.c0 + 16 * cs;
      const double2 wv = cscale(cfms_conj_val(L.bd.w[j], h.beta, rj[cs]), h.inv);
      wj[cs] = (cs > CSK || j > k) ? wv : cmk(0.0, 0.0);  // w_j = 0 for j <= k (y_k = |x|^2 is not w_k)
    }
  }
  {
    // u (zero when the column is already zero: H_k = I, stored as such)
    double2 u[4];
#pragma unroll
    for (int rs = 0; rs < 4; ++rs) {
      const int i = a.r0 + 32 * rs;
      double2 uv = cmk(0.0, 0.0);
      if (!h.zero) {
        if (rs > RSK) uv = cscale(x[rs], h.inv);
        else if (rs == RSK && i >= k) uv = i == k ? uk : cscale(x[rs], h.inv);
      }
      u[rs] = uv;
      if (a.trans && a.c0 == 0 && (rs > RSK || (rs == RSK && i >= k)) && i < a.p) a.Hg[(long)k * a.ldh + i] = uv;
    }
    if (!h.zero) {
#pragma unroll
      for (int cs = CSK; cs < 8; ++cs)
#pragma unroll
        for (int rs = RSK; rs < 4; ++rs) cfms(X[rs][cs], u[rs], wj[cs]);
    }
  }
  if (k >= a.q - 1) return;
  // ---- G_k on row k after H_k, columns k+1 .. q-1: every 16-lane row group
  // rebuilds the row from rowb and w (the owner's registers hold the same
  // values) and sums its norm, so no exchange is needed.
  if (!h.zero) {
#pragma unroll
    for (int cs = CSK; cs < 8; ++cs) cfms(rj[cs], uk, wj[cs]);
  }
  double s = 0.0;
#pragma unroll
  for (int cs = CSK; cs < 8; ++cs) s += cabs2(rj[cs]);
  // the 16-lane sum's rounding depends on the lane; lane 0's value is used everywhere
  s = uni(row16_sum(s));
  double2 rk1 = cmk(0.0, 0.0);
  if (k + 1 < a.q) {
    rk1 = rowb[k + 1];
    if (!h.zero) cfms(rk1, uk, cscale(cfms_conj_val(L.bd.w[k + 1], h.beta, rk1), h.inv));
    rk1 = cmk(uni(rk1.x), uni(rk1.y));
  }
  const HhScalars g = hh_scalars(s, rk1);
  if (tid == 0) L.ec[k] = g.beta;
  // v (zero when the row is already zero: G_k = I, stored as such)
  double2 vv[8];
#pragma unroll
  for (int cs = 0; cs < 8; ++cs) vv[cs] = cmk(0.0, 0.0);
  if (!g.zero) {
    // rj is zero for j <= k; column k + 1 (the pivot) lies in slot CSK or CSK + 1
    const double2 head = cscale(g.ph, g.head);
#pragma unroll
    for (int cs = CSK; cs < 8; ++cs) {
      const int j = a.c0 + 16 * cs;
      const double2 xv = cscale(rj[cs], g.inv);
      vv[cs] = cconj((cs <= CSK + 1 && j == k + 1) ? head : xv);
    }
  }
  if (!a.trans && a.r0 == 0) {
#pragma unroll
    for (int cs = CSK; cs < 8; ++cs) {
      const int j = a.c0 + 16 * cs;
      if ((cs > CSK || j > k) && j < a.q) a.Hg[(long)k * a.ldh + j] = vv[cs];
    }
  }
  if (g.zero) return;
  // z_i = sum_j X_ij v_j; rows are whole within a 16-lane row of the wave
  double2 zp[4];
#pragma unroll
  for (int rs = 0; rs < 4; ++rs) {
    double2 acc = cmk(0.0, 0.0);
    if (rs >= RSK) {
#pragma unroll
      for (int cs = CSK; cs < 8; ++cs) cfma(acc, X[rs][cs], vv[cs]);
      acc.x = row16_sum(acc.x);
      acc.y = row16_sum(acc.y);
      if (rs == RSK && a.r0 + 32 * rs <= k) acc = cmk(0.0, 0.0);
    }
    zp[rs] = acc;
  }
#pragma unroll
  for (int rs = RSK; rs < 4; ++rs)
#pragma unroll
    for (int cs = CSK; cs < 8; ++cs) cfms_conj(X[rs][cs], zp[rs], vv[cs]);
}

template <int KS>
__device__ __forceinline__ void bd_phase(double2 (&X)[4][8], const BdArgs& a, GateLds& L) {
  if (16 * KS >= a.q) return;
  for (int k1 = 0; k1 < 16; ++k1) {
    const int k = 16 * KS + k1;
    if (k >= a.q) break;
    bd_step<KS>(X, k, a, L);
  }
}

// ---- Phase B (default): SVD by Golub-Kahan bidiagonalisation (registers),
// bisection on the Golub-Kahan tridiagonal for the kept singular values,
// twisted factorisations for their vectors (LDS), CholQR and back-
// transformation through the reflectors.  Output: L.sig[0..keep) descending,
// v.W rows = kept rows of W^H (n wide), L.sdisc.  Returns keep, or -1 if the
// vectors could not be certified (the caller then uses the Jacobi path).
// Requires min(m, n) <= kQB, max(m, n) <= ws, D <= kKB.  The four steps are
// separate functions; each starts and ends with every thread in step.
struct SvdShape {
  int m, nn, p, q, D, ws;
  bool trans;
  double cutoff;
};

__device__ __forceinline__ SvdShape svd_shape(int m, int nn, int D, double cutoff, int ws) {
  SvdShape sh;
  sh.m = uni(m);
  sh.nn = uni(nn);
  sh.D = uni(D);
  sh.ws = uni(ws);
  sh.cutoff = uni(cutoff);
  sh.trans = sh.m < sh.nn;
  sh.p = sh.trans ? sh.nn : sh.m;
  sh.q = sh.trans ? sh.m : sh.nn;
  return sh;
}

// Step 1: bidiagonal (L.dc, L.ec) and the reflectors for step 4 (v.H).
__device__ __noinline__ void svd_bidiag(const SlotView& v, GateLds& L, const SvdShape& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = uni(sh.p), q = uni(sh.q), nn = uni(sh.nn);
  const bool trans = p != uni(sh.m);
  (void)tid; (void)lane; (void)wave; (void)trans; (void)p; (void)q; (void)nn;
  double2* Hg = v.H;  // reflector k in row k (stride ws)
  const int ws = uni(sh.ws);
  {
    BdArgs a;
    a.Hg = Hg;
    a.ldh = ws;
    a.p = p;
    a.q = q;
    a.r0 = 4 * wave + (lane >> 4);
    a.c0 = lane & 15;
    a.lane = lane;
    a.wave = wave;
    a.trans = trans;
    double2 X[4][8];
#pragma unroll
    for (int rs = 0; rs < 4; ++rs)
#pragma unroll
      for (int cs = 0; cs < 8; ++cs) {
        const int i = a.r0 + 32 * rs, j = a.c0 + 16 * cs;
        double2 x = cmk(0.0, 0.0);
        if (i < p && j < q) x = trans ? cconj(v.A[(long)j * nn + i]) : v.A[(long)i * nn + j];
        X[rs][cs] = x;
      }
    bd_phase<0>(X, a, L);
    bd_phase<1>(X, a, L);
    bd_phase<2>(X, a, L);
    bd_phase<3>(X, a, L);
    bd_phase<4>(X, a, L);
    bd_phase<5>(X, a, L);
    bd_phase<6>(X, a, L);
    bd_phase<7>(X, a, L);
  }
  __syncthreads();
}

// Step 2: kept singular values (L.sig, scaled by 1/L.sgersh), keep count
// (L.skeep, -1 on failure), discarded weight (L.sdisc) and the split
// tridiagonal (L.t, L.t2, L.blo/bhi).
__device__ __noinline__ void svd_values(GateLds& L, const SvdShape& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = uni(sh.p), q = uni(sh.q), nn = uni(sh.nn);
  const bool trans = p != uni(sh.m);
  (void)tid; (void)lane; (void)wave; (void)trans; (void)p; (void)q; (void)nn;
  const int D = uni(sh.D);
  const double cutoff = uni(sh.cutoff);
  // -- real bidiagonal by diagonal phase scaling; Golub-Kahan tridiagonal t
  if (tid < q) {
    const double2 d = L.dc[tid];
    const double ad = sqrt(cabs2(d));
    L.t[2 * tid] = ad;
    L.pa[tid] = ad > 0.0 ? cscale(d, 1.0 / ad) : cmk(1.0, 0.0);
    if (tid + 1 < q) {
      const double2 e = L.ec[tid];
      const double ae = sqrt(cabs2(e));
      L.t[2 * tid + 1] = ae;
      L.pb[tid + 1] = ae > 0.0 ? cscale(cconj(e), 1.0 / ae) : cmk(0.0, 0.0);
    }
  }
  __syncthreads();
  const int nT = 2 * q;
  if (wave == 0) {
    if (lane == 0) {
      // phases: a_k = (d_k/|d_k|) b_k, b_{k+1} = a_k conj(e_k)/|e_k| (b restarts at 1 after e_k = 0)
      double2 bk = cmk(1.0, 0.0);
#pragma unroll 4
      for (int k = 0; k < q; ++k) {
        const double2 ak = cmul(L.pa[k], bk);
        const double2 ue = k + 1 < q ? L.pb[k + 1] : cmk(0.0, 0.0);
        L.pa[k] = ak;
        L.pb[k] = bk;
        bk = (ue.x != 0.0 || ue.y != 0.0) ? cmul(ak, ue) : cmk(1.0, 0.0);
      }
    }
    // split at negligible entries, scale to norm <= 1, find the blocks
    double tm = 0.0;
    for (int i = lane; i < nT - 1; i += 64) tm = fmax(tm, L.t[i]);
    tm = wave_max(tm);
    for (int i = lane; i < nT - 1; i += 64)
      if (L.t[i] <= 1e-15 * tm) L.t[i] = 0.0;
    wave_sync();
    double gs = 0.0;
    for (int i = lane; i < nT; i += 64) gs = fmax(gs, (i < nT - 1 ? L.t[i] : 0.0) + (i > 0 ? L.t[i - 1] : 0.0));
    gs = wave_max(gs);
    const double sc = gs > 0.0 ? 1.0 / gs : 1.0;
    wave_sync();
    for (int i = lane; i < nT + 15; i += 64) {
      const double x = i < nT - 1 ? L.t[i] * sc : 0.0;
      if (i < nT - 1) L.t[i] = x;
      L.t2[i] = x * x;
    }
    wave_sync();
    int nb = 0, start = 0;
    for (int base = 0; base < nT - 1; base += 64) {
      const int i = base + lane;
      unsigned long long msk = __ballot(i < nT - 1 && L.t[i] == 0.0);
      while (msk) {
        const int ii = base + __ffsll((long long)msk) - 1;
        msk &= msk - 1;
        if (lane == 0) {
          L.blo[nb] = start;
          L.bhi[nb] = ii + 1;
        }
        ++nb;
        start = ii + 1;
      }
    }
    if (lane == 0) {
      L.blo[nb] = start;
      L.bhi[nb] = nT;
      L.snblk = nb + 1;
      L.sgersh = gs;
      L.stmax = tm;
    }
  }
  __syncthreads();
  const double tscale = L.sgersh;  // singular values = scaled values * tscale
  const int kk = D < q ? D : q;
  // -- bisection on the scaled T: 8 lanes (one point each) per value ->
  // 9-section, 18 steps (9^18 > 1e17)
  {
    const int j0 = tid >> 3, s8 = tid & 7;
    const int j = j0 < kk ? j0 : kk - 1;
    const int idx = nT - 1 - j;  // the value has exactly idx eigenvalues below it
    double lo = 0.0, hi = 1.0 + 1e-14;
    for (int it = 0; it < 18; ++it) {
      const double w = (hi - lo) * (1.0 / 9.0);
      const double x = lo + (s8 + 1) * w;
      const int c = sturm_count(L.t2, nT, x);
      double nlo = c <= idx ? x : lo;
      double nhi = c <= idx ? hi : x;
#pragma unroll
      for (int o = 1; o < 8; o <<= 1) {
        nlo = fmax(nlo, __shfl_xor(nlo, o, 64));
        nhi = fmin(nhi, __shfl_xor(nhi, o, 64));
      }
      lo = nlo;
      hi = nhi;
    }
    if (s8 == 0 && j0 < kk) L.sig[j0] = 0.5 * (lo + hi);  // scaled
  }
  __syncthreads();
  if (tid == 0) {
    int keep = -1;
    const double s0 = L.sig[0];
    if (s0 > 0.0 && isfinite(s0) && tscale > 0.0) {
      const int nz = nT - sturm_count(L.t2, nT, cutoff * s0);
      keep = nz < kk ? nz : kk;
      if (keep < 1) keep = 1;
      double kept = 0.0;
      for (int j = 0; j < keep; ++j) {
        const double sj = L.sig[j] * tscale;
        kept += sj * sj;
      }
      L.sdisc = fmax(0.0, L.stot - kept);
    }
    L.skeep = keep;
    L.sfail = 0;
  }
  __syncthreads();
}

// Step 3: orthonormal real vectors of the bidiagonal for the kept values in
// rows 2k + off of L.Z (off = 1 when X = M'^H).  Unscales L.sig.  Returns
// false if the vectors could not be certified.
// One Cholesky QR pass on the q x keep columns Y (row k at Yb + 2 k kZS) with
// the summed Gram matrix in Gb2: G = L L^T (lower triangle), reciprocal
// diagonal in L.ldiag, then Y <- Y L^{-T}.  False if G is not numerically
// positive definite.  A separate function: its register use stays out of the
// common path of svd_vectors.
__device__ __noinline__ bool vec_cholqr(GateLds& L, double* Yb, double* Gb2, int q, int keep) {
  const int tid = threadIdx.x;
  q = uni(q);
  keep = uni(keep);
  for (int jj = 0; jj < keep; ++jj) {
    const double djj = Gb2[(long)(2 * jj) * kZS + jj];
    if (!(djj > 1e-10) || !isfinite(djj)) return false;  // the same value in every thread
    const double rinv = 1.0 / sqrt(djj);
    for (int ra = jj + 1 + tid; ra < keep; ra += blockDim.x) Gb2[(long)(2 * ra) * kZS + jj] *= rinv;
    if (tid == 0) L.ldiag[jj] = rinv;
    __syncthreads();
    const int rem = keep - jj - 1;
    for (int e = tid; e < rem * rem; e += blockDim.x) {
      const int ra = jj + 1 + e / rem, rc = jj + 1 + e % rem;
      if (rc <= ra) Gb2[(long)(2 * ra) * kZS + rc] -= Gb2[(long)(2 * ra) * kZS + jj] * Gb2[(long)(2 * rc) * kZS + jj];
    }
    __syncthreads();
  }
  {
    // row k of Y solves L x = y; thread (k, s4) holds entries s4 + 4 t
    const int k = tid >> 2, s4 = tid & 3;
    double* yr = Yb + (long)(2 * k) * kZS;
    double y[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int e = s4 + 4 * t;
      y[t] = (k < q && e < keep) ? yr[e] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < kKB; ++c) {
      if (c < keep) {
        double part = 0.0;
#pragma unroll
        for (int t = 0; t < (c + 3) / 4; ++t) {
          const int e = 4 * t + s4;
          if (e < c) part = fma(y[t], Gb2[(long)(2 * c) * kZS + e], part);
        }
        part = quad_sum(part);
        if (s4 == (c & 3)) y[c >> 2] = (y[c >> 2] - part) * L.ldiag[c];
      }
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int e = s4 + 4 * t;
      if (k < q && e < keep) yr[e] = y[t];
    }
  }
  __syncthreads();
  return true;
}

__device__ __noinline__ bool svd_vectors(GateLds& L, const SvdShape& sh, int keep) {
  keep = uni(keep);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = uni(sh.p), q = uni(sh.q), nn = uni(sh.nn);
  const bool trans = p != uni(sh.m);
  (void)tid; (void)lane; (void)wave; (void)trans; (void)p; (void)q; (void)nn;
  const int nT = 2 * q;
  const double tscale = L.sgersh;  // singular values = scaled values * tscale
  // -- vectors of T (one lane per kept value): twisted factorisation of T - s I
  // inside the block that holds s.  Column j of Z: D+ pivots, then D- pivots,
  // then the vector.  Rows 2k + off (k < q) of the vector are the bidiagonal's
  // right vector (X = M') or left vector (X = M'^H).
  const double pivmin = 2.3e-308;  // T is scaled to norm <= 1
  const int off = trans ? 1 : 0;
  double* Z = L.Z;
  if (wave == 0 && lane < keep) {
    const int j = lane;
    const double sj = L.sig[j];  // scaled
    int b0 = L.blo[0], b1 = L.bhi[0];
    if (L.snblk > 1) {
      // coincident values, which the split produces in pairs, go to distinct blocks
      const double tol = 1e-13 * L.sig[0];
      int inst = 0;
      for (int jp = 0; jp < j; ++jp) inst += fabs(L.sig[jp] - sj) <= tol ? 1 : 0;
      int seen = 0;
      bool found = false;
      for (int bk = 0; bk < L.snblk && !found; ++bk) {
        const int lo_ = L.blo[bk], n_ = L.bhi[bk] - lo_;
        const int mult = sturm_count(L.t2 + lo_, n_, sj + tol) - sturm_count(L.t2 + lo_, n_, sj - tol);
        if (mult > 0 && seen + mult > inst) {
          b0 = lo_;
          b1 = lo_ + n_;
          found = true;
        }
        seen += mult;
      }
    }
    double* zc = Z + j;  // element i at zc[i * kZS]
    if (b1 - b0 == 1) {
      zc[b0 * kZS] = 1.0;
    } else {
      // twisted factorisation T - s I = N_r Delta_r N_r^T with forward pivots
      // D+, backward pivots D- and twist r = argmin |D+_r + D-_r + s|
      // forward pivots D+
      double dd = -sj;
      zc[b0 * kZS] = dd;
      for (int i = b0 + 1; i < b1; ++i) {
        if (fabs(dd) < pivmin) dd = -pivmin;
        dd = fma(-L.t2[i - 1], rcp_nr(dd), -sj);
        zc[i * kZS] = dd;
      }
      // backward pivots D- (overwriting D+) and the twist r = argmin |D+ + D- + s|
      dd = -sj;
      int r = b1 - 1;
      double gmin = fabs(zc[(b1 - 1) * kZS]);
      zc[(b1 - 1) * kZS] = dd;
      for (int i = b1 - 2; i >= b0; --i) {
        if (fabs(dd) < pivmin) dd = -pivmin;
        dd = fma(-L.t2[i], rcp_nr(dd), -sj);
        const double g = fabs(zc[i * kZS] + dd + sj);
        if (g <= gmin) {
          gmin = g;
          r = i;
        }
        zc[i * kZS] = dd;
      }
      // forward pivots again above the twist
      dd = -sj;
      if (r > b0) zc[b0 * kZS] = dd;
      for (int i = b0 + 1; i < r; ++i) {
        if (fabs(dd) < pivmin) dd = -pivmin;
        dd = fma(-L.t2[i - 1], rcp_nr(dd), -sj);
        zc[i * kZS] = dd;
      }
      // twisted solve: z_r = 1, up with L+, down with U-
      double z = 1.0;
      for (int i = r - 1; i >= b0; --i) {
        double dpi = zc[i * kZS];
        if (fabs(dpi) < pivmin) dpi = -pivmin;
        z = -(L.t[i] * rcp_nr(dpi)) * z;
        zc[i * kZS] = z;
      }
      zc[r * kZS] = 1.0;
      z = 1.0;
      for (int i = r + 1; i < b1; ++i) {
        double dmi = zc[i * kZS];
        if (fabs(dmi) < pivmin) dmi = -pivmin;
        z = -(L.t[i - 1] * rcp_nr(dmi)) * z;
        zc[i * kZS] = z;
      }
    }
    // the rows kept (2k + off) hold half of the vector's weight in exact
    // arithmetic; normalise them directly
    double h2 = 0.0;
    for (int k = 0; k < q; ++k) {
      const int i = 2 * k + off;
      const double x = (i >= b0 && i < b1) ? zc[i * kZS] : 0.0;
      zc[i * kZS] = x;
      h2 = fma(x, x, h2);
    }
    const double inv = h2 > 0.0 ? 1.0 / sqrt(h2) : 0.0;
    for (int k = 0; k < q; ++k) zc[(2 * k + off) * kZS] *= inv;
  }
  __syncthreads();
  for (int j = tid; j < keep; j += blockDim.x) L.sig[j] *= tscale;  // unscaled singular values
  // -- orthonormalisation of Y (q x keep), Y(k, j) = Yb[2 k kZS + j].  The
  // Gram matrix G = Y^T Y lives in the interleaved rows no longer needed:
  // G(a, c) = Gb[2 a kZS + c], a second partial sum in rows 128 + 2 a.  When
  // max |G - I| <= 1e-3 the columns are refined by Newton-Schulz steps towards
  // the orthogonal polar factor, Y <- Y (3 I - G) / 2 (the error squares at
  // every step); otherwise by a Cholesky QR pass.  Stops once max |G - I| is
  // at rounding level.
  double* Yb = Z + off * kZS;
  double* Gb = Z + (1 - off) * kZS;
  double* Gb2 = Gb + 128 * kZS;
  for (int it = 0; it < 6; ++it) {
    {
      // G = Y^T Y (keep x keep) on FP64 MFMA 16x16x4 into Gb2: 16 x 16 tiles,
      // up to two per wave, K = q in steps of 4
      using Op = MfmaOps<double2>;
      const int li = lane & 15, lk = lane >> 4;
      const int nt = (keep + 15) >> 4;
      for (int t = wave; t < nt * nt; t += 8) {
        const int ti = t / nt, tj = t - ti * nt;
        const int m = 16 * ti + li, n = 16 * tj + li;
        mfma_d4 acc = mfma_d4{0, 0, 0, 0};
        for (int k0 = 0; k0 < q; k0 += 4) {
          const int k = k0 + lk;
          const double* yr = Yb + (long)(2 * k) * kZS;
          const double av = (k < q && m < keep) ? yr[m] : 0.0;  // A(m, k) = Y(k, m)
          const double bv = (k < q && n < keep) ? yr[n] : 0.0;  // B(k, n) = Y(k, n)
          acc = Op::mma(av, bv, acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * ti + Op::row(lk, r), col = 16 * tj + li;
          if (row < keep && col < keep) Gb2[(long)(2 * row) * kZS + col] = acc[r];
        }
      }
    }
    __syncthreads();
    {
      // err = max |G - I|; Gb <- 3/2 I - G/2 is kept for the refinement
      double err = 0.0;
      for (int e = tid; e < keep * keep; e += blockDim.x) {
        const int ra = e / keep, rc = e - ra * keep;
        const long o = (long)(2 * ra) * kZS + rc;
        const double g = Gb2[o];
        const double d = g - (ra == rc ? 1.0 : 0.0);
        err = fmax(err, fabs(d));
        Gb[o] = (ra == rc ? 1.0 : 0.0) - 0.5 * d;
      }
      if (!(err <= 1e300)) err = 1e300;  // NaN or Inf
      err = wave_max(err);
      if (lane == 0) L.red[wave] = err;
    }
    __syncthreads();
    double err = L.red[0];
#pragma unroll
    for (int w = 1; w < 8; ++w) err = fmax(err, L.red[w]);
    if (err >= 1e300) return false;
    if (err <= 1e-14) break;  // orthonormal to working precision
    if (err <= 1e-3) {
      // Y <- Y C, C = Gb, on FP64 MFMA: 16 x 16 tiles of the q x keep product,
      // up to four per wave, all computed before any is written
      using Op = MfmaOps<double2>;
      const int li = lane & 15, lk = lane >> 4;
      const int ntr = (q + 15) >> 4, ntc = (keep + 15) >> 4;
      mfma_d4 acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        acc[c] = mfma_d4{0, 0, 0, 0};
        const int t = wave + 8 * c;
        if (t < ntr * ntc) {
          const int ti = t / ntc, tj = t - ti * ntc;
          const int i = 16 * ti + li, n = 16 * tj + li;
          for (int e0 = 0; e0 < keep; e0 += 4) {
            const int e = e0 + lk;
            const double av = (i < q && e < keep) ? Yb[(long)(2 * i) * kZS + e] : 0.0;     // A(i, e) = Y(i, e)
            const double bv = (e < keep && n < keep) ? Gb[(long)(2 * e) * kZS + n] : 0.0;  // B(e, n) = C(e, n)
            acc[c] = Op::mma(av, bv, acc[c]);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int t = wave + 8 * c;
        if (t < ntr * ntc) {
          const int ti = t / ntc, tj = t - ti * ntc;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * ti + Op::row(lk, r), col = 16 * tj + li;
            if (row < q && col < keep) Yb[(long)(2 * row) * kZS + col] = acc[c][r];
          }
        }
      }
      __syncthreads();
      // ||I - G||_2 <= keep * err; one step leaves about 0.75 (keep err)^2
      if (err * keep <= 1e-7) break;
      continue;
    }
    if (!vec_cholqr(L, Yb, Gb2, q, keep)) return false;
    __syncthreads();
  }
  return true;
}

// Step 4: kept rows of W^H into v.W (keep x nn).  W (nn x keep, complex) =
// the bidiagonal's vectors times the phases, then through the reflectors in
// blocks of 16 (compact WY, reflectors H = I - u u^H with |u|^2 = 2, tau = 1):
// H_k1 H_k1+1 ... H_k1+15 = I - V T V^H, T upper triangular with unit
// diagonal, T(0:c, c) = -T(0:c, 0:c) (V^H V)(0:c, c); W <- W - V (T (V^H W)).
// The products run on FP64 MFMA 16x16x4.  W stays in registers in the MFMA
// output layout: wave w holds columns 16 (w % 4) .. + 15 and rows
// 64 (w / 4) .. + 63 as four 16 x 16 tiles, lane l and register r of tile t
// holding row 64 (w / 4) + 16 t + l / 16 + 4 r, column 16 (w % 4) + l % 16.
// That is the layout of the B operand of a 16x16x4 product whose k-block is
// the tile's rows 4 r .. 4 r + 3, so V^H W and V Z take W and Z straight
// from registers.  Reflector k (row k of v.H, stride ws) is read from the
// workspace and masked to its support [st_k, st_k + len_k).
__device__ __noinline__ void svd_back(const SlotView& v, GateLds& L, const SvdShape& sh, int keep) {
  using Op = MfmaOps<double2>;
  using Acc = mfma_d4;
  keep = uni(keep);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = uni(sh.p), q = uni(sh.q), nn = uni(sh.nn);
  const bool trans = p != uni(sh.m);
  const int ws = uni(sh.ws);
  const double2* Hg = v.H;
  const int off = trans ? 1 : 0;
  const double* Yb = L.Z + off * kZS;
  const int ct = wave & 3, rh = wave >> 2;
  const int li = lane & 15, lk = lane >> 4;
  const int kstart = trans ? q - 1 : q - 2;  // last reflector
  // reflector k: support start and length (zero beyond kstart)
  auto refl = [&](int k, int i) -> double2 {
    if (k > kstart) return cmk(0.0, 0.0);
    const int st = trans ? k : k + 1, len = trans ? p - k : q - k - 1;
    return (i >= st && i < st + len) ? Hg[(long)k * ws + i] : cmk(0.0, 0.0);
  };
  // -- W = phases * bidiagonal vectors
  Acc wre[4], wim[4];
  {
    const double2* phase = trans ? L.pa : L.pb;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pos = 64 * rh + 16 * t + lk + 4 * r, j = 16 * ct + li;
        double2 x = cmk(0.0, 0.0);
        if (j < keep && pos < q) x = cscale(phase[pos], Yb[(long)(2 * pos) * kZS + j]);
        wre[t][r] = x.x;
        wim[t][r] = x.y;
      }
  }
  __syncthreads();  // Yb is read; L.Z becomes scratch
  double2* Tb = reinterpret_cast<double2*>(L.Z);  // [8][16][16]: T of block b (reflectors 16 b ..)
  double2* Vb = Tb + 8 * 256;                     // [2][16][128]: V of a block, V(i, n) at n * 128 + i
  double2* Sp = Vb + 2 * 16 * 128;                // [2][16][64]: partial V^H W by row half
  if (kstart < 0) goto store;
  {
    const int nblk = kstart / 16 + 1;  // <= 8
    // -- T of every block, wave w for block w: G = V^H V on MFMA (rows from the
    // block's first support row), then row n of T in lane n:
    // T(n, c) = -sum_{n <= m < c} T(n, m) G(m, c)
    if (wave < nblk) {
      const int k1 = 16 * wave, st1 = trans ? k1 : k1 + 1;
      Acc gr = Acc{0, 0, 0, 0}, gi = Acc{0, 0, 0, 0};
      for (int i0 = (st1 / 4) * 4; i0 < p; i0 += 4) {
        const double2 u = refl(k1 + li, i0 + lk);  // A = conj(V)(li, i), B = V(i, li): the same element
        gr = Op::mma(u.x, u.x, gr);
        gr = Op::mma(u.y, u.y, gr);   // Re conj(a) b = ar br + ai bi
        gi = Op::mma(u.x, u.y, gi);
        gi = Op::mma(-u.y, u.x, gi);  // Im conj(a) b = ar bi - ai br
      }
      double2* Tw = Tb + wave * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) Tw[(lk + 4 * r) * 16 + li] = cmk(gr[r], gi[r]);  // G for now
      wave_sync();
      double2 trow[16];
      const int n = li;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        double2 acc = cmk(0.0, 0.0);
#pragma unroll
        for (int m = 0; m < c; ++m)
          if (m >= n) cfma(acc, trow[m], Tw[m * 16 + c]);
        trow[c] = c < n ? cmk(0.0, 0.0) : (c == n ? cmk(1.0, 0.0) : cmk(-acc.x, -acc.y));
      }
      wave_sync();
      if (lane < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) Tw[n * 16 + c] = trow[c];
      }
    }
    // -- V of block b goes to Vb[b & 1]; each thread stages 4 entries per block
    auto vload = [&](int k1, double2 (&nv)[4]) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int idx = tid + 512 * e, n = idx >> 7, i = idx & 127;
        nv[e] = refl(k1 + n, i);
      }
    };
    double2 nv[4];
    vload(16 * (nblk - 1), nv);
#pragma unroll
    for (int e = 0; e < 4; ++e) Vb[((nblk - 1) & 1) * 2048 + tid + 512 * e] = nv[e];
    // a wave whose 16 columns are all at or beyond keep has W = 0 there, and
    // it stays 0: it skips its products (no other wave reads its S rows)
    const bool colact = 16 * ct < keep;
    for (int b = nblk - 1; b >= 0; --b) {
      const int k1 = 16 * b, st1 = trans ? k1 : k1 + 1;
      const double2* V = Vb + (b & 1) * 2048;
      const double2* T = Tb + b * 256;
      __syncthreads();  // V of this block (and every T) staged; the previous block's Sp reads are done
      if (b > 0) vload(k1 - 16, nv);  // next block's V, in flight during this one
      // -- partial S = V^H W over this wave's rows, for its 16 columns
      if (colact) {
        Acc sr = Acc{0, 0, 0, 0}, si = Acc{0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          // the same for the whole wave: rows before the block's support, or
          // at or beyond p (V and W are zero there)
          if (64 * rh + 16 * t + 15 < st1 || 64 * rh + 16 * t >= p) continue;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 64 * rh + 16 * t + 4 * r + lk;
            const double2 u = V[li * 128 + i];  // A(li, i) = conj(V(i, li))
            sr = Op::mma(u.x, wre[t][r], sr);
            sr = Op::mma(u.y, wim[t][r], sr);   // Re conj(u) w = ur wr + ui wi
            si = Op::mma(u.x, wim[t][r], si);
            si = Op::mma(-u.y, wre[t][r], si);  // Im conj(u) w = ur wi - ui wr
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) Sp[rh * 1024 + (lk + 4 * r) * 64 + 16 * ct + li] = cmk(sr[r], si[r]);
      }
      __syncthreads();
      // -- Z = T S for this wave's columns (both row halves compute it), then W -= V Z
      if (colact) {
        Acc zr = Acc{0, 0, 0, 0}, zi = Acc{0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int m = 4 * s4 + lk;
          const double2 a = T[li * 16 + m];
          const double2 bs = cadd(Sp[m * 64 + 16 * ct + li], Sp[1024 + m * 64 + 16 * ct + li]);
          zr = Op::mma(a.x, bs.x, zr);
          zr = Op::mma(-a.y, bs.y, zr);
          zi = Op::mma(a.x, bs.y, zi);
          zi = Op::mma(a.y, bs.x, zi);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (64 * rh + 16 * t + 15 < st1 || 64 * rh + 16 * t >= p) continue;
          const int i = 64 * rh + 16 * t + li;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double2 u = V[(4 * r + lk) * 128 + i];  // A(i, n) = -V(i, n), n = 4 r + lk; B = Z register r
            wre[t] = Op::mma(-u.x, zr[r], wre[t]);
            wre[t] = Op::mma(u.y, zi[r], wre[t]);
            wim[t] = Op::mma(-u.x, zi[r], wim[t]);
            wim[t] = Op::mma(-u.y, zr[r], wim[t]);
          }
        }
      }
      if (b > 0) {
        double2* Vn = Vb + ((b - 1) & 1) * 2048;  // last read two blocks ago
#pragma unroll
        for (int e = 0; e < 4; ++e) Vn[tid + 512 * e] = nv[e];
      }
    }
  }
store:
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pos = 64 * rh + 16 * t + lk + 4 * r, j = 16 * ct + li;
      if (j < keep && pos < nn) v.W[(long)j * nn + pos] = cmk(wre[t][r], -wim[t][r]);  // rows of W^H
    }
  __syncthreads();
}

__device__ int svd_bisect(SlotView& v, GateLds& L, int m, int nn, int D, double cutoff, int ws, long long* tcyc) {
  const SvdShape sh = svd_shape(m, nn, D, cutoff, ws);
  svd_bidiag(v, L, sh);
  tcyc[0] = clock64();
  svd_values(L, sh);
  tcyc[1] = clock64();
  const int keep = uni(L.skeep);
  if (keep < 0) return -1;
  if (!svd_vectors(L, sh, keep)) return -1;
  tcyc[2] = clock64();
  svd_back(v, L, sh, keep);
  return keep;
}

// ---- Phase B (fallback): LQ + QR preconditioning and one-sided row Jacobi.
// Same outputs as svd_bisect.  *sweeps_out / *conv_out report convergence.
template <int kMaxPerLane>  // Jacobi row length <= 64 * kMaxPerLane
__device__ int svd_jacobi(const DevBatch& b, SlotView& v, GateLds& L, int m, int nn, SvdParams sp, int* sweeps_out,
                          bool* conv_out, long long* tcyc) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  const int r = m < nn ? m : nn;
  // LQ: A <- A H_0 H_1 ... (reflectors on rows, stored in H)
  for (int k = 0; k < r; ++k) {
    if (wave == 0) {
      bool z;
      wave_householder(v.A + (long)k * nn + k, nn - k, true, v.H + (long)k * nn + k, &L.sbeta, &z);
      if (lane == 0) L.szero = z;
    }
    __syncthreads();
    if (!L.szero) {
      for (int a = k + 1 + wave; a < m; a += nwaves) {
        double2* row = v.A + (long)a * nn;
        const double2* u = v.H + (long)k * nn;
        double wr = 0.0, wi = 0.0;
        for (int j = k + lane; j < nn; j += 64) {
          const double2 pr = cmul(row[j], u[j]);
          wr += pr.x;
          wi += pr.y;
        }
        const double2 w = cmk(wave_sum(wr), wave_sum(wi));
        for (int j = k + lane; j < nn; j += 64) row[j] = csub(row[j], cmul(w, cconj(u[j])));
      }
    }
    for (int j = k + tid; j < nn; j += blockDim.x) v.A[(long)k * nn + j] = j == k ? L.sbeta : cmk(0.0, 0.0);
    __syncthreads();
  }
  // QR of the m x r lower-trapezoidal L (reflectors on columns)
  for (int k = 0; k < r; ++k) {
    const int Lc = m - k;
    for (int i = tid; i < Lc; i += blockDim.x) L.uq[i] = v.A[(long)(k + i) * nn + k];
    __syncthreads();
    if (wave == 0) {
      bool z;
      wave_householder(L.uq, Lc, false, L.uq, &L.sbeta, &z);
      if (lane == 0) L.szero = z;
    }
    __syncthreads();
    if (!L.szero) {
      for (int c = k + 1 + wave; c < r; c += nwaves) {
        double wr = 0.0, wi = 0.0;
        for (int i = lane; i < Lc; i += 64) {
          const double2 pr = cmul(cconj(L.uq[i]), v.A[(long)(k + i) * nn + c]);
          wr += pr.x;
          wi += pr.y;
        }
        const double2 w = cmk(wave_sum(wr), wave_sum(wi));
        for (int i = lane; i < Lc; i += 64) {
          double2* e = &v.A[(long)(k + i) * nn + c];
          *e = csub(*e, cmul(L.uq[i], w));
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < Lc; i += blockDim.x) v.A[(long)(k + i) * nn + k] = i == 0 ? L.sbeta : cmk(0.0, 0.0);
    __syncthreads();
  }
  tcyc[0] = clock64();
  // one-sided Jacobi on the rows of the r x r upper triangle
  int sweeps = 0;
  bool converged = r < 2;
  if (r >= 2) {
    const int Pe = r + (r & 1);
    for (int sw = 0; sw < sp.max_sweeps; ++sw) {
      if (tid == 0) L.srot = 0;
      __syncthreads();
      for (int t = 0; t < Pe - 1; ++t) {
        for (int kp = wave; kp < Pe / 2; kp += nwaves) {
          const int pr_ = rr_row(kp, t, Pe), qr_ = rr_row(Pe - 1 - kp, t, Pe);
          if (pr_ >= r || qr_ >= r) continue;
          double2* rp = v.A + (long)pr_ * nn;
          double2* rq = v.A + (long)qr_ * nn;
          double2 xp[kMaxPerLane], xq[kMaxPerLane];
          double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
          for (int e = 0; e < kMaxPerLane; ++e) {
            const int j = lane + 64 * e;
            if (j < r) {
              xp[e] = rp[j];
              xq[e] = rq[j];
            } else {
              xp[e] = cmk(0.0, 0.0);
              xq[e] = cmk(0.0, 0.0);
            }
            al += cabs2(xp[e]);
            be += cabs2(xq[e]);
            gr += xp[e].x * xq[e].x + xp[e].y * xq[e].y;
            gi += xp[e].y * xq[e].x - xp[e].x * xq[e].y;
          }
          al = wave_sum(al);
          be = wave_sum(be);
          gr = wave_sum(gr);
          gi = wave_sum(gi);
          const double ag = sqrt(gr * gr + gi * gi);
          if (!(al > 0.0 && be > 0.0) || !(ag > sp.tol * sqrt(al) * sqrt(be))) continue;
          const double zeta = (be - al) / (2.0 * ag);
          double tt;
          if (fabs(zeta) > 1e150)
            tt = 0.5 / zeta;
          else
            tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
          const double2 s_ip = cscale(cmk(gr / ag, gi / ag), sn);
          const double2 s_im = cconj(s_ip);
#pragma unroll
          for (int e = 0; e < kMaxPerLane; ++e) {
            const int j = lane + 64 * e;
            if (j < r) {
              rp[j] = csub(cscale(xp[e], cs), cmul(s_ip, xq[e]));
              rq[j] = cadd(cmul(s_im, xp[e]), cscale(xq[e], cs));
            }
          }
          if (lane == 0) L.srot = 1;
        }
        __syncthreads();
      }
      sweeps = sw + 1;
      const int any = L.srot;
      __syncthreads();
      if (!any) {
        converged = true;
        break;
      }
    }
  }
  *sweeps_out = sweeps;
  *conv_out = converged;
  tcyc[1] = clock64();
  // back-transform rows: [F, 0] H_{r-1} ... H_0 -> s_k w_k^H; row norms
  for (int a = wave; a < r; a += nwaves) {
    double2* row = v.A + (long)a * nn;
    for (int j = r + lane; j < nn; j += 64) row[j] = cmk(0.0, 0.0);
    for (int k = r - 1; k >= 0; --k) {
      const double2* u = v.H + (long)k * nn;
      double wr = 0.0, wi = 0.0;
      for (int j = k + lane; j < nn; j += 64) {
        const double2 pr = cmul(row[j], u[j]);
        wr += pr.x;
        wi += pr.y;
      }
      const double2 w = cmk(wave_sum(wr), wave_sum(wi));
      for (int j = k + lane; j < nn; j += 64) row[j] = csub(row[j], cmul(w, cconj(u[j])));
    }
    double s2 = 0.0;
    for (int j = lane; j < nn; j += 64) s2 += cabs2(row[j]);
    s2 = wave_sum(s2);
    if (lane == 0) v.S[a] = sqrt(s2);
  }
  __syncthreads();
  tcyc[2] = clock64();
  // sort descending (ties by index), truncate, normalised rows -> W
  for (int a = tid; a < r; a += blockDim.x) {
    const double sa = v.S[a];
    int rank = 0;
    for (int qq = 0; qq < r; ++qq) {
      const double sq = v.S[qq];
      rank += (sq > sa || (sq == sa && qq < a)) ? 1 : 0;
    }
    v.P[rank] = a;
  }
  __syncthreads();
  if (tid == 0) {
    int keep = -1;
    const double s1 = v.S[v.P[0]];
    if (s1 > 0.0 && isfinite(s1)) {
      int nz = 0;
      for (int qq = 0; qq < r; ++qq) nz += v.S[qq] > sp.cutoff_rel * s1 ? 1 : 0;
      keep = nz < b.max_bond ? nz : b.max_bond;
      double disc = 0.0;
      for (int qq = keep; qq < r; ++qq) {
        const double s = v.S[v.P[qq]];
        disc += s * s;
      }
      L.sdisc = disc;
      for (int qq = 0; qq < keep; ++qq) L.sig[qq] = v.S[v.P[qq]];
    }
    L.skeep = keep;
  }
  __syncthreads();
  const int keep = L.skeep;
  for (int idx = tid; keep > 0 && idx < keep * nn; idx += blockDim.x) {
    const int k = idx / nn, col = idx - k * nn;
    const int src = v.P[k];
    v.W[idx] = cscale(v.A[(long)src * nn + col], 1.0 / v.S[src]);
  }
  __syncthreads();
  return keep;
}

// kSmall: every bond <= 64 (two-site matrices <= 128 x 128): bisection SVD
// with a compact Jacobi fallback.  Otherwise: Jacobi with rows up to 512.
template <bool kSmall, typename S>
__global__ __launch_bounds__(kBlock) void k_gates(DevBatch b, const int* __restrict__ gsite,
                                                  const int* __restrict__ grot, const double2* __restrict__ gpre,
                                                  const double2* __restrict__ gpost, const double* __restrict__ phi_all,
                                                  int n_rot, int g0, int g1, SvdParams sp) {
  __shared__ GateLds L;
  const int slot = b.slot0 + blockIdx.x;
  const int tid = threadIdx.x;
  SlotView v = slot_view(b, slot);
  const double* phi = phi_all ? phi_all + (long)slot * n_rot : nullptr;
  if (b.cursor) {
    // per-slot progress: up to g1 - g0 gates from the slot's cursor
    const int c = b.cursor[slot];
    g1 = min(c + (g1 - g0), b.n_gates);
    g0 = c;
  }
  if (tid == 0) L.sabort = (*v.flags & kFlagNumeric) ? 1 : 0;
  __syncthreads();
  if (L.sabort || g0 >= g1) return;

  for (int g = g0; g < g1; ++g) {
    const int n = gsite[g];
    const int rot = grot[g];
    if (tid < 16) {
      if (rot < 0) {
        L.O[tid] = gpre[(long)g * 16 + tid];
      } else {
        const double ph = phi[rot];
        const double2 dm = cmk(cos(0.5 * ph), -sin(0.5 * ph));  // exp(-i phi/2)
        const double2 dp = cmk(cos(0.5 * ph), sin(0.5 * ph));   // exp(+i phi/2)
        const int i = tid >> 2, j = tid & 3;
        double2 s = cmk(0.0, 0.0);
        for (int k = 0; k < 4; ++k) {
          const double2 d = (k & 1) ? dp : dm;
          cfma(s, cmul(gpost[(long)g * 16 + i * 4 + k], d), gpre[(long)g * 16 + k * 4 + j]);
        }
        L.O[tid] = s;
      }
    }
    const int chil = v.chi[n], chim = v.chi[n + 1], chir = v.chi[n + 2];
    const int m = 2 * chil, nn = 2 * chir;
    const int qmin = m < nn ? m : nn;
    __syncthreads();
    long long tc[8];
    tc[0] = clock64();
    gate_contract<S>(b, v, L, n, chil, chim, chir);
    tc[1] = clock64();

    int keep = -1, sweeps = 0;
    bool conv = true, used_bisect = false, fell_back = false;
    long long tb[3] = {tc[1], tc[1], tc[1]};
    if (kSmall && sp.algo == 0 && qmin <= kQB) {
      used_bisect = true;
      keep = svd_bisect(v, L, m, nn, b.max_bond, sp.cutoff_rel, b.ws, tb);
      if (keep < 0) {
        fell_back = true;
        restore_mprime<S>(b, v, n, chil, chir);
      }
    }
    if (keep < 0) keep = svd_jacobi<kSmall ? 2 : 8>(b, v, L, m, nn, sp, &sweeps, &conv, tb);
    tc[2] = tb[0];
    tc[3] = tb[1];
    tc[4] = tb[2];
    tc[5] = clock64();
    if (tid == 0 && keep < 1) {
      *v.flags |= kFlagNumeric;
      L.sabort = 1;
    }
    __syncthreads();
    if (L.sabort) return;

    // ---- Phase C: truncate (Eq. 9), update (Eq. 10)
    const int capl_r = b.cap[n + 1], capr_r = b.cap[n + 2];
    S* Bn = reinterpret_cast<S*>(v.sites) + b.site_off[n];
    S* Bn1 = reinterpret_cast<S*>(v.sites) + b.site_off[n + 1];
    if (tid == 0) {
      double kept = 0.0;
      for (int k = 0; k < keep; ++k) kept += L.sig[k] * L.sig[k];
      const double d = L.sdisc / (kept + L.sdisc);
      L.snorm = sqrt(kept);
      v.stats[kStatDisc] += d;
      if (d > v.stats[kStatMaxDisc]) v.stats[kStatMaxDisc] = d;
      if (keep > v.stats[kStatMaxChi]) v.stats[kStatMaxChi] = keep;
      if (sweeps > v.stats[kStatSweeps]) v.stats[kStatSweeps] = sweeps;
      v.stats[kStatSweepSum] += sweeps;
      if (fell_back) v.stats[kStatFallbacks] += 1.0;
      if (used_bisect && !fell_back) v.stats[kStatBisect] += 1.0;
      if (!conv) *v.flags |= kFlagNoConv;
      const double cl = chil, cmd = chim, cr = chir;
      const double mm = m > nn ? m : nn, nm = qmin;
      v.stats[kStatFlops] += 32.0 * cl * cmd * cr + 128.0 * cl * cr + 4.0 * (4.0 * mm * nm * nm + 8.0 * nm * nm * nm) +
                             8.0 * double(m) * double(nn) * keep;
    }
    __syncthreads();
    const double nrm = L.snorm;
    // B_{n+1} = kept rows of W^H (Eq. 10); lambda_n = S_kept / ||S_kept||
    for (int idx = tid; idx < keep * nn; idx += blockDim.x) {
      const int k = idx / nn, col = idx - k * nn;
      const int jj = col / chir, c = col - jj * chir;
      Bn1[(long)(2 * k + jj) * capr_r + c] = cfrom<S>(v.W[idx]);
    }
    for (int k = tid; k < keep; k += blockDim.x) v.lam[b.lam_off[n] + k] = L.sig[k] / nrm;
    __syncthreads();
    // B_n = M W / ||S_kept||  (Eq. 10: no division by Schmidt values)
    if constexpr (sizeof(S) == sizeof(double2)) {
      zgemm_mfma<false, true, S, 4>(m, keep, nn, reinterpret_cast<const S*>(v.M), nn, reinterpret_cast<const S*>(v.W),
                                    nn, Bn, capl_r, cval<S>(1.0 / nrm, 0.0), false);
    } else {
      // mixed path: the kept rows of W^H rounded to complex64 (reflector scratch), then M W in FP32
      S* Wf = reinterpret_cast<S*>(v.H);
      for (int idx = tid; idx < keep * nn; idx += blockDim.x) Wf[idx] = cfrom<S>(v.W[idx]);
      __syncthreads();
      zgemm_mfma<false, true, S, 4>(m, keep, nn, reinterpret_cast<const S*>(v.M), nn, Wf, nn, Bn, capl_r,
                                    cval<S>(1.0 / nrm, 0.0), false);
    }
    if (tid == 0) {
      v.chi[n + 1] = keep;
      const long long te = clock64();
      v.stats[kStatCycContract] += double(tc[1] - tc[0]);
      v.stats[kStatCycLQ] += double(tc[2] - tc[1]);
      v.stats[kStatCycQR] += double(tc[3] - tc[2]);
      v.stats[kStatCycJacobi] += double(tc[4] - tc[3]);
      v.stats[kStatCycBack] += double(tc[5] - tc[4]);
      v.stats[kStatCycUpdate] += double(te - tc[5]);
    }
    __syncthreads();
  }
  if (b.cursor && tid == 0) b.cursor[slot] = g1;
}

// ----------------------------------------------------------- environments --

// L[0] = 1; L[k+1] = sum_i B_i^H L[k] B_i.   Rt[N] = 1; Rt[k] = sum_i B_i Rt[k+1] B_i^H.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_envs(DevBatch b) {
  __shared__ S lds_gemm[2 * 64 * 8];
  const int slot = b.slot0 + blockIdx.x;
  const int N = b.n_qubits;
  SlotView v = slot_view(b, slot);
  S* L = reinterpret_cast<S*>(b.envL + slot * b.env_stride);
  S* R = reinterpret_cast<S*>(b.envR + slot * b.env_stride);
  S* X = reinterpret_cast<S*>(v.M);  // scratch
  if (threadIdx.x == 0) {
    L[b.env_off[0]] = cval<S>(1.0, 0.0);
    R[b.env_off[N]] = cval<S>(1.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    const int cl = v.chi[k], cr = v.chi[k + 1];
    const int capl = b.cap[k], capr = b.cap[k + 1];
    const S* Bk = reinterpret_cast<const S*>(v.sites) + b.site_off[k];
    for (int i = 0; i < 2; ++i) {
      bgemm<false, false, S>(cl, cr, cl, L + b.env_off[k], capl, Bk + i * capr, 2 * capr, X, cr, cval<S>(1.0, 0.0),
                          false, lds_gemm);
      bgemm<true, false, S>(cr, cr, cl, Bk + i * capr, 2 * capr, X, cr, L + b.env_off[k + 1], capr,
                         cval<S>(1.0, 0.0), i == 1, lds_gemm);
    }
  }
  for (int k = N - 1; k >= 0; --k) {
    const int cl = v.chi[k], cr = v.chi[k + 1];
    const int capl = b.cap[k], capr = b.cap[k + 1];
    const S* Bk = reinterpret_cast<const S*>(v.sites) + b.site_off[k];
    for (int i = 0; i < 2; ++i) {
      bgemm<false, false, S>(cl, cr, cr, Bk + i * capr, 2 * capr, R + b.env_off[k + 1], capr, X, cr, cval<S>(1.0, 0.0),
                          false, lds_gemm);
      bgemm<false, true, S>(cl, cl, cr, X, cr, Bk + i * capr, 2 * capr, R + b.env_off[k], capl, cval<S>(1.0, 0.0),
                         i == 1, lds_gemm);
    }
  }
  if (threadIdx.x == 0) v.stats[kStatNorm] = double(L[b.env_off[N]].x);
}

// --------------------------------------------------------- Pauli sweeps ---

// Transfer sweeps of the Pauli strings (Eq. 2 by exact contraction).  The
// strings are visited in a prefix order (lowest non-identity site, then the
// letters site by site): string t shares its first share[t] transfer steps
// with string t - 1, so a workgroup walking a contiguous run of the order
// keeps a stack of partial left transfers and recomputes only the rest (the
// prefix trie of the strings, one node per transfer step).  Without order,
// strings go in their own order with no reuse.
template <typename S, int BM, int BN, int BK>
__global__ __launch_bounds__(kBlock) void k_pauli(DevBatch b, const uint64_t* __restrict__ sx,
                                                  const uint64_t* __restrict__ sz, int n_strings,
                                                  const int* __restrict__ order, const int* __restrict__ share,
                                                  double2* scratch, int cm, double* ev_re, double* ev_im) {
  __shared__ S lds_gemm[(BM + BN) * BK];
  __shared__ double red[kBlock / 64];
  const int r = blockIdx.y, slot = b.slot0 + r;  // outputs and scratch are indexed from the first slot
  const int N = b.n_qubits;
  SlotView v = slot_view(b, slot);
  const S* L = reinterpret_cast<const S*>(b.envL + slot * b.env_stride);
  const S* R = reinterpret_cast<const S*>(b.envR + slot * b.env_stride);
  const long mat = (long)cm * cm;
  // per workgroup: X, then the stack of transfers after 1 .. N sites
  S* X = reinterpret_cast<S*>(scratch) + ((long)r * gridDim.x + blockIdx.x) * (N + 2) * mat;
  S* stk = X + mat;  // transfer after d sites at stk + (d - 1) * mat
  const double nrm = double(L[b.env_off[N]].x);
  const int per = (n_strings + gridDim.x - 1) / gridDim.x;
  const int t0 = blockIdx.x * per, t1 = min(n_strings, t0 + per);
  for (int t = t0; t < t1; ++t) {
    const int s = order ? order[t] : t;
    const uint64_t x = sx[s], z = sz[s];
    const uint64_t mk = x | z;
    double2 ev = cmk(0.0, 0.0);
    if (mk == 0) {
      ev = cmk(1.0, 0.0);
    } else {
      const int lo = __builtin_ctzll(mk), hi = 63 - __builtin_clzll(mk);
      const int d0 = (t == t0 || !share) ? 0 : share[t];
      for (int d = d0; d <= hi - lo; ++d) {
        const int k = lo + d;
        const S* T = d == 0 ? L + b.env_off[lo] : stk + (long)(d - 1) * mat;
        const int ldt = d == 0 ? b.cap[lo] : cm;
        S* Tn = stk + (long)d * mat;
        const int cl = v.chi[k], cr = v.chi[k + 1];
        const int capr = b.cap[k + 1];
        const S* Bk = reinterpret_cast<const S*>(v.sites) + b.site_off[k];
        const int xb = (x >> k) & 1, zb = (z >> k) & 1;
        for (int i = 0; i < 2; ++i) {
          const int ip = xb ? 1 - i : i;
          S ph = cval<S>(1.0, 0.0);
          if (zb && !xb) ph = cval<S>(i == 0 ? 1.0 : -1.0, 0.0);  // Z
          if (zb && xb) ph = cval<S>(0.0, i == 0 ? -1.0 : 1.0);   // Y: <0|Y|1> = -i
          bgemm_tiled<false, false, S, BM, BN, BK>(cl, cr, cl, T, ldt, Bk + ip * capr, 2 * capr, X, cm,
                                                   cval<S>(1.0, 0.0), false, lds_gemm);
          bgemm_tiled<true, false, S, BM, BN, BK>(cr, cr, cl, Bk + i * capr, 2 * capr, X, cm, Tn, cm, ph, i == 1,
                                                  lds_gemm);
        }
      }
      // <P> = sum_{c,c'} T[c][c'] R[c][c'],  R[c][c'] = Rt[c'][c]
      const S* T = stk + (long)(hi - lo) * mat;
      const int ch = v.chi[hi + 1];
      const S* Rh = R + b.env_off[hi + 1];
      const int ldr = b.cap[hi + 1];
      double pr = 0.0, pi = 0.0;
      for (int idx = threadIdx.x; idx < ch * ch; idx += blockDim.x) {
        const int a = idx / ch, c = idx - a * ch;
        const double2 p = cmul(c64(T[(long)a * cm + c]), c64(Rh[(long)c * ldr + a]));
        pr += p.x;
        pi += p.y;
      }
      pr = block_sum(pr, red);
      pi = block_sum(pi, red);
      ev = cmk(pr / nrm, pi / nrm);
    }
    if (threadIdx.x == 0) {
      ev_re[(long)r * n_strings + s] = ev.x;
      ev_im[(long)r * n_strings + s] = ev.y;
    }
    __syncthreads();
  }
}

// Neumaier-compensated sum in term order, identity coefficient last.
__global__ void k_energy_reduce(const double* coeff, const double* ev_re, const double* ev_im, int n_strings,
                                double c_identity, double* energy, double* stats, int slot0) {
  const int r = blockIdx.x, slot = slot0 + r;  // inputs and energy indexed from the first slot
  if (threadIdx.x != 0) return;
  double s = 0.0, comp = 0.0, mi = 0.0;
  auto add = [&](double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x))
      comp += (s - t) + x;
    else
      comp += (x - t) + s;
    s = t;
  };
  for (int i = 0; i < n_strings; ++i) {
    add(coeff[i] * ev_re[(long)r * n_strings + i]);
    mi = fmax(mi, fabs(ev_im[(long)r * n_strings + i]));
  }
  add(c_identity);
  energy[r] = s + comp;
  stats[slot * kNStats + kStatMaxImag] = mi;
}

// --------------------------------------------------------------- launchers --

hipError_t launch_init_product(const DevBatch& b, const uint8_t* d_occ, hipStream_t st) {
  if (b.mixed)
    hipLaunchKernelGGL(k_init_product<float2>, dim3(b.n_slots), dim3(64), 0, st, b, d_occ);
  else
    hipLaunchKernelGGL(k_init_product<double2>, dim3(b.n_slots), dim3(64), 0, st, b, d_occ);
  return hipGetLastError();
}

hipError_t launch_copy_slots(const DevBatch& src, const DevBatch& dst, const int2* d_pairs, int n_pairs, int2 one,
                             bool clear_work, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_slots, dim3(d_pairs ? n_pairs : 1), dim3(256), 0, st, src, dst, d_pairs, one,
                     clear_work ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_angles(const DevBatch& b, const DevProblem& p, const double* d_theta, int n_theta,
                         const int* d_shift_rot, const double* d_shift_val, hipStream_t st) {
  if (p.n_rot == 0) return hipSuccess;
  dim3 grid((p.n_rot + 255) / 256, b.n_slots);
  hipLaunchKernelGGL(k_angles, grid, dim3(256), 0, st, b.phi, p.n_rot, p.rot_c, p.rot_param, d_theta, n_theta,
                     d_shift_rot, d_shift_val, b.slot0);
  return hipGetLastError();
}

hipError_t launch_gates(const DevBatch& b, const int* d_site, const int* d_rot, const double2* d_pre,
                        const double2* d_post, int g0, int g1, int n_rot, SvdParams sp, hipStream_t st) {
  if (g1 <= g0) return hipSuccess;
  int cm = 1;
  for (int i = 0; i <= b.n_qubits; ++i) cm = cm > b.cap[i] ? cm : b.cap[i];
  const dim3 grid(b.n_slots), block(kBlock);
  if (cm <= kKB && !b.mixed)
    hipLaunchKernelGGL((k_gates<true, double2>), grid, block, 0, st, b, d_site, d_rot, d_pre, d_post, b.phi, n_rot, g0,
                       g1, sp);
  else if (cm <= kKB)
    hipLaunchKernelGGL((k_gates<true, float2>), grid, block, 0, st, b, d_site, d_rot, d_pre, d_post, b.phi, n_rot, g0,
                       g1, sp);
  else if (!b.mixed)
    hipLaunchKernelGGL((k_gates<false, double2>), grid, block, 0, st, b, d_site, d_rot, d_pre, d_post, b.phi, n_rot,
                       g0, g1, sp);
  else
    hipLaunchKernelGGL((k_gates<false, float2>), grid, block, 0, st, b, d_site, d_rot, d_pre, d_post, b.phi, n_rot,
                       g0, g1, sp);
  return hipGetLastError();
}

hipError_t launch_envs(const DevBatch& b, hipStream_t st) {
  if (b.mixed)
    hipLaunchKernelGGL(k_envs<float2>, dim3(b.n_slots), dim3(kBlock), 0, st, b);
  else
    hipLaunchKernelGGL(k_envs<double2>, dim3(b.n_slots), dim3(kBlock), 0, st, b);
  return hipGetLastError();
}

template <typename S>
static void launch_pauli_t(int tile, dim3 grid, hipStream_t st, const DevBatch& b, const uint64_t* d_x,
                           const uint64_t* d_z, int n_strings, const int* d_order, const int* d_share,
                           double2* d_scratch, int cm, double* d_ev_re, double* d_ev_im) {
  switch (tile) {
    case 1:
      hipLaunchKernelGGL((k_pauli<S, 64, 64, 16>), grid, dim3(kBlock), 0, st, b, d_x, d_z, n_strings, d_order,
                         d_share, d_scratch, cm, d_ev_re, d_ev_im);
      break;
    case 2:
      hipLaunchKernelGGL((k_pauli<S, 32, 32, 16>), grid, dim3(kBlock), 0, st, b, d_x, d_z, n_strings, d_order,
                         d_share, d_scratch, cm, d_ev_re, d_ev_im);
      break;
    default:
      hipLaunchKernelGGL((k_pauli<S, 64, 64, 8>), grid, dim3(kBlock), 0, st, b, d_x, d_z, n_strings, d_order,
                         d_share, d_scratch, cm, d_ev_re, d_ev_im);
  }
}

hipError_t launch_pauli(const DevBatch& b, const uint64_t* d_x, const uint64_t* d_z, int n_strings, const int* d_order,
                        const int* d_share, double2* d_scratch, int n_wg, int cm, double* d_ev_re, double* d_ev_im,
                        int tile, hipStream_t st) {
  if (n_strings == 0) return hipSuccess;
  if (tile < 0 || tile >= kPauliTiles) return hipErrorInvalidValue;
  const dim3 grid(n_wg, b.n_slots);
  if (b.mixed)
    launch_pauli_t<float2>(tile, grid, st, b, d_x, d_z, n_strings, d_order, d_share, d_scratch, cm, d_ev_re, d_ev_im);
  else
    launch_pauli_t<double2>(tile, grid, st, b, d_x, d_z, n_strings, d_order, d_share, d_scratch, cm, d_ev_re,
                            d_ev_im);
  return hipGetLastError();
}

hipError_t launch_energy_reduce(const DevBatch& b, const double* d_coeff, const double* d_ev_re, const double* d_ev_im,
                                int n_strings, double c_identity, double* d_energy, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_reduce, dim3(b.n_slots), dim3(64), 0, st, d_coeff, d_ev_re, d_ev_im, n_strings,
                     c_identity, d_energy, b.stats, b.slot0);
  return hipGetLastError();
}

}  // namespace q2c
