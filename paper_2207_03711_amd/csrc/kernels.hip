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

// Block-level complex GEMM: C = alpha * op(A) * op(B) (+ C if accumulate).
// op(A)[i][k] = TA ? conj(A[k*lda+i]) : A[i*lda+k]
// op(B)[k][j] = TB ? conj(B[j*ldb+k]) : B[k*ldb+j]
// lds: 2*64*8 double2.  All threads of the block must call it.
template <bool TA, bool TB>
__device__ void bgemm(int M, int N, int K, const double2* __restrict__ A, int lda,
                      const double2* __restrict__ B, int ldb, double2* __restrict__ C, int ldc,
                      double2 alpha, bool accumulate, double2* lds) {
  constexpr int BM = 64, BN = 64, BK = 8;
  double2* As = lds;
  double2* Bs = lds + BK * BM;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;  // 16 x 32 threads
  __syncthreads();
  for (int i0 = 0; i0 < M; i0 += BM) {
    for (int j0 = 0; j0 < N; j0 += BN) {
      double2 acc[2][4];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = cmk(0.0, 0.0);
      for (int k0 = 0; k0 < K; k0 += BK) {
        {
          const int r = tid >> 3, k = tid & 7;
          const int gi = i0 + r, gk = k0 + k;
          double2 v = cmk(0.0, 0.0);
          if (gi < M && gk < K) v = TA ? cconj(A[(long)gk * lda + gi]) : A[(long)gi * lda + gk];
          As[k * BM + r] = v;
        }
        {
          const int k = tid >> 6, c = tid & 63;
          const int gk = k0 + k, gj = j0 + c;
          double2 v = cmk(0.0, 0.0);
          if (gk < K && gj < N) v = TB ? cconj(B[(long)gj * ldb + gk]) : B[(long)gk * ldb + gj];
          Bs[k * BN + c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BK; ++k) {
          const double2 a0 = As[k * BM + ty * 2], a1 = As[k * BM + ty * 2 + 1];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double2 bv = Bs[k * BN + tx * 4 + q];
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
            double2 v = cmul(alpha, acc[r][q]);
            double2* dst = &C[(long)gi * ldc + gj];
            *dst = accumulate ? cadd(*dst, v) : v;
          }
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

__global__ void k_init_product(DevBatch b, const uint8_t* occ) {
  const int slot = blockIdx.x;
  const int N = b.n_qubits;
  double2* sites = b.sites + slot * b.site_stride;
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    double2* B = sites + b.site_off[n];
    const int o = occ[n] ? 1 : 0;
    // chi_l = chi_r = 1: element [0][i][0] at i * cap_r
    B[0] = cmk(o == 0 ? 1.0 : 0.0, 0.0);
    B[b.cap[n + 1]] = cmk(o == 1 ? 1.0 : 0.0, 0.0);
  }
  for (int i = threadIdx.x; i <= N; i += blockDim.x) b.chi[slot * (N + 1) + i] = 1;
  for (int n = threadIdx.x; n < N - 1; n += blockDim.x) b.lam[slot * b.lam_stride + b.lam_off[n]] = 1.0;
  for (int i = threadIdx.x; i < kNStats; i += blockDim.x) b.stats[slot * kNStats + i] = 0.0;
  if (threadIdx.x == 0) {
    b.stats[slot * kNStats + kStatMaxChi] = 1.0;
    b.flags[slot] = 0;
  }
}

__global__ void k_angles(double* phi, int n_rot, const double* rot_c, const int* rot_param,
                         const double* theta, int n_theta, const int* shift_rot, const double* shift_val) {
  const int slot = blockIdx.y;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_rot) return;
  double v = -2.0 * rot_c[m] * theta[(long)slot * n_theta + rot_param[m]];
  if (shift_rot && shift_rot[slot] == m) v += shift_val[slot];
  phi[(long)slot * n_rot + m] = v;
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


constexpr int kQB = 128;        // bisection path: q = min(m, n) <= kQB
constexpr int kKB = 64;         // bisection path: kept vectors <= kKB

// Static LDS of the gate kernel (about 100 KB of the 160 KB per CU).
struct GateLds {
  double2 gemm[2 * 64 * 8];
  double2 O[16];
  union {
    struct {
      double2 uq[512], wq[512], vq[512], zq[512];  // reflector work vectors
    };
    double Y[kQB * kKB];  // real kept vectors of the bidiagonal (bisection path)
  };
  double2 dc[kQB], ec[kQB], pa[kQB], pb[kQB];  // bidiagonal and its phases
  double t[2 * kQB], t2[2 * kQB];               // Golub-Kahan tridiagonal
  double sig[512];                              // kept singular values, descending
  double G[kKB * kKB];                          // Gram / Cholesky factor
  int blo[2 * kQB], bhi[2 * kQB];               // blocks of the split tridiagonal
  double red[16];
  double2 sbeta;
  int szero, srot, sabort, skeep, sfail, snblk;
  double sdisc, stot, snorm, sgersh, stmax;
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Number of eigenvalues below x of the symmetric tridiagonal with zero
// diagonal and squared off-diagonals t2[b0 .. b1-2] (indices b0 .. b1-1).
// With p_{-1} = 1, p_0 = -x, p_i = -x p_{i-1} - t2[i-1] p_{i-2}, the count is
// the number of sign changes of the sequence (a zero takes the sign opposite
// to its predecessor); a zero off-diagonal restarts the recurrence with the
// current sign.  Division-free; kept in range by power-of-two rescaling.
__device__ int tgk_count1(const double* t2, int b0, int b1, double x) {
  double pp = 1.0, p = -x;
  double sg = p < 0.0 ? -1.0 : 1.0;
  int c = p <= 0.0 ? 1 : 0;
  if (p == 0.0) sg = -1.0;
  // entries are scaled to |t| <= 1 and |x| <= 1: four steps grow the values
  // by at most 2^4 and shrink them by at most t^8, so range checks every
  // fourth step suffice
  int i = b0;
  while (i < b1 - 1) {
    const int lim = i + 4 < b1 - 1 ? i + 4 : b1 - 1;
    for (; i < lim; ++i) {
      const double tt = t2[i];
      double pn;
      if (tt == 0.0) {
        pp = sg;
        pn = -x * sg;
      } else {
        pn = fma(-x, p, -tt * pp);
        pp = p;
      }
      p = pn;
      const double sn = pn > 0.0 ? 1.0 : (pn < 0.0 ? -1.0 : -sg);
      c += sn != sg ? 1 : 0;
      sg = sn;
    }
    const double mg = fmax(fabs(p), fabs(pp));
    if (mg > 1e100 || (mg < 1e-100 && mg > 0.0)) {
      const int e = ilogb(mg);
      p = ldexp(p, -e);
      pp = ldexp(pp, -e);
    }
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

// ---- Phase A: Theta = B_n B_{n+1}, gate mixing (Eq. 7), lambda scaling (Eq. 8)
__device__ void gate_contract(const DevBatch& b, SlotView& v, GateLds& L, int n, int chil, int chim, int chir) {
  const int tid = threadIdx.x;
  const int nn = 2 * chir, m = 2 * chil;
  const int capl_r = b.cap[n + 1], capr_r = b.cap[n + 2];
  const double2* Bn = v.sites + b.site_off[n];
  const double2* Bn1 = v.sites + b.site_off[n + 1];
  for (int j = 0; j < 2; ++j)
    bgemm<false, false>(m, chir, chim, Bn, capl_r, Bn1 + j * capr_r, 2 * capr_r, v.M + j * chir, nn,
                        cmk(1.0, 0.0), false, L.gemm);
  double part = 0.0;
  for (int idx = tid; idx < chil * chir; idx += blockDim.x) {
    const int a = idx / chir, c = idx - a * chir;
    double2 t[4];
#pragma unroll
    for (int ip = 0; ip < 2; ++ip)
#pragma unroll
      for (int jp = 0; jp < 2; ++jp) t[2 * ip + jp] = v.M[(long)(2 * a + ip) * nn + jp * chir + c];
    const double la = n == 0 ? 1.0 : v.lam[b.lam_off[n - 1] + a];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        double2 s = cmk(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < 4; ++q) cfma(s, L.O[(2 * i + jj) * 4 + q], t[q]);
        const long off = (long)(2 * a + i) * nn + jj * chir + c;
        v.M[off] = s;
        const double2 sp = cscale(s, la);
        v.A[off] = sp;
        part += cabs2(sp);
      }
  }
  const double tot = block_sum(part, L.red);
  if (tid == 0) L.stot = tot;
  __syncthreads();
}

// M' = lambda * M again (the bisection path overwrites A).
__device__ void restore_mprime(const DevBatch& b, SlotView& v, int n, int chil, int chir) {
  const int nn = 2 * chir;
  for (int idx = threadIdx.x; idx < 2 * chil * nn; idx += blockDim.x) {
    const int row = idx / nn;
    const double la = n == 0 ? 1.0 : v.lam[b.lam_off[n - 1] + (row >> 1)];
    v.A[idx] = cscale(v.M[idx], la);
  }
  __syncthreads();
}

// ---- Phase B (default): SVD by Golub-Kahan bidiagonalisation, bisection on
// the Golub-Kahan tridiagonal for the kept singular values, twisted
// factorisations for their vectors, CholQR2 and back-transformation.
// Output: L.sig[0..keep) descending, v.W rows = kept rows of W^H (n wide),
// L.sdisc.  Returns keep, or -1 if the vectors could not be certified (the
// caller then uses the Jacobi path).  Requires min(m, n) <= kQB, D <= kKB.
__device__ int svd_bisect(SlotView& v, GateLds& L, int m, int nn, int D, double cutoff, long long* tcyc) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  const bool trans = m < nn;
  const int p = trans ? nn : m, q = trans ? m : nn;
  double2* X = trans ? v.H : v.A;
  const int ldx = q;
  if (trans) {
    // X = A^H, p = nn rows, q = m columns
    for (int idx = tid; idx < p * q; idx += blockDim.x) {
      const int i = idx / q, j = idx - i * q;
      X[idx] = cconj(v.A[(long)j * nn + i]);
    }
    __syncthreads();
  }
  // -- Golub-Kahan: H_k from the left on column k, G_k from the right on row k
  for (int k = 0; k < q; ++k) {
    const int Lc = p - k;
    for (int i = tid; i < Lc; i += blockDim.x) L.uq[i] = X[(long)(k + i) * ldx + k];
    __syncthreads();
    if (wave == 0) {
      bool z;
      wave_householder(L.uq, Lc, false, L.uq, &L.sbeta, &z);
      if (lane == 0) L.szero = z;
    }
    __syncthreads();
    if (tid == 0) L.dc[k] = L.sbeta;
    const int nw = q - k - 1;
    if (!L.szero && nw > 0) {
      // w_j = sum_i conj(u_i) X[k+i][k+1+j]: 4 row groups x up to 128 columns per pass
      for (int j0 = 0; j0 < nw; j0 += 128) {
        const int jj = j0 + (tid & 127), g = tid >> 7;
        double wr = 0.0, wi = 0.0;
        if (jj < nw) {
          for (int i = g; i < Lc; i += 4) {
            const double2 pr = cmul(cconj(L.uq[i]), X[(long)(k + i) * ldx + k + 1 + jj]);
            wr += pr.x;
            wi += pr.y;
          }
        }
        L.zq[tid] = cmk(wr, wi);
        __syncthreads();
        if (tid < 128 && j0 + tid < nw)
          L.wq[j0 + tid] = cadd(cadd(L.zq[tid], L.zq[tid + 128]), cadd(L.zq[tid + 256], L.zq[tid + 384]));
        __syncthreads();
      }
      for (int idx = tid; idx < Lc * nw; idx += blockDim.x) {
        const int i = idx / nw, jj = idx - i * nw;
        double2* e = &X[(long)(k + i) * ldx + k + 1 + jj];
        *e = csub(*e, cmul(L.uq[i], L.wq[jj]));
      }
    }
    for (int i = tid; i < Lc; i += blockDim.x) X[(long)(k + i) * ldx + k] = L.uq[i];  // left reflector
    __syncthreads();
    if (nw > 0) {
      if (wave == 0) {
        bool z;
        wave_householder(X + (long)k * ldx + k + 1, nw, true, L.vq, &L.sbeta, &z);
        if (lane == 0) L.szero = z;
      }
      __syncthreads();
      if (tid == 0) L.ec[k] = L.sbeta;
      const int nr = p - k - 1;
      if (!L.szero && nr > 0) {
        // z_i = sum_j X[k+1+i][k+1+j] v_j, 4 lanes per row
        for (int i0 = 0; i0 < nr; i0 += 128) {
          const int ii = i0 + (tid >> 2), s4 = tid & 3;
          double zr = 0.0, zi = 0.0;
          if (ii < nr) {
            for (int j = s4; j < nw; j += 4) {
              const double2 pr = cmul(X[(long)(k + 1 + ii) * ldx + k + 1 + j], L.vq[j]);
              zr += pr.x;
              zi += pr.y;
            }
          }
          zr += __shfl_xor(zr, 1, 64);
          zi += __shfl_xor(zi, 1, 64);
          zr += __shfl_xor(zr, 2, 64);
          zi += __shfl_xor(zi, 2, 64);
          if (s4 == 0 && ii < nr) L.zq[ii] = cmk(zr, zi);
        }
        __syncthreads();
        for (int idx = tid; idx < nr * nw; idx += blockDim.x) {
          const int i = idx / nw, j = idx - i * nw;
          double2* e = &X[(long)(k + 1 + i) * ldx + k + 1 + j];
          *e = csub(*e, cmul(L.zq[i], cconj(L.vq[j])));
        }
      }
      for (int j = tid; j < nw; j += blockDim.x) X[(long)k * ldx + k + 1 + j] = L.vq[j];  // right reflector
      __syncthreads();
    }
  }
  tcyc[0] = clock64();
  // -- real bidiagonal by diagonal phase scaling; Golub-Kahan tridiagonal t
  if (tid == 0) {
    double2 bk = cmk(1.0, 0.0);
    double tmax = 0.0;
    for (int k = 0; k < q; ++k) {
      const double2 d = L.dc[k];
      const double ad = sqrt(cabs2(d));
      const double2 ak = ad > 0.0 ? cscale(cmul(d, bk), 1.0 / ad) : bk;
      L.pa[k] = ak;
      L.pb[k] = bk;
      L.t[2 * k] = ad;
      tmax = fmax(tmax, ad);
      if (k + 1 < q) {
        const double2 e = L.ec[k];
        const double ae = sqrt(cabs2(e));
        bk = ae > 0.0 ? cscale(cmul(ak, cconj(e)), 1.0 / ae) : cmk(1.0, 0.0);
        L.t[2 * k + 1] = ae;
        tmax = fmax(tmax, ae);
      }
    }
    const int nt = 2 * q - 1;
    double gersh = 0.0;
    int nb = 0, start = 0;
    for (int i = 0; i < nt; ++i) {
      if (L.t[i] <= 1e-15 * tmax) L.t[i] = 0.0;  // split at negligible entries
      L.t2[i] = L.t[i] * L.t[i];
      gersh = fmax(gersh, L.t[i] + (i > 0 ? L.t[i - 1] : 0.0));
      if (L.t[i] == 0.0) {
        L.blo[nb] = start;
        L.bhi[nb] = i + 1;
        ++nb;
        start = i + 1;
      }
    }
    gersh = fmax(gersh, L.t[nt - 1]);
    // scale to |t| <= 1 (eigenvalues scale by 1/gersh, vectors unchanged)
    const double sc = gersh > 0.0 ? 1.0 / gersh : 1.0;
    for (int i = 0; i < nt; ++i) {
      L.t[i] *= sc;
      L.t2[i] = L.t[i] * L.t[i];
    }
    L.blo[nb] = start;
    L.bhi[nb] = 2 * q;
    ++nb;
    L.snblk = nb;
    L.sgersh = gersh;
    L.stmax = tmax;
  }
  __syncthreads();
  const int nT = 2 * q;
  const double pivmin = 2.3e-308;  // T is scaled to norm <= 1
  const double tscale = L.sgersh;   // singular values = scaled values * tscale
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
      const int c = tgk_count1(L.t2, 0, nT, x);
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
      const int nz = nT - tgk_count1(L.t2, 0, nT, cutoff * s0);
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
  tcyc[1] = clock64();
  const int keep = L.skeep;
  if (keep < 0) return -1;
  // -- vectors: one lane per kept value, spread over 4 waves
  // global scratch: 4 q kk <= 4 ws^2 doubles of the 8 ws^2 available
  const int KV = kk;
  double* Dp = v.V;                    // [2q][KV]: D+ pivots, then the vector
  double* Dm = v.V + (long)nT * KV;    // [2q][KV]: D- pivots
  double* Y = L.Y;                     // [q][kKB]: real vectors (LDS)
  if (tid < 4 * kKB) {
    const int j = (tid & 63) * 4 + (tid >> 6);
    if (j < keep) {
      const double sj = L.sig[j];  // scaled
      const double tol = 1e-13 * L.sig[0];
      int inst = 0;
      for (int jp = 0; jp < j; ++jp) inst += fabs(L.sig[jp] - sj) <= tol ? 1 : 0;
      int b0 = L.blo[0], b1 = L.bhi[0], seen = 0;
      bool found = false;
      for (int bk = 0; bk < L.snblk && !found; ++bk) {
        const int mult = tgk_count1(L.t2, L.blo[bk], L.bhi[bk], sj + tol) -
                         tgk_count1(L.t2, L.blo[bk], L.bhi[bk], sj - tol);
        if (mult > 0 && seen + mult > inst) {
          b0 = L.blo[bk];
          b1 = L.bhi[bk];
          found = true;
        }
        seen += mult;
      }
      double nrm2 = 1.0;
      if (b1 - b0 == 1) {
        Dp[b0 * KV + j] = 1.0;
      } else {
        // forward pivots D+ of (T - s I) on the block
        double dd = -sj;
        Dp[b0 * KV + j] = dd;
        for (int i = b0 + 1; i < b1; ++i) {
          if (fabs(dd) < pivmin) dd = -pivmin;
          dd = fma(-L.t2[i - 1], rcp_nr(dd), -sj);
          Dp[i * KV + j] = dd;
        }
        // backward pivots D- and the twist index r = argmin |D+ + D- + s|
        dd = -sj;
        Dm[(b1 - 1) * KV + j] = dd;
        int r = b1 - 1;
        double gmin = fabs(Dp[(b1 - 1) * KV + j]);
        for (int i = b1 - 2; i >= b0; --i) {
          if (fabs(dd) < pivmin) dd = -pivmin;
          dd = fma(-L.t2[i], rcp_nr(dd), -sj);
          Dm[i * KV + j] = dd;
          const double g = fabs(Dp[i * KV + j] + dd + sj);
          if (g <= gmin) {
            gmin = g;
            r = i;
          }
        }
        // twisted solve: z_r = 1, up with L+, down with U-
        double z = 1.0;
        for (int i = r - 1; i >= b0; --i) {
          double dpi = Dp[i * KV + j];
          if (fabs(dpi) < pivmin) dpi = -pivmin;
          z = -(L.t[i] * rcp_nr(dpi)) * z;
          Dp[i * KV + j] = z;
          nrm2 += z * z;
        }
        Dp[r * KV + j] = 1.0;
        z = 1.0;
        for (int i = r + 1; i < b1; ++i) {
          double dmi = Dm[i * KV + j];
          if (fabs(dmi) < pivmin) dmi = -pivmin;
          z = -(L.t[i - 1] * rcp_nr(dmi)) * z;
          Dp[i * KV + j] = z;
          nrm2 += z * z;
        }
      }
      const double inv = 1.0 / sqrt(nrm2);
      const int off = trans ? 1 : 0;  // X = A: right vectors (even); X = A^H: left vectors (odd)
      for (int k = 0; k < q; ++k) {
        const int i = 2 * k + off;
        Y[k * kKB + j] = (i >= b0 && i < b1) ? Dp[i * KV + j] * inv : 0.0;
      }
    }
  }
  __syncthreads();
  for (int j = tid; j < keep; j += blockDim.x) L.sig[j] *= tscale;  // unscaled singular values
  __syncthreads();
  // -- CholQR2 on Y (q x keep), all in LDS
  for (int pass = 0; pass < 2; ++pass) {
    // Gram, 4x4 register tiles of the lower triangle
    const int nb4 = (keep + 3) >> 2;
    for (int tIdx = tid; tIdx < nb4 * nb4; tIdx += blockDim.x) {
      const int ba = tIdx / nb4, bc = tIdx - ba * nb4;
      if (bc > ba) continue;
      double acc[4][4] = {};
      for (int k = 0; k < q; ++k) {
        double ya[4], yc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ya[u] = Y[k * kKB + 4 * ba + u];
          yc[u] = Y[k * kKB + 4 * bc + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int w = 0; w < 4; ++w) acc[u][w] = fma(ya[u], yc[w], acc[u][w]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int a = 4 * ba + u, c = 4 * bc + w;
          if (a < keep && c <= a) L.G[a * kKB + c] = acc[u][w];
        }
    }
    __syncthreads();
    // right-looking Cholesky, lower triangle in place
    for (int j = 0; j < keep; ++j) {
      const double djj = L.G[j * kKB + j];
      if (!(djj > 1e-10) || !isfinite(djj)) {
        if (tid == 0) L.sfail = 1;
        break;
      }
      const double ljj = sqrt(djj);
      __syncthreads();
      for (int a = j + 1 + tid; a < keep; a += blockDim.x) L.G[a * kKB + j] /= ljj;
      if (tid == 0) L.G[j * kKB + j] = ljj;
      __syncthreads();
      const int rem = keep - j - 1;
      for (int e = tid; e < rem * rem; e += blockDim.x) {
        const int a = j + 1 + e / rem, c = j + 1 + e % rem;
        if (c <= a) L.G[a * kKB + c] -= L.G[a * kKB + j] * L.G[c * kKB + j];
      }
      __syncthreads();
    }
    __syncthreads();
    if (L.sfail) return -1;
    // Y <- Y L^{-T}: forward substitution per row of Y, 4 rows per wave-quarter
    for (int k = tid; k < q; k += blockDim.x) {
      for (int c = 0; c < keep; ++c) {
        double sacc = Y[k * kKB + c];
        for (int e = 0; e < c; ++e) sacc -= Y[k * kKB + e] * L.G[c * kKB + e];
        Y[k * kKB + c] = sacc / L.G[c * kKB + c];
      }
    }
    __syncthreads();
  }
  tcyc[2] = clock64();
  // -- complex vectors of the bidiagonal, then through the reflectors.
  // Wt rows j (length nn) in global; per reflector: dots for all kept
  // vectors (4 lanes x 128 vectors per pass), one barrier, then the update.
  double2* Wt = v.W;  // [keep][nn]
  for (int idx = tid; idx < keep * nn; idx += blockDim.x) {
    const int j = idx / nn, k = idx - j * nn;
    double2 w = cmk(0.0, 0.0);
    if (k < q) w = cscale(trans ? L.pa[k] : L.pb[k], Y[k * kKB + j]);
    Wt[idx] = w;
  }
  __syncthreads();
  const int kstart = trans ? q - 1 : q - 2;
  for (int k = kstart; k >= 0; --k) {
    const int off = trans ? k : k + 1;
    const int len = trans ? p - k : q - k - 1;
    // u_i = X[k+i][k] (left reflector, trans) or X[k][k+1+i] (right reflector)
    for (int i = tid; i < len; i += blockDim.x) L.uq[i] = trans ? X[(long)(k + i) * ldx + k] : X[(long)k * ldx + k + 1 + i];
    __syncthreads();
    {
      const int j = tid >> 3, s8 = tid & 7;  // 8 lanes per vector, 64 vectors
      double dr = 0.0, di = 0.0;
      if (j < keep) {
        const double2* w = Wt + (long)j * nn + off;
        for (int i = s8; i < len; i += 8) {
          const double2 pr = cmul(cconj(L.uq[i]), w[i]);
          dr += pr.x;
          di += pr.y;
        }
      }
#pragma unroll
      for (int o = 1; o < 8; o <<= 1) {
        dr += __shfl_xor(dr, o, 64);
        di += __shfl_xor(di, o, 64);
      }
      if (s8 == 0 && j < keep) L.wq[j] = cmk(dr, di);
    }
    __syncthreads();
    for (int idx = tid; idx < keep * len; idx += blockDim.x) {
      const int j = idx / len, i = idx - j * len;
      double2* e = Wt + (long)j * nn + off + i;
      *e = csub(*e, cmul(L.uq[i], L.wq[j]));
    }
    __syncthreads();
  }
  for (int idx = tid; idx < keep * nn; idx += blockDim.x) Wt[idx] = cconj(Wt[idx]);  // rows of W^H
  __syncthreads();
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
template <bool kSmall>
__global__ __launch_bounds__(kBlock) void k_gates(DevBatch b, const int* __restrict__ gsite,
                                                  const int* __restrict__ grot, const double2* __restrict__ gpre,
                                                  const double2* __restrict__ gpost, const double* __restrict__ phi_all,
                                                  int n_rot, int g0, int g1, SvdParams sp) {
  __shared__ GateLds L;
  const int slot = blockIdx.x;
  const int tid = threadIdx.x;
  SlotView v = slot_view(b, slot);
  const double* phi = phi_all ? phi_all + (long)slot * n_rot : nullptr;
  if (tid == 0) L.sabort = (*v.flags & kFlagNumeric) ? 1 : 0;
  __syncthreads();
  if (L.sabort) return;

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
    gate_contract(b, v, L, n, chil, chim, chir);
    tc[1] = clock64();

    int keep = -1, sweeps = 0;
    bool conv = true, used_bisect = false, fell_back = false;
    long long tb[3] = {tc[1], tc[1], tc[1]};
    if (kSmall && sp.algo == 0 && qmin <= kQB) {
      used_bisect = true;
      keep = svd_bisect(v, L, m, nn, b.max_bond, sp.cutoff_rel, tb);
      if (keep < 0) {
        fell_back = true;
        restore_mprime(b, v, n, chil, chir);
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
    double2* Bn = v.sites + b.site_off[n];
    double2* Bn1 = v.sites + b.site_off[n + 1];
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
      Bn1[(long)(2 * k + jj) * capr_r + c] = v.W[idx];
    }
    for (int k = tid; k < keep; k += blockDim.x) v.lam[b.lam_off[n] + k] = L.sig[k] / nrm;
    __syncthreads();
    // B_n = M W / ||S_kept||  (Eq. 10: no division by Schmidt values)
    bgemm<false, true>(m, keep, nn, v.M, nn, v.W, nn, Bn, capl_r, cmk(1.0 / nrm, 0.0), false, L.gemm);
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
}

// ----------------------------------------------------------- environments --

// L[0] = 1; L[k+1] = sum_i B_i^H L[k] B_i.   Rt[N] = 1; Rt[k] = sum_i B_i Rt[k+1] B_i^H.
__global__ __launch_bounds__(kBlock) void k_envs(DevBatch b) {
  __shared__ double2 lds_gemm[2 * 64 * 8];
  const int slot = blockIdx.x;
  const int N = b.n_qubits;
  SlotView v = slot_view(b, slot);
  double2* L = b.envL + slot * b.env_stride;
  double2* R = b.envR + slot * b.env_stride;
  double2* X = v.M;  // scratch
  if (threadIdx.x == 0) {
    L[b.env_off[0]] = cmk(1.0, 0.0);
    R[b.env_off[N]] = cmk(1.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    const int cl = v.chi[k], cr = v.chi[k + 1];
    const int capl = b.cap[k], capr = b.cap[k + 1];
    const double2* Bk = v.sites + b.site_off[k];
    for (int i = 0; i < 2; ++i) {
      bgemm<false, false>(cl, cr, cl, L + b.env_off[k], capl, Bk + i * capr, 2 * capr, X, cr, cmk(1.0, 0.0),
                          false, lds_gemm);
      bgemm<true, false>(cr, cr, cl, Bk + i * capr, 2 * capr, X, cr, L + b.env_off[k + 1], capr,
                         cmk(1.0, 0.0), i == 1, lds_gemm);
    }
  }
  for (int k = N - 1; k >= 0; --k) {
    const int cl = v.chi[k], cr = v.chi[k + 1];
    const int capl = b.cap[k], capr = b.cap[k + 1];
    const double2* Bk = v.sites + b.site_off[k];
    for (int i = 0; i < 2; ++i) {
      bgemm<false, false>(cl, cr, cr, Bk + i * capr, 2 * capr, R + b.env_off[k + 1], capr, X, cr, cmk(1.0, 0.0),
                          false, lds_gemm);
      bgemm<false, true>(cl, cl, cr, X, cr, Bk + i * capr, 2 * capr, R + b.env_off[k], capl, cmk(1.0, 0.0),
                         i == 1, lds_gemm);
    }
  }
  if (threadIdx.x == 0) v.stats[kStatNorm] = L[b.env_off[N]].x;
}

// --------------------------------------------------------- Pauli sweeps ---

__global__ __launch_bounds__(kBlock) void k_pauli(DevBatch b, const uint64_t* __restrict__ sx,
                                                  const uint64_t* __restrict__ sz, int n_strings,
                                                  double2* scratch, int cm, double* ev_re, double* ev_im) {
  __shared__ double2 lds_gemm[2 * 64 * 8];
  __shared__ double red[kBlock / 64];
  const int slot = blockIdx.y;
  const int N = b.n_qubits;
  SlotView v = slot_view(b, slot);
  const double2* L = b.envL + slot * b.env_stride;
  const double2* R = b.envR + slot * b.env_stride;
  double2* T0 = scratch + ((long)slot * gridDim.x + blockIdx.x) * 3 * (long)cm * cm;
  double2* T1 = T0 + (long)cm * cm;
  double2* X = T1 + (long)cm * cm;
  const double nrm = L[b.env_off[N]].x;
  for (int s = blockIdx.x; s < n_strings; s += gridDim.x) {
    const uint64_t x = sx[s], z = sz[s];
    const uint64_t mk = x | z;
    double2 ev = cmk(0.0, 0.0);
    if (mk == 0) {
      ev = cmk(1.0, 0.0);
    } else {
      const int lo = __builtin_ctzll(mk), hi = 63 - __builtin_clzll(mk);
      const int c0 = v.chi[lo];
      const double2* Llo = L + b.env_off[lo];
      for (int idx = threadIdx.x; idx < c0 * c0; idx += blockDim.x) {
        const int a = idx / c0, c = idx - a * c0;
        T0[(long)a * cm + c] = Llo[(long)a * b.cap[lo] + c];
      }
      __syncthreads();
      double2* T = T0;
      double2* Tn = T1;
      for (int k = lo; k <= hi; ++k) {
        const int cl = v.chi[k], cr = v.chi[k + 1];
        const int capr = b.cap[k + 1];
        const double2* Bk = v.sites + b.site_off[k];
        const int xb = (x >> k) & 1, zb = (z >> k) & 1;
        for (int i = 0; i < 2; ++i) {
          const int ip = xb ? 1 - i : i;
          double2 ph = cmk(1.0, 0.0);
          if (zb && !xb) ph = i == 0 ? cmk(1.0, 0.0) : cmk(-1.0, 0.0);  // Z
          if (zb && xb) ph = i == 0 ? cmk(0.0, -1.0) : cmk(0.0, 1.0);   // Y: <0|Y|1> = -i
          bgemm<false, false>(cl, cr, cl, T, cm, Bk + ip * capr, 2 * capr, X, cm, cmk(1.0, 0.0), false, lds_gemm);
          bgemm<true, false>(cr, cr, cl, Bk + i * capr, 2 * capr, X, cm, Tn, cm, ph, i == 1, lds_gemm);
        }
        double2* t = T;
        T = Tn;
        Tn = t;
      }
      // <P> = sum_{c,c'} T[c][c'] R[c][c'],  R[c][c'] = Rt[c'][c]
      const int ch = v.chi[hi + 1];
      const double2* Rh = R + b.env_off[hi + 1];
      const int ldr = b.cap[hi + 1];
      double pr = 0.0, pi = 0.0;
      for (int idx = threadIdx.x; idx < ch * ch; idx += blockDim.x) {
        const int a = idx / ch, c = idx - a * ch;
        const double2 p = cmul(T[(long)a * cm + c], Rh[(long)c * ldr + a]);
        pr += p.x;
        pi += p.y;
      }
      pr = block_sum(pr, red);
      pi = block_sum(pi, red);
      ev = cmk(pr / nrm, pi / nrm);
    }
    if (threadIdx.x == 0) {
      ev_re[(long)slot * n_strings + s] = ev.x;
      ev_im[(long)slot * n_strings + s] = ev.y;
    }
    __syncthreads();
  }
}

// Neumaier-compensated sum in term order, identity coefficient last.
__global__ void k_energy_reduce(const double* coeff, const double* ev_re, const double* ev_im, int n_strings,
                                double c_identity, double* energy, double* stats) {
  const int slot = blockIdx.x;
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
    add(coeff[i] * ev_re[(long)slot * n_strings + i]);
    mi = fmax(mi, fabs(ev_im[(long)slot * n_strings + i]));
  }
  add(c_identity);
  energy[slot] = s + comp;
  stats[slot * kNStats + kStatMaxImag] = mi;
}

// --------------------------------------------------------------- launchers --

hipError_t launch_init_product(const DevBatch& b, const uint8_t* d_occ, hipStream_t st) {
  hipLaunchKernelGGL(k_init_product, dim3(b.n_slots), dim3(64), 0, st, b, d_occ);
  return hipGetLastError();
}

hipError_t launch_angles(const DevBatch& b, const DevProblem& p, const double* d_theta, int n_theta,
                         const int* d_shift_rot, const double* d_shift_val, hipStream_t st) {
  if (p.n_rot == 0) return hipSuccess;
  dim3 grid((p.n_rot + 255) / 256, b.n_slots);
  hipLaunchKernelGGL(k_angles, grid, dim3(256), 0, st, b.phi, p.n_rot, p.rot_c, p.rot_param, d_theta, n_theta,
                     d_shift_rot, d_shift_val);
  return hipGetLastError();
}

hipError_t launch_gates(const DevBatch& b, const int* d_site, const int* d_rot, const double2* d_pre,
                        const double2* d_post, int g0, int g1, int n_rot, SvdParams sp, hipStream_t st) {
  if (g1 <= g0) return hipSuccess;
  int cm = 1;
  for (int i = 0; i <= b.n_qubits; ++i) cm = cm > b.cap[i] ? cm : b.cap[i];
  if (cm <= kKB)
    hipLaunchKernelGGL(k_gates<true>, dim3(b.n_slots), dim3(kBlock), 0, st, b, d_site, d_rot, d_pre, d_post, b.phi,
                       n_rot, g0, g1, sp);
  else
    hipLaunchKernelGGL(k_gates<false>, dim3(b.n_slots), dim3(kBlock), 0, st, b, d_site, d_rot, d_pre, d_post, b.phi,
                       n_rot, g0, g1, sp);
  return hipGetLastError();
}

hipError_t launch_envs(const DevBatch& b, hipStream_t st) {
  hipLaunchKernelGGL(k_envs, dim3(b.n_slots), dim3(kBlock), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_pauli(const DevBatch& b, const uint64_t* d_x, const uint64_t* d_z, int n_strings, double2* d_scratch,
                        int n_wg, int cm, double* d_ev_re, double* d_ev_im, hipStream_t st) {
  if (n_strings == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pauli, dim3(n_wg, b.n_slots), dim3(kBlock), 0, st, b, d_x, d_z, n_strings, d_scratch, cm,
                     d_ev_re, d_ev_im);
  return hipGetLastError();
}

hipError_t launch_energy_reduce(const DevBatch& b, const double* d_coeff, const double* d_ev_re, const double* d_ev_im,
                                int n_strings, double c_identity, double* d_energy, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_reduce, dim3(b.n_slots), dim3(64), 0, st, d_coeff, d_ev_re, d_ev_im, n_strings,
                     c_identity, d_energy, b.stats);
  return hipGetLastError();
}

}  // namespace q2c
