// Correlation-energy stage (Sec. 2, E_c^RPA with Tr ln = ln det), FP64 complex:
//   per q: v(q) = L L^H (blocked Cholesky);  per (q, omega): B = L^H chi L,
//   f = ln det(I - B) + Tr B = 2 sum_i ln Re(L_A)_ii + Tr B with I - B = L_A L_A^H.
// Kernels: batched complex GEMM on MFMA f64 (4 real products per complex tile),
// blocked right-looking Cholesky (diagonal block in LDS, triangular solve by the
// explicit inverse of the diagonal factor, Hermitian rank-k update by the GEMM),
// trace / identity-minus, log-diagonal and quadrature reductions.
// At a q point where chi(q, i omega) and v(q) are both real (a time-reversal invariant q with a
// real basis), the same steps run on real matrices in a real row-major layout: a real GEMM with
// 128 x 128 tiles (one real product where the complex form takes four, and twice the flops
// per byte of a tile), the Cholesky pieces reading and writing the real layout.
#include "ec_kernels.h"

#include <type_traits>

namespace {

constexpr int ZB = 64, ZK = 16, ZT = 256;
// LDS tiles are [k][row]; row r of k-row kk sits at r ^ zswz(kk), which puts the 32 lanes of
// each half wave into distinct bank pairs both for the stores (16 consecutive k of one row, or
// 32 consecutive rows of one k) and for the MFMA operand reads (16 rows of two k)
static __device__ __forceinline__ int zswz(int kk) { return ((kk & 1) << 4) | ((kk >> 1) << 1); }

// OPA / OPB: 0 the operand as stored, 1 its conjugate transpose.  All loads of the K loop are
// raw buffer loads through views of this block's operands (bytesA, bytesB), unconditional:
// elements outside M, N or K are addressed past the view and read zero, so no load waits for
// another and the compiler's wait counts keep the next K step's loads in flight.
template <int OPA, int OPB>
__global__ __launch_bounds__(ZT) void zgemm_kernel(ZgemmArgs g, unsigned bytesA, unsigned bytesB) {
  __shared__ double Ar[2][ZK][ZB], Ai[2][ZK][ZB], Br[2][ZK][ZB], Bi[2][ZK][ZB];
  const int n0 = blockIdx.x * ZB, m0 = blockIdx.y * ZB, bz = blockIdx.z;
  if (g.lower_only && n0 > m0 + ZB - 1) return;
  const int gb = g.boff + bz, bi = g.binner > 0 ? g.binner : 1;
  const int go = gb / bi, gi = gb - go * bi;
  if (g.skip && g.skip[go]) return;
  const bool realA = g.realA && g.realA[go];   // block-uniform
  const double *A = g.A + (size_t)bz * g.strideA + (size_t)go * g.outerA + (size_t)gi * g.innerA;
  const double *B = g.B + (size_t)bz * g.strideB + (size_t)go * g.outerB + (size_t)gi * g.innerB;
  double *C = g.C + (size_t)bz * g.strideC;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1, col = lane & 15, grp = lane >> 4;

  int kbeg = 0;
  if (g.kmode == 1) kbeg = n0;
  if (g.kmode == 2) kbeg = m0;
  kbeg = (kbeg / ZK) * ZK;

  double2 ra[4], rb[4];
  const __amdgpu_buffer_rsrc_t rA = buffer_view(A, bytesA), rB = buffer_view(B, bytesB);
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int akk = OPA == 0 ? (tid & 15) : (tid >> 6) + 4 * e;
      const int arow = OPA == 0 ? (tid >> 4) + 16 * e : (tid & 63);
      const unsigned ia = (unsigned)((OPA == 0 ? (size_t)(m0 + arow) * g.lda + k0 + akk
                                               : (size_t)(k0 + akk) * g.lda + m0 + arow) * 16);
      const unsigned oa = ((m0 + arow < g.M) & (k0 + akk < g.K)) ? ia : bytesA;
      ra[e] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rA, oa, 0, 0));
      if (OPA) ra[e].y = -ra[e].y;
      const int bkk = OPB == 0 ? (tid >> 6) + 4 * e : (tid & 15);
      const int bcol = OPB == 0 ? (tid & 63) : (tid >> 4) + 16 * e;
      const unsigned ib = (unsigned)((OPB == 0 ? (size_t)(k0 + bkk) * g.ldb + n0 + bcol
                                               : (size_t)(n0 + bcol) * g.ldb + k0 + bkk) * 16);
      const unsigned ob = ((n0 + bcol < g.N) & (k0 + bkk < g.K)) ? ib : bytesB;
      rb[e] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rB, ob, 0, 0));
      if (OPB) rb[e].y = -rb[e].y;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int kk = OPA == 0 ? (tid & 15) : (tid >> 6) + 4 * e;
      const int row = OPA == 0 ? (tid >> 4) + 16 * e : (tid & 63);
      Ar[buf][kk][row ^ zswz(kk)] = ra[e].x;
      Ai[buf][kk][row ^ zswz(kk)] = ra[e].y;
      kk = OPB == 0 ? (tid >> 6) + 4 * e : (tid & 15);
      const int cc = OPB == 0 ? (tid & 63) : (tid >> 4) + 16 * e;
      Br[buf][kk][cc ^ zswz(kk)] = rb[e].x;
      Bi[buf][kk][cc ^ zswz(kk)] = rb[e].y;
    }
  };

  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) accR[a][b] = accI[a][b] = Mfma<double>::zero();

  const int nk = g.K > kbeg ? (g.K - kbeg + ZK - 1) / ZK : 0;
  if (nk > 0) {                            // block-uniform
    load(kbeg);
    store(0);
  }
  __syncthreads();
  // the K loop, with four real products per complex product, or two when A is real (the same
  // sums without the terms whose A factor is an exact zero)
  auto kloop = [&](auto real_tag) {
    constexpr bool kReal = decltype(real_tag)::value;
    for (int it = 0; it < nk; ++it) {
      const int cur = it & 1;
      if (it + 1 < nk) load(kbeg + (it + 1) * ZK);
#pragma unroll
      for (int ks = 0; ks < ZK / 4; ++ks) {
        const int kk = ks * 4 + grp;
        double ar[2], ai[2], br[2], bi[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          ar[q] = Ar[cur][kk][(wm * 32 + q * 16 + col) ^ zswz(kk)];
          ai[q] = kReal ? 0.0 : Ai[cur][kk][(wm * 32 + q * 16 + col) ^ zswz(kk)];
          br[q] = Br[cur][kk][(wn * 32 + q * 16 + col) ^ zswz(kk)];
          bi[q] = Bi[cur][kk][(wn * 32 + q * 16 + col) ^ zswz(kk)];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            accR[a][b] = Mfma<double>::fma(ar[a], br[b], accR[a][b]);
            if (!kReal) accR[a][b] = Mfma<double>::fma(-ai[a], bi[b], accR[a][b]);
            accI[a][b] = Mfma<double>::fma(ar[a], bi[b], accI[a][b]);
            if (!kReal) accI[a][b] = Mfma<double>::fma(ai[a], br[b], accI[a][b]);
          }
      }
      if (it + 1 < nk) store(cur ^ 1);
      __syncthreads();
    }
  };
  if (realA)
    kloop(std::true_type{});
  else
    kloop(std::false_type{});
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm * 32 + a * 16 + Mfma<double>::row(grp, r);
        const int j = n0 + wn * 32 + b * 16 + col;
        if (i < g.M && j < g.N) {
          double2 *p = reinterpret_cast<double2 *>(C) + (size_t)i * g.ldc + j;
          double2 o = make_double2(g.alpha * accR[a][b][r], g.alpha * accI[a][b][r]);
          if (g.beta != 0.0) {
            const double2 c = *p;
            o.x += g.beta * c.x;
            o.y += g.beta * c.y;
          }
          *p = o;
        }
      }
}

// Real batched GEMM, C = alpha op(A) op(B) + beta C, a 128 x BN output tile per workgroup of 4
// waves: BN = 128 as 2 x 2 waves of 64 x 64 (4 x 4 MFMA tiles of 16 x 16), BN = 32 (products with
// at most 32 columns, such as the Cholesky panel updates) as 4 x 1 waves of 32 x 32.  K step 16
// through double-buffered LDS tiles [k][row] with row r of k-row kk at r ^ dswz(kk): the MFMA
// operand reads (16 rows of four k) then take the two LDS cycles a 64-lane 8-byte read needs.  Every K-loop load is a raw buffer
// load of one element, unconditional (elements outside M, N or K read zero).  A thread's eight
// elements of a tile are 16 consecutive k of a row per 16 lanes when the operand is stored
// row by row along k, else 128 consecutive rows of one k per 128 threads, so each load
// instruction reads whole cache lines.
constexpr int DB = 128, DK = 16, DT = 256;
template <int W> static __device__ __forceinline__ int dswz(int kk) { return ((kk & 15) << 3) & (W - 1); }

template <int OPA, int OPB, int BN>
__global__ __launch_bounds__(DT, 2) void dgemm_kernel(DgemmArgs g, unsigned bytesA, unsigned bytesB) {
  constexpr int WN = BN == 128 ? 2 : 1, WM = 4 / WN;        // waves along n and m
  constexpr int TM = DB / (16 * WM), TN = BN / (16 * WN);   // MFMA tiles per wave
  constexpr int NB = BN / 16;                               // B elements per thread and K step
  __shared__ double As[2][DK][DB], Bs[2][DK][BN];
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * DB, bz = blockIdx.z;
  if (g.lower_only && n0 > m0 + DB - 1) return;
  const int gb = g.boff + bz, bi = g.binner > 0 ? g.binner : 1;
  const int go = gb / bi, gi = gb - go * bi;
  if (g.sel && !g.sel[go]) return;
  const double *A = g.A + (size_t)bz * g.strideA + (size_t)go * g.outerA + (size_t)gi * g.innerA;
  const double *B = g.B + (size_t)bz * g.strideB + (size_t)go * g.outerB + (size_t)gi * g.innerB;
  double *C = g.C + (size_t)bz * g.strideC;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / WN, wn = w % WN, col = lane & 15, grp = lane >> 4;

  int kbeg = 0;
  if (g.kmode == 1) kbeg = n0;
  if (g.kmode == 2) kbeg = m0;
  kbeg = (kbeg / DK) * DK;

  // this thread's elements: (row, k) = (rc + 16 e, kc) in the along-k form, (rt, kt + 2 e) in
  // the other (for B with BN columns: (ct, ktb + (256 / BN) e))
  const int kc = tid & 15, rc = tid >> 4, rt = tid & 127, kt = tid >> 7;
  const int ct = tid % BN, ktb = tid / BN;
  double ra[8], rb[NB];
  const __amdgpu_buffer_rsrc_t rA = buffer_view(A, bytesA), rB = buffer_view(B, bytesB);
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int akk = OPA == 0 ? kc : kt + 2 * e, arow = OPA == 0 ? rc + 16 * e : rt;
      const unsigned ia = (unsigned)((OPA == 0 ? (size_t)(m0 + arow) * g.lda + k0 + akk
                                               : (size_t)(k0 + akk) * g.lda + m0 + arow) * 8);
      ra[e] = buffer_load<double>(rA, ((m0 + arow < g.M) & (k0 + akk < g.K)) ? ia : bytesA);
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int bkk = OPB == 0 ? ktb + (DT / BN) * e : kc, bcol = OPB == 0 ? ct : rc + 16 * e;
      const unsigned ib = (unsigned)((OPB == 0 ? (size_t)(k0 + bkk) * g.ldb + n0 + bcol
                                               : (size_t)(n0 + bcol) * g.ldb + k0 + bkk) * 8);
      rb[e] = buffer_load<double>(rB, ((n0 + bcol < g.N) & (k0 + bkk < g.K)) ? ib : bytesB);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int akk = OPA == 0 ? kc : kt + 2 * e, arow = OPA == 0 ? rc + 16 * e : rt;
      As[buf][akk][arow ^ dswz<DB>(akk)] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int bkk = OPB == 0 ? ktb + (DT / BN) * e : kc, bcol = OPB == 0 ? ct : rc + 16 * e;
      Bs[buf][bkk][bcol ^ dswz<BN>(bkk)] = rb[e];
    }
  };

  d4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = Mfma<double>::zero();

  const int nk = g.K > kbeg ? (g.K - kbeg + DK - 1) / DK : 0;
  if (nk > 0) {                            // block-uniform
    load(kbeg);
    store(0);
  }
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) load(kbeg + (it + 1) * DK);
#pragma unroll
    for (int ks = 0; ks < DK / 4; ++ks) {
      const int kk = ks * 4 + grp;
      double ar[TM], br[TN];
#pragma unroll
      for (int q = 0; q < TM; ++q) ar[q] = As[cur][kk][(wm * TM * 16 + q * 16 + col) ^ dswz<DB>(kk)];
#pragma unroll
      for (int q = 0; q < TN; ++q) br[q] = Bs[cur][kk][(wn * TN * 16 + q * 16 + col) ^ dswz<BN>(kk)];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = Mfma<double>::fma(ar[a], br[b], acc[a][b]);
    }
    if (it + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm * TM * 16 + a * 16 + Mfma<double>::row(grp, r);
        const int j = n0 + wn * TN * 16 + b * 16 + col;
        if (i < g.M && j < g.N) {
          double *p = C + (size_t)i * g.ldc + j;
          double o = g.alpha * acc[a][b][r];
          if (g.beta != 0.0) o += g.beta * *p;
          *p = o;
        }
      }
}

// dst[m * dstride + e] = Re src_m[e] for the matrices m whose outer index is selected.
__global__ __launch_bounds__(256) void pack_real_kernel(const double *__restrict__ src, long long outer,
                                                        long long inner, int boff, int binner,
                                                        double *__restrict__ dst, size_t dstride, size_t n2,
                                                        const int *__restrict__ sel) {
  const int m = blockIdx.y;
  const int gb = boff + m, bi = binner > 0 ? binner : 1;
  const int go = gb / bi, gi = gb - go * bi;
  if (sel && !sel[go]) return;
  const double2 *S = reinterpret_cast<const double2 *>(src + (size_t)go * outer + (size_t)gi * inner);
  double *D = dst + (size_t)m * dstride;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += (size_t)gridDim.x * blockDim.x)
    D[e] = S[e].x;
}

__global__ void both_real_kernel(const int *realchi, const int *realv, int nq, int nomega, int *both, int *pair) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nq) both[e] = realchi[e] && realv[e];
  if (e < nq * nomega) {
    const int q = e / nomega;
    pair[e] = realchi[q] && realv[q];
  }
}

// counts[0] = number of q with chi and v real, counts[1] = nq - counts[0]; one workgroup.
__global__ __launch_bounds__(256) void count_real_kernel(const int *realchi, const int *realv, int nq, int *counts) {
  __shared__ int red[256];
  int c = 0;
  for (int q = threadIdx.x; q < nq; q += blockDim.x) c += (realchi[q] && realv[q]) ? 1 : 0;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    counts[0] = red[0];
    counts[1] = nq - red[0];
  }
}

// real[q] &= (imaginary part == 0) over the nomega matrices of q; the flags start at 1.
__global__ __launch_bounds__(256) void real_flags_kernel(const double *__restrict__ X, size_t mat, int nq,
                                                         int nomega, int *__restrict__ real) {
  const int q = blockIdx.y;
  const size_t per = (size_t)nomega * (mat / 2);   // complex elements of q over all omega
  bool zero = true;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < per; e += (size_t)gridDim.x * blockDim.x) {
    const size_t w = e / (mat / 2), i = e - w * (mat / 2);
    zero &= X[(w * nq + q) * mat + 2 * i + 1] == 0.0;
  }
  if (!__all(zero) && (threadIdx.x & 63) == 0) real[q] = 0;
}

// ---- Cholesky pieces (block width CB) ----
constexpr int CB = 32;

// Element helpers for the diagonal-block factorisation: double (real layout) or double2
// (complex interleaved), with the products it needs.
static __device__ __forceinline__ double el_zero(double) { return 0.0; }
static __device__ __forceinline__ double2 el_zero(double2) { return make_double2(0.0, 0.0); }
static __device__ __forceinline__ double el_real(double, double v) { return v; }
static __device__ __forceinline__ double2 el_real(double2, double v) { return make_double2(v, 0.0); }
static __device__ __forceinline__ double el_re(double a) { return a; }
static __device__ __forceinline__ double el_re(double2 a) { return a.x; }
static __device__ __forceinline__ double el_scale(double a, double s) { return a * s; }
static __device__ __forceinline__ double2 el_scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// a - b conj(c)
static __device__ __forceinline__ double el_sub_mulc(double a, double b, double c) { return a - b * c; }
static __device__ __forceinline__ double2 el_sub_mulc(double2 a, double2 b, double2 c) {
  return make_double2(a.x - (b.x * c.x + b.y * c.y), a.y - (b.y * c.x - b.x * c.y));
}
// a - b c
static __device__ __forceinline__ double el_sub_mul(double a, double b, double c) { return a - b * c; }
static __device__ __forceinline__ double2 el_sub_mul(double2 a, double2 b, double2 c) {
  return make_double2(a.x - (b.x * c.x - b.y * c.y), a.y - (b.x * c.y + b.y * c.x));
}
static __device__ __forceinline__ double2 el_conj_c(double a) { return make_double2(a, 0.0); }
static __device__ __forceinline__ double2 el_conj_c(double2 a) { return make_double2(a.x, -a.y); }
// the value lane l holds (l wave-uniform)
static __device__ __forceinline__ double el_lane(double v, int l) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
static __device__ __forceinline__ double2 el_lane(double2 v, int l) { return make_double2(el_lane(v.x, l), el_lane(v.y, l)); }

// Factor the CB x CB diagonal block at (p, p) of one matrix (element type E, row-major with
// row length n): lane i < CB holds row i in registers, and the column of each step reaches the
// other lanes by readlane, so the factorisation needs neither LDS nor barriers.  The factor goes
// back to the matrix (lower triangle) and to LDS, where lane c forms column c of
// X = L11^{-1} by forward substitution (its entries above the diagonal come out exactly zero);
// W = X^H (complex layout) is left for the panel solve.  A pivot that is not positive and finite is
// replaced by 1 and flagged (1: not positive definite, 2: NaN or Inf met; the first failure of
// a matrix is the one kept).
template <typename E>
__device__ __forceinline__ void chol_diag_block(E *M, int n, int p, double2 *W, int *flag, void *lds) {
  E(*Ls)[CB + 1] = reinterpret_cast<E(*)[CB + 1]>(lds);
  const int lane = threadIdx.x;
  const int b = min(CB, n - p);
  const E z = el_zero(E{});
  E a[CB];
#pragma unroll
  for (int k = 0; k < CB; ++k) a[k] = (lane < b && k <= lane) ? M[(size_t)(p + lane) * n + p + k] : z;
  int bad = 0;                                      // wave-uniform
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    if (j < b) {
      const double d = el_re(el_lane(a[j], j));
      double piv = 1.0;
      if (!(d > 0.0) || !isfinite(d)) {
        if (!bad) bad = isfinite(d) ? 1 : 2;
      } else {
        piv = sqrt(d);
      }
      const double inv = 1.0 / piv;
      if (lane == j)
        a[j] = el_real(E{}, piv);
      else if (lane > j)
        a[j] = el_scale(a[j], inv);
#pragma unroll
      for (int k = j + 1; k < CB; ++k) {
        const E lkj = el_lane(a[j], k);
        if (lane >= k) a[k] = el_sub_mulc(a[k], a[j], lkj);
      }
    }
  }
  if (lane < CB)
#pragma unroll
    for (int k = 0; k < CB; ++k) Ls[lane][k] = a[k];
  if (lane < b)
#pragma unroll
    for (int k = 0; k < CB; ++k)
      if (k <= lane) M[(size_t)(p + lane) * n + p + k] = a[k];
  __syncthreads();
  // column c = lane of X: x[r] = (delta_rc - sum_{k<r} L[r][k] x[k]) / L[r][r] for the rows of
  // the block, zero beyond it
  E x[CB];
#pragma unroll
  for (int r = 0; r < CB; ++r) {
    E sum = el_real(E{}, r == lane ? 1.0 : 0.0);
#pragma unroll
    for (int k = 0; k < r; ++k) sum = el_sub_mul(sum, Ls[r][k], x[k]);
    x[r] = r < b ? el_scale(sum, 1.0 / el_re(Ls[r][r])) : z;
  }
  // W[c][r] = conj(X[r][c]): lane c writes row c
  if (lane < CB)
#pragma unroll
    for (int r = 0; r < CB; ++r) W[lane * CB + r] = el_conj_c(x[r]);
  if (lane == 0 && bad && *flag == 0) *flag = bad;
}

// One workgroup (one wave) per matrix of the batch; real[m] != 0 selects the real layout.
__global__ __launch_bounds__(64) void chol_diag_kernel(double *A, size_t stride, int n, int p, double *Wout,
                                                        int *flags, int flag_base, const int *real) {
  __shared__ double2 lds[CB * (CB + 1)];
  const int mtx = blockIdx.x;
  double2 *W = reinterpret_cast<double2 *>(Wout) + (size_t)mtx * CB * CB;
  if (real && real[mtx])
    chol_diag_block<double>(A + (size_t)mtx * stride, n, p, W, flags + flag_base + mtx, lds);
  else
    chol_diag_block<double2>(reinterpret_cast<double2 *>(A + (size_t)mtx * stride), n, p, W, flags + flag_base + mtx,
                             lds);
}

// Panel solve A21 <- A21 W for rows [p + CB, n) of every matrix (in place; each workgroup
// owns 64 whole rows of the panel).
__global__ __launch_bounds__(256) void chol_trsm_kernel(double *A, size_t stride, int n, int p,
                                                        const double *Win, const int *real) {
  __shared__ double2 W[CB][CB + 1];
  __shared__ double2 P[64][CB + 1];
  const int mtx = blockIdx.y;
  const bool rl = real && real[mtx];
  double2 *M = reinterpret_cast<double2 *>(A + (size_t)mtx * stride);
  double *Mr = A + (size_t)mtx * stride;
  const double2 *Wm = reinterpret_cast<const double2 *>(Win) + (size_t)mtx * CB * CB;
  const int r0 = p + CB + blockIdx.x * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < CB * CB; e += blockDim.x) W[e / CB][e % CB] = Wm[e];
  for (int e = tid; e < 64 * CB; e += blockDim.x) {
    const int r = e / CB, c = e % CB;
    const size_t o = (size_t)(r0 + r) * n + p + c;
    P[r][c] = (r0 + r < n) ? (rl ? make_double2(Mr[o], 0.0) : M[o]) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int e = tid; e < 64 * CB; e += blockDim.x) {
    const int r = e / CB, c = e % CB;
    if (r0 + r >= n) continue;
    const size_t o = (size_t)(r0 + r) * n + p + c;
    if (rl) {   // real matrix: the real parts only
      double s = 0.0;
      for (int k = 0; k < CB; ++k) s += P[r][k].x * W[k][c].x;
      Mr[o] = s;
      continue;
    }
    double2 s = make_double2(0.0, 0.0);
    for (int k = 0; k < CB; ++k) {
      const double2 a = P[r][k], w = W[k][c];
      s.x += a.x * w.x - a.y * w.y;
      s.y += a.x * w.y + a.y * w.x;
    }
    M[o] = s;
  }
}

__global__ void zero_upper_kernel(double *A, size_t stride, int n, const int *real) {
  const bool rl = real && real[blockIdx.y];
  double2 *M = reinterpret_cast<double2 *>(A + (size_t)blockIdx.y * stride);
  double *Mr = A + (size_t)blockIdx.y * stride;
  const size_t total = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / n, j = e % n;
    if (j > i) {
      if (rl)
        Mr[e] = 0.0;
      else
        M[e] = make_double2(0.0, 0.0);
    }
  }
}

// trB[m] = sum_i Re B_ii, then B <- I - B (lower triangle and diagonal).
__global__ __launch_bounds__(256) void trace_kernel(const double *B, size_t stride, int n, double *trB,
                                                    const int *real) {
  __shared__ double red[256];
  const bool rl = real && real[blockIdx.x];
  const double2 *M = reinterpret_cast<const double2 *>(B + (size_t)blockIdx.x * stride);
  const double *Mr = B + (size_t)blockIdx.x * stride;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += rl ? Mr[(size_t)i * n + i] : M[(size_t)i * n + i].x;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) trB[blockIdx.x] = red[0];
}

__global__ void identity_minus_kernel(double *B, size_t stride, int n, const int *real) {
  const bool rl = real && real[blockIdx.y];
  double2 *M = reinterpret_cast<double2 *>(B + (size_t)blockIdx.y * stride);
  double *Mr = B + (size_t)blockIdx.y * stride;
  const size_t total = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / n, j = e % n;
    if (j <= i && rl) {
      Mr[e] = (i == j ? 1.0 : 0.0) - Mr[e];
    } else if (j <= i) {
      double2 v = M[e];
      v.x = (i == j ? 1.0 : 0.0) - v.x;
      v.y = -v.y;
      M[e] = v;
    }
  }
}

// f[m] = 2 sum_i ln Re L_ii + trB[m]; flags non-finite results.
__global__ __launch_bounds__(256) void logdet_kernel(const double *A, size_t stride, int n, const double *trB,
                                                     double *f, int *flags, int flag_base, const int *real) {
  __shared__ double red[256];
  const bool rl = real && real[blockIdx.x];
  const double2 *M = reinterpret_cast<const double2 *>(A + (size_t)blockIdx.x * stride);
  const double *Mr = A + (size_t)blockIdx.x * stride;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += log(rl ? Mr[(size_t)i * n + i] : M[(size_t)i * n + i].x);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = 2.0 * red[0] + trB[blockIdx.x];
    f[blockIdx.x] = v;
    if (!isfinite(v) && flags[flag_base + blockIdx.x] == 0) flags[flag_base + blockIdx.x] = 2;
  }
}

// ecq[q] = sum_k w_k f[q][k] / (2 pi nq), ecq[nq] = sum_q ecq[q]; one workgroup.
__global__ __launch_bounds__(256) void quadrature_kernel(const double *f, const double *w, int nq, int nomega,
                                                         double *ecq) {
  __shared__ double part[256];
  const double scale = 1.0 / (2.0 * M_PI * nq);
  double tot = 0.0;
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < nomega; ++k) s += w[k] * f[(size_t)q * nomega + k];
    ecq[q] = s * scale;
    tot += s * scale;
  }
  part[threadIdx.x] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) t += part[i];
    ecq[nq] = t;
  }
}

// First nonzero status flag in index order: out[0] = its value (0 if none), out[1] = its index.
// One workgroup; each thread scans a strided range, the minimum index wins.
__global__ __launch_bounds__(256) void first_flag_kernel(const int *flags, int n, int *out) {
  __shared__ int best[256];
  int b = n;
  for (int e = threadIdx.x; e < n; e += blockDim.x)
    if (flags[e] != 0) {
      b = e;
      break;
    }
  best[threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = n;
    for (int i = 0; i < (int)blockDim.x; ++i) m = best[i] < m ? best[i] : m;
    out[0] = m < n ? flags[m] : 0;
    out[1] = m < n ? m : -1;
  }
}

__global__ void fill_int_kernel(int *p, size_t n, int v) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) p[e] = v;
}

// plain copy of n 4-byte words (16-byte vectors when both ends allow it); a kernel rather than
// a memcpy so that captured graphs hold kernel nodes only
__global__ void copy_words_kernel(unsigned *__restrict__ dst, const unsigned *__restrict__ src, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15) == 0) {
    const size_t n4 = n / 4;
    for (size_t e = t; e < n4; e += stride) reinterpret_cast<uint4 *>(dst)[e] = reinterpret_cast<const uint4 *>(src)[e];
    for (size_t e = 4 * n4 + t; e < n; e += stride) dst[e] = src[e];
  } else {
    for (size_t e = t; e < n; e += stride) dst[e] = src[e];
  }
}

}  // namespace

hipError_t launch_first_flag(const int *flags, int n, int *out, hipStream_t s) {
  hipLaunchKernelGGL(first_flag_kernel, dim3(1), dim3(256), 0, s, flags, n, out);
  return hipGetLastError();
}

hipError_t launch_fill_int(int *p, size_t n, int v, hipStream_t s) {
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(fill_int_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_real_flags(const double *X, int n, int nq, int nomega, int *real, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  hipError_t e = launch_fill_int(real, (size_t)nq, 1, s);
  if (e != hipSuccess || nomega <= 0 || n <= 0) return e;
  const size_t mat = (size_t)n * n * 2, per = (size_t)nomega * n * n;
  const int bx = (int)std::min<size_t>((per + 255) / 256, 2048);
  hipLaunchKernelGGL(real_flags_kernel, dim3(bx, nq), dim3(256), 0, s, X, mat, nq, nomega, real);
  return hipGetLastError();
}

hipError_t launch_copy_words(void *dst, const void *src, size_t nwords, hipStream_t s) {
  if (nwords == 0) return hipSuccess;
  const int blocks = (int)std::min<size_t>((nwords / 4 + 255) / 256 + 1, 4096);
  hipLaunchKernelGGL(copy_words_kernel, dim3(blocks), dim3(256), 0, s, (unsigned *)dst, (const unsigned *)src, nwords);
  return hipGetLastError();
}

hipError_t launch_zgemm(const ZgemmArgs &g, int batch, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || batch <= 0) return hipSuccess;
  // bytes of one block's operands as addressed (0 for an empty contraction): A is stored
  // M x K (opA = 0) or K x M, B is stored K x N (opB = 0) or N x K, rows ld elements apart
  const auto span = [&](int outer, int inner, long long ld) -> size_t {
    return g.K <= 0 ? 0 : ((size_t)(outer - 1) * ld + inner) * 16;
  };
  const size_t ba = g.opA == 0 ? span(g.M, g.K, g.lda) : span(g.K, g.M, g.lda);
  const size_t bb = g.opB == 0 ? span(g.K, g.N, g.ldb) : span(g.N, g.K, g.ldb);
  if (ba > 0xffff0000u || bb > 0xffff0000u) return hipErrorInvalidValue;   // 32-bit buffer views
  dim3 grid((g.N + ZB - 1) / ZB, (g.M + ZB - 1) / ZB, batch);
  const unsigned ua = (unsigned)ba, ub = (unsigned)bb;
  if (g.opA == 0 && g.opB == 0)
    hipLaunchKernelGGL((zgemm_kernel<0, 0>), grid, dim3(ZT), 0, s, g, ua, ub);
  else if (g.opA == 0)
    hipLaunchKernelGGL((zgemm_kernel<0, 1>), grid, dim3(ZT), 0, s, g, ua, ub);
  else if (g.opB == 0)
    hipLaunchKernelGGL((zgemm_kernel<1, 0>), grid, dim3(ZT), 0, s, g, ua, ub);
  else
    hipLaunchKernelGGL((zgemm_kernel<1, 1>), grid, dim3(ZT), 0, s, g, ua, ub);
  return hipGetLastError();
}

hipError_t launch_dgemm(const DgemmArgs &g, int batch, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || batch <= 0) return hipSuccess;
  const auto span = [&](int outer, int inner, long long ld) -> size_t {
    return g.K <= 0 ? 0 : ((size_t)(outer - 1) * ld + inner) * 8;
  };
  const size_t ba = g.opA == 0 ? span(g.M, g.K, g.lda) : span(g.K, g.M, g.lda);
  const size_t bb = g.opB == 0 ? span(g.K, g.N, g.ldb) : span(g.N, g.K, g.ldb);
  if (ba > 0xffff0000u || bb > 0xffff0000u) return hipErrorInvalidValue;   // 32-bit buffer views
  const unsigned ua = (unsigned)ba, ub = (unsigned)bb;
  if (g.N <= 32) {
    // narrow products (panel updates): 128 x 32 tiles
    dim3 grid(1, (g.M + DB - 1) / DB, batch);
    if (g.opA == 0 && g.opB == 0)
      hipLaunchKernelGGL((dgemm_kernel<0, 0, 32>), grid, dim3(DT), 0, s, g, ua, ub);
    else if (g.opA == 0)
      hipLaunchKernelGGL((dgemm_kernel<0, 1, 32>), grid, dim3(DT), 0, s, g, ua, ub);
    else if (g.opB == 0)
      hipLaunchKernelGGL((dgemm_kernel<1, 0, 32>), grid, dim3(DT), 0, s, g, ua, ub);
    else
      hipLaunchKernelGGL((dgemm_kernel<1, 1, 32>), grid, dim3(DT), 0, s, g, ua, ub);
    return hipGetLastError();
  }
  dim3 grid((g.N + DB - 1) / DB, (g.M + DB - 1) / DB, batch);
  if (g.opA == 0 && g.opB == 0)
    hipLaunchKernelGGL((dgemm_kernel<0, 0, 128>), grid, dim3(DT), 0, s, g, ua, ub);
  else if (g.opA == 0)
    hipLaunchKernelGGL((dgemm_kernel<0, 1, 128>), grid, dim3(DT), 0, s, g, ua, ub);
  else if (g.opB == 0)
    hipLaunchKernelGGL((dgemm_kernel<1, 0, 128>), grid, dim3(DT), 0, s, g, ua, ub);
  else
    hipLaunchKernelGGL((dgemm_kernel<1, 1, 128>), grid, dim3(DT), 0, s, g, ua, ub);
  return hipGetLastError();
}

hipError_t launch_pack_real(const double *src, long long outer, long long inner, int boff, int binner, int nmat,
                            double *dst, size_t dstride, size_t n2, const int *sel, hipStream_t s) {
  if (nmat <= 0 || n2 == 0) return hipSuccess;
  const int bx = (int)std::min<size_t>((n2 + 255) / 256, 1024);
  hipLaunchKernelGGL(pack_real_kernel, dim3(bx, nmat), dim3(256), 0, s, src, outer, inner, boff, binner, dst, dstride,
                     n2, sel);
  return hipGetLastError();
}

hipError_t launch_both_real(const int *realchi, const int *realv, int nq, int nomega, int *both, int *pair,
                            int *counts, hipStream_t s) {
  const int n = nq * std::max(nomega, 1);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(both_real_kernel, dim3((n + 255) / 256), dim3(256), 0, s, realchi, realv, nq, nomega, both, pair);
  hipLaunchKernelGGL(count_real_kernel, dim3(1), dim3(256), 0, s, realchi, realv, nq, counts);
  return hipGetLastError();
}

// In-place lower Cholesky of `batch` n x n complex matrices spaced `stride` doubles apart.
// Wscratch: batch * CB * CB complex; flags[flag_base + m] set non-zero on failure.
// Right-looking in blocks of np CB-wide panels: the panels of a block are factored in turn
// (diagonal block, panel solve), each after the block's earlier panels have updated its CB
// columns, then the trailing matrix takes one rank-(np CB) update.  The trailing update reads
// and writes the whole remaining matrix, so wider blocks cut that traffic (the diagonal-block
// kernel stays CB wide: its cost grows with the cube of the width).  Measured: 4 panels for
// n = 800 and 8 for n = 2400 (energy stage 124 -> 108 ms and 369 -> 304 ms against 1 panel),
// 16 for n = 7440 (404 -> 399 ms against 8).
static int chol_panels(int n) { return n >= 4096 ? 16 : (n >= 1536 ? 8 : 4); }
hipError_t launch_cholesky(double *A, size_t stride, int n, int batch, double *Wscratch, int *flags, int flag_base,
                           const int *real, hipStream_t s, int kinds) {
  hipError_t err = hipSuccess;
  // A[r0.., c0..c0+nc) -= A[r0.., k0..k0+K) A[c0..c0+nc, k0..k0+K)^H for rows r0 <= r < n: the
  // complex matrices by the complex GEMM, the real ones (if any) by the real GEMM
  auto update = [&](int r0, int c0, int nc, int k0, int K, int lower_only) -> hipError_t {
    if (real && (kinds & 2)) {
      DgemmArgs d{};
      d.M = n - r0;
      d.N = nc;
      d.K = K;
      d.A = A + (size_t)r0 * n + k0;
      d.lda = n;
      d.strideA = stride;
      d.opA = 0;
      d.B = A + (size_t)c0 * n + k0;
      d.ldb = n;
      d.strideB = stride;
      d.opB = 1;
      d.C = A + (size_t)r0 * n + c0;
      d.ldc = n;
      d.strideC = stride;
      d.alpha = -1.0;
      d.beta = 1.0;
      d.lower_only = lower_only;
      d.sel = real;
      const hipError_t e = launch_dgemm(d, batch, s);
      if (e != hipSuccess) return e;
    }
    if (!(kinds & 1)) return hipSuccess;
    ZgemmArgs g{};
    g.M = n - r0;
    g.N = nc;
    g.K = K;
    g.A = A + 2 * ((size_t)r0 * n + k0);
    g.lda = n;
    g.strideA = stride;
    g.opA = 0;
    g.B = A + 2 * ((size_t)c0 * n + k0);
    g.ldb = n;
    g.strideB = stride;
    g.opB = 1;
    g.C = A + 2 * ((size_t)r0 * n + c0);
    g.ldc = n;
    g.strideC = stride;
    g.alpha = -1.0;
    g.beta = 1.0;
    g.lower_only = lower_only;
    g.kmode = 0;
    g.skip = real;
    return launch_zgemm(g, batch, s);
  };
  auto panel = [&](int p) -> hipError_t {   // factor columns [p, p + CB) given all updates
    hipLaunchKernelGGL(chol_diag_kernel, dim3(batch), dim3(64), 0, s, A, stride, n, p, Wscratch, flags, flag_base,
                       real);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n - p - CB <= 0) return e;
    hipLaunchKernelGGL(chol_trsm_kernel, dim3((n - p - CB + 63) / 64, batch), dim3(256), 0, s, A, stride, n, p,
                       (const double *)Wscratch, real);
    return hipGetLastError();
  };
  const int np = chol_panels(n);
  for (int p = 0; p < n; p += np * CB) {
    for (int j = 0; j < np; ++j) {
      const int pj = p + j * CB;
      if (pj >= n) return hipSuccess;
      // the block's earlier panels' contribution to this panel's columns (rows pj..n; the
      // diagonal block's upper triangle takes values nothing reads)
      if (j > 0 && (err = update(pj, pj, std::min(CB, n - pj), p, j * CB, 0)) != hipSuccess) return err;
      if ((err = panel(pj)) != hipSuccess) return err;
    }
    const int t = p + np * CB;
    if (t >= n) break;
    // the whole block's contribution to the trailing matrix, lower triangle
    if ((err = update(t, t, n - t, p, np * CB, 1)) != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t launch_zero_upper(double *A, size_t stride, int n, int batch, const int *real, hipStream_t s) {
  const int blocks = (int)std::min<size_t>(((size_t)n * n + 255) / 256, 4096);
  hipLaunchKernelGGL(zero_upper_kernel, dim3(blocks, batch), dim3(256), 0, s, A, stride, n, real);
  return hipGetLastError();
}

hipError_t launch_trace_identity_minus(double *B, size_t stride, int n, int batch, double *trB, const int *real,
                                       hipStream_t s) {
  hipLaunchKernelGGL(trace_kernel, dim3(batch), dim3(256), 0, s, (const double *)B, stride, n, trB, real);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int blocks = (int)std::min<size_t>(((size_t)n * n + 255) / 256, 4096);
  hipLaunchKernelGGL(identity_minus_kernel, dim3(blocks, batch), dim3(256), 0, s, B, stride, n, real);
  return hipGetLastError();
}

hipError_t launch_logdet(const double *A, size_t stride, int n, int batch, const double *trB, double *f, int *flags,
                         int flag_base, const int *real, hipStream_t s) {
  hipLaunchKernelGGL(logdet_kernel, dim3(batch), dim3(256), 0, s, A, stride, n, trB, f, flags, flag_base, real);
  return hipGetLastError();
}

hipError_t launch_quadrature(const double *f, const double *w, int nq, int nomega, double *ecq, hipStream_t s) {
  hipLaunchKernelGGL(quadrature_kernel, dim3(1), dim3(256), 0, s, f, w, nq, nomega, ecq);
  return hipGetLastError();
}
