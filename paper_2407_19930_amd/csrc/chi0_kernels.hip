// chi(R, tau) build for gfx950 (Sec. 2 chi0 matrix formula, Algorithm 1).
//
// Algorithm 1 is evaluated through its N intermediate only:
//   N^{s,nu}_{jk}(V, K, dR) = sum_{L(dL) in N[V]} sum_l C^nu_{jl}(V, L, dL) G^s_{lk}(dR - dL)
// For real Green's functions with G^s(-R) = G^s(R)^T the other intermediates are
// views of N:  X^{s,nu}_{ij}(U, V, R) = N^{s,nu}_{ji}(V, U, -R), and the Z terms summed
// over K(R1) equal sum_ij X^{s,nu}_{ij}(U,V,R) N^{s',mu}_{ij}(U,V,R).  Hence
//   chi_{mu nu}(U, V, R) = -s [ sum_{K(R1) in N[U]} sum_{ik} C^mu_{ik}(R1) O^nu_{ik}
//                               + sum_{ij} ( N^{occ,mu}_{ij}(U,V,R) N^{un,nu}_{ji}(V,U,-R)
//                                           + N^{un,mu}_{ij}(U,V,R) N^{occ,nu}_{ji}(V,U,-R) ) ]
//   O^nu_{ik} = sum_j G^un_{ij}(R) N^{occ,nu}_{jk}(V,K,R1-R) + G^occ_{ij}(R) N^{un,nu}_{jk}(V,K,R1-R)
//
// Kernels:
//   pack_c    : LRI blocks [mu][i][k] (FP64) -> [k][i][mu] in the compute precision
//   nstage    : N for every (V, K, dR, s): a GEMM whose A operand gathers rows of G
//   fused     : one workgroup per (U <= V, R): Z terms, then the K(R1) loop of
//               O = [G^un | G^occ](R) [N^occ ; N^un] (MFMA) feeding chi += C O (MFMA)
//               straight from the accumulator registers; writes chi_UV(R) and its
//               Hermitian partner chi_VU(-R) = chi_UV(R)^T.
#include "chi0_kernels.h"
#include "item_table.h"

namespace {

template <typename T>
__global__ __launch_bounds__(256) void pack_c_kernel(PackTables pt, const double *__restrict__ C,
                                                     T *__restrict__ Cp) {
  // block b: [mu][i][k] (FP64) -> [k][(i, mu)] with rows padded to stride[b] (zeros)
  const int b = blockIdx.x;
  const int a = pt.a[b], ni = pt.ni[b], nk = pt.nk[b], st = pt.stride[b];
  const int rowlen = a * ni;
  const long long total = (long long)nk * st;
  const double *src = C + pt.in_off[b];
  T *dst = Cp + pt.out_off[b];
  for (long long e = (long long)blockIdx.y * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.y * blockDim.x) {
    const int k = (int)(e / st);
    const int w = (int)(e - (long long)k * st);
    T v = T(0);
    if (w < rowlen) {
      const int i = w / a, mu = w - i * a;
      v = (T)src[((long long)mu * ni + i) * nk + k];
    }
    dst[e] = v;
  }
}

// Per-tau scale of G (north of the FP32 subnormal range for any tau): partial maxima of |G^s|,
// then one block turns them into the exponents e_s with max |G^s| 2^e_s in [1, 2).
constexpr int GS_THREADS = 256;
__global__ __launch_bounds__(GS_THREADS) void gmax_kernel(const double *__restrict__ Gocc,
                                                          const double *__restrict__ Gun, size_t n,
                                                          double *__restrict__ part) {
  __shared__ double red[2][GS_THREADS];
  double m0 = 0.0, m1 = 0.0;
  for (size_t e = (size_t)blockIdx.x * GS_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * GS_THREADS) {
    m0 = fmax(m0, fabs(Gocc[e]));
    m1 = fmax(m1, fabs(Gun[e]));
  }
  red[0][threadIdx.x] = m0;
  red[1][threadIdx.x] = m1;
  __syncthreads();
  for (int h = GS_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + h]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 2) part[threadIdx.x * kGscaleBlocks + blockIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kGscaleBlocks) void gexp_kernel(const double *__restrict__ part, int *__restrict__ gexp) {
  __shared__ double red[2][kGscaleBlocks];
  red[0][threadIdx.x] = part[threadIdx.x];
  red[1][threadIdx.x] = part[kGscaleBlocks + threadIdx.x];
  __syncthreads();
  for (int h = kGscaleBlocks / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + h]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 2) {
    const double m = red[threadIdx.x][0];
    int x = 1;
    if (m > 0.0 && isfinite(m)) frexp(m, &x);   // m = f 2^x, f in [0.5, 1)
    gexp[threadIdx.x] = 1 - x;
  }
}

// G^occ, G^un of one tau (FP64, [nR][nb][nb] each) -> Gp[s][R][nbp][nbp] = G^s 2^gexp[s] in the
// compute precision (no scale for a null gexp), s = 0 occ, 1 un, zero padding up to nbp (a
// multiple of 8).
template <typename T>
__global__ __launch_bounds__(256) void pad_g_kernel(const double *__restrict__ Gocc, const double *__restrict__ Gun,
                                                    int nR, int nb, int nbp, const int *__restrict__ gexp,
                                                    T *__restrict__ Gp) {
  const double sc0 = gexp ? ldexp(1.0, gexp[0]) : 1.0, sc1 = gexp ? ldexp(1.0, gexp[1]) : 1.0;
  const size_t total = (size_t)2 * nR * nbp * nbp;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % nbp);
    const size_t t = e / nbp;
    const int r = (int)(t % nbp);
    const size_t sR = t / nbp;
    const int R = (int)(sR % nR), s = (int)(sR / nR);
    T v = T(0);
    if (r < nb && c < nb) v = (T)((s ? Gun : Gocc)[((size_t)R * nb + r) * nb + c] * (s ? sc1 : sc0));
    Gp[e] = v;
  }
}

// ---------------------------------------------------------------------------
// N-stage: out[(s, dR, k)][(j, nu)] = sum_r A[(s,dR,k)][r] B[r][(j,nu)]
//   A[(s,dR,k)][r] = Gp[s][dR - dL(r)][g(r)][k],  B[r][(j,nu)] = Cp[cp(r) + j*a_V + nu]
// Rows (s, dR, k) run over the padded NAO range nbp (multiple of 8), so every 8-row chunk
// lies in one (s, dR) and in one padded G row; packed C rows are padded to a multiple of 8.
// Each thread loads, per contraction row, 8 consecutive elements of A and of B with 16-byte
// vector loads.  128x128 output tile, 4 waves of 64x64 (16x16x4 MFMA), K step BK, LDS
// double buffer with a padded row stride (conflict-free MFMA operand reads).
// kSplit: the partial sums of every 256 contraction rows are added into a second accumulator
// of type A2 (rounding error growing with sqrt(256) + sqrt(S/256) instead of sqrt(S) for S
// contraction rows); not used by the launchers, since its registers halve the occupancy.
// ---------------------------------------------------------------------------
constexpr int NS_BM = 128, NS_BN = 128, NS_THREADS = 256;

template <typename T> struct alignas(16) Vec16 {
  T v[16 / sizeof(T)];
};

// kBuf: the K loop reads its row records with scalar loads (the 4 rows of a wave's lanes) and A
// and B through raw buffer views of Gp and Cp (gp_bytes, cp_bytes below 2^32), unconditionally:
// rows past the contraction or tiles past M or N address the view's end and read zero, so the
// compiler keeps the next step's loads in flight across the MFMAs.  Without kBuf the loads are
// masked by branches, and the compiler then waits for them before the MFMAs.
template <typename T, bool kSplit, int BK, typename A2, bool kBuf>
__global__ __launch_bounds__(NS_THREADS) void nstage_kernel(Chi0Tables tb, NTiles tiles, const T *__restrict__ Gp,
                                                            const T *__restrict__ Cp, T *__restrict__ Nbuf,
                                                            unsigned gp_bytes, unsigned cp_bytes) {
  typedef typename Mfma<T>::acc Acc;
  constexpr int PAD = sizeof(T) == 4 ? 16 : 8;
  constexpr int RPT = BK / 16;                 // contraction rows per thread and step
  constexpr int VEC = 16 / sizeof(T);          // elements per 16-byte vector
  constexpr int NVEC = 8 / VEC;                // vectors per 8-element chunk
  constexpr int kFlush = 256 / BK;
  __shared__ __align__(16) T As[2][BK][NS_BM + PAD];
  __shared__ __align__(16) T Bs[2][BK][NS_BN + PAD];

  const int t = blockIdx.x;
  const int V = tiles.V[t], m0 = tiles.m0[t], n0 = tiles.n0[t];
  const int nV = tb.nao[V], aV = tb.naux[V];
  const int NV = nV * aV, NVp = tb.cp_stride[V];
  const int nbp = tb.nbp, nR = tb.nR, nb = tb.nb;
  const size_t plane = (size_t)nbp * nbp;
  const int M = 2 * nR * nbp;
  const int r0 = tb.rows_start[V];
  const int S = tb.rows_start[V + 1] - r0;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int col = lane & 15, grp = lane >> 4;

  // loader coordinates: chunk c of 8 rows/columns, contraction rows rr + 16 q
  const int c = tid & 15, rr = tid >> 4;
  const int m = m0 + 8 * c;
  const bool mvalid = m < M;
  int ss = 0, d0 = 0, d1 = 0, d2 = 0, kp = 0;
  if (mvalid) {
    ss = m / (nR * nbp);
    const int rem = m - ss * nR * nbp;
    const int dR = rem / nbp;
    kp = rem - dR * nbp;
    tb.bvk.split(dR, d0, d1, d2);
  }
  const int n0m = tb.bvk.n0, n1m = tb.bvk.n1, n2m = tb.bvk.n2;
  const T *Abase = Gp + (size_t)ss * nR * plane + kp;
  const int n = n0 + 8 * c;
  const bool nvalid = n < NVp;
  const T *Bbase = Cp + n;

  Vec16<T> ra[RPT][NVEC], rb[RPT][NVEC];
  const __amdgpu_buffer_rsrc_t gview = buffer_view(Gp, gp_bytes), cview = buffer_view(Cp, cp_bytes);
  const size_t abase = (size_t)ss * nR * plane + kp;
  // row records of a K step (one per contraction row of this thread), loaded one step ahead
  // of the data they address; the index is clamped so that the load is unconditional
  auto load_ri = [&](int k0, int4 (&dst)[RPT]) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = k0 + rr + 16 * q;
      dst[q] = tb.row_info[r0 + max(min(r, S - 1), 0)];
    }
  };
  auto load_buf = [&](int k0, const int4 (&rix)[RPT]) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int4 ri = rix[q];
      const bool rvalid = k0 + rr + 16 * q < S;
      int c0 = d0 - (ri.y & 1023), c1 = d1 - ((ri.y >> 10) & 1023), c2 = d2 - (ri.y >> 20);
      c0 += c0 < 0 ? n0m : 0;
      c1 += c1 < 0 ? n1m : 0;
      c2 += c2 < 0 ? n2m : 0;
      const int Rp = (c0 * n1m + c1) * n2m + c2;
      const unsigned ia = (unsigned)((abase + (size_t)Rp * plane + (size_t)ri.x * nbp) * sizeof(T));
      const unsigned ib = (unsigned)((((long long)(unsigned)ri.z | ((long long)ri.w << 32)) + n) * sizeof(T));
      const unsigned oa = (rvalid & mvalid) ? ia : gp_bytes;
      const unsigned ob = (rvalid & nvalid) ? ib : cp_bytes;
#pragma unroll
      for (int v = 0; v < NVEC; ++v) {
        ra[q][v] = __builtin_bit_cast(Vec16<T>, __builtin_amdgcn_raw_buffer_load_b128(gview, oa + 16 * v, 0, 0));
        rb[q][v] = __builtin_bit_cast(Vec16<T>, __builtin_amdgcn_raw_buffer_load_b128(cview, ob + 16 * v, 0, 0));
      }
    }
  };
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = k0 + rr + 16 * q;
#pragma unroll
      for (int v = 0; v < NVEC; ++v)
#pragma unroll
        for (int x = 0; x < VEC; ++x) ra[q][v].v[x] = rb[q][v].v[x] = T(0);
      if (r < S) {
        const int4 ri = tb.row_info[r0 + r];
        if (mvalid) {
          int c0 = d0 - (ri.y & 1023), c1 = d1 - ((ri.y >> 10) & 1023), c2 = d2 - (ri.y >> 20);
          c0 += c0 < 0 ? n0m : 0;
          c1 += c1 < 0 ? n1m : 0;
          c2 += c2 < 0 ? n2m : 0;
          const int Rp = (c0 * n1m + c1) * n2m + c2;
          const Vec16<T> *src = reinterpret_cast<const Vec16<T> *>(Abase + (size_t)Rp * plane + (size_t)ri.x * nbp);
#pragma unroll
          for (int v = 0; v < NVEC; ++v) ra[q][v] = src[v];
        }
        if (nvalid) {
          const Vec16<T> *src =
              reinterpret_cast<const Vec16<T> *>(Bbase + ((long long)(unsigned)ri.z | ((long long)ri.w << 32)));
#pragma unroll
          for (int v = 0; v < NVEC; ++v) rb[q][v] = src[v];
        }
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
      for (int v = 0; v < NVEC; ++v) {
        *reinterpret_cast<Vec16<T> *>(&As[buf][rr + 16 * q][8 * c + v * VEC]) = ra[q][v];
        *reinterpret_cast<Vec16<T> *>(&Bs[buf][rr + 16 * q][8 * c + v * VEC]) = rb[q][v];
      }
  };

  Acc acc[4][4];
  A2 acc64[4][4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      acc[a][b] = Mfma<T>::zero();
      if (kSplit)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[a][b][r] = 0.0;
    }

  const int nk = (S + BK - 1) / BK;
  int4 ri_next[RPT];
  if (kBuf) {
    int4 ri0[RPT];
    load_ri(0, ri0);
    load_buf(0, ri0);
    load_ri(BK, ri_next);
  } else {
    load(0);
  }
  store(0);
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (kBuf) {
      // data of step it + 1 (past the last step it reads zero) and the records of step it + 2
      load_buf((it + 1) * BK, ri_next);
      load_ri((it + 2) * BK, ri_next);
      // keep the prefetch ahead of the MFMAs (the scheduler would sink it below them)
      __builtin_amdgcn_sched_barrier(0);
    } else if (it + 1 < nk) {
      load((it + 1) * BK);
    }
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      T a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[cur][ks * 4 + grp][wm * 64 + q * 16 + col];
        b[q] = Bs[cur][ks * 4 + grp][wn * 64 + q * 16 + col];
      }
#pragma unroll
      for (int tm = 0; tm < 4; ++tm)
#pragma unroll
        for (int tn = 0; tn < 4; ++tn) acc[tm][tn] = Mfma<T>::fma(a[tm], b[tn], acc[tm][tn]);
    }
    if (kSplit && (((it + 1) % kFlush) == 0 || it + 1 == nk)) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[a][b][r] += (A2)acc[a][b][r];
          acc[a][b] = Mfma<T>::zero();
        }
    }
    // kBuf: unconditional (past the last step it stores the zeros it loaded into a buffer that
    // is not read again), so that the compiler cannot sink the prefetch into a branch
    if (kBuf || it + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  // epilogue: scatter rows (s, dR, k) into N blocks (V, K(k), dR), layout [k][s][j][nu]
#pragma unroll
  for (int tm = 0; tm < 4; ++tm) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mm = m0 + wm * 64 + tm * 16 + Mfma<T>::row(grp, r);
      if (mm >= M) continue;
      const int s2 = mm / (nR * nbp);
      const int rem = mm - s2 * nR * nbp;
      const int dR2 = rem / nbp;
      const int k2 = rem - dR2 * nbp;
      if (k2 >= nb) continue;
      const int K = tb.atom_of_ao[k2];
      const int kl = k2 - tb.ao_off[K];
      T *dst = Nbuf + tb.noff[((size_t)V * tb.natoms + K) * nR + dR2] + (size_t)(kl * 2 + s2) * NV;
#pragma unroll
      for (int tn = 0; tn < 4; ++tn) {
        const int nn = n0 + wn * 64 + tn * 16 + col;
        if (nn < NV) dst[nn] = kSplit ? (T)acc64[tm][tn][r] : (T)acc[tm][tn][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// fused M + chi + Z kernel, one workgroup (8 waves) per item (U <= V, R).
// Wave w owns ABF columns nu in [16w, 16w+16) of V and all MT mu-tiles of U.
// Per slice (neighbour K(R1), NAO k of K):
//   O[i][nu] = sum_j' A[i][j'] N[k][j'][nu]   (JS MFMA K-steps, A = [G^un | G^occ](R) in registers)
//   chi[mu][nu] += sum_i C[k][i][mu] O[i][nu] (O straight from the accumulator registers)
// The C slice is staged in LDS mu-major with the i index laid out so that the four
// contraction rows an accumulator register set covers are adjacent (one 16-byte read);
// padding rows/columns stay zero.  N rows of the next slice are prefetched into
// registers, the next C slice through registers into the other LDS buffer.
// ---------------------------------------------------------------------------
constexpr int FU_THREADS = 512;
constexpr int FU_MAXNBR = 1024;
constexpr int FU_LOADS = kMaxNao * kMaxNaux / FU_THREADS;

template <typename T> struct Lds;
template <> struct Lds<float> {
  static constexpr int IP = 36;   // padded i extent per mu row (16-byte aligned rows)
  static __device__ __forceinline__ int slot(int i) { return i; }
  static __device__ __forceinline__ void read4(const float *p, float c[4]) {
    const float4 v = *reinterpret_cast<const float4 *>(p);
    c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
  }
};
template <> struct Lds<double> {
  static constexpr int IP = 34;
  // register r of lane group g covers row g + 4r: place it at slot 4g + r
  static __device__ __forceinline__ int slot(int i) { return 16 * (i / 16) + 4 * (i % 4) + (i % 16) / 4; }
  static __device__ __forceinline__ void read4(const double *p, double c[4]) {
    const double2 a = *reinterpret_cast<const double2 *>(p);
    const double2 b = *reinterpret_cast<const double2 *>(p + 2);
    c[0] = a.x; c[1] = a.y; c[2] = b.x; c[3] = b.y;
  }
};

template <typename T, bool kSplit, int MT, int JS, int HC>
__global__ __launch_bounds__(FU_THREADS) void fused_kernel(Chi0Tables tb, PairItems items,
                                                           const T *__restrict__ Gp,
                                                           const T *__restrict__ Cp,
                                                           const T *__restrict__ Nbuf, double negs,
                                                           const int *__restrict__ gexp, Screen sc,
                                                           double *__restrict__ chi) {
  typedef typename Mfma<T>::acc Acc;
  constexpr int IP = Lds<T>::IP;
  constexpr int CG = sizeof(T) == 4 ? 4 : 1;    // mu-tiles per group of C fragment reads
  // two C slice buffers; the element after them takes the stores of idle threads
  __shared__ __align__(16) T Cs[2 * kMaxNaux * IP + 4];
  __shared__ long long nbr_c[FU_MAXNBR], nbr_n[FU_MAXNBR];
  __shared__ int nbr_k[FU_MAXNBR], nbr_g[FU_MAXNBR], nbr_pos[FU_MAXNBR + 1], nbr_meta[3];

  const int item = blockIdx.x;
  const int U = items.U[item], V = items.V[item], R = items.R[item];
  const int nU = tb.nao[U], aU = tb.naux[U], nV = tb.nao[V], aV = tb.naux[V];
  const int natoms = tb.natoms, nR = tb.nR, nbp = tb.nbp;
  const size_t plane = (size_t)nbp * nbp;
  const int tid = threadIdx.x, lane = tid & 63, w = uniform(tid >> 6);
  const int col = lane & 15, grp = lane >> 4;
  const int nu = w * 16 + col;
  const bool wave_active = w * 16 < aV;
  const bool nu_ok = nu < aV;
  const int hc = HC;                          // i-tiles of U (nU <= 16 HC)
  // neighbour table of this item (the entries whose M terms the screening keeps; all without
  // screening) and zeroed C buffers
  const int3 kept =
      item_table<FU_THREADS>(tb, sc, tb.nbr_cp, tb.noff, U, V, R, nbr_c, nbr_n, nbr_k, nbr_g, nbr_pos, nbr_meta);
  const int ne = kept.x;
  item_stats(sc, blockIdx.x, kept);
  for (int e = tid; e < 2 * kMaxNaux * IP + 4; e += FU_THREADS) Cs[e] = T(0);

  // A operand of the O GEMM: A[i][j'] = G^un_ij(R) for j' = j, G^occ_ij(R) for j' = nV + j
  T afr[HC][JS];
#pragma unroll
  for (int h = 0; h < HC; ++h)
#pragma unroll
    for (int st = 0; st < JS; ++st) {
      T v = T(0);
      const int i = 16 * h + col, jp = 4 * st + grp;
      if (h < hc && i < nU && jp < 2 * nV) {
        const int s = jp >= nV;                  // j' < nV pairs with N^occ and takes G^un
        const int j = jp - s * nV;
        v = Gp[(size_t)(1 - s) * nR * plane + (size_t)R * plane + (size_t)(tb.ao_off[U] + i) * nbp + tb.ao_off[V] + j];
      }
      afr[h][st] = v;
    }

  Acc acc[MT];
  double acc64[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    acc[m] = Mfma<T>::zero();
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[m][r] = 0.0;
  }
  auto flush = [&]() {
    if (kSplit) {
#pragma unroll
      for (int m = 0; m < MT; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[m][r] += (double)acc[m][r];
        acc[m] = Mfma<T>::zero();
      }
    }
  };

  // ---- Z terms: contraction over (s, i, j) of N(U,V,R)[j][s][i][mu] and N(V,U,-R)[i][1-s][j][nu]
  const int negR = tb.bvk.neg(R);
  {
    const T *NA = Nbuf + uniform(tb.noff[((size_t)U * natoms + V) * nR + R]);
    const T *NB = Nbuf + uniform(tb.noff[((size_t)V * natoms + U) * nR + negR]);
    if (wave_active && kept.z) {
      const int F = 2 * nU * nV;
      // views of the two N blocks (elements outside them read zero): the loads of ZB iterations
      // are issued together and waited for once; each accumulator sees the same MFMA sequence
      const unsigned endA = (unsigned)((size_t)nV * 2 * nU * aU * sizeof(T));
      const unsigned endB = (unsigned)((size_t)nU * 2 * nV * aV * sizeof(T));
      const __amdgpu_buffer_rsrc_t vA = buffer_view(NA, endA), vB = buffer_view(NB, endB);
      constexpr int ZB = sizeof(T) == 4 ? 4 : 2;
      for (int f0 = 0; f0 < F; f0 += 4 * ZB) {
        T bz[ZB], az[ZB][MT];
#pragma unroll
        for (int u = 0; u < ZB; ++u) {
          const int f = f0 + 4 * u + grp;
          const bool fv = f < F;
          const int fc = fv ? f : 0;
          const int s = fc / (nU * nV);
          const int rem = fc - s * nU * nV;
          const int i = rem / nV, j = rem - i * nV;
          const unsigned ob =
              (fv && nu_ok) ? (unsigned)((((i * 2 + 1 - s) * nV + j) * aV + nu) * sizeof(T)) : endB;
          bz[u] = buffer_load<T>(vB, ob);
#pragma unroll
          for (int m = 0; m < MT; ++m) {
            const int mu = 16 * m + col;
            const unsigned oa =
                (fv && mu < aU) ? (unsigned)((((j * 2 + s) * nU + i) * aU + mu) * sizeof(T)) : endA;
            az[u][m] = buffer_load<T>(vA, oa);
          }
        }
#pragma unroll
        for (int u = 0; u < ZB; ++u)
#pragma unroll
          for (int m = 0; m < MT; ++m) acc[m] = Mfma<T>::fma(az[u][m], bz[u], acc[m]);
      }
    }
    flush();
  }
  __syncthreads();   // neighbour table and zeroed buffers visible

  // per-thread LDS destinations of the slice elements (same for every slice of this item);
  // the 4-slot groups of mu-row mu are XOR-swizzled by (mu / 16) % 4 so that the 64 lanes of
  // a store hit distinct banks while a register set still reads one aligned 16-byte group.
  // Threads past the slice store to the spare element.
  const int sliceN = nU * aU;
  const int sliceStride = tb.cp_stride[U];
  constexpr int kSpare = 2 * kMaxNaux * IP;
  int soff[FU_LOADS];
#pragma unroll
  for (int q = 0; q < FU_LOADS; ++q) {
    const int idx = tid + q * FU_THREADS;
    soff[q] = kSpare;
    if (idx < sliceN) {
      const int i = idx / aU, mu = idx - i * aU;
      soff[q] = mu * IP + (Lds<T>::slot(i) ^ (4 * ((mu >> 4) & 3)));
    }
  }
  T rc[FU_LOADS];
  auto load_slice = [&](const T *src) {
    const __amdgpu_buffer_rsrc_t r = buffer_view(src, (unsigned)(sliceN * sizeof(T)));
#pragma unroll
    for (int q = 0; q < FU_LOADS; ++q) rc[q] = buffer_load<T>(r, (unsigned)((tid + q * FU_THREADS) * sizeof(T)));
  };
  auto store_slice = [&](int buf) {
    T *dst = Cs + buf * (kMaxNaux * IP);
#pragma unroll
    for (int q = 0; q < FU_LOADS; ++q) (soff[q] == kSpare ? Cs : dst)[soff[q]] = rc[q];
  };
  // N rows of the O GEMM: two register sets used in turn (the loop body is unrolled twice so
  // that no register copy forces a wait on the loads just issued for the next slice).  Rows
  // j' >= 2 nV read zero (their A columns are zero too); columns nu >= aV are never stored.
  const size_t nstride = (size_t)2 * nV * aV;
  T nbA[JS], nbB[JS];
  // (idle waves get an empty view: their loads return zero without a memory access, and the
  // loads stay unconditional so that the wait counts after them are exact)
  const unsigned nview = wave_active ? (unsigned)(nstride * sizeof(T)) : 0u;
  auto load_n = [&](const T *nrow, T *dst) {
    const __amdgpu_buffer_rsrc_t r = buffer_view(nrow, nview);
#pragma unroll
    for (int st = 0; st < JS; ++st) dst[st] = buffer_load<T>(r, (unsigned)(((4 * st + grp) * aV + nu) * sizeof(T)));
  };
  // Slice order: the entries e of U's neighbourhood come in runs [g0, g1) of one atom K (its
  // periodic images R1); a run is walked NAO k outer, image inner, so that the workgroups of
  // one atom pair at different R read the N rows N(V, K, .)[k] at about the same time and
  // share them in L2.  Partial sums are folded into FP64 at the end of a pass over the images
  // once kFoldSlices slices have been added since the last fold, and at the end of each run.
  int e = 0, k = 0, cur = 0, g0 = 0, g1 = 0, run = 0;
  // one slice: prefetch C and N of the next slice (slice (0, 0) again after the last),
  // O GEMM, chi += C O, stage the next C slice, barrier.  The loop runs over pairs of slices;
  // the second slice of the last pair may be past the end, and then only its GEMMs are
  // skipped: loads, stores and barriers run on every path so that the wait counts the
  // compiler derives are exact and the prefetch stays in flight across the barrier.
  auto slice = [&](const T *nbcur, T *nbnext, bool live) __attribute__((always_inline)) {
    int e2 = e, k2 = k;
    bool pass_end = false, fold = false;
    if (live) {
      e2 = e + 1;
      ++run;
      if (e2 == g1) {
        pass_end = true;
        e2 = g0;
        k2 = k + 1;
        if (k2 == uniform(nbr_k[g0])) {
          k2 = 0;
          e2 = g1;
        }
        fold = e2 == g1 || run >= kFoldSlices;
        if (fold) run = 0;
      }
    }
    // past the last slice the loads go to slice (0, 0), which every item has (ne > 0)
    const bool more = e2 < ne;
    const int ea = more ? e2 : 0, ka = more ? k2 : 0;
    load_slice(Cp + uniform(nbr_c[ea]) + (size_t)ka * sliceStride);
    load_n(Nbuf + uniform(nbr_n[ea]) + (size_t)ka * nstride, nbnext);
    // keep the prefetch ahead of the GEMMs (the scheduler would otherwise sink it to shorten
    // register lifetimes, and the next slice would wait for it)
    __builtin_amdgcn_sched_barrier(0);
    if (live && wave_active) {
      Acc o[HC];
#pragma unroll
      for (int h = 0; h < HC; ++h) o[h] = Mfma<T>::zero();
#pragma unroll
      for (int st = 0; st < JS; ++st)
#pragma unroll
        for (int h = 0; h < HC; ++h) o[h] = Mfma<T>::fma(afr[h][st], nbcur[st], o[h]);
      const T *cs = Cs + cur * (kMaxNaux * IP) + col * IP;
      // C fragments of CG mu-tiles are read first, then their MFMAs issued round-robin over
      // the tiles so that consecutive MFMAs never wait on each other's accumulator
#pragma unroll
      for (int h = 0; h < HC; ++h)
#pragma unroll
        for (int m0 = 0; m0 < MT; m0 += CG) {
          T c[CG][4];
#pragma unroll
          for (int m = m0; m < m0 + CG && m < MT; ++m)
            Lds<T>::read4(cs + 16 * m * IP + 16 * h + 4 * (grp ^ (m & 3)), c[m - m0]);
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int m = m0; m < m0 + CG && m < MT; ++m) acc[m] = Mfma<T>::fma(c[m - m0][r], o[h][r], acc[m]);
        }
    }
    if (fold) flush();
    store_slice(cur ^ 1);
    __syncthreads();
    if (pass_end && e2 == g1) {
      g0 = g1;
      g1 = more ? uniform(nbr_g[ea]) : g1;
    }
    e = e2;
    k = k2;
    cur ^= 1;
  };

  const int nsl = kept.y;
  if (ne > 0) {
    load_slice(Cp + uniform(nbr_c[0]));
    store_slice(0);
    load_n(Nbuf + uniform(nbr_n[0]), nbA);
    __syncthreads();
    g1 = uniform(nbr_g[0]);
    for (int t = 0; t < nsl; t += 2) {
      slice(nbA, nbB, true);
      slice(nbB, nbA, t + 1 < nsl);
    }
  }

  // ---- epilogue: chi_UV(R) and chi_VU(-R) = chi_UV(R)^T, G scale removed
  if (!wave_active || !nu_ok) return;
  const double scale = gexp ? ldexp(negs, -(gexp[0] + gexp[1])) : negs;
  const size_t N = tb.nauxtot;
  const int au0 = tb.aux_off[U], av0 = tb.aux_off[V];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mu = 16 * m + Mfma<T>::row(grp, r);
      if (mu < aU) {
        const double v = scale * (kSplit ? acc64[m][r] : (double)acc[m][r]);
        chi[((size_t)R * N + au0 + mu) * N + av0 + nu] = v;
        if (U != V) chi[((size_t)negR * N + av0 + nu) * N + au0 + mu] = v;
      }
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_pack_c(const PackTables &pt, const double *C, T *Cp, long long maxblk, hipStream_t s) {
  if (pt.nblk == 0) return hipSuccess;
  const int ychunks = (int)((maxblk + 256 * 16 - 1) / (256 * 16));
  dim3 grid(pt.nblk, ychunks > 0 ? ychunks : 1);
  hipLaunchKernelGGL(pack_c_kernel<T>, grid, dim3(256), 0, s, pt, C, Cp);
  return hipGetLastError();
}

hipError_t launch_gscale(const double *Gocc, const double *Gun, size_t n, double *part, int *gexp, hipStream_t s) {
  hipLaunchKernelGGL(gmax_kernel, dim3(kGscaleBlocks), dim3(GS_THREADS), 0, s, Gocc, Gun, n, part);
  hipLaunchKernelGGL(gexp_kernel, dim3(1), dim3(kGscaleBlocks), 0, s, part, gexp);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pad_g(const double *Gocc, const double *Gun, int nR, int nb, int nbp, const int *gexp, T *Gp,
                        hipStream_t s) {
  const size_t n = (size_t)2 * nR * nbp * nbp;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(pad_g_kernel<T>, dim3(blocks), dim3(256), 0, s, Gocc, Gun, nR, nb, nbp, gexp, Gp);
  return hipGetLastError();
}

template <typename T, int BK>
static void launch_nstage_bk(const Chi0Tables &tb, const NTiles &tiles, const T *Gp, const T *Cp, T *Nbuf,
                             size_t gp_bytes, size_t cp_bytes, hipStream_t s) {
  constexpr size_t kViewMax = 0xffff0000u;
  if (gp_bytes <= kViewMax && cp_bytes <= kViewMax)
    hipLaunchKernelGGL((nstage_kernel<T, false, BK, T, true>), dim3(tiles.count), dim3(NS_THREADS), 0, s, tb, tiles,
                       Gp, Cp, Nbuf, (unsigned)gp_bytes, (unsigned)cp_bytes);
  else
    hipLaunchKernelGGL((nstage_kernel<T, false, BK, T, false>), dim3(tiles.count), dim3(NS_THREADS), 0, s, tb, tiles,
                       Gp, Cp, Nbuf, 0u, 0u);
}

template <typename T>
hipError_t launch_nstage(const Chi0Tables &tb, const NTiles &tiles, const T *Gp, const T *Cp, T *Nbuf,
                         size_t cp_elems, int kstep, hipStream_t s) {
  if (tiles.count == 0) return hipSuccess;
  // plain accumulation in T over the contraction (about 5000 rows on the 8-atom cell): a
  // second accumulator level needs 64 or 128 more registers per lane and halves the occupancy.
  // K step 16 (FP32: 37 KB of LDS tiles, four workgroups per CU) or 32 (twice the LDS, half
  // the barriers); the plan's tuning picks one, 16 by default.
  const size_t gp_bytes = (size_t)2 * tb.nR * tb.nbp * tb.nbp * sizeof(T), cp_bytes = cp_elems * sizeof(T);
  if (kstep == 32)
    launch_nstage_bk<T, 32>(tb, tiles, Gp, Cp, Nbuf, gp_bytes, cp_bytes, s);
  else
    launch_nstage_bk<T, 16>(tb, tiles, Gp, Cp, Nbuf, gp_bytes, cp_bytes, s);
  return hipGetLastError();
}

// template classes of the fused kernel: mu-tiles of U and O-GEMM K steps of V
static const int kMtClass[] = {1, 2, 3, 4, 5, 6, 7, 8};
static const int kJsClass[] = {2, 4, 7, 10, 13, 16};

int fused_mt_class(int naux) {
  const int mt = (naux + 15) / 16;
  for (int c : kMtClass)
    if (mt <= c) return c;
  return -1;
}
int fused_js_class(int nao) {
  const int js = (2 * nao + 3) / 4;
  for (int c : kJsClass)
    if (js <= c) return c;
  return -1;
}

template <typename T, int MT, int JS>
static void launch_one(int hc, const Chi0Tables &tb, const PairItems &items, const T *Gp, const T *Cp,
                       const T *Nbuf, double negs, const int *gexp, const Screen &sc, double *chi, hipStream_t s) {
  if (hc == 1)
    hipLaunchKernelGGL((fused_kernel<T, sizeof(T) == 4, MT, JS, 1>), dim3(items.count), dim3(FU_THREADS), 0, s, tb,
                       items, Gp, Cp, Nbuf, negs, gexp, sc, chi);
  else
    hipLaunchKernelGGL((fused_kernel<T, sizeof(T) == 4, MT, JS, 2>), dim3(items.count), dim3(FU_THREADS), 0, s, tb,
                       items, Gp, Cp, Nbuf, negs, gexp, sc, chi);
}

template <typename T, int MT>
static hipError_t launch_js(int js, int hc, const Chi0Tables &tb, const PairItems &items, const T *Gp, const T *Cp,
                            const T *Nbuf, double negs, const int *gexp, const Screen &sc, double *chi,
                            hipStream_t s) {
  switch (js) {
    case 2: launch_one<T, MT, 2>(hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s); break;
    case 4: launch_one<T, MT, 4>(hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s); break;
    case 7: launch_one<T, MT, 7>(hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s); break;
    case 10: launch_one<T, MT, 10>(hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s); break;
    case 13: launch_one<T, MT, 13>(hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s); break;
    case 16: launch_one<T, MT, 16>(hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fused(const Chi0Tables &tb, const PairItems &items, int mt, int js, int hc, const T *Gp,
                        const T *Cp, const T *Nbuf, double negs, const int *gexp, const Screen &sc, double *chi,
                        hipStream_t s) {
  if (items.count == 0) return hipSuccess;
  switch (mt) {
    case 1: return launch_js<T, 1>(js, hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s);
    case 2: return launch_js<T, 2>(js, hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s);
    case 3: return launch_js<T, 3>(js, hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s);
    case 4: return launch_js<T, 4>(js, hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s);
    case 5: return launch_js<T, 5>(js, hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s);
    case 6: return launch_js<T, 6>(js, hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s);
    case 7: return launch_js<T, 7>(js, hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s);
    case 8: return launch_js<T, 8>(js, hc, tb, items, Gp, Cp, Nbuf, negs, gexp, sc, chi, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_pack_c<double>(const PackTables &, const double *, double *, long long, hipStream_t);
template hipError_t launch_pack_c<float>(const PackTables &, const double *, float *, long long, hipStream_t);
template hipError_t launch_pad_g<double>(const double *, const double *, int, int, int, const int *, double *,
                                         hipStream_t);
template hipError_t launch_pad_g<float>(const double *, const double *, int, int, int, const int *, float *,
                                        hipStream_t);
template hipError_t launch_nstage<double>(const Chi0Tables &, const NTiles &, const double *, const double *,
                                          double *, size_t, int, hipStream_t);
template hipError_t launch_nstage<float>(const Chi0Tables &, const NTiles &, const float *, const float *, float *,
                                         size_t, int, hipStream_t);
template hipError_t launch_fused<double>(const Chi0Tables &, const PairItems &, int, int, int, const double *,
                                         const double *, const double *, double, const int *, const Screen &,
                                         double *, hipStream_t);
template hipError_t launch_fused<float>(const Chi0Tables &, const PairItems &, int, int, int, const float *,
                                        const float *, const float *, double, const int *, const Screen &, double *,
                                        hipStream_t);
