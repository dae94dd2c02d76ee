// Split-BF16 (3-term) variant of the fused chi kernel for gfx950.
//
// Same restructured Algorithm 1 as the FP32 fused kernel (one workgroup per (U <= V, R); Z terms
// from two N blocks; K(R1) loop of O = [G^un | G^occ](R) [N^occ ; N^un] feeding chi += C O), with
// both contractions of the loop on the bf16 MFMAs: every operand x is carried as hi + lo,
// hi = bf16(x), lo = bf16(x - hi), and a product a b as a_hi b_hi + a_hi b_lo + a_lo b_hi
// (the dropped a_lo b_lo is below 2^-16 relative), accumulated in FP32 and folded into FP64
// after every neighbour block.  G is rescaled per tau by a power of two (pad_g), so the
// split never meets the FP32 subnormal range; the epilogue removes the scale in FP64.
// The N intermediate stays FP32 and is split in registers.  It comes from the split-BF16 N stage
// at the end of this file, or from the FP32 N stage when its operands do not fit 32-bit views.
#include "chi0_kernels.h"
#include "item_table.h"

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

// bf16 MFMAs with KW contraction values per lane: KW = 8 -> 16x16x32, KW = 4 -> 16x16x16.
// Operand layout (measured on gfx950 with exact small integers): A lane l holds
// A[l % 16][KW (l / 16) + e], B lane l holds B[KW (l / 16) + e][l % 16]; the FP32 result is
// laid out as for the f32 16x16x4 MFMA (row 4 (l / 16) + r, column l % 16).
template <int KW> struct BfMfma;
template <> struct BfMfma<8> {
  typedef bf8 vec;
  static __device__ __forceinline__ f4 fma(vec a, vec b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct BfMfma<4> {
  typedef bf4 vec;
  static __device__ __forceinline__ f4 fma(vec a, vec b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a), __builtin_bit_cast(s4, b), c, 0, 0,
                                                      0);
  }
};

static __device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)x;                       // round to nearest even
  lo = (__bf16)(x - (float)hi);         // x - hi is exact in FP32
}

// The same split for two values at once, as packed pairs (element 0 in the low half): one
// packed conversion per part, the hi values widened back by shift and mask.
static __device__ __forceinline__ void split_bf16x2(float x0, float x1, unsigned &hi, unsigned &lo) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector((f2){x0, x1}, b2));
  const float h0 = __builtin_bit_cast(float, hi << 16), h1 = __builtin_bit_cast(float, hi & 0xffff0000u);
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector((f2){x0 - h0, x1 - h1}, b2));
}

// Contraction slot of NAO index i of U in the chi GEMM.  With HC i-tiles of 16, lane group g
// holds as its KW = 4 HC values the O accumulator registers r of tiles h, i = 16 h + 4 g + r,
// in the order 4 h + r, so O feeds the next MFMA without moving between lanes.
static __device__ __forceinline__ int nao_of_slot(int slot, int hc) {
  if (hc == 1) return slot;
  const int g = slot / 8, h = (slot % 8) / 4, r = slot % 4;
  return 16 * h + 4 * g + r;
}

// LRI blocks [mu][i][k] (FP64) -> per k, rows mu of 16 hc hi values then 16 hc lo values in
// slot order (zero for slots past n_I), hc = 1 for n_I <= 16 else 2.  A workgroup takes
// kPackMu rows mu of one block: each row C[mu][.][.] (n_I n_K <= 1024 values, contiguous) is
// read once, coalesced, into LDS, and the k-major output rows are written from there.
constexpr int kPackMu = 8;
__global__ __launch_bounds__(256) void pack_cb_kernel(PackTables pt, const double *__restrict__ C,
                                                      __bf16 *__restrict__ Cb) {
  __shared__ float row[kMaxNao * kMaxNao];
  const int b = blockIdx.x;
  const int a = pt.a[b], ni = pt.ni[b], nk = pt.nk[b];
  const int mu0 = blockIdx.y * kPackMu;
  if (mu0 >= a) return;                          // workgroup-uniform
  const int hc = ni > 16 ? 2 : 1, S = 16 * hc;
  const double *src = C + pt.in_off[b];
  __bf16 *dst = Cb + pt.cb_off[b];
  const int mu1 = min(a, mu0 + kPackMu);
  for (int mu = mu0; mu < mu1; ++mu) {
    const double *r = src + (long long)mu * ni * nk;
    for (int e = threadIdx.x; e < ni * nk; e += blockDim.x) row[e] = (float)r[e];
    __syncthreads();
    for (int e = threadIdx.x; e < nk * S; e += blockDim.x) {
      const int k = e / S, slot = e - k * S;
      const int i = nao_of_slot(slot, hc);
      const float x = i < ni ? row[i * nk + k] : 0.f;
      __bf16 hi, lo;
      split_bf16(x, hi, lo);
      const long long o = ((long long)k * a + mu) * 2 * S;
      dst[o + slot] = hi;
      dst[o + S + slot] = lo;
    }
    __syncthreads();
  }
}

constexpr int FB_THREADS = 512;

// LDS row stride (dwords) of the staged C slices: hi, lo slots and 4 dwords of padding
template <int HC> constexpr int fb_row_stride() { return 16 * HC + 4; }

// LDS of one workgroup of the fused kernel, carved by the kernel that runs the body: two C slice
// buffers of kMaxNaux rows (Cs), the item's neighbour table and its scratch.
struct FusedLds {
  unsigned *Cs;
  long long *nbr_c, *nbr_n;
  int *nbr_k, *nbr_g, *pos, *meta;
};

// One item (U <= V, R) of one tau: MT mu-tiles of U, KS O-GEMM steps of 32 over j' < 2 n_V, HC
// i-tiles of U (n_U <= 16 HC), NW waves of 64 lanes, NU column tiles of 16 per wave.  Wave w owns
// the ABF columns nu of V in the tiles NU (half NW + w) + t, t < NU: a workgroup of 8 waves with
// one tile each, or of 4 waves with two, covers up to 128 columns; one of 4 waves with one tile
// each covers the half `half` of them (two workgroups per item when a_V > 64).  With two tiles
// per wave each C fragment read from LDS feeds both tiles' MFMAs.  Every thread of the workgroup
// runs it; it leaves no barrier pending, and the caller must synchronise before the LDS is used
// again.  stat: index of the item's statistics record (Screen::stats).
template <int MT, int KS, int HC, int NW, int NU = 1>
__device__ __forceinline__ void fused_bf16_body(const Chi0Tables &tb, int U, int V, int R, int half,
                                                const float *__restrict__ Gp, const __bf16 *__restrict__ Cb,
                                                const float *__restrict__ Nbuf, const __bf16 *__restrict__ Ns,
                                                double negs,
                                                const int *__restrict__ gexp, const Screen &sc, int stat,
                                                double *__restrict__ chi, const FusedLds &lds) {
  constexpr int NT = 64 * NW;            // threads of the workgroup
  constexpr int KW = 4 * HC;             // contraction values per lane in the chi GEMM
  constexpr int S = 16 * HC;             // slots per C row and part (hi, lo)
  constexpr int RS = fb_row_stride<HC>();
  constexpr int CH = 4 * HC;             // 16-byte chunks per C row
  constexpr int CG = 4;                  // mu-tiles whose C fragments are all read before the O GEMM
  typedef typename BfMfma<KW>::vec CVec;
  typedef typename BfMfma<8>::vec NVec;
  unsigned *const Cs0 = lds.Cs, *const Cs1 = lds.Cs + kMaxNaux * RS;
  long long *const nbr_c = lds.nbr_c, *const nbr_n = lds.nbr_n;
  int *const nbr_k = lds.nbr_k, *const nbr_g = lds.nbr_g;

  const int nU = tb.nao[U], aU = tb.naux[U], nV = tb.nao[V], aV = tb.naux[V];
  const int natoms = tb.natoms, nR = tb.nR, nbp = tb.nbp;
  const size_t plane = (size_t)nbp * nbp;
  const int tid = threadIdx.x, lane = tid & 63, w = uniform(half * NW + (tid >> 6));
  const int col = lane & 15, grp = lane >> 4;
  int nu[NU];
  bool nu_ok[NU], tile_on[NU];
#pragma unroll
  for (int t = 0; t < NU; ++t) {
    nu[t] = (NU * w + t) * 16 + col;
    tile_on[t] = (NU * w + t) * 16 < aV;
    nu_ok[t] = nu[t] < aV;
  }
  const bool wave_active = tile_on[0];
  // neighbour table (the entries whose M terms the screening keeps; all without screening)
  const int3 kept =
      item_table<NT>(tb, sc, tb.nbr_cb, tb.noffs, U, V, R, nbr_c, nbr_n, nbr_k, nbr_g, lds.pos, lds.meta);
  const int ne = kept.x;
  item_stats(sc, stat, kept);

  // A operand of the O GEMM, split: A[i][j'] = G^un_ij(R) for j' = j < n_V, G^occ_ij(R) for
  // j' = n_V + j; lane (col, grp) holds i = 16 h + col, j' = 32 ks + 8 grp + e
  NVec ah[HC][KS], al[HC][KS];
#pragma unroll
  for (int h = 0; h < HC; ++h)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int i = 16 * h + col, jp = 32 * ks + 8 * grp + e;
        float v = 0.f;
        if (i < nU && jp < 2 * nV) {
          const int s = jp >= nV;
          const int j = jp - s * nV;
          v = Gp[(size_t)(1 - s) * nR * plane + (size_t)R * plane + (size_t)(tb.ao_off[U] + i) * nbp + tb.ao_off[V] + j];
        }
        __bf16 hi, lo;
        split_bf16(v, hi, lo);
        ah[h][ks][e] = hi;
        al[h][ks][e] = lo;
      }

  f4 acc[NU][MT];
  double acc64[NU][MT][4];
#pragma unroll
  for (int t = 0; t < NU; ++t)
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      acc[t][m] = Mfma<float>::zero();
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[t][m][r] = 0.0;
    }
  auto flush = [&]() {
#pragma unroll
    for (int t = 0; t < NU; ++t)
#pragma unroll
      for (int m = 0; m < MT; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[t][m][r] += (double)acc[t][m][r];
        acc[t][m] = Mfma<float>::zero();
      }
  };

  // ---- Z terms (FP32 MFMA on the FP32 N blocks), as in the FP32 kernel
  const int negR = tb.bvk.neg(R);
  {
    const float *NA = Nbuf + uniform(tb.noff[((size_t)U * natoms + V) * nR + R]);
    const float *NB = Nbuf + uniform(tb.noff[((size_t)V * natoms + U) * nR + negR]);
    if (wave_active && kept.z) {
      const int F = 2 * nU * nV;
      // views of the two N blocks (elements outside them read zero): the loads of ZB iterations
      // are issued together and waited for once; each accumulator sees the same MFMA sequence
      const unsigned endA = (unsigned)((size_t)nV * 2 * nU * aU * sizeof(float));
      const unsigned endB = (unsigned)((size_t)nU * 2 * nV * aV * sizeof(float));
      const __amdgpu_buffer_rsrc_t vA = buffer_view(NA, endA), vB = buffer_view(NB, endB);
      constexpr int ZB = 4;
      for (int f0 = 0; f0 < F; f0 += 4 * ZB) {
        float bz[ZB][NU], az[ZB][MT];
#pragma unroll
        for (int u = 0; u < ZB; ++u) {
          const int f = f0 + 4 * u + grp;
          const bool fv = f < F;
          const int fc = fv ? f : 0;
          const int s = fc / (nU * nV);
          const int rem = fc - s * nU * nV;
          const int i = rem / nV, j = rem - i * nV;
#pragma unroll
          for (int t = 0; t < NU; ++t) {
            const unsigned ob = (fv && nu_ok[t])
                                    ? (unsigned)((((i * 2 + 1 - s) * nV + j) * aV + nu[t]) * sizeof(float))
                                    : endB;
            bz[u][t] = buffer_load<float>(vB, ob);
          }
#pragma unroll
          for (int m = 0; m < MT; ++m) {
            const int mu = 16 * m + col;
            const unsigned oa =
                (fv && mu < aU) ? (unsigned)((((j * 2 + s) * nU + i) * aU + mu) * sizeof(float)) : endA;
            az[u][m] = buffer_load<float>(vA, oa);
          }
        }
#pragma unroll
        for (int u = 0; u < ZB; ++u)
#pragma unroll
          for (int t = 0; t < NU; ++t)
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[t][m] = Mfma<float>::fma(az[u][m], bz[u][t], acc[t][m]);
      }
    }
    flush();
  }
  __syncthreads();   // neighbour table visible

  // C slices: aU rows of CH 16-byte chunks, copied chunk for chunk into LDS rows of RS dwords.
  // NLD loads of NT threads cover the CH kMaxNaux chunks of all rows; rows past aU read zero.
  constexpr int NLD = CH * kMaxNaux / NT;
  const unsigned sliceBytes = (unsigned)(aU * CH * 16);
  const size_t sliceElems = (size_t)aU * 2 * S;
  auto load_slice = [&](const __bf16 *src, u4 *rc) {
    const __amdgpu_buffer_rsrc_t r = buffer_view(src, sliceBytes);
#pragma unroll
    for (int q = 0; q < NLD; ++q)
      rc[q] = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(r, (unsigned)((tid + q * NT) * 16), 0, 0));
  };
  auto store_slice = [&](int buf, const u4 *rc) {
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int c = tid + q * NT;
      *reinterpret_cast<u4 *>(&(buf ? Cs1 : Cs0)[(c / CH) * RS + 4 * (c % CH)]) = rc[q];
    }
  };
  // N rows, split BF16 (noffs layout [k][part][nu][JP]): lane (nu, grp) holds j' = 32 ks + 8 grp + e
  // of each part, one 16-byte load per part and ks.  Past 2 n_V the rows read the zero padding,
  // then the next rows (finite values that meet the zero A columns j' >= 2 n_V); past the slice
  // the view reads zero.
  const int JP = (2 * nV + 7) / 8 * 8;
  const size_t nslice = (size_t)2 * aV * JP;
  const unsigned nview = wave_active ? (unsigned)(nslice * sizeof(__bf16)) : 0u;
  struct NRows {
    NVec h[NU][KS], l[NU][KS];
  };
  NRows nb0, nb1, nb2;
  auto load_n = [&](const __bf16 *nrow, NRows &dst) {
    const __amdgpu_buffer_rsrc_t r = buffer_view(nrow, nview);
#pragma unroll
    for (int t = 0; t < NU; ++t)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const unsigned o = (unsigned)(((size_t)nu[t] * JP + 32 * ks + 8 * grp) * sizeof(__bf16));
        dst.h[t][ks] = __builtin_bit_cast(NVec, __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0));
        dst.l[t][ks] =
            __builtin_bit_cast(NVec, __builtin_amdgcn_raw_buffer_load_b128(r, o + (unsigned)(aV * JP * 2), 0, 0));
      }
  };
  // Slice order: the entries e of U's neighbourhood come in runs [g0, g1) of one atom K (its
  // periodic images R1); a run is walked NAO k outer, image inner, so that the workgroups of
  // one atom pair at different R read the N rows N(V, K, .)[k] of a few hundred KB at about the
  // same time and share them in L2.  FP32 partial sums are folded into FP64 at the end of a pass
  // over the images once kFoldSlices slices have been added since the last fold, and at the end
  // of each run.  The cursor (e, k) runs two slices ahead of the slice being computed.
  // The run's NAO count and the table entry of the cursor stay in scalar registers: the LDS
  // table is read when a run starts and when the cursor moves to another entry, so a run of one
  // image (every run at the Gamma point) reads it once for all its slices.
  int e = 0, k = 0, g0 = 0, g1 = 0, run = 0, nk_run = 0;
  auto advance = [&]() -> bool {   // next slice; true if the slice left is followed by a fold
    int e2 = e + 1, k2 = k;
    bool fold = false;
    ++run;
    if (e2 == g1) {
      e2 = g0;
      k2 = k + 1;
      bool run_end = false;
      if (k2 == nk_run) {
        k2 = 0;
        e2 = g1;
        g0 = g1;
        g1 = e2 < ne ? uniform(nbr_g[e2]) : g1;
        nk_run = e2 < ne ? uniform(nbr_k[e2]) : 0;
        run_end = true;
      }
      fold = run_end || run >= kFoldSlices;
      if (fold) run = 0;
    }
    e = e2;
    k = k2;
    return fold;
  };
  // N rows at the cursor into nb, and the cursor's C slice address into cnext (slice 0 again
  // once the cursor is past the end: in bounds, never used).
  const __bf16 *cnext = Cb;
  int e_at = -1;
  long long c_at = 0, n_at = 0;
  auto load_at = [&](NRows &nb) {
    const bool more = e < ne;
    const int ea = more ? e : 0, ka = more ? k : 0;
    if (ea != e_at) {
      c_at = uniform(nbr_c[ea]);
      n_at = uniform(nbr_n[ea]);
      e_at = ea;
    }
    cnext = Cb + c_at + (size_t)ka * sliceElems;
    load_n(Ns + n_at + (size_t)ka * nslice, nb);
  };
  bool fcur = false;   // fold after the slice being computed
  u4 rc[NLD];
  // O of a slice, A [G^un | G^occ](R) times the slice's split N rows (3 products)
  auto ogemm = [&](const NRows &nb, f4 (*o)[HC]) __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < NU; ++t)
#pragma unroll
      for (int h = 0; h < HC; ++h) o[t][h] = Mfma<float>::zero();
#pragma unroll
    for (int t = 0; t < NU; ++t)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int h = 0; h < HC; ++h) {
          o[t][h] = BfMfma<8>::fma(ah[h][ks], nb.h[t][ks], o[t][h]);
          o[t][h] = BfMfma<8>::fma(ah[h][ks], nb.l[t][ks], o[t][h]);
          o[t][h] = BfMfma<8>::fma(al[h][ks], nb.h[t][ks], o[t][h]);
        }
  };
  // The O GEMM runs one slice ahead of chi += C O: slice t takes O(t) from the slice before and
  // issues O(t + 1) on the MFMAs while O(t) is split into its bf16 parts, so the split does not
  // wait for its own GEMM.
  f4 onext[NU][HC];
  // slice t: loads of slice t + 1's C (into rc) and of slice t + 2's N rows (into nbld), O GEMM of
  // t + 1 (N rows nbnext), chi += C O(t) with the C slice of t in LDS buffer cur, then rc to LDS.
  // live: t is a slice; live1: t + 1 is a slice.  Past the last slice the cursor reads slice 0
  // again, so every O GEMM sees finite rows.
  auto slice = [&](const NRows &nbnext, NRows &nbld, int cur, bool live, bool live1) __attribute__((always_inline)) {
    load_slice(cnext, rc);
    const bool f1 = live1 ? advance() : false;
    load_at(nbld);
    __builtin_amdgcn_sched_barrier(0);
    if (live && wave_active) {
      // C fragments of the first M0 mu-tiles (all of them up to CG) first: their LDS reads
      // complete under the O GEMM; the others are read before the chi MFMAs
      const unsigned *cs = &(cur ? Cs1 : Cs0)[col * RS + grp * (KW / 2)];
      constexpr int M0 = MT <= CG ? MT : CG - 1, M1 = MT - M0 > 0 ? MT - M0 : 1;
      CVec ch0[M0], cl0[M0];
#pragma unroll
      for (int m = 0; m < M0; ++m) {
        ch0[m] = *reinterpret_cast<const CVec *>(cs + 16 * m * RS);
        cl0[m] = *reinterpret_cast<const CVec *>(cs + 16 * m * RS + 8 * HC);
      }
      __builtin_amdgcn_sched_barrier(0);
      f4 o[NU][HC];
#pragma unroll
      for (int t = 0; t < NU; ++t)
#pragma unroll
        for (int h = 0; h < HC; ++h) o[t][h] = onext[t][h];
      ogemm(nbnext, onext);
      typedef unsigned UPairs __attribute__((ext_vector_type(KW / 2)));
      CVec bh[NU], bl[NU];
#pragma unroll
      for (int t = 0; t < NU; ++t) {
        UPairs ph, pl;
#pragma unroll
        for (int h = 0; h < HC; ++h)
#pragma unroll
          for (int r = 0; r < 4; r += 2) {
            unsigned hi, lo;
            split_bf16x2(o[t][h][r], o[t][h][r + 1], hi, lo);
            ph[2 * h + r / 2] = hi;
            pl[2 * h + r / 2] = lo;
          }
        bh[t] = __builtin_bit_cast(CVec, ph);
        bl[t] = __builtin_bit_cast(CVec, pl);
      }
      CVec ch1[M1], cl1[M1];
#pragma unroll
      for (int m = M0; m < MT; ++m) {
        ch1[m - M0] = *reinterpret_cast<const CVec *>(cs + 16 * m * RS);
        cl1[m - M0] = *reinterpret_cast<const CVec *>(cs + 16 * m * RS + 8 * HC);
      }
#pragma unroll
      for (int t = 0; t < NU; ++t) {
#pragma unroll
        for (int m = 0; m < M0; ++m) acc[t][m] = BfMfma<KW>::fma(ch0[m], bh[t], acc[t][m]);
#pragma unroll
        for (int m = 0; m < M0; ++m) acc[t][m] = BfMfma<KW>::fma(ch0[m], bl[t], acc[t][m]);
#pragma unroll
        for (int m = 0; m < M0; ++m) acc[t][m] = BfMfma<KW>::fma(cl0[m], bh[t], acc[t][m]);
      }
#pragma unroll
      for (int t = 0; t < NU; ++t) {
#pragma unroll
        for (int m = M0; m < MT; ++m) acc[t][m] = BfMfma<KW>::fma(ch1[m - M0], bh[t], acc[t][m]);
#pragma unroll
        for (int m = M0; m < MT; ++m) acc[t][m] = BfMfma<KW>::fma(ch1[m - M0], bl[t], acc[t][m]);
#pragma unroll
        for (int m = M0; m < MT; ++m) acc[t][m] = BfMfma<KW>::fma(cl1[m - M0], bh[t], acc[t][m]);
      }
    }
    if (fcur) flush();
    fcur = f1;
    store_slice(cur ^ 1, rc);
    __syncthreads();
  };

  const int nsl = kept.y;
  if (ne > 0) {
    g1 = uniform(nbr_g[0]);
    nk_run = uniform(nbr_k[0]);
    load_at(nb0);
    load_slice(cnext, rc);
    store_slice(0, rc);
    fcur = advance();
    load_at(nb1);
    __syncthreads();
    ogemm(nb0, onext);
    for (int t = 0; t < nsl; t += 6) {
      slice(nb1, nb2, 0, true, t + 1 < nsl);
      slice(nb2, nb0, 1, t + 1 < nsl, t + 2 < nsl);
      slice(nb0, nb1, 0, t + 2 < nsl, t + 3 < nsl);
      slice(nb1, nb2, 1, t + 3 < nsl, t + 4 < nsl);
      slice(nb2, nb0, 0, t + 4 < nsl, t + 5 < nsl);
      slice(nb0, nb1, 1, t + 5 < nsl, t + 6 < nsl);
    }
  }

  // ---- epilogue: chi_UV(R) and chi_VU(-R) = chi_UV(R)^T, G scale removed
  const double scale = ldexp(negs, -(gexp[0] + gexp[1]));
  const size_t N = tb.nauxtot;
  const int au0 = tb.aux_off[U], av0 = tb.aux_off[V];
#pragma unroll
  for (int t = 0; t < NU; ++t) {
    if (!tile_on[t] || !nu_ok[t]) continue;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mu = 16 * m + Mfma<float>::row(grp, r);
        if (mu < aU) {
          const double v = scale * acc64[t][m][r];
          chi[((size_t)R * N + au0 + mu) * N + av0 + nu[t]] = v;
          if (U != V) chi[((size_t)negR * N + av0 + nu[t]) * N + au0 + mu] = v;
        }
      }
    }
  }
}

// Per-class launch: workgroup b runs item b of the list.
template <int MT, int KS, int HC>
__global__ __launch_bounds__(FB_THREADS) void fused_bf16_kernel(Chi0Tables tb, PairItems items,
                                                                const float *__restrict__ Gp,
                                                                const __bf16 *__restrict__ Cb,
                                                                const float *__restrict__ Nbuf,
                                                                const __bf16 *__restrict__ Ns, double negs,
                                                                const int *__restrict__ gexp, Screen sc,
                                                                double *__restrict__ chi) {
  __shared__ __align__(16) unsigned Cs[2 * kMaxNaux * fb_row_stride<HC>()];
  __shared__ long long nbr_c[kMaxNbr], nbr_n[kMaxNbr];
  __shared__ int nbr_k[kMaxNbr], nbr_g[kMaxNbr], nbr_pos[kMaxNbr + 1], nbr_meta[3];
  const FusedLds lds{Cs, nbr_c, nbr_n, nbr_k, nbr_g, nbr_pos, nbr_meta};
  const int item = blockIdx.x;
  fused_bf16_body<MT, KS, HC, 8>(tb, items.U[item], items.V[item], items.R[item], 0, Gp, Cb, Nbuf, Ns, negs, gexp,
                                 sc, item, chi, lds);
}

// One launch over the work of several tau points and every template class.  Work unit u of slot
// w / nunits is a.order[w % nunits]: with 8-wave workgroups an item, with 4-wave workgroups an
// item and the half of its ABF columns of V (code 2 item + half; only halves with columns).  The
// units of a slot come in order of decreasing work, and the hardware hands the workgroups to the
// compute units in index order as they free up, so the launch ends on the smallest units.  The
// item's class code (mt - 1) 4 + (ks - 1) 2 + (hc - 1) picks the instantiation of the body.
template <int MT, int KS, int HC, int NW, int NU>
__device__ __forceinline__ void single_item(const Chi0Tables &tb, const SingleLaunch &a, int item, int half, int slot,
                                            const FusedLds &lds) {
  Screen sc{nullptr, nullptr, nullptr, nullptr};
  if (a.gb) {
    const size_t nb3 = (size_t)tb.natoms * tb.natoms * tb.nR;
    sc = Screen{a.gb + slot * nb3, a.gn + slot * nb3, a.gc + 2 * slot,
                a.stats ? a.stats + (size_t)slot * a.stats_stride : nullptr};
  }
  fused_bf16_body<MT, KS, HC, NW, NU>(tb, a.U[item], a.V[item], a.R[item], half, a.Gp + slot * a.gp_stride,
                                  reinterpret_cast<const __bf16 *>(a.Cb), a.Nbuf + slot * a.n_stride,
                                  reinterpret_cast<const __bf16 *>(a.Ns) + slot * a.ns_stride, a.negs,
                                  a.gexp + 2 * slot, sc, item, a.chi + slot * a.chi_stride, lds);
}

// NW = 8, NU = 1: a workgroup per item, one column tile per wave; NW = 4, NU = 1: a workgroup per
// half item; NW = 4, NU = 2: a workgroup per item, two column tiles per wave (one wave per SIMD,
// with the register file of a whole SIMD).
template <int NW, int NU>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3 - NU, 3 - NU))) void fused_bf16_single(
    Chi0Tables tb, SingleLaunch a) {
  __shared__ __align__(16) unsigned Cs[2 * kMaxNaux * fb_row_stride<2>()];
  __shared__ long long nbr_c[kMaxNbr], nbr_n[kMaxNbr];
  __shared__ int nbr_k[kMaxNbr], nbr_g[kMaxNbr], nbr_pos[kMaxNbr + 1], nbr_meta[3];
  const FusedLds lds{Cs, nbr_c, nbr_n, nbr_k, nbr_g, nbr_pos, nbr_meta};
  const int w = blockIdx.x;
  const int slot = w / a.nitems;
  const int code = a.order[w - slot * a.nitems];
  const bool halves = NW == 4 && NU == 1;
  const int item = halves ? code >> 1 : code, half = halves ? code & 1 : 0;
  switch (a.cls[item]) {
#define RPA_CLS(mt, ks, hc) \
  case (mt - 1) * 4 + (ks - 1) * 2 + (hc - 1): single_item<mt, ks, hc, NW, NU>(tb, a, item, half, slot, lds); break;
#define RPA_CLS_MT(mt) RPA_CLS(mt, 1, 1) RPA_CLS(mt, 1, 2) RPA_CLS(mt, 2, 1) RPA_CLS(mt, 2, 2)
    RPA_CLS_MT(1) RPA_CLS_MT(2) RPA_CLS_MT(3) RPA_CLS_MT(4) RPA_CLS_MT(5) RPA_CLS_MT(6) RPA_CLS_MT(7) RPA_CLS_MT(8)
#undef RPA_CLS_MT
#undef RPA_CLS
    default: break;
  }
}

template <int MT, int KS, int HC>
void launch_one_bf16(const Chi0Tables &tb, const PairItems &items, const float *Gp, const __bf16 *Cb,
                     const float *Nbuf, const __bf16 *Ns, double negs, const int *gexp, const Screen &sc, double *chi,
                     hipStream_t s) {
  hipLaunchKernelGGL((fused_bf16_kernel<MT, KS, HC>), dim3(items.count), dim3(FB_THREADS), 0, s, tb, items, Gp, Cb,
                     Nbuf, Ns, negs, gexp, sc, chi);
}

template <int MT>
hipError_t launch_ks_hc(int ks, int hc, const Chi0Tables &tb, const PairItems &items, const float *Gp,
                        const __bf16 *Cb, const float *Nbuf, const __bf16 *Ns, double negs, const int *gexp,
                        const Screen &sc, double *chi, hipStream_t s) {
  if (ks == 1 && hc == 1) launch_one_bf16<MT, 1, 1>(tb, items, Gp, Cb, Nbuf, Ns, negs, gexp, sc, chi, s);
  else if (ks == 1 && hc == 2) launch_one_bf16<MT, 1, 2>(tb, items, Gp, Cb, Nbuf, Ns, negs, gexp, sc, chi, s);
  else if (ks == 2 && hc == 1) launch_one_bf16<MT, 2, 1>(tb, items, Gp, Cb, Nbuf, Ns, negs, gexp, sc, chi, s);
  else if (ks == 2 && hc == 2) launch_one_bf16<MT, 2, 2>(tb, items, Gp, Cb, Nbuf, Ns, negs, gexp, sc, chi, s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

int fused_bf16_ks_class(int js_class) { return 4 * js_class <= 32 ? 1 : 2; }

hipError_t launch_pack_cb(const PackTables &pt, const double *C, uint16_t *Cb, long long maxblk, hipStream_t s) {
  (void)maxblk;
  if (pt.nblk == 0) return hipSuccess;
  dim3 grid(pt.nblk, (kMaxNaux + kPackMu - 1) / kPackMu);
  hipLaunchKernelGGL(pack_cb_kernel, grid, dim3(256), 0, s, pt, C, reinterpret_cast<__bf16 *>(Cb));
  return hipGetLastError();
}

hipError_t launch_fused_bf16(const Chi0Tables &tb, const PairItems &items, int mt, int ks, int hc, const float *Gp,
                             const uint16_t *Cb, const float *Nbuf, const uint16_t *Nsplit, double negs,
                             const int *gexp, const Screen &sc, double *chi, hipStream_t s) {
  if (items.count == 0) return hipSuccess;
  const __bf16 *cb = reinterpret_cast<const __bf16 *>(Cb);
  const __bf16 *Ns = reinterpret_cast<const __bf16 *>(Nsplit);
  switch (mt) {
    case 1: return launch_ks_hc<1>(ks, hc, tb, items, Gp, cb, Nbuf, Ns, negs, gexp, sc, chi, s);
    case 2: return launch_ks_hc<2>(ks, hc, tb, items, Gp, cb, Nbuf, Ns, negs, gexp, sc, chi, s);
    case 3: return launch_ks_hc<3>(ks, hc, tb, items, Gp, cb, Nbuf, Ns, negs, gexp, sc, chi, s);
    case 4: return launch_ks_hc<4>(ks, hc, tb, items, Gp, cb, Nbuf, Ns, negs, gexp, sc, chi, s);
    case 5: return launch_ks_hc<5>(ks, hc, tb, items, Gp, cb, Nbuf, Ns, negs, gexp, sc, chi, s);
    case 6: return launch_ks_hc<6>(ks, hc, tb, items, Gp, cb, Nbuf, Ns, negs, gexp, sc, chi, s);
    case 7: return launch_ks_hc<7>(ks, hc, tb, items, Gp, cb, Nbuf, Ns, negs, gexp, sc, chi, s);
    case 8: return launch_ks_hc<8>(ks, hc, tb, items, Gp, cb, Nbuf, Ns, negs, gexp, sc, chi, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Split-BF16 N stage.  Same GEMM as the FP32 N stage,
//   N[(s, dR, k)][(j, nu)] = sum_r A[(s, dR, k)][r] B[r][(j, nu)],
//   A[(s,dR,k)][r] = G^s(dR - dL)_{g, k},  B[r][(j, nu)] = C^nu_{j l}(V, L, dL),
// over contraction rows r = (neighbour L(dL) of V, NAO l of L), with both operands stored so
// that 8 consecutive rows of one neighbour block are 16 contiguous bytes:
//   GT[s][Y][k][g'] = G^s(Y)_{g k}, the NAO columns g = (L, l) of each atom padded to a multiple
//     of 8 (g' = aopad_off[L] + l, zero padding), rows k padded to nbp;
//   CtN[block][j a_V + nu][l'] = C^nu_{j l'} (l' padded to a multiple of 8 with zeros);
// each split into a hi and a lo bf16 array.  GEMM rows run in the order (s, k, dR): the 128
// rows of a tile then take their A values from G of only two or three NAO rows k (all cells),
// about 0.1 MB of transposed G per tile, which stays in L2 while the tile gathers it.  A K step
// of 32 takes 4 groups of 8 rows; each lane of an MFMA reads its 8 contraction values with one
// 16-byte LDS load.  N is written in FP32.
// ---------------------------------------------------------------------------
namespace {

// CtN of every LRI block into the hi and lo arrays.
__global__ __launch_bounds__(256) void pack_ctn_kernel(PackTables pt, const double *__restrict__ C,
                                                       __bf16 *__restrict__ Cth, __bf16 *__restrict__ Ctl) {
  const int b = blockIdx.x;
  const int a = pt.a[b], ni = pt.ni[b], nk = pt.nk[b];
  const int st = (nk + 7) / 8 * 8;
  const long long total = (long long)ni * a * st;
  const double *src = C + pt.in_off[b];
  const long long o = pt.ctn_off[b];
  for (long long e = (long long)blockIdx.y * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.y * blockDim.x) {
    const int lp = (int)(e % st);
    const long long n = e / st;
    const int j = (int)(n / a), nu = (int)(n % a);
    const float x = lp < nk ? (float)src[((long long)nu * ni + j) * nk + lp] : 0.f;
    __bf16 hi, lo;
    split_bf16(x, hi, lo);
    Cth[o + e] = hi;
    Ctl[o + e] = lo;
  }
}

// GT of one tau from G^occ, G^un (FP64 [nR][nb][nb]) times 2^gexp[s]; gsrc[g'] = g or -1.
__global__ __launch_bounds__(256) void pad_gt_kernel(const double *__restrict__ Gocc, const double *__restrict__ Gun,
                                                     int nR, int nb, int nbp, int nbq, const int *__restrict__ gsrc,
                                                     const int *__restrict__ gexp, __bf16 *__restrict__ GTh,
                                                     __bf16 *__restrict__ GTl) {
  const double sc0 = ldexp(1.0, gexp[0]), sc1 = ldexp(1.0, gexp[1]);
  const size_t total = (size_t)2 * nR * nbp * nbq;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int gp = (int)(e % nbq);
    const size_t t = e / nbq;
    const int k = (int)(t % nbp);
    const size_t sY = t / nbp;
    const int Y = (int)(sY % nR), s = (int)(sY / nR);
    const int g = gsrc[gp];
    float x = 0.f;
    if (k < nb && g >= 0) x = (float)((s ? Gun : Gocc)[((size_t)Y * nb + g) * nb + k] * (s ? sc1 : sc0));
    __bf16 hi, lo;
    split_bf16(x, hi, lo);
    GTh[e] = hi;
    GTl[e] = lo;
  }
}

constexpr int NB_RS = 40;            // LDS row stride (bf16): 32 contraction values + 8 padding

// gt_bytes, ct_bytes: bytes of one part (hi or lo), at most 2^32 - 2^16 (a masked load sits at
// the view's end, so offset plus load size never wraps).  BM: tile rows, 128 (4 waves) or 256
// (8 waves, each B tile then serves twice the rows); 128 columns, waves of 64 x 64.
template <int BM>
__global__ __launch_bounds__(2 * BM) __attribute__((amdgpu_waves_per_eu(2))) void nstage_bf16_kernel(Chi0Tables tb, NTiles tiles,
                                                             const __bf16 *__restrict__ GTh,
                                                             const __bf16 *__restrict__ GTl, unsigned gt_bytes,
                                                             const __bf16 *__restrict__ Cth,
                                                             const __bf16 *__restrict__ Ctl, unsigned ct_bytes,
                                                             float *__restrict__ Nbuf, size_t gt_slot,
                                                             size_t n_slot) {
  // [buffer][part hi/lo][rows x NB_RS]
  __shared__ __align__(16) __bf16 As[2][2][BM * NB_RS];
  __shared__ __align__(16) __bf16 Bs[2][2][128 * NB_RS];
  // B loader: 128 rows x 4 groups of 8 over the 2 BM threads, BG groups per thread
  constexpr int BG = 512 / (2 * BM);

  const int t = blockIdx.x;
  // tau slot of the launch
  GTh += (size_t)blockIdx.y * gt_slot;
  GTl += (size_t)blockIdx.y * gt_slot;
  Nbuf += (size_t)blockIdx.y * n_slot;
  const int V = tiles.V[t], m0 = tiles.m0[t], n0 = tiles.n0[t];
  const int nV = tb.nao[V], aV = tb.naux[V];
  const int NV = nV * aV;
  const int nbp = tb.nbp, nR = tb.nR, nb = tb.nb, nbq = tb.nbq;
  const int M = 2 * nR * nbp;
  const int g0 = tb.ngrp_start[V], ng = tb.ngrp_start[V + 1] - g0;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int col = lane & 15, grp = lane >> 4;

  // loader: row / column tid >> 1 of the tile, groups 2 (tid & 1) and 2 (tid & 1) + 1 of a K step
  const int lr = tid >> 1, lh = tid & 1;
  const int m = m0 + lr;
  const bool mvalid = m < M;
  int ss = 0, d0 = 0, d1 = 0, d2 = 0, kk = 0;
  if (mvalid) {
    ss = m / (nR * nbp);
    const int rem = m - ss * nR * nbp;
    kk = rem / nR;
    const int dR = rem - kk * nR;
    tb.bvk.split(dR, d0, d1, d2);
  }
  const int br = BG == 2 ? lr : tid >> 2, bq0 = BG == 2 ? 2 * lh : tid & 3;   // B row, first group
  const int n = n0 + br;
  const bool nvalid = n < NV;
  const __amdgpu_buffer_rsrc_t gvh = buffer_view(GTh, gt_bytes), gvl = buffer_view(GTl, gt_bytes);
  const __amdgpu_buffer_rsrc_t cvh = buffer_view(Cth, ct_bytes), cvl = buffer_view(Ctl, ct_bytes);
  const int n0m = tb.bvk.n0, n1m = tb.bvk.n1, n2m = tb.bvk.n2;

  // two register sets of the staged operands, [group][part]: the loads of K step ks + 2 are
  // issued before the MFMAs of step ks and written to LDS after those of step ks + 1
  u4 ra0[2][2], rb0[BG][2], ra1[2][2], rb1[BG][2];
  auto load = [&](int ks, u4 (&ra)[2][2], u4 (&rb)[BG][2]) {
    // the 4 groups of the K step: wave-uniform table reads (scalar loads)
    int4 gq[4];
    long long oq[4];
    bool vq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gi = 4 * ks + q;
      vq[q] = gi < ng;
      gq[q] = make_int4(0, 0, 0, 0);
      oq[q] = 0;
      if (vq[q]) {
        gq[q] = tb.ngrp[g0 + gi];              // {A column g', dL packed, CtN row stride, 0}
        oq[q] = tb.ngrp_off[g0 + gi];
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int4 gr = lh ? gq[2 + q] : gq[q];
      const bool valid = lh ? vq[2 + q] : vq[q];
      unsigned oa = gt_bytes;                 // default: past the view, the load reads zero
      if (valid && mvalid) {
        int c0 = d0 - (gr.y & 1023), c1 = d1 - ((gr.y >> 10) & 1023), c2 = d2 - (gr.y >> 20);
        c0 += c0 < 0 ? n0m : 0;
        c1 += c1 < 0 ? n1m : 0;
        c2 += c2 < 0 ? n2m : 0;
        const int Y = (c0 * n1m + c1) * n2m + c2;
        oa = (unsigned)(((((size_t)ss * nR + Y) * nbp + kk) * nbq + gr.x) * sizeof(__bf16));
      }
      ra[q][0] = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(gvh, oa, 0, 0));
      ra[q][1] = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(gvl, oa, 0, 0));
    }
#pragma unroll
    for (int q = 0; q < BG; ++q) {
      // group bq0 + q of the K step, chosen by selects (a per-lane index into the group arrays
      // would put them in scratch memory)
      const int bq = bq0 + q;
      const bool vb = bq == 0 ? vq[0] : bq == 1 ? vq[1] : bq == 2 ? vq[2] : vq[3];
      const long long obq = bq == 0 ? oq[0] : bq == 1 ? oq[1] : bq == 2 ? oq[2] : oq[3];
      const int zb = bq == 0 ? gq[0].z : bq == 1 ? gq[1].z : bq == 2 ? gq[2].z : gq[3].z;
      unsigned ob = ct_bytes;
      if (vb && nvalid) ob = (unsigned)((obq + (size_t)n * zb) * sizeof(__bf16));
      rb[q][0] = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(cvh, ob, 0, 0));
      rb[q][1] = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(cvl, ob, 0, 0));
    }
  };
  auto store = [&](int buf, const u4 (&ra)[2][2], const u4 (&rb)[BG][2]) {
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int p = 0; p < 2; ++p)
        *reinterpret_cast<u4 *>(&As[buf][p][lr * NB_RS + 8 * (2 * lh + q)]) = ra[q][p];
#pragma unroll
    for (int q = 0; q < BG; ++q)
#pragma unroll
      for (int p = 0; p < 2; ++p)
        *reinterpret_cast<u4 *>(&Bs[buf][p][br * NB_RS + 8 * (bq0 + q)]) = rb[q][p];
  };

  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<float>::zero();

  const int nks = (ng + 3) / 4;
  // B fragments of the step first, then one row tile of A at a time (3 x 4 MFMAs per row tile,
  // four independent accumulators between two products into the same one)
  auto compute = [&](int cur) {
    bf8 bh[4], bl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ob_ = (wn * 64 + q * 16 + col) * NB_RS + 8 * grp;
      bh[q] = *reinterpret_cast<const bf8 *>(&Bs[cur][0][ob_]);
      bl[q] = *reinterpret_cast<const bf8 *>(&Bs[cur][1][ob_]);
    }
#pragma unroll
    for (int tm = 0; tm < 4; ++tm) {
      const int oa_ = (wm * 64 + tm * 16 + col) * NB_RS + 8 * grp;
      const bf8 ah = *reinterpret_cast<const bf8 *>(&As[cur][0][oa_]);
      const bf8 al = *reinterpret_cast<const bf8 *>(&As[cur][1][oa_]);
#pragma unroll
      for (int tn = 0; tn < 4; ++tn) acc[tm][tn] = BfMfma<8>::fma(ah, bh[tn], acc[tm][tn]);
#pragma unroll
      for (int tn = 0; tn < 4; ++tn) acc[tm][tn] = BfMfma<8>::fma(ah, bl[tn], acc[tm][tn]);
#pragma unroll
      for (int tn = 0; tn < 4; ++tn) acc[tm][tn] = BfMfma<8>::fma(al, bh[tn], acc[tm][tn]);
    }
  };
  // Loads are unconditional: a K step past the last group reads zeros (its table entries are
  // invalid, so every lane addresses the end of its view), which keeps the wait counts exact.
  load(0, ra0, rb0);
  load(1, ra1, rb1);
  store(0, ra0, rb0);
  __syncthreads();
  for (int ks = 0; ks < nks; ks += 2) {
    // step ks from LDS buffer 0; step ks + 1 is in ra1 / rb1
    load(ks + 2, ra0, rb0);
    compute(0);
    if (ks + 1 >= nks) break;
    store(1, ra1, rb1);
    __syncthreads();
    // step ks + 1 from LDS buffer 1; step ks + 2 is in ra0 / rb0
    load(ks + 3, ra1, rb1);
    compute(1);
    if (ks + 2 < nks) store(0, ra0, rb0);
    __syncthreads();
  }

  // epilogue: scatter rows (s, k, dR) into N blocks (V, K(k), dR), layout [k][s][j][nu]
#pragma unroll
  for (int tm = 0; tm < 4; ++tm) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mm = m0 + wm * 64 + tm * 16 + Mfma<float>::row(grp, r);
      if (mm >= M) continue;
      const int s2 = mm / (nR * nbp);
      const int rem = mm - s2 * nR * nbp;
      const int k2 = rem / nR;
      const int dR2 = rem - k2 * nR;
      if (k2 >= nb) continue;
      const int K = tb.atom_of_ao[k2];
      const int kl = k2 - tb.ao_off[K];
      float *dst = Nbuf + tb.noff[((size_t)V * tb.natoms + K) * nR + dR2] + (size_t)(kl * 2 + s2) * NV;
#pragma unroll
      for (int tn = 0; tn < 4; ++tn) {
        const int nn = n0 + wn * 64 + tn * 16 + col;
        if (nn < NV) dst[nn] = acc[tm][tn][r];
      }
    }
  }
}

}  // namespace

namespace {

// Split-BF16 copy of N for the fused kernel's O GEMM: workgroup (x, y) = (block (V, K, dR) of
// index x, slot y), over the block's n_K slices in turn.  Each K(R1) slice's FP32 rows
// N[k][s][j][nu] (2 n_V x a_V, contiguous) are read coalesced into LDS; each thread unit (part,
// nu, 8 rows j') then takes its 8 values from LDS (zero past 2 n_V) and writes them as one 16-byte
// store, consecutive units to consecutive addresses of [k][part][nu][j'].
constexpr int SPLIT_MAX_ROWS = 2 * kMaxNao;
__global__ __launch_bounds__(256) void split_n_kernel(Chi0Tables tb, const float *__restrict__ N,
                                                      __bf16 *__restrict__ Ns, size_t n_slot, size_t ns_slot) {
  __shared__ float sl[SPLIT_MAX_ROWS * kMaxNaux];
  const int blk = blockIdx.x;
  const int nR = tb.nR, na = tb.natoms;
  const int vk = blk / nR, V = vk / na, K = vk - V * na;
  const int nV = tb.nao[V], aV = tb.naux[V], nK = tb.nao[K];
  const int JP = (2 * nV + 7) / 8 * 8, NO = JP / 8;
  const int rows = 2 * nV;
  const int units = 2 * aV * NO;
  const float *src = N + (size_t)blockIdx.y * n_slot + tb.noff[blk];
  __bf16 *dst = Ns + (size_t)blockIdx.y * ns_slot + tb.noffs[blk];
  for (int k = 0; k < nK; ++k, src += (size_t)rows * aV, dst += (size_t)2 * aV * JP) {
    for (int e = threadIdx.x; e < rows * aV; e += blockDim.x) sl[e] = src[e];
    __syncthreads();
    for (int u = threadIdx.x; u < units; u += blockDim.x) {
      const int o = u % NO, pn = u / NO;
      const int nu = pn % aV, part = pn / aV;
      bf8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int jp = 8 * o + e;
        const float xv = jp < rows ? sl[jp * aV + nu] : 0.f;
        __bf16 h, l;
        split_bf16(xv, h, l);
        v[e] = part ? l : h;
      }
      *reinterpret_cast<bf8 *>(dst + (size_t)pn * JP + 8 * o) = v;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_split_n(const Chi0Tables &tb, const float *N, uint16_t *Ns, int nslots, size_t n_slot,
                          size_t ns_slot, hipStream_t s) {
  const long long nblk = (long long)tb.natoms * tb.natoms * tb.nR;
  if (nblk == 0 || nslots <= 0) return hipSuccess;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(split_n_kernel, dim3((unsigned)nblk, nslots), dim3(256), 0, s, tb, N,
                     reinterpret_cast<__bf16 *>(Ns), n_slot, ns_slot);
  return hipGetLastError();
}

hipError_t launch_pack_ctn(const PackTables &pt, const double *C, uint16_t *Cth, uint16_t *Ctl, long long maxblk,
                           hipStream_t s) {
  if (pt.nblk == 0) return hipSuccess;
  const int ychunks = (int)((maxblk + 256 * 16 - 1) / (256 * 16));
  dim3 grid(pt.nblk, ychunks > 0 ? ychunks : 1);
  hipLaunchKernelGGL(pack_ctn_kernel, grid, dim3(256), 0, s, pt, C, reinterpret_cast<__bf16 *>(Cth),
                     reinterpret_cast<__bf16 *>(Ctl));
  return hipGetLastError();
}

hipError_t launch_pad_gt(const double *Gocc, const double *Gun, int nR, int nb, int nbp, int nbq, const int *gsrc,
                         const int *gexp, uint16_t *GTh, uint16_t *GTl, hipStream_t s) {
  const size_t n = (size_t)2 * nR * nbp * nbq;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(pad_gt_kernel, dim3(blocks), dim3(256), 0, s, Gocc, Gun, nR, nb, nbp, nbq, gsrc, gexp,
                     reinterpret_cast<__bf16 *>(GTh), reinterpret_cast<__bf16 *>(GTl));
  return hipGetLastError();
}

hipError_t launch_nstage_bf16(const Chi0Tables &tb, const NTiles &tiles, int bm, const uint16_t *GTh,
                              const uint16_t *GTl, unsigned gt_bytes, const uint16_t *Cth, const uint16_t *Ctl,
                              unsigned ct_bytes, float *Nbuf, int nslots, size_t gt_slot, size_t n_slot,
                              hipStream_t s) {
  if (tiles.count == 0 || nslots <= 0) return hipSuccess;
  const __bf16 *gh = reinterpret_cast<const __bf16 *>(GTh), *gl = reinterpret_cast<const __bf16 *>(GTl);
  const __bf16 *ch = reinterpret_cast<const __bf16 *>(Cth), *cl = reinterpret_cast<const __bf16 *>(Ctl);
  if (bm == 256)
    hipLaunchKernelGGL(nstage_bf16_kernel<256>, dim3(tiles.count, nslots), dim3(512), 0, s, tb, tiles, gh, gl,
                       gt_bytes, ch, cl, ct_bytes, Nbuf, gt_slot, n_slot);
  else if (bm == 128)
    hipLaunchKernelGGL(nstage_bf16_kernel<128>, dim3(tiles.count, nslots), dim3(256), 0, s, tb, tiles, gh, gl,
                       gt_bytes, ch, cl, ct_bytes, Nbuf, gt_slot, n_slot);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fused_bf16_single(const Chi0Tables &tb, const SingleLaunch &a, int mode, hipStream_t s) {
  const long long n = (long long)a.nslots * a.nitems;
  if (n == 0) return hipSuccess;
  if (n > 0x7fffffffLL || mode < 1 || mode > 3) return hipErrorInvalidValue;
  if (mode == 1)
    hipLaunchKernelGGL((fused_bf16_single<8, 1>), dim3((unsigned)n), dim3(512), 0, s, tb, a);
  else if (mode == 2)
    hipLaunchKernelGGL((fused_bf16_single<4, 1>), dim3((unsigned)n), dim3(256), 0, s, tb, a);
  else
    hipLaunchKernelGGL((fused_bf16_single<4, 2>), dim3((unsigned)n), dim3(256), 0, s, tb, a);
  return hipGetLastError();
}
