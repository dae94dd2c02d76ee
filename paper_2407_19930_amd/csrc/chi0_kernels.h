// Device tables and launchers of the chi0(R, tau) build (Algorithm 1 restructured for gfx950).
#pragma once

#include "common.h"

// Read-only tables built by the plan.  Indices:
//   atoms a in [0, natoms); NAO k in [0, nb); lattice vectors R in [0, nR) (flattened BvK).
struct Chi0Tables {
  const int *nao, *naux, *ao_off, *aux_off;   // [natoms]
  const int *atom_of_ao;                      // [nb]
  // neighbourhood N[U] (CSR over first atom U): entry e = block with I = U
  const int *nbr_start;                       // [natoms + 1]
  const int *nbr_K, *nbr_R1;                  // [nblk] second atom, folded lattice vector
  const int *nbr_run_end;                     // [nblk] end of the run of entries with the same K
  const long long *nbr_cp;                    // [nblk] offset of the packed block [k][i][mu]
  const long long *nbr_cb;                    // [nblk] offset of the split-BF16 block (BF16X3 plans)
  const int *nslices;                         // [natoms] sum of nao[K] over the neighbours of U
  // split-BF16 N stage: groups of 8 contraction rows of atom V (CSR), each {A column g' of the
  // padded GT layout, BvK components of dL packed as for row_info, CtN row stride, 0} and the
  // CtN element offset of the group's first row
  const int *ngrp_start;                      // [natoms + 1]
  const int4 *ngrp;
  const long long *ngrp_off;
  int nbq;                                    // padded NAO columns of GT (sum of nao rounded up to 8)
  // contraction rows of the N-stage for atom V: r in [rows_start[V], rows_start[V+1])
  //   row r <-> (neighbour L(dL) of V, NAO l of L); row_info[r] = {G row ao_off[L] + l,
  //   BvK components of dL packed as d0 | d1 << 10 | d2 << 20, packed-C offset of row
  //   [l][j][nu] (low, high 32 bits)}
  const int *rows_start;                      // [natoms + 1]
  const int4 *row_info;
  // N buffer: block (V, K, dR) at noff[(V * natoms + K) * nR + dR], layout [k][s][j][nu]
  const long long *noff;
  // split-BF16 copy of N for the O GEMM of the split-BF16 fused kernel: block (V, K, dR) at
  // noffs[...] (bf16 elements), layout [k][part hi/lo][nu][JP], JP = 2 n_V rounded up to 8, zeros
  // in the j' >= 2 n_V padding
  const long long *noffs;
  const int *cp_stride;                       // [natoms] packed row stride of atom U's blocks
  int natoms, nb, nbp, nauxtot, nR;           // nbp: nb rounded up to a multiple of 8
  Bvk bvk;
};

// Green's-function screening of one tau (the decay of G that limits the range of R, Sec. 2 after
// Algorithm 1; the threshold on G of the case study, Sec. 6).  For every (U, V, R):
//   gb[(U natoms + V) nR + R] = max over s, i in U, j in V of |G^s_ij(R)|,
//   gn[(V natoms + K) nR + dR] = max over L(dL) in N[V] of gb(L, K, dR - dL),
//   gc[0] = g = max gb, gc[1] = cut = (theta g) g.
// A fused-kernel item (U, V, R) keeps the M terms of neighbour K(R1) of U when
// gb(U, V, R) gn(V, K, R1 - R) >= cut and its Z terms when gn(U, V, R) gn(V, U, -R) >= cut
// (FP64 products and comparisons).  stats (may be null): per launched item {neighbour entries
// kept, K(R1) slices kept, Z terms kept (0 or 1)}.  Screening is off when gb is null.
struct Screen {
  const double *gb, *gn, *gc;
  int *stats;
};

// Work lists.
struct NTiles {      // N-stage output tiles: atom V, first row (s, dR, k), first column (j, nu)
  const int *V, *m0, *n0;
  int count;
};
struct PairItems {   // fused-kernel items: atom pair U <= V and lattice vector R
  const int *U, *V, *R;
  int count;
};

struct PackTables {  // repack of the caller's LRI blocks
  const long long *in_off, *out_off;
  const long long *cb_off;                    // split-BF16 layout (BF16X3 plans)
  const long long *ctn_off;                   // split-BF16 N-stage layout of C (BF16X3 plans)
  const int *a, *ni, *nk, *stride;
  int nblk;
};

// launchers (return hipError_t of the launch)
template <typename T>
hipError_t launch_pack_c(const PackTables &pt, const double *C, T *Cp, long long maxblk, hipStream_t s);
// Per-tau power-of-two scale of G: gexp[s] = e with max |G^s| 2^e in [1, 2) (0 for an all-zero
// G); part holds 2 * kGscaleBlocks doubles of partial maxima.
constexpr int kGscaleBlocks = 256;
hipError_t launch_gscale(const double *Gocc, const double *Gun, size_t n, double *part, int *gexp, hipStream_t s);
// Gp[s][R][nbp][nbp] = G^s 2^gexp[s] in the compute precision (gexp may be null: no scale).
template <typename T>
hipError_t launch_pad_g(const double *Gocc, const double *Gun, int nR, int nb, int nbp, const int *gexp, T *Gp,
                        hipStream_t s);
template <typename T>
hipError_t launch_nstage(const Chi0Tables &tb, const NTiles &tiles, const T *Gp, const T *Cp, T *Nbuf,
                         size_t cp_elems, int kstep, hipStream_t s);  // kstep 16 or 32; cp_elems: size of Cp
// Fused kernel for a group of items whose atoms share the template classes
// mt = fused_mt_class(naux_U), js = fused_js_class(nao_V) and hc = i-tiles of U (1 or 2).
int fused_mt_class(int naux);
int fused_js_class(int nao);
// chi is written as negs 2^-(gexp[0] + gexp[1]) times the contraction (gexp may be null).
template <typename T>
hipError_t launch_fused(const Chi0Tables &tb, const PairItems &items, int mt, int js, int hc, const T *Gp,
                        const T *Cp, const T *Nbuf, double negs, const int *gexp, const Screen &sc, double *chi,
                        hipStream_t s);

// Split-BF16 (3-term) fused kernel on FP32 G and N, with C packed by launch_pack_cb (bf16 bits
// as uint16_t); ks = O-GEMM steps of 32 for the group's js class.
int fused_bf16_ks_class(int js_class);
hipError_t launch_pack_cb(const PackTables &pt, const double *C, uint16_t *Cb, long long maxblk, hipStream_t s);
// Split-BF16 N stage (see chi0_bf16.hip): C packed once, G transposed and padded per tau,
// hi / lo parts in separate arrays of below 2^32 bytes each.
hipError_t launch_pack_ctn(const PackTables &pt, const double *C, uint16_t *Cth, uint16_t *Ctl, long long maxblk,
                           hipStream_t s);
hipError_t launch_pad_gt(const double *Gocc, const double *Gun, int nR, int nb, int nbp, int nbq, const int *gsrc,
                         const int *gexp, uint16_t *GTh, uint16_t *GTl, hipStream_t s);
// nslots tau points in one launch (grid.y): slot t reads GTh/GTl + t gt_slot (elements) and
// writes Nbuf + t n_slot (elements).  bm: tile rows, 128 or 256 (tiles listed for that height).
hipError_t launch_nstage_bf16(const Chi0Tables &tb, const NTiles &tiles, int bm, const uint16_t *GTh,
                              const uint16_t *GTl, unsigned gt_bytes, const uint16_t *Cth, const uint16_t *Ctl,
                              unsigned ct_bytes, float *Nbuf, int nslots, size_t gt_slot, size_t n_slot,
                              hipStream_t s);
hipError_t launch_fused_bf16(const Chi0Tables &tb, const PairItems &items, int mt, int ks, int hc, const float *Gp,
                             const uint16_t *Cb, const float *Nbuf, const uint16_t *Ns, double negs, const int *gexp,
                             const Screen &sc, double *chi, hipStream_t s);
// Split-BF16 copy Ns (noffs layout, hi and lo parts) of the FP32 N intermediate of nslots tau
// points (slot t at N + t n_slot and Ns + t ns_slot, elements); one workgroup per block (V, K,
// dR) and slot, over the block's K(R1) slices.
hipError_t launch_split_n(const Chi0Tables &tb, const float *N, uint16_t *Ns, int nslots, size_t n_slot,
                          size_t ns_slot, hipStream_t s);

// Single split-BF16 fused launch over the items of nslots tau points, every template class in one
// launch (chi0_bf16.hip).  Per slot (tau of the launch): Gp, N, the two G-scale exponents, chi,
// and the screening bounds and statistics, each at slot * stride from the first.
struct SingleLaunch {
  const int *U, *V, *R, *cls;        // per plan item; cls = single_class(mt, ks, hc)
  const int *order;                  // [nitems] work units of a slot in launch order: items (8-wave
                                     // workgroups) or 2 item + half (4-wave workgroups)
  int nitems, nslots;
  const float *Gp;
  size_t gp_stride;
  const uint16_t *Cb;
  const float *Nbuf;
  size_t n_stride;
  const uint16_t *Ns;                // split-BF16 N (noffs layout)
  size_t ns_stride;
  const int *gexp;                   // [nslots][2]
  double negs;
  double *chi;
  size_t chi_stride;
  const double *gb, *gn, *gc;        // null: no screening; else strides natoms^2 nR, natoms^2 nR, 2
  int *stats;                        // null or per slot stats_stride ints, record = plan item
  size_t stats_stride;
};
// Class code of the single launch for (mt, ks, hc).
inline int single_class(int mt, int ks, int hc) { return (mt - 1) * 4 + (ks - 1) * 2 + (hc - 1); }
// mode 1: 8-wave workgroups, one per item; 2: 4-wave workgroups, one per half of an item's ABF
// columns (a.order holds 2 item + half); 3: 4-wave workgroups, one per item, two column tiles per
// wave
hipError_t launch_fused_bf16_single(const Chi0Tables &tb, const SingleLaunch &a, int mode, hipStream_t s);

// Screening bounds of one tau from FP64 G (see Screen): gb, then g and cut, then gn.
hipError_t launch_screen_norms(const Chi0Tables &tb, const double *Gocc, const double *Gun, double theta, double *gb,
                               double *gn, double *gc, hipStream_t s);

// compile-time limits of the kernels
constexpr int kMaxNao = 32;     // NAOs per atom
constexpr int kMaxNaux = 128;   // ABFs per atom
constexpr int kMaxNbr = 1024;   // LRI blocks (neighbours) per atom
// fused kernels: FP32 partial sums are folded into FP64 after at least this many K(R1) slices
constexpr int kFoldSlices = 16;
