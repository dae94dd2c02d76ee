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
  const long long *nbr_cp;                    // [nblk] offset of the packed block [k][i][mu]
  // contraction rows of the N-stage for atom V: r in [rows_start[V], rows_start[V+1])
  //   row r <-> (neighbour L(dL) of V, NAO l of L)
  const int *rows_start;                      // [natoms + 1]
  const int *row_g;                           // G row index ao_off[L] + l
  const int *row_dl;                          // folded dL
  const long long *row_cp;                    // offset of packed row [l][j][nu] (n_V * a_V values)
  // N buffer: block (V, K, dR) at noff[(V * natoms + K) * nR + dR], layout [k][s][j][nu]
  const long long *noff;
  int natoms, nb, nauxtot, nR;
  Bvk bvk;
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
  const int *a, *ni, *nk;
  int nblk;
};

// launchers (return hipError_t of the launch)
template <typename T>
hipError_t launch_pack_c(const PackTables &pt, const double *C, T *Cp, long long maxblk, hipStream_t s);
hipError_t launch_convert_g(const double *src, float *dst, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_nstage(const Chi0Tables &tb, const NTiles &tiles, const T *Gocc, const T *Gun,
                         const T *Cp, T *Nbuf, hipStream_t s);
template <typename T>
hipError_t launch_fused(const Chi0Tables &tb, const PairItems &items, const T *Gocc, const T *Gun,
                        const T *Cp, const T *Nbuf, double negs, double *chi, hipStream_t s);

// compile-time limits of the kernels
constexpr int kMaxNao = 32;     // NAOs per atom
constexpr int kMaxNaux = 128;   // ABFs per atom
