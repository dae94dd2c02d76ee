// Neighbour table of one fused-kernel item (U <= V, R), shared by the FP64/FP32 and split-BF16
// fused kernels.
#pragma once

#include "chi0_kernels.h"

// Fills the LDS tables of item (U, V, R) with one row per kept entry e of the neighbourhood N[U]
// (Algorithm 1's loop over K(R1)): nbr_k = NAO count of K, nbr_c = cofs[e] (offset of the C block
// in the kernel's packed layout), nbr_n = nofs of the N block (V, K, R1 - R), nbr_g = end of the
// run of kept entries with the same atom K.  Without screening every entry is kept.  With
// screening the M terms of entry e are kept when gb(U, V, R) gn(V, K, R1 - R) >= cut, and the
// kept entries keep their order, so each atom's run stays contiguous.  pos: LDS scratch of
// kMaxNbr + 1 ints; meta: LDS scratch of 3 ints.  Every thread of the workgroup calls it; the
// tables are complete after the caller's next barrier.  Returns {entries kept, K(R1) slices
// kept, Z terms kept} (wave-uniform).
template <int NT>
__device__ __forceinline__ int3 item_table(const Chi0Tables &tb, const Screen &sc, const long long *__restrict__ cofs,
                                           const long long *__restrict__ nofs, int U, int V, int R, long long *nbr_c,
                                           long long *nbr_n, int *nbr_k, int *nbr_g, int *pos, int *meta) {
  const int tid = threadIdx.x;
  const int natoms = tb.natoms, nR = tb.nR;
  const int e0 = tb.nbr_start[U], ne = tb.nbr_start[U + 1] - e0;
  if (!sc.gb) {
    for (int e = tid; e < ne; e += NT) {
      const int K = tb.nbr_K[e0 + e];
      nbr_k[e] = tb.nao[K];
      nbr_c[e] = cofs[e0 + e];
      nbr_n[e] = nofs[((size_t)V * natoms + K) * nR + tb.bvk.sub(tb.nbr_R1[e0 + e], R)];
      nbr_g[e] = tb.nbr_run_end[e0 + e] - e0;
    }
    return make_int3(ne, tb.nslices[U], 1);
  }
  const double cut = sc.gc[1];
  const double gUV = sc.gb[((size_t)U * natoms + V) * nR + R];
  for (int e = tid; e < ne; e += NT) {
    const int K = tb.nbr_K[e0 + e];
    const double gk = sc.gn[((size_t)V * natoms + K) * nR + tb.bvk.sub(tb.nbr_R1[e0 + e], R)];
    pos[e] = gUV * gk >= cut ? 1 : 0;
  }
  __syncthreads();
  if (tid < 64) {
    // wave 0: exclusive prefix sum of the keep flags (pos[ne] = entries kept) and the slice count
    int base = 0, nsl = 0;
    for (int c = 0; c < ne; c += 64) {
      const int e = c + tid;
      const int f = e < ne ? pos[e] : 0;
      const unsigned long long m = __ballot(f);
      if (e < ne) pos[e] = base + __popcll(m & ((1ull << tid) - 1ull));
      if (f) nsl += tb.nao[tb.nbr_K[e0 + e]];
      base += __popcll(m);
    }
    for (int o = 32; o > 0; o >>= 1) nsl += __shfl_xor(nsl, o);
    if (tid == 0) {
      pos[ne] = base;
      const double gz = sc.gn[((size_t)U * natoms + V) * nR + R] * sc.gn[((size_t)V * natoms + U) * nR + tb.bvk.neg(R)];
      meta[0] = base;
      meta[1] = nsl;
      meta[2] = gz >= cut ? 1 : 0;
    }
  }
  __syncthreads();
  for (int e = tid; e < ne; e += NT) {
    const int p = pos[e];
    if (pos[e + 1] != p) {
      const int K = tb.nbr_K[e0 + e];
      nbr_k[p] = tb.nao[K];
      nbr_c[p] = cofs[e0 + e];
      nbr_n[p] = nofs[((size_t)V * natoms + K) * nR + tb.bvk.sub(tb.nbr_R1[e0 + e], R)];
      nbr_g[p] = pos[tb.nbr_run_end[e0 + e] - e0];
    }
  }
  return make_int3(uniform(meta[0]), uniform(meta[1]), uniform(meta[2]));
}

// Per-item screening statistics (thread 0 of the workgroup) at record `index`.
__device__ __forceinline__ void item_stats(const Screen &sc, int index, int3 kept) {
  if (sc.stats && threadIdx.x == 0) {
    int *st = sc.stats + 3 * (size_t)index;
    st[0] = kept.x;
    st[1] = kept.y;
    st[2] = kept.z;
  }
}
