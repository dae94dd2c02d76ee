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

namespace {

template <typename T>
__global__ __launch_bounds__(256) void pack_c_kernel(PackTables pt, const double *__restrict__ C,
                                                     T *__restrict__ Cp) {
  const int b = blockIdx.x;
  const int a = pt.a[b], ni = pt.ni[b], nk = pt.nk[b];
  const long long total = (long long)a * ni * nk;
  const double *src = C + pt.in_off[b];
  T *dst = Cp + pt.out_off[b];
  for (long long e = (long long)blockIdx.y * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.y * blockDim.x) {
    const int mu = (int)(e % a);
    const long long t = e / a;
    const int i = (int)(t % ni);
    const int k = (int)(t / ni);
    dst[e] = (T)src[((long long)mu * ni + i) * nk + k];
  }
}

__global__ __launch_bounds__(256) void convert_g_kernel(const double *__restrict__ src,
                                                        float *__restrict__ dst, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

// ---------------------------------------------------------------------------
// N-stage: out[(s, dR, k)][(j, nu)] = sum_r A[(s,dR,k)][r] B[r][(j,nu)]
//   A[(s,dR,k)][r] = G^s[dR - dL(r)][g(r)][k],  B[r][(j,nu)] = Cp[row_cp(r) + j*a_V + nu]
// 128x128 output tile per workgroup, 4 waves of 64x64, K step 16, LDS double buffer.
// kSplit: FP32 MFMA partial sums are added into FP64 every kFlush K steps.
// ---------------------------------------------------------------------------
constexpr int NS_BM = 128, NS_BN = 128, NS_BK = 16, NS_THREADS = 256;

template <typename T, bool kSplit>
__global__ __launch_bounds__(NS_THREADS) void nstage_kernel(Chi0Tables tb, NTiles tiles,
                                                            const T *__restrict__ Gocc,
                                                            const T *__restrict__ Gun,
                                                            const T *__restrict__ Cp,
                                                            T *__restrict__ Nbuf) {
  typedef typename Mfma<T>::acc Acc;
  constexpr int kFlush = 8;
  __shared__ T As[2][NS_BK][NS_BM];
  __shared__ T Bs[2][NS_BK][NS_BN];

  const int t = blockIdx.x;
  const int V = tiles.V[t], m0 = tiles.m0[t], n0 = tiles.n0[t];
  const int nV = tb.nao[V], aV = tb.naux[V];
  const int NV = nV * aV;
  const int nb = tb.nb, nR = tb.nR;
  const size_t nbnb = (size_t)nb * nb;
  const int M = 2 * nR * nb;
  const int r0 = tb.rows_start[V];
  const int S = tb.rows_start[V + 1] - r0;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int col = lane & 15, grp = lane >> 4;

  // loader coordinates (fixed over the K loop)
  const int lm = tid & 127, lr = (tid >> 7) * 8;
  const int m = m0 + lm;
  const bool mvalid = m < M;
  int ss = 0, dR = 0, kk = 0;
  if (mvalid) {
    ss = m / (nR * nb);
    const int rem = m - ss * nR * nb;
    dR = rem / nb;
    kk = rem - dR * nb;
  }
  const T *Gs = ss ? Gun : Gocc;
  const int n = n0 + lm;
  const bool nvalid = n < NV;

  T ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = k0 + lr + e;
      T va = T(0), vb = T(0);
      if (r < S) {
        const int rr = r0 + r;
        if (mvalid) {
          const int Rp = tb.bvk.sub(dR, tb.row_dl[rr]);
          va = Gs[(size_t)Rp * nbnb + (size_t)tb.row_g[rr] * nb + kk];
        }
        if (nvalid) vb = Cp[tb.row_cp[rr] + n];
      }
      ra[e] = va;
      rb[e] = vb;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[buf][lr + e][lm] = ra[e];
      Bs[buf][lr + e][lm] = rb[e];
    }
  };

  Acc acc[4][4];
  double acc64[4][4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      acc[a][b] = Mfma<T>::zero();
      if (kSplit)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[a][b][r] = 0.0;
    }

  const int nk = (S + NS_BK - 1) / NS_BK;
  load(0);
  store(0);
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) load((it + 1) * NS_BK);
#pragma unroll
    for (int ks = 0; ks < NS_BK / 4; ++ks) {
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
          for (int r = 0; r < 4; ++r) acc64[a][b][r] += (double)acc[a][b][r];
          acc[a][b] = Mfma<T>::zero();
        }
    }
    if (it + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  // epilogue: scatter rows (s, dR, k) into N blocks (V, K(k), dR), layout [k][s][j][nu]
#pragma unroll
  for (int tm = 0; tm < 4; ++tm) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mm = m0 + wm * 64 + tm * 16 + Mfma<T>::row(grp, r);
      if (mm >= M) continue;
      const int s2 = mm / (nR * nb);
      const int rem = mm - s2 * nR * nb;
      const int dR2 = rem / nb;
      const int k2 = rem - dR2 * nb;
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
// Wave w owns ABF columns nu in [16w, 16w+16) of V and all mu-tiles of U.
// ---------------------------------------------------------------------------
constexpr int FU_THREADS = 512;
constexpr int FU_MAXMT = kMaxNaux / 16;     // mu tiles
constexpr int FU_MAXJS = 2 * kMaxNao / 4;   // K steps of the O GEMM (j' = (s, j))
constexpr int FU_SLICE = kMaxNao * kMaxNaux;
constexpr int FU_LOADS = FU_SLICE / FU_THREADS;

template <typename T, bool kSplit>
__global__ __launch_bounds__(FU_THREADS) void fused_kernel(Chi0Tables tb, PairItems items,
                                                           const T *__restrict__ Gocc,
                                                           const T *__restrict__ Gun,
                                                           const T *__restrict__ Cp,
                                                           const T *__restrict__ Nbuf, double negs,
                                                           double *__restrict__ chi) {
  typedef typename Mfma<T>::acc Acc;
  __shared__ T Cs[2][FU_SLICE];

  const int item = blockIdx.x;
  const int U = items.U[item], V = items.V[item], R = items.R[item];
  const int nU = tb.nao[U], aU = tb.naux[U], nV = tb.nao[V], aV = tb.naux[V];
  const int natoms = tb.natoms, nR = tb.nR, nb = tb.nb;
  const size_t nbnb = (size_t)nb * nb;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int nu = w * 16 + col;
  const bool wave_active = w * 16 < aV;
  const bool nu_ok = nu < aV;
  const int mt = (aU + 15) / 16;
  const int hc = nU > 16 ? 2 : 1;
  const int js = (2 * nV + 3) / 4;

  // A operand of the O GEMM: A[i][j'] = G^{un}_{ij}(R) for j' = j (pairs with N^occ),
  //                                     G^{occ}_{ij}(R) for j' = nV + j (pairs with N^un)
  T afr[2][FU_MAXJS];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int st = 0; st < FU_MAXJS; ++st) {
      T v = T(0);
      const int i = 16 * h + col, jp = 4 * st + grp;
      if (h < hc && st < js && i < nU && jp < 2 * nV) {
        const int s = jp >= nV;
        const int j = jp - s * nV;
        const T *G = s ? Gocc : Gun;
        v = G[(size_t)R * nbnb + (size_t)(tb.ao_off[U] + i) * nb + tb.ao_off[V] + j];
      }
      afr[h][st] = v;
    }

  Acc acc[FU_MAXMT];
  double acc64[FU_MAXMT][4];
#pragma unroll
  for (int m = 0; m < FU_MAXMT; ++m) {
    acc[m] = Mfma<T>::zero();
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[m][r] = 0.0;
  }
  auto flush = [&]() {
    if (kSplit) {
#pragma unroll
      for (int m = 0; m < FU_MAXMT; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[m][r] += (double)acc[m][r];
        acc[m] = Mfma<T>::zero();
      }
    }
  };

  // ---- Z terms: contraction over (s, i, j) of N(U,V,R)[j][s][i][mu] and N(V,U,-R)[i][1-s][j][nu]
  const int negR = tb.bvk.neg(R);
  {
    const T *NA = Nbuf + tb.noff[((size_t)U * natoms + V) * nR + R];
    const T *NB = Nbuf + tb.noff[((size_t)V * natoms + U) * nR + negR];
    if (wave_active) {
      const int F = 2 * nU * nV;
      for (int f0 = 0; f0 < F; f0 += 4) {
        const int f = f0 + grp;
        const bool fv = f < F;
        int s = 0, i = 0, j = 0;
        if (fv) {
          s = f / (nU * nV);
          const int rem = f - s * nU * nV;
          i = rem / nV;
          j = rem - i * nV;
        }
        const T bz = (fv && nu_ok) ? NB[((size_t)(i * 2 + 1 - s) * nV + j) * aV + nu] : T(0);
#pragma unroll
        for (int m = 0; m < FU_MAXMT; ++m) {
          if (m < mt) {
            const int mu = 16 * m + col;
            const T az = (fv && mu < aU) ? NA[((size_t)(j * 2 + s) * nU + i) * aU + mu] : T(0);
            acc[m] = Mfma<T>::fma(az, bz, acc[m]);
          }
        }
      }
    }
    flush();
  }

  // ---- K(R1) loop over slices k of the packed C blocks [k][i][mu]
  const int e0 = tb.nbr_start[U], e1 = tb.nbr_start[U + 1];
  const int sliceN = nU * aU;
  T rc[FU_LOADS];
  auto load_slice = [&](const T *src) {
#pragma unroll
    for (int q = 0; q < FU_LOADS; ++q) {
      const int idx = tid + q * FU_THREADS;
      rc[q] = idx < sliceN ? src[idx] : T(0);
    }
  };
  auto store_slice = [&](int buf) {
#pragma unroll
    for (int q = 0; q < FU_LOADS; ++q) {
      const int idx = tid + q * FU_THREADS;
      if (idx < sliceN) Cs[buf][idx] = rc[q];
    }
  };

  if (e0 < e1) {
    int e = e0, k = 0, cur = 0;
    int nK = tb.nao[tb.nbr_K[e]];
    const T *Cblk = Cp + tb.nbr_cp[e];
    const T *Nblk = Nbuf + tb.noff[((size_t)V * natoms + tb.nbr_K[e]) * nR + tb.bvk.sub(tb.nbr_R1[e], R)];
    load_slice(Cblk);
    store_slice(0);
    __syncthreads();
    while (e < e1) {
      int e2 = e, k2 = k + 1;
      if (k2 == nK) {
        e2 = e + 1;
        k2 = 0;
      }
      if (e2 < e1) {
        const T *src = (e2 == e) ? Cblk : (Cp + tb.nbr_cp[e2]);
        load_slice(src + (size_t)k2 * sliceN);
      }
      if (wave_active) {
        // O[i][nu] = sum_j' A[i][j'] N[k][j'][nu]
        Acc o0 = Mfma<T>::zero(), o1 = Mfma<T>::zero();
        const T *nrow = Nblk + (size_t)k * 2 * nV * aV;
#pragma unroll
        for (int st = 0; st < FU_MAXJS; ++st) {
          if (st < js) {
            const int jp = 4 * st + grp;
            const T b = (jp < 2 * nV && nu_ok) ? nrow[(size_t)jp * aV + nu] : T(0);
            o0 = Mfma<T>::fma(afr[0][st], b, o0);
            if (hc > 1) o1 = Mfma<T>::fma(afr[1][st], b, o1);
          }
        }
        // chi[mu][nu] += sum_i C[k][i][mu] O[i][nu]; register r of O holds row i = row(grp, r)
        const T *cs = Cs[cur];
#pragma unroll
        for (int m = 0; m < FU_MAXMT; ++m) {
          if (m < mt) {
            const int mu = 16 * m + col;
            const bool muok = mu < aU;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = Mfma<T>::row(grp, r);
              const T c = (muok && i < nU) ? cs[i * aU + mu] : T(0);
              acc[m] = Mfma<T>::fma(c, o0[r], acc[m]);
            }
            if (hc > 1) {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int i = 16 + Mfma<T>::row(grp, r);
                const T c = (muok && i < nU) ? cs[i * aU + mu] : T(0);
                acc[m] = Mfma<T>::fma(c, o1[r], acc[m]);
              }
            }
          }
        }
      }
      if (e2 != e) flush();
      if (e2 < e1) store_slice(cur ^ 1);
      __syncthreads();
      if (e2 != e && e2 < e1) {
        const int K2 = tb.nbr_K[e2];
        nK = tb.nao[K2];
        Cblk = Cp + tb.nbr_cp[e2];
        Nblk = Nbuf + tb.noff[((size_t)V * natoms + K2) * nR + tb.bvk.sub(tb.nbr_R1[e2], R)];
      }
      e = e2;
      k = k2;
      cur ^= 1;
    }
  }

  // ---- epilogue: chi_UV(R) and chi_VU(-R) = chi_UV(R)^T
  if (!wave_active || !nu_ok) return;
  const size_t N = tb.nauxtot;
  const int au0 = tb.aux_off[U], av0 = tb.aux_off[V];
#pragma unroll
  for (int m = 0; m < FU_MAXMT; ++m) {
    if (m < mt) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mu = 16 * m + Mfma<T>::row(grp, r);
        if (mu < aU) {
          const double v = negs * (kSplit ? acc64[m][r] : (double)acc[m][r]);
          chi[((size_t)R * N + au0 + mu) * N + av0 + nu] = v;
          if (U != V) chi[((size_t)negR * N + av0 + nu) * N + au0 + mu] = v;
        }
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

hipError_t launch_convert_g(const double *src, float *dst, size_t n, hipStream_t s) {
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(convert_g_kernel, dim3(blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_nstage(const Chi0Tables &tb, const NTiles &tiles, const T *Gocc, const T *Gun,
                         const T *Cp, T *Nbuf, hipStream_t s) {
  if (tiles.count == 0) return hipSuccess;
  if (sizeof(T) == 4)
    hipLaunchKernelGGL((nstage_kernel<T, true>), dim3(tiles.count), dim3(NS_THREADS), 0, s, tb, tiles, Gocc,
                       Gun, Cp, Nbuf);
  else
    hipLaunchKernelGGL((nstage_kernel<T, false>), dim3(tiles.count), dim3(NS_THREADS), 0, s, tb, tiles, Gocc,
                       Gun, Cp, Nbuf);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fused(const Chi0Tables &tb, const PairItems &items, const T *Gocc, const T *Gun,
                        const T *Cp, const T *Nbuf, double negs, double *chi, hipStream_t s) {
  if (items.count == 0) return hipSuccess;
  if (sizeof(T) == 4)
    hipLaunchKernelGGL((fused_kernel<T, true>), dim3(items.count), dim3(FU_THREADS), 0, s, tb, items, Gocc,
                       Gun, Cp, Nbuf, negs, chi);
  else
    hipLaunchKernelGGL((fused_kernel<T, false>), dim3(items.count), dim3(FU_THREADS), 0, s, tb, items, Gocc,
                       Gun, Cp, Nbuf, negs, chi);
  return hipGetLastError();
}

template hipError_t launch_pack_c<double>(const PackTables &, const double *, double *, long long, hipStream_t);
template hipError_t launch_pack_c<float>(const PackTables &, const double *, float *, long long, hipStream_t);
template hipError_t launch_nstage<double>(const Chi0Tables &, const NTiles &, const double *, const double *,
                                          const double *, double *, hipStream_t);
template hipError_t launch_nstage<float>(const Chi0Tables &, const NTiles &, const float *, const float *,
                                         const float *, float *, hipStream_t);
template hipError_t launch_fused<double>(const Chi0Tables &, const PairItems &, const double *, const double *,
                                         const double *, const double *, double, double *, hipStream_t);
template hipError_t launch_fused<float>(const Chi0Tables &, const PairItems &, const float *, const float *,
                                        const float *, const float *, double, double *, hipStream_t);
