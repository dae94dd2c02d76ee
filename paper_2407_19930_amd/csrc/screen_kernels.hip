// Bounds of the Green's-function screening of one tau (the decay of G limits the range of the
// lattice vector R, Sec. 2 after Algorithm 1; the case study screens on G with a threshold,
// Sec. 6).  All in FP64 from the caller's G; maxima are exact, so the keep decisions of the fused
// kernels do not depend on the order of the reductions.
#include "chi0_kernels.h"

namespace {

// gb[(U natoms + V) nR + R] = max over s, i in U, j in V of |G^s_ij(R)|: one wave per (U, V, R).
__global__ __launch_bounds__(64) void gblock_kernel(const double *__restrict__ Gocc, const double *__restrict__ Gun,
                                                    const int *__restrict__ nao, const int *__restrict__ ao_off,
                                                    int natoms, int nR, int nb, double *__restrict__ gb) {
  const int idx = blockIdx.x;
  const int R = idx % nR, uv = idx / nR;
  const int V = uv % natoms, U = uv / natoms;
  const int nU = nao[U], nV = nao[V], i0 = ao_off[U], j0 = ao_off[V];
  double m = 0.0;
  for (int e = threadIdx.x; e < nU * nV; e += 64) {
    const int i = e / nV, j = e - i * nV;
    const size_t o = ((size_t)R * nb + i0 + i) * nb + j0 + j;
    m = fmax(m, fmax(fabs(Gocc[o]), fabs(Gun[o])));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if (threadIdx.x == 0) gb[idx] = m;
}

// gc[0] = g = max of gb, gc[1] = (theta g) g: one workgroup.
constexpr int GC_THREADS = 1024;
__global__ __launch_bounds__(GC_THREADS) void gcut_kernel(const double *__restrict__ gb, size_t n, double theta,
                                                          double *__restrict__ gc) {
  __shared__ double red[GC_THREADS];
  double m = 0.0;
  for (size_t e = threadIdx.x; e < n; e += GC_THREADS) m = fmax(m, gb[e]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = GC_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double g = red[0];
    gc[0] = g;
    gc[1] = (theta * g) * g;
  }
}

// gn[(V natoms + K) nR + dR] = max over entries L(dL) of N[V] of gb(L, K, dR - dL); zero for an
// atom without neighbours.  One thread per (V, K, dR).
__global__ __launch_bounds__(256) void gneigh_kernel(Chi0Tables tb, const double *__restrict__ gb,
                                                     double *__restrict__ gn) {
  const int natoms = tb.natoms, nR = tb.nR;
  const size_t n = (size_t)natoms * natoms * nR;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int dR = (int)(idx % nR);
  const size_t vk = idx / nR;
  const int K = (int)(vk % natoms), V = (int)(vk / natoms);
  double m = 0.0;
  for (int e = tb.nbr_start[V]; e < tb.nbr_start[V + 1]; ++e) {
    const int L = tb.nbr_K[e];
    m = fmax(m, gb[((size_t)L * natoms + K) * nR + tb.bvk.sub(dR, tb.nbr_R1[e])]);
  }
  gn[idx] = m;
}

}  // namespace

hipError_t launch_screen_norms(const Chi0Tables &tb, const double *Gocc, const double *Gun, double theta, double *gb,
                               double *gn, double *gc, hipStream_t s) {
  const size_t n = (size_t)tb.natoms * tb.natoms * tb.nR;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(gblock_kernel, dim3((unsigned)n), dim3(64), 0, s, Gocc, Gun, tb.nao, tb.ao_off, tb.natoms, tb.nR,
                     tb.nb, gb);
  hipLaunchKernelGGL(gcut_kernel, dim3(1), dim3(GC_THREADS), 0, s, gb, n, theta, gc);
  hipLaunchKernelGGL(gneigh_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tb, gb, gn);
  return hipGetLastError();
}
