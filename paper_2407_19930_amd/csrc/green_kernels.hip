// Real-space imaginary-time Green's functions from Bloch eigenpairs (Sec. 2, Eq. (green_mat),
// factors of i taken out):
//   G^occ_{ij}(R, tau) = (1/N_k) sum_k e^{-i k.R} sum_{n occ} c_{in}(k) c*_{jn}(k) e^{-(mu - eps_nk) tau}
//   G^un_{ij}(R, tau)  = (1/N_k) sum_k e^{-i k.R} sum_{n un}  c_{in}(k) c*_{jn}(k) e^{-(eps_nk - mu) tau}
// Per (tau, channel): green_weight_kernel forms X_k = c_k[:, bands] diag(w) (complex), the batched
// complex GEMM of the energy stage gives W_k = X_k c_k[:, bands]^H for every k, and
// k2r_real_kernel sums the phases: G(R) = Re sum_k ph[R][k] W_k with ph = e^{-i k.R} / N_k.
// The imaginary part, zero for a time-reversal-symmetric H, is not formed.
#include <algorithm>

#include "green_kernels.h"

namespace {

// X[k][i][n'] = c[k][i][n0 + n'] w(k, n0 + n'), n' < nbs; w = e^{-(mu - eps) tau} (occupied) or
// e^{-(eps - mu) tau} (unoccupied).  Complex interleaved, X rows of nbs entries.
__global__ __launch_bounds__(256) void green_weight_kernel(const double *__restrict__ eps,
                                                           const double *__restrict__ wfc, int nk, int nb, int n0,
                                                           int nbs, double mu, double tau, int occupied,
                                                           double *__restrict__ X) {
  const size_t total = (size_t)nk * nb * nbs;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int np = (int)(e % nbs);
    const size_t ki = e / nbs;
    const int i = (int)(ki % nb);
    const int k = (int)(ki / nb);
    const int n = n0 + np;
    const double x = occupied ? mu - eps[(size_t)k * nb + n] : eps[(size_t)k * nb + n] - mu;
    const double w = exp(-x * tau);
    const double2 c = reinterpret_cast<const double2 *>(wfc)[((size_t)k * nb + i) * nb + n];
    reinterpret_cast<double2 *>(X)[e] = make_double2(c.x * w, c.y * w);
  }
}

// G[R][e] = sum_k Re(ph[R][k] W[k][e]), e < m; ph [nR][nk] complex in LDS; kRG lattice vectors
// per register group.
constexpr int kRG = 8;
__global__ __launch_bounds__(256) void k2r_real_kernel(const double *__restrict__ ph, int nR, int nk, size_t m,
                                                       const double *__restrict__ W, double *__restrict__ G) {
  extern __shared__ double phs[];          // [nR][nk][2]
  for (int i = threadIdx.x; i < 2 * nR * nk; i += blockDim.x) phs[i] = ph[i];
  __syncthreads();
  const double2 *W2 = reinterpret_cast<const double2 *>(W);
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (size_t)gridDim.x * blockDim.x) {
    for (int r0 = 0; r0 < nR; r0 += kRG) {
      double acc[kRG];
#pragma unroll
      for (int g = 0; g < kRG; ++g) acc[g] = 0.0;
      for (int k = 0; k < nk; ++k) {
        const double2 w = W2[(size_t)k * m + e];
#pragma unroll
        for (int g = 0; g < kRG; ++g) {
          const int r = r0 + g < nR ? r0 + g : nR - 1;
          const double pr = phs[(r * nk + k) * 2], pi = phs[(r * nk + k) * 2 + 1];
          acc[g] = fma(pr, w.x, fma(-pi, w.y, acc[g]));
        }
      }
#pragma unroll
      for (int g = 0; g < kRG; ++g)
        if (r0 + g < nR) G[(size_t)(r0 + g) * m + e] = acc[g];
    }
  }
}

}  // namespace

hipError_t launch_green_weight(const double *eps, const double *wfc, int nk, int nb, int n0, int nbs, double mu,
                               double tau, int occupied, double *X, hipStream_t s) {
  const size_t n = (size_t)nk * nb * nbs;
  if (n == 0) return hipSuccess;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(green_weight_kernel, dim3(blocks), dim3(256), 0, s, eps, wfc, nk, nb, n0, nbs, mu, tau, occupied,
                     X);
  return hipGetLastError();
}

hipError_t launch_k2r_real(const double *ph, int nR, int nk, size_t m, const double *W, double *G, hipStream_t s) {
  const size_t lds = (size_t)2 * nR * nk * sizeof(double);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  if (m == 0) return hipSuccess;
  const int blocks = (int)std::min<size_t>((m + 255) / 256, 4096);
  hipLaunchKernelGGL(k2r_real_kernel, dim3(blocks), dim3(256), lds, s, ph, nR, nk, m, W, G);
  return hipGetLastError();
}

namespace {

__global__ void clear2_kernel(double *out) {
  out[0] = 0.0;
  out[1] = 0.0;
}

// One workgroup per (s, tau, R): the largest deviation from G(-R) = G(R)^T and the largest
// entry, merged into out with integer maxima of the bit patterns (both values are >= 0).
__global__ __launch_bounds__(256) void green_symmetry_kernel(const double *__restrict__ Gocc,
                                                             const double *__restrict__ Gun, int ntau, int m0, int m1,
                                                             int m2, int nb, double *__restrict__ out) {
  const int nR = m0 * m1 * m2;
  const int R = blockIdx.x % nR, t = (blockIdx.x / nR) % ntau, s = blockIdx.x / (nR * ntau);
  const int c2 = R % m2, c1 = (R / m2) % m1, c0 = R / (m1 * m2);
  const int negR = (((m0 - c0) % m0) * m1 + (m1 - c1) % m1) * m2 + (m2 - c2) % m2;
  const double *G = (s ? Gun : Gocc) + (size_t)t * nR * nb * nb;
  const double *A = G + (size_t)R * nb * nb, *B = G + (size_t)negR * nb * nb;
  double dev = 0.0, mx = 0.0;
  for (size_t e = threadIdx.x; e < (size_t)nb * nb; e += blockDim.x) {
    const int i = (int)(e / nb), j = (int)(e % nb);
    const double a = A[e];
    dev = fmax(dev, fabs(B[(size_t)j * nb + i] - a));
    mx = fmax(mx, fabs(a));
  }
  for (int off = 32; off > 0; off >>= 1) {
    dev = fmax(dev, __shfl_xor(dev, off));
    mx = fmax(mx, __shfl_xor(mx, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(reinterpret_cast<unsigned long long *>(out), (unsigned long long)__double_as_longlong(dev));
    atomicMax(reinterpret_cast<unsigned long long *>(out + 1), (unsigned long long)__double_as_longlong(mx));
  }
}

}  // namespace

hipError_t launch_green_symmetry(const double *Gocc, const double *Gun, int ntau, const int mesh[3], int nb,
                                 double *out, hipStream_t s) {
  hipLaunchKernelGGL(clear2_kernel, dim3(1), dim3(1), 0, s, out);
  const long long blocks = 2LL * ntau * mesh[0] * mesh[1] * mesh[2];
  if (blocks <= 0 || nb <= 0) return hipGetLastError();
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(green_symmetry_kernel, dim3((unsigned)blocks), dim3(256), 0, s, Gocc, Gun, ntau, mesh[0], mesh[1],
                     mesh[2], nb, out);
  return hipGetLastError();
}
