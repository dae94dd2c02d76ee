// tau -> i omega cosine transform and R -> q Fourier transform (Sec. 2), FP64.
// Both are streaming kernels bound by HBM bandwidth: each thread owns one matrix
// element and walks the short tau (or R) axis, reading each input once.
#include "common.h"

namespace {

constexpr int kMaxTau = 64;

// y[k][e] = sum_j W[k][j] x[j][e]; W staged in LDS, kKG frequencies per register group.
constexpr int kKG = 8;
__global__ __launch_bounds__(256) void cos_transform_kernel(const double *__restrict__ W, int ntau, int nomega,
                                                            size_t n, const double *__restrict__ x,
                                                            double *__restrict__ y) {
  __shared__ double Ws[kMaxTau * kMaxTau];
  for (int i = threadIdx.x; i < ntau * nomega; i += blockDim.x) Ws[i] = W[i];
  __syncthreads();
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    for (int k0 = 0; k0 < nomega; k0 += kKG) {
      double acc[kKG];
#pragma unroll
      for (int g = 0; g < kKG; ++g) acc[g] = 0.0;
      for (int j = 0; j < ntau; ++j) {
        const double v = x[(size_t)j * n + e];
#pragma unroll
        for (int g = 0; g < kKG; ++g) {
          const int k = k0 + g < nomega ? k0 + g : nomega - 1;
          acc[g] = fma(Ws[k * ntau + j], v, acc[g]);
        }
      }
#pragma unroll
      for (int g = 0; g < kKG; ++g)
        if (k0 + g < nomega) y[(size_t)(k0 + g) * n + e] = acc[g];
    }
  }
}

// y[b][q][e] = sum_R (cos, sin)[q][R] x[b][R][e], complex interleaved output.
constexpr int kQG = 8;   // q points per register group
__global__ __launch_bounds__(256) void r2q_kernel(const double *__restrict__ ph, int nR, int nq, size_t m,
                                                  const double *__restrict__ x, double *__restrict__ y) {
  extern __shared__ double phs[];          // [nq][nR][2]
  for (int i = threadIdx.x; i < 2 * nq * nR; i += blockDim.x) phs[i] = ph[i];
  __syncthreads();
  const int b = blockIdx.y;
  const double *xb = x + (size_t)b * nR * m;
  double *yb = y + (size_t)b * nq * m * 2;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (size_t)gridDim.x * blockDim.x) {
    for (int q0 = 0; q0 < nq; q0 += kQG) {
      double re[kQG], im[kQG];
#pragma unroll
      for (int g = 0; g < kQG; ++g) re[g] = im[g] = 0.0;
      for (int r = 0; r < nR; ++r) {
        const double v = xb[(size_t)r * m + e];
#pragma unroll
        for (int g = 0; g < kQG; ++g) {
          const int q = q0 + g < nq ? q0 + g : nq - 1;
          re[g] = fma(phs[(q * nR + r) * 2], v, re[g]);
          im[g] = fma(phs[(q * nR + r) * 2 + 1], v, im[g]);
        }
      }
#pragma unroll
      for (int g = 0; g < kQG; ++g) {
        if (q0 + g < nq) {
          double2 o;
          o.x = re[g];
          o.y = im[g];
          reinterpret_cast<double2 *>(yb)[(size_t)(q0 + g) * m + e] = o;
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_cos_transform(const double *W_dev, int ntau, int nomega, size_t n, const double *x, double *y,
                                hipStream_t s) {
  if (ntau > kMaxTau || nomega > kMaxTau) return hipErrorInvalidValue;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(cos_transform_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, W_dev, ntau, nomega,
                     n, x, y);
  return hipGetLastError();
}

hipError_t launch_r2q(const double *ph_dev, int nR, int nq, int nbatch, size_t m, const double *x, double *y,
                      hipStream_t s) {
  const size_t lds = (size_t)2 * nq * nR * sizeof(double);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  const int blocks = (int)std::min<size_t>((m + 255) / 256, 4096);
  hipLaunchKernelGGL(r2q_kernel, dim3(blocks > 0 ? blocks : 1, nbatch), dim3(256), lds, s, ph_dev, nR, nq, m, x, y);
  return hipGetLastError();
}
