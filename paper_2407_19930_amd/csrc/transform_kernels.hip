// tau -> i omega cosine transform and R -> q Fourier transform (Sec. 2), FP64.
// Both are streaming kernels bound by HBM bandwidth: each element's short tau (or R) axis is
// walked by one thread (or, for R -> q, by the few lanes that share its q points), reading each
// input once.
#include "common.h"

namespace {

constexpr int kMaxTau = 64;

// y[k][e] = sum_j W[k][j] x[j][e]; W staged in LDS, kKG frequencies per register group.
constexpr int kKG = 8;
constexpr int kTauUnroll = 8;   // loads in flight before their use
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
      auto fold = [&](int j, double v) __attribute__((always_inline)) {
#pragma unroll
        for (int g = 0; g < kKG; ++g) {
          const int k = k0 + g < nomega ? k0 + g : nomega - 1;
          acc[g] = fma(Ws[k * ntau + j], v, acc[g]);
        }
      };
      int j = 0;
      for (; j + kTauUnroll <= ntau; j += kTauUnroll) {
        double v[kTauUnroll];
#pragma unroll
        for (int u = 0; u < kTauUnroll; ++u) v[u] = x[(size_t)(j + u) * n + e];
#pragma unroll
        for (int u = 0; u < kTauUnroll; ++u) fold(j + u, v[u]);
      }
      for (; j < ntau; ++j) fold(j, x[(size_t)j * n + e]);
#pragma unroll
      for (int g = 0; g < kKG; ++g)
        if (k0 + g < nomega) y[(size_t)(k0 + g) * n + e] = acc[g];
    }
  }
}

// y[b][q][e] = sum_R (cos, sin)[q][R] x[b][R][e], complex interleaved output.  Each element
// e has gp lanes (adjacent in the wave); lane g of e takes q = g, g + gp, g + 2 gp, ..., kQG
// per pass, so the gp lanes read x[R][e] at one address and x is read once.  The phase table
// sits in LDS as [R][q] (cos, sin): lanes g read neighbouring q.
constexpr int kQG = 8;   // q points per register group
constexpr int kUnroll = 8;
__global__ __launch_bounds__(256) void r2q_kernel(const double *__restrict__ ph, int nR, int nq, int gp, size_t m,
                                                  const double *__restrict__ x, double *__restrict__ y) {
  extern __shared__ __align__(16) double phs[];   // [nR][nq][2]
  for (int i = threadIdx.x; i < nq * nR; i += blockDim.x) {
    const int q = i % nq, r = i / nq;
    phs[2 * i] = ph[(q * nR + r) * 2];
    phs[2 * i + 1] = ph[(q * nR + r) * 2 + 1];
  }
  __syncthreads();
  const int b = blockIdx.y;
  const double *xb = x + (size_t)b * nR * m;
  double2 *yb = reinterpret_cast<double2 *>(y + (size_t)b * nq * m * 2);
  const int g = threadIdx.x % gp;          // gp divides the block size
  const size_t epb = blockDim.x / gp;      // elements per block and pass
  // two elements per lane (e and e + half), so every phase read from LDS serves both
  const size_t half = (m + 1) / 2;
  for (size_t e = (size_t)blockIdx.x * epb + threadIdx.x / gp; e < half; e += (size_t)gridDim.x * epb) {
    const size_t e2 = e + half;
    const bool two = e2 < m;
    const size_t e2c = two ? e2 : e;       // a valid address when there is no second element
    for (int q0 = g; q0 < nq; q0 += gp * kQG) {
      double re[2][kQG], im[2][kQG];
#pragma unroll
      for (int j = 0; j < kQG; ++j) re[0][j] = im[0][j] = re[1][j] = im[1][j] = 0.0;
      // kUnroll loads per element in flight before their use (a load per iteration would wait
      // out the memory latency nR times)
      auto fold = [&](int r, double v0, double v1) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < kQG; ++j) {
          const int q = q0 + j * gp < nq ? q0 + j * gp : nq - 1;
          const double2 c = reinterpret_cast<const double2 *>(phs)[r * nq + q];
          re[0][j] = fma(c.x, v0, re[0][j]);
          im[0][j] = fma(c.y, v0, im[0][j]);
          re[1][j] = fma(c.x, v1, re[1][j]);
          im[1][j] = fma(c.y, v1, im[1][j]);
        }
      };
      int r = 0;
      for (; r + kUnroll <= nR; r += kUnroll) {
        double v0[kUnroll], v1[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          v0[u] = xb[(size_t)(r + u) * m + e];
          v1[u] = xb[(size_t)(r + u) * m + e2c];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) fold(r + u, v0[u], v1[u]);
      }
      for (; r < nR; ++r) fold(r, xb[(size_t)r * m + e], xb[(size_t)r * m + e2c]);
#pragma unroll
      for (int j = 0; j < kQG; ++j)
        if (q0 + j * gp < nq) {
          yb[(size_t)(q0 + j * gp) * m + e] = make_double2(re[0][j], im[0][j]);
          if (two) yb[(size_t)(q0 + j * gp) * m + e2] = make_double2(re[1][j], im[1][j]);
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
  // lanes per element: the q groups of kQG, rounded up to a power of two, at most 64
  int gp = 1;
  while (gp < 64 && gp * kQG < nq) gp *= 2;
  const size_t epb = 256 / gp;
  const size_t half = (m + 1) / 2;
  const int blocks = (int)std::min<size_t>((half + epb - 1) / epb, 8192);
  hipLaunchKernelGGL(r2q_kernel, dim3(blocks > 0 ? blocks : 1, nbatch), dim3(256), lds, s, ph_dev, nR, nq, gp, m, x,
                     y);
  return hipGetLastError();
}
