// Launchers of the correlation-energy stage (complex FP64).
#pragma once

#include "common.h"

// C[l] = alpha op(A[g]) op(B[g]) + beta C[l] for local batch index l = blockIdx.z and global
// index g = boff + l; complex interleaved, row-major.  Each operand X sits at
//   X + (g / binner) * outerX + (g % binner) * innerX + l * strideX   (doubles),
// which covers plain strided batches (outer = inner = 0) and the (q, omega) pairs of the
// energy stage (q = g / nomega, omega = g % nomega).  Leading dimensions in complex elements.
struct ZgemmArgs {
  int M, N, K;
  const double *A;
  long long lda, strideA, outerA, innerA;
  int opA;                  // 0: A, 1: A^H
  const double *B;
  long long ldb, strideB, outerB, innerB;
  int opB;                  // 0: B, 1: B^H
  double *C;
  long long ldc, strideC;
  int boff, binner;
  double alpha, beta;
  int lower_only;           // skip output tiles strictly above the diagonal
  int kmode;                // 0: all k; 1: k >= first column of the tile (op(B) lower
                            // triangular); 2: k >= first row of the tile (op(A) upper triangular)
  const int *realA;         // null, or per outer index g / binner: 1 if that A is real (its imaginary
                            // parts all zero), and the GEMM then takes the two real products only
};

hipError_t launch_zgemm(const ZgemmArgs &g, int batch, hipStream_t s);
hipError_t launch_cholesky(double *A, size_t stride, int n, int batch, double *Wscratch, int *flags, int flag_base,
                           hipStream_t s);
hipError_t launch_zero_upper(double *A, size_t stride, int n, int batch, hipStream_t s);
hipError_t launch_trace_identity_minus(double *B, size_t stride, int n, int batch, double *trB, hipStream_t s);
hipError_t launch_logdet(const double *A, size_t stride, int n, int batch, const double *trB, double *f, int *flags,
                         int flag_base, hipStream_t s);
hipError_t launch_fill_int(int *p, size_t n, int v, hipStream_t s);
// real[q] = 1 if every imaginary part of the nomega matrices X[omega][q] (complex n x n) is zero,
// else 0 (real must hold nq ints; it is cleared by the launcher's own kernel first)
hipError_t launch_real_flags(const double *X, int n, int nq, int nomega, int *real, hipStream_t s);
// out[0] = first nonzero of flags[0, n) in index order (0 if none), out[1] = its index (-1 if none)
hipError_t launch_first_flag(const int *flags, int n, int *out, hipStream_t s);
hipError_t launch_copy_words(void *dst, const void *src, size_t nwords, hipStream_t s);
hipError_t launch_quadrature(const double *f, const double *w, int nq, int nomega, double *ecq, hipStream_t s);

constexpr int kCholBlock = 32;
