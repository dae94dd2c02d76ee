// Launchers of the correlation-energy stage (FP64: complex, and real where the q point allows it).
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
  const int *skip;          // null, or per outer index: non-zero where the matrix is left alone
                            // (those matrices run through the real-layout kernels instead)
};

// The same batched product for real matrices stored as plain row-major n x n doubles (op 1:
// transpose); leading dimensions and strides in doubles.  Only the matrices whose outer index
// has sel[g / binner] != 0 are computed (all of them when sel is null).
struct DgemmArgs {
  int M, N, K;
  const double *A;
  long long lda, strideA, outerA, innerA;
  int opA;
  const double *B;
  long long ldb, strideB, outerB, innerB;
  int opB;
  double *C;
  long long ldc, strideC;
  int boff, binner;
  double alpha, beta;
  int lower_only, kmode;    // as in ZgemmArgs
  const int *sel;
};

hipError_t launch_zgemm(const ZgemmArgs &g, int batch, hipStream_t s);
hipError_t launch_dgemm(const DgemmArgs &g, int batch, hipStream_t s);
// Matrix m of a batch (spaced `stride` doubles apart) is complex interleaved, or, where
// real[m] != 0 (real may be null: none), real: its first n^2 doubles hold it row-major.
// kinds: bit 0 set if the batch may hold complex matrices, bit 1 if it may hold real ones (the
// launches of an absent kind are left out)
hipError_t launch_cholesky(double *A, size_t stride, int n, int batch, double *Wscratch, int *flags, int flag_base,
                           const int *real, hipStream_t s, int kinds = 3);
hipError_t launch_zero_upper(double *A, size_t stride, int n, int batch, const int *real, hipStream_t s);
hipError_t launch_trace_identity_minus(double *B, size_t stride, int n, int batch, double *trB, const int *real,
                                       hipStream_t s);
hipError_t launch_logdet(const double *A, size_t stride, int n, int batch, const double *trB, double *f, int *flags,
                         int flag_base, const int *real, hipStream_t s);
// dst[m * dstride + e] = real part of complex element e of matrix m, for the nmat matrices of a
// batch addressed like a ZgemmArgs operand (src + (g / binner) outer + (g % binner) inner,
// g = boff + m), n2 elements each, only where sel[g / binner] != 0
hipError_t launch_pack_real(const double *src, long long outer, long long inner, int boff, int binner, int nmat,
                            double *dst, size_t dstride, size_t n2, const int *sel, hipStream_t s);
// both[q] = realchi[q] && realv[q]; pair[q nomega + k] = both[q]; counts[0] = number of q with
// both real, counts[1] = the others
hipError_t launch_both_real(const int *realchi, const int *realv, int nq, int nomega, int *both, int *pair,
                            int *counts, hipStream_t s);
hipError_t launch_fill_int(int *p, size_t n, int v, hipStream_t s);
// real[q] = 1 if every imaginary part of the nomega matrices X[omega][q] (complex n x n) is zero,
// else 0 (real must hold nq ints; it is cleared by the launcher's own kernel first)
hipError_t launch_real_flags(const double *X, int n, int nq, int nomega, int *real, hipStream_t s);
// out[0] = first nonzero of flags[0, n) in index order (0 if none), out[1] = its index (-1 if none)
hipError_t launch_first_flag(const int *flags, int n, int *out, hipStream_t s);
hipError_t launch_copy_words(void *dst, const void *src, size_t nwords, hipStream_t s);
hipError_t launch_quadrature(const double *f, const double *w, int nq, int nomega, double *ecq, hipStream_t s);

constexpr int kCholBlock = 32;
