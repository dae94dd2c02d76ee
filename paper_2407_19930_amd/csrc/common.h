// Shared device helpers for the gfx950 kernels: MFMA wrappers and launch checks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA, wave64.  Operand layout (both precisions):
//   A[i][kk]: lane l holds A[l % 16][l / 16]
//   B[kk][j]: lane l holds B[l / 16][l % 16]
//   D[i][j] : register r of lane l holds D[row(l / 16, r)][l % 16] with
//             row = 4 * (l / 16) + r for f32 and row = l / 16 + 4 * r for f64
//             (measured on gfx950 with an in-bounds probe of both builtins).
template <typename T> struct Mfma;

template <> struct Mfma<double> {
  typedef d4 acc;
  static __device__ __forceinline__ acc fma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ int row(int grp, int r) { return grp + 4 * r; }
};

template <> struct Mfma<float> {
  typedef f4 acc;
  static __device__ __forceinline__ acc fma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ int row(int grp, int r) { return 4 * grp + r; }
};

// Component-wise BvK arithmetic on flattened lattice-vector indices.
struct Bvk {
  int n0, n1, n2;
  __host__ __device__ __forceinline__ void split(int r, int &a, int &b, int &c) const {
    c = r % n2;
    b = (r / n2) % n1;
    a = r / (n1 * n2);
  }
  __host__ __device__ __forceinline__ int join(int a, int b, int c) const { return (a * n1 + b) * n2 + c; }
  // (ra - rb) mod mesh
  __host__ __device__ __forceinline__ int sub(int ra, int rb) const {
    int a0, a1, a2, b0, b1, b2;
    split(ra, a0, a1, a2);
    split(rb, b0, b1, b2);
    int c0 = a0 - b0, c1 = a1 - b1, c2 = a2 - b2;
    c0 += (c0 < 0) ? n0 : 0;
    c1 += (c1 < 0) ? n1 : 0;
    c2 += (c2 < 0) ? n2 : 0;
    return join(c0, c1, c2);
  }
  __host__ __device__ __forceinline__ int neg(int r) const { return sub(0, r); }
};

// wave-uniform copies of values every lane holds alike (loop state from LDS tables)
static __device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
static __device__ __forceinline__ long long uniform(long long x) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((int)(x & 0xffffffffll));
  const unsigned hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
// raw buffer view of [p, p + nbytes): loads at byte offsets >= nbytes return zero without a
// memory access, so the masked loads of the slice loop need no branches
static __device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_view(const void *p, unsigned nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)nbytes, 0x00020000);
}
template <typename T> __device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, unsigned off);
template <> __device__ __forceinline__ float buffer_load<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ __forceinline__ double buffer_load<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
