// Device helpers shared by the kernel translation units of libh2sp
// (gfx950): vector types, raw buffer loads, the 16 x 16 MFMA wrappers,
// the XCD-aware tile order and the kernel entries of generated operands.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace h2 {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// Raw buffer loads, declared as the LLVM intrinsics they are (the clang
// builtin of the 128-bit form returns a single dword with this compiler).
__device__ f4 raw_buffer_load_f4(__amdgpu_buffer_rsrc_t rsrc, int voffset, int soffset, int aux) __asm(
    "llvm.amdgcn.raw.ptr.buffer.load.v4f32");
__device__ d2 raw_buffer_load_d2(__amdgpu_buffer_rsrc_t rsrc, int voffset, int soffset, int aux) __asm(
    "llvm.amdgcn.raw.ptr.buffer.load.v2f64");

__device__ float raw_buffer_load_f1(__amdgpu_buffer_rsrc_t rsrc, int voffset, int soffset, int aux) __asm(
    "llvm.amdgcn.raw.ptr.buffer.load.f32");
__device__ double raw_buffer_load_d1(__amdgpu_buffer_rsrc_t rsrc, int voffset, int soffset, int aux) __asm(
    "llvm.amdgcn.raw.ptr.buffer.load.f64");

namespace {

template <class T> struct Mfma;
// Output layout of the 16x16x4 instructions (lane l, accumulator element v):
// f64 holds D[l/16 + 4v][l%16], f32 holds D[4(l/16) + v][l%16] (measured on
// gfx950).  `row` returns that D row.
template <> struct Mfma<double> {
  using V = d4;
  static __device__ __forceinline__ V run(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return lane / 16 + 4 * v; }
};
template <> struct Mfma<float> {
  using V = f4;
  static __device__ __forceinline__ V run(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane / 16) + v; }
};

// Work-groups are handed to the 8 XCDs round-robin by block index, and each
// XCD has its own L2.  Tile lists put tiles that share operands next to each
// other; this mapping gives XCD x the x-th contiguous eighth of the list, so
// neighbouring tiles meet in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int x = b % 8, q = b / 8, base = n / 8, rem = n % 8;
  return x * base + min(x, rem) + q;
}

// 1 / sqrt(x) in FP64: the hardware reciprocal square root (relative error
// about 5e-8) refined by two Newton steps y <- y + y (1 - x y^2) / 2, which
// bring it below one unit in the last place (measured 1.4e-16 over
// x in [1e-12, 1e2]).
__device__ __forceinline__ double inv_sqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(y, 0.5 * fma(-(x * y), y, 1.0), y);
  y = fma(y, 0.5 * fma(-(x * y), y, 1.0), y);
  return y;
}

// Off-diagonal kernel value at squared distance d2: scale / r (KERN 0),
// scale exp(-r^2) (KERN 1), scale r / d below d and scale d / r from d on
// (KERN 2, Example 5.4 of Section 5.5, d = param).  Generated GEMM operands and
// kernel_blocks_kernel both form their values here.
template <int KERN>
__device__ __forceinline__ double kernel_value(double d2, double scale, double param) {
  if constexpr (KERN == 0) {
    return scale * inv_sqrt(d2);
  } else if constexpr (KERN == 1) {
    return scale * exp(-d2);
  } else {
    const double r = sqrt(d2);
    return r < param ? scale * (r / param) : scale * (param / r);
  }
}

// Buffer resources: reads outside [base, base + size) return zero and move no
// memory.
constexpr int kRsrcFlags = 0x00020000;  // raw 32-bit buffer, no swizzle (gfx9 family)

// The base and the size are wave-uniform; readfirstlane keeps them in SGPRs
// (a resource in VGPRs would make the compiler loop over the lanes).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(a))));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(a >> 32))));
  const int n = __builtin_amdgcn_readfirstlane(int(bytes));
  void* q = reinterpret_cast<void*>((uint64_t(hi) << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(q, 0, n, kRsrcFlags);
}

template <class T> struct BufLoad4;
template <> struct BufLoad4<float> {
  static __device__ __forceinline__ void run(__amdgpu_buffer_rsrc_t rs, uint32_t off, float (&v)[4]) {
    const f4 x = raw_buffer_load_f4(rs, int(off), 0, 0);
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = x[s];
  }
};
template <> struct BufLoad4<double> {
  static __device__ __forceinline__ void run(__amdgpu_buffer_rsrc_t rs, uint32_t off, double (&v)[4]) {
    const d2 x = raw_buffer_load_d2(rs, int(off), 0, 0);
    const d2 y = raw_buffer_load_d2(rs, int(off + 16), 0, 0);
    v[0] = x[0];
    v[1] = x[1];
    v[2] = y[0];
    v[3] = y[1];
  }
};

constexpr uint32_t kOutside = 0x80000000u;  // a buffer offset past every resource used here

template <class T> struct BufLoad1;
template <> struct BufLoad1<float> {
  static __device__ __forceinline__ float run(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return raw_buffer_load_f1(rs, int(off), 0, 0);
  }
};
template <> struct BufLoad1<double> {
  static __device__ __forceinline__ double run(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return raw_buffer_load_d1(rs, int(off), 0, 0);
  }
};
}  // namespace
}  // namespace h2
