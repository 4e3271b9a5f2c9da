// Device helpers shared by the gfx950 kernels (wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include <hip/hip_ext.h>

#include "index_maps.h"
#include "kernels.h"

// Kernel launch that carries the profiled stage's timing events, if any.
#define TLT_LAUNCH(KERNEL, GRID, BLOCK, LDS, STREAM, ...)                                  \
  do {                                                                                      \
    ::tlt::StageEvents &ev_ = ::tlt::stage_events();                                        \
    if (ev_.stop) {                                                                         \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, STREAM, ev_.start, ev_.stop, 0,       \
                            __VA_ARGS__);                                                   \
      ev_.start = nullptr;                                                                  \
      ev_.launches += 1;                                                                    \
    } else {                                                                                \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, STREAM, __VA_ARGS__);                    \
    }                                                                                       \
  } while (0)

namespace tlt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Storage loads: every storage type widens exactly to the compute type.
template <typename VT, typename CT> __device__ __forceinline__ CT ld(const VT *p, int64_t i);
template <> __device__ __forceinline__ double ld<double, double>(const double *p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ float ld<float, float>(const float *p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ float ld<bf16s, float>(const bf16s *p, int64_t i) {
  return __uint_as_float(((uint32_t)p[i].u) << 16);
}
template <> __device__ __forceinline__ float ld<f16s, float>(const f16s *p, int64_t i) {
  return (float)__builtin_bit_cast(_Float16, p[i].u);
}

// Streaming (non-temporal) loads of the transport: read once per render,
// kept out of the way of the gathered irradiance rows in L2.
template <typename VT, typename CT> __device__ __forceinline__ CT ld_nt(const VT *p, int64_t i);
template <> __device__ __forceinline__ double ld_nt<double, double>(const double *p, int64_t i) {
  return __builtin_nontemporal_load(p + i);
}
template <> __device__ __forceinline__ float ld_nt<float, float>(const float *p, int64_t i) {
  return __builtin_nontemporal_load(p + i);
}
template <> __device__ __forceinline__ float ld_nt<bf16s, float>(const bf16s *p, int64_t i) {
  const uint16_t u = __builtin_nontemporal_load(&p[i].u);
  return __uint_as_float(((uint32_t)u) << 16);
}
template <> __device__ __forceinline__ float ld_nt<f16s, float>(const f16s *p, int64_t i) {
  const uint16_t u = __builtin_nontemporal_load(&p[i].u);
  return (float)__builtin_bit_cast(_Float16, u);
}

// float32 -> bfloat16, rounded to nearest even.
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Contiguous row load of CPL compute-type values (16-byte vector loads).
template <typename CT, int CPL> struct RowLoad;
template <int CPL> struct RowLoad<float, CPL> {
  static __device__ __forceinline__ void load(const float *p, float (&v)[CPL]) {
    static_assert(CPL % 4 == 0, "float rows load as float4");
#pragma unroll
    for (int q = 0; q < CPL / 4; ++q) {
      const float4 t = reinterpret_cast<const float4 *>(p)[q];
      v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
    }
  }
};
template <int CPL> struct RowLoad<double, CPL> {
  static __device__ __forceinline__ void load(const double *p, double (&v)[CPL]) {
    static_assert(CPL % 2 == 0, "double rows load as double2");
#pragma unroll
    for (int q = 0; q < CPL / 2; ++q) {
      const double2 t = reinterpret_cast<const double2 *>(p)[q];
      v[2 * q] = t.x; v[2 * q + 1] = t.y;
    }
  }
};

// 16x16x4 matrix instruction in the compute type, and the row of result
// element v held by lane group lk (lanes 16*lk .. 16*lk+15; the column is
// lane % 16).  The f64 form lays its result out differently (measured on
// gfx950 with known operands).
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename CT> struct MfmaOut;
template <> struct MfmaOut<float> {
  typedef f32x4 V4;
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};
template <> struct MfmaOut<double> {
  typedef f64x4 V4;
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};

// Hardware workgroup b runs on XCD b % 8: remap so that each XCD gets a
// contiguous range of logical blocks (neighbouring vertices share L2 lines).
__device__ __forceinline__ int xcd_remap(int b, int n_logical) {
  const int per = (n_logical + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

}  // namespace tlt
