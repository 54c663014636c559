// Plane-wise buffer addressing shared by the z-marching kernels (device code only).
//
// A kernel that marches up z reads one plane of an array per load.  The plane is a
// buffer resource (a 128-bit descriptor in scalar registers, the same for the whole
// workgroup) and each thread keeps 32-bit byte offsets in the plane, computed once
// (N <= 1024: a plane is at most 8 MiB).  A plane outside the grid gets a record count
// of 0, so every load from it returns 0 without a branch.
#pragma once

#include <hip/hip_runtime.h>

namespace mg {
namespace buf {

template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
};
template <>
struct Vec2<float> {
  using type = float2;
};

using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kBufferWord3 = 0x00020000;   // raw 32-bit-dword buffer, range-checked (gfx9)

template <typename T>
__device__ __forceinline__ Rsrc plane_rsrc(const T* a, int kk, int q) {
  const int k = __builtin_amdgcn_readfirstlane(kk);   // uniform: keeps the descriptor scalar
  const bool in = k >= 0 && k < (1 << q);
  const T* base = a + (static_cast<long long>(in ? k : 0) << (2 * q));
  const int bytes = in ? static_cast<int>(sizeof(T)) << (2 * q) : 0;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), static_cast<short>(0), bytes, kBufferWord3);
}

// byte offset of cell (i, j) in a plane, x and y periodic
template <typename T>
__device__ __forceinline__ unsigned off_of(int i, int j, int q) {
  const int m = (1 << q) - 1;
  return static_cast<unsigned>(((j & m) << q) | (i & m)) * static_cast<unsigned>(sizeof(T));
}

__device__ __forceinline__ double ld1(Rsrc r, unsigned off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float ld1(Rsrc r, unsigned off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double2 ld2(Rsrc r, unsigned off, double) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  double2 d;
  __builtin_memcpy(&d, &v, sizeof d);
  return d;
}
__device__ __forceinline__ float2 ld2(Rsrc r, unsigned off, float) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  float2 d;
  __builtin_memcpy(&d, &v, sizeof d);
  return d;
}

}  // namespace buf
}  // namespace mg
