// Device-side helpers: storage-dtype loads/stores and rounding.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fe {

typedef uint16_t bf16_t;  // raw bfloat16 bits

// bfloat16 -> float is exact: the bf16 bits are the top half of the float.
__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// float -> bfloat16, round to nearest, ties to even (IEEE 754 roundTiesToEven
// applied at bit 16): add 0x7FFF plus the lowest kept bit, then truncate.
// NaN keeps its sign and becomes a quiet NaN.
__device__ __forceinline__ uint32_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return ((u >> 16) | 0x40u) & 0xFFFFu;
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// double -> bfloat16 with a single rounding: first to float rounding toward
// zero with the inexact flag folded into the last bit (round-to-odd), which
// keeps enough information for the final round-to-nearest-even to be exact.
__device__ __forceinline__ uint32_t f64_to_bf16(double d) {
  float t = __double2float_rz(d);
  uint32_t u = __float_as_uint(t);
  if ((double)t != d && (u & 0x7FFFFFFFu) < 0x7F800000u) u |= 1u;
  return f32_to_bf16(__uint_as_float(u));
}

template <typename T>
struct Acc;
template <>
struct Acc<double> {
  using type = double;
};
template <>
struct Acc<float> {
  using type = float;
};
template <>
struct Acc<bf16_t> {
  using type = float;
};

// Raw bit containers for 2..16-byte accesses (clang vector types, which the
// non-temporal builtins accept).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
template <int BYTES>
struct Raw;
template <>
struct Raw<16> {
  using type = u32x4;
};
template <>
struct Raw<8> {
  using type = u32x2;
};
template <>
struct Raw<4> {
  using type = uint32_t;
};
template <>
struct Raw<2> {
  using type = uint16_t;
};

// Load VEC consecutive storage elements (aligned to VEC*sizeof(T)) as A values.
template <typename T, int VEC, typename A>
__device__ __forceinline__ void load_vec(const T* p, A* out) {
  using R = typename Raw<VEC * sizeof(T)>::type;
  R r = *reinterpret_cast<const R*>(p);
  T e[VEC];
  __builtin_memcpy(e, &r, sizeof(R));
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    if constexpr (sizeof(T) == 2)
      out[v] = (A)bf16_to_f32(e[v]);
    else
      out[v] = (A)e[v];
  }
}

template <typename T, int VEC, typename A>
__device__ __forceinline__ void load_vec_nt(const T* p, A* out) {
  using R = typename Raw<VEC * sizeof(T)>::type;
  R r = __builtin_nontemporal_load(reinterpret_cast<const R*>(p));
  T e[VEC];
  __builtin_memcpy(e, &r, sizeof(R));
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    if constexpr (sizeof(T) == 2)
      out[v] = (A)bf16_to_f32(e[v]);
    else
      out[v] = (A)e[v];
  }
}

template <typename T, typename A>
__device__ __forceinline__ T to_storage(A x) {
  if constexpr (sizeof(T) == 2) {
    if constexpr (sizeof(A) == 8)
      return (T)f64_to_bf16(x);
    else
      return (T)f32_to_bf16(x);
  } else {
    return (T)x;
  }
}

// Store VEC values rounded to T (aligned to VEC*sizeof(T)).
template <typename T, int VEC, typename A>
__device__ __forceinline__ void store_vec(T* p, const A* in) {
  using R = typename Raw<VEC * sizeof(T)>::type;
  T e[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) e[v] = to_storage<T, A>(in[v]);
  R r;
  __builtin_memcpy(&r, e, sizeof(R));
  *reinterpret_cast<R*>(p) = r;
}

template <typename T, int VEC, typename A>
__device__ __forceinline__ void store_vec_nt(T* p, const A* in) {
  using R = typename Raw<VEC * sizeof(T)>::type;
  T e[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) e[v] = to_storage<T, A>(in[v]);
  R r;
  __builtin_memcpy(&r, e, sizeof(R));
  __builtin_nontemporal_store(r, reinterpret_cast<R*>(p));
}

template <typename T>
__device__ __forceinline__ double load_f64(const T* p) {
  if constexpr (sizeof(T) == 2)
    return (double)bf16_to_f32(*p);
  else
    return (double)*p;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of two
// 32x32->64 multiplies (0xD2511F53, 0xCD9E8D57), Weyl key bumps
// (0x9E3779B9, 0xBB67AE85).
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

}  // namespace fe
