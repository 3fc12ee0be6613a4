// Device helpers shared by the 2D and 3D sweep kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "s5d_internal.h"

// Every lambda of the kernel bodies must be inlined: their arrays are register
// state and only become registers (not scratch memory) once inlined.
#define S5D_INL __attribute__((always_inline))

namespace s5d {

template <int N>
using ic = std::integral_constant<int, N>;

template <typename F, int... Is>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(ic<Is>{}), ...);
}
// Compile-time loop: f(ic<0>{}), ..., f(ic<N-1>{}).
template <int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int pmod(int a, int m) { return ((a % m) + m) % m; }
constexpr int gcd_i(int a, int b) { return b == 0 ? a : gcd_i(b, a % b); }
constexpr int lcm_i(int a, int b) { return a / gcd_i(a, b) * b; }

// DPP whole-wavefront shifts by one lane.  wave_shr:1 (0x138) hands lane l
// the value of lane l-1; wave_shl:1 (0x130) hands lane l the value of lane
// l+1.  bound_ctrl makes the lane without a source read 0, so no old value
// has to be materialised.
__device__ __forceinline__ int lane_from_lower_i32(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ int lane_from_upper_i32(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ float lane_from_lower(float v) {
  return __int_as_float(lane_from_lower_i32(__float_as_int(v)));
}
__device__ __forceinline__ float lane_from_upper(float v) {
  return __int_as_float(lane_from_upper_i32(__float_as_int(v)));
}
__device__ __forceinline__ double lane_from_lower(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_from_lower_i32(static_cast<int>(b));
  const int hi = lane_from_lower_i32(static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double lane_from_upper(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_from_upper_i32(static_cast<int>(b));
  const int hi = lane_from_upper_i32(static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// The same shifts folded into the float32 product of a term (VOP2 DPP):
// fma_dpp<true>(s, x, c) = fma(x of lane l-1, c, s), fma_dpp<false> takes lane
// l+1; mul_dpp likewise returns x * c.  One instruction instead of a DPP move
// plus the FMA, with the same bits (the product is commutative and exact in
// the FMA).  A DPP read of a VGPR must come at least two wait states after the
// VALU write of that VGPR; the compiler cannot see the DPP inside the asm, so
// each carries its own s_nop 1.  c must be a VGPR (VOP2 src1).
template <bool SHR>
__device__ __forceinline__ float fma_dpp(float s, float x, float c) {
  if constexpr (SHR)
    asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "+v"(s) : "v"(x), "v"(c));
  else
    asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "+v"(s) : "v"(x), "v"(c));
  return s;
}
template <bool SHR>
__device__ __forceinline__ float mul_dpp(float x, float c) {
  float p;
  if constexpr (SHR)
    asm("s_nop 1\n\tv_mul_f32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=v"(p) : "v"(x), "v"(c));
  else
    asm("s_nop 1\n\tv_mul_f32_dpp %0, %1, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=v"(p) : "v"(x), "v"(c));
  return p;
}
// A wave-uniform float copied into a VGPR (an SGPR cannot be a VOP2 DPP
// operand).
__device__ __forceinline__ float to_vgpr(float c) {
  float v;
  asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(c));
  return v;
}

// Copy of a wave-uniform struct in global memory, dword by dword through
// readfirstlane, so that the compiler keeps every field in SGPRs: a plain
// struct copy may be lowered to vector loads, after which buffer descriptors
// built from its fields would need a waterfall loop per access.
template <typename S>
__device__ __forceinline__ S uniform_copy(const S& src) {
  static_assert(sizeof(S) % 4 == 0, "dword-sized structs only");
  S out;
  const int* p = reinterpret_cast<const int*>(&src);
  int* q = reinterpret_cast<int*>(&out);
#pragma unroll
  for (int i = 0; i < static_cast<int>(sizeof(S) / 4); ++i) q[i] = __builtin_amdgcn_readfirstlane(p[i]);
  return out;
}

// Correctly rounded square roots (the build keeps HIP's IEEE-exact division
// and square root; no fast-math).
__device__ __forceinline__ float ieee_sqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double ieee_sqrt(double x) { return __builtin_sqrt(x); }

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Cache policy of the kernels' stores (the buffer instructions' aux operand):
// non-temporal (nt), as a round's output is read only by the next launch.
// Measured on MI355X against the default policy: +0.6 % for the headline
// launch, +0.8 % for batched rounds, +3 % for the persistent batch (whose
// per-item L2 write-back has less to write).
constexpr int kStoreAux = 2;

// Buffer descriptors (gfx9 family: 3rd dword 0x00020000, raw byte
// addressing).  An access whose byte offset is >= nbytes reads 0 / is dropped.
constexpr uint32_t kOutOfRange = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), static_cast<short>(0),
                                           static_cast<int>(nbytes), 0x00020000);
}
__device__ __forceinline__ void buf_load(float& v, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
  v = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, static_cast<int>(off), 0, 0));
}
__device__ __forceinline__ void buf_load(double& v, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
  v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, static_cast<int>(off), 0, 0));
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, static_cast<int>(off), 0, kStoreAux);
}
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
  using u2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs, static_cast<int>(off), 0, kStoreAux);
}
// A lane's CPL consecutive cells as the widest stores that tile them (16, 8
// or 4 bytes); an out-of-range offset drops the whole vector.
template <typename T, int CPL>
__device__ __forceinline__ void buf_store_lane(const T (&v)[CPL], __amdgpu_buffer_rsrc_t rs, uint32_t off) {
  constexpr int BYTES = CPL * sizeof(T);
  constexpr int PIECE = BYTES % 16 == 0 ? 16 : (BYTES % 8 == 0 ? 8 : 4);
  constexpr int PER = PIECE / sizeof(T) > 0 ? PIECE / sizeof(T) : 1;
#pragma unroll
  for (int q = 0; q < CPL / PER; ++q) {
    T piece[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) piece[j] = v[q * PER + j];
    const uint32_t o = off == kOutOfRange ? kOutOfRange : off + q * static_cast<uint32_t>(PIECE);
    if constexpr (PIECE == 16) {
      using u4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(rs, 0, 0, 0));
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, piece), rs, static_cast<int>(o), 0, kStoreAux);
    } else if constexpr (PIECE == 8) {
      using u2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0, 0, 0));
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, piece), rs, static_cast<int>(o), 0, kStoreAux);
    } else {
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, piece), rs, static_cast<int>(o), 0, kStoreAux);
    }
  }
}

// Accumulation of a cell's stencil terms, one accumulator per pending output.
//  ACC = 0: one fused multiply-add per term in the working precision.
//  ACC = 1 (float only): compensated dot product (Ogita, Rump and Oishi,
//  2005): each product is split exactly into its rounded value h and error e
//  by an FMA, h enters the running sum s through Knuth's error-free two-sum,
//  and the errors gather in a second accumulator q; the value is s + q, rounded
//  once.  Contraction must stay off here: fusing c*x into the following add
//  would destroy the error-free transformations.
template <typename T, int ACC>
struct Accum;

template <typename T>
struct Accum<T, 0> {
  T s;
  __device__ __forceinline__ void zero() { s = T(0); }
  __device__ __forceinline__ void first(T c, T x) { s = c * x; }
  __device__ __forceinline__ void add(T c, T x) { s = fmadd(c, x, s); }
  __device__ __forceinline__ T value() const { return s; }
};

template <>
struct Accum<float, 1> {
  float s, q;
  __device__ __forceinline__ void zero() { s = q = 0.0f; }
  __device__ __forceinline__ void first(float c, float x) {
#pragma clang fp contract(off)
    const float h = c * x;
    q = __builtin_fmaf(c, x, -h);
    s = h;
  }
  __device__ __forceinline__ void add(float c, float x) {
#pragma clang fp contract(off)
    const float h = c * x;
    const float e = __builtin_fmaf(c, x, -h);
    const float t1 = s + h;
    const float z = t1 - s;
    const float t = (s - (t1 - z)) + (h - z);
    s = t1;
    q = q + (e + t);
  }
  __device__ __forceinline__ float value() const {
#pragma clang fp contract(off)
    return s + q;
  }
};

// The value a finished output cell takes: its sum, or (EXPR_DIV) its sum
// divided by the last coefficient c0 -- one correctly rounded division.
template <int EXPR, typename T, typename Pack>
__device__ __forceinline__ T finish(T sum, const Pack& cf) {
  if constexpr (EXPR == EXPR_DIV) {
    constexpr int n = sizeof(cf.c) / sizeof(cf.c[0]);
    return sum / cf.c[n - 1];
  } else {
    return sum;
  }
}

// A lane's CPL consecutive cells, element-aligned, read as one vector access.
template <typename T, int N>
struct __attribute__((packed, aligned(sizeof(T)))) LaneVec {
  T v[N];
};

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
// that consecutive logical blocks (neighbouring tiles, which share BT*R
// overlap columns) run on the same XCD and share its L2.
__device__ __forceinline__ int xcd_logical_block(int b, int nblk) {
  const int q = nblk >> 3, rem = nblk & 7, x = b & 7, i = b >> 3;
  return x < rem ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
}

}  // namespace s5d
