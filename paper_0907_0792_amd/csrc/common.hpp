// Shared device-side helpers of libmoa (HIP, gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "moa.h"

namespace moa {

typedef __attribute__((__vector_size__(4 * sizeof(double)))) double doublex4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;

constexpr int kWave = 64;
constexpr int kNumXcd = 8;  // MI355X: 8 XCDs, workgroups dealt round-robin

// Workgroups are dispatched to the XCDs round-robin (id % 8). Renumber them so
// that consecutive logical tiles share an XCD and hence its L2: logical id =
// (id % 8) * (n / 8) + id / 8 when n is a multiple of 8.
__device__ __forceinline__ int64_t xcd_swizzle(int64_t id, int64_t n) {
  if (n % kNumXcd != 0) return id;
  return (id % kNumXcd) * (n / kNumXcd) + id / kNumXcd;
}

// Grouped raster order over a tiles_m x tiles_n grid: walk `group` tile rows
// at a time so a window of consecutive tiles reuses the same A rows and B
// columns.
__device__ __forceinline__ void grouped_tile(int64_t t, int64_t tiles_m, int64_t tiles_n, int64_t group, int64_t &tm,
                                             int64_t &tn) {
  const int64_t per_group = group * tiles_n;
  const int64_t g = t / per_group;
  const int64_t first_m = g * group;
  const int64_t rows = (tiles_m - first_m) < group ? (tiles_m - first_m) : group;
  const int64_t r = t % per_group;
  tm = first_m + r % rows;
  tn = r / rows;
}

// ---------------------------------------------------------------------------
// Element operations of the generalized products. int32 max/min are signed.
// FP max/min are the IEEE 754-2019 maximum/minimum: a NaN operand gives NaN
// and -0 orders below +0. That makes them associative and commutative bit for
// bit (NaN payloads aside), so a fold over them has one value in any order.

template <int OP, typename T>
__device__ __forceinline__ T apply_op(T a, T b);

template <int OP, typename T>
struct OpImpl;

template <typename T>
struct OpImpl<MOA_ADD, T> {
  static __device__ __forceinline__ T f(T a, T b) { return a + b; }
};
template <typename T>
struct OpImpl<MOA_SUB, T> {
  static __device__ __forceinline__ T f(T a, T b) { return a - b; }
};
template <typename T>
struct OpImpl<MOA_MUL, T> {
  static __device__ __forceinline__ T f(T a, T b) { return a * b; }
};
template <typename T>
struct OpImpl<MOA_DIV, T> {
  static __device__ __forceinline__ T f(T a, T b) { return a / b; }
};
template <typename T>
struct OpImpl<MOA_MAX, T> {
  static __device__ __forceinline__ T f(T a, T b) {
    if constexpr (T(1) / 2 == 0) return (a < b) ? b : a;
    else return __builtin_elementwise_maximum(a, b);
  }
};
template <typename T>
struct OpImpl<MOA_MIN, T> {
  static __device__ __forceinline__ T f(T a, T b) {
    if constexpr (T(1) / 2 == 0) return (b < a) ? b : a;
    else return __builtin_elementwise_minimum(a, b);
  }
};
template <typename T>
struct OpImpl<MOA_AND, T> {
  static __device__ __forceinline__ T f(T a, T b) { return a & b; }
};
template <typename T>
struct OpImpl<MOA_OR, T> {
  static __device__ __forceinline__ T f(T a, T b) { return a | b; }
};
template <typename T>
struct OpImpl<MOA_XOR, T> {
  static __device__ __forceinline__ T f(T a, T b) { return a ^ b; }
};
// int32 + - * wrap: do them on uint32.
template <>
struct OpImpl<MOA_ADD, int32_t> {
  static __device__ __forceinline__ int32_t f(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }
};
template <>
struct OpImpl<MOA_SUB, int32_t> {
  static __device__ __forceinline__ int32_t f(int32_t a, int32_t b) { return (int32_t)((uint32_t)a - (uint32_t)b); }
};
template <>
struct OpImpl<MOA_MUL, int32_t> {
  static __device__ __forceinline__ int32_t f(int32_t a, int32_t b) { return (int32_t)((uint32_t)a * (uint32_t)b); }
};

template <int OP, typename T>
__device__ __forceinline__ T apply_op(T a, T b) {
  return OpImpl<OP, T>::f(a, b);
}

// Identity of a fold op: the value a fold starts from. Folding every term
// into it gives the left fold from the first term bit for bit, so for FP
// addition it is -0 (-0 + x = x for every x, +0 and -0 included). An empty
// fold gives +0 instead (launch_fill_identity).
template <int OP, typename T>
__device__ __forceinline__ T fold_identity() {
  if constexpr (OP == MOA_ADD && T(1) / 2 != 0) return -T(0);
  if constexpr (OP == MOA_ADD || OP == MOA_OR || OP == MOA_XOR) return T(0);
  if constexpr (OP == MOA_MUL) return T(1);
  if constexpr (OP == MOA_AND) return T(-1);
  if constexpr (OP == MOA_MAX) {
    if constexpr (sizeof(T) == 4 && T(1) / 2 == 0) return T(INT32_MIN);
    else return -__builtin_huge_val();
  }
  if constexpr (OP == MOA_MIN) {
    if constexpr (sizeof(T) == 4 && T(1) / 2 == 0) return T(INT32_MAX);
    else return __builtin_huge_val();
  }
  return T(0);
}

// A fold op whose result does not depend on the association order in type T:
// every int32 fold (wrapping + and * included) and FP max/min (IEEE 754-2019
// maximum/minimum, see above). Such folds may combine two terms before
// folding them in.
template <int OP, typename T>
constexpr bool fold_reassociable() {
  if constexpr (T(1) / 2 == 0) return true;  // integer type
  return OP == MOA_MAX || OP == MOA_MIN;
}

// acc op x op y for a reassociable fold. For int32 max, min and (wrapping)
// add this is one three-operand VALU instruction; written as inline asm
// because the compiler otherwise rebalances an unrolled chain of these into a
// tree (two-operand op per pair of terms, plus a three-operand one per four),
// which costs 1.75 instead of 1.5 instructions per term with the add.
template <int OP, typename T>
__device__ __forceinline__ T fold_pair(T acc, T x, T y) {
  if constexpr (sizeof(T) == 4 && T(1) / 2 == 0) {
    int32_t r;
    if constexpr (OP == MOA_MAX) {
      asm("v_max3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(acc), "v"(x), "v"(y));
      return r;
    } else if constexpr (OP == MOA_MIN) {
      asm("v_min3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(acc), "v"(x), "v"(y));
      return r;
    } else if constexpr (OP == MOA_ADD) {
      asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(acc), "v"(x), "v"(y));
      return r;
    }
  }
  return apply_op<OP>(acc, apply_op<OP>(x, y));
}

}  // namespace moa
