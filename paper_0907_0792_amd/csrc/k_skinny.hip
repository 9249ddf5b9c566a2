// Inner product with few result rows (M <= 8): the paper's row form as an
// HBM stream.
//
// D[i, j] = op1-fold over l of op2(A[i, l], B[l, j]), i < M <= 8
//                                              (Section I, Eq. inner)
//
// Section II.B's workload multiplies an m x 128 matrix (m = 1..4 threads) by
// a 128 x n matrix with n up to the memory size: every element of B is used
// M times, so the product is bound by reading B once from HBM. Each thread
// owns a 16-byte run of columns j for all M rows; for l = 0, 1, ... it loads
// the run of row <l> psi B (coalesced, each element of B read exactly once)
// and combines it with the M elements A[i, l] (wave-uniform, read through the
// scalar cache) — row <i> psi D accumulates op2(A[i, l], <l> psi B) under op1,
// as in the paper's Appendix A fragment, with threads over columns instead of
// rows. The fold runs in ascending l from the identity of op1, one IEEE
// operation per step, so results match a sequential fold bit for bit.
#pragma clang fp contract(off)

#include "common.hpp"
#include "internal.hpp"

namespace moa {

template <typename T, int OP1, int OP2, int MR>
__global__ __launch_bounds__(256) void k_skinny(const T *__restrict__ A, const T *__restrict__ B, T *__restrict__ D,
                                                int64_t K, int64_t N, bool vec_ok) {
  constexpr int VEC = 16 / sizeof(T);
  const int64_t j0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * VEC;
  if (j0 >= N) return;
  const bool full = j0 + VEC <= N;
  T acc[MR][VEC];
#pragma unroll
  for (int i = 0; i < MR; ++i)
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[i][v] = fold_identity<OP1, T>();
  using V = T __attribute__((ext_vector_type(VEC)));
  // Unrolled so several rows of B are in flight per thread.
#pragma unroll 4
  for (int64_t l = 0; l < K; ++l) {
    T b[VEC];
    if (full && vec_ok) {
      const V bv = __builtin_nontemporal_load((const V *)(B + l * N + j0));
#pragma unroll
      for (int v = 0; v < VEC; ++v) b[v] = bv[v];
    } else {
#pragma unroll
      for (int v = 0; v < VEC; ++v) b[v] = (j0 + v < N) ? B[l * N + j0 + v] : T(0);
    }
#pragma unroll
    for (int i = 0; i < MR; ++i) {
      const T a = A[(int64_t)i * K + l];
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[i][v] = apply_op<OP1>(acc[i][v], apply_op<OP2>(a, b[v]));
    }
  }
#pragma unroll
  for (int i = 0; i < MR; ++i)
#pragma unroll
    for (int v = 0; v < VEC; ++v)
      if (j0 + v < N) D[(int64_t)i * N + j0 + v] = acc[i][v];
}

template <typename T, int OP1, int OP2>
static hipError_t launch_m(const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, hipStream_t s) {
  constexpr int VEC = 16 / sizeof(T);
  const int64_t blocks = (N + 256 * VEC - 1) / (256 * VEC);
  if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  const dim3 g((unsigned)blocks), b(256);
  // 16-byte loads of B rows need N % VEC == 0 and a 16-byte aligned B.
  const bool vec_ok = (N % VEC) == 0 && ((uintptr_t)B % 16) == 0;
  switch (M) {
    case 1: hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 1>), g, b, 0, s, A, B, D, K, N, vec_ok); break;
    case 2: hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 2>), g, b, 0, s, A, B, D, K, N, vec_ok); break;
    case 3: hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 3>), g, b, 0, s, A, B, D, K, N, vec_ok); break;
    case 4: hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 4>), g, b, 0, s, A, B, D, K, N, vec_ok); break;
    case 5: hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 5>), g, b, 0, s, A, B, D, K, N, vec_ok); break;
    case 6: hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 6>), g, b, 0, s, A, B, D, K, N, vec_ok); break;
    case 7: hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 7>), g, b, 0, s, A, B, D, K, N, vec_ok); break;
    case 8: hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 8>), g, b, 0, s, A, B, D, K, N, vec_ok); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int OP1>
static hipError_t dispatch_op2(moa_op op2, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N,
                               hipStream_t s) {
  switch (op2) {
    case MOA_ADD: return launch_m<T, OP1, MOA_ADD>(A, B, D, M, K, N, s);
    case MOA_SUB: return launch_m<T, OP1, MOA_SUB>(A, B, D, M, K, N, s);
    case MOA_MUL: return launch_m<T, OP1, MOA_MUL>(A, B, D, M, K, N, s);
    case MOA_MAX: return launch_m<T, OP1, MOA_MAX>(A, B, D, M, K, N, s);
    case MOA_MIN: return launch_m<T, OP1, MOA_MIN>(A, B, D, M, K, N, s);
    default: break;
  }
  if constexpr (T(1) / 2 == 0) {
    switch (op2) {
      case MOA_AND: return launch_m<T, OP1, MOA_AND>(A, B, D, M, K, N, s);
      case MOA_OR: return launch_m<T, OP1, MOA_OR>(A, B, D, M, K, N, s);
      case MOA_XOR: return launch_m<T, OP1, MOA_XOR>(A, B, D, M, K, N, s);
      default: break;
    }
  } else {
    if (op2 == MOA_DIV) return launch_m<T, OP1, MOA_DIV>(A, B, D, M, K, N, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t dispatch_op1(moa_op op1, moa_op op2, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N,
                               hipStream_t s) {
  switch (op1) {
    case MOA_ADD: return dispatch_op2<T, MOA_ADD>(op2, A, B, D, M, K, N, s);
    case MOA_MUL: return dispatch_op2<T, MOA_MUL>(op2, A, B, D, M, K, N, s);
    case MOA_MAX: return dispatch_op2<T, MOA_MAX>(op2, A, B, D, M, K, N, s);
    case MOA_MIN: return dispatch_op2<T, MOA_MIN>(op2, A, B, D, M, K, N, s);
    default: break;
  }
  if constexpr (T(1) / 2 == 0) {
    switch (op1) {
      case MOA_AND: return dispatch_op2<T, MOA_AND>(op2, A, B, D, M, K, N, s);
      case MOA_OR: return dispatch_op2<T, MOA_OR>(op2, A, B, D, M, K, N, s);
      case MOA_XOR: return dispatch_op2<T, MOA_XOR>(op2, A, B, D, M, K, N, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_skinny_inner(moa_dtype dt, moa_op op1, moa_op op2, const void *A, const void *B, void *D, int64_t M,
                               int64_t K, int64_t N, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  if (M > kSkinnyMaxRows) return hipErrorInvalidValue;
  switch (dt) {
    case MOA_F64:
      return dispatch_op1<double>(op1, op2, (const double *)A, (const double *)B, (double *)D, M, K, N, s);
    case MOA_F32: return dispatch_op1<float>(op1, op2, (const float *)A, (const float *)B, (float *)D, M, K, N, s);
    case MOA_I32:
      return dispatch_op1<int32_t>(op1, op2, (const int32_t *)A, (const int32_t *)B, (int32_t *)D, M, K, N, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace moa
