#pragma once
// Few-result-row inner product kernel (shared by k_skinny.hip and
// k_skinny_wide.hip, which instantiate it for one and four runs per thread).
//
// D[i, j] = op1-fold over l of op2(A[i, l], B[l, j]), i < M <= 8
//                                              (Section I, Eq. inner)
//
// Section II.B's workload multiplies an m x 128 matrix (m = 1..4 threads) by
// a 128 x n matrix with n up to the memory size: every element of B is used
// M times, so the product is bound by reading B once from HBM. Each thread
// owns R 16-byte runs of columns j for all M rows; for l = 0, 1, ... it loads
// those runs of row <l> psi B (coalesced, each element of B read exactly once)
// and combines it with the M elements A[i, l] (wave-uniform, read through the
// scalar cache) — row <i> psi D accumulates op2(A[i, l], <l> psi B) under op1,
// as in the paper's Appendix A fragment, with threads over columns instead of
// rows. The fold runs in ascending l from the identity of op1, one IEEE
// operation per step, so results match a sequential fold bit for bit.
#pragma clang fp contract(off)

#include "common.hpp"
#include "internal.hpp"

namespace moa {

// R runs of 16 bytes per thread, 256 * VEC columns apart (each run is one
// coalesced row segment of the wave): R x 16 bytes of B in flight per thread
// and row, which keeps enough bytes in flight per CU with fewer waves.
// MR: rows held per thread (1, 2, 4 or 8; rows M..MR-1 repeat row M - 1 and
// are never stored).
// blockIdx.y selects a group of MR rows (a grid with gridDim.y > 1 splits
// the rows over workgroups: each reads B again, from cache when B is small).
// RING: stream B through a per-thread prefetch ring (used for four or more
// rows per thread on grids of at most four workgroups per CU; see below).
template <typename T, int OP1, int OP2, int MR, int R, bool RING = false>
__global__ __launch_bounds__(256) void k_skinny(const T *__restrict__ A, const T *__restrict__ B, T *__restrict__ D,
                                                int M, int64_t K, int64_t N, bool vec_ok) {
  constexpr int VEC = 16 / sizeof(T);
  const int row0 = (int)blockIdx.y * MR;
  A += (int64_t)row0 * K;
  D += (int64_t)row0 * N;
  M = M - row0 < MR ? M - row0 : MR;
  constexpr int64_t SPAN = 256 * VEC;  // columns between a thread's runs
  const int64_t blk0 = (int64_t)blockIdx.x * SPAN * R;
  const int64_t j0 = blk0 + threadIdx.x * VEC;
  T acc[MR][R][VEC];
#pragma unroll
  for (int i = 0; i < MR; ++i)
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[i][r][v] = fold_identity<OP1, T>();
  auto fold_row = [&](int64_t l, const T (&b)[R][VEC]) {
#pragma unroll
    for (int i = 0; i < MR; ++i) {
      // Rows past M reuse row M - 1 (never stored): an unconditional scalar
      // load the compiler can batch and issue early.
      const T a = A[(int64_t)(i < M ? i : M - 1) * K + l];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[i][r][v] = apply_op<OP1>(acc[i][r][v], apply_op<OP2>(a, b[r][v]));
    }
  };
  using V = T __attribute__((ext_vector_type(VEC)));
  if (RING && vec_ok && blk0 + SPAN * R <= N) {
    // Whole block inside the row: 16-byte non-temporal loads through a ring
    // of PF rows of B per thread. Row l + PF is requested as soon as row l is
    // folded, so PF - 1 rows stay in flight however few waves the grid gives
    // each SIMD (the fold itself must stay sequential in l).
    constexpr int PF = 8;
    V ring[PF][R];
    auto fetch = [&](int64_t l, V(&dst)[R]) {
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r] = __builtin_nontemporal_load((const V *)(B + l * N + j0 + r * SPAN));
    };
    auto fold_v = [&](int64_t l, const V(&src)[R]) {
      T b[R][VEC];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < VEC; ++v) b[r][v] = src[r][v];
      fold_row(l, b);
    };
    int64_t l0 = 0;
    if (K >= 2 * PF) {
      // Branch-free steady state: the ring holds rows l0 .. l0 + PF - 1 and
      // every row fetched inside the loop exists.
#pragma unroll
      for (int p = 0; p < PF; ++p) fetch(p, ring[p]);
      for (; l0 + 2 * PF <= K; l0 += PF) {
#pragma unroll
        for (int p = 0; p < PF; ++p) {
          // Fold, then refill the slot: the new row takes the registers of
          // the row just used (no copy, so no wait for the new load).
          fold_v(l0 + p, ring[p]);
          fetch(l0 + PF + p, ring[p]);
          // Keep each refill where it is (not sunk below later folds).
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (int p = 0; p < PF; ++p) fold_v(l0 + p, ring[p]);
      l0 += PF;
    }
    // Remaining rows (fewer than PF, or all of a short contraction).
#pragma unroll 4
    for (int64_t l = l0; l < K; ++l) {
      V cur[R];
      fetch(l, cur);
      fold_v(l, cur);
    }
  } else if (vec_ok && blk0 + SPAN * R <= N) {
    // Whole block inside the row: 16-byte non-temporal loads, unrolled so
    // that several rows of B are in flight per thread.
#pragma unroll 4
    for (int64_t l = 0; l < K; ++l) {
      T b[R][VEC];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const V bv = __builtin_nontemporal_load((const V *)(B + l * N + j0 + r * SPAN));
#pragma unroll
        for (int v = 0; v < VEC; ++v) b[r][v] = bv[v];
      }
      fold_row(l, b);
    }
  } else {
    for (int64_t l = 0; l < K; ++l) {
      T b[R][VEC];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int64_t j = j0 + r * SPAN + v;
          b[r][v] = j < N ? B[l * N + j] : T(0);
        }
      fold_row(l, b);
    }
  }
#pragma unroll
  for (int i = 0; i < MR; ++i)
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int64_t j = j0 + r * SPAN + v;
        if (i < M && j < N) D[(int64_t)i * N + j] = acc[i][r][v];
      }
}

template <typename T, int OP1, int OP2, int R>
static hipError_t launch_mr(const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, hipStream_t s) {
  constexpr int VEC = 16 / sizeof(T);
  const int64_t blocks = (N + 256 * VEC * R - 1) / (256 * VEC * R);
  if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  const dim3 g((unsigned)blocks), b(256);
  // 16-byte loads of B rows need N % VEC == 0 and a 16-byte aligned B.
  const bool vec_ok = (N % VEC) == 0 && ((uintptr_t)B % 16) == 0;
  const int m = (int)M;
  // Few column blocks, several rows and a B small enough to stay in the
  // last-level cache (256 MB on MI355X; B is then read from HBM about once):
  // one row per workgroup row instead, so the GPU holds M times as many
  // waves and the dependency chain of one thread's fold no longer decides
  // the time (3-4 rows of 128 . 128 x 2^16 FP64: 53 us with four rows per
  // thread). Larger B keeps all rows in one pass, reading B once.
  if (M > 2 && blocks < 1024 && K * N * (int64_t)sizeof(T) <= ((int64_t)64 << 20)) {
    hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 1, R>), dim3((unsigned)blocks, (unsigned)M), b, 0, s, A, B, D, m, K, N,
                       vec_ok);
    return hipGetLastError();
  }
  if (M == 1)
    hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 1, R>), g, b, 0, s, A, B, D, m, K, N, vec_ok);
  else if (M == 2)
    hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 2, R>), g, b, 0, s, A, B, D, m, K, N, vec_ok);
  // Four or more rows per thread on a grid of at most four workgroups per CU
  // (n up to 2^19 FP64 columns with one run per thread, 2^21 with four): the
  // waves are too few to keep HBM busy with a few rows of B in flight each,
  // so each thread streams B through its prefetch ring. 4 x 128 . 128 x n
  // FP64: n = 2^18 0.076 -> 0.047 ms, n = 2^20 0.21 -> 0.17 ms. On larger
  // grids the ring's registers cost occupancy (n = 2^22: 0.68 -> 0.78 ms).
  else if (M <= 4 && blocks <= 1024)
    hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 4, R, true>), g, b, 0, s, A, B, D, m, K, N, vec_ok);
  else if (M <= 4)
    hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 4, R>), g, b, 0, s, A, B, D, m, K, N, vec_ok);
  else if (M <= 8 && blocks <= 1024)
    hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 8, R, true>), g, b, 0, s, A, B, D, m, K, N, vec_ok);
  else if (M <= 8)
    hipLaunchKernelGGL((k_skinny<T, OP1, OP2, 8, R>), g, b, 0, s, A, B, D, m, K, N, vec_ok);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T, int OP1, int R>
static hipError_t dispatch_op2(moa_op op2, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N,
                               hipStream_t s) {
  switch (op2) {
    case MOA_ADD: return launch_mr<T, OP1, MOA_ADD, R>(A, B, D, M, K, N, s);
    case MOA_SUB: return launch_mr<T, OP1, MOA_SUB, R>(A, B, D, M, K, N, s);
    case MOA_MUL: return launch_mr<T, OP1, MOA_MUL, R>(A, B, D, M, K, N, s);
    case MOA_MAX: return launch_mr<T, OP1, MOA_MAX, R>(A, B, D, M, K, N, s);
    case MOA_MIN: return launch_mr<T, OP1, MOA_MIN, R>(A, B, D, M, K, N, s);
    default: break;
  }
  if constexpr (T(1) / 2 == 0) {
    switch (op2) {
      case MOA_AND: return launch_mr<T, OP1, MOA_AND, R>(A, B, D, M, K, N, s);
      case MOA_OR: return launch_mr<T, OP1, MOA_OR, R>(A, B, D, M, K, N, s);
      case MOA_XOR: return launch_mr<T, OP1, MOA_XOR, R>(A, B, D, M, K, N, s);
      default: break;
    }
  } else {
    if (op2 == MOA_DIV) return launch_mr<T, OP1, MOA_DIV, R>(A, B, D, M, K, N, s);
  }
  return hipErrorInvalidValue;
}

// Every op pair for one dtype and run count (external linkage, so that the
// large instance sets can be compiled in separate units).
template <typename T, int R>
hipError_t skinny_dispatch(moa_op op1, moa_op op2, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N,
                           hipStream_t s) {
  switch (op1) {
    case MOA_ADD: return dispatch_op2<T, MOA_ADD, R>(op2, A, B, D, M, K, N, s);
    case MOA_MUL: return dispatch_op2<T, MOA_MUL, R>(op2, A, B, D, M, K, N, s);
    case MOA_MAX: return dispatch_op2<T, MOA_MAX, R>(op2, A, B, D, M, K, N, s);
    case MOA_MIN: return dispatch_op2<T, MOA_MIN, R>(op2, A, B, D, M, K, N, s);
    default: break;
  }
  if constexpr (T(1) / 2 == 0) {
    switch (op1) {
      case MOA_AND: return dispatch_op2<T, MOA_AND, R>(op2, A, B, D, M, K, N, s);
      case MOA_OR: return dispatch_op2<T, MOA_OR, R>(op2, A, B, D, M, K, N, s);
      case MOA_XOR: return dispatch_op2<T, MOA_XOR, R>(op2, A, B, D, M, K, N, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

// Few-row stream with R runs per thread, every dtype and op pair.
template <int R>
hipError_t skinny_launch_r(moa_dtype dt, moa_op op1, moa_op op2, const void *A, const void *B, void *D, int64_t M,
                           int64_t K, int64_t N, hipStream_t s) {
  switch (dt) {
    case MOA_F64:
      return skinny_dispatch<double, R>(op1, op2, (const double *)A, (const double *)B, (double *)D, M, K, N, s);
    case MOA_F32:
      return skinny_dispatch<float, R>(op1, op2, (const float *)A, (const float *)B, (float *)D, M, K, N, s);
    case MOA_I32:
      return skinny_dispatch<int32_t, R>(op1, op2, (const int32_t *)A, (const int32_t *)B, (int32_t *)D, M, K, N, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace moa
