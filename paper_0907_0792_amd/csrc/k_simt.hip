// Generic (op1, op2) inner product on the vector ALUs.
//
// D[i, j] = op1-fold over l = 0..K-1 of op2(A[i, l], B[l, j])   (Section I, Eq. inner)
//
// A is the flattened M x K view of rho A, B the K x N view of rho B, D the
// M x N view of the result (row-major throughout; the rank only changes how
// the same flat vectors are read, as in the MoA code fragment of Appendix A).
// For a contraction over other axes, A is read as (P_a, K, Q_a) and B as
// (P_b, K, Q_b) with row i = p * Q_a + q and column j = p' * Q_b + q':
//     A[i, l] = A[(i / Q_a) * K * Q_a + l * Q_a + i % Q_a],
//     B[l, j] = B[(j / Q_b) * K * Q_b + l * Q_b + j % Q_b],
// which is the last-with-first case for Q_a = 1, Q_b = N.
//
// Layout of the work: the paper builds one row of the result at a time from
// contiguous rows of B, each scaled by an element of A (Section I). Here a
// workgroup owns a BM x BN block of D; each thread keeps a TM x TN register
// block of it and, for every l, combines TM elements of column l of A with
// TN contiguous elements of row l of B (both staged in LDS) — the same row
// form, blocked over rows so every element of A and B fetched from LDS is
// reused TN (resp. TM) times. The fold runs in ascending l from the identity
// of op1, one IEEE operation per step, so FP results equal a sequential fold
// bit for bit. Folds whose result is association-independent (all int32 folds,
// FP max/min) fold two terms at a time: one three-operand max/min/add per
// pair for int32.
#pragma clang fp contract(off)

#include "common.hpp"
#include "internal.hpp"

namespace moa {

template <typename T, int OP1, int OP2, int TM, int TN>
__global__ __launch_bounds__(256) void k_simt_inner(const T *__restrict__ A, const T *__restrict__ B,
                                                    T *__restrict__ D, int64_t M, int64_t K, int64_t N,
                                                    int64_t tiles_m, int64_t tiles_n, int64_t Qa, int64_t Qb) {
  constexpr int BM = 16 * TM, BN = 16 * TN, BK = 16;
  constexpr int PAD = 16 / sizeof(T);
  __shared__ __attribute__((aligned(16))) T As[BK][BM + PAD];
  __shared__ __attribute__((aligned(16))) T Bs[BK][BN];

  int64_t tm, tn;
  const int64_t nt = tiles_m * tiles_n;
  grouped_tile(xcd_swizzle(blockIdx.x, nt), tiles_m, tiles_n, 8, tm, tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;

  T acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = fold_identity<OP1, T>();

  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    // Stage A[m0:m0+BM, k0:k0+BK] transposed into As[k][m], B[k0:k0+BK, n0:n0+BN] into Bs[k][n].
    // The view test is wave-uniform and sits outside the unrolled loops, so
    // the plain layout's staging carries no code of the strided one.
    if (Qa == 1) {
#pragma unroll
      for (int p = 0; p < (BM * BK) / 256; ++p) {
        const int idx = tid + 256 * p;
        const int r = idx / BK, c = idx % BK;  // lanes along k
        const int64_t gm = m0 + r, gk = k0 + c;
        As[c][r] = (gm < M && gk < K) ? A[gm * K + gk] : T(0);
      }
    } else {
#pragma unroll
      for (int p = 0; p < (BM * BK) / 256; ++p) {
        const int idx = tid + 256 * p;
        const int r = idx % BM, c = idx / BM;  // lanes along i, contiguous when Qa > 1
        const int64_t gm = m0 + r, gk = k0 + c;
        As[c][r] = (gm < M && gk < K) ? A[(gm / Qa) * K * Qa + gk * Qa + gm % Qa] : T(0);
      }
    }
    if (Qb == N) {
#pragma unroll
      for (int p = 0; p < (BN * BK) / 256; ++p) {
        const int idx = tid + 256 * p;
        const int r = idx / BN, c = idx % BN;  // lanes along j
        const int64_t gk = k0 + r, gn = n0 + c;
        Bs[r][c] = (gk < K && gn < N) ? B[gk * N + gn] : T(0);
      }
    } else {
#pragma unroll
      for (int p = 0; p < (BN * BK) / 256; ++p) {
        const int idx = tid + 256 * p;
        // Along j, except when B's inner extent Qb is 1 (then along k).
        const int r = Qb == 1 ? idx % BK : idx / BN, c = Qb == 1 ? idx / BK : idx % BN;
        const int64_t gk = k0 + r, gn = n0 + c;
        Bs[r][c] = (gk < K && gn < N) ? B[(gn / Qb) * K * Qb + gk * Qb + gn % Qb] : T(0);
      }
    }
    __syncthreads();
    const int kmax = (K - k0) < BK ? (int)(K - k0) : BK;
    if (kmax == BK && fold_reassociable<OP1, T>()) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        T a0[TM], b0[TN], a1[TM], b1[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          a0[i] = As[kk][ty * TM + i];
          a1[i] = As[kk + 1][ty * TM + i];
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          b0[j] = Bs[kk][tx * TN + j];
          b1[j] = Bs[kk + 1][tx * TN + j];
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = fold_pair<OP1>(acc[i][j], apply_op<OP2>(a0[i], b0[j]), apply_op<OP2>(a1[i], b1[j]));
      }
    } else if (kmax == BK) {
#pragma unroll
      for (int kk = 0; kk < BK; ++kk) {
        T a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[kk][ty * TM + i];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[kk][tx * TN + j];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = apply_op<OP1>(acc[i][j], apply_op<OP2>(a[i], b[j]));
      }
    } else {
      for (int kk = 0; kk < kmax; ++kk) {
        T a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[kk][ty * TM + i];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[kk][tx * TN + j];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = apply_op<OP1>(acc[i][j], apply_op<OP2>(a[i], b[j]));
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int64_t gm = m0 + ty * TM + i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t gn = n0 + tx * TN + j;
      if (gn < N) D[gm * N + gn] = acc[i][j];
    }
  }
}

template <typename T, int OP1, int OP2>
static hipError_t launch_tiles(const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, int tile,
                               int64_t Qa, int64_t Qb, hipStream_t s) {
  int64_t tm, tn;
  if (tile == 8) {
    tm = (M + 127) / 128;
    tn = (N + 127) / 128;
    hipLaunchKernelGGL((k_simt_inner<T, OP1, OP2, 8, 8>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, A, B, D, M, K,
                       N, tm, tn, Qa, Qb);
  } else if (tile == 4) {
    tm = (M + 63) / 64;
    tn = (N + 63) / 64;
    hipLaunchKernelGGL((k_simt_inner<T, OP1, OP2, 4, 4>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, A, B, D, M, K,
                       N, tm, tn, Qa, Qb);
  } else {
    tm = (M + 31) / 32;
    tn = (N + 31) / 32;
    hipLaunchKernelGGL((k_simt_inner<T, OP1, OP2, 2, 2>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, A, B, D, M, K,
                       N, tm, tn, Qa, Qb);
  }
  return hipGetLastError();
}

// Tile choice: the largest register block that still gives every CU a few
// workgroups.
static int pick_tile(int64_t M, int64_t N) {
  const int64_t big = ((M + 127) / 128) * ((N + 127) / 128);
  if (big >= 512) return 8;
  const int64_t mid = ((M + 63) / 64) * ((N + 63) / 64);
  if (mid >= 256) return 4;
  return 2;
}

template <typename T, int OP1>
static hipError_t dispatch_op2(moa_op op2, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, int tile,
                               int64_t Qa, int64_t Qb, hipStream_t s) {
  switch (op2) {
    case MOA_ADD: return launch_tiles<T, OP1, MOA_ADD>(A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_SUB: return launch_tiles<T, OP1, MOA_SUB>(A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_MUL: return launch_tiles<T, OP1, MOA_MUL>(A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_MAX: return launch_tiles<T, OP1, MOA_MAX>(A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_MIN: return launch_tiles<T, OP1, MOA_MIN>(A, B, D, M, K, N, tile, Qa, Qb, s);
    default: break;
  }
  if constexpr (T(1) / 2 == 0) {
    switch (op2) {
      case MOA_AND: return launch_tiles<T, OP1, MOA_AND>(A, B, D, M, K, N, tile, Qa, Qb, s);
      case MOA_OR: return launch_tiles<T, OP1, MOA_OR>(A, B, D, M, K, N, tile, Qa, Qb, s);
      case MOA_XOR: return launch_tiles<T, OP1, MOA_XOR>(A, B, D, M, K, N, tile, Qa, Qb, s);
      default: break;
    }
  } else {
    if (op2 == MOA_DIV) return launch_tiles<T, OP1, MOA_DIV>(A, B, D, M, K, N, tile, Qa, Qb, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t dispatch_op1(moa_op op1, moa_op op2, const T *A, const T *B, T *D, int64_t M, int64_t K,
                               int64_t N, int tile, int64_t Qa, int64_t Qb, hipStream_t s) {
  switch (op1) {
    case MOA_ADD: return dispatch_op2<T, MOA_ADD>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_MUL: return dispatch_op2<T, MOA_MUL>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_MAX: return dispatch_op2<T, MOA_MAX>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_MIN: return dispatch_op2<T, MOA_MIN>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
    default: break;
  }
  if constexpr (T(1) / 2 == 0) {
    switch (op1) {
      case MOA_AND: return dispatch_op2<T, MOA_AND>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
      case MOA_OR: return dispatch_op2<T, MOA_OR>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
      case MOA_XOR: return dispatch_op2<T, MOA_XOR>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_simt_inner(moa_dtype dt, moa_op op1, moa_op op2, const void *A, const void *B, void *D, int64_t M,
                             int64_t K, int64_t N, int tile, hipStream_t s, int64_t Qa, int64_t Qb) {
  if (M == 0 || N == 0) return hipSuccess;
  if (Qb <= 0) Qb = N;
  if (Qa <= 0) Qa = 1;
  if (tile <= 0) tile = pick_tile(M, N);
  switch (dt) {
    case MOA_F64:
      return dispatch_op1<double>(op1, op2, (const double *)A, (const double *)B, (double *)D, M, K, N, tile, Qa, Qb, s);
    case MOA_F32:
      return dispatch_op1<float>(op1, op2, (const float *)A, (const float *)B, (float *)D, M, K, N, tile, Qa, Qb, s);
    case MOA_I32:
      return dispatch_op1<int32_t>(op1, op2, (const int32_t *)A, (const int32_t *)B, (int32_t *)D, M, K, N, tile, Qa, Qb, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace moa
