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
// pair for int32. The next k panel is loaded into registers while the
// current one is folded, as 16-byte vectors when the layout is plain and the
// rows are aligned (VEC).
#include "common.hpp"
#include "internal.hpp"

namespace moa {

// Instantiated in k_simt_f64.hip, k_simt_f32.hip, k_simt_i32.hip and
// k_simt_i32_bits.hip.
template <typename T, int OP1>
hipError_t simt_fold(moa_op op2, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, int tile,
                     int64_t Qa, int64_t Qb, hipStream_t s);

// Tile choice: the largest register block that still gives every CU a few
// workgroups.
static int pick_tile(int64_t M, int64_t N) {
  const int64_t big = ((M + 127) / 128) * ((N + 127) / 128);
  if (big >= 512) return 8;
  const int64_t mid = ((M + 63) / 64) * ((N + 63) / 64);
  if (mid >= 256) return 4;
  return 2;
}

template <typename T>
static hipError_t dispatch_op1(moa_op op1, moa_op op2, const T *A, const T *B, T *D, int64_t M, int64_t K,
                               int64_t N, int tile, int64_t Qa, int64_t Qb, hipStream_t s) {
  switch (op1) {
    case MOA_ADD: return simt_fold<T, MOA_ADD>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_MUL: return simt_fold<T, MOA_MUL>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_MAX: return simt_fold<T, MOA_MAX>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_MIN: return simt_fold<T, MOA_MIN>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
    default: break;
  }
  if constexpr (T(1) / 2 == 0) {
    switch (op1) {
      case MOA_AND: return simt_fold<T, MOA_AND>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
      case MOA_OR: return simt_fold<T, MOA_OR>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
      case MOA_XOR: return simt_fold<T, MOA_XOR>(op2, A, B, D, M, K, N, tile, Qa, Qb, s);
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
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace moa
