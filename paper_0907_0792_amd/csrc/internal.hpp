// Internal launchers of libmoa. Every launcher takes the flattened sizes the
// host layer computed (rank never reaches the device), launches on `s`, and
// returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "moa.h"

namespace moa {

// D (M x N) = op1-fold_l op2(A[i,l], B[l,j]) on the vector ALUs, ascending l.
// tile: 8, 4 or 2 (register block per thread, side), 0 = automatic.
// Qa, Qb: strided views for a contraction over any axis pair (A read as
// (P_a, K, Qa), B as (P_b, K, Qb)); Qa = 1, Qb = N (or <= 0) is last-with-first.
hipError_t launch_simt_inner(moa_dtype dt, moa_op op1, moa_op op2, const void *A, const void *B, void *D, int64_t M,
                             int64_t K, int64_t N, int tile, hipStream_t s, int64_t Qa = 1, int64_t Qb = 0);

// Few-row inner product (M <= kSkinnyMaxRows): the row form as an HBM stream,
// every element of B read once, ascending-l fold (bit-exact, any op pair).
constexpr int64_t kSkinnyMaxRows = 8;
hipError_t launch_skinny_inner(moa_dtype dt, moa_op op1, moa_op op2, const void *A, const void *B, void *D, int64_t M,
                               int64_t K, int64_t N, hipStream_t s);

// Few-column inner product (N <= kFewColsMax) for association-independent
// folds (int32, FP max/min): the fold over l split across a wave's lanes and
// combined by a wavefront reduction.
constexpr int64_t kFewColsMax = 16;
bool fewcols_applies(moa_dtype dt, moa_op op1, int64_t M, int64_t K, int64_t N);
hipError_t launch_fewcols_inner(moa_dtype dt, moa_op op1, moa_op op2, const void *A, const void *B, void *D,
                                int64_t M, int64_t K, int64_t N, hipStream_t s);

// C (NA x NB) = op(A[i], B[j]).
hipError_t launch_outer(moa_dtype dt, moa_op op, const void *A, const void *B, void *C, int64_t NA, int64_t NB,
                        hipStream_t s);

// D (M x N) = A (M x K) * B (K x N) on the matrix cores, FP64 or FP32.
// trans_a: A is stored K x M (row-major) instead of M x K.
// trans_b: B is stored N x K instead of K x N.
// lda/ldb are implied by the stored shapes. tile: 0 automatic, 1 = 128x128, 2 = 64x64,
// 3 = 32x32.
hipError_t launch_gemm(moa_dtype dt, bool trans_a, bool trans_b, const void *A, const void *B, void *D, int64_t M,
                       int64_t K, int64_t N, int tile, hipStream_t s);

// Both products of the (+,*) backward, dA (M x K) = G (M x N) . B^T and
// dB (K x N) = A^T . G, with A stored M x K, B stored K x N, G stored M x N;
// one launch when both products take the same tile size. M, K, N > 0.
hipError_t launch_gemm_grad(moa_dtype dt, const void *G, const void *A, const void *B, void *dA, void *dB, int64_t M,
                            int64_t K, int64_t N, hipStream_t s);

// (+,*) on the matrix cores over the strided views above (general axes).
hipError_t launch_gemm_strided(moa_dtype dt, const void *A, const void *B, void *D, int64_t M, int64_t K, int64_t N,
                               int64_t Qa, int64_t Qb, hipStream_t s);

// Fill n elements of dtype dt at p with the identity of op (empty fold).
hipError_t launch_fill_identity(moa_dtype dt, moa_op op, void *p, int64_t n, hipStream_t s);

// Split (Ozaki) FP64 product.
struct SplitPlan {
  int64_t M, K, N;
  int64_t Mp, Kp, Np;  // padded extents
  int fmt, S, beta;
  size_t off_ea, off_fb, off_ap, off_bp, total;
};
// Largest slice count of a split format (0 for an unknown format).
int split_max_slices(int fmt);
bool split_plan(int64_t M, int64_t K, int64_t N, int fmt, int S, SplitPlan *p);
hipError_t launch_split_prepare(const SplitPlan &p, const double *A, const double *B, void *ws, hipStream_t s);
hipError_t launch_split_multiply(const SplitPlan &p, double *D, void *ws, hipStream_t s);

// Batched persistent (+,*) products.
struct BatchDesc {  // one problem (host side, while the work list is built)
  const void *A;
  const void *B;
  void *D;
  int32_t M, K, N;
  int32_t tile;     // tile variant
  int32_t tiles_n;  // tiles along N for this problem
};
// One work item: one output tile of one problem, self-contained (the
// kernel reads one record per item, with no second, dependent load).
struct BatchItem {
  const void *A;
  const void *B;
  void *D;
  int32_t M, K, N;
  int32_t tile;    // tile variant
  int32_t m0, n0;  // tile origin
};

}  // namespace moa
