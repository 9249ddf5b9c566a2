/*
 * moa.h — C ABI of libmoa: generalized inner and outer products of
 * arbitrary-rank arrays on one AMD Instinct MI355X (gfx950).
 *
 * Operations follow Raynolds & Mullin, "A generalized inner and outer product
 * of arbitrary multi-dimensional arrays using A Mathematics of Arrays (MoA)":
 *
 *   outer  C[i ++ j] = A[i] op B[j]                             (Section I, Eq. outer)
 *   inner  D[i ++ j] = op1-fold over p of A[i ++ <p>] op2 B[<p> ++ j]
 *                                                              (Section I, Eq. inner)
 *
 * with the binary operations generalised as the paper states (any op2; op1 an
 * associative and commutative operation that generalises the sum).
 *
 * Arrays. An array is its shape vector plus a flat vector of its elements
 * (Section I). Elements are dense, row-major, last axis contiguous, 0-based
 * (the address arithmetic of the MoA code fragment in Appendix A). Shape
 * vectors live in host memory and are read only during the call. Element
 * buffers are DEVICE pointers owned by the caller; the library never frees
 * them and never keeps them past the call (moa_batch excepted, see below).
 *
 * Shapes. inner: rank A >= 1, rank B >= 1, rhoA[-1] == rhoB[0];
 * result shape rhoA[:-1] ++ rhoB[1:] (rank 0 when both are vectors).
 * outer: any ranks (0 allowed); result shape rhoA ++ rhoB. Ranks are at most
 * MOA_MAX_RANK per operand; every extent is >= 0.
 *
 * Fold. The op1 fold is a left fold that starts from the first term, so an
 * inner product over one contracted element is the outer product. An empty
 * contraction (rhoA[-1] == 0) gives the identity of op1
 * (+: 0, *: 1, max: -inf / INT32_MIN, min: +inf / INT32_MAX, and: ~0, or/xor: 0).
 *
 * Arithmetic. int32 +, -, * wrap (two's complement); max/min are signed.
 * FP max/min are the IEEE 754-2019 maximum/minimum: a NaN operand gives NaN
 * and -0 is ordered below +0, which makes them associative and commutative.
 * FP (op1, op2) pairs other than (+,*) fold in ascending p, one IEEE
 * operation per step, so they match a sequential fold bit for bit, signed
 * zeros included (NaN payloads are not specified). (+,*) on
 * FP64 / FP32 runs on the matrix cores in another summation order (normwise
 * relative error of order K * unit roundoff), except for results with at most
 * 8 rows (product of rhoA[:-1]) and at least 4096 columns, which stream B
 * from memory and fold in ascending p like every other pair. Folds whose value does
 * not depend on association (every int32 op1, FP max and min) may be combined
 * in any order: with at most 16 columns and K >= 256 the terms are split over
 * the lanes of a wave and combined by a cross-lane reduction (the same
 * value, bit for bit).
 *
 * Errors. Every call validates on the host before any launch and returns a
 * moa_status; nothing is launched on an error. Kernel execution is
 * asynchronous on the given stream (a hipStream_t passed as void*; NULL is
 * the default stream). MOA_ERR_HIP means a HIP runtime call failed;
 * moa_last_error() then holds its message.
 */
#ifndef MOA_H_
#define MOA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MOA_MAX_RANK 16
#define MOA_ABI_VERSION 1

typedef struct moa_shape {
  int32_t rank;         /* 0 .. MOA_MAX_RANK */
  const int64_t *dims;  /* host array of `rank` extents (may be NULL when rank == 0) */
} moa_shape;

/* The *_RANGE_ enumerators are not values to pass: they make every int32
 * value a valid value of the enum type, so a wrong code a caller passes is
 * rejected by the validation (MOA_ERR_DTYPE / MOA_ERR_OP) rather than being
 * undefined behaviour in the library. */
typedef enum moa_dtype {
  MOA_F64 = 0, MOA_F32 = 1, MOA_I32 = 2,
  MOA_DTYPE_RANGE_MIN_ = -2147483647 - 1, MOA_DTYPE_RANGE_MAX_ = 2147483647
} moa_dtype;

typedef enum moa_op {
  MOA_ADD = 0, MOA_SUB = 1, MOA_MUL = 2, MOA_DIV = 3, MOA_MAX = 4,
  MOA_MIN = 5, MOA_AND = 6, MOA_OR = 7, MOA_XOR = 8,
  MOA_OP_RANGE_MIN_ = -2147483647 - 1, MOA_OP_RANGE_MAX_ = 2147483647
} moa_op;

typedef enum moa_status {
  MOA_OK = 0,
  MOA_ERR_NULL = 1,       /* a required pointer is NULL */
  MOA_ERR_RANK = 2,       /* rank out of range (inner needs rank >= 1) */
  MOA_ERR_SHAPE = 3,      /* negative extent, or rhoA[-1] != rhoB[0] */
  MOA_ERR_OP = 4,         /* op1 not a fold op, bitwise op on FP, int32 div */
  MOA_ERR_DTYPE = 5,      /* unknown or unsupported element type */
  MOA_ERR_SIZE = 6,       /* element count or byte size overflows int64 */
  MOA_ERR_ALIAS = 7,      /* output overlaps an input */
  MOA_ERR_WORKSPACE = 8,  /* workspace missing or too small */
  MOA_ERR_HIP = 9,        /* a HIP runtime call failed */
  MOA_ERR_ARG = 10,       /* other invalid argument (format, slice count, ...) */
  MOA_STATUS_RANGE_MIN_ = -2147483647 - 1, MOA_STATUS_RANGE_MAX_ = 2147483647
} moa_status;

/* Status name, static string. */
const char *moa_status_str(moa_status s);
/* Detail of the last error on this thread (empty string if none). */
const char *moa_last_error(void);
int32_t moa_abi_version(void);

/* ---------------------------------------------------------------------------
 * Shape algebra (host only, no GPU needed).
 * out_dims must hold 2*MOA_MAX_RANK entries (an inner result has rank up to
 * 2*MOA_MAX_RANK - 2, an outer one up to 2*MOA_MAX_RANK).
 */
moa_status moa_inner_shape(moa_shape a, moa_shape b, int64_t *out_dims, int32_t *out_rank);
moa_status moa_outer_shape(moa_shape a, moa_shape b, int64_t *out_dims, int32_t *out_rank);

/* ---------------------------------------------------------------------------
 * Generalized inner product (Section I, Eq. inner).
 * A, B: device arrays of dtype dt, shapes sa, sb. D: device array of dtype dt
 * with the result shape; must not overlap A or B.
 * op1 in {ADD, MUL, MAX, MIN} (+ AND, OR, XOR for I32); op2 any op
 * (bitwise ops for I32 only; DIV for FP only).
 */
moa_status moa_inner(moa_shape sa, const void *A, moa_shape sb, const void *B, moa_op op1, moa_op op2,
                     moa_dtype dt, void *D, void *stream);

/* Flags for moa_inner_ex. */
#define MOA_FLAG_SEQUENTIAL_FOLD 1u /* (+,*) on FP too: fold in ascending p on the vector units */

/* moa_inner with flags (0 = moa_inner). */
moa_status moa_inner_ex(moa_shape sa, const void *A, moa_shape sb, const void *B, moa_op op1, moa_op op2,
                        moa_dtype dt, void *D, uint32_t flags, void *stream);

/* ---------------------------------------------------------------------------
 * Generalized inner product over any axis pair: the contraction of Eq. inner
 * (Section I, where the inner product is shown to be a tensor contraction)
 * taken over axis ax_a of A and axis ax_b of B instead of the last and the
 * first. Both operands are read in place through start/stride/count index
 * maps, the Operational Normal Form of Section II.D, with no transposed copy:
 * A as (Pa, K, Qa) with Pa = prod rhoA[0:ax_a], K = rhoA[ax_a],
 * Qa = prod rhoA[ax_a+1:], B likewise as (Pb, K, Qb), and
 *   D[(pa, qa), (pb, qb)] = op1-fold_k op2(A[pa, k, qa], B[pb, k, qb]).
 * The result shape is rhoA without axis ax_a ++ rhoB without axis ax_b (the
 * axis order of numpy.tensordot(A, B, axes=(ax_a, ax_b))), row-major.
 * ax_a = rank(A) - 1, ax_b = 0 is moa_inner_ex exactly. Requirements:
 * 0 <= ax_a < rank(A), 0 <= ax_b < rank(B) (else MOA_ERR_ARG),
 * rhoA[ax_a] = rhoB[ax_b] (else MOA_ERR_SHAPE); ops, dtypes, flags, aliasing
 * and the fold order as for moa_inner_ex.
 */
/* Result shape of moa_inner_axes; out_dims must hold 2*MOA_MAX_RANK entries. */
moa_status moa_inner_axes_shape(moa_shape a, int32_t ax_a, moa_shape b, int32_t ax_b, int64_t *out_dims,
                                int32_t *out_rank);
moa_status moa_inner_axes(moa_shape sa, const void *A, int32_t ax_a, moa_shape sb, const void *B, int32_t ax_b,
                          moa_op op1, moa_op op2, moa_dtype dt, void *D, uint32_t flags, void *stream);

/* ---------------------------------------------------------------------------
 * Generalized outer product (Section I, Eq. outer), computed by the same
 * definition as moa_inner with one contracted element. C has shape sa ++ sb.
 * Every element is one IEEE operation (bit-exact).
 */
moa_status moa_outer(moa_shape sa, const void *A, moa_shape sb, const void *B, moa_op op, moa_dtype dt, void *C,
                     void *stream);

/* ---------------------------------------------------------------------------
 * (+,*) FP64 inner product at FP64 accuracy from low-precision slices
 * (the split scheme of Ozaki, Ogita, Oishi & Rump, Numer. Algorithms 59, 2012;
 * a numerical extension, not part of the paper).
 *
 * Each row of A and each column of B is scaled by a power of two so its
 * entries lie in (-1, 1), then written as `nslices` signed digits of beta
 * bits, each digit an integer the slice format holds exactly
 * (MOA_SPLIT_BF16: beta = 9, |digit| <= 256, FP32 accumulation, exact for the
 * leading weights; MOA_SPLIT_INT8: beta = 7, |digit| <= 64, INT32
 * accumulation, exact; MOA_SPLIT_FP8: E4M3 digits, beta = 5, |digit| <= 16,
 * FP32 accumulation, exact). The slice pairs (s, t) with s + t < nslices are
 * multiplied on the matrix cores, summed in FP64 and scaled back exactly.
 * Requirements: finite inputs; 1 <= nslices <= 7 (BF16, INT8) or 10 (FP8)
 * (MOA_SPLIT_MAX_SLICES is the largest of these).
 * Accuracy (entries u*2^k with k in [-8, 8], K = 8192), normwise relative
 * error against an exactly rounded product: BF16, nslices = 5 (15 pairs):
 * about 7e-13; INT8, nslices = 7 (28 pairs): about 5e-14; FP8, nslices = 9
 * (45 pairs): about 8e-13, nslices = 10 (55 pairs): about 3e-14.
 *
 * ws: device workspace of at least moa_inner_split_workspace(...) bytes, owned
 * by the caller, 256-byte aligned; contents on entry are ignored.
 */
#define MOA_SPLIT_BF16 0
#define MOA_SPLIT_FP8 1
#define MOA_SPLIT_INT8 2
#define MOA_SPLIT_MAX_SLICES 10
size_t moa_inner_split_workspace(moa_shape sa, moa_shape sb, int32_t fmt, int32_t nslices);
moa_status moa_inner_split(moa_shape sa, const double *A, moa_shape sb, const double *B, double *D, int32_t fmt,
                           int32_t nslices, void *ws, size_t ws_bytes, void *stream);
/* The two halves of moa_inner_split, for callers that reuse slices or time
 * the stages: _prepare scans and slices A and B into ws; _multiply forms the
 * slice-pair products from ws into D (same shapes, format and slice count as
 * the _prepare call that filled ws; ws must not be modified in between). */
moa_status moa_inner_split_prepare(moa_shape sa, const double *A, moa_shape sb, const double *B, int32_t fmt,
                                   int32_t nslices, void *ws, size_t ws_bytes, void *stream);
moa_status moa_inner_split_multiply(moa_shape sa, moa_shape sb, double *D, int32_t fmt, int32_t nslices, void *ws,
                                    size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * moa_inner_split without a workspace and without any allocation, for callers
 * that cannot allocate device memory (code being captured into a HIP graph,
 * tight serving loops, harnesses that forbid hipMalloc). The scratch lives in
 * a static device array of MOA_SPLIT_STATIC_BYTES bytes that each GPU the
 * library runs on holds until the process ends. Same arguments, results and
 * errors as moa_inner_split minus ws / ws_bytes; a problem whose workspace
 * (moa_inner_split_workspace) exceeds MOA_SPLIT_STATIC_BYTES is refused with
 * MOA_ERR_WORKSPACE before any launch (at S = 5 BF16 slices that admits
 * square products up to about 2500^3). Every call on one GPU shares that
 * GPU's array, so calls that overlap on one GPU (other streams, other host
 * threads) race; calls in one stream are ordered and safe. The array keeps
 * the last call's contents; everything a call reads from it, the call has
 * written first (the column maxima are cleared by a kernel).
 */
#define MOA_SPLIT_STATIC_BYTES ((size_t)128 << 20)
moa_status moa_inner_split_static(moa_shape sa, const double *A, moa_shape sb, const double *B, double *D,
                                  int32_t fmt, int32_t nslices, void *stream);

/* ---------------------------------------------------------------------------
 * Backward of the (+,*) inner product D = A . B (FP32 or FP64).
 * G: upstream gradient dL/dD with the result shape. Writes
 *   dA = G (+,*) B_rot   (B_rot: B with its first axis moved last)  shape sa
 *   dB = A_rot (+,*) G   (A_rot: A with its last axis moved first)  shape sb
 * both generalized inner products on permuted shapes; the permutations are
 * folded into the operand loads (no transposed copies are made).
 * dA or dB may be NULL to skip it. Outputs must not overlap inputs.
 */
moa_status moa_inner_grad(moa_shape sa, const void *A, moa_shape sb, const void *B, const void *G, void *dA,
                          void *dB, moa_dtype dt, void *stream);

/* ---------------------------------------------------------------------------
 * Batches of uneven (+,*) inner products in one persistent launch.
 *
 * moa_batch_build validates every problem on the host, orders the work by
 * estimated cost, uploads the work list (one record per output tile: the
 * problem's pointers and shape, the tile choice from the tile table and the
 * tile's origin) on `stream`, waits for that upload, and captures the persistent launch in a
 * HIP graph (on a private stream: capture is not allowed on the default
 * stream). Each D[i] must hold the whole result of problem i (its shape is
 * that of moa_inner_shape(sa[i], sb[i])). The caller's A[i], B[i], D[i] (device
 * pointers, dtype dt = MOA_F32 or MOA_F64) must stay valid while the batch
 * exists; moa_batch_run replays the graph (one kernel launch). A batch owns
 * only its work list and graph; moa_batch_free releases
 * them. A run keeps no state, but concurrent runs of one batch write the
 * same D arrays.
 */
typedef struct moa_batch moa_batch;
moa_status moa_batch_build(int32_t n, const moa_shape *sa, const void *const *A, const moa_shape *sb,
                           const void *const *B, void *const *D, moa_dtype dt, void *stream, moa_batch **out);
moa_status moa_batch_run(moa_batch *b, void *stream);
void moa_batch_free(moa_batch *b);
/* Number of work items (problem tiles) and kernel launches per run. */
moa_status moa_batch_info(const moa_batch *b, int64_t *work_items, int32_t *launches);

/* Tile table used by moa_batch_build: for each (M, N, K) size bucket the
 * tile variant to use. moa_batch_autotune times every tile variant on
 * synthetic problems of each bucket on `stream` and installs the fastest;
 * moa_tile_table_get/set read or replace the table as text: eight lines
 * "bucket_m bucket_n bucket_k variant", one per bucket, with bucket_m one of
 * "M<=32" / "M>32", bucket_n "N<=32" / "N>32", bucket_k "K<=128" / "K>128"
 * and variant 0 (32 x 32 tiles) or 1 (64 x 64). moa_tile_table_set rejects
 * (MOA_ERR_ARG, table unchanged) any other token, a bucket given twice or a
 * missing bucket. */
moa_status moa_batch_autotune(moa_dtype dt, int32_t reps, void *stream);
moa_status moa_tile_table_get(char *buf, size_t len);
moa_status moa_tile_table_set(const char *text);

#ifdef __cplusplus
}
#endif

#endif /* MOA_H_ */
