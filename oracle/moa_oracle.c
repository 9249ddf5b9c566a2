/*
 * TEST INFRASTRUCTURE ONLY. Plain, slow, obviously correct CPU oracle for the
 * MoA generalized inner and outer products (Raynolds & Mullin, "A generalized
 * inner and outer product of arbitrary multi-dimensional arrays using A
 * Mathematics of Arrays"). Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product never does. It shares
 * no code, header or constant with the HIP path.
 *
 * Arrays are (shape vector, flat element vector) pairs, row-major with the
 * last axis contiguous and 0-based (Section I; Appendix A, MoA code fragment,
 * whose address arithmetic puts the last axis innermost).
 *
 * Definitions written out here:
 *   outer  C[i ++ j] = A[i] op B[j]                         (Section I, Eq. outer)
 *   inner  D[i ++ j] = fold_l op1 of (A[i ++ <l>] op2 B[<l> ++ j])
 *                                                          (Section I, Eq. inner)
 * The inner product is evaluated in the row form the paper describes: a row
 * <i> psi D of the result is built from rows <l> psi B of B, each combined with
 * one element of A (Section I, worked example and Fig. inner_fig).
 *
 * Readings of points the paper leaves open:
 *   - op1 generalises the sum; the fold is a left fold that starts from the
 *     l = 0 term, in ascending l, so an inner product with one contracted
 *     element is the outer product.
 *   - an empty contraction (K = 0) yields the identity of op1.
 *   - int32 +, -, * wrap in two's complement; max/min are signed.
 *   - FP max/min are the IEEE 754-2019 maximum/minimum (NaN if either
 *     operand is NaN; -0 below +0).
 *
 * Also here (published methods, not in the paper):
 *   - a compensated (+,*) FP64 dot product, Dot2 of Ogita, Rump & Oishi,
 *     "Accurate sum and dot product", SIAM J. Sci. Comput. 26 (2005), used as
 *     the accurate reference for FP64-accuracy results;
 *   - the split ("Ozaki") scheme of Ozaki, Ogita, Oishi & Rump, "Error-free
 *     transformations of matrix multiplication by using fast routines of
 *     matrix multiplication and its applications", Numer. Algorithms 59 (2012),
 *     with signed digits and exact integer slice products, so the BF16/FP8
 *     slice path can be checked tightly against the same scheme.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no FMA contraction:
 * every FP operation below is one IEEE operation).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Operation codes of the oracle (its own numbering). */
enum { O_ADD = 0, O_SUB, O_MUL, O_DIV, O_MAX, O_MIN, O_AND, O_OR, O_XOR };
/* Element types. */
enum { T_F64 = 0, T_F32 = 1, T_I32 = 2 };
/* Arithmetic modes for FP32 inputs: fold in FP64 (the accurate reference) or
 * round every operation to FP32 (what an FP32 device fold computes). */
enum { MODE_WIDE = 0, MODE_NATIVE = 1 };

#define OR_EINVAL (-1)

/* ------------------------------------------------------------------------- */
/* Shapes and psi indexing.                                                   */

/* gamma: row-major flat offset of a full index vector idx into shape dims. */
static int64_t gamma_rm(int rank, const int64_t *dims, const int64_t *idx) {
  int64_t off = 0;
  for (int k = 0; k < rank; ++k) off = off * dims[k] + idx[k];
  return off;
}

static int64_t prod(int rank, const int64_t *dims) {
  int64_t p = 1;
  for (int k = 0; k < rank; ++k) p *= dims[k];
  return p;
}

/* Unravel a flat offset into an index vector (inverse of gamma). */
static void unravel(int rank, const int64_t *dims, int64_t flat, int64_t *idx) {
  for (int k = rank - 1; k >= 0; --k) {
    idx[k] = dims[k] ? flat % dims[k] : 0;
    flat = dims[k] ? flat / dims[k] : 0;
  }
}

/* Offset of <p> psi X for a partial index vector p (length np <= rank): the
 * start of the contiguous sub-array of shape dims[np:], i.e. gamma(p ++ 0...). */
static int64_t psi_offset(int rank, const int64_t *dims, int np, const int64_t *p) {
  int64_t full[32];
  for (int k = 0; k < rank; ++k) full[k] = (k < np) ? p[k] : 0;
  return gamma_rm(rank, dims, full);
}

/* ------------------------------------------------------------------------- */
/* Scalar operations.                                                         */

static double op_f64(int op, double a, double b) {
  switch (op) {
    case O_ADD: return a + b;
    case O_SUB: return a - b;
    case O_MUL: return a * b;
    case O_DIV: return a / b;
    /* IEEE 754-2019 maximum / minimum: a NaN operand gives NaN, and -0 is
     * ordered below +0, so both are associative and commutative. */
    case O_MAX:
      if (isnan(a) || isnan(b)) return NAN;
      if (a == b) return signbit(a) ? b : a;
      return (a < b) ? b : a;
    case O_MIN:
      if (isnan(a) || isnan(b)) return NAN;
      if (a == b) return signbit(a) ? a : b;
      return (b < a) ? b : a;
  }
  return NAN;
}

/* FP32 operation: computed in FP64 and rounded once to FP32. For + - * / of
 * FP32 operands this equals the correctly rounded FP32 result, because FP64
 * carries more than 2*24+2 significand bits (Figueroa, "When is double
 * rounding innocuous?", SIGNUM 1995). */
static float op_f32(int op, float a, float b) {
  return (float)op_f64(op, (double)a, (double)b);
}

static int32_t op_i32(int op, int32_t a, int32_t b) {
  uint32_t ua = (uint32_t)a, ub = (uint32_t)b;
  switch (op) {
    case O_ADD: return (int32_t)(ua + ub);
    case O_SUB: return (int32_t)(ua - ub);
    case O_MUL: return (int32_t)(ua * ub);
    case O_MAX: return (a < b) ? b : a;
    case O_MIN: return (b < a) ? b : a;
    case O_AND: return (int32_t)(ua & ub);
    case O_OR: return (int32_t)(ua | ub);
    case O_XOR: return (int32_t)(ua ^ ub);
  }
  return 0;
}

static int op_is_fold(int op, int dtype) {
  if (op == O_ADD || op == O_MUL || op == O_MAX || op == O_MIN) return 1;
  if (dtype == T_I32 && (op == O_AND || op == O_OR || op == O_XOR)) return 1;
  return 0;
}

static int op_is_elem(int op, int dtype) {
  if (op <= O_MIN) return !(dtype == T_I32 && op == O_DIV);
  return dtype == T_I32 && op <= O_XOR;
}

/* Identity of op1, the value of an empty fold. */
static double ident_f64(int op) {
  switch (op) {
    case O_ADD: return 0.0;
    case O_MUL: return 1.0;
    case O_MAX: return -INFINITY;
    case O_MIN: return INFINITY;
  }
  return NAN;
}
static int32_t ident_i32(int op) {
  switch (op) {
    case O_ADD: return 0;
    case O_MUL: return 1;
    case O_MAX: return INT32_MIN;
    case O_MIN: return INT32_MAX;
    case O_AND: return -1;
    case O_OR: return 0;
    case O_XOR: return 0;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Generalized inner product (Section I, Eq. inner), row form.                */

/*
 * ra, da: rank and shape of A (ra >= 1); rb, db: rank and shape of B (rb >= 1)
 * with da[ra-1] == db[0]. Result shape is da[:ra-1] ++ db[1:].
 * rows: if non-NULL, the flat indices (over da[:ra-1]) of the result rows to
 * compute, nrows of them; D then holds nrows consecutive rows. If NULL, all
 * rows are computed into D in order.
 * Output element type: F64 for dtype F64, and for F32 in MODE_WIDE; F32 for
 * F32 in MODE_NATIVE; I32 for I32.
 */
int oracle_inner(int ra, const int64_t *da, const void *A, int rb, const int64_t *db, const void *B,
                 int op1, int op2, int dtype, int mode, void *D, const int64_t *rows, int64_t nrows) {
  if (ra < 1 || rb < 1 || ra > 16 || rb > 16) return OR_EINVAL;
  if (da[ra - 1] != db[0]) return OR_EINVAL;
  if (!op_is_fold(op1, dtype) || !op_is_elem(op2, dtype)) return OR_EINVAL;
  const int64_t K = da[ra - 1];
  const int64_t M = prod(ra - 1, da);
  const int64_t N = prod(rb - 1, db + 1);
  const int64_t nr = rows ? nrows : M;

#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r = 0; r < nr; ++r) {
    int64_t irow = rows ? rows[r] : r;
    /* Index vector i over rho A without its last axis. */
    int64_t ivec[16];
    unravel(ra - 1, da, irow, ivec);
    /* A[i ++ <l>] lives at psi_offset(i) + l: <i> psi A is the contiguous
     * vector of the K elements the row contracts over. */
    const int64_t a_off = psi_offset(ra, da, ra - 1, ivec);
    const int64_t d_off = r * N;
    for (int64_t l = 0; l < K; ++l) {
      /* <l> psi B: the l-th row of B, a contiguous block of N elements. */
      const int64_t lvec[1] = {l};
      const int64_t b_off = psi_offset(rb, db, 1, lvec);
      for (int64_t j = 0; j < N; ++j) {
        if (dtype == T_F64) {
          double t = op_f64(op2, ((const double *)A)[a_off + l], ((const double *)B)[b_off + j]);
          double *d = (double *)D + d_off + j;
          *d = (l == 0) ? t : op_f64(op1, *d, t);
        } else if (dtype == T_F32 && mode == MODE_WIDE) {
          double t = op_f64(op2, (double)((const float *)A)[a_off + l], (double)((const float *)B)[b_off + j]);
          double *d = (double *)D + d_off + j;
          *d = (l == 0) ? t : op_f64(op1, *d, t);
        } else if (dtype == T_F32) {
          float t = op_f32(op2, ((const float *)A)[a_off + l], ((const float *)B)[b_off + j]);
          float *d = (float *)D + d_off + j;
          *d = (l == 0) ? t : op_f32(op1, *d, t);
        } else {
          int32_t t = op_i32(op2, ((const int32_t *)A)[a_off + l], ((const int32_t *)B)[b_off + j]);
          int32_t *d = (int32_t *)D + d_off + j;
          *d = (l == 0) ? t : op_i32(op1, *d, t);
        }
      }
    }
    if (K == 0) {
      for (int64_t j = 0; j < N; ++j) {
        if (dtype == T_F64 || (dtype == T_F32 && mode == MODE_WIDE))
          ((double *)D)[d_off + j] = ident_f64(op1);
        else if (dtype == T_F32)
          ((float *)D)[d_off + j] = (float)ident_f64(op1);
        else
          ((int32_t *)D)[d_off + j] = ident_i32(op1);
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Generalized outer product (Section I, Eq. outer).                          */

/* C has shape da ++ db (either rank may be 0). Output element type as for
 * oracle_inner (FP32 inputs: F64 in MODE_WIDE, F32 in MODE_NATIVE). */
int oracle_outer(int ra, const int64_t *da, const void *A, int rb, const int64_t *db, const void *B,
                 int op, int dtype, int mode, void *C) {
  if (ra < 0 || rb < 0 || ra + rb > 32) return OR_EINVAL;
  if (!op_is_elem(op, dtype)) return OR_EINVAL;
  const int64_t NA = prod(ra, da), NB = prod(rb, db);
  int64_t dc[32];
  for (int k = 0; k < ra; ++k) dc[k] = da[k];
  for (int k = 0; k < rb; ++k) dc[ra + k] = db[k];

#pragma omp parallel for schedule(static)
  for (int64_t ia = 0; ia < NA; ++ia) {
    int64_t idx[32];
    unravel(ra, da, ia, idx);
    const int64_t a_el = gamma_rm(ra, da, idx);
    for (int64_t jb = 0; jb < NB; ++jb) {
      unravel(rb, db, jb, idx + ra);
      const int64_t b_el = gamma_rm(rb, db, idx + ra);
      const int64_t c_el = gamma_rm(ra + rb, dc, idx);
      if (dtype == T_F64) {
        ((double *)C)[c_el] = op_f64(op, ((const double *)A)[a_el], ((const double *)B)[b_el]);
      } else if (dtype == T_F32 && mode == MODE_WIDE) {
        ((double *)C)[c_el] = op_f64(op, (double)((const float *)A)[a_el], (double)((const float *)B)[b_el]);
      } else if (dtype == T_F32) {
        ((float *)C)[c_el] = op_f32(op, ((const float *)A)[a_el], ((const float *)B)[b_el]);
      } else {
        ((int32_t *)C)[c_el] = op_i32(op, ((const int32_t *)A)[a_el], ((const int32_t *)B)[b_el]);
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Compensated (+,*) FP64 inner product: Dot2 (Ogita, Rump & Oishi 2005).     */

/* Error-free product: a*b = p + e exactly (fma is exactly rounded). */
static void two_prod(double a, double b, double *p, double *e) {
  *p = a * b;
  *e = fma(a, b, -*p);
}
/* Error-free sum (Knuth): a+b = s + e exactly. */
static void two_sum(double a, double b, double *s, double *e) {
  *s = a + b;
  double z = *s - a;
  *e = (a - (*s - z)) + (b - z);
}

/* Same shape contract as oracle_inner with op1 = +, op2 = *, dtype F64 (or
 * F32 inputs widened to F64). Output F64. */
int oracle_dot2_inner(int ra, const int64_t *da, const void *A, int rb, const int64_t *db, const void *B,
                      int dtype, double *D, const int64_t *rows, int64_t nrows) {
  if (ra < 1 || rb < 1 || ra > 16 || rb > 16) return OR_EINVAL;
  if (da[ra - 1] != db[0]) return OR_EINVAL;
  if (dtype != T_F64 && dtype != T_F32) return OR_EINVAL;
  const int64_t K = da[ra - 1];
  const int64_t M = prod(ra - 1, da);
  const int64_t N = prod(rb - 1, db + 1);
  const int64_t nr = rows ? nrows : M;

#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r = 0; r < nr; ++r) {
    int64_t irow = rows ? rows[r] : r;
    int64_t ivec[16];
    unravel(ra - 1, da, irow, ivec);
    const int64_t a_off = psi_offset(ra, da, ra - 1, ivec);
    double *s = (double *)malloc(sizeof(double) * (size_t)(N ? N : 1));
    double *c = (double *)malloc(sizeof(double) * (size_t)(N ? N : 1));
    for (int64_t j = 0; j < N; ++j) s[j] = c[j] = 0.0;
    for (int64_t l = 0; l < K; ++l) {
      const int64_t lvec[1] = {l};
      const int64_t b_off = psi_offset(rb, db, 1, lvec);
      double a = (dtype == T_F64) ? ((const double *)A)[a_off + l] : (double)((const float *)A)[a_off + l];
      for (int64_t j = 0; j < N; ++j) {
        double b = (dtype == T_F64) ? ((const double *)B)[b_off + j] : (double)((const float *)B)[b_off + j];
        double p, q, t, e;
        two_prod(a, b, &p, &e);
        two_sum(s[j], p, &t, &q);
        s[j] = t;
        c[j] = c[j] + (q + e);
      }
    }
    for (int64_t j = 0; j < N; ++j) D[r * N + j] = s[j] + c[j];
    free(s);
    free(c);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Split (Ozaki) scheme with signed digits.                                   */
/*
 * A row of A (or a column of B) is scaled by a power of two 2^-e, where e is
 * the exponent with max|x| < 2^e, so every scaled entry x lies in (-1, 1).
 * x is then written as signed base-2^beta digits:
 *     sigma_0 = rint(x * 2^(beta-1)),           r_0 = x * 2^(beta-1) - sigma_0
 *     sigma_s = rint(r_{s-1} * 2^beta),         r_s = r_{s-1} * 2^beta - sigma_s
 * so x = sum_s sigma_s * 2^-(beta-1+beta*s) + residual, with every
 * |sigma_s| <= 2^(beta-1). All of these steps are exact in FP64.
 * The product keeps the pairs (s, t) with s + t < S ("triangular" set):
 *     D_ij = 2^(e_i+f_j) * sum_{s+t<S} 2^-(2(beta-1)+beta(s+t)) * T_st[i,j],
 *     T_st = sigma^A_s . sigma^B_t, an exact integer dot product.
 */

/* Row exponents: e[i] with max_l |X[i,l]| < 2^e[i] (0 for an all-zero row).
 * X is rows x cols, row stride ld, column stride cs (so columns of a
 * row-major matrix are scanned with ld = 1, cs = ncols). */
static void scan_exponents(int64_t rows, int64_t cols, const double *X, int64_t ld, int64_t cs, int32_t *e) {
  for (int64_t i = 0; i < rows; ++i) {
    double mx = 0.0;
    for (int64_t l = 0; l < cols; ++l) {
      double v = fabs(X[i * ld + l * cs]);
      if (v > mx) mx = v;
    }
    int ex = 0;
    (void)frexp(mx, &ex);
    e[i] = (int32_t)ex;
  }
}

/* Signed digits of one scaled value. */
static void digits_of(double x, int beta, int S, int32_t *sig) {
  double r = ldexp(x, beta - 1);
  for (int s = 0; s < S; ++s) {
    double d = rint(r);
    sig[s] = (int32_t)d;
    r = ldexp(r - d, beta);
  }
}

/*
 * Digits of a row-major rows x cols matrix X, scaled per row (by_rows = 1) or
 * per column (by_rows = 0). Writes exps (rows or cols entries) and
 * sig[s * rows * cols + i * cols + l].
 */
int oracle_split_digits(int64_t rows, int64_t cols, const double *X, int by_rows, int beta, int S,
                        int32_t *exps, int32_t *sig) {
  if (beta < 2 || beta > 12 || S < 1 || S > 16) return OR_EINVAL;
  if (by_rows)
    scan_exponents(rows, cols, X, cols, 1, exps);
  else
    scan_exponents(cols, rows, X, 1, cols, exps);
  const int64_t n = rows * cols;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < rows; ++i) {
    int32_t tmp[16];
    for (int64_t l = 0; l < cols; ++l) {
      int e = by_rows ? exps[i] : exps[l];
      digits_of(ldexp(X[i * cols + l], -e), beta, S, tmp);
      for (int s = 0; s < S; ++s) sig[(int64_t)s * n + i * cols + l] = tmp[s];
    }
  }
  return 0;
}

/*
 * D = A * B (flattened M x K and K x N, row-major FP64) by the triangular
 * split scheme with S digits of beta bits. rows/nrows select result rows as
 * in oracle_inner. Output FP64, nrows x N (or M x N).
 */
int oracle_split_inner(int64_t M, int64_t K, int64_t N, const double *A, const double *B, int beta, int S,
                       double *D, const int64_t *rows, int64_t nrows) {
  if (beta < 2 || beta > 12 || S < 1 || S > 16) return OR_EINVAL;
  const int64_t nr = rows ? nrows : M;
  int32_t *eA = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M ? M : 1));
  int32_t *fB = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
  const int64_t nsb = (int64_t)S * K * N;
  int32_t *sB = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nsb > 0 ? nsb : 1));
  if (!eA || !fB || !sB) { free(eA); free(fB); free(sB); return OR_EINVAL; }
  scan_exponents(M, K, A, K, 1, eA);
  /* B digits scaled per column of B. */
  oracle_split_digits(K, N, B, 0, beta, S, fB, sB);

#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r = 0; r < nr; ++r) {
    const int64_t i = rows ? rows[r] : r;
    int32_t *sA = (int32_t *)malloc(sizeof(int32_t) * (size_t)(S * (K ? K : 1)));
    int64_t *T = (int64_t *)calloc((size_t)(S * S * (N ? N : 1)), sizeof(int64_t));
    for (int64_t l = 0; l < K; ++l) {
      int32_t tmp[16];
      digits_of(ldexp(A[i * K + l], -eA[i]), beta, S, tmp);
      for (int s = 0; s < S; ++s) sA[s * K + l] = tmp[s];
    }
    /* Exact integer slice products, row form: T_st[j] += sA_s[l] * sB_t[l, j]. */
    for (int s = 0; s < S; ++s)
      for (int t = 0; s + t < S; ++t)
        for (int64_t l = 0; l < K; ++l) {
          const int64_t a = sA[s * K + l];
          const int32_t *brow = sB + (int64_t)t * K * N + l * N;
          int64_t *Trow = T + ((int64_t)s * S + t) * N;
          for (int64_t j = 0; j < N; ++j) Trow[j] += a * brow[j];
        }
    /* FP64 slice sum, smallest weights first, then the exact power-of-two
     * descaling. */
    for (int64_t j = 0; j < N; ++j) {
      double acc = 0.0;
      for (int d = S - 1; d >= 0; --d)
        for (int s = 0; s <= d; ++s) {
          const int t = d - s;
          acc += ldexp((double)T[((int64_t)s * S + t) * N + j], -(2 * (beta - 1) + beta * d));
        }
      D[r * N + j] = ldexp(acc, eA[i] + fB[j]);
    }
    free(sA);
    free(T);
  }
  free(eA);
  free(fB);
  free(sB);
  return 0;
}
