// Host side of the C ABI: validation, shape algebra, flattening and dispatch.
//
// Every rank reduces to one M x K by K x N fold: with row-major flat element
// vectors, rho A = a_0..a_{p-1} and rho B = b_0..b_{q-1} give
// M = prod a_0..a_{p-2}, K = a_{p-1} = b_0, N = prod b_1..b_{q-1}, and the
// result rho D = a_0..a_{p-2} ++ b_1..b_{q-1} is the M x N row-major matrix.
// This is the flattening the MoA code fragment of Appendix A performs with its
// row count, reduction length and row length. The outer product is the same
// with K = 1 (rho A ++ <1> against <1> ++ rho B; Section I states that both
// operations share one code).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "common.hpp"
#include "internal.hpp"

namespace {

thread_local std::string g_last_error;

moa_status fail(moa_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
moa_status fail(moa_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

moa_status hip_status(hipError_t e, const char *what) {
  if (e == hipSuccess) return MOA_OK;
  return fail(MOA_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t elem_size(moa_dtype dt) {
  switch (dt) {
    case MOA_F64: return 8;
    case MOA_F32: return 4;
    case MOA_I32: return 4;
    default: break;
  }
  return 0;
}

bool valid_dtype(int dt) { return dt == MOA_F64 || dt == MOA_F32 || dt == MOA_I32; }

bool is_fold_op(moa_op op, moa_dtype dt) {
  if (op == MOA_ADD || op == MOA_MUL || op == MOA_MAX || op == MOA_MIN) return true;
  return dt == MOA_I32 && (op == MOA_AND || op == MOA_OR || op == MOA_XOR);
}

bool is_elem_op(moa_op op, moa_dtype dt) {
  switch (op) {
    case MOA_ADD:
    case MOA_SUB:
    case MOA_MUL:
    case MOA_MAX:
    case MOA_MIN: return true;
    case MOA_DIV: return dt != MOA_I32;
    case MOA_AND:
    case MOA_OR:
    case MOA_XOR: return dt == MOA_I32;
    default: break;
  }
  return false;
}

// Product of extents with overflow check (extents already validated >= 0).
bool checked_prod(const int64_t *d, int n, int64_t *out) {
  int64_t p = 1;
  for (int i = 0; i < n; ++i) {
    if (d[i] != 0 && p > INT64_MAX / d[i]) return false;
    p *= d[i];
  }
  *out = p;
  return true;
}

moa_status check_shape(moa_shape s, const char *name, int min_rank) {
  if (s.rank < min_rank || s.rank > MOA_MAX_RANK)
    return fail(MOA_ERR_RANK, "%s: rank %d outside [%d, %d]", name, s.rank, min_rank, MOA_MAX_RANK);
  if (s.rank > 0 && !s.dims) return fail(MOA_ERR_NULL, "%s: dims is NULL", name);
  for (int i = 0; i < s.rank; ++i)
    if (s.dims[i] < 0) return fail(MOA_ERR_SHAPE, "%s: extent %d is negative", name, i);
  return MOA_OK;
}

struct Flat {
  int64_t M, K, N;  // inner: M x K . K x N ; outer: NA = M, NB = N, K = 1
  int64_t nA, nB, nD;
};

moa_status flatten_inner(moa_shape a, moa_shape b, Flat *f) {
  moa_status st;
  if ((st = check_shape(a, "A", 1)) != MOA_OK) return st;
  if ((st = check_shape(b, "B", 1)) != MOA_OK) return st;
  if (a.dims[a.rank - 1] != b.dims[0])
    return fail(MOA_ERR_SHAPE, "contracted extents differ: rhoA[-1] = %lld, rhoB[0] = %lld",
                (long long)a.dims[a.rank - 1], (long long)b.dims[0]);
  if (!checked_prod(a.dims, a.rank - 1, &f->M) || !checked_prod(b.dims + 1, b.rank - 1, &f->N))
    return fail(MOA_ERR_SIZE, "element count overflows int64");
  f->K = a.dims[a.rank - 1];
  if (!checked_prod(a.dims, a.rank, &f->nA) || !checked_prod(b.dims, b.rank, &f->nB))
    return fail(MOA_ERR_SIZE, "element count overflows int64");
  if (f->N != 0 && f->M > INT64_MAX / f->N) return fail(MOA_ERR_SIZE, "result element count overflows int64");
  f->nD = f->M * f->N;
  const int64_t lim = INT64_MAX / 8;
  if (f->nA > lim || f->nB > lim || f->nD > lim) return fail(MOA_ERR_SIZE, "byte size overflows int64");
  return MOA_OK;
}

moa_status flatten_outer(moa_shape a, moa_shape b, Flat *f) {
  moa_status st;
  if ((st = check_shape(a, "A", 0)) != MOA_OK) return st;
  if ((st = check_shape(b, "B", 0)) != MOA_OK) return st;
  if (!checked_prod(a.dims, a.rank, &f->nA) || !checked_prod(b.dims, b.rank, &f->nB))
    return fail(MOA_ERR_SIZE, "element count overflows int64");
  if (f->nB != 0 && f->nA > INT64_MAX / f->nB) return fail(MOA_ERR_SIZE, "result element count overflows int64");
  f->M = f->nA;
  f->N = f->nB;
  f->K = 1;
  f->nD = f->nA * f->nB;
  const int64_t lim = INT64_MAX / 8;
  if (f->nA > lim || f->nB > lim || f->nD > lim) return fail(MOA_ERR_SIZE, "byte size overflows int64");
  return MOA_OK;
}

// Contraction of axis ax_a of A with axis ax_b of B: A is read as
// (Pa, K, Qa) and B as (Pb, K, Qb); the result is (Pa Qa) x (Pb Qb).
struct FlatAxes {
  Flat f;
  int64_t Pa, Qa, Pb, Qb;
};

moa_status flatten_axes(moa_shape a, int32_t ax_a, moa_shape b, int32_t ax_b, FlatAxes *g) {
  moa_status st;
  if ((st = check_shape(a, "A", 1)) != MOA_OK) return st;
  if ((st = check_shape(b, "B", 1)) != MOA_OK) return st;
  if (ax_a < 0 || ax_a >= a.rank) return fail(MOA_ERR_ARG, "axis %d of A outside [0, %d)", ax_a, a.rank);
  if (ax_b < 0 || ax_b >= b.rank) return fail(MOA_ERR_ARG, "axis %d of B outside [0, %d)", ax_b, b.rank);
  if (a.dims[ax_a] != b.dims[ax_b])
    return fail(MOA_ERR_SHAPE, "contracted extents differ: rhoA[%d] = %lld, rhoB[%d] = %lld", ax_a,
                (long long)a.dims[ax_a], ax_b, (long long)b.dims[ax_b]);
  Flat &f = g->f;
  if (!checked_prod(a.dims, ax_a, &g->Pa) || !checked_prod(a.dims + ax_a + 1, a.rank - ax_a - 1, &g->Qa) ||
      !checked_prod(b.dims, ax_b, &g->Pb) || !checked_prod(b.dims + ax_b + 1, b.rank - ax_b - 1, &g->Qb) ||
      !checked_prod(a.dims, a.rank, &f.nA) || !checked_prod(b.dims, b.rank, &f.nB))
    return fail(MOA_ERR_SIZE, "element count overflows int64");
  f.K = a.dims[ax_a];
  // Pa Qa <= nA and Pb Qb <= nB unless K = 0, so check those products too.
  if ((g->Qa != 0 && g->Pa > INT64_MAX / g->Qa) || (g->Qb != 0 && g->Pb > INT64_MAX / g->Qb))
    return fail(MOA_ERR_SIZE, "element count overflows int64");
  f.M = g->Pa * g->Qa;
  f.N = g->Pb * g->Qb;
  if (f.N != 0 && f.M > INT64_MAX / f.N) return fail(MOA_ERR_SIZE, "result element count overflows int64");
  f.nD = f.M * f.N;
  const int64_t lim = INT64_MAX / 8;
  if (f.nA > lim || f.nB > lim || f.nD > lim) return fail(MOA_ERR_SIZE, "byte size overflows int64");
  return MOA_OK;
}

bool overlaps(const void *p, int64_t np, const void *q, int64_t nq) {
  if (np == 0 || nq == 0 || !p || !q) return false;
  const uintptr_t a0 = (uintptr_t)p, a1 = a0 + (uintptr_t)np;
  const uintptr_t b0 = (uintptr_t)q, b1 = b0 + (uintptr_t)nq;
  return a0 < b1 && b0 < a1;
}

moa_status check_ptrs(const Flat &f, size_t es, const void *A, const void *B, const void *D) {
  if (f.nA > 0 && !A) return fail(MOA_ERR_NULL, "A is NULL");
  if (f.nB > 0 && !B) return fail(MOA_ERR_NULL, "B is NULL");
  if (f.nD > 0 && !D) return fail(MOA_ERR_NULL, "result pointer is NULL");
  const int64_t bA = f.nA * (int64_t)es, bB = f.nB * (int64_t)es, bD = f.nD * (int64_t)es;
  if (overlaps(D, bD, A, bA) || overlaps(D, bD, B, bB)) return fail(MOA_ERR_ALIAS, "result overlaps an input");
  return MOA_OK;
}


// Launch D = A (op1 . op2) B over the (Pa, K, Qa) . (Pb, K, Qb) views
// (Qa = 1, Qb = N: last axis of A with first axis of B). f.nD > 0.
moa_status run_inner(const Flat &f, int64_t Qa, int64_t Qb, const void *A, const void *B, void *D, moa_op op1,
                     moa_op op2, moa_dtype dt, uint32_t flags, hipStream_t s) {
  if (f.K == 0) return hip_status(moa::launch_fill_identity(dt, op1, D, f.nD, s), "identity fill");
  const bool plain = Qa == 1 && Qb == f.N;
  // Few result rows and long rows of B: the row-form stream reads B once.
  if (plain && f.M <= moa::kSkinnyMaxRows && f.N >= 4096)
    return hip_status(moa::launch_skinny_inner(dt, op1, op2, A, B, D, f.M, f.K, f.N, s), "inner (few rows)");
  // Few columns, association-independent fold: lanes share the fold over l.
  if (plain && moa::fewcols_applies(dt, op1, f.M, f.K, f.N))
    return hip_status(moa::launch_fewcols_inner(dt, op1, op2, A, B, D, f.M, f.K, f.N, s), "inner (few columns)");
  const bool mfma = op1 == MOA_ADD && op2 == MOA_MUL && dt != MOA_I32 && !(flags & MOA_FLAG_SEQUENTIAL_FOLD);
  if (mfma) {
    // A is M x K (Qa = 1) or K x M (Pa = 1); B is K x N (Pb = 1) or N x K (Qb = 1).
    const bool a_mat = Qa == 1 || Qa == f.M, b_mat = Qb == f.N || Qb == 1;
    if (a_mat && b_mat)
      return hip_status(moa::launch_gemm(dt, Qa != 1, Qb != f.N, A, B, D, f.M, f.K, f.N, 0, s), "inner (+,*)");
    return hip_status(moa::launch_gemm_strided(dt, A, B, D, f.M, f.K, f.N, Qa, Qb, s), "inner (+,*), strided");
  }
  return hip_status(moa::launch_simt_inner(dt, op1, op2, A, B, D, f.M, f.K, f.N, 0, s, Qa, Qb), "inner");
}

}  // namespace

extern "C" {

const char *moa_status_str(moa_status s) {
  switch (s) {
    case MOA_OK: return "MOA_OK";
    case MOA_ERR_NULL: return "MOA_ERR_NULL";
    case MOA_ERR_RANK: return "MOA_ERR_RANK";
    case MOA_ERR_SHAPE: return "MOA_ERR_SHAPE";
    case MOA_ERR_OP: return "MOA_ERR_OP";
    case MOA_ERR_DTYPE: return "MOA_ERR_DTYPE";
    case MOA_ERR_SIZE: return "MOA_ERR_SIZE";
    case MOA_ERR_ALIAS: return "MOA_ERR_ALIAS";
    case MOA_ERR_WORKSPACE: return "MOA_ERR_WORKSPACE";
    case MOA_ERR_HIP: return "MOA_ERR_HIP";
    case MOA_ERR_ARG: return "MOA_ERR_ARG";
    default: break;
  }
  return "MOA_ERR_UNKNOWN";
}

const char *moa_last_error(void) { return g_last_error.c_str(); }

int32_t moa_abi_version(void) { return MOA_ABI_VERSION; }

moa_status moa_inner_shape(moa_shape a, moa_shape b, int64_t *out_dims, int32_t *out_rank) {
  if (!out_dims || !out_rank) return fail(MOA_ERR_NULL, "output shape pointer is NULL");
  Flat f;
  moa_status st = flatten_inner(a, b, &f);
  if (st != MOA_OK) return st;
  int r = 0;
  for (int i = 0; i < a.rank - 1; ++i) out_dims[r++] = a.dims[i];
  for (int i = 1; i < b.rank; ++i) out_dims[r++] = b.dims[i];
  *out_rank = r;
  return MOA_OK;
}

moa_status moa_outer_shape(moa_shape a, moa_shape b, int64_t *out_dims, int32_t *out_rank) {
  if (!out_dims || !out_rank) return fail(MOA_ERR_NULL, "output shape pointer is NULL");
  Flat f;
  moa_status st = flatten_outer(a, b, &f);
  if (st != MOA_OK) return st;
  int r = 0;
  for (int i = 0; i < a.rank; ++i) out_dims[r++] = a.dims[i];
  for (int i = 0; i < b.rank; ++i) out_dims[r++] = b.dims[i];
  *out_rank = r;
  return MOA_OK;
}

moa_status moa_inner_ex(moa_shape sa, const void *A, moa_shape sb, const void *B, moa_op op1, moa_op op2,
                        moa_dtype dt, void *D, uint32_t flags, void *stream) {
  if (!valid_dtype(dt)) return fail(MOA_ERR_DTYPE, "unknown dtype %d", (int)dt);
  if (!is_fold_op(op1, dt)) return fail(MOA_ERR_OP, "op1 %d is not a fold operation for this dtype", (int)op1);
  if (!is_elem_op(op2, dt)) return fail(MOA_ERR_OP, "op2 %d is not defined for this dtype", (int)op2);
  if (flags & ~MOA_FLAG_SEQUENTIAL_FOLD) return fail(MOA_ERR_ARG, "unknown flags 0x%x", flags);
  Flat f;
  moa_status st = flatten_inner(sa, sb, &f);
  if (st != MOA_OK) return st;
  if ((st = check_ptrs(f, elem_size(dt), A, B, D)) != MOA_OK) return st;
  if (f.nD == 0) return MOA_OK;
  return run_inner(f, 1, f.N, A, B, D, op1, op2, dt, flags, (hipStream_t)stream);
}

moa_status moa_inner(moa_shape sa, const void *A, moa_shape sb, const void *B, moa_op op1, moa_op op2, moa_dtype dt,
                     void *D, void *stream) {
  return moa_inner_ex(sa, A, sb, B, op1, op2, dt, D, 0u, stream);
}

moa_status moa_inner_axes_shape(moa_shape a, int32_t ax_a, moa_shape b, int32_t ax_b, int64_t *out_dims,
                                int32_t *out_rank) {
  if (!out_dims || !out_rank) return fail(MOA_ERR_NULL, "output shape pointer is NULL");
  FlatAxes g;
  moa_status st = flatten_axes(a, ax_a, b, ax_b, &g);
  if (st != MOA_OK) return st;
  int r = 0;
  for (int i = 0; i < a.rank; ++i)
    if (i != ax_a) out_dims[r++] = a.dims[i];
  for (int i = 0; i < b.rank; ++i)
    if (i != ax_b) out_dims[r++] = b.dims[i];
  *out_rank = r;
  return MOA_OK;
}

moa_status moa_inner_axes(moa_shape sa, const void *A, int32_t ax_a, moa_shape sb, const void *B, int32_t ax_b,
                          moa_op op1, moa_op op2, moa_dtype dt, void *D, uint32_t flags, void *stream) {
  if (!valid_dtype(dt)) return fail(MOA_ERR_DTYPE, "unknown dtype %d", (int)dt);
  if (!is_fold_op(op1, dt)) return fail(MOA_ERR_OP, "op1 %d is not a fold operation for this dtype", (int)op1);
  if (!is_elem_op(op2, dt)) return fail(MOA_ERR_OP, "op2 %d is not defined for this dtype", (int)op2);
  if (flags & ~MOA_FLAG_SEQUENTIAL_FOLD) return fail(MOA_ERR_ARG, "unknown flags 0x%x", flags);
  FlatAxes g;
  moa_status st = flatten_axes(sa, ax_a, sb, ax_b, &g);
  if (st != MOA_OK) return st;
  if ((st = check_ptrs(g.f, elem_size(dt), A, B, D)) != MOA_OK) return st;
  if (g.f.nD == 0) return MOA_OK;
  return run_inner(g.f, g.Qa, g.Qb, A, B, D, op1, op2, dt, flags, (hipStream_t)stream);
}

moa_status moa_outer(moa_shape sa, const void *A, moa_shape sb, const void *B, moa_op op, moa_dtype dt, void *C,
                     void *stream) {
  if (!valid_dtype(dt)) return fail(MOA_ERR_DTYPE, "unknown dtype %d", (int)dt);
  if (!is_elem_op(op, dt)) return fail(MOA_ERR_OP, "op %d is not defined for this dtype", (int)op);
  Flat f;
  moa_status st = flatten_outer(sa, sb, &f);
  if (st != MOA_OK) return st;
  if ((st = check_ptrs(f, elem_size(dt), A, B, C)) != MOA_OK) return st;
  if (f.nD == 0) return MOA_OK;
  return hip_status(moa::launch_outer(dt, op, A, B, C, f.nA, f.nB, (hipStream_t)stream), "outer");
}

size_t moa_inner_split_workspace(moa_shape sa, moa_shape sb, int32_t fmt, int32_t nslices) {
  Flat f;
  if (flatten_inner(sa, sb, &f) != MOA_OK) return 0;
  moa::SplitPlan p;
  if (!moa::split_plan(f.M, f.K, f.N, fmt, nslices, &p)) return 0;
  return p.total;
}

}  // extern "C"

namespace {

// Shared validation of the split entry points. A/B/D may be NULL when the
// caller does not pass them (checked by the caller).
moa_status split_check(moa_shape sa, moa_shape sb, int32_t fmt, int32_t nslices, void *ws, size_t ws_bytes, Flat *f,
                       moa::SplitPlan *p) {
  if (fmt != MOA_SPLIT_BF16 && fmt != MOA_SPLIT_FP8 && fmt != MOA_SPLIT_INT8)
    return fail(MOA_ERR_ARG, "unknown split format %d", fmt);
  if (nslices < 1 || nslices > moa::split_max_slices(fmt))
    return fail(MOA_ERR_ARG, "nslices %d outside [1, %d] for this format", nslices, moa::split_max_slices(fmt));
  moa_status st = flatten_inner(sa, sb, f);
  if (st != MOA_OK) return st;
  if (!moa::split_plan(f->M, f->K, f->N, fmt, nslices, p)) return fail(MOA_ERR_ARG, "split plan failed");
  if (f->nD == 0 || f->K == 0) return MOA_OK;
  if (!ws) return fail(MOA_ERR_WORKSPACE, "workspace is NULL");
  if (ws_bytes < p->total) return fail(MOA_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, p->total);
  if (((uintptr_t)ws & 255) != 0) return fail(MOA_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  return MOA_OK;
}

}  // namespace

extern "C" {

moa_status moa_inner_split_prepare(moa_shape sa, const double *A, moa_shape sb, const double *B, int32_t fmt,
                                   int32_t nslices, void *ws, size_t ws_bytes, void *stream) {
  Flat f;
  moa::SplitPlan p;
  moa_status st = split_check(sa, sb, fmt, nslices, ws, ws_bytes, &f, &p);
  if (st != MOA_OK) return st;
  if (f.nA > 0 && !A) return fail(MOA_ERR_NULL, "A is NULL");
  if (f.nB > 0 && !B) return fail(MOA_ERR_NULL, "B is NULL");
  if (f.nD == 0 || f.K == 0) return MOA_OK;
  if (overlaps(ws, (int64_t)p.total, A, f.nA * 8) || overlaps(ws, (int64_t)p.total, B, f.nB * 8))
    return fail(MOA_ERR_ALIAS, "workspace overlaps an operand");
  return hip_status(moa::launch_split_prepare(p, A, B, ws, (hipStream_t)stream), "inner_split_prepare");
}

moa_status moa_inner_split_multiply(moa_shape sa, moa_shape sb, double *D, int32_t fmt, int32_t nslices, void *ws,
                                    size_t ws_bytes, void *stream) {
  Flat f;
  moa::SplitPlan p;
  moa_status st = split_check(sa, sb, fmt, nslices, ws, ws_bytes, &f, &p);
  if (st != MOA_OK) return st;
  if (f.nD > 0 && !D) return fail(MOA_ERR_NULL, "D is NULL");
  if (f.nD == 0) return MOA_OK;
  hipStream_t s = (hipStream_t)stream;
  if (f.K == 0) return hip_status(moa::launch_fill_identity(MOA_F64, MOA_ADD, D, f.nD, s), "identity fill");
  if (overlaps(ws, (int64_t)p.total, D, f.nD * 8)) return fail(MOA_ERR_ALIAS, "workspace overlaps D");
  return hip_status(moa::launch_split_multiply(p, D, ws, s), "inner_split_multiply");
}

moa_status moa_inner_split(moa_shape sa, const double *A, moa_shape sb, const double *B, double *D, int32_t fmt,
                           int32_t nslices, void *ws, size_t ws_bytes, void *stream) {
  Flat f;
  moa::SplitPlan p;
  moa_status st = split_check(sa, sb, fmt, nslices, ws, ws_bytes, &f, &p);
  if (st != MOA_OK) return st;
  if ((st = check_ptrs(f, 8, A, B, D)) != MOA_OK) return st;
  if (f.nD == 0) return MOA_OK;
  hipStream_t s = (hipStream_t)stream;
  if (f.K == 0) return hip_status(moa::launch_fill_identity(MOA_F64, MOA_ADD, D, f.nD, s), "identity fill");
  if (overlaps(ws, (int64_t)p.total, A, f.nA * 8) || overlaps(ws, (int64_t)p.total, B, f.nB * 8) ||
      overlaps(ws, (int64_t)p.total, D, f.nD * 8))
    return fail(MOA_ERR_ALIAS, "workspace overlaps an operand");
  hipError_t e = moa::launch_split_prepare(p, A, B, ws, s);
  if (e != hipSuccess) return hip_status(e, "inner_split_prepare");
  return hip_status(moa::launch_split_multiply(p, D, ws, s), "inner_split_multiply");
}

moa_status moa_inner_grad(moa_shape sa, const void *A, moa_shape sb, const void *B, const void *G, void *dA,
                          void *dB, moa_dtype dt, void *stream) {
  if (dt != MOA_F32 && dt != MOA_F64) return fail(MOA_ERR_DTYPE, "gradient needs MOA_F32 or MOA_F64");
  Flat f;
  moa_status st = flatten_inner(sa, sb, &f);
  if (st != MOA_OK) return st;
  const size_t es = elem_size(dt);
  if (f.nA > 0 && !A) return fail(MOA_ERR_NULL, "A is NULL");
  if (f.nB > 0 && !B) return fail(MOA_ERR_NULL, "B is NULL");
  if (f.nD > 0 && !G) return fail(MOA_ERR_NULL, "G is NULL");
  const int64_t bA = f.nA * (int64_t)es, bB = f.nB * (int64_t)es, bG = f.nD * (int64_t)es;
  if (dA && (overlaps(dA, bA, A, bA) || overlaps(dA, bA, B, bB) || overlaps(dA, bA, G, bG)))
    return fail(MOA_ERR_ALIAS, "dA overlaps an input");
  if (dB && (overlaps(dB, bB, A, bA) || overlaps(dB, bB, B, bB) || overlaps(dB, bB, G, bG) ||
             (dA && overlaps(dB, bB, dA, bA))))
    return fail(MOA_ERR_ALIAS, "dB overlaps an input or dA");
  hipStream_t s = (hipStream_t)stream;
  // Both gradients of a non-degenerate product: one paired launch.
  if (dA && dB && f.M > 0 && f.K > 0 && f.N > 0)
    return hip_status(moa::launch_gemm_grad(dt, G, A, B, dA, dB, f.M, f.K, f.N, s), "grad dA, dB");
  // dA (M x K) = G (M x N) . B^T, B stored K x N = (N x K)^T.
  if (dA && f.nA > 0) {
    hipError_t e = (f.N == 0) ? moa::launch_fill_identity(dt, MOA_ADD, dA, f.nA, s)
                              : moa::launch_gemm(dt, false, true, G, B, dA, f.M, f.N, f.K, 0, s);
    if (e != hipSuccess) return hip_status(e, "grad dA");
  }
  // dB (K x N) = A^T . G, A stored M x K = (K x M)^T.
  if (dB && f.nB > 0) {
    hipError_t e = (f.M == 0) ? moa::launch_fill_identity(dt, MOA_ADD, dB, f.nB, s)
                              : moa::launch_gemm(dt, true, false, A, G, dB, f.K, f.M, f.N, 0, s);
    if (e != hipSuccess) return hip_status(e, "grad dB");
  }
  return MOA_OK;
}

}  // extern "C"

// Exposed to the batch module for error reporting.
namespace moa {
moa_status set_error(moa_status st, const char *msg) { return fail(st, "%s", msg); }
moa_status validate_inner(moa_shape a, moa_shape b, int64_t *M, int64_t *K, int64_t *N) {
  Flat f;
  moa_status st = flatten_inner(a, b, &f);
  if (st != MOA_OK) return st;
  *M = f.M;
  *K = f.K;
  *N = f.N;
  return MOA_OK;
}
}  // namespace moa
