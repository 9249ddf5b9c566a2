"""TEST INFRASTRUCTURE ONLY: the CPU oracle for the MoA generalized products.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It never touches the HIP library and
the HIP library never touches it.

Python entry points (all host NumPy, row-major):

* :func:`inner`  — Eq. inner of Section I, op1 generalising the sum, row form.
* :func:`outer`  — Eq. outer of Section I.
* :func:`inner_dot2` — compensated (+,*) FP64 reference (Ogita-Rump-Oishi Dot2).
* :func:`split_digits`, :func:`split_inner` — the signed-digit split (Ozaki)
  scheme with exact integer slice products.
* :func:`normwise_error`, :func:`maxnorm_error`, :func:`componentwise_error`
  (with :func:`abs_product`) — the error measures results are judged by
  (normwise is the gate; the other two are reported).
* :mod:`oracle.brute` — pure-Python brute force over full index tuples.

Op names: ``add sub mul div max min and or xor``.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "max": 4, "min": 5, "and": 6, "or": 7, "xor": 8}
_DT = {np.dtype(np.float64): 0, np.dtype(np.float32): 1, np.dtype(np.int32): 2}

# Default digit widths of the split formats: a signed digit of beta bits has
# |sigma| <= 2**(beta-1), which must be an exactly representable integer in
# the slice format. BF16 (8 significand bits) holds every integer of
# magnitude <= 256, so beta = 9 fits as well (the width the GPU path uses,
# always passed explicitly); the default 8 keeps |sigma| <= 128. FP8 E4M3
# (4 significand bits) holds integers up to 16: beta = 5.
SPLIT_BETA = {"bf16": 8, "fp8": 5}

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(
            os.path.join(HERE, "moa_oracle.c")):
        from . import build as _b  # noqa: WPS433
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    i64p = ctypes.POINTER(ctypes.c_int64)
    vp = ctypes.c_void_p
    lib.oracle_inner.argtypes = [ctypes.c_int, i64p, vp, ctypes.c_int, i64p, vp, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, vp, i64p, ctypes.c_int64]
    lib.oracle_outer.argtypes = [ctypes.c_int, i64p, vp, ctypes.c_int, i64p, vp, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, vp]
    lib.oracle_dot2_inner.argtypes = [ctypes.c_int, i64p, vp, ctypes.c_int, i64p, vp, ctypes.c_int, vp, i64p,
                                      ctypes.c_int64]
    lib.oracle_split_digits.argtypes = [ctypes.c_int64, ctypes.c_int64, vp, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, vp, vp]
    lib.oracle_split_inner.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, vp, vp, ctypes.c_int,
                                       ctypes.c_int, vp, i64p, ctypes.c_int64]
    for f in (lib.oracle_inner, lib.oracle_outer, lib.oracle_dot2_inner, lib.oracle_split_digits,
              lib.oracle_split_inner):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _dims(shape):
    arr = (ctypes.c_int64 * max(1, len(shape)))(*[int(x) for x in shape])
    return arr


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _rows_arg(rows):
    if rows is None:
        return None, 0, None
    r = np.asarray(np.asarray(rows, dtype=np.int64), order="C")
    return r.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(r), r


def inner_shape(sa, sb):
    """Result shape of Eq. inner: rho A without its last axis ++ rho B without its first."""
    sa, sb = tuple(sa), tuple(sb)
    if len(sa) < 1 or len(sb) < 1 or sa[-1] != sb[0]:
        raise ValueError("inner product needs rank >= 1 operands with rhoA[-1] == rhoB[0]")
    return sa[:-1] + sb[1:]


def inner(a, b, op1="add", op2="mul", mode="wide", rows=None):
    """Generalized inner product by the oracle.

    mode: for FP32 inputs, ``"wide"`` folds in FP64 (returns FP64) and
    ``"native"`` rounds each operation to FP32 (returns FP32). FP64 and int32
    inputs are always computed in their own type.
    rows: optional flat indices into rho A without its last axis; the result
    is then those rows only, shape (len(rows),) + rho B[1:].
    """
    a = np.asarray(a, order="C")
    b = np.asarray(b, order="C")
    if a.dtype != b.dtype or a.dtype not in _DT:
        raise TypeError("operands must share dtype float64, float32 or int32")
    dt = _DT[a.dtype]
    md = 1 if mode == "native" else 0
    rs = inner_shape(a.shape, b.shape)
    M = math.prod(a.shape[:-1])
    N = math.prod(b.shape[1:])
    out_dt = a.dtype if (dt != 1 or md == 1) else np.dtype(np.float64)
    rp, nr, keep = _rows_arg(rows)
    out = np.empty((nr if rows is not None else M) * N, dtype=out_dt)
    rc = _load().oracle_inner(a.ndim, _dims(a.shape), _ptr(a), b.ndim, _dims(b.shape), _ptr(b), OPS[op1], OPS[op2],
                              dt, md, _ptr(out), rp, nr)
    if rc != 0:
        raise ValueError("oracle_inner rejected the arguments")
    if rows is not None:
        return out.reshape((nr,) + tuple(b.shape[1:]))
    return out.reshape(rs)


def inner_axes(a, ax_a, b, ax_b, op1="add", op2="mul", mode="wide", rows=None):
    """Eq. inner contracted over axis ax_a of A and axis ax_b of B (Section I:
    the inner product as a tensor contraction over a chosen index pair).
    Definition: move the contracted axis of A to the end and that of B to the
    front (a transposition, no arithmetic), then the last-with-first product.
    Result axes: A's free axes, then B's; ``rows`` indexes A's free part."""
    a = np.asarray(a, order="C")
    b = np.asarray(b, order="C")
    if a.ndim < 1 or b.ndim < 1:
        raise ValueError("inner product needs rank >= 1 operands")
    ax_a = ax_a + a.ndim if ax_a < 0 else ax_a
    ax_b = ax_b + b.ndim if ax_b < 0 else ax_b
    if not (0 <= ax_a < a.ndim and 0 <= ax_b < b.ndim):
        raise ValueError("axis out of range")
    return inner(np.moveaxis(a, ax_a, -1), np.moveaxis(b, ax_b, 0), op1, op2, mode, rows)


def outer(a, b, op="mul", mode="native"):
    """Generalized outer product C[i ++ j] = A[i] op B[j]. FP32 inputs give
    FP32 (each element one correctly rounded FP32 op) unless mode="wide"."""
    a = np.asarray(a, order="C")
    b = np.asarray(b, order="C")
    if a.dtype != b.dtype or a.dtype not in _DT:
        raise TypeError("operands must share dtype float64, float32 or int32")
    dt = _DT[a.dtype]
    md = 1 if mode == "native" else 0
    out_dt = a.dtype if (dt != 1 or md == 1) else np.dtype(np.float64)
    out = np.empty(a.size * b.size, dtype=out_dt)
    rc = _load().oracle_outer(a.ndim, _dims(a.shape), _ptr(a), b.ndim, _dims(b.shape), _ptr(b), OPS[op], dt, md,
                              _ptr(out))
    if rc != 0:
        raise ValueError("oracle_outer rejected the arguments")
    return out.reshape(tuple(a.shape) + tuple(b.shape))


def inner_dot2(a, b, rows=None):
    """Compensated (+,*) inner product in FP64 (Dot2); FP32 inputs are widened."""
    a = np.asarray(a, order="C")
    b = np.asarray(b, order="C")
    if a.dtype != b.dtype or a.dtype not in (np.float64, np.float32):
        raise TypeError("Dot2 oracle takes float64 or float32 operands")
    rs = inner_shape(a.shape, b.shape)
    M = math.prod(a.shape[:-1])
    N = math.prod(b.shape[1:])
    rp, nr, keep = _rows_arg(rows)
    out = np.empty((nr if rows is not None else M) * N, dtype=np.float64)
    rc = _load().oracle_dot2_inner(a.ndim, _dims(a.shape), _ptr(a), b.ndim, _dims(b.shape), _ptr(b),
                                   _DT[a.dtype], _ptr(out), rp, nr)
    if rc != 0:
        raise ValueError("oracle_dot2_inner rejected the arguments")
    if rows is not None:
        return out.reshape((nr,) + tuple(b.shape[1:]))
    return out.reshape(rs)


def split_digits(x, by_rows=True, fmt="bf16", nslices=6, beta=None):
    """Signed digits of a 2-D FP64 matrix scaled per row (or per column).

    Returns (exponents int32, digits int32 of shape (nslices,) + x.shape).
    """
    x = np.asarray(x, dtype=np.float64, order="C")
    if x.ndim != 2:
        raise ValueError("split_digits takes a matrix")
    beta = beta or SPLIT_BETA[fmt]
    rows, cols = x.shape
    exps = np.empty(rows if by_rows else cols, dtype=np.int32)
    sig = np.empty((nslices, rows, cols), dtype=np.int32)
    rc = _load().oracle_split_digits(rows, cols, _ptr(x), 1 if by_rows else 0, beta, nslices, _ptr(exps), _ptr(sig))
    if rc != 0:
        raise ValueError("oracle_split_digits rejected the arguments")
    return exps, sig


def split_inner(a, b, fmt="bf16", nslices=6, rows=None, beta=None):
    """(+,*) FP64 inner product by the triangular signed-digit split scheme.

    The operands may have any rank; they are flattened to M x K and K x N.
    """
    a = np.asarray(a, dtype=np.float64, order="C")
    b = np.asarray(b, dtype=np.float64, order="C")
    rs = inner_shape(a.shape, b.shape)
    K = a.shape[-1]
    M = math.prod(a.shape[:-1])
    N = math.prod(b.shape[1:])
    beta = beta or SPLIT_BETA[fmt]
    rp, nr, keep = _rows_arg(rows)
    out = np.empty((nr if rows is not None else M) * N, dtype=np.float64)
    rc = _load().oracle_split_inner(M, K, N, _ptr(a), _ptr(b), beta, nslices, _ptr(out), rp, nr)
    if rc != 0:
        raise ValueError("oracle_split_inner rejected the arguments")
    if rows is not None:
        return out.reshape((nr,) + tuple(b.shape[1:]))
    return out.reshape(rs)


def identity_of(op, dtype):
    """Identity element of op1 (the value of an empty fold)."""
    dtype = np.dtype(dtype)
    if dtype == np.int32:
        return {"add": 0, "mul": 1, "max": -2**31, "min": 2**31 - 1, "and": -1, "or": 0, "xor": 0}[op]
    return {"add": 0.0, "mul": 1.0, "max": -np.inf, "min": np.inf}[op]


def normwise_error(x, ref):
    """||x - ref||_F / ||ref||_F in FP64."""
    x = np.asarray(x, dtype=np.float64, order="C")
    ref = np.asarray(ref, dtype=np.float64, order="C")
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((x - ref).ravel())
    return float(num / den) if den > 0 else float(num)


def maxnorm_error(x, ref):
    """max |x - ref| / max |ref| in FP64."""
    x = np.asarray(x, dtype=np.float64, order="C")
    ref = np.asarray(ref, dtype=np.float64, order="C")
    den = float(np.abs(ref).max()) if ref.size else 0.0
    num = float(np.abs(x - ref).max()) if ref.size else 0.0
    return num / den if den > 0 else num


def abs_product(a, b, rows=None):
    """(|A| (+,*) |B|) in FP64: the scale of a (+,*) result's rounding error,
    element by element (Eq. inner with both operands replaced by their
    magnitudes). rows: as for :func:`inner`."""
    a = np.abs(np.asarray(a, dtype=np.float64, order="C"))
    b = np.abs(np.asarray(b, dtype=np.float64, order="C"))
    return inner(a, b, "add", "mul", rows=rows)


def componentwise_error(x, ref, scale):
    """max over elements of |x - ref| / scale, with scale = abs_product(A, B)
    of the same elements. Where scale is 0 the result is exactly 0, so any
    difference there gives inf."""
    x = np.asarray(x, dtype=np.float64, order="C")
    ref = np.asarray(ref, dtype=np.float64, order="C")
    scale = np.asarray(scale, dtype=np.float64, order="C")
    d = np.abs(x - ref)
    if not d.size:
        return 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(scale > 0, d / np.where(scale > 0, scale, 1.0), np.where(d > 0, np.inf, 0.0))
    return float(r.max())
