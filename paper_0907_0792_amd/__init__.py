"""MoA generalized inner and outer products on AMD Instinct MI355X (gfx950).

Thin Python binding of ``libmoa.so`` (C ABI in ``include/moa.h``). This module
only marshals arguments: PyTorch supplies device memory and the current HIP
stream; every step of every product runs in the library's HIP kernels. If the
library is missing or cannot be loaded, every call raises — there is no CPU
fallback.

Entry points mirror the C ABI:

* :func:`inner` / :func:`inner_ex` — generalized inner product
  ``D = A (op1 . op2) B`` (Section I, Eq. inner).
* :func:`inner_axes` — the same contraction over any axis pair, read in place.
* :func:`outer` — generalized outer product ``C = A op B`` (Section I, Eq. outer).
* :func:`inner_split` — (+,*) FP64 at FP64 accuracy from BF16 or INT8 slices
  (:func:`split_prepare` / :func:`split_multiply` run its two stages apart).
* :func:`inner_grad` — backward of the (+,*) inner product.
* :class:`Batch` — many uneven (+,*) products in one persistent graph launch.
* :class:`MoaInner` — ``torch.autograd.Function`` over inner / inner_grad.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmoa.so")

OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "max": 4, "min": 5, "and": 6, "or": 7, "xor": 8}
DTYPES = {torch.float64: 0, torch.float32: 1, torch.int32: 2}
SPLIT_FORMATS = {"bf16": 0, "fp8": 1, "int8": 2}
FLAG_SEQUENTIAL_FOLD = 1
MAX_RANK = 16

STATUS = ["MOA_OK", "MOA_ERR_NULL", "MOA_ERR_RANK", "MOA_ERR_SHAPE", "MOA_ERR_OP", "MOA_ERR_DTYPE", "MOA_ERR_SIZE",
          "MOA_ERR_ALIAS", "MOA_ERR_WORKSPACE", "MOA_ERR_HIP", "MOA_ERR_ARG"]


class MoaError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        super().__init__("%s: %s" % (name, detail))


class _Shape(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("dims", ctypes.POINTER(ctypes.c_int64))]


_lib = None


def lib():
    """The loaded ``libmoa.so`` (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmoa.so is not built: run `python -m paper_0907_0792_amd.build` (%s)" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_size_t
    S = _Shape
    L.moa_status_str.restype = ctypes.c_char_p
    L.moa_status_str.argtypes = [i32]
    L.moa_last_error.restype = ctypes.c_char_p
    L.moa_last_error.argtypes = []
    L.moa_abi_version.restype = i32
    L.moa_inner_shape.argtypes = [S, S, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.moa_outer_shape.argtypes = [S, S, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.moa_inner.argtypes = [S, vp, S, vp, i32, i32, i32, vp, vp]
    L.moa_inner_ex.argtypes = [S, vp, S, vp, i32, i32, i32, vp, u32, vp]
    L.moa_outer.argtypes = [S, vp, S, vp, i32, i32, vp, vp]
    L.moa_inner_axes_shape.argtypes = [S, i32, S, i32, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.moa_inner_axes.argtypes = [S, vp, i32, S, vp, i32, i32, i32, i32, vp, u32, vp]
    L.moa_inner_split_workspace.restype = sz
    L.moa_inner_split_workspace.argtypes = [S, S, i32, i32]
    L.moa_inner_split.argtypes = [S, vp, S, vp, vp, i32, i32, vp, sz, vp]
    L.moa_inner_split_prepare.argtypes = [S, vp, S, vp, i32, i32, vp, sz, vp]
    L.moa_inner_split_multiply.argtypes = [S, S, vp, i32, i32, vp, sz, vp]
    L.moa_inner_split_static.argtypes = [S, vp, S, vp, vp, i32, i32, vp]
    L.moa_inner_grad.argtypes = [S, vp, S, vp, vp, vp, vp, i32, vp]
    L.moa_batch_build.argtypes = [i32, ctypes.POINTER(S), ctypes.POINTER(vp), ctypes.POINTER(S), ctypes.POINTER(vp),
                                  ctypes.POINTER(vp), i32, vp, ctypes.POINTER(vp)]
    L.moa_batch_run.argtypes = [vp, vp]
    L.moa_batch_free.argtypes = [vp]
    L.moa_batch_free.restype = None
    L.moa_batch_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.moa_batch_autotune.argtypes = [i32, i32, vp]
    L.moa_tile_table_get.argtypes = [ctypes.c_char_p, sz]
    L.moa_tile_table_set.argtypes = [ctypes.c_char_p]
    for name in ("moa_inner_shape", "moa_outer_shape", "moa_inner", "moa_inner_ex", "moa_outer", "moa_inner_split",
                 "moa_inner_axes_shape", "moa_inner_axes",
                 "moa_inner_split_prepare", "moa_inner_split_multiply", "moa_inner_split_static", "moa_inner_grad", "moa_batch_build", "moa_batch_run", "moa_batch_info", "moa_batch_autotune",
                 "moa_tile_table_get", "moa_tile_table_set"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise MoaError(status, lib().moa_last_error().decode())


_SHAPES = {}


def _shape(dims):
    """moa_shape for a shape tuple. The structs are immutable once built, so
    they are cached per shape (building one costs a few microseconds, which
    small products notice)."""
    key = tuple(dims)
    s = _SHAPES.get(key)
    if s is None:
        ints = [int(d) for d in key]
        arr = (ctypes.c_int64 * max(1, len(ints)))(*ints)
        s = _Shape(len(ints), ctypes.cast(arr, ctypes.POINTER(ctypes.c_int64)))
        s._keep = arr  # keep the array alive with the struct
        if len(_SHAPES) < 4096:
            _SHAPES[key] = s
    return s


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _dev_operands(*ts):
    dev = None
    for t in ts:
        if not t.is_cuda:
            raise ValueError("operands must be device tensors")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError("operands must be on one device")
    return dev


def _check_out(out, rs, dtype, dev):
    """A caller-supplied result tensor: right shape, dtype, dense layout and
    device (the library writes rs elements from its first address)."""
    if tuple(out.shape) != tuple(rs) or out.dtype != dtype or not out.is_contiguous():
        raise ValueError("out has the wrong shape, dtype or layout")
    if not out.is_cuda or out.device != dev:
        raise ValueError("out must be on the operands' device")


_RESULT_SHAPES = {}


def _cached_shape(key, compute):
    """Result shapes come from the library's shape algebra (moa_*_shape) and
    are cached per operand-shape key, so the binding keeps no second copy of
    it and small products do not pay a shape call each."""
    rs = _RESULT_SHAPES.get(key)
    if rs is None:
        rs = compute()
        if len(_RESULT_SHAPES) < 4096:
            _RESULT_SHAPES[key] = rs
    return rs


def _shape_call(fn, *args):
    out = (ctypes.c_int64 * (2 * MAX_RANK))()
    r = ctypes.c_int32()
    _check(fn(*args, out, ctypes.byref(r)))
    return tuple(out[i] for i in range(r.value))


def inner_shape(sa, sb):
    """Result shape of Eq. inner (moa_inner_shape): rho A[:-1] ++ rho B[1:]."""
    sa, sb = tuple(sa), tuple(sb)
    return _cached_shape(("inner", sa, sb), lambda: _shape_call(lib().moa_inner_shape, _shape(sa), _shape(sb)))


def _axis(ax, rank):
    ax = int(ax)
    return ax + rank if ax < 0 else ax


def inner_axes_shape(sa, ax_a, sb, ax_b):
    """Result shape of a contraction over axes (ax_a, ax_b) (moa_inner_axes_shape)."""
    sa, sb = tuple(sa), tuple(sb)
    ax_a, ax_b = _axis(ax_a, len(sa)), _axis(ax_b, len(sb))
    return _cached_shape(("axes", sa, ax_a, sb, ax_b),
                         lambda: _shape_call(lib().moa_inner_axes_shape, _shape(sa), ax_a, _shape(sb), ax_b))


def inner_axes(a: torch.Tensor, b: torch.Tensor, axes=(-1, 0), op1: str = "add", op2: str = "mul", flags: int = 0,
               out: torch.Tensor | None = None) -> torch.Tensor:
    """Generalized inner product contracting axis axes[0] of A with axis axes[1]
    of B, read in place (Section I, Eq. inner; index maps of Section II.D).
    Axes may be negative. Result axes: A's free axes, then B's."""
    if a.dtype != b.dtype or a.dtype not in DTYPES:
        raise TypeError("operands must share dtype float64, float32 or int32")
    dev = _dev_operands(a, b)
    a = a.contiguous()
    b = b.contiguous()
    ax_a, ax_b = _axis(axes[0], a.dim()), _axis(axes[1], b.dim())
    rs = inner_axes_shape(a.shape, ax_a, b.shape, ax_b)  # A's free axes, then B's
    if out is None:
        out = torch.empty(rs, dtype=a.dtype, device=dev)
    else:
        _check_out(out, rs, a.dtype, dev)
    _check(lib().moa_inner_axes(_shape(a.shape), _ptr(a), ax_a, _shape(b.shape), _ptr(b), ax_b, OPS[op1], OPS[op2],
                                DTYPES[a.dtype], _ptr(out), flags, _stream(dev)))
    return out


def outer_shape(sa, sb):
    """Result shape of Eq. outer (moa_outer_shape): rho A ++ rho B."""
    sa, sb = tuple(sa), tuple(sb)
    return _cached_shape(("outer", sa, sb), lambda: _shape_call(lib().moa_outer_shape, _shape(sa), _shape(sb)))


def inner_ex(a: torch.Tensor, b: torch.Tensor, op1: str = "add", op2: str = "mul", flags: int = 0,
             out: torch.Tensor | None = None) -> torch.Tensor:
    if a.dtype != b.dtype or a.dtype not in DTYPES:
        raise TypeError("operands must share dtype float64, float32 or int32")
    dev = _dev_operands(a, b)
    a = a.contiguous()
    b = b.contiguous()
    rs = inner_shape(a.shape, b.shape)
    if out is None:
        out = torch.empty(rs, dtype=a.dtype, device=dev)
    else:
        _check_out(out, rs, a.dtype, dev)
    _check(lib().moa_inner_ex(_shape(a.shape), _ptr(a), _shape(b.shape), _ptr(b), OPS[op1], OPS[op2],
                              DTYPES[a.dtype], _ptr(out), flags, _stream(dev)))
    return out


def inner(a, b, op1="add", op2="mul", out=None):
    """Generalized inner product D = A (op1 . op2) B (Section I, Eq. inner)."""
    return inner_ex(a, b, op1, op2, 0, out)


def outer(a: torch.Tensor, b: torch.Tensor, op: str = "mul", out: torch.Tensor | None = None) -> torch.Tensor:
    """Generalized outer product C = A op B over rho A ++ rho B (Section I, Eq. outer)."""
    if a.dtype != b.dtype or a.dtype not in DTYPES:
        raise TypeError("operands must share dtype float64, float32 or int32")
    dev = _dev_operands(a, b)
    a = a.contiguous()
    b = b.contiguous()
    rs = outer_shape(a.shape, b.shape)
    if out is None:
        out = torch.empty(rs, dtype=a.dtype, device=dev)
    else:
        _check_out(out, rs, a.dtype, dev)
    _check(lib().moa_outer(_shape(a.shape), _ptr(a), _shape(b.shape), _ptr(b), OPS[op], DTYPES[a.dtype], _ptr(out),
                           _stream(dev)))
    return out


def split_workspace_bytes(sa, sb, fmt="bf16", nslices=5) -> int:
    return int(lib().moa_inner_split_workspace(_shape(sa), _shape(sb), SPLIT_FORMATS[fmt], nslices))


def inner_split(a: torch.Tensor, b: torch.Tensor, fmt: str = "bf16", nslices: int = 5,
                workspace: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """(+,*) FP64 inner product at FP64 accuracy from low-precision slices."""
    if a.dtype != torch.float64 or b.dtype != torch.float64:
        raise TypeError("inner_split takes float64 operands")
    dev = _dev_operands(a, b)
    a = a.contiguous()
    b = b.contiguous()
    rs = inner_shape(a.shape, b.shape)
    if out is None:
        out = torch.empty(rs, dtype=torch.float64, device=dev)
    else:
        _check_out(out, rs, torch.float64, dev)
    nbytes = split_workspace_bytes(a.shape, b.shape, fmt, nslices)
    if workspace is None:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    else:
        _check_workspace(workspace, dev)
    _check(lib().moa_inner_split(_shape(a.shape), _ptr(a), _shape(b.shape), _ptr(b), _ptr(out), SPLIT_FORMATS[fmt],
                                 nslices, ctypes.c_void_p(workspace.data_ptr()), _nbytes(workspace), _stream(dev)))
    return out


def inner_split_static(a: torch.Tensor, b: torch.Tensor, fmt: str = "bf16", nslices: int = 5,
                       out: torch.Tensor | None = None) -> torch.Tensor:
    """inner_split with the library's static scratch instead of a workspace
    (moa_inner_split_static: no device allocation inside the library)."""
    if a.dtype != torch.float64 or b.dtype != torch.float64:
        raise TypeError("inner_split_static takes float64 operands")
    dev = _dev_operands(a, b)
    a = a.contiguous()
    b = b.contiguous()
    rs = inner_shape(a.shape, b.shape)
    if out is None:
        out = torch.empty(rs, dtype=torch.float64, device=dev)
    else:
        _check_out(out, rs, torch.float64, dev)
    _check(lib().moa_inner_split_static(_shape(a.shape), _ptr(a), _shape(b.shape), _ptr(b), _ptr(out),
                                        SPLIT_FORMATS[fmt], nslices, _stream(dev)))
    return out


def _nbytes(t):
    return t.numel() * t.element_size()


def _check_workspace(workspace, dev):
    if not workspace.is_contiguous() or not workspace.is_cuda or workspace.device != dev:
        raise ValueError("workspace must be a dense tensor on the operands' device")


def split_prepare(a: torch.Tensor, b: torch.Tensor, workspace: torch.Tensor, fmt: str = "bf16", nslices: int = 5):
    """Scan and slice A and B into `workspace` (first half of inner_split)."""
    if a.dtype != torch.float64 or b.dtype != torch.float64:
        raise TypeError("split_prepare takes float64 operands")
    dev = _dev_operands(a, b)
    _check_workspace(workspace, dev)
    a = a.contiguous()
    b = b.contiguous()
    _check(lib().moa_inner_split_prepare(_shape(a.shape), _ptr(a), _shape(b.shape), _ptr(b), SPLIT_FORMATS[fmt],
                                         nslices, ctypes.c_void_p(workspace.data_ptr()), _nbytes(workspace),
                                         _stream(dev)))


def split_multiply(sa, sb, out: torch.Tensor, workspace: torch.Tensor, fmt: str = "bf16", nslices: int = 5,
                   stream=None):
    """Slice-pair products from `workspace` into `out` (second half of inner_split)."""
    dev = _dev_operands(out)
    _check_out(out, inner_shape(sa, sb), torch.float64, dev)
    _check_workspace(workspace, dev)
    st = stream if stream is not None else _stream(out.device)
    _check(lib().moa_inner_split_multiply(_shape(sa), _shape(sb), _ptr(out), SPLIT_FORMATS[fmt], nslices,
                                          ctypes.c_void_p(workspace.data_ptr()), _nbytes(workspace), st))


def inner_grad(a, b, g, need_a=True, need_b=True, out_a=None, out_b=None):
    """(dA, dB) of the (+,*) inner product for upstream gradient g.
    out_a / out_b: optional caller-supplied result tensors (dense, A's and
    B's shape and dtype, on their device)."""
    if not (a.dtype == b.dtype == g.dtype) or a.dtype not in (torch.float32, torch.float64):
        raise TypeError("inner_grad takes float32 or float64 operands")
    dev = _dev_operands(a, b, g)
    a, b, g = a.contiguous(), b.contiguous(), g.contiguous()
    if tuple(g.shape) != inner_shape(a.shape, b.shape):
        raise ValueError("g must have the result shape")
    da = db = None
    if need_a:
        da = torch.empty_like(a) if out_a is None else out_a
        _check_out(da, tuple(a.shape), a.dtype, dev)
    if need_b:
        db = torch.empty_like(b) if out_b is None else out_b
        _check_out(db, tuple(b.shape), b.dtype, dev)
    _check(lib().moa_inner_grad(_shape(a.shape), _ptr(a), _shape(b.shape), _ptr(b), _ptr(g),
                                _ptr(da) if da is not None else ctypes.c_void_p(0),
                                _ptr(db) if db is not None else ctypes.c_void_p(0), DTYPES[a.dtype], _stream(dev)))
    return da, db


class MoaInner(torch.autograd.Function):
    """Differentiable (+,*) generalized inner product with a hand-written backward.

    dA = G (+,*) B_rot and dB = A_rot (+,*) G, where B_rot moves B's first
    axis last and A_rot moves A's last axis first: both are generalized inner
    products on permuted shapes, computed by ``moa_inner_grad``.
    """

    @staticmethod
    def forward(ctx, a, b):
        ctx.save_for_backward(a, b)
        return inner(a, b, "add", "mul")

    @staticmethod
    def backward(ctx, g):
        a, b = ctx.saved_tensors
        da, db = inner_grad(a, b, g, ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        return da, db


def moa_inner(a, b):
    return MoaInner.apply(a, b)


class Batch:
    """Many uneven (+,*) inner products, built once and replayed as one graph launch."""

    def __init__(self, As, Bs, Ds, stream=None):
        n = len(As)
        if not (len(Bs) == n == len(Ds)):
            raise ValueError("A, B, D lists differ in length")
        dt = As[0].dtype if n else torch.float32
        if n:
            _dev_operands(*As, *Bs, *Ds)
        self._check_results(As, Bs, Ds)
        self._shapes = []
        sa = (_Shape * max(1, n))()
        sb = (_Shape * max(1, n))()
        pa = (ctypes.c_void_p * max(1, n))()
        pb = (ctypes.c_void_p * max(1, n))()
        pd = (ctypes.c_void_p * max(1, n))()
        for i, (a, b, d) in enumerate(zip(As, Bs, Ds)):
            if not (a.is_contiguous() and b.is_contiguous() and d.is_contiguous()):
                raise ValueError("batch tensors must be contiguous")
            if a.dtype != dt or b.dtype != dt or d.dtype != dt:
                raise TypeError("batch tensors must share one dtype")
            s1, s2 = _shape(a.shape), _shape(b.shape)
            self._shapes += [s1, s2]
            sa[i], sb[i] = s1, s2
            pa[i], pb[i], pd[i] = a.data_ptr(), b.data_ptr(), d.data_ptr()
        self._keep = (As, Bs, Ds)
        h = ctypes.c_void_p()
        st = stream if stream is not None else _stream(As[0].device if n else None)
        _check(lib().moa_batch_build(n, sa, pa, sb, pb, pd, DTYPES[dt], st, ctypes.byref(h)))
        self._h = h

    @staticmethod
    def _check_results(As, Bs, Ds):
        """The library writes the whole result of problem i from D[i]'s first
        address, so each D[i] must have exactly that result's shape."""
        for i, (a, b, d) in enumerate(zip(As, Bs, Ds)):
            rs = inner_shape(a.shape, b.shape)
            if tuple(d.shape) != rs:
                raise ValueError("D[%d] has shape %s; problem %d's result has shape %s" % (i, tuple(d.shape), i, rs))

    def run(self, stream=None):
        st = stream if stream is not None else _stream()
        _check(lib().moa_batch_run(self._h, st))

    def info(self):
        items = ctypes.c_int64()
        launches = ctypes.c_int32()
        _check(lib().moa_batch_info(self._h, ctypes.byref(items), ctypes.byref(launches)))
        return items.value, launches.value

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().moa_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_autotune(dtype=torch.float32, reps=5):
    _check(lib().moa_batch_autotune(DTYPES[dtype], reps, _stream()))
    return tile_table()


def tile_table() -> str:
    buf = ctypes.create_string_buffer(4096)
    _check(lib().moa_tile_table_get(buf, 4096))
    return buf.value.decode()


def set_tile_table(text: str):
    _check(lib().moa_tile_table_set(text.encode()))
