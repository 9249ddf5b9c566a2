"""TEST INFRASTRUCTURE ONLY: pure-Python brute force of Eq. outer and Eq. inner.

Every element of the result is computed from its full index tuple, straight
from the component formulas of Section I:

    C[i ++ j] = A[i] op B[j]
    D[i ++ j] = fold over p of op1, of A[i ++ <p>] op2 B[<p> ++ j]

Arithmetic uses Python ints (int32 wrap applied after each operation),
Python floats for FP64, and NumPy float32 scalars for FP32 (so every FP32
operation is NumPy's own IEEE single-precision operation, independent of how
the C oracle forms it). For tiny inputs only.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _wrap32(v: int) -> int:
    v &= 0xFFFFFFFF
    return v - (1 << 32) if v >= (1 << 31) else v


def _fkey(x):
    # Order of the IEEE 754-2019 maximum / minimum on non-NaN values: by
    # value, and -0 before +0.
    return (float(x), math.copysign(1.0, float(x)))


def _fmax(a, b):
    if math.isnan(a) or math.isnan(b):
        return a + b  # a NaN
    return a if _fkey(a) >= _fkey(b) else b


def _fmin(a, b):
    if math.isnan(a) or math.isnan(b):
        return a + b
    return a if _fkey(a) <= _fkey(b) else b


def _apply(op, a, b, kind):
    if kind == "i":
        if op == "add":
            return _wrap32(a + b)
        if op == "sub":
            return _wrap32(a - b)
        if op == "mul":
            return _wrap32(a * b)
        if op == "max":
            return b if a < b else a
        if op == "min":
            return b if b < a else a
        if op == "and":
            return _wrap32(a & b)
        if op == "or":
            return _wrap32(a | b)
        if op == "xor":
            return _wrap32(a ^ b)
        raise ValueError(op)
    if kind == "f32":
        a, b = np.float32(a), np.float32(b)
        with np.errstate(all="ignore"):
            if op == "add":
                return np.float32(a + b)
            if op == "sub":
                return np.float32(a - b)
            if op == "mul":
                return np.float32(a * b)
            if op == "div":
                return np.float32(a / b)
            if op == "max":
                return _fmax(a, b)
            if op == "min":
                return _fmin(a, b)
        raise ValueError(op)
    if op == "add":
        r = a + b
    elif op == "sub":
        r = a - b
    elif op == "mul":
        r = a * b
    elif op == "div":
        r = a / b if b != 0 else (math.copysign(math.inf, a) * math.copysign(1.0, b) if a != 0 else math.nan)
    elif op == "max":
        r = _fmax(a, b)
    elif op == "min":
        r = _fmin(a, b)
    else:
        raise ValueError(op)
    return r


def _kind(dtype):
    dtype = np.dtype(dtype)
    if dtype == np.int32:
        return "i"
    if dtype == np.float32:
        return "f32"
    return "f64"


def _elem(x: np.ndarray, idx):
    v = x[tuple(idx)] if x.ndim else x[()]
    if x.dtype == np.int32:
        return int(v)
    if x.dtype == np.float32:
        return np.float32(v)
    return float(v)


def outer(a: np.ndarray, b: np.ndarray, op: str) -> np.ndarray:
    kind = _kind(a.dtype)
    out = np.empty(tuple(a.shape) + tuple(b.shape), dtype=a.dtype)
    for i in itertools.product(*[range(n) for n in a.shape]):
        for j in itertools.product(*[range(n) for n in b.shape]):
            out[tuple(i) + tuple(j)] = _apply(op, _elem(a, i), _elem(b, j), kind)
    return out


def inner(a: np.ndarray, b: np.ndarray, op1: str, op2: str, identity=None) -> np.ndarray:
    kind = _kind(a.dtype)
    assert a.ndim >= 1 and b.ndim >= 1 and a.shape[-1] == b.shape[0]
    K = a.shape[-1]
    out = np.empty(tuple(a.shape[:-1]) + tuple(b.shape[1:]), dtype=a.dtype)
    for i in itertools.product(*[range(n) for n in a.shape[:-1]]):
        for j in itertools.product(*[range(n) for n in b.shape[1:]]):
            if K == 0:
                acc = identity
            else:
                acc = None
                for p in range(K):
                    t = _apply(op2, _elem(a, tuple(i) + (p,)), _elem(b, (p,) + tuple(j)), kind)
                    acc = t if acc is None else _apply(op1, acc, t, kind)
            out[tuple(i) + tuple(j)] = acc
    return out


def inner_axes(a: np.ndarray, ax_a: int, b: np.ndarray, ax_b: int, op1: str, op2: str, identity=None) -> np.ndarray:
    """Eq. inner contracted over axis ax_a of A and ax_b of B: every result
    element is built from its free index tuples with p inserted at the
    contracted positions."""
    kind = _kind(a.dtype)
    assert a.shape[ax_a] == b.shape[ax_b]
    K = a.shape[ax_a]
    fa = [n for d, n in enumerate(a.shape) if d != ax_a]
    fb = [n for d, n in enumerate(b.shape) if d != ax_b]
    out = np.empty(tuple(fa) + tuple(fb), dtype=a.dtype)
    for i in itertools.product(*[range(n) for n in fa]):
        for j in itertools.product(*[range(n) for n in fb]):
            acc = identity
            for p in range(K):
                ia = tuple(i[:ax_a]) + (p,) + tuple(i[ax_a:])
                jb = tuple(j[:ax_b]) + (p,) + tuple(j[ax_b:])
                t = _apply(op2, _elem(a, ia), _elem(b, jb), kind)
                acc = t if p == 0 else _apply(op1, acc, t, kind)
            out[tuple(i) + tuple(j)] = acc
    return out
