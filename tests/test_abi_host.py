"""Host-only tests of the C ABI: the library loads, exports every symbol the
header declares, and validates arguments before any launch (no GPU needed:
every call here returns before touching the device)."""
import ctypes
import os
import re
import sys

import numpy as np
import pytest

import paper_0907_0792_amd as moa
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "moa.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(moa_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = moa.lib()
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_exports_match_nm():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", moa.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (moa_[a-z0-9_]+)", out))
    assert set(_declared_functions()) <= exported


def test_abi_version_and_status_strings():
    lib = moa.lib()
    assert lib.moa_abi_version() == 1
    for i, name in enumerate(moa.STATUS):
        assert lib.moa_status_str(i).decode() == name


@pytest.mark.parametrize("sa,sb", [((2, 3), (3, 4)), ((4,), (4,)), ((2, 2, 5), (5, 1, 3)), ((7, 0), (0, 2)),
                                   ((0, 3), (3, 2)), ((1, 1, 1, 1), (1,))])
def test_inner_shape_matches_oracle(sa, sb):
    assert moa.inner_shape(sa, sb) == oracle.inner_shape(sa, sb)


@pytest.mark.parametrize("sa,sb", [((), ()), ((3,), ()), ((), (2, 2)), ((2, 3), (3, 4)), ((0,), (5, 5))])
def test_outer_shape(sa, sb):
    assert moa.outer_shape(sa, sb) == tuple(sa) + tuple(sb)


def _status(fn):
    try:
        fn()
    except moa.MoaError as e:
        return moa.STATUS[e.status]
    return "MOA_OK"


def test_shape_errors():
    assert _status(lambda: moa.inner_shape((2, 3), (4, 2))) == "MOA_ERR_SHAPE"
    assert _status(lambda: moa.inner_shape((), (3,))) == "MOA_ERR_RANK"
    assert _status(lambda: moa.inner_shape((3,), ())) == "MOA_ERR_RANK"
    assert _status(lambda: moa.inner_shape((2, -1), (-1, 2))) == "MOA_ERR_SHAPE"
    assert _status(lambda: moa.inner_shape((1,) * 17, (1,))) == "MOA_ERR_RANK"
    big = 2 ** 40
    assert _status(lambda: moa.inner_shape((big, big, 2), (2, 3))) == "MOA_ERR_SIZE"
    assert _status(lambda: moa.outer_shape((big, big), (big,))) == "MOA_ERR_SIZE"


def _call_inner(sa, pa, sb, pb, op1, op2, dt, pd, flags=0):
    L = moa.lib()
    return L.moa_inner_ex(moa._shape(sa), ctypes.c_void_p(pa), moa._shape(sb), ctypes.c_void_p(pb), op1, op2, dt,
                          ctypes.c_void_p(pd), flags, ctypes.c_void_p(0))


def test_inner_validation_before_launch():
    # Fake, never-dereferenced device addresses: validation must fail first.
    A, B, D = 0x100000, 0x200000, 0x300000
    ok_a, ok_b = (4, 8), (8, 2)
    S = moa.STATUS
    assert S[_call_inner(ok_a, A, ok_b, B, moa.OPS["sub"], moa.OPS["mul"], 0, D)] == "MOA_ERR_OP"     # op1 not a fold
    assert S[_call_inner(ok_a, A, ok_b, B, moa.OPS["div"], moa.OPS["mul"], 0, D)] == "MOA_ERR_OP"
    assert S[_call_inner(ok_a, A, ok_b, B, moa.OPS["and"], moa.OPS["mul"], 0, D)] == "MOA_ERR_OP"     # bitwise on FP
    assert S[_call_inner(ok_a, A, ok_b, B, moa.OPS["add"], moa.OPS["xor"], 1, D)] == "MOA_ERR_OP"
    assert S[_call_inner(ok_a, A, ok_b, B, moa.OPS["add"], moa.OPS["div"], 2, D)] == "MOA_ERR_OP"     # int division
    assert S[_call_inner(ok_a, A, ok_b, B, moa.OPS["add"], 42, 0, D)] == "MOA_ERR_OP"
    assert S[_call_inner(ok_a, A, ok_b, B, moa.OPS["add"], moa.OPS["mul"], 7, D)] == "MOA_ERR_DTYPE"
    assert S[_call_inner(ok_a, 0, ok_b, B, moa.OPS["add"], moa.OPS["mul"], 0, D)] == "MOA_ERR_NULL"
    assert S[_call_inner(ok_a, A, ok_b, 0, moa.OPS["add"], moa.OPS["mul"], 0, D)] == "MOA_ERR_NULL"
    assert S[_call_inner(ok_a, A, ok_b, B, moa.OPS["add"], moa.OPS["mul"], 0, 0)] == "MOA_ERR_NULL"
    assert S[_call_inner((4, 7), A, ok_b, B, moa.OPS["add"], moa.OPS["mul"], 0, D)] == "MOA_ERR_SHAPE"
    # D overlapping A (A spans 4*8*8 = 256 bytes).
    assert S[_call_inner(ok_a, A, ok_b, B, moa.OPS["add"], moa.OPS["mul"], 0, A + 128)] == "MOA_ERR_ALIAS"
    assert S[_call_inner(ok_a, A, ok_b, B, moa.OPS["add"], moa.OPS["mul"], 0, B - 8)] == "MOA_ERR_ALIAS"
    assert "overlaps" in moa.lib().moa_last_error().decode()
    assert S[_call_inner(ok_a, A, ok_b, B, moa.OPS["add"], moa.OPS["mul"], 0, D, flags=8)] == "MOA_ERR_ARG"
    # Empty result: nothing to do, no launch, even with NULL pointers for empty arrays.
    assert S[_call_inner((0, 8), 0, ok_b, B, moa.OPS["add"], moa.OPS["mul"], 0, 0)] == "MOA_OK"


def test_outer_validation():
    L = moa.lib()
    S = moa.STATUS
    sh = moa._shape
    z = ctypes.c_void_p
    assert S[L.moa_outer(sh((2,)), z(0x1000), sh((3,)), z(0x2000), moa.OPS["xor"], 0, z(0x3000), z(0))] == "MOA_ERR_OP"
    assert S[L.moa_outer(sh((2,)), z(0x1000), sh((3,)), z(0x2000), moa.OPS["div"], 2, z(0x3000), z(0))] == "MOA_ERR_OP"
    assert S[L.moa_outer(sh((2,)), z(0), sh((3,)), z(0x2000), moa.OPS["add"], 0, z(0x3000), z(0))] == "MOA_ERR_NULL"
    assert S[L.moa_outer(sh((2,)), z(0x1000), sh((3,)), z(0x2000), moa.OPS["add"], 0, z(0x1008), z(0))] == "MOA_ERR_ALIAS"
    assert S[L.moa_outer(sh((0,)), z(0), sh((3,)), z(0x2000), moa.OPS["add"], 0, z(0), z(0))] == "MOA_OK"


def test_split_workspace_and_validation():
    L = moa.lib()
    S = moa.STATUS
    n = moa.split_workspace_bytes((8192, 8192), (8192, 8192), "bf16", 5)
    # 2 operands x 5 slices x 8192^2 x 2 bytes, plus the scale vectors.
    assert n >= 2 * 5 * 8192 * 8192 * 2
    assert n < 2 * 5 * 8192 * 8192 * 2 + 4 * 8192 * 8 + 4096
    assert moa.split_workspace_bytes((3, 5), (6, 2), "bf16", 5) == 0
    assert moa.split_workspace_bytes((3, 5), (5, 2), "bf16", 9) == 0
    n8 = moa.split_workspace_bytes((8192, 8192), (8192, 8192), "int8", 7)
    assert 2 * 7 * 8192 * 8192 <= n8 < 2 * 7 * 8192 * 8192 + 4 * 8192 * 8 + 4096
    # FP8: one byte per digit, up to 10 slices; BF16 and INT8 stop at 7.
    nf = moa.split_workspace_bytes((8192, 8192), (8192, 8192), "fp8", 10)
    assert 2 * 10 * 8192 * 8192 <= nf < 2 * 10 * 8192 * 8192 + 4 * 8192 * 8 + 4096
    assert moa.split_workspace_bytes((3, 5), (5, 2), "fp8", 11) == 0
    assert moa.split_workspace_bytes((3, 5), (5, 2), "int8", 8) == 0
    assert moa.split_workspace_bytes((3, 5), (5, 2), "fp8", 8) > 0
    sh = moa._shape
    z = ctypes.c_void_p
    args = (sh((4, 8)), z(0x100000), sh((8, 2)), z(0x200000), z(0x300000))
    assert S[L.moa_inner_split(*args, 0, 0, z(0x400000), 1 << 20, z(0))] == "MOA_ERR_ARG"
    assert S[L.moa_inner_split(*args, 0, 8, z(0x400000), 1 << 20, z(0))] == "MOA_ERR_ARG"
    assert S[L.moa_inner_split(*args, 5, 5, z(0x400000), 1 << 20, z(0))] == "MOA_ERR_ARG"
    assert S[L.moa_inner_split(*args, 1, 11, z(0x400000), 1 << 20, z(0))] == "MOA_ERR_ARG"   # FP8 > 10 slices
    assert S[L.moa_inner_split(*args, 2, 8, z(0x400000), 1 << 20, z(0))] == "MOA_ERR_ARG"    # INT8 > 7 slices
    assert S[L.moa_inner_split(*args, 0, 5, z(0), 1 << 20, z(0))] == "MOA_ERR_WORKSPACE"
    assert S[L.moa_inner_split(*args, 0, 5, z(0x400000), 16, z(0))] == "MOA_ERR_WORKSPACE"
    assert S[L.moa_inner_split(*args, 0, 5, z(0x400010), 1 << 20, z(0))] == "MOA_ERR_WORKSPACE"
    assert S[L.moa_inner_split(*args, 0, 5, z(0x100000), 1 << 20, z(0))] == "MOA_ERR_ALIAS"


def test_grad_and_batch_validation():
    L = moa.lib()
    S = moa.STATUS
    sh = moa._shape
    z = ctypes.c_void_p
    assert S[L.moa_inner_grad(sh((4, 8)), z(0x1000), sh((8, 2)), z(0x2000), z(0x3000), z(0x4000), z(0x5000), 2,
                              z(0))] == "MOA_ERR_DTYPE"
    assert S[L.moa_inner_grad(sh((4, 8)), z(0x1000), sh((8, 2)), z(0x2000), z(0), z(0x4000), z(0x5000), 1,
                              z(0))] == "MOA_ERR_NULL"
    assert S[L.moa_inner_grad(sh((4, 8)), z(0x100000), sh((8, 2)), z(0x200000), z(0x300000), z(0x100010), z(0), 1,
                              z(0))] == "MOA_ERR_ALIAS"
    out = z()
    assert S[L.moa_batch_build(1, None, None, None, None, None, 1, z(0), ctypes.byref(out))] == "MOA_ERR_NULL"
    assert S[L.moa_batch_build(0, None, None, None, None, None, 2, z(0), ctypes.byref(out))] == "MOA_ERR_DTYPE"


def test_tile_table_roundtrip():
    t = moa.tile_table()
    lines = t.strip().splitlines()
    assert len(lines) == 8
    flipped = "\n".join(" ".join(l.split()[:3] + [str(1 - int(l.split()[3]))]) for l in lines)
    moa.set_tile_table(flipped)
    assert moa.tile_table().strip() == flipped.strip()
    moa.set_tile_table(t)
    assert moa.tile_table() == t
    with pytest.raises(moa.MoaError):
        moa.set_tile_table("M<=32 N<=32 K<=128 7\n")
    # Unknown tokens, a bucket set twice, a missing bucket or a trailing
    # malformed line are rejected, and the table stays as it was.
    bad_token = flipped.replace("N>32", "N>=32", 1)
    dup = "\n".join(lines[:7] + [lines[0]])
    missing = "\n".join(lines[:7])
    trailing = t + "M>32 N>32\n"
    for text in (bad_token, dup, missing, trailing, ""):
        with pytest.raises(moa.MoaError) as e:
            moa.set_tile_table(text)
        assert moa.STATUS[e.value.status] == "MOA_ERR_ARG"
        assert moa.tile_table() == t
    # Lines in any order are accepted.
    moa.set_tile_table("\n".join(reversed(lines)) + "\n")
    assert moa.tile_table() == t


def test_binding_checks_batch_result_shapes():
    # Each D[i] must hold exactly problem i's result: the library writes
    # M * N elements from its first address (shapes checked before any launch;
    # meta tensors carry shapes without memory).
    import torch
    a = torch.empty(4, 8, device="meta")
    b = torch.empty(8, 3, device="meta")
    with pytest.raises(ValueError):
        moa.Batch._check_results([a], [b], [torch.empty(4, 2, device="meta")])
    with pytest.raises(ValueError):
        moa.Batch._check_results([a], [b], [torch.empty(3, 4, device="meta")])
    moa.Batch._check_results([a], [b], [torch.empty(4, 3, device="meta")])


def test_no_cpu_fallback_when_library_missing(monkeypatch, tmp_path):
    import importlib
    monkeypatch.setattr(moa, "_lib", None)
    monkeypatch.setattr(moa, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        moa.lib()


@pytest.mark.parametrize("sa,ax_a,sb,ax_b", [((2, 3, 4), 1, (3, 2), 0), ((2, 3, 4), 0, (5, 2), 1),
                                             ((3, 2), 0, (2, 4, 3), 2), ((4,), 0, (4,), 0), ((2, 0, 3), 2, (3, 5), 0)])
def test_inner_axes_shape(sa, ax_a, sb, ax_b):
    want = oracle.inner_axes(np.zeros(sa), ax_a, np.zeros(sb), ax_b).shape
    assert moa.inner_axes_shape(sa, ax_a, sb, ax_b) == want
    # Negative axes count from the end, as in numpy.
    assert moa.inner_axes_shape(sa, ax_a - len(sa), sb, ax_b - len(sb)) == want


def test_inner_axes_validation_before_launch():
    L = moa.lib()
    S = moa.STATUS
    sh = moa._shape
    z = ctypes.c_void_p
    A, B, D = z(0x100000), z(0x200000), z(0x300000)
    add, mul = moa.OPS["add"], moa.OPS["mul"]

    def call(sa, ax_a, sb, ax_b, op1=add, op2=mul, dt=0, d=D, flags=0):
        return S[L.moa_inner_axes(sh(sa), A, ax_a, sh(sb), B, ax_b, op1, op2, dt, d, flags, z(0))]

    assert call((4, 8), 2, (4, 2), 0) == "MOA_ERR_ARG"
    assert call((4, 8), -1, (8, 2), 0) == "MOA_ERR_ARG"
    assert call((4, 8), 0, (8, 2), 0) == "MOA_ERR_SHAPE"
    assert call((4, 8), 0, (2, 4), 1, dt=9) == "MOA_ERR_DTYPE"
    assert call((4, 8), 0, (2, 4), 1, op1=moa.OPS["sub"]) == "MOA_ERR_OP"
    assert call((4, 8), 0, (2, 4), 1, flags=4) == "MOA_ERR_ARG"
    assert call((4, 8), 0, (2, 4), 1, d=z(0)) == "MOA_ERR_NULL"
    assert call((4, 8), 0, (2, 4), 1, d=z(0x100000 + 64)) == "MOA_ERR_ALIAS"
    assert call((), 0, (2, 4), 1) == "MOA_ERR_RANK"
    assert call((8, 0), 0, (2, 8), 1, d=z(0)) == "MOA_OK"      # empty result: no launch
    big = 2 ** 40
    assert call((big, 2, big), 1, (2, 3), 0) == "MOA_ERR_SIZE"


def test_inner_shape_of_two_rank16_operands():
    # The result of an inner product of two rank-16 arrays has rank 30; the
    # shape query must return all of it (out_dims holds 2 * MOA_MAX_RANK).
    sa = (1, 2, 3) + (1,) * 12 + (4,)
    sb = (4,) + (2,) * 14 + (5,)
    got = moa.inner_shape(sa, sb)
    assert got == sa[:-1] + sb[1:] and len(got) == 30
    assert moa.inner_axes_shape(sa, 15, sb, 0) == got
    assert moa.outer_shape((1,) * 16, (2,) * 16) == (1,) * 16 + (2,) * 16


def test_bench_refuses_more_than_one_gpu():
    # One GPU only: --gpus N > 1 exits with a message before touching a GPU.
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_binding_rejects_host_tensors_before_any_launch():
    # Host (CPU) tensors never reach the library: every entry checks devices first.
    import torch
    a = torch.zeros(4, 4, dtype=torch.float64)
    b = torch.zeros(4, 4, dtype=torch.float64)
    for call in (lambda: moa.inner(a, b), lambda: moa.outer(a, b), lambda: moa.inner_axes(a, b, (0, 1)),
                 lambda: moa.inner_split(a, b), lambda: moa.split_prepare(a, b, torch.zeros(64, dtype=torch.uint8)),
                 lambda: moa.split_multiply((4, 4), (4, 4), a, torch.zeros(64, dtype=torch.uint8)),
                 lambda: moa.inner_grad(a, b, a), lambda: moa.Batch([a], [b], [a.clone()])):
        with pytest.raises(ValueError):
            call()
