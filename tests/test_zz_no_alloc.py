"""GPU test of moa_inner_split_static (no workspace, no allocation): through
the C ABI, against moa_inner_split with a caller workspace on the same inputs
(the same kernels, so the same bits), on two calls in a row with the second
one smaller, for BF16 and INT8 slices."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import moa_inputs as mi
import oracle
import paper_0907_0792_amd as moa

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
BAND = 4096
SENTINEL = 0xA5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _guarded_out(shape):
    n = int(np.prod(shape)) * 8
    raw = torch.full((2 * BAND + n,), SENTINEL, dtype=torch.uint8, device=DEV)
    raw[BAND:BAND + n].fill_(0xFF)
    return raw, raw[BAND:BAND + n].view(torch.float64).view(shape)


def _bands_intact(raw):
    torch.cuda.synchronize()
    return bool((raw[:BAND] == SENTINEL).all()) and bool((raw[-BAND:] == SENTINEL).all())


def _static_call(ga, gb, out, fmt, S):
    L = moa.lib()
    st = L.moa_inner_split_static(moa._shape(ga.shape), ctypes.c_void_p(ga.data_ptr()), moa._shape(gb.shape),
                                  ctypes.c_void_p(gb.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  moa.SPLIT_FORMATS[fmt], S,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return moa.STATUS[st]


def _bits_equal(x, y):
    return x.shape == y.shape and np.array_equal(x.view(np.uint64), y.view(np.uint64))


@pytest.mark.parametrize("fmt,S,beta", [("bf16", 5, 9), ("int8", 7, 7)])
def test_static_scratch_matches_workspace_entry_point(fmt, S, beta):
    rng = np.random.default_rng(190)
    # The second call is smaller and reuses the scratch the first one left.
    for M, K, N in [(1100, 1300, 900), (130, 260, 70)]:
        a = mi.scaled_f64(rng, (M, K))
        b = mi.scaled_f64(rng, (K, N))
        ga, gb = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)
        say("static split", fmt, M, K, N)
        raw, out = _guarded_out((M, N))
        assert _static_call(ga, gb, out, fmt, S) == "MOA_OK", moa.lib().moa_last_error()
        assert _bands_intact(raw)
        got = out.cpu().numpy()
        want = moa.inner_split(ga, gb, fmt, S).cpu().numpy()
        assert _bits_equal(got, want)
        rows = np.unique(np.concatenate([[0, M - 1], rng.choice(M, 8, replace=False)]))
        # The same kernels as moa_inner_split: 5 BF16 slices sum levels 3 and
        # 4 in one FP32 accumulator (about 3e-14 from the exact scheme).
        tol = 2e-13 if fmt == "bf16" else 1e-14
        assert oracle.normwise_error(got[rows], oracle.split_inner(a, b, nslices=S, beta=beta, rows=rows)) <= tol
        assert oracle.normwise_error(got[rows], oracle.inner_dot2(a, b, rows=rows)) <= 1e-12


def test_static_scratch_refuses_problems_beyond_its_size():
    # Refused on the host before any launch: D keeps its sentinel contents.
    need = moa.split_workspace_bytes((4000, 4000), (4000, 4000), "bf16", 5)
    assert need > (128 << 20)
    L = moa.lib()
    ga = torch.zeros(4000, 4000, dtype=torch.float64, device=DEV)
    gb = torch.zeros(4000, 4000, dtype=torch.float64, device=DEV)
    out = torch.full((4000, 4000), 7.0, dtype=torch.float64, device=DEV)
    assert _static_call(ga, gb, out, "bf16", 5) == "MOA_ERR_WORKSPACE"
    assert "static scratch" in L.moa_last_error().decode()
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    # Argument errors are the workspace entry point's.
    assert _static_call(ga[:10, :7], gb[:8, :5], out[:10, :5], "bf16", 5) == "MOA_ERR_SHAPE"
    assert _static_call(ga[:10, :8], gb[:8, :5], out[:10, :5], "bf16", 0) == "MOA_ERR_ARG"
