"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bit-exact for int32, tropical, outer products and sequential-fold FP pairs;
normwise tolerances for the matrix-core (+,*) paths:
  FP64 (+,*)          ||D - D*||_F / ||D*||_F <= 1e-13   (D* = Dot2 reference)
  FP32 (+,*)          <= 1e-5
  split BF16, S = 5   <= 1e-12 against Dot2 (the FP64-accuracy bound), and
                      against the oracle's own split scheme (same digits,
                      same kept pairs) <= scheme_tol(fmt, S): 1e-14 where the
                      GPU sums every level exactly, 2e-13 for 5 BF16 slices,
                      whose kernel sums levels 3 and 4 in one FP32
                      accumulator (about 3e-14 measured)
Full-size workloads are checked on sampled rows the oracle computes one by one.
"""
import math
import sys

import numpy as np
import pytest
import torch

import moa_inputs as mi
import oracle
import paper_0907_0792_amd as moa

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")

FOLD_F = ["add", "mul", "max", "min"]
ELEM_F = ["add", "sub", "mul", "div", "max", "min"]
FOLD_I = ["add", "mul", "max", "min", "and", "or", "xor"]
ELEM_I = ["add", "sub", "mul", "max", "min", "and", "or", "xor"]


# ---------------------------------------------------------------------------
# Every result (and every split workspace) the tests request lies between
# sentinel bands of BAND bytes; after each call the bands must be intact, so
# a store past either end of an output fails the test. The result itself is
# pre-filled with 0xFF bytes (NaN for FP, -1 for int32), so an element a
# kernel never writes shows up in the comparison.

BAND = 4096
SENTINEL = 0xA5
UNWRITTEN = 0xFF


class GuardPool:
    """Buffers of the given (shape, dtype) laid out in one allocation, each
    with BAND sentinel bytes before and after it (offsets 256-byte aligned)."""

    def __init__(self, specs, fill=UNWRITTEN):
        offs, pos = [], BAND
        sizes = []
        for shape, dtype in specs:
            nb = math.prod(tuple(int(d) for d in shape)) * torch.empty((), dtype=dtype).element_size()
            offs.append(pos)
            sizes.append(nb)
            pos += (nb + 255) // 256 * 256 + BAND
        self.raw = torch.full((pos,), SENTINEL, dtype=torch.uint8, device=DEV)
        self.t = []
        # Byte ranges outside every buffer: the bands, plus each buffer's
        # padding up to the next 256-byte boundary.
        self.bands = []
        prev = 0
        for (shape, dtype), off, nb in zip(specs, offs, sizes):
            self.raw[off:off + nb].fill_(fill)
            self.t.append(self.raw[off:off + nb].view(dtype).view(tuple(int(d) for d in shape)))
            self.bands.append((prev, off))
            prev = off + nb
        self.bands.append((prev, pos))
        idx = torch.cat([torch.arange(a, b, dtype=torch.int64) for a, b in self.bands])
        self.idx = idx.to(DEV)

    def check(self, what):
        torch.cuda.synchronize()
        bad = self.raw[self.idx] != SENTINEL
        if bool(bad.any()):
            first = int(self.idx[torch.nonzero(bad)[0, 0]])
            raise AssertionError("%s wrote %d bytes outside its buffers (first at byte %d of %d)"
                                 % (what, int(bad.sum()), first, self.raw.numel()))


def guarded(shape, dtype, fill=UNWRITTEN):
    p = GuardPool([(shape, dtype)], fill)
    return p, p.t[0]


class _Guarded:
    """The binding's entry points with guarded results: same names and
    arguments, every output between sentinel bands, bands checked after each
    call (which also synchronises)."""

    def inner_ex(self, a, b, op1="add", op2="mul", flags=0):
        p, out = guarded(moa.inner_shape(a.shape, b.shape), a.dtype)
        moa.inner_ex(a, b, op1, op2, flags, out=out)
        p.check("inner %s . %s (%s, %s)" % (tuple(a.shape), tuple(b.shape), op1, op2))
        return out

    def inner(self, a, b, op1="add", op2="mul"):
        return self.inner_ex(a, b, op1, op2, 0)

    def outer(self, a, b, op="mul"):
        p, out = guarded(moa.outer_shape(a.shape, b.shape), a.dtype)
        moa.outer(a, b, op, out=out)
        p.check("outer %s o %s (%s)" % (tuple(a.shape), tuple(b.shape), op))
        return out

    def inner_axes(self, a, b, axes=(-1, 0), op1="add", op2="mul", flags=0):
        p, out = guarded(moa.inner_axes_shape(a.shape, axes[0], b.shape, axes[1]), a.dtype)
        moa.inner_axes(a, b, axes, op1, op2, flags, out=out)
        p.check("inner_axes %s . %s over %s" % (tuple(a.shape), tuple(b.shape), tuple(axes)))
        return out

    def inner_split(self, a, b, fmt="bf16", nslices=5):
        nb = max(1, moa.split_workspace_bytes(a.shape, b.shape, fmt, nslices))
        p = GuardPool([(moa.inner_shape(a.shape, b.shape), torch.float64), ((nb,), torch.uint8)])
        p.t[1].fill_(0x3C)  # workspace contents on entry are ignored
        moa.inner_split(a, b, fmt, nslices, workspace=p.t[1], out=p.t[0])
        p.check("inner_split %s . %s (%s, S=%d)" % (tuple(a.shape), tuple(b.shape), fmt, nslices))
        return p.t[0]

    def inner_grad(self, a, b, g, need_a=True, need_b=True):
        p = GuardPool([(a.shape, a.dtype), (b.shape, b.dtype)])
        da, db = moa.inner_grad(a, b, g, need_a, need_b, out_a=p.t[0] if need_a else None,
                                out_b=p.t[1] if need_b else None)
        p.check("inner_grad %s . %s" % (tuple(a.shape), tuple(b.shape)))
        return da, db


G = _Guarded()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu(x):
    # np.asarray keeps 0-d arrays 0-d (ascontiguousarray would make them 1-d).
    return torch.from_numpy(np.asarray(x, order="C")).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def eq(x, y):
    """Bit for bit (+0 and -0 differ); any NaN matches any NaN, since NaN
    payloads are not specified."""
    x = np.asarray(x)
    y = np.asarray(y)
    assert x.shape == y.shape, (x.shape, y.shape)
    assert x.dtype == y.dtype, (x.dtype, y.dtype)
    if x.dtype.kind == "f":
        u = np.dtype("u%d" % x.dtype.itemsize)
        nan = np.isnan(x) & np.isnan(y)
        bad = ~((x.view(u) == y.view(u)) | nan)
        assert not bad.any(), "mismatch at %s: %r vs %r" % (np.argwhere(bad)[0], x[bad][0], y[bad][0])
    else:
        assert np.array_equal(x, y), "mismatch at %s" % (np.argwhere(x != y)[0],)


def nerr(x, ref):
    return oracle.normwise_error(x, ref)


def scheme_tol(fmt, S):
    """Normwise tolerance of a GPU split result against the oracle's exact
    evaluation of the same scheme. The kernels sum each level exactly (FP32
    while exact, INT32, FP64 folds), except 5 BF16 slices: there levels 3 and
    4 share one FP32 accumulator per 256 k, rounded to 2^-24 of a level-3 sum
    (weight 2^-27 against level 0), which on these inputs moves the result by
    about 3e-14 of its norm."""
    return 2e-13 if (fmt == "bf16" and S == 5) else 1e-14


def rand(rng, shape, dt):
    if dt == np.int32:
        return mi.uniform_i32(rng, shape, -60, 60)
    x = rng.uniform(0.5, 2.0, size=shape) * rng.choice([-1.0, 1.0], size=shape)
    return np.asarray(x, dtype=dt, order="C")


# ---------------------------------------------------------------------------

def test_worked_example():
    say("worked example 2x3 . 3x4")
    for dt in (np.float64, np.float32, np.int32):
        a = np.arange(6, dtype=dt).reshape(2, 3)
        b = np.arange(12, dtype=dt).reshape(3, 4)
        eq(host(G.inner(gpu(a), gpu(b))), np.array([[20, 23, 26, 29], [56, 68, 80, 92]], dtype=dt))
        eq(host(G.inner(gpu(a), gpu(b), "max", "add")), np.array([[10, 11, 12, 13], [13, 14, 15, 16]], dtype=dt))
        eq(host(G.outer(gpu(a), gpu(b), "mul")), oracle.outer(a, b, "mul"))


SIMT_SHAPES = [
    ((19,), (19,)),                 # rank-0 result
    ((37, 19), (19, 53)),           # ragged, below one tile
    ((3, 4, 5), (5, 2, 7)),
    ((1, 1), (1, 1)),
    ((6, 1), (1, 9)),               # K = 1
    ((133, 21), (21, 70)),          # several 32/64 tiles and a tail
]


@pytest.mark.parametrize("dt", [np.int32, np.float64, np.float32])
def test_simt_all_op_pairs_bit_exact(dt):
    rng = np.random.default_rng(100)
    folds = FOLD_I if dt == np.int32 else FOLD_F
    elems = ELEM_I if dt == np.int32 else ELEM_F
    for sa, sb in SIMT_SHAPES:
        a = rand(rng, sa, dt)
        b = rand(rng, sb, dt)
        ga, gb = gpu(a), gpu(b)
        for op1 in folds:
            for op2 in elems:
                say("simt", np.dtype(dt).name, sa, sb, op1, op2)
                d = G.inner_ex(ga, gb, op1, op2, flags=moa.FLAG_SEQUENTIAL_FOLD)
                eq(host(d), oracle.inner(a, b, op1, op2, mode="native"))


@pytest.mark.parametrize("tile", [(300, 40, 260), (513, 33, 129), (1100, 20, 1030)])
def test_simt_tiles_and_tails(tile):
    # Sizes that select each register-block variant with ragged edges.
    M, K, N = tile
    rng = np.random.default_rng(101)
    a = mi.uniform_i32(rng, (M, K))
    b = mi.uniform_i32(rng, (K, N))
    for op1, op2 in (("max", "add"), ("min", "sub"), ("add", "mul"), ("xor", "and")):
        say("simt tile", tile, op1, op2)
        eq(host(G.inner(gpu(a), gpu(b), op1, op2)), oracle.inner(a, b, op1, op2))
    af = rand(rng, (M, K), np.float32)
    bf = rand(rng, (K, N), np.float32)
    say("simt tile f32 (+,-)", tile)
    eq(host(G.inner(gpu(af), gpu(bf), "add", "sub")), oracle.inner(af, bf, "add", "sub", mode="native"))


@pytest.mark.parametrize("dt", [np.int32, np.float64, np.float32])
def test_simt_vector_staging_ragged_and_misaligned(dt):
    # K and N multiples of 4: 16-byte staging loads, ragged M and N edges;
    # the same operands one element past a 16-byte boundary: scalar loads.
    rng = np.random.default_rng(114)
    pairs = [("max", "add"), ("min", "sub")] + ([("xor", "and")] if dt == np.int32 else [("add", "mul")])
    for M, K, N in [(300, 40, 260), (1030, 64, 200), (70, 36, 4)]:
        a = rand(rng, (M, K), dt)
        b = rand(rng, (K, N), dt)
        ta = torch.zeros(a.size + 1, dtype=gpu(a).dtype, device=DEV)
        ta[1:] = gpu(a.ravel())
        av = ta[1:].view(M, K)
        assert av.data_ptr() % 16 != 0
        for op1, op2 in pairs:
            ref = oracle.inner(a, b, op1, op2, mode="native")
            for name, ga in (("aligned", gpu(a)), ("misaligned", av)):
                say("simt staging", name, np.dtype(dt).name, M, K, N, op1, op2)
                eq(host(G.inner_ex(ga, gpu(b), op1, op2, flags=moa.FLAG_SEQUENTIAL_FOLD)), ref)


@pytest.mark.parametrize("dt", [np.float64, np.float32, np.int32])
def test_few_rows_stream_all_pairs_bit_exact(dt):
    # At most 8 result rows and >= 4096 columns: the row-form stream kernel,
    # ascending fold for every pair, (+,*) included.
    rng = np.random.default_rng(109)
    folds = FOLD_I if dt == np.int32 else FOLD_F
    elems = ELEM_I if dt == np.int32 else ELEM_F
    for M, K, N in [(1, 128, 4096), (3, 37, 5003), (8, 5, 4100), (2, 1, 8192)]:
        a = rand(rng, (M, K), dt)
        b = rand(rng, (K, N), dt)
        ga, gb = gpu(a), gpu(b)
        for op1 in folds:
            for op2 in elems:
                say("few rows", np.dtype(dt).name, M, K, N, op1, op2)
                eq(host(G.inner(ga, gb, op1, op2)), oracle.inner(a, b, op1, op2, mode="native"))


@pytest.mark.parametrize("dt", [np.float64, np.float32, np.int32])
def test_few_rows_wide_runs_ragged(dt):
    # Rows long enough for four 16-byte runs per thread, with a partial last
    # workgroup (N not a multiple of its span) and with unaligned rows
    # (N not a multiple of the vector width: scalar loads everywhere).
    rng = np.random.default_rng(110)
    vec = 16 // np.dtype(dt).itemsize
    span = 256 * vec * 4
    base = 512 * span
    for M, K, N in [(3, 5, base + vec), (4, 3, base + span + 1), (1, 2, base)]:
        a = rand(rng, (M, K), dt)
        b = rand(rng, (K, N), dt)
        ga, gb = gpu(a), gpu(b)
        for op1, op2 in ([("add", "mul"), ("max", "add"), ("xor", "and")] if dt == np.int32 else
                         [("add", "mul"), ("max", "add"), ("min", "div")]):
            say("few rows wide", np.dtype(dt).name, M, K, N, op1, op2)
            eq(host(G.inner(ga, gb, op1, op2)), oracle.inner(a, b, op1, op2, mode="native"))


@pytest.mark.parametrize("dt", [np.int32, np.float64, np.float32])
def test_few_columns_wave_reduction_bit_exact(dt):
    # N <= 16 and an association-independent fold: the fold over l is split
    # across the lanes of a wave and combined by a wavefront reduction.
    rng = np.random.default_rng(111)
    folds = FOLD_I if dt == np.int32 else ["max", "min"]
    elems = ELEM_I if dt == np.int32 else ELEM_F
    # The first six shapes take the chunked kernel (or, for K = 256, B
    # resident in LDS); the last five keep all of B resident in LDS (K a
    # multiple of one 16-byte run per lane of a wave, B at most 128 KiB).
    for M, K, N in [(300, 1000, 1), (257, 777, 3), (5, 4100, 16), (1, 256, 7), (33, 300, 4), (9, 513, 9),
                    (300, 512, 1), (257, 1024, 3), (33, 768, 5), (100, 1024, 9), (70, 2048, 16)]:
        a = rand(rng, (M, K), dt)
        b = rand(rng, (K, N), dt)
        ga, gb = gpu(a), gpu(b)
        for op1 in folds:
            for op2 in elems:
                say("few columns", np.dtype(dt).name, M, K, N, op1, op2)
                eq(host(G.inner(ga, gb, op1, op2)), oracle.inner(a, b, op1, op2, mode="native"))


@pytest.mark.parametrize("dt", [np.int32, np.float64])
def test_few_columns_misaligned_rows(dt):
    # A one element past a 16-byte boundary: the per-element loads instead of
    # the vector loads, same results.
    rng = np.random.default_rng(113)
    M, K, N = 70, 1000, 5
    a = rand(rng, (M, K), dt)
    b = rand(rng, (K, N), dt)
    ta = torch.zeros(a.size + 1, dtype=gpu(a).dtype, device=DEV)
    ta[1:] = gpu(a.ravel())
    av = ta[1:].view(M, K)
    assert av.data_ptr() % 16 != 0
    op1 = "xor" if dt == np.int32 else "max"
    say("few columns misaligned", np.dtype(dt).name, op1)
    eq(host(G.inner(av, gpu(b), op1, "add")), oracle.inner(a, b, op1, "add", mode="native"))


def test_few_columns_workload_sampled():
    # int32 (max,+) <65536 4096> . <4096 8>: rows checked against the oracle.
    a, b = mi.workload_fewcols()
    say("few columns 65536 x 4096 . 4096 x 8")
    d = host(G.inner(gpu(a), gpu(b), "max", "add"))
    rows = np.sort(np.random.default_rng(112).choice(a.shape[0], 64, replace=False))
    eq(d[rows], oracle.inner(a, b, "max", "add", rows=rows))


def test_few_rows_paper_workload_full():
    # Section II.B: A m x 128 (m = 4), B 128 x n, n = 2^22; every row checked.
    a, b = mi.workload_skinny()
    say("few rows 4 x 128 . 128 x 2^22")
    d = host(G.inner(gpu(a), gpu(b)))
    eq(d, oracle.inner(a, b))
    assert nerr(d, oracle.inner_dot2(a, b)) <= 1e-14


def test_empty_and_degenerate():
    for dt in (np.float64, np.int32):
        a = np.zeros((3, 0), dtype=dt)
        b = np.zeros((0, 5), dtype=dt)
        folds = FOLD_I if dt == np.int32 else FOLD_F
        for op1 in folds:
            say("K=0", op1)
            d = host(G.inner(gpu(a), gpu(b), op1, "add"))
            eq(d, np.full((3, 5), oracle.identity_of(op1, dt), dtype=dt))
        assert G.inner(gpu(np.zeros((0, 4), dt)), gpu(np.ones((4, 3), dt))).shape == (0, 3)
    d = host(G.inner_split(gpu(np.zeros((3, 0))), gpu(np.zeros((0, 2)))))
    eq(d, np.zeros((3, 2)))
    c = host(G.outer(gpu(np.array(3.0)), gpu(np.array(4.0)), "sub"))
    assert c.shape == () and c == -1.0


@pytest.mark.parametrize("dt", [np.float64, np.float32, np.int32])
def test_outer_all_ops_bit_exact(dt):
    rng = np.random.default_rng(102)
    elems = ELEM_I if dt == np.int32 else ELEM_F
    for sa, sb in [((), (5,)), ((3, 2), (7,)), ((17, 3), (2, 129)), ((4,), (1024,)), ((5, 5), (300, 3))]:
        a = rand(rng, sa, dt)
        b = rand(rng, sb, dt)
        for op in elems:
            say("outer", np.dtype(dt).name, sa, sb, op)
            eq(host(G.outer(gpu(a), gpu(b), op)), oracle.outer(a, b, op))


@pytest.mark.parametrize("dt,tol", [(np.float64, 1e-13), (np.float32, 1e-5)])
def test_mfma_plus_times(dt, tol):
    rng = np.random.default_rng(103)
    for sa, sb in [((37, 19), (19, 53)), ((2, 3, 70), (70, 5, 9)), ((257, 130), (130, 129)), ((640, 333), (333, 512)),
                   ((9,), (9, 4))]:
        a = mi.uniform_f64(rng, sa).astype(dt)
        b = mi.uniform_f64(rng, sb).astype(dt)
        say("mfma", np.dtype(dt).name, sa, sb)
        d = host(G.inner(gpu(a), gpu(b)))
        ref = oracle.inner_dot2(a, b)
        assert nerr(d, ref) <= tol, nerr(d, ref)


@pytest.mark.parametrize("dt,tol", [(np.float64, 1e-13), (np.float32, 1e-5)])
def test_mfma_vector_panels_ragged_and_misaligned(dt, tol):
    # Contiguous extents that are multiples of 4 take the 16-byte vector panel
    # loads; ragged M and N exercise their edges. The same operands at an
    # address 1 element past a 16-byte boundary must take the scalar loads.
    rng = np.random.default_rng(109)
    for sa, sb in [((257, 132), (132, 516)), ((3, 45, 64), (64, 6, 10)), ((1030, 68), (68, 36))]:
        a = mi.uniform_f64(rng, sa).astype(dt)
        b = mi.uniform_f64(rng, sb).astype(dt)
        ref = oracle.inner_dot2(a, b)
        say("mfma vector panels", np.dtype(dt).name, sa, sb)
        assert nerr(host(G.inner(gpu(a), gpu(b))), ref) <= tol
        ta = torch.zeros(a.size + 1, dtype=gpu(a).dtype, device=DEV)
        tb = torch.zeros(b.size + 1, dtype=gpu(b).dtype, device=DEV)
        ta[1:] = gpu(a.ravel())
        tb[1:] = gpu(b.ravel())
        av, bv = ta[1:].view(sa), tb[1:].view(sb)
        assert av.data_ptr() % 16 != 0 and bv.data_ptr() % 16 != 0
        say("mfma misaligned", np.dtype(dt).name, sa, sb)
        assert nerr(host(G.inner(av, bv)), ref) <= tol


def test_mfma_f32_large_tiles_transposed_operands():
    # FP32 products in 128 x 128 tiles (32-bit index kernel) with A stored
    # K x M and B stored K x N or N x K, ragged edges (M = N = 3000).
    rng = np.random.default_rng(118)
    a = mi.uniform_f64(rng, (64, 3000)).astype(np.float32)
    for sb, ax_b in (((64, 3000), 0), ((3000, 64), 1)):
        b = mi.uniform_f64(rng, sb).astype(np.float32)
        say("mfma f32 large tiles, axes", (0, ax_b))
        got = host(G.inner_axes(gpu(a), gpu(b), (0, ax_b)))
        am, bm = _moved(a, 0, b, ax_b)
        rows = np.sort(rng.choice(3000, 20, replace=False))
        ref = oracle.inner_dot2(np.ascontiguousarray(am), np.ascontiguousarray(bm), rows=rows)
        assert nerr(got[rows], ref) <= 1e-5


def test_mfma_f64_exact_integers():
    # Integer entries with |x| <= 8 and K <= 8192: every partial sum is exact,
    # so any summation order gives the exact product. Small grids with long
    # contractions (the first two) split k over wave groups.
    rng = np.random.default_rng(104)
    for sa, sb in [((200, 1000), (1000, 130)), ((97, 333), (333, 61)), ((512, 512), (512, 512)),
                   ((1100, 300), (300, 700))]:
        a = mi.small_int_f64(rng, sa, 8)
        b = mi.small_int_f64(rng, sb, 8)
        say("mfma exact ints", sa, sb)
        eq(host(G.inner(gpu(a), gpu(b))), (a.astype(np.int64) @ b.astype(np.int64)).astype(np.float64))


# ---------------------------------------------------------------------------
# Full-size workloads, sampled rows.

def _sample_rows(rng, m, n=24):
    rows = np.unique(np.concatenate([[0, m - 1], rng.integers(0, m, n)]))
    return rows


def test_small_mixed_full():
    a, b, oa, ob = mi.workload_small_mixed()
    say("512^3 fp64 + outer 32x32 o 16x16")
    d = host(G.inner(gpu(a), gpu(b)))
    assert nerr(d, oracle.inner_dot2(a, b)) <= 1e-13
    eq(host(G.outer(gpu(oa), gpu(ob), "mul")), oracle.outer(oa, ob, "mul"))


def test_rank_general_fp64_full_sampled():
    a, b = mi.workload_rank_general_f64()
    say("rank-5 fp64", a.shape, b.shape)
    ga, gb = gpu(a), gpu(b)
    d = G.inner(ga, gb)
    assert tuple(d.shape) == (64, 64, 32, 128, 64)
    m = 64 * 64 * 32
    rows = _sample_rows(np.random.default_rng(5), m)
    dflat = d.reshape(m, -1)
    got = host(dflat[torch.from_numpy(rows).to(DEV)])
    ref = oracle.inner_dot2(a, b, rows=rows).reshape(len(rows), -1)
    assert nerr(got, ref) <= 1e-13
    del d, dflat
    torch.cuda.empty_cache()


def test_tropical_full_sampled():
    a, b = mi.workload_tropical()
    say("tropical 2048^3 (max,+)")
    d = G.inner(gpu(a), gpu(b), "max", "add")
    rows = _sample_rows(np.random.default_rng(6), 2048, 64)
    got = host(d[torch.from_numpy(rows).to(DEV)])
    eq(got, oracle.inner(a, b, "max", "add", rows=rows))


def test_outer_f32_full_sampled():
    a, b = mi.workload_outer_f32()
    say("outer fp32 (-) <512 512> o <64 64>")
    c = G.outer(gpu(a), gpu(b), "sub")
    assert tuple(c.shape) == (512, 512, 64, 64)
    rows = _sample_rows(np.random.default_rng(7), 512 * 512, 64)
    got = host(c.reshape(512 * 512, -1)[torch.from_numpy(rows).to(DEV)])
    eq(got, oracle.outer(a.reshape(-1)[rows], b.reshape(-1), "sub"))
    del c
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# Split precision.

@pytest.mark.parametrize("shape", [(100, 300, 70), (64, 64, 128), (1, 1, 1), (257, 1000, 131), (33, 65, 200)])
def test_split_matches_oracle_scheme(shape):
    M, K, N = shape
    rng = np.random.default_rng(105)
    a = mi.scaled_f64(rng, (M, K))
    b = mi.scaled_f64(rng, (K, N))
    ref = oracle.inner_dot2(a, b)
    for S in range(1, 8):
        say("split", shape, "S", S)
        d = host(G.inner_split(gpu(a), gpu(b), "bf16", S))
        want = oracle.split_inner(a, b, nslices=S, beta=9)
        assert nerr(d, want) <= scheme_tol("bf16", S), (S, nerr(d, want))
        if S >= 5:
            assert nerr(d, ref) <= 1e-12, (S, nerr(d, ref))


def test_split_exact_cases():
    rng = np.random.default_rng(106)
    # Integers in [-255, 255] with a row/column maximum in [128, 256) are one
    # signed 9-bit digit each: one slice gives the exact product.
    a = mi.small_int_f64(rng, (70, 400), 255)
    b = mi.small_int_f64(rng, (400, 90), 255)
    a[:, 0] = 200.0
    b[0, :] = -200.0
    say("split exact integers")
    d = host(G.inner_split(gpu(a), gpu(b), "bf16", 1))
    eq(d, (a.astype(np.int64) @ b.astype(np.int64)).astype(np.float64))
    # Power-of-two row/column scaling commutes exactly with the scheme.
    a = mi.scaled_f64(rng, (40, 300))
    b = mi.scaled_f64(rng, (300, 50))
    d = host(G.inner_split(gpu(a), gpu(b), "bf16", 5))
    a2 = a.copy()
    a2[7] = np.ldexp(a2[7], 11)
    d2 = host(G.inner_split(gpu(a2), gpu(b), "bf16", 5))
    want = d.copy()
    want[7] = np.ldexp(want[7], 11)
    eq(d2, want)


def test_split_full_size_sampled():
    a, b = mi.workload_split()
    say("split 8192^3 S=5")
    d = G.inner_split(gpu(a), gpu(b), "bf16", 5)
    rows = _sample_rows(np.random.default_rng(8), 8192, 14)
    got = host(d[torch.from_numpy(rows).to(DEV)])
    ref = oracle.inner_dot2(a, b, rows=rows)
    e = nerr(got, ref)
    scale = oracle.abs_product(a, b, rows=rows)
    cw = oracle.componentwise_error(got, ref, scale)
    say("split 8192^3 vs Dot2: normwise %.3e, max-norm %.3e, componentwise %.3e"
        % (e, oracle.maxnorm_error(got, ref), cw))
    assert e <= 1e-12
    want = oracle.split_inner(a, b, nslices=5, beta=9, rows=rows[:6])
    assert nerr(got[:6], want) <= scheme_tol("bf16", 5)
    # Element by element the GPU carries the scheme's own truncation error,
    # plus at most its merged-level rounding (bounded normwise above).
    cw_scheme = oracle.componentwise_error(want, ref[:6], scale[:6])
    assert oracle.componentwise_error(got[:6], ref[:6], scale[:6]) <= 1.1 * cw_scheme + scheme_tol("bf16", 5)


@pytest.mark.parametrize("shape", [(100, 300, 70), (64, 32, 128), (1, 1, 1), (257, 1000, 131), (33, 65, 200)])
def test_split_int8_matches_oracle_scheme(shape):
    M, K, N = shape
    rng = np.random.default_rng(107)
    a = mi.scaled_f64(rng, (M, K))
    b = mi.scaled_f64(rng, (K, N))
    ref = oracle.inner_dot2(a, b)
    for S in range(1, 8):
        say("split int8", shape, "S", S)
        d = host(G.inner_split(gpu(a), gpu(b), "int8", S))
        want = oracle.split_inner(a, b, nslices=S, beta=7)
        assert nerr(d, want) <= 1e-14, (S, nerr(d, want))
        if S == 7:
            assert nerr(d, ref) <= 1e-12, (S, nerr(d, ref))


def test_split_int8_exact_integers():
    # Integers in [-63, 63] whose row/column maximum lies in [32, 64) are one
    # signed 7-bit digit each: one INT8 slice gives the exact product.
    rng = np.random.default_rng(108)
    a = mi.small_int_f64(rng, (90, 700), 63)
    b = mi.small_int_f64(rng, (700, 70), 63)
    a[:, 3] = 40.0
    b[5, :] = -50.0
    say("split int8 exact integers")
    d = host(G.inner_split(gpu(a), gpu(b), "int8", 1))
    eq(d, (a.astype(np.int64) @ b.astype(np.int64)).astype(np.float64))


def test_split_int8_full_size_sampled():
    a, b = mi.workload_split()
    say("split int8 8192^3 S=7")
    d = G.inner_split(gpu(a), gpu(b), "int8", 7)
    rows = _sample_rows(np.random.default_rng(9), 8192, 10)
    got = host(d[torch.from_numpy(rows).to(DEV)])
    ref = oracle.inner_dot2(a, b, rows=rows)
    e = nerr(got, ref)
    scale = oracle.abs_product(a, b, rows=rows)
    say("split int8 8192^3 vs Dot2: normwise %.3e, max-norm %.3e, componentwise %.3e"
        % (e, oracle.maxnorm_error(got, ref), oracle.componentwise_error(got, ref, scale)))
    assert e <= 1e-12
    want = oracle.split_inner(a, b, nslices=7, beta=7, rows=rows[:4])
    assert nerr(got[:4], want) <= 1e-14
    cw_scheme = oracle.componentwise_error(want, ref[:4], scale[:4])
    assert oracle.componentwise_error(got[:4], ref[:4], scale[:4]) <= 1.1 * cw_scheme + 1e-16


# ---------------------------------------------------------------------------
# Differentiation.

def test_grad_finite_differences_fp64():
    rng = mi.rng_for(mi.DIFFERENTIATION, salt=1)
    a = mi.uniform_f64(rng, (4, 4, 8))
    b = mi.uniform_f64(rng, (8, 4, 4))
    g = mi.uniform_f64(rng, (4, 4, 4, 4))
    say("grad FD 4x4x8 . 8x4x4")
    da, db = G.inner_grad(gpu(a), gpu(b), gpu(g))
    da, db = host(da), host(db)
    gb, gg = gpu(b), gpu(g)
    h = 2.0 ** -8

    def loss(x, y):
        return float(torch.sum(G.inner(gpu(x), gpu(y)) * gg).item())

    fa = np.zeros_like(a)
    for idx in np.ndindex(a.shape):
        ap, am = a.copy(), a.copy()
        ap[idx] += h
        am[idx] -= h
        fa[idx] = (loss(ap, b) - loss(am, b)) / (2 * h)
    fb = np.zeros_like(b)
    for idx in np.ndindex(b.shape):
        bp, bm = b.copy(), b.copy()
        bp[idx] += h
        bm[idx] -= h
        fb[idx] = (loss(a, bp) - loss(a, bm)) / (2 * h)
    # L is linear in each element, so central differences are exact up to rounding.
    assert np.max(np.abs(fa - da)) <= 1e-12
    assert np.max(np.abs(fb - db)) <= 1e-12


def test_grad_full_size_vs_oracle():
    a, b, g = mi.workload_grad()
    say("grad fp32 <32 128 512> . <512 64 64>")
    ta = gpu(a).requires_grad_(True)
    tb = gpu(b).requires_grad_(True)
    d = moa.moa_inner(ta, tb)
    d.backward(gpu(g))
    da, db = host(ta.grad), host(tb.grad)
    # dA = G (+,*) B_rot, B_rot = B with its first axis moved last;
    # dB = A_rot (+,*) G, A_rot = A with its last axis moved first.
    b_rot = np.ascontiguousarray(np.moveaxis(b, 0, -1))
    a_rot = np.ascontiguousarray(np.moveaxis(a, -1, 0))
    g2 = g.reshape(32, 128, 64 * 64)
    ref_da = oracle.inner(g2, b_rot.reshape(64 * 64, 512)).reshape(a.shape)
    ref_db = oracle.inner(a_rot.reshape(512, 32 * 128), g.reshape(32 * 128, 64, 64)).reshape(b.shape)
    assert nerr(da, ref_da) <= 1e-5
    assert nerr(db, ref_db) <= 1e-5
    assert nerr(host(d.detach()), oracle.inner(a, b)) <= 1e-5


@pytest.mark.parametrize("dt,tol", [(np.float32, 1e-5), (np.float64, 1e-13)])
def test_grad_shapes_paired_and_separate(dt, tol):
    # Both gradients in one launch when dA and dB take the same tile size
    # (ragged edges included), two launches when they do not (last shape:
    # dA 8192 x 2048 in 128 x 128 tiles, dB 2048 x 64 in 32 x 32), and only
    # the requested one when the other is not needed.
    rng = np.random.default_rng(117)
    for M, K, N in [(37, 53, 29), (300, 70, 130), (4100, 36, 260), (8192, 2048, 64)]:
        a = mi.uniform_f64(rng, (M, K)).astype(dt)
        b = mi.uniform_f64(rng, (K, N)).astype(dt)
        g = mi.uniform_f64(rng, (M, N)).astype(dt)
        say("grad", np.dtype(dt).name, M, K, N)
        da, db = G.inner_grad(gpu(a), gpu(b), gpu(g))
        rows = None if M <= 4100 else np.sort(rng.choice(M, 16, replace=False))
        ref_da = oracle.inner_dot2(g, np.ascontiguousarray(b.T), rows=rows)
        got_da = host(da) if rows is None else host(da)[rows]
        assert nerr(got_da, ref_da) <= tol
        assert nerr(host(db), oracle.inner_dot2(np.ascontiguousarray(a.T), g)) <= tol
    a = mi.uniform_f64(rng, (70, 40)).astype(dt)
    b = mi.uniform_f64(rng, (40, 90)).astype(dt)
    g = mi.uniform_f64(rng, (70, 90)).astype(dt)
    da, db = G.inner_grad(gpu(a), gpu(b), gpu(g), need_a=True, need_b=False)
    assert db is None and nerr(host(da), oracle.inner_dot2(g, np.ascontiguousarray(b.T))) <= tol
    da, db = G.inner_grad(gpu(a), gpu(b), gpu(g), need_a=False, need_b=True)
    assert da is None and nerr(host(db), oracle.inner_dot2(np.ascontiguousarray(a.T), g)) <= tol


# ---------------------------------------------------------------------------
# Batching.

def _check_batch(probs, ds, idx):
    for i in idx:
        p = probs[i]
        got = ds[i]
        ref = oracle.inner(p.a, p.b)
        e = nerr(got, ref)
        assert e <= 1e-5, (i, p.shape_a, p.shape_b, e)


def test_batch_small_full_check():
    probs = mi.batch_problems(mi.rng_for(mi.BATCH, salt=1), 600)
    As = [gpu(p.a) for p in probs]
    Bs = [gpu(p.b) for p in probs]
    pool = GuardPool([(moa.inner_shape(p.shape_a, p.shape_b), torch.float32) for p in probs])
    Ds = pool.t
    say("batch 600")
    bt = moa.Batch(As, Bs, Ds)
    items, launches = bt.info()
    assert launches == 1 and items >= 600
    for rep in range(3):
        for d in Ds:
            d.fill_(float("nan"))
        bt.run()
        pool.check("batch of 600, run %d" % rep)
        hd = [d.cpu().numpy() for d in Ds]
        _check_batch(probs, hd, range(len(probs)))
    bt.close()


BATCH_VARIANTS = (0, 1)


class _tile_variant:
    """Every bucket of the batch tile table set to one variant, restored on exit."""

    def __init__(self, v):
        self.v = v

    def __enter__(self):
        self.saved = moa.tile_table()
        moa.set_tile_table("\n".join(" ".join(l.split()[:3] + [str(self.v)])
                                     for l in self.saved.strip().splitlines()))

    def __exit__(self, *exc):
        moa.set_tile_table(self.saved)


@pytest.mark.parametrize("variant", BATCH_VARIANTS)
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_batch_degenerate_and_ragged_problems(variant, dt):
    # Empty sums (K = 0: the result is all zeros), empty results (M or N = 0:
    # nothing written), 1 x 1 x 1, K that is not a multiple of the 16-wide
    # panels, M and N one past a tile, and a full 64 x 64 tile, in one batch.
    # Small integers: exact sums, compared element by element. FP32 batches
    # run the LDS-fed tile, FP64 the register-staged one.
    rng = np.random.default_rng(171)
    shapes = [((5, 0), (0, 7)), ((0, 9), (9, 4)), ((6, 9), (9, 0)), ((1, 1), (1, 1)), ((3, 17), (17, 2)),
              ((33, 31), (31, 65)), ((64, 512), (512, 64)), ((65, 16), (16, 33)), ((2, 3, 47), (47, 5, 2))]
    a_s = [mi.small_int_f64(rng, sa, 8).astype(dt) for sa, _ in shapes]
    b_s = [mi.small_int_f64(rng, sb, 8).astype(dt) for _, sb in shapes]
    tdt = torch.float32 if dt == np.float32 else torch.float64
    pool = GuardPool([(moa.inner_shape(sa, sb), tdt) for sa, sb in shapes])
    say("batch degenerate and ragged", np.dtype(dt).name, "tile variant", variant)
    with _tile_variant(variant):
        bt = moa.Batch([gpu(a) for a in a_s], [gpu(b) for b in b_s], pool.t)
    bt.run()
    pool.check("degenerate batch")
    for a, b, d in zip(a_s, b_s, pool.t):
        eq(host(d), np.tensordot(a.astype(np.float64), b.astype(np.float64), axes=([a.ndim - 1], [0])).astype(dt))
    bt.close()


@pytest.mark.parametrize("variant", BATCH_VARIANTS)
def test_batch_wide_problem_64bit_offsets(variant):
    # A problem whose padded extents pass 2^31 offsets makes the whole batch
    # use 64-bit tile index arithmetic. Small integer entries: exact sums.
    rng = np.random.default_rng(115)
    shapes = [((2, 3), (3, 32_100_000)), ((5, 7), (7, 9)), ((40, 130), (130, 33))]
    a_s = [rng.integers(-2, 3, size=sa).astype(np.float32) for sa, _ in shapes]
    b_s = [rng.integers(-2, 3, size=sb).astype(np.float32) for _, sb in shapes]
    As, Bs = [gpu(a) for a in a_s], [gpu(b) for b in b_s]
    pool = GuardPool([((sa[0], sb[1]), torch.float32) for sa, sb in shapes])
    Ds = pool.t
    say("batch with a 2 x 3 . 3 x 32.1M problem, tile variant", variant)
    with _tile_variant(variant):
        bt = moa.Batch(As, Bs, Ds)
    bt.run()
    pool.check("batch with 64-bit offsets")
    for a, b, d in zip(a_s, b_s, Ds):
        eq(host(d), (a.astype(np.int64) @ b.astype(np.int64)).astype(np.float32))
    bt.close()
    del As, Bs, Ds
    torch.cuda.empty_cache()


def test_batch_full_size_sampled():
    probs = mi.batch_problems(mi.rng_for(mi.BATCH), 10000)
    As = [gpu(p.a) for p in probs]
    Bs = [gpu(p.b) for p in probs]
    pool = GuardPool([(moa.inner_shape(p.shape_a, p.shape_b), torch.float32) for p in probs])
    Ds = pool.t
    say("batch 10000")
    bt = moa.Batch(As, Bs, Ds)
    bt.run()
    bt.run()
    pool.check("batch of 10000")
    idx = np.random.default_rng(9).choice(len(probs), 400, replace=False)
    _check_batch(probs, {int(i): Ds[int(i)].cpu().numpy() for i in idx}, [int(i) for i in idx])
    bt.close()


def test_batch_autotune_then_build():
    say("batch autotune")
    table = moa.batch_autotune(torch.float32, reps=2)
    assert len(table.strip().splitlines()) == 8
    probs = mi.batch_problems(mi.rng_for(mi.BATCH, salt=2), 200)
    As = [gpu(p.a) for p in probs]
    Bs = [gpu(p.b) for p in probs]
    pool = GuardPool([(moa.inner_shape(p.shape_a, p.shape_b), torch.float32) for p in probs])
    Ds = pool.t
    bt = moa.Batch(As, Bs, Ds)
    bt.run()
    pool.check("autotuned batch")
    _check_batch(probs, [d.cpu().numpy() for d in Ds], range(len(probs)))
    bt.close()


def test_binding_checks_out_workspace_and_layout():
    # A result or workspace tensor on the host, or of the wrong shape, is
    # rejected before any launch; non-contiguous operands are made dense.
    rng = np.random.default_rng(116)
    a = mi.uniform_f64(rng, (40, 24))
    b = mi.uniform_f64(rng, (24, 30))
    ga, gb = gpu(a), gpu(b)
    with pytest.raises(ValueError):
        moa.inner(ga, gb, out=torch.empty(40, 30, dtype=torch.float64))
    with pytest.raises(ValueError):
        moa.outer(ga, gb, out=torch.empty(40, 24, 30, 24, dtype=torch.float64, device=DEV))
    with pytest.raises(ValueError):
        moa.inner_split(ga, gb, workspace=torch.empty(1 << 20, dtype=torch.uint8))
    # Expanded (stride-0) and transposed views as split operands.
    at = gpu(np.ascontiguousarray(a.T)).t()
    bx = gpu(b[:1]).expand(24, 30)
    ref = moa.inner_split(gpu(a), gpu(np.repeat(b[:1], 24, axis=0)))
    ws = torch.empty(moa.split_workspace_bytes((40, 24), (24, 30)), dtype=torch.uint8, device=DEV)
    out = torch.empty(40, 30, dtype=torch.float64, device=DEV)
    say("split two-stage on strided views")
    moa.split_prepare(at, bx, ws)
    moa.split_multiply((40, 24), (24, 30), out, ws)
    eq(host(out), host(ref))


def test_errors_on_device_tensors():
    a = gpu(np.ones((3, 4)))
    b = gpu(np.ones((5, 2)))
    with pytest.raises(moa.MoaError) as e:
        moa.inner(a, b)
    assert moa.STATUS[e.value.status] == "MOA_ERR_SHAPE"
    with pytest.raises(moa.MoaError) as e:
        moa.inner(a, gpu(np.ones((4, 2))), "sub", "mul")
    assert moa.STATUS[e.value.status] == "MOA_ERR_OP"


# ---------------------------------------------------------------------------
# Contraction over any axis pair, read in place through (P, K, Q) views.

AXES_CASES = [
    ((7, 45, 33), 1, (20, 45, 13), 1),     # general strides on both sides, ragged tiles
    ((45, 150), 0, (130, 45), 1),          # A stored K x M, B stored N x K
    ((3, 70, 2, 5), 1, (70, 140), 0),      # A strided, B plain
    ((90, 37), 1, (11, 37, 12), 1),        # A plain, B strided
    ((17, 130), 0, (17,), 0),              # A stored K x M, vector result
    ((5, 36, 8), 1, (12, 36, 20), 1),      # inner extents multiples of 4: vector panels, strided
    ((9, 40, 4), 1, (7, 40), 1),           # A strided (Qa = 4), B stored N x K (K = 40)
    ((48, 132), 0, (68, 48), 1),           # A stored K x M, B stored N x K, vector panels, ragged
]


def _moved(a, ax_a, b, ax_b):
    return np.moveaxis(a, ax_a, -1), np.moveaxis(b, ax_b, 0)


@pytest.mark.parametrize("dt", [np.float64, np.float32, np.int32])
def test_inner_axes_all_pairs_bit_exact(dt):
    rng = np.random.default_rng(41)
    folds = FOLD_I if dt == np.int32 else FOLD_F
    elems = ELEM_I if dt == np.int32 else ELEM_F
    for sa, ax_a, sb, ax_b in AXES_CASES[:3]:
        say("axes", dt.__name__, sa, ax_a, sb, ax_b)
        a, b = rand(rng, sa, dt), rand(rng, sb, dt)
        ga, gb = gpu(a), gpu(b)
        for op1 in folds:
            for op2 in elems:
                got = host(G.inner_axes(ga, gb, (ax_a, ax_b), op1, op2, flags=moa.FLAG_SEQUENTIAL_FOLD))
                eq(got, oracle.inner_axes(a, ax_a, b, ax_b, op1, op2, mode="native"))


@pytest.mark.parametrize("dt,tol", [(np.float64, 1e-13), (np.float32, 1e-5)])
def test_inner_axes_mfma(dt, tol):
    rng = np.random.default_rng(42)
    for sa, ax_a, sb, ax_b in AXES_CASES:
        say("axes (+,*)", dt.__name__, sa, ax_a, sb, ax_b)
        a, b = rand(rng, sa, dt), rand(rng, sb, dt)
        got = host(G.inner_axes(gpu(a), gpu(b), (ax_a, ax_b)))
        ref = oracle.inner_dot2(*_moved(a.astype(np.float64), ax_a, b.astype(np.float64), ax_b))
        assert got.shape == ref.shape
        assert nerr(got, ref) <= tol


def test_inner_axes_mfma_exact_integers():
    # Small integers: every partial sum is exact, so any summation order gives
    # the oracle's value bit for bit.
    rng = np.random.default_rng(43)
    for sa, ax_a, sb, ax_b in AXES_CASES:
        a = mi.small_int_f64(rng, sa, 8)
        b = mi.small_int_f64(rng, sb, 8)
        eq(host(G.inner_axes(gpu(a), gpu(b), (ax_a, ax_b))), oracle.inner_axes(a, ax_a, b, ax_b))


def test_inner_axes_last_with_first_equals_inner():
    rng = np.random.default_rng(44)
    a, b = rand(rng, (40, 9, 33), np.float64), rand(rng, (33, 70), np.float64)
    ga, gb = gpu(a), gpu(b)
    eq(host(G.inner_axes(ga, gb, (-1, 0))), host(G.inner(ga, gb)))
    eq(host(G.inner_axes(ga, gb, (2, 0), "max", "add")), host(G.inner(ga, gb, "max", "add")))


def test_inner_axes_large_sampled():
    # 3072 x 512 . 512 x 1280 through general strides on both operands.
    rng = np.random.default_rng(45)
    a = mi.uniform_f64(rng, (64, 512, 48))
    b = mi.uniform_f64(rng, (32, 512, 40))
    got = host(G.inner_axes(gpu(a), gpu(b), (1, 1))).reshape(3072, 1280)
    am, bm = _moved(a, 1, b, 1)
    rows = np.sort(rng.choice(3072, 24, replace=False))
    ref = oracle.inner_dot2(am, bm, rows=rows).reshape(len(rows), 1280)
    assert nerr(got[rows], ref) <= 1e-13
    at, bt = rand(rng, (300, 64, 7), np.int32), rand(rng, (9, 64, 150), np.int32)
    got = host(G.inner_axes(gpu(at), gpu(bt), (1, 1), "max", "add")).reshape(2100, 1350)
    rows = np.sort(rng.choice(2100, 24, replace=False))
    ref = oracle.inner_axes(at, 1, bt, 1, "max", "add", rows=rows).reshape(len(rows), 1350)
    eq(got[rows], ref)


# ---------------------------------------------------------------------------
# API corners: the two-stage split API, FP64 batches, non-default streams.

def test_split_two_stage_api_matches_one_call():
    # moa_inner_split_prepare + moa_inner_split_multiply run the same kernels
    # as moa_inner_split: identical bits, and the oracle's scheme to 1e-14.
    rng = np.random.default_rng(120)
    a = mi.scaled_f64(rng, (200, 700))
    b = mi.scaled_f64(rng, (700, 150))
    ga, gb = gpu(a), gpu(b)
    for fmt, S, beta in (("bf16", 5, 9), ("int8", 7, 7), ("fp8", 9, 5)):
        say("split two-stage", fmt)
        one = host(G.inner_split(ga, gb, fmt, S))
        ws = torch.empty(moa.split_workspace_bytes(a.shape, b.shape, fmt, S), dtype=torch.uint8, device=DEV)
        out = torch.full((200, 150), float("nan"), dtype=torch.float64, device=DEV)
        moa.split_prepare(ga, gb, ws, fmt, S)
        moa.split_multiply(a.shape, b.shape, out, ws, fmt, S)
        two = host(out)
        eq(two, one)
        assert nerr(two, oracle.split_inner(a, b, nslices=S, beta=beta)) <= scheme_tol(fmt, S)
        # The multiply stage alone can be replayed on the same workspace.
        out.fill_(float("nan"))
        moa.split_multiply(a.shape, b.shape, out, ws, fmt, S)
        eq(host(out), one)


@pytest.mark.parametrize("variant", BATCH_VARIANTS)
def test_batch_fp64(variant):
    rng = np.random.default_rng(121)
    shapes = mi.batch_shapes(rng, 300)
    probs = [(sa, sb, mi.uniform_f64(rng, sa), mi.uniform_f64(rng, sb)) for sa, sb in shapes]
    As = [gpu(a) for _, _, a, _ in probs]
    Bs = [gpu(b) for _, _, _, b in probs]
    pool = GuardPool([(moa.inner_shape(sa, sb), torch.float64) for sa, sb, _, _ in probs])
    Ds = pool.t
    say("batch fp64 300, tile variant", variant)
    with _tile_variant(variant):
        bt = moa.Batch(As, Bs, Ds)
    bt.run()
    pool.check("batch fp64")
    for (sa, sb, a, b), d in zip(probs, Ds):
        assert nerr(d.cpu().numpy(), oracle.inner_dot2(a, b)) <= 1e-13, (sa, sb)
    bt.close()


def test_non_default_stream():
    # Work is enqueued on the caller's current stream; results are complete
    # once that stream is synchronised.
    rng = np.random.default_rng(122)
    a = rand(rng, (300, 500), np.int32)
    b = rand(rng, (500, 200), np.int32)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ga, gb = gpu(a), gpu(b)
        d = G.inner(ga, gb, "max", "add")
        c = G.outer(ga[:3], gb[0], "sub")
    s.synchronize()
    eq(d.cpu().numpy(), oracle.inner(a, b, "max", "add"))
    eq(c.cpu().numpy(), oracle.outer(a[:3], b[0], "sub"))


def test_int32_wraparound_every_path():
    # Large int32 entries: +, - and * overflow and must wrap exactly as the
    # oracle's two's-complement arithmetic in every kernel that folds int32.
    rng = np.random.default_rng(130)
    big = lambda shape: rng.integers(-2**31, 2**31, size=shape, dtype=np.int64).astype(np.int32)
    cases = [((70, 90), (90, 50)),          # register-blocked SIMT
             ((3, 40), (40, 5000)),         # few rows, stream over B
             ((40, 600), (600, 5)),         # few columns, wavefront reduction
             ((2, 3, 7), (7, 2, 2))]        # rank 3, small
    for sa, sb in cases:
        a, b = big(sa), big(sb)
        ga, gb = gpu(a), gpu(b)
        for op1, op2 in [("add", "mul"), ("mul", "add"), ("add", "sub"), ("max", "mul"), ("xor", "mul")]:
            say("int32 wrap", sa, sb, op1, op2)
            eq(host(G.inner(ga, gb, op1, op2)), oracle.inner(a, b, op1, op2))
    a, b = big((33, 17)), big((9, 129))
    for op in ("add", "sub", "mul"):
        eq(host(G.outer(gpu(a), gpu(b), op)), oracle.outer(a, b, op))


def test_maximum_rank_and_unit_axes():
    rng = np.random.default_rng(131)
    sa = (1, 2, 1, 3, 1, 1, 2, 1, 1, 1, 1, 1, 1, 2, 1, 5)          # rank 16
    sb = (5, 1, 1, 1, 1, 1, 1, 1, 2, 1, 1, 1, 1, 1, 1, 3)          # rank 16
    a = rand(rng, sa, np.int32)
    b = rand(rng, sb, np.int32)
    d = host(G.inner(gpu(a), gpu(b), "add", "mul"))
    assert d.shape == sa[:-1] + sb[1:]
    eq(d, oracle.inner(a, b, "add", "mul"))
    with pytest.raises(moa.MoaError):
        moa.inner(gpu(np.zeros((1,) * 17, np.int32)), gpu(np.zeros((1, 1), np.int32)))
    x = rand(rng, (1, 1, 4), np.float64)
    y = rand(rng, (4, 1, 1), np.float64)
    eq(host(G.inner(gpu(x), gpu(y), "max", "sub")), oracle.inner(x, y, "max", "sub", mode="native"))


def test_plain_fp64_8192_sampled():
    # The plain FP64 comparator of the split benchmark, at its full size.
    a, b = mi.workload_split()
    say("plain fp64 8192^3")
    d = host(G.inner(gpu(a), gpu(b)))
    rows = np.sort(np.random.default_rng(140).choice(8192, 12, replace=False))
    ref = oracle.inner_dot2(a, b, rows=rows)
    assert nerr(d[rows], ref) <= 1e-13
    # Any summation order of K rounded products stays within gamma_K |A||B|.
    u = 2.0 ** -53
    gamma = 8192 * u / (1 - 8192 * u)
    cw = oracle.componentwise_error(d[rows], ref, oracle.abs_product(a, b, rows=rows))
    say("plain fp64 8192^3 componentwise %.3e (gamma_K %.3e)" % (cw, gamma))
    assert cw <= gamma


def test_axes_bench_config_sampled():
    # <16 2048 512> . <16 2048 512> over axes (1, 1), as benchmarked.
    a, b = mi.workload_axes()
    say("axes <16 2048 512> . <16 2048 512>")
    d = host(G.inner_axes(gpu(a), gpu(b), (1, 1))).reshape(8192, 8192)
    am, bm = np.moveaxis(a, 1, -1), np.moveaxis(b, 1, 0)
    rows = np.sort(np.random.default_rng(141).choice(8192, 12, replace=False))
    ref = oracle.inner_dot2(am, bm, rows=rows).reshape(len(rows), 8192)
    assert nerr(d[rows], ref) <= 1e-13



# ---------------------------------------------------------------------------
# Exact FP32 cases for every matrix-core kernel variant: small integer
# entries (|x| <= 8) keep every partial sum an exact FP32 integer (below
# 2^24), so any summation order gives the exact product, element by element.

def _ints32(rng, shape):
    return mi.small_int_f64(rng, shape, 8).astype(np.float32)


def _exact_tensordot(a, ax_a, b, ax_b):
    return np.tensordot(a.astype(np.float64), b.astype(np.float64), axes=([ax_a], [ax_b])).astype(np.float32)


FP32_GEMM_VARIANTS = [
    # (shape A, axis, shape B, axis, what the dispatch picks)
    ((200, 50), 1, (50, 130), 0, "32x32 tiles, scalar panels"),
    ((200, 52), 1, (52, 132), 0, "32x32 tiles, vector panels"),
    ((1100, 36), 1, (36, 1000), 0, "64x64 tiles, vector panels"),
    ((1100, 37), 1, (37, 1001), 0, "64x64 tiles, scalar panels"),
    ((3000, 64), 1, (64, 3000), 0, "128x128 tiles, 32-bit index kernel"),
    ((3000, 65), 1, (65, 3001), 0, "128x128 tiles, 64-bit index, scalar panels"),
    ((64, 3000), 0, (64, 3000), 0, "A stored K x M (TA), 128x128, 32-bit index"),
    ((3000, 64), 1, (3000, 64), 1, "B stored N x K (TB), 128x128, 32-bit index"),
    ((64, 3000), 0, (3000, 64), 1, "TA and TB, 128x128, 32-bit index"),
    ((45, 150), 0, (130, 45), 1, "TA and TB, 32x32"),
    ((7, 45, 33), 1, (20, 45, 13), 1, "strided views (GEN), scalar"),
    ((5, 36, 8), 1, (12, 36, 20), 1, "strided views (GEN), vector panels"),
    ((3, 2, 70), 2, (70, 5, 9), 0, "rank 3 . rank 3"),
    ((200, 1000), 1, (1000, 132), 0, "32x32 tiles, k split over 4 wave groups, vector panels"),
    ((97, 333), 1, (333, 61), 0, "32x32 tiles, k split over 4 wave groups, scalar panels"),
    ((200, 512), 1, (512, 132), 0, "32x32 tiles, k sliced over 16 waves, K = 512"),
    ((97, 300), 1, (300, 61), 0, "32x32 tiles, k sliced over 16 waves, K = 300 (last waves past K)"),
    ((33, 256), 1, (256, 33), 0, "32x32 tiles, k sliced over 16 waves, K = 256, one row and column past a tile"),
]


# FP64 small grids: the k-sliced kernel (K = 256..512, 16-byte aligned rows)
# and the kernel that splits k over four wave groups (longer K, or rows that
# are not 16-byte multiples), on small integers (exact in FP64).
FP64_SMALL_GRID = [
    ((512, 512), (512, 512), "k sliced, the 512^3 workload shape"),
    ((200, 300), (300, 130), "k sliced, K = 300"),
    ((33, 256), (256, 40), "k sliced, K = 256, ragged"),
    ((200, 1000), (1000, 132), "k split over 4 wave groups, vector panels"),
    ((97, 333), (333, 61), "k split over 4 wave groups, scalar panels"),
]


@pytest.mark.parametrize("case", FP64_SMALL_GRID, ids=[c[2] for c in FP64_SMALL_GRID])
def test_fp64_small_grid_exact_integers(case):
    sa, sb, what = case
    rng = np.random.default_rng(163)
    a, b = mi.small_int_f64(rng, sa, 8), mi.small_int_f64(rng, sb, 8)
    say("fp64 exact", what, sa, sb)
    eq(host(G.inner(gpu(a), gpu(b))), a @ b)


@pytest.mark.parametrize("case", FP32_GEMM_VARIANTS, ids=[c[4] for c in FP32_GEMM_VARIANTS])
def test_fp32_gemm_variants_exact_integers(case):
    sa, ax_a, sb, ax_b, what = case
    rng = np.random.default_rng(160)
    a, b = _ints32(rng, sa), _ints32(rng, sb)
    say("fp32 exact", what, sa, ax_a, sb, ax_b)
    got = host(G.inner_axes(gpu(a), gpu(b), (ax_a, ax_b)))
    eq(got, _exact_tensordot(a, ax_a, b, ax_b))


@pytest.mark.parametrize("M,K,N", [(300, 70, 130), (1030, 260, 900), (4096, 512, 4096), (3000, 3000, 3000)])
def test_fp32_grad_exact_integers(M, K, N):
    # Paired gradient launches (32x32, 64x64 and the workload's 64x64
    # vector kernel) and the 128x128 pair, element by element.
    rng = np.random.default_rng(161)
    a, b, g = _ints32(rng, (M, K)), _ints32(rng, (K, N)), _ints32(rng, (M, N))
    say("fp32 grad exact", M, K, N)
    da, db = G.inner_grad(gpu(a), gpu(b), gpu(g))
    ra = np.sort(rng.choice(M, min(M, 64), replace=False))
    rb = np.sort(rng.choice(K, min(K, 64), replace=False))
    g64, b64, a64 = g.astype(np.float64), b.astype(np.float64), a.astype(np.float64)
    eq(host(da)[ra], (g64[ra] @ b64.T).astype(np.float32))
    eq(host(db)[rb], (a64.T[rb] @ g64).astype(np.float32))


def test_fp32_batch_exact_integers_32bit_index():
    # The production batch kernel (32-bit tile offsets, every tile variant via
    # the table) on the batch workload's shape distribution, every problem
    # compared element by element.
    rng = np.random.default_rng(162)
    shapes = mi.batch_shapes(rng, 800)
    a_s = [_ints32(rng, sa) for sa, _ in shapes]
    b_s = [_ints32(rng, sb) for _, sb in shapes]
    for variant in BATCH_VARIANTS:
        pool = GuardPool([(moa.inner_shape(sa, sb), torch.float32) for sa, sb in shapes])
        say("batch exact, tile variant", variant)
        with _tile_variant(variant):
            bt = moa.Batch([gpu(a) for a in a_s], [gpu(b) for b in b_s], pool.t)
        bt.run()
        pool.check("exact batch, variant %d" % variant)
        for a, b, d in zip(a_s, b_s, pool.t):
            eq(host(d), _exact_tensordot(a, a.ndim - 1, b, 0))
        bt.close()


# ---------------------------------------------------------------------------
# Split products with K past 8192: the INT8 kernel folds its INT32 levels into
# FP64 in the middle of the loop (every 8192 k), the FP8 product runs as three
# 4096-k slab launches (the last one partial) that accumulate in D, and the
# BF16 kernel ends inside its 256-k fold cycle.

@pytest.mark.parametrize("fmt,S,beta", [("bf16", 5, 9), ("int8", 7, 7), ("fp8", 10, 5)])
def test_split_contraction_longer_than_8192(fmt, S, beta):
    rng = np.random.default_rng(163)
    a = mi.scaled_f64(rng, (200, 12000))
    b = mi.scaled_f64(rng, (12000, 150))
    say("split", fmt, "200 x 12000 . 12000 x 150")
    d = host(G.inner_split(gpu(a), gpu(b), fmt, S))
    rows = np.sort(np.concatenate([[0, 199], rng.choice(np.arange(1, 199), 14, replace=False)]))
    want = oracle.split_inner(a, b, nslices=S, beta=beta, rows=rows)
    assert nerr(d[rows], want) <= scheme_tol(fmt, S), nerr(d[rows], want)
    ref = oracle.inner_dot2(a, b, rows=rows)
    assert nerr(d[rows], ref) <= 1e-12, nerr(d[rows], ref)


# ---------------------------------------------------------------------------
# Contractions long enough that a slice stream reaches 2^31 bytes: the
# pipelined kernels' buffer descriptors cannot reach that far, so these run the
# plain-loop kernels (BF16, INT8) and the single-launch FP8 kernel. The INT8
# case also needs more than 65535 row bands in the column scan. A
# componentwise bound (error over sum |a_k b_k|) allows the FP64 folds of
# ~10^5 partial sums; a wrong index or a missed stage is off by far more.

@pytest.mark.parametrize("fmt,S,K", [("bf16", 5, 6_800_000), ("int8", 7, 9_700_000), ("fp8", 10, 3_400_000)])
def test_split_contraction_past_the_descriptor_reach(fmt, S, K):
    rng = np.random.default_rng(191)
    a = mi.scaled_f64(rng, (2, K))
    b = mi.scaled_f64(rng, (K, 3))
    say("split", fmt, "2 x %d . %d x 3" % (K, K))
    d = host(G.inner_split(gpu(a), gpu(b), fmt, S))
    ref = oracle.inner_dot2(a, b)
    err = oracle.componentwise_error(d, ref, oracle.abs_product(a, b))
    assert err <= 1e-11, err


# ---------------------------------------------------------------------------
# Differentiation through torch.autograd: MoaInner.apply forward, the
# hand-written backward through torch.autograd.grad, against FP64 central
# differences (L = <G, D> is linear in each element, so they are exact up to
# rounding).

def test_grad_finite_differences_through_autograd():
    rng = mi.rng_for(mi.DIFFERENTIATION, salt=1)
    a = mi.uniform_f64(rng, (4, 4, 8))
    b = mi.uniform_f64(rng, (8, 4, 4))
    g = mi.uniform_f64(rng, (4, 4, 4, 4))
    ta = gpu(a).requires_grad_(True)
    tb = gpu(b).requires_grad_(True)
    gg = gpu(g)
    say("grad FD through MoaInner.apply")
    loss = torch.sum(moa.MoaInner.apply(ta, tb) * gg)
    da, db = torch.autograd.grad(loss, (ta, tb))
    da, db = host(da), host(db)
    h = 2.0 ** -8

    def L(x, y):
        with torch.no_grad():
            return float(torch.sum(moa.MoaInner.apply(gpu(x), gpu(y)) * gg).item())

    fa = np.zeros_like(a)
    for idx in np.ndindex(a.shape):
        ap, am = a.copy(), a.copy()
        ap[idx] += h
        am[idx] -= h
        fa[idx] = (L(ap, b) - L(am, b)) / (2 * h)
    fb = np.zeros_like(b)
    for idx in np.ndindex(b.shape):
        bp, bm = b.copy(), b.copy()
        bp[idx] += h
        bm[idx] -= h
        fb[idx] = (L(a, bp) - L(a, bm)) / (2 * h)
    assert np.max(np.abs(fa - da)) <= 1e-12
    assert np.max(np.abs(fb - db)) <= 1e-12
    # Only the input that needs a gradient gets one.
    tc = gpu(b)
    (only_a,) = torch.autograd.grad(torch.sum(moa.MoaInner.apply(ta, tc) * gg), (ta,))
    eq(host(only_a), da)


# ---------------------------------------------------------------------------
# NaN and signed zero: FP max/min are the IEEE 754-2019 maximum/minimum and
# FP folds equal the left fold from the first term, on every fold path,
# compared bit for bit.

SPECIAL = np.array([-0.0, 0.0, -0.0, 0.0, 1.0, -1.0, 2.0, -2.0, np.inf, np.nan], dtype=np.float64)


def _special(rng, shape, dt, nan=True):
    pool = SPECIAL if nan else SPECIAL[:-1]
    return np.ascontiguousarray(rng.choice(pool, size=shape).astype(dt))


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_nan_and_signed_zero_sequential_folds(dt):
    rng = np.random.default_rng(170)
    for sa, sb in [((37, 19), (19, 53)), ((6, 1), (1, 9)), ((133, 21), (21, 70))]:
        a, b = _special(rng, sa, dt), _special(rng, sb, dt)
        ga, gb = gpu(a), gpu(b)
        for op1 in FOLD_F:
            for op2 in ELEM_F:
                say("special values, simt", np.dtype(dt).name, sa, sb, op1, op2)
                got = host(G.inner_ex(ga, gb, op1, op2, flags=moa.FLAG_SEQUENTIAL_FOLD))
                eq(got, oracle.inner(a, b, op1, op2, mode="native"))


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_nan_and_signed_zero_few_rows_and_columns(dt):
    # Few rows (the row-form stream) for every fold, few columns (the
    # cross-lane reduction) for max and min: both bit for bit.
    rng = np.random.default_rng(171)
    a, b = _special(rng, (3, 64), dt), _special(rng, (64, 4100), dt)
    ga, gb = gpu(a), gpu(b)
    for op1 in FOLD_F:
        for op2 in ("add", "mul", "max", "min"):
            say("special values, few rows", np.dtype(dt).name, op1, op2)
            eq(host(G.inner(ga, gb, op1, op2)), oracle.inner(a, b, op1, op2, mode="native"))
    # Mostly zeros and ones with a few NaNs: max/min results often tie at +-0.
    a = np.ascontiguousarray(rng.choice(SPECIAL[:5], size=(70, 600)).astype(dt))
    b = np.ascontiguousarray(rng.choice(SPECIAL[:5], size=(600, 5)).astype(dt))
    a[3, 7] = np.nan
    for op1 in ("max", "min"):
        for op2 in ("add", "mul", "max", "min", "sub"):
            say("special values, few columns", np.dtype(dt).name, op1, op2)
            eq(host(G.inner(gpu(a), gpu(b), op1, op2)), oracle.inner(a, b, op1, op2, mode="native"))


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_nan_and_signed_zero_outer(dt):
    rng = np.random.default_rng(172)
    a, b = _special(rng, (17, 3), dt), _special(rng, (2, 129), dt)
    for op in ELEM_F:
        eq(host(G.outer(gpu(a), gpu(b), op)), oracle.outer(a, b, op))


# ---------------------------------------------------------------------------
# Few-row stream instances that the cache-resident path never reaches: B
# larger than 64 MiB or at least 1024 column blocks keep every row in one
# thread (row groups of 2, 4 or 8; rows past M repeat row M - 1 unstored),
# one or four 16-byte runs per thread, ragged and unaligned column counts.

SKINNY_BIG = [
    (np.float64, 5, 16, 600_001, "FP64, R = 1, row group 8, ragged N"),
    (np.float64, 3, 16, 600_000, "FP64, R = 1, row group 4, vector loads"),
    (np.float64, 7, 8, 1_048_578, "FP64, R = 4, row group 8, vector loads"),
    (np.float64, 3, 8, 1_048_579, "FP64, R = 4, row group 4, odd N"),
    (np.int32, 8, 8, 1_100_003, "int32, R = 1, row group 8, odd N"),
    (np.int32, 3, 8, 2_100_004, "int32, R = 4, row group 4, vector loads"),
    (np.int32, 5, 8, 2_100_001, "int32, R = 4, row group 8, odd N"),
]


@pytest.mark.parametrize("case", SKINNY_BIG, ids=[c[4] for c in SKINNY_BIG])
def test_few_rows_all_rows_per_thread(case):
    dt, M, K, N, what = case
    rng = np.random.default_rng(173)
    a, b = rand(rng, (M, K), dt), rand(rng, (K, N), dt)
    ga, gb = gpu(a), gpu(b)
    pairs = ([("add", "mul"), ("max", "add"), ("min", "sub"), ("xor", "and")] if dt == np.int32 else
             [("add", "mul"), ("max", "add"), ("min", "sub"), ("mul", "div")])
    for op1, op2 in pairs:
        say("few rows", what, op1, op2)
        eq(host(G.inner(ga, gb, op1, op2)), oracle.inner(a, b, op1, op2, mode="native"))



# ---------------------------------------------------------------------------
# FP8 (E4M3) slices: 5-bit signed digits, exact FP32 levels folded every
# 4096 k, so the GPU sums the oracle's scheme exactly (up to FP64 rounding).

@pytest.mark.parametrize("shape", [(100, 300, 70), (64, 64, 128), (1, 1, 1), (257, 1000, 131), (33, 65, 200)])
def test_split_fp8_matches_oracle_scheme(shape):
    M, K, N = shape
    rng = np.random.default_rng(180)
    a = mi.scaled_f64(rng, (M, K))
    b = mi.scaled_f64(rng, (K, N))
    ref = oracle.inner_dot2(a, b)
    for S in range(1, 11):
        say("split fp8", shape, "S", S)
        d = host(G.inner_split(gpu(a), gpu(b), "fp8", S))
        want = oracle.split_inner(a, b, nslices=S, beta=5)
        assert nerr(d, want) <= scheme_tol("fp8", S), (S, nerr(d, want))
        if S >= 10:
            assert nerr(d, ref) <= 1e-12, (S, nerr(d, ref))


def test_split_fp8_exact_integers():
    # Integers in [-15, 15] whose row/column maximum lies in [8, 16) are one
    # signed 5-bit digit each: one FP8 slice gives the exact product.
    rng = np.random.default_rng(181)
    a = mi.small_int_f64(rng, (90, 700), 15)
    b = mi.small_int_f64(rng, (700, 70), 15)
    a[:, 3] = 9.0
    b[5, :] = -12.0
    say("split fp8 exact integers")
    d = host(G.inner_split(gpu(a), gpu(b), "fp8", 1))
    eq(d, (a.astype(np.int64) @ b.astype(np.int64)).astype(np.float64))


def test_split_fp8_full_size_sampled():
    a, b = mi.workload_split()
    say("split fp8 8192^3 S=10")
    d = G.inner_split(gpu(a), gpu(b), "fp8", 10)
    rows = _sample_rows(np.random.default_rng(10), 8192, 10)
    got = host(d[torch.from_numpy(rows).to(DEV)])
    ref = oracle.inner_dot2(a, b, rows=rows)
    e = nerr(got, ref)
    scale = oracle.abs_product(a, b, rows=rows)
    say("split fp8 8192^3 vs Dot2: normwise %.3e, max-norm %.3e, componentwise %.3e"
        % (e, oracle.maxnorm_error(got, ref), oracle.componentwise_error(got, ref, scale)))
    assert e <= 1e-12
    want = oracle.split_inner(a, b, nslices=10, beta=5, rows=rows[:4])
    assert nerr(got[:4], want) <= 1e-14
