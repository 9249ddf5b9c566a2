"""Pins for the CPU oracle: checks against what the paper and mathematics fix.

None of these retype the oracle's formulas. They use the worked example of
Section I, independent brute force over full index tuples, library routines
that compute the same special cases (NumPy tensordot / matmul / ufunc.outer),
exact rational arithmetic, and invariants of Eq. inner and Eq. outer.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
import moa_inputs as mi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

FOLD_F = ["add", "mul", "max", "min"]
ELEM_F = ["add", "sub", "mul", "div", "max", "min"]
FOLD_I = ["add", "mul", "max", "min", "and", "or", "xor"]
ELEM_I = ["add", "sub", "mul", "max", "min", "and", "or", "xor"]


def _rand(rng, shape, dtype):
    if dtype == np.int32:
        return mi.uniform_i32(rng, shape, -50, 50)
    x = rng.uniform(0.5, 2.0, size=shape) * rng.choice([-1.0, 1.0], size=shape)
    return np.ascontiguousarray(x.astype(dtype))


def _equal(x, y):
    """Equal bit for bit (so +0 and -0 differ); any NaN matches any NaN."""
    x = np.asarray(x)
    y = np.asarray(y)
    assert x.shape == y.shape and x.dtype == y.dtype, (x.shape, y.shape, x.dtype, y.dtype)
    if x.dtype.kind == "f":
        u = np.dtype("u%d" % x.dtype.itemsize)
        both_nan = np.isnan(x) & np.isnan(y)
        same = x.view(u) == y.view(u)
        assert np.all(same | both_nan), (x[~(same | both_nan)][:4], y[~(same | both_nan)][:4])
    else:
        assert np.array_equal(x, y)


# --------------------------------------------------------------------------
# Worked example (Section I, Fig. inner_fig).

def test_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    for dt in (np.float64, np.float32, np.int32):
        a = np.array(g["A"], dtype=dt).reshape(g["A_shape"])
        b = np.array(g["B"], dtype=dt).reshape(g["B_shape"])
        d = oracle.inner(a, b, "add", "mul", mode="native")
        assert d.shape == tuple(g["inner_add_mul"]["shape"])
        assert np.array_equal(d.ravel(), np.array(g["inner_add_mul"]["value"], dtype=dt))
        t = oracle.inner(a, b, "max", "add", mode="native")
        assert np.array_equal(t.ravel(), np.array(g["inner_max_add"]["value"], dtype=dt))
        c = oracle.outer(a, b, "mul")
        assert c.shape == tuple(g["outer_mul"]["shape"])
        for idx, v in g["outer_mul"]["spot"]:
            assert c[tuple(idx)] == v


def test_worked_example_row_form():
    # <0> psi C is A[0,0]*<0>psiB + A[0,1]*<1>psiB + A[0,2]*<2>psiB (Section I).
    a = np.arange(6, dtype=np.int32).reshape(2, 3)
    b = np.arange(12, dtype=np.int32).reshape(3, 4)
    d = oracle.inner(a, b)
    assert np.array_equal(d[0], 0 * b[0] + 1 * b[1] + 2 * b[2])


# --------------------------------------------------------------------------
# Brute force over full index tuples, every op pair and dtype.

SHAPE_PAIRS = [
    ((3,), (3,)),            # rank-0 result
    ((2, 3), (3, 4)),        # the worked-example shapes
    ((1, 1), (1, 1)),
    ((2, 1, 3), (3, 2)),
    ((4,), (4, 2, 3)),
    ((2, 2, 1, 2), (2, 1, 3)),
    ((3, 1), (1, 5)),        # K = 1
    ((5, 2), (2,)),
]


@pytest.mark.parametrize("dt", [np.float64, np.float32, np.int32])
def test_inner_matches_brute_force_all_pairs(dt):
    rng = np.random.default_rng(11)
    folds = FOLD_I if dt == np.int32 else FOLD_F
    elems = ELEM_I if dt == np.int32 else ELEM_F
    for sa, sb in SHAPE_PAIRS:
        a = _rand(rng, sa, dt)
        b = _rand(rng, sb, dt)
        for op1 in folds:
            for op2 in elems:
                want = brute.inner(a, b, op1, op2)
                got = oracle.inner(a, b, op1, op2, mode="native")
                _equal(got, want)


@pytest.mark.parametrize("dt", [np.float64, np.float32, np.int32])
def test_outer_matches_brute_force(dt):
    rng = np.random.default_rng(12)
    elems = ELEM_I if dt == np.int32 else ELEM_F
    for sa, sb in [((), ()), ((3,), ()), ((), (2, 2)), ((2, 3), (3, 4)), ((2, 1, 2), (3,))]:
        a = _rand(rng, sa, dt)
        b = _rand(rng, sb, dt)
        for op in elems:
            _equal(oracle.outer(a, b, op), brute.outer(a, b, op))


def test_empty_contraction_gives_identity():
    for dt, folds in ((np.float64, FOLD_F), (np.int32, FOLD_I)):
        a = np.zeros((3, 0), dtype=dt)
        b = np.zeros((0, 2), dtype=dt)
        for op1 in folds:
            d = oracle.inner(a, b, op1, "add" if dt == np.float64 else "xor")
            want = np.full((3, 2), oracle.identity_of(op1, dt), dtype=dt)
            assert np.array_equal(d, want)


def test_empty_axes():
    a = np.zeros((0, 4), dtype=np.float64)
    b = np.ones((4, 3), dtype=np.float64)
    assert oracle.inner(a, b).shape == (0, 3)
    assert oracle.outer(a, b).shape == (0, 4, 4, 3)


def test_rejects_bad_shapes():
    with pytest.raises(ValueError):
        oracle.inner(np.zeros((2, 3)), np.zeros((4, 2)))
    with pytest.raises(ValueError):
        oracle.inner(np.zeros(()), np.zeros((1,)))


# --------------------------------------------------------------------------
# Library special cases.

def test_matmul_special_case():
    # Rank-2 (+,*) is the standard matrix product (Section I).
    rng = np.random.default_rng(13)
    a = mi.uniform_f64(rng, (37, 53))
    b = mi.uniform_f64(rng, (53, 29))
    d = oracle.inner(a, b)
    assert np.allclose(d, a @ b, rtol=0, atol=1e-13)
    ai = mi.uniform_i32(rng, (17, 40))
    bi = mi.uniform_i32(rng, (40, 9))
    assert np.array_equal(oracle.inner(ai, bi), (ai.astype(np.int64) @ bi.astype(np.int64)).astype(np.int32))


def test_tensordot_any_rank():
    # Eq. inner with + and * is a tensor contraction of the last axis of A with
    # the first axis of B: numpy.tensordot(A, B, axes=1).
    rng = np.random.default_rng(14)
    for sa, sb in [((2, 3, 4, 5), (5, 3, 2)), ((7, 6), (6, 2, 2, 2)), ((3,), (3, 4, 5)), ((4, 2, 9), (9,))]:
        a = mi.uniform_f64(rng, sa)
        b = mi.uniform_f64(rng, sb)
        want = np.tensordot(a, b, axes=1)
        got = oracle.inner(a, b)
        assert got.shape == want.shape
        assert oracle.normwise_error(got, want) < 1e-15
        ai = mi.uniform_i32(rng, sa)
        bi = mi.uniform_i32(rng, sb)
        wi = np.tensordot(ai.astype(np.int64), bi.astype(np.int64), axes=1)
        assert np.array_equal(oracle.inner(ai, bi), wi.astype(np.int32))


def test_int32_wraps():
    a = np.array([[2 ** 30, 2 ** 30, 2 ** 30]], dtype=np.int32)
    b = np.array([[2], [2], [1]], dtype=np.int32)
    # 2^31 + 2^31 + 2^30 = 5 * 2^30, wrapped to int32.
    want = np.array([[(5 * 2 ** 30 + 2 ** 31) % 2 ** 32 - 2 ** 31]], dtype=np.int64).astype(np.int32)
    assert np.array_equal(oracle.inner(a, b), want)


@pytest.mark.parametrize("dt", [np.float64, np.float32, np.int32])
def test_outer_matches_ufunc_outer(dt):
    rng = np.random.default_rng(15)
    a = _rand(rng, (4, 3), dt)
    b = _rand(rng, (2, 5), dt)
    table = {"add": np.add, "sub": np.subtract, "mul": np.multiply, "max": np.maximum, "min": np.minimum}
    if dt == np.int32:
        table.update({"and": np.bitwise_and, "or": np.bitwise_or, "xor": np.bitwise_xor})
    else:
        table["div"] = np.divide
    for name, uf in table.items():
        with np.errstate(all="ignore"):
            want = uf.outer(a, b)
        if dt == np.int32:
            want = want.astype(np.int32)
        _equal(oracle.outer(a, b, name), want)


def test_f32_native_fold_matches_numpy_scalar_fold():
    # An FP32 fold in native mode is a sequence of FP32 operations in
    # ascending l; numpy float32 scalars compute the same sequence.
    rng = np.random.default_rng(16)
    a = mi.uniform_f32(rng, (3, 50))
    b = mi.uniform_f32(rng, (50, 4))
    got = oracle.inner(a, b, "add", "sub", mode="native")
    for i in range(3):
        for j in range(4):
            acc = np.float32(a[i, 0] - b[0, j])
            for l in range(1, 50):
                acc = np.float32(acc + np.float32(a[i, l] - b[l, j]))
            assert got[i, j] == acc
    wide = oracle.inner(a, b, "add", "sub", mode="wide")
    assert wide.dtype == np.float64
    assert np.allclose(wide, got, rtol=1e-5)


def test_sampled_rows_match_full():
    rng = np.random.default_rng(17)
    a = mi.uniform_f64(rng, (4, 3, 8))
    b = mi.uniform_f64(rng, (8, 5))
    full = oracle.inner(a, b, "max", "mul").reshape(12, 5)
    rows = [11, 0, 5]
    part = oracle.inner(a, b, "max", "mul", rows=rows)
    assert np.array_equal(part, full[rows])
    assert np.array_equal(oracle.inner_dot2(a, b, rows=rows), oracle.inner_dot2(a, b).reshape(12, 5)[rows])


# --------------------------------------------------------------------------
# Invariants of Eq. inner / Eq. outer.

def test_inner_is_outer_reduced_on_paired_axes():
    rng = np.random.default_rng(18)
    for op1, op2, dt in [("add", "mul", np.int32), ("max", "add", np.int32), ("min", "sub", np.int32),
                         ("xor", "and", np.int32), ("max", "mul", np.float64)]:
        a = _rand(rng, (2, 3, 4), dt)
        b = _rand(rng, (4, 2, 3), dt)
        c = oracle.outer(a, b, op2)                  # shape 2 3 4 4 2 3
        diag = np.diagonal(c, axis1=2, axis2=3)      # shape 2 3 2 3 4 (paired axes last)
        red = {"add": lambda x: np.add.reduce(x.astype(np.int64), axis=-1).astype(dt),
               "max": lambda x: np.max(x, axis=-1), "min": lambda x: np.min(x, axis=-1),
               "xor": lambda x: np.bitwise_xor.reduce(x, axis=-1)}[op1]
        _equal(oracle.inner(a, b, op1, op2), red(diag))


def test_k1_inner_is_outer():
    rng = np.random.default_rng(19)
    a = mi.uniform_f64(rng, (3, 4))
    b = mi.uniform_f64(rng, (2, 5))
    for op in ELEM_F:
        d = oracle.inner(a.reshape(3, 4, 1), b.reshape(1, 2, 5), "add", op)
        _equal(d, oracle.outer(a, b, op))


def test_identity_operands():
    rng = np.random.default_rng(20)
    a = mi.uniform_i32(rng, (3, 2, 6))
    eye = np.eye(6, dtype=np.int32)
    assert np.array_equal(oracle.inner(a, eye), a)
    b = mi.uniform_i32(rng, (6, 4, 2))
    assert np.array_equal(oracle.inner(eye, b), b)
    # Tropical identity: 0 on the diagonal, a large negative sentinel off it.
    big = -(2 ** 30)
    te = np.full((6, 6), big, dtype=np.int32)
    np.fill_diagonal(te, 0)
    assert np.array_equal(oracle.inner(a, te, "max", "add"), a)
    assert np.array_equal(oracle.inner(te, b, "max", "add"), b)
    tm = -te
    assert np.array_equal(oracle.inner(a, tm, "min", "add"), a)
    # Boolean identity for (or, and).
    bits = (mi.uniform_i32(rng, (4, 6), 0, 1)).astype(np.int32)
    assert np.array_equal(oracle.inner(bits, eye, "or", "and"), bits)
    # FP64 identity is exact.
    af = mi.uniform_f64(rng, (5, 6))
    assert np.array_equal(oracle.inner(af, np.eye(6)), af)


def test_associativity_exact_semirings():
    rng = np.random.default_rng(21)
    for op1, op2 in [("add", "mul"), ("max", "add"), ("min", "add"), ("or", "and"), ("xor", "and")]:
        a = mi.uniform_i32(rng, (3, 4), -20, 20)
        b = mi.uniform_i32(rng, (4, 5), -20, 20)
        c = mi.uniform_i32(rng, (5, 2), -20, 20)
        left = oracle.inner(oracle.inner(a, b, op1, op2), c, op1, op2)
        right = oracle.inner(a, oracle.inner(b, c, op1, op2), op1, op2)
        assert np.array_equal(left, right), (op1, op2)


def test_power_of_two_row_scaling():
    rng = np.random.default_rng(22)
    a = mi.uniform_f64(rng, (6, 40))
    b = mi.uniform_f64(rng, (40, 7))
    d = oracle.inner(a, b)
    a2 = a.copy()
    a2[3] = np.ldexp(a2[3], 5)
    d2 = oracle.inner(a2, b)
    assert np.array_equal(d2[3], np.ldexp(d[3], 5))
    assert np.array_equal(np.delete(d2, 3, 0), np.delete(d, 3, 0))


# --------------------------------------------------------------------------
# Dot2 against exact rational arithmetic.

def _exact_dot(a, b):
    return sum((Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b)), Fraction(0))


def test_dot2_against_exact_rationals():
    rng = np.random.default_rng(23)
    a = mi.scaled_f64(rng, (4, 300))
    b = mi.scaled_f64(rng, (300, 3))
    d = oracle.inner_dot2(a, b)
    for i in range(4):
        for j in range(3):
            ex = _exact_dot(a[i], b[:, j])
            # Dot2 is as accurate as a twice-working-precision dot product,
            # then rounded: error <= u|s| + gamma_n^2 * sum|a b| (Ogita-Rump-Oishi).
            u = 2.0 ** -53
            n = 300
            g = n * u / (1 - n * u)
            bound = u * abs(float(ex)) + g * g * float(sum(abs(Fraction(float(x)) * Fraction(float(y)))
                                                          for x, y in zip(a[i], b[:, j])))
            assert abs(Fraction(float(d[i, j])) - ex) <= Fraction(bound)


def test_dot2_ill_conditioned_exact():
    # Catastrophic cancellation: plain FP64 loses everything, Dot2 is exact.
    a = np.array([[1e16, 1.0, -1e16, 3.0]])
    b = np.array([[1.0], [1.0], [1.0], [1.0]])
    assert oracle.inner_dot2(a, b)[0, 0] == 4.0
    assert oracle.inner(a, b)[0, 0] != 4.0


# --------------------------------------------------------------------------
# Split scheme (Ozaki et al. 2012), signed digits.

@pytest.mark.parametrize("fmt,beta", [("bf16", 8), ("bf16", 9), ("fp8", 5), ("bf16", 7)])
def test_split_digits_bounds_and_exact_reconstruction(fmt, beta):
    rng = np.random.default_rng(24)
    x = mi.scaled_f64(rng, (20, 33))
    S = (53 + 17 + beta - 1) // beta + 1
    for by_rows in (True, False):
        e, sig = oracle.split_digits(x, by_rows=by_rows, fmt=fmt, nslices=S, beta=beta)
        assert np.abs(sig).max() <= 2 ** (beta - 1)
        # Rebuild with exact rationals: x = 2^e * sum_s sigma_s 2^-(beta-1+beta*s).
        for i in range(x.shape[0]):
            for l in range(x.shape[1]):
                ex = int(e[i] if by_rows else e[l])
                v = sum(Fraction(int(sig[s, i, l])) * Fraction(2) ** (-(beta - 1) - beta * s) for s in range(S))
                assert v * Fraction(2) ** ex == Fraction(float(x[i, l]))
        # Scaled values lie in (-1, 1): row/column maxima are below 2^e.
        mx = np.abs(x).max(axis=1 if by_rows else 0)
        assert np.all(mx < np.ldexp(1.0, e)) and np.all(mx >= np.ldexp(0.5, e))


def test_split_digit_representable_in_format():
    # Every digit must be an integer the slice format holds exactly.
    import torch
    rng = np.random.default_rng(25)
    x = mi.scaled_f64(rng, (16, 64))
    _, sig = oracle.split_digits(x, fmt="bf16", nslices=5, beta=9)
    t = torch.from_numpy(sig.astype(np.float32))
    assert torch.equal(t.to(torch.bfloat16).to(torch.float32), t)
    _, sig8 = oracle.split_digits(x, fmt="fp8", nslices=8)
    t8 = torch.from_numpy(sig8.astype(np.float32))
    assert torch.equal(t8.to(torch.float8_e4m3fn).to(torch.float32), t8)
    # 7-bit signed digits fit INT8.
    _, sig7 = oracle.split_digits(x, nslices=7, beta=7)
    assert np.array_equal(sig7.astype(np.int8).astype(np.int32), sig7)


def test_split_exact_for_small_integers():
    # Integer entries whose row / column maxima lie in [2^(beta-2), 2^(beta-1))
    # are one digit each, so one slice reproduces the exact integer product.
    rng = np.random.default_rng(26)
    a = mi.small_int_f64(rng, (9, 70), 127)
    b = mi.small_int_f64(rng, (70, 11), 127)
    a[:, 0] = 100.0
    b[0, :] = -100.0
    exact = a.astype(np.int64) @ b.astype(np.int64)
    d = oracle.split_inner(a, b, nslices=1, beta=8)
    assert np.array_equal(d, exact.astype(np.float64))


def test_split_full_digits_equals_exact_rounded():
    # With enough slices every pair product is kept to full precision; the only
    # remaining error is the final FP64 slice sum, well inside 4 ulps here.
    rng = np.random.default_rng(27)
    a = mi.scaled_f64(rng, (5, 200))
    b = mi.scaled_f64(rng, (200, 4))
    d = oracle.split_inner(a, b, nslices=9, beta=9)
    for i in range(5):
        for j in range(4):
            ex = float(_exact_dot(a[i], b[:, j]))
            assert abs(d[i, j] - ex) <= 4 * np.spacing(abs(ex)) + 1e-300


def test_split_error_decreases_with_slices_and_meets_bound():
    rng = np.random.default_rng(28)
    a = mi.scaled_f64(rng, (8, 2048))
    b = mi.scaled_f64(rng, (2048, 16))
    ref = oracle.inner_dot2(a, b)
    errs = [oracle.normwise_error(oracle.split_inner(a, b, nslices=s, beta=9), ref) for s in range(1, 7)]
    assert all(errs[i + 1] < errs[i] for i in range(4)), errs
    # Componentwise truncation bound of the triangular scheme: each dropped
    # digit is below 2^-(beta*S) of its row (column) scale, so
    # |D - D_S| <= (S+1) * 2^(e_i+f_j) * K * 2^-(beta*S) * 2 (loose).
    S, beta = 5, 9
    d = oracle.split_inner(a, b, nslices=S, beta=beta)
    ea = np.frexp(np.abs(a).max(axis=1))[1]
    fb = np.frexp(np.abs(b).max(axis=0))[1]
    bound = (S + 1) * 2.0 * a.shape[1] * np.ldexp(1.0, -beta * S) * np.ldexp(1.0, ea[:, None] + fb[None, :])
    assert np.all(np.abs(d - ref) <= bound)


def test_split_power_of_two_scaling_invariance():
    rng = np.random.default_rng(29)
    a = mi.scaled_f64(rng, (6, 300))
    b = mi.scaled_f64(rng, (300, 5))
    d = oracle.split_inner(a, b, nslices=4, beta=9)
    a2 = a.copy()
    a2[2] = np.ldexp(a2[2], -7)
    b2 = b.copy()
    b2[:, 1] = np.ldexp(b2[:, 1], 3)
    d2 = oracle.split_inner(a2, b2, nslices=4, beta=9)
    want = d.copy()
    want[2] = np.ldexp(want[2], -7)
    want[:, 1] = np.ldexp(want[:, 1], 3)
    assert np.array_equal(d2, want)


def test_split_int8_parameters_meet_tolerance_on_workload_distribution():
    # INT8 digits of 7 bits, 7 slices (28 pairs), same distribution.
    rng = mi.rng_for(mi.SPLIT_PRECISION, salt=4)
    a = mi.scaled_f64(rng, (8, 8192))
    b = mi.scaled_f64(rng, (8192, 32))
    ref = oracle.inner_dot2(a, b)
    err = oracle.normwise_error(oracle.split_inner(a, b, nslices=7, beta=7), ref)
    assert err <= 1e-12, err
    # Six slices are not enough at this distribution.
    assert oracle.normwise_error(oracle.split_inner(a, b, nslices=6, beta=7), ref) > 1e-12


def test_split_chosen_parameters_meet_tolerance_on_workload_distribution():
    # BF16 digits of 9 bits, 5 slices (15 slice pairs) on the 2^[-8,8]-scaled
    # distribution, K = 8192, against Dot2.
    rng = mi.rng_for(mi.SPLIT_PRECISION, salt=3)
    a = mi.scaled_f64(rng, (8, 8192))
    b = mi.scaled_f64(rng, (8192, 32))
    ref = oracle.inner_dot2(a, b)
    err = oracle.normwise_error(oracle.split_inner(a, b, nslices=5, beta=9), ref)
    assert err <= 1e-12, err


# --------------------------------------------------------------------------
# Contraction over any axis pair (Section I: Eq. inner as a tensor contraction;
# index maps of Section II.D).

AXES_SHAPES = [((2, 3, 4), 1, (3, 2), 0), ((2, 3, 4), 0, (5, 2), 1), ((3, 2), 0, (2, 4, 3), 2),
               ((4,), 0, (2, 4, 1), 1), ((2, 2, 3), 2, (3,), 0), ((1, 3, 2), 1, (2, 3, 2), 1)]


@pytest.mark.parametrize("dt", [np.float64, np.float32, np.int32])
def test_inner_axes_matches_brute_force(dt):
    rng = np.random.default_rng(31)
    pairs = ([("add", "mul"), ("max", "add"), ("min", "sub"), ("xor", "and")] if dt == np.int32 else
             [("add", "mul"), ("max", "add"), ("min", "sub"), ("mul", "div")])
    for sa, ax_a, sb, ax_b in AXES_SHAPES:
        a = _rand(rng, sa, dt)
        b = _rand(rng, sb, dt)
        for op1, op2 in pairs:
            _equal(oracle.inner_axes(a, ax_a, b, ax_b, op1, op2, mode="native"),
                   brute.inner_axes(a, ax_a, b, ax_b, op1, op2))


def test_inner_axes_is_tensordot():
    rng = np.random.default_rng(32)
    for sa, ax_a, sb, ax_b in AXES_SHAPES + [((5, 6, 7, 3), 2, (2, 7, 4), 1), ((9, 8), 0, (8, 9), 1)]:
        ai = mi.uniform_i32(rng, sa)
        bi = mi.uniform_i32(rng, sb)
        want = np.tensordot(ai.astype(np.int64), bi.astype(np.int64), axes=([ax_a], [ax_b])).astype(np.int32)
        assert np.array_equal(oracle.inner_axes(ai, ax_a, bi, ax_b), want)
        a = mi.uniform_f64(rng, sa)
        b = mi.uniform_f64(rng, sb)
        want = np.tensordot(a, b, axes=([ax_a], [ax_b]))
        assert oracle.normwise_error(oracle.inner_axes(a, ax_a, b, ax_b), want) < 1e-15


def test_inner_axes_last_with_first_is_inner():
    rng = np.random.default_rng(33)
    a = mi.uniform_f64(rng, (3, 4, 5))
    b = mi.uniform_f64(rng, (5, 2))
    _equal(oracle.inner_axes(a, -1, b, 0, "max", "add"), oracle.inner(a, b, "max", "add"))


def test_inner_axes_operand_swap_transposes_result():
    # For a commutative op2, swapping the operands swaps the two groups of
    # free axes of the result and nothing else.
    rng = np.random.default_rng(34)
    a = _rand(rng, (2, 5, 3), np.int32)
    b = _rand(rng, (4, 5), np.int32)
    for op1, op2 in [("add", "mul"), ("max", "min"), ("or", "xor")]:
        d = oracle.inner_axes(a, 1, b, 1, op1, op2)            # axes (2, 3, 4)
        e = oracle.inner_axes(b, 1, a, 1, op1, op2)            # axes (4, 2, 3)
        _equal(np.moveaxis(e, 0, -1), d)


def test_error_measures_pins():
    # Max-norm: hand values.
    assert oracle.maxnorm_error([1.0, -4.0, 2.0], [1.0, -4.0, 2.0]) == 0.0
    assert oracle.maxnorm_error([1.0, -4.5, 2.0], [1.0, -4.0, 2.0]) == 0.125
    # |A| . |B| against brute-force sums of magnitudes.
    a = np.array([[1.0, -2.0, 3.0], [-4.0, 0.5, -1.0]])
    b = np.array([[-1.0, 2.0], [3.0, -0.25], [0.0, -8.0]])
    want = np.array([[sum(abs(a[i, l]) * abs(b[l, j]) for l in range(3)) for j in range(2)] for i in range(2)])
    assert np.array_equal(oracle.abs_product(a, b), want)
    # Componentwise: hand values, zero scale.
    assert oracle.componentwise_error([[3.5]], [[3.0]], [[7.0]]) == 0.5 / 7.0
    assert oracle.componentwise_error([0.0, 1.0], [0.0, 1.0], [0.0, 2.0]) == 0.0
    assert oracle.componentwise_error([1e-300, 1.0], [0.0, 1.0], [0.0, 2.0]) == np.inf


def test_componentwise_error_meets_recursive_summation_bound():
    # A sequential FP32 fold of FP32 operands satisfies |fl - exact| <= gamma_K (|A||B|)
    # with gamma_K = K u / (1 - K u), u = 2^-24 (the textbook bound for a
    # recursively summed dot product); the measured error must sit below it.
    rng = np.random.default_rng(77)
    K = 300
    a = rng.uniform(-1, 1, (20, K)).astype(np.float32)
    b = rng.uniform(-1, 1, (K, 30)).astype(np.float32)
    got = oracle.inner(a, b, mode="native")
    ref = oracle.inner_dot2(a, b)
    u = 2.0 ** -24
    gamma = K * u / (1 - K * u)
    err = oracle.componentwise_error(got, ref, oracle.abs_product(a, b))
    assert 0 < err <= gamma
    # With the signed products in place of magnitudes the "scale" can cancel
    # to near zero and the same error exceeds the bound.
    bad = oracle.componentwise_error(got, ref, np.abs(oracle.inner(a.astype(np.float64), b.astype(np.float64))))
    assert bad > err


def test_normwise_error_hand_values():
    # ||x - ref||_F / ||ref||_F: 3-4-5 triangles make every value exact.
    assert oracle.normwise_error([3.0, 4.0], [3.0, 4.0]) == 0.0
    assert oracle.normwise_error([0.0, 0.0], [3.0, 4.0]) == 1.0
    # The denominator is the reference's norm (5), not the result's (10).
    assert oracle.normwise_error([6.0, 8.0], [3.0, 4.0]) == 1.0
    # Frobenius over a matrix: ||ref||_F = 5, ||x - ref||_F = 3.
    ref = [[1.0, 2.0], [2.0, 4.0]]
    assert oracle.normwise_error([[1.0, 2.0], [2.0, 7.0]], ref) == 0.6
    assert oracle.normwise_error([[2.0, 0.0], [0.0, 4.0]], ref) == 0.6
    # A zero reference: the absolute norm of the difference.
    assert oracle.normwise_error([3.0, -4.0], [0.0, 0.0]) == 5.0


# --------------------------------------------------------------------------
# FP max / min: the IEEE 754-2019 maximum and minimum (NaN if either operand
# is NaN, -0 below +0), the reading taken where the paper is silent on NaN and
# signed zero. These rules make both operations associative and commutative.

NZ, PZ, NAN = -0.0, 0.0, float("nan")


def _bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_max_min_nan_and_signed_zero_hand_values(dt):
    a = np.array([NZ, PZ, NAN, 1.0], dtype=dt)
    b = np.array([PZ, NZ, 2.0], dtype=dt)
    # max: -0 vs +0 gives +0 in either order; NaN wins; otherwise the larger.
    want_max = np.array([[PZ, NZ, 2.0], [PZ, PZ, 2.0], [NAN, NAN, NAN], [1.0, 1.0, 2.0]], dtype=dt)
    want_min = np.array([[NZ, NZ, NZ], [PZ, NZ, PZ], [NAN, NAN, NAN], [PZ, NZ, 1.0]], dtype=dt)
    _equal(oracle.outer(a, b, "max"), want_max)
    _equal(oracle.outer(a, b, "min"), want_min)
    _equal(brute.outer(a, b, "max"), want_max)
    _equal(brute.outer(a, b, "min"), want_min)
    # Fold over [NaN, 5] in either order: NaN (an order-dependent rule such as
    # "a < b ? b : a" gives 5 one way round).
    for row in ([NAN, 5.0], [5.0, NAN]):
        x = np.array([row], dtype=dt)
        z = np.zeros((2, 1), dtype=dt)
        assert np.isnan(oracle.inner(x, z, "max", "add", mode="native")).all()
        assert np.isnan(oracle.inner(x, z, "min", "add", mode="native")).all()
    # Terms (+0, -0) and (-0, +0): max +0, min -0.
    for row in ([1.0, -1.0], [-1.0, 1.0]):
        x = np.array([row], dtype=dt)
        z = np.zeros((2, 1), dtype=dt)
        _equal(oracle.inner(x, z, "max", "mul", mode="native"), np.array([[PZ]], dtype=dt))
        _equal(oracle.inner(x, z, "min", "mul", mode="native"), np.array([[NZ]], dtype=dt))
    # A sum of -0 terms is -0 (the left fold from the first term), a sum of
    # +0 and -0 terms +0.
    x = np.array([[-1.0, -2.0, -3.0]], dtype=dt)
    _equal(oracle.inner(x, np.zeros((3, 1), dtype=dt), "add", "mul", mode="native"), np.array([[NZ]], dtype=dt))
    x = np.array([[-1.0, 2.0, -3.0]], dtype=dt)
    _equal(oracle.inner(x, np.zeros((3, 1), dtype=dt), "add", "mul", mode="native"), np.array([[PZ]], dtype=dt))


def test_max_min_fold_independent_of_order():
    # Any permutation of the terms folds to the same bits (NaN-ness for NaN).
    rng = np.random.default_rng(61)
    pool = np.array([NZ, PZ, NZ, PZ, 1.5, -1.5, np.inf, -np.inf, NAN, 3.0], dtype=np.float64)
    for trial in range(200):
        terms = rng.choice(pool, size=rng.integers(1, 7))
        if trial % 3:
            terms = terms[~np.isnan(terms)] if (~np.isnan(terms)).any() else terms
        for op in ("max", "min"):
            a = terms[None, :]
            b = np.zeros((len(terms), 1))
            want = oracle.inner(a, b, op, "add")
            for _ in range(4):
                p = rng.permutation(len(terms))
                got = oracle.inner(terms[p][None, :], b, op, "add")
                if np.isnan(want).all():
                    assert np.isnan(got).all()
                else:
                    assert _bits(got) == _bits(want), (op, terms, p)


def test_max_min_with_nan_and_zeros_match_brute_force():
    rng = np.random.default_rng(62)
    pool = np.array([NZ, PZ, 1.0, -1.0, 2.0, NAN, np.inf], dtype=np.float64)
    for dt in (np.float64, np.float32):
        a = rng.choice(pool, size=(3, 4, 5)).astype(dt)
        b = rng.choice(pool, size=(5, 6)).astype(dt)
        for op1 in ("max", "min", "add", "mul"):
            for op2 in ("add", "mul", "max", "min"):
                _equal(oracle.inner(a, b, op1, op2, mode="native"), brute.inner(a, b, op1, op2))


def test_split_s5_beta9_meets_tolerance_on_more_seeds():
    # The chosen BF16 parameters (9-bit digits, 5 slices) on six further
    # seeds of the workload distribution (entries u 2^k, k in [-8, 8]) at
    # K = 8192, each against Dot2; all must stay within 1e-12.
    errs = []
    for salt in (11, 12, 13, 14, 15, 16):
        rng = mi.rng_for(mi.SPLIT_PRECISION, salt=salt)
        a = mi.scaled_f64(rng, (8, 8192))
        b = mi.scaled_f64(rng, (8192, 24))
        ref = oracle.inner_dot2(a, b)
        errs.append(oracle.normwise_error(oracle.split_inner(a, b, nslices=5, beta=9), ref))
    assert max(errs) <= 1e-12, errs


def test_split_fp8_parameters_meet_tolerance_on_workload_distribution():
    # FP8 E4M3 digits of 5 bits: 10 slices (55 pairs) meet 1e-12 with a wide
    # margin on the workload distribution at K = 8192; 8 slices do not.
    rng = mi.rng_for(mi.SPLIT_PRECISION, salt=5)
    a = mi.scaled_f64(rng, (8, 8192))
    b = mi.scaled_f64(rng, (8192, 24))
    ref = oracle.inner_dot2(a, b)
    assert oracle.normwise_error(oracle.split_inner(a, b, nslices=10, beta=5), ref) <= 1e-13
    assert oracle.normwise_error(oracle.split_inner(a, b, nslices=8, beta=5), ref) > 1e-12
