"""Seeded synthetic inputs for the MoA generalized inner/outer product workloads.

This module only draws random arrays and shapes. It holds none of the
arithmetic of the method: the oracle (``oracle/``) and the HIP path
(``paper_0907_0792_amd``) both consume what it returns, and neither of them is
imported here.

Every generator takes a NumPy ``Generator`` or a seed and returns host arrays
(row-major, contiguous) together with their shape vectors, which is how the
paper describes an array: a shape vector plus a flat vector of elements
(Section I).

Workloads (value distributions as stated for each workload):

* ``plain_f64``      FP64 (+,*) inner product, entries uniform[-1, 1].
* ``outer``          outer product of two arrays, any dtype.
* ``tropical_i32``   int32 (max,+) inner product, entries uniform in [-1000, 1000].
* ``split_f64``      FP64 entries u * 2**k, u ~ uniform[-1, 1], k ~ uniform{-8..8}.
* ``batch_f32``      many uneven FP32 (+,*) inner products (shape recipe below).
* ``grad_f32``       FP32 forward operands plus an upstream gradient G.

Seeds: workload number ``c`` uses ``numpy.random.default_rng(1000 + c)``; the
draw order is A, then B, then (batch) shapes before values, then (grad) G.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Workload numbers used for seeding (1000 + number).
SMALL_MIXED = 0       # 512^3 FP64 (+,*) plus a <32 32> x <16 16> FP64 outer product
RANK_GENERAL = 1      # rank-5 FP64 (+,*), 2048^3 int32 (max,+), FP32 (-) outer
SPLIT_PRECISION = 2   # 8192^3 FP64 at FP64 accuracy from BF16 slices
BATCH = 3             # 10,000 uneven FP32 (+,*) products
DIFFERENTIATION = 4   # FP32 forward + backward


def rng_for(workload: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng(1000 + workload + 7919 * salt)


def _as_rng(rng_or_seed) -> np.random.Generator:
    if isinstance(rng_or_seed, np.random.Generator):
        return rng_or_seed
    return np.random.default_rng(rng_or_seed)


def uniform_f64(rng, shape) -> np.ndarray:
    rng = _as_rng(rng)
    return np.asarray(rng.uniform(-1.0, 1.0, size=tuple(shape)), dtype=np.float64, order="C")


def uniform_f32(rng, shape) -> np.ndarray:
    return uniform_f64(rng, shape).astype(np.float32)


def uniform_i32(rng, shape, lo=-1000, hi=1000) -> np.ndarray:
    rng = _as_rng(rng)
    return np.asarray(rng.integers(lo, hi + 1, size=tuple(shape)), dtype=np.int32, order="C")


def scaled_f64(rng, shape, kmin=-8, kmax=8) -> np.ndarray:
    """Entries u * 2**k with u ~ uniform[-1,1] and integer k ~ uniform{kmin..kmax}.

    The power of two is applied with ``ldexp`` so the scaling itself is exact.
    """
    rng = _as_rng(rng)
    u = rng.uniform(-1.0, 1.0, size=tuple(shape))
    k = rng.integers(kmin, kmax + 1, size=tuple(shape))
    return np.asarray(np.ldexp(u, k), dtype=np.float64, order="C")


def small_int_f64(rng, shape, bound) -> np.ndarray:
    """Integer-valued FP64 entries in [-bound, bound] (exact-arithmetic cases)."""
    rng = _as_rng(rng)
    return np.asarray(rng.integers(-bound, bound + 1, size=tuple(shape)), dtype=np.float64, order="C")


def random_factorisation(rng: np.random.Generator, n: int, parts: int) -> list[int]:
    """A uniformly drawn ordered factorisation of ``n`` into ``parts`` factors (factors may be 1)."""
    out = []
    rest = n
    for _ in range(parts - 1):
        divs = [d for d in range(1, rest + 1) if rest % d == 0]
        d = int(divs[rng.integers(0, len(divs))])
        out.append(d)
        rest //= d
    out.append(rest)
    return out


@dataclass
class Problem:
    shape_a: tuple
    shape_b: tuple
    a: np.ndarray
    b: np.ndarray

    @property
    def mkn(self):
        m = math.prod(self.shape_a[:-1])
        k = self.shape_a[-1]
        n = math.prod(self.shape_b[1:])
        return m, k, n


def batch_shapes(rng, count, mn_range=(4, 64), k_range=(16, 512), ranks=(2, 3, 4)):
    """Shape pairs for the uneven batch.

    The flattened non-contracted extents M and N are each drawn uniform in
    ``mn_range`` and split into rank-1 axes by a random ordered factorisation;
    the contracted extent K is uniform in ``k_range``; the ranks of A and B are
    uniform over ``ranks``.
    """
    rng = _as_rng(rng)
    shapes = []
    for _ in range(count):
        ra = int(rng.choice(ranks))
        rb = int(rng.choice(ranks))
        m = int(rng.integers(mn_range[0], mn_range[1] + 1))
        n = int(rng.integers(mn_range[0], mn_range[1] + 1))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        sa = tuple(random_factorisation(rng, m, ra - 1)) + (k,)
        sb = (k,) + tuple(random_factorisation(rng, n, rb - 1))
        shapes.append((sa, sb))
    return shapes


def batch_problems(rng, count, **kw) -> list[Problem]:
    rng = _as_rng(rng)
    shapes = batch_shapes(rng, count, **kw)
    probs = []
    for sa, sb in shapes:
        a = uniform_f32(rng, sa)
        b = uniform_f32(rng, sb)
        probs.append(Problem(sa, sb, a, b))
    return probs


# ---------------------------------------------------------------------------
# Full-size workloads (the shapes named for each workload).

def workload_small_mixed(rng=None):
    rng = rng or rng_for(SMALL_MIXED)
    a = uniform_f64(rng, (512, 512))
    b = uniform_f64(rng, (512, 512))
    oa = uniform_f64(rng, (32, 32))
    ob = uniform_f64(rng, (16, 16))
    return a, b, oa, ob


def workload_rank_general_f64(rng=None, scale=1):
    rng = rng or rng_for(RANK_GENERAL)
    sa = (64 // scale, 64 // scale, 32, 256)
    sb = (256, 128 // scale, 64)
    return uniform_f64(rng, sa), uniform_f64(rng, sb)


def workload_tropical(rng=None, n=2048):
    rng = rng or rng_for(RANK_GENERAL, salt=1)
    return uniform_i32(rng, (n, n)), uniform_i32(rng, (n, n))


def workload_outer_f32(rng=None, sa=(512, 512), sb=(64, 64)):
    rng = rng or rng_for(RANK_GENERAL, salt=2)
    return uniform_f32(rng, sa), uniform_f32(rng, sb)


def workload_split(rng=None, m=8192, k=8192, n=8192):
    rng = rng or rng_for(SPLIT_PRECISION)
    return scaled_f64(rng, (m, k)), scaled_f64(rng, (k, n))


def workload_skinny(rng=None, m=4, k=128, n=1 << 22):
    """Section II.B's matrix product: A is m x 128 (m = 1..4), B is 128 x n."""
    rng = rng or rng_for(RANK_GENERAL, salt=5)
    return uniform_f64(rng, (m, k)), uniform_f64(rng, (k, n))


def workload_axes(rng=None, sa=(16, 2048, 512), sb=(16, 2048, 512)):
    """Contraction over a middle axis of both operands (axes (1, 1)):
    8192 x 2048 . 2048 x 8192 read through strided views, U[-1, 1]."""
    rng = rng or rng_for(RANK_GENERAL, salt=6)
    return uniform_f64(rng, sa), uniform_f64(rng, sb)


def workload_fewcols(rng=None, m=65536, k=4096, n=8):
    """int32 (max,+) with few result columns: A m x k, B k x n, entries U{-1000..1000}."""
    rng = rng or rng_for(RANK_GENERAL, salt=7)
    return uniform_i32(rng, (m, k)), uniform_i32(rng, (k, n))


def workload_grad(rng=None, sa=(32, 128, 512), sb=(512, 64, 64)):
    rng = rng or rng_for(DIFFERENTIATION)
    a = uniform_f32(rng, sa)
    b = uniform_f32(rng, sb)
    g = uniform_f32(rng, tuple(sa[:-1]) + tuple(sb[1:]))
    return a, b, g
