"""Pins for the CPU oracle: it is checked against things other than itself --
arbitrary-precision brute force on tiny inputs, exact-rational fma rounding, closed
forms, invariants and IEEE special cases -- so that a dropped term, a wrong sign, a
transposed operand or a lost rounding step in it fails here."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import brute

I32_EDGES = [-2 ** 31, -2 ** 31 + 1, -2, -1, 0, 1, 2, 2 ** 31 - 2, 2 ** 31 - 1, 12345, -99999]


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ---------------------------------------------------------------- int32 affine + int64 sum
@pytest.mark.parametrize("n", list(range(0, 18)))
def test_affine_sum_matches_bigint_brute_force(n):
    rng = np.random.default_rng(100 + n)
    pool = np.array(I32_EDGES, dtype=np.int64)
    for trial in range(12):
        if trial % 2:
            x = rng.choice(pool, n).astype(np.int32)
        else:
            x = rng.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
        a, b = (int(v) for v in rng.choice(pool, 2)) if trial < 6 else \
            (int(v) for v in rng.integers(-2 ** 31, 2 ** 31, 2))
        y, s = oracle.affine_sum_i32(x, a, b)
        yb, sb = brute.affine_sum([int(v) for v in x], a, b)
        assert y.tolist() == yb
        assert s == sb


def test_affine_exhaustive_edge_grid():
    x = np.array(I32_EDGES, dtype=np.int32)
    for a, b in itertools.product(I32_EDGES, repeat=2):
        y, s = oracle.affine_sum_i32(x, a, b)
        yb, sb = brute.affine_sum([int(v) for v in x], a, b)
        assert y.tolist() == yb and s == sb, (a, b)


def test_affine_special_cases_closed_forms():
    rng = np.random.default_rng(7)
    x = rng.integers(-2 ** 31, 2 ** 31, 5000, dtype=np.int64).astype(np.int32)
    # a = 1, b = 0: identity
    y, s = oracle.affine_sum_i32(x, 1, 0)
    assert np.array_equal(y, x) and s == int(x.astype(np.int64).sum())
    # a = 0: y == b everywhere, s = n*b
    for b in (-2 ** 31, -7, 0, 2 ** 31 - 1):
        y, s = oracle.affine_sum_i32(x, 0, b)
        assert np.all(y == b) and s == x.size * b
    # x = 0: y == b
    y, s = oracle.affine_sum_i32(np.zeros(33, np.int32), 123456789, -5)
    assert np.all(y == -5) and s == -5 * 33
    # a = -1, b = 0: negation mod 2^32; INT32_MIN maps to itself
    y, _ = oracle.affine_sum_i32(np.array([-2 ** 31, -1, 0, 1, 2 ** 31 - 1], np.int32), -1, 0)
    assert y.tolist() == [-2 ** 31, 1, 0, -1, -2 ** 31 + 1]
    # a = 2, b = 0 on 2^30 wraps to INT32_MIN
    y, _ = oracle.affine_sum_i32(np.array([2 ** 30], np.int32), 2, 0)
    assert y.tolist() == [-2 ** 31]


def test_int64_sum_is_order_independent_and_never_wraps():
    rng = np.random.default_rng(11)
    x = rng.integers(-2 ** 31, 2 ** 31, 1 << 16, dtype=np.int64).astype(np.int32)
    s = oracle.sum_i32_i64(x)
    assert s == sum(int(v) for v in x)
    assert s == oracle.sum_i32_i64(np.ascontiguousarray(x[::-1]))
    # pairwise tree order
    v = [int(t) for t in x]
    while len(v) > 1:
        v = [v[i] + (v[i + 1] if i + 1 < len(v) else 0) for i in range(0, len(v), 2)]
    assert s == v[0]
    # all INT32_MIN: the sum exceeds int32 range, no wrap in int64
    big = np.full(1 << 12, -2 ** 31, np.int32)
    assert oracle.sum_i32_i64(big) == -(2 ** 31) * (1 << 12)
    assert oracle.sum_i32_i64(np.zeros(0, np.int32)) == 0


# ---------------------------------------------------------------- fp32 SAXPY (single fma)
def _bits(a):
    return np.asarray(a, dtype=np.float32).view(np.uint32)


def _f32_pool(rng, n):
    kinds = rng.integers(0, 6, n)
    v = rng.standard_normal(n).astype(np.float32)
    v[kinds == 1] = (rng.standard_normal((kinds == 1).sum()) * 1e-40).astype(np.float32)  # subnormal
    v[kinds == 2] = (rng.standard_normal((kinds == 2).sum()) * 1e37).astype(np.float32)   # near overflow
    v[kinds == 3] = np.float32(0.0) * np.sign(rng.standard_normal((kinds == 3).sum())).astype(np.float32)
    v[kinds == 4] = rng.integers(-64, 64, (kinds == 4).sum()).astype(np.float32) / np.float32(8)
    return v


@pytest.mark.parametrize("seed", range(6))
def test_saxpy_matches_exact_rational_rounding(seed):
    rng = np.random.default_rng(seed)
    n = 400
    x = _f32_pool(rng, n)
    y = _f32_pool(rng, n)
    for alpha in [np.float32(rng.uniform(-2, 2)), np.float32(1e-38), np.float32(-3e30), np.float32(0.5)]:
        yo = oracle.saxpy_f32(alpha, x, y.copy())
        yb = np.array(brute.saxpy(alpha, x, y), dtype=np.float32)
        assert np.array_equal(_bits(yo), _bits(yb)), alpha


def test_saxpy_is_a_fused_multiply_add_not_mul_then_add():
    # a*x = 1 + 2^-11 + 2^-24 exactly; with y = -1 the single-rounding result keeps the
    # 2^-24 term, while rounding the product first loses it.
    a = np.float32(1 + 2 ** -12)
    x = np.array([1 + 2 ** -12], np.float32)
    y = np.array([-1.0], np.float32)
    out = oracle.saxpy_f32(a, x, y.copy())
    assert out[0] == np.float32(2 ** -11 + 2 ** -24)
    two_step = np.float32(np.float32(a * x[0]) + y[0])
    assert out[0] != two_step


def test_saxpy_special_values():
    def f(a, x, y):
        return oracle.saxpy_f32(np.float32(a), np.array([x], np.float32), np.array([y], np.float32))[0]
    inf, nan = np.float32(np.inf), np.float32(np.nan)
    assert f(2, inf, 1) == inf
    assert math.isnan(f(0, inf, 1))          # 0 * inf is invalid
    assert math.isnan(f(1, inf, -inf))       # inf - inf is invalid
    assert math.isnan(f(1, 1, nan))
    assert f(-1, 3e38, -3e38) == -inf        # overflow of the exact sum
    # exact zero results: +0 unless both product and addend are -0
    assert _bits(f(1, 2.0, -2.0)) == _bits(np.float32(0.0))
    assert _bits(f(0, -1.0, -0.0)) == _bits(np.float32(-0.0))
    assert _bits(f(0, 1.0, -0.0)) == _bits(np.float32(0.0))
    # alpha = 2^k: exact product, so the result is the single rounding of the sum
    rng = np.random.default_rng(3)
    x = rng.standard_normal(1000).astype(np.float32)
    y = rng.standard_normal(1000).astype(np.float32)
    out = oracle.saxpy_f32(np.float32(0.25), x, y.copy())
    ref = (x.astype(np.float64) * 0.25 + y.astype(np.float64))  # one f64 rounding of an
    # exact product + f32 addend whose exponent gap is small, then the f32 rounding;
    # the f64 step is exact here because |x/4| and |y| are within 2^29 of each other.
    ok = np.abs(np.log2(np.abs(x) / 4 + 1e-30) - np.log2(np.abs(y) + 1e-30)) < 28
    assert np.array_equal(_bits(out[ok]), _bits(ref[ok].astype(np.float32)))


def test_saxpy_preserves_subnormals():
    x = np.array([1e-45, -1e-45, 1e-39], np.float32)
    y = np.zeros(3, np.float32)
    out = oracle.saxpy_f32(np.float32(1.0), x, y)
    assert np.array_equal(_bits(out), _bits(x))


def test_saxpy_chain_matches_brute_and_is_order_sensitive():
    rng = np.random.default_rng(21)
    alphas = rng.uniform(-2, 2, 200).astype(np.float32)
    x, y = np.float32(rng.standard_normal()), np.float32(rng.standard_normal())
    got = oracle.saxpy_chain_elem(x, y, alphas)
    ref = y
    for a in alphas:
        ref = brute.fma_f32(a, x, ref)
    assert _bits(got) == _bits(ref)
    assert _bits(oracle.saxpy_chain_elem(x, y, alphas[::-1].copy())) != _bits(got)


def test_copy_is_bitwise():
    rng = np.random.default_rng(5)
    src = rng.integers(0, 2 ** 32, 777, dtype=np.uint64).astype(np.uint32).view(np.float32)
    dst = oracle.copy_f32(src)
    assert np.array_equal(src.view(np.uint32), dst.view(np.uint32))


# ---------------------------------------------------------------- cluster slicing
def test_slices_partition_the_range():
    for n in list(range(0, 600, 37)) + [4096, 8191, 262144, 262145, 16384, 10 ** 6]:
        for k in (1, 2, 3, 7, 32, 256):
            covered = 0
            prev_hi = 0
            for j in range(k):
                lo, hi = oracle.slice_bounds(n, k, j)
                assert (lo, hi) == brute.slice_bounds(n, k, j)
                assert lo == prev_hi and lo <= hi <= n
                assert lo % 256 == 0 or lo == n
                covered += hi - lo
                prev_hi = hi
            assert covered == n and prev_hi == n
    assert oracle.slice_bounds(262144, 32, 5) == (5 * 8192, 6 * 8192)
    assert oracle.slice_bounds(100, 4, 0) == (0, 100)   # one 256-group holds everything
    assert oracle.slice_bounds(100, 4, 3) == (100, 100)


def test_cluster_item_equals_whole_item():
    rng = np.random.default_rng(9)
    n = 262144 + 77
    x = rng.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
    y1, y2 = np.empty_like(x), np.empty_like(x)
    s1 = oracle.exec_item(oracle.AFFINE_SUM_I32, x, y1, a=-3, b=99)
    s2 = oracle.exec_cluster(oracle.AFFINE_SUM_I32, 32, x, y2, a=-3, b=99)
    assert s1 == s2 and np.array_equal(y1, y2)
    assert s1 == brute.affine_sum([int(v) for v in x[:2000]], -3, 99)[1] + \
        oracle.affine_sum_i32(x[2000:].copy(), -3, 99)[1]


# ---------------------------------------------------------------- mailbox FIFO specification
def test_fifo_runs_in_submission_order():
    rng = np.random.default_rng(13)
    x = rng.standard_normal(64).astype(np.float32)
    y0 = rng.standard_normal(64).astype(np.float32)
    alphas = rng.uniform(-2, 2, 50).astype(np.float32)
    y = y0.copy()
    oracle.run_fifo([dict(op=oracle.SAXPY_F32, inp=x, out=y, alpha=a) for a in alphas])
    ref = np.array([oracle.saxpy_chain_elem(x[i], y0[i], alphas) for i in range(64)], np.float32)
    assert np.array_equal(_bits(y), _bits(ref))
    yr = y0.copy()
    oracle.run_fifo([dict(op=oracle.SAXPY_F32, inp=x, out=yr, alpha=a) for a in alphas[::-1]])
    assert not np.array_equal(_bits(yr), _bits(y))


def test_packed_chain_runs_the_same_fifo():
    rng = np.random.default_rng(14)
    x = rng.standard_normal(300).astype(np.float32)
    y0 = rng.standard_normal(300).astype(np.float32)
    alphas = rng.uniform(-2, 2, 40).astype(np.float32)
    y1, y2 = y0.copy(), y0.copy()
    oracle.run_fifo([dict(op=oracle.SAXPY_F32, inp=x, out=y1, alpha=a) for a in alphas])
    res = oracle.run_packed(oracle.pack_chain(oracle.SAXPY_F32, x, y2, alphas))
    assert np.array_equal(_bits(y1), _bits(y2)) and not res.any()
    xi = np.arange(-7, 9, dtype=np.int32)
    yi = np.empty_like(xi)
    res = oracle.run_packed(oracle.pack_chain(oracle.AFFINE_SUM_I32, xi, yi, np.zeros(3), a=3, b=-2))
    assert res.tolist() == [sum(3 * v - 2 for v in range(-7, 9))] * 3
    with pytest.raises(ValueError):
        oracle.run_packed(oracle.pack_chain(99, None, None, np.zeros(1), n=0))


def test_fifo_results_and_unknown_op():
    x = np.arange(-5, 5, dtype=np.int32)
    y = np.empty_like(x)
    res = oracle.run_fifo([dict(op=oracle.SUM_I32_I64, inp=x),
                           dict(op=oracle.AFFINE_SUM_I32, inp=x, out=y, a=2, b=1),
                           dict(op=oracle.NOP, n=0)])
    assert res.tolist() == [-5, sum(2 * v + 1 for v in range(-5, 5)), 0]
    with pytest.raises(ValueError):
        oracle.run_fifo([dict(op=99, n=0)])


def test_out_of_place_axpy_matches_brute_force_and_leaves_y():
    rng = np.random.default_rng(31)
    x = _f32_pool(rng, 300)
    y = _f32_pool(rng, 300)
    y_before = y.copy()
    for alpha in (np.float32(-1.25), np.float32(3e-39), np.float32(7.0)):
        out = oracle.axpy_f32(alpha, x, y)
        want = np.array(brute.saxpy(alpha, x, y), dtype=np.float32)
        assert np.array_equal(_bits(out), _bits(want))
        assert np.array_equal(_bits(y), _bits(y_before))
    got = np.empty_like(y)
    oracle.exec_item(oracle.AXPY_F32, inp=x, out=got, in2=y, alpha=np.float32(0.5))
    assert np.array_equal(_bits(got), _bits(np.array(brute.saxpy(np.float32(0.5), x, y), np.float32)))


# ---------------------------------------------------------------- the paper's compute-only item
SENT_WORD = 0x7FBADBAD


@pytest.mark.parametrize("iters", [0, 1, 20000, 2 ** 31 - 1])
def test_spin_item_leaves_memory_untouched_and_returns_zero(iters):
    """Sec. 3: the benchmark item loops without memory traffic.  Given in/out references
    and a length anyway, it must leave both buffers bit for bit as they were, whole or
    sliced over a cluster, and its result is 0."""
    inp = np.full(1000, SENT_WORD, np.uint32).view(np.float32)
    out = np.full(1000, SENT_WORD ^ 0xFFFF, np.uint32).view(np.float32)
    assert oracle.spin(iters) == 0
    assert oracle.exec_item(oracle.SPIN, inp=inp, out=out, a=iters) == 0
    assert oracle.exec_cluster(oracle.SPIN, 7, inp=inp, out=out, a=iters) == 0
    assert np.all(inp.view(np.uint32) == SENT_WORD)
    assert np.all(out.view(np.uint32) == (SENT_WORD ^ 0xFFFF))


def test_spin_and_nop_inside_a_saxpy_fifo_change_nothing():
    """A mailbox FIFO of SAXPY items with SPIN and NOP items between them (pointing at the
    same x and y) leaves y equal to the brute-force chain of the SAXPY items alone; the
    SPIN and NOP results are 0, and the chain stays order-sensitive."""
    rng = np.random.default_rng(41)
    x = rng.standard_normal(16).astype(np.float32)
    y0 = rng.standard_normal(16).astype(np.float32)
    alphas = rng.uniform(-2, 2, 12).astype(np.float32)
    items, kinds = [], []
    y = y0.copy()
    for k, a in enumerate(alphas):
        items.append(dict(op=oracle.SAXPY_F32, inp=x, out=y, alpha=a))
        kinds.append("saxpy")
        extra = oracle.SPIN if k % 2 == 0 else oracle.NOP
        items.append(dict(op=extra, inp=x, out=y, n=x.size, a=20000, alpha=np.float32(3.0)))
        kinds.append("other")
    res = oracle.run_fifo(items)
    want = []
    for i in range(x.size):
        v = y0[i]
        for a in alphas:
            v = brute.fma_f32(a, x[i], v)
        want.append(v)
    assert np.array_equal(_bits(y), _bits(np.array(want, np.float32)))
    assert all(r == 0 for r, kd in zip(res, kinds) if kd == "other")
    yr = y0.copy()
    oracle.run_fifo([dict(op=oracle.SAXPY_F32, inp=x, out=yr, alpha=a) for a in alphas[::-1]])
    assert not np.array_equal(_bits(yr), _bits(y))


def test_fifo_rejects_negative_spin_counts_and_non_items():
    assert oracle.spin(-1) == -1
    for bad in (dict(op=oracle.SPIN, n=0, a=-5), dict(op=6, n=0), dict(op=8, n=0)):
        with pytest.raises(ValueError):
            oracle.run_fifo([dict(op=oracle.NOP, n=0), bad])
    assert oracle.run_fifo([dict(op=oracle.SPIN, n=0, a=0)]).tolist() == [0]
