"""GPU parity of general predicates (rel_pred_*): compiled and interpreted
modes against the oracle's row-by-row evaluation, bit-exact selection
vectors, over every column type and operator, conjunctions of up to eight
terms, ragged sizes and the edge cases (empty input, all or nothing selected,
NaN, integer extremes, bad arguments)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2608_13696_amd import rel

pytestmark = pytest.mark.gpu

NP_DT = [np.int8, np.int16, np.int32, np.int64, np.float32, np.float64]
TORCH_DT = {np.dtype(np.int8): torch.int8, np.dtype(np.int16): torch.int16, np.dtype(np.int32): torch.int32,
            np.dtype(np.int64): torch.int64, np.dtype(np.float32): torch.float32, np.dtype(np.float64): torch.float64}
OPS = ["lt", "le", "gt", "ge", "eq", "ne", "between", "in"]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = rel.Context(0)
    yield c
    c.close()


def _run(ctx, cols, terms, mode):
    dts = [None if c is None else TORCH_DT[c.dtype] for c in cols]
    dev = [None if c is None else torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in cols]
    p = rel.Predicate(ctx, terms, dts, mode)
    idx, c = p.filter(dev)
    p.close()
    return idx.cpu().numpy(), c


def _random_case(seed, n):
    """1-6 columns of random types (some with small domains, floats with NaN)
    and 1-8 terms whose literals come from the data: comparisons at a quantile
    that keeps most rows, EQ/IN on values present in the column. Trailing
    terms are dropped while the oracle selects nothing (the cases test the
    masks, not empty outputs)."""
    rng = np.random.default_rng(seed)
    ncol = int(rng.integers(1, 7))
    cols = []
    for _ in range(ncol):
        dt = NP_DT[int(rng.integers(0, 6))]
        small = rng.random() < 0.5
        if np.dtype(dt).kind == "f":
            c = (rng.integers(-8, 9, size=n) if small else rng.normal(scale=50, size=n)).astype(dt)
            c[rng.random(n) < 0.02] = np.nan
        else:
            info = np.iinfo(dt)
            lo, hi = (-8, 9) if small else (max(info.min, -100_000), min(info.max, 100_000))
            c = rng.integers(lo, hi, size=n).astype(dt)
            c[rng.random(n) < 0.001] = info.min
            c[rng.random(n) < 0.001] = info.max
        cols.append(c)
    terms = []
    for _ in range(int(rng.integers(1, 9))):
        ci = int(rng.integers(0, ncol))
        col = cols[ci]
        fp = np.dtype(col.dtype).kind == "f"
        finite = col[~np.isnan(col)] if fp else col
        conv = float if fp else int
        q = lambda f: conv(np.quantile(finite, f, method="nearest")) if finite.size else conv(0)
        op = OPS[int(rng.integers(0, 8))]
        if op in ("lt", "le"):
            values = [q(rng.uniform(0.6, 0.99))]
        elif op in ("gt", "ge"):
            values = [q(rng.uniform(0.01, 0.4))]
        elif op == "between":
            values = [q(rng.uniform(0.0, 0.2)), q(rng.uniform(0.8, 1.0))]
        elif op == "ne":
            values = [conv(col[int(rng.integers(0, n))])]
        else:  # eq / in: values present in the column (NaN allowed: it never matches)
            k = 1 if op == "eq" else int(rng.integers(1, 17))
            values = [conv(col[int(rng.integers(0, n))]) for _ in range(k)]
        terms.append(dict(column=ci, op=op, values=values))
    while len(terms) > 1 and oracle.pred_filter(cols, terms).shape[0] == 0:
        terms.pop()
    return cols, terms


@pytest.mark.parametrize("mode", ["compiled", "interpreted"])
@pytest.mark.parametrize("seed,n", [(1, 1), (2, 15), (3, 16), (4, 17), (5, 4095), (6, 4096), (7, 4097), (8, 100_003),
                                    (9, 1_000_000), (10, 65_537), (11, 31), (12, 33), (13, 8191), (14, 8192),
                                    (15, 8193)])
def test_random_predicates_match_oracle(ctx, mode, seed, n):
    cols, terms = _random_case(seed, n)
    exp = oracle.pred_filter(cols, terms)
    got, c = _run(ctx, cols, terms, mode)
    assert c == exp.shape[0]
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("mode", ["compiled", "interpreted"])
def test_every_type_and_operator(ctx, mode):
    rng = np.random.default_rng(21)
    n = 20_011
    for dt in NP_DT:
        c = rng.integers(-50, 50, size=n).astype(dt)
        if np.dtype(dt).kind == "f":
            c[::13] = np.nan
            c[5] = -0.0
        terms = [dict(column=0, op=op, values={"between": [-10, 20], "in": [-3, 0, 7, 49, 51]}.get(op, [4]))
                 for op in OPS]
        for t in terms:  # one term at a time, then all at once
            got, _ = _run(ctx, [c], [t], mode)
            assert np.array_equal(got, oracle.pred_filter([c], [t])), (dt, t["op"])


@pytest.mark.parametrize("mode", ["compiled", "interpreted"])
def test_edge_cases(ctx, mode):
    big = np.array([np.iinfo(np.int64).min, -1, 0, 1, np.iinfo(np.int64).max] * 1000, np.int64)
    # all rows pass, no row passes, extremes as literals
    for terms, expect_all in (([dict(column=0, op="ge", values=[int(np.iinfo(np.int64).min)])], True),
                              ([dict(column=0, op="gt", values=[int(np.iinfo(np.int64).max)])], False),
                              ([dict(column=0, op="in", values=[int(np.iinfo(np.int64).min), int(np.iinfo(np.int64).max)])], None)):
        got, c = _run(ctx, [big], terms, mode)
        exp = oracle.pred_filter([big], terms)
        assert np.array_equal(got, exp)
        if expect_all is True:
            assert c == big.shape[0]
        if expect_all is False:
            assert c == 0
    # an unused column slot, a column used twice, NaN on both sides of IN
    f = np.array([np.nan, 1.5, -2.0, np.inf, -np.inf, 0.0] * 777, np.float64)
    i = np.arange(f.shape[0], dtype=np.int32)
    terms = [dict(column=2, op="in", values=[np.nan, 1.5, np.inf]), dict(column=0, op="ge", values=[10]),
             dict(column=0, op="lt", values=[4000])]
    got, _ = _run(ctx, [i, None, f], terms, mode)
    assert np.array_equal(got, oracle.pred_filter([i, None, f], terms))
    # empty input
    e = torch.zeros(0, dtype=torch.int32, device="cuda:0")
    p = rel.Predicate(ctx, [dict(column=0, op="lt", values=[3])], [torch.int32], mode)
    idx, c = p.filter([e])
    assert c == 0
    p.close()


def test_bad_arguments(ctx):
    with pytest.raises(rel.RelError) as e:
        rel.Predicate(ctx, [dict(column=0, op="between", values=[1])], [torch.int32])
    assert e.value.status == rel.INVALID_ARG
    with pytest.raises(rel.RelError) as e:
        rel.Predicate(ctx, [dict(column=0, op="lt", values=[1])] * 9, [torch.int32])
    assert e.value.status == rel.INVALID_ARG
    h = ctypes.c_void_p()  # one column declared with two types
    assert rel.lib().rel_pred_create(ctx.h, _two_types(), 2, 0, ctypes.byref(h)) == rel.INVALID_ARG
    p = rel.Predicate(ctx, [dict(column=0, op="lt", values=[1])], [torch.int32])
    x = torch.arange(64, dtype=torch.int32, device="cuda:0")
    with pytest.raises(rel.RelError) as e:
        p.filter([x[1:]])  # not 16-byte aligned
    assert e.value.status == rel.INVALID_ARG
    p.close()


def _two_types():
    arr = (rel.PredTerm * 2)()
    arr[0].column, arr[0].dtype, arr[0].op, arr[0].n_values = 0, 2, 0, 1
    arr[1].column, arr[1].dtype, arr[1].op, arr[1].n_values = 0, 5, 0, 1
    return arr
