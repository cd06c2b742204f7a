"""Pins for the CPU oracle: a hand-worked example, brute force on tiny inputs,
library routines (numpy) for special cases, and invariants of a PK-FK join."""
import json
import os

import numpy as np
import pytest

import datagen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
INT32_MIN, INT32_MAX = -(2 ** 31), 2 ** 31 - 1


def _tiny():
    return json.load(open(os.path.join(GOLD, "tiny_query.json")))


@pytest.mark.parametrize("group_by", ["fk", "prio_flag", "dim_grp"])
@pytest.mark.parametrize("brute", [False, True])
def test_hand_worked_example(group_by, brute):
    d = _tiny()
    f, dm = d["fact"], d["dim"]
    groups, stats = oracle.filter_join_agg(f["fk"], f["price"], f["qty"], f["day"], f["flag"], dm["pk"], dm["prio"],
                                           dm["grp"], d["day_lt"], group_by, brute=brute)
    exp = d["expected"][group_by]
    for k in ("key", "sum_price", "sum_qty", "count"):
        assert groups[k].tolist() == exp[k], k
    assert stats["rows_passed"] == d["stats"]["rows_passed"]
    assert stats["join_matches"] == d["stats"]["join_matches"]


def _random_tiny(rng, n, m, key_lo, key_hi, group_by):
    pk = rng.choice(np.arange(key_lo, key_hi + 1, dtype=np.int64), size=m, replace=False).astype(np.int32) if m else np.zeros(0, np.int32)
    fk = rng.integers(key_lo, key_hi + 1, size=n, dtype=np.int64).astype(np.int32)
    price = rng.integers(-(2 ** 62), 2 ** 62, size=n, dtype=np.int64)
    qty = rng.integers(INT32_MIN, INT32_MAX, size=n, dtype=np.int64, endpoint=True).astype(np.int32)
    day = rng.integers(-5, 20, size=n).astype(np.int32)
    flag = rng.integers(-128, 128, size=n).astype(np.int8)
    prio = rng.integers(-128, 128, size=m).astype(np.int8)
    grp = rng.integers(INT32_MIN, INT32_MAX, size=m, endpoint=True).astype(np.int32) if rng.random() < 0.5 else \
        rng.integers(0, 4, size=m).astype(np.int32)
    return fk, price, qty, day, flag, pk, prio, grp


def test_oracle_matches_brute_force_on_random_tiny_instances():
    rng = np.random.default_rng(12345)
    for it in range(1200):
        n = int(rng.integers(0, 120))
        m = int(rng.integers(0, 40))
        group_by = ["fk", "prio_flag", "dim_grp"][it % 3]
        # alternate between keys near zero and keys at the int32 extremes
        if it % 4 == 3:
            lo, hi = INT32_MAX - 60, INT32_MAX
        elif it % 4 == 2:
            lo, hi = INT32_MIN, INT32_MIN + 60
        else:
            lo, hi = -30, 50
        fk, price, qty, day, flag, pk, prio, grp = _random_tiny(rng, n, m, lo, hi, group_by)
        T = int(rng.integers(-6, 21))
        a, sa = oracle.filter_join_agg(fk, price, qty, day, flag, pk, prio, grp, T, group_by)
        b, sb = oracle.filter_join_agg(fk, price, qty, day, flag, pk, prio, grp, T, group_by, brute=True)
        for k in a:
            assert np.array_equal(a[k], b[k]), (it, k)
        assert sa == sb, it


def test_duplicate_pk_is_an_error_in_both():
    pk = [1, 2, 3, 2]
    args = ([1], [5], [1], [0], [0], pk, [0, 0, 0, 0], [0, 0, 0, 0], 10, "fk")
    with pytest.raises(oracle.OracleError, match="duplicate"):
        oracle.filter_join_agg(*args)
    with pytest.raises(oracle.OracleError, match="duplicate"):
        oracle.filter_join_agg(*args, brute=True)


@pytest.mark.parametrize("case", ["empty_fact", "empty_dim", "all_filtered", "no_match", "one_group"])
def test_degenerate_cases(case):
    n, m = 50, 10
    fk = np.arange(n, dtype=np.int32) % m
    pk = np.arange(m, dtype=np.int32)
    price = np.full(n, 7, np.int64)
    qty = np.full(n, 3, np.int32)
    day = np.zeros(n, np.int32)
    flag = np.zeros(n, np.int8)
    prio = np.zeros(m, np.int8)
    grp = np.zeros(m, np.int32)
    T = 1
    if case == "empty_fact":
        fk, price, qty, day, flag = fk[:0], price[:0], qty[:0], day[:0], flag[:0]
    elif case == "empty_dim":
        pk, prio, grp = pk[:0], prio[:0], grp[:0]
    elif case == "all_filtered":
        T = 0
    elif case == "no_match":
        fk = fk + 1000
    g, s = oracle.filter_join_agg(fk, price, qty, day, flag, pk, prio, grp, T, "dim_grp")
    if case == "one_group":
        assert g["key"].tolist() == [0] and g["count"].tolist() == [n]
        assert g["sum_price"].tolist() == [7 * n] and g["sum_qty"].tolist() == [3 * n]
    else:
        assert g["key"].shape[0] == 0 and s["groups"] == 0
    assert s["join_matches"] <= len(fk)


def test_wraparound_is_mod_2_64():
    # Two rows of price 2^62 + 2^62 + ... wrap exactly like uint64 addition.
    n = 5
    price = np.full(n, 2 ** 62, np.int64)
    g, _ = oracle.filter_join_agg(np.zeros(n, np.int32), price, np.ones(n, np.int32), np.zeros(n, np.int32),
                                  np.zeros(n, np.int8), [0], [0], [0], 1, "fk")
    expect = np.array([(5 * 2 ** 62) % 2 ** 64], dtype=np.uint64).view(np.int64)[0]
    assert g["sum_price"][0] == expect


def test_small_workload_invariants():
    T = datagen.small()
    g, s = oracle.run_tables(T)
    mask = T.day < T.day_lt
    # textbook counts (numpy): every fk is in [0, M) and pk is a permutation, so every passing row matches
    assert s["rows_passed"] == int(mask.sum())
    assert s["join_matches"] == s["rows_passed"]
    assert s["join_matches"] <= T.n
    assert int(g["count"].sum()) == s["join_matches"]
    # ungrouped totals through numpy
    assert int(g["sum_price"].sum()) == int(T.price_cents[mask].astype(np.int64).sum())
    assert int(g["sum_qty"].sum()) == int(T.qty[mask].astype(np.int64).sum())
    # 5 prio values x 3 flags
    assert s["groups"] == 15
    assert np.all(np.diff(g["key"]) > 0)
    # selectivity within 5 sigma of 1800/2557
    p = T.day_lt / datagen.DAY_DOMAIN
    assert abs(s["rows_passed"] / T.n - p) < 5 * np.sqrt(p * (1 - p) / T.n)


def test_group_by_fk_equals_numpy_unique():
    T = datagen.make_tables(50_000, 12_000, 77, day_lt=1200, group_by="fk", fk_zipf=0.8)
    g, s = oracle.run_tables(T)
    mask = T.day < T.day_lt
    keys, inv = np.unique(T.fk[mask], return_inverse=True)
    assert g["key"].tolist() == keys.tolist()
    cnt = np.bincount(inv)
    assert g["count"].tolist() == cnt.tolist()
    sp = np.zeros(keys.shape[0], np.uint64)
    np.add.at(sp, inv, T.price_cents[mask].astype(np.uint64))
    assert np.array_equal(g["sum_price"].view(np.uint64), sp)


def test_filter_compact_matches_flatnonzero():
    rng = np.random.default_rng(3)
    col = rng.integers(-50, 50, size=5000).astype(np.int32)
    for op, f in [("lt", np.less), ("le", np.less_equal), ("gt", np.greater), ("ge", np.greater_equal),
                  ("eq", np.equal), ("ne", np.not_equal)]:
        assert np.array_equal(oracle.filter_compact(col, op, 7), np.flatnonzero(f(col, 7)).astype(np.int32))
    assert oracle.filter_compact(col[:0], "lt", 0).shape[0] == 0


def test_join_probe_pairs():
    rng = np.random.default_rng(9)
    pk = rng.permutation(3000).astype(np.int32) - 1000
    fk = rng.integers(-2000, 3000, size=20000).astype(np.int32)
    sel = np.flatnonzero(rng.random(20000) < 0.4).astype(np.int32)
    fi, pl = oracle.join_probe(fk, sel, pk)
    # every pair is a real match, fact ids come out ascending, and the count is the textbook isin count
    assert np.all(fk[fi] == pk[pl])
    assert np.all(np.diff(fi) > 0)
    assert fi.shape[0] == int(np.isin(fk[sel], pk).sum())
    assert set(fi.tolist()) <= set(sel.tolist())
    payload = (np.arange(3000) * 7).astype(np.int32)
    fi2, pl2 = oracle.join_probe(fk, None, pk, payload)
    order = np.argsort(pk)
    j = order[np.searchsorted(pk[order], fk[fi2])]  # dim row of each matched fk, via sorting
    assert np.array_equal(pl2, payload[j])
    assert fi2.shape[0] == int(np.isin(fk, pk).sum())


def test_groupby_agg_matches_numpy():
    rng = np.random.default_rng(5)
    n = 30000
    key = rng.integers(-(2 ** 63), 2 ** 63 - 1, size=64, dtype=np.int64)[rng.integers(0, 64, size=n)]
    key[::1000] = np.iinfo(np.int64).min  # the minimum int64 is a valid key too
    price = rng.integers(-(2 ** 40), 2 ** 40, size=n, dtype=np.int64)
    qty = rng.integers(-1000, 1000, size=n).astype(np.int32)
    sel = np.flatnonzero(rng.random(n) < 0.6).astype(np.int32)
    g = oracle.groupby_agg(key, price, qty, sel)
    keys, inv = np.unique(key[sel], return_inverse=True)
    assert g["key"].tolist() == keys.tolist()
    sq = np.zeros(keys.shape[0], np.int64)
    np.add.at(sq, inv, qty[sel].astype(np.int64))
    assert g["sum_qty"].tolist() == sq.tolist()
    assert g["count"].tolist() == np.bincount(inv).tolist()
    # SUM(price) of the selected rows, summed modulo 2^64 as unsigned
    sp = np.zeros(keys.shape[0], np.uint64)
    np.add.at(sp, inv, price[sel].view(np.uint64))
    assert g["sum_price"].view(np.uint64).tolist() == sp.tolist()


def test_groupby_agg_sum_price_wraps_and_uses_selected_rows():
    # prices near 2^62 so that group sums wrap modulo 2^64, and a selection
    # vector that is not the identity: a key's sum must add the price of each
    # selected row (not of position k in the selection)
    rng = np.random.default_rng(6)
    n = 5000
    key = rng.integers(0, 7, size=n).astype(np.int64)
    price = rng.integers(2 ** 61, 2 ** 62, size=n, dtype=np.int64)
    price[rng.random(n) < 0.5] *= -1
    qty = rng.integers(1, 50, size=n).astype(np.int32)
    sel = np.sort(rng.choice(n, size=1800, replace=False)).astype(np.int32)
    g = oracle.groupby_agg(key, price, qty, sel)
    want = {}
    for r in sel.tolist():
        want[int(key[r])] = (want.get(int(key[r]), 0) + int(price[r])) % (1 << 64)
    assert g["key"].tolist() == sorted(want)
    assert g["sum_price"].view(np.uint64).tolist() == [want[k] for k in sorted(want)]
    assert any(v >= (1 << 63) for v in want.values())  # at least one sum wrapped past 2^63


# -- join-output materialisation (gather) ---------------------------------------------------------------------------------

def test_join_gather_hand_example():
    # worked by hand: rows 3, 0, 0, 2 of [10, 20, 30, 40]
    src = np.array([10, 20, 30, 40], np.int64)
    assert oracle.join_gather(np.array([3, 0, 0, 2], np.int32), src).tolist() == [40, 10, 10, 30]
    assert oracle.join_gather(np.array([1, 1, 0], np.int32), np.array([7, -3], np.int8)).tolist() == [-3, -3, 7]
    assert oracle.join_gather(np.zeros(0, np.int32), src).shape == (0,)


@pytest.mark.parametrize("dtype", [np.int8, np.int16, np.int32, np.int64, np.float64])
def test_join_gather_equals_numpy_take(dtype):
    rng = np.random.default_rng(5)
    src = rng.integers(-100, 100, size=1001).astype(dtype)
    idx = rng.integers(0, 1001, size=5000).astype(np.int32)
    assert np.array_equal(oracle.join_gather(idx, src), np.take(src, idx))


def test_join_gather_identity_and_join_keys():
    rng = np.random.default_rng(6)
    src = rng.integers(-(2 ** 31), 2 ** 31 - 1, size=777).astype(np.int32)
    assert np.array_equal(oracle.join_gather(np.arange(777, dtype=np.int32), src), src)
    # through a probe: the fact side's fk and the dim side's pk agree pair by pair
    pk = datagen.permutation(2000, 0, 7, 1)
    fk = rng.integers(-500, 2500, size=9000).astype(np.int32)
    fi, di = oracle.join_probe(fk, None, pk)
    assert np.array_equal(oracle.join_gather(fi, fk), oracle.join_gather(di, pk))


def test_join_gather_rejects_out_of_range_rows():
    src = np.arange(10, dtype=np.int32)
    for bad in (10, -1):
        with pytest.raises(oracle.OracleError):
            oracle.join_gather(np.array([0, bad], np.int32), src)


# -- general predicates ---------------------------------------------------------------------------------------------------

def _np_term(col, op, values):
    x = col.astype(np.float64) if col.dtype.kind == "f" else col.astype(np.int64)
    if op == "between":
        return (x >= values[0]) & (x <= values[1])
    if op == "in":
        m = np.zeros(x.shape[0], bool)
        for v in values:
            m |= x == v
        return m
    return {"lt": x < values[0], "le": x <= values[0], "gt": x > values[0], "ge": x >= values[0],
            "eq": x == values[0], "ne": x != values[0]}[op]


def test_pred_filter_hand_example():
    a = np.array([5, 1, 7, 3, 9], np.int32)
    b = np.array([1.0, np.nan, 2.5, -1.0, 0.0])
    assert oracle.pred_filter([a, b], [dict(column=0, op="between", values=[2, 8])]).tolist() == [0, 2, 3]
    assert oracle.pred_filter([a, b], [dict(column=0, op="in", values=[1, 9, 4]),
                                       dict(column=1, op="ne", values=[5.0])]).tolist() == [1, 4]
    assert oracle.pred_filter([a, b], [dict(column=1, op="lt", values=[1.0])]).tolist() == [3, 4]


@pytest.mark.parametrize("dtype", [np.int8, np.int16, np.int32, np.int64, np.float32, np.float64])
@pytest.mark.parametrize("op", ["lt", "le", "gt", "ge", "eq", "ne", "between", "in"])
def test_pred_filter_single_terms_equal_numpy(dtype, op):
    rng = np.random.default_rng(hash((str(dtype), op)) % 2 ** 32)
    col = rng.integers(-60, 60, size=3001).astype(dtype)
    if col.dtype.kind == "f":
        col[::97] = np.nan
    values = {"between": [-20, 35], "in": [-7, 0, 3, 59, 100]}.get(op, [5])
    got = oracle.pred_filter([col], [dict(column=0, op=op, values=values)])
    assert np.array_equal(got, np.flatnonzero(_np_term(col, op, values)))


def test_pred_filter_conjunction_is_intersection():
    rng = np.random.default_rng(12)
    cols = [rng.integers(0, 100, size=5000).astype(np.int32), rng.normal(size=5000), rng.integers(-5, 5, size=5000).astype(np.int8)]
    terms = [dict(column=0, op="ge", values=[30]), dict(column=1, op="between", values=[-0.5, 1.0]),
             dict(column=2, op="in", values=[-5, 0, 4]), dict(column=0, op="ne", values=[50])]
    expect = np.arange(5000)
    for t in terms:
        expect = np.intersect1d(expect, oracle.pred_filter(cols, [t]))
    assert np.array_equal(oracle.pred_filter(cols, terms), expect)
    # one lt term over int32 is the plain compaction
    assert np.array_equal(oracle.pred_filter(cols, [dict(column=0, op="lt", values=[42])]),
                          oracle.filter_compact(cols[0], "lt", 42))
