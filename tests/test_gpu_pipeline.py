"""GPU parity: librel's fused pipeline and standalone operators against the CPU
oracle, element by element after canonical sorting (all results are integers,
so the bar is bit-exact)."""
import json
import os

import numpy as np
import pytest
import torch

import datagen
import oracle
from paper_2608_13696_amd import rel
from tests.gpu_util import assert_groups_equal, gpu_groups, to_dev

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = rel.Context(0)
    yield c
    c.close()


def run_both(ctx, T, plan=None, repeats=1):
    fact, dim = to_dev(T)
    ora, ostats = oracle.run_tables(T)
    for r in range(repeats):
        out, st = ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, plan=plan)
        g = gpu_groups(out)
        assert_groups_equal(g, ora, f"{T.meta} rep {r}")
        assert st["rows_passed"] == ostats["rows_passed"]
        assert st["join_matches"] == ostats["join_matches"]
        assert st["groups"] == ostats["groups"]
    return st


@pytest.mark.parametrize("group_by", ["fk", "prio_flag", "dim_grp"])
def test_hand_worked_example(ctx, group_by):
    d = json.load(open(os.path.join(GOLD, "tiny_query.json")))
    f, dm = d["fact"], d["dim"]
    dev = lambda a, dt: torch.tensor(a, dtype=dt, device="cuda:0")
    fact = {"fk": dev(f["fk"], torch.int32), "price_cents": dev(f["price"], torch.int64), "qty": dev(f["qty"], torch.int32),
            "day": dev(f["day"], torch.int32), "flag": dev(f["flag"], torch.int8)}
    dim = {"pk": dev(dm["pk"], torch.int32), "prio": dev(dm["prio"], torch.int8), "grp": dev(dm["grp"], torch.int32)}
    out, st = ctx.filter_join_agg(fact, dim, d["day_lt"], group_by)
    g = gpu_groups(out)
    exp = d["expected"][group_by]
    for k in ("key", "sum_price", "sum_qty", "count"):
        assert g[k].tolist() == exp[k], k
    assert st["rows_passed"] == d["stats"]["rows_passed"] and st["join_matches"] == d["stats"]["join_matches"]


def test_small_workload(ctx):
    st = run_both(ctx, datagen.small(), repeats=3)
    assert st["groups"] == 15 and st["group_placement"] == "lds"


def test_medium_workload(ctx):
    # by default the plain path (a dense join index over the 1.5M dim keys);
    # forced, the radix-partitioned path
    T = datagen.medium()
    st = run_both(ctx, T, repeats=3)
    assert st["groups"] == 15 and st["join_placement"] == "global"
    plan = rel.Plan(group_capacity=0, group_placement=0, join_placement=rel.PLACE["partitioned"], allow_fallback=0)
    st = run_both(ctx, T, plan=plan)
    assert st["groups"] == 15 and st["join_placement"] == "partitioned"


@pytest.mark.parametrize("group_by", ["fk", "dim_grp", "prio_flag"])
@pytest.mark.parametrize("n,m", [(1, 1), (3, 2), (1023, 300), (1025, 257), (60_001, 15_000), (250_007, 40_009)])
def test_ragged_sizes(ctx, group_by, n, m):
    T = datagen.make_tables(n, m, 1000 + n, day_lt=1500, group_by=group_by, fk_zipf=0.9 if group_by == "fk" else 0.0,
                            fk_domain=m + m // 3, grp_card=97 if group_by == "dim_grp" else None)
    run_both(ctx, T)


def test_large_shape_scaled_down(ctx):
    """The 60M-row workload's distributions (Zipf 0.8 fk, group by fk) at 6M x 1.5M, fully compared."""
    T = datagen.large(seed=33, n=6_000_000, m=1_500_000)
    run_both(ctx, T, repeats=2)


@pytest.mark.parametrize("case", ["empty_fact", "empty_dim", "all_filtered", "no_match", "extreme_keys"])
def test_degenerate(ctx, case):
    T = datagen.make_tables(5000, 1000, 77, day_lt=1800, group_by="dim_grp", grp_card=50)
    if case == "empty_fact":
        T = datagen.make_tables(0, 1000, 77, day_lt=1800, group_by="dim_grp", grp_card=50)
    elif case == "empty_dim":
        T = datagen.make_tables(5000, 0, 77, day_lt=1800, group_by="dim_grp", grp_card=50)
        T.grp = np.zeros(0, np.int32)
    elif case == "all_filtered":
        T.day_lt = 0
    elif case == "no_match":
        T.fk = T.fk + 5000
    elif case == "extreme_keys":
        # keys at both int32 ends and -1 (the key that needs the side slot), plus negative payloads
        ext = np.array([-(2 ** 31), 2 ** 31 - 1, -1, -2, -1_000_000], np.int32)
        T.pk[:5] = ext
        T.fk[:200] = np.resize(ext, 200)
        T.grp[:5] = np.array([-1, -(2 ** 31), 2 ** 31 - 1, 5, -7], np.int32)
    run_both(ctx, T)
    T.group_by = "fk"
    run_both(ctx, T)


@pytest.mark.parametrize("keys", ["dense_offset", "dense_negative", "dense_gaps", "just_too_wide", "sparse"])
@pytest.mark.parametrize("group_by", ["prio_flag", "dim_grp", "fk"])
def test_join_index_dense_or_hash(ctx, keys, group_by):
    # The plain path's join index is a dense array when the dim keys span at
    # most 2m values and a hash table otherwise; both must give the oracle's
    # groups, with fact keys inside, below and above the key range.
    m, n = 3000, 40_000
    T = datagen.make_tables(n, m, 91, day_lt=2000, group_by=group_by, grp_card=37 if group_by == "dim_grp" else None)
    rng = np.random.default_rng(91)
    if keys == "dense_offset":
        base = 1_000_000
    elif keys == "dense_negative":
        base = -(2 ** 31)  # the range starts at the smallest key
    else:
        base = -2000
    if keys in ("dense_gaps", "just_too_wide"):
        # 2m - 1 wide: still dense, half the entries empty; 2m + 1 wide: the
        # hash table. Both ends are keys, the rest distinct keys in between.
        width = 2 * m - 1 if keys == "dense_gaps" else 2 * m + 1
        inner = 1 + rng.choice(width - 2, size=m - 2, replace=False)
        T.pk = (base + np.concatenate([[0, width - 1], inner])).astype(np.int32)
        T.pk = T.pk[rng.permutation(m)]
    elif keys == "sparse":
        T.pk = rng.choice(np.arange(-(2 ** 31), 2 ** 31 - 1, 7919, dtype=np.int64), size=m, replace=False).astype(np.int32)
    else:
        T.pk = (base + rng.permutation(m)).astype(np.int32)
    lo, hi = int(T.pk.min()), int(T.pk.max())
    # fact keys: mostly dim keys, some just outside the range on both sides, some in gaps
    T.fk = T.pk[rng.integers(0, m, size=n)]
    T.fk[::7] = np.clip(rng.integers(lo - 5, hi + 6, size=T.fk[::7].shape[0]), -(2 ** 31), 2 ** 31 - 1).astype(np.int32)
    run_both(ctx, T)


@pytest.mark.parametrize("group_by", ["prio_flag", "dim_grp", "fk"])
def test_join_index_duplicate_key(ctx, group_by):
    # a repeated pk in a dense key range (same payload byte, so only the row
    # number tells the two entries apart) and in a hash-table one
    for base, spread in ((0, 1), (-100_000_000, 997)):
        T = datagen.make_tables(3000, 500, 92, group_by=group_by, grp_card=11 if group_by == "dim_grp" else None)
        T.pk = (base + spread * np.arange(500)).astype(np.int32)
        T.pk[300] = T.pk[17]
        T.prio[300] = T.prio[17]
        if T.grp is not None:
            T.grp[300] = T.grp[17]
        fact, dim = to_dev(T)
        with pytest.raises(rel.RelError) as e:
            ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by)
        assert e.value.status == rel.DUPLICATE_KEY, (base, spread)


def test_negative_prio_and_flag(ctx):
    T = datagen.make_tables(20_000, 3_000, 5, day_lt=2000, group_by="prio_flag")
    T.prio = datagen.uniform(T.m, -128, 127, np.int8, 5, 100)
    T.flag = datagen.uniform(T.n, -128, 127, np.int8, 5, 101)
    run_both(ctx, T)


def test_duplicate_pk_reported(ctx):
    T = datagen.make_tables(1000, 100, 3, group_by="fk")
    T.pk[7] = T.pk[8]
    fact, dim = to_dev(T)
    with pytest.raises(rel.RelError) as e:
        ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by)
    assert e.value.status == rel.DUPLICATE_KEY


@pytest.mark.parametrize("path", ["plain", "partitioned"])
def test_status_bits_of_earlier_calls(ctx, path):
    # Bits left in the sticky status word by earlier calls are neither charged
    # to a synchronising fused call nor dropped by it.
    n = 300_000 if path == "plain" else 1_200_000
    T = datagen.make_tables(n, n // 4, 12, day_lt=1500, group_by="fk", fk_zipf=0.8)
    fact, dim = to_dev(T)
    ora, _ = oracle.run_tables(T)
    assert ctx.sync() == 0
    # an out-of-range gather index: a device-side argument error
    src = torch.arange(10, dtype=torch.int32, device="cuda:0")
    idx = torch.tensor([1, 12, 3, 0], dtype=torch.int32, device="cuda:0")
    ctx.join_gather(idx, None, torch.tensor([4], dtype=torch.int64, device="cuda:0"), [(src, "fact")], max_pairs=4)
    # a fused call without statistics whose output is too small: an overflow it cannot report
    ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, stats=False, out_cap=5)
    # a synchronising call afterwards succeeds with the right result
    out, st = ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by)
    assert st["join_placement"] == ("global" if path == "plain" else "partitioned")
    assert_groups_equal(gpu_groups(out), ora, "after earlier status bits")
    # and the earlier conditions are still there for rel_ctx_sync, once
    bits = ctx.sync()
    assert bits & rel.DEV_BADARG and bits & rel.DEV_OVERFLOW
    assert ctx.sync() == 0


@pytest.mark.parametrize("placement", ["lds", "global"])
def test_planned_overflow_falls_back_to_plain(ctx, placement):
    T = datagen.make_tables(200_000, 50_000, 9, day_lt=1800, group_by="dim_grp", grp_card=5000)
    plan = rel.Plan(group_capacity=16, group_placement=rel.PLACE[placement], join_placement=0, allow_fallback=1)
    fact, dim = to_dev(T)
    ora, _ = oracle.run_tables(T)
    out, st = ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, plan=plan)
    assert st["fell_back"] == 1 and st["overflowed"] == 1
    assert_groups_equal(gpu_groups(out), ora, "fallback")
    plan.allow_fallback = 0
    with pytest.raises(rel.RelError) as e:
        ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, plan=plan)
    assert e.value.status == rel.OVERFLOW


def test_planned_right_size_is_identical(ctx):
    T = datagen.make_tables(300_000, 75_000, 10, day_lt=1200, group_by="dim_grp", grp_card=300)
    for placement in ("lds", "global"):
        plan = rel.Plan(group_capacity=400, group_placement=rel.PLACE[placement], join_placement=0, allow_fallback=1)
        st = run_both(ctx, T, plan=plan)
        assert st["fell_back"] == 0 and st["group_placement"] == placement


# -- standalone operators -------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("n", [0, 1, 15, 31, 33, 4096, 4097, 8191, 8192, 8193, 1_000_003])
@pytest.mark.parametrize("op", ["lt", "le", "gt", "ge", "eq", "ne"])
def test_filter_compact(ctx, n, op):
    col = datagen.uniform(n, -20, 20, np.int32, n + 7, 3)
    idx, c = ctx.filter_compact(torch.from_numpy(col).cuda(), op, 3)
    exp = oracle.filter_compact(col, op, 3)
    assert c == exp.shape[0]
    assert np.array_equal(idx.cpu().numpy(), exp)


def test_filter_compact_large_selectivities(ctx):
    col = datagen.uniform(60_000_000, 0, 2556, np.int32, 3, datagen.S_DAY)
    d = torch.from_numpy(col).cuda()
    for lit in (0, 1200, 2557):
        idx, c = ctx.filter_compact(d, "lt", lit)
        exp = oracle.filter_compact(col, "lt", lit)
        assert c == exp.shape[0] and np.array_equal(idx.cpu().numpy(), exp)


@pytest.mark.parametrize("with_sel", [False, True])
@pytest.mark.parametrize("with_payload", [False, True])
@pytest.mark.parametrize("n", [0, 1, 63, 511, 512, 513, 300_001])  # a wave's step is 8 x 64 probe rows
def test_join_probe(ctx, with_sel, with_payload, n):
    rng = np.random.default_rng(11 + n)
    m = 40_000
    pk = datagen.permutation(m, 0, 4, 1)
    pk[0] = -1  # the key kept in the side slot (replaces a key from 0..m-1, so pk stays unique)
    fk = rng.integers(-30_000, 30_000, size=n).astype(np.int32)
    fk[: min(50, n)] = -1
    payload = rng.integers(-(2 ** 31), 2 ** 31 - 1, size=m).astype(np.int32) if with_payload else None
    sel = np.flatnonzero(rng.random(n) < 0.45).astype(np.int32) if with_sel else None
    t = ctx.join_build(torch.from_numpy(pk).cuda(), torch.from_numpy(payload).cuda() if with_payload else None)
    fi, pl, c = t.probe(torch.from_numpy(fk).cuda(), torch.from_numpy(sel).cuda() if with_sel else None)
    efi, epl = oracle.join_probe(fk, sel, pk, payload)
    fi, pl = fi.cpu().numpy(), pl.cpu().numpy()
    o = np.argsort(fi)
    assert c == efi.shape[0]
    assert np.array_equal(fi[o], efi) and np.array_equal(pl[o], epl)
    t.close()


@pytest.mark.parametrize("placement", ["auto", "lds", "global"])
@pytest.mark.parametrize("n_keys", [1, 40, 3000, 200_000])
def test_groupby_agg(ctx, placement, n_keys):
    rng = np.random.default_rng(n_keys)
    n = 500_000
    keys = rng.integers(-(2 ** 63), 2 ** 63 - 1, size=n_keys, dtype=np.int64)
    keys[0] = np.iinfo(np.int64).min
    key = keys[rng.integers(0, n_keys, size=n)]
    price = rng.integers(-(2 ** 62), 2 ** 62, size=n, dtype=np.int64)
    qty = rng.integers(-(2 ** 31), 2 ** 31 - 1, size=n).astype(np.int32)
    sel = np.flatnonzero(rng.random(n) < 0.7).astype(np.int32)
    D = lambda a: torch.from_numpy(a).cuda()
    g = ctx.groupby_agg(D(key), D(price), D(qty), D(sel), placement=placement)
    assert_groups_equal(gpu_groups(g), oracle.groupby_agg(key, price, qty, sel), f"groupby {placement} {n_keys}")
    g = ctx.groupby_agg(D(key), D(price), D(qty), None, placement=placement)
    assert_groups_equal(gpu_groups(g), oracle.groupby_agg(key, price, qty, None), f"groupby nosel {placement} {n_keys}")


def test_invalid_arguments_are_rejected(ctx):
    x = torch.zeros(16, dtype=torch.int32, device="cuda:0")
    with pytest.raises(rel.RelError) as e:
        ctx.filter_compact(x[1:], "lt", 3)  # 4-byte offset: misaligned column
    assert e.value.status == rel.INVALID_ARG


# -- radix-partitioned groupjoin ------------------------------------------------------------------------------------------

def _partitioned():
    return rel.Plan(group_capacity=0, group_placement=0, join_placement=rel.PLACE["partitioned"], allow_fallback=0)


def _same_partition_keys(count: int, top16: int) -> np.ndarray:
    """Distinct int32 keys whose multiplicative hash (key * 2654435769 mod 2^32)
    shares its top 16 bits, so they all land in one partition at any depth <= 16."""
    inv = pow(2654435769, -1, 2 ** 32)
    h = (np.uint64(top16) << np.uint64(16)) | np.arange(count, dtype=np.uint64)
    return ((h * np.uint64(inv)) & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.int32)


# (3M, 2000): a single groupjoin unit that takes all 1.4M fact rows that pass.
@pytest.mark.parametrize("n,m,zipf", [(1, 1, 0.0), (1000, 17, 0.0), (100_003, 25_001, 0.0), (2_000_000, 500_000, 1.2),
                                      (3_000_000, 700_000, 0.8), (3_000_000, 2000, 0.0)])
def test_partitioned_groupjoin(ctx, n, m, zipf):
    T = datagen.make_tables(n, m, 500 + n, day_lt=1200, group_by="fk", fk_zipf=zipf, fk_domain=m + m // 5)
    st = run_both(ctx, T, plan=_partitioned(), repeats=2)
    assert st["join_placement"] == "partitioned"


@pytest.mark.parametrize("n,m,zipf", [(2_000_000, 200_000, 1.1), (3_000_000, 2000, 0.0)])
def test_partitioned_extreme_quantities(ctx, n, m, zipf):
    # Quantities over the whole int32 range, a third of them at its ends: the
    # per-group quantity sums reach about rows x 2^31 in either sign, in
    # split sub-units (Zipf 1.1) and in one unit of 1.8M rows (2000 dim keys).
    T = datagen.make_tables(n, m, 700 + m, day_lt=1500, group_by="fk", fk_zipf=zipf)
    rng = np.random.default_rng(m)
    q = rng.integers(-(2 ** 31), 2 ** 31, size=n, dtype=np.int64)
    ends = rng.random(n)
    q = np.where(ends < 1 / 6, -(2 ** 31), np.where(ends < 1 / 3, 2 ** 31 - 1, q))
    T.qty = q.astype(np.int32)
    st = run_both(ctx, T, plan=_partitioned())
    assert st["join_placement"] == "partitioned"


@pytest.mark.parametrize("case", ["signed_small", "high_words", "one_value", "wide_price", "wide_qty"])
def test_partitioned_narrow_row_ranges(ctx, case):
    # In the dense key order the second level writes each fact row as one
    # 64-bit word (slot, in-range bit, quantity and price offsets) when the
    # passing rows' quantities and prices span few enough values, and 16 bytes
    # otherwise: ranges around zero, far from it, a single value, and prices
    # or quantities too wide for the word (the 16-byte rows).
    n, m = 1_500_000, 200_000
    T = datagen.make_tables(n, m, 93, day_lt=1500, group_by="fk", fk_zipf=0.9)
    rng = np.random.default_rng(94)
    if case == "signed_small":
        T.price_cents = rng.integers(-5_000_000, 5_000_000, size=n, dtype=np.int64)
        T.qty = rng.integers(-100, 101, size=n).astype(np.int32)
    elif case == "high_words":
        T.price_cents = rng.integers(2 ** 40 - 10 ** 6, 2 ** 40 + 10 ** 6, size=n, dtype=np.int64)
        T.qty = rng.integers(-(2 ** 31), -(2 ** 31) + 1000, size=n).astype(np.int32)
    elif case == "one_value":
        T.price_cents = np.full(n, -123456789, np.int64)
        T.qty = np.full(n, 7, np.int32)
    elif case == "wide_price":
        T.price_cents = rng.integers(-(2 ** 62), 2 ** 62, size=n, dtype=np.int64)
    else:
        T.qty = rng.integers(-(2 ** 31), 2 ** 31, size=n, dtype=np.int64).astype(np.int32)
    st = run_both(ctx, T, plan=_partitioned(), repeats=2)
    assert st["join_placement"] == "partitioned"


@pytest.mark.parametrize("layout", ["from_int32_min", "to_int32_max", "stride3", "stride40"])
def test_partitioned_key_layouts(ctx, layout):
    # The partitions follow the dense key order when the dim keys span at most
    # 2048 x the partition count (a bijection of the key range, direct-mapped
    # LDS tables), else the hash order. Keys at either end of int32, a range
    # three times the key count (dense order, half-empty slots) and forty times
    # (hash order); about 1 in 7 fact keys lie outside the dim keys' range.
    m = 300_000
    perm = datagen.permutation(m, 0, 81, 1).astype(np.int64)
    pk = {"from_int32_min": perm - 2 ** 31, "to_int32_max": perm + (2 ** 31 - m), "stride3": 3 * perm - 7,
          "stride40": 40 * perm + 11}[layout]
    T = datagen.make_tables(1_500_000, m, 82, day_lt=1500, group_by="fk", fk_zipf=0.9)
    T.pk = pk.astype(np.int32)
    fk = T.pk[T.fk.astype(np.int64)].astype(np.int64)
    off = datagen.uniform(T.n, -3 * m, 3 * m, np.int64, 82, 5)
    out = datagen.unit(T.n, 82, 6) < 0.15
    fk = np.where(out, np.clip(fk + np.where(off >= 0, off + 1, off), -2 ** 31, 2 ** 31 - 1), fk)
    T.fk = fk.astype(np.int32)
    st = run_both(ctx, T, plan=_partitioned(), repeats=2)
    assert st["join_placement"] == "partitioned"


def test_partitioned_dense_order_widest_partitions(ctx):
    # 33M dim keys at stride 4 (a range of 2^27 less a little): the deepest
    # partitioning (16 bits over two levels of 8) with the widest dense order
    # (2^11 key positions per final partition, 2^19 per first-level partition),
    # so the presence bitmap's kernel fills the largest LDS block it asks for.
    m = 33_000_000
    perm = datagen.permutation(m, 0, 91, 1).astype(np.int64)
    T = datagen.make_tables(2_000_000, m, 92, day_lt=1500, group_by="fk", fk_zipf=0.7)
    T.pk = (4 * perm + 5).astype(np.int32)
    T.fk = T.pk[T.fk.astype(np.int64)]
    st = run_both(ctx, T, plan=_partitioned())
    assert st["join_placement"] == "partitioned"


def test_partitioned_oversized_partition_is_chunked(ctx):
    # 3000 keys in one partition exceed one LDS chunk (1400 keys): the partition
    # is processed as several units that each see all of its fact rows.
    hot = _same_partition_keys(3000, 0x1234)
    rest = datagen.permutation(2000, 1_000_000, 6, 1)
    pk = np.concatenate([hot, rest]).astype(np.int32)
    T = datagen.make_tables(400_000, pk.shape[0], 61, day_lt=1800, group_by="fk")
    T.pk = pk
    T.fk = pk[datagen.uniform(T.n, 0, pk.shape[0] - 1, np.int64, 61, 77)]
    T.fk[::7] = 5  # a key that is not in the dim table
    run_both(ctx, T, plan=_partitioned())


def test_partitioned_hot_partitions_are_split(ctx):
    # Zipf(1.5): the hottest key alone holds about a third of the rows, so its
    # partition is split into sub-units that merge through a device accumulator.
    # Three calls in a row: each must find the accumulators cleared by the last.
    T = datagen.make_tables(2_000_000, 400_000, 71, day_lt=1800, group_by="fk", fk_zipf=1.5, fk_domain=420_000)
    run_both(ctx, T, plan=_partitioned(), repeats=3)


def test_partitioned_more_hot_partitions_than_split_slots(ctx):
    # 300 hot keys take 80% of 12M rows: more hot partitions than a call can
    # split (the rest run whole). Hot keys include -1 and a key absent from dim.
    n, m = 12_000_000, 2_000_000
    T = datagen.make_tables(n, m, 72, day_lt=2557, group_by="fk", fk_domain=m)
    hot = T.pk[datagen.sample_index(300, m, 72, 90)].copy()
    T.pk[int(datagen.sample_index(1, m, 72, 91)[0])] = -1
    hot[0], hot[1] = -1, m + 100  # m + 100 is not a dim key
    pick = datagen.uniform(n, 0, 299, np.int64, 72, 92)
    is_hot = datagen.unit(n, 72, 93) < 0.8
    T.fk = np.where(is_hot, hot[pick], T.fk).astype(np.int32)
    run_both(ctx, T, plan=_partitioned(), repeats=2)


@pytest.mark.parametrize("case", ["empty_fact", "empty_dim", "all_filtered", "no_match"])
def test_partitioned_degenerate(ctx, case):
    n, m = (0 if case == "empty_fact" else 50_000), (0 if case == "empty_dim" else 9_000)
    T = datagen.make_tables(n, m, 8, day_lt=0 if case == "all_filtered" else 1800, group_by="fk")
    if case == "no_match":
        T.fk = T.fk + 100_000
    run_both(ctx, T, plan=_partitioned())


def test_partitioned_duplicate_pk_reported(ctx):
    T = datagen.make_tables(10_000, 1000, 3, group_by="fk")
    T.pk[7] = T.pk[8]
    fact, dim = to_dev(T)
    with pytest.raises(rel.RelError) as e:
        ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, plan=_partitioned())
    assert e.value.status == rel.DUPLICATE_KEY


def test_auto_picks_partitioned_for_large_fk_grouping(ctx):
    T = datagen.large(seed=34, n=2_000_000, m=500_000)
    st = run_both(ctx, T)
    assert st["join_placement"] == "partitioned"


# -- radix-partitioned join with a dim-attribute group key -----------------------------------------------------------------

@pytest.mark.parametrize("group_by,grp_card", [("prio_flag", None), ("dim_grp", 7), ("dim_grp", 300), ("dim_grp", 20_000),
                                               ("dim_grp", 3_000_000)])
@pytest.mark.parametrize("n,m,zipf", [(1, 1, 0.0), (1000, 17, 0.0), (100_003, 25_001, 0.0), (2_000_000, 500_000, 1.2)])
def test_partitioned_join_agg(ctx, group_by, grp_card, n, m, zipf):
    T = datagen.make_tables(n, m, 900 + n, day_lt=1200, group_by=group_by, fk_zipf=zipf, fk_domain=m + m // 5,
                            grp_card=grp_card)
    st = run_both(ctx, T, plan=_partitioned(), repeats=2)
    assert st["join_placement"] == "partitioned"


@pytest.mark.parametrize("placement", ["lds", "global"])
def test_partitioned_join_agg_group_placement(ctx, placement):
    # the LDS tables in front of the device table (lds), or none at all (global)
    T = datagen.make_tables(300_000, 75_000, 12, day_lt=1500, group_by="dim_grp", fk_zipf=1.1, fk_domain=80_000,
                            grp_card=3000)
    plan = rel.Plan(group_capacity=4000, group_placement=rel.PLACE[placement],
                    join_placement=rel.PLACE["partitioned"], allow_fallback=0)
    st = run_both(ctx, T, plan=plan, repeats=2)
    assert st["group_placement"] == placement and st["join_placement"] == "partitioned"


@pytest.mark.parametrize("group_by", ["prio_flag", "dim_grp"])
def test_partitioned_join_agg_chunked_and_split(ctx, group_by):
    # one partition of 3000 keys (several chunks) and a Zipf(1.5) head (split
    # partitions): every fact row still matches in exactly one unit
    hot = _same_partition_keys(3000, 0x0abc)
    rest = datagen.permutation(400_000, 2_000_000, 13, 1)
    pk = np.concatenate([hot, rest]).astype(np.int32)
    T = datagen.make_tables(2_000_000, pk.shape[0], 13, day_lt=1800, group_by=group_by, grp_card=5000)
    T.pk = pk
    T.fk = pk[datagen.zipf(T.n, pk.shape[0], 1.5, 13, 77)]
    T.fk[: T.n // 3] = hot[datagen.uniform(T.n // 3, 0, 2999, np.int64, 13, 78)]
    T.fk[::11] = -5  # not a dim key
    run_both(ctx, T, plan=_partitioned(), repeats=2)


@pytest.mark.parametrize("case", ["empty_fact", "empty_dim", "all_filtered", "no_match", "extreme_keys"])
def test_partitioned_join_agg_degenerate(ctx, case):
    n, m = (0 if case == "empty_fact" else 50_000), (0 if case == "empty_dim" else 9_000)
    T = datagen.make_tables(n, m, 14, day_lt=0 if case == "all_filtered" else 1800, group_by="dim_grp", grp_card=50)
    if case == "no_match":
        T.fk = T.fk + 100_000
    elif case == "extreme_keys":
        ext = np.array([-(2 ** 31), 2 ** 31 - 1, -1, -2, -1_000_000], np.int32)
        T.pk[:5] = ext
        T.fk[:200] = np.resize(ext, 200)
        T.grp[:5] = np.array([-1, -(2 ** 31), 2 ** 31 - 1, 5, -7], np.int32)
    run_both(ctx, T, plan=_partitioned())
    T.group_by = "prio_flag"
    if case == "extreme_keys":
        T.prio = datagen.uniform(T.m, -128, 127, np.int8, 14, 100)
        T.flag = datagen.uniform(T.n, -128, 127, np.int8, 14, 101)
    run_both(ctx, T, plan=_partitioned())


@pytest.mark.parametrize("m", [400, 1000])  # group bound min(n, m): LDS group table / per-dim-key partials
def test_partitioned_join_agg_duplicate_pk_reported(ctx, m):
    T = datagen.make_tables(10_000, m, 15, group_by="dim_grp", grp_card=40)
    T.pk[7] = T.pk[8]
    fact, dim = to_dev(T)
    with pytest.raises(rel.RelError) as e:
        ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, plan=_partitioned())
    assert e.value.status == rel.DUPLICATE_KEY


@pytest.mark.parametrize("placement", ["lds", "global"])
def test_partitioned_planned_overflow_falls_back(ctx, placement):
    T = datagen.make_tables(1_500_000, 400_000, 16, day_lt=1800, group_by="dim_grp", grp_card=5000)
    plan = rel.Plan(group_capacity=16, group_placement=rel.PLACE[placement], join_placement=rel.PLACE["partitioned"],
                    allow_fallback=1)
    fact, dim = to_dev(T)
    ora, _ = oracle.run_tables(T)
    out, st = ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, plan=plan)
    assert st["fell_back"] == 1 and st["overflowed"] == 1
    assert_groups_equal(gpu_groups(out), ora, "partitioned fallback")
    plan.allow_fallback = 0
    with pytest.raises(rel.RelError) as e:
        ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, plan=plan)
    assert e.value.status == rel.OVERFLOW


@pytest.mark.parametrize("group_by", ["fk", "dim_grp"])
@pytest.mark.parametrize("pair", [(0, 2999), (1, 1500), (700, 2100)])
def test_partitioned_duplicate_across_chunks_reported(ctx, group_by, pair):
    # 3000 keys in one partition are processed as three chunk units; a key
    # repeated far apart in the partition usually lands in two of them, where
    # each unit's own table cannot see the other copy.
    hot = _same_partition_keys(3000, 0x2468)
    rest = datagen.permutation(2000, 1_000_000, 17, 1)
    pk = np.concatenate([hot, rest]).astype(np.int32)
    pk[pair[1]] = pk[pair[0]]
    T = datagen.make_tables(50_000, pk.shape[0], 17, day_lt=1800, group_by=group_by, grp_card=40)
    T.pk = pk
    fact, dim = to_dev(T)
    with pytest.raises(rel.RelError) as e:
        ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, plan=_partitioned())
    assert e.value.status == rel.DUPLICATE_KEY
