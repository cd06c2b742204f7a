"""GPU parity of the batched (graph-captured, persistent-kernel) form against
the CPU oracle, instance by instance."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from paper_2608_13696_amd import rel
from tests.gpu_util import assert_groups_equal, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = rel.Context(0)
    yield c
    c.close()


def _instances(k, seed, n_hi=1e5, modes=("dim_grp", "fk", "prio_flag"), hint_every=2):
    specs = datagen.batch_specs(k, seed=seed, n_hi=n_hi)
    tables, insts = [], []
    for i, s in enumerate(specs):
        T = datagen.batch_instance(s)
        T.group_by = modes[i % len(modes)]
        fact, dim = to_dev(T)
        hint = s.groups if (T.group_by == "dim_grp" and i % hint_every == 0) else 0
        tables.append(T)
        insts.append((fact, dim, T.day_lt, T.group_by, hint))
    return tables, insts


def _check(batch, tables, stats=None):
    for i, T in enumerate(tables):
        ora, ost = oracle.run_tables(T)
        g = rel.sorted_groups(batch.outs[i].host())
        assert_groups_equal(g, ora, f"instance {i} n={T.n} m={T.m} group_by={T.group_by}")
        if stats is not None:
            assert stats[i]["rows_passed"] == ost["rows_passed"], i
            assert stats[i]["join_matches"] == ost["join_matches"], i
            assert stats[i]["groups"] == ost["groups"], i


def test_batch_matches_oracle(ctx):
    tables, insts = _instances(48, seed=7)
    b = rel.Batch(ctx, insts)
    b.run()
    st = b.sync()
    _check(b, tables, st)
    b.close()


def test_batch_graph_replays_with_eager_work_between(ctx):
    tables, insts = _instances(24, seed=8)
    b = rel.Batch(ctx, insts)
    junk = torch.zeros(1 << 20, device="cuda:0")
    for rep in range(3):
        for out in b.outs:  # poison the outputs so that a replay that writes nothing fails
            out.key.fill_(-7)
            out.n_groups.fill_(-1)
        b.run()
        junk.add_(1.0)  # eager work between replays
        torch.cuda.synchronize()
        st = b.sync()
        _check(b, tables, st)
    assert float(junk[0]) == 3.0
    b.close()


@pytest.mark.parametrize("tuning", [
    [dict(log2_rows_below=31, items_per_thread=1, block=64, lds_groups_max=0, rows_per_item=512)],
    [dict(log2_rows_below=14, items_per_thread=8, block=512, lds_groups_max=512, rows_per_item=4096),
     dict(log2_rows_below=31, items_per_thread=2, block=128, lds_groups_max=64, rows_per_item=1024)],
    [dict(log2_rows_below=31, items_per_thread=4, block=256, lds_groups_max=512, rows_per_item=4096, lds_join_max=1024)],
    [dict(log2_rows_below=13, items_per_thread=1, block=64, lds_groups_max=0, rows_per_item=512, lds_join_max=1024),
     dict(log2_rows_below=31, items_per_thread=8, block=512, lds_groups_max=128, rows_per_item=8192, lds_join_max=256)],
])
def test_batch_tuning_variants_agree(ctx, tuning):
    tables, insts = _instances(16, seed=9)
    b = rel.Batch(ctx, insts, tuning=tuning)
    b.run()
    _check(b, tables, b.sync())
    b.close()


@pytest.mark.parametrize("group_by", ["fk", "dim_grp", "prio_flag"])
def test_batch_lds_join_tables(ctx, group_by):
    """Instances of at most 1024 dim keys probe a join table that each work
    item builds in LDS: a dim key of -1 (the side slot) and payloads of -1
    included, fact keys outside the dim keys, one instance past the limit
    (device-memory table)."""
    tables, insts = [], []
    for i, (n, m) in enumerate([(3000, 1024), (70_000, 700), (20_000, 1), (5000, 1025), (900, 300)]):
        T = datagen.make_tables(n, m, 40 + i, day_lt=1500, group_by=group_by, grp_card=50 if group_by == "dim_grp" else None)
        if m > 2:
            T.pk[m // 2] = -1
            if T.grp is not None:
                T.grp[m // 3] = -1
            T.prio[m // 4] = -1
        T.fk[::5] = T.pk[datagen.uniform((n + 4) // 5, 0, m - 1, np.int64, 40 + i, 9)]
        T.fk[::11] = -1
        T.fk[::13] = 5_000_000 + i
        fact, dim = to_dev(T)
        tables.append(T)
        insts.append((fact, dim, T.day_lt, T.group_by, 0))
    tuning = [dict(log2_rows_below=31, items_per_thread=4, block=256, lds_groups_max=512, rows_per_item=4096,
                   lds_join_max=1024)]
    b = rel.Batch(ctx, insts, tuning=tuning)
    b.run()
    st = b.sync()
    _check(b, tables, st)
    assert [s["join_placement"] for s in st] == ["lds", "lds", "lds", "global", "lds"]
    b.close()


def test_batch_with_empty_instances(ctx):
    tables, insts = _instances(6, seed=10)
    for n, m in ((0, 100), (500, 0), (0, 0)):
        T = datagen.make_tables(n, m, 11 + n + m, day_lt=900, group_by="dim_grp", grp_card=7)
        if T.grp is None:
            T.grp = np.zeros(0, np.int32)
        fact, dim = to_dev(T)
        tables.append(T)
        insts.append((fact, dim, T.day_lt, T.group_by, 0))
    b = rel.Batch(ctx, insts)
    b.run()
    _check(b, tables, b.sync())
    b.close()


def test_batch_undersized_hint_reports_overflow(ctx):
    T = datagen.make_tables(50_000, 12_000, 12, day_lt=2000, group_by="dim_grp", grp_card=5000)
    fact, dim = to_dev(T)
    b = rel.Batch(ctx, [(fact, dim, T.day_lt, T.group_by, 8)])
    b.run()
    with pytest.raises(rel.RelError) as e:
        b.sync()
    assert e.value.status == rel.OVERFLOW
    b.close()


def test_batch_duplicate_key_reported(ctx):
    """A repeated pk in one instance is reported by rel_batch_sync; the other
    instances' results are unaffected."""
    tables, insts = _instances(6, seed=14, n_hi=3e4)
    bad = 3
    dim = insts[bad][1]
    assert dim["pk"].numel() > 2
    dim["pk"][2] = dim["pk"][1]
    b = rel.Batch(ctx, insts)
    b.run()
    with pytest.raises(rel.RelError) as e:
        b.sync()
    assert e.value.status == rel.DUPLICATE_KEY
    for i, T in enumerate(tables):
        if i == bad:
            continue
        ora, _ = oracle.run_tables(T)
        assert_groups_equal(rel.sorted_groups(b.outs[i].host()), ora, f"instance {i}")
    b.close()
    assert ctx.sync() == 0  # the status bits were cleared by the failing sync


def test_invalid_tuning_rejected(ctx):
    tables, insts = _instances(2, seed=13)
    with pytest.raises(rel.RelError) as e:
        rel.Batch(ctx, insts, tuning=[dict(log2_rows_below=31, items_per_thread=3, block=256, lds_groups_max=0,
                                           rows_per_item=768)])
    assert e.value.status == rel.INVALID_ARG
