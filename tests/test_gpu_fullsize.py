"""GPU parity at the benchmark sizes, in the launch configurations bench.py
times, each compared in full with the CPU oracle (bit-exact after canonical
sorting):
- the 60M-row GROUP BY fk workload (the headline);
- the 6M-row workload both as the library runs it by default (partitioned)
  and in the configuration that names it: join table in device memory, group
  table in LDS;
- the 60M-row learned-planner workload at each of its six group counts, run
  with the committed model's plan;
- all 4096 instances of the batch, one graph launch, every instance against
  the oracle (the oracle runs fan out over host threads: its C code releases
  the interpreter lock), plus invariants and a second replay.
"""
import concurrent.futures as cf
import hashlib
import os

import numpy as np
import pytest
import torch

import datagen
import oracle
from paper_2608_13696_amd import autotune, planner_train, rel
from tests.gpu_util import assert_groups_equal, gpu_groups, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = rel.Context(0)
    yield c
    c.close()


def _compare_full(ctx, T, plan=None):
    fact, dim = to_dev(T)
    out, st = ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, plan=plan)
    g = gpu_groups(out)
    del out, fact, dim
    ora, ost = oracle.run_tables(T)
    assert_groups_equal(g, ora, f"{T.meta}")
    for k in ("rows_passed", "join_matches", "groups"):
        assert st[k] == ost[k], k
    # PK-FK: every passing row joins at most once, and the counts add up to the joined rows
    assert ost["join_matches"] <= ost["rows_passed"] <= T.n
    assert int(g["count"].sum()) == ost["join_matches"]
    return st


def test_headline_60m_group_by_fk(ctx):
    """fact 60M x dim 15M, fk ~ Zipf(0.8), day < 1200, GROUP BY fk (the default bench)."""
    st = _compare_full(ctx, datagen.large())
    assert st["join_placement"] == "partitioned" and st["groups"] > 8_000_000


def test_large_uniform_60m_group_by_fk(ctx):
    """The headline's sizes with fk uniform over the 15M dim keys (12.7M groups):
    every partition and unit is full, no partition is split."""
    st = _compare_full(ctx, datagen.large_uniform())
    assert st["join_placement"] == "partitioned" and st["groups"] > 12_000_000


def test_headline_sizes_sparse_keys_hash_order(ctx):
    """The headline's sizes with the dim keys spread 40 times their count, so
    the partitions follow the hash order (not the dense one) at full size."""
    T = datagen.large()
    T.pk = (T.pk.astype(np.int64) * 40 + 3).astype(np.int32)
    T.fk = (T.fk.astype(np.int64) * 40 + 3).astype(np.int32)
    st = _compare_full(ctx, T)
    assert st["join_placement"] == "partitioned" and st["groups"] > 8_000_000


def test_medium_6m_default_path(ctx):
    """fact 6M x dim 1.5M, fk uniform, day < 1800, GROUP BY (prio, flag): the
    library's default placement for it (radix-partitioned)."""
    st = _compare_full(ctx, datagen.medium())
    assert st["groups"] == 15


def test_medium_6m_global_join_lds_groups(ctx):
    """The same 6M workload in the placement its configuration names: the dim
    hash table in device memory, the 15-group table in LDS."""
    plan = rel.Plan(group_capacity=0, group_placement=rel.PLACE["lds"], join_placement=rel.PLACE["global"],
                    allow_fallback=0)
    st = _compare_full(ctx, datagen.medium(), plan=plan)
    assert st["groups"] == 15 and st["join_placement"] == "global" and st["group_placement"] == "lds"


@pytest.mark.parametrize("G", [100, 1_000, 10_000, 100_000, 1_000_000, 10_000_000])
def test_planner_60m_planned_run(ctx, G):
    """fact 60M x dim 15M, fk ~ Zipf(1.2), GROUP BY dim.grp with grp uniform in
    [0, G), run with the committed model's plan as the planner bench runs it."""
    if not os.path.exists(planner_train.MODEL):
        pytest.skip("no trained planner model")
    T = datagen.planner_eval(G)
    params, mean, scale, margin, _ = planner_train.load_model()
    p = rel.Planner(ctx, params, mean, scale, margin)
    fact, dim = to_dev(T)
    fs = torch.from_numpy(datagen.sample_index(256, T.n, T.meta["seed"], datagen.S_SAMPLE)).cuda()
    ds = torch.from_numpy(datagen.sample_index(256, T.m, T.meta["seed"], datagen.S_SAMPLE + 1)).cuda()
    plan, _ = p.plan(fact, dim, T.day_lt, T.group_by, fs, ds)
    p.close()
    del fact, dim
    st = _compare_full(ctx, T, plan=plan)
    assert st["fell_back"] == 0


def _digest(g: dict) -> str:
    h = hashlib.sha256()
    for k in ("key", "sum_price", "sum_qty", "count"):
        h.update(np.ascontiguousarray(g[k], np.int64).tobytes())
    return h.hexdigest()


def _oracle_instance(spec):
    T = datagen.batch_instance(spec)
    ora, ost = oracle.run_tables(T)
    return _digest(ora), ost


def test_batch_4096_instances(ctx):
    """The batch bench's 4096 instances with the committed tuning, as one graph
    launch: every instance compared with the oracle, its statistics checked
    against its group bound and output, and a second replay required to agree."""
    specs = datagen.batch_specs(4096, seed=4)
    insts = []
    for s in specs:
        T = datagen.batch_instance(s)
        fact, dim = to_dev(T)
        insts.append((fact, dim, T.day_lt, "dim_grp", s.groups))
    del T
    b = rel.Batch(ctx, insts, tuning=autotune.load())
    b.run()
    st = b.sync()
    b.run()  # a second replay of the graph must give the same result
    st2 = b.sync()
    assert st == st2
    got = []
    for i, s in enumerate(specs):
        g = rel.sorted_groups(b.outs[i].host())
        assert g["n_groups"] == st[i]["groups"] <= min(s.groups, s.m, s.n)
        assert int(g["count"].sum()) == st[i]["join_matches"] <= st[i]["rows_passed"] <= s.n
        got.append(_digest(g))
    b.close()
    del insts
    oracle.lib(), datagen.lib()  # loaded once, before the threads share them
    with cf.ThreadPoolExecutor(max_workers=min(12, os.cpu_count() or 1)) as ex:
        ref = list(ex.map(_oracle_instance, specs))
    bad = [i for i in range(len(specs)) if got[i] != ref[i][0] or
           (st[i]["rows_passed"], st[i]["join_matches"], st[i]["groups"]) !=
           (ref[i][1]["rows_passed"], ref[i][1]["join_matches"], ref[i][1]["groups"])]
    assert not bad, f"{len(bad)} of {len(specs)} instances differ from the oracle; first {bad[:8]}"
