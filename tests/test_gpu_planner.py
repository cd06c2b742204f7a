"""The learned planner never changes results: planned runs equal the plain
pipeline and the oracle, and an undersized plan falls back to the plain
pipeline with identical output. Uses the committed model."""
import os

import numpy as np
import pytest
import torch

import datagen
import oracle
from paper_2608_13696_amd import planner_train, rel
from tests.gpu_util import assert_groups_equal, gpu_groups, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = rel.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def planner(ctx):
    if not os.path.exists(planner_train.MODEL):
        pytest.skip("no trained planner model")
    params, mean, scale, margin, _ = planner_train.load_model()
    p = rel.Planner(ctx, params, mean, scale, margin)
    yield p
    p.close()


def _samples(T):
    fs = torch.from_numpy(datagen.sample_index(256, max(T.n, 1), T.meta["seed"], datagen.S_SAMPLE)).cuda()
    ds = torch.from_numpy(datagen.sample_index(256, max(T.m, 1), T.meta["seed"], datagen.S_SAMPLE + 1)).cuda()
    return fs, ds


@pytest.mark.parametrize("groups", [100, 10_000, 1_000_000])
def test_planned_equals_plain_and_oracle(ctx, planner, groups):
    T = datagen.planner_eval(groups, seed=55, n=3_000_000, m=750_000)
    fact, dim = to_dev(T)
    fs, ds = _samples(T)
    plan, pred = planner.plan(fact, dim, T.day_lt, T.group_by, fs, ds)
    assert plan.allow_fallback == 1 and plan.group_capacity >= 1
    out_p, st_p = ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, plan=plan)
    out_0, st_0 = ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by)
    ora, ost = oracle.run_tables(T)
    gp, g0 = gpu_groups(out_p), gpu_groups(out_0)
    assert_groups_equal(gp, ora, f"planned G={groups}")
    assert_groups_equal(g0, ora, f"plain G={groups}")
    assert st_p["groups"] == ost["groups"]
    # what the network buys: a group table sized near the real group count
    # instead of the plain bound min(N, M), and no fallback
    assert st_p["fell_back"] == 0
    assert st_p["group_capacity"] < st_0["group_capacity"]
    assert st_p["group_capacity"] <= 8 * max(ost["groups"], 64), (st_p["group_capacity"], ost["groups"])


def test_undersized_plan_falls_back_identically(ctx):
    # a network whose outputs are -64 whatever the input predicts far below one
    # group: the plan is one slot, it overflows and the plain pipeline reruns
    z = np.zeros(6914, np.float32)
    z[-2:] = -64.0  # the output biases
    p = rel.Planner(ctx, z, np.zeros(40, np.float32), np.ones(40, np.float32), 0.0)
    T = datagen.planner_eval(5000, seed=56, n=1_000_000, m=250_000)
    fact, dim = to_dev(T)
    fs, ds = _samples(T)
    plan, pred = p.plan(fact, dim, T.day_lt, T.group_by, fs, ds)
    assert plan.group_capacity == 1 and pred[1] < -30
    out, st = ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, plan=plan)
    assert st["fell_back"] == 1 and st["overflowed"] == 1
    assert_groups_equal(gpu_groups(out), oracle.run_tables(T)[0], "fallback")
    p.close()


def test_prediction_tracks_group_count(ctx, planner):
    # not a parity check (the prediction has no oracle): on inputs 15x larger
    # than any training run the trained network should order group counts
    # correctly across four decades and land within a factor of 4 of each
    preds, actual = [], []
    for groups in (100, 10_000, 1_000_000):
        T = datagen.planner_eval(groups, seed=57, n=2_000_000, m=500_000)
        fact, dim = to_dev(T)
        fs, ds = _samples(T)
        _, pred = planner.plan(fact, dim, T.day_lt, T.group_by, fs, ds)
        _, st = ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by)
        preds.append(pred[1])
        actual.append(np.log2(1.0 + st["groups"]))
    assert preds[0] < preds[1] < preds[2]
    assert all(abs(p - a) < 2.0 for p, a in zip(preds, actual)), (preds, actual)


def test_planned_run_is_not_slower_than_plain(ctx, planner):
    """The gain the network buys, timed: on the 60M-row planner workload with
    1e6 groups, the planned run (sketch, network, one host read and the sized
    run) is not slower than the plain run, and both give the same groups."""
    T = datagen.planner_eval(1_000_000)
    fact, dim = to_dev(T)
    fs, ds = _samples(T)

    def plain():
        return ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, stats=False)[0]

    def planned():
        plan, _ = planner.plan(fact, dim, T.day_lt, T.group_by, fs, ds)
        return ctx.filter_join_agg(fact, dim, T.day_lt, T.group_by, plan=plan, stats=False)[0]

    a, b = gpu_groups(plain()), gpu_groups(planned())
    assert a["n_groups"] == b["n_groups"]
    for k in ("key", "sum_price", "sum_qty", "count"):
        assert np.array_equal(a[k], b[k]), k
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = {}
    for name, fn in (("plain", plain), ("planned", planned)):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms[name] = e0.elapsed_time(e1) / 5
    print(f"plain {ms['plain']:.3f} ms, planned {ms['planned']:.3f} ms", flush=True)
    assert ms["planned"] <= ms["plain"], ms
