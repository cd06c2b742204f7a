"""Pins for the planner parts of the oracle: HyperLogLog, sketch features, the
float64 MLP and Adam, and the roofline calculator against Table 2."""
import json
import math
import os

import numpy as np
import pytest

import datagen
import oracle
from oracle import mlp
from paper_2608_13696_amd import roofline

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# -- HyperLogLog (Flajolet, Fusy, Gandouet, Meunier 2007) ---------------------------------------------------------------

def test_hll_single_key_sets_one_register():
    r = oracle.hll_registers(np.array([42], np.int32))
    assert int((r > 0).sum()) == 1 and 1 <= int(r.max()) <= 59


def test_hll_is_idempotent_and_mergeable():
    rng = np.random.default_rng(1)
    a = rng.integers(-10 ** 6, 10 ** 6, size=5000).astype(np.int32)
    b = rng.integers(-10 ** 6, 10 ** 6, size=7000).astype(np.int32)
    ra, rb = oracle.hll_registers(a), oracle.hll_registers(b)
    assert np.array_equal(oracle.hll_registers(np.concatenate([a, a, a])), ra)  # duplicates change nothing
    assert np.array_equal(oracle.hll_registers(np.concatenate([a, b])), np.maximum(ra, rb))  # union = max
    assert np.array_equal(oracle.hll_registers(a[::-1]), ra)  # order independent


@pytest.mark.parametrize("n", [10, 100, 1000, 30_000, 1_000_000])
def test_hll_estimate_within_error_bound(n):
    # standard error 1.04/sqrt(m) for m = 64 registers; allow 3 standard errors
    keys = datagen.permutation(n, -n // 2, 11, 99)
    est = oracle.hll_estimate(oracle.hll_registers(keys))
    assert abs(est - n) <= 3 * 1.04 / math.sqrt(64) * n + 2, (n, est)


def test_hll_estimate_empty_and_linear_counting():
    assert oracle.hll_estimate(np.zeros(64, np.uint8)) == 0.0  # m ln(m/m) = 0
    regs = np.zeros(64, np.uint8)
    regs[:8] = 1  # 8 occupied registers -> linear counting 64 ln(64/56)
    assert oracle.hll_estimate(regs) == pytest.approx(64 * math.log(64 / 56), rel=1e-12)


# -- sketch features ------------------------------------------------------------------------------------------------------

def test_sketch_features_against_numpy():
    T = datagen.make_tables(40_000, 10_000, 21, day_lt=1000, group_by="dim_grp", fk_zipf=1.0, grp_card=300)
    fs = datagen.sample_index(256, T.n, 5, 1)
    ds = datagen.sample_index(256, T.m, 5, 2)
    hf = oracle.hll_registers(T.fk)
    hg = oracle.hll_registers(T.grp)
    f = oracle.sketch_features(T.fk, T.day, T.pk, T.grp, T.day_lt, "dim_grp", fs, ds, hf, hg)
    assert f.shape == (40,)
    assert f[0] == pytest.approx(math.log2(1 + T.n)) and f[1] == pytest.approx(math.log2(1 + T.m))
    assert f[3] == pytest.approx(np.mean(T.day[fs] < T.day_lt))
    assert f[4:7].tolist() == [0.0, 1.0, 0.0]
    vals, cnt = np.unique(T.fk[fs], return_counts=True)
    assert f[7] == pytest.approx(len(vals) / 256) and f[8] == pytest.approx(np.sum(cnt == 1) / 256)
    assert f[9] == pytest.approx(np.sum(cnt == 2) / 256) and f[10] == pytest.approx(cnt.max() / 256)
    assert f[39] == pytest.approx(np.corrcoef(T.day[fs].astype(float), T.fk[fs].astype(float))[0, 1], abs=1e-12)
    assert f[21:37].sum() == pytest.approx(1.0)
    assert f[17] == pytest.approx(math.log2(1 + oracle.hll_estimate(hf)))
    gv = np.unique(T.grp[ds])
    assert f[14] == pytest.approx(len(gv) / 256)


# -- MLP -----------------------------------------------------------------------------------------------------------------

def _theta(seed=3):
    return mlp.he_uniform(datagen.unit(mlp.N_PARAMS, seed, 7))


def test_param_count():
    assert mlp.N_PARAMS == 6914


def test_forward_hand_built_network():
    # W1 copies the input into the first 40 hidden units, W2 is the identity and
    # W3 sums the hidden units into output 0 and takes unit 3 into output 1:
    # y0 = sum_i relu(x_i) + b3_0, y1 = relu(x_3).
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    p["W1"][np.arange(40), np.arange(40)] = 1.0
    p["W2"] = np.eye(64)
    p["W3"][:, 0] = 1.0
    p["W3"][3, 1] = 1.0
    p["b3"][0] = 0.5
    x = np.random.default_rng(0).normal(size=(7, 40))
    y, _ = mlp.forward(mlp.pack(p), x)
    assert np.allclose(y[:, 0], np.maximum(x, 0).sum(1) + 0.5, rtol=0, atol=1e-12)
    assert np.allclose(y[:, 1], np.maximum(x[:, 3], 0), rtol=0, atol=1e-12)


def test_gradient_matches_central_differences():
    theta = _theta()
    rng = np.random.default_rng(4)
    x = rng.normal(size=(16, 40))
    t = rng.normal(size=(16, 2))
    _, g = mlp.backward(theta, x, t)
    idx = np.concatenate([np.arange(0, mlp.N_PARAMS, 53), np.arange(mlp.N_PARAMS - 130, mlp.N_PARAMS)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        num = (mlp.loss(theta + e, x, t) - mlp.loss(theta - e, x, t)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, num, g[i])


def test_adam_first_step_and_constant_gradient_closed_form():
    rng = np.random.default_rng(8)
    theta0 = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    # With a constant gradient the bias-corrected moments are exactly g and g^2,
    # so every step moves by lr * g / (|g| + eps).
    th = theta0
    for t in range(1, 6):
        th, m, v = mlp.adam_step(th, m, v, g, t, lr=lr, eps=eps)
        assert np.allclose(th, theta0 - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-13)


# -- roofline arithmetic, pinned to Table 2 -------------------------------------------------------------------------------

def test_roofline_reproduces_table2():
    d = json.load(open(os.path.join(GOLD, "table2_roofline.json")))
    for dev, key in ((roofline.L4, "L4"), (roofline.GH200, "GH200")):
        row = d[key]
        # the printed clock is rounded to 10 MHz, so the product reproduces the
        # printed throughput to within 132 x 4 x 5 MHz = 2.6 G inst/s
        assert dev.inst_per_s / 1e9 == pytest.approx(row["inst_throughput_g"], abs=2.7)
        # Table 2 rounds a measured clock; some clock inside its +-5 MHz rounding
        # window reproduces both the printed throughput and the printed ridge
        # (throughput / (bandwidth / 32 B sectors)) with this calculator.
        ok = []
        for mhz in range(-5, 6):
            f = row["measured_clock_ghz"] * 1e9 + mhz * 1e6
            thr = roofline.inst_throughput(row["sm"], row["smsp_per_sm"], f)
            ridge = roofline.ridge_per_sector(thr, row["bandwidth_gbs"] * 1e9)
            ok.append(round(thr / 1e9) == row["inst_throughput_g"] and round(ridge, 1) == row["ridge_inst_per_sector"])
        assert any(ok), key
    assert roofline.GH200.inst_per_s / roofline.L4.inst_per_s == pytest.approx(d["ratios"]["inst_throughput"], abs=0.01)
    assert roofline.GH200.hbm_bytes_per_s / roofline.L4.hbm_bytes_per_s == pytest.approx(d["ratios"]["bandwidth"], abs=0.015)  # 4022/300 = 13.41; printed 13.42
    assert roofline.L4.ridge_sector / roofline.GH200.ridge_sector == pytest.approx(5.3, abs=0.05)


def test_mi355x_ridge():
    dev = roofline.MI355X
    assert dev.inst_per_s == pytest.approx(614.4e9)
    assert dev.ridge_byte == pytest.approx(0.0768)
    assert dev.attainable_inst_per_s(0.01) == pytest.approx(0.01 * 8e12)
    assert dev.attainable_inst_per_s(1.0) == dev.inst_per_s
