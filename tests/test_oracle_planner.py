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


# SplitMix64 (Steele, Lea and Flood 2014; Vigna's reference generator): state
# advances by the golden-ratio increment, each output is the finaliser below of
# the new state. Its published first five outputs from state 0:
SPLITMIX64_SEED0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC,
                    0x1B39896A51A8749B]
_GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def _splitmix_finalise(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def test_splitmix_finaliser_reproduces_published_sequence():
    state, outs = 0, []
    for _ in range(5):
        state = (state + _GAMMA) & _M64
        outs.append(_splitmix_finalise(state))
    assert outs == SPLITMIX64_SEED0


def test_hll_hash_is_first_splitmix64_output_of_the_key():
    # key 0 seeds the generator with 0: its hash is the published first output
    assert oracle.hll_hash(0) == SPLITMIX64_SEED0[0]
    # any key: the generator seeded with the key as an unsigned 32-bit value
    rng = np.random.default_rng(17)
    keys = [1, -1, 2 ** 31 - 1, -(2 ** 31), 12345] + rng.integers(-(2 ** 31), 2 ** 31, size=200).tolist()
    for v in keys:
        assert oracle.hll_hash(v) == _splitmix_finalise(((v & 0xFFFFFFFF) + _GAMMA) & _M64), v


def _index_rho(h: int):
    idx = h >> 58
    rest = h & ((1 << 58) - 1)
    rho = 59 if rest == 0 else 58 - rest.bit_length() + 1
    return idx, rho


def test_hll_registers_by_hand():
    # 0xE220A8397B1DCDAF: top six bits 111000 = register 56; the next bit is 1, so rho = 1
    r = oracle.hll_registers(np.array([0], np.int32))
    want = np.zeros(64, np.uint8)
    want[56] = 1
    assert np.array_equal(r, want)
    # a key whose remaining bits start with several zeros, and a register that
    # keeps the larger of two values
    found = next(v for v in range(1, 1 << 20) if _index_rho(oracle.hll_hash(v))[1] >= 6)
    i1, rho1 = _index_rho(oracle.hll_hash(found))
    other = next(v for v in range(found + 1, 1 << 21) if _index_rho(oracle.hll_hash(v))[0] == i1
                 and _index_rho(oracle.hll_hash(v))[1] < rho1)
    r = oracle.hll_registers(np.array([other, found, other], np.int32))
    want = np.zeros(64, np.uint8)
    want[i1] = rho1
    assert np.array_equal(r, want), (found, other)


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


def test_sketch_features_remaining_against_numpy():
    # fk over twice the pk range, so part of the sampled fk lies outside the sampled
    # pk range; a grp domain wide enough that the grp sample has singletons and repeats
    T = datagen.make_tables(30_000, 7_000, 23, day_lt=900, group_by="dim_grp", fk_domain=14_000, grp_card=400)
    fs = datagen.sample_index(256, T.n, 6, 1)
    ds = datagen.sample_index(256, T.m, 6, 2)
    hf = oracle.hll_registers(T.fk)
    hg = oracle.hll_registers(T.grp)
    f = oracle.sketch_features(T.fk, T.day, T.pk, T.grp, T.day_lt, "dim_grp", fs, ds, hf, hg)
    sfk, spk, sgrp = T.fk[fs].astype(np.int64), T.pk[ds].astype(np.int64), T.grp[ds].astype(np.int64)
    assert f[2] == pytest.approx(math.log2((1 + T.n) / (1 + T.m)), abs=1e-12)
    inside = np.mean((sfk >= spk.min()) & (sfk <= spk.max()))
    assert 0.2 < inside < 0.8  # the case is not degenerate
    assert f[11] == pytest.approx(inside, abs=1e-12)
    assert f[12] == pytest.approx(math.log2(1 + sfk.max() - sfk.min()), abs=1e-12)
    assert f[13] == pytest.approx(math.log2(1 + spk.max() - spk.min()), abs=1e-12)
    _, gcnt = np.unique(sgrp, return_counts=True)
    assert 0 < np.sum(gcnt == 1) < len(gcnt)  # singletons and repeats both occur
    assert f[15] == pytest.approx(np.sum(gcnt == 1) / 256, abs=1e-12)
    assert f[16] == pytest.approx(math.log2(1 + sgrp.max() - sgrp.min()), abs=1e-12)
    assert f[18] == pytest.approx(np.mean(hf == 0), abs=1e-12)
    assert f[19] == pytest.approx(hf.astype(float).mean() / 16, abs=1e-12)
    assert f[20] == pytest.approx(hf.max() / 64, abs=1e-12)
    assert f[37] == pytest.approx(math.log2(1 + oracle.hll_estimate(hg)), abs=1e-12)
    assert f[38] == pytest.approx(np.mean(hg == 0), abs=1e-12)
    assert np.allclose(f[21:37], np.bincount(np.minimum(hf, 15), minlength=16) / 64, rtol=0, atol=1e-12)


def test_sketch_register_features_from_given_registers():
    # the register features read the registers they are given: a hand-made set
    # with zeros and values above the histogram's last bin (15)
    T = datagen.make_tables(1000, 250, 24, group_by="dim_grp", grp_card=10)
    fs = datagen.sample_index(256, T.n, 7, 1)
    ds = datagen.sample_index(256, T.m, 7, 2)
    hf = (np.arange(64) % 21).astype(np.uint8)  # 0..20, then 0..20, 0..20, 0
    hg = np.zeros(64, np.uint8)
    hg[:48] = 3
    f = oracle.sketch_features(T.fk, T.day, T.pk, T.grp, T.day_lt, "dim_grp", fs, ds, hf, hg)
    assert f[18] == pytest.approx(4 / 64)  # zeros at 0, 21, 42, 63
    assert f[19] == pytest.approx((3 * sum(range(21))) / 64 / 16)
    assert f[20] == pytest.approx(20 / 64)
    hist = np.zeros(16)
    hist[:15] = 3 / 64
    hist[0] = 4 / 64
    hist[15] = 3 * 6 / 64  # values 15..20, three times each
    assert np.allclose(f[21:37], hist, rtol=0, atol=1e-15)
    assert f[38] == pytest.approx(16 / 64)
    # 16 of 64 registers are zero, raw estimate above 5m/2: no linear counting
    z = 16 * 1.0 + 48 * 2.0 ** -3
    raw = 0.709 * 64 * 64 / z
    assert f[37] == pytest.approx(math.log2(1 + (raw if raw > 2.5 * 64 else 64 * math.log(64 / 16))), abs=1e-12)


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
