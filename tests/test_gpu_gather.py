"""GPU parity of join-output materialisation (rel_join_gather) against the
oracle's element-by-element gather: bit-exact for every element type, on
index arrays the oracle's own probe produced, with ragged tails, both sides,
and the device-side error paths."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from paper_2608_13696_amd import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = rel.Context(0)
    yield c
    c.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _cnt(n):
    return torch.tensor([n], dtype=torch.int64, device="cuda:0")


def _columns(m, n, seed):
    rng = np.random.default_rng(seed)
    fact = [rng.integers(-(2 ** 62), 2 ** 62, size=n).astype(np.int64), rng.integers(-(2 ** 31), 2 ** 31 - 1, size=n).astype(np.int32),
            rng.integers(-128, 127, size=n).astype(np.int8)]
    dim = [rng.integers(-(2 ** 31), 2 ** 31 - 1, size=m).astype(np.int32), rng.integers(-128, 127, size=m).astype(np.int8),
           rng.integers(-(2 ** 15), 2 ** 15 - 1, size=m).astype(np.int16), rng.normal(size=m).astype(np.float64)]
    return fact, dim


@pytest.mark.parametrize("n,m", [(1, 1), (3, 2), (4, 4), (5, 3), (1027, 300), (300_001, 40_000)])
def test_gather_matches_oracle(ctx, n, m):
    T = datagen.make_tables(n, m, 60 + n, day_lt=1500, group_by="fk", fk_domain=m + m // 3)
    sel = oracle.filter_compact(T.day, "lt", T.day_lt)
    fi, di = oracle.join_probe(T.fk, sel, T.pk)  # index pairs from the oracle, not the GPU
    fact, dim = _columns(m, n, n)
    cols = [(f, "fact") for f in fact] + [(d, "dim") for d in dim]
    outs = ctx.join_gather(_dev(fi) if fi.size else None, _dev(di) if di.size else None, _cnt(fi.shape[0]),
                           [(_dev(c), side) for c, side in cols], max_pairs=fi.shape[0])
    assert ctx.sync() == 0
    for (c, side), o in zip(cols, outs):
        exp = oracle.join_gather(fi if side == "fact" else di, c)
        got = o.cpu().numpy()[: fi.shape[0]]
        assert got.dtype == exp.dtype and np.array_equal(got.view(np.uint8), exp.view(np.uint8)), (side, c.dtype)


def test_probe_then_gather_end_to_end(ctx):
    # GPU probe -> GPU gather with the device count; the fact row id rides along
    # as a gathered column, so sorting by it makes the output canonical
    T = datagen.make_tables(500_003, 120_000, 61, day_lt=1800, group_by="fk", fk_zipf=0.8, fk_domain=130_000)
    sel = oracle.filter_compact(T.day, "lt", T.day_lt)
    efi, edi = oracle.join_probe(T.fk, sel, T.pk)
    t = ctx.join_build(_dev(T.pk))
    fi, di, cnt = t.probe(_dev(T.fk), _dev(sel), sync=False)
    rows = np.arange(T.n, dtype=np.int32)
    outs = ctx.join_gather(fi, di, cnt, [(_dev(rows), "fact"), (_dev(T.price_cents), "fact"), (_dev(T.prio), "dim"),
                                         (_dev(T.pk), "dim")])
    c = int(cnt.item())
    assert c == efi.shape[0]
    got_row, got_price, got_prio, got_pk = (o.cpu().numpy()[:c] for o in outs)
    o = np.argsort(got_row)
    assert np.array_equal(got_row[o], efi)
    assert np.array_equal(got_price[o], oracle.join_gather(efi, T.price_cents))
    assert np.array_equal(got_prio[o], oracle.join_gather(edi, T.prio))
    assert np.array_equal(got_pk[o], T.fk[efi])  # the joined dim key is the fact's fk
    t.close()


def test_gather_zero_pairs_and_clamped_count(ctx):
    src = _dev(np.arange(100, dtype=np.int64))
    idx = _dev(np.array([5, 6, 7, 8, 9, 10, 11, 12], np.int32))
    (o,) = ctx.join_gather(idx, None, _cnt(0), [(src, "fact")], max_pairs=8)
    assert ctx.sync() == 0
    (o,) = ctx.join_gather(idx, None, _cnt(50), [(src, "fact")], max_pairs=8)  # count above the capacity
    assert ctx.sync() & rel.DEV_BADARG
    assert o.cpu().numpy()[:8].tolist() == list(range(5, 13))


def test_gather_out_of_range_row_is_reported(ctx):
    src = _dev(np.arange(10, dtype=np.int32))
    idx = _dev(np.array([1, 2, 10, 3, -1], np.int32))
    (o,) = ctx.join_gather(idx, None, _cnt(5), [(src, "fact")], max_pairs=5)
    assert ctx.sync() & rel.DEV_BADARG
    assert o.cpu().numpy()[:5].tolist() == [1, 2, 0, 3, 0]


def test_gather_rejects_bad_arguments(ctx):
    src = _dev(np.arange(16, dtype=np.int32))
    idx = _dev(np.arange(16, dtype=np.int32))
    with pytest.raises(rel.RelError) as e:
        ctx.join_gather(idx, None, _cnt(4), [], max_pairs=4)
    assert e.value.status == rel.INVALID_ARG
    with pytest.raises(rel.RelError) as e:
        ctx.join_gather(idx, None, _cnt(4), [(src, "fact")] * 9, max_pairs=4)
    assert e.value.status == rel.INVALID_ARG
    with pytest.raises(rel.RelError) as e:
        ctx.join_gather(idx[1:], None, _cnt(4), [(src, "fact")], max_pairs=4)  # misaligned index array
    assert e.value.status == rel.INVALID_ARG
    with pytest.raises(rel.RelError) as e:
        ctx.join_gather(None, None, _cnt(4), [(src, "dim")], max_pairs=4)  # the dim side needs dim_idx
    assert e.value.status == rel.INVALID_ARG
