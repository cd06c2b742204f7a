"""The allocation-free selection entry point, rel_filter_compact_noalloc,
against rel_filter_compact (the entry point it mirrors) and the oracle:
bit-exact on two calls in a row, the second with a smaller input so that tile
states left in the shared scratch array by the first would show; plus its
size limit and empty input."""
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


def _compare(ctx, n, seed, op, lit):
    print(f"noalloc case n={n} seed={seed} op={op} literal={lit}", flush=True)
    col = datagen.uniform(n, 0, 2556, np.int32, seed, 3)
    d = torch.from_numpy(col).cuda()
    out = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda:0")
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
    ctx.filter_compact_noalloc(d, op, lit, out, cnt)
    ref_idx, ref_n = ctx.filter_compact(d, op, lit)  # the existing entry point, same input
    c = int(cnt.item())
    got = out[:c].cpu().numpy()
    assert c == ref_n
    assert np.array_equal(got, ref_idx.cpu().numpy())
    assert np.array_equal(got, oracle.filter_compact(col, op, lit))
    assert ctx.sync() == 0


def test_noalloc_matches_filter_compact_on_two_calls(ctx):
    _compare(ctx, 3_000_017, 41, "lt", 1200)  # 367 tiles, ragged tail
    _compare(ctx, 70_001, 42, "ge", 600)      # fewer tiles than the first call left behind


def test_noalloc_empty_input_and_size_limit(ctx):
    col = torch.zeros(16, dtype=torch.int32, device="cuda:0")
    out = torch.empty(16, dtype=torch.int32, device="cuda:0")
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
    ctx.filter_compact_noalloc(col, "lt", 5, out, cnt, n=0)
    assert int(cnt.item()) == 0
    # above the fixed array's 2^30 rows: rejected on the host before any launch
    # (the 16-row output would also fail the capacity check that follows)
    with pytest.raises(rel.RelError) as e:
        ctx.filter_compact_noalloc(col, "lt", 5, out, cnt, n=(1 << 30) + 1)
    assert e.value.status == rel.UNSUPPORTED
    assert ctx.sync() == 0
