"""Host-side logic of the batch autotuner, driven by injected timings."""
from paper_2608_13696_amd import autotune


def test_candidates_are_valid_configs():
    cs = autotune.candidates()
    assert cs
    for c in cs:
        assert c.rows_per_item % (c.items_per_thread * c.block) == 0
        assert c.lds_groups_max <= 512


def test_successive_halving_finds_the_fastest():
    cs = autotune.candidates()
    target = autotune.Candidate(4, 256, 128, 16384)
    calls = []

    def measure(c):
        calls.append(c)
        # a smooth cost with a unique minimum at target
        return 1.0 + abs(c.items_per_thread - 4) + abs(c.block - 256) / 128 + abs(c.lds_groups_max - 128) / 128 + \
            abs(c.rows_per_item - 16384) / 16384

    best, times = autotune.successive_halving(cs, measure, rounds=3)
    assert best == target
    assert len(calls) < 3 * len(cs)  # later rounds measure fewer candidates


def test_noisy_measurements_keep_running_minimum():
    cs = autotune.candidates()[:9]
    seq = iter([5.0] * 9 + [0.1] + [9.0] * 20)  # the first candidate of round two gets a lucky fast run

    best, times = autotune.successive_halving(cs, lambda c: next(seq), rounds=2)
    assert min(times.values()) == 0.1


def test_tune_builds_ascending_table_and_skips_empty_buckets():
    def bucket_measure(i):
        if i == 1:
            return None
        return lambda c: 1.0 / c.block + c.items_per_thread * 1e-3

    table, report = autotune.tune(bucket_measure)
    assert [e["log2_rows_below"] for e in table] == [12, 18, 31]
    assert all(e["block"] == 512 and e["items_per_thread"] == 1 for e in table)
    assert all(e["lds_join_max"] == 0 for e in table)  # equal times: the smaller option


def test_tune_picks_the_faster_join_placement():
    # the main search runs with device-memory join tables; then every join
    # option is measured for the winner, and the faster one is kept
    def bucket_measure(i):
        return lambda c: 1.0 / c.block + (0.0 if c.lds_join_max == 1024 else 0.5)

    table, report = autotune.tune(bucket_measure)
    assert all(e["lds_join_max"] == 1024 and e["block"] == 512 for e in table)
    assert all(any(k.startswith("join ") for k in r) for r in report.values())


def test_bucket_of_matches_library_rule():
    assert autotune.bucket_of(100) == 0
    assert autotune.bucket_of(4095) == 0 and autotune.bucket_of(4096) == 1
    assert autotune.bucket_of(10 ** 9) == len(autotune.BUCKETS) - 1
