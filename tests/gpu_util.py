"""Helpers for the GPU parity tests: move generated tables to the device and
compare GPU groups with oracle groups after canonical sorting."""
from __future__ import annotations

import numpy as np
import torch

from paper_2608_13696_amd import rel


def to_dev(T, device="cuda:0"):
    def d(a):
        return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)

    fact = {"fk": d(T.fk), "price_cents": d(T.price_cents), "qty": d(T.qty), "day": d(T.day), "flag": d(T.flag)}
    dim = {"pk": d(T.pk), "prio": d(T.prio), "grp": d(T.grp)}
    return fact, dim


def gpu_groups(groups: rel.Groups) -> dict:
    return rel.sorted_groups(groups.host())


def assert_groups_equal(gpu: dict, ora: dict, label: str = ""):
    n_o = ora["key"].shape[0]
    assert gpu["n_groups"] == n_o, f"{label}: {gpu['n_groups']} groups vs oracle {n_o}"
    for k in ("key", "sum_price", "sum_qty", "count"):
        a, b = gpu[k], ora[k]
        if not np.array_equal(a, b):
            bad = np.flatnonzero(a != b)
            raise AssertionError(f"{label}: column {k} differs at {bad.size} of {a.size} groups; first {bad[:5]}: "
                                 f"gpu {a[bad[:5]]} oracle {b[bad[:5]]}")
