"""Seeded synthetic inputs shared by the CPU checker and the GPU library.

Only input columns are produced here: no predicate, join or aggregation. The
arrays are host numpy arrays; the GPU side copies them to device memory.

Workloads (fact:dim = 4:1, the shape of the star-schema join in the paper's
TPC-H runs, Section 3.2; the data itself is synthetic):

* ``small``  -- 60,000 fact rows x 15,000 dim rows, group by (prio, flag).
* ``medium`` -- 6,000,000 x 1,500,000, same query.
* ``large``  -- 60,000,000 x 15,000,000, fk ~ Zipf(0.8), group by fk.
* ``batch``  -- 4096 independent instances of uneven size.
* ``planner`` -- 60,000,000 x 15,000,000, fk ~ Zipf(1.2), group by dim.grp.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libdatagen.so")

# One stream id per column, so that every column is an independent sequence.
S_FK, S_PRICE, S_QTY, S_DAY, S_FLAG, S_PK, S_PRIO, S_GRP, S_INST, S_SAMPLE = range(1, 11)

DAY_DOMAIN = 2557  # day uniform in [0, 2557)


def build(force: bool = True) -> str:
    """Compile libdatagen.so with gcc (OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-o", tmp, os.path.join(_HERE, "datagen.c"), "-lm"]
        )
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        i64, u64, vp, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_double
        for name in ("dg_uniform_i64", "dg_uniform_i32", "dg_uniform_i8"):
            getattr(L, name).argtypes = [vp, i64, i64, i64, u64, u64]
            getattr(L, name).restype = None
        L.dg_unit_f64.argtypes = [vp, i64, u64, u64]
        L.dg_permutation_i32.argtypes = [vp, i64, i64, u64, u64]
        L.dg_zipf_i32.argtypes = [vp, i64, i64, dbl, i64, u64, u64]
        L.dg_zipf_i32.restype = ctypes.c_int
        L.dg_sample_index_i64.argtypes = [vp, i64, i64, u64, u64]
        L.dg_correlated_i32.argtypes = [vp, vp, i64, i64, i64, i64, i64, i64, u64, u64]
        L.dg_draw_u64.argtypes = [u64, u64, u64]
        L.dg_draw_u64.restype = u64
        L.dg_draw_unit.argtypes = [u64, u64, u64]
        L.dg_draw_unit.restype = dbl
        _lib = L
    return _lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


def uniform(n: int, lo: int, hi: int, dtype, seed: int, stream: int) -> np.ndarray:
    """n integers uniform in the closed range [lo, hi]."""
    out = np.empty(n, dtype=dtype)
    fn = {np.dtype(np.int64): "dg_uniform_i64", np.dtype(np.int32): "dg_uniform_i32", np.dtype(np.int8): "dg_uniform_i8"}[
        np.dtype(dtype)
    ]
    getattr(lib(), fn)(_p(out), n, lo, hi, seed, stream)
    return out


def unit(n: int, seed: int, stream: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().dg_unit_f64(_p(out), n, seed, stream)
    return out


def permutation(m: int, base: int, seed: int, stream: int) -> np.ndarray:
    out = np.empty(m, dtype=np.int32)
    lib().dg_permutation_i32(_p(out), m, base, seed, stream)
    return out


def zipf(n: int, m: int, s: float, seed: int, stream: int, offset: int = 0) -> np.ndarray:
    """n keys in [offset, offset+m): rank r (key r-1+offset) has probability proportional to r^-s."""
    out = np.empty(n, dtype=np.int32)
    if lib().dg_zipf_i32(_p(out), n, m, float(s), offset, seed, stream) != 0:
        raise MemoryError("zipf alias table")
    return out


def sample_index(k: int, n: int, seed: int, stream: int = S_SAMPLE) -> np.ndarray:
    out = np.empty(k, dtype=np.int64)
    lib().dg_sample_index_i64(_p(out), k, n, seed, stream)
    return out


def correlated(key: np.ndarray, kmin: int, kmax: int, lo: int, hi: int, jitter: int, seed: int, stream: int) -> np.ndarray:
    key = np.ascontiguousarray(key, dtype=np.int32)
    out = np.empty(key.shape[0], dtype=np.int32)
    lib().dg_correlated_i32(_p(out), _p(key), key.shape[0], kmin, kmax, lo, hi, jitter, seed, stream)
    return out


def draw_unit(seed: int, stream: int, i: int) -> float:
    return float(lib().dg_draw_unit(seed, stream, i))


@dataclass
class Tables:
    """Columnar fact and dim tables (host numpy arrays) plus the query."""

    fk: np.ndarray
    price_cents: np.ndarray
    qty: np.ndarray
    day: np.ndarray
    flag: np.ndarray
    pk: np.ndarray
    prio: np.ndarray
    grp: np.ndarray | None
    day_lt: int
    group_by: str  # "prio_flag" | "fk" | "dim_grp"
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.fk.shape[0])

    @property
    def m(self) -> int:
        return int(self.pk.shape[0])

    def nbytes(self) -> int:
        tot = sum(a.nbytes for a in (self.fk, self.price_cents, self.qty, self.day, self.flag, self.pk, self.prio))
        return tot + (self.grp.nbytes if self.grp is not None else 0)


def make_tables(
    n: int,
    m: int,
    seed: int,
    *,
    day_lt: int = 1800,
    group_by: str = "prio_flag",
    fk_zipf: float = 0.0,
    fk_domain: int | None = None,
    grp_card: int | None = None,
) -> Tables:
    """Fact/dim tables with the column distributions of the star-join workloads.

    fact: fk (uniform in [0, fk_domain) or Zipf over the dim keys), price_cents
    uniform in [90000, 10500000], qty uniform in [1, 50], day uniform in
    [0, 2557), flag uniform in {0, 1, 2}. dim: pk a permutation of 0..m-1, prio
    uniform in {0..4}, and grp uniform in [0, grp_card) when grp_card is given.
    """
    dom = m if fk_domain is None else fk_domain
    if fk_zipf > 0.0:
        fk = zipf(n, max(dom, 1), fk_zipf, seed, S_FK) if n > 0 else np.empty(0, np.int32)
    else:
        fk = uniform(n, 0, max(dom, 1) - 1, np.int32, seed, S_FK)
    price = uniform(n, 90000, 10500000, np.int64, seed, S_PRICE)
    qty = uniform(n, 1, 50, np.int32, seed, S_QTY)
    day = uniform(n, 0, DAY_DOMAIN - 1, np.int32, seed, S_DAY)
    flag = uniform(n, 0, 2, np.int8, seed, S_FLAG)
    pk = permutation(m, 0, seed, S_PK)
    prio = uniform(m, 0, 4, np.int8, seed, S_PRIO)
    grp = uniform(m, 0, grp_card - 1, np.int32, seed, S_GRP) if grp_card else None
    return Tables(fk, price, qty, day, flag, pk, prio, grp, day_lt, group_by,
                  meta=dict(n=n, m=m, seed=seed, fk_zipf=fk_zipf, fk_domain=dom, grp_card=grp_card))


# -- named workloads --------------------------------------------------------------------------------------------------

def small(seed: int = 1) -> Tables:
    """60,000 x 15,000, fk uniform in [0, 15000), day < 1800, group by (prio, flag)."""
    return make_tables(60_000, 15_000, seed, day_lt=1800, group_by="prio_flag")


def medium(seed: int = 2) -> Tables:
    """6,000,000 x 1,500,000, fk uniform over the dim keys, day < 1800, group by (prio, flag)."""
    return make_tables(6_000_000, 1_500_000, seed, day_lt=1800, group_by="prio_flag")


def large(seed: int = 3, n: int = 60_000_000, m: int = 15_000_000) -> Tables:
    """60,000,000 x 15,000,000, fk ~ Zipf(0.8) over the dim keys, day < 1200, group by fk."""
    return make_tables(n, m, seed, day_lt=1200, group_by="fk", fk_zipf=0.8)


def large_uniform(seed: int = 3, n: int = 60_000_000, m: int = 15_000_000) -> Tables:
    """The large workload's sizes and query with fk uniform over the dim keys
    (no skew); a companion of `large` that isolates the cost of Zipf hot keys."""
    return make_tables(n, m, seed, day_lt=1200, group_by="fk")


def planner_eval(groups: int, seed: int = 5, n: int = 60_000_000, m: int = 15_000_000) -> Tables:
    """fk ~ Zipf(1.2) over the dim keys, day < 1200, group by dim.grp with grp uniform in [0, groups)."""
    return make_tables(n, m, seed, day_lt=1200, group_by="dim_grp", fk_zipf=1.2, grp_card=groups)


@dataclass
class InstanceSpec:
    n: int
    m: int
    groups: int
    day_lt: int
    seed: int


def batch_specs(k: int = 4096, seed: int = 4, n_lo: float = 1e3, n_hi: float = 1e6) -> list[InstanceSpec]:
    """Per-instance sizes of the batched workload.

    n log-uniform in [n_lo, n_hi], m = n // 4, group cardinality log-uniform in
    [1, 65536], selectivity uniform in [0.05, 0.95] mapped to day < round(sel * 2557).
    """
    u = unit(4 * k, seed, S_INST).reshape(k, 4)
    out = []
    for i in range(k):
        n = int(round(math.exp(math.log(n_lo) + u[i, 0] * (math.log(n_hi) - math.log(n_lo)))))
        g = int(round(math.exp(u[i, 1] * math.log(65536.0))))
        sel = 0.05 + 0.90 * u[i, 2]
        out.append(InstanceSpec(n=n, m=max(n // 4, 1), groups=max(g, 1), day_lt=int(round(sel * DAY_DOMAIN)),
                                seed=(seed << 32) | i))
    return out


def batch_instance(spec: InstanceSpec) -> Tables:
    return make_tables(spec.n, spec.m, spec.seed, day_lt=spec.day_lt, group_by="dim_grp", grp_card=spec.groups)
