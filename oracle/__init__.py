"""CPU oracle for the filter -> PK-FK hash join -> hash group-by pipeline.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use it; the GPU library never does. It shares no code
with the GPU library (see oracle.cpp for the definition it implements).

The relational parts are single-threaded C++ (oracle.cpp, built with g++ into
liboracle.so); the planner's MLP reference is float64 numpy (mlp.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

GROUP_BY = {"prio_flag": 0, "fk": 1, "dim_grp": 2}
CMP = {"lt": 0, "le": 1, "gt": 2, "ge": 3, "eq": 4, "ne": 5}
ERR_DUPLICATE_KEY, ERR_CAPACITY, ERR_INVALID = -1, -2, -3


class OracleError(RuntimeError):
    pass


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile liboracle.so with g++ (single-threaded, no OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        flags = ["-O2", "-g"] if not sanitize else ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
        subprocess.check_call(["g++", "-std=c++17", "-fPIC", "-shared", *flags, "-o", tmp, os.path.join(_HERE, "oracle.cpp")])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        sig = [i64, vp, vp, vp, vp, vp, i64, vp, vp, vp, i32, i32, vp, vp, vp, vp, i64, vp]
        for name in ("or_filter_join_agg", "or_brute_filter_join_agg"):
            getattr(L, name).argtypes = sig
            getattr(L, name).restype = i64
        L.or_filter_compact.argtypes = [i64, vp, i32, i32, vp, i64]
        L.or_filter_compact.restype = i64
        L.or_join_probe.argtypes = [i64, vp, vp, i64, vp, vp, vp, vp, i64]
        L.or_join_probe.restype = i64
        L.or_pred_filter.argtypes = [i64, vp, i32, vp, i32, vp, i64]
        L.or_pred_filter.restype = i64
        L.or_join_gather.argtypes = [i64, vp, vp, i64, i32, vp]
        L.or_join_gather.restype = i64
        L.or_groupby_agg.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, i64]
        L.or_groupby_agg.restype = i64
        L.or_hll_hash.argtypes = [i32]
        L.or_hll_hash.restype = ctypes.c_uint64
        L.or_hll_registers.argtypes = [i64, vp, vp]
        L.or_hll_registers.restype = None
        L.or_hll_estimate.argtypes = [vp]
        L.or_hll_estimate.restype = ctypes.c_double
        L.or_sketch_features.argtypes = [i64, vp, vp, i64, vp, vp, i32, i32, i64, vp, vp, vp, vp, vp]
        L.or_sketch_features.restype = None
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def _check(rc: int) -> int:
    if rc == ERR_DUPLICATE_KEY:
        raise OracleError("duplicate key")
    if rc == ERR_CAPACITY:
        raise OracleError("output capacity")
    if rc == ERR_INVALID:
        raise OracleError("invalid argument")
    return rc


def filter_join_agg(fk, price, qty, day, flag, pk, prio, grp, day_lt: int, group_by: str, brute: bool = False):
    """The whole query. Returns (groups, stats): groups = dict of int64 arrays
    key/sum_price/sum_qty/count sorted by key; stats = rows_passed, join_matches, groups."""
    fk, price, qty, day, flag = _c(fk, np.int32), _c(price, np.int64), _c(qty, np.int32), _c(day, np.int32), _c(flag, np.int8)
    pk, prio, grp = _c(pk, np.int32), _c(prio, np.int8), _c(grp, np.int32)
    n, m = fk.shape[0], pk.shape[0]
    cap = max(1, min(n, max(m, 1)) if group_by != "prio_flag" else min(n, 65536))
    cap = max(cap, 1)
    out = {k: np.empty(cap, np.int64) for k in ("key", "sum_price", "sum_qty", "count")}
    stats = np.zeros(3, np.int64)
    fn = lib().or_brute_filter_join_agg if brute else lib().or_filter_join_agg
    ng = _check(fn(n, _p(fk), _p(price), _p(qty), _p(day), _p(flag), m, _p(pk), _p(prio), _p(grp), int(day_lt),
                   GROUP_BY[group_by], _p(out["key"]), _p(out["sum_price"]), _p(out["sum_qty"]), _p(out["count"]), cap,
                   _p(stats)))
    groups = {k: v[:ng].copy() for k, v in out.items()}
    return groups, {"rows_passed": int(stats[0]), "join_matches": int(stats[1]), "groups": int(stats[2])}


def run_tables(T, brute: bool = False):
    """filter_join_agg over a datagen.Tables."""
    return filter_join_agg(T.fk, T.price_cents, T.qty, T.day, T.flag, T.pk, T.prio, T.grp, T.day_lt, T.group_by, brute)


def filter_compact(col, op: str, literal: int) -> np.ndarray:
    col = _c(col, np.int32)
    out = np.empty(max(col.shape[0], 1), np.int32)
    c = _check(lib().or_filter_compact(col.shape[0], _p(col), CMP[op], int(literal), _p(out), out.shape[0]))
    return out[:c].copy()


def join_probe(fk, sel, pk, payload=None):
    """(fact_idx, payload) pairs in probe order; payload None means the dim row id."""
    fk, sel, pk, payload = _c(fk, np.int32), _c(sel, np.int32), _c(pk, np.int32), _c(payload, np.int32)
    n = sel.shape[0] if sel is not None else fk.shape[0]
    oi = np.empty(max(n, 1), np.int32)
    op = np.empty(max(n, 1), np.int32)
    c = _check(lib().or_join_probe(n, _p(fk), _p(sel), pk.shape[0], _p(pk), _p(payload), _p(oi), _p(op), oi.shape[0]))
    return oi[:c].copy(), op[:c].copy()


PRED_OPS = {"lt": 0, "le": 1, "gt": 2, "ge": 3, "eq": 4, "ne": 5, "between": 6, "in": 7}
_PRED_DT = {np.dtype(np.int8): 0, np.dtype(np.int16): 1, np.dtype(np.int32): 2, np.dtype(np.int64): 3,
            np.dtype(np.float32): 4, np.dtype(np.float64): 5}
_TERM = np.dtype([("column", "<i4"), ("dtype", "<i4"), ("op", "<i4"), ("n_values", "<i4"), ("iv", "<i8", 16),
                  ("fv", "<f8", 16)])


def pred_filter(columns, terms) -> np.ndarray:
    """Ascending rows where every term holds. columns: list of numpy arrays (one
    length n; None for unused slots); terms: dicts column / op / values, the
    column's dtype decides integer (int64) or floating (double) comparison."""
    cols = [None if c is None else np.ascontiguousarray(c) for c in columns]
    n = next(c.shape[0] for c in cols if c is not None)
    t = np.zeros(len(terms), _TERM)
    for i, d in enumerate(terms):
        col = cols[d["column"]]
        fp = col.dtype.kind == "f"
        t[i]["column"], t[i]["dtype"], t[i]["op"] = d["column"], _PRED_DT[col.dtype], PRED_OPS[d["op"]]
        t[i]["n_values"] = len(d["values"])
        for j, v in enumerate(d["values"]):
            if fp:
                t[i]["fv"][j] = v
            else:
                t[i]["iv"][j] = v
    ptrs = (ctypes.c_void_p * len(cols))(*[None if c is None else c.ctypes.data for c in cols])
    out = np.empty(max(n, 1), np.int32)
    c = _check(lib().or_pred_filter(n, ptrs, len(cols), t.ctypes.data, len(terms), _p(out), out.shape[0]))
    return out[:c].copy()


def join_gather(idx, src) -> np.ndarray:
    """dst[i] = src[idx[i]] (join-output materialisation, Section 7's gather),
    element by element in plain C++; any fixed-width numpy dtype."""
    idx = _c(idx, np.int32)
    src = np.ascontiguousarray(src)
    dst = np.empty(idx.shape[0], src.dtype)
    _check(lib().or_join_gather(idx.shape[0], _p(idx), _p(src), src.shape[0], src.dtype.itemsize, _p(dst)))
    return dst


def groupby_agg(key, price, qty, sel=None):
    key, price, qty, sel = _c(key, np.int64), _c(price, np.int64), _c(qty, np.int32), _c(sel, np.int32)
    n = sel.shape[0] if sel is not None else key.shape[0]
    cap = max(n, 1)
    out = {k: np.empty(cap, np.int64) for k in ("key", "sum_price", "sum_qty", "count")}
    ng = _check(lib().or_groupby_agg(n, _p(key), _p(price), _p(qty), _p(sel), _p(out["key"]), _p(out["sum_price"]),
                                     _p(out["sum_qty"]), _p(out["count"]), cap))
    return {k: v[:ng].copy() for k, v in out.items()}


def hll_hash(key: int) -> int:
    """The sketch's 64-bit hash of one int32 key."""
    return int(lib().or_hll_hash(int(key)))


def hll_registers(keys) -> np.ndarray:
    keys = _c(keys, np.int32)
    regs = np.zeros(64, np.uint8)
    lib().or_hll_registers(keys.shape[0], _p(keys), _p(regs))
    return regs


def hll_estimate(regs) -> float:
    regs = _c(regs, np.uint8)
    return float(lib().or_hll_estimate(_p(regs)))


def sketch_features(fk, day, pk, grp, day_lt: int, group_by: str, fact_sample, dim_sample, hll_fk, hll_grp=None):
    fk, day, pk, grp = _c(fk, np.int32), _c(day, np.int32), _c(pk, np.int32), _c(grp, np.int32)
    fs, ds = _c(fact_sample, np.int64), _c(dim_sample, np.int64)
    hf = _c(hll_fk, np.uint8)
    hg = _c(hll_grp if hll_grp is not None else np.zeros(64, np.uint8), np.uint8)
    f = np.zeros(40, np.float64)
    lib().or_sketch_features(fk.shape[0], _p(fk), _p(day), pk.shape[0], _p(pk), _p(grp), int(day_lt), GROUP_BY[group_by],
                             fs.shape[0], _p(fs), _p(ds), _p(hf), _p(hg), _p(f))
    return f
