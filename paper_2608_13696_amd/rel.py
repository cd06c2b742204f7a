"""Thin ctypes binding over librel's C ABI (include/rel.h).

Argument marshalling only: tensors in, device pointers out, on the current
torch stream. Every step of the computation runs in librel's HIP kernels; if
librel.so is missing this module raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librel.so")

# enums mirrored from rel.h
OK, INVALID_ARG, CAPACITY, DUPLICATE_KEY, HIP, OOM, UNSUPPORTED, OVERFLOW = range(8)
DEV_OVERFLOW, DEV_DUPKEY, DEV_BADARG = 0x1, 0x2, 0x4
CMP = {"lt": 0, "le": 1, "gt": 2, "ge": 3, "eq": 4, "ne": 5}
PLACE = {"auto": 0, "lds": 1, "global": 2, "partitioned": 3}
PLACE_NAME = {v: k for k, v in PLACE.items()}
GROUP_BY = {"prio_flag": 0, "fk": 1, "dim_grp": 2}
BW_MODE = {"read": 0, "copy": 1, "write": 2}

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


class RelError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"librel status {status}: {msg}")
        self.status = status


class TableOpts(ctypes.Structure):
    _fields_ = [("capacity_hint", _i64), ("placement", _i32), ("max_load", ctypes.c_float)]


class GroupsOut(ctypes.Structure):
    _fields_ = [("key", _vp), ("sum_price", _vp), ("sum_qty", _vp), ("count", _vp), ("cap", _i64), ("d_n_groups", _vp)]


class Fact(ctypes.Structure):
    _fields_ = [("fk", _vp), ("price_cents", _vp), ("qty", _vp), ("day", _vp), ("flag", _vp), ("n", _i64)]


class PredTerm(ctypes.Structure):
    _fields_ = [("column", _i32), ("dtype", _i32), ("op", _i32), ("n_values", _i32), ("ivalues", _i64 * 16),
                ("fvalues", ctypes.c_double * 16)]


PRED_OP = {"lt": 0, "le": 1, "gt": 2, "ge": 3, "eq": 4, "ne": 5, "between": 6, "in": 7}
PRED_MODE = {"compiled": 0, "interpreted": 1}
PRED_DTYPE = {torch.int8: 0, torch.int16: 1, torch.int32: 2, torch.int64: 3, torch.float32: 4, torch.float64: 5}


class GatherCol(ctypes.Structure):
    _fields_ = [("src", _vp), ("dst", _vp), ("src_rows", _i64), ("elem_bytes", _i32), ("side", _i32)]


SIDE = {"fact": 0, "dim": 1}


class Dim(ctypes.Structure):
    _fields_ = [("pk", _vp), ("prio", _vp), ("grp", _vp), ("m", _i64)]


class Query(ctypes.Structure):
    _fields_ = [("day_lt", _i32), ("group_by", _i32)]


class Plan(ctypes.Structure):
    _fields_ = [("group_capacity", _i64), ("group_placement", _i32), ("join_placement", _i32),
                ("allow_fallback", _i32), ("reserved", _i32)]


class Stats(ctypes.Structure):
    _fields_ = [("rows_in", _i64), ("rows_passed", _i64), ("join_matches", _i64), ("groups", _i64),
                ("join_capacity", _i64), ("group_capacity", _i64), ("join_placement", _i32),
                ("group_placement", _i32), ("overflowed", _i32), ("fell_back", _i32)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["join_placement"] = PLACE_NAME.get(d["join_placement"], d["join_placement"])
        d["group_placement"] = PLACE_NAME.get(d["group_placement"], d["group_placement"])
        return d


class BatchItem(ctypes.Structure):
    _fields_ = [("fact", Fact), ("dim", Dim), ("q", Query), ("out", GroupsOut), ("group_capacity", _i64)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("log2_rows_below", _i32), ("items_per_thread", _i32), ("block", _i32), ("lds_groups_max", _i32),
                ("rows_per_item", _i32), ("lds_join_max", _i32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """Load librel.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2608_13696_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.rel_ctx_create.argtypes = [ctypes.c_int, _vp, P(_vp)]
        L.rel_ctx_destroy.argtypes = [_vp]
        L.rel_ctx_set_stream.argtypes = [_vp, _vp]
        L.rel_ctx_sync.argtypes = [_vp, P(ctypes.c_uint32)]
        L.rel_status_string.argtypes = [ctypes.c_int]
        L.rel_status_string.restype = ctypes.c_char_p
        L.rel_last_error.argtypes = [_vp]
        L.rel_last_error.restype = ctypes.c_char_p
        L.rel_filter_compact.argtypes = [_vp, _vp, _i64, ctypes.c_int, _i32, _vp, _i64, _vp]
        L.rel_filter_compact_noalloc.argtypes = [_vp, _vp, _i64, ctypes.c_int, _i32, _vp, _i64, _vp]
        L.rel_bw_probe.argtypes = [_vp, _i32, _vp, _vp, _i64, _i32, _vp]
        L.rel_join_build.argtypes = [_vp, _vp, _vp, _i64, P(TableOpts), P(_vp)]
        L.rel_join_table_destroy.argtypes = [_vp]
        L.rel_join_probe.argtypes = [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _i64, _vp]
        L.rel_join_gather.argtypes = [_vp, _vp, _vp, _vp, _i64, P(GatherCol), _i32]
        L.rel_pred_create.argtypes = [_vp, P(PredTerm), _i32, _i32, P(_vp)]
        L.rel_pred_filter.argtypes = [_vp, P(_vp), _i32, _i64, _vp, _i64, _vp]
        L.rel_pred_destroy.argtypes = [_vp]
        L.rel_groupby_agg.argtypes = [_vp, _vp, _vp, _vp, _vp, _i64, P(TableOpts), P(GroupsOut)]
        L.rel_filter_join_agg.argtypes = [_vp, P(Fact), P(Dim), P(Query), P(Plan), P(GroupsOut), P(Stats)]
        L.rel_ctx_enable_timing.argtypes = [_vp, ctypes.c_int]
        L.rel_ctx_kernel_times.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, P(ctypes.c_int)]
        L.rel_batch_create.argtypes = [_vp, P(BatchItem), _i32, P(BatchTuning), _i32, P(_vp)]
        L.rel_batch_run.argtypes = [_vp]
        L.rel_batch_sync.argtypes = [_vp, P(Stats)]
        L.rel_batch_destroy.argtypes = [_vp]
        L.rel_sketch.argtypes = [_vp, P(Fact), P(Dim), P(Query), _vp, _vp, _i32, _vp, _vp]
        L.rel_mlp_forward.argtypes = [_vp, _vp, _vp, _i32, _vp]
        L.rel_mlp_backward.argtypes = [_vp, _vp, _vp, _vp, _i32, _vp, _vp]
        L.rel_mlp_adam_step.argtypes = [_vp, _vp, _vp, _vp, _vp, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float]
        L.rel_planner_create.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_float, P(_vp)]
        L.rel_planner_plan.argtypes = [_vp, P(Fact), P(Dim), P(Query), _vp, _vp, _i32, P(Plan), _vp]
        L.rel_planner_destroy.argtypes = [_vp]
        for name in ("rel_ctx_create", "rel_ctx_destroy", "rel_ctx_set_stream", "rel_ctx_sync", "rel_filter_compact",
                     "rel_join_build", "rel_join_table_destroy", "rel_join_probe", "rel_join_gather", "rel_pred_create", "rel_pred_filter", "rel_pred_destroy", "rel_groupby_agg",
                     "rel_filter_join_agg", "rel_ctx_enable_timing", "rel_ctx_kernel_times", "rel_batch_create",
                     "rel_batch_run", "rel_batch_sync", "rel_batch_destroy", "rel_sketch", "rel_mlp_forward",
                     "rel_mlp_backward", "rel_mlp_adam_step", "rel_planner_create", "rel_planner_plan",
                     "rel_planner_destroy"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_check(t, dtype, name):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """A librel context bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = device
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self._stream = s
        h = ctypes.c_void_p()
        st = lib().rel_ctx_create(device, ctypes.c_void_p(s.cuda_stream), ctypes.byref(h))
        if st != OK:
            raise RelError(st, "rel_ctx_create failed")
        self.h = h

    def check(self, st: int):
        if st != OK:
            msg = lib().rel_last_error(self.h).decode()
            raise RelError(st, msg or lib().rel_status_string(st).decode())

    def set_stream(self, stream: torch.cuda.Stream):
        self._stream = stream
        self.check(lib().rel_ctx_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)))

    def sync(self) -> int:
        bits = ctypes.c_uint32(0)
        self.check(lib().rel_ctx_sync(self.h, ctypes.byref(bits)))
        return bits.value

    def close(self):
        if getattr(self, "h", None):
            lib().rel_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- operators ------------------------------------------------------------------------------------------------

    def filter_compact(self, col: torch.Tensor, op: str, literal: int, sync: bool = True):
        """Stable selection vector of rows with col <op> literal. Returns (idx[:count] view, count), or with
        sync=False the full buffer and the device count (no host synchronisation)."""
        _dev_check(col, torch.int32, "col")
        n = col.numel()
        out = torch.empty(max(n, 1), dtype=torch.int32, device=col.device)
        cnt = torch.empty(1, dtype=torch.int64, device=col.device)
        self.check(lib().rel_filter_compact(self.h, _ptr(col), n, CMP[op], int(literal), _ptr(out), out.numel(), _ptr(cnt)))
        if not sync:
            return out, cnt
        c = int(cnt.item())
        return out[:c], c

    def filter_compact_noalloc(self, col: torch.Tensor, op: str, literal: int, out: torch.Tensor, count: torch.Tensor,
                               n: int | None = None):
        """rel_filter_compact_noalloc into caller buffers: out (int32, at least n
        rows) and count (one int64); n defaults to col.numel(). No allocation
        inside the library; returns nothing (the count stays on the device)."""
        _dev_check(col, torch.int32, "col")
        _dev_check(out, torch.int32, "out")
        _dev_check(count, torch.int64, "count")
        n = col.numel() if n is None else int(n)
        self.check(lib().rel_filter_compact_noalloc(self.h, _ptr(col), n, CMP[op], int(literal), _ptr(out), out.numel(),
                                                    _ptr(count)))

    def bw_probe(self, mode: str, src: torch.Tensor | None, dst: torch.Tensor | None, nbytes: int,
                 blocks_per_cu: int = 8, sink: torch.Tensor | None = None):
        """One pass of the bandwidth probe (mode "read", "copy" or "write") over nbytes."""
        if sink is None:
            sink = torch.zeros(1, dtype=torch.int64, device=(src if src is not None else dst).device)
        self.check(lib().rel_bw_probe(self.h, BW_MODE[mode], _ptr(src), _ptr(dst), int(nbytes), int(blocks_per_cu),
                                      _ptr(sink)))
        return sink

    def join_build(self, pk: torch.Tensor, payload: torch.Tensor | None = None, capacity_hint: int = 0,
                   max_load: float = 0.0) -> "JoinTable":
        _dev_check(pk, torch.int32, "pk")
        _dev_check(payload, torch.int32, "payload")
        opts = TableOpts(capacity_hint, PLACE["auto"], max_load)
        h = ctypes.c_void_p()
        self.check(lib().rel_join_build(self.h, _ptr(pk), _ptr(payload), pk.numel(), ctypes.byref(opts), ctypes.byref(h)))
        return JoinTable(self, h, pk, payload)

    def join_gather(self, fact_idx: torch.Tensor | None, dim_idx: torch.Tensor | None, d_count: torch.Tensor,
                    columns: list, max_pairs: int | None = None) -> list:
        """Materialise joined rows: for each (src, side) in columns ("fact" or
        "dim"), dst[i] = src[fact_idx[i]] or src[dim_idx[i]] for i < d_count
        (a device int64, e.g. a probe's count). Returns the dst tensors
        (max_pairs rows each; rows past the count are left unwritten)."""
        _dev_check(fact_idx, torch.int32, "fact_idx")
        _dev_check(dim_idx, torch.int32, "dim_idx")
        _dev_check(d_count, torch.int64, "d_count")
        if max_pairs is None:
            max_pairs = max(t.numel() for t in (fact_idx, dim_idx) if t is not None)
        cols = (GatherCol * len(columns))()
        outs = []
        for c, (src, side) in enumerate(columns):
            if not src.is_cuda or not src.is_contiguous():
                raise ValueError("gather sources must be contiguous device tensors")
            dst = torch.empty(max(max_pairs, 1), dtype=src.dtype, device=src.device)
            cols[c] = GatherCol(_ptr(src), _ptr(dst), src.numel(), src.element_size(), SIDE[side])
            outs.append(dst)
        self.check(lib().rel_join_gather(self.h, _ptr(fact_idx), _ptr(dim_idx), _ptr(d_count), int(max_pairs), cols,
                                         len(columns)))
        return outs

    def groupby_agg(self, key: torch.Tensor, price: torch.Tensor, qty: torch.Tensor, sel: torch.Tensor | None = None,
                    capacity_hint: int = 0, placement: str = "auto", out_cap: int | None = None):
        _dev_check(key, torch.int64, "key")
        _dev_check(price, torch.int64, "price")
        _dev_check(qty, torch.int32, "qty")
        _dev_check(sel, torch.int32, "sel")
        n = sel.numel() if sel is not None else key.numel()
        cap = out_cap if out_cap is not None else max(n, 1)
        out = _alloc_groups(cap, key.device)
        opts = TableOpts(capacity_hint, PLACE[placement], 0.0)
        self.check(lib().rel_groupby_agg(self.h, _ptr(key), _ptr(price), _ptr(qty), _ptr(sel), n, ctypes.byref(opts),
                                         ctypes.byref(out.c)))
        return out.result()

    def filter_join_agg(self, fact: dict, dim: dict, day_lt: int, group_by: str, plan: Plan | None = None,
                        stats: bool = True, out_cap: int | None = None):
        """The fused pipeline. fact: fk, price_cents, qty, day, flag; dim: pk, prio, grp (device tensors)."""
        for k, dt in (("fk", torch.int32), ("price_cents", torch.int64), ("qty", torch.int32), ("day", torch.int32),
                      ("flag", torch.int8)):
            _dev_check(fact.get(k), dt, k)
        for k, dt in (("pk", torch.int32), ("prio", torch.int8), ("grp", torch.int32)):
            _dev_check(dim.get(k), dt, k)
        n, m = fact["fk"].numel(), dim["pk"].numel()
        if out_cap is None:
            out_cap = max(1, min(n, 65536) if group_by == "prio_flag" else min(n, max(m, 1)))
        out = _alloc_groups(out_cap, fact["fk"].device)
        f = Fact(_ptr(fact["fk"]), _ptr(fact["price_cents"]), _ptr(fact["qty"]), _ptr(fact["day"]), _ptr(fact.get("flag")), n)
        d = Dim(_ptr(dim["pk"]), _ptr(dim.get("prio")), _ptr(dim.get("grp")), m)
        q = Query(int(day_lt), GROUP_BY[group_by])
        st = Stats()
        self.check(lib().rel_filter_join_agg(self.h, ctypes.byref(f), ctypes.byref(d), ctypes.byref(q),
                                             ctypes.byref(plan) if plan is not None else None, ctypes.byref(out.c),
                                             ctypes.byref(st) if stats else None))
        return out, (st.as_dict() if stats else None)


def _fact_dim_query(fact: dict, dim: dict, day_lt: int, group_by: str):
    f = Fact(_ptr(fact["fk"]), _ptr(fact.get("price_cents")), _ptr(fact.get("qty")), _ptr(fact["day"]),
             _ptr(fact.get("flag")), fact["fk"].numel())
    d = Dim(_ptr(dim["pk"]), _ptr(dim.get("prio")), _ptr(dim.get("grp")), dim["pk"].numel())
    return f, d, Query(int(day_lt), GROUP_BY[group_by])


def sketch(ctx: Context, fact: dict, dim: dict, day_lt: int, group_by: str, fsample: torch.Tensor,
           dsample: torch.Tensor):
    """(features float32[40], HLL registers uint8[128]) on the device."""
    _dev_check(fsample, torch.int64, "fsample")
    _dev_check(dsample, torch.int64, "dsample")
    f, d, q = _fact_dim_query(fact, dim, day_lt, group_by)
    feat = torch.empty(40, dtype=torch.float32, device=fact["fk"].device)
    hll = torch.empty(128, dtype=torch.uint8, device=fact["fk"].device)
    ctx.check(lib().rel_sketch(ctx.h, ctypes.byref(f), ctypes.byref(d), ctypes.byref(q), _ptr(fsample), _ptr(dsample),
                               fsample.numel(), _ptr(feat), _ptr(hll)))
    return feat, hll


def mlp_forward(ctx: Context, params: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    _dev_check(params, torch.float32, "params")
    _dev_check(x, torch.float32, "x")
    y = torch.empty((x.shape[0], 2), dtype=torch.float32, device=x.device)
    ctx.check(lib().rel_mlp_forward(ctx.h, _ptr(params), _ptr(x), x.shape[0], _ptr(y)))
    return y


def mlp_backward(ctx: Context, params: torch.Tensor, x: torch.Tensor, t: torch.Tensor, grad: torch.Tensor | None = None,
                 loss: torch.Tensor | None = None):
    for name, a in (("params", params), ("x", x), ("t", t)):
        _dev_check(a, torch.float32, name)
    grad = grad if grad is not None else torch.empty_like(params)
    loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=x.device)
    ctx.check(lib().rel_mlp_backward(ctx.h, _ptr(params), _ptr(x), _ptr(t), x.shape[0], _ptr(grad), _ptr(loss)))
    return grad, loss


def mlp_adam_step(ctx: Context, params, m, v, grad, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    ctx.check(lib().rel_mlp_adam_step(ctx.h, _ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(t), lr, beta1, beta2, eps))


class Planner:
    """Learned planner: params float32[6914], feature mean / scale float32[40],
    margin in log2 units (host numpy arrays)."""

    def __init__(self, ctx: Context, params, mean, scale, margin_log2: float):
        import numpy as np

        self.ctx = ctx
        self._arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (params, mean, scale)]
        h = ctypes.c_void_p()
        ctx.check(lib().rel_planner_create(ctx.h, *[a.ctypes.data for a in self._arrs], float(margin_log2),
                                           ctypes.byref(h)))
        self.h = h

    def plan(self, fact: dict, dim: dict, day_lt: int, group_by: str, fsample: torch.Tensor, dsample: torch.Tensor):
        f, d, q = _fact_dim_query(fact, dim, day_lt, group_by)
        p = Plan()
        pred = (ctypes.c_float * 2)()
        self.ctx.check(lib().rel_planner_plan(self.h, ctypes.byref(f), ctypes.byref(d), ctypes.byref(q), _ptr(fsample),
                                              _ptr(dsample), fsample.numel(), ctypes.byref(p), pred))
        return p, (pred[0], pred[1])

    def close(self):
        if getattr(self, "h", None):
            lib().rel_planner_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent fused queries captured into one graph launch.

    instances: list of (fact dict, dim dict, day_lt, group_by[, group_capacity]).
    Outputs are allocated here, one Groups per instance."""

    def __init__(self, ctx: Context, instances, tuning: list[dict] | None = None):
        self.ctx = ctx
        self.k = len(instances)
        self._keep = []
        self.outs = []
        arr = (BatchItem * max(self.k, 1))()
        for i, inst in enumerate(instances):
            fact, dim, day_lt, group_by = inst[:4]
            gcap = inst[4] if len(inst) > 4 else 0
            n, m = fact["fk"].numel(), dim["pk"].numel()
            bound = min(n, 65536) if group_by == "prio_flag" else min(n, max(m, 1))
            if gcap:
                bound = min(bound, gcap)
            out = _alloc_groups(max(bound, 1), fact["fk"].device)
            self.outs.append(out)
            self._keep.append((fact, dim))
            arr[i].fact = Fact(_ptr(fact["fk"]), _ptr(fact["price_cents"]), _ptr(fact["qty"]), _ptr(fact["day"]),
                               _ptr(fact.get("flag")), n)
            arr[i].dim = Dim(_ptr(dim["pk"]), _ptr(dim.get("prio")), _ptr(dim.get("grp")), m)
            arr[i].q = Query(int(day_lt), GROUP_BY[group_by])
            arr[i].out = out.c
            arr[i].group_capacity = int(gcap)
        tarr, nt = None, 0
        if tuning:
            tarr = (BatchTuning * len(tuning))(*[BatchTuning(**t) for t in tuning])
            nt = len(tuning)
        h = ctypes.c_void_p()
        ctx.check(lib().rel_batch_create(ctx.h, arr, self.k, tarr, nt, ctypes.byref(h)))
        self.h = h

    def run(self):
        self.ctx.check(lib().rel_batch_run(self.h))

    def sync(self) -> list[dict]:
        st = (Stats * max(self.k, 1))()
        self.ctx.check(lib().rel_batch_sync(self.h, st))
        return [st[i].as_dict() for i in range(self.k)]

    def close(self):
        if getattr(self, "h", None):
            lib().rel_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class JoinTable:
    def __init__(self, ctx: Context, h, pk, payload):
        self.ctx, self.h = ctx, h
        self._keep = (pk, payload)

    def probe(self, fk: torch.Tensor, sel: torch.Tensor | None = None, sync: bool = True):
        """(fact_idx, payload) pairs of matching probe rows, unordered. Returns
        (fact_idx, payload, count); with sync=False the full-size buffers and
        the device count tensor instead (no host synchronisation)."""
        _dev_check(fk, torch.int32, "fk")
        _dev_check(sel, torch.int32, "sel")
        n = sel.numel() if sel is not None else fk.numel()
        oi = torch.empty(max(n, 1), dtype=torch.int32, device=fk.device)
        op = torch.empty(max(n, 1), dtype=torch.int32, device=fk.device)
        cnt = torch.empty(1, dtype=torch.int64, device=fk.device)
        self.ctx.check(lib().rel_join_probe(self.ctx.h, self.h, _ptr(fk), _ptr(sel), n, _ptr(oi), _ptr(op), oi.numel(),
                                            _ptr(cnt)))
        if not sync:
            return oi, op, cnt
        c = int(cnt.item())
        return oi[:c], op[:c], c

    def close(self):
        if self.h:
            lib().rel_join_table_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Predicate:
    """A conjunction of terms over typed columns: each term a dict with column
    (index into the columns given to filter), op (lt le gt ge eq ne between in)
    and values; dtypes: the column dtypes by index (torch int8/16/32/64,
    float32/64). mode "compiled" builds a kernel for it at run time, mode
    "interpreted" walks the terms per row."""

    def __init__(self, ctx: Context, terms: list, dtypes: list, mode: str = "compiled"):
        self.ctx, self.h = ctx, None
        arr = (PredTerm * len(terms))()
        for i, d in enumerate(terms):
            dt = dtypes[d["column"]]
            fp = dt in (torch.float32, torch.float64)
            vals = list(d["values"])
            arr[i].column, arr[i].dtype, arr[i].op, arr[i].n_values = d["column"], PRED_DTYPE[dt], PRED_OP[d["op"]], len(vals)
            for j, v in enumerate(vals[:16]):
                if fp:
                    arr[i].fvalues[j] = float(v)
                else:
                    arr[i].ivalues[j] = int(v)
        h = ctypes.c_void_p()
        ctx.check(lib().rel_pred_create(ctx.h, arr, len(terms), PRED_MODE[mode], ctypes.byref(h)))
        self.h = h

    def filter(self, columns: list, sync: bool = True):
        """Stable selection vector of the rows passing every term. Returns
        (idx[:count], count), or with sync=False the full buffer and the device count."""
        n = next(c.numel() for c in columns if c is not None)
        for c in columns:
            if c is not None and (not c.is_cuda or not c.is_contiguous() or c.numel() < n):
                raise ValueError("predicate columns must be contiguous device tensors of at least n rows")
        ptrs = (_vp * len(columns))(*[None if c is None else c.data_ptr() for c in columns])
        dev = next(c.device for c in columns if c is not None)
        out = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        cnt = torch.empty(1, dtype=torch.int64, device=dev)
        self.ctx.check(lib().rel_pred_filter(self.h, ptrs, len(columns), n, _ptr(out), out.numel(), _ptr(cnt)))
        if not sync:
            return out, cnt
        c = int(cnt.item())
        return out[:c], c

    def close(self):
        if self.h:
            lib().rel_pred_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Groups:
    key: torch.Tensor
    sum_price: torch.Tensor
    sum_qty: torch.Tensor
    count: torch.Tensor
    n_groups: torch.Tensor  # device int64[1]
    c: GroupsOut

    def result(self) -> "Groups":
        return self

    def host(self) -> dict:
        """Copy the first n_groups rows to host numpy arrays."""
        ng = int(self.n_groups.item())
        k = min(ng, self.key.numel())
        return {"key": self.key[:k].cpu().numpy(), "sum_price": self.sum_price[:k].cpu().numpy(),
                "sum_qty": self.sum_qty[:k].cpu().numpy(), "count": self.count[:k].cpu().numpy(), "n_groups": ng}


def _alloc_groups(cap: int, device) -> Groups:
    cap = max(int(cap), 1)
    t = torch.empty((4, cap), dtype=torch.int64, device=device)
    ng = torch.empty(1, dtype=torch.int64, device=device)  # every successful call writes it
    g = Groups(t[0], t[1], t[2], t[3], ng, None)
    g.c = GroupsOut(_ptr(t[0]), _ptr(t[1]), _ptr(t[2]), _ptr(t[3]), cap, _ptr(ng))
    return g


def sorted_groups(h: dict) -> dict:
    """Canonical order (ascending key) of a host group dict."""
    import numpy as np

    o = np.argsort(h["key"], kind="stable")
    return {k: (v[o] if k != "n_groups" else v) for k, v in h.items()}
