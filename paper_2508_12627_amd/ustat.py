"""Python binding of libustat (C ABI in ``include/ustat.h``).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libustat.so``.  torch provides device memory and streams.  The
functions carry the C names (``ustat_plan_create``, ``ustat_eval``,
``vstat_eval``, ...); ``Plan`` is a small convenience wrapper over them.

Importing this module loads the library and raises if it has not been built
(``python -c "import __graft_entry__ as g; g.build()"``); there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import torch  # loads the HIP runtime the library shares

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libustat.so")
# Order cost model trained on MI355X timings (written by costmodel_train);
# the default weights of order="learned" plans.
DEFAULT_COST_MODEL = os.path.join(HERE, "costmodel_mi355x.txt")

F64, F32, BF16X3, I8 = 0, 1, 2, 3
ORDER_MINFILL, ORDER_EXHAUSTIVE, ORDER_LEARNED = 0, 1, 2
PRECISIONS = {"f64": F64, "f32": F32, "bf16x3": BF16X3, "i8": I8}
ORDERS = {"minfill": ORDER_MINFILL, "exhaustive": ORDER_EXHAUSTIVE, "learned": ORDER_LEARNED}
STATUS = {0: "ok", 1: "invalid", 2: "unsupported", 3: "nomem", 4: "hip", 5: "overflow",
          6: "infeasible"}
FLAG_NO_CSE = 1
FLAG_SYMMETRIC = 2
FLAG_NO_SYM_GEMM = 4
FLAG_OVERLAP_LEVELS = 8
FACTOR_DTYPE = {F64: torch.float64, F32: torch.float32, BF16X3: torch.float32, I8: torch.int8}
PROFILE_KINDS = {"prep": 0, "gemm": 1, "elim1": 2, "reduce": 3, "rbf": 4, "lowrank_step": 5,
                 "lowrank_reduce": 6, "lowrank_outer": 7}


class UstatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ustat {STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class PlanOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("order", ctypes.c_int32),
                ("sparsify", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("workspace_limit", ctypes.c_uint64), ("cost_model_path", ctypes.c_char_p),
                ("n_hint", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("value", ctypes.c_double), ("exact_hi", ctypes.c_int64),
                ("exact_lo", ctypes.c_uint64), ("err_scale", ctypes.c_double),
                ("err_est", ctypes.c_double), ("num_vstats", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    @property
    def exact(self) -> int:
        return (int(self.exact_hi) << 64) + int(self.exact_lo)

    def as_dict(self) -> dict:
        return {"value": self.value, "exact": self.exact, "err_scale": self.err_scale,
                "err_est": self.err_est, "num_vstats": self.num_vstats}


_lib = None

EXPORTS = ["ustat_plan_opts_default", "ustat_plan_create", "ustat_plan_destroy", "ustat_plan_info",
           "ustat_plan_cost", "ustat_plan_workspace", "ustat_plan_partition", "ustat_plan_order", "ustat_graph_treewidth",
           "ustat_eval", "ustat_eval_samples", "vstat_eval", "ustat_eval_batched",
           "ustat_build_rbf", "ustat_profile_enable", "ustat_profile_reset", "ustat_profile_read",
           "ustat_order_features", "vstat_eval_ordered", "ustat_mlp_num_params",
           "ustat_mlp_predict", "ustat_mlp_loss_grad", "ustat_mlp_train", "ustat_mlp_save",
           "ustat_plan_tuning", "ustat_plan_set_tuning", "ustat_plan_autotune",
           "ustat_eval_noalloc", "ustat_debug_inject", "ustat_plan_create_motifs",
           "ustat_motif_counts", "ustat_eval_lowrank", "ustat_lowrank_info",
           "ustat_plan_autotune_batched", "ustat_peak_mfma", "ustat_peak_copy",
           "ustat_status_string", "ustat_last_error"]
NUM_FEATURES = 18


class LowrankStats(ctypes.Structure):
    _fields_ = [("madds", ctypes.c_double), ("madds_unmerged", ctypes.c_double),
                ("workspace_bytes", ctypes.c_int64), ("num_partitions", ctypes.c_int32),
                ("num_steps", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("num_exact_orders", ctypes.c_int32), ("num_greedy_orders", ctypes.c_int32),
                ("num_gemm_steps", ctypes.c_int32)]


def load_library(path: str = LIB_PATH):
    """Load libustat.so; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; the HIP engine has no fallback")
    L = ctypes.CDLL(path)
    P, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    pi32, pi64, pdbl = ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(dbl)
    L.ustat_plan_opts_default.argtypes = [ctypes.POINTER(PlanOpts)]
    L.ustat_plan_create.argtypes = [i32, i32, pi32, ctypes.POINTER(PlanOpts), ctypes.POINTER(P)]
    L.ustat_plan_destroy.argtypes = [P]
    L.ustat_plan_info.argtypes = [P, pi32, pi32, pi64, pi32]
    L.ustat_plan_cost.argtypes = [P, i64, pdbl, pdbl, ctypes.POINTER(u64)]
    L.ustat_plan_workspace.argtypes = [P, i32, pi64, i32, ctypes.POINTER(u64)]
    L.ustat_plan_partition.argtypes = [P, i32, pi32, pi64, pi32, pi32]
    L.ustat_plan_order.argtypes = [P, i32, pi32, pi32, pi32]
    L.ustat_graph_treewidth.argtypes = [i32, i32, pi32, pi32]
    L.ustat_eval.argtypes = [P, i64, ctypes.POINTER(P), P, ctypes.POINTER(Result)]
    L.ustat_eval_noalloc.argtypes = [P, i64, ctypes.POINTER(P), P, ctypes.POINTER(Result)]
    L.ustat_eval_samples.argtypes = [P, i64, i32, P, dbl, P, ctypes.POINTER(Result)]
    L.vstat_eval.argtypes = [P, pi32, i64, ctypes.POINTER(P), P, ctypes.POINTER(Result)]
    L.ustat_eval_batched.argtypes = [P, i32, pi64, i32, ctypes.POINTER(P), dbl, P,
                                     ctypes.POINTER(Result)]
    L.ustat_build_rbf.argtypes = [i64, i32, P, dbl, i32, P, P]
    L.ustat_peak_mfma.argtypes = [i32, i64, P, P, pdbl]
    L.ustat_peak_copy.argtypes = [P, P, i64, P, pdbl]
    L.ustat_profile_enable.argtypes = [i32]
    L.ustat_profile_reset.argtypes = []
    L.ustat_profile_read.argtypes = [i32, pdbl, pi64, pdbl, pdbl]
    pf32 = ctypes.POINTER(ctypes.c_float)
    L.ustat_order_features.argtypes = [P, pi32, pi32, i32, i32, i64, pf32]
    L.vstat_eval_ordered.argtypes = [P, pi32, pi32, i32, i32, i64, ctypes.POINTER(P), P,
                                     ctypes.POINTER(Result)]
    L.ustat_mlp_num_params.argtypes = [i32, i32, i32]
    L.ustat_mlp_num_params.restype = ctypes.c_size_t
    L.ustat_mlp_predict.argtypes = [i32, i32, i32, pf32, pf32, i64, pf32]
    L.ustat_mlp_loss_grad.argtypes = [i32, i32, i32, pf32, pf32, pf32, i64, pdbl, pf32]
    L.ustat_mlp_train.argtypes = [i32, i32, i32, pf32, pf32, pf32, i64, i32, ctypes.c_float, pdbl]
    L.ustat_mlp_save.argtypes = [ctypes.c_char_p, i32, i32, i32, pf32]
    L.ustat_plan_tuning.argtypes = [P, pi64, pi64]
    L.ustat_plan_set_tuning.argtypes = [P, i64, i64]
    L.ustat_plan_autotune.argtypes = [P, i64, ctypes.POINTER(P), P, i32, pdbl]
    L.ustat_plan_autotune_batched.argtypes = [P, i32, pi64, i32, ctypes.POINTER(P), dbl, P, i32, pdbl]
    L.ustat_debug_inject.argtypes = [i32, i64]
    L.ustat_plan_create_motifs.argtypes = [i32, ctypes.POINTER(PlanOpts), ctypes.POINTER(P)]
    L.ustat_motif_counts.argtypes = [P, i64, P, P, pi64]
    L.ustat_eval_lowrank.argtypes = [P, i64, i32, ctypes.POINTER(P), ctypes.POINTER(P), P,
                                     ctypes.POINTER(Result)]
    L.ustat_lowrank_info.argtypes = [P, i64, i32, pi32, ctypes.POINTER(LowrankStats)]
    L.ustat_status_string.argtypes = [i32]
    L.ustat_status_string.restype = ctypes.c_char_p
    L.ustat_last_error.argtypes = []
    L.ustat_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        f = getattr(L, name)
        if name != "ustat_mlp_num_params" and (f.restype is None or f.restype is ctypes.c_int):
            f.restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        msg = _lib.ustat_last_error().decode()
        raise UstatError(rc, msg)


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _edges_array(edges: Sequence[Tuple[int, int]]):
    flat = [int(x) for e in edges for x in e]
    return (ctypes.c_int32 * len(flat))(*flat)


# ------------------------------------------------------------------ C names

def ustat_plan_create(m: int, edges, precision="f64", order="minfill", sparsify=False,
                      workspace_limit: int = 0, cost_model_path: Optional[str] = None,
                      cse: bool = True, n_hint: int = 0, symmetric: bool = False,
                      sym_gemm: bool = True, overlap: bool = False):
    L = load_library()
    o = PlanOpts()
    _check(L.ustat_plan_opts_default(ctypes.byref(o)))
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.order = ORDERS[order] if isinstance(order, str) else int(order)
    o.sparsify = 1 if sparsify else 0
    o.flags = ((0 if cse else FLAG_NO_CSE) | (FLAG_SYMMETRIC if symmetric else 0)
               | (0 if sym_gemm else FLAG_NO_SYM_GEMM) | (FLAG_OVERLAP_LEVELS if overlap else 0))
    o.workspace_limit = int(workspace_limit)
    if o.order == ORDER_LEARNED and not cost_model_path:
        cost_model_path = DEFAULT_COST_MODEL
    o.cost_model_path = cost_model_path.encode() if cost_model_path else None
    o.n_hint = int(n_hint)
    h = ctypes.c_void_p()
    _check(L.ustat_plan_create(int(m), len(edges), _edges_array(edges), ctypes.byref(o),
                               ctypes.byref(h)))
    return h


def ustat_plan_destroy(h):
    if h:
        _check(load_library().ustat_plan_destroy(h))


def ustat_plan_info(h, m: int) -> dict:
    nv, M, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    Nl = (ctypes.c_int64 * (m + 1))()
    _check(load_library().ustat_plan_info(h, ctypes.byref(nv), ctypes.byref(M), Nl, ctypes.byref(w)))
    return {"num_vstats": nv.value, "M": M.value, "N_l": list(Nl), "max_width": w.value}


def ustat_plan_cost(h, n: int) -> dict:
    f, b, ws = ctypes.c_double(), ctypes.c_double(), ctypes.c_uint64()
    _check(load_library().ustat_plan_cost(h, int(n), ctypes.byref(f), ctypes.byref(b), ctypes.byref(ws)))
    return {"flops": f.value, "bytes": b.value, "workspace": ws.value}


def ustat_plan_workspace(h, ns, shared_factor: bool = True) -> int:
    arr = (ctypes.c_int64 * len(ns))(*[int(x) for x in ns])
    b = ctypes.c_uint64()
    _check(load_library().ustat_plan_workspace(h, len(ns), arr, 1 if shared_factor else 0,
                                               ctypes.byref(b)))
    return b.value


def ustat_plan_partition(h, idx: int, m: int) -> dict:
    blk = (ctypes.c_int32 * m)()
    mu, tw, w = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().ustat_plan_partition(h, int(idx), blk, ctypes.byref(mu), ctypes.byref(tw),
                                               ctypes.byref(w)))
    return {"block_of": list(blk), "mu": mu.value, "tw": tw.value, "width": w.value}


def ustat_plan_order(h, idx: int, m: int):
    """(order, slice_var): the elimination order of partition idx and the
    quotient vertex it conditions on (-1 for none)."""
    buf = (ctypes.c_int32 * m)()
    ln = ctypes.c_int32()
    sv = ctypes.c_int32()
    _check(load_library().ustat_plan_order(h, int(idx), buf, ctypes.byref(ln), ctypes.byref(sv)))
    return list(buf)[: ln.value], sv.value


GEMM_BIG_NEVER = 1 << 62


def ustat_plan_tuning(h) -> dict:
    gb, cb = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().ustat_plan_tuning(h, ctypes.byref(gb), ctypes.byref(cb)))
    return {"gemm_big_min": gb.value, "colred_blocks": cb.value}


def ustat_plan_set_tuning(h, gemm_big_min: int, colred_blocks: int):
    _check(load_library().ustat_plan_set_tuning(h, int(gemm_big_min), int(colred_blocks)))


def ustat_plan_autotune(h, n: int, factors, stream=None, reps: int = 3) -> float:
    """Tunes the plan's launch shapes on these factors; returns ms per eval."""
    ms = ctypes.c_double()
    _check(load_library().ustat_plan_autotune(h, int(n), _factor_ptrs(factors),
                                              _stream_handle(stream), int(reps), ctypes.byref(ms)))
    return ms.value


MOTIFS = {3: ["v-shape", "triangle"],
          4: ["3-star", "path", "tailed-triangle", "square", "diamond", "k4"]}


def ustat_plan_autotune_batched(h, Xs, divisor: float, stream=None, reps: int = 2) -> float:
    ns = (ctypes.c_int64 * len(Xs))(*[int(x.shape[0]) for x in Xs])
    ptrs = (ctypes.c_void_p * len(Xs))(*[ctypes.c_void_p(x.data_ptr()) for x in Xs])
    ms = ctypes.c_double()
    _check(load_library().ustat_plan_autotune_batched(h, len(Xs), ns, int(Xs[0].shape[1]), ptrs,
                                                      float(divisor), _stream_handle(stream), int(reps),
                                                      ctypes.byref(ms)))
    return ms.value


def ustat_plan_create_motifs(size: int, order="minfill", cse: bool = True,
                             workspace_limit: int = 0):
    L = load_library()
    o = PlanOpts()
    _check(L.ustat_plan_opts_default(ctypes.byref(o)))
    o.order = ORDERS[order] if isinstance(order, str) else int(order)
    o.flags = 0 if cse else FLAG_NO_CSE
    o.workspace_limit = int(workspace_limit)
    h = ctypes.c_void_p()
    _check(L.ustat_plan_create_motifs(int(size), ctypes.byref(o), ctypes.byref(h)))
    return h


def ustat_motif_counts(h, A: torch.Tensor, size: int, stream=None) -> List[int]:
    assert A.dtype == torch.int8 and A.is_cuda and A.is_contiguous() and A.dim() == 2
    k = len(MOTIFS[size])
    out = (ctypes.c_int64 * k)()
    _check(load_library().ustat_motif_counts(h, A.shape[0], ctypes.c_void_p(A.data_ptr()),
                                             _stream_handle(stream), out))
    return [int(x) for x in out]


class MotifPlan:
    """Owning wrapper of a motif plan (ustat_plan_create_motifs)."""

    def __init__(self, size: int, order="minfill", cse: bool = True, workspace_limit: int = 0):
        self.size = int(size)
        self.names = MOTIFS[self.size]
        self.h = ustat_plan_create_motifs(size, order, cse, workspace_limit)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.ustat_plan_destroy(h)
            self.h = None

    def counts(self, A, stream=None) -> List[int]:
        return ustat_motif_counts(self.h, A, self.size, stream)


INJECT_HOST_ALLOC, INJECT_DEVICE_ALLOC, INJECT_HIP = 0, 1, 2


def ustat_debug_inject(kind: int, countdown: int):
    """Arm a one-shot failure for tests of the error paths (see ustat.h)."""
    _check(load_library().ustat_debug_inject(int(kind), int(countdown)))


def ustat_graph_treewidth(m: int, edges) -> int:
    tw = ctypes.c_int32()
    arr = _edges_array(edges) if edges else (ctypes.c_int32 * 1)()
    _check(load_library().ustat_graph_treewidth(int(m), len(edges), arr, ctypes.byref(tw)))
    return tw.value


def _factor_ptrs(factors):
    return (ctypes.c_void_p * len(factors))(*[ctypes.c_void_p(t.data_ptr()) for t in factors])


def ustat_eval(h, n: int, factors, stream=None) -> Result:
    r = Result()
    _check(load_library().ustat_eval(h, int(n), _factor_ptrs(factors), _stream_handle(stream),
                                     ctypes.byref(r)))
    return r


def ustat_eval_noalloc(h, n: int, factors, stream=None) -> Result:
    r = Result()
    _check(load_library().ustat_eval_noalloc(h, int(n), _factor_ptrs(factors), _stream_handle(stream),
                                             ctypes.byref(r)))
    return r


def ustat_eval_lowrank(h, n: int, r: int, F, G, stream=None) -> Result:
    res = Result()
    _check(load_library().ustat_eval_lowrank(h, int(n), int(r), _factor_ptrs(F), _factor_ptrs(G),
                                             _stream_handle(stream), ctypes.byref(res)))
    return res


def ustat_lowrank_info(h, n: int, r: int, panel_ids=None) -> dict:
    st = LowrankStats()
    ids = None if panel_ids is None else (ctypes.c_int32 * len(panel_ids))(*[int(i) for i in panel_ids])
    _check(load_library().ustat_lowrank_info(h, int(n), int(r), ids, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in LowrankStats._fields_}


def ustat_eval_samples(h, X: torch.Tensor, divisor: float, stream=None) -> Result:
    assert X.dtype == torch.float64 and X.is_cuda and X.is_contiguous() and X.dim() == 2
    r = Result()
    _check(load_library().ustat_eval_samples(h, X.shape[0], X.shape[1], ctypes.c_void_p(X.data_ptr()),
                                             float(divisor), _stream_handle(stream), ctypes.byref(r)))
    return r


def vstat_eval(h, block_of: Sequence[int], n: int, factors, stream=None) -> Result:
    blk = (ctypes.c_int32 * len(block_of))(*[int(b) for b in block_of])
    r = Result()
    _check(load_library().vstat_eval(h, blk, int(n), _factor_ptrs(factors), _stream_handle(stream),
                                     ctypes.byref(r)))
    return r


def ustat_eval_batched(h, Xs: Sequence[torch.Tensor], divisor: float, stream=None) -> List[Result]:
    B = len(Xs)
    d = Xs[0].shape[1]
    for X in Xs:
        assert X.dtype == torch.float64 and X.is_cuda and X.is_contiguous() and X.shape[1] == d
    ns = (ctypes.c_int64 * B)(*[int(X.shape[0]) for X in Xs])
    ptrs = (ctypes.c_void_p * B)(*[ctypes.c_void_p(X.data_ptr()) for X in Xs])
    out = (Result * B)()
    _check(load_library().ustat_eval_batched(h, B, ns, int(d), ptrs, float(divisor),
                                             _stream_handle(stream), out))
    return list(out)


def ustat_build_rbf(X: torch.Tensor, divisor: float, precision="f64", stream=None) -> torch.Tensor:
    assert X.dtype == torch.float64 and X.is_cuda and X.is_contiguous() and X.dim() == 2
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    n, d = X.shape
    out = torch.empty((n, n), dtype=torch.float64 if p == F64 else torch.float32, device=X.device)
    _check(load_library().ustat_build_rbf(n, d, ctypes.c_void_p(X.data_ptr()), float(divisor), p,
                                          ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


PEAK_KINDS = {"bf16": 0, "f64": 1, "i8": 2, "f32": 3}


def ustat_peak_mfma(kind, iters: int = 20000, stream=None) -> float:
    """Measured MFMA rate (operations/s) of one instruction kind (see ustat.h)."""
    k = PEAK_KINDS[kind] if isinstance(kind, str) else int(kind)
    sink = torch.empty(4096 * 32, dtype=torch.uint8, device="cuda")
    rate = ctypes.c_double()
    _check(load_library().ustat_peak_mfma(k, int(iters), ctypes.c_void_p(sink.data_ptr()),
                                          _stream_handle(stream), ctypes.byref(rate)))
    return rate.value


def ustat_peak_copy(nbytes: int = 1 << 30, stream=None) -> float:
    """Measured streaming-copy rate (bytes read + written per second)."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    rate = ctypes.c_double()
    _check(load_library().ustat_peak_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                          int(nbytes), _stream_handle(stream), ctypes.byref(rate)))
    return rate.value


def ustat_profile_enable(on: bool = True):
    _check(load_library().ustat_profile_enable(1 if on else 0))


def ustat_profile_reset():
    _check(load_library().ustat_profile_reset())


def ustat_profile_read(kind) -> dict:
    k = PROFILE_KINDS[kind] if isinstance(kind, str) else int(kind)
    ms, nl, fl, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().ustat_profile_read(k, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(fl),
                                             ctypes.byref(by)))
    return {"ms": ms.value, "launches": nl.value, "flops": fl.value, "bytes": by.value}


def ustat_order_features(h, block_of, order, n: int, slice_var: int = -1):
    import numpy as np
    blk = (ctypes.c_int32 * len(block_of))(*[int(b) for b in block_of])
    od = (ctypes.c_int32 * max(1, len(order)))(*[int(o) for o in order])
    out = np.zeros(NUM_FEATURES, dtype=np.float32)
    _check(load_library().ustat_order_features(h, blk, od, len(order), int(slice_var), int(n),
                                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def vstat_eval_ordered(h, block_of, order, n: int, factors, stream=None,
                       slice_var: int = -1) -> Result:
    blk = (ctypes.c_int32 * len(block_of))(*[int(b) for b in block_of])
    od = (ctypes.c_int32 * max(1, len(order)))(*[int(o) for o in order])
    r = Result()
    _check(load_library().vstat_eval_ordered(h, blk, od, len(order), int(slice_var), int(n),
                                             _factor_ptrs(factors),
                                             _stream_handle(stream), ctypes.byref(r)))
    return r


def _f32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def ustat_mlp_num_params(F: int, H1: int, H2: int) -> int:
    return int(load_library().ustat_mlp_num_params(F, H1, H2))


def ustat_mlp_predict(F, H1, H2, params, X):
    import numpy as np
    params = np.ascontiguousarray(params, dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    out = np.zeros(X.shape[0], dtype=np.float32)
    _check(load_library().ustat_mlp_predict(F, H1, H2, _f32p(params), _f32p(X), X.shape[0], _f32p(out)))
    return out


def ustat_mlp_loss_grad(F, H1, H2, params, X, y):
    import numpy as np
    params = np.ascontiguousarray(params, dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    g = np.zeros_like(params)
    loss = ctypes.c_double()
    _check(load_library().ustat_mlp_loss_grad(F, H1, H2, _f32p(params), _f32p(X), _f32p(y), X.shape[0],
                                              ctypes.byref(loss), _f32p(g)))
    return loss.value, g


def ustat_mlp_train(F, H1, H2, params, X, y, steps: int, lr: float):
    import numpy as np
    p = np.array(params, dtype=np.float32, copy=True)
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    losses = np.zeros(steps, dtype=np.float64)
    _check(load_library().ustat_mlp_train(F, H1, H2, _f32p(p), _f32p(X), _f32p(y), X.shape[0], steps,
                                          float(lr), losses.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return p, losses


def ustat_mlp_save(path: str, F, H1, H2, params):
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(load_library().ustat_mlp_save(path.encode(), F, H1, H2, _f32p(p)))


# ------------------------------------------------------------------ wrapper

class Plan:
    """Owning wrapper of a ustat_plan handle."""

    def __init__(self, m: int, edges, precision="f64", order="minfill", sparsify=False,
                 workspace_limit: int = 0, cost_model_path: Optional[str] = None,
                 cse: bool = True, n_hint: int = 0, symmetric: bool = False,
                 sym_gemm: bool = True, overlap: bool = False):
        self.m = int(m)
        self.edges = [tuple(e) for e in edges]
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.h = ustat_plan_create(m, edges, precision, order, sparsify, workspace_limit,
                                   cost_model_path, cse, n_hint, symmetric, sym_gemm, overlap)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.ustat_plan_destroy(h)
            self.h = None

    @property
    def factor_dtype(self):
        return FACTOR_DTYPE[self.precision]

    def info(self) -> dict:
        return ustat_plan_info(self.h, self.m)

    def cost(self, n: int) -> dict:
        return ustat_plan_cost(self.h, n)

    def workspace(self, ns, shared_factor: bool = True) -> int:
        return ustat_plan_workspace(self.h, ns, shared_factor)

    def partition(self, idx: int) -> dict:
        return ustat_plan_partition(self.h, idx, self.m)

    def order(self, idx: int) -> List[int]:
        return ustat_plan_order(self.h, idx, self.m)[0]

    def tuning(self) -> dict:
        return ustat_plan_tuning(self.h)

    def set_tuning(self, gemm_big_min: int, colred_blocks: int):
        ustat_plan_set_tuning(self.h, gemm_big_min, colred_blocks)

    def autotune(self, factors, stream=None, reps: int = 3) -> float:
        n = self._check_factors(factors)
        return ustat_plan_autotune(self.h, n, factors, stream, reps)

    def autotune_batched(self, Xs, divisor: float, stream=None, reps: int = 2) -> float:
        for x in Xs:
            assert x.dtype == torch.float64 and x.is_cuda and x.is_contiguous() and x.dim() == 2
        return ustat_plan_autotune_batched(self.h, Xs, divisor, stream, reps)

    def slice_var(self, idx: int) -> int:
        return ustat_plan_order(self.h, idx, self.m)[1]

    def partitions(self) -> list:
        return [self.partition(i) for i in range(self.info()["num_vstats"])]

    def _check_factors(self, factors):
        assert len(factors) == len(self.edges), "one factor per edge"
        n = factors[0].shape[0]
        for t in factors:
            assert t.is_cuda and t.is_contiguous() and t.shape == (n, n)
            assert t.dtype == self.factor_dtype, f"factor dtype must be {self.factor_dtype}"
        return n

    def eval(self, factors, stream=None) -> Result:
        n = self._check_factors(factors)
        return ustat_eval(self.h, n, factors, stream)

    def eval_noalloc(self, factors, stream=None) -> Result:
        n = self._check_factors(factors)
        return ustat_eval_noalloc(self.h, n, factors, stream)

    def eval_samples(self, X, divisor: float, stream=None) -> Result:
        return ustat_eval_samples(self.h, X, divisor, stream)

    def eval_lowrank(self, F, G, stream=None) -> Result:
        """U from factors T_e = F[e] G[e]^T (fp64 n x r device panels)."""
        assert len(F) == len(self.edges) and len(G) == len(self.edges), "two panels per edge"
        n, r = F[0].shape
        for t in list(F) + list(G):
            assert t.is_cuda and t.is_contiguous() and t.dtype == torch.float64 and t.shape == (n, r)
        return ustat_eval_lowrank(self.h, n, r, F, G, stream)

    def lowrank_info(self, n: int, r: int, panel_ids=None) -> dict:
        return ustat_lowrank_info(self.h, n, r, panel_ids)

    def vstat(self, block_of, factors, stream=None) -> Result:
        n = self._check_factors(factors)
        return vstat_eval(self.h, block_of, n, factors, stream)

    def eval_batched(self, Xs, divisor: float, stream=None) -> List[Result]:
        return ustat_eval_batched(self.h, Xs, divisor, stream)
