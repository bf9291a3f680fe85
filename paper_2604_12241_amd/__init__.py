"""MI355X-native temporal pattern miner (thin Python binding of libamlm.so).

Every step of the mining path runs in the HIP library; this module only
marshals arguments.  PyTorch supplies device memory and streams.  If the
library has not been built the import of :func:`lib` raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamlm.so")

AMLM_FAN_OUT, AMLM_FAN_IN, AMLM_SG, AMLM_GS, AMLM_CYCLES = 1, 2, 4, 8, 16
AMLM_ALL = 31
AMLM_SG_UNORDERED = 32  # modifier of AMLM_SG: an intermediate's two legs in either order
AMLM_DEG_OUT, AMLM_DEG_IN = 64, 128  # distinct counterparties (columns after the cycle columns)
AMLM_SG_PHASE = 256       # modifier of AMLM_SG: every scatter leg before every gather leg
AMLM_CYC_ANY_ORDER = 512  # modifier of AMLM_CYCLES: a cycle's edges in any order within delta
AMLM_PART = 1024          # participation columns: the SG / GS instances each edge belongs to
AMLM_SG_SIZES = 2048      # four SG size bins: exactly k, k+1, k+2, at least k+3 intermediates (last columns)
AMLM_SCHED_STATIC, AMLM_SCHED_LEARNED, AMLM_SCHED_LENGTH, AMLM_SCHED_GIVEN = 0, 1, 2, 3
STATUS = {0: "AMLM_OK", 1: "AMLM_E_INVALID", 2: "AMLM_E_RANGE", 3: "AMLM_E_NOMEM",
          4: "AMLM_E_DEVICE", 5: "AMLM_E_ORDER", 6: "AMLM_E_BUSY"}

# every symbol the C header declares
EXPORTS = [
    "amlm_graph_create", "amlm_graph_rebuild", "amlm_graph_destroy", "amlm_graph_info",
    "amlm_num_columns", "amlm_mine", "amlm_graph_sync", "amlm_mine_work", "amlm_mine_batch",
    "amlm_costmodel_train", "amlm_costmodel_load", "amlm_costmodel_save",
    "amlm_server_create", "amlm_server_submit", "amlm_server_wait", "amlm_server_ticket_times",
    "amlm_server_destroy", "amlm_last_error", "amlm_set_timing", "amlm_stage_times",
    "amlm_costmodel_get", "amlm_mlp_forward", "amlm_mlp_grad",
    "amlm_batch_create", "amlm_batch_info", "amlm_autotune", "amlm_copy", "amlm_mlp_predict",
    "amlm_tune_set", "amlm_graph_status", "amlm_graph_set_ceiling", "amlm_graph_inject_device_error",
    "amlm_server_stats", "amlm_mine_static", "amlm_costmodel_eval", "amlm_costmodel_length_coef",
    "amlm_graph_set_costs", "amlm_server_snapshot", "amlm_server_resume", "amlm_mine_program",
]


class AmlmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class amlm_params(ctypes.Structure):
    _fields_ = [("patterns", ctypes.c_uint32), ("delta", ctypes.c_int64),
                ("max_cycle_len", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("schedule", ctypes.c_uint32)]


_lib = None


def lib():
    """Load libamlm.so (built by ``paper_2604_12241_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        p, u32, u64, i64, st = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int
        pp = ctypes.POINTER(amlm_params)
        sig = {
            "amlm_graph_create": (st, [p, p, p, p, u64, u32, ctypes.c_int, p, ctypes.POINTER(p)]),
            "amlm_graph_rebuild": (st, [p, p, p, p, u64, u32, ctypes.c_int, p]),
            "amlm_graph_destroy": (None, [p]),
            "amlm_graph_info": (st, [p, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u32),
                                     ctypes.POINTER(i64)]),
            "amlm_num_columns": (u32, [pp]),
            "amlm_mine": (st, [p, pp, p, p]),
            "amlm_graph_sync": (st, [p, p]),
            "amlm_mine_work": (st, [p, pp, p, p, p]),
            "amlm_mine_static": (st, [p, pp, p, p]),
            "amlm_mine_program": (st, [p, p, u32, i64, u32, p, p]),
            "amlm_costmodel_eval": (st, [p, pp, u64, p, p, p, ctypes.POINTER(u64), p]),
            "amlm_costmodel_length_coef": (st, [ctypes.POINTER(ctypes.c_float)]),
            "amlm_graph_set_costs": (st, [p, p]),
            "amlm_mine_batch": (st, [p, pp, p, p]),
            "amlm_batch_create": (st, [p, p, p, p, p, u32, ctypes.c_int, p, ctypes.POINTER(p)]),
            "amlm_batch_info": (st, [p, ctypes.POINTER(u32), ctypes.POINTER(u32)]),
            "amlm_autotune": (st, [p, pp, u32, p, ctypes.c_char_p, p, p]),
            "amlm_copy": (st, [p, p, u64, p]),
            "amlm_costmodel_train": (st, [p, pp, u32, u32, u32, u64, ctypes.c_char_p, p]),
            "amlm_costmodel_load": (st, [ctypes.c_char_p]),
            "amlm_costmodel_save": (st, [ctypes.c_char_p]),
            "amlm_server_create": (st, [p, pp, u64, u32, ctypes.POINTER(p)]),
            "amlm_server_submit": (st, [p, p, p, p, u64, ctypes.c_int, ctypes.POINTER(u64)]),
            "amlm_server_wait": (st, [p, u64, p, ctypes.POINTER(u64), p, p, p, u64]),
            "amlm_server_ticket_times": (st, [p, u64, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double)]),
            "amlm_server_destroy": (None, [p]),
            "amlm_server_snapshot": (st, [p, ctypes.c_char_p]),
            "amlm_server_resume": (st, [ctypes.c_char_p, u64, u32, ctypes.POINTER(p)]),
            "amlm_server_stats": (st, [p, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64),
                                       ctypes.POINTER(u64)]),
            "amlm_last_error": (ctypes.c_char_p, []),
            "amlm_set_timing": (st, [p, ctypes.c_int]),
            "amlm_tune_set": (st, [p, u32, u32, u32, u32]),
            "amlm_costmodel_get": (st, [p, p, p]),
            "amlm_mlp_forward": (st, [p, p, u32, p]),
            "amlm_mlp_predict": (st, [p, p, u32, p]),
            "amlm_mlp_grad": (st, [p, p, p, u32, p, p]),
            "amlm_stage_times": (st, [p, ctypes.POINTER(ctypes.c_float)]),
            "amlm_graph_status": (st, [p]),
            "amlm_graph_set_ceiling": (st, [p, u32]),
            "amlm_graph_inject_device_error": (st, [p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise AmlmError(status, lib().amlm_last_error().decode())


def params(patterns=AMLM_ALL, delta=86400, L=4, k=2, schedule=AMLM_SCHED_STATIC) -> amlm_params:
    return amlm_params(patterns, int(delta), int(L), int(k), int(schedule))


def amlm_num_columns(p: amlm_params) -> int:
    return int(lib().amlm_num_columns(ctypes.byref(p)))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _ptr(x):
    """Device pointer of a torch tensor or host pointer of a numpy array."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return ctypes.c_void_p(x.ctypes.data)
    return ctypes.c_void_p(int(x.data_ptr()))


class Graph:
    """Owns an ``amlm_graph`` handle (device graph store)."""

    def __init__(self, src, dst, ts, n_vertices: int, amount=None, stream=None):
        import torch
        self.handle = ctypes.c_void_p()
        on_dev = not isinstance(src, np.ndarray)
        if on_dev:
            src = src.contiguous(); dst = dst.contiguous(); ts = ts.contiguous()
            assert src.dtype == torch.int32 and dst.dtype == torch.int32 and ts.dtype == torch.int64
            n = int(src.numel())
        else:
            src = np.ascontiguousarray(src, dtype=np.uint32)
            dst = np.ascontiguousarray(dst, dtype=np.uint32)
            ts = np.ascontiguousarray(ts, dtype=np.int64)
            n = int(src.shape[0])
        self._keep = (src, dst, ts)
        _check(lib().amlm_graph_create(_ptr(src), _ptr(dst), _ptr(ts), _ptr(amount), n, int(n_vertices),
                                       1 if on_dev else 0, _stream_handle(stream), ctypes.byref(self.handle)))
        self._keep = None
        self.n_edges = n
        self.n_vertices = int(n_vertices)

    def info(self):
        ne, nv_, nvert, tb = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_int64()
        _check(lib().amlm_graph_info(self.handle, ctypes.byref(ne), ctypes.byref(nv_), ctypes.byref(nvert),
                                     ctypes.byref(tb)))
        return {"n_edges": ne.value, "n_valid": nv_.value, "n_vertices": nvert.value, "t_base": tb.value}

    def rebuild(self, src, dst, ts, n_vertices: int, stream=None):
        on_dev = not isinstance(src, np.ndarray)
        n = int(src.numel()) if on_dev else int(src.shape[0])
        if not on_dev:
            src = np.ascontiguousarray(src, dtype=np.uint32)
            dst = np.ascontiguousarray(dst, dtype=np.uint32)
            ts = np.ascontiguousarray(ts, dtype=np.int64)
        _check(lib().amlm_graph_rebuild(self.handle, _ptr(src), _ptr(dst), _ptr(ts), n, int(n_vertices),
                                        1 if on_dev else 0, _stream_handle(stream)))
        self.n_edges = n
        self.n_vertices = int(n_vertices)

    def close(self):
        if self.handle:
            lib().amlm_graph_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def amlm_mine(g: Graph, p: amlm_params, counts=None, stream=None):
    """Mine every edge; returns an int32 tensor [ncols, n_edges] (bit pattern
    of the uint32 counts) on the current device."""
    import torch
    ncols = amlm_num_columns(p)
    if ncols == 0:
        _check(lib().amlm_mine(g.handle, ctypes.byref(p), None, _stream_handle(stream)))
    if counts is None:
        counts = torch.empty((ncols, g.n_edges), dtype=torch.int32, device="cuda")
    assert counts.is_contiguous() and counts.numel() >= ncols * g.n_edges
    _check(lib().amlm_mine(g.handle, ctypes.byref(p), _ptr(counts), _stream_handle(stream)))
    return counts


def amlm_mine_static(g: Graph, p: amlm_params, counts=None, stream=None):
    """amlm_mine with the mining scratch in the library's static device array
    (no device allocation inside the call); the counts tensor, if not given,
    is allocated here by torch before the call."""
    import torch
    ncols = amlm_num_columns(p)
    if ncols == 0:
        _check(lib().amlm_mine_static(g.handle, ctypes.byref(p), None, _stream_handle(stream)))
    if counts is None:
        counts = torch.empty((ncols, g.n_edges), dtype=torch.int32, device="cuda")
    assert counts.is_contiguous() and counts.numel() >= ncols * g.n_edges
    _check(lib().amlm_mine_static(g.handle, ctypes.byref(p), _ptr(counts), _stream_handle(stream)))
    return counts


# stage-cell programs (amlm_mine_program)
AMLM_CELL_FOR_OUT, AMLM_CELL_FOR_IN, AMLM_CELL_PROBE = 0, 1, 2
AMLM_T_WINDOW, AMLM_T_AFTER = 0, 1
AMLM_T_THROUGH, AMLM_T_BEFORE = 0, 1
AMLM_AGG_SUM, AMLM_AGG_AT_LEAST, AMLM_AGG_AT_LEAST_K = 0, 1, 2
VAR_U, VAR_V = 0, 1


class amlm_cell(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint8), ("node", ctypes.c_uint8), ("peer", ctypes.c_uint8),
                ("tlo", ctypes.c_uint8), ("tref", ctypes.c_uint8), ("thi", ctypes.c_uint8),
                ("skip", ctypes.c_uint8), ("distinct", ctypes.c_uint8), ("agg", ctypes.c_uint8),
                ("pad", ctypes.c_uint8 * 3), ("threshold", ctypes.c_uint32)]


def cell(op, node, peer=0, tlo=AMLM_T_WINDOW, tref=0, thi=AMLM_T_THROUGH, skip=(), distinct=False,
         agg=AMLM_AGG_SUM, threshold=0) -> amlm_cell:
    """One stage cell; `skip` lists the vertices whose equals are skipped."""
    mask = 0
    for b in skip:
        mask |= 1 << b
    return amlm_cell(op, node, peer, tlo, tref, thi, mask, 1 if distinct else 0, agg, (0, 0, 0), threshold)


def amlm_mine_program(g: Graph, cells, delta: int, k: int = 1, out=None, stream=None):
    """The first cell's value per anchor: an int32 tensor [n_edges] holding
    uint32 bit patterns."""
    import torch
    arr = (amlm_cell * len(cells))(*cells)
    if out is None:
        out = torch.empty(max(1, g.n_edges), dtype=torch.int32, device="cuda")
    _check(lib().amlm_mine_program(g.handle, arr, len(cells), int(delta), int(k), _ptr(out),
                                   _stream_handle(stream)))
    return out[:g.n_edges]


WORK_ROWS = ["io", "sg", "cyc", "sg_impl"]


def amlm_mine_work(g: Graph, p: amlm_params, counts=None, work=None, stream=None):
    """Mining plus per-anchor byte counters: returns (counts, work) with work
    an int64 tensor [4, n_edges] (rows WORK_ROWS: the method's algorithmic
    bytes B_io, B_sg/gs, B_cyc, then the scatter-gather kernel's own bytes)."""
    import torch
    ncols = amlm_num_columns(p)
    if counts is None:
        counts = torch.empty((ncols, g.n_edges), dtype=torch.int32, device="cuda")
    if work is None:
        work = torch.empty((4, g.n_edges), dtype=torch.int64, device="cuda")
    _check(lib().amlm_mine_work(g.handle, ctypes.byref(p), _ptr(counts), _ptr(work), _stream_handle(stream)))
    return counts, work


STAGES = ["build", "anchor", "lists", "sg", "cyc", "model", "units", "mine"]


def amlm_set_timing(g: Graph, enable: bool = True):
    _check(lib().amlm_set_timing(g.handle, 1 if enable else 0))


def amlm_tune_set(g: Graph, block=0, sg_blocks=0, cyc_blocks=0, split_bytes=0):
    """Pin the launch shape of later mining calls on g (0 = default)."""
    _check(lib().amlm_tune_set(g.handle, block, sg_blocks, cyc_blocks, split_bytes))


def amlm_stage_times(g: Graph) -> dict:
    arr = (ctypes.c_float * 8)()
    _check(lib().amlm_stage_times(g.handle, arr))
    return {STAGES[i]: float(arr[i]) for i in range(8) if arr[i] >= 0}


def amlm_graph_sync(g: Graph, stream=None):
    _check(lib().amlm_graph_sync(g.handle, _stream_handle(stream)))


def amlm_graph_status(g: Graph) -> int:
    """The handle's sticky status (0 = healthy)."""
    return int(lib().amlm_graph_status(g.handle))


def amlm_graph_set_ceiling(g: Graph, ceiling: int):
    """Counts of later mining calls saturate at ``ceiling`` (0 = 2^32 - 1)."""
    _check(lib().amlm_graph_set_ceiling(g.handle, int(ceiling)))


def amlm_graph_inject_device_error(g: Graph):
    """Testing aid: the next build or mining call fails with a sticky
    AMLM_E_DEVICE."""
    _check(lib().amlm_graph_inject_device_error(g.handle))


class Batch(Graph):
    """A batched store: many independent graphs mined in one launch."""

    def __init__(self, graphs, stream=None):
        srcs = [np.ascontiguousarray(g[0], np.uint32) for g in graphs]
        dsts = [np.ascontiguousarray(g[1], np.uint32) for g in graphs]
        tss = [np.ascontiguousarray(g[2], np.int64) for g in graphs]
        nvs = np.array([int(g[3]) for g in graphs], np.uint32)
        sizes = np.array([s.shape[0] for s in srcs], np.uint64)
        self.eoff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
        src = np.concatenate(srcs) if srcs else np.zeros(0, np.uint32)
        dst = np.concatenate(dsts) if dsts else np.zeros(0, np.uint32)
        ts = np.concatenate(tss) if tss else np.zeros(0, np.int64)
        self.handle = ctypes.c_void_p()
        _check(lib().amlm_batch_create(_ptr(src), _ptr(dst), _ptr(ts), _ptr(self.eoff), _ptr(nvs),
                                       len(graphs), 0, _stream_handle(stream), ctypes.byref(self.handle)))
        self.n_graphs = len(graphs)
        self.n_edges = int(self.eoff[-1])
        self.sizes = sizes

    def info_batch(self):
        n, c = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().amlm_batch_info(self.handle, ctypes.byref(n), ctypes.byref(c)))
        return n.value, c.value


def amlm_mine_batch(b: Batch, ps, outs=None, stream=None):
    """Mine a batched store; ps: one amlm_params per graph.  Returns the list
    of per-graph int32 tensors [ncols_i, n_edges_i]."""
    import torch
    if outs is None:
        outs = [torch.empty((amlm_num_columns(p), int(b.sizes[i])), dtype=torch.int32, device="cuda")
                for i, p in enumerate(ps)]
    pa = (amlm_params * len(ps))(*ps)
    ptrs = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
    _check(lib().amlm_mine_batch(b.handle, pa, ptrs, _stream_handle(stream)))
    return outs


def amlm_autotune(g: Graph, ps, outs, cache_path=None, stream=None):
    pa = (amlm_params * len(ps))(*ps)
    ptrs = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
    chosen = (ctypes.c_uint32 * 3)()
    _check(lib().amlm_autotune(g.handle, pa, len(ps), ptrs, cache_path.encode() if cache_path else None,
                               _stream_handle(stream), chosen))
    return list(chosen)


class Server:
    """Continuous-batching server over a resident graph (amlm_server_*), or
    resumed from a snapshot (``Server.resume``)."""

    def __init__(self, resident: Graph, p: amlm_params, hbm_budget: int = 0, max_slots: int = 4):
        self.handle = ctypes.c_void_p()
        self.p = p
        self.ncols = amlm_num_columns(p)
        self.sizes = {}
        if resident is None:
            return
        _check(lib().amlm_server_create(resident.handle, ctypes.byref(p), int(hbm_budget), int(max_slots),
                                        ctypes.byref(self.handle)))

    @classmethod
    def resume(cls, path: str, p: amlm_params, hbm_budget: int = 0, max_slots: int = 4):
        """A server continuing the stream saved by ``snapshot`` (p: the
        parameters it was saved with, for the column count)."""
        S = cls(None, p)
        _check(lib().amlm_server_resume(path.encode(), int(hbm_budget), int(max_slots), ctypes.byref(S.handle)))
        return S

    def snapshot(self, path: str):
        _check(lib().amlm_server_snapshot(self.handle, path.encode()))

    def submit(self, src, dst, ts, wait: bool = False) -> int:
        src = np.ascontiguousarray(src, np.uint32)
        dst = np.ascontiguousarray(dst, np.uint32)
        ts = np.ascontiguousarray(ts, np.int64)
        t = ctypes.c_uint64()
        _check(lib().amlm_server_submit(self.handle, _ptr(src), _ptr(dst), _ptr(ts), src.shape[0],
                                        1 if wait else 0, ctypes.byref(t)))
        self.sizes[t.value] = src.shape[0]
        return t.value

    def wait(self, ticket: int, cap: int = 1 << 22):
        n = self.sizes.pop(ticket)
        counts = np.empty((self.ncols, n), np.uint32)   # every entry is written
        nd = ctypes.c_uint64()
        # only the first n_deltas entries are written (untouched pages of the
        # rest are never committed)
        de = np.empty(cap, np.uint64)
        dc = np.empty(cap, np.uint32)
        dv = np.empty(cap, np.uint32)
        _check(lib().amlm_server_wait(self.handle, ticket, _ptr(counts), ctypes.byref(nd), _ptr(de), _ptr(dc),
                                      _ptr(dv), cap))
        m = min(nd.value, cap)
        return counts, (de[:m], dc[:m], dv[:m]), nd.value

    def stats(self) -> dict:
        """Edges in the current window store, the most it held, group commits
        and batches mined so far."""
        v = [ctypes.c_uint64() for _ in range(4)]
        _check(lib().amlm_server_stats(self.handle, *[ctypes.byref(x) for x in v]))
        return dict(zip(("window_edges", "max_window_edges", "commits", "batches_done"), (x.value for x in v)))

    def times(self, ticket: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().amlm_server_ticket_times(self.handle, ticket, ctypes.byref(a), ctypes.byref(b),
                                              ctypes.byref(c)))
        return a.value, b.value, c.value

    def close(self):
        if self.handle:
            lib().amlm_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def amlm_costmodel_eval(g: Graph, p: amlm_params, stream=None):
    """(predicted log1p bytes, true log1p bytes, sender-window length) of
    every scatter-gather anchor of g, as numpy arrays."""
    cap = max(1, int(g.n_edges))
    pred = np.empty(cap, np.float32)
    lab = np.empty(cap, np.float32)
    wl = np.empty(cap, np.uint32)
    n = ctypes.c_uint64()
    _check(lib().amlm_costmodel_eval(g.handle, ctypes.byref(p), cap, _ptr(pred), _ptr(lab), _ptr(wl),
                                     ctypes.byref(n), _stream_handle(stream)))
    k = min(n.value, cap)
    return pred[:k].copy(), lab[:k].copy(), wl[:k].copy()


def amlm_costmodel_length_coef() -> float:
    c = ctypes.c_float()
    _check(lib().amlm_costmodel_length_coef(ctypes.byref(c)))
    return float(c.value)


def amlm_graph_set_costs(g: Graph, log_cost):
    """Per-edge log1p(bytes) (a float32 device tensor of n_edges, kept
    alive by the caller) for AMLM_SCHED_GIVEN; None clears."""
    _check(lib().amlm_graph_set_costs(g.handle, None if log_cost is None else _ptr(log_cost)))


MLP_PARAMS = 5057
MLP_F = 12


def amlm_costmodel_train(graphs, ps, epochs=0, batch=0, seed=1, out_path=None, stream=None):
    n = len(graphs)
    arr = (ctypes.c_void_p * n)(*[g.handle.value for g in graphs])
    pa = (amlm_params * n)(*ps)
    _check(lib().amlm_costmodel_train(arr, pa, n, epochs, batch, seed,
                                      out_path.encode() if out_path else None, _stream_handle(stream)))


def amlm_costmodel_load(path: str):
    _check(lib().amlm_costmodel_load(path.encode()))


def amlm_costmodel_save(path: str):
    _check(lib().amlm_costmodel_save(path.encode()))


def amlm_costmodel_get():
    w = np.zeros(MLP_PARAMS, np.float32)
    m = np.zeros(MLP_F, np.float32)
    s = np.zeros(MLP_F, np.float32)
    _check(lib().amlm_costmodel_get(_ptr(w), _ptr(m), _ptr(s)))
    return w, m, s


def amlm_mlp_forward(w, x):
    w = np.ascontiguousarray(w, np.float32)
    x = np.ascontiguousarray(x, np.float32)
    y = np.zeros(x.shape[0], np.float32)
    _check(lib().amlm_mlp_forward(_ptr(w), _ptr(x), x.shape[0], _ptr(y)))
    return y


def amlm_mlp_predict(w, x):
    w = np.ascontiguousarray(w, np.float32)
    x = np.ascontiguousarray(x, np.float32)
    y = np.zeros(x.shape[0], np.float32)
    _check(lib().amlm_mlp_predict(_ptr(w), _ptr(x), x.shape[0], _ptr(y)))
    return y


def amlm_mlp_grad(w, x, y):
    w = np.ascontiguousarray(w, np.float32)
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    g = np.zeros(MLP_PARAMS, np.float32)
    loss = ctypes.c_float()
    _check(lib().amlm_mlp_grad(_ptr(w), _ptr(x), _ptr(y), x.shape[0], _ptr(g), ctypes.byref(loss)))
    return g, loss.value


def amlm_copy(dst, src, stream=None):
    _check(lib().amlm_copy(_ptr(dst), _ptr(src), src.numel() * src.element_size(), _stream_handle(stream)))


def to_u32(t) -> np.ndarray:
    """Device int32 tensor holding uint32 bit patterns -> numpy uint32."""
    return t.cpu().numpy().view(np.uint32)
