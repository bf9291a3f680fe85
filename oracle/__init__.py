"""CPU oracle for the per-edge pattern counts (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It wraps ``liboracle.so`` (plain single-threaded C, built from
``oracle.c`` by ``build_oracle``) and shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

FAN_OUT, FAN_IN, SG, GS, CYC = 1, 2, 4, 8, 16
ALL = FAN_OUT | FAN_IN | SG | GS | CYC
SG_UNORDERED = 32  # modifier of SG: the two legs of an intermediate in either order
DEG_OUT, DEG_IN = 64, 128   # distinct counterparties in the FAN windows (columns after the cycles)
SG_PHASE = 256     # modifier of SG: every scatter leg before every gather leg
CYC_ANY_ORDER = 512  # modifier of CYC: the cycle's edges in any order within delta
PART = 1024        # participation columns: the SG / GS instances each edge belongs to
SG_SIZES = 2048    # SG_k instances binned by size: exactly k, k+1, k+2, at least k+3 intermediates


def build_oracle() -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, no parallelism)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", LIB + ".tmp", os.path.join(HERE, "oracle.c")]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        lib = ctypes.CDLL(LIB)
        u64, u32, i64, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_void_p
        lib.oracle_num_columns.argtypes = [u32, u32]
        lib.oracle_num_columns.restype = u32
        lib.oracle_mine.argtypes = [u64, u32, p, p, p, u32, i64, u32, u32, p]
        lib.oracle_mine.restype = ctypes.c_int
        lib.oracle_mine_range.argtypes = [u64, u32, p, p, p, u32, i64, u32, u32, u64, u64, p, p]
        lib.oracle_mine_range.restype = ctypes.c_int
        lib.oracle_mine_ex.argtypes = [u64, u32, p, p, p, u32, i64, u32, u32, u64, u64, u32, p, p, p]
        lib.oracle_mine_ex.restype = ctypes.c_int
        lib.oracle_mine_selected.argtypes = [u64, u32, p, p, p, u32, i64, u32, u32, p, u64, p]
        lib.oracle_mine_selected.restype = ctypes.c_int
        lib.oracle_count_cycles_first.argtypes = [u64, u32, p, p, p, i64, u32, p]
        lib.oracle_count_cycles_first.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_columns(patterns: int, L: int) -> int:
    return int(_load().oracle_num_columns(patterns, L))


def _arrays(src, dst, ts):
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    ts = np.ascontiguousarray(ts, dtype=np.int64)
    return src, dst, ts


def _check(rc):
    if rc != 0:
        raise ValueError({1: "vertex id out of range", 2: "out of memory",
                          3: "invalid parameters"}.get(rc, f"oracle error {rc}"))


def mine(src, dst, ts, n_vertices: int, patterns: int = ALL, delta: int = 86400,
         L: int = 4, k: int = 2) -> np.ndarray:
    """Every column for every edge; returns uint32 [ncols, n_edges]."""
    lib = _load()
    src, dst, ts = _arrays(src, dst, ts)
    n = src.shape[0]
    out = np.zeros((num_columns(patterns, L), n), dtype=np.uint32)
    _check(lib.oracle_mine(n, n_vertices, src.ctypes.data, dst.ctypes.data, ts.ctypes.data,
                           patterns, delta, L, k, out.ctypes.data))
    return out


def mine_range(src, dst, ts, n_vertices: int, a_lo: int, a_hi: int, patterns: int = ALL,
               delta: int = 86400, L: int = 4, k: int = 2):
    """Anchors restricted to edge ids [a_lo, a_hi); returns (counts, seconds
    spent in the anchor loops)."""
    lib = _load()
    src, dst, ts = _arrays(src, dst, ts)
    n = src.shape[0]
    out = np.zeros((num_columns(patterns, L), n), dtype=np.uint32)
    sec = ctypes.c_double()
    _check(lib.oracle_mine_range(n, n_vertices, src.ctypes.data, dst.ctypes.data, ts.ctypes.data,
                                 patterns, delta, L, k, a_lo, a_hi, out.ctypes.data, ctypes.byref(sec)))
    return out, sec.value


def mine_ex(src, dst, ts, n_vertices: int, patterns: int = ALL, delta: int = 86400, L: int = 4,
            k: int = 2, a_lo: int = 0, a_hi: int | None = None, ceiling: int = 0, work: bool = False):
    """Anchors restricted to edge ids [a_lo, a_hi) (default: all), counts
    saturating at ``ceiling`` (0 = 2^32 - 1).  Returns (counts uint32
    [ncols, n], work uint64 [3, n] or None, seconds): work rows are the
    algorithmic bytes B_io, B_sg/gs, B_cyc of each anchor."""
    lib = _load()
    src, dst, ts = _arrays(src, dst, ts)
    n = src.shape[0]
    if a_hi is None:
        a_hi = n
    out = np.zeros((num_columns(patterns, L), n), dtype=np.uint32)
    wk = np.zeros((3, n), dtype=np.uint64) if work else None
    sec = ctypes.c_double()
    _check(lib.oracle_mine_ex(n, n_vertices, src.ctypes.data, dst.ctypes.data, ts.ctypes.data, patterns,
                              delta, L, k, a_lo, a_hi, ceiling, out.ctypes.data,
                              wk.ctypes.data if work else None, ctypes.byref(sec)))
    return out, wk, sec.value


def mine_selected(src, dst, ts, n_vertices: int, sel, patterns: int = ALL, delta: int = 86400,
                  L: int = 4, k: int = 2) -> np.ndarray:
    """Every column for the edges in ``sel`` only (cycle columns from an
    independent through-edge enumeration); returns uint32 [ncols, len(sel)]."""
    lib = _load()
    src, dst, ts = _arrays(src, dst, ts)
    sel = np.ascontiguousarray(sel, dtype=np.uint64)
    out = np.zeros((num_columns(patterns, L), sel.shape[0]), dtype=np.uint32)
    _check(lib.oracle_mine_selected(src.shape[0], n_vertices, src.ctypes.data, dst.ctypes.data,
                                    ts.ctypes.data, patterns, delta, L, k, sel.ctypes.data,
                                    sel.shape[0], out.ctypes.data))
    return out


def count_cycles_first(src, dst, ts, n_vertices: int, delta: int, L: int) -> np.ndarray:
    """Number of distinct l-cycles (each counted once, from its first edge);
    returns uint64 [L+1] indexed by l."""
    lib = _load()
    src, dst, ts = _arrays(src, dst, ts)
    cnt = np.zeros(L + 1, dtype=np.uint64)
    _check(lib.oracle_count_cycles_first(src.shape[0], n_vertices, src.ctypes.data, dst.ctypes.data,
                                         ts.ctypes.data, delta, L, cnt.ctypes.data))
    return cnt
