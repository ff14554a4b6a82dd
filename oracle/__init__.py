"""Test infrastructure: the CPU oracle for alignment plots.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path and
never imports it.

The oracle is the plain definition of the alignment plot (Krusche & Tiskin,
Section 2): WLCS(i, j) is the LLCS of the w-windows x[i:i+w] and y[j:j+w], for
i < m-w and j < n-w (the paper's 1..m-w and 1..n-w, stored 0-based), each
entry computed by the standard dynamic program in ``wlcs_oracle.c``.  The
epilogues follow the problem statement: a dot-plot bit marks a window pair whose
similarity clears a threshold (Section 1), and the indel distance of two
w-windows is 2w - 2*LLCS (the LCS alignment with gap score 0, Section 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wlcs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-Werror", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u8p, i64p = ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int64)
        lib.oracle_llcs.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64]
        lib.oracle_llcs.restype = ctypes.c_int
        lib.oracle_wlcs.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_int32, u8p, ctypes.c_int64, ctypes.c_int32]
        lib.oracle_wlcs.restype = ctypes.c_int
        lib.oracle_wlcs_strided.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, ctypes.c_int32,
                                            ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, u8p,
                                            ctypes.c_int64, ctypes.c_int32]
        lib.oracle_wlcs_strided.restype = ctypes.c_int
        lib.oracle_wlcs_rows.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_int32, i64p, ctypes.c_int64, u8p,
                                         ctypes.c_int64, ctypes.c_int32]
        lib.oracle_wlcs_rows.restype = ctypes.c_int
        lib.oracle_wlcs_batch.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int32, i64p, ctypes.c_int64, u8p, ctypes.c_int64,
                                          ctypes.c_int32]
        lib.oracle_wlcs_batch.restype = ctypes.c_int
        lib.oracle_wlcs_at.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, ctypes.c_int32,
                                       i64p, i64p, ctypes.c_int64, u8p]
        lib.oracle_wlcs_at.restype = ctypes.c_int
        lib.oracle_score2.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int32)]
        lib.oracle_score2.restype = ctypes.c_int
        lib.oracle_score_plot.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int8), ctypes.c_int64,
                                          ctypes.c_int32]
        lib.oracle_score_plot.restype = ctypes.c_int
        _lib = lib
    return _lib


def _bytes(s) -> np.ndarray:
    if isinstance(s, str):
        s = s.encode("ascii")
    if isinstance(s, (bytes, bytearray)):
        return np.frombuffer(bytes(s), dtype=np.uint8)
    a = np.ascontiguousarray(s, dtype=np.uint8)
    return a


def default_threads() -> int:
    """Host threads for the oracle: every CPU this process may run on (its
    affinity mask), bounded by OMP_NUM_THREADS when that is set (the share of
    the host a job is given)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def _p(a: np.ndarray, t=ctypes.c_uint8):
    return a.ctypes.data_as(ctypes.POINTER(t))


def n_windows(length: int, w: int, full_range: bool = False) -> int:
    """Windows per string: length-w (the paper's range 1..length-w), or
    length-w+1 when every window is wanted."""
    return max(length - w + (1 if full_range else 0), 0)


def llcs(a, b) -> int:
    """LLCS of two byte strings by the standard dynamic program (<= 4096 each)."""
    a, b = _bytes(a), _bytes(b)
    r = _load().oracle_llcs(_p(a), a.size, _p(b), b.size)
    if r < 0:
        raise ValueError(f"oracle_llcs failed ({r})")
    return r


def wlcs(x, y, w: int, full_range: bool = False, nthreads: int | None = None) -> np.ndarray:
    """The whole alignment plot as a (rows, cols) uint8 matrix."""
    x, y = _bytes(x), _bytes(y)
    rows, cols = n_windows(x.size, w, full_range), n_windows(y.size, w, full_range)
    out = np.zeros((rows, cols), dtype=np.uint8)
    if rows and cols:
        nt = nthreads or default_threads()
        r = _load().oracle_wlcs(_p(x), x.size, _p(y), y.size, w, int(full_range), _p(out),
                                cols, nt)
        if r != 0:
            raise ValueError(f"oracle_wlcs failed ({r})")
    return out


def wlcs_strided(x, y, w: int, hx: int = 1, hy: int = 1, full_range: bool = False,
                 nthreads: int | None = None) -> np.ndarray:
    """The plot with step sizes (Section 3): entry (r, c) is WLCS of the
    x-window starting at r*hx and the y-window starting at c*hy."""
    x, y = _bytes(x), _bytes(y)
    if hx < 1 or hy < 1:
        raise ValueError("steps must be >= 1")
    rows, cols = n_windows(x.size, w, full_range), n_windows(y.size, w, full_range)
    orows, ocols = -(-rows // hx), -(-cols // hy)
    out = np.zeros((orows, ocols), dtype=np.uint8)
    if orows and ocols:
        nt = nthreads or default_threads()
        r = _load().oracle_wlcs_strided(_p(x), x.size, _p(y), y.size, w, hx, hy, int(full_range),
                                        _p(out), ocols, nt)
        if r != 0:
            raise ValueError(f"oracle_wlcs_strided failed ({r})")
    return out


DOT = np.dtype([("i", "<u4"), ("j", "<u4"), ("wlcs", "<u2"), ("indel", "<u2")])


def dot_list(plot: np.ndarray, w: int, threshold: int, hx: int = 1, hy: int = 1) -> np.ndarray:
    """The sparse dot plot (Section 1: a dot for each window pair whose
    similarity clears a threshold): one record per entry with WLCS >= threshold,
    holding the window starts i = r*hx, j = c*hy, the WLCS and the indel
    distance 2w - 2*WLCS, in row-major order of (i, j)."""
    r, c = np.nonzero(plot >= threshold)
    out = np.zeros(r.size, dtype=DOT)
    out["i"], out["j"] = r * hx, c * hy
    out["wlcs"] = plot[r, c]
    out["indel"] = 2 * w - 2 * plot[r, c].astype(np.int32)
    return out


def wlcs_rows(x, y, w: int, rows, full_range: bool = False,
              nthreads: int | None = None) -> np.ndarray:
    """Selected rows (x-windows) of the plot, each against every y-window."""
    x, y = _bytes(x), _bytes(y)
    ids = np.ascontiguousarray(rows, dtype=np.int64)
    cols = n_windows(y.size, w, full_range)
    out = np.zeros((ids.size, cols), dtype=np.uint8)
    if ids.size and cols:
        nt = nthreads or default_threads()
        r = _load().oracle_wlcs_rows(_p(x), x.size, _p(y), y.size, w, int(full_range),
                                     _p(ids, ctypes.c_int64), ids.size, _p(out), cols, nt)
        if r != 0:
            raise ValueError(f"oracle_wlcs_rows failed ({r})")
    return out


def wlcs_batch(x, y, w: int, rows=None, full_range: bool = False,
               nthreads: int | None = None) -> np.ndarray:
    """The plot (or the selected rows, as wlcs_rows) by O-batch: the same
    dynamic program per window pair, evaluated for 64 neighbouring y-windows
    side by side (loops interchanged over independent windows; see
    wlcs_oracle.c).  Equal to wlcs() entry by entry."""
    x, y = _bytes(x), _bytes(y)
    cols = n_windows(y.size, w, full_range)
    if rows is None:
        ids, nrows = None, n_windows(x.size, w, full_range)
    else:
        ids = np.ascontiguousarray(rows, dtype=np.int64)
        nrows = ids.size
    out = np.zeros((nrows, cols), dtype=np.uint8)
    if nrows and cols:
        nt = nthreads or default_threads()
        r = _load().oracle_wlcs_batch(_p(x), x.size, _p(y), y.size, w, int(full_range),
                                      _p(ids, ctypes.c_int64) if ids is not None else None, nrows,
                                      _p(out), cols, nt)
        if r != 0:
            raise ValueError(f"oracle_wlcs_batch failed ({r})")
    return out


def wlcs_at(x, y, w: int, ii, jj) -> np.ndarray:
    """Individual plot entries at window starts (ii[k], jj[k])."""
    x, y = _bytes(x), _bytes(y)
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    if ii.shape != jj.shape:
        raise ValueError("ii and jj differ in shape")
    out = np.zeros(ii.size, dtype=np.uint8)
    if ii.size:
        r = _load().oracle_wlcs_at(_p(x), x.size, _p(y), y.size, w, _p(ii, ctypes.c_int64),
                                   _p(jj, ctypes.c_int64), ii.size, _p(out))
        if r != 0:
            raise ValueError(f"oracle_wlcs_at failed ({r})")
    return out


def dot_bitmap(plot: np.ndarray, threshold: int) -> np.ndarray:
    """Thresholded dot plot: bit j of row i is set iff WLCS(i, j) >= threshold.

    Packed as little-endian uint64 words, bit b of word q <-> column 64q+b,
    ceil(cols/64) words per row, padding bits zero."""
    rows, cols = plot.shape
    words = (cols + 63) // 64
    bits = np.zeros((rows, words * 64), dtype=np.uint8)
    bits[:, :cols] = plot >= threshold
    packed = np.packbits(bits, axis=1, bitorder="little")
    return packed.view("<u8").reshape(rows, words)


def indel(plot: np.ndarray, w: int) -> np.ndarray:
    """Indel (insert/delete) distance of the window pairs: 2w - 2*WLCS."""
    return (2 * w - 2 * plot.astype(np.int32)).astype(np.uint16)


def score(a, b) -> float:
    """Alignment score of a and b: match 1, mismatch 0, gap -1/2 (Section 2),
    by its own dynamic program."""
    a, b = _bytes(a), _bytes(b)
    v = ctypes.c_int32()
    r = _load().oracle_score2(_p(a), a.size, _p(b), b.size, ctypes.byref(v))
    if r != 0:
        raise ValueError(f"oracle_score2 failed ({r})")
    return v.value / 2.0


def score_plot(x, y, w: int, step: int = 1, full_range: bool = False,
               nthreads: int | None = None) -> np.ndarray:
    """Alignment-score plot: int8 scores of the x-windows 0, step, 2*step, ...
    against every y-window (w <= 127)."""
    x, y = _bytes(x), _bytes(y)
    rows_all = n_windows(x.size, w, full_range)
    rows = (rows_all + step - 1) // step if rows_all else 0
    cols = n_windows(y.size, w, full_range)
    out = np.zeros((rows, cols), dtype=np.int8)
    if rows and cols:
        nt = nthreads or default_threads()
        r = _load().oracle_score_plot(_p(x), x.size, _p(y), y.size, w, step, int(full_range),
                                      _p(out, ctypes.c_int8), cols, nt)
        if r != 0:
            raise ValueError(f"oracle_score_plot failed ({r})")
    return out
