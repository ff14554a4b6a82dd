"""Alignment plots on MI355X (gfx950): Python binding of libwlcs.so.

The library (C ABI in ``include/wlcs.h``) computes the alignment plot of
Krusche & Tiskin ("Computing alignment plots efficiently"): WLCS(i, j), the LLCS
of every pair of w-windows of x and y, by the windowed seaweed algorithm of
Theorem 3.1 in hand-written HIP kernels.  This module only marshals arguments:
PyTorch provides the device memory and the stream; every step of the computation
runs in the library's kernels.  There is no CPU fallback: if the library is not
built, importing works but every call raises ``WlcsUnavailable``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loaded before libwlcs.so so that both share one HIP runtime

__all__ = ["Context", "Pair", "BatchGraph", "Job", "WlcsError", "WlcsUnavailable", "plot", "plot_dp", "n_windows",
           "library_path", "exported_symbols", "DNA", "PROTEIN", "DOT", "dot_records"]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwlcs.so")

DNA = b"ACGT"
PROTEIN = b"ACDEFGHIKLMNPQRSTVWY"

WLCS_FULL_RANGE = 1
_STATUS = {0: "ok", -1: "invalid argument", -2: "window or length out of range",
           -3: "bad alphabet or letter outside the alphabet", -4: "HIP runtime error",
           -5: "out of memory", -6: "file could not be written"}
WLCS_TUNE_FORCE = 1


class WlcsUnavailable(RuntimeError):
    """libwlcs.so is not built or cannot be loaded."""


class WlcsError(RuntimeError):
    def __init__(self, status: int, where: str, hip_error: int = 0):
        self.status = status
        self.hip_error = hip_error
        msg = f"{where}: {_STATUS.get(status, 'unknown status')} ({status})"
        if hip_error:
            msg += f", hip error {hip_error}"
        super().__init__(msg)


class Job(ctypes.Structure):
    """wlcs_job of include/wlcs.h."""
    _fields_ = [("pair", ctypes.c_void_p), ("w", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("wlcs", ctypes.c_void_p), ("ld", ctypes.c_int64),
                ("bitmap", ctypes.c_void_p), ("ld_words", ctypes.c_int64),
                ("threshold", ctypes.c_int32), ("indel", ctypes.c_void_p),
                ("ld_indel", ctypes.c_int64), ("hx", ctypes.c_int32), ("hy", ctypes.c_int32),
                ("dots", ctypes.c_void_p), ("dot_cap", ctypes.c_int64), ("dot_count", ctypes.c_void_p)]


_lib = None


def library_path() -> str:
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise WlcsUnavailable(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "or python -m paper_0909_2000_amd.build")
    try:
        lib = ctypes.CDLL(LIB_PATH)
    except OSError as e:
        raise WlcsUnavailable(f"cannot load {LIB_PATH}: {e}") from e
    vp, u8p = ctypes.c_void_p, ctypes.c_void_p
    i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.wlcs_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    lib.wlcs_ctx_destroy.argtypes = [vp]
    lib.wlcs_ctx_last_hip_error.argtypes = [vp]
    lib.wlcs_status_str.argtypes = [ctypes.c_int]
    lib.wlcs_status_str.restype = ctypes.c_char_p
    lib.wlcs_ctx_set_tile.argtypes = [vp, i32, i32, i32]
    lib.wlcs_ctx_set_tiles.argtypes = [vp, i32, i32, i32, i32, i32]
    lib.wlcs_measure_valu_peak.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
    lib.wlcs_measure_valu_issue.argtypes = [vp, i32, i32, i32, ctypes.POINTER(ctypes.c_double)]
    plot_args = [vp, u8p, i64, u8p, i64, i32, u8p, i32, vp, i64, vp, i64, i32, vp, i64, u32, vp]
    lib.wlcs_plot.argtypes = plot_args
    lib.wlcs_plot_dp.argtypes = plot_args
    lib.wlcs_plot_blcs.argtypes = plot_args
    lib.wlcs_pair_create.argtypes = [vp, u8p, i64, u8p, i64, u8p, i32, vp, ctypes.POINTER(vp)]
    lib.wlcs_pair_destroy.argtypes = [vp]
    pair_args = [vp, vp, i32, vp, i64, vp, i64, i32, vp, i64, u32, vp]
    lib.wlcs_pair_plot.argtypes = pair_args
    lib.wlcs_pair_plot_dp.argtypes = pair_args
    lib.wlcs_pair_plot_blcs.argtypes = pair_args
    lib.wlcs_score_plot.argtypes = [vp, u8p, i64, u8p, i64, i32, i32, u8p, i32, vp, i64, vp, i64, i32,
                                    u32, vp]
    lib.wlcs_batch.argtypes = [vp, ctypes.POINTER(Job), i32, vp]
    lib.wlcs_batch_noalloc.argtypes = [vp, ctypes.POINTER(Job), i32, vp]
    lib.wlcs_batch_graph.argtypes = [vp, ctypes.POINTER(Job), i32, ctypes.POINTER(vp)]
    lib.wlcs_graph_launch.argtypes = [vp, vp]
    lib.wlcs_graph_destroy.argtypes = [vp]
    lib.wlcs_ctx_set_batch_tile.argtypes = [vp, i32, i32, i32]
    lib.wlcs_ctx_set_batch_grid.argtypes = [vp, i32]
    lib.wlcs_ctx_set_batch_min_units.argtypes = [vp, i64]
    lib.wlcs_ctx_get_batch_tile.argtypes = [vp, i32, ctypes.POINTER(i32)]
    lib.wlcs_ctx_get_batch_grid.argtypes = [vp, ctypes.POINTER(i32)]
    lib.wlcs_tune.argtypes = [vp, ctypes.c_char_p, ctypes.c_uint32]
    lib.wlcs_tune_plot.argtypes = [vp, vp, i32, i32, ctypes.c_uint32, ctypes.c_char_p, ctypes.c_uint32]
    lib.wlcs_ctx_get_plot_tiling.argtypes = [vp, i64, i64, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                             ctypes.POINTER(i32)]
    strided_args = [vp, vp, i32, i32, i32, vp, i64, vp, i64, i32, vp, i64, vp, i64, vp, ctypes.c_uint32, vp]
    lib.wlcs_pair_plot_strided.argtypes = strided_args
    lib.wlcs_pair_dots_filtered.argtypes = [vp, vp, i32, i32, i32, i64, vp, i64, vp, ctypes.c_uint32, vp]
    lib.wlcs_pair_plot_dp_strided.argtypes = strided_args
    for f in ("wlcs_ctx_create", "wlcs_ctx_destroy", "wlcs_ctx_last_hip_error", "wlcs_ctx_set_tile", "wlcs_ctx_set_tiles",
              "wlcs_measure_valu_peak", "wlcs_measure_valu_issue",
              "wlcs_plot", "wlcs_plot_dp", "wlcs_pair_create", "wlcs_pair_destroy", "wlcs_pair_plot",
              "wlcs_pair_plot_dp", "wlcs_batch", "wlcs_batch_noalloc", "wlcs_batch_graph",
              "wlcs_graph_launch", "wlcs_graph_destroy", "wlcs_ctx_set_batch_tile", "wlcs_ctx_set_batch_grid",
              "wlcs_ctx_set_batch_min_units",
              "wlcs_score_plot", "wlcs_ctx_get_batch_tile", "wlcs_ctx_get_batch_grid", "wlcs_tune",
              "wlcs_pair_plot_strided", "wlcs_pair_plot_dp_strided", "wlcs_plot_blcs",
              "wlcs_pair_plot_blcs", "wlcs_pair_dots_filtered", "wlcs_tune_plot", "wlcs_ctx_get_plot_tiling"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def exported_symbols() -> list:
    """Names of the C ABI entry points the binding uses."""
    return ["wlcs_ctx_create", "wlcs_ctx_destroy", "wlcs_ctx_last_hip_error", "wlcs_status_str",
            "wlcs_ctx_set_tile", "wlcs_ctx_set_tiles", "wlcs_measure_valu_peak", "wlcs_measure_valu_issue",
            "wlcs_plot", "wlcs_plot_dp", "wlcs_pair_create", "wlcs_pair_destroy", "wlcs_pair_plot", "wlcs_pair_plot_dp", "wlcs_batch",
            "wlcs_batch_noalloc", "wlcs_batch_graph", "wlcs_graph_launch", "wlcs_graph_destroy", "wlcs_ctx_set_batch_tile", "wlcs_ctx_set_batch_grid",
            "wlcs_score_plot", "wlcs_ctx_get_batch_tile", "wlcs_ctx_get_batch_grid", "wlcs_tune",
            "wlcs_pair_plot_strided", "wlcs_pair_plot_dp_strided", "wlcs_plot_blcs", "wlcs_pair_plot_blcs",
            "wlcs_pair_dots_filtered",
            "wlcs_tune_plot", "wlcs_ctx_get_plot_tiling"]


# the wlcs_dot record
DOT = np.dtype([("i", "<u4"), ("j", "<u4"), ("wlcs", "<u2"), ("indel", "<u2")])


def dot_records(res: dict) -> np.ndarray:
    """The listed dots of a plot_strided result as a numpy record array
    (fields i, j, wlcs, indel; waits for the device), sorted by (i, j), and
    the total count (which may exceed the list's capacity)."""
    torch.cuda.synchronize(res["dot_count"].device)
    count = int(res["dot_count"].item())
    dots = res["dots"]
    k = min(count, int(dots.shape[0])) if dots is not None else 0
    recs = dots[:k].cpu().numpy().view(DOT).reshape(-1) if k else np.zeros(0, dtype=DOT)
    return np.sort(recs, order=("i", "j")), count


def plot_rows(rows: int, cols: int, dtype, device):
    """A rows x cols output (plot or indel distances) whose rows start a
    multiple of 16 bytes apart (a view of a padded allocation): the kernels
    store each strip's block of windows with 16-byte stores, where rows of any
    other length take one store per window.  The padding is never written."""
    per = 16 // torch.empty((), dtype=dtype).element_size()
    ld = max(-(-cols // per) * per, per)
    return torch.empty((rows, ld), dtype=dtype, device=device)[:, :cols]


def n_windows(length: int, w: int, full_range: bool = False) -> int:
    return max(length - w + (1 if full_range else 0), 0)


def _as_bytes(s) -> np.ndarray:
    if isinstance(s, str):
        s = s.encode("ascii")
    if isinstance(s, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(s), dtype=np.uint8)
    if isinstance(s, torch.Tensor):
        s = s.cpu().numpy()
    return np.ascontiguousarray(s, dtype=np.uint8)


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


class Context:
    """One library context on one device (default: the current torch device)."""

    def __init__(self, device: int | None = None):
        lib = _load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        st = lib.wlcs_ctx_create(self.device, ctypes.byref(h))
        if st != 0:
            raise WlcsError(st, "wlcs_ctx_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _load().wlcs_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tile(self, w_lo: int, w_hi: int, tile: int):
        st = _load().wlcs_ctx_set_tile(self._h, w_lo, w_hi, tile)
        if st != 0:
            raise WlcsError(st, "wlcs_ctx_set_tile")

    def measure_valu_peak(self, iters: int = 2000) -> float:
        """wlcs_measure_valu_peak: sustained packed 16-bit VALU element
        operations per second on this device (a measurement helper)."""
        v = ctypes.c_double(0.0)
        st = _load().wlcs_measure_valu_peak(self._h, int(iters), ctypes.byref(v))
        if st != 0:
            raise WlcsError(st, "wlcs_measure_valu_peak", _load().wlcs_ctx_last_hip_error(self._h))
        return v.value

    VALU_KINDS = {"pk16": 0, "b32": 1, "cell": 2, "cell_xor": 3, "cell_two_xor": 4, "bitop3": 5}

    def measure_valu_issue(self, kind: str, waves_per_simd: int, iters: int = 100000) -> float:
        """wlcs_measure_valu_issue: wave64 VALU instructions issued per second
        per SIMD with waves_per_simd (1..4) waves resident on every SIMD, for
        one kind of stream ("pk16", "b32", "cell" or "cell_xor"; a measurement
        helper)."""
        v = ctypes.c_double(0.0)
        st = _load().wlcs_measure_valu_issue(self._h, self.VALU_KINDS[kind], int(waves_per_simd), int(iters),
                                             ctypes.byref(v))
        if st != 0:
            raise WlcsError(st, "wlcs_measure_valu_issue", _load().wlcs_ctx_last_hip_error(self._h))
        return v.value

    def set_tiles(self, w_lo: int, w_hi: int, long_tile: int, short_tile: int, long_pairs: int):
        """wlcs_ctx_set_tiles: long tiles for the first long_pairs tile pairs
        of every strip block, short tiles after them."""
        st = _load().wlcs_ctx_set_tiles(self._h, w_lo, w_hi, long_tile, short_tile, long_pairs)
        if st != 0:
            raise WlcsError(st, "wlcs_ctx_set_tiles")

    def _outputs(self, rows, cols, threshold, indel, out, bitmap_out, indel_out, want_plot):
        dev = torch.device("cuda", self.device)
        if out is None and want_plot:
            out = plot_rows(rows, cols, torch.uint8, dev)
        words = (cols + 63) // 64
        if threshold is not None and bitmap_out is None:
            bitmap_out = torch.empty((rows, words), dtype=torch.int64, device=dev)
        if indel and indel_out is None:
            indel_out = plot_rows(rows, cols, torch.int16, dev)
        for t in (out, bitmap_out, indel_out):
            if t is not None and (t.device != dev or t.dim() != 2 or t.stride(1) != 1):
                raise ValueError("outputs must be 2-D row-major tensors on the context's device")
        return out, bitmap_out, indel_out

    @staticmethod
    def _out_args(out, bitmap_out, indel_out, threshold):
        return (ctypes.c_void_p(out.data_ptr()) if out is not None else None,
                out.stride(0) if out is not None else 0,
                ctypes.c_void_p(bitmap_out.data_ptr()) if bitmap_out is not None else None,
                bitmap_out.stride(0) if bitmap_out is not None else 0,
                int(threshold) if threshold is not None else 0,
                ctypes.c_void_p(indel_out.data_ptr()) if indel_out is not None else None,
                indel_out.stride(0) if indel_out is not None else 0)

    @staticmethod
    def _result(out, bitmap_out, indel_out):
        res = {"wlcs": out}
        if bitmap_out is not None:
            res["bitmap"] = bitmap_out
        if indel_out is not None:
            res["indel"] = indel_out
        return res

    def _stream(self, stream):
        return stream if stream is not None else torch.cuda.current_stream(torch.device("cuda", self.device))

    def _call(self, fn: str, x, y, w: int, alphabet, threshold, indel: bool, full_range: bool,
              out, bitmap_out, indel_out, want_plot: bool, stream):
        lib = _load()
        xa, ya = _as_bytes(x), _as_bytes(y)
        alpha = _as_bytes(alphabet)
        rows, cols = n_windows(xa.size, w, full_range), n_windows(ya.size, w, full_range)
        out, bitmap_out, indel_out = self._outputs(rows, cols, threshold, indel, out, bitmap_out,
                                                   indel_out, want_plot)
        stream = self._stream(stream)
        flags = WLCS_FULL_RANGE if full_range else 0
        st = getattr(lib, fn)(self._h, _ptr(xa), xa.size, _ptr(ya), ya.size, int(w), _ptr(alpha),
                              alpha.size, *self._out_args(out, bitmap_out, indel_out, threshold),
                              flags, ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise WlcsError(st, fn, lib.wlcs_ctx_last_hip_error(self._h))
        return self._result(out, bitmap_out, indel_out)

    def set_batch_tile(self, w_lo: int, w_hi: int, tile: int):
        st = _load().wlcs_ctx_set_batch_tile(self._h, w_lo, w_hi, tile)
        if st != 0:
            raise WlcsError(st, "wlcs_ctx_set_batch_tile")

    def set_batch_grid(self, waves_per_cu: int):
        st = _load().wlcs_ctx_set_batch_grid(self._h, waves_per_cu)
        if st != 0:
            raise WlcsError(st, "wlcs_ctx_set_batch_grid")

    def set_batch_min_units(self, min_units: int):
        """wlcs_ctx_set_batch_min_units: batched jobs with fewer units than
        this get shorter tiles (0: off)."""
        st = _load().wlcs_ctx_set_batch_min_units(self._h, int(min_units))
        if st != 0:
            raise WlcsError(st, "wlcs_ctx_set_batch_min_units")

    def batch_tile(self, w: int) -> int:
        """Tile set for batched plots of window w (0: the built-in choice)."""
        v = ctypes.c_int32(0)
        st = _load().wlcs_ctx_get_batch_tile(self._h, w, ctypes.byref(v))
        if st != 0:
            raise WlcsError(st, "wlcs_ctx_get_batch_tile")
        return v.value

    def batch_grid(self) -> int:
        """Persistent grid of the batched launch (0: the default)."""
        v = ctypes.c_int32(0)
        st = _load().wlcs_ctx_get_batch_grid(self._h, ctypes.byref(v))
        if st != 0:
            raise WlcsError(st, "wlcs_ctx_get_batch_grid")
        return v.value

    def tune(self, cache_path: str | None = None, force: bool = False):
        """wlcs_tune: apply this device's entry of the JSON cache, or time the
        candidates on the device, apply the best and add them to the cache."""
        lib = _load()
        path = os.fsencode(cache_path) if cache_path is not None else None
        st = lib.wlcs_tune(self._h, path, WLCS_TUNE_FORCE if force else 0)
        if st != 0:
            raise WlcsError(st, "wlcs_tune", lib.wlcs_ctx_last_hip_error(self._h))

    def tune_plot(self, pair, w: int, hx: int = 1, full_range: bool = False, cache_path: str | None = None,
                  force: bool = False):
        """wlcs_tune_plot: measure the fastest tiling of this plot shape on the
        device (or apply the one recorded in the cache) for the plots of that
        shape made through this context."""
        lib = _load()
        path = os.fsencode(cache_path) if cache_path is not None else None
        st = lib.wlcs_tune_plot(self._h, pair._h, w, hx, WLCS_FULL_RANGE if full_range else 0, path,
                                WLCS_TUNE_FORCE if force else 0)
        if st != 0:
            raise WlcsError(st, "wlcs_tune_plot", lib.wlcs_ctx_last_hip_error(self._h))

    def plot_tiling(self, rows: int, cols: int, w: int) -> tuple:
        """The measured tiling (long tile, short tile, long pairs) that applies
        to plots of rows x cols windows of length w; (0, 0, 0) if none."""
        vals = [ctypes.c_int32(0) for _ in range(3)]
        st = _load().wlcs_ctx_get_plot_tiling(self._h, rows, cols, w, *[ctypes.byref(v) for v in vals])
        if st != 0:
            raise WlcsError(st, "wlcs_ctx_get_plot_tiling")
        return tuple(v.value for v in vals)

    def _jobs(self, specs):
        """specs: dicts with pair, w and optional threshold, indel, full_range,
        want_plot, out, bitmap_out, indel_out, and for strided or sparse jobs
        hx, hy, bitmap (default: a threshold and hy == 1 and no dot list),
        dot_cap, dots_out, count_out (as Pair.plot_strided).  Returns (Job
        array, results)."""
        arr = (Job * max(len(specs), 1))()
        results = []
        dev = torch.device("cuda", self.device)
        for k, sp in enumerate(specs):
            pair, w = sp["pair"], int(sp["w"])
            hx, hy = int(sp.get("hx", 1)), int(sp.get("hy", 1))
            full = bool(sp.get("full_range", False))
            rows = -(-n_windows(pair.m, w, full) // max(hx, 1))
            cols = -(-n_windows(pair.n, w, full) // max(hy, 1))
            thr = sp.get("threshold")
            listing = sp.get("dot_cap") is not None or sp.get("dots_out") is not None
            bitmap = sp.get("bitmap")
            if bitmap is None:
                bitmap = thr is not None and hy == 1 and not listing
            out, bm, ind = self._outputs(rows, cols, thr if bitmap else None, sp.get("indel", False),
                                         sp.get("out"), sp.get("bitmap_out"), sp.get("indel_out"),
                                         sp.get("want_plot", True))
            o = self._out_args(out, bm, ind, thr)
            dots, count = sp.get("dots_out"), None
            if listing:
                if thr is None:
                    raise ValueError("a dot list needs a threshold")
                if dots is None and sp.get("dot_cap"):
                    dots = torch.empty((int(sp["dot_cap"]), 3), dtype=torch.int32, device=dev)
                count = sp.get("count_out")
                if count is None:
                    count = torch.empty(1, dtype=torch.int64, device=dev)
            arr[k] = Job(pair._h.value, w, WLCS_FULL_RANGE if full else 0, o[0].value if o[0] else None,
                         o[1], o[2].value if o[2] else None, o[3], o[4],
                         o[5].value if o[5] else None, o[6], hx, hy,
                         dots.data_ptr() if dots is not None else None,
                         int(dots.shape[0]) if dots is not None else 0,
                         count.data_ptr() if count is not None else None)
            res = self._result(out, bm, ind)
            if listing:
                res["dots"], res["dot_count"] = dots, count
            results.append(res)
        return arr, results

    def batch(self, specs, stream=None) -> list:
        """All plots of specs in persistent work-stealing launches (wlcs_batch)."""
        lib = _load()
        arr, results = self._jobs(specs)
        stream = self._stream(stream)
        st = lib.wlcs_batch(self._h, arr, len(specs), ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise WlcsError(st, "wlcs_batch", lib.wlcs_ctx_last_hip_error(self._h))
        return results

    def batch_noalloc(self, specs, stream=None) -> list:
        """The same plots through wlcs_batch_noalloc: the library allocates no
        device memory for the call (the outputs here are still torch tensors
        unless the specs bring their own).  Calls that overlap on one device
        race on its fixed scratch."""
        lib = _load()
        arr, results = self._jobs(specs)
        stream = self._stream(stream)
        st = lib.wlcs_batch_noalloc(self._h, arr, len(specs), ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise WlcsError(st, "wlcs_batch_noalloc", lib.wlcs_ctx_last_hip_error(self._h))
        return results

    def batch_graph(self, specs) -> "BatchGraph":
        """The batch captured into a replayable HIP graph (wlcs_batch_graph)."""
        return BatchGraph(self, specs)

    def score_plot(self, x, y, w: int, step: int = 1, alphabet=DNA, threshold: int | None = None,
                   full_range: bool = False, out=None, bitmap_out=None, want_plot: bool = True,
                   stream=None) -> dict:
        """Alignment-score plot (match 1, mismatch 0, gap -1/2) of the x-windows
        0, step, 2*step, ... against every y-window: 'score' (int8 in [-w, w])
        and 'bitmap' (score >= threshold) when asked for."""
        lib = _load()
        xa, ya, alpha = _as_bytes(x), _as_bytes(y), _as_bytes(alphabet)
        rows_all = n_windows(xa.size, w, full_range)
        rows = (rows_all + step - 1) // step if rows_all and step >= 1 else 0
        cols = n_windows(ya.size, w, full_range)
        dev = torch.device("cuda", self.device)
        if out is None and want_plot:
            out = plot_rows(rows, cols, torch.int8, dev)
        if threshold is not None and bitmap_out is None:
            bitmap_out = torch.empty((rows, (cols + 63) // 64), dtype=torch.int64, device=dev)
        for t in (out, bitmap_out):
            if t is not None and (t.device != dev or t.dim() != 2 or t.stride(1) != 1):
                raise ValueError("outputs must be 2-D row-major tensors on the context's device")
        stream = self._stream(stream)
        st = lib.wlcs_score_plot(
            self._h, _ptr(xa), xa.size, _ptr(ya), ya.size, int(w), int(step), _ptr(alpha), alpha.size,
            ctypes.c_void_p(out.data_ptr()) if out is not None else None,
            out.stride(0) if out is not None else 0,
            ctypes.c_void_p(bitmap_out.data_ptr()) if bitmap_out is not None else None,
            bitmap_out.stride(0) if bitmap_out is not None else 0,
            int(threshold) if threshold is not None else 0,
            WLCS_FULL_RANGE if full_range else 0, ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise WlcsError(st, "wlcs_score_plot", lib.wlcs_ctx_last_hip_error(self._h))
        res = {"score": out}
        if bitmap_out is not None:
            res["bitmap"] = bitmap_out
        return res

    def pair(self, x, y, alphabet=DNA, stream=None) -> "Pair":
        """Upload and encode x and y once; plot them any number of times."""
        return Pair(self, x, y, alphabet, stream)

    def plot(self, x, y, w: int, alphabet=DNA, threshold: int | None = None, indel: bool = False,
             full_range: bool = False, out=None, bitmap_out=None, indel_out=None,
             want_plot: bool = True, stream=None) -> dict:
        """Alignment plot by the seaweed kernels.  Returns a dict with 'wlcs'
        (uint8 rows x cols), and 'bitmap' (int64 words holding the uint64 bit
        rows) and 'indel' (int16 holding uint16 2w-2*WLCS) when asked for."""
        return self._call("wlcs_plot", x, y, w, alphabet, threshold, indel, full_range, out,
                          bitmap_out, indel_out, want_plot, stream)

    def plot_dp(self, x, y, w: int, alphabet=DNA, threshold: int | None = None, indel: bool = False,
                full_range: bool = False, out=None, bitmap_out=None, indel_out=None,
                want_plot: bool = True, stream=None) -> dict:
        """The same plot by the plain per-window dynamic program on the GPU."""
        return self._call("wlcs_plot_dp", x, y, w, alphabet, threshold, indel, full_range, out,
                          bitmap_out, indel_out, want_plot, stream)

    def plot_blcs(self, x, y, w: int, alphabet=DNA, threshold: int | None = None, indel: bool = False,
                  full_range: bool = False, out=None, bitmap_out=None, indel_out=None,
                  want_plot: bool = True, stream=None) -> dict:
        """The same plot by bit-parallel LCS per window pair on the GPU."""
        return self._call("wlcs_plot_blcs", x, y, w, alphabet, threshold, indel, full_range, out,
                          bitmap_out, indel_out, want_plot, stream)


class Pair:
    """x and y resident on the device as letter codes (wlcs_pair)."""

    def __init__(self, ctx: Context, x, y, alphabet=DNA, stream=None):
        lib = _load()
        xa, ya, alpha = _as_bytes(x), _as_bytes(y), _as_bytes(alphabet)
        self.ctx, self.m, self.n = ctx, int(xa.size), int(ya.size)
        h = ctypes.c_void_p()
        st = lib.wlcs_pair_create(ctx.handle, _ptr(xa), xa.size, _ptr(ya), ya.size, _ptr(alpha),
                                  alpha.size, ctypes.c_void_p(ctx._stream(stream).cuda_stream),
                                  ctypes.byref(h))
        if st != 0:
            raise WlcsError(st, "wlcs_pair_create", lib.wlcs_ctx_last_hip_error(ctx.handle))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _load().wlcs_pair_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _run(self, fn, w, threshold, indel, full_range, out, bitmap_out, indel_out, want_plot,
             stream):
        lib = _load()
        rows, cols = n_windows(self.m, w, full_range), n_windows(self.n, w, full_range)
        c = self.ctx
        out, bitmap_out, indel_out = c._outputs(rows, cols, threshold, indel, out, bitmap_out,
                                                indel_out, want_plot)
        stream = c._stream(stream)
        st = getattr(lib, fn)(c.handle, self._h, int(w),
                              *c._out_args(out, bitmap_out, indel_out, threshold),
                              WLCS_FULL_RANGE if full_range else 0,
                              ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise WlcsError(st, fn, lib.wlcs_ctx_last_hip_error(c.handle))
        return c._result(out, bitmap_out, indel_out)

    def plot(self, w, threshold=None, indel=False, full_range=False, out=None, bitmap_out=None,
             indel_out=None, want_plot=True, stream=None) -> dict:
        return self._run("wlcs_pair_plot", w, threshold, indel, full_range, out, bitmap_out,
                         indel_out, want_plot, stream)

    def plot_dp(self, w, threshold=None, indel=False, full_range=False, out=None, bitmap_out=None,
                indel_out=None, want_plot=True, stream=None) -> dict:
        return self._run("wlcs_pair_plot_dp", w, threshold, indel, full_range, out, bitmap_out,
                         indel_out, want_plot, stream)

    def plot_blcs(self, w, threshold=None, indel=False, full_range=False, out=None, bitmap_out=None,
                  indel_out=None, want_plot=True, stream=None) -> dict:
        return self._run("wlcs_pair_plot_blcs", w, threshold, indel, full_range, out, bitmap_out,
                         indel_out, want_plot, stream)

    def _run_strided(self, fn, w, hx, hy, threshold, indel, want_plot, bitmap, dot_cap, full_range,
                     out, bitmap_out, indel_out, dots_out, count_out, stream):
        lib = _load()
        c = self.ctx
        rows = -(-n_windows(self.m, w, full_range) // hx) if hx >= 1 else 0
        cols = -(-n_windows(self.n, w, full_range) // hy) if hy >= 1 else 0
        if bitmap is None:
            bitmap = threshold is not None and hy == 1 and dot_cap is None and dots_out is None
        out, bitmap_out, indel_out = c._outputs(rows, cols, threshold if bitmap else None, indel, out,
                                                bitmap_out, indel_out, want_plot)
        dev = torch.device("cuda", c.device)
        count = None
        if dot_cap is not None or dots_out is not None:
            if threshold is None:
                raise ValueError("a dot list needs a threshold")
            if dots_out is None and dot_cap:
                dots_out = torch.empty((int(dot_cap), 3), dtype=torch.int32, device=dev)
            count = count_out if count_out is not None else torch.empty(1, dtype=torch.int64, device=dev)
            if count.device != dev or count.dtype != torch.int64 or count.numel() < 1:
                raise ValueError("count_out must be an int64 tensor on the context's device")
        cap = int(dots_out.shape[0]) if dots_out is not None else 0
        if dots_out is not None and (dots_out.device != dev or dots_out.dtype != torch.int32
                                     or tuple(dots_out.shape[1:]) != (3,) or not dots_out.is_contiguous()):
            raise ValueError("dots_out must be a contiguous (cap, 3) int32 tensor on the context's device")
        stream = c._stream(stream)
        a = c._out_args(out, bitmap_out, indel_out, threshold)
        st = getattr(lib, fn)(c.handle, self._h, int(w), int(hx), int(hy), *a,
                              ctypes.c_void_p(dots_out.data_ptr()) if dots_out is not None else None, cap,
                              ctypes.c_void_p(count.data_ptr()) if count is not None else None,
                              WLCS_FULL_RANGE if full_range else 0, ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise WlcsError(st, fn, lib.wlcs_ctx_last_hip_error(c.handle))
        res = c._result(out, bitmap_out, indel_out)
        if count is not None:
            res["dots"], res["dot_count"] = dots_out, count
        return res

    def plot_strided(self, w, hx=1, hy=1, threshold=None, indel=False, want_plot=True, bitmap=None,
                     dot_cap=None, full_range=False, out=None, bitmap_out=None, indel_out=None,
                     dots_out=None, count_out=None, stream=None) -> dict:
        """wlcs_pair_plot_strided: the plot at x-windows r*hx and y-windows
        c*hy.  With dot_cap (or dots_out) the dots (WLCS >= threshold) are
        listed too: result "dots" holds wlcs_dot records as a (cap, 3) int32
        tensor and "dot_count" their number (one int64); read them with
        dot_records().  bitmap defaults to True when a threshold is given,
        hy == 1 and no dot list is asked for."""
        return self._run_strided("wlcs_pair_plot_strided", w, hx, hy, threshold, indel, want_plot, bitmap,
                                 dot_cap, full_range, out, bitmap_out, indel_out, dots_out, count_out, stream)

    def dots_filtered(self, w, threshold, probe_step=8, probe_cap=0, dot_cap=None, dots_out=None,
                      count_out=None, full_range=False, stream=None) -> dict:
        """The exact dot list (WLCS >= threshold) through the probe filter
        (wlcs_pair_dots_filtered): 'dots' (records as plot_strided lists them)
        and 'dot_count' (device), for wl.dot_records."""
        lib = _load()
        c = self.ctx
        dev = torch.device("cuda", c.device)
        if dots_out is None and dot_cap:
            dots_out = torch.empty((int(dot_cap), 3), dtype=torch.int32, device=dev)
        if count_out is None:
            count_out = torch.empty(1, dtype=torch.int64, device=dev)
        stream = c._stream(stream)
        st = lib.wlcs_pair_dots_filtered(c.handle, self._h, int(w), int(threshold), int(probe_step),
                                         int(probe_cap), dots_out.data_ptr() if dots_out is not None else None,
                                         int(dots_out.shape[0]) if dots_out is not None else 0,
                                         count_out.data_ptr(), WLCS_FULL_RANGE if full_range else 0,
                                         ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise WlcsError(st, "wlcs_pair_dots_filtered", lib.wlcs_ctx_last_hip_error(c.handle))
        return {"dots": dots_out, "dot_count": count_out}

    def plot_dp_strided(self, w, hx=1, hy=1, threshold=None, indel=False, want_plot=True, bitmap=None,
                        dot_cap=None, full_range=False, out=None, bitmap_out=None, indel_out=None,
                        dots_out=None, count_out=None, stream=None) -> dict:
        """The same by the plain per-window dynamic program."""
        return self._run_strided("wlcs_pair_plot_dp_strided", w, hx, hy, threshold, indel, want_plot, bitmap,
                                 dot_cap, full_range, out, bitmap_out, indel_out, dots_out, count_out, stream)


class BatchGraph:
    """A captured batch; launch() replays every plot of it into its outputs."""

    def __init__(self, ctx: Context, specs):
        lib = _load()
        self.ctx = ctx
        self.specs = specs  # keeps the pairs alive
        arr, self.results = ctx._jobs(specs)
        h = ctypes.c_void_p()
        st = lib.wlcs_batch_graph(ctx.handle, arr, len(specs), ctypes.byref(h))
        if st != 0:
            raise WlcsError(st, "wlcs_batch_graph", lib.wlcs_ctx_last_hip_error(ctx.handle))
        self._h = h

    def launch(self, stream=None):
        stream = self.ctx._stream(stream)
        st = _load().wlcs_graph_launch(self._h, ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise WlcsError(st, "wlcs_graph_launch")
        return self.results

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _load().wlcs_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def _ctx(device=None) -> Context:
    d = torch.cuda.current_device() if device is None else int(device)
    if d not in _default_ctx:
        _default_ctx[d] = Context(d)
    return _default_ctx[d]


def plot(x, y, w: int, alphabet=DNA, threshold=None, indel=False, full_range=False, **kw) -> dict:
    return _ctx(kw.pop("device", None)).plot(x, y, w, alphabet, threshold, indel, full_range, **kw)


def plot_dp(x, y, w: int, alphabet=DNA, threshold=None, indel=False, full_range=False, **kw) -> dict:
    return _ctx(kw.pop("device", None)).plot_dp(x, y, w, alphabet, threshold, indel, full_range, **kw)
