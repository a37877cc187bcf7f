"""Exact closest pair, fixed-radius neighbours and time-series motifs on MI355X.

Thin ctypes binding of the cpmi C ABI (include/cpmi.h). Every step of the
search runs in the HIP library libcpmi.so built from csrc/; this module only
marshals arguments: it takes torch tensors that already live on the GPU and
passes their device pointers, shapes and the current HIP stream. There is no
CPU fallback: importing the package fails if the library is missing.

    from paper_1407_5609_amd import closest_pair, frnn, points, motif, motif_batch
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

__all__ = ["CpmiError", "Pair", "Stats", "Context", "closest_pair", "frnn", "points", "motif", "motif_batch",
           "PREC_AUTO", "PREC_F32", "PREC_BF16", "PREC_I8", "library_path", "default_context"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcpmi.so")

OK, ERR_ARG, ERR_NOPAIR, ERR_NONFINITE, ERR_DEGENERATE, ERR_CAPACITY, ERR_HIP, ERR_RANGE = 0, -1, -2, -3, -4, -5, -6, -7
F32, I8 = 0, 1
PREC_AUTO, PREC_F32, PREC_BF16, PREC_I8 = 0, 1, 2, 3
_PREC = {"auto": PREC_AUTO, "f32": PREC_F32, "fp32": PREC_F32, "bf16": PREC_BF16, "i8": PREC_I8, "int8": PREC_I8}
_ERRNAME = {ERR_ARG: "ERR_ARG", ERR_NOPAIR: "ERR_NOPAIR", ERR_NONFINITE: "ERR_NONFINITE",
            ERR_DEGENERATE: "ERR_DEGENERATE", ERR_CAPACITY: "ERR_CAPACITY", ERR_HIP: "ERR_HIP", ERR_RANGE: "ERR_RANGE"}


class _CPair(C.Structure):
    _fields_ = [("i", C.c_int64), ("j", C.c_int64), ("d2", C.c_double), ("d", C.c_double),
                ("screen_err", C.c_double), ("screen_bound", C.c_double), ("status", C.c_int32),
                ("reserved", C.c_int32)]


class _CMatchPair(C.Structure):
    _fields_ = [("i", C.c_int64), ("j", C.c_int64), ("matches", C.c_int64), ("length", C.c_int64),
                ("status", C.c_int32), ("reserved", C.c_int32)]


class _CStats(C.Structure):
    _fields_ = [("valid_pairs", C.c_int64), ("tiles_total", C.c_int64), ("tiles_rescreened", C.c_int64),
                ("cpp_candidates", C.c_int64), ("frnn_candidates", C.c_int64), ("frnn_pairs", C.c_int64),
                ("reruns", C.c_int64), ("max_err_over_bound", C.c_double), ("kernel_ms", C.c_double),
                ("screen_ms", C.c_double), ("screen_pairs", C.c_int64), ("precision", C.c_int32),
                ("tile", C.c_int32), ("tiles_pruned", C.c_int64)]


class _CTune(C.Structure):
    _fields_ = [("precision", C.c_int32), ("tile", C.c_int32), ("ms", (C.c_double * 2) * 4), ("band", C.c_int32),
                ("reserved", C.c_int32), ("band_ms", (C.c_double * 3) * 4)]


# Tuned choices measured on MI355X (written by `python -m paper_1407_5609_amd.autotune`);
# a Context reads it unless another cache is named.
DEFAULT_TUNE_CACHE = os.path.join(_HERE, "tune_gfx950.json")


def library_path() -> str:
    return _LIB_PATH


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
                          " (hipcc, gfx950); there is no CPU fallback")
    # torch's HIP runtime must be the process's runtime (the library resolves
    # libamdhip64.so.7 to whichever copy is loaded first), and torch must be the
    # first to initialise the device (see Context)
    import torch  # noqa: F401
    L = C.CDLL(_LIB_PATH)
    vp, i64, dbl, i32 = C.c_void_p, C.c_int64, C.c_double, C.c_int
    L.cpmi_create.argtypes = [C.POINTER(vp), i32, C.c_char_p]
    L.cpmi_destroy.argtypes = [vp]
    L.cpmi_last_error.argtypes = [vp]
    L.cpmi_last_error.restype = C.c_char_p
    L.cpmi_last_stats.argtypes = [vp, C.POINTER(_CStats)]
    L.cpmi_set_tile.argtypes = [vp, i32, i32]
    L.cpmi_set_pruning.argtypes = [vp, i32, dbl, C.c_uint64]
    L.cpmi_version.restype = i32
    L.cpmi_closest_pair.argtypes = [vp, vp, i32, i64, i64, i64, i32, vp, C.POINTER(_CPair)]
    L.cpmi_closest_pair_noalloc.argtypes = [vp, vp, i32, i64, i64, i64, i32, vp, C.POINTER(_CPair)]
    L.cpmi_frnn.argtypes = [vp, vp, i32, i64, i64, i64, dbl, i32, vp, vp, vp, i64, C.POINTER(i64)]
    L.cpmi_tune_lookup_band.argtypes = [vp, i32, i64, dbl, C.POINTER(C.c_int32)]
    L.cpmi_dbg_screen_sample.argtypes = [vp, vp, i32, i64, i64, i64, i32, i32, i32, vp, i64, vp, vp, vp,
                                         C.POINTER(dbl), vp]
    L.cpmi_points.argtypes = [vp, vp, i32, i64, i64, i64, i32, dbl, vp, C.POINTER(_CPair), vp, vp, i64,
                              C.POINTER(i64)]
    L.cpmi_motif.argtypes = [vp, vp, i64, i64, i64, i32, dbl, vp, C.POINTER(_CPair), vp, vp, i64, C.POINTER(i64)]
    L.cpmi_motif_batch.argtypes = [vp, C.POINTER(vp), C.POINTER(i64), C.POINTER(i64), i64, i32, vp,
                                   C.POINTER(_CPair)]
    L.cpmi_strings_pair.argtypes = [vp, vp, i64, i64, i64, i32, i32, vp, C.POINTER(_CMatchPair)]
    L.cpmi_two_locus.argtypes = [vp, vp, i64, i64, i64, i64, i32, vp, C.POINTER(_CMatchPair)]
    L.cpmi_strings_lightbulb.argtypes = [vp, vp, i64, i64, i64, i32, i32, i32, i32, C.c_uint64, i64, vp,
                                         C.POINTER(_CMatchPair), C.POINTER(i64)]
    L.cpmi_autotune.argtypes = [vp, vp, i32, i64, i64, i64, i32, vp, i32, C.POINTER(_CTune)]
    L.cpmi_save_tune_cache.argtypes = [vp, C.c_char_p]
    L.cpmi_tune_lookup.argtypes = [vp, i32, i32, i64, dbl, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.cpmi_dbg_mfma_probe.argtypes = [i32, vp, vp, vp, vp]
    L.cpmi_dbg_copy.argtypes = [vp, vp, i64, vp]
    L.cpmi_dbg_mfma_peak.restype = dbl
    L.cpmi_dbg_mfma_peak.argtypes = [i32, i32, i32, C.POINTER(dbl)]
    L.cpmi_dbg_znorm.argtypes = [vp, vp, i64, i64, i32, vp, vp, vp]
    L.cpmi_pairs_to_csr.argtypes = [vp, vp, i64, i64, vp, vp, vp]
    L.cpmi_dbg_pruned_tiles_gpu.restype = i64
    L.cpmi_dbg_pruned_tiles_gpu.argtypes = [vp, i64, i32, i32, vp, vp, dbl, i64, i32, vp, i64, C.POINTER(i64),
                                            C.POINTER(i64), vp]
    L.cpmi_dbg_set_prune_order.argtypes = [vp, i32, dbl]
    return L


_lib = _load()


class CpmiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAME.get(code, code)}: {msg}")
        self.code = code


@dataclass
class Pair:
    i: int
    j: int
    d2: float
    d: float
    screen_err: float
    screen_bound: float


@dataclass
class MatchPair:
    """A string pair (cpmi_strings_pair) or SNP pair (cpmi_two_locus): i < j,
    `matches` positions (bits of the D columns) in agreement out of `length`."""
    i: int
    j: int
    matches: int
    length: int


@dataclass
class Stats:
    valid_pairs: int
    tiles_total: int
    tiles_rescreened: int
    cpp_candidates: int
    frnn_candidates: int
    frnn_pairs: int
    reruns: int
    max_err_over_bound: float
    kernel_ms: float
    screen_ms: float
    screen_pairs: int
    precision: int
    tile: int
    tiles_pruned: int


def _prec(p) -> int:
    if isinstance(p, str):
        return _PREC[p.lower()]
    return int(p)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _pair(cp: _CPair) -> Pair:
    return Pair(cp.i, cp.j, cp.d2, cp.d, cp.screen_err, cp.screen_bound)


class Context:
    """One cpmi context (device workspace, tuned tiles). Not thread-safe."""

    def __init__(self, device: int | None = None, tune_cache: str | None = DEFAULT_TUNE_CACHE):
        """tune_cache: JSON file of tuned choices (default: the packaged
        MI355X cache if present); None uses the built-in rule only."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("cpmi needs a ROCm GPU; none is visible")
        self.device = torch.cuda.current_device() if device is None else int(device)
        # the library shares torch's HIP runtime; let torch initialise the device first
        torch.cuda.set_device(self.device)
        h = C.c_void_p()
        path = tune_cache.encode() if tune_cache and os.path.exists(tune_cache) else None
        rc = _lib.cpmi_create(C.byref(h), self.device, path)
        if rc != OK:
            raise CpmiError(rc, f"cpmi_create failed on device {self.device} "
                                f"(torch sees {torch.cuda.device_count()} devices)")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.cpmi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- helpers
    def _check(self, rc: int):
        if rc != OK:
            raise CpmiError(rc, _lib.cpmi_last_error(self._h).decode(errors="replace"))

    def last_error(self) -> str:
        return _lib.cpmi_last_error(self._h).decode(errors="replace")

    def stats(self) -> Stats:
        s = _CStats()
        self._check(_lib.cpmi_last_stats(self._h, C.byref(s)))
        return Stats(*(getattr(s, f) for f, _ in _CStats._fields_))

    def set_tile(self, precision, tile: int):
        self._check(_lib.cpmi_set_tile(self._h, _prec(precision), int(tile)))

    def set_pruning(self, q: int, f: float = 10.0, seed: int = 0):
        """Reference-point tile pruning for point sets and single-series
        motifs (cpmi_set_pruning): q references projected by f; q = 0 turns it
        off. Answers are unchanged."""
        self._check(_lib.cpmi_set_pruning(self._h, int(q), float(f), int(seed)))

    def autotune(self, pts, precision="auto", reps: int = 3, stream=None) -> dict:
        """Time the screen configurations on `pts` and record the fastest in
        this context (cpmi_autotune). Returns the choice and the timings."""
        dt, n, d, ld = self._points_args(pts)
        out = _CTune()
        self._check(_lib.cpmi_autotune(self._h, C.c_void_p(pts.data_ptr()), dt, n, d, ld, _prec(precision),
                                       _stream_ptr(stream), int(reps), C.byref(out)))
        names = {PREC_F32: "f32", PREC_BF16: "bf16", PREC_I8: "i8"}
        ms = {f"{names[p]}/{t}": out.ms[p][k] for p in names for k, t in enumerate((128, 256)) if out.ms[p][k] > 0}
        band_ms = {f"{names[p]}/band{b}": out.band_ms[p][k] for p in names for k, b in enumerate((4, 8, 16))
                   if out.band_ms[p][k] > 0}
        return {"precision": names[out.precision], "tile": out.tile, "band": out.band, "ms": ms, "band_ms": band_ms}

    def tune_lookup_band(self, precision, d: int, pairs: float) -> int:
        """Band height of the tile order a problem would use (cpmi_tune_lookup_band)."""
        b = C.c_int32(0)
        self._check(_lib.cpmi_tune_lookup_band(self._h, _prec(precision), int(d), float(pairs), C.byref(b)))
        return int(b.value)

    def save_tune_cache(self, path: str):
        self._check(_lib.cpmi_save_tune_cache(self._h, path.encode()))

    def tune_lookup(self, dtype: str, precision, d: int, pairs: float):
        """(precision code, tile) a call of this shape would use."""
        p, t = C.c_int32(), C.c_int32()
        self._check(_lib.cpmi_tune_lookup(self._h, I8 if dtype in ("i8", "int8") else F32, _prec(precision),
                                          int(d), float(pairs), C.byref(p), C.byref(t)))
        return int(p.value), int(t.value)

    @staticmethod
    def _points_args(pts):
        import torch
        if pts.device.type != "cuda":
            raise ValueError("points must be a GPU tensor")
        if pts.dim() != 2 or pts.stride(1) != 1:
            raise ValueError("points must be a 2-D tensor with unit column stride")
        if pts.dtype == torch.float32:
            dt = F32
        elif pts.dtype == torch.int8:
            dt = I8
        else:
            raise TypeError("points must be float32 or int8")
        return dt, pts.shape[0], pts.shape[1], max(pts.stride(0), pts.shape[1])

    def _radius_call(self, fn, cap, out=None):
        """Two-call capacity protocol: try with `cap`, retry with the count.
        With `out` = (pairs, d2), caller-owned int64 (m, 2) and float64 (m,)
        device tensors, the pairs go there (capacity m, no allocation and no
        retry: a larger count raises the capacity error)."""
        import torch
        if out is not None:
            pairs, d2 = out
            if pairs.dtype != torch.int64 or d2.dtype != torch.float64 or pairs.dim() != 2 or \
                    pairs.shape[1] != 2 or d2.dim() != 1 or not pairs.is_contiguous() or not d2.is_contiguous() \
                    or pairs.device.type != "cuda" or d2.device.type != "cuda":
                raise ValueError("out must be a contiguous int64 (m, 2) and float64 (m,) pair of GPU tensors")
            cap = min(pairs.shape[0], d2.shape[0])
            cnt = C.c_int64(0)
            rc = fn(pairs, d2, cap, cnt)
            return rc, pairs[:min(cnt.value, cap)], d2[:min(cnt.value, cap)]
        cap = max(int(cap), 1)
        while True:
            pairs = torch.empty((cap, 2), dtype=torch.int64, device=f"cuda:{self.device}")
            d2 = torch.empty(cap, dtype=torch.float64, device=f"cuda:{self.device}")
            cnt = C.c_int64(0)
            rc = fn(pairs, d2, cap, cnt)
            if rc == ERR_CAPACITY and cnt.value > cap:
                cap = int(cnt.value)
                continue
            return rc, pairs[:cnt.value], d2[:cnt.value]

    # ---- the calls of cpmi.h
    @staticmethod
    def _int8_matrix(x, what):
        import torch
        if x.device.type != "cuda" or x.dtype != torch.int8 or x.dim() != 2 or x.stride(1) != 1:
            raise ValueError(f"{what} must be a 2-D int8 GPU tensor with unit column stride")
        return x.shape[0], x.shape[1], max(x.stride(0), x.shape[1])

    def strings_pair(self, strings, sigma: int, mode: str = "most", stream=None) -> MatchPair:
        """Most or least correlated pair of the rows of `strings` (int8 symbols
        in 0..sigma-1; cpmi_strings_pair)."""
        n, k, ld = self._int8_matrix(strings, "strings")
        m = {"most": 0, "least": 1}[mode]
        out = _CMatchPair()
        self._check(_lib.cpmi_strings_pair(self._h, C.c_void_p(strings.data_ptr()), n, k, ld, int(sigma), m,
                                           _stream_ptr(stream), C.byref(out)))
        return MatchPair(out.i, out.j, out.matches, out.length)

    def strings_lightbulb(self, strings, sigma: int, mode: str = "most", iterations: int = 16, columns: int = 8,
                          seed: int = 0, cap: int = 1 << 22, stream=None):
        """Randomised light-bulb bucketing (cpmi_strings_lightbulb): returns
        (MatchPair, pairs collected)."""
        n, k, ld = self._int8_matrix(strings, "strings")
        m = {"most": 0, "least": 1}[mode]
        out, pairs = _CMatchPair(), C.c_int64(0)
        self._check(_lib.cpmi_strings_lightbulb(self._h, C.c_void_p(strings.data_ptr()), n, k, ld, int(sigma), m,
                                                int(iterations), int(columns), int(seed), int(cap),
                                                _stream_ptr(stream), C.byref(out), C.byref(pairs)))
        return MatchPair(out.i, out.j, out.matches, out.length), int(pairs.value)

    def two_locus(self, genotypes, m1: int, m2: int, direction: int = 0, stream=None) -> MatchPair:
        """Two-locus association pair of the SNP columns of `genotypes`
        ((m1 + m2) x n int8 in {0, 1, 2}, cases first; cpmi_two_locus)."""
        rows, n, ld = self._int8_matrix(genotypes, "genotypes")
        if rows != m1 + m2:
            raise ValueError("genotypes must have m1 + m2 rows")
        out = _CMatchPair()
        self._check(_lib.cpmi_two_locus(self._h, C.c_void_p(genotypes.data_ptr()), int(m1), int(m2), n, ld,
                                        int(direction), _stream_ptr(stream), C.byref(out)))
        return MatchPair(out.i, out.j, out.matches, out.length)

    def closest_pair(self, pts, precision="auto", stream=None) -> Pair:
        dt, n, d, ld = self._points_args(pts)
        out = _CPair()
        self._check(_lib.cpmi_closest_pair(self._h, C.c_void_p(pts.data_ptr()), dt, n, d, ld, _prec(precision),
                                           _stream_ptr(stream), C.byref(out)))
        return _pair(out)

    def closest_pair_noalloc(self, pts, precision="auto", stream=None) -> Pair:
        """cpmi_closest_pair_noalloc: the closest pair with every device buffer
        taken from the library's static scratch (no allocation)."""
        dt, n, d, ld = self._points_args(pts)
        out = _CPair()
        self._check(_lib.cpmi_closest_pair_noalloc(self._h, C.c_void_p(pts.data_ptr()), dt, n, d, ld,
                                                   _prec(precision), _stream_ptr(stream), C.byref(out)))
        return _pair(out)

    def frnn(self, pts, R2: float, precision="auto", stream=None, cap: int = 1 << 16, out=None):
        dt, n, d, ld = self._points_args(pts)
        rc, pairs, d2 = self._radius_call(
            lambda P, D, k, cnt: _lib.cpmi_frnn(self._h, C.c_void_p(pts.data_ptr()), dt, n, d, ld, float(R2),
                                                _prec(precision), _stream_ptr(stream), C.c_void_p(P.data_ptr()),
                                                C.c_void_p(D.data_ptr()), k, C.byref(cnt)), cap, out)
        self._check(rc)
        return pairs, d2

    def frnn_count(self, pts, R2: float, precision="auto", stream=None) -> int:
        """Number of pairs within the radius, from cpmi_frnn with no room for
        pairs (the first call of the two-call protocol; exact beyond 2^32)."""
        dt, n, d, ld = self._points_args(pts)
        cnt = C.c_int64(0)
        rc = _lib.cpmi_frnn(self._h, C.c_void_p(pts.data_ptr()), dt, n, d, ld, float(R2), _prec(precision),
                            _stream_ptr(stream), None, None, 0, C.byref(cnt))
        if rc != ERR_CAPACITY:
            self._check(rc)
        return int(cnt.value)

    def points(self, pts, R2: float | None = None, precision="auto", stream=None, cap: int = 1 << 16,
               want_pair: bool = True, out=None):
        dt, n, d, ld = self._points_args(pts)
        best = _CPair() if want_pair else None
        r2 = -1.0 if R2 is None else float(R2)
        if R2 is None:
            self._check(_lib.cpmi_points(self._h, C.c_void_p(pts.data_ptr()), dt, n, d, ld, _prec(precision), r2,
                                         _stream_ptr(stream), C.byref(best), None, None, 0, None))
            return _pair(best), None
        rc, pairs, d2 = self._radius_call(
            lambda P, D, k, cnt: _lib.cpmi_points(self._h, C.c_void_p(pts.data_ptr()), dt, n, d, ld,
                                                  _prec(precision), r2, _stream_ptr(stream),
                                                  C.byref(best) if best is not None else None,
                                                  C.c_void_p(P.data_ptr()), C.c_void_p(D.data_ptr()), k,
                                                  C.byref(cnt)), cap, out)
        self._check(rc)
        return (_pair(best) if best is not None else None), (pairs, d2)

    def motif(self, series, ell: int, excl: int = 0, R2: float | None = None, precision="auto", stream=None,
              cap: int = 1 << 16, want_pair: bool = True, out=None):
        import torch
        if series.device.type != "cuda" or series.dtype != torch.float32 or series.dim() != 1 or \
                series.stride(0) != 1:
            raise ValueError("series must be a contiguous 1-D float32 GPU tensor")
        best = _CPair() if want_pair else None
        L = series.shape[0]
        if R2 is None:
            self._check(_lib.cpmi_motif(self._h, C.c_void_p(series.data_ptr()), L, int(ell), int(excl),
                                        _prec(precision), -1.0, _stream_ptr(stream), C.byref(best), None, None, 0,
                                        None))
            return _pair(best), None
        rc, pairs, d2 = self._radius_call(
            lambda P, D, k, cnt: _lib.cpmi_motif(self._h, C.c_void_p(series.data_ptr()), L, int(ell), int(excl),
                                                 _prec(precision), float(R2), _stream_ptr(stream),
                                                 C.byref(best) if best is not None else None,
                                                 C.c_void_p(P.data_ptr()), C.c_void_p(D.data_ptr()), k,
                                                 C.byref(cnt)), cap, out)
        self._check(rc)
        return (_pair(best) if best is not None else None), (pairs, d2)

    def motif_batch(self, series_list, ells, precision="auto", stream=None):
        """Per-series motifs; returns a list of Pair or CpmiError (per-series status)."""
        import torch
        ns = len(series_list)
        ptrs = (C.c_void_p * ns)()
        lens = (C.c_int64 * ns)()
        ell_arr = (C.c_int64 * ns)()
        for k, (t, e) in enumerate(zip(series_list, ells)):
            if t.device.type != "cuda" or t.dtype != torch.float32 or t.dim() != 1 or t.stride(0) != 1:
                raise ValueError("each series must be a contiguous 1-D float32 GPU tensor")
            ptrs[k] = t.data_ptr()
            lens[k] = t.shape[0]
            ell_arr[k] = int(e)
        out = (_CPair * ns)()
        self._check(_lib.cpmi_motif_batch(self._h, ptrs, lens, ell_arr, ns, _prec(precision), _stream_ptr(stream),
                                          out))
        res = []
        for k in range(ns):
            if out[k].status != OK:
                res.append(CpmiError(out[k].status, f"series {k}"))
            else:
                res.append(_pair(out[k]))
        return res

    # ---- diagnostics
    def dbg_screen_sample(self, src, tiles, tile: int, precision="bf16", ell: int | None = None, stream=None):
        """cpmi_dbg_screen_sample: screen values and canonical d2 of every
        element of the listed tiles ((I, J) block pairs of edge `tile`) of a
        point set, or (ell given) of the windows of a series. Returns
        (dump [m, tile, tile], d2 [m, tile, tile] (NaN where no pair),
        bounds [m], max ratio)."""
        import numpy as np
        import torch
        tiles = np.ascontiguousarray(np.asarray(tiles, dtype=np.int64).reshape(-1, 2))
        m = tiles.shape[0]
        dev = f"cuda:{self.device}"
        if ell is None:
            dt, n, d, ld = self._points_args(src)
            series = 0
        else:
            if src.device.type != "cuda" or src.dtype != torch.float32 or src.dim() != 1 or not src.is_contiguous():
                raise ValueError("series must be a contiguous 1-D float32 GPU tensor")
            dt, n, d, ld, series = F32, src.shape[0], int(ell), 1, 1
        i8 = dt == I8
        dump = torch.empty((m, tile, tile), dtype=torch.int32 if i8 else torch.float32, device=dev)
        d2 = torch.full((m, tile, tile), float("nan"), dtype=torch.float64, device=dev)
        bounds = np.zeros(m, dtype=np.float64)
        ratio = C.c_double(0.0)
        self._check(_lib.cpmi_dbg_screen_sample(
            self._h, C.c_void_p(src.data_ptr()), dt, n, d, ld, series, _prec(precision), int(tile),
            tiles.ctypes.data_as(C.c_void_p), m, C.c_void_p(dump.data_ptr()), C.c_void_p(d2.data_ptr()),
            bounds.ctypes.data_as(C.c_void_p), C.byref(ratio), _stream_ptr(stream)))
        return dump, d2, bounds, float(ratio.value)

    def pairs_to_csr(self, pairs, n: int, stream=None):
        """Neighbour lists N(i) (Section 3.5) of a radius search's pairs
        (device int64 [m, 2], i < j) as compressed rows (cpmi_pairs_to_csr):
        returns (row_ptr [n + 1], cols [2m]), device int64; the neighbours of v
        are cols[row_ptr[v]:row_ptr[v + 1]], ascending."""
        import torch
        if pairs.dtype != torch.int64 or pairs.dim() != 2 or pairs.shape[1] != 2 or not pairs.is_contiguous():
            raise ValueError("pairs must be a contiguous int64 [m, 2] tensor")
        m = pairs.shape[0]
        row_ptr = torch.empty(int(n) + 1, dtype=torch.int64, device=pairs.device)
        cols = torch.empty(max(2 * m, 1), dtype=torch.int64, device=pairs.device)
        self._check(_lib.cpmi_pairs_to_csr(self._h, C.c_void_p(pairs.data_ptr()) if m else None, m, int(n),
                                           C.c_void_p(row_ptr.data_ptr()), C.c_void_p(cols.data_ptr()),
                                           _stream_ptr(stream)))
        return row_ptr, cols[:2 * m]

    def dbg_pruned_tiles_gpu(self, n: int, tile: int, lo, hi, T: float, excl: int = 1, permuted: bool = False,
                             stream=None):
        """cpmi_dbg_pruned_tiles_gpu: the pruned tile list built on the device
        from per-block intervals lo, hi (host arrays [nT, q]). Returns
        (entries as uint64 array, full slots, tiles dropped)."""
        import numpy as np
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        nT = -(-int(n) // int(tile))
        out = np.zeros(nT * (nT + 1) // 2 + 8, dtype=np.uint64)
        nf, npr = C.c_int64(0), C.c_int64(0)
        cnt = _lib.cpmi_dbg_pruned_tiles_gpu(self._h, int(n), int(tile), lo.shape[1], lo.ctypes.data, hi.ctypes.data,
                                             float(T), int(excl), int(bool(permuted)), out.ctypes.data, len(out),
                                             C.byref(nf), C.byref(npr), _stream_ptr(stream))
        if cnt < 0:
            self._check(int(cnt))
        return out[:cnt].copy(), nf.value, npr.value

    def dbg_set_prune_order(self, order: int, w: float = 1.0):
        """Row order of pruned radius searches (cpmi_dbg_set_prune_order): 0 =
        two references (buckets of width w R), 1 = the first reference only."""
        self._check(_lib.cpmi_dbg_set_prune_order(self._h, int(order), float(w)))

    def dbg_znorm(self, series, ell: int, precision="f32", stream=None):
        import torch
        N = series.shape[0] - ell + 1
        mu = torch.empty(N, dtype=torch.float64, device=series.device)
        sg = torch.empty(N, dtype=torch.float64, device=series.device)
        self._check(_lib.cpmi_dbg_znorm(self._h, C.c_void_p(series.data_ptr()), series.shape[0], int(ell),
                                        _prec(precision), C.c_void_p(mu.data_ptr()), C.c_void_p(sg.data_ptr()),
                                        _stream_ptr(stream)))
        return mu, sg


def dbg_mfma_probe(precision, A, B, C_out, stream=None):
    rc = _lib.cpmi_dbg_mfma_probe(_prec(precision), C.c_void_p(A.data_ptr()), C.c_void_p(B.data_ptr()),
                                  C.c_void_p(C_out.data_ptr()), _stream_ptr(stream))
    if rc != OK:
        raise CpmiError(rc, "mfma probe failed")


def dbg_copy(dst, src, stream=None):
    """Plain device copy of src into dst (same byte size, a multiple of 16):
    a launch of known traffic for scaling hardware byte counters."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("dbg_copy needs contiguous tensors of equal byte size")
    rc = _lib.cpmi_dbg_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nb, _stream_ptr(stream))
    if rc != OK:
        raise CpmiError(rc, "copy failed")


def dbg_mfma_peak(precision="bf16", iters: int = 100000, device: int = 0):
    """Sustained matrix-core rate (TFLOP/s, TOP/s for int8) of a pure
    multiply-accumulate kernel in the screen's instructions
    (cpmi_dbg_mfma_peak); returns (rate, milliseconds)."""
    ms = C.c_double(0.0)
    r = _lib.cpmi_dbg_mfma_peak(int(device), _prec(precision), int(iters), C.byref(ms))
    if r < 0:
        raise CpmiError(int(r), "matrix-core rate probe failed")
    return float(r), float(ms.value)


_default = None


def default_context() -> Context:
    global _default
    if _default is None:
        _default = Context()
    return _default


def closest_pair(pts, precision="auto", stream=None) -> Pair:
    return default_context().closest_pair(pts, precision, stream)


def frnn(pts, R2: float, precision="auto", stream=None):
    return default_context().frnn(pts, R2, precision, stream)


def points(pts, R2=None, precision="auto", stream=None):
    return default_context().points(pts, R2, precision, stream)


def motif(series, ell: int, excl: int = 0, R2=None, precision="auto", stream=None):
    return default_context().motif(series, ell, excl, R2, precision, stream)


def motif_batch(series_list, ells, precision="auto", stream=None):
    return default_context().motif_batch(series_list, ells, precision, stream)
