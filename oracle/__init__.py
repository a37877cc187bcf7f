"""Python access to the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package. It loads oracle/liboracle.so (plain C, FP64 brute force; see
oracle.c for the definitions and the canonical arithmetic it follows) and
wraps it for numpy arrays. It imports nothing from the GPU package.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

NOPAIR = -2
DEGENERATE = -4

_i64 = C.c_int64
_p = C.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB)
        L.orc_d2_f32.restype = C.c_double
        L.orc_d2_f32.argtypes = [_p, _i64, _i64, _i64, _i64]
        L.orc_d2_f64.restype = C.c_double
        L.orc_d2_f64.argtypes = [_p, _i64, _i64, _i64, _i64]
        L.orc_d2_i8.restype = _i64
        L.orc_d2_i8.argtypes = [_p, _i64, _i64, _i64, _i64]
        for nm in ("orc_row_d2_f32", "orc_row_d2_f64", "orc_row_d2_i8"):
            getattr(L, nm).restype = None
            getattr(L, nm).argtypes = [_p, _i64, _i64, _i64, _i64, _p]
        L.orc_znorm.restype = C.c_int
        L.orc_znorm.argtypes = [_p, _i64, _i64, _p, _p, _p]
        for nm in ("orc_cpp_f32", "orc_cpp_f64", "orc_cpp_i8"):
            getattr(L, nm).restype = C.c_int
            getattr(L, nm).argtypes = [_p, _i64, _i64, _i64, _i64, _p, _p, _p]
        L.orc_cpp_f64_lanes.restype = C.c_int
        L.orc_cpp_f64_lanes.argtypes = [_p, _i64, _i64, _i64, _i64, _p, _p, _p]
        for nm in ("orc_frnn_f32", "orc_frnn_f64", "orc_frnn_i8"):
            getattr(L, nm).restype = _i64
            getattr(L, nm).argtypes = [_p, _i64, _i64, _i64, _i64, C.c_double, _p, _p, _i64]
        for nm in ("orc_block_d2_f32", "orc_block_d2_f64", "orc_block_d2_i8"):
            getattr(L, nm).restype = None
            getattr(L, nm).argtypes = [_p, _i64, _i64, _i64, _i64, _i64, _i64, _p]
        L.orc_frnn_f64_lanes.restype = _i64
        L.orc_frnn_f64_lanes.argtypes = [_p, _i64, _i64, _i64, _i64, C.c_double, _p, _p, _i64]
        L.orc_frnn_count_f32.restype = _i64
        L.orc_frnn_count_f32.argtypes = [_p, _i64, _i64, _i64, _i64, C.c_double]
        L.orc_nn_f32.restype = C.c_int
        L.orc_nn_f32.argtypes = [_p, _i64, _i64, _i64, _p]
        L.orc_matches.restype = _i64
        L.orc_matches.argtypes = [_p, _i64, _i64, _i64, _i64]
        L.orc_encode.restype = None
        L.orc_encode.argtypes = [_p, _i64, _i64, _i64, C.c_int, C.c_int, _p]
        L.orc_bit_matches.restype = _i64
        L.orc_bit_matches.argtypes = [_p, _p, _i64, _i64, _i64]
        L.orc_strings_pair.restype = C.c_int
        L.orc_strings_pair.argtypes = [_p, _i64, _i64, _i64, C.c_int, C.c_int, _p, _p, _p]
        L.orc_two_locus.restype = C.c_int
        L.orc_two_locus.argtypes = [_p, _i64, _i64, _i64, _i64, C.c_int, _p, _p, _p]
        L.orc_max_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _kind(X: np.ndarray) -> str:
    if X.dtype == np.float32:
        return "f32"
    if X.dtype == np.float64:
        return "f64"
    if X.dtype == np.int8:
        return "i8"
    raise TypeError(f"unsupported dtype {X.dtype}")


def _rows(X: np.ndarray):
    if X.ndim != 2:
        raise ValueError("expected a 2-D array")
    if X.strides[1] != X.itemsize or X.strides[0] % X.itemsize:
        X = np.ascontiguousarray(X)
    return X, X.shape[0], X.shape[1], X.strides[0] // X.itemsize


def max_threads() -> int:
    return lib().orc_max_threads()


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def d2(X: np.ndarray, i: int, j: int):
    """Canonical squared distance between rows i and j (float, or int for int8)."""
    X, n, d, ld = _rows(X)
    return getattr(lib(), "orc_d2_" + _kind(X))(X.ctypes.data, d, ld, int(i), int(j))


def row_d2(X: np.ndarray, i: int) -> np.ndarray:
    """Canonical squared distance from row i to every row (entry i is 0)."""
    X, n, d, ld = _rows(X)
    k = _kind(X)
    out = np.empty(n, dtype=np.int64 if k == "i8" else np.float64)
    getattr(lib(), "orc_row_d2_" + k)(X.ctypes.data, n, d, ld, int(i), out.ctypes.data)
    return out


def closest_pair(X: np.ndarray, excl: int = 1):
    """(i, j, d2) minimising the canonical d2 over i<j, j-i>=excl; ties go to
    the lexicographically smallest (i, j). None if there is no admissible pair."""
    X, n, d, ld = _rows(X)
    oi, oj, od = _i64(), _i64(), C.c_double()
    rc = getattr(lib(), "orc_cpp_" + _kind(X))(X.ctypes.data, n, d, ld, int(excl),
                                               C.byref(oi), C.byref(oj), C.byref(od))
    if rc == NOPAIR:
        return None
    if rc != 0:
        raise RuntimeError(f"oracle closest pair failed: {rc}")
    if X.dtype == np.int8:
        return oi.value, oj.value, int(od.value)
    return oi.value, oj.value, od.value


def closest_pair_lanes(X: np.ndarray, excl: int = 1):
    """closest_pair for float64 rows with SIMD lanes across pairs j: each
    pair's arithmetic and the tie rule are those of closest_pair, so the
    result is the same bit for bit; only faster on large inputs."""
    X, n, d, ld = _rows(X)
    if X.dtype != np.float64:
        raise TypeError("closest_pair_lanes takes float64 rows")
    oi, oj, od = _i64(), _i64(), C.c_double()
    rc = lib().orc_cpp_f64_lanes(X.ctypes.data, n, d, ld, int(excl), C.byref(oi), C.byref(oj), C.byref(od))
    if rc == NOPAIR:
        return None
    if rc != 0:
        raise RuntimeError(f"oracle closest pair failed: {rc}")
    return oi.value, oj.value, od.value


def frnn(X: np.ndarray, R2: float, excl: int = 1, lanes: bool = False):
    """All pairs i<j (j-i>=excl) with canonical d2 <= R2, sorted by (i, j).
    Returns (pairs int64 [m,2], d2 [m]). lanes=True (float64 rows) uses the
    lane-parallel scan (same result, faster on large inputs)."""
    X, n, d, ld = _rows(X)
    if lanes and X.dtype != np.float64:
        raise TypeError("frnn(lanes=True) takes float64 rows")
    fn = lib().orc_frnn_f64_lanes if lanes else getattr(lib(), "orc_frnn_" + _kind(X))
    cap = 1 << 16
    while True:
        pairs = np.empty((cap, 2), dtype=np.int64)
        dd = np.empty(cap, dtype=np.float64)
        cnt = fn(X.ctypes.data, n, d, ld, int(excl), float(R2), pairs.ctypes.data, dd.ctypes.data, cap)
        if cnt < 0:
            raise RuntimeError(f"oracle frnn failed: {cnt}")
        if cnt <= cap:
            pairs, dd = pairs[:cnt].copy(), dd[:cnt].copy()
            if X.dtype == np.int8:
                dd = dd.astype(np.int64)
            return pairs, dd
        cap = int(cnt)


def neighbour_lists(pairs: np.ndarray, n: int):
    """Section 3.5's output form: N(i), the other points within the radius,
    for every point i, from the pair list (i, j), i < j, of frnn: j is added
    to N(i) and i to N(j), each list ascending. Returned as compressed rows
    (row_ptr int64 [n + 1], cols int64 [2m]). Plain loops over the pairs."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    lists = [[] for _ in range(n)]
    for i, j in pairs.tolist():
        if not 0 <= i < j < n:
            raise ValueError(f"pair ({i}, {j}) outside 0 <= i < j < {n}")
        lists[i].append(j)
        lists[j].append(i)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cols = []
    for v in range(n):
        lists[v].sort()
        cols.extend(lists[v])
        row_ptr[v + 1] = row_ptr[v] + len(lists[v])
    return row_ptr, np.array(cols, dtype=np.int64)


def block_d2(X: np.ndarray, i0: int, ni: int, j0: int, nj: int) -> np.ndarray:
    """Canonical d2 of rows i0..i0+ni-1 against rows j0..j0+nj-1: float64
    [ni, nj] (int8 rows: exact integers as float64)."""
    X, n, d, ld = _rows(X)
    if not (0 <= i0 and i0 + ni <= n and 0 <= j0 and j0 + nj <= n):
        raise IndexError("block out of range")
    out = np.empty((ni, nj), dtype=np.float64)
    getattr(lib(), "orc_block_d2_" + _kind(X))(X.ctypes.data, d, ld, int(i0), int(ni), int(j0), int(nj),
                                               out.ctypes.data)
    return out


def frnn_count(X: np.ndarray, R2: float, excl: int = 1) -> int:
    """Number of pairs i<j (j-i>=excl) with canonical d2 <= R2 (float32 rows)."""
    X, n, d, ld = _rows(X)
    if X.dtype != np.float32:
        raise TypeError("frnn_count takes float32 points")
    return int(lib().orc_frnn_count_f32(X.ctypes.data, n, d, ld, int(excl), float(R2)))


def nearest_neighbour_d2(X: np.ndarray) -> np.ndarray:
    """min over j != i of the canonical d2, for every row i (float32 input)."""
    X, n, d, ld = _rows(X)
    if X.dtype != np.float32:
        raise TypeError("nearest_neighbour_d2 takes float32 points")
    out = np.empty(n, dtype=np.float64)
    rc = lib().orc_nn_f32(X.ctypes.data, n, d, ld, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle nn failed: {rc}")
    return out


def znorm(T: np.ndarray, ell: int):
    """Canonical z-normalised windows of T: (Xhat [N, ell] float64, mu, sigma).
    Raises ValueError if some window has sigma == 0."""
    T = np.ascontiguousarray(T, dtype=np.float32)
    N = T.shape[0] - ell + 1
    if N < 1:
        raise ValueError("series shorter than the window")
    Xhat = np.empty((N, ell), dtype=np.float64)
    mu = np.empty(N, dtype=np.float64)
    sg = np.empty(N, dtype=np.float64)
    rc = lib().orc_znorm(T.ctypes.data, T.shape[0], int(ell), Xhat.ctypes.data, mu.ctypes.data, sg.ctypes.data)
    if rc == DEGENERATE:
        raise ValueError("a window has zero variance")
    if rc != 0:
        raise RuntimeError(f"oracle znorm failed: {rc}")
    return Xhat, mu, sg


def motif(T: np.ndarray, ell: int, excl: int | None = None, R2: float | None = None, lanes: bool = False):
    """Motif of a series: closest pair of z-normalised windows with j-i >= excl
    (default excl = ell), plus all admissible pairs with d2 <= R2 if R2 given.
    lanes=True takes the closest pair from closest_pair_lanes (same result).
    Returns (best (i, j, d2) or None, frnn (pairs, d2) or None)."""
    if excl is None or excl <= 0:
        excl = ell
    Xhat, _, _ = znorm(T, ell)
    best = closest_pair_lanes(Xhat, excl) if lanes else closest_pair(Xhat, excl)
    fr = frnn(Xhat, R2, excl) if R2 is not None and R2 >= 0 else None
    return best, fr


# ---------------------------------------------------------------------------
# strings (Sections 5 and 6)
# ---------------------------------------------------------------------------

def _int8_rows(S: np.ndarray) -> np.ndarray:
    S = np.ascontiguousarray(S)
    if S.dtype != np.int8 or S.ndim != 2:
        raise TypeError("expected a 2-D int8 array")
    return S


def matches(S: np.ndarray, i: int, j: int) -> int:
    """m(S_i, S_j): positions where strings i and j agree (Section 5)."""
    S = _int8_rows(S)
    return int(lib().orc_matches(S.ctypes.data, S.shape[1], S.shape[1], i, j))


def encode(S: np.ndarray, sigma: int, complement: bool = False) -> np.ndarray:
    """Section 5's deterministic mapping (symbol v -> sigma bits, one set, the
    paper's order 0 -> 0..001), optionally complemented: n x (sigma k) 0/1."""
    S = _int8_rows(S)
    n, k = S.shape
    X = np.zeros((n, sigma * k), dtype=np.int8)
    lib().orc_encode(S.ctypes.data, n, k, k, int(sigma), int(bool(complement)), X.ctypes.data)
    return X


def bit_matches(X: np.ndarray, Y: np.ndarray, i: int, j: int) -> int:
    """M(X_i, Y_j): equal bits of two rows of 0/1 matrices of one width."""
    X, Y = _int8_rows(X), _int8_rows(Y)
    assert X.shape[1] == Y.shape[1]
    return int(lib().orc_bit_matches(X.ctypes.data, Y.ctypes.data, X.shape[1], i, j))


def strings_pair(S: np.ndarray, sigma: int, mode: str = "most"):
    """(i, j, u): the most correlated pair (plain definition) or the least
    correlated one (Section 5's code/complement reduction), u = m(S_i, S_j)."""
    S = _int8_rows(S)
    n, k = S.shape
    oi, oj, om = C.c_int64(), C.c_int64(), C.c_int64()
    rc = lib().orc_strings_pair(S.ctypes.data, n, k, k, int(sigma), {"most": 0, "least": 1}[mode],
                                C.byref(oi), C.byref(oj), C.byref(om))
    if rc == NOPAIR:
        return None
    if rc != 0:
        raise MemoryError("oracle out of memory")
    return int(oi.value), int(oj.value), int(om.value)


def two_locus(G: np.ndarray, m1: int, m2: int, direction: int = 0):
    """(i, j, matches): Section 6's pair of columns (i, n + j), i != j, of D =
    [A' A'; B' ~B'] (direction 1: [A' ~A'; B' B']) with the most equal bits.
    G: (m1 + m2) x n genotypes in {0, 1, 2}, cases first."""
    G = _int8_rows(G)
    assert G.shape[0] == m1 + m2
    n = G.shape[1]
    oi, oj, om = C.c_int64(), C.c_int64(), C.c_int64()
    rc = lib().orc_two_locus(G.ctypes.data, int(m1), int(m2), n, n, int(direction), C.byref(oi), C.byref(oj),
                             C.byref(om))
    if rc == NOPAIR:
        return None
    if rc != 0:
        raise MemoryError("oracle out of memory")
    return int(oi.value), int(oj.value), int(om.value)


# ---------------------------------------------------------------------------
# randomised light-bulb bucketing (Section 4, MLBA; Section 5's codes and
# complements for the least correlated pair)
# ---------------------------------------------------------------------------

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(state: int) -> int:
    """SplitMix64 (Steele, Lea and Flood, 2014): the output for `state`, i.e.
    the state advanced by the golden-ratio increment, then mixed."""
    z = (state + _GOLDEN) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def lightbulb_columns(seed: int, iterations: int, columns: int, ncols: int):
    """The columns each iteration draws: the first `columns` entries of a
    partial Fisher-Yates shuffle of 0..ncols-1, restarted per iteration; step
    q swaps entries q and q + splitmix64(c) mod (ncols - q), c counting up
    from seed * golden (mod 2^64) over all steps."""
    c = (seed * _GOLDEN) & _M64
    out = []
    for _ in range(iterations):
        pool = list(range(ncols))
        for q in range(columns):
            r = q + splitmix64(c) % (ncols - q)
            c = (c + 1) & _M64
            pool[q], pool[r] = pool[r], pool[q]
        out.append(pool[:columns])
    return out


def lightbulb(S: np.ndarray, sigma: int, mode: str, iterations: int, columns: int, seed: int):
    """MLBA as a candidate generator: per iteration, the rows whose values in
    the drawn columns agree form a bucket and every pair in a bucket is a
    candidate. Most correlated: rows are the strings, columns positions.
    Least correlated: rows are the one-hot codes of the strings and their
    complements, columns bit positions of the codes, and the candidates are
    the (code i, complement j) pairs with i != j. Returns (candidate pairs
    over all iterations, best) with best = (i, j, m(S_i, S_j)) over the
    candidates, the most (least) matches first, then the smallest (i, j); or
    None without candidates. Plain loops over buckets: small inputs."""
    S = _int8_rows(S)
    n, k = S.shape
    if mode == "most":
        R = S.astype(np.int64)
        ncol = k
    else:
        X = encode(S, sigma).astype(np.int64)
        R = np.concatenate([X, 1 - X])                  # rows n..2n-1: complements
        ncol = sigma * k
    total = 0
    cands = set()
    for cols in lightbulb_columns(seed, iterations, columns, ncol):
        buckets = {}
        for r in range(R.shape[0]):
            buckets.setdefault(tuple(R[r, cols].tolist()), []).append(r)
        for rows in buckets.values():
            for x in range(len(rows)):
                for y in range(x + 1, len(rows)):
                    a, b = rows[x], rows[y]
                    if mode == "least":
                        if (a < n) == (b < n):
                            continue
                        a, b = (a, b - n) if a < n else (b, a - n)
                        if a == b:
                            continue
                    total += 1
                    cands.add((min(a, b), max(a, b)))
    if not cands:
        return total, None
    scored = [(matches(S, i, j), i, j) for i, j in cands]
    if mode == "most":
        u, i, j = min(scored, key=lambda t: (-t[0], t[1], t[2]))
    else:
        u, i, j = min(scored, key=lambda t: (t[0], t[1], t[2]))
    return total, (i, j, u)
