"""Write the expected results of the workloads, computed by the CPU oracle.

Every value stored under tests/golden/ by this script comes from ``oracle``
(plain FP64 brute force) applied to the seeded inputs of ``workloads``; nothing
here touches the GPU library. Floats are stored with ``float.hex`` so that the
comparison in the tests is exact.

Usage:  python tests/golden/make_golden.py [points|motif|walk|strings|two_locus|snp|mixture|batch|mixture_radius ...]
        (no argument: all). Threads: ORACLE_THREADS (default: all cores).

Run times on 8 cores (latency-bound scalar FP64): points < 1 s, motif ~4 min,
walk ~45 min, snp ~20 min, mixture ~1 h (one nearest-neighbour pass), batch (all 512 series,
lane-parallel closest pair) ~30 min, mixture_radius (lane-parallel radius list) ~6 min.
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def _hex(v):
    return float(v).hex()


def _write(name, obj):
    path = os.path.join(HERE, name + ".json")
    with open(path + ".tmp", "w") as f:
        json.dump(obj, f, indent=1)
        f.write("\n")
    os.replace(path + ".tmp", path)
    print("wrote", path, flush=True)


def _frnn_obj(pairs, d2, as_int=False):
    return {"count": int(len(pairs)),
            "pairs": [[int(a), int(b)] for a, b in pairs],
            "d2": [int(v) for v in d2] if as_int else [_hex(v) for v in d2]}


def points():
    c = W.cfg_points_small()
    t = time.time()
    i, j, d2 = oracle.closest_pair(c["X"])
    pairs, dd = oracle.frnn(c["X"], c["R2"])
    _write(c["name"], {
        "workload": c["name"], "source": "oracle.closest_pair / oracle.frnn on workloads.cfg_points_small",
        "plant": list(c["plant"]), "R2": _hex(c["R2"]),
        "closest_pair": {"i": i, "j": j, "d2": _hex(d2)},
        "frnn": _frnn_obj(pairs, dd), "oracle_seconds": time.time() - t})


def motif():
    c = W.cfg_motif()
    t = time.time()
    best, (pairs, dd) = oracle.motif(c["T"], c["ell"], c["excl"], c["R2"])
    _write(c["name"], {
        "workload": c["name"], "source": "oracle.motif on workloads.cfg_motif",
        "ell": c["ell"], "excl": c["excl"], "plant": list(c["plant"]), "R2": _hex(c["R2"]),
        "closest_pair": {"i": best[0], "j": best[1], "d2": _hex(best[2])},
        "frnn": _frnn_obj(pairs, dd), "oracle_seconds": time.time() - t})


def walk():
    c = W.cfg_walk()
    t = time.time()
    best, (pairs, dd) = oracle.motif(c["T"], c["ell"], c["excl"], c["R2"])
    _write(c["name"], {
        "workload": c["name"], "source": "oracle.motif on workloads.cfg_walk",
        "ell": c["ell"], "excl": c["excl"], "plant": list(c["plant"]), "R2": _hex(c["R2"]),
        "closest_pair": {"i": best[0], "j": best[1], "d2": _hex(best[2])},
        "frnn": _frnn_obj(pairs, dd), "oracle_seconds": time.time() - t})


def strings():
    c = W.cfg_strings()
    t = time.time()
    most = oracle.strings_pair(c["S"], c["sigma"], "most")
    least = oracle.strings_pair(c["S"], c["sigma"], "least")
    _write(c["name"], {
        "workload": c["name"], "source": "oracle.strings_pair on workloads.cfg_strings",
        "sigma": c["sigma"], "near": list(c["near"]), "far": list(c["far"]),
        "most": {"i": most[0], "j": most[1], "matches": most[2]},
        "least": {"i": least[0], "j": least[1], "matches": least[2]},
        "oracle_seconds": time.time() - t})


def two_locus():
    c = W.cfg_two_locus()
    t = time.time()
    out = {}
    for direction in (0, 1):
        i, j, m = oracle.two_locus(c["G"], c["m1"], c["m2"], direction)
        out[str(direction)] = {"i": i, "j": j, "matches": m}
    _write(c["name"], {
        "workload": c["name"], "source": "oracle.two_locus on workloads.cfg_two_locus",
        "m1": c["m1"], "m2": c["m2"], "pair": list(c["pair"]), "direction": out,
        "oracle_seconds": time.time() - t})


def snp():
    c = W.cfg_snp()
    t = time.time()
    i, j, d2 = oracle.closest_pair(c["X"])
    pairs, dd = oracle.frnn(c["X"], c["R2"])
    _write(c["name"], {
        "workload": c["name"], "source": "oracle.closest_pair / oracle.frnn on workloads.cfg_snp (int8, exact)",
        "plants": [list(p) for p in c["plants"]], "R2": c["R2"],
        "closest_pair": {"i": i, "j": j, "d2": int(d2)},
        "frnn": _frnn_obj(pairs, dd, as_int=True), "oracle_seconds": time.time() - t})


def mixture():
    """Radius = half the lower-median nearest-neighbour distance (over all n
    points, planted rows included); closest pair and FRNN set from the same
    nearest-neighbour pass: a pair (i,j) at squared distance v has nn[i] <= v
    and nn[j] <= v, so only rows with nn <= the threshold need a row scan."""
    c = W.cfg_mixture()
    X = c["X"]
    n = X.shape[0]
    t = time.time()
    nn = oracle.nearest_neighbour_d2(X)
    med = float(np.sort(nn)[n // 2 - 1])
    R = 0.5 * math.sqrt(med)
    R2 = R * R
    dmin = float(nn.min())
    best = None
    for i in np.flatnonzero(nn == dmin):
        row = oracle.row_d2(X, int(i))
        js = [j for j in np.flatnonzero(row == dmin) if j > i]
        if js:
            best = (int(i), int(js[0]), dmin)
            break
    pairs, dd = [], []
    for i in np.flatnonzero(nn <= R2):
        row = oracle.row_d2(X, int(i))
        for j in np.flatnonzero(row <= R2):
            if j > i:
                pairs.append((int(i), int(j)))
                dd.append(float(row[j]))
    order = sorted(range(len(pairs)), key=lambda k: pairs[k])
    pairs = [pairs[k] for k in order]
    dd = [dd[k] for k in order]
    _write(c["name"], {
        "workload": c["name"],
        "source": "oracle.nearest_neighbour_d2 + oracle.row_d2 on workloads.cfg_mixture",
        "plant": list(c["plant"]), "R": _hex(R), "R2": _hex(R2),
        "median_nn_d2": _hex(med), "nn_d2_min": _hex(dmin),
        "nn_d2_quantiles": {q: _hex(np.quantile(nn, float(q))) for q in ("0.001", "0.01", "0.5", "0.99")},
        "closest_pair": {"i": best[0], "j": best[1], "d2": _hex(best[2])},
        "frnn": _frnn_obj(pairs, dd), "oracle_seconds": time.time() - t})


def batch():
    """Every series of the batch: z-normalised windows and their closest pair
    by the oracle's lane-parallel brute force (closest_pair_lanes, equal bit
    for bit to the plain loop; tests/test_oracle_pins.py checks that)."""
    c = W.cfg_batch()
    t = time.time()
    out = []
    for s, (T, ell) in enumerate(zip(c["series"], c["ells"])):
        best, _ = oracle.motif(T, ell, lanes=True)
        out.append({"series": s, "len": int(T.shape[0]), "ell": int(ell),
                    "plant": list(c["plants"][s]),
                    "closest_pair": {"i": best[0], "j": best[1], "d2": _hex(best[2])}})
        print("batch series", s, "len", int(T.shape[0]), "ell", int(ell), "done", round(time.time() - t, 1),
              flush=True)
    _write(c["name"], {
        "workload": c["name"], "source": "oracle.motif(lanes=True) on every workloads.cfg_batch series",
        "series": out, "oracle_seconds": time.time() - t})


MIXTURE_RADIUS_R2 = 832.0


def radius_digest(pairs, d2):
    """SHA-256 of a radius list: the (i, j) pairs as little-endian int64, then
    the squared distances as little-endian float64."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pairs, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(d2, dtype="<f8").tobytes())
    return h.hexdigest()


def mixture_radius():
    """The mixture points with a radius that holds several hundred thousand
    pairs (squared radius 832 against a typical squared distance of about
    1,000 inside a cluster): the whole list by the oracle's lane-parallel
    scan, stored as its length, digest and first and last pairs."""
    c = W.cfg_mixture()
    X = c["X"].astype(np.float64)          # exact: every float32 is a double
    t = time.time()
    pairs, dd = oracle.frnn(X, MIXTURE_RADIUS_R2, lanes=True)
    head = [[int(a), int(b), _hex(v)] for (a, b), v in zip(pairs[:10], dd[:10])]
    tail = [[int(a), int(b), _hex(v)] for (a, b), v in zip(pairs[-10:], dd[-10:])]
    _write(c["name"] + "_radius", {
        "workload": c["name"] + "_radius",
        "source": "oracle.frnn(lanes=True) on workloads.cfg_mixture rows promoted to float64",
        "R2": _hex(MIXTURE_RADIUS_R2), "count": int(len(pairs)), "sha256": radius_digest(pairs, dd),
        "digest": "sha256 of the pairs as little-endian int64 (i, j), then the d2 as little-endian float64",
        "head": head, "tail": tail, "oracle_seconds": time.time() - t})


JOBS = {"points": points, "motif": motif, "walk": walk, "strings": strings, "two_locus": two_locus, "snp": snp,
        "mixture": mixture, "batch": batch, "mixture_radius": mixture_radius}

if __name__ == "__main__":
    if os.environ.get("ORACLE_THREADS"):
        oracle.set_threads(int(os.environ["ORACLE_THREADS"]))
    names = sys.argv[1:] or list(JOBS)
    for nm in names:
        t0 = time.time()
        JOBS[nm]()
        print(nm, "took", round(time.time() - t0, 1), "s", flush=True)
