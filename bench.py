"""Benchmark: exact closest pair + fixed-radius pairs on the precision-form workload.

Default workload (the headline): n = 262,144 points, d = 512, float32, 64-cluster
Gaussian mixture with one planted pair (workloads.cfg_mixture); radius R = half
the lower-median nearest-neighbour distance (an oracle-computed input read from
tests/golden/mixture_n262144_d512.json). One step = one call of the whole hot
path: row prep -> BF16 matrix-core screen (tile minima) -> bound reduction and
tile selection -> second screen of the selected tiles -> FP64 verification ->
closest pair + sorted radius pairs, result exact (checked against the oracle's
stored answer). The plain FP32 screen is timed on the same workload for the
BF16-vs-FP32 speedup.

Prints one JSON line. `roofline` refers to the dominant kernel (the full-tile
pass-1 screen), timed with HIP events on the call's stream; `cpu_baseline` is
the CPU oracle on a bounded sample (rank 0, N = 1 only).

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
    python bench.py --workload {mixture,mixture_radius,points,motif,walk,batch,snp,strings,two_locus,lightbulb}   (same JSON form)
    python bench.py --workload walk --prune 10                   (reference-point tile pruning)
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact pair-evals/s + % MFMA roofline; BF16-screened vs plain FP32 speedup"
# published dense matrix-core peaks of MI355X
PEAK = {"bf16": (2500.0, "TFLOP/s"), "f32": (157.3, "TFLOP/s"), "i8": (5000.0, "TOP/s")}
PREC_NAME = {1: "f32", 2: "bf16", 3: "i8"}
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")
TRAFFIC = os.path.join(ROOT, "profiles", "screen256_bf16_mixture_n262144_d512.traffic.json")
# sources of the dominant kernel: the counters are only valid for this exact code
SCREEN_SRCS = [os.path.join(ROOT, "paper_1407_5609_amd", "csrc", f)
               for f in ("screen256.hip", "screen256_tile.inc", "layout256.h", "bound.h", "cpmi_internal.h")]


def note(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _traffic_per_launch():
    """HBM bytes per launch of the dominant kernel from the committed rocprof
    counter summary, or None if absent or taken on a different kernel source."""
    try:
        t = json.load(open(TRAFFIC))
        h = hashlib.sha256()
        for f in SCREEN_SRCS:
            h.update(open(f, "rb").read())
        if t.get("kernel_source_sha256") != h.hexdigest():
            return None
        return float(t["hbm_bytes_per_launch"])
    except Exception:
        return None


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _golden(name):
    return json.load(open(os.path.join(GOLDEN_DIR, name)))


def _want(g, as_int=False):
    import numpy as np
    conv = float if as_int else float.fromhex
    pair = (g["closest_pair"]["i"], g["closest_pair"]["j"], conv(g["closest_pair"]["d2"]))
    pairs = np.array(g["frnn"]["pairs"], dtype=np.int64).reshape(-1, 2)
    d2 = np.array([conv(v) for v in g["frnn"]["d2"]], dtype=np.float64)
    return pair, pairs, d2


def _timed_oracle(fn, grow, target_s):
    """Run fn(size) on a small size, then on the size expected to take ~target_s."""
    size = grow(None, None)
    t = time.perf_counter()
    fn(size)
    dt = time.perf_counter() - t
    size = grow(size, max(dt, 1e-6) / target_s)
    t = time.perf_counter()
    fn(size)
    return size, time.perf_counter() - t


# ---------------------------------------------------------------------------
# workloads: step(ctx, prec) runs one call of the hot path and returns whether
# the result equals the oracle's stored answer
# ---------------------------------------------------------------------------

class Workload:
    precs = ("bf16", "f32")        # primary precision first; the second is the comparison leg
    flops_per_pair = None          # algorithmic flops (int ops) per admissible pair
    graph = False                  # launches replayed from a captured graph (no per-launch events)
    roofline = True                # the step's dominant launch is a matrix-core screen
    out_cap = 0                    # radius pairs a step's caller-owned output holds (0: no radius output)

    def reserve(self, torch, steps):
        """The radius outputs of the next `steps` steps, allocated before the
        timed region: each step's outputs stay alive until they are checked
        after it, so a step allocating its own would call the device
        allocator inside the timed region."""
        self._outs = [(torch.empty((self.out_cap, 2), dtype=torch.int64, device="cuda:0"),
                       torch.empty(self.out_cap, dtype=torch.float64, device="cuda:0"))
                      for _ in range(steps)] if self.out_cap else []

    def _out(self):
        outs = getattr(self, "_outs", None)
        return outs.pop() if outs else None


class Points(Workload):
    """Common part of the point workloads (closest pair + radius pairs of one set)."""

    def _setup(self, torch, X, golden, as_int=False):
        g = _golden(golden)
        self.R2 = float(g["R2"]) if as_int else float.fromhex(g["R2"])
        self.want = _want(g, as_int)
        self.Xh = X
        self.n, self.d = X.shape
        self.X = torch.from_numpy(X).to("cuda:0")
        self.flops_per_pair = 2.0 * self.d
        return g

    query = "points"   # "cpp": the closest pair alone
    out_cap = 1 << 16

    def step(self, ctx, prec):
        import numpy as np
        wp, wpairs, wd = self.want
        if self.query == "cpp":
            best = ctx.closest_pair(self.X, precision=prec)
            return (best.i, best.j, best.d2) == wp
        best, (p, dd) = ctx.points(self.X, R2=self.R2, precision=prec, out=self._out())
        # the radius pairs stay on the device; they are compared after the timed steps
        return lambda: ((best.i, best.j, best.d2) == wp and np.array_equal(p.cpu().numpy(), wpairs)
                        and np.array_equal(dd.cpu().numpy(), wd))

    def cpu_baseline(self, target_s):
        import oracle
        X, m0 = self.Xh, min(self.Xh.shape[0], 2048)

        def grow(m, ratio):
            return m0 if m is None else int(min(X.shape[0], max(m0, m / ratio ** 0.5)))
        m, dt = _timed_oracle(lambda m: oracle.closest_pair(X[:m]), grow, target_s)
        pairs = m * (m - 1) // 2
        return pairs / dt, (f"closest pair over the first {m} of {X.shape[0]} rows ({pairs} pairs, "
                            f"d={X.shape[1]} {X.dtype}), {dt:.1f} s")


class Mixture(Points):
    name = "mixture"

    def __init__(self, W, torch):
        g = self._setup(torch, W.cfg_mixture()["X"], "mixture_n262144_d512.json")
        self.config = {"workload": f"mixture_n{self.n}_d{self.d}: exact closest pair + all pairs within R "
                                   "(BF16 matrix-core screen, FP64 verification)",
                       "n": self.n, "d": self.d, "R": float.fromhex(g["R"])}


def _radius_digest(pairs, d2):
    """SHA-256 of a radius list: pairs as little-endian int64, then d2 as little-endian float64."""
    import numpy as np
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pairs, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(d2, dtype="<f8").tobytes())
    return h.hexdigest()


class MixtureRadius(Mixture):
    """The headline points with a radius holding about 4*10^5 pairs (squared
    radius 832): the radius path (emission, FP64 verification, sort) at
    volume. Exactness: the list's length and digest equal the oracle's."""
    name = "mixture_radius"

    def __init__(self, W, torch):
        super().__init__(W, torch)
        g = _golden("mixture_n262144_d512_radius.json")
        self.R2 = float.fromhex(g["R2"])
        self.count, self.sha = g["count"], g["sha256"]
        self.out_cap = self.count
        self.config = dict(self.config, workload=f"mixture_n{self.n}_d{self.d}: exact closest pair + all "
                           f"{self.count} pairs within R = sqrt({self.R2:g}) (BF16 matrix-core screen, FP64 "
                           "verification)", R=self.R2 ** 0.5, radius_pairs=self.count)

    def step(self, ctx, prec):
        wp = self.want[0]
        best, (p, dd) = ctx.points(self.X, R2=self.R2, precision=prec, cap=self.count, out=self._out())
        return lambda: ((best.i, best.j, best.d2) == wp and len(p) == self.count
                        and _radius_digest(p.cpu().numpy(), dd.cpu().numpy()) == self.sha)


class SmallPoints(Points):
    name = "points"
    precs = ("f32", "bf16")

    def __init__(self, W, torch):
        self._setup(torch, W.cfg_points_small()["X"], "points_n4096_d64.json")
        self.config = {"workload": f"points_n{self.n}_d{self.d}: exact closest pair + all pairs within R=8",
                       "n": self.n, "d": self.d}


class Snp(Points):
    name = "snp"
    precs = ("i8",)

    def __init__(self, W, torch):
        self._setup(torch, W.cfg_snp()["X"], "snp_n100000_d4096.json", as_int=True)
        self.config = {"workload": f"snp_n{self.n}_d{self.d}: exact int8 closest pair + all pairs with d2 <= 800 "
                                   "(INT8 matrix-core screen, exact)", "n": self.n, "d": self.d}


class Motif(Workload):
    name = "motif"
    query = "points"   # "cpp": the motif alone, no radius pairs
    out_cap = 1 << 16

    def __init__(self, W, torch):
        self._setup(torch, W.cfg_motif(), "motif_L65536_l256.json")

    def _setup(self, torch, c, golden):
        g = _golden(golden)
        self.R2 = float.fromhex(g["R2"])
        self.want = _want(g)
        self.Th, self.ell, self.excl = c["T"], c["ell"], c["excl"]
        self.T = torch.from_numpy(self.Th).to("cuda:0")
        self.flops_per_pair = 2.0 * self.ell
        self.config = {"workload": f"{c['name']}: exact z-normalised motif + all window pairs within "
                                   f"R={c['R']:g} (exclusion l)", "length": len(self.Th), "ell": self.ell}

    def step(self, ctx, prec):
        import numpy as np
        wp, wpairs, wd = self.want
        if self.query == "cpp":
            best, _ = ctx.motif(self.T, self.ell, excl=self.excl, precision=prec)
            return (best.i, best.j, best.d2) == wp
        best, (p, dd) = ctx.motif(self.T, self.ell, excl=self.excl, R2=self.R2, precision=prec, out=self._out())
        # the radius pairs stay on the device; they are compared after the timed steps
        return lambda: ((best.i, best.j, best.d2) == wp and np.array_equal(p.cpu().numpy(), wpairs)
                        and np.array_equal(dd.cpu().numpy(), wd))

    def cpu_baseline(self, target_s):
        import oracle
        import workloads as W
        T, ell, L0 = self.Th, self.ell, 4 * self.ell + 2048

        def grow(L, ratio):
            return L0 if L is None else int(min(len(T), max(L0, L / ratio ** 0.5)))
        L, dt = _timed_oracle(lambda L: oracle.motif(T[:L], ell), grow, target_s)
        pairs = W.valid_pairs_motif(L, ell, ell)
        return pairs / dt, f"motif of the first {L} samples of the series ({pairs} window pairs, l={ell}), {dt:.1f} s"


class Walk(Motif):
    """The random-walk shape the paper measures reference-point pruning on
    (100,000 samples, windows of 1,024); run it with --prune 10."""
    name = "walk"

    def __init__(self, W, torch):
        self._setup(torch, W.cfg_walk(), "walk_L100000_l1024.json")


class Strings(Workload):
    """Least correlated pair of 20,000 strings of length 64 over 4 letters
    (Section 5: codes against complements on the INT8 matrix cores);
    --query most runs the most correlated pair (Hamming closest pair)."""
    name = "strings"
    precs = ("i8",)
    query = "least"

    def __init__(self, W, torch):
        c = W.cfg_strings()
        self.g = _golden(f"{c['name']}.json")
        self.Sh, self.sigma = c["S"], c["sigma"]
        self.S = torch.from_numpy(self.Sh).to("cuda:0")
        self.n, self.k = self.Sh.shape
        self.flops_per_pair = 2.0 * self.sigma * self.k   # one multiply-add per code bit
        self.config = {"workload": f"{c['name']}: exact least correlated pair of strings (one-hot codes vs "
                                   "complements, INT8 matrix cores)", "n": self.n, "k": self.k,
                       "sigma": self.sigma}

    def step(self, ctx, prec):
        r = ctx.strings_pair(self.S, self.sigma, self.query)
        w = self.g[self.query]
        return (r.i, r.j, r.matches) == (w["i"], w["j"], w["matches"])

    def cpu_baseline(self, target_s):
        import oracle
        S, m0 = self.Sh, 1000

        def grow(m, ratio):
            return m0 if m is None else int(min(S.shape[0], max(m0, m / ratio ** 0.5)))
        m, dt = _timed_oracle(lambda m: oracle.strings_pair(S[:m], self.sigma, self.query), grow, target_s)
        pairs = m * (m - 1) // 2
        return pairs / dt, f"{self.query} correlated pair of the first {m} strings ({pairs} pairs), {dt:.1f} s"


class LightBulb(Workload):
    """Randomised light-bulb bucketing (Section 4, MLBA) on the 20,000 strings:
    16 iterations of 8 random columns find the planted most correlated pair
    (seeded, so the run is repeatable); reports the pairs collected, the
    paper's measure of its work. Sort/bucket work, not a matrix-core screen:
    no roofline line."""
    name = "lightbulb"
    precs = ("i8",)
    roofline = False

    def __init__(self, W, torch):
        c = W.cfg_strings()
        self.g = _golden(f"{c['name']}.json")
        self.Sh, self.sigma = c["S"], c["sigma"]
        self.S = torch.from_numpy(self.Sh).to("cuda:0")
        self.n, self.k = self.Sh.shape
        self.pairs_collected = 0
        self.flops_per_pair = 0.0
        self.config = {"workload": f"{c['name']}: randomised light-bulb bucketing (16 iterations x 8 columns, "
                                   "seed 7) for the most correlated pair", "n": self.n, "k": self.k,
                       "sigma": self.sigma}

    def step(self, ctx, prec):
        r, self.pairs_collected = ctx.strings_lightbulb(self.S, self.sigma, "most", iterations=16, columns=8, seed=7)
        w = self.g["most"]
        return (r.i, r.j, r.matches) == (w["i"], w["j"], w["matches"])

    def cpu_baseline(self, target_s):
        return Strings.cpu_baseline(self, target_s)

    query = "most"


class TwoLocus(Workload):
    """Two-locus association on NOISE genotypes: 200 cases + 200 controls,
    50,000 SNPs, one injected pair (Section 6, D = [A' A'; B' ~B'] on the
    INT8 matrix cores)."""
    name = "two_locus"
    precs = ("i8",)

    def __init__(self, W, torch):
        c = W.cfg_two_locus()
        self.g = _golden(f"{c['name']}.json")
        self.Gh, self.m1, self.m2 = c["G"], c["m1"], c["m2"]
        self.G = torch.from_numpy(self.Gh).to("cuda:0")
        self.n = self.Gh.shape[1]
        self.flops_per_pair = 2.0 * 3 * (self.m1 + self.m2)
        self.config = {"workload": f"{c['name']}: exact two-locus SNP pair (columns of D = [A' A'; B' ~B'], INT8 "
                                   "matrix cores)", "snps": self.n, "cases": self.m1, "controls": self.m2}

    def step(self, ctx, prec):
        r = ctx.two_locus(self.G, self.m1, self.m2, 0)
        w = self.g["direction"]["0"]
        return (r.i, r.j, r.matches) == (w["i"], w["j"], w["matches"])

    def cpu_baseline(self, target_s):
        import numpy as np
        import oracle
        G, m0 = self.Gh, 500

        def grow(m, ratio):
            return m0 if m is None else int(min(G.shape[1], max(m0, m / ratio ** 0.5)))
        m, dt = _timed_oracle(lambda m: oracle.two_locus(np.ascontiguousarray(G[:, :m]), self.m1, self.m2, 0),
                              grow, target_s)
        pairs = m * (m - 1) // 2
        return pairs / dt, f"two-locus pair among the first {m} SNPs ({pairs} pairs), {dt:.1f} s"


class Batch(Workload):
    name = "batch"
    precs = ("auto", "f32")
    graph = True

    def __init__(self, W, torch):
        g = _golden("batch_512.json")
        c = W.cfg_batch()
        self.series, self.ells = c["series"], c["ells"]
        self.ts = [torch.from_numpy(T).to("cuda:0") for T in self.series]
        self.expected = g["series"]          # every series' motif, by the oracle
        pairs = [W.valid_pairs_motif(len(T), e, e) for T, e in zip(self.series, self.ells)]
        self.flops = sum(2.0 * e * p for e, p in zip(self.ells, pairs))
        self.config = {"workload": f"batch_{len(self.series)}: exact z-normalised motif of each of 512 series "
                                   "(lengths 4096-65536, l in {64,128,256,512}) in one graph-replayed batch",
                       "series": len(self.series), "algorithmic_flops": self.flops}

    def step(self, ctx, prec):
        res = ctx.motif_batch(self.ts, self.ells, precision=prec)
        return lambda: all((res[e["series"]].i, res[e["series"]].j, res[e["series"]].d2) ==
                           (e["closest_pair"]["i"], e["closest_pair"]["j"], float.fromhex(e["closest_pair"]["d2"]))
                           for e in self.expected)

    def cpu_baseline(self, target_s):
        import oracle
        import workloads as W
        t0, k, pairs = time.perf_counter(), 0, 0
        while k < len(self.series) and time.perf_counter() - t0 < target_s:
            oracle.motif(self.series[k], self.ells[k])
            pairs += W.valid_pairs_motif(len(self.series[k]), self.ells[k], self.ells[k])
            k += 1
        dt = time.perf_counter() - t0
        return pairs / dt, f"motifs of the first {k} series of the batch ({pairs} window pairs), {dt:.1f} s"


WORKLOADS = {w.name: w for w in (Mixture, MixtureRadius, SmallPoints, Motif, Walk, Batch, Snp, Strings, TwoLocus, LightBulb)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixture", choices=sorted(WORKLOADS))
    ap.add_argument("--fp32-steps", type=int, default=2, help="steps of the comparison precision (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peak-probe", action="store_true",
                    help="skip the sustained matrix-core rate probe reported beside the published peak")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--query", default=None, choices=["points", "cpp", "most", "least"],
                    help="point and single-series motif workloads: closest pair + radius pairs (points, the "
                         "default) or the closest pair alone (cpp); strings: least (default) or most correlated")
    ap.add_argument("--prune", type=int, default=0,
                    help="reference-point tile pruning with this many references (point and single-series motif workloads; 0: off)")
    ap.add_argument("--prune-f", type=float, default=10.0, help="projection factor of the references")
    ap.add_argument("--prune-order", type=int, default=0, choices=[0, 1],
                    help="row order of pruned radius queries with two or more references: 0 = buckets of the first "
                         "reference's distance sorted by the second's (the default), 1 = the first reference alone")
    ap.add_argument("--prune-w", type=float, default=1.0, help="bucket width of order 0, in units of R")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (a reference launch for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU split of the tile "
              "list is a design note, not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1407_5609_amd as cp
    import workloads as W

    torch.cuda.set_device(0)
    note(f"generating the {args.workload} workload")
    wl = WORKLOADS[args.workload](W, torch)
    if args.query == "cpp":
        if not isinstance(wl, (Points, Motif)):
            sys.exit("--query cpp applies to the point and single-series motif workloads only")
        wl.query = args.query
        wl.out_cap = 0
        wl.config = dict(wl.config, query="closest pair only")
    elif args.query in ("most", "least"):
        if not isinstance(wl, Strings):
            sys.exit(f"--query {args.query} applies to the strings workload only")
        wl.query = args.query
        wl.config = dict(wl.config, query=f"{args.query} correlated pair")
    ctx = cp.Context(0)
    if args.prune:
        ctx.set_pruning(args.prune, args.prune_f, seed=1)
        ctx.dbg_set_prune_order(args.prune_order, args.prune_w)

    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        cp.dbg_copy(dst, src)
        del src, dst

    def run(prec, steps, warmup):
        for _ in range(warmup):
            wl.step(ctx, prec)
        wl.reserve(torch, steps)
        torch.cuda.synchronize()
        screen_ms, checks, t0 = [], [], time.perf_counter()
        for _ in range(steps):
            checks.append(wl.step(ctx, prec))
            st = ctx.stats()
            screen_ms.append(st.screen_ms)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # every timed step's answer against the oracle's stored one (device
        # outputs are copied back only now, outside the timed region)
        exact = all(bool(c() if callable(c) else c) for c in checks)
        return wall / steps, sum(screen_ms) / len(screen_ms), st, exact

    prec = wl.precs[0]
    note(f"timing the {prec} path")
    ms_step, screen_ms, st, exact = run(prec, args.steps, args.warmup)
    note(f"{prec}: {ms_step * 1e3:.2f} ms/step")
    pprec = PREC_NAME.get(st.precision, "i8")
    peak, punit = PEAK[pprec]
    pairs = st.valid_pairs
    if wl.graph:
        # a graph replay records no per-launch events: the whole step's device work is the unit
        work, dur_ms, kernel = wl.flops, ms_step * 1e3, "whole batched step (graph replay)"
    else:
        work, dur_ms = wl.flops_per_pair * st.screen_pairs, screen_ms
        kernel = (f"screen256_kernel<{pprec}, min, full tiles>" if st.tile == 256
                  else f"screen_kernel<{pprec}, min> (128-row tiles, all tiles)")
        if args.prune and isinstance(wl, Motif):
            kernel = f"screen256_kernel<{pprec}, min, masked tiles> (windows in reference order)"
    achieved = work / (dur_ms * 1e-3) / 1e12 if dur_ms > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": pairs / ms_step,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": pprec,
        "data": "synthetic",
        "config": dict(wl.config, valid_pairs=pairs, tile=st.tile),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": punit, "frac": achieved / peak,
                     "traffic": _traffic_per_launch() if args.workload == "mixture" else None,
                     "kernel": kernel, "avg_launch_ms": dur_ms, "work_per_launch": work},
        "exact_match": bool(exact),
        "screen_err_over_bound": st.max_err_over_bound,
        # the last step's second pass: tiles screened again, candidates it emitted (the radius verifier
        # drops first those that the bound of their own two rows puts outside R)
        "pass2": {"tiles": st.tiles_rescreened, "of_tiles": st.tiles_total,
                  "candidates": st.cpp_candidates + st.frnn_candidates},
    }
    if wl.roofline and not args.no_peak_probe:
        # context: what a pure multiply-accumulate kernel in the same instructions sustains on this
        # GPU under load (clock-limited), beside the published peak the fraction is taken against
        note("probing the sustained matrix-core rate")
        mp, _ = cp.dbg_mfma_peak(pprec)
        out["roofline"]["measured_peak"] = mp
        out["roofline"]["frac_of_measured_peak"] = achieved / mp
    if not wl.roofline:
        out["roofline"] = None
        out["config"]["pairs_collected"] = wl.pairs_collected
    if isinstance(wl, (Points, Motif)) and not args.prune and st.precision != 3:
        # the screen bound on this workload, on the hardware: every element of
        # 16 seeded tiles, screen value against the verifier's canonical d2
        import numpy as np
        rows = wl.n if isinstance(wl, Points) else len(wl.Th) - wl.ell + 1
        nT = (rows + st.tile - 1) // st.tile
        rng = np.random.default_rng(20240607)
        tl = sorted({(nT - 1, nT - 1)} | {tuple(sorted(int(v) for v in rng.integers(0, nT, 2))) for _ in range(15)})
        src = wl.X if isinstance(wl, Points) else wl.T
        _, _, _, ratio = ctx.dbg_screen_sample(src, tl, st.tile, precision=pprec,
                                               ell=None if isinstance(wl, Points) else wl.ell)
        out["screen_sample"] = {"tiles": len(tl), "pairs": len(tl) * st.tile ** 2, "max_err_over_bound": ratio}
    if args.prune:
        # the paper's measure of pruned work (Section 3.6, Tables 1-2) is the
        # pairs that reach an exact distance; here: the pairs in the tiles the
        # screen still evaluates, and the candidates verified in FP64
        out["config"]["pruning"] = {"references": args.prune, "f": args.prune_f, "order": args.prune_order,
                                    "bucket_width_over_R": args.prune_w, "tiles_pruned": st.tiles_pruned,
                                    "tiles_screened": st.tiles_total,
                                    "pairs_in_screened_tiles_at_most": st.tiles_total * st.tile ** 2,
                                    "fp64_verified_pairs": st.cpp_candidates + st.frnn_candidates}
    if len(wl.precs) > 1 and args.fp32_steps > 0:
        cprec = wl.precs[1]
        note(f"timing the {cprec} comparison path")
        c_ms, c_screen_ms, st2, c_exact = run(cprec, args.fp32_steps, 1)
        out["exact_match"] = bool(exact and c_exact)
        leg = {"value": pairs / c_ms, "ms_per_step": c_ms * 1e3, "tile": st2.tile,
               f"speedup_{prec}_vs_{cprec}": c_ms / ms_step}
        if not wl.graph:
            tf = wl.flops_per_pair * st2.screen_pairs / (c_screen_ms * 1e-3) / 1e12
            leg.update(screen_tflops=tf, screen_frac_of_peak=tf / PEAK[PREC_NAME[st2.precision]][0])
        out["fp32_plain" if cprec == "f32" else f"{cprec}_screen"] = leg
    if not args.no_cpu_baseline:
        note("timing the CPU oracle on a sample")
        import oracle
        # every host core this process may use, at most 16 (the host share of one GPU)
        avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        threads = max(1, min(16, avail))
        oracle.set_threads(threads)
        v, sample = wl.cpu_baseline(args.cpu_seconds)
        oracle.set_threads(1)
        v1, sample1 = wl.cpu_baseline(args.cpu_seconds / 3)
        oracle.set_threads(threads)
        out["cpu_baseline"] = {"value": v, "unit": "pair-evals/s", "cores": threads, "kind": "oracle",
                               "sample": sample, "host_cpus": avail, "cpu_model": _cpu_model(),
                               "one_core": {"value": v1, "sample": sample1}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
