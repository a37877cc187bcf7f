"""GPU parity at the workloads' full sizes, in the configuration the benchmark
times (a context with the tuned tile choices).

The closest pair and radius pairs must equal the oracle's stored answers
bit for bit (tests/golden/, written by make_golden.py from the oracle only).
Where the oracle cannot afford the whole workload (the 512-series batch), it
checks a seeded sample of series whole and every other series one output at a
time: the reported pair is admissible, its squared distance is the oracle's
canonical value for that pair, and it is no larger than the oracle's value for
the planted pair (an admissible pair, so an upper bound of the minimum).
"""
import json
import os

import numpy as np
import pytest
import torch  # noqa: F401

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx(torch_dev):
    import paper_1407_5609_amd as cp
    c = cp.Context(0)
    yield c
    c.close()


def _dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _golden(name):
    return json.load(open(os.path.join(GOLDEN, name)))


def _want(g):
    pair = (g["closest_pair"]["i"], g["closest_pair"]["j"], float.fromhex(g["closest_pair"]["d2"]))
    pairs = np.array(g["frnn"]["pairs"], dtype=np.int64).reshape(-1, 2)
    d2 = np.array([float.fromhex(v) for v in g["frnn"]["d2"]])
    return pair, pairs, d2


def test_mixture_full_size_golden(ctx, torch_dev):
    g = _golden("mixture_n262144_d512.json")
    want_pair, want_pairs, want_d2 = _want(g)
    c = W.cfg_mixture()
    X = c["X"]
    t = _dev(X, torch_dev)
    R2 = float.fromhex(g["R2"])
    for prec in ("bf16", "f32"):
        best, (p, d) = ctx.points(t, R2=R2, precision=prec)
        assert (best.i, best.j, best.d2) == want_pair, (prec, best)
        assert np.array_equal(p.cpu().numpy(), want_pairs)
        assert np.array_equal(d.cpu().numpy(), want_d2)
        st = ctx.stats()
        assert st.valid_pairs == W.valid_pairs_points(X.shape[0])
        assert st.max_err_over_bound <= 1.0
        assert 0.0 <= best.screen_err <= best.screen_bound
    # sampled pairs, one at a time: none beats the reported minimum
    rng = np.random.default_rng(11)
    for _ in range(200):
        i, j = sorted(rng.choice(X.shape[0], 2, replace=False).tolist())
        assert oracle.d2(X, i, j) >= want_pair[2]


def test_mixture_full_size_golden_with_pruning(ctx, torch_dev):
    """The same answer with reference-point tile pruning on; most tiles are
    dropped (the rows cluster around 64 centres)."""
    g = _golden("mixture_n262144_d512.json")
    want_pair, want_pairs, want_d2 = _want(g)
    X = W.cfg_mixture()["X"]
    t = _dev(X, torch_dev)
    ctx.set_pruning(8, 10.0, seed=1)
    try:
        best, (p, d) = ctx.points(t, R2=float.fromhex(g["R2"]), precision="bf16")
        st = ctx.stats()
    finally:
        ctx.set_pruning(0)
    assert (best.i, best.j, best.d2) == want_pair
    assert np.array_equal(p.cpu().numpy(), want_pairs)
    assert np.array_equal(d.cpu().numpy(), want_d2)
    assert st.tiles_pruned > 0 and st.valid_pairs == W.valid_pairs_points(X.shape[0])
    print("pruned", st.tiles_pruned, "of", st.tiles_pruned + st.tiles_total, "tiles")


def test_motif_full_size_golden_with_pruning(ctx, torch_dev):
    """The 65,536-sample random walk (windows of 256) with reference-point
    pruning: the windows are screened in reference order and the answers
    equal the oracle's stored ones."""
    g = _golden("motif_L65536_l256.json")
    want_pair, want_pairs, want_d2 = _want(g)
    c = W.cfg_motif()
    t = _dev(c["T"], torch_dev)
    ctx.set_pruning(10, 10.0, seed=1)
    try:
        for prec in ("f32", "bf16"):
            best, (p, d) = ctx.motif(t, c["ell"], excl=c["excl"], R2=c["R2"], precision=prec)
            st = ctx.stats()
            assert (best.i, best.j, best.d2) == want_pair, (prec, best)
            assert np.array_equal(p.cpu().numpy(), want_pairs)
            assert np.array_equal(d.cpu().numpy(), want_d2)
            assert st.valid_pairs == W.valid_pairs_motif(65536, 256, 256)
            assert st.max_err_over_bound <= 1.0
            print(prec, "pruned", st.tiles_pruned, "of", st.tiles_pruned + st.tiles_total, "tiles")
    finally:
        ctx.set_pruning(0)


@pytest.mark.parametrize("q,order", [(0, 0), (10, 0), (10, 1)])
def test_walk_full_size_golden(ctx, torch_dev, q, order):
    """Random walk of 100,000 samples, windows of 1,024 (the shape the paper
    measures reference-point pruning on), unpruned and with q = 10 references
    projected by f = 10, the radius query in the two-reference order (0) or
    the first reference's (1): motif and radius pairs equal the oracle's."""
    g = _golden("walk_L100000_l1024.json")
    want_pair, want_pairs, want_d2 = _want(g)
    c = W.cfg_walk()
    t = _dev(c["T"], torch_dev)
    ctx.set_pruning(q, 10.0, seed=1)
    ctx.dbg_set_prune_order(order)
    try:
        best, (p, d) = ctx.motif(t, c["ell"], excl=c["excl"], R2=float.fromhex(g["R2"]), precision="bf16")
        st = ctx.stats()
        only, _ = ctx.motif(t, c["ell"], excl=c["excl"], precision="bf16")
    finally:
        ctx.set_pruning(0)
        ctx.dbg_set_prune_order(0)
    print("order", order, "tiles screened", st.tiles_total, "pruned", st.tiles_pruned)
    assert (best.i, best.j, best.d2) == want_pair
    assert (only.i, only.j, only.d2) == want_pair
    assert np.array_equal(p.cpu().numpy(), want_pairs)
    assert np.array_equal(d.cpu().numpy(), want_d2)
    assert st.max_err_over_bound <= 1.0
    assert (st.tiles_pruned > 0) == (q > 0)


def test_strings_full_size_golden(ctx, torch_dev):
    g = _golden("strings_n20000_k64_s4.json")
    c = W.cfg_strings()
    t = _dev(c["S"], torch_dev)
    for mode in ("most", "least"):
        r = ctx.strings_pair(t, c["sigma"], mode)
        assert (r.i, r.j, r.matches) == (g[mode]["i"], g[mode]["j"], g[mode]["matches"]), mode


def test_two_locus_full_size_golden(ctx, torch_dev):
    g = _golden("two_locus_n50000_m200+200.json")
    c = W.cfg_two_locus()
    t = _dev(c["G"], torch_dev)
    for direction in (0, 1):
        r = ctx.two_locus(t, c["m1"], c["m2"], direction)
        w = g["direction"][str(direction)]
        assert (r.i, r.j, r.matches) == (w["i"], w["j"], w["matches"]), direction
    assert tuple(c["pair"]) == (g["direction"]["0"]["i"], g["direction"]["0"]["j"])


def _radius_digest(pairs, d2):
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pairs, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(d2, dtype="<f8").tobytes())
    return h.hexdigest()


@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_mixture_radius_at_volume(ctx, torch_dev, prec):
    """262,144 points of d = 512 with a radius that holds about 4*10^5 pairs:
    the emitted candidates, their FP64 verification and the sorted list equal
    the oracle's list bit for bit (length, digest, first and last pairs)."""
    g = _golden("mixture_n262144_d512_radius.json")
    gm = _golden("mixture_n262144_d512.json")
    c = W.cfg_mixture()
    t = _dev(c["X"], torch_dev)
    R2 = float.fromhex(g["R2"])
    best, (p, d) = ctx.points(t, R2=R2, precision=prec, cap=g["count"])
    p, d = p.cpu().numpy(), d.cpu().numpy()
    assert len(p) == g["count"] > 100_000
    for (i, j, v), (a, b), x in zip(g["head"], p[:10], d[:10]):
        assert (i, j, float.fromhex(v)) == (a, b, x)
    for (i, j, v), (a, b), x in zip(g["tail"], p[-10:], d[-10:]):
        assert (i, j, float.fromhex(v)) == (a, b, x)
    assert _radius_digest(p, d) == g["sha256"]
    assert (best.i, best.j, best.d2) == (gm["closest_pair"]["i"], gm["closest_pair"]["j"],
                                         float.fromhex(gm["closest_pair"]["d2"]))
    st = ctx.stats()
    assert st.frnn_pairs == g["count"] and st.frnn_candidates >= g["count"]


@pytest.mark.parametrize("prec", ["auto", "f32"])
def test_batch_full_size(ctx, torch_dev, prec):
    """512 series of lengths 4,096-65,536 and windows of 64-512 in one batched
    call: every series' motif (i, j, d2) equals the oracle's bit for bit."""
    g = _golden("batch_512.json")
    c = W.cfg_batch()
    series, ells, plants = c["series"], c["ells"], c["plants"]
    assert len(g["series"]) == len(series)
    ts = [_dev(T, torch_dev) for T in series]
    first = ctx.motif_batch(ts, ells, precision=prec)
    st = ctx.stats()
    assert st.valid_pairs == sum(W.valid_pairs_motif(len(T), e, e) for T, e in zip(series, ells))
    again = ctx.motif_batch(ts, ells, precision=prec)          # replayed from the captured graph
    assert [(r.i, r.j, r.d2) for r in first] == [(r.i, r.j, r.d2) for r in again]
    for e in g["series"]:
        s = e["series"]
        assert (e["len"], e["ell"]) == (len(series[s]), ells[s])
        r = first[s]
        assert (r.i, r.j, r.d2) == (e["closest_pair"]["i"], e["closest_pair"]["j"],
                                    float.fromhex(e["closest_pair"]["d2"])), s
        assert 0.0 <= r.screen_err <= r.screen_bound or r.screen_bound == 0.0
    # the plants were found wherever the oracle found them
    hits = sum((e["closest_pair"]["i"], e["closest_pair"]["j"]) == tuple(e["plant"]) for e in g["series"])
    assert hits == sum((r.i, r.j) == tuple(p) for r, p in zip(first, plants))


def test_int8_genotypes_full_size_golden(ctx, torch_dev):
    """100,000 x 4096 int8 rows: the INT8 screen is exact, so the closest pair
    and the pairs within R2 = 800 must equal the oracle's bit for bit."""
    g = _golden("snp_n100000_d4096.json")
    c = W.cfg_snp()
    X = c["X"]
    t = _dev(X, torch_dev)
    best, (p, d) = ctx.points(t, R2=float(g["R2"]), precision="i8")
    assert (best.i, best.j, best.d2) == (g["closest_pair"]["i"], g["closest_pair"]["j"],
                                         float(g["closest_pair"]["d2"]))
    assert best.screen_err == 0.0 and best.screen_bound == 0.0
    assert np.array_equal(p.cpu().numpy(), np.array(g["frnn"]["pairs"], dtype=np.int64).reshape(-1, 2))
    assert np.array_equal(d.cpu().numpy(), np.array(g["frnn"]["d2"], dtype=np.float64))
    st = ctx.stats()
    assert st.valid_pairs == W.valid_pairs_points(X.shape[0])
    # the plants are the radius set (reading of the workload) and every reported d2 is exact
    assert sorted(map(tuple, p.cpu().numpy().tolist())) == sorted((a, b) for a, b, _ in c["plants"])
    for (i, j), v in zip(p.cpu().numpy().tolist(), d.cpu().numpy().tolist()):
        assert oracle.d2(X, i, j) == v
