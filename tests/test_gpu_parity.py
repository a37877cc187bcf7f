"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Closest-pair indices and radius pair sets must match exactly; because both
sides follow the same canonical FP64 arithmetic, squared distances must match
bit for bit (the required tolerance is 1e-9 relative; equality is checked).
Cases span several tiles with ragged tails, every screening precision, the
exclusion boundary, exact ties, and the degenerate inputs.
"""
import json
import os

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)

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


def _check_pair(best, want):
    assert (best.i, best.j) == tuple(want[:2]), (best, want)
    assert best.d2 == want[2], (best.d2.hex(), float(want[2]).hex())
    assert abs(best.d2 - want[2]) <= 1e-9 * max(abs(want[2]), 1e-300)


def _window_d2(T, ell, i, j):
    """Canonical squared distance of windows i and j, each z-normalised on its own."""
    a, _, _ = oracle.znorm(T[i:i + ell], ell)
    b, _, _ = oracle.znorm(T[j:j + ell], ell)
    return oracle.d2(np.concatenate([a, b]), 0, 1)


def _check_frnn(got, want):
    gp, gd = got
    wp, wd = want
    gp = gp.cpu().numpy()
    gd = gd.cpu().numpy()
    assert gp.shape == wp.shape, (gp.shape, wp.shape)
    assert np.array_equal(gp, wp)
    assert np.array_equal(gd, wd.astype(np.float64))


# ---------------------------------------------------------------------------
# device behaviour the screen relies on
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f32", "bf16", "i8"])
def test_mfma_lane_layout(torch_dev, prec):
    import torch

    import paper_1407_5609_amd as cp
    rng = np.random.default_rng(1)
    if prec == "f32":
        A = rng.normal(size=(32, 8)).astype(np.float32)
        B = rng.normal(size=(32, 8)).astype(np.float32)
        want = A.astype(np.float64) @ B.astype(np.float64).T
        tol = 1e-5
    elif prec == "bf16":
        A = rng.integers(-8, 8, (32, 16)).astype(np.float32)   # exact in bf16
        B = rng.integers(-8, 8, (32, 16)).astype(np.float32)
        want = A.astype(np.float64) @ B.astype(np.float64).T
        A = (A.view(np.uint32) >> 16).astype(np.uint16)
        B = (B.view(np.uint32) >> 16).astype(np.uint16)
        tol = 0
    else:
        A = rng.integers(-128, 128, (32, 32)).astype(np.int8)
        B = rng.integers(-128, 128, (32, 32)).astype(np.int8)
        want = A.astype(np.int64) @ B.astype(np.int64).T
        tol = 0
    C = torch.zeros((32, 32), dtype=torch.float32, device=torch_dev)
    cp.dbg_mfma_probe(prec, _dev(A, torch_dev), _dev(B, torch_dev), C)
    got = C.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want)), np.argwhere(np.abs(got - want) > 1e-3)[:5]


@pytest.mark.parametrize("ell", [16, 100, 256, 512])
def test_window_stats_are_canonical_bitwise(ctx, torch_dev, ell):
    rng = np.random.default_rng(ell)
    T = W.random_walk(rng, 5000)
    mu, sg = ctx.dbg_znorm(_dev(T, torch_dev), ell)
    _, omu, osg = oracle.znorm(T, ell)
    assert np.array_equal(mu.cpu().numpy(), omu)
    assert np.array_equal(sg.cpu().numpy(), osg)


# ---------------------------------------------------------------------------
# points
# ---------------------------------------------------------------------------

SHAPES = [(2, 1), (3, 5), (129, 7), (300, 64), (1000, 33), (1500, 200), (700, 512), (2300, 96)]


@pytest.fixture(params=[128, 256])
def tile(request, ctx):
    for p in ("f32", "bf16", "i8"):
        ctx.set_tile(p, request.param)
    yield request.param
    for p in ("f32", "bf16", "i8"):
        ctx.set_tile(p, 0)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("n,d", SHAPES)
def test_points_match_oracle(ctx, torch_dev, tile, prec, n, d):
    rng = np.random.default_rng(n * 1000 + d)
    X = rng.normal(0, 1, (n, d)).astype(np.float32)
    if n > 10:
        a, b = rng.choice(n, 2, replace=False)
        X[b] = (X[a] + rng.normal(0, 1e-3, d)).astype(np.float32)
    R2 = float(d)
    best, fr = ctx.points(_dev(X, torch_dev), R2=R2, precision=prec)
    _check_pair(best, oracle.closest_pair(X))
    _check_frnn(fr, oracle.frnn(X, R2))
    assert ctx.stats().max_err_over_bound <= 1.0


def test_radius_pairs_into_caller_owned_outputs(ctx, torch_dev):
    """`out=` hands the radius pairs to caller-owned tensors (no allocation
    in the call): the same pairs as the allocating call, for points and for
    windows; an output too small for the list raises the capacity error and
    reports the count."""
    import torch
    import paper_1407_5609_amd as cp
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (1500, 12)).astype(np.float32)
    Xd = _dev(X, torch_dev)
    best0, fr0 = ctx.points(Xd, R2=4.0, precision="bf16")
    m = len(fr0[0])
    assert m > 10
    out = (torch.full((m + 7, 2), -1, dtype=torch.int64, device=torch_dev),
           torch.full((m + 7,), -1.0, dtype=torch.float64, device=torch_dev))
    best1, fr1 = ctx.points(Xd, R2=4.0, precision="bf16", out=out)
    assert (best1.i, best1.j, best1.d2) == (best0.i, best0.j, best0.d2)
    assert fr1[0].data_ptr() == out[0].data_ptr() and fr1[1].data_ptr() == out[1].data_ptr()
    _check_frnn(fr1, (fr0[0].cpu().numpy(), fr0[1].cpu().numpy()))
    _check_frnn(fr1, oracle.frnn(X, 4.0))
    small = (torch.empty((m - 1, 2), dtype=torch.int64, device=torch_dev),
             torch.empty((m - 1,), dtype=torch.float64, device=torch_dev))
    with pytest.raises(cp.CpmiError, match="capacity"):
        ctx.points(Xd, R2=4.0, precision="bf16", out=small)
    with pytest.raises(ValueError):
        ctx.points(Xd, R2=4.0, out=(out[0].float(), out[1]))
    T = np.cumsum(rng.normal(0, 1, 3000)).astype(np.float32)
    Td = _dev(T, torch_dev)
    mb0, mf0 = ctx.motif(Td, 64, R2=9.0)
    k = len(mf0[0])
    out = (torch.empty((k + 3, 2), dtype=torch.int64, device=torch_dev),
           torch.empty((k + 3,), dtype=torch.float64, device=torch_dev))
    mb1, mf1 = ctx.motif(Td, 64, R2=9.0, out=out)
    assert (mb1.i, mb1.j, mb1.d2) == (mb0.i, mb0.j, mb0.d2)
    _check_frnn(mf1, (mf0[0].cpu().numpy(), mf0[1].cpu().numpy()))


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_points_strided_rows(ctx, torch_dev, prec):
    rng = np.random.default_rng(9)
    Xfull = rng.normal(0, 1, (600, 80)).astype(np.float32)
    X = Xfull[:, :70]                      # ld = 80 > d = 70
    import torch
    t = _dev(Xfull, torch_dev)[:, :70]
    assert t.stride(0) == 80
    best, fr = ctx.points(t, R2=70.0, precision=prec)
    Xc = np.ascontiguousarray(X)
    _check_pair(best, oracle.closest_pair(Xc))
    _check_frnn(fr, oracle.frnn(Xc, 70.0))


@pytest.mark.parametrize("n,d,R2", [(1, 3, 1.0), (2, 3, 0.0), (700, 6, 3.0), (5000, 8, 6.0)])
def test_neighbour_lists_match_oracle(ctx, torch_dev, n, d, R2):
    """Section 3.5's N(i) for every point: the radius pairs of the GPU search
    turned into compressed rows on the device equal the oracle's lists built
    from its own pairs (row pointers and columns bit for bit), also from the
    pairs in a shuffled order; isolated points have empty rows."""
    import torch
    rng = np.random.default_rng(n + d)
    X = rng.normal(0, 1, (max(n, 2), d)).astype(np.float32)
    if n >= 2:
        p, _ = ctx.frnn(_dev(X, torch_dev), R2, precision="bf16")
        want_pairs, _ = oracle.frnn(X, R2)
    else:
        p = torch.zeros((0, 2), dtype=torch.int64, device=torch_dev)
        want_pairs = np.zeros((0, 2), dtype=np.int64)
    want_rp, want_cols = oracle.neighbour_lists(want_pairs, n)
    rp, cols = ctx.pairs_to_csr(p, n)
    assert np.array_equal(rp.cpu().numpy(), want_rp)
    assert np.array_equal(cols.cpu().numpy(), want_cols)
    if p.shape[0] > 1:
        perm = torch.from_numpy(rng.permutation(p.shape[0])).to(torch_dev)
        rp2, cols2 = ctx.pairs_to_csr(p[perm].contiguous(), n)
        assert torch.equal(rp2, rp) and torch.equal(cols2, cols)


def test_neighbour_lists_refuse_bad_pairs(ctx, torch_dev):
    import torch
    import paper_1407_5609_amd as cp
    for bad in ([[0, 1], [2, 2]], [[0, 1], [3, 1]], [[-1, 2]], [[0, 5]]):
        t = torch.tensor(bad, dtype=torch.int64, device=torch_dev)
        with pytest.raises(cp.CpmiError) as e:
            ctx.pairs_to_csr(t, 5)
        assert e.value.code == cp.ERR_ARG
    with pytest.raises(cp.CpmiError):
        ctx.pairs_to_csr(torch.zeros((0, 2), dtype=torch.int64, device=torch_dev), 0)
    rp, cols = ctx.pairs_to_csr(torch.tensor([[1, 3]], dtype=torch.int64, device=torch_dev), 5)
    assert rp.tolist() == [0, 0, 1, 1, 2, 2] and cols.tolist() == [3, 1]


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_exact_ties_go_to_lexicographic_minimum(ctx, torch_dev, tile, prec):
    rng = np.random.default_rng(31)
    X = rng.integers(-50, 50, (900, 12)).astype(np.float32)
    # several exact duplicates: d2 = 0 ties, lexicographic minimum wins
    for a, b in [(700, 800), (5, 600), (5, 400), (300, 301)]:
        X[b] = X[a]
    best = ctx.closest_pair(_dev(X, torch_dev), precision=prec)
    assert (best.i, best.j, best.d2) == oracle.closest_pair(X) == (5, 400, 0.0)


def test_points_full_size_golden(ctx, torch_dev, tile):
    g = json.load(open(os.path.join(GOLDEN, "points_n4096_d64.json")))
    c = W.cfg_points_small()
    want_pair = (g["closest_pair"]["i"], g["closest_pair"]["j"], float.fromhex(g["closest_pair"]["d2"]))
    want_fr = (np.array(g["frnn"]["pairs"], dtype=np.int64).reshape(-1, 2),
               np.array([float.fromhex(v) for v in g["frnn"]["d2"]]))
    t = _dev(c["X"], torch_dev)
    for prec in ("f32", "bf16"):
        best, fr = ctx.points(t, R2=c["R2"], precision=prec)
        _check_pair(best, want_pair)
        _check_frnn(fr, want_fr)
        st = ctx.stats()
        assert st.valid_pairs == W.valid_pairs_points(4096)
        assert st.max_err_over_bound <= 1.0


@pytest.mark.parametrize("n,d", [(2, 1), (257, 33), (1500, 4096), (1100, 300)])
def test_int8_points_bit_exact(ctx, torch_dev, tile, n, d):
    rng = np.random.default_rng(n + d)
    if d == 4096:
        X = W.snp_matrix(rng, n, d)
        W.plant_snp_pairs(rng, X)
        R2 = 800
    else:
        X = rng.integers(-128, 128, (n, d)).astype(np.int8)
        R2 = int(2 * d * 5461 * 0.9)      # ~ lower tail of 2 d Var(U[-128,127])
    best, fr = ctx.points(_dev(X, torch_dev), R2=R2, precision="i8")
    oi, oj, od = oracle.closest_pair(X)
    assert (best.i, best.j, best.d2) == (oi, oj, float(od))
    _check_frnn(fr, oracle.frnn(X, R2))


# ---------------------------------------------------------------------------
# motifs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("length,ell,excl", [(700, 16, 0), (3000, 64, 0), (5000, 100, 50), (6000, 256, 0),
                                              (4500, 512, 0), (2100, 128, 1), (3001, 37, 0), (2500, 301, 0)])
def test_motif_matches_oracle(ctx, torch_dev, tile, prec, length, ell, excl):
    rng = np.random.default_rng(length + ell)
    T = W.random_walk(rng, length)
    W.plant_motif(rng, T, ell)
    R2 = 0.05 * ell
    best, fr = ctx.motif(_dev(T, torch_dev), ell, excl=excl, R2=R2, precision=prec)
    ob, ofr = oracle.motif(T, ell, excl=excl if excl > 0 else ell, R2=R2)
    _check_pair(best, ob)
    _check_frnn(fr, ofr)
    assert ctx.stats().max_err_over_bound <= 1.0


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_motif_exclusion_boundary_and_ties(ctx, torch_dev, tile, prec):
    P, ell = 37, 16
    rng = np.random.default_rng(15)
    T = np.tile(rng.normal(0, 1, P).astype(np.float32), 12)
    t = _dev(T, torch_dev)
    best, _ = ctx.motif(t, ell, excl=P, precision=prec)
    assert (best.i, best.j, best.d2) == (0, P, 0.0)
    best, _ = ctx.motif(t, ell, excl=P + 1, precision=prec)
    assert (best.i, best.j, best.d2) == (0, 2 * P, 0.0)
    _, fr = ctx.motif(t, ell, excl=P + 1, R2=0.0, precision=prec, want_pair=False)
    _check_frnn(fr, oracle.motif(T, ell, excl=P + 1, R2=0.0)[1])


def test_motif_full_size_golden(ctx, torch_dev, tile):
    g = json.load(open(os.path.join(GOLDEN, "motif_L65536_l256.json")))
    c = W.cfg_motif()
    want_pair = (g["closest_pair"]["i"], g["closest_pair"]["j"], float.fromhex(g["closest_pair"]["d2"]))
    want_fr = (np.array(g["frnn"]["pairs"], dtype=np.int64).reshape(-1, 2),
               np.array([float.fromhex(v) for v in g["frnn"]["d2"]]))
    t = _dev(c["T"], torch_dev)
    for prec in ("f32", "bf16"):
        best, fr = ctx.motif(t, c["ell"], excl=c["excl"], R2=c["R2"], precision=prec)
        _check_pair(best, want_pair)
        _check_frnn(fr, want_fr)
        st = ctx.stats()
        assert st.valid_pairs == W.valid_pairs_motif(65536, 256, 256)
        assert st.max_err_over_bound <= 1.0


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_motif_batch_matches_oracle(ctx, torch_dev, tile, prec):
    rng = np.random.default_rng(77)
    series, ells, plants = W.batch_series(rng, 20, 600, 4000, ells=(16, 37, 64, 128, 201, 256))
    ts = [_dev(T, torch_dev) for T in series]
    for rep in range(2):                    # second call replays the captured graph
        res = ctx.motif_batch(ts, ells, precision=prec)
        for s, (T, ell) in enumerate(zip(series, ells)):
            ob, _ = oracle.motif(T, ell)
            if ob is None:
                assert isinstance(res[s], Exception)
                continue
            _check_pair(res[s], ob)
    assert ctx.stats().valid_pairs == sum(W.valid_pairs_motif(len(T), e, e) for T, e in zip(series, ells))


@pytest.mark.parametrize("prec", ["f32", "bf16", "i8"])
def test_radius_boundary_is_inclusive_to_the_last_bit(ctx, torch_dev, tile, prec):
    """R^2 equal to a pair's canonical d^2 keeps that pair; the next double
    below drops it (the screen's thresholds carry the bound and a margin, the
    FP64 verifier decides)."""
    rng = np.random.default_rng(21)
    if prec == "i8":
        X = rng.integers(-3, 4, (900, 40), dtype=np.int8)
    else:
        X = rng.normal(0, 1, (900, 40)).astype(np.float32)
    P, D = oracle.frnn(X, float(np.inf))
    r2 = float(np.sort(D)[40])                     # the 41st smallest d^2 (ties at it included)
    at = {tuple(p) for p in P[D == r2].tolist()}
    for R2, inside in ((r2, True), (float(np.nextafter(r2, -np.inf)), False)):
        _, fr = ctx.points(_dev(X, torch_dev), R2=R2, precision=prec, want_pair=False)
        got = {tuple(p) for p in fr[0].cpu().numpy().tolist()}
        assert (at <= got) if inside else not (at & got), (R2, inside)
        _check_frnn(fr, oracle.frnn(X, R2))


def test_candidate_buffers_grow_and_the_answers_stay_exact(torch_dev):
    """More candidates than the internal buffers hold (closest-pair
    candidates 2^18, radius candidates 2^20 by default): the call grows them,
    runs again, and returns the exact answers (a fresh context, so the
    buffers start at their defaults)."""
    import paper_1407_5609_amd as cp
    c = cp.Context(0)
    try:
        # 1200 identical rows: all 719,400 pairs tie at d^2 = 0
        X = np.tile(np.random.default_rng(3).normal(0, 1, (1, 16)).astype(np.float32), (1200, 1))
        best, _ = c.points(_dev(X, torch_dev), precision="bf16")
        assert (best.i, best.j, best.d2) == (0, 1, 0.0)
        assert c.stats().reruns >= 1
        # every one of 1,279,200 pairs within the radius
        Y = np.random.default_rng(4).normal(0, 1, (1600, 8)).astype(np.float32)
        best, fr = c.points(_dev(Y, torch_dev), R2=1e9, precision="bf16", cap=1 << 21)
        assert c.stats().reruns >= 1
        _check_pair(best, oracle.closest_pair(Y))
        _check_frnn(fr, oracle.frnn(Y, 1e9))
        assert len(fr[0]) == 1600 * 1599 // 2
    finally:
        c.close()


# ---------------------------------------------------------------------------
# error paths (forced from the host; every kernel still exits normally)
# ---------------------------------------------------------------------------

def test_error_codes(ctx, torch_dev):
    import torch

    import paper_1407_5609_amd as cp
    X = np.random.default_rng(0).normal(size=(300, 8)).astype(np.float32)
    Xn = X.copy()
    Xn[123, 4] = np.nan
    with pytest.raises(cp.CpmiError) as e:
        ctx.closest_pair(_dev(Xn, torch_dev))
    assert e.value.code == cp.ERR_NONFINITE
    Xi = X.copy()
    Xi[7, 0] = np.inf
    with pytest.raises(cp.CpmiError) as e:
        ctx.frnn(_dev(Xi, torch_dev), 1.0, precision="f32")
    assert e.value.code == cp.ERR_NONFINITE
    with pytest.raises(cp.CpmiError) as e:
        ctx.closest_pair(_dev(X[:1], torch_dev))
    assert e.value.code == cp.ERR_NOPAIR
    with pytest.raises(cp.CpmiError) as e:
        ctx.closest_pair(_dev(X.astype(np.int8), torch_dev), precision="bf16")
    assert e.value.code == cp.ERR_ARG
    T = W.random_walk(np.random.default_rng(3), 500)
    T[100:200] = 5.0                        # constant windows: sigma = 0
    with pytest.raises(cp.CpmiError) as e:
        ctx.motif(_dev(T, torch_dev), 50)
    assert e.value.code == cp.ERR_DEGENERATE
    best, _ = ctx.motif(_dev(T[:90], torch_dev), 45)   # 46 windows, exclusion 45: exactly one pair
    assert (best.i, best.j) == (0, 45)
    T2 = W.random_walk(np.random.default_rng(4), 89)
    with pytest.raises(cp.CpmiError) as e:
        ctx.motif(_dev(T2, torch_dev), 45)       # 45 windows, exclusion 45 -> none
    assert e.value.code == cp.ERR_NOPAIR
    # capacity protocol: the first call reports the size needed
    import ctypes as C
    t = _dev(X, torch_dev)
    pairs = torch.empty((1, 2), dtype=torch.int64, device=torch_dev)
    d2 = torch.empty(1, dtype=torch.float64, device=torch_dev)
    cnt = C.c_int64(0)
    rc = cp._lib.cpmi_frnn(ctx._h, C.c_void_p(t.data_ptr()), cp.F32, 300, 8, 8, 16.0, cp.PREC_F32,
                           cp._stream_ptr(None), C.c_void_p(pairs.data_ptr()), C.c_void_p(d2.data_ptr()), 1,
                           C.byref(cnt))
    want = len(oracle.frnn(X, 16.0)[0])
    assert want > 1 and rc == cp.ERR_CAPACITY and cnt.value == want


def test_range_nonfinite_series_and_strided_int8(ctx, torch_dev):
    """Error paths the call contract names: a squared norm of 2^100 or more
    (too large for the FP32 screen) gives ERR_RANGE on both float screens; a
    NaN or an infinity inside a series gives ERR_NONFINITE from the motif
    search (single and batched); int8 rows with a stride larger than d give
    the oracle's exact answer."""
    import paper_1407_5609_amd as cp
    rng = np.random.default_rng(31)
    X = rng.normal(size=(700, 16)).astype(np.float32)
    X[333, 3] = np.float32(2.0 ** 51)                     # ||x||^2 = 2^102
    for prec in ("f32", "bf16"):
        with pytest.raises(cp.CpmiError) as e:
            ctx.closest_pair(_dev(X, torch_dev), precision=prec)
        assert e.value.code == cp.ERR_RANGE, prec
    X[333, 3] = np.float32(2.0 ** 49)                     # ||x||^2 ~ 2^98: accepted
    want = oracle.closest_pair(X)
    best = ctx.closest_pair(_dev(X, torch_dev), precision="f32")
    assert (best.i, best.j, best.d2) == want

    T = W.random_walk(rng, 3000)
    for bad in (np.nan, np.inf, -np.inf):
        Tb = T.copy()
        Tb[1717] = bad
        with pytest.raises(cp.CpmiError) as e:
            ctx.motif(_dev(Tb, torch_dev), 64)
        assert e.value.code == cp.ERR_NONFINITE, bad
        res = ctx.motif_batch([_dev(T, torch_dev), _dev(Tb, torch_dev)], [64, 64])
        assert isinstance(res[1], cp.CpmiError) and res[1].code == cp.ERR_NONFINITE, bad
        ob, _ = oracle.motif(T, 64)
        assert (res[0].i, res[0].j, res[0].d2) == ob

    G = rng.integers(0, 3, (1500, 200)).astype(np.int8)
    G[1200, :150] = G[40, :150]
    G[1200, 7] = (G[40, 7] + 1) % 3                        # d2 1 or 4 over the first 150 columns
    view = _dev(G, torch_dev)[:, :150]                     # rows of stride 200, d = 150
    assert view.stride(0) == 200
    Gv = np.ascontiguousarray(G[:, :150])
    best, (p, d) = ctx.points(view, R2=40.0, precision="i8")
    oi, oj, od = oracle.closest_pair(Gv)
    assert (best.i, best.j, best.d2) == (oi, oj, float(od))
    wp, wd = oracle.frnn(Gv, 40.0)
    assert np.array_equal(p.cpu().numpy(), wp) and np.array_equal(d.cpu().numpy(), wd.astype(np.float64))


def test_repeat_calls_are_deterministic(ctx, torch_dev):
    """The result sets are identical over 5 runs although the candidates
    reach their buffers in whatever order the atomics give: points with a
    radius that holds tens of thousands of pairs, a motif with a radius, and
    a batch of series."""
    rng = np.random.default_rng(4713)
    X = rng.normal(0, 1, (6000, 24)).astype(np.float32)
    tx = _dev(X, torch_dev)
    T = W.random_walk(rng, 20000)
    tt = _dev(T, torch_dev)
    series = [_dev(W.random_walk(rng, L), torch_dev) for L in (3000, 5000, 7000)]
    outs = []
    for _ in range(5):
        best, (p, d) = ctx.points(tx, R2=18.0, precision="bf16", cap=1 << 17)
        mb, (mp, md) = ctx.motif(tt, 64, R2=12.8, precision="bf16", cap=1 << 20)
        bb = ctx.motif_batch(series, [64, 128, 100])
        outs.append((best.i, best.j, best.d2, p.cpu().numpy().tobytes(), d.cpu().numpy().tobytes(),
                     mb.i, mb.j, mb.d2, mp.cpu().numpy().tobytes(), md.cpu().numpy().tobytes(),
                     tuple((q.i, q.j, q.d2) for q in bb)))
    assert len(np.frombuffer(outs[0][3], dtype=np.int64)) > 2 * 10_000
    assert all(o == outs[0] for o in outs[1:])


# ---------------------------------------------------------------------------
# autotuner and the traffic-calibration copy
# ---------------------------------------------------------------------------

def test_autotune_records_choices_and_answers_stay_exact(torch_dev, tmp_path):
    import paper_1407_5609_amd as cp
    c = cp.Context(0, tune_cache=None)
    try:
        rng = np.random.default_rng(77)
        X, plant = W.planted_gaussian_points(rng, 3000, 96, 1e-3)
        t = _dev(X, torch_dev)
        r = c.autotune(t, "auto", reps=1)
        assert set(r["ms"]) == {"f32/128", "f32/256", "bf16/128", "bf16/256"}
        assert all(v > 0 for v in r["ms"].values())
        best_key = f'{r["precision"]}/{r["tile"]}'
        assert r["ms"][best_key] == min(r["ms"].values())
        # later AUTO calls of this shape use the recorded choice, and stay exact
        pairs = 3000 * 2999 / 2
        p, tile = c.tune_lookup("f32", "auto", 96, pairs)
        assert ({1: "f32", 2: "bf16"}[p], tile) == (r["precision"], r["tile"])
        best = c.closest_pair(t, precision="auto")
        st = c.stats()
        assert (st.precision, st.tile) == (p, tile)
        _check_pair(best, oracle.closest_pair(X))
        # the band height of the tile order is timed where the 256 tile wins
        # (a larger problem), recorded per precision and saved with the rest
        import torch
        g = torch.Generator(device=torch_dev)
        g.manual_seed(5)
        Xb = torch.randn((65536, 32), generator=g, device=torch_dev)
        rb = c.autotune(Xb, "auto", reps=1)
        pb = 65536 * 65535 / 2
        timed = set()
        for pr in ("f32", "bf16"):
            bms = {k: v for k, v in rb["band_ms"].items() if k.startswith(pr + "/")}
            if not bms:
                assert c.tune_lookup("f32", pr, 32, pb)[1] == 128
                continue
            timed.add(pr)
            assert set(bms) == {f"{pr}/band4", f"{pr}/band8", f"{pr}/band16"} and all(v > 0 for v in bms.values())
            fastest = int(min(bms, key=bms.get).split("band")[1])
            assert c.tune_lookup_band(pr, 32, pb) == fastest
        assert timed, rb
        assert rb["band"] == (c.tune_lookup_band(rb["precision"], 32, pb) if rb["tile"] == 256 else 0)
        # the saved cache reproduces the choices in a new context
        path = str(tmp_path / "tune.json")
        c.save_tune_cache(path)
        c2 = cp.Context(0, tune_cache=path)
        assert c2.tune_lookup("f32", "auto", 96, pairs) == (p, tile)
        for pr in timed:
            assert c2.tune_lookup_band(pr, 32, pb) == c.tune_lookup_band(pr, 32, pb)
        c2.close()
        # int8 tunes the INT8 screen only
        Xi = rng.integers(0, 3, (1200, 200)).astype(np.int8)
        ri = c.autotune(_dev(Xi, torch_dev), "auto", reps=1)
        assert ri["precision"] == "i8" and set(ri["ms"]) == {"i8/128", "i8/256"}
    finally:
        c.close()


def test_batch_takes_each_series_band_from_the_tune_cache(torch_dev, tmp_path):
    """Tuned band heights are per (precision, K bucket, size bucket): in one
    batched call each series orders its tiles with the band of its own l and
    pair count, and every answer stays the oracle's."""
    import json
    import paper_1407_5609_amd as cp
    rng = np.random.default_rng(78)
    lens, ells = [9000, 7000, 12000, 6000], [64, 512, 64, 512]
    series = [W.random_walk(rng, L) for L in lens]
    plants = [W.plant_motif(rng, T, e) for T, e in zip(series, ells)]
    cache = {"auto:k64:r14": 2, "auto:k512:r14": 2, "bf16:k512:r16": 256, "bf16:k64:r16": 256}
    for e, b in ((64, 4), (512, 16)):
        for rb in range(8, 20):
            cache[f"band.bf16:k{e}:r{rb}"] = b
    path = str(tmp_path / "bands.json")
    json.dump(cache, open(path, "w"))
    c = cp.Context(0, tune_cache=path)
    d = cp.Context(0, tune_cache=None)
    try:
        for L, e in zip(lens, ells):
            pairs = W.valid_pairs_motif(L, e, e)
            assert c.tune_lookup_band("bf16", e, pairs) == (4 if e == 64 else 16)
            assert d.tune_lookup_band("bf16", e, pairs) == 8
        ts = [_dev(T, torch_dev) for T in series]
        got = c.motif_batch(ts, ells, precision="bf16")
        ref = d.motif_batch(ts, ells, precision="bf16")
        for T, e, plant, g, r in zip(series, ells, plants, got, ref):
            ob, _ = oracle.motif(T, e)
            assert (g.i, g.j, g.d2) == (r.i, r.j, r.d2) == ob
            assert (g.i, g.j) == plant
    finally:
        c.close()
        d.close()


def test_calibration_copy_moves_every_byte(torch_dev):
    import torch

    import paper_1407_5609_amd as cp
    src = torch.arange((1 << 20) + 4, dtype=torch.int32, device=torch_dev)
    dst = torch.full_like(src, -1)
    cp.dbg_copy(dst, src)
    assert torch.equal(dst, src)
    with pytest.raises(ValueError):
        cp.dbg_copy(dst[:-1], src)


# ---------------------------------------------------------------------------
# reference-point tile pruning (Section 3, MPR): same answers, fewer tiles
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("q,order", [(1, 0), (4, 0), (4, 1)])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_pruned_points_match_oracle(ctx, torch_dev, tile, prec, q, order):
    rng = np.random.default_rng(100 + q)
    X, _ = W.mixture_points(rng, 3000, 48)
    R2 = 30.0
    ctx.set_pruning(q, 10.0, seed=q)
    ctx.dbg_set_prune_order(order)
    try:
        best, fr = ctx.points(_dev(X, torch_dev), R2=R2, precision=prec)
        st = ctx.stats()
    finally:
        ctx.set_pruning(0)
        ctx.dbg_set_prune_order(0)
    _check_pair(best, oracle.closest_pair(X))
    _check_frnn(fr, oracle.frnn(X, R2))
    assert st.tiles_pruned > 0
    assert st.max_err_over_bound <= 1.0


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_pruned_ties_go_to_lexicographic_minimum_in_input_order(ctx, torch_dev, tile, prec):
    """Exact duplicates land anywhere in the reference order; the reported pair
    is still the lexicographically least in the caller's indices."""
    rng = np.random.default_rng(8)
    X, _ = W.mixture_points(rng, 2500, 32)
    for a, b in ((1700, 90), (2400, 90), (90, 600)):
        X[a] = X[b]
    ctx.set_pruning(3, 10.0, seed=5)
    try:
        best, fr = ctx.points(_dev(X, torch_dev), R2=0.0, precision=prec)
    finally:
        ctx.set_pruning(0)
    assert (best.i, best.j, best.d2) == oracle.closest_pair(X) == (90, 600, 0.0)
    _check_frnn(fr, oracle.frnn(X, 0.0))


def test_pruned_int8_and_frnn_only(ctx, torch_dev, tile):
    rng = np.random.default_rng(21)
    X = W.snp_matrix(rng, 1500, 512)
    W.plant_snp_pairs(rng, X, m=(2, 9, 30))
    ctx.set_pruning(4, 10.0)
    try:
        best = ctx.closest_pair(_dev(X, torch_dev), precision="i8")
        p, d = ctx.frnn(_dev(X, torch_dev), 40, precision="i8")
    finally:
        ctx.set_pruning(0)
    oi, oj, od = oracle.closest_pair(X)
    assert (best.i, best.j, best.d2) == (oi, oj, float(od))
    _check_frnn((p, d), oracle.frnn(X, 40))


@pytest.mark.parametrize("q,order", [(1, 0), (4, 0), (4, 1)])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("length,ell,excl", [(3000, 64, 0), (5000, 100, 50), (2100, 128, 1), (1300, 16, 0)])
def test_pruned_motif_matches_oracle(ctx, torch_dev, prec, q, order, length, ell, excl):
    """Windows in reference order (one reference, or buckets of one and the
    order of a second): the exclusion zone is applied to window positions,
    not screen rows; answers equal the oracle's."""
    rng = np.random.default_rng(length + ell + q)
    T = W.random_walk(rng, length)
    W.plant_motif(rng, T, ell)
    R2 = 0.05 * ell
    ctx.set_pruning(q, 10.0, seed=q)
    ctx.dbg_set_prune_order(order)
    try:
        best, fr = ctx.motif(_dev(T, torch_dev), ell, excl=excl, R2=R2, precision=prec)
        st = ctx.stats()
        best_only, _ = ctx.motif(_dev(T, torch_dev), ell, excl=excl, precision=prec)
    finally:
        ctx.set_pruning(0)
        ctx.dbg_set_prune_order(0)
    ob, ofr = oracle.motif(T, ell, excl=excl if excl > 0 else ell, R2=R2)
    _check_pair(best, ob)
    _check_pair(best_only, ob)
    _check_frnn(fr, ofr)
    assert st.tile == 256 and st.max_err_over_bound <= 1.0
    assert st.valid_pairs == W.valid_pairs_motif(length, ell, excl if excl > 0 else ell)


@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_pruned_motif_many_selected_tiles(ctx, torch_dev, prec):
    """Short windows and a wide radius: the second screen pass gets several
    selected tiles per work-group, so a work-group emits one tile while its
    waves have already prefetched the positions of the next ones; the
    radius pairs must still respect the exclusion zone and equal the
    oracle's."""
    rng = np.random.default_rng(32)
    T = W.random_walk(rng, 20000)
    ell, R2 = 32, 3.0
    ctx.set_pruning(4, 10.0, seed=3)
    try:
        best, fr = ctx.motif(_dev(T, torch_dev), ell, R2=R2, precision=prec)
        st = ctx.stats()
    finally:
        ctx.set_pruning(0)
    ob, ofr = oracle.motif(T, ell, R2=R2)
    _check_pair(best, ob)
    _check_frnn(fr, ofr)
    print("selected tiles", st.tiles_rescreened, "radius pairs", len(ofr[0]))
    assert st.tiles_rescreened > 300   # more than the 256 work-groups of the pass


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_pruned_motif_exclusion_boundary_and_ties(ctx, torch_dev, prec):
    """A periodic series: windows one period apart are identical, so the
    reference order puts whole runs of exact duplicates side by side; the
    exclusion zone (on positions) decides which of them may pair, and ties go
    to the lexicographic minimum in window positions."""
    P, ell = 37, 16
    rng = np.random.default_rng(15)
    T = np.tile(rng.normal(0, 1, P).astype(np.float32), 40)
    t = _dev(T, torch_dev)
    ctx.set_pruning(3, 10.0, seed=2)
    try:
        best, _ = ctx.motif(t, ell, excl=P, precision=prec)
        assert (best.i, best.j, best.d2) == (0, P, 0.0)
        best, _ = ctx.motif(t, ell, excl=P + 1, precision=prec)
        assert (best.i, best.j, best.d2) == (0, 2 * P, 0.0)
        _, fr = ctx.motif(t, ell, excl=P + 1, R2=0.0, precision=prec, want_pair=False)
    finally:
        ctx.set_pruning(0)
    _check_frnn(fr, oracle.motif(T, ell, excl=P + 1, R2=0.0)[1])


def test_pruned_motif_drops_tiles_on_a_random_walk(ctx, torch_dev):
    """Random walk of 20,000 samples, windows of 1,024 (the shapes the paper
    measures MPR on), q = 10, f = 10: tiles are dropped and the reported pair
    is admissible, its squared distance is the oracle's canonical value for
    that pair and no larger than the oracle's value for the planted pair."""
    rng = np.random.default_rng(5609)
    ell = 1024
    T = W.random_walk(rng, 20000)
    a, b = W.plant_motif(rng, T, ell, 0.01)
    ctx.set_pruning(10, 10.0, seed=1)
    try:
        best, _ = ctx.motif(_dev(T, torch_dev), ell, precision="bf16")
        st = ctx.stats()
    finally:
        ctx.set_pruning(0)
    assert best.j - best.i >= ell
    assert best.d2 == _window_d2(T, ell, best.i, best.j)
    assert best.d2 <= _window_d2(T, ell, a, b)
    assert st.tiles_pruned > 0
    print("pruned", st.tiles_pruned, "of", st.tiles_pruned + st.tiles_total, "tiles")


def _intervals(rng, nT, q, order):
    """Per-block distance intervals [nT, q] with the blocks in the order of
    reference 0 (order 0) or in buckets of reference 0 sorted by reference 1
    (order 1: reference 0 not monotone)."""
    lo = rng.uniform(0, 60, (nT, q))
    if order == 0:
        lo[:, 0] = np.sort(lo[:, 0])
    elif q >= 2:
        idx = np.lexsort((lo[:, 1], np.floor(lo[:, 0] / 6.0)))
        lo[:, :2] = lo[idx, :2]
    return lo, lo + rng.uniform(0.05, 3.0, (nT, q))


def _list_rule(n, tile, lo, hi, T, excl=1, permuted=False, G=8):
    """The pruned list written out: tiles I <= J with an admissible pair whose
    widened intervals (2^-34 |hi| on each side) come within T for every
    reference, in bands of G block rows (columns ascending, rows ascending);
    full tiles first, split into 8 chunks interleaved slot by slot (empty
    slots all ones), then the partial tiles."""
    nT = lo.shape[0]
    m = 2.0 ** -34 * np.abs(hi)
    lw, hw = lo - m, hi + m
    full, part = [], []
    for b0 in range(0, nT, G):
        for J in range(b0, nT):
            for I in range(b0, min(b0 + G, nT)):
                if I > J:
                    continue
                if not permuted and min(J * tile + tile - 1, n - 1) - I * tile < excl:
                    continue
                if T < 0 or np.any((lw[J] - hw[I] > T) | (lw[I] - hw[J] > T)):
                    continue
                e = (I << 22) | J
                isfull = (not permuted and J * tile - (I * tile + tile - 1) >= excl and (I + 1) * tile <= n
                          and (J + 1) * tile <= n)
                (full if isfull else part).append(e)
    C8 = (len(full) + 7) // 8
    slots = [2 ** 64 - 1] * (8 * C8)
    for s in range(8 * C8):
        src = (s % 8) * C8 + s // 8
        if src < len(full):
            slots[s] = full[src]
    return np.array(slots + part, dtype=np.uint64), 8 * C8, nT * (nT + 1) // 2 - len(full) - len(part)


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("edge", [128, 256])
@pytest.mark.parametrize("nT,q", [(1, 1), (5, 1), (37, 3), (140, 2)])
def test_pruned_list_on_the_device_is_the_interval_gap_rule(ctx, torch_dev, order, edge, nT, q):
    """The device-built list of the pruned searches (MPR's test of step 5 per
    tile, Section 3): the same entries in the same order as the rule written
    out, and as the host's list, for every threshold, both row orders, both
    tile edges, ragged last blocks, exclusion zones and windows in reference
    order (every tile partial)."""
    import ctypes as C
    import paper_1407_5609_amd as cp
    rng = np.random.default_rng(1000 * nT + 10 * q + order)
    lo, hi = _intervals(rng, nT, q, order)
    n = max(2, nT * edge - 17)
    hf = cp._lib.cpmi_dbg_pruned_tiles
    hf.restype = C.c_int64
    hf.argtypes = [C.c_int64, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_int64, C.c_void_p,
                   C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    for T in (-1.0, 0.0, 0.7, 2.5, 9.0, float("inf")):
        got, gnf, gnp = ctx.dbg_pruned_tiles_gpu(n, edge, lo, hi, T)
        want, wnf, wnp = _list_rule(n, edge, lo, hi, T)
        assert np.array_equal(got, want), (T, len(got), len(want))
        assert (gnf, gnp) == (wnf, wnp)
        hout = np.zeros(len(want) + 8, dtype=np.uint64)
        hnf, hnp = C.c_int64(0), C.c_int64(0)
        cnt = hf(n, edge, q, lo.ctypes.data, hi.ctypes.data, T, -1, hout.ctypes.data, len(hout), C.byref(hnf),
                 C.byref(hnp))
        assert np.array_equal(hout[:cnt], want) and (hnf.value, hnp.value) == (wnf, wnp)
        for excl, permuted in ((3 * edge // 2, False), (1, True)):
            got, gnf, gnp = ctx.dbg_pruned_tiles_gpu(n, edge, lo, hi, T, excl=excl, permuted=permuted)
            want, wnf, wnp = _list_rule(n, edge, lo, hi, T, excl=excl, permuted=permuted)
            assert np.array_equal(got, want), (T, excl, permuted)
            assert (gnf, gnp) == (wnf, wnp)


def test_pruned_list_on_the_device_at_size(ctx, torch_dev):
    """1,024 blocks (the 262,144-point mixture at edge 256): 524,800 tiles in
    66,048 segments, several scan blocks; equal to the rule (vectorised)."""
    rng = np.random.default_rng(5)
    nT, q, edge = 1024, 2, 256
    lo, hi = _intervals(rng, nT, q, 1)
    n = nT * edge
    T = 4.0
    got, gnf, gnp = ctx.dbg_pruned_tiles_gpu(n, edge, lo, hi, T)
    m = 2.0 ** -34 * np.abs(hi)
    lw, hw = lo - m, hi + m
    far = np.zeros((nT, nT), dtype=bool)
    for k in range(q):
        far |= (lw[None, :, k] - hw[:, None, k] > T) | (lw[:, None, k] - hw[None, :, k] > T)
    I, J = np.nonzero(np.triu(~far))
    kept = {(int(i), int(j)) for i, j in zip(I, J)}
    real = got[got != np.uint64(2 ** 64 - 1)]
    gotset = {(int(e >> np.uint64(22)) & 0x3FFFFF, int(e) & 0x3FFFFF) for e in real}
    assert len(real) == len(gotset) == len(kept) and gotset == kept
    assert gnp == nT * (nT + 1) // 2 - len(kept)
    full = [(i, j) for i, j in kept if i != j]
    assert gnf == 8 * ((len(full) + 7) // 8)


def test_pruning_arguments(ctx):
    import paper_1407_5609_amd as cp
    for q, f in ((-1, 10.0), (33, 10.0), (2, 0.0), (2, float("nan"))):
        with pytest.raises(cp.CpmiError):
            ctx.set_pruning(q, f)
    ctx.set_pruning(0)
    for order, w in ((2, 2.0), (-1, 2.0), (0, 0.0), (0, float("inf"))):
        with pytest.raises(cp.CpmiError):
            ctx.dbg_set_prune_order(order, w)
    ctx.dbg_set_prune_order(0)


@pytest.mark.parametrize("prec,published", [("bf16", 2500.0), ("f32", 157.3), ("i8", 5000.0)])
def test_sustained_matrix_core_rate_is_below_the_published_peak(torch_dev, prec, published):
    """The rate probe reported beside the published peak: positive, a sizeable
    share of the datasheet figure, never above it."""
    import paper_1407_5609_amd as cp
    rate, ms = cp.dbg_mfma_peak(prec, iters=2000)
    print(prec, "sustained", round(rate, 1), "of", published, "in", round(ms, 3), "ms")
    assert ms > 0 and 0.2 * published < rate <= 1.02 * published
