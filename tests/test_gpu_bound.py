"""GPU: the screen bound on the hardware, over every element of sampled tiles.

The screen is exact only if |D~ - d2_c| <= E for every pair, where D~ is the
matrix-core screen value, d2_c the canonical squared distance and E the
per-tile bound of the screen (gamma_K at unit 2^-23 for the FP32 accumulation
of the matrix cores, operand rounding, epilogue and FP64 terms). Here the
real screen kernel writes D~ for every element of seeded tiles (about 10^6
pairs per configuration, tiles drawn at random, diagonal and ragged ones
included), the oracle computes d2_c for each, and the ratio must stay <= 1.
The verifier's own d2 for the same pairs must equal the oracle's bit for bit.
Adversarial rows aim at the accumulation assumption: large common offsets
(D~ a small difference of large terms), long K, alternating large terms,
and a wide exponent range.
"""
import numpy as np
import pytest
import torch  # noqa: F401

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

RATIOS = {}


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
    if RATIOS:
        print("\nlargest |screen - d2| / bound per case:")
        for k, v in sorted(RATIOS.items()):
            print(f"  {k}: {v:.4g}")


def _tiles(rng, rows, tile, count):
    """`count` distinct (I, J) block pairs with I <= J: the last (ragged) block
    row and a diagonal tile always included."""
    nT = (rows + tile - 1) // tile
    out = {(nT - 1, nT - 1), (0, 0), (0, nT - 1)}
    while len(out) < min(count, nT * (nT + 1) // 2):
        I, J = sorted(int(v) for v in rng.integers(0, nT, 2))
        out.add((I, J))
    return sorted(out)


def _check(ctx, name, src, rows_fn, tiles, tile, prec, ell=None):
    """rows_fn(a0, na, b0, nb) -> oracle d2 block. Returns the ratio."""
    dump, d2, bounds, lib_ratio = ctx.dbg_screen_sample(src, tiles, tile, precision=prec, ell=ell)
    dump = dump.cpu().numpy().astype(np.float64)
    d2 = d2.cpu().numpy()
    rows = rows_fn(None, None, None, None)
    worst = 0.0
    for t, (I, J) in enumerate(tiles):
        a0, b0 = I * tile, J * tile
        na, nb = min(tile, rows - a0), min(tile, rows - b0)
        want = rows_fn(a0, na, b0, nb)
        got = d2[t, :na, :nb]
        assert np.array_equal(got, want), (name, I, J)            # verifier == oracle, bit for bit
        assert np.isnan(d2[t, na:, :]).all() and np.isnan(d2[t, :, nb:]).all()
        err = np.abs(dump[t, :na, :nb] - want)
        if prec == "i8":
            assert bounds[t] == 0.0 and err.max() == 0.0, (name, I, J)
            continue
        assert bounds[t] > 0.0
        r = float(err.max() / bounds[t])
        assert r <= 1.0, (name, I, J, r)
        worst = max(worst, r)
    if prec != "i8":
        # the library's own maximum agrees (it rounds the ratio up to float)
        assert worst <= lib_ratio <= np.nextafter(np.float32(max(worst, 1e-30)), np.float32(np.inf)) * (1 + 1e-6)
    RATIOS[f"{name}/{prec}/{tile}"] = worst
    return worst


def _points_rows(X):
    def f(a0, na, b0, nb):
        if a0 is None:
            return X.shape[0]
        return oracle.block_d2(X, a0, na, b0, nb)
    return f


def _window_rows(T, ell):
    Xhat, _, _ = oracle.znorm(T, ell)
    return _points_rows(Xhat)


@pytest.mark.parametrize("prec,tile", [("bf16", 256), ("f32", 256), ("bf16", 128), ("f32", 128)])
def test_bound_points_small(ctx, torch_dev, prec, tile):
    c = W.cfg_points_small()
    X = c["X"]
    rng = np.random.default_rng(9001)
    tiles = _tiles(rng, X.shape[0], tile, 1_048_576 // (tile * tile))
    _check(ctx, "points_n4096_d64", torch.from_numpy(X).to(torch_dev), _points_rows(X), tiles, tile, prec)


@pytest.fixture(scope="module")
def mixture(torch_dev):
    c = W.cfg_mixture()
    return c["X"], torch.from_numpy(c["X"]).to(torch_dev)


@pytest.mark.parametrize("prec,tile,count", [("bf16", 256, 16), ("f32", 256, 4), ("bf16", 128, 16)])
def test_bound_mixture_full_size(ctx, mixture, prec, tile, count):
    X, t = mixture
    rng = np.random.default_rng(9002)
    tiles = _tiles(rng, X.shape[0], tile, count)
    _check(ctx, "mixture_n262144_d512", t, _points_rows(X), tiles, tile, prec)


@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_bound_motif_full_size(ctx, torch_dev, prec):
    c = W.cfg_motif()
    T, ell = c["T"], c["ell"]
    rng = np.random.default_rng(9003)
    rows = T.shape[0] - ell + 1
    tiles = _tiles(rng, rows, 256, 16)
    _check(ctx, "motif_L65536_l256", torch.from_numpy(T).to(torch_dev), _window_rows(T, ell), tiles, 256, prec,
           ell=ell)


def test_bound_batch_series(ctx, torch_dev):
    c = W.cfg_batch()
    rng = np.random.default_rng(9004)
    seen = set()
    for s in range(len(c["series"])):
        T, ell = c["series"][s], int(c["ells"][s])
        if ell in seen:
            continue
        seen.add(ell)
        rows = T.shape[0] - ell + 1
        tiles = _tiles(rng, rows, 256, 4)
        _check(ctx, f"batch_series{s}_l{ell}", torch.from_numpy(T).to(torch_dev), _window_rows(T, ell), tiles,
               256, "bf16", ell=ell)
    assert seen == {64, 128, 256, 512}


def test_bound_int8_is_exact(ctx, torch_dev):
    rng = np.random.default_rng(9005)
    X = W.snp_matrix(rng, 6000, 4096)
    tiles = _tiles(rng, X.shape[0], 256, 4)
    _check(ctx, "snp_n6000_d4096", torch.from_numpy(X).to(torch_dev), _points_rows(X), tiles, 256, "i8")


def _adversarial(kind, rng):
    if kind == "offset_d64":          # D~ a small difference of large terms
        return (1000.0 + rng.normal(0, 1, (700, 64))).astype(np.float32)
    if kind == "offset_d4096":        # the same over a long K
        return (300.0 + rng.normal(0, 1, (600, 4096))).astype(np.float32)
    if kind == "alternating_d2048":   # large terms of both signs, near-equal rows
        s = rng.choice([-1.0, 1.0], 2048) * 512.0
        return (s + rng.normal(0, 1e-2, (600, 2048))).astype(np.float32)
    if kind == "wide_exponents_d256":  # 2^-30 .. 2^30 within a row
        return (rng.normal(0, 1, (600, 256)) * np.exp2(rng.integers(-30, 31, (600, 256)))).astype(np.float32)
    if kind == "near_duplicates_d512":  # many pairs at the rounding level of the operands
        base = rng.normal(0, 1, (40, 512))
        return (np.repeat(base, 15, axis=0) + rng.normal(0, 1e-6, (600, 512))).astype(np.float32)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["offset_d64", "offset_d4096", "alternating_d2048", "wide_exponents_d256",
                                  "near_duplicates_d512"])
@pytest.mark.parametrize("prec,tile", [("bf16", 256), ("f32", 256), ("f32", 128)])
def test_bound_adversarial(ctx, torch_dev, kind, prec, tile):
    rng = np.random.default_rng(9100 + ["offset_d64", "offset_d4096", "alternating_d2048", "wide_exponents_d256",
                                        "near_duplicates_d512"].index(kind))
    X = _adversarial(kind, rng)
    nT = (X.shape[0] + tile - 1) // tile
    tiles = [(I, J) for I in range(nT) for J in range(I, nT)]
    _check(ctx, kind, torch.from_numpy(X).to(torch_dev), _points_rows(X), tiles, tile, prec)


@pytest.mark.parametrize("prec,d,dpad", [("bf16", 64, 128), ("f32", 32, 64), ("f32", 96, 128), ("i8", 100, 250)])
def test_rows_of_two_slice_pairs_screen_like_zero_padded_rows(ctx, torch_dev, prec, d, dpad):
    """Rows of 4k + 2 K slices of the 256-tile screen (its K2 form, whose
    tiles start at either half of the load ring) give the same screen value in
    every element as the same rows zero-padded by the caller to a whole number
    of ring turns (the form without K2): the padding adds exact zero products.
    600 listed tiles, so that most work-groups screen two or three of them in a
    row and the ring stage alternates between tiles. The verifier's canonical
    d2 of every pair is the same too (appended zeros add +0 to each term sum).
    """
    import torch
    rng = np.random.default_rng(d * 7 + dpad)
    n = 256 * 40
    if prec == "i8":
        X = rng.integers(0, 3, (n, d)).astype(np.int8)
    else:
        X = rng.normal(0, 1, (n, d)).astype(np.float32)
    Xp = np.zeros((n, dpad), dtype=X.dtype)
    Xp[:, :d] = X
    tiles = _tiles(rng, n, 256, 600)
    assert len(tiles) == 600
    src = torch.from_numpy(X).to(torch_dev)
    srcp = torch.from_numpy(Xp).to(torch_dev)
    dump, d2, _, _ = ctx.dbg_screen_sample(src, tiles, 256, precision=prec)
    dump_p, d2_p, _, _ = ctx.dbg_screen_sample(srcp, tiles, 256, precision=prec)
    assert torch.equal(dump, dump_p)
    assert torch.equal(torch.nan_to_num(d2, nan=-1.0), torch.nan_to_num(d2_p, nan=-1.0))
