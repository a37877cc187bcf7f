"""GPU: radius searches at volume, through the C ABI, against the oracle.

Section 3.5's output (every pair within R) can hold billions of pairs. The
library counts them in 64 bits; past the largest list one call returns it
counts them without storing them (pairs proved inside by the screen value
alone are counted, the band within the screening bound of R2 is verified in
FP64). The counts must equal the oracle's exactly.
"""
import numpy as np
import pytest
import torch  # noqa: F401

import oracle

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def big(torch_dev):
    """100,000 points in the plane: 4,999,950,000 pairs, more than 2^32."""
    rng = np.random.default_rng(3505)
    X = rng.normal(0, 1, (100_000, 2)).astype(np.float32)
    return X, torch.from_numpy(X).to(torch_dev)


def test_count_beyond_32_bits(ctx, big):
    X, t = big
    n = X.shape[0]
    want = n * (n - 1) // 2
    assert want > 2 ** 32
    for prec in ("f32", "bf16"):
        got = ctx.frnn_count(t, 1e30, precision=prec)
        assert got == want, prec
        assert ctx.stats().frnn_pairs == want


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_counting_form_matches_the_oracle(ctx, big, prec):
    # about a fifth of the pairs inside (d2 of two N(0, I_2) points is
    # 2 chi^2_2: P(d2 <= R2) = 1 - exp(-R2 / 4)), far more than one call
    # stores, so the band within the screening bound of R2 is verified
    X, t = big
    R2 = 0.892
    want = oracle.frnn_count(X, R2)
    assert want > 2 ** 28
    assert ctx.frnn_count(t, R2, precision=prec) == want


def test_capacity_query_then_full_list(ctx, torch_dev):
    """The two-call protocol at a volume that one call returns: the count of
    the first call (no room) is the length of the second call's exact list."""
    import torch
    rng = np.random.default_rng(3506)
    X = rng.normal(0, 1, (3000, 4)).astype(np.float32)
    R2 = 1.5
    t = torch.from_numpy(X).to(torch_dev)
    cnt = ctx.frnn_count(t, R2, precision="bf16")
    pairs, d2 = ctx.frnn(t, R2, precision="bf16", cap=cnt)
    wp, wd = oracle.frnn(X, R2)
    assert cnt == len(wp) > 10_000
    assert np.array_equal(pairs.cpu().numpy(), wp)
    assert np.array_equal(d2.cpu().numpy(), wd)


@pytest.mark.parametrize("prec,q", [("bf16", 0), ("f32", 0), ("bf16", 4)])
def test_window_radius_at_volume(ctx, torch_dev, prec, q):
    """z-normalised windows (12,000-sample walk, l = 64) with a radius that
    holds 457,249 pairs: the window verifier takes its candidates 16 to a
    work-group in many rounds; the motif, the list and every d2 equal the
    oracle's bit for bit, unpruned and with reference-point pruning."""
    import workloads as W
    rng = np.random.default_rng(4711)
    T = W.random_walk(rng, 12000)
    ell, R2 = 64, 12.8
    Xhat, _, _ = oracle.znorm(T, ell)
    want_best = oracle.closest_pair_lanes(Xhat, ell)
    wp, wd = oracle.frnn(Xhat, R2, ell, lanes=True)
    assert len(wp) == 457249
    t = torch.from_numpy(T).to(torch_dev)
    ctx.set_pruning(q, 10.0, seed=2)
    try:
        best, (p, d) = ctx.motif(t, ell, R2=R2, precision=prec, cap=1 << 20)
    finally:
        ctx.set_pruning(0)
    assert (best.i, best.j, best.d2) == tuple(want_best)
    assert np.array_equal(p.cpu().numpy(), wp)
    assert np.array_equal(d.cpu().numpy(), wd)


@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_window_count_beyond_one_list(ctx, torch_dev, prec):
    """z-normalised windows have d2 = 2l(1 - rho) <= 4l: with R2 above that,
    every admissible pair of a 40,000-sample walk (l = 16) is within the
    radius, 798,780,465 of them, more than one call stores. The count from
    the call with no room for pairs is exact (pairs proved inside by the
    screen are counted, the band near R2 verified)."""
    import ctypes as C
    import paper_1407_5609_amd as cp
    import workloads as W
    rng = np.random.default_rng(4712)
    T = W.random_walk(rng, 40000)
    ell = 16
    want = W.valid_pairs_motif(40000, ell, ell)
    assert want > 2 ** 28
    t = torch.from_numpy(T).to(torch_dev)
    cnt = C.c_int64(0)
    best = cp._CPair()
    rc = cp._lib.cpmi_motif(ctx._h, C.c_void_p(t.data_ptr()), 40000, ell, 0, cp._prec(prec), 4.0 * ell + 1.0,
                            cp._stream_ptr(None), C.byref(best), None, None, 0, C.byref(cnt))
    assert rc == cp.ERR_CAPACITY
    assert cnt.value == want
    assert ctx.stats().frnn_pairs == want
