"""GPU parity of the string problems (Sections 5 and 6) against the oracle.

cpmi_strings_pair (most and least correlated pair of strings over a small
alphabet) and cpmi_two_locus (the SNP pair of the two-locus association
problem) run as exact INT8 matrix-core searches over encoded rows; the pair
and its match count must equal the oracle's, which computes them by brute
force (the least correlated pair and the two-locus pair through the paper's
code/complement matrices, written independently).
"""
import numpy as np
import pytest
import torch  # noqa: F401

import oracle
import workloads as W

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


def _dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("mode", ["most", "least"])
@pytest.mark.parametrize("sigma,n,k", [(2, 300, 64), (3, 1000, 40), (4, 2100, 17), (4, 513, 1), (3, 2, 9),
                                       (5, 777, 130)])
def test_strings_pair_matches_oracle(ctx, torch_dev, mode, sigma, n, k):
    rng = np.random.default_rng(sigma * 1000 + n + k)
    S = W.random_strings(rng, n, k, sigma)
    if n > 10 and k > 4:
        W.plant_string_pair(rng, S, sigma, k - 2 if mode == "most" else 1)
    r = ctx.strings_pair(_dev(S, torch_dev), sigma, mode)
    assert (r.i, r.j, r.matches) == oracle.strings_pair(S, sigma, mode), (r, mode)
    assert r.length == k
    st = ctx.stats()
    assert st.valid_pairs == n * (n - 1) // 2


@pytest.mark.parametrize("mode", ["most", "least"])
def test_strings_pair_ties_go_to_the_first_pair(ctx, torch_dev, mode):
    """Many exact ties (duplicated strings; strings with no agreeing position):
    the lexicographically first pair is reported."""
    rng = np.random.default_rng(9)
    S = W.random_strings(rng, 700, 12, 3)
    for a, b in ((400, 650), (20, 600), (20, 30), (5, 300)):
        S[b] = S[a] if mode == "most" else (S[a] + 1) % 3
    r = ctx.strings_pair(_dev(S, torch_dev), 3, mode)
    assert (r.i, r.j, r.matches) == oracle.strings_pair(S, 3, mode)


def test_strings_pair_strided_rows(ctx, torch_dev):
    rng = np.random.default_rng(4)
    S = W.random_strings(rng, 600, 50, 4)
    t = _dev(S, torch_dev)[:, 3:40]          # row stride 50, 37 columns
    for mode in ("most", "least"):
        r = ctx.strings_pair(t, 4, mode)
        assert (r.i, r.j, r.matches) == oracle.strings_pair(np.ascontiguousarray(S[:, 3:40]), 4, mode)


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("m1,m2,n", [(200, 200, 1500), (37, 90, 700), (5, 3, 300), (200, 200, 2)])
def test_two_locus_matches_oracle(ctx, torch_dev, direction, m1, m2, n):
    rng = np.random.default_rng(m1 + m2 + n + direction)
    G = rng.integers(0, 3, (m1 + m2, n), dtype=np.int8)
    if n > 2:
        W.inject_two_locus_pair(rng, G, m1, int(0.8 * m1), int(0.5 * m2), levels=3)
    r = ctx.two_locus(_dev(G, torch_dev), m1, m2, direction)
    assert (r.i, r.j, r.matches) == oracle.two_locus(G, m1, m2, direction), r
    assert r.length == 3 * (m1 + m2)


def test_two_locus_noise_data_finds_the_injected_pair(ctx, torch_dev):
    """The paper's injection run: NOISE genotypes (200 cases, 200 controls),
    one pair with p = 0.8, q = 0.5 (D-column correlation 0.6)."""
    rng = np.random.default_rng(6)
    G = W.noise_genotypes(rng, 200, 200, 3000)
    a, b = W.inject_two_locus_pair(rng, G, 200, 160, 100)
    r = ctx.two_locus(_dev(G, torch_dev), 200, 200)
    assert (r.i, r.j, r.matches) == oracle.two_locus(G, 200, 200, 0)
    assert (r.i, r.j) == (a, b) and r.matches == 200 + 2 * 160 + 2 * (200 - 100)


def test_string_errors(ctx, torch_dev):
    import paper_1407_5609_amd as cp
    S = np.zeros((10, 4), dtype=np.int8)
    S[3, 2] = 5
    with pytest.raises(cp.CpmiError) as e:
        ctx.strings_pair(_dev(S, torch_dev), 4, "most")
    assert e.value.code == cp.ERR_ARG
    with pytest.raises(cp.CpmiError) as e:
        ctx.strings_pair(_dev(np.zeros((1, 4), np.int8), torch_dev), 4, "least")
    assert e.value.code == cp.ERR_NOPAIR
    G = np.zeros((6, 8), dtype=np.int8)
    G[1, 1] = 3
    with pytest.raises(cp.CpmiError) as e:
        ctx.two_locus(_dev(G, torch_dev), 3, 3)
    assert e.value.code == cp.ERR_ARG
    with pytest.raises(cp.CpmiError):
        ctx.strings_pair(_dev(np.zeros((10, 4), np.int8), torch_dev), 1, "most")   # sigma < 2
    # the context still works after the errors
    r = ctx.strings_pair(_dev(np.array([[0, 1], [0, 1], [1, 0]], np.int8), torch_dev), 2, "most")
    assert (r.i, r.j, r.matches) == (0, 1, 2)


# ---------------------------------------------------------------------------
# randomised light-bulb bucketing (Section 4, MLBA)
# ---------------------------------------------------------------------------

def test_lightbulb_finds_the_planted_most_correlated_pair(ctx, torch_dev):
    """A pair agreeing in 58 of 64 positions among 5,000 random strings over 4
    letters: with 8 random columns it shares a bucket in an iteration with
    probability (58/64)^8 = 0.45, so 24 iterations find it (the exact best
    pair) and collect far fewer pairs than the n(n-1)/2 of brute force."""
    rng = np.random.default_rng(41)
    S = W.random_strings(rng, 5000, 64, 4)
    a, b = W.plant_string_pair(rng, S, 4, 58)
    want = oracle.strings_pair(S, 4, "most")
    assert want[:2] == (a, b)
    r, pairs = ctx.strings_lightbulb(_dev(S, torch_dev), 4, "most", iterations=24, columns=8, seed=7)
    assert (r.i, r.j, r.matches) == want
    assert 0 < pairs < 5000 * 4999 // 2 // 100
    # the same seed gives the same run
    r2, pairs2 = ctx.strings_lightbulb(_dev(S, torch_dev), 4, "most", iterations=24, columns=8, seed=7)
    assert (r2.i, r2.j, r2.matches, pairs2) == (r.i, r.j, r.matches, pairs)


def test_lightbulb_finds_the_least_correlated_binary_pair(ctx, torch_dev):
    """Binary strings (Section 5's light bulbs): a pair disagreeing everywhere
    makes a code and the other's complement identical, so it shares a bucket
    in every iteration."""
    rng = np.random.default_rng(42)
    S = W.random_strings(rng, 3000, 64, 2)
    W.plant_string_pair(rng, S, 2, 0)
    want = oracle.strings_pair(S, 2, "least")
    r, pairs = ctx.strings_lightbulb(_dev(S, torch_dev), 2, "least", iterations=4, columns=20, seed=1)
    assert (r.i, r.j, r.matches) == want
    assert pairs > 0


@pytest.mark.parametrize("mode,sigma,columns", [("most", 3, 4), ("least", 3, 12), ("most", 5, 3)])
def test_lightbulb_reports_exact_counts(ctx, torch_dev, mode, sigma, columns):
    """Whatever pairs the random buckets yield, the reported pair's count is
    its exact one and never beats the exact optimum."""
    rng = np.random.default_rng(sigma + columns)
    S = W.random_strings(rng, 800, 24, sigma)
    r, pairs = ctx.strings_lightbulb(_dev(S, torch_dev), sigma, mode, iterations=6, columns=columns, seed=3)
    assert 0 <= r.i < r.j < 800
    assert r.matches == oracle.matches(S, r.i, r.j)
    best = oracle.strings_pair(S, sigma, mode)[2]
    assert r.matches <= best if mode == "most" else r.matches >= best


def test_lightbulb_errors(ctx, torch_dev):
    import paper_1407_5609_amd as cp
    S = _dev(np.zeros((100, 8), np.int8), torch_dev)
    with pytest.raises(cp.CpmiError):
        ctx.strings_lightbulb(S, 4, "most", columns=33)          # 33 x 2 bits > 64
    with pytest.raises(cp.CpmiError):
        ctx.strings_lightbulb(S, 4, "most", iterations=0)
    with pytest.raises(cp.CpmiError) as e:
        ctx.strings_lightbulb(S, 4, "most", columns=2, cap=10)   # identical strings: one bucket of 100
    assert e.value.code == cp.ERR_CAPACITY
    r, pairs = ctx.strings_lightbulb(S, 4, "most", columns=2, cap=10000)
    assert (r.i, r.j, r.matches) == (0, 1, 8) and pairs == 100 * 99 // 2 * 16
    # a match count of k or more than 22 bits would not fit the packed best pair
    import torch
    L = torch.zeros((2, 1 << 22), dtype=torch.int8, device=torch_dev)
    with pytest.raises(cp.CpmiError) as e:
        ctx.strings_lightbulb(L, 2, "most", columns=4)
    assert e.value.code == cp.ERR_ARG and "2^22" in ctx.last_error()


@pytest.mark.parametrize("mode,n,k,sigma,iterations,columns,seed", [
    ("most", 900, 24, 4, 16, 6, 7),       # one batch, keys tagged with the iteration
    ("most", 500, 20, 4, 1, 4, 9),        # a single iteration: plain sort, no tag
    ("most", 300, 12, 4, 300, 5, 3),      # two batches (at most 256 iterations each)
    ("most", 400, 40, 4, 6, 32, 5),       # 64 key bits: no room for the tag, segmented sort
    ("least", 300, 16, 2, 40, 12, 11),    # codes against complements (600 rows)
    ("least", 250, 10, 3, 5, 8, 2),       # 8 of the 30 bits of the codes of three-letter strings
])
def test_lightbulb_candidates_match_oracle(ctx, torch_dev, mode, n, k, sigma, iterations, columns, seed):
    """The candidates collected over all iterations (the paper's work measure)
    and the best candidate equal the oracle's MLBA with the same column draw
    (SplitMix64 on both sides, each written from its published definition)."""
    rng = np.random.default_rng(500 + n + k)
    S = W.random_strings(rng, n, k, sigma)
    W.plant_string_pair(rng, S, sigma, k - 1 if mode == "most" else 0)
    for r in range(5):                                    # a few near-duplicates: real buckets
        S[10 + r] = S[200 + r]
        S[10 + r, r % k] = (S[10 + r, r % k] + 1) % sigma
    want_total, want_best = oracle.lightbulb(S, sigma, mode, iterations, columns, seed)
    got, pairs = ctx.strings_lightbulb(_dev(S, torch_dev), sigma, mode, iterations=iterations, columns=columns,
                                       seed=seed)
    assert pairs == want_total
    assert want_best is not None and (got.i, got.j, got.matches) == want_best
