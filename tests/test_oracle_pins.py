"""Pins for the CPU oracle: it is checked here against things other than itself.

The paper prints no distance values, pair indices or neighbour sets for the
Euclidean path, so the oracle is pinned by mathematics and construction:

* exact rational arithmetic on tiny inputs (the brute-force ground truth the
  paper uses to verify answers, Section 6.1);
* special cases that reduce to textbook routines: d=1 (sort + adjacent gaps),
  d=2 (divide-and-conquer closest pair, the O(n log n) algorithm cited in the
  introduction), scipy's pdist;
* planted pairs whose answer is known by construction (the injection
  methodology of Section 6.1);
* invariants: symmetry, exclusion zone, radius monotonicity, permutation and
  power-of-two scaling, z-normalisation identities, the int8 Gram identity.

A plausible mistake in the oracle (a dropped term, a wrong sign or index, a
sample instead of population variance, an off-by-one exclusion, the wrong tie
order) fails at least one test here.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.spatial.distance as ssd

import oracle
import workloads as W

U64 = 2.0 ** -53


def gamma(m):
    return m * U64 / (1 - m * U64)


def exact_d2(x, y):
    return sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(x, y))


# --------------------------------------------------------------------------
# exact rationals
# --------------------------------------------------------------------------

def _tiny_sets():
    rng = np.random.default_rng(101)
    out = []
    for n, d in [(12, 3), (20, 5), (24, 8), (16, 16)]:
        X = rng.normal(0, 1, (n, d)).astype(np.float32)
        X[3] = X[7]                                    # exact duplicate -> d2 = 0
        X[5] = X[2]
        X[5, 0] = np.nextafter(X[2, 0], np.float32(np.inf))  # last-ulp difference
        out.append(X)
    # wide dynamic range
    X = (rng.normal(0, 1, (18, 4)) * np.exp2(rng.integers(-20, 20, (18, 4)))).astype(np.float32)
    out.append(X)
    return out


@pytest.mark.parametrize("X", _tiny_sets())
def test_d2_against_exact_rationals(X):
    n, d = X.shape
    tol = gamma(d + 2)
    for i, j in itertools.combinations(range(n), 2):
        ex = exact_d2(X[i], X[j])
        got = oracle.d2(X, i, j)
        if ex == 0:
            assert got == 0.0
        else:
            assert abs(Fraction(got) - ex) <= Fraction(tol) * ex, (i, j)


@pytest.mark.parametrize("X", _tiny_sets())
def test_closest_pair_and_frnn_against_exact_enumeration(X):
    n, d = X.shape
    exact = {(i, j): exact_d2(X[i], X[j]) for i, j in itertools.combinations(range(n), 2)}
    best_val = min(exact.values())
    bi, bj, bd2 = oracle.closest_pair(X)
    tol = Fraction(gamma(d + 2))
    # the oracle's winner is an exact minimiser up to the rounding bound ...
    assert exact[(bi, bj)] <= best_val * (1 + 2 * tol)
    # ... and wherever the exact minimum is separated, it is the same pair
    second = sorted(set(exact.values()))
    if len(second) > 1 and second[1] > best_val * (1 + 4 * tol):
        winners = sorted(k for k, v in exact.items() if v == best_val)
        assert (bi, bj) == winners[0]
    # FRNN at a radius placed between two well-separated exact values
    vals = sorted(exact.values())
    gaps = [(vals[k + 1] - vals[k]) / vals[k + 1] for k in range(len(vals) // 3, len(vals) - 1)]
    k = len(vals) // 3 + int(np.argmax(gaps))
    R2 = float((vals[k] + vals[k + 1]) / 2)
    pairs, _ = oracle.frnn(X, R2)
    want = sorted(p for p, v in exact.items() if v <= Fraction(R2))
    assert [tuple(p) for p in pairs] == want


def test_exact_ties_go_to_lexicographic_minimum():
    # integer coordinates: every d2 is exact in double, so ties are exact
    X = np.array([[5, 5], [9, 9], [0, 0], [6, 5], [1, 0], [20, 20], [21, 20]], dtype=np.float32)
    # pairs at d2=1: (0,3), (2,4), (5,6) -> lexicographic minimum is (0,3)
    assert oracle.closest_pair(X) == (0, 3, 1.0)
    Xp = X[[2, 4, 0, 3, 1, 5, 6]]        # now the tied pairs are (0,1), (2,3), (5,6)
    assert oracle.closest_pair(Xp) == (0, 1, 1.0)


# --------------------------------------------------------------------------
# special cases reducing to textbook routines
# --------------------------------------------------------------------------

def test_one_dimension_is_sorted_adjacent_gap():
    rng = np.random.default_rng(7)
    x = rng.normal(0, 1, 3000).astype(np.float32)
    X = x.reshape(-1, 1)
    order = np.argsort(x, kind="stable")
    xs = x[order].astype(np.float64)
    gaps = np.diff(xs)                      # exact: differences of nearby float32 values
    k = int(np.argmin(gaps))
    assert np.count_nonzero(gaps == gaps[k]) == 1
    i, j = sorted((int(order[k]), int(order[k + 1])))
    bi, bj, bd2 = oracle.closest_pair(X)
    assert (bi, bj) == (i, j)
    assert bd2 == gaps[k] * gaps[k]
    # fixed radius in 1-D by a sorted sweep
    R = 1e-3
    pairs, _ = oracle.frnn(X, R * R)
    want = set()
    for a in range(len(xs)):
        b = a + 1
        while b < len(xs) and (xs[b] - xs[a]) * (xs[b] - xs[a]) <= R * R:
            want.add(tuple(sorted((int(order[a]), int(order[b])))))
            b += 1
    assert set(map(tuple, pairs.tolist())) == want


def _closest_pair_dc(P):
    """Divide-and-conquer closest pair in the plane (exact rationals)."""
    pts = sorted(P, key=lambda p: (p[0], p[1]))

    def rec(lo, hi):
        if hi - lo <= 3:
            best = (None, None)
            for a in range(lo, hi):
                for b in range(a + 1, hi):
                    v = (pts[a][0] - pts[b][0]) ** 2 + (pts[a][1] - pts[b][1]) ** 2
                    if best[0] is None or v < best[0]:
                        best = (v, (pts[a][2], pts[b][2]))
            return best
        mid = (lo + hi) // 2
        xm = pts[mid][0]
        l, r = rec(lo, mid), rec(mid, hi)
        best = l if r[0] is None or (l[0] is not None and l[0] <= r[0]) else r
        strip = sorted((p for p in pts[lo:hi] if (p[0] - xm) ** 2 < best[0]), key=lambda p: p[1])
        for a in range(len(strip)):
            for b in range(a + 1, len(strip)):
                if (strip[b][1] - strip[a][1]) ** 2 >= best[0]:
                    break
                v = (strip[a][0] - strip[b][0]) ** 2 + (strip[a][1] - strip[b][1]) ** 2
                if v < best[0]:
                    best = (v, (strip[a][2], strip[b][2]))
        return best

    return rec(0, len(pts))


def test_two_dimensions_against_divide_and_conquer():
    rng = np.random.default_rng(11)
    X = rng.uniform(-100, 100, (2500, 2)).astype(np.float32)
    P = [(Fraction(float(a)), Fraction(float(b)), k) for k, (a, b) in enumerate(X)]
    v, (a, b) = _closest_pair_dc(P)
    bi, bj, bd2 = oracle.closest_pair(X)
    assert (bi, bj) == tuple(sorted((a, b)))
    assert abs(Fraction(bd2) - v) <= Fraction(gamma(4)) * v


def test_against_scipy_pdist():
    rng = np.random.default_rng(3)
    X, plant = W.planted_gaussian_points(rng, 1500, 64, 1e-3)
    ref = ssd.squareform(ssd.pdist(X.astype(np.float64), "sqeuclidean"))
    for i in (0, 17, plant[0], 1499):
        row = oracle.row_d2(X, i)
        np.testing.assert_allclose(row, ref[i], rtol=1e-12, atol=0)
    iu = np.triu_indices(1500, 1)
    flat = ref[iu]
    k = int(np.argmin(flat))
    assert oracle.closest_pair(X)[:2] == (int(iu[0][k]), int(iu[1][k]))
    R2 = 64.0
    pairs, d2 = oracle.frnn(X, R2)
    sel = flat <= R2
    margin = np.min(np.abs(flat - R2) / R2)
    assert margin > 1e-10
    assert np.array_equal(pairs, np.stack([iu[0][sel], iu[1][sel]], 1))
    np.testing.assert_allclose(d2, flat[sel], rtol=1e-12)


def test_nearest_neighbour_against_scipy_and_duplicates():
    """Per-point nearest-neighbour squared distance (used to derive the
    mixture workload's radius): scipy's FP64 distances give the same minimum
    per row, duplicated rows give exactly 0, and a point's own distance is
    never taken."""
    rng = np.random.default_rng(5)
    X, _ = W.mixture_points(rng, 700, 48)
    X[10] = X[300]                                        # an exact duplicate
    nn = oracle.nearest_neighbour_d2(X)
    ref = ssd.squareform(ssd.pdist(X.astype(np.float64), "sqeuclidean"))
    np.fill_diagonal(ref, np.inf)
    np.testing.assert_allclose(nn, ref.min(axis=1), rtol=1e-12, atol=0)
    assert nn[10] == 0.0 and nn[300] == 0.0
    assert np.all(nn[np.arange(700) != 10][:299] > 0)
    # a single point apart from the rest has its own nearest neighbour, not itself
    Y = np.zeros((3, 4), np.float32)
    Y[1, 0] = 1.0
    Y[2, 0] = 3.0
    assert oracle.nearest_neighbour_d2(Y).tolist() == [1.0, 1.0, 4.0]


# --------------------------------------------------------------------------
# planted answers (known by construction)
# --------------------------------------------------------------------------

def test_planted_points_full_size():
    c = W.cfg_points_small()
    i, j, d2 = oracle.closest_pair(c["X"])
    assert (i, j) == c["plant"]
    assert d2 < 1e-3                      # 64 coords of N(0, 1e-3) noise
    pairs, _ = oracle.frnn(c["X"], c["R2"])
    assert tuple(c["plant"]) in set(map(tuple, pairs.tolist()))


def test_planted_motif_small_series():
    rng = np.random.default_rng(21)
    T = W.random_walk(rng, 8192)
    plant = W.plant_motif(rng, T, 256)
    best, _ = oracle.motif(T, 256)
    assert best[:2] == plant
    assert best[2] < 0.05


def test_planted_mixture_small():
    rng = np.random.default_rng(5)
    X, plant = W.mixture_points(rng, 3000, 512, plant_dist=1e-2)
    i, j, d2 = oracle.closest_pair(X)
    assert (i, j) == plant
    assert abs(math.sqrt(d2) - 1e-2) < 1e-4   # float32 rounding of the planted row


def test_planted_snp_pairs_small():
    rng = np.random.default_rng(8)
    X = W.snp_matrix(rng, 1500, 4096)
    plants = W.plant_snp_pairs(rng, X)
    best = oracle.closest_pair(X)
    assert best == (plants[0][0], plants[0][1], 3)
    pairs, d2 = oracle.frnn(X, 800)
    assert sorted(map(tuple, pairs.tolist())) == sorted((a, b) for a, b, _ in plants)
    got = {tuple(p): int(v) for p, v in zip(pairs.tolist(), d2)}
    for a, b, m in plants:
        assert got[(a, b)] == m


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------

def test_symmetry_is_bitwise():
    rng = np.random.default_rng(4)
    X = rng.normal(0, 3, (200, 37)).astype(np.float32)
    for i, j in rng.integers(0, 200, (300, 2)):
        assert oracle.d2(X, i, j) == oracle.d2(X, j, i)


def test_power_of_two_scaling_is_exact():
    rng = np.random.default_rng(12)
    X = rng.normal(0, 1, (300, 24)).astype(np.float32)
    base = oracle.closest_pair(X)
    for k in (-3, 5):
        Y = (X * np.float32(2.0 ** k)).astype(np.float32)
        got = oracle.closest_pair(Y)
        assert got[:2] == base[:2]
        assert got[2] == base[2] * 4.0 ** k
        assert oracle.d2(Y, 3, 9) == oracle.d2(X, 3, 9) * 4.0 ** k


def test_permutation_maps_the_answer():
    rng = np.random.default_rng(13)
    X = rng.normal(0, 1, (700, 16)).astype(np.float32)
    i, j, d2 = oracle.closest_pair(X)
    perm = rng.permutation(700)
    inv = np.argsort(perm)
    pi, pj, pd2 = oracle.closest_pair(X[perm])
    assert tuple(sorted((int(inv[i]), int(inv[j])))) == (pi, pj)
    assert pd2 == d2


def test_frnn_radius_monotone_and_contains_closest_pair():
    rng = np.random.default_rng(14)
    X = rng.normal(0, 1, (600, 8)).astype(np.float32)
    i, j, dmin = oracle.closest_pair(X)
    at, _ = oracle.frnn(X, dmin)
    assert [tuple(p) for p in at] == [(i, j)] or (i, j) in set(map(tuple, at.tolist()))
    below, _ = oracle.frnn(X, float(np.nextafter(dmin, 0.0)))
    assert len(below) == 0
    prev = set()
    for R2 in (1.0, 2.0, 4.0, 6.0):
        cur = set(map(tuple, oracle.frnn(X, R2)[0].tolist()))
        assert prev <= cur
        prev = cur


def test_exclusion_zone_boundary():
    # period-P series: windows i and i+P are identical, so d2(i, i+P) == 0.
    P, ell = 37, 16
    rng = np.random.default_rng(15)
    base = rng.normal(0, 1, P).astype(np.float32)
    T = np.tile(base, 12)
    best, _ = oracle.motif(T, ell, excl=P)
    assert best == (0, P, 0.0)
    best, _ = oracle.motif(T, ell, excl=P + 1)
    assert best == (0, 2 * P, 0.0)
    _, (pairs, _) = oracle.motif(T, ell, excl=P + 1, R2=0.0)
    assert np.all(pairs[:, 1] - pairs[:, 0] >= P + 1)
    assert len(pairs) > 0 and np.all((pairs[:, 1] - pairs[:, 0]) % P == 0)


def test_znorm_against_numpy_and_identities():
    rng = np.random.default_rng(16)
    T = W.random_walk(rng, 3000)
    ell = 128
    Xhat, mu, sg = oracle.znorm(T, ell)
    win = np.lib.stride_tricks.sliding_window_view(T.astype(np.float64), ell)
    np.testing.assert_allclose(mu, win.mean(axis=1), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sg, win.std(axis=1, ddof=0), rtol=1e-12)   # population sigma
    np.testing.assert_allclose(Xhat.sum(axis=1), 0.0, atol=1e-9)
    np.testing.assert_allclose((Xhat ** 2).sum(axis=1), ell, rtol=1e-12)
    # d2 = 2 l (1 - rho) with rho the Pearson correlation of the raw windows
    for i, j in [(0, 500), (10, 2000), (1234, 2870), (77, 78)]:
        rho = np.corrcoef(win[i], win[j])[0, 1]
        assert abs(oracle.d2(Xhat, i, j) - 2 * ell * (1 - rho)) <= 1e-10 * ell


def test_znorm_power_of_two_invariance_is_bitwise():
    rng = np.random.default_rng(17)
    T = W.random_walk(rng, 1500)
    a, mu, sg = oracle.znorm(T, 64)
    b, mu2, sg2 = oracle.znorm((T * np.float32(8.0)).astype(np.float32), 64)
    assert np.array_equal(a, b)
    assert np.array_equal(mu2, mu * 8) and np.array_equal(sg2, sg * 8)


def test_znorm_zero_variance_is_reported():
    T = np.concatenate([np.ones(50, np.float32), np.arange(50, dtype=np.float32)])
    with pytest.raises(ValueError):
        oracle.znorm(T, 20)


def test_int8_gram_identity_and_float_agreement():
    rng = np.random.default_rng(18)
    X = W.snp_matrix(rng, 300, 512)
    Xi = X.astype(np.int64)
    s = (Xi * Xi).sum(1)
    G = Xi @ Xi.T
    for i, j in rng.integers(0, 300, (200, 2)):
        assert oracle.d2(X, i, j) == s[i] + s[j] - 2 * G[i, j]
    assert oracle.closest_pair(X)[:2] == oracle.closest_pair(X.astype(np.float32))[:2]
    a, da = oracle.frnn(X, 700)
    b, db = oracle.frnn(X.astype(np.float32), 700.0)
    assert np.array_equal(a, b) and np.array_equal(da, db.astype(np.int64))


def test_no_admissible_pair():
    X = np.zeros((1, 4), np.float32)
    assert oracle.closest_pair(X) is None
    T = W.random_walk(np.random.default_rng(1), 40)
    best, _ = oracle.motif(T, 20)       # 21 windows, exclusion 20: one admissible pair
    assert best[:2] == (0, 20)
    best, _ = oracle.motif(T, 21)       # 20 windows, exclusion 21: none
    assert best is None


# ---------------------------------------------------------------------------
# strings and correlation by matches (Sections 5 and 6)
# ---------------------------------------------------------------------------

def test_matches_worked_example():
    """Section 5's example: x = 10010 and y = 00111 agree in 2 positions."""
    S = np.array([[1, 0, 0, 1, 0], [0, 0, 1, 1, 1]], dtype=np.int8)
    assert oracle.matches(S, 0, 1) == 2


def test_mapping_codes_and_their_matches():
    """Section 5's alphabet {001, 010, 100}: 0 -> 001, 1 -> 010, 2 -> 100; two
    codes agree in 3 bits if equal and 1 otherwise; a code and a complement
    agree in 0 bits if the symbols are equal and 2 otherwise."""
    S = np.array([[0], [1], [2]], dtype=np.int8)
    A = oracle.encode(S, 3)
    assert A.tolist() == [[0, 0, 1], [0, 1, 0], [1, 0, 0]]
    Ac = oracle.encode(S, 3, complement=True)
    assert np.array_equal(Ac, 1 - A)
    for x in range(3):
        for y in range(3):
            assert oracle.bit_matches(A, A, x, y) == (3 if x == y else 1)
            assert oracle.bit_matches(A, Ac, x, y) == (0 if x == y else 2)


@pytest.mark.parametrize("sigma", [2, 3, 4, 7])
def test_mapping_identities(sigma):
    """M(A'_i, A'_j) = k + 2 u_ij and M(A'_i, ~A'_j) = 2 (k - u_ij) for the
    three-letter mapping (Section 5); for sigma letters the first becomes
    (sigma - 2) k + 2 u_ij (equal symbols agree in sigma bits, different ones
    in sigma - 2) and the second is unchanged."""
    rng = np.random.default_rng(sigma)
    S = W.random_strings(rng, 30, 25, sigma)
    k = S.shape[1]
    A, Ac = oracle.encode(S, sigma), oracle.encode(S, sigma, complement=True)
    for i in range(30):
        for j in range(30):
            u = int((S[i] == S[j]).sum())
            assert oracle.matches(S, i, j) == u
            assert oracle.bit_matches(A, A, i, j) == (sigma - 2) * k + 2 * u
            assert oracle.bit_matches(A, Ac, i, j) == 2 * (k - u)


def test_transformed_correlations():
    """Section 5's run-time analysis: with p = u / k, the mapped correlation of
    two codes is 1/3 + 2p/3 and of a code and a complement (2/3)(1 - p)."""
    from fractions import Fraction as F
    rng = np.random.default_rng(3)
    S = W.random_strings(rng, 20, 33, 3)
    k = S.shape[1]
    A, Ac = oracle.encode(S, 3), oracle.encode(S, 3, complement=True)
    for i in range(20):
        for j in range(20):
            p = F(oracle.matches(S, i, j), k)
            assert F(oracle.bit_matches(A, A, i, j), 3 * k) == F(1, 3) + F(2, 3) * p
            assert F(oracle.bit_matches(A, Ac, i, j), 3 * k) == F(2, 3) * (1 - p)


def _brute_pair(S, better):
    """Lexicographically first pair i < j whose u = m(S_i, S_j) is best."""
    n = S.shape[0]
    best = None
    for i in range(n):
        for j in range(i + 1, n):
            u = int((S[i] == S[j]).sum())
            if best is None or better(u, best[2]):
                best = (i, j, u)
    return best


@pytest.mark.parametrize("sigma,n,k", [(2, 40, 16), (3, 50, 12), (4, 35, 9), (3, 2, 5)])
def test_strings_pair_against_brute_force(sigma, n, k):
    """The most correlated pair equals the plain argmax of u (and the closest
    pair of the one-hot rows, whose squared distance is 2 (k - u)); the least
    correlated pair found through codes and complements equals the plain
    argmin of u, ties to the first pair."""
    rng = np.random.default_rng(n + k)
    S = W.random_strings(rng, n, k, sigma)
    if n > 3:
        S[n // 2] = S[1]                 # a duplicate: a tie candidate for the most
        W.plant_string_pair(rng, S, sigma, 0)
    most = oracle.strings_pair(S, sigma, "most")
    assert most == _brute_pair(S, lambda u, b: u > b)
    ci, cj, cd2 = oracle.closest_pair(oracle.encode(S, sigma))
    assert (ci, cj) == most[:2] and cd2 == 2 * (k - most[2])
    assert oracle.strings_pair(S, sigma, "least") == _brute_pair(S, lambda u, b: u < b)


def _brute_two_locus(G, m1, direction):
    """Lexicographically first SNP pair i < j maximising u_A - u_B (direction
    0) or u_B - u_A, with u the subjects in which the two SNPs agree."""
    n = G.shape[1]
    best = None
    for i in range(n):
        for j in range(i + 1, n):
            same = G[:, i] == G[:, j]
            uA, uB = int(same[:m1].sum()), int(same[m1:].sum())
            v = uA - uB if direction == 0 else uB - uA
            if best is None or v > best[2]:
                best = (i, j, v)
    return best


@pytest.mark.parametrize("m1,m2,n,direction", [(20, 20, 40, 0), (20, 20, 40, 1), (13, 25, 30, 0), (9, 4, 2, 1)])
def test_two_locus_against_brute_force(m1, m2, n, direction):
    """Section 6: the columns (i, n + j) of D agree in m1 + 2 u_A + 2 (m2 - u_B)
    bits (direction 0), so the pair with the most agreeing bits is the pair
    maximising u_A - u_B."""
    rng = np.random.default_rng(m1 * 100 + n + direction)
    G = rng.integers(0, 3, (m1 + m2, n), dtype=np.int8)
    i, j, m = oracle.two_locus(G, m1, m2, direction)
    bi, bj, v = _brute_two_locus(G, m1, direction)
    assert (i, j) == (bi, bj)
    assert m == m1 + 2 * m2 + 2 * v if direction == 0 else m == m2 + 2 * m1 + 2 * v


def test_two_locus_correlation_identity():
    """Section 6: with as many cases as controls, the correlation of columns i
    and n + j of D is 1/2 + (p - q)/3, p and q the fractions of cases and of
    controls in which SNPs i and j agree."""
    from fractions import Fraction as F
    rng = np.random.default_rng(504)
    m = 30
    G = rng.integers(0, 3, (2 * m, 12), dtype=np.int8)
    A = oracle.encode(np.ascontiguousarray(G[:m].T), 3)
    B = oracle.encode(np.ascontiguousarray(G[m:].T), 3)
    Bc = oracle.encode(np.ascontiguousarray(G[m:].T), 3, complement=True)
    D1 = np.concatenate([A, B], axis=1)
    D2 = np.concatenate([A, Bc], axis=1)
    for i in range(12):
        for j in range(12):
            same = G[:, i] == G[:, j]
            p, q = F(int(same[:m].sum()), m), F(int(same[m:].sum()), m)
            assert F(oracle.bit_matches(D1, D2, i, j), 6 * m) == F(1, 2) + (p - q) / 3


# --------------------------------------------------------------------------
# light-bulb bucketing (Section 4, MLBA): the draw and the candidates
# --------------------------------------------------------------------------

def test_splitmix64_published_test_vector():
    """SplitMix64's reference stream from state 1234567 (the test vector of
    its published reference implementation): output k is the output for
    state 1234567 + k golden."""
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
            16408922859458223821]
    state = 1234567
    got = []
    for _ in want:
        got.append(oracle.splitmix64(state))
        state = (state + 0x9E3779B97F4A7C15) % (1 << 64)
    assert got == want


def test_lightbulb_columns_are_distinct_draws():
    cols = oracle.lightbulb_columns(5, 40, 9, 30)
    assert len(cols) == 40
    for c in cols:
        assert len(set(c)) == 9 and all(0 <= v < 30 for v in c)
    assert cols != oracle.lightbulb_columns(6, 40, 9, 30)
    # every column turns up: the draw covers the range
    assert set(itertools.chain.from_iterable(cols)) == set(range(30))
    # drawing all columns gives a permutation
    assert sorted(oracle.lightbulb_columns(3, 1, 30, 30)[0]) == list(range(30))


def _pairs_in(counts):
    return sum(c * (c - 1) // 2 for c in counts)


def test_lightbulb_all_columns_buckets_identical_strings():
    """With every position drawn the buckets are the classes of identical
    strings: candidates = sum of C(multiplicity, 2) per iteration, and the
    best pair agrees everywhere."""
    rng = np.random.default_rng(41)
    S = W.random_strings(rng, 60, 6, 3)
    S[7] = S[3]
    S[40] = S[3]
    S[21] = S[50]
    mult = {}
    for r in S:
        mult[r.tobytes()] = mult.get(r.tobytes(), 0) + 1
    total, best = oracle.lightbulb(S, 3, "most", 3, 6, seed=2)
    assert total == 3 * _pairs_in(mult.values())
    assert best == (3, 7, 6)


def test_lightbulb_one_column_is_a_histogram():
    """One drawn column: the buckets are that column's symbol classes."""
    rng = np.random.default_rng(42)
    S = W.random_strings(rng, 50, 9, 4)
    for seed in range(3):
        (col,), = oracle.lightbulb_columns(seed, 1, 1, 9)
        total, best = oracle.lightbulb(S, 4, "most", 1, 1, seed)
        assert total == _pairs_in(np.bincount(S[:, col], minlength=4))
        # the best candidate by brute force over the pairs sharing that symbol
        pool = [(oracle.matches(S, i, j), i, j) for i in range(50) for j in range(i + 1, 50) if S[i, col] == S[j, col]]
        u, i, j = max(pool, key=lambda t: (t[0], -t[1], -t[2]))
        assert best == (i, j, u)


def test_lightbulb_least_against_brute_force():
    """Least correlated: a candidate is a string i whose code agrees on the
    drawn bits with the complement of a string j != i. Brute force over all
    ordered (i, j) per iteration, from the codes written out directly."""
    rng = np.random.default_rng(43)
    n, k, sigma, c, its = 14, 5, 3, 4, 5
    S = W.random_strings(rng, n, k, sigma)
    X = np.zeros((n, sigma * k), dtype=np.int64)     # Section 5's order: symbol 0 -> 0..01
    for i in range(n):
        for p in range(k):
            X[i, p * sigma + sigma - 1 - S[i, p]] = 1
    total, cands = 0, set()
    for cols in oracle.lightbulb_columns(9, its, c, sigma * k):
        for i in range(n):
            for j in range(n):
                if i != j and all(X[i, b] == 1 - X[j, b] for b in cols):
                    total += 1
                    cands.add((min(i, j), max(i, j)))
    got_total, got_best = oracle.lightbulb(S, sigma, "least", its, c, 9)
    assert got_total == total
    u, i, j = min(((sum(S[a] == S[b]), a, b) for a, b in cands), key=lambda t: (t[0], t[1], t[2]))
    assert got_best == (i, j, int(u))


# --------------------------------------------------------------------------
# the lane-parallel closest pair (used for the large batch's expected values)
# --------------------------------------------------------------------------

def _lane_cases():
    rng = np.random.default_rng(7)
    out = []
    for n, d, excl in [(2, 1, 1), (3, 5, 1), (9, 2, 1), (37, 7, 3), (64, 16, 64), (65, 16, 64), (130, 33, 1),
                       (257, 65, 40), (300, 128, 128), (1001, 12, 500)]:
        X = rng.normal(0, 1, (n, d))
        if n > 10:
            X[n // 3] = X[n // 2]                            # an exact duplicate
            X[n - 1] = X[1]                                  # a second one, later in the order
        out.append((X, excl))
    # integer coordinates: exact ties at d2 = 1, first of them must win
    X = np.array([[5, 5], [9, 9], [0, 0], [6, 5], [1, 0], [20, 20], [21, 20]], dtype=np.float64)
    out.append((X, 1))
    out.append((np.ascontiguousarray(X[::-1]), 1))
    return out


@pytest.mark.parametrize("case", range(len(_lane_cases())))
def test_lanes_closest_pair_equals_the_plain_loop(case):
    X, excl = _lane_cases()[case]
    assert oracle.closest_pair_lanes(X, excl) == oracle.closest_pair(X, excl)


def test_lanes_closest_pair_on_windows_and_strides():
    rng = np.random.default_rng(8)
    T = W.random_walk(rng, 3000)
    for ell in (16, 64, 100):
        Xhat, _, _ = oracle.znorm(T, ell)
        assert oracle.closest_pair_lanes(Xhat, ell) == oracle.closest_pair(Xhat, ell)
        assert oracle.motif(T, ell, lanes=True) == oracle.motif(T, ell)
    big = rng.normal(0, 1, (200, 40))
    view = big[:, :33]                                        # rows with a stride larger than d
    assert oracle.closest_pair_lanes(view, 2) == oracle.closest_pair(np.ascontiguousarray(view), 2)
    assert oracle.closest_pair_lanes(rng.normal(0, 1, (5, 3)), 5) is None


def test_frnn_count_against_scipy_and_closed_form():
    """The pair count of a radius: scipy's pdist counted at the same squared
    radius (away from ties), n(n-1)/2 above the largest distance, and the
    exclusion zone removing exactly the pairs with j - i < excl."""
    rng = np.random.default_rng(15)
    X = rng.normal(0, 1, (700, 5)).astype(np.float32)
    d2 = ssd.pdist(X.astype(np.float64), "sqeuclidean")
    for R2 in (2.0, 6.5, 11.0):
        assert oracle.frnn_count(X, R2) == int(np.count_nonzero(d2 <= R2))
        assert oracle.frnn_count(X, R2) == len(oracle.frnn(X, R2)[0])
    n = X.shape[0]
    assert oracle.frnn_count(X, 1e30) == n * (n - 1) // 2
    assert oracle.frnn_count(X, 1e30, excl=10) == (n - 10) * (n - 9) // 2
    assert oracle.frnn_count(X, -1.0) == 0


def test_block_d2_is_the_pairwise_distance():
    rng = np.random.default_rng(16)
    X = rng.normal(0, 1, (50, 9)).astype(np.float32)
    B = oracle.block_d2(X, 3, 20, 30, 17)
    ref = ssd.cdist(X[3:23].astype(np.float64), X[30:47].astype(np.float64), "sqeuclidean")
    assert np.allclose(B, ref, rtol=1e-13, atol=0)
    assert B[5, 7] == oracle.d2(X, 8, 37)
    G = rng.integers(0, 3, (40, 33)).astype(np.int8)
    Bi = oracle.block_d2(G, 0, 40, 0, 40)
    Gi = G.astype(np.int64)
    assert np.array_equal(Bi, ((Gi[:, None, :] - Gi[None, :, :]) ** 2).sum(-1).astype(np.float64))


@pytest.mark.parametrize("case", range(len(_lane_cases())))
def test_lanes_radius_list_equals_the_plain_loop(case):
    X, excl = _lane_cases()[case]
    if X.shape[0] < 3:
        return
    d2 = ssd.pdist(X, "sqeuclidean")
    for R2 in (0.0, float(np.quantile(d2, 0.1)), float(np.quantile(d2, 0.5)), 1e300):
        a = oracle.frnn(X, R2, excl)
        b = oracle.frnn(X, R2, excl, lanes=True)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_neighbour_lists_are_the_other_points_within_the_radius():
    """Section 3.5's output N(i): from the radius pairs, every point's list
    equals the brute-force set {j != i : d2(i, j) <= R2} of scipy's full
    distance matrix (margin checked), ascending; the lists are symmetric and
    hold 2m entries; isolated points have empty rows; an empty pair list gives
    empty rows; a pair outside 0 <= i < j < n is refused."""
    rng = np.random.default_rng(17)
    X = rng.normal(0, 1, (300, 4)).astype(np.float32)
    D = ssd.squareform(ssd.pdist(X.astype(np.float64), "sqeuclidean"))
    for R2 in (0.5, 2.0):
        off = D[~np.eye(300, dtype=bool)]
        assert np.min(np.abs(off - R2)) / R2 > 1e-10
        pairs, _ = oracle.frnn(X, R2)
        row_ptr, cols = oracle.neighbour_lists(pairs, 300)
        assert row_ptr[0] == 0 and row_ptr[-1] == 2 * len(pairs) == len(cols)
        for v in range(300):
            want = [j for j in range(300) if j != v and D[v, j] <= R2]
            got = cols[row_ptr[v]:row_ptr[v + 1]].tolist()
            assert got == want, v
        edges = {(v, int(u)) for v in range(300) for u in cols[row_ptr[v]:row_ptr[v + 1]]}
        assert all((u, v) in edges for v, u in edges)
    rp, c = oracle.neighbour_lists(np.zeros((0, 2), dtype=np.int64), 5)
    assert rp.tolist() == [0] * 6 and len(c) == 0
    for bad in ((2, 2), (3, 1), (-1, 2), (0, 5)):
        with pytest.raises(ValueError):
            oracle.neighbour_lists(np.array([bad]), 5)
