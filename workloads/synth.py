"""Synthetic workloads for the closest-pair / fixed-radius / motif hot path.

The paper evaluates on random-walk series ("the most difficult case" for motif
mining, Section 3.6) of lengths 10K-100K and verifies answers with brute force
and with injected pairs whose answer is known (Section 6.1). These generators
reproduce those shapes with a fixed master seed (the arXiv number) so that every
consumer sees identical inputs:

  * ``cfg_points_small``  n=4096, d=64 i.i.d. N(0,1) points, one planted pair.
  * ``cfg_motif``         random walk of length 65,536, l=256, one planted motif.
  * ``cfg_mixture``       n=262,144, d=512 points from 64 Gaussian clusters,
                          planted pair at distance 1e-2.
  * ``cfg_batch``         512 random walks, lengths U[4096, 65536], l in
                          {64,128,256,512}, each with one planted motif.
  * ``cfg_snp``           100,000 x 4096 genotype rows in {0,1,2} (int8), five
                          planted near-duplicate pairs at known squared distance.

"normal(mu, s)" below always means standard deviation s (numpy ``scale``).
Nothing here computes a distance; planted answers are known by construction.
"""
from __future__ import annotations

import numpy as np

MASTER_SEED = 14075609  # the arXiv identifier 1407.5609


def config_rng(index: int) -> np.random.Generator:
    """Generator for workload ``index`` (0..15): PCG64 seeded from child
    ``index`` of ``SeedSequence(MASTER_SEED).spawn(16)`` (children do not
    depend on how many are spawned)."""
    return np.random.default_rng(np.random.SeedSequence(MASTER_SEED).spawn(16)[index])


# ----------------------------------------------------------------------------
# building blocks (usable at any size, with any generator)
# ----------------------------------------------------------------------------

def gaussian_points(rng: np.random.Generator, n: int, d: int) -> np.ndarray:
    """n x d float32 points with i.i.d. N(0,1) coordinates."""
    return rng.normal(0.0, 1.0, (n, d)).astype(np.float32)


def planted_gaussian_points(rng: np.random.Generator, n: int, d: int, noise: float):
    """Gaussian points plus one planted near-duplicate pair.

    Row b is replaced by row a plus N(0, noise) per coordinate (added in float64,
    then rounded to float32). Returns (X, (min(a,b), max(a,b)))."""
    X = gaussian_points(rng, n, d)
    a, b = (int(v) for v in rng.choice(n, 2, replace=False))
    X[b] = (X[a].astype(np.float64) + rng.normal(0.0, noise, d)).astype(np.float32)
    return X, (min(a, b), max(a, b))


def random_walk(rng: np.random.Generator, length: int) -> np.ndarray:
    """Random walk: cumulative sum (float64) of N(0,1) steps, rounded to float32."""
    return np.cumsum(rng.normal(0.0, 1.0, length)).astype(np.float32)


def plant_motif(rng: np.random.Generator, T: np.ndarray, ell: int, noise: float = 0.01):
    """Copy a length-``ell`` segment onto a non-overlapping position, plus noise.

    Source a and destination b are uniform window starts with |a-b| >= ell.
    T[b:b+ell] := T[a:a+ell] + N(0, noise) (float64, then float32). Modifies T in
    place and returns (min(a,b), max(a,b))."""
    nwin = T.shape[0] - ell + 1
    if nwin < ell + 1:
        raise ValueError("series too short to plant two non-overlapping windows")
    while True:
        a = int(rng.integers(0, nwin))
        b = int(rng.integers(0, nwin))
        if abs(a - b) >= ell:
            break
    T[b:b + ell] = (T[a:a + ell].astype(np.float64) + rng.normal(0.0, noise, ell)).astype(np.float32)
    return (min(a, b), max(a, b))


def mixture_points(rng: np.random.Generator, n: int, d: int, k: int = 64,
                   center_sd: float = 4.0, sd: float = 1.0, plant_dist: float = 1e-2,
                   chunk: int = 16384):
    """Mixture of ``k`` isotropic Gaussians plus one planted pair.

    centers ~ N(0, center_sd) (k x d); labels uniform; X = centers[label] +
    N(0, sd). Rows a != b are drawn and X[b] := X[a] + plant_dist * u with u a
    uniform random unit vector (float64, then float32). Generated in row chunks
    (identical stream to one big draw) to bound host memory.
    Returns (X float32, (min(a,b), max(a,b)))."""
    centers = rng.normal(0.0, center_sd, (k, d))
    labels = rng.integers(0, k, n)
    X = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        X[s:e] = (centers[labels[s:e]] + rng.normal(0.0, sd, (e - s, d))).astype(np.float32)
    a, b = (int(v) for v in rng.choice(n, 2, replace=False))
    u = rng.normal(0.0, 1.0, d)
    u /= np.sqrt(np.sum(u * u))
    X[b] = (X[a].astype(np.float64) + plant_dist * u).astype(np.float32)
    return X, (min(a, b), max(a, b))


def snp_matrix(rng: np.random.Generator, n: int, d: int, chunk: int = 8192) -> np.ndarray:
    """n x d int8 genotype rows: column allele frequency p ~ U(0.05, 0.5),
    entries Binomial(2, p) in {0,1,2} (the NOISE-style SNP data of Section 6.1)."""
    p = rng.uniform(0.05, 0.5, d)
    X = np.empty((n, d), dtype=np.int8)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        X[s:e] = rng.binomial(2, p, (e - s, d)).astype(np.int8)
    return X


def plant_snp_pairs(rng: np.random.Generator, X: np.ndarray, m=(3, 17, 60, 200, 640)):
    """Plant len(m) near-duplicate row pairs with exactly known squared distance.

    For pair t: rows a_t, b_t (all 2*len(m) rows distinct); row b_t := row a_t,
    then +1 at m_t distinct random columns where row a_t <= 1. Each changed entry
    differs by exactly 1, so the squared distance of the pair is exactly m_t.
    Modifies X in place; returns [(min(a,b), max(a,b), m_t), ...]."""
    n, d = X.shape
    rows = rng.choice(n, 2 * len(m), replace=False)
    out = []
    for t, mt in enumerate(m):
        a, b = int(rows[2 * t]), int(rows[2 * t + 1])
        X[b] = X[a]
        eligible = np.flatnonzero(X[a] <= 1)
        cols = rng.choice(eligible, mt, replace=False)
        X[b, cols] += 1
        out.append((min(a, b), max(a, b), int(mt)))
    return out


def batch_series(rng: np.random.Generator, count: int, lmin: int, lmax: int,
                 ells=(64, 128, 256, 512), noise: float = 0.01):
    """``count`` random walks with lengths U[lmin, lmax] and l drawn from ``ells``;
    each gets one planted motif. Returns (series list, ells list, plants list)."""
    series, ell_list, plants = [], [], []
    for _ in range(count):
        L = int(rng.integers(lmin, lmax + 1))
        ell = int(rng.choice(np.asarray(ells)))
        T = random_walk(rng, L)
        plants.append(plant_motif(rng, T, ell, noise))
        series.append(T)
        ell_list.append(ell)
    return series, ell_list, plants


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def random_strings(rng: np.random.Generator, n: int, k: int, sigma: int) -> np.ndarray:
    """n strings of length k, symbols uniform in 0..sigma-1 (int8 rows)."""
    return rng.integers(0, sigma, (n, k), dtype=np.int8)


def plant_string_pair(rng: np.random.Generator, S: np.ndarray, sigma: int, agree: int):
    """Overwrite string b with string a changed so that they agree in exactly
    `agree` positions (the others get a different symbol). Returns (a, b),
    a < b."""
    n, k = S.shape
    a, b = sorted(rng.choice(n, 2, replace=False).tolist())
    keep = np.zeros(k, dtype=bool)
    keep[rng.choice(k, agree, replace=False)] = True
    shift = rng.integers(1, sigma, k)   # a non-zero shift changes the symbol
    S[b] = np.where(keep, S[a], (S[a].astype(np.int64) + shift) % sigma).astype(np.int8)
    return a, b


def noise_genotypes(rng: np.random.Generator, m1: int, m2: int, n: int) -> np.ndarray:
    """The NOISE data of the two-locus experiments (Section 6): (m1 + m2)
    subjects x n SNPs, each value 0 or 1 with equal probability (int8)."""
    return rng.integers(0, 2, (m1 + m2, n), dtype=np.int8)


def inject_two_locus_pair(rng: np.random.Generator, G: np.ndarray, m1: int, agree_cases: int,
                          agree_controls: int, levels: int = 2):
    """Inject a SNP pair (a, b): SNP b copies SNP a in `agree_cases` random
    cases and `agree_controls` random controls and differs in the other
    subjects (value x -> (x + 1) mod levels: 0 <-> 1 for the binary NOISE
    data). Returns (a, b), a < b."""
    m, n = G.shape
    a, b = sorted(rng.choice(n, 2, replace=False).tolist())
    same = np.zeros(m, dtype=bool)
    same[rng.choice(m1, agree_cases, replace=False)] = True
    same[m1 + rng.choice(m - m1, agree_controls, replace=False)] = True
    G[:, b] = np.where(same, G[:, a], (G[:, a].astype(np.int64) + 1) % levels).astype(np.int8)
    return a, b


def cfg_strings(n: int = 20000, k: int = 64, sigma: int = 4):
    """Strings over a 4-letter alphabet (the discretised series of Section 4
    use {1, 2, 3, 4}; here 0..3): n = 20,000 uniform random strings of length
    64, one planted near-duplicate pair (agreeing in 60 of 64 positions) and
    one planted opposite pair (agreeing in none)."""
    rng = config_rng(6)
    S = random_strings(rng, n, k, sigma)
    near = plant_string_pair(rng, S, sigma, k - 4)
    far = plant_string_pair(rng, S, sigma, 0)
    return {"name": f"strings_n{n}_k{k}_s{sigma}", "S": S, "sigma": sigma, "near": near, "far": far}


def cfg_two_locus(n: int = 50000, m1: int = 200, m2: int = 200):
    """Two-locus NOISE data (Section 6): 200 cases and 200 controls, n =
    50,000 SNPs, one injected pair whose columns (a, n + b) of D have
    correlation 0.6 (1/2 + (p - q)/3 with p = 0.8 among cases, q = 0.5 among
    controls), as in the paper's injection runs."""
    rng = config_rng(7)
    G = noise_genotypes(rng, m1, m2, n)
    pair = inject_two_locus_pair(rng, G, m1, int(0.8 * m1), int(0.5 * m2))
    return {"name": f"two_locus_n{n}_m{m1}+{m2}", "G": G, "m1": m1, "m2": m2, "pair": pair}


def cfg_points_small():
    """Plain CPP + FRNN: n=4096, d=64, one planted pair (noise sd 1e-3), R=8."""
    rng = config_rng(0)
    X, plant = planted_gaussian_points(rng, 4096, 64, 1e-3)
    return {"name": "points_n4096_d64", "X": X, "plant": plant, "R": 8.0, "R2": 64.0, "excl": 1}


def cfg_motif(length: int = 65536, ell: int = 256):
    """Plain motif: random walk of length 65,536, l=256, exclusion |i-j| < l,
    one planted motif (noise sd 0.01), FRNN radius 2.0 in z-normalised units."""
    rng = config_rng(1)
    T = random_walk(rng, length)
    plant = plant_motif(rng, T, ell, 0.01)
    return {"name": f"motif_L{length}_l{ell}", "T": T, "ell": ell, "excl": ell,
            "plant": plant, "R": 2.0, "R2": 4.0}


def cfg_walk(length: int = 100000, ell: int = 1024):
    """Reference-point pruning shape (the paper's MPR runs: random walks of
    10,000-100,000 samples, windows of 1,024): random walk of length 100,000,
    l=1024, exclusion |i-j| < l, one planted motif (noise sd 0.01), FRNN
    radius 2.0 in z-normalised units."""
    rng = config_rng(5)
    T = random_walk(rng, length)
    plant = plant_motif(rng, T, ell, 0.01)
    return {"name": f"walk_L{length}_l{ell}", "T": T, "ell": ell, "excl": ell,
            "plant": plant, "R": 2.0, "R2": 4.0}


def cfg_mixture(n: int = 262144, d: int = 512):
    """Precision form: 64-cluster mixture, n=262,144, d=512, planted pair at 1e-2.
    The FRNN radius (half the lower-median nearest-neighbour distance) is an
    oracle-computed input and is not produced here."""
    rng = config_rng(2)
    X, plant = mixture_points(rng, n, d)
    return {"name": f"mixture_n{n}_d{d}", "X": X, "plant": plant, "excl": 1}


def cfg_batch(count: int = 512, lmin: int = 4096, lmax: int = 65536):
    """Batched motif: 512 random walks, lengths U[4096, 65536], l from
    {64,128,256,512}, one planted motif each; exclusion l per series."""
    rng = config_rng(3)
    series, ells, plants = batch_series(rng, count, lmin, lmax)
    return {"name": f"batch_{count}", "series": series, "ells": ells, "plants": plants}


def cfg_snp(n: int = 100000, d: int = 4096):
    """Integer exact: n=100,000 x 4096 int8 in {0,1,2}, five planted pairs with
    squared distance (3, 17, 60, 200, 640); FRNN squared radius 800."""
    rng = config_rng(4)
    X = snp_matrix(rng, n, d)
    plants = plant_snp_pairs(rng, X)
    return {"name": f"snp_n{n}_d{d}", "X": X, "plants": plants, "R2": 800, "excl": 1}


def valid_pairs_points(n: int) -> int:
    """Unordered pairs i<j among n points."""
    return n * (n - 1) // 2


def valid_pairs_motif(length: int, ell: int, excl: int) -> int:
    """Pairs i<j of the N = length-ell+1 windows with j-i >= excl."""
    N = length - ell + 1
    m = N - excl
    return m * (m + 1) // 2 if m > 0 else 0
