"""GPU: the allocation-free closest pair (cpmi_closest_pair_noalloc) against
cpmi_closest_pair, through the C ABI.

Both calls must give the same pair and the same canonical squared distance
bit for bit (the allocating entry point is itself checked against the oracle
elsewhere). Two calls in a row, the second on a smaller input, check that the
static scratch left by the first call does not leak into the second.
"""
import numpy as np
import pytest
import torch  # noqa: F401

import paper_1407_5609_amd as cp
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
    c = cp.Context(0)
    yield c
    c.close()


def _same(a, b):
    assert (a.i, a.j, a.d2, a.d) == (b.i, b.j, b.d2, b.d), (a, b)


@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_noalloc_equals_closest_pair_twice(ctx, torch_dev, prec):
    import torch
    rng = np.random.default_rng(707)
    big, plant_big = W.planted_gaussian_points(rng, 9000, 200, 1e-3)
    small, plant_small = W.planted_gaussian_points(rng, 1300, 77, 1e-3)
    tb = torch.from_numpy(big).to(torch_dev)
    ts = torch.from_numpy(small).to(torch_dev)
    first = ctx.closest_pair_noalloc(tb, precision=prec)
    second = ctx.closest_pair_noalloc(ts, precision=prec)      # smaller, right after
    _same(first, ctx.closest_pair(tb, precision=prec))
    _same(second, ctx.closest_pair(ts, precision=prec))
    assert (first.i, first.j) == plant_big and (second.i, second.j) == plant_small


def test_noalloc_int8_and_strided_rows(ctx, torch_dev):
    import torch
    rng = np.random.default_rng(708)
    X = rng.integers(0, 3, (2500, 96)).astype(np.int8)
    X[2000] = X[17]
    X[2000, 5] += 1 if X[2000, 5] < 2 else -1                  # d2 = 1
    t = torch.from_numpy(X).to(torch_dev)
    _same(ctx.closest_pair_noalloc(t), ctx.closest_pair(t))
    F = torch.from_numpy(rng.normal(0, 1, (3000, 72)).astype(np.float32)).to(torch_dev)[:, :65]
    _same(ctx.closest_pair_noalloc(F, precision="bf16"), ctx.closest_pair(F, precision="bf16"))


def test_noalloc_rejects_what_does_not_fit(ctx, torch_dev):
    import torch
    # 70,000 x 512 BF16 rows need 70 MB of screen operand: more than the 64 MiB
    # scratch; refused on the host before any work is queued
    t = torch.zeros((70_000, 512), dtype=torch.float32, device=torch_dev)
    with pytest.raises(cp.CpmiError) as e:
        ctx.closest_pair_noalloc(t, precision="bf16")
    assert e.value.code == cp.ERR_CAPACITY
    assert "scratch" in ctx.last_error()
    with pytest.raises(cp.CpmiError) as e:
        ctx.closest_pair_noalloc(t[:1], precision="bf16")
    assert e.value.code == cp.ERR_NOPAIR
