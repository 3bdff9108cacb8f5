"""GPU radix sort (fl_sort_keys) against numpy's stable argsort, bit for bit.

The sort is a tile-by-tile pass with decoupled look-back over 4096-key
tiles, so the sizes cover one partial tile, exact tile multiples and ragged
tails up to 2M keys (489 tiles, the iteration's size), plus 4.2M keys (1026
tiles), which take the three-launch pass instead; the key sets
cover random, sorted, reversed, few distinct values (long runs of equal
digits, where stability shows) and a single value.  Sorted keys and the
permutation must equal the stable order exactly; a second call on the same
context checks that the per-call state (tickets, look-back words) starts
clean.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03504_amd import fa2lay
    c = fa2lay.Context(0)
    yield c
    c.close()


def keys(kind, n, bits, seed):
    rng = np.random.default_rng(seed)
    top = 1 << (2 * bits)
    if kind == "random":
        k = rng.integers(0, top, n, dtype=np.uint64)
    elif kind == "sorted":
        k = np.sort(rng.integers(0, top, n, dtype=np.uint64))
    elif kind == "reversed":
        k = np.sort(rng.integers(0, top, n, dtype=np.uint64))[::-1]
    elif kind == "few":
        k = rng.choice(rng.integers(0, top, 5, dtype=np.uint64), n)
    elif kind == "single":
        k = np.full(n, top // 3, np.uint64)
    else:
        raise ValueError(kind)
    return np.ascontiguousarray(k.astype(np.uint32))


def check(ctx, k, bits):
    kd = torch.from_numpy(k.view(np.int32)).cuda()
    sk, perm = ctx.sort_keys(kd, bits)
    torch.cuda.synchronize()
    ref = np.argsort(k, kind="stable")
    assert np.array_equal(perm.cpu().numpy(), ref.astype(np.int32))
    assert np.array_equal(sk.cpu().numpy().view(np.uint32), k[ref])


@pytest.mark.parametrize("n", [1, 63, 4095, 4096, 4097, 3 * 4096, 100_003, 2_000_000, 4_200_011])
@pytest.mark.parametrize("kind", ["random", "few"])
def test_sizes(ctx, n, kind):
    _note("sort", kind, n)
    check(ctx, keys(kind, n, 16, n), 16)


@pytest.mark.parametrize("kind", ["sorted", "reversed", "single"])
def test_orders(ctx, kind):
    _note("sort order", kind)
    check(ctx, keys(kind, 300_007, 16, 3), 16)


@pytest.mark.parametrize("bits", [1, 4, 7, 12])
def test_digit_counts(ctx, bits):
    # 2 bits .. 24 bits of key: one to three passes
    _note("sort bits", bits)
    check(ctx, keys("random", 70_001, bits, bits), bits)


def test_repeated_calls(ctx):
    _note("sort repeated")
    for s in range(3):
        check(ctx, keys("random", 250_000 - 37 * s, 16, 10 + s), 16)
