"""Input generators: permutations are bijections, outputs are reproducible
from the seed, and the structural properties each workload promises hold."""
import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("n", [1, 2, 3, 5, 1000, 4096, 65536 + 3])
def test_perm_is_bijection_and_reproducible(n):
    p = workloads.perm(n, seed=7, stream=3)
    assert np.array_equal(np.sort(p), np.arange(n, dtype=np.uint32))
    assert np.array_equal(p, workloads.perm(n, seed=7, stream=3))
    if n > 100:
        assert not np.array_equal(p, workloads.perm(n, seed=8, stream=3))


def test_block_order_locality():
    n, B = 4096 * 7 + 123, 4096
    o = workloads.block_order(n, B, seed=5, stream=1)
    assert np.array_equal(np.sort(o), np.arange(n, dtype=np.uint32))
    blk = o.astype(np.int64) // B
    # blocks are visited contiguously: the block id changes exactly (#blocks - 1) times
    assert int(np.count_nonzero(np.diff(blk))) == (n + B - 1) // B - 1


def test_random_list_is_one_list():
    L = workloads.random_list(10000, seed=3)
    s = L.succ.astype(np.int64)
    assert np.count_nonzero(s == np.arange(s.size)) == 1
    assert np.unique(s[s != np.arange(s.size)]).size == s.size - 1


def test_forest_lengths_mean_and_total():
    lens = workloads.forest_lengths(3, 1 << 20, 64.0, 2, 1000)
    assert int(lens.sum()) == (1 << 20) + 2000
    assert 55 < float(lens[:-2].mean()) < 73
    assert lens.min() >= 1


def test_euler_tour_shape():
    E = workloads.euler_tour(1000, seed=4)
    assert E.succ.size == 2 * 999
    assert np.all(E.parent[1:] < np.arange(1, 1000))
    assert int(E.weight.sum()) == 0
    s = E.succ.astype(np.int64)
    assert np.count_nonzero(s == np.arange(s.size)) == 1


def test_serving_trace_sizes():
    tr = workloads.serving_trace(count=512, rate_per_s=1000.0, seed=5)
    ns = np.array([r.n for r in tr])
    assert ns.min() >= 1 << 10 and ns.max() < 1 << 24
    t = np.array([r.arrival_s for r in tr])
    assert np.all(np.diff(t) > 0)
    assert {r.kind for r in tr} == {"random", "block"}


@pytest.mark.parametrize("gamma", [0.0, 0.001, 0.25, 1.0])
def test_gamma_order(gamma):
    """List(n, gamma): a permutation that moves at most round(gamma n) ids, and
    only ids of the sampled positions; gamma = 0 is the identity."""
    n = 100003
    o = workloads.gamma_order(n, gamma, seed=6)
    assert np.array_equal(np.sort(o), np.arange(n, dtype=np.uint32))
    moved = np.nonzero(o != np.arange(n))[0]
    assert moved.size <= round(gamma * n)
    assert np.array_equal(np.sort(o[moved]), moved)       # ids stay within the sampled positions
    if gamma >= 0.25:
        assert moved.size > 0.9 * gamma * n               # almost every sampled id moves
    assert np.array_equal(o, workloads.gamma_order(n, gamma, seed=6))
    L = workloads.gamma_list(n, gamma, seed=6)
    assert np.array_equal(L.succ[L.order[:-1]], L.order[1:])
    with pytest.raises(ValueError):
        workloads.gamma_order(10, 1.5, seed=1)


@pytest.mark.parametrize("n", [1, 4096, 4097, 300001])
def test_striped_list(n):
    """Kept tiles are single stretches in id order; the list covers every id."""
    L = workloads.striped_list(n, 4096, 16, seed=5)
    assert np.array_equal(np.sort(L.order), np.arange(n, dtype=np.uint32))
    assert np.array_equal(L.succ[L.order[:-1]], L.order[1:])
    pos = np.empty(n, np.int64)
    pos[L.order] = np.arange(n)
    for t in range(0, (n + 4095) // 4096, 16):
        ids = np.arange(t * 4096, min(n, (t + 1) * 4096))
        assert np.all(np.diff(pos[ids]) == 1)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 1000, 65537, (1 << 20) + 3])
def test_device_generator_is_one_list(n):
    """The device-side generator (keyed Feistel over the smallest even-width
    domain holding [0, n), cycle walking), run on the CPU: its order is a
    permutation of [0, n) and its successors link that order into one list."""
    import torch
    succ, order = workloads.random_list_device(n, device="cpu")
    o = order.numpy().astype(np.int64)
    assert np.array_equal(np.sort(o), np.arange(n))
    s = succ.numpy().astype(np.int64)
    assert np.array_equal(s[o[:-1]], o[1:]) and s[o[-1]] == o[-1]
    again, _ = workloads.random_list_device(n, device="cpu")
    assert torch.equal(succ, again)
