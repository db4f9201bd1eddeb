"""GPU parity of tile-local contraction (LR_LOCAL, Section 2.3): the contracted
path against the CPU oracle, bit-exact, on inputs from no locality (random
lists) to full locality (succ[i] = i + 1), with and without weights, alone and
batched, valid and malformed."""
import itertools

import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from gpu_util import dev, gpu_prefix, gpu_rank, host_u32

pytestmark = pytest.mark.gpu

LOCAL = lr.LR_LOCAL


def local_opts(**kw):
    kw["flags"] = kw.get("flags", 0) | LOCAL
    return lr.make_opts(**kw)


def check_rank(succ, opts=None, want_root=True):
    opts = opts if opts is not None else local_opts()
    st, r, t = gpu_rank(succ, opts, want_root=want_root)
    assert st == lr.LR_OK, lr.status_string(st)
    ost, er, et, _ = oracle.rank(succ)
    assert ost == oracle.OK
    assert np.array_equal(r, er), f"rank mismatch at {np.nonzero(r != er)[0][:10]}"
    if want_root:
        assert np.array_equal(t, et), f"root mismatch at {np.nonzero(t != et)[0][:10]}"


@pytest.mark.parametrize("n", [1, 2, 3, 31, 32, 33, 4095, 4096, 4097, 8191, 8193, 12345, 100003, 1 << 18])
def test_random_lists(n):
    """No locality: almost every element starts its own chain."""
    print(f"case: local random list n={n}", flush=True)
    check_rank(workloads.random_list(n, seed=300 + n).succ)


@pytest.mark.parametrize("gamma", [0.0, 1e-4, 0.001, 0.01, 0.1, 0.5, 1.0])
@pytest.mark.parametrize("n", [300007, 1 << 20])
def test_gamma_lists(gamma, n):
    """The paper's List(n, gamma); ranks also against the closed form n-1-j."""
    print(f"case: local List(n={n}, gamma={gamma})", flush=True)
    L = workloads.gamma_list(n, gamma, seed=11)
    st, r, t = gpu_rank(L.succ, local_opts())
    assert st == lr.LR_OK
    exp = np.empty(n, np.uint32)
    exp[L.order] = np.arange(n - 1, -1, -1, dtype=np.uint32)
    assert np.array_equal(r, exp)
    assert np.all(t == L.order[-1])
    check_rank(L.succ)


def test_structured_lists():
    n = 100000
    print("case: local identity / reversed / singletons / pairs / blocks", flush=True)
    check_rank(np.minimum(np.arange(n) + 1, n - 1).astype(np.uint32))
    check_rank(np.maximum(np.arange(n) - 1, 0).astype(np.uint32))
    check_rank(np.arange(n, dtype=np.uint32))
    pairs = np.arange(n, dtype=np.uint32)
    pairs[0::2] = np.arange(1, n, 2, dtype=np.uint32)
    check_rank(pairs)
    for block, seed in [(4096, 5), (64, 6), (5000, 7), (8192, 8)]:
        check_rank(workloads.block_list(n, block=block, seed=seed).succ)


def test_long_chains_inside_tiles():
    """Every tile holds one chain of 4096 in random order: the deepest jumping."""
    n = (1 << 20) + 77
    print(f"case: local block list n={n}", flush=True)
    check_rank(workloads.block_list(n, block=4096, seed=21).succ)
    check_rank(workloads.block_list(n, block=4096, seed=21).succ, local_opts(base_max=64))


@pytest.mark.parametrize("spacing,base", [((2, 2, 2), 8), ((16,), 16384), ((4, 8, 2), 16), ((), 1)])
def test_forced_levels(spacing, base):
    """The contracted list's size is only known on the device; any level plan works."""
    print(f"case: local spacing={spacing} base={base}", flush=True)
    for g in (0.0, 0.05, 1.0):
        check_rank(workloads.gamma_list(60013, g, seed=12).succ, local_opts(spacing=spacing, base_max=base))
    check_rank(workloads.forest(60013, mean=8, n_long=1, long_len=3000, seed=13).succ,
               local_opts(spacing=spacing, base_max=base))


@pytest.mark.parametrize("mean", [2.0, 64.0])
def test_forests(mean):
    print(f"case: local forest mean={mean}", flush=True)
    check_rank(workloads.forest(250000, mean=mean, n_long=4, long_len=10000, seed=31).succ)


@pytest.mark.parametrize("wdtype", [np.int64, np.int32, None])
@pytest.mark.parametrize("gamma", [0.0, 0.02, 1.0])
def test_prefix_sums(wdtype, gamma):
    """Weighted chains: the contracted record carries the chain's weight."""
    print(f"case: local prefix sum wdtype={wdtype} gamma={gamma}", flush=True)
    n = 200003
    L = workloads.gamma_list(n, gamma, seed=14)
    w = workloads.weights(n, 14, 3, -1000, 1000, wdtype) if wdtype is not None else None
    st, s, r, t = gpu_prefix(L.succ, w, local_opts())
    assert st == lr.LR_OK, lr.status_string(st)
    ost, er, et, es = oracle.rank(L.succ, w)
    assert ost == 0
    assert np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)


def test_prefix_sum_forest_and_optional_outputs():
    F = workloads.forest(250000, mean=64, n_long=4, long_len=10000, seed=31)
    _, er, et, es = oracle.rank(F.succ, F.weight)
    st, s, r, t = gpu_prefix(F.succ, F.weight, local_opts())
    assert st == lr.LR_OK
    assert np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)
    st, s, _, _ = gpu_prefix(F.succ, F.weight, local_opts(), want_rank=False, want_root=False)
    assert st == lr.LR_OK and np.array_equal(s, es)


@pytest.mark.parametrize("V", [2, 3, 1000, 1 << 16])
def test_euler_tour_depths(V):
    print(f"case: local euler V={V}", flush=True)
    E = workloads.euler_tour(V, seed=14)
    st, s, r, t = gpu_prefix(E.succ, E.weight, local_opts(base_max=256))
    assert st == lr.LR_OK
    ost, er, et, es = oracle.rank(E.succ, E.weight)
    assert np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)


def test_all_tiny_forests():
    """Every valid successor array with n <= 5 (one tile, all chain shapes)."""
    o = local_opts()
    for n in range(1, 6):
        print(f"case: local all forests n={n}", flush=True)
        for succ in itertools.product(range(n), repeat=n):
            a = np.array(succ, np.uint32)
            if oracle.rank(a)[0] != oracle.OK:
                continue
            st, r, t = gpu_rank(a, o)
            assert st == 0
            _, er, et, _ = oracle.rank(a)
            assert np.array_equal(r, er) and np.array_equal(t, et), a


def test_local_equals_plain_path():
    """Same outputs with and without contraction (and across seeds)."""
    for g in (0.0, 0.003, 0.3):
        L = workloads.gamma_list(500009, g, seed=15)
        st1, r1, t1 = gpu_rank(L.succ, lr.make_opts(seed=3))
        st2, r2, t2 = gpu_rank(L.succ, local_opts(seed=4))
        assert st1 == st2 == lr.LR_OK
        assert np.array_equal(r1, r2) and np.array_equal(t1, t2)


def test_batch():
    """A batch is one forest over the concatenated ids; tiles may straddle requests."""
    sizes = [1000, 17, 65536, 3, 200001, 4096, 5000, 1]
    items, inputs = [], []
    for i, n in enumerate(sizes):
        L = workloads.random_list(n, seed=900 + i) if i % 2 == 0 else workloads.block_list(n, 4096, seed=900 + i)
        items.append((dev(L.succ), torch.full((n,), -7, dtype=torch.int32, device="cuda"),
                      torch.full((n,), -7, dtype=torch.int32, device="cuda") if i % 3 else None))
        inputs.append(L)
    o = local_opts()
    reqs = lr.requests(items)
    ws = lr.workspace(lr.lr_batch_workspace_bytes(reqs, len(items), o))
    assert lr.lr_rank_batch(reqs, len(items), ws, o) == lr.LR_OK
    torch.cuda.synchronize()
    for (s, r, t), L in zip(items, inputs):
        _, er, et, _ = oracle.rank(L.succ)
        assert np.array_equal(host_u32(r), er)
        if t is not None:
            assert np.array_equal(host_u32(t), et)


def test_validate():
    o = local_opts(flags=lr.LR_VALIDATE | LOCAL, base_max=64)
    L = workloads.gamma_list(100000, 0.01, seed=2)
    assert gpu_rank(L.succ, o)[0] == lr.LR_OK
    F = workloads.forest(50000, mean=8, n_long=1, long_len=1000, seed=3)
    assert gpu_rank(F.succ, o)[0] == lr.LR_OK
    assert gpu_prefix(F.succ, F.weight, o)[0] == lr.LR_OK
    n = 20000
    ident = np.minimum(np.arange(n) + 1, n - 1).astype(np.uint32)
    inside = ident.copy()
    inside[99] = 99
    inside[110] = 100                      # cycle 100..110 inside one tile
    assert gpu_rank(inside, o)[0] == lr.LR_ERR_BAD_LIST
    across = ident.copy()
    across[4000] = 4000
    across[12000] = 4001                   # cycle 4001..12000 across tiles
    assert gpu_rank(across, o)[0] == lr.LR_ERR_BAD_LIST
    dbl = ident.copy()
    dbl[10] = 12                           # two predecessors for 12
    assert gpu_rank(dbl, o)[0] == lr.LR_ERR_BAD_LIST
    oob = ident.copy()
    oob[123] = n + 5
    assert gpu_rank(oob, o)[0] == lr.LR_ERR_BAD_LIST
    assert gpu_rank(np.array([1, 2, 0, 3], np.uint32), o)[0] == lr.LR_ERR_BAD_LIST


def test_invalid_input_is_memory_safe():
    """Without LR_VALIDATE, malformed input returns (garbage) without faults."""
    n = 50000
    rng = np.random.default_rng(5)
    bad = rng.integers(0, n, size=n).astype(np.uint32)
    assert gpu_rank(bad, local_opts(base_max=64))[0] == lr.LR_OK
    near = np.clip(np.arange(n) + rng.integers(-3, 4, size=n), 0, n - 1).astype(np.uint32)  # local, many cycles
    assert gpu_rank(near, local_opts(base_max=64))[0] == lr.LR_OK
    bad2 = bad.copy()
    bad2[::7] = 0xfffffff0
    assert gpu_rank(bad2, local_opts(base_max=64))[0] == lr.LR_OK
    assert gpu_prefix(near, None, local_opts(base_max=64))[0] == lr.LR_OK


def test_large_random_takes_capacity_levels():
    """A contracted list as long as the input (no locality), with and without
    the visit log for its first level."""
    n = (1 << 22) + 12345
    print(f"case: local random list n={n}", flush=True)
    succ = workloads.random_list(n, seed=17).succ
    check_rank(succ, want_root=False)
    check_rank(succ, local_opts(flags=lr.LR_VISIT_LOG), want_root=False)


# ------------------------------------------------------------------------
# Automatic choice (default flags, inputs of 2^21 elements or more): the
# head-sum pass counts local links on the device and one of the two enqueued
# paths runs. Outputs must not depend on the choice.

AUTO_N = (1 << 21) + 4099


@pytest.mark.parametrize("gamma", [0.0, 0.02, 0.2, 0.3, 1.0])
def test_automatic_choice(gamma):
    print(f"case: auto List(n={AUTO_N}, gamma={gamma})", flush=True)
    L = workloads.gamma_list(AUTO_N, gamma, seed=16)
    exp = np.empty(AUTO_N, np.uint32)
    exp[L.order] = np.arange(AUTO_N - 1, -1, -1, dtype=np.uint32)
    for flags in (0, lr.LR_NO_LOCAL, LOCAL):
        st, r, t = gpu_rank(L.succ, lr.make_opts(flags=flags))
        assert st == lr.LR_OK
        assert np.array_equal(r, exp), f"flags={flags}"
        assert np.all(t == L.order[-1])
    check_rank(L.succ, lr.make_opts())


def test_automatic_choice_forest_and_weights():
    F = workloads.forest(AUTO_N, mean=64, n_long=2, long_len=100000, seed=18)
    check_rank(F.succ, lr.make_opts())
    L = workloads.gamma_list(AUTO_N, 0.01, seed=19)
    w = workloads.weights(AUTO_N, 19, 3, -1000, 1000, np.int32)
    st, s, r, t = gpu_prefix(L.succ, w, lr.make_opts())
    assert st == lr.LR_OK
    _, er, et, es = oracle.rank(L.succ, w)
    assert np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)


def test_automatic_choice_validate():
    o = lr.make_opts(flags=lr.LR_VALIDATE)
    ident = np.minimum(np.arange(AUTO_N) + 1, AUTO_N - 1).astype(np.uint32)
    assert gpu_rank(ident, o)[0] == lr.LR_OK
    bad = ident.copy()
    bad[99] = 99
    bad[110] = 100                          # a cycle inside one tile
    assert gpu_rank(bad, o)[0] == lr.LR_ERR_BAD_LIST
    R = workloads.random_list(AUTO_N, seed=20)
    assert gpu_rank(R.succ, o)[0] == lr.LR_OK
    rb = R.succ.copy()
    rb[R.order[7]] = R.order[9]             # two predecessors
    assert gpu_rank(rb, o)[0] == lr.LR_ERR_BAD_LIST


def test_automatic_choice_batch():
    """A batch of block-local requests takes the contracted path as one forest."""
    sizes = [1 << 20, 5, 777777, 4096, 300001]
    items, inputs = [], []
    for i, n in enumerate(sizes):
        L = workloads.block_list(n, 4096, seed=700 + i)
        items.append((dev(L.succ), torch.full((n,), -7, dtype=torch.int32, device="cuda"),
                      torch.full((n,), -7, dtype=torch.int32, device="cuda") if i % 2 else None))
        inputs.append(L)
    assert sum(sizes) >= 1 << 21
    reqs = lr.requests(items)
    ws = lr.workspace(lr.lr_batch_workspace_bytes(reqs, len(items)))
    assert lr.lr_rank_batch(reqs, len(items), ws) == lr.LR_OK
    torch.cuda.synchronize()
    for (s, r, t), L in zip(items, inputs):
        _, er, et, _ = oracle.rank(L.succ)
        assert np.array_equal(host_u32(r), er)
        if t is not None:
            assert np.array_equal(host_u32(t), et)


def test_automatic_choice_wrong_guess():
    """The choice is guessed from every 16th tile of 4096 ids. Here exactly
    those tiles are local and the rest is random, so the guess picks
    contraction, the contracted list is far larger than its levels hold, and
    the contracted path must hand over to the plain path on the device."""
    L = workloads.striped_list(AUTO_N, 4096, 16, seed=21)
    print(f"case: striped n={AUTO_N}", flush=True)
    exp = np.empty(AUTO_N, np.uint32)
    exp[L.order] = np.arange(AUTO_N - 1, -1, -1, dtype=np.uint32)
    for flags in (0, lr.LR_VALIDATE):
        st, r, t = gpu_rank(L.succ, lr.make_opts(flags=flags))
        assert st == lr.LR_OK
        assert np.array_equal(r, exp), f"flags={flags}"
        assert np.all(t == L.order[-1])
    w = workloads.weights(AUTO_N, 21, 3, -1000, 1000, np.int64)
    st, s, r, t = gpu_prefix(L.succ, w, lr.make_opts())
    assert st == lr.LR_OK
    _, er, et, es = oracle.rank(L.succ, w)
    assert np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)
    bad = L.succ.copy()
    bad[L.order[5]] = L.order[5]            # a second terminal: two lists
    check_rank(bad, lr.make_opts())


@pytest.mark.parametrize("cycle_len", [1, 2, 3, 4, 7, 16, 100, 4096])
def test_validate_cycles_inside_a_tile(cycle_len):
    """A cycle of any length inside one tile beside a valid list: the jumps of
    a cycle element can come back to the element itself, which must still be
    reported (the element is not a chain start)."""
    o = local_opts(flags=lr.LR_VALIDATE | LOCAL)
    n = 3 * 4096
    succ = np.minimum(np.arange(n) + 1, n - 1).astype(np.uint32)
    c0 = 4096 + 17 if cycle_len < 4000 else 4096
    succ[c0 - 1] = c0 - 1                                   # the list before the cycle ends here
    idx = np.arange(c0, c0 + cycle_len)
    succ[idx] = np.roll(idx, -1)                            # close the cycle
    if cycle_len == 1:
        succ[c0] = c0 + 1 if c0 + 1 < n else c0            # a self-loop is a terminal: use a 2-cycle instead
        succ[c0 + 1] = c0
    assert gpu_rank(succ, o)[0] == lr.LR_ERR_BAD_LIST, cycle_len
    assert gpu_rank(succ, local_opts())[0] == lr.LR_OK     # without validation: no fault
