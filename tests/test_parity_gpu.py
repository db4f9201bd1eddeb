"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element
by element, bit-exact (all outputs are integers, tolerance 0)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from gpu_util import dev, gpu_prefix, gpu_rank, gpu_wyllie

pytestmark = pytest.mark.gpu


def check_rank(succ, opts=None):
    st, r, t = gpu_rank(succ, opts)
    assert st == lr.LR_OK, lr.status_string(st)
    ost, er, et, _ = oracle.rank(succ)
    assert ost == oracle.OK
    assert np.array_equal(r, er), f"rank mismatch at {np.nonzero(r != er)[0][:10]}"
    assert np.array_equal(t, et), f"root mismatch at {np.nonzero(t != et)[0][:10]}"


def test_random_list_2p20():
    """Single random list of 2^20 elements (the small configuration)."""
    print("case: random list n=2^20 seed=1", flush=True)
    check_rank(workloads.random_list(1 << 20, seed=1).succ)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 63, 64, 65, 1000, 4095, 4096, 4097, 8191, 8192, 8193,
                               12345, 65537, 100003, 1 << 18])
def test_random_list_sizes(n):
    print(f"case: random list n={n}", flush=True)
    check_rank(workloads.random_list(n, seed=100 + n).succ)


@pytest.mark.parametrize("k0", [2, 4, 8, 16, 32, 64, 128, 256, 1024, 4096])
@pytest.mark.parametrize("lane_walks", [1, 2])
def test_spacing_invariance(k0, lane_walks):
    """Outputs do not depend on the ruler spacing or walks per lane (several levels forced)."""
    print(f"case: spacing k0={k0} lane_walks={lane_walks}", flush=True)
    L = workloads.random_list(200003, seed=7)
    check_rank(L.succ, lr.make_opts(spacing=(k0,), base_max=64, seed=k0, lane_walks=lane_walks))


@pytest.mark.parametrize("spacing,base", [((2, 2, 2, 2, 2), 8), ((4, 8, 2), 16), ((64, 2), 1), ((16,), 16384)])
def test_deep_recursion(spacing, base):
    print(f"case: spacing={spacing} base={base}", flush=True)
    L = workloads.random_list(30011, seed=9)
    check_rank(L.succ, lr.make_opts(spacing=spacing, base_max=base))


@pytest.mark.parametrize("seed", [0, 1, 2, 12345678901])
def test_seed_invariance_and_determinism(seed):
    print(f"case: seed={seed}", flush=True)
    L = workloads.random_list(150000, seed=3)
    o = lr.make_opts(seed=seed, base_max=256)
    st1, r1, t1 = gpu_rank(L.succ, o)
    st2, r2, t2 = gpu_rank(L.succ, o)
    assert st1 == st2 == lr.LR_OK
    assert np.array_equal(r1, r2) and np.array_equal(t1, t2)
    check_rank(L.succ, o)


def test_structured_lists():
    n = 100000
    print("case: identity / reversed / singletons / pairs / block-local", flush=True)
    check_rank(np.minimum(np.arange(n) + 1, n - 1).astype(np.uint32), lr.make_opts(base_max=512))
    check_rank(np.maximum(np.arange(n) - 1, 0).astype(np.uint32), lr.make_opts(base_max=512))
    check_rank(np.arange(n, dtype=np.uint32), lr.make_opts(base_max=512))
    pairs = np.arange(n, dtype=np.uint32)
    pairs[0::2] = np.arange(1, n, 2, dtype=np.uint32)
    check_rank(pairs, lr.make_opts(base_max=512))
    check_rank(workloads.block_list(n, block=4096, seed=5).succ, lr.make_opts(base_max=512))
    check_rank(workloads.block_list(n, block=64, seed=6).succ, lr.make_opts(base_max=512))


@pytest.mark.parametrize("mean,base", [(2.0, 128), (8.0, 1024), (64.0, 0)])
def test_forest_ranks(mean, base):
    print(f"case: forest mean={mean} base={base}", flush=True)
    F = workloads.forest(300000, mean=mean, n_long=3, long_len=20000, seed=int(mean))
    check_rank(F.succ, lr.make_opts(base_max=base))


@pytest.mark.parametrize("wdtype", [np.int64, np.int32, None])
@pytest.mark.parametrize("base", [0, 64])
def test_prefix_sum_forest(wdtype, base):
    print(f"case: prefix sum forest wdtype={wdtype} base={base}", flush=True)
    F = workloads.forest(250000, mean=64, n_long=4, long_len=10000, seed=31,
                         wdtype=wdtype if wdtype is not None else np.int64)
    w = F.weight if wdtype is not None else None
    st, s, r, t = gpu_prefix(F.succ, w, lr.make_opts(base_max=base))
    assert st == lr.LR_OK, lr.status_string(st)
    ost, er, et, es = oracle.rank(F.succ, w)
    assert ost == 0
    assert np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)


def test_prefix_sum_optional_outputs():
    F = workloads.forest(50000, mean=16, n_long=1, long_len=5000, seed=32)
    st, s, r, t = gpu_prefix(F.succ, F.weight, lr.make_opts(base_max=128), want_rank=False, want_root=False)
    assert st == lr.LR_OK
    assert np.array_equal(s, oracle.rank(F.succ, F.weight)[3])


@pytest.mark.parametrize("V", [2, 3, 1000, 1 << 16])
def test_euler_tour_depths(V):
    print(f"case: euler V={V}", flush=True)
    E = workloads.euler_tour(V, seed=14)
    st, s, r, t = gpu_prefix(E.succ, E.weight, lr.make_opts(base_max=256))
    assert st == lr.LR_OK
    ost, er, et, es = oracle.rank(E.succ, E.weight)
    assert np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)
    m = E.succ.size
    h = int(np.setdiff1d(np.arange(m), E.succ[E.succ != np.arange(m)])[0])
    v = np.arange(1, V)
    assert np.array_equal(s[h] - s[E.down_arc[v]] + 1, E.depth[1:].astype(np.int64))


@pytest.mark.parametrize("n", [1, 2, 5, 1000, 70001])
def test_wyllie_baseline(n):
    print(f"case: wyllie n={n}", flush=True)
    F = workloads.forest(n, mean=16, n_long=0, long_len=0, seed=n)
    st, r, t, _ = gpu_wyllie(F.succ)
    assert st == lr.LR_OK
    ost, er, et, es = oracle.rank(F.succ, F.weight)
    assert np.array_equal(r, er) and np.array_equal(t, et)
    st, r, t, s = gpu_wyllie(F.succ, F.weight, weighted=True)
    assert st == lr.LR_OK
    assert np.array_equal(r, er) and np.array_equal(t, et) and np.array_equal(s, es)


def test_all_tiny_forests():
    """Every valid successor array with n <= 5, each ranked alone."""
    import itertools
    for n in range(1, 6):
        print(f"case: all forests n={n}", flush=True)
        for succ in itertools.product(range(n), repeat=n):
            a = np.array(succ, np.uint32)
            if oracle.rank(a)[0] != oracle.OK:
                continue
            st, r, t = gpu_rank(a)
            assert st == 0
            _, er, et, _ = oracle.rank(a)
            assert np.array_equal(r, er) and np.array_equal(t, et), a


def test_relabelled_input_gives_relabelled_output():
    F = workloads.forest(123457, mean=32, n_long=2, long_len=9000, seed=41)
    n = F.succ.size
    sigma = workloads.perm(n, seed=77)
    succ2 = np.empty(n, np.uint32)
    succ2[sigma] = sigma[F.succ]
    o = lr.make_opts(base_max=300)
    _, r, t = gpu_rank(F.succ, o)
    _, r2, t2 = gpu_rank(succ2, o)
    assert np.array_equal(r2[sigma], r) and np.array_equal(t2[sigma], sigma[t])


def test_validate_accepts_valid_and_flags_invalid():
    o = lr.make_opts(flags=lr.LR_VALIDATE, base_max=64)
    L = workloads.random_list(100000, seed=2)
    st, r, _ = gpu_rank(L.succ, o)
    assert st == lr.LR_OK
    F = workloads.forest(50000, mean=8, n_long=1, long_len=1000, seed=3)
    assert gpu_rank(F.succ, o)[0] == lr.LR_OK
    assert gpu_prefix(F.succ, F.weight, o)[0] == lr.LR_OK
    # a pure cycle beside a list
    cyc = L.succ.copy()
    a, c = int(L.order[10]), int(L.order[12])
    cyc[L.order[9]] = L.order[9]          # cut the list after position 9
    cyc[c] = a                            # close positions 10..12 into a cycle; 13.. stays a list
    assert gpu_rank(cyc, o)[0] == lr.LR_ERR_BAD_LIST
    dbl = L.succ.copy()
    dbl[L.order[5]] = L.order[7]          # two predecessors for order[7]
    assert gpu_rank(dbl, o)[0] == lr.LR_ERR_BAD_LIST
    oob = L.succ.copy()
    oob[123] = 100000 + 5
    assert gpu_rank(oob, o)[0] == lr.LR_ERR_BAD_LIST
    small = np.array([1, 2, 0, 3], np.uint32)  # cycle in a case small enough for the base case alone
    assert gpu_rank(small, o)[0] == lr.LR_ERR_BAD_LIST


def test_invalid_input_without_validation_is_memory_safe():
    """Without LR_VALIDATE, malformed input returns (garbage) without faults."""
    n = 50000
    rng = np.random.default_rng(5)
    bad = rng.integers(0, n, size=n).astype(np.uint32)  # many double predecessors and cycles
    st, _, _ = gpu_rank(bad, lr.make_opts(base_max=64))
    assert st == lr.LR_OK
    bad2 = bad.copy()
    bad2[::7] = 0xfffffff0
    st, _, _ = gpu_rank(bad2, lr.make_opts(base_max=64))
    assert st == lr.LR_OK


def test_profile_phases():
    L = workloads.random_list(1 << 20, seed=1)
    st, _, _ = gpu_rank(L.succ, lr.make_opts(flags=lr.LR_PROFILE))
    assert st == 0
    ms = lr.lr_profile_last()
    assert len(ms) == 8 and all(x >= 0 for x in ms) and ms[6] > 0
    assert ms[7] == 0.0  # an ordinary random list never needs the fallback
    torch.cuda.synchronize()


# ------------------------------------------------------------------------
# Inputs of 2^25 elements and more take the visit-log path at level 0 by
# default; LR_VISIT_LOG takes it from 2^16 on, so these cases stay small.

LOG = lr.LR_VISIT_LOG


def test_visit_log_threshold():
    """The default switches to the visit log at 2^25; the result is the closed
    form of the generator either way (checked on the device: the oracle would
    take seconds per call at this size)."""
    n = (1 << 25) + 3
    print(f"case: default visit log n={n}", flush=True)
    L = workloads.random_list(n, seed=25)
    succ = dev(L.succ)
    r = torch.empty(n, dtype=torch.int32, device="cuda")
    t = torch.empty(n, dtype=torch.int32, device="cuda")
    exp = torch.empty(n, dtype=torch.int32, device="cuda")
    exp[dev(L.order).long()] = torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda")
    for flags in (0, lr.LR_NO_LOCAL):
        ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_NONE, lr.make_opts(flags=flags)))
        assert lr.lr_rank(succ, r, t, ws, lr.make_opts(flags=flags)) == lr.LR_OK
        torch.cuda.synchronize()
        assert torch.equal(r, exp)
        assert bool((t == int(L.order[-1])).all())
        del ws


@pytest.mark.parametrize("n", [1 << 22, (1 << 22) + 12345, 5000011])
@pytest.mark.parametrize("lane_walks", [1, 2])
def test_log_mode_random_lists(n, lane_walks):
    print(f"case: log mode random list n={n} lane_walks={lane_walks}", flush=True)
    p = lr.lr_plan_query(n)
    assert p.levels >= 1
    L = workloads.random_list(n, seed=n % 1000)
    check_rank(L.succ, lr.make_opts(flags=LOG, lane_walks=lane_walks))
    st, r, _ = gpu_rank(L.succ, lr.make_opts(flags=LOG, lane_walks=lane_walks), want_root=False)
    assert st == lr.LR_OK and np.array_equal(r, oracle.rank(L.succ)[1])


def test_log_mode_block_list_and_forest():
    n = (1 << 22) + 77
    print("case: log mode block list / forest", flush=True)
    o = lr.make_opts(flags=LOG)
    check_rank(workloads.block_list(n, block=4096, seed=8).succ, o)
    F = workloads.forest(n, mean=64, n_long=4, long_len=100000, seed=9)
    check_rank(F.succ, o)
    st, s, r, t = gpu_prefix(F.succ, F.weight, o)
    assert st == lr.LR_OK
    ost, er, et, es = oracle.rank(F.succ, F.weight)
    assert np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)
    F32 = workloads.forest(n, mean=8, n_long=1, long_len=300000, seed=10, wdtype=np.int32)
    st, s, r, t = gpu_prefix(F32.succ, F32.weight, o)
    ost, er, et, es = oracle.rank(F32.succ, F32.weight)
    assert st == lr.LR_OK and np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)


def test_log_mode_all_singletons_and_pairs():
    n = (1 << 22) + 3
    print("case: log mode singletons / pairs", flush=True)
    o = lr.make_opts(flags=LOG)
    check_rank(np.arange(n, dtype=np.uint32), o)
    pairs = np.arange(n, dtype=np.uint32)
    pairs[0:n - 1:2] = np.arange(1, n, 2, dtype=np.uint32)
    check_rank(pairs, o)


@pytest.mark.parametrize("bits", [1, 3, 7])
def test_packed_log_continuations(bits):
    """Packed visit-log records with the offset field capped at `bits` bits:
    a walk goes on under a new continuation id every 2^bits visits; ranks,
    roots and weighted sums still equal the oracle's."""
    n = (1 << 22) + 4321
    print(f"case: packed log continuations bits={bits}", flush=True)
    o = lr.make_opts(flags=LOG | lr.LR_NO_LOCAL, log_off_bits=bits)
    L = workloads.random_list(n, seed=31)
    check_rank(L.succ, o)
    F = workloads.forest(n, mean=64, n_long=4, long_len=100000, seed=32)
    st, s, r, t = gpu_prefix(F.succ, F.weight, o)
    ost, er, et, es = oracle.rank(F.succ, F.weight)
    assert st == lr.LR_OK and np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)


@pytest.mark.parametrize("bits", [0, 2])
def test_packed_log_contracted_list(bits):
    """The contracted list of tile-local contraction through the packed
    visit log: its steps count whole chains, so with a 2-bit offset field
    nearly every record of a walk starts a continuation."""
    n = (1 << 22) + 99
    print(f"case: packed log contracted list bits={bits}", flush=True)
    o = lr.make_opts(flags=LOG | lr.LR_LOCAL, log_off_bits=bits)
    check_rank(workloads.gamma_list(n, 0.1, seed=33).succ, o)
    check_rank(workloads.block_list(n, block=4096, seed=34).succ, o)
    F = workloads.forest(n, mean=8, n_long=1, long_len=300000, seed=35, wdtype=np.int32)
    st, s, r, t = gpu_prefix(F.succ, F.weight, o)
    ost, er, et, es = oracle.rank(F.succ, F.weight)
    assert st == lr.LR_OK and np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)


@pytest.mark.parametrize("wdtype", [np.int32, np.int64])
def test_log_mode_unaligned_weights_and_successors(wdtype):
    """The head-sum pass interleaves (successor, weight) records with vector
    loads only when both arrays are 16-byte aligned; views that start one
    element in take its scalar path. Sums, ranks and roots equal the oracle's."""
    n = (1 << 22) + 5
    print(f"case: log mode unaligned inputs {wdtype.__name__}", flush=True)
    F = workloads.forest(n, mean=64, n_long=4, long_len=100000, seed=36, wdtype=wdtype)
    o = lr.make_opts(flags=LOG | lr.LR_NO_LOCAL)
    wbig = torch.empty(n + 1, dtype=torch.from_numpy(F.weight[:1]).dtype, device="cuda")
    wbig[1:] = torch.from_numpy(F.weight).cuda()
    sbig = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    sbig[1:] = dev(F.succ)
    ost, er, et, es = oracle.rank(F.succ, F.weight)
    for succ, w in ((dev(F.succ), wbig[1:]), (sbig[1:], wbig[1:]), (sbig[1:], torch.from_numpy(F.weight).cuda())):
        sm = torch.empty(n, dtype=torch.int64, device="cuda")
        r = torch.empty(n, dtype=torch.int32, device="cuda")
        t = torch.empty(n, dtype=torch.int32, device="cuda")
        ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_I64, o))
        assert lr.lr_prefix_sum(succ, w, sm, r, t, ws, o) == lr.LR_OK
        torch.cuda.synchronize()
        assert np.array_equal(sm.cpu().numpy(), es)
        assert np.array_equal(r.cpu().numpy().view(np.uint32), er) and np.array_equal(t.cpu().numpy().view(np.uint32), et)


def test_log_mode_validate():
    n = 1 << 22
    o = lr.make_opts(flags=lr.LR_VALIDATE | LOG)
    L = workloads.random_list(n, seed=4)
    assert gpu_rank(L.succ, o)[0] == lr.LR_OK
    cyc = L.succ.copy()
    cyc[L.order[999]] = L.order[999]
    cyc[L.order[2000]] = L.order[1000]
    assert gpu_rank(cyc, o)[0] == lr.LR_ERR_BAD_LIST
    dbl = L.succ.copy()
    dbl[L.order[5]] = L.order[7]
    assert gpu_rank(dbl, o)[0] == lr.LR_ERR_BAD_LIST


def test_log_mode_invalid_input_is_memory_safe():
    n = 1 << 22
    rng = np.random.default_rng(11)
    bad = rng.integers(0, n, size=n).astype(np.uint32)
    assert gpu_rank(bad, lr.make_opts(flags=LOG))[0] == lr.LR_OK
    assert gpu_rank(bad)[0] == lr.LR_OK


# The base case's slot columns (4096, 8192 or 16384 slots, padded with
# self-loops): levels of every size around the column boundaries, alone and
# as the last level under one ruling-set level, unweighted and weighted
# (weighted levels above 8192 elements take the separate-array layout).
@pytest.mark.parametrize("n,base,spacing", [
    (1, 0, ()), (1023, 0, ()), (1025, 0, ()), (4095, 0, ()), (4097, 0, ()), (8191, 0, ()), (8193, 0, ()),
    (12289, 0, ()), (16383, 0, ()), (16384, 0, ()), (16383 * 2, 16384, (2,)), (8193 * 4, 8193, (4,)),
    (4097 * 8, 4097, (8,)), (12000 * 8, 12000, (8,))])
def test_base_case_columns(n, base, spacing):
    print(f"case: base columns n={n} base={base} spacing={spacing}", flush=True)
    o = lr.make_opts(base_max=base, spacing=spacing) if (base or spacing) else None
    check_rank(workloads.random_list(n, seed=300 + n).succ, o)
    F = workloads.forest(n, mean=5, n_long=1, long_len=max(1, n // 3), seed=400 + n)
    check_rank(F.succ, o)


@pytest.mark.parametrize("n,base,spacing", [
    (1, 0, ()), (4095, 4096, ()), (4097, 8192, ()), (8192, 8192, ()), (8193, 10000, ()), (10000, 10000, ()),
    (4097 * 4, 4097, (4,)), (8192 * 4, 8192, (4,)), (10000 * 4, 10000, (4,)), (50001, 0, ())])
def test_base_case_columns_weighted(n, base, spacing):
    print(f"case: weighted base columns n={n} base={base} spacing={spacing}", flush=True)
    o = lr.make_opts(base_max=base, spacing=spacing) if (base or spacing) else None
    for L in (workloads.random_list(n, seed=500 + n), workloads.forest(n, mean=5, n_long=1,
                                                                      long_len=max(1, n // 3), seed=600 + n)):
        w = workloads.weights(n, seed=700 + n, stream=0, lo=-(1 << 40), hi=1 << 40)
        st, s, r, t = gpu_prefix(L.succ, w, o)
        assert st == lr.LR_OK, lr.status_string(st)
        ost, er, et, es = oracle.rank(L.succ, w)
        assert ost == 0
        assert np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)
