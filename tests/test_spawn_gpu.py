"""GPU parity of ruler spawning (LR_SPAWN, Section 2.2): the spawning chase
and the ranking of its walks against the CPU oracle, bit-exact, on random,
local and structured lists, forests, weighted inputs, batches and malformed
inputs. The walks depend on timing; the results may not."""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from gpu_util import certificate_gpu, dev, gpu_prefix, gpu_rank, host_u32

pytestmark = pytest.mark.gpu

SPAWN = lr.LR_SPAWN


def sp_opts(**kw):
    kw["flags"] = kw.get("flags", 0) | SPAWN
    return lr.make_opts(**kw)


def check_rank(succ, opts=None, want_root=True):
    opts = opts if opts is not None else sp_opts()
    st, r, t = gpu_rank(succ, opts, want_root=want_root)
    assert st == lr.LR_OK, lr.status_string(st)
    ost, er, et, _ = oracle.rank(succ)
    assert ost == oracle.OK
    assert np.array_equal(r, er), f"rank mismatch at {np.nonzero(r != er)[0][:10]}"
    if want_root:
        assert np.array_equal(t, et), f"root mismatch at {np.nonzero(t != et)[0][:10]}"


@pytest.mark.parametrize("n", [1, 2, 3, 31, 63, 64, 65, 1000, 4095, 4097, 12345, 100003, 1 << 18, (1 << 20) + 7])
def test_random_lists(n):
    print(f"case: spawn random list n={n}", flush=True)
    check_rank(workloads.random_list(n, seed=400 + n % 97).succ)


@pytest.mark.parametrize("k0", [2, 8, 256, 4096])
def test_sampling_spacing(k0):
    """Few sampled rulers (k0 = 4096): the walks are mostly spawned ones."""
    print(f"case: spawn k0={k0}", flush=True)
    for n in (777, 60013, 300007):
        check_rank(workloads.random_list(n, seed=41).succ, sp_opts(spacing=(k0,)))
    check_rank(workloads.forest(60013, mean=8, n_long=1, long_len=3000, seed=42).succ, sp_opts(spacing=(k0, 4)))


@pytest.mark.parametrize("spacing,base", [((64, 2, 2, 2), 8), ((16, 16), 16384), ((64, 4, 8, 2), 16), ((), 1)])
def test_forced_levels(spacing, base):
    """The walks' list has a size known only on the device; any level plan works."""
    print(f"case: spawn spacing={spacing} base={base}", flush=True)
    check_rank(workloads.random_list(60013, seed=43).succ, sp_opts(spacing=spacing, base_max=base))
    check_rank(workloads.forest(60013, mean=8, n_long=1, long_len=3000, seed=44).succ,
               sp_opts(spacing=spacing, base_max=base))


def test_structured_lists():
    n = 100000
    print("case: spawn identity / reversed / singletons / pairs / blocks / gamma", flush=True)
    check_rank(np.minimum(np.arange(n) + 1, n - 1).astype(np.uint32))
    check_rank(np.maximum(np.arange(n) - 1, 0).astype(np.uint32))
    check_rank(np.arange(n, dtype=np.uint32))
    pairs = np.arange(n, dtype=np.uint32)
    pairs[0::2] = np.arange(1, n, 2, dtype=np.uint32)
    check_rank(pairs)
    for block, seed in [(4096, 5), (64, 6)]:
        check_rank(workloads.block_list(n, block=block, seed=seed).succ)
    for g in (0.0, 0.01, 0.3):
        check_rank(workloads.gamma_list(n, g, seed=45).succ)


@pytest.mark.parametrize("mean", [1.5, 8.0, 64.0])
def test_forests(mean):
    print(f"case: spawn forest mean={mean}", flush=True)
    check_rank(workloads.forest(250000, mean=mean, n_long=4, long_len=10000, seed=46).succ)


@pytest.mark.parametrize("wdtype", [np.int64, np.int32, None])
def test_prefix_sums(wdtype):
    print(f"case: spawn prefix sum wdtype={wdtype}", flush=True)
    n = 200003
    F = workloads.forest(n, mean=64, n_long=2, long_len=30000, seed=47)
    w = workloads.weights(n, 47, 3, -1000, 1000, wdtype) if wdtype is not None else None
    st, s, r, t = gpu_prefix(F.succ, w, sp_opts())
    assert st == lr.LR_OK, lr.status_string(st)
    ost, er, et, es = oracle.rank(F.succ, w)
    assert ost == 0
    assert np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)
    st, s2, _, _ = gpu_prefix(F.succ, w, sp_opts(), want_rank=False, want_root=False)
    assert st == lr.LR_OK and np.array_equal(s2, es)


@pytest.mark.parametrize("V", [2, 3, 1000, 1 << 16])
def test_euler_tour_depths(V):
    print(f"case: spawn euler V={V}", flush=True)
    E = workloads.euler_tour(V, seed=48)
    st, s, r, t = gpu_prefix(E.succ, E.weight, sp_opts(base_max=256))
    assert st == lr.LR_OK
    ost, er, et, es = oracle.rank(E.succ, E.weight)
    assert np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)


def test_repeated_calls_same_result():
    """Spawning depends on timing; ten calls on one workspace give one answer."""
    n = 300007
    L = workloads.random_list(n, seed=49)
    succ = dev(L.succ)
    r = torch.empty(n, dtype=torch.int32, device="cuda")
    o = sp_opts()
    ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_NONE, o))
    exp = torch.empty(n, dtype=torch.int32, device="cuda")
    exp[dev(L.order).long()] = torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda")
    for i in range(10):
        r.fill_(-1)
        assert lr.lr_rank(succ, r, None, ws, o) == lr.LR_OK
        torch.cuda.synchronize()
        assert torch.equal(r, exp), f"call {i}"


def test_large_random_certificate():
    """2^22 + 5 elements, checked on the device."""
    n = (1 << 22) + 5
    print(f"case: spawn n={n}", flush=True)
    L = workloads.random_list(n, seed=50)
    succ = dev(L.succ)
    r = torch.empty(n, dtype=torch.int32, device="cuda")
    t = torch.empty(n, dtype=torch.int32, device="cuda")
    o = sp_opts()
    ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_NONE, o))
    assert lr.lr_rank(succ, r, t, ws, o) == lr.LR_OK
    torch.cuda.synchronize()
    assert certificate_gpu(succ, r, t)
    exp = torch.empty(n, dtype=torch.int32, device="cuda")
    exp[dev(L.order).long()] = torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda")
    assert torch.equal(r, exp)


def test_batch():
    sizes = [1 << 16, 5, 77777, 1, 300001]
    items, inputs = [], []
    for i, n in enumerate(sizes):
        L = workloads.random_list(n, seed=900 + i) if i % 2 else workloads.block_list(n, 4096, seed=900 + i)
        items.append((dev(L.succ), torch.full((n,), -7, dtype=torch.int32, device="cuda"),
                      torch.full((n,), -7, dtype=torch.int32, device="cuda")))
        inputs.append(L)
    reqs = lr.requests(items)
    o = sp_opts()
    ws = lr.workspace(lr.lr_batch_workspace_bytes(reqs, len(items), o))
    assert lr.lr_rank_batch(reqs, len(items), ws, o) == lr.LR_OK
    torch.cuda.synchronize()
    for (s, r, t), L in zip(items, inputs):
        _, er, et, _ = oracle.rank(L.succ)
        assert np.array_equal(host_u32(r), er) and np.array_equal(host_u32(t), et)


def test_validate():
    o = sp_opts(flags=lr.LR_VALIDATE)
    n = 50000
    ident = np.minimum(np.arange(n) + 1, n - 1).astype(np.uint32)
    assert gpu_rank(ident, o)[0] == lr.LR_OK
    for cyc in (2, 3, 100, 4096):
        bad = ident.copy()
        bad[1000 + cyc - 1] = 1000              # a cycle over 1000 .. 1000+cyc-1
        bad[999] = 999                          # whose entry is cut, so only the cycle is wrong
        assert gpu_rank(bad, o)[0] == lr.LR_ERR_BAD_LIST, f"cycle {cyc}"
    R = workloads.random_list(n, seed=51)
    rb = R.succ.copy()
    rb[R.order[7]] = R.order[9]                 # two predecessors
    assert gpu_rank(rb, o)[0] == lr.LR_ERR_BAD_LIST
    rr = R.succ.copy()
    rr[5] = n + 3                               # out of range
    assert gpu_rank(rr, o)[0] == lr.LR_ERR_BAD_LIST
    whole = R.succ.copy()
    whole[R.order[-1]] = R.order[0]             # one cycle through every element
    assert gpu_rank(whole, o)[0] == lr.LR_ERR_BAD_LIST


def test_flag_conflict():
    n = 1000
    assert lr.lr_workspace_bytes(n, lr.LR_W_NONE, lr.make_opts(flags=SPAWN | lr.LR_LOCAL)) == 0
    succ = dev(np.arange(n, dtype=np.uint32))
    r = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = lr.workspace(1 << 20)
    assert lr.lr_rank(succ, r, None, ws, lr.make_opts(flags=SPAWN | lr.LR_LOCAL)) == lr.LR_ERR_INVALID_ARG
