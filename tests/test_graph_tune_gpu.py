"""A ranking call captured into a HIP graph replays correctly (inputs changed
between replays, other work and synchronisations in between), and the plan
autotuner returns options whose results equal the oracle's."""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from gpu_util import dev, host_u32

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,flags", [(1 << 16, 0), ((1 << 22) + 5, 0), ((1 << 22) + 5, lr.LR_VISIT_LOG)])
def test_graph_capture_and_replays(n, flags):
    print(f"case: graph capture n={n} flags={flags}", flush=True)
    o = lr.make_opts(flags=flags)
    lists = [workloads.random_list(n, seed=60 + i) if i % 2 == 0 else workloads.block_list(n, 4096, seed=60 + i)
             for i in range(4)]
    succ = dev(lists[0].succ)
    rank = torch.empty(n, dtype=torch.int32, device="cuda")
    root = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_NONE, o))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        assert lr.lr_rank(succ, rank, root, ws, o, s) == lr.LR_OK  # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        st = lr.lr_rank(succ, rank, root, ws, o, s)
    assert st == lr.LR_OK
    for i, L in enumerate(lists * 2):
        succ.copy_(torch.from_numpy(L.succ.view(np.int32)))
        rank.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _, er, et, _ = oracle.rank(L.succ)
        assert np.array_equal(host_u32(rank), er), f"replay {i}"
        assert np.array_equal(host_u32(root), et), f"replay {i}"
        torch.empty(1 << 20, device="cuda").normal_()  # unrelated work between replays


@pytest.fixture
def empty_cache():
    lr.autotune_cache_clear()
    yield
    lr.autotune_cache_clear()


@pytest.mark.parametrize("weighted", [False, True])
def test_autotune_returns_valid_options(weighted, empty_cache):
    n = (1 << 22) + 77
    print(f"case: autotune weighted={weighted}", flush=True)
    F = workloads.forest(n, mean=64, n_long=2, long_len=1 << 20, seed=71)
    succ = dev(F.succ)
    w = dev(F.weight) if weighted else None
    ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_I64, lr.make_opts(spacing=(16, 8))) + n * 8 + 4096)
    st, best, ms = lr.lr_autotune(succ, w, ws)
    assert st == lr.LR_OK, lr.status_string(st)
    assert len(ms) >= 4 and all(t > 0 for t in ms)
    ks = [best.spacing[i] for i in range(lr.LR_MAX_LEVELS) if best.spacing[i]]
    assert ks and all(k & (k - 1) == 0 for k in ks)
    p = lr.lr_plan_query(n, lr.LR_W_I64 if weighted else lr.LR_W_NONE, best)
    assert [p.spacing[i] for i in range(p.levels)] == ks
    ost, er, et, es = oracle.rank(F.succ, F.weight if weighted else None)
    if weighted:
        s_, r, t = lr.prefix_sum(succ, w, opts=best)
        torch.cuda.synchronize()
        assert np.array_equal(s_.cpu().numpy(), es) and np.array_equal(host_u32(r), er)
    else:
        r, t = lr.rank(succ, opts=best)
        torch.cuda.synchronize()
        assert np.array_equal(host_u32(r), er) and np.array_equal(host_u32(t), et)


def test_graph_capture_prefix_sum_switching_paths():
    """A captured prefix sum whose automatic choice flips between replays
    (local chains, then a random forest, then local chains again)."""
    n = (1 << 21) + 3
    print(f"case: graph capture prefix sum n={n}", flush=True)
    inputs = []
    for i in range(3):
        if i % 2 == 0:
            L = workloads.gamma_list(n, 0.001, seed=80 + i)
            inputs.append((L.succ, workloads.weights(n, 80 + i, 3, -1000, 1000, np.int64)))
        else:
            F = workloads.forest(n, mean=64, n_long=1, long_len=1 << 19, seed=80 + i)
            inputs.append((F.succ, F.weight))
    succ = dev(inputs[0][0])
    w = dev(inputs[0][1])
    sm = torch.empty(n, dtype=torch.int64, device="cuda")
    rank = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_I64))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        assert lr.lr_prefix_sum(succ, w, sm, rank, None, ws, None, s) == lr.LR_OK
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        st = lr.lr_prefix_sum(succ, w, sm, rank, None, ws, None, s)
    assert st == lr.LR_OK
    for i, (sc, wc) in enumerate(inputs * 2):
        succ.copy_(torch.from_numpy(sc.view(np.int32)))
        w.copy_(torch.from_numpy(wc))
        sm.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _, er, _, es = oracle.rank(sc, wc)
        assert np.array_equal(sm.cpu().numpy(), es), f"replay {i}"
        assert np.array_equal(host_u32(rank), er), f"replay {i}"
        torch.empty(1 << 20, device="cuda").normal_()


def test_autotune_cache_feeds_default_calls(empty_cache, tmp_path):
    """After lr_autotune on a 2^20-element list, calls with default options on
    inputs of the same size bucket take the tuned plan (and still equal the
    oracle), batches of that total too; the entry survives a save/load."""
    n = (1 << 20) + 5
    print("case: autotune cache", flush=True)
    L = workloads.random_list(n, seed=72)
    succ = dev(L.succ)
    ws = lr.workspace(4 * lr.lr_workspace_bytes(n, lr.LR_W_NONE, lr.make_opts(spacing=(16, 8))) + n * 8 + 4096)
    st, best, ms = lr.lr_autotune(succ, None, ws)
    assert st == lr.LR_OK and len(ms) >= 12
    assert lr.autotune_cache_entries() == 1
    tuned = [best.spacing[i] for i in range(lr.LR_MAX_LEVELS) if best.spacing[i]]
    p = lr.lr_plan_query(n)
    assert [p.spacing[i] for i in range(p.levels)][:2] == tuned[:2] and p.base_max == best.base_max
    _, er, et, _ = oracle.rank(L.succ)
    r, t = lr.rank(succ)
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(r), er) and np.array_equal(host_u32(t), et)
    # another list of the same size bucket, alone and as a batch of two
    M = workloads.block_list((1 << 20) + 999, 4096, seed=73)
    m2 = dev(M.succ)
    r2, _ = lr.rank(m2, want_root=False)
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(r2), oracle.rank(M.succ)[1])
    half = [workloads.random_list(600000, seed=74), workloads.random_list(500000, seed=75)]
    items = [(dev(h.succ), torch.full((h.succ.size,), -1, dtype=torch.int32, device="cuda"), None) for h in half]
    reqs = lr.requests(items)
    bws = lr.workspace(lr.lr_batch_workspace_bytes(reqs, 2))
    assert lr.lr_rank_batch(reqs, 2, bws) == lr.LR_OK
    torch.cuda.synchronize()
    for h, (_, rk, _) in zip(half, items):
        assert np.array_equal(host_u32(rk), oracle.rank(h.succ)[1])
    f = str(tmp_path / "tuned.txt")
    assert lr.autotune_cache_save(f) == lr.LR_OK
    lr.autotune_cache_clear()
    assert lr.autotune_cache_load(f) == lr.LR_OK
    p2 = lr.lr_plan_query(n)
    assert [p2.spacing[i] for i in range(p2.levels)] == [p.spacing[i] for i in range(p.levels)]
