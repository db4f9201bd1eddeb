"""Batched ranking and the serving loop: every request's result is
bit-identical alone and in the mix, and equals the oracle."""
import ctypes
import itertools

import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from gpu_util import dev, gpu_rank, host_u32

pytestmark = pytest.mark.gpu


def make_requests(sizes, seed):
    items, inputs = [], []
    for i, n in enumerate(sizes):
        L = workloads.random_list(n, seed=seed + i) if i % 2 == 0 else workloads.block_list(n, 4096, seed=seed + i)
        s = dev(L.succ)
        r = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        t = torch.full((n,), -7, dtype=torch.int32, device="cuda") if i % 3 else None
        items.append((s, r, t))
        inputs.append(L)
    return items, inputs


@pytest.mark.parametrize("sizes", [[1], [5, 1, 3], [1000, 17, 65536, 3, 200001, 4096],
                                   [int(2 ** (10 + 6 * ((i * 0.37) % 1))) for i in range(40)]])
def test_batch_equals_alone_and_oracle(sizes):
    print(f"case: batch sizes={sizes[:8]}... count={len(sizes)}", flush=True)
    items, inputs = make_requests(sizes, seed=1000)
    reqs = lr.requests(items)
    ws = lr.workspace(lr.lr_batch_workspace_bytes(reqs, len(items)))
    st = lr.lr_rank_batch(reqs, len(items), ws)
    torch.cuda.synchronize()
    assert st == lr.LR_OK, lr.status_string(st)
    for (s, r, t), L in zip(items, inputs):
        ost, er, et, _ = oracle.rank(L.succ)
        assert np.array_equal(host_u32(r), er)
        if t is not None:
            assert np.array_equal(host_u32(t), et)
        st, ar, at = gpu_rank(L.succ)
        assert np.array_equal(ar, host_u32(r))


def test_batch_of_every_tiny_forest():
    forests = []
    for n in range(1, 6):
        for succ in itertools.product(range(n), repeat=n):
            a = np.array(succ, np.uint32)
            if oracle.rank(a)[0] == oracle.OK:
                forests.append(a)
    print(f"case: batch of {len(forests)} tiny forests", flush=True)
    items = [(dev(a), torch.empty(a.size, dtype=torch.int32, device="cuda"),
              torch.empty(a.size, dtype=torch.int32, device="cuda")) for a in forests]
    reqs = lr.requests(items)
    ws = lr.workspace(lr.lr_batch_workspace_bytes(reqs, len(items)))
    assert lr.lr_rank_batch(reqs, len(items), ws) == lr.LR_OK
    torch.cuda.synchronize()
    for a, (_, r, t) in zip(forests, items):
        _, er, et, _ = oracle.rank(a)
        assert np.array_equal(host_u32(r), er) and np.array_equal(host_u32(t), et)


def test_batch_log_mode_without_roots():
    """A batch whose concatenation takes the visit-log path, no root outputs."""
    sizes = [1 << 21, 3, (1 << 21) + 999, 70000, 1]
    items, inputs = [], []
    for i, n in enumerate(sizes):
        L = workloads.random_list(n, seed=500 + i) if i % 2 == 0 else workloads.block_list(n, 4096, seed=500 + i)
        items.append((dev(L.succ), torch.full((n,), -3, dtype=torch.int32, device="cuda"), None))
        inputs.append(L)
    reqs = lr.requests(items)
    assert sum(sizes) >= 1 << 22
    o = lr.make_opts(flags=lr.LR_VISIT_LOG)
    ws = lr.workspace(lr.lr_batch_workspace_bytes(reqs, len(items), o))
    assert lr.lr_rank_batch(reqs, len(items), ws, o) == lr.LR_OK
    torch.cuda.synchronize()
    for (s, r, t), L in zip(items, inputs):
        assert np.array_equal(host_u32(r), oracle.rank(L.succ)[1])


@pytest.mark.parametrize("with_forest", [False, True])
def test_batch_of_single_lists_and_a_forest(with_forest):
    """Every request one list: each request's head comes from its own head
    sum and no predecessor marks are needed; one request that is a forest of
    several lists (and an empty request) sends the batch down the marking
    path. Both against the oracle, in the visit-log path and below it."""
    sizes = [1 << 20, 5000, 1, (1 << 19) + 7, 0, 70001]
    items, inputs = [], []
    for i, n in enumerate(sizes):
        if n == 0:
            a = np.zeros(0, np.uint32)
        elif with_forest and i == 3:
            a = workloads.forest(n, mean=50, n_long=2, long_len=10000, seed=600 + i).succ
        else:
            a = (workloads.random_list(n, seed=600 + i) if i % 2 == 0 else workloads.block_list(n, 4096, seed=600 + i)).succ
        inputs.append(a)
        items.append((dev(a) if n else torch.empty(0, dtype=torch.int32, device="cuda"),
                      torch.full((max(n, 1),), -5, dtype=torch.int32, device="cuda")[:n],
                      torch.full((max(n, 1),), -5, dtype=torch.int32, device="cuda")[:n]))
    print(f"case: batch of single lists, forest={with_forest}", flush=True)
    reqs = lr.requests(items)
    for flags in (0, lr.LR_VISIT_LOG | lr.LR_NO_LOCAL):
        o = lr.make_opts(flags=flags)
        ws = lr.workspace(lr.lr_batch_workspace_bytes(reqs, len(items), o))
        assert lr.lr_rank_batch(reqs, len(items), ws, o) == lr.LR_OK
        torch.cuda.synchronize()
        for a, (_, r, t) in zip(inputs, items):
            if a.size == 0:
                continue
            _, er, et, _ = oracle.rank(a)
            assert np.array_equal(host_u32(r), er) and np.array_equal(host_u32(t), et)


def test_batch_forced_levels():
    sizes = [3000, 50000, 1, 70000, 999]
    items, inputs = make_requests(sizes, seed=77)
    reqs = lr.requests(items)
    o = lr.make_opts(spacing=(4, 4, 2), base_max=32)
    ws = lr.workspace(lr.lr_batch_workspace_bytes(reqs, len(items), o))
    assert lr.lr_rank_batch(reqs, len(items), ws, o) == lr.LR_OK
    torch.cuda.synchronize()
    for (s, r, t), L in zip(items, inputs):
        assert np.array_equal(host_u32(r), oracle.rank(L.succ)[1])


@pytest.mark.parametrize("max_batch,inflight", [(1, 1), (8, 2), (64, 2)])
def test_server_replay_results_match_solo(max_batch, inflight):
    tr = workloads.serving_trace(count=48, lo_log2=10, hi_log2=17, rate_per_s=4000.0, seed=5)
    print(f"case: server replay max_batch={max_batch} inflight={inflight}", flush=True)
    items, inputs = [], []
    for q in tr:
        L = workloads.request_input(q)
        items.append((dev(L.succ), torch.full((q.n,), -1, dtype=torch.int32, device="cuda"),
                      torch.full((q.n,), -1, dtype=torch.int32, device="cuda")))
        inputs.append(L)
    reqs = lr.requests(items)
    cfg = lr.lr_server_config()
    cfg.hbm_budget = 256 << 20
    cfg.max_inflight = inflight
    cfg.max_batch = max_batch
    torch.cuda.synchronize()
    st, lat, sts, mk = lr.lr_server_replay(cfg, reqs, [q.arrival_s for q in tr], len(tr))
    assert st == lr.LR_OK
    assert all(s == lr.LR_OK for s in sts)
    assert all(x > 0 for x in lat) and mk > 0
    for (s, r, t), L in zip(items, inputs):
        expect = np.empty(L.succ.size, np.uint32)
        expect[L.order] = np.arange(L.succ.size - 1, -1, -1, dtype=np.uint32)
        assert np.array_equal(host_u32(r), expect)
        assert np.all(host_u32(t) == L.order[-1])


def test_server_rejects_oversize_request_alone():
    small = workloads.random_list(1000, seed=1)
    big = workloads.random_list(1 << 20, seed=2)
    items = [(dev(small.succ), torch.empty(1000, dtype=torch.int32, device="cuda"), None),
             (dev(big.succ), torch.empty(1 << 20, dtype=torch.int32, device="cuda"), None),
             (dev(small.succ), torch.empty(1000, dtype=torch.int32, device="cuda"), None)]
    reqs = lr.requests(items)
    cfg = lr.lr_server_config()
    cfg.hbm_budget = 4 << 20     # fits the small requests only
    cfg.max_inflight = 1
    cfg.max_batch = 4
    st, lat, sts, mk = lr.lr_server_replay(cfg, reqs, [0.0, 0.0001, 0.0002], 3)
    assert st == lr.LR_OK
    assert sts == [lr.LR_OK, lr.LR_ERR_WORKSPACE, lr.LR_OK]
    expect = oracle.rank(small.succ)[1]
    assert np.array_equal(host_u32(items[0][1]), expect) and np.array_equal(host_u32(items[2][1]), expect)
