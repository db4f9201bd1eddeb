"""Batches captured once as a HIP graph (lr_batch_graph) and replayed with
other requests: every replay equals each request ranked alone and the
oracle, whatever the requests (sizes, counts, forests, an order built
against the sampling) as long as they fit the graph's capacity. The graph's
kernels read the actual sizes from the device, including the visit-log
path of large capacities."""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from adversarial import level_seed, sampled
from gpu_util import dev, host_u32

pytestmark = pytest.mark.gpu


def make(kind, n, seed):
    if kind == "random":
        return workloads.random_list(n, seed=seed).succ
    if kind == "block":
        return workloads.block_list(n, 4096, seed=seed).succ
    return workloads.forest(n, mean=40, n_long=2, long_len=max(1, n // 8), seed=seed).succ


def run_graph(g, inputs, roots):
    items = []
    for a, want in zip(inputs, roots):
        n = a.size
        items.append((dev(a), torch.full((n,), -9, dtype=torch.int32, device="cuda"),
                      torch.full((n,), -9, dtype=torch.int32, device="cuda") if want else None))
    reqs = lr.requests(items)
    st = g.launch(reqs, len(items))
    torch.cuda.synchronize()
    return st, items


def check(inputs, items):
    for a, (_, r, t) in zip(inputs, items):
        ost, er, et, _ = oracle.rank(a)
        assert ost == 0
        assert np.array_equal(host_u32(r), er)
        if t is not None:
            assert np.array_equal(host_u32(t), et)
        alone, _ = lr.rank(dev(a), want_root=False)
        torch.cuda.synchronize()
        assert np.array_equal(host_u32(alone), er)


@pytest.mark.parametrize("flags", [0, lr.LR_VISIT_LOG])
def test_graph_replays_with_other_requests(flags):
    cfg = lr.batch_graph_config(max_elements=(1 << 21) + 5, max_requests=16, want_root=True,
                                opts=lr.make_opts(flags=flags))
    ws = lr.workspace(lr.lr_batch_graph_workspace_bytes(cfg))
    g = lr.BatchGraph(cfg, ws)
    sets = [
        [("random", 5000), ("block", 70001), ("random", 1), ("block", 300000)],
        [("random", 1 << 20), ("random", 12345)],
        [("block" if i % 2 else "random", 1000 + 37 * i * i) for i in range(16)],
        [("forest", 200000), ("random", 65536), ("forest", 7)],
        [("random", (1 << 21) + 5)],                       # exactly the capacity
        [("random", 5000), ("block", 70001), ("random", 1), ("block", 300000)],
    ]
    for k, spec in enumerate(sets):
        print(f"case: graph flags={flags} replay {k}: {spec[:4]}", flush=True)
        inputs = [make(kind, n, 900 + 10 * k + i) for i, (kind, n) in enumerate(spec)]
        roots = [(i % 2 == 0) for i in range(len(inputs))]
        st, items = run_graph(g, inputs, roots)
        assert st == lr.LR_OK, lr.status_string(st)
        check(inputs, items)
    g.close()


def test_graph_visit_log_capacity():
    """A capacity above the visit-log threshold (2^25): level 0 goes through
    the visit log and the grouped placement with device-side sizes."""
    cfg = lr.batch_graph_config(max_elements=(1 << 25) + 1000, max_requests=8)
    ws = lr.workspace(lr.lr_batch_graph_workspace_bytes(cfg))
    g = lr.BatchGraph(cfg, ws)
    for k, spec in enumerate([[("random", 3_000_017), ("block", 1_000_000)],
                              [("random", 70001), ("forest", 2_000_000), ("block", 4096)]]):
        print(f"case: graph visit-log capacity, replay {k}", flush=True)
        inputs = [make(kind, n, 950 + 10 * k + i) for i, (kind, n) in enumerate(spec)]
        st, items = run_graph(g, inputs, [False] * len(inputs))
        assert st == lr.LR_OK
        check(inputs, items)
    g.close()


def test_graph_falls_back_on_an_order_against_the_sampling():
    """One request ordered with the level-0 rulers of its id range last (the
    sampling of the concatenation the graph ranks, sized on the device): the
    walk cap and the fallback work with device-side sizes too."""
    sizes = [5000, 1 << 18, 3]
    cfg = lr.batch_graph_config(max_elements=1 << 20, max_requests=4, want_root=True)
    ws = lr.workspace(lr.lr_batch_graph_workspace_bytes(cfg))
    g = lr.BatchGraph(cfg, ws)
    N = sum(sizes)
    k0 = int(lr.lr_plan_query(1 << 20, lr.LR_W_NONE, lr.make_opts(flags=lr.LR_NO_LOCAL)).spacing[0])
    r = sampled(N, k0, level_seed(0, 0))
    r = r[(r >= sizes[0]) & (r < sizes[0] + sizes[1])] - sizes[0]
    is_r = np.zeros(sizes[1], bool)
    is_r[r] = True
    others = np.nonzero(~is_r)[0].astype(np.uint32)
    order = np.concatenate([others[workloads.perm(others.size, 7, 1)], r[workloads.perm(r.size, 7, 2)]])
    inputs = [make("random", sizes[0], 1), workloads.link_order(order.astype(np.uint32)), make("random", 3, 2)]
    print("case: graph with a rulers-last request", flush=True)
    st, items = run_graph(g, inputs, [True, True, False])
    assert st == lr.LR_OK
    check(inputs, items)
    g.close()


def test_graph_rejects_what_it_cannot_run():
    cfg = lr.batch_graph_config(max_elements=100000, max_requests=2)
    ws = lr.workspace(lr.lr_batch_graph_workspace_bytes(cfg))
    g = lr.BatchGraph(cfg, ws)
    a = make("random", 60000, 3)
    b = make("random", 60000, 4)
    st, _ = run_graph(g, [a, b], [False, False])
    assert st == lr.LR_ERR_WORKSPACE                       # 120000 elements > 100000
    st, _ = run_graph(g, [a[:10] * 0 + np.arange(10, dtype=np.uint32)] * 3, [False] * 3)
    assert st == lr.LR_ERR_WORKSPACE                       # 3 requests > 2
    st, _ = run_graph(g, [make("random", 1000, 5)], [True])
    assert st == lr.LR_ERR_INVALID_ARG                     # roots asked, graph made without
    st, items = run_graph(g, [make("random", 1000, 5)], [False])
    assert st == lr.LR_OK
    g.close()
    for flags in (lr.LR_VALIDATE, lr.LR_PROFILE, lr.LR_SPAWN, lr.LR_LOCAL):
        bad = lr.batch_graph_config(max_elements=1000, max_requests=2, opts=lr.make_opts(flags=flags))
        assert lr.lr_batch_graph_workspace_bytes(bad) == 0
        with pytest.raises(lr.LrError):
            lr.BatchGraph(bad, ws)


@pytest.mark.parametrize("max_batch", [64, 4])
def test_server_with_graphs_equals_closed_form(max_batch):
    tr = workloads.serving_trace(count=48, lo_log2=10, hi_log2=20, rate_per_s=4000.0, seed=57)
    print(f"case: server with graphs, max_batch={max_batch}", flush=True)
    items, inputs = [], []
    for i, q in enumerate(tr):
        L = workloads.request_input(q)
        items.append((dev(L.succ), torch.full((q.n,), -1, dtype=torch.int32, device="cuda"),
                      torch.full((q.n,), -1, dtype=torch.int32, device="cuda") if i % 3 == 0 else None))
        inputs.append(L)
    reqs = lr.requests(items)
    cfg = lr.lr_server_config()
    cfg.hbm_budget = 2 << 30
    cfg.max_inflight = 2
    cfg.max_batch = max_batch
    cfg.graphs = 1
    torch.cuda.synchronize()
    st, lat, sts, mk = lr.lr_server_replay(cfg, reqs, [q.arrival_s for q in tr], len(tr))
    assert st == lr.LR_OK and all(s == lr.LR_OK for s in sts)
    for (s, r, t), L in zip(items, inputs):
        expect = np.empty(L.succ.size, np.uint32)
        expect[L.order] = np.arange(L.succ.size - 1, -1, -1, dtype=np.uint32)
        assert np.array_equal(host_u32(r), expect)
        if t is not None:
            assert np.all(host_u32(t) == L.order[-1])
