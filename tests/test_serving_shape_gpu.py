"""Requests of the serving workload's shape: sizes log-uniform over
2^10..2^24 (with both ends of the range present), random-order and
block-local (4096) lists alternating. Every request ranked alone, in one
lr_rank_batch call with the others, and through the continuous-batching
server (batched and one launch per request) gives the same ranks, equal to
the closed form of its generated order (rank of the j-th element in list
order = n - 1 - j; root = the last element)."""
import numpy as np
import pytest
import torch

import paper_2606_09318_amd as lr
import workloads
from gpu_util import dev

pytestmark = pytest.mark.gpu

COUNT = 64


@pytest.fixture(scope="module")
def requests_c5():
    tr = workloads.serving_trace(count=COUNT, lo_log2=10, hi_log2=24, rate_per_s=2000.0, seed=55)
    # both ends of the size range
    tr[0].n = 1 << 10
    tr[1].n = (1 << 24) - 1
    tr[2].n = 1 << 24
    reqs = []
    for q in tr:
        L = workloads.request_input(q)
        reqs.append(dict(n=q.n, kind=q.kind, arrival=q.arrival_s, succ=dev(L.succ), order=dev(L.order),
                         last=int(L.order[-1])))
    sizes = [r["n"] for r in reqs]
    assert min(sizes) == 1 << 10 and max(sizes) == 1 << 24
    assert {r["kind"] for r in reqs} == {"random", "block"}
    return reqs


def closed_form_failures(reqs, ranks, roots) -> list:
    bad = []
    for i, (q, r) in enumerate(zip(reqs, ranks)):
        expect = torch.arange(q["n"] - 1, -1, -1, dtype=torch.int32, device="cuda")
        ok = bool(torch.equal(r.index_select(0, q["order"]), expect))
        if roots is not None and roots[i] is not None:
            ok = ok and bool((roots[i] == q["last"]).all())
        if not ok:
            bad.append(i)
    return bad


def outputs(reqs, with_roots):
    ranks = [torch.full((q["n"],), -1, dtype=torch.int32, device="cuda") for q in reqs]
    roots = [torch.full((q["n"],), -1, dtype=torch.int32, device="cuda") if (with_roots and i % 3 == 0) else None
             for i, q in enumerate(reqs)]
    return ranks, roots


def test_alone_equals_batch_equals_closed_form(requests_c5):
    reqs = requests_c5
    print(f"case: {len(reqs)} serving-shape requests alone and in one batch", flush=True)
    alone = []
    for q in reqs:
        r, _ = lr.rank(q["succ"], want_root=False)
        alone.append(r)
    torch.cuda.synchronize()
    assert closed_form_failures(reqs, alone, None) == []
    ranks, roots = outputs(reqs, True)
    items = [(q["succ"], r, t) for q, r, t in zip(reqs, ranks, roots)]
    creqs = lr.requests(items)
    ws = lr.workspace(lr.lr_batch_workspace_bytes(creqs, len(items)))
    assert lr.lr_rank_batch(creqs, len(items), ws) == lr.LR_OK
    torch.cuda.synchronize()
    assert closed_form_failures(reqs, ranks, roots) == []
    for a, b in zip(alone, ranks):
        assert torch.equal(a, b)


@pytest.mark.parametrize("max_batch,inflight", [(COUNT, 2), (1, 1)])
def test_server_replay_equals_closed_form(requests_c5, max_batch, inflight):
    reqs = requests_c5
    print(f"case: serving-shape replay max_batch={max_batch} inflight={inflight}", flush=True)
    ranks, roots = outputs(reqs, True)
    items = [(q["succ"], r, t) for q, r, t in zip(reqs, ranks, roots)]
    creqs = lr.requests(items)
    cfg = lr.lr_server_config()
    cfg.hbm_budget = 8 << 30
    cfg.max_inflight = inflight
    cfg.max_batch = max_batch
    torch.cuda.synchronize()
    st, lat, sts, mk = lr.lr_server_replay(cfg, creqs, [q["arrival"] for q in reqs], len(reqs))
    assert st == lr.LR_OK and all(s == lr.LR_OK for s in sts)
    assert all(x > 0 for x in lat) and mk > 0
    assert closed_form_failures(reqs, ranks, roots) == []
