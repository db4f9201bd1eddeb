"""lr_rank_noalloc (workspace in a static device array, no allocation) gives
exactly lr_rank's results, on calls in a row whose sizes shrink, so stale
scratch contents from a larger call cannot leak into a smaller one."""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from gpu_util import dev, host_u32

SCRATCH = 128 << 20  # LR_NOALLOC_SCRATCH_BYTES


def max_noalloc_n(opts=None) -> int:
    lo, hi = 1, 1 << 26
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if 0 < lr.lr_workspace_bytes(mid, lr.LR_W_NONE, opts) <= SCRATCH:
            lo = mid
        else:
            hi = mid
    return lo


def both(succ_np, opts=None):
    succ = dev(succ_np)
    n = succ.numel()
    r1 = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    t1 = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    print(f"lr_rank_noalloc n={n}", flush=True)
    s = lr.lr_rank_noalloc(succ, r1, t1, opts)
    torch.cuda.synchronize()
    assert s == lr.LR_OK, lr.status_string(s)
    r2 = torch.full((n,), -2, dtype=torch.int32, device="cuda")
    t2 = torch.full((n,), -2, dtype=torch.int32, device="cuda")
    ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_NONE, opts))
    s = lr.lr_rank(succ, r2, t2, ws, opts)
    torch.cuda.synchronize()
    assert s == lr.LR_OK
    return host_u32(r1), host_u32(t1), host_u32(r2), host_u32(t2)


@pytest.mark.gpu
def test_noalloc_matches_lr_rank_on_shrinking_calls():
    torch.cuda.set_device(0)
    nmax = max_noalloc_n()
    assert nmax > 6_000_000
    # first call: a forest at the largest size the scratch array holds
    F = workloads.forest(nmax, mean=64, n_long=4, long_len=1 << 16, seed=31)
    r1, t1, r2, t2 = both(F.succ)
    assert np.array_equal(r1, r2) and np.array_equal(t1, t2)
    st, er, et, _ = oracle.rank(F.succ)
    assert st == 0 and np.array_equal(r1, er) and np.array_equal(t1, et)
    # second call, smaller: one random list with a ragged tail
    L = workloads.random_list(100_003, seed=32)
    r1, t1, r2, t2 = both(L.succ)
    assert np.array_equal(r1, r2) and np.array_equal(t1, t2)
    st, er, et, _ = oracle.rank(L.succ)
    assert st == 0 and np.array_equal(r1, er) and np.array_equal(t1, et)
    # third call, between the two: a list with mostly tile-local links (the
    # contracted path) and the rank output only
    G = workloads.gamma_list(3_000_017, 0.02, seed=33)
    succ = dev(G.succ)
    r = torch.full((G.succ.size,), -1, dtype=torch.int32, device="cuda")
    print(f"lr_rank_noalloc n={G.succ.size} gamma list", flush=True)
    assert lr.lr_rank_noalloc(succ, r, None) == lr.LR_OK
    torch.cuda.synchronize()
    st, er, _, _ = oracle.rank(G.succ)
    assert np.array_equal(host_u32(r), er)


@pytest.mark.gpu
def test_noalloc_rejects_what_it_cannot_run():
    torch.cuda.set_device(0)
    nmax = max_noalloc_n()
    succ = torch.zeros(nmax + 1, dtype=torch.int32, device="cuda")
    r = torch.empty_like(succ)
    # beyond the scratch array: rejected before any work is enqueued
    assert lr.lr_rank_noalloc(succ, r, None) == lr.LR_ERR_WORKSPACE
    assert lr.lr_rank_noalloc(succ[:10], r[:10], None, lr.make_opts(flags=lr.LR_PROFILE)) == lr.LR_ERR_INVALID_ARG
    assert lr.lr_rank_noalloc(succ[:0], r[:0], None) == lr.LR_OK
