"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (default options). Every output element is checked: against
the closed form of the generated order where one exists, otherwise against
the local certificate (whose solution on a valid forest is unique) and the
Euler-tour depth recurrence."""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from gpu_util import certificate_gpu, dev, host_u32

pytestmark = pytest.mark.gpu


def closed_form_ok(rank, root, order_np):
    n = order_np.size
    order = dev(order_np)
    expect = torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda")
    ok = bool(torch.equal(rank.index_select(0, order), expect))
    return ok and bool((root == int(order_np[-1])).all())


def test_wide_visit_log_above_2p28():
    """Above 2^28 elements the visit log keeps wide 12-byte records (the packed
    64-bit ones hold up to 2^28): ranks and roots of a random list of
    2^28 + 4097 elements equal the closed form of its generator."""
    n = (1 << 28) + 4097
    print(f"case: wide visit log n={n}", flush=True)
    L = workloads.random_list(n, seed=41)
    succ = dev(L.succ)
    r, t = lr.rank(succ)
    torch.cuda.synchronize()
    assert closed_form_ok(r, t, L.order)


@pytest.mark.timeout(300)
def test_largest_input_2p31_minus_1():
    """The largest input the boundary takes (n = 2^31 - 1; indices and ranks
    are uint32 below 2^31): a random list whose order is a keyed Feistel
    permutation of [0, n) (cycle walking), computed on the device (the host
    generator takes minutes at this size). Every rank and root equals the
    closed form of that order, and the result passes lr_verify."""
    n = (1 << 31) - 1
    torch.cuda.empty_cache()
    print(f"case: largest input n={n}: order and successors", flush=True)
    succ, order32 = workloads.random_list_device(n)
    torch.cuda.empty_cache()
    print("case: largest input: ranking", flush=True)
    r, t = lr.rank(succ)
    torch.cuda.synchronize()
    print("case: largest input: checking", flush=True)
    assert bool((t == order32[-1]).all())
    got = r.index_select(0, order32)
    expect = torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda")
    assert torch.equal(got, expect)  # also proves order32 a permutation: ranks are n distinct values
    del got, expect
    assert lr.lr_verify(succ, rank=r, root=t) == lr.LR_OK
    del succ, r, t, order32
    torch.cuda.empty_cache()


def test_packed_visit_log_continuations_2p28():
    """The 2^28 random list with the visit log's offset field cut to 4 bits:
    a walk takes a continuation id every 16 visits (about 16 M of them, from
    wavefront-owned blocks); every rank and root still equals the closed form
    of the generator."""
    n = 1 << 28
    print("case: packed visit log, 4-bit offsets, n=2^28", flush=True)
    L = workloads.random_list(n, seed=2, stream=0)
    succ = dev(L.succ)
    r, t = lr.rank(succ, opts=lr.make_opts(log_off_bits=4))
    torch.cuda.synchronize()
    assert closed_form_ok(r, t, L.order)


@pytest.mark.parametrize("kind", ["random", "block4096"])
def test_single_list_2p28(kind):
    n = 1 << 28
    print(f"case: {kind} list n=2^28", flush=True)
    L = workloads.random_list(n, seed=2, stream=0) if kind == "random" else \
        workloads.block_list(n, block=4096, seed=2, stream=1)
    succ = dev(L.succ)
    r, t = lr.rank(succ)
    torch.cuda.synchronize()
    assert closed_form_ok(r, t, L.order)
    assert certificate_gpu(succ, r, t)
    if kind == "random":
        # the GPU baseline agrees bit for bit
        r2 = torch.empty_like(r)
        t2 = torch.empty_like(t)
        del L
        ws = lr.workspace(lr.lr_wyllie_workspace_bytes(n))
        assert lr.lr_rank_wyllie(succ, r2, t2, ws) == lr.LR_OK
        torch.cuda.synchronize()
        assert torch.equal(r, r2) and torch.equal(t, t2)
    torch.cuda.empty_cache()


def test_forest_2p27_int64_weights():
    n = 1 << 27
    print("case: forest n=2^27 geometric(64) + 16 x 2^20, int64 weights", flush=True)
    F = workloads.forest(n, mean=64, n_long=16, long_len=1 << 20, seed=3)
    succ, w = dev(F.succ), dev(F.weight)
    s, r, t = lr.prefix_sum(succ, w)
    torch.cuda.synchronize()
    assert certificate_gpu(succ, r, t, s, w)
    # each list's ranks are a permutation of 0..len-1 and |S| stays in int64
    lens = torch.bincount(t.to(torch.int64), minlength=n)
    assert bool((r.to(torch.int64) < lens.index_select(0, t.to(torch.int64))).all())
    assert int(lens.max()) == 1 << 20
    # spot check whole lists against the generator's order
    for i in list(range(0, F.starts.size - 1, (F.starts.size - 1) // 64)) + [F.starts.size - 2]:
        a, b = int(F.starts[i]), int(F.starts[i + 1])
        ids = torch.from_numpy(F.order[a:b].astype(np.int64)).cuda()
        assert torch.equal(r.index_select(0, ids).cpu(), torch.arange(b - a - 1, -1, -1, dtype=torch.int32))
    torch.cuda.empty_cache()


def test_euler_tour_2p26_depths():
    V = 1 << 26
    print("case: Euler tour of a random recursive tree, V=2^26", flush=True)
    E = workloads.euler_tour(V, seed=4)
    succ, w = dev(E.succ), dev(E.weight)
    s, r, t = lr.prefix_sum(succ, w)
    torch.cuda.synchronize()
    assert certificate_gpu(succ, r, t, s, w)
    m = E.succ.size
    idx = torch.arange(m, dtype=torch.int32, device="cuda")
    head = int(torch.nonzero(r == m - 1)[0])
    down = dev(E.down_arc[1:].view(np.int32) if E.down_arc.dtype == np.uint32 else E.down_arc[1:])
    depth = s[head] - s.index_select(0, down) + 1
    assert torch.equal(depth.cpu(), torch.from_numpy(E.depth[1:].astype(np.int64)))
    del idx
    torch.cuda.empty_cache()


def test_euler_tree_2p26():
    """Tree computations on the 2^26-vertex random recursive tree, every vertex
    checked twice: against the oracle's depth-first traversal, and against a
    complete certificate evaluated on the device (children in ascending id
    order): depth(v) = depth(parent) + 1, size(v) = 1 + the sizes of v's
    children, preorder(first child of v) = preorder(v) + 1 and
    preorder(next sibling) = preorder(sibling) + size(sibling). These
    equations, with the root's depth 0 and preorder 0, have exactly one
    solution, so passing them is exactness without the oracle."""
    V = 1 << 26
    print(f"case: euler tree V={V}", flush=True)
    E = workloads.euler_tour(V, seed=4)
    d, p, z = lr.euler_tree(dev(E.succ), dev(E.down_arc), dev(E.up_arc), 0)
    torch.cuda.synchronize()
    st, ed, ep, ez = oracle.tree(E.parent, 0)
    assert st == 0
    assert np.array_equal(host_u32(d), ed)
    assert np.array_equal(host_u32(p), ep)
    assert np.array_equal(host_u32(z), ez)
    # the certificate, on the device
    par = dev(E.parent).long()
    nr = torch.arange(V, device="cuda") != 0
    dl, pl, zl = d.long(), p.long(), z.long()
    assert int(d[0]) == 0 and int(p[0]) == 0
    assert torch.equal(dl[nr], dl[par[nr]] + 1)
    child_sum = torch.zeros(V, dtype=torch.int64, device="cuda").index_add_(0, par[nr], zl[nr])
    assert torch.equal(zl, child_sum + 1)
    kids = torch.nonzero(nr).squeeze(1)
    kids = kids[torch.argsort(par[kids] * V + kids)]      # children grouped by parent, ascending ids
    kp = par[kids]
    first = torch.ones_like(kp, dtype=torch.bool)
    first[1:] = kp[1:] != kp[:-1]
    assert torch.equal(pl[kids[first]], pl[kp[first]] + 1)
    nxt, prev = kids[1:][~first[1:]], kids[:-1][~first[1:]]
    assert torch.equal(pl[nxt], pl[prev] + zl[prev])


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n", [(1 << 25) - 1, 1 << 25, (3 << 26) - 1, 3 << 26])
def test_planner_thresholds(n):
    """Sizes on both sides of the planner's switches: short walks, a doubled
    base case and random slot stores below 2^25, the visit log and
    first-level spacing 32 from 2^25, spacing 64 from 3 * 2^26. Every rank and
    root equals the closed form of a device-generated order."""
    torch.cuda.empty_cache()
    print(f"case: planner threshold n={n}", flush=True)
    succ, order = workloads.random_list_device(n)
    r, t = lr.rank(succ)
    torch.cuda.synchronize()
    assert bool((t == order[-1]).all())
    assert torch.equal(r.index_select(0, order), torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda"))
    del succ, order, r, t
    torch.cuda.empty_cache()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n", [(1 << 25) - 1, (1 << 27) - 1, 1 << 27])
def test_planner_thresholds_weighted(n):
    """Weighted inputs on both sides of their switches (short walks and an
    8192-element base case below 2^25, first-level spacing 64 from 2^27):
    every prefix sum equals the sum of the weights from the element up to its
    list's tail (the tail's own weight not included), taken in list order."""
    torch.cuda.empty_cache()
    print(f"case: weighted planner threshold n={n}", flush=True)
    succ, order = workloads.random_list_device(n)
    g = torch.Generator(device="cuda")
    g.manual_seed(n)
    w = torch.randint(-(1 << 40), 1 << 40, (n,), dtype=torch.int64, device="cuda", generator=g)
    s, r, t = lr.prefix_sum(succ, w)
    torch.cuda.synchronize()
    ws = w.index_select(0, order)
    ws[-1] = 0
    expect = torch.flip(torch.cumsum(torch.flip(ws, [0]), 0), [0])
    assert torch.equal(s.index_select(0, order), expect)
    assert torch.equal(r.index_select(0, order), torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda"))
    assert bool((t == order[-1]).all())
    del succ, order, w, s, r, t, ws, expect
    torch.cuda.empty_cache()
