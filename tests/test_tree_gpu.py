"""GPU parity of the Euler-tour tree computations (lr_euler_tree): depth,
preorder number and subtree size of every vertex against the oracle's plain
depth-first traversal, bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from gpu_util import dev, host_u32

pytestmark = pytest.mark.gpu


def gpu_tree(E, root=0, opts=None, outputs=(True, True, True)):
    V = E.parent.size
    s = dev(E.succ) if E.succ.size else torch.empty(1, dtype=torch.int32, device="cuda")
    d_, u_ = dev(E.down_arc), dev(E.up_arc)
    outs = [torch.full((V,), -5, dtype=torch.int32, device="cuda") if want else None for want in outputs]
    ws = lr.workspace(lr.lr_euler_tree_workspace_bytes(V, opts))
    st = lr.lr_euler_tree(s, d_, u_, V, root, outs[0], outs[1], outs[2], ws, opts)
    torch.cuda.synchronize()
    return st, [host_u32(o) if o is not None else None for o in outs]


def check(parent, seed=1, opts=None):
    E = workloads.tour_of(parent, seed=seed)
    st, (d, p, z) = gpu_tree(E, 0, opts)
    assert st == lr.LR_OK, lr.status_string(st)
    ost, ed, ep, ez = oracle.tree(parent, 0)
    assert ost == oracle.OK
    assert np.array_equal(d, ed), f"depth mismatch at {np.nonzero(d != ed)[0][:10]}"
    assert np.array_equal(p, ep), f"preorder mismatch at {np.nonzero(p != ep)[0][:10]}"
    assert np.array_equal(z, ez), f"size mismatch at {np.nonzero(z != ez)[0][:10]}"


@pytest.mark.parametrize("V", [1, 2, 3, 4, 17, 1000, 4097, 100003, 1 << 20])
def test_random_recursive_trees(V):
    print(f"case: tree rrt V={V}", flush=True)
    check(workloads.recursive_tree(V, seed=V), seed=V)


@pytest.mark.parametrize("V", [3, 1000, 300007])
def test_relabelled_trees(V):
    """Parents with larger ids than their children; children order by id."""
    print(f"case: tree relabelled V={V}", flush=True)
    check(workloads.relabel_tree(workloads.recursive_tree(V, seed=5), seed=6), seed=7)


def test_path_star_caterpillar():
    V = 200001
    print("case: path / star / caterpillar", flush=True)
    check(np.maximum(np.arange(V) - 1, 0).astype(np.uint32))            # depth V-1: one long chain of arcs
    check(np.zeros(V, np.uint32))                                        # every vertex a child of the root
    cat = np.maximum(np.arange(V) - 1, 0).astype(np.uint32)
    cat[V // 2:] = np.arange(V - V // 2, dtype=np.uint32) % (V // 2)     # spine of V/2 with one leaf each
    check(cat)


@pytest.mark.parametrize("flags", [lr.LR_LOCAL, lr.LR_NO_LOCAL, lr.LR_SPAWN, lr.LR_NO_LOCAL | lr.LR_VISIT_LOG])
def test_modes_and_forced_levels(flags):
    parent = workloads.recursive_tree(300000, seed=8)
    check(parent, opts=lr.make_opts(flags=flags))
    check(parent, opts=lr.make_opts(flags=flags, spacing=(4, 4), base_max=64))


@pytest.mark.parametrize("flags", [0, lr.LR_NO_LOCAL | lr.LR_VISIT_LOG])
def test_optional_outputs_and_other_root(flags):
    """Output subsets and a root other than vertex 0; with the visit log the
    arc weights come from the grouped passes, which skip the root's entry."""
    V = 50000
    opt = lr.make_opts(flags=flags)
    parent = workloads.recursive_tree(V, seed=9)
    E = workloads.tour_of(parent, seed=9)
    _, ed, ep, ez = oracle.tree(parent, 0)
    for mask in [(True, False, False), (False, True, False), (False, False, True), (False, False, False)]:
        st, outs = gpu_tree(E, 0, opt, mask)
        assert st == lr.LR_OK
        for o, e in zip(outs, (ed, ep, ez)):
            if o is not None:
                assert np.array_equal(o, e)
    # the same tree with root and vertex r swapped: depth and size follow the names
    r = 777
    sigma = np.arange(V, dtype=np.uint32)
    sigma[0], sigma[r] = r, 0
    parent2 = np.empty(V, np.uint32)
    parent2[sigma] = sigma[parent]
    E2 = workloads.EulerInput(E.succ, E.weight, parent2, E.down_arc[np.argsort(sigma)], E.up_arc[np.argsort(sigma)],
                              None)
    st, (d, p, z) = gpu_tree(E2, r, opt)
    assert st == lr.LR_OK
    _, d2, _, z2 = oracle.tree(parent2, r)
    assert np.array_equal(d, d2) and np.array_equal(z, z2)
    assert np.array_equal(np.sort(p), np.arange(V)) and p[r] == 0


def test_validate():
    o = lr.make_opts(flags=lr.LR_VALIDATE)
    parent = workloads.recursive_tree(20000, seed=10)
    E = workloads.tour_of(parent, seed=10)
    st, outs = gpu_tree(E, 0, o)               # validating: both weights stored, values as without
    assert st == lr.LR_OK
    _, ed, ep, ez = oracle.tree(parent, 0)
    for got, exp in zip(outs, (ed, ep, ez)):
        assert np.array_equal(got, exp)
    bad = workloads.EulerInput(E.succ, E.weight, parent, E.down_arc.copy(), E.up_arc, None)
    bad.down_arc[5] = E.down_arc[6]                       # one arc named twice, one arc by nobody
    assert gpu_tree(bad, 0, o)[0] == lr.LR_ERR_BAD_LIST
    oob = workloads.EulerInput(E.succ, E.weight, parent, E.down_arc, E.up_arc.copy(), None)
    oob.up_arc[9] = 10 ** 9
    assert gpu_tree(oob, 0, o)[0] == lr.LR_ERR_BAD_LIST
    split = E.succ.copy()
    a = int(E.down_arc[3])
    split[a] = a                                         # the tour cut into two lists
    cut = workloads.EulerInput(split, E.weight, parent, E.down_arc, E.up_arc, None)
    assert gpu_tree(cut, 0, o)[0] == lr.LR_ERR_BAD_LIST
    # without validation the same inputs return without faults
    for X in (bad, oob, cut):
        assert gpu_tree(X, 0, None)[0] == lr.LR_OK
