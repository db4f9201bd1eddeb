"""Pins for the oracle's tree quantities (oracle_tree: depth, preorder number
with children in ascending id order, subtree size) against facts it does not
compute itself:
  * enumeration of every parent array with at most 6 vertices rooted at 0: the
    oracle accepts exactly the trees, whose number is Cayley's V^(V-2) for a
    fixed root, and its outputs equal a recursive definition (ancestor walks
    for depth, descendant counts for size, recursive traversal for preorder);
  * closed forms for paths and stars;
  * invariants of larger trees (sum of sizes = sum of (depth + 1); preorder is a
    permutation; the descendants of v are exactly the preorder interval
    [pre(v), pre(v) + size(v)));
  * the Euler-tour identities the GPU path uses, evaluated with the list
    ranking oracle: over the tour suffix from arc a, #down + #up = rank(a) and
    #down - #up = sum(a) with weights +1 down / -1 up, so depth, preorder and
    size follow from rank and sum at the head, down(v) and up(v).
"""
import itertools
import sys

import numpy as np
import pytest

import oracle
import workloads


def definitional(parent, root=0):
    """Depth by walking to the root, size by counting descendants, preorder by
    a recursive traversal with children sorted by id. None if not a tree."""
    V = len(parent)
    depth = []
    for v in range(V):
        d, x = 0, v
        while x != root:
            x = parent[x]
            d += 1
            if d > V:
                return None
        depth.append(d)
    anc = [set() for _ in range(V)]
    for v in range(V):
        x = v
        anc[v].add(v)
        while x != root:
            x = parent[x]
            anc[v].add(x)
    size = [sum(1 for u in range(V) if v in anc[u]) for v in range(V)]
    kids = {v: sorted(u for u in range(V) if u != root and parent[u] == v) for v in range(V)}
    pre = [None] * V
    counter = [0]

    def visit(v):
        pre[v] = counter[0]
        counter[0] += 1
        for c in kids[v]:
            visit(c)

    sys.setrecursionlimit(max(1000, 4 * V))
    visit(root)
    return depth, pre, size


@pytest.mark.parametrize("V", [1, 2, 3, 4, 5, 6])
def test_every_parent_array(V):
    trees = 0
    for rest in itertools.product(range(V), repeat=V - 1):
        parent = np.array((0,) + rest, np.uint32)
        st, d, p, z = oracle.tree(parent, 0)
        ref = definitional(list(parent), 0) if all(parent[v] != v for v in range(1, V)) else None
        if ref is None:
            assert st != oracle.OK, parent
            continue
        trees += 1
        assert st == oracle.OK, parent
        assert list(d) == ref[0] and list(p) == ref[1] and list(z) == ref[2], parent
    assert trees == (V ** (V - 2) if V >= 2 else 1)  # Cayley: labelled trees with a given root


def test_path_and_star():
    V = 1000
    st, d, p, z = oracle.tree(np.maximum(np.arange(V) - 1, 0).astype(np.uint32), 0)
    assert st == 0
    assert np.array_equal(d, np.arange(V)) and np.array_equal(p, np.arange(V))
    assert np.array_equal(z, V - np.arange(V))
    st, d, p, z = oracle.tree(np.zeros(V, np.uint32), 0)
    assert st == 0
    assert d[0] == 0 and np.all(d[1:] == 1) and np.array_equal(p, np.arange(V))
    assert z[0] == V and np.all(z[1:] == 1)
    # the same star rooted at the last vertex
    parent = np.full(V, V - 1, np.uint32)
    st, d, p, z = oracle.tree(parent, V - 1)
    assert st == 0 and p[V - 1] == 0 and np.array_equal(p[:-1], np.arange(1, V))


def test_rejects_bad_input():
    assert oracle.tree(np.array([1, 0], np.uint32), 0)[0] != 0          # root is not its own parent
    assert oracle.tree(np.array([0, 2, 1], np.uint32), 0)[0] == oracle.ERR_CYCLE
    assert oracle.tree(np.array([0, 5], np.uint32), 0)[0] == oracle.ERR_RANGE
    assert oracle.tree(np.array([0, 1], np.uint32), 0)[0] == oracle.ERR_RANGE  # a second root


def tree_invariants(parent, root, d, p, z):
    V = parent.size
    assert np.array_equal(np.sort(p), np.arange(V))
    assert int(z.astype(np.int64).sum()) == int((d.astype(np.int64) + 1).sum())
    nr = np.arange(V) != root
    assert np.all(d[nr] == d[parent[nr]] + 1)
    assert np.all(p[nr] > p[parent[nr]]) and np.all(p[nr] < p[parent[nr]] + z[parent[nr]])
    assert z[root] == V and p[root] == 0 and d[root] == 0


@pytest.mark.parametrize("V,relabel", [(100000, False), (100000, True), (7, True)])
def test_invariants_random_trees(V, relabel):
    parent = workloads.recursive_tree(V, seed=21)
    if relabel:
        parent = workloads.relabel_tree(parent, seed=22)
    st, d, p, z = oracle.tree(parent, 0)
    assert st == 0
    tree_invariants(parent, 0, d, p, z)
    if not relabel:
        E = workloads.tour_of(parent, seed=21)
        assert np.array_equal(d, E.depth)


def tour_formulas(E, V):
    """Depth, preorder, size from the list-ranking oracle on the Euler tour."""
    st, r, _, s = oracle.rank(E.succ, E.weight)
    assert st == 0
    m = E.succ.size
    r = r.astype(np.int64)
    h = int(np.nonzero(r == m - 1)[0][0])
    v = np.arange(1, V)
    dv, uv = E.down_arc[v], E.up_arc[v]
    depth = np.zeros(V, np.int64)
    pre = np.zeros(V, np.int64)
    size = np.full(V, V, np.int64)
    depth[1:] = s[h] - s[dv] + 1
    pre[1:] = (r[h] + s[h]) // 2 - (r[dv] + s[dv]) // 2 + 1
    size[1:] = (r[dv] - r[uv] + 1) // 2
    return depth, pre, size


@pytest.mark.parametrize("V,relabel", [(2, False), (3, False), (1000, True), (50000, False), (50000, True)])
def test_euler_tour_identities(V, relabel):
    parent = workloads.recursive_tree(V, seed=23)
    if relabel:
        parent = workloads.relabel_tree(parent, seed=24)
    E = workloads.tour_of(parent, seed=25)
    st, d, p, z = oracle.tree(parent, 0)
    assert st == 0
    depth, pre, size = tour_formulas(E, V)
    assert np.array_equal(depth, d) and np.array_equal(pre, p) and np.array_equal(size, z)


def test_euler_tour_identities_path_and_star():
    for parent in (np.maximum(np.arange(500) - 1, 0).astype(np.uint32), np.zeros(500, np.uint32)):
        E = workloads.tour_of(parent, seed=26)
        st, d, p, z = oracle.tree(parent, 0)
        depth, pre, size = tour_formulas(E, parent.size)
        assert np.array_equal(depth, d) and np.array_equal(pre, p) and np.array_equal(size, z)
