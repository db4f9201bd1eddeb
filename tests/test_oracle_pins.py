"""Pins for the CPU oracle against facts it does not compute itself.

Each test checks the oracle (oracle/oracle.c) against something fixed by the
problem definition of Section 1.1 or by mathematics:
  * brute force: every successor array of size <= 7 is enumerated; the number
    of valid ones must equal the number of ways to split n labelled items into
    ordered lists (Lah-number sums), the oracle must accept exactly those, and
    its outputs must equal hop-by-hop stepping from each element;
  * closed forms of generated inputs (a list built from a visiting order has
    rank[order[j]] = n-1-j; forests are chunks of an order; Euler-tour depths
    equal the parent recurrence);
  * the local certificate (rank[t] = 0, rank[x] = rank[succ x] + 1, ...), whose
    solution on a valid forest is unique;
  * hand-worked examples under tests/golden/ and special cases.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


# ---------------------------------------------------------------- helpers --

def certificate(succ, rank=None, root=None, sum_=None, weight=None):
    """Local equations of Section 1.1 that a ranking must satisfy. On a valid
    forest they have exactly one solution (induction from each terminal)."""
    succ = succ.astype(np.int64)
    idx = np.arange(succ.size)
    term = succ == idx
    nt = ~term
    if rank is not None:
        assert np.all(rank[term] == 0)
        assert np.all(rank[nt].astype(np.int64) == rank[succ[nt]].astype(np.int64) + 1)
    if root is not None:
        assert np.all(root[term] == idx[term])
        assert np.all(root[nt] == root[succ[nt]])
    if sum_ is not None:
        w = np.ones(succ.size, np.int64) if weight is None else weight.astype(np.int64)
        assert np.all(sum_[term] == 0)
        assert np.all(sum_[nt] == sum_[succ[nt]] + w[nt])


def lah_sum(n):
    """Number of ways to partition n labelled items into nonempty ordered lists:
    sum over k of the Lah numbers L(n, k) = C(n-1, k-1) n! / k!."""
    if n == 0:
        return 1
    return sum(math.comb(n - 1, k - 1) * math.factorial(n) // math.factorial(k) for k in range(1, n + 1))


def all_arrays(n):
    """Every successor array over [0, n) as rows of an (n**n, n) uint8 matrix."""
    grids = np.indices((n,) * n, dtype=np.uint8).reshape(n, -1).T
    return np.ascontiguousarray(grids)


def brute_force(A):
    """Validity, rank, root and weighted sum by stepping each element one link at
    a time, n times (rows of A are successor arrays)."""
    N, n = A.shape
    rows = np.arange(N)[:, None]
    idx = np.broadcast_to(np.arange(n, dtype=np.int64), (N, n))
    # in-degree of every element, self links excluded
    indeg = np.zeros((N, n), np.int64)
    for i in range(n):
        m = A[:, i] != i
        indeg[np.nonzero(m)[0], A[m, i]] += 1
    X = idx.copy()
    steps = np.zeros((N, n), np.int64)
    for _ in range(n):
        nxt = A[rows, X]
        moving = nxt != X
        steps += moving
        X = np.where(moving, nxt, X)
    reaches_terminal = A[rows, X] == X
    valid = np.all(indeg <= 1, axis=1) & np.all(reaches_terminal, axis=1)
    return valid, steps, X


# ------------------------------------------------------------- brute force --

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_valid_forest_count_matches_lah_numbers(n):
    A = all_arrays(n)
    valid, _, _ = brute_force(A)
    assert int(valid.sum()) == lah_sum(n)
    assert [lah_sum(k) for k in range(8)] == [1, 1, 3, 13, 73, 501, 4051, 37633]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_oracle_equals_stepping_on_every_forest(n):
    A = all_arrays(n)
    valid, steps, X = brute_force(A)
    rng = np.random.default_rng(100 + n)
    V = A[valid]
    W = rng.integers(-50, 51, size=V.shape).astype(np.int64)
    # weighted reference by stepping: add w[x] for each link taken
    N = V.shape[0]
    rows = np.arange(N)[:, None]
    Xw = np.broadcast_to(np.arange(n, dtype=np.int64), (N, n)).copy()
    S = np.zeros((N, n), np.int64)
    for _ in range(n):
        nxt = V[rows, Xw]
        moving = nxt != Xw
        S += np.where(moving, W[rows, Xw], 0)
        Xw = np.where(moving, nxt, Xw)
    vs, vX = steps[valid], X[valid]
    for j in range(N):
        succ = V[j].astype(np.uint32)
        st, r, t, s = oracle.rank(succ, W[j])
        assert st == oracle.OK
        assert np.array_equal(r, vs[j])
        assert np.array_equal(t, vX[j])
        assert np.array_equal(s, S[j])
        st, r2, _, s2 = oracle.rank(succ)
        assert st == oracle.OK and np.array_equal(r2, vs[j]) and np.array_equal(s2, vs[j])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_oracle_rejects_every_invalid_array(n):
    A = all_arrays(n)
    valid, _, _ = brute_force(A)
    for row in A[~valid]:
        st, _, _, _ = oracle.rank(row.astype(np.uint32))
        assert st in (oracle.ERR_INDEGREE, oracle.ERR_CYCLE)


def test_oracle_rejects_sampled_invalid_arrays_n7():
    A = all_arrays(7)
    valid, _, _ = brute_force(A)
    bad = A[~valid]
    pick = np.random.default_rng(7).choice(bad.shape[0], 5000, replace=False)
    for row in bad[pick]:
        assert oracle.rank(row.astype(np.uint32))[0] in (oracle.ERR_INDEGREE, oracle.ERR_CYCLE)


def test_oracle_error_kinds():
    assert oracle.rank(np.array([0, 5], np.uint32))[0] == oracle.ERR_RANGE
    assert oracle.rank(np.array([2, 2, 2], np.uint32))[0] == oracle.ERR_INDEGREE
    assert oracle.rank(np.array([1, 0], np.uint32))[0] == oracle.ERR_CYCLE
    # a pure cycle next to a valid list: no in-degree violation, still rejected
    assert oracle.rank(np.array([1, 1, 3, 2], np.uint32))[0] == oracle.ERR_CYCLE
    assert oracle.rank(np.zeros(0, np.uint32))[0] == oracle.OK


# ----------------------------------------------------------------- golden --

def test_hand_worked_examples():
    cases = json.load(open(GOLDEN))["cases"]
    assert len(cases) >= 5
    for c in cases:
        succ = np.array(c["succ"], np.uint32)
        w = np.array(c["weight"], np.int64) if "weight" in c else None
        st, r, t, s = oracle.rank(succ, w)
        assert st == oracle.OK, c["name"]
        if "rank" in c:
            assert r.tolist() == c["rank"], c["name"]
        if "root" in c:
            assert t.tolist() == c["root"], c["name"]
        if "sum" in c:
            assert s.tolist() == c["sum"], c["name"]
        if "depth" in c:
            head = int(np.setdiff1d(np.arange(succ.size), succ[succ != np.arange(succ.size)])[0])
            for v, d in enumerate(c["depth"]):
                if v:
                    assert s[head] - s[c["down_arc"][v]] + 1 == d


# ---------------------------------------------------------- closed forms ---

@pytest.mark.parametrize("n", [1, 2, 3, 1000, 65537, 1 << 18])
def test_random_list_closed_form(n):
    L = workloads.random_list(n, seed=11)
    st, r, t, s = oracle.rank(L.succ)
    assert st == oracle.OK
    expect = np.empty(n, np.uint32)
    expect[L.order] = np.arange(n - 1, -1, -1, dtype=np.uint32)
    assert np.array_equal(r, expect)
    assert np.all(t == L.order[-1])
    assert np.array_equal(s, expect.astype(np.int64))


@pytest.mark.parametrize("n,block", [(4096 * 3, 4096), (4096 * 5 + 17, 4096), (1000, 64)])
def test_block_list_closed_form(n, block):
    L = workloads.block_list(n, block=block, seed=12)
    st, r, t, _ = oracle.rank(L.succ)
    assert st == oracle.OK
    expect = np.empty(n, np.uint32)
    expect[L.order] = np.arange(n - 1, -1, -1, dtype=np.uint32)
    assert np.array_equal(r, expect)
    assert np.all(t == L.order[-1])


def forest_truth(F):
    """Per-list rank, root and weighted sum from the generation order."""
    n = F.succ.size
    lens = np.diff(F.starts)
    lid = np.repeat(np.arange(lens.size), lens)
    pos = np.arange(n) - F.starts[lid]
    rank_o = (lens[lid] - 1 - pos).astype(np.uint32)
    last = F.order[F.starts[1:] - 1]
    w_o = F.weight[F.order].astype(np.int64)
    w_o[F.starts[1:] - 1] = 0                       # a terminal's weight never counts
    # suffix sums within each chunk of the order
    c = np.cumsum(w_o[::-1])[::-1]
    end_next = np.append(c, 0)[F.starts[1:]]
    sum_o = c - end_next[lid]
    rank, root, sm = (np.empty(n, np.uint32), np.empty(n, np.uint32), np.empty(n, np.int64))
    rank[F.order] = rank_o
    root[F.order] = last[lid]
    sm[F.order] = sum_o
    return rank, root, sm


@pytest.mark.parametrize("n,n_long,long_len", [(20000, 4, 1000), (1 << 18, 16, 4096)])
def test_forest_closed_form(n, n_long, long_len):
    F = workloads.forest(n, mean=64, n_long=n_long, long_len=long_len, seed=13)
    st, r, t, s = oracle.rank(F.succ, F.weight)
    assert st == oracle.OK
    er, et, es = forest_truth(F)
    assert np.array_equal(r, er) and np.array_equal(t, et) and np.array_equal(s, es)
    assert F.starts.size - 1 > n_long  # short lists present


@pytest.mark.parametrize("V", [2, 3, 50, 5000, 1 << 16])
def test_euler_tour_depth(V):
    E = workloads.euler_tour(V, seed=14)
    st, r, t, s = oracle.rank(E.succ, E.weight)
    assert st == oracle.OK
    m = E.succ.size
    head = np.setdiff1d(np.arange(m), E.succ[E.succ != np.arange(m)])
    assert head.size == 1
    h = int(head[0])
    v = np.arange(1, V)
    depth = s[h] - s[E.down_arc[v]] + 1
    assert np.array_equal(depth, E.depth[1:].astype(np.int64))
    # every arc lies on the single tour
    assert np.all(t == t[h]) and r[h] == m - 1


# ----------------------------------------------------- special cases ------

def test_identity_and_reversed_lists():
    n = 1001
    succ = np.minimum(np.arange(n) + 1, n - 1).astype(np.uint32)
    st, r, t, _ = oracle.rank(succ)
    assert st == 0 and np.array_equal(r, np.arange(n - 1, -1, -1)) and np.all(t == n - 1)
    succ = np.maximum(np.arange(n) - 1, 0).astype(np.uint32)
    st, r, t, _ = oracle.rank(succ)
    assert st == 0 and np.array_equal(r, np.arange(n)) and np.all(t == 0)


def test_singletons_and_tiny():
    n = 37
    st, r, t, s = oracle.rank(np.arange(n, dtype=np.uint32), np.full(n, 9, np.int64))
    assert st == 0 and not r.any() and np.array_equal(t, np.arange(n)) and not s.any()
    st, r, t, _ = oracle.rank(np.array([0], np.uint32))
    assert st == 0 and r.tolist() == [0] and t.tolist() == [0]
    st, r, t, _ = oracle.rank(np.array([1, 1], np.uint32))
    assert st == 0 and r.tolist() == [1, 0] and t.tolist() == [1, 1]


def test_unit_weights_equal_ranks_and_terminal_weight_ignored():
    F = workloads.forest(5000, mean=8, n_long=2, long_len=500, seed=15)
    ones = np.ones(F.succ.size, np.int64)
    st, r, _, s = oracle.rank(F.succ, ones)
    assert st == 0 and np.array_equal(s, r.astype(np.int64))
    w = F.weight.copy()
    term = F.succ == np.arange(F.succ.size)
    st, _, _, s1 = oracle.rank(F.succ, w)
    w[term] = 123456
    st2, _, _, s2 = oracle.rank(F.succ, w)
    assert st == st2 == 0 and np.array_equal(s1, s2)


def test_int32_and_int64_weights_agree():
    F = workloads.forest(20000, mean=16, n_long=1, long_len=5000, seed=16)
    st, _, _, s64 = oracle.rank(F.succ, F.weight)
    st2, _, _, s32 = oracle.rank(F.succ, F.weight.astype(np.int32))
    assert st == st2 == 0 and np.array_equal(s64, s32)


def test_relabelling_is_equivariant():
    F = workloads.forest(30000, mean=32, n_long=2, long_len=3000, seed=17)
    n = F.succ.size
    sigma = workloads.perm(n, seed=99)
    succ2 = np.empty(n, np.uint32)
    succ2[sigma] = sigma[F.succ]
    w2 = np.empty_like(F.weight)
    w2[sigma] = F.weight
    st, r, t, s = oracle.rank(F.succ, F.weight)
    st2, r2, t2, s2 = oracle.rank(succ2, w2)
    assert st == st2 == 0
    assert np.array_equal(r2[sigma], r) and np.array_equal(t2[sigma], sigma[t]) and np.array_equal(s2[sigma], s)


@pytest.mark.parametrize("seed", [21, 22])
def test_certificate_on_generated_inputs(seed):
    F = workloads.forest(1 << 17, mean=64, n_long=4, long_len=8192, seed=seed)
    st, r, t, s = oracle.rank(F.succ, F.weight)
    assert st == 0
    certificate(F.succ, r, t, s, F.weight)
    # ranks of each list are a permutation of 0..len-1
    key = t.astype(np.int64) * (1 << 32) + r
    assert np.unique(key).size == key.size
    lens = np.bincount(t, minlength=F.succ.size)
    assert np.all(r < lens[t])


def test_certificate_rejects_planted_mistakes():
    """The certificate itself must catch a wrong sign, a dropped weight and an
    off-by-one, so that passing it means something."""
    F = workloads.forest(4000, mean=16, n_long=1, long_len=300, seed=23)
    st, r, t, s = oracle.rank(F.succ, F.weight)
    certificate(F.succ, r, t, s, F.weight)
    nonterm = np.nonzero(F.succ != np.arange(F.succ.size))[0]
    x = nonterm[0]
    for bad in (lambda a: a.__setitem__(x, a[x] + 1), lambda a: a.__setitem__(x, -a[x] - 1)):
        s2 = s.copy()
        bad(s2)
        with pytest.raises(AssertionError):
            certificate(F.succ, sum_=s2, weight=F.weight)
    r2 = r.copy()
    r2[x] += 1
    with pytest.raises(AssertionError):
        certificate(F.succ, rank=r2)
    with pytest.raises(AssertionError):
        certificate(F.succ, sum_=s, weight=-F.weight)
