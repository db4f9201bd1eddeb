"""The write-counting debug build (liblr_debug.so, LR_DEBUG_WRITES=1): every
store that relies on a single writer -- a slot per visited element, a
predecessor mark per element (Section 1.1: in a forest every element has at
most one predecessor) -- counts itself, and a call fails with LR_ERR_BAD_LIST
unless each slot of a chased level was written exactly once and each mark at
most once. Valid inputs pass and equal the oracle; an input with two
predecessors of one element fails in the debug build without LR_VALIDATE,
where the release build, not validating, reports nothing."""
import ctypes
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from paper_2606_09318_amd import build as lr_build

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dbg():
    if not os.path.exists(lr_build.DEBUG_LIB):
        pytest.fail(f"{lr_build.DEBUG_LIB} is missing: run __graft_entry__.build()")
    lr.load()  # torch's HIP runtime first, as the binding does
    L = ctypes.CDLL(lr_build.DEBUG_LIB)
    L.lr_rank.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t,
                                                  ctypes.c_void_p, ctypes.c_void_p]
    L.lr_rank.restype = ctypes.c_int
    L.lr_workspace_bytes.restype = ctypes.c_size_t
    L.lr_workspace_bytes.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
    return L


def run(L, succ_np, opts=None):
    n = succ_np.size
    succ = torch.from_numpy(succ_np.view(np.int32)).cuda()
    r = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    t = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    o = ctypes.byref(opts) if opts is not None else None
    ws = torch.empty(L.lr_workspace_bytes(n, 0, o), dtype=torch.uint8, device="cuda")
    st = L.lr_rank(succ.data_ptr(), r.data_ptr(), t.data_ptr(), n, ws.data_ptr(), ws.numel(), o,
                   torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return st, r.cpu().numpy().view(np.uint32), t.cpu().numpy().view(np.uint32)


CASES = [
    ("random 2^20", lambda: workloads.random_list(1 << 20, seed=31).succ, None),
    ("forest 2^20", lambda: workloads.forest(1 << 20, mean=64, n_long=2, long_len=1 << 16, seed=32).succ, None),
    ("deep recursion", lambda: workloads.random_list(100_003, seed=33).succ, dict(spacing=(2, 2, 2), base_max=64)),
    ("visit log 2^18", lambda: workloads.random_list(1 << 18, seed=34).succ, dict(flags=lr.LR_VISIT_LOG)),
    ("forest, visit log", lambda: workloads.forest(1 << 18, mean=16, n_long=1, long_len=5000, seed=35).succ,
     dict(flags=lr.LR_VISIT_LOG)),
    ("contracted (not counted)", lambda: workloads.block_list(1 << 18, 4096, seed=36).succ, dict(flags=lr.LR_LOCAL)),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_valid_inputs_have_one_writer_per_slot(dbg, name, make, kw):
    print(f"case: debug writes, {name}", flush=True)
    a = make()
    st, r, t = run(dbg, a, lr.make_opts(**kw) if kw else None)
    assert st == lr.LR_OK, lr.status_string(st)
    ost, er, et, _ = oracle.rank(a)
    assert ost == 0
    assert np.array_equal(r, er) and np.array_equal(t, et)


@pytest.mark.parametrize("forest", [False, True])
def test_two_predecessors_counted(dbg, forest):
    """succ[a] = succ[b] for two non-terminals: the element after them is
    marked twice (a forest's predecessor marks), and the elements from it to
    the next ruler are visited twice or the ones the change cut off from
    every walk not at all. A base case of 256 elements makes the 5000-element
    inputs take the ruling-set levels (alone in the base case nothing is
    chased)."""
    print(f"case: debug writes, two predecessors, forest={forest}", flush=True)
    if forest:
        a = workloads.forest(5000, mean=8, n_long=1, long_len=500, seed=37).succ.copy()
    else:
        a = workloads.random_list(5000, seed=38).succ.copy()
    nonterm = np.nonzero(a != np.arange(a.size, dtype=np.uint32))[0]
    x, y = int(nonterm[10]), int(nonterm[2000])
    a[y] = a[x]
    st, _, _ = run(dbg, a, lr.make_opts(base_max=256))
    assert st == lr.LR_ERR_BAD_LIST
    # the release build without validation does not look (unspecified outputs)
    succ = torch.from_numpy(a.view(np.int32)).cuda()
    rel, _ = lr.rank(succ, want_root=False)
    torch.cuda.synchronize()
    # and with validation it reports the input itself
    o = lr.make_opts(flags=lr.LR_VALIDATE)
    ws = lr.workspace(lr.lr_workspace_bytes(a.size, lr.LR_W_NONE, o))
    r = torch.empty(a.size, dtype=torch.int32, device="cuda")
    assert lr.lr_rank(succ, r, None, ws, o) == lr.LR_ERR_BAD_LIST
