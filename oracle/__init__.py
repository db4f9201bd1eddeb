"""CPU oracle for list ranking -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library does not use it.

`rank(succ, weight=None)` returns (status, rank, root, sum) computed by plain
sequential pointer chasing in C (oracle.c): the definition of list ranking
from Section 1.1 of the paper, written out.

`tree(parent, root)` returns (status, depth, preorder, size) of a rooted tree
by a plain depth-first traversal (children in ascending id order): the tree
quantities that Euler-tour list ranking computes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, ERR_RANGE, ERR_INDEGREE, ERR_CYCLE, ERR_NOMEM, ERR_ARG = 0, -1, -2, -3, -4, -5
_WTYPE = {None: 0, np.dtype(np.int32): 1, np.dtype(np.int64): 2}


def build(force: bool = True) -> str:
    """Compile the oracle with the paper's flags (Section 3: -O3 -march=native)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-march=native", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.oracle_rank.restype = ctypes.c_int
        lib.oracle_rank.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_int, vp, vp, vp]
        lib.oracle_tree.restype = ctypes.c_int
        lib.oracle_tree.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint32, vp, vp, vp]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def rank(succ: np.ndarray, weight: np.ndarray | None = None, want=("rank", "root", "sum")):
    """Rank a forest of lists. Returns (status, rank u32, root u32, sum i64);
    arrays not in `want` are None."""
    succ = np.ascontiguousarray(succ, dtype=np.uint32)
    n = succ.size
    wt = 0
    if weight is not None:
        weight = np.ascontiguousarray(weight)
        wt = _WTYPE[weight.dtype]
        if weight.size != n:
            raise ValueError("weight size")
    r = np.empty(n, dtype=np.uint32) if "rank" in want else None
    t = np.empty(n, dtype=np.uint32) if "root" in want else None
    s = np.empty(n, dtype=np.int64) if "sum" in want else None
    st = _load().oracle_rank(_p(succ), n, _p(weight), wt, _p(r), _p(t), _p(s))
    return st, r, t, s


def tree(parent: np.ndarray, root: int = 0):
    """Depth, preorder number and subtree size of every vertex of the tree
    parent[] (parent[root] == root). Returns (status, depth, preorder, size)."""
    parent = np.ascontiguousarray(parent, dtype=np.uint32)
    V = parent.size
    d = np.empty(V, dtype=np.uint32)
    p = np.empty(V, dtype=np.uint32)
    z = np.empty(V, dtype=np.uint32)
    st = _load().oracle_tree(_p(parent), V, root, _p(d), _p(p), _p(z))
    return st, d, p, z
