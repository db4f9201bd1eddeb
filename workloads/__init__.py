"""Seeded synthetic workloads for list ranking (input generators only).

The inputs follow the paper's instance families (Section 3, "Input
Instances"): random lists (List(n, gamma=1)), lists with locality, forests of
lists, and Euler tours of trees. Each generator builds its lists from an
explicit visiting order, so the expected ranks are known in closed form from
that order; nothing here ranks a list.

Both the CPU oracle tests and the GPU path draw their inputs from here, and
this module imports neither of them.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libworkloads.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator library (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    u64, u32p = ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32)
    vp = ctypes.c_void_p
    lib.wl_draw.restype = u64
    lib.wl_draw.argtypes = [u64, u64, u64]
    lib.wl_perm.argtypes = [u64, u64, u64, vp]
    lib.wl_link_order.argtypes = [vp, u64, vp]
    lib.wl_block_order.argtypes = [u64, u64, u64, u64, vp]
    lib.wl_gamma_order.argtypes = [u64, u64, u64, u64, vp]
    lib.wl_forest_lengths.restype = u64
    lib.wl_forest_lengths.argtypes = [u64, u64, ctypes.c_double, u64, u64, vp, u64]
    lib.wl_link_chunks.argtypes = [vp, vp, u64, vp]
    lib.wl_weights_i64.argtypes = [u64, u64, u64, ctypes.c_int64, ctypes.c_int64, vp]
    lib.wl_weights_i32.argtypes = [u64, u64, u64, ctypes.c_int32, ctypes.c_int32, vp]
    lib.wl_recursive_tree.argtypes = [u64, u64, vp]
    lib.wl_tree_depth.argtypes = [vp, u64, vp]
    lib.wl_euler_tour.restype = ctypes.c_int
    lib.wl_euler_tour.argtypes = [u64, vp, u64, vp, vp, vp, vp]
    del u32p
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def draw(seed: int, stream: int, i: int) -> int:
    return int(_load().wl_draw(seed, stream, i))


def perm(n: int, seed: int, stream: int = 0) -> np.ndarray:
    """Pseudorandom permutation of [0, n) as uint32 (keyed Feistel + cycle walking)."""
    out = np.empty(n, dtype=np.uint32)
    if n:
        _load().wl_perm(seed, stream, n, _ptr(out))
    return out


def link_order(order: np.ndarray) -> np.ndarray:
    """Successor array of the single list visiting `order` (last element is the terminal)."""
    order = np.ascontiguousarray(order, dtype=np.uint32)
    succ = np.empty(order.size, dtype=np.uint32)
    if order.size:
        _load().wl_link_order(_ptr(order), order.size, _ptr(succ))
    return succ


def block_order(n: int, block: int, seed: int, stream: int = 0) -> np.ndarray:
    """Visiting order with locality: blocks of `block` consecutive ids in random
    order, each block's ids in random order (the last block may be shorter)."""
    out = np.empty(n, dtype=np.uint32)
    if n:
        _load().wl_block_order(seed, stream, n, block, _ptr(out))
    return out


def gamma_order(n: int, gamma: float, seed: int, stream: int = 0) -> np.ndarray:
    """Visiting order of List(n, gamma): identity order with round(gamma n)
    uniformly chosen positions holding a random permutation of their ids."""
    if not 0.0 <= gamma <= 1.0:
        raise ValueError("gamma must lie in [0, 1]")
    out = np.empty(n, dtype=np.uint32)
    if n:
        _load().wl_gamma_order(seed, stream, n, int(round(gamma * n)), _ptr(out))
    return out


@dataclass
class ListInput:
    succ: np.ndarray          # uint32[n]
    order: np.ndarray         # uint32[n]: visiting order; rank[order[j]] = n-1-j


def random_list(n: int, seed: int = 1, stream: int = 0) -> ListInput:
    """One list over [0, n) in pseudorandom order (the paper's List(n, 1.0))."""
    order = perm(n, seed, stream)
    return ListInput(link_order(order), order)


def feistel_torch(x, keys, half=16):
    """A keyed balanced Feistel network on 2 * half-bit values (half-bit
    halves) in int64 tensor arithmetic (any torch device): a bijection of
    [0, 2^(2 half)), half <= 16."""
    mask = (1 << half) - 1
    lo, hi = x & mask, (x >> half) & mask
    for k in keys:
        f = ((lo * 0x9E37 + k) ^ (lo >> 5) ^ (lo * 0x85EB >> 7)) & mask
        lo, hi = hi ^ f, lo
    return (hi << half) | lo


def feistel32_torch(x, keys):
    """feistel_torch on 32-bit values (16-bit halves)."""
    return feistel_torch(x, keys, 16)


DEVICE_ORDER_KEYS = (0x3A51, 0x7C2D, 0x1E93, 0x5B07)


def random_list_device(n: int, device="cuda", keys=DEVICE_ORDER_KEYS):
    """One list over [0, n) (n <= 2^31 - 1) in the order of a keyed Feistel
    permutation, restricted to [0, n) by cycle walking, built on the device
    for sizes where the host generator takes minutes. Returns (succ int32,
    order int32) tensors; rank[order[j]] = n-1-j."""
    import torch
    assert 0 < n < (1 << 31)
    bits = 2
    while (1 << bits) < n:
        bits += 1
    bits += bits & 1
    half = bits // 2  # the smallest even-width domain that holds [0, n): at most 4 n values
    order = feistel_torch(torch.arange(n, dtype=torch.int64, device=device), keys, half)
    for _ in range(256):  # each walk step leaves a value outside [0, n) with probability <= 3/4
        out = order >= n
        if not bool(out.any()):
            break
        order[out] = feistel_torch(order[out], keys, half)
    if bool((order >= n).any()):
        raise RuntimeError("cycle walking did not finish")
    succ = torch.empty(n, dtype=torch.int32, device=device)
    succ[order[:-1]] = order[1:].to(torch.int32)
    succ[order[-1:]] = order[-1:].to(torch.int32)
    order32 = order.to(torch.int32)
    del order, out
    return succ, order32


def block_list(n: int, block: int = 4096, seed: int = 2, stream: int = 1) -> ListInput:
    """One list with block locality (blocks of `block` ids, chained in random order)."""
    order = block_order(n, block, seed, stream)
    return ListInput(link_order(order), order)


def gamma_list(n: int, gamma: float, seed: int = 6, stream: int = 0) -> ListInput:
    """The paper's List(n, gamma): locality from gamma = 0 (succ[i] = i + 1)
    to gamma = 1 (a random list)."""
    order = gamma_order(n, gamma, seed, stream)
    return ListInput(link_order(order), order)


def striped_list(n: int, tile: int, stride: int, seed: int = 7, stream: int = 2) -> ListInput:
    """One list whose tiles t = 0, stride, 2*stride, ... (of `tile` ids each)
    are walked in id order as one stretch, while every other element sits at
    a random place between the stretches: local where a strided sample looks,
    random almost everywhere else."""
    ntiles = (n + tile - 1) // tile
    kept = np.arange(0, ntiles, stride, dtype=np.int64)
    is_kept = np.zeros(ntiles, bool)
    is_kept[kept] = True
    tile_of = np.arange(n, dtype=np.int64) // tile
    loose = np.flatnonzero(~is_kept[tile_of]).astype(np.int64)
    # units: one per kept tile (ids 0..len(kept)-1), one per loose element
    nu = kept.size + loose.size
    units = perm(nu, seed, stream).astype(np.int64)
    is_tile = units < kept.size
    tile_first = kept[units[is_tile]] * tile
    lens = np.ones(nu, np.int64)
    lens[is_tile] = np.minimum(tile, n - tile_first)
    first = np.empty(nu, np.int64)
    first[is_tile] = tile_first
    first[~is_tile] = loose[units[~is_tile] - kept.size]
    starts = np.concatenate(([0], np.cumsum(lens)))
    order = np.repeat(first, lens) + (np.arange(n, dtype=np.int64) - np.repeat(starts[:-1], lens))
    order = order.astype(np.uint32)
    return ListInput(link_order(order), order)


def identity_list(n: int) -> ListInput:
    """succ[i] = i + 1: the paper's List(n, 0.0) on one PE."""
    order = np.arange(n, dtype=np.uint32)
    return ListInput(link_order(order), order)


@dataclass
class ForestInput:
    succ: np.ndarray          # uint32[n]
    weight: np.ndarray        # int64[n] or int32[n]
    order: np.ndarray         # uint32[n]; list i visits order[starts[i]:starts[i+1]]
    starts: np.ndarray        # int64[count+1]


def forest_lengths(seed: int, short_total: int, mean: float, n_long: int, long_len: int) -> np.ndarray:
    lib = _load()
    cnt = int(lib.wl_forest_lengths(seed, short_total, mean, n_long, long_len, None, 0))
    lens = np.empty(cnt, dtype=np.uint64)
    lib.wl_forest_lengths(seed, short_total, mean, n_long, long_len, _ptr(lens), cnt)
    return lens


def forest(n: int, mean: float = 64.0, n_long: int = 16, long_len: int = 1 << 20, seed: int = 3,
           wlo: int = -1000, whi: int = 1000, wdtype=np.int64) -> ForestInput:
    """Forest of lists: geometric lengths (support {1, 2, ...}, given mean) filling
    n - n_long*long_len elements, the last truncated, plus n_long long lists;
    ids placed in pseudorandom order; per-element weights uniform in [wlo, whi]."""
    short_total = n - n_long * long_len
    if short_total < 0:
        raise ValueError("long lists exceed n")
    lens = forest_lengths(seed, short_total, mean, n_long, long_len)
    starts = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens.astype(np.int64), out=starts[1:])
    order = perm(n, seed, 33)
    succ = np.empty(n, dtype=np.uint32)
    if n:
        _load().wl_link_chunks(_ptr(order), _ptr(starts), lens.size, _ptr(succ))
    w = weights(n, seed, 35, wlo, whi, wdtype)
    return ForestInput(succ, w, order, starts)


def weights(n: int, seed: int, stream: int, lo: int, hi: int, dtype=np.int64) -> np.ndarray:
    w = np.empty(n, dtype=dtype)
    if n:
        if dtype == np.int64:
            _load().wl_weights_i64(seed, stream, n, lo, hi, _ptr(w))
        elif dtype == np.int32:
            _load().wl_weights_i32(seed, stream, n, lo, hi, _ptr(w))
        else:
            raise TypeError(dtype)
    return w


@dataclass
class EulerInput:
    succ: np.ndarray          # uint32[2(V-1)]
    weight: np.ndarray        # int32: +1 down arcs, -1 up arcs
    parent: np.ndarray        # uint32[V]
    down_arc: np.ndarray      # uint32[V]: arc id of parent(v) -> v (entry 0 unused)
    up_arc: np.ndarray        # uint32[V]: arc id of v -> parent(v) (entry 0 unused)
    depth: np.ndarray | None  # uint32[V]: depth from the parent recurrence (trees with parent[v] < v)


def recursive_tree(V: int, seed: int = 4) -> np.ndarray:
    """Random recursive tree: parent[0] = 0, parent[v] uniform in [0, v)."""
    parent = np.empty(V, dtype=np.uint32)
    if V:
        _load().wl_recursive_tree(seed, V, _ptr(parent))
    return parent


def relabel_tree(parent: np.ndarray, seed: int) -> np.ndarray:
    """The same tree with vertices 1..V-1 renamed by a random permutation (the
    root stays 0), so parents no longer have smaller ids."""
    V = parent.size
    if V < 3:
        return parent.copy()
    sigma = np.concatenate([[0], 1 + perm(V - 1, seed, 61)]).astype(np.uint32)
    out = np.empty(V, dtype=np.uint32)
    out[sigma] = sigma[parent]
    return out


def tour_of(parent: np.ndarray, seed: int = 4) -> EulerInput:
    """Euler tour (arcs in random order, children visited in ascending id
    order) of the tree parent[] rooted at 0."""
    lib = _load()
    parent = np.ascontiguousarray(parent, dtype=np.uint32)
    V = parent.size
    m = 2 * (V - 1) if V >= 2 else 0
    succ = np.empty(m, dtype=np.uint32)
    w = np.empty(m, dtype=np.int32)
    down = np.full(V, 0xFFFFFFFF, dtype=np.uint32)
    up = np.full(V, 0xFFFFFFFF, dtype=np.uint32)
    if V >= 2:
        rc = lib.wl_euler_tour(seed, _ptr(parent), V, _ptr(succ), _ptr(w), _ptr(down), _ptr(up))
        if rc != 0:
            raise MemoryError("wl_euler_tour")
    depth = None
    if V and bool(np.all(parent[1:] < np.arange(1, V, dtype=np.uint32))):
        depth = np.empty(V, dtype=np.uint32)
        lib.wl_tree_depth(_ptr(parent), V, _ptr(depth))
    return EulerInput(succ, w, parent, down, up, depth)


def euler_tour(V: int, seed: int = 4) -> EulerInput:
    """Euler tour of a random recursive tree (parent[v] uniform in [0, v))."""
    return tour_of(recursive_tree(V, seed), seed)


# ------------------------------------------------------------ serving trace --

@dataclass
class Request:
    idx: int
    n: int
    kind: str                 # "random" or "block"
    seed: int
    arrival_s: float


def serving_trace(count: int = 4096, lo_log2: float = 10.0, hi_log2: float = 24.0, rate_per_s: float = 1000.0,
                  seed: int = 5, block: int = 4096) -> list[Request]:
    """Requests with sizes floor(2^U), U ~ U[lo_log2, hi_log2], alternating
    random/block-local order, and Poisson arrivals (exponential gaps, mean 1/rate)."""
    out = []
    t = 0.0
    for i in range(count):
        u = (draw(seed, 51, i) >> 11) / float(1 << 53)
        n = int(math.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)))
        g = ((draw(seed, 53, i) >> 11) + 1) / float(1 << 53)
        t += -math.log(g) / rate_per_s
        out.append(Request(i, n, "random" if i % 2 == 0 else "block", int(draw(seed, 55, i) & 0x7FFFFFFF), t))
    return out


def request_input(req: Request, block: int = 4096) -> ListInput:
    if req.kind == "random":
        return random_list(req.n, seed=req.seed, stream=0)
    return block_list(req.n, block=block, seed=req.seed, stream=1)


# ------------------------------------------------------ named workloads -----

WORKLOADS = {
    "random_2^20": dict(kind="random", n=1 << 20, seed=1),
    "random_2^28": dict(kind="random", n=1 << 28, seed=2),
    "block4096_2^28": dict(kind="block", n=1 << 28, seed=2),
    "forest_2^27": dict(kind="forest", n=1 << 27, seed=3),
    "euler_rrt_2^26": dict(kind="euler", V=1 << 26, seed=4),
}
