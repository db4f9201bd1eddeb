"""Lists whose order is built against the ranking library's ruler sampling
(test inputs only; nothing here ranks anything).

The library's sampler, as its device code documents it: level l with
spacing k = 2^j cuts its ids into blocks of k consecutive ids and makes
exactly one element of every block a ruler, at offset hash32(seed_l, block)
within the block (taken mod the length of a short last block). seed_l is the
low 32 bits of the splitmix64 finaliser of opts.seed * 0x2545f4914f6cdd1d +
0x1000 + l (64-bit arithmetic); hash32 is the "lowbias32" integer hash of
x * 0x9e3779b9 xor the seed. Knowing the seed, an order can put every sampled
ruler after all other elements, so that the walk from the list's head covers
almost the whole list: the case the walk cap and its fallback exist for."""
import numpy as np

import workloads

M64 = (1 << 64) - 1


def mix64(z: int) -> int:
    z = (z + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def level_seed(seed: int, level: int) -> int:
    return mix64((seed * 0x2545F4914F6CDD1D + 0x1000 + level) & M64) & 0xFFFFFFFF


def hash32(seed: int, x: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        h = (x.astype(np.uint32) * np.uint32(0x9E3779B9)) ^ np.uint32(seed)
        h ^= h >> np.uint32(16)
        h *= np.uint32(0x7FEB352D)
        h ^= h >> np.uint32(15)
        h *= np.uint32(0x846CA68B)
        h ^= h >> np.uint32(16)
    return h


def sampled(m: int, k: int, seed_l: int) -> np.ndarray:
    """Ids of the sampled rulers of a level of m elements at spacing k, by block."""
    blocks = np.arange((m + k - 1) // k, dtype=np.uint64)
    base = blocks * np.uint64(k)
    length = np.minimum(np.uint64(k), np.uint64(m) - base)
    h = hash32(seed_l, blocks.astype(np.uint32)).astype(np.uint64)
    pos = np.where(length == k, h & np.uint64(k - 1), h % length)
    return (base + pos).astype(np.uint32)


def rulers_last(n: int, k0: int, seed: int = 0, perm_seed: int = 91) -> workloads.ListInput:
    """One list over [0, n): every other element first (random order), then
    every level-0 sampled ruler (random order)."""
    r = sampled(n, k0, level_seed(seed, 0))
    is_r = np.zeros(n, bool)
    is_r[r] = True
    others = np.nonzero(~is_r)[0].astype(np.uint32)
    others = others[workloads.perm(others.size, perm_seed, 1)]
    r = r[workloads.perm(r.size, perm_seed, 2)]
    order = np.concatenate([others, r])
    return workloads.ListInput(workloads.link_order(order), order)


def level1_rulers_last(n: int, k0: int, k1: int, seed: int = 0, perm_seed: int = 92) -> workloads.ListInput:
    """One list over [0, n) whose level-0 walks are ordinary (the sampled
    rulers spread evenly, k0 - 1 other elements between two of them on
    average) but whose level-1 list is adversarial: the rulers whose block is
    sampled at level 1 come after all other rulers."""
    r0 = sampled(n, k0, level_seed(seed, 0))       # ruler of block c is r0[c]
    S = r0.size
    c1 = sampled(S, k1, level_seed(seed, 1))        # level-1 sampled blocks
    is_c1 = np.zeros(S, bool)
    is_c1[c1] = True
    blocks = np.concatenate([np.nonzero(~is_c1)[0], np.nonzero(is_c1)[0]]).astype(np.int64)
    front = blocks[: S - c1.size][workloads.perm(S - c1.size, perm_seed, 3)]
    back = blocks[S - c1.size:][workloads.perm(c1.size, perm_seed, 4)]
    rseq = r0[np.concatenate([front, back])]
    is_r = np.zeros(n, bool)
    is_r[r0] = True
    others = np.nonzero(~is_r)[0].astype(np.uint32)
    others = others[workloads.perm(others.size, perm_seed, 5)]
    # ruler i follows the i-th of S near-equal chunks of the other elements
    cuts = (np.arange(1, S + 1, dtype=np.int64) * others.size) // S
    parts, lo = [], 0
    for i in range(S):
        parts.append(others[lo:cuts[i]])
        parts.append(rseq[i:i + 1])
        lo = cuts[i]
    order = np.concatenate(parts).astype(np.uint32)
    assert order.size == n
    return workloads.ListInput(workloads.link_order(order), order)


def walk_lengths(order: np.ndarray, is_ruler: np.ndarray) -> np.ndarray:
    """Host model of one level's walks: for a list given by its order, the
    number of elements each walk visits (walks start at every ruler and at the
    head, and stop at the next ruler or after the terminal)."""
    r = np.concatenate([[0], np.nonzero(is_ruler[order])[0], [order.size]])
    r = np.unique(r)
    return np.diff(r)
