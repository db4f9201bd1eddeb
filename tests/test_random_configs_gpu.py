"""Randomised parity: seeded draws of size, input family, path (default,
tile-local contraction forced or forbidden, ruler spawning, visit log forced
on the plain or the contracted list), level spacings, base-case size, the
visit log's offset field width and weight type, each ranked on the GPU and
compared with the oracle element by element. The draws are fixed by the
seed, so a failure names a reproducible case."""
import numpy as np
import pytest

import oracle
import paper_2606_09318_amd as lr
import workloads
from gpu_util import gpu_prefix, gpu_rank

pytestmark = pytest.mark.gpu

FLAG_SETS = [0, lr.LR_LOCAL, lr.LR_NO_LOCAL, lr.LR_SPAWN, lr.LR_NO_LOCAL | lr.LR_VISIT_LOG,
             lr.LR_LOCAL | lr.LR_VISIT_LOG]


def draw(i):
    rng = np.random.default_rng(90210 + i)
    n = int(np.exp(rng.uniform(0, np.log(3000000)))) + 1   # up to 3e6: the automatic choice from 2^21
    family = ["random", "block", "gamma", "forest", "identity"][rng.integers(5)]
    flags = FLAG_SETS[rng.integers(len(FLAG_SETS))]
    spacing = () if rng.random() < 0.5 else tuple(int(2 ** rng.integers(1, 8)) for _ in range(rng.integers(1, 4)))
    base = [0, 16, 256, 4096][rng.integers(4)]
    wt = [None, np.int32, np.int64][rng.integers(3)]
    seed = int(rng.integers(1 << 30))
    bits = [0, 0, 1, 2, 5][rng.integers(5)]  # offset field of packed visit-log records (0 = widest)
    return n, family, flags, spacing, base, wt, seed, bits


def make(n, family, seed):
    if family == "random":
        return workloads.random_list(n, seed=seed).succ
    if family == "block":
        return workloads.block_list(n, block=int(2 ** (seed % 13)), seed=seed).succ
    if family == "gamma":
        return workloads.gamma_list(n, [0.0, 0.01, 0.3][seed % 3], seed=seed).succ
    if family == "forest":
        return workloads.forest(n, mean=[1.5, 8.0, 64.0][seed % 3], n_long=0, long_len=0, seed=seed).succ
    return np.minimum(np.arange(n) + 1, n - 1).astype(np.uint32)


@pytest.mark.parametrize("i", range(200))
def test_random_config(i):
    n, family, flags, spacing, base, wt, seed, bits = draw(i)
    print(f"case {i}: n={n} {family} flags={flags} spacing={spacing} base={base} wt={wt} seed={seed} "
          f"log_off_bits={bits}", flush=True)
    succ = make(n, family, seed)
    o = lr.make_opts(flags=flags, spacing=spacing, base_max=base, seed=seed, log_off_bits=bits)
    if wt is None:
        st, r, t = gpu_rank(succ, o)
        assert st == lr.LR_OK, lr.status_string(st)
        ost, er, et, _ = oracle.rank(succ)
        assert ost == oracle.OK
        assert np.array_equal(r, er) and np.array_equal(t, et)
    else:
        w = workloads.weights(n, seed, 7, -1000, 1000, wt)
        st, s, r, t = gpu_prefix(succ, w, o)
        assert st == lr.LR_OK, lr.status_string(st)
        ost, er, et, es = oracle.rank(succ, w)
        assert ost == oracle.OK
        assert np.array_equal(s, es) and np.array_equal(r, er) and np.array_equal(t, et)
