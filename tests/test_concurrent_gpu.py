"""Calls from several host threads at once, each with its own stream and
workspace (the library's contract: a workspace is never shared by calls that
may overlap): every result equals the oracle. The library's one-time lookups
(device properties, persistent grid sizes) happen inside these calls, so the
first calls of each kind race on them here."""
import threading

import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from gpu_util import dev, host_u32

pytestmark = pytest.mark.gpu


def test_threads_with_own_streams_and_workspaces():
    cases = [
        ("random", workloads.random_list(300_007, seed=61).succ, None),
        ("forest", workloads.forest(200_003, mean=32, n_long=2, long_len=20_000, seed=62).succ, None),
        ("weighted", workloads.forest(150_001, mean=64, n_long=1, long_len=50_000, seed=63).succ,
         workloads.weights(150_001, seed=63, stream=0, lo=-1000, hi=1000)),
        ("visit log", workloads.random_list(1 << 17, seed=64).succ, lr.LR_VISIT_LOG),
    ]
    expect = []
    for name, a, extra in cases:
        w = extra if isinstance(extra, np.ndarray) else None
        expect.append(oracle.rank(a, w))
    errors = []

    def worker(i):
        try:
            name, a, extra = cases[i]
            stream = torch.cuda.Stream()
            w = extra if isinstance(extra, np.ndarray) else None
            flags = extra if isinstance(extra, int) else 0
            with torch.cuda.stream(stream):
                succ = dev(a)
                wt = torch.from_numpy(w).cuda() if w is not None else None
                n = a.size
                o = lr.make_opts(flags=flags)
                for rep in range(5):
                    r = torch.full((n,), -1, dtype=torch.int32, device="cuda")
                    t = torch.full((n,), -1, dtype=torch.int32, device="cuda")
                    if wt is None:
                        ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_NONE, o))
                        st = lr.lr_rank(succ, r, t, ws, o, stream)
                        s = None
                    else:
                        s = torch.empty(n, dtype=torch.int64, device="cuda")
                        ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_I64, o))
                        st = lr.lr_prefix_sum(succ, wt, s, r, t, ws, o, stream)
                    stream.synchronize()
                    ost, er, et, es = expect[i]
                    if st != lr.LR_OK or not np.array_equal(host_u32(r), er) or not np.array_equal(host_u32(t), et):
                        errors.append((name, rep, st))
                    if s is not None and not np.array_equal(s.cpu().numpy(), es):
                        errors.append((name, rep, "sum"))
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append((i, repr(e)))

    print("case: four threads, own streams and workspaces", flush=True)
    threads = [threading.Thread(target=worker, args=(i,)) for i in range(len(cases))]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
        assert not th.is_alive()
    assert errors == []
