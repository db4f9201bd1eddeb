"""lr_verify: the device-side check of a result against the local equations
of the definition. Correct outputs pass; a single wrong rank, root or sum
fails, and so do outputs for input with a cycle. Checked at a full workload
size too (the 2^27 forest with int64 weights)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from gpu_util import dev

pytestmark = pytest.mark.gpu


def oracle_outputs(succ_np, w_np=None):
    st, r, t, s = oracle.rank(succ_np, w_np)
    assert st == 0
    return dev(r), dev(t), torch.from_numpy(s).cuda()


@pytest.mark.parametrize("n", [1, 2, 4099, 100_003])
def test_correct_outputs_pass_and_one_wrong_value_fails(n):
    L = workloads.random_list(n, seed=110)
    succ = dev(L.succ)
    r, t, s = oracle_outputs(L.succ)
    assert lr.lr_verify(succ, r, t, s) == lr.LR_OK
    assert lr.lr_verify(succ, rank=r) == lr.LR_OK and lr.lr_verify(succ, root=t) == lr.LR_OK
    j = int(L.order[n // 2])
    for which in ("rank", "root", "sum"):
        rr, tt, ss = r.clone(), t.clone(), s.clone()
        if which == "rank":
            rr[j] += 1
        elif which == "root":
            tt[j] = (int(tt[j]) + 1) % max(n, 2)
        else:
            ss[j] -= 1
        if n == 1 and which == "root":
            continue
        assert lr.lr_verify(succ, rr, tt, ss) == lr.LR_ERR_BAD_LIST, which


def test_weighted_forest_and_cycle():
    F = workloads.forest(200_000, mean=30, n_long=2, long_len=20_000, seed=111)
    succ, w = dev(F.succ), dev(F.weight)
    r, t, s = oracle_outputs(F.succ, F.weight)
    assert lr.lr_verify(succ, r, t, s, weight=w) == lr.LR_OK
    s2 = s.clone()
    s2[int(F.order[5])] += 7
    assert lr.lr_verify(succ, sum_=s2, weight=w) == lr.LR_ERR_BAD_LIST
    # a cycle (0 -> 1 -> 2 -> 0) next to a list: no outputs satisfy the equations
    c = np.array([1, 2, 0, 4, 4], np.uint32)
    cs = dev(c)
    for guess in (np.array([2, 1, 0, 1, 0], np.uint32), np.zeros(5, np.uint32)):
        assert lr.lr_verify(cs, rank=dev(guess)) == lr.LR_ERR_BAD_LIST


def test_library_results_pass_at_full_size():
    n = 1 << 27
    print("case: verify forest 2^27 int64 weights", flush=True)
    F = workloads.forest(n, mean=64, n_long=16, long_len=1 << 20, seed=3)
    succ, w = dev(F.succ), dev(F.weight)
    s, r, t = lr.prefix_sum(succ, w)
    assert lr.lr_verify(succ, r, t, s, weight=w) == lr.LR_OK
    r[12345] += 1
    assert lr.lr_verify(succ, rank=r) == lr.LR_ERR_BAD_LIST
