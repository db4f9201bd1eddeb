"""Orders built against the ruler sampling. On the CPU, a model of the walk
lengths shows the problem: with every sampled ruler placed last, the head's
walk covers all other elements, n (1 - 1/k) of them, while on a random order
the longest walk stays a few times k ln(n/k). On the GPU the walk cap (64 k
steps) stops such a walk, the bounded fallback ranks the list, and the
results equal the oracle's."""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_09318_amd as lr
import workloads
from adversarial import level1_rulers_last, level_seed, rulers_last, sampled, walk_lengths

CAP_MULT = 64


def plan_spacings(n, opts=None):
    p = lr.lr_plan_query(n, lr.LR_W_NONE, opts)
    return [int(p.spacing[i]) for i in range(p.levels)]


def test_sampler_model_matches_plan_sizes():
    """The host model of the sampler picks exactly one ruler per block of k
    ids (ceil(n / k) rulers, each inside its block)."""
    for n, k in [(1 << 18, 16), (100_003, 64), (5000, 2)]:
        r = sampled(n, k, level_seed(0, 0))
        assert r.size == -(-n // k)
        assert np.array_equal(r // k, np.arange(r.size))
        assert int(r.max()) < n


def test_host_model_rulers_last_makes_one_long_walk():
    n = 1 << 18
    k0 = plan_spacings(n)[0]
    L = rulers_last(n, k0)
    is_r = np.zeros(n, bool)
    is_r[sampled(n, k0, level_seed(0, 0))] = True
    lens = walk_lengths(L.order, is_r)
    S = int(is_r.sum())
    assert int(lens.max()) == n - S          # the head's walk: every other element
    assert int(lens.max()) > CAP_MULT * k0   # far beyond the cap
    R = workloads.random_list(n, seed=3)
    lens_r = walk_lengths(R.order, is_r)
    assert int(lens_r.max()) < CAP_MULT * k0  # an ordinary order never comes near it
    assert int(lens_r.max()) < 4 * k0 * np.log(S)


def test_host_model_level1_rulers_last():
    n = 1 << 18
    k0, k1 = plan_spacings(n, lr.make_opts(spacing=(16, 16)))[:2]
    L = level1_rulers_last(n, k0, k1)
    r0 = sampled(n, k0, level_seed(0, 0))
    is_r = np.zeros(n, bool)
    is_r[r0] = True
    assert int(walk_lengths(L.order, is_r).max()) < CAP_MULT * k0       # level 0 is ordinary
    # level 1: the rulers in list order, as block ids
    pos = np.empty(n, np.int64)
    pos[L.order] = np.arange(n)
    seq = (L.order[np.sort(pos[r0])] // k0).astype(np.int64)
    is_c1 = np.zeros(r0.size, bool)
    is_c1[sampled(r0.size, k1, level_seed(0, 1))] = True
    assert int(walk_lengths(seq, is_c1).max()) > CAP_MULT * k1           # level 1 is not


def check_rank(succ_np, opts=None):
    succ = torch.from_numpy(succ_np.view(np.int32)).cuda()
    n = succ.numel()
    r = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    t = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    flags = (opts.flags if opts is not None else 0) | lr.LR_PROFILE
    o = lr.make_opts(flags=flags) if opts is None else opts
    o.flags = flags
    ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_NONE, o))
    st = lr.lr_rank(succ, r, t, ws, o)
    fell_back = lr.lr_profile_last()[7]
    torch.cuda.synchronize()
    assert st == lr.LR_OK, lr.status_string(st)
    _, er, et, _ = oracle.rank(succ_np)
    assert np.array_equal(r.cpu().numpy().view(np.uint32), er)
    assert np.array_equal(t.cpu().numpy().view(np.uint32), et)
    return fell_back


@pytest.mark.gpu
@pytest.mark.parametrize("flags", [0, lr.LR_VISIT_LOG | lr.LR_NO_LOCAL, lr.LR_VALIDATE])
def test_rulers_last_falls_back_and_matches_oracle(flags):
    n = 1 << 18
    print(f"case: rulers last, n={n}, flags={flags}", flush=True)
    L = rulers_last(n, plan_spacings(n, lr.make_opts(flags=flags))[0])
    assert check_rank(L.succ, lr.make_opts(flags=flags)) == 1.0
    # another seed samples other rulers: the same list is ordinary then
    assert check_rank(L.succ, lr.make_opts(seed=12345, flags=flags)) == 0.0


@pytest.mark.gpu
def test_rulers_last_above_2p21_sixteen_fold_rounds():
    """Above 2^21 elements the fallback jumps 16 records per round (6 rounds
    here) instead of 128; level 0 through the visit log as well."""
    n = (1 << 22) + 5
    print(f"case: rulers last, n={n}", flush=True)
    L = rulers_last(n, plan_spacings(n)[0])
    assert check_rank(L.succ) == 1.0
    L = rulers_last(n, plan_spacings(n, lr.make_opts(flags=lr.LR_VISIT_LOG | lr.LR_NO_LOCAL))[0])
    assert check_rank(L.succ, lr.make_opts(flags=lr.LR_VISIT_LOG | lr.LR_NO_LOCAL)) == 1.0


@pytest.mark.gpu
def test_level1_rulers_last_falls_back_and_matches_oracle():
    n = 1 << 18
    o = lr.make_opts(spacing=(16, 16))
    print(f"case: level-1 rulers last, n={n}", flush=True)
    L = level1_rulers_last(n, *plan_spacings(n, o)[:2])
    assert check_rank(L.succ, lr.make_opts(spacing=(16, 16))) == 1.0


@pytest.mark.gpu
def test_random_list_never_falls_back():
    L = workloads.random_list(1 << 20, seed=8)
    assert check_rank(L.succ) == 0.0


@pytest.mark.gpu
def test_rulers_last_prefix_sums():
    n = (1 << 18) + 77
    L = rulers_last(n, plan_spacings(n)[0])
    w = workloads.weights(n, seed=9, stream=0, lo=-1000, hi=1000)
    print(f"case: rulers last, prefix sums, n={n}", flush=True)
    succ, wt = torch.from_numpy(L.succ.view(np.int32)).cuda(), torch.from_numpy(w).cuda()
    s, r, t = lr.prefix_sum(succ, wt, opts=lr.make_opts(flags=lr.LR_PROFILE))
    assert lr.lr_profile_last()[7] == 1.0
    torch.cuda.synchronize()
    _, er, et, es = oracle.rank(L.succ, w)
    assert np.array_equal(s.cpu().numpy(), es)
    assert np.array_equal(r.cpu().numpy().view(np.uint32), er)
    assert np.array_equal(t.cpu().numpy().view(np.uint32), et)


@pytest.mark.gpu
def test_batch_with_a_rulers_last_request():
    """A batch holding one adversarial request: the whole batch falls back and
    every request still equals the oracle."""
    sizes = [5000, 1 << 18, 70001, 3]
    inputs, items = [], []
    for i, n in enumerate(sizes):
        a = workloads.random_list(n, seed=70 + i).succ if i != 1 else None
        inputs.append(a)
    # the adversarial request is built against the batch's own sampling: the
    # batch is one forest over the concatenation, so its rulers are those of
    # the concatenated id range
    N = sum(sizes)
    k0 = plan_spacings(N)[0]
    base = sizes[0]
    r = sampled(N, k0, level_seed(0, 0))
    r = r[(r >= base) & (r < base + sizes[1])] - base
    is_r = np.zeros(sizes[1], bool)
    is_r[r] = True
    others = np.nonzero(~is_r)[0].astype(np.uint32)
    order = np.concatenate([others[workloads.perm(others.size, 5, 1)], r[workloads.perm(r.size, 5, 2)]])
    inputs[1] = workloads.link_order(order.astype(np.uint32))
    for a in inputs:
        items.append((torch.from_numpy(a.view(np.int32)).cuda(), torch.full((a.size,), -1, dtype=torch.int32,
                                                                            device="cuda"),
                      torch.full((a.size,), -1, dtype=torch.int32, device="cuda")))
    print("case: batch with a rulers-last request", flush=True)
    reqs = lr.requests(items)
    o = lr.make_opts(flags=lr.LR_PROFILE)
    ws = lr.workspace(lr.lr_batch_workspace_bytes(reqs, len(items), o))
    assert lr.lr_rank_batch(reqs, len(items), ws, o) == lr.LR_OK
    assert lr.lr_profile_last()[7] == 1.0
    torch.cuda.synchronize()
    for a, (_, rk, rt) in zip(inputs, items):
        _, er, et, _ = oracle.rank(a)
        assert np.array_equal(rk.cpu().numpy().view(np.uint32), er)
        assert np.array_equal(rt.cpu().numpy().view(np.uint32), et)
