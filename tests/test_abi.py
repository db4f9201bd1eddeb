"""The C ABI library loads on a machine without a GPU, exports every function
include/lr.h declares, and answers its host-only queries and argument checks
(no call here reaches a kernel)."""
import ctypes
import os
import re

import pytest

import paper_2606_09318_amd as lr

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "lr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(lr_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = lr.load()
    names = declared_functions()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name


def test_debug_library_exports_the_same_functions_and_larger_workspaces():
    """liblr_debug.so (write counters) has the release library's ABI; its
    workspaces hold the counters as well."""
    from paper_2606_09318_amd import build as lr_build
    lr.load()
    dbg = ctypes.CDLL(lr_build.DEBUG_LIB)
    for name in declared_functions():
        assert hasattr(dbg, name), name
    dbg.lr_workspace_bytes.restype = ctypes.c_size_t
    dbg.lr_workspace_bytes.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
    n = 1 << 20
    assert dbg.lr_workspace_bytes(n, 0, None) >= lr.lr_workspace_bytes(n, lr.LR_W_NONE) + 8 * (n + n // 16)


def test_status_strings():
    for s in range(7):
        assert lr.status_string(s).startswith("LR_")


def test_plan_levels_and_sizes():
    p = lr.lr_plan_query(1 << 28)
    assert p.levels >= 2
    assert p.m[0] == 1 << 28
    for l in range(p.levels):
        k = p.spacing[l]
        assert k & (k - 1) == 0 and 2 <= k <= 4096
        assert p.m[l + 1] == -(-p.m[l] // k)
    assert p.m[p.levels] <= p.base_max
    small = lr.lr_plan_query(5000)
    assert small.levels == 0


def test_plan_honours_spacing_and_base():
    o = lr.make_opts(spacing=(4, 2), base_max=16)
    p = lr.lr_plan_query(1000, lr.LR_W_NONE, o)
    assert [p.spacing[i] for i in range(p.levels)][:2] == [4, 2]
    assert p.m[1] == 250 and p.m[2] == 125
    assert p.m[p.levels] <= 16
    with pytest.raises(lr.LrError):
        lr.lr_plan_query(1000, lr.LR_W_NONE, lr.make_opts(spacing=(3,)))
    with pytest.raises(lr.LrError):
        lr.lr_plan_query(1000, lr.LR_W_NONE, lr.make_opts(base_max=1 << 20))


def plan_of(n, w=lr.LR_W_NONE, opts=None):
    p = lr.lr_plan_query(n, w, opts)
    return int(p.base_max), [int(p.spacing[i]) for i in range(p.levels)]


def test_default_plans_follow_the_measured_rules():
    """The planner's defaults (chosen by per-size measurements on MI355X):
    below 2^25 short walks and a doubled base case where it saves a level,
    from 2^25 first-level spacing 32, then 64 from 3 * 2^26 elements
    (weighted: from 2^27); the last level the smallest spacing that fits."""
    assert plan_of(1 << 14) == (16384, [])
    assert plan_of(1 << 18) == (8192, [8, 4])
    assert plan_of(1 << 20) == (16384, [8, 8])
    assert plan_of(1 << 22) == (16384, [8, 8, 4])
    assert plan_of(1 << 24) == (16384, [32, 8, 4])
    assert plan_of(1 << 25) == (8192, [32, 16, 8])
    assert plan_of(1 << 26) == (8192, [32, 16, 16])
    assert plan_of(1 << 27) == (8192, [32, 16, 16, 2])
    assert plan_of(3 << 26) == (8192, [64, 16, 16, 2])
    assert plan_of(1 << 28) == (8192, [64, 16, 16, 2])
    w = lr.LR_W_I64
    assert plan_of(1 << 13, w) == (8192, [])
    assert plan_of(1 << 14, w) == (4096, [4])
    assert plan_of(1 << 16, w) == (8192, [8])
    assert plan_of(1 << 26, w) == (4096, [32, 16, 16, 2])
    assert plan_of(1 << 27, w) == (4096, [64, 16, 16, 2])


def test_plans_stay_within_the_level_limit():
    """Where short walks would need more than the 8 levels (many user levels
    of spacing 2, a tiny base), the planner takes the long walks instead."""
    base, sp = plan_of(30011, opts=lr.make_opts(spacing=(2, 2, 2, 2, 2), base_max=8))
    assert sp[:5] == [2, 2, 2, 2, 2] and len(sp) <= 8
    assert plan_of(30011, opts=lr.make_opts(spacing=(64, 2), base_max=1))[1][:2] == [64, 2]
    p = lr.lr_plan_query(158309, lr.LR_W_NONE, lr.make_opts(flags=lr.LR_SPAWN, spacing=(8, 4, 2), base_max=16))
    assert p.levels <= 6  # spawning keeps one level entry for its input


def test_workspace_monotone_and_weighted_larger():
    prev = 0
    for e in range(0, 31):
        b = lr.lr_workspace_bytes((1 << e) + 3 if e < 30 else (1 << 31) - 1)
        assert b >= prev
        prev = b
    assert lr.lr_workspace_bytes(1 << 31) == 0
    assert lr.lr_workspace_bytes(1 << 20, lr.LR_W_I64) > lr.lr_workspace_bytes(1 << 20)
    assert lr.lr_workspace_bytes(1 << 20, lr.LR_W_I32) == lr.lr_workspace_bytes(1 << 20, lr.LR_W_I64)
    assert lr.lr_workspace_bytes(10, 7) == 0
    assert lr.lr_wyllie_workspace_bytes(1 << 20) >= 2 * 8 * (1 << 20)


def test_argument_errors_before_any_device_work():
    L = lr.load()
    vp = ctypes.c_void_p
    fake = vp(0x1000)
    assert L.lr_rank(None, fake, None, 0, None, 0, None, None) == lr.LR_OK          # n == 0: no-op
    assert L.lr_rank(None, fake, None, 10, fake, 1 << 20, None, None) == lr.LR_ERR_INVALID_ARG
    assert L.lr_rank(fake, None, None, 10, fake, 1 << 20, None, None) == lr.LR_ERR_INVALID_ARG
    assert L.lr_rank(fake, fake, None, 1 << 31, fake, 1 << 20, None, None) == lr.LR_ERR_UNSUPPORTED
    assert L.lr_rank(fake, fake, None, 100000, fake, 16, None, None) == lr.LR_ERR_WORKSPACE
    assert L.lr_rank(fake, fake, None, 100000, None, 1 << 30, None, None) == lr.LR_ERR_WORKSPACE
    assert L.lr_prefix_sum(fake, None, 1, fake, None, None, 10, fake, 1 << 20, None, None) == lr.LR_ERR_INVALID_ARG
    assert L.lr_prefix_sum(fake, fake, 9, fake, None, None, 10, fake, 1 << 20, None, None) == lr.LR_ERR_INVALID_ARG
    assert L.lr_prefix_sum(fake, fake, 2, None, None, None, 10, fake, 1 << 20, None, None) == lr.LR_ERR_INVALID_ARG
    bad = lr.make_opts(spacing=(5,))
    assert L.lr_rank(fake, fake, None, 100000, fake, 1 << 30, ctypes.byref(bad), None) == lr.LR_ERR_INVALID_ARG
    assert L.lr_rank_wyllie(fake, fake, None, 1000, fake, 8, None) == lr.LR_ERR_WORKSPACE
    reqs = (lr.lr_request * 2)()
    reqs[0].succ, reqs[0].rank, reqs[0].n = 0x1000, None, 5
    assert L.lr_rank_batch(reqs, 2, fake, 1 << 20, None, None) == lr.LR_ERR_INVALID_ARG
    assert L.lr_rank_batch(None, 0, None, 0, None, None) == lr.LR_OK
    cfg = lr.lr_server_config()
    out = ctypes.c_void_p()
    assert L.lr_server_create(ctypes.byref(cfg), ctypes.byref(out)) == lr.LR_ERR_INVALID_ARG


def test_batch_workspace_counts_all_requests():
    reqs = (lr.lr_request * 3)()
    for i, n in enumerate((1000, 20000, 300000)):
        reqs[i].succ, reqs[i].rank, reqs[i].n = 0x1000, 0x2000, n
    b3 = lr.lr_batch_workspace_bytes(reqs, 3)
    b1 = lr.lr_batch_workspace_bytes(reqs, 1)
    assert b3 > b1 > 0
    assert b3 >= lr.lr_workspace_bytes(321000)


def test_local_contraction_workspace():
    """LR_LOCAL sizes the contraction arrays (start counts, start bits, per
    element chain position, contracted records) on top of the levels."""
    for n, w in [(1, lr.LR_W_NONE), (5000, lr.LR_W_NONE), (1 << 20, lr.LR_W_NONE), (1 << 20, lr.LR_W_I64)]:
        o = lr.make_opts(flags=lr.LR_LOCAL)
        b = lr.lr_workspace_bytes(n, w, o)
        rec = 16 if w != lr.LR_W_NONE else 8
        assert b >= n * (4 + rec + (8 if w != lr.LR_W_NONE else 0)) + n // 4
        p = lr.lr_plan_query(n, w, o)
        assert p.workspace_bytes == b
        plain = lr.lr_plan_query(n, w)
        assert p.levels == plain.levels and list(p.m) == list(plain.m)


def test_spawn_workspace_and_flags():
    """LR_SPAWN sizes the input level's slots, predecessor bytes and head
    counts plus the walks' records (at most n) on top of the walks' levels;
    it excludes LR_LOCAL; spacing[0] is the input level's spacing and
    spacing[1..] the levels above."""
    for n, w in [(1, lr.LR_W_NONE), (5000, lr.LR_W_NONE), (1 << 20, lr.LR_W_NONE), (1 << 20, lr.LR_W_I64)]:
        o = lr.make_opts(flags=lr.LR_SPAWN)
        b = lr.lr_workspace_bytes(n, w, o)
        rec = 16 if w != lr.LR_W_NONE else 8
        assert b >= n * (2 * rec + 1)
        assert lr.lr_plan_query(n, w, o).workspace_bytes == b
    assert lr.lr_workspace_bytes(1000, lr.LR_W_NONE, lr.make_opts(flags=lr.LR_SPAWN | lr.LR_LOCAL)) == 0
    assert lr.lr_workspace_bytes(1000, lr.LR_W_NONE, lr.make_opts(flags=lr.LR_SPAWN, spacing=(3,))) == 0
    p = lr.lr_plan_query(1 << 20, lr.LR_W_NONE, lr.make_opts(flags=lr.LR_SPAWN, spacing=(64, 8, 4)))
    assert [p.spacing[i] for i in range(2)] == [8, 4]


def test_visit_log_flag_sizes_the_log():
    """LR_VISIT_LOG adds the visit log below 2^25 (from 2^16 on) and changes
    nothing for smaller inputs."""
    n = 1 << 20
    plain = lr.lr_workspace_bytes(n, lr.LR_W_NONE, lr.make_opts(flags=lr.LR_NO_LOCAL))
    logged = lr.lr_workspace_bytes(n, lr.LR_W_NONE, lr.make_opts(flags=lr.LR_NO_LOCAL | lr.LR_VISIT_LOG))
    assert logged > plain + 12 * n
    small = 1 << 15
    assert lr.lr_workspace_bytes(small, lr.LR_W_NONE, lr.make_opts(flags=lr.LR_VISIT_LOG)) == \
        lr.lr_workspace_bytes(small, lr.LR_W_NONE)


def test_packed_visit_log_sizing():
    """Visit logs of up to 2^28 elements add a continuation table (a smaller
    offset field needs a larger one); above 2^28 the records stay wide and no
    table is added; an offset field above 31 bits is rejected."""
    n = 1 << 26
    base = lr.lr_workspace_bytes(n)
    assert lr.lr_workspace_bytes(n, lr.LR_W_NONE, lr.make_opts(log_off_bits=1)) > base
    assert lr.lr_workspace_bytes(n, lr.LR_W_NONE, lr.make_opts(log_off_bits=20)) == base
    big = (1 << 28) + 1
    assert lr.lr_workspace_bytes(big) == lr.lr_workspace_bytes(big, lr.LR_W_NONE, lr.make_opts(log_off_bits=1))
    assert lr.lr_workspace_bytes(n, lr.LR_W_NONE, lr.make_opts(log_off_bits=32)) == 0
