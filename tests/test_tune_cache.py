"""The autotune cache (host-only): an entry for this process's device key and
a size bucket changes the plan of calls that leave the plan options at
their defaults, and only those; entries round-trip through a file; bad
entries are refused whole."""
import os

import pytest

import paper_2606_09318_amd as lr


@pytest.fixture(autouse=True)
def empty_cache():
    lr.autotune_cache_clear()
    yield
    lr.autotune_cache_clear()


def spacings(n, w=lr.LR_W_NONE, opts=None):
    p = lr.lr_plan_query(n, w, opts)
    return [int(p.spacing[i]) for i in range(p.levels)], int(p.base_max)


def write(path, rows):
    with open(path, "w") as fh:
        fh.write("# test cache\n")
        for r in rows:
            fh.write(" ".join(str(x) for x in r) + "\n")


def test_entry_applies_to_its_bucket_only(tmp_path):
    arch = lr.autotune_arch()
    assert arch
    default20, base20 = spacings(1 << 20)
    default22, _ = spacings(1 << 22)
    default20w, _ = spacings(1 << 20, lr.LR_W_I64)
    f = str(tmp_path / "cache.txt")
    # bucket floor(log2 n) = 20, unweighted: k0 = 128, k1 = 4, base 2048
    write(f, [(arch, 20, 0, 128, 4, 2048, 1, 1, 0.5)])
    assert lr.autotune_cache_load(f) == lr.LR_OK
    assert lr.autotune_cache_entries() == 1
    ks, base = spacings(1 << 20)
    assert ks[:2] == [128, 4] and base == 2048
    assert spacings((1 << 21) - 1)[0][:2] == [128, 4]       # same bucket
    assert spacings(1 << 22)[0] == default22                 # other bucket
    assert spacings(1 << 20, lr.LR_W_I64)[0] == default20w   # weighted: other key
    # explicit options win over the cache
    assert spacings(1 << 20, lr.LR_W_NONE, lr.make_opts(spacing=(32, 16)))[0][:2] == [32, 16]
    assert spacings(1 << 20, lr.LR_W_NONE, lr.make_opts(base_max=4096))[1] == 4096
    # the workspace size follows the plan the cache gives
    assert lr.lr_workspace_bytes(1 << 20) == lr.lr_plan_query(1 << 20).workspace_bytes
    lr.autotune_cache_clear()
    assert spacings(1 << 20) == (default20, base20)


def test_other_device_entries_do_not_apply(tmp_path):
    f = str(tmp_path / "cache.txt")
    default, _ = spacings(1 << 20)
    write(f, [("gfx000:1", 20, 0, 128, 4, 2048, 1, 1, 0.5)])
    assert lr.autotune_cache_load(f) == lr.LR_OK
    assert spacings(1 << 20)[0] == default


def test_save_load_round_trip(tmp_path):
    arch = lr.autotune_arch()
    f, g = str(tmp_path / "a.txt"), str(tmp_path / "b.txt")
    write(f, [(arch, 18, 0, 32, 8, 4096, 2, 1, 0.25), (arch, 24, 1, 64, 16, 4096, 1, 8, 2.5)])
    assert lr.autotune_cache_load(f) == lr.LR_OK
    assert lr.autotune_cache_save(g) == lr.LR_OK
    lr.autotune_cache_clear()
    assert lr.autotune_cache_load(g) == lr.LR_OK
    assert lr.autotune_cache_entries() == 2
    assert spacings(1 << 18)[0][:2] == [32, 8]
    assert spacings(1 << 24, lr.LR_W_I32)[0][:2] == [64, 16]


@pytest.mark.parametrize("row", [("x", 20, 0, 3, 4, 2048, 1, 1, 0.5),        # spacing not a power of two
                                 ("x", 20, 0, 64, 4, 1 << 20, 1, 1, 0.5),    # base too large
                                 ("x", 20, 0, 64, 4, 2048, 3, 1, 0.5),       # walks per lane
                                 ("x", 20, 2, 64, 4, 2048, 1, 1, 0.5),       # weighted flag
                                 ("x", 20, 0, 64)])                          # short line
def test_bad_entries_refused(tmp_path, row):
    f = str(tmp_path / "bad.txt")
    write(f, [(lr.autotune_arch(), 20, 0, 32, 8, 8192, 1, 1, 0.1), row])
    assert lr.autotune_cache_load(f) == lr.LR_ERR_INVALID_ARG
    assert lr.autotune_cache_entries() == 0                  # nothing half-loaded
    assert lr.autotune_cache_load(str(tmp_path / "missing.txt")) == lr.LR_ERR_INVALID_ARG
