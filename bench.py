"""Benchmark: sparse ruling-set list ranking of one random 2^28-element list on
one MI355X, plus the context numbers the metric asks for.

A step is one lr_rank call (every kernel of the method: predecessor marks,
head compaction, chase, upper levels, base case, expand) on a list already
resident in HBM. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G elements ranked/s and achieved HBM GB/s, 2^28 random list; batched p50/p99"
HBM_PEAK_GBS = 8000.0
N_MAIN = 1 << 28


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N_MAIN, help="list length (default 2^28)")
    ap.add_argument("--only-main", action="store_true", help="time the main step only (for profilers)")
    ap.add_argument("--list", choices=["random", "block", "forest", "euler", "tree", "batch", "rulers-last"],
                    default="random",
                    help="with --only-main: the random list, the block-local list of the same size, the "
                         "2^27 forest with int64 weights (prefix sums, rank and root), the Euler tour / tree, "
                         "the 64-request batch, or a list of the same size ordered against the ruler sampling")
    ap.add_argument("--batch-graph", action="store_true",
                    help="with --list batch: replay the batch as a captured graph (lr_batch_graph)")
    ap.add_argument("--autotune", action="store_true",
                    help="the plan autotuner on the random list of --n elements: default plan, search, tuned plan")
    ap.add_argument("--no-largest", action="store_true", help="skip the 2^31 - 1 element list")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only the CPU oracle on the 2^28 random list itself (1 untimed + 3 timed runs)")
    ap.add_argument("--no-weighted", action="store_true")
    ap.add_argument("--serve-count", type=int, default=4096)
    ap.add_argument("--gamma", type=float, nargs="*", default=[0.0, 0.01, 0.1, 0.3],
                    help="List(n, gamma) locality sweep (empty: none)")
    ap.add_argument("--calibrate", action="store_true",
                    help="only the device access-rate calibration (lr_calibrate), one JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--sweep", choices=["spawn", "visit-log"],
                    help="only a size sweep, one JSON line: ruler spawning (LR_SPAWN, first-level spacing 16/32/64) "
                         "against the default path, or the first level with and without the visit log")
    return ap.parse_args()


def code_only(text: str) -> str:
    """Source text without comments and with whitespace collapsed, so that a
    comment edit does not mark recorded counters as stale (string literals in
    these files contain no comment markers)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def chase_code(text: str) -> str:
    """The chase kernel's definition (template line to closing brace) out of
    the comment-free kernels source, and the launch-configuration macros."""
    i = text.index("void k_chase(")
    start = text.rfind("template", 0, i)
    depth, j = 0, text.index("{", i)
    for k in range(j, len(text)):
        depth += {"{": 1, "}": -1}.get(text[k], 0)
        if depth == 0:
            break
    macros = " ".join(m for m in text.split("#") if m.startswith(("define LR_CHASE_TPB", "define LR_XCD")))
    return text[start:k + 1] + macros


def library_code_hash(root: str = ROOT) -> str:
    """Hash of the code (not the comments) of every library source: the
    whole-call traffic recorded in profiles/chase_traffic.json is used only
    while it matches."""
    csrc = os.path.join(root, "paper_2606_09318_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".cpp", ".hpp")):
            with open(os.path.join(csrc, f), encoding="utf-8") as fh:
                h.update(code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def kernel_source_hash(root: str = ROOT) -> str:
    """Hash of the code (not the comments) of the level-0 chase kernel and the
    headers it builds on (values, sources, sampler, plan constants): the
    traffic recorded in profiles/chase_traffic.json is used only while it
    matches."""
    csrc = os.path.join(root, "paper_2606_09318_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(csrc, "kernels.hip"), encoding="utf-8") as fh:
        h.update(chase_code(code_only(fh.read())).encode())
    for f in ("device.hpp", "plan.hpp"):
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build ranks one GPU's share and has no multi-GPU path; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2606_09318_amd as lr
    import workloads

    torch.cuda.set_device(0)
    dev = "cuda:0"
    stream = torch.cuda.current_stream()

    if args.calibrate:
        print(json.dumps({"calibration": lr.calibrate(dev)}))
        return

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(1)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": a.numel() * 4, "bytes_written": b.numel() * 4, "reps": 5}))
        return

    if args.autotune:
        autotune_bench(args, stream)
        return

    if args.cpu_full:
        print(json.dumps({"cpu_oracle_2p28": cpu_baseline(28, warmup=1, reps=3)}))
        return

    if args.sweep:
        print(json.dumps({"sweep": args.sweep, "unit": "ms per lr_rank call (median of 15), rank and root outputs",
                          "rows": size_sweep(args.sweep, stream)}))
        return

    n = args.n
    if args.list != "random" and not args.only_main:
        raise SystemExit("--list applies to --only-main runs")
    if args.list == "forest":
        forest_only(args, stream)
        return
    if args.list in ("euler", "tree"):
        euler_only(args, stream, tree=args.list == "tree")
        return
    if args.list == "batch":
        batch_only(args, stream)
        return
    t0 = time.time()
    if args.list == "rulers-last":
        # every level-0 sampled ruler after all other elements: the order the
        # walk cap and its fallback exist for (test-input builder)
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from adversarial import rulers_last
        L = rulers_last(n, int(lr.lr_plan_query(n).spacing[0]))
    elif args.list == "random":
        L = workloads.random_list(n, seed=2, stream=0)
    else:
        L = workloads.block_list(n, block=4096, seed=2, stream=1)
    gen_s = time.time() - t0
    succ = torch.from_numpy(L.succ.view(np.int32)).to(dev)
    rank = torch.empty(n, dtype=torch.int32, device=dev)
    root = torch.empty(n, dtype=torch.int32, device=dev)
    plan = lr.lr_plan_query(n)
    ws = lr.workspace(lr.lr_workspace_bytes(n), dev)

    def step(want_root=False):
        s = lr.lr_rank(succ, rank, root if want_root else None, ws, None, stream)
        if s:
            raise lr.LrError(s, "lr_rank")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    value = n / (ms * 1e-3) / 1e9

    # correctness of what was timed: closed form of the generated order
    order = torch.from_numpy(L.order.view(np.int32)).to(dev)
    expect = torch.arange(n - 1, -1, -1, dtype=torch.int32, device=dev)
    ok = bool(torch.equal(rank.index_select(0, order), expect))
    if not ok:
        raise SystemExit("bench: ranks do not match the closed form of the generated list")
    # the distribution of single calls (events around each call, after the
    # timed region): median, min and max of 10
    call_ts = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        step()
        e1.record(stream)
        e1.synchronize()
        call_ts.append(e0.elapsed_time(e1))
    call_ms = {"median": round(float(np.median(call_ts)), 4), "min": round(min(call_ts), 4),
               "max": round(max(call_ts), 4), "calls": len(call_ts)}
    # the same call with the root output as well (context; the configuration asks for ranks)
    step(True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(5):
        step(True)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_root = ev0.elapsed_time(ev1) / 5
    ok = bool(torch.equal(rank.index_select(0, order), expect)) and bool((root == int(L.order[-1])).all())
    del order, expect
    if not ok:
        raise SystemExit("bench: ranks/roots do not match the closed form of the generated list")
    if args.only_main:
        line = {"metric": METRIC, "value": round(value, 4), "unit": "G elements/s",
                "ms_per_step": round(ms, 4), "n": n, "list": args.list}
        if args.list == "rulers-last":
            lr.lr_rank(succ, rank, None, ws, lr.make_opts(flags=lr.LR_PROFILE), stream)
            ph = lr.lr_profile_last()
            line["fallback_ran"] = bool(ph[7])
            line["phases_ms"] = [round(v, 4) for v in ph[:7]]
        print(json.dumps(line))
        return

    # per-phase times with HIP events on the launch stream (LR_PROFILE), and
    # the level-0 chase (the dominant kernel) for the roofline
    popt = lr.make_opts(flags=lr.LR_PROFILE)
    phases = []
    for _ in range(5):
        lr.lr_rank(succ, rank, None, ws, popt, stream)
        phases.append(lr.lr_profile_last())
    ph = np.median(np.array(phases), axis=0)
    chase_ms = float(ph[2])
    S = int(plan.m[1])
    # algorithmic bytes of the chase per element, as the method's byte budget
    # counts them: a 4 B successor gather, a 4 B ruler-bit gather and an 8 B
    # store of (walk, offset). This chase tests the ruler by arithmetic on the
    # id (one ruler per block at a hashed position) and moves no ruler bit,
    # so its own count is 4 B + the visit-log record (one 8 B word up to 2^28
    # elements, 12 B above) per element and 9 B per walk (walk record and
    # predecessor mark); both are reported, the budget's is the roofline's
    rec = 8 if n <= (1 << 28) else 12
    chase_bytes = n * (4 + 4 + 8)
    own_bytes = n * (4 + rec) + S * (8 + 1)
    achieved = chase_bytes / (chase_ms * 1e-3) / 1e9
    traffic = None
    call_traffic = None
    tfile = os.path.join(ROOT, "profiles", "chase_traffic.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tj = json.load(fh)
        if tj.get("kernel_hash") == kernel_source_hash() and tj.get("n") == n:
            traffic = tj.get("hbm_bytes_per_launch")
        if tj.get("call_code_hash") == library_code_hash() and tj.get("n") == n:
            call_traffic = tj.get("call_hbm_bytes")
    roofline = {"bound": "hbm", "kernel": "k_chase (level 0)", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "chase_ms": round(chase_ms, 4),
                "algorithmic_bytes": chase_bytes, "bytes_per_element": 16,
                "own_count_bytes": own_bytes,
                "own_count_frac": round(own_bytes / (chase_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if traffic:
        # the HBM rate the counted bytes imply (each 4 B gather moves a whole line)
        roofline["traffic_gb_s"] = round(traffic / (chase_ms * 1e-3) / 1e9, 1)
        roofline["traffic_frac"] = round(roofline["traffic_gb_s"] / HBM_PEAK_GBS, 4)
    # per element over the level-0 passes of the timed call (rank only): head sum 4 B read;
    # chase 4 B gather + log record write; place1 log record read + 8 B write;
    # place2 8 + 8; place3 8 B read + 4 B rank write  -> 60 B with 8 B records
    whole_bytes = n * (4 + 4 + rec + rec + 8 + 8 + 8 + 8 + 4)
    extra = {"phases_ms": {"detect": round(float(ph[0]), 4), "heads": round(float(ph[1]), 4),
                           "chase_level0": round(chase_ms, 4), "upper_levels_and_base": round(float(ph[3]), 4),
                           "resolve_and_group": round(float(ph[4]), 4),
                           "expand": round(float(ph[5]), 4), "total": round(float(ph[6]), 4)},
             "useful_bytes_gbs_whole_step": round(whole_bytes / (ms * 1e-3) / 1e9, 1),
             # HBM bytes of one whole call from the counters (FETCH_SIZE + WRITE_SIZE over
             # every library kernel of a rank-only call, scaled by the copy calibration;
             # profiles/chase_traffic.json) over the timed step; null when the sources
             # changed since the counters were taken
             "hbm_whole_step": None if call_traffic is None else {
                 "bytes": call_traffic, "gb_s": round(call_traffic / (ms * 1e-3) / 1e9, 1),
                 "frac_of_peak": round(call_traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
             "plan": {"levels": plan.levels, "m": [int(plan.m[i]) for i in range(plan.levels + 1)],
                      "spacing": [int(plan.spacing[i]) for i in range(plan.levels)]},
             "generation_s": round(gen_s, 2),
             "rank_and_root": {"ms": round(ms_root, 4), "g_elements_per_s": round(n / (ms_root * 1e-3) / 1e9, 4)}}

    # GPU baseline: Wyllie pointer doubling on the same list
    del ws
    torch.cuda.empty_cache()
    wsw = lr.workspace(lr.lr_wyllie_workspace_bytes(n), dev)
    lr.lr_rank_wyllie(succ, rank, root, wsw, stream)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(3):
        lr.lr_rank_wyllie(succ, rank, root, wsw, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wy_ms = ev0.elapsed_time(ev1) / 3
    extra["wyllie"] = {"ms": round(wy_ms, 3), "srs_speedup": round(wy_ms / ms, 2)}
    del wsw
    torch.cuda.empty_cache()

    # inputs with locality (Section 2.3): the default call contracts tile-local
    # chains when most links are local; LR_NO_LOCAL forces the plain path and
    # LR_LOCAL the contracted one, for comparison
    del succ
    torch.cuda.empty_cache()
    extra["locality"] = locality_bench(n, rank, stream, args.gamma)
    extra["block_local_4096"] = extra["locality"]["block_local_4096"]
    del rank, root, L
    torch.cuda.empty_cache()

    if not args.no_largest:
        extra["largest_input"] = largest_bench(stream)
        torch.cuda.empty_cache()

    extra["calibration"] = lr.calibrate(dev)
    torch.cuda.empty_cache()
    # the chase against the part's measured random-access ceiling: its n
    # dependent 4 B gathers per launch against independent 4 B gathers over a
    # 1 GiB array (lr_calibrate), the rate a random line fill allows
    g_ceiling = extra["calibration"].get("gather4_1gib_g_s")
    if g_ceiling:
        g_rate = n / (chase_ms * 1e-3) / 1e9
        roofline["gather_ceiling"] = {"achieved_g_per_s": round(g_rate, 2), "ceiling_g_per_s": g_ceiling,
                                      "frac": round(g_rate / g_ceiling, 4),
                                      "ceiling": "independent random 4 B gathers over 1 GiB (lr_calibrate)"}

    if not args.no_weighted:
        extra.update(weighted_bench())

    if not args.no_serve:
        extra["serving"] = serve_bench(args.serve_count)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline()

    out = {"metric": METRIC, "value": round(value, 4), "unit": "G elements/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "single random list, n=2^28, uint32 succ (seed 2), uint32 rank output",
                      "n": n, "parallelism": "single GPU"},
           "roofline": roofline, "cpu_baseline": cpu, "call_ms": call_ms}
    out.update(extra)
    print(json.dumps(out))


def forest_only(args, stream):
    """Profiling entry: the forest of 2^27 elements with int64 weights (lists of
    geometric length, mean 64, plus 16 of 2^20), lr_prefix_sum with all outputs."""
    import numpy as np
    import torch

    import paper_2606_09318_amd as lr
    import workloads

    n = 1 << 27
    F = workloads.forest(n, mean=64, n_long=16, long_len=1 << 20, seed=3)
    succ = torch.from_numpy(F.succ.view(np.int32)).cuda()
    w = torch.from_numpy(F.weight).cuda()
    sm = torch.empty(n, dtype=torch.int64, device="cuda")
    r = torch.empty(n, dtype=torch.int32, device="cuda")
    t = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_I64))

    def step():
        st = lr.lr_prefix_sum(succ, w, sm, r, t, ws, None, stream)
        if st:
            raise lr.LrError(st, "lr_prefix_sum")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    print(json.dumps({"workload": "forest 2^27 int64 weights", "ms_per_step": round(ms, 4),
                      "g_elements_per_s": round(n / (ms * 1e-3) / 1e9, 3), "list": "forest"}))


def size_sweep(kind: str, stream) -> list:
    """Ruler spawning or the visit-log threshold across input sizes. Every
    timed configuration is checked against the closed form of the generator
    (random lists) or the local certificate (forests)."""
    import numpy as np
    import torch

    import paper_2606_09318_amd as lr
    import workloads

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import certificate_gpu

    def median_ms(fn, reps=15):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return round(sorted(ts)[len(ts) // 2], 4)

    rows = []
    if kind == "spawn":
        sizes, inputs = [14, 16, 18, 20, 22, 23, 24, 25], ["random"]
        modes = [("default", 0, ())] + [(f"spawn_k{k}", lr.LR_SPAWN, (k,)) for k in (16, 32, 64)]
    else:
        sizes, inputs = [21, 22, 23, 24, 25, 26], ["random", "forest"]
        modes = [("default", lr.LR_NO_LOCAL, ()), ("visit_log", lr.LR_NO_LOCAL | lr.LR_VISIT_LOG, ())]
    for logn in sizes:
        n = 1 << logn
        for kind_in in inputs:
            if kind_in == "random":
                L = workloads.random_list(n, seed=2)
                succ_np, order = L.succ, L.order
            else:
                F = workloads.forest(n, mean=64, n_long=4, long_len=n // 64, seed=3)
                succ_np, order = F.succ, None
            succ = torch.from_numpy(succ_np.view(np.int32)).cuda()
            r = torch.empty(n, dtype=torch.int32, device="cuda")
            t = torch.empty(n, dtype=torch.int32, device="cuda")
            exp = None
            if order is not None:
                exp = torch.empty(n, dtype=torch.int32, device="cuda")
                exp[torch.from_numpy(order.view(np.int32)).cuda().long()] = torch.arange(
                    n - 1, -1, -1, dtype=torch.int32, device="cuda")
            row = {"n": n, "input": kind_in}
            for name, flags, sp in modes:
                o = lr.make_opts(flags=flags, spacing=sp)
                ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_NONE, o))
                row[name] = median_ms(lambda: lr.lr_rank(succ, r, t, ws, o, stream))
                ok = torch.equal(r, exp) if exp is not None else certificate_gpu(succ, r, t)
                if not ok:
                    raise SystemExit(f"sweep: wrong result, n={n} {kind_in} {name}")
                del ws
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
            del succ, r, t, exp
            torch.cuda.empty_cache()
    return rows


def locality_bench(n: int, rank, stream, gammas) -> dict:
    """Block-local list and the paper's List(n, gamma) at the main size: the
    default call (automatic contraction) against the forced paths."""
    import numpy as np
    import torch

    import paper_2606_09318_amd as lr
    import workloads

    dev = rank.device
    modes = {"default": 0, "plain": lr.LR_NO_LOCAL, "contracted": lr.LR_LOCAL}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def measure(L):
        succ = torch.from_numpy(L.succ.view(np.int32)).to(dev)
        order = torch.from_numpy(L.order.view(np.int32)).to(dev)
        expect = torch.arange(n - 1, -1, -1, dtype=torch.int32, device=dev)
        row = {}
        for name, flags in modes.items():
            o = lr.make_opts(flags=flags)
            ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_NONE, o), dev)
            rank.fill_(-1)
            for _ in range(2):
                lr.lr_rank(succ, rank, None, ws, o, stream)
            torch.cuda.synchronize()
            ev0.record(stream)
            for _ in range(5):
                lr.lr_rank(succ, rank, None, ws, o, stream)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / 5
            ok = bool(torch.equal(rank.index_select(0, order), expect))
            if not ok:
                raise SystemExit(f"bench: locality workload ranks do not match the closed form ({name})")
            row[name + "_ms"] = round(ms, 3)
            del ws
            torch.cuda.empty_cache()
        row["default_g_elements_per_s"] = round(n / (row["default_ms"] * 1e-3) / 1e9, 3)
        row["default_speedup_over_plain"] = round(row["plain_ms"] / row["default_ms"], 2)
        del succ, order, expect
        torch.cuda.empty_cache()
        return row

    out = {"block_local_4096": measure(workloads.block_list(n, block=4096, seed=2, stream=1))}
    out["gamma_sweep"] = []
    for g in gammas:
        r = measure(workloads.gamma_list(n, g, seed=6))
        r["gamma"] = g
        out["gamma_sweep"].append(r)
    return out


def euler_only(args, stream, tree=False):
    """Profiling entry: the Euler tour of a 2^26-vertex random recursive tree
    (2^27 - 2 arcs in random order, +1/-1 int32 weights), lr_prefix_sum with
    the sums only (they give the depths); with tree, lr_euler_tree on the same
    tour (depth, preorder number and subtree size of every vertex)."""
    import numpy as np
    import torch

    import paper_2606_09318_amd as lr
    import workloads

    V = 1 << 26
    E = workloads.euler_tour(V, seed=4)
    m = E.succ.size
    succ = torch.from_numpy(E.succ.view(np.int32)).cuda()
    if tree:
        dn = torch.from_numpy(E.down_arc.view(np.int32)).cuda()
        upa = torch.from_numpy(E.up_arc.view(np.int32)).cuda()
        dv, pv, zv = (torch.empty(V, dtype=torch.int32, device="cuda") for _ in range(3))
        ws = lr.workspace(lr.lr_euler_tree_workspace_bytes(V))

        def step():
            st = lr.lr_euler_tree(succ, dn, upa, V, 0, dv, pv, zv, ws, None, stream)
            if st:
                raise lr.LrError(st, "lr_euler_tree")
    else:
        w = torch.from_numpy(E.weight).cuda()
        sm = torch.empty(m, dtype=torch.int64, device="cuda")
        ws = lr.workspace(lr.lr_workspace_bytes(m, lr.LR_W_I32))

        def step():
            st = lr.lr_prefix_sum(succ, w, sm, None, None, ws, None, stream)
            if st:
                raise lr.LrError(st, "lr_prefix_sum")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    if tree:
        if not bool(torch.equal(dv.cpu(), torch.from_numpy(E.depth.view(np.int32)))):
            raise SystemExit("bench: tree depths do not match the generator's")
        print(json.dumps({"workload": "tree computations on a 2^26-vertex tree's Euler tour",
                          "ms_per_step": round(ms, 4), "g_vertices_per_s": round(V / (ms * 1e-3) / 1e9, 3),
                          "list": "tree"}))
    else:
        print(json.dumps({"workload": "Euler tour of a 2^26-vertex tree, int32 weights", "ms_per_step": round(ms, 4),
                          "g_arcs_per_s": round(m / (ms * 1e-3) / 1e9, 3), "list": "euler"}))


def batch_only(args, stream):
    """Profiling entry: the first 64 requests of the serving trace (sizes
    log-uniform over 2^10..2^24, random and block-local lists alternating)
    ranked by one lr_rank_batch call; every request checked against its
    closed form after the timed steps."""
    import numpy as np
    import torch

    import paper_2606_09318_amd as lr
    import workloads

    tr = workloads.serving_trace(count=64, lo_log2=10, hi_log2=24, rate_per_s=1.0, seed=5)
    items, orders = [], []
    for q in tr:
        Lq = workloads.request_input(q)
        items.append((torch.from_numpy(Lq.succ.view(np.int32)).cuda(), torch.empty(q.n, dtype=torch.int32, device="cuda"),
                      None))
        orders.append(Lq.order)
    total = sum(q.n for q in tr)
    reqs = lr.requests(items)
    if args.batch_graph:
        # captured once for a capacity equal to this batch, replayed per step
        cfg = lr.batch_graph_config(max_elements=total, max_requests=len(items))
        ws = lr.workspace(lr.lr_batch_graph_workspace_bytes(cfg))
        g = lr.BatchGraph(cfg, ws)

        def step():
            st = g.launch(reqs, len(items), stream)
            if st:
                raise lr.LrError(st, "lr_batch_graph_launch")
    else:
        ws = lr.workspace(lr.lr_batch_workspace_bytes(reqs, len(items)))

        def step():
            st = lr.lr_rank_batch(reqs, len(items), ws, None, stream)
            if st:
                raise lr.LrError(st, "lr_rank_batch")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    for (s, r, _), order in zip(items, orders):
        n = s.numel()
        expect = torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda")
        if not torch.equal(r.index_select(0, torch.from_numpy(order.view(np.int32)).cuda()), expect):
            raise SystemExit("bench: a batched request does not match its closed form")
    if args.batch_graph:
        g.close()
    call = "one lr_batch_graph replay" if args.batch_graph else "one lr_rank_batch call"
    print(json.dumps({"workload": f"64 serving-trace requests in {call}", "requests": len(items),
                      "elements": total, "ms_per_step": round(ms, 4),
                      "g_elements_per_s": round(total / (ms * 1e-3) / 1e9, 3), "list": "batch"}))


def autotune_bench(args, stream):
    """The plan autotuner on the random list (seed 2): default calls timed with
    the built-in plan, lr_autotune on the same input, then default calls again
    (the planner now takes the cached entry); every timed result checked
    against the closed form."""
    import numpy as np
    import torch

    import paper_2606_09318_amd as lr
    import workloads

    n = args.n
    L = workloads.random_list(n, seed=2, stream=0)
    succ = torch.from_numpy(L.succ.view(np.int32)).cuda()
    rank = torch.empty(n, dtype=torch.int32, device="cuda")
    order = torch.from_numpy(L.order.view(np.int32)).cuda()
    expect = torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda")

    def timed():
        ws = lr.workspace(lr.lr_workspace_bytes(n))
        for _ in range(max(1, args.warmup)):
            lr.lr_rank(succ, rank, None, ws, None, stream)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            if lr.lr_rank(succ, rank, None, ws, None, stream):
                raise SystemExit("bench: lr_rank failed")
        ev1.record(stream)
        torch.cuda.synchronize()
        if not torch.equal(rank.index_select(0, order), expect):
            raise SystemExit("bench: ranks do not match the closed form")
        p = lr.lr_plan_query(n)
        return round(ev0.elapsed_time(ev1) / args.steps, 4), [int(p.spacing[i]) for i in range(p.levels)]

    lr.autotune_cache_clear()
    default_ms, default_plan = timed()
    tws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_NONE, lr.make_opts(spacing=(16, 8))) + n * 4 + 4096)
    t0 = time.time()
    st, best, trials = lr.lr_autotune(succ, None, tws, None, stream)
    tune_s = time.time() - t0
    if st:
        raise lr.LrError(st, "lr_autotune")
    del tws
    torch.cuda.empty_cache()
    tuned_ms, tuned_plan = timed()
    print(json.dumps({"autotune": {"n": n, "list": "random (seed 2)", "default_ms": default_ms,
                                   "default_spacing": default_plan, "tuned_ms": tuned_ms, "tuned_spacing": tuned_plan,
                                   "tuned_base_max": int(best.base_max), "tuned_lane_walks": int(best.lane_walks),
                                   "tuned_refill": int(best.refill), "candidates": len(trials),
                                   "trial_ms": [round(t, 4) for t in trials], "search_s": round(tune_s, 2)}}))


def largest_bench(stream, steps: int = 5) -> dict:
    """The largest input the boundary takes, n = 2^31 - 1: a random list in
    the order of a keyed Feistel permutation built on the device (the host
    generator takes minutes at this size), rank output, default options;
    the timed result is checked against the closed form."""
    import torch

    import paper_2606_09318_amd as lr
    import workloads

    n = (1 << 31) - 1
    print(json.dumps({"bench": "largest input", "n": n}), file=sys.stderr, flush=True)
    succ, order = workloads.random_list_device(n)
    torch.cuda.empty_cache()
    rank = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = lr.workspace(lr.lr_workspace_bytes(n))
    if lr.lr_rank(succ, rank, None, ws, None, stream):
        raise SystemExit("bench: lr_rank failed on the largest input")
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        lr.lr_rank(succ, rank, None, ws, None, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    del ws
    expect = torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda")
    ok = bool(torch.equal(rank.index_select(0, order), expect))
    del succ, order, rank, expect
    if not ok:
        raise SystemExit("bench: the largest input's ranks do not match the closed form")
    return {"n": n, "ms": round(ms, 3), "g_elements_per_s": round(n / (ms * 1e-3) / 1e9, 3),
            "list": "keyed Feistel order built on the device", "steps": steps}


def weighted_bench() -> dict:
    """The weighted workloads: the 2^27-element forest with int64 weights
    (rank, root and exact sums) and the Euler tour of a 2^26-vertex random
    recursive tree with +1/-1 int32 weights (sums give depths)."""
    import numpy as np
    import torch

    import paper_2606_09318_amd as lr
    import workloads

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import certificate_gpu

    out = {}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()

    def timed(call, reps=5):
        call()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(reps):
            call()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    n = 1 << 27
    F = workloads.forest(n, mean=64, n_long=16, long_len=1 << 20, seed=3)
    succ = torch.from_numpy(F.succ.view(np.int32)).cuda()
    w = torch.from_numpy(F.weight).cuda()
    sm = torch.empty(n, dtype=torch.int64, device="cuda")
    rk = torch.empty(n, dtype=torch.int32, device="cuda")
    rt = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_I64))

    def call():
        st = lr.lr_prefix_sum(succ, w, sm, rk, rt, ws, None, stream)
        if st:
            raise lr.LrError(st, "lr_prefix_sum")
    ms = timed(call)
    ok = certificate_gpu(succ, rk, rt, sm, w)
    out["forest_2p27_int64"] = {"ms": round(ms, 3), "g_elements_per_s": round(n / (ms * 1e-3) / 1e9, 3),
                                "lists": int(F.starts.size - 1), "outputs": "rank, root, int64 sum",
                                "certificate_ok": bool(ok)}
    del F, succ, w, sm, rk, rt, ws
    torch.cuda.empty_cache()

    V = 1 << 26
    E = workloads.euler_tour(V, seed=4)
    m = E.succ.size
    succ = torch.from_numpy(E.succ.view(np.int32)).cuda()
    w = torch.from_numpy(E.weight).cuda()
    sm = torch.empty(m, dtype=torch.int64, device="cuda")
    ws = lr.workspace(lr.lr_workspace_bytes(m, lr.LR_W_I32))

    def call2():
        st = lr.lr_prefix_sum(succ, w, sm, None, None, ws, None, stream)
        if st:
            raise lr.LrError(st, "lr_prefix_sum")
    ms = timed(call2)
    # depths from the sums: depth(v) = sum[head] - sum[down(v)] + 1; the head is the arc without predecessor
    has_pred = torch.zeros(m, dtype=torch.bool, device="cuda")
    nt = succ != torch.arange(m, dtype=torch.int32, device="cuda")
    has_pred[succ[nt].long()] = True
    head = int(torch.nonzero(~has_pred)[0])
    down = torch.from_numpy(E.down_arc[1:].astype(np.int64)).cuda()
    depth = sm[head] - sm.index_select(0, down) + 1
    ok = bool(torch.equal(depth.cpu(), torch.from_numpy(E.depth[1:].astype(np.int64))))
    out["euler_2p26_int32"] = {"ms": round(ms, 3), "g_elements_per_s": round(m / (ms * 1e-3) / 1e9, 3),
                               "arcs": m, "outputs": "int64 sum (depths)", "depths_ok": ok}
    del sm, ws, has_pred, nt, down, depth
    torch.cuda.empty_cache()

    # tree computations on the same tour: depth, preorder number and subtree
    # size of every vertex (one prefix sum over the tour + per-vertex pass)
    dn = torch.from_numpy(E.down_arc.view(np.int32)).cuda()
    upa = torch.from_numpy(E.up_arc.view(np.int32)).cuda()
    dv, pv, zv = (torch.empty(V, dtype=torch.int32, device="cuda") for _ in range(3))
    tws = lr.workspace(lr.lr_euler_tree_workspace_bytes(V))

    def call3():
        st = lr.lr_euler_tree(succ, dn, upa, V, 0, dv, pv, zv, tws, None, stream)
        if st:
            raise lr.LrError(st, "lr_euler_tree")
    ms = timed(call3)
    ok = bool(torch.equal(dv.cpu(), torch.from_numpy(E.depth.view(np.int32)))) and int(zv[0]) == V \
        and int(zv.long().sum()) == int((dv.long() + 1).sum())
    out["euler_tree_2p26"] = {"ms": round(ms, 3), "g_vertices_per_s": round(V / (ms * 1e-3) / 1e9, 3),
                              "vertices": V, "outputs": "depth, preorder, subtree size", "checks_ok": ok}
    del E, succ, w, dn, upa, dv, pv, zv, tws
    torch.cuda.empty_cache()
    return out


def serve_bench(count: int) -> dict:
    """Continuous batching vs one launch sequence per request on the serving
    trace (Poisson arrivals, sizes log-uniform over 2^10..2^24). After every
    replay all requests are checked against the closed form of their
    generated order on the device (outputs reset before each replay), and
    the number of failing requests is reported."""
    import numpy as np
    import torch

    import paper_2606_09318_amd as lr
    import workloads

    tr = workloads.serving_trace(count=count, lo_log2=10, hi_log2=24, rate_per_s=1.0, seed=5)
    items, orders = [], []
    total = 0
    t0 = time.time()
    for q in tr:
        Lq = workloads.request_input(q)
        s = torch.from_numpy(Lq.succ.view(np.int32)).to("cuda:0", non_blocking=False)
        items.append((s, torch.empty(q.n, dtype=torch.int32, device="cuda:0"), None))
        orders.append(torch.from_numpy(Lq.order.view(np.int32)).to("cuda:0"))
        total += q.n
    gen_s = time.time() - t0
    reqs = lr.requests(items)
    budget = 32 << 30

    def cfg(inflight, max_batch, graphs=1):
        c = lr.lr_server_config()
        c.hbm_budget, c.max_inflight, c.max_batch, c.graphs = budget, inflight, max_batch, graphs
        return c

    def failures() -> int:
        bad = 0
        for (_, r, _), o in zip(items, orders):
            n = r.numel()
            if not torch.equal(r.index_select(0, o), torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda:0")):
                bad += 1
        return bad

    def replay(c, arrivals) -> dict:
        for _, r, _ in items:
            r.fill_(-1)
        torch.cuda.synchronize()
        st, lat, sts, mk = lr.lr_server_replay(c, reqs, arrivals, count)
        lat = np.array(lat) * 1e3
        return {"status_ok": bool(st == 0 and all(x == 0 for x in sts)),
                "throughput_g_elements_per_s": round(total / mk / 1e9, 3), "makespan_s": round(mk, 3),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "closed_form_failures": failures()}

    def arrivals(rate) -> list:
        return [q.arrival_s for q in workloads.serving_trace(count=count, lo_log2=10, hi_log2=24, rate_per_s=rate,
                                                              seed=5)]

    torch.cuda.synchronize()
    mean_n = total / count
    # saturation throughputs: every request present at t = 0 (batched: each
    # batch replays the captured graph of its size bucket; also without graphs)
    sat_b = replay(cfg(2, count), [0.0] * count)
    sat_b_plain = replay(cfg(2, count, 0), [0.0] * count)
    sat_p = replay(cfg(1, 1, 0), [0.0] * count)
    sat = total / sat_b["makespan_s"]
    rate = 0.8 * sat / mean_n
    arr = arrivals(rate)
    res = {"requests": count, "total_elements": total, "offered_rate_req_per_s": round(rate, 1),
           "hbm_budget_gib": budget >> 30, "saturation_g_elements_per_s": round(sat / 1e9, 3),
           "saturation_per_request_g_elements_per_s": sat_p["throughput_g_elements_per_s"],
           "saturation_runs": {"batched": sat_b, "batched_without_graphs": sat_b_plain, "per_request": sat_p},
           "input_generation_s": round(gen_s, 1),
           "latency": "host clock from each request's scheduled arrival to the server seeing it complete",
           "correctness": "closed_form_failures = requests whose ranks differ from the closed form of "
                          "their generated order, all requests checked after every replay"}
    res["batched"] = replay(cfg(2, count), arr)
    res["batched_without_graphs"] = replay(cfg(2, count, 0), arr)
    res["per_request"] = replay(cfg(1, 1, 0), arr)
    # a load both servers sustain: 0.7 x the per-request saturation, so the
    # latencies compare at equal throughput
    rate_eq = 0.7 * (sat_p["throughput_g_elements_per_s"] * 1e9) / mean_n
    arr_eq = arrivals(rate_eq)
    res["equal_load"] = {"offered_rate_req_per_s": round(rate_eq, 1),
                         "offered_g_elements_per_s": round(rate_eq * mean_n / 1e9, 3),
                         "batched": replay(cfg(2, count), arr_eq), "per_request": replay(cfg(1, 1, 0), arr_eq)}
    # offered-load sweep for the batched server (same trace, arrival times scaled)
    res["load_sweep"] = []
    for load in (0.1, 0.5, 0.7, 0.9, 1.1):
        r = replay(cfg(2, count), [a * 0.8 / load for a in arr])
        r["load"] = load
        res["load_sweep"].append(r)
    res["closed_form_failures_total"] = sum(x["closed_form_failures"] for x in
                                            [sat_b, sat_b_plain, sat_p, res["batched"],
                                             res["batched_without_graphs"], res["per_request"],
                                             res["equal_load"]["batched"], res["equal_load"]["per_request"]]
                                            + res["load_sweep"])
    del items, orders
    torch.cuda.empty_cache()
    return res


def cpu_baseline(log2n: int = 26, warmup: int = 0, reps: int = 1) -> dict:
    """The oracle as it stands (sequential pointer chasing, one thread) on the
    random-list workload's generator (seed 2, stream 0): by default a bounded
    sample of 2^26 elements, one run; --cpu-full runs the 2^28 list itself."""
    import numpy as np

    import oracle
    import workloads

    n = 1 << log2n
    L = workloads.random_list(n, seed=2, stream=0)
    ts = []
    for i in range(warmup + reps):
        t0 = time.perf_counter()
        st, r, t, _ = oracle.rank(L.succ, want=("rank", "root"))
        dt = time.perf_counter() - t0
        assert st == 0
        if i >= warmup:
            ts.append(dt)
        print(json.dumps({"cpu_oracle_run": i, "n": n, "seconds": round(dt, 2), "timed": i >= warmup}),
              file=sys.stderr, flush=True)
    expect = np.empty(n, np.uint32)
    expect[L.order] = np.arange(n - 1, -1, -1, dtype=np.uint32)
    assert np.array_equal(r, expect)
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    med = float(np.median(ts))
    what = "the 2^28 random list itself" if log2n == 28 else f"a random list of 2^{log2n} elements"
    return {"value": round(n / med / 1e9, 5), "unit": "G elements/s", "cores": 1, "kind": "oracle",
            "sample": f"{what} from the same generator (seed 2), rank + root, {warmup} untimed + {reps} timed "
                      f"run(s), median",
            "seconds": {"median": round(med, 2), "min": round(min(ts), 2), "max": round(max(ts), 2)},
            "host_cpu": model, "host_nproc": os.cpu_count(), "build": "gcc -O3 -march=native"}


if __name__ == "__main__":
    main()
