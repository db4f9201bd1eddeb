"""MI355X (gfx950) sparse ruling-set list ranking.

A thin ctypes binding over liblr.so (include/lr.h): every function with an
lr_ name marshals torch tensors (device memory) into the C call of the same
name. All ranking work runs in the library's HIP kernels; there is no other
implementation behind these names, and loading fails loudly if the library
has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LR_LIBRARY selects another build of the same library (tuning-constant sweeps)
LIB_PATH = os.environ.get("LR_LIBRARY") or os.path.join(HERE, "liblr.so")

LR_OK, LR_ERR_INVALID_ARG, LR_ERR_UNSUPPORTED, LR_ERR_WORKSPACE = 0, 1, 2, 3
LR_ERR_OUT_OF_MEMORY, LR_ERR_BAD_LIST, LR_ERR_HIP = 4, 5, 6
LR_W_NONE, LR_W_I32, LR_W_I64 = 0, 1, 2
LR_VALIDATE, LR_PROFILE, LR_LOCAL, LR_NO_LOCAL, LR_SPAWN, LR_VISIT_LOG = 1, 2, 4, 8, 16, 32
LR_MAX_LEVELS = 8


class LrError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}")


class lr_opts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32), ("base_max", ctypes.c_uint32),
                ("spacing", ctypes.c_uint32 * LR_MAX_LEVELS), ("refill", ctypes.c_uint32),
                ("lane_walks", ctypes.c_uint32), ("log_off_bits", ctypes.c_uint32)]


class lr_plan(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_uint32), ("base_max", ctypes.c_uint32),
                ("m", ctypes.c_uint64 * (LR_MAX_LEVELS + 1)), ("spacing", ctypes.c_uint32 * LR_MAX_LEVELS),
                ("workspace_bytes", ctypes.c_uint64)]


class lr_request(ctypes.Structure):
    _fields_ = [("succ", ctypes.c_void_p), ("rank", ctypes.c_void_p), ("root", ctypes.c_void_p),
                ("n", ctypes.c_uint64)]


class lr_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("opts", lr_opts), ("graphs", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class lr_batch_graph_config(ctypes.Structure):
    _fields_ = [("max_elements", ctypes.c_uint64), ("max_requests", ctypes.c_uint32), ("want_root", ctypes.c_uint32),
                ("opts", lr_opts)]


_lib = None


def load():
    """Load liblr.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
    # torch's HIP runtime first: the library then binds to that runtime. Loaded
    # before torch, it would pull in the system runtime, torch would add its
    # own copy, and torch's streams would be unknown handles to the library.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_size_t
    st = ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "lr_status_string": (ctypes.c_char_p, [st]),
        "lr_plan_query": (st, [u64, st, P(lr_opts), P(lr_plan)]),
        "lr_workspace_bytes": (sz, [u64, st, P(lr_opts)]),
        "lr_rank": (st, [vp, vp, vp, u64, vp, sz, P(lr_opts), vp]),
        "lr_rank_noalloc": (st, [vp, vp, vp, u64, P(lr_opts), vp]),
        "lr_prefix_sum": (st, [vp, vp, st, vp, vp, vp, u64, vp, sz, P(lr_opts), vp]),
        "lr_batch_workspace_bytes": (sz, [P(lr_request), u32, P(lr_opts)]),
        "lr_rank_batch": (st, [P(lr_request), u32, vp, sz, P(lr_opts), vp]),
        "lr_wyllie_workspace_bytes": (sz, [u64, st]),
        "lr_rank_wyllie": (st, [vp, vp, vp, u64, vp, sz, vp]),
        "lr_prefix_sum_wyllie": (st, [vp, vp, st, vp, vp, vp, u64, vp, sz, vp]),
        "lr_profile_last": (st, [P(ctypes.c_double), st]),
        "lr_verify": (st, [vp, vp, st, vp, vp, vp, u64, vp, sz, vp]),
        "lr_autotune": (st, [vp, vp, st, u64, vp, sz, P(lr_opts), P(lr_opts), P(ctypes.c_double), st, P(st), vp]),
        "lr_autotune_arch": (ctypes.c_char_p, []),
        "lr_autotune_cache_entries": (st, []),
        "lr_autotune_cache_clear": (None, []),
        "lr_autotune_cache_save": (st, [ctypes.c_char_p]),
        "lr_autotune_cache_load": (st, [ctypes.c_char_p]),
        "lr_euler_tree_workspace_bytes": (sz, [u64, P(lr_opts)]),
        "lr_calibrate_workspace_bytes": (sz, []),
        "lr_calibrate": (st, [vp, sz, P(ctypes.c_double), st, vp]),
        "lr_euler_tree": (st, [vp, vp, vp, u64, u32, vp, vp, vp, vp, sz, P(lr_opts), vp]),
        "lr_batch_graph_workspace_bytes": (sz, [P(lr_batch_graph_config)]),
        "lr_batch_graph_create": (st, [P(lr_batch_graph_config), vp, sz, P(vp)]),
        "lr_batch_graph_launch": (st, [vp, P(lr_request), u32, vp]),
        "lr_batch_graph_destroy": (None, [vp]),
        "lr_server_create": (st, [P(lr_server_config), P(vp)]),
        "lr_server_submit": (st, [vp, P(lr_request), P(u64)]),
        "lr_server_poll": (st, [vp, u64, P(st), P(ctypes.c_double)]),
        "lr_server_drain": (st, [vp]),
        "lr_server_destroy": (None, [vp]),
        "lr_server_replay": (st, [P(lr_server_config), P(lr_request), P(ctypes.c_double), u32,
                                  P(ctypes.c_double), P(st), P(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def status_string(s: int) -> str:
    return load().lr_status_string(s).decode()


# ------------------------------------------------------------- marshalling --

def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def make_opts(seed: int = 0, flags: int = 0, base_max: int = 0, spacing=(), refill: int = 0,
              lane_walks: int = 0, log_off_bits: int = 0) -> lr_opts:
    o = lr_opts()
    o.seed, o.flags, o.base_max, o.refill, o.lane_walks = seed, flags, base_max, refill, lane_walks
    o.log_off_bits = log_off_bits
    for i, k in enumerate(spacing):
        o.spacing[i] = k
    return o


def _opts(opts):
    return None if opts is None else ctypes.byref(opts)


def _wtype(weight) -> int:
    if weight is None:
        return LR_W_NONE
    import torch
    if weight.dtype == torch.int32:
        return LR_W_I32
    if weight.dtype == torch.int64:
        return LR_W_I64
    raise TypeError(f"weights must be int32 or int64, not {weight.dtype}")


def lr_plan_query(n: int, w: int = LR_W_NONE, opts: lr_opts | None = None) -> lr_plan:
    p = lr_plan()
    s = load().lr_plan_query(n, w, _opts(opts), ctypes.byref(p))
    if s:
        raise LrError(s, "lr_plan_query")
    return p


def lr_workspace_bytes(n: int, w: int = LR_W_NONE, opts: lr_opts | None = None) -> int:
    return int(load().lr_workspace_bytes(n, w, _opts(opts)))


def lr_wyllie_workspace_bytes(n: int, w: int = LR_W_NONE) -> int:
    return int(load().lr_wyllie_workspace_bytes(n, w))


def lr_rank(succ, rank, root, ws, opts=None, stream=None) -> int:
    return load().lr_rank(_ptr(succ), _ptr(rank), _ptr(root), succ.numel(), _ptr(ws),
                          0 if ws is None else ws.numel() * ws.element_size(), _opts(opts), _stream(stream))


def lr_rank_noalloc(succ, rank, root, opts=None, stream=None) -> int:
    return load().lr_rank_noalloc(_ptr(succ), _ptr(rank), _ptr(root), succ.numel(), _opts(opts), _stream(stream))


def lr_prefix_sum(succ, weight, sum_, rank, root, ws, opts=None, stream=None) -> int:
    return load().lr_prefix_sum(_ptr(succ), _ptr(weight), _wtype(weight), _ptr(sum_), _ptr(rank), _ptr(root),
                                succ.numel(), _ptr(ws), 0 if ws is None else ws.numel() * ws.element_size(),
                                _opts(opts), _stream(stream))


def lr_rank_wyllie(succ, rank, root, ws, stream=None) -> int:
    return load().lr_rank_wyllie(_ptr(succ), _ptr(rank), _ptr(root), succ.numel(), _ptr(ws),
                                 0 if ws is None else ws.numel() * ws.element_size(), _stream(stream))


def lr_prefix_sum_wyllie(succ, weight, sum_, rank, root, ws, stream=None) -> int:
    return load().lr_prefix_sum_wyllie(_ptr(succ), _ptr(weight), _wtype(weight), _ptr(sum_), _ptr(rank),
                                       _ptr(root), succ.numel(), _ptr(ws),
                                       0 if ws is None else ws.numel() * ws.element_size(), _stream(stream))


def lr_verify(succ, rank=None, root=None, sum_=None, weight=None, stream=None) -> int:
    """Check outputs against the local equations on the device (LR_OK or LR_ERR_BAD_LIST)."""
    import torch
    ws = torch.empty(512, dtype=torch.uint8, device=succ.device)
    return load().lr_verify(_ptr(succ), _ptr(weight), _wtype(weight), _ptr(rank), _ptr(root), _ptr(sum_),
                            succ.numel(), _ptr(ws), ws.numel(), _stream(stream))


def requests(items) -> ctypes.Array:
    """items: iterable of (succ, rank, root-or-None) device tensors."""
    items = list(items)
    arr = (lr_request * max(len(items), 1))()
    for i, (s, r, t) in enumerate(items):
        arr[i].succ, arr[i].rank, arr[i].root, arr[i].n = s.data_ptr(), r.data_ptr(), \
            (t.data_ptr() if t is not None else None), s.numel()
    return arr


def lr_batch_workspace_bytes(reqs: ctypes.Array, count: int, opts=None) -> int:
    return int(load().lr_batch_workspace_bytes(reqs, count, _opts(opts)))


def lr_rank_batch(reqs: ctypes.Array, count: int, ws, opts=None, stream=None) -> int:
    return load().lr_rank_batch(reqs, count, _ptr(ws), ws.numel() * ws.element_size(), _opts(opts),
                                _stream(stream))


def batch_graph_config(max_elements: int, max_requests: int, want_root: bool = False,
                       opts: lr_opts | None = None) -> lr_batch_graph_config:
    c = lr_batch_graph_config()
    c.max_elements, c.max_requests, c.want_root = max_elements, max_requests, int(want_root)
    if opts is not None:
        c.opts = opts
    return c


def lr_batch_graph_workspace_bytes(cfg: lr_batch_graph_config) -> int:
    return int(load().lr_batch_graph_workspace_bytes(ctypes.byref(cfg)))


class BatchGraph:
    """lr_batch_graph: a batch captured once as a HIP graph (for a capacity of
    requests and elements) and replayed with other requests. The workspace
    tensor is kept alive with the graph."""

    def __init__(self, cfg: lr_batch_graph_config, ws):
        self.ws = ws
        h = ctypes.c_void_p()
        s = load().lr_batch_graph_create(ctypes.byref(cfg), _ptr(ws), ws.numel() * ws.element_size(),
                                         ctypes.byref(h))
        if s:
            raise LrError(s, "lr_batch_graph_create")
        self.h = h

    def launch(self, reqs: ctypes.Array, count: int, stream=None) -> int:
        return load().lr_batch_graph_launch(self.h, reqs, count, _stream(stream))

    def close(self):
        if self.h:
            load().lr_batch_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lr_euler_tree_workspace_bytes(V: int, opts: lr_opts | None = None) -> int:
    return int(load().lr_euler_tree_workspace_bytes(V, _opts(opts)))


def lr_euler_tree(succ, down, up, V: int, root: int, depth, preorder, size, ws, opts=None, stream=None) -> int:
    return load().lr_euler_tree(_ptr(succ), _ptr(down), _ptr(up), V, root, _ptr(depth), _ptr(preorder), _ptr(size),
                                _ptr(ws), 0 if ws is None else ws.numel() * ws.element_size(), _opts(opts),
                                _stream(stream))


def lr_autotune(succ, weight, ws, base=None, stream=None):
    """Time candidate ruler spacings on this input; returns (status, best lr_opts, timings in ms)."""
    best = lr_opts()
    ms = (ctypes.c_double * 64)()
    tried = ctypes.c_int()
    s = load().lr_autotune(_ptr(succ), _ptr(weight), _wtype(weight), succ.numel(), _ptr(ws),
                           ws.numel() * ws.element_size(), _opts(base), ctypes.byref(best), ms, 64,
                           ctypes.byref(tried), _stream(stream))
    return s, best, list(ms[:tried.value])


def autotune_arch() -> str:
    return load().lr_autotune_arch().decode()


def autotune_cache_entries() -> int:
    return int(load().lr_autotune_cache_entries())


def autotune_cache_clear() -> None:
    load().lr_autotune_cache_clear()


def autotune_cache_save(path: str) -> int:
    return load().lr_autotune_cache_save(path.encode())


def autotune_cache_load(path: str) -> int:
    return load().lr_autotune_cache_load(path.encode())


def lr_profile_last() -> list[float]:
    """Phase times (ms) of the last LR_PROFILE call on this thread, then 1.0
    if that call ran the bounded fallback, else 0.0."""
    buf = (ctypes.c_double * 8)()
    k = load().lr_profile_last(buf, 8)
    return list(buf[:k])


def lr_server_replay(cfg: lr_server_config, reqs: ctypes.Array, arrivals, count: int):
    """Replay arrivals (seconds) through a server; returns (status, latencies, statuses, makespan)."""
    arr = (ctypes.c_double * max(count, 1))(*arrivals)
    lat = (ctypes.c_double * max(count, 1))()
    sts = (ctypes.c_int * max(count, 1))()
    mk = ctypes.c_double()
    s = load().lr_server_replay(ctypes.byref(cfg), reqs, arr, count, lat, sts, ctypes.byref(mk))
    return s, list(lat[:count]), list(sts[:count]), mk.value


# --------------------------------------------------------- conveniences ----

def workspace(nbytes: int, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def rank(succ, want_root: bool = True, opts: lr_opts | None = None, stream=None):
    """Rank a device uint32 successor array (as int32 tensor); returns (rank, root)."""
    import torch
    n = succ.numel()
    r = torch.empty(n, dtype=torch.int32, device=succ.device)
    t = torch.empty(n, dtype=torch.int32, device=succ.device) if want_root else None
    ws = workspace(lr_workspace_bytes(n, LR_W_NONE, opts), succ.device)
    s = lr_rank(succ, r, t, ws, opts, stream)
    if s:
        raise LrError(s, "lr_rank")
    return r, t


def prefix_sum(succ, weight=None, want_rank=True, want_root=True, opts=None, stream=None):
    import torch
    n = succ.numel()
    sm = torch.empty(n, dtype=torch.int64, device=succ.device)
    r = torch.empty(n, dtype=torch.int32, device=succ.device) if want_rank else None
    t = torch.empty(n, dtype=torch.int32, device=succ.device) if want_root else None
    ws = workspace(lr_workspace_bytes(n, _wtype(weight) if weight is not None else LR_W_I64, opts), succ.device)
    s = lr_prefix_sum(succ, weight, sm, r, t, ws, opts, stream)
    if s:
        raise LrError(s, "lr_prefix_sum")
    return sm, r, t


def euler_tree(succ, down, up, root: int = 0, opts=None, stream=None):
    """Depth, preorder number and subtree size of every vertex from an Euler
    tour on the device (uint32 data as int32 tensors). Returns three tensors."""
    import torch
    V = down.numel()
    dev = down.device
    d = torch.empty(V, dtype=torch.int32, device=dev)
    p = torch.empty(V, dtype=torch.int32, device=dev)
    z = torch.empty(V, dtype=torch.int32, device=dev)
    ws = workspace(lr_euler_tree_workspace_bytes(V, opts), dev)
    s = lr_euler_tree(succ, down, up, V, root, d, p, z, ws, opts, stream)
    if s:
        raise LrError(s, "lr_euler_tree")
    return d, p, z


def calibrate(device="cuda", stream=None) -> dict:
    """Device access rates (lr_calibrate): streaming copy GB/s and random
    gather / store / bit-set rates in G accesses/s."""
    ws = workspace(load().lr_calibrate_workspace_bytes(), device)
    out = (ctypes.c_double * 7)()
    k = load().lr_calibrate(_ptr(ws), ws.numel(), out, 7, _stream(stream))
    if k < 0:
        raise LrError(-k, "lr_calibrate")
    names = ["copy_gb_s", "gather4_1gib_g_s", "store8_1gib_g_s", "store8_256mib_g_s", "store1_256mib_g_s",
             "bitset_32mib_g_s", "store4_xcd_ranges_g_s"]
    return {nm: round(out[i], 2) for i, nm in enumerate(names[:k])}
