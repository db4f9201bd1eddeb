"""Helpers shared by the GPU tests: move seeded inputs to the device, call the
library through its C ABI, and bring results back."""
import numpy as np
import torch

import paper_2606_09318_amd as lr


def dev(a: np.ndarray) -> torch.Tensor:
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host_u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def gpu_rank(succ_np, opts=None, want_root=True, stream=None):
    succ = dev(succ_np)
    n = succ.numel()
    r = torch.empty(n, dtype=torch.int32, device="cuda")
    t = torch.empty(n, dtype=torch.int32, device="cuda") if want_root else None
    ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_NONE, opts))
    s = lr.lr_rank(succ, r, t, ws, opts, stream)
    torch.cuda.synchronize()
    return s, host_u32(r), (host_u32(t) if want_root else None)


def gpu_prefix(succ_np, w_np=None, opts=None, want_rank=True, want_root=True):
    succ = dev(succ_np)
    n = succ.numel()
    w = dev(w_np) if w_np is not None else None
    sm = torch.empty(n, dtype=torch.int64, device="cuda")
    r = torch.empty(n, dtype=torch.int32, device="cuda") if want_rank else None
    t = torch.empty(n, dtype=torch.int32, device="cuda") if want_root else None
    ws = lr.workspace(lr.lr_workspace_bytes(n, lr.LR_W_I64, opts))
    s = lr.lr_prefix_sum(succ, w, sm, r, t, ws, opts)
    torch.cuda.synchronize()
    return s, sm.cpu().numpy(), (host_u32(r) if want_rank else None), (host_u32(t) if want_root else None)


def gpu_wyllie(succ_np, w_np=None, weighted=False):
    succ = dev(succ_np)
    n = succ.numel()
    r = torch.empty(n, dtype=torch.int32, device="cuda")
    t = torch.empty(n, dtype=torch.int32, device="cuda")
    if not weighted:
        ws = lr.workspace(lr.lr_wyllie_workspace_bytes(n, lr.LR_W_NONE))
        s = lr.lr_rank_wyllie(succ, r, t, ws)
        torch.cuda.synchronize()
        return s, host_u32(r), host_u32(t), None
    w = dev(w_np) if w_np is not None else None
    sm = torch.empty(n, dtype=torch.int64, device="cuda")
    ws = lr.workspace(lr.lr_wyllie_workspace_bytes(n, lr.LR_W_I64))
    s = lr.lr_prefix_sum_wyllie(succ, w, sm, r, t, ws)
    torch.cuda.synchronize()
    return s, host_u32(r), host_u32(t), sm.cpu().numpy()


def certificate_gpu(succ: torch.Tensor, rank: torch.Tensor, root: torch.Tensor | None = None,
                    sum_: torch.Tensor | None = None, weight: torch.Tensor | None = None) -> bool:
    """Local equations of the ranking (unique solution on a valid forest),
    evaluated on the device for full-size outputs."""
    n = succ.numel()
    idx = torch.arange(n, dtype=torch.int32, device=succ.device)
    term = succ == idx
    nt = ~term
    s_nt = succ[nt]
    ok = bool((rank[term] == 0).all()) and bool((rank[nt] == rank.index_select(0, s_nt) + 1).all())
    if root is not None:
        ok = ok and bool((root[term] == idx[term]).all()) and bool((root[nt] == root.index_select(0, s_nt)).all())
    if sum_ is not None:
        w = weight[nt].to(torch.int64) if weight is not None else torch.ones_like(s_nt, dtype=torch.int64)
        ok = ok and bool((sum_[term] == 0).all()) and bool((sum_[nt] == sum_.index_select(0, s_nt) + w).all())
    return ok
