// Tree computations by the Euler-tour technique on top of list prefix sums.
//
// The paper ranks Euler tours of BFS trees as one of its two input families
// (Section 3, input instances) and names tree algorithms as the users of list
// ranking (Section 1). An Euler tour lists every tree edge twice, as a down
// arc parent(v) -> v and an up arc v -> parent(v). With weight +1 on down arcs
// and -1 on up arcs, one weighted ranking of the tour gives for every arc a
//   rank(a) = #down + #up  and  sum(a) = #down - #up
// over the arcs from a to the end of the tour (the last arc, the terminal,
// excluded). With h the tour's first arc and d, u the down and up arcs of a
// non-root vertex v:
//   depth(v)    = sum(h) - sum(d) + 1            (down arcs minus up arcs before v, plus its own)
//   preorder(v) = #down arcs before d + 1 = (rank(h) + sum(h)) / 2 - (rank(d) + sum(d)) / 2 + 1
//   size(v)     = (rank(d) - rank(u) + 1) / 2    (the arcs from d to u enter and leave the subtree)
// and the root has depth 0, preorder 0, size V. The tour of a tree with V
// vertices has m = 2(V - 1) arcs and ends on an up arc into the root, so
// rank(h) = m - 1 and sum(h) = (V - 1) - (V - 2) = 1 are known in advance:
//   depth(v) = 2 - sum(d),  preorder(v) = V - (rank(d) + sum(d)) / 2.
// The prefix sum writes rank and sum of an arc as one 16-byte record, so a
// vertex costs two random record gathers (d and u).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device.hpp"
#include "lr.h"
#include "runner.hpp"

namespace lr {

constexpr int TREE_TPB = 256;
constexpr uint32_t TREE_NONE = 0xffffffffu;

static inline size_t tree_align(size_t v) { return (v + 255) / 256 * 256; }

// w[down(v)] = +1 for every non-root vertex. Validating (BOTH): w was
// cleared to 0 and w[up(v)] = -1 is stored too, so an arc that no vertex
// names keeps weight 0 and arc ids out of range set the error word.
// Otherwise w was cleared to -1, every arc not named as a down arc is an up
// arc, and half the random stores are saved. One byte per arc: the stores
// land in an array a quarter the size of an int32 one.
template <bool BOTH>
__global__ __launch_bounds__(TREE_TPB) void k_tree_weights(const uint32_t* __restrict__ down,
                                                           const uint32_t* __restrict__ up, uint32_t V,
                                                           uint32_t root, uint32_t m, int8_t* __restrict__ w,
                                                           uint32_t* err) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += stride) {
        if (v == root) continue;
        const uint32_t d = down[v];
        if (d < m) w[d] = 1;
        if constexpr (BOTH) {
            const uint32_t u = up[v];
            if (u < m) w[u] = -1;
            if (d >= m || u >= m || d == u) atomicOr(err, 1u);
        }
    }
}

// Sets every weight byte (0 or -1), the head arc and the error word (a
// kernel, not a memset, so the sequence can be captured into a graph).
__global__ __launch_bounds__(TREE_TPB) void k_tree_clear(int8_t* __restrict__ w, uint32_t m, uint32_t fill,
                                                         uint32_t* __restrict__ ctl) {
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) {
        ctl[0] = TREE_NONE;  // head arc
        ctl[1] = 0;          // error bits
    }
    const uint32_t words = (m + 3) / 4;  // w is 256-byte aligned with room for whole words
    for (uint32_t i = g; i < words; i += stride) reinterpret_cast<uint32_t*>(w)[i] = fill;
}

// Validation: every arc must carry +1 or -1 (each named by exactly one vertex).
__global__ __launch_bounds__(TREE_TPB) void k_tree_cover(const int8_t* __restrict__ w, uint32_t m, uint32_t* err) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < m; a += stride)
        if (w[a] == 0) atomicOr(err, 2u);
}

using TRes = Lay<true>::Res;  // (rank, root, sum) of one arc

// Validation: the tour is one list whose first arc has rank m - 1 and sum 1.
__global__ __launch_bounds__(TREE_TPB) void k_tree_head(const TRes* __restrict__ rec, uint32_t m, uint32_t* head,
                                                        uint32_t* err) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < m; a += stride) {
        const TRes r = rec[a];
        if (r.c == m - 1) {
            *head = a;
            if (r.s != 1) atomicOr(err, 4u);
        }
    }
}

__global__ __launch_bounds__(TREE_TPB) void k_tree_headless(const uint32_t* head, uint32_t* err) {
    if (threadIdx.x == 0 && *head == TREE_NONE) atomicOr(err, 4u);  // no arc has rank m - 1
}

__global__ __launch_bounds__(TREE_TPB) void k_tree_vertex(const uint32_t* __restrict__ down,
                                                          const uint32_t* __restrict__ up, uint32_t V, uint32_t root,
                                                          uint32_t m, const TRes* __restrict__ rec, uint32_t* depth,
                                                          uint32_t* preorder, uint32_t* size) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += stride) {
        uint32_t dep = 0, pre = 0, sz = V;
        if (v != root) {
            const uint32_t d = down[v], u = up[v];
            if (d < m && u < m) {
                const TRes rd = rec[d], ru = rec[u];
                dep = (uint32_t)(2 - rd.s);
                pre = (uint32_t)((int64_t)V - ((int64_t)rd.c + rd.s) / 2);
                sz = (uint32_t)(((int64_t)rd.c - (int64_t)ru.c + 1) / 2);
            } else {
                dep = pre = sz = TREE_NONE;
            }
        }
        if (depth) depth[v] = dep;
        if (preorder) preorder[v] = pre;
        if (size) size[v] = sz;
    }
}

static uint32_t tree_grid(uint64_t work) {
    const uint64_t cap = (uint64_t)device_cus() * 8;
    uint64_t g = (work + TREE_TPB * 4 - 1) / (TREE_TPB * 4);
    return (uint32_t)std::max<uint64_t>(1, std::min(g, cap));
}

struct TreeLayout {
    size_t w = 0, rec = 0, ctl = 0, inner = 0, inner_bytes = 0, total = 0;
};

static bool tree_layout(uint64_t V, const lr_opts* opts, TreeLayout* t) {
    const uint64_t m = V >= 2 ? 2 * (V - 1) : 0;
    size_t off = 0;
    t->w = off;
    off += tree_align(m + 4);
    t->rec = off;
    off += tree_align(m * sizeof(TRes) + sizeof(TRes));
    t->ctl = off;  // head arc, error word
    off += 256;
    t->inner = off;
    t->inner_bytes = m ? lr_workspace_bytes(m, LR_W_I32, opts) : 0;
    if (m && !t->inner_bytes) return false;
    off += t->inner_bytes;
    t->total = off + 256;
    return true;
}

}  // namespace lr

using namespace lr;

extern "C" size_t lr_euler_tree_workspace_bytes(uint64_t V, const lr_opts* opts) {
    if (V == 0 || V > (1ull << 30)) return 0;
    TreeLayout t;
    return tree_layout(V, opts, &t) ? t.total : 0;
}

extern "C" lr_status lr_euler_tree(const uint32_t* succ, const uint32_t* down, const uint32_t* up, uint64_t V,
                                   uint32_t root, uint32_t* depth, uint32_t* preorder, uint32_t* size, void* ws,
                                   size_t ws_bytes, const lr_opts* opts, void* stream) {
    if (V == 0) return LR_OK;
    if (V > (1ull << 30)) return LR_ERR_UNSUPPORTED;
    if (root >= V) return LR_ERR_INVALID_ARG;
    const uint64_t m = V >= 2 ? 2 * (V - 1) : 0;
    if (m && (!succ || !down || !up)) return LR_ERR_INVALID_ARG;
    TreeLayout t;
    if (!tree_layout(V, opts, &t)) return LR_ERR_INVALID_ARG;
    if (!ws || ws_bytes < t.total) return LR_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* w0 = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) / 256 * 256);
    int8_t* w = reinterpret_cast<int8_t*>(w0 + t.w);
    TRes* rec = reinterpret_cast<TRes*>(w0 + t.rec);
    uint32_t* head = reinterpret_cast<uint32_t*>(w0 + t.ctl);
    uint32_t* err = head + 1;
    const bool validate = opts && (opts->flags & LR_VALIDATE);
    lr_opts inner = opts ? *opts : lr_opts{};
    inner.flags &= ~(uint32_t)LR_PROFILE;
    // without validation, large tours get their weights from the grouped
    // passes (every byte written in order) instead of a random store per vertex
    bool grouped = false;
    if (m && !validate &&
        tree_arc_weights(down, (uint32_t)V, root, w, (uint32_t)m, w0 + t.inner, &inner, st, &grouped) != hipSuccess)
        return LR_ERR_HIP;
    hipLaunchKernelGGL(k_tree_clear, dim3(grouped ? 1 : tree_grid(m / 4 + 1)), dim3(TREE_TPB), 0, st, w,
                       grouped ? 0u : (uint32_t)m, validate ? 0u : 0xffffffffu, head);
    if (hipGetLastError() != hipSuccess) return LR_ERR_HIP;
    if (m) {
        if (validate)
            hipLaunchKernelGGL(k_tree_weights<true>, dim3(tree_grid(V)), dim3(TREE_TPB), 0, st, down, up,
                               (uint32_t)V, root, (uint32_t)m, w, err);
        else if (!grouped)
            hipLaunchKernelGGL(k_tree_weights<false>, dim3(tree_grid(V)), dim3(TREE_TPB), 0, st, down, up,
                               (uint32_t)V, root, (uint32_t)m, w, err);
        if (validate)
            hipLaunchKernelGGL(k_tree_cover, dim3(tree_grid(m)), dim3(TREE_TPB), 0, st, w, (uint32_t)m, err);
        if (hipGetLastError() != hipSuccess) return LR_ERR_HIP;
        const lr_status s = prefix_sum_records(succ, w, 3, rec, m, w0 + t.inner, t.inner_bytes, &inner, stream);
        if (s != LR_OK) return s;
        if (validate) {
            hipLaunchKernelGGL(k_tree_head, dim3(tree_grid(m)), dim3(TREE_TPB), 0, st, rec, (uint32_t)m, head, err);
            hipLaunchKernelGGL(k_tree_headless, dim3(1), dim3(64), 0, st, head, err);
            if (hipGetLastError() != hipSuccess) return LR_ERR_HIP;
        }
    }
    hipLaunchKernelGGL(k_tree_vertex, dim3(tree_grid(V)), dim3(TREE_TPB), 0, st, down, up, (uint32_t)V, root,
                       (uint32_t)m, rec, depth, preorder, size);
    if (hipGetLastError() != hipSuccess) return LR_ERR_HIP;
    if (validate) {
        uint32_t e = 0;
        if (hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return LR_ERR_HIP;
        if (hipStreamSynchronize(st) != hipSuccess) return LR_ERR_HIP;
        if (e) return LR_ERR_BAD_LIST;
    }
    return LR_OK;
}
