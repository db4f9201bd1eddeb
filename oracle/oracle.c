/*
 * CPU ORACLE FOR LIST RANKING -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * use this file. The GPU library neither links nor calls it, and it shares no
 * code with the GPU library.
 *
 * What it computes (problem definition, Section 1.1 of the paper):
 *   A successor array succ[0..n) describes a set of singly linked lists; a
 *   terminal element points to itself; an element is initial when nothing
 *   points to it. For every element i:
 *     root[i] = the terminal of i's list,
 *     rank[i] = number of links followed from i to reach root[i],
 *     sum[i]  = sum of the link weights w[j] over the elements j on the path
 *               from i to root[i], excluding root[i] itself (a terminal has no
 *               outgoing link, so its weight never counts; sum[t] = 0).
 *   With w[j] = 1 for every non-terminal, sum == rank (the paper notes that
 *   weights 1 on links and 0 on terminals give the unweighted problem).
 *
 * How: sequential pointer chasing (Section 1, the trivial linear-time
 * algorithm). A first pass counts predecessors to find initial elements and
 * rejects malformed input; then, from each initial element, one walk measures
 * the list (length and total weight) and a second walk assigns the values,
 * counting down from the head. Elements never reached from an initial element
 * lie on cycles, which are rejected.
 *
 * Parity status: pinned (brute-force enumeration of every successor array of
 * size <= 7, closed forms of generated inputs, local certificate, special
 * cases; see tests/test_oracle_pins.py).
 *
 * oracle_tree: the tree quantities that list ranking serves through Euler
 * tours (Section 1 names tree algorithms as its users; Section 3 ranks Euler
 * tours of BFS trees), by their plain definitions on a parent array: depth,
 * preorder number (depth-first from the root, children in ascending id order)
 * and subtree size. Pinned by enumeration of every parent array with at most
 * 6 vertices (Cayley's count of rooted labelled trees), closed forms for paths
 * and stars, and structural invariants.
 */
#include <stdint.h>
#include <stdlib.h>

enum {
    ORACLE_OK = 0,
    ORACLE_ERR_RANGE = -1,     /* some succ[i] >= n */
    ORACLE_ERR_INDEGREE = -2,  /* an element has two or more predecessors */
    ORACLE_ERR_CYCLE = -3,     /* some element is not on a path to a terminal */
    ORACLE_ERR_NOMEM = -4,
    ORACLE_ERR_ARG = -5,
};

enum { ORACLE_W_NONE = 0, ORACLE_W_I32 = 1, ORACLE_W_I64 = 2 };

static int64_t link_weight(const void* weight, int wtype, uint64_t i) {
    if (wtype == ORACLE_W_I32) return (int64_t)((const int32_t*)weight)[i];
    if (wtype == ORACLE_W_I64) return ((const int64_t*)weight)[i];
    return 1;
}

/* Rank every element. Any of rank, root, sum may be NULL. Returns ORACLE_OK or
 * a negative ORACLE_ERR_* code (outputs are then unspecified). */
int oracle_rank(const uint32_t* succ, uint64_t n, const void* weight, int wtype,
                uint32_t* rank, uint32_t* root, int64_t* sum) {
    if (n == 0) return ORACLE_OK;
    if (!succ || n > 0xffffffffULL) return ORACLE_ERR_ARG;
    if (wtype != ORACLE_W_NONE && !weight) return ORACLE_ERR_ARG;
    if (wtype < ORACLE_W_NONE || wtype > ORACLE_W_I64) return ORACLE_ERR_ARG;

    /* Pass 1: range check and predecessor marks. */
    uint8_t* has_pred = (uint8_t*)calloc(n, 1);
    if (!has_pred) return ORACLE_ERR_NOMEM;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t s = succ[i];
        if (s >= n) { free(has_pred); return ORACLE_ERR_RANGE; }
        if (s != i) {
            if (has_pred[s]) { free(has_pred); return ORACLE_ERR_INDEGREE; }
            has_pred[s] = 1;
        }
    }

    /* Pass 2: from each initial element, walk the list twice. */
    uint64_t assigned = 0;
    for (uint64_t h = 0; h < n; h++) {
        if (has_pred[h]) continue;
        /* walk 1: number of elements and total link weight */
        uint64_t len = 1, x = h;
        int64_t total = 0;
        while (succ[x] != x) {
            total += link_weight(weight, wtype, x);
            x = succ[x];
            len++;
            if (len > n) { free(has_pred); return ORACLE_ERR_CYCLE; }
        }
        uint64_t term = x;
        /* walk 2: distance and weight to the terminal, counted down from the head */
        uint64_t r = len - 1;
        int64_t s = total;
        x = h;
        for (;;) {
            if (rank) rank[x] = (uint32_t)r;
            if (root) root[x] = (uint32_t)term;
            if (sum) sum[x] = s;
            if (x == term) break;
            s -= link_weight(weight, wtype, x);
            r--;
            x = succ[x];
        }
        assigned += len;
    }
    free(has_pred);
    /* every element of a valid forest lies on exactly one head-to-terminal path */
    return assigned == n ? ORACLE_OK : ORACLE_ERR_CYCLE;
}

/* Tree quantities of a rooted tree given by parent[0..V) with
 * parent[root] == root:
 *   depth[v]    = number of edges on the path from the root to v,
 *   preorder[v] = position of v in the depth-first order from the root that
 *                 takes children in ascending id order (the root is 0),
 *   size[v]     = number of vertices in the subtree rooted at v.
 * Any output may be NULL. Returns ORACLE_OK, ORACLE_ERR_ARG (bad root),
 * ORACLE_ERR_RANGE (a parent id >= V or a second self-parent) or
 * ORACLE_ERR_CYCLE (some vertex does not reach the root). */
int oracle_tree(const uint32_t* parent, uint64_t V, uint32_t root,
                uint32_t* depth, uint32_t* preorder, uint32_t* size) {
    if (V == 0) return ORACLE_OK;
    if (!parent || V > 0xffffffffULL || root >= V || parent[root] != root) return ORACLE_ERR_ARG;
    uint64_t* first = (uint64_t*)calloc(V + 1, sizeof(uint64_t));  /* children of v: kids[first[v] .. first[v+1]) */
    uint32_t* kids = (uint32_t*)malloc((V > 1 ? V - 1 : 1) * sizeof(uint32_t));
    uint64_t* fill = (uint64_t*)malloc(V * sizeof(uint64_t));
    uint32_t* stack = (uint32_t*)malloc(V * sizeof(uint32_t));
    uint32_t* order = (uint32_t*)malloc(V * sizeof(uint32_t));
    uint32_t* dep = (uint32_t*)malloc(V * sizeof(uint32_t));
    uint32_t* sz = (uint32_t*)malloc(V * sizeof(uint32_t));
    int rc = ORACLE_OK;
    if (!first || !kids || !fill || !stack || !order || !dep || !sz) { rc = ORACLE_ERR_NOMEM; goto out; }
    for (uint64_t v = 0; v < V; v++) {
        if (v == root) continue;
        if (parent[v] >= V || parent[v] == v) { rc = ORACLE_ERR_RANGE; goto out; }
        first[parent[v] + 1]++;
    }
    for (uint64_t v = 0; v < V; v++) first[v + 1] += first[v];
    for (uint64_t v = 0; v < V; v++) fill[v] = first[v];
    for (uint64_t v = 0; v < V; v++)                 /* ascending v: each child list ascending */
        if (v != root) kids[fill[parent[v]]++] = (uint32_t)v;
    /* depth-first order: pop a vertex, number it, push its children last-first */
    uint64_t top = 0, visited = 0;
    stack[top++] = root;
    dep[root] = 0;
    while (top) {
        uint32_t v = stack[--top];
        order[visited++] = v;
        for (uint64_t j = first[v + 1]; j > first[v]; j--) {
            uint32_t c = kids[j - 1];
            dep[c] = dep[v] + 1;
            stack[top++] = c;
        }
    }
    if (visited != V) { rc = ORACLE_ERR_CYCLE; goto out; }
    /* sizes: every vertex after all of its descendants in reverse order */
    for (uint64_t v = 0; v < V; v++) sz[v] = 1;
    for (uint64_t j = V; j-- > 1;) {
        uint32_t v = order[j];
        sz[parent[v]] += sz[v];
    }
    for (uint64_t j = 0; j < V; j++) {
        uint32_t v = order[j];
        if (preorder) preorder[v] = (uint32_t)j;
        if (depth) depth[v] = dep[v];
        if (size) size[v] = sz[v];
    }
out:
    free(first); free(kids); free(fill); free(stack); free(order); free(dep); free(sz);
    return rc;
}
