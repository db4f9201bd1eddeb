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
