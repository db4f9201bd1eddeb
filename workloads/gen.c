/*
 * Seeded synthetic input generators for list ranking.
 *
 * This module builds successor arrays (and weights) shaped like the paper's
 * workloads: random lists, lists with locality, forests of lists, and Euler
 * tours of trees (Section 3, "Input Instances"). It holds none of the ranking
 * arithmetic: every generator builds a list from an explicit visiting order,
 * so the expected ranks follow from that order in closed form.
 *
 * Randomness is counter based, so results do not depend on the thread count:
 *   draw(seed, stream, i) = mix64(mix64(seed ^ mix64(stream)) + i)
 * where mix64 is the splitmix64 output function (Steele, Lea, Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014).
 *
 * Random permutations are a keyed pseudorandom permutation: a 4-round
 * balanced Feistel network (Luby-Rackoff) over the smallest even bit width
 * covering the domain, with cycle walking (Black-Rogaway, "Ciphers with
 * arbitrary finite domains", CT-RSA 2002) to restrict it to [0, n).
 * Evaluation is O(1) per index, so orders are built in parallel.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t wl_draw(uint64_t seed, uint64_t stream, uint64_t i) {
    return mix64(mix64(seed ^ mix64(stream)) + i);
}

/* ---------------------------------------------------------------- PRP ---- */

typedef struct {
    uint64_t key[4];
    unsigned half;      /* bits per Feistel half */
    uint64_t mask;      /* (1 << half) - 1 */
    uint64_t n;         /* domain size */
} prp_t;

static void prp_init(prp_t* p, uint64_t seed, uint64_t stream, uint64_t n) {
    unsigned bits = 2;
    while (bits < 64 && (1ULL << bits) < n) bits++;
    if (bits & 1u) bits++;
    p->half = bits / 2;
    p->mask = (1ULL << p->half) - 1;
    p->n = n;
    for (int r = 0; r < 4; r++) p->key[r] = wl_draw(seed, stream, 0x5eed0000ULL + (uint64_t)r);
}

static inline uint64_t prp_round_trip(const prp_t* p, uint64_t x) {
    uint64_t L = x >> p->half, R = x & p->mask;
    for (int r = 0; r < 4; r++) {
        uint64_t nl = R;
        R = L ^ (mix64(p->key[r] ^ R) & p->mask);
        L = nl;
    }
    return (L << p->half) | R;
}

static inline uint64_t prp_eval(const prp_t* p, uint64_t x) {
    uint64_t y = x;
    do { y = prp_round_trip(p, y); } while (y >= p->n);
    return y;
}

/* out[j] = pi(j) for a pseudorandom permutation pi of [0, n). */
void wl_perm(uint64_t seed, uint64_t stream, uint64_t n, uint32_t* out) {
    if (n == 0) return;
    prp_t p;
    prp_init(&p, seed, stream, n);
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < (int64_t)n; j++) out[j] = (uint32_t)prp_eval(&p, (uint64_t)j);
}

/* ------------------------------------------------------------ orders ---- */

/* Link the elements in visiting order: succ[order[j]] = order[j+1]; the last
 * element is the terminal and points to itself. */
void wl_link_order(const uint32_t* order, uint64_t n, uint32_t* succ) {
    if (n == 0) return;
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < (int64_t)n - 1; j++) succ[order[j]] = order[j + 1];
    succ[order[n - 1]] = order[n - 1];
}

/* Order of a list with block locality: the index range is cut into blocks of
 * `block` consecutive ids (the last one may be shorter); blocks are visited in
 * a random order and each block's ids in a random order of their own. */
void wl_block_order(uint64_t seed, uint64_t stream, uint64_t n, uint64_t block, uint32_t* order) {
    if (n == 0 || block == 0) return;
    uint64_t nb = (n + block - 1) / block;
    uint64_t last_len = n - (nb - 1) * block;
    prp_t bp;
    prp_init(&bp, seed, stream * 2 + 1, nb);
    /* list position of the (possibly partial) last block in the block order */
    uint64_t q_partial = 0;
    for (uint64_t q = 0; q < nb; q++)
        if (prp_eval(&bp, q) == nb - 1) { q_partial = q; break; }
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < (int64_t)nb; q++) {
        uint64_t b = prp_eval(&bp, (uint64_t)q);
        uint64_t len = (b == nb - 1) ? last_len : block;
        uint64_t start = (uint64_t)q * block - (((uint64_t)q > q_partial) ? (block - last_len) : 0);
        prp_t ip;
        prp_init(&ip, wl_draw(seed, stream * 2 + 2, b), 7, len);
        for (uint64_t i = 0; i < len; i++) order[start + i] = (uint32_t)(b * block + prp_eval(&ip, i));
    }
}

/* Order of the paper's List(n, gamma) (Section 3, input instances): the
 * identity order 0, 1, ..., n-1, then the ids at k = round(gamma n) list
 * positions, drawn uniformly without replacement, are permuted at random
 * among those positions. k = 0 gives succ[i] = i + 1; k = n a random list. */
void wl_gamma_order(uint64_t seed, uint64_t stream, uint64_t n, uint64_t k, uint32_t* order) {
    if (n == 0) return;
    if (k > n) k = n;
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < (int64_t)n; j++) order[j] = (uint32_t)j;
    if (k == 0) return;
    prp_t pos, sh;
    prp_init(&pos, seed, stream * 2 + 1, n);
    prp_init(&sh, seed, stream * 2 + 2, k);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)k; i++)
        order[prp_eval(&pos, (uint64_t)i)] = (uint32_t)prp_eval(&pos, prp_eval(&sh, (uint64_t)i));
}

/* ------------------------------------------------------------ forest ---- */

/* List lengths for a forest: lengths drawn from the geometric distribution on
 * {1, 2, ...} with the given mean until `short_total` elements are used (the
 * last one truncated to fit), then `n_long` lists of `long_len`.
 * Returns the number of lists; writes at most `cap` lengths (call with
 * lens == NULL to count). */
uint64_t wl_forest_lengths(uint64_t seed, uint64_t short_total, double mean, uint64_t n_long,
                           uint64_t long_len, uint64_t* lens, uint64_t cap) {
    uint64_t cnt = 0, used = 0, i = 0;
    double lq = log1p(-1.0 / mean);
    while (used < short_total) {
        uint64_t d = wl_draw(seed, 31, i++);
        double u = ((double)(d >> 11) + 1.0) * (1.0 / 9007199254740992.0); /* (0, 1] */
        uint64_t len = 1 + (uint64_t)floor(log(u) / lq);
        if (len > short_total - used) len = short_total - used;
        if (lens && cnt < cap) lens[cnt] = len;
        cnt++;
        used += len;
    }
    for (uint64_t j = 0; j < n_long; j++) {
        if (lens && cnt < cap) lens[cnt] = long_len;
        cnt++;
    }
    return cnt;
}

/* Link consecutive chunks of `order` into separate lists; starts[i] is the
 * first position of list i in `order`, starts[count] == n. */
void wl_link_chunks(const uint32_t* order, const uint64_t* starts, uint64_t count, uint32_t* succ) {
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < (int64_t)count; i++) {
        uint64_t a = starts[i], b = starts[i + 1];
        if (a >= b) continue;
        for (uint64_t j = a; j + 1 < b; j++) succ[order[j]] = order[j + 1];
        succ[order[b - 1]] = order[b - 1];
    }
}

/* w[i] uniform in [lo, hi] (inclusive). */
void wl_weights_i64(uint64_t seed, uint64_t stream, uint64_t n, int64_t lo, int64_t hi, int64_t* w) {
    uint64_t span = (uint64_t)(hi - lo) + 1;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; i++)
        w[i] = lo + (int64_t)(((unsigned __int128)wl_draw(seed, stream, (uint64_t)i) * span) >> 64);
}

void wl_weights_i32(uint64_t seed, uint64_t stream, uint64_t n, int32_t lo, int32_t hi, int32_t* w) {
    uint64_t span = (uint64_t)((int64_t)hi - lo) + 1;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; i++)
        w[i] = lo + (int32_t)(((unsigned __int128)wl_draw(seed, stream, (uint64_t)i) * span) >> 64);
}

/* -------------------------------------------------------- Euler tour ---- */

/* Random recursive tree on V vertices: parent[0] = 0 (the root), and
 * parent[v] uniform in [0, v) for v >= 1. */
void wl_recursive_tree(uint64_t seed, uint64_t V, uint32_t* parent) {
    if (V == 0) return;
    parent[0] = 0;
    #pragma omp parallel for schedule(static)
    for (int64_t v = 1; v < (int64_t)V; v++)
        parent[v] = (uint32_t)(((unsigned __int128)wl_draw(seed, 41, (uint64_t)v) * (uint64_t)v) >> 64);
}

/* Depth of every vertex of a tree whose parents have smaller ids:
 * depth[0] = 0, depth[v] = depth[parent[v]] + 1. */
void wl_tree_depth(const uint32_t* parent, uint64_t V, uint32_t* depth) {
    if (V == 0) return;
    depth[0] = 0;
    for (uint64_t v = 1; v < V; v++) depth[v] = depth[parent[v]] + 1;
}

/* Euler tour of a rooted tree as a successor array over its 2(V-1) arcs.
 * Arc ids before relabelling: down(v) = 2(v-1) (parent -> v) and
 * up(v) = 2(v-1)+1 (v -> parent), for v >= 1; ids are then relabelled by a
 * pseudorandom permutation so the arcs sit in random order.
 * Children are visited in ascending id order. The tour starts at the down
 * arc of the root's first child and ends at the up arc of its last child.
 * w32: +1 on down arcs, -1 on up arcs. down_arc[v] = relabelled down(v),
 * up_arc[v] = relabelled up(v) (entries of the root are UINT32_MAX; up_arc
 * may be NULL). The root is vertex 0 (parent[0] == 0); other parents may have
 * any id. */
int wl_euler_tour(uint64_t seed, const uint32_t* parent, uint64_t V, uint32_t* succ, int32_t* w32,
                  uint32_t* down_arc, uint32_t* up_arc) {
    if (V < 2) return 0;
    uint64_t m = 2 * (V - 1);
    uint32_t* first = (uint32_t*)malloc(V * sizeof(uint32_t));
    uint32_t* nexts = (uint32_t*)malloc(V * sizeof(uint32_t));
    if (!first || !nexts) { free(first); free(nexts); return -1; }
    const uint32_t NONE = 0xffffffffu;
    for (uint64_t v = 0; v < V; v++) first[v] = NONE;
    for (uint64_t v = V - 1; v >= 1; v--) {  /* descending: sibling chains come out ascending */
        nexts[v] = first[parent[v]];
        first[parent[v]] = (uint32_t)v;
    }
    nexts[0] = NONE;
    prp_t p;
    prp_init(&p, seed, 43, m);
    down_arc[0] = NONE;
    if (up_arc) up_arc[0] = NONE;
    #pragma omp parallel for schedule(static)
    for (int64_t v = 1; v < (int64_t)V; v++) {
        uint32_t dv = (uint32_t)prp_eval(&p, 2 * (uint64_t)(v - 1));
        uint32_t uv = (uint32_t)prp_eval(&p, 2 * (uint64_t)(v - 1) + 1);
        down_arc[v] = dv;
        if (up_arc) up_arc[v] = uv;
        /* after entering v: go down to its first child, else come back up */
        uint32_t c = first[v];
        succ[dv] = (c != NONE) ? (uint32_t)prp_eval(&p, 2 * (uint64_t)(c - 1)) : uv;
        /* after leaving v: go down to the next sibling, else up from the parent */
        uint32_t s = nexts[v];
        uint32_t pv = parent[v];
        if (s != NONE) succ[uv] = (uint32_t)prp_eval(&p, 2 * (uint64_t)(s - 1));
        else if (pv != 0) succ[uv] = (uint32_t)prp_eval(&p, 2 * (uint64_t)(pv - 1) + 1);
        else succ[uv] = uv; /* last arc of the tour */
        w32[dv] = 1;
        w32[uv] = -1;
    }
    free(first);
    free(nexts);
    return 0;
}
