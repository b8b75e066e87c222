/*
 * oracle.c -- reference CPU implementation of k-way Powersort.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain, slow and sequential on
 * purpose: every step is written so that it can be checked against the
 * paper by eye.  Nothing here is blocked, fused or reordered.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Key order                                                           */
/* ------------------------------------------------------------------ */

static size_t key_size(int kt) { return kt == ORC_I64 ? 8 : 4; }

/* IEEE-754 total order on the bit patterns of two float32 values:
 * negative values come before non-negative ones (so -0 < +0); among
 * non-negative values a larger magnitude is larger; among negative values a
 * larger magnitude is smaller. */
static int f32_bits_cmp(uint32_t a, uint32_t b) {
    int neg_a = (int)(a >> 31), neg_b = (int)(b >> 31);
    if (neg_a != neg_b) return neg_a ? -1 : 1;
    if (a == b) return 0;
    if (!neg_a) return a < b ? -1 : 1;
    return a > b ? -1 : 1;
}

int oracle_key_cmp(const void *keys, int kt, uint64_t i, uint64_t j) {
    if (kt == ORC_I32) {
        int32_t a = ((const int32_t *)keys)[i], b = ((const int32_t *)keys)[j];
        return (a > b) - (a < b);
    }
    if (kt == ORC_I64) {
        int64_t a = ((const int64_t *)keys)[i], b = ((const int64_t *)keys)[j];
        return (a > b) - (a < b);
    }
    uint32_t a = ((const uint32_t *)keys)[i], b = ((const uint32_t *)keys)[j];
    return f32_bits_cmp(a, b);
}

/* ------------------------------------------------------------------ */
/* Runs (Section 2)                                                    */
/* ------------------------------------------------------------------ */

/* One left-to-right scan.  A run starting at i is strictly decreasing if
 * its first pair is strictly decreasing (then it extends while the keys keep
 * strictly decreasing); otherwise it is weakly increasing and extends while
 * the keys do not decrease.  Equal neighbours therefore start an increasing
 * run.  A run starting at the last element has length 1. */
uint64_t oracle_runs(const void *keys, int kt, uint64_t n,
                     uint64_t *run_start, uint8_t *run_desc) {
    uint64_t r = 0, i = 0;
    while (i < n) {
        uint64_t j = i + 1;
        uint8_t desc = 0;
        if (j < n && oracle_key_cmp(keys, kt, j, i) < 0) {
            desc = 1;
            while (j < n && oracle_key_cmp(keys, kt, j, j - 1) < 0) j++;
        } else {
            while (j < n && oracle_key_cmp(keys, kt, j, j - 1) >= 0) j++;
        }
        run_start[r] = i;
        run_desc[r] = desc;
        r++;
        i = j;
    }
    run_start[r] = n;
    return r;
}

/* Reverse elements [b, e) of keys (and payload). */
static void reverse_range(unsigned char *keys, size_t ks, uint32_t *payload,
                          uint64_t b, uint64_t e);

/* Three-way comparison of two key values given by address. */
static int value_cmp(int kt, const unsigned char *a, const unsigned char *b) {
    unsigned char pair[16];
    size_t ks = key_size(kt);
    memcpy(pair, a, ks);
    memcpy(pair + ks, b, ks);
    return oracle_key_cmp(pair, kt, 0, 1);
}

/* Runs with a minimal run length (the 4-way Powersort implementation of
 * Appendix A.3, as in Timsort).  Scanning left to right from b = 0: the
 * natural run starting at b is found as in oracle_runs and, if strictly
 * decreasing, reversed at once.  If it is shorter than min_run it is
 * extended to min(n, b + min_run) elements, and the added elements are put
 * into place one by one by a stable insertion sort (each is shifted left past
 * the strictly larger keys only).  The next run starts where this one ends.
 * Keys and payload are rearranged in place.  run_desc[i] is 1 iff run i is
 * a strictly decreasing natural run that was reversed and not extended.
 * min_run <= 1 gives exactly the natural runs (and reverses them). */
uint64_t oracle_runs_min(void *keys_v, int kt, uint32_t *payload, uint64_t n,
                         uint32_t min_run, uint64_t *run_start, uint8_t *run_desc) {
    unsigned char *keys = keys_v;
    size_t ks = key_size(kt);
    unsigned char x[8];
    uint64_t r = 0, b = 0;
    while (b < n) {
        uint64_t e = b + 1;
        uint8_t desc = 0;
        if (e < n && oracle_key_cmp(keys, kt, e, b) < 0) {
            desc = 1;
            while (e < n && oracle_key_cmp(keys, kt, e, e - 1) < 0) e++;
        } else {
            while (e < n && oracle_key_cmp(keys, kt, e, e - 1) >= 0) e++;
        }
        if (desc) reverse_range(keys, ks, payload, b, e);
        int extended = 0;
        if (min_run > 1 && e - b < min_run) {
            uint64_t e2 = b + min_run < n ? b + min_run : n;
            extended = e2 > e;
            for (uint64_t i = e; i < e2; i++) {
                memcpy(x, keys + i * ks, ks);
                uint32_t xv = payload ? payload[i] : 0;
                uint64_t j = i;
                while (j > b && value_cmp(kt, keys + (j - 1) * ks, x) > 0) {
                    memcpy(keys + j * ks, keys + (j - 1) * ks, ks);
                    if (payload) payload[j] = payload[j - 1];
                    j--;
                }
                memcpy(keys + j * ks, x, ks);
                if (payload) payload[j] = xv;
            }
            e = e2;
        }
        run_start[r] = b;
        run_desc[r] = (uint8_t)(desc && !extended);
        r++;
        b = e;
    }
    run_start[r] = n;
    return r;
}

/* Reverse elements [b, e) of keys (and payload). */
static void reverse_range(unsigned char *keys, size_t ks, uint32_t *payload,
                          uint64_t b, uint64_t e) {
    unsigned char tmp[8];
    while (e > b + 1) {
        e--;
        memcpy(tmp, keys + b * ks, ks);
        memcpy(keys + b * ks, keys + e * ks, ks);
        memcpy(keys + e * ks, tmp, ks);
        if (payload) {
            uint32_t t = payload[b];
            payload[b] = payload[e];
            payload[e] = t;
        }
        b++;
    }
}

/* ------------------------------------------------------------------ */
/* Node power (Definition 3.1)                                         */
/* ------------------------------------------------------------------ */

/* The midpoints of the two runs, normalised by n, are a = A/(2n) and
 * b = B/(2n) with A = s_prev + s_cur and B = s_cur + s_next.  The power is
 * the least p with floor(a k^p) < floor(b k^p), i.e. the first base-k digit
 * after the radix point in which a and b differ.  The digits are produced
 * exactly: multiply the remainder by k, the integer part of the quotient by
 * 2n is the next digit, keep the remainder.  p = 0 never qualifies because
 * 0 <= a < b < 1. */
int oracle_power(uint64_t n, uint64_t s_prev, uint64_t s_cur, uint64_t s_next,
                 uint32_t k) {
    if (k < 2 || !(s_prev < s_cur && s_cur < s_next && s_next <= n)) return -1;
    unsigned __int128 den = (unsigned __int128)2 * n;
    unsigned __int128 ra = (unsigned __int128)s_prev + s_cur;
    unsigned __int128 rb = (unsigned __int128)s_cur + s_next;
    for (int p = 1; p < 200; p++) {
        ra *= k;
        rb *= k;
        unsigned __int128 da = ra / den, db = rb / den;
        if (da != db) return p;
        ra -= da * den;
        rb -= db * den;
    }
    return -1; /* unreachable: b - a >= 1/n */
}

int oracle_powers(const uint64_t *run_start, uint64_t r, uint32_t k,
                  uint8_t *power) {
    if (r < 2) return 0;
    uint64_t base = run_start[0];
    uint64_t n = run_start[r] - base;
    for (uint64_t i = 1; i < r; i++) {
        int p = oracle_power(n, run_start[i - 1] - base, run_start[i] - base,
                             run_start[i + 1] - base, k);
        if (p < 1 || p > 255) return -1;
        power[i - 1] = (uint8_t)p;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Stable merge of adjacent segments (Section 2.2)                     */
/* ------------------------------------------------------------------ */

typedef struct {
    unsigned char *keys;
    int kt;
    size_t ks;
    uint32_t *payload;
    unsigned char *tmp_keys;   /* scratch of n keys */
    uint32_t *tmp_payload;     /* scratch of n payloads */
} mover;

/* Merges the d sorted adjacent segments [bound[j], bound[j+1]) into
 * [bound[0], bound[d]).  Each output is the least remaining head; a strict
 * comparison keeps the leftmost segment on equal keys, so the merge is
 * stable. */
static void merge_segments(mover *mv, const uint64_t *bound, uint32_t d) {
    uint64_t b = bound[0], e = bound[d];
    size_t ks = mv->ks;
    memcpy(mv->tmp_keys + b * ks, mv->keys + b * ks, (size_t)(e - b) * ks);
    if (mv->payload)
        memcpy(mv->tmp_payload + b, mv->payload + b, (size_t)(e - b) * 4);
    uint64_t head[64];
    for (uint32_t j = 0; j < d; j++) head[j] = bound[j];
    for (uint64_t out = b; out < e; out++) {
        int best = -1;
        for (uint32_t j = 0; j < d; j++) {
            if (head[j] >= bound[j + 1]) continue;
            if (best < 0 ||
                oracle_key_cmp(mv->tmp_keys, mv->kt, head[j], head[best]) < 0)
                best = (int)j;
        }
        memcpy(mv->keys + out * ks, mv->tmp_keys + head[best] * ks, ks);
        if (mv->payload) mv->payload[out] = mv->tmp_payload[head[best]];
        head[best]++;
    }
}

/* ------------------------------------------------------------------ */
/* Merge policy (Algorithm 2)                                          */
/* ------------------------------------------------------------------ */

typedef struct {
    uint64_t begin, end;
    uint64_t first_run;   /* run index of the leftmost run of the segment */
    int64_t node;         /* node that produced the segment, -1 for a run */
    uint32_t power;       /* power of the boundary right of the segment */
} stack_entry;

typedef struct {
    const uint64_t *run_start;
    uint64_t r;
    const uint8_t *power;
    mover *mv;                  /* NULL: build the tree only */
    oracle_node *nodes;
    uint64_t n_nodes;
    uint64_t *boundary_node;    /* r-1 */
    int64_t *leaf_parent;       /* r */
    stack_entry *stack;
    uint64_t top;               /* number of entries (the power-0 sentinel is implicit) */
    uint64_t max_stack;
    uint64_t merge_cost;
    uint32_t k;
    int merge_down;             /* final phase of Appendix A.3 instead of Algorithm 2's */
} policy;

/* Pops the top g entries and merges them together with the current segment;
 * the merged segment becomes the current segment.  The new node records the
 * power pw. */
static int merge_top(policy *pl, stack_entry *cur, uint64_t g, uint32_t pw) {
    uint32_t d = (uint32_t)g + 1;
    if (d > 64) return -1;
    stack_entry parts[64];
    for (uint64_t j = 0; j < g; j++) parts[j] = pl->stack[pl->top - g + j];
    parts[g] = *cur;
    pl->top -= g;

    uint64_t bound[65];
    for (uint32_t j = 0; j < d; j++) bound[j] = parts[j].begin;
    bound[d] = cur->end;
    if (pl->mv) merge_segments(pl->mv, bound, d);

    int64_t id = (int64_t)pl->n_nodes++;
    oracle_node *v = &pl->nodes[id];
    v->begin = bound[0];
    v->end = bound[d];
    v->first_boundary = parts[1].first_run;
    v->arity = d;
    v->power = pw;
    v->depth = 0;
    v->parent = -1;
    for (uint32_t j = 0; j < d; j++) {
        if (parts[j].node >= 0) pl->nodes[parts[j].node].parent = id;
        else pl->leaf_parent[parts[j].first_run] = id;
        if (j > 0) pl->boundary_node[parts[j].first_run - 1] = (uint64_t)id;
    }
    pl->merge_cost += bound[d] - bound[0];
    cur->begin = bound[0];
    cur->first_run = parts[0].first_run;
    cur->node = id;
    return 0;
}

/* Pops the whole group of top entries that share the top power and merges
 * them together with the current segment, as in the inner loop of
 * Algorithm 2. */
static int merge_group(policy *pl, stack_entry *cur) {
    uint32_t pw = pl->stack[pl->top - 1].power;
    uint64_t g = 0;
    while (g < pl->top && pl->stack[pl->top - 1 - g].power == pw) g++;
    return merge_top(pl, cur, g, pw);
}

/* The final phase of the 4-way implementation in Appendix A.3 ("merge
 * down"), for any k: with s entries left on the stack there are s + 1 runs;
 * first the top e = s mod (k-1) entries are merged with the current segment
 * (a 2- or 3-way merge for k = 4), so that every later merge takes k - 1
 * entries, a k-way merge.  A node made here records the power of its first
 * boundary (the boundary right of its first child). */
static uint32_t first_boundary_power(const policy *pl, const stack_entry *cur, uint64_t g) {
    uint64_t b = g >= 2 ? pl->stack[pl->top - g + 1].first_run : cur->first_run;
    return pl->power[b - 1];
}

static int merge_down(policy *pl, stack_entry *cur) {
    uint64_t km1 = pl->k - 1;
    uint64_t e = pl->top % km1;
    if (e > 0 && merge_top(pl, cur, e, first_boundary_power(pl, cur, e))) return -1;
    while (pl->top > 0) {
        uint64_t g = pl->top < km1 ? pl->top : km1;
        if (merge_top(pl, cur, g, first_boundary_power(pl, cur, g))) return -1;
    }
    return 0;
}

static int run_policy(policy *pl) {
    uint64_t r = pl->r;
    if (r == 0) return 0;
    stack_entry cur = {pl->run_start[0], pl->run_start[1], 0, -1, 0};
    for (uint64_t i = 1; i < r; i++) {
        uint32_t p = pl->power[i - 1];  /* P_i: boundary between runs i-1 and i */
        while (pl->top > 0 && pl->stack[pl->top - 1].power > p)
            if (merge_group(pl, &cur)) return -1;
        cur.power = p;
        pl->stack[pl->top++] = cur;
        if (pl->top > pl->max_stack) pl->max_stack = pl->top;
        stack_entry next = {pl->run_start[i], pl->run_start[i + 1], i, -1, 0};
        cur = next;
    }
    if (pl->merge_down) return merge_down(pl, &cur);
    /* Final phase: keep merging whole equal-power groups, exactly as if one
     * more boundary of power 0 (below every real power) arrived. */
    while (pl->top > 0)
        if (merge_group(pl, &cur)) return -1;
    return 0;
}

/* Depths: every parent is created after its children, so a reverse sweep
 * over the creation order sees each parent before its children. */
static void fill_depths(oracle_node *nodes, uint64_t n_nodes) {
    for (uint64_t t = n_nodes; t-- > 0;) {
        int64_t p = nodes[t].parent;
        nodes[t].depth = p < 0 ? 0 : nodes[p].depth + 1;
    }
}

static int build_trace(const uint64_t *run_start, uint64_t r, uint32_t k,
                       const uint8_t *power_in, mover *mv, int merge_down,
                       oracle_trace *tr) {
    memset(tr, 0, sizeof *tr);
    tr->r = r;
    tr->k = k;
    tr->n = r ? run_start[r] - run_start[0] : 0;
    tr->run_start = malloc((r + 1) * sizeof(uint64_t));
    tr->run_desc = calloc(r ? r : 1, 1);
    tr->power = calloc(r ? r : 1, 1);
    tr->nodes = calloc(r ? r : 1, sizeof(oracle_node));
    tr->boundary_node = calloc(r ? r : 1, sizeof(uint64_t));
    tr->leaf_depth = calloc(r ? r : 1, sizeof(uint32_t));
    int64_t *leaf_parent = malloc((r ? r : 1) * sizeof(int64_t));
    stack_entry *stack = malloc((r ? r : 1) * sizeof(stack_entry));
    if (!tr->run_start || !tr->run_desc || !tr->power || !tr->nodes ||
        !tr->boundary_node || !tr->leaf_depth || !leaf_parent || !stack) {
        free(leaf_parent);
        free(stack);
        oracle_trace_free(tr);
        return -2;
    }
    memcpy(tr->run_start, run_start, (r + 1) * sizeof(uint64_t));
    if (power_in) {
        if (r > 1) memcpy(tr->power, power_in, r - 1);
    } else if (oracle_powers(run_start, r, k, tr->power)) {
        free(leaf_parent);
        free(stack);
        oracle_trace_free(tr);
        return -1;
    }
    for (uint64_t i = 0; i < r; i++) leaf_parent[i] = -1;

    policy pl = {0};
    pl.run_start = run_start;
    pl.r = r;
    pl.power = tr->power;
    pl.mv = mv;
    pl.nodes = tr->nodes;
    pl.boundary_node = tr->boundary_node;
    pl.leaf_parent = leaf_parent;
    pl.stack = stack;
    pl.k = k;
    pl.merge_down = merge_down;
    int rc = run_policy(&pl);
    if (rc == 0) {
        tr->n_nodes = pl.n_nodes;
        tr->merge_cost = pl.merge_cost;
        tr->max_stack = pl.max_stack;
        fill_depths(tr->nodes, tr->n_nodes);
        for (uint64_t i = 0; i < r; i++)
            tr->leaf_depth[i] =
                leaf_parent[i] < 0 ? 0 : tr->nodes[leaf_parent[i]].depth + 1;
    }
    free(leaf_parent);
    free(stack);
    if (rc) oracle_trace_free(tr);
    return rc;
}

int oracle_tree_from_runs(const uint64_t *run_start, uint64_t r, uint32_t k,
                          oracle_trace *trace) {
    if (!run_start || !trace || k < 2) return -1;
    return build_trace(run_start, r, k, NULL, NULL, 0, trace);
}

int oracle_tree_from_runs_ex(const uint64_t *run_start, uint64_t r, uint32_t k,
                             int merge_down, oracle_trace *trace) {
    if (!run_start || !trace || k < 2) return -1;
    return build_trace(run_start, r, k, NULL, NULL, merge_down, trace);
}

int oracle_sort(void *keys, int kt, uint32_t *payload, uint64_t n, uint32_t k,
                oracle_trace *trace) {
    return oracle_sort_ex(keys, kt, payload, n, k, 1, 0, trace);
}

int oracle_sort_ex(void *keys, int kt, uint32_t *payload, uint64_t n, uint32_t k,
                   uint32_t min_run, int merge_down, oracle_trace *trace) {
    if (k < 2 || k > 64 || (n > 0 && !keys)) return -1;
    if (kt != ORC_I32 && kt != ORC_I64 && kt != ORC_F32) return -1;
    size_t ks = key_size(kt);
    uint64_t *run_start = malloc((n + 1) * sizeof(uint64_t));
    uint8_t *run_desc = malloc(n ? n : 1);
    mover mv = {keys, kt, ks, payload, malloc((n ? n : 1) * ks),
                payload ? malloc((n ? n : 1) * 4) : NULL};
    if (!run_start || !run_desc || !mv.tmp_keys || (payload && !mv.tmp_payload)) {
        free(run_start);
        free(run_desc);
        free(mv.tmp_keys);
        free(mv.tmp_payload);
        return -2;
    }
    uint64_t r;
    if (min_run <= 1) {
        r = oracle_runs(keys, kt, n, run_start, run_desc);
        /* Strictly decreasing runs hold no equal keys, so reversing them keeps
         * the sort stable. */
        for (uint64_t i = 0; i < r; i++)
            if (run_desc[i])
                reverse_range(keys, ks, payload, run_start[i], run_start[i + 1]);
    } else {
        r = oracle_runs_min(keys, kt, payload, n, min_run, run_start, run_desc);
    }

    oracle_trace local;
    oracle_trace *tr = trace ? trace : &local;
    int rc = build_trace(run_start, r, k, NULL, &mv, merge_down, tr);
    if (rc == 0) memcpy(tr->run_desc, run_desc, r);
    if (!trace && rc == 0) oracle_trace_free(&local);
    free(run_start);
    free(run_desc);
    free(mv.tmp_keys);
    free(mv.tmp_payload);
    return rc;
}

void oracle_trace_free(oracle_trace *tr) {
    if (!tr) return;
    free(tr->run_start);
    free(tr->run_desc);
    free(tr->power);
    free(tr->nodes);
    free(tr->boundary_node);
    free(tr->leaf_depth);
    memset(tr, 0, sizeof *tr);
}

/* ------------------------------------------------------------------ */
/* Merge tree by recursion (Algorithm 1)                               */
/* ------------------------------------------------------------------ */

/* KwayTree over runs [lo, hi): split at every boundary of least power,
 * recurse into the pieces left to right, then emit the node.  Returns the
 * node index, or -1 for a single run (a leaf). */
static int64_t kway_rec(const uint64_t *run_start, const uint8_t *power,
                        uint64_t lo, uint64_t hi, oracle_node *nodes,
                        uint64_t *count) {
    if (hi - lo <= 1) return -1;
    uint32_t minp = 0xFFFFFFFFu;
    for (uint64_t i = lo + 1; i < hi; i++)
        if (power[i - 1] < minp) minp = power[i - 1];
    int64_t kids[256];
    uint32_t d = 0;
    uint64_t piece_lo = lo, first = 0;
    for (uint64_t i = lo + 1; i <= hi; i++) {
        if (i == hi || power[i - 1] == minp) {
            if (d >= 256) return -2;
            if (i < hi && first == 0) first = i;
            kids[d++] = kway_rec(run_start, power, piece_lo, i, nodes, count);
            piece_lo = i;
        }
    }
    int64_t id = (int64_t)(*count)++;
    oracle_node *v = &nodes[id];
    v->begin = run_start[lo];
    v->end = run_start[hi];
    v->first_boundary = first;
    v->arity = d;
    v->power = minp;
    v->parent = -1;
    v->depth = 0;
    for (uint32_t j = 0; j < d; j++)
        if (kids[j] >= 0) nodes[kids[j]].parent = id;
    return id;
}

int64_t oracle_kway_tree(const uint64_t *run_start, uint64_t r,
                         const uint8_t *power, oracle_node *nodes) {
    if (r < 2) return 0;
    uint64_t count = 0;
    kway_rec(run_start, power, 0, r, nodes, &count);
    fill_depths(nodes, count);
    return (int64_t)count;
}

/* ------------------------------------------------------------------ */
/* Many independent arrays                                             */
/* ------------------------------------------------------------------ */

/* Sorts each segment [offsets[i], offsets[i+1]) on its own with
 * oracle_sort (its own n, its own runs and tree).  merge_cost, if not NULL,
 * receives each segment's merge cost. */
int oracle_sort_many(void *keys, int kt, uint32_t *payload,
                     const uint64_t *offsets, uint64_t m, uint32_t k,
                     uint64_t *merge_cost) {
    size_t ks = key_size(kt);
    for (uint64_t i = 0; i < m; i++) {
        uint64_t b = offsets[i], e = offsets[i + 1];
        if (e < b) return -1;
        oracle_trace tr;
        int rc = oracle_sort((unsigned char *)keys + b * ks, kt,
                             payload ? payload + b : NULL, e - b, k,
                             merge_cost ? &tr : NULL);
        if (rc) return rc;
        if (merge_cost) {
            merge_cost[i] = tr.merge_cost;
            oracle_trace_free(&tr);
        }
    }
    return 0;
}
