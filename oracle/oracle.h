/*
 * oracle.h -- reference CPU implementation of k-way Powersort.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded
 * checker that the GPU library is compared against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does.  It shares no code with the GPU library.
 *
 * Every function follows the paper (Cawley Gelling, Nebel, Smith, Wild,
 * "Multiway Powersort", arXiv 2209.06909) step by step:
 *   - runs:            Section 2 (maximal weakly increasing or strictly
 *                      decreasing segments, found by one left-to-right scan;
 *                      decreasing runs are reversed); optionally extended to
 *                      a minimal run length by insertion sort (Appendix A.3)
 *   - node power:      Definition 3.1 (run-boundary power), evaluated in
 *                      exact integer arithmetic
 *   - merge policy:    Algorithm 2 (KwayPowerSort_k, left-to-right run stack
 *                      that merges a whole group of equal powers at once);
 *                      optionally Appendix A.3's "merge down" final phase
 *   - merge tree:      Algorithm 1 (KwayTree_k), an independent recursive
 *                      construction used as a cross-check
 *   - merging:         Section 2.2 (stable merge of up to k runs; on equal
 *                      keys the leftmost run wins)
 *
 * Parity status: every function here is pinned by the CPU test suite
 * (worked examples of Figures 1 and 3, brute force over all tie patterns
 * of tiny inputs, library stable sorts, and the invariants of Section 3.3).
 * No function is "parity unpinned".
 */
#ifndef MPS_ORACLE_H
#define MPS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Key types.  The oracle orders signed integers numerically and float32 by
 * the IEEE-754 total order (sign-magnitude; -0 < +0; NaNs by bit pattern). */
enum { ORC_I32 = 0, ORC_I64 = 1, ORC_F32 = 2 };

/* Three-way comparison of keys[i] and keys[j]. */
int oracle_key_cmp(const void *keys, int kt, uint64_t i, uint64_t j);

/* Greedy left-to-right run partition (Section 2).
 * run_start must hold n+1 entries, run_desc n entries.  Returns r (0 for n=0).
 * run_start[r] = n.  Keys are not modified. */
uint64_t oracle_runs(const void *keys, int kt, uint64_t n,
                     uint64_t *run_start, uint8_t *run_desc);

/* Runs with a minimal run length min_run (Appendix A.3): natural runs shorter
 * than min_run are extended to min(n, start + min_run) elements by a stable
 * insertion sort; the next run starts where the extended one ends.  Keys and
 * payload (nullable) are rearranged in place: every run is left ascending.
 * run_desc[i] = 1 iff run i is a strictly decreasing natural run that was
 * reversed whole (not extended).  min_run <= 1: the natural runs, reversed. */
uint64_t oracle_runs_min(void *keys, int kt, uint32_t *payload, uint64_t n,
                         uint32_t min_run, uint64_t *run_start, uint8_t *run_desc);

/* Definition 3.1: k-way power of the boundary at s_cur between the run
 * [s_prev, s_cur) and the run [s_cur, s_next) of an array of length n.
 * Returns P >= 1, or -1 on invalid arguments. */
int oracle_power(uint64_t n, uint64_t s_prev, uint64_t s_cur, uint64_t s_next,
                 uint32_t k);

/* All boundary powers of a run partition: power[i-1] = P_i for i = 1..r-1. */
int oracle_powers(const uint64_t *run_start, uint64_t r, uint32_t k,
                  uint8_t *power);

/* One merge-tree node.  Children are the d = arity adjacent segments
 * [child_bound[0], child_bound[1]), ..., [child_bound[d-1], child_bound[d]);
 * child_bound[0] = begin, child_bound[d] = end.  Boundaries are given as
 * boundary indices (boundary i starts run i). */
typedef struct {
    uint64_t begin, end;        /* element span */
    uint64_t first_boundary;    /* leftmost boundary index of the node */
    uint32_t arity;             /* d, 2 <= d <= k */
    uint32_t power;             /* common power of the node's d-1 boundaries */
    uint32_t depth;             /* edges to the root */
    int64_t parent;             /* node index, -1 for the root */
} oracle_node;

typedef struct {
    uint64_t n, r;
    uint32_t k;
    uint64_t *run_start;        /* r+1 */
    uint8_t *run_desc;          /* r */
    uint8_t *power;             /* r-1: power[i-1] = P_i */
    uint64_t n_nodes;
    oracle_node *nodes;         /* in the order the merges happen */
    uint64_t *boundary_node;    /* r-1: node that owns boundary i (index i-1) */
    uint32_t *leaf_depth;       /* r */
    uint64_t merge_cost;        /* sum of all merge output sizes */
    uint64_t max_stack;         /* largest run-stack height seen (no sentinel) */
} oracle_trace;

/* Stable k-way Powersort of keys (and payload, if not NULL) in place,
 * following Algorithm 2 with the final phase that keeps merging whole
 * equal-power groups (the tree of Algorithm 1).  If trace is not NULL it is
 * filled with malloc'ed arrays; release with oracle_trace_free.
 * Returns 0 on success, negative on error. */
int oracle_sort(void *keys, int kt, uint32_t *payload, uint64_t n, uint32_t k,
                oracle_trace *trace);
void oracle_trace_free(oracle_trace *trace);

/* oracle_sort with a minimal run length (oracle_runs_min; min_run <= 1: the
 * natural runs) and, if merge_down is set, the final phase of the 4-way
 * implementation in Appendix A.3 in place of Algorithm 2's: with s entries
 * left on the stack, the top s mod (k-1) entries are merged with the current
 * segment first, then k-1 entries at a time.  Such a node records the power
 * of its first boundary. */
int oracle_sort_ex(void *keys, int kt, uint32_t *payload, uint64_t n, uint32_t k,
                   uint32_t min_run, int merge_down, oracle_trace *trace);

/* Algorithm 1 (KwayTree_k) over a given run partition and its powers.
 * nodes must hold r-1 entries; returns the node count (post-order:
 * children left to right, then the node).  depth and parent are filled. */
int64_t oracle_kway_tree(const uint64_t *run_start, uint64_t r,
                         const uint8_t *power, oracle_node *nodes);

/* Merge-tree construction alone (Algorithm 2's stack discipline over the
 * given runs and powers, no element movement).  Fills a trace whose
 * run_start/run_desc/power are copies of the inputs. */
int oracle_tree_from_runs(const uint64_t *run_start, uint64_t r,
                          uint32_t k, oracle_trace *trace);
/* The same with the merge-down final phase (see oracle_sort_ex) if set. */
int oracle_tree_from_runs_ex(const uint64_t *run_start, uint64_t r, uint32_t k,
                             int merge_down, oracle_trace *trace);

/* Sorts each segment [offsets[i], offsets[i+1]) independently (its own n,
 * runs and tree); merge_cost (nullable) receives each segment's cost. */
int oracle_sort_many(void *keys, int kt, uint32_t *payload,
                     const uint64_t *offsets, uint64_t m, uint32_t k,
                     uint64_t *merge_cost);

#ifdef __cplusplus
}
#endif
#endif
