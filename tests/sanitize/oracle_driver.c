/*
 * oracle_driver.c -- drives every entry point of the CPU oracle (oracle.c) over
 * small seeded inputs, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py).  Test
 * infrastructure: it checks only what holds by definition of a stable sort
 * (the output is ordered, and equal keys keep their input order, which the
 * index payload shows) and of the merge cost (the sum of the merge output
 * sizes over the trace's nodes); the sanitizers catch out-of-bounds accesses,
 * leaks and undefined arithmetic.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t rng_state = 0x2209069092209069ull;

static uint64_t next_u64(void) {   /* xorshift64 */
  uint64_t x = rng_state;
  x ^= x << 13;
  x ^= x >> 7;
  x ^= x << 17;
  rng_state = x;
  return x;
}

static int failures = 0;

#define CHECK(cond, ...)                  \
  do {                                    \
    if (!(cond)) {                        \
      fprintf(stderr, __VA_ARGS__);       \
      fprintf(stderr, "\n");              \
      failures++;                         \
    }                                     \
  } while (0)

/* keys of type kt drawn from `distinct` values (0: the full range), in runs
 * of random lengths, some ascending and some strictly descending */
static void *make_keys(int kt, uint64_t n, uint64_t distinct) {
  size_t ks = kt == ORC_I64 ? 8 : 4;
  unsigned char *k = malloc(n * ks + 8);
  uint64_t i = 0;
  while (i < n) {
    uint64_t len = 1 + next_u64() % 40;
    int dir = (int)(next_u64() % 3);   /* 0 random, 1 ascending-ish, 2 descending-ish */
    uint64_t base = next_u64();
    for (uint64_t j = 0; j < len && i < n; j++, i++) {
      uint64_t v = dir == 0 ? next_u64() : (dir == 1 ? base + j * 977 : base - j * 977);
      if (distinct) v %= distinct;
      if (kt == ORC_I64) {
        int64_t x = (int64_t)v;
        memcpy(k + i * 8, &x, 8);
      } else if (kt == ORC_I32) {
        int32_t x = (int32_t)(uint32_t)v;
        memcpy(k + i * 4, &x, 4);
      } else {
        uint32_t bits = (uint32_t)v;
        if (((bits >> 23) & 0xFF) == 0xFF) bits &= ~(1u << 23);   /* no NaN / inf */
        memcpy(k + i * 4, &bits, 4);
      }
    }
  }
  return k;
}

static void check_sorted_stable(const void *keys, int kt, const uint32_t *pay, uint64_t n,
                                const char *what) {
  for (uint64_t i = 1; i < n; i++) {
    int c = oracle_key_cmp(keys, kt, i - 1, i);
    CHECK(c <= 0, "%s: keys out of order at %llu", what, (unsigned long long)i);
    if (c == 0 && pay)
      CHECK(pay[i - 1] < pay[i], "%s: equal keys out of input order at %llu", what,
            (unsigned long long)i);
  }
}

static void check_trace(const oracle_trace *t, uint64_t n, const char *what) {
  uint64_t m = 0;
  for (uint64_t v = 0; v < t->n_nodes; v++) {
    CHECK(t->nodes[v].end > t->nodes[v].begin && t->nodes[v].end <= n, "%s: bad node span", what);
    m += t->nodes[v].end - t->nodes[v].begin;
  }
  CHECK(m == t->merge_cost, "%s: merge cost %llu != sum of node sizes %llu", what,
        (unsigned long long)t->merge_cost, (unsigned long long)m);
  CHECK(t->r == 0 || t->run_start[t->r] == n, "%s: runs do not end at n", what);
}

static void one_case(int kt, uint64_t n, uint64_t distinct, uint32_t k, uint32_t min_run,
                     int merge_down) {
  char what[160];
  snprintf(what, sizeof what, "kt=%d n=%llu distinct=%llu k=%u min_run=%u merge_down=%d", kt,
           (unsigned long long)n, (unsigned long long)distinct, k, min_run, merge_down);
  void *keys = make_keys(kt, n, distinct);
  uint32_t *pay = malloc((n + 1) * 4);
  for (uint64_t i = 0; i < n; i++) pay[i] = (uint32_t)i;

  /* the run scans on a copy */
  size_t ks = kt == ORC_I64 ? 8 : 4;
  void *kc = malloc(n * ks + 8);
  memcpy(kc, keys, n * ks);
  uint64_t *rs = malloc((n + 2) * 8);
  uint8_t *rd = malloc(n + 1);
  uint64_t r = oracle_runs(kc, kt, n, rs, rd);
  CHECK(n == 0 || (r >= 1 && rs[r] == n), "%s: natural runs", what);
  if (r > 1) {
    uint8_t *pw = malloc(r);
    CHECK(oracle_powers(rs, r, k, pw) == 0, "%s: powers", what);
    oracle_node *nodes = malloc(r * sizeof(oracle_node));
    CHECK(oracle_kway_tree(rs, r, pw, nodes) >= 0, "%s: kway tree", what);
    free(nodes);
    free(pw);
    oracle_trace tt;
    memset(&tt, 0, sizeof tt);
    CHECK(oracle_tree_from_runs_ex(rs, r, k, merge_down, &tt) == 0, "%s: tree from runs", what);
    oracle_trace_free(&tt);
  }
  uint32_t *pc = malloc((n + 1) * 4);
  memcpy(pc, pay, n * 4);
  uint64_t r2 = oracle_runs_min(kc, kt, pc, n, min_run, rs, rd);
  CHECK(n == 0 || rs[r2] == n, "%s: extended runs", what);
  free(pc);

  oracle_trace t;
  memset(&t, 0, sizeof t);
  CHECK(oracle_sort_ex(keys, kt, pay, n, k, min_run, merge_down, &t) == 0, "%s: sort", what);
  check_sorted_stable(keys, kt, pay, n, what);
  check_trace(&t, n, what);
  oracle_trace_free(&t);
  free(kc);
  free(rs);
  free(rd);
  free(keys);
  free(pay);
}

static void many_case(int kt, uint64_t m, uint32_t k) {
  uint64_t *off = malloc((m + 1) * 8);
  off[0] = 0;
  for (uint64_t i = 0; i < m; i++) off[i + 1] = off[i] + next_u64() % 300;   /* empty arrays too */
  uint64_t n = off[m];
  void *keys = make_keys(kt, n ? n : 1, 50);
  uint32_t *pay = malloc((n + 1) * 4);
  for (uint64_t i = 0; i < n; i++) pay[i] = (uint32_t)i;
  uint64_t *mc = malloc(m * 8);
  CHECK(oracle_sort_many(keys, kt, pay, off, m, k, mc) == 0, "sort_many kt=%d", kt);
  for (uint64_t i = 0; i < m; i++) {
    size_t ks = kt == ORC_I64 ? 8 : 4;
    check_sorted_stable((unsigned char *)keys + off[i] * ks, kt, pay + off[i], off[i + 1] - off[i],
                        "sort_many");
  }
  free(mc);
  free(keys);
  free(pay);
  free(off);
}

int main(void) {
  const uint64_t sizes[] = {0, 1, 2, 3, 7, 64, 1000, 20011};
  const uint64_t distincts[] = {0, 2, 16};
  const uint32_t ks[] = {2, 3, 4, 8};
  const uint32_t min_runs[] = {1, 2, 24, 32};
  for (int kt = 0; kt < 3; kt++)
    for (size_t a = 0; a < sizeof sizes / sizeof *sizes; a++)
      for (size_t b = 0; b < sizeof distincts / sizeof *distincts; b++)
        for (size_t c = 0; c < sizeof ks / sizeof *ks; c++)
          for (size_t d = 0; d < sizeof min_runs / sizeof *min_runs; d++)
            for (int md = 0; md < 2; md++)
              one_case(kt, sizes[a], distincts[b], ks[c], min_runs[d], md);
  for (int kt = 0; kt < 3; kt++) many_case(kt, 37, 4);
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("oracle driver: all cases passed\n");
  return 0;
}
