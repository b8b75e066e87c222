// mps_minrun.hip -- runs with a minimal run length (Appendix A.3).
//
// The paper's implementation finds runs left to right and, when the natural
// run starting at b is shorter than the minimal run length m, extends it to
// min(n, b + m) elements by insertion sort; the next run starts where that one
// ends.  The run starts are therefore the chain b_0 = 0, b_{i+1} = next(b_i),
//   next(b) = max(runend(b), min(n, b + m)),
// where runend(b) ends the natural run that starts at b (weakly increasing, or
// strictly decreasing if its first pair is).
//
// runend(b) matters only where it exceeds b + m.  With the natural runs
// R_i = [s_i, t_i) of the whole array (direction d_i) there are two kinds of
// such "jump sources":
//  - b in R_i with b <= t_i - m - 1: the run from b continues to t_i;
//  - b = t_i - 1 with t_i < n: the pair (b, b+1) runs against d_i, so the run
//    from b covers R_{i+1} iff R_{i+1} runs that way (else it has length 2);
//    it jumps iff it covers R_{i+1} and t_{i+1} - t_i >= m.
// Every other position advances by exactly m.
//
// The chain is resolved in chunks of kMrChunk positions.  It enters chunk c
// (first position c0) either at c0 + j, j < m, or, after a jump that lands
// beyond c0 + m - 1, at the end of the run from c0 - 1: a run from b < c0 that
// covers c0 - 1 and c0 runs in the direction of that pair and ends where the
// run from c0 - 1 ends.  Each chunk walks all m + 1 candidate entries and
// records, for each, the runs it starts and the candidate entry of the next
// chunk it leaves by.  These maps are composed over groups of kMrGroup chunks,
// then over the groups from chunk 0's entry 0; each chunk finally re-walks its
// actual entry and writes its run starts.  The runs that were extended are
// then sorted in place by a stable rank sort in registers, staged through LDS.
#include "mps_internal.h"

namespace mps {
namespace {

constexpr int kMrThreads = 256;
constexpr int kMrStage = kMrChunk / 2 + 8;   // natural runs staged per chunk (>= chunk/2 + 4)
constexpr uint8_t kMrEnd = 254;              // the chain has reached n
constexpr uint8_t kMrBad = 255;              // unused candidate
constexpr int kMrSortRuns = 128;             // runs per workgroup of the run sort
constexpr uint32_t kErrMinRun = 1024u;       // plan->error bit of a failed chain check

// Natural runs that overlap [c0 - 1, c1) of chunk c, plus the next two
// starts, staged as 32-bit positions (n <= 2^31).
struct MrSmem {
  uint32_t rs[kMrStage];
  uint8_t d[kMrStage];
  uint16_t seg[2 * kMrStage];      // jump sources: local run index * 2 + kind
  uint32_t rec[kMrChunk / 2 + 4];  // chain positions of the emitting walk
  int scan[kMrThreads / 64];
  int misc[4];
};

__device__ inline int block_excl_scan(int v, int *tmp, int &total) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) tmp[wave] = incl;
  __syncthreads();
  int pre = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < kMrThreads / 64; w++) {
    const int x = tmp[w];
    pre += w < wave ? x : 0;
    total += x;
  }
  __syncthreads();
  return pre + incl - v;
}

// Stages runs ia .. ib - 1 (those overlapping [c0 - 1, c1)) with the starts up
// to run ib + 1, and lists their jump sources in position order (the interval
// of run j, then the point t_j - 1, then run j + 1's interval).  Returns the
// number of staged runs (ib - ia), or -1 if they do not fit.
__device__ inline int mr_stage(const uint64_t *__restrict__ rs, const uint8_t *__restrict__ desc,
                               uint64_t r, uint64_t ia, uint64_t ib, uint32_t N, uint32_t m,
                               MrSmem &sm) {
  constexpr int kPer = (kMrStage + kMrThreads - 1) / kMrThreads;
  const int t = threadIdx.x;
  const uint64_t last = ib + 1 < r ? ib + 1 : r;
  const int ns = (int)(last - ia + 1);
  const int nrun = (int)(ib - ia);
  if (ns > kMrStage) return -1;
  // every load of a thread is issued before the first store
  uint32_t v[kPer];
  uint8_t dv[kPer];
#pragma unroll
  for (int u = 0; u < kPer; u++) {
    const int j = t + u * kMrThreads;
    v[u] = 0;
    dv[u] = 0;
    if (j < ns) {
      v[u] = (uint32_t)rs[ia + j];
      if (ia + j < r) dv[u] = desc[ia + j];
    }
  }
#pragma unroll
  for (int u = 0; u < kPer; u++) {
    const int j = t + u * kMrThreads;
    if (j < ns) {
      sm.rs[j] = v[u];
      sm.d[j] = dv[u];
    }
  }
  __syncthreads();
  // thread t lists the jump sources of runs [t*kPer, t*kPer + kPer) in order;
  // one scan gives every thread its place in the list
  const int j0 = t * kPer;
  uint32_t fl = 0;   // bit 2u: interval of run j0+u, bit 2u+1: its end point
  int c = 0;
#pragma unroll
  for (int u = 0; u < kPer; u++) {
    const int j = j0 + u;
    if (j < nrun) {
      const uint32_t s = sm.rs[j], e = sm.rs[j + 1];
      const bool hi = e - s > m;
      bool hp = false;
      if (e < N) {
        const uint8_t against = sm.d[j] ^ 1;
        hp = sm.d[j + 1] == against && sm.rs[j + 2] - e >= m;
      }
      fl |= (hi ? 1u : 0u) << (2 * u);
      fl |= (hp ? 1u : 0u) << (2 * u + 1);
      c += (int)hi + (int)hp;
    }
  }
  int tot;
  int pos = block_excl_scan(c, sm.scan, tot);
#pragma unroll
  for (int u = 0; u < kPer; u++) {
    if (fl >> (2 * u) & 1u) sm.seg[pos++] = (uint16_t)(2 * (j0 + u));
    if (fl >> (2 * u + 1) & 1u) sm.seg[pos++] = (uint16_t)(2 * (j0 + u) + 1);
  }
  if (t == 0) sm.misc[0] = tot;
  __syncthreads();
  return nrun;
}

__device__ inline uint32_t seg_lo(const MrSmem &sm, int e, uint32_t) {
  const int j = e >> 1;
  return (e & 1) ? sm.rs[j + 1] - 1 : sm.rs[j];
}
__device__ inline uint32_t seg_hi(const MrSmem &sm, int e, uint32_t m) {
  const int j = e >> 1;
  return (e & 1) ? sm.rs[j + 1] - 1 : sm.rs[j + 1] - m - 1;
}
__device__ inline uint32_t seg_tgt(const MrSmem &sm, int e) {
  const int j = e >> 1;
  return (e & 1) ? sm.rs[j + 2] : sm.rs[j + 1];
}

// The end of the run that starts at q, for q inside staged run j.
__device__ inline uint32_t run_end_at(const MrSmem &sm, int j, uint32_t q, uint32_t N) {
  const uint32_t e = sm.rs[j + 1];
  if (q + 1 < e) return e;
  if (e == N) return N;
  return sm.d[j + 1] == (sm.d[j] ^ 1) ? sm.rs[j + 2] : e + 1;
}

// Follows the chain from b through the chunk ending at c1; counts the runs it
// starts (and records their starts if rec is set).  Returns where it leaves.
// Between jump sources the chain is an arithmetic progression of step m, so
// it is advanced to the next jump source (or the chunk end) in one step.
__device__ inline uint32_t mr_walk(const MrSmem &sm, int nseg, uint32_t b, uint32_t c1,
                                   uint32_t N, uint32_t m, int &cnt, uint32_t *rec) {
  int j = 0;
  cnt = 0;
  while (b < c1) {
    while (j < nseg && seg_hi(sm, sm.seg[j], m) < b) j++;
    if (j < nseg && seg_lo(sm, sm.seg[j], m) <= b) {
      if (rec) rec[cnt] = b;
      b = seg_tgt(sm, sm.seg[j]);
      cnt++;
      continue;
    }
    // no jump source holds b: runs of m start at b, b+m, ... up to the first
    // position at or past the next jump source's start (or c1)
    uint32_t lim = j < nseg ? seg_lo(sm, sm.seg[j], m) : c1;
    lim = lim < c1 ? lim : c1;
    const uint32_t steps = (lim - b + m - 1) / m;
    if (rec)
      for (uint32_t q = 0; q < steps; q++) rec[cnt + (int)q] = b + q * m;
    cnt += (int)steps;
    b = N - b > steps * m ? b + steps * m : N;
  }
  return b;
}

// first[c] = index of the first natural run starting at or after c * kMrChunk.
__global__ __launch_bounds__(256) void k_mr_first(const uint64_t *__restrict__ rs,
                                                  const Plan *__restrict__ plan, uint64_t nch,
                                                  uint32_t *__restrict__ first) {
  const uint64_t r = plan->r;
  for (uint64_t c = blockIdx.x * 256ull + threadIdx.x; c <= nch; c += gridDim.x * 256ull) {
    const uint64_t x = c * kMrChunk;
    uint64_t lo = 0, hi = r;   // first index in [0, r] with rs[index] >= x
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (rs[mid] < x) lo = mid + 1; else hi = mid;
    }
    first[c] = (uint32_t)(c == nch ? r : lo);
  }
}

// Per chunk: the exit candidate and run count of every candidate entry.
__global__ __launch_bounds__(kMrThreads) void k_mr_chunk(
    const uint64_t *__restrict__ rs, const uint8_t *__restrict__ desc, Plan *plan, uint32_t N,
    uint32_t m, uint64_t nch, const uint32_t *__restrict__ first, uint8_t *__restrict__ nxt,
    uint16_t *__restrict__ cnt) {
  __shared__ MrSmem sm;
  const int t = threadIdx.x;
  const uint64_t r = plan->r;
  for (uint64_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const uint32_t c0 = (uint32_t)(c * kMrChunk);
    const uint32_t c1 = N - c0 > (uint32_t)kMrChunk ? c0 + kMrChunk : N;
    const uint64_t ia = c > 0 ? first[c] - 1 : 0, ib = first[c + 1];
    const int nrun = mr_stage(rs, desc, r, ia, ib, N, m, sm);
    if (nrun < 0) {
      if (t == 0) atomicOr(&plan->error, kErrMinRun);
      __syncthreads();
      continue;
    }
    const int nseg = sm.misc[0];
    if (t <= (int)m) {
      uint32_t e = 0;
      bool ok;
      if (t < (int)m) {
        e = c0 + t;
        ok = e < N;
      } else {
        e = c > 0 ? run_end_at(sm, 0, c0 - 1, N) : 0;
        ok = c > 0 && e >= c0 + m;
      }
      uint8_t code = kMrBad;
      int k = 0;
      if (ok) {
        const uint32_t X = mr_walk(sm, nseg, e, c1, N, m, k, nullptr);
        if (X >= N) {
          code = kMrEnd;
        } else if (X - c1 < m) {
          code = (uint8_t)(X - c1);
        } else {
          // a jump past the next chunk's first m positions: it must end where
          // the run from c1 - 1 ends (staged run nrun - 1 holds c1 - 1)
          code = (uint8_t)m;
          if (X != run_end_at(sm, nrun - 1, c1 - 1, N)) atomicOr(&plan->error, kErrMinRun);
        }
      }
      nxt[c * kMrCand + t] = code;
      cnt[c * kMrCand + t] = (uint16_t)k;
    }
    __syncthreads();
  }
}

// One wave per group of kMrGroup chunks: composes the chunk maps.  Lane i
// follows candidate i; the row of a chunk (lane j holds candidate j's exit and
// count) is loaded ahead, independently of where the walk stands, and each
// lane picks its entry with a shuffle.
__global__ __launch_bounds__(64) void k_mr_group(const uint8_t *__restrict__ nxt,
                                                 const uint16_t *__restrict__ cnt, uint64_t nch,
                                                 uint64_t ng, uint32_t m,
                                                 uint8_t *__restrict__ gnxt,
                                                 uint32_t *__restrict__ gcnt) {
  const int lane = threadIdx.x;
  for (uint64_t g = blockIdx.x; g < ng; g += gridDim.x) {
    const uint64_t cb = g * kMrGroup, ce = cb + kMrGroup < nch ? cb + kMrGroup : nch;
    uint32_t idx = lane <= (int)m ? (uint32_t)lane : kMrBad;
    uint32_t tot = 0;
    for (uint64_t c = cb; c < ce; c += 8) {
      uint32_t a[8], b[8];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        a[u] = kMrBad;
        b[u] = 0;
        if (c + u < ce && lane < kMrCand) {
          a[u] = nxt[(c + u) * kMrCand + lane];
          b[u] = cnt[(c + u) * kMrCand + lane];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int sel = idx < (uint32_t)kMrCand ? (int)idx : 0;
        const uint32_t na = (uint32_t)__shfl((int)a[u], sel), nb = (uint32_t)__shfl((int)b[u], sel);
        if (c + u < ce && idx < (uint32_t)kMrCand) {
          tot += nb;
          idx = na;
        }
      }
    }
    if (lane < kMrCand) {
      gnxt[g * kMrCand + lane] = (uint8_t)idx;
      gcnt[g * kMrCand + lane] = tot;
    }
  }
}

// One wave: follows the chain over the groups from chunk 0's entry 0, giving
// every group its entry and first output run; sets r and the end sentinel.
__global__ __launch_bounds__(64) void k_mr_top(const uint8_t *__restrict__ gnxt,
                                               const uint32_t *__restrict__ gcnt, uint64_t ng,
                                               uint64_t N, uint64_t rmax,
                                               uint8_t *__restrict__ gentry,
                                               uint32_t *__restrict__ goff,
                                               uint64_t *__restrict__ out_rs, Plan *plan) {
  const int lane = threadIdx.x;
  uint32_t idx = 0;
  uint64_t tot = 0;
  for (uint64_t g = 0; g < ng; g += 8) {
    uint32_t a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      a[u] = kMrBad;
      b[u] = 0;
      if (g + u < ng && lane < kMrCand) {
        a[u] = gnxt[(g + u) * kMrCand + lane];
        b[u] = gcnt[(g + u) * kMrCand + lane];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int sel = idx < (uint32_t)kMrCand ? (int)idx : 0;
      const uint32_t na = (uint32_t)__shfl((int)a[u], sel), nb = (uint32_t)__shfl((int)b[u], sel);
      if (g + u < ng) {
        if (lane == 0) {
          gentry[g + u] = (uint8_t)idx;
          goff[g + u] = (uint32_t)tot;
        }
        if (idx < (uint32_t)kMrCand) {
          tot += nb;
          idx = na;
        }
      }
    }
  }
  if (lane == 0) {
    plan->r_nat = plan->r;   // the natural runs are still read by the emitting pass
    if (idx != kMrEnd || tot == 0 || tot > rmax) {
      atomicOr(&plan->error, kErrMinRun);
      tot = tot == 0 ? 1 : (tot > rmax ? rmax : tot);
    }
    plan->r = tot;
    out_rs[tot] = N;
  }
}

// One wave per group: the entry and first output run of every chunk.
__global__ __launch_bounds__(64) void k_mr_assign(const uint8_t *__restrict__ nxt,
                                                  const uint16_t *__restrict__ cnt, uint64_t nch,
                                                  uint64_t ng, const uint8_t *__restrict__ gentry,
                                                  const uint32_t *__restrict__ goff,
                                                  uint8_t *__restrict__ centry,
                                                  uint32_t *__restrict__ coff) {
  const int lane = threadIdx.x;
  for (uint64_t g = blockIdx.x; g < ng; g += gridDim.x) {
    const uint64_t cb = g * kMrGroup, ce = cb + kMrGroup < nch ? cb + kMrGroup : nch;
    uint32_t idx = gentry[g], tot = goff[g];
    for (uint64_t c = cb; c < ce; c += 8) {
      uint32_t a[8], b[8];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        a[u] = kMrBad;
        b[u] = 0;
        if (c + u < ce && lane < kMrCand) {
          a[u] = nxt[(c + u) * kMrCand + lane];
          b[u] = cnt[(c + u) * kMrCand + lane];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int sel = idx < (uint32_t)kMrCand ? (int)idx : 0;
        const uint32_t na = (uint32_t)__shfl((int)a[u], sel), nb = (uint32_t)__shfl((int)b[u], sel);
        if (c + u < ce) {
          if (lane == 0) {
            centry[c + u] = (uint8_t)idx;
            coff[c + u] = tot;
          }
          if (idx < (uint32_t)kMrCand) {
            tot += nb;
            idx = na;
          }
        }
      }
    }
  }
}

// Per chunk: re-walks the chain from the chunk's entry and writes the run
// starts it meets, with the flag of a run that is a strictly decreasing
// natural run left whole (placement reverses those).
__global__ __launch_bounds__(kMrThreads) void k_mr_emit(
    const uint64_t *__restrict__ rs, const uint8_t *__restrict__ desc, Plan *plan, uint32_t N,
    uint32_t m, uint64_t nch, const uint32_t *__restrict__ first,
    const uint8_t *__restrict__ centry, const uint32_t *__restrict__ coff, uint64_t rmax,
    uint64_t *__restrict__ out_rs, uint8_t *__restrict__ out_desc) {
  __shared__ MrSmem sm;
  const int t = threadIdx.x;
  const uint64_t r = plan->r_nat;
  for (uint64_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const uint32_t ent = centry[c];
    if (ent >= (uint32_t)kMrCand) continue;   // the chain does not pass through this chunk
    const uint32_t c0 = (uint32_t)(c * kMrChunk);
    const uint32_t c1 = N - c0 > (uint32_t)kMrChunk ? c0 + kMrChunk : N;
    const uint64_t ia = c > 0 ? first[c] - 1 : 0, ib = first[c + 1];
    const int nrun = mr_stage(rs, desc, r, ia, ib, N, m, sm);
    if (nrun < 0) {
      if (t == 0) atomicOr(&plan->error, kErrMinRun);
      __syncthreads();
      continue;
    }
    if (t == 0) {
      const uint32_t e = ent < m ? c0 + ent : run_end_at(sm, 0, c0 - 1, N);
      int k = 0;
      sm.misc[2] = (int)mr_walk(sm, sm.misc[0], e, c1, N, m, k, sm.rec);
      sm.misc[1] = k;
    }
    __syncthreads();
    const int K = sm.misc[1];
    const uint32_t X = (uint32_t)sm.misc[2];
    const uint64_t o = coff[c];
    for (int k = t; k < K; k += kMrThreads) {
      const uint32_t b = sm.rec[k];
      const uint32_t e = k + 1 < K ? sm.rec[k + 1] : X;
      int lo = 0, hi = nrun - 1;   // staged run holding b
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sm.rs[mid] <= b) lo = mid; else hi = mid - 1;
      }
      const uint32_t ne = run_end_at(sm, lo, b, N);
      const uint8_t nd = b + 1 < sm.rs[lo + 1] ? sm.d[lo] : (b + 1 == N ? 0 : sm.d[lo] ^ 1);
      if (o + k < rmax) {
        out_rs[o + k] = b;
        out_desc[o + k] = (uint8_t)(ne == e && nd);
      }
    }
    __syncthreads();
  }
}

// The stable rank sort of one run of len <= W elements held in registers
// (the unused slots are padded with the largest key, which never precedes a
// real key).  Runs that are monotone (a run left whole is weakly increasing or
// strictly decreasing; an extended one is neither) are left alone.  Each
// element's place is the number of elements that are smaller, or equal and
// earlier: the order a stable insertion sort gives.
template <typename U, typename V, int W, typename Load, typename Store>
__device__ inline void rank_sort_run(uint32_t len, Load ld, Store st) {
  U k[W];
  V v[W];
#pragma unroll
  for (int i = 0; i < W; i++) {
    k[i] = (U)~(U)0;
    v[i] = 0;
    if ((uint32_t)i < len) ld(i, k[i], v[i]);
  }
  bool up = true, dn = true;
#pragma unroll
  for (int i = 0; i + 1 < W; i++) {
    if ((uint32_t)(i + 1) < len) {
      up = up && !(k[i + 1] < k[i]);
      dn = dn && (k[i + 1] < k[i]);
    }
  }
  if (up || dn) return;
#pragma unroll
  for (int i = 0; i < W; i++) {
    if ((uint32_t)i < len) {
      uint32_t rank = 0;
#pragma unroll
      for (int q = 0; q < W; q++) {
        if (q < i) rank += k[q] <= k[i];
        else if (q > i) rank += k[q] < k[i];
      }
      st(rank, k[i], v[i]);
    }
  }
}

// Sorts the extended runs in place, after the tree is built: a run inside a
// small subtree is skipped, since the small-subtree pass sorts the subtree's
// whole span anyway (the stable sort of a span does not depend on the order
// inside its runs).  A workgroup takes kMrSortRuns consecutive runs; when
// their span fits in LDS it is staged there with coalesced loads, each thread
// sorts its own run between LDS and registers, and the span is stored back
// coalesced (positions that carry a co-rank sample refresh it).  A longer
// span (a long natural run among them) is handled run by run straight from
// memory.
template <int KT, int W, typename V>
__global__ __launch_bounds__(kMrSortRuns) void k_mr_sort(typename Key<KT>::U *__restrict__ keys,
                                                         V *__restrict__ vals,
                                                         const uint64_t *__restrict__ rs,
                                                         const uint8_t *__restrict__ leaf_depth,
                                                         const Plan *__restrict__ plan,
                                                         uint32_t m, uint64_t *__restrict__ smp) {
  using U = typename Key<KT>::U;
  constexpr uint64_t SM = kSampleStride - 1;
  constexpr uint32_t kCap = kMrSortRuns * W;
  __shared__ U sk[kCap];
  __shared__ V sv[kCap];
  const int t = threadIdx.x;
  const uint64_t r = plan->r;
  for (uint64_t j0 = (uint64_t)blockIdx.x * kMrSortRuns; j0 < r;
       j0 += (uint64_t)gridDim.x * kMrSortRuns) {
    const uint64_t j1 = j0 + kMrSortRuns < r ? j0 + kMrSortRuns : r;
    const uint64_t S0 = rs[j0], span = rs[j1] - S0;
    const uint64_t j = j0 + t;
    uint64_t s = 0;
    uint32_t len = 0;
    if (j < j1) {
      s = rs[j];
      len = (uint32_t)(rs[j + 1] - s);
    }
    const bool mine = len >= 2 && len <= m && !(leaf_depth[j] & kLeafInSmall);
    if (!__syncthreads_or(mine)) continue;   // uniform: nothing to sort here
    if (span <= kCap) {
      const uint32_t sp = (uint32_t)span;
      for (uint32_t x = t; x < sp; x += kMrSortRuns) {
        sk[x] = Key<KT>::ord(keys[S0 + x]);
        if (vals) sv[x] = vals[S0 + x];
      }
      __syncthreads();
      if (mine) {
        const uint32_t o = (uint32_t)(s - S0);
        rank_sort_run<U, V, W>(
            len,
            [&](int i, U &kk, V &vv) {
              kk = sk[o + i];
              if (vals) vv = sv[o + i];
            },
            [&](uint32_t rank, U kk, V vv) {
              sk[o + rank] = kk;
              if (vals) sv[o + rank] = vv;
            });
      }
      __syncthreads();
      for (uint32_t x = t; x < sp; x += kMrSortRuns) {
        const U kk = sk[x];
        keys[S0 + x] = Key<KT>::unord(kk);
        if (vals) vals[S0 + x] = sv[x];
        if (((S0 + x) & SM) == 0) smp[(S0 + x) / kSampleStride] = (uint64_t)kk;
      }
      __syncthreads();
    } else if (mine) {
      rank_sort_run<U, V, W>(
          len,
          [&](int i, U &kk, V &vv) {
            kk = Key<KT>::ord(keys[s + i]);
            if (vals) vv = vals[s + i];
          },
          [&](uint32_t rank, U kk, V vv) {
            const uint64_t dst = s + rank;
            keys[dst] = Key<KT>::unord(kk);
            if (vals) vals[dst] = vv;
            if ((dst & SM) == 0) smp[dst / kSampleStride] = (uint64_t)kk;
          });
    }
  }
}

template <int W, typename V>
void launch_mr_sort_v(int kt, void *keys, V *vals, const Work &w, uint32_t m, unsigned gs,
                      hipStream_t s) {
  switch (kt) {
    case 0: hipLaunchKernelGGL((k_mr_sort<0, W, V>), dim3(gs), dim3(kMrSortRuns), 0, s, (uint32_t *)keys, vals, w.run_start, w.leaf_depth, w.plan, m, w.samples); break;
    case 1: hipLaunchKernelGGL((k_mr_sort<1, W, V>), dim3(gs), dim3(kMrSortRuns), 0, s, (uint64_t *)keys, vals, w.run_start, w.leaf_depth, w.plan, m, w.samples); break;
    default: hipLaunchKernelGGL((k_mr_sort<2, W, V>), dim3(gs), dim3(kMrSortRuns), 0, s, (uint32_t *)keys, vals, w.run_start, w.leaf_depth, w.plan, m, w.samples); break;
  }
}

template <int W>
hipError_t launch_mr_sort(int kt, void *keys, uint32_t *vals, const Work &w, uint32_t m,
                          unsigned gs, hipStream_t s) {
  if (vals && w.pay8) launch_mr_sort_v<W, uint64_t>(kt, keys, reinterpret_cast<uint64_t *>(vals), w, m, gs, s);
  else launch_mr_sort_v<W, uint32_t>(kt, keys, vals, w, m, gs, s);
  return hipGetLastError();
}

unsigned grid_for(uint64_t items, uint64_t per, unsigned cap) {
  const uint64_t g = (items + per - 1) / per;
  return (unsigned)(g < 1 ? 1 : (g < cap ? g : cap));
}

}  // namespace

hipError_t launch_minrun(int kt, void *keys, uint32_t *vals, const Work &w, hipStream_t s) {
  const uint64_t N = w.N;
  const uint32_t m = (uint32_t)w.min_run;
  const uint64_t nch = (N + kMrChunk - 1) / kMrChunk;
  const uint64_t ng = (nch + kMrGroup - 1) / kMrGroup;
  hipLaunchKernelGGL(k_mr_first, dim3(grid_for(nch + 1, 256, 4096)), dim3(256), 0, s,
                     w.nat_start, w.plan, nch, w.mr_first);
  hipLaunchKernelGGL(k_mr_chunk, dim3(grid_for(nch, 1, 8192)), dim3(kMrThreads), 0, s,
                     w.nat_start, w.nat_desc, w.plan, (uint32_t)N, m, nch, w.mr_first, w.mr_nxt,
                     w.mr_cnt);
  hipLaunchKernelGGL(k_mr_group, dim3(grid_for(ng, 1, 8192)), dim3(64), 0, s, w.mr_nxt, w.mr_cnt,
                     nch, ng, m, w.mr_gnxt, w.mr_gcnt);
  hipLaunchKernelGGL(k_mr_top, dim3(1), dim3(64), 0, s, w.mr_gnxt, w.mr_gcnt, ng, N, w.rmax,
                     w.mr_gentry, w.mr_goff, w.run_start, w.plan);
  hipLaunchKernelGGL(k_mr_assign, dim3(grid_for(ng, 1, 8192)), dim3(64), 0, s, w.mr_nxt,
                     w.mr_cnt, nch, ng, w.mr_gentry, w.mr_goff, w.mr_centry, w.mr_coff);
  hipLaunchKernelGGL(k_mr_emit, dim3(grid_for(nch, 1, 8192)), dim3(kMrThreads), 0, s,
                     w.nat_start, w.nat_desc, w.plan, (uint32_t)N, m, nch, w.mr_first, w.mr_centry,
                     w.mr_coff, w.rmax, w.run_start, w.run_desc);
  return hipGetLastError();
}

hipError_t launch_minrun_sort(int kt, void *keys, uint32_t *vals, const Work &w, hipStream_t s) {
  const uint32_t m = (uint32_t)w.min_run;
  const unsigned gs = grid_for(w.N / 2 + 2, kMrSortRuns, 16384);
  if (m <= 8) return launch_mr_sort<8>(kt, keys, vals, w, m, gs, s);
  if (m <= 16) return launch_mr_sort<16>(kt, keys, vals, w, m, gs, s);
  if (m <= 24) return launch_mr_sort<24>(kt, keys, vals, w, m, gs, s);
  return launch_mr_sort<32>(kt, keys, vals, w, m, gs, s);
}

}  // namespace mps
