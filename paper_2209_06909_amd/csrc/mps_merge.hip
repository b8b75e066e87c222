// mps_merge.hip -- leaf placement and the per-level k-way merges.
//
// Buffers alternate by depth: a node at depth d writes buffer d mod 2
// (buffer 0 is the caller's array, buffer 1 the workspace copy), so it always
// reads its children from the other buffer.  Levels run deepest first; a
// node's children (depth d+1) are complete before it runs and nothing else
// inside its span is still needed, so no level needs a third buffer.
//
// Leaves start in buffer 0.  A leaf at odd depth is copied to buffer 1; a
// strictly decreasing run is reversed on the way (paper, Section 2: such runs
// hold no equal keys, so reversing keeps the sort stable).
//
// The level merges themselves are in mps_merge.h.
#include "mps_merge.h"

namespace mps {

// ---------------------------------------------------------------- placement
constexpr int kPlaceThreads = 256;
constexpr int kPlaceE = (int)(kPlaceBlock / kPlaceThreads);   // positions per thread
static_assert(kPlaceE * kPlaceThreads == (int)kPlaceBlock && kPlaceE % 2 == 0, "placement block");

// Placement flags of a run: bit 0 odd depth, bit 1 strictly descending.  A run
// whose parent is a small node is left to the small-subtree pass (flags 0).
__device__ inline uint8_t place_flags(uint8_t leaf_depth, uint8_t desc) {
  if (leaf_depth & kLeafInSmall) return 0;
  return (uint8_t)((leaf_depth & 1) | (desc ? 2 : 0));
}

__device__ inline uint64_t run_of(const uint64_t *rs, uint64_t lo, uint64_t hi, uint64_t e) {
  // last j in [lo, hi] with rs[j] <= e
  while (hi > lo) {
    uint64_t mid = (lo + hi + 1) >> 1;
    if (rs[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Positions of a block that is not one ascending run: each finds its run in
// the staged table and acts on it, in two halves of kPlaceE/2 positions per
// thread.
template <int KT, typename V>
__device__ inline void place_general(typename Key<KT>::U *__restrict__ keys,
                                     V *__restrict__ vals,
                                     typename Key<KT>::U *__restrict__ akeys,
                                     V *__restrict__ avals, uint64_t *__restrict__ smp,
                                     const uint64_t *sRs, const uint8_t *sFl, int nr, uint64_t bs,
                                     uint64_t be, int t) {
  using U = typename Key<KT>::U;
  constexpr uint64_t SM = kSampleStride - 1;
  constexpr int T = kPlaceThreads;
  constexpr int HE = kPlaceE / 2;
#pragma unroll 1
  for (int h = 0; h < 2; h++) {
    uint64_t dst[HE];
    int act[HE];
#pragma unroll
    for (int i = 0; i < HE; i++) {
      const uint64_t e = bs + t + (uint64_t)(h * HE + i) * T;
      act[i] = 0;
      dst[i] = e;
      if (e < be) {
        int lo = 0, hi = nr - 1;   // last staged run with start <= e
        while (hi > lo) {
          int mid = (lo + hi + 1) >> 1;
          if (sRs[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const uint64_t s = sRs[lo], f = sRs[lo + 1];
        const int fl = sFl[lo];
        if (fl & 1) {
          act[i] = 1;
          dst[i] = (fl & 2) ? s + f - 1 - e : e;
        } else if ((fl & 2) && e - s < (f - s) / 2) {
          act[i] = 2;
          dst[i] = s + f - 1 - e;
        }
      }
    }
    U ka[HE], kb[HE];
    V va[HE], vb[HE];
#pragma unroll
    for (int i = 0; i < HE; i++) {
      const uint64_t e = bs + t + (uint64_t)(h * HE + i) * T;
      if (act[i]) {
        ka[i] = keys[e];
        if (vals) va[i] = vals[e];
      }
      if (act[i] == 2) {
        kb[i] = keys[dst[i]];
        if (vals) vb[i] = vals[dst[i]];
      }
    }
#pragma unroll
    for (int i = 0; i < HE; i++) {
      const uint64_t e = bs + t + (uint64_t)(h * HE + i) * T;
      // a key that lands on a new position refreshes that position's co-rank sample
      if (act[i] == 1) {
        akeys[dst[i]] = ka[i];
        if (vals) avals[dst[i]] = va[i];
        if (dst[i] != e && (dst[i] & SM) == 0) smp[dst[i] / kSampleStride] = Key<KT>::ord(ka[i]);
      } else if (act[i] == 2) {
        keys[e] = kb[i];
        keys[dst[i]] = ka[i];
        if (vals) {
          vals[e] = vb[i];
          vals[dst[i]] = va[i];
        }
        if ((e & SM) == 0) smp[e / kSampleStride] = Key<KT>::ord(kb[i]);
        if ((dst[i] & SM) == 0) smp[dst[i] / kSampleStride] = Key<KT>::ord(ka[i]);
      }
    }
  }
}

// Blocks that lie inside one run get that run's flag (the leaf-depth pass
// flagged only the first and last block of every run that moves).  One thread
// per block, binary search in the run table.
__global__ __launch_bounds__(256) void k_place_blocks(const uint64_t *__restrict__ rs,
                                                      const uint8_t *__restrict__ desc,
                                                      const uint8_t *__restrict__ leaf_depth,
                                                      const Plan *__restrict__ plan, uint64_t N,
                                                      uint32_t *__restrict__ pflag) {
  const uint64_t r = plan->r;
  const uint64_t nblk = (N + kPlaceBlock - 1) / kPlaceBlock;
  if (r == 0) return;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nblk;
       b += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t bs = b * kPlaceBlock, be = bs + kPlaceBlock < N ? bs + kPlaceBlock : N;
    const uint64_t j = run_of(rs, 0, r - 1, bs);
    if (rs[j + 1] >= be) pflag[b] = place_flags(leaf_depth[j], desc[j]) != 0 ? 1u : 0u;
  }
}

// Each workgroup takes a contiguous range of blocks of kPlaceBlock positions.
// For every block the threads stage, in one round of loads, the starts and
// flags (bit 0 odd depth, bit 1 descending) of the kPlaceThreads runs from the
// one holding the block's first position; barrier counts over that table give
// the runs overlapping the block and the run holding the next block's first
// position.  A block inside one ascending run is copied to the other buffer
// (odd depth) or left alone (even depth).  Otherwise every position finds its
// run and what to do with it: odd-depth leaves are copied to the other buffer
// (reversed if descending); even-depth descending runs are reversed in place
// by the threads of their first half, each swapping with its mirror position.
// A block overlapping more than kPlaceThreads runs stages all of them (at most
// one per position) in a second round.
template <int KT, typename V>
__global__ __launch_bounds__(kPlaceThreads) void k_place(typename Key<KT>::U *__restrict__ keys,
                                                         V *__restrict__ vals,
                                                         typename Key<KT>::U *__restrict__ akeys,
                                                         V *__restrict__ avals, uint64_t N,
                                                         const uint64_t *__restrict__ rs,
                                                         const uint8_t *__restrict__ desc,
                                                         const uint8_t *__restrict__ leaf_depth,
                                                         const uint32_t *__restrict__ pflag,
                                                         const Plan *__restrict__ plan,
                                                         uint64_t *__restrict__ smp) {
  using U = typename Key<KT>::U;
  constexpr uint64_t SM = kSampleStride - 1;
  constexpr int T = kPlaceThreads;
  // starts and flags of the runs overlapping a block: at most kPlaceBlock
  // (the run holding the first position, then at most one new run per position)
  __shared__ uint64_t sRs[kPlaceBlock + 1];
  __shared__ uint8_t sFl[kPlaceBlock];
  __shared__ uint64_t sJ;
  const uint64_t r = plan->r;
  const int t = threadIdx.x;
  const uint64_t nblk = (N + kPlaceBlock - 1) / kPlaceBlock;
  const uint64_t per = (nblk + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * per;
  const uint64_t b1 = b0 + per < nblk ? b0 + per : nblk;
  if (b0 >= b1 || r == 0) return;   // uniform in the workgroup
  uint64_t jc = 0;      // run holding the current block's first position
  bool known = false;   // jc is current
  for (uint64_t b = b0; b < b1; b++) {
    const uint64_t bs = b * kPlaceBlock, be = bs + kPlaceBlock < N ? bs + kPlaceBlock : N;
    // blocks in which no run moves (flagged by the leaf-depth pass) are skipped
    if (pflag[b] == 0u) {   // uniform
      known = false;
      continue;
    }
    if (!known) {
      if (t == 0) sJ = run_of(rs, 0, r - 1, bs);
      __syncthreads();
      jc = sJ;
      known = true;
      __syncthreads();   // sJ is read before it is written again
    }
    {
      const uint64_t i = jc + (uint64_t)t;
      sRs[t] = i <= r ? rs[i] : ~0ull;   // rs[r] = N
      sFl[t] = i < r ? place_flags(leaf_depth[i], desc[i]) : (uint8_t)0;
      if (t == 0) sRs[T] = jc + T <= r ? rs[jc + T] : ~0ull;
    }
    // runs overlapping [bs, be): jc .. jc+nr-1 (sRs[0] <= bs, so nr >= 1)
    // the values that choose the path are uniform; readfirstlane lets the
    // compiler branch on them as such
    int nr = __builtin_amdgcn_readfirstlane(__syncthreads_count(sRs[t] < be));
    if (__builtin_amdgcn_readfirstlane(nr == T && sRs[T] < be ? 1 : 0)) {
      // more than T runs overlap the block: stage the rest of them too
      for (int x = T + 1 + t; x <= (int)kPlaceBlock; x += T) {
        const uint64_t i = jc + (uint64_t)x;
        sRs[x] = i <= r ? rs[i] : ~0ull;
        if (x < (int)kPlaceBlock)
          sFl[x] = i < r ? place_flags(leaf_depth[i], desc[i]) : (uint8_t)0;
      }
      if (t == 0) sFl[T] = jc + T < r ? place_flags(leaf_depth[jc + T], desc[jc + T]) : (uint8_t)0;
      __syncthreads();
      int lo = T, hi = (int)kPlaceBlock;   // first staged start >= be (sRs[kPlaceBlock] >= be)
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sRs[mid] < be) lo = mid + 1; else hi = mid;
      }
      nr = __builtin_amdgcn_readfirstlane(lo);
    }
    const uint64_t jn = jc + (uint64_t)(nr - 1) + (sRs[nr] == be ? 1u : 0u);
    const int fl0 = __builtin_amdgcn_readfirstlane((int)sFl[0]);
    if (nr == 1 && fl0 == 1) {
      // one odd-depth ascending run: straight copy to the other buffer
      const int lim = (int)(be - bs);
      const U *ks = keys + bs;
      U *kd = akeys + bs;
      U kv[kPlaceE];
      V vv[kPlaceE];
#pragma unroll
      for (int i = 0; i < kPlaceE; i++) {
        const int o = t + i * T;
        if (o < lim) {
          kv[i] = ks[o];
          if (vals) vv[i] = vals[bs + o];
        }
      }
#pragma unroll
      for (int i = 0; i < kPlaceE; i++) {
        const int o = t + i * T;
        if (o < lim) {
          kd[o] = kv[i];
          if (vals) avals[bs + o] = vv[i];
        }
      }
    } else if (!(nr == 1 && fl0 == 0)) {
      // blocks whose runs all stay where they are (even depth, ascending, or
      // inside a small subtree) have nothing to move
      bool mine = false;
      for (int x = t; x < nr; x += T) mine = mine || sFl[x] != 0;
      if (__syncthreads_or(mine)) place_general<KT, V>(keys, vals, akeys, avals, smp, sRs, sFl, nr, bs, be, t);
    }
    jc = jn;
    __syncthreads();   // the run table is restaged for the next block
  }
}

// ---------------------------------------------------------------- host side
template <int KT, typename V>
static void launch_place_v(void *keys, void *vals, const Work &w, unsigned g, hipStream_t s) {
  using U = typename Key<KT>::U;
  hipLaunchKernelGGL((k_place<KT, V>), dim3(g), dim3(kPlaceThreads), 0, s, (U *)keys, (V *)vals,
                     (U *)w.alt_keys, (V *)w.alt_vals, w.N, w.run_start, w.run_desc, w.leaf_depth,
                     w.pflag, w.plan, w.samples);
}

template <int KT>
static void launch_place_kt(void *keys, uint32_t *vals, const Work &w, unsigned g, hipStream_t s) {
  if (vals && w.pay8) launch_place_v<KT, uint64_t>(keys, vals, w, g, s);
  else launch_place_v<KT, uint32_t>(keys, vals, w, g, s);
}

hipError_t launch_place(int kt, void *keys, uint32_t *vals, const Work &w, hipStream_t s) {
  uint64_t nblk = (w.N + kPlaceBlock - 1) / kPlaceBlock;
  unsigned g = (unsigned)(nblk < 8192 ? nblk : 8192);
  if (g == 0) return hipSuccess;
  const unsigned gb = (unsigned)((nblk + 255) / 256 < 4096 ? (nblk + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_place_blocks, dim3(gb), dim3(256), 0, s, w.run_start, w.run_desc,
                     w.leaf_depth, w.plan, w.N, w.pflag);
  if (kt == 1) launch_place_kt<1>(keys, vals, w, g, s);
  else if (kt == 2) launch_place_kt<2>(keys, vals, w, g, s);
  else launch_place_kt<0>(keys, vals, w, g, s);
  return hipGetLastError();
}

// Co-rank and descriptor launches of one level (tile size is a run-time value).
template <int KT, int K>
static void launch_cuts_t(const LevelArgs &a, const Work &w, const uint32_t *tj,
                          const uint64_t *tile_base, int level, hipStream_t s) {
  using U = typename Key<KT>::U;
  const unsigned gc = 512;
  // the co-rank runs one group of K lanes per tile boundary
  const uint64_t cgroups = (w.N / (uint64_t)w.tile + 2) * K;
  const unsigned gk = (unsigned)((cgroups + 255) / 256 < 16384 ? (cgroups + 255) / 256 : 16384);
  hipLaunchKernelGGL((k_corank<KT, K>), dim3(gk), dim3(256), 0, s, (const U *)a.in_keys,
                     w.run_start, w.Ls, w.Rs, w.nd_mem, w.nd_arity, w.lvl_list, w.lvl_np, tj,
                     tile_base, w.plan, level, w.tile, w.corank, (const uint64_t *)w.samples);
  using Tab = TileTabFor<U, K>;
  Tab *desc = reinterpret_cast<Tab *>(w.tile_desc);
  hipLaunchKernelGGL((k_tile_desc<K, Tab::kPieces>), dim3(gc), dim3(256), 0, s, w.run_start, w.Ls, w.Rs,
                     w.nd_mem, w.nd_arity, w.lvl_list, w.lvl_np, tj, tile_base, w.plan, level,
                     w.tile, w.corank, desc, w.gen_list);
}

static hipError_t launch_cuts(int kt, const LevelArgs &a, const Work &w, const uint32_t *tj,
                              const uint64_t *tile_base, int level, hipStream_t s) {
  switch (w.k * 4 + kt) {
    case 2 * 4 + 0: launch_cuts_t<0, 2>(a, w, tj, tile_base, level, s); break;
    case 2 * 4 + 1: launch_cuts_t<1, 2>(a, w, tj, tile_base, level, s); break;
    case 2 * 4 + 2: launch_cuts_t<2, 2>(a, w, tj, tile_base, level, s); break;
    case 4 * 4 + 0: launch_cuts_t<0, 4>(a, w, tj, tile_base, level, s); break;
    case 4 * 4 + 1: launch_cuts_t<1, 4>(a, w, tj, tile_base, level, s); break;
    case 4 * 4 + 2: launch_cuts_t<2, 4>(a, w, tj, tile_base, level, s); break;
    case 8 * 4 + 0: launch_cuts_t<0, 8>(a, w, tj, tile_base, level, s); break;
    case 8 * 4 + 1: launch_cuts_t<1, 8>(a, w, tj, tile_base, level, s); break;
    case 8 * 4 + 2: launch_cuts_t<2, 8>(a, w, tj, tile_base, level, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_merges(int kt, const LevelArgs &a, const Work &w, const uint32_t *tj,
                                const uint64_t *tile_base, int level, hipStream_t s) {
  if (w.tile == 1024 && w.threads == 256) return launch_merges_1024x256(kt, a, w, tj, tile_base, level, s);
  if (w.tile == 2048 && w.threads == 256) return launch_merges_2048x256(kt, a, w, tj, tile_base, level, s);
  if (w.tile == 2048 && w.threads == 512) return launch_merges_2048x512(kt, a, w, tj, tile_base, level, s);
  if (w.tile == 4096 && w.threads == 512) return launch_merges_4096x512(kt, a, w, tj, tile_base, level, s);
  if (w.tile == 4096 && w.threads == 1024) return launch_merges_4096x1024(kt, a, w, tj, tile_base, level, s);
  return hipErrorInvalidValue;
}

hipError_t launch_level_timed(int kt, const LevelArgs &a, const Work &w, const uint32_t *tj,
                              const uint64_t *tile_base, int level, hipStream_t s,
                              hipEvent_t e0, hipEvent_t e1, hipEvent_t e2) {
  if (e0) (void)hipEventRecord(e0, s);
  hipError_t e = launch_cuts(kt, a, w, tj, tile_base, level, s);
  if (e != hipSuccess) return e;
  if (e1) (void)hipEventRecord(e1, s);
  e = launch_merges(kt, a, w, tj, tile_base, level, s);
  if (e != hipSuccess) return e;
  if (e2) (void)hipEventRecord(e2, s);
  return hipSuccess;
}

hipError_t launch_level(int kt, const LevelArgs &a, const Work &w, const uint32_t *tj,
                        const uint64_t *tile_base, int level, hipStream_t s) {
  return launch_level_timed(kt, a, w, tj, tile_base, level, s, nullptr, nullptr, nullptr);
}

}  // namespace mps
