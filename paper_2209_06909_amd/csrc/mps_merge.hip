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
constexpr int kPlaceE = 8;                                   // positions per thread
constexpr uint64_t kPlaceBlock = (uint64_t)kPlaceThreads * kPlaceE;
constexpr int kPlaceRuns = 512;                              // run table entries staged in LDS

__device__ inline uint64_t run_of(const uint64_t *rs, uint64_t lo, uint64_t hi, uint64_t e) {
  // last j in [lo, hi] with rs[j] <= e
  while (hi > lo) {
    uint64_t mid = (lo + hi + 1) >> 1;
    if (rs[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Same, for an answer expected close to lo (rs[lo] <= e): exponential steps
// from lo, then a binary search inside the last step.
__device__ inline uint64_t run_near(const uint64_t *rs, uint64_t lo, uint64_t hi, uint64_t e) {
  uint64_t step = 1;
  while (lo + step <= hi && rs[lo + step] <= e) {
    lo += step;
    step <<= 1;
  }
  return run_of(rs, lo, lo + step - 1 < hi ? lo + step - 1 : hi, e);
}

// Each workgroup takes a contiguous range of blocks of kPlaceBlock positions,
// so the runs of one block are found by a short search onward from the
// previous block's.  The runs overlapping it
// are staged in LDS (start and a flag byte: bit 0 odd depth, bit 1 descending)
// unless there are too many; then every position finds its run and what to do
// with it, all loads are issued, then all stores.  Odd-depth leaves are copied
// to the other buffer (reversed if descending); even-depth descending runs are
// reversed in place by the threads of their first half, each swapping with
// its mirror position.
template <int KT>
__global__ __launch_bounds__(kPlaceThreads) void k_place(typename Key<KT>::U *__restrict__ keys,
                                                         uint32_t *__restrict__ vals,
                                                         typename Key<KT>::U *__restrict__ akeys,
                                                         uint32_t *__restrict__ avals, uint64_t N,
                                                         const uint64_t *__restrict__ rs,
                                                         const uint8_t *__restrict__ desc,
                                                         const uint8_t *__restrict__ leaf_depth,
                                                         const Plan *__restrict__ plan,
                                                         uint64_t *__restrict__ smp) {
  using U = typename Key<KT>::U;
  constexpr uint64_t SM = kSampleStride - 1;
  __shared__ uint64_t sRs[kPlaceRuns + 1];
  __shared__ uint8_t sFl[kPlaceRuns];
  __shared__ uint64_t sJ[2];
  const uint64_t r = plan->r;
  const int t = threadIdx.x;
  const uint64_t nblk = (N + kPlaceBlock - 1) / kPlaceBlock;
  const uint64_t per = (nblk + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * per;
  const uint64_t b1 = b0 + per < nblk ? b0 + per : nblk;
  uint64_t jc = 0;   // thread 0: run containing the current block's first position
  if (t == 0 && b0 < b1) jc = run_of(rs, 0, r - 1, b0 * kPlaceBlock);
  for (uint64_t b = b0; b < b1; b++) {
    const uint64_t bs = b * kPlaceBlock, be = bs + kPlaceBlock < N ? bs + kPlaceBlock : N;
    if (t == 0) {
      const uint64_t j1 = run_near(rs, jc, r - 1, be - 1);
      sJ[0] = jc;
      sJ[1] = j1;
      if (be < N) jc = run_near(rs, j1, r - 1, be);
    }
    __syncthreads();
    const uint64_t j0 = sJ[0], j1 = sJ[1];
    const int nr = (int)(j1 - j0 + 1);
    const bool staged = nr <= kPlaceRuns;
    int any = 0;
    if (staged) {
      for (int i = t; i <= nr; i += kPlaceThreads) sRs[i] = rs[j0 + i];
      for (int i = t; i < nr; i += kPlaceThreads) {
        uint8_t f = (uint8_t)((leaf_depth[j0 + i] & 1) | (desc[j0 + i] ? 2 : 0));
        sFl[i] = f;
        any |= f;
      }
    }
    any = __syncthreads_or(any) || !staged;
    if (any) {
      uint64_t dst[kPlaceE];
      int act[kPlaceE];
#pragma unroll
      for (int i = 0; i < kPlaceE; i++) {
        const uint64_t e = bs + t + (uint64_t)i * kPlaceThreads;
        act[i] = 0;
        dst[i] = e;
        if (e < be) {
          uint64_t s, f;
          int fl;
          if (staged) {
            int lo = 0, hi = nr - 1;   // last run with start <= e
            while (hi > lo) {
              int mid = (lo + hi + 1) >> 1;
              if (sRs[mid] <= e) lo = mid; else hi = mid - 1;
            }
            s = sRs[lo];
            f = sRs[lo + 1];
            fl = sFl[lo];
          } else {
            uint64_t j = run_of(rs, j0, j1, e);
            s = rs[j];
            f = rs[j + 1];
            fl = (leaf_depth[j] & 1) | (desc[j] ? 2 : 0);
          }
          if (fl & 1) {
            act[i] = 1;
            dst[i] = (fl & 2) ? s + f - 1 - e : e;
          } else if ((fl & 2) && e - s < (f - s) / 2) {
            act[i] = 2;
            dst[i] = s + f - 1 - e;
          }
        }
      }
      U ka[kPlaceE], kb[kPlaceE];
      uint32_t va[kPlaceE], vb[kPlaceE];
#pragma unroll
      for (int i = 0; i < kPlaceE; i++) {
        const uint64_t e = bs + t + (uint64_t)i * kPlaceThreads;
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
      for (int i = 0; i < kPlaceE; i++) {
        const uint64_t e = bs + t + (uint64_t)i * kPlaceThreads;
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
    __syncthreads();
  }
}

// ---------------------------------------------------------------- host side
hipError_t launch_place(int kt, void *keys, uint32_t *vals, const Work &w, hipStream_t s) {
  uint64_t nblk = (w.N + kPlaceBlock - 1) / kPlaceBlock;
  unsigned g = (unsigned)(nblk < 8192 ? nblk : 8192);
  if (g == 0) return hipSuccess;
  if (kt == 1)
    hipLaunchKernelGGL(k_place<1>, dim3(g), dim3(kPlaceThreads), 0, s, (uint64_t *)keys, vals,
                       (uint64_t *)w.alt_keys, w.alt_vals, w.N, w.run_start, w.run_desc,
                       w.leaf_depth, w.plan, w.samples);
  else if (kt == 2)
    hipLaunchKernelGGL(k_place<2>, dim3(g), dim3(kPlaceThreads), 0, s, (uint32_t *)keys, vals,
                       (uint32_t *)w.alt_keys, w.alt_vals, w.N, w.run_start, w.run_desc,
                       w.leaf_depth, w.plan, w.samples);
  else
    hipLaunchKernelGGL(k_place<0>, dim3(g), dim3(kPlaceThreads), 0, s, (uint32_t *)keys, vals,
                       (uint32_t *)w.alt_keys, w.alt_vals, w.N, w.run_start, w.run_desc,
                       w.leaf_depth, w.plan, w.samples);
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
  TileDesc<K> *desc = reinterpret_cast<TileDesc<K> *>(w.tile_desc);
  hipLaunchKernelGGL((k_tile_desc<K>), dim3(gc), dim3(256), 0, s, w.run_start, w.Ls, w.Rs,
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
