// mps_tree.hip -- node powers and the merge tree, built without a stack.
//
// Powers (paper, Definition 3.1): with A = s_{i-1}+s_i and B = s_i+s_{i+1}
// the run midpoints are a = A/2n and b = B/2n.  The 2-way power is the
// index of the first binary digit in which a and b differ; with 32-bit
// fixed point x = floor(A*2^31/n), y = floor(B*2^31/n) (exact prefixes of
// the binary expansions, and x != y because b - a >= 1/n) it is
// clz32(x ^ y) + 1.  For k = 2^q the k-way power groups q binary digits per
// base-k digit: P_k = floor((P_2 - 1)/q) + 1 (Section 3.1, the "squish" of
// adjacent levels).
//
// Tree (Algorithm 1): a node is a maximal group of equal-power boundaries
// with only larger powers between them, delimited by the nearest strictly
// smaller powers on both sides.  Those nearest-smaller positions come from a
// ballot-based all-nearest-smaller-values pass (powers are small integers).
// The parent of a node is the node owning the larger of its two delimiting
// powers; depths follow by pointer jumping.  Segment edges (and the array
// ends) carry power 0, below every real power, so nothing merges across them.
#include "mps_internal.h"

namespace mps {

constexpr int kTreeThreads = 1024;   // boundaries per block
constexpr int kTreeWaves = kTreeThreads / kWave;

// ---------------------------------------------------------------- powers
// floor(a * 2^31 / n) for a < 2n, n <= 2^31 (so the quotient is < 2^32 and
// q * n < 2^63): a double estimate (relative error about 2^-52, hence off by
// at most one), corrected with exact integer products.
__device__ inline uint32_t quot31(uint64_t a, uint64_t n, double inv) {
  const uint64_t num = a << 31;
  uint64_t q = (uint64_t)((double)a * inv);
  if (q * n > num) q--;
  else if ((q + 1) * n <= num) q++;
  return (uint32_t)q;
}

// Workgroup-wide fold of one value per thread (256 threads) into a plan
// field with one atomic per workgroup.  Many atomics on one address are
// serviced one after another, so a per-wave atomic at the end of a short
// kernel costs more than the kernel's own work.  A maximum is only sent when
// it would raise the field.
template <typename T>
__device__ inline void block_max_into(T v, T *dst) {
  __shared__ T part[4];
  for (int o = 32; o > 0; o >>= 1) {
    const T y = __shfl_down(v, o);
    v = y > v ? y : v;
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    T m = part[0];
    for (int w = 1; w < 4; w++) m = part[w] > m ? part[w] : m;
    if (m > __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(dst, m);
  }
}

__device__ inline void block_add_into(uint64_t v, uint64_t *dst) {
  __shared__ uint64_t part[4];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t m = part[0] + part[1] + part[2] + part[3];
    if (m) atomicAdd((unsigned long long *)dst, (unsigned long long)m);
  }
}

__global__ __launch_bounds__(256) void k_powers(const uint64_t *__restrict__ rs,
                                                const uint64_t *__restrict__ off, uint64_t m,
                                                Plan *__restrict__ plan, int logk,
                                                uint8_t *__restrict__ P) {
  const uint64_t r = plan->r;
  uint32_t pmax = 0;
  // the segment of the last boundary and its length's inverse (a division
  // per segment change, not per boundary)
  uint32_t sgc = 0xFFFFFFFFu;
  uint64_t base = 0, n = 1;
  double inv = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= r;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint8_t p = 0;
    if (i > 0 && i < r) {
      const uint64_t s0 = rs[i - 1], s = rs[i], s2 = rs[i + 1];
      const uint32_t sg = seg_of(off, m, s);
      if (sg != sgc) {
        sgc = sg;
        base = off[sg];
        n = off[sg + 1] - base;
        inv = 2147483648.0 / (double)n;
      }
      if (s != base) {
        uint64_t A = (s0 - base) + (s - base);
        uint64_t B = (s - base) + (s2 - base);
        uint32_t x = quot31(A, n, inv);
        uint32_t y = quot31(B, n, inv);
        uint32_t p2 = (uint32_t)__clz(x ^ y) + 1;
        uint32_t pk = (p2 - 1) / (uint32_t)logk + 1;
        if (x == y || pk >= (uint32_t)kVMax) {  // impossible: b - a >= 1/n, n <= 2^31
          atomicOr(&plan->error, 8u);
          pk = kVMax - 1;
        }
        p = (uint8_t)pk;
      }
    }
    P[i] = p;
    pmax = p > pmax ? p : pmax;
  }
  block_max_into<uint32_t>(pmax, &plan->pmax);
}

// ---------------------------------------------------------------- ANSV
// Per block of 1024 boundaries: for every value v in [1, kVMax], the last
// (stored +1; 0 = none) and first (kNone32 = none) boundary with power < v.
// Only v <= vmax = 1 + the largest power present are ever asked for.
__device__ inline void wave_masks(const uint8_t *__restrict__ P, uint64_t r, uint64_t i,
                                  uint64_t *masks /* [kVMax] per wave, LDS */, int lane, int vmax) {
  uint32_t p = i <= r ? P[i] : 255u;
  for (int v = 1; v <= vmax; v++) {
    uint64_t mk = ballot64(p < (uint32_t)v);
    if (lane == 0) masks[v - 1] = mk;
  }
}

// Thread t = v * kTreeWaves + ww (v < vmax) looks at wave ww's mask for value
// v + 1: the last boundary + 1 (0 = none) and the first boundary (kNone32 =
// none) with power <= v.  The kTreeWaves threads of one value are consecutive
// lanes, so their scans over the waves are shuffles within groups of
// kTreeWaves lanes.
__device__ inline void wave_ends(const uint64_t (*sM)[kVMax], uint64_t b, int v, int ww,
                                 uint32_t &last1, uint32_t &first) {
  const uint64_t mk = sM[ww][v];
  const uint64_t base = b * kTreeThreads + (uint64_t)ww * kWave;
  last1 = mk ? (uint32_t)(base + 63 - __clzll(mk)) + 1 : 0u;
  first = mk ? (uint32_t)(base + __ffsll((long long)mk) - 1) : kNone32;
}

__global__ __launch_bounds__(kTreeThreads) void k_ansv_block(const uint8_t *__restrict__ P,
                                                             const Plan *__restrict__ plan,
                                                             uint32_t *__restrict__ BL,
                                                             uint32_t *__restrict__ BF) {
  __shared__ uint64_t sM[kTreeWaves][kVMax];
  const uint64_t r = plan->r;
  const uint64_t nbb = (r + 1 + kTreeThreads - 1) / kTreeThreads;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int vmax = (int)plan->pmax + 1;
  for (uint64_t b = blockIdx.x; b < nbb; b += gridDim.x) {
    uint64_t i = b * kTreeThreads + t;
    wave_masks(P, r, i, sM[w], lane, vmax);
    __syncthreads();
    if (t < vmax * kTreeWaves) {
      const int v = t / kTreeWaves, ww = t % kTreeWaves;
      uint32_t last, first;
      wave_ends(sM, b, v, ww, last, first);
#pragma unroll
      for (int o = kTreeWaves / 2; o > 0; o >>= 1) {
        const uint32_t l2 = __shfl_xor(last, o, kTreeWaves), f2 = __shfl_xor(first, o, kTreeWaves);
        last = l2 > last ? l2 : last;
        first = f2 < first ? f2 : first;
      }
      if (ww == 0) {
        BL[b * kVMax + v] = last;
        BF[b * kVMax + v] = first;
      }
    }
    __syncthreads();
  }
}

// Carries across blocks, for every value v: CL = exclusive prefix max of BL
// and CR = exclusive suffix min of BF over the blocks.  Done in two steps so
// that every step is parallel: k_ansv_scan scans each chunk of kTreeThreads
// blocks on its own (workgroup (chunk, v)) and records the chunk's total in
// TL / TR; k_ansv_carry turns the chunk totals into exclusive carries over
// the chunks; k_ansv_final combines the two.
template <bool MAX>
__device__ inline uint32_t blk_scan_incl(uint32_t x, uint32_t *sw, int t) {
  const int lane = t & 63, w = t >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(x, d);
    if (lane >= d) x = MAX ? (o > x ? o : x) : (o < x ? o : x);
  }
  if (lane == 63) sw[w] = x;
  __syncthreads();
  for (int ww = 0; ww < w; ww++) {
    const uint32_t o = sw[ww];
    x = MAX ? (o > x ? o : x) : (o < x ? o : x);
  }
  return x;
}

__global__ __launch_bounds__(kTreeThreads) void k_ansv_scan(const uint32_t *__restrict__ BL,
                                                            const uint32_t *__restrict__ BF,
                                                            const Plan *__restrict__ plan,
                                                            uint32_t *__restrict__ CL,
                                                            uint32_t *__restrict__ CR,
                                                            uint32_t *__restrict__ TL,
                                                            uint32_t *__restrict__ TR) {
  __shared__ uint32_t sw[kTreeWaves];
  const uint64_t r = plan->r;
  const uint64_t nbb = (r + 1 + kTreeThreads - 1) / kTreeThreads;
  const uint64_t nch = (nbb + kTreeThreads - 1) / kTreeThreads;
  const int v = blockIdx.y, t = threadIdx.x;
  if (v > (int)plan->pmax) return;   // value v + 1 is never asked for
  for (uint64_t c = blockIdx.x; c < nch; c += gridDim.x) {
    // prefix max, blocks in order
    const uint64_t b = c * kTreeThreads + t;
    const uint32_t x = b < nbb ? BL[b * kVMax + v] : 0u;
    const uint32_t inc = blk_scan_incl<true>(x, sw, t);
    const uint32_t prev = __shfl_up(inc, 1);
    uint32_t ex = prev;
    if ((t & 63) == 0) {
      ex = 0;
      for (int ww = 0; ww < (t >> 6); ww++) ex = sw[ww] > ex ? sw[ww] : ex;
    }
    if (b < nbb) CL[b * kVMax + v] = ex;
    if (t == kTreeThreads - 1) TL[c * kVMax + v] = inc;
    __syncthreads();
    // suffix min: slot t holds the chunk's block kTreeThreads-1-t
    const uint64_t bb = c * kTreeThreads + (kTreeThreads - 1 - t);
    const uint32_t y = bb < nbb ? BF[bb * kVMax + v] : kNone32;
    const uint32_t inc2 = blk_scan_incl<false>(y, sw, t);
    const uint32_t prev2 = __shfl_up(inc2, 1);
    uint32_t ex2 = prev2;
    if ((t & 63) == 0) {
      ex2 = kNone32;
      for (int ww = 0; ww < (t >> 6); ww++) ex2 = sw[ww] < ex2 ? sw[ww] : ex2;
    }
    if (bb < nbb) CR[bb * kVMax + v] = ex2;
    if (t == kTreeThreads - 1) TR[c * kVMax + v] = inc2;
    __syncthreads();
  }
}

// Chunk totals -> exclusive carries over the chunks (prefix max for TL,
// suffix min for TR), one workgroup per value.
__global__ __launch_bounds__(kTreeThreads) void k_ansv_carry(const Plan *__restrict__ plan,
                                                             uint32_t *__restrict__ TL,
                                                             uint32_t *__restrict__ TR) {
  __shared__ uint32_t sw[kTreeWaves];
  __shared__ uint32_t stot;
  const uint64_t r = plan->r;
  const uint64_t nbb = (r + 1 + kTreeThreads - 1) / kTreeThreads;
  const uint64_t nch = (nbb + kTreeThreads - 1) / kTreeThreads;
  const int v = blockIdx.x, t = threadIdx.x;
  if (v > (int)plan->pmax) return;
  uint32_t carry = 0;
  for (uint64_t base = 0; base < nch; base += kTreeThreads) {
    const uint64_t c = base + t;
    const uint32_t x = c < nch ? TL[c * kVMax + v] : 0u;
    const uint32_t inc = blk_scan_incl<true>(x, sw, t);
    uint32_t ex = __shfl_up(inc, 1);
    if ((t & 63) == 0) {
      ex = 0;
      for (int ww = 0; ww < (t >> 6); ww++) ex = sw[ww] > ex ? sw[ww] : ex;
    }
    ex = carry > ex ? carry : ex;
    if (t == kTreeThreads - 1) stot = inc;
    __syncthreads();
    if (c < nch) TL[c * kVMax + v] = ex;
    carry = stot > carry ? stot : carry;
    __syncthreads();
  }
  carry = kNone32;
  for (uint64_t done = 0; done < nch; done += kTreeThreads) {
    const uint64_t rc = done + t;   // chunk nch-1-rc
    const uint32_t x = rc < nch ? TR[(nch - 1 - rc) * kVMax + v] : kNone32;
    const uint32_t inc = blk_scan_incl<false>(x, sw, t);
    uint32_t ex = __shfl_up(inc, 1);
    if ((t & 63) == 0) {
      ex = kNone32;
      for (int ww = 0; ww < (t >> 6); ww++) ex = sw[ww] < ex ? sw[ww] : ex;
    }
    ex = carry < ex ? carry : ex;
    if (t == kTreeThreads - 1) stot = inc;
    __syncthreads();
    if (rc < nch) TR[(nch - 1 - rc) * kVMax + v] = ex;
    carry = stot < carry ? stot : carry;
    __syncthreads();
  }
}

// Nearest strictly smaller (Ls, Rs) and smaller-or-equal (Le, Re) powers on
// both sides of every boundary 1 <= i < r with power > 0.
__global__ __launch_bounds__(kTreeThreads) void k_ansv_final(
    const uint8_t *__restrict__ P, Plan *__restrict__ plan, const uint32_t *__restrict__ CL,
    const uint32_t *__restrict__ CR, const uint32_t *__restrict__ TL,
    const uint32_t *__restrict__ TR, uint32_t *__restrict__ Ls, uint32_t *__restrict__ Rs,
    uint32_t *__restrict__ Le, uint32_t *__restrict__ Re) {
  __shared__ uint64_t sM[kTreeWaves][kVMax];
  __shared__ uint32_t sPL[kTreeWaves][kVMax];   // last+1 in earlier waves (0 = none)
  __shared__ uint32_t sPR[kTreeWaves][kVMax];   // first in later waves (kNone32 = none)
  const uint64_t r = plan->r;
  const uint64_t nbb = (r + 1 + kTreeThreads - 1) / kTreeThreads;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int vmax = (int)plan->pmax + 1;
  for (uint64_t b = blockIdx.x; b < nbb; b += gridDim.x) {
    uint64_t i = b * kTreeThreads + t;
    wave_masks(P, r, i, sM[w], lane, vmax);
    __syncthreads();
    if (t < vmax * kTreeWaves) {
      // exclusive prefix max of the last ends over the earlier waves, exclusive
      // suffix min of the first ones over the later waves
      const int v = t / kTreeWaves, ww = t % kTreeWaves;
      uint32_t last, first;
      wave_ends(sM, b, v, ww, last, first);
      uint32_t pl = last, pr = first;
#pragma unroll
      for (int o = 1; o < kTreeWaves; o <<= 1) {
        const uint32_t a = __shfl_up(pl, o, kTreeWaves), c = __shfl_down(pr, o, kTreeWaves);
        if (ww >= o) pl = a > pl ? a : pl;
        if (ww + o < kTreeWaves) pr = c < pr ? c : pr;
      }
      // inclusive to exclusive: the neighbour's inclusive value
      const uint32_t el = __shfl_up(pl, 1, kTreeWaves), er = __shfl_down(pr, 1, kTreeWaves);
      sPL[ww][v] = ww > 0 ? el : 0u;
      sPR[ww][v] = ww + 1 < kTreeWaves ? er : kNone32;
    }
    __syncthreads();
    if (i > 0 && i < r) {
      uint32_t p = P[i];
      if (p > 0) {
        uint64_t below = (1ull << lane) - 1;
        uint64_t above = ~below & ~(1ull << lane);
        uint64_t wbase = b * kTreeThreads + (uint64_t)w * kWave;
        uint32_t res[4];
        for (int q = 0; q < 2; q++) {
          int vi = (int)p - 1 + q;  // q=0: power < p (strict); q=1: power <= p
          uint64_t mk = sM[w][vi] & below;
          uint32_t L;
          if (mk) L = (uint32_t)(wbase + 63 - __clzll(mk));
          else if (sPL[w][vi]) L = sPL[w][vi] - 1;
          else {
            const uint32_t c0 = CL[b * kVMax + vi], c1 = TL[(b / kTreeThreads) * kVMax + vi];
            L = (c0 > c1 ? c0 : c1) - 1;
          }
          uint64_t mr = sM[w][vi] & above;
          uint32_t R;
          if (mr) R = (uint32_t)(wbase + __ffsll((long long)mr) - 1);
          else if (sPR[w][vi] != kNone32) R = sPR[w][vi];
          else {
            const uint32_t c0 = CR[b * kVMax + vi], c1 = TR[(b / kTreeThreads) * kVMax + vi];
            R = c0 < c1 ? c0 : c1;
          }
          if (L >= i || R <= i || R > r) {  // P[0] = P[r] = 0 make both always exist
            atomicOr(&plan->error, 64u);
            L = 0;
            R = (uint32_t)r;
          }
          res[q * 2] = L;
          res[q * 2 + 1] = R;
        }
        Ls[i] = res[0];
        Rs[i] = res[1];
        Le[i] = res[2];
        Re[i] = res[3];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- merge down
// The final phase of the 4-way implementation in Appendix A.3 ("merge down"):
// after the last run, the stack holds the subtrees hanging off the tree's
// right spine, separated by the boundaries whose power is <= every power to
// their right (the chain of nearest smaller-or-equal powers from boundary
// r-1).  Instead of merging equal-power groups, the top s mod (k-1) entries
// are merged first, then k-1 at a time.  The same tree comes out of the
// power-based construction if every such group of spine boundaries gets the
// power of its leftmost boundary: spine powers rise weakly to the right and
// at most k-1 in a row are equal (Fact 3.2), so these values rise strictly
// from group to group, and none exceeds a power inside the subtrees between
// them.  One lane walks the spine (at most kMaxSpine boundaries).
constexpr int kMaxSpine = 256;
__global__ __launch_bounds__(64) void k_spine(uint8_t *__restrict__ P, const uint32_t *__restrict__ Le,
                                              Plan *__restrict__ plan, int k) {
  __shared__ uint32_t sb[kMaxSpine];
  if (threadIdx.x != 0) return;
  const uint64_t r = plan->r;
  if (r < 3) return;
  int s = 0;
  uint32_t b = (uint32_t)(r - 1);
  while (b > 0 && s < kMaxSpine) {
    sb[s++] = b;
    b = Le[b];
  }
  if (b > 0) {
    atomicOr(&plan->error, 2048u);
    return;
  }
  // sb[0] is the rightmost spine boundary; groups are taken from the right
  const int km1 = k - 1;
  int at = 0;
  for (int len = s % km1; at < s; len = km1) {
    if (len == 0) continue;
    const uint8_t v = P[sb[at + len - 1]];
    for (int t = at; t < at + len; t++) P[sb[t]] = v;
    at += len;
  }
}

// ---------------------------------------------------------------- nodes
// Leader of the equal-power group containing boundary i: follow the chain of
// nearest smaller-or-equal boundaries while the power stays equal.  A group
// has at most k-1 members (the "m <= k-1" statement after Algorithm 1).
__device__ inline uint32_t group_leader(const uint8_t *P, const uint32_t *Le, uint32_t i,
                                        uint32_t *slot) {
  uint32_t p = P[i], j = i, s = 0;
  while (s < 64 && P[Le[j]] == p) {
    j = Le[j];
    s++;
  }
  *slot = s;
  return j;
}

// Node records, one boundary at a time: the leader (first boundary) of a
// group gets its parent's leader and distance 1, or itself and 0 for a root.
// A node's span is [rs[Ls], rs[Rs]) for every boundary of its group.  The
// leader of a node of span <= kSmallSpan gets sflag kSmallNode, plus
// kSmallRoot when its parent is larger or it has none; the leader of a larger
// node gets kBigLeader; every other boundary gets 0.
//
// FULL builds every node.  Otherwise only what the sort itself reads is
// built: the member lists, arities and parent links of the larger nodes, and
// the parent links of the small roots (inside a small subtree only the root's
// span and depth parity matter, the small-subtree pass sorts the rest).
template <bool FULL>
__global__ __launch_bounds__(256) void k_nodes(const uint8_t *__restrict__ P,
                                               const uint32_t *__restrict__ Ls,
                                               const uint32_t *__restrict__ Rs,
                                               const uint32_t *__restrict__ Le,
                                               const uint32_t *__restrict__ Re,
                                               const uint64_t *__restrict__ rs, Plan *plan, int k,
                                               uint32_t *__restrict__ mem,
                                               uint8_t *__restrict__ arity,
                                               uint32_t *__restrict__ jump,
                                               uint8_t *__restrict__ dist,
                                               uint8_t *__restrict__ sflag) {
  const uint64_t r = plan->r;
  uint32_t n_small = 0;
  for (uint64_t ii = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; ii < r;
       ii += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t i = (uint32_t)ii;
    // The loads at i, then those through them, each level issued together and
    // before any branch: indices are clamped into [0, r] (entries of boundaries
    // of power 0 are never used).  A load issued under a branch is waited for
    // before the branch joins, which made these a chain of single loads; the
    // empty asm statement keeps the compiler from moving the second level
    // into the branches that use it.
    const uint32_t p = P[i];
    const uint32_t l0 = Ls[i], r0 = Rs[i], le0 = Le[i];
    const uint32_t l = l0 <= (uint32_t)r ? l0 : 0u, rr = r0 <= (uint32_t)r ? r0 : 0u;
    const uint32_t le = le0 <= (uint32_t)r ? le0 : 0u;
    const uint64_t sl = rs[l], sr = rs[rr];
    const uint32_t Pl = P[l], Pr = P[rr], Ple = P[le];
    asm volatile("" ::"v"(sl), "v"(sr), "v"(Pl), "v"(Pr), "v"(Ple));
    const bool small = sr - sl <= (uint64_t)kSmallSpan;
    const uint32_t pb = Pl >= Pr ? l : rr;   // the parent's boundary
    const uint32_t Ppb = Pl >= Pr ? Pl : Pr;
    uint8_t f = 0;
    if (p > 0) {
      if (FULL || !small) {
        uint32_t slot;
        const uint32_t lead = group_leader(P, Le, i, &slot);
        if ((int)slot > k - 2) {
          atomicOr(&plan->error, 1u);
        } else {
          mem[(uint64_t)lead * (k - 1) + slot] = i;
          if (P[Re[i]] < p) arity[lead] = (uint8_t)(slot + 2);
          if (slot == 0) {
            bool parent_small = false;
            if (Ppb == 0) {
              jump[i] = i;
              dist[i] = 0;
            } else {
              uint32_t s2;
              const uint32_t pl = group_leader(P, Le, pb, &s2);
              jump[i] = pl;
              dist[i] = 1;
              if (small) parent_small = rs[Rs[pl]] - rs[Ls[pl]] <= (uint64_t)kSmallSpan;
            }
            if (small) {
              f = (uint8_t)(kSmallNode | (parent_small ? 0 : kSmallRoot));
              n_small++;
            } else {
              f = kBigLeader;
            }
          }
        }
      } else if (Ple < p) {   // the leader of a small node
        n_small++;
        if (Ppb == 0) {
          f = kSmallNode | kSmallRoot;
          jump[i] = i;
          dist[i] = 0;
        } else if (rs[Rs[pb]] - rs[Ls[pb]] > (uint64_t)kSmallSpan) {
          uint32_t s2;
          f = kSmallNode | kSmallRoot;
          jump[i] = group_leader(P, Le, pb, &s2);
          dist[i] = 1;
        } else {
          f = kSmallNode;
        }
      }
    }
    sflag[i] = f;
  }
  block_add_into(n_small, &plan->n_small);
}

// The boundaries whose sflag has a bit of `mask` (the leaders whose depth is
// wanted; their parents are among them), listed in jlist in no particular
// order: 16 boundaries per thread from one 16-byte load of their flags (sflag
// has rmax + 1 >= r entries, padded to 16 bytes by the workspace layout), a
// block scan of the counts, and one atomic per workgroup for its slot.
__global__ __launch_bounds__(256) void k_jump_list(const uint8_t *__restrict__ sflag, uint8_t mask,
                                                   Plan *__restrict__ plan,
                                                   uint32_t *__restrict__ jlist) {
  __shared__ uint32_t sw[4];
  __shared__ uint32_t sbase;
  const uint64_t r = plan->r;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint64_t ng = (r + 15) / 16;
  for (uint64_t g0 = (uint64_t)blockIdx.x * 256; g0 < ng; g0 += (uint64_t)gridDim.x * 256) {
    const uint64_t g = g0 + t;
    uint32_t fw[4] = {0u, 0u, 0u, 0u};
    if (g < ng) {
      const uint4 fv = reinterpret_cast<const uint4 *>(sflag)[g];
      fw[0] = fv.x; fw[1] = fv.y; fw[2] = fv.z; fw[3] = fv.w;
    }
    uint32_t bits = 0;   // bit q: boundary g*16+q is listed
#pragma unroll
    for (int q = 0; q < 16; q++) {
      const uint32_t i = (uint32_t)(g * 16 + q);
      if (((fw[q >> 2] >> ((q & 3) * 8)) & mask) && i > 0 && i < r) bits |= 1u << q;
    }
    const uint32_t cnt = (uint32_t)__popc(bits);
    uint32_t incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    if (lane == 63) sw[w] = incl;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int ww = 0; ww < 4; ww++) {
      pre += ww < w ? sw[ww] : 0u;
      tot += sw[ww];
    }
    if (t == 0) sbase = tot ? atomicAdd(&plan->n_jump, tot) : 0u;
    __syncthreads();
    uint32_t at = sbase + pre + incl - cnt;
    while (bits) {
      const int q = __ffs(bits) - 1;
      bits &= bits - 1;
      jlist[at++] = (uint32_t)(g * 16 + q);
    }
    __syncthreads();   // sw and sbase are rewritten
  }
}

// One pointer-jumping round over the listed leaders: the jump target moves to
// the target's target and the distance adds up.  Roots point to themselves
// with distance 0, so once every target is a root further rounds change
// nothing; a round that finds this recorded by its predecessor only copies.
__global__ __launch_bounds__(256) void k_jump(const uint32_t *__restrict__ jlist,
                                              Plan *__restrict__ plan, int round,
                                              const uint32_t *__restrict__ jin,
                                              const uint8_t *__restrict__ din,
                                              uint32_t *__restrict__ jout,
                                              uint8_t *__restrict__ dout) {
  const uint64_t nj = plan->n_jump;
  const bool copy = round > 0 && plan->jump_more[round - 1] == 0;
  bool more = false;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < nj;
       x += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t i = jlist[x];
    if (copy) {
      jout[i] = jin[i];
      dout[i] = din[i];
      continue;
    }
    const uint32_t j = jin[i];
    dout[i] = din[i] + din[j];
    const uint32_t j2 = jin[j];
    jout[i] = j2;
    more = more || jin[j2] != j2;
  }
  if (__syncthreads_or(more) && threadIdx.x == 0) atomicOr(&plan->jump_more[round], 1u);
}

// Leaf depth: run j sits between boundaries j and j+1 and hangs below the
// node owning the larger of their powers (the leaf-depth identity in the
// proof of Theorem 3.3); both 0 means the run is a whole segment.  Bit 7
// (kLeafInSmall) marks a run whose parent is a small node: the small-subtree
// pass, not placement, reads it; without FULL its depth is not computed.
//
// A run that placement has to move (odd depth or strictly descending, and not
// inside a small subtree) flags the first and the last placement block it
// touches (pflag, cleared by k_zero32 before).
template <bool FULL>
__global__ __launch_bounds__(256) void k_leaves(const uint8_t *__restrict__ P,
                                                const uint32_t *__restrict__ Ls,
                                                const uint32_t *__restrict__ Rs,
                                                const uint32_t *__restrict__ Le,
                                                const uint8_t *__restrict__ dist,
                                                const uint64_t *__restrict__ rs, Plan *plan,
                                                int want_cost, const uint8_t *__restrict__ sflag,
                                                const uint8_t *__restrict__ desc,
                                                uint8_t *__restrict__ leaf_depth,
                                                uint32_t *__restrict__ pflag) {
  const uint64_t r = plan->r;
  uint64_t cost = 0;
  uint32_t dend = 0;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < r;
       j += (uint64_t)gridDim.x * blockDim.x) {
    // the run's larger delimiting boundary b: its node's span, or the node's
    // leader; the entries of both candidates are loaded together
    const uint32_t pa = P[j], pb = P[j + 1];
    const bool left = pa >= pb;
    const uint32_t b = left ? (uint32_t)j : (uint32_t)(j + 1);
    const uint32_t Pb = left ? pa : pb;
    uint64_t span = 0;
    if (!FULL) {
      // clamped into [0, r] (a boundary of power 0 has no node) and loaded
      // before the branch that uses them, as in k_nodes
      const uint32_t l0 = Ls[j], l1 = Ls[j + 1], r0 = Rs[j], r1 = Rs[j + 1];
      uint32_t lb = left ? l0 : l1, rb = left ? r0 : r1;
      lb = lb <= (uint32_t)r ? lb : 0u;
      rb = rb <= (uint32_t)r ? rb : 0u;
      const uint64_t slb = rs[lb], srb = rs[rb];
      asm volatile("" ::"v"(slb), "v"(srb));
      span = srb - slb;
    }
    uint8_t d = 0, in_small = 0;
    if (Pb > 0) {
      if (!FULL && span <= (uint64_t)kSmallSpan) {
        in_small = kLeafInSmall;
      } else {
        uint32_t s;
        const uint32_t lead = group_leader(P, Le, b, &s);
        d = (uint8_t)(dist[lead] + 1);
        in_small = (sflag[lead] & kSmallNode) ? kLeafInSmall : 0;
      }
    }
    leaf_depth[j] = d | in_small;
    if (!in_small && ((d & 1) || desc[j])) {
      pflag[rs[j] / kPlaceBlock] = 1u;
      pflag[(rs[j + 1] - 1) / kPlaceBlock] = 1u;
    }
    if (FULL && in_small && d > dend) dend = d;
    if (want_cost) cost += (uint64_t)d * (rs[j + 1] - rs[j]);
  }
  // the deepest small node sits just above the deepest leaf of a small subtree
  if (FULL) block_max_into<uint32_t>(dend, &plan->small_depth_end);
  if (want_cost) block_add_into(cost, &plan->merge_cost);
}

// ---------------------------------------------------------------- level lists
// Stable counting sort of the nodes (leaders) by depth.
__global__ __launch_bounds__(kTreeThreads) void k_lvl_count(const uint8_t *__restrict__ dist,
                                                            const uint8_t *__restrict__ sflag,
                                                            const Plan *__restrict__ plan,
                                                            uint32_t *__restrict__ cnt) {
  __shared__ uint32_t sc[kMaxLevels];
  const uint64_t r = plan->r;
  const uint64_t nbb = (r + 1 + kTreeThreads - 1) / kTreeThreads;
  const int t = threadIdx.x;
  for (uint64_t b = blockIdx.x; b < nbb; b += gridDim.x) {
    if (t < kMaxLevels) sc[t] = 0;
    __syncthreads();
    uint64_t i = b * kTreeThreads + t;
    if (i > 0 && i < r && (sflag[i] & kBigLeader)) atomicAdd(&sc[dist[i]], 1u);
    __syncthreads();
    if (t < kMaxLevels) cnt[b * kMaxLevels + t] = sc[t];
    __syncthreads();
  }
}

// Exclusive prefix sums of the per-block counts over the blocks, for every
// depth, in two parallel steps: workgroup (chunk, d) scans a chunk of
// kTreeThreads blocks and records its total; k_lvl_carry turns the chunk
// totals into exclusive carries (and the depth's total).  A block's offset is
// its chunk-local prefix plus its chunk's carry.
__device__ inline uint32_t blk_sum_incl(uint32_t x, uint32_t *sw, int t) {
  const int lane = t & 63, w = t >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(x, d);
    if (lane >= d) x += o;
  }
  if (lane == 63) sw[w] = x;
  __syncthreads();
  for (int ww = 0; ww < w; ww++) x += sw[ww];
  return x;
}

__global__ __launch_bounds__(kTreeThreads) void k_lvl_scan(uint32_t *__restrict__ cnt,
                                                           const Plan *__restrict__ plan,
                                                           uint32_t *__restrict__ car) {
  __shared__ uint32_t sw[kTreeWaves];
  const uint64_t r = plan->r;
  const uint64_t nbb = (r + 1 + kTreeThreads - 1) / kTreeThreads;
  const uint64_t nch = (nbb + kTreeThreads - 1) / kTreeThreads;
  const int d = blockIdx.y, t = threadIdx.x;
  for (uint64_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const uint64_t b = c * kTreeThreads + t;
    const uint32_t x = b < nbb ? cnt[b * kMaxLevels + d] : 0u;
    const uint32_t inc = blk_sum_incl(x, sw, t);
    if (b < nbb) cnt[b * kMaxLevels + d] = inc - x;
    if (t == kTreeThreads - 1) car[c * kMaxLevels + d] = inc;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kTreeThreads) void k_lvl_carry(const Plan *__restrict__ plan,
                                                            uint32_t *__restrict__ car,
                                                            uint64_t *__restrict__ totals) {
  __shared__ uint32_t sw[kTreeWaves];
  __shared__ uint32_t stot;
  const uint64_t r = plan->r;
  const uint64_t nbb = (r + 1 + kTreeThreads - 1) / kTreeThreads;
  const uint64_t nch = (nbb + kTreeThreads - 1) / kTreeThreads;
  const int d = blockIdx.x, t = threadIdx.x;
  uint64_t carry = 0;
  for (uint64_t base = 0; base < nch; base += kTreeThreads) {
    const uint64_t c = base + t;
    const uint32_t x = c < nch ? car[c * kMaxLevels + d] : 0u;
    const uint32_t inc = blk_sum_incl(x, sw, t);
    if (t == kTreeThreads - 1) stot = inc;
    __syncthreads();
    if (c < nch) car[c * kMaxLevels + d] = (uint32_t)(carry + inc - x);
    carry += stot;
    __syncthreads();
  }
  if (t == 0) totals[d] = carry;
}

__global__ void k_lvl_plan(Plan *plan, const uint64_t *__restrict__ totals, int full,
                           uint64_t cap) {
  if (threadIdx.x != 0) return;
  uint64_t acc = 0;
  uint32_t nl = 0;
  for (int d = 0; d < kMaxLevels; d++) {
    plan->lvl_begin[d] = acc;
    acc += totals[d];
    if (totals[d]) nl = d + 1;
  }
  if (acc > cap) {   // never expected: the lists are sized by a bound on such nodes
    atomicOr(&plan->error, 4096u);
    acc = 0;
    nl = 0;
    for (int d = 0; d < kMaxLevels; d++) plan->lvl_begin[d] = 0;
  }
  plan->lvl_begin[kMaxLevels] = acc;
  // the level lists hold the nodes above the small subtrees; the small ones
  // count towards the tree's size and depth all the same
  plan->n_nodes = acc + plan->n_small;
  plan->lvl_levels = nl;
  plan->n_levels = nl > plan->small_depth_end ? nl : plan->small_depth_end;
  plan->lean = full ? 0u : 1u;
}

__global__ __launch_bounds__(kTreeThreads) void k_lvl_scatter(
    const uint8_t *__restrict__ dist, const uint8_t *__restrict__ sflag,
    const Plan *__restrict__ plan, const uint32_t *__restrict__ cnt,
    const uint32_t *__restrict__ car, uint64_t cap, uint32_t *__restrict__ list) {
  __shared__ uint32_t sw[kTreeWaves][kMaxLevels];
  const uint64_t r = plan->r;
  const uint64_t nbb = (r + 1 + kTreeThreads - 1) / kTreeThreads;
  const int nl = (int)plan->lvl_levels;   // every listed leader's depth is below this
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (uint64_t b = blockIdx.x; b < nbb; b += gridDim.x) {
    uint64_t i = b * kTreeThreads + t;
    bool lead = i > 0 && i < r && (sflag[i] & kBigLeader);
    int myd = lead ? dist[i] : -1;
    uint32_t rank = 0;
    for (int d = 0; d < nl; d++) {
      uint64_t mk = ballot64(myd == d);
      if (myd == d) rank = __popcll(mk & ((1ull << lane) - 1));
      if (lane == 0) sw[w][d] = __popcll(mk);
    }
    __syncthreads();
    if (t < nl) {
      uint32_t acc = 0;
      for (int ww = 0; ww < kTreeWaves; ww++) {
        uint32_t c = sw[ww][t];
        sw[ww][t] = acc;
        acc += c;
      }
    }
    __syncthreads();
    if (lead) {
      uint64_t pos = plan->lvl_begin[myd] + car[(b / kTreeThreads) * kMaxLevels + myd] +
                     cnt[b * kMaxLevels + myd] + sw[w][myd] + rank;
      if (pos < cap) list[pos] = (uint32_t)i;
    }
    __syncthreads();
  }
}

// Node sizes in list order (into np, scanned afterwards).
__global__ __launch_bounds__(256) void k_node_sizes(const uint32_t *__restrict__ list,
                                                    const uint32_t *__restrict__ Ls,
                                                    const uint32_t *__restrict__ Rs,
                                                    const uint64_t *__restrict__ rs,
                                                    const Plan *__restrict__ plan,
                                                    uint64_t *__restrict__ np) {
  const uint64_t nn = plan->lvl_begin[kMaxLevels];   // nodes in the level lists
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nn;
       j += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t v = list[j];
    np[j] = rs[Rs[v]] - rs[Ls[v]];
  }
}

// ---------------------------------------------------------------- u64 exclusive scan
// In place over a[0..n) with n = the level lists' length; a[n] receives the total.
constexpr int kScanBlk = 1024;

__device__ inline uint64_t blk_incl_sum(uint64_t v, uint64_t *s) {
  int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int o = 1; o < kScanBlk; o <<= 1) {
    uint64_t y = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += y;
    __syncthreads();
  }
  uint64_t r = s[t];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kScanBlk) void k_scan_sums(const uint64_t *__restrict__ a,
                                                        const Plan *__restrict__ plan,
                                                        uint64_t *__restrict__ bsum) {
  __shared__ uint64_t s[kScanBlk];
  const uint64_t n = plan->lvl_begin[kMaxLevels];   // nodes in the level lists
  const uint64_t nb = (n + kScanBlk - 1) / kScanBlk;
  for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    uint64_t i = b * kScanBlk + threadIdx.x;
    uint64_t v = blk_incl_sum(i < n ? a[i] : 0, s);
    if (threadIdx.x == kScanBlk - 1) bsum[b] = v;
  }
}

__global__ __launch_bounds__(kScanBlk) void k_scan_top(uint64_t *__restrict__ bsum,
                                                       const Plan *__restrict__ plan) {
  __shared__ uint64_t s[kScanBlk];
  __shared__ uint64_t carry;
  const uint64_t n = plan->lvl_begin[kMaxLevels];   // nodes in the level lists
  const uint64_t nb = (n + kScanBlk - 1) / kScanBlk;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint64_t base = 0; base < nb; base += kScanBlk) {
    uint64_t b = base + threadIdx.x;
    uint64_t x = b < nb ? bsum[b] : 0;
    uint64_t inc = blk_incl_sum(x, s);
    if (b < nb) bsum[b] = carry + inc - x;
    __syncthreads();
    if (threadIdx.x == kScanBlk - 1) carry += inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(kScanBlk) void k_scan_apply(uint64_t *__restrict__ a,
                                                         const Plan *__restrict__ plan,
                                                         const uint64_t *__restrict__ bsum) {
  __shared__ uint64_t s[kScanBlk];
  const uint64_t n = plan->lvl_begin[kMaxLevels];   // nodes in the level lists
  const uint64_t nb = (n + kScanBlk - 1) / kScanBlk;
  for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    uint64_t i = b * kScanBlk + threadIdx.x;
    uint64_t x = i < n ? a[i] : 0;
    uint64_t inc = blk_incl_sum(x, s);
    if (i < n) a[i] = bsum[b] + inc - x;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a[n] = bsum[nb];
}

// Per-level totals and tile counts; tile tables are laid out level after level.
__global__ void k_lvl_tiles(Plan *plan, const uint64_t *__restrict__ np, int tile,
                            uint64_t *__restrict__ tile_base) {
  if (threadIdx.x != 0) return;
  uint64_t acc = 0;
  for (int d = 0; d < kMaxLevels; d++) {
    uint64_t lb = plan->lvl_begin[d], le = plan->lvl_begin[d + 1];
    uint64_t tot = np[le] - np[lb];
    plan->lvl_total[d] = tot;
    uint64_t tiles = (tot + tile - 1) / tile;
    plan->lvl_tiles[d] = tiles;
    tile_base[d] = acc;
    acc += tiles + 1;
  }
  tile_base[kMaxLevels] = acc;
}

// Tile -> node map for every level at once: entry t of level d holds the
// index (within the level's node list) of the node containing output
// position t*tile; entry `tiles` holds the level's node count.  One thread per
// tile, binary search over the level's node prefix sums.
__global__ __launch_bounds__(256) void k_tile_map(const uint64_t *__restrict__ np,
                                                  const Plan *__restrict__ plan, int tile,
                                                  const uint64_t *__restrict__ tile_base,
                                                  uint32_t *__restrict__ tj) {
  const uint64_t total = tile_base[kMaxLevels];
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (uint64_t)gridDim.x * blockDim.x) {
    int d = 0;
    while (tile_base[d + 1] <= g) d++;
    uint64_t t = g - tile_base[d];
    uint64_t lb = plan->lvl_begin[d], le = plan->lvl_begin[d + 1];
    if (t >= plan->lvl_tiles[d]) {
      tj[g] = (uint32_t)(le - lb);
      continue;
    }
    uint64_t Q = np[lb] + t * (uint64_t)tile;
    uint64_t lo = lb, hi = le - 1;   // last j with np[j] <= Q
    while (hi > lo) {
      uint64_t mid = (lo + hi + 1) >> 1;
      if (np[mid] <= Q) lo = mid; else hi = mid - 1;
    }
    tj[g] = (uint32_t)(lo - lb);
  }
}

// Before the tree of a sort built without FULL is rebuilt in full (for a
// trace): the counters that the full build adds up start again.
__global__ void k_tree_reset(Plan *plan) {
  if (threadIdx.x != 0) return;
  plan->n_small = 0;
  plan->small_depth_end = 0;
  plan->merge_cost = 0;
  plan->n_jump = 0;
  for (int i = 0; i < 8; i++) plan->jump_more[i] = 0;
}

// Sets n_levels from the rebuilt tree (the level lists keep their depths).
__global__ void k_tree_done(Plan *plan) {
  if (threadIdx.x != 0) return;
  plan->n_levels = plan->lvl_levels > plan->small_depth_end ? plan->lvl_levels : plan->small_depth_end;
  plan->lean = 0;
}

__global__ __launch_bounds__(256) void k_zero32(uint32_t *__restrict__ a, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

// ---------------------------------------------------------------- host side
static void launch_ansv_carries(const Work &w, hipStream_t s) {
  const uint64_t nbb = (w.rmax + 1 + kTreeThreads - 1) / kTreeThreads;
  const uint64_t nch = (nbb + kTreeThreads - 1) / kTreeThreads;
  const unsigned gx = (unsigned)(nch < 1024 ? nch : 1024);
  hipLaunchKernelGGL(k_ansv_scan, dim3(gx, kVMax), dim3(kTreeThreads), 0, s, w.ansv_bl, w.ansv_bf, w.plan,
                     w.ansv_cl, w.ansv_cr, w.ansv_tl, w.ansv_tr);
  hipLaunchKernelGGL(k_ansv_carry, dim3(kVMax), dim3(kTreeThreads), 0, s, w.plan, w.ansv_tl, w.ansv_tr);
}

hipError_t launch_tree(const Work &w, int want_cost, uint64_t *lvl_tot, uint64_t *tile_base,
                       uint32_t *tj, unsigned gtree, hipStream_t s) {
  const dim3 g256(8192), b256(256);
  hipLaunchKernelGGL(k_powers, g256, b256, 0, s, w.run_start, w.off, w.m, w.plan, w.logk, w.power);
  if (w.merge_down && w.k > 2) {
    // nearest smaller values of the true powers give the spine; its groups
    // get their new powers, and the pass below runs on those
    hipLaunchKernelGGL(k_ansv_block, dim3(gtree), dim3(kTreeThreads), 0, s, w.power, w.plan, w.ansv_bl, w.ansv_bf);
    launch_ansv_carries(w, s);
    hipLaunchKernelGGL(k_ansv_final, dim3(gtree), dim3(kTreeThreads), 0, s, w.power, w.plan, w.ansv_cl, w.ansv_cr, w.ansv_tl, w.ansv_tr, w.Ls, w.Rs, w.Le, w.Re);
    hipLaunchKernelGGL(k_spine, dim3(1), dim3(64), 0, s, w.power, w.Le, w.plan, w.k);
  }
  hipLaunchKernelGGL(k_ansv_block, dim3(gtree), dim3(kTreeThreads), 0, s, w.power, w.plan, w.ansv_bl, w.ansv_bf);
  launch_ansv_carries(w, s);
  hipLaunchKernelGGL(k_ansv_final, dim3(gtree), dim3(kTreeThreads), 0, s, w.power, w.plan, w.ansv_cl, w.ansv_cr, w.ansv_tl, w.ansv_tr, w.Ls, w.Rs, w.Le, w.Re);
  const bool full = want_cost != 0;
  if (full)
    hipLaunchKernelGGL(k_nodes<true>, g256, b256, 0, s, w.power, w.Ls, w.Rs, w.Le, w.Re, w.run_start, w.plan, w.k, w.nd_mem, w.nd_arity, w.jump0, w.dist0, w.sflag);
  else
    hipLaunchKernelGGL(k_nodes<false>, g256, b256, 0, s, w.power, w.Ls, w.Rs, w.Le, w.Re, w.run_start, w.plan, w.k, w.nd_mem, w.nd_arity, w.jump0, w.dist0, w.sflag);
  const uint8_t mask = full ? (uint8_t)(kBigLeader | kSmallNode) : (uint8_t)(kBigLeader | kSmallRoot);
  hipLaunchKernelGGL(k_jump_list, g256, b256, 0, s, w.sflag, mask, w.plan, w.jlist);
  for (int round = 0; round < 6; round++) {  // depths < 64
    bool even = (round & 1) == 0;
    hipLaunchKernelGGL(k_jump, g256, b256, 0, s, w.jlist, w.plan, round, even ? w.jump0 : w.jump1,
                       even ? w.dist0 : w.dist1, even ? w.jump1 : w.jump0, even ? w.dist1 : w.dist0);
  }
  {
    const uint64_t nb = w.N / kPlaceBlock + 2;
    hipLaunchKernelGGL(k_zero32, dim3((unsigned)((nb + 255) / 256 < 4096 ? (nb + 255) / 256 : 4096)),
                       b256, 0, s, w.pflag, nb);
  }
  if (full)
    hipLaunchKernelGGL(k_leaves<true>, g256, b256, 0, s, w.power, w.Ls, w.Rs, w.Le, w.dist0, w.run_start, w.plan, want_cost, w.sflag, w.run_desc, w.leaf_depth, w.pflag);
  else
    hipLaunchKernelGGL(k_leaves<false>, g256, b256, 0, s, w.power, w.Ls, w.Rs, w.Le, w.dist0, w.run_start, w.plan, want_cost, w.sflag, w.run_desc, w.leaf_depth, w.pflag);
  hipLaunchKernelGGL(k_lvl_count, dim3(gtree), dim3(kTreeThreads), 0, s, w.dist0, w.sflag, w.plan, w.lvl_cnt);
  {
    const uint64_t nbb = (w.rmax + 1 + kTreeThreads - 1) / kTreeThreads;
    const uint64_t nch = (nbb + kTreeThreads - 1) / kTreeThreads;
    const unsigned gx = (unsigned)(nch < 1024 ? nch : 1024);
    hipLaunchKernelGGL(k_lvl_scan, dim3(gx, kMaxLevels), dim3(kTreeThreads), 0, s, w.lvl_cnt, w.plan, w.lvl_car);
    hipLaunchKernelGGL(k_lvl_carry, dim3(kMaxLevels), dim3(kTreeThreads), 0, s, w.plan, w.lvl_car, lvl_tot);
  }
  hipLaunchKernelGGL(k_lvl_plan, dim3(1), dim3(64), 0, s, w.plan, lvl_tot, full ? 1 : 0, w.lvl_cap);
  hipLaunchKernelGGL(k_lvl_scatter, dim3(gtree), dim3(kTreeThreads), 0, s, w.dist0, w.sflag, w.plan, w.lvl_cnt, w.lvl_car, w.lvl_cap, w.lvl_list);
  hipLaunchKernelGGL(k_node_sizes, g256, b256, 0, s, w.lvl_list, w.Ls, w.Rs, w.run_start, w.plan, w.lvl_np);
  hipLaunchKernelGGL(k_scan_sums, dim3(1024), dim3(kScanBlk), 0, s, w.lvl_np, w.plan, w.scan_tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlk), 0, s, w.scan_tmp, w.plan);
  hipLaunchKernelGGL(k_scan_apply, dim3(1024), dim3(kScanBlk), 0, s, w.lvl_np, w.plan, w.scan_tmp);
  hipLaunchKernelGGL(k_lvl_tiles, dim3(1), dim3(64), 0, s, w.plan, w.lvl_np, w.tile, tile_base);
  hipLaunchKernelGGL(k_tile_map, dim3(2048), b256, 0, s, w.lvl_np, w.plan, w.tile, tile_base, tj);
  return hipGetLastError();
}

// After a sort, for its trace: the nearest smaller values again from the
// powers (the merges may have reused the bytes of Le / Re; Ls / Rs come out
// the same), and with nodes every node record, depth and leaf depth and the
// merge cost of a tree built without FULL, from the powers and runs still in
// the workspace.  The sort's output is not touched.
hipError_t launch_tree_complete(const Work &w, bool nodes, unsigned gtree, hipStream_t s) {
  const dim3 g256(8192), b256(256);
  hipLaunchKernelGGL(k_ansv_block, dim3(gtree), dim3(kTreeThreads), 0, s, w.power, w.plan, w.ansv_bl, w.ansv_bf);
  launch_ansv_carries(w, s);
  hipLaunchKernelGGL(k_ansv_final, dim3(gtree), dim3(kTreeThreads), 0, s, w.power, w.plan, w.ansv_cl, w.ansv_cr, w.ansv_tl, w.ansv_tr, w.Ls, w.Rs, w.Le, w.Re);
  if (!nodes) return hipGetLastError();
  hipLaunchKernelGGL(k_tree_reset, dim3(1), dim3(64), 0, s, w.plan);
  hipLaunchKernelGGL(k_nodes<true>, g256, b256, 0, s, w.power, w.Ls, w.Rs, w.Le, w.Re, w.run_start, w.plan, w.k, w.nd_mem, w.nd_arity, w.jump0, w.dist0, w.sflag);
  hipLaunchKernelGGL(k_jump_list, g256, b256, 0, s, w.sflag, (uint8_t)(kBigLeader | kSmallNode), w.plan, w.jlist);
  for (int round = 0; round < 6; round++) {
    bool even = (round & 1) == 0;
    hipLaunchKernelGGL(k_jump, g256, b256, 0, s, w.jlist, w.plan, round,
                       even ? w.jump0 : w.jump1, even ? w.dist0 : w.dist1, even ? w.jump1 : w.jump0,
                       even ? w.dist1 : w.dist0);
  }
  hipLaunchKernelGGL(k_leaves<true>, g256, b256, 0, s, w.power, w.Ls, w.Rs, w.Le, w.dist0, w.run_start, w.plan, 1, w.sflag, w.run_desc, w.leaf_depth, w.pflag);
  hipLaunchKernelGGL(k_tree_done, dim3(1), dim3(64), 0, s, w.plan);
  return hipGetLastError();
}

}  // namespace mps
