// mps_leaf.hip -- the small-subtree pass.
//
// Every merge of the tree (Algorithm 1) is stable with the left input
// winning ties, and strictly descending runs are reversed before they take
// part (Section 2).  Whatever the shape of a subtree, the output of its root
// is therefore the stable sort of the root's span: the elements ordered by
// key, equal keys in their original order (a strictly descending run holds no
// equal keys, so reversing it decides no tie).  A node whose span is at most
// kSmallSpan elements is finished with its whole subtree here, in LDS: the
// span is read once, stably sorted, and written once, to the buffer of the
// root's depth parity (a node at depth d writes buffer d mod 2).  The level
// merges then start above these subtrees.
//
// The array is taken in chunks of kLeafChunk positions; the workgroup of a
// chunk handles the maximal small subtrees (the small roots) whose spans
// start in it.  Their spans are adjacent or separated by runs that hang
// directly below larger nodes, and all end within kLeafCap positions of the
// chunk start.  The tile [lo, hi) they cover is cut into pieces: every small
// root's span, and every stretch between two of them.  Each piece is sorted
// on its own and stays in its span; the stretches (runs that placement
// copies) are not written back.
//
// The sort is a block merge sort over the whole tile: every thread sorts
// kLeafItems consecutive positions in registers, then each round merges
// adjacent sorted blocks of w positions pairwise.  Because pieces are
// contiguous and keep their spans, a pair of blocks needs merging only inside
// the one piece that straddles the boundary between them (if any); every
// other position already holds its element for the doubled block.  That
// merge is a plain merge-path merge of two sorted key ranges, the left range
// winning ties.
#include "mps_merge.h"

namespace mps {

constexpr int kLeafThreads = 256;
constexpr int kLeafItems = kLeafCap / kLeafThreads;
static_assert(kLeafItems * kLeafThreads == kLeafCap, "leaf tile");
static_assert((kLeafItems & (kLeafItems - 1)) == 0 && (kLeafCap & (kLeafCap - 1)) == 0,
              "merge rounds pair power-of-two blocks");

// The run holding the first position of every chunk (entry nch: the last run
// index r), and the chunks' root counts cleared.  One thread per chunk,
// binary search in the run table.
__global__ __launch_bounds__(256) void k_chunk_runs(const uint64_t *__restrict__ rs,
                                                    const Plan *__restrict__ plan, uint64_t N,
                                                    uint32_t *__restrict__ cfirst,
                                                    uint32_t *__restrict__ croot) {
  const uint64_t r = plan->r;
  const uint64_t nch = (N + kLeafChunk - 1) / kLeafChunk;
  for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= nch;
       c += (uint64_t)gridDim.x * blockDim.x) {
    croot[c * kChunkRec] = 0;
    const uint64_t p = c * kLeafChunk < N ? c * kLeafChunk : N;
    uint64_t lo = 0, hi = r;   // last j in [0, r] with rs[j] <= p (rs[r] = N)
    while (hi > lo) {
      const uint64_t mid = (lo + hi + 1) >> 1;
      if (rs[mid] <= p) lo = mid; else hi = mid - 1;
    }
    cfirst[c] = (uint32_t)lo;
  }
}

// Records every small root in the chunk where its span starts.  A thread
// takes 16 boundaries at a time, their flags in one 16-byte load (sflag holds
// 16 bytes of slack past r).
__global__ __launch_bounds__(256) void k_chunk_mark(const uint64_t *__restrict__ rs,
                                                    const uint32_t *__restrict__ Ls,
                                                    const uint32_t *__restrict__ Rs,
                                                    const uint8_t *__restrict__ sflag,
                                                    const uint8_t *__restrict__ dist,
                                                    const Plan *__restrict__ plan,
                                                    uint32_t *__restrict__ croot) {
  const uint64_t r = plan->r;
  if (plan->n_small == 0) return;
  const uint64_t ng = (r + 15) / 16;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint4 fv = reinterpret_cast<const uint4 *>(sflag)[g];
    const uint32_t fw[4] = {fv.x, fv.y, fv.z, fv.w};
    uint32_t bits = 0;   // bit q: boundary g*16+q is a small root
#pragma unroll
    for (int q = 0; q < 16; q++) {
      const uint64_t i = g * 16 + q;
      if (((fw[q >> 2] >> ((q & 3) * 8)) & kSmallRoot) && i > 0 && i < r) bits |= 1u << q;
    }
    while (bits) {
      const int q = __ffs(bits) - 1;
      bits &= bits - 1;
      const uint64_t i = g * 16 + q;
      const uint64_t st = rs[Ls[i]], en = rs[Rs[i]];
      const uint64_t c = st / kLeafChunk, c0 = c * kLeafChunk;
      const uint32_t slot = atomicAdd(&croot[c * kChunkRec], 1u);
      if (slot + 1 < (uint32_t)kChunkRec)
        croot[c * kChunkRec + 1 + slot] =
            (uint32_t)(st - c0) | (uint32_t)(en - c0) << 11 | (uint32_t)(dist[i] & 1) << 23;
    }
  }
}

// Piece table entries: start position | kPc* flags << 13.
constexpr uint32_t kPcIn = 1;    // a small root's span
constexpr uint32_t kPcOdd = 2;   // ... whose depth is odd
constexpr int kPcShift = 13;
constexpr uint32_t kPcPos = (1u << kPcShift) - 1;
// Tags of the sort: source position | piece flags << kTagFlagShift.
constexpr int kTagFlagShift = 16;
static_assert(kChunkRec == 8, "a chunk record is read as two 16-byte words");
constexpr uint32_t kTagPos = (1u << kTagFlagShift) - 1;
static_assert(kLeafCap <= (int)kTagPos, "tag positions");
// Mark bits per position (fallback path): one byte per position.
constexpr uint32_t kMkEnd = 1, kMkStart = 2, kMkOdd = 4;

// Keys and tags are padded by one slot per kLeafItems, so the contiguous
// per-thread write-backs spread over the LDS banks.
constexpr int kLeafPad = kLeafCap + kLeafCap / kLeafItems;
static_assert(kLeafItems == 8, "lph divides by shifting");
__device__ inline int lph(int p) { return p + (p >> 3); }   // p >= 0

template <typename O, bool HV, typename V>
struct LeafSmem {
  O key[kLeafPad];                   // order keys
  uint32_t tag[kLeafPad];            // source positions and piece flags; before the sort: the root list and marks
  V val[HV ? kLeafCap : 1];          // payloads in source order
  uint16_t pinfo[kLeafCap + 2];      // piece table
  uint32_t wsum[kLeafThreads / 64];
  uint32_t misc[8];
  uint32_t todo[64];                 // chunks of the current batch in which a small root starts
};

template <typename O>
struct LeafItem {
  O k;
  uint32_t g;
};

// last piece x in [0, np] whose start is <= p
__device__ inline int leaf_piece(const uint16_t *pinfo, int np, int p) {
  int lo = 0, hi = np;
  while (hi > lo) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int)(pinfo[mid] & kPcPos) <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Positions held by one wave (a thread holds kLeafItems consecutive ones).
constexpr int kWaveSpan = 64 * kLeafItems;

// Orders the LDS accesses of one wave around the call.  A wave's LDS
// operations complete in the order they are issued, so lanes of one wave
// exchange data through LDS with no hardware barrier; only the compiler has
// to keep the accesses on their side of the call.
__device__ inline void leaf_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive block scan of one u32 per thread; the total goes to *total (LDS,
// visible after the call's last barrier).
__device__ inline uint32_t leaf_scan_excl(uint32_t v, uint32_t *wsum, uint32_t *total, int t) {
  const int lane = t & 63, wave = t >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kLeafThreads / 64; w++) {
    const uint32_t s = wsum[w];
    pre += w < wave ? s : 0;
    tot += s;
  }
  if (t == 0) *total = tot;
  __syncthreads();
  return pre + incl - v;
}

template <int KT, bool HV, typename V>
__global__ __launch_bounds__(kLeafThreads, 4) void k_leaf_pass(
    typename Key<KT>::U *__restrict__ keys, V *__restrict__ vals,
    typename Key<KT>::U *__restrict__ akeys, V *__restrict__ avals, uint64_t N,
    const uint64_t *__restrict__ rs, const uint32_t *__restrict__ Ls,
    const uint32_t *__restrict__ Rs, const uint8_t *__restrict__ sflag,
    const uint8_t *__restrict__ dist, const uint32_t *__restrict__ cfirst,
    const uint32_t *__restrict__ croot, Plan *__restrict__ plan, uint64_t *__restrict__ smp) {
  using Kt = Key<KT>;
  using U = typename Kt::U;
  using O = U;   // order keys have the storage width
  using It = LeafItem<O>;
  constexpr int CAP = kLeafCap;
  constexpr int T = kLeafThreads;
  constexpr int E = kLeafItems;
  __shared__ LeafSmem<O, HV, V> sm;
  uint32_t *roots = sm.tag;                // fallback root list [kLeafChunk]
  uint32_t *mark = sm.tag + kLeafChunk;    // fallback marks [CAP / 4]
  const int t = threadIdx.x;
  if (plan->n_small == 0) return;
  const uint64_t nch = (N + kLeafChunk - 1) / kLeafChunk;
  // chunks are taken in batches of 64; the first wave lists a batch's flagged ones
  for (uint64_t batch = (uint64_t)blockIdx.x * 64; batch < nch; batch += (uint64_t)gridDim.x * 64) {
    if (t < 64) {
      const bool f = batch + t < nch && croot[(batch + t) * kChunkRec] != 0u;
      const uint64_t mk = ballot64(f);
      if (f) sm.todo[__popcll(mk & ((1ull << t) - 1))] = (uint32_t)(batch + t);
      if (t == 0) sm.misc[7] = (uint32_t)__popcll(mk);
    }
    __syncthreads();
    const uint32_t ntodo = sm.misc[7];
    for (uint32_t ti = 0; ti < ntodo; ti++) {
      const uint64_t c = (uint64_t)__builtin_amdgcn_readfirstlane((int)sm.todo[ti]);
      const uint64_t c0 = c * kLeafChunk, c1 = c0 + kLeafChunk;
      // the chunk's whole root record in one round trip (uniform: scalar loads)
      const uint4 *rec4 = reinterpret_cast<const uint4 *>(croot + c * kChunkRec);
      const uint4 rq0 = rec4[0], rq1 = rec4[1];
      const uint32_t rv[kChunkRec] = {rq0.x, rq0.y, rq0.z, rq0.w, rq1.x, rq1.y, rq1.z, rq1.w};
      const uint32_t nrec = rv[0];
      const bool inl = nrec < (uint32_t)kChunkRec;   // uniform
      uint32_t ra = 0xFFFFFFFFu, rb = 0;   // first root start, last root end (- c0)
      if (inl) {
#pragma unroll
        for (int x = 0; x + 1 < kChunkRec; x++) {
          const uint32_t v = rv[1 + x];
          if ((uint32_t)x < nrec) {
            ra = (v & 0x7FF) < ra ? (v & 0x7FF) : ra;
            rb = ((v >> 11) & 0xFFF) > rb ? ((v >> 11) & 0xFFF) : rb;
          }
        }
      } else {
        // more roots than the record holds: leaders among the boundaries of
        // the runs covering [c0, c0 + 2C) whose spans start in [c0, c1)
        const uint32_t j0 = cfirst[c];
        const uint32_t j2 = cfirst[c + 2 < nch ? c + 2 : nch];
        if (t == 0) {
          sm.misc[0] = 0xFFFFFFFFu;
          sm.misc[1] = 0;
          sm.misc[2] = 0;
        }
        for (int x = t; x < CAP / 4; x += T) mark[x] = 0;
        __syncthreads();
        for (uint32_t i = j0 + 1 + (uint32_t)t; i < j2; i += T) {
          if (sflag[i] & kSmallRoot) {
            const uint64_t st = rs[Ls[i]];
            if (st >= c0 && st < c1) {
              const uint32_t a = (uint32_t)(st - c0), b = (uint32_t)(rs[Rs[i]] - c0);
              atomicMin(&sm.misc[0], a);
              atomicMax(&sm.misc[1], b);
              const uint32_t slot = atomicAdd(&sm.misc[2], 1u);
              if (slot < (uint32_t)kLeafChunk) roots[slot] = a | b << 11 | (uint32_t)(dist[i] & 1) << 23;
            }
          }
        }
        __syncthreads();
        ra = sm.misc[0];
        rb = sm.misc[1];
      }
      const int Tt = (int)rb - (int)ra;
      if (ra == 0xFFFFFFFFu || Tt <= 0 || Tt > CAP) {   // never expected: spans are at most kSmallSpan
        if (t == 0) atomicOr(&plan->error, 1024u);
        __syncthreads();
        continue;
      }
      const uint64_t lo = c0 + ra;
      const int Tp = (Tt + E - 1) & ~(E - 1);
      // ---- source elements, coalesced
      U kr[E];
      V vr[E];
#pragma unroll
      for (int q = 0; q < E; q++) {
        const int e = t + q * T;
        const int ec = e < Tt ? e : Tt - 1;
        kr[q] = keys[lo + (uint64_t)ec];
        if (HV) vr[q] = vals[lo + (uint64_t)ec];
      }
      // ---- the piece table
      if (inl) {
        if (t == 0) {
          // roots in position order: odd-even transposition over the record's
          // kChunkRec - 1 slots, absent ones (all ones) last; starts differ
          constexpr int NR = kChunkRec - 1;
          uint32_t v[NR];
#pragma unroll
          for (int x = 0; x < NR; x++) v[x] = (uint32_t)x < nrec ? rv[1 + x] : 0xFFFFFFFFu;
#pragma unroll
          for (int rnd = 0; rnd < NR; rnd++) {
#pragma unroll
            for (int x = rnd & 1; x + 1 < NR; x += 2) {
              const uint32_t a = v[x], b = v[x + 1];
              const bool sw = (b & 0x7FF) < (a & 0x7FF);
              v[x] = sw ? b : a;
              v[x + 1] = sw ? a : b;
            }
          }
          int np = 0;
          uint32_t prev = ra;
#pragma unroll
          for (int x = 0; x < NR; x++) {
            if ((uint32_t)x < nrec) {
              const uint32_t st = v[x] & 0x7FF, en = (v[x] >> 11) & 0xFFF;
              if (st > prev) sm.pinfo[np++] = (uint16_t)(prev - ra);   // a stretch
              sm.pinfo[np++] = (uint16_t)((st - ra) | (kPcIn | (((v[x] >> 23) & 1) ? kPcOdd : 0u)) << kPcShift);
              prev = en;
            }
          }
          sm.pinfo[np] = (uint16_t)Tt;       // padding piece
          sm.pinfo[np + 1] = (uint16_t)Tp;   // end
          sm.misc[3] = (uint32_t)np;
        }
      } else {
        const uint32_t nroots = sm.misc[2] < (uint32_t)kLeafChunk ? sm.misc[2] : (uint32_t)kLeafChunk;
        for (uint32_t x = t; x < nroots; x += T) {
          const uint32_t v = roots[x];
          const int a = (int)(v & 0x7FF) - (int)ra, b = (int)((v >> 11) & 0xFFF) - (int)ra;
          const uint32_t sb = kMkStart | (((v >> 23) & 1) ? kMkOdd : 0u);
          atomicOr(&mark[a >> 2], sb << ((a & 3) * 8));
          if (b < Tt) atomicOr(&mark[b >> 2], kMkEnd << ((b & 3) * 8));
        }
        __syncthreads();
        // piece starts: thread t counts the marks of positions [t*E, t*E + E)
        const int p0 = t * E;
        uint32_t cnt = 0;
        for (int q = 0; q < E; q++) {
          const int p = p0 + q;
          cnt += (p < Tt && ((mark[p >> 2] >> ((p & 3) * 8)) & 0xFFu) != 0u) ? 1u : 0u;
        }
        uint32_t x = leaf_scan_excl(cnt, sm.wsum, &sm.misc[3], t);
        for (int q = 0; q < E; q++) {
          const int p = p0 + q;
          const uint32_t m = p < Tt ? (mark[p >> 2] >> ((p & 3) * 8)) & 0xFFu : 0u;
          if (m != 0u)
            sm.pinfo[x++] = (uint16_t)(p | ((m & kMkStart) ? (kPcIn | ((m & kMkOdd) ? kPcOdd : 0u)) : 0u) << kPcShift);
        }
        if (t == 0) {
          const uint32_t np = sm.misc[3];
          sm.pinfo[np] = (uint16_t)Tt;
          sm.pinfo[np + 1] = (uint16_t)Tp;
        }
      }
#pragma unroll
      for (int q = 0; q < E; q++) {
        const int e = t + q * T;
        if (e < Tt) {
          sm.key[lph(e)] = Kt::ord(kr[q]);
          if (HV) sm.val[e] = vr[q];
        }
      }
      __syncthreads();   // piece table, keys, payloads; root list and marks are dead
      const int np = (int)sm.misc[3];
      // ---- per-thread stable sort of E items (odd-even transposition: only
      // neighbours in one piece are exchanged, and only when strictly out of
      // order); a position's piece never changes
      const int p0 = t * E;
      It it[E];
      int pc[E];
      {
        int x = leaf_piece(sm.pinfo, np, p0 < Tp ? p0 : 0);
#pragma unroll
        for (int q = 0; q < E; q++) {
          const int p = p0 + q;
          while (x < np && (int)(sm.pinfo[x + 1] & kPcPos) <= p) x++;
          pc[q] = x;
          it[q].k = p < Tt ? sm.key[lph(p)] : (O)~(O)0;
          // the tag: source position, and the flags of its piece (an element
          // never leaves its piece, so they travel with it to the store)
          it[q].g = (uint32_t)p |
                    (HV ? ((uint32_t)sm.pinfo[pc[q]] >> kPcShift) << kTagFlagShift : 0u);
        }
      }
#pragma unroll
      for (int rnd = 0; rnd < E; rnd++) {
#pragma unroll
        for (int q = rnd & 1; q + 1 < E; q += 2) {
          if (pc[q] == pc[q + 1] && it[q + 1].k < it[q].k) {
            const It y = it[q];
            it[q] = it[q + 1];
            it[q + 1] = y;
          }
        }
      }
      if (p0 < Tp) {
#pragma unroll
        for (int q = 0; q < E; q++) {
          sm.key[lph(p0 + q)] = it[q].k;
          if (HV) sm.tag[lph(p0 + q)] = it[q].g;
        }
      }
      // ---- merge rounds: blocks of w sorted positions, merged in pairs.  A
      // pair of 2w <= kWaveSpan positions lies in one wave's positions, so
      // such a round exchanges data only among the lanes of one wave.
      if (E < Tp) leaf_wave_sync(); else __syncthreads();
      for (int w = E; w < Tp; w <<= 1) {
        const bool wave_round = 2 * w <= kWaveSpan;
        const int base = p0 & ~(2 * w - 1), m = base + w;
        int s = 0, e = 0;
        bool act = false;
        if (p0 < Tp && m < Tp) {
          const int x = leaf_piece(sm.pinfo, np, m);
          const int ps = (int)(sm.pinfo[x] & kPcPos);
          // the piece holding position m straddles the boundary, and its
          // two halves are not already in order
          if (ps < m && sm.key[lph(m)] < sm.key[lph(m - 1)]) {
            const int pe = (int)(sm.pinfo[x + 1] & kPcPos);
            s = ps > base ? ps : base;
            e = pe < m + w ? pe : m + w;
            act = p0 + E > s && p0 < e;
          }
        }
        // this thread writes positions [p0 + q0, p0 + q0 + cnt) of [s, e)
        const int q0 = s > p0 ? s - p0 : 0;
        const int cnt = (e - p0 < E ? e - p0 : E) - q0;
        if (act) {
          // merge path: the outputs of [s, e) before this thread's first take
          // i from [s, m) and d - i from [m, e)
          const int d = p0 + q0 - s, la = m - s, lb = e - m;   // la, lb >= 1
          int lo2 = d - lb > 0 ? d - lb : 0, hi2 = d < la ? d : la;
          while (lo2 < hi2) {
            const int mid = (lo2 + hi2) >> 1;
            if (sm.key[lph(m + d - 1 - mid)] < sm.key[lph(s + mid)]) hi2 = mid; else lo2 = mid + 1;
          }
          // E merge steps without predication: ia / jb are the next positions
          // of the two halves; steps past cnt are computed and not stored
          int ia = s + lo2, jb = m + d - lo2;
          O ak = sm.key[lph(ia < m ? ia : m - 1)], bk = sm.key[lph(jb < e ? jb : e - 1)];
          int ix[E];
#pragma unroll
          for (int q = 0; q < E; q++) {
            const bool tb = jb < e && (ia >= m || bk < ak);   // ties: the left half
            it[q].k = tb ? bk : ak;
            ix[q] = tb ? jb : (ia < m ? ia : m - 1);
            if (q + 1 < E) {
              jb += tb ? 1 : 0;
              ia += tb ? 0 : 1;
              const int src = tb ? (jb < e ? jb : e - 1) : (ia < m ? ia : m - 1);
              const O nk = sm.key[lph(src)];
              bk = tb ? nk : bk;
              ak = tb ? ak : nk;
            }
          }
          if (HV) {
#pragma unroll
            for (int q = 0; q < E; q++) it[q].g = sm.tag[lph(ix[q])];
          }
        }
        if (wave_round) leaf_wave_sync(); else __syncthreads();
        if (act) {
#pragma unroll
          for (int q = 0; q < E; q++) {
            if (q < cnt) {
              sm.key[lph(p0 + q0 + q)] = it[q].k;
              if (HV) sm.tag[lph(p0 + q0 + q)] = it[q].g;
            }
          }
        }
        // the next round reads only this wave's positions if it is a wave round
        if (2 * w < Tp && 4 * w <= kWaveSpan) leaf_wave_sync(); else __syncthreads();
      }
      // ---- store every small root's span to the buffer of its depth parity
#pragma unroll
      for (int q = 0; q < E; q++) {
        const int e = t + q * T;
        if (e < Tt) {
          uint32_t f, src = 0;
          if (HV) {
            const uint32_t tg = sm.tag[lph(e)];
            f = tg >> kTagFlagShift;
            src = tg & kTagPos;
          } else {
            f = (uint32_t)sm.pinfo[leaf_piece(sm.pinfo, np, e)] >> kPcShift;
          }
          if (f & kPcIn) {
            const uint64_t g = lo + (uint64_t)e;
            const O ok = sm.key[lph(e)];
            U *dk = (f & kPcOdd) ? akeys : keys;
            dk[g] = Kt::unord(ok);
            if (HV) {
              V *dv = (f & kPcOdd) ? avals : vals;
              dv[g] = sm.val[src];
            }
            if ((g & (kSampleStride - 1)) == 0) smp[g / kSampleStride] = (uint64_t)ok;
          }
        }
      }
      __syncthreads();   // the tile's LDS is reused
    }
    __syncthreads();   // the batch list is rewritten
  }
}

template <int KT, bool HV, typename V>
static void launch_leaf_v(void *keys, uint32_t *vals, const Work &w, unsigned g, hipStream_t s) {
  using U = typename Key<KT>::U;
  hipLaunchKernelGGL((k_leaf_pass<KT, HV, V>), dim3(g), dim3(kLeafThreads), 0, s, (U *)keys,
                     (V *)vals, (U *)w.alt_keys, (V *)w.alt_vals, w.N, w.run_start, w.Ls, w.Rs,
                     w.sflag, w.dist0, w.cfirst, w.croot, w.plan, w.samples);
}

template <int KT>
static void launch_leaf_kt(void *keys, uint32_t *vals, const Work &w, hipStream_t s) {
  const uint64_t nch = (w.N + kLeafChunk - 1) / kLeafChunk;
  const uint64_t nbatch = (nch + 63) / 64;
  const unsigned g = (unsigned)(nbatch < 8192 ? nbatch : 8192);
  if (!vals) launch_leaf_v<KT, false, uint32_t>(keys, vals, w, g, s);
  else if (w.pay8) launch_leaf_v<KT, true, uint64_t>(keys, vals, w, g, s);
  else launch_leaf_v<KT, true, uint32_t>(keys, vals, w, g, s);
}

hipError_t launch_leaf(int kt, void *keys, uint32_t *vals, const Work &w, hipStream_t s) {
  const uint64_t nch = (w.N + kLeafChunk - 1) / kLeafChunk;
  const unsigned gc = (unsigned)((nch + 1 + 255) / 256 < 4096 ? (nch + 1 + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_chunk_runs, dim3(gc), dim3(256), 0, s, w.run_start, w.plan, w.N, w.cfirst,
                     w.croot);
  hipLaunchKernelGGL(k_chunk_mark, dim3(8192), dim3(256), 0, s, w.run_start, w.Ls, w.Rs, w.sflag,
                     w.dist0, w.plan, w.croot);
  switch (kt) {
    case 0: launch_leaf_kt<0>(keys, vals, w, s); break;
    case 1: launch_leaf_kt<1>(keys, vals, w, s); break;
    case 2: launch_leaf_kt<2>(keys, vals, w, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mps
