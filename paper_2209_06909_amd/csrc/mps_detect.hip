// mps_detect.hip -- run detection (paper, Section 2: runs are maximal weakly
// increasing or strictly decreasing segments, found by one left-to-right scan).
//
// The greedy left-to-right scan is a two-state automaton; it is evaluated in
// parallel as follows.  For position p >= 1 let D_p = [x_p < x_{p-1}] (the pair
// ending at p is strictly decreasing) and C_p = [D_p != D_{p-1}] (direction
// change).  A run boundary ("break") falls at p iff C_p = 1 and the pair
// ending at p-1 was not itself a break; unrolled, this says: p is a break iff
// the streak of consecutive C = 1 ending at p has odd length, i.e. p - z(p) is
// odd where z(p) is the last position <= p with C = 0.  Segment starts are
// forced breaks and the first pair of every segment is forced to C = 0.
//
// Three launches: (1) direction bits by wavefront ballot plus per-block
// aggregates, (2) one workgroup scans the block aggregates (carry of z and
// the run count offsets), (3) break bits are recomputed from the direction
// bits (no key reads) and compacted into run_start / run_desc.
#include "mps_internal.h"

namespace mps {

constexpr int kDetThreads = 256;          // one 64-bit word (64 positions) per thread
constexpr uint64_t kDetBlockPos = 256 * 64;

// Break bits of one 64-position word.  C: direction-change bits (already 0 at
// forced positions and beyond the end), SB: segment starts, zpar: parity of
// the last zero position before the word.
__device__ inline uint64_t word_breaks(uint64_t C, uint64_t SB, uint64_t valid, int zpar) {
  uint64_t brk = 0;
#pragma unroll 8
  for (int j = 0; j < 64; j++) {
    if ((C >> j) & 1) {
      if ((j & 1) != zpar) brk |= 1ull << j;   // streak length p - z(p) odd
    } else {
      zpar = j & 1;
    }
  }
  return (brk | SB) & valid;
}

struct WordInfo {
  uint64_t C, SB, valid, D;
};

// Load the 256 words of a block into LDS (direction bits D and segment-start
// bits SB) and derive C for this thread's word.
__device__ inline WordInfo word_info(const uint64_t *sD, const uint64_t *sSB, int t,
                                     uint64_t prevD, uint64_t prevSB, uint64_t wstart,
                                     uint64_t N) {
  WordInfo w;
  w.D = sD[t];
  w.SB = sSB[t];
  uint64_t pd = t > 0 ? (sD[t - 1] >> 63) : prevD;
  uint64_t ps = t > 0 ? (sSB[t - 1] >> 63) : prevSB;
  uint64_t Dp = (w.D << 1) | pd;
  uint64_t FS = (w.SB << 1) | ps;  // first pair of a segment
  w.valid = (wstart + 64 <= N) ? ~0ull : (wstart >= N ? 0ull : ((1ull << (N - wstart)) - 1));
  w.C = (w.D ^ Dp) & ~(w.SB | FS) & w.valid;
  return w;
}

// Exclusive max-scan (over the 256 threads) of v; -1 marks "none".
__device__ inline int64_t block_excl_max(int64_t v, int64_t *scratch) {
  int t = threadIdx.x;
  scratch[t] = v;
  __syncthreads();
  for (int d = 1; d < kDetThreads; d <<= 1) {
    int64_t o = (t >= d) ? scratch[t - d] : -1;
    __syncthreads();
    if (o > scratch[t]) scratch[t] = o;
    __syncthreads();
  }
  int64_t r = t > 0 ? scratch[t - 1] : -1;
  __syncthreads();
  return r;
}

__device__ inline uint64_t block_excl_sum(uint64_t v, uint64_t *scratch, uint64_t *total) {
  int t = threadIdx.x;
  scratch[t] = v;
  __syncthreads();
  for (int d = 1; d < kDetThreads; d <<= 1) {
    uint64_t o = (t >= d) ? scratch[t - d] : 0;
    __syncthreads();
    scratch[t] += o;
    __syncthreads();
  }
  uint64_t r = scratch[t] - v;
  *total = scratch[kDetThreads - 1];
  __syncthreads();
  return r;
}

// D bit of position p (p >= 1): strictly decreasing pair inside a segment.
template <int KT>
__device__ inline uint64_t dbit_at(const typename Key<KT>::U *keys, const uint64_t *off, uint64_t m,
                                   uint64_t p, uint64_t N) {
  if (p == 0 || p >= N) return 0;
  if (is_seg_start(off, m, p)) return 0;
  return Key<KT>::ord(keys[p]) < Key<KT>::ord(keys[p - 1]) ? 1 : 0;
}

// ---------------------------------------------------------------- segment starts
// For batched calls: bit b of word w is set iff position 64w+b starts a
// non-empty segment, so run detection reads one word per 64 positions
// instead of searching the segment offsets.
__global__ __launch_bounds__(256) void k_seg_zero(uint64_t *__restrict__ segb, uint64_t nwords) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
       i += (uint64_t)gridDim.x * blockDim.x)
    segb[i] = 0;
}

// (Offsets are checked on the device by the caller's plan check; an offset
// past the end is not marked here, so nothing is written out of bounds.)
__global__ __launch_bounds__(256) void k_seg_set(const uint64_t *__restrict__ off, uint64_t m,
                                                 uint64_t nwords, uint64_t *__restrict__ segb) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t p = off[i];
    if (off[i + 1] > p && (p >> 6) < nwords)
      atomicOr((unsigned long long *)&segb[p >> 6], (unsigned long long)(1ull << (p & 63)));
  }
}

// ---------------------------------------------------------------- pass 1
template <int KT>
__global__ __launch_bounds__(kDetThreads) void k_detect_bits(
    const typename Key<KT>::U *__restrict__ keys, uint64_t N, const uint64_t *__restrict__ off,
    uint64_t m, const uint64_t *__restrict__ segb, uint64_t *__restrict__ dbits,
    DetAgg *__restrict__ agg, uint64_t *__restrict__ smp) {
  static_assert(kSampleStride % 64 == 0, "samples fall on 64-key word starts");
  using K = Key<KT>;
  using O = typename K::U;
  __shared__ uint64_t sD[kDetThreads], sSB[kDetThreads];
  __shared__ int64_t sScan[kDetThreads];
  __shared__ uint64_t sCarry[2];
  const uint64_t nwords = (N + 63) / 64;
  const uint64_t word0 = (uint64_t)blockIdx.x * kDetThreads;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const uint64_t my_word = word0 + t;

  uint64_t sb_own = my_word < nwords ? (segb ? segb[my_word] : seg_start_mask(off, m, my_word * 64)) : 0;
  uint64_t d_own = 0;
  const uint64_t wave_word0 = word0 + (uint64_t)wave * 64;
  O prev_last = 0;
  if (wave_word0 < nwords && wave_word0 > 0) prev_last = K::ord(keys[wave_word0 * 64 - 1]);
  // 64 words per wave, eight at a time: the eight coalesced loads are issued
  // together, then the words are processed in order.  Positions past the end
  // are clamped to the last key (loaded, never decisive: d is false there),
  // and the keys are converted where they are used: a load under a branch,
  // or one converted at once, would be waited for before the next is issued.
  constexpr int kU = 8;
  for (int i0 = 0; i0 < 64; i0 += kU) {
    if (wave_word0 + i0 >= nwords) break;  // uniform across the wave
    O xs[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const uint64_t p = (wave_word0 + i0 + u) * 64 + lane;
      xs[u] = keys[p < N ? p : N - 1];
    }
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const int i = i0 + u;
      const uint64_t p = (wave_word0 + i) * 64 + lane;
      const O x = K::ord(xs[u]);
      O xprev = shfl_any<O>(x, lane > 0 ? lane - 1 : 0);
      if (lane == 0) xprev = prev_last;
      prev_last = shfl_any<O>(x, 63);
      const uint64_t sbw = shfl64(sb_own, i);
      const bool d = p < N && p > 0 && !((sbw >> lane) & 1) && x < xprev;
      const uint64_t mask = ballot64(d);
      if (lane == i) d_own = mask;
      if (lane == 0 && p < N && (p & (kSampleStride - 1)) == 0)
        smp[p / kSampleStride] = (uint64_t)x;   // co-rank sample
    }
  }
  if (my_word < nwords) dbits[my_word] = d_own;
  sD[t] = d_own;
  sSB[t] = sb_own;
  if (t == 0) {
    uint64_t p = word0 * 64;  // block start; carry bits of position p-1
    sCarry[0] = p > 0 ? dbit_at<KT>(keys, off, m, p - 1, N) : 0;
    sCarry[1] = p > 0 ? (is_seg_start(off, m, p - 1) ? 1 : 0) : 0;
  }
  __syncthreads();

  const uint64_t wstart = my_word * 64;
  WordInfo wi = word_info(sD, sSB, t, sCarry[0], sCarry[1], wstart, N);
  uint64_t Z = ~wi.C & wi.valid;
  int64_t lz = Z ? (int64_t)(wstart + 63 - __clzll(Z)) : -1;
  int64_t zin = block_excl_max(lz, sScan);
  uint64_t cnt;
  if (zin >= 0) {
    cnt = __popcll(word_breaks(wi.C, wi.SB, wi.valid, (int)(zin & 1)));
  } else if (Z) {
    int fz = __ffsll((long long)Z) - 1;
    uint64_t b = word_breaks(wi.C, wi.SB, wi.valid, 0);
    cnt = __popcll(b & ~((1ull << fz) - 1));
  } else {
    cnt = 0;
  }
  // The block's first zero lies in the first word that has a zero and no zero
  // before it (exactly one thread); its last zero is the inclusive max-scan
  // value of the last thread.
  __shared__ uint64_t sFz;
  __shared__ int64_t sLz;
  if (t == 0) sFz = kNone64;
  __syncthreads();
  if (zin < 0 && Z) sFz = wstart + (__ffsll((long long)Z) - 1);
  if (t == kDetThreads - 1) sLz = lz > zin ? lz : zin;
  uint64_t total;
  block_excl_sum(cnt, reinterpret_cast<uint64_t *>(sScan), &total);
  if (t == 0) {
    uint64_t bend = (word0 + kDetThreads) * 64;
    if (bend > N) bend = N;
    DetAgg a;
    a.cnt = total;
    a.fz = sFz == kNone64 ? bend : sFz;
    a.lz = sLz >= 0 ? (uint64_t)sLz : kNone64;
    agg[blockIdx.x] = a;
  }
}

// ---------------------------------------------------------------- pass 2
// One workgroup of 1024 threads walks the blocks in chunks.
constexpr int kScanThreads = 1024;

__device__ inline int64_t wg_incl_max(int64_t v, int64_t *s) {
  int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    int64_t o = t >= d ? s[t - d] : -1;
    __syncthreads();
    if (o > s[t]) s[t] = o;
    __syncthreads();
  }
  int64_t r = s[t];
  __syncthreads();
  return r;
}

__device__ inline uint64_t wg_incl_sum(uint64_t v, uint64_t *s) {
  int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    uint64_t o = t >= d ? s[t - d] : 0;
    __syncthreads();
    s[t] += o;
    __syncthreads();
  }
  uint64_t r = s[t];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kScanThreads) void k_detect_scan(
    const DetAgg *__restrict__ agg, uint64_t nblk, uint64_t N, uint64_t rmax,
    uint64_t *__restrict__ zin_out, uint64_t *__restrict__ off_out,
    uint64_t *__restrict__ run_start, Plan *plan) {
  __shared__ int64_t s64[kScanThreads];
  __shared__ uint64_t carry_sum;
  __shared__ int64_t carry_z;
  const int t = threadIdx.x;
  if (t == 0) { carry_sum = 0; carry_z = -1; }
  __syncthreads();
  for (uint64_t base = 0; base < nblk; base += kScanThreads) {
    uint64_t b = base + t;
    DetAgg a = b < nblk ? agg[b] : DetAgg{kNone64, 0, 0};
    int64_t lz = a.lz == kNone64 ? -1 : (int64_t)a.lz;
    int64_t incl = wg_incl_max(lz, s64);
    int64_t excl = t > 0 ? s64[t - 1] : -1;  // s64 still holds the inclusive scan
    __syncthreads();
    int64_t z = excl > carry_z ? excl : carry_z;
    uint64_t cnt = 0;
    if (b < nblk) {
      uint64_t bs = b * kDetBlockPos;
      uint64_t len = a.fz - bs;  // positions before the first zero: all direction changes
      if (len > 0) {
        // count p in [bs, bs+len) with p - z odd; bs is even
        int zp = (int)(z & 1);
        cnt = zp == 0 ? len / 2 : (len + 1) / 2;
      }
      cnt += a.cnt;
      zin_out[b] = z >= 0 ? (uint64_t)z : kNone64;
    }
    uint64_t inc = wg_incl_sum(cnt, reinterpret_cast<uint64_t *>(s64));
    if (b < nblk) off_out[b] = carry_sum + inc - cnt;
    __syncthreads();
    if (t == kScanThreads - 1) {
      carry_sum += inc;
      if (incl > carry_z) carry_z = incl;
    }
    __syncthreads();
  }
  if (t == 0) {
    uint64_t r = carry_sum;
    if (r > rmax) {  // impossible for a correct scan: every array of length L has <= ceil(L/2) runs
      atomicOr(&plan->error, 4u);
      r = rmax;
    }
    plan->r = r;
    run_start[r] = N;
  }
}

// ---------------------------------------------------------------- pass 3
template <int KT>
__global__ __launch_bounds__(kDetThreads) void k_detect_emit(
    const typename Key<KT>::U *__restrict__ keys, uint64_t N, const uint64_t *__restrict__ off,
    uint64_t m, const uint64_t *__restrict__ segb, const uint64_t *__restrict__ dbits,
    const uint64_t *__restrict__ zin_blk,
    const uint64_t *__restrict__ off_blk, uint64_t rmax, uint64_t *__restrict__ run_start,
    uint8_t *__restrict__ run_desc) {
  __shared__ uint64_t sD[kDetThreads + 1], sSB[kDetThreads];
  __shared__ int64_t sScan[kDetThreads];
  __shared__ uint64_t sCarry[2];
  // the block's runs in order: start position within the block | direction << 15
  __shared__ uint16_t sRun[kDetBlockPos];
  static_assert(kDetBlockPos <= (1u << 15), "block positions fit in 15 bits");
  const uint64_t nwords = (N + 63) / 64;
  const uint64_t word0 = (uint64_t)blockIdx.x * kDetThreads;
  const int t = threadIdx.x;
  const uint64_t my_word = word0 + t;
  sD[t] = my_word < nwords ? dbits[my_word] : 0;
  sSB[t] = my_word < nwords ? (segb ? segb[my_word] : seg_start_mask(off, m, my_word * 64)) : 0;
  if (t == 0) {
    uint64_t nxt = word0 + kDetThreads;
    sD[kDetThreads] = nxt < nwords ? dbits[nxt] : 0;
    uint64_t p = word0 * 64;
    sCarry[0] = p > 0 ? (dbits[word0 - 1] >> 63) : 0;
    sCarry[1] = p > 0 ? (is_seg_start(off, m, p - 1) ? 1 : 0) : 0;
  }
  __syncthreads();
  const uint64_t wstart = my_word * 64;
  WordInfo wi = word_info(sD, sSB, t, sCarry[0], sCarry[1], wstart, N);
  uint64_t Z = ~wi.C & wi.valid;
  int64_t lz = Z ? (int64_t)(wstart + 63 - __clzll(Z)) : -1;
  int64_t zin = block_excl_max(lz, sScan);
  if (zin < 0) {
    uint64_t zb = zin_blk[blockIdx.x];
    zin = zb == kNone64 ? 0 : (int64_t)zb;  // block 0 starts with a forced zero
  }
  uint64_t brk = word_breaks(wi.C, wi.SB, wi.valid, (int)(zin & 1));
  uint64_t total;
  uint32_t q = (uint32_t)block_excl_sum(__popcll(brk), reinterpret_cast<uint64_t *>(sScan), &total);
  uint64_t nextD = sD[t + 1];
  // a thread's runs go to LDS first; the block then writes its runs with
  // consecutive lanes on consecutive entries (a thread's own runs would be
  // stores whose lanes lie many entries apart)
  while (brk) {
    int j = __ffsll((long long)brk) - 1;
    brk &= brk - 1;
    uint32_t dnext = j < 63 ? (uint32_t)((wi.D >> (j + 1)) & 1) : (uint32_t)(nextD & 1);
    sRun[q++] = (uint16_t)((uint32_t)(t * 64 + j) | dnext << 15);
  }
  __syncthreads();
  const uint64_t base = off_blk[blockIdx.x];
  for (uint32_t i = t; i < (uint32_t)total; i += kDetThreads) {
    const uint64_t pos = base + i;
    const uint32_t v = sRun[i];
    if (pos < rmax) {
      run_start[pos] = word0 * 64 + (v & 0x7FFFu);
      run_desc[pos] = (uint8_t)(v >> 15);
    }
  }
}

// ---------------------------------------------------------------- host side
hipError_t launch_detect(int kt, const void *keys, const Work &w, hipStream_t s) {
  uint64_t N = w.N;
  uint64_t nblk = (N + kDetBlockPos - 1) / kDetBlockPos;
  if (nblk == 0) return hipSuccess;
  dim3 g((unsigned)nblk), b(kDetThreads);
  if (w.seg_bits) {
    const uint64_t nwords = (N + 63) / 64;
    const unsigned gz = (unsigned)((nwords + 255) / 256 < 8192 ? (nwords + 255) / 256 : 8192);
    hipLaunchKernelGGL(k_seg_zero, dim3(gz), dim3(256), 0, s, w.seg_bits, nwords);
    const unsigned gs = (unsigned)((w.m + 255) / 256 < 8192 ? (w.m + 255) / 256 : 8192);
    hipLaunchKernelGGL(k_seg_set, dim3(gs), dim3(256), 0, s, w.off, w.m, nwords, w.seg_bits);
  }
  switch (kt) {
    case 0: hipLaunchKernelGGL(k_detect_bits<0>, g, b, 0, s, (const uint32_t *)keys, N, w.off, w.m, w.seg_bits, w.dbits, w.det_agg, w.samples); break;
    case 1: hipLaunchKernelGGL(k_detect_bits<1>, g, b, 0, s, (const uint64_t *)keys, N, w.off, w.m, w.seg_bits, w.dbits, w.det_agg, w.samples); break;
    default: hipLaunchKernelGGL(k_detect_bits<2>, g, b, 0, s, (const uint32_t *)keys, N, w.off, w.m, w.seg_bits, w.dbits, w.det_agg, w.samples); break;
  }
  hipLaunchKernelGGL(k_detect_scan, dim3(1), dim3(kScanThreads), 0, s, w.det_agg, nblk, N, w.rmax,
                     w.det_zin, w.det_off, w.run_start, w.plan);
  switch (kt) {
    case 0: hipLaunchKernelGGL(k_detect_emit<0>, g, b, 0, s, (const uint32_t *)keys, N, w.off, w.m, w.seg_bits, w.dbits, w.det_zin, w.det_off, w.rmax, w.run_start, w.run_desc); break;
    case 1: hipLaunchKernelGGL(k_detect_emit<1>, g, b, 0, s, (const uint64_t *)keys, N, w.off, w.m, w.seg_bits, w.dbits, w.det_zin, w.det_off, w.rmax, w.run_start, w.run_desc); break;
    default: hipLaunchKernelGGL(k_detect_emit<2>, g, b, 0, s, (const uint32_t *)keys, N, w.off, w.m, w.seg_bits, w.dbits, w.det_zin, w.det_off, w.rmax, w.run_start, w.run_desc); break;
  }
  return hipGetLastError();
}

}  // namespace mps
