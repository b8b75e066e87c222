// mps_internal.h -- shared definitions of the gfx950 multiway-Powersort kernels.
//
// Everything here is integer work: keys are compared through an order-
// preserving map to unsigned integers (sign-bit flip for signed integers, the
// IEEE-754 total-order bit flip for float32), so no floating point is used.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mps {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kMaxLevels = 64;       // bound on merge-tree depth (powers fit in a byte)
constexpr int kVMax = 40;            // powers are < kVMax (k=2: P <= ceil(log2(2n)) <= 33)
constexpr uint32_t kNone32 = 0xFFFFFFFFu;
// Error-word bit set by the host-requested test of the error path
// (MPS_OPT_TEST_DEVICE_ERROR); the device checks use the low bits.
constexpr uint32_t kErrTestForced = 1u << 30;
constexpr uint64_t kNone64 = ~0ull;

// Key traits: storage type U and the order-preserving map to unsigned O.
template <int KT> struct Key;
template <> struct Key<0> {  // int32
  using U = uint32_t;
  __device__ static inline uint32_t ord(uint32_t b) { return b ^ 0x80000000u; }
  __device__ static inline uint32_t unord(uint32_t o) { return o ^ 0x80000000u; }
};
template <> struct Key<1> {  // int64
  using U = uint64_t;
  __device__ static inline uint64_t ord(uint64_t b) { return b ^ 0x8000000000000000ull; }
  __device__ static inline uint64_t unord(uint64_t o) { return o ^ 0x8000000000000000ull; }
};
template <> struct Key<2> {  // float32, IEEE-754 total order
  using U = uint32_t;
  __device__ static inline uint32_t ord(uint32_t b) {
    return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
  }
  __device__ static inline uint32_t unord(uint32_t o) {
    return (o & 0x80000000u) ? (o ^ 0x80000000u) : ~o;
  }
};

// Device-resident plan: everything the per-level launches need, written by
// the planning kernels so that no host synchronisation is required.
struct Plan {
  uint64_t n;                        // total elements
  uint64_t m;                        // arrays
  uint32_t kt, has_payload, k, pad;  // what the workspace was laid out for
  uint64_t r;                        // runs found
  uint64_t n_nodes;                  // internal merge-tree nodes
  uint32_t n_levels;                 // 1 + deepest internal-node depth (0: nothing to merge)
  uint32_t error;                    // nonzero: a device-side check failed
  uint64_t merge_cost;               // filled when a trace is requested or fetched
  uint64_t lvl_begin[kMaxLevels + 1];  // level-sorted node list offsets
  uint64_t lvl_total[kMaxLevels];    // sum of node sizes per level
  uint64_t lvl_tiles[kMaxLevels];    // merge tiles per level
  uint32_t gen_cnt[kMaxLevels];      // tiles per level that need the general merge path
  uint32_t q_fast[kMaxLevels];       // work-queue heads of the two merge kernels, per level
  uint32_t q_gen[kMaxLevels];
  uint32_t jump_more[8];             // pointer-jumping round i left a target that is not a root
  uint64_t r_nat;                    // natural runs, when a minimal run length replaced them
  uint64_t n_small;                  // nodes of span <= kSmallSpan (merged by the small-subtree pass)
  uint32_t small_depth_end;          // 1 + deepest depth of such a node (0: none, or not computed)
  uint32_t lvl_levels;               // levels holding a node of the level lists (1 + deepest depth)
  uint32_t lean;                     // 1: the tree was built without FULL (see launch_tree)
  uint32_t pmax;                     // the largest node power
  uint32_t n_jump;                   // leaders listed for pointer jumping (Work::jlist)
  uint32_t pad3;
};

// Small subtrees: a node whose span is at most kSmallSpan elements is
// finished, with its whole subtree, by one workgroup in LDS (the small-subtree
// pass); the level merges handle only the larger nodes.  The pass takes the
// array in chunks of kLeafChunk positions: a chunk's workgroup sorts the
// maximal small subtrees whose spans start in it, which end within kLeafCap
// positions of the chunk start.
constexpr int kSmallSpan = 1024;
constexpr int kLeafChunk = 1024;
constexpr int kLeafCap = kLeafChunk + kSmallSpan;
// Work::sflag, per boundary: kSmallNode on the leader (first boundary) of a
// node of span <= kSmallSpan, plus kSmallRoot if its parent is larger or it
// has none; kBigLeader on the leader of a larger node; 0 on every other
// boundary.
constexpr uint8_t kSmallNode = 0x80;
constexpr uint8_t kSmallRoot = 0x40;
constexpr uint8_t kBigLeader = 0x20;   // the leader of a node of span > kSmallSpan
// Per chunk, kChunkRec words: the number of small roots whose spans start in
// the chunk, then the first kChunkRec - 1 of them to be recorded (start -
// chunk start | end - chunk start << 11 | depth parity << 23).  With more
// roots the pass finds them from the boundaries instead.
constexpr int kChunkRec = 8;
static_assert(kLeafChunk <= 2048 && kLeafCap <= 4096, "root records pack 11 + 12 bits");
// Placement works in blocks of kPlaceBlock positions; Work::pflag[b] != 0
// when a run overlapping block b has to move (odd depth or strictly
// descending, and not inside a small subtree).
constexpr uint64_t kPlaceBlock = 2048;
// leaf_depth bit 7: the run's parent node is small (the small-subtree pass reads it)
constexpr uint8_t kLeafInSmall = 0x80;

// Minimal run length (runs extended to at least min_run elements): the chain
// of run starts is resolved in chunks of kMrChunk positions, composed over
// groups of kMrGroup chunks; each chunk keeps kMrCand candidate entries.
constexpr int kMrChunk = 4096;
constexpr int kMrGroup = 256;
constexpr int kMrMaxMinRun = 32;
constexpr int kMrCand = kMrMaxMinRun + 1;

// Run-detection block aggregate (16384 positions per block).
struct DetAgg {
  uint64_t lz;    // last position in the block whose direction-change bit is 0 (kNone64: none)
  uint64_t fz;    // first such position (block end if none)
  uint64_t cnt;   // breaks at or after fz (they do not depend on earlier blocks)
};

// Device views of the workspace.
struct Work {
  uint64_t N, m, rmax;
  int k, logk, tile, threads;         // arity; merge tile (outputs) and workgroup size
  void *alt_keys;
  uint32_t *alt_vals;
  const uint64_t *off;               // segment offsets [m+1]
  uint64_t *seg_off_local;           // 2-entry offsets for single-array calls
  uint64_t *dbits;
  uint64_t *seg_bits;                // [nwords] segment-start bits (batched calls; else null)
  DetAgg *det_agg;
  uint64_t *det_zin, *det_off;
  uint64_t *run_start;               // [rmax+1]
  uint8_t *run_desc;                 // [rmax]
  int min_run;                       // 1: natural runs; 2..kMrMaxMinRun: extended runs
  int merge_down;                    // final phase of Appendix A.3 (single arrays)
  int pay8;                          // the payload is 8 bytes per key (its pointers are cast)
  uint64_t *nat_start;               // [rmax+1] natural runs when min_run > 1 (single arrays)
  uint8_t *nat_desc;                 // [rmax]
  uint32_t *mr_first;                // [nch+1] first natural run at or after each chunk start
  uint8_t *mr_nxt;                   // [nch*kMrCand] exit candidate per chunk and entry
  uint16_t *mr_cnt;                  // [nch*kMrCand] runs started per chunk and entry
  uint8_t *mr_gnxt;                  // [ng*kMrCand] the same per group of chunks
  uint32_t *mr_gcnt;                 // [ng*kMrCand]
  uint8_t *mr_gentry, *mr_centry;    // [ng], [nch] entry of the chain
  uint32_t *mr_goff, *mr_coff;       // [ng], [nch] index of the first run started there
  uint8_t *power;                    // [rmax+1], power[0] = power[r] = 0
  uint32_t *ansv_bl, *ansv_bf, *ansv_cl, *ansv_cr;   // [nbb * kVMax]
  uint32_t *ansv_tl, *ansv_tr;       // [(nbb / 1024 + 1) * kVMax] carries per chunk of 1024 blocks
  uint32_t *Ls, *Rs, *Le, *Re;       // [rmax+1]
  uint8_t *nd_arity;                 // [rmax+1] (indexed by leader boundary)
  uint32_t *nd_mem;                  // [(rmax+1)*(k-1)]
  uint32_t *jump0, *jump1;           // [rmax+1]
  uint8_t *dist0, *dist1;            // [rmax+1]
  uint8_t *leaf_depth;               // [rmax] depth of every run; bit 7: kLeafInSmall
  uint8_t *sflag;                    // [rmax+1] small-node flags per boundary
  uint32_t *pflag;                   // [N/kPlaceBlock + 2] placement blocks with a run to move
  uint32_t *jlist;                   // [rmax + 1] leaders that take part in pointer jumping
  uint32_t *cfirst;                  // [N/kLeafChunk + 2] run holding each chunk's first position
  uint32_t *croot;                   // [(N/kLeafChunk + 2) * kChunkRec] small roots starting in each chunk
  uint32_t *lvl_cnt;                 // [nbb * kMaxLevels]
  uint32_t *lvl_car;                 // [(nbb / 1024 + 1) * kMaxLevels] carries per chunk of 1024 blocks
  uint32_t *lvl_list;                // [lvl_cap] nodes spanning more than kSmallSpan, by depth
  uint64_t lvl_cap;
  uint64_t *lvl_np;                  // [lvl_cap+2] exclusive prefix of node sizes
  uint64_t *scan_tmp;                // [nbb + 1024]
  uint32_t *corank;                  // [(N/tile + 2) * k]
  void *tile_desc;                   // [(N/tile + 2)] per-tile merge descriptors
  uint32_t *gen_list;                // [(N/tile + 2)] tiles of the current level on the general path
  uint64_t *samples;                 // [N/kSampleStride + 2] order key at every kSampleStride-th
                                     // position of the array as the last kernel left it
  Plan *plan;
};

// ---------------------------------------------------------------- barriers
// Workgroup barrier that orders LDS only: waits for this wave's LDS
// operations (lgkmcnt(0); the gfx9 s_waitcnt encoding keeps vmcnt and expcnt
// at their maxima) and joins s_barrier.  Unlike __syncthreads it does not wait
// for outstanding global loads and stores, so prefetched loads stay in flight
// across it.  Only for code where no global memory is exchanged between the
// workgroup's threads.
__device__ inline void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// ---------------------------------------------------------------- wave helpers
__device__ inline uint64_t ballot64(bool p) { return __ballot(p); }

__device__ inline uint64_t shfl64(uint64_t v, int src) {
  uint32_t lo = __shfl((uint32_t)v, src), hi = __shfl((uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint32_t shfl32(uint32_t v, int src) { return __shfl(v, src); }
template <typename T> __device__ inline T shfl_any(T v, int src);
template <> __device__ inline uint32_t shfl_any<uint32_t>(uint32_t v, int src) { return shfl32(v, src); }
template <> __device__ inline uint64_t shfl_any<uint64_t>(uint64_t v, int src) { return shfl64(v, src); }

// The segment containing position p (p < N): last i with off[i] <= p; that
// segment is non-empty because it contains p.
__device__ inline uint32_t seg_of(const uint64_t *off, uint64_t m, uint64_t p) {
  uint64_t lo = 0, hi = m;  // answer in [0, m)
  while (hi - lo > 1) {
    uint64_t mid = (lo + hi) >> 1;
    if (off[mid] <= p) lo = mid; else hi = mid;
  }
  return (uint32_t)lo;
}

__device__ inline bool is_seg_start(const uint64_t *off, uint64_t m, uint64_t p) {
  return off[seg_of(off, m, p)] == p;
}

// Bit b set iff position w0+b starts a non-empty segment.
__device__ inline uint64_t seg_start_mask(const uint64_t *off, uint64_t m, uint64_t w0) {
  uint64_t lo = 0, hi = m + 1;  // first i with off[i] >= w0
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (off[mid] < w0) lo = mid + 1; else hi = mid;
  }
  uint64_t mask = 0;
  for (uint64_t i = lo; i < m && off[i] < w0 + 64; i++)
    if (off[i + 1] > off[i]) mask |= 1ull << (off[i] - w0);
  return mask;
}

// ---------------------------------------------------------------- host entry points
struct LevelArgs {
  const void *in_keys;
  const uint32_t *in_vals;
  void *out_keys;
  uint32_t *out_vals;
};

// Merge tile configurations (outputs per tile x threads per workgroup):
// 1024x256, 2048x256, 2048x512 (default), 4096x512 and 4096x1024.
constexpr int kTileMin = 1024;
// Co-rank sample: the order key at every kSampleStride-th position, kept
// current by the kernels that write keys (run detection, placement, every
// level merge).  A multiple of 64.
constexpr uint64_t kSampleStride = 64;
constexpr int kTileDefault = 2048;
constexpr int kTileDescBytes = 256;  // >= sizeof(TileTab<8>), the per-tile merge table

inline bool tile_config_ok(int tile, int threads) {
  return (tile == 1024 && threads == 256) || (tile == 2048 && threads == 256) ||
         (tile == 2048 && threads == 512) || (tile == 4096 && threads == 512) ||
         (tile == 4096 && threads == 1024);
}

// Records the calling thread's error message (read by mps_last_error) and returns code.
int fail_msg(int code, const char *msg);

hipError_t launch_detect(int kt, const void *keys, const Work &w, hipStream_t s);
// Powers, nearest smaller values, nodes, depths, leaf depths and the level
// lists.  With want_cost (a traced sort) the whole tree is built and the
// merge cost summed; otherwise the records inside small subtrees are left
// out (plan->lean), and launch_tree_complete adds them later if a trace of
// the sort is fetched.
hipError_t launch_tree(const Work &w, int want_cost, uint64_t *lvl_tot, uint64_t *tile_base,
                       uint32_t *tj, unsigned grid_blocks, hipStream_t s);
// Rebuilds Ls / Rs / Le / Re from the powers (the merges may have reused the
// bytes of Le / Re); with nodes, also every node record, depth and leaf depth
// and the merge cost of a tree built without want_cost.
hipError_t launch_tree_complete(const Work &w, bool nodes, unsigned grid_blocks, hipStream_t s);
hipError_t launch_place(int kt, void *keys, uint32_t *vals, const Work &w, hipStream_t s);
// The small-subtree pass: every maximal subtree of span <= kSmallSpan is
// finished in LDS, from the runs in keys / vals (buffer 0) to the buffer of
// its root's depth parity.
hipError_t launch_leaf(int kt, void *keys, uint32_t *vals, const Work &w, hipStream_t s);
// Replaces the natural runs (w.nat_start / w.nat_desc, plan->r) by the runs
// extended to w.min_run (w.run_start / w.run_desc, plan->r).
hipError_t launch_minrun(int kt, void *keys, uint32_t *vals, const Work &w, hipStream_t s);
// Sorts the extended runs of keys / vals in place, except those inside small
// subtrees (after launch_tree: it reads the leaf depths).
hipError_t launch_minrun_sort(int kt, void *keys, uint32_t *vals, const Work &w, hipStream_t s);
hipError_t launch_level(int kt, const LevelArgs &a, const Work &w, const uint32_t *tj,
                        const uint64_t *tile_base, int level, hipStream_t s);
// The merge launches of one level for one tile configuration (each defined in
// its own translation unit).
#define MPS_DECLARE_MERGES(NAME)                                                          \
  hipError_t NAME(int kt, const LevelArgs &a, const Work &w, const uint32_t *tj,         \
                  const uint64_t *tile_base, int level, hipStream_t s);
MPS_DECLARE_MERGES(launch_merges_1024x256)
MPS_DECLARE_MERGES(launch_merges_2048x256)
MPS_DECLARE_MERGES(launch_merges_2048x512)
MPS_DECLARE_MERGES(launch_merges_4096x512)
MPS_DECLARE_MERGES(launch_merges_4096x1024)
#undef MPS_DECLARE_MERGES
// Same as launch_level, with events recorded before the co-rank, between co-rank and merge,
// and after the merge launch (all on stream s).
hipError_t launch_level_timed(int kt, const LevelArgs &a, const Work &w, const uint32_t *tj,
                              const uint64_t *tile_base, int level, hipStream_t s,
                              hipEvent_t e0, hipEvent_t e1, hipEvent_t e2);

}  // namespace mps
