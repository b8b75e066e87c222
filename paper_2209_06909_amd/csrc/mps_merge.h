// mps_merge.h -- device code of the per-level k-way merges, shared by the
// merge translation units (one per tile configuration, so that they compile
// in parallel).
//
// Each level is cut into tiles of exactly `tile` outputs over the
// concatenation of its nodes (a tile may cover the tail of one node, whole
// small nodes and the head of another).  For every tile boundary a co-rank
// step finds how many elements of each child precede it in the stable merged
// order (key, then child index: equal keys keep their input order, as in the
// paper's merges where the left run wins ties).  A workgroup then stages the
// tile's input slices in LDS and merges them by a binary tree of 2-way
// merge-path merges (log2 k stages), all in LDS, and writes the tile back
// with coalesced stores.  Workgroups take tiles from a per-level work queue
// (an atomic counter in the plan).
#pragma once
#include <mutex>

#include "mps_internal.h"

namespace mps {

// ---------------------------------------------------------------- node access
struct NodeIn {
  uint64_t c[9];   // child boundaries: c[0] = span start, c[d] = span end
  int d;
};

// Child boundaries of node v; false (and nothing read through a bad index)
// if the node record is inconsistent.
template <int K>
__device__ inline bool load_node(uint32_t v, uint64_t r, const uint64_t *rs, const uint32_t *Ls,
                                 const uint32_t *Rs, const uint32_t *mem,
                                 const uint8_t *arity, NodeIn &nd) {
  if (v >= r) return false;
  int d = arity[v];
  if (d < 2 || d > K) return false;
  nd.d = d;
  uint32_t l = Ls[v], rr = Rs[v];
  if (l >= v || rr > r || rr <= v) return false;
  nd.c[0] = rs[l];
  uint32_t prev = l;
  for (int j = 1; j < d; j++) {
    uint32_t b = mem[(uint64_t)v * (K - 1) + (j - 1)];
    if (b <= prev || b >= rr) return false;
    nd.c[j] = rs[b];
    prev = b;
  }
  nd.c[d] = rs[rr];
  return true;
}

// Stable order across children: (key, child index).
template <typename O>
__device__ inline bool st_less(O x, int a, O y, int b) {
  return x < y || (x == y && a < b);
}

// ---------------------------------------------------------------- co-rank
// Cut of a node at output rank q: c_j = number of elements of child j among
// the first q outputs, found by a group of K lanes, lane j holding child j's
// window [lo_j, hi_j], which always contains c_j.  Each round splits the
// remaining rank over the windows proportionally and checks whether the split
// is a consistent cut (largest taken < smallest untaken in the stable order);
// otherwise the windows are narrowed around the split.  Lanes j >= d hold
// empty windows.  Sums, the split correction and the largest-taken /
// smallest-untaken choice are group reductions over shuffles, so one round
// costs a few instructions per lane and its probes are issued by different
// lanes.  The loop condition is uniform within a group.  Returns lane j's cut;
// `spent` becomes 1 if the round limit ended the search before a consistent
// cut was found (never expected: the windows shrink by at least one position
// per lane pair every round).
template <int K>
__device__ inline uint32_t gsum(uint32_t v) {
#pragma unroll
  for (int o = 1; o < K; o <<= 1) v += __shfl_xor(v, o, K);
  return v;
}

template <int K>
__device__ inline uint32_t gexcl(uint32_t v, int j) {   // exclusive prefix sum in the group
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < K; o <<= 1) {
    uint32_t y = __shfl_up(incl, o, K);
    if (j >= o) incl += y;
  }
  return incl - v;
}

template <typename O>
__device__ inline O gshfl(O v, int src, int width);
template <>
__device__ inline uint32_t gshfl<uint32_t>(uint32_t v, int src, int width) {
  return __shfl(v, src, width);
}
template <>
__device__ inline uint64_t gshfl<uint64_t>(uint64_t v, int src, int width) {
  uint32_t lo = __shfl((uint32_t)v, src, width), hi = __shfl((uint32_t)(v >> 32), src, width);
  return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t gshfl_up64(uint64_t v, int o) {
  const uint32_t lo = __shfl_up((uint32_t)v, o), hi = __shfl_up((uint32_t)(v >> 32), o);
  return ((uint64_t)hi << 32) | lo;
}

constexpr int kCorankRounds = 4096;
constexpr uint32_t kErrCorankRounds = 8192u;   // plan->error bit: a co-rank search ran out of rounds

template <typename O, int K, typename Get, typename Conv>
__device__ inline uint32_t corank_group(uint32_t q, uint32_t lo, uint32_t hi, int j, Get get,
                                       Conv conv, uint32_t &spent) {
  uint32_t mm = 0;
  spent = 1;
  for (int it = 0; it < kCorankRounds; it++) {
    const uint32_t w = hi - lo;
    const uint32_t slo = gsum<K>(lo), W = gsum<K>(w);
    const uint32_t rem = q - slo;
    if (rem == 0) { mm = 0; spent = 0; break; }
    if (rem == W) { mm = w; spent = 0; break; }
    const float f = (float)rem / (float)W;
    uint32_t v = (uint32_t)((float)w * f);
    v = v < w ? v : w;
    const uint32_t sm = gsum<K>(v);
    if (sm > rem) {          // take the excess from the lanes in order
      const uint32_t ex = sm - rem, before = gexcl<K>(v, j);
      const uint32_t dec = ex > before ? (ex - before < v ? ex - before : v) : 0;
      v -= dec;
    } else if (sm < rem) {   // give the deficit to the lanes in order
      const uint32_t de = rem - sm, cap = w - v, before = gexcl<K>(cap, j);
      const uint32_t inc = de > before ? (de - before < cap ? de - before : cap) : 0;
      v += inc;
    }
    mm = v;
    // candidate largest taken (x) and smallest untaken (y) of this lane
    const bool hx = mm > 0, hy = mm < w;
    // both probes are loaded unconditionally (the getter clamps its index)
    // and converted afterwards, so they are in flight together: a load under
    // a branch is waited for before the branch joins
    const auto xr = get(j, (uint64_t)(lo + (hx ? mm - 1 : 0)));
    const auto yr = get(j, (uint64_t)(lo + mm));
    O x = hx ? conv(xr) : (O)0;
    O y = hy ? conv(yr) : (O)0;
    const O xj = x, yj = y;
    int a = hx ? j : -1, b = hy ? j : -1;
#pragma unroll
    for (int o = 1; o < K; o <<= 1) {
      const int sl = j ^ o;
      const O xo = gshfl<O>(x, sl, K), yo = gshfl<O>(y, sl, K);
      const int ao = __shfl(a, sl, K), bo = __shfl(b, sl, K);
      // stable order (key, child): keep the later of the two taken candidates and
      // the earlier of the two untaken ones
      if (ao >= 0 && (a < 0 || st_less(x, a, xo, ao))) { x = xo; a = ao; }
      if (bo >= 0 && (b < 0 || st_less(yo, bo, y, b))) { y = yo; b = bo; }
    }
    if (a < 0 || b < 0 || a == b || st_less(x, a, y, b)) { spent = 0; break; }
    // Inconsistent: the true cut leaves x (child a) untaken and takes y
    // (child b), hence leaves everything after x untaken and takes everything
    // before y.  Every lane narrows its own window with that.
    const uint32_t at = lo + mm;
    if (j == a) hi = at - 1;
    else if (hy && st_less(x, a, yj, j)) hi = hi < at ? hi : at;
    if (j == b) lo = at + 1;
    else if (hx && st_less(xj, j, y, b)) lo = at;
  }
  return lo + mm;
}

// Cuts of every tile boundary of a level, one group of K lanes per boundary.
// For a large node the windows are first narrowed on the sample: the order
// key at every S-th position of the level's input, kept current by the
// kernels that write keys.  Child j's samples are those whose positions fall
// in the child (local positions o_j + x*S).  If the true cut takes c_j* samples of child j, then
// a_j*/S - 1 < c_j* < a_j*/S + 1, so the sample rank Q* = sum c_j* lies
// strictly between q/S - d and q/S + d.  Sample cuts are nested in the stable
// order, so the sample cut at rank Qlo <= Q* takes only truly taken samples (a
// lower bound per child) and the one at Qhi >= Q* leaves only truly untaken
// samples untaken (an upper bound).
template <int KT, int K>
__global__ __launch_bounds__(256, 8) void k_corank(const typename Key<KT>::U *__restrict__ in_keys,
                                                const uint64_t *__restrict__ rs,
                                                const uint32_t *__restrict__ Ls,
                                                const uint32_t *__restrict__ Rs,
                                                const uint32_t *__restrict__ mem,
                                                const uint8_t *__restrict__ arity,
                                                const uint32_t *__restrict__ list,
                                                const uint64_t *__restrict__ np,
                                                const uint32_t *__restrict__ tj,
                                                const uint64_t *__restrict__ tile_base,
                                                Plan *__restrict__ plan, int level,
                                                int tile, uint32_t *__restrict__ cr,
                                                const uint64_t *__restrict__ smp) {
  using O = typename Key<KT>::U;
  constexpr uint64_t S = kSampleStride;
  const uint64_t tiles = plan->lvl_tiles[level];
  if (tiles == 0) return;
  const uint64_t r = plan->r;
  const uint64_t lb = plan->lvl_begin[level];
  const uint64_t nlev = plan->lvl_begin[level + 1] - lb;
  const uint64_t np0 = np[lb];
  const uint32_t *tjl = tj + tile_base[level];
  const int j = (int)(threadIdx.x % K);
  // whole groups iterate together: the bound is a multiple of the group size
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < tiles * K;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t t = g / K;
    uint32_t out = 0;
    if (t > 0) {
      uint64_t Q = t * (uint64_t)tile;
      uint32_t jn = tjl[t];
      uint64_t q = jn < nlev ? Q - (np[lb + jn] - np0) : 0;
      NodeIn nd;
      if (jn >= nlev || !load_node<K>(list[lb + jn], r, rs, Ls, Rs, mem, arity, nd) ||
          q >= nd.c[nd.d] - nd.c[0]) {
        if (j == 0) atomicOr(&plan->error, 128u);
        q = 0;
      }
      if (q > 0) {   // uniform within the group
        uint32_t spent = 0, nspent = 0;   // uniform within the group
        const int d = nd.d;
        const bool live = j < d;
        const uint64_t cj = live ? nd.c[j] : 0, len = live ? nd.c[j + 1] - nd.c[j] : 0;
        uint32_t lo = 0, hi = (uint32_t)(len < q ? len : q);
        if (nd.c[d] - nd.c[0] >= 16 * S * (uint64_t)d) {
          const uint64_t i0 = live ? (cj + S - 1) / S : 0;
          const uint32_t m = live ? (uint32_t)((nd.c[j + 1] + S - 1) / S - i0) : 0;
          const uint64_t off = live ? i0 * S - cj : 0;
          const uint32_t ms = gsum<K>(m);
          // a lane's sample index stays in [i0, i0 + m - 1] (i0 alone when m
          // is 0: smp has N / S + 2 entries)
          const uint64_t m1 = m > 0 ? m - 1 : 0;
          auto gs = [&](int, uint64_t x) { return smp[i0 + (x < m1 ? x : m1)]; };
          auto cs = [](uint64_t v) { return (O)v; };
          const uint64_t qs = q / S;
          uint64_t qlo = qs > (uint64_t)d ? qs - d : 0;
          qlo = qlo < ms ? qlo : ms;
          const uint64_t qhi = qs + d + 1 < ms ? qs + d + 1 : ms;
          const uint32_t clo = corank_group<O, K>((uint32_t)qlo, 0u,
                                                  m < qlo ? m : (uint32_t)qlo, j, gs, cs, spent);
          nspent |= spent;
          // the cut at qhi contains the one at qlo and exceeds it by qhi - qlo in total
          const uint32_t dq = (uint32_t)(qhi - qlo);
          const uint32_t chi = corank_group<O, K>((uint32_t)qhi, clo,
                                                  m - clo < dq ? m : clo + dq, j, gs, cs, spent);
          nspent |= spent;
          uint64_t nlo = clo >= 1 ? off + (uint64_t)(clo - 1) * S + 1 : 0;
          uint64_t nhi = chi < m ? off + (uint64_t)chi * S : len;
          if (nhi > hi) nhi = hi;
          if (!live) nlo = nhi = 0;
          const uint32_t sl = gsum<K>((uint32_t)nlo), sh = gsum<K>((uint32_t)nhi);
          const uint32_t bad = gsum<K>(nlo > nhi ? 1u : 0u);
          if (bad == 0 && sl <= q && sh >= q) {
            lo = (uint32_t)nlo;
            hi = (uint32_t)nhi;
          } else if (j == 0) {
            atomicOr(&plan->error, 512u);   // never expected: keep the whole windows
          }
        }
        // a lane's key index stays in its child (a live child is never empty;
        // an idle lane reads key 0)
        const uint64_t l1 = len > 0 ? len - 1 : 0;
        auto gk = [&](int, uint64_t x) { return in_keys[cj + (x < l1 ? x : l1)]; };
        auto ck = [](O v) { return Key<KT>::ord(v); };
        out = corank_group<O, K>((uint32_t)q, lo, hi, j, gk, ck, spent);
        nspent |= spent;
        if (nspent && j == 0) atomicOr(&plan->error, kErrCorankRounds);
        if (!live) out = 0;
      }
    }
    cr[t * K + j] = out;
  }
}

// ---------------------------------------------------------------- tile merge
// A tile covers output positions [Q0, Q1) of the level's node concatenation;
// j0/j1 are the first and last node it touches.
struct TileGeom {
  uint64_t Q0, Q1, j0, j1;
  bool ok;
};

__device__ inline TileGeom tile_geom(uint64_t tile, int tsize, uint64_t L, uint64_t nlev,
                                     const uint64_t *np, uint64_t lb, uint64_t np0,
                                     const uint32_t *tjl) {
  TileGeom g;
  g.Q0 = tile * (uint64_t)tsize;
  g.Q1 = g.Q0 + tsize < L ? g.Q0 + tsize : L;
  g.j0 = tjl[tile];
  if (g.Q1 == L) {
    g.j1 = nlev - 1;
  } else {
    uint64_t jn = tjl[tile + 1];
    g.j1 = (jn < nlev && np[lb + jn] - np0 == g.Q1) ? jn - 1 : jn;
  }
  g.ok = g.j0 <= g.j1 && g.j1 < nlev;
  return g;
}

// Tables of a tile that touches at most PM nodes, built by the descriptor kernel for the merge
// kernel, which copies them to LDS word by word: the tile's input slices are
// staged back to back in LDS; slice s starts at LDS position sl_off[s], and
// the global index of LDS position e of slice s is delta[s] + e.  Piece p (a
// node's part of the tile) starts at LDS position pc_loff[p] and slice
// pc_sl[p], and its first output goes to global index pc_out[p].  kind says
// which merge path takes the tile (kTabFast: this table; kTabGeneral: the
// general kernel; kTabBad: an inconsistent cut).
enum { kTabNone = 0, kTabFast = 1, kTabGeneral = 2, kTabBad = 3 };

template <int K, int PM>
struct TileTab {
  static constexpr int kPieces = PM;
  uint64_t delta[PM * K];
  uint64_t pc_out[PM];
  uint16_t sl_off[PM * K + 2];
  uint16_t pc_loff[PM + 1];
  uint16_t pc_sl[PM + 1];
  int32_t S, P, Tt, kind;
};
// PM: three pieces for 8-byte keys and k <= 4, else two.  Above the small
// subtrees every node of a level is longer than half a 2048-position tile, so
// such a tile never touches more than three nodes; the 4-byte-key kernels keep
// two, which holds them within their register bound.
template <typename O, int K>
using TileTabFor = TileTab<K, (sizeof(O) == 8 && K <= 4) ? 3 : 2>;
template <int K, int PM>
constexpr bool tab_fits() {
  return sizeof(TileTab<K, PM>) <= kTileDescBytes && sizeof(TileTab<K, PM>) % 4 == 0 &&
         sizeof(TileTab<K, PM>) / 4 <= 64;
}
static_assert(tab_fits<2, 2>() && tab_fits<2, 3>() && tab_fits<4, 2>() && tab_fits<4, 3>() &&
                  tab_fits<8, 2>(),
              "a tile table fits its slot and is copied by the lanes of one wave, a word each");

template <int K, int PM>
__global__ __launch_bounds__(256) void k_tile_desc(
    const uint64_t *__restrict__ rs, const uint32_t *__restrict__ Ls,
    const uint32_t *__restrict__ Rs, const uint32_t *__restrict__ mem,
    const uint8_t *__restrict__ arity, const uint32_t *__restrict__ list,
    const uint64_t *__restrict__ np, const uint32_t *__restrict__ tj,
    const uint64_t *__restrict__ tile_base, Plan *__restrict__ plan, int level, int tsize,
    const uint32_t *__restrict__ cr, TileTab<K, PM> *__restrict__ desc,
    uint32_t *__restrict__ gen_list) {
  const uint64_t tiles = plan->lvl_tiles[level];
  if (tiles == 0) return;
  const uint64_t r = plan->r;
  const uint64_t lb = plan->lvl_begin[level], le = plan->lvl_begin[level + 1];
  const uint64_t nlev = le - lb;
  const uint64_t np0 = np[lb];
  const uint64_t L = np[le] - np0;
  const uint32_t *tjl = tj + tile_base[level];
  for (uint64_t tile = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; tile < tiles;
       tile += (uint64_t)gridDim.x * blockDim.x) {
    TileTab<K, PM> X;
    for (int s = 0; s < PM * K; s++) X.delta[s] = 0;
    for (int s = 0; s < PM * K + 2; s++) X.sl_off[s] = 0;
    for (int p = 0; p < PM + 1; p++) { X.pc_loff[p] = 0; X.pc_sl[p] = 0; }
    for (int p = 0; p < PM; p++) X.pc_out[p] = 0;
    X.S = 0;
    X.P = 0;
    TileGeom g = tile_geom(tile, tsize, L, nlev, np, lb, np0, tjl);
    X.Tt = (int32_t)(g.Q1 - g.Q0);
    if (!g.ok) {
      X.kind = kTabBad;
    } else if (g.j1 - g.j0 + 1 <= (uint64_t)PM) {
      const int P = (int)(g.j1 - g.j0 + 1);
      int off = 0, s = 0;
      bool bad = false;
      for (int p = 0; p < P && !bad; p++) {
        uint64_t j = g.j0 + p;
        NodeIn nd;
        if (!load_node<K>(list[lb + j], r, rs, Ls, Rs, mem, arity, nd)) { bad = true; break; }
        const bool first = p == 0;
        const bool cut_end = p == P - 1 && g.Q1 < np[lb + j + 1] - np0;
        X.pc_loff[p] = (uint16_t)off;
        X.pc_sl[p] = (uint16_t)s;
        X.pc_out[p] = nd.c[0] + (first ? g.Q0 - (np[lb + j] - np0) : 0);
        for (int jj = 0; jj < nd.d; jj++) {
          const uint32_t len = (uint32_t)(nd.c[jj + 1] - nd.c[jj]);
          const uint32_t c0 = first ? cr[tile * K + jj] : 0;
          const uint32_t c1 = cut_end ? cr[(tile + 1) * K + jj] : len;
          if (c1 > len || c0 > c1 || off + (int)(c1 - c0) > X.Tt) { bad = true; break; }
          X.sl_off[s] = (uint16_t)off;
          X.delta[s] = nd.c[jj] + c0 - (uint64_t)off;
          off += (int)(c1 - c0);
          s++;
        }
      }
      X.pc_loff[P] = (uint16_t)off;
      X.pc_sl[P] = (uint16_t)s;
      X.sl_off[s] = (uint16_t)off;
      X.S = s;
      X.P = P;
      X.kind = (bad || off != X.Tt) ? kTabBad : kTabFast;
    } else {
      X.kind = kTabGeneral;
      gen_list[atomicAdd(&plan->gen_cnt[level], 1u)] = (uint32_t)tile;
    }
    desc[tile] = X;
  }
}

// LDS of the descriptor-tile kernel: one stage buffer (the stages merge in
// place through registers) and the tables of the current and the next tile.
// The keys have 16 bytes of padding in front and behind: a lane's outputs are
// written back 16 bytes at a time, and a search probe of an empty range may
// read one element before or after the keys.
template <typename O, int K, int TILE, int VB = 4>
struct FastSmem {
  static constexpr size_t kKeyBytes = (size_t)(TILE + 4) * 8;
  static constexpr size_t kBuf = kKeyBytes + (size_t)TILE * VB;
  using Tab = TileTabFor<O, K>;
  static constexpr int kTabWords = (int)(sizeof(Tab) / 4);
  alignas(16) unsigned char bufA[kBuf];
  Tab tab[2];
  uint32_t claim[2];   // tile indices taken from the work queue
};

// LDS of the general kernel (tiles spanning many small nodes): one tile buffer
// (the stages merge in place) and the piece and slice tables.
template <typename O, int K, int TILE, int THREADS, int VB = 4>
struct GenSmem {
  static constexpr int kMaxSlices = TILE + 2 * K + 2;
  static constexpr int kMaxPieces = TILE / 2 + 4;
  static constexpr int kWaves = THREADS / 64;
  static constexpr size_t kBuf = (size_t)TILE * (sizeof(O) + VB);
  static constexpr size_t kAux = kBuf > (size_t)kMaxSlices * 8 ? kBuf : (size_t)kMaxSlices * 8;
  alignas(16) unsigned char bufA[kAux];   // the tile; holds the slices' global starts during setup
  uint64_t pc_out[kMaxPieces];
  uint16_t sl_off[kMaxSlices];
  uint16_t pc_loff[kMaxPieces];
  uint16_t pc_sl[kMaxPieces];
  uint16_t sl_pc[kMaxSlices];             // piece of each slice
  uint16_t pos_sl[TILE];                  // slice of each tile position
  uint64_t wsum[kWaves];
  int misc[8];
};

template <typename T>
__device__ inline int ub16(const uint16_t *a, int n, T x) {
  // first index in [0, n) with a[i] > x
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if ((T)a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Global addresses of a thread's E positions (t + i*THREADS).  Positions past
// the tile end are clamped to its last element (loaded, never used), so the
// loads that follow form one straight-line block: the compiler then issues
// all of them before the first wait instead of waiting between them.
template <int E, int THREADS>
__device__ inline void addr_table(uint64_t (&g)[E], const uint16_t *pos_sl,
                                  const uint16_t *sl_off, const uint64_t *sl_g, int Tt, int t) {
#pragma unroll
  for (int i = 0; i < E; i++) {
    int e = t + i * THREADS;
    int ec = e < Tt ? e : Tt - 1;
    int s = pos_sl[ec];
    g[i] = sl_g[s] + (uint64_t)(ec - sl_off[s]);
  }
}

// Same for a descriptor tile: the global index of LDS position e in slice s
// is delta[s] + e.  A wave's 64 consecutive positions t + i*THREADS usually
// lie in one slice, found with one ballot over the slice starts (lane j holds
// the start of slice j); only a wave whose positions cross a slice start
// compares per lane.
template <int E, int THREADS, typename Tab>
__device__ inline void addr_desc(uint64_t (&g)[E], const Tab &T, int t) {
  const int lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int S = T.S, Tt = T.Tt;
  const int so = (lane >= 1 && lane < S) ? (int)T.sl_off[lane] : 0x7FFFFFFF;
#pragma unroll
  for (int i = 0; i < E; i++) {
    const int x0 = (w + i * (THREADS / 64)) * 64;
    const int e = x0 + lane;
    const int ec = e < Tt ? e : Tt - 1;
    const int x1 = x0 + 63 < Tt - 1 ? x0 + 63 : Tt - 1;
    const int s0 = __builtin_popcountll(__ballot(so <= x0));
    const int s1 = __builtin_popcountll(__ballot(so <= x1));
    int s = s0;
    if (s1 != s0) {
      for (int j = s0 + 1; j <= s1; j++) s += (int)T.sl_off[j] <= ec ? 1 : 0;
    }
    g[i] = T.delta[s] + (uint64_t)ec;
  }
}

template <typename O, typename V, int E, bool HV>
__device__ inline void issue_at(O (&kreg)[E], V (&vreg)[E], const O *in_keys,
                                const V *in_vals, const uint64_t (&g)[E]) {
#pragma unroll
  for (int i = 0; i < E; i++) {
    kreg[i] = in_keys[g[i]];
    if (HV) vreg[i] = in_vals[g[i]];
  }
}

template <typename Kt, typename O, typename V, int E, int THREADS>
__device__ inline void commit_loads(const O (&kreg)[E], const V (&vreg)[E], O *kA,
                                    V *vA, bool has_vals, int Tt, int t) {
#pragma unroll
  for (int i = 0; i < E; i++) {
    int e = t + i * THREADS;
    if (e < Tt) {
      kA[e] = Kt::ord(kreg[i]);
      if (has_vals) vA[e] = vreg[i];
    }
  }
}

// log2(K) stages of pairwise merge-path merges of a general tile (any number
// of pieces), in place in one LDS buffer: a lane merges its E outputs
// [t*E, t*E+E) into registers, unit by unit, and writes them back after a
// barrier (every read of the stage done).  A lane's outputs may come from
// several merge units; output q of the lane is selected into register q.
template <typename O, typename V, int K, int TILE, int THREADS, bool HV>
__device__ inline void merge_stages_gen(O *ks, V *vs, const uint16_t *sl_off,
                                        const uint16_t *pos_sl, const uint16_t *sl_pc,
                                        const uint16_t *pc_sl, int Tt, int t) {
  constexpr int E = TILE / THREADS;
  constexpr int LOGK = K == 2 ? 1 : (K == 4 ? 2 : 3);
  const int e0 = t * E;
  const int e1 = e0 + E < Tt ? e0 + E : Tt;
  for (int st = 1; st <= LOGK; st++) {
    O ok[E];
    uint32_t os[E];   // LDS index of each output's source
#pragma unroll
    for (int i = 0; i < E; i++) {
      ok[i] = 0;
      os[i] = 0;
    }
    int e = e0;
    while (e < e1) {
      int s = pos_sl[e];
      int p = sl_pc[s];
      int s0 = pc_sl[p];
      int pd = pc_sl[p + 1] - s0;
      int jj = s - s0;
      int h = 1 << (st - 1);
      int g0 = (jj >> st) << st;
      int iM = g0 + h < pd ? g0 + h : pd;
      int iR = g0 + 2 * h < pd ? g0 + 2 * h : pd;
      int u0 = sl_off[s0 + g0], u1 = sl_off[s0 + iM], u2 = sl_off[s0 + iR];
      int nL = u1 - u0, nR = u2 - u1, diag = e - u0;
      int lo = diag - nR > 0 ? diag - nR : 0;
      int hi = diag < nL ? diag : nL;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (ks[u0 + mid] <= ks[u1 + diag - 1 - mid]) lo = mid + 1; else hi = mid;
      }
      int ia = u0 + lo, ib = u1 + diag - lo;
      int stop = e1 < u2 ? e1 : u2;
      if (stop <= e) break;  // cannot happen with valid tables (e < u2)
      // heads kept in registers; one LDS key load per output
      O ka = ks[ia < TILE ? ia : TILE - 1];
      O kb = ks[ib < TILE ? ib : TILE - 1];
      for (; e < stop; e++) {
        const bool takeL = ib >= u2 || (ia < u1 && ka <= kb);
        const O kv = takeL ? ka : kb;
        const uint32_t src = (uint32_t)(takeL ? ia : ib);
        const int q = e - e0;
#pragma unroll
        for (int i = 0; i < E; i++) {
          ok[i] = i == q ? kv : ok[i];
          os[i] = i == q ? src : os[i];
        }
        ia += takeL ? 1 : 0;
        ib += takeL ? 0 : 1;
        const int nx = takeL ? ia : ib;
        const O kn = ks[nx < TILE ? nx : TILE - 1];
        if (takeL) ka = kn; else kb = kn;
      }
    }
    V pv[E];
    if (HV) {
#pragma unroll
      for (int i = 0; i < E; i++) pv[i] = vs[os[i]];
    }
    lds_barrier();   // every read of this stage is done
#pragma unroll
    for (int i = 0; i < E; i++) {
      if (e0 + i < e1) {
        ks[e0 + i] = ok[i];
        if (HV) vs[e0 + i] = pv[i];
      }
    }
    lds_barrier();
  }
}

// Merge-path cut of one lane: the smallest i in [lo, hi] with a[i] > b[-i],
// where a[i] <= b[-i] holds for a prefix of [lo, hi) and hi - lo <= TILE/2.
// Binary lifting over uniform steps: lo only moves past positions whose
// comparison holds.  Unrolled for 8-byte keys; kept rolled for 4-byte keys,
// whose kernels would otherwise lose a workgroup per CU to register use.
template <typename O, int TILE>
__device__ inline int lift_search(const O *a, const O *b, int lo, int hi) {
  if constexpr (sizeof(O) == 8) {
#pragma unroll
    for (int step = TILE / 2; step > 0; step >>= 1) {
      const int j = lo + step - 1;
      if (j < hi && a[j] <= b[-j]) lo = j + 1;
    }
  } else {
#pragma unroll 1
    for (int step = TILE / 2; step > 0; step >>= 1) {
      const int j = lo + step - 1;
      if (j < hi && a[j] <= b[-j]) lo = j + 1;
    }
  }
  return lo;
}

// The same stages for a descriptor tile (at most PM pieces, PM*K slices), in
// place in one LDS buffer.  A lane owns the E outputs [t*E, t*E+E) at every
// stage: it merges them into registers, and after a barrier (every read of
// the stage done) writes them back over the stage's input.  The slices holding
// the lane's first and last output are found once per tile.  At stage st the
// merge unit of slice s is the group of 2^st slices of its piece that contains
// s, and the unit's bounds are read from the slice-offset table in LDS.  When
// all E outputs lie in one unit, or run from one unit into the next, one
// merge-path search (in the first unit; the next one starts at diagonal 0) and
// an unrolled E-step merge produce them.  Lanes spanning more units (only when
// a unit is shorter than E) walk unit by unit.  The key buffer carries one element of padding,
// so reading one past a unit is harmless.
template <typename O, typename V, int K, int TILE, int THREADS, bool HV, int PM>
__device__ inline void merge_stages_inplace(O *ks, V *vs, const uint16_t *sl_off_l, int S,
                                            const uint16_t *pc_sl_l, int P, int Tt, int t) {
  constexpr int E = TILE / THREADS;
  constexpr int LOGK = K == 2 ? 1 : (K == 4 ? 2 : 3);
  constexpr int KS = (int)sizeof(O);
  // first slices of the second and third pieces (S where there is none)
  const int s1 = P >= 2 ? (int)pc_sl_l[1] : S;
  const int s2 = PM >= 3 && P >= 3 ? (int)pc_sl_l[PM - 1] : S;
  // first slice of the piece holding slice s, and the end of its slices
  auto pstart = [&](int s) {
    if constexpr (PM >= 3) return s >= s2 ? s2 : (s >= s1 ? s1 : 0);
    else return s >= s1 ? s1 : 0;
  };
  auto pend = [&](int s) {
    if constexpr (PM >= 3) return s >= s2 ? S : (s >= s1 ? s2 : s1);
    else return s >= s1 ? S : s1;
  };
  const int e0 = t * E;
  const int e1 = e0 + E < Tt ? e0 + E : Tt;
  const bool full = e1 - e0 == E;
  // slices of the lane's first and last output.  8-byte keys: counts of the
  // slice starts at or below them (the starts are the same for the whole
  // workgroup); 4-byte keys: binary searches in the LDS table, which keeps
  // that kernel within 64 registers
  int sa = 0, sb = 0;
  if (e0 < e1) {
    if constexpr (sizeof(O) == 8) {
#pragma unroll
      for (int j = 1; j < PM * K; j++) {
        const int so = __builtin_amdgcn_readfirstlane(j < S ? (int)sl_off_l[j] : 0x7FFFFFFF);
        sa += so <= e0 ? 1 : 0;
        sb += so <= e1 - 1 ? 1 : 0;
      }
    } else {
      sa = ub16(sl_off_l, S + 1, e0) - 1;
      sb = ub16(sl_off_l, S + 1, e1 - 1) - 1;
    }
  }
  const char *kb8 = reinterpret_cast<const char *>(ks);
#pragma unroll
  for (int st = 1; st <= LOGK; st++) {
    const int h = 1 << (st - 1);
    const int pa0 = pstart(sa);
    const int ga = pa0 + (((sa - pa0) >> st) << st);
    const int pb0 = pstart(sb);
    const int gb = pb0 + (((sb - pb0) >> st) << st);
    O ok[E];
    uint32_t os[E];   // LDS byte offset of each output's source key
#pragma unroll
    for (int i = 0; i < E; i++) {
      ok[i] = 0;
      os[i] = 0;
    }
    // unit A holds the lane's first output; a lane whose outputs run on into
    // the next unit B (it starts where A ends) takes the same path, switching
    // to B's start mid-merge
    const int pendA = pend(sa);
    const int iMA = ga + h < pendA ? ga + h : pendA;
    const int iRA = ga + 2 * h < pendA ? ga + 2 * h : pendA;
    const int u0 = sl_off_l[ga], u1 = sl_off_l[iMA], u2 = sl_off_l[iRA];
    const bool two = full && ga != gb && (int)sl_off_l[gb] == u2;
    if (full && (ga == gb || two)) {
      const int nL = u1 - u0, nR = u2 - u1, diag = e0 - u0;
      int lo = diag - nR > 0 ? diag - nR : 0;
      const int hi = diag < nL ? diag : nL;
      // smallest i in [lo, hi] with ks[u0+i] > ks[u1+diag-1-i]
      lo = lift_search<O, TILE>(ks + u0, ks + u1 + diag - 1, lo, hi);
      uint32_t pa = (uint32_t)(u0 + lo) * KS, pb = (uint32_t)(u1 + diag - lo) * KS;
      uint32_t ea = (uint32_t)u1 * KS, eb = (uint32_t)u2 * KS;
      O ka = *reinterpret_cast<const O *>(kb8 + pa);
      O kb = *reinterpret_cast<const O *>(kb8 + pb);
      // B starts at output u2 - e0 (1..E-1) of the lane; it begins at
      // diagonal 0, so its heads are the first elements of its two halves
      const int swi = two ? u2 - e0 : E;
#pragma unroll
      for (int i = 0; i < E; i++) {
        // few waves hold a lane that switches units: a wave vote skips the
        // switch for the others
        if (i > 0 && __any(i == swi)) {
          if (i == swi) {
            const int pendB = pend(sb);
            const int iMB = gb + h < pendB ? gb + h : pendB;
            const int iRB = gb + 2 * h < pendB ? gb + 2 * h : pendB;
            pa = (uint32_t)u2 * KS;
            pb = (uint32_t)sl_off_l[iMB] * KS;
            ea = pb;
            eb = (uint32_t)sl_off_l[iRB] * KS;
            ka = *reinterpret_cast<const O *>(kb8 + pa);
            kb = *reinterpret_cast<const O *>(kb8 + pb);
          }
        }
        const bool takeL = pa < ea && (pb >= eb || ka <= kb);
        ok[i] = takeL ? ka : kb;
        os[i] = takeL ? pa : pb;
        pa += takeL ? KS : 0;
        pb += takeL ? 0 : KS;
        if (i + 1 < E) {
          const O kn = *reinterpret_cast<const O *>(kb8 + (takeL ? pa : pb));
          ka = takeL ? kn : ka;
          kb = takeL ? kb : kn;
        }
      }
    } else if (e0 < e1) {
      int e = e0;
      while (e < e1) {
        const int s = ub16(sl_off_l, S + 1, e) - 1;
        const int s0 = pstart(s);
        const int pe = pend(s);
        const int g0 = s0 + (((s - s0) >> st) << st);
        const int iM = g0 + h < pe ? g0 + h : pe;
        const int iR = g0 + 2 * h < pe ? g0 + 2 * h : pe;
        const int u0 = sl_off_l[g0], u1 = sl_off_l[iM], u2 = sl_off_l[iR];
        const int nL = u1 - u0, nR = u2 - u1, diag = e - u0;
        int lo = diag - nR > 0 ? diag - nR : 0;
        int cnt = (diag < nL ? diag : nL) - lo;
        while (cnt > 0) {
          const int half = cnt >> 1;
          const int mid = lo + half;
          const bool p = ks[u0 + mid] <= ks[u1 + diag - 1 - mid];
          lo = p ? mid + 1 : lo;
          cnt = p ? cnt - half - 1 : half;
        }
        const int stop = e1 < u2 ? e1 : u2;
        if (stop <= e) break;  // cannot happen with valid tables (e < u2)
        uint32_t pa = (uint32_t)(u0 + lo) * KS, pb = (uint32_t)(u1 + diag - lo) * KS;
        const uint32_t ea = (uint32_t)u1 * KS, eb = (uint32_t)u2 * KS;
        O ka = *reinterpret_cast<const O *>(kb8 + pa);
        O kb = *reinterpret_cast<const O *>(kb8 + pb);
        for (; e < stop; e++) {
          const bool takeL = pa < ea && (pb >= eb || ka <= kb);
          const O kv = takeL ? ka : kb;
          const uint32_t src = takeL ? pa : pb;
          const int q = e - e0;
#pragma unroll
          for (int i = 0; i < E; i++) {
            ok[i] = i == q ? kv : ok[i];
            os[i] = i == q ? src : os[i];
          }
          pa += takeL ? KS : 0;
          pb += takeL ? 0 : KS;
          const O kn = *reinterpret_cast<const O *>(kb8 + (takeL ? pa : pb));
          ka = takeL ? kn : ka;
          kb = takeL ? kb : kn;
        }
      }
    }
    V pv[E];
    if (HV) {
#pragma unroll
      for (int i = 0; i < E; i++) pv[i] = vs[os[i] / KS];
    }
    lds_barrier();   // every read of this stage is done
    if (full) {
      // 8-byte keys: 16 bytes per LDS write (ks + e0 and vs + e0 are 16-byte
      // aligned); 4-byte keys: one element per write, which keeps that kernel
      // within 64 registers
      if constexpr (sizeof(O) == 8) {
        typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int i = 0; i < E / 2; i++) {
          u64x2 v;
          v.x = ok[2 * i];
          v.y = ok[2 * i + 1];
          reinterpret_cast<u64x2 *>(ks + e0)[i] = v;
        }
        if (HV) {
          if constexpr (sizeof(V) == 8) {
#pragma unroll
            for (int i = 0; i < E / 2; i++) {
              u64x2 v;
              v.x = pv[2 * i];
              v.y = pv[2 * i + 1];
              reinterpret_cast<u64x2 *>(vs + e0)[i] = v;
            }
          } else {
#pragma unroll
            for (int i = 0; i < E / 4; i++)
              reinterpret_cast<uint4 *>(vs + e0)[i] =
                  make_uint4(pv[4 * i], pv[4 * i + 1], pv[4 * i + 2], pv[4 * i + 3]);
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < E; i++) ks[e0 + i] = ok[i];
        if (HV) {
#pragma unroll
          for (int i = 0; i < E; i++) vs[e0 + i] = pv[i];
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < E; i++) {
        if (e0 + i < e1) {
          ks[e0 + i] = ok[i];
          if (HV) vs[e0 + i] = pv[i];
        }
      }
    }
    lds_barrier();
  }
}

// Coalesced stores of a merged tile; outputs at multiples of kSampleStride also
// refresh the co-rank sample of their position.
template <typename Kt, typename O, typename V, int E, int THREADS>
__device__ inline void store_tile(const O *ks, const V *vs, O *out_keys,
                                  V *out_vals, bool has_vals, const uint16_t *pc_loff,
                                  const uint64_t *pc_out, const uint16_t *pos_sl,
                                  const uint16_t *sl_pc, int Tt, int t, uint64_t *smp) {
#pragma unroll
  for (int i = 0; i < E; i++) {
    int e = t + i * THREADS;
    if (e < Tt) {
      int p = sl_pc[pos_sl[e]];
      uint64_t g = pc_out[p] + (uint64_t)(e - pc_loff[p]);
      out_keys[g] = Kt::unord(ks[e]);
      if (has_vals) out_vals[g] = vs[e];
      if ((g & (kSampleStride - 1)) == 0) smp[g / kSampleStride] = (uint64_t)ks[e];
    }
  }
}

// Coalesced stores of a descriptor tile (up to PM pieces): the output index
// of position e is base_p + e in piece p.  The base is chosen once per wave
// unless a piece split falls among the wave's 64 positions.
template <typename Kt, typename O, typename V, int E, int THREADS, int PM>
__device__ inline void store_fast(const O *ks, const V *vs, O *out_keys, V *out_vals,
                                  bool has_vals, const uint16_t *pc_loff, const uint64_t *pc_out,
                                  int P, int Tt, int t) {
  const int sp1 = P >= 2 ? (int)pc_loff[1] : Tt;
  const int sp2 = PM >= 3 && P >= 3 ? (int)pc_loff[PM - 1] : Tt;
  const uint64_t base0 = pc_out[0] - (uint64_t)pc_loff[0];
  const uint64_t base1 = P >= 2 ? pc_out[1] - (uint64_t)pc_loff[1] : base0;
  const uint64_t base2 = PM >= 3 && P >= 3 ? pc_out[PM - 1] - (uint64_t)pc_loff[PM - 1] : base1;
  const int lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
#pragma unroll
  for (int i = 0; i < E; i++) {
    const int x0 = (w + i * (THREADS / 64)) * 64;
    const int e = x0 + lane;
    uint64_t base;
    if constexpr (PM >= 3) {
      if (x0 + 63 < sp1) base = base0;
      else if (x0 >= sp2) base = base2;
      else if (x0 >= sp1 && x0 + 63 < sp2) base = base1;
      else base = e < sp1 ? base0 : (e < sp2 ? base1 : base2);
    } else {
      if (x0 + 63 < sp1) base = base0;
      else if (x0 >= sp1) base = base1;
      else base = e < sp1 ? base0 : base1;
    }
    if (e < Tt) {
      const uint64_t g = base + (uint64_t)e;
      out_keys[g] = Kt::unord(ks[e]);
      if (has_vals) out_vals[g] = vs[e];
    }
  }
}

// The co-rank samples among a descriptor tile's outputs (every
// kSampleStride-th global position), written by the lanes of one wave.
template <typename O, int PM>
__device__ inline void store_samples(const O *ks, const uint16_t *pc_loff, const uint64_t *pc_out,
                                     int P, int Tt, int lane, uint64_t *smp) {
  for (int p = 0; p < P && p < PM; p++) {
    const int l0 = pc_loff[p], l1 = p + 1 < P ? (int)pc_loff[p + 1] : Tt;
    const uint64_t g0 = pc_out[p], g1 = g0 + (uint64_t)(l1 - l0);
    const uint64_t q0 = (g0 + kSampleStride - 1) / kSampleStride;
    for (uint64_t q = q0 + (uint64_t)lane; q * kSampleStride < g1; q += 64)
      smp[q] = (uint64_t)ks[l0 + (int)(q * kSampleStride - g0)];
  }
}

// Tiles per work-queue claim of the descriptor-tile kernel: the claiming wave
// waits for the claim's return, which also waits for all of its outstanding
// memory operations, so claims should be rare.
constexpr int kFastClaim = 8;
// Tiles per claim of the general kernel (its tiles are fewer and longer).
constexpr int kGenClaim = 4;

// Descriptor tiles.  Each workgroup takes tiles from the level's work queue
// (kFastClaim at a time, skipping those of the general path) and processes
// them software-pipelined: while tile i is merged in LDS, the table of tile
// i+2 and the input slices of tile i+1 are already being fetched into
// registers, so global latency overlaps the LDS work.  A tile's table is
// copied to LDS by the lanes of the first wave, one word each.
template <int KT, int K, int TILE, int THREADS, bool HV, typename V = uint32_t>
// With 4-byte keys, 4-byte payloads, k <= 4 and 4 outputs per lane the kernel
// fits in 64 registers, which lets 4 workgroups of 512 threads share a CU.
__global__ __launch_bounds__(THREADS, (sizeof(typename Key<KT>::U) == 4 && sizeof(V) == 4 && K <= 4 && TILE == 4 * THREADS) ? 8 : 1)
void k_merge_fast(
    const typename Key<KT>::U *__restrict__ in_keys, const V *__restrict__ in_vals,
    typename Key<KT>::U *__restrict__ out_keys, V *__restrict__ out_vals,
    Plan *__restrict__ plan, int level, const TileTabFor<typename Key<KT>::U, K> *__restrict__ desc,
    uint64_t *__restrict__ smp) {
  using Kt = Key<KT>;
  using O = typename Kt::U;
  using SM = FastSmem<O, K, TILE, (int)sizeof(V)>;
  constexpr int E = TILE / THREADS;
  constexpr int NW = SM::kTabWords;
  constexpr int PM = SM::Tab::kPieces;
  __shared__ SM sm;
  O *kA = reinterpret_cast<O *>(sm.bufA + 16);
  V *vA = reinterpret_cast<V *>(sm.bufA + SM::kKeyBytes);
  const uint32_t *descw = reinterpret_cast<const uint32_t *>(desc);

  const uint64_t tiles = plan->lvl_tiles[level];
  if (tiles == 0) return;
  uint32_t *queue = &plan->q_fast[level];
  const int t = threadIdx.x;
  const int lane = t & 63;

  if (t == 0) sm.claim[0] = atomicAdd(queue, (uint32_t)kFastClaim);
  __syncthreads();
  uint64_t cbase = sm.claim[0];
  int cidx = 2;
  uint64_t tile = cbase;
  uint64_t nxt = cbase + 1;
  if (tile >= tiles) return;

  O kreg[E];
  V vreg[E];
  uint64_t ga[E];
  uint32_t dreg = 0;   // one word of a prefetched table (lanes 0..NW-1)

  // prologue: table of the first tile, then the loads of the first tile and
  // the table of the second
  if (t < NW) reinterpret_cast<uint32_t *>(&sm.tab[0])[t] = descw[tile * NW + t];
  lds_barrier();
  if (t < NW && nxt < tiles) dreg = descw[nxt * NW + t];
  if (sm.tab[0].kind == kTabFast) {
    addr_desc<E, THREADS>(ga, sm.tab[0], t);
    issue_at<O, V, E, HV>(kreg, vreg, in_keys, in_vals, ga);
  }
  int cur = 0;

  while (tile < tiles) {
    // claim the tile after next now; its index is published after the next barrier
    const bool reclaim = cidx == kFastClaim;
    uint32_t claimed = 0;
    if (reclaim && t == 0) claimed = atomicAdd(queue, (uint32_t)kFastClaim);
    typename SM::Tab &T = sm.tab[cur];
    typename SM::Tab &N = sm.tab[cur ^ 1];
    const int kind = T.kind;
    if (kind == kTabFast) commit_loads<Kt, O, V, E, THREADS>(kreg, vreg, kA, vA, HV, T.Tt, t);
    // next tile's table from its prefetched words (kTabNone past the end)
    if (t < NW) reinterpret_cast<uint32_t *>(&N)[t] = nxt < tiles ? dreg : 0u;
    if (t == 0 && reclaim) sm.claim[1] = claimed;
    lds_barrier();
    if (reclaim) {
      cbase = sm.claim[1];
      cidx = 0;
    }
    const uint64_t after = cbase + (uint64_t)cidx++;
    if (t < NW && after < tiles) dreg = descw[after * NW + t];
    if (N.kind == kTabFast) {
      addr_desc<E, THREADS>(ga, N, t);
      issue_at<O, V, E, HV>(kreg, vreg, in_keys, in_vals, ga);
    }
    if (kind == kTabFast) {
      merge_stages_inplace<O, V, K, TILE, THREADS, HV, PM>(kA, vA, T.sl_off, T.S, T.pc_sl, T.P,
                                                           T.Tt, t);
      store_fast<Kt, O, V, E, THREADS, PM>(kA, vA, out_keys, out_vals, HV, T.pc_loff, T.pc_out,
                                           T.P, T.Tt, t);
      if (t >= THREADS - 64) store_samples<O, PM>(kA, T.pc_loff, T.pc_out, T.P, T.Tt, lane, smp);
    } else if (kind == kTabBad) {
      if (t == 0) atomicOr(&plan->error, 32u);
    }
    lds_barrier();
    cur ^= 1;
    tile = nxt;
    nxt = after;
  }
}

// Tiles spanning many small nodes (listed by the descriptor kernel): piece
// and slice tables are built from the node records, then the same staged
// merge runs.  Not pipelined.
template <int KT, int K, int TILE, int THREADS, bool HV, typename V = uint32_t>
__global__ __launch_bounds__(THREADS, K <= 4 ? 6 : 1) void k_merge_general(
    const typename Key<KT>::U *__restrict__ in_keys, const V *__restrict__ in_vals,
    typename Key<KT>::U *__restrict__ out_keys, V *__restrict__ out_vals,
    const uint64_t *__restrict__ rs, const uint32_t *__restrict__ Ls,
    const uint32_t *__restrict__ Rs, const uint32_t *__restrict__ mem,
    const uint8_t *__restrict__ arity, const uint32_t *__restrict__ list,
    const uint64_t *__restrict__ np, const uint32_t *__restrict__ tj,
    const uint64_t *__restrict__ tile_base, Plan *__restrict__ plan, int level,
    const uint32_t *__restrict__ cr, const uint32_t *__restrict__ gen_list,
    uint64_t *__restrict__ smp) {
  using Kt = Key<KT>;
  using O = typename Kt::U;
  using SM = GenSmem<O, K, TILE, THREADS, (int)sizeof(V)>;
  constexpr int E = TILE / THREADS;
  __shared__ SM sm;
  O *kA = reinterpret_cast<O *>(sm.bufA);
  V *vA = reinterpret_cast<V *>(sm.bufA + (size_t)TILE * sizeof(O));
  uint64_t *sl_g = reinterpret_cast<uint64_t *>(sm.bufA);

  const uint32_t ngen = plan->gen_cnt[level];
  if (ngen == 0) return;
  const uint64_t rr_total = plan->r;
  const uint64_t lb = plan->lvl_begin[level], le = plan->lvl_begin[level + 1];
  const uint64_t nlev = le - lb;
  const uint64_t np0 = np[lb];
  const uint64_t L = np[le] - np0;
  const uint32_t *tjl = tj + tile_base[level];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  uint64_t ga[E];

  // Tiles are claimed kGenClaim at a time: a claim's returned value makes the
  // wave wait for all of its outstanding memory operations.
  uint32_t *queue = &plan->q_gen[level];
  uint32_t cbase = 0;
  int cidx = kGenClaim;
  for (;;) {
    if (cidx == kGenClaim) {
      if (t == 0) sm.misc[5] = (int)atomicAdd(queue, (uint32_t)kGenClaim);
      __syncthreads();
      cbase = (uint32_t)sm.misc[5];
      cidx = 0;
    }
    const uint32_t gi = cbase + (uint32_t)cidx++;
    if (gi >= ngen) break;
    const uint64_t tile = gen_list[gi];
    TileGeom g = tile_geom(tile, TILE, L, nlev, np, lb, np0, tjl);
    const int Tt = (int)(g.Q1 - g.Q0);
    const int P = (int)(g.j1 - g.j0 + 1);
    bool bad = !g.ok || P + 1 > SM::kMaxPieces;
    if (t == 0) sm.misc[4] = bad ? 1 : 0;
    __syncthreads();
    if (!bad) {
      const uint64_t Q0 = g.Q0, Q1 = g.Q1, j0 = g.j0;
      uint64_t carry_len = 0, carry_sl = 0;
      for (int pbase = 0; pbase < P; pbase += THREADS) {
        int p = pbase + t;
        NodeIn nd;
        uint32_t c0[K], c1[K];
        uint64_t plen = 0;
        int pd = 0;
        if (p < P) {
          uint64_t j = j0 + p;
          if (!load_node<K>(list[lb + j], rr_total, rs, Ls, Rs, mem, arity, nd)) {
            sm.misc[4] = 1;
            nd.d = 2;
            nd.c[0] = nd.c[1] = nd.c[2] = 0;
          }
          pd = nd.d;
          bool first = p == 0, last = p == P - 1;
          bool cut_end = last && Q1 < np[lb + j + 1] - np0;
          for (int jj = 0; jj < K; jj++) {
            if (jj >= pd) { c0[jj] = c1[jj] = 0; continue; }
            uint32_t len = (uint32_t)(nd.c[jj + 1] - nd.c[jj]);
            c0[jj] = first ? cr[tile * K + jj] : 0;
            c1[jj] = cut_end ? cr[(tile + 1) * K + jj] : len;
            if (c1[jj] > len || c0[jj] > c1[jj]) {  // inconsistent cut: never index with it
              sm.misc[4] = 1;
              c0[jj] = c1[jj] = 0;
            }
            plen += c1[jj] - c0[jj];
          }
        }
        // exclusive scan of (slices, length) over the pieces: within each wave
        // by shuffles, then across the waves' totals
        const uint64_t packed = ((uint64_t)pd << 32) | plen;
        uint64_t incl = packed;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const uint64_t y = gshfl_up64(incl, o);
          if (lane >= o) incl += y;
        }
        if (lane == 63) sm.wsum[wave] = incl;
        __syncthreads();
        uint64_t ex = incl - packed, tot = 0;
        for (int w = 0; w < SM::kWaves; w++) {
          const uint64_t ws = sm.wsum[w];
          ex += w < wave ? ws : 0;
          tot += ws;
        }
        __syncthreads();
        if (p < P && carry_len + (ex & 0xFFFFFFFFull) + plen <= (uint64_t)Tt &&
            carry_sl + (ex >> 32) + pd < (uint64_t)SM::kMaxSlices) {
          uint64_t loff = carry_len + (ex & 0xFFFFFFFFull);
          uint64_t sl0 = carry_sl + (ex >> 32);
          sm.pc_loff[p] = (uint16_t)loff;
          sm.pc_sl[p] = (uint16_t)sl0;
          sm.pc_out[p] = nd.c[0] + (p == 0 ? Q0 - (np[lb + j0] - np0) : 0);
          uint64_t acc = loff;
          for (int jj = 0; jj < pd; jj++) {
            sm.sl_off[sl0 + jj] = (uint16_t)acc;
            sm.sl_pc[sl0 + jj] = (uint16_t)p;
            sl_g[sl0 + jj] = nd.c[jj] + c0[jj];
            acc += c1[jj] - c0[jj];
          }
        }
        carry_len += tot & 0xFFFFFFFFull;
        carry_sl += tot >> 32;
      }
      const int S = (int)carry_sl;
      if (carry_len != (uint64_t)Tt || S + 1 > SM::kMaxSlices) sm.misc[4] = 1;
      __syncthreads();
      if (t == 0 && !sm.misc[4]) {
        sm.pc_loff[P] = (uint16_t)Tt;
        sm.pc_sl[P] = (uint16_t)S;
        sm.sl_off[S] = (uint16_t)Tt;
      }
      __syncthreads();
      if (!sm.misc[4]) {
        // slice of every tile position: each non-empty slice marks its start,
        // then a running maximum over the positions (thread t owns E of them)
        const int b0 = t * E;
#pragma unroll
        for (int i = 0; i < E; i++)
          if (b0 + i < Tt) sm.pos_sl[b0 + i] = 0;
        lds_barrier();
        for (int s2 = t; s2 < S; s2 += THREADS)
          if (sm.sl_off[s2 + 1] > sm.sl_off[s2]) sm.pos_sl[sm.sl_off[s2]] = (uint16_t)s2;
        lds_barrier();
        uint32_t run = 0, rv[E];
#pragma unroll
        for (int i = 0; i < E; i++) {
          const uint32_t v = b0 + i < Tt ? sm.pos_sl[b0 + i] : 0u;
          run = v > run ? v : run;
          rv[i] = run;
        }
        uint32_t incl = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const uint32_t y = __shfl_up(incl, o);
          if (lane >= o) incl = y > incl ? y : incl;
        }
        if (lane == 63) sm.wsum[wave] = incl;
        uint32_t pre = __shfl_up(incl, 1);
        if (lane == 0) pre = 0;
        lds_barrier();
        for (int w = 0; w < wave; w++) {
          const uint32_t ws = (uint32_t)sm.wsum[w];
          pre = ws > pre ? ws : pre;
        }
#pragma unroll
        for (int i = 0; i < E; i++)
          if (b0 + i < Tt) sm.pos_sl[b0 + i] = (uint16_t)(rv[i] > pre ? rv[i] : pre);
        lds_barrier();
        O k2[E];
        V v2[E];
        addr_table<E, THREADS>(ga, sm.pos_sl, sm.sl_off, sl_g, Tt, t);
        issue_at<O, V, E, HV>(k2, v2, in_keys, in_vals, ga);
        lds_barrier();   // the slice starts, kept in the tile buffer, are read
        commit_loads<Kt, O, V, E, THREADS>(k2, v2, kA, vA, HV, Tt, t);
        lds_barrier();
        merge_stages_gen<O, V, K, TILE, THREADS, HV>(kA, vA, sm.sl_off, sm.pos_sl, sm.sl_pc,
                                                     sm.pc_sl, Tt, t);
        store_tile<Kt, O, V, E, THREADS>(kA, vA, out_keys, out_vals, HV, sm.pc_loff, sm.pc_out,
                                      sm.pos_sl, sm.sl_pc, Tt, t, smp);
      }
    }
    if (t == 0 && sm.misc[4]) atomicOr(&plan->error, 16u);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- host side
// Workgroups that fill the device once (CUs x resident workgroups per CU) for
// a queue-driven kernel; computed once per kernel and device.  The cache is a
// fixed table, so a launch allocates no host memory (a full table only means
// recomputing).
inline unsigned fill_grid(const void *kernel, int threads, unsigned fallback) {
  struct Entry {
    const void *kernel;
    int dev;
    unsigned grid;
  };
  constexpr int kSlots = 512;
  static std::mutex mu;
  static Entry tab[kSlots];
  static int used = 0;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fallback;
  std::lock_guard<std::mutex> lk(mu);
  for (int i = 0; i < used; i++)
    if (tab[i].kernel == kernel && tab[i].dev == dev) return tab[i].grid;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      cus <= 0 || per_cu <= 0)
    return fallback;
  const unsigned g = (unsigned)(cus * per_cu);
  if (used < kSlots) tab[used++] = Entry{kernel, dev, g};
  return g;
}

template <int KT, int K, int TILE, int THREADS, bool HV, typename V>
void launch_merges_v(const LevelArgs &a, const Work &w, const uint32_t *tj,
                     const uint64_t *tile_base, int level, hipStream_t s) {
  using U = typename Key<KT>::U;
  const TileTabFor<U, K> *desc = reinterpret_cast<const TileTabFor<U, K> *>(w.tile_desc);
  auto kf = k_merge_fast<KT, K, TILE, THREADS, HV, V>;
  auto kg = k_merge_general<KT, K, TILE, THREADS, HV, V>;
  unsigned gf = fill_grid((const void *)kf, THREADS, 1024);
  unsigned gg = fill_grid((const void *)kg, THREADS, 1024);
  const V *iv = reinterpret_cast<const V *>(a.in_vals);
  V *ov = reinterpret_cast<V *>(a.out_vals);
  hipLaunchKernelGGL(kf, dim3(gf), dim3(THREADS), 0, s, (const U *)a.in_keys, iv, (U *)a.out_keys,
                     ov, w.plan, level, desc, w.samples);
  hipLaunchKernelGGL(kg, dim3(gg), dim3(THREADS), 0, s, (const U *)a.in_keys, iv, (U *)a.out_keys,
                     ov, w.run_start, w.Ls, w.Rs, w.nd_mem, w.nd_arity, w.lvl_list, w.lvl_np, tj,
                     tile_base, w.plan, level, w.corank, w.gen_list, w.samples);
}

// The two merge launches of one level (descriptor tiles, then general tiles)
// for one tile configuration; the payload is absent, 4 or 8 bytes per key.
template <int KT, int K, int TILE, int THREADS>
void launch_merges_kt(const LevelArgs &a, const Work &w, const uint32_t *tj,
                      const uint64_t *tile_base, int level, hipStream_t s) {
  if (!a.in_vals)
    launch_merges_v<KT, K, TILE, THREADS, false, uint32_t>(a, w, tj, tile_base, level, s);
  else if (w.pay8)
    launch_merges_v<KT, K, TILE, THREADS, true, uint64_t>(a, w, tj, tile_base, level, s);
  else
    launch_merges_v<KT, K, TILE, THREADS, true, uint32_t>(a, w, tj, tile_base, level, s);
}

template <int TILE, int THREADS>
hipError_t launch_merges_cfg(int kt, const LevelArgs &a, const Work &w, const uint32_t *tj,
                             const uint64_t *tile_base, int level, hipStream_t s) {
  switch (w.k * 4 + kt) {
    case 2 * 4 + 0: launch_merges_kt<0, 2, TILE, THREADS>(a, w, tj, tile_base, level, s); break;
    case 2 * 4 + 1: launch_merges_kt<1, 2, TILE, THREADS>(a, w, tj, tile_base, level, s); break;
    case 2 * 4 + 2: launch_merges_kt<2, 2, TILE, THREADS>(a, w, tj, tile_base, level, s); break;
    case 4 * 4 + 0: launch_merges_kt<0, 4, TILE, THREADS>(a, w, tj, tile_base, level, s); break;
    case 4 * 4 + 1: launch_merges_kt<1, 4, TILE, THREADS>(a, w, tj, tile_base, level, s); break;
    case 4 * 4 + 2: launch_merges_kt<2, 4, TILE, THREADS>(a, w, tj, tile_base, level, s); break;
    case 8 * 4 + 0: launch_merges_kt<0, 8, TILE, THREADS>(a, w, tj, tile_base, level, s); break;
    case 8 * 4 + 1: launch_merges_kt<1, 8, TILE, THREADS>(a, w, tj, tile_base, level, s); break;
    case 8 * 4 + 2: launch_merges_kt<2, 8, TILE, THREADS>(a, w, tj, tile_base, level, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mps
