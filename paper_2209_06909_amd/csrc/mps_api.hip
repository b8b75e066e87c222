// mps_api.hip -- host planner and C ABI of libmps.
//
// A sort is a fixed sequence of launches on one stream; every data-dependent
// quantity (run count, node counts per level, tiles per level) lives in the
// device-resident Plan and is read by the kernels themselves, so a sort
// enqueues without any host synchronisation (and can be captured in a HIP
// graph).  Levels are launched for every depth the powers allow; levels
// deeper than the actual tree find zero tiles and return at once.
#include <mutex>
#include <tuple>
#include <vector>
#include <map>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "mps.h"
#include "mps_internal.h"

namespace mps {

// Zero the plan and (for single-array calls) write the 2-entry offsets.
// init_error presets the plan's error word (testing: a reported device error
// on a sort that otherwise runs normally).
__global__ void k_init(Plan *plan, uint64_t *seg_off, uint64_t n, uint64_t m, uint32_t kt,
                       uint32_t has_payload, uint32_t k, int single, uint32_t init_error) {
  uint64_t *p = reinterpret_cast<uint64_t *>(plan);
  for (size_t i = threadIdx.x; i < sizeof(Plan) / 8; i += blockDim.x) p[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    plan->n = n;
    plan->m = m;
    plan->kt = kt;
    plan->has_payload = has_payload;
    plan->k = k;
    plan->error = init_error;
    if (single) {
      seg_off[0] = 0;
      seg_off[1] = n;
    }
  }
}

// The last launch of a sort that was given an error word: ORs the plan's
// device-side check results into it (sticky across sorts).
__global__ void k_report(const Plan *plan, uint32_t *error_out) {
  if (threadIdx.x == 0 && plan->error) atomicOr(error_out, plan->error);
}


__global__ void k_check_offsets(const uint64_t *off, uint64_t m, uint64_t total, Plan *plan) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t a = off[i], b = off[i + 1];
    bool bad = b < a || (b - a) > (1ull << 31) || (i == 0 && a != 0) || (i + 1 == m && b != total);
    if (bad) atomicOr(&plan->error, 2u);
  }
}

}  // namespace mps

using namespace mps;

// ---------------------------------------------------------------- errors
// The calling thread's last message, in a fixed buffer: reporting an error
// allocates nothing.
static thread_local char g_err[512];

static int fail(int code, const char *msg) {
  snprintf(g_err, sizeof g_err, "%s", msg);
  return code;
}

__attribute__((format(printf, 2, 3))) static int failf(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) return failf(MPS_E_HIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

extern "C" const char *mps_last_error(void) { return g_err; }

int mps::fail_msg(int code, const char *msg) { return fail(code, msg); }

// ---------------------------------------------------------------- layout
namespace {

struct Layout {
  size_t total = 0;
  size_t alt_keys, alt_vals, seg_off, seg_bits, dbits, det_agg, det_zin, det_off, run_start, run_desc,
      power, ansv_bl, ansv_bf, ansv_cl, ansv_cr, ansv_tl, ansv_tr, Ls, Rs, Le, Re, nd_arity, nd_mem, jump0, jump1,
      dist0, dist1, leaf_depth, sflag, pflag, jlist, cfirst, croot, lvl_cnt, lvl_car, lvl_tot, lvl_list, lvl_np, scan_tmp, corank, tile_desc, gen_list, tile_base,
      tj, samples, plan, nat_start, nat_desc, mr_first, mr_nxt, mr_cnt, mr_gnxt, mr_gcnt,
      mr_gentry, mr_goff, mr_centry, mr_coff;
  uint64_t rmax, nbb, tiles_max, tj_cap, lvl_cap;
  int levels;
  bool tree_tmp_in_alt;   // Le, Re, jump0/1, dist1 share the ping-pong buffer's bytes
  bool jlist_in_alt;      // so does the pointer-jumping list
};

size_t take(size_t &cur, size_t bytes) {
  size_t at = (cur + 255) & ~(size_t)255;
  cur = at + bytes;
  return at;
}

int levels_for(uint64_t n, uint32_t k) {
  // every power satisfies k^(P-1) < 2n, so depths are < P <= this bound
  int p = 0;
  unsigned __int128 v = 1;
  while (v < (unsigned __int128)2 * n) {
    v *= k;
    p++;
  }
  return p < 1 ? 1 : p;
}

// The ping-pong buffer (alt_keys, alt_vals) is first written by placement,
// after the tree is built.  Until then its bytes hold, when they fit, arrays
// that die earlier: the natural runs of a minimal-run-length sort (dead once
// the extended runs are made) and then the tree's scratch -- the nearest
// smaller-or-equal boundaries Le / Re and the pointer-jumping buffers -- (dead
// once the level lists and leaf depths are built; a trace fetched later
// rebuilds them from the powers).  The level lists hold only nodes spanning
// more than kSmallSpan elements: nodes of one depth are disjoint, so at most
// N / (kSmallSpan + 1) per depth.
bool make_layout(uint64_t N, uint64_t m, int kt, int pb, uint32_t k, Layout &L) {
  if (N == 0 || m == 0) return false;
  size_t ks = kt == MPS_I64 ? 8 : 4;
  uint64_t rmax = N / 2 + m + 2;
  if (rmax > N + 1) rmax = N + 1;
  uint64_t nwords = (N + 63) / 64;
  uint64_t nblk = (N + 16383) / 16384;
  uint64_t nbb = (rmax + 1 + 1023) / 1024 + 1;
  uint64_t tiles_max = N / kTileMin + 2;   // enough for every tile configuration
  int levels = levels_for(N, k);
  if (levels >= kMaxLevels) return false;
  uint64_t lvl_cap = (uint64_t)levels * (N / (kSmallSpan + 1) + m) + 2;
  if (lvl_cap > rmax) lvl_cap = rmax;
  size_t c = 0;
  L.plan = take(c, sizeof(Plan));    // first: a later trace fetch finds it at the base
  L.alt_keys = take(c, N * ks);
  L.alt_vals = take(c, N * (uint64_t)pb);   // pb: payload bytes per key (0, 4 or 8)
  const size_t alt_end = c;
  // the tree's scratch inside the ping-pong buffer if it fits there
  {
    size_t t = L.alt_keys;
    const size_t le = take(t, (rmax + 1) * 4), re = take(t, (rmax + 1) * 4);
    const size_t j0 = take(t, (rmax + 1) * 4), j1 = take(t, (rmax + 1) * 4);
    const size_t d1 = take(t, rmax + 1);
    L.tree_tmp_in_alt = t <= alt_end;
    if (L.tree_tmp_in_alt) {
      L.Le = le;
      L.Re = re;
      L.jump0 = j0;
      L.jump1 = j1;
      L.dist1 = d1;
    }
    // the pointer-jumping list, after them, or alone at the start
    size_t tl = L.tree_tmp_in_alt ? t : L.alt_keys;
    const size_t jl = take(tl, (rmax + 1) * 4);
    L.jlist_in_alt = tl <= alt_end;
    if (L.jlist_in_alt) L.jlist = jl;
  }
  bool nat_in_alt = false;
  if (m == 1) {
    size_t t = L.alt_keys;
    const size_t ns = take(t, (rmax + 1) * 8), nd = take(t, rmax);
    nat_in_alt = t <= alt_end;
    if (nat_in_alt) {
      L.nat_start = ns;
      L.nat_desc = nd;
    }
  }
  L.seg_off = take(c, 16);
  L.seg_bits = take(c, m > 1 ? nwords * 8 + 8 : 0);
  L.dbits = take(c, nwords * 8 + 8);
  L.det_agg = take(c, nblk * sizeof(DetAgg));
  L.det_zin = take(c, nblk * 8);
  L.det_off = take(c, nblk * 8);
  L.run_start = take(c, (rmax + 1) * 8);
  L.run_desc = take(c, rmax);
  L.power = take(c, rmax + 1);
  L.ansv_bl = take(c, nbb * kVMax * 4);
  L.ansv_bf = take(c, nbb * kVMax * 4);
  L.ansv_cl = take(c, nbb * kVMax * 4);
  L.ansv_cr = take(c, nbb * kVMax * 4);
  L.ansv_tl = take(c, (nbb / 1024 + 1) * kVMax * 4);   // chunks of 1024 blocks
  L.ansv_tr = take(c, (nbb / 1024 + 1) * kVMax * 4);
  L.Ls = take(c, (rmax + 1) * 4);
  L.Rs = take(c, (rmax + 1) * 4);
  if (!L.tree_tmp_in_alt) {
    L.Le = take(c, (rmax + 1) * 4);
    L.Re = take(c, (rmax + 1) * 4);
  }
  L.nd_arity = take(c, rmax + 1);
  L.nd_mem = take(c, (rmax + 1) * (k - 1) * 4);
  if (!L.tree_tmp_in_alt) {
    L.jump0 = take(c, (rmax + 1) * 4);
    L.jump1 = take(c, (rmax + 1) * 4);
  }
  L.dist0 = take(c, rmax + 1);
  if (!L.tree_tmp_in_alt) L.dist1 = take(c, rmax + 1);
  L.leaf_depth = take(c, rmax);
  L.sflag = take(c, rmax + 17);   // read 16 flags at a time
  if (!L.jlist_in_alt) L.jlist = take(c, (rmax + 1) * 4);
  L.pflag = take(c, (N / kPlaceBlock + 2) * 4);
  L.cfirst = take(c, (N / kLeafChunk + 2) * 4);
  L.croot = take(c, (N / kLeafChunk + 2) * kChunkRec * 4);
  L.lvl_cnt = take(c, nbb * kMaxLevels * 4);
  L.lvl_car = take(c, (nbb / 1024 + 1) * kMaxLevels * 4);
  L.lvl_tot = take(c, kMaxLevels * 8);
  L.lvl_list = take(c, lvl_cap * 4);
  L.lvl_np = take(c, (lvl_cap + 2) * 8);
  L.scan_tmp = take(c, (lvl_cap / 1024 + 2) * 8);
  L.corank = take(c, tiles_max * k * 4);
  L.tile_desc = take(c, tiles_max * kTileDescBytes);
  L.gen_list = take(c, tiles_max * 4);
  L.samples = take(c, (N / kSampleStride + 2) * 8);
  L.tile_base = take(c, (kMaxLevels + 1) * 8);
  L.tj_cap = (tiles_max + 1) * (uint64_t)levels + 64;
  L.tj = take(c, L.tj_cap * 4);
  // single arrays may ask for a minimal run length: room for the natural runs
  // and the chunk maps that turn them into extended runs
  const uint64_t nch = m == 1 ? (N + kMrChunk - 1) / kMrChunk : 0;
  const uint64_t ng = (nch + kMrGroup - 1) / kMrGroup;
  if (!nat_in_alt) {
    L.nat_start = take(c, m == 1 ? (rmax + 1) * 8 : 0);
    L.nat_desc = take(c, m == 1 ? rmax : 0);
  }
  L.mr_first = take(c, (nch + 1) * 4);
  L.mr_nxt = take(c, nch * kMrCand);
  L.mr_cnt = take(c, nch * kMrCand * 2);
  L.mr_gnxt = take(c, ng * kMrCand);
  L.mr_gcnt = take(c, ng * kMrCand * 4);
  L.mr_gentry = take(c, ng);
  L.mr_goff = take(c, ng * 4);
  L.mr_centry = take(c, nch);
  L.mr_coff = take(c, nch * 4);
  L.total = c + 256;
  L.rmax = rmax;
  L.nbb = nbb;
  L.tiles_max = tiles_max;
  L.lvl_cap = lvl_cap;
  L.levels = levels;
  return true;
}

// Defaults of the zero-valued option fields, overridable from the environment:
// MPS_K (2, 4 or 8), MPS_TILE (1024, 2048 or 4096) and MPS_LANE_SLICE (4 or 8).
// Read once; an unparsable or unsupported value is ignored.
struct EnvDefaults {
  uint32_t k = 4, tile = (uint32_t)kTileDefault, lane_slice = 4;
  EnvDefaults() {
    auto num = [](const char *name) -> long {
      const char *v = getenv(name);
      if (!v || !*v) return -1;
      char *end = nullptr;
      long x = strtol(v, &end, 10);
      return (end && *end == 0) ? x : -1;
    };
    long x = num("MPS_K");
    if (x == 2 || x == 4 || x == 8) k = (uint32_t)x;
    x = num("MPS_TILE");
    if (x == 1024 || x == 2048 || x == 4096) tile = (uint32_t)x;
    x = num("MPS_LANE_SLICE");
    if (x == 4 || x == 8) lane_slice = (uint32_t)x;
  }
};
const EnvDefaults &env_defaults() {
  static const EnvDefaults d;
  return d;
}

int check_k(uint32_t &k) {
  if (k == 0) k = env_defaults().k;
  if (k != 2 && k != 4 && k != 8)
    return fail(MPS_E_UNSUPPORTED, "k must be 2, 4 or 8");
  return MPS_OK;
}

// Library-managed workspaces, one per (device, stream), grown on demand.  A
// stream runs its sorts one after another, so sorts on one stream never share
// a workspace with sorts still running on another.  Growing waits for the
// stream (its earlier sorts may still use the old allocation) before freeing.
struct WsKey {
  int dev;
  hipStream_t s;
  bool operator<(const WsKey &o) const { return std::tie(dev, s) < std::tie(o.dev, o.s); }
};
std::mutex g_ws_mu;
std::map<WsKey, std::pair<void *, size_t>> g_ws;

int get_workspace(size_t need, hipStream_t s, void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto &e = g_ws[WsKey{dev, s}];
  if (e.second < need) {
    if (e.first) {
      HIP_TRY(hipStreamSynchronize(s));
      HIP_TRY(hipFree(e.first));
      e.first = nullptr;
      e.second = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) return fail(MPS_E_NOMEM, "workspace allocation failed");
    e.first = p;
    e.second = need;
  }
  *out = e.first;
  return MPS_OK;
}

// The library-managed workspace of (current device, s), or nullptr.
void *find_workspace(hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto it = g_ws.find(WsKey{dev, s});
  if (it == g_ws.end() || !it->second.first) return nullptr;
  return reinterpret_cast<void *>((reinterpret_cast<uintptr_t>(it->second.first) + 255) & ~(uintptr_t)255);
}

template <typename T> T *at(void *base, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

// Device views of the workspace at `base` (laid out by L).
void bind_work(Work &w, void *base, const Layout &L, uint64_t N, uint64_t m, uint32_t k, int tile,
               int threads, int pb, const uint64_t *d_off) {
  w.N = N;
  w.m = m;
  w.rmax = L.rmax;
  w.k = (int)k;
  w.logk = k == 2 ? 1 : (k == 4 ? 2 : 3);
  w.tile = tile;
  w.threads = threads;
  w.alt_keys = at<void>(base, L.alt_keys);
  w.alt_vals = pb ? at<uint32_t>(base, L.alt_vals) : nullptr;
  w.pay8 = pb == 8 ? 1 : 0;
  w.seg_off_local = at<uint64_t>(base, L.seg_off);
  w.off = d_off ? d_off : w.seg_off_local;
  w.seg_bits = m > 1 ? at<uint64_t>(base, L.seg_bits) : nullptr;
  w.dbits = at<uint64_t>(base, L.dbits);
  w.det_agg = at<DetAgg>(base, L.det_agg);
  w.det_zin = at<uint64_t>(base, L.det_zin);
  w.det_off = at<uint64_t>(base, L.det_off);
  w.run_start = at<uint64_t>(base, L.run_start);
  w.run_desc = at<uint8_t>(base, L.run_desc);
  if (m == 1) {
    w.nat_start = at<uint64_t>(base, L.nat_start);
    w.nat_desc = at<uint8_t>(base, L.nat_desc);
    w.mr_first = at<uint32_t>(base, L.mr_first);
    w.mr_nxt = at<uint8_t>(base, L.mr_nxt);
    w.mr_cnt = at<uint16_t>(base, L.mr_cnt);
    w.mr_gnxt = at<uint8_t>(base, L.mr_gnxt);
    w.mr_gcnt = at<uint32_t>(base, L.mr_gcnt);
    w.mr_gentry = at<uint8_t>(base, L.mr_gentry);
    w.mr_goff = at<uint32_t>(base, L.mr_goff);
    w.mr_centry = at<uint8_t>(base, L.mr_centry);
    w.mr_coff = at<uint32_t>(base, L.mr_coff);
  }
  w.power = at<uint8_t>(base, L.power);
  w.ansv_bl = at<uint32_t>(base, L.ansv_bl);
  w.ansv_bf = at<uint32_t>(base, L.ansv_bf);
  w.ansv_cl = at<uint32_t>(base, L.ansv_cl);
  w.ansv_cr = at<uint32_t>(base, L.ansv_cr);
  w.ansv_tl = at<uint32_t>(base, L.ansv_tl);
  w.ansv_tr = at<uint32_t>(base, L.ansv_tr);
  w.Ls = at<uint32_t>(base, L.Ls);
  w.Rs = at<uint32_t>(base, L.Rs);
  w.Le = at<uint32_t>(base, L.Le);
  w.Re = at<uint32_t>(base, L.Re);
  w.nd_arity = at<uint8_t>(base, L.nd_arity);
  w.nd_mem = at<uint32_t>(base, L.nd_mem);
  w.jump0 = at<uint32_t>(base, L.jump0);
  w.jump1 = at<uint32_t>(base, L.jump1);
  w.dist0 = at<uint8_t>(base, L.dist0);
  w.dist1 = at<uint8_t>(base, L.dist1);
  w.leaf_depth = at<uint8_t>(base, L.leaf_depth);
  w.sflag = at<uint8_t>(base, L.sflag);
  w.jlist = at<uint32_t>(base, L.jlist);
  w.pflag = at<uint32_t>(base, L.pflag);
  w.cfirst = at<uint32_t>(base, L.cfirst);
  w.croot = at<uint32_t>(base, L.croot);
  w.lvl_cnt = at<uint32_t>(base, L.lvl_cnt);
  w.lvl_car = at<uint32_t>(base, L.lvl_car);
  w.lvl_list = at<uint32_t>(base, L.lvl_list);
  w.lvl_cap = L.lvl_cap;
  w.lvl_np = at<uint64_t>(base, L.lvl_np);
  w.scan_tmp = at<uint64_t>(base, L.scan_tmp);
  w.corank = at<uint32_t>(base, L.corank);
  w.tile_desc = at<void>(base, L.tile_desc);
  w.gen_list = at<uint32_t>(base, L.gen_list);
  w.samples = at<uint64_t>(base, L.samples);
  w.plan = at<Plan>(base, L.plan);
}

// Copies the trace of the sort that last used the workspace at `base`.
int fill_trace(void *base, mps_trace *tr) {
  Plan plan;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(&plan, base, sizeof(Plan), hipMemcpyDeviceToHost));
  if (plan.error)
    return failf(MPS_E_DEVICE, "device-side consistency check failed (error word 0x%x)", plan.error);
  if (plan.n >= 2 && plan.r > 1) {
    Layout L;
    if (!make_layout(plan.n, plan.m, (int)plan.kt, (int)plan.has_payload, plan.k, L))
      return fail(MPS_E_DEVICE, "workspace header does not describe a layout");
    if (plan.lean || L.tree_tmp_in_alt) {
      // the merges reused the tree's scratch, or the sort left the insides of
      // its small subtrees out: rebuild them from the powers
      Work w{};
      bind_work(w, base, L, plan.n, plan.m, plan.k, 0, 0, (int)plan.has_payload, nullptr);
      HIP_TRY(launch_tree_complete(w, plan.lean != 0, (unsigned)(L.nbb < 4096 ? L.nbb : 4096), nullptr));
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipMemcpy(&plan, base, sizeof(Plan), hipMemcpyDeviceToHost));
      if (plan.error)
        return failf(MPS_E_DEVICE, "device-side consistency check failed (error word 0x%x)", plan.error);
    }
  }
  tr->r = plan.r;
  tr->n_nodes = plan.n_nodes;
  tr->merge_cost = plan.merge_cost;
  tr->n_levels = plan.n_levels;
  tr->k = plan.k;
  Layout L;
  if (plan.n < 2 || !make_layout(plan.n, plan.m, (int)plan.kt, (int)plan.has_payload, plan.k, L))
    return MPS_OK;
  const uint64_t r = plan.r;
  bool want_runs = tr->run_start || tr->run_desc || tr->power || tr->leaf_depth;
  bool want_nodes = tr->node_begin || tr->node_end || tr->node_first || tr->node_arity ||
                    tr->node_power || tr->node_depth;
  if (!want_runs && !want_nodes) return MPS_OK;
  if (tr->r_cap < r + 1)
    return failf(MPS_E_NOMEM, "trace r_cap too small (need r+1 = %llu)", (unsigned long long)(r + 1));
  std::vector<uint64_t> rs(r + 1);
  HIP_TRY(hipMemcpy(rs.data(), at<uint64_t>(base, L.run_start), (r + 1) * 8, hipMemcpyDeviceToHost));
  std::vector<uint8_t> P(r + 1);
  HIP_TRY(hipMemcpy(P.data(), at<uint8_t>(base, L.power), r + 1, hipMemcpyDeviceToHost));
  if (tr->run_start) memcpy(tr->run_start, rs.data(), (r + 1) * 8);
  if (tr->run_desc && r) HIP_TRY(hipMemcpy(tr->run_desc, at<uint8_t>(base, L.run_desc), r, hipMemcpyDeviceToHost));
  if (tr->power && r > 1) memcpy(tr->power, P.data() + 1, r - 1);
  if (tr->leaf_depth && r) {
    HIP_TRY(hipMemcpy(tr->leaf_depth, at<uint8_t>(base, L.leaf_depth), r, hipMemcpyDeviceToHost));
    for (uint64_t j = 0; j < r; j++) tr->leaf_depth[j] &= (uint8_t)~kLeafInSmall;
  }
  if (want_nodes && r > 1) {
    std::vector<uint32_t> Ls(r + 1), Rs(r + 1), Le(r + 1);
    std::vector<uint8_t> ar(r + 1), dep(r + 1);
    HIP_TRY(hipMemcpy(Ls.data(), at<uint32_t>(base, L.Ls), (r + 1) * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(Rs.data(), at<uint32_t>(base, L.Rs), (r + 1) * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(Le.data(), at<uint32_t>(base, L.Le), (r + 1) * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ar.data(), at<uint8_t>(base, L.nd_arity), r + 1, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(dep.data(), at<uint8_t>(base, L.dist0), r + 1, hipMemcpyDeviceToHost));
    uint64_t c = 0;
    for (uint64_t i = 1; i < r; i++) {
      if (P[i] == 0 || P[Le[i]] >= P[i]) continue;  // group leaders are the nodes
      if (c >= tr->r_cap) return fail(MPS_E_NOMEM, "trace r_cap too small for nodes");
      if (tr->node_begin) tr->node_begin[c] = rs[Ls[i]];
      if (tr->node_end) tr->node_end[c] = rs[Rs[i]];
      if (tr->node_first) tr->node_first[c] = (uint32_t)i;
      if (tr->node_arity) tr->node_arity[c] = ar[i];
      if (tr->node_power) tr->node_power[c] = P[i];
      if (tr->node_depth) tr->node_depth[c] = dep[i];
      c++;
    }
    if (c != plan.n_nodes) return fail(MPS_E_DEVICE, "node count mismatch in trace");
  }
  return MPS_OK;
}

void *g_last_base[64];  // library-managed workspace base per device (for mps_trace_fetch)

// Per-device record of the last sort that asked for level timing.
struct LevelTiming {
  std::vector<hipEvent_t> ev;  // 3 per level: before co-rank, before merge, after merge
  int levels = 0;
  void *base = nullptr;        // its workspace (holds the plan)
};
std::mutex g_time_mu;
LevelTiming g_time[64];

// The launch sequence of one sort on stream s (also what a graph captures).
int enqueue_sort(void *keys, int kt, uint32_t *payload, const uint64_t *d_off, const Work &w,
                 const Layout &L, uint64_t *lvl_tot, uint64_t *tile_base, uint32_t *tj,
                 int want_cost, LevelTiming *tm, uint32_t init_error, uint32_t *error_out,
                 hipStream_t s) {
  const unsigned gtree = (unsigned)(L.nbb < 4096 ? L.nbb : 4096);
  hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, s, w.plan, w.seg_off_local, w.N, w.m,
                     (uint32_t)kt, payload ? (w.pay8 ? 8u : 4u) : 0u, (uint32_t)w.k, d_off ? 0 : 1,
                     init_error);
  if (d_off)
    hipLaunchKernelGGL(k_check_offsets, dim3(64), dim3(256), 0, s, d_off, w.m, w.N, w.plan);
  HIP_TRY(hipGetLastError());
  if (w.min_run > 1) {
    // natural runs into their own arrays, then the extended runs
    Work wn = w;
    wn.run_start = w.nat_start;
    wn.run_desc = w.nat_desc;
    HIP_TRY(launch_detect(kt, keys, wn, s));
    HIP_TRY(launch_minrun(kt, keys, payload, w, s));
  } else {
    HIP_TRY(launch_detect(kt, keys, w, s));
  }
  HIP_TRY(launch_tree(w, want_cost, lvl_tot, tile_base, tj, gtree, s));
  HIP_TRY(hipGetLastError());
  if (w.min_run > 1) HIP_TRY(launch_minrun_sort(kt, keys, payload, w, s));
  HIP_TRY(launch_place(kt, keys, payload, w, s));
  HIP_TRY(launch_leaf(kt, keys, payload, w, s));
  for (int d = L.levels - 1; d >= 0; d--) {
    LevelArgs a;
    bool out_user = (d & 1) == 0;
    a.in_keys = out_user ? w.alt_keys : keys;
    a.in_vals = payload ? (out_user ? w.alt_vals : payload) : nullptr;
    a.out_keys = out_user ? keys : w.alt_keys;
    a.out_vals = payload ? (out_user ? payload : w.alt_vals) : nullptr;
    if (tm) {
      HIP_TRY(launch_level_timed(kt, a, w, tj, tile_base, d, s, tm->ev[3 * d], tm->ev[3 * d + 1],
                                 tm->ev[3 * d + 2]));
    } else {
      HIP_TRY(launch_level(kt, a, w, tj, tile_base, d, s));
    }
  }
  if (error_out) {
    hipLaunchKernelGGL(k_report, dim3(1), dim3(64), 0, s, (const Plan *)w.plan, error_out);
    HIP_TRY(hipGetLastError());
  }
  return MPS_OK;
}

// ---------------------------------------------------------------- graphs
// Instantiated graphs of whole sorts, keyed by every argument that shapes the
// launch sequence.  Captured on a library stream (capture only records), then
// launched on the caller's stream.
struct GraphKey {
  int dev, kt, k, tile, threads, want_cost, min_run, merge_down, pb;
  uint32_t init_error;
  const void *keys, *payload, *off, *base, *error_out;
  uint64_t m, N;
  bool operator<(const GraphKey &o) const {
    return std::tie(dev, kt, k, tile, threads, want_cost, min_run, merge_down, pb, init_error,
                    keys, payload, off, base, error_out, m, N) <
           std::tie(o.dev, o.kt, o.k, o.tile, o.threads, o.want_cost, o.min_run, o.merge_down,
                    o.pb, o.init_error, o.keys, o.payload, o.off, o.base, o.error_out, o.m, o.N);
  }
};
std::mutex g_graph_mu;
std::map<GraphKey, hipGraphExec_t> g_graphs;
hipStream_t g_capture_stream[64];
constexpr size_t kMaxGraphs = 256;

int graph_launch(const GraphKey &key, void *keys, int kt, uint32_t *payload,
                 const uint64_t *d_off, const Work &w, const Layout &L, uint64_t *lvl_tot,
                 uint64_t *tile_base, uint32_t *tj, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto it = g_graphs.find(key);
  if (it == g_graphs.end()) {
    if (key.dev < 0 || key.dev >= 64) return fail(MPS_E_UNSUPPORTED, "device index out of range");
    hipStream_t &cs = g_capture_stream[key.dev];
    if (!cs) HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    if (g_graphs.size() >= kMaxGraphs) {
      for (auto &e : g_graphs) (void)hipGraphExecDestroy(e.second);
      g_graphs.clear();
    }
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    int rc = enqueue_sort(keys, kt, payload, d_off, w, L, lvl_tot, tile_base, tj, key.want_cost,
                          nullptr, key.init_error, (uint32_t *)key.error_out, cs);
    hipGraph_t g = nullptr;
    hipError_t ec = hipStreamEndCapture(cs, &g);
    if (rc != MPS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return failf(MPS_E_HIP, "graph capture: %s", hipGetErrorString(ec));
    hipGraphExec_t ge = nullptr;
    hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return failf(MPS_E_HIP, "graph instantiate: %s", hipGetErrorString(ei));
    it = g_graphs.emplace(key, ge).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, s));
  return MPS_OK;
}

int resolve_tile(const mps_opts *opts, int &tile, int &threads) {
  const EnvDefaults &ed = env_defaults();
  uint32_t t = opts && opts->tile ? opts->tile : ed.tile;
  uint32_t e = opts ? opts->lane_slice : 0;
  if (e == 0) e = opts && opts->tile ? 4 : ed.lane_slice;
  if (!tile_config_ok((int)t, (int)(t / e))) {
    // an environment default that does not pair with the tile falls back to 4
    if (!(opts && opts->lane_slice)) e = 4;
  }
  if (t != 1024 && t != 2048 && t != 4096) return fail(MPS_E_UNSUPPORTED, "tile must be 1024, 2048 or 4096");
  if (e != 4 && e != 8) return fail(MPS_E_UNSUPPORTED, "lane_slice must be 4 or 8");
  if (!tile_config_ok((int)t, (int)(t / e)))
    return fail(MPS_E_UNSUPPORTED,
                "unsupported tile / lane_slice pair (1024/4, 2048/8, 2048/4, 4096/8, 4096/4)");
  tile = (int)t;
  threads = (int)(t / e);
  return MPS_OK;
}

// pb: payload bytes per key when payload is not NULL (4, or 8 for records).
int run_sort(void *keys, int kt, uint32_t *payload, const uint64_t *d_off, uint64_t m,
             uint64_t N, const mps_opts *opts, mps_trace *trace, hipStream_t s, int pb = 4) {
  if (!payload) pb = 0;
  uint32_t k = opts ? opts->k : 0;
  int rc = check_k(k);
  if (rc) return rc;
  int tile = 0, threads = 0;
  rc = resolve_tile(opts, tile, threads);
  if (rc) return rc;
  const uint32_t flags = opts ? opts->flags : 0;
  const uint32_t min_run = opts && opts->min_run > 1 ? opts->min_run : 1;
  if (min_run > (uint32_t)kMrMaxMinRun)
    return failf(MPS_E_UNSUPPORTED, "min_run above %d", kMrMaxMinRun);
  if (min_run > 1 && m > 1)
    return fail(MPS_E_UNSUPPORTED, "a minimal run length applies to single-array sorts only");
  if ((flags & MPS_OPT_MERGE_DOWN) && m > 1)
    return fail(MPS_E_UNSUPPORTED, "MPS_OPT_MERGE_DOWN applies to single-array sorts only");
  if ((flags & MPS_OPT_GRAPH) && (flags & MPS_OPT_TIME_LEVELS))
    return fail(MPS_E_INVALID, "MPS_OPT_GRAPH cannot be combined with MPS_OPT_TIME_LEVELS");
  Layout L;
  if (!make_layout(N, m, kt, pb, k, L)) return fail(MPS_E_INVALID, "bad sizes");
  void *base = nullptr;
  if (opts && opts->workspace) {
    if (opts->workspace_bytes < L.total)
      return failf(MPS_E_NOMEM, "workspace too small: need %llu bytes", (unsigned long long)L.total);
    base = opts->workspace;
  } else {
    rc = get_workspace(L.total, s, &base);
    if (rc) return rc;
  }
  base = reinterpret_cast<void *>((reinterpret_cast<uintptr_t>(base) + 255) & ~(uintptr_t)255);

  Work w{};
  bind_work(w, base, L, N, m, k, tile, threads, pb, d_off);
  w.min_run = (int)min_run;
  w.merge_down = (flags & MPS_OPT_MERGE_DOWN) ? 1 : 0;
  uint64_t *lvl_tot = at<uint64_t>(base, L.lvl_tot);
  uint64_t *tile_base = at<uint64_t>(base, L.tile_base);
  uint32_t *tj = at<uint32_t>(base, L.tj);
  const int want_cost = trace ? 1 : 0;
  const uint32_t init_error = (flags & MPS_OPT_TEST_DEVICE_ERROR) ? kErrTestForced : 0u;
  uint32_t *error_out = opts ? opts->error_out : nullptr;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));

  if (flags & MPS_OPT_GRAPH) {
    GraphKey key{dev, kt, (int)k, tile, threads, want_cost, w.min_run, w.merge_down, pb, init_error,
                 keys, payload, d_off, base, error_out, m, N};
    rc = graph_launch(key, keys, kt, payload, d_off, w, L, lvl_tot, tile_base, tj, s);
    if (rc) return rc;
  } else {
    LevelTiming *tm = nullptr;
    std::unique_lock<std::mutex> tlk(g_time_mu, std::defer_lock);
    if (flags & MPS_OPT_TIME_LEVELS) {
      if (dev < 0 || dev >= 64) return fail(MPS_E_UNSUPPORTED, "device index out of range");
      tlk.lock();
      tm = &g_time[dev];
      while (tm->ev.size() < (size_t)L.levels * 3) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        tm->ev.push_back(e);
      }
      tm->levels = L.levels;
      tm->base = base;
    }
    rc = enqueue_sort(keys, kt, payload, d_off, w, L, lvl_tot, tile_base, tj, want_cost, tm,
                      init_error, error_out, s);
    if (rc) return rc;
  }
  if (!(opts && opts->workspace) && dev >= 0 && dev < 64) g_last_base[dev] = base;
  if (trace) return fill_trace(base, trace);
  return MPS_OK;
}

}  // namespace

// ---------------------------------------------------------------- C entry points
extern "C" uint64_t mps_workspace_bytes(uint64_t n, uint64_t m, mps_key_type kt, int has_payload,
                                        uint32_t k) {
  if (k == 0) k = 4;
  if (k != 2 && k != 4 && k != 8) return 0;
  if (kt != MPS_I32 && kt != MPS_I64 && kt != MPS_F32) return 0;
  if (has_payload < 0 || has_payload > 2 || (has_payload == 2 && m > 1)) return 0;
  Layout L;
  if (!make_layout(n < 2 ? 2 : n, m < 1 ? 1 : m, kt, has_payload == 2 ? 8 : (has_payload ? 4 : 0), k, L))
    return 0;
  return L.total;
}

extern "C" int mps_sort_ex(void *keys, mps_key_type kt, uint32_t *payload, uint64_t n,
                           const mps_opts *opts, mps_trace *trace, void *stream) {
  g_err[0] = 0;
  if (kt != MPS_I32 && kt != MPS_I64 && kt != MPS_F32) return fail(MPS_E_INVALID, "unknown key type");
  if (n > 0 && !keys) return fail(MPS_E_INVALID, "keys is NULL");
  if (n > (1ull << 31)) return fail(MPS_E_UNSUPPORTED, "arrays longer than 2^31 are not supported");
  if (n <= 1) {
    if (trace) {
      uint32_t k = opts && opts->k ? opts->k : 4;
      trace->r = n;
      trace->n_nodes = 0;
      trace->merge_cost = 0;
      trace->n_levels = 0;
      trace->k = k;
      if (n == 1) {
        if (trace->r_cap < 2 && (trace->run_start || trace->run_desc || trace->leaf_depth))
          return fail(MPS_E_NOMEM, "trace r_cap too small");
        if (trace->run_start) { trace->run_start[0] = 0; trace->run_start[1] = 1; }
        if (trace->run_desc) trace->run_desc[0] = 0;
        if (trace->leaf_depth) trace->leaf_depth[0] = 0;
      } else if (trace->run_start && trace->r_cap >= 1) {
        trace->run_start[0] = 0;
      }
    }
    return MPS_OK;
  }
  return run_sort(keys, kt, payload, nullptr, 1, n, opts, trace, (hipStream_t)stream);
}

extern "C" int mps_sort_kv64(void *keys, mps_key_type kt, uint64_t *payload, uint64_t n,
                             const mps_opts *opts, mps_trace *trace, void *stream) {
  g_err[0] = 0;
  if (!payload || n <= 1) return mps_sort_ex(keys, kt, nullptr, n, opts, trace, stream);
  if (kt != MPS_I32 && kt != MPS_I64 && kt != MPS_F32) return fail(MPS_E_INVALID, "unknown key type");
  if (!keys) return fail(MPS_E_INVALID, "keys is NULL");
  if (n > (1ull << 31)) return fail(MPS_E_UNSUPPORTED, "arrays longer than 2^31 are not supported");
  // the merges carry the 8-byte payload with its key
  return run_sort(keys, kt, reinterpret_cast<uint32_t *>(payload), nullptr, 1, n, opts, trace,
                  (hipStream_t)stream, 8);
}

// ---------------------------------------------------------------- fixed scratch
// The allocation-free entry point keeps a sort's whole workspace in this
// file-scope device array.  Every device the library runs on holds its own
// copy until the process ends.  In host code the name `scratch` is only a
// stand-in for the symbol: the device address of a device's copy comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is ever passed to a kernel.
namespace {
constexpr uint64_t kScratchBytes = 64ull << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[64];   // per device; set by the first call on that device

int scratch_of_current_device(void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MPS_E_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MPS_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MPS_OK;
}
}  // namespace

extern "C" uint64_t mps_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int mps_sort_noalloc(void *keys, mps_key_type kt, uint32_t *payload, uint64_t n,
                                const mps_opts *opts, void *stream) {
  g_err[0] = 0;
  if (kt != MPS_I32 && kt != MPS_I64 && kt != MPS_F32) return fail(MPS_E_INVALID, "unknown key type");
  if (n > 0 && !keys) return fail(MPS_E_INVALID, "keys is NULL");
  if (n > (1ull << 31)) return fail(MPS_E_UNSUPPORTED, "arrays longer than 2^31 are not supported");
  if (n <= 1) return MPS_OK;
  mps_opts o{};
  if (opts) o = *opts;
  if (o.workspace)
    return fail(MPS_E_INVALID, "mps_sort_noalloc uses the library's fixed scratch; opts->workspace must be NULL");
  if (o.flags & (MPS_OPT_GRAPH | MPS_OPT_TIME_LEVELS))
    return fail(MPS_E_UNSUPPORTED,
                "MPS_OPT_GRAPH and MPS_OPT_TIME_LEVELS create HIP objects; not with mps_sort_noalloc");
  uint32_t k = o.k;
  int rc = check_k(k);
  if (rc) return rc;
  Layout L;
  if (!make_layout(n, 1, kt, payload ? 4 : 0, k, L)) return fail(MPS_E_INVALID, "bad sizes");
  if (L.total > kScratchBytes)
    return failf(MPS_E_NOMEM,
                 "this sort needs %llu bytes of workspace; the fixed scratch of mps_sort_noalloc "
                 "holds %llu (use mps_sort_ex for larger arrays)",
                 (unsigned long long)L.total, (unsigned long long)kScratchBytes);
  void *base = nullptr;
  rc = scratch_of_current_device(&base);
  if (rc) return rc;
  o.workspace = base;
  o.workspace_bytes = kScratchBytes;
  return run_sort(keys, kt, payload, nullptr, 1, n, &o, nullptr, (hipStream_t)stream);
}

extern "C" int mps_sort(void *keys, mps_key_type kt, uint32_t *payload, uint64_t n, void *stream) {
  return mps_sort_ex(keys, kt, payload, n, nullptr, nullptr, stream);
}
extern "C" int mps_sort_i32(int32_t *keys, uint32_t *payload, uint64_t n, void *stream) {
  return mps_sort_ex(keys, MPS_I32, payload, n, nullptr, nullptr, stream);
}
extern "C" int mps_sort_i64(int64_t *keys, uint32_t *payload, uint64_t n, void *stream) {
  return mps_sort_ex(keys, MPS_I64, payload, n, nullptr, nullptr, stream);
}
extern "C" int mps_sort_f32(float *keys, uint32_t *payload, uint64_t n, void *stream) {
  return mps_sort_ex(keys, MPS_F32, payload, n, nullptr, nullptr, stream);
}

extern "C" int mps_sort_batched(void *keys, mps_key_type kt, uint32_t *payload,
                                const uint64_t *offsets, const uint64_t *h_offsets, uint64_t m,
                                uint64_t total_n, const mps_opts *opts, mps_trace *trace,
                                void *stream) {
  g_err[0] = 0;
  if (kt != MPS_I32 && kt != MPS_I64 && kt != MPS_F32) return fail(MPS_E_INVALID, "unknown key type");
  if (m == 0 || total_n == 0) {
    if (trace) memset(trace, 0, offsetof(mps_trace, r_cap));
    return MPS_OK;
  }
  if (!keys || !offsets) return fail(MPS_E_INVALID, "keys or offsets is NULL");
  if (total_n > (1ull << 40)) return fail(MPS_E_UNSUPPORTED, "total too large");
  if (h_offsets) {
    if (h_offsets[0] != 0 || h_offsets[m] != total_n) return fail(MPS_E_INVALID, "offsets must run from 0 to total_n");
    for (uint64_t i = 0; i < m; i++) {
      if (h_offsets[i + 1] < h_offsets[i]) return fail(MPS_E_INVALID, "offsets must be non-decreasing");
      if (h_offsets[i + 1] - h_offsets[i] > (1ull << 31)) return fail(MPS_E_UNSUPPORTED, "an array is longer than 2^31");
    }
  }
  return run_sort(keys, kt, payload, offsets, m, total_n, opts, trace, (hipStream_t)stream);
}

extern "C" int mps_sort_status(const void *workspace, void *stream) {
  g_err[0] = 0;
  hipStream_t s = (hipStream_t)stream;
  void *base = workspace ? reinterpret_cast<void *>((reinterpret_cast<uintptr_t>(workspace) + 255) &
                                                    ~(uintptr_t)255)
                         : find_workspace(s);
  if (!base)
    return fail(MPS_E_NOTFOUND, "no sort has used the library-managed workspace of this device and stream");
  HIP_TRY(hipStreamSynchronize(s));
  uint32_t err = 0;
  HIP_TRY(hipMemcpy(&err, static_cast<char *>(base) + offsetof(Plan, error), 4, hipMemcpyDeviceToHost));
  if (err) return failf(MPS_E_DEVICE, "device-side consistency check failed (error word 0x%x)", err);
  return MPS_OK;
}

extern "C" int mps_free_workspaces(void) {
  g_err[0] = 0;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if (g_ws.empty()) return MPS_OK;
  }
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto &e : g_ws) {
      if (!e.second.first) continue;
      HIP_TRY(hipSetDevice(e.first.dev));
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(e.second.first));
      e.second.first = nullptr;
      e.second.second = 0;
    }
    g_ws.clear();
    for (auto &b : g_last_base) b = nullptr;
  }
  {
    std::lock_guard<std::mutex> lk(g_time_mu);
    for (auto &t : g_time) t.base = nullptr;
  }
  HIP_TRY(hipSetDevice(cur));
  return MPS_OK;
}

extern "C" int mps_trace_fetch(const void *workspace, mps_trace *trace) {
  g_err[0] = 0;
  if (!trace) return fail(MPS_E_INVALID, "trace is NULL");
  void *base = nullptr;
  if (workspace) {
    base = reinterpret_cast<void *>((reinterpret_cast<uintptr_t>(workspace) + 255) & ~(uintptr_t)255);
  } else {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64 || !g_last_base[dev]) return fail(MPS_E_NOTFOUND, "no sort has used the library workspace");
    base = g_last_base[dev];
  }
  return fill_trace(base, trace);
}

extern "C" int mps_last_level_stats(uint32_t cap, uint32_t *n_levels, uint64_t *level_elems,
                                    float *corank_ms, float *merge_ms) {
  g_err[0] = 0;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MPS_E_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_time_mu);
  LevelTiming &tm = g_time[dev];
  if (!tm.base || tm.levels == 0) return fail(MPS_E_NOTFOUND, "no timed sort on this device");
  Plan plan;
  HIP_TRY(hipEventSynchronize(tm.ev[2]));  // level 0's merge is the last launch
  HIP_TRY(hipMemcpy(&plan, tm.base, sizeof(Plan), hipMemcpyDeviceToHost));
  uint32_t nl = plan.lvl_levels;   // the levels the level merges ran
  if (n_levels) *n_levels = nl;
  for (uint32_t d = 0; d < nl && d < cap && d < (uint32_t)tm.levels; d++) {
    if (level_elems) level_elems[d] = plan.lvl_total[d];
    float a = 0, b = 0;
    HIP_TRY(hipEventElapsedTime(&a, tm.ev[3 * d], tm.ev[3 * d + 1]));
    HIP_TRY(hipEventElapsedTime(&b, tm.ev[3 * d + 1], tm.ev[3 * d + 2]));
    if (corank_ms) corank_ms[d] = a;
    if (merge_ms) merge_ms[d] = b;
  }
  return MPS_OK;
}
