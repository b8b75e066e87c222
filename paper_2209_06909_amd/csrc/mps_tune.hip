// mps_tune.hip -- autotuner for batched sorts: picks the merge arity and the
// merge tile configuration (tile size and per-thread LDS slice) by timing
// every candidate on a sample of the caller's batch.
//
// The sample is a prefix of the batch (whole arrays, up to a key budget),
// copied once into tuner-owned memory; each candidate sorts a fresh copy of
// it, timed with HIP events on the caller's stream.  Results are cached per
// (device, key type, payload presence, log2 of the total size, log2 of the
// mean array size), so later batches of the same shape skip the timing.
//
// If the environment names a file in MPS_AUTOTUNE_CACHE, choices also persist
// across processes: the file holds one JSON object per line (the GPU
// architecture name, key type, payload presence, the two size buckets, graph
// replay, and the chosen k, tile and lane slice).  It is read once, at the
// first tuning call; every new choice is appended to it.  Lines of another
// architecture, or that do not parse, are ignored.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "mps.h"
#include "mps_internal.h"

namespace {

struct TuneKey {
  int dev, kt, has_payload, lg_total, lg_mean, graph;
  bool operator<(const TuneKey &o) const {
    return std::tie(dev, kt, has_payload, lg_total, lg_mean, graph) <
           std::tie(o.dev, o.kt, o.has_payload, o.lg_total, o.lg_mean, o.graph);
  }
};
struct TuneVal {
  uint32_t k, tile, lane_slice;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune_cache;
bool g_file_loaded[64];

// Architecture name of a device (e.g. "gfx950:sramecc+:xnack-"); "" on failure.
std::string arch_of(int dev) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return std::string();
  return std::string(p.gcnArchName);
}

const char *cache_path() {
  const char *p = getenv("MPS_AUTOTUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// Loads the persisted choices of this device's architecture (call with g_tune_mu held).
void load_cache_file(int dev, const std::string &arch) {
  if (dev < 0 || dev >= 64 || g_file_loaded[dev]) return;
  g_file_loaded[dev] = true;
  const char *path = cache_path();
  if (!path || arch.empty()) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  char line[512], a[128];
  while (fgets(line, sizeof line, f)) {
    int kt, pay, lt, lm, gr;
    unsigned k, tile, ls;
    if (sscanf(line,
               " {\"arch\": \"%127[^\"]\", \"kt\": %d, \"payload\": %d, \"lg_total\": %d, "
               "\"lg_mean\": %d, \"graph\": %d, \"k\": %u, \"tile\": %u, \"lane_slice\": %u}",
               a, &kt, &pay, &lt, &lm, &gr, &k, &tile, &ls) != 9)
      continue;
    if (arch != a) continue;
    if ((k != 2 && k != 4 && k != 8) || (tile != 1024 && tile != 2048 && tile != 4096) ||
        (ls != 4 && ls != 8))
      continue;
    g_tune_cache[TuneKey{dev, kt, pay, lt, lm, gr}] = TuneVal{k, tile, ls};
  }
  fclose(f);
}

void append_cache_file(const std::string &arch, const TuneKey &key, const TuneVal &v) {
  const char *path = cache_path();
  if (!path || arch.empty()) return;
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f,
          "{\"arch\": \"%s\", \"kt\": %d, \"payload\": %d, \"lg_total\": %d, \"lg_mean\": %d, "
          "\"graph\": %d, \"k\": %u, \"tile\": %u, \"lane_slice\": %u}\n",
          arch.c_str(), key.kt, key.has_payload, key.lg_total, key.lg_mean, key.graph, v.k, v.tile,
          v.lane_slice);
  fclose(f);
}

// Candidates: arity x tile configuration.
const uint32_t kArities[3] = {4, 2, 8};
const uint32_t kTiles[5][2] = {{2048, 8}, {1024, 4}, {2048, 4}, {4096, 8}, {4096, 4}};

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

int ilog2(uint64_t x) {
  int l = 0;
  while (x > 1) {
    x >>= 1;
    l++;
  }
  return l;
}

}  // namespace

extern "C" int mps_autotune(const void *keys, mps_key_type kt, const uint32_t *payload,
                            const uint64_t *h_offsets, uint64_t m, uint64_t sample_cap,
                            uint32_t flags, mps_opts *best, float *cand_ms, void *stream) {
  if (!best) return mps::fail_msg(MPS_E_INVALID, "best is NULL");
  if (kt != MPS_I32 && kt != MPS_I64 && kt != MPS_F32) return mps::fail_msg(MPS_E_INVALID, "unknown key type");
  if (m == 0 || !h_offsets || !keys) return mps::fail_msg(MPS_E_INVALID, "keys / host offsets missing");
  if (flags & ~MPS_OPT_GRAPH) return mps::fail_msg(MPS_E_INVALID, "only MPS_OPT_GRAPH may be set");
  const uint64_t total = h_offsets[m];
  if (h_offsets[0] != 0) return mps::fail_msg(MPS_E_INVALID, "offsets must start at 0");
  for (uint64_t i = 0; i < m; i++)
    if (h_offsets[i + 1] < h_offsets[i]) return mps::fail_msg(MPS_E_INVALID, "offsets must be non-decreasing");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return mps::fail_msg(MPS_E_HIP, "hipGetDevice failed");
  const TuneKey key{dev, (int)kt, payload ? 1 : 0, ilog2(total ? total : 1),
                    ilog2(total / m ? total / m : 1), (flags & MPS_OPT_GRAPH) ? 1 : 0};
  const std::string arch = cache_path() ? arch_of(dev) : std::string();
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_file(dev, arch);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end() && !cand_ms) {
      best->k = it->second.k;
      best->tile = it->second.tile;
      best->lane_slice = it->second.lane_slice;
      return MPS_OK;
    }
  }
  // sample: whole arrays from the start, up to sample_cap keys (at least one array)
  if (sample_cap == 0) sample_cap = 1ull << 27;   // well beyond the last-level cache
  uint64_t ms = 0;
  while (ms < m && (ms == 0 || h_offsets[ms + 1] <= sample_cap)) ms++;
  const uint64_t sn = h_offsets[ms];
  std::vector<float> times(15, INFINITY);
  hipStream_t s = (hipStream_t)stream;
  uint32_t bk = 4, bt = 2048, bl = 8;
  if (sn >= 2) {
    const size_t ksz = kt == MPS_I64 ? 8 : 4;
    uint64_t wsb = 0;
    for (uint32_t k : kArities) {
      uint64_t b = mps_workspace_bytes(sn, ms, kt, payload != nullptr, k);
      if (b > wsb) wsb = b;
    }
    DevBuf pk, pv, wk, wv, off, ws;
    if (hipMalloc(&pk.p, sn * ksz) != hipSuccess || hipMalloc(&wk.p, sn * ksz) != hipSuccess ||
        (payload && (hipMalloc(&pv.p, sn * 4) != hipSuccess || hipMalloc(&wv.p, sn * 4) != hipSuccess)) ||
        hipMalloc(&off.p, (ms + 1) * 8) != hipSuccess || hipMalloc(&ws.p, wsb) != hipSuccess)
      return mps::fail_msg(MPS_E_NOMEM, "autotune: sample buffers do not fit");
    if (hipMemcpyAsync(pk.p, keys, sn * ksz, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        (payload && hipMemcpyAsync(pv.p, payload, sn * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) ||
        hipMemcpyAsync(off.p, h_offsets, (ms + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return mps::fail_msg(MPS_E_HIP, "autotune: sample copy failed");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      return mps::fail_msg(MPS_E_HIP, "autotune: event creation failed");
    float best_ms = INFINITY;
    int ci = 0;
    int rc = MPS_OK;
    for (uint32_t k : kArities) {
      for (auto &tc : kTiles) {
        mps_opts o{};
        o.k = k;
        o.flags = flags & MPS_OPT_GRAPH;
        o.workspace = ws.p;
        o.workspace_bytes = wsb;
        o.tile = tc[0];
        o.lane_slice = tc[1];
        float acc = 0;
        const int reps = 3;
        for (int r = 0; r <= reps && rc == MPS_OK; r++) {   // r = 0: warm-up (and graph capture)
          if (hipMemcpyAsync(wk.p, pk.p, sn * ksz, hipMemcpyDeviceToDevice, s) != hipSuccess ||
              (payload && hipMemcpyAsync(wv.p, pv.p, sn * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)) {
            rc = mps::fail_msg(MPS_E_HIP, "autotune: restore copy failed");
            break;
          }
          (void)hipEventRecord(e0, s);
          int r2 = mps_sort_batched(wk.p, kt, (uint32_t *)wv.p, (const uint64_t *)off.p, h_offsets,
                                    ms, sn, &o, nullptr, s);
          if (r2 != MPS_OK) {
            rc = r2;
            break;
          }
          (void)hipEventRecord(e1, s);
          if (hipEventSynchronize(e1) != hipSuccess) {
            rc = mps::fail_msg(MPS_E_HIP, "autotune: sort failed");
            break;
          }
          float t = 0;
          (void)hipEventElapsedTime(&t, e0, e1);
          if (r > 0) acc += t;
        }
        if (rc != MPS_OK) break;
        times[ci] = acc / reps;
        if (times[ci] < best_ms) {
          best_ms = times[ci];
          bk = k;
          bt = tc[0];
          bl = tc[1];
        }
        ci++;
      }
      if (rc != MPS_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != MPS_OK) return rc;
  }
  if (cand_ms)
    for (int i = 0; i < 15; i++) cand_ms[i] = times[i];
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = TuneVal{bk, bt, bl};
    append_cache_file(arch, key, TuneVal{bk, bt, bl});
  }
  best->k = bk;
  best->tile = bt;
  best->lane_slice = bl;
  return MPS_OK;
}
