// mps_serve.hip -- continuous-batching sort server.
//
// Callers submit device-resident sort requests at any time.  A scheduler
// thread admits them in arrival order into batches whose device memory
// (packed copies of the requests, offsets, copy table and the sort
// workspace) fits in the free part of an arena reserved once at creation
// (the HBM budget).  Each batch runs on one of several streams as: upload of
// the copy table, a gather kernel that packs the requests back to back, one
// batched multiway Powersort of the packed arrays, and a scatter kernel that
// writes every sorted request to its output buffers.  Requests that arrive
// while batches are running form the next batch as soon as a stream and
// memory are free, so their work overlaps on the device.  Every request is
// sorted exactly as mps_sort sorts it alone (each array of a batch keeps its
// own runs and its own power normaliser).
#include <stddef.h>
#include <stdint.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mps.h"
#include "mps_internal.h"
#include "mps_serve_core.h"

namespace mps {
namespace serve {

struct ReqDesc {            // one request of a batch, as the copy kernels see it
  const void *kin;
  const uint32_t *pin;
  void *kout;
  uint32_t *pout;
};

constexpr int kCopyThreads = 256;
constexpr int kCopyChunk = 4096;   // packed positions per workgroup step

// Packed position p belongs to the request r with off[r] <= p < off[r+1].
__device__ inline uint32_t req_of(const uint64_t *off, uint32_t m, uint64_t p) {
  uint32_t lo = 0, hi = m;   // off[lo] <= p < off[hi]
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= p) lo = mid; else hi = mid;
  }
  return lo;
}

// dir 0: gather requests into the packed buffers; dir 1: scatter back.
template <typename U>
__global__ __launch_bounds__(kCopyThreads) void k_pack(const ReqDesc *__restrict__ d,
                                                       const uint64_t *__restrict__ off,
                                                       uint32_t m, U *__restrict__ pk,
                                                       uint32_t *__restrict__ pp, int dir) {
  __shared__ uint32_t s_r;
  const uint64_t T = off[m];
  for (uint64_t c0 = (uint64_t)blockIdx.x * kCopyChunk; c0 < T;
       c0 += (uint64_t)gridDim.x * kCopyChunk) {
    if (threadIdx.x == 0) s_r = req_of(off, m, c0);
    __syncthreads();
    uint32_t r = s_r;
    const uint64_t c1 = c0 + kCopyChunk < T ? c0 + kCopyChunk : T;
    if (c1 - c0 == kCopyChunk && off[r + 1] >= c1) {
      // The whole chunk lies in request r: every lane issues all of its loads
      // before its first store, so a wave keeps kCopyChunk / kCopyThreads
      // accesses of each array in flight.
      constexpr int E = kCopyChunk / kCopyThreads;
      const uint64_t b = c0 - off[r] + threadIdx.x;
      const U *src = dir == 0 ? static_cast<const U *>(d[r].kin) + b : pk + c0 + threadIdx.x;
      U *dst = dir == 0 ? pk + c0 + threadIdx.x : static_cast<U *>(d[r].kout) + b;
      U kv[E];
#pragma unroll
      for (int e = 0; e < E; e++) kv[e] = src[e * kCopyThreads];
      if (pp) {
        const uint32_t *psrc = dir == 0 ? d[r].pin + b : pp + c0 + threadIdx.x;
        uint32_t *pdst = dir == 0 ? pp + c0 + threadIdx.x : d[r].pout + b;
        uint32_t pv[E];
#pragma unroll
        for (int e = 0; e < E; e++) pv[e] = psrc[e * kCopyThreads];
#pragma unroll
        for (int e = 0; e < E; e++) pdst[e * kCopyThreads] = pv[e];
      }
#pragma unroll
      for (int e = 0; e < E; e++) dst[e * kCopyThreads] = kv[e];
      __syncthreads();
      continue;
    }
    for (uint64_t p = c0 + threadIdx.x; p < c1; p += kCopyThreads) {
      while (off[r + 1] <= p) r++;
      const uint64_t i = p - off[r];
      if (dir == 0) {
        pk[p] = static_cast<const U *>(d[r].kin)[i];
        if (pp) pp[p] = d[r].pin[i];
      } else {
        static_cast<U *>(d[r].kout)[i] = pk[p];
        if (pp) d[r].pout[i] = pp[p];
      }
    }
    __syncthreads();
  }
}

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  mps_request req;
  uint64_t t_submit = 0, t_admit = 0, t_done = 0, batch = 0;
  uint32_t batch_requests = 0;
  int status = MPS_PENDING;
};

struct Slot {                  // one stream and what its batch holds
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void *pinned = nullptr;      // host copy table + offsets + device-error word
  bool busy = false;
  uint64_t arena_off = 0, arena_bytes = 0, batch = 0;
  std::vector<uint64_t> ids;
  bool forced_fail = false;
};

}  // namespace serve
}  // namespace mps

using namespace mps;
using namespace mps::serve;

struct mps_server {
  mps_serve_cfg cfg{};
  int device = 0;
  void *arena_base = nullptr;
  Arena arena;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Pending> queue;
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_id = 1, next_batch = 1, batches_run = 0;
  bool stopping = false;
  std::thread worker;
  std::string thread_error;

  size_t table_bytes() const { return (size_t)cfg.max_batch * (sizeof(ReqDesc) + 8) + 8 + 64; }

  uint64_t need(uint64_t total, uint64_t count, int kt, bool payload) const {
    const uint64_t ks = kt == MPS_I64 ? 8 : 4;
    uint64_t ws = mps_workspace_bytes(total < 2 ? 2 : total, count, (mps_key_type)kt, payload ? 1 : 0,
                                      cfg.k);
    if (ws == 0) return 0;
    return Arena::round(total * ks) + Arena::round(payload ? total * 4 : 0) +
           Arena::round((count + 1) * 8) + Arena::round(count * sizeof(ReqDesc)) + ws + 256;
  }

  // Launch the batch formed by the first `count` queued requests on slot s.
  // Called with mu held.
  void launch(Slot &s, size_t count, uint64_t total, uint64_t bytes, uint64_t aoff) {
    const int kt = queue.front().kt;
    const bool pl = queue.front().payload;
    const uint64_t ks = kt == MPS_I64 ? 8 : 4;
    s.busy = true;
    s.arena_off = aoff;
    s.arena_bytes = bytes;
    s.batch = next_batch++;
    s.ids.clear();
    s.forced_fail = cfg.fail_every && (s.batch % cfg.fail_every) == 0;
    // host tables in pinned memory: descriptors, then offsets, then the error word
    ReqDesc *hd = static_cast<ReqDesc *>(s.pinned);
    uint64_t *ho = reinterpret_cast<uint64_t *>(hd + cfg.max_batch);
    uint32_t *herr = reinterpret_cast<uint32_t *>(ho + cfg.max_batch + 1);
    *herr = 0;
    const uint64_t t_admit = now_ns();
    ho[0] = 0;
    for (size_t i = 0; i < count; i++) {
      Pending p = queue.front();
      queue.pop_front();
      Request &r = reqs[p.id];
      r.t_admit = t_admit;
      r.batch = s.batch;
      r.batch_requests = (uint32_t)count;
      hd[i] = ReqDesc{r.req.keys, r.req.payload, r.req.keys_out, r.req.payload_out};
      ho[i + 1] = ho[i] + p.n;
      s.ids.push_back(p.id);
    }
    char *base = static_cast<char *>(arena_base) + aoff;
    char *pk = base;
    char *pp = pk + Arena::round(total * ks);
    uint64_t *doff = reinterpret_cast<uint64_t *>(pp + Arena::round(pl ? total * 4 : 0));
    ReqDesc *dd = reinterpret_cast<ReqDesc *>(reinterpret_cast<char *>(doff) + Arena::round((count + 1) * 8));
    char *ws = reinterpret_cast<char *>(dd) + Arena::round(count * sizeof(ReqDesc));
    const uint64_t ws_bytes = bytes - (uint64_t)(ws - base);
    bool ok = !s.forced_fail;
    for (uint64_t id : s.ids) {
      void *ev = reqs[id].req.ready_event;
      if (ok && ev) ok = hipStreamWaitEvent(s.stream, (hipEvent_t)ev, 0) == hipSuccess;
    }
    if (ok) {
      ok = hipMemcpyAsync(doff, ho, (count + 1) * 8, hipMemcpyHostToDevice, s.stream) == hipSuccess &&
           hipMemcpyAsync(dd, hd, count * sizeof(ReqDesc), hipMemcpyHostToDevice, s.stream) == hipSuccess;
    }
    uint64_t blocks = (total + kCopyChunk - 1) / kCopyChunk;
    unsigned grid = (unsigned)(blocks < 4096 ? (blocks ? blocks : 1) : 4096);
    if (ok && total) {
      if (ks == 8)
        hipLaunchKernelGGL(k_pack<uint64_t>, dim3(grid), dim3(kCopyThreads), 0, s.stream, dd, doff,
                           (uint32_t)count, (uint64_t *)pk, pl ? (uint32_t *)pp : nullptr, 0);
      else
        hipLaunchKernelGGL(k_pack<uint32_t>, dim3(grid), dim3(kCopyThreads), 0, s.stream, dd, doff,
                           (uint32_t)count, (uint32_t *)pk, pl ? (uint32_t *)pp : nullptr, 0);
      ok = hipGetLastError() == hipSuccess;
    }
    if (ok && total) {
      mps_opts o{};
      o.k = cfg.k;
      o.workspace = ws;
      o.workspace_bytes = ws_bytes;
      o.tile = cfg.tile;
      o.lane_slice = cfg.lane_slice;
      ok = mps_sort_batched(pk, (mps_key_type)kt, pl ? (uint32_t *)pp : nullptr, doff, ho, count,
                            total, &o, nullptr, s.stream) == MPS_OK;
      // the device-side consistency word of the batch's plan
      void *wsa = reinterpret_cast<void *>((reinterpret_cast<uintptr_t>(ws) + 255) & ~(uintptr_t)255);
      ok = ok && hipMemcpyAsync(herr, static_cast<char *>(wsa) + offsetof(Plan, error), 4,
                                hipMemcpyDeviceToHost, s.stream) == hipSuccess;
    }
    if (ok && total) {
      if (ks == 8)
        hipLaunchKernelGGL(k_pack<uint64_t>, dim3(grid), dim3(kCopyThreads), 0, s.stream, dd, doff,
                           (uint32_t)count, (uint64_t *)pk, pl ? (uint32_t *)pp : nullptr, 1);
      else
        hipLaunchKernelGGL(k_pack<uint32_t>, dim3(grid), dim3(kCopyThreads), 0, s.stream, dd, doff,
                           (uint32_t)count, (uint32_t *)pk, pl ? (uint32_t *)pp : nullptr, 1);
      ok = hipGetLastError() == hipSuccess;
    }
    if (ok) ok = hipEventRecord(s.done, s.stream) == hipSuccess;
    if (!ok) {
      // nothing more is enqueued for this batch (a forced failure enqueues nothing at
      // all); its memory is released once whatever was enqueued has drained
      (void)hipStreamSynchronize(s.stream);
      finish(s, MPS_E_HIP);
    }
    batches_run++;
  }

  // Mark a slot's requests finished and release its memory.  mu held.
  void finish(Slot &s, int status) {
    const uint64_t t = now_ns();
    for (uint64_t id : s.ids) {
      Request &r = reqs[id];
      r.t_done = t;
      r.status = status;
    }
    s.ids.clear();
    arena.release(s.arena_off, s.arena_bytes);
    s.busy = false;
  }

  void run() {
    if (hipSetDevice(device) != hipSuccess) {
      std::lock_guard<std::mutex> lk(mu);
      thread_error = "scheduler could not select the device";
    }
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      bool any_busy = false;
      for (Slot &s : slots) {
        if (!s.busy) continue;
        hipError_t q = hipEventQuery(s.done);
        if (q == hipSuccess) {
          const uint32_t *herr = reinterpret_cast<const uint32_t *>(
              reinterpret_cast<const uint64_t *>(static_cast<const ReqDesc *>(s.pinned) + cfg.max_batch) +
              cfg.max_batch + 1);
          finish(s, *herr ? MPS_E_DEVICE : MPS_OK);
        } else if (q != hipErrorNotReady) {
          finish(s, MPS_E_HIP);
        } else {
          any_busy = true;
        }
      }
      // admit as many batches as streams and memory allow
      for (Slot &s : slots) {
        if (s.busy || queue.empty()) continue;
        uint64_t keys = 0, bytes = 0;
        size_t c = form_batch(queue, cfg.max_batch, arena.largest_free(),
                              [this](uint64_t t, uint64_t n, int kt, bool pl) { return need(t, n, kt, pl); },
                              &keys, &bytes);
        if (c == 0) break;   // the oldest request waits for memory
        uint64_t off = arena.alloc(bytes);
        if (off == ~0ull) break;
        launch(s, c, keys, bytes, off);
        any_busy = true;
      }
      if (stopping && queue.empty() && !any_busy) {
        bool busy = false;
        for (Slot &s : slots) busy = busy || s.busy;
        if (!busy) break;
      }
      if (any_busy)
        cv.wait_for(lk, std::chrono::microseconds(cfg.poll_us));
      else
        cv.wait(lk, [this] { return stopping || !queue.empty(); });
    }
  }
};

// ---------------------------------------------------------------- C entry points
extern "C" int mps_serve_create(const mps_serve_cfg *cfg, mps_server **out) {
  if (!cfg || !out) return fail_msg(MPS_E_INVALID, "cfg or out is NULL");
  *out = nullptr;
  mps_serve_cfg c = *cfg;
  if (c.n_streams == 0) c.n_streams = 2;
  if (c.max_batch == 0) c.max_batch = 256;
  if (c.k == 0) c.k = 4;
  if (c.poll_us == 0) c.poll_us = 20;
  if (c.n_streams > 16) return fail_msg(MPS_E_UNSUPPORTED, "at most 16 streams");
  if (c.k != 2 && c.k != 4 && c.k != 8) return fail_msg(MPS_E_UNSUPPORTED, "k must be 2, 4 or 8");
  if (c.hbm_budget_bytes < (1u << 20)) return fail_msg(MPS_E_INVALID, "HBM budget below 1 MiB");
  auto *s = new (std::nothrow) mps_server();
  if (!s) return fail_msg(MPS_E_NOMEM, "out of host memory");
  s->cfg = c;
  auto cleanup = [s](int code, const char *msg) {
    for (Slot &sl : s->slots) {
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.pinned) (void)hipHostFree(sl.pinned);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
    return fail_msg(code, msg);
  };
  if (hipGetDevice(&s->device) != hipSuccess) return cleanup(MPS_E_HIP, "hipGetDevice failed");
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return cleanup(MPS_E_HIP, "hipMemGetInfo failed");
  if (c.hbm_budget_bytes > free_b) return cleanup(MPS_E_NOMEM, "HBM budget exceeds free device memory");
  if (hipMalloc(&s->arena_base, c.hbm_budget_bytes) != hipSuccess)
    return cleanup(MPS_E_NOMEM, "arena allocation failed");
  s->arena.reset(c.hbm_budget_bytes);
  s->slots.resize(c.n_streams);
  for (Slot &sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc(&sl.pinned, s->table_bytes(), hipHostMallocDefault) != hipSuccess)
      return cleanup(MPS_E_HIP, "stream / event / pinned buffer creation failed");
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return MPS_OK;
}

extern "C" int mps_serve_submit(mps_server *s, const mps_request *req, uint64_t *req_id) {
  if (!s || !req || !req_id) return fail_msg(MPS_E_INVALID, "server, request or id is NULL");
  if (req->kt != MPS_I32 && req->kt != MPS_I64 && req->kt != MPS_F32)
    return fail_msg(MPS_E_INVALID, "unknown key type");
  if (req->n > 0 && (!req->keys || !req->keys_out)) return fail_msg(MPS_E_INVALID, "keys or keys_out is NULL");
  if ((req->payload == nullptr) != (req->payload_out == nullptr))
    return fail_msg(MPS_E_INVALID, "payload and payload_out must both be given or both be NULL");
  if (req->n > (1ull << 31)) return fail_msg(MPS_E_UNSUPPORTED, "requests longer than 2^31 are not supported");
  const uint64_t need = s->need(req->n, 1, req->kt, req->payload != nullptr);
  if (need == 0 || need > s->arena.size())
    return fail_msg(MPS_E_NOMEM, "request needs more device memory than the server's whole HBM budget");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return fail_msg(MPS_E_INVALID, "server is shutting down");
  const uint64_t id = s->next_id++;
  Request r;
  r.req = *req;
  r.t_submit = now_ns();
  s->reqs.emplace(id, r);
  s->queue.push_back(Pending{id, req->n, (int)req->kt, req->payload != nullptr});
  *req_id = id;
  s->cv.notify_one();
  return MPS_OK;
}

extern "C" int mps_serve_poll(mps_server *s, uint64_t req_id, mps_req_info *info) {
  if (!s) return fail_msg(MPS_E_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return fail_msg(MPS_E_NOTFOUND, "unknown request id");
  const Request &r = it->second;
  if (info) {
    info->t_submit_ns = r.t_submit;
    info->t_admit_ns = r.t_admit;
    info->t_done_ns = r.t_done;
    info->batch = r.batch;
    info->batch_requests = r.batch_requests;
    info->status = r.status;
  }
  if (r.status < 0) fail_msg(r.status, "request failed");
  return r.status;
}

extern "C" int mps_serve_release(mps_server *s, uint64_t req_id) {
  if (!s) return fail_msg(MPS_E_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return fail_msg(MPS_E_NOTFOUND, "unknown request id");
  if (it->second.status == MPS_PENDING) return fail_msg(MPS_E_INVALID, "request still pending");
  s->reqs.erase(it);
  return MPS_OK;
}

extern "C" int mps_serve_stats(mps_server *s, mps_serve_stats_t *st) {
  if (!s || !st) return fail_msg(MPS_E_INVALID, "server or stats is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  st->queued = s->queue.size();
  st->batches = s->batches_run;
  st->arena_bytes = s->arena.size();
  st->arena_used = s->arena.used();
  uint32_t busy = 0;
  for (Slot &sl : s->slots) busy += sl.busy ? 1 : 0;
  st->busy_streams = busy;
  return MPS_OK;
}

extern "C" int mps_serve_destroy(mps_server *s) {
  if (!s) return fail_msg(MPS_E_INVALID, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (Slot &sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.pinned) (void)hipHostFree(sl.pinned);
  }
  if (s->arena_base) (void)hipFree(s->arena_base);
  delete s;
  return MPS_OK;
}

extern "C" int mps_serve_selftest(void) { return mps::serve::selftest(); }
