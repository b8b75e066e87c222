// mps_serve_core.h -- host-only parts of the request server: the device-arena
// sub-allocator and the batch-formation policy.  No HIP calls here, so the
// policy is unit-tested on machines without a GPU (mps_serve_selftest).
#pragma once

#include <stdint.h>

#include <deque>
#include <functional>
#include <map>
#include <vector>

namespace mps {
namespace serve {

// First-fit allocator over [0, size) with 256-byte granularity; free blocks
// are coalesced with their neighbours.
class Arena {
 public:
  static constexpr uint64_t kAlign = 256;
  explicit Arena(uint64_t size = 0) { reset(size); }
  void reset(uint64_t size) {
    size_ = size & ~(kAlign - 1);
    free_.clear();
    used_ = 0;
    if (size_) free_[0] = size_;
  }
  // Offset of a block of at least `bytes`, or ~0 if no free block is large enough.
  uint64_t alloc(uint64_t bytes) {
    uint64_t need = round(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= need) {
        uint64_t off = it->first, rest = it->second - need;
        free_.erase(it);
        if (rest) free_[off + need] = rest;
        used_ += need;
        return off;
      }
    }
    return ~0ull;
  }
  void release(uint64_t off, uint64_t bytes) {
    uint64_t len = round(bytes ? bytes : 1);
    used_ -= len;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {  // merge with the following block
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {  // merge with the preceding block
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }
  uint64_t largest_free() const {
    uint64_t b = 0;
    for (auto &f : free_) b = f.second > b ? f.second : b;
    return b;
  }
  uint64_t size() const { return size_; }
  uint64_t used() const { return used_; }
  size_t fragments() const { return free_.size(); }
  static uint64_t round(uint64_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

 private:
  uint64_t size_ = 0, used_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

// One pending request as the policy sees it.
struct Pending {
  uint64_t id;
  uint64_t n;
  int kt;           // key type
  bool payload;     // has a payload
};

// Device bytes a batch of `count` requests holding `total` keys needs: packed
// keys and payloads, offsets, the copy table and the sort workspace.
using NeedFn = std::function<uint64_t(uint64_t total, uint64_t count, int kt, bool payload)>;

// Batch formation: take requests in arrival order, starting with the oldest,
// as long as they share its key type and payload presence, the batch stays
// within max_batch requests, and its memory need fits in `avail` bytes.
// Returns how many leading requests form the batch (0: the oldest does not
// fit yet) and the batch's key count and byte need.
inline size_t form_batch(const std::deque<Pending> &q, size_t max_batch, uint64_t avail,
                         const NeedFn &need, uint64_t *keys_out, uint64_t *bytes_out) {
  *keys_out = 0;
  *bytes_out = 0;
  if (q.empty() || max_batch == 0) return 0;
  const int kt = q.front().kt;
  const bool pl = q.front().payload;
  uint64_t total = 0, bytes = 0;
  size_t c = 0;
  for (const Pending &p : q) {
    if (c == max_batch || p.kt != kt || p.payload != pl) break;
    uint64_t b = need(total + p.n, c + 1, kt, pl);
    if (b == 0 || b > avail) break;
    total += p.n;
    bytes = b;
    c++;
  }
  *keys_out = total;
  *bytes_out = bytes;
  return c;
}

// Self-test of the allocator and the policy; returns 0, or the number of the
// first failed check.
inline int selftest() {
  int check = 0;
#define MPS_ST(cond) \
  do {               \
    ++check;         \
    if (!(cond)) return check; \
  } while (0)
  Arena a(1 << 20);
  uint64_t x = a.alloc(1000), y = a.alloc(5000), z = a.alloc(256);
  MPS_ST(x == 0 && y == 1024 && z == 1024 + 5120);
  MPS_ST(a.used() == 1024 + 5120 + 256);
  a.release(y, 5000);
  MPS_ST(a.fragments() == 2);
  uint64_t w = a.alloc(4096);          // first fit reuses the hole
  MPS_ST(w == 1024);
  a.release(w, 4096);
  a.release(x, 1000);                  // coalesces with the hole after it
  MPS_ST(a.fragments() == 2 && a.largest_free() == (1 << 20) - (1024 + 5120 + 256));
  a.release(z, 256);                   // everything free again, one block
  MPS_ST(a.fragments() == 1 && a.used() == 0 && a.largest_free() == (1u << 20));
  MPS_ST(a.alloc((1 << 20) + 1) == ~0ull);
  // many random alloc/free keep the books balanced
  std::vector<std::pair<uint64_t, uint64_t>> live;
  uint64_t s = 12345;
  for (int i = 0; i < 2000; i++) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    if ((s >> 60) < 9 || live.empty()) {
      uint64_t b = 1 + ((s >> 20) % 20000);
      uint64_t o = a.alloc(b);
      if (o != ~0ull) {
        for (auto &l : live) MPS_ST(o + Arena::round(b) <= l.first || l.first + Arena::round(l.second) <= o);
        live.push_back({o, b});
      }
    } else {
      size_t j = (s >> 8) % live.size();
      a.release(live[j].first, live[j].second);
      live.erase(live.begin() + j);
    }
  }
  for (auto &l : live) a.release(l.first, l.second);
  MPS_ST(a.used() == 0 && a.fragments() == 1);
  // policy
  NeedFn need = [](uint64_t t, uint64_t c, int, bool) { return t * 10 + c * 100; };
  std::deque<Pending> q = {{1, 100, 0, true}, {2, 50, 0, true}, {3, 70, 2, true}, {4, 10, 0, true}};
  uint64_t keys = 0, bytes = 0;
  MPS_ST(form_batch(q, 8, 1 << 20, need, &keys, &bytes) == 2 && keys == 150 && bytes == 1700);
  MPS_ST(form_batch(q, 1, 1 << 20, need, &keys, &bytes) == 1 && keys == 100);
  MPS_ST(form_batch(q, 8, 1500, need, &keys, &bytes) == 1 && bytes == 1100);
  MPS_ST(form_batch(q, 8, 1000, need, &keys, &bytes) == 0);
  q.pop_front();
  q.pop_front();
  MPS_ST(form_batch(q, 8, 1 << 20, need, &keys, &bytes) == 1 && keys == 70);  // type change ends a batch
#undef MPS_ST
  return 0;
}

}  // namespace serve
}  // namespace mps
