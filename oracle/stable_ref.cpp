// stable_ref.cpp -- std::stable_sort of (key, payload) records, one thread.
//
// A library reference beside the oracle (TEST INFRASTRUCTURE ONLY): the tests
// pin the oracle's output to it, and the CPU-baseline leg of the benchmark
// times it next to the oracle.  Keys are compared as signed integers (key
// types 0: int32, 1: int64) or by the IEEE-754 total order of float32 (key
// type 2: the bit pattern with the sign bit flipped for positives and all bits
// flipped for negatives, compared as unsigned).  Equal keys keep their input
// order, which is what std::stable_sort guarantees.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

template <typename K>
struct Rec {
  K key;
  uint32_t pay;
};

inline uint32_t f32_order(uint32_t b) { return (b & 0x80000000u) ? ~b : (b | 0x80000000u); }

template <typename K, typename Less>
void run(const void *keys, const uint32_t *pay, uint64_t n, void *keys_out, uint32_t *pay_out,
         Less less) {
  const K *k = static_cast<const K *>(keys);
  std::vector<Rec<K>> v(n);
  for (uint64_t i = 0; i < n; i++) v[i] = Rec<K>{k[i], pay ? pay[i] : (uint32_t)i};
  std::stable_sort(v.begin(), v.end(), [&](const Rec<K> &a, const Rec<K> &b) { return less(a.key, b.key); });
  K *ko = static_cast<K *>(keys_out);
  for (uint64_t i = 0; i < n; i++) {
    ko[i] = v[i].key;
    if (pay_out) pay_out[i] = v[i].pay;
  }
}

}  // namespace

extern "C" int ref_stable_sort(const void *keys, const uint32_t *pay, uint64_t n, int kt,
                               void *keys_out, uint32_t *pay_out) {
  switch (kt) {
    case 0: run<int32_t>(keys, pay, n, keys_out, pay_out, [](int32_t a, int32_t b) { return a < b; }); return 0;
    case 1: run<int64_t>(keys, pay, n, keys_out, pay_out, [](int64_t a, int64_t b) { return a < b; }); return 0;
    case 2:
      run<uint32_t>(keys, pay, n, keys_out, pay_out,
                    [](uint32_t a, uint32_t b) { return f32_order(a) < f32_order(b); });
      return 0;
    default: return -1;
  }
}
