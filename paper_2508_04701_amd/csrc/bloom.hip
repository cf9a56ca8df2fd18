// Bloom filter build: the semi-join reduction ("predicate transfer") that
// the paper lists among its planned optimizations (Section 3.4): a compact
// filter over one table's join keys lets a scan of the other table drop rows
// that cannot find a partner before they reach a hash table.
//
// Blocked layout (device.h): each key sets one bit in each of the eight
// 32-bit words of one 32-byte block. The build clears the filter with a fill
// kernel (no memset, so the call can be captured in a graph) and then sets
// every key's bits with device-scope atomic ORs, one thread per key and four
// keys per thread in flight.

#include "internal.h"

namespace rel {

namespace {

constexpr int kBloomThreads = 256;
constexpr int kBloomKeys = 4;

__global__ void __launch_bounds__(kBloomThreads) bloom_build_kernel(BloomBuildParams p) {
  const uint64_t n = static_cast<uint64_t>(p.n);
  const uint64_t step = static_cast<uint64_t>(gridDim.x) * kBloomThreads * kBloomKeys;
  for (uint64_t base = static_cast<uint64_t>(blockIdx.x) * kBloomThreads * kBloomKeys; base < n;
       base += step) {
    int64_t key[kBloomKeys];
#pragma unroll
    for (int j = 0; j < kBloomKeys; ++j) {
      const uint64_t i = base + static_cast<uint64_t>(j) * kBloomThreads + threadIdx.x;
      const uint64_t row = i < n ? (p.idx ? p.idx[i] : i) : 0;
      key[j] = i < n ? load_elem(p.keys, p.type, static_cast<int64_t>(row)) : 0;
    }
#pragma unroll
    for (int j = 0; j < kBloomKeys; ++j) {
      const uint64_t i = base + static_cast<uint64_t>(j) * kBloomThreads + threadIdx.x;
      if (i >= n) continue;
      const uint64_t h = bloom_hash(key[j]);
      uint32_t* w = p.words + bloom_block(h, p.bmask) * 8;
#pragma unroll
      for (int b = 0; b < 8; ++b) atomicOr(w + b, bloom_bit(h, b));
    }
  }
}

}  // namespace

void launch_bloom_build(const BloomBuildParams& p, hipStream_t s) {
  ProfileScope ps(kKBloom, s);
  launch_fill64(reinterpret_cast<uint64_t*>(p.words), (p.bmask + 1) * 4, 0, s);
  if (p.n <= 0) return;
  uint64_t blocks = (static_cast<uint64_t>(p.n) + kBloomThreads * kBloomKeys - 1) /
                    (kBloomThreads * kBloomKeys);
  const uint64_t limit = static_cast<uint64_t>(device_info().cu_count) * 16;
  if (blocks > limit) blocks = limit;
  hipLaunchKernelGGL(bloom_build_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBloomThreads),
                     0, s, p);
}

}  // namespace rel
