// Per-workgroup group tables in LDS, shared by the group-by and the fused
// pipeline kernels. Slots use the same layout as the global table: [0] packed
// key, [1] COUNT, then the accumulators. A key that finds no LDS slot within
// a short probe window is aggregated in the global table instead.
#pragma once

#include "internal.h"

namespace rel {

constexpr int kLdsProbe = 16;

__device__ __forceinline__ void lds_group_init(uint64_t* t, int slots, const GroupDesc& g) {
  for (int i = threadIdx.x; i < slots * g.words; i += blockDim.x) {
    const int w = i % g.words;
    uint64_t v = 0;
    if (w == 0) v = kEmpty64;
    else if (w >= 2 && w - 2 < g.ap.nacc) v = acc_identity(g.ap.kind[w - 2]);
    t[i] = v;
  }
}

// Hash of a packed key for the LDS table (32-bit arithmetic only).
__device__ __forceinline__ uint32_t lds_hash(uint64_t pk) {
  return hash32(static_cast<uint32_t>(pk) ^ hash32(static_cast<uint32_t>(pk >> 32) + 0x9e3779b9u));
}

// Partition of packed key pk among `parts` (a power of two): the top bits of
// its LDS hash, so that an LDS table indexed by the low bits spreads one
// partition's keys over all its slots.
__device__ __forceinline__ uint32_t rec_part(uint64_t pk, uint32_t parts) {
  return static_cast<uint32_t>((static_cast<uint64_t>(lds_hash(pk)) * parts) >> 32);
}

// Packed key of a narrow record's 32 key bits (see RecDesc).
__device__ __forceinline__ uint64_t narrow_key(uint32_t k, uint32_t narrow) {
  return narrow == 1 ? static_cast<uint64_t>(static_cast<int64_t>(static_cast<int32_t>(k)))
                     : static_cast<uint64_t>(k);
}

// Index of the LDS slot holding (or newly claimed for) packed key pk, or -1
// when the key is the sentinel pattern, there is no LDS table, or no slot is
// free within the probe window.
__device__ __forceinline__ int32_t lds_group_find(uint64_t* t, int slots, int words, uint64_t pk,
                                                  int window = kLdsProbe) {
  if (pk == kEmpty64 || slots == 0) return -1;
  const uint32_t mask = static_cast<uint32_t>(slots - 1);
  uint32_t h = lds_hash(pk) & mask;
  if (window > slots) window = slots;
  for (int probe = 0; probe < window; ++probe) {
    uint64_t* s = t + h * words;
    const uint64_t cur = __hip_atomic_load(s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == pk) return static_cast<int32_t>(h);
    if (cur == kEmpty64) {
      unsigned long long prev = atomicCAS(reinterpret_cast<unsigned long long*>(s),
                                          static_cast<unsigned long long>(kEmpty64),
                                          static_cast<unsigned long long>(pk));
      if (prev == kEmpty64 || prev == pk) return static_cast<int32_t>(h);
    }
    h = (h + 1) & mask;
  }
  return -1;
}

__device__ __forceinline__ uint64_t* lds_group_slot(uint64_t* t, int slots, int words, uint64_t pk) {
  const int32_t i = lds_group_find(t, slots, words, pk);
  return i < 0 ? nullptr : t + i * words;
}

// Adds `cnt` rows (default one) with accumulator contributions acc[] to
// LDS slot s.
__device__ __forceinline__ void lds_group_update(uint64_t* s, const AccPlan& ap, const uint64_t* acc,
                                                 uint64_t cnt = 1) {
  atomicAdd(reinterpret_cast<unsigned long long*>(s + 1), static_cast<unsigned long long>(cnt));
  // unrolled to the bound so that acc[] stays in registers
#pragma unroll
  for (int a = 0; a < kMaxAcc; ++a) {
    if (a >= ap.nacc) break;
    uint64_t* w = s + 2 + a;
    if (ap.kind[a] == kAccSum) {
      atomicAdd(reinterpret_cast<unsigned long long*>(w), static_cast<unsigned long long>(acc[a]));
    } else if (ap.kind[a] == kAccMin) {
      if (static_cast<long long>(acc[a]) < *reinterpret_cast<long long*>(w))
        atomicMin(reinterpret_cast<long long*>(w), static_cast<long long>(acc[a]));
    } else {
      if (static_cast<long long>(acc[a]) > *reinterpret_cast<long long*>(w))
        atomicMax(reinterpret_cast<long long*>(w), static_cast<long long>(acc[a]));
    }
  }
}

// Merges a workgroup's LDS table into its replica of the global table (call
// after a barrier).
__device__ __forceinline__ void lds_group_flush(const uint64_t* t, int slots, const GroupDesc& g) {
  const GroupTable gt = group_replica(g, blockIdx.x % g.replicas);
  for (int i = threadIdx.x; i < slots; i += blockDim.x) {
    const uint64_t* s = t + i * g.words;
    if (s[0] == kEmpty64) continue;
    uint64_t* d = group_slot(gt, s[0]);
    if (d) group_update_global(d, g.ap, s[1], s + 2);
  }
}

}  // namespace rel
