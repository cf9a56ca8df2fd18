// Hash group-by on a variable-length string key, optionally with one integer
// key beside it: the group-by cost the paper reports on string-keyed
// ClickBench queries (Section 4.2), done on the hash path rather than by
// sorting. Strings come in the Arrow layout (row i = bytes[offsets[i] ..
// offsets[i+1])), directly or dictionary-encoded (row i = dictionary entry
// codes[i]); either way the group key is the string's bytes, so equal
// strings under different codes fall into one group.
//
// Slots of the open-addressing table (words of 64 bits): [0] the claim word,
// [1] COUNT, [2] the smallest row id of the group, then the accumulators.
// The claim word packs a 32-bit key tag over the row whose insert claimed the
// slot, in one 64-bit CAS (a reader never waits for a second store). Arrow
// layout: the tag is 32 bits of the string's hash, and a row that meets an
// equal tag compares its string (and integer key) with the claiming row's,
// so hash collisions never merge groups. Dictionary layout: the tag is the
// canonical dictionary id itself (below), exact by construction; only an
// integer key, if any, is compared through the claiming row.
//
// Dictionary-encoded columns are canonicalised first: one pass over the
// dictionary gives every entry the id of an entry with equal bytes (the one
// whose insert claimed the string's slot in a table of the dictionary's
// strings), so a row's key is then the integer pair (canonical id, integer
// key) and the per-row work has no string hashing or comparison. Without an
// integer key, when the group table has room for every dictionary string,
// the slots are claimed per canonical entry up front and a row only reads
// its entry's slot.
//
// Pre-aggregation in LDS: each workgroup keeps a small direct-mapped table
// keyed by global slot index; a row whose slot has (or claims) one of its
// two LDS candidates updates LDS with shared-memory atomics, any other row
// updates the global slot. The LDS tables are added into their global
// slots when the workgroup ends, so a hot key costs one set of global
// atomics per workgroup instead of one per row (same-address global atomics
// serialise, and a Zipf-skewed key column sends most rows to a few slots).

#include "internal.h"

namespace rel {

namespace {

constexpr int kStrThreads = 256;

// String row i of the key column: byte offset and length.
__device__ __forceinline__ void str_span(const StrGroupParams& p, int64_t row, int64_t& off,
                                         int64_t& len) {
  const int64_t e = p.codes ? static_cast<int64_t>(p.codes[row]) : row;
  off = p.offsets[e];
  len = p.offsets[e + 1] - off;
}

// Four string bytes from byte position a (little-endian), read as aligned
// words: both words hold bytes of the string, so they lie inside the buffer.
__device__ __forceinline__ uint32_t str_word(const uint8_t* bytes, int64_t a) {
  const uint32_t* w = reinterpret_cast<const uint32_t*>(bytes + (a & ~int64_t(3)));
  const uint32_t m = static_cast<uint32_t>(a & 3);
  const uint32_t lo = w[0];
  if (m == 0) return lo;
  const uint32_t hi = w[1];
  return (lo >> (8 * m)) | (hi << (32 - 8 * m));
}

__device__ __forceinline__ uint32_t str_byte(const uint8_t* bytes, int64_t a) { return bytes[a]; }

// 64-bit hash of the string bytes (whole 32-bit words, then the tail bytes,
// then the length), mixed with the integer key.
__device__ __forceinline__ uint64_t str_hash(const uint8_t* bytes, int64_t off, int64_t len,
                                             int64_t ikey) {
  uint64_t h = 0x243f6a8885a308d3ULL ^ static_cast<uint64_t>(len);
  int64_t k = 0;
  for (; k + 4 <= len; k += 4) {
    h ^= str_word(bytes, off + k);
    h *= 0x9e3779b97f4a7c15ULL;
    h ^= h >> 29;
  }
  for (; k < len; ++k) {
    h ^= str_byte(bytes, off + k) << (8 * (k & 3));
    h *= 0x9e3779b97f4a7c15ULL;
    h ^= h >> 29;
  }
  return hash64(h ^ hash64(static_cast<uint64_t>(ikey) + 0x13198a2e03707344ULL));
}

__device__ __forceinline__ bool str_equal(const uint8_t* bytes, int64_t oa, int64_t ob, int64_t len) {
  int64_t k = 0;
  for (; k + 4 <= len; k += 4)
    if (str_word(bytes, oa + k) != str_word(bytes, ob + k)) return false;
  for (; k < len; ++k)
    if (bytes[oa + k] != bytes[ob + k]) return false;
  return true;
}

__device__ __forceinline__ int64_t str_ikey(const StrGroupParams& p, int64_t row) {
  return p.ikey ? load_elem(p.ikey, p.ikey_type, row) : 0;
}

constexpr uint64_t kStrEmpty = ~0ULL;

// The slot index of row `row` (claiming an empty slot if its key is new), or
// -1 if the table is full.
__device__ __forceinline__ int64_t str_slot(const StrGroupParams& p, int64_t row) {
  int64_t off, len;
  str_span(p, row, off, len);
  const int64_t ik = str_ikey(p, row);
  const uint64_t h = str_hash(p.bytes, off, len, ik);
  const uint64_t mine = (static_cast<uint64_t>(static_cast<uint32_t>(h >> 32)) << 32) |
                        static_cast<uint32_t>(row);
  uint64_t s = h & p.mask;
  for (uint64_t probes = 0; probes <= p.mask; ++probes) {
    uint64_t* w = p.slots + s * p.words;
    uint64_t cur = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == kStrEmpty) {
      const unsigned long long prev =
          atomicCAS(reinterpret_cast<unsigned long long*>(w), static_cast<unsigned long long>(kStrEmpty),
                    static_cast<unsigned long long>(mine));
      if (prev == kStrEmpty) return static_cast<int64_t>(s);
      cur = prev;
    }
    if ((cur >> 32) == (mine >> 32)) {
      const int64_t other = static_cast<int64_t>(static_cast<uint32_t>(cur));
      int64_t ooff, olen;
      str_span(p, other, ooff, olen);
      if (olen == len && str_ikey(p, other) == ik && str_equal(p.bytes, off, ooff, len))
        return static_cast<int64_t>(s);
    }
    s = (s + 1) & p.mask;
  }
  atomicOr(p.overflow, 1);
  return -1;
}

// Canonical id of every dictionary entry: the entry whose insert claimed
// the entry's string in a table of the dictionary's strings (claim word:
// 32-bit string hash << 32 | entry). The table holds at least twice as many
// slots as entries, so every probe sequence ends.
__global__ void __launch_bounds__(kStrThreads) dict_canon_kernel(StrGroupParams p) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kStrThreads + threadIdx.x; e < p.n_dict;
       e += static_cast<int64_t>(gridDim.x) * kStrThreads) {
    const int64_t off = p.offsets[e];
    const int64_t len = p.offsets[e + 1] - off;
    const uint64_t h = str_hash(p.bytes, off, len, 0);
    const uint64_t mine = (h >> 32 << 32) | static_cast<uint32_t>(e);
    uint32_t canon = static_cast<uint32_t>(e);
    uint64_t s = h & p.dict_mask;
    for (uint64_t probes = 0; probes <= p.dict_mask; ++probes) {
      uint64_t* w = p.dict_slots + s;
      uint64_t cur = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (cur == kStrEmpty) {
        const unsigned long long prev =
            atomicCAS(reinterpret_cast<unsigned long long*>(w), static_cast<unsigned long long>(kStrEmpty),
                      static_cast<unsigned long long>(mine));
        if (prev == kStrEmpty) break;
        cur = prev;
      }
      if ((cur >> 32) == (mine >> 32)) {
        const int64_t other = static_cast<int64_t>(static_cast<uint32_t>(cur));
        const int64_t ooff = p.offsets[other];
        if (p.offsets[other + 1] - ooff == len && str_equal(p.bytes, off, ooff, len)) {
          canon = static_cast<uint32_t>(other);
          break;
        }
      }
      s = (s + 1) & p.dict_mask;
    }
    p.canon[e] = canon;
  }
}

// The slot index of dictionary-encoded row `row`, keyed by (canonical id,
// integer key), claiming an empty slot if the key is new; -1 if the table is
// full. Canonical ids and row ids stay below 2^32 - 1, so a claim word never
// equals the empty pattern.
__device__ __forceinline__ int64_t dict_slot(const StrGroupParams& p, int64_t row) {
  const uint32_t c = p.canon[p.codes[row]];
  const int64_t ik = str_ikey(p, row);
  const uint64_t h =
      hash64((static_cast<uint64_t>(c) << 32 | c) ^ hash64(static_cast<uint64_t>(ik) + 0x13198a2e03707344ULL));
  const uint64_t mine = (static_cast<uint64_t>(c) << 32) | static_cast<uint32_t>(row);
  uint64_t s = h & p.mask;
  for (uint64_t probes = 0; probes <= p.mask; ++probes) {
    uint64_t* w = p.slots + s * p.words;
    uint64_t cur = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == kStrEmpty) {
      const unsigned long long prev =
          atomicCAS(reinterpret_cast<unsigned long long*>(w), static_cast<unsigned long long>(kStrEmpty),
                    static_cast<unsigned long long>(mine));
      if (prev == kStrEmpty) return static_cast<int64_t>(s);
      cur = prev;
    }
    if ((cur >> 32) == c && (!p.ikey || str_ikey(p, static_cast<uint32_t>(cur)) == ik))
      return static_cast<int64_t>(s);
    s = (s + 1) & p.mask;
  }
  atomicOr(p.overflow, 1);
  return -1;
}

// Without an integer key, and with room in the group table for every
// string of the dictionary, rows need no probe at all: the group slot of each
// canonical entry is claimed once up front, every entry learns its string's
// slot, and a row's slot is one read, slot_of[codes[row]]. Slots of
// dictionary strings that no row uses keep COUNT 0 and are not groups.
__global__ void __launch_bounds__(kStrThreads) dict_claim_kernel(StrGroupParams p) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kStrThreads + threadIdx.x; e < p.n_dict;
       e += static_cast<int64_t>(gridDim.x) * kStrThreads) {
    const uint32_t c = p.canon[e];
    if (c != static_cast<uint32_t>(e)) continue;  // not the canonical entry of its string
    const uint64_t h = hash64(static_cast<uint64_t>(c) << 32 | c);
    const uint64_t mine = static_cast<uint64_t>(c) << 32;
    uint64_t slot = h & p.mask;
    // at least twice as many slots as dictionary entries: every run ends
    for (uint64_t probes = 0; probes <= p.mask; ++probes) {
      uint64_t* w = p.slots + slot * p.words;
      const unsigned long long prev =
          atomicCAS(reinterpret_cast<unsigned long long*>(w), static_cast<unsigned long long>(kStrEmpty),
                    static_cast<unsigned long long>(mine));
      if (prev == kStrEmpty) break;
      slot = (slot + 1) & p.mask;
    }
    p.slot_of[e] = static_cast<uint32_t>(slot);
  }
}

// Every other entry takes the slot of its string's canonical entry.
__global__ void __launch_bounds__(kStrThreads) dict_alias_kernel(StrGroupParams p) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kStrThreads + threadIdx.x; e < p.n_dict;
       e += static_cast<int64_t>(gridDim.x) * kStrThreads) {
    const uint32_t c = p.canon[e];
    if (c != static_cast<uint32_t>(e)) p.slot_of[e] = p.slot_of[c];
  }
}

// Adds `cnt` rows with first row `first` and accumulator inputs acc[] to slot s.
__device__ __forceinline__ void str_update(const StrGroupParams& p, int64_t s, uint64_t cnt,
                                           uint64_t first, const int64_t* acc) {
  uint64_t* w = p.slots + s * p.words;
  atomicAdd(reinterpret_cast<unsigned long long*>(w + 1), static_cast<unsigned long long>(cnt));
  atomicMin(reinterpret_cast<unsigned long long*>(w + 2), static_cast<unsigned long long>(first));
#pragma unroll
  for (int a = 0; a < kMaxAcc; ++a) {
    if (a >= p.ap.nacc) break;
    uint64_t* x = w + 3 + a;
    if (p.ap.kind[a] == kAccSum)
      atomicAdd(reinterpret_cast<unsigned long long*>(x), static_cast<unsigned long long>(acc[a]));
    else if (p.ap.kind[a] == kAccMin)
      atomicMin(reinterpret_cast<long long*>(x), static_cast<long long>(acc[a]));
    else
      atomicMax(reinterpret_cast<long long*>(x), static_cast<long long>(acc[a]));
  }
}

__global__ void __launch_bounds__(kStrThreads) str_init_kernel(StrGroupParams p) {
  const uint64_t total = (p.mask + 1) * static_cast<uint64_t>(p.words);
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kStrThreads + threadIdx.x; i < total;
       i += static_cast<uint64_t>(gridDim.x) * kStrThreads) {
    const int w = static_cast<int>(i % p.words);
    uint64_t v = 0;
    if (w == 0 || w == 2) v = kStrEmpty;
    else if (w >= 3) v = acc_identity(p.ap.kind[w - 3]);
    p.slots[i] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *p.overflow = 0;
    *p.d_groups = 0;
  }
}

constexpr uint32_t kLdsEmpty = ~0u;

// LDS pre-aggregation table of a workgroup (K entries): COUNT (K words),
// accumulators (nacc x K words), global slot index (K), smallest row (K).
struct StrLds {
  uint64_t* cnt;
  uint64_t* acc;
  uint32_t* key;
  uint32_t* first;
};

// kMode 0: Arrow strings (hash and compare bytes); 1: dictionary codes,
// keyed by (canonical id, integer key); 2: dictionary codes with the slots
// claimed up front (no integer key).
template <int kMode>
__global__ void __launch_bounds__(kStrThreads) str_agg_kernel(StrGroupParams p) {
  extern __shared__ uint64_t str_lds[];
  const uint32_t K = static_cast<uint32_t>(p.lds_slots);
  const int nacc = p.ap.nacc;
  StrLds t;
  t.cnt = str_lds;
  t.acc = str_lds + K;
  t.key = reinterpret_cast<uint32_t*>(str_lds + static_cast<uint64_t>(K) * (1 + nacc));
  t.first = t.key + K;
  for (uint32_t i = threadIdx.x; i < K; i += kStrThreads) {
    t.cnt[i] = 0;
    t.key[i] = kLdsEmpty;
    t.first[i] = kLdsEmpty;
    for (int a = 0; a < nacc; ++a) t.acc[a * K + i] = acc_identity(p.ap.kind[a]);
  }
  __syncthreads();

  const uint64_t n = static_cast<uint64_t>(p.n);
  const uint64_t step = static_cast<uint64_t>(gridDim.x) * kStrThreads;
  for (uint64_t row = static_cast<uint64_t>(blockIdx.x) * kStrThreads + threadIdx.x; row < n;
       row += step) {
    const int64_t slot = kMode == 2 ? static_cast<int64_t>(p.slot_of[p.codes[row]])
                       : kMode == 1 ? dict_slot(p, static_cast<int64_t>(row))
                                    : str_slot(p, static_cast<int64_t>(row));
    if (slot < 0) continue;
    int64_t acc[kMaxAcc];
#pragma unroll
    for (int a = 0; a < kMaxAcc; ++a)
      acc[a] = a < nacc ? load_elem(p.val[p.ap.col[a]], p.val_type[p.ap.col[a]], static_cast<int64_t>(row))
                        : 0;
    bool done = false;
    if (K != 0) {
      const uint32_t s32 = static_cast<uint32_t>(slot);
      for (uint32_t probe = 0; probe < 2 && !done; ++probe) {
        const uint32_t i = (s32 + probe) & (K - 1);
        uint32_t cur = __hip_atomic_load(&t.key[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == kLdsEmpty) {
          cur = atomicCAS(&t.key[i], kLdsEmpty, s32);
          if (cur == kLdsEmpty) cur = s32;
        }
        if (cur == s32) {
          atomicAdd(reinterpret_cast<unsigned long long*>(&t.cnt[i]), 1ULL);
          atomicMin(&t.first[i], static_cast<uint32_t>(row));
#pragma unroll
          for (int a = 0; a < kMaxAcc; ++a)
            if (a < nacc) lds_acc_update(&t.acc[a * K + i], p.ap.kind[a], acc[a]);
          done = true;
        }
      }
    }
    if (!done) str_update(p, slot, 1, row, acc);
  }

  // the workgroup's LDS table into the global slots
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < K; i += kStrThreads) {
    const uint32_t key = t.key[i];
    if (key == kLdsEmpty) continue;
    int64_t acc[kMaxAcc];
#pragma unroll
    for (int a = 0; a < kMaxAcc; ++a) acc[a] = a < nacc ? static_cast<int64_t>(t.acc[a * K + i]) : 0;
    str_update(p, key, t.cnt[i], t.first[i], acc);
  }
}

__global__ void __launch_bounds__(kStrThreads) str_final_kernel(StrGroupParams p) {
  const int lane = lane_id();
  const uint64_t slots = p.mask + 1;
  const uint64_t step = static_cast<uint64_t>(gridDim.x) * kStrThreads;
  for (uint64_t base = static_cast<uint64_t>(blockIdx.x) * kStrThreads + threadIdx.x - lane;
       base < slots; base += step) {
    const uint64_t s = base + lane;
    const uint64_t* w = p.slots + (s < slots ? s : 0) * p.words;
    // a slot claimed for a dictionary string that no row uses has COUNT 0
    const bool used = s < slots && w[0] != kStrEmpty && w[1] != 0;
    const uint64_t m = ballot(used);
    if (m == 0) continue;
    unsigned long long at = 0;
    if (lane == __ffsll(static_cast<long long>(m)) - 1)
      at = atomicAdd(p.d_groups, static_cast<unsigned long long>(popc64(m)));
    at = __shfl(at, __ffsll(static_cast<long long>(m)) - 1, kWave);
    if (!used) continue;
    const int64_t g = static_cast<int64_t>(at + rank_below(m));
    if (g >= p.cap) continue;
    const uint64_t cnt = w[1];
    const uint32_t first = static_cast<uint32_t>(w[2]);
    p.out_rows[g] = first;
    if (p.ikey && p.out_ikey) store_elem(p.out_ikey, p.ikey_type, g, str_ikey(p, first));
    for (int a = 0; a < p.naggs; ++a) {
      int64_t v;
      if (p.agg_op[a] == 1) {  // COUNT
        v = static_cast<int64_t>(cnt);
      } else if (p.agg_op[a] == 4) {  // AVG: one binary64 division of the exact values
        const double q = static_cast<double>(static_cast<int64_t>(w[3 + p.agg_acc[a]])) /
                         static_cast<double>(cnt);
        v = __double_as_longlong(q);
      } else {
        v = static_cast<int64_t>(w[3 + p.agg_acc[a]]);
      }
      static_cast<int64_t*>(p.out_aggs[a])[g] = v;
    }
  }
}

__global__ void str_overflow_kernel(StrGroupParams p) {
  if (*p.overflow) *p.d_groups = static_cast<unsigned long long>(-1LL);
}

}  // namespace

template <int kMode>
void launch_str_agg(const StrGroupParams& p, hipStream_t s) {
  const size_t lds = static_cast<size_t>(p.lds_slots) * (16 + 8 * static_cast<size_t>(p.ap.nacc));
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, str_agg_kernel<kMode>, kStrThreads, lds) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  // every workgroup flushes its whole LDS table once: as many as are resident
  uint64_t blocks = (static_cast<uint64_t>(p.n) + kStrThreads - 1) / kStrThreads;
  const uint64_t limit = static_cast<uint64_t>(device_info().cu_count) * per_cu;
  if (blocks > limit) blocks = limit;
  hipLaunchKernelGGL(str_agg_kernel<kMode>, dim3(static_cast<unsigned>(blocks)), dim3(kStrThreads), lds,
                     s, p);
}

void launch_groupby_str(const StrGroupParams& p, hipStream_t s) {
  {
    ProfileScope ps(kKFill, s);
    const uint64_t total = (p.mask + 1) * static_cast<uint64_t>(p.words);
    uint64_t blocks = (total + kStrThreads - 1) / kStrThreads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(str_init_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kStrThreads), 0, s,
                       p);
  }
  if (p.codes && p.n > 0) launch_fill64(p.dict_slots, p.dict_mask + 1, kStrEmpty, s);
  {
    ProfileScope ps(kKGroupAgg, s);
    if (p.n > 0) {
      if (p.codes) {
        uint64_t blocks = (static_cast<uint64_t>(p.n_dict) + kStrThreads - 1) / kStrThreads;
        if (blocks > 8192) blocks = 8192;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(dict_canon_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kStrThreads), 0,
                           s, p);
        if (!p.ikey && static_cast<uint64_t>(p.n_dict) * 2 <= p.mask + 1) {
          hipLaunchKernelGGL(dict_claim_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kStrThreads),
                             0, s, p);
          hipLaunchKernelGGL(dict_alias_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kStrThreads),
                             0, s, p);
          launch_str_agg<2>(p, s);
        } else {
          launch_str_agg<1>(p, s);
        }
      } else {
        launch_str_agg<0>(p, s);
      }
    }
  }
  {
    ProfileScope ps(kKFinalize, s);
    uint64_t blocks = (p.mask + 1 + kStrThreads - 1) / kStrThreads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(str_final_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kStrThreads), 0,
                       s, p);
    hipLaunchKernelGGL(str_overflow_kernel, dim3(1), dim3(1), 0, s, p);
  }
}

}  // namespace rel
