// Device helpers shared by the gfx950 kernels: hashing, wave64 ballot
// arithmetic, typed column access and the open-addressing slot formats.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rel {

constexpr int kWave = 64;

// Key sentinel of every hash table: a slot whose key word holds it is empty.
// A real key equal to it never enters the open-addressing array; it goes to
// an out-of-band area instead, so the key domain is not restricted.
constexpr int32_t kEmpty32 = INT32_MIN;
constexpr uint64_t kEmpty64 = 0x8000000000000000ULL;

// MurmurHash3 finalisers (Appleby, public domain): full avalanche, cheap.
__device__ __forceinline__ uint32_t hash32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

__device__ __forceinline__ uint64_t hash64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Number of set bits of `m` held by lanes below this one.
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return __popcll(m); }

template <typename T>
__device__ __forceinline__ T first_lane(T v) {
  return __shfl(v, 0, kWave);
}

// 64-bit atomic adds whose address space is explicit, so that the compiler
// emits ds_add (LDS) or global_atomic_add (HBM) rather than one generic flat
// atomic for a pointer that may be either.
__device__ __forceinline__ void lds_add_u64(uint64_t* p, uint64_t v) {
  typedef __attribute__((address_space(3))) uint64_t LdsU64;
  __atomic_fetch_add((LdsU64*)p, v, __ATOMIC_RELAXED);
}

__device__ __forceinline__ uint32_t lds_fetch_add_u32(uint32_t* p, uint32_t v) {
  typedef __attribute__((address_space(3))) uint32_t LdsU32;
  return __atomic_fetch_add((LdsU32*)p, v, __ATOMIC_RELAXED);
}

__device__ __forceinline__ void global_add_u64(uint64_t* p, uint64_t v) {
  typedef __attribute__((address_space(1))) uint64_t GlobalU64;
  __hip_atomic_fetch_add((GlobalU64*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Agent-scope atomic loads/stores: coherent across the eight XCD L2s.
__device__ __forceinline__ uint64_t load_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Column element types (numerically equal to rel_dtype).
enum : int32_t { kI8 = 1, kI32 = 2, kI64 = 3 };

__device__ __forceinline__ int64_t load_elem(const void* p, int32_t type, int64_t i) {
  if (type == kI32) return static_cast<const int32_t*>(p)[i];
  if (type == kI64) return static_cast<const int64_t*>(p)[i];
  return static_cast<const int8_t*>(p)[i];
}

// Four consecutive elements starting at r0 (a multiple of 4) of a plain
// column, with one vector load when the chunk is whole and the column is
// 16-byte aligned (`vec`).
__device__ __forceinline__ void load4(const void* p, int32_t type, bool vec, int64_t r0,
                                      int64_t n, int64_t v[4]) {
  if (vec && r0 + 4 <= n) {
    if (type == kI32) {
      int4 x = *reinterpret_cast<const int4*>(static_cast<const int32_t*>(p) + r0);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else if (type == kI64) {
      const longlong2* q = reinterpret_cast<const longlong2*>(static_cast<const int64_t*>(p) + r0);
      longlong2 a = q[0], b = q[1];
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
      int32_t w = *reinterpret_cast<const int32_t*>(static_cast<const int8_t*>(p) + r0);
      v[0] = static_cast<int8_t>(w); v[1] = static_cast<int8_t>(w >> 8);
      v[2] = static_cast<int8_t>(w >> 16); v[3] = static_cast<int8_t>(w >> 24);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (r0 + e < n) ? load_elem(p, type, r0 + e) : 0;
  }
}

// As load4, for columns read once: the vector loads are marked
// non-temporal so that streamed data does not displace hash tables in the
// caches.
__device__ __forceinline__ void load4s(const void* p, int32_t type, bool vec, int64_t r0,
                                       int64_t n, int64_t v[4]) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  typedef long long v2l __attribute__((ext_vector_type(2)));
  if (vec && r0 + 4 <= n) {
    if (type == kI32) {
      const v4i x = __builtin_nontemporal_load(
          reinterpret_cast<const v4i*>(static_cast<const int32_t*>(p) + r0));
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else if (type == kI64) {
      const v2l* q = reinterpret_cast<const v2l*>(static_cast<const int64_t*>(p) + r0);
      const v2l a = __builtin_nontemporal_load(q), b = __builtin_nontemporal_load(q + 1);
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
      const int32_t w = __builtin_nontemporal_load(
          reinterpret_cast<const int32_t*>(static_cast<const int8_t*>(p) + r0));
      v[0] = static_cast<int8_t>(w); v[1] = static_cast<int8_t>(w >> 8);
      v[2] = static_cast<int8_t>(w >> 16); v[3] = static_cast<int8_t>(w >> 24);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (r0 + e < n) ? load_elem(p, type, r0 + e) : 0;
  }
}

// As load4s for int8 and int32 columns, holding the values as int32.
__device__ __forceinline__ void load4n(const void* p, int32_t type, bool vec, int64_t r0,
                                       int64_t n, int32_t v[4]) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  if (vec && r0 + 4 <= n) {
    if (type == kI32) {
      const v4i x = __builtin_nontemporal_load(
          reinterpret_cast<const v4i*>(static_cast<const int32_t*>(p) + r0));
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else {
      const int32_t w = __builtin_nontemporal_load(
          reinterpret_cast<const int32_t*>(static_cast<const int8_t*>(p) + r0));
      v[0] = static_cast<int8_t>(w); v[1] = static_cast<int8_t>(w >> 8);
      v[2] = static_cast<int8_t>(w >> 16); v[3] = static_cast<int8_t>(w >> 24);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      v[e] = (r0 + e < n) ? static_cast<int32_t>(load_elem(p, type, r0 + e)) : 0;
  }
}

// Comparison term on a widened value (operators numerically equal to rel_cmp).
__device__ __forceinline__ bool term_holds(int32_t op, int64_t v, int64_t lo, int64_t hi) {
  switch (op) {
    case 0: return v < lo;
    case 1: return v <= lo;
    case 2: return v > lo;
    case 3: return v >= lo;
    case 4: return v == lo;
    case 5: return v != lo;
    default: return v >= lo && v < hi;
  }
}

// ---------------------------------------------------------- Bloom filters
//
// Blocked Bloom filter over int32/int64 keys (blocked filters: Putze, Sanders
// and Singler, "Cache-, Hash- and Space-Efficient Bloom Filters", 2007): a
// power-of-two number of 32-byte blocks, each eight 32-bit words. A key's
// 64-bit hash picks one block (high half) and, in each of the block's eight
// words, one bit (five bits of the low half times a per-word odd multiplier),
// so a test reads one 32-byte sector. Keys are widened to int64 before
// hashing, so an int32 key and the int64 key of equal value hash alike.

struct BloomDesc {
  const uint32_t* words;  // blocks * 8 words
  uint64_t bmask;         // blocks - 1
};

// Odd multipliers: the high halves of the first eight outputs of SplitMix64
// from state 0, each made odd.
__device__ __forceinline__ uint32_t bloom_salt(int w) {
  switch (w) {
    case 0: return 0xe220a839u;
    case 1: return 0x6e789e6bu;
    case 2: return 0x06c45d19u;
    case 3: return 0xf88bb8a9u;
    case 4: return 0x1b39896bu;
    case 5: return 0x53cb9f0du;
    case 6: return 0x2c829abfu;
    default: return 0xc584133bu;
  }
}

__device__ __forceinline__ uint64_t bloom_hash(int64_t key) {
  return hash64(static_cast<uint64_t>(key) ^ 0x6a09e667f3bcc909ULL);
}

__device__ __forceinline__ uint64_t bloom_block(uint64_t h, uint64_t bmask) {
  return (h >> 32) & bmask;
}

__device__ __forceinline__ uint32_t bloom_bit(uint64_t h, int w) {
  return 1u << ((static_cast<uint32_t>(h) * bloom_salt(w)) >> 27);
}

// Whether the block q (words 0-3 in a, 4-7 in b) holds every bit of hash h.
__device__ __forceinline__ bool bloom_match(uint64_t h, uint4 a, uint4 b) {
  return ((a.x & bloom_bit(h, 0)) != 0) & ((a.y & bloom_bit(h, 1)) != 0) &
         ((a.z & bloom_bit(h, 2)) != 0) & ((a.w & bloom_bit(h, 3)) != 0) &
         ((b.x & bloom_bit(h, 4)) != 0) & ((b.y & bloom_bit(h, 5)) != 0) &
         ((b.z & bloom_bit(h, 6)) != 0) & ((b.w & bloom_bit(h, 7)) != 0);
}

// ---------------------------------------------------------------- hash maps
//
// Multimap key -> 32-bit value with linear probing over a power-of-two slot
// array. int32 keys: one 64-bit word per slot, key in the low half and value
// in the high half, published by a single 64-bit CAS. int64 keys: 16-byte
// slots {key, value, pad}; the key word is claimed by CAS and the value is
// stored after it (readers only run in later kernels). Entries whose key is
// the sentinel are appended to an out-of-band list {count, values[]}.

struct Map32 {
  uint64_t* slots;
  uint64_t mask;
  unsigned long long* oob_count;
  uint32_t* oob_vals;
};

struct Map64 {
  ulonglong2* slots;  // .x = key bits, .y = value (low 32 bits)
  uint64_t mask;
  unsigned long long* oob_count;
  uint32_t* oob_vals;
};

// Probe runs start at the first slot of the 16-byte bucket holding the hash
// slot, so one aligned 16-byte read covers the first two key/value slots (or
// four key-only slots) of every run. Key/value maps take their home slot from
// the top hash bits, so that the keys of one range of the slot array share a
// hash prefix (the partitioned build builds each range on its own).
__device__ __forceinline__ uint64_t home32(int32_t key, uint64_t mask) {
  const uint64_t h = hash32(static_cast<uint32_t>(key));
  const int sh = __clzll(static_cast<long long>(mask | 1)) - 32;  // 32 - log2(slots)
  return ((sh >= 0 ? h >> sh : h << -sh) & mask) & ~1ULL;
}
__device__ __forceinline__ uint64_t home_set(int32_t key, uint64_t mask) {
  return (hash32(static_cast<uint32_t>(key)) & mask) & ~3ULL;
}
__device__ __forceinline__ uint64_t home64(int64_t key, uint64_t mask) {
  return mask ? hash64(static_cast<uint64_t>(key)) >> __clzll(static_cast<long long>(mask)) : 0;
}

__device__ __forceinline__ uint64_t pack32(int32_t key, uint32_t val) {
  return static_cast<uint64_t>(static_cast<uint32_t>(key)) | (static_cast<uint64_t>(val) << 32);
}

constexpr uint64_t kEmptySlot32 = 0x0000000080000000ULL;  // pack32(kEmpty32, 0)

// Inserts report a duplicate key through *dup: a CAS that loses returns the
// occupant, and an equal occupant on the probe path is a duplicate.
__device__ __forceinline__ void map_insert(const Map32& m, int32_t key, uint32_t val, int32_t* dup) {
  if (key == kEmpty32) {
    unsigned long long pos = atomicAdd(m.oob_count, 1ULL);
    m.oob_vals[pos] = val;
    if (pos > 0) *dup = 1;
    return;
  }
  uint64_t h = home32(key, m.mask);
  const unsigned long long want = pack32(key, val);
  while (true) {
    unsigned long long prev = atomicCAS(reinterpret_cast<unsigned long long*>(m.slots + h),
                                        static_cast<unsigned long long>(kEmptySlot32), want);
    if (prev == kEmptySlot32) return;
    if (static_cast<int32_t>(static_cast<uint32_t>(prev)) == key) *dup = 1;
    h = (h + 1) & m.mask;
  }
}

__device__ __forceinline__ void map_insert(const Map64& m, int64_t key, uint32_t val, int32_t* dup) {
  if (static_cast<uint64_t>(key) == kEmpty64) {
    unsigned long long pos = atomicAdd(m.oob_count, 1ULL);
    m.oob_vals[pos] = val;
    if (pos > 0) *dup = 1;
    return;
  }
  uint64_t h = home64(key, m.mask);
  while (true) {
    unsigned long long* kw = reinterpret_cast<unsigned long long*>(&m.slots[h].x);
    unsigned long long prev = atomicCAS(kw, static_cast<unsigned long long>(kEmpty64),
                                        static_cast<unsigned long long>(key));
    if (prev == kEmpty64) {
      m.slots[h].y = val;
      return;
    }
    if (static_cast<int64_t>(prev) == key) *dup = 1;
    h = (h + 1) & m.mask;
  }
}

// Key-only multiset of int32 keys (membership dims): one 32-bit word per
// slot, claimed by a 32-bit CAS; sentinel keys are only counted out of band.
__device__ __forceinline__ void set_insert(uint32_t* slots, uint64_t mask,
                                           unsigned long long* oob_count, int32_t key,
                                           int32_t* dup) {
  if (key == kEmpty32) {
    if (atomicAdd(oob_count, 1ULL) > 0) *dup = 1;
    return;
  }
  uint64_t h = home_set(key, mask);
  while (true) {
    uint32_t prev = atomicCAS(slots + h, static_cast<uint32_t>(kEmpty32), static_cast<uint32_t>(key));
    if (prev == static_cast<uint32_t>(kEmpty32)) return;
    if (static_cast<int32_t>(prev) == key) *dup = 1;
    h = (h + 1) & mask;
  }
}

// ---------------------------------------------------------- compact sets
//
// Exact multiset of int32 keys in 16-bit entries, for large membership dims.
// hash32 (the MurmurHash3 finaliser) is a bijection on 32-bit words, so a key
// is determined by its home bucket (the top `32 - rbits` hash bits) and the
// remaining `rbits` <= 14 hash bits. A bucket is 16 bytes: eight entries of
// (displacement:2 | remainder:14); 0xFFFF marks an empty entry. A key lives in
// its home bucket or one of the next two (displacement 1, 2); a key finding
// no room there goes to an out-of-band key list. Reading the home bucket with
// one 16-byte load resolves nearly every probe, from a table of two bytes per
// slot (4 MB for 1.5M keys).

constexpr uint32_t kCsetEmpty = 0xFFFFu;
constexpr int kCsetMaxDisp = 2;

struct CsetDesc {
  uint32_t* words;     // buckets * 4 words
  uint64_t bmask;      // buckets - 1
  int32_t rbits;       // remainder bits (<= 14)
  int32_t* dup;
  // Keys that find no room within the displacement window go to a plain
  // key-only set (4-byte slots) with its own sentinel count.
  uint32_t* over;
  uint64_t over_mask;
  unsigned long long* over_sentinel;
};

__device__ __forceinline__ void cset_split(const CsetDesc& c, int32_t key, uint64_t& b, uint32_t& r) {
  const uint32_t h = hash32(static_cast<uint32_t>(key));
  b = (h >> c.rbits) & c.bmask;
  r = h & ((1u << c.rbits) - 1u);
}

__device__ __forceinline__ void cset_insert(const CsetDesc& c, int32_t key) {
  uint64_t b0;
  uint32_t r;
  cset_split(c, key, b0, r);
  for (int d = 0; d <= kCsetMaxDisp; ++d) {
    uint32_t* w = c.words + ((b0 + d) & c.bmask) * 4;
    const uint32_t mine = (static_cast<uint32_t>(d) << 14) | r;
    for (int i = 0; i < 4; ++i) {
      uint32_t cur = __hip_atomic_load(w + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      while (true) {
        const uint32_t lo = cur & 0xFFFFu, hi = cur >> 16;
        if (lo == mine || hi == mine) *c.dup = 1;
        uint32_t want;
        if (lo == kCsetEmpty) want = (cur & 0xFFFF0000u) | mine;
        else if (hi == kCsetEmpty) want = (cur & 0x0000FFFFu) | (mine << 16);
        else break;  // both entries taken: next word
        const uint32_t prev = atomicCAS(w + i, cur, want);
        if (prev == cur) return;
        cur = prev;  // lost a race: re-examine the word
      }
    }
  }
  set_insert(c.over, c.over_mask, c.over_sentinel, key, c.dup);
}

// Matches of `key` in the overflow set, counted up to `limit`.
__device__ __forceinline__ int cset_over_count(const CsetDesc& c, int32_t key, int limit) {
  if (key == kEmpty32) {
    const unsigned long long n = *c.over_sentinel;
    return n < static_cast<unsigned long long>(limit) ? static_cast<int>(n) : limit;
  }
  int found = 0;
  uint64_t h = home_set(key, c.over_mask);
  while (found < limit) {
    const int32_t s = static_cast<int32_t>(c.over[h]);
    if (s == kEmpty32) break;
    found += s == key;
    h = (h + 1) & c.over_mask;
  }
  return found;
}

// Counts the entries of `key` in one 16-byte bucket at displacement d;
// `open` tells whether the bucket still has an empty entry (then no key of
// this home lies further on).
__device__ __forceinline__ int cset_bucket_count(uint4 q, uint32_t target, bool& open) {
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
  int n = 0;
  open = false;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t lo = w[i] & 0xFFFFu, hi = w[i] >> 16;
    n += (lo == target) + (hi == target);
    open |= (lo == kCsetEmpty) | (hi == kCsetEmpty);
  }
  return n;
}

// Whether one 16-byte bucket holds `target` at displacement d (for probes
// that stop at the first match), with `open` as above. The eight entries are
// compared as 16-bit pairs: the minimum of entry ^ target is zero exactly
// when some entry equals the target, and the maximum of the entries is
// kCsetEmpty exactly when one is empty (stored entries are at most
// (kCsetMaxDisp << 14) | 0x3FFF, below it).
typedef unsigned short U16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ U16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(U16x2, v); }
__device__ __forceinline__ bool cset_bucket_has(uint4 q, uint32_t target, bool& open) {
  static_assert(((static_cast<uint32_t>(kCsetMaxDisp) << 14) | 0x3FFFu) < kCsetEmpty);
  const uint32_t t2 = target * 0x10001u;
  const U16x2 m = __builtin_elementwise_min(
      __builtin_elementwise_min(as_u16x2(q.x ^ t2), as_u16x2(q.y ^ t2)),
      __builtin_elementwise_min(as_u16x2(q.z ^ t2), as_u16x2(q.w ^ t2)));
  const U16x2 e = __builtin_elementwise_max(__builtin_elementwise_max(as_u16x2(q.x), as_u16x2(q.y)),
                                            __builtin_elementwise_max(as_u16x2(q.z), as_u16x2(q.w)));
  open = (e.x == kCsetEmpty) | (e.y == kCsetEmpty);
  return (m.x == 0) | (m.y == 0);
}

// Cursor over the matches of one key: `pos` walks the probe chain (or the
// out-of-band list when `oob`); next() yields one match per call.
struct MapCursor {
  uint64_t pos;
  bool oob;
  bool live;
  bool direct;  // pipeline dims held as a direct table: pos = found << 32 | payload
};

__device__ __forceinline__ MapCursor map_start32(const Map32& m, int32_t key) {
  MapCursor c;
  c.oob = (key == kEmpty32);
  c.pos = c.oob ? 0 : home32(key, m.mask);
  c.live = true;
  c.direct = false;
  return c;
}

__device__ __forceinline__ MapCursor map_start64(const Map64& m, int64_t key) {
  MapCursor c;
  c.oob = (static_cast<uint64_t>(key) == kEmpty64);
  c.pos = c.oob ? 0 : home64(key, m.mask);
  c.live = true;
  c.direct = false;
  return c;
}

// Advances to the next match of `key`; returns false (and ends the cursor)
// when there is none. `slots` may point to an LDS copy of the table.
__device__ __forceinline__ bool map_next(const uint64_t* slots, uint64_t mask,
                                         const unsigned long long* oob_count,
                                         const uint32_t* oob_vals, int32_t key, MapCursor& c,
                                         uint32_t& val) {
  if (!c.live) return false;
  if (c.oob) {
    if (c.pos < *oob_count) {
      val = oob_vals[c.pos++];
      return true;
    }
    c.live = false;
    return false;
  }
  while (true) {
    uint64_t s = slots[c.pos];
    c.pos = (c.pos + 1) & mask;
    int32_t k = static_cast<int32_t>(static_cast<uint32_t>(s));
    if (k == kEmpty32) {
      c.live = false;
      return false;
    }
    if (k == key) {
      val = static_cast<uint32_t>(s >> 32);
      return true;
    }
  }
}

// Next occurrence of `key` in a key-only set (`val` is left unchanged).
__device__ __forceinline__ bool set_next(const uint32_t* slots, uint64_t mask,
                                         const unsigned long long* oob_count, int32_t key,
                                         MapCursor& c) {
  if (!c.live) return false;
  if (c.oob) {
    if (c.pos < *oob_count) {
      ++c.pos;
      return true;
    }
    c.live = false;
    return false;
  }
  while (true) {
    int32_t k = static_cast<int32_t>(slots[c.pos]);
    c.pos = (c.pos + 1) & mask;
    if (k == kEmpty32) {
      c.live = false;
      return false;
    }
    if (k == key) return true;
  }
}

__device__ __forceinline__ bool map_next(const ulonglong2* slots, uint64_t mask,
                                         const unsigned long long* oob_count,
                                         const uint32_t* oob_vals, int64_t key, MapCursor& c,
                                         uint32_t& val) {
  if (!c.live) return false;
  if (c.oob) {
    if (c.pos < *oob_count) {
      val = oob_vals[c.pos++];
      return true;
    }
    c.live = false;
    return false;
  }
  while (true) {
    ulonglong2 s = slots[c.pos];
    c.pos = (c.pos + 1) & mask;
    if (s.x == kEmpty64) {
      c.live = false;
      return false;
    }
    if (static_cast<int64_t>(s.x) == key) {
      val = static_cast<uint32_t>(s.y);
      return true;
    }
  }
}

// ---------------------------------------------------------- group tables
//
// A group slot is `words` 64-bit words: [0] packed key, [1] COUNT, then one
// accumulator per (op, value column): SUM adds modulo 2^64, MIN/MAX keep the
// signed extreme. The packed key of a key tuple is injective (see
// GroupKeyPack); the sentinel pattern goes to one extra slot after the array.

enum : int32_t { kAccSum = 0, kAccMin = 1, kAccMax = 2 };

// An accumulator update in an LDS group slot (SUM: add; MIN, MAX: signed).
__device__ __forceinline__ void lds_acc_update(uint64_t* p, int32_t kind, int64_t v) {
  typedef __attribute__((address_space(3))) uint64_t LdsU64;
  typedef __attribute__((address_space(3))) int64_t LdsI64;
  if (kind == kAccSum) __atomic_fetch_add((LdsU64*)p, static_cast<uint64_t>(v), __ATOMIC_RELAXED);
  else if (kind == kAccMin) __atomic_fetch_min((LdsI64*)p, v, __ATOMIC_RELAXED);
  else __atomic_fetch_max((LdsI64*)p, v, __ATOMIC_RELAXED);
}


constexpr int kMaxAcc = 8;

struct AccPlan {
  int32_t nacc;
  int32_t kind[kMaxAcc];
  int32_t col[kMaxAcc];  // index of the value column
};

struct GroupTable {
  uint64_t* slots;  // (mask + 2) slots; slot mask + 1 is the out-of-band slot
  uint64_t mask;
  int32_t words;
  int32_t* overflow;
};

__device__ __forceinline__ uint64_t acc_identity(int32_t kind) {
  return kind == kAccMin ? 0x7FFFFFFFFFFFFFFFULL : (kind == kAccMax ? 0x8000000000000000ULL : 0ULL);
}

// Finds or claims the slot of packed key pk; NULL if the table is full.
__device__ __forceinline__ uint64_t* group_slot(const GroupTable& t, uint64_t pk) {
  if (pk == kEmpty64) return t.slots + (t.mask + 1) * t.words;
  // The top hash bits index the slots: keys whose hashes share a prefix land
  // in one range of the table (a partition of the partitioned aggregation).
  uint64_t h = t.mask ? hash64(pk) >> __clzll(static_cast<long long>(t.mask)) : 0;
  for (uint64_t probes = 0; probes <= t.mask; ++probes) {
    uint64_t* s = t.slots + h * t.words;
    uint64_t cur = __hip_atomic_load(s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == pk) return s;
    if (cur == kEmpty64) {
      unsigned long long prev = atomicCAS(reinterpret_cast<unsigned long long*>(s),
                                          static_cast<unsigned long long>(kEmpty64),
                                          static_cast<unsigned long long>(pk));
      if (prev == kEmpty64 || prev == pk) return s;
    }
    h = (h + 1) & t.mask;
  }
  atomicOr(t.overflow, 1);
  return nullptr;
}

// Adds `cnt` rows with accumulator contributions acc[] to slot s (HBM).
__device__ __forceinline__ void group_update_global(uint64_t* s, const AccPlan& ap, uint64_t cnt,
                                                    const uint64_t* acc) {
  atomicAdd(reinterpret_cast<unsigned long long*>(s + 1), static_cast<unsigned long long>(cnt));
  // unrolled to the bound so that acc[] stays in registers
#pragma unroll
  for (int a = 0; a < kMaxAcc; ++a) {
    if (a >= ap.nacc) break;
    uint64_t* w = s + 2 + a;
    if (ap.kind[a] == kAccSum) {
      atomicAdd(reinterpret_cast<unsigned long long*>(w), static_cast<unsigned long long>(acc[a]));
    } else if (ap.kind[a] == kAccMin) {
      atomicMin(reinterpret_cast<long long*>(w), static_cast<long long>(acc[a]));
    } else {
      atomicMax(reinterpret_cast<long long*>(w), static_cast<long long>(acc[a]));
    }
  }
}

// Key tuple packing: up to two keys of 8/32/64 bits whose widths sum to at
// most 64. Key 0 occupies the high bits, key 1 the low bits; a single key is
// its sign-extended value.
struct GroupKeyPack {
  int32_t nkeys;
  int32_t type[2];
  int32_t shift0;  // bit width of key 1 (key 0 is shifted left by it)
};

__device__ __forceinline__ uint64_t width_mask(int32_t type) {
  return type == kI8 ? 0xFFULL : (type == kI32 ? 0xFFFFFFFFULL : ~0ULL);
}

__device__ __forceinline__ uint64_t pack_keys(const GroupKeyPack& kp, int64_t k0, int64_t k1) {
  if (kp.nkeys == 0) return 0;
  if (kp.nkeys == 1) return static_cast<uint64_t>(k0);
  return ((static_cast<uint64_t>(k0) & width_mask(kp.type[0])) << kp.shift0) |
         (static_cast<uint64_t>(k1) & width_mask(kp.type[1]));
}

__device__ __forceinline__ int64_t sign_extend(uint64_t v, int32_t type) {
  if (type == kI8) return static_cast<int8_t>(v);
  if (type == kI32) return static_cast<int32_t>(v);
  return static_cast<int64_t>(v);
}

__device__ __forceinline__ void unpack_keys(const GroupKeyPack& kp, uint64_t pk, int64_t& k0,
                                            int64_t& k1) {
  if (kp.nkeys == 1) {
    k0 = static_cast<int64_t>(pk);
    k1 = 0;
  } else {
    k0 = sign_extend(kp.shift0 >= 64 ? 0 : (pk >> kp.shift0), kp.type[0]);
    k1 = sign_extend(pk & width_mask(kp.type[1]), kp.type[1]);
  }
}

__device__ __forceinline__ void store_elem(void* p, int32_t type, int64_t i, int64_t v) {
  if (type == kI32) static_cast<int32_t*>(p)[i] = static_cast<int32_t>(v);
  else if (type == kI64) static_cast<int64_t*>(p)[i] = v;
  else static_cast<int8_t*>(p)[i] = static_cast<int8_t>(v);
}

}  // namespace rel
