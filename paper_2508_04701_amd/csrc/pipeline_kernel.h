// Fused plan: conjunctive filter -> inner join with up to two dims ->
// group-by, in one pass over the fact table ("the entire query plan on the
// GPU, from scan to result", Section 3.1).
//
// Persistent workgroups walk fact tiles. Each thread owns four consecutive
// rows of a tile and streams the predicate column (one tile ahead) and the
// foreign keys with coalesced vector loads marked non-temporal (16 bytes per
// lane for int32 columns). Passing rows are then compacted per wave:
// a ballot per row position and the lanes' mbcnt ranks place each passing
// row's id and foreign keys in a small LDS queue. Every time 64 rows are
// queued the wave takes them as one batch with all 64 lanes active: one probe
// read per lane and dim (the 16-byte bucket where the key's run starts, so
// the first read nearly always decides), issued together with the gathers of
// the row's group-key and value columns, then the group update. Random reads and LDS atomics therefore run
// at full lane occupancy whatever the selectivity, which is what bounds
// their throughput. Small dim tables can live in an LDS copy, large ones are
// read from HBM; membership-only dims use key-only tables. Groups are
// aggregated in a per-workgroup LDS table (keys that do not fit go to the
// global table), then merged into one of several replicas of the global
// table, so that few groups do not serialise every workgroup's merge on the
// same global slots; a separate pass folds the replicas. Rows whose dim keys
// match more than once
// (duplicate dim keys) take a row-at-a-time path that enumerates every
// combination. Plans whose dims all resolved to direct tables (dense unique
// keys, decided by the builds on the device) run a twin kernel with a leaner
// drain; each of the two kernels returns at once when the plan is the
// other's.

#pragma once

#include "group_lds.h"
#include "internal.h"

namespace rel {
namespace pipe {

// Dim table access modes (template arguments).
enum : int {
  kNone = 0,
  kMap = 1,     // int32 key -> value, HBM
  kMapLds = 2,  // int32 key -> value, LDS copy
  kSet = 3,     // int32 key only, HBM
  kSetLds = 4,  // int32 key only, LDS copy
  kMap64 = 5,   // int64 key -> value, HBM
  kCSet = 6,    // int32 key only, compact 16-bit entries, HBM
};

__device__ __forceinline__ CsetDesc cset_of(const PipeDim& d) {
  return CsetDesc{static_cast<uint32_t*>(d.map.slots), d.map.cap - 1, d.map.rbits, d.map.dup,
                  d.map.over, d.map.over_cap - 1, d.map.oob_count};
}

// Matches of `key` in a compact set, counted up to `limit`.
__device__ __forceinline__ int cset_matches(const PipeDim& d, int32_t key, uint4 first, int limit) {
  const CsetDesc c = cset_of(d);
  uint64_t b0;
  uint32_t r;
  cset_split(c, key, b0, r);
  const uint4* buckets = reinterpret_cast<const uint4*>(c.words);
  int found = 0;
  uint4 q = first;
  for (int disp = 0; disp <= kCsetMaxDisp; ++disp) {
    bool open;
    found += cset_bucket_count(q, (static_cast<uint32_t>(disp) << 14) | r, open);
    if (found >= limit || open) return found < limit ? found : limit;
    if (disp < kCsetMaxDisp) q = buckets[(b0 + disp + 1) & c.bmask];
  }
  // all three buckets full: the key may have been placed in the overflow set
  return found + cset_over_count(c, key, limit - found);
}

template <int D>
__device__ __forceinline__ const void* dim_slots(const PipeDim& d, const void* lds_copy) {
  if constexpr (D == kMapLds || D == kSetLds) return lds_copy;
  return d.map.slots;
}

// Split probe: probe_first() loads the aligned 16-byte bucket where the
// key's probe run starts (two key/value slots, four key-only slots or one
// int64 slot), so that the first reads of all rows and dims are in flight
// together; probe_finish() scans it and walks on in the rare case that the
// run continues. It returns the number of matches capped at `limit` (1 when
// the build saw no duplicate key, else 2) and the value of the first match
// (key-only sets leave `val` unchanged).
template <int D>
__device__ __forceinline__ uint64_t probe_home(const PipeDim& d, int64_t key) {
  const uint64_t mask = d.map.cap - 1;
  if constexpr (D == kMap64) return home64(key, mask);
  else if constexpr (D == kSet || D == kSetLds) return home_set(static_cast<int32_t>(key), mask);
  else return home32(static_cast<int32_t>(key), mask);
}

template <int D>
__device__ __forceinline__ uint4 probe_first(const PipeDim& d, const void* lds_copy, int64_t key) {
  const uint4* groups = static_cast<const uint4*>(dim_slots<D>(d, lds_copy));
  if constexpr (D == kCSet) {
    uint64_t b0;
    uint32_t r;
    cset_split(cset_of(d), static_cast<int32_t>(key), b0, r);
    return groups[b0];
  }
  const uint64_t h = probe_home<D>(d, key);
  if constexpr (D == kMap64) return groups[h];
  else if constexpr (D == kSet || D == kSetLds) return groups[h >> 2];
  else return groups[h >> 1];
}

template <int D>
__device__ __forceinline__ int probe_finish(const PipeDim& d, const void* lds_copy, int64_t key,
                                            int limit, uint4 first, uint32_t& val) {
  const uint64_t mask = d.map.cap - 1;
  const uint4* groups = static_cast<const uint4*>(dim_slots<D>(d, lds_copy));
  int found = 0;
  if constexpr (D == kCSet) {
    (void)mask;
    (void)groups;
    (void)val;
    const int m = cset_matches(d, static_cast<int32_t>(key), first, limit);
    return m > 2 ? 2 : m;
  } else if constexpr (D == kMap64) {
    if (static_cast<uint64_t>(key) == kEmpty64) {
      const unsigned long long c = *d.map.oob_count;
      if (c) val = d.map.oob_vals[0];
      return c > 1 ? 2 : static_cast<int>(c);
    }
    uint64_t h = probe_home<D>(d, key);
    uint4 q = first;
    while (true) {
      const uint64_t sk = static_cast<uint64_t>(q.x) | (static_cast<uint64_t>(q.y) << 32);
      if (sk == kEmpty64) break;
      if (static_cast<int64_t>(sk) == key) {
        if (found == 0) val = q.z;
        if (++found == limit) break;
      }
      h = (h + 1) & mask;
      q = groups[h];
    }
  } else {
    const int32_t k = static_cast<int32_t>(key);
    if (k == kEmpty32) {
      const unsigned long long c = *d.map.oob_count;
      if constexpr (D == kMap || D == kMapLds)
        if (c) val = d.map.oob_vals[0];
      return c > 1 ? 2 : static_cast<int>(c);
    }
    constexpr int per = (D == kSet || D == kSetLds) ? 4 : 2;  // slots per bucket
    const uint64_t gmask = mask / per;
    uint64_t g = probe_home<D>(d, key) / per;
    uint4 q = first;
    bool done = false;
    while (true) {
      if constexpr (per == 4) {
        const int32_t sv[4] = {static_cast<int32_t>(q.x), static_cast<int32_t>(q.y),
                               static_cast<int32_t>(q.z), static_cast<int32_t>(q.w)};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (done) continue;
          if (sv[i] == kEmpty32) done = true;
          else if (sv[i] == k && ++found == limit) done = true;
        }
      } else {
        const int32_t sk[2] = {static_cast<int32_t>(q.x), static_cast<int32_t>(q.z)};
        const uint32_t sval[2] = {q.y, q.w};
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          if (done) continue;
          if (sk[i] == kEmpty32) {
            done = true;
          } else if (sk[i] == k) {
            if (found == 0) val = sval[i];
            if (++found == limit) done = true;
          }
        }
      }
      if (done) break;
      g = (g + 1) & gmask;
      q = groups[g];
    }
  }
  return found;
}

template <int D>
__device__ __forceinline__ MapCursor dim_start(const PipeDim& d, int64_t key) {
  MapCursor c;
  c.live = true;
  c.direct = false;
  if constexpr (D == kMap || D == kSet || D == kCSet) {
    const DirectView v = direct_view(d.map);
    if (v.mode) {
      uint32_t val = 0;
      c.direct = true;
      c.oob = false;
      c.pos = direct_probe(v, key, val) ? ((1ull << 32) | val) : 0;
      return c;
    }
  }
  if constexpr (D == kCSet) {
    // the cursor counts down the key's multiplicity
    const CsetDesc cs = cset_of(d);
    uint64_t b0;
    uint32_t r;
    cset_split(cs, static_cast<int32_t>(key), b0, r);
    const uint4 first = reinterpret_cast<const uint4*>(cs.words)[b0];
    c.oob = false;
    c.pos = static_cast<uint64_t>(cset_matches(d, static_cast<int32_t>(key), first, 1 << 30));
    return c;
  } else if constexpr (D == kMap64) {
    c.oob = static_cast<uint64_t>(key) == kEmpty64;
    c.pos = c.oob ? 0 : home64(key, d.map.cap - 1);
  } else {
    const int32_t k = static_cast<int32_t>(key);
    c.oob = k == kEmpty32;
    c.pos = c.oob ? 0 : ((D == kSet || D == kSetLds) ? home_set(k, d.map.cap - 1)
                                                       : home32(k, d.map.cap - 1));
  }
  return c;
}

template <int D>
__device__ __forceinline__ bool dim_next(const PipeDim& d, const void* lds_copy, int64_t key,
                                         MapCursor& c, uint32_t& val) {
  const uint64_t mask = d.map.cap - 1;
  const void* base = dim_slots<D>(d, lds_copy);
  if (c.direct) {
    if (!c.live || (c.pos >> 32) == 0) {
      c.live = false;
      return false;
    }
    val = static_cast<uint32_t>(c.pos);
    c.pos = 0;
    return true;
  }
  if constexpr (D == kCSet) {
    (void)mask;
    (void)base;
    (void)key;
    (void)val;
    if (!c.live || c.pos == 0) {
      c.live = false;
      return false;
    }
    --c.pos;
    return true;
  } else if constexpr (D == kMap64) {
    return map_next(static_cast<const ulonglong2*>(base), mask, d.map.oob_count, d.map.oob_vals,
                    key, c, val);
  } else if constexpr (D == kSet || D == kSetLds) {
    return set_next(static_cast<const uint32_t*>(base), mask, d.map.oob_count,
                    static_cast<int32_t>(key), c);
  } else {
    return map_next(static_cast<const uint64_t*>(base), mask, d.map.oob_count, d.map.oob_vals,
                    static_cast<int32_t>(key), c, val);
  }
}

__device__ __forceinline__ uint64_t row_key(const PipelineParams& p, int64_t r, uint32_t v0,
                                            uint32_t v1) {
  int64_t k[2] = {0, 0};
  for (int j = 0; j < p.g.kp.nkeys; ++j) {
    const int src = p.key_src[j];
    if (src == 0) k[j] = load_elem(p.fact[p.key_col[j]], p.fact_type[p.key_col[j]], r);
    else k[j] = static_cast<int32_t>(src == 1 ? v0 : v1);
  }
  return pack_keys(p.g.kp, k[0], k[1]);
}

// Adds one row (count 1, accumulator inputs read from the fact table) to the
// group of packed key pk.
__device__ __forceinline__ void add_row(const PipelineParams& p, int64_t r, uint64_t pk,
                                        uint64_t* lds_group, const GroupTable& gt) {
  uint64_t acc[kMaxAcc];
  for (int a = 0; a < p.g.ap.nacc; ++a)
    acc[a] = static_cast<uint64_t>(load_elem(p.fact[p.acc_col[a]], p.fact_type[p.acc_col[a]], r));
  uint64_t* ls = lds_group_slot(lds_group, p.lds_slots, p.g.words, pk);
  if (ls) {
    lds_group_update(ls, p.g.ap, acc);
  } else {
    uint64_t* gs = group_slot(gt, pk);
    if (gs) group_update_global(gs, p.g.ap, 1, acc);
  }
}

// Row-at-a-time path: every combination of matching dim rows.
template <int D0, int D1>
__device__ __forceinline__ void enumerate_row(const PipelineParams& p, int64_t r, const void* ld0,
                                           const void* ld1, uint64_t* lds_group,
                                           const GroupTable& gt) {
  const int64_t fk0 = load_elem(p.fact[p.dim[0].fk_col], p.fact_type[p.dim[0].fk_col], r);
  int64_t fk1 = 0;
  if constexpr (D1 != kNone)
    fk1 = load_elem(p.fact[p.dim[1].fk_col], p.fact_type[p.dim[1].fk_col], r);
  MapCursor c0 = dim_start<D0>(p.dim[0], fk0);
  uint32_t v0 = 0;
  while (dim_next<D0>(p.dim[0], ld0, fk0, c0, v0)) {
    if constexpr (D1 == kNone) {
      add_row(p, r, row_key(p, r, v0, 0), lds_group, gt);
    } else {
      MapCursor c1 = dim_start<D1>(p.dim[1], fk1);
      uint32_t v1 = 0;
      while (dim_next<D1>(p.dim[1], ld1, fk1, c1, v1))
        add_row(p, r, row_key(p, r, v0, v1), lds_group, gt);
    }
  }
}

// Predicate of four rows whose first term's column was already loaded into
// `first` (the remaining terms are loaded here).
__device__ __forceinline__ uint32_t eval_prefetched(const PipelineParams& p, int64_t r0,
                                                    const int32_t first[4], bool prefetched) {
  uint32_t bits = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) bits |= (r0 + e < p.n) ? (1u << e) : 0u;
  for (int t = 0; t < p.nterms; ++t) {
    int64_t v[4];
    if (t == 0 && prefetched) {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = first[e];
    } else {
      const int c = p.term_col[t];
      load4(p.fact[c], p.fact_type[c], p.fact_vec[c] != 0, r0, p.n, v);
    }
    uint32_t m = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      m |= term_holds(p.term_op[t], v[e], p.term_lo[t], p.term_hi[t]) ? (1u << e) : 0u;
    bits &= m;
  }
  return bits;
}

__device__ __forceinline__ void load_col4(const PipelineParams& p, int c, int64_t r0,
                                          int64_t v[4]) {
  load4(p.fact[c], p.fact_type[c], p.fact_vec[c] != 0, r0, p.n, v);
}

// Foreign keys are held in the width of the dim's keys.
template <int D>
struct KeyOf {
  using T = int32_t;
};
template <>
struct KeyOf<kMap64> {
  using T = int64_t;
};

template <int D>
__device__ __forceinline__ void load_keys4(const PipelineParams& p, int c, int64_t r0,
                                           typename KeyOf<D>::T k[4]) {
  int64_t v[4];
  load4s(p.fact[c], p.fact_type[c], p.fact_vec[c] != 0, r0, p.n, v);
#pragma unroll
  for (int e = 0; e < 4; ++e) k[e] = static_cast<typename KeyOf<D>::T>(v[e]);
}

template <int D>
__device__ __forceinline__ void copy_dim_to_lds(const PipeDim& d, void* lds_copy) {
  if constexpr (D == kMapLds || D == kSetLds) {
    const uint64_t n16 = d.map.cap * (D == kSetLds ? 4 : 8) / 16;
    const uint4* src = static_cast<const uint4*>(d.map.slots);
    uint4* dst = static_cast<uint4*>(lds_copy);
    for (uint64_t i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
  }
}

// Per-wave row queue in LDS: arrays of kPipeQueue entries for the row ids,
// the foreign keys of dims 0 and 1 (8 bytes for int64 dims, else 4), then the
// probe states of dims 0 and 1; fields of absent dims take no space. The
// layout follows from the dim modes (the host sizes it by the same rule).
template <int D0, int D1, int F>
__device__ constexpr uint32_t queue_offset() {
  uint32_t o = kPipeQueue * 4;
  if (F == kQRow) return 0;
  if (F == kQFk0) return o;
  if (D0 != kNone) o += kPipeQueue * (D0 == kMap64 ? 8 : 4);
  if (F == kQFk1) return o;
  if (D1 != kNone) o += kPipeQueue * (D1 == kMap64 ? 8 : 4);
  if (F == kQSt0) return o;
  if (D0 != kNone) o += kPipeQueue * 4;
  return o;
}

template <int D0, int D1>
__device__ constexpr uint32_t queue_stride() {
  return queue_offset<D0, D1, kQSt1>() + (D1 != kNone ? kPipeQueue * 4 : 0);
}

template <int D0, int D1, int F>
struct QueueField {
  typedef typename std::conditional<
      F == kQFk0, typename KeyOf<D0>::T,
      typename std::conditional<F == kQFk1, typename KeyOf<D1>::T, uint32_t>::type>::type T;
};

template <int D0, int D1, int F>
__device__ __forceinline__ void qput(unsigned char* wq, uint32_t i, int64_t v) {
  typedef typename QueueField<D0, D1, F>::T T;
  reinterpret_cast<T*>(wq + queue_offset<D0, D1, F>())[i] = static_cast<T>(v);
}

template <int D0, int D1, int F>
__device__ __forceinline__ int64_t qget(const unsigned char* wq, uint32_t i) {
  typedef typename QueueField<D0, D1, F>::T T;
  return reinterpret_cast<const T*>(wq + queue_offset<D0, D1, F>())[i];
}

// ------------------------------------------------------ resumable probes
//
// A probe of an HBM dim without duplicate keys reads one bucket per batch.
// If the key's run continues past that bucket, the row goes back to the
// queue with the number of buckets scanned, and is resumed in a later batch.
// With 64 lanes per batch, waiting for the longest run of the batch would
// otherwise cost several dependent reads per batch even when few runs are
// long. A dim whose key was found keeps the slot index, and a resumed row
// rereads only that slot's bucket (maps) or nothing (sets).

constexpr uint32_t kResolved = 0x80000000u;

template <int D>
constexpr bool kResumable = (D == kMap || D == kSet || D == kCSet || D == kMap64);

// Dims whose build may pick a direct table (int32 keys read from HBM).
template <int D>
constexpr bool kDirectable = (D == kMap || D == kSet || D == kCSet);

template <int D>
__device__ __forceinline__ DirectView dim_direct(const PipeDim& d) {
  if constexpr (kDirectable<D>) {
    return direct_view(d.map);
  } else {
    DirectView v;
    v.mode = 0;
    return v;
  }
}

template <int D>
__device__ __forceinline__ uint64_t start_bucket(const PipeDim& d, int64_t key) {
  if constexpr (D == kMap64) {
    return home64(key, d.map.cap - 1);
  } else if constexpr (D == kCSet) {
    uint64_t b0;
    uint32_t r;
    cset_split(cset_of(d), static_cast<int32_t>(key), b0, r);
    return b0;
  } else if constexpr (D == kSet) {
    return home_set(static_cast<int32_t>(key), d.map.cap - 1) >> 2;
  } else {
    return home32(static_cast<int32_t>(key), d.map.cap - 1) >> 1;
  }
}

template <int D>
__device__ __forceinline__ uint64_t bucket_mask(const PipeDim& d) {
  if constexpr (D == kMap64 || D == kCSet) return d.map.cap - 1;
  else if constexpr (D == kSet) return (d.map.cap - 1) >> 2;
  else return (d.map.cap - 1) >> 1;
}

// The bucket a probe in state `st` reads next (sets that are resolved need none).
template <int D>
__device__ __forceinline__ uint4 probe_load(const PipeDim& d, int64_t key, uint32_t st) {
  const uint4* buckets = static_cast<const uint4*>(d.map.slots);
  if (st & kResolved) {
    const uint32_t slot = st & ~kResolved;
    if constexpr (D == kMap) return buckets[slot >> 1];
    else if constexpr (D == kMap64) return buckets[slot];
    else return make_uint4(0, 0, 0, 0);
  }
  return buckets[(start_bucket<D>(d, key) + st) & bucket_mask<D>(d)];
}

// Examines the bucket read for state `st`: 0 = no match, 1 = match (`val`
// set, `st` resolved), 2 = the run continues (`st` advanced).
template <int D>
__device__ __forceinline__ int probe_examine(const PipeDim& d, int64_t key, uint4 q, uint32_t& st,
                                             uint32_t& val) {
  if (st & kResolved) {
    const uint32_t slot = st & ~kResolved;
    if constexpr (D == kMap) val = (slot & 1) ? q.w : q.y;
    else if constexpr (D == kMap64) val = q.z;
    return 1;
  }
  const uint64_t g = (start_bucket<D>(d, key) + st) & bucket_mask<D>(d);
  if constexpr (D == kCSet) {
    const CsetDesc c = cset_of(d);
    uint64_t b0;
    uint32_t r;
    cset_split(c, static_cast<int32_t>(key), b0, r);
    bool open;
    if (cset_bucket_has(q, (st << 14) | r, open)) {
      st = kResolved;
      return 1;
    }
    if (open) return 0;
    if (st == kCsetMaxDisp) {
      if (cset_over_count(c, static_cast<int32_t>(key), 1) > 0) {
        st = kResolved;
        return 1;
      }
      return 0;
    }
    ++st;
    return 2;
  } else if constexpr (D == kMap64) {
    if (static_cast<uint64_t>(key) == kEmpty64) {  // out-of-band key, unique build
      if (*d.map.oob_count == 0) return 0;
      val = d.map.oob_vals[0];
      return 1;
    }
    const uint64_t sk = static_cast<uint64_t>(q.x) | (static_cast<uint64_t>(q.y) << 32);
    if (sk == kEmpty64) return 0;
    if (static_cast<int64_t>(sk) == key) {
      val = q.z;
      st = kResolved | static_cast<uint32_t>(g);
      return 1;
    }
    ++st;
    return 2;
  } else {
    const int32_t k = static_cast<int32_t>(key);
    if (k == kEmpty32) {
      if (*d.map.oob_count == 0) return 0;
      if constexpr (D == kMap) val = d.map.oob_vals[0];
      return 1;
    }
    if constexpr (D == kSet) {
      const int32_t sv[4] = {static_cast<int32_t>(q.x), static_cast<int32_t>(q.y),
                             static_cast<int32_t>(q.z), static_cast<int32_t>(q.w)};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (sv[i] == k) {
          st = kResolved;
          return 1;
        }
        if (sv[i] == kEmpty32) return 0;
      }
    } else {
      const int32_t sk[2] = {static_cast<int32_t>(q.x), static_cast<int32_t>(q.z)};
      const uint32_t sval[2] = {q.y, q.w};
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (sk[i] == k) {
          val = sval[i];
          st = kResolved | static_cast<uint32_t>(g * 2 + i);
          return 1;
        }
        if (sk[i] == kEmpty32) return 0;
      }
    }
    ++st;
    return 2;
  }
}

// The plan's accumulators packed four bits each, first in the low bits: one
// plus (kind | source << 2), the source 0 or 1 for the early-gathered columns
// and 2 for a late load; a zero field ends the list. Computed once per
// workgroup, so that the update loop reads no memory between its atomics (a
// scalar load there also waits on the LDS counter, which serialised the
// atomics of a row).
__device__ __forceinline__ uint32_t acc_code(const PipelineParams& p) {
  uint32_t c = 0;
  for (int a = 0; a < p.g.ap.nacc; ++a) {
    const uint32_t src = p.acc_src[a] == 0 ? 0u : (p.acc_src[a] == 1 ? 1u : 2u);
    c |= (1u + (static_cast<uint32_t>(p.g.ap.kind[a]) | (src << 2))) << (4 * a);
  }
  return c;
}

// Writes row r's update of group pk as a record (batched plans with
// records; see RecDesc): the active lanes take consecutive places in the
// item's record run (one LDS atomic per wave on the item's count) and count
// the record in its partition's LDS histogram entry. The item is the run of
// item_tiles tiles that holds row r.
__device__ __forceinline__ void spill_record(const PipelineParams& p, int64_t r, uint64_t pk,
                                             int64_t va, int64_t vb, uint64_t* lg) {
  const RecDesc& rd = p.rec;
  uint32_t* hist = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(lg) + rd.lds_offset);
  const uint64_t m = ballot(true);
  const uint32_t rank = rank_below(m);
  uint32_t base = 0;
  if (rank == 0) base = lds_fetch_add_u32(hist + rd.parts, popc64(m));
  base = __builtin_amdgcn_readfirstlane(base);
  lds_fetch_add_u32(hist + rec_part(pk, rd.parts), 1u);
  const uint32_t tile = static_cast<uint32_t>(static_cast<uint64_t>(r) / kPipeTile);
  const uint64_t at = static_cast<uint64_t>(tile - tile % rd.item_tiles) * kPipeTile + base + rank;
  if (rd.narrow) {
    __builtin_nontemporal_store(static_cast<uint32_t>(pk), rd.rkeys + at);
    __builtin_nontemporal_store(static_cast<uint64_t>(va), rd.recs + at);
    return;
  }
  uint64_t* w = rd.recs + at * rd.words;
  if (rd.words == 2) {
    typedef uint64_t v2u64 __attribute__((ext_vector_type(2)));
    v2u64 x;
    x.x = pk;
    x.y = static_cast<uint64_t>(va);
    __builtin_nontemporal_store(x, reinterpret_cast<v2u64*>(w));
  } else {
    __builtin_nontemporal_store(pk, w);
    if (rd.words > 1) __builtin_nontemporal_store(static_cast<uint64_t>(va), w + 1);
    if (rd.words > 2) __builtin_nontemporal_store(static_cast<uint64_t>(vb), w + 2);
  }
}

// Adds row r to group pk (va, vb: the early-gathered value columns; acode:
// acc_code(p)): one branch per row, the workgroup's LDS table or its global
// replica (or, kRec and a plan with records, a record).
template <bool kRec = false>
__device__ __forceinline__ void update_group(const PipelineParams& p, int64_t r, uint64_t pk,
                                             int64_t va, int64_t vb, uint64_t* lg,
                                             const GroupTable& gt, uint32_t acode) {
  const int words = p.g.words;
  const int32_t li = lds_group_find(lg, p.lds_slots, words, pk);
  if (li >= 0) {
    uint64_t* s = lg + li * words;
    lds_add_u64(s + 1, 1);
    int a = 0;
    for (uint32_t code = acode; code != 0; code >>= 4, ++a) {
      const uint32_t c = (code & 15u) - 1u;
      const uint32_t src = c >> 2;
      const int64_t v = src == 0 ? va
                      : src == 1 ? vb
                                 : load_elem(p.fact[p.acc_col[a]], p.fact_type[p.acc_col[a]], r);
      lds_acc_update(s + 2 + a, static_cast<int>(c & 3u), v);
    }
  } else {
    if constexpr (kRec) {
      if (p.rec.parts) {
        spill_record(p, r, pk, va, vb, lg);
        return;
      }
    }
    uint64_t* gs = group_slot(gt, pk);
    if (!gs) return;
    global_add_u64(gs + 1, 1);
    int a = 0;
    for (uint32_t code = acode; code != 0; code >>= 4, ++a) {
      const uint32_t c = (code & 15u) - 1u;
      const uint32_t src = c >> 2;
      const int64_t v = src == 0 ? va
                      : src == 1 ? vb
                                 : load_elem(p.fact[p.acc_col[a]], p.fact_type[p.acc_col[a]], r);
      const int kind = static_cast<int>(c & 3u);
      uint64_t* w = gs + 2 + a;
      if (kind == kAccSum)
        atomicAdd(reinterpret_cast<unsigned long long*>(w), static_cast<unsigned long long>(v));
      else if (kind == kAccMin)
        atomicMin(reinterpret_cast<long long*>(w), static_cast<long long>(v));
      else
        atomicMax(reinterpret_cast<long long*>(w), static_cast<long long>(v));
    }
  }
}

// One queued row: probe the dims and update the row's group. Returns true
// when the row has to go back to the queue (a resumable probe continues).
template <int D0, int D1, bool kRec = false>
__device__ __forceinline__ bool process_row(const PipelineParams& p, int64_t r, int64_t fk0,
                                            int64_t fk1, uint32_t& st0, uint32_t& st1,
                                            const void* ld0, const void* ld1, uint64_t* lg,
                                            const GroupTable& gt, int limit0, int limit1,
                                            const DirectView& dv0, const DirectView& dv1,
                                            uint32_t acode) {
  const bool dir0 = kDirectable<D0> && dv0.mode != 0;
  const bool dir1 = kDirectable<D1> && dv1.mode != 0;
  const bool res0 = kResumable<D0> && limit0 == 1;
  const bool res1 = kResumable<D1> && limit1 == 1;
  uint4 q0 = make_uint4(0, 0, 0, 0), q1 = make_uint4(0, 0, 0, 0);
  if constexpr (D0 != kNone)
    if (!dir0) q0 = res0 ? probe_load<D0>(p.dim[0], fk0, st0) : probe_first<D0>(p.dim[0], ld0, fk0);
  if constexpr (D1 != kNone)
    if (!dir1) q1 = res1 ? probe_load<D1>(p.dim[1], fk1, st1) : probe_first<D1>(p.dim[1], ld1, fk1);
  // Group-key and value columns, gathered by row id while the probe reads
  // are in flight (lines the batch shares are fetched once); rows that the
  // joins drop discard them.
  int64_t k0 = 0, k1 = 0;
  if (p.g.kp.nkeys > 0 && p.key_src[0] == 0)
    k0 = load_elem(p.fact[p.key_col[0]], p.fact_type[p.key_col[0]], r);
  if (p.g.kp.nkeys > 1 && p.key_src[1] == 0)
    k1 = load_elem(p.fact[p.key_col[1]], p.fact_type[p.key_col[1]], r);
  int64_t va = 0, vb = 0;
  if (p.early_col[0] >= 0) va = load_elem(p.fact[p.early_col[0]], p.fact_type[p.early_col[0]], r);
  if (p.early_col[1] >= 0) vb = load_elem(p.fact[p.early_col[1]], p.fact_type[p.early_col[1]], r);
  uint32_t v0 = 0, v1 = 0;
  bool more = false, multi = false;
  if constexpr (D0 != kNone) {
    if (dir0) {
      if (!direct_probe(dv0, fk0, v0)) return false;
    } else if (res0) {
      const int m = probe_examine<D0>(p.dim[0], fk0, q0, st0, v0);
      if (m == 0) return false;
      more |= m == 2;
    } else {
      const int m = probe_finish<D0>(p.dim[0], ld0, fk0, limit0, q0, v0);
      if (m == 0) return false;
      multi |= m == 2;
    }
  }
  if constexpr (D1 != kNone) {
    if (dir1) {
      if (!direct_probe(dv1, fk1, v1)) return false;
    } else if (res1) {
      const int m = probe_examine<D1>(p.dim[1], fk1, q1, st1, v1);
      if (m == 0) return false;
      more |= m == 2;
    } else {
      const int m = probe_finish<D1>(p.dim[1], ld1, fk1, limit1, q1, v1);
      if (m == 0) return false;
      multi |= m == 2;
    }
  }
  if (more) return true;
  if (multi) return false;  // several dim matches: left to the enumeration pass
  if (p.g.kp.nkeys > 0 && p.key_src[0] != 0) k0 = static_cast<int32_t>(p.key_src[0] == 1 ? v0 : v1);
  if (p.g.kp.nkeys > 1 && p.key_src[1] != 0) k1 = static_cast<int32_t>(p.key_src[1] == 1 ? v0 : v1);
  update_group<kRec>(p, r, pack_keys(p.g.kp, k0, k1), va, vb, lg, gt, acode);
  return false;
}

// ------------------------------------------------------ row specs
//
// A row spec fixes at compile time where a plan's group keys and values come
// from, so that the per-row work of the drain (gathers, key packing, the
// accumulator inputs) has no run-time type or source decisions: spec S packs
// key source k0 (bits 0-2), key source k1 (bits 3-5) and the value source
// (bit 6; 1 = every accumulator reads one int64 fact column). Key sources:
// the payload of dim 0 or dim 1, or a fact column of int8 or int32. S = 0 is
// the generic interpreter. The host derives S from the plan (PipelineParams::
// spec) and launches the specialised kernel when its (dims, S) variant is
// built; a plan whose dims turn out to hold duplicate keys leaves the work to
// the generic kernel.

enum : int { kKNone = 0, kKDim0 = 1, kKDim1 = 2, kKF8 = 3, kKF32 = 4 };

constexpr int spec_of(int k0, int k1, int v) { return k0 | (k1 << 3) | (v << 6); }

// The row specs that are built: (dim 1 payload, int8 fact column) keys, as
// in a star join grouped by a dim attribute and a fact flag; one dim-payload
// key, as in a join grouped by an attribute of the build side.
constexpr int kSpecDim1F8 = spec_of(kKDim1, kKF8, 1);
constexpr int kSpecDim0 = spec_of(kKDim0, kKNone, 1);
constexpr int kSpecDim1 = spec_of(kKDim1, kKNone, 1);

template <int S>
struct RowSpec {
  static constexpr int k0 = S & 7;
  static constexpr int k1 = (S >> 3) & 7;
  static constexpr int nkeys = (k0 != kKNone) + (k1 != kKNone);
  static constexpr bool value = ((S >> 6) & 1) != 0;
};

// Whether spec S can run with dim modes D0, D1: dim-payload keys need that
// dim to be a key -> value map, and only HBM hash tables are specialised.
template <int D>
constexpr bool kSpecDim = D == kNone || D == kMap || D == kSet || D == kCSet;

template <int D0, int D1, int S>
constexpr bool spec_ok() {
  if (S == 0) return true;
  if (!kSpecDim<D0> || !kSpecDim<D1> || D0 == kNone) return false;
  constexpr int k0 = RowSpec<S>::k0, k1 = RowSpec<S>::k1;
  if ((k0 == kKDim0 || k1 == kKDim0) && D0 != kMap) return false;
  if ((k0 == kKDim1 || k1 == kKDim1) && D1 != kMap) return false;
  return true;
}

// Key j of a specialised row (fact keys gathered by row id).
template <int K>
__device__ __forceinline__ int64_t spec_key(const PipelineParams& p, int j, int64_t r, uint32_t v0,
                                            uint32_t v1) {
  if constexpr (K == kKDim0) return static_cast<int32_t>(v0);
  else if constexpr (K == kKDim1) return static_cast<int32_t>(v1);
  else if constexpr (K == kKF8) return static_cast<const int8_t*>(p.spec_key[j])[r];
  else if constexpr (K == kKF32) return static_cast<const int32_t*>(p.spec_key[j])[r];
  else return 0;
}

template <int S>
__device__ __forceinline__ uint64_t spec_pack(const GroupKeyPack& kp, int64_t k0, int64_t k1) {
  if constexpr (RowSpec<S>::nkeys == 0) return 0;
  else if constexpr (RowSpec<S>::nkeys == 1) return static_cast<uint64_t>(k0);
  else
    return ((static_cast<uint64_t>(k0) & width_mask(kp.type[0])) << kp.shift0) |
           (static_cast<uint64_t>(k1) & width_mask(kp.type[1]));
}

// Adds a row with value v to group pk under a specialised plan: every
// accumulator reads v (acode's sources are ignored).
__device__ __forceinline__ void spec_update(const PipelineParams& p, uint64_t pk, int64_t v,
                                            uint64_t* lg, const GroupTable& gt, uint32_t acode) {
  const int words = p.g.words;
  const int32_t li = lds_group_find(lg, p.lds_slots, words, pk);
  if (li >= 0) {
    uint64_t* s = lg + li * words;
    lds_add_u64(s + 1, 1);
    int a = 0;
    for (uint32_t code = acode; code != 0; code >>= 4, ++a)
      lds_acc_update(s + 2 + a, static_cast<int>(((code & 15u) - 1u) & 3u), v);
  } else {
    uint64_t* gs = group_slot(gt, pk);
    if (!gs) return;
    global_add_u64(gs + 1, 1);
    int a = 0;
    for (uint32_t code = acode; code != 0; code >>= 4, ++a) {
      const int kind = static_cast<int>(((code & 15u) - 1u) & 3u);
      uint64_t* w = gs + 2 + a;
      if (kind == kAccSum)
        atomicAdd(reinterpret_cast<unsigned long long*>(w), static_cast<unsigned long long>(v));
      else if (kind == kAccMin)
        atomicMin(reinterpret_cast<long long*>(w), static_cast<long long>(v));
      else
        atomicMax(reinterpret_cast<long long*>(w), static_cast<long long>(v));
    }
  }
}

// process_row for spec S: hash-table dims without duplicate keys, so every
// probe stops at its first match. A probe that meets a full bucket reads the
// next one in place (a specialised plan's dims are built at load factors
// that keep such runs short), so rows are never queued twice.
template <int D0, int D1, int S>
__device__ __forceinline__ void spec_row(const PipelineParams& p, int64_t r, int32_t fk0,
                                         int32_t fk1, uint64_t* lg, const GroupTable& gt,
                                         uint32_t acode) {
  typedef RowSpec<S> R;
  uint32_t st0 = 0, st1 = 0;
  uint4 q0 = make_uint4(0, 0, 0, 0), q1 = make_uint4(0, 0, 0, 0);
  if constexpr (D0 != kNone) q0 = probe_load<D0>(p.dim[0], fk0, 0);
  if constexpr (D1 != kNone) q1 = probe_load<D1>(p.dim[1], fk1, 0);
  // fact keys and the value, gathered while the probe reads are in flight
  int64_t f0 = 0, f1 = 0, v = 0;
  if constexpr (R::k0 == kKF8 || R::k0 == kKF32) f0 = spec_key<R::k0>(p, 0, r, 0, 0);
  if constexpr (R::k1 == kKF8 || R::k1 == kKF32) f1 = spec_key<R::k1>(p, 1, r, 0, 0);
  if constexpr (R::value) v = p.spec_val[r];
  uint32_t v0 = 0, v1 = 0;
  int m0 = 1, m1 = 1;
  if constexpr (D0 != kNone) {
    m0 = probe_examine<D0>(p.dim[0], fk0, q0, st0, v0);
    while (m0 == 2) m0 = probe_examine<D0>(p.dim[0], fk0, probe_load<D0>(p.dim[0], fk0, st0), st0, v0);
  }
  if constexpr (D1 != kNone) {
    m1 = probe_examine<D1>(p.dim[1], fk1, q1, st1, v1);
    while (m1 == 2) m1 = probe_examine<D1>(p.dim[1], fk1, probe_load<D1>(p.dim[1], fk1, st1), st1, v1);
  }
  if (m0 == 0 || m1 == 0) return;
  const int64_t k0 = (R::k0 == kKF8 || R::k0 == kKF32) ? f0 : spec_key<R::k0>(p, 0, r, v0, v1);
  const int64_t k1 = (R::k1 == kKF8 || R::k1 == kKF32) ? f1 : spec_key<R::k1>(p, 1, r, v0, v1);
  spec_update(p, spec_pack<S>(p.g.kp, k0, k1), v, lg, gt, acode);
}

// direct_row for spec S.
template <int D0, int D1, int S>
__device__ __forceinline__ void spec_direct_row(const PipelineParams& p, int64_t r, int64_t fk0,
                                                int64_t fk1, uint64_t* lg, const GroupTable& gt,
                                                const DirectView& dv0, const DirectView& dv1,
                                                uint32_t acode) {
  typedef RowSpec<S> R;
  int64_t f0 = 0, f1 = 0, v = 0;
  if constexpr (R::k0 == kKF8 || R::k0 == kKF32) f0 = spec_key<R::k0>(p, 0, r, 0, 0);
  if constexpr (R::k1 == kKF8 || R::k1 == kKF32) f1 = spec_key<R::k1>(p, 1, r, 0, 0);
  if constexpr (R::value) v = p.spec_val[r];
  uint32_t v0 = 0, v1 = 0;
  if constexpr (D0 != kNone)
    if (!direct_probe(dv0, fk0, v0)) return;
  if constexpr (D1 != kNone)
    if (!direct_probe(dv1, fk1, v1)) return;
  const int64_t k0 = (R::k0 == kKF8 || R::k0 == kKF32) ? f0 : spec_key<R::k0>(p, 0, r, v0, v1);
  const int64_t k1 = (R::k1 == kKF8 || R::k1 == kKF32) ? f1 : spec_key<R::k1>(p, 1, r, v0, v1);
  spec_update(p, spec_pack<S>(p.g.kp, k0, k1), v, lg, gt, acode);
}

// Processes the top `take` (<= 64) rows of the wave's queue, one per lane;
// rows whose probes continue are written back. Returns the new queue length.
template <int D0, int D1, bool kRec = false>
__device__ __forceinline__ uint32_t drain(const PipelineParams& p, unsigned char* wq,
                                          uint32_t queued, uint32_t take, int lane,
                                          const void* ld0, const void* ld1, uint64_t* lg,
                                          const GroupTable& gt, int limit0, int limit1,
                                          const DirectView& dv0, const DirectView& dv1,
                                          uint32_t acode) {
  const uint32_t base = queued - take;
  const bool mine = static_cast<uint32_t>(lane) < take;
  int64_t r = 0, fk0 = 0, fk1 = 0;
  uint32_t st0 = 0, st1 = 0;
  if (mine) {
    const uint32_t i = base + lane;
    r = static_cast<uint32_t>(qget<D0, D1, kQRow>(wq, i));
    if constexpr (D0 != kNone) {
      fk0 = qget<D0, D1, kQFk0>(wq, i);
      st0 = static_cast<uint32_t>(qget<D0, D1, kQSt0>(wq, i));
    }
    if constexpr (D1 != kNone) {
      fk1 = qget<D0, D1, kQFk1>(wq, i);
      st1 = static_cast<uint32_t>(qget<D0, D1, kQSt1>(wq, i));
    }
  }
  __builtin_amdgcn_wave_barrier();
  bool again = false;
  if (mine)
    again = process_row<D0, D1, kRec>(p, r, fk0, fk1, st0, st1, ld0, ld1, lg, gt, limit0, limit1,
                                      dv0, dv1, acode);
  const uint64_t b = ballot(again);
  if (again) {
    const uint32_t at = base + rank_below(b);
    qput<D0, D1, kQRow>(wq, at, r);
    if constexpr (D0 != kNone) {
      qput<D0, D1, kQFk0>(wq, at, fk0);
      qput<D0, D1, kQSt0>(wq, at, st0);
    }
    if constexpr (D1 != kNone) {
      qput<D0, D1, kQFk1>(wq, at, fk1);
      qput<D0, D1, kQSt1>(wq, at, st1);
    }
  }
  __builtin_amdgcn_wave_barrier();
  return base + popc64(b);
}

// ------------------------------------------------------ direct dims
//
// When every dim of the plan resolved to a direct table at build time (dense
// unique int32 keys), a probe is a range test plus at most a bit and a payload
// read at computed addresses: no bucket walks, no row returns to the queue,
// no probe states. run_tiles then takes a leaner drain whose queue entries
// are the row id and the foreign keys only, which keeps the loop within its
// register budget.

template <int D>
constexpr bool kDirectOk = D == kNone || kDirectable<D>;

template <int D0, int D1>
__device__ __forceinline__ void direct_row(const PipelineParams& p, int64_t r, int64_t fk0,
                                           int64_t fk1, uint64_t* lg, const GroupTable& gt,
                                           const DirectView& dv0, const DirectView& dv1,
                                           uint32_t acode) {
  int64_t k0 = 0, k1 = 0;
  if (p.g.kp.nkeys > 0 && p.key_src[0] == 0)
    k0 = load_elem(p.fact[p.key_col[0]], p.fact_type[p.key_col[0]], r);
  if (p.g.kp.nkeys > 1 && p.key_src[1] == 0)
    k1 = load_elem(p.fact[p.key_col[1]], p.fact_type[p.key_col[1]], r);
  int64_t va = 0, vb = 0;
  if (p.early_col[0] >= 0) va = load_elem(p.fact[p.early_col[0]], p.fact_type[p.early_col[0]], r);
  if (p.early_col[1] >= 0) vb = load_elem(p.fact[p.early_col[1]], p.fact_type[p.early_col[1]], r);
  uint32_t v0 = 0, v1 = 0;
  if constexpr (D0 != kNone)
    if (!direct_probe(dv0, fk0, v0)) return;
  if constexpr (D1 != kNone)
    if (!direct_probe(dv1, fk1, v1)) return;
  if (p.g.kp.nkeys > 0 && p.key_src[0] != 0) k0 = static_cast<int32_t>(p.key_src[0] == 1 ? v0 : v1);
  if (p.g.kp.nkeys > 1 && p.key_src[1] != 0) k1 = static_cast<int32_t>(p.key_src[1] == 1 ? v0 : v1);
  update_group(p, r, pack_keys(p.g.kp, k0, k1), va, vb, lg, gt, acode);
}

// Processes queue entries [base, base + take), take <= 64, one per lane.
template <int D0, int D1, int S>
__device__ __forceinline__ void drain_direct(const PipelineParams& p, const unsigned char* wq,
                                             uint32_t base, uint32_t take, int lane,
                                             uint64_t* lg, const GroupTable& gt,
                                             const DirectView& dv0, const DirectView& dv1,
                                             uint32_t acode) {
  if (static_cast<uint32_t>(lane) < take) {
    const uint32_t i = base + lane;
    const int64_t r = static_cast<uint32_t>(qget<D0, D1, kQRow>(wq, i));
    int64_t fk0 = 0, fk1 = 0;
    if constexpr (D0 != kNone) fk0 = qget<D0, D1, kQFk0>(wq, i);
    if constexpr (D1 != kNone) fk1 = qget<D0, D1, kQFk1>(wq, i);
    if constexpr (S != 0)
      spec_direct_row<D0, D1, S>(p, r, fk0, fk1, lg, gt, dv0, dv1, acode);
    else
      direct_row<D0, D1>(p, r, fk0, fk1, lg, gt, dv0, dv1, acode);
  }
  __builtin_amdgcn_wave_barrier();
}

// Walks tiles `tile`, `tile + step`, ... below `end` of plan p: streams the
// predicate column (two tiles ahead) and the foreign keys, queues the passing
// rows per wave and drains them in full-lane batches. Returns with the
// wave's queue empty.
template <int D0, int D1, bool kDirect, int S = 0, bool kRec = false>
__device__ __forceinline__ void run_tiles(const PipelineParams& p, int64_t tile, int64_t end,
                                          int64_t step, unsigned char* wq, int lane,
                                          const void* ld0, const void* ld1, uint64_t* lg,
                                          const GroupTable& gt, int limit0, int limit1) {
  const DirectView dv0 = dim_direct<D0>(p.dim[0]);
  const DirectView dv1 = dim_direct<D1>(p.dim[1]);
  const uint32_t acode = acc_code(p);
  const int tid = threadIdx.x;
  // The first term's column is read two tiles ahead when its rows are at
  // most four bytes wide (held as int32; an int64 column is read in place),
  // so that each wave keeps several loads in flight.
  const int c_pred = p.nterms > 0 ? p.term_col[0] : 0;
  const bool prefetch = p.nterms > 0 && p.fact_type[c_pred] != kI64;
  const void* pcol = p.fact[c_pred];
  const int32_t ptype = p.fact_type[c_pred];
  const bool pvec = p.fact_vec[c_pred] != 0;
  int32_t pre[4] = {0, 0, 0, 0}, pre2[4] = {0, 0, 0, 0};
  if (prefetch && tile < end)
    load4n(pcol, ptype, pvec, tile * static_cast<int64_t>(kPipeTile) + tid * 4, p.n, pre);
  if (prefetch && tile + step < end)
    load4n(pcol, ptype, pvec, (tile + step) * static_cast<int64_t>(kPipeTile) + tid * 4, p.n,
           pre2);
  // While most lanes of a wave see passing rows, nearly every line of the
  // foreign-key columns is needed: they are then loaded before the predicate
  // is evaluated, overlapping both; otherwise only for lanes with passing
  // rows (wave-uniform switch, updated per tile).
  bool eager = true;
  uint32_t queued = 0;  // wave-uniform
  for (; tile < end; tile += step) {
    const int64_t r0 = tile * static_cast<int64_t>(kPipeTile) + tid * 4;
    typename KeyOf<D0>::T fk0[4] = {0, 0, 0, 0};
    typename KeyOf<D1>::T fk1[4] = {0, 0, 0, 0};
    if (eager) {
      if constexpr (D0 != kNone) load_keys4<D0>(p, p.dim[0].fk_col, r0, fk0);
      if constexpr (D1 != kNone) load_keys4<D1>(p, p.dim[1].fk_col, r0, fk1);
    }
    const uint32_t bits = eval_prefetched(p, r0, pre, prefetch);
    const int64_t ahead = tile + 2 * step;
#pragma unroll
    for (int e = 0; e < 4; ++e) pre[e] = pre2[e];
    if (prefetch && ahead < end)
      load4n(pcol, ptype, pvec, ahead * static_cast<int64_t>(kPipeTile) + tid * 4, p.n, pre2);
    if (!eager && bits) {
      if constexpr (D0 != kNone) load_keys4<D0>(p, p.dim[0].fk_col, r0, fk0);
      if constexpr (D1 != kNone) load_keys4<D1>(p, p.dim[1].fk_col, r0, fk1);
    }
    eager = popc64(ballot(bits != 0)) >= kWave / 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const bool pass = (bits >> e) & 1u;
      const uint64_t b = ballot(pass);
      if (b == 0) continue;
      if (pass) {
        const uint32_t at = queued + rank_below(b);
        qput<D0, D1, kQRow>(wq, at, r0 + e);
        if constexpr (D0 != kNone) {
          qput<D0, D1, kQFk0>(wq, at, fk0[e]);
          if constexpr (!kDirect) qput<D0, D1, kQSt0>(wq, at, 0);
        }
        if constexpr (D1 != kNone) {
          qput<D0, D1, kQFk1>(wq, at, fk1[e]);
          if constexpr (!kDirect) qput<D0, D1, kQSt1>(wq, at, 0);
        }
      }
      queued += popc64(b);
      __builtin_amdgcn_wave_barrier();
      if constexpr (kDirect) {
        // at most 127 rows are queued here: one batch leaves fewer than 64
        if (queued >= kWave) {
          queued -= kWave;
          drain_direct<D0, D1, S>(p, wq, queued, kWave, lane, lg, gt, dv0, dv1, acode);
        }
      } else {
        while (queued >= kWave)
          queued = drain<D0, D1, kRec>(p, wq, queued, kWave, lane, ld0, ld1, lg, gt, limit0,
                                       limit1, dv0, dv1, acode);
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  if constexpr (kDirect) {
    if (queued > 0) drain_direct<D0, D1, S>(p, wq, 0, queued, lane, lg, gt, dv0, dv1, acode);
  } else {
    while (queued > 0)
      queued = drain<D0, D1, kRec>(p, wq, queued, queued < kWave ? queued : kWave, lane, ld0, ld1,
                                   lg, gt, limit0, limit1, dv0, dv1, acode);
  }
}

// ------------------------------------------------------ specialised pass
//
// The tile loop of the specialised kernels: at most one predicate term, on
// an int32 column, held as the half-open range [spec_lo, spec_lo + spec_span)
// of the widened value (the host folds every comparison but NE into it);
// int32 foreign keys; every column that is streamed is 16-byte aligned. The
// queue holds row ids, foreign keys and probe states as in run_tiles.

// Four consecutive int32 values from r0 (non-temporal), zero past n.
__device__ __forceinline__ void spec_load4(const int32_t* c, int64_t r0, int64_t n, int32_t v[4]) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  if (r0 + 4 <= n) {
    const v4i x = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(c + r0));
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = r0 + e < n ? c[r0 + e] : 0;
  }
}

// Processes the top `take` (<= 64) rows of the wave's queue under spec S,
// one per lane. Returns the new queue length.
template <int D0, int D1, int S>
__device__ __forceinline__ uint32_t spec_drain(const PipelineParams& p, unsigned char* wq,
                                               uint32_t queued, uint32_t take, int lane,
                                               uint64_t* lg, const GroupTable& gt,
                                               uint32_t acode) {
  const uint32_t base = queued - take;
  const bool mine = static_cast<uint32_t>(lane) < take;
  int64_t r = 0;
  int32_t fk0 = 0, fk1 = 0;
  if (mine) {
    const uint32_t i = base + lane;
    r = static_cast<uint32_t>(qget<D0, D1, kQRow>(wq, i));
    if constexpr (D0 != kNone) fk0 = static_cast<int32_t>(qget<D0, D1, kQFk0>(wq, i));
    if constexpr (D1 != kNone) fk1 = static_cast<int32_t>(qget<D0, D1, kQFk1>(wq, i));
  }
  __builtin_amdgcn_wave_barrier();
  if (mine) spec_row<D0, D1, S>(p, r, fk0, fk1, lg, gt, acode);
  __builtin_amdgcn_wave_barrier();
  return base;
}

// One of four register values by a wave-uniform index (no indexed
// register access, which would go through scratch).
__device__ __forceinline__ int32_t pick4(const int32_t v[4], int e) {
  return e == 0 ? v[0] : (e == 1 ? v[1] : (e == 2 ? v[2] : v[3]));
}

// The loop is one state machine with a single drain site and a single tile
// site (the drain is large; inlined once per row position it would fill the
// instruction cache): each step either drains a full batch (or, once the
// tiles are done, the rest of the queue), loads the next tile, or appends
// the passing rows of one row position of the current tile.
template <int D0, int D1, int S>
__device__ __forceinline__ void spec_tiles(const PipelineParams& p, int64_t tile, int64_t end,
                                           int64_t step, unsigned char* wq, int lane,
                                           uint64_t* lg, const GroupTable& gt) {
  const uint32_t acode = acc_code(p);
  const int tid = threadIdx.x;
  const int64_t n = p.n;
  const bool has_pred = p.nterms > 0;
  const int32_t* pcol = static_cast<const int32_t*>(p.fact[p.term_col[0]]);
  const int64_t lo = p.spec_lo;
  const uint64_t span = p.spec_span;
  const int32_t* fc0 = static_cast<const int32_t*>(p.fact[p.dim[0].fk_col]);
  const int32_t* fc1 = static_cast<const int32_t*>(p.fact[p.dim[1].fk_col]);
  int32_t pre[4] = {0, 0, 0, 0}, pre2[4] = {0, 0, 0, 0};
  if (has_pred && tile < end) spec_load4(pcol, tile * static_cast<int64_t>(kPipeTile) + tid * 4, n, pre);
  if (has_pred && tile + step < end)
    spec_load4(pcol, (tile + step) * static_cast<int64_t>(kPipeTile) + tid * 4, n, pre2);
  bool eager = true;
  uint32_t queued = 0;  // wave-uniform
  int e = 4;            // next row position of the current tile (4: none left)
  int64_t r0 = 0;
  uint32_t bits = 0;
  int32_t fk0[4] = {0, 0, 0, 0}, fk1[4] = {0, 0, 0, 0};
  while (true) {
    if (queued >= kWave || (e == 4 && tile >= end && queued > 0)) {
      queued = spec_drain<D0, D1, S>(p, wq, queued, queued < kWave ? queued : kWave, lane, lg, gt,
                                     acode);
      continue;
    }
    if (e == 4) {
      if (tile >= end) break;
      r0 = tile * static_cast<int64_t>(kPipeTile) + tid * 4;
      if (eager) {
        if constexpr (D0 != kNone) spec_load4(fc0, r0, n, fk0);
        if constexpr (D1 != kNone) spec_load4(fc1, r0, n, fk1);
      }
      bits = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool in = r0 + k < n;
        const bool ok = !has_pred || static_cast<uint64_t>(static_cast<int64_t>(pre[k]) - lo) < span;
        bits |= (in && ok) ? (1u << k) : 0u;
      }
      const int64_t ahead = tile + 2 * step;
#pragma unroll
      for (int k = 0; k < 4; ++k) pre[k] = pre2[k];
      if (has_pred && ahead < end)
        spec_load4(pcol, ahead * static_cast<int64_t>(kPipeTile) + tid * 4, n, pre2);
      if (!eager && bits) {
        if constexpr (D0 != kNone) spec_load4(fc0, r0, n, fk0);
        if constexpr (D1 != kNone) spec_load4(fc1, r0, n, fk1);
      }
      eager = popc64(ballot(bits != 0)) >= kWave / 4;
      tile += step;
      e = 0;
      continue;
    }
    const bool pass = (bits >> e) & 1u;
    const uint64_t b = ballot(pass);
    if (pass) {
      const uint32_t at = queued + rank_below(b);
      qput<D0, D1, kQRow>(wq, at, r0 + e);
      if constexpr (D0 != kNone) qput<D0, D1, kQFk0>(wq, at, pick4(fk0, e));
      if constexpr (D1 != kNone) qput<D0, D1, kQFk1>(wq, at, pick4(fk1, e));
    }
    queued += popc64(b);
    ++e;
    __builtin_amdgcn_wave_barrier();
  }
}

// Dims built without duplicate keys stop probing at the first match.
template <int D>
__device__ __forceinline__ int match_limit(const PipeDim& d) {
  if constexpr (D == kNone) return 1;
  else return *d.map.dup ? 2 : 1;
}

// Whether every dim of plan p resolved to a direct table (a plan without
// dims qualifies); read by each workgroup from the builds' state.
template <int D0, int D1>
__device__ __forceinline__ bool all_direct(const PipelineParams& p) {
  if constexpr (!kDirectOk<D0> || !kDirectOk<D1>) {
    return false;
  } else {
    if constexpr (D0 != kNone)
      if (!dim_direct<D0>(p.dim[0]).mode) return false;
    if constexpr (D1 != kNone)
      if (!dim_direct<D1>(p.dim[1]).mode) return false;
    return true;
  }
}

// Whether some dim resolved to a direct table.
template <int D0, int D1>
__device__ __forceinline__ bool any_direct(const PipelineParams& p) {
  if constexpr (D0 != kNone)
    if (dim_direct<D0>(p.dim[0]).mode) return true;
  if constexpr (D1 != kNone)
    if (dim_direct<D1>(p.dim[1]).mode) return true;
  return false;
}

// Whether a dim build saw a duplicate key.
template <int D0, int D1>
__device__ __forceinline__ bool has_dup_dims(const PipelineParams& p) {
  if constexpr (D0 == kNone) return false;
  else if constexpr (D1 == kNone) return *p.dim[0].map.dup != 0;
  else return *p.dim[0].map.dup != 0 || *p.dim[1].map.dup != 0;
}

// Eight waves per SIMD (four resident workgroups per CU) where the variant
// fits 64 VGPRs without spilling; variants with an int64 dim or an LDS copy
// as second dim keep the compiler's own register budget.
template <int D0, int D1>
constexpr int kFusedWaves = (D1 == kMapLds || D1 == kSetLds || D1 == kMap64) ? 1 : 8;

template <int D0, int D1>
__global__ void __launch_bounds__(kPipeThreads)
__attribute__((amdgpu_waves_per_eu(kFusedWaves<D0, D1>))) fused_kernel(PipelineParams p) {
  if (all_direct<D0, D1>(p)) return;  // fused_direct_kernel's case
  // fused_spec_kernel's case
  if (p.spec != 0 && !has_dup_dims<D0, D1>(p) && !any_direct<D0, D1>(p)) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  void* ld0 = lds + p.dim[0].lds_offset;
  void* ld1 = lds + p.dim[1].lds_offset;
  uint64_t* lg = reinterpret_cast<uint64_t*>(lds + p.lds_group_offset);
  const int lane = lane_id();
  unsigned char* wq = lds + p.queue_offset + (threadIdx.x / kWave) * p.queue_stride;
  copy_dim_to_lds<D0>(p.dim[0], ld0);
  copy_dim_to_lds<D1>(p.dim[1], ld1);
  if (p.lds_slots > 0) lds_group_init(lg, p.lds_slots, p.g);
  __syncthreads();
  const GroupTable gt = group_replica(p.g, blockIdx.x % p.g.replicas);
  run_tiles<D0, D1, false>(p, blockIdx.x, p.ntiles, gridDim.x, wq, lane, ld0, ld1, lg, gt,
                           match_limit<D0>(p.dim[0]), match_limit<D1>(p.dim[1]));
  if (p.lds_slots == 0) return;
  __syncthreads();
  lds_group_flush(lg, p.lds_slots, p.g);
}

// The plan under row spec S (p.spec == S) with hash-table dims free of
// duplicate keys; fused_kernel then returns at once.
template <int D0, int D1, int S>
__global__ void __launch_bounds__(kPipeThreads)
__attribute__((amdgpu_waves_per_eu(8, 8))) fused_spec_kernel(PipelineParams p) {
  if (any_direct<D0, D1>(p) || has_dup_dims<D0, D1>(p)) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  uint64_t* lg = reinterpret_cast<uint64_t*>(lds + p.lds_group_offset);
  const int lane = lane_id();
  unsigned char* wq = lds + p.queue_offset + (threadIdx.x / kWave) * p.queue_stride;
  if (p.lds_slots > 0) lds_group_init(lg, p.lds_slots, p.g);
  __syncthreads();
  const GroupTable gt = group_replica(p.g, blockIdx.x % p.g.replicas);
  spec_tiles<D0, D1, S>(p, blockIdx.x, p.ntiles, gridDim.x, wq, lane, lg, gt);
  if (p.lds_slots == 0) return;
  __syncthreads();
  lds_group_flush(lg, p.lds_slots, p.g);
}

// The same plan when all_direct holds (fused_kernel then returns at once):
// its own kernel, so that the lean loop gets its own register allocation.
template <int D0, int D1, int S = 0>
__global__ void __launch_bounds__(kPipeThreads)
__attribute__((amdgpu_waves_per_eu(8))) fused_direct_kernel(PipelineParams p) {
  if (!all_direct<D0, D1>(p)) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  uint64_t* lg = reinterpret_cast<uint64_t*>(lds + p.lds_group_offset);
  const int lane = lane_id();
  unsigned char* wq = lds + p.queue_offset + (threadIdx.x / kWave) * p.queue_stride;
  if (p.lds_slots > 0) lds_group_init(lg, p.lds_slots, p.g);
  __syncthreads();
  const GroupTable gt = group_replica(p.g, blockIdx.x % p.g.replicas);
  run_tiles<D0, D1, true, S>(p, blockIdx.x, p.ntiles, gridDim.x, wq, lane, nullptr, nullptr, lg,
                             gt, 1, 1);
  if (p.lds_slots == 0) return;
  __syncthreads();
  lds_group_flush(lg, p.lds_slots, p.g);
}

// ------------------------------------------------------ enumeration pass
//
// Rows with several matches in a dim (duplicate dim keys) are skipped by the
// fused kernel and handled here, one row per thread: every combination of
// matching dim rows is aggregated. The pass returns at once when no dim build
// saw a duplicate key, so plans over unique dims pay only a launch.

template <int D>
struct HbmMode {
  static constexpr int value = D == kMapLds ? kMap : (D == kSetLds ? kSet : D);
};

__device__ __forceinline__ bool row_passes(const PipelineParams& p, int64_t r) {
  for (int t = 0; t < p.nterms; ++t) {
    const int c = p.term_col[t];
    if (!term_holds(p.term_op[t], load_elem(p.fact[c], p.fact_type[c], r), p.term_lo[t],
                    p.term_hi[t]))
      return false;
  }
  return true;
}

template <int D>
__device__ __forceinline__ int count_upto2(const PipeDim& d, int64_t key) {
  uint32_t v = 0;
  if constexpr (D == kMap || D == kSet || D == kCSet) {
    const DirectView dv = direct_view(d.map);
    if (dv.mode) return direct_probe(dv, key, v) ? 1 : 0;
  }
  return probe_finish<D>(d, nullptr, key, 2, probe_first<D>(d, nullptr, key), v);
}


// Rows r, r + stride, ... below `end`: aggregates every row that passes and
// matches some dim more than once.
template <int D0, int D1>
__device__ __forceinline__ void multi_rows(const PipelineParams& p, int64_t r, int64_t end,
                                           int64_t stride, uint64_t* lg, const GroupTable& gt) {
  constexpr int H0 = HbmMode<D0>::value, H1 = HbmMode<D1>::value;
  for (; r < end; r += stride) {
    if (!row_passes(p, r)) continue;
    const int64_t fk0 = load_elem(p.fact[p.dim[0].fk_col], p.fact_type[p.dim[0].fk_col], r);
    const int m0 = count_upto2<H0>(p.dim[0], fk0);
    if (m0 == 0) continue;
    int m1 = 1;
    if constexpr (D1 != kNone) {
      const int64_t fk1 = load_elem(p.fact[p.dim[1].fk_col], p.fact_type[p.dim[1].fk_col], r);
      m1 = count_upto2<H1>(p.dim[1], fk1);
      if (m1 == 0) continue;
    }
    if (m0 < 2 && m1 < 2) continue;  // single match: aggregated by the fused kernel
    enumerate_row<H0, H1>(p, r, nullptr, nullptr, lg, gt);
  }
}

template <int D0, int D1>
__global__ void __launch_bounds__(256) multi_kernel(PipelineParams p) {
  if (!has_dup_dims<D0, D1>(p)) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  uint64_t* lg = reinterpret_cast<uint64_t*>(lds);
  if (p.lds_slots > 0) lds_group_init(lg, p.lds_slots, p.g);
  __syncthreads();
  const GroupTable gt = group_replica(p.g, blockIdx.x % p.g.replicas);
  multi_rows<D0, D1>(p, blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x, p.n,
                     static_cast<int64_t>(gridDim.x) * blockDim.x, lg, gt);
  if (p.lds_slots == 0) return;
  __syncthreads();
  lds_group_flush(lg, p.lds_slots, p.g);
}

template <int D0, int D1>
hipError_t launch_multi(const PipelineParams& p, hipStream_t s) {
  if constexpr (D0 == kNone) {
    return hipSuccess;
  } else {
    const size_t lds = static_cast<size_t>(p.lds_slots) * p.g.words * 8;
    int64_t blocks = (p.n + 255) / 256;
    const int64_t limit = static_cast<int64_t>(device_info().cu_count) * 8;
    if (blocks > limit) blocks = limit;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((multi_kernel<D0, D1>), dim3(static_cast<unsigned>(blocks)), dim3(256), lds,
                       s, p);
    return hipGetLastError();
  }
}

// grid <= 0 sizes the persistent grid of kernel k to `rounds` times the
// workgroups that can be resident at once (registers and LDS), capped by the
// tile count. `max_dynamic` caches the kernel's dynamic LDS limit (set on
// first use).
inline hipError_t launch_persistent(const void* k, const PipelineParams& p, int grid,
                                    int& max_dynamic, hipStream_t s, int rounds = 1) {
  if (max_dynamic < 0) {
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, k);
    if (e != hipSuccess) return e;
    const int dyn = device_info().lds_per_block - static_cast<int>(attr.sharedSizeBytes);
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    if (e != hipSuccess) return e;
    max_dynamic = dyn;
  }
  if (static_cast<int>(p.lds_bytes) > max_dynamic) return hipErrorInvalidValue;
  if (grid <= 0) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kPipeThreads,
                                                                p.lds_bytes);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    int64_t g = static_cast<int64_t>(device_info().cu_count) * per_cu * rounds;
    if (g > p.ntiles) g = p.ntiles;
    if (g > kMaxPipeGrid) g = kMaxPipeGrid;
    grid = static_cast<int>(g < 1 ? 1 : g);
  }
  if (grid > kMaxPipeGrid) grid = kMaxPipeGrid;
  void* args[] = {const_cast<PipelineParams*>(&p)};
  hipError_t e = hipLaunchKernel(k, dim3(grid), dim3(kPipeThreads), args, p.lds_bytes, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// Launches the fused kernel, its direct-table twin where the dim modes allow
// one (exactly one of the two does the work, decided on the device from the
// builds), and the duplicate-key pass; under row spec S (p.spec == S) the
// specialised kernel and twin as well. Returns the first failing HIP status.
template <int D0, int D1, int S>
hipError_t launch_fused_spec(const PipelineParams& p, int grid, hipStream_t s) {
  static int max_general = -1;
  hipError_t e = launch_persistent(reinterpret_cast<const void*>(fused_kernel<D0, D1>), p, grid,
                                   max_general, s);
  if (e != hipSuccess) return e;
  if constexpr (S != 0) {
    // two rounds of workgroups: the hash probes make tiles uneven in cost,
    // and workgroups that start as others end even out the tail (600M-row
    // star plan: 4.38 against 4.48 ms; the direct-table twin is faster with
    // one round)
    static int max_spec = -1;
    e = launch_persistent(reinterpret_cast<const void*>(fused_spec_kernel<D0, D1, S>), p, grid,
                          max_spec, s, 2);
    if (e != hipSuccess) return e;
  }
  if constexpr (kDirectOk<D0> && kDirectOk<D1>) {
    if (p.directable) {
      static int max_direct = -1;
      e = launch_persistent(reinterpret_cast<const void*>(fused_direct_kernel<D0, D1, S>), p, grid,
                            max_direct, s);
      if (e != hipSuccess) return e;
    }
  }
  return launch_multi<D0, D1>(p, s);
}

// Dispatch on the plan's row spec: the specialised variants built for dim
// modes (D0, D1), else the generic kernel (p.spec is then cleared, so that
// the generic kernel does the work).
template <int D0, int D1>
hipError_t launch_fused(const PipelineParams& p, int grid, hipStream_t s) {
  if constexpr (spec_ok<D0, D1, kSpecDim1F8>())
    if (p.spec == kSpecDim1F8) return launch_fused_spec<D0, D1, kSpecDim1F8>(p, grid, s);
  if constexpr (spec_ok<D0, D1, kSpecDim0>())
    if (p.spec == kSpecDim0) return launch_fused_spec<D0, D1, kSpecDim0>(p, grid, s);
  if constexpr (spec_ok<D0, D1, kSpecDim1>())
    if (p.spec == kSpecDim1) return launch_fused_spec<D0, D1, kSpecDim1>(p, grid, s);
  if (p.spec == 0) return launch_fused_spec<D0, D1, 0>(p, grid, s);
  PipelineParams q = p;
  q.spec = 0;
  return launch_fused_spec<D0, D1, 0>(q, grid, s);
}

// ------------------------------------------------------------ batched plans

// Rows in place: with no predicate every row of a tile is processed, so the
// row queue's compaction buys nothing. Each thread takes its own four rows
// of a tile and issues their value loads and payload reads together before
// any update, one memory round trip per tile instead of one per queued
// 64-row batch. For batched plans whose one dim resolved to a direct table.
template <int D0>
__device__ __forceinline__ void inplace_tiles(const PipelineParams& p, int64_t tile, int64_t end,
                                              uint64_t* lg, const GroupTable& gt) {
  const DirectView dv0 = dim_direct<D0>(p.dim[0]);
  const uint32_t acode = acc_code(p);
  const int64_t n = p.n;
  const int nkeys = p.g.kp.nkeys;
  const bool fkey0 = nkeys > 0 && p.key_src[0] == 0;
  const bool fkey1 = nkeys > 1 && p.key_src[1] == 0;
  for (; tile < end; ++tile) {
    const int64_t r0 = tile * static_cast<int64_t>(kPipeTile) + threadIdx.x * 4;
    typename KeyOf<D0>::T fk[4];
    load_keys4<D0>(p, p.dim[0].fk_col, r0, fk);
    int64_t va[4] = {0, 0, 0, 0}, vb[4] = {0, 0, 0, 0}, f0[4] = {0, 0, 0, 0}, f1[4] = {0, 0, 0, 0};
    if (p.early_col[0] >= 0) load_col4(p, p.early_col[0], r0, va);
    if (p.early_col[1] >= 0) load_col4(p, p.early_col[1], r0, vb);
    if (fkey0) load_col4(p, p.key_col[0], r0, f0);
    if (fkey1) load_col4(p, p.key_col[1], r0, f1);
    uint32_t v0[4] = {0, 0, 0, 0};
    bool ok[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) ok[e] = r0 + e < n && direct_probe(dv0, fk[e], v0[e]);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (!ok[e]) continue;
      const int64_t k0 = fkey0 ? f0[e] : static_cast<int32_t>(v0[e]);
      const int64_t k1 = fkey1 ? f1[e] : static_cast<int32_t>(v0[e]);
      update_group<true>(p, r0 + e, pack_keys(p.g.kp, k0, k1), va[e], vb[e], lg, gt, acode);
    }
  }
}
//
// Persistent workgroups take (instance, tile range) items from the batch's
// device counter and walk the tiles of that instance's plan exactly as the
// single-plan kernel does; the LDS group table is set up and flushed per
// item. Dim tables stay in HBM, where L2 keeps the small ones.

// The batched kernel keeps more per-item state: the eight-wave budget only
// for plans with one dim.
template <int D0, int D1>
constexpr int kBatchWaves = D1 == kNone ? 8 : 1;

template <int D0, int D1>
__global__ void __launch_bounds__(kPipeThreads)
__attribute__((amdgpu_waves_per_eu(kBatchWaves<D0, D1>))) batch_fused_kernel(BatchParams b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ uint32_t s_item;
  uint64_t* lg = reinterpret_cast<uint64_t*>(lds);
  const int lane = lane_id();
  for (;;) {
    if (threadIdx.x == 0) s_item = static_cast<uint32_t>(atomicAdd(b.counter, 1ULL));
    __syncthreads();
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
    if (item >= b.ntile) return;
    const BatchItem& it = batch_at(b.tile_items, item);
    const PipelineParams& p = batch_at(b.plans, it.inst);
    unsigned char* wq = lds + p.queue_offset + (threadIdx.x / kWave) * p.queue_stride;
    if (p.lds_slots > 0) lds_group_init(lg, p.lds_slots, p.g);
    const uint32_t parts = p.rec.parts;
    uint32_t* hist = reinterpret_cast<uint32_t*>(lds + p.rec.lds_offset);
    if (parts)
      for (uint32_t q = threadIdx.x; q <= parts; q += blockDim.x) hist[q] = 0;
    __syncthreads();
    const GroupTable gt = group_replica(p.g, blockIdx.x % p.g.replicas);
    bool done = false;
    if constexpr (D1 == kNone && kDirectable<D0>) {
      if (p.nterms == 0 && dim_direct<D0>(p.dim[0]).mode) {
        inplace_tiles<D0>(p, it.begin, it.end, lg, gt);
        done = true;
      }
    }
    if (!done)
      run_tiles<D0, D1, false, 0, true>(p, it.begin, it.end, 1, wq, lane, nullptr, nullptr, lg,
                                        gt, match_limit<D0>(p.dim[0]), match_limit<D1>(p.dim[1]));
    __syncthreads();
    if (p.lds_slots > 0 || parts) {
      if (p.lds_slots > 0) lds_group_flush(lg, p.lds_slots, p.g);
      if (parts) {
        // the item's record count per partition, added to the partition's
        // total
        const uint32_t j = static_cast<uint32_t>(it.begin / p.rec.item_tiles);
        uint32_t* row = p.rec.counts + static_cast<uint64_t>(j) * parts;
        for (uint32_t q = threadIdx.x; q < parts; q += blockDim.x) {
          const uint32_t c = hist[q];
          row[q] = c;
          if (c) atomicAdd(p.rec.cursor + q, c);
        }
        if (threadIdx.x == 0) p.rec.item_n[j] = hist[parts];
      }
      __syncthreads();
    }
  }
}

// One workgroup per tile item: the rows of duplicate-key matches.
template <int D0, int D1>
__global__ void __launch_bounds__(256) batch_multi_kernel(BatchParams b) {
  const BatchItem& it = batch_at(b.tile_items, blockIdx.x);
  const PipelineParams& p = batch_at(b.plans, it.inst);
  if (!has_dup_dims<D0, D1>(p)) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  uint64_t* lg = reinterpret_cast<uint64_t*>(lds);
  if (p.lds_slots > 0) lds_group_init(lg, p.lds_slots, p.g);
  __syncthreads();
  const GroupTable gt = group_replica(p.g, blockIdx.x % p.g.replicas);
  int64_t end = static_cast<int64_t>(it.end) * kPipeTile;
  if (end > p.n) end = p.n;
  multi_rows<D0, D1>(p, static_cast<int64_t>(it.begin) * kPipeTile + threadIdx.x, end, blockDim.x,
                     lg, gt);
  if (p.lds_slots == 0) return;
  __syncthreads();
  lds_group_flush(lg, p.lds_slots, p.g);
}

template <int D0, int D1>
hipError_t launch_batch_fused(const BatchParams& b, int grid, hipStream_t s) {
  auto k = batch_fused_kernel<D0, D1>;
  static int max_dynamic = -1;
  if (max_dynamic < 0) {
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(k));
    if (e != hipSuccess) return e;
    const int dyn = device_info().lds_per_block - static_cast<int>(attr.sharedSizeBytes);
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                            hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    if (e != hipSuccess) return e;
    max_dynamic = dyn;
  }
  if (static_cast<int>(b.lds_bytes) > max_dynamic) return hipErrorInvalidValue;
  if (b.ntile == 0) return hipSuccess;
  if (grid <= 0) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kPipeThreads,
                                                                b.lds_bytes);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    int64_t g = static_cast<int64_t>(device_info().cu_count) * per_cu;
    if (g > b.ntile) g = b.ntile;
    grid = static_cast<int>(g < 1 ? 1 : g);
  }
  if (grid > kMaxPipeGrid) grid = kMaxPipeGrid;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kPipeThreads), b.lds_bytes, s, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if constexpr (D0 != kNone) {
    hipLaunchKernelGGL((batch_multi_kernel<D0, D1>), dim3(b.ntile), dim3(256), b.group_lds_bytes,
                       s, b);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace pipe
}  // namespace rel
