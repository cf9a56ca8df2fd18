// Radix-partitioned hash aggregation for many groups (the hash-based
// grouping of Section 4.2 when the group table is far larger than the
// caches: there every row would otherwise pay a random read-modify-write of a
// table line in HBM).
//
//   count     workgroup w of kPartGroups takes a fixed range of rows and
//             counts them per bucket (top b1 hash bits); a prefix sum over
//             the (bucket, workgroup) counts places every segment;
//   scatter 1 the same ranges: rows -> records in their segment, at the
//             workgroup's own LDS cursor (no global atomics). A small LDS
//             table aggregates the keys it already holds (under skew, the hot
//             ones, met first); only the other rows become records, so a
//             segment may end short of its count (its fill is recorded). The
//             pass also counts the records of every partition;
//   scatter 2 each segment's records -> records grouped by partition (the
//             next b2 hash bits), at exact offsets;
//   aggregate each partition, in pieces of at most `piece` records, is
//             folded into an LDS table sized to hold all of a partition's
//             keys, which then merges into the global table with one update
//             per key. A key that finds no LDS slot updates the global table
//             directly, so results never depend on the sizing.
//
// The same counting and scatter passes serve the partitioned map build
// (rel_hash_join over large build sides): records are (key, row id),
// partitioned by the top bits of the map's home hash, so that a partition
// holds exactly the keys whose home slots fall in its range of the slot
// array. Each range is built in LDS by linear probing and written out whole;
// a key whose probe run passes the end of its range is inserted afterwards by
// global CAS, once every range is in place.
//
// Within a tile of the second scatter, a record's position is the tile's
// claim on its partition (one atomic per partition and tile, on a cursor of
// its own 128-byte line) plus the record's rank among the tile's records for
// it (an LDS atomic). Record order inside a partition is therefore
// arbitrary; the aggregates are exact integer sums, minima and maxima, so
// they do not depend on it.

#include "internal.h"
#include "group_lds.h"

namespace rel {

namespace {

constexpr uint32_t kNoRecord = 0xFFFFFFFFu;
// LDS probe windows: the first scatter's table only serves keys it met early
// (short window); the aggregation table is sized for its partition.
constexpr int kPreProbe = 8;
constexpr int kAggProbe = 64;
constexpr int kAggRows = 4;
// Rows per thread and step of the first scatter (16 would hold twice the
// loads in flight per wave, but at its register count only one workgroup
// fits a CU and the LDS table probes go unhidden).
constexpr int kScatterRows = 8;

__device__ __forceinline__ uint64_t row_col(const PartParams& p, int c, uint64_t r) {
  const int64_t i = p.col_idx[c] ? static_cast<int64_t>(p.col_idx[c][r]) : static_cast<int64_t>(r);
  return static_cast<uint64_t>(load_elem(p.col_data[c], p.col_type[c], i));
}

// Elements r0 + e * step (e < N) of a column, gathered through idx when
// given. Rows at or past n read row 0 (callers ignore them; n > 0), and the
// type test is outside the row loop, so the N loads issue back to back.
template <int N>
__device__ __forceinline__ void load_rows(const void* data, int32_t type, const uint32_t* idx,
                                          uint64_t r0, uint64_t step, uint64_t n, int64_t* out) {
  uint64_t at[N];
#pragma unroll
  for (int e = 0; e < N; ++e) {
    const uint64_t r = r0 + static_cast<uint64_t>(e) * step;
    at[e] = r < n ? r : 0;
  }
  if (idx) {
#pragma unroll
    for (int e = 0; e < N; ++e) at[e] = idx[at[e]];
  }
  if (type == kI64) {
    const int64_t* d = static_cast<const int64_t*>(data);
#pragma unroll
    for (int e = 0; e < N; ++e) out[e] = d[at[e]];
  } else if (type == kI32) {
    const int32_t* d = static_cast<const int32_t*>(data);
#pragma unroll
    for (int e = 0; e < N; ++e) out[e] = d[at[e]];
  } else {
    const int8_t* d = static_cast<const int8_t*>(data);
#pragma unroll
    for (int e = 0; e < N; ++e) out[e] = d[at[e]];
  }
}

// Packed keys of rows r0 + e * step (e < N; at least one key column).
template <int N>
__device__ __forceinline__ void load_keys(const PartParams& p, uint64_t r0, uint64_t step,
                                          uint64_t n, uint64_t* pk) {
  int64_t k0[N], k1[N];
  load_rows<N>(p.key_data[0], p.g.kp.type[0], p.key_idx[0], r0, step, n, k0);
  if (p.g.kp.nkeys > 1) {
    load_rows<N>(p.key_data[1], p.g.kp.type[1], p.key_idx[1], r0, step, n, k1);
  } else {
#pragma unroll
    for (int e = 0; e < N; ++e) k1[e] = 0;
  }
#pragma unroll
  for (int e = 0; e < N; ++e) pk[e] = pack_keys(p.g.kp, k0[e], k1[e]);
}

// The hash whose top bits pick a record's partition: the map's home hash for
// map builds of int32 keys, else hash64 of the packed key (which is also the
// home hash of int64 maps and of group tables).
__device__ __forceinline__ uint64_t part_hash(const PartParams& p, uint64_t pk) {
  if (p.map_key == kI32) return static_cast<uint64_t>(hash32(static_cast<uint32_t>(pk))) << 32;
  return hash64(pk);
}

__device__ __forceinline__ uint32_t part_of(const PartParams& p, uint64_t pk, int bits) {
  return static_cast<uint32_t>(part_hash(p, pk) >> (64 - bits));
}

// Map builds: the sentinel key pattern never enters a slot array.
__device__ __forceinline__ bool map_sentinel(const PartParams& p, uint64_t pk) {
  if (p.map_key == kI64) return pk == kEmpty64;
  return p.map_key == kI32 && static_cast<int32_t>(static_cast<uint32_t>(pk)) == kEmpty32;
}

// Exclusive prefix of v over the workgroup (thread order); *total gets the
// sum. Every thread must call it.
__device__ __forceinline__ unsigned long long block_scan(unsigned long long v,
                                                         unsigned long long* total) {
  __shared__ unsigned long long s_w[1024 / kWave];
  const int lane = lane_id(), wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  unsigned long long incl = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const unsigned long long t = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += t;
  }
  if (lane == kWave - 1) s_w[wave] = incl;
  __syncthreads();
  unsigned long long before = 0, sum = 0;
  for (int w = 0; w < nwaves; ++w) {
    if (w < wave) before += s_w[w];
    sum += s_w[w];
  }
  __syncthreads();
  *total = sum;
  return before + incl - v;
}

// Tiles [*t0, *t1) of workgroup w (the same in the count and first scatter).
__device__ __forceinline__ void group_tiles(uint64_t n, uint32_t w, uint64_t* t0, uint64_t* t1) {
  const uint64_t ntiles = (n + kPartTile - 1) / kPartTile;
  const uint64_t per = (ntiles + kPartGroups - 1) / kPartGroups;
  *t0 = w * per;
  *t1 = *t0 + per < ntiles ? *t0 + per : ntiles;
}

__global__ void __launch_bounds__(kPartThreads) part_count_kernel(PartParams p) {
  __shared__ uint32_t h[1 << kPartLevelBits];
  const int nb = 1 << p.b1;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const uint64_t n = static_cast<uint64_t>(p.n);
  uint64_t t0, t1;
  group_tiles(n, blockIdx.x, &t0, &t1);
  for (uint64_t tile = t0; tile < t1; ++tile) {
    const uint64_t r0 = tile * kPartTile + threadIdx.x;
    uint64_t pk[kPartRows];
    load_keys<kPartRows>(p, r0, kPartThreads, n, pk);
#pragma unroll
    for (int e = 0; e < kPartRows; ++e)
      if (r0 + static_cast<uint64_t>(e) * kPartThreads < n) atomicAdd(&h[part_of(p, pk[e], p.b1)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    p.ctl[kCtlSegCount + static_cast<uint64_t>(b) * kPartGroups + blockIdx.x] = h[b];
}

// Segment starts from the segment counts, bucket-major (one workgroup of
// 1024; 2^b1 * kPartGroups is a multiple of 1024).
__global__ void __launch_bounds__(1024) part_scan1_kernel(PartParams p) {
  const uint64_t segs = static_cast<uint64_t>(kPartGroups) << p.b1;
  const uint64_t per = segs / blockDim.x;
  const uint64_t lo = threadIdx.x * per;
  unsigned long long sum = 0;
  for (uint64_t i = lo; i < lo + per; ++i) sum += p.ctl[kCtlSegCount + i];
  unsigned long long total;
  unsigned long long at = block_scan(sum, &total);
  for (uint64_t i = lo; i < lo + per; ++i) {
    p.ctl[kCtlSegStart + i] = at;
    at += p.ctl[kCtlSegCount + i];
  }
  if (threadIdx.x == 0) p.ctl[kCtlSegStart + segs] = total;
}

// kPair: one value column (two-word records); the values are loaded with
// the keys, so that writing a record needs no load. kRows: rows per thread
// and step; a tile is taken in kPartRows / kRows steps.
template <bool kPair, int kRows>
__global__ void __launch_bounds__(kPartThreads) part_scatter1_kernel(PartParams p) {
  extern __shared__ uint64_t lds[];
  const GroupDesc& g = p.g;
  const int pb = p.b1 + p.b2;
  const uint32_t nparts = 1u << pb;
  const int nb = 1 << p.b1;
  uint64_t* pre = lds;
  uint32_t* h2 = reinterpret_cast<uint32_t*>(lds + static_cast<size_t>(p.pre_slots) * g.words);
  uint32_t* cnt = h2 + nparts;
  unsigned long long* cur = reinterpret_cast<unsigned long long*>(cnt + (1 << kPartLevelBits));
  if (p.pre_slots > 0) lds_group_init(pre, p.pre_slots, g);
  for (uint32_t i = threadIdx.x; i < nparts; i += blockDim.x) h2[i] = 0;
  const uint64_t seg0 = blockIdx.x;  // segment of bucket b: seg0 + b * kPartGroups
  if (threadIdx.x < nb) {
    cnt[threadIdx.x] = 0;
    cur[threadIdx.x] = p.ctl[kCtlSegStart + seg0 + static_cast<uint64_t>(threadIdx.x) * kPartGroups];
  }
  __syncthreads();

  const uint64_t n = static_cast<uint64_t>(p.n);
  uint64_t t0, t1;
  group_tiles(n, blockIdx.x, &t0, &t1);
  for (uint64_t step = t0 * (kPartRows / kRows); step < t1 * (kPartRows / kRows); ++step) {
    const uint64_t r0 = step * (kPartThreads * kRows) + threadIdx.x;
    uint64_t pk[kRows];
    int64_t val[kPair ? kRows : 1];
    uint32_t code[kRows];
    load_keys<kRows>(p, r0, kPartThreads, n, pk);
    if constexpr (kPair) {
      if (p.value_row) {
#pragma unroll
        for (int e = 0; e < kRows; ++e) {
          const uint64_t r = r0 + static_cast<uint64_t>(e) * kPartThreads;
          const uint64_t at = r < n ? r : 0;
          val[e] = p.key_idx[0] ? static_cast<int64_t>(p.key_idx[0][at]) : static_cast<int64_t>(at);
        }
      } else {
        load_rows<kRows>(p.col_data[0], p.col_type[0], p.col_idx[0], r0, kPartThreads, n, val);
      }
    }
#pragma unroll
    for (int e = 0; e < kRows; ++e) {
      const uint64_t r = r0 + static_cast<uint64_t>(e) * kPartThreads;
      code[e] = kNoRecord;
      if (r >= n) continue;
      if (kPair && map_sentinel(p, pk[e])) {
        // out of band, as the map's own inserts do
        const unsigned long long pos = atomicAdd(p.oob_count, 1ULL);
        p.oob_vals[pos] = static_cast<uint32_t>(val[e]);
        if (pos > 0) *p.dup = 1;
        continue;
      }
      const int32_t s = lds_group_find(pre, p.pre_slots, g.words, pk[e], kPreProbe);
      if (s >= 0) {
        uint64_t acc[kMaxAcc];
#pragma unroll
        for (int a = 0; a < kMaxAcc; ++a)
          if (a < g.ap.nacc) acc[a] = kPair ? static_cast<uint64_t>(val[e]) : row_col(p, p.src[a], r);
        lds_group_update(pre + static_cast<size_t>(s) * g.words, g.ap, acc);
      } else {
        const uint32_t q = part_of(p, pk[e], pb);
        const uint32_t b = q >> p.b2;
        const uint32_t rank = atomicAdd(&cnt[b], 1u);
        atomicAdd(&h2[q], 1u);
        code[e] = (b << 16) | rank;
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kRows; ++e) {
      if (code[e] == kNoRecord) continue;
      const uint64_t r = r0 + static_cast<uint64_t>(e) * kPartThreads;
      const uint64_t pos = cur[code[e] >> 16] + (code[e] & 0xFFFFu);
      if constexpr (kPair) {
        *reinterpret_cast<ulonglong2*>(p.rec_a + 2 * pos) =
            make_ulonglong2(pk[e], static_cast<uint64_t>(val[e]));
      } else {
        uint64_t* w = p.rec_a + pos * p.rw;
        w[0] = pk[e];
        for (int c = 0; c < p.ncols; ++c) w[1 + c] = row_col(p, c, r);
      }
    }
    __syncthreads();
    if (threadIdx.x < nb) {
      cur[threadIdx.x] += cnt[threadIdx.x];
      cnt[threadIdx.x] = 0;
    }
    __syncthreads();
  }
  if (threadIdx.x < nb) {
    const uint64_t sg = seg0 + static_cast<uint64_t>(threadIdx.x) * kPartGroups;
    p.ctl[kCtlSegFill + sg] = cur[threadIdx.x] - p.ctl[kCtlSegStart + sg];
  }
  if (p.pre_slots > 0) lds_group_flush(pre, p.pre_slots, g);
  for (uint32_t i = threadIdx.x; i < nparts; i += blockDim.x)
    if (h2[i]) atomicAdd(&p.ctl[kCtlHist2 + i], static_cast<unsigned long long>(h2[i]));
}

// Partition starts and cursors, the aggregation pieces of every partition,
// and the second scatter's tiles per bucket (one workgroup of 1024).
__global__ void __launch_bounds__(1024) part_scan2_kernel(PartParams p) {
  const int pb = p.b1 + p.b2;
  const uint32_t nparts = 1u << pb;
  const uint32_t per = (nparts + blockDim.x - 1) / blockDim.x;
  const uint32_t lo = threadIdx.x * per;
  unsigned long long recs = 0, pieces = 0;
  for (uint32_t q = lo; q < lo + per && q < nparts; ++q) {
    const unsigned long long c = p.ctl[kCtlHist2 + q];
    recs += c;
    pieces += (c + p.piece - 1) / p.piece;
  }
  unsigned long long total_recs, total_pieces;
  unsigned long long at = block_scan(recs, &total_recs);
  unsigned long long pat = block_scan(pieces, &total_pieces);
  for (uint32_t q = lo; q < lo + per && q < nparts; ++q) {
    const unsigned long long c = p.ctl[kCtlHist2 + q];
    p.ctl[kCtlStart2 + q] = at;
    p.ctl[kCtlCur2 + static_cast<uint64_t>(q) * kPartPad] = at;
    p.ctl[kCtlPieces + q] = pat;
    at += c;
    pat += (c + p.piece - 1) / p.piece;
  }
  if (threadIdx.x == 0) {
    p.ctl[kCtlStart2 + nparts] = total_recs;
    p.ctl[kCtlPieces + nparts] = total_pieces;
  }
  // second-scatter tiles per segment
  const uint64_t segs = static_cast<uint64_t>(kPartGroups) << p.b1;
  const uint64_t sper = segs / blockDim.x;
  const uint64_t slo = threadIdx.x * sper;
  unsigned long long tiles = 0;
  for (uint64_t i = slo; i < slo + sper; ++i) tiles += (p.ctl[kCtlSegFill + i] + kPartTile - 1) / kPartTile;
  unsigned long long total_tiles;
  unsigned long long tat = block_scan(tiles, &total_tiles);
  for (uint64_t i = slo; i < slo + sper; ++i) {
    p.ctl[kCtlTiles + i] = tat;
    tat += (p.ctl[kCtlSegFill + i] + kPartTile - 1) / kPartTile;
  }
  if (threadIdx.x == 0) p.ctl[kCtlTiles + segs] = total_tiles;
}

// kPair: records of two words (one value column), held in registers between
// the counting and the writing half of a tile; wider records are read again
// (from L2) when written.
template <bool kPair>
__global__ void __launch_bounds__(kPartThreads) part_scatter2_kernel(PartParams p) {
  __shared__ uint32_t cnt[1 << kPartLevelBits];
  __shared__ unsigned long long base[1 << kPartLevelBits];
  const int n2 = 1 << p.b2;
  const int pb = p.b1 + p.b2;
  const uint64_t segs = static_cast<uint64_t>(kPartGroups) << p.b1;
  const unsigned long long* tiles = p.ctl + kCtlTiles;
  const unsigned long long ntiles = tiles[segs];
  for (unsigned long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    // segment sg: the last with tiles[sg] <= t
    uint64_t lo = 0, hi = segs;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) / 2;
      if (tiles[mid] <= t) lo = mid;
      else hi = mid;
    }
    const uint64_t sg = lo;
    const uint64_t b = sg / kPartGroups;
    const uint64_t sstart = p.ctl[kCtlSegStart + sg];
    const uint64_t first = sstart + (t - tiles[sg]) * kPartTile;
    const uint64_t end = sstart + p.ctl[kCtlSegFill + sg];
    if (threadIdx.x < n2) cnt[threadIdx.x] = 0;
    __syncthreads();
    uint64_t pk[kPartRows], val[kPair ? kPartRows : 1];
    uint32_t code[kPartRows];
#pragma unroll
    for (int e = 0; e < kPartRows; ++e) {
      uint64_t i = first + threadIdx.x + static_cast<uint64_t>(e) * kPartThreads;
      i = i < end ? i : first;  // past the end: a valid record, ignored below
      if constexpr (kPair) {
        const ulonglong2 r = *reinterpret_cast<const ulonglong2*>(p.rec_a + 2 * i);
        pk[e] = r.x;
        val[e] = r.y;
      } else {
        pk[e] = p.rec_a[i * p.rw];
      }
    }
#pragma unroll
    for (int e = 0; e < kPartRows; ++e) {
      const uint64_t i = first + threadIdx.x + static_cast<uint64_t>(e) * kPartThreads;
      code[e] = kNoRecord;
      if (i >= end) continue;
      const uint32_t j = part_of(p, pk[e], pb) & static_cast<uint32_t>(n2 - 1);
      code[e] = (j << 16) | atomicAdd(&cnt[j], 1u);
    }
    __syncthreads();
    if (threadIdx.x < n2 && cnt[threadIdx.x]) {
      const uint64_t q = (b << p.b2) + threadIdx.x;
      base[threadIdx.x] = atomicAdd(&p.ctl[kCtlCur2 + q * kPartPad],
                                    static_cast<unsigned long long>(cnt[threadIdx.x]));
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kPartRows; ++e) {
      if (code[e] == kNoRecord) continue;
      const uint64_t i = first + threadIdx.x + static_cast<uint64_t>(e) * kPartThreads;
      const uint64_t pos = base[code[e] >> 16] + (code[e] & 0xFFFFu);
      if constexpr (kPair) {
        *reinterpret_cast<ulonglong2*>(p.rec_b + 2 * pos) = make_ulonglong2(pk[e], val[e]);
      } else {
        const uint64_t* src = p.rec_a + i * p.rw;
        uint64_t* dst = p.rec_b + pos * p.rw;
        dst[0] = pk[e];
        for (int c = 1; c < p.rw; ++c) dst[c] = src[c];
      }
    }
    __syncthreads();
  }
}

// kPair: two-word records, read with one 16-byte load each.
template <bool kPair>
__global__ void __launch_bounds__(kPartAggThreads) part_agg_kernel(PartParams p) {
  extern __shared__ uint64_t table[];
  const GroupDesc& g = p.g;
  const GroupTable gt = group_replica(g, 0);
  const uint32_t nparts = 1u << (p.b1 + p.b2);
  const unsigned long long* pieces = p.ctl + kCtlPieces;
  const unsigned long long total = pieces[nparts];
  for (unsigned long long pc = blockIdx.x; pc < total; pc += gridDim.x) {
    // partition q: the last with pieces[q] <= pc
    uint32_t lo = 0, hi = nparts;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (pieces[mid] <= pc) lo = mid;
      else hi = mid;
    }
    const uint32_t q = lo;
    const uint64_t pstart = p.ctl[kCtlStart2 + q];
    const uint64_t first = pstart + (pc - pieces[q]) * p.piece;
    uint64_t end = pstart + p.ctl[kCtlHist2 + q];
    if (end > first + p.piece) end = first + p.piece;
    lds_group_init(table, p.agg_slots, g);
    __syncthreads();
    // kAggRows records per thread and step: their loads are issued together.
    for (uint64_t i0 = first + threadIdx.x; i0 < end; i0 += kAggRows * blockDim.x) {
      uint64_t pk[kAggRows], acc[kAggRows][kMaxAcc];
#pragma unroll
      for (int e = 0; e < kAggRows; ++e) {
        uint64_t i = i0 + static_cast<uint64_t>(e) * blockDim.x;
        i = i < end ? i : i0;  // past the end: a valid record, ignored below
        if constexpr (kPair) {
          const ulonglong2 r = *reinterpret_cast<const ulonglong2*>(p.rec_b + 2 * i);
          pk[e] = r.x;
#pragma unroll
          for (int a = 0; a < kMaxAcc; ++a) acc[e][a] = r.y;
        } else {
          const uint64_t* rec = p.rec_b + i * p.rw;
          pk[e] = rec[0];
#pragma unroll
          for (int a = 0; a < kMaxAcc; ++a)
            if (a < g.ap.nacc) acc[e][a] = rec[1 + p.src[a]];
        }
      }
#pragma unroll
      for (int e = 0; e < kAggRows; ++e) {
        const uint64_t i = i0 + static_cast<uint64_t>(e) * blockDim.x;
        if (i >= end) continue;
        const int32_t s = lds_group_find(table, p.agg_slots, g.words, pk[e], kAggProbe);
        if (s >= 0) {
          lds_group_update(table + static_cast<size_t>(s) * g.words, g.ap, acc[e]);
        } else {
          uint64_t* d = group_slot(gt, pk[e]);
          if (d) group_update_global(d, g.ap, 1, acc[e]);
        }
      }
    }
    __syncthreads();
    lds_group_flush(table, p.agg_slots, g);
    __syncthreads();
  }
}

// Map builds: partition q covers `sub` consecutive ranges of 2^span_log2
// slots; each range is built in LDS from the partition's records whose home
// slot lies in it, then written out whole.
template <typename K>
__global__ void __launch_bounds__(kPartAggThreads) part_build_kernel(PartParams p, MapDesc m,
                                                                     int span_log2, int sub) {
  extern __shared__ uint64_t slots[];  // 2^span_log2 slots of 16 (int64) or 8 (int32) bytes
  constexpr bool k64 = sizeof(K) == 8;
  const uint32_t nparts = 1u << (p.b1 + p.b2);
  const uint64_t mask = m.cap - 1;
  const uint32_t span = 1u << span_log2;
  for (uint32_t q = blockIdx.x; q < nparts; q += gridDim.x) {
    const uint64_t first = p.ctl[kCtlStart2 + q];
    const uint64_t end = first + p.ctl[kCtlHist2 + q];
    for (int g = 0; g < sub; ++g) {
      const uint64_t range = static_cast<uint64_t>(q) * sub + g;
      const uint64_t base = range << span_log2;
      for (uint32_t i = threadIdx.x; i < span; i += blockDim.x) {
        if constexpr (k64) {
          slots[2 * i] = kEmpty64;
          slots[2 * i + 1] = 0;
        } else {
          slots[i] = kEmptySlot32;
        }
      }
      __syncthreads();
      for (uint64_t i = first + threadIdx.x; i < end; i += blockDim.x) {
        const ulonglong2 rec = reinterpret_cast<const ulonglong2*>(p.rec_b)[i];
        const K key = static_cast<K>(rec.x);
        const uint32_t val = static_cast<uint32_t>(rec.y);
        const uint64_t home = k64 ? home64(key, mask) : home32(static_cast<int32_t>(key), mask);
        if ((home >> span_log2) != range) continue;
        bool placed = false;
        for (uint32_t at = static_cast<uint32_t>(home - base); at < span; ++at) {
          if constexpr (k64) {
            const unsigned long long prev =
                atomicCAS(reinterpret_cast<unsigned long long*>(slots + 2 * at),
                          static_cast<unsigned long long>(kEmpty64), static_cast<unsigned long long>(key));
            if (prev == kEmpty64) {
              slots[2 * at + 1] = val;
              placed = true;
              break;
            }
            if (static_cast<int64_t>(prev) == static_cast<int64_t>(key)) *p.dup = 1;
          } else {
            const unsigned long long prev =
                atomicCAS(reinterpret_cast<unsigned long long*>(slots + at),
                          static_cast<unsigned long long>(kEmptySlot32),
                          static_cast<unsigned long long>(pack32(static_cast<int32_t>(key), val)));
            if (prev == kEmptySlot32) {
              placed = true;
              break;
            }
            if (static_cast<int32_t>(static_cast<uint32_t>(prev)) == static_cast<int32_t>(key)) *p.dup = 1;
          }
        }
        if (!placed) {
          const unsigned long long pos = atomicAdd(&p.ctl[kCtlSpill], 1ULL);
          reinterpret_cast<ulonglong2*>(p.rec_a)[pos] = rec;
        }
      }
      __syncthreads();
      if constexpr (k64) {
        ulonglong2* dst = static_cast<ulonglong2*>(m.slots) + base;
        for (uint32_t i = threadIdx.x; i < span; i += blockDim.x)
          dst[i] = make_ulonglong2(slots[2 * i], slots[2 * i + 1]);
      } else {
        uint64_t* dst = static_cast<uint64_t*>(m.slots) + base;
        for (uint32_t i = threadIdx.x; i < span; i += blockDim.x) dst[i] = slots[i];
      }
      __syncthreads();
    }
  }
}

// Map builds: keys whose probe run left their range, inserted into the
// finished slot array from their home slot on.
template <typename K>
__global__ void __launch_bounds__(256) part_spill_kernel(PartParams p, MapDesc m) {
  const unsigned long long n = p.ctl[kCtlSpill];
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n; i += stride) {
    const ulonglong2 rec = reinterpret_cast<const ulonglong2*>(p.rec_a)[i];
    if constexpr (sizeof(K) == 8) {
      map_insert(Map64{static_cast<ulonglong2*>(m.slots), m.cap - 1, m.oob_count, m.oob_vals},
                 static_cast<int64_t>(rec.x), static_cast<uint32_t>(rec.y), m.dup);
    } else {
      map_insert(Map32{static_cast<uint64_t*>(m.slots), m.cap - 1, m.oob_count, m.oob_vals},
                 static_cast<int32_t>(rec.x), static_cast<uint32_t>(rec.y), m.dup);
    }
  }
}

// Lets a kernel take up to all of a workgroup's LDS as dynamic LDS.
hipError_t allow_dynamic_lds(const void* k) {
  hipFuncAttributes attr;
  hipError_t e = hipFuncGetAttributes(&attr, k);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                             device_info().lds_per_block - static_cast<int>(attr.sharedSizeBytes));
}

hipError_t allow_dynamic_lds_all() {
  const void* kernels[] = {reinterpret_cast<const void*>(part_scatter1_kernel<true, kScatterRows>),
                           reinterpret_cast<const void*>(part_scatter1_kernel<false, kScatterRows>),
                           reinterpret_cast<const void*>(part_agg_kernel<true>),
                           reinterpret_cast<const void*>(part_agg_kernel<false>),
                           reinterpret_cast<const void*>(part_build_kernel<int32_t>),
                           reinterpret_cast<const void*>(part_build_kernel<int64_t>)};
  for (const void* k : kernels) {
    hipError_t e = allow_dynamic_lds(k);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

size_t part_scatter1_lds(const PartParams& p) {
  return static_cast<size_t>(p.pre_slots) * p.g.words * 8 + (sizeof(uint32_t) << (p.b1 + p.b2)) +
         (sizeof(uint32_t) + sizeof(unsigned long long)) * (1u << kPartLevelBits);
}

// The counting and scatter passes (records end up grouped by partition in
// rec_b, with their starts and counts in the control words).
void launch_partition_passes(const PartParams& p, hipStream_t s) {
  hipLaunchKernelGGL(part_count_kernel, dim3(kPartGroups), dim3(kPartThreads), 0, s, p);
  hipLaunchKernelGGL(part_scan1_kernel, dim3(1), dim3(1024), 0, s, p);
  if (p.rw == 2)
    hipLaunchKernelGGL((part_scatter1_kernel<true, kScatterRows>), dim3(kPartGroups),
                       dim3(kPartThreads), part_scatter1_lds(p), s, p);
  else
    hipLaunchKernelGGL((part_scatter1_kernel<false, kScatterRows>), dim3(kPartGroups),
                       dim3(kPartThreads), part_scatter1_lds(p), s, p);
  hipLaunchKernelGGL(part_scan2_kernel, dim3(1), dim3(1024), 0, s, p);
  const int grid = device_info().cu_count * 2;
  if (p.rw == 2)
    hipLaunchKernelGGL(part_scatter2_kernel<true>, dim3(grid), dim3(kPartThreads), 0, s, p);
  else
    hipLaunchKernelGGL(part_scatter2_kernel<false>, dim3(grid), dim3(kPartThreads), 0, s, p);
}

hipError_t launch_group_partitioned(const PartParams& p, hipStream_t s) {
  const int cus = device_info().cu_count;
  static const hipError_t attrs = allow_dynamic_lds_all();  // once per process
  if (attrs != hipSuccess) return attrs;
  {
    ProfileScope ps(kKGroupPartition, s);
    launch_partition_passes(p, s);
  }
  ProfileScope ps(kKGroupAgg, s);
  const size_t agg_lds = static_cast<size_t>(p.agg_slots) * p.g.words * 8;
  if (p.rw == 2)
    hipLaunchKernelGGL(part_agg_kernel<true>, dim3(cus), dim3(kPartAggThreads), agg_lds, s, p);
  else
    hipLaunchKernelGGL(part_agg_kernel<false>, dim3(cus), dim3(kPartAggThreads), agg_lds, s, p);
  return hipGetLastError();
}

hipError_t launch_map_partitioned(const PartParams& p, const MapDesc& m, int span_log2, int sub,
                                  hipStream_t s) {
  const int cus = device_info().cu_count;
  static const hipError_t attrs = allow_dynamic_lds_all();  // once per process
  if (attrs != hipSuccess) return attrs;
  ProfileScope ps(kKMapBuild, s);
  launch_partition_passes(p, s);
  const size_t lds = (static_cast<size_t>(1) << span_log2) * (m.key_type == kI64 ? 16 : 8);
  if (m.key_type == kI64) {
    hipLaunchKernelGGL(part_build_kernel<int64_t>, dim3(cus), dim3(kPartAggThreads), lds, s, p, m,
                       span_log2, sub);
    hipLaunchKernelGGL(part_spill_kernel<int64_t>, dim3(cus), dim3(256), 0, s, p, m);
  } else {
    hipLaunchKernelGGL(part_build_kernel<int32_t>, dim3(cus), dim3(kPartAggThreads), lds, s, p, m,
                       span_log2, sub);
    hipLaunchKernelGGL(part_spill_kernel<int32_t>, dim3(cus), dim3(256), 0, s, p, m);
  }
  return hipGetLastError();
}

}  // namespace rel
