// Radix-partitioned hash aggregation for many groups (the hash-based
// grouping of Section 4.2 when the group table is far larger than the
// caches: there every row would otherwise pay a random read-modify-write of a
// table line in HBM).
//
//   count     per bucket (top b1 hash bits), the rows: an upper bound of
//             each bucket's records, so the first scatter has its regions;
//   scatter 1 rows -> records grouped by bucket. A small per-workgroup LDS
//             table aggregates the keys it already holds (under skew, the
//             hot ones, met first); only the other rows become records. The
//             pass also counts the records of every partition;
//   scatter 2 each bucket's records -> records grouped by partition (the
//             next b2 hash bits), at exact offsets;
//   aggregate each partition, in pieces of at most `piece` records, is
//             folded into an LDS table sized to hold all of a partition's
//             keys, which then merges into the global table with one update
//             per key. A key that finds no LDS slot updates the global table
//             directly, so results never depend on the sizing.
//
// Within a scatter tile, a record's position in its destination is the
// tile's claim on that destination (one atomic per destination and tile on a
// cursor of its own 128-byte line) plus the record's rank among the tile's
// records for it (an LDS atomic). Record order inside a partition is
// therefore arbitrary; the aggregates are exact integer sums, minima and
// maxima, so they do not depend on it.

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

__device__ __forceinline__ uint64_t row_key(const PartParams& p, uint64_t r) {
  int64_t k[2] = {0, 0};
  for (int j = 0; j < p.g.kp.nkeys; ++j) {
    const int64_t i = p.key_idx[j] ? static_cast<int64_t>(p.key_idx[j][r]) : static_cast<int64_t>(r);
    k[j] = load_elem(p.key_data[j], p.g.kp.type[j], i);
  }
  return pack_keys(p.g.kp, k[0], k[1]);
}

__device__ __forceinline__ uint64_t row_col(const PartParams& p, int c, uint64_t r) {
  const int64_t i = p.col_idx[c] ? static_cast<int64_t>(p.col_idx[c][r]) : static_cast<int64_t>(r);
  return static_cast<uint64_t>(load_elem(p.col_data[c], p.col_type[c], i));
}

__device__ __forceinline__ uint32_t part_of(uint64_t pk, int pb) {
  return static_cast<uint32_t>(hash64(pk) >> (64 - pb));
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

__global__ void __launch_bounds__(256) part_count_kernel(PartParams p) {
  __shared__ uint32_t h[1 << kPartLevelBits];
  const int nb = 1 << p.b1;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t r = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
       r < static_cast<uint64_t>(p.n); r += stride)
    atomicAdd(&h[part_of(row_key(p, r), p.b1)], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    if (h[i]) atomicAdd(&p.ctl[kCtlHist1 + i], static_cast<unsigned long long>(h[i]));
}

// Bucket starts and cursors from the bucket counts (one workgroup of 256).
__global__ void __launch_bounds__(256) part_scan1_kernel(PartParams p) {
  const int nb = 1 << p.b1;
  const int b = threadIdx.x;
  const unsigned long long v = b < nb ? p.ctl[kCtlHist1 + b] : 0ULL;
  unsigned long long total;
  const unsigned long long excl = block_scan(v, &total);
  if (b < nb) {
    p.ctl[kCtlStart1 + b] = excl;
    p.ctl[kCtlCur1 + static_cast<uint64_t>(b) * kPartPad] = excl;
  }
  if (b == 0) p.ctl[kCtlStart1 + nb] = total;
}

__global__ void __launch_bounds__(kPartThreads) part_scatter1_kernel(PartParams p) {
  extern __shared__ uint64_t lds[];
  const GroupDesc& g = p.g;
  const int pb = p.b1 + p.b2;
  const uint32_t nparts = 1u << pb;
  const int nb = 1 << p.b1;
  uint64_t* pre = lds;
  uint32_t* h2 = reinterpret_cast<uint32_t*>(lds + static_cast<size_t>(p.pre_slots) * g.words);
  uint32_t* cnt = h2 + nparts;
  unsigned long long* base = reinterpret_cast<unsigned long long*>(cnt + (1 << kPartLevelBits));
  if (p.pre_slots > 0) lds_group_init(pre, p.pre_slots, g);
  for (uint32_t i = threadIdx.x; i < nparts; i += blockDim.x) h2[i] = 0;

  const uint64_t n = static_cast<uint64_t>(p.n);
  const uint64_t ntiles = (n + kPartTile - 1) / kPartTile;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    if (threadIdx.x < nb) cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t r0 = tile * kPartTile + threadIdx.x;
    uint64_t pk[kPartRows];
    uint32_t code[kPartRows];
#pragma unroll
    for (int e = 0; e < kPartRows; ++e) {
      const uint64_t r = r0 + static_cast<uint64_t>(e) * kPartThreads;
      pk[e] = r < n ? row_key(p, r) : 0;
    }
#pragma unroll
    for (int e = 0; e < kPartRows; ++e) {
      const uint64_t r = r0 + static_cast<uint64_t>(e) * kPartThreads;
      code[e] = kNoRecord;
      if (r >= n) continue;
      const int32_t s = lds_group_find(pre, p.pre_slots, g.words, pk[e], kPreProbe);
      if (s >= 0) {
        uint64_t acc[kMaxAcc];
#pragma unroll
        for (int a = 0; a < kMaxAcc; ++a)
          if (a < g.ap.nacc) acc[a] = row_col(p, p.src[a], r);
        lds_group_update(pre + static_cast<size_t>(s) * g.words, g.ap, acc);
      } else {
        const uint32_t q = part_of(pk[e], pb);
        const uint32_t b = q >> p.b2;
        const uint32_t rank = atomicAdd(&cnt[b], 1u);
        atomicAdd(&h2[q], 1u);
        code[e] = (b << 16) | rank;
      }
    }
    __syncthreads();
    if (threadIdx.x < nb && cnt[threadIdx.x])
      base[threadIdx.x] = atomicAdd(&p.ctl[kCtlCur1 + static_cast<uint64_t>(threadIdx.x) * kPartPad],
                                    static_cast<unsigned long long>(cnt[threadIdx.x]));
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kPartRows; ++e) {
      if (code[e] == kNoRecord) continue;
      const uint64_t r = r0 + static_cast<uint64_t>(e) * kPartThreads;
      const uint64_t pos = base[code[e] >> 16] + (code[e] & 0xFFFFu);
      uint64_t* w = p.rec_a + pos * p.rw;
      w[0] = pk[e];
      for (int c = 0; c < p.ncols; ++c) w[1 + c] = row_col(p, c, r);
    }
  }
  __syncthreads();
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
  const int nb = 1 << p.b1;
  const int b = threadIdx.x;
  unsigned long long tiles = 0;
  if (b < nb) {
    const unsigned long long filled =
        p.ctl[kCtlCur1 + static_cast<uint64_t>(b) * kPartPad] - p.ctl[kCtlStart1 + b];
    tiles = (filled + kPartTile - 1) / kPartTile;
  }
  unsigned long long total_tiles;
  const unsigned long long texcl = block_scan(tiles, &total_tiles);
  if (b < nb) p.ctl[kCtlTiles + b] = texcl;
  if (b == 0) p.ctl[kCtlTiles + nb] = total_tiles;
}

// kPair: records of two words (one value column), held in registers between
// the counting and the writing half of a tile; wider records are read again
// (from L2) when written.
template <bool kPair>
__global__ void __launch_bounds__(kPartThreads) part_scatter2_kernel(PartParams p) {
  __shared__ unsigned long long s_tiles[(1 << kPartLevelBits) + 1];
  __shared__ unsigned long long s_start[1 << kPartLevelBits];
  __shared__ unsigned long long s_end[1 << kPartLevelBits];
  __shared__ uint32_t cnt[1 << kPartLevelBits];
  __shared__ unsigned long long base[1 << kPartLevelBits];
  const int nb = 1 << p.b1;
  const int n2 = 1 << p.b2;
  const int pb = p.b1 + p.b2;
  for (int b = threadIdx.x; b <= nb; b += blockDim.x) s_tiles[b] = p.ctl[kCtlTiles + b];
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    s_start[b] = p.ctl[kCtlStart1 + b];
    s_end[b] = p.ctl[kCtlCur1 + static_cast<uint64_t>(b) * kPartPad];
  }
  __syncthreads();
  const unsigned long long ntiles = s_tiles[nb];
  for (unsigned long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    // bucket b: the last with s_tiles[b] <= t
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (s_tiles[mid] <= t) lo = mid;
      else hi = mid;
    }
    const int b = lo;
    const uint64_t first = s_start[b] + (t - s_tiles[b]) * kPartTile;
    const uint64_t end = s_end[b];
    if (threadIdx.x < n2) cnt[threadIdx.x] = 0;
    __syncthreads();
    uint64_t pk[kPartRows], val[kPair ? kPartRows : 1];
    uint32_t code[kPartRows];
#pragma unroll
    for (int e = 0; e < kPartRows; ++e) {
      const uint64_t i = first + threadIdx.x + static_cast<uint64_t>(e) * kPartThreads;
      if (i < end) {
        if constexpr (kPair) {
          const ulonglong2 r = *reinterpret_cast<const ulonglong2*>(p.rec_a + 2 * i);
          pk[e] = r.x;
          val[e] = r.y;
        } else {
          pk[e] = p.rec_a[i * p.rw];
        }
      }
    }
#pragma unroll
    for (int e = 0; e < kPartRows; ++e) {
      const uint64_t i = first + threadIdx.x + static_cast<uint64_t>(e) * kPartThreads;
      code[e] = kNoRecord;
      if (i >= end) continue;
      const uint32_t j = part_of(pk[e], pb) & static_cast<uint32_t>(n2 - 1);
      code[e] = (j << 16) | atomicAdd(&cnt[j], 1u);
    }
    __syncthreads();
    if (threadIdx.x < n2 && cnt[threadIdx.x]) {
      const uint64_t q = (static_cast<uint64_t>(b) << p.b2) + threadIdx.x;
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
        const uint64_t i = i0 + static_cast<uint64_t>(e) * blockDim.x;
        if (i >= end) continue;
        const uint64_t* rec = p.rec_b + i * p.rw;
        pk[e] = rec[0];
#pragma unroll
        for (int a = 0; a < kMaxAcc; ++a)
          if (a < g.ap.nacc) acc[e][a] = rec[1 + p.src[a]];
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

template <typename K>
hipError_t allow_dynamic_lds(K k) {
  static int done = 0;
  if (done) return hipSuccess;
  hipFuncAttributes attr;
  hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(k));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          device_info().lds_per_block - static_cast<int>(attr.sharedSizeBytes));
  if (e == hipSuccess) done = 1;
  return e;
}

}  // namespace

size_t part_scatter1_lds(const PartParams& p) {
  return static_cast<size_t>(p.pre_slots) * p.g.words * 8 + (sizeof(uint32_t) << (p.b1 + p.b2)) +
         (sizeof(uint32_t) + sizeof(unsigned long long)) * (1u << kPartLevelBits);
}

hipError_t launch_group_partitioned(const PartParams& p, hipStream_t s) {
  const int cus = device_info().cu_count;
  hipError_t e = allow_dynamic_lds(part_scatter1_kernel);
  if (e != hipSuccess) return e;
  e = allow_dynamic_lds(part_agg_kernel);
  if (e != hipSuccess) return e;
  {
    ProfileScope ps(kKGroupPartition, s);
    hipLaunchKernelGGL(part_count_kernel, dim3(cus * 8), dim3(256), 0, s, p);
    hipLaunchKernelGGL(part_scan1_kernel, dim3(1), dim3(256), 0, s, p);
    hipLaunchKernelGGL(part_scatter1_kernel, dim3(cus * 2), dim3(kPartThreads),
                       part_scatter1_lds(p), s, p);
    hipLaunchKernelGGL(part_scan2_kernel, dim3(1), dim3(1024), 0, s, p);
    if (p.rw == 2)
      hipLaunchKernelGGL(part_scatter2_kernel<true>, dim3(cus * 2), dim3(kPartThreads), 0, s, p);
    else
      hipLaunchKernelGGL(part_scatter2_kernel<false>, dim3(cus * 2), dim3(kPartThreads), 0, s, p);
  }
  ProfileScope ps(kKGroupAgg, s);
  hipLaunchKernelGGL(part_agg_kernel, dim3(cus), dim3(kPartAggThreads),
                     static_cast<size_t>(p.agg_slots) * p.g.words * 8, s, p);
  return hipGetLastError();
}

}  // namespace rel
