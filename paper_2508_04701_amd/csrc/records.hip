// Record passes of batched plans whose groups outgrow the fused pass's LDS
// table (hash grouping, Section 4.2, with the table far larger than a
// workgroup's LDS). The fused pass has written each spilled row as a record
// (packed key, then the early value columns) into its item's run and counted
// it per partition; see RecDesc. Then, for every plan with records:
//
//   scan      one workgroup per plan: the partitions' record totals (which
//             the fused pass summed, one atomic per item and partition)
//             become their places in partition-major order, and each
//             aggregation partition (a run of consecutive partitions whose
//             keys fit one LDS table) is cut into pieces of at most
//             kRecPiece records, appended to the batch's piece list (one
//             atomic per plan);
//   scatter   one workgroup per fused-pass item: the item reserves its share
//             of each partition with one atomic on the partition's cursor
//             and its records go there, sorted by
//             partition in LDS a chunk at a time so that each partition's
//             share of a chunk is written by consecutive lanes (order within
//             a partition is arbitrary);
//   aggregate persistent workgroups take pieces in order from a device
//             counter and fold each into an LDS table sized for a
//             partition's keys, which then merges into the plan's global
//             group table with one update per key. A key that finds no LDS
//             slot updates the global table directly, so results never
//             depend on the sizing.
//
// The aggregates are exact integer sums, minima and maxima, so the record
// order does not change the results.

#include <type_traits>

#include "pipeline_kernel.h"

namespace rel {

namespace {

constexpr int kRecScanThreads = 1024;
constexpr int kRecScatterThreads = 256;
constexpr int kRecAggThreads = 512;
constexpr int kRecProbe = 32;  // LDS probe window of the aggregation table
// Records the scatter sorts in LDS at a time: each partition's share of a
// chunk is one contiguous store run (on the 256-instance batch: 1024 records
// 7.7 ms of record passes, 2048 7.2, 4096 6.7, 8192 6.7).
constexpr uint32_t kScatterChunk = 4096;
static_assert(kMaxRecParts <= 65536, "partition numbers fit 16 bits");
constexpr int kRecUnroll = 4;  // records per thread and step of the aggregation

typedef uint64_t v2u64 __attribute__((ext_vector_type(2)));

// acc_code of a plan whose one accumulator is a SUM of the first value word
constexpr uint32_t kSumOfFirst = 1u + static_cast<uint32_t>(kAccSum);

// Exclusive prefix sum of v over the workgroup (blockDim.x a multiple of the
// wave size); `total` receives the sum. s_wave holds one word per wave. All
// threads must call it.
__device__ uint32_t block_exclusive(uint32_t v, uint32_t* s_wave, uint32_t& total) {
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += t;
  }
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  uint32_t before = 0;
  total = 0;
  for (int w = 0; w < nwaves; ++w) {
    const uint32_t x = s_wave[w];
    if (w < wave) before += x;
    total += x;
  }
  __syncthreads();
  return before + incl - v;
}

__global__ void __launch_bounds__(kRecScanThreads) rec_scan_kernel(BatchParams b) {
  __shared__ uint32_t s_wave[kRecScanThreads / kWave];
  __shared__ uint32_t s_base;
  const PipelineParams& p = batch_at(b.plans, blockIdx.x);
  const uint32_t parts = p.rec.parts;
  if (parts == 0) return;
  uint32_t* pb = p.rec.part_begin;
  // the partitions' places: an exclusive prefix sum of their totals, each
  // also the partition's first free place (parts <= blockDim.x)
  const uint32_t c = threadIdx.x < parts ? p.rec.cursor[threadIdx.x] : 0u;
  uint32_t total = 0;
  const uint32_t at = block_exclusive(c, s_wave, total);
  if (threadIdx.x < parts) {
    pb[threadIdx.x] = at;
    p.rec.cursor[threadIdx.x] = at;
  }
  if (threadIdx.x == 0) pb[parts] = total;
  __syncthreads();
  // pieces of kRecPiece records, aggregation partition by aggregation
  // partition (agg_parts <= parts <= blockDim.x)
  const uint32_t q = threadIdx.x;
  const uint32_t agg_parts = p.rec.agg_parts;
  const uint32_t run_parts = parts / agg_parts;
  uint32_t np = 0, qb = 0, qe = 0;
  if (q < agg_parts) {
    qb = pb[q * run_parts];
    qe = pb[(q + 1) * run_parts];
    np = (qe - qb + kRecPiece - 1) / kRecPiece;
  }
  uint32_t pieces = 0;
  const uint32_t before = block_exclusive(np, s_wave, pieces);
  if (threadIdx.x == 0)
    s_base = pieces ? static_cast<uint32_t>(atomicAdd(b.npieces, static_cast<unsigned long long>(pieces)))
                    : 0u;
  __syncthreads();
  for (uint32_t k = 0; k < np; ++k) {
    RecPiece pc;
    pc.inst = blockIdx.x;
    pc.part = q;
    pc.begin = qb + k * kRecPiece;
    pc.end = qe - pc.begin > kRecPiece ? pc.begin + kRecPiece : qe;
    b.pieces[s_base + before + k] = pc;
  }
}

// Record forms the scatter moves: narrow (32-bit key and value word in two
// arrays) and two-word (key and value word side by side).
struct NarrowRecs {
  static constexpr uint32_t kChunk = kScatterChunk;
  uint32_t k;
  uint64_t v;
};
struct WideRecs {
  static constexpr uint32_t kChunk = kScatterChunk * 3 / 4;  // 16 bytes a record
  v2u64 x;
};

// LDS of the scatter: the staged chunk (48 KB: narrow keys then values, or
// two-word records), each staged record's partition, the partitions' running
// places and a chunk's histogram, offsets and write bases.
struct ScatterLds {
  uint64_t stage[kScatterChunk * 3 / 2];
  uint16_t part[kScatterChunk];
  uint32_t cur[kMaxRecParts];
  uint32_t cnt[kMaxRecParts];
  uint32_t wave[kRecScatterThreads / kWave];
};

// Records [0, n) of one item run (src), scattered to their partitions' places
// (dst) a chunk at a time: a histogram over the chunk, its offsets, the
// records placed in LDS in partition order, then written out in that order so
// that each partition's share of the chunk is stored by consecutive lanes.
// Each thread owns partitions [tid * per, tid * per + per) of the offsets.
template <typename R>
__device__ __forceinline__ void scatter_chunks(ScatterLds& L, const RecDesc& rd, uint64_t run,
                                               uint32_t n) {
  constexpr uint32_t kC = R::kChunk;
  constexpr int kPer = kC / kRecScatterThreads;
  static_assert(kC % kRecScatterThreads == 0, "whole records per thread");
  const uint32_t parts = rd.parts;
  const uint32_t narrow = rd.narrow;
  const uint32_t per = (parts + kRecScatterThreads - 1) / kRecScatterThreads;
  constexpr uint32_t kMaxPer = (kMaxRecParts + kRecScatterThreads - 1) / kRecScatterThreads;
  const uint32_t q_lo = threadIdx.x * per;
  uint32_t* stage_k = reinterpret_cast<uint32_t*>(L.stage);
  uint64_t* stage_v = L.stage + kC / 2;
  v2u64* stage_x = reinterpret_cast<v2u64*>(L.stage);
  for (uint32_t c0 = 0; c0 < n; c0 += kC) {
    const uint32_t m = n - c0 < kC ? n - c0 : kC;
    for (uint32_t q = threadIdx.x; q < parts; q += blockDim.x) L.cnt[q] = 0;
    R x[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const uint32_t i = u * blockDim.x + threadIdx.x;
      if (i < m) {
        if constexpr (std::is_same_v<R, NarrowRecs>) {
          x[u].k = __builtin_nontemporal_load(rd.rkeys + run + c0 + i);
          x[u].v = __builtin_nontemporal_load(rd.recs + run + c0 + i);
        } else {
          x[u].x = __builtin_nontemporal_load(reinterpret_cast<const v2u64*>(rd.recs) + run + c0 + i);
        }
      }
    }
    __syncthreads();
    uint32_t qq[kPer], rank[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const uint32_t i = u * blockDim.x + threadIdx.x;
      if (i < m) {
        uint64_t pk;
        if constexpr (std::is_same_v<R, NarrowRecs>) pk = narrow_key(x[u].k, narrow);
        else pk = x[u].x.x;
        qq[u] = rec_part(pk, parts);
        rank[u] = lds_fetch_add_u32(L.cnt + qq[u], 1u);
      }
    }
    __syncthreads();
    // offsets over the partitions, and each partition's write base
    uint32_t c[kMaxPer], sum = 0;
#pragma unroll
    for (uint32_t e = 0; e < kMaxPer; ++e) {
      const uint32_t q = q_lo + e;
      c[e] = (e < per && q < parts) ? L.cnt[q] : 0u;
      sum += c[e];
    }
    uint32_t total = 0;
    uint32_t off = block_exclusive(sum, L.wave, total);
    uint32_t base[kMaxPer];
#pragma unroll
    for (uint32_t e = 0; e < kMaxPer; ++e) {
      const uint32_t q = q_lo + e;
      base[e] = 0;
      if (e < per && q < parts) {
        const uint32_t at = L.cur[q];
        L.cur[q] = at + c[e];
        base[e] = at - off;  // modulo 2^32: at + (s - off) for s >= off
        L.cnt[q] = off;
        off += c[e];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const uint32_t i = u * blockDim.x + threadIdx.x;
      if (i < m) {
        const uint32_t at = L.cnt[qq[u]] + rank[u];
        if constexpr (std::is_same_v<R, NarrowRecs>) {
          stage_k[at] = x[u].k;
          stage_v[at] = x[u].v;
        } else {
          stage_x[at] = x[u].x;
        }
        L.part[at] = static_cast<uint16_t>(qq[u]);
      }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t e = 0; e < kMaxPer; ++e) {
      const uint32_t q = q_lo + e;
      if (e < per && q < parts) L.cnt[q] = base[e];
    }
    __syncthreads();
    // plain stores: a partition's run fills its lines from several chunks,
    // which L2 merges before they reach HBM
    for (uint32_t s2 = threadIdx.x; s2 < m; s2 += blockDim.x) {
      const uint32_t at = L.cnt[L.part[s2]] + s2;
      if constexpr (std::is_same_v<R, NarrowRecs>) {
        rd.pkeys[at] = stage_k[s2];
        rd.parted[at] = stage_v[s2];
      } else {
        reinterpret_cast<v2u64*>(rd.parted)[at] = stage_x[s2];
      }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kRecScatterThreads) rec_scatter_kernel(BatchParams b) {
  __shared__ __attribute__((aligned(16))) ScatterLds L;
  const BatchItem& it = batch_at(b.tile_items, blockIdx.x);
  const PipelineParams& p = batch_at(b.plans, it.inst);
  const uint32_t parts = p.rec.parts;
  if (parts == 0) return;
  const uint32_t j = static_cast<uint32_t>(it.begin / p.rec.item_tiles);
  const uint32_t n = p.rec.item_n[j];
  if (n == 0) return;
  // the item's place in each partition: one atomic on the partition's
  // cursor per partition the item has records of
  const uint32_t* row = p.rec.counts + static_cast<uint64_t>(j) * parts;
  for (uint32_t q = threadIdx.x; q < parts; q += blockDim.x) {
    const uint32_t c = row[q];
    L.cur[q] = c ? atomicAdd(p.rec.cursor + q, c) : 0u;
  }
  __syncthreads();
  const uint32_t words = p.rec.words;
  const uint64_t run = static_cast<uint64_t>(j) * p.rec.item_tiles * kPipeTile;
  if (p.rec.narrow) {
    scatter_chunks<NarrowRecs>(L, p.rec, run, n);
  } else if (words == 2) {
    scatter_chunks<WideRecs>(L, p.rec, run, n);
  } else {
    const uint64_t* src = p.rec.recs + run * words;
    uint64_t* dst = p.rec.parted;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint64_t* x = src + static_cast<uint64_t>(i) * words;
      const uint64_t pk = x[0];
      const uint32_t at = lds_fetch_add_u32(L.cur + rec_part(pk, parts), 1u);
      uint64_t* y = dst + static_cast<uint64_t>(at) * words;
      y[0] = pk;
      for (uint32_t w = 1; w < words; ++w) y[w] = x[w];
    }
  }
}

// One record of plan p: COUNT plus each accumulator (value source 0: the
// record's first value word, 1: its second).
__device__ __forceinline__ void rec_update(const PipelineParams& p, uint64_t pk, int64_t va,
                                           int64_t vb, uint64_t* lt, int slots, int words,
                                           const GroupTable& gt, uint32_t acode) {
  const int32_t li = lds_group_find(lt, slots, words, pk, kRecProbe);
  if (li >= 0) {
    uint64_t* s = lt + li * words;
    lds_add_u64(s + 1, 1);
    if (acode == kSumOfFirst) {
      lds_add_u64(s + 2, static_cast<uint64_t>(va));
      return;
    }
    int a = 0;
    for (uint32_t code = acode; code != 0; code >>= 4, ++a) {
      const uint32_t c = (code & 15u) - 1u;
      lds_acc_update(s + 2 + a, static_cast<int>(c & 3u), (c >> 2) == 0 ? va : vb);
    }
    return;
  }
  uint64_t* gs = group_slot(gt, pk);
  if (!gs) return;
  global_add_u64(gs + 1, 1);
  int a = 0;
  for (uint32_t code = acode; code != 0; code >>= 4, ++a) {
    const uint32_t c = (code & 15u) - 1u;
    const int64_t v = (c >> 2) == 0 ? va : vb;
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

__global__ void __launch_bounds__(kRecAggThreads) rec_agg_kernel(BatchParams b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ uint32_t s_item;
  uint64_t* lt = reinterpret_cast<uint64_t*>(lds);
  const unsigned long long total = *b.npieces;
  for (;;) {
    if (threadIdx.x == 0) s_item = static_cast<uint32_t>(atomicAdd(b.agg_counter, 1ULL));
    __syncthreads();
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
    if (item >= total) return;
    const RecPiece pc = b.pieces[item];
    const PipelineParams& p = batch_at(b.plans, pc.inst);
    const int slots = static_cast<int>(p.rec.agg_slots);
    const int words = p.g.words;
    lds_group_init(lt, slots, p.g);
    __syncthreads();
    const uint32_t acode = pipe::acc_code(p);
    const GroupTable gt = group_replica(p.g, blockIdx.x % p.g.replicas);
    const uint32_t rw = p.rec.words;
    if (p.rec.narrow) {
      // the next step's records are loaded while this step's are folded
      const uint32_t narrow = p.rec.narrow;
      const uint32_t* ks = p.rec.pkeys;
      const uint64_t* vs = p.rec.parted;
      const uint32_t step = kRecUnroll * blockDim.x;
      uint32_t xk[kRecUnroll], yk[kRecUnroll];
      uint64_t xv[kRecUnroll], yv[kRecUnroll];
      uint32_t i0 = pc.begin + threadIdx.x;
#pragma unroll
      for (int u = 0; u < kRecUnroll; ++u) {
        const uint32_t i = i0 + u * blockDim.x;
        if (i < pc.end) {
          xk[u] = __builtin_nontemporal_load(ks + i);
          xv[u] = __builtin_nontemporal_load(vs + i);
        }
      }
      for (; i0 < pc.end; i0 += step) {
        const uint32_t i1 = i0 + step;
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u) {
          const uint32_t i = i1 + u * blockDim.x;
          if (i < pc.end) {
            yk[u] = __builtin_nontemporal_load(ks + i);
            yv[u] = __builtin_nontemporal_load(vs + i);
          }
        }
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u)
          if (i0 + u * blockDim.x < pc.end)
            rec_update(p, narrow_key(xk[u], narrow), static_cast<int64_t>(xv[u]), 0, lt, slots,
                       words, gt, acode);
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u) {
          xk[u] = yk[u];
          xv[u] = yv[u];
        }
      }
    } else if (rw == 2) {
      // the next step's records are loaded while this step's are folded
      const v2u64* src = reinterpret_cast<const v2u64*>(p.rec.parted);
      const uint32_t step = kRecUnroll * blockDim.x;
      v2u64 x[kRecUnroll], y[kRecUnroll];
      uint32_t i0 = pc.begin + threadIdx.x;
#pragma unroll
      for (int u = 0; u < kRecUnroll; ++u)
        if (i0 + u * blockDim.x < pc.end) x[u] = __builtin_nontemporal_load(src + i0 + u * blockDim.x);
      for (; i0 < pc.end; i0 += step) {
        const uint32_t i1 = i0 + step;
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u)
          if (i1 + u * blockDim.x < pc.end) y[u] = __builtin_nontemporal_load(src + i1 + u * blockDim.x);
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u)
          if (i0 + u * blockDim.x < pc.end)
            rec_update(p, x[u].x, static_cast<int64_t>(x[u].y), 0, lt, slots, words, gt, acode);
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u) x[u] = y[u];
      }
    } else {
      for (uint32_t i = pc.begin + threadIdx.x; i < pc.end; i += blockDim.x) {
        const uint64_t* x = p.rec.parted + static_cast<uint64_t>(i) * rw;
        const int64_t va = rw > 1 ? static_cast<int64_t>(x[1]) : 0;
        const int64_t vb = rw > 2 ? static_cast<int64_t>(x[2]) : 0;
        rec_update(p, x[0], va, vb, lt, slots, words, gt, acode);
      }
    }
    __syncthreads();
    lds_group_flush(lt, slots, p.g);
    __syncthreads();
  }
}

}  // namespace

void launch_batch_records(const BatchParams& b, hipStream_t s) {
  if (b.rec_plans == 0) return;
  ProfileScope ps(kKGroupAgg, s);
  hipLaunchKernelGGL(rec_scan_kernel, dim3(b.nplans), dim3(kRecScanThreads), 0, s, b);
  hipLaunchKernelGGL(rec_scatter_kernel, dim3(b.ntile_all), dim3(kRecScatterThreads), 0, s, b);
  // persistent aggregation grid: as many workgroups as fit the CUs at the
  // largest LDS table (kRecAggLds), at most one per possible piece
  static const int per_cu = [] {
    int k = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, rec_agg_kernel, kRecAggThreads,
                                                     kRecAggLds) != hipSuccess || k < 1)
      k = 1;
    return k;
  }();
  uint64_t grid = static_cast<uint64_t>(device_info().cu_count) * per_cu;
  if (grid > b.piece_cap) grid = b.piece_cap;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(rec_agg_kernel, dim3(static_cast<unsigned>(grid)), dim3(kRecAggThreads),
                     b.agg_lds_bytes, s, b);
}

}  // namespace rel
