// Hash join: open-addressing multimap build and probe with pair output.
//
// Build: each element claims the first empty slot of its linear-probe chain
// with one CAS (int32 keys publish key and value in the same 64-bit word);
// each lane keeps four elements' loads and CAS in flight. Large build sides
// take the partitioned build instead (partition.hip).
// Probe: each lane walks the chains of four probe keys, one slot per key and
// round; a round's matches are ranked within the wave (ballot, mbcnt) and
// staged in LDS, and a wave writes its staged pairs in runs, with one atomic
// add per run on the global cursor. The cursor always ends at the exact pair
// count; pairs beyond the output capacity are counted but not written.

#include "internal.h"

namespace rel {

namespace {

__global__ void fill64_kernel(uint64_t* p, uint64_t n, uint64_t pattern) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = pattern;
}

__global__ void fill_map64_kernel(ulonglong2* p, uint64_t n) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = make_ulonglong2(kEmpty64, 0ULL);
}

__device__ __forceinline__ uint32_t element_value(const MapBuildParams& p, int64_t i) {
  if (p.val_col) {
    int64_t r = p.idx ? static_cast<int64_t>(p.idx[i]) : i;
    return static_cast<uint32_t>(load_elem(p.val_col, p.val_type, r));
  }
  return p.idx ? p.idx[i] : static_cast<uint32_t>(i);
}

// Inserts elements i, i + stride, ... below `end` of build p.
template <typename K>
__device__ __forceinline__ void build_rows(const MapBuildParams& p, uint64_t i, uint64_t end,
                                           uint64_t stride) {
  for (; i < end; i += stride) {
    int64_t r = p.idx ? static_cast<int64_t>(p.idx[i]) : static_cast<int64_t>(i);
    K key = static_cast<K>(load_elem(p.keys, p.type, r));
    if constexpr (sizeof(K) == 4) {
      if (p.map.compact) {
        CsetDesc c{static_cast<uint32_t*>(p.map.slots), p.map.cap - 1, p.map.rbits, p.map.dup,
                   p.map.over, p.map.over_cap - 1, p.map.oob_count};
        cset_insert(c, key);
        continue;
      }
      if (p.map.key_only) {
        set_insert(static_cast<uint32_t*>(p.map.slots), p.map.cap - 1, p.map.oob_count, key,
                   p.map.dup);
        continue;
      }
    }
    uint32_t val = element_value(p, static_cast<int64_t>(i));
    if constexpr (sizeof(K) == 4) {
      Map32 m{static_cast<uint64_t*>(p.map.slots), p.map.cap - 1, p.map.oob_count, p.map.oob_vals};
      map_insert(m, key, val, p.map.dup);
    } else {
      Map64 m{static_cast<ulonglong2*>(p.map.slots), p.map.cap - 1, p.map.oob_count, p.map.oob_vals};
      map_insert(m, key, val, p.map.dup);
    }
  }
}

// Elements at[e] of a column; the type test is outside the element loop, so
// the N loads issue back to back.
template <int N>
__device__ __forceinline__ void gather_elems(const void* data, int32_t type, const uint64_t* at,
                                             int64_t* out) {
  if (type == kI64) {
#pragma unroll
    for (int e = 0; e < N; ++e) out[e] = static_cast<const int64_t*>(data)[at[e]];
  } else if (type == kI32) {
#pragma unroll
    for (int e = 0; e < N; ++e) out[e] = static_cast<const int32_t*>(data)[at[e]];
  } else {
#pragma unroll
    for (int e = 0; e < N; ++e) out[e] = static_cast<const int8_t*>(data)[at[e]];
  }
}

// Keys per lane and step of the batched map build.
constexpr int kBuildKeys = 4;

// Map (key -> value) inserts of elements i, i + stride, ... below `end`,
// kBuildKeys per lane at a time: their loads, and each round's CAS on the
// slot arrays, are independent and in flight together. Same slots, same
// duplicate detection and out-of-band handling as map_insert.
template <typename K>
__device__ __forceinline__ void build_map_batched(const MapBuildParams& p, uint64_t i0, uint64_t end,
                                                  uint64_t stride) {
  constexpr int J = kBuildKeys;
  const uint64_t mask = p.map.cap - 1;
  for (; i0 < end; i0 += J * stride) {
    uint64_t at[J];
    bool pend[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const uint64_t i = i0 + static_cast<uint64_t>(j) * stride;
      pend[j] = i < end;
      at[j] = pend[j] ? i : i0;
    }
    uint32_t val[J];
    if (p.idx) {
#pragma unroll
      for (int j = 0; j < J; ++j) at[j] = p.idx[at[j]];
    }
    int64_t kv[J];
    gather_elems<J>(p.keys, p.type, at, kv);
    if (p.val_col) {
      int64_t pv[J];
      gather_elems<J>(p.val_col, p.val_type, at, pv);
#pragma unroll
      for (int j = 0; j < J; ++j) val[j] = static_cast<uint32_t>(pv[j]);
    } else {
#pragma unroll
      for (int j = 0; j < J; ++j) val[j] = static_cast<uint32_t>(at[j]);
    }
    K key[J];
    uint64_t h[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      key[j] = static_cast<K>(kv[j]);
      h[j] = 0;
      if (!pend[j]) continue;
      if constexpr (sizeof(K) == 4) {
        if (key[j] == kEmpty32) {
          map_insert(Map32{nullptr, mask, p.map.oob_count, p.map.oob_vals}, key[j], val[j], p.map.dup);
          pend[j] = false;
        } else {
          h[j] = home32(key[j], mask);
        }
      } else {
        if (static_cast<uint64_t>(key[j]) == kEmpty64) {
          map_insert(Map64{nullptr, mask, p.map.oob_count, p.map.oob_vals}, key[j], val[j], p.map.dup);
          pend[j] = false;
        } else {
          h[j] = home64(key[j], mask);
        }
      }
    }
    while (true) {
      bool any = false;
#pragma unroll
      for (int j = 0; j < J; ++j) any |= pend[j];
      if (!any) break;
      unsigned long long prev[J];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        prev[j] = 0;
        if (!pend[j]) continue;
        if constexpr (sizeof(K) == 4) {
          prev[j] = atomicCAS(static_cast<unsigned long long*>(p.map.slots) + h[j],
                              static_cast<unsigned long long>(kEmptySlot32),
                              static_cast<unsigned long long>(pack32(key[j], val[j])));
        } else {
          prev[j] = atomicCAS(reinterpret_cast<unsigned long long*>(
                                  &static_cast<ulonglong2*>(p.map.slots)[h[j]].x),
                              static_cast<unsigned long long>(kEmpty64),
                              static_cast<unsigned long long>(key[j]));
        }
      }
#pragma unroll
      for (int j = 0; j < J; ++j) {
        if (!pend[j]) continue;
        if constexpr (sizeof(K) == 4) {
          if (prev[j] == kEmptySlot32) {
            pend[j] = false;
            continue;
          }
          if (static_cast<int32_t>(static_cast<uint32_t>(prev[j])) == key[j]) *p.map.dup = 1;
        } else {
          if (prev[j] == kEmpty64) {
            static_cast<ulonglong2*>(p.map.slots)[h[j]].y = val[j];
            pend[j] = false;
            continue;
          }
          if (static_cast<int64_t>(prev[j]) == key[j]) *p.map.dup = 1;
        }
        h[j] = (h[j] + 1) & mask;
      }
    }
  }
}

__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
  return v;
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
  return v;
}

// Build pass 1 over elements i, i + stride, ... (the workgroup's loop bound
// is uniform): key and payload ranges, reduced per wave, then one atomic
// per wave and bound.
__device__ __forceinline__ void range_rows(const MapBuildParams& p, uint64_t base, uint64_t end,
                                           uint64_t stride) {
  if (p.map.direct_cap == 0) return;
  // each lane folds its rows in registers (four loads in flight per step);
  // the wave then reduces once and publishes with at most four atomics
  int32_t kmin = INT32_MAX, kmax = INT32_MIN, pmin = INT32_MAX, pmax = INT32_MIN;
  const bool pay = p.val_col != nullptr;
  auto row = [&](uint64_t i) {
    return p.idx ? static_cast<int64_t>(p.idx[i]) : static_cast<int64_t>(i);
  };
  uint64_t i = base + threadIdx.x;
  for (; i + 3 * stride < end; i += 4 * stride) {
    int32_t k[4], v[4] = {0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < 4; ++u) k[u] = static_cast<int32_t>(load_elem(p.keys, p.type, row(i + u * stride)));
    if (pay) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        v[u] = static_cast<int32_t>(load_elem(p.val_col, p.val_type, row(i + u * stride)));
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      kmin = k[u] < kmin ? k[u] : kmin;
      kmax = k[u] > kmax ? k[u] : kmax;
      if (pay) {
        pmin = v[u] < pmin ? v[u] : pmin;
        pmax = v[u] > pmax ? v[u] : pmax;
      }
    }
  }
  for (; i < end; i += stride) {
    const int32_t k = static_cast<int32_t>(load_elem(p.keys, p.type, row(i)));
    kmin = k < kmin ? k : kmin;
    kmax = k > kmax ? k : kmax;
    if (pay) {
      const int32_t v = static_cast<int32_t>(load_elem(p.val_col, p.val_type, row(i)));
      pmin = v < pmin ? v : pmin;
      pmax = v > pmax ? v : pmax;
    }
  }
  kmin = wave_min_i32(kmin);
  kmax = wave_max_i32(kmax);
  if (pay) {
    pmin = wave_min_i32(pmin);
    pmax = wave_max_i32(pmax);
  }
  if (lane_id() == 0 && kmin <= kmax) {
    int32_t* st = p.map.dstate;
    if (kmin < st[kDKmin]) atomicMin(st + kDKmin, kmin);
    if (kmax > st[kDKmax]) atomicMax(st + kDKmax, kmax);
    if (pay) {
      if (pmin < st[kDPmin]) atomicMin(st + kDPmin, pmin);
      if (pmax > st[kDPmax]) atomicMax(st + kDPmax, pmax);
    }
  }
}

// Build pass 2: when the key range fits, set each key's presence bit and
// store its narrowed payload; a bit already set means a duplicate key.
__device__ __forceinline__ void direct_rows(const MapBuildParams& p, uint64_t i, uint64_t end,
                                            uint64_t stride) {
  const MapDesc& m = p.map;
  if (m.direct_cap == 0) return;
  const uint64_t range = direct_range(m);
  if (range == 0 || range > m.direct_cap) return;
  const int32_t kmin = m.dstate[kDKmin];
  const int32_t pmin = m.dstate[kDPmin];
  const int width = p.val_col ? direct_width(pmin, m.dstate[kDPmax]) : 0;
  // kBuildKeys elements per lane and step: their loads, and their bitmap
  // atomics, are in flight together
  constexpr int J = kBuildKeys;
  for (; i < end; i += J * stride) {
    uint64_t at[J];
    bool ok[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const uint64_t e = i + static_cast<uint64_t>(j) * stride;
      ok[j] = e < end;
      at[j] = ok[j] ? e : i;
    }
    if (p.idx) {
#pragma unroll
      for (int j = 0; j < J; ++j) at[j] = p.idx[at[j]];
    }
    int64_t kv[J], pv[J];
    gather_elems<J>(p.keys, p.type, at, kv);
    if (width) gather_elems<J>(p.val_col, p.val_type, at, pv);
    uint32_t k[J], old[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      k[j] = static_cast<uint32_t>(kv[j] - kmin);
      old[j] = ok[j] ? atomicOr(m.dbits + (k[j] >> 5), 1u << (k[j] & 31)) : 0u;
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (!ok[j]) continue;
      if (old[j] & (1u << (k[j] & 31))) {
        *m.dup = 1;
        continue;
      }
      if (width == 0) continue;
      const uint32_t v = static_cast<uint32_t>(pv[j]) - static_cast<uint32_t>(pmin);
      if (width == 1) static_cast<uint8_t*>(m.dvals)[k[j]] = static_cast<uint8_t>(v);
      else if (width == 2) static_cast<uint16_t*>(m.dvals)[k[j]] = static_cast<uint16_t>(v);
      else static_cast<uint32_t*>(m.dvals)[k[j]] = v;
    }
  }
}

// Build pass 3 (the slot array) is skipped when the direct table took every
// key exactly once.
__device__ __forceinline__ bool slots_needed(const MapDesc& m) { return direct_view(m).mode == 0; }

template <typename K>
__global__ void __launch_bounds__(256) map_build_kernel(MapBuildParams p, int pass) {
  const uint64_t first = blockIdx.x * static_cast<uint64_t>(blockDim.x);
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  if (pass == 0) {
    range_rows(p, first, static_cast<uint64_t>(p.n), stride);
  } else if (pass == 1) {
    direct_rows(p, first + threadIdx.x, static_cast<uint64_t>(p.n), stride);
  } else if (slots_needed(p.map)) {
    if (p.map.compact || p.map.key_only)
      build_rows<K>(p, first + threadIdx.x, static_cast<uint64_t>(p.n), stride);
    else
      build_map_batched<K>(p, first + threadIdx.x, static_cast<uint64_t>(p.n), stride);
  }
}

// One workgroup per build item: rows [begin, end) of one dim of one instance.
__global__ void __launch_bounds__(256) batch_build_kernel(BatchParams b, int pass) {
  const BatchItem& it = batch_at(b.build_items, blockIdx.x);
  const MapBuildParams& p = batch_at(b.builds, 2 * static_cast<uint64_t>(it.inst) + it.aux);
  if (pass == 0) {
    range_rows(p, it.begin, it.end, blockDim.x);
  } else if (pass == 1) {
    direct_rows(p, it.begin + threadIdx.x, it.end, blockDim.x);
  } else if (slots_needed(p.map)) {
    if (p.map.key_type == kI32)
      build_rows<int32_t>(p, it.begin + threadIdx.x, it.end, blockDim.x);
    else
      build_rows<int64_t>(p, it.begin + threadIdx.x, it.end, blockDim.x);
  }
}

// Windowed direct-table builds of a batch (dims with payloads and at most
// kMaxWins windows of kWinKeys keys): the payloads of a slice build were
// random 1-4 byte stores, each its own memory transaction. Instead the build
// rows are grouped by window first (count, place, scatter: the same totals
// and per-item reservations as the pipeline's records), and then one
// workgroup per window sets its bits and payloads in LDS and writes both out
// in order.

// Whether build params p hold a windowed direct table this batch builds.
__device__ __forceinline__ bool windowed(const MapBuildParams& p) {
  if (p.nwin == 0) return false;
  const uint64_t range = direct_range(p.map);
  return range != 0 && range <= p.map.direct_cap;
}

__device__ __forceinline__ int64_t build_row(const MapBuildParams& p, uint64_t i) {
  return p.idx ? static_cast<int64_t>(p.idx[i]) : static_cast<int64_t>(i);
}

// Rows per window of one build item, added to the windows' totals.
__global__ void __launch_bounds__(256) batch_win_count_kernel(BatchParams b) {
  __shared__ uint32_t hist[kMaxWins];
  const BatchItem& it = batch_at(b.build_items, blockIdx.x);
  const MapBuildParams& p = batch_at(b.builds, 2 * static_cast<uint64_t>(it.inst) + it.aux);
  if (!windowed(p)) return;
  const int32_t kmin = p.map.dstate[kDKmin];
  const uint32_t nwin = p.nwin;
  for (uint32_t w = threadIdx.x; w < nwin; w += blockDim.x) hist[w] = 0;
  __syncthreads();
  // four rows per thread and step, their loads in flight together
  for (uint64_t i0 = it.begin + threadIdx.x; i0 < it.end; i0 += 4 * blockDim.x) {
    int32_t key[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t i = i0 + u * blockDim.x;
      key[u] = i < it.end ? static_cast<int32_t>(load_elem(p.keys, p.type, build_row(p, i))) : kmin;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u * blockDim.x < it.end)
        atomicAdd(hist + (static_cast<uint32_t>(key[u] - kmin) >> kWinBits), 1u);
  }
  __syncthreads();
  for (uint32_t w = threadIdx.x; w < nwin; w += blockDim.x)
    if (hist[w]) atomicAdd(p.wcursor + w, hist[w]);
}

// One workgroup per dim: the windows' places (an exclusive prefix sum of
// their totals), each also the window's first free place.
constexpr int kWinScanThreads = 1024;
constexpr uint32_t kWinPer = kMaxWins / kWinScanThreads;

__global__ void __launch_bounds__(kWinScanThreads) batch_win_scan_kernel(BatchParams b) {
  __shared__ uint32_t s_wave[kWinScanThreads / kWave];
  const MapBuildParams& p = batch_at(b.builds, blockIdx.x);
  if (!windowed(p)) return;
  const uint32_t nwin = p.nwin;
  const uint32_t w0 = threadIdx.x * kWinPer;
  uint32_t c[kWinPer], sum = 0;
#pragma unroll
  for (uint32_t e = 0; e < kWinPer; ++e) {
    c[e] = w0 + e < nwin ? p.wcursor[w0 + e] : 0u;
    sum += c[e];
  }
  // exclusive prefix over the workgroup
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  uint32_t incl = sum;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += t;
  }
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  uint32_t at = incl - sum, total = 0;
  for (int w = 0; w < kWinScanThreads / kWave; ++w) {
    if (w < wave) at += s_wave[w];
    total += s_wave[w];
  }
#pragma unroll
  for (uint32_t e = 0; e < kWinPer; ++e) {
    if (w0 + e < nwin) {
      p.wbegin[w0 + e] = at;
      p.wcursor[w0 + e] = at;
    }
    at += c[e];
  }
  if (threadIdx.x == 0) p.wbegin[nwin] = total;
}

// The rows of one build item to their windows: a histogram (each row's
// rank within its window from the LDS atomic), one atomic per window on its
// cursor for the item's share, then the pairs placed in LDS in window order
// and written out in that order, so that each window's share of the item is
// stored by consecutive lanes. Pairs are (key, payload) as two 32-bit halves.
constexpr int kWinScatterThreads = 1024;
constexpr int kWinRows = static_cast<int>(kBuildChunk) / kWinScatterThreads;
static_assert(kBuildChunk % kWinScatterThreads == 0, "whole rows per thread");
constexpr uint32_t kWinOwn = kMaxWins / kWinScatterThreads;  // windows per thread in the offsets

struct WinScatterLds {
  uint64_t stage[kBuildChunk];
  uint16_t win[kBuildChunk];
  uint32_t cur[kMaxWins];  // counts, then offsets within the item, then write bases
  uint32_t wave[kWinScatterThreads / kWave];
};

__global__ void __launch_bounds__(kWinScatterThreads) batch_win_scatter_kernel(BatchParams b) {
  __shared__ __attribute__((aligned(16))) WinScatterLds L;
  const BatchItem& it = batch_at(b.build_items, blockIdx.x);
  const MapBuildParams& p = batch_at(b.builds, 2 * static_cast<uint64_t>(it.inst) + it.aux);
  if (!windowed(p)) return;
  const int32_t kmin = p.map.dstate[kDKmin];
  const uint32_t nwin = p.nwin;
  const uint32_t m = static_cast<uint32_t>(it.end - it.begin);  // <= kBuildChunk
  for (uint32_t w = threadIdx.x; w < nwin; w += blockDim.x) L.cur[w] = 0;
  uint64_t x[kWinRows];
  uint32_t wq[kWinRows], rank[kWinRows];
#pragma unroll
  for (int u = 0; u < kWinRows; ++u) {
    const uint32_t i = u * blockDim.x + threadIdx.x;
    if (i < m) {
      const int64_t r = build_row(p, it.begin + i);
      const int32_t key = static_cast<int32_t>(load_elem(p.keys, p.type, r));
      const int32_t pay = static_cast<int32_t>(load_elem(p.val_col, p.val_type, r));
      x[u] = static_cast<uint64_t>(static_cast<uint32_t>(key)) |
             static_cast<uint64_t>(static_cast<uint32_t>(pay)) << 32;
      wq[u] = static_cast<uint32_t>(key - kmin) >> kWinBits;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kWinRows; ++u)
    if (u * blockDim.x + threadIdx.x < m) rank[u] = lds_fetch_add_u32(L.cur + wq[u], 1u);
  __syncthreads();
  // offsets within the item and the global write bases, windows
  // [tid * kWinOwn, tid * kWinOwn + kWinOwn) per thread
  const uint32_t w0 = threadIdx.x * kWinOwn;
  uint32_t c[kWinOwn], sum = 0;
#pragma unroll
  for (uint32_t e = 0; e < kWinOwn; ++e) {
    c[e] = w0 + e < nwin ? L.cur[w0 + e] : 0u;
    sum += c[e];
  }
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  uint32_t incl = sum;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += t;
  }
  if (lane == kWave - 1) L.wave[wave] = incl;
  __syncthreads();
  uint32_t off = incl - sum;
  for (int w = 0; w < wave; ++w) off += L.wave[w];
  uint32_t base[kWinOwn];
#pragma unroll
  for (uint32_t e = 0; e < kWinOwn; ++e) {
    base[e] = 0;
    if (w0 + e < nwin) {
      if (c[e]) base[e] = atomicAdd(p.wcursor + w0 + e, c[e]) - off;  // modulo 2^32
      L.cur[w0 + e] = off;
      off += c[e];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kWinRows; ++u) {
    if (u * blockDim.x + threadIdx.x < m) {
      const uint32_t at = L.cur[wq[u]] + rank[u];
      L.stage[at] = x[u];
      L.win[at] = static_cast<uint16_t>(wq[u]);
    }
  }
  __syncthreads();
#pragma unroll
  for (uint32_t e = 0; e < kWinOwn; ++e)
    if (w0 + e < nwin) L.cur[w0 + e] = base[e];
  __syncthreads();
  for (uint32_t s2 = threadIdx.x; s2 < m; s2 += blockDim.x)
    p.wpairs[L.cur[L.win[s2]] + s2] = L.stage[s2];
}

// One workgroup per window: its keys' bits (an LDS atomic OR each; a bit
// already set is a duplicate) and narrowed payloads, set in LDS from the
// window's pairs and written out in order (windows are disjoint and
// word-aligned; the bitmap was zero-filled).
constexpr int kWinThreads = 256;

__global__ void __launch_bounds__(kWinThreads) batch_win_build_kernel(BatchParams b) {
  __shared__ uint32_t bits[kWinKeys / 32];
  __shared__ uint32_t vals[kWinKeys];
  const BatchItem& it = batch_at(b.win_items, blockIdx.x);
  const MapBuildParams& p = batch_at(b.builds, 2 * static_cast<uint64_t>(it.inst) + it.aux);
  if (!windowed(p)) return;
  const MapDesc& m = p.map;
  const uint64_t range = direct_range(m);
  const uint32_t w = static_cast<uint32_t>(it.begin);
  const uint64_t lo = static_cast<uint64_t>(w) << kWinBits;
  if (lo >= range) return;
  const uint32_t span = static_cast<uint32_t>(range - lo < kWinKeys ? range - lo : kWinKeys);
  const uint32_t begin = p.wbegin[w], end = p.wbegin[w + 1];
  if (begin == end) return;
  const int32_t kmin = m.dstate[kDKmin];
  const int32_t pmin = m.dstate[kDPmin];
  const int width = direct_width(pmin, m.dstate[kDPmax]);
  const uint32_t words = (span + 31) / 32;
  for (uint32_t t = threadIdx.x; t < words; t += blockDim.x) bits[t] = 0;
  __syncthreads();
  // four pairs per thread and step, their loads in flight together
  constexpr int kU = 4;
  for (uint32_t i0 = begin + threadIdx.x; i0 < end; i0 += kU * blockDim.x) {
    uint64_t pr[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t i = i0 + u * blockDim.x;
      if (i < end) pr[u] = __builtin_nontemporal_load(p.wpairs + i);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (i0 + u * blockDim.x >= end) continue;
      const uint32_t off =
          static_cast<uint32_t>(static_cast<int32_t>(pr[u]) - kmin) - static_cast<uint32_t>(lo);
      const uint32_t bit = 1u << (off & 31);
      if (atomicOr(bits + (off >> 5), bit) & bit) {
        *m.dup = 1;
        continue;
      }
      vals[off] = static_cast<uint32_t>(static_cast<int32_t>(pr[u] >> 32)) - static_cast<uint32_t>(pmin);
    }
  }
  __syncthreads();
  uint32_t* out = m.dbits + (lo >> 5);
  for (uint32_t t = threadIdx.x; t < words; t += blockDim.x) out[t] = bits[t];
  // payloads of absent keys are whatever LDS held: the bitmap hides them
  if (width == 1) {
    uint8_t* d = static_cast<uint8_t*>(m.dvals) + lo;
    for (uint32_t t = threadIdx.x; t < span; t += blockDim.x) d[t] = static_cast<uint8_t>(vals[t]);
  } else if (width == 2) {
    uint16_t* d = static_cast<uint16_t*>(m.dvals) + lo;
    for (uint32_t t = threadIdx.x; t < span; t += blockDim.x) d[t] = static_cast<uint16_t>(vals[t]);
  } else {
    uint32_t* d = static_cast<uint32_t*>(m.dvals) + lo;
    for (uint32_t t = threadIdx.x; t < span; t += blockDim.x) d[t] = vals[t];
  }
}

// Build pass 2 of a batch, one workgroup per slice item: bits [lo, lo +
// slice_bits) of one dim's direct table, set in LDS from one part of the
// dim's build rows. The workgroup reads its part's keys and takes those that
// fall in its slice: an LDS atomic OR per key (its old value shows a
// duplicate) instead of a device-scope one. A slice built from one part is
// written out with plain stores (slices are disjoint and word-aligned); the
// parts of a split slice OR their non-zero words into the table, and a bit
// that another part had already set is a duplicate too.
constexpr int kSliceThreads = 1024;

__global__ void __launch_bounds__(kSliceThreads) batch_direct_slice_kernel(BatchParams b) {
  extern __shared__ uint32_t sbits[];
  const BatchItem& it = batch_at(b.slice_items, blockIdx.x);
  const MapBuildParams& p = batch_at(b.builds, 2 * static_cast<uint64_t>(it.inst) + it.aux);
  const MapDesc& m = p.map;
  const uint64_t range = direct_range(m);
  if (range == 0 || range > m.direct_cap) return;  // no direct table for this dim
  if (p.nwin) return;                              // built by windows
  const uint64_t lo = it.begin;
  if (lo >= range) return;
  const uint64_t hi = lo + b.slice_bits < range ? lo + b.slice_bits : range;
  const uint32_t words = static_cast<uint32_t>((hi - lo + 31) / 32);
  for (uint32_t w = threadIdx.x; w < words; w += kSliceThreads) sbits[w] = 0;
  __syncthreads();
  const int32_t kmin = m.dstate[kDKmin];
  const int32_t pmin = m.dstate[kDPmin];
  const int width = p.val_col ? direct_width(pmin, m.dstate[kDPmax]) : 0;
  // rows [r_lo, r_hi) of the dim: part `part` of `nparts`
  const uint32_t part = static_cast<uint32_t>(it.end >> 32);
  const uint32_t nparts = static_cast<uint32_t>(it.end);
  const uint64_t rows = static_cast<uint64_t>(p.n);
  const uint64_t r_lo = rows * part / nparts;
  const uint64_t n = rows * (part + 1) / nparts;
  // one key of the slice: its bit (the old word shows a duplicate) and payload
  auto take = [&](uint64_t row, int64_t key) {
    const uint64_t k = static_cast<uint64_t>(static_cast<uint32_t>(key - kmin));
    if (k < lo || k >= hi) return;
    const uint32_t off = static_cast<uint32_t>(k - lo);
    const uint32_t bit = 1u << (off & 31);
    const uint32_t old = atomicOr(&sbits[off >> 5], bit);
    if (old & bit) {
      *m.dup = 1;
      return;
    }
    if (width == 0) return;
    const uint32_t v = static_cast<uint32_t>(load_elem(p.val_col, p.val_type, static_cast<int64_t>(row))) -
                       static_cast<uint32_t>(pmin);
    if (width == 1) static_cast<uint8_t*>(m.dvals)[k] = static_cast<uint8_t>(v);
    else if (width == 2) static_cast<uint16_t*>(m.dvals)[k] = static_cast<uint16_t>(v);
    else static_cast<uint32_t*>(m.dvals)[k] = v;
  };
  if (!p.idx && p.type == kI32 && reinterpret_cast<uintptr_t>(p.keys) % 16 == 0) {
    // every slice reads all the keys: 16-byte loads, four per lane in flight
    // (plain loads: the dim's other slices read the same lines)
    typedef int32_t v4 __attribute__((ext_vector_type(4)));
    const v4* k4 = static_cast<const v4*>(p.keys);
    // whole 16-byte groups of the part; the rows before the first and after
    // the last one singly
    const uint64_t g_lo = (r_lo + 3) / 4;
    const uint64_t n4 = n / 4 > g_lo ? n / 4 : g_lo;
    for (uint64_t r = r_lo + threadIdx.x; r < 4 * g_lo && r < n; r += kSliceThreads)
      take(r, static_cast<const int32_t*>(p.keys)[r]);
    constexpr int U = 4;
    // int32 payloads come with the keys, four per load, so that a key of the
    // slice needs no further read
    const bool pvec = width != 0 && p.val_type == kI32 && reinterpret_cast<uintptr_t>(p.val_col) % 16 == 0;
    const v4* v4p = static_cast<const v4*>(p.val_col);
    for (uint64_t q = g_lo + threadIdx.x; q < n4; q += U * kSliceThreads) {
      v4 x[U], y[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t at = q + static_cast<uint64_t>(u) * kSliceThreads;
        x[u] = at < n4 ? k4[at] : v4{0, 0, 0, 0};
        y[u] = (pvec && at < n4) ? v4p[at] : v4{0, 0, 0, 0};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t at = q + static_cast<uint64_t>(u) * kSliceThreads;
        if (at >= n4) continue;
        const int32_t key[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
        const int32_t pay[4] = {y[u].x, y[u].y, y[u].z, y[u].w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (!pvec) {
            take(4 * at + e, key[e]);
            continue;
          }
          const uint64_t k = static_cast<uint64_t>(static_cast<uint32_t>(key[e] - kmin));
          if (k < lo || k >= hi) continue;
          const uint32_t off = static_cast<uint32_t>(k - lo);
          const uint32_t bit = 1u << (off & 31);
          if (atomicOr(&sbits[off >> 5], bit) & bit) {
            *m.dup = 1;
            continue;
          }
          const uint32_t v = static_cast<uint32_t>(pay[e]) - static_cast<uint32_t>(pmin);
          if (width == 1) static_cast<uint8_t*>(m.dvals)[k] = static_cast<uint8_t>(v);
          else if (width == 2) static_cast<uint16_t*>(m.dvals)[k] = static_cast<uint16_t>(v);
          else static_cast<uint32_t*>(m.dvals)[k] = v;
        }
      }
    }
    for (uint64_t r = 4 * n4 + threadIdx.x; r < n; r += kSliceThreads)
      take(r, static_cast<const int32_t*>(p.keys)[r]);
  } else {
    for (uint64_t i = r_lo + threadIdx.x; i < n; i += kSliceThreads) {
      const uint64_t row = p.idx ? p.idx[i] : i;
      take(row, load_elem(p.keys, p.type, static_cast<int64_t>(row)));
    }
  }
  __syncthreads();
  uint32_t* out = m.dbits + lo / 32;
  if (nparts == 1) {
    for (uint32_t w = threadIdx.x; w < words; w += kSliceThreads) out[w] = sbits[w];
  } else {
    for (uint32_t w = threadIdx.x; w < words; w += kSliceThreads) {
      const uint32_t mine = sbits[w];
      if (mine == 0) continue;
      if (atomicOr(out + w, mine) & mine) *m.dup = 1;
    }
  }
}

// One workgroup per fill item.
__global__ void __launch_bounds__(256) batch_fill_kernel(BatchParams b) {
  const FillItem& f = batch_at(b.fill, blockIdx.x);
  const int32_t kind = f.kind;
  uint64_t* out = f.p;
  if (kind == kFillGroup) {
    const GroupDesc& g = batch_at(b.plans, f.inst).g;
    const uint32_t words = static_cast<uint32_t>(g.words);
    // word index within the slot, stepped by blockDim mod words (no division
    // in the loop)
    const uint64_t first = f.begin + threadIdx.x;
    uint32_t w = static_cast<uint32_t>(first % words);
    const uint32_t step = blockDim.x % words;
    for (uint64_t i = first; i < f.end; i += blockDim.x) {
      uint64_t v = 0;
      if (w == 0) v = kEmpty64;
      else if (w >= 2 && static_cast<int>(w) - 2 < g.ap.nacc) v = acc_identity(g.ap.kind[w - 2]);
      out[i] = v;
      w += step;
      if (w >= words) w -= words;
    }
  } else {
    const uint64_t pattern = f.pattern;
    for (uint64_t i = f.begin + threadIdx.x; i < f.end; i += blockDim.x)
      out[i] = kind == kFillPairs ? ((i & 1) ? 0ULL : kEmpty64) : pattern;
  }
}

// Matched pairs are staged per wave in LDS and written in runs: one cursor
// atomic per run of at least kProbeFlush pairs instead of one per wave and
// round (a single global counter shared by every wave serialises otherwise).
// Each lane walks kProbeKeys probe keys at once: their key loads, and every
// round's slot loads, are independent and in flight together.
constexpr int kProbeStage = 1024;
constexpr int kProbeKeys = 4;
constexpr int kProbeFlush = kProbeStage - kProbeKeys * kWave;

__device__ __forceinline__ void flush_pairs(const MapProbeParams& p, const uint32_t* sb,
                                            const uint32_t* sp, uint32_t staged, int lane) {
  __builtin_amdgcn_wave_barrier();
  unsigned long long at = 0;
  if (lane == 0) at = atomicAdd(p.d_count, static_cast<unsigned long long>(staged));
  at = first_lane(at);
  for (uint32_t i = lane; i < staged; i += kWave) {
    const unsigned long long pos = at + i;
    if (pos < static_cast<unsigned long long>(p.cap)) {
      p.out_build[pos] = sb[i];
      p.out_probe[pos] = sp[i];
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// Cursor states of a probe key.
constexpr uint32_t kWalkDone = 0, kWalkSlots = 1, kWalkOob = 2;

template <typename K>
__global__ void __launch_bounds__(256) map_probe_kernel(MapProbeParams p) {
  __shared__ uint32_t s_build[256 / kWave][kProbeStage];
  __shared__ uint32_t s_probe[256 / kWave][kProbeStage];
  using Slot = typename std::conditional<sizeof(K) == 4, uint64_t, ulonglong2>::type;
  const Slot* slots = static_cast<const Slot*>(p.map.slots);
  const K* keys = static_cast<const K*>(p.keys);
  const uint64_t mask = p.map.cap - 1;
  // Without duplicate build keys a probe key has at most one match, and its
  // walk ends there.
  const bool unique = *p.map.dup == 0;
  const unsigned long long oob_n = *p.map.oob_count;
  const int lane = lane_id();
  uint32_t* sb = s_build[threadIdx.x / kWave];
  uint32_t* sp = s_probe[threadIdx.x / kWave];
  uint32_t staged = 0;  // wave-uniform
  const uint64_t n = static_cast<uint64_t>(p.n);
  const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x * kProbeKeys;
  // The loop bound is uniform across the workgroup, so whole waves stay
  // together through the ballots below.
  for (uint64_t base = blockIdx.x * static_cast<uint64_t>(blockDim.x) * kProbeKeys; base < n;
       base += step) {
    uint64_t row[kProbeKeys], pos[kProbeKeys];
    uint32_t state[kProbeKeys];
    K key[kProbeKeys];
#pragma unroll
    for (int j = 0; j < kProbeKeys; ++j) {
      const uint64_t i = base + static_cast<uint64_t>(j) * blockDim.x + threadIdx.x;
      row[j] = i < n ? i : 0;
      state[j] = i < n ? kWalkSlots : kWalkDone;
    }
    if (p.idx) {
#pragma unroll
      for (int j = 0; j < kProbeKeys; ++j) row[j] = p.idx[row[j]];
    }
#pragma unroll
    for (int j = 0; j < kProbeKeys; ++j) key[j] = keys[row[j]];
    if (p.bloom.words) {
      // semi-join reduction: keys absent from the build side's Bloom filter
      // end here, before their walk through the table
      uint64_t h[kProbeKeys];
      uint4 qa[kProbeKeys], qb[kProbeKeys];
#pragma unroll
      for (int j = 0; j < kProbeKeys; ++j) {
        h[j] = bloom_hash(static_cast<int64_t>(key[j]));
        qa[j] = make_uint4(0, 0, 0, 0);
        qb[j] = qa[j];
        if (state[j] != kWalkDone) {
          const uint4* q = reinterpret_cast<const uint4*>(
              p.bloom.words + bloom_block(h[j], p.bloom.bmask) * 8);
          qa[j] = q[0];
          qb[j] = q[1];
        }
      }
#pragma unroll
      for (int j = 0; j < kProbeKeys; ++j)
        if (state[j] != kWalkDone && !bloom_match(h[j], qa[j], qb[j])) state[j] = kWalkDone;
    }
#pragma unroll
    for (int j = 0; j < kProbeKeys; ++j) {
      bool oob;
      if constexpr (sizeof(K) == 4) {
        oob = key[j] == kEmpty32;
        pos[j] = oob ? 0 : home32(key[j], mask);
      } else {
        oob = static_cast<uint64_t>(key[j]) == kEmpty64;
        pos[j] = oob ? 0 : home64(key[j], mask);
      }
      if (oob && state[j] != kWalkDone) state[j] = kWalkOob;
    }
    while (true) {
      uint32_t any = kWalkDone;
#pragma unroll
      for (int j = 0; j < kProbeKeys; ++j) any |= state[j];
      if (ballot(any != kWalkDone) == 0) break;
      Slot sl[kProbeKeys];
#pragma unroll
      for (int j = 0; j < kProbeKeys; ++j)
        if (state[j] == kWalkSlots) sl[j] = slots[pos[j]];
#pragma unroll
      for (int j = 0; j < kProbeKeys; ++j) {
        bool found = false;
        uint32_t val = 0;
        if (state[j] == kWalkSlots) {
          K k;
          if constexpr (sizeof(K) == 4) {
            k = static_cast<int32_t>(static_cast<uint32_t>(sl[j]));
            val = static_cast<uint32_t>(sl[j] >> 32);
          } else {
            k = static_cast<int64_t>(sl[j].x);
            val = static_cast<uint32_t>(sl[j].y);
          }
          const bool empty = sizeof(K) == 4 ? (k == static_cast<K>(kEmpty32))
                                            : (static_cast<uint64_t>(k) == kEmpty64);
          found = !empty && k == key[j];
          if (empty || (found && unique)) state[j] = kWalkDone;
          pos[j] = (pos[j] + 1) & mask;
        } else if (state[j] == kWalkOob) {
          if (pos[j] < oob_n) {
            val = p.map.oob_vals[pos[j]++];
            found = true;
          } else {
            state[j] = kWalkDone;
          }
        }
        const uint64_t m = ballot(found);
        if (found) {
          const uint32_t at = staged + rank_below(m);
          sb[at] = val;
          sp[at] = static_cast<uint32_t>(row[j]);
        }
        staged += popc64(m);
      }
      if (staged > static_cast<uint32_t>(kProbeFlush)) {
        flush_pairs(p, sb, sp, staged, lane);
        staged = 0;
      }
    }
  }
  if (staged > 0) flush_pairs(p, sb, sp, staged, lane);
}

}  // namespace

void launch_fill64(uint64_t* p, uint64_t n, uint64_t pattern, hipStream_t s) {
  if (n == 0) return;
  ProfileScope ps(kKFill, s);
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill64_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, n,
                     pattern);
}

void launch_map_init(const MapDesc& m, hipStream_t s) {
  if (m.compact) {
    // every 16-bit entry empty (0xFFFF); cap counts 16-byte buckets
    launch_fill64(static_cast<uint64_t*>(m.slots), m.cap * 2, ~0ULL, s);
    launch_fill64(reinterpret_cast<uint64_t*>(m.over), m.over_cap / 2, 0x8000000080000000ULL, s);
  } else if (m.key_only) {
    // two empty 32-bit slots per word (cap >= 64 is even)
    launch_fill64(static_cast<uint64_t*>(m.slots), m.cap / 2, 0x8000000080000000ULL, s);
  } else if (m.key_type == kI32) {
    launch_fill64(static_cast<uint64_t*>(m.slots), m.cap, kEmptySlot32, s);
  } else {
    ProfileScope ps(kKFill, s);
    uint64_t blocks = (m.cap + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_map64_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<ulonglong2*>(m.slots), m.cap);
  }
  // the out-of-band count and the duplicate flag share the header
  launch_fill64(reinterpret_cast<uint64_t*>(m.oob_count), 2, 0, s);
  if (m.direct_cap) {
    // empty key and payload ranges, no key present
    launch_fill64(reinterpret_cast<uint64_t*>(m.dstate), 2, kDirectStateInit, s);
    launch_fill64(reinterpret_cast<uint64_t*>(m.dbits), m.direct_cap / 64, 0, s);
  }
}

void launch_map_build(const MapBuildParams& p, hipStream_t s) {
  if (p.n == 0) return;
  ProfileScope ps(kKMapBuild, s);
  const DeviceInfo& di = device_info();
  uint64_t blocks = (static_cast<uint64_t>(p.n) + 255) / 256;
  uint64_t limit = static_cast<uint64_t>(di.cu_count) * 8;
  if (blocks > limit) blocks = limit;
  // the range and direct passes only for maps with a direct table
  for (int pass = p.map.direct_cap ? 0 : 2; pass < 3; ++pass) {
    if (p.map.key_type == kI32)
      hipLaunchKernelGGL(map_build_kernel<int32_t>, dim3(static_cast<unsigned>(blocks)), dim3(256),
                         0, s, p, pass);
    else
      hipLaunchKernelGGL(map_build_kernel<int64_t>, dim3(static_cast<unsigned>(blocks)), dim3(256),
                         0, s, p, pass);
  }
}

void launch_batch_fill(const BatchParams& b, hipStream_t s) {
  if (b.nfill == 0) return;
  ProfileScope ps(kKFill, s);
  hipLaunchKernelGGL(batch_fill_kernel, dim3(b.nfill), dim3(256), 0, s, b);
}

void launch_batch_build(const BatchParams& b, hipStream_t s) {
  if (b.nbuild == 0) return;
  ProfileScope ps(kKMapBuild, s);
  hipLaunchKernelGGL(batch_build_kernel, dim3(b.nbuild), dim3(256), 0, s, b, 0);
  if (b.nwin > 0) {
    hipLaunchKernelGGL(batch_win_count_kernel, dim3(b.nbuild), dim3(256), 0, s, b);
    hipLaunchKernelGGL(batch_win_scan_kernel, dim3(2 * b.nplans), dim3(kWinScanThreads), 0, s, b);
    hipLaunchKernelGGL(batch_win_scatter_kernel, dim3(b.nbuild), dim3(kWinScatterThreads), 0, s, b);
    hipLaunchKernelGGL(batch_win_build_kernel, dim3(b.nwin), dim3(kWinThreads), 0, s, b);
  }
  if (b.nslice > 0) {
    const size_t lds = static_cast<size_t>(b.slice_bits) / 8;
    static size_t allowed = 0;
    if (allowed < lds &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(batch_direct_slice_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) == hipSuccess)
      allowed = lds;
    hipLaunchKernelGGL(batch_direct_slice_kernel, dim3(b.nslice), dim3(kSliceThreads), lds, s, b);
  }
  hipLaunchKernelGGL(batch_build_kernel, dim3(b.nbuild), dim3(256), 0, s, b, 2);
}

void launch_map_probe(const MapProbeParams& p, int grid, int block, hipStream_t s) {
  if (p.n == 0) return;
  ProfileScope ps(kKMapProbe, s);
  if (p.map.key_type == kI32)
    hipLaunchKernelGGL(map_probe_kernel<int32_t>, dim3(grid), dim3(block), 0, s, p);
  else
    hipLaunchKernelGGL(map_probe_kernel<int64_t>, dim3(grid), dim3(block), 0, s, p);
}

}  // namespace rel
