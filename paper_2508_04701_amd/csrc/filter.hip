// Selection with ordered stream compaction, one pass over the columns.
//
// A workgroup of 512 threads takes one tile of 16384 rows. Thread t of the
// tile reads rows (j * 2048 + 4 t .. + 3) for j = 0..7, so every column read
// is a coalesced 16-byte-per-lane vector load. Each passing row sets one bit;
// per chunk a wave64 ballot per row position gives the wave's count (popcount)
// and each lane's rank (mbcnt), which places every passing row id at its
// ascending position inside the tile. The tile's base in the output comes
// from a decoupled look-back over the preceding tiles: each tile publishes
// its count (flag AGG) and later its inclusive prefix (flag PREFIX) in one
// 64-bit word with agent-scope atomics, so the eight XCD L2 caches never hold
// a stale state. Tiles are numbered by an atomic ticket in launch order, so
// every tile that a look-back waits on has already started and will publish.
// Each lane then writes its passing rows' ids straight to their positions.

#include <mutex>
#include <type_traits>

#include "internal.h"

namespace rel {

// Tile states of rel_filter_noalloc (a file-scope device array: each GPU the
// library runs on holds its own copy until the process ends). Host code
// never passes this name to a kernel: it takes the device address that
// filter_scratch() looks up.
static __device__ __align__(256) unsigned char scratch[kFilterScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

hipError_t filter_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

namespace {

typedef int32_t v4i32 __attribute__((ext_vector_type(4)));
typedef int64_t v2i64 __attribute__((ext_vector_type(2)));

constexpr uint64_t kFlagAgg = 1ULL << 62;
constexpr uint64_t kFlagPrefix = 2ULL << 62;
constexpr uint64_t kValueMask = (1ULL << 62) - 1;

__device__ __forceinline__ uint32_t eval_chunk(const FilterParams& p, int64_t r0) {
  uint32_t bits = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) bits |= (r0 + e < p.n) ? (1u << e) : 0u;
  if (bits == 0) return 0;
  for (int t = 0; t < p.nterms; ++t) {
    const FilterTerm& term = p.term[t];
    int64_t v[4];
    if (p.idx) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        v[e] = (r0 + e < p.n) ? load_elem(term.data, term.type, p.idx[r0 + e]) : 0;
    } else {
      load4(term.data, term.type, term.vec != 0, r0, p.n, v);
    }
    uint32_t m = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) m |= term_holds(term.op, v[e], term.lo, term.hi) ? (1u << e) : 0u;
    bits &= m;
  }
  return bits;
}

// A whole tile of plain columns: per term, the loads of the thread's four
// chunks are issued together (the type and alignment tests are uniform), and
// only then compared. Each column byte is read once: non-temporal loads keep
// the stream from displacing reused lines in the caches.
__device__ __forceinline__ uint32_t holds4(const FilterTerm& t, int64_t a, int64_t b, int64_t c,
                                           int64_t d) {
  return (term_holds(t.op, a, t.lo, t.hi) ? 1u : 0u) | (term_holds(t.op, b, t.lo, t.hi) ? 2u : 0u) |
         (term_holds(t.op, c, t.lo, t.hi) ? 4u : 0u) | (term_holds(t.op, d, t.lo, t.hi) ? 8u : 0u);
}

__device__ __forceinline__ void eval_whole(const FilterParams& p, int64_t r0,
                                           uint32_t bits[kFilterChunks]) {
  constexpr int64_t kChunk = kFilterThreads * 4;
#pragma unroll
  for (int j = 0; j < kFilterChunks; ++j) bits[j] = 0xFu;
  for (int t = 0; t < p.nterms; ++t) {
    const FilterTerm& term = p.term[t];
    if (term.vec && term.type == kI32) {
      const int32_t* d = static_cast<const int32_t*>(term.data) + r0;
      v4i32 x[kFilterChunks];
#pragma unroll
      for (int j = 0; j < kFilterChunks; ++j)
        x[j] = __builtin_nontemporal_load(reinterpret_cast<const v4i32*>(d + j * kChunk));
#pragma unroll
      for (int j = 0; j < kFilterChunks; ++j) bits[j] &= holds4(term, x[j].x, x[j].y, x[j].z, x[j].w);
    } else if (term.vec && term.type == kI64) {
      // four chunks at a time (eight would hold 64 registers of loaded data)
      const int64_t* d = static_cast<const int64_t*>(term.data) + r0;
#pragma unroll
      for (int g = 0; g < kFilterChunks; g += 4) {
        v2i64 a[4], b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          a[j] = __builtin_nontemporal_load(reinterpret_cast<const v2i64*>(d + (g + j) * kChunk));
          b[j] = __builtin_nontemporal_load(reinterpret_cast<const v2i64*>(d + (g + j) * kChunk) + 1);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) bits[g + j] &= holds4(term, a[j].x, a[j].y, b[j].x, b[j].y);
      }
    } else if (term.vec) {
      const int8_t* d = static_cast<const int8_t*>(term.data) + r0;
      int32_t w[kFilterChunks];
#pragma unroll
      for (int j = 0; j < kFilterChunks; ++j)
        w[j] = __builtin_nontemporal_load(reinterpret_cast<const int32_t*>(d + j * kChunk));
#pragma unroll
      for (int j = 0; j < kFilterChunks; ++j)
        bits[j] &= holds4(term, static_cast<int8_t>(w[j]), static_cast<int8_t>(w[j] >> 8),
                          static_cast<int8_t>(w[j] >> 16), static_cast<int8_t>(w[j] >> 24));
    } else {
#pragma unroll
      for (int j = 0; j < kFilterChunks; ++j) {
        const int64_t q = r0 + j * kChunk;
        bits[j] &= holds4(term, load_elem(term.data, term.type, q), load_elem(term.data, term.type, q + 1),
                          load_elem(term.data, term.type, q + 2), load_elem(term.data, term.type, q + 3));
      }
    }
  }
}

// eval_whole for plans whose terms all read 16-byte aligned int32 columns:
// the one load shape, so the kernel that uses it keeps few registers.
__device__ __forceinline__ void eval_whole_i32(const FilterParams& p, int64_t r0,
                                               uint32_t bits[kFilterChunks]) {
  constexpr int64_t kChunk = kFilterThreads * 4;
#pragma unroll
  for (int j = 0; j < kFilterChunks; ++j) bits[j] = 0xFu;
  for (int t = 0; t < p.nterms; ++t) {
    const FilterTerm& term = p.term[t];
    const int32_t* d = static_cast<const int32_t*>(term.data) + r0;
    v4i32 x[kFilterChunks];
#pragma unroll
    for (int j = 0; j < kFilterChunks; ++j)
      x[j] = __builtin_nontemporal_load(reinterpret_cast<const v4i32*>(d + j * kChunk));
#pragma unroll
    for (int j = 0; j < kFilterChunks; ++j) bits[j] &= holds4(term, x[j].x, x[j].y, x[j].z, x[j].w);
  }
}

// Semi-join reduction of one chunk: clears the bits of rows r0..r0+3 whose
// key is absent from the Bloom filter (the four rows' filter blocks are read
// together).
__device__ __forceinline__ uint32_t bloom_chunk(const FilterParams& p, int64_t r0, uint32_t bits) {
  if (!p.bloom.words || bits == 0) return bits;
  int64_t key[4];
  if (!p.idx) {
    load4(p.bloom_keys, p.bloom_type, p.bloom_vec != 0, r0, p.n, key);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      key[e] = (r0 + e < p.n) ? load_elem(p.bloom_keys, p.bloom_type, p.idx[r0 + e]) : 0;
  }
  uint64_t h[4];
  uint4 a[4], b[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    h[e] = bloom_hash(key[e]);
    a[e] = make_uint4(0, 0, 0, 0);
    b[e] = a[e];
    if ((bits >> e) & 1u) {
      const uint4* q =
          reinterpret_cast<const uint4*>(p.bloom.words + bloom_block(h[e], p.bloom.bmask) * 8);
      a[e] = q[0];
      b[e] = q[1];
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (((bits >> e) & 1u) && !bloom_match(h[e], a[e], b[e])) bits &= ~(1u << e);
  return bits;
}

// kPlain: no selection vector and no Bloom filter (its own register
// allocation, without the registers those paths need).
template <bool kPlain>
__global__ void __launch_bounds__(kFilterThreads) filter_kernel(FilterParams p) {
  __shared__ uint32_t s_wave_total[kFilterChunks][kFilterThreads / kWave];
  __shared__ int64_t s_tile;
  __shared__ uint64_t s_excl;

  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = lane_id();

  if (tid == 0) s_tile = atomicAdd(p.ticket, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t base = tile * kFilterTile;

  uint32_t bits[kFilterChunks];
  if ((kPlain || !p.idx) && base + kFilterTile <= p.n) {
    eval_whole(p, base + tid * 4, bits);
  } else {
#pragma unroll
    for (int j = 0; j < kFilterChunks; ++j)
      bits[j] = eval_chunk(p, base + j * (kFilterThreads * 4) + tid * 4);
  }
  if (!kPlain && p.bloom.words) {
#pragma unroll
    for (int j = 0; j < kFilterChunks; ++j)
      bits[j] = bloom_chunk(p, base + j * (kFilterThreads * 4) + tid * 4, bits[j]);
  }

  // Per chunk: this lane's rank among the wave's passing rows, and the
  // wave's count.
  uint32_t lane_prefix[kFilterChunks];
#pragma unroll
  for (int j = 0; j < kFilterChunks; ++j) {
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      uint64_t b = ballot((bits[j] >> e) & 1u);
      pre += rank_below(b);
      tot += popc64(b);
    }
    lane_prefix[j] = pre;
    if (lane == 0) s_wave_total[j][wave] = tot;
  }
  __syncthreads();

  // Offsets in tile order (chunk, wave, lane, row).
  uint32_t chunk_base[kFilterChunks];
  uint32_t running = 0;
#pragma unroll
  for (int j = 0; j < kFilterChunks; ++j) {
    for (int w = 0; w < kFilterThreads / kWave; ++w) {
      if (w == wave) chunk_base[j] = running;
      running += s_wave_total[j][w];
    }
  }
  const uint32_t total = running;

  if (wave == 0) {
    uint64_t excl = 0;
    if (tile == 0) {
      if (lane == 0) store_agent(&p.tile_state[0], kFlagPrefix | total);
    } else {
      if (lane == 0) store_agent(&p.tile_state[tile], kFlagAgg | total);
      int64_t pos = tile - 1;
      while (true) {
        int64_t t = pos - lane;
        uint64_t st = t >= 0 ? load_agent(&p.tile_state[t]) : kFlagPrefix;
        uint64_t flag = st >> 62;
        uint64_t pm = ballot(flag == 2);
        uint64_t inv = ballot(flag == 0);
        uint64_t upto = pm ? (((pm & (~pm + 1)) << 1) - 1) : ~0ULL;
        if (inv & upto) {
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += wave_sum_u64(((upto >> lane) & 1ULL) ? (st & kValueMask) : 0ULL);
        if (pm) break;
        pos -= kWave;
      }
      if (lane == 0) store_agent(&p.tile_state[tile], kFlagPrefix | (excl + total));
    }
    if (lane == 0) s_excl = excl;
  }

  __syncthreads();
  // Each lane writes its passing rows' ids at their output positions; a
  // wave's stores of one row position land in a few consecutive lines.
  const uint64_t excl = s_excl;
#pragma unroll
  for (int j = 0; j < kFilterChunks; ++j) {
    if (bits[j] == 0) continue;
    const int64_t r0 = base + j * (kFilterThreads * 4) + tid * 4;
    uint64_t pos = excl + chunk_base[j] + lane_prefix[j];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if ((bits[j] >> e) & 1u) {
        if (static_cast<int64_t>(pos) < p.cap)
          p.out[pos] = (!kPlain && p.idx) ? p.idx[r0 + e] : static_cast<uint32_t>(r0 + e);
        ++pos;
      }
    }
  }
  if (tile == p.ntiles - 1 && tid == 0) *p.d_count = static_cast<long long>(excl + total);
}

// ------------------------------------------------ selection bitmap path
//
// rel_filter with a workspace: three passes instead of one with a look-back
// chain. (1) Mark: each workgroup evaluates one tile of rows exactly as above
// and writes the tile's selection bitmap (bit r of word w = row 32 w + r of
// the tile) and its count; no ticket, no look-back, so workgroups never wait
// on each other and the pass streams the columns. (2) Scan: one workgroup
// turns the tile counts into exclusive offsets and the total. (3) Expand:
// each workgroup reads its tile's bitmap (2 KB instead of the columns),
// places the set bits' row ids in LDS at their ranks and writes them out with
// coalesced stores.

constexpr int kTileWords = kFilterTile / 32;  // bitmap words per tile

// kMode 2: every term an aligned int32 column, no selection vector, no Bloom
// term; 1: no selection vector and no Bloom term; 0: anything.
template <int kMode>
__global__ void __launch_bounds__(kFilterThreads) filter_mark_kernel(FilterParams p) {
  constexpr bool kPlain = kMode > 0;
  __shared__ uint32_t s_wave[kFilterThreads / kWave];
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * kFilterTile;
  uint32_t bits[kFilterChunks];
  if (kMode == 2 && base + kFilterTile <= p.n) {
    eval_whole_i32(p, base + tid * 4, bits);
  } else if (kMode != 2 && (kPlain || !p.idx) && base + kFilterTile <= p.n) {
    eval_whole(p, base + tid * 4, bits);
  } else {
#pragma unroll
    for (int j = 0; j < kFilterChunks; ++j)
      bits[j] = eval_chunk(p, base + j * (kFilterThreads * 4) + tid * 4);
  }
  if (!kPlain && p.bloom.words) {
#pragma unroll
    for (int j = 0; j < kFilterChunks; ++j)
      bits[j] = bloom_chunk(p, base + j * (kFilterThreads * 4) + tid * 4, bits[j]);
  }
  // eight lanes' four-row nibbles make one word of 32 consecutive rows
  uint32_t* words = p.bitmap + tile * kTileWords;
  uint32_t cnt = 0;
#pragma unroll
  for (int j = 0; j < kFilterChunks; ++j) {
    uint32_t x = bits[j] << (4 * (lane & 7));
    x |= __shfl_xor(x, 1, kWave);
    x |= __shfl_xor(x, 2, kWave);
    x |= __shfl_xor(x, 4, kWave);
    if ((lane & 7) == 0) words[j * (kFilterThreads * 4 / 32) + tid / 8] = x;
    cnt += __popc(bits[j]);
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
  if (lane == 0) s_wave[tid / kWave] = cnt;
  __syncthreads();
  if (tid == 0) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kFilterThreads / kWave; ++w) t += s_wave[w];
    p.tile_count[tile] = t;
  }
}

constexpr int kScanThreads = 1024;

// Exclusive offsets of groups of kFilterGroupTiles tiles (one workgroup:
// each step, thread g sums one group's counts with 16-byte loads, and the
// step's sums are scanned across the block), and the total.
__global__ void __launch_bounds__(kScanThreads) filter_scan_kernel(FilterParams p) {
  __shared__ uint64_t s_wave[kScanThreads / kWave];
  __shared__ uint64_t s_carry;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int64_t nt = p.ntiles;
  const int64_t ng = (nt + kFilterGroupTiles - 1) / kFilterGroupTiles;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int64_t g0 = 0; g0 < ng; g0 += kScanThreads) {
    const int64_t g = g0 + tid;
    uint64_t sum = 0;
    if (g < ng) {
      const int64_t t0 = g * kFilterGroupTiles;
      if (t0 + kFilterGroupTiles <= nt) {
        const uint4* c = reinterpret_cast<const uint4*>(p.tile_count + t0);
        uint4 v[kFilterGroupTiles / 4];
#pragma unroll
        for (int i = 0; i < kFilterGroupTiles / 4; ++i) v[i] = c[i];
#pragma unroll
        for (int i = 0; i < kFilterGroupTiles / 4; ++i) sum += v[i].x + v[i].y + v[i].z + v[i].w;
      } else {
        for (int64_t t = t0; t < nt; ++t) sum += p.tile_count[t];
      }
    }
    uint64_t x = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t lo = __shfl_up(static_cast<uint32_t>(x), off, kWave);
      const uint32_t hi = __shfl_up(static_cast<uint32_t>(x >> 32), off, kWave);
      if (lane >= off) x += static_cast<uint64_t>(hi) << 32 | lo;
    }
    if (lane == kWave - 1) s_wave[tid / kWave] = x;
    __syncthreads();
    uint64_t before = s_carry;
    uint64_t step = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
      if (w < tid / kWave) before += s_wave[w];
      step += s_wave[w];
    }
    if (g < ng) p.group_offset[g] = before + x - sum;
    __syncthreads();
    if (tid == 0) s_carry += step;
    __syncthreads();
  }
  if (tid == 0) *p.d_count = static_cast<long long>(s_carry);
}

// Row ids are staged in LDS as their 16-bit offsets within the tile (32 KB,
// so four workgroups fit a CU), or whole when a selection vector maps them.
template <bool kIdx>
__global__ void __launch_bounds__(kFilterThreads) filter_expand_kernel(FilterParams p) {
  typedef typename std::conditional<kIdx, uint32_t, uint16_t>::type Staged;
  __shared__ Staged s_rows[kFilterTile];
  __shared__ uint32_t s_wave[kFilterThreads / kWave];
  __shared__ uint64_t s_first;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid / kWave;
  const int64_t tile = blockIdx.x;
  // the tile's offset: its group's, plus the counts of the group's earlier
  // tiles (wave 0 reads them together with the bitmap words)
  const int64_t t0 = tile / kFilterGroupTiles * kFilterGroupTiles;
  uint32_t c0 = 0;
  uint64_t g0 = 0;
  if (wave == 0) {
    if (t0 + lane < tile) c0 = p.tile_count[t0 + lane];
    if (lane == 0) g0 = p.group_offset[tile / kFilterGroupTiles];
  }
  const uint32_t w = p.bitmap[tile * kTileWords + tid];
  const uint32_t c = __popc(w);
  uint32_t x = c;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  if (lane == kWave - 1) s_wave[wave] = x;
  if (wave == 0) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) c0 += __shfl_xor(c0, off, kWave);
    if (lane == 0) s_first = g0 + c0;
  }
  __syncthreads();
  uint32_t at = x - c;
  uint32_t total = 0;
#pragma unroll
  for (int v = 0; v < kFilterThreads / kWave; ++v) {
    if (v < wave) at += s_wave[v];
    total += s_wave[v];
  }
  const int64_t tile_row0 = tile * kFilterTile;
  const uint32_t local0 = static_cast<uint32_t>(tid) * 32;
  for (uint32_t m = w; m != 0; m &= m - 1) {
    const uint32_t local = local0 + (__ffs(m) - 1);
    if constexpr (kIdx) s_rows[at++] = p.idx[tile_row0 + local];
    else s_rows[at++] = static_cast<Staged>(local);
  }
  __syncthreads();
  const uint64_t first = s_first;
  for (uint32_t i = tid; i < total; i += kFilterThreads) {
    const uint64_t pos = first + i;
    if (static_cast<int64_t>(pos) < p.cap)
      p.out[pos] = kIdx ? static_cast<uint32_t>(s_rows[i])
                        : static_cast<uint32_t>(tile_row0) + static_cast<uint32_t>(s_rows[i]);
  }
}

}  // namespace

void launch_filter_marked(const FilterParams& p, hipStream_t s) {
  ProfileScope ps(kKFilter, s);
  const dim3 grid(static_cast<unsigned>(p.ntiles));
  bool all_i32 = true;
  for (int t = 0; t < p.nterms; ++t) all_i32 = all_i32 && p.term[t].type == kI32 && p.term[t].vec;
  if (!p.idx && !p.bloom.words && all_i32)
    hipLaunchKernelGGL(filter_mark_kernel<2>, grid, dim3(kFilterThreads), 0, s, p);
  else if (!p.idx && !p.bloom.words)
    hipLaunchKernelGGL(filter_mark_kernel<1>, grid, dim3(kFilterThreads), 0, s, p);
  else
    hipLaunchKernelGGL(filter_mark_kernel<0>, grid, dim3(kFilterThreads), 0, s, p);
  hipLaunchKernelGGL(filter_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, p);
  if (p.idx)
    hipLaunchKernelGGL(filter_expand_kernel<true>, grid, dim3(kFilterThreads), 0, s, p);
  else
    hipLaunchKernelGGL(filter_expand_kernel<false>, grid, dim3(kFilterThreads), 0, s, p);
}

void launch_filter(const FilterParams& p, hipStream_t s) {
  ProfileScope ps(kKFilter, s);
  if (!p.idx && !p.bloom.words)
    hipLaunchKernelGGL(filter_kernel<true>, dim3(static_cast<unsigned>(p.ntiles)), dim3(kFilterThreads),
                       0, s, p);
  else
    hipLaunchKernelGGL(filter_kernel<false>, dim3(static_cast<unsigned>(p.ntiles)),
                       dim3(kFilterThreads), 0, s, p);
}

}  // namespace rel
