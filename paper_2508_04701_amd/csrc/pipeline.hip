// Fused plan: conjunctive filter -> inner join with up to two dims ->
// group-by, in one pass over the fact table ("the entire query plan on the
// GPU, from scan to result", Section 3.1).
//
// Persistent workgroups walk fact tiles. Per tile every thread evaluates the
// predicate on four consecutive rows with coalesced vector loads of the
// predicate columns only. Passing rows are compacted per wave (ballot +
// mbcnt rank) into a small LDS queue; whenever 64 rows are queued the wave
// processes them with all 64 lanes busy: it gathers the remaining fact
// columns of its rows, probes each dim table (an LDS copy when the table is
// small, the HBM table otherwise) and aggregates into the workgroup's LDS
// group table, spilling keys that find no LDS slot to the global table.
// Compaction keeps lanes busy in the random-access phase whatever the
// selectivity, and columns other than the predicate's are only touched for
// passing rows. At the end the workgroup merges its LDS groups into the
// global table.

#include "group_lds.h"
#include "internal.h"

namespace rel {

namespace {

// Dim table access modes (template arguments).
constexpr int kDimNone = 0;
constexpr int kDimI32 = 1;     // int32 keys, HBM table
constexpr int kDimI32Lds = 2;  // int32 keys, LDS copy
constexpr int kDimI64 = 3;     // int64 keys, HBM table

template <int D>
__device__ __forceinline__ MapCursor dim_start(const PipeDim& d, int64_t key) {
  if constexpr (D == kDimI64) {
    Map64 m{nullptr, d.map.cap - 1, nullptr, nullptr};
    return map_start64(m, key);
  } else {
    Map32 m{nullptr, d.map.cap - 1, nullptr, nullptr};
    return map_start32(m, static_cast<int32_t>(key));
  }
}

template <int D>
__device__ __forceinline__ bool dim_next(const PipeDim& d, const uint64_t* lds_slots, int64_t key,
                                         MapCursor& c, uint32_t& val) {
  const uint64_t mask = d.map.cap - 1;
  if constexpr (D == kDimI64) {
    return map_next(static_cast<const ulonglong2*>(d.map.slots), mask, d.map.oob_count,
                    d.map.oob_vals, key, c, val);
  } else if constexpr (D == kDimI32Lds) {
    return map_next(lds_slots, mask, d.map.oob_count, d.map.oob_vals, static_cast<int32_t>(key), c,
                    val);
  } else {
    return map_next(static_cast<const uint64_t*>(d.map.slots), mask, d.map.oob_count,
                    d.map.oob_vals, static_cast<int32_t>(key), c, val);
  }
}

__device__ __forceinline__ void emit_group(const PipelineParams& p, const int64_t kf[2],
                                           uint32_t v0, uint32_t v1, const uint64_t* acc,
                                           uint64_t* lds_group, const GroupTable& gt) {
  int64_t k[2] = {0, 0};
  for (int j = 0; j < p.g.kp.nkeys; ++j) {
    const int src = p.key_src[j];
    k[j] = src == 0 ? kf[j] : static_cast<int64_t>(static_cast<int32_t>(src == 1 ? v0 : v1));
  }
  const uint64_t pk = pack_keys(p.g.kp, k[0], k[1]);
  uint64_t* ls = lds_group_slot(lds_group, p.lds_slots, p.g.words, pk);
  if (ls) {
    lds_group_update(ls, p.g.ap, acc);
  } else {
    uint64_t* gs = group_slot(gt, pk);
    if (gs) group_update_global(gs, p.g.ap, 1, acc);
  }
}

template <int D0, int D1>
__device__ __forceinline__ void process_row(const PipelineParams& p, int64_t r,
                                            const uint64_t* lds_dim0, const uint64_t* lds_dim1,
                                            uint64_t* lds_group, const GroupTable& gt) {
  int64_t kf[2] = {0, 0};
  for (int j = 0; j < p.g.kp.nkeys; ++j)
    if (p.key_src[j] == 0) kf[j] = load_elem(p.fact[p.key_col[j]], p.fact_type[p.key_col[j]], r);
  uint64_t acc[kMaxAcc];
  for (int a = 0; a < p.g.ap.nacc; ++a)
    acc[a] = static_cast<uint64_t>(load_elem(p.fact[p.acc_col[a]], p.fact_type[p.acc_col[a]], r));
  if constexpr (D0 == kDimNone) {
    emit_group(p, kf, 0, 0, acc, lds_group, gt);
  } else {
    const int64_t fk0 = load_elem(p.fact[p.dim[0].fk_col], p.fact_type[p.dim[0].fk_col], r);
    int64_t fk1 = 0;
    if constexpr (D1 != kDimNone)
      fk1 = load_elem(p.fact[p.dim[1].fk_col], p.fact_type[p.dim[1].fk_col], r);
    MapCursor c0 = dim_start<D0>(p.dim[0], fk0);
    uint32_t v0 = 0;
    while (dim_next<D0>(p.dim[0], lds_dim0, fk0, c0, v0)) {
      if constexpr (D1 == kDimNone) {
        emit_group(p, kf, v0, 0, acc, lds_group, gt);
      } else {
        MapCursor c1 = dim_start<D1>(p.dim[1], fk1);
        uint32_t v1 = 0;
        while (dim_next<D1>(p.dim[1], lds_dim1, fk1, c1, v1))
          emit_group(p, kf, v0, v1, acc, lds_group, gt);
      }
    }
  }
}

__device__ __forceinline__ uint32_t eval_rows(const PipelineParams& p, int64_t r0) {
  uint32_t bits = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) bits |= (r0 + e < p.n) ? (1u << e) : 0u;
  if (bits == 0) return 0;
  for (int t = 0; t < p.nterms; ++t) {
    const int c = p.term_col[t];
    int64_t v[4];
    load4(p.fact[c], p.fact_type[c], p.fact_vec[c] != 0, r0, p.n, v);
    uint32_t m = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      m |= term_holds(p.term_op[t], v[e], p.term_lo[t], p.term_hi[t]) ? (1u << e) : 0u;
    bits &= m;
  }
  return bits;
}

template <int D0, int D1>
__global__ void __launch_bounds__(kPipeThreads) pipeline_kernel(PipelineParams p) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  uint64_t* lds_dim0 = reinterpret_cast<uint64_t*>(lds + p.dim[0].lds_offset);
  uint64_t* lds_dim1 = reinterpret_cast<uint64_t*>(lds + p.dim[1].lds_offset);
  uint64_t* lds_group = reinterpret_cast<uint64_t*>(lds + p.lds_group_offset);
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = lane_id();
  uint32_t* queue = reinterpret_cast<uint32_t*>(lds + p.lds_queue_offset) + wave * kPipeQueue;

  if constexpr (D0 == kDimI32Lds) {
    const uint64_t* src = static_cast<const uint64_t*>(p.dim[0].map.slots);
    for (uint64_t i = tid; i < p.dim[0].map.cap; i += kPipeThreads) lds_dim0[i] = src[i];
  }
  if constexpr (D1 == kDimI32Lds) {
    const uint64_t* src = static_cast<const uint64_t*>(p.dim[1].map.slots);
    for (uint64_t i = tid; i < p.dim[1].map.cap; i += kPipeThreads) lds_dim1[i] = src[i];
  }
  if (p.lds_slots > 0) lds_group_init(lds_group, p.lds_slots, p.g);
  __syncthreads();

  const GroupTable gt{p.g.slots, p.g.cap - 1, p.g.words, p.g.overflow};
  uint32_t queued = 0;  // wave-uniform
  for (int64_t tile = blockIdx.x; tile < p.ntiles; tile += gridDim.x) {
    const int64_t base = tile * kPipeTile;
#pragma unroll
    for (int j = 0; j < kPipeChunks; ++j) {
      const int64_t r0 = base + j * (kPipeThreads * 4) + tid * 4;
      const uint32_t bits = eval_rows(p, r0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool pass = (bits >> e) & 1u;
        const uint64_t b = ballot(pass);
        if (b == 0) continue;
        if (pass) queue[queued + rank_below(b)] = static_cast<uint32_t>(r0 + e);
        queued += popc64(b);
        if (queued >= kWave) {
          __builtin_amdgcn_wave_barrier();
          const int64_t r = queue[queued - kWave + lane];
          __builtin_amdgcn_wave_barrier();
          queued -= kWave;
          process_row<D0, D1>(p, r, lds_dim0, lds_dim1, lds_group, gt);
        }
      }
    }
  }
  if (queued > 0) {
    __builtin_amdgcn_wave_barrier();
    if (static_cast<uint32_t>(lane) < queued)
      process_row<D0, D1>(p, queue[lane], lds_dim0, lds_dim1, lds_group, gt);
  }
  if (p.lds_slots > 0) {
    __syncthreads();
    lds_group_flush(lds_group, p.lds_slots, p.g);
  }
}

template <int D0, int D1>
void launch_variant(const PipelineParams& p, int grid, hipStream_t s) {
  auto k = pipeline_kernel<D0, D1>;
  static bool attr_set = false;
  if (!attr_set) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                        hipFuncAttributeMaxDynamicSharedMemorySize,
                        device_info().lds_per_block);
    attr_set = true;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(kPipeThreads), p.lds_bytes, s, p);
}

int dim_mode(const PipelineParams& p, int d) {
  if (d >= p.ndims) return kDimNone;
  if (p.dim[d].map.key_type == kI64) return kDimI64;
  return p.dim[d].in_lds ? kDimI32Lds : kDimI32;
}

template <int D0>
void launch_d1(const PipelineParams& p, int grid, hipStream_t s) {
  switch (dim_mode(p, 1)) {
    case kDimNone: launch_variant<D0, kDimNone>(p, grid, s); break;
    case kDimI32: launch_variant<D0, kDimI32>(p, grid, s); break;
    case kDimI32Lds: launch_variant<D0, kDimI32Lds>(p, grid, s); break;
    default: launch_variant<D0, kDimI64>(p, grid, s); break;
  }
}

}  // namespace

void launch_pipeline(const PipelineParams& p, int grid, hipStream_t s) {
  ProfileScope ps(kKPipeline, s);
  switch (dim_mode(p, 0)) {
    case kDimNone: launch_variant<kDimNone, kDimNone>(p, grid, s); break;
    case kDimI32: launch_d1<kDimI32>(p, grid, s); break;
    case kDimI32Lds: launch_d1<kDimI32Lds>(p, grid, s); break;
    default: launch_d1<kDimI64>(p, grid, s); break;
  }
}

}  // namespace rel
