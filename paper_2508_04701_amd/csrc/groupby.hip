// Hash group-by aggregation.
//
// Every workgroup keeps a private open-addressing group table in LDS (when
// lds_slots > 0): a row whose key finds or claims an LDS slot within a short
// probe window is aggregated there with LDS atomics, so few-group inputs
// never touch HBM per row (the few-groups memory contention named in
// Section 4.2). Rows whose key does not fit go straight to the global table
// in HBM (CAS on the packed key, then device-scope atomics on COUNT and the
// accumulators). At the end the workgroup merges its LDS table into the
// global one with one update per occupied slot. With many groups the LDS
// table still absorbs the keys a workgroup meets first, which under skew are
// the hot ones. A finalize pass compacts occupied global slots into the
// output columns with a ballot and one atomic per wave.

#include "internal.h"
#include "group_lds.h"

namespace rel {

namespace {

__global__ void group_init_kernel(GroupDesc g) {
  const uint64_t total = g.replicas * (g.cap + 1) * static_cast<uint64_t>(g.words);
  const uint64_t first = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  const uint32_t words = static_cast<uint32_t>(g.words);
  // word index within the slot, stepped by the stride mod words
  uint32_t w = static_cast<uint32_t>(first % words);
  const uint32_t step = static_cast<uint32_t>(stride % words);
  for (uint64_t i = first; i < total; i += stride) {
    uint64_t v = 0;
    if (w == 0) v = kEmpty64;
    else if (w >= 2 && static_cast<int>(w) - 2 < g.ap.nacc) v = acc_identity(g.ap.kind[w - 2]);
    g.slots[i] = v;
    w += step;
    if (w >= words) w -= words;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *g.overflow = 0;
    *g.d_groups = 0;
  }
}

__global__ void __launch_bounds__(256) group_agg_kernel(GroupAggParams p) {
  extern __shared__ uint64_t lds_table[];
  const GroupDesc& g = p.g;
  const GroupTable gt = group_replica(g, blockIdx.x % g.replicas);
  if (p.lds_slots > 0) {
    lds_group_init(lds_table, p.lds_slots, g);
    __syncthreads();
  }
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
       i < static_cast<uint64_t>(p.n); i += stride) {
    int64_t k[2] = {0, 0};
    for (int j = 0; j < g.kp.nkeys; ++j) {
      int64_t r = p.key_idx[j] ? static_cast<int64_t>(p.key_idx[j][i]) : static_cast<int64_t>(i);
      k[j] = load_elem(p.key_data[j], g.kp.type[j], r);
    }
    const uint64_t pk = pack_keys(g.kp, k[0], k[1]);
    uint64_t acc[kMaxAcc];
    for (int a = 0; a < g.ap.nacc; ++a) {
      int64_t r = p.val_idx[a] ? static_cast<int64_t>(p.val_idx[a][i]) : static_cast<int64_t>(i);
      acc[a] = static_cast<uint64_t>(load_elem(p.val_data[a], p.val_type[a], r));
    }
    uint64_t* ls = lds_group_slot(lds_table, p.lds_slots, g.words, pk);
    if (ls) {
      lds_group_update(ls, g.ap, acc);
    } else {
      uint64_t* gs = group_slot(gt, pk);
      if (gs) group_update_global(gs, g.ap, 1, acc);
    }
  }
  if (p.lds_slots > 0) {
    __syncthreads();
    lds_group_flush(lds_table, p.lds_slots, g);
  }
}

// Folds entries i, i + stride, ... below `end` of replicas 1.. (numbered
// from the start of replica 1) into replica 0.
__device__ __forceinline__ void merge_range(const GroupDesc& g, uint64_t i, uint64_t end,
                                            uint64_t stride) {
  const uint64_t per = g.cap + 1;
  const GroupTable dst = group_replica(g, 0);
  for (; i < end; i += stride) {
    const uint64_t r = 1 + i / per, slot = i % per;
    const uint64_t* s = g.slots + (r * per + slot) * g.words;
    const bool oob = slot == g.cap;
    if (oob ? s[1] == 0 : s[0] == kEmpty64) continue;
    uint64_t* d = group_slot(dst, oob ? kEmpty64 : s[0]);
    if (d) group_update_global(d, g.ap, s[1], s + 2);
  }
}

__global__ void __launch_bounds__(256) group_merge_kernel(GroupDesc g) {
  merge_range(g, blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x,
              (g.replicas - 1) * (g.cap + 1), static_cast<uint64_t>(gridDim.x) * blockDim.x);
}

// Slots per thread in one finalize chunk (a chunk spans blockDim.x times as
// many slots).
constexpr int kFinalizeSlots = 8;

__device__ __forceinline__ void write_group(const FinalizeParams& p, uint64_t i,
                                            unsigned long long pos) {
  const GroupDesc& g = p.g;
  if (pos >= static_cast<unsigned long long>(p.cap)) return;
  const uint64_t* s = g.slots + i * g.words;
  const uint64_t pk = (g.kp.nkeys > 0 && i == g.cap) ? kEmpty64 : s[0];
  if (g.kp.nkeys > 0) {
    int64_t k0, k1;
    unpack_keys(g.kp, pk, k0, k1);
    store_elem(p.out_keys[0], p.out_key_type[0], pos, k0);
    if (g.kp.nkeys > 1) store_elem(p.out_keys[1], p.out_key_type[1], pos, k1);
  }
  const uint64_t count = s[1];
  for (int a = 0; a < p.naggs; ++a) {
    const int op = p.op[a];
    int64_t* out = static_cast<int64_t*>(p.out_aggs[a]);
    if (op == 1) {
      out[pos] = static_cast<int64_t>(count);
    } else if (op == 4) {
      double avg;
      if (count == 0) {
        avg = __longlong_as_double(0x7FF8000000000000LL);
      } else {
        avg = static_cast<double>(static_cast<int64_t>(s[2 + p.acc[a]])) /
              static_cast<double>(static_cast<int64_t>(count));
      }
      static_cast<double*>(p.out_aggs[a])[pos] = avg;
    } else {
      out[pos] = static_cast<int64_t>(s[2 + p.acc[a]]);
    }
  }
}

// Writes the occupied slots of the chunks starting at `chunk`, `chunk +
// stride`, ... below `end` (all uniform across the workgroup). Per chunk the
// workgroup counts its occupied slots, takes their output positions with one
// atomic on the group counter, then writes them: one atomic per chunk rather
// than per wave, since every workgroup shares the counter.
__device__ __forceinline__ void finalize_range(const FinalizeParams& p, uint64_t chunk,
                                               uint64_t end, uint64_t stride) {
  __shared__ uint32_t s_wave[1024 / kWave];
  __shared__ unsigned long long s_base;
  const GroupDesc& g = p.g;
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;
  const uint64_t nslots = g.kp.nkeys == 0 ? 1 : g.cap + 1;
  if (end > nslots) end = nslots;
  for (; chunk < end; chunk += stride) {
    // the key words (COUNT for the out-of-band slot) of the thread's slots,
    // loaded together; slots past the end read the chunk's first slot
    uint64_t word[kFinalizeSlots];
#pragma unroll
    for (int j = 0; j < kFinalizeSlots; ++j) {
      uint64_t i = chunk + static_cast<uint64_t>(j) * blockDim.x + threadIdx.x;
      i = i < end ? i : chunk;
      word[j] = g.slots[i * g.words + (i < g.cap ? 0 : 1)];
    }
    uint32_t occ = 0;
#pragma unroll
    for (int j = 0; j < kFinalizeSlots; ++j) {
      const uint64_t i = chunk + static_cast<uint64_t>(j) * blockDim.x + threadIdx.x;
      if (i >= end) continue;
      bool o;
      if (g.kp.nkeys == 0) o = true;                 // the one ungrouped row
      else if (i < g.cap) o = (word[j] != kEmpty64);
      else o = (word[j] != 0);                       // out-of-band slot
      occ |= o ? (1u << j) : 0u;
    }
    const uint32_t c = __popc(occ);
    uint32_t incl = c;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t t = __shfl_up(incl, off, kWave);
      if (lane >= off) incl += t;
    }
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < nwaves; ++w) {
      if (w < wave) before += s_wave[w];
      total += s_wave[w];
    }
    if (threadIdx.x == 0)
      s_base = total ? atomicAdd(g.d_groups, static_cast<unsigned long long>(total)) : 0ULL;
    __syncthreads();
    unsigned long long pos = s_base + before + incl - c;
#pragma unroll
    for (int j = 0; j < kFinalizeSlots; ++j)
      if ((occ >> j) & 1u)
        write_group(p, chunk + static_cast<uint64_t>(j) * blockDim.x + threadIdx.x, pos++);
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) group_finalize_kernel(FinalizeParams p) {
  if (*p.g.overflow) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p.g.d_groups = static_cast<unsigned long long>(-1LL);
    return;
  }
  const uint64_t span = static_cast<uint64_t>(blockDim.x) * kFinalizeSlots;
  finalize_range(p, blockIdx.x * span, ~0ULL, static_cast<uint64_t>(gridDim.x) * span);
}

// One workgroup per item of the batch's merge and finalize lists.
__global__ void __launch_bounds__(256) batch_merge_kernel(BatchParams b) {
  const BatchItem& it = batch_at(b.merge_items, blockIdx.x);
  merge_range(batch_at(b.plans, it.inst).g, it.begin + threadIdx.x, it.end, blockDim.x);
}

__global__ void __launch_bounds__(256) batch_finalize_kernel(BatchParams b) {
  const BatchItem& it = batch_at(b.fin_items, blockIdx.x);
  const FinalizeParams& p = batch_at(b.fins, it.inst);
  if (*p.g.overflow) {
    if (it.begin == 0 && threadIdx.x == 0) *p.g.d_groups = static_cast<unsigned long long>(-1LL);
    return;
  }
  finalize_range(p, it.begin, it.end, static_cast<uint64_t>(blockDim.x) * kFinalizeSlots);
}

}  // namespace

void launch_group_init(const GroupDesc& g, hipStream_t s) {
  ProfileScope ps(kKFill, s);
  uint64_t total = g.replicas * (g.cap + 1) * static_cast<uint64_t>(g.words);
  uint64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(group_init_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, g);
}

void launch_group_agg(const GroupAggParams& p, int grid, int block, hipStream_t s) {
  ProfileScope ps(kKGroupAgg, s);
  size_t lds = static_cast<size_t>(p.lds_slots) * p.g.words * sizeof(uint64_t);
  hipLaunchKernelGGL(group_agg_kernel, dim3(grid), dim3(block), lds, s, p);
}

void launch_group_merge(const GroupDesc& g, hipStream_t s) {
  if (g.replicas <= 1) return;
  ProfileScope ps(kKFinalize, s);
  uint64_t total = (g.replicas - 1) * (g.cap + 1);
  uint64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(group_merge_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, g);
}

void launch_group_finalize(const FinalizeParams& p, hipStream_t s) {
  ProfileScope ps(kKFinalize, s);
  uint64_t nslots = p.g.kp.nkeys == 0 ? 1 : p.g.cap + 1;
  uint64_t blocks = (nslots + 256 * kFinalizeSlots - 1) / (256 * kFinalizeSlots);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(group_finalize_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                     p);
}

void launch_batch_merge(const BatchParams& b, hipStream_t s) {
  if (b.nmerge == 0) return;
  ProfileScope ps(kKFinalize, s);
  hipLaunchKernelGGL(batch_merge_kernel, dim3(b.nmerge), dim3(256), 0, s, b);
}

void launch_batch_finalize(const BatchParams& b, hipStream_t s) {
  if (b.nfin == 0) return;
  ProfileScope ps(kKFinalize, s);
  hipLaunchKernelGGL(batch_finalize_kernel, dim3(b.nfin), dim3(256), 0, s, b);
}

}  // namespace rel
