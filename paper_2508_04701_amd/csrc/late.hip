// Late materialisation and order-by / top-N over result tables.
//
// The engine passes row ids between operators and materialises columns only
// at the end (Section 3.2.2 names materialisation among its custom kernels;
// Section 3.2.3 discusses the row-id type); the ClickBench discussion
// (Section 4.2) names order-by / top-N among the costs on top of scans and
// aggregation. Two kernels:
//
//  * gather: out_c[i] = col_c[ids[i]] for up to eight columns at once, each
//    thread taking four consecutive ids (one 16-byte load) so that the id
//    array is read once for all columns;
//
//  * top-N: the first N rows of a table in the order of one column
//    (ascending or descending), ties broken by the key tuple and then the row
//    position, so that the answer is unique. Every row becomes a composite
//    sort key (order word, key words, row) of order-preserving unsigned
//    integers. Phase one: each workgroup walks a contiguous range of rows
//    and keeps the P smallest keys seen so far (P: the power of two >= N, at
//    most 1024) as a sorted list in LDS. The list's last entry is a running
//    threshold: a row whose order word is above it cannot enter the list, so
//    most rows cost one 8-byte load and one compare; the others are appended
//    to a P-entry candidate buffer in LDS, which, when full (and once at the
//    end), is sorted (bitonic) and merged into the list (element-wise
//    minimum against the reversed list, bitonic merge), lowering the
//    threshold. Then rounds of merges, each workgroup folding up to
//    kTopFanIn sorted lists the same way (without the sort; a list whose
//    first entry does not beat the last one kept is skipped), until one
//    workgroup writes the first N row positions in order.

#include "internal.h"

namespace rel {

namespace {

// ------------------------------------------------------------------ gather

constexpr int kGatherThreads = 256;

__device__ __forceinline__ void store_any(void* p, int32_t type, int64_t i, int64_t v) {
  if (type == kI64) static_cast<int64_t*>(p)[i] = v;
  else if (type == kI32) static_cast<int32_t*>(p)[i] = static_cast<int32_t>(v);
  else static_cast<int8_t*>(p)[i] = static_cast<int8_t>(v);
}

__global__ void __launch_bounds__(kGatherThreads) gather_kernel(GatherParams p) {
  const uint64_t n = static_cast<uint64_t>(p.n);
  const uint64_t step = static_cast<uint64_t>(gridDim.x) * kGatherThreads * 4;
  for (uint64_t i0 = (static_cast<uint64_t>(blockIdx.x) * kGatherThreads + threadIdx.x) * 4; i0 < n;
       i0 += step) {
    uint32_t id[4];
    if (i0 + 4 <= n && p.ids_vec) {
      const uint4 v = *reinterpret_cast<const uint4*>(p.ids + i0);
      id[0] = v.x; id[1] = v.y; id[2] = v.z; id[3] = v.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) id[e] = i0 + e < n ? p.ids[i0 + e] : 0;
    }
    for (int c = 0; c < p.ncols; ++c) {
      int64_t v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = i0 + e < n ? load_elem(p.src[c], p.type[c], id[e]) : 0;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (i0 + e < n) store_any(p.dst[c], p.type[c], static_cast<int64_t>(i0 + e), v[e]);
    }
  }
}

// ------------------------------------------------------------------- top-N

constexpr int kTopThreads = 512;

// Order-preserving map of a signed value (or a binary64, for the order
// column) to an unsigned word.
__device__ __forceinline__ uint64_t sortable_i64(int64_t v) {
  return static_cast<uint64_t>(v) ^ 0x8000000000000000ULL;
}
__device__ __forceinline__ uint64_t sortable_f64(uint64_t bits) {
  if (bits == 0x8000000000000000ULL) bits = 0;  // -0.0 orders as 0.0
  return (bits & 0x8000000000000000ULL) ? ~bits : (bits | 0x8000000000000000ULL);
}

struct TopLds {
  uint64_t a[2 * kTopMax];
  uint64_t b[2 * kTopMax];
  uint64_t c[2 * kTopMax];
  uint32_t row[2 * kTopMax];
  int32_t cnt;  // candidates appended to [P, 2P) (may overshoot P)
};

__device__ __forceinline__ bool item_less(const TopLds& s, int i, int j) {
  if (s.a[i] != s.a[j]) return s.a[i] < s.a[j];
  if (s.b[i] != s.b[j]) return s.b[i] < s.b[j];
  if (s.c[i] != s.c[j]) return s.c[i] < s.c[j];
  return s.row[i] < s.row[j];
}

__device__ __forceinline__ void item_swap(TopLds& s, int i, int j) {
  uint64_t t = s.a[i]; s.a[i] = s.a[j]; s.a[j] = t;
  t = s.b[i]; s.b[i] = s.b[j]; s.b[j] = t;
  t = s.c[i]; s.c[i] = s.c[j]; s.c[j] = t;
  const uint32_t u = s.row[i]; s.row[i] = s.row[j]; s.row[j] = u;
}

// Bitonic steps over entries [base, base + P) that turn a bitonic sequence
// into an ascending one (merge), or sort them from scratch (sort).
__device__ __forceinline__ void bitonic_merge(TopLds& s, int base, int P) {
  for (int j = P / 2; j > 0; j >>= 1) {
    for (int t = threadIdx.x; t < P / 2; t += kTopThreads) {
      const int i = base + (t / j) * 2 * j + (t % j);
      if (item_less(s, i + j, i)) item_swap(s, i, i + j);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void bitonic_sort(TopLds& s, int base, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k / 2; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += kTopThreads) {
        const int i = base + (t / j) * 2 * j + (t % j);
        const bool up = (((i - base) & k) == 0);
        if (item_less(s, i + j, i) == up) item_swap(s, i, i + j);
      }
      __syncthreads();
    }
  }
}

// Entry i of the list holds the largest possible key when empty.
__device__ __forceinline__ void set_empty(TopLds& s, int i) {
  s.a[i] = ~0ULL;
  s.b[i] = ~0ULL;
  s.c[i] = ~0ULL;
  s.row[i] = 0xFFFFFFFFu;
}

// Merges the P entries at [P, 2P) (a chunk, sorted already when `sorted`)
// into the sorted list at [0, P): afterwards [0, P) holds the P smallest of
// both, sorted.
__device__ __forceinline__ void merge_chunk(TopLds& s, int P, bool sorted) {
  if (!sorted) bitonic_sort(s, P, P);
  // element-wise minimum of the list and the reversed chunk: a bitonic
  // sequence holding the P smallest entries of the two
  for (int i = threadIdx.x; i < P; i += kTopThreads) {
    const int j = 2 * P - 1 - i;
    if (item_less(s, j, i)) {
      s.a[i] = s.a[j];
      s.b[i] = s.b[j];
      s.c[i] = s.c[j];
      s.row[i] = s.row[j];
    }
  }
  __syncthreads();
  bitonic_merge(s, 0, P);
}

// Phase one: workgroup w takes rows [w * span, (w + 1) * span) and writes
// its P smallest keys (sorted) to the candidate buffers at w * P.
__global__ void __launch_bounds__(kTopThreads) topn_local_kernel(TopNParams p) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  TopLds& s = *reinterpret_cast<TopLds*>(lds_raw);
  const int P = p.pow2;
  const int64_t begin = static_cast<int64_t>(blockIdx.x) * p.span;
  int64_t end = begin + p.span;
  if (end > p.n) end = p.n;
  for (int i = threadIdx.x; i < P; i += kTopThreads) set_empty(s, i);
  if (threadIdx.x == 0) s.cnt = 0;
  __syncthreads();
  const uint64_t* ord = static_cast<const uint64_t*>(p.order);
  constexpr int kRows = 4;  // rows per thread and step, lane-strided (coalesced)
  for (int64_t c0 = begin; c0 < end; c0 += kTopThreads * kRows) {
    uint64_t a[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int64_t r = c0 + k * kTopThreads + threadIdx.x;
      a[k] = ~0ULL;
      if (r < end) {
        const uint64_t o = p.order_is_double ? sortable_f64(ord[r]) : sortable_i64(static_cast<int64_t>(ord[r]));
        a[k] = p.desc ? ~o : o;
      }
    }
    // rows whose order word does not exceed the threshold are candidates
    // (equal words are decided by the full key when merged)
    uint64_t thr = s.a[P - 1];
    uint32_t pend = 0;
#pragma unroll
    for (int k = 0; k < kRows; ++k)
      if (c0 + k * kTopThreads + threadIdx.x < end && a[k] <= thr) pend |= 1u << k;
    while (true) {
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        if (!((pend >> k) & 1u)) continue;
        const int pos = atomicAdd(&s.cnt, 1);
        if (pos >= P) break;  // buffer full: the rest waits for the merge
        const int64_t r = c0 + k * kTopThreads + threadIdx.x;
        const int e = P + pos;
        s.a[e] = a[k];
        s.b[e] = p.nkeys > 0 ? sortable_i64(load_elem(p.keys[0], p.key_type[0], r)) : 0;
        s.c[e] = p.nkeys > 1 ? sortable_i64(load_elem(p.keys[1], p.key_type[1], r)) : 0;
        s.row[e] = static_cast<uint32_t>(r);
        pend &= ~(1u << k);
      }
      __syncthreads();
      const int placed = s.cnt;
      // no thread may append for the next step before every thread has read
      // the count
      __syncthreads();
      if (placed < P) break;  // every candidate placed (block-uniform)
      merge_chunk(s, P, false);
      __syncthreads();
      if (threadIdx.x == 0) s.cnt = 0;
      thr = s.a[P - 1];
#pragma unroll
      for (int k = 0; k < kRows; ++k)
        if (a[k] > thr) pend &= ~(1u << k);
      __syncthreads();
    }
  }
  // the partly filled buffer
  const int left = s.cnt;
  if (left > 0) {
    for (int i = left + threadIdx.x; i < P; i += kTopThreads) set_empty(s, P + i);
    __syncthreads();
    merge_chunk(s, P, false);
  }
  __syncthreads();
  const int64_t out = static_cast<int64_t>(blockIdx.x) * P;
  const TopBuf& dst = p.buf[0];
  for (int i = threadIdx.x; i < P; i += kTopThreads) {
    dst.a[out + i] = s.a[i];
    dst.b[out + i] = s.b[i];
    dst.c[out + i] = s.c[i];
    dst.row[out + i] = s.row[i];
  }
}

// Merge rounds: workgroup w merges the sorted lists [w * per, (w + 1) * per)
// of buffer `src` (nsrc lists of P entries) into one, written to list w of
// buffer `dst`; the last round (one workgroup) writes the first min(N, n)
// row positions in order instead.
__global__ void __launch_bounds__(kTopThreads) topn_merge_kernel(TopNParams p, int src, int nsrc,
                                                                 int per, int last) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  TopLds& s = *reinterpret_cast<TopLds*>(lds_raw);
  const int P = p.pow2;
  const TopBuf& in = p.buf[src];
  const TopBuf& outb = p.buf[src ^ 1];
  for (int i = threadIdx.x; i < P; i += kTopThreads) set_empty(s, i);
  __syncthreads();
  int first = static_cast<int>(blockIdx.x) * per;
  int stop = first + per < nsrc ? first + per : nsrc;
  for (int l = first; l < stop; ++l) {
    const int64_t c0 = static_cast<int64_t>(l) * P;
    for (int i = threadIdx.x; i < P; i += kTopThreads) {
      const int k = P + i;
      s.a[k] = in.a[c0 + i];
      s.b[k] = in.b[c0 + i];
      s.c[k] = in.c[c0 + i];
      s.row[k] = in.row[c0 + i];
    }
    __syncthreads();
    // a sorted list whose first entry does not beat the last kept one
    // brings nothing
    if (item_less(s, P, P - 1)) merge_chunk(s, P, true);
    __syncthreads();
  }
  if (last) {
    const int64_t m = p.limit < p.n ? p.limit : p.n;
    for (int i = threadIdx.x; i < m; i += kTopThreads) p.out[i] = s.row[i];
    if (threadIdx.x == 0) *p.d_count = m;
    return;
  }
  const int64_t o = static_cast<int64_t>(blockIdx.x) * P;
  for (int i = threadIdx.x; i < P; i += kTopThreads) {
    outb.a[o + i] = s.a[i];
    outb.b[o + i] = s.b[i];
    outb.c[o + i] = s.c[i];
    outb.row[o + i] = s.row[i];
  }
}

}  // namespace

void launch_gather(const GatherParams& p, hipStream_t s) {
  ProfileScope ps(kKGather, s);
  if (p.n <= 0 || p.ncols == 0) return;
  uint64_t blocks = (static_cast<uint64_t>(p.n) + kGatherThreads * 4 - 1) / (kGatherThreads * 4);
  const uint64_t limit = static_cast<uint64_t>(device_info().cu_count) * 16;
  if (blocks > limit) blocks = limit;
  hipLaunchKernelGGL(gather_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kGatherThreads), 0,
                     s, p);
}

hipError_t launch_topn(const TopNParams& p, hipStream_t s) {
  ProfileScope ps(kKTopN, s);
  static bool attr = false;
  const size_t lds = sizeof(TopLds);
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(topn_local_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e == hipSuccess)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(topn_merge_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    attr = true;
  }
  // rows -> nlists sorted lists in buffer 0, then rounds of up to
  // kTopFanIn lists per workgroup until one workgroup writes the answer
  int src = 0, nsrc = p.nlists;
  if (nsrc > 0)
    hipLaunchKernelGGL(topn_local_kernel, dim3(static_cast<unsigned>(nsrc)), dim3(kTopThreads), lds,
                       s, p);
  while (true) {
    const int per = nsrc > kTopFanIn ? kTopFanIn : (nsrc > 0 ? nsrc : 1);
    const int groups = nsrc > 0 ? (nsrc + per - 1) / per : 1;
    const int last = groups == 1 ? 1 : 0;
    hipLaunchKernelGGL(topn_merge_kernel, dim3(static_cast<unsigned>(groups)), dim3(kTopThreads),
                       lds, s, p, src, nsrc, per, last);
    if (last) break;
    src ^= 1;
    nsrc = groups;
  }
  return hipGetLastError();
}

}  // namespace rel
