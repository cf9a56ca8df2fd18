// Streaming-read ceiling: every byte of a device buffer read exactly once,
// with nothing else to do. This is the achievable rate that a scan-bound
// operator is compared with beside the 8 TB/s HBM3E specification (the
// paper measures its engine on data resident in device memory, Section 4.1).
//
// Each thread reads 16-byte non-temporal vector loads, two in flight per
// step, from consecutive 16-byte slots of a grid-strided block, so that a
// wave reads 2 x 1 KB of contiguous lines per step. The loaded words are
// folded with XOR (so the loads cannot be dropped), combined per wave with a
// butterfly of lane swaps and per workgroup through LDS, and published with
// one device-scope atomic XOR per workgroup; the result is the XOR of every
// 64-bit word of the buffer (a tail shorter than 8 bytes is zero-padded),
// which a host can check.

#include "internal.h"

namespace rel {

namespace {

constexpr int kStreamThreads = 256;
constexpr int kStreamUnroll = 2;

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kStreamThreads)
stream_read_kernel(const v4u* __restrict__ p, uint64_t n16, const unsigned char* tail,
                   uint32_t tail_bytes, unsigned long long* out) {
  uint64_t acc = 0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kStreamThreads;
  uint64_t i = static_cast<uint64_t>(blockIdx.x) * kStreamThreads + threadIdx.x;
  // whole steps: kStreamUnroll loads per thread, each a grid-wide coalesced sweep
  for (; i + (kStreamUnroll - 1) * stride < n16; i += kStreamUnroll * stride) {
    v4u x[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) x[u] = __builtin_nontemporal_load(p + i + u * stride);
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u)
      acc ^= (static_cast<uint64_t>(x[u].y) << 32 | x[u].x) ^
             (static_cast<uint64_t>(x[u].w) << 32 | x[u].z);
  }
  for (; i < n16; i += stride) {
    const v4u x = __builtin_nontemporal_load(p + i);
    acc ^= (static_cast<uint64_t>(x.y) << 32 | x.x) ^ (static_cast<uint64_t>(x.w) << 32 | x.z);
  }
  // bytes past the last whole 16-byte slot, as zero-padded 64-bit words
  if (blockIdx.x == 0 && threadIdx.x < 2) {
    uint64_t w = 0;
    for (uint32_t b = 0; b < 8; ++b) {
      const uint32_t at = threadIdx.x * 8 + b;
      if (at < tail_bytes) w |= static_cast<uint64_t>(tail[at]) << (8 * b);
    }
    acc ^= w;
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const uint32_t lo = __shfl_xor(static_cast<uint32_t>(acc), off, kWave);
    const uint32_t hi = __shfl_xor(static_cast<uint32_t>(acc >> 32), off, kWave);
    acc ^= static_cast<uint64_t>(hi) << 32 | lo;
  }
  // one atomic per workgroup: same-address atomics serialise, and one per
  // wave of a large grid cost as much as the reads of a smaller column
  __shared__ uint64_t s_wave[kStreamThreads / kWave];
  if (lane_id() == 0) s_wave[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t x = 0;
#pragma unroll
    for (int w = 0; w < kStreamThreads / kWave; ++w) x ^= s_wave[w];
    atomicXor(out, static_cast<unsigned long long>(x));
  }
}

__global__ void stream_clear_kernel(unsigned long long* out) { *out = 0; }

}  // namespace

hipError_t launch_stream_read(const void* data, uint64_t bytes, unsigned long long* out,
                              hipStream_t s) {
  ProfileScope ps(kKStream, s);
  hipLaunchKernelGGL(stream_clear_kernel, dim3(1), dim3(1), 0, s, out);
  const uint64_t n16 = bytes / 16;
  const unsigned char* tail = static_cast<const unsigned char*>(data) + n16 * 16;
  const uint32_t tail_bytes = static_cast<uint32_t>(bytes - n16 * 16);
  // four workgroups of 256 threads per CU, two 16-byte loads in flight per
  // thread (measured on MI355X over a 4.8 GB buffer: 6.9 TB/s; 7.0-7.1 TB/s
  // took 8-16k workgroups, whose one atomic each would cost more than the
  // difference; plain instead of non-temporal loads: 4.7-5.2 TB/s)
  uint64_t blocks = static_cast<uint64_t>(device_info().cu_count) * 4;
  const uint64_t need = (n16 + kStreamThreads * kStreamUnroll - 1) / (kStreamThreads * kStreamUnroll);
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(stream_read_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kStreamThreads),
                     0, s, static_cast<const v4u*>(data), n16, tail, tail_bytes, out);
  return hipGetLastError();
}

}  // namespace rel
