// Launch dispatch of the fused pipeline kernel (pipeline_kernel.h).
//
// The kernel is a template over the access mode of each dim table. This file
// is compiled once per first-dim mode with REL_PIPE_D0=<mode> (instantiating
// every second-dim mode for it) and once without, which yields the
// dispatcher; the split lets the variants compile in parallel.

#include "pipeline_kernel.h"

namespace rel {
namespace pipe {

#define REL_FOR_EACH_D1(M, D0) \
  M(D0, kNone) M(D0, kMap) M(D0, kMapLds) M(D0, kSet) M(D0, kSetLds) M(D0, kMap64) M(D0, kCSet)

#if defined(REL_PIPE_D0)

#define REL_INSTANTIATE(A, B) template hipError_t launch_fused<A, B>(const PipelineParams&, int, hipStream_t);
REL_FOR_EACH_D1(REL_INSTANTIATE, REL_PIPE_D0)

#else

#define REL_DECLARE(A, B) extern template hipError_t launch_fused<A, B>(const PipelineParams&, int, hipStream_t);
REL_FOR_EACH_D1(REL_DECLARE, kMap)
REL_FOR_EACH_D1(REL_DECLARE, kMapLds)
REL_FOR_EACH_D1(REL_DECLARE, kSet)
REL_FOR_EACH_D1(REL_DECLARE, kSetLds)
REL_FOR_EACH_D1(REL_DECLARE, kMap64)
REL_FOR_EACH_D1(REL_DECLARE, kCSet)

namespace {

int dim_mode(const PipelineParams& p, int d) {
  if (d >= p.ndims) return kNone;
  const PipeDim& dm = p.dim[d];
  if (dm.map.key_type == kI64) return kMap64;
  if (dm.map.compact) return kCSet;
  if (dm.map.key_only) return dm.in_lds ? kSetLds : kSet;
  return dm.in_lds ? kMapLds : kMap;
}

template <int D0>
hipError_t launch_second(const PipelineParams& p, int grid, hipStream_t s) {
  switch (dim_mode(p, 1)) {
    case kNone: return launch_fused<D0, kNone>(p, grid, s);
    case kMap: return launch_fused<D0, kMap>(p, grid, s);
    case kMapLds: return launch_fused<D0, kMapLds>(p, grid, s);
    case kSet: return launch_fused<D0, kSet>(p, grid, s);
    case kSetLds: return launch_fused<D0, kSetLds>(p, grid, s);
    case kCSet: return launch_fused<D0, kCSet>(p, grid, s);
    default: return launch_fused<D0, kMap64>(p, grid, s);
  }
}

}  // namespace

}  // namespace pipe

hipError_t launch_pipeline(const PipelineParams& p, int grid, hipStream_t s) {
  using namespace pipe;
  ProfileScope ps(kKPipeline, s);
  switch (dim_mode(p, 0)) {
    case kNone: return launch_fused<kNone, kNone>(p, grid, s);
    case kMap: return launch_second<kMap>(p, grid, s);
    case kMapLds: return launch_second<kMapLds>(p, grid, s);
    case kSet: return launch_second<kSet>(p, grid, s);
    case kSetLds: return launch_second<kSetLds>(p, grid, s);
    case kCSet: return launch_second<kCSet>(p, grid, s);
    default: return launch_second<kMap64>(p, grid, s);
  }
}

namespace pipe {

#endif

}  // namespace pipe
}  // namespace rel
