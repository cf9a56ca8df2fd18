// Launch dispatch of the batched fused pass (pipeline_kernel.h).
//
// Batched plans read every dim table from HBM, so the variants are the HBM
// access modes only. As for the single-plan kernel, this file is compiled
// once per first-dim mode with REL_BATCH_D0=<mode> and once without, which
// yields the dispatcher.

#include "pipeline_kernel.h"

namespace rel {
namespace pipe {

#define REL_BATCH_D1(M, D0) M(D0, kNone) M(D0, kMap) M(D0, kSet) M(D0, kMap64)

#if defined(REL_BATCH_D0)

#define REL_INSTANTIATE(A, B) template hipError_t launch_batch_fused<A, B>(const BatchParams&, int, hipStream_t);
#if REL_BATCH_D0 == 0
REL_INSTANTIATE(kNone, kNone)
#else
REL_BATCH_D1(REL_INSTANTIATE, REL_BATCH_D0)
#endif

#else

#define REL_DECLARE(A, B) extern template hipError_t launch_batch_fused<A, B>(const BatchParams&, int, hipStream_t);
REL_DECLARE(kNone, kNone)
REL_BATCH_D1(REL_DECLARE, kMap)
REL_BATCH_D1(REL_DECLARE, kSet)
REL_BATCH_D1(REL_DECLARE, kMap64)

namespace {

int batch_mode(const PipelineParams& p, int d) {
  if (d >= p.ndims) return kNone;
  const MapDesc& m = p.dim[d].map;
  if (m.key_type == kI64) return kMap64;
  return m.key_only ? kSet : kMap;
}

template <int D0>
hipError_t batch_second(const BatchParams& b, const PipelineParams& shape, int grid,
                        hipStream_t s) {
  switch (batch_mode(shape, 1)) {
    case kNone: return launch_batch_fused<D0, kNone>(b, grid, s);
    case kMap: return launch_batch_fused<D0, kMap>(b, grid, s);
    case kSet: return launch_batch_fused<D0, kSet>(b, grid, s);
    default: return launch_batch_fused<D0, kMap64>(b, grid, s);
  }
}

}  // namespace

}  // namespace pipe

hipError_t launch_batch_pipeline(const BatchParams& b, const PipelineParams& shape, int grid,
                                 hipStream_t s) {
  using namespace pipe;
  ProfileScope ps(kKPipeline, s);
  switch (batch_mode(shape, 0)) {
    case kNone: return launch_batch_fused<kNone, kNone>(b, grid, s);
    case kMap: return batch_second<kMap>(b, shape, grid, s);
    case kSet: return batch_second<kSet>(b, shape, grid, s);
    default: return batch_second<kMap64>(b, shape, grid, s);
  }
}

namespace pipe {

#endif

}  // namespace pipe
}  // namespace rel
