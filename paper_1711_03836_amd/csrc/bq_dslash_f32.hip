// Hopping stencil instantiations for P32 storage (residual in P32).
#include "bq_dslash_impl.h"

namespace bq {
hipError_t launch_hop_f32(const HopLaunch& L, hipStream_t st) { return dslash::by_R<P32, P32>(L, st); }
}  // namespace bq
