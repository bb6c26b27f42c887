// Hopping stencil instantiations for P16 storage (residual in P32).
#include "bq_dslash_impl.h"

namespace bq {
hipError_t launch_hop_f16(const HopLaunch& L, hipStream_t st) { return dslash::by_R<P16, P32>(L, st); }
}  // namespace bq
