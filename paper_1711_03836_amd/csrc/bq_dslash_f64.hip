// Hopping stencil instantiations for P64 storage (residual in P64).
#include "bq_dslash_impl.h"

namespace bq {
hipError_t launch_hop_f64(const HopLaunch& L, hipStream_t st) { return dslash::by_R<P64, P64>(L, st); }
}  // namespace bq
