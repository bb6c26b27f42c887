// Hopping stencil instantiations for one storage precision and one number of columns per
// thread.  The build compiles this file once per (BQ_INST_PREC, BQ_INST_R) pair, so that the
// variants compile in parallel; the host side dispatches on (prec, R) in launch_hop.
#include "bq_dslash_impl.h"

#if !defined(BQ_INST_PREC) || !defined(BQ_INST_R)
#error "compile with -DBQ_INST_PREC=<0|1|2> -DBQ_INST_R=<columns per thread>"
#endif

namespace bq {
#if BQ_INST_PREC == 0
using InstP = P64;
using InstPR = P64;
#elif BQ_INST_PREC == 1
using InstP = P32;
using InstPR = P32;
#else
using InstP = P16;  // FP16 storage keeps its residual in FP32
using InstPR = P32;
#endif
static_assert(BQ_INST_R >= 1 && BQ_INST_R <= dslash::max_R<InstP>(), "no such column count");

#define BQ_INST_NAME2(p, r) launch_hop_p##p##_r##r
#define BQ_INST_NAME(p, r) BQ_INST_NAME2(p, r)
hipError_t BQ_INST_NAME(BQ_INST_PREC, BQ_INST_R)(const HopLaunch& L, hipStream_t st)
{
    return dslash::by_dag<InstP, InstPR, BQ_INST_R>(L, st);
}
}  // namespace bq
