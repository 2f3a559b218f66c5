// Instantiations of the fused likelihood kernels (pointwise and time-marginalised): compiled mode set 2, FP32 policy.
#include "k_lnl_impl.h"
#include "k_tmarg_impl.h"

namespace ile {
template hipError_t launch_eval_sp<2, 1>(int, bool, size_t, const EvalJob *, const Tile *, int,
                                           int, hipStream_t);
template hipError_t launch_tmarg_sp<2, 1>(int, int, bool, size_t, const EvalJob *, const Tile *, int,
                                             int, hipStream_t);
}  // namespace ile
