// Instantiations of the fused likelihood kernels (pointwise and time-marginalised): compiled mode set 0, FP64 policy.
#include "k_lnl_impl.h"
#include "k_tmarg_impl.h"

namespace ile {
template hipError_t launch_eval_sp<0, 0>(int, bool, size_t, const EvalJob *, const Tile *, int,
                                           int, hipStream_t);
template hipError_t launch_tmarg_sp<0, 0>(int, int, bool, size_t, const EvalJob *, const Tile *, int,
                                             int, hipStream_t);
}  // namespace ile
