// Instantiations of the fused likelihood kernel: compiled mode set 3, mixed policy.
#include "k_lnl_impl.h"

namespace ile {
template hipError_t launch_eval_sp<3, 2>(int, bool, size_t, const EvalJob *, const Tile *, int,
                                           int, hipStream_t);
}  // namespace ile
