// Instantiations of the likelihood kernel of the FP32 + FP64-cancellation policy: compiled mode set 2.
#include "k_lnl_ref_impl.h"

namespace ile {
template hipError_t launch_ref_sp<2>(int, size_t, const EvalJob *, const Tile *, int, int, hipStream_t);
}  // namespace ile
