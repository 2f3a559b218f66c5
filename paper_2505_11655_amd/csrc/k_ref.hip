// Reference terms of the FP32 + FP64-cancellation policy: the builder for
// every compiled mode set, and the reference point taken from a mixture.
#include "k_lnl_ref_impl.h"

namespace ile {

// theta_ref = mean of the heaviest component; columns outside the mixture
// take the middle of their prior range.  One thread.
__global__ void k_ref_from_gmm(const GmmDev *__restrict__ g, const PriorDev pr, double *theta_ref) {
    if (threadIdx.x != 0) return;
    const double mid[7] = {3.141592653589793, 0.0, 0.0, 0.5 * (pr.d_min + pr.d_max), 0.0, 3.141592653589793,
                           1.5707963267948966};
    double t[7];
    for (int c = 0; c < 7; c++) t[c] = mid[c];
    int jb = -1;
    double wb = -1.0;
    if (g->valid)
        for (int j = 0; j < g->n_comp; j++)
            if (g->w[j] > wb) {
                wb = g->w[j];
                jb = j;
            }
    if (jb >= 0) {
        for (int a = 0; a < g->n_dim; a++) t[g->dims[a]] = g->mean[jb][a];
        if (g->shear) t[6] = shear_phase(t[6], t[5], -g->shear);   // mean in the sheared phases
    }
    for (int c = 0; c < 7; c++) theta_ref[c] = t[c];
}

hipError_t launch_ref_from_gmm(const GmmDev *g, PriorDev pr, double *theta_ref, hipStream_t st) {
    hipLaunchKernelGGL(k_ref_from_gmm, dim3(1), dim3(64), 0, st, g, pr, theta_ref);
    return hipGetLastError();
}

hipError_t launch_ref_build(int set, int kdet, const EvalJob &job, const RefBuild &rb, hipStream_t st) {
    switch (set) {
        case 0: return launch_ref_build_sp<0>(kdet, job, rb, st);
        case 1: return launch_ref_build_sp<1>(kdet, job, rb, st);
        case 2: return launch_ref_build_sp<2>(kdet, job, rb, st);
        case 3: return launch_ref_build_sp<3>(kdet, job, rb, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ile
