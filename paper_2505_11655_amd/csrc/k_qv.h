// The decimated route for Q of eq. (QUV) (k_qv.hip); the direct route's
// launcher is declared with the other kernels.
#pragma once
#include <cstdint>
#include <hip/hip_runtime.h>

namespace ile {

// The radix R of the decimated route for a grid of n bins, a band of n_band
// bins and the window (n_time, win_half): of the R in {2, 4, 8, 16} that
// divide n and put the window on at most 64 decimated times
// floor((i - win_half) / R) (one 32- or 64-row time tile), the one of lowest
// estimated cost, or 0 when there is none.  With `force` false it is also 0
// when that cost exceeds the direct sum's.
int qv_radix(int64_t n, int64_t n_band, int n_time, int win_half, bool force);

// Band slices of the decimated route's matrix-core stage and its scratch
// (twiddles, band list, the radix-R partial sums and the slice partials,
// each 256-byte aligned).
int qv_dec_slices(int64_t n, int64_t cols, int n_time, int win_half, int radix);
size_t qv_dec_scratch_bytes(int64_t n, int64_t n_band, int64_t cols, int n_time, int win_half, int radix,
                            int n_slices);

// Q (decimated route), U and V.  The band is f_lo <= |m' df| <= f_hi (m' the
// signed index), tested on the device with the host's expression; h_band:
// host list of its grid indices (pinned, so the upload is asynchronous).
hipError_t launch_qv_dec(const void *hlm, const void *data, const double *inv_psd, int64_t n, int na, int nd,
                         int np, double df, double f_lo, double f_hi, const int64_t *h_band, int64_t n_band,
                         int n_time, int win_half, int radix, void *Q, void *U, void *V, void *scratch,
                         int n_slices, hipStream_t st);

}  // namespace ile
