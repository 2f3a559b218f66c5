// Host-side state behind the opaque handles of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ile.h"
#include "ile_internal.h"

struct ile_ctx {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;
    std::atomic<bool> sticky{false};
    std::mutex mu;                        // budget accounting and the pools below
    // device and pinned-host buffers recycled by power-of-two size class; a
    // buffer goes back to its pool only when no queued work can still use it
    std::map<size_t, std::vector<void *>> dev_pool, pin_pool;
    size_t pool_cached = 0;
    struct DistEntry {
        ile::DistTable tab;
        void *buf;
    };
    std::mutex dist_mu;
    std::map<std::tuple<double, double, double>, DistEntry> dist;
    // batched-launch descriptors: a ring of device scratch slots with pinned
    // staging; a slot is reused only after the kernel that read it finished.
    struct Slot {
        void *d = nullptr;
        void *h = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool armed = false;
    };
    static constexpr int kSlots = 8;
    std::mutex batch_mu;
    Slot slots[kSlots];
    int next_slot = 0;
};

struct ile_job {
    ile_ctx *ctx = nullptr;
    int policy = 0, set = 0, kp = 2, n_det = 1, n_time = 0, n_kept = 0;
    bool dist_marg = false;
    ile::PriorDev pr{};
    // resident inputs: one device blob [Q | U table | V table | estimator state]
    void *d_blob = nullptr, *h_blob = nullptr;   // h_blob: pinned staging of the upload
    size_t blob_bytes = 0;
    void *d_Q = nullptr, *d_Ut = nullptr, *d_Vt = nullptr;
    size_t q_bytes = 0, uv_bytes = 0, device_bytes = 0;
    ile::EvalJob ej{};
    ile::MargState *d_ms = nullptr;
    ile::MargState *h_ms = nullptr;       // pinned
    ile::MargPartial *d_part = nullptr;
    size_t part_cap = 0;
    ile::GmmDev *d_gmm = nullptr;
    ile::GmmDev *h_gmm = nullptr;         // pinned
    uint32_t *d_zcount = nullptr;
    bool has_prop = false;
    double *d_em = nullptr;
    size_t em_cap = 0;
    // adaptive-volume grid and update workspace (one allocation, made on
    // first use and grown with the largest update)
    ile::AvBufs av{};
    void *av_mem = nullptr;
    size_t av_bytes = 0;
    int64_t av_cap = 0;
    ile::AvDev *h_av = nullptr;           // pinned readback
    // adaptive Cartesian marginals (allocated on first use)
    ile::AcDev *d_ac = nullptr;
    // fair-draw scratch (prefix sums of the sample masses), grown as needed
    void *fair_mem = nullptr;
    size_t fair_cap = 0;
    // FP32 + FP64-cancellation policy: the FP64 window and overlaps its
    // reference terms are built from, and where those terms live (all in the
    // job's blob); pinned staging of a reference point set from the host
    ile::RefBuild rb{};
    double *h_ref = nullptr;
};

namespace ile {

template <int S, int POL>
hipError_t launch_eval_sp(int kdet, bool dm, size_t lds_bytes, const EvalJob *jobs, const Tile *tiles,
                          int n_tiles, int nthreads, hipStream_t st);
extern template hipError_t launch_eval_sp<0, 0>(int, bool, size_t, const EvalJob *, const Tile *, int,
                                                   int, hipStream_t);
extern template hipError_t launch_eval_sp<0, 1>(int, bool, size_t, const EvalJob *, const Tile *, int,
                                                   int, hipStream_t);
extern template hipError_t launch_eval_sp<1, 0>(int, bool, size_t, const EvalJob *, const Tile *, int,
                                                   int, hipStream_t);
extern template hipError_t launch_eval_sp<1, 1>(int, bool, size_t, const EvalJob *, const Tile *, int,
                                                   int, hipStream_t);
extern template hipError_t launch_eval_sp<2, 0>(int, bool, size_t, const EvalJob *, const Tile *, int,
                                                   int, hipStream_t);
extern template hipError_t launch_eval_sp<2, 1>(int, bool, size_t, const EvalJob *, const Tile *, int,
                                                   int, hipStream_t);
extern template hipError_t launch_eval_sp<3, 0>(int, bool, size_t, const EvalJob *, const Tile *, int,
                                                   int, hipStream_t);
extern template hipError_t launch_eval_sp<3, 1>(int, bool, size_t, const EvalJob *, const Tile *, int,
                                                   int, hipStream_t);

// The FP32 + FP64-cancellation policy's kernel (reference-subtracted form).
template <int S>
hipError_t launch_ref_sp(int kdet, size_t lds_bytes, const EvalJob *jobs, const Tile *tiles, int n_tiles,
                         int nthreads, hipStream_t st);
extern template hipError_t launch_ref_sp<0>(int, size_t, const EvalJob *, const Tile *, int, int, hipStream_t);
extern template hipError_t launch_ref_sp<1>(int, size_t, const EvalJob *, const Tile *, int, int, hipStream_t);
extern template hipError_t launch_ref_sp<2>(int, size_t, const EvalJob *, const Tile *, int, int, hipStream_t);
extern template hipError_t launch_ref_sp<3>(int, size_t, const EvalJob *, const Tile *, int, int, hipStream_t);

template <int S, int POL>
hipError_t launch_tmarg_sp(int kdet, int R, bool dm, size_t lds_bytes, const EvalJob *jobs, const Tile *tiles, int n_tiles,
                           int nthreads, hipStream_t st);
extern template hipError_t launch_tmarg_sp<0, 0>(int, int, bool, size_t, const EvalJob *, const Tile *, int,
                                                     int, hipStream_t);
extern template hipError_t launch_tmarg_sp<0, 1>(int, int, bool, size_t, const EvalJob *, const Tile *, int,
                                                     int, hipStream_t);
extern template hipError_t launch_tmarg_sp<1, 0>(int, int, bool, size_t, const EvalJob *, const Tile *, int,
                                                     int, hipStream_t);
extern template hipError_t launch_tmarg_sp<1, 1>(int, int, bool, size_t, const EvalJob *, const Tile *, int,
                                                     int, hipStream_t);
extern template hipError_t launch_tmarg_sp<2, 0>(int, int, bool, size_t, const EvalJob *, const Tile *, int,
                                                     int, hipStream_t);
extern template hipError_t launch_tmarg_sp<2, 1>(int, int, bool, size_t, const EvalJob *, const Tile *, int,
                                                     int, hipStream_t);
extern template hipError_t launch_tmarg_sp<3, 0>(int, int, bool, size_t, const EvalJob *, const Tile *, int,
                                                     int, hipStream_t);
extern template hipError_t launch_tmarg_sp<3, 1>(int, int, bool, size_t, const EvalJob *, const Tile *, int,
                                                     int, hipStream_t);

struct BatchItem {
    ile_job *job;
    int64_t n;
    const void *theta;
    int64_t ld;
    const void *lnpmps;
    void *lnL;
    void *lw;
};

// A problem whose arrays are host memory: the caller's own when they are,
// else copies of its device arrays.
struct HostProblem {
    std::vector<int32_t> ml, mm;
    std::vector<double> pos, resp, Q, U, V;
    ile_problem p{};
};
ile_status problem_on_host(const ile_problem *P, HostProblem *out, const ile_problem **use);
ile_status set_err(ile_status st, const std::string &msg);
ile_status dev_fail(ile_ctx *ctx, hipError_t e, const char *what);
ile_status ctx_check(ile_ctx *ctx);
ile_status ctx_alloc(ile_ctx *ctx, void **p, size_t bytes, const char *what);
void ctx_free(ile_ctx *ctx, void *p, size_t bytes);
void *pin_alloc(ile_ctx *ctx, size_t bytes);
void pin_free(ile_ctx *ctx, void *p, size_t bytes);
void ctx_pool_release(ile_ctx *ctx);
// Build and upload a job; with a stream the upload is asynchronous on it
// (the pinned staging stays with the job until release).
ile_status job_create(ile_ctx *ctx, const ile_problem *P, ile_job **out, hipStream_t st, bool async);
// Release without a device-wide sync: the caller guarantees no queued work
// still uses the job's buffers.
void job_release_nosync(ile_job *job);
ile_status eval_batch(ile_ctx *ctx, const std::vector<BatchItem> &items, hipStream_t st);
// Time-marginalised evaluation of several jobs (oversampling R = 1 or 4).
ile_status tmarg_batch(ile_ctx *ctx, const std::vector<BatchItem> &items, int R, hipStream_t st);
// Copy two host arrays into a scratch slot (caller holds batch_mu); after
// enqueueing the kernel that reads them, call batch_done with the slot.
// `extra` bytes of device scratch (and the same of pinned host staging) follow
// the copied arrays in the slot, for kernel outputs read back by the caller.
ile_status batch_upload(ile_ctx *ctx, const void *a, size_t na, const void *b, size_t nb, void **da, void **db,
                        int *slot, hipStream_t st, size_t extra = 0, void **dextra = nullptr,
                        void **hextra = nullptr);
ile_status batch_done(ile_ctx *ctx, int slot, hipStream_t st);
ile_status draw_batch(ile_ctx *ctx, int policy, const std::vector<DrawJob> &jobs, hipStream_t st);
// Mixture-pool updates of adaptive jobs of one policy (tiles of 2048 samples).
ile_status pool_batch(ile_ctx *ctx, int policy, const std::vector<PoolJob> &jobs, hipStream_t st);
ile_status marg_batch(ile_ctx *ctx, ile_job *const *jobs, int n_jobs, const int64_t *n, const void *const *lw,
                      const uint32_t *flags, ile_marg *out, hipStream_t st);
ile_status job_marg_launch(ile_job *job, int64_t n, const void *lw, bool reset, hipStream_t st);
ile_status job_adapt(ile_job *job, int64_t n, const void *theta, int64_t ld, const void *lw, const ile_gmm_opts *o,
                     hipStream_t st);
// One job of a batched refit: its samples and the key/round of its in-support
// mass draws.
struct AdaptItem {
    ile_job *job;
    int64_t n;
    const void *theta;
    int64_t ld;
    const void *lw;
    uint64_t z_seed;
    uint32_t z_round;
};
// Refit the mixtures of several jobs of one precision policy with the same
// options: every EM stage and the mass estimate are one launch for all jobs.
ile_status adapt_batch(ile_ctx *ctx, int policy, const std::vector<AdaptItem> &items, const ile_gmm_opts *o,
                       hipStream_t st);
void marg_from_state(const MargState &m, ile_marg *out);
// Mixed policy: rebuild the reference terms from job->rb.theta_ref, or set
// that point from the job's mixture first (no-ops for the other policies).
ile_status ref_rebuild(ile_job *job, hipStream_t st);
ile_status ref_from_proposal(ile_job *job, hipStream_t st);
// Look up the no-alloc estimator's scratch address on a device (the device
// must be current); done once per device, by ile_ctx_create.
ile_status noalloc_init_device(int device);
// Adaptive volume: buffers for updates of up to `cap` samples (the first call
// also installs the whole-cube grid over the job's sampled columns); bytes a
// job's AV buffers take for that cap.
ile_status av_ensure(ile_job *job, int64_t cap, hipStream_t st);
size_t av_bytes_for(int64_t cap);
// Batched AV draws (update = false; policy: the jobs' policy, theta type) or
// updates (update = true; log-weight type) of several jobs.
ile_status av_batch(ile_ctx *ctx, bool update, int policy, const std::vector<AvJob> &jobs, hipStream_t st);
// Adaptive Cartesian: the job's marginals (uniform over the sampled columns
// on first use), and batched draws / updates as for AV.
ile_status ac_ensure(ile_job *job, hipStream_t st);
ile_status ac_batch(ile_ctx *ctx, bool update, int policy, const std::vector<AcJob> &jobs, hipStream_t st);
void eval_geometry(const ile_job *job, int64_t n, size_t *lds, int64_t *tile, int *block);
size_t theta_size(int policy);
size_t out_size(int policy);
// Samples per stage-1 tile of the estimator for a job of n samples: at least
// 64 tiles while a tile keeps one 2048-sample step of a block (small jobs
// spread over the CUs), at most eight steps (16384 samples, from n = 2^20 up:
// large batches keep few, long tiles).  A function of n alone: the single-job
// and the batched estimator use it and agree to the bit.
inline int64_t marg_tile(int64_t n) {
    const int64_t t = ((n + 63) / 64 + 2047) / 2048 * 2048;
    return t < 2048 ? 2048 : (t > 16384 ? 16384 : t);
}

}  // namespace ile
