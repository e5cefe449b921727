// common.hpp -- shared launch-side definitions of the HIP library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nphc.h"

namespace nphc {

constexpr int kMaxM = NPHC_MAX_N - 1;      // free spins
constexpr int kMaxClasses = NPHC_MAX_N;    // one queue class per ring size
constexpr int kBatchMaxM = 8;              // rings of mixed size: N <= 9

// One class = all systems of one ring size, a contiguous range of items.
struct ClassDesc {
    int32_t M;
    int32_t pad;
    int64_t item_lo, item_hi;
};

// Work-queue state, in the caller's workspace.
struct QueueState {
    unsigned long long next[kMaxClasses];  // next queue position per class
    int64_t qhi[kMaxClasses];              // end of the class's positions
};

struct TrackOptsDev {
    double h0, hmax, hmin, corr_tol, R_inf, t_stall, t_end;
    int32_t max_corr, max_steps, predictor, resume;
    double handoff_norm;       // > 0: stop with HANDOFF once ||z|| exceeds it
    int32_t handoff_rejects;   // > 0: stop with HANDOFF after this many rejections in a row
    int32_t pad;
    double t_endzone;          // end zone: t >= t_endzone
    double hmin_rel;           // end zone: a step below hmin_rel (1 - t) with ||z|| > collapse_norm is a collapse
    double collapse_norm;
    double grow_ratio;         // end zone: ||z|| grew by this factor over the last step ...
    double grow_cap;           // ... then the next step is at most grow_cap (1 - t)
    int32_t handoff_steps;     // > 0: stop with HANDOFF after this many steps
    int32_t pad2;
    double pred_tol;           // > 0: reject when the first correction exceeds pred_tol (1 + ||z||)
    int32_t step_ctrl;         // 0: double after three accepted steps; 1: predictor-error control
    int32_t drain_steps;       // > 0: steps a path may take after the queue drained, then HANDOFF
};

struct TrackArgs {
    // batch
    int32_t num_systems;
    int32_t num_classes;
    const int32_t* N;          // device
    const int64_t* path_off;   // device, num_systems + 1
    const double* gamma;       // device, 2 per system
    const void* Jpack;         // device, packed couplings in the tracking type
    const void* Jpack64;       // device, the same in float64 (== Jpack for float64 tracking)
    const int64_t* Jpack_off;  // device, per system
    ClassDesc cls[kMaxClasses];
    // work list
    const int64_t* ids;        // device or null (= all items)
    QueueState* q;             // device workspace
    TrackOptsDev o;
    // outputs, indexed by queue position
    int64_t out_stride;        // >= number of positions
    double* z;                 // 2 * n_max planes of out_stride doubles (re, im per unknown)
    double* t;
    int32_t* status;
    int32_t* accepted;
    int32_t* rejected;
    int32_t* solves;           // nullable
    double* h;                 // nullable (required with o.resume)
};

__device__ __forceinline__ int64_t find_system(const int64_t* path_off, int32_t num_systems,
                                               int64_t item)
{
    int32_t lo = 0, hi = num_systems;  // path_off[lo] <= item < path_off[hi]
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) >> 1;
        if (path_off[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace nphc
