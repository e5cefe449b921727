// track.hip -- persistent path-tracker kernels (one path per lane).
//
// Each wave runs a loop: lanes without a path take the next queue positions
// (one atomic per wave), then every lane with a path does one
// predictor-corrector step at its own t.  A lane whose path ends writes its
// endpoint and takes new work at the next iteration, so paths with very
// different step counts (finite roots, paths to infinity, singular endpoints)
// do not leave lanes idle until the queue drains.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "path.hpp"
#include "xy_group.hpp"

namespace nphc {

// float32 tracking runs on a float64 point with a float64 Newton residual;
// float64 tracking keeps everything in float64.
template <class T, int M> struct StoreFor { using type = PathStore<T, M>; };
template <int M> struct StoreFor<float, M> { using type = MixedStore<M>; };

// A lane's store inside the block's LDS (64 lanes x 64 M bytes).
template <int M>
__device__ __forceinline__ void make_store(cx<double>* lds, int lane, PathStore<double, M>& st)
{
    st.base = lds + lane;
    st.stride = 64;
}
template <int M>
__device__ __forceinline__ void make_store(cx<double>* lds, int lane, MixedStore<M>& st)
{
    st.zb = lds + lane;
    st.wb = reinterpret_cast<cx<float>*>(lds + 64 * 2 * M) + lane;
    st.db = st.wb + 64 * 2 * M;
    st.stride = 64;
}

template <class Store, int M>
__device__ __forceinline__ void write_path(const TrackArgs& A, int64_t item, const LanePath<Store, M>& S)
{
    const int64_t st = A.out_stride;
#pragma unroll
    for (int i = 0; i < 2 * M; ++i) {
        const cx<double> v = S.st.get(i);
        A.z[(2 * i) * st + item] = v.re;
        A.z[(2 * i + 1) * st + item] = v.im;
    }
    A.t[item] = S.t;
    A.status[item] = S.status;
    A.accepted[item] = S.acc;
    A.rejected[item] = S.rej;
    if (A.solves) A.solves[item] = S.solves;
    if (A.h) A.h[item] = S.h;
}

template <class Store, int M>
__device__ __forceinline__ void read_path(const TrackArgs& A, int64_t item, LanePath<Store, M>& S)
{
    const int64_t st = A.out_stride;
#pragma unroll
    for (int i = 0; i < 2 * M; ++i)
        S.st.put(i, {A.z[(2 * i) * st + item], A.z[(2 * i + 1) * st + item]});
    S.t = A.t[item];
    S.h = A.h[item];
    S.acc = A.accepted[item];
    S.rej = A.rejected[item];
    S.solves = A.solves ? A.solves[item] : 0;
}

// Process every queue position of class c.  UNIFORM: the batch has a single
// system, whose couplings are then read through scalar loads.
template <class T, int M, bool UNIFORM>
__device__ void run_class(const TrackArgs& A, int c, cx<double>* lds)
{
    using Store = typename StoreFor<T, M>::type;
    const int lane = __lane_id();
    const int64_t qhi = A.q->qhi[c];

    LanePath<Store, M> S;
    make_store<M>(lds, lane, S.st);
    Couplings<T, M> C;
    Couplings<double, M> C64;
    cx<double> gamma64;
    if (UNIFORM) {
        C.p = (const NPHC_RO T*)(A.Jpack);
        C64.p = (const NPHC_RO double*)(A.Jpack64);
        gamma64 = {A.gamma[0], A.gamma[1]};
    }
    int64_t item = -1;
    bool active = false, drained = false;
    int post = 0;  // steps of the current path since this wave saw the queue drained

    for (;;) {
        if (!drained) {
            const unsigned long long need = __ballot(!active);
            if (need) {
                const int cnt = __popcll(need);
                const int leader = __ffsll((long long)need) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(&A.q->next[c], (unsigned long long)cnt);
                base = __shfl(base, leader);
                if ((int64_t)(base + cnt) >= qhi) drained = true;
                if (!active) {
                    const int rank = __popcll(need & ((1ull << lane) - 1ull));
                    const int64_t qpos = (int64_t)base + rank;
                    if (qpos < qhi) {
                        item = A.ids ? A.ids[qpos] : qpos;
                        int64_t pid;
                        if (UNIFORM) {
                            pid = item;
                        } else {
                            const int64_t sys = find_system(A.path_off, A.num_systems, item);
                            pid = item - A.path_off[sys];
                            C.p = (const NPHC_RO T*)(A.Jpack) + A.Jpack_off[sys];
                            C64.p = (const NPHC_RO double*)(A.Jpack64) + A.Jpack_off[sys];
                            gamma64 = {A.gamma[2 * sys], A.gamma[2 * sys + 1]};
                        }
                        if (A.o.resume) {
                            read_path<Store, M>(A, item, S);
                        } else {
#pragma unroll
                            for (int k = 0; k < M; ++k) {
                                S.st.put(k, {((pid >> k) & 1) ? -1.0 : 1.0, 0.0});
                                S.st.put(M + k, {((pid >> (M + k)) & 1) ? -1.0 : 1.0, 0.0});
                            }
                            S.t = 0.0;
                            S.h = A.o.h0;
                            S.acc = S.rej = S.solves = 0;
                        }
                        S.h_acc = S.h;
                        {
                            Point<T, M> zc;
                            S.st.load_point(zc);
                            S.znorm = double(norm_inf<T, M>(zc));
                        }
                        S.streak = S.rej_run = 0;
                        S.status = NPHC_PATH_PENDING;
                        active = true;
                    }
                }
            }
        }
        if (!__any(active)) break;
        if (active) {
            const cx<T> gamma = {T(gamma64.re), T(gamma64.im)};
            path_step<Store, M>(C, gamma, C64, gamma64, A.o, S);
            if (drained) ++post;
            if (S.status == NPHC_PATH_PENDING && A.o.drain_steps > 0 && post >= A.o.drain_steps)
                S.status = NPHC_PATH_HANDOFF;
            if (S.status != NPHC_PATH_PENDING) {
                write_path<Store, M>(A, item, S);
                active = false;
            }
        }
    }
}

// One path per group of 16 lanes, float64 (4 paths per wave).  Every lane of
// a group holds the path's scalars and point and runs the same step; the
// linear solves are shared (xy_group.hpp); the group's point and RK4
// accumulator sit in one LDS slot that all its lanes address.
template <int M, bool UNIFORM>
__device__ void run_class_group(const TrackArgs& A, int c, cx<double>* lds)
{
    using Store = PathStore<double, M>;
    const int lane = __lane_id();
    const int r = lane & (kGroup - 1);
    const int grp = lane / kGroup;
    const int64_t qhi = A.q->qhi[c];

    LanePath<Store, M> S;
    S.st.base = lds + grp;
    S.st.stride = 64 / kGroup;
    Couplings<double, M> C;
    GroupRow<double, M> G;
    cx<double> gamma;
    if (UNIFORM) {
        C.p = (const NPHC_RO double*)(A.Jpack);
        gamma = {A.gamma[0], A.gamma[1]};
        load_group_row<double, M>(C, r, G);
    }
    int64_t item = -1;
    bool active = false, drained = false;
    int post = 0;

    for (;;) {
        if (!drained) {
            // the leader lane (r = 0) of every idle group asks for a path
            const unsigned long long need = __ballot(!active && r == 0);
            if (need) {
                const int cnt = __popcll(need);
                const int leader = __ffsll((long long)need) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(&A.q->next[c], (unsigned long long)cnt);
                base = __shfl(base, leader);
                if ((int64_t)(base + cnt) >= qhi) drained = true;
                if (!active) {
                    const int rank = __popcll(need & ((1ull << (grp * kGroup)) - 1ull));
                    const int64_t qpos = (int64_t)base + rank;
                    if (qpos < qhi) {
                        item = A.ids ? A.ids[qpos] : qpos;
                        int64_t pid;
                        if (UNIFORM) {
                            pid = item;
                        } else {
                            const int64_t sys = find_system(A.path_off, A.num_systems, item);
                            pid = item - A.path_off[sys];
                            C.p = (const NPHC_RO double*)(A.Jpack) + A.Jpack_off[sys];
                            gamma = {A.gamma[2 * sys], A.gamma[2 * sys + 1]};
                            load_group_row<double, M>(C, r, G);
                        }
                        if (A.o.resume) {
                            read_path<Store, M>(A, item, S);
                        } else {
#pragma unroll
                            for (int k = 0; k < M; ++k) {
                                S.st.put(k, {((pid >> k) & 1) ? -1.0 : 1.0, 0.0});
                                S.st.put(M + k, {((pid >> (M + k)) & 1) ? -1.0 : 1.0, 0.0});
                            }
                            S.t = 0.0;
                            S.h = A.o.h0;
                            S.acc = S.rej = S.solves = 0;
                        }
                        S.h_acc = S.h;
                        {
                            Point<double, M> zc;
                            S.st.load_point(zc);
                            S.znorm = norm_inf<double, M>(zc);
                        }
                        S.streak = S.rej_run = 0;
                        S.status = NPHC_PATH_PENDING;
                        post = 0;
                        active = true;
                    }
                }
            }
        }
        if (!__any(active)) break;
        if (active) {
            path_step<Store, M, GroupSolver<M>>(C, gamma, C, gamma, A.o, S, GroupSolver<M>{&G});
            if (drained) ++post;
            if (S.status == NPHC_PATH_PENDING && A.o.drain_steps > 0 && post >= A.o.drain_steps)
                S.status = NPHC_PATH_HANDOFF;
            if (S.status != NPHC_PATH_PENDING) {
                if (r == 0) write_path<Store, M>(A, item, S);
                active = false;
            }
        }
    }
}

template <int M>
__global__ __launch_bounds__(64) void track_group_uniform_kernel(TrackArgs A)
{
    __shared__ cx<double> lds[(64 / kGroup) * 4 * M];
    run_class_group<M, true>(A, 0, lds);
}

__global__ __launch_bounds__(64) void track_group_batch_kernel(TrackArgs A)
{
    __shared__ cx<double> lds[(64 / kGroup) * 4 * kBatchMaxM];
    for (int c = 0; c < A.num_classes; ++c) {
        switch (A.cls[c].M) {
#define NPHC_CASE(m) \
    case m: run_class_group<m, false>(A, c, lds); break;
            NPHC_CASE(1) NPHC_CASE(2) NPHC_CASE(3) NPHC_CASE(4)
            NPHC_CASE(5) NPHC_CASE(6) NPHC_CASE(7) NPHC_CASE(8)
#undef NPHC_CASE
            default: break;
        }
    }
}

// Per-lane path state in LDS: 64 M bytes per lane (float64 tracking: point
// and RK4 accumulator, 4M complex float64; float32 tracking: float64 point
// plus float32 accumulator and increment).
template <class T, int M>
__global__ __launch_bounds__(64) void track_uniform_kernel(TrackArgs A)
{
    __shared__ cx<double> lds[64 * 4 * M];
    run_class<T, M, true>(A, 0, lds);
}

template <class T>
__global__ __launch_bounds__(64) void track_batch_kernel(TrackArgs A)
{
    __shared__ cx<double> lds[64 * 4 * kBatchMaxM];
    for (int c = 0; c < A.num_classes; ++c) {
        switch (A.cls[c].M) {
#define NPHC_CASE(m) \
    case m: run_class<T, m, false>(A, c, lds); break;
            NPHC_CASE(1) NPHC_CASE(2) NPHC_CASE(3) NPHC_CASE(4)
            NPHC_CASE(5) NPHC_CASE(6) NPHC_CASE(7) NPHC_CASE(8)
#undef NPHC_CASE
            default: break;
        }
    }
}

// Setup: pack the couplings in the tracking type (and in float64 for the
// wide residual of float32 tracking), and turn the classes' item
// ranges into queue-position ranges (binary search in the sorted id list).
template <class T>
__global__ void track_setup_kernel(TrackArgs A, const double* J, const int64_t* J_off,
                                   int64_t count, const int64_t* count_dev, T* Jpack,
                                   double* Jpack64, int64_t* Jpack_off)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        int64_t off = 0;
        for (int b = 0; b < A.num_systems; ++b) {
            Jpack_off[b] = off;
            const int64_t m = A.N[b] - 1;
            off += m * m + m;
        }
    }
    __syncthreads();
    for (int b = blockIdx.x; b < A.num_systems; b += gridDim.x) {
        const int N = A.N[b];
        const int m = N - 1;
        const double* Jb = J + J_off[b];
        T* out = Jpack + Jpack_off[b];
        // rows 0..m-1 of J (N columns each), diagonal zeroed
        for (int e = tid; e < m * N; e += blockDim.x) {
            const int k = e / N, j = e % N;
            const double v = (k == j) ? 0.0 : Jb[e];
            out[e] = T(v);
            if (Jpack64 != static_cast<void*>(Jpack)) Jpack64[Jpack_off[b] + e] = v;
        }
    }
    if (blockIdx.x == 0 && tid < A.num_classes) {
        const int c = tid;
        int64_t n = count;
        if (count_dev) n = min(n, *count_dev);
        if (n < 0) n = 0;
        int64_t lo, hi;
        if (!A.ids) {
            lo = A.cls[c].item_lo;
            hi = A.cls[c].item_hi;
        } else {
            // first position with ids[pos] >= item_lo, first with >= item_hi
            int64_t a = 0, bnd = n;
            while (a < bnd) { int64_t mid = (a + bnd) >> 1; if (A.ids[mid] < A.cls[c].item_lo) a = mid + 1; else bnd = mid; }
            lo = a;
            bnd = n;
            while (a < bnd) { int64_t mid = (a + bnd) >> 1; if (A.ids[mid] < A.cls[c].item_hi) a = mid + 1; else bnd = mid; }
            hi = a;
        }
        A.q->next[c] = (unsigned long long)lo;
        A.q->qhi[c] = hi;
    }
}

}  // namespace nphc

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace nphc {

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct TrackLayout {
    size_t q_off, jp_off, jp64_off, jpo_off, total;
};

static TrackLayout track_layout(const nphc_batch* b, int precision)
{
    TrackLayout L;
    size_t elems = 0;
    for (int s = 0; s < b->num_systems; ++s) {
        size_t m = size_t(b->N_host[s] - 1);
        elems += m * m + m;
    }
    const size_t esz = precision == NPHC_FP32 ? sizeof(float) : sizeof(double);
    L.q_off = 0;
    L.jp_off = align256(sizeof(QueueState));
    // float32 tracking also needs the float64 pack (its Newton residual)
    L.jp64_off = precision == NPHC_FP32 ? L.jp_off + align256(elems * esz) : L.jp_off;
    L.jpo_off = L.jp64_off + align256(elems * sizeof(double));
    L.total = L.jpo_off + align256(sizeof(int64_t) * size_t(b->num_systems));
    return L;
}

int check_batch(const nphc_batch* b, bool* mixed, int* minN, int* maxN);

template <class T>
static int launch_track(const nphc_batch* b, const int64_t* ids, int64_t count,
                        const int64_t* count_dev, const nphc_track_opts* o, double* z,
                        int64_t item_stride, double* t, int32_t* status, int32_t* accepted,
                        int32_t* rejected, int32_t* solves, double* h, void* ws,
                        size_t ws_bytes, hipStream_t stream, int precision)
{
    bool mixed;
    int minN, maxN;
    int rc = check_batch(b, &mixed, &minN, &maxN);
    if (rc) return rc;
    if (mixed && maxN > NPHC_BATCH_MAX_N) return NPHC_EUNSUPPORTED;
    TrackLayout L = track_layout(b, precision);
    if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return NPHC_EWORKSPACE;
    if (!z || !t || !status || !accepted || !rejected || !o) return NPHC_EINVAL;
    if (count < 0 || (ids && count > item_stride)) return NPHC_EINVAL;
    if (item_stride < b->path_off_host[b->num_systems]) return NPHC_EINVAL;
    if (o->max_corr < 1 || o->max_corr > 16 || o->max_steps < 1 || !(o->t_end > 0.0) ||
        o->t_end > 1.0 || !(o->h0 > 0.0) || !(o->hmax > 0.0) || (o->predictor != 0 && o->predictor != 1))
        return NPHC_EINVAL;
    if ((o->lanes_per_path != 1 && o->lanes_per_path != kGroup) || o->drain_steps < 0) return NPHC_EINVAL;
    const bool grouped = o->lanes_per_path == kGroup;
    if (grouped && precision != NPHC_FP64) return NPHC_EUNSUPPORTED;

    char* base = static_cast<char*>(ws);
    TrackArgs A = {};
    A.num_systems = b->num_systems;
    A.N = b->N;
    A.path_off = b->path_off;
    A.gamma = b->gamma;
    A.Jpack = base + L.jp_off;
    A.Jpack64 = base + L.jp64_off;
    A.Jpack_off = reinterpret_cast<const int64_t*>(base + L.jpo_off);
    A.ids = ids;
    A.q = reinterpret_cast<QueueState*>(base + L.q_off);
    A.o.h0 = o->h0;
    A.o.hmax = o->hmax;
    A.o.hmin = o->hmin;
    A.o.corr_tol = o->corr_tol;
    A.o.R_inf = o->R_inf;
    A.o.t_stall = o->t_stall;
    A.o.t_end = o->t_end;
    A.o.max_corr = o->max_corr;
    A.o.max_steps = o->max_steps;
    A.o.predictor = o->predictor;
    A.o.resume = o->resume;
    A.o.handoff_norm = o->handoff_norm;
    A.o.handoff_rejects = o->handoff_rejects;
    A.o.t_endzone = o->t_endzone;
    A.o.hmin_rel = o->hmin_rel;
    A.o.collapse_norm = o->collapse_norm;
    A.o.grow_ratio = o->grow_ratio;
    A.o.grow_cap = o->grow_cap;
    A.o.handoff_steps = o->handoff_steps;
    A.o.pred_tol = o->pred_tol;
    A.o.step_ctrl = o->step_ctrl;
    A.o.drain_steps = o->drain_steps;
    A.out_stride = item_stride;
    A.z = z;
    A.t = t;
    A.status = status;
    A.accepted = accepted;
    A.rejected = rejected;
    A.solves = solves;
    A.h = h;
    if (o->resume && !h) return NPHC_EINVAL;
    // classes: maximal runs of equal N (systems are sorted by N)
    int nc = 0;
    for (int s = 0; s < b->num_systems; ++s) {
        const int M = b->N_host[s] - 1;
        if (nc == 0 || A.cls[nc - 1].M != M) {
            if (nc == kMaxClasses) return NPHC_EINVAL;
            A.cls[nc].M = M;
            A.cls[nc].item_lo = b->path_off_host[s];
            ++nc;
        }
        A.cls[nc - 1].item_hi = b->path_off_host[s + 1];
    }
    A.num_classes = nc;
    if (!ids) count = b->path_off_host[b->num_systems];

    int setup_blocks = b->num_systems < 1024 ? b->num_systems : 1024;
    if (setup_blocks < 1) setup_blocks = 1;
    hipLaunchKernelGGL(track_setup_kernel<T>, dim3(setup_blocks), dim3(256), 0, stream, A, b->J,
                       b->J_off, count, count_dev, reinterpret_cast<T*>(base + L.jp_off),
                       reinterpret_cast<double*>(base + L.jp64_off),
                       reinterpret_cast<int64_t*>(base + L.jpo_off));
    if (hipGetLastError() != hipSuccess) return NPHC_EHIP;

    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NPHC_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return NPHC_EHIP;

    const void* fn = nullptr;
    if (!mixed) {
        switch (minN - 1) {
#define NPHC_UCASE(m)                                                                 \
    case m:                                                                           \
        fn = grouped ? reinterpret_cast<const void*>(&track_group_uniform_kernel<m>) \
                     : reinterpret_cast<const void*>(&track_uniform_kernel<T, m>);    \
        break;
            NPHC_UCASE(1) NPHC_UCASE(2) NPHC_UCASE(3) NPHC_UCASE(4) NPHC_UCASE(5) NPHC_UCASE(6)
            NPHC_UCASE(7) NPHC_UCASE(8) NPHC_UCASE(9) NPHC_UCASE(10) NPHC_UCASE(11) NPHC_UCASE(12)
#undef NPHC_UCASE
            default: return NPHC_EUNSUPPORTED;
        }
        if (b->num_systems != 1) fn = nullptr;  // several rings of one size: per-lane couplings
    }
    if (!fn) {
        if (maxN > NPHC_BATCH_MAX_N) return NPHC_EUNSUPPORTED;
        fn = grouped ? reinterpret_cast<const void*>(&track_group_batch_kernel)
                     : reinterpret_cast<const void*>(&track_batch_kernel<T>);
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int grid = o->grid_blocks > 0 ? o->grid_blocks : cus * per_cu;
    void* args[] = {&A};
    if (hipLaunchKernel(fn, dim3(grid), dim3(64), args, 0, stream) != hipSuccess) return NPHC_EHIP;
    if (hipGetLastError() != hipSuccess) return NPHC_EHIP;
    return NPHC_OK;
}

}  // namespace nphc

extern "C" size_t nphc_track_workspace_size(const nphc_batch* b, int precision)
{
    if (!b || b->num_systems < 1 || !b->N_host) return 0;
    return nphc::track_layout(b, precision).total;
}

extern "C" int nphc_track_paths(const nphc_batch* b, const int64_t* ids, int64_t count,
                                const int64_t* count_dev, int precision, const nphc_track_opts* o,
                                double* z, int64_t item_stride, double* t, int32_t* status,
                                int32_t* accepted, int32_t* rejected, int32_t* solves,
                                double* h, void* workspace, size_t ws_bytes, hipStream_t stream)
{
    if (precision == NPHC_FP64)
        return nphc::launch_track<double>(b, ids, count, count_dev, o, z, item_stride, t, status,
                                          accepted, rejected, solves, h, workspace, ws_bytes, stream,
                                          precision);
    if (precision == NPHC_FP32)
        return nphc::launch_track<float>(b, ids, count, count_dev, o, z, item_stride, t, status,
                                         accepted, rejected, solves, h, workspace, ws_bytes, stream,
                                         precision);
    return NPHC_EUNSUPPORTED;
}
