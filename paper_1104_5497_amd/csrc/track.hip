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
#include "xy_lane.hpp"

namespace nphc {

template <class T, int M>
struct LanePath {
    Point<T, M> z;
    double t, h;
    int32_t streak, acc, rej, status;
};

template <class T, int M>
__device__ __forceinline__ void start_point(int64_t pid, Point<T, M>& z)
{
#pragma unroll
    for (int k = 0; k < M; ++k) {
        z.x[k] = {((pid >> k) & 1) ? T(-1) : T(1), T(0)};
        z.y[k] = {((pid >> (M + k)) & 1) ? T(-1) : T(1), T(0)};
    }
}

// One predictor-corrector step of one lane's path (paper, section "NPHC
// method": predictor, then Newton's corrector; step control as documented in
// nphc_track_paths).  Sets S.status when the path ends.
template <class T, int M>
__device__ __forceinline__ void path_step(const Couplings<T, M>& C, cx<T> gamma,
                                          const TrackOptsDev& o, LanePath<T, M>& S)
{
    const bool last = S.h >= o.t_end - S.t;
    const double hh = last ? (o.t_end - S.t) : S.h;
    const double t1 = last ? o.t_end : S.t + hh;
    const int nst = o.predictor == 0 ? 4 : 1;

    Point<T, M> k;   // previous stage's tangent
    Point<T, M> w;   // RK4 accumulator, then the corrected point
    bool ok = true, conv = false, bad = false;
    T prev = T(0);

    for (int s = 0; s < nst + o.max_corr; ++s) {
        const bool pred = s < nst;
        const bool want = pred ? ok : (ok && !conv && !bad);
        if (!want) continue;
        // evaluation point and time
        double cs = 0.0;
        if (pred) cs = (s == 0) ? 0.0 : (s == 3 ? 1.0 : 0.5);
        const double tq = pred ? (s == 3 ? t1 : S.t + cs * hh) : t1;
        Point<T, M> zq;
        if (pred) {
            const T ch = T(cs * hh);
#pragma unroll
            for (int i = 0; i < M; ++i) {
                zq.x[i] = (s == 0) ? S.z.x[i] : fma(mk(ch, T(0)), k.x[i], S.z.x[i]);
                zq.y[i] = (s == 0) ? S.z.y[i] : fma(mk(ch, T(0)), k.y[i], S.z.y[i]);
            }
        } else {
            zq = w;
        }
        Point<T, M> d;
        const bool sok = solve_step<T, M>(C, gamma, T(tq), T(1.0 - tq), !pred, zq, d);
        if (pred) {
            ok = ok && sok;
            const T ws = (s == 0 || s == 3) ? T(1) : T(2);
#pragma unroll
            for (int i = 0; i < M; ++i) {
                w.x[i] = (s == 0) ? d.x[i] : fma(mk(ws, T(0)), d.x[i], w.x[i]);
                w.y[i] = (s == 0) ? d.y[i] : fma(mk(ws, T(0)), d.y[i], w.y[i]);
            }
            k = d;
            if (s == nst - 1) {
                const T f = T(nst == 4 ? hh / 6.0 : hh);
#pragma unroll
                for (int i = 0; i < M; ++i) {
                    w.x[i] = fma(mk(f, T(0)), w.x[i], S.z.x[i]);
                    w.y[i] = fma(mk(f, T(0)), w.y[i], S.z.y[i]);
                }
            }
        } else {
            if (!sok) {
                bad = true;
            } else {
#pragma unroll
                for (int i = 0; i < M; ++i) {
                    w.x[i] = w.x[i] + d.x[i];
                    w.y[i] = w.y[i] + d.y[i];
                }
                const T nd = norm_inf<T, M>(d);
                if (s > nst && nd > T(0.5) * prev) bad = true;
                prev = nd;
                if (!bad && nd <= T(o.corr_tol) * (T(1) + norm_inf<T, M>(w))) conv = true;
            }
        }
    }

    const T wn = norm_inf<T, M>(w);
    const bool finite = (wn - wn == T(0));
    if (ok && conv && !bad && !finite) {
        S.status = NPHC_PATH_FAIL_NONFINITE;
        return;
    }
    if (ok && conv && !bad) {
        S.z = w;
        S.t = t1;
        S.acc += 1;
        if (++S.streak == 3) {
            S.h = fmin(2.0 * (last ? hh : S.h), o.hmax);
            S.streak = 0;
        } else if (last) {
            S.h = hh;
        }
        if (double(wn) > o.R_inf) S.status = NPHC_PATH_DIVERGED;
        else if (S.t >= o.t_end) S.status = NPHC_PATH_REACHED;
    } else {
        S.rej += 1;
        S.streak = 0;
        S.h = 0.5 * hh;
        if (S.h < o.hmin) S.status = (S.t >= o.t_stall) ? NPHC_PATH_STALLED : NPHC_PATH_FAIL_MINSTEP;
    }
    if (S.status == NPHC_PATH_PENDING && S.acc + S.rej >= o.max_steps)
        S.status = NPHC_PATH_FAIL_MAXSTEPS;
}

template <class T, int M>
__device__ __forceinline__ void write_path(const TrackArgs& A, int64_t item, const LanePath<T, M>& S)
{
    const int64_t st = A.out_stride;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        A.z[(2 * k) * st + item] = double(S.z.x[k].re);
        A.z[(2 * k + 1) * st + item] = double(S.z.x[k].im);
        A.z[(2 * (M + k)) * st + item] = double(S.z.y[k].re);
        A.z[(2 * (M + k) + 1) * st + item] = double(S.z.y[k].im);
    }
    A.t[item] = S.t;
    A.status[item] = S.status;
    A.accepted[item] = S.acc;
    A.rejected[item] = S.rej;
}

// Process every queue position of class c.  UNIFORM: the batch has a single
// system, whose couplings are then read through scalar loads.
template <class T, int M, bool UNIFORM>
__device__ void run_class(const TrackArgs& A, int c)
{
    const int lane = __lane_id();
    const int64_t qhi = A.q->qhi[c];
    const int64_t item_lo = A.cls[c].item_lo;

    LanePath<T, M> S;
    Couplings<T, M> C;
    cx<T> gamma;
    if (UNIFORM) {
        C.p = reinterpret_cast<const T*>(A.Jpack);
        gamma = {T(A.gamma[0]), T(A.gamma[1])};
    }
    int64_t item = -1;
    bool active = false, drained = false;

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
                            C.p = reinterpret_cast<const T*>(A.Jpack) + A.Jpack_off[sys];
                            gamma = {T(A.gamma[2 * sys]), T(A.gamma[2 * sys + 1])};
                        }
                        start_point<T, M>(pid, S.z);
                        S.t = 0.0;
                        S.h = A.o.h0;
                        S.streak = S.acc = S.rej = 0;
                        S.status = NPHC_PATH_PENDING;
                        active = true;
                    }
                }
            }
        }
        if (!__any(active)) break;
        if (active) {
            path_step<T, M>(C, gamma, A.o, S);
            if (S.status != NPHC_PATH_PENDING) {
                write_path<T, M>(A, item, S);
                active = false;
            }
        }
    }
    (void)item_lo;
}

template <class T, int M>
__global__ __launch_bounds__(64) void track_uniform_kernel(TrackArgs A)
{
    run_class<T, M, true>(A, 0);
}

template <class T>
__global__ __launch_bounds__(64) void track_batch_kernel(TrackArgs A)
{
    for (int c = 0; c < A.num_classes; ++c) {
        switch (A.cls[c].M) {
#define NPHC_CASE(m) \
    case m: run_class<T, m, false>(A, c); break;
            NPHC_CASE(1) NPHC_CASE(2) NPHC_CASE(3) NPHC_CASE(4)
            NPHC_CASE(5) NPHC_CASE(6) NPHC_CASE(7) NPHC_CASE(8)
#undef NPHC_CASE
            default: break;
        }
    }
}

// Setup: pack the couplings in the tracking type, and turn the classes' item
// ranges into queue-position ranges (binary search in the sorted id list).
template <class T>
__global__ void track_setup_kernel(TrackArgs A, const double* J, const int64_t* J_off,
                                   int64_t count, const int64_t* count_dev, T* Jpack,
                                   int64_t* Jpack_off)
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
        for (int e = tid; e < m * m + m; e += blockDim.x) {
            double v;
            if (e < m * m) {
                const int k = e / m, j = e % m;
                v = (k == j) ? 0.0 : Jb[k * N + j];
            } else {
                const int k = e - m * m;
                v = Jb[k * N + (N - 1)];
            }
            out[e] = T(v);
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
    size_t q_off, jp_off, jpo_off, total;
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
    L.jpo_off = L.jp_off + align256(elems * esz);
    L.total = L.jpo_off + align256(sizeof(int64_t) * size_t(b->num_systems));
    return L;
}

int check_batch(const nphc_batch* b, bool* mixed, int* minN, int* maxN);

template <class T>
static int launch_track(const nphc_batch* b, const int64_t* ids, int64_t count,
                        const int64_t* count_dev, const nphc_track_opts* o, double* z,
                        int64_t item_stride, double* t, int32_t* status, int32_t* accepted,
                        int32_t* rejected, void* ws, size_t ws_bytes, hipStream_t stream,
                        int precision)
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

    char* base = static_cast<char*>(ws);
    TrackArgs A = {};
    A.num_systems = b->num_systems;
    A.N = b->N;
    A.path_off = b->path_off;
    A.gamma = b->gamma;
    A.Jpack = base + L.jp_off;
    A.Jpack_off = reinterpret_cast<const int64_t*>(base + L.jpo_off);
    A.ids = ids;
    A.q = reinterpret_cast<QueueState*>(base + L.q_off);
    A.o = {o->h0, o->hmax, o->hmin, o->corr_tol, o->R_inf, o->t_stall, o->t_end,
           o->max_corr, o->max_steps, o->predictor, 0};
    A.out_stride = item_stride;
    A.z = z;
    A.t = t;
    A.status = status;
    A.accepted = accepted;
    A.rejected = rejected;
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
                       reinterpret_cast<int64_t*>(base + L.jpo_off));
    if (hipGetLastError() != hipSuccess) return NPHC_EHIP;

    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NPHC_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return NPHC_EHIP;

    const void* fn = nullptr;
    if (!mixed) {
        switch (minN - 1) {
#define NPHC_UCASE(m) case m: fn = reinterpret_cast<const void*>(&track_uniform_kernel<T, m>); break;
            NPHC_UCASE(1) NPHC_UCASE(2) NPHC_UCASE(3) NPHC_UCASE(4) NPHC_UCASE(5) NPHC_UCASE(6)
            NPHC_UCASE(7) NPHC_UCASE(8) NPHC_UCASE(9) NPHC_UCASE(10) NPHC_UCASE(11) NPHC_UCASE(12)
#undef NPHC_UCASE
            default: return NPHC_EUNSUPPORTED;
        }
        if (b->num_systems != 1) fn = nullptr;  // several rings of one size: per-lane couplings
    }
    if (!fn) {
        if (maxN > NPHC_BATCH_MAX_N) return NPHC_EUNSUPPORTED;
        fn = reinterpret_cast<const void*>(&track_batch_kernel<T>);
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int grid = cus * per_cu;
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
                                int32_t* accepted, int32_t* rejected, void* workspace,
                                size_t ws_bytes, hipStream_t stream)
{
    if (precision == NPHC_FP64)
        return nphc::launch_track<double>(b, ids, count, count_dev, o, z, item_stride, t, status,
                                          accepted, rejected, workspace, ws_bytes, stream, precision);
    if (precision == NPHC_FP32)
        return nphc::launch_track<float>(b, ids, count, count_dev, o, z, item_stride, t, status,
                                         accepted, rejected, workspace, ws_bytes, stream, precision);
    return NPHC_EUNSUPPORTED;
}
