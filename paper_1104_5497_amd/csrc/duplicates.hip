// duplicates.hip -- the path-jump check: two nonsingular endpoints of one
// system at the same root.
//
// Candidates are bucketed by a hash table keyed by (system, cell of u), with
// u = sum_k a_k Re z_k + b_k Im z_k a fixed linear combination of all
// coordinates.  Two endpoints within tol in max-norm differ in u by at most
// tol * S, S = sum_k (a_k + b_k), so with cells of width 2 tol S they fall in
// the same or neighbouring cells; each query walks three cells and compares
// the coordinates of what it finds.  Expected work is linear in the number
// of candidates (a fixed combination of all coordinates separates distinct
// roots, unlike any single coordinate, which many symmetric roots share).
// Everything is a kernel (the table is cleared by a fill kernel), so the
// sequence can be captured in a graph.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.hpp"

namespace nphc {

constexpr unsigned long long kEmpty = ~0ull;
constexpr int kSysBits = 20;                       // systems per batch < 2^20
constexpr long long kCellClamp = 1ll << 42;        // |cell| clamped (keys stay below kEmpty)

struct DupArgs {
    int32_t num_systems;
    int32_t log2T;
    const int32_t* N;
    const int64_t* path_off;
    const int64_t* cand;         // sorted NONSINGULAR item ids
    const int64_t* cand_count;   // device
    const int64_t* probe;        // sorted items to check (or null: every candidate)
    const int64_t* probe_count;  // device
    double tol;
    double width;                // cell width 2 tol S
    const double* z;
    int64_t stride;
    int32_t* endpoint;
    unsigned long long* marked;
    int64_t cap;                 // capacity: candidates beyond it are ignored
    unsigned long long* keys;    // T slots
    int64_t* heads;              // T slots: first candidate position of the slot's chain
    int64_t* next;               // per candidate position: next in the chain
    int64_t T;
};

// coefficient of coordinate plane c (2k: Re z_k, 2k+1: Im z_k), in [1, 2)
__device__ __forceinline__ double dup_coef(int c)
{
    const double g = 0.6180339887498949 * double(c + 1);
    return 1.0 + (g - floor(g));
}

__device__ __forceinline__ double dup_u(const DupArgs& A, int64_t g, int n)
{
    double u = 0.0;
    for (int c = 0; c < 2 * n; ++c) u += dup_coef(c) * A.z[c * A.stride + g];
    return u;
}

__device__ __forceinline__ unsigned long long dup_key(long long cell, int64_t sys)
{
    cell = cell < -kCellClamp ? -kCellClamp : (cell > kCellClamp ? kCellClamp : cell);
    return ((unsigned long long)(cell + 2 * kCellClamp) << kSysBits) | (unsigned long long)sys;
}

__device__ __forceinline__ int64_t dup_hash(const DupArgs& A, unsigned long long key)
{
    return (int64_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - A.log2T));
}

// the calls do nothing in probe mode when there are no probes
__device__ __forceinline__ bool dup_idle(const DupArgs& A)
{
    return A.probe && *A.probe_count <= 0;
}

__global__ void dup_zero_kernel(unsigned long long* c) { *c = 0ull; }

__global__ __launch_bounds__(256) void dup_clear_kernel(DupArgs A)
{
    if (dup_idle(A)) return;
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < A.T;
         s += int64_t(gridDim.x) * blockDim.x) {
        A.keys[s] = kEmpty;
        A.heads[s] = -1;
    }
}

__global__ __launch_bounds__(256) void dup_insert_kernel(DupArgs A)
{
    if (dup_idle(A)) return;
    const int64_t K = min(*A.cand_count, A.cap);
    const int64_t mask = A.T - 1;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < K;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t g = A.cand[i];
        const int64_t sys = find_system(A.path_off, A.num_systems, g);
        const int n = 2 * (A.N[sys] - 1);
        const long long cell = (long long)floor(dup_u(A, g, n) / A.width);
        const unsigned long long key = dup_key(cell, sys);
        int64_t h = dup_hash(A, key);
        // the table has at least twice as many slots as candidates: a free
        // or matching slot is always found
        for (;;) {
            const unsigned long long old = atomicCAS(&A.keys[h], kEmpty, key);
            if (old == kEmpty || old == key) break;
            h = (h + 1) & mask;
        }
        A.next[i] = (int64_t)atomicExch((unsigned long long*)&A.heads[h], (unsigned long long)i);
    }
}

__device__ __forceinline__ void mark_dup(int32_t* endpoint, int64_t g, unsigned long long* marked)
{
    const int old = atomicExch(&endpoint[g], NPHC_END_DUPLICATE);
    if (old != NPHC_END_DUPLICATE) atomicAdd(marked, 1ull);
}

__global__ __launch_bounds__(256) void dup_query_kernel(DupArgs A)
{
    if (dup_idle(A)) return;
    const int64_t K = min(*A.cand_count, A.cap);
    const int64_t Q = A.probe ? *A.probe_count : K;
    const int64_t mask = A.T - 1;
    for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < Q;
         q += int64_t(gridDim.x) * blockDim.x) {
        const int64_t gi = A.probe ? A.probe[q] : A.cand[q];
        if (A.probe && A.endpoint[gi] != NPHC_END_NONSINGULAR) continue;
        const int64_t sys = find_system(A.path_off, A.num_systems, gi);
        const int n = 2 * (A.N[sys] - 1);
        const long long cell = (long long)floor(dup_u(A, gi, n) / A.width);
        for (int dc = -1; dc <= 1; ++dc) {
            const unsigned long long key = dup_key(cell + dc, sys);
            int64_t h = dup_hash(A, key);
            int64_t j = -1;
            for (;;) {
                const unsigned long long k = A.keys[h];
                if (k == key) { j = A.heads[h]; break; }
                if (k == kEmpty) break;
                h = (h + 1) & mask;
            }
            for (; j >= 0; j = A.next[j]) {
                const int64_t gj = A.cand[j];
                // all pairs: each pair once (from its smaller item); probes:
                // every other candidate
                if (gj == gi || (!A.probe && gj < gi)) continue;
                bool close = true;
                for (int c = 0; c < 2 * n && close; ++c)
                    close = fabs(A.z[c * A.stride + gi] - A.z[c * A.stride + gj]) < A.tol;
                if (close) {
                    mark_dup(A.endpoint, gi, A.marked);
                    mark_dup(A.endpoint, gj, A.marked);
                }
            }
        }
    }
}

int check_batch(const nphc_batch* b, bool* mixed, int* minN, int* maxN);

struct DupLayout {
    int64_t T;
    int log2T;
    size_t keys_off, heads_off, next_off, total;
};

static DupLayout dup_layout(int64_t capacity)
{
    DupLayout L;
    int64_t need = capacity < 1 ? 2 : 2 * capacity;
    L.log2T = 1;
    while ((int64_t(1) << L.log2T) < need) ++L.log2T;
    L.T = int64_t(1) << L.log2T;
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    L.keys_off = 0;
    L.heads_off = al(size_t(L.T) * 8);
    L.next_off = L.heads_off + al(size_t(L.T) * 8);
    L.total = L.next_off + al(size_t(capacity < 1 ? 1 : capacity) * 8);
    return L;
}

}  // namespace nphc

using namespace nphc;

extern "C" size_t nphc_duplicates_workspace_size(int64_t capacity)
{
    if (capacity < 0) return 0;
    return dup_layout(capacity).total;
}

extern "C" int nphc_mark_duplicates(const nphc_batch* b, const int64_t* ids, int64_t count,
                                    const int64_t* count_dev, const int64_t* probe_ids,
                                    const int64_t* probe_count_dev, double dup_tol, const double* z,
                                    int64_t item_stride, int32_t* endpoint, int64_t* num_marked,
                                    void* workspace, size_t ws_bytes, hipStream_t stream)
{
    bool mixed;
    int minN, maxN;
    int rc = check_batch(b, &mixed, &minN, &maxN);
    if (rc) return rc;
    if (!ids || !count_dev || !z || !endpoint || !num_marked || !(dup_tol > 0.0) || count < 0)
        return NPHC_EINVAL;
    if (probe_ids && !probe_count_dev) return NPHC_EINVAL;
    if (b->num_systems >= (1 << kSysBits)) return NPHC_EUNSUPPORTED;
    const int64_t total = b->path_off_host[b->num_systems];
    if (item_stride < total || count > total) return NPHC_EINVAL;
    const DupLayout L = dup_layout(count);
    if (!workspace || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return NPHC_EWORKSPACE;
    char* base = static_cast<char*>(workspace);
    DupArgs A = {};
    A.num_systems = b->num_systems;
    A.log2T = L.log2T;
    A.N = b->N;
    A.path_off = b->path_off;
    A.cand = ids;
    A.cand_count = count_dev;
    A.probe = probe_ids;
    A.probe_count = probe_count_dev;
    A.tol = dup_tol;
    double S = 0.0;  // sum of the coefficients over the widest system's planes
    const int planes = 4 * (maxN - 1);
    for (int c = 0; c < planes; ++c) {
        const double g = 0.6180339887498949 * double(c + 1);
        S += 1.0 + (g - std::floor(g));
    }
    A.width = 2.0 * dup_tol * S;
    A.z = z;
    A.stride = item_stride;
    A.endpoint = endpoint;
    A.marked = reinterpret_cast<unsigned long long*>(num_marked);
    A.keys = reinterpret_cast<unsigned long long*>(base + L.keys_off);
    A.heads = reinterpret_cast<int64_t*>(base + L.heads_off);
    A.next = reinterpret_cast<int64_t*>(base + L.next_off);
    A.T = L.T;
    A.cap = count;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NPHC_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return NPHC_EHIP;
    hipLaunchKernelGGL(dup_zero_kernel, dim3(1), dim3(1), 0, stream, A.marked);
    const unsigned grid = unsigned(cus) * 8;
    hipLaunchKernelGGL(dup_clear_kernel, dim3(grid), dim3(256), 0, stream, A);
    hipLaunchKernelGGL(dup_insert_kernel, dim3(grid), dim3(256), 0, stream, A);
    hipLaunchKernelGGL(dup_query_kernel, dim3(grid), dim3(256), 0, stream, A);
    if (hipGetLastError() != hipSuccess) return NPHC_EHIP;
    return NPHC_OK;
}
