// select.hip -- ordered stream compaction of item ids by endpoint code, over
// all items or over a given list of item ids.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace nphc {

// The candidates: items 0..n-1, or list[0..len-1] with len = min(n, *n_dev)
// when n_dev is given.
struct SelSrc {
    const int32_t* code;
    const int64_t* list;   // null: the identity
    const int64_t* n_dev;  // null: n
    int64_t n;
    uint64_t mask;
    __device__ __forceinline__ int64_t len() const
    {
        if (!n_dev) return n;
        const int64_t c = *n_dev;
        return c < 0 ? 0 : (c < n ? c : n);
    }
    __device__ __forceinline__ int64_t item(int64_t i) const { return list ? list[i] : i; }
    __device__ __forceinline__ bool match(int64_t g) const
    {
        const int32_t v = code[g];
        return v >= 0 && v < 64 && ((mask >> v) & 1ull);
    }
};

// One block of 1024 threads; thread i scans a contiguous chunk, the chunk
// counts are scanned in LDS, then every thread writes its matches in order.
__global__ __launch_bounds__(1024) void select_kernel(SelSrc S, int64_t* out, int64_t* out_count)
{
    __shared__ int64_t cnt[1024];
    const int tid = threadIdx.x;
    const int64_t n = S.len();
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t b = tid * chunk;
    const int64_t e = min(n, b + chunk);
    int64_t c = 0;
    for (int64_t i = b; i < e; ++i) c += S.match(S.item(i)) ? 1 : 0;
    cnt[tid] = c;
    __syncthreads();
    // Hillis-Steele inclusive scan
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t add = tid >= off ? cnt[tid - off] : 0;
        __syncthreads();
        cnt[tid] += add;
        __syncthreads();
    }
    int64_t pos = cnt[tid] - c;
    for (int64_t i = b; i < e; ++i) {
        const int64_t g = S.item(i);
        if (S.match(g)) out[pos++] = g;
    }
    if (tid == 1023) *out_count = cnt[1023];
}

// Multi-block version (with workspace): block b owns the contiguous tile
// [b * tile, (b + 1) * tile) of the candidate positions (sized on the host
// from the largest length).  Pass 1 counts each tile's matches, pass 2 turns
// the counts into tile offsets (one block), pass 3 writes every tile's
// matches in order: 256 positions at a time, the place of a match from a
// ballot within its wave plus the counts of the waves before.
constexpr int kSelThreads = 256;
constexpr int kSelMaxBlocks = 1024;

__global__ __launch_bounds__(kSelThreads) void select_count_kernel(SelSrc S, int64_t tile,
                                                                   int64_t* counts)
{
    __shared__ int64_t part[kSelThreads / 64];
    const int64_t n = S.len();
    const int64_t b0 = int64_t(blockIdx.x) * tile;
    const int64_t e0 = min(n, b0 + tile);
    int64_t c = 0;
    for (int64_t i = b0 + threadIdx.x; i < e0; i += kSelThreads) c += S.match(S.item(i)) ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (__lane_id() == 0) part[threadIdx.x / 64] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < kSelThreads / 64; ++w) t += part[w];
        counts[blockIdx.x] = t;
    }
}

// exclusive scan of the block counts in place; the total to *out_count
__global__ __launch_bounds__(kSelMaxBlocks) void select_scan_kernel(int64_t* counts, int nblocks,
                                                                    int64_t* out_count)
{
    __shared__ int64_t s[kSelMaxBlocks];
    const int t = threadIdx.x;
    const int64_t mine = t < nblocks ? counts[t] : 0;
    s[t] = mine;
    __syncthreads();
    for (int off = 1; off < kSelMaxBlocks; off <<= 1) {
        const int64_t add = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    if (t < nblocks) counts[t] = s[t] - mine;
    if (t == kSelMaxBlocks - 1) *out_count = s[t];
}

__global__ __launch_bounds__(kSelThreads) void select_write_kernel(SelSrc S, int64_t tile,
                                                                   const int64_t* offsets,
                                                                   int64_t* out)
{
    __shared__ int64_t wsum[kSelThreads / 64];
    const int64_t n = S.len();
    const int64_t b0 = int64_t(blockIdx.x) * tile;
    const int64_t e0 = min(n, b0 + tile);
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    int64_t base = offsets[blockIdx.x];
    for (int64_t c0 = b0; c0 < e0; c0 += kSelThreads) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t g = i < e0 ? S.item(i) : 0;
        const bool m = i < e0 && S.match(g);
        const unsigned long long bal = __ballot(m);
        if (lane == 0) wsum[wave] = __popcll(bal);
        __syncthreads();
        int64_t before = 0, total = 0;
        for (int w = 0; w < kSelThreads / 64; ++w) {
            before += w < wave ? wsum[w] : 0;
            total += wsum[w];
        }
        if (m) out[base + before + __popcll(bal & ((1ull << lane) - 1ull))] = g;
        base += total;
        __syncthreads();
    }
}

static int select_blocks(int64_t n, int64_t* tile)
{
    int64_t nb = (n + kSelThreads - 1) / kSelThreads;
    if (nb > kSelMaxBlocks) nb = kSelMaxBlocks;
    if (nb < 1) nb = 1;
    *tile = (n + nb - 1) / nb;
    if (*tile < 1) *tile = 1;
    return int(nb);
}

static int launch_select(const SelSrc& S, int64_t* out_ids, int64_t* out_count, void* workspace,
                         size_t ws_bytes, hipStream_t stream)
{
    if (!workspace) {
        hipLaunchKernelGGL(select_kernel, dim3(1), dim3(1024), 0, stream, S, out_ids, out_count);
        return hipGetLastError() == hipSuccess ? NPHC_OK : NPHC_EHIP;
    }
    int64_t tile;
    const int nb = select_blocks(S.n, &tile);
    if (ws_bytes < size_t(nb) * sizeof(int64_t) || (reinterpret_cast<uintptr_t>(workspace) & 7))
        return NPHC_EWORKSPACE;
    int64_t* counts = static_cast<int64_t*>(workspace);
    hipLaunchKernelGGL(select_count_kernel, dim3(nb), dim3(kSelThreads), 0, stream, S, tile, counts);
    hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(kSelMaxBlocks), 0, stream, counts, nb,
                       out_count);
    hipLaunchKernelGGL(select_write_kernel, dim3(nb), dim3(kSelThreads), 0, stream, S, tile, counts,
                       out_ids);
    return hipGetLastError() == hipSuccess ? NPHC_OK : NPHC_EHIP;
}

}  // namespace nphc

extern "C" size_t nphc_select_workspace_size(int64_t num_items)
{
    if (num_items < 0) return 0;
    int64_t tile;
    return size_t(nphc::select_blocks(num_items, &tile)) * sizeof(int64_t);
}

extern "C" int nphc_select(const int32_t* code, int64_t num_items, uint64_t mask, int64_t* out_ids,
                           int64_t* out_count, void* workspace, size_t ws_bytes, hipStream_t stream)
{
    if (!code || !out_ids || !out_count || num_items < 0) return NPHC_EINVAL;
    const nphc::SelSrc S{code, nullptr, nullptr, num_items, mask};
    return nphc::launch_select(S, out_ids, out_count, workspace, ws_bytes, stream);
}

extern "C" int nphc_select_list(const int32_t* code, const int64_t* ids, int64_t count,
                                const int64_t* count_dev, uint64_t mask, int64_t* out_ids,
                                int64_t* out_count, void* workspace, size_t ws_bytes,
                                hipStream_t stream)
{
    if (!code || !ids || !out_ids || !out_count || count < 0) return NPHC_EINVAL;
    const nphc::SelSrc S{code, ids, count_dev, count, mask};
    return nphc::launch_select(S, out_ids, out_count, workspace, ws_bytes, stream);
}
