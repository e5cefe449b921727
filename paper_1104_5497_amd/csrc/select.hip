// select.hip -- ordered stream compaction of item ids by endpoint code.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace nphc {

// One block of 1024 threads; thread i scans a contiguous chunk, the chunk
// counts are scanned in LDS, then every thread writes its matches in order.
__global__ __launch_bounds__(1024) void select_kernel(const int32_t* code, int64_t n, uint64_t mask,
                                                      int64_t* out, int64_t* out_count)
{
    __shared__ int64_t cnt[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t b = tid * chunk;
    const int64_t e = min(n, b + chunk);
    int64_t c = 0;
    for (int64_t i = b; i < e; ++i) {
        const int32_t v = code[i];
        c += (v >= 0 && v < 64 && ((mask >> v) & 1ull)) ? 1 : 0;
    }
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
        const int32_t v = code[i];
        if (v >= 0 && v < 64 && ((mask >> v) & 1ull)) out[pos++] = i;
    }
    if (tid == 1023) *out_count = cnt[1023];
}

}  // namespace nphc

extern "C" size_t nphc_select_workspace_size(int64_t num_items)
{
    (void)num_items;
    return 0;
}

extern "C" int nphc_select(const int32_t* code, int64_t num_items, uint64_t mask, int64_t* out_ids,
                           int64_t* out_count, void* workspace, size_t ws_bytes, hipStream_t stream)
{
    (void)workspace;
    (void)ws_bytes;
    if (!code || !out_ids || !out_count || num_items < 0) return NPHC_EINVAL;
    hipLaunchKernelGGL(nphc::select_kernel, dim3(1), dim3(1024), 0, stream, code, num_items, mask,
                       out_ids, out_count);
    if (hipGetLastError() != hipSuccess) return NPHC_EHIP;
    return NPHC_OK;
}
