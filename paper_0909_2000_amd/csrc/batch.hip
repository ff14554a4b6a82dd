// Batched alignment plots: many pairs of uneven m, n and w in one persistent
// launch.
//
// The host builds a job table (one entry per plot: code arrays, geometry,
// outputs, and the index of the job's first unit in one global unit list).  A
// grid sized to the resident capacity of the device loops: each wave takes the
// next unit index from a device-wide atomic counter (work stealing), finds its
// job by binary search over the jobs' first-unit indices, and combs that unit
// (64 strips x 2 y-tiles) with the same per-unit code as the single-plot
// kernel.  Jobs are ordered by decreasing unit cost so the tail of the queue
// holds the cheapest units.  Windows up to 128 run here; longer windows run
// as separate single-plot launches on the same stream.
#include <algorithm>

#include "kernels.hpp"
#include "seaweed_unit.hpp"

namespace wlcs {
namespace {

template <int WC, bool EXACT, bool SP>
__device__ __forceinline__ void run_unit(const JobDesc& jd, int64_t local, uint32_t* ring, uint32_t* stage) {
    // pair-major within a job, as in the single-plot kernel
    const int64_t nblocks = (jd.g.rows + 63) / 64;
    const int pr = (int)(local / nblocks);
    const int64_t sb = local - (int64_t)pr * nblocks;
    comb_unit<WC, EXACT, 1, SP>(jd.xf, jd.yg32, jd.out, jd.bm32, jd.indel, SP ? jd.dots : nullptr,
                                SP ? jd.dot_count : nullptr, jd.g, sb, pr, ring, stage);
}

template <bool SP>
__global__ __launch_bounds__(64, 2) void batch_kernel(const JobDesc* __restrict__ jobs, int32_t njobs,
                                                      int64_t total_units, unsigned long long* __restrict__ counter) {
    __shared__ uint32_t ring[ring_words(128) * 64];
    __shared__ uint32_t stage[stage_dwords(128)];
    const int lane = threadIdx.x;
    for (;;) {
        uint32_t ulo = 0, uhi = 0;
        if (lane == 0) {
            const unsigned long long v = atomicAdd(counter, 1ull);
            ulo = (uint32_t)v;
            uhi = (uint32_t)(v >> 32);
        }
        // lane 0 holds the ticket; make it wave-uniform (scalar registers)
        const unsigned long long u = ((unsigned long long)__builtin_amdgcn_readfirstlane(uhi) << 32) |
                                     __builtin_amdgcn_readfirstlane(ulo);
        if ((int64_t)u >= total_units) break;  // queue drained: every wave leaves
        // job whose unit range holds u (jobs[k].unit0 ascending)
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].unit0 <= (int64_t)u) lo = mid;
            else hi = mid - 1;
        }
        const JobDesc jd = jobs[lo];
        const int64_t local = (int64_t)u - jd.unit0;
        switch (jd.variant) {
            case 0: run_unit<16, true, SP>(jd, local, ring, stage); break;
            case 1: run_unit<32, true, SP>(jd, local, ring, stage); break;
            case 2: run_unit<64, true, SP>(jd, local, ring, stage); break;
            case 3: run_unit<128, true, SP>(jd, local, ring, stage); break;
            default: run_unit<128, false, SP>(jd, local, ring, stage); break;
        }
    }
}

__global__ void zero_counter(unsigned long long* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0ull;
}

__global__ void zero_each(unsigned long long* const* __restrict__ ptrs, int32_t n) {
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) *ptrs[k] = 0ull;
}

}  // namespace

int batch_variant(int w) {
    switch (w) {
        case 16: return 0;
        case 32: return 1;
        case 64: return 2;
        case 128: return 3;
        default: return 4;  // any other w <= 128
    }
}

hipError_t launch_batch(const JobDesc* jobs_dev, int32_t njobs, int64_t total_units, unsigned long long* counter,
                        int32_t grid, bool sparse, hipStream_t stream) {
    if (total_units <= 0 || njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_counter, dim3(1), dim3(64), 0, stream, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (sparse)
        hipLaunchKernelGGL(batch_kernel<true>, dim3((uint32_t)grid), dim3(64), 0, stream, jobs_dev, njobs,
                           total_units, counter);
    else
        hipLaunchKernelGGL(batch_kernel<false>, dim3((uint32_t)grid), dim3(64), 0, stream, jobs_dev, njobs,
                           total_units, counter);
    return hipGetLastError();
}

hipError_t launch_zero_each(unsigned long long* const* ptrs, int32_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int32_t blocks = std::min<int32_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_each, dim3((uint32_t)blocks), dim3(256), 0, stream, ptrs, n);
    return hipGetLastError();
}

}  // namespace wlcs
