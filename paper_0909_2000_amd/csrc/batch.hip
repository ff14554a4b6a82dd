// Batched alignment plots: many pairs of uneven m, n and w in a few
// persistent launches.
//
// The host builds a job table (one entry per plot: code arrays, geometry,
// outputs, and the index of the job's first unit in its group's unit list).
// Jobs fall into three groups by window class (up to 32 rows, 64 rows, 128
// rows), and each group runs as one persistent launch of a kernel that holds
// only its classes' unit code, so each runs at the occupancy of its own
// largest class: four waves per SIMD up to 32 rows, three at 64 rows, and
// the 128-row class with every strip split over two waves of a workgroup
// (three waves per SIMD, as in the single-plot kernel) instead of two waves
// per SIMD for a kernel that holds every class.  A grid sized to the
// resident capacity of the device loops: each wave (split: workgroup) takes
// the next unit index from a device-wide atomic counter (work stealing),
// finds its job by binary search over the jobs' first-unit indices, and
// combs that unit (64 strips x 2 y-tiles) with the same per-unit code as the
// single-plot kernel.  Within a group, every job's tile pairs but the last
// come first, by decreasing unit cost, then the jobs' last pairs (each split
// evenly over its two tiles, so usually shorter), again by decreasing cost:
// the tail of the queue holds the cheapest units.  Windows up to 128
// run here; longer windows run as separate single-plot launches on the same
// stream.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "kernels.hpp"
#include "seaweed_unit.hpp"

namespace wlcs {
namespace {

template <int WC, bool EXACT, bool SP, int PART = 0>
__device__ __forceinline__ void run_unit(const JobDesc& jd, int64_t local, uint32_t* ring, uint32_t* stage,
                                         uint32_t* hand = nullptr) {
    // pair-major within an entry, as in the single-plot kernel: unit local
    // is strip block local % nblocks of the entry's pair local / nblocks
    const int64_t nblocks = (jd.g.rows + 63) / 64;
    const int64_t q = local / nblocks;
    const int64_t sb = local - q * nblocks;
    const int pr = jd.pr0 + (int)q;
    comb_unit<WC, EXACT, 1, SP, false, PART>(jd.xf, jd.yg32, jd.out, jd.bm32, jd.indel, SP ? jd.dots : nullptr,
                                             SP ? jd.dot_count : nullptr, jd.g, sb, pr, ring, stage, hand);
}

// the job whose unit range holds u (jobs[k].unit0 ascending, jobs[0].unit0 == 0)
__device__ __forceinline__ int find_job(const JobDesc* __restrict__ jobs, int32_t njobs, int64_t u) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].unit0 <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int64_t uniform_u64(unsigned long long v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (int64_t)(((unsigned long long)hi << 32) | lo);
}

constexpr int group_class(int grp) { return grp == 0 ? 32 : 64; }

// Groups 0 (classes 16 and 32) and 1 (class 64): one wave per unit.
template <int GRP, bool SP>
__global__ __launch_bounds__(64, group_waves_per_simd(GRP)) void batch_kernel(const JobDesc* __restrict__ jobs,
                                                                             int32_t njobs, int64_t total_units,
                                                                             unsigned long long* __restrict__ counter) {
    __shared__ uint32_t ring[ring_words(group_class(GRP)) * 64];
    __shared__ uint32_t stage[stage_dwords(group_class(GRP))];
    const int lane = threadIdx.x;
    for (;;) {
        unsigned long long v = 0;
        if (lane == 0) v = atomicAdd(counter, 1ull);
        const int64_t u = uniform_u64(v);  // lane 0 holds the ticket
        if (u >= total_units) break;       // queue drained: every wave leaves
        const JobDesc jd = jobs[find_job(jobs, njobs, u)];
        const int64_t local = u - jd.unit0;
        if constexpr (GRP == 0) {
            switch (jd.variant) {
                case kBatch16: run_unit<16, true, SP>(jd, local, ring, stage); break;
                case kBatch16Short: run_unit<16, false, SP>(jd, local, ring, stage); break;
                case kBatch32: run_unit<32, true, SP>(jd, local, ring, stage); break;
                default: run_unit<32, false, SP>(jd, local, ring, stage); break;
            }
        } else {
            if (jd.variant == kBatch64) run_unit<64, true, SP>(jd, local, ring, stage);
            else run_unit<64, false, SP>(jd, local, ring, stage);
        }
    }
}

// Group 2 (class 128): every unit on the two waves of a workgroup, the upper
// rows on wave 0 and the lower rows on wave 1.  Wave 0 takes the ticket and
// passes it on through LDS.  The barrier after each ticket is written also
// keeps the units apart: wave 0 starts a unit only once wave 1 has left the
// previous one (its flushes and LDS ring included).  The ticket slot
// alternates, so a ticket is never overwritten before wave 1 has read it.
template <bool SP>
__global__ __launch_bounds__(128, min_waves_per_simd_split(128)) void batch_kernel_split(
    const JobDesc* __restrict__ jobs, int32_t njobs, int64_t total_units, unsigned long long* __restrict__ counter) {
    __shared__ uint32_t ring[ring_words(128) * 64];
    __shared__ uint32_t stage[stage_dwords(128, 1)];
    __shared__ uint32_t hand[kDlHandDwords];
    __shared__ unsigned long long ticket[2];
    const bool upper = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0;
    for (int slot = 0;; slot ^= 1) {
        if (threadIdx.x == 0) ticket[slot] = atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t u = uniform_u64(ticket[slot]);
        if (u >= total_units) break;  // the same ticket in both waves: both leave
        const JobDesc jd = jobs[find_job(jobs, njobs, u)];
        const int64_t local = u - jd.unit0;
        const bool exact = jd.variant == kBatch128;
        if (upper) {
            if (exact) run_unit<128, true, SP, 1>(jd, local, ring, stage, hand);
            else run_unit<128, false, SP, 1>(jd, local, ring, stage, hand);
        } else {
            if (exact) run_unit<128, true, SP, 2>(jd, local, ring, stage, hand);
            else run_unit<128, false, SP, 2>(jd, local, ring, stage, hand);
        }
    }
}

// Scratch of the allocation-free batch (wlcs_batch_noalloc): the job table,
// the groups' work counters and the dot counters' addresses of one batch.
// Each device holds its own copy for the life of the process; host code uses
// the address hipGetSymbolAddress gives for the device (scratch_address),
// never this name.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

// One piece of the host bytes to place in the scratch, carried in the
// launch's own argument: nothing on the host has to outlive the call, and
// no copy engine or staging buffer is involved.
struct UploadChunk {
    uint32_t off;    // byte offset in the destination (a multiple of 4)
    uint32_t words;  // dwords carried
    uint32_t data[kUploadChunkWords];
};
static_assert(sizeof(UploadChunk) + sizeof(void*) <= 4096, "kernel arguments");

__global__ void upload_chunk(uint8_t* __restrict__ dst, UploadChunk c) {
    uint32_t* d = (uint32_t*)(dst + c.off);
    for (uint32_t k = threadIdx.x; k < c.words; k += blockDim.x) d[k] = c.data[k];
}

__global__ void zero_counter(unsigned long long* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0ull;
}

__global__ void zero_each(unsigned long long* const* __restrict__ ptrs, int32_t n) {
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) *ptrs[k] = 0ull;
}

template <int GRP>
void launch_group(const JobDesc* jobs_dev, int32_t njobs, int64_t total_units, unsigned long long* counter,
                  int32_t grid, bool sparse, hipStream_t stream) {
    if constexpr (GRP == 2) {
        if (sparse)
            hipLaunchKernelGGL(batch_kernel_split<true>, dim3((uint32_t)grid), dim3(128), 0, stream, jobs_dev, njobs,
                               total_units, counter);
        else
            hipLaunchKernelGGL(batch_kernel_split<false>, dim3((uint32_t)grid), dim3(128), 0, stream, jobs_dev, njobs,
                               total_units, counter);
    } else {
        if (sparse)
            hipLaunchKernelGGL((batch_kernel<GRP, true>), dim3((uint32_t)grid), dim3(64), 0, stream, jobs_dev, njobs,
                               total_units, counter);
        else
            hipLaunchKernelGGL((batch_kernel<GRP, false>), dim3((uint32_t)grid), dim3(64), 0, stream, jobs_dev, njobs,
                               total_units, counter);
    }
}

}  // namespace

hipError_t launch_batch(int group, const JobDesc* jobs_dev, int32_t njobs, int64_t total_units,
                        unsigned long long* counter, int32_t grid, bool sparse, hipStream_t stream) {
    if (total_units <= 0 || njobs <= 0) return hipSuccess;
    if (group < 0 || group >= kBatchGroups || grid <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(zero_counter, dim3(1), dim3(64), 0, stream, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (group) {
        case 0: launch_group<0>(jobs_dev, njobs, total_units, counter, grid, sparse, stream); break;
        case 1: launch_group<1>(jobs_dev, njobs, total_units, counter, grid, sparse, stream); break;
        default: launch_group<2>(jobs_dev, njobs, total_units, counter, grid, sparse, stream); break;
    }
    return hipGetLastError();
}

hipError_t launch_zero_each(unsigned long long* const* ptrs, int32_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int32_t blocks = std::min<int32_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_each, dim3((uint32_t)blocks), dim3(256), 0, stream, ptrs, n);
    return hipGetLastError();
}

hipError_t scratch_address(int device, uint8_t** ptr) {
    static std::mutex mu;
    static uint8_t* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        // the caller has made `device` current; each device has its own copy
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = (uint8_t*)p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

hipError_t launch_upload(uint8_t* dst, const uint8_t* src, size_t bytes, hipStream_t stream) {
    if (bytes % 4) return hipErrorInvalidValue;
    for (size_t off = 0; off < bytes; off += 4 * kUploadChunkWords) {
        UploadChunk c;
        c.off = (uint32_t)off;
        c.words = (uint32_t)std::min<size_t>(kUploadChunkWords, (bytes - off) / 4);
        memcpy(c.data, src + off, 4 * (size_t)c.words);
        hipLaunchKernelGGL(upload_chunk, dim3(1), dim3(256), 0, stream, dst, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace wlcs
