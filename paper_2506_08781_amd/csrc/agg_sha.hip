// The POSLO hot kernel (AVer steps SR-PRF-H-sum per entry, paper section
// "POSLO Parallel Batch Verification", SHA-256 instantiation): one entry per
// lane, x_t by one SHA-256 compression of the epoch's seed and j, the digest
// of m_t || x_t, raw digests summed into a 288-bit accumulator, then wave
// and workgroup reductions to one partial per workgroup.
#include "ctx.h"
#include "device_entry.h"

namespace poslo {

template <bool FAST, bool VEC>
__global__ __launch_bounds__(kAggShaBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_agg_ekeys_sha(
    BatchArgs a, uint32_t* partials) {
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t pos = (uint64_t)blockIdx.x * kAggShaBlock + threadIdx.x; pos < a.n;
         pos += (uint64_t)gridDim.x * kAggShaBlock) {
        if (skipped(a, pos)) continue;
        uint32_t xw[4], dig[8];
        one_time_seed_sha(a, pos, xw);
        digest_sha<FAST, VEC>(entry_view(a, pos), xw, dig);
        acc288_add256(acc, dig);
    }
    block_reduce288_store<kAggShaBlock>(acc, partials + (uint64_t)blockIdx.x * 9);
}

int launch_agg_sha(int layout, uint32_t grid, const void* args, uint32_t* partials, hipStream_t s) {
    const BatchArgs& a = *static_cast<const BatchArgs*>(args);
    if (layout == 2)
        hipLaunchKernelGGL((k_agg_ekeys_sha<true, true>), dim3(grid), dim3(kAggShaBlock), 0, s, a, partials);
    else if (layout == 1)
        hipLaunchKernelGGL((k_agg_ekeys_sha<true, false>), dim3(grid), dim3(kAggShaBlock), 0, s, a, partials);
    else
        hipLaunchKernelGGL((k_agg_ekeys_sha<false, false>), dim3(grid), dim3(kAggShaBlock), 0, s, a, partials);
    return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
}

}  // namespace poslo
