// The POSLO hot kernel (AVer steps SR-PRF-H-sum per entry, paper section
// "POSLO Parallel Batch Verification", SHA-256 instantiation): one entry per
// lane, x_t by one SHA-256 compression of the epoch's seed and j, the digest
// of m_t || x_t, raw digests summed into a 288-bit accumulator, then wave
// and workgroup reductions to one partial per workgroup.
#include "ctx.h"
#include "device_entry.h"
#include "fourq.h"
#include "device_verify.h"

namespace poslo {

// LAYOUT 2: 16-byte aligned, length divisible by 16 (128-byte line loads);
// 1: 4-byte aligned, length divisible by 4; 0: any length and alignment
// (word loads funnel-shifted to the message's alignment).  EMIT: also store
// every entry's e_t = H(m_t || x_t) mod q (eight LE words) and the bytes of
// x_t (four LE words, when x_out is set).
template <int LAYOUT, bool EMIT = false>
__global__ __launch_bounds__(kAggShaBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_agg_ekeys_sha(
    BatchArgs a, uint32_t* partials, uint32_t* e_out, uint32_t* x_out) {
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t pos = (uint64_t)blockIdx.x * kAggShaBlock + threadIdx.x; pos < a.n;
         pos += (uint64_t)gridDim.x * kAggShaBlock) {
        if (skipped(a, pos)) continue;
        uint32_t xw[4], dig[8];
        one_time_seed_sha(a, pos, xw);
        if constexpr (LAYOUT == 0)
            digest_sha_any(entry_view(a, pos), a.end, xw, dig);
        else
            digest_sha<true, LAYOUT == 2>(entry_view(a, pos), xw, dig);
        acc288_add256(acc, dig);
        if constexpr (EMIT) {
            uint32_t e[8];
            if (a.emit_fq)
                scN_reduce<8>(e, dig);
            else
                sc_reduce256(e, dig);
#pragma unroll
            for (int w = 0; w < 8; w++) e_out[pos * 8 + w] = e[w];
            if (x_out)
#pragma unroll
                for (int w = 0; w < 4; w++) x_out[pos * 4 + w] = bswap32(xw[w]);
        }
    }
    block_reduce288_store<kAggShaBlock>(acc, partials + (uint64_t)blockIdx.x * 9);
}

template <bool EMIT>
static int launch_sha(int layout, uint32_t grid, const BatchArgs& a, uint32_t* partials, uint32_t* e_out,
                      uint32_t* x_out, hipStream_t s) {
    if (layout == 2)
        hipLaunchKernelGGL((k_agg_ekeys_sha<2, EMIT>), dim3(grid), dim3(kAggShaBlock), 0, s, a, partials, e_out,
                           x_out);
    else if (layout == 1)
        hipLaunchKernelGGL((k_agg_ekeys_sha<1, EMIT>), dim3(grid), dim3(kAggShaBlock), 0, s, a, partials, e_out,
                           x_out);
    else
        hipLaunchKernelGGL((k_agg_ekeys_sha<0, EMIT>), dim3(grid), dim3(kAggShaBlock), 0, s, a, partials, e_out,
                           x_out);
    return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
}

int launch_agg_sha(int layout, uint32_t grid, const void* args, uint32_t* partials, hipStream_t s) {
    return launch_sha<false>(layout, grid, *static_cast<const BatchArgs*>(args), partials, nullptr, nullptr, s);
}

int launch_agg_sha_emit(int layout, uint32_t grid, const void* args, uint32_t* partials, uint32_t* e_out,
                        uint32_t* x_out, hipStream_t s) {
    return launch_sha<true>(layout, grid, *static_cast<const BatchArgs*>(args), partials, e_out, x_out, s);
}

}  // namespace poslo
