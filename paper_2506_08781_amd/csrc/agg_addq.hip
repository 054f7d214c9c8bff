// The POSLO++ hot kernel (AVer steps SR-PRF-H-sum per entry with H = Add_q,
// paper table "Instantiations of POSLO schemes"): e_t = LE(m_t) + LE(x_t).
// For messages of at most 31 bytes that sum is below 2^249 < q, so it is e_t
// itself, and the digests go unreduced into the 288-bit accumulator as the
// other instantiations' do.  Per entry: x_t by one AES under the epoch's
// hoisted MMO schedule (the second block of PRF_0(x_0[i] || LE32(j)), as in
// the POSLO+ kernel) and at most 31 message bytes, so the AES rounds' LDS
// lookups bound the kernel rather than HBM.
//
// Work unit: a wave takes the 64 log positions t = 64u .. 64u + 63 (those in
// the batch).  With n2 >= 64 a unit lies in one epoch, so its 44 round-key
// words are loaded once per unit into scalar registers (SGPR operands of the
// round xors) instead of by every lane; smaller epochs take the per-lane form.
// Consecutive waves take consecutive units, so a wave instruction's message
// loads cover one contiguous span.
#include "ctx.h"
#include "aes_perm.h"
#include "device_entry.h"

namespace poslo {

namespace {

constexpr int kAddqBlock = 1024;

// a word that is the same in every lane, through the scalar unit when its
// address is uniform (constant address space: read-only for the kernel)
__device__ __forceinline__ uint32_t uload(const uint32_t* p) {
    return *reinterpret_cast<const __attribute__((address_space(4))) uint32_t*>(reinterpret_cast<uintptr_t>(p));
}

// UNI: n2 >= 64 (a unit lies in one epoch).  EMIT: also store e_t (eight
// LE words; all-ones words for a message longer than 31 bytes) and x_t.
template <int LAYOUT, bool UNI, bool EMIT>
__global__ __launch_bounds__(kAddqBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_agg_addq(
    BatchArgs a, uint32_t* partials, uint32_t* e_out, uint32_t* x_out) {
    __shared__ uint32_t lds[2 * 256 * 32];
    perm_tables_fill<2, 32>(lds);
    __syncthreads();
    const PermTables<2, 32> tb = perm_tables<2, 32>(lds);
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    bool bad = false;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t waves_per_block = kAddqBlock / 64;
    const uint32_t wave =
        (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * waves_per_block + (threadIdx.x >> 6)));
    const uint64_t nwaves = (uint64_t)gridDim.x * waves_per_block;
    const uint64_t t_end = a.t0 + a.n;
    const uint64_t u_end = (t_end + 63) >> 6;
    const uint64_t jmask = (1ull << a.log2_n2) - 1;
    for (uint64_t u = (a.t0 >> 6) + wave; u < u_end; u += nwaves) {
        const uint64_t t = (u << 6) | lane;
        if (t < a.t0 || t >= t_end) continue;
        const uint64_t pos = t - a.t0;
        if (skipped(a, pos)) continue;
        // the message first, so its loads are in flight during the AES
        const uint8_t* m;
        uint64_t L;
        if (LAYOUT == 0 && a.offsets) {
            const uint64_t o0 = gload(a.offsets + pos), o1 = gload(a.offsets + pos + 1);
            m = a.data + o0;
            L = o1 - o0;
        } else {
            m = a.data + pos * a.msg_len;
            L = a.msg_len;
        }
        if (L > kAddqMaxLen) {
            bad = true;
            if constexpr (EMIT)
#pragma unroll
                for (int w = 0; w < 8; w++) e_out[pos * 8 + w] = 0xffffffffu;
            continue;
        }
        uint32_t mw[8];
        addq_message<LAYOUT>(m, (uint32_t)L, mw);
        const uint32_t j = (uint32_t)(t & jmask);
        uint32_t x[4] = {j, 0u, 0u, 0u};
        if constexpr (UNI) {
            const uint32_t* row = a.tab + (((u << 6) >> a.log2_n2) - a.epoch_first) * kEpochWords;
            uint32_t rk[44];
#pragma unroll
            for (int k = 0; k < 44; k++) rk[k] = uload(row + k);
            penc_rk(tb, rk, x);
        } else {
            penc_rk(tb, a.tab + ((t >> a.log2_n2) - a.epoch_first) * kEpochWords, x);
        }
        x[0] ^= j;
        x[3] &= a.xmask;
        uint32_t e[8];
        addq_digest(mw, x, e);
        acc288_add256(acc, e);
        if constexpr (EMIT) {
#pragma unroll
            for (int w = 0; w < 8; w++) e_out[pos * 8 + w] = e[w];
            if (x_out)
#pragma unroll
                for (int w = 0; w < 4; w++) x_out[pos * 4 + w] = x[w];
        }
    }
    if (bad) *a.bad = 1u;  // every writer stores the same value
    __syncthreads();       // every lane is done with the tables
    block_reduce288_scratch<kAddqBlock>(acc, partials + (uint64_t)blockIdx.x * 9, lds);
}

template <bool UNI, bool EMIT>
void launch_layout(int layout, uint32_t grid, const BatchArgs& a, uint32_t* partials, uint32_t* e_out,
                   uint32_t* x_out, hipStream_t s) {
    if (layout == 2)
        hipLaunchKernelGGL((k_agg_addq<2, UNI, EMIT>), dim3(grid), dim3(kAddqBlock), 0, s, a, partials, e_out, x_out);
    else if (layout == 1)
        hipLaunchKernelGGL((k_agg_addq<1, UNI, EMIT>), dim3(grid), dim3(kAddqBlock), 0, s, a, partials, e_out, x_out);
    else
        hipLaunchKernelGGL((k_agg_addq<0, UNI, EMIT>), dim3(grid), dim3(kAddqBlock), 0, s, a, partials, e_out, x_out);
}

}  // namespace

int agg_addq_block() { return kAddqBlock; }

int launch_agg_addq(int layout, uint32_t grid, const void* args, uint32_t* partials, uint32_t* e_out,
                    uint32_t* x_out, hipStream_t s) {
    const BatchArgs& a = *static_cast<const BatchArgs*>(args);
    if (layout < 0 || layout > 2 || !a.bad) return POSLO_E_INVAL;
    const bool uni = a.log2_n2 >= 6;
    if (uni) {
        if (e_out) launch_layout<true, true>(layout, grid, a, partials, e_out, x_out, s);
        else launch_layout<true, false>(layout, grid, a, partials, e_out, x_out, s);
    } else {
        if (e_out) launch_layout<false, true>(layout, grid, a, partials, e_out, x_out, s);
        else launch_layout<false, false>(layout, grid, a, partials, e_out, x_out, s);
    }
    return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
}

}  // namespace poslo
