// The POSLO+ hot kernel (AVer steps SR-PRF-H-sum per entry, paper section
// "POSLO Parallel Batch Verification"): one entry per lane, x_t by one AES
// under the epoch's hoisted schedule, MDC-2-AES-128 over m_t || x_t with the
// key schedule expanded on the fly for every block (the two MDC-2 lanes
// interleaved for independent work), raw digests summed into a 288-bit
// accumulator, then wave and workgroup reductions to one partial per
// workgroup.
//
// The paper keeps a single T-table copy in shared memory.  On gfx950 the
// 160 KB LDS affords bank-replicated copies, which removes most bank
// conflicts of the random table lookups; the variants below trade LDS
// footprint (and so occupancy) against conflicts and rotate instructions.
#include "ctx.h"
#include "aes_perm.h"
#include "device_entry.h"
#include "fourq.h"
#include "device_verify.h"

namespace poslo {

template <int NT, int C, int BLOCK, bool FAST>
__global__ __launch_bounds__(BLOCK) void k_agg_ekeys_aes(BatchArgs a, uint32_t* partials) {
    __shared__ uint32_t lds[NT * 256 * C];
    lds_tables_fill<NT, C>(lds);
    __syncthreads();
    LdsTables<NT, C> tb{lds + (threadIdx.x % C)};
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t pos = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; pos < a.n; pos += (uint64_t)gridDim.x * BLOCK) {
        if (skipped(a, pos)) continue;
        uint32_t x[4], dig[8];
        one_time_seed_aes(tb, a, pos, x);
        digest_mdc2<FAST>(tb, entry_view(a, pos), x, dig);
        acc288_add256(acc, dig);
    }
    block_reduce288_store<BLOCK>(acc, partials + (uint64_t)blockIdx.x * 9);
}

// The same computation over the byte-addressed 64-copy layout (aes_perm.h):
// one v_perm_b32 per lookup address, fully unrolled rounds, three-input xors.

// one MDC-2 block: (h, h') <- (E_h(m) ^ m, E_h'(m) ^ m) with the half swap
template <int NT, int CP>
__device__ __forceinline__ void mdc2_block_perm(const PermTables<NT, CP>& tb, uint32_t h[4], uint32_t hp[4],
                                                const uint32_t m[4], bool first) {
    uint32_t sa[4] = {m[0], m[1], m[2], m[3]}, sb[4] = {m[0], m[1], m[2], m[3]};
    if (first)
        penc2_rk(tb, c_iv.a, sa, c_iv.b, sb);  // keyed by the constant IVs
    else
        penc2_otf(tb, h, sa, hp, sb);
#pragma unroll
    for (int w = 0; w < 4; w++) {
        sa[w] ^= m[w];
        sb[w] ^= m[w];
    }
    h[0] = sa[0], h[1] = sa[1], h[2] = sb[2], h[3] = sb[3];
    hp[0] = sb[0], hp[1] = sb[1], hp[2] = sa[2], hp[3] = sa[3];
}

// MDC-2 over m || x.  FAST (16-byte aligned, length divisible by 16): each
// 128-byte line of the message is loaded once, all eight blocks at a time,
// so no line has to survive in the cache between block loads.  LEAN loads
// four blocks (64 bytes, one L2 sector) at a time instead and
// derives x_t only for the final block: about half the live registers, so
// twice the resident waves where LDS allows.  xf(x) writes x_t.
template <int NT, int CP, bool FAST, bool LEAN, class XF>
__device__ __forceinline__ void digest_mdc2_perm(const PermTables<NT, CP>& tb, const EntryView& v, const uint8_t* end,
                                                 const XF& xf, uint32_t dig[8]) {
    uint32_t h[4], hp[4];
    uint64_t b = 0;
    if constexpr (FAST) {
        const uint4* p = reinterpret_cast<const uint4*>(v.m);
        uint64_t lines = v.L / 128;
        for (uint64_t ln = 0; ln < lines; ln++) {
            if constexpr (LEAN) {
#pragma unroll 1
                for (int k = 0; k < 8; k += 4) {
                    uint4 q[4];
#pragma unroll
                    for (int r = 0; r < 4; r++) q[r] = p[8 * ln + k + r];
#pragma unroll 1
                    for (int r = 0; r < 4; r++, b++) {
                        const uint32_t m[4] = {q[0].x, q[0].y, q[0].z, q[0].w};
                        mdc2_block_perm(tb, h, hp, m, b == 0);
#pragma unroll
                        for (int u = 0; u < 3; u++) q[u] = q[u + 1];
                    }
                }
            } else {
                uint4 q[8];
#pragma unroll
                for (int k = 0; k < 8; k++) q[k] = p[8 * ln + k];
#pragma unroll 1
                for (int k = 0; k < 8; k++, b++) {
                    uint32_t m[4] = {q[0].x, q[0].y, q[0].z, q[0].w};
                    mdc2_block_perm(tb, h, hp, m, b == 0);
#pragma unroll
                    for (int r = 0; r < 7; r++) q[r] = q[r + 1];
                }
            }
        }
        for (; 16 * b < v.L; b++) {
            uint4 u = p[b];
            uint32_t m[4] = {u.x, u.y, u.z, u.w};
            mdc2_block_perm(tb, h, hp, m, b == 0);
        }
        uint32_t x[4];
        xf(x);
        mdc2_block_perm(tb, h, hp, x, b == 0);  // the final block is x_t
    } else {
        // any length and alignment: word loads funnel-shifted to the
        // message's alignment, bounded by the end of the data buffer
        uint32_t x[4];
        digest_mdc2_any_late(tb, v, end, xf, x, dig, Mdc2BlockPerm{});
        return;
    }
#pragma unroll
    for (int w = 0; w < 4; w++) {
        dig[w] = h[w];
        dig[4 + w] = hp[w];
    }
}

// EMIT: also store every entry's e_t = H(m_t || x_t) mod q (eight LE words)
// and x_t (four LE words, when x_out is set); the hashing is the same code.
// CP: table copies (aes_perm.h).
template <int NT, int BLOCK, bool FAST, bool LEAN, int WPE, bool EMIT = false, int CP = 64>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) void k_agg_ekeys_aes_perm(
    BatchArgs a, uint32_t* partials, uint32_t* e_out, uint32_t* x_out) {
    // the kernel's only LDS allocation: tables first, then reduction scratch
    __shared__ uint32_t lds[NT * 256 * CP];
    perm_tables_fill<NT, CP>(lds);
    __syncthreads();
    const PermTables<NT, CP> tb = perm_tables<NT, CP>(lds);
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t pos = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; pos < a.n; pos += (uint64_t)gridDim.x * BLOCK) {
        if (skipped(a, pos)) continue;
        const uint64_t t = a.t0 + pos;
        const uint32_t j = (uint32_t)(t & ((1ull << a.log2_n2) - 1));
        const uint32_t* rk = a.tab + ((t >> a.log2_n2) - a.epoch_first) * kEpochWords;
        uint32_t xo[4];
        auto xf = [&](uint32_t x[4]) {
            x[0] = j, x[1] = 0u, x[2] = 0u, x[3] = 0u;
            penc_rk(tb, rk, x);
            x[0] ^= j;
            x[3] &= a.xmask;
            if constexpr (EMIT)
#pragma unroll
                for (int w = 0; w < 4; w++) xo[w] = x[w];
        };
        uint32_t dig[8];
        digest_mdc2_perm<NT, CP, FAST, LEAN>(tb, entry_view(a, pos), a.end, xf, dig);
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
                for (int w = 0; w < 4; w++) x_out[pos * 4 + w] = xo[w];
        }
    }
    __syncthreads();  // every lane is done with the tables
    block_reduce288_scratch<BLOCK>(acc, partials + (uint64_t)blockIdx.x * 9, lds);
}

static const AggVariant kVariants[] = {
    {"nt4_c1_b256", 4, 1, 256, 0},     {"nt4_c4_b256", 4, 4, 256, 0},   {"nt4_c8_b256", 4, 8, 256, 0},
    {"nt4_c16_b512", 4, 16, 512, 0},   {"nt4_c32_b1024", 4, 32, 1024, 0}, {"nt1_c16_b256", 1, 16, 256, 0},
    {"nt1_c32_b256", 1, 32, 256, 0},   {"nt1_c32_b512", 1, 32, 512, 0},  {"nt1_c64_b512", 1, 64, 512, 0},
    {"nt2_c32_b512", 2, 32, 512, 0},   {"perm2_c64_b1024", 2, 64, 1024, 1}, {"perm1_c64_b1024", 1, 64, 1024, 1},
    {"perm1_c64_b512", 1, 64, 512, 1}, {"perm2_c64_b512", 2, 64, 512, 1},
    {"perm2_lean_b1024", 2, 64, 1024, 1}, {"perm1_lean_b1024_w8", 1, 64, 1024, 1},
    {"perm1_lean_b512_w8", 1, 64, 512, 1},   {"perm2x32_lean_b1024_w8", 2, 32, 1024, 1},
    {"perm4x32_b1024", 4, 32, 1024, 1},      {"perm4x32_lean_b1024", 4, 32, 1024, 1},
};

int agg_aes_variant_count() { return (int)(sizeof kVariants / sizeof kVariants[0]); }
const AggVariant& agg_aes_variant(int v) { return kVariants[v]; }
// perm2x32_lean_b1024_w8: fastest in the sweep on MI355X (0.47 ms against
// 0.51 ms for perm1_lean_b1024_w8 at 2^20 x 256 B: the two-table layout
// needs a third of the rotations, and 32 copies keep it in 64 KB)
int agg_aes_default_variant() { return 17; }
size_t agg_aes_lds_bytes(int v) { return (size_t)kVariants[v].nt * 256 * kVariants[v].copies * 4; }

#define LAUNCH(NT, C, B)                                                                              \
    hipLaunchKernelGGL((k_agg_ekeys_aes<NT, C, B, true>), dim3(grid), dim3(B), 0, s, a, partials); \
    break

#define LAUNCHP(NT, B, LEAN, WPE)                                                                      \
    hipLaunchKernelGGL((k_agg_ekeys_aes_perm<NT, B, true, LEAN, WPE>), dim3(grid), dim3(B), 0, s, a, partials, \
                       nullptr, nullptr);                                                                   \
    break

int agg_aes_any_block() { return 1024; }

int launch_agg_aes(int v, bool fast, uint32_t grid, const void* args, uint32_t* partials, hipStream_t s) {
    const BatchArgs& a = *static_cast<const BatchArgs*>(args);
    if (!fast) {
        // any layout: the default variant's tables and shape with word loads
        hipLaunchKernelGGL((k_agg_ekeys_aes_perm<2, 1024, false, true, 8, false, 32>), dim3(grid), dim3(1024), 0,
                           s, a, partials, nullptr, nullptr);
        return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
    }
    switch (v) {
        case 0: LAUNCH(4, 1, 256);
        case 1: LAUNCH(4, 4, 256);
        case 2: LAUNCH(4, 8, 256);
        case 3: LAUNCH(4, 16, 512);
        case 4: LAUNCH(4, 32, 1024);
        case 5: LAUNCH(1, 16, 256);
        case 6: LAUNCH(1, 32, 256);
        case 7: LAUNCH(1, 32, 512);
        case 8: LAUNCH(1, 64, 512);
        case 9: LAUNCH(2, 32, 512);
        case 10: LAUNCHP(2, 1024, false, 4);
        case 11: LAUNCHP(1, 1024, false, 4);
        case 12: LAUNCHP(1, 512, false, 4);
        case 13: LAUNCHP(2, 512, false, 4);
        case 14: LAUNCHP(2, 1024, true, 4);
        case 15: LAUNCHP(1, 1024, true, 8);
        case 16: LAUNCHP(1, 512, true, 8);
        case 17:
            hipLaunchKernelGGL((k_agg_ekeys_aes_perm<2, 1024, true, true, 8, false, 32>), dim3(grid), dim3(1024), 0,
                               s, a, partials, nullptr, nullptr);
            break;
        case 18:
            hipLaunchKernelGGL((k_agg_ekeys_aes_perm<4, 1024, true, false, 4, false, 32>), dim3(grid), dim3(1024), 0,
                               s, a, partials, nullptr, nullptr);
            break;
        case 19:
            hipLaunchKernelGGL((k_agg_ekeys_aes_perm<4, 1024, true, true, 4, false, 32>), dim3(grid), dim3(1024), 0,
                               s, a, partials, nullptr, nullptr);
            break;
        default: return POSLO_E_INVAL;
    }
    return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
}

// The default variant (or the any-layout form) with every entry's e_t and
// x_t stored: the per-entry outputs of the kernel that AVer runs.
int launch_agg_aes_emit(bool fast, uint32_t grid, const void* args, uint32_t* partials, uint32_t* e_out,
                        uint32_t* x_out, hipStream_t s) {
    const BatchArgs& a = *static_cast<const BatchArgs*>(args);
    if (fast)
        hipLaunchKernelGGL((k_agg_ekeys_aes_perm<2, 1024, true, true, 8, true, 32>), dim3(grid), dim3(1024), 0, s,
                           a, partials, e_out, x_out);
    else
        hipLaunchKernelGGL((k_agg_ekeys_aes_perm<2, 1024, false, true, 8, true, 32>), dim3(grid), dim3(1024), 0, s,
                           a, partials, e_out, x_out);
    return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
}

}  // namespace poslo
