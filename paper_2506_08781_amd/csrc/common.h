// Shared definitions for the POSLO-F verifier library (host and gfx950 device).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

// Inline on both sides: the same arithmetic serves the host signer and the
// device kernels.
#define PD __host__ __device__ __forceinline__
#define PDC __host__ __device__ constexpr

namespace poslo {

// instantiations (paper, table "Instantiations of POSLO schemes")
enum Inst : uint32_t {
    INST_SHA256 = 0,    // POSLO: PRF and H from SHA-256
    INST_AES = 1,       // POSLO+: PRF from MMO-AES-128, H = MDC-2-AES-128
    INST_AES_ADDQ = 2,  // POSLO++: PRF from MMO-AES-128, H = Add_q (messages of at most 31 bytes)
};
// The host-side instantiation word: the instantiation, plus INST_K127 when
// kappa = 127 (an AES-based PRF whose tree PRF is one AES block)
constexpr uint32_t INST_K127 = 4;
PD uint32_t inst_base(uint32_t spec) { return spec & 3u; }
PD bool prf_is_aes(uint32_t spec) { return (spec & 3u) != INST_SHA256; }
PD bool kappa127(uint32_t spec) { return (spec & INST_K127) != 0; }
// messages that Add_q can take: below 2^248 < q
constexpr uint64_t kAddqMaxLen = 31;

PD uint32_t rotl32(uint32_t x, int n) { return (x << n) | (x >> ((32 - n) & 31)); }
PD uint32_t rotr32(uint32_t x, int n) { return (x >> n) | (x << ((32 - n) & 31)); }
PD uint32_t bswap32(uint32_t x) {
    return (x >> 24) | ((x >> 8) & 0xff00u) | ((x << 8) & 0xff0000u) | (x << 24);
}

PD uint32_t load_le32(const uint8_t* p) {
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
PD void store_le32(uint8_t* p, uint32_t v) {
    p[0] = (uint8_t)v;
    p[1] = (uint8_t)(v >> 8);
    p[2] = (uint8_t)(v >> 16);
    p[3] = (uint8_t)(v >> 24);
}

}  // namespace poslo
