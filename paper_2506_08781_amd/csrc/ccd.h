// Cold cryptographic data (CCD) of a distilled batch, shared by the
// fine-grained (POSLO-F, entry-granular) and coarse-grained (POSLO-C,
// epoch-granular) Distill and SeBVer entry points.
#pragma once

#include <stdint.h>

#include <vector>

struct poslo_ccd {
    uint32_t inst = 0, log2_n1 = 0, log2_n2 = 0;
    uint32_t coarse = 0;                // 1: POSLO-C, invalid items are epochs
    uint64_t t0 = 0, n = 0;             // first entry and entry count of the batch
    uint64_t span = 0;                  // umbrella span: entries (POSLO-F) or epochs (POSLO-C)
    std::vector<uint8_t> ds;
    uint8_t valid_tag[64] = {};
    std::vector<uint8_t> umb_tags;      // 64 bytes per umbrella
    std::vector<uint64_t> invalid;      // sorted entry indices t, or epoch indices i when coarse
    std::vector<uint8_t> invalid_sigs;  // 80 bytes per invalid item: sigma_t, or
                                        // LE32B(s~_i) || enc(R~_i) || 16 zero bytes when coarse
};
