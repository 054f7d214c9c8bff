// Layout of the fixed-base comb tables read by device_ec.h: 32 windows of
// 128 affine points, t[w][i] = (i + 1) * 256^w * P stored as the canonical
// (y + x, y - x, 2d*x*y), 24 words; 393,216 bytes per point P.  The
// generator also has a wide table for the per-entry checks: 16 windows of
// 32,768 points (i + 1) * 65536^w * G, 50,331,648 bytes.
#pragma once

#include "ge25519.h"

namespace poslo {

constexpr int kCombWindows = 32;     // signed 8-bit digits of a scalar below 2^253
constexpr int kCombPerWindow = 128;  // digit magnitudes 1..128
constexpr int kCombEntryWords = 24;
constexpr int kCombWords = kCombWindows * kCombPerWindow * kCombEntryWords;
constexpr int kWideWindows = 16;        // signed 16-bit digits of a scalar below 2^253
constexpr int kWidePerWindow = 32768;  // digit magnitudes 1..32768
constexpr uint64_t kWideWords = (uint64_t)kWideWindows * kWidePerWindow * kCombEntryWords;

// table entry of the point (X : Y : Z) given zi = 1 / Z
PD void comb_entry_zinv(uint32_t o[kCombEntryWords], const fe& X, const fe& Y, const fe& zi) {
    const fe d2 = POSLO_FE_D2;
    fe x, y, a, b, t;
    fe_mul(x, X, zi);
    fe_mul(y, Y, zi);
    fe_add(a, y, x);
    fe_sub(b, y, x);
    fe_mul(t, x, y);
    fe_mul(t, t, d2);
    fe_freeze(a, a);
    fe_freeze(b, b);
    fe_freeze(t, t);
    for (int k = 0; k < 8; k++) {
        o[k] = a.v[k];
        o[8 + k] = b.v[k];
        o[16 + k] = t.v[k];
    }
}

// table entry of P
PD void comb_entry_of(uint32_t o[kCombEntryWords], const ge& P) {
    fe zi;
    fe_inv(zi, P.Z);
    comb_entry_zinv(o, P.X, P.Y, zi);
}

}  // namespace poslo
