/*
 * POSLO oracle: byte-level primitives.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or generator with the GPU library under
 * paper_2506_08781_amd/, and that library never calls it.
 *
 * Plain, single-threaded, byte-oriented C with no intrinsics.  Each function
 * follows a published definition and says which:
 *   - AES-128 ................ FIPS-197 (sections 5.1 and 5.2); the S-box is
 *                              computed from its definition (multiplicative
 *                              inverse in GF(2^8) followed by the affine map)
 *   - SHA-256 ................ FIPS 180-4 (sections 4.1.2, 5.1.1, 6.2); the
 *                              constants are computed from their definition
 *                              (fractional parts of square and cube roots of
 *                              the first primes)
 *   - MMO .................... paper, Preliminaries, Definition "MMO"
 *   - MDC-2 .................. paper, Preliminaries, Definition "MDC-2"
 *   - PRF_b, F ............... paper, Instantiations, "Instantiations of PRF"
 *   - H ...................... paper, Instantiations, "Instantiations of H"
 *
 * Readings of the paper taken here (the paper is silent or garbled):
 *   - MMO/MDC-2 split a k-byte input into max(1, ceil(k/16)) blocks and pad
 *     the last block with zero bytes; no length block is appended.  This
 *     makes a 16-byte input cost exactly one block cipher call per lane, as
 *     the paper requires for the 128-bit MDC-2 case.
 *   - the chaining value is the AES key and the message block the plaintext.
 *   - initial values: MMO and the first MDC-2 lane use 0x52 repeated 16
 *     times, the second MDC-2 lane uses 0x25 repeated 16 times.
 *   - the MDC-2 definition's "xor x_i" is read as "xor m_i".
 *   - F for the SHA-256 instantiation is SHA-256 truncated to its first 16
 *     bytes, so that PRF outputs are kappa = 128 bits in both instantiations.
 *   - PRF_b(z) = F(z || b) appends b as one whole byte (0x00 or 0x01).
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------------ */
/* GF(2^8) with the AES polynomial x^8 + x^4 + x^3 + x + 1 (FIPS-197 4.2)   */
/* ------------------------------------------------------------------------ */

static uint8_t gf_mul(uint8_t a, uint8_t b)
{
    uint8_t r = 0;
    for (int i = 0; i < 8; i++) {
        if (b & 1)
            r ^= a;
        uint8_t hi = a & 0x80;
        a = (uint8_t)(a << 1);
        if (hi)
            a ^= 0x1b;
        b >>= 1;
    }
    return r;
}

static uint8_t gf_inv(uint8_t a)
{
    /* the multiplicative inverse, found by search; 0 maps to 0 (FIPS-197 5.1.1) */
    if (a == 0)
        return 0;
    for (int b = 1; b < 256; b++)
        if (gf_mul(a, (uint8_t)b) == 1)
            return (uint8_t)b;
    return 0;
}

static uint8_t SBOX[256];
static int sbox_ready = 0;

static void sbox_init(void)
{
    if (sbox_ready)
        return;
    for (int x = 0; x < 256; x++) {
        uint8_t b = gf_inv((uint8_t)x);
        uint8_t s = 0;
        /* affine map: b'_i = b_i ^ b_{i+4} ^ b_{i+5} ^ b_{i+6} ^ b_{i+7} ^ c_i, c = 0x63 */
        for (int i = 0; i < 8; i++) {
            int bit = ((b >> i) ^ (b >> ((i + 4) % 8)) ^ (b >> ((i + 5) % 8)) ^
                       (b >> ((i + 6) % 8)) ^ (b >> ((i + 7) % 8)) ^ (0x63 >> i)) & 1;
            s |= (uint8_t)(bit << i);
        }
        SBOX[x] = s;
    }
    sbox_ready = 1;
}

/* ------------------------------------------------------------------------ */
/* AES-128 (FIPS-197)                                                       */
/* ------------------------------------------------------------------------ */

/* Key expansion (FIPS-197 5.2): 44 four-byte words w[0..43]. */
static void aes128_key_expansion(const uint8_t key[16], uint8_t w[44][4])
{
    uint8_t rcon = 0x01;
    for (int i = 0; i < 4; i++)
        for (int b = 0; b < 4; b++)
            w[i][b] = key[4 * i + b];
    for (int i = 4; i < 44; i++) {
        uint8_t temp[4];
        memcpy(temp, w[i - 1], 4);
        if (i % 4 == 0) {
            /* RotWord, then SubWord, then xor Rcon[i/4] */
            uint8_t t0 = temp[0];
            temp[0] = temp[1];
            temp[1] = temp[2];
            temp[2] = temp[3];
            temp[3] = t0;
            for (int b = 0; b < 4; b++)
                temp[b] = SBOX[temp[b]];
            temp[0] ^= rcon;
            rcon = gf_mul(rcon, 0x02);
        }
        for (int b = 0; b < 4; b++)
            w[i][b] = w[i - 4][b] ^ temp[b];
    }
}

/* The cipher (FIPS-197 5.1): state[r][c] = in[r + 4c]. */
void oracle_aes128_encrypt(const uint8_t key[16], const uint8_t in[16], uint8_t out[16])
{
    sbox_init();
    uint8_t w[44][4];
    aes128_key_expansion(key, w);
    uint8_t s[4][4];
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            s[r][c] = in[r + 4 * c];

    for (int round = 0; round <= 10; round++) {
        if (round > 0) {
            /* SubBytes */
            for (int r = 0; r < 4; r++)
                for (int c = 0; c < 4; c++)
                    s[r][c] = SBOX[s[r][c]];
            /* ShiftRows: row r rotates left by r */
            for (int r = 1; r < 4; r++) {
                uint8_t tmp[4];
                for (int c = 0; c < 4; c++)
                    tmp[c] = s[r][(c + r) % 4];
                for (int c = 0; c < 4; c++)
                    s[r][c] = tmp[c];
            }
            /* MixColumns, not in the final round */
            if (round < 10) {
                for (int c = 0; c < 4; c++) {
                    uint8_t a0 = s[0][c], a1 = s[1][c], a2 = s[2][c], a3 = s[3][c];
                    s[0][c] = gf_mul(a0, 2) ^ gf_mul(a1, 3) ^ a2 ^ a3;
                    s[1][c] = a0 ^ gf_mul(a1, 2) ^ gf_mul(a2, 3) ^ a3;
                    s[2][c] = a0 ^ a1 ^ gf_mul(a2, 2) ^ gf_mul(a3, 3);
                    s[3][c] = gf_mul(a0, 3) ^ a1 ^ a2 ^ gf_mul(a3, 2);
                }
            }
        }
        /* AddRoundKey with words w[4*round .. 4*round+3] */
        for (int c = 0; c < 4; c++)
            for (int r = 0; r < 4; r++)
                s[r][c] ^= w[4 * round + c][r];
    }
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            out[r + 4 * c] = s[r][c];
}

/* ------------------------------------------------------------------------ */
/* SHA-256 (FIPS 180-4)                                                     */
/* ------------------------------------------------------------------------ */

static uint32_t SHA_K[64];
static uint32_t SHA_H0[8];
static int sha_ready = 0;

static void sha_init(void)
{
    if (sha_ready)
        return;
    /* first 64 primes */
    int primes[64];
    int n = 0;
    for (int c = 2; n < 64; c++) {
        int is_p = 1;
        for (int d = 2; d * d <= c; d++)
            if (c % d == 0) {
                is_p = 0;
                break;
            }
        if (is_p)
            primes[n++] = c;
    }
    /* 4.2.2: first 32 bits of the fractional parts of the cube roots;
       5.3.3: first 32 bits of the fractional parts of the square roots */
    for (int i = 0; i < 64; i++) {
        long double r = cbrtl((long double)primes[i]);
        long double f = r - floorl(r);
        SHA_K[i] = (uint32_t)floorl(f * 4294967296.0L);
    }
    for (int i = 0; i < 8; i++) {
        long double r = sqrtl((long double)primes[i]);
        long double f = r - floorl(r);
        SHA_H0[i] = (uint32_t)floorl(f * 4294967296.0L);
    }
    sha_ready = 1;
}

static uint32_t rotr32(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

static void sha256_compress(uint32_t H[8], const uint8_t block[64])
{
    uint32_t W[64];
    for (int t = 0; t < 16; t++)
        W[t] = ((uint32_t)block[4 * t] << 24) | ((uint32_t)block[4 * t + 1] << 16) |
               ((uint32_t)block[4 * t + 2] << 8) | (uint32_t)block[4 * t + 3];
    for (int t = 16; t < 64; t++) {
        uint32_t s0 = rotr32(W[t - 15], 7) ^ rotr32(W[t - 15], 18) ^ (W[t - 15] >> 3);
        uint32_t s1 = rotr32(W[t - 2], 17) ^ rotr32(W[t - 2], 19) ^ (W[t - 2] >> 10);
        W[t] = s1 + W[t - 7] + s0 + W[t - 16];
    }
    uint32_t a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7];
    for (int t = 0; t < 64; t++) {
        uint32_t S1 = rotr32(e, 6) ^ rotr32(e, 11) ^ rotr32(e, 25);
        uint32_t ch = (e & f) ^ (~e & g);
        uint32_t T1 = h + S1 + ch + SHA_K[t] + W[t];
        uint32_t S0 = rotr32(a, 2) ^ rotr32(a, 13) ^ rotr32(a, 22);
        uint32_t maj = (a & b) ^ (a & c) ^ (b & c);
        uint32_t T2 = S0 + maj;
        h = g;
        g = f;
        f = e;
        e = d + T1;
        d = c;
        c = b;
        b = a;
        a = T1 + T2;
    }
    H[0] += a;
    H[1] += b;
    H[2] += c;
    H[3] += d;
    H[4] += e;
    H[5] += f;
    H[6] += g;
    H[7] += h;
}

void oracle_sha256(const uint8_t *in, size_t len, uint8_t out[32])
{
    sha_init();
    uint32_t H[8];
    memcpy(H, SHA_H0, sizeof H);
    /* 5.1.1 padding: append 0x80, zeros, then the 64-bit big-endian bit length */
    size_t total = ((len + 9 + 63) / 64) * 64;
    uint8_t block[64];
    for (size_t off = 0; off < total; off += 64) {
        for (size_t k = 0; k < 64; k++) {
            size_t pos = off + k;
            uint8_t v;
            if (pos < len)
                v = in[pos];
            else if (pos == len)
                v = 0x80;
            else if (pos >= total - 8) {
                uint64_t bits = (uint64_t)len * 8u;
                int shift = (int)(8 * (total - 1 - pos));
                v = (uint8_t)(bits >> shift);
            } else
                v = 0;
            block[k] = v;
        }
        sha256_compress(H, block);
    }
    for (int i = 0; i < 8; i++) {
        out[4 * i] = (uint8_t)(H[i] >> 24);
        out[4 * i + 1] = (uint8_t)(H[i] >> 16);
        out[4 * i + 2] = (uint8_t)(H[i] >> 8);
        out[4 * i + 3] = (uint8_t)H[i];
    }
}

/* ------------------------------------------------------------------------ */
/* MMO and MDC-2 over AES-128 (paper, Definitions "MMO" and "MDC-2")        */
/* ------------------------------------------------------------------------ */

static size_t block_count(size_t len) { return len == 0 ? 1 : (len + 15) / 16; }

static void get_block(const uint8_t *in, size_t len, size_t i, uint8_t m[16])
{
    for (size_t k = 0; k < 16; k++) {
        size_t pos = 16 * i + k;
        m[k] = pos < len ? in[pos] : 0; /* zero padding of the last block */
    }
}

/* h_0 = IV; h_i = E_{h_{i-1}}(m_i) xor m_i; output h_t */
void oracle_mmo(const uint8_t *in, size_t len, uint8_t out[16])
{
    uint8_t h[16], m[16], c[16];
    memset(h, 0x52, 16);
    size_t t = block_count(len);
    for (size_t i = 0; i < t; i++) {
        get_block(in, len, i, m);
        oracle_aes128_encrypt(h, m, c);
        for (int k = 0; k < 16; k++)
            h[k] = c[k] ^ m[k];
    }
    memcpy(out, h, 16);
}

/* two MMO lanes whose right halves are swapped after every block; output h_t || h'_t */
void oracle_mdc2(const uint8_t *in, size_t len, uint8_t out[32])
{
    uint8_t h[16], hp[16], m[16], a[16], b[16];
    memset(h, 0x52, 16);
    memset(hp, 0x25, 16);
    size_t t = block_count(len);
    for (size_t i = 0; i < t; i++) {
        get_block(in, len, i, m);
        oracle_aes128_encrypt(h, m, a);
        oracle_aes128_encrypt(hp, m, b);
        for (int k = 0; k < 16; k++) {
            a[k] ^= m[k];
            b[k] ^= m[k];
        }
        /* h = a^1 || b^2, h' = b^1 || a^2 (halves of 8 bytes) */
        memcpy(h, a, 8);
        memcpy(h + 8, b + 8, 8);
        memcpy(hp, b, 8);
        memcpy(hp + 8, a + 8, 8);
    }
    memcpy(out, h, 16);
    memcpy(out + 16, hp, 16);
}

/* ------------------------------------------------------------------------ */
/* Instantiations (paper, table "Instantiations of POSLO schemes")          */
/*   inst 0 = POSLO  (PRF and H from SHA-256)                               */
/*   inst 1 = POSLO+ (PRF from MMO-AES-128, H = MDC-2-AES-128)              */
/* ------------------------------------------------------------------------ */

int oracle_F(int inst, const uint8_t *in, size_t len, uint8_t out[16])
{
    if (inst == 1) {
        oracle_mmo(in, len, out);
        return 0;
    }
    if (inst == 0) {
        uint8_t d[32];
        oracle_sha256(in, len, d);
        memcpy(out, d, 16);
        return 0;
    }
    return -1;
}

int oracle_H(int inst, const uint8_t *in, size_t len, uint8_t out[32])
{
    if (inst == 1) {
        oracle_mdc2(in, len, out);
        return 0;
    }
    if (inst == 0) {
        oracle_sha256(in, len, out);
        return 0;
    }
    return -1;
}
