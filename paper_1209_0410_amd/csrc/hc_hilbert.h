// Extended keys of a 16-dim point with 8-bit coordinates: the Hilbert key of
// the method and, for comparison, the Z-order key.  Compiled for gfx950 and
// for the host search of the cooperative path.
//
// The curve is the Butz-type Hilbert curve the paper uses (Sec. 2.2.1), in the
// transposed form of J. Skilling ("Programming the Hilbert curve", AIP Conf.
// Proc. 707, 2004).  The order is 8 because the coordinates have 8 bits, so a
// key has 16 * 8 = 128 bits.  Written branch-free for wavefront execution:
// every lane runs the same instruction stream whatever its coordinates.
#pragma once

#include "hc_internal.h"

namespace hc {

// 8x8 bit-matrix transpose of a 64-bit word whose byte r (r = 0 is the most
// significant) is row r and whose bit 7-c is column c (Hacker's Delight 7-3).
__host__ __device__ inline uint64_t transpose8x8(uint64_t x)
{
    uint64_t t;
    t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x ^= t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x ^= t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    x ^= t ^ (t << 28);
    return x;
}

// Moves the four bytes of a 32-bit word to the odd byte positions (counted
// from the most significant byte) of a 64-bit word: b0 b1 b2 b3 ->
// 0 b0 0 b1 0 b2 0 b3.
__host__ __device__ inline uint64_t spread_bytes(uint32_t v)
{
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    return x;
}

// Bit-plane transpose of 16 8-bit values into a key: level 7 of dims 0..15,
// then level 6, and so on.  Dims 0..7 and 8..15 are transposed as two 8x8 bit
// matrices whose rows are interleaved byte by byte.
__host__ __device__ inline Key interleave_key16(const uint32_t (&x)[kDpc])
{
    uint64_t a = 0, b = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        a |= (uint64_t)(x[i] & 0xFFu) << (56 - 8 * i);
        b |= (uint64_t)(x[i + 8] & 0xFFu) << (56 - 8 * i);
    }
    a = transpose8x8(a);   // byte r: level 7-r of dims 0..7
    b = transpose8x8(b);   // byte r: level 7-r of dims 8..15
    Key k;
    k.hi = (spread_bytes((uint32_t)(a >> 32)) << 8) | spread_bytes((uint32_t)(b >> 32));
    k.lo = (spread_bytes((uint32_t)a) << 8) | spread_bytes((uint32_t)b);
    return k;
}

__host__ __device__ inline Key hilbert_key16(const uint32_t (&coord)[kDpc])
{
    uint32_t x[kDpc];
#pragma unroll
    for (int i = 0; i < kDpc; i++) x[i] = coord[i];

    // Walk the levels from the top: where coordinate i has its level bit set,
    // the lower bits of x[0] are inverted; otherwise the lower bits of x[0]
    // and x[i] are exchanged.
#pragma unroll
    for (int lvl = 7; lvl >= 1; lvl--) {
        const uint32_t low = (1u << lvl) - 1u;
#pragma unroll
        for (int i = 0; i < kDpc; i++) {
            const uint32_t set = 0u - ((x[i] >> lvl) & 1u);   // all ones if set
            const uint32_t swap = (x[0] ^ x[i]) & low & ~set;
            x[0] ^= swap ^ (low & set);
            if (i != 0) x[i] ^= swap;
        }
    }
    // Gray code along the dims.
#pragma unroll
    for (int i = 1; i < kDpc; i++) x[i] ^= x[i - 1];
    // Final correction: bit b is flipped in every coordinate when the number
    // of set bits of x[15] above level b (levels b+1..7, level 0 excluded)
    // is odd -- a suffix parity, computed by a shift-xor scan.
    uint32_t par = (x[kDpc - 1] & 0xFEu) >> 1;
    par ^= par >> 1;
    par ^= par >> 2;
    par ^= par >> 4;
#pragma unroll
    for (int i = 0; i < kDpc; i++) x[i] ^= par;

    return interleave_key16(x);
}

// Z-order (Morton) key: the coordinates' bits interleaved as they are, with
// no Hilbert rotation.
__host__ __device__ inline Key zorder_key16(const uint32_t (&coord)[kDpc])
{
    return interleave_key16(coord);
}

__host__ __device__ inline Key curve_key16(const uint32_t (&coord)[kDpc], uint32_t curve)
{
    return curve == HC_CURVE_ZORDER ? zorder_key16(coord) : hilbert_key16(coord);
}

// Loads the 16 coordinates of curve c of a 128-byte row.
__host__ __device__ inline void project16(const uint8_t *row, const IndexView &v, uint32_t c,
                                 uint32_t (&coord)[kDpc])
{
    if (v.identity) {
        const uint4 w = *reinterpret_cast<const uint4 *>(row + kDpc * c);
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int i = 0; i < kDpc; i++) coord[i] = (words[i >> 2] >> (8 * (i & 3))) & 0xFFu;
    } else {
#pragma unroll
        for (int i = 0; i < kDpc; i++) coord[i] = row[v.perm[kDpc * c + i]];
    }
}

}  // namespace hc
