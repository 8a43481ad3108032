// Balanced radix-2^8 digits of 64-bit words and the digit-tile layout the int8 matrix-core
// kernels read (shared by the product kernels and the verification kernels that write
// tiles of their own).
#pragma once
#include "common.h"

namespace mpc3 {
namespace limb {

constexpr int KB = 32;                    // k-block depth of one v_mfma_i32_32x32x32_i8 step
constexpr int PLANE = 64 * KB;            // bytes of one digit plane of a 64 x 32 tile
constexpr int TILE_BYTES = 8 * PLANE;     // the eight digit planes of a 64 x 32 tile
constexpr u64 OFF = 0x8080808080808080ull;

// 4x4 byte transpose: out_j byte i = in_i byte j.
__device__ __forceinline__ void bt4(u32 a, u32 b, u32 c, u32 d, u32& o0, u32& o1, u32& o2, u32& o3) {
    const u32 ab_lo = (a & 0x00FF00FFu) | ((b & 0x00FF00FFu) << 8);     // a0 b0 a2 b2
    const u32 ab_hi = ((a >> 8) & 0x00FF00FFu) | (b & 0xFF00FF00u);     // a1 b1 a3 b3
    const u32 cd_lo = (c & 0x00FF00FFu) | ((d & 0x00FF00FFu) << 8);
    const u32 cd_hi = ((c >> 8) & 0x00FF00FFu) | (d & 0xFF00FF00u);
    o0 = (ab_lo & 0xFFFFu) | (cd_lo << 16);
    o2 = (ab_lo >> 16) | (cd_lo & 0xFFFF0000u);
    o1 = (ab_hi & 0xFFFFu) | (cd_hi << 16);
    o3 = (ab_hi >> 16) | (cd_hi & 0xFFFF0000u);
}

// Balanced digits of 8 words: q[d] byte i = digit d of word i.  The digits of a are the
// bytes of (a + 0x8080..80) xor 0x8080..80 read as int8.
__device__ __forceinline__ void to_digits(const u64 w[8], u64 q[8]) {
    u32 lo[8], hi[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const u64 v = (w[i] + OFF) ^ OFF;
        lo[i] = (u32)v;
        hi[i] = (u32)(v >> 32);
    }
    u32 t0[4], t1[4], t2[4], t3[4];
    bt4(lo[0], lo[1], lo[2], lo[3], t0[0], t0[1], t0[2], t0[3]);   // digits 0..3 of words 0..3
    bt4(lo[4], lo[5], lo[6], lo[7], t1[0], t1[1], t1[2], t1[3]);   // digits 0..3 of words 4..7
    bt4(hi[0], hi[1], hi[2], hi[3], t2[0], t2[1], t2[2], t2[3]);   // digits 4..7 of words 0..3
    bt4(hi[4], hi[5], hi[6], hi[7], t3[0], t3[1], t3[2], t3[3]);   // digits 4..7 of words 4..7
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        q[d] = (u64)t0[d] | ((u64)t1[d] << 32);
        q[4 + d] = (u64)t2[d] | ((u64)t3[d] << 32);
    }
}

// A digit tile is k-block kb (32 deep) of 64 consecutive B columns: 8 digit planes x 64 rows
// x 32 bytes, stored exactly as it sits in LDS.  Within a row the two 16-byte halves are
// swapped when swz(row) = 1, so the 16-byte fragment reads of 16 consecutive rows fall on
// distinct banks.
__device__ __forceinline__ int swz(int row) { return ((row >> 2) ^ (row >> 3)) & 1; }

// byte offset of digit plane d, tile row r, k-octet o (8 bytes) within a tile
__device__ __forceinline__ int toff(int d, int r, int o) {
    return d * PLANE + r * KB + (((o >> 1) ^ swz(r)) << 4) + ((o & 1) << 3);
}

}  // namespace limb
}  // namespace mpc3
