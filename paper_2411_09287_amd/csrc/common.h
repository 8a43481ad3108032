// Shared device/host definitions for the mpc3 library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint64_t u64;
typedef uint32_t u32;

namespace mpc3 {

constexpr int D = 64;            // degree of the Galois-ring extension (the paper's d = 64)
// x^64 = -(x^4 + x^3 + x + 1): the low-order terms of the monic modulus.
constexpr int NTAPS = 4;
__host__ __device__ constexpr int tap(int i) { return i == 0 ? 0 : i == 1 ? 1 : i == 2 ? 3 : 4; }

// PRG key and 96-bit nonce (ChaCha20, RFC 8439).
struct Key { u32 w[8]; };
struct Tag { u32 n0, n1, n2; };

__host__ __device__ inline Tag make_tag(u32 op, u32 purpose, u32 comp, u32 sub) {
    Tag t; t.n0 = op; t.n1 = (purpose & 0xFFFFu) | (comp << 16); t.n2 = sub; return t;
}

// Purposes of keystream draws (the component lives in the nonce's upper half-word):
// component 0 = an m word (eta_12), 1 = a [.]_1 word (eta_01), 2 = a [.]_2 word (eta_02).
enum Purpose : u32 {
    P_SHARE_R = 1, P_INNER_RZ = 2, P_INNER_GAMMA = 3, P_TRUNC_B = 4, P_TRUNC_WX_R = 5,
    P_TRUNC_WX_GAMMA = 6, P_TRUNC_WZ_R = 7, P_TRUNC_WZ_GAMMA = 8, P_MULT_RZ = 9, P_MULT_GAMMA = 10,
    P_VER_R = 16, P_VER_H0_R = 17, P_VER_H0_GAMMA = 18, P_VER_H2_R = 19, P_VER_H2_GAMMA = 20,
    P_VER_ZETA = 21, P_VER_ALPHA = 22, P_VER_XP_R = 23, P_VER_XP_GAMMA = 24, P_VER_DELTA_R = 25,
    P_VER_DELTA_GAMMA = 26
};

__device__ __forceinline__ u32 rotl32(u32 v, int c) { return (v << c) | (v >> (32 - c)); }

#define MPC3_QR(a, b, c, d)                 \
    a += b; d ^= a; d = rotl32(d, 16);      \
    c += d; b ^= c; b = rotl32(b, 12);      \
    a += b; d ^= a; d = rotl32(d, 8);       \
    c += d; b ^= c; b = rotl32(b, 7);

// RFC 8439 Sec. 2.3 block function: 16 keystream words for one block counter.
__device__ __forceinline__ void chacha_block(const Key& k, u32 ctr, const Tag& t, u32 o[16]) {
    u32 x0 = 0x61707865u, x1 = 0x3320646eu, x2 = 0x79622d32u, x3 = 0x6b206574u;
    u32 x4 = k.w[0], x5 = k.w[1], x6 = k.w[2], x7 = k.w[3];
    u32 x8 = k.w[4], x9 = k.w[5], x10 = k.w[6], x11 = k.w[7];
    u32 x12 = ctr, x13 = t.n0, x14 = t.n1, x15 = t.n2;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        MPC3_QR(x0, x4, x8, x12) MPC3_QR(x1, x5, x9, x13) MPC3_QR(x2, x6, x10, x14) MPC3_QR(x3, x7, x11, x15)
        MPC3_QR(x0, x5, x10, x15) MPC3_QR(x1, x6, x11, x12) MPC3_QR(x2, x7, x8, x13) MPC3_QR(x3, x4, x9, x14)
    }
    o[0] = x0 + 0x61707865u; o[1] = x1 + 0x3320646eu; o[2] = x2 + 0x79622d32u; o[3] = x3 + 0x6b206574u;
    o[4] = x4 + k.w[0]; o[5] = x5 + k.w[1]; o[6] = x6 + k.w[2]; o[7] = x7 + k.w[3];
    o[8] = x8 + k.w[4]; o[9] = x9 + k.w[5]; o[10] = x10 + k.w[6]; o[11] = x11 + k.w[7];
    o[12] = x12 + ctr; o[13] = x13 + t.n0; o[14] = x14 + t.n1; o[15] = x15 + t.n2;
}

// Eight consecutive 64-bit words 8*blk .. 8*blk+7 of G(key, tag, .).
__device__ __forceinline__ void prg_block8(const Key& k, const Tag& t, u64 blk, u64 w[8]) {
    u32 o[16];
    chacha_block(k, (u32)blk, t, o);
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = (u64)o[2 * i] | ((u64)o[2 * i + 1] << 32);
}

// One word G(key, tag, i) (computes the whole block; for scattered accesses).
__device__ __forceinline__ u64 prg_word(const Key& k, const Tag& t, u64 i) {
    u32 o[16];
    chacha_block(k, (u32)(i >> 3), t, o);
    int j = (int)(i & 7);
    u32 lo = o[0], hi = o[1];
#pragma unroll
    for (int q = 1; q < 8; ++q)
        if (q == j) { lo = o[2 * q]; hi = o[2 * q + 1]; }
    return (u64)lo | ((u64)hi << 32);
}

// Arithmetic right shift of a two's-complement word.
__host__ __device__ __forceinline__ u64 ash(u64 v, int t) { return (u64)((int64_t)v >> t); }

}  // namespace mpc3
