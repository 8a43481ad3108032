// Launch wrappers of the non-linear layers (Sec. 4.3): edaBits and daBits, bit extraction,
// B2A, Boolean Pi_Mult on bit-sliced words, and Pi_MultVerify over GF(2^64).
#pragma once
#include "kernels.h"

namespace mpc3 {

// Keystream purposes of the non-linear layers (beside the linear path's).
enum NlPurpose : u32 { P_EDA_BITS = 32, P_DA_BITS = 33, P_AND_RZ = 34, P_AND_GAMMA = 35, P_EDA_W_R = 36,
                       P_EDA_W_GAMMA = 37 };

// Three planes (m, [r]_1, [r]_2) of a share.
struct P3 {
    u64* p[3];
};
struct C3 {
    const u64* p[3];
};

// out[i] = (neg ? -1 : 1) * bit (i % per) of B[i / per]  (per = 64: the 64 bits of a word;
// per = 1: bit 0).
void launch_lift_bits(int64_t n, int per, const u64* B, int neg, u64* out, hipStream_t s);
// out = x + y - 2 z on three planes (n words each).
void launch_lin3(int64_t n, C3 x, C3 y, C3 z, P3 out, hipStream_t s);
// out = a + b (sign = 1) or a - b (sign = -1) on three planes.
void launch_addsub3(int64_t n, C3 a, C3 b, int sign, P3 out, hipStream_t s);
// edaBits rows: for row p (64 elements), x_j = 2^(j+1) mb_j on the m plane (written to Xm),
// the inner product w = Pi_Inner(x, rp) with fresh masks (op, P_EDA_W_R / P_EDA_W_GAMMA,
// injection on P1's message of row inj.index), and r = sum_j 2^j (mb_j + rp_j) - w.
void launch_eda_rows(int64_t n, const Keys& k, u32 op, const u64* Mb, C3 rp, Inj m1inj, u64* Xm, P3 w, P3 r,
                     hipStream_t s);
// Boolean Pi_Mult on n words: c = a AND b with fresh masks (op, P_AND_RZ / P_AND_GAMMA);
// injection XORs e into P0's [Gamma]_2 of word inj.index.
void launch_and_words(int64_t n, const Keys& k, u32 op, C3 a, C3 b, Inj g2inj, P3 c, hipStream_t s);
// Delta = (x - r) opened: m - r1 - r2 of the difference.
void launch_open_diff(int64_t n, C3 x, C3 r, u64* delta, hipStream_t s);
// Prefix adder set-up: P0 = R XOR Delta (m plane), G = R AND Delta (every plane); P = P0.
void launch_a2b_init(int64_t n, C3 R, const u64* delta, P3 P0, P3 G, P3 P, hipStream_t s);
// Operands of one prefix level at distance k: A = [P, P], B = [G << k, P << k] (2n words per
// plane), or A = P, B = G << k when last.
void launch_ks_prep(int64_t n, int k, bool last, C3 P, C3 G, P3 A, P3 B, hipStream_t s);
// After the level's AND: G ^= C[0..n), and P = C[n..2n) unless last.
void launch_ks_update(int64_t n, bool last, C3 C, P3 G, P3 P, hipStream_t s);
// Top bit of the sum: (P0 XOR (G << 1)) >> 63 per plane, XOR 1 into m when flip.
void launch_msb_final(int64_t n, C3 P0, C3 G, bool flip, P3 out, hipStream_t s);
// B2A: e = (d XOR sb) bit 0 opened, dl = e + (1 - 2e) s.
void launch_b2a(int64_t n, C3 d, C3 sb, C3 sa, P3 dl, hipStream_t s);
// 2x2 window corners of an NHWC tensor: p = [top-left, bottom-left], q = [top-right,
// bottom-right] (2 * B * H/2 * W/2 * C words per plane).
void launch_pool_gather(int B, int H, int W, int C, C3 x, P3 p, P3 q, hipStream_t s);

// Gate-scaled lift for a Pi_BIVerify of row gates: out[c][e, k] = a_c[e] * P[e / per, k]
// (P: one 64-word power per gate; null planes give 0), output planes ps words apart.
void launch_scale_gates(int64_t n, int per, C3 a, const u64* P, u64* out, int64_t ps, hipStream_t s);

// --- Pi_MultVerify over GF(2^64) ------------------------------------------
// A random <.>^1 element of GF(2^64): one word from each pairwise PRG under (op, purpose,
// comp, sub); share3 = (m, r1, r2), value (nullable) = m ^ r1 ^ r2, log (nullable) = value.
void launch_gf_random(const Keys& k, u32 op, u32 purpose, u32 sub, u64* share3, u64* value, u64* log,
                      hipStream_t s);
// Power tables of the revealed r: T0[b] = r^b (b < 64), T1[w] = r^(64 w) (w < W).
void launch_gf_pow_tables(const u64* r, int64_t W, u64* T0, u64* T1, hipStream_t s);
// Pi_Tran of W words of Boolean triples: gate g = 64 w + b; x planes r^g (bit of A), y planes
// the bits of B, as six planes of npad words (plane c at XY + c * npad; words G .. npad-1 are
// written 0); z = XOR of r^g over the set bits of C, per plane (zout: 3 words).
void launch_gf_tran(int64_t W, const u64* T0, const u64* T1, C3 A, C3 B, C3 C, u64* XY, int64_t npad, u64* zout,
                    void* (*ws)(void*, size_t), void* wss, hipStream_t s);
struct GfRoundArgs {
    Keys k;
    u32 op, sub;
    u64 inv[3];            // 1/x, 1/(1+x), 1/(x(1+x))
    u64* z;                // claimed share (3 words), updated
    u64* zeta;             // revealed point (1 word)
    u64* log_zeta; u64* log_h0; u64* log_h2;    // nullable; h logs: m1, m2, g2 at word 0 of three slots 64 apart
};
// One Pi_Reduce round over GF(2^64) of n pairs (2n rows per plane, planes ps apart): h(0) and
// h(x) as two Pi_PolyEvl, zeta revealed, z updated; then the fold into XYn (planes psn apart).
void launch_gf_round(int64_t n, const u64* XY, int64_t ps, u64* XYn, int64_t psn, const GfRoundArgs& a,
                     void* (*ws)(void*, size_t), void* wss, hipStream_t s);
struct GfDeltaArgs {
    Keys k;
    u32 op, sub;
    const u64* z;          // claimed share (3 words)
    u64* log_delta; u64* log_tr;   // nullable; tr: m1, m2, g2 at word 0 of three slots 64 apart
    int* flag;             // set when Delta != 0
};
// Pi_InnerVerify over GF(2^64) of n pairs (planes ps apart).
void launch_gf_inner_verify(int64_t n, const u64* XY, int64_t ps, const GfDeltaArgs& a, void* (*ws)(void*, size_t),
                            void* wss, hipStream_t s);

// Host GF(2^64) arithmetic (constants of the Lagrange step).
u64 gf_mul_host(u64 a, u64 b);
u64 gf_inv_host(u64 a);

}  // namespace mpc3
