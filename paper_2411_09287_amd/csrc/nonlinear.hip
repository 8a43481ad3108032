// Non-linear layers (Sec. 4.3, Fig. "The maliciously edaBits generation") on gfx950:
// edaBits / daBits preprocessing, bit extraction by a parallel-prefix carry on bit-sliced
// Boolean shares, B2A, and Pi_MultVerify of the Boolean triples over GF(2^64).
//
// Boolean shares <v>^1 = (m, r1, r2), m = v ^ r1 ^ r2, one uint64 word per plane holds 64
// Boolean values (for a 64-bit ring value: its bit i in bit i).  GF(2^64) elements are one
// word each, bit k the coefficient of x^k, modulo x^64 + x^4 + x^3 + x + 1.
#include "nonlinear.h"

namespace mpc3 {

namespace {

constexpr int TPB = 256;

__host__ inline unsigned nblk(int64_t work, int per_block) { return (unsigned)((work + per_block - 1) / per_block); }

// ---------------------------------------------------------------------------
// GF(2^64) arithmetic
// ---------------------------------------------------------------------------

// x^64 = x^4 + x^3 + x + 1: hi x^64 = hi ^ hi<<1 ^ hi<<3 ^ hi<<4, whose bits past x^63
// (hi>>63, hi>>61, hi>>60: at most four) are folded the same way once more.
__host__ __device__ __forceinline__ u64 gf_reduce(u64 lo, u64 hi) {
    const u64 over = (hi >> 60) ^ (hi >> 61) ^ (hi >> 63);
    const u64 r = lo ^ hi ^ (hi << 1) ^ (hi << 3) ^ (hi << 4);
    return r ^ over ^ (over << 1) ^ (over << 3) ^ (over << 4);
}

// Carry-less 32 x 32 -> 64 product by integer multiplies with spaced bits: each factor is
// split into four masks of every fourth bit, so the 16 integer products of the pieces
// cannot carry into a neighbouring bit of the same residue class (at most 8 terms per
// column of a 4-spaced product, < 16), and the wanted residue classes are masked out.
__device__ __forceinline__ u64 clmul32(u32 x, u32 y) {
    const u64 m0 = 0x1111111111111111ull, m1 = 0x2222222222222222ull, m2 = 0x4444444444444444ull,
              m3 = 0x8888888888888888ull;
    const u64 x0 = x & 0x11111111u, x1 = x & 0x22222222u, x2 = x & 0x44444444u, x3 = x & 0x88888888u;
    const u64 y0 = y & 0x11111111u, y1 = y & 0x22222222u, y2 = y & 0x44444444u, y3 = y & 0x88888888u;
    u64 z0 = (x0 * y0) ^ (x1 * y3) ^ (x2 * y2) ^ (x3 * y1);
    u64 z1 = (x0 * y1) ^ (x1 * y0) ^ (x2 * y3) ^ (x3 * y2);
    u64 z2 = (x0 * y2) ^ (x1 * y1) ^ (x2 * y0) ^ (x3 * y3);
    u64 z3 = (x0 * y3) ^ (x1 * y2) ^ (x2 * y1) ^ (x3 * y0);
    return (z0 & m0) | (z1 & m1) | (z2 & m2) | (z3 & m3);
}

// Carry-less 64 x 64 -> 128 product, Karatsuba over 32-bit halves.
__device__ __forceinline__ void clmul64(u64 a, u64 b, u64& lo, u64& hi) {
    const u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
    const u64 p0 = clmul32(a0, b0), p2 = clmul32(a1, b1);
    const u64 p1 = clmul32(a0 ^ a1, b0 ^ b1) ^ p0 ^ p2;
    lo = p0 ^ (p1 << 32);
    hi = p2 ^ (p1 >> 32);
}

__device__ __forceinline__ u64 gf_mul(u64 a, u64 b) {
    u64 lo, hi;
    clmul64(a, b, lo, hi);
    return gf_reduce(lo, hi);
}

// x * v
__device__ __forceinline__ u64 gf_xtime(u64 v) { return (v << 1) ^ ((v >> 63) ? 0x1Bull : 0ull); }

__device__ __forceinline__ u64 gf_pow(u64 a, u64 e) {
    u64 out = 1;
    while (e) {
        if (e & 1) out = gf_mul(out, a);
        a = gf_mul(a, a);
        e >>= 1;
    }
    return out;
}

__device__ __forceinline__ u64 wave_xor(u64 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v ^= __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ u64 wave_sum(u64 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Preprocessing and conversions
// ---------------------------------------------------------------------------

__global__ void k_lift_bits(int64_t n, int per, const u64* B, int neg, u64* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j = per == 64 ? (int)(i & 63) : 0;
    const u64 bit = (B[per == 64 ? (i >> 6) : i] >> j) & 1ull;
    out[i] = neg ? 0 - bit : bit;
}

__global__ void k_lin3(int64_t n, C3 x, C3 y, C3 z, P3 out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) out.p[c][i] = x.p[c][i] + y.p[c][i] - 2 * z.p[c][i];
}

__global__ void k_addsub3(int64_t n, C3 a, C3 b, int sign, P3 out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) out.p[c][i] = sign > 0 ? a.p[c][i] + b.p[c][i] : a.p[c][i] - b.p[c][i];
}

// One wave per edaBit row p, lane j = bit position j.
__global__ __launch_bounds__(256) void k_eda_rows(int64_t n, Keys k, u32 op, const u64* Mb, C3 rp, Inj m1inj,
                                                  u64* Xm, P3 w, P3 r) {
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= n) return;
    const int64_t e = p * 64 + lane;
    const u64 mb = (Mb[p] >> lane) & 1ull;
    const u64 xm = lane == 63 ? 0ull : mb << (lane + 1);     // 2^(j+1) mb_j (0 at j = 63)
    Xm[e] = xm;
    const u64 ym = rp.p[0][e], y1 = rp.p[1][e], y2 = rp.p[2][e];
    // P1: sum -x.m y.r1 (x has no mask planes); P2: sum x.m (y.m - y.r2)
    const u64 s1 = wave_sum(xm * y1);
    const u64 s2 = wave_sum(xm * (ym - y2));
    // sum_j 2^j (mb_j + rp_j) per plane
    const u64 l0 = wave_sum((mb + ym) << lane);
    const u64 l1 = wave_sum(y1 << lane);
    const u64 l2 = wave_sum(y2 << lane);
    if (lane == 0) {
        const u64 r1 = prg_word(k.k01, make_tag(op, P_EDA_W_R, 1, 0), (u64)p);
        const u64 r2 = prg_word(k.k02, make_tag(op, P_EDA_W_R, 2, 0), (u64)p);
        const u64 g1 = prg_word(k.k01, make_tag(op, P_EDA_W_GAMMA, 1, 0), (u64)p);
        const u64 g2 = r1 + r2 - g1;                  // P0: Gamma = 0 + r1 + r2 (x has no r planes)
        u64 m1 = g1 - s1;                             // P1 -> P2
        if (p == m1inj.index) m1 += m1inj.e;
        const u64 m2 = s2 + g2;                       // P2 -> P1
        const u64 wm = m1 + m2;
        w.p[0][p] = wm;
        w.p[1][p] = r1;
        w.p[2][p] = r2;
        r.p[0][p] = l0 - wm;
        r.p[1][p] = l1 - r1;
        r.p[2][p] = l2 - r2;
    }
}

__global__ void k_and_words(int64_t n, Keys k, u32 op, C3 a, C3 b, Inj g2inj, P3 c) {
    const int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i0 = blk * 8;
    if (i0 >= n) return;
    u64 rz1[8], rz2[8], g1[8];
    prg_block8(k.k01, make_tag(op, P_AND_RZ, 1, 0), blk, rz1);
    prg_block8(k.k02, make_tag(op, P_AND_RZ, 2, 0), blk, rz2);
    prg_block8(k.k01, make_tag(op, P_AND_GAMMA, 1, 0), blk, g1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t i = i0 + q;
        if (i >= n) break;
        const u64 am = a.p[0][i], a1 = a.p[1][i], a2 = a.p[2][i];
        const u64 bm = b.p[0][i], b1 = b.p[1][i], b2 = b.p[2][i];
        const u64 gamma = ((a1 ^ a2) & (b1 ^ b2)) ^ rz1[q] ^ rz2[q];       // P0
        u64 g2 = gamma ^ g1[q];
        if (i == g2inj.index) g2 ^= g2inj.e;
        const u64 m1 = (am & b1) ^ (bm & a1) ^ g1[q];                      // P1
        const u64 m2 = (am & bm) ^ (am & b2) ^ (bm & a2) ^ g2;             // P2
        c.p[0][i] = m1 ^ m2;
        c.p[1][i] = rz1[q];
        c.p[2][i] = rz2[q];
    }
}

__global__ void k_open_diff(int64_t n, C3 x, C3 r, u64* delta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    delta[i] = (x.p[0][i] - r.p[0][i]) - (x.p[1][i] - r.p[1][i]) - (x.p[2][i] - r.p[2][i]);
}

__global__ void k_a2b_init(int64_t n, C3 R, const u64* delta, P3 P0, P3 G, P3 P) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u64 d = delta[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const u64 v = R.p[c][i];
        const u64 pv = c == 0 ? v ^ d : v;
        P0.p[c][i] = pv;
        P.p[c][i] = pv;
        G.p[c][i] = v & d;
    }
}

__global__ void k_ks_prep(int64_t n, int k, int last, C3 P, C3 G, P3 A, P3 B) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const u64 pv = P.p[c][i], gv = G.p[c][i];
        A.p[c][i] = pv;
        B.p[c][i] = gv << k;
        if (!last) {
            A.p[c][n + i] = pv;
            B.p[c][n + i] = pv << k;
        }
    }
}

__global__ void k_ks_update(int64_t n, int last, C3 C, P3 G, P3 P) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        G.p[c][i] ^= C.p[c][i];
        if (!last) P.p[c][i] = C.p[c][n + i];
    }
}

__global__ void k_msb_final(int64_t n, C3 P0, C3 G, int flip, P3 out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        u64 v = (P0.p[c][i] ^ (G.p[c][i] << 1)) >> 63;
        if (c == 0 && flip) v ^= 1;
        out.p[c][i] = v;
    }
}

__global__ void k_b2a(int64_t n, C3 d, C3 sb, C3 sa, P3 dl) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u64 e = (d.p[0][i] ^ sb.p[0][i] ^ d.p[1][i] ^ sb.p[1][i] ^ d.p[2][i] ^ sb.p[2][i]) & 1ull;
    const u64 f = 1 - 2 * e;
    dl.p[0][i] = e + f * sa.p[0][i];
    dl.p[1][i] = f * sa.p[1][i];
    dl.p[2][i] = f * sa.p[2][i];
}

__global__ void k_pool_gather(int B, int H, int W, int C, C3 x, P3 p, P3 q) {
    const int64_t N = (int64_t)B * (H / 2) * (W / 2) * C;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int ch = (int)(i % C);
    int64_t t = i / C;
    const int j = (int)(t % (W / 2));
    t /= (W / 2);
    const int h = (int)(t % (H / 2));
    const int64_t b = t / (H / 2);
    const int64_t base = ((b * H + 2 * h) * W + 2 * j) * C + ch;
    const int64_t right = C, down = (int64_t)W * C;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const u64* v = x.p[c];
        p.p[c][i] = v[base];
        p.p[c][N + i] = v[base + down];
        q.p[c][i] = v[base + right];
        q.p[c][N + i] = v[base + down + right];
    }
}

// out[c][e, k] = a_c[e] * P[e / per, k] (element e of a gate scaled by the gate's power;
// null planes give 0), planes ps apart.
__global__ void k_scale_gates(int64_t n, int per, C3 a, const u64* P, u64* out, int64_t ps) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * 64) return;
    const int64_t e = idx >> 6;
    const u64 p = P[(e / per) * 64 + (idx & 63)];
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * ps + idx] = a.p[c] ? a.p[c][e] * p : 0;
}

// ---------------------------------------------------------------------------
// Pi_MultVerify over GF(2^64)
// ---------------------------------------------------------------------------

__global__ void k_gf_random(Keys k, u32 op, u32 purpose, u32 sub, u64* share3, u64* value, u64* log) {
    if (threadIdx.x != 0) return;
    const u64 m = prg_word(k.k12, make_tag(op, purpose, 0, sub), 0);
    const u64 r1 = prg_word(k.k01, make_tag(op, purpose, 1, sub), 0);
    const u64 r2 = prg_word(k.k02, make_tag(op, purpose, 2, sub), 0);
    if (share3) {
        share3[0] = m;
        share3[1] = r1;
        share3[2] = r2;
    }
    if (value) value[0] = m ^ r1 ^ r2;
    if (log) log[0] = m ^ r1 ^ r2;
}

__global__ void k_gf_pow_tables(const u64* rp, int64_t W, u64* T0, u64* T1) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const u64 r = rp[0];
    if (i < 64) T0[i] = gf_pow(r, (u64)i);
    if (i < W) T1[i] = gf_pow(gf_pow(r, 64), (u64)i);
}

// One wave per word w of the triples, lane b = gate 64 w + b.
__global__ __launch_bounds__(256) void k_gf_tran(int64_t W, const u64* T0, const u64* T1, C3 A, C3 B, C3 C, u64* XY,
                                                 int64_t npad, u64* zpart) {
    __shared__ u64 zs[4][3];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t w = (int64_t)blockIdx.x * 4 + wv;
    u64 z0 = 0, z1 = 0, z2 = 0;
    if (w < W) {
        const u64 pw = gf_mul(T1[w], T0[lane]);
        const int64_t g = w * 64 + lane;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            XY[c * npad + g] = ((A.p[c][w] >> lane) & 1ull) ? pw : 0ull;
            XY[(3 + c) * npad + g] = (B.p[c][w] >> lane) & 1ull;
        }
        z0 = ((C.p[0][w] >> lane) & 1ull) ? pw : 0ull;
        z1 = ((C.p[1][w] >> lane) & 1ull) ? pw : 0ull;
        z2 = ((C.p[2][w] >> lane) & 1ull) ? pw : 0ull;
    }
    z0 = wave_xor(z0);
    z1 = wave_xor(z1);
    z2 = wave_xor(z2);
    if (lane == 0) {
        zs[wv][0] = z0;
        zs[wv][1] = z1;
        zs[wv][2] = z2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int c = threadIdx.x;
        zpart[(int64_t)blockIdx.x * 3 + c] = zs[0][c] ^ zs[1][c] ^ zs[2][c] ^ zs[3][c];
    }
}

// XOR of nparts groups of `width` words into out (one block).
__global__ void k_gf_xor_parts(int64_t nparts, int width, const u64* part, u64* out) {
    __shared__ u64 red[256];
    for (int c = 0; c < width; ++c) {
        u64 v = 0;
        for (int64_t i = threadIdx.x; i < nparts; i += blockDim.x) v ^= part[i * width + c];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] ^= red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = red[0];
        __syncthreads();
    }
}

// zero padding rows of the six planes
__global__ void k_gf_pad(u64* XY, int64_t from, int64_t npad) {
    const int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
#pragma unroll
    for (int c = 0; c < 6; ++c) XY[c * npad + i] = 0;
}

// The three party sums of a Pi_PolyEvl term a * b (a = (am, a1, a2), b likewise).
__device__ __forceinline__ void gf_party(u64 am, u64 a1, u64 a2, u64 bm, u64 b1, u64 b2, u64& s0, u64& s1, u64& s2) {
    s0 ^= gf_mul(a1 ^ a2, b1 ^ b2);                            // P0
    s1 ^= gf_mul(am, b1) ^ gf_mul(bm, a1);                     // P1
    s2 ^= gf_mul(am, bm) ^ gf_mul(am, b2) ^ gf_mul(bm, a2);    // P2
}

// Per block: the six sums (h(0): P0, P1, P2; h(x): P0, P1, P2) over its pairs.
__global__ __launch_bounds__(256) void k_gf_round_dot(int64_t n, const u64* XY, int64_t ps, u64* part) {
    __shared__ u64 red[6][256];
    const int t = threadIdx.x;
    u64 s[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + t; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        u64 f0[6], f1[6], f2[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            f0[c] = XY[c * ps + 2 * i];
            f1[c] = XY[c * ps + 2 * i + 1];
            f2[c] = gf_xtime(f1[c] ^ f0[c]) ^ f0[c];           // x f(1) + (x + 1) f(0)
        }
        gf_party(f0[0], f0[1], f0[2], f0[3], f0[4], f0[5], s[0], s[1], s[2]);
        gf_party(f2[0], f2[1], f2[2], f2[3], f2[4], f2[5], s[3], s[4], s[5]);
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) red[q][t] = s[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int q = 0; q < 6; ++q) red[q][t] ^= red[q][t + h];
        __syncthreads();
    }
    if (t < 6) part[(int64_t)blockIdx.x * 6 + t] = red[t][0];
}

// Pi_PolyEvl outputs over GF(2^64) from the three party sums (masks from (op, pr / pg, sub)).
struct GfPe {
    u64 m1, m2, g2, out[3];
};
__device__ GfPe gf_pe(const Keys& k, u32 op, u32 pr, u32 pg, u32 sub, u64 s0, u64 s1, u64 s2) {
    GfPe o;
    const u64 rc1 = prg_word(k.k01, make_tag(op, pr, 1, sub), 0);
    const u64 rc2 = prg_word(k.k02, make_tag(op, pr, 2, sub), 0);
    const u64 g1 = prg_word(k.k01, make_tag(op, pg, 1, sub), 0);
    o.g2 = s0 ^ rc1 ^ rc2 ^ g1;          // P0 -> P2
    o.m1 = s1 ^ g1;                      // P1 -> P2
    o.m2 = s2 ^ o.g2;                    // P2 -> P1
    o.out[0] = o.m1 ^ o.m2;
    o.out[1] = rc1;
    o.out[2] = rc2;
    return o;
}

__global__ void k_gf_round_finish(int64_t nparts, const u64* part, GfRoundArgs a) {
    __shared__ u64 red[6][256];
    const int t = threadIdx.x;
    u64 s[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = t; i < nparts; i += blockDim.x)
#pragma unroll
        for (int q = 0; q < 6; ++q) s[q] ^= part[i * 6 + q];
#pragma unroll
    for (int q = 0; q < 6; ++q) red[q][t] = s[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int q = 0; q < 6; ++q) red[q][t] ^= red[q][t + h];
        __syncthreads();
    }
    if (t != 0) return;
    const GfPe h0 = gf_pe(a.k, a.op, P_VER_H0_R, P_VER_H0_GAMMA, a.sub, red[0][0], red[1][0], red[2][0]);
    const GfPe h2 = gf_pe(a.k, a.op, P_VER_H2_R, P_VER_H2_GAMMA, a.sub, red[3][0], red[4][0], red[5][0]);
    const u64 zm = prg_word(a.k.k12, make_tag(a.op, P_VER_ZETA, 0, a.sub), 0);
    const u64 z1 = prg_word(a.k.k01, make_tag(a.op, P_VER_ZETA, 1, a.sub), 0);
    const u64 z2 = prg_word(a.k.k02, make_tag(a.op, P_VER_ZETA, 2, a.sub), 0);
    const u64 zeta = zm ^ z1 ^ z2;                       // revealed
    const u64 X = 2;
    const u64 L0 = gf_mul(gf_mul(zeta ^ 1, zeta ^ X), a.inv[0]);
    const u64 L1 = gf_mul(gf_mul(zeta, zeta ^ X), a.inv[1]);
    const u64 L2 = gf_mul(gf_mul(zeta, zeta ^ 1), a.inv[2]);
    for (int c = 0; c < 3; ++c) {
        const u64 h1 = a.z[c] ^ h0.out[c];               // h(1) = z - h(0)
        a.z[c] = gf_mul(L0, h0.out[c]) ^ gf_mul(L1, h1) ^ gf_mul(L2, h2.out[c]);
    }
    a.zeta[0] = zeta;
    if (a.log_zeta) a.log_zeta[0] = zeta;
    if (a.log_h0) {
        a.log_h0[0] = h0.m1;
        a.log_h0[64] = h0.m2;
        a.log_h0[128] = h0.g2;
        a.log_h2[0] = h2.m1;
        a.log_h2[64] = h2.m2;
        a.log_h2[128] = h2.g2;
    }
}

// f(zeta) = zeta f(1) + (zeta + 1) f(0) = zeta (f(1) ^ f(0)) ^ f(0), six planes.
__global__ void k_gf_fold(int64_t n, const u64* XY, int64_t ps, const u64* zetap, u64* XYn, int64_t psn) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u64 zeta = zetap[0];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const u64 v0 = XY[c * ps + 2 * i], v1 = XY[c * ps + 2 * i + 1];
        XYn[c * psn + i] = gf_mul(zeta, v1 ^ v0) ^ v0;
    }
}

// Pi_InnerVerify, part 1: x'_i = Pi_Mult(x_i, alpha) with fresh masks (rows of 8 words per
// thread, one PRG block each), and the block sums of sum x'_i y_i for the three parties.
__global__ __launch_bounds__(256) void k_gf_xp_dot(int64_t n, const u64* XY, int64_t ps, Keys k, u32 op, u32 sub,
                                                   const u64* alpha, u64* part) {
    __shared__ u64 red[3][256];
    const int t = threadIdx.x;
    const int64_t blk = (int64_t)blockIdx.x * blockDim.x + t;
    const int64_t i0 = blk * 8;
    u64 s0 = 0, s1 = 0, s2 = 0;
    if (i0 < n) {
        u64 r1[8], r2[8], g1[8];
        prg_block8(k.k01, make_tag(op, P_VER_XP_R, 1, sub), blk, r1);
        prg_block8(k.k02, make_tag(op, P_VER_XP_R, 2, sub), blk, r2);
        prg_block8(k.k01, make_tag(op, P_VER_XP_GAMMA, 1, sub), blk, g1);
        const u64 am = alpha[0], a1 = alpha[1], a2 = alpha[2];
        for (int q = 0; q < 8; ++q) {
            const int64_t i = i0 + q;
            if (i >= n) break;
            const u64 xm = XY[i], x1 = XY[ps + i], x2 = XY[2 * ps + i];
            const u64 gamma = gf_mul(x1 ^ x2, a1 ^ a2) ^ r1[q] ^ r2[q];            // P0
            const u64 g2 = gamma ^ g1[q];
            const u64 m1 = gf_mul(xm, a1) ^ gf_mul(am, x1) ^ g1[q];                 // P1
            const u64 m2 = gf_mul(xm, am) ^ gf_mul(xm, a2) ^ gf_mul(am, x2) ^ g2;   // P2
            gf_party(m1 ^ m2, r1[q], r2[q], XY[3 * ps + i], XY[4 * ps + i], XY[5 * ps + i], s0, s1, s2);
        }
    }
    red[0][t] = s0;
    red[1][t] = s1;
    red[2][t] = s2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int q = 0; q < 3; ++q) red[q][t] ^= red[q][t + h];
        __syncthreads();
    }
    if (t < 3) part[(int64_t)blockIdx.x * 3 + t] = red[t][0];
}

// Pi_InnerVerify, part 2: the pair (-alpha, z) = (alpha, z), the Pi_PolyEvl outputs, the
// opening of Delta, and the flag.
__global__ void k_gf_delta_finish(int64_t nparts, const u64* part, const u64* alpha, GfDeltaArgs a) {
    __shared__ u64 red[3][256];
    const int t = threadIdx.x;
    u64 s[3] = {0, 0, 0};
    for (int64_t i = t; i < nparts; i += blockDim.x)
#pragma unroll
        for (int q = 0; q < 3; ++q) s[q] ^= part[i * 3 + q];
#pragma unroll
    for (int q = 0; q < 3; ++q) red[q][t] = s[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int q = 0; q < 3; ++q) red[q][t] ^= red[q][t + h];
        __syncthreads();
    }
    if (t != 0) return;
    u64 s0 = red[0][0], s1 = red[1][0], s2 = red[2][0];
    gf_party(alpha[0], alpha[1], alpha[2], a.z[0], a.z[1], a.z[2], s0, s1, s2);
    const GfPe d = gf_pe(a.k, a.op, P_VER_DELTA_R, P_VER_DELTA_GAMMA, a.sub, s0, s1, s2);
    const u64 delta = d.out[0] ^ d.out[1] ^ d.out[2];
    if (a.log_delta) a.log_delta[0] = delta;
    if (a.log_tr) {
        a.log_tr[0] = d.m1;
        a.log_tr[64] = d.m2;
        a.log_tr[128] = d.g2;
    }
    if (delta) atomicOr(a.flag, 1);
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------

void launch_lift_bits(int64_t n, int per, const u64* B, int neg, u64* out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_lift_bits, dim3(nblk(n, TPB)), dim3(TPB), 0, s, n, per, B, neg, out);
}
void launch_lin3(int64_t n, C3 x, C3 y, C3 z, P3 out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_lin3, dim3(nblk(n, TPB)), dim3(TPB), 0, s, n, x, y, z, out);
}
void launch_addsub3(int64_t n, C3 a, C3 b, int sign, P3 out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_addsub3, dim3(nblk(n, TPB)), dim3(TPB), 0, s, n, a, b, sign, out);
}
void launch_eda_rows(int64_t n, const Keys& k, u32 op, const u64* Mb, C3 rp, Inj m1inj, u64* Xm, P3 w, P3 r,
                     hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_eda_rows, dim3(nblk(n, 4)), dim3(256), 0, s, n, k, op, Mb, rp, m1inj, Xm, w, r);
}
void launch_and_words(int64_t n, const Keys& k, u32 op, C3 a, C3 b, Inj g2inj, P3 c, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_and_words, dim3(nblk((n + 7) / 8, TPB)), dim3(TPB), 0, s, n, k, op, a, b, g2inj, c);
}
void launch_open_diff(int64_t n, C3 x, C3 r, u64* delta, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_open_diff, dim3(nblk(n, TPB)), dim3(TPB), 0, s, n, x, r, delta);
}
void launch_a2b_init(int64_t n, C3 R, const u64* delta, P3 P0, P3 G, P3 P, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_a2b_init, dim3(nblk(n, TPB)), dim3(TPB), 0, s, n, R, delta, P0, G, P);
}
void launch_ks_prep(int64_t n, int k, bool last, C3 P, C3 G, P3 A, P3 B, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_ks_prep, dim3(nblk(n, TPB)), dim3(TPB), 0, s, n, k, last ? 1 : 0, P, G, A, B);
}
void launch_ks_update(int64_t n, bool last, C3 C, P3 G, P3 P, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_ks_update, dim3(nblk(n, TPB)), dim3(TPB), 0, s, n, last ? 1 : 0, C, G, P);
}
void launch_msb_final(int64_t n, C3 P0, C3 G, bool flip, P3 out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_msb_final, dim3(nblk(n, TPB)), dim3(TPB), 0, s, n, P0, G, flip ? 1 : 0, out);
}
void launch_b2a(int64_t n, C3 d, C3 sb, C3 sa, P3 dl, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_b2a, dim3(nblk(n, TPB)), dim3(TPB), 0, s, n, d, sb, sa, dl);
}
void launch_pool_gather(int B, int H, int W, int C, C3 x, P3 p, P3 q, hipStream_t s) {
    const int64_t N = (int64_t)B * (H / 2) * (W / 2) * C;
    if (N <= 0) return;
    hipLaunchKernelGGL(k_pool_gather, dim3(nblk(N, TPB)), dim3(TPB), 0, s, B, H, W, C, x, p, q);
}

void launch_scale_gates(int64_t n, int per, C3 a, const u64* P, u64* out, int64_t ps, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scale_gates, dim3(nblk(n * 64, TPB)), dim3(TPB), 0, s, n, per, a, P, out, ps);
}

void launch_gf_random(const Keys& k, u32 op, u32 purpose, u32 sub, u64* share3, u64* value, u64* log,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_gf_random, dim3(1), dim3(64), 0, s, k, op, purpose, sub, share3, value, log);
}
void launch_gf_pow_tables(const u64* r, int64_t W, u64* T0, u64* T1, hipStream_t s) {
    const int64_t n = W > 64 ? W : 64;
    hipLaunchKernelGGL(k_gf_pow_tables, dim3(nblk(n, TPB)), dim3(TPB), 0, s, r, W, T0, T1);
}
void launch_gf_tran(int64_t W, const u64* T0, const u64* T1, C3 A, C3 B, C3 C, u64* XY, int64_t npad, u64* zout,
                    void* (*ws)(void*, size_t), void* wss, hipStream_t s) {
    const int64_t nb = (W + 3) / 4;
    u64* part = (u64*)ws(wss, (size_t)(nb > 0 ? nb : 1) * 3 * 8);
    if (W > 0) hipLaunchKernelGGL(k_gf_tran, dim3((unsigned)nb), dim3(256), 0, s, W, T0, T1, A, B, C, XY, npad, part);
    if (npad > W * 64)
        hipLaunchKernelGGL(k_gf_pad, dim3(nblk(npad - W * 64, TPB)), dim3(TPB), 0, s, XY, W * 64, npad);
    hipLaunchKernelGGL(k_gf_xor_parts, dim3(1), dim3(256), 0, s, nb, 3, part, zout);
}
void launch_gf_round(int64_t n, const u64* XY, int64_t ps, u64* XYn, int64_t psn, const GfRoundArgs& a,
                     void* (*ws)(void*, size_t), void* wss, hipStream_t s) {
    int64_t nb = (n + TPB - 1) / TPB;
    if (nb > 2048) nb = 2048;
    if (nb < 1) nb = 1;
    u64* part = (u64*)ws(wss, (size_t)nb * 6 * 8);
    hipLaunchKernelGGL(k_gf_round_dot, dim3((unsigned)nb), dim3(TPB), 0, s, n, XY, ps, part);
    hipLaunchKernelGGL(k_gf_round_finish, dim3(1), dim3(TPB), 0, s, nb, part, a);
    if (n > 0) hipLaunchKernelGGL(k_gf_fold, dim3(nblk(n, TPB)), dim3(TPB), 0, s, n, XY, ps, a.zeta, XYn, psn);
}
void launch_gf_inner_verify(int64_t n, const u64* XY, int64_t ps, const GfDeltaArgs& a, void* (*ws)(void*, size_t),
                            void* wss, hipStream_t s) {
    u64* alpha = (u64*)ws(wss, 3 * 8);
    hipLaunchKernelGGL(k_gf_random, dim3(1), dim3(64), 0, s, a.k, a.op, (u32)P_VER_ALPHA, a.sub, alpha, (u64*)nullptr,
                       (u64*)nullptr);
    int64_t nb = ((n + 7) / 8 + TPB - 1) / TPB;
    if (nb < 1) nb = 1;
    u64* part = (u64*)ws(wss, (size_t)nb * 3 * 8);
    hipLaunchKernelGGL(k_gf_xp_dot, dim3((unsigned)nb), dim3(TPB), 0, s, n, XY, ps, a.k, a.op, a.sub, alpha, part);
    hipLaunchKernelGGL(k_gf_delta_finish, dim3(1), dim3(TPB), 0, s, nb, part, alpha, a);
}

// host GF(2^64)
static void clmul_host(u64 a, u64 b, u64& lo, u64& hi) {
    lo = hi = 0;
    for (int k = 0; k < 64; ++k)
        if ((b >> k) & 1) {
            lo ^= a << k;
            if (k) hi ^= a >> (64 - k);
        }
}
u64 gf_mul_host(u64 a, u64 b) {
    u64 lo, hi;
    clmul_host(a, b, lo, hi);
    return gf_reduce(lo, hi);
}
u64 gf_inv_host(u64 a) {
    // a^(2^64 - 2) = a^(2 + 4 + ... + 2^63)
    u64 out = 1, sq = a;
    for (int i = 1; i < 64; ++i) {
        sq = gf_mul_host(sq, sq);       // a^(2^i)
        out = gf_mul_host(out, sq);
    }
    return out;
}

}  // namespace mpc3
