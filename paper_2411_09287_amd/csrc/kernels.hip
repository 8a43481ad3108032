// Elementwise, PRG and Galois-ring kernels of the protocol (gfx950).
#include "kernels.h"
#include "limb_digits.h"

namespace mpc3 {

namespace {

constexpr int TPB = 256;

__host__ inline unsigned nblocks(int64_t work, int per_block) {
    return (unsigned)((work + per_block - 1) / per_block);
}

// ---------------------------------------------------------------------------
// Z_{2^64} elementwise
// ---------------------------------------------------------------------------

__global__ void k_fill(u64* out, int64_t n, int64_t start, Key k, Tag t) {
    // thread = one keystream block = 8 words of G(k, t, .) starting at an 8-aligned index
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t first = (start >> 3) + b;
    const int64_t w0 = first * 8;
    if (w0 >= start + n) return;
    u64 w[8];
    prg_block8(k, t, (u64)first, w);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t i = w0 + q - start;
        if (i >= 0 && i < n) out[i] = w[q];
    }
}

__global__ void k_encode(const double* x, int64_t n, double scale, u64* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (u64)(int64_t)floor(x[i] * scale);
}

__global__ void k_decode(const u64* v, int64_t n, double scale, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)(int64_t)v[i] / scale;
}

__global__ void k_share(const u64* x, int64_t n, Key k1, Tag t1, Key k2, Tag t2, u64* m, u64* r1, u64* r2,
                        const u32* op_off) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i0 = b * 8;
    if (i0 >= n) return;
    if (op_off) {
        t1.n0 += *op_off;
        t2.n0 += *op_off;
    }
    u64 w1[8], w2[8];
    prg_block8(k1, t1, (u64)b, w1);
    prg_block8(k2, t2, (u64)b, w2);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t i = i0 + q;
        if (i < n) {
            r1[i] = w1[q];
            r2[i] = w2[q];
            m[i] = x[i] + w1[q] + w2[q];   // the owner's message m = x + [r]_1 + [r]_2
        }
    }
}

// Pi_Trunc preprocessing for outputs p: bit words B1 (P0,P1) and B2 (P0,P2); the two
// inner products over the 64 bit positions collapse to word operations:
//   sum_j 2^{j+1} b1_j * (-b2_j) = -2 (B1 & B2),   sum_j 2 c_j b1_j * (-b2_j) = -2 ash(B1 & B2, t).
// The words 8 blk0 .. 8 blk0 + 511 of G(key, tag, .) for one wave: each lane computes
// block blk0 + lane, and the 64 x 8 words are exchanged through lds (64 x 9 words) so that
// out[q] is word 8 blk0 + 64 q + lane (consecutive lanes, consecutive words).
__device__ __forceinline__ void prg_wave512(const Key& k, const Tag& t, u64 blk0, u64* lds, u64 out[8]) {
    const int lane = threadIdx.x & 63;
    u64 w[8];
    prg_block8(k, t, blk0 + lane, w);
#pragma unroll
    for (int q = 0; q < 8; ++q) lds[lane * 9 + q] = w[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) out[q] = lds[(q * 8 + (lane >> 3)) * 9 + (lane & 7)];
    __syncthreads();
}

// A wave covers 512 consecutive elements and its lanes take consecutive ones (the keystream
// words come through prg_wave512); the eight streams are drawn one after another.
__global__ void k_trunc_pair(int64_t n, int t, Keys k, u32 op, Inj g2x, Inj m1z, u64* rxm, u64* rx1,
                             u64* rx2, u64* rzm, u64* rz1, u64* rz2, const u32* op_off) {
    if (op_off) op += *op_off;
    __shared__ u64 lds[4][64 * 9];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t blk0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;
    const int64_t base = blk0 * 8 + lane;
    u64 B1[8], B2[8], acc[8], w[8];
    prg_wave512(k.k01, make_tag(op, P_TRUNC_B, 1, 0), blk0, lds[wv], B1);
    prg_wave512(k.k02, make_tag(op, P_TRUNC_B, 2, 0), blk0, lds[wv], B2);
    // r_x product: fresh output mask [r_w]_1, [r_w]_2 and P0's [Gamma]_1
    prg_wave512(k.k01, make_tag(op, P_TRUNC_WX_R, 1, 0), blk0, lds[wv], w);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t p = base + 64 * q;
        acc[q] = (0 - 2 * (B1[q] & B2[q])) + w[q];                            // P0's gamma, part
        if (p < n) rx1[p] = w[q] - B1[q];       // + sum 2^j <b1_j> = (0, -B1, 0)
    }
    prg_wave512(k.k02, make_tag(op, P_TRUNC_WX_R, 2, 0), blk0, lds[wv], w);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t p = base + 64 * q;
        acc[q] += w[q];
        if (p < n) rx2[p] = w[q] - B2[q];       // + sum 2^j <b2_j> = (0, 0, -B2)
    }
    prg_wave512(k.k01, make_tag(op, P_TRUNC_WX_GAMMA, 1, 0), blk0, lds[wv], w);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t p = base + 64 * q;
        u64 g2 = acc[q] - w[q];                                                // P0 -> P2
        if (p == g2x.index) g2 += g2x.e;
        if (p < n) rxm[p] = w[q] + g2;                                         // P1 <-> P2 exchange
    }
    // r_z product
    prg_wave512(k.k01, make_tag(op, P_TRUNC_WZ_R, 1, 0), blk0, lds[wv], w);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t p = base + 64 * q;
        acc[q] = (0 - 2 * ash(B1[q] & B2[q], t)) + w[q];
        if (p < n) rz1[p] = w[q] - ash(B1[q], t);
    }
    prg_wave512(k.k02, make_tag(op, P_TRUNC_WZ_R, 2, 0), blk0, lds[wv], w);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t p = base + 64 * q;
        acc[q] += w[q];
        if (p < n) rz2[p] = w[q] - ash(B2[q], t);
    }
    prg_wave512(k.k01, make_tag(op, P_TRUNC_WZ_GAMMA, 1, 0), blk0, lds[wv], w);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t p = base + 64 * q;
        const u64 g2 = acc[q] - w[q];
        u64 m1 = w[q];
        if (p == m1z.index) m1 += m1z.e;
        if (p < n) rzm[p] = m1 + g2;
    }
}

// Pi_Inner preprocessing: output-wire mask [r_Z] (fresh, or the truncation pair's r_x) and
// [Gamma]_1.  A wave covers 512 consecutive words; its lanes take consecutive words.
__global__ void k_inner_pre(int64_t n, Keys k, u32 op, const u64* pm, const u64* p1, const u64* p2,
                            u64* zr1, u64* zr2, u64* g1, const u32* op_off) {
    if (op_off) op += *op_off;
    __shared__ u64 lds[4][64 * 9];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t blk0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;   // the wave's first block
    const int64_t base = blk0 * 8 + lane;
    u64 w[8], v[8];
    prg_wave512(k.k01, make_tag(op, P_INNER_GAMMA, 1, 0), blk0, lds[wv], w);
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if (base + 64 * q < n) g1[base + 64 * q] = w[q];
    if (pm) {   // P1: [r_x]_1 = m_{r_x} - [r_{r_x}]_1 ; P2: [r_x]_2 = -[r_{r_x}]_2
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = base + 64 * q;
            if (i < n) {
                zr1[i] = pm[i] - p1[i];
                zr2[i] = 0 - p2[i];
            }
        }
    } else {
        prg_wave512(k.k01, make_tag(op, P_INNER_RZ, 1, 0), blk0, lds[wv], w);
        prg_wave512(k.k02, make_tag(op, P_INNER_RZ, 2, 0), blk0, lds[wv], v);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = base + 64 * q;
            if (i < n) {
                zr1[i] = w[q];
                zr2[i] = v[q];
            }
        }
    }
}

// Pi_Inner messages and output from the party accumulators.
__global__ void k_inner_post(int64_t n, const u64* c0, const u64* c1, const u64* c2, const u64* zr1,
                             const u64* zr2, const u64* g1, Inj g2inj, Inj m1inj, u64* zm, u64* mg2,
                             u64* mm1, u64* mm2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u64 gamma = c0[i] + zr1[i] + zr2[i];        // P0: R_X R_W + r_Z
    u64 g2 = gamma - g1[i];                           // P0 -> P2
    if (i == g2inj.index) g2 += g2inj.e;
    u64 m1 = g1[i] - c1[i];                           // P1
    if (i == m1inj.index) m1 += m1inj.e;
    const u64 m2 = c2[i] + g2;                        // P2
    zm[i] = m1 + m2;                                  // after the P1 <-> P2 exchange
    if (mg2) {
        mg2[i] = g2;
        mm1[i] = m1;
        mm2[i] = m2;
    }
}

__global__ void k_trunc_shift(int64_t n, int t, const u64* zm, const u64* rzm, const u64* rz1,
                              const u64* rz2, u64* om, u64* o1, u64* o2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    om[i] = ash(zm[i], t);
    o1[i] = rzm[i] - rz1[i];
    o2[i] = 0 - rz2[i];
}

__global__ void k_mult(int64_t n, Keys k, u32 op, const u64* am, const u64* a1, const u64* a2,
                       const u64* bm, const u64* b1, const u64* b2, Inj g2inj, u64* cm, u64* c1, u64* c2,
                       u64* mg2, u64* mm1, u64* mm2) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i0 = b * 8;
    if (i0 >= n) return;
    u64 rz1[8], rz2[8], g1[8];
    prg_block8(k.k01, make_tag(op, P_MULT_RZ, 1, 0), b, rz1);
    prg_block8(k.k02, make_tag(op, P_MULT_RZ, 2, 0), b, rz2);
    prg_block8(k.k01, make_tag(op, P_MULT_GAMMA, 1, 0), b, g1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t i = i0 + q;
        if (i >= n) break;
        const u64 gamma = (a1[i] + a2[i]) * (b1[i] + b2[i]) + rz1[q] + rz2[q];
        u64 g2 = gamma - g1[q];
        if (i == g2inj.index) g2 += g2inj.e;
        const u64 m1 = g1[q] - am[i] * b1[i] - bm[i] * a1[i];
        const u64 m2 = am[i] * bm[i] - am[i] * b2[i] - bm[i] * a2[i] + g2;
        cm[i] = m1 + m2;
        c1[i] = rz1[q];
        c2[i] = rz2[q];
        if (mg2) {
            mg2[i] = g2;
            mm1[i] = m1;
            mm2[i] = m2;
        }
    }
}

// rows (b, oh, ow), columns (kh, kw, c) of a stride-1 convolution with zero padding
__global__ void k_im2col(const u64* x, int B, int H, int W, int C, int KH, int KW, int pad, int stride, int OH,
                         int OW, int64_t ld, u64* out) {
    const int64_t K = (int64_t)KH * KW * C;
    const int64_t total = (int64_t)B * OH * OW * ld;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int64_t row = idx / ld;
    const int col = (int)(idx - row * ld);
    if (col >= K) {                      // zero columns of a padded contraction width
        out[idx] = 0;
        return;
    }
    const int c = col % C;
    const int kw = (col / C) % KW;
    const int kh = col / (C * KW);
    const int ow = (int)(row % OW);
    const int oh = (int)((row / OW) % OH);
    const int b = (int)(row / ((int64_t)OW * OH));
    const int ih = stride * oh + kh - pad, iw = stride * ow + kw - pad;
    u64 v = 0;
    if (ih >= 0 && ih < H && iw >= 0 && iw < W) v = x[(((int64_t)b * H + ih) * W + iw) * C + c];
    out[idx] = v;
}

// floor(n / d) for n < 2^31 by one multiply and shift: with s = ceil(log2 d) and
// M = ceil(2^(32+s) / d), M d = 2^(32+s) + e (0 <= e < d) and n e < 2^(32+s), so the error
// term stays below 1/d and the quotient is exact.
struct FastDiv {
    u64 M;
    u32 d;
    int sh;
};
__host__ inline FastDiv make_fastdiv(u32 d) {
    FastDiv f{};
    f.d = d;
    f.sh = 0;
    while ((1ull << f.sh) < d) ++f.sh;
    const u64 p = 1ull << (32 + f.sh);
    f.M = p / d + (p % d ? 1 : 0);
    return f;
}
__device__ __forceinline__ u32 fdiv(u32 n, const FastDiv& f) { return (u32)(((u64)n * f.M) >> (32 + f.sh)); }

struct Im2colArgs {
    const u64* x[3];
    u64* out[3];
    int H, W, C, KW, OH, OW, pad, stride;
    u32 K, ld, total;      // words per output row (KH KW C) and the row stride ld >= K
                           // (columns K .. ld-1 are zero); V-word groups in a plane
    FastDiv fLD, fC, fKW, fOW, fOH;
};

// V consecutive output words per thread (V = 2: 16-byte loads and stores, C and K even),
// 32-bit index arithmetic; blockIdx.y is the share plane.
template <int V>
__global__ void k_im2col3(Im2colArgs a) {
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.total) return;
    const u64* x = a.x[blockIdx.y];
    u64* out = a.out[blockIdx.y];
    const u32 w = i * V;                          // word index within the plane
    const u32 row = fdiv(w, a.fLD), col = w - row * a.ld;
    if (col >= a.K) {                             // zero columns (K and ld even when V = 2)
        if (V == 2) *(ulonglong2*)(out + w) = ulonglong2{0, 0};
        else out[w] = 0;
        return;
    }
    const u32 seg = fdiv(col, a.fC), c = col - seg * a.C;
    const u32 kh = fdiv(seg, a.fKW), kw = seg - kh * a.KW;
    const u32 t = fdiv(row, a.fOW), ow = row - t * a.OW;
    const u32 b = fdiv(t, a.fOH), oh = t - b * a.OH;
    const int ih = a.stride * (int)oh + (int)kh - a.pad, iw = a.stride * (int)ow + (int)kw - a.pad;
    const bool in = ih >= 0 && ih < a.H && iw >= 0 && iw < a.W;
    const int64_t src = (((int64_t)b * a.H + ih) * a.W + iw) * a.C + c;
    if (V == 2) {
        ulonglong2 v = {0, 0};
        if (in) v = *(const ulonglong2*)(x + src);
        *(ulonglong2*)(out + w) = v;
    } else {
        out[w] = in ? x[src] : 0;
    }
}

__global__ void k_sumpool2(const u64* x, int B, int H, int W, int C, u64* out) {
    const int OH = H / 2, OW = W / 2;
    const int64_t total = (int64_t)B * OH * OW * C;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int c = (int)(idx % C);
    const int ow = (int)((idx / C) % OW);
    const int oh = (int)((idx / ((int64_t)C * OW)) % OH);
    const int b = (int)(idx / ((int64_t)C * OW * OH));
    const u64* p = x + (((int64_t)b * H + 2 * oh) * W + 2 * ow) * C + c;
    out[idx] = p[0] + p[C] + p[(int64_t)W * C] + p[(int64_t)W * C + C];
}

// Pi_Rec: P2 compares the [r]_1 that P0 sent (with an injected error, if any) with P1's
// hash of its own copy (equal hashes <=> equal words); any difference sets the flag.
__global__ void k_rec_check(int64_t n, const u64* r1, Inj inj, int* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u64 mine = r1[i];
    const u64 sent = r1[i] + (i == inj.index ? inj.e : 0);
    if (sent != mine) atomicOr(flag, 1);
}

// The opened values, written only if no receiver saw an inconsistency.
__global__ void k_rec_open(int64_t n, const u64* m, const u64* r1, const u64* r2, const int* flag, u64* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || *flag) return;
    out[i] = m[i] - r1[i] - r2[i];
}

// ---------------------------------------------------------------------------
// Galois ring GR(2^64, 64): products and reduction inside one 64-lane group
// ---------------------------------------------------------------------------

// Reduce the product whose coefficient k is `lo` and coefficient 64 + k is `hi` (lane k).
__device__ u64 reduce_lane(u64 lo, u64 hi, u64* sh, int k) {
    sh[k] = hi;
    __syncthreads();
    u64 v = lo;
#pragma unroll
    for (int q = 0; q < NTAPS; ++q) {
        const int j = k - tap(q);
        if (j >= 0) v -= sh[j];
    }
    // positions 64 + p (p <= 2) reached by x^{64+j} x^{t} with j + t >= 64 are reduced again
#pragma unroll
    for (int q = 0; q < NTAPS; ++q) {
        const int p = k - tap(q);
        if (p >= 0 && p <= 2) {
            u64 ov = 0;
#pragma unroll
            for (int r = 0; r < NTAPS; ++r) {
                const int j = 64 + p - tap(r);
                if (j >= 0 && j <= 62) ov -= sh[j];
            }
            v -= ov;
        }
    }
    __syncthreads();
    return v;
}

// Coefficient k of a * b with a, b visible to the 64-lane group.
__device__ u64 gr_mul_lane(const u64* a, const u64* b, u64* sh, int k) {
    u64 lo = 0, hi = 0;
    for (int i = 0; i < 64; ++i) {
        const u64 p = a[i] * b[(k - i) & 63];
        if (i <= k) lo += p; else hi += p;
    }
    return reduce_lane(lo, hi, sh, k);
}

// Words 0..63 of G(key_j, tag_j) for three streams j into out[j][.]: thread t < 24 computes
// block t % 8 of stream t / 8 (one ChaCha block per eight words).  Every thread of the
// block calls it (it synchronises the block; blockDim.x >= 24).
__device__ void prg_rows3(const Key& k0, const Tag& t0, const Key& k1, const Tag& t1, const Key& k2,
                          const Tag& t2, u64 (*out)[64]) {
    const int t = threadIdx.x;
    if (t < 24) {
        const int j = t >> 3, b = t & 7;
        u64 w[8];
        prg_block8(j == 0 ? k0 : j == 1 ? k1 : k2, j == 0 ? t0 : j == 1 ? t1 : t2, (u64)b, w);
#pragma unroll
        for (int q = 0; q < 8; ++q) out[j][8 * b + q] = w[q];
    }
    __syncthreads();
}

__global__ void k_random_gr(Keys k, u32 op, u32 purpose, u32 sub, u64* share3, u64* value, u64* log) {
    __shared__ u64 rows[3][64];
    const int c = threadIdx.x;
    prg_rows3(k.k12, make_tag(op, purpose, 0, sub), k.k01, make_tag(op, purpose, 1, sub), k.k02,
              make_tag(op, purpose, 2, sub), rows);
    const u64 m = rows[0][c], r1 = rows[1][c], r2 = rows[2][c];
    if (share3) {
        share3[c] = m;
        share3[64 + c] = r1;
        share3[128 + c] = r2;
    }
    const u64 v = m - r1 - r2;
    if (value) value[c] = v;
    if (log) log[c] = v;
}

__global__ void k_mulmat(const u64* src, int64_t stride, u64* W) {
    __shared__ u64 cur[64];
    const int k = threadIdx.x;
    const u64* v = src + blockIdx.x * stride;
    u64* out = W + (int64_t)blockIdx.x * 4096;
    u64 c = v[k];
    for (int j = 0; j < 64; ++j) {
        out[j * 64 + k] = c;          // row j = v * x^j
        cur[k] = c;
        __syncthreads();
        const u64 top = cur[63];
        u64 nc = k ? cur[k - 1] : 0;
#pragma unroll
        for (int q = 0; q < NTAPS; ++q)
            if (k == tap(q)) nc -= top;
        __syncthreads();
        c = nc;
    }
}

// Anti-diagonal sums of a 64x64 matrix (row j, column l -> coefficient j + l), reduced.
// 256 threads: the matrix is staged in LDS with coalesced loads; thread (q, k) sums the
// rows 16q .. 16q+15 of diagonal k and 64 + k; the four partial sums are then combined.
__device__ u64 fold_block(const u64* C, u64* tile /* 4096 */, u64* part /* 2*256 */, u64* sh, int t) {
#pragma unroll
    for (int i = 0; i < 16; ++i) tile[i * 256 + t] = C[i * 256 + t];
    __syncthreads();
    const int k = t & 63, q = t >> 6;
    u64 lo = 0, hi = 0;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const int j = 16 * q + jj;
        if (j <= k) lo += tile[j * 64 + (k - j)];
        else hi += tile[j * 64 + (k + 64 - j)];
    }
    part[t] = lo;
    part[256 + t] = hi;
    __syncthreads();
    u64 v = 0;
    if (t < 64) {
        lo = part[t] + part[64 + t] + part[128 + t] + part[192 + t];
        hi = part[256 + t] + part[320 + t] + part[384 + t] + part[448 + t];
    }
    // reduce_lane synchronises the block; all threads take part
    if (t < 64) sh[t] = hi;
    __syncthreads();
    if (t < 64) {
        v = lo;
#pragma unroll
        for (int qq = 0; qq < NTAPS; ++qq) {
            const int j = t - tap(qq);
            if (j >= 0) v -= sh[j];
        }
#pragma unroll
        for (int qq = 0; qq < NTAPS; ++qq) {
            const int p = t - tap(qq);
            if (p >= 0 && p <= 2) {
                u64 ov = 0;
#pragma unroll
                for (int r = 0; r < NTAPS; ++r) {
                    const int j = 64 + p - tap(r);
                    if (j >= 0 && j <= 62) ov -= sh[j];
                }
                v -= ov;
            }
        }
    }
    __syncthreads();
    return v;
}

// one-wave variant for the small ring products below
__device__ u64 fold_lane(const u64* C, u64* sh, int k) {
    u64 lo = 0, hi = 0;
    for (int j = 0; j <= k; ++j) lo += C[j * 64 + (k - j)];
    for (int j = k + 1; j < 64; ++j) hi += C[j * 64 + (k + 64 - j)];
    return reduce_lane(lo, hi, sh, k);
}

// out[i] = sum over l < nsum of C[l words + i], i < words (one word per thread)
__global__ void k_sum_blocks(const u64* C, int nsum, int64_t words, u64* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= words) return;
    u64 v0 = 0, v1 = 0, v2 = 0, v3 = 0;
    int l = 0;
    for (; l + 4 <= nsum; l += 4) {
        v0 += C[(int64_t)l * words + i];
        v1 += C[(int64_t)(l + 1) * words + i];
        v2 += C[(int64_t)(l + 2) * words + i];
        v3 += C[(int64_t)(l + 3) * words + i];
    }
    for (; l < nsum; ++l) v0 += C[(int64_t)l * words + i];
    out[i] = v0 + v1 + v2 + v3;
}

__global__ void k_fold_plain(const u64* C, u64* out) {
    __shared__ u64 tile[4096];
    __shared__ u64 part[512];
    __shared__ u64 sh[64];
    const int t = threadIdx.x;
    const u64 v = fold_block(C + (int64_t)blockIdx.x * 4096, tile, part, sh, t);
    if (t < 64) out[blockIdx.x * 64 + t] = v;
}

__global__ void k_polyevl_finish(PolyEvlArgs a) {
    __shared__ u64 tile[4096];
    __shared__ u64 part[512];
    __shared__ u64 sh[64];
    __shared__ int nz;
    const int t = threadIdx.x;
    if (t == 0) nz = 0;
    u64 s0, s1, s2;
    if (a.prefolded) {
        s0 = t < 64 ? a.C[t] : 0;
        s1 = t < 64 ? a.C[64 + t] : 0;
        s2 = t < 64 ? a.C[128 + t] : 0;
    } else {
        s0 = fold_block(a.C, tile, part, sh, t);             // sum R_a R_b            (P0)
        s1 = fold_block(a.C + 4096, tile, part, sh, t);      // sum m_a r1_b + m_b r1_a (P1)
        s2 = fold_block(a.C + 8192, tile, part, sh, t);      // sum m_a (m_b - r2_b) - r2_a m_b (P2)
    }
    u64 (*rows)[64] = (u64(*)[64])part;                       // part is free again here
    __syncthreads();
    prg_rows3(a.k.k01, make_tag(a.op, a.pr, 1, a.sub), a.k.k02, make_tag(a.op, a.pr, 2, a.sub), a.k.k01,
              make_tag(a.op, a.pg, 1, a.sub), rows);
    if (t < 64) {
        const int k = t;
        const u64 rc1 = rows[0][k], rc2 = rows[1][k], g1 = rows[2][k];
        u64 g2 = s0 + rc1 + rc2 - g1;                     // P0 -> P2
        if (k == a.inj_g2) g2 += a.e_g2;
        u64 m1 = g1 - s1;                                 // P1 -> P2
        if (k == a.inj_m1) m1 += a.e_m1;
        const u64 m2 = s2 + g2;                           // P2 -> P1
        const u64 m = m1 + m2;
        a.out[k] = m;
        a.out[64 + k] = rc1;
        a.out[128 + k] = rc2;
        if (a.log_m1) {
            a.log_m1[k] = m1;
            a.log_m2[k] = m2;
            a.log_g2[k] = g2;
        }
        if (a.reveal) {
            const u64 v = m - rc1 - rc2;
            a.reveal[k] = v;
            if (v) atomicOr(&nz, 1);
        }
    }
    __syncthreads();
    if (t == 0 && a.reveal && nz) atomicOr(a.nonzero_flag, 1);
}

// x * v for lane k: shift up by one coefficient and reduce x^64.
__device__ __forceinline__ u64 xmul_coeff(const u64* v, int k) {
    u64 r = k ? v[k - 1] : 0;
#pragma unroll
    for (int q = 0; q < NTAPS; ++q)
        if (k == tap(q)) r -= v[63];
    return r;
}

// One pass over the pairs of every plane c: D = f(1) - f(0) and F = f(0) + x D, the line
// through (0, f(0)) and (1, f(1)) at the node x (block: one (plane, pair); lanes =
// coefficients).
__global__ void k_at_x_diff(const u64* XY, int64_t n, u64* F, u64* D) {
    const int k = threadIdx.x;
    const int64_t i = blockIdx.x;
    const int c = blockIdx.y;
    const u64* f0 = XY + ((int64_t)c * n + 2 * i) * 64;
    const u64* f1 = f0 + 64;
    __shared__ u64 dsh[64];
    const u64 a = f0[k], d = f1[k] - a;
    dsh[k] = d;
    __syncthreads();
    const int64_t o = ((int64_t)c * (n / 2) + i) * 64 + k;
    D[o] = d;
    F[o] = a + xmul_coeff(dsh, k);
}

// The line through (0, f(0)) and (1, f(1)) at the node x for every pair of every plane c:
// F = f(0) + x (f(1) - f(0)); one wave per (plane, pair), four per block, lanes =
// coefficients, x (.) as a shift across the lanes with x^64 = -(x^4 + x^3 + x + 1).
__global__ __launch_bounds__(256) void k_at_x(const u64* XY, int64_t n, int64_t items, u64* F) {
    const int k = threadIdx.x & 63;
    const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= items) return;
    const int64_t half = n / 2;
    const int64_t c = item / half, i = item - c * half;
    const u64* f0 = XY + (c * n + 2 * i) * 64;
    const u64 a = f0[k], d = f0[64 + k] - a;
    const u64 top = __shfl(d, 63, 64);
    u64 xd = __shfl_up(d, 1, 64);
    if (k == 0) xd = 0;
#pragma unroll
    for (int q = 0; q < NTAPS; ++q)
        if (k == tap(q)) xd -= top;
    F[item * 64 + k] = a + xd;
}

// [Mat(1 - z); Mat(z)] (128 x 64) from Mat(z): the fold f(z) = f(0) (1 - z) + f(1) z of a
// stored pair (f(0), f(1)) is the pair's 128 words times this matrix.
__global__ void k_mat_pair(const u64* Wz, u64* out) {
    const int j = blockIdx.x, k = threadIdx.x;
    const u64 w = Wz[j * 64 + k];
    out[j * 64 + k] = (j == k ? 1 : 0) - w;
    out[(64 + j) * 64 + k] = w;
}

// Ring product of per-wave operands: wave w multiplies a[w] by b[w] (64 lanes = coefficients).
// Every thread of the block calls it (it synchronises the block).
__device__ u64 gr_mul_waves(const u64* a, const u64* b, u64* sh, int k) {
    u64 lo = 0, hi = 0;
    for (int i = 0; i < 64; ++i) {
        const u64 p = a[i] * b[(k - i) & 63];
        if (i <= k) lo += p; else hi += p;
    }
    return reduce_lane(lo, hi, sh, k);
}

__global__ void k_round_finish(RoundArgs a) {
    // 256 threads = 4 waves; wave w works on its own operands in LDS
    __shared__ u64 sh[4][64];
    __shared__ u64 opa[4][64], opb[4][64], res[4][64];
    __shared__ u64 zeta[64], zm1[64], zmx[64], L[3][64], hh[3][3][64];
    const int t = threadIdx.x, w = t >> 6, k = t & 63;
    prg_rows3(a.k.k12, make_tag(a.op, P_VER_ZETA, 0, a.sub), a.k.k01, make_tag(a.op, P_VER_ZETA, 1, a.sub), a.k.k02,
              make_tag(a.op, P_VER_ZETA, 2, a.sub), res);
    if (w == 0) {
        const u64 m = res[0][k], r1 = res[1][k], r2 = res[2][k];
        const u64 z = m - r1 - r2;                   // revealed point
        zeta[k] = z;
        zm1[k] = z - (k == 0 ? 1 : 0);               // zeta - 1
        zmx[k] = z - (k == 1 ? 1 : 0);               // zeta - x
        a.zeta_out[k] = z;
        if (a.log_zeta) a.log_zeta[k] = z;
    } else {
        const int c = w - 1;
        hh[0][c][k] = a.h0[c * 64 + k];
        hh[2][c][k] = a.h2[c * 64 + k];
        hh[1][c][k] = a.z[c * 64 + k] - a.h0[c * 64 + k];    // h(1) = z - h(0)
    }
    __syncthreads();
    // Lagrange weights over the nodes {0, 1, x}: L0 = (z-1)(z-x)/x, L1 = z(z-x)/(1-x),
    // L2 = z(z-1)/(x(x-1)); waves 0..2 compute one each, wave 3 idles
    if (w < 3) {
        opa[w][k] = w == 0 ? zm1[k] : zeta[k];
        opb[w][k] = w == 2 ? zm1[k] : zmx[k];
    } else {
        opa[w][k] = 0;
        opb[w][k] = 0;
    }
    __syncthreads();
    u64 v = gr_mul_waves(opa[w], opb[w], sh[w], k);
    res[w][k] = v;
    __syncthreads();
    opa[w][k] = res[w][k];
    opb[w][k] = w < 3 ? a.inv[w * 64 + k] : 0;
    __syncthreads();
    v = gr_mul_waves(opa[w], opb[w], sh[w], k);
    if (w < 3) L[w][k] = v;
    __syncthreads();
    // z'_c = sum_i L_i h_i,c : 9 products, waves take (i, c) pairs in three passes
    u64 acc = 0;
    for (int pass = 0; pass < 3; ++pass) {
        const int c = pass;         // plane handled in this pass
        if (w < 3) {
            opa[w][k] = L[w][k];
            opb[w][k] = hh[w][c][k];
        }
        __syncthreads();
        v = gr_mul_waves(opa[w], opb[w], sh[w], k);
        res[w][k] = w < 3 ? v : 0;
        __syncthreads();
        if (w == 0) a.z[c * 64 + k] = res[0][k] + res[1][k] + res[2][k];
        __syncthreads();
    }
    (void)acc;
    if (a.mat_out && w == 0) {
        // row j + 1 = x * row j: shift the coefficients up by one and reduce x^64
        u64 c = zeta[k];
        for (int j = 0; j < 64; ++j) {
            a.mat_out[j * 64 + k] = c;
            const u64 top = __shfl(c, 63, 64);
            u64 nc = __shfl_up(c, 1, 64);
            if (k == 0) nc = 0;
#pragma unroll
            for (int q = 0; q < NTAPS; ++q)
                if (k == tap(q)) nc -= top;
            c = nc;
        }
    }
}

// Orders the LDS accesses of one wave around it (a wave's LDS operations complete in order;
// this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// reduce_lane within one wave (sh: 64 words of LDS of the wave's own)
__device__ u64 reduce_wave(u64 lo, u64 hi, u64* sh, int k) {
    sh[k] = hi;
    wave_sync();
    u64 v = lo;
#pragma unroll
    for (int q = 0; q < NTAPS; ++q) {
        const int j = k - tap(q);
        if (j >= 0) v -= sh[j];
    }
#pragma unroll
    for (int q = 0; q < NTAPS; ++q) {
        const int p = k - tap(q);
        if (p >= 0 && p <= 2) {
            u64 ov = 0;
#pragma unroll
            for (int r = 0; r < NTAPS; ++r) {
                const int j = 64 + p - tap(r);
                if (j >= 0 && j <= 62) ov -= sh[j];
            }
            v -= ov;
        }
    }
    wave_sync();
    return v;
}

__device__ __forceinline__ u64 readlane64(u64 v, int i) {
    const u32 lo = __builtin_amdgcn_readlane((int)(u32)v, i), hi = __builtin_amdgcn_readlane((int)(u32)(v >> 32), i);
    return (u64)lo | ((u64)hi << 32);
}

// Coefficient k of a * b in GR(2^64, 64) within one wave: av is lane k's coefficient of a,
// b is in LDS written by this wave.  a_i is read across the lanes (uniform), b_(k-i) from LDS.
__device__ u64 gr_mul_wave(u64 av, const u64* b, u64* sh, int k) {
    wave_sync();
    u64 lo = 0, hi = 0;
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        const u64 p = readlane64(av, i) * b[(k - i) & 63];
        if (i <= k) lo += p; else hi += p;
    }
    return reduce_wave(lo, hi, sh, k);
}

// Coefficient k of a0 b0 + a1 b1 + a2 b2 within one wave (as gr_mul_wave, one reduction).
__device__ u64 gr_mul3_wave(u64 a0, const u64* b0, u64 a1, const u64* b1, u64 a2, const u64* b2, u64* sh, int k) {
    wave_sync();
    u64 lo = 0, hi = 0;
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        const int j = (k - i) & 63;
        const u64 p = readlane64(a0, i) * b0[j] + readlane64(a1, i) * b1[j] + readlane64(a2, i) * b2[j];
        if (i <= k) lo += p; else hi += p;
    }
    return reduce_wave(lo, hi, sh, k);
}

// The keystream rows of rounds k0 .. k0 + gridDim.x - 1 of a verification instance (block b =
// round k0 + b; nine rows of 64 words each): 0..2 h(0)'s [r]_1, [r]_2 and [Gamma]_1 masks of
// Pi_PolyEvl, 3..5 the same for h(x), 6..8 the three shares of the revealed point.  Each row
// is one party's local keystream, drawn ahead of the round.
__global__ void k_round_rows(Keys kk, u32 op, u32 inst, int k0, u64* out) {
    const int t = threadIdx.x;
    if (t >= 72) return;
    const u32 sub = (inst << 8) | (u32)(k0 + blockIdx.x);
    const int row = t >> 3, b = t & 7;
    const int grp = row / 3, comp = row % 3;
    Key key;
    u32 pur;
    if (grp < 2) {
        key = comp == 1 ? kk.k02 : kk.k01;
        pur = comp == 2 ? (grp ? P_VER_H2_GAMMA : P_VER_H0_GAMMA) : (grp ? P_VER_H2_R : P_VER_H0_R);
    } else {
        key = comp == 0 ? kk.k12 : comp == 1 ? kk.k01 : kk.k02;
        pur = P_VER_ZETA;
    }
    const u32 cc = grp < 2 ? (comp == 2 ? 1u : (u32)comp + 1) : (u32)comp;
    u64 wv[8];
    prg_block8(key, make_tag(op, pur, cc, sub), (u64)b, wv);
    u64* o = out + (int64_t)blockIdx.x * 9 * 64 + row * 64 + 8 * b;
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = wv[q];
}

// Quarter q (coefficients i of a in [16 q, 16 q + 16)) of the anti-diagonal sums of
// a (x) b at lane k: lo takes the terms with i <= k (coefficient k), hi the others
// (coefficient 64 + k, for reduce_wave); a and b in LDS, a read as a broadcast.
__device__ __forceinline__ void gr_acc_quarter(const u64* a, const u64* b, int k, int q, u64& lo, u64& hi) {
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) {
        const int i = 16 * q + ii;
        const u64 p = a[i] * b[(k - i) & 63];
        if (i <= k) lo += p;
        else hi += p;
    }
}

// The middle of a Pi_Reduce round in one workgroup, from the partial anti-diagonal sums of
// the parties' h(0) and h(x) products (hpair_party): their sum and reduction modulo the
// ring's modulus, both Pi_PolyEvl exchanges (P0's [Gamma]_2, P1's and P2's m shares), the
// revealed point zeta, the Lagrange step of the claim z, and the digit tiles of the
// multiplication matrix of zeta for the fold on the matrix cores.  The keystream rows come
// drawn ahead (k_round_rows).  Each of the ring products (the three Lagrange weights in
// two products each, then the three planes of the new claim) is split over four waves by
// quarters of its first factor's coefficients, twelve waves at a time, and summed and
// reduced by one wave; a thirteenth wave builds the point's matrix and its tiles meanwhile.
constexpr int RM_THREADS = 13 * 64;
__global__ __launch_bounds__(RM_THREADS) void k_round_mid(RoundMidArgs a) {
    __shared__ u64 rows[9][64];
    __shared__ u64 raw[3][256];                       // [party][point][lo 64 | hi 64]
    __shared__ u64 ssum[6][64];                       // [point * 3 + party]
    __shared__ u64 sh[4][64];
    __shared__ u64 zeta[64], zm1[64], zmx[64], inv[3][64], V[3][64], L[3][64], hh[3][3][64];
    __shared__ u64 qpart[3][4][128];                  // [product][quarter][lo 64 | hi 64]
    __shared__ u64 mat[64 * 64];
    const int t = threadIdx.x, w = t >> 6, k = t & 63;
    for (int i = t; i < 9 * 64; i += RM_THREADS) rows[i >> 6][i & 63] = a.rows[i];
    if (t < 192) inv[t >> 6][k] = a.inv[t];
    // the workgroups' partials, summed per party (units: P0 0; P1 1, 2; P2 3, 4): thread t =
    // (point t >> 7, word t & 127)
    if (t < 256) {
        for (int p = 0; p < 3; ++p) {
            u64 s0 = 0, s1 = 0, s2 = 0, s3 = 0;
            const int u0 = p == 0 ? 0 : 2 * p - 1, u1 = p == 0 ? 1 : 2 * p + 1;
            for (int u = u0; u < u1 && u < a.nunits; ++u) {
                const u64* src = a.part + (int64_t)u * 256 + t;
                const int64_t st = (int64_t)a.nunits * 256;
                int g = 0;
                for (; g + 4 <= a.groups; g += 4) {
                    s0 += src[g * st];
                    s1 += src[(g + 1) * st];
                    s2 += src[(g + 2) * st];
                    s3 += src[(g + 3) * st];
                }
                for (; g < a.groups; ++g) s0 += src[g * st];
            }
            raw[p][t] = s0 + s1 + s2 + s3;
        }
    }
    __syncthreads();
    // reduced sums: wave w takes (point, party) w and w + 4
    if (w < 4)
        for (int pp = w; pp < 6; pp += 4) {
            const int pt = pp / 3, party = pp % 3;
            ssum[pp][k] = reduce_wave(raw[party][pt * 128 + k], raw[party][pt * 128 + 64 + k], sh[w], k);
        }
    __syncthreads();
    if (w < 2) {
        // wave pt: the Pi_PolyEvl exchange of h(0) (pt 0) or h(x) (pt 1); its share (m, r1, r2)
        // goes to hh[0] (h(0)) or hh[2] (h(x))
        const int pt = w;
        const u64 rc1 = rows[3 * pt][k], rc2 = rows[3 * pt + 1][k], g1 = rows[3 * pt + 2][k];
        u64 g2 = ssum[3 * pt][k] + rc1 + rc2 - g1;            // P0 -> P2
        if (pt == 1 && k == a.inj_h2_g2) g2 += a.e_h2_g2;
        u64 m1 = g1 - ssum[3 * pt + 1][k];                     // P1 -> P2
        if (pt == 0 && k == a.inj_h0_m1) m1 += a.e_h0_m1;
        const u64 m2 = ssum[3 * pt + 2][k] + g2;               // P2 -> P1
        const int hi = pt ? 2 : 0;
        hh[hi][0][k] = m1 + m2;
        hh[hi][1][k] = rc1;
        hh[hi][2][k] = rc2;
        u64* l0 = pt ? a.log_h2[0] : a.log_h0[0];
        u64* l1 = pt ? a.log_h2[1] : a.log_h0[1];
        u64* l2 = pt ? a.log_h2[2] : a.log_h0[2];
        if (l0) {
            l0[k] = m1;
            l1[k] = m2;
            l2[k] = g2;
        }
    } else if (w == 2) {
        const u64 z = rows[6][k] - rows[7][k] - rows[8][k];   // revealed point
        zeta[k] = z;
        zm1[k] = z - (k == 0 ? 1 : 0);
        zmx[k] = z - (k == 1 ? 1 : 0);
        if (a.log_zeta) a.log_zeta[k] = z;
    }
    __syncthreads();
    // Lagrange weights over {0, 1, x}: L0 = (z-1)(z-x)/x, L1 = z(z-x)/(1-x),
    // L2 = z(z-1)/(x(x-1)); first v_p = (z-1)(z-x), z(z-x), z(z-1) on waves 4p .. 4p + 3
    if (w < 12) {
        const int p = w >> 2, q = w & 3;
        u64 lo = 0, hi = 0;
        gr_acc_quarter(p == 0 ? zm1 : zeta, p == 2 ? zm1 : zmx, k, q, lo, hi);
        qpart[p][q][k] = lo;
        qpart[p][q][64 + k] = hi;
    } else {
        // the multiplication matrix of zeta: row j = zeta x^j (shift up, reduce x^64)
        u64 cz = zeta[k];
        for (int j = 0; j < 64; ++j) {
            mat[j * 64 + k] = cz;
            const u64 top = __shfl(cz, 63, 64);
            u64 nc = __shfl_up(cz, 1, 64);
            if (k == 0) nc = 0;
#pragma unroll
            for (int q = 0; q < NTAPS; ++q)
                if (k == tap(q)) nc -= top;
            cz = nc;
        }
    }
    __syncthreads();
    if (w < 3) {
        hh[1][w][k] = a.z[w * 64 + k] - hh[0][w][k];          // h(1) = z - h(0), plane w
        const u64 lo = qpart[w][0][k] + qpart[w][1][k] + qpart[w][2][k] + qpart[w][3][k];
        const u64 hi = qpart[w][0][64 + k] + qpart[w][1][64 + k] + qpart[w][2][64 + k] + qpart[w][3][64 + k];
        V[w][k] = reduce_wave(lo, hi, sh[w], k);
    }
    __syncthreads();
    // L_p = v_p times the public inverse
    if (w < 12) {
        const int p = w >> 2, q = w & 3;
        u64 lo = 0, hi = 0;
        gr_acc_quarter(V[p], inv[p], k, q, lo, hi);
        qpart[p][q][k] = lo;
        qpart[p][q][64 + k] = hi;
    } else {
        // the matrix's digit tiles as the fold's B operand: tile row r = column r of the
        // matrix, k = its row index (k-block kb = rows 32 kb .. 32 kb + 31), k-octet oc
        for (int item = k; item < 512; item += 64) {
            const int r = item & 63, oc = (item >> 6) & 3, kb = item >> 8;
            u64 w8[8], q8[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) w8[i] = mat[(32 * kb + 8 * oc + i) * 64 + r];
            limb::to_digits(w8, q8);
            int8_t* base = a.ztiles + kb * limb::TILE_BYTES;
#pragma unroll
            for (int d = 0; d < 8; ++d) *(u64*)(base + limb::toff(d, r, oc)) = q8[d];
        }
    }
    __syncthreads();
    if (w < 3) {
        const u64 lo = qpart[w][0][k] + qpart[w][1][k] + qpart[w][2][k] + qpart[w][3][k];
        const u64 hi = qpart[w][0][64 + k] + qpart[w][1][64 + k] + qpart[w][2][64 + k] + qpart[w][3][64 + k];
        L[w][k] = reduce_wave(lo, hi, sh[w], k);
    }
    __syncthreads();
    // z'_c = sum_i L_i h_i,c: plane c on waves 4c .. 4c + 3
    if (w < 12) {
        const int c = w >> 2, q = w & 3;
        u64 lo = 0, hi = 0;
#pragma unroll
        for (int i3 = 0; i3 < 3; ++i3) gr_acc_quarter(L[i3], hh[i3][c], k, q, lo, hi);
        qpart[c][q][k] = lo;
        qpart[c][q][64 + k] = hi;
    }
    __syncthreads();
    if (w < 3) {
        const u64 lo = qpart[w][0][k] + qpart[w][1][k] + qpart[w][2][k] + qpart[w][3][k];
        const u64 hi = qpart[w][0][64 + k] + qpart[w][1][64 + k] + qpart[w][2][64 + k] + qpart[w][3][64 + k];
        a.z[w * 64 + k] = reduce_wave(lo, hi, sh[w], k);
    }
}

__global__ void k_xp_epilogue(int64_t n, Keys k, u32 op, u32 sub, const u64* C0, const u64* C1,
                              const u64* C2, u64* XPm, u64* XP1, u64* XP2) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w0 = b * 8;
    if (w0 >= n * 64) return;
    u64 r1[8], r2[8], g1[8];
    prg_block8(k.k01, make_tag(op, P_VER_XP_R, 1, sub), b, r1);
    prg_block8(k.k02, make_tag(op, P_VER_XP_R, 2, sub), b, r2);
    prg_block8(k.k01, make_tag(op, P_VER_XP_GAMMA, 1, sub), b, g1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t w = w0 + q;
        const u64 g2 = C0[w] + r1[q] + r2[q] - g1[q];   // P0: R_x R_alpha + r; sends [Gamma]_2
        const u64 m1 = g1[q] - C1[w];                    // P1
        const u64 m2 = C2[w] + g2;                       // P2
        XPm[w] = m1 + m2;
        XP1[w] = r1[q];
        XP2[w] = r2[q];
    }
}

__global__ void k_neg_elem(const u64* src, int64_t psi, u64* dst, int64_t pso) {
    const int k = threadIdx.x;
    for (int c = 0; c < 3; ++c) dst[c * pso + k] = 0 - src[c * psi + k];
}

__global__ void k_scale_rows(int64_t n, const u64* a0, const u64* a1, const u64* a2, const u64* P, u64* out,
                             int64_t ps) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * 64) return;
    const int64_t i = idx >> 6;
    const u64 p = P[idx];
    out[idx] = a0 ? a0[i] * p : 0;
    out[ps + idx] = a1 ? a1[i] * p : 0;
    out[2 * ps + idx] = a2 ? a2[i] * p : 0;
}

__global__ void k_lift_rows(int64_t n, const u64* a0, const u64* a1, const u64* a2, u64* out, int64_t ps) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * 64) return;
    const int64_t i = idx >> 6;
    const bool c0 = (idx & 63) == 0;
    out[idx] = (c0 && a0) ? a0[i] : 0;
    out[ps + idx] = (c0 && a1) ? a1[i] : 0;
    out[2 * ps + idx] = (c0 && a2) ? a2[i] : 0;
}

// element e = 128 q + 64 s + j of truncation lo + q (gate g = 2q + s):
//   x'_e = r^g (0, w_s(j) b1_j, 0),  y_e = (0, 0, -b2_j) lifted
__global__ void k_trunc_instance(int64_t T, int t, const u64* B1, const u64* B2, const u64* P, u64* x1,
                                 u64* y2) {
    const int k = threadIdx.x;
    const int64_t e = blockIdx.x;
    const int64_t q = e >> 7;
    const int s = (int)((e >> 6) & 1);
    const int j = (int)(e & 63);
    const u64 b1 = (B1[q] >> j) & 1, b2 = (B2[q] >> j) & 1;
    u64 w;
    if (s == 0) {
        w = j == 63 ? 0 : (u64)1 << (j + 1);            // 2^{j+1} (2^64 = 0)
    } else {
        u64 c = 0;
        if (j >= t && j < 63) c = (u64)1 << (j - t);
        if (j == 63) c = 0 - ((u64)1 << (63 - t));
        w = 2 * c;
    }
    const int64_t g = 2 * q + s;
    x1[e * 64 + k] = (w * b1) * P[g * 64 + k];
    y2[e * 64 + k] = k == 0 ? 0 - b2 : 0;
}

__global__ void k_trunc_w(int64_t lo, int64_t T, int t, const u64* B1, const u64* B2, const u64* rxm,
                          const u64* rx1, const u64* rx2, const u64* rzm, const u64* rz1, const u64* rz2,
                          u64* w3) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= T) return;
    const int64_t p = lo + q;
    const u64 b1 = B1[q], b2 = B2[q];
    // gate outputs <w> = <r> - (linear part): w_x = (m, r1 + B1, r2 + B2), w_z with ash(B, t)
    w3[2 * q] = rxm[p];
    w3[2 * T + 2 * q] = rx1[p] + b1;
    w3[4 * T + 2 * q] = rx2[p] + b2;
    w3[2 * q + 1] = rzm[p];
    w3[2 * T + 2 * q + 1] = rz1[p] + ash(b1, t);
    w3[4 * T + 2 * q + 1] = rz2[p] + ash(b2, t);
}

__global__ void k_set_one(u64* p) { p[threadIdx.x] = threadIdx.x == 0 ? 1 : 0; }

// weight of bit j in gate s of a truncation: 2^{j+1} (x-gate), 2 c_j (z-gate), with
// c_j = 2^{j-t} for t <= j < 63, c_63 = -2^{63-t}, 0 below t
__device__ __forceinline__ u64 gate_weight(int s, int j, int t) {
    if (s == 0) return j == 63 ? 0 : (u64)1 << (j + 1);
    u64 c = 0;
    if (j >= t && j < 63) c = (u64)1 << (j - t);
    if (j == 63) c = 0 - ((u64)1 << (63 - t));
    return 2 * c;
}

// The gates of the truncation chunk, written out per gate g = 2q + s (q the truncation in the
// chunk, s = 0 the x-gate, 1 the z-gate): 64 x values alpha_k = w_s(k) bit_k(B1_q) and 64 y
// values gamma_k = -bit_k(B2_q).  After j symbolic folds, element i of a gate is
// sum_S alpha_{i,S} zeta^S over the subsets S of the j folded points, with
//     alpha_{i,S} = sum_{m subset of S} (-1)^{|S \ m|} alpha_{i 2^j + m}
// (each fold keeps f(0) as the coefficient of a new point's absence and f(1) - f(0) as that
// of its presence; zeta itself does not enter).  sym_stage writes these level-j values for
// `ng` gates into LDS rows of SYM_ROW words: the gate values, then j in-place
// difference passes over the low j bits of the element index.
constexpr int SYM_GB = 16, SYM_ROW = 129;
// first round whose power-weight rows are point values (measured: fewer products pay off
// from four pairs per gate down; below, the direct coefficients are faster)
constexpr int SYM_POINTS = 3;
// y-side coefficients are differences of 0 / -1 values over at most j <= 5 bits
// (|value| <= 2^(j-1)), held as 16-bit integers; a read converts them to Z_{2^64} by sign
// extension.
__device__ void sym_stage(int j, int64_t g0, int ng, int t, const u64* B1, const u64* B2, u64* sa, short* sg) {
    for (int e = threadIdx.x; e < ng * 64; e += blockDim.x) {
        const int gg = e >> 6, k = e & 63;
        const int64_t g = g0 + gg;
        const int64_t q = g >> 1;
        sa[gg * SYM_ROW + k] = gate_weight((int)(g & 1), k, t) * ((B1[q] >> k) & 1);
        sg[gg * SYM_ROW + k] = (short)-(int)((B2[q] >> k) & 1);
    }
    for (int b = 0; b < j; ++b) {
        __syncthreads();
        // every word whose index has bit b set subtracts its partner without it
        for (int e = threadIdx.x; e < ng * 32; e += blockDim.x) {
            const int gg = e >> 5, h = e & 31;
            const int k = ((h >> b) << (b + 1)) | (1 << b) | (h & ((1 << b) - 1));
            sa[gg * SYM_ROW + k] -= sa[gg * SYM_ROW + (k ^ (1 << b))];
            sg[gg * SYM_ROW + k] = (short)(sg[gg * SYM_ROW + k] - sg[gg * SYM_ROW + (k ^ (1 << b))]);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int pow3(int j) {
    int r = 1;
    for (int i = 0; i < j; ++i) r *= 3;
    return r;
}

// Monomial order for the threads of k_sym_coeffs: u < 3^j by the number of its base-3
// digits equal to 1 (the work per (gate, u) is 2 to that power), so the lanes of a wave
// take monomials of equal cost.
struct SymOrder {
    unsigned short u[243];
};

// Power-weight rows of round j: for every gate, sum_i f_i(x) g_i(x) over its pairs i, as a
// polynomial of degree <= 2 in x and in each of the j revealed points zeta_b; row
// (u + 3^j e) of cx with row stride ld (columns G .. ld-1 are written as 0), u = sum_b u_b 3^b.
// One thread handles one (gate, u), with f = a0 + x (a1 - a0) and g = b0 + x (b1 - b0):
//  * rounds j < SYM_POINTS: the coefficients of x^e zeta^u.  The subset pairs (S, T) with
//    S_b + T_b = u_b are: digit 0 -> (0,0), 2 -> (1,1), 1 -> (0,1) or (1,0); the three
//    x-coefficients are a0 b0, a1 b1 - a0 b0 - da db and da db.
//  * rounds j >= SYM_POINTS: the values at the point (x, zeta) in {0, 1, inf}^(1 + j) given
//    by the digits (0 -> 0, 1 -> 1, 2 -> inf, the leading coefficient in that variable).  A
//    multilinear factor evaluates there as the sum of its coefficients over the subsets S
//    with S_b = 0 for digit 0, S_b = 1 for digit 2 and either for digit 1, and the x-points
//    take a0 b0, a1 b1 and (a1 - a0)(b1 - b0): three products per pair instead of three per
//    pair and subset split (k_interp3 turns the power-weighted sums of the values back into
//    coefficients).
// The round j is a template parameter (pair count and LDS strides constant).
template <int J>
__global__ __launch_bounds__(256) void k_sym_coeffs(int64_t G, int64_t ld, int t, const u64* B1, const u64* B2,
                                                     u64* cx, SymOrder ord) {
    constexpr int j = J;
    __shared__ u64 sa[SYM_GB * SYM_ROW];
    __shared__ short sg[SYM_GB * SYM_ROW];
    const int64_t g0 = (int64_t)blockIdx.x * SYM_GB;
    const int ng = (int)max((int64_t)0, min((int64_t)SYM_GB, G - g0));
    sym_stage(j, g0, ng, t, B1, B2, sa, sg);
    constexpr int L = 1 << j;              // coefficients per element
    constexpr int NP = 32 >> j;            // pairs per gate
    const int nu = pow3(j);
    for (int item = threadIdx.x; item < SYM_GB * nu; item += blockDim.x) {
        const int gg = item % SYM_GB, u = ord.u[item / SYM_GB];
        const int64_t g = g0 + gg;
        if (g >= ld) continue;
        if (gg >= ng) {                    // padding columns
            cx[(int64_t)u * ld + g] = 0;
            cx[(int64_t)(u + nu) * ld + g] = 0;
            cx[(int64_t)(u + 2 * nu) * ld + g] = 0;
            continue;
        }
        const u64* A = sa + gg * SYM_ROW;
        const short* C = sg + gg * SYM_ROW;
        int base = 0, ones[8], nones = 0;
        int uu = u;
#pragma unroll
        for (int b = 0; b < j; ++b) {
            const int d = uu % 3;
            uu /= 3;
            if (d == 2) base |= 1 << b;
            if (d == 1) ones[nones++] = b;
        }
        u64 v0 = 0, v1 = 0, v2 = 0;
        if constexpr (j < SYM_POINTS) {
            u64 e0 = 0, e2 = 0, s1 = 0;
            for (int m = 0; m < (1 << nones); ++m) {
                int S = base, T = base;
                for (int q = 0; q < nones; ++q) {
                    if ((m >> q) & 1) S |= 1 << ones[q];
                    else T |= 1 << ones[q];
                }
                for (int i = 0; i < NP; ++i) {
                    const u64 a0 = A[(2 * i) * L + S], a1 = A[(2 * i + 1) * L + S];
                    const u64 b0 = (u64)(int64_t)C[(2 * i) * L + T], b1 = (u64)(int64_t)C[(2 * i + 1) * L + T];
                    e0 += a0 * b0;
                    s1 += a1 * b1;
                    e2 += (a1 - a0) * (b1 - b0);
                }
            }
            v0 = e0;
            v1 = s1 - e0 - e2;
            v2 = e2;
        } else {
            // every pair's four sums advance together per subset (4 NP independent LDS
            // reads in flight), then three products per pair
            u64 a0[NP], a1[NP], b0[NP], b1[NP];
#pragma unroll
            for (int i = 0; i < NP; ++i) a0[i] = a1[i] = b0[i] = b1[i] = 0;
            for (int m = 0; m < (1 << nones); ++m) {
                int S = base;
                for (int q = 0; q < nones; ++q)
                    if ((m >> q) & 1) S |= 1 << ones[q];
#pragma unroll
                for (int i = 0; i < NP; ++i) {
                    a0[i] += A[(2 * i) * L + S];
                    a1[i] += A[(2 * i + 1) * L + S];
                    b0[i] += (u64)(int64_t)C[(2 * i) * L + S];
                    b1[i] += (u64)(int64_t)C[(2 * i + 1) * L + S];
                }
            }
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                v0 += a0[i] * b0[i];
                v1 += a1[i] * b1[i];
                v2 += (a1[i] - a0[i]) * (b1[i] - b0[i]);
            }
        }
        cx[(int64_t)u * ld + g] = v0;
        cx[(int64_t)(u + nu) * ld + g] = v1;
        cx[(int64_t)(u + 2 * nu) * ld + g] = v2;
    }
}

// Round 0 of the power-weight rows, one thread per gate straight from the bit words: with
// alpha_k = w_s(k) bit_k(B1_q) and gamma_k = -bit_k(B2_q) (gate g = 2q + s), the x^0, x^1,
// x^2 coefficients of sum_i f_i(x) g_i(x) over the 32 pairs (2i, 2i + 1) are a0 b0,
// a1 b1 - a0 b0 - da db and da db summed (rows 0, 1, 2 of cx, row stride ld; columns
// G .. ld-1 written as 0).
__global__ void k_sym_round0(int64_t G, int64_t ld, int t, const u64* B1, const u64* B2, u64* cx) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ld) return;
    u64 e0 = 0, s1 = 0, e2 = 0;
    if (g < G) {
        const int s = (int)(g & 1);
        const u64 x = B1[g >> 1], y = B2[g >> 1];
#pragma unroll 8
        for (int i = 0; i < 32; ++i) {
            const int k = 2 * i;
            const u64 a0 = gate_weight(s, k, t) * ((x >> k) & 1), a1 = gate_weight(s, k + 1, t) * ((x >> (k + 1)) & 1);
            const u64 b0 = 0 - ((y >> k) & 1), b1 = 0 - ((y >> (k + 1)) & 1);
            e0 += a0 * b0;
            s1 += a1 * b1;
            e2 += (a1 - a0) * (b1 - b0);
        }
    }
    cx[g] = e0;
    cx[ld + g] = s1 - e0 - e2;
    cx[2 * ld + g] = e2;
}

// Symbolic round 1 likewise: level-1 element i of a gate has coefficients (v_2i, v_2i+1 - v_2i) in
// zeta_0 (v = alpha or gamma), its pairs are the elements (2p, 2p + 1), and monomial u of
// zeta_0 takes the subset splits (S, T) = (0, 0) for u = 0, (1, 1) for u = 2, (0, 1) and
// (1, 0) for u = 1.  Rows u + 3 e of cx.
__global__ void k_sym_round1(int64_t G, int64_t ld, int t, const u64* B1, const u64* B2, u64* cx) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ld) return;
    u64 e0[3] = {0, 0, 0}, s1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
    if (g < G) {
        const int s = (int)(g & 1);
        const u64 x = B1[g >> 1], y = B2[g >> 1];
        auto al = [&](int k) { return gate_weight(s, k, t) * ((x >> k) & 1); };
        auto ga = [&](int k) { return 0 - ((y >> k) & 1); };
#pragma unroll 4
        for (int p = 0; p < 16; ++p) {
            const int k = 4 * p;
            const u64 a0[2] = {al(k), al(k + 1) - al(k)}, a1[2] = {al(k + 2), al(k + 3) - al(k + 2)};
            const u64 b0[2] = {ga(k), ga(k + 1) - ga(k)}, b1[2] = {ga(k + 2), ga(k + 3) - ga(k + 2)};
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                // splits: (0,0) -> u 0, (1,1) -> u 2, (0,1) and (1,0) -> u 1
                const int S = sp == 1 || sp == 3 ? 1 : 0, T = sp == 1 || sp == 2 ? 1 : 0;
                const int u = sp == 0 ? 0 : sp == 1 ? 2 : 1;
                e0[u] += a0[S] * b0[T];
                s1[u] += a1[S] * b1[T];
                e2[u] += (a1[S] - a0[S]) * (b1[T] - b0[T]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        cx[u * ld + g] = e0[u];
        cx[(u + 3) * ld + g] = s1[u] - e0[u] - e2[u];
        cx[(u + 6) * ld + g] = e2[u];
    }
}

// Symbolic round 2 likewise: level-2 element i covers the values v_4i .. v_4i+3 and has the
// coefficients (v0, v1 - v0, v2 - v0, v3 - v2 - v1 + v0) in (zeta_0, zeta_1) (bit b of S for
// zeta_b); its pairs are the elements (2p, 2p + 1), and monomial u = d0 + 3 d1 takes, per
// digit, the splits (0, 0) for 0, (1, 1) for 2, (0, 1) and (1, 0) for 1.  Rows u + 9 e of cx.
__global__ __launch_bounds__(256) void k_sym_round2(int64_t G, int64_t ld, int t, const u64* B1, const u64* B2,
                                                     u64* cx) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ld) return;
    u64 e0[9], s1[9], e2[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) e0[u] = s1[u] = e2[u] = 0;
    if (g < G) {
        const int s = (int)(g & 1);
        const u64 x = B1[g >> 1], y = B2[g >> 1];
        auto al = [&](int k) { return gate_weight(s, k, t) * ((x >> k) & 1); };
        auto ga = [&](int k) { return 0 - ((y >> k) & 1); };
        auto mob = [](u64 v0, u64 v1, u64 v2, u64 v3, u64* c) {
            c[0] = v0;
            c[1] = v1 - v0;
            c[2] = v2 - v0;
            c[3] = v3 - v2 - v1 + v0;
        };
        for (int p = 0; p < 8; ++p) {
            const int k = 8 * p;
            u64 a0[4], a1[4], b0[4], b1[4];
            mob(al(k), al(k + 1), al(k + 2), al(k + 3), a0);
            mob(al(k + 4), al(k + 5), al(k + 6), al(k + 7), a1);
            mob(ga(k), ga(k + 1), ga(k + 2), ga(k + 3), b0);
            mob(ga(k + 4), ga(k + 5), ga(k + 6), ga(k + 7), b1);
#pragma unroll
            for (int u = 0; u < 9; ++u) {
                const int d0 = u % 3, d1 = u / 3;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    if ((d0 != 1 && (m & 1)) || (d1 != 1 && (m & 2))) continue;
                    const int S0 = d0 == 2 ? 1 : d0 == 1 ? (m & 1) : 0;
                    const int T0 = d0 == 2 ? 1 : d0 == 1 ? 1 - (m & 1) : 0;
                    const int S1 = d1 == 2 ? 1 : d1 == 1 ? (m >> 1) & 1 : 0;
                    const int T1 = d1 == 2 ? 1 : d1 == 1 ? 1 - ((m >> 1) & 1) : 0;
                    const int S = S0 | S1 << 1, T = T0 | T1 << 1;
                    e0[u] += a0[S] * b0[T];
                    s1[u] += a1[S] * b1[T];
                    e2[u] += (a1[S] - a0[S]) * (b1[T] - b0[T]);
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 9; ++u) {
        cx[u * ld + g] = e0[u];
        cx[(u + 9) * ld + g] = s1[u] - e0[u] - e2[u];
        cx[(u + 18) * ld + g] = e2[u];
    }
}

// Values at {0, 1, inf}^nvar -> coefficients of degree <= 2 per variable, in place: rows
// r = sum_b d_b 3^b (3^nvar <= 243 rows of 64 words); along each variable the triple
// (h(0), h(1), h(inf)) becomes (c0, c1, c2) = (h(0), h(1) - h(0) - h(inf), h(inf)).
__global__ __launch_bounds__(256) void k_interp3(u64* P, int nvar) {
    __shared__ u64 T[243 * 64];
    const int t = threadIdx.x, col = t & 63, grp = t >> 6;
    int nr = 1;
    for (int b = 0; b < nvar; ++b) nr *= 3;
    for (int i = t; i < nr * 64; i += 256) T[i] = P[i];
    __syncthreads();
    for (int b = 0, st = 1; b < nvar; ++b, st *= 3) {
        // triples: rows with digit b = 0, r = lo + 3 st hi (lo < st)
        for (int q = grp; q < nr / 3; q += 4) {
            const int r = q % st + 3 * st * (q / st);
            const u64 h0 = T[r * 64 + col], h1 = T[(r + st) * 64 + col], hi = T[(r + 2 * st) * 64 + col];
            T[(r + st) * 64 + col] = h1 - h0 - hi;
        }
        __syncthreads();
    }
    for (int i = t; i < nr * 64; i += 256) P[i] = T[i];
}

// The level-j values themselves (G x 64 words each, element-major as in LDS).
__global__ __launch_bounds__(256) void k_sym_level(int j, int64_t G, int t, const u64* B1, const u64* B2,
                                                    u64* alpha, u64* gamma) {
    __shared__ u64 sa[SYM_GB * SYM_ROW];
    __shared__ short sg[SYM_GB * SYM_ROW];
    const int64_t g0 = (int64_t)blockIdx.x * SYM_GB;
    const int ng = (int)min((int64_t)SYM_GB, G - g0);
    sym_stage(j, g0, ng, t, B1, B2, sa, sg);
    for (int e = threadIdx.x; e < ng * 64; e += blockDim.x) {
        const int gg = e >> 6, k = e & 63;
        alpha[(g0 + gg) * 64 + k] = sa[gg * SYM_ROW + k];
        gamma[(g0 + gg) * 64 + k] = (u64)(int64_t)sg[gg * SYM_ROW + k];
    }
}

__global__ void k_xshift_rows(const u64* in, int64_t n, int e, u64* out) {
    __shared__ u64 v[64];
    const int k = threadIdx.x;
    const int64_t i = blockIdx.x;
    v[k] = in[i * 64 + k];
    __syncthreads();
    u64 a = xmul_coeff(v, k);
    if (e == 2) {
        __syncthreads();
        v[k] = a;
        __syncthreads();
        a = xmul_coeff(v, k);
    }
    out[i * 64 + k] = a;
}

// Job blockIdx.z: rows 2 blockIdx.x and 2 blockIdx.x + 1 of plane blockIdx.y of its Q times
// its element P, in place (one pass over the coefficients for both rows).
__global__ void k_gr_scale_rows(const RowsJob* jobs, int64_t pstride) {
    __shared__ u64 a[64], b0[64], b1[64], sh[64];
    const RowsJob& j = jobs[blockIdx.z];
    const int k = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 2;
    if (i >= j.n) return;
    u64* q = j.Q + (int64_t)blockIdx.y * pstride;
    const bool two = i + 1 < j.n;
    a[k] = j.P[k];
    b0[k] = q[i * 64 + k];
    b1[k] = two ? q[(i + 1) * 64 + k] : 0;
    __syncthreads();
    u64 lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
    for (int m = 0; m < 64; ++m) {
        const u64 x = a[m];
        const int c = (k - m) & 63;
        const u64 p0 = x * b0[c], p1 = x * b1[c];
        if (m <= k) { lo0 += p0; lo1 += p1; } else { hi0 += p0; hi1 += p1; }
    }
    const u64 v0 = reduce_lane(lo0, hi0, sh, k);
    const u64 v1 = reduce_lane(lo1, hi1, sh, k);
    q[i * 64 + k] = v0;
    if (two) q[(i + 1) * 64 + k] = v1;
}

// One workgroup (one wave) per rpb consecutive rows (even), taken two at a time: rows 2j and
// 2j + 1 with the same multiplier share its loads in one pass over the coefficients.
__global__ void k_gr_mul_rows(const u64* P, const u64* Q, int64_t n, int64_t per, u64* out, int64_t pstride,
                              int rpb) {
    __shared__ u64 a[64], b0[64], b1[64], sh[64];
    const int k = threadIdx.x;
    const int64_t pl = (int64_t)blockIdx.y * pstride;              // plane blockIdx.y
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    for (int64_t i = r0; i < min(r0 + rpb, n); i += 2) {
        const bool two = i + 1 < n && (i + 1) / per == i / per;
        a[k] = P[(i / per) * 64 + k];
        b0[k] = Q[pl + i * 64 + k];
        if (two) b1[k] = Q[pl + (i + 1) * 64 + k];
        __syncthreads();
        if (two) {
            u64 lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
            for (int j = 0; j < 64; ++j) {
                const u64 x = a[j];
                const int c = (k - j) & 63;
                const u64 p0 = x * b0[c], p1 = x * b1[c];
                if (j <= k) { lo0 += p0; lo1 += p1; } else { hi0 += p0; hi1 += p1; }
            }
            const u64 v0 = reduce_lane(lo0, hi0, sh, k);
            const u64 v1 = reduce_lane(lo1, hi1, sh, k);
            out[pl + i * 64 + k] = v0;
            out[pl + (i + 1) * 64 + k] = v1;
        } else {
            out[pl + i * 64 + k] = gr_mul_lane(a, b0, sh, k);
            if (i + 1 < n) {                                       // row i + 1 alone
                a[k] = P[((i + 1) / per) * 64 + k];
                b0[k] = Q[pl + (i + 1) * 64 + k];
                __syncthreads();
                out[pl + (i + 1) * 64 + k] = gr_mul_lane(a, b0, sh, k);
            }
        }
        __syncthreads();
    }
}



// out[i * nq + j] = P[i] * Q[j] (one 64-lane group per product).
__global__ void k_gr_outer(const u64* P, const u64* Q, int64_t nq, u64* out) {
    __shared__ u64 a[64], b[64], sh[64];
    const int k = threadIdx.x;
    const int64_t i = blockIdx.x / nq, j = blockIdx.x % nq;
    a[k] = P[i * 64 + k];
    b[k] = Q[j * 64 + k];
    __syncthreads();
    out[(int64_t)blockIdx.x * 64 + k] = gr_mul_lane(a, b, sh, k);
}

// One doubling level of a power table: out[len + i] = out[i] * P for i < cnt (blocks
// 0 .. cnt-1) and, when Pn is given, Pn = P * P (block cnt).
// (the first level, len = 1, also writes out[0] = 1 and takes it as 1 without reading it)
__global__ void k_pow_level(u64* out, int64_t len, int64_t cnt, const u64* P, u64* Pn) {
    __shared__ u64 a[64], b[64], sh[64];
    const int k = threadIdx.x;
    const int64_t i = blockIdx.x;
    const bool first = len == 1;
    a[k] = P[k];
    b[k] = i < cnt ? (first ? (u64)(k == 0) : out[i * 64 + k]) : P[k];
    if (first && i == 0) out[k] = (u64)(k == 0);
    __syncthreads();
    const u64 v = gr_mul_lane(a, b, sh, k);
    if (i < cnt) out[(len + i) * 64 + k] = v;
    else Pn[k] = v;
}

// out[j] = r^{e0 + j step} from two power tables: lo[i] = r^i (i < L), hi[q] = r^{L q}.
// Two progressions in one launch: blocks < n give r^(e0a + step j) into outa, the rest
// r^(e0b + step j) into outb.
__global__ void k_pow_ap2(const u64* lo, const u64* hi, int64_t L, int64_t e0a, int64_t e0b, int64_t step,
                          int64_t n, u64* outa, u64* outb) {
    __shared__ u64 a[64], b[64], sh[64];
    const int k = threadIdx.x;
    const bool second = blockIdx.x >= n;
    const int64_t j = second ? blockIdx.x - n : blockIdx.x;
    const int64_t e = (second ? e0b : e0a) + j * step;
    a[k] = hi[(e / L) * 64 + k];
    b[k] = lo[(e % L) * 64 + k];
    __syncthreads();
    (second ? outb : outa)[j * 64 + k] = gr_mul_lane(a, b, sh, k);
}

__global__ void k_pow_ap(const u64* lo, const u64* hi, int64_t L, int64_t e0, int64_t step, u64* out) {
    __shared__ u64 a[64], b[64], sh[64];
    const int k = threadIdx.x;
    const int64_t e = e0 + (int64_t)blockIdx.x * step;
    a[k] = hi[(e / L) * 64 + k];
    b[k] = lo[(e % L) * 64 + k];
    __syncthreads();
    out[(int64_t)blockIdx.x * 64 + k] = gr_mul_lane(a, b, sh, k);
}

// ---------------------------------------------------------------------------
// Pi_InnerVerify of a few final pairs in one workgroup
// ---------------------------------------------------------------------------
// For n <= IV_MAX pairs (the default choice of R leaves at most 8) (x_i, y_i) (share planes; a null plane is 0) and the claim z: the
// random alpha, x'_i = Pi_Mult(x_i, alpha) (P0's [Gamma]_2, P1's and P2's m shares, as
// k_xp_epilogue), then Pi_PolyEvl of the n + 1 pairs (x'_i, y_i) and (-alpha, z) with the
// reveal of Delta (as k_polyevl_finish).  Every keystream row is drawn first; the ring
// products are spread over the four waves, each summing its share of a party's terms.
constexpr int IV_MAX = 8;

// lo/hi of sum over a list of ring products a_t b_t for lane k (a, b: 64-word vectors in LDS)
__device__ __forceinline__ void gr_acc(const u64* a, const u64* b, int k, u64& lo, u64& hi) {
#pragma unroll 8
    for (int i = 0; i < 64; ++i) {
        const u64 p = a[i] * b[(k - i) & 63];
        if (i <= k) lo += p; else hi += p;
    }
}

constexpr int IV_WAVES = 16;
__global__ __launch_bounds__(IV_WAVES * 64) void k_inner_verify_small(InnerVerifyArgs a) {
    const int n = a.n, n1 = n + 1;
    __shared__ u64 xa[IV_MAX + 1][5][64];    // x'_i (m, r1, r2, r1 + r2) and its [Gamma]_1; row n: -alpha
    __shared__ u64 yb[IV_MAX + 1][5][64];    // y_i (m, r1, r2, r1 + r2, m - r2); row n: z
    __shared__ u64 xs[IV_MAX][4][64];        // x_i: m, r1, r1 + r2, -r2
    __shared__ u64 cp[IV_MAX][3][64];        // the parties' sums of x_i alpha
    __shared__ u64 al[5][64];                // alpha: m, r1, r2, r1 + r2, m - r2
    __shared__ u64 red[IV_WAVES][3][128];
    __shared__ u64 dr[3][64];                // Delta's masks: r1, r2, [Gamma]_1
    __shared__ u64 sh[IV_WAVES][64];
    __shared__ int nz;
    const int t = threadIdx.x, w = t >> 6, k = t & 63;
    constexpr int NTH = IV_WAVES * 64;
    if (t == 0) nz = 0;
    // keystream: alpha (3 rows), Delta's masks (3 rows), and x'_i's masks (3 n rows), one
    // block of 8 words per thread
    for (int blk = t; blk < 8 * (6 + 3 * n); blk += NTH) {
        const int row = blk >> 3, b = blk & 7;
        u64 wv[8];
        if (row < 3) {
            const Key& key = row == 0 ? a.k.k12 : row == 1 ? a.k.k01 : a.k.k02;
            prg_block8(key, make_tag(a.op, P_VER_ALPHA, (u32)row, a.inst), (u64)b, wv);
#pragma unroll
            for (int q = 0; q < 8; ++q) al[row][8 * b + q] = wv[q];
        } else if (row < 6) {
            const int c = row - 3;      // r1 (k01, comp 1), r2 (k02, comp 2), [Gamma]_1 (k01, comp 1)
            const Key& key = c == 1 ? a.k.k02 : a.k.k01;
            prg_block8(key, make_tag(a.op, c == 2 ? P_VER_DELTA_GAMMA : P_VER_DELTA_R, c == 1 ? 2u : 1u, a.inst),
                       (u64)b, wv);
#pragma unroll
            for (int q = 0; q < 8; ++q) dr[c][8 * b + q] = wv[q];
        } else {
            // x'_i masks at words 64 i .. 64 i + 63: blocks 8 i .. 8 i + 7 of each stream
            const int r = row - 6, i = r / 3, c = r % 3;
            const Key& key = c == 1 ? a.k.k02 : a.k.k01;
            prg_block8(key, make_tag(a.op, c == 2 ? P_VER_XP_GAMMA : P_VER_XP_R, c == 1 ? 2u : 1u, a.inst),
                       (u64)(8 * i + b), wv);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (c == 0) xa[i][1][8 * b + q] = wv[q];       // r1 of x'_i
                else if (c == 1) xa[i][2][8 * b + q] = wv[q];  // r2 of x'_i
                else xa[i][4][8 * b + q] = wv[q];              // [Gamma]_1 of x'_i
            }
        }
    }
    // the pairs' y sides and the claim; the x_i
    for (int idx = t; idx < n1 * 64; idx += NTH) {
        const int i = idx >> 6, kk = idx & 63;
        u64 m, r1, r2;
        if (i < n) {
            m = a.p[3] ? a.p[3][(int64_t)i * 64 + kk] : 0;
            r1 = a.p[4] ? a.p[4][(int64_t)i * 64 + kk] : 0;
            r2 = a.p[5] ? a.p[5][(int64_t)i * 64 + kk] : 0;
            const u64 xm = a.p[0] ? a.p[0][(int64_t)i * 64 + kk] : 0;
            const u64 x1 = a.p[1] ? a.p[1][(int64_t)i * 64 + kk] : 0;
            const u64 x2 = a.p[2] ? a.p[2][(int64_t)i * 64 + kk] : 0;
            xs[i][0][kk] = xm;
            xs[i][1][kk] = x1;
            xs[i][2][kk] = x1 + x2;
            xs[i][3][kk] = 0 - x2;
        } else {
            m = a.z[kk];
            r1 = a.z[64 + kk];
            r2 = a.z[128 + kk];
        }
        yb[i][0][kk] = m;
        yb[i][1][kk] = r1;
        yb[i][2][kk] = r2;
        yb[i][3][kk] = r1 + r2;
        yb[i][4][kk] = m - r2;
    }
    __syncthreads();
    if (t < 64) {
        al[3][k] = al[1][k] + al[2][k];
        al[4][k] = al[0][k] - al[2][k];
        // alpha's revealed value is m - r1 - r2; its shares stay (m, r1, r2)
    }
    __syncthreads();
    // x'_i = Pi_Mult(x_i, alpha): one wave per (element i, party): P0 R_x R_alpha; P1
    // m_x r1_alpha + r1_x m_alpha; P2 m_x (m_alpha - r2_alpha) - r2_x m_alpha
    for (int u = w; u < 3 * n; u += IV_WAVES) {
        const int i = u / 3, p = u - 3 * i;
        u64 lo = 0, hi = 0;
        if (p == 0) {
            gr_acc(xs[i][2], al[3], k, lo, hi);
        } else if (p == 1) {
            gr_acc(xs[i][0], al[1], k, lo, hi);
            gr_acc(xs[i][1], al[0], k, lo, hi);
        } else {
            gr_acc(xs[i][0], al[4], k, lo, hi);
            gr_acc(xs[i][3], al[0], k, lo, hi);
        }
        cp[i][p][k] = reduce_wave(lo, hi, sh[w], k);
    }
    __syncthreads();
    if (w < n) {
        const int i = w;
        const u64 r1 = xa[i][1][k], r2 = xa[i][2][k], g1 = xa[i][4][k];
        const u64 g2 = cp[i][0][k] + r1 + r2 - g1;             // P0 -> P2
        const u64 m1 = g1 - cp[i][1][k];                       // P1
        const u64 m2 = cp[i][2][k] + g2;                       // P2
        xa[i][0][k] = m1 + m2;
        xa[i][3][k] = r1 + r2;
    } else if (w == IV_WAVES - 1) {
        // row n: -alpha
        xa[n][0][k] = 0 - al[0][k];
        xa[n][1][k] = 0 - al[1][k];
        xa[n][2][k] = 0 - al[2][k];
        xa[n][3][k] = 0 - al[3][k];
    }
    __syncthreads();
    // Pi_PolyEvl sums over the n + 1 pairs: terms (party 0: R R), (party 1: m r1, r1 m),
    // (party 2: m (m - r2), -r2 m); one wave per (pair, party), partial sums per wave
    u64 plo[3] = {0, 0, 0}, phi[3] = {0, 0, 0};
    for (int u = w; u < 3 * n1; u += IV_WAVES) {
        const int i = u / 3, p = u - 3 * i;
        if (p == 0) {
            gr_acc(xa[i][3], yb[i][3], k, plo[0], phi[0]);
        } else if (p == 1) {
            gr_acc(xa[i][0], yb[i][1], k, plo[1], phi[1]);
            gr_acc(xa[i][1], yb[i][0], k, plo[1], phi[1]);
        } else {
            gr_acc(xa[i][0], yb[i][4], k, plo[2], phi[2]);
            u64 l2 = 0, h2 = 0;
            gr_acc(xa[i][2], yb[i][0], k, l2, h2);
            plo[2] -= l2;
            phi[2] -= h2;
        }
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        red[w][p][k] = plo[p];
        red[w][p][64 + k] = phi[p];
    }
    __syncthreads();
    if (w < 3) {
        const int p = w;
        u64 lo = 0, hi = 0;
#pragma unroll
        for (int q = 0; q < IV_WAVES; ++q) {
            lo += red[q][p][k];
            hi += red[q][p][64 + k];
        }
        al[p][k] = reduce_wave(lo, hi, sh[w], k);              // the party sums s0, s1, s2
    }
    __syncthreads();
    if (w == 0) {
        const u64 rc1 = dr[0][k], rc2 = dr[1][k], g1 = dr[2][k];
        u64 g2 = al[0][k] + rc1 + rc2 - g1;                    // P0 -> P2
        u64 m1 = g1 - al[1][k];                                // P1 -> P2
        if (k == a.inj_m1) m1 += a.e_m1;
        const u64 m2 = al[2][k] + g2;                          // P2 -> P1
        const u64 v = m1 + m2 - rc1 - rc2;                     // Delta
        a.log_m1[k] = m1;
        a.log_m2[k] = m2;
        a.log_g2[k] = g2;
        a.reveal[k] = v;
        if (v) atomicOr(&nz, 1);
    }
    __syncthreads();
    if (t == 0 && nz) atomicOr(a.flag, 1);
}

// ---------------------------------------------------------------------------
// The x side of a same-padded, stride-1 convolution's compressed pairs from its input
// ---------------------------------------------------------------------------
// With output row m = b H W + oh W + ow and input position n = b H W + y W + x (OH = H,
// OW = W), column k = (kh, kw, c) of the lowered input holds h[n, c] at m = n - delta,
// delta = (kh - pad) W + (kw - pad), for the positions n whose output lies inside the image.
// So sum_m r^(o + m) X[m, k] = r^(o - delta) (S_c - E_(kh,kw),c) with S_c = sum_n r^n h[n, c]
// over every position and E the same sum over the positions left out: the top (kh - pad) or
// bottom (pad - kh) rows and the left or right columns (their union; the corner cells are in
// both bands once too many).  The band sums are over "sets": rows y < pad and y >= H - pad,
// columns x < pad and x >= W - pad, and the 4 pad^2 corner cells.

// Set s of the band sums: the number of positions and position j's (b, y, x).
__device__ __forceinline__ int64_t band_size(const ConvBandArgs& a, int s) {
    const int p2 = 2 * a.pad;
    return s < p2 ? (int64_t)a.B * a.W : s < 2 * p2 ? (int64_t)a.B * a.H : (int64_t)a.B;
}
__device__ __forceinline__ int64_t band_pos(const ConvBandArgs& a, int s, int64_t j) {
    const int p = a.pad, p2 = 2 * p;
    int64_t b, y, x;
    if (s < p2) {                                   // row band: y fixed
        y = s < p ? s : a.H - p2 + s;
        b = j / a.W;
        x = j - b * a.W;
    } else if (s < 2 * p2) {                        // column band: x fixed
        const int q = s - p2;
        x = q < p ? q : a.W - p2 + q;
        b = j / a.H;
        y = j - b * a.H;
    } else {                                        // corner cell (y index, x index)
        const int q = s - 2 * p2, qy = q / p2, qx = q % p2;
        y = qy < p ? qy : a.H - p2 + qy;
        x = qx < p ? qx : a.W - p2 + qx;
        b = j;
    }
    return (b * a.H + y) * a.W + x;
}

// Block (set s, plane, chunk and group of 64 channels): for its positions n (at most 64),
// sum_n h[n, c] r^n over the 64 coefficients for each channel c of the group ->
// part[chunk][plane][s][c][64].  The positions' power rows and channel values are staged in
// LDS first (all loads in flight at once), then thread (k = lane, wave w) sums channels w,
// w + 4, ... of the group.
// Block (set s, plane, z = chunk * cgroups + channel group of 64 channels) of nchunks chunks.
__device__ __forceinline__ void conv_bands_block(const ConvBandArgs& a, int s, int plane, int z, int nchunks) {
    __shared__ u64 Lt[64][64];                   // [position][coefficient]
    __shared__ u64 Ht[64][65];                   // [position][channel] (padded row)
    const int cgroups = (a.C + 63) / 64;
    const int chunk = z / cgroups, cg = z % cgroups;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t size = band_size(a, s);
    const int64_t per = (size + nchunks - 1) / nchunks;
    const int64_t j0 = (int64_t)chunk * per;
    const int np = (int)max<int64_t>(0, min<int64_t>(per, size - j0));   // per <= 64 (host)
    const u64* h = a.h[plane];
    u64* out = a.part + (((int64_t)chunk * 3 + plane) * a.nsets + s) * (int64_t)a.C * 64;
    __shared__ int64_t pos[64];
    if (t < 64) pos[t] = t < np ? band_pos(a, s, j0 + t) : 0;
    __syncthreads();
    for (int i = t; i < 64 * 64; i += 256) {
        const int jj = i >> 6, k = i & 63;
        Lt[jj][k] = jj < np ? a.lo[pos[jj] * 64 + k] : 0;
    }
    {
        const int c0 = cg * 64, cw = min(64, a.C - c0);
        __syncthreads();
        for (int i = t; i < 64 * 64; i += 256) {
            const int jj = i >> 6, cc = i & 63;
            Ht[jj][cc] = jj < np && cc < cw ? h[pos[jj] * a.C + c0 + cc] : 0;
        }
        __syncthreads();
        u64 acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0;
        for (int jj = 0; jj < np; ++jj) {
            const u64 rv = Lt[jj][lane];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] += Ht[jj][4 * q + w] * rv;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = 4 * q + w;
            if (c < cw) out[(int64_t)(c0 + c) * 64 + lane] = acc[q];
        }
    }
}

__global__ __launch_bounds__(256) void k_conv_bands(ConvBandArgs a) {
    conv_bands_block(a, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.z / ((a.C + 63) / 64));
}

// Job blockIdx.y / 3, plane blockIdx.y % 3; blocks past a job's sets or chunks return.
__global__ __launch_bounds__(256) void k_conv_bands_jobs(const BandJob* jobs) {
    const BandJob& j = jobs[blockIdx.y / 3];
    const int cgroups = (j.a.C + 63) / 64;
    if ((int)blockIdx.x >= j.a.nsets || (int)blockIdx.z >= j.chunks * cgroups) return;
    conv_bands_block(j.a, blockIdx.x, blockIdx.y % 3, blockIdx.z, j.chunks);
}

// Block b = kh KW + kw: r^(e0 - kh W - kw) from the two power tables (e0 = o + pad W + pad).
__global__ void k_pow_shifts(const u64* lo, const u64* hi, int64_t L, int64_t e0, int KW, int W, u64* out) {
    __shared__ u64 pa[64], pb[64], sh[64];
    const int k = threadIdx.x, b = blockIdx.x;
    const int64_t e = e0 - (int64_t)(b / KW) * W - (b % KW);
    pa[k] = hi[(e / L) * 64 + k];
    pb[k] = lo[(e % L) * 64 + k];
    __syncthreads();
    out[(int64_t)b * 64 + k] = gr_mul_lane(pa, pb, sh, k);
}

// Wave (k, plane): U[plane][k] = (S_c - E_(kh,kw),c) r^(o - delta), 0 for the zero columns
// k >= KH KW C.  Four waves per block.
__device__ __forceinline__ void conv_x_block(const ConvXArgs& a, int64_t bx, int plane) {
    __shared__ u64 vb[4][64], sh[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t kk = bx * 4 + w;
    if (kk >= a.K) return;                          // whole waves: no block barrier below
    u64* out = a.U + plane * a.ustride + kk * 64;
    if (kk >= (int64_t)a.KH * a.KW * a.C) {
        out[lane] = 0;
        return;
    }
    const int c = (int)(kk % a.C), kw = (int)((kk / a.C) % a.KW), kh = (int)(kk / ((int64_t)a.C * a.KW));
    const int p = a.pad, p2 = 2 * p, dy = kh - p, dx = kw - p;
    const int64_t cs = (int64_t)a.C * 64;
    const u64* E = a.E + (int64_t)plane * a.nsets * cs + (int64_t)c * 64 + lane;
    u64 v = a.S[(int64_t)plane * cs + (int64_t)c * 64 + lane];
    // row band: dy > 0 leaves out rows 0 .. dy-1 (sets 0 .. dy-1); dy < 0 rows H+dy .. H-1
    // (sets p2 + dy .. p2 - 1); likewise the columns (sets p2 + ...) and their corner cells
    const int r0 = dy > 0 ? 0 : p2 + dy, r1 = dy > 0 ? dy : p2;
    const int q0 = dx > 0 ? 0 : p2 + dx, q1 = dx > 0 ? dx : p2;
    if (dy)
        for (int r = r0; r < r1; ++r) v -= E[(int64_t)r * cs];
    if (dx)
        for (int q = q0; q < q1; ++q) v -= E[(int64_t)(p2 + q) * cs];
    if (dy && dx)
        for (int r = r0; r < r1; ++r)
            for (int q = q0; q < q1; ++q) v += E[(int64_t)(2 * p2 + r * p2 + q) * cs];
    vb[w][lane] = v;
    const u64 f = a.F[(int64_t)(kh * a.KW + kw) * 64 + lane];
    out[lane] = gr_mul_wave(f, vb[w], sh[w], lane);
}

__global__ __launch_bounds__(256) void k_conv_x(ConvXArgs a) { conv_x_block(a, blockIdx.x, blockIdx.y); }

// Job blockIdx.y / 3, plane blockIdx.y % 3 (conv_x_block returns per wave past the job's K).
__global__ __launch_bounds__(256) void k_conv_x_jobs(const ConvXArgs* jobs) {
    conv_x_block(jobs[blockIdx.y / 3], blockIdx.x, blockIdx.y % 3);
}

// One exponent per block: r^e = hi[e / L] lo[e mod L].
__global__ void k_pow_list(const u64* lo, const u64* hi, int64_t L, const PowJob* jobs) {
    __shared__ u64 pa[64], pb[64], sh[64];
    const int k = threadIdx.x;
    const PowJob j = jobs[blockIdx.x];
    pa[k] = hi[(j.e / L) * 64 + k];
    pb[k] = lo[(j.e % L) * 64 + k];
    __syncthreads();
    j.out[k] = gr_mul_lane(pa, pb, sh, k);
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------

void launch_fill(u64* out, int64_t n, Key k, Tag t, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(nblocks((n + 7) / 8 + 1, TPB)), dim3(TPB), 0, s, out, n, (int64_t)0, k, t);
}
void launch_fill_at(u64* out, int64_t n, int64_t start, Key k, Tag t, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(nblocks((n + 7) / 8 + 2, TPB)), dim3(TPB), 0, s, out, n, start, k, t);
}
void launch_encode(const double* x, int64_t n, int frac, u64* out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_encode, dim3(nblocks(n, TPB)), dim3(TPB), 0, s, x, n, (double)((u64)1 << frac), out);
}
void launch_decode(const u64* v, int64_t n, int frac, double* out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_decode, dim3(nblocks(n, TPB)), dim3(TPB), 0, s, v, n, (double)((u64)1 << frac), out);
}
void launch_share(const u64* x, int64_t n, Key k1, Tag t1, Key k2, Tag t2, u64* m, u64* r1, u64* r2,
                  hipStream_t s, const u32* op_off) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_share, dim3(nblocks((n + 7) / 8, TPB)), dim3(TPB), 0, s, x, n, k1, t1, k2, t2, m, r1, r2,
                       op_off);
}
void launch_trunc_pair(int64_t n, int t, const Keys& k, u32 op, Inj g2x, Inj m1z, u64* rxm, u64* rx1,
                       u64* rx2, u64* rzm, u64* rz1, u64* rz2, hipStream_t s, const u32* op_off) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_trunc_pair, dim3(nblocks((n + 7) / 8, TPB)), dim3(TPB), 0, s, n, t, k, op, g2x, m1z,
                       rxm, rx1, rx2, rzm, rz1, rz2, op_off);
}
void launch_inner_pre(int64_t n, const Keys& k, u32 op, const u64* pm, const u64* p1, const u64* p2,
                      u64* zr1, u64* zr2, u64* g1, hipStream_t s, const u32* op_off) {
    if (n <= 0) return;
    static_assert(TPB == 256, "k_inner_pre holds four waves' exchange buffers");
    hipLaunchKernelGGL(k_inner_pre, dim3(nblocks((n + 7) / 8, TPB)), dim3(TPB), 0, s, n, k, op, pm, p1, p2, zr1,
                       zr2, g1, op_off);
}
__global__ void k_set_word(u32* p, u32 v) { *p = v; }
void launch_set_word(u32* p, u32 v, hipStream_t s) { hipLaunchKernelGGL(k_set_word, dim3(1), dim3(1), 0, s, p, v); }
void launch_inner_post(int64_t n, const u64* c0, const u64* c1, const u64* c2, const u64* zr1,
                       const u64* zr2, const u64* g1, Inj g2inj, Inj m1inj, u64* zm, u64* msg_g2,
                       u64* msg_m1, u64* msg_m2, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_inner_post, dim3(nblocks(n, TPB)), dim3(TPB), 0, s, n, c0, c1, c2, zr1, zr2, g1, g2inj,
                       m1inj, zm, msg_g2, msg_m1, msg_m2);
}
void launch_trunc_shift(int64_t n, int t, const u64* zm, const u64* rzm, const u64* rz1, const u64* rz2,
                        u64* om, u64* o1, u64* o2, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_trunc_shift, dim3(nblocks(n, TPB)), dim3(TPB), 0, s, n, t, zm, rzm, rz1, rz2, om, o1, o2);
}
void launch_mult(int64_t n, const Keys& k, u32 op, const u64* am, const u64* a1, const u64* a2,
                 const u64* bm, const u64* b1, const u64* b2, Inj g2inj, u64* cm, u64* c1, u64* c2,
                 u64* msg_g2, u64* msg_m1, u64* msg_m2, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mult, dim3(nblocks((n + 7) / 8, TPB)), dim3(TPB), 0, s, n, k, op, am, a1, a2, bm, b1, b2,
                       g2inj, cm, c1, c2, msg_g2, msg_m1, msg_m2);
}
void launch_im2col(const u64* x, int B, int H, int W, int C, int KH, int KW, int pad, int64_t ld, u64* out,
                   hipStream_t s, int stride) {
    const int OH = (H + 2 * pad - KH) / stride + 1, OW = (W + 2 * pad - KW) / stride + 1;
    const int64_t total = (int64_t)B * OH * OW * ld;
    if (total <= 0) return;
    hipLaunchKernelGGL(k_im2col, dim3(nblocks(total, TPB)), dim3(TPB), 0, s, x, B, H, W, C, KH, KW, pad, stride, OH,
                       OW, ld, out);
}

void launch_im2col3(const u64* const x[3], int B, int H, int W, int C, int KH, int KW, int pad, int64_t ld,
                    u64* const out[3], hipStream_t s, int stride) {
    const int OH = (H + 2 * pad - KH) / stride + 1, OW = (W + 2 * pad - KW) / stride + 1;
    const int64_t K = (int64_t)KH * KW * C;
    const int64_t total = (int64_t)B * OH * OW * ld;
    if (total <= 0 || ld < K) return;
    bool aligned = true;
    for (int p = 0; p < 3; ++p) aligned = aligned && (((uintptr_t)x[p] | (uintptr_t)out[p]) & 15) == 0;
    if (total >= ((int64_t)1 << 31)) {       // beyond 32-bit word indices: one word per thread
        for (int p = 0; p < 3; ++p) launch_im2col(x[p], B, H, W, C, KH, KW, pad, ld, out[p], s, stride);
        return;
    }
    Im2colArgs a{};
    for (int p = 0; p < 3; ++p) {
        a.x[p] = x[p];
        a.out[p] = out[p];
    }
    a.H = H; a.W = W; a.C = C; a.KW = KW; a.OH = OH; a.OW = OW; a.pad = pad; a.stride = stride;
    a.K = (u32)K;
    a.ld = (u32)ld;
    a.fLD = make_fastdiv((u32)ld); a.fC = make_fastdiv((u32)C); a.fKW = make_fastdiv((u32)KW);
    a.fOW = make_fastdiv((u32)OW); a.fOH = make_fastdiv((u32)OH);
    if (aligned && C % 2 == 0 && ld % 2 == 0) {
        a.total = (u32)(total / 2);
        hipLaunchKernelGGL(k_im2col3<2>, dim3(nblocks(a.total, TPB), 3), dim3(TPB), 0, s, a);
    } else {
        a.total = (u32)total;
        hipLaunchKernelGGL(k_im2col3<1>, dim3(nblocks(a.total, TPB), 3), dim3(TPB), 0, s, a);
    }
}
void launch_sumpool2(const u64* x, int B, int H, int W, int C, u64* out, hipStream_t s) {
    const int64_t total = (int64_t)B * (H / 2) * (W / 2) * C;
    if (total <= 0) return;
    hipLaunchKernelGGL(k_sumpool2, dim3(nblocks(total, TPB)), dim3(TPB), 0, s, x, B, H, W, C, out);
}
void launch_rec_check(int64_t n, const u64* r1, Inj r1inj, int* flag, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rec_check, dim3(nblocks(n, TPB)), dim3(TPB), 0, s, n, r1, r1inj, flag);
}
void launch_rec_open(int64_t n, const u64* m, const u64* r1, const u64* r2, const int* flag, u64* out,
                     hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rec_open, dim3(nblocks(n, TPB)), dim3(TPB), 0, s, n, m, r1, r2, flag, out);
}
void launch_random_gr(const Keys& k, u32 op, u32 purpose, u32 sub, u64* share3, u64* value, u64* log,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_random_gr, dim3(1), dim3(64), 0, s, k, op, purpose, sub, share3, value, log);
}
void launch_gr_outer(const u64* P, int64_t np, const u64* Q, int64_t nq, u64* out, hipStream_t s) {
    if (np <= 0 || nq <= 0) return;
    hipLaunchKernelGGL(k_gr_outer, dim3((unsigned)(np * nq)), dim3(64), 0, s, P, Q, nq, out);
}
void launch_mulmat(const u64* src, int64_t stride, int nb, u64* W, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_mulmat, dim3(nb), dim3(64), 0, s, src, stride, W);
}
void launch_sum_blocks(const u64* C, int nsum, int64_t words, u64* out, hipStream_t s) {
    if (words <= 0) return;
    hipLaunchKernelGGL(k_sum_blocks, dim3(nblocks(words, TPB)), dim3(TPB), 0, s, C, nsum, words, out);
}
void launch_pow_ap2(const u64* lo, const u64* hi, int64_t L, int64_t e0a, int64_t e0b, int64_t step, int64_t n,
                    u64* outa, u64* outb, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pow_ap2, dim3((unsigned)(2 * n)), dim3(64), 0, s, lo, hi, L, e0a, e0b, step, n, outa, outb);
}
void launch_fold_plain(const u64* C, int nb, u64* out, hipStream_t s) {
    hipLaunchKernelGGL(k_fold_plain, dim3(nb), dim3(256), 0, s, C, out);
}
void launch_polyevl_finish(const PolyEvlArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_polyevl_finish, dim3(1), dim3(256), 0, s, a);
}
void launch_at_x_diff(const u64* XY, int nc, int64_t n, u64* F, u64* D, hipStream_t s) {
    if (n < 2) return;
    hipLaunchKernelGGL(k_at_x_diff, dim3((unsigned)(n / 2), nc), dim3(64), 0, s, XY, n, F, D);
}
void launch_at_x(const u64* XY, int nc, int64_t n, u64* F, hipStream_t s) {
    if (n < 2) return;
    const int64_t items = (int64_t)nc * (n / 2);
    hipLaunchKernelGGL(k_at_x, dim3(nblocks(items, 4)), dim3(256), 0, s, XY, n, items, F);
}
void launch_mat_pair(const u64* Wz, u64* out, hipStream_t s) {
    hipLaunchKernelGGL(k_mat_pair, dim3(64), dim3(64), 0, s, Wz, out);
}
void launch_round_finish(const RoundArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_round_finish, dim3(1), dim3(256), 0, s, a);
}
void launch_round_mid(const RoundMidArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_round_mid, dim3(1), dim3(RM_THREADS), 0, s, a);
}
void launch_round_rows(const Keys& k, u32 op, u32 inst, int k0, int rounds, u64* out, hipStream_t s) {
    if (rounds <= 0) return;
    hipLaunchKernelGGL(k_round_rows, dim3((unsigned)rounds), dim3(128), 0, s, k, op, inst, k0, out);
}
void launch_xp_epilogue(int64_t n, const Keys& k, u32 op, u32 sub, const u64* C0, const u64* C1,
                        const u64* C2, u64* XPm, u64* XP1, u64* XP2, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_xp_epilogue, dim3(nblocks(n * 8, TPB)), dim3(TPB), 0, s, n, k, op, sub, C0, C1, C2, XPm,
                       XP1, XP2);
}
void launch_neg_elem(const u64* src, int64_t ps_in, u64* dst, int64_t ps_out, hipStream_t s) {
    hipLaunchKernelGGL(k_neg_elem, dim3(1), dim3(64), 0, s, src, ps_in, dst, ps_out);
}
void launch_scale_rows(int64_t n, const u64* a0, const u64* a1, const u64* a2, const u64* P, u64* out,
                       int64_t ps, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scale_rows, dim3(nblocks(n * 64, TPB)), dim3(TPB), 0, s, n, a0, a1, a2, P, out, ps);
}
void launch_lift_rows(int64_t n, const u64* a0, const u64* a1, const u64* a2, u64* out, int64_t ps,
                      hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_lift_rows, dim3(nblocks(n * 64, TPB)), dim3(TPB), 0, s, n, a0, a1, a2, out, ps);
}
void launch_trunc_instance2(int64_t lo, int64_t T, int t, const u64* B1, const u64* B2, const u64* P,
                            const u64* rxm, const u64* rx1, const u64* rx2, const u64* rzm, const u64* rz1,
                            const u64* rz2, u64* x1plane, u64* y2plane, u64* w3, hipStream_t s) {
    if (T <= 0) return;
    hipLaunchKernelGGL(k_trunc_instance, dim3((unsigned)(T * 128)), dim3(64), 0, s, T, t, B1, B2, P, x1plane,
                       y2plane);
    hipLaunchKernelGGL(k_trunc_w, dim3(nblocks(T, TPB)), dim3(TPB), 0, s, lo, T, t, B1, B2, rxm, rx1, rx2, rzm,
                       rz1, rz2, w3);
}
void launch_set_one(u64* p, hipStream_t s) { hipLaunchKernelGGL(k_set_one, dim3(1), dim3(64), 0, s, p); }
void launch_trunc_w(int64_t lo, int64_t T, int t, const u64* B1, const u64* B2, const u64* rxm, const u64* rx1,
                    const u64* rx2, const u64* rzm, const u64* rz1, const u64* rz2, u64* w3, hipStream_t s) {
    if (T <= 0) return;
    hipLaunchKernelGGL(k_trunc_w, dim3(nblocks(T, TPB)), dim3(TPB), 0, s, lo, T, t, B1, B2, rxm, rx1, rx2, rzm, rz1,
                       rz2, w3);
}
void launch_sym_coeffs(int j, int64_t G, int64_t ld, int t, const u64* B1, const u64* B2, u64* cx,
                       hipStream_t s) {
    if (ld <= 0) return;
    SymOrder ord{};
    int nu = 1;
    for (int i = 0; i < j; ++i) nu *= 3;
    int r = 0;
    for (int ones = 0; ones <= j; ++ones)
        for (int u = 0; u < nu; ++u) {
            int c = 0;
            for (int v = u; v; v /= 3) c += v % 3 == 1;
            if (c == ones) ord.u[r++] = (unsigned short)u;
        }
    const dim3 gr(nblocks(ld, SYM_GB)), bl(256);
    switch (j) {
        case 0: hipLaunchKernelGGL(k_sym_round0, dim3(nblocks(ld, TPB)), dim3(TPB), 0, s, G, ld, t, B1, B2, cx); break;
        case 1: hipLaunchKernelGGL(k_sym_round1, dim3(nblocks(ld, TPB)), dim3(TPB), 0, s, G, ld, t, B1, B2, cx); break;
        case 2: hipLaunchKernelGGL(k_sym_round2, dim3(nblocks(ld, TPB)), dim3(TPB), 0, s, G, ld, t, B1, B2, cx); break;
        case 3: hipLaunchKernelGGL(k_sym_coeffs<3>, gr, bl, 0, s, G, ld, t, B1, B2, cx, ord); break;
        case 4: hipLaunchKernelGGL(k_sym_coeffs<4>, gr, bl, 0, s, G, ld, t, B1, B2, cx, ord); break;
        default: break;     // j < 5: at most five symbolic rounds
    }
}
int sym_points_from() { return SYM_POINTS; }
void launch_interp3(u64* P, int nvar, hipStream_t s) {
    if (nvar < 1 || nvar > 5) return;
    hipLaunchKernelGGL(k_interp3, dim3(1), dim3(256), 0, s, P, nvar);
}
void launch_sym_level(int j, int64_t G, int t, const u64* B1, const u64* B2, u64* alpha, u64* gamma,
                      hipStream_t s) {
    if (G <= 0) return;
    hipLaunchKernelGGL(k_sym_level, dim3(nblocks(G, SYM_GB)), dim3(256), 0, s, j, G, t, B1, B2, alpha, gamma);
}
void launch_xshift_rows(const u64* in, int64_t n, int e, u64* out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_xshift_rows, dim3((unsigned)n), dim3(64), 0, s, in, n, e, out);
}
void launch_pow_level(u64* out, int64_t len, int64_t cnt, const u64* P, u64* Pn, hipStream_t s) {
    hipLaunchKernelGGL(k_pow_level, dim3((unsigned)(cnt + (Pn ? 1 : 0))), dim3(64), 0, s, out, len, cnt, P, Pn);
}
void launch_pow_ap(const u64* lo, const u64* hi, int64_t L, int64_t e0, int64_t step, int64_t n, u64* out,
                   hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pow_ap, dim3((unsigned)n), dim3(64), 0, s, lo, hi, L, e0, step, out);
}
bool launch_inner_verify_small(const InnerVerifyArgs& a, hipStream_t s) {
    if (a.n < 1 || a.n > IV_MAX) return false;
    hipLaunchKernelGGL(k_inner_verify_small, dim3(1), dim3(IV_WAVES * 64), 0, s, a);
    return true;
}
void launch_conv_bands(const ConvBandArgs& a, int chunks, hipStream_t s) {
    if (a.nsets <= 0 || chunks <= 0) return;
    hipLaunchKernelGGL(k_conv_bands, dim3((unsigned)a.nsets, 3, (unsigned)(chunks * ((a.C + 63) / 64))), dim3(256), 0,
                       s, a);
}
void launch_pow_shifts(const u64* lo, const u64* hi, int64_t L, int64_t e0, int KH, int KW, int W, u64* out,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_pow_shifts, dim3((unsigned)(KH * KW)), dim3(64), 0, s, lo, hi, L, e0, KW, W, out);
}
void launch_conv_x(const ConvXArgs& a, hipStream_t s) {
    if (a.K <= 0) return;
    hipLaunchKernelGGL(k_conv_x, dim3((unsigned)((a.K + 3) / 4), 3), dim3(256), 0, s, a);
}
void launch_pow_list(const u64* lo, const u64* hi, int64_t L, const PowJob* jobs, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pow_list, dim3((unsigned)n), dim3(64), 0, s, lo, hi, L, jobs);
}
void launch_gr_scale_rows(const RowsJob* jobs, int njobs, int64_t max_n, int64_t pstride, hipStream_t s) {
    if (njobs <= 0 || max_n <= 0) return;
    hipLaunchKernelGGL(k_gr_scale_rows, dim3((unsigned)((max_n + 1) / 2), 3, (unsigned)njobs), dim3(64), 0, s, jobs,
                       pstride);
}
void launch_conv_bands_jobs(const BandJob* jobs, int njobs, int max_sets, int max_z, hipStream_t s) {
    if (njobs <= 0 || max_sets <= 0 || max_z <= 0) return;
    hipLaunchKernelGGL(k_conv_bands_jobs, dim3((unsigned)max_sets, (unsigned)(3 * njobs), (unsigned)max_z), dim3(256),
                       0, s, jobs);
}
void launch_conv_x_jobs(const ConvXArgs* jobs, int njobs, int64_t max_k, hipStream_t s) {
    if (njobs <= 0 || max_k <= 0) return;
    hipLaunchKernelGGL(k_conv_x_jobs, dim3((unsigned)((max_k + 3) / 4), (unsigned)(3 * njobs)), dim3(256), 0, s, jobs);
}
void launch_gr_mul_rows(const u64* P, const u64* Q, int64_t n, int64_t per, u64* out, hipStream_t s, int planes,
                        int64_t pstride) {
    if (n <= 0 || planes <= 0) return;
    // many rows: 16 per workgroup (fewer, longer workgroups); few: 2, so they still spread
    const int rpb = n >= 65536 ? 16 : 2;
    hipLaunchKernelGGL(k_gr_mul_rows, dim3((unsigned)((n + rpb - 1) / rpb), (unsigned)planes), dim3(64), 0, s, P, Q, n,
                       per, out, pstride, rpb);
}


}  // namespace mpc3
