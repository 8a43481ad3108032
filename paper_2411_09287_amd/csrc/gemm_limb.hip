// Z_{2^64} matrix products on int8 MFMA (gfx950).
//
// Every 64-bit word is written in balanced radix 2^8: a = sum_{i<8} 2^{8i} a_i with
// a_i in [-128, 127].  Modulo 2^64 only the digit pairs with i + j <= 7 survive, so
//     A B = sum_{s<8} 2^{8s} P_s,   P_s = sum_{i+j=s} A_i B_j,
// 36 int8 matrix products accumulated into 8 int32 planes.  |P_s| <= K 8 2^14, so the
// int32 planes are folded into 64-bit partial sums every 8192 of K.  The result is
// bit-identical to the 64-bit integer product.
//
// The balanced digits of a are the bytes of (a + 0x8080..80) xor 0x8080..80 read as
// int8: the byte carries of that addition are exactly the carries of the balanced
// representation.  Tiles are read as 64-bit words, converted in registers, transposed
// to digit planes in LDS and fed to v_mfma_i32_32x32x32_i8; no digit planes touch HBM.
#include <cstring>
#include <type_traits>
#include <vector>

#include "gemm.h"
#include "limb_digits.h"

namespace mpc3 {

hipError_t gemm_u64(const GemmArgs& g, hipStream_t stream);

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

using limb::KB;
using limb::PLANE;
using limb::TILE_BYTES;
using limb::to_digits;
using limb::swz;
using limb::toff;
using limb::OFF;
using limb::bt4;
constexpr int TM = 64, TN = 64, KSEG = 8192, NT = 256;

// One operand of a product segment: v(r, k) = sum_i c_i P_i[b + r*s_r + k*s_k].
struct Opnd {
    const u64* p[2];
    int c[2];
    int64_t s_r, s_k;
    int64_t rows;                         // valid rows (M for A, N for B)
};

// A product: up to two K segments (each padded to Kp), operands for each.
struct Prod {
    Opnd a[2], b[2];
    int nseg;
    OutView C;
};

struct LArgs {
    Prod prod[3];
    int64_t M, N, K, Kp;                  // Kp: K rounded up to KB
    int64_t kchunk;                       // per split, multiple of KB
    int splits;
    int atomic;
    View D;
    u64* part;                            // split-K partial sums: plane (split, product) of M x N
};

// 8 consecutive k of one row of an operand, loaded raw: w[i] = v(row, k0 + i).
__device__ __forceinline__ void load8(const Opnd& o, int64_t row, int64_t k0, int64_t K, u64 w[8]) {
    const bool inrow = row < o.rows;
    const int64_t base = row * o.s_r + k0 * o.s_k;
    if (inrow && o.s_k == 1 && k0 + 8 <= K && (base & 1) == 0 && ((uintptr_t)o.p[0] & 15) == 0 &&
        (!o.c[1] || ((int64_t)(uintptr_t)o.p[1] & 15) == 0)) {
        // 16-byte vector loads of the 8 contiguous words
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const ulonglong2 x = *(const ulonglong2*)(o.p[0] + base + 2 * h);
            w[2 * h] = x.x;
            w[2 * h + 1] = x.y;
        }
        if (o.c[0] < 0)
#pragma unroll
            for (int i = 0; i < 8; ++i) w[i] = 0 - w[i];
        if (o.c[1]) {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const ulonglong2 x = *(const ulonglong2*)(o.p[1] + base + 2 * h);
                w[2 * h] += o.c[1] > 0 ? x.x : (0 - x.x);
                w[2 * h + 1] += o.c[1] > 0 ? x.y : (0 - x.y);
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t k = k0 + i;
        u64 v = 0;
        if (inrow && k < K) {
            const int64_t off = base + i * o.s_k;
            v = o.p[0][off];
            if (o.c[0] < 0) v = 0 - v;
            if (o.c[1]) {
                const u64 x = o.p[1][off];
                v += o.c[1] > 0 ? x : (0 - x);
            }
        }
        w[i] = v;
    }
}

// Thread -> (row, k-octet) of a 64 x 32 tile.  When k is contiguous in memory, 4 threads
// share a row and read 64 contiguous bytes each; otherwise 64 threads cover 64 rows of
// one k-octet so a wave reads 64 consecutive words per k.
__device__ __forceinline__ void tile_coord(const Opnd& o, int t, int& row, int& oct) {
    if (o.s_k == 1) { row = t >> 2; oct = t & 3; }
    else { row = t & 63; oct = t >> 6; }
}

__device__ __forceinline__ void fetch(const Prod& P, int64_t kglob, int64_t Kp, int64_t K, int64_t r0a,
                                      int64_t r0b, int t, u64 wa[8], u64 wb[8], int& ra, int& oa, int& rb,
                                      int& ob) {
    const int seg = (int)(kglob / Kp);
    const int64_t k0 = kglob - seg * Kp;
    const Opnd& A = P.a[seg];
    const Opnd& B = P.b[seg];
    tile_coord(A, t, ra, oa);
    tile_coord(B, t, rb, ob);
    load8(A, r0a + ra, k0 + 8 * oa, K, wa);
    load8(B, r0b + rb, k0 + 8 * ob, K, wb);
}

// LDS layouts of a 64 x 32 digit tile (PLANE bytes per digit):
//   KC (operand read with k contiguous): [row][32 k]      - 16-byte fragment reads
//   otherwise:                           [octet][row][8 k] - conflict-free 8-byte stores
template <bool KC>
__device__ __forceinline__ void stash(int8_t* lds, int row, int oct, const u64 w[8]) {
    u64 q[8];
    to_digits(w, q);
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        if constexpr (KC) *(u64*)(lds + d * PLANE + row * KB + oct * 8) = q[d];
        else *(u64*)(lds + d * PLANE + oct * 512 + row * 8) = q[d];
    }
}

// 16 consecutive k (kh .. kh+15) of one tile row for digit plane `plane`
template <bool KC>
__device__ __forceinline__ v4i frag(const int8_t* plane, int row, int kh) {
    if constexpr (KC) {
        return *(const v4i*)(plane + row * KB + kh);
    } else {
        const int o = kh >> 3;
        const u64 lo = *(const u64*)(plane + o * 512 + row * 8);
        const u64 hi = *(const u64*)(plane + (o + 1) * 512 + row * 8);
        v4i r;
        r.x = (int)(u32)lo; r.y = (int)(u32)(lo >> 32); r.z = (int)(u32)hi; r.w = (int)(u32)(hi >> 32);
        return r;
    }
}

template <bool AK, bool BK>
__global__ __launch_bounds__(NT, 2) void k_lgemm(LArgs a) {
    __shared__ __attribute__((aligned(16))) int8_t As[2][8 * PLANE];
    __shared__ __attribute__((aligned(16))) int8_t Bs[2][8 * PLANE];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int prod = blockIdx.z / a.splits, split = blockIdx.z % a.splits;
    const Prod& P = a.prod[prod];
    const int64_t Ktot = (int64_t)P.nseg * a.Kp;
    const int64_t kbeg = (int64_t)split * a.kchunk;
    const int64_t kend = min(Ktot, kbeg + a.kchunk);     // kchunk <= KSEG: no int32 overflow
    const int64_t r0a = (int64_t)blockIdx.y * TM, r0b = (int64_t)blockIdx.x * TN;
    const int wy = w >> 1, wx = w & 1;
    const int r = lane & 31, kh = (lane >> 5) * 16;
    const int arow = wy * 32 + r, brow = wx * 32 + r;

    v16i acc[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[s] = v16i{0};

    u64 wa[8], wb[8];
    int ra, oa, rb, ob;
    if (kbeg < kend) {
        fetch(P, kbeg, a.Kp, a.K, r0a, r0b, t, wa, wb, ra, oa, rb, ob);
        stash<AK>(As[0], ra, oa, wa);
        stash<BK>(Bs[0], rb, ob, wb);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += KB) {
        const bool more = k0 + KB < kend;
        if (more) fetch(P, k0 + KB, a.Kp, a.K, r0a, r0b, t, wa, wb, ra, oa, rb, ob);
        v4i B[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) B[d] = frag<BK>(Bs[buf] + d * PLANE, brow, kh);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const v4i A = frag<AK>(As[buf] + i * PLANE, arow, kh);
#pragma unroll
            for (int s = i; s < 8; ++s)
                acc[s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B[s - i], acc[s], 0, 0, 0);
        }
        if (more) {
            stash<AK>(As[buf ^ 1], ra, oa, wa);
            stash<BK>(Bs[buf ^ 1], rb, ob, wb);
        }
        __syncthreads();
        buf ^= 1;
    }
    // 32x32 accumulator layout: lane -> column (lane & 31); register v -> row
    // 8 (v >> 2) + 4 (lane >> 5) + (v & 3)
    const int64_t n = r0b + wx * 32 + (lane & 31);
    if (n >= a.N) return;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int64_t m = r0a + wy * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (m >= a.M) continue;
        u64 val = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) val += ((u64)(int64_t)acc[s][v]) << (8 * s);
        if (a.part) {
            a.part[((int64_t)split * (gridDim.z / a.splits) + prod) * a.M * a.N + m * a.N + n] = val;
            continue;
        }
        u64* p = P.C.p + m * P.C.s0 + n * P.C.s1;
        if (a.atomic) {
            atomicAdd((unsigned long long*)p, (unsigned long long)val);
        } else {
            if (a.D.p) val += a.D.p[m * a.D.s0 + n * a.D.s1];
            *p = val;
        }
    }
}

// ---------------------------------------------------------------------------
// Second form: B pre-converted to digit tiles.
//
// When B is re-read by many row tiles (a layer's weights, K x N against M >> 64 rows) its
// balanced digits are written once to a tile buffer and the product kernel copies them to
// LDS unchanged; only A is converted in the kernel.  A tile is k-block kb (32 deep) of 64
// consecutive B columns: 8 digit planes x 64 rows x 32 bytes (16 KiB), stored exactly as
// it sits in LDS (limb_digits.h).

// Digit tiles of up to five operands (rows x K, any strides, optional two-plane
// combination), operand blockIdx.y: tile (t, kb) at byte (t * nkb + kb) * TILE_BYTES;
// rows >= o.rows and k >= K are zero.
// blockIdx.z is a batch: operand planes advance by ob words, tiles by tb bytes.
struct TileJob {
    Opnd o[5];
    int8_t* out[5];
    int64_t ob, tb;
};
__global__ void k_to_tiles(TileJob job, int64_t K, int64_t nkb, int64_t rows_pad) {
    Opnd o = job.o[blockIdx.y];
    o.p[0] += blockIdx.z * job.ob;
    if (o.p[1]) o.p[1] += blockIdx.z * job.ob;
    int8_t* out = job.out[blockIdx.y] + blockIdx.z * job.tb;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    u64 w[8], q[8];
    if (o.s_k == 1) {
        // k contiguous: consecutive threads take consecutive octets of a row (the four of a
        // k-block together write its 32-byte row segment of each plane)
        if (idx >= rows_pad * nkb * 4) return;
        const int64_t o8 = idx % (nkb * 4), r = idx / (nkb * 4);
        load8(o, r, o8 * 8, K, w);
        to_digits(w, q);
        int8_t* base = out + ((r >> 6) * nkb + (o8 >> 2)) * TILE_BYTES;
        const int rr = (int)(r & 63), oc = (int)(o8 & 3);
#pragma unroll
        for (int d = 0; d < 8; ++d) *(u64*)(base + toff(d, rr, oc)) = q[d];
        return;
    }
    // rows contiguous: quads of threads take consecutive rows (coalesced loads of 16 rows per
    // octet), the four threads of a quad the four octets of one k-block's row segment, so that
    // each store of a wave writes whole 32-byte segments (8-byte pieces of one octet from
    // every row made partial-sector writes: four times the bytes at the memory)
    if (idx >= rows_pad * nkb * 4) return;
    const int oc = (int)(idx & 3);
    const int64_t r = (idx >> 2) % rows_pad, kb = (idx >> 2) / rows_pad;
    load8(o, r, (kb * 4 + oc) * 8, K, w);
    to_digits(w, q);
    int8_t* base = out + ((r >> 6) * nkb + kb) * TILE_BYTES;
    const int rr = (int)(r & 63);
#pragma unroll
    for (int d = 0; d < 8; ++d) *(u64*)(base + toff(d, rr, oc)) = q[d];
}

// A segment of a product: one A plane (k contiguous, row stride lda), or the sum of two
// planes when p2 is set, and the digit tiles of its B operand.  Every sign of the party
// form sits on the B side.
struct Seg2 {
    const u64* p;
    const u64* p2;
    const int8_t* bt;
};
struct Prod2 {
    Seg2 seg[2];
    int nseg;
    OutView C;
};
struct L2Args {
    Prod2 prod[3];
    int64_t M, N, K, lda, ldk;   // A element (row, k) at row * lda + k * ldk
    int nkb;                     // k-blocks per segment
    int bnkb;                    // k-blocks per column tile in the B tile buffers
    int kcb;                     // k-blocks per split (two segments interleaved)
    int nprod, splits;
    int tn;                      // column groups of the grid (NS tiles of 64 each)
    int tn64;                    // 64-column tiles of B
    int tm;                      // 64-row tiles
    int rb;                      // row tiles per group of the launch order
    // implicit lowering (CONV kernels): A is the NHWC input of a stride-1 convolution, row m
    // = output position (b, oh, ow) of cOH x cOW per image, column k = (kh, kw, c) with
    // C = 32 ccb channels; positions outside the input read as 0
    int cH, cW, cC, cKW, cpad, cOH, cOW, ccb;
    int atomic;
    View D;
    u64* part;                   // split-K partial sums: plane (batch, split, product) of M x N
    int64_t sbA, sbC, sbT;       // per batch: A planes and C (words), B tiles (bytes)
};

// 8 raw words of one A row: rp points at k = k0 (the thread's octet); words at k >= K read
// as 0.  FAST: every row is 16-byte aligned and K is a multiple of the k-block, so the
// octet is four 16-byte loads.  Otherwise eight 8-byte loads of clamped (valid)
// addresses, masked afterwards, with no branches.
template <bool FAST>
__device__ __forceinline__ void raw8(const u64* rp, int64_t k0, int64_t K, u64 x[8]) {
    if (FAST) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const ulonglong2 v = *(const ulonglong2*)(rp + 2 * h);
            x[2 * h] = v.x;
            x[2 * h + 1] = v.y;
        }
    } else {
        const int64_t last = K - 1 - k0;      // index of the row's last word relative to rp
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const u64 v = rp[min((int64_t)i, last)];
            x[i] = i <= last ? v : 0;
        }
    }
}

// the 8 digit bytes of an octet of k (q[d]: digit d) at byte offset off of each plane
__device__ __forceinline__ void storeA8(int8_t* tile, int off, const u64 q[8]) {
#pragma unroll
    for (int d = 0; d < 8; ++d) *(u64*)(tile + d * PLANE + off) = q[d];
}

// s_waitcnt with only the vector-memory counter constrained (vmcnt <= n)
template <int n>
__device__ __forceinline__ void wait_vm() {
    __builtin_amdgcn_s_waitcnt((n & 15) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// One workgroup computes a 64 x (64 NS) tile of one product with 4 NS waves (32 x 32 each).
// Per k-block g (FAST: K a multiple of 32, aligned rows):
//   - the B digit tiles of block g+1 are loaded into registers and the A words of block
//     g+2 are loaded, all before the MFMAs of block g;
//   - block g+1's A words (loaded one block earlier) are converted to digits in pieces
//     placed between the MFMA rows of block g, so the vector ALU works while the matrix
//     cores do, and stored to the other LDS buffer afterwards.  Only plain loads are in
//     flight, so every wait the compiler places is exact.
// Otherwise (NS = 1): B tiles are copied straight into LDS (global_load_lds) and A words are
// converted after the MFMAs.
// One workgroup's tile: workgroup L of the nwg of product a.
template <bool FAST, int NS, bool TA, bool CONV>
__device__ __forceinline__ void lgemm2_tile(const L2Args& a, const int L, const int nwg) {
    static_assert(!CONV || (FAST && !TA), "the implicit lowering loads 16-byte pieces of k-contiguous rows");
    constexpr int WPT = 8 / NS;                  // A words converted per thread and k-block
    __shared__ __attribute__((aligned(16))) int8_t As[2][TILE_BYTES];
    __shared__ __attribute__((aligned(16))) int8_t Bs[2][NS * TILE_BYTES];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int sub = w >> 2, wl = w & 3;
    // Workgroup ids are dealt round-robin to the 8 XCDs; renumber so that every XCD works
    // through a contiguous run of T.  In T order, groups of rb row tiles take every column
    // group of one (product, split) before the next: the workgroups an XCD runs at once
    // walk K together over the same B tiles, and the column groups of a row tile share
    // its A rows, in that XCD's L2.
    if (L >= nwg) return;                        // a group's padding workgroup
    const int q8 = nwg / 8;
    const int T0 = L < 8 * q8 ? (L % 8) * q8 + L / 8 : L;
    const int per = a.tn * a.nprod * a.splits;   // workgroups per row tile
    const int bI = T0 / (per * a.tm);            // batch (consecutive runs of T)
    const int T = T0 - bI * per * a.tm;
    const int grp = T / (a.rb * per);
    const int first = grp * a.rb, rows = min(a.tm - first, a.rb);
    const int within = T - grp * a.rb * per;
    const int tmi = first + within % rows;
    int rest = within / rows;
    const int tni = rest % a.tn;
    rest /= a.tn;
    const int prod = rest % a.nprod;
    const int split = rest / a.nprod;
    const Prod2& P = a.prod[prod];
    const int nkb = a.nkb;
    const int gbeg = split * a.kcb;
    const int gend = min(P.nseg * nkb, gbeg + a.kcb);
    const int tcol = tni * NS + sub;             // this wave group's 64-column tile
    const int64_t r0a = (int64_t)tmi * TM, r0b = (int64_t)tcol * TN;
    // A loader: row ra, WPT consecutive words at k = part * WPT
    // A loader: row ra, WPT consecutive k at k = part * WPT.  With k contiguous (TA false)
    // 32 / WPT threads share a row; with rows contiguous (TA, a transposed view) 64
    // consecutive threads take 64 consecutive rows, so each of their loads is coalesced.
    const int ra = TA ? t & 63 : (NS == 1 ? t >> 2 : t >> 3);
    const int part = TA ? t >> 6 : (NS == 1 ? t & 3 : t & 7);
    // rows past M load row M-1: they only feed accumulator rows that are never stored.  With
    // the implicit lowering the row's offset is that of input position (oh - pad, ow - pad)
    // of its image (possibly outside the input; only valid positions are dereferenced).
    int64_t aoff;
    int ohw = 0;                                 // CONV: oh << 16 | ow
    if constexpr (CONV) {
        const int64_t m = min(r0a + ra, a.M - 1), per_img = (int64_t)a.cOH * a.cOW;
        const int64_t b = m / per_img;
        const int rem = (int)(m - b * per_img), oh = rem / a.cOW, ow = rem - oh * a.cOW;
        ohw = (oh << 16) | ow;
        aoff = ((b * a.cH + oh - a.cpad) * a.cW + (ow - a.cpad)) * a.cC + part * WPT;
    } else {
        aoff = min(r0a + ra, a.M - 1) * a.lda + part * WPT * a.ldk;
    }
    const int tt = t & (NT - 1);
    // column tiles past the last one read the last one: their outputs are never stored
    const int64_t boff = (int64_t)min(tcol, a.tn64 - 1) * a.bnkb * TILE_BYTES + tt * 16;
    const u64* pa[2];
    const int8_t* pb[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const Seg2& S = P.seg[s < P.nseg ? s : 0];
        pa[s] = S.p + aoff + bI * a.sbA;
        pb[s] = S.bt + boff + bI * a.sbT;
    }
    // a summed segment (only ever the first): its second plane
    const u64* pa2 = P.seg[0].p2 ? P.seg[0].p2 + aoff + bI * a.sbA : nullptr;
    const int wy = wl >> 1, wx = wl & 1, r = lane & 31, hf = lane >> 5;
    const int arow = wy * 32 + r, brow = wx * 32 + r;
    const int aread = arow * KB + ((hf ^ swz(arow)) << 4);
    const int bread = sub * TILE_BYTES + brow * KB + ((hf ^ swz(brow)) << 4);
    // A digits of this thread's words: NS = 1 an 8-byte octet, NS = 2 a 4-byte quad
    const int astore = NS == 1 ? ra * KB + (((part >> 1) ^ swz(ra)) << 4) + ((part & 1) << 3)
                               : ra * KB + (((part >> 2) ^ swz(ra)) << 4) + ((part & 3) << 2);

    v16i acc[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[s] = v16i{0};

    // two segments alternate block by block, so that the three products of a row tile,
    // which share its A planes two by two, read each k-block of a plane at about the same
    // time and the second read hits L2 (measured on 32768 x 576 x 64: 689 -> 533 MB fetched)
    // With the implicit lowering the blocks are visited channel block by channel block, the
    // KH KW kernel offsets of one innermost: consecutive blocks then read the same channels
    // at nearby shifts of the input, which stay in cache (the sum is the same in any order).
    auto seg_of = [&](int g, int& kb) {
        const int s = P.nseg == 2 ? g & 1 : 0;
        kb = P.nseg == 2 ? g >> 1 : g;
        if constexpr (CONV) {
            const int khkw = a.nkb / a.ccb, cb = kb / khkw;
            kb = (kb - cb * khkw) * a.ccb + cb;
        }
        return s;
    };
    // the WPT words of block g at x[0, WPT); with SUM the second plane's at x[WPT, 2 WPT).
    // Returns the mask the conversion applies to them: all ones, or 0 for a position of the
    // implicit lowering outside the input (then the loads read the row's own first words;
    // masking at conversion keeps the loads in flight until then).
    auto loadA = [&](int g, u64* x, auto sum_c) -> u64 {
        constexpr bool SUM = decltype(sum_c)::value;
        int kb;
        const int s = seg_of(g, kb);
        const int64_t k0 = (int64_t)kb * KB;
        u64 zm = ~0ull;
        int64_t d = k0 * a.ldk;
        if constexpr (CONV) {
            const int khkw = kb / a.ccb, c0 = (kb - khkw * a.ccb) * KB;
            const int kh = khkw / a.cKW, kw = khkw - kh * a.cKW;
            const int ih = (ohw >> 16) + kh - a.cpad, iw = (ohw & 0xFFFF) + kw - a.cpad;
            const bool ok = (unsigned)ih < (unsigned)a.cH && (unsigned)iw < (unsigned)a.cW;
            // invalid: the words at the image's first position (always inside the plane)
            const int64_t b0 = -((int64_t)((ohw >> 16) - a.cpad) * a.cW + ((ohw & 0xFFFF) - a.cpad)) * a.cC;
            d = ok ? ((int64_t)kh * a.cW + kw) * a.cC + c0 : b0;
            zm = ok ? ~0ull : 0ull;
        }
#pragma unroll
        for (int h = 0; h < (SUM ? 2 : 1); ++h) {
            const u64* rp = (h ? pa2 : s ? pa[1] : pa[0]) + d;
            u64* xh = x + h * WPT;
            if (TA) {
#pragma unroll
                for (int i = 0; i < WPT; ++i) xh[i] = rp[i * a.ldk];
            } else if (FAST) {
#pragma unroll
                for (int q = 0; q < WPT / 2; ++q) {
                    const ulonglong2 v = *(const ulonglong2*)(rp + 2 * q);
                    xh[2 * q] = v.x;
                    xh[2 * q + 1] = v.y;
                }
            } else {
                raw8<false>(rp, k0 + part * WPT, a.K, xh);
            }
        }
        return zm;
    };
    auto dmaB = [&](int g, int buf) {
        int kb;
        const int s = seg_of(g, kb);
        const int8_t* bp = (s ? pb[1] : pb[0]) + (int64_t)kb * TILE_BYTES;
        int8_t* bl = Bs[buf] + w * 1024;
#pragma unroll
        for (int h = 0; h < 4; ++h)
            __builtin_amdgcn_global_load_lds((const void*)(bp + h * 4096), (void*)(bl + h * 4096), 16, 0, 0);
    };
    v4i bx[4];
    auto loadB = [&](int g) {
        int kb;
        const int s = seg_of(g, kb);
        const int8_t* bp = (s ? pb[1] : pb[0]) + (int64_t)kb * TILE_BYTES;
#pragma unroll
        for (int h = 0; h < 4; ++h) bx[h] = *(const v4i*)(bp + h * 4096);
    };
    auto storeB = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 4; ++h) *(v4i*)(Bs[buf] + sub * TILE_BYTES + tt * 16 + h * 4096) = bx[h];
    };
    // digits of WPT words as 4 x (WPT/2) transposed dwords tq[b]: b = 0, 1 the low words'
    // digits 0..3 (WPT = 8: words 0..3, 4..7), then the high digits 4..7
    auto store_digits = [&](const u32 tq[4][4], int buf) {
        if (WPT == 8) {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                *(u64*)(As[buf] + d * PLANE + astore) = (u64)tq[0][d] | ((u64)tq[1][d] << 32);
                *(u64*)(As[buf] + (4 + d) * PLANE + astore) = (u64)tq[2][d] | ((u64)tq[3][d] << 32);
            }
        } else {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                *(u32*)(As[buf] + d * PLANE + astore) = tq[0][d];
                *(u32*)(As[buf] + (4 + d) * PLANE + astore) = tq[1][d];
            }
        }
    };
    // conversion piece c of WPT words (c = 0: balanced bytes; c >= 1: one 4x4 transpose)
    auto piece = [&](int c, const u64* xc, u64 zm, u32 lo[WPT], u32 hi[WPT], u32 tq[4][4], auto sum_c) {
        constexpr bool SUM = decltype(sum_c)::value;
        if (c == 0) {
#pragma unroll
            for (int j = 0; j < WPT; ++j) {
                const u64 v = (((SUM ? xc[j] + xc[WPT + j] : xc[j]) & zm) + OFF) ^ OFF;
                lo[j] = (u32)v;
                hi[j] = (u32)(v >> 32);
                asm volatile("" : "+v"(lo[j]), "+v"(hi[j]));
            }
        } else if (c <= WPT / 2) {
            const int b = c - 1;
            const u32* src = WPT == 8 ? (b < 2 ? lo : hi) + 4 * (b & 1) : (b == 0 ? lo : hi);
            bt4(src[0], src[1], src[2], src[3], tq[b][0], tq[b][1], tq[b][2], tq[b][3]);
            asm volatile("" : "+v"(tq[b][0]), "+v"(tq[b][1]), "+v"(tq[b][2]), "+v"(tq[b][3]));
        }
    };

    int buf = 0;
    // SUM: the product's only segment is over the sum of two A planes
    auto mainloop = [&](auto sum_c) {
        constexpr bool SUM = decltype(sum_c)::value;
        constexpr int XW = SUM ? 2 * WPT : WPT;
        u64 xa[XW], xb[XW];
        if constexpr (!FAST) {
            auto convert = [&](int to) {
                if (SUM)
#pragma unroll
                    for (int i = 0; i < WPT; ++i) xa[i] += xa[WPT + i];
                u64 q[8];
                to_digits(xa, q);
                storeA8(As[to], astore, q);
            };
            if (gbeg < gend) {
                dmaB(gbeg, 0);
                loadA(gbeg, xa, sum_c);
                convert(0);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            for (int g = gbeg; g < gend; ++g) {
                v4i B[8], A[8];
#pragma unroll
                for (int d = 0; d < 8; ++d) B[d] = *(const v4i*)(Bs[buf] + d * PLANE + bread);
#pragma unroll
                for (int d = 0; d < 8; ++d) A[d] = *(const v4i*)(As[buf] + d * PLANE + aread);
                const int g1 = min(g + 1, gend - 1);      // past the end: re-reads a valid block
                dmaB(g1, buf ^ 1);
                loadA(g1, xa, sum_c);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int s = i; s < 8; ++s)
                        acc[s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[i], B[s - i], acc[s], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                convert(buf ^ 1);
                wait_vm<0>();
                __syncthreads();
                buf ^= 1;
            }
        } else {
            u64 ma = ~0ull, mb = ~0ull;          // the conversion masks of xa, xb
            if (gbeg < gend) {
                loadB(gbeg);
                const u64 m0 = loadA(gbeg, xb, sum_c);
                u32 lo[WPT], hi[WPT], tq[4][4];
#pragma unroll
                for (int c = 0; c <= WPT / 2; ++c) piece(c, xb, m0, lo, hi, tq, sum_c);
                store_digits(tq, 0);
                storeB(0);
                ma = loadA(min(gbeg + 1, gend - 1), xa, sum_c);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            auto body = [&](int g, const u64* xc, u64 mc, u64* xn, u64& mn) {
                loadB(min(g + 1, gend - 1));              // past the end: re-reads valid blocks
                mn = loadA(min(g + 2, gend - 1), xn, sum_c);
                __builtin_amdgcn_sched_barrier(0);
                v4i B[8];
#pragma unroll
                for (int d = 0; d < 8; ++d) B[d] = *(const v4i*)(Bs[buf] + d * PLANE + bread);
                u32 lo[WPT], hi[WPT], tq[4][4];
                v4i A = *(const v4i*)(As[buf] + aread);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    // the next row's A fragment is read while this row's MFMAs run
                    const v4i An = i < 7 ? *(const v4i*)(As[buf] + (i + 1) * PLANE + aread) : A;
#pragma unroll
                    for (int s = i; s < 8; ++s)
                        acc[s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B[s - i], acc[s], 0, 0, 0);
                    A = An;
                    // (the empty asm in piece() pins each part here: without it the compiler
                    // sinks the arithmetic to its use after the last MFMA)
                    piece(i, xc, mc, lo, hi, tq, sum_c);
                    __builtin_amdgcn_sched_barrier(0);
                }
                store_digits(tq, buf ^ 1);
                storeB(buf ^ 1);
                // B of block g+1 is stored; the A words of block g+2 may still be in flight
                wait_vm<(SUM ? 2 : 1) * (TA ? WPT : WPT / 2)>();
                __syncthreads();
                buf ^= 1;
            };
            int g = gbeg;
            for (; g + 1 < gend; g += 2) {
                body(g, xa, ma, xb, mb);
                body(g + 1, xb, mb, xa, ma);
            }
            if (g < gend) body(g, xa, ma, xb, mb);
        }
    };
    // (one-tile FAST kernels convert 8 words per thread: a second plane would spill)
    if constexpr (NS == 2 || !FAST) {
        if (pa2) mainloop(std::true_type{});
        else mainloop(std::false_type{});
    } else {
        mainloop(std::false_type{});
    }

    const int64_t n = r0b + wx * 32 + (lane & 31);
    if (n >= a.N) return;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int64_t m = r0a + wy * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (m >= a.M) continue;
        u64 val = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) val += ((u64)(int64_t)acc[s][v]) << (8 * s);
        if (a.part) {
            a.part[(((int64_t)bI * a.splits + split) * a.nprod + prod) * a.M * a.N + m * a.N + n] = val;
            continue;
        }
        u64* p = P.C.p + bI * a.sbC + m * P.C.s0 + n * P.C.s1;
        if (a.atomic) {
            atomicAdd((unsigned long long*)p, (unsigned long long)val);
        } else {
            if (a.D.p) val += a.D.p[bI * a.D.sb + m * a.D.s0 + n * a.D.s1];
            *p = val;
        }
    }
}

template <bool FAST, int NS, bool TA = false, bool CONV = false>
__global__ __launch_bounds__(NT * NS, 2 / NS) void k_lgemm2(L2Args a) {
    lgemm2_tile<FAST, NS, TA, CONV>(a, blockIdx.x, gridDim.x);
}

// The products of a group in one grid: product j takes workgroups start[j] ..
// start[j] + count[j] - 1; start[j] is a multiple of 8, so each product's workgroups reach
// the XCDs in the order its tile numbering assumes.  The block index decides the product
// for the whole workgroup, so its fields are read as scalars.
template <bool FAST, int NS, bool TA = false, bool CONV = false>
__global__ __launch_bounds__(NT * NS, 2 / NS) void k_lgemm2_group(const L2Args* tab, const int* start,
                                                                   const int* count, int n) {
    const int blk = blockIdx.x;
    int j = 0;
    for (int i = 1; i < n; ++i)
        if (start[i] <= blk) j = i;
    lgemm2_tile<FAST, NS, TA, CONV>(tab[j], blk - start[j], count[j]);
}

inline int64_t rup(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Plain products of one or two k-blocks (K <= 64, one split), whose workgroups k_lgemm2
// would run as a short chain of dependent steps (load, convert, multiply, store) with little
// to overlap: a fixed grid walks the 64 x 64 output tiles instead, and each workgroup loads
// the next step's A words and B tiles while the matrix cores and the stores of the current
// one run (a step is one k-block of one tile; one LDS buffer per operand).  The stores are
// buffer stores whose offset is moved out of the buffer's range for outputs past M or N, so
// that every step issues the same count and the wait for the next step's loads does not wait
// for them.  Workgroups are dealt to the 8 XCDs round-robin: each XCD takes a contiguous
// range of tiles, so the tiles one XCD runs at once share their B tiles in its L2.  Tile
// order: column tile fastest, then product, row tile, batch.  gridDim.x is a multiple of 8;
// C plain (no D, no atomics), strides >= 0, a tile's outputs within 2^31 bytes of its first.
typedef u32 v2u __attribute__((ext_vector_type(2)));

template <int NKB>
__global__ __launch_bounds__(NT, 2) void k_lgemm_stream(L2Args a, int ntiles) {
    __shared__ __attribute__((aligned(16))) int8_t As[TILE_BYTES];
    __shared__ __attribute__((aligned(16))) int8_t Bs[TILE_BYTES];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wy = w >> 1, wx = w & 1, r = lane & 31, hf = lane >> 5;
    const int arow = wy * 32 + r, brow = wx * 32 + r;
    const int aread = arow * KB + ((hf ^ swz(arow)) << 4);
    const int bread = brow * KB + ((hf ^ swz(brow)) << 4);
    // A loader: row ra of the tile, the 8 words of octet part of the k-block
    const int ra = t >> 2, part = t & 3;
    const int astore = ra * KB + (((part >> 1) ^ swz(ra)) << 4) + ((part & 1) << 3);
    const int per_x = (ntiles + 7) >> 3, nx = (int)(gridDim.x >> 3);
    const int lo = (int)(blockIdx.x & 7) * per_x, hi = min(ntiles, lo + per_x);
    int T = lo + (int)(blockIdx.x >> 3);
    if (T >= hi) return;                         // the whole workgroup
    struct Tile {
        int bI, tmi, prod, tni;
    };
    auto decode = [&](int v) {
        const unsigned u = (unsigned)v, q1 = u / (unsigned)a.tn, q2 = q1 / (unsigned)a.nprod,
                       q3 = q2 / (unsigned)a.tm;
        Tile d;
        d.tni = __builtin_amdgcn_readfirstlane((int)(u - q1 * (unsigned)a.tn));
        d.prod = __builtin_amdgcn_readfirstlane((int)(q1 - q2 * (unsigned)a.nprod));
        d.tmi = __builtin_amdgcn_readfirstlane((int)(q2 - q3 * (unsigned)a.tm));
        d.bI = __builtin_amdgcn_readfirstlane((int)q3);
        return d;
    };
    u64 x[8];
    v4i bx[4];
    // rows past M load row M-1 (their accumulator rows are never stored)
    auto load = [&](const Tile& d, int kb) {
        const Seg2& S = a.prod[d.prod].seg[0];
        const u64* rp = S.p + d.bI * a.sbA + min((int64_t)d.tmi * TM + ra, a.M - 1) * a.lda + part * 8 + kb * KB;
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const ulonglong2 u = *(const ulonglong2*)(rp + 2 * h);
            x[2 * h] = u.x;
            x[2 * h + 1] = u.y;
        }
        const int8_t* bp = S.bt + d.bI * a.sbT + ((int64_t)d.tni * a.bnkb + kb) * TILE_BYTES + t * 16;
#pragma unroll
        for (int h = 0; h < 4; ++h) bx[h] = *(const v4i*)(bp + h * 4096);
    };
    v16i acc[8];
    // one tile: its k-blocks, then its stores; the loads of the next step are issued before
    // the MFMAs of each step (past the range they re-read the current tile: always issued)
    auto tile = [&](const Tile& cur, const Tile& nxt) {
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            u64 q[8];
            to_digits(x, q);
            __syncthreads();                     // the previous step's fragment reads are done
            storeA8(As, astore, q);
#pragma unroll
            for (int h = 0; h < 4; ++h) *(v4i*)(Bs + t * 16 + h * 4096) = bx[h];
            __syncthreads();
            if (kb + 1 < NKB) load(cur, kb + 1);
            else load(nxt, 0);
            if (kb == 0) {
#pragma unroll
                for (int s = 0; s < 8; ++s) acc[s] = v16i{0};
            }
            v4i B[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) B[d] = *(const v4i*)(Bs + d * PLANE + bread);
            v4i A = *(const v4i*)(As + aread);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const v4i An = i < 7 ? *(const v4i*)(As + (i + 1) * PLANE + aread) : A;
#pragma unroll
                for (int s = i; s < 8; ++s)
                    acc[s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B[s - i], acc[s], 0, 0, 0);
                A = An;
            }
        }
        const OutView& C = a.prod[cur.prod].C;
        u64* base = C.p + (int64_t)cur.bI * a.sbC + (int64_t)cur.tmi * TM * C.s0;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(base, 0, 0x7FFFFFFF, 0x00020000);
        const int n = cur.tni * TN + wx * 32 + r;
        const bool nok = n < a.N;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int mloc = wy * 32 + 8 * (v >> 2) + 4 * hf + (v & 3);
            const bool ok = nok && cur.tmi * TM + mloc < a.M;
            const int off = ok ? (int)((mloc * C.s0 + n * C.s1) * 8) : (int)0x80000000;
            u64 val = 0;
#pragma unroll
            for (int s = 0; s < 8; ++s) val += ((u64)(int64_t)acc[s][v]) << (8 * s);
            const v2u u = {(u32)val, (u32)(val >> 32)};
            __builtin_amdgcn_raw_buffer_store_b64(u, rs, off, 0, 0);
        }
    };
    // the first tile outside the loop, so that every path into the loop has issued the same
    // loads and stores and the wait for the loads is exact
    Tile cur = decode(T);
    load(cur, 0);
    int Tn = T + nx;
    Tile nxt = Tn < hi ? decode(Tn) : cur;
    tile(cur, nxt);
    while (Tn < hi) {
        cur = nxt;
        Tn += nx;
        nxt = Tn < hi ? decode(Tn) : cur;
        tile(cur, nxt);
    }
}

// Workgroups of k_lgemm_stream for ntiles tiles: per XCD at most as many as its CUs hold at
// once (the device's own figures, per device).
int stream_grid(int64_t ntiles) {
    static int per_xcd[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (!per_xcd[dev]) {
        int cus = 0, occ = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_lgemm_stream<1>, NT, 0) != hipSuccess)
            return 0;
        per_xcd[dev] = std::max(1, cus / 8) * std::max(1, occ);
    }
    const int64_t per_x = (ntiles + 7) / 8;
    return 8 * (int)std::min<int64_t>(per_x, per_xcd[dev]);
}


Opnd opnd(const View& v, int64_t b, bool transpose, int64_t rows, int c0 = 1) {
    Opnd o{};
    o.p[0] = v.p + b * v.sb;
    o.c[0] = c0;
    o.p[1] = nullptr;
    o.c[1] = 0;
    o.s_r = transpose ? v.s1 : v.s0;
    o.s_k = transpose ? v.s0 : v.s1;
    o.rows = rows;
    return o;
}

// c0 * P[i0] + c1 * P[i1] over the three planes of a party operand
Opnd combo(const View* v, int64_t b, bool transpose, int64_t rows, int i0, int c0, int i1, int c1) {
    Opnd o = opnd(v[i0], b, transpose, rows, c0);
    if (i1 >= 0) {
        o.p[1] = v[i1].p + b * v[i1].sb;
        o.c[1] = c1;
    }
    return o;
}


// ---------------------------------------------------------------------------
// The two Pi_PolyEvl products of a Pi_Reduce round, h(0) and h(x), as the parties' local
// sums, in one pass over the stored pairs (f(2i), f(2i+1)) of every plane:
//     at 0:  sum_i a(f_i(0)) (x) b(g_i(0)),   at x:  sum_i a(F_i) (x) b(G_i),
//     F_i = f(2i) + x (f(2i+1) - f(2i))
// where (x) is the 64 x 64 outer product of the coefficient vectors (its anti-diagonal sums,
// reduced modulo the ring's modulus, are the ring product) and a, b are the combinations of
// share planes one party multiplies: a workgroup takes one party (blockIdx.y) and adds up
// its segments (a . b products) over blocks of 32 pairs.  Wave w reads pairs 8w .. 8w+7
// (lane = coefficient, 512 coalesced bytes per row), forms both points in registers (x (.)
// is a shift across the lanes), and writes their balanced digits as transposed k-octets
// (row = coefficient, k = pair) to LDS; each wave then multiplies one 32 x 32 quadrant of
// both outer products on the matrix cores and adds the recombined 64-bit values to its
// running sums.  At the end the workgroup folds its two 64 x 64 sums to anti-diagonal sums
// (lo: j + l = k, hi: j + l = 64 + k) and adds them atomically into acc; the reduction
// modulo the ring's modulus is linear and is left to the consumer.
// ---------------------------------------------------------------------------
constexpr int HP_OPS = 4;                       // a f(0), a F, b f(0), b F

// Units of work: segment s of party p's sum, side 0 (a, the x side) or 1 (b, the y side):
// c0 * plane i0 + c1 * plane i1.  Dense (six planes x: m 0, r1 1, r2 2; y: m 3, r1 4, r2 5),
// the sums of k_polyevl_finish, five units: P0 (r1 + r2)_x (r1 + r2)_y (unit 0); P1 m_x r1_y
// (1) + r1_x m_y (2); P2 m_x (m_y - r2_y) (3) - r2_x m_y (4).  Sparse (the truncation gates:
// x's [r]_1 plane 0, y's [r]_2 plane 1): one unit, P0's only product.
struct HSide {
    int i0, c0, i1, c1;
};
__device__ constexpr HSide hunit(bool dense, int unit, int side) {
    return !dense ? (side == 0 ? HSide{0, 1, 0, 0} : HSide{1, 1, 0, 0})
           : unit == 0 ? (side == 0 ? HSide{1, 1, 2, 1} : HSide{4, 1, 5, 1})
           : unit == 1 ? (side == 0 ? HSide{0, 1, 0, 0} : HSide{4, 1, 0, 0})
           : unit == 2 ? (side == 0 ? HSide{1, 1, 0, 0} : HSide{3, 1, 0, 0})
           : unit == 3 ? (side == 0 ? HSide{0, 1, 0, 0} : HSide{3, 1, 5, -1})
                       : (side == 0 ? HSide{2, -1, 0, 0} : HSide{3, 1, 0, 0});
}

__device__ __forceinline__ u64 hp_load(const u64* XY, int64_t n, const HSide& sd, int64_t row, int lane) {
    u64 v = XY[(int64_t)sd.i0 * n * 64 + row * 64 + lane];
    if (sd.c0 < 0) v = 0 - v;
    if (sd.c1) {
        const u64 x = XY[(int64_t)sd.i1 * n * 64 + row * 64 + lane];
        v += sd.c1 > 0 ? x : (0 - x);
    }
    return v;
}

// f(0) and F = f(0) + x (f(1) - f(0)) of one side for the wave's 8 pairs, as balanced-digit
// k-octets (row = coefficient lane) in tiles T0 (f(0)) and T1 (F); ev, ov: f(0), f(1).
__device__ __forceinline__ void hp_stash(u64 ev[8], u64 ov[8], int w, int lane, int8_t* T0, int8_t* T1) {
    u64 q[8];
    to_digits(ev, q);
#pragma unroll
    for (int d = 0; d < 8; ++d) *(u64*)(T0 + d * PLANE + w * 512 + lane * 8) = q[d];
#pragma unroll
    for (int pq = 0; pq < 8; ++pq) {
        const u64 e = ev[pq];
        const u64 dd = ov[pq] - e;
        const u64 top = __shfl(dd, 63, 64);
        u64 xd = __shfl_up(dd, 1, 64);
        if (lane == 0) xd = 0;
        if (lane == 0 || lane == 1 || lane == 3 || lane == 4) xd -= top;
        ov[pq] = e + xd;
    }
    to_digits(ov, q);
#pragma unroll
    for (int d = 0; d < 8; ++d) *(u64*)(T1 + d * PLANE + w * 512 + lane * 8) = q[d];
}

template <bool DENSE, int UNIT>
__device__ __forceinline__ void hp_unit(const HPartyArgs& a, int8_t (*T)[8 * PLANE], u64 c0[16], u64 c2[16]) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wy = w >> 1, wx = w & 1, r = lane & 31, kh = (lane >> 5) * 16;
    const int arow = wy * 32 + r, brow = wx * 32 + r;
    constexpr HSide sa = hunit(DENSE, UNIT, 0), sb = hunit(DENSE, UNIT, 1);
    for (int64_t blk = blockIdx.x; blk < a.nblocks; blk += gridDim.x) {
        // both sides' loads first (the block's 8 pairs per wave), then the conversions
        u64 ea[8], oa[8], eb[8], ob[8];
#pragma unroll
        for (int pq = 0; pq < 8; ++pq) {
            const int64_t pr = blk * 32 + w * 8 + pq;
            const bool in = pr < a.npairs;
            ea[pq] = in ? hp_load(a.XY, a.n, sa, 2 * pr, lane) : 0;
            oa[pq] = in ? hp_load(a.XY, a.n, sa, 2 * pr + 1, lane) : 0;
            eb[pq] = in ? hp_load(a.XY, a.n, sb, 2 * pr, lane) : 0;
            ob[pq] = in ? hp_load(a.XY, a.n, sb, 2 * pr + 1, lane) : 0;
        }
        hp_stash(ea, oa, w, lane, T[0], T[1]);
        hp_stash(eb, ob, w, lane, T[2], T[3]);
        __syncthreads();
#pragma unroll
        for (int pt = 0; pt < 2; ++pt) {            // point 0: f(0) products; point 1: F products
            const int8_t* TA = T[pt];
            const int8_t* TB = T[2 + pt];
            v4i A[8], B[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                A[d] = frag<false>(TA + d * PLANE, arow, kh);
                B[d] = frag<false>(TB + d * PLANE, brow, kh);
            }
            // digit planes 2u and 2u + 1 of the product (sums over i + j = s2 of A_i B_j)
            // on two accumulators at a time (two independent MFMA chains), joined in 32 bits
            // and added into the 64-bit sums: a plane sums at most 8 x 32 products of digits
            // in [-128, 127], |acc| <= 2^22, so acc_2u + 2^8 acc_2u+1 < 2^31 in magnitude
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v16i a0 = v16i{0}, a1 = v16i{0};
#pragma unroll
                for (int i = 0; i <= 2 * u + 1; ++i) {
                    if (i <= 2 * u) a0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[i], B[2 * u - i], a0, 0, 0, 0);
                    a1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[i], B[2 * u + 1 - i], a1, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int32_t j = (int32_t)((u32)a0[v] + ((u32)a1[v] << 8));
                    const u64 val = ((u64)(int64_t)j) << (16 * u);
                    if (pt == 0) c0[v] += val;
                    else c2[v] += val;
                }
            }
        }
        __syncthreads();
    }
}

// grid: (G, units): units 5 (dense) or 1 (sparse); each workgroup writes one partial
template <bool DENSE>
__global__ __launch_bounds__(NT, 2) void k_hpair_party(HPartyArgs a) {
    __shared__ __attribute__((aligned(16))) int8_t T[HP_OPS][8 * PLANE];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wy = w >> 1, wx = w & 1;
    const int unit = blockIdx.y;
    u64 c0[16], c2[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) c0[v] = c2[v] = 0;
    if (!DENSE || unit == 0) hp_unit<DENSE, 0>(a, T, c0, c2);
    else if (unit == 1) hp_unit<DENSE, 1>(a, T, c0, c2);
    else if (unit == 2) hp_unit<DENSE, 2>(a, T, c0, c2);
    else if (unit == 3) hp_unit<DENSE, 3>(a, T, c0, c2);
    else hp_unit<DENSE, 4>(a, T, c0, c2);
    // the two sums as 64 x 64 matrices in LDS (row j = coefficient of a, column l = of b)
    u64* M0 = (u64*)T[0];
    u64* M2 = (u64*)T[2];
    const int n = wx * 32 + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int m = wy * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        M0[m * 64 + n] = c0[v];
        M2[m * 64 + n] = c2[v];
    }
    __syncthreads();
    // thread (q, k): rows 16q .. 16q+15 of anti-diagonals k and 64 + k of both matrices
    const int k = t & 63, qq = t >> 6;
    u64 lo0 = 0, hi0 = 0, lo2 = 0, hi2 = 0;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const int j = 16 * qq + jj;
        const int col = j <= k ? k - j : k + 64 - j;
        const u64 x0 = M0[j * 64 + col], x2 = M2[j * 64 + col];
        if (j <= k) { lo0 += x0; lo2 += x2; }
        else { hi0 += x0; hi2 += x2; }
    }
    __syncthreads();
    u64* red = (u64*)T[1];                         // [q][point][lo 64 | hi 64]
    red[(qq * 2 + 0) * 128 + k] = lo0;
    red[(qq * 2 + 0) * 128 + 64 + k] = hi0;
    red[(qq * 2 + 1) * 128 + k] = lo2;
    red[(qq * 2 + 1) * 128 + 64 + k] = hi2;
    __syncthreads();
    // this workgroup's partial: [point][lo 64 | hi 64], thread t = point (t >> 7), word t & 127
    u64 sum = 0;
#pragma unroll
    for (int q2 = 0; q2 < 4; ++q2) sum += red[(q2 * 2 + (t >> 7)) * 128 + (t & 127)];
    a.part[((int64_t)blockIdx.x * gridDim.y + unit) * 256 + t] = sum;
}


// ---------------------------------------------------------------------------
// The fold of a Pi_Reduce round: rows of 128 words are pairs (f(0), f(1)) of 64-word
// elements (the planes stacked), and out = f(0) + (f(1) - f(0)) Z with Z the multiplication
// matrix of the revealed point: f(0) + zeta (f(1) - f(0)) in GR(2^64, 64).  Z's digit tiles
// (two 32-deep k-blocks, from limb_btiles) stay in LDS for the workgroup's whole run over
// 64-row tiles; the A operand f(1) - f(0) is formed while loading and converted to digits,
// and the epilogue adds f(0) (read again, from cache).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT, 2) void k_fold(const u64* XY, int64_t rows, const int8_t* zt, u64* out) {
    __shared__ __attribute__((aligned(16))) int8_t Bs[2 * TILE_BYTES];
    __shared__ __attribute__((aligned(16))) int8_t As[2][8 * PLANE];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wy = w >> 1, wx = w & 1, r = lane & 31, hf = lane >> 5;
    const int arow = wy * 32 + r, brow = wx * 32 + r;
    for (int i = t; i < 2 * TILE_BYTES / 16; i += NT) ((v4i*)Bs)[i] = ((const v4i*)zt)[i];
    __syncthreads();
    const int ra = t >> 2, oa = t & 3;            // A loader: row ra, k-octet oa of each k-block
    const int bread = brow * KB + ((hf ^ swz(brow)) << 4);
    const int aread = arow * KB + ((hf ^ swz(arow)) << 4);
    const int64_t ntiles = (rows + 63) / 64;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * 64;
        const u64* f = XY + min(r0 + ra, rows - 1) * 128;
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            u64 w8[8], q[8];
            const int k0 = kb * 32 + oa * 8;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const ulonglong2 a0 = *(const ulonglong2*)(f + k0 + 2 * h);
                const ulonglong2 a1 = *(const ulonglong2*)(f + 64 + k0 + 2 * h);
                w8[2 * h] = a1.x - a0.x;
                w8[2 * h + 1] = a1.y - a0.y;
            }
            to_digits(w8, q);
            // the row's two 16-byte halves swapped as in the digit tiles (swz), so that the
            // fragment reads of consecutive rows fall on distinct banks
#pragma unroll
            for (int d = 0; d < 8; ++d) *(u64*)(As[kb] + toff(d, ra, oa)) = q[d];
        }
        __syncthreads();
        // f(0) of this lane's outputs, loaded while the matrix cores run
        const int n = wx * 32 + (lane & 31);
        u64 f0v[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t m = r0 + wy * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            f0v[v] = XY[min(m, rows - 1) * 128 + n];
        }
        v16i acc[8];
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) acc[s2] = v16i{0};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            v4i B[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) B[d] = *(const v4i*)(Bs + kb * TILE_BYTES + d * PLANE + bread);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const v4i A = *(const v4i*)(As[kb] + i * PLANE + aread);
#pragma unroll
                for (int s2 = i; s2 < 8; ++s2)
                    acc[s2] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B[s2 - i], acc[s2], 0, 0, 0);
            }
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t m = r0 + wy * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            if (m >= rows) continue;
            u64 val = 0;
#pragma unroll
            for (int s2 = 0; s2 < 8; ++s2) val += ((u64)(int64_t)acc[s2][v]) << (8 * s2);
            out[m * 64 + n] = val + f0v[v];
        }
        __syncthreads();
    }
}

}  // namespace

size_t limb_btiles_bytes(int64_t K, int64_t N) {
    return (size_t)(rup(N, TN) / TN) * (size_t)(rup(K, KB) / KB) * TILE_BYTES;
}

hipError_t limb_btiles(const View& B, int64_t K, int64_t N, int8_t* out, hipStream_t st) {
    const int64_t nkb = rup(K, KB) / KB, rows_pad = rup(N, TN);
    if (K <= 0 || N <= 0) return hipSuccess;
    TileJob job{};
    job.o[0] = opnd(B, 0, true, N);
    job.out[0] = out;
    const int64_t threads = rows_pad * nkb * 4;
    hipLaunchKernelGGL(k_to_tiles, dim3((unsigned)((threads + 255) / 256), 1), dim3(256), 0, st, job, K, nkb, rows_pad);
    return hipGetLastError();
}

int hpair_groups(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n / 2 + 31) / 32, 1024)); }

hipError_t hpair_party(const HPartyArgs& args, hipStream_t st) {
    HPartyArgs a = args;
    a.npairs = a.n / 2;
    a.nblocks = (a.npairs + 31) / 32;
    const int groups = hpair_groups(a.n);
    if (a.nblocks <= 0) return hipErrorInvalidValue;
    if (a.dense)
        hipLaunchKernelGGL(k_hpair_party<true>, dim3((unsigned)groups, 5), dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL(k_hpair_party<false>, dim3((unsigned)groups, 1), dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t fold_rows(const u64* XY, int64_t rows, const int8_t* ztiles, u64* out, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    const int64_t ntiles = (rows + 63) / 64;
    const int groups = (int)std::min<int64_t>(ntiles, 1024);
    hipLaunchKernelGGL(k_fold, dim3((unsigned)groups), dim3(NT), 0, st, XY, rows, ztiles, out);
    return hipGetLastError();
}

bool limb_conv_ok(const GemmArgs& g) {
    if (!g.conv) return false;
    const int np = g.party ? 3 : 1;
    bool ok = g.batch == 1 && g.ws_alloc && g.cC > 0 && g.cC % KB == 0 && g.K == (int64_t)g.cKH * g.cKW * g.cC &&
              g.cOH == g.cH + 2 * g.cpad - g.cKH + 1 && g.cOW == g.cW + 2 * g.cpad - g.cKW + 1 && g.cOH > 0 &&
              g.cOW > 0 && g.cOH < 32768 && g.cOW < 65536 && g.M % ((int64_t)g.cOH * g.cOW) == 0 && g.shared <= 1;
    for (int p = 0; p < np && ok; ++p) ok = ((uintptr_t)g.A[p].p & 15) == 0;
    return ok;
}

// Recorded products per kernel variant (0: <false, 1>, 1: <true, 1>, 2: <true, 2>, 3 and 4:
// the transposed-view kernels with 1 and 2 column tiles, 5 and 6: the implicit lowering),
// their reductions, and the host staging of the device tables.
struct GemmGroup {
    static constexpr int NVAR = 7;
    std::vector<L2Args> args[NVAR];
    std::vector<int> count[NVAR];
    std::vector<RedArgs> red;
    std::vector<char> stage[NVAR + 1];
};

GemmGroup* gemm_group_new() { return new GemmGroup(); }
void gemm_group_free(GemmGroup* g) { delete g; }

hipError_t gemm_group_run(GemmGroup* g, void* (*ws_alloc)(void*, size_t), void* ws_self, hipStream_t st) {
    // a table of n entries of type T, then the n + 1 prefix starts (workgroups rounded up to
    // a multiple of 8, or blocks) and the n counts, copied to the workspace in one transfer
    auto upload = [&](std::vector<char>& h, const void* tab, size_t tbytes, const std::vector<int64_t>& start,
                      const std::vector<int>& cnt, bool wide, char** dev) -> hipError_t {
        const size_t sbytes = start.size() * (wide ? 8 : 4), cbytes = cnt.size() * 4;
        const size_t o1 = (tbytes + 255) & ~(size_t)255, o2 = (o1 + sbytes + 255) & ~(size_t)255;
        h.assign(o2 + cbytes, 0);
        std::memcpy(h.data(), tab, tbytes);
        for (size_t i = 0; i < start.size(); ++i) {
            if (wide) ((int64_t*)(h.data() + o1))[i] = start[i];
            else ((int*)(h.data() + o1))[i] = (int)start[i];
        }
        if (cbytes) std::memcpy(h.data() + o2, cnt.data(), cbytes);
        *dev = (char*)ws_alloc(ws_self, h.size());
        if (!*dev) return hipErrorOutOfMemory;
        return hipMemcpyAsync(*dev, h.data(), h.size(), hipMemcpyHostToDevice, st);
    };
    for (int v = 0; v < GemmGroup::NVAR; ++v) {
        const int n = (int)g->args[v].size();
        if (n == 0) continue;
        std::vector<int64_t> start(n + 1, 0);
        for (int i = 0; i < n; ++i) start[i + 1] = start[i] + (g->count[v][i] + 7) / 8 * 8;
        if (start[n] > 0x7FFFFFFF) return hipErrorInvalidValue;
        char* dev = nullptr;
        hipError_t e = upload(g->stage[v], g->args[v].data(), n * sizeof(L2Args), start, g->count[v], false, &dev);
        if (e != hipSuccess) return e;
        const size_t o1 = (n * sizeof(L2Args) + 255) & ~(size_t)255;
        const size_t o2 = (o1 + (n + 1) * 4 + 255) & ~(size_t)255;
        const L2Args* tab = (const L2Args*)dev;
        const int* sp = (const int*)(dev + o1);
        const int* cp = (const int*)(dev + o2);
        const dim3 gr((unsigned)start[n]);
        switch (v) {
            case 0: hipLaunchKernelGGL((k_lgemm2_group<false, 1>), gr, dim3(NT), 0, st, tab, sp, cp, n); break;
            case 1: hipLaunchKernelGGL((k_lgemm2_group<true, 1>), gr, dim3(NT), 0, st, tab, sp, cp, n); break;
            case 2: hipLaunchKernelGGL((k_lgemm2_group<true, 2>), gr, dim3(2 * NT), 0, st, tab, sp, cp, n); break;
            case 3: hipLaunchKernelGGL((k_lgemm2_group<true, 1, true>), gr, dim3(NT), 0, st, tab, sp, cp, n); break;
            case 4: hipLaunchKernelGGL((k_lgemm2_group<true, 2, true>), gr, dim3(2 * NT), 0, st, tab, sp, cp, n); break;
            case 5:
                hipLaunchKernelGGL((k_lgemm2_group<true, 1, false, true>), gr, dim3(NT), 0, st, tab, sp, cp, n);
                break;
            default:
                hipLaunchKernelGGL((k_lgemm2_group<true, 2, false, true>), gr, dim3(2 * NT), 0, st, tab, sp, cp, n);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        g->args[v].clear();
        g->count[v].clear();
    }
    const int nr = (int)g->red.size();
    if (nr > 0) {
        std::vector<int64_t> start(nr + 1, 0);
        int W = 1;
        for (int i = 0; i < nr; ++i) {
            const RedArgs& r = g->red[i];
            start[i + 1] = start[i] + ((int64_t)r.batch * r.nprod * r.M * r.N + 63) / 64;
            W = std::max(W, std::min(r.splits, 16));
        }
        char* dev = nullptr;
        hipError_t e = upload(g->stage[GemmGroup::NVAR], g->red.data(), nr * sizeof(RedArgs), start, {}, true, &dev);
        if (e != hipSuccess) return e;
        const size_t o1 = (nr * sizeof(RedArgs) + 255) & ~(size_t)255;
        e = split_reduce_group((const RedArgs*)dev, (const int64_t*)(dev + o1), nr, start[nr], W, st);
        if (e != hipSuccess) return e;
        g->red.clear();
    }
    return hipSuccess;
}

hipError_t gemm_limb(const GemmArgs& g, hipStream_t st) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    if (g.conv && !limb_conv_ok(g)) return hipErrorInvalidValue;
    const bool conv = g.conv != 0;
    const int64_t tm = rup(g.M, TM) / TM, tn = rup(g.N, TN) / TN;
    const int64_t Kp = rup(g.K, KB);
    // B pre-converted to digit tiles when every A plane is k-contiguous with one row
    // stride (or a transposed view with contiguous rows) and B is re-read by at least two
    // row tiles, or the caller has converted B already, or one row tile of at least 32
    // rows against one column tile and a long K (the conversion pass costs one more read
    // and write of B, converting in the kernel a load latency per k-block; with fewer A
    // rows B dominates the traffic); two 64-column tiles per workgroup (one workgroup per
    // CU) when rows are aligned, K is whole k-blocks and N spans more than one tile
    const int nprod = g.party ? 3 : (g.shared > 1 ? g.shared : 1);
    const int na = g.party ? 3 : nprod;
    bool kc = (tm >= 2 || (g.btiles && !g.party) || (Kp >= 4096 && tn == 1 && g.M >= 32)) && g.ws_alloc;
    bool ta = kc && g.K % KB == 0;
    for (int p = 0; p < na; ++p) {
        kc = kc && g.A[p].s1 == 1 && g.A[p].s0 == g.A[0].s0;
        ta = ta && g.A[p].s0 == 1 && g.A[p].s1 == g.A[0].s1;   // transposed view, rows contiguous
    }
    if (conv) {
        kc = true;
        ta = false;
    }
    const bool two = kc || ta;
    // Batches with uniform strides (every A plane, every B plane and every output) run in
    // one launch of the converted-B kernel
    bool uni = two && g.batch > 1 && g.batch <= 65535;
    for (int p = 0; p < na; ++p) uni = uni && g.A[p].sb == g.A[0].sb;
    for (int p = 0; p < (g.party ? 3 : 1); ++p) uni = uni && g.B[p].sb == g.B[0].sb;
    for (int p = 0; p < nprod; ++p) uni = uni && g.C[p].sb == g.C[0].sb;
    // Small products stay on the vector ALU, where the launch is cheaper (a uniform batch
    // counts as one launch).
    const double work = (double)g.M * (double)g.N * (double)g.K * (uni ? (double)g.batch : 1.0);
    if ((work < (double)(1 << 22) && !conv) || g.K == 0) return gemm(g, 0, st);
    for (int b = 0; b < g.batch; ++b) {
        LArgs a{};
        a.M = g.M; a.N = g.N; a.K = g.K; a.Kp = Kp;
        a.atomic = g.accumulate ? 1 : 0;
        a.D = g.Dadd;
        if (a.D.p) a.D.p += b * a.D.sb;
        int64_t maxseg;
        if (!g.party) {
            // one product, or up to three A operands against one B (g.shared)
            maxseg = 1;
            for (int p = 0; p < nprod; ++p) {
                Prod& P = a.prod[p];
                P.nseg = 1;
                P.a[0] = opnd(g.A[p], b, false, g.M);
                P.b[0] = opnd(g.B[0], b, true, g.N);
                P.C = g.C[p];
                P.C.p += b * P.C.sb;
            }
        } else {
            // planes 0, 1, 2 = m, [r]_1, [r]_2
            maxseg = 2;
            const View* A = g.A;
            const View* B = g.B;
            // C0 = (A1 + A2)(B1 + B2)
            Prod& P0 = a.prod[0];
            P0.nseg = 1;
            P0.a[0] = combo(A, b, false, g.M, 1, 1, 2, 1);
            P0.b[0] = combo(B, b, true, g.N, 1, 1, 2, 1);
            // C1 = A1 Bm + Am B1
            Prod& P1 = a.prod[1];
            P1.nseg = 2;
            P1.a[0] = combo(A, b, false, g.M, 1, 1, -1, 0);
            P1.b[0] = combo(B, b, true, g.N, 0, 1, -1, 0);
            P1.a[1] = combo(A, b, false, g.M, 0, 1, -1, 0);
            P1.b[1] = combo(B, b, true, g.N, 1, 1, -1, 0);
            // C2 = Am (Bm - B2) + (-A2) Bm
            Prod& P2 = a.prod[2];
            P2.nseg = 2;
            P2.a[0] = combo(A, b, false, g.M, 0, 1, -1, 0);
            P2.b[0] = combo(B, b, true, g.N, 0, 1, 2, -1);
            P2.a[1] = combo(A, b, false, g.M, 2, -1, -1, 0);
            P2.b[1] = combo(B, b, true, g.N, 0, 1, -1, 0);
            for (int p = 0; p < 3; ++p) {
                a.prod[p].C = g.C[p];
                a.prod[p].C.p += b * a.prod[p].C.sb;
            }
        }
        bool fast = ta || (kc && g.K % KB == 0 && g.A[0].s0 % 2 == 0);
        for (int p = 0; p < na && fast && !ta; ++p) fast = ((uintptr_t)(g.A[p].p + b * g.A[p].sb) & 15) == 0;
        if (conv) fast = true;                   // limb_conv_ok: aligned planes, K in whole k-blocks
        const int ns = fast && tn >= 2 && g.lt_ns != 1 ? 2 : 1;
        // K is split when the 64 x 64 tiles number fewer than the CUs (measured: a split costs
        // more than a half-filled second wave) and when it exceeds what the 32-bit digit sums
        // hold.  The splits write partial sums to the workspace and one pass adds them up
        // (atomic adds into the output only for accumulating callers without a workspace).
        // (measured: splitting to fill the last round of 64 x 128 workgroups costs more in
        // partial sums than the idle CUs)
        // a uniform batch: nbl batches from b = 0 in one launch (with 16-byte aligned rows in
        // every batch for the kernels that load A in 16-byte pieces)
        const int64_t nbl = uni && b == 0 && (!fast || ta || g.A[0].sb % 2 == 0) ? g.batch : 1;
        const int64_t groups = tm * tn * nprod, fill = 256;
        const int64_t need = (maxseg * Kp + KSEG - 1) / KSEG;
        int64_t splits = need;
        if (groups < fill && maxseg * Kp >= 2048) {
            const int64_t want = (4 * fill + groups - 1) / groups;
            splits = std::max<int64_t>(splits, std::min<int64_t>(want, maxseg * Kp / 64));
        }
        if (g.lt_split > 1) splits = std::max<int64_t>(splits, std::min<int64_t>(splits * g.lt_split, maxseg * Kp / 64));
        // a grouped product need not fill the GPU alone: at least 1024 of K per split, so
        // that a workgroup's k-loop outweighs its partial-sum tile
        if (g.group) splits = std::max<int64_t>(need, std::min<int64_t>(splits, maxseg * Kp / 1024));
        const size_t plane = (size_t)nprod * g.M * g.N * 8 * nbl;
        const bool part_ok = g.ws_alloc != nullptr && !g.no_part && plane * need <= part_cap(g);
        if (part_ok) splits = std::min<int64_t>(splits, std::max<int64_t>(need, (int64_t)(part_cap(g) / plane)));
        else splits = need;
        if (splits > 1 && !part_ok) {
            // without room for partials: atomic adds, into a zeroed output when the caller
            // does not accumulate (a dense output with nothing added); a batched launch
            // takes the vector-ALU path instead
            if (nbl > 1) return gemm(g, 0, st);
            bool dense = !g.accumulate && !a.D.p;
            for (int p = 0; p < nprod; ++p) dense = dense && a.prod[p].C.s1 == 1 && a.prod[p].C.s0 == g.N;
            if (!g.accumulate && !dense) return gemm(g, 0, st);
            for (int p = 0; p < nprod && !g.accumulate; ++p) {
                hipError_t e = zero_words32(a.prod[p].C.p, 2 * g.M * g.N, st);
                if (e != hipSuccess) return e;
            }
            a.atomic = 1;
        }
        // K blocks never straddle a segment (Kp is a multiple of KB); chunks may
        const int64_t kchunk = rup((maxseg * Kp + splits - 1) / splits, KB);
        splits = (maxseg * Kp + kchunk - 1) / kchunk;
        a.kchunk = kchunk;
        a.splits = (int)splits;
        if (nprod * splits > 65535) return hipErrorInvalidValue;
        a.part = nullptr;
        if (splits > 1 && part_ok) {
            a.part = (u64*)g.ws_alloc(g.ws_self, plane * splits);
            if (!a.part) return hipErrorOutOfMemory;
            a.atomic = 0;
        }
        OutView outs[3];
        for (int p = 0; p < nprod; ++p) outs[p] = a.prod[p].C;
        auto finish = [&]() -> hipError_t {
            hipError_t e = hipGetLastError();
            if (e != hipSuccess || !a.part) return e;
            return split_reduce(a.part, g.M, g.N, nprod, (int)splits, (int)nbl, outs, a.D, g.accumulate, st);
        };
        if (two) {
            const int64_t nkb = Kp / KB, rows_pad = tn * TN;
            if (nkb * 2 > 0x7FFFFFFF || tn * tm * nprod * splits * nbl > 0x7FFFFFFF || nbl > 65535)
                return hipErrorInvalidValue;
            const size_t tbytes = (size_t)tn * nkb * TILE_BYTES;
            // the digit tiles of n B operands (of every batch of the launch) in one launch
            auto tiles = [&](const Opnd* bo, int n, const int8_t** tb) -> bool {
                TileJob job{};
                job.ob = g.B[0].sb;
                job.tb = (int64_t)tbytes;
                for (int i = 0; i < n; ++i) {
                    job.o[i] = bo[i];
                    job.out[i] = (int8_t*)g.ws_alloc(g.ws_self, tbytes * nbl);
                    if (!job.out[i]) return false;
                    tb[i] = job.out[i];
                }
                const int64_t threads = rows_pad * nkb * 4;           // a thread per octet
                hipLaunchKernelGGL(k_to_tiles, dim3((unsigned)((threads + 255) / 256), (unsigned)n, (unsigned)nbl),
                                   dim3(256), 0, st, job, g.K, nkb, rows_pad);
                return true;
            };
            L2Args l{};
            l.M = g.M; l.N = g.N; l.K = g.K;
            l.lda = ta ? 1 : g.A[0].s0;
            l.ldk = ta ? g.A[0].s1 : 1;
            if (conv) {
                l.lda = 0;
                l.cH = g.cH; l.cW = g.cW; l.cC = g.cC; l.cKW = g.cKW; l.cpad = g.cpad;
                l.cOH = g.cOH; l.cOW = g.cOW; l.ccb = g.cC / KB;
            }
            l.nkb = (int)nkb; l.bnkb = (int)nkb; l.kcb = (int)(kchunk / KB); l.nprod = nprod; l.splits = (int)splits;
            l.atomic = a.atomic; l.D = a.D; l.part = a.part;
            l.sbA = g.A[0].sb; l.sbC = g.C[0].sb; l.sbT = (int64_t)tbytes;
            const u64* Ap[3];
            for (int p = 0; p < na; ++p) Ap[p] = g.A[p].p + b * g.A[p].sb;
            if (!g.party) {
                const Opnd bo = opnd(g.B[0], b, true, g.N);
                const int8_t* t0 = nullptr;
                if (g.btiles && g.batch == 1 && g.btiles_nkb >= nkb) {
                    t0 = g.btiles;             // converted by the caller
                    l.bnkb = (int)g.btiles_nkb;
                } else if (!tiles(&bo, 1, &t0)) {
                    return hipErrorOutOfMemory;
                }
                for (int p = 0; p < nprod; ++p) {
                    l.prod[p].nseg = 1;
                    l.prod[p].seg[0] = Seg2{Ap[p], nullptr, t0};
                    l.prod[p].C = a.prod[p].C;
                }
            } else {
                // planes 0, 1, 2 = m, [r]_1, [r]_2; signs and the B sum on the B side:
                //   C0 = (A1 + A2)(B1 + B2)       (one segment over two A planes)
                //   C1 = A1 Bm + Am B1
                //   C2 = Am (Bm - B2) + A2 (-Bm)
                const View* B = g.B;
                const Opnd bos[5] = {combo(B, b, true, g.N, 1, 1, 2, 1), combo(B, b, true, g.N, 0, 1, -1, 0),
                                     combo(B, b, true, g.N, 1, 1, -1, 0), combo(B, b, true, g.N, 0, 1, 2, -1),
                                     combo(B, b, true, g.N, 0, -1, -1, 0)};
                const int8_t* tb[5];
                if (!tiles(bos, 5, tb)) return hipErrorOutOfMemory;
                const int8_t *s12 = tb[0], *bm = tb[1], *b1 = tb[2], *bm2 = tb[3], *nbm = tb[4];
                // (kernels that convert 8 A words per thread take C0 as two segments)
                const bool sum = ns == 2 || !fast;
                const Seg2 segs[3][2] = {{{Ap[1], sum ? Ap[2] : nullptr, s12}, {Ap[2], nullptr, s12}},
                                         {{Ap[1], nullptr, bm}, {Ap[0], nullptr, b1}},
                                         {{Ap[0], nullptr, bm2}, {Ap[2], nullptr, nbm}}};
                for (int p = 0; p < 3; ++p) {
                    l.prod[p].nseg = p == 0 && sum ? 1 : 2;
                    l.prod[p].seg[0] = segs[p][0];
                    l.prod[p].seg[1] = segs[p][1];
                    l.prod[p].C = a.prod[p].C;
                }
            }
            l.tn64 = (int)tn;
            l.tn = (int)((tn + ns - 1) / ns);
            l.tm = (int)tm;
            // B tiles that fit an XCD's L2 with room to spare, or a grid that the CUs hold
            // at once (one workgroup per CU with two column tiles, else two): the products
            // and column groups of one row tile run together and share its A rows (rb = 1);
            // otherwise about as many workgroups per group as one XCD holds at once (32 CUs),
            // sharing B tiles (measured: 2048 x 2304 x 256, 192 workgroups, 5% faster with
            // rb = 1; 32768 x 2304 x 256 5% faster with rb = 16)
            const size_t bbytes = (size_t)(g.party ? 5 : 1) * tn * nkb * TILE_BYTES;
            const int64_t nwg = l.tn * tm * nprod * splits * nbl;
            l.rb = bbytes <= ((size_t)2 << 20) || nwg <= (ns == 2 ? 256 : 512)
                       ? 1
                       : (int)std::max<int64_t>(1, std::min<int64_t>(tm, (ns == 2 ? 32 : 64) / l.tn));
            if (g.lt_rb > 0) l.rb = (int)std::min<int64_t>(g.lt_rb, tm);
            const dim3 gr((unsigned)(l.tn * tm * nprod * splits * nbl));
            if (g.group) {
                // recorded for gemm_group_run (kernel variant, arguments, workgroups, reduction)
                const int vid = conv ? (ns == 2 ? 6 : 5) : ta ? (ns == 2 ? 4 : 3) : ns == 2 ? 2 : fast ? 1 : 0;
                g.group->args[vid].push_back(l);
                g.group->count[vid].push_back((int)gr.x);
                if (a.part) {
                    RedArgs r{};
                    r.part = a.part;
                    r.M = g.M; r.N = g.N; r.nprod = nprod; r.splits = (int)splits; r.batch = (int)nbl;
                    r.atomic = g.accumulate ? 1 : 0;
                    for (int p = 0; p < nprod; ++p) r.C[p] = outs[p];
                    r.D = nprod == 1 ? a.D : View{nullptr, 0, 0, 0};
                    g.group->red.push_back(r);
                }
                if (nbl > 1) return hipSuccess;
                continue;
            }
            const int64_t ntiles = (int64_t)gr.x;
            bool stream = fast && !ta && !conv && ns == 1 && !g.party && nkb <= 2 && splits == 1 && !a.part &&
                          !a.atomic && !a.D.p && ntiles < ((int64_t)1 << 31) && g.M < ((int64_t)1 << 31) &&
                          g.N < ((int64_t)1 << 31);
            for (int p = 0; p < nprod && stream; ++p) {
                const OutView& C = l.prod[p].C;
                stream = C.s0 >= 0 && C.s1 >= 0 && ((TM - 1) * C.s0 + (g.N - 1) * C.s1) * 8 + 8 <= 0x7FFFFFFF;
            }
            const int sg = stream ? stream_grid(ntiles) : 0;
            if (sg > 0 && nkb == 1) hipLaunchKernelGGL(k_lgemm_stream<1>, dim3((unsigned)sg), dim3(NT), 0, st, l, (int)ntiles);
            else if (sg > 0) hipLaunchKernelGGL(k_lgemm_stream<2>, dim3((unsigned)sg), dim3(NT), 0, st, l, (int)ntiles);
            else if (conv && ns == 2) hipLaunchKernelGGL((k_lgemm2<true, 2, false, true>), gr, dim3(2 * NT), 0, st, l);
            else if (conv) hipLaunchKernelGGL((k_lgemm2<true, 1, false, true>), gr, dim3(NT), 0, st, l);
            else if (ta && ns == 2) hipLaunchKernelGGL((k_lgemm2<true, 2, true>), gr, dim3(2 * NT), 0, st, l);
            else if (ta) hipLaunchKernelGGL((k_lgemm2<true, 1, true>), gr, dim3(NT), 0, st, l);
            else if (ns == 2) hipLaunchKernelGGL((k_lgemm2<true, 2>), gr, dim3(2 * NT), 0, st, l);
            else if (fast) hipLaunchKernelGGL((k_lgemm2<true, 1>), gr, dim3(NT), 0, st, l);
            else hipLaunchKernelGGL((k_lgemm2<false, 1>), gr, dim3(NT), 0, st, l);
            hipError_t e = finish();
            if (e != hipSuccess) return e;
            if (nbl > 1) return hipSuccess;     // every batch done
            continue;
        }
        if (tm > 65535) return hipErrorInvalidValue;
        const dim3 grid((unsigned)tn, (unsigned)tm, (unsigned)(nprod * splits));
        const bool ak = a.prod[0].a[0].s_k == 1, bk = a.prod[0].b[0].s_k == 1;
        if (ak && bk) hipLaunchKernelGGL((k_lgemm<true, true>), grid, dim3(NT), 0, st, a);
        else if (ak) hipLaunchKernelGGL((k_lgemm<true, false>), grid, dim3(NT), 0, st, a);
        else if (bk) hipLaunchKernelGGL((k_lgemm<false, true>), grid, dim3(NT), 0, st, a);
        else hipLaunchKernelGGL((k_lgemm<false, false>), grid, dim3(NT), 0, st, a);
        hipError_t e = finish();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace mpc3
