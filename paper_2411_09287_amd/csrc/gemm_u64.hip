// Z_{2^64} matrix products on the vector ALU (64-bit integer multiply-accumulate).
//
// Each product a*b mod 2^64 is split as a_lo*b_lo (a 64-bit multiply-add,
// v_mad_u64_u32) plus 2^32 (a_lo*b_hi + a_hi*b_lo), whose low 32 bits are
// accumulated separately and folded in once at the end.
#include <algorithm>

#include "gemm.h"

namespace mpc3 {

hipError_t gemm_limb(const GemmArgs& g, hipStream_t stream);

namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

struct Acc {
    u64 lo;
    u32 x;
};

__device__ __forceinline__ void mac(Acc& c, u64 a, u64 b) {
    const u32 alo = (u32)a, ahi = (u32)(a >> 32), blo = (u32)b, bhi = (u32)(b >> 32);
    c.lo += (u64)alo * (u64)blo;
    c.x += alo * bhi + ahi * blo;
}

__device__ __forceinline__ u64 val(const Acc& c) { return c.lo + ((u64)c.x << 32); }

template <int NP>
__device__ __forceinline__ void load_a(u64 (*As)[BK][BM], const GemmArgs& g, int b, int64_t m0,
                                       int64_t k0, int64_t kend, int tid) {
    const View& v0 = g.A[0];
    if (v0.s1 == 1) {  // k contiguous: each thread reads 4 consecutive k of one row
        const int row = tid >> 2, kq = (tid & 3) * 4;
        const int64_t m = m0 + row;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const View& v = g.A[p];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t k = k0 + kq + q;
                As[p][kq + q][row] = (m < g.M && k < kend) ? v.p[b * v.sb + m * v.s0 + k] : 0;
            }
        }
    } else {  // rows contiguous (or general): each thread reads 4 consecutive rows of one k
        const int kk = tid >> 4, mq = (tid & 15) * 4;
        const int64_t k = k0 + kk;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const View& v = g.A[p];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t m = m0 + mq + q;
                As[p][kk][mq + q] = (m < g.M && k < kend) ? v.p[b * v.sb + m * v.s0 + k * v.s1] : 0;
            }
        }
    }
}

template <int NP>
__device__ __forceinline__ void load_b(u64 (*Bs)[BK][BN], const GemmArgs& g, int b, int64_t n0,
                                       int64_t k0, int64_t kend, int tid) {
    const View& v0 = g.B[0];
    if (v0.s1 == 1) {  // n contiguous
        const int kk = tid >> 4, nq = (tid & 15) * 4;
        const int64_t k = k0 + kk;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const View& v = g.B[p];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t n = n0 + nq + q;
                Bs[p][kk][nq + q] = (n < g.N && k < kend) ? v.p[b * v.sb + k * v.s0 + n] : 0;
            }
        }
    } else {  // k contiguous (or general)
        const int col = tid >> 2, kq = (tid & 3) * 4;
        const int64_t n = n0 + col;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const View& v = g.B[p];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t k = k0 + kq + q;
                Bs[p][kq + q][col] = (n < g.N && k < kend) ? v.p[b * v.sb + k * v.s0 + n * v.s1] : 0;
            }
        }
    }
}

__device__ __forceinline__ void store(const OutView& o, int b, int64_t m, int64_t n, u64 v, bool atomic) {
    u64* p = o.p + b * o.sb + m * o.s0 + n * o.s1;
    if (atomic)
        atomicAdd((unsigned long long*)p, (unsigned long long)v);
    else
        *p = v;
}

// MODE 0: plain; 1: party (three sums from the share planes); 2: three A planes against
// one B (shared right operand), three outputs.
template <int MODE>
__global__ __launch_bounds__(NT) void k_gemm_u64(GemmArgs g, int ksplit, int64_t kchunk, u64* part) {
    constexpr bool PARTY = MODE == 1;
    constexpr int NP = MODE != 0 ? 3 : 1;      // A planes
    constexpr int NB = PARTY ? 3 : 1;          // B planes
    constexpr int NA = MODE != 0 ? 3 : 1;      // accumulators
    __shared__ u64 As[NP][BK][BM];
    __shared__ u64 Bs[NB][BK][BN];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int b = blockIdx.z / ksplit, split = blockIdx.z % ksplit;
    const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
    const int64_t kbeg = split * kchunk;
    const int64_t kend = min(g.K, kbeg + kchunk);

    Acc acc[NA][4][4];
#pragma unroll
    for (int p = 0; p < NA; ++p)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[p][i][j] = Acc{0, 0};

    for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
        load_a<NP>(As, g, b, m0, k0, kend, tid);
        load_b<NB>(Bs, g, b, n0, k0, kend, tid);
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < BK; ++kk) {
            if constexpr (!PARTY) {
                u64 bb[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) bb[j] = Bs[0][kk][tx * 4 + j];
#pragma unroll
                for (int p = 0; p < NA; ++p) {
                    u64 a[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) a[i] = As[p][kk][ty * 4 + i];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) mac(acc[p][i][j], a[i], bb[j]);
                }
            } else {
                u64 am[4], a1[4], ra[4], na2[4], bm[4], b1[4], rb[4], bd[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    am[i] = As[0][kk][ty * 4 + i];
                    a1[i] = As[1][kk][ty * 4 + i];
                    const u64 a2 = As[2][kk][ty * 4 + i];
                    ra[i] = a1[i] + a2;
                    na2[i] = 0 - a2;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    bm[j] = Bs[0][kk][tx * 4 + j];
                    b1[j] = Bs[1][kk][tx * 4 + j];
                    const u64 b2 = Bs[2][kk][tx * 4 + j];
                    rb[j] = b1[j] + b2;
                    bd[j] = bm[j] - b2;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        mac(acc[0][i][j], ra[i], rb[j]);
                        mac(acc[1][i][j], am[i], b1[j]);
                        mac(acc[1][i][j], a1[i], bm[j]);
                        mac(acc[2][i][j], am[i], bd[j]);
                        mac(acc[2][i][j], na2[i], bm[j]);
                    }
            }
        }
        __syncthreads();
    }

    // partial sums (split-K through part): plane (b, split, p) of M x N words
    const bool atomic = g.accumulate;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t m = m0 + ty * 4 + i;
        if (m >= g.M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t n = n0 + tx * 4 + j;
            if (n >= g.N) continue;
#pragma unroll
            for (int p = 0; p < NA; ++p) {
                u64 v = val(acc[p][i][j]);
                if (part) {
                    part[(((int64_t)b * ksplit + split) * NA + p) * g.M * g.N + m * g.N + n] = v;
                    continue;
                }
                if (!PARTY && !atomic && g.Dadd.p) v += g.Dadd.p[b * g.Dadd.sb + m * g.Dadd.s0 + n * g.Dadd.s1];
                store(g.C[p], b, m, n, v, atomic);
            }
        }
    }
}

// Small outputs (M, N <= 64): a workgroup per 4 x 4 output block, its 256 threads splitting K
// (thread t takes k = t, t + 256, ...) and adding their sums in a wave reduction and LDS.
// MODE as for k_gemm_u64.
template <int MODE>
__global__ __launch_bounds__(256) void k_gemm_kpar(GemmArgs g) {
    constexpr bool PARTY = MODE == 1;
    constexpr int NP = MODE != 0 ? 3 : 1;
    constexpr int NB = PARTY ? 3 : 1;
    constexpr int NA = MODE != 0 ? 3 : 1;
    constexpr int NV = NA * 16;
    __shared__ u64 red[4][NV];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int b = blockIdx.z;
    const int64_t m0 = (int64_t)blockIdx.y * 4, n0 = (int64_t)blockIdx.x * 4;
    u64 acc[NA][4][4];
#pragma unroll
    for (int p = 0; p < NA; ++p)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[p][i][j] = 0;
    for (int64_t k = t; k < g.K; k += 256) {
        u64 a[NP][4], bb[NB][4];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const View& v = g.A[p];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a[p][i] = m0 + i < g.M ? v.p[b * v.sb + (m0 + i) * v.s0 + k * v.s1] : 0;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const View& v = g.B[q];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bb[q][j] = n0 + j < g.N ? v.p[b * v.sb + k * v.s0 + (n0 + j) * v.s1] : 0;
        }
        if constexpr (PARTY) {
            // planes 0, 1, 2 = m, [r]_1, [r]_2 (sums as in k_gemm_u64)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[0][i][j] += (a[1][i] + a[2][i]) * (bb[1][j] + bb[2][j]);
                    acc[1][i][j] += a[0][i] * bb[1][j] + a[1][i] * bb[0][j];
                    acc[2][i][j] += a[0][i] * (bb[0][j] - bb[2][j]) - a[2][i] * bb[0][j];
                }
        } else {
#pragma unroll
            for (int p = 0; p < NA; ++p)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[p][i][j] += a[p][i] * bb[0][j];
        }
    }
    // wave sums, then the four waves through LDS
#pragma unroll
    for (int p = 0; p < NA; ++p)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                u64 v = acc[p][i][j];
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
                if (lane == 0) red[w][(p * 4 + i) * 4 + j] = v;
            }
    __syncthreads();
    if (t >= NV) return;
    const int p = t >> 4, i = (t >> 2) & 3, j = t & 3;
    const int64_t m = m0 + i, n = n0 + j;
    if (m >= g.M || n >= g.N) return;
    u64 v = red[0][t] + red[1][t] + red[2][t] + red[3][t];
    if (MODE == 0 && !g.accumulate && g.Dadd.p) v += g.Dadd.p[b * g.Dadd.sb + m * g.Dadd.s0 + n * g.Dadd.s1];
    store(g.C[p], b, m, n, v, g.accumulate);
}

// Block = 64 consecutive output words x W waves: wave w adds the partials of splits w,
// w + W, ... for its 64 words (coalesced 512-byte reads), then the W sums are added in LDS.
__device__ __forceinline__ void split_reduce_block(const RedArgs& r, int64_t blk) {
    __shared__ u64 acc[16][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, W = blockDim.x >> 6;
    const int64_t mn = r.M * r.N;
    const int64_t idx = blk * 64 + lane;
    const bool live = idx < (int64_t)r.batch * r.nprod * mn;
    const int64_t e = idx % mn, bp = idx / mn;
    const int p = (int)(bp % r.nprod);
    const int64_t b = bp / r.nprod;
    u64 v = 0;
    if (live) {
        const u64* q = r.part + (b * r.splits * r.nprod + p) * mn + e;
        const int64_t step = (int64_t)r.nprod * mn;
        int s = w;
        for (; s + 3 * W < r.splits; s += 4 * W)
            v += q[s * step] + q[(s + W) * step] + q[(s + 2 * W) * step] + q[(s + 3 * W) * step];
        for (; s < r.splits; s += W) v += q[s * step];
    }
    acc[w][lane] = v;
    __syncthreads();
    if (w != 0 || !live) return;
    for (int i = 1; i < W; ++i) v += acc[i][lane];
    const int64_t m = e / r.N, n = e % r.N;
    const OutView& o = r.C[p];
    u64* dst = o.p + b * o.sb + m * o.s0 + n * o.s1;
    if (r.atomic) {
        atomicAdd((unsigned long long*)dst, (unsigned long long)v);
    } else {
        if (r.D.p) v += r.D.p[b * r.D.sb + m * r.D.s0 + n * r.D.s1];
        *dst = v;
    }
}

__global__ __launch_bounds__(1024) void k_split_reduce(RedArgs r) { split_reduce_block(r, blockIdx.x); }

// Job j takes blocks start[j] .. start[j + 1] - 1 (the block index decides the job for the
// whole workgroup, so the job's fields are read as scalars).
__global__ __launch_bounds__(1024) void k_split_reduce_group(const RedArgs* tab, const int64_t* start, int n) {
    const int64_t blk = blockIdx.x;
    int j = 0;
    for (int i = 1; i < n; ++i)
        if (start[i] <= blk) j = i;
    split_reduce_block(tab[j], blk - start[j]);
}

// A few rows against a tall operand (up to RD_M rows of A, N <= 64, long K): a workgroup
// per range of kc rows of B (a multiple of 64), lane n for column n; each B row is one
// 512-byte read.  Partial sums of the range at part[(split * M + m) * N + n].
constexpr int RD_M = 8;
struct RowsArgs {
    const u64* a[RD_M];          // row m of A: a[m][k * as1]
    int64_t as1;
    View B;
    int M, N;
    int64_t K, kc;
    u64* part;
};
__device__ __forceinline__ u64 lane_word(u64 v, int i) {       // v of lane i (i wave-uniform)
    const u32 lo = (u32)__builtin_amdgcn_readlane((int)(u32)v, i);
    const u32 hi = (u32)__builtin_amdgcn_readlane((int)(u32)(v >> 32), i);
    return (u64)hi << 32 | lo;
}

// Wave w takes the 64-row pieces kb = k0 + 64 w, k0 + 64 (w + 4), ... of the range: its
// lanes load the piece's A words (one vector load per row of A), then for each of the 64
// rows every lane reads its column of B and takes the A words from the loading lane.
__global__ __launch_bounds__(256) void k_rows_dot(RowsArgs r) {
    __shared__ u64 red[4][RD_M][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t k0 = (int64_t)blockIdx.x * r.kc, k1 = min(r.K, k0 + r.kc);
    const bool col = lane < r.N;
    const u64* bp = r.B.p + lane * r.B.s1;
    const int64_t bs = r.B.s0, as = r.as1;
    u64 acc[RD_M];
#pragma unroll
    for (int m = 0; m < RD_M; ++m) acc[m] = 0;
    for (int64_t kb = k0 + 64 * w; kb < k1; kb += 256) {
        const int n = (int)min((int64_t)64, k1 - kb);
        u64 av[RD_M];
#pragma unroll
        for (int m = 0; m < RD_M; ++m) av[m] = m < r.M && lane < n ? r.a[m][(kb + lane) * as] : 0;
        int i = 0;
        for (; i + 4 <= n; i += 4) {
            u64 b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) b[u] = col ? bp[(kb + i + u) * bs] : 0;
#pragma unroll
            for (int m = 0; m < RD_M; ++m) {
                if (m >= r.M) break;
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[m] += lane_word(av[m], i + u) * b[u];
            }
        }
        for (; i < n; ++i) {
            const u64 b = col ? bp[(kb + i) * bs] : 0;
#pragma unroll
            for (int m = 0; m < RD_M; ++m) {
                if (m >= r.M) break;
                acc[m] += lane_word(av[m], i) * b;
            }
        }
    }
#pragma unroll
    for (int m = 0; m < RD_M; ++m) red[w][m][lane] = acc[m];
    __syncthreads();
    if (w != 0 || !col) return;
    for (int m = 0; m < r.M; ++m)
        r.part[((int64_t)blockIdx.x * r.M + m) * r.N + lane] =
            red[0][m][lane] + red[1][m][lane] + red[2][m][lane] + red[3][m][lane];
}

}  // namespace

hipError_t gemm_u64(const GemmArgs& g, hipStream_t stream) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    if (g.M <= 64 && g.N <= 64 && g.K <= 1024 && g.batch <= 65535) {
        // one output tile: K across the threads of 4 x 4 output blocks
        const dim3 grid((unsigned)((g.N + 3) / 4), (unsigned)((g.M + 3) / 4), (unsigned)g.batch);
        if (g.party) hipLaunchKernelGGL(k_gemm_kpar<1>, grid, dim3(256), 0, stream, g);
        else if (g.shared == 3) hipLaunchKernelGGL(k_gemm_kpar<2>, grid, dim3(256), 0, stream, g);
        else hipLaunchKernelGGL(k_gemm_kpar<0>, grid, dim3(256), 0, stream, g);
        return hipGetLastError();
    }
    const int64_t tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
    if (tm > 65535) return hipErrorInvalidValue;
    // K is split when the output tiles number fewer than the CUs (or the caller accumulates):
    // partial sums to the workspace and one reduction pass, else atomic adds (accumulating
    // callers without a workspace)
    const int nprod = g.party || g.shared == 3 ? 3 : 1;
    const int64_t tiles = tm * tn * g.batch;
    int ksplit = 1;
    const bool part_ok = g.ws_alloc != nullptr && !g.no_part;
    if (g.K > BK && (part_ok || g.accumulate) && (g.accumulate || tiles < 256)) {
        const int64_t want = (1024 + tiles - 1) / tiles;          // aim for ~1k workgroups
        const int64_t maxs = (g.K + BK - 1) / BK;                  // at least one K step per split
        int64_t cap = 4096;
        if (part_ok) cap = std::min<int64_t>(cap, (int64_t)(part_cap(g) / ((size_t)nprod * g.M * g.N * 8 * g.batch)));
        ksplit = (int)std::max<int64_t>(1, std::min<int64_t>({want, maxs, cap}));
    }
    int64_t kchunk = (g.K + ksplit - 1) / ksplit;
    kchunk = ((kchunk + BK - 1) / BK) * BK;
    ksplit = (int)((g.K + kchunk - 1) / kchunk);
    if (ksplit < 1) ksplit = 1;
    if ((int64_t)g.batch * ksplit > 65535) return hipErrorInvalidValue;
    u64* part = nullptr;
    if (ksplit > 1 && part_ok) {
        part = (u64*)g.ws_alloc(g.ws_self, (size_t)g.batch * ksplit * nprod * g.M * g.N * 8);
        if (!part) return hipErrorOutOfMemory;
    }
    dim3 grid((unsigned)tn, (unsigned)tm, (unsigned)(g.batch * ksplit));
    if (g.party)
        hipLaunchKernelGGL(k_gemm_u64<1>, grid, dim3(NT), 0, stream, g, ksplit, kchunk, part);
    else if (g.shared == 3)
        hipLaunchKernelGGL(k_gemm_u64<2>, grid, dim3(NT), 0, stream, g, ksplit, kchunk, part);
    else
        hipLaunchKernelGGL(k_gemm_u64<0>, grid, dim3(NT), 0, stream, g, ksplit, kchunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !part) return e;
    return split_reduce(part, g.M, g.N, nprod, ksplit, g.batch, g.C, g.Dadd, g.accumulate, stream);
}

__global__ __launch_bounds__(256) void k_zero32(uint32_t* p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = 0;
}
__global__ __launch_bounds__(256) void k_zero128(uint4* p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

hipError_t zero_words32(void* p, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    uint32_t* w = (uint32_t*)p;
    // 32-bit words up to a 16-byte boundary, 16-byte stores for the body, 32-bit words for the tail
    int64_t head = (int64_t)(((16 - ((uintptr_t)w & 15)) & 15) / 4);
    if (head > n) head = n;
    const int64_t body = (n - head) / 4, tail = n - head - 4 * body;
    if (head) hipLaunchKernelGGL(k_zero32, dim3(1), dim3(256), 0, stream, w, head);
    if (body) {
        const int64_t blocks = std::min<int64_t>((body + 255) / 256, 16384);
        hipLaunchKernelGGL(k_zero128, dim3((unsigned)blocks), dim3(256), 0, stream, (uint4*)(w + head), body);
    }
    if (tail) hipLaunchKernelGGL(k_zero32, dim3(1), dim3(256), 0, stream, w + head + 4 * body, tail);
    return hipGetLastError();
}

hipError_t split_reduce(const u64* part, int64_t M, int64_t N, int nprod, int splits, int batch,
                        const OutView* C, const View& D, bool atomic, hipStream_t stream) {
    RedArgs r{};
    r.part = part;
    r.M = M; r.N = N; r.nprod = nprod; r.splits = splits; r.batch = batch; r.atomic = atomic ? 1 : 0;
    for (int p = 0; p < nprod; ++p) r.C[p] = C[p];
    r.D = nprod == 1 ? D : View{nullptr, 0, 0, 0};
    const int64_t n = (int64_t)batch * nprod * M * N;
    if (n == 0) return hipSuccess;
    if ((n + 63) / 64 > 0x7FFFFFFF) return hipErrorInvalidValue;
    const int W = std::min(splits, 16);
    hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)((n + 63) / 64)), dim3(64 * W), 0, stream, r);
    return hipGetLastError();
}

hipError_t split_reduce_group(const RedArgs* tab, const int64_t* start, int n, int64_t nblk, int W,
                              hipStream_t stream) {
    if (n <= 0 || nblk <= 0) return hipSuccess;
    if (nblk > 0x7FFFFFFF || W < 1 || W > 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_split_reduce_group, dim3((unsigned)nblk), dim3(64 * W), 0, stream, tab, start, n);
    return hipGetLastError();
}


// Plain or shared products with at most RD_M rows of A in all, N <= 64 and a long K
// (A planes with one k stride): k_rows_dot over about 1024 ranges of K, then the split
// reduction (which adds D, or adds into C with atomics when accumulating).
static bool rows_fit(const GemmArgs& g) {
    const int na = std::max(1, g.shared);
    if (g.party || g.M <= 0 || g.M * na > RD_M || g.N <= 0 || g.N > 64 || g.K <= 1024 || !g.ws_alloc || g.no_part)
        return false;
    for (int p = 1; p < na; ++p)
        if (g.A[p].s1 != g.A[0].s1) return false;
    const int64_t kc = std::max<int64_t>(256, ((g.K + 1023) / 1024 + 63) / 64 * 64);
    return (size_t)((g.K + kc - 1) / kc) * (size_t)(g.M * na * g.N) * 8 <= part_cap(g);
}
static hipError_t gemm_rows(const GemmArgs& g, hipStream_t stream) {
    const int na = std::max(1, g.shared);
    const int64_t kc = std::max<int64_t>(256, ((g.K + 1023) / 1024 + 63) / 64 * 64);
    const int64_t splits = (g.K + kc - 1) / kc;
    if (splits > 0x7FFFFFFF) return hipErrorInvalidValue;
    for (int b = 0; b < g.batch; ++b) {
        RowsArgs r{};
        r.M = (int)(g.M * na);
        r.N = (int)g.N;
        r.K = g.K;
        r.kc = kc;
        r.as1 = g.A[0].s1;
        for (int p = 0; p < na; ++p)
            for (int64_t m = 0; m < g.M; ++m) r.a[p * g.M + m] = g.A[p].p + b * g.A[p].sb + m * g.A[p].s0;
        r.B = g.B[0];
        r.B.p += b * r.B.sb;
        r.part = (u64*)g.ws_alloc(g.ws_self, (size_t)splits * r.M * g.N * 8);
        if (!r.part) return hipErrorOutOfMemory;
        View D = g.Dadd;
        if (D.p) D.p += b * D.sb;
        OutView C[3];
        for (int p = 0; p < na; ++p) {
            C[p] = g.C[p];
            C[p].p += b * C[p].sb;
        }
        hipLaunchKernelGGL(k_rows_dot, dim3((unsigned)splits), dim3(256), 0, stream, r);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = split_reduce(r.part, g.M, g.N, na, (int)splits, 1, C, D, g.accumulate, stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t gemm(const GemmArgs& g, int variant, hipStream_t stream) {
    if (g.shared > 1 && (g.party || g.shared > 3 || g.Dadd.p)) return hipErrorInvalidValue;
    // the implicit lowering of a convolution exists in the limb kernel only
    if (g.conv) return variant == 1 ? gemm_limb(g, stream) : hipErrorInvalidValue;
    // a few rows against a long K: one pass over B at full bandwidth, whichever backend
    if (rows_fit(g)) return gemm_rows(g, stream);
    // one small output tile: the K-parallel kernel, whichever backend was asked for (both
    // give the exact result)
    if (g.M <= 64 && g.N <= 64 && g.K <= 1024 && g.shared != 2) return gemm_u64(g, stream);
    if (variant == 0 && g.shared == 2) {
        // the vector-ALU kernel takes the shared-B products one at a time
        for (int p = 0; p < g.shared; ++p) {
            GemmArgs s = g;
            s.shared = 0;
            s.A[0] = g.A[p];
            s.C[0] = g.C[p];
            hipError_t e = gemm(s, 0, stream);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    // the row tiles of both backends' two-dimensional grids stay below 65535: taller
    // products run as row slices (A, C and the added D advance by whole rows)
    const int64_t maxm = (int64_t)65535 * 64;
    for (int64_t r0 = 0; r0 < g.M || r0 == 0; r0 += maxm) {
        GemmArgs s = g;
        s.M = std::min(maxm, g.M - r0);
        if (r0) {
            for (int p = 0; p < (g.party ? 3 : std::max(1, g.shared)); ++p) {
                s.A[p].p += r0 * g.A[p].s0;
                s.C[p].p += r0 * g.C[p].s0;
            }
            if (s.Dadd.p) s.Dadd.p += r0 * g.Dadd.s0;
        }
        hipError_t e = variant != 0 ? gemm_limb(s, stream) : gemm_u64(s, stream);
        if (e != hipSuccess || g.M <= 0) return e;
    }
    return hipSuccess;
}

}  // namespace mpc3
