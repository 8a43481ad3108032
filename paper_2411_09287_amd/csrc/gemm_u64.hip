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

template <bool PARTY>
__global__ __launch_bounds__(NT) void k_gemm_u64(GemmArgs g, int ksplit, int64_t kchunk) {
    constexpr int NP = PARTY ? 3 : 1;
    constexpr int NA = PARTY ? 3 : 1;
    __shared__ u64 As[NP][BK][BM];
    __shared__ u64 Bs[NP][BK][BN];
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
        load_b<NP>(Bs, g, b, n0, k0, kend, tid);
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < BK; ++kk) {
            if constexpr (!PARTY) {
                u64 a[4], bb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = As[0][kk][ty * 4 + i];
#pragma unroll
                for (int j = 0; j < 4; ++j) bb[j] = Bs[0][kk][tx * 4 + j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) mac(acc[0][i][j], a[i], bb[j]);
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
                if (!PARTY && !atomic && g.Dadd.p) v += g.Dadd.p[b * g.Dadd.sb + m * g.Dadd.s0 + n * g.Dadd.s1];
                store(g.C[p], b, m, n, v, atomic);
            }
        }
    }
}

}  // namespace

hipError_t gemm_u64(const GemmArgs& g, hipStream_t stream) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    const int64_t tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
    if (tm > 65535) return hipErrorInvalidValue;
    int ksplit = 1;
    if (g.accumulate && g.K > BK) {
        const int64_t tiles = tm * tn * g.batch;
        const int64_t want = (1024 + tiles - 1) / tiles;          // aim for ~1k workgroups
        const int64_t maxs = (g.K + BK - 1) / BK;                  // at least one K step per split
        ksplit = (int)std::max<int64_t>(1, std::min<int64_t>({want, maxs, 4096}));
    }
    int64_t kchunk = (g.K + ksplit - 1) / ksplit;
    kchunk = ((kchunk + BK - 1) / BK) * BK;
    ksplit = (int)((g.K + kchunk - 1) / kchunk);
    if (ksplit < 1) ksplit = 1;
    if ((int64_t)g.batch * ksplit > 65535) return hipErrorInvalidValue;
    dim3 grid((unsigned)tn, (unsigned)tm, (unsigned)(g.batch * ksplit));
    if (g.party)
        hipLaunchKernelGGL(k_gemm_u64<true>, grid, dim3(NT), 0, stream, g, ksplit, kchunk);
    else
        hipLaunchKernelGGL(k_gemm_u64<false>, grid, dim3(NT), 0, stream, g, ksplit, kchunk);
    return hipGetLastError();
}

hipError_t gemm(const GemmArgs& g, int variant, hipStream_t stream) {
    // the row tiles of both backends' two-dimensional grids stay below 65535: taller
    // products run as row slices (A, C and the added D advance by whole rows)
    const int64_t maxm = (int64_t)65535 * 64;
    for (int64_t r0 = 0; r0 < g.M || r0 == 0; r0 += maxm) {
        GemmArgs s = g;
        s.M = std::min(maxm, g.M - r0);
        if (r0) {
            for (int p = 0; p < (g.party ? 3 : 1); ++p) {
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
