// Z_{2^64} matrix products on int8 MFMA (gfx950).
//
// Every 64-bit word is written in balanced radix 2^8: a = sum_{i<8} 2^{8i} a_i with
// a_i in [-128, 127].  Modulo 2^64 only the digit pairs with i + j <= 7 survive, so
//     A B = sum_{s<8} 2^{8s} P_s,   P_s = sum_{i+j=s} A_i B_j,
// 36 int8 matrix products accumulated into 8 int32 planes.  |P_s| <= K 8 2^14, so the
// int32 planes are folded into 64-bit partial sums every 8192 of K.  The result is
// bit-identical to the 64-bit integer product.
#include "gemm.h"

namespace mpc3 {

hipError_t gemm_u64(const GemmArgs& g, hipStream_t stream);

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int TM = 64, TN = 64, KB = 32, KSEG = 8192;

inline int64_t rup(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Source of a digit conversion: v(r, k) = sum_i c_i P_i[r*s_r + k*s_k] (up to 3 planes).
struct DigitSrc {
    const u64* p[3];
    int c[3];
    int64_t s_r, s_k;
};

// dst[d*plane + r*ld + koff + k]: balanced digit d of v(r, k); zero for r >= rows or k >= K.
// One thread converts 16 consecutive k of one row.
__global__ void k_digits(DigitSrc s, int64_t rows, int64_t K, int64_t Rp, int64_t nch, int8_t* dst,
                         int64_t plane, int64_t ld, int64_t koff, int kfast) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Rp * nch) return;
    int64_t r, ch;
    if (kfast) { r = idx / nch; ch = idx - r * nch; }
    else { ch = idx / Rp; r = idx - ch * Rp; }
    u32 out[8][4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        u32 pk[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t k = ch * 16 + w * 4 + b;
            u64 v = 0;
            if (r < rows && k < K) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    if (s.c[i]) {
                        const u64 x = s.p[i][r * s.s_r + k * s.s_k];
                        v += s.c[i] > 0 ? x : (0 - x);
                    }
            }
            int carry = 0;
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int x = (int)((v >> (8 * d)) & 0xFF) + carry;
                carry = x >= 128;
                x -= carry << 8;
                pk[d] |= ((u32)(x & 0xFF)) << (8 * b);
            }
        }
#pragma unroll
        for (int d = 0; d < 8; ++d) out[d][w] = pk[d];
    }
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        v4i q;
        q.x = (int)out[d][0]; q.y = (int)out[d][1]; q.z = (int)out[d][2]; q.w = (int)out[d][3];
        *(v4i*)(dst + d * plane + r * ld + koff + ch * 16) = q;
    }
}

struct LArgs {
    const int8_t* A8;
    int64_t a_plane, lda;
    const int8_t* B8;
    int64_t b_plane, ldb;
    int64_t M, N, Kc;           // Kc: contraction length (multiple of 32)
    int64_t kchunk;             // per split (multiple of 32)
    OutView C;
    View D;
    int atomic;
};

__device__ __forceinline__ void flush(u64 part[16], v16i acc[8]) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        u64 t = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) t += ((u64)(int64_t)acc[s][v]) << (8 * s);
        part[v] += t;
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[s] = v16i{0};
}

__global__ __launch_bounds__(256) void k_lgemm(LArgs a) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t m0 = (int64_t)blockIdx.y * TM + (w >> 1) * 32;
    const int64_t n0 = (int64_t)blockIdx.x * TN + (w & 1) * 32;
    const int r = lane & 31, kh = (lane >> 5) * 16;
    const int64_t kbeg = (int64_t)blockIdx.z * a.kchunk;
    const int64_t kend = min(a.Kc, kbeg + a.kchunk);
    const int8_t* ap = a.A8 + (m0 + r) * a.lda + kh;
    const int8_t* bp = a.B8 + (n0 + r) * a.ldb + kh;
    v16i acc[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[s] = v16i{0};
    u64 part[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) part[v] = 0;
    int64_t since = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += KB) {
        v4i A[8], B[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            A[d] = *(const v4i*)(ap + d * a.a_plane + k0);
            B[d] = *(const v4i*)(bp + d * a.b_plane + k0);
        }
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
            for (int i = 0; i <= s; ++i)
                acc[s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[i], B[s - i], acc[s], 0, 0, 0);
        since += KB;
        if (since == KSEG) {
            flush(part, acc);
            since = 0;
        }
    }
    flush(part, acc);
    // 32x32 accumulator layout: lane -> column (lane & 31); register v -> row
    // 8 (v >> 2) + 4 (lane >> 5) + (v & 3)
    const int64_t n = n0 + (lane & 31);
    if (n >= a.N) return;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int64_t m = m0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (m >= a.M) continue;
        u64* p = a.C.p + m * a.C.s0 + n * a.C.s1;
        u64 val = part[v];
        if (a.atomic) {
            atomicAdd((unsigned long long*)p, (unsigned long long)val);
        } else {
            if (a.D.p) val += a.D.p[m * a.D.s0 + n * a.D.s1];
            *p = val;
        }
    }
}

struct Planes {
    int8_t* p;
    int64_t plane, ld;
};

// Convert rows x K (view with strides) into digit planes at k offset koff.
void digits(const DigitSrc& s, int64_t rows, int64_t K, const Planes& P, int64_t Rp, int64_t Kp, int64_t koff,
            hipStream_t st) {
    const int64_t nch = Kp / 16;
    const int64_t work = Rp * nch;
    const int kfast = s.s_k == 1 ? 1 : 0;
    hipLaunchKernelGGL(k_digits, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st, s, rows, K, Rp, nch, P.p,
                       P.plane, P.ld, koff, kfast);
}

DigitSrc src1(const View& v, int64_t b, bool transpose) {
    DigitSrc s{};
    s.p[0] = v.p + b * v.sb;
    s.c[0] = 1;
    s.s_r = transpose ? v.s1 : v.s0;
    s.s_k = transpose ? v.s0 : v.s1;
    return s;
}

DigitSrc combo(const View* v, int64_t b, bool transpose, int c0, int c1, int c2) {
    DigitSrc s{};
    const int cs[3] = {c0, c1, c2};
    for (int i = 0; i < 3; ++i) {
        s.p[i] = v[i].p ? v[i].p + b * v[i].sb : nullptr;
        s.c[i] = v[i].p ? cs[i] : 0;
    }
    s.s_r = transpose ? v[0].s1 : v[0].s0;
    s.s_k = transpose ? v[0].s0 : v[0].s1;
    return s;
}

hipError_t launch_lgemm(const Planes& A, const Planes& B, int64_t M, int64_t N, int64_t Kc, const OutView& C,
                        const View& D, bool atomic, hipStream_t st) {
    const int64_t tm = rup(M, TM) / TM, tn = rup(N, TN) / TN;
    if (tm > 65535) return hipErrorInvalidValue;
    int64_t splits = 1;
    if (atomic) {
        const int64_t tiles = tm * tn;
        const int64_t want = (1024 + tiles - 1) / tiles;
        splits = std::max<int64_t>(1, std::min<int64_t>(want, Kc / 256));
    }
    int64_t kchunk = rup((Kc + splits - 1) / splits, KB);
    splits = (Kc + kchunk - 1) / kchunk;
    if (splits < 1) splits = 1;
    LArgs a{A.p, A.plane, A.ld, B.p, B.plane, B.ld, M, N, Kc, kchunk, C, D, atomic ? 1 : 0};
    hipLaunchKernelGGL(k_lgemm, dim3((unsigned)tn, (unsigned)tm, (unsigned)splits), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t gemm_limb(const GemmArgs& g, hipStream_t st) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    // Small products stay on the vector ALU: the digit conversions would dominate.
    if ((double)g.M * (double)g.N * (double)g.K < (double)(1 << 22) || !g.ws_alloc) return gemm_u64(g, st);
    if (g.K == 0) return gemm_u64(g, st);
    const int64_t Mp = rup(g.M, TM), Np = rup(g.N, TN), Kp = rup(g.K, KB);
    for (int b = 0; b < g.batch; ++b) {
        if (!g.party) {
            Planes A{(int8_t*)g.ws_alloc(g.ws_self, (size_t)8 * Mp * Kp), Mp * Kp, Kp};
            Planes B{(int8_t*)g.ws_alloc(g.ws_self, (size_t)8 * Np * Kp), Np * Kp, Kp};
            digits(src1(g.A[0], b, false), g.M, g.K, A, Mp, Kp, 0, st);
            digits(src1(g.B[0], b, true), g.N, g.K, B, Np, Kp, 0, st);
            OutView C = g.C[0];
            C.p += b * C.sb;
            View D = g.Dadd;
            if (D.p) D.p += b * D.sb;
            hipError_t e = launch_lgemm(A, B, g.M, g.N, Kp, C, D, g.accumulate, st);
            if (e != hipSuccess) return e;
        } else {
            // A segments along k: [A1 | Am | -A2 | A1 + A2]
            const int64_t lda = 4 * Kp;
            Planes A{(int8_t*)g.ws_alloc(g.ws_self, (size_t)8 * Mp * lda), Mp * lda, lda};
            const View* av = g.A;
            digits(combo(av, b, false, 0, 1, 0), g.M, g.K, A, Mp, Kp, 0, st);
            digits(combo(av, b, false, 1, 0, 0), g.M, g.K, A, Mp, Kp, Kp, st);
            digits(combo(av, b, false, 0, 0, -1), g.M, g.K, A, Mp, Kp, 2 * Kp, st);
            digits(combo(av, b, false, 0, 1, 1), g.M, g.K, A, Mp, Kp, 3 * Kp, st);
            const View* bv = g.B;
            // C1 = A1 Bm + Am B1 ; C2 = Am (Bm - B2) + (-A2) Bm ; C0 = (A1 + A2)(B1 + B2)
            Planes B1{(int8_t*)g.ws_alloc(g.ws_self, (size_t)8 * Np * 2 * Kp), Np * 2 * Kp, 2 * Kp};
            Planes B2{(int8_t*)g.ws_alloc(g.ws_self, (size_t)8 * Np * 2 * Kp), Np * 2 * Kp, 2 * Kp};
            Planes B0{(int8_t*)g.ws_alloc(g.ws_self, (size_t)8 * Np * Kp), Np * Kp, Kp};
            digits(combo(bv, b, true, 1, 0, 0), g.N, g.K, B1, Np, Kp, 0, st);
            digits(combo(bv, b, true, 0, 1, 0), g.N, g.K, B1, Np, Kp, Kp, st);
            digits(combo(bv, b, true, 1, 0, -1), g.N, g.K, B2, Np, Kp, 0, st);
            digits(combo(bv, b, true, 1, 0, 0), g.N, g.K, B2, Np, Kp, Kp, st);
            digits(combo(bv, b, true, 0, 1, 1), g.N, g.K, B0, Np, Kp, 0, st);
            const View noD{nullptr, 0, 0, 0};
            OutView C0 = g.C[0], C1 = g.C[1], C2 = g.C[2];
            C0.p += b * C0.sb; C1.p += b * C1.sb; C2.p += b * C2.sb;
            Planes A1m{A.p, A.plane, A.ld}, Amn{A.p + Kp, A.plane, A.ld}, As{A.p + 3 * Kp, A.plane, A.ld};
            hipError_t e = launch_lgemm(A1m, B1, g.M, g.N, 2 * Kp, C1, noD, g.accumulate, st);
            if (e == hipSuccess) e = launch_lgemm(Amn, B2, g.M, g.N, 2 * Kp, C2, noD, g.accumulate, st);
            if (e == hipSuccess) e = launch_lgemm(As, B0, g.M, g.N, Kp, C0, noD, g.accumulate, st);
            if (e != hipSuccess) return e;
        }
    }
    return hipGetLastError();
}

}  // namespace mpc3
