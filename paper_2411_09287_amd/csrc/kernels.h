// Launch wrappers for the elementwise, PRG and Galois-ring kernels.
#pragma once
#include "common.h"

namespace mpc3 {

// An additive error on one word of one message (index < 0: inactive).
struct Inj {
    int64_t index;
    u64 e;
};

struct Keys {
    Key k01, k02, k12, kall;
};

// --- Z_{2^64} elementwise steps -------------------------------------------
void launch_fill(u64* out, int64_t n, Key k, Tag t, hipStream_t s);
// out[i] = G(k, t, start + i) for i < n
void launch_fill_at(u64* out, int64_t n, int64_t start, Key k, Tag t, hipStream_t s);
void launch_encode(const double* x, int64_t n, int frac, u64* out, hipStream_t s);
void launch_decode(const u64* v, int64_t n, int frac, double* out, hipStream_t s);
// op_off (nullable): a device word added to the operation id of every keystream tag the
// launch draws (graph replays run under a new id range without re-recording).
void launch_share(const u64* x, int64_t n, Key k1, Tag t1, Key k2, Tag t2, u64* m, u64* r1, u64* r2,
                  hipStream_t s, const u32* op_off = nullptr);
void launch_trunc_pair(int64_t n, int t, const Keys& k, u32 op, Inj g2x, Inj m1z, u64* rxm, u64* rx1,
                       u64* rx2, u64* rzm, u64* rz1, u64* rz2, hipStream_t s, const u32* op_off = nullptr);
void launch_inner_pre(int64_t n, const Keys& k, u32 op, const u64* pm, const u64* p1, const u64* p2,
                      u64* zr1, u64* zr2, u64* g1, hipStream_t s, const u32* op_off = nullptr);
void launch_set_word(u32* p, u32 v, hipStream_t s);
void launch_inner_post(int64_t n, const u64* c0, const u64* c1, const u64* c2, const u64* zr1,
                       const u64* zr2, const u64* g1, Inj g2inj, Inj m1inj, u64* zm, u64* msg_g2,
                       u64* msg_m1, u64* msg_m2, hipStream_t s);
void launch_trunc_shift(int64_t n, int t, const u64* zm, const u64* rzm, const u64* rz1, const u64* rz2,
                        u64* om, u64* o1, u64* o2, hipStream_t s);
void launch_mult(int64_t n, const Keys& k, u32 op, const u64* am, const u64* a1, const u64* a2,
                 const u64* bm, const u64* b1, const u64* b2, Inj g2inj, u64* cm, u64* c1, u64* c2,
                 u64* msg_g2, u64* msg_m1, u64* msg_m2, hipStream_t s);
// Output rows of ld >= KH KW C words: columns KH KW C .. ld-1 are written as 0.  Output
// (oh, ow) reads input (stride oh + kh - pad, stride ow + kw - pad).
void launch_im2col(const u64* x, int B, int H, int W, int C, int KH, int KW, int pad, int64_t ld, u64* out,
                   hipStream_t s, int stride = 1);
// The same for the three share planes in one launch.
void launch_im2col3(const u64* const x[3], int B, int H, int W, int C, int KH, int KW, int pad, int64_t ld,
                    u64* const out[3], hipStream_t s, int stride = 1);
void launch_sumpool2(const u64* x, int B, int H, int W, int C, u64* out, hipStream_t s);

// Pi_InnerVerify of n <= 8 final pairs in one launch (kernels.hip): p[0..2] the x planes,
// p[3..5] the y planes (n x 64 each; a null plane is 0), z the claim share (3 x 64).  Returns
// false (nothing launched) for larger n.
struct InnerVerifyArgs {
    Keys k;
    u32 op, inst;
    int n;
    const u64* p[6];
    const u64* z;
    int inj_m1;            // Delta's P1 -> P2 message: coefficient index or -1
    u64 e_m1;
    u64* log_m1; u64* log_m2; u64* log_g2;
    u64* reveal;           // Delta (64 words)
    int* flag;             // set when Delta is not 0
};
bool launch_inner_verify_small(const InnerVerifyArgs& a, hipStream_t s);

// The x side of a same-padded stride-1 convolution's compressed pairs from its input h
// (B x H x W x C per plane, NHWC): band sums of the positions a shift leaves out, the powers
// r^(o - delta) of the KH KW shifts, and U[k] = (S_c - E) r^(o - delta) (kernels.hip).
struct ConvBandArgs {
    const u64* h[3];       // input planes
    const u64* lo;         // r^n, n < B H W (64 words each)
    int B, H, W, C, pad;
    int nsets;             // 4 pad + 4 pad^2: rows, columns, corner cells
    u64* part;             // chunks x 3 x nsets x C x 64
};
void launch_conv_bands(const ConvBandArgs& a, int chunks, hipStream_t s);
void launch_pow_shifts(const u64* lo, const u64* hi, int64_t L, int64_t e0, int KH, int KW, int W, u64* out,
                       hipStream_t s);
struct ConvXArgs {
    const u64* S;          // 3 x C x 64: sum_n r^n h[n, c]
    const u64* E;          // 3 x nsets x C x 64: the band sums
    const u64* F;          // KH KW x 64: r^(o - delta) per shift
    int KH, KW, C, pad, nsets;
    int64_t K;             // columns of the lowered input (>= KH KW C; the rest are zero)
    u64* U;                // plane p at U + p ustride: K x 64
    int64_t ustride;
};
void launch_conv_x(const ConvXArgs& a, hipStream_t s);

// Many products' steps in one launch each, from tables in device memory (the tables' host
// copies built by the caller; every job independent of the others):
//   r^e for a list of exponents (r^e = r^(L (e / L)) r^(e mod L) from the two power tables)
struct PowJob {
    int64_t e;
    u64* out;              // 64 words
};
void launch_pow_list(const u64* lo, const u64* hi, int64_t L, const PowJob* jobs, int64_t n, hipStream_t s);
//   rows [0, n) of three planes (plane stride pstride) of Q times the element P, in place
struct RowsJob {
    const u64* P;
    u64* Q;
    int64_t n;
};
void launch_gr_scale_rows(const RowsJob* jobs, int njobs, int64_t max_n, int64_t pstride, hipStream_t s);
//   convolutions' band sums (launch_conv_bands per job, chunks per job)
struct BandJob {
    ConvBandArgs a;
    int chunks;
};
void launch_conv_bands_jobs(const BandJob* jobs, int njobs, int max_sets, int max_z, hipStream_t s);
//   convolutions' x sides (launch_conv_x per job)
void launch_conv_x_jobs(const ConvXArgs* jobs, int njobs, int64_t max_k, hipStream_t s);
void launch_rec_check(int64_t n, const u64* r1, Inj r1inj, int* flag, hipStream_t s);
void launch_rec_open(int64_t n, const u64* m, const u64* r1, const u64* r2, const int* flag, u64* out,
                     hipStream_t s);

// --- Galois-ring steps (d = 64; an element is 64 consecutive words) ---------
// v = m - r1 - r2 of a random <.>^{l[x]} drawn with (op, purpose, sub); also keeps the share.
void launch_random_gr(const Keys& k, u32 op, u32 purpose, u32 sub, u64* share3 /* m,r1,r2: 3*64 */,
                      u64* value /* nullable */, u64* log /* nullable */, hipStream_t s);
// Multiplication matrices: W_b row j = v_b * x^j for nb elements v_b = src + b*stride.
void launch_mulmat(const u64* src, int64_t stride, int nb, u64* W, hipStream_t s);
// out[i * nq + j] = P[i] * Q[j] for i < np, j < nq (GR products).
void launch_gr_outer(const u64* P, int64_t np, const u64* Q, int64_t nq, u64* out, hipStream_t s);
// Anti-diagonal fold of 64x64 products and reduction modulo f, nb matrices (stride 4096).
void launch_fold_plain(const u64* C, int nb, u64* out, hipStream_t s);
// out[i] = sum over l < nsum of C[l words + i], i < words.
void launch_sum_blocks(const u64* C, int nsum, int64_t words, u64* out, hipStream_t s);
// r^(e0a + step j) and r^(e0b + step j), j < n, into outa and outb (as launch_pow_ap).
void launch_pow_ap2(const u64* lo, const u64* hi, int64_t L, int64_t e0a, int64_t e0b, int64_t step, int64_t n,
                    u64* outa, u64* outb, hipStream_t s);
// Pi_PolyEvl outputs from the three party products C0, C1, C2 (each 64x64).
struct PolyEvlArgs {
    const u64* C;          // 3 consecutive 64x64 matrices
    Keys k;
    u32 op, pr, pg, sub;
    int inj_m1, inj_g2;    // coefficient index or -1
    u64 e_m1, e_g2;
    u64* out;              // share m, r1, r2 (3*64)
    u64* log_m1; u64* log_m2; u64* log_g2;   // nullable
    u64* reveal;           // nullable: writes the opened value
    int* nonzero_flag;     // nullable: set if the opened value is not 0
    int prefolded;         // C holds the three reduced sums (3*64 words) instead of 64x64 products
};
void launch_polyevl_finish(const PolyEvlArgs& a, hipStream_t s);
// For nc planes of n rows (rows 2i, 2i+1 -> row i): F = f0 + x (f1 - f0).
void launch_at_x(const u64* XY, int nc, int64_t n, u64* F, hipStream_t s);
// [Mat(1 - z); Mat(z)] (128 x 64 words) from Mat(z) (64 x 64).
void launch_mat_pair(const u64* Wz, u64* out, hipStream_t s);
// For nc planes of n rows (rows 2i, 2i+1 -> row i): D = f1 - f0 and F = f0 + x D.
void launch_at_x_diff(const u64* XY, int nc, int64_t n, u64* F, u64* D, hipStream_t s);
struct RoundArgs {
    Keys k;
    u32 op, sub;
    const u64* inv;        // inv_x, inv_1mx, inv_xxm1 (3*64)
    const u64* h0;         // share (3*64)
    const u64* h2;         // share (3*64)
    u64* z;                // share (3*64), updated in place
    u64* zeta_out;         // 64
    u64* log_zeta;         // nullable
    u64* mat_out;          // nullable: multiplication matrix of zeta (64 x 64, row j = zeta x^j)
};
void launch_round_finish(const RoundArgs& a, hipStream_t s);
// Everything of a Pi_Reduce round between the h products and the fold, in one launch: the
// party sums from the partial anti-diagonal sums of hpair_party, both Pi_PolyEvl exchanges, the
// revealed point, the Lagrange step of z and the digit tiles of the point's multiplication
// matrix (the fold's B operand, limb_btiles layout).
struct RoundMidArgs {
    Keys k;
    u32 op, sub;
    const u64* rows;       // the round's nine keystream rows (launch_round_rows)
    const u64* part;       // hpair_party's partials: groups x nunits x 256 words
    int nunits, groups;
    const u64* inv;        // inv_x, inv_1mx, inv_xxm1 (3*64)
    u64* z;                // share (3*64), updated in place
    int inj_h0_m1, inj_h2_g2;   // coefficient index or -1
    u64 e_h0_m1, e_h2_g2;
    u64* log_h0[3];        // m1, m2, g2 of h(0) (nullable)
    u64* log_h2[3];        // m1, m2, g2 of h(x) (nullable)
    u64* log_zeta;         // nullable
    int8_t* ztiles;        // two 32-deep k-blocks of digit tiles (2 x 16 KiB)
};
void launch_round_mid(const RoundMidArgs& a, hipStream_t s);
// The keystream rows of rounds k0 .. k0 + rounds - 1 of verification instance inst (9 x 64
// words per round: both Pi_PolyEvl exchanges' masks and the point's three shares).
void launch_round_rows(const Keys& k, u32 op, u32 inst, int k0, int rounds, u64* out, hipStream_t s);
// x'_i = Pi_Mult over GR of x_i and alpha from the party products (n x 64 each), with fresh masks.
void launch_xp_epilogue(int64_t n, const Keys& k, u32 op, u32 sub, const u64* C0, const u64* C1,
                        const u64* C2, u64* XPm, u64* XP1, u64* XP2, hipStream_t s);
// out[c] = -src[c] for the 3 planes of one element (64 words each, plane stride ps_in/ps_out).
void launch_neg_elem(const u64* src, int64_t ps_in, u64* dst, int64_t ps_out, hipStream_t s);
// Scaled lift: out[c][i] = a_c[i] * P[i] (P: n x 64 power table), 3 planes a_c (any may be null -> 0).
void launch_scale_rows(int64_t n, const u64* a0, const u64* a1, const u64* a2, const u64* P, u64* out,
                       int64_t plane_stride, hipStream_t s);
// Constant-term lift: out[c][i] = (a_c[i], 0, ..., 0).
void launch_lift_rows(int64_t n, const u64* a0, const u64* a1, const u64* a2, u64* out,
                      int64_t plane_stride, hipStream_t s);
// Truncation-gate instance of outputs [lo, lo + T) from their bit words B1, B2 (T each):
// writes the x' r1-plane (scaled by r^g from P), the y r2-plane (lifted) and the gate
// outputs w (3 planes of 2T words).
void launch_trunc_instance2(int64_t lo, int64_t T, int t, const u64* B1, const u64* B2, const u64* P,
                            const u64* rxm, const u64* rx1, const u64* rx2, const u64* rzm, const u64* rz1,
                            const u64* rz2, u64* x1plane, u64* y2plane, u64* w3, hipStream_t s);
void launch_set_one(u64* p, hipStream_t s);   // the ring element 1
// Gate outputs <w> of truncations [lo, lo + T): w3 = 3 planes of 2T words (x-gate, z-gate).
void launch_trunc_w(int64_t lo, int64_t T, int t, const u64* B1, const u64* B2, const u64* rxm, const u64* rx1,
                    const u64* rx2, const u64* rzm, const u64* rz1, const u64* rz2, u64* w3, hipStream_t s);

// Symbolic reduction rounds of truncation gates.  After j folds, element i of gate g is
// x = r^g sum_S alpha[g][i][S] zeta^S and y = sum_S gamma[g][i][S] zeta^S (S a subset of
// the j revealed points, bit b <-> point b+1); 64 coefficients per gate and side.
// Initial coefficients (j = 0): alpha = gate weight * bit of B1, gamma = -bit of B2; level j
// is computed from them directly (B1, B2: the chunk's T words each, G = 2T gates).
// sym_coeffs: the 3 * 3^j power-weight rows of round j (cx row stride ld >= G, zero-padded):
// coefficients of x^e zeta^u for j < sym_points_from(), else values at the points
// {0, 1, inf}^(1 + j) of (x, zeta); interp3 takes rows of such values (here after the
// weighted sums over the gates) to the coefficients.
// sym_level: the level-j alpha and gamma (G x 64 words each).
void launch_sym_coeffs(int j, int64_t G, int64_t ld, int t, const u64* B1, const u64* B2, u64* cx,
                       hipStream_t s);
void launch_sym_level(int j, int64_t G, int t, const u64* B1, const u64* B2, u64* alpha, u64* gamma,
                      hipStream_t s);
void launch_interp3(u64* P, int nvar, hipStream_t s);
int sym_points_from();
// rows out[i] = x^e * in[i] for e = 1, 2 (n rows of 64 words).
void launch_xshift_rows(const u64* in, int64_t n, int e, u64* out, hipStream_t s);
// out[i] = P[i / per] * Q[i] (ring products, one 64-lane group per row), for each of
// `planes` planes of Q and out pstride words apart.
void launch_gr_mul_rows(const u64* P, const u64* Q, int64_t n, int64_t per, u64* out, hipStream_t s, int planes = 1,
                        int64_t pstride = 0);
// One doubling level of a power table: out[len + i] = out[i] * P for i < cnt; Pn = P^2
// when Pn is not null.
void launch_pow_level(u64* out, int64_t len, int64_t cnt, const u64* P, u64* Pn, hipStream_t s);
// out[j] = r^(e0 + j step) for j < n, from lo[i] = r^i (i < L) and hi[q] = r^(L q)
// (every exponent below L times the rows of hi).
void launch_pow_ap(const u64* lo, const u64* hi, int64_t L, int64_t e0, int64_t step, int64_t n, u64* out,
                   hipStream_t s);



}  // namespace mpc3
