/*
 * mpc3.h -- three-party secure linear-function evaluation over Z_{2^64}
 * (Lu, Zhang, Li, Ren, arXiv 2411.09287) on one MI355X.
 *
 * All three parties P0, P1, P2 run in one process on one GPU.  A "sent" message
 * is a device buffer; its size is counted per (phase, sender, receiver) and
 * nothing is transmitted.  Ring arithmetic is uint64 with wrap-around.
 *
 * Shares (Preliminaries, "<.>-sharing"): a shared value v is held as three
 * planes m, r1, r2 with m = v + r1 + r2.  P1 holds (m, r1), P2 holds (m, r2),
 * P0 holds (r1, r2).  Verification runs in the Galois ring
 * GR(2^64, d) = Z_{2^64}[x] / (x^64 + x^4 + x^3 + x + 1) (Sec. 3), whose
 * elements are d = 64 uint64 coefficients, x^0 first.
 *
 * Conventions for every entry point:
 *   - Pointers named *_dev are device pointers (hipMalloc'd or torch tensors
 *     used as raw 64-bit storage) owned by the caller.  The library never
 *     frees caller memory.  Matrices are row-major and dense (rows x cols).
 *   - Calls are asynchronous on the context's HIP stream unless stated.
 *     mpc3_verify, mpc3_reconstruct and mpc3_comm_stats synchronise.
 *   - Return value: MPC3_OK or a negative MPC3_E_* code.  After a failed
 *     verification every call returns MPC3_E_ABORTED (security with abort,
 *     Sec. 2 "Security Model").
 *   - The context keeps pointers to the operands of every product until it
 *     is verified: keep X, W, Z and truncation-pair planes alive and
 *     unmodified until mpc3_verify has covered them.
 */
#ifndef MPC3_H
#define MPC3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpc3_ctx mpc3_ctx;

/* <v> as three device planes of rows*cols uint64 each (m, [r]_1, [r]_2). */
typedef struct {
    uint64_t *m, *r1, *r2;
    int64_t rows, cols;
} mpc3_share_t;

/* Truncation pair of Pi_Trunc^t (Fig. "The maliciously secure truncation
 * protocol"): <r_x> and <r_z> = <ash(r_x, t)> for n outputs.  The caller
 * allocates the six planes (n words each); mpc3_trunc_pair fills them and id. */
typedef struct {
    mpc3_share_t rx, rz;
    int32_t t;
    int64_t n;
    uint64_t id;
} mpc3_trunc_pair_t;

/* Bytes per [phase][sender][receiver] and communication rounds per phase. */
typedef struct {
    uint64_t bytes[4][3][3];
    uint32_t rounds[4];
} mpc3_comm;

enum {
    MPC3_OK = 0,
    MPC3_E_ARG = -1,        /* null pointer or out-of-range parameter */
    MPC3_E_SHAPE = -2,      /* operand shapes do not match */
    MPC3_E_NOMEM = -3,      /* device allocation failed */
    MPC3_E_ABORTED = -4,    /* a verification failed or Pi_Rec saw inconsistent shares */
    MPC3_E_UNVERIFIED = -5, /* reconstruct requested while products await verification */
    MPC3_E_HIP = -6,        /* a HIP runtime call failed */
    MPC3_E_STATE = -7,      /* call not valid in the current state */
    MPC3_E_LIMIT = -8       /* operands exceed the fixed workspace of mpc3_inner_static */
};

enum { MPC3_VARIANT_U64 = 0, MPC3_VARIANT_LIMB_I8 = 1, MPC3_VARIANT_AUTO = 2 };

/* Phases of the communication counters. */
enum { MPC3_PH_OFFLINE = 0, MPC3_PH_ONLINE = 1, MPC3_PH_VERIFY_OFFLINE = 2, MPC3_PH_VERIFY_ONLINE = 3 };

/* Kinds of pending products, for mpc3_verify's selection mask.  NONLINEAR: the edaBit
 * inner products and the Boolean triples of mpc3_edabits / mpc3_relu / mpc3_maxpool2 (their
 * Pi_Mult triples over Z_{2^64} are of kind MULT). */
enum { MPC3_VERIFY_INNER = 1, MPC3_VERIFY_TRUNC = 2, MPC3_VERIFY_MULT = 4, MPC3_VERIFY_NONLINEAR = 8,
       MPC3_VERIFY_ALL = 15 };

/* Message sites for mpc3_inject (an additive error on one word of one message). */
enum {
    MPC3_SITE_INNER_GAMMA2 = 1,  /* P0 -> P2 [Gamma]_2 of Pi_Inner; index = output element */
    MPC3_SITE_INNER_M1 = 2,      /* P1 -> P2 [m_Z]_1 of Pi_Inner; index = output element */
    MPC3_SITE_TRUNC_GAMMA2 = 3,  /* P0 -> P2 [Gamma]_2 of the r_x product of Pi_Trunc; index = output */
    MPC3_SITE_TRUNC_M1 = 4,      /* P1 -> P2 [m]_1 of the r_z product of Pi_Trunc; index = output */
    MPC3_SITE_MULT_GAMMA2 = 5,   /* P0 -> P2 [Gamma]_2 of Pi_Mult; index = element */
    MPC3_SITE_VER_H0_M1 = 6,     /* P1 -> P2 [m]_1 of h(0) in Pi_Reduce; index = inst<<16 | round<<8 | coeff */
    MPC3_SITE_VER_H2_GAMMA2 = 7, /* P0 -> P2 [Gamma]_2 of h(x) in Pi_Reduce; same index layout */
    MPC3_SITE_VER_DELTA_M1 = 8,  /* P1 -> P2 [m]_1 of Delta in Pi_InnerVerify; index = inst<<16 | coeff */
    MPC3_SITE_REC_R1 = 9,        /* P0 -> P2 [r]_1 in Pi_Rec of mpc3_reconstruct; index = element */
    MPC3_SITE_AND_GAMMA2 = 10,   /* P0 -> P2 [Gamma]_2 of a Boolean Pi_Mult; index = word, e XORed */
    MPC3_SITE_EDA_W_M1 = 11      /* P1 -> P2 [m]_1 of an edaBit inner product; index = edaBit */
};

/* Messages of the most recent Pi_Inner / Pi_Mult, for mpc3_message. */
enum { MPC3_MSG_GAMMA2 = 0, MPC3_MSG_M1 = 1, MPC3_MSG_M2 = 2 };

/* Public transcript slots of one verification instance, for mpc3_verify_log.
 * Each slot is d words.  Round-indexed slots take round = 0 .. R-1. */
enum {
    MPC3_LOG_R = 0,          /* revealed challenge r of Pi_Tran / Pi_BIVerify */
    MPC3_LOG_Z = 1,          /* claimed <z> after the power-weighted sum, m plane */
    MPC3_LOG_ZETA = 2,       /* revealed point of round k */
    MPC3_LOG_H0_M1 = 3, MPC3_LOG_H0_M2 = 4, MPC3_LOG_H0_G2 = 5,
    MPC3_LOG_H2_M1 = 6, MPC3_LOG_H2_M2 = 7, MPC3_LOG_H2_G2 = 8,
    MPC3_LOG_DELTA = 9,      /* revealed Delta of Pi_InnerVerify */
    MPC3_LOG_DELTA_M1 = 10, MPC3_LOG_DELTA_M2 = 11, MPC3_LOG_DELTA_G2 = 12
};

/* Context: seeds eta_01, eta_02, eta_12 (and an all-party seed for inputs
 * owned by P1 or P2) are SHA-256(master_seed || "eta" || ids).  d must be 64.
 * frac_bits is the fixed-point precision (13).  workspace_bytes sizes the
 * initial device arena (0 = grow on demand).  hip_stream is a hipStream_t or
 * NULL for the default stream.  Preliminaries, "Notation" and "Secret sharing". */
int mpc3_ctx_create(const uint8_t master_seed[32], int d, int frac_bits, size_t workspace_bytes,
                    void* hip_stream, mpc3_ctx** out);
int mpc3_ctx_destroy(mpc3_ctx* ctx);

/* Return the device memory the context caches between calls: the call workspaces (they
 * grow to the largest call made and are otherwise kept), the verification workspaces and
 * results, and the free buffers of its own lowerings (mpc3_inner_conv without cols).
 * Memory of products not yet verified, message copies and recorded graphs stay.  The
 * next call that needs a workspace allocates it again.  Synchronises the context's
 * streams.  *freed_bytes (may be NULL) is the amount returned.  MPC3_E_STATE while a
 * verification is in flight or while recording. */
int mpc3_trim(mpc3_ctx* ctx, int64_t* freed_bytes);

/* Kernel family for every matrix product: MPC3_VARIANT_U64 (64-bit integer
 * VALU) or MPC3_VARIANT_LIMB_I8 (8-bit limbs on int8 MFMA, recombined modulo
 * 2^64).  Both give bit-identical results. */
int mpc3_set_variant(mpc3_ctx* ctx, int variant);

/* Autotuner: time both kernel families on the three-party product of an M x K by K x N
 * layer (random operands in the context's workspace, `reps` timed runs each after one
 * warm-up) and remember the faster one for that shape.  The choice is kept per
 * (M rounded up to a power of two, K, N), so one call covers every M in (2^(k-1), 2^k].
 * With MPC3_VARIANT_AUTO every Pi_Inner uses the remembered choice for its shape (the
 * limb family when the shape was never tuned).  *choice receives the pick; ms_u64 / ms_limb (nullable) the median times.
 * Synchronises.  Results are bit-identical either way; only speed differs. */
int mpc3_autotune(mpc3_ctx* ctx, int64_t M, int64_t K, int64_t N, int reps, int* choice, double* ms_u64,
                  double* ms_limb);

/* Launch-shape autotuner of the limb kernel (MPC3_VARIANT_LIMB_I8) for the three-party
 * product of an M x K by K x N layer: times (random operands in the context's workspace,
 * `reps` timed runs each after one warm-up) the built-in launch and the candidates -- one
 * or two 64-column tiles per workgroup, the built-in launch order or 1, 2, 4, ..., 64 row
 * tiles per group of the order in which workgroups reach the XCDs, K splits as built in or
 * doubled -- and remembers the fastest for (M rounded up to a power of two, K, N) if it
 * beats the built-in launch by 2% both in the sweep and when the two are timed again,
 * else forgets any earlier choice for that shape.  shape[3] receives (ns, rb, split), all
 * 0 for the built-in launch; ms_default / ms_best (nullable) the median times (of the
 * second timing when a shape is kept).  Every Pi_Inner of that shape on the limb kernel then uses
 * the remembered launch.  Synchronises.  Results are bit-identical for every launch shape. */
int mpc3_autotune_launch(mpc3_ctx* ctx, int64_t M, int64_t K, int64_t N, int reps, int* shape,
                         double* ms_default, double* ms_best);

/* Remember a launch shape for the limb kernel's three-party products of shape (M, K, N)
 * without timing (a tuning result kept from an earlier process): ns 0 or 1 (1 keeps one
 * column tile per workgroup), rb 0..65535 (0 = built-in launch order), split 0..16 (0 or 1
 * = built-in K splits); all zero forgets the shape's entry.  MPC3_E_ARG otherwise. */
int mpc3_set_launch(mpc3_ctx* ctx, int64_t M, int64_t K, int64_t N, int ns, int rb, int split);

/* Truncations per Pi_BIVerify instance of the truncation gates (default and maximum
 * 524288 = 2^19; a chunk of T truncations holds about 20 KiB x T of workspace while
 * verified).  MPC3_E_ARG outside 1 .. 2^19. */
int mpc3_set_chunk(mpc3_ctx* ctx, int64_t truncations_per_instance);

/* Instance sizes of the other verifications: Pi_Mult triples per Pi_MultVerify instance
 * (default 2^20, at most 2^24; about 3.5 KiB of workspace per triple while verified) and
 * edaBit inner products per Pi_BIVerify instance (default 2^14, at most 2^18; about
 * 200 KiB each).  0 keeps a value.  MPC3_E_ARG outside the ranges. */
int mpc3_set_verify_chunks(mpc3_ctx* ctx, int64_t mult_triples, int64_t edabit_rows);

/* R argument of mpc3_verify: per instance, the number of Pi_Reduce rounds of least
 * modelled time on the network set by mpc3_set_network. */
enum { MPC3_R_NETWORK = -2 };

/* Network cost model for the choice of R (Sec. 5.1, the trade-off of R between the
 * rounds of more reductions and the size of the final check, on the LAN / MAN / WAN
 * settings of the experiments).  An instance of n pairs (ring elements of w bytes: 512
 * in GR(2^64, 64), 8 in GF(2^64)) with R reductions and n_R = n / 2^R final pairs
 * sends w (2R + n_R + 1) bytes P0 -> P2 offline and has 2R + 4 online rounds whose
 * busiest link carries w (2R + n_R + 1) + 32 (R + 2) bytes (the counters of
 * mpc3_comm_stats); each phase costs rounds x rtt plus bytes over the bandwidth, plus
 * gpu_round_ms of GPU latency per reduction round.  mpc3_verify(R = MPC3_R_NETWORK)
 * takes the R in 0 .. ceil(log2 n) of least total (MPC3_E_STATE before this call). */
int mpc3_set_network(mpc3_ctx* ctx, double rtt_ms, double mbit_per_s, double gpu_round_ms);

/* Keep the messages of each Pi_Inner / Pi_Mult for mpc3_message (default off). */
int mpc3_keep_messages(mpc3_ctx* ctx, int on);

/* Fixed-point encoding (Preliminaries, "Notation"): out = floor(x * 2^f) mod 2^64
 * for n doubles.  x_dev and out_dev are device buffers of n elements. */
int mpc3_encode(mpc3_ctx* ctx, const double* x_dev, int64_t n, uint64_t* out_dev);

/* Decoding: out = (int64) v / 2^f as double. */
int mpc3_decode(mpc3_ctx* ctx, const uint64_t* v_dev, int64_t n, double* out_dev);

/* Pi_<.>^{l,k}(x) (Preliminaries, "Secret sharing"): owner k in {0,1,2}
 * shares rows*cols words x_dev into the caller's planes out->m, r1, r2
 * (out->rows, out->cols give the shape).  [r]_1 and [r]_2 come from the
 * pairwise PRGs; the owner sends m = x + r1 + r2. */
int mpc3_share(mpc3_ctx* ctx, int owner, const uint64_t* x_dev, mpc3_share_t* out);

/* Preprocessing of Pi_Trunc^t for n outputs (Fig. "The maliciously secure
 * truncation protocol", Sec. 4.2): draws the bit lists of P0+P1 and P0+P2, runs
 * the two inner products (over all 64 bit positions) that give <r_x> and
 * <r_z> = <ash(r_x, t)>, and registers both for verification.  1 <= t <= 62. */
int mpc3_trunc_pair(mpc3_ctx* ctx, int64_t n, int t, mpc3_trunc_pair_t* out);

/* Pi_Inner for every output of Z = X W (Fig. "The Inner Product Protocol";
 * Sec. 4.1 treats a matrix product as M*N inner products).  X is M x K, W is
 * K x N, Z (caller planes) is M x N.  out_mask != NULL makes the output mask
 * the pair's r_x (the truncation pair is generated first, Sec. 4.2);
 * NULL draws a fresh mask.  Registers the product for verification. */
int mpc3_inner(mpc3_ctx* ctx, const mpc3_share_t* X, const mpc3_share_t* W,
               const mpc3_trunc_pair_t* out_mask, mpc3_share_t* Z);

/* mpc3_inner for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * results, registration and counters as mpc3_inner, bit for bit, but the call's
 * device workspace (the three party sums, P0's [Gamma]_1 and the matrix-core digit
 * tiles of W) is one fixed array of 256 MiB per GPU, held from the library's load to
 * the end of the process, so the call makes no hipMalloc, hipFree or other device
 * allocation (the host-side list of pending products grows as for mpc3_inner).  Split-K
 * partial sums of the product take what the rest of its workspace leaves of the array
 * (without room, K is split only where the 32-bit digit sums require it, with atomic
 * adds).  MPC3_E_LIMIT, before any launch, when the operands need more
 * than the array: about 32 bytes per output plus 40 bytes per element of W (VGG-style
 * layers of a batch of 64 fit).  MPC3_E_STATE with mpc3_keep_messages on (message
 * copies would need device memory); profiling (mpc3_profile) does not time it.  Every
 * call on one GPU uses the same array: calls ordered on one stream are safe, calls
 * of different contexts or streams that overlap in time on one GPU race. */
int mpc3_inner_static(mpc3_ctx* ctx, const mpc3_share_t* X, const mpc3_share_t* W,
                      const mpc3_trunc_pair_t* out_mask, mpc3_share_t* Z);

/* A convolution layer's Pi_Inner: the lowering of mpc3_im2col_strided of x (W->rows =
 * ld >= KH KW C columns, the extra ones 0), then mpc3_inner(lowering, W) with the same
 * arguments, results and counters, bit for bit.  The product is registered with its input
 * x as well: for a same-padded stride-1 convolution (KH = KW = 2 pad + 1) the verification
 * forms each compressed x-side element sum_m r^(o+m) cols[m, k] from x directly -- column
 * k = (kh, kw, c) is channel c shifted by delta = (kh - pad) W + (kw - pad) positions, so
 * the sum is r^(o - delta) times the power-weighted sum of channel c over the whole input
 * minus the same sum over the border rows and columns that shift leaves out -- reading x
 * (KH KW times smaller than cols) instead of cols; the values are identical (this needs
 * o >= pad W + pad, o the gates of the products registered before it in its batch).
 * cols receives the lowering; cols = NULL lets the library choose: when that condition
 * holds, C is a multiple of 32, ld = KH KW C and the product runs on the limb kernel, the
 * kernel reads the lowered rows straight from x (no lowering is written); otherwise the
 * lowering goes to device memory of the library's, held until the product is verified.
 * x, cols (if given), W and Z must stay alive and unmodified until verified. */
int mpc3_inner_conv(mpc3_ctx* ctx, const mpc3_share_t* x, int B, int H, int W, int C, int KH, int KW,
                    int pad, int stride, mpc3_share_t* cols, const mpc3_share_t* Wt,
                    const mpc3_trunc_pair_t* out_mask, mpc3_share_t* Z);

/* Convolution lowering: cols (B*OH*OW rows, KH*KW*C cols) from an NHWC shared
 * tensor x (B*H*W*C words per plane), zero padding pad, stride 1.  Each plane
 * is rearranged alone (a local linear map); Sec. 4.1 evaluates a convolution
 * as one inner product per output.  cols may be wider than KH*KW*C: the extra
 * columns are written as 0 in every plane (a share of 0), so a product with
 * matching zero-padded weights is unchanged while its contraction width becomes
 * a multiple of the matrix-core k-block.  MPC3_E_SHAPE if cols has another row
 * count or fewer columns. */
int mpc3_im2col(mpc3_ctx* ctx, const mpc3_share_t* x, int B, int H, int W, int C, int KH, int KW,
                int pad, mpc3_share_t* cols);

/* The same lowering with stride s: output (oh, ow) reads input (s oh + kh - pad,
 * s ow + kw - pad); OH = (H + 2 pad - KH) / s + 1 (the S-NN layer of Sec. 5.2 has
 * stride 2). */
int mpc3_im2col_strided(mpc3_ctx* ctx, const mpc3_share_t* x, int B, int H, int W, int C, int KH, int KW,
                        int pad, int stride, mpc3_share_t* cols);

/* 2x2 sum pooling (stride 2) of an NHWC shared tensor x (B*H*W*C words per plane)
 * into out (B*(H/2)*(W/2)*C): each plane is summed alone, a local linear map
 * (Preliminaries, linear homomorphism of <.>-shares).  H and W must be even. */
int mpc3_sumpool2(mpc3_ctx* ctx, const mpc3_share_t* x, int B, int H, int W, int C, mpc3_share_t* out);

/* Pi_Mult elementwise on rows*cols values (Fig. "The Multiplication Protocol"). */
int mpc3_mult(mpc3_ctx* ctx, const mpc3_share_t* a, const mpc3_share_t* b, mpc3_share_t* c);

/* --- Non-linear layers (Sec. 4.3 "Secure Non-linear Function Evaluation") ---------
 * Boolean shares <v>^1 = (m, [r]_1, [r]_2) with m = v XOR r1 XOR r2 are bit-sliced: one
 * uint64 word per plane, for a 64-bit value its bit i in bit i.  The Boolean products
 * (Pi_Mult with AND and XOR) are verified by Pi_MultVerify over GF(2^64) = GR(2, 64)
 * (kind MPC3_VERIFY_NONLINEAR), the products over Z_{2^64} by Pi_MultVerify as for
 * mpc3_mult.  Intermediate buffers are the context's and are freed once verified. */

/* n edaBits (Fig. "The maliciously edaBits generation"): arith (n words per plane) receives
 * <r>^l and bits (n words per plane) <r[0..63]>^1 of the same random r.  The bit products
 * are one Pi_Mult of 64 n elements; the second multiplication is one 64-element inner
 * product per edaBit: r = sum_i 2^i (m_i + r'_i) - sum_i 2^(i+1) m_i r'_i.  The paper's
 * arithmetic bit shares (0, b, 0) and (0, 0, b) are taken as (0, -b, 0) and (0, 0, -b)
 * so that they open to +b under m = v + r. */
int mpc3_edabits(mpc3_ctx* ctx, int64_t n, mpc3_share_t* arith, mpc3_share_t* bits);

/* n daBits: a random bit s per word in both sharings (arith <s>^l, bits <s>^1 in bit 0),
 * from two Pi_Mult rounds: r' = b_1 XOR b_2, s = m XOR r'. */
int mpc3_dabits(mpc3_ctx* ctx, int64_t n, mpc3_share_t* arith, mpc3_share_t* bits);

/* ReLU of every value of x (rows*cols words per plane) into out: x * (1 - msb(x)).  Per
 * value one edaBit and one daBit; Delta = x - r is opened (Pi_Rec), the carry into bit 63
 * of Delta + r comes from a parallel-prefix adder (six Boolean Pi_Mult rounds on whole
 * words); e = (1 - msb) XOR s is opened and <1 - msb>^l = e + (1 - 2e) <s>^l (B2A) is
 * multiplied with x by Pi_Mult.  x and out must stay alive until verified. */
int mpc3_relu(mpc3_ctx* ctx, const mpc3_share_t* x, mpc3_share_t* out);

/* 2x2 max pooling (stride 2) of an NHWC tensor x (B*H*W*C words per plane, H and W even)
 * into out (B*(H/2)*(W/2)*C): max(p, q) = q + ReLU(p - q) over the two pairs of a window,
 * then over the two results.  x and out must stay alive until verified. */
int mpc3_maxpool2(mpc3_ctx* ctx, const mpc3_share_t* x, int B, int H, int W, int C, mpc3_share_t* out);

/* Online Pi_Trunc: out.m = ash(Z.m, t); the output mask is the pair's r_z.
 * No communication (Sec. 4.2). */
int mpc3_trunc(mpc3_ctx* ctx, const mpc3_trunc_pair_t* p, const mpc3_share_t* Z, mpc3_share_t* out);

/* --- Recorded forward passes (HIP graphs) -------------------------------------------
 * The online layers of one network at one batch size are the same launches on the same
 * buffers every time; only the operation ids behind the keystream tags (which make every
 * mask and every truncation pair fresh) change.  The calls between mpc3_capture_begin and
 * mpc3_capture_end are recorded into one HIP graph by stream capture on the context's
 * stream instead of being run.  Only calls that neither allocate nor synchronise may be
 * recorded: mpc3_encode, mpc3_decode, mpc3_share, mpc3_trunc_pair, mpc3_inner_static,
 * mpc3_trunc, mpc3_im2col(_strided) and mpc3_sumpool2; every other call on the context
 * returns MPC3_E_STATE while recording.  Recording leaves the context as it was (no
 * operation id used, nothing counted, nothing pending); the context keeps the calls'
 * effects instead: operation ids used, counted bytes and rounds, and products registered
 * for verification.  The keystream kernels read one device word that is added to every
 * recorded operation id; mpc3_graph_launch sets it (by a kernel on the stream, before the
 * graph) to the distance from the recording's first id to the context's next id, so a
 * replay draws exactly what the same calls made directly at that point would draw, and
 * then applies the recorded effects under the shifted ids.  The graph holds kernel nodes
 * only (no memset or copy nodes).  The pair structures the caller passed while recording
 * keep the ids of the recording. */

/* Start recording on the context's stream (MPC3_E_STATE when the context runs on the
 * null stream, is recording already, keeps messages or has an injection armed). */
int mpc3_capture_begin(mpc3_ctx* ctx);

/* Stop recording; *graph_id (> 0) names the instantiated graph.  A call that failed while
 * recording makes this return that failure's code (or MPC3_E_HIP if the stream capture
 * was invalidated) with no graph created; the context is as before mpc3_capture_begin. */
int mpc3_capture_end(mpc3_ctx* ctx, int* graph_id);

/* Replay a graph on the context's stream with fresh operation ids (asynchronous, like the
 * calls it recorded).  The buffers the recording named must be alive; the caller fills
 * the recorded input buffers (on the same stream) before.  MPC3_E_STATE while products
 * of this graph's previous replay are still pending (its buffers would be overwritten
 * before they are verified) or while recording; MPC3_E_ARG for an unknown id. */
int mpc3_graph_launch(mpc3_ctx* ctx, int graph_id);

/* Node counts of a graph: kernel nodes and nodes of any other type (memset, copy, ...). */
int mpc3_graph_nodes(mpc3_ctx* ctx, int graph_id, int64_t* kernel_nodes, int64_t* other_nodes);

/* Free a graph (waits for the context's stream).  Graphs are also freed with the context. */
int mpc3_graph_destroy(mpc3_ctx* ctx, int graph_id);

/* Post-processing verification (Sec. 3) of the pending products selected by kinds
 * (MPC3_VERIFY_* mask).  The non-linear layers' edaBit inner products run as
 * Pi_BIVerify instances of 64-element gates (16384 per instance), their Boolean
 * triples as one Pi_MultVerify over GF(2^64) per layer call.  Instance 0 is one Pi_BIVerify^R over every pending Pi_Inner
 * product together: the batch verification gives gate (m, n) of product l, in call
 * order, the index i = o_l + M_l n + m (o_l = the number of gates of the products
 * before it) and the weight r^i on its x side.  Because r^i = r^(o_l) r^m (r^(M_l))^n
 * factorises, each product's M_l N_l K_l consolidated pairs compress exactly into K_l
 * pairs (x_k = r^(o_l) sum_m r^m X[m,k], y_k = sum_n r^(M_l n) W[k,n]) with an
 * unchanged claimed z.  Then one instance per chunk of truncation gates, and one
 * Pi_MultVerify^R per chunk of each Pi_Mult call's triples.  R = -1 picks max(0, ceil(log2 n) - 3) for an
 * instance of n pairs, MPC3_R_NETWORK the least modelled time (mpc3_set_network).  *ok = 1 iff every Delta is 0; otherwise *ok = 0 and the
 * context is aborted.  Synchronises. */
int mpc3_verify(mpc3_ctx* ctx, int R, int kinds, int* ok);

/* mpc3_verify in two halves, for pipelining: mpc3_verify_begin takes the selected pending
 * products off the pending list (with the same operation ids, draws and transcript as
 * mpc3_verify at that point) and enqueues their verification on the context's worker
 * streams after everything enqueued on its stream so far; it returns without waiting.  Later
 * calls on the context's stream (for example the next batch's layers) run alongside.
 * mpc3_verify_end waits for it and reports as mpc3_verify (*ok, abort, transcript).  One
 * verification may be in flight: mpc3_verify_begin and mpc3_verify return MPC3_E_STATE
 * while one is; mpc3_reconstruct returns MPC3_E_UNVERIFIED and mpc3_verify_log
 * MPC3_E_STATE until it has ended.  The operands of the products in flight must stay alive
 * and unmodified until mpc3_verify_end. */
int mpc3_verify_begin(mpc3_ctx* ctx, int R, int kinds);
int mpc3_verify_end(mpc3_ctx* ctx, int* ok);

/* Pi_Rec (Preliminaries, "Verifiability of share reconstruction"): open X into
 * out_dev (rows*cols words) after cross-checking the copies the receivers got.
 * to_party < 0 opens to all three parties (Pi_Rec^l); to_party = k opens to P_k
 * alone (Pi_Rec^{l,k}): only P_k's missing plane (P0: m from P1, P1: [r]_2 from P0,
 * P2: [r]_1 from P0) and the hash that checks it are sent and counted, and out_dev
 * is P_k's output.  Requires every pending product to be verified (else
 * MPC3_E_UNVERIFIED).  An inconsistency aborts the context and returns
 * MPC3_E_ABORTED with out_dev left unwritten.  Synchronises. */
int mpc3_reconstruct(mpc3_ctx* ctx, const mpc3_share_t* X, int to_party, uint64_t* out_dev);

/* Counted communication so far (host struct).  Synchronises. */
int mpc3_comm_stats(mpc3_ctx* ctx, mpc3_comm* out);

/* Testing: add e (mod 2^64) to one word of the next message at site
 * (MPC3_SITE_*).  The error models the additive attack of a malicious party. */
int mpc3_inject(mpc3_ctx* ctx, int site, int64_t index, uint64_t e);

/* Testing: copy n words of message `which` (MPC3_MSG_*) of the most recent
 * Pi_Inner or Pi_Mult into out_dev.  Needs mpc3_keep_messages(ctx, 1). */
int mpc3_message(mpc3_ctx* ctx, int kind /* 0 inner, 1 mult */, int which, uint64_t* out_dev, int64_t n);

/* Testing: d words of one transcript slot (MPC3_LOG_*) of verification
 * instance `instance` of the most recent mpc3_verify, into host memory.
 * Also reports the instance's R and padded dimension when the pointers are
 * not NULL. */
int mpc3_verify_log(mpc3_ctx* ctx, int64_t instance, int slot, int round, uint64_t* out_host,
                    int* R_out, int64_t* dim_out);

/* Measurement: while on, every Pi_Inner matrix-product launch is bracketed by HIP
 * events on the context's stream.  mpc3_profile_read synchronises and returns the
 * summed event time (ms), the number of launches and their algorithmic work in ring
 * multiply-accumulates (5 M K N per Pi_Inner: P0 1, P1 2, P2 2), then clears them. */
int mpc3_profile(mpc3_ctx* ctx, int on);
int mpc3_profile_read(mpc3_ctx* ctx, double* total_ms, int64_t* launches, double* ring_macs);

/* The last failure of an entry point on this context: returns its MPC3_E_* code (0 if
 * none; a failed verification is not recorded here), *hip_error the hipError_t of a
 * failed HIP call (0 otherwise), and `where` (nullable, where_len bytes including the
 * terminating 0) the entry point's name followed by the failing HIP call as written. */
int mpc3_last_error(const mpc3_ctx* ctx, int* hip_error, char* where, size_t where_len);

/* Static description of a return code. */
const char* mpc3_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* MPC3_H */
