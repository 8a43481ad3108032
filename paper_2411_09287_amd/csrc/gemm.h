// Matrix products over Z_{2^64}: the one contraction shape behind every heavy step.
#pragma once
#include "common.h"

namespace mpc3 {

// A strided view: element (i, j) of batch b is p[b*sb + i*s0 + j*s1].
struct GemmGroup;

struct View {
    const u64* p;
    int64_t s0, s1, sb;
};
struct OutView {
    u64* p;
    int64_t s0, s1, sb;
};

// C = A B over Z_{2^64}.  A is M x K, B is K x N (per batch).
//   plain:  C = A B (+ D when D.p != null), or C += A B (atomic) when accumulate.
//   party:  three accumulators from the share planes of A = (Am, A1, A2), B = (Bm, B1, B2):
//           C0 = (A1 + A2)(B1 + B2)              (P0: r_x r_y)
//           C1 = Am B1 + A1 Bm                   (P1: m_x [r_y]_1 + m_y [r_x]_1)
//           C2 = Am (Bm - B2) - A2 Bm            (P2: m_x m_y - m_x [r_y]_2 - m_y [r_x]_2)
struct GemmArgs {
    int64_t M, N, K;
    int batch;
    bool party;
    int shared;               // plain, 2 or 3: C[p] = A[p] B[0] for p < shared in one launch
    bool accumulate;          // C += A B with 64-bit atomic adds (C initialised by the caller)
    View A[3], B[3];          // plain uses index 0
    OutView C[3];
    View Dadd;                // plain, non-accumulating: C = AB + Dadd
    // device workspace (stream-ordered bump allocator of the caller): digit tiles of the limb
    // backend, split-K partial sums of both backends; without it K is split only with
    // atomic adds into an accumulating (or zeroed) output
    void* (*ws_alloc)(void* self, size_t bytes);
    void* ws_self;
    // optional, plain form: B[0] already in the limb kernel's digit-tile form (limb_btiles),
    // 64-column tiles of btiles_nkb 32-deep k-blocks each, of which the first K rows are
    // used; read only by the limb kernel that takes converted B (B[0] must still be valid)
    const int8_t* btiles;
    int64_t btiles_nkb;
    // the workspace takes digit tiles only: K is split only where the 32-bit digit sums
    // require it, with atomic adds into the (zero-filled) output
    bool no_part;
    // bytes of split-K partial sums the workspace can take (0: PART_MAX)
    size_t part_max;
    // launch shape of the limb kernel, 0 = the built-in choice: lt_ns = 1 keeps one 64-column
    // tile per workgroup where two would be taken; lt_rb row tiles per launch-order group;
    // lt_split multiplies the number of K splits (where the workspace takes the partials).
    // Results do not depend on them.
    int lt_ns, lt_rb, lt_split;
    // implicit lowering of a stride-1 convolution (limb kernel, where limb_conv_ok): A[p]
    // are the planes of the NHWC input (images of cH x cW x cC words); row m of the product
    // is output position (b, oh, ow) of cOH x cOW per image, column k = (kh, kw, c) of
    // K = cKH cKW cC; input positions outside the image (padding cpad) read as 0
    int conv;
    int cH, cW, cC, cKH, cKW, cpad, cOH, cOW;
    // record instead of launch (gemm_group_run)
    GemmGroup* group;
};

// Products launched together: with GemmArgs::group set, a product that runs on the limb
// kernel's converted-B path is recorded instead of launched (any B conversion it needs is
// still launched at once), and gemm_group_run launches every recorded product of one kernel
// variant as one grid over a device table of the products (each workgroup finds its product
// and tile there), then all their split-K reductions as one more grid.  Other products
// launch at once.  The group keeps the host copies of its tables until its next run.
GemmGroup* gemm_group_new();
void gemm_group_free(GemmGroup* g);
hipError_t gemm_group_run(GemmGroup* g, void* (*ws_alloc)(void*, size_t), void* ws_self, hipStream_t stream);

// Whether the limb kernel takes g's implicit lowering (C a multiple of 32, K = KH KW C,
// stride 1, 16-byte aligned planes, one batch, a workspace for the B tiles).
bool limb_conv_ok(const GemmArgs& g);

// The cap on split-K partial sums of one product.
inline size_t part_cap(const GemmArgs& g);

// Launch on `stream` with the chosen backend (0 = u64 VALU, 1 = int8 limbs on MFMA).
hipError_t gemm(const GemmArgs& g, int variant, hipStream_t stream);

// One split-K reduction: part holds batch x splits x nprod planes of M x N words (n
// fastest); C[p] = their sum (+ D for nprod 1), or C[p] += sum with atomics.
struct RedArgs {
    const u64* part;
    int64_t M, N;
    int nprod, splits, batch, atomic;
    OutView C[3];
    View D;
};
// Many reductions in one grid: tab (device) holds n jobs, start (device) n + 1 prefix counts
// of 64-output blocks; W waves per block (at most 16) share each block's splits.
hipError_t split_reduce_group(const RedArgs* tab, const int64_t* start, int n, int64_t nblk, int W,
                              hipStream_t stream);

// Split-K partial sums: part holds batch x splits x nprod planes of M x N words (n fastest).
// C[p] = sum over splits (+ D when D.p is set, nprod == 1), or C[p] += sum (64-bit atomic
// add) when atomic.
hipError_t split_reduce(const u64* part, int64_t M, int64_t N, int nprod, int splits, int batch,
                        const OutView* C, const View& D, bool atomic, hipStream_t stream);

// Digit tiles of a K x N operand (any strides) for GemmArgs::btiles: limb_btiles_bytes(K, N)
// bytes at out, k-blocks per column tile = (K + 31) / 32.
size_t limb_btiles_bytes(int64_t K, int64_t N);
hipError_t limb_btiles(const View& B, int64_t K, int64_t N, int8_t* out, hipStream_t stream);

// Fills n 32-bit words with 0 (a kernel, so that it can also be captured in a graph).
hipError_t zero_words32(void* p, int64_t n, hipStream_t stream);

// The h(0) and h(x) party sums of a Pi_Reduce round over planes of n rows (pairs (2i, 2i+1))
// stacked in XY (plane p at XY + p n 64): dense, six planes (x: m, r1, r2; y: m, r1, r2) and
// the three parties' sums; sparse, two planes (x's [r]_1, y's [r]_2) and P0's sum alone.
// The parties' sums are split into units of one product each (dense: P0 unit 0, P1 units 1
// and 2, P2 units 3 and 4; sparse: P0 unit 0).  Each of the G = hpair_groups(n) workgroups
// per unit writes its partial: part[(g units + unit) 256 + point 128 + i], point 0 = h(0), 1 =
// h(x), i < 64 the anti-diagonal sums j + l = i of the unit's 64 x 64 outer-product sum,
// i >= 64 those with j + l = i (= 64 + k); summing a party's partials and reducing the second
// half modulo the ring's modulus gives the party's ring element.
struct HPartyArgs {
    const u64* XY;
    int64_t n;
    int64_t npairs, nblocks;      // set by hpair_party
    bool dense;
    u64* part;                    // G x (5 or 1) x 256 words
};
int hpair_groups(int64_t n);
hipError_t hpair_party(const HPartyArgs& a, hipStream_t stream);

// The fold of a Pi_Reduce round on the matrix cores: rows of 128 words are pairs (f(0),
// f(1)) of 64-word GR(2^64, 64) elements; out row i (64 words) = f(0) + (f(1) - f(0)) Z,
// ztiles the digit tiles (limb_btiles) of the 64 x 64 multiplication matrix Z of the point.
hipError_t fold_rows(const u64* XY, int64_t rows, const int8_t* ztiles, u64* out, hipStream_t stream);

// Bytes of partial sums one product may use before the split count is cut back.
constexpr size_t PART_MAX = (size_t)1 << 30;

inline size_t part_cap(const GemmArgs& g) { return g.part_max && g.part_max < PART_MAX ? g.part_max : PART_MAX; }

}  // namespace mpc3
