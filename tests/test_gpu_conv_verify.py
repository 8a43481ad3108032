"""mpc3_inner_conv (lowering + Pi_Inner, the product verified from the layer's input) against
mpc3_im2col + mpc3_inner on the same seeds and call sequence: every share plane, the counted
messages and the batched Pi_BIVerify transcript (claim, every round's messages and points,
the final Delta) bit for bit.  The cases cover same-padded convolutions that take the
input-side compression (3x3 and 5x5, channel counts below and above 64, a zero-padded
contraction width, batch > 1, H != W), the cases that keep the lowered form (stride 2, no
padding, a convolution as the first product), and an injected error in a convolution's
output share."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_09287_amd import mpc3  # noqa: E402

SEED = bytes(range(21, 53))


def u64(g, *shape):
    return g.integers(0, 1 << 64, size=shape, dtype=np.uint64, endpoint=False)


# (B, H, W, C, K, pad, stride, N, ld)
CASES = [
    [(2, 8, 8, 3, 3, 1, 1, 16, 32), (1, 6, 10, 70, 3, 1, 1, 9, None), (2, 7, 7, 5, 5, 2, 1, 4, None)],
    [(1, 8, 8, 4, 3, 1, 2, 6, None), (2, 6, 6, 3, 3, 0, 1, 5, None), (3, 5, 9, 64, 3, 1, 1, 8, None)],
]


# same-padded convolutions whose channel counts are multiples of 32: with no cols buffer the
# limb kernel lowers them implicitly (one and two 64-column tiles per workgroup, 3x3 and 5x5,
# ragged row counts); the u64 kernel family lowers into the library's own memory
CASES_IMPLICIT = [(2, 8, 8, 32, 3, 1, 1, 64, None), (1, 6, 10, 64, 3, 1, 1, 130, None),
                  (2, 7, 5, 32, 5, 2, 1, 9, None), (3, 9, 7, 96, 3, 1, 1, 200, None)]


def run(use_conv, convs, seed, first_dense=True, variant=1, inject=None, own_cols=False):
    g = np.random.default_rng(seed)
    c = mpc3.Context(SEED)
    c.set_variant(variant)
    if first_dense:
        c.inner(c.share(mpc3.to_words(u64(g, 40, 24))), c.share(mpc3.to_words(u64(g, 24, 7))))
    zs = []
    for B, H, W, C, K, pad, stride, N, ld in convs:
        kk = ld or K * K * C
        x = c.share(mpc3.to_words(u64(g, B, H * W * C)))
        w = u64(g, kk, N)
        w[K * K * C:] = 0
        Wt = c.share(mpc3.to_words(w))
        if use_conv:
            cols = None
            if own_cols:
                OH, OW = (H + 2 * pad - K) // stride + 1, (W + 2 * pad - K) // stride + 1
                cols = mpc3.DShare.empty(B * OH * OW, kk, "cuda")
            Z = c.inner_conv(x, B, H, W, C, K, K, pad, Wt, ld=ld, stride=stride, cols=cols)
        else:
            cols = c.im2col(x, B, H, W, C, K, K, pad, ld, stride=stride)
            Z = c.inner(cols, Wt)
        zs.append(Z)
    if inject is not None:
        li, row, col = inject
        zs[li].m[row, col] += 1
    ok = c.verify()
    _, R, _ = c.verify_log(0, mpc3.LOG_R)
    log = [c.verify_log(0, sl)[0] for sl in (mpc3.LOG_R, mpc3.LOG_Z, mpc3.LOG_DELTA, mpc3.LOG_DELTA_M1)]
    for k in range(R):
        log += [c.verify_log(0, sl, k)[0] for sl in (mpc3.LOG_ZETA, mpc3.LOG_H0_M1, mpc3.LOG_H2_G2)]
    planes = [z.numpy() for z in zs]
    comm = c.comm_stats()
    c.close()
    return ok, planes, log, comm


@pytest.mark.parametrize("variant", [1, 0])
@pytest.mark.parametrize("case", [0, 1])
def test_inner_conv_matches_lowered_product(case, variant):
    a = run(True, CASES[case], seed=100 + case, variant=variant)
    b = run(False, CASES[case], seed=100 + case, variant=variant)
    assert a[0] and b[0], "honest verification failed"
    for za, zb in zip(a[1], b[1]):
        for pa, pb in zip(za, zb):
            assert np.array_equal(pa, pb)
    assert len(a[2]) == len(b[2])
    for la, lb in zip(a[2], b[2]):
        assert np.array_equal(la, lb)
    assert np.array_equal(a[3][0], b[3][0]) and a[3][1] == b[3][1]


def test_inner_conv_first_product_keeps_lowered_form():
    convs = [(2, 6, 6, 3, 3, 1, 1, 5, None), (1, 6, 6, 8, 3, 1, 1, 4, None)]
    a = run(True, convs, seed=7, first_dense=False)
    b = run(False, convs, seed=7, first_dense=False)
    assert a[0] and b[0]
    for la, lb in zip(a[2], b[2]):
        assert np.array_equal(la, lb)


@pytest.mark.parametrize("inject", [(0, 5, 3), (2, 0, 1)])
def test_inner_conv_error_detected(inject):
    ok, _, _, _ = run(True, CASES[0], seed=300, inject=inject)
    assert not ok


@pytest.mark.parametrize("variant", [1, 0])
@pytest.mark.parametrize("own_cols", [False, True])
def test_inner_conv_implicit_lowering_matches_lowered_product(variant, own_cols):
    a = run(True, CASES_IMPLICIT, seed=500, variant=variant, own_cols=own_cols)
    b = run(False, CASES_IMPLICIT, seed=500, variant=variant)
    assert a[0] and b[0], "honest verification failed"
    for za, zb in zip(a[1], b[1]):
        for pa, pb in zip(za, zb):
            assert np.array_equal(pa, pb)
    assert len(a[2]) == len(b[2])
    for la, lb in zip(a[2], b[2]):
        assert np.array_equal(la, lb)
    assert np.array_equal(a[3][0], b[3][0]) and a[3][1] == b[3][1]


def test_inner_conv_first_product_with_32_channels_is_lowered():
    # the batch's first product (o = 0) cannot be verified from its input: the library
    # lowers it into its own memory and verifies the lowered form
    convs = [(2, 6, 6, 32, 3, 1, 1, 64, None), (1, 6, 6, 64, 3, 1, 1, 70, None)]
    a = run(True, convs, seed=9, first_dense=False)
    b = run(False, convs, seed=9, first_dense=False)
    assert a[0] and b[0]
    for za, zb in zip(a[1], b[1]):
        for pa, pb in zip(za, zb):
            assert np.array_equal(pa, pb)
    for la, lb in zip(a[2], b[2]):
        assert np.array_equal(la, lb)


def test_inner_conv_implicit_error_detected():
    ok, _, _, _ = run(True, CASES_IMPLICIT, seed=501, inject=(1, 3, 77))
    assert not ok


def batches(trim, seed):
    """Two batches (a dense product, then lowered convolutions that use the library's pooled
    buffers and the implicit path), each verified; with trim, mpc3_trim between them."""
    g = np.random.default_rng(seed)
    c = mpc3.Context(SEED)
    c.set_variant(1)
    res, freed = [], None
    for rep in range(2):
        c.inner(c.share(mpc3.to_words(u64(g, 40, 24))), c.share(mpc3.to_words(u64(g, 24, 7))))
        zs = []
        for B, H, W, C, K, pad, stride, N, _ in (CASES[0][1], CASES_IMPLICIT[1]):
            x = c.share(mpc3.to_words(u64(g, B, H * W * C)))
            Wt = c.share(mpc3.to_words(u64(g, K * K * C, N)))
            zs.append(c.inner_conv(x, B, H, W, C, K, K, pad, Wt, stride=stride))
        ok = c.verify()
        log = [c.verify_log(0, sl)[0] for sl in (mpc3.LOG_R, mpc3.LOG_Z, mpc3.LOG_DELTA)]
        res.append((ok, [z.numpy() for z in zs], log))
        if trim and rep == 0:
            freed = c.trim()
    c.close()
    return res, freed


def test_trim_keeps_results_and_releases_memory():
    a, freed = batches(True, 900)
    b, _ = batches(False, 900)
    assert freed > 0
    for (oka, za, la), (okb, zb, lb) in zip(a, b):
        assert oka and okb, "honest verification failed"
        for pa, pb in zip(za, zb):
            for qa, qb in zip(pa, pb):
                assert np.array_equal(qa, qb)
        for x, y in zip(la, lb):
            assert np.array_equal(x, y)


def test_trim_refused_while_verifying_or_recording():
    g = np.random.default_rng(901)
    c = mpc3.Context(SEED, stream=torch.cuda.Stream())
    c.inner(c.share(mpc3.to_words(u64(g, 16, 8))), c.share(mpc3.to_words(u64(g, 8, 4))))
    c.verify_begin()
    with pytest.raises(mpc3.Mpc3Error) as e:
        c.trim()
    assert e.value.code == mpc3.E_STATE
    assert c.verify_end()
    c.capture_begin()
    with pytest.raises(mpc3.Mpc3Error) as e:
        c.trim()
    assert e.value.code == mpc3.E_STATE
    with pytest.raises(mpc3.Mpc3Error):
        c.capture_end()
    assert c.trim() >= 0
    c.close()
