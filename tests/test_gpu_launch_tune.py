"""Launch shapes of the limb kernel (mpc3_set_launch, mpc3_autotune_launch): every shape the
tuner tries gives the built-in launch's shares, counters and Pi_BIVerify transcript bit for
bit (dense shapes with one and two column tiles per workgroup, a ragged K that takes the
slow path, a product whose K is split), and the tuner's pick is one of its candidates."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_09287_amd import mpc3  # noqa: E402

SEED = bytes(range(41, 73))
SHAPES = [(2048, 576, 128), (1000, 300, 130), (256, 2304, 256), (4096, 64, 64)]
LAUNCHES = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 4, 0), (1, 16, 0), (0, 64, 2), (1, 1, 2), (0, 0, 2)]


def u64(g, *shape):
    return g.integers(0, 1 << 64, size=shape, dtype=np.uint64, endpoint=False)


def run(M, K, N, launch=None, tune=False):
    g = np.random.default_rng(M + K + N)
    c = mpc3.Context(SEED)
    c.set_variant(mpc3.VARIANT_LIMB_I8)
    picked = None
    if tune:
        picked = c.autotune_launch(M, K, N, reps=2)
    elif launch is not None:
        c.set_launch(M, K, N, *launch)
    X = c.share(mpc3.to_words(u64(g, M, K)))
    W = c.share(mpc3.to_words(u64(g, K, N)))
    Z = c.inner(X, W)
    planes = Z.numpy()
    ok = c.verify(-1, mpc3.VERIFY_INNER)
    _, R, _ = c.verify_log(0, mpc3.LOG_R)
    log = [c.verify_log(0, sl)[0] for sl in (mpc3.LOG_R, mpc3.LOG_Z, mpc3.LOG_DELTA)]
    log += [c.verify_log(0, mpc3.LOG_ZETA, k)[0] for k in range(R)]
    comm = c.comm_stats()
    c.close()
    return ok, planes, log, comm, picked


@pytest.mark.parametrize("shape", SHAPES)
def test_every_launch_shape_is_bit_identical(shape):
    ref = run(*shape)
    assert ref[0]
    for launch in LAUNCHES[1:]:
        out = run(*shape, launch=launch)
        assert out[0], launch
        for a, b in zip(out[1], ref[1]):
            assert np.array_equal(a, b), launch
        for a, b in zip(out[2], ref[2]):
            assert np.array_equal(a, b), launch
        assert np.array_equal(out[3][0], ref[3][0]) and out[3][1] == ref[3][1]


def test_tuner_pick_is_a_candidate_and_bit_identical():
    M, K, N = SHAPES[0]
    ref = run(M, K, N)
    out = run(M, K, N, tune=True)
    (ns, rb, split), ms_default, ms_best = out[4]
    assert ns in (0, 1) and rb in (0, 1, 2, 4, 8, 16, 32, 64) and split in (0, 2)
    assert 0 < ms_best <= ms_default
    if (ns, rb, split) != (0, 0, 0):
        assert ms_best < 0.98 * ms_default
    assert out[0]
    for a, b in zip(out[1], ref[1]):
        assert np.array_equal(a, b)


def test_set_launch_rejects_bad_arguments():
    c = mpc3.Context(SEED)
    for bad in ((2, 0, 0), (-1, 0, 0), (0, -1, 0), (0, 70000, 0), (0, 0, 17)):
        with pytest.raises(mpc3.Mpc3Error) as e:
            c.set_launch(64, 64, 64, *bad)
        assert e.value.code == mpc3.E_ARG
    c.set_launch(64, 64, 64, 1, 4, 2)
    c.set_launch(64, 64, 64)        # forget
    c.close()
