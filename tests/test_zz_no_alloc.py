"""mpc3_inner_static (the allocation-free Pi_Inner, workspace in the library's fixed device
array) against mpc3_inner on the same seeds and call sequence: shares, messages counted,
verification transcript and opened values identical, bit for bit, on two calls in a row
(the second smaller, so it runs over the first call's leftovers in the array)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_09287_amd import mpc3  # noqa: E402

SEED = bytes(range(7, 39))


def u64(g, *shape):
    return g.integers(0, 1 << 64, size=shape, dtype=np.uint64, endpoint=False)


def run(static, variant, shapes, seed):
    """One context: share, truncation pair, Pi_Inner (static or not), truncation per shape;
    then verify and open.  Returns every share plane, the counters and the transcript."""
    g = np.random.default_rng(seed)
    c = mpc3.Context(SEED)
    c.set_variant(variant)
    out = []
    for M, K, N in shapes:
        X0, W0 = u64(g, M, K), u64(g, K, N)
        X, W = c.share(mpc3.to_words(X0)), c.share(mpc3.to_words(W0))
        pair = c.trunc_pair(M * N, 13)
        Z = c.inner_static(X, W, pair) if static else c.inner(X, W, pair)
        T = c.trunc(pair, Z)
        out.append((Z.numpy(), T))
    ok = c.verify()
    log = [c.verify_log(0, s) for s in (mpc3.LOG_R, mpc3.LOG_Z, mpc3.LOG_DELTA)]
    opened = [mpc3.from_words(c.reconstruct(T)) for _, T in out]
    comm = c.comm_stats()
    planes = [z for z, _ in out]
    c.close()
    return ok, planes, log, opened, comm


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("shapes", [
    # a 64 x 128-tile layer with B tiles beyond one XCD's L2, then a ragged small product
    [(2048, 1152, 256), (100, 300, 70)],
    # K long enough that the digit sums force a split (atomic adds into a zero-filled output),
    # then an aligned 64-column layer with fewer rows
    [(64, 5000, 64), (4096, 576, 64)],
])
def test_static_matches_allocating_entry_point(variant, shapes):
    a = run(False, variant, shapes, seed=len(shapes[0]) * 31 + shapes[0][1])
    b = run(True, variant, shapes, seed=len(shapes[0]) * 31 + shapes[0][1])
    assert a[0] and b[0], "honest verification failed"
    for za, zb in zip(a[1], b[1]):
        for pa, pb in zip(za, zb):
            assert np.array_equal(pa, pb)
    for la, lb in zip(a[2], b[2]):
        assert np.array_equal(la[0], lb[0]) and la[1:] == lb[1:]
    for oa, ob in zip(a[3], b[3]):
        assert np.array_equal(oa, ob)
    assert np.array_equal(a[4][0], b[4][0]) and a[4][1] == b[4][1]


def test_static_limits_and_state():
    c = mpc3.Context(SEED)
    # 2^24 outputs need 512 MiB of party sums: refused before any launch
    X = mpc3.DShare.empty(1 << 18, 8)
    W = mpc3.DShare.empty(8, 64)
    Z = mpc3.DShare.empty(1 << 18, 64)
    with pytest.raises(mpc3.Mpc3Error) as e:
        c.inner_static(X, W, out=Z)
    assert e.value.code == mpc3.E_LIMIT
    # message copies would need device memory
    c.keep_messages(True)
    Xs = c.share(mpc3.to_words(np.arange(6, dtype=np.uint64).reshape(2, 3)))
    Ws = c.share(mpc3.to_words(np.arange(12, dtype=np.uint64).reshape(3, 4)))
    with pytest.raises(mpc3.Mpc3Error) as e:
        c.inner_static(Xs, Ws)
    assert e.value.code == mpc3.E_STATE
    c.keep_messages(False)
    Z = c.inner_static(Xs, Ws)
    assert c.verify()
    want = (np.arange(6, dtype=np.uint64).reshape(2, 3) @ np.arange(12, dtype=np.uint64).reshape(3, 4))
    assert np.array_equal(mpc3.from_words(c.reconstruct(Z)), want)
