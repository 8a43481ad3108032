"""The library's choice of R on a network model (mpc3_verify with MPC3_R_NETWORK) against the
host cost model over the per-instance message list (Sec. 5.1's trade-off of R on the LAN /
MAN / WAN settings), and the counted bytes of the chosen instance against that list."""
import numpy as np
import pytest

from paper_2411_09287_amd import netmodel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_09287_amd import mpc3  # noqa: E402

SEED = bytes(range(11, 43))


@pytest.mark.parametrize("net", ["LAN", "MAN", "WAN"])
@pytest.mark.parametrize("n", [1 << 12, 5000, 1 << 16])
def test_model_r_of_mult_verify(net, n):
    rtt, bw = netmodel.NETWORKS[net]
    g = np.random.default_rng(n)
    c = mpc3.Context(SEED)
    c.set_network(rtt * 1e3, bw / 1e6, 0.1)
    a = c.share(mpc3.to_words(g.integers(0, 1 << 63, (n, 1), dtype=np.uint64)))
    b = c.share(mpc3.to_words(g.integers(0, 1 << 63, (n, 1), dtype=np.uint64)))
    c.mult(a, b)
    before = c.comm_stats()
    assert c.verify(mpc3.R_NETWORK, mpc3.VERIFY_MULT)
    db, dr = netmodel.diff(c.comm_stats(), before)
    _, R, npad = c.verify_log(0, mpc3.LOG_R)
    want_R, _ = netmodel.model_r(n, 512, net, 0.1e-3)
    assert R == want_R
    wb, wr = netmodel.instance_messages(512, R, npad >> R)
    assert np.array_equal(db, np.array(wb, dtype=np.uint64)) and dr == wr


def test_model_r_of_boolean_instance():
    """A ReLU's Boolean triples are GF(2^64) elements of 8 bytes: the model picks their R
    with w = 8."""
    g = np.random.default_rng(3)
    n = 300
    x = g.integers(0, 1 << 40, (n, 1), dtype=np.uint64)
    c = mpc3.Context(SEED)
    rtt, bw = netmodel.NETWORKS["WAN"]
    c.set_network(rtt * 1e3, bw / 1e6, 0.1)
    c.relu(c.share(mpc3.to_words(x)))
    assert c.verify(mpc3.R_NETWORK)
    kinds = ["mult", "rows", "mult", "mult", "and", "mult"]
    for s, k in enumerate(kinds):
        _, R, npad = c.verify_log(s, mpc3.LOG_R)
        if k == "and":
            assert R == netmodel.model_r(64 * 11 * n, 8, "WAN", 0.1e-3)[0]


def test_network_mode_needs_a_model():
    c = mpc3.Context(SEED)
    a = c.share(mpc3.to_words(np.arange(4, dtype=np.uint64).reshape(4, 1)))
    c.mult(a, a)
    with pytest.raises(mpc3.Mpc3Error) as e:
        c.verify(mpc3.R_NETWORK)
    assert e.value.code == mpc3.E_STATE


@pytest.mark.parametrize("inj", [None, (mpc3.SITE_MULT_GAMMA2, 17, 1 << 40)])
def test_depth_circuit_verifies(inj):
    """A multiplication circuit of depth 12 (Fig. "dep"): the opened product equals the
    plaintext product mod 2^64 and every layer's triples verify; an error injected into
    one layer's message is caught."""
    g = np.random.default_rng(21)
    width, depth = 1000, 12
    c = mpc3.Context(SEED)
    rtt, bw = netmodel.NETWORKS["MAN"]
    c.set_network(rtt * 1e3, bw / 1e6, 0.1)
    x0 = g.integers(0, 1 << 64, (width, 1), dtype=np.uint64, endpoint=False)
    ys = [g.integers(0, 1 << 64, (width, 1), dtype=np.uint64, endpoint=False) for _ in range(depth)]
    X = c.share(mpc3.to_words(x0))
    Ys = [c.share(mpc3.to_words(y)) for y in ys]
    for k in range(depth):
        if inj and k == 5:
            c.inject(*inj)
        X = c.mult(X, Ys[k])
    ok = c.verify(mpc3.R_NETWORK)
    assert ok == (inj is None)
    if ok:
        want = x0.reshape(-1).copy()
        for y in ys:
            want = want * y.reshape(-1)
        assert np.array_equal(mpc3.from_words(c.reconstruct(X)).reshape(-1), want)
