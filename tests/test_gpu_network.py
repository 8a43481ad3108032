"""Chained secure networks on the GPU: sum pooling parity, decoded outputs against an FP64
model of the same linear network, the autotuner and the request-packing server."""
import numpy as np
import pytest

from oracle.layers import sumpool2_share
from oracle.protocol import Ctx
from oracle.ring import decode as o_decode
from oracle.ring import encode as o_encode

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_09287_amd import mpc3, network, serve, workloads  # noqa: E402

SEED = bytes(range(7, 39))


def u64(g, *shape):
    return g.integers(0, 1 << 64, size=shape, dtype=np.uint64, endpoint=False)


@pytest.mark.parametrize("B,H,W,C", [(1, 2, 2, 1), (2, 6, 4, 3), (3, 8, 8, 5)])
def test_sumpool_parity(B, H, W, C):
    g = np.random.default_rng(H * W)
    x0 = u64(g, B, H * W * C)
    o = Ctx(SEED)
    c = mpc3.Context(SEED)
    xo, xg = o.share(x0), c.share(mpc3.to_words(x0))
    po = sumpool2_share(xo, B, H, W, C)
    pg = c.sumpool2(xg, B, H, W, C)
    for a, b in zip(pg.numpy(), po.comps()):
        assert np.array_equal(a.reshape(-1), b.reshape(-1))


def fp64_forward(name, x, nonlinear=False):
    """FP64 model on the decoded fixed-point input and weights (conv as im2col products;
    with nonlinear, ReLU after every layer but the last and 2x2 max pooling, else 2x2 sum
    pooling)."""
    from oracle.layers import im2col
    frac = workloads.FRAC_BITS
    ws = [o_decode(o_encode(w, frac), frac) for w in network.float_weights(name, nonlinear=nonlinear)]
    h = o_decode(o_encode(x, frac), frac)
    B = x.shape[0]
    plan = network.plan(name)
    for li, (d, w) in enumerate(zip(plan, ws)):
        layer = d["layer"]
        act = nonlinear and li + 1 < len(plan)
        if layer[0] == "conv":
            _, kh, kw, cin, cout, pad, (hh, ww) = layer[:7]
            st = workloads.conv_stride(layer)
            # patches of the padded float input: output (oh, ow) reads (st oh + i - pad, st ow + j - pad)
            xi = h.reshape(B, hh, ww, cin)
            xp = np.zeros((B, hh + 2 * pad, ww + 2 * pad, cin))
            xp[:, pad:pad + hh, pad:pad + ww] = xi
            oh, ow = workloads.conv_out_hw(layer)
            cols = np.zeros((B, oh, ow, kh, kw, cin))
            for i in range(kh):
                for j in range(kw):
                    cols[:, :, :, i, j] = xp[:, i:i + st * (oh - 1) + 1:st, j:j + st * (ow - 1) + 1:st]
            y = cols.reshape(B * oh * ow, -1) @ w
            if act:
                y = np.maximum(y, 0.0)
            if d["pool_after"]:
                y = y.reshape(B, oh // 2, 2, ow // 2, 2, cout)
                y = y.max(axis=(2, 4)) if nonlinear else y.sum(axis=(2, 4))
            h = y.reshape(B, -1)
        else:
            h = h.reshape(B, -1) @ w
            if act:
                h = np.maximum(h, 0.0)
    del im2col
    return h


@pytest.mark.parametrize("name,batch", [("mlp", 16), ("lenet", 4), ("vgg", 2)])
@pytest.mark.parametrize("variant", [mpc3.VARIANT_U64, mpc3.VARIANT_LIMB_I8])
def test_network_matches_fp64_model(name, batch, variant):
    c = mpc3.Context(workloads.master_seed(3))
    c.set_variant(variant)
    net = network.Network(c, name)
    x = workloads.rng(31).random((batch,) + tuple(workloads.MODELS[name]["input"]))
    out = net.forward(torch.from_numpy(x).cuda())
    assert c.verify()
    y = c.decode(c.reconstruct(out)).cpu().numpy().reshape(batch, -1)
    ref = fp64_forward(name, x)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err <= 2.0 ** -10, err


@pytest.mark.parametrize("name,batch,variant", [("mlp", 16, 0), ("mlp", 16, 1), ("lenet", 2, 0), ("lenet", 2, 1),
                                                ("snn", 4, 1)])
def test_nonlinear_network_matches_fp64_model(name, batch, variant):
    """ReLU and max pooling through edaBits (Sec. 4.3): every product verified (linear,
    truncation gates, Pi_Mult and the Boolean triples), decoded logits within 2^-10
    (normwise) of the FP64 model with ReLU and max pooling on the decoded inputs."""
    c = mpc3.Context(workloads.master_seed(2))
    c.set_variant(variant)
    net = network.Network(c, name, nonlinear=True)
    x = workloads.rng(33).random((batch,) + tuple(workloads.MODELS[name]["input"]))
    out = net.forward(torch.from_numpy(x).cuda())
    assert c.verify()
    y = c.decode(c.reconstruct(out)).cpu().numpy().reshape(batch, -1)
    ref = fp64_forward(name, x, nonlinear=True)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err <= 2.0 ** -10, err


def oracle_forward_nonlinear(o, name, x, batch):
    """The oracle through network.Network's calls with ReLU and max pooling."""
    from oracle.layers import im2col_share
    from oracle.protocol import Share

    frac = workloads.FRAC_BITS
    plan = network.plan(name)
    weights = []
    for d, w in zip(plan, network.float_weights(name, nonlinear=True)):
        if d.get("kpad", w.shape[0]) > w.shape[0]:
            w = np.concatenate([w, np.zeros((d["kpad"] - w.shape[0], w.shape[1]))])
        weights.append(o.share(o_encode(w, frac)))
    h = o.share(o_encode(x, frac).reshape(batch, -1))
    for i, (d, W) in enumerate(zip(plan, weights)):
        layer = d["layer"]
        if layer[0] == "conv":
            _, kh, kw, cin, cout, pad, (hh, ww) = layer[:7]
            X = im2col_share(h.map(lambda a: a.reshape(batch, hh, ww, cin)), kh, kw, pad, workloads.conv_stride(layer))
            extra = d["kpad"] - X.m.shape[1]
            if extra:
                X = X.map(lambda a: np.concatenate([a, np.zeros((a.shape[0], extra), dtype=np.uint64)], axis=1))
        else:
            X = h.map(lambda a: a.reshape(batch, -1))
        pair = o.trunc_pair(X.m.shape[0] * W.m.shape[1], frac)
        Y = o.trunc(pair, o.inner(X, W, pair))
        if i + 1 < len(plan):
            Y = o.relu(Y)
        if d["pool_after"]:
            oh, ow = d["out_hw"]
            Y = o.maxpool2(Y.map(lambda a: a.reshape(batch, -1)), batch, oh, ow, layer[4])
        h = Share(*[a.reshape(batch, -1) for a in Y.comps()])
    return h


@pytest.mark.parametrize("name,batch", [("mlp", 3), ("snn", 2), ("lenet5", 1)])
def test_nonlinear_network_chain_matches_oracle(name, batch):
    """A network with ReLU and max pooling against the oracle running the same calls on the
    same seeds: the shared logits bit for bit and the counted communication; the GPU then
    verifies every product and opens the oracle's logits.  (LeNet-5's small logits sit a few
    units in the last place of f = 13, beyond a 2^-10 comparison with an FP64 model; the
    bit-exact comparison covers it.)"""
    seed = workloads.master_seed(8)
    x = workloads.rng(34).random((batch,) + tuple(workloads.MODELS[name]["input"]))
    o = Ctx(seed)
    ho = oracle_forward_nonlinear(o, name, x, batch)
    c = mpc3.Context(seed)
    c.set_variant(mpc3.VARIANT_LIMB_I8)
    net = network.Network(c, name, nonlinear=True)
    hg = net.forward(torch.from_numpy(x).cuda())
    for a, b in zip(hg.numpy(), ho.comps()):
        assert np.array_equal(a.reshape(-1), b.reshape(-1))
    bg, rg = c.comm_stats()
    assert np.array_equal(bg, np.array(o.comm, dtype=np.uint64)) and rg == o.rounds
    assert c.verify()
    assert np.array_equal(mpc3.from_words(c.reconstruct(hg)).reshape(-1), ho.value().reshape(-1))


def test_autotune_records_a_choice_and_auto_matches():
    c = mpc3.Context(SEED)
    choice, t_u64, t_limb = c.autotune(256, 576, 64, reps=3)
    assert choice in (mpc3.VARIANT_U64, mpc3.VARIANT_LIMB_I8) and t_u64 > 0 and t_limb > 0
    g = np.random.default_rng(4)
    X0, W0 = u64(g, 256, 576), u64(g, 576, 64)
    outs = []
    for v in (mpc3.VARIANT_U64, mpc3.VARIANT_AUTO):
        cc = mpc3.Context(SEED)
        cc.set_variant(v)
        if v == mpc3.VARIANT_AUTO:
            cc.autotune(256, 576, 64, reps=2)
        outs.append(cc.inner(cc.share(mpc3.to_words(X0)), cc.share(mpc3.to_words(W0))).numpy())
    assert all(np.array_equal(a, b) for a, b in zip(*outs))


def test_server_packs_and_verifies_small_mix():
    reqs = [(0, "mlp", 3), (1, "lenet", 2), (2, "mlp", 5), (3, "mlp", 1), (4, "lenet", 1)]
    c = mpc3.Context(SEED)
    c.set_chunk(1 << 12)
    srv = serve.Server(c, models=("mlp", "lenet"), cap={"mlp": 8, "lenet": 4, "vgg": 4})
    packed = serve.packs_of(reqs, srv.cap)
    assert [[r[0] for r in p] for p in packed] == [[0, 2], [1, 4], [3]]
    res = srv.run(reqs)
    assert res["ok"] and set(res["latency"]) == {0, 1, 2, 3, 4}
    s = serve.summary(res)
    assert s["images"] == 12 and s["p50_ms"] <= s["p99_ms"]


def oracle_forward(o, name, x, batch):
    """The oracle through the call sequence of network.Network (weights shared first with
    the convolutions' zero-padded rows, then per layer: im2col with zero columns up to the
    padded width, truncation pair, Pi_Inner, truncation, sum pooling)."""
    from oracle.layers import im2col_share
    from oracle.protocol import Share

    frac = workloads.FRAC_BITS
    plan = network.plan(name)
    weights = []
    for d, w in zip(plan, network.float_weights(name)):
        if d.get("kpad", w.shape[0]) > w.shape[0]:
            w = np.concatenate([w, np.zeros((d["kpad"] - w.shape[0], w.shape[1]))])
        weights.append(o.share(o_encode(w, frac)))
    h = o.share(o_encode(x, frac).reshape(batch, -1))
    for d, W in zip(plan, weights):
        layer = d["layer"]
        if layer[0] == "conv":
            _, kh, kw, cin, cout, pad, (hh, ww) = layer[:7]
            X = im2col_share(h.map(lambda a: a.reshape(batch, hh, ww, cin)), kh, kw, pad, workloads.conv_stride(layer))
            extra = d["kpad"] - X.m.shape[1]
            if extra:
                X = X.map(lambda a: np.concatenate([a, np.zeros((a.shape[0], extra), dtype=np.uint64)], axis=1))
        else:
            X = h.map(lambda a: a.reshape(batch, -1))
        M, N = X.m.shape[0], W.m.shape[1]
        pair = o.trunc_pair(M * N, frac)
        Y = o.trunc(pair, o.inner(X, W, pair))
        if d["pool_after"]:
            oh, ow = d["out_hw"]
            Y = sumpool2_share(Y.map(lambda a: a.reshape(batch, -1)), batch, oh, ow, layer[4])
        h = Share(*[a.reshape(batch, -1) for a in Y.comps()])
    return h


_ORACLE_NET = {}


@pytest.mark.parametrize("name,batch", [("lenet", 4), ("vgg", 2), ("snn", 3)])
@pytest.mark.parametrize("variant", [mpc3.VARIANT_U64, mpc3.VARIANT_LIMB_I8])
def test_network_chain_matches_oracle(name, batch, variant):
    """The chained network against the oracle running the same calls on the same seeds:
    every layer's shares, the whole transcript of the batched verification of all the
    layer products (r, z, every zeta, the h(0) / h(x) messages, Delta and its messages),
    and the opened logits, bit for bit; the truncation gates then verify on the GPU."""
    seed = workloads.master_seed(4)
    x = workloads.rng(32).random((batch,) + tuple(workloads.MODELS[name]["input"]))
    if (name, batch) not in _ORACLE_NET:      # the oracle's side is the same for both variants
        o = Ctx(seed)
        ho = oracle_forward(o, name, x, batch)
        assert o.verify(kinds=1)
        _ORACLE_NET[(name, batch)] = (ho, o.vlog[0])
    ho, log = _ORACLE_NET[(name, batch)]
    c = mpc3.Context(seed)
    c.set_variant(variant)
    net = network.Network(c, name)
    hg = net.forward(torch.from_numpy(x).cuda())
    for a, b in zip(hg.numpy(), ho.comps()):
        assert np.array_equal(a.reshape(-1), b.reshape(-1))
    assert c.verify(kinds=mpc3.VERIFY_INNER)
    r, R, dim = c.verify_log(0, mpc3.LOG_R)
    assert np.array_equal(r, log["r"]) and R == log["R"] and dim == log["npad"]
    assert R >= 7
    assert np.array_equal(c.verify_log(0, mpc3.LOG_Z)[0], log["z"].m)
    for k, rl in enumerate(log["rounds"]):
        assert np.array_equal(c.verify_log(0, mpc3.LOG_ZETA, k)[0], rl["zeta"]), k
        for slot, key in [(mpc3.LOG_H0_M1, "m1"), (mpc3.LOG_H0_M2, "m2"), (mpc3.LOG_H0_G2, "gamma2")]:
            assert np.array_equal(c.verify_log(0, slot, k)[0], rl["h0"][key]), (k, key)
        for slot, key in [(mpc3.LOG_H2_M1, "m1"), (mpc3.LOG_H2_M2, "m2"), (mpc3.LOG_H2_G2, "gamma2")]:
            assert np.array_equal(c.verify_log(0, slot, k)[0], rl["h2"][key]), (k, key)
    assert np.array_equal(c.verify_log(0, mpc3.LOG_DELTA)[0], log["delta"])
    for slot, key in [(mpc3.LOG_DELTA_M1, "m1"), (mpc3.LOG_DELTA_M2, "m2"), (mpc3.LOG_DELTA_G2, "gamma2")]:
        assert np.array_equal(c.verify_log(0, slot)[0], log["delta_tr"][key]), key
    assert c.verify(kinds=mpc3.VERIFY_TRUNC)
    logits = mpc3.from_words(c.reconstruct(hg)).reshape(-1)
    assert np.array_equal(logits, ho.value().reshape(-1))
