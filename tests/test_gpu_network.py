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


def fp64_forward(name, x):
    """FP64 model on the decoded fixed-point input and weights (conv as im2col products)."""
    from oracle.layers import im2col
    frac = workloads.FRAC_BITS
    ws = [o_decode(o_encode(w, frac), frac) for w in network.float_weights(name)]
    h = o_decode(o_encode(x, frac), frac)
    B = x.shape[0]
    for d, w in zip(network.plan(name), ws):
        layer = d["layer"]
        if layer[0] == "conv":
            _, kh, kw, cin, cout, pad, (hh, ww) = layer
            # im2col on float planes through the integer routine's indexing (values as float)
            xi = h.reshape(B, hh, ww, cin)
            xp = np.zeros((B, hh + 2 * pad, ww + 2 * pad, cin))
            xp[:, pad:pad + hh, pad:pad + ww] = xi
            oh, ow = hh + 2 * pad - kh + 1, ww + 2 * pad - kw + 1
            cols = np.zeros((B, oh, ow, kh, kw, cin))
            for i in range(kh):
                for j in range(kw):
                    cols[:, :, :, i, j] = xp[:, i:i + oh, j:j + ow]
            y = cols.reshape(B * oh * ow, -1) @ w
            if d["pool_after"]:
                y = y.reshape(B, oh // 2, 2, ow // 2, 2, cout).sum(axis=(2, 4))
            h = y.reshape(B, -1)
        else:
            h = h.reshape(B, -1) @ w
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
