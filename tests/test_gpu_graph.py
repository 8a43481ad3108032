"""Recorded forward passes (mpc3_capture_begin / mpc3_capture_end / mpc3_graph_launch): the
linear forward of a network replayed as a HIP graph against the same calls made directly
on a second context with the same seed and history.  Shares, counted messages, verification
transcripts and opened logits must agree bit for bit on every replay, each replay must draw
fresh masks, and a replay's products must really be verified (a corrupted output word is
caught).  The graph may hold kernel nodes only."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_09287_amd import mpc3, network, serve, workloads  # noqa: E402

SEED = bytes(range(11, 43))


def images(name, b, seed):
    shape = (b,) + tuple(workloads.MODELS[name]["input"])
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.rand(shape, generator=g, dtype=torch.float64, device="cuda")


def planes(s):
    return [t.clone() for t in (s.m, s.r1, s.r2)]


def step_record(ctx, out):
    ok = ctx.verify()
    log = [ctx.verify_log(i, sl)[0] for i in (0, 1) for sl in (mpc3.LOG_R, mpc3.LOG_Z, mpc3.LOG_DELTA)]
    shares = planes(out)
    opened = ctx.reconstruct(out).clone()
    b, r = ctx.comm_stats()
    return ok, shares, log, opened, (b.copy(), list(r))


@pytest.mark.parametrize("name,batch,variant", [("mlp", 3, 1), ("lenet", 2, 1), ("lenet", 2, 0), ("snn", 2, 1)])
def test_replays_match_direct_calls(name, batch, variant):
    ca = mpc3.Context(SEED, stream=torch.cuda.Stream())
    cb = mpc3.Context(SEED)
    for c in (ca, cb):
        c.set_variant(variant)
    na, nb = network.Network(ca, name), network.Network(cb, name)
    rf = network.RecordedForward(na, batch)
    kern, other = rf.nodes()
    assert other == 0 and kern >= 3 * len(na.plan), (kern, other)
    xs = [images(name, batch, 1), images(name, batch, 1), images(name, batch - 1, 2)]
    prev = None
    for i, x in enumerate(xs):
        a = step_record(ca, rf(x))
        xb = x if x.shape[0] == batch else torch.cat([x, torch.zeros_like(x[:batch - x.shape[0]])])
        b = step_record(cb, nb.forward(xb))
        assert a[0] and b[0], f"replay {i}: honest verification failed"
        for pa, pb in zip(a[1], b[1]):
            assert torch.equal(pa, pb), f"replay {i}: shares differ"
        for la, lb in zip(a[2], b[2]):
            assert np.array_equal(la, lb), f"replay {i}: transcripts differ"
        assert torch.equal(a[3], b[3])
        assert np.array_equal(a[4][0], b[4][0]) and a[4][1] == b[4][1], f"replay {i}: counters differ"
        if prev is not None and i == 1:
            # the same images again under fresh masks: other shares, and the same logits up to
            # the last bits, which the probabilistic truncation draws from the masks
            assert not torch.equal(a[1][1], prev[1][1])
            assert int((a[3] - prev[3]).abs().max()) <= 64
        prev = a
    rf.close()
    ca.close()
    cb.close()


def test_replay_products_are_verified():
    c = mpc3.Context(SEED, stream=torch.cuda.Stream())
    net = network.Network(c, "mlp")
    rf = network.RecordedForward(net, 4)
    x = images("mlp", 4, 3)
    rf(x)
    assert c.verify()
    rf(x)
    # an additive error on one output word of the first layer's Pi_Inner (P1's message)
    with torch.cuda.stream(c.stream):
        rf.layers[0]["Z"].m[1, 2] += 1
    assert not c.verify(kinds=mpc3.VERIFY_INNER)
    c.close()


def test_replay_refused_while_its_products_are_pending():
    c = mpc3.Context(SEED, stream=torch.cuda.Stream())
    net = network.Network(c, "mlp")
    rf = network.RecordedForward(net, 2)
    x = images("mlp", 2, 4)
    rf(x)
    with pytest.raises(mpc3.Mpc3Error) as e:
        rf(x)
    assert e.value.code == mpc3.E_STATE
    assert c.verify(kinds=mpc3.VERIFY_INNER)
    with pytest.raises(mpc3.Mpc3Error):          # the truncation gates are still pending
        rf(x)
    assert c.verify()
    rf(x)
    assert c.verify()
    c.close()


def test_recording_rejects_calls_that_allocate_or_synchronise():
    import ctypes

    L = mpc3.lib()
    ca = mpc3.Context(SEED, stream=torch.cuda.Stream())
    cb = mpc3.Context(SEED)
    x = mpc3.to_words(np.arange(12, dtype=np.uint64).reshape(3, 4))
    ca.share(x), cb.share(x)
    s = mpc3.DShare.empty(3, 4)
    torch.cuda.synchronize()
    before = ca.comm_stats()
    ca.capture_begin()
    ca.share(x, out=s)                           # recorded
    sc, ok, comm = s.c(), ctypes.c_int(0), mpc3.Comm()
    codes = [L.mpc3_verify(ca.h, -1, mpc3.VERIFY_ALL, ctypes.byref(ok)),
             L.mpc3_comm_stats(ca.h, ctypes.byref(comm)),
             L.mpc3_mult(ca.h, ctypes.byref(sc), ctypes.byref(sc), ctypes.byref(sc)),
             L.mpc3_inner(ca.h, ctypes.byref(sc), ctypes.byref(sc), None, ctypes.byref(sc)),
             L.mpc3_inject(ca.h, mpc3.SITE_INNER_M1, 0, 1),
             L.mpc3_capture_begin(ca.h)]
    assert codes == [mpc3.E_STATE] * len(codes), codes
    with pytest.raises(mpc3.Mpc3Error) as e:
        ca.capture_end()
    assert e.value.code == mpc3.E_STATE
    # nothing of the failed recording is left: the next direct call draws what it would have
    after = ca.comm_stats()
    assert np.array_equal(after[0], before[0]) and after[1] == before[1]
    a, b = ca.share(x), cb.share(x)
    for pa, pb in zip(a.numpy(), b.numpy()):
        assert np.array_equal(pa, pb)
    ca.close()
    cb.close()


def test_recording_fails_with_a_recorded_call():
    """A call refused by its own checks while recording (here the fixed workspace's limit)
    makes the recording fail with that code; no graph is left behind."""
    c = mpc3.Context(SEED, stream=torch.cuda.Stream())
    X, W, Z = mpc3.DShare.empty(1 << 18, 8), mpc3.DShare.empty(8, 64), mpc3.DShare.empty(1 << 18, 64)
    torch.cuda.synchronize()
    c.capture_begin()
    with pytest.raises(mpc3.Mpc3Error) as e:
        c.inner_static(X, W, out=Z)
    assert e.value.code == mpc3.E_LIMIT
    with pytest.raises(mpc3.Mpc3Error) as e:
        c.capture_end()
    assert e.value.code == mpc3.E_LIMIT
    with pytest.raises(mpc3.Mpc3Error) as e:
        c.graph_launch(1)
    assert e.value.code == mpc3.E_ARG
    c.close()


def test_recording_needs_a_stream_of_its_own():
    c = mpc3.Context(SEED, stream=torch.cuda.default_stream())
    with pytest.raises(mpc3.Mpc3Error) as e:
        c.capture_begin()
    assert e.value.code == mpc3.E_STATE
    c.close()


def test_server_with_graphs_matches_direct_packs():
    """Packs replayed from graphs recorded per (model, batch bucket) open to the same logits
    as the same packs, padded to the same buckets, evaluated by direct calls (the same
    masks: the probabilistic truncation makes the last bits depend on them)."""
    reqs = [(0, "mlp", 3), (1, "lenet", 2), (2, "mlp", 5), (3, "lenet", 1), (4, "mlp", 2)]
    cap = {"mlp": 8, "lenet": 4, "vgg": 2}
    ca = mpc3.Context(SEED, stream=torch.cuda.Stream())
    cb = mpc3.Context(SEED, stream=torch.cuda.Stream())
    sa = serve.Server(ca, models=("mlp", "lenet"), cap=cap, graphs=True)
    sb = serve.Server(cb, models=("mlp", "lenet"), cap=cap, graphs=False, buckets=True)
    # arrivals far closer together than a pack's service time, so that the packs (and so
    # the masks) do not depend on the measured times
    arr = serve.poisson_arrivals(reqs, rate=1e8)
    for kw in ({}, {"arrivals": arr}):
        ra = sa.run(reqs, keep_logits=True, **kw)
        rb = sb.run(reqs, keep_logits=True, **kw)
        assert ra["ok"] and rb["ok"]
        assert ra["graph_packs"] > 0 and rb["graph_packs"] == 0
        assert set(ra["latency"]) == {r[0] for r in reqs}
        for r in reqs:
            la, lb = ra["logits"][r[0]], rb["logits"][r[0]]
            assert la.shape == (r[2], 10) and torch.equal(la, lb)
    ca.close()
    cb.close()


def test_server_auto_graphs_matches_direct_packs():
    """graphs="auto": every (model, bucket) up to the cap gets a measured pick, and packs
    served with the picked graphs (the others unpadded, by direct calls) open to the same
    logits as a twin server that makes the same calls directly (its tuning makes the same
    forwards and it pads the same packs, so both draw the same masks)."""
    reqs = [(0, "mlp", 3), (1, "lenet", 2), (2, "mlp", 5), (3, "lenet", 1), (4, "mlp", 2)]
    cap = {"mlp": 8, "lenet": 4, "vgg": 2}
    ca = mpc3.Context(SEED, stream=torch.cuda.Stream())
    cb = mpc3.Context(SEED, stream=torch.cuda.Stream())
    sa = serve.Server(ca, models=("mlp", "lenet"), cap=cap, graphs="auto")
    sb = serve.Server(cb, models=("mlp", "lenet"), cap=cap, graphs=False, buckets="picked")
    pa = sa.tune_graphs(reps=1)
    sb.tune_graphs(reps=1)
    sb.graph_pick = dict(pa)
    assert set(pa) == {("mlp", b) for b in (1, 2, 4, 8)} | {("lenet", b) for b in (1, 2, 4)}
    ra = sa.run(reqs, keep_logits=True)
    rb = sb.run(reqs, keep_logits=True)
    assert ra["ok"] and rb["ok"] and rb["graph_packs"] == 0
    picked = sum(int(pa[(p[0][1], serve.bucket_of(sum(r[2] for r in p), cap[p[0][1]]))])
                 for p in serve.packs_of(reqs, cap))
    assert ra["graph_packs"] == picked
    for r in reqs:
        assert torch.equal(ra["logits"][r[0]], rb["logits"][r[0]])
    ca.close()
    cb.close()
