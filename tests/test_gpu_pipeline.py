"""mpc3_verify_begin / mpc3_verify_end: a batch's verification in flight while the next
batch's layers are evaluated on the context's stream.  Against a twin context that verifies
each batch synchronously in the same call order: every opened logit, every counter and the
batched instance's transcript agree bit for bit; the state rules (one verification in flight,
no opening or transcript read before it ends) hold; an injected error is still caught."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_09287_amd import mpc3, network, workloads  # noqa: E402

SEED = bytes(range(31, 63))


def images(name, b, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.rand((b,) + tuple(workloads.MODELS[name]["input"]), generator=g, dtype=torch.float64,
                      device="cuda")


def transcript(ctx):
    out = [ctx.verify_log(0, sl)[0] for sl in (mpc3.LOG_R, mpc3.LOG_Z, mpc3.LOG_DELTA)]
    _, R, _ = ctx.verify_log(0, mpc3.LOG_R)
    out += [ctx.verify_log(0, mpc3.LOG_ZETA, k)[0] for k in range(R)]
    return out


@pytest.mark.parametrize("name,batch", [("lenet", 3), ("vgg", 1)])
def test_pipelined_steps_match_synchronous(name, batch):
    xs = [images(name, batch, s) for s in (1, 2, 3)]
    # pipelined: forward(i), end(i-1), begin(i)
    ca = mpc3.Context(SEED)
    na = network.Network(ca, name)
    outs_a, logs_a = [], []
    for i, x in enumerate(xs):
        outs_a.append(na.forward(x))
        if i > 0:
            assert ca.verify_end()
            logs_a.append(transcript(ca))
        ca.verify_begin(-1, mpc3.VERIFY_INNER)
    assert ca.verify_end()
    logs_a.append(transcript(ca))
    assert ca.verify(-1, mpc3.VERIFY_TRUNC)
    opened_a = [ca.reconstruct(o) for o in outs_a]
    comm_a = ca.comm_stats()
    # synchronous twin in the same call order (forward, verify, forward, verify, ...)
    cb = mpc3.Context(SEED)
    nb = network.Network(cb, name)
    outs_b, logs_b = [], []
    for x in xs:
        outs_b.append(nb.forward(x))
        assert cb.verify(-1, mpc3.VERIFY_INNER)
        logs_b.append(transcript(cb))
    assert cb.verify(-1, mpc3.VERIFY_TRUNC)
    opened_b = [cb.reconstruct(o) for o in outs_b]
    comm_b = cb.comm_stats()
    for la, lb in zip(logs_a, logs_b):
        for a, b in zip(la, lb):
            assert np.array_equal(a, b)
    for a, b in zip(opened_a, opened_b):
        assert torch.equal(a, b)
    assert np.array_equal(comm_a[0], comm_b[0]) and comm_a[1] == comm_b[1]
    ca.close()
    cb.close()


def test_state_rules_while_in_flight():
    c = mpc3.Context(SEED)
    net = network.Network(c, "mlp")
    out = net.forward(images("mlp", 2, 5))
    c.verify_begin(-1, mpc3.VERIFY_ALL)
    for call in (lambda: c.verify_begin(-1, mpc3.VERIFY_ALL), lambda: c.verify(-1, mpc3.VERIFY_ALL),
                 lambda: c.verify_log(0, mpc3.LOG_R)):
        with pytest.raises(mpc3.Mpc3Error) as e:
            call()
        assert e.value.code == mpc3.E_STATE
    with pytest.raises(mpc3.Mpc3Error) as e:
        c.reconstruct(out)
    assert e.value.code == mpc3.E_UNVERIFIED
    assert c.verify_end()
    with pytest.raises(mpc3.Mpc3Error) as e:
        c.verify_end()
    assert e.value.code == mpc3.E_STATE
    c.reconstruct(out)
    c.close()


def test_injected_error_caught_through_begin_end():
    c = mpc3.Context(SEED)
    net = network.Network(c, "mlp")
    net.forward(images("mlp", 2, 6))
    c.inject(mpc3.SITE_VER_H0_M1, (0 << 16) | (1 << 8) | 7, 1)
    c.verify_begin(-1, mpc3.VERIFY_INNER)
    net.forward(images("mlp", 2, 7))          # the next batch's layers meanwhile
    assert not c.verify_end()
    c.close()
