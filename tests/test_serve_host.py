"""Host logic of the request-packing server (no GPU): batch buckets, packing of a seeded
request mix into per-model packs, and the open-loop arrival times."""
import numpy as np
import pytest

serve = pytest.importorskip("paper_2411_09287_amd.serve")


@pytest.mark.parametrize("M", [1, 2, 3, 7, 64, 65, 1000, 1024, 1025])
def test_m_bucket_is_the_next_power_of_two(M):
    b = serve.m_bucket(M)
    assert b >= M and b & (b - 1) == 0 and (b == 1 or b // 2 < M)


@pytest.mark.parametrize("b,cap", [(1, 64), (5, 64), (33, 64), (64, 64), (65, 64), (100, 256), (300, 256)])
def test_bucket_of_caps_at_the_pack_limit(b, cap):
    bk = serve.bucket_of(b, cap)
    assert bk >= b
    assert bk == min(serve.m_bucket(b), max(cap, b))


def test_request_mix_is_seeded_and_in_range():
    a, b = serve.request_mix(256, seed=11), serve.request_mix(256, seed=11)
    assert a == b
    assert [r[0] for r in a] == list(range(256))
    assert all(r[1] in serve.MODEL_NAMES and 1 <= r[2] <= 64 for r in a)
    assert serve.request_mix(256, seed=12) != a


@pytest.mark.parametrize("pack", [True, False])
def test_packs_cover_every_request_once_per_model_in_order(pack):
    reqs = serve.request_mix(300, seed=3)
    cap = dict(serve.DEFAULT_CAP)
    packs = serve.packs_of(reqs, cap, pack)
    ids = [r[0] for p in packs for r in p]
    assert sorted(ids) == [r[0] for r in reqs]
    for p in packs:
        assert len({r[1] for r in p}) == 1                      # one model per pack
        assert [r[0] for r in p] == sorted(r[0] for r in p)      # arrival order inside
        n = sum(r[2] for r in p)
        assert n <= cap[p[0][1]] or len(p) == 1
        if not pack:
            assert len(p) == 1
    firsts = [p[0][0] for p in packs]
    assert firsts == sorted(firsts)                              # packs in first-request order
    if pack:
        # greedy: a pack is closed only when the model's next request would not fit
        for name in serve.MODEL_NAMES:
            mine = [p for p in packs if p[0][1] == name]
            for p, q in zip(mine, mine[1:]):
                assert sum(r[2] for r in p) + q[0][2] > cap[name]


def test_poisson_arrivals_increase_with_the_given_mean_gap():
    reqs = serve.request_mix(4000, seed=5)
    t = serve.poisson_arrivals(reqs, rate=50.0, seed=7)
    ts = np.array([t[r[0]] for r in reqs])
    assert np.all(np.diff(ts) > 0)
    gaps = np.diff(np.concatenate([[0.0], ts]))
    assert abs(gaps.mean() - 1 / 50.0) < 0.1 / 50.0
    assert t == serve.poisson_arrivals(reqs, rate=50.0, seed=7)
