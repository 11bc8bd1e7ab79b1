"""CPU checks of the serving driver's seeded request stream."""
import numpy as np

from paper_2111_09512_amd import serve as S


def test_pool_spec_seeded_and_in_range():
    a = S.pool_spec()
    assert a == S.pool_spec() and len(a) == 64
    assert set(a) <= set(S.SIDES)


def test_request_plan_shape_and_rate():
    plan = S.request_plan(64)
    assert len(plan) == 1280 and plan == S.request_plan(64)
    mids = [p[0] for p in plan]
    assert all(mids.count(m) == 20 for m in range(64))  # 20 right-hand sides per matrix
    assert len({p[1] for p in plan}) == 1280
    outers = np.array([p[2] for p in plan])
    assert outers.min() == 1 and outers.max() == 4
    t = np.array([p[3] for p in plan])
    assert np.all(np.diff(t) > 0)
    rate = (len(t) - 1) / (t[-1] - t[0])
    assert 1800 < rate < 2200  # Poisson arrivals at 2000 requests/s
