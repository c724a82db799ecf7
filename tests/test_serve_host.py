"""Host logic of the serving loop (no GPU): the admission policy."""
import pytest

from paper_2605_25403_amd.serve import Request, admit


def reqs(specs):
    return [Request(id=i, t_arrive=t, n=n, k=3.14, nu=0.01, steps=5, dt=1e-3)
            for i, (t, n) in enumerate(specs)]


def fp(req):
    return {8: 10, 16: 40, 32: 160}[req.n]


def test_admits_only_arrived_requests_in_order():
    q = reqs([(0.0, 8), (0.1, 8), (0.5, 8)])
    assert admit(q, now=0.2, active_count=0, active_bytes=0, footprint_of=fp,
                 max_slots=10, hbm_budget=1000) == 2


def test_slot_cap_limits_admission():
    q = reqs([(0.0, 8)] * 5)
    assert admit(q, 1.0, 3, 0, fp, max_slots=4, hbm_budget=1000) == 1
    assert admit(q, 1.0, 4, 0, fp, max_slots=4, hbm_budget=1000) == 0


def test_footprint_budget_limits_admission_head_of_line():
    q = reqs([(0.0, 16), (0.0, 32), (0.0, 8)])
    # 40 fits (used 40 + 100 = 140 <= 200); 160 does not; the small one behind waits
    assert admit(q, 1.0, 1, 100, fp, max_slots=10, hbm_budget=200) == 1
    # an idle server admits even a request that fills the whole budget
    assert admit(reqs([(0.0, 32)]), 1.0, 0, 0, fp, max_slots=10, hbm_budget=160) == 1


def test_request_larger_than_budget_is_an_error():
    with pytest.raises(ValueError):
        admit(reqs([(0.0, 32)]), 1.0, 0, 0, fp, max_slots=10, hbm_budget=100)


def test_serving_stream_is_seeded_and_shaped():
    from paper_2605_25403_amd.workloads import serving_requests
    a = serving_requests(seed=0, count=256)
    b = serving_requests(seed=0, count=256)
    assert a == b
    assert len(a) == 256 and {r["n"] for r in a} <= {32, 64, 128, 256}
    t = [r["t_arrive"] for r in a]
    assert all(x < y for x, y in zip(t, t[1:]))
    # Poisson arrivals at 20/s: 256 arrivals take about 12.8 s
    assert 9.0 < t[-1] < 17.0
