"""Host-only tests of the continuous-batching scheduler with a scripted
backend (virtual clock, scripted iteration times and workspace sizes)."""

import math

from paper_2306_08212_amd.serve import FakeBackend, Request, Server, summarize


def _reqs(n, gap=0.0, D=lambda i: 3 + i % 3, tol=1e-3, max_iters=30):
    return [Request(id=i, d=2, D=D(i), chi=D(i) ** 2, seed=i, t_arrival=i * gap,
                    tol=tol, max_iters=max_iters) for i in range(n)]


def test_all_requests_finish_with_expected_iterations():
    be = FakeBackend(10 ** 12, iter_time=lambda r: 0.01 * r.D, bytes_of=lambda r: 1000)
    res = Server(be, budget_bytes=10 ** 9, max_slots=4).run(_reqs(10, gap=0.005))
    assert [r.id for r in res] == list(range(10))
    need = math.ceil(math.log2(1.0 / 1e-3))       # delta halves from 1 until < tol
    for r in res:
        assert r.status == "ok" and r.iters == need and r.e_site == -0.5


def test_max_iters_caps_a_solve():
    be = FakeBackend(10 ** 12, iter_time=lambda r: 0.01, bytes_of=lambda r: 1)
    res = Server(be, budget_bytes=100, max_slots=2).run(_reqs(3, tol=1e-30, max_iters=5))
    assert all(r.iters == 5 for r in res)


def test_budget_and_slots_are_respected():
    size = lambda r: 100 * r.D ** 3
    be = FakeBackend(10 ** 12, iter_time=lambda r: 0.02, bytes_of=size)
    budget = 100 * (5 ** 3 + 4 ** 3)
    srv = Server(be, budget_bytes=budget, max_slots=3)
    res = srv.run(_reqs(12, gap=0.001))
    assert len(res) == 12
    assert be.peak_bytes <= budget
    assert be.max_concurrent <= 3
    assert srv.used == 0 and not srv.active


def test_fifo_admission_and_latency_bookkeeping():
    # one slot, fixed 0.1 s per iteration, 10 iterations each: serial service
    be = FakeBackend(10 ** 12, iter_time=lambda r: 0.1, bytes_of=lambda r: 1)
    reqs = _reqs(4, gap=0.0, tol=0.6 ** 10 * 1.1, max_iters=50)
    res = Server(be, budget_bytes=10, max_slots=1).run(reqs)
    admits = sorted(res, key=lambda r: r.t_admit)
    assert [r.id for r in admits] == [0, 1, 2, 3]
    for r in res:
        assert abs(r.latency - (r.id + 1) * r.iters * 0.1) < 1e-9
    s = summarize(res)
    assert s["solves"] == 4 and s["p50_s"] <= s["p99_s"]
    assert abs(s["solves_per_s"] - 4 / (4 * res[0].iters * 0.1)) < 1e-9


def test_request_larger_than_budget_is_rejected():
    be = FakeBackend(10 ** 12, iter_time=lambda r: 0.01, bytes_of=lambda r: 10 ** 6 * r.D)
    srv = Server(be, budget_bytes=4 * 10 ** 6, max_slots=4)
    res = srv.run(_reqs(6))
    assert sorted(srv.rejected) == [i for i in range(6) if 3 + i % 3 > 4]
    assert all(r.D <= 4 for r in res)


def test_numeric_failure_is_isolated():
    be = FakeBackend(10 ** 12, iter_time=lambda r: 0.01, bytes_of=lambda r: 1, fail_ids=[2])
    res = Server(be, budget_bytes=100, max_slots=4).run(_reqs(5))
    st = {r.id: r.status for r in res}
    assert st[2] == "numeric" and all(st[i] == "ok" for i in (0, 1, 3, 4))
    assert summarize(res)["failed"] == 1


def test_later_arrivals_overlap_running_solves():
    """A request arriving while others run is admitted before they finish."""
    be = FakeBackend(10 ** 12, iter_time=lambda r: 0.05, bytes_of=lambda r: 1)
    res = Server(be, budget_bytes=100, max_slots=8).run(_reqs(4, gap=0.03))
    first_done = min(r.t_done for r in res)
    assert sum(r.t_admit < first_done for r in res) >= 3


def test_warm_start_environment_is_passed_and_returned():
    """A request's starting environment reaches the backend's solve, and
    return_env hands the final one back (the FFU-style reuse of
    environments between optimisation steps)."""
    be = FakeBackend(10 ** 12, iter_time=lambda r: 0.01, bytes_of=lambda r: 1)
    reqs = _reqs(3, tol=1e-30, max_iters=4)
    reqs[1].env = {"C1a": "start-env"}
    reqs[1].return_env = True
    reqs[2].return_env = True
    res = Server(be, budget_bytes=100, max_slots=2).run(reqs)
    assert res[0].env is None
    assert res[1].env == {"iterations": 4, "start": {"C1a": "start-env"}}
    assert res[2].env == {"iterations": 4, "start": None}
