"""Serving on the GPU: every result is the same alone and in the mix."""

import numpy as np
import pytest

from gpu_util import log
from paper_2306_08212_amd.serve import GpuBackend, Request, Server, summarize

pytestmark = pytest.mark.gpu


def _stream(n, seed0=0):
    rng = np.random.default_rng(123)
    out = []
    t = 0.0
    for i in range(n):
        D = int(rng.integers(2, 4))
        chi = int(rng.integers(D * D, 4 * D * D + 1))
        t += float(rng.exponential(0.05))
        out.append(Request(id=i, d=2, D=D, chi=chi, seed=seed0 + i, t_arrival=t,
                           max_iters=4, tol=0.0, precision=1))
    return out


def test_results_identical_alone_and_in_the_mix():
    reqs = _stream(8)
    be = GpuBackend()
    mixed = Server(be, budget_bytes=8 * 2 ** 30, max_slots=8).run(reqs)
    s = summarize(mixed)
    log("mix:", s)
    assert s["solves"] == len(reqs)
    for r in reqs:
        alone = Server(be, budget_bytes=8 * 2 ** 30, max_slots=1).run(
            [Request(**{**r.__dict__, "t_arrival": 0.0})])[0]
        m = mixed[r.id]
        log(f"req {r.id} D={r.D} chi={r.chi}: alone {alone.e_site!r} mix {m.e_site!r}")
        assert alone.iters == m.iters == r.max_iters
        assert alone.e_site == m.e_site          # bitwise
        assert alone.e_bond == m.e_bond
