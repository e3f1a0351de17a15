"""Graph replay of moves (ctm_set_graphs): a move whose launch sequence comes
up a second time is captured into a HIP graph and replayed afterwards.  The
graph holds the same kernels with the same arguments, so every replay must
give bitwise the environment of eager launches.  Each iteration below is
followed by reads of all 16 tensors (synchronising copies), so replays
alternate with the program's own eager work, as they do in use."""

import numpy as np
import pytest

import oracle as O
import paper_2306_08212_amd as P
from gpu_util import log
from synth import site_tensors

pytestmark = pytest.mark.gpu


def _env(s):
    return [s.get_env(P.env_index(n)) for n in O.ENV_KEYS]


@pytest.mark.parametrize("D,chi,prec", [(2, 8, P.FP64), (3, 16, P.FP32), (4, 20, P.BF16)])
def test_replay_bitwise_equal_to_eager(D, chi, prec):
    log("graph replay", D, chi, prec)
    A, B = site_tensors(2, D, 3)
    cfg = P.Config(d=2, D=D, chi=chi, method=P.REDUCED, precision=prec)
    eager = P.Solver(cfg, A, B)
    eager.set_graphs(False)
    graph = P.Solver(cfg, A, B)
    # iteration 1 is the bootstrap, 2 sees each key once, 3 captures, 4.. replay
    for it in range(6):
        eager.iterate(1)
        graph.iterate(1)
        for name, a, b in zip(O.ENV_KEYS, _env(eager), _env(graph)):
            assert a.shape == b.shape, (it, name)
            assert np.array_equal(a, b), (it, name, np.abs(a - b).max())
    # single moves in every direction replay too
    for mv in (0, 2, 1, 3, 0):
        eager.move(mv)
        graph.move(mv)
        for name, a, b in zip(O.ENV_KEYS, _env(eager), _env(graph)):
            assert np.array_equal(a, b), (mv, name)
    ea, eb = eager.energy(), graph.energy()
    assert ea[0] == eb[0] and list(ea[1]) == list(eb[1])
    eager.close()
    graph.close()


def test_graphs_off_and_on_again():
    """Switching replay off and on drops the captured graphs; the solver
    keeps stepping correctly either way."""
    A, B = site_tensors(2, 2, 5)
    cfg = P.Config(d=2, D=2, chi=8, method=P.REDUCED, precision=P.FP64)
    ref = P.Solver(cfg, A, B)
    ref.set_graphs(False)
    s = P.Solver(cfg, A, B)
    for it in range(8):
        if it == 4:
            s.set_graphs(False)
        if it == 5:
            s.set_graphs(True)
        ref.iterate(1)
        s.iterate(1)
    for a, b in zip(_env(ref), _env(s)):
        assert np.array_equal(a, b)
    ref.close()
    s.close()
