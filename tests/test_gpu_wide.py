"""Parity with the CPU oracle at two Deps words (W = 2) for the paths added
beside the plain search: Res-learning, several answer sets with restarts,
the activity and Jeroslow-Wang Decision scores, and several conflicts per
step -- whole solves on tiny programs and a deep search whose levels pass
64 (the first word saturates into the second).
"""
import os

import numpy as np
import pytest

import aspgen
import oracle
from brute import is_stable
from parity import assert_same_stats, STATUS

pytestmark = pytest.mark.gpu

LIM_MS = int(os.environ.get("ASP_TEST_MAX_MS", "60000"))

CASES = [
    dict(learning=1),
    dict(max_models=32, restart_every=4),
    dict(decision=3),
    dict(decision=2, learning=1),
    dict(learn_conflicts=3),
    dict(learn_conflicts=2, learning=1, max_models=8),
]


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1909_01786_amd as P
    P.lib()
    return P


def _check(P, prog, kw, threads=64, max_conflicts=-1):
    o = oracle.Solver(prog, W=2, **kw)
    rc = o.run(oracle.make_limits(max_conflicts))
    st = o.stats()
    g = P.Program(prog, W=2, **kw)
    g.bind("cuda", threads=threads)
    grc, gm, gst = g.solve(P.limits(max_conflicts, LIM_MS))
    assert grc == STATUS[rc], (prog.name, kw, grc, rc)
    assert_same_stats(st, gst, (prog.name, kw))
    ms = o.models()
    gms = g.models()
    keep = min(len(ms), max(1, kw.get("max_models", 1)))
    assert len(gms) == keep
    for a, b in zip(gms, ms):
        assert np.array_equal(a, b)
        assert is_stable(prog, a)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_wide_tiny(P, case):
    for seed in range(60):
        _check(P, aspgen.tiny_program(96000 + seed, 4, 14), CASES[case])


@pytest.mark.parametrize("case", range(len(CASES)))
def test_wide_deep(P, case):
    """The 2000-vertex colouring under a budget: levels pass 64."""
    _check(P, aspgen.gnp_coloring(2000), CASES[case], threads=256, max_conflicts=40)
