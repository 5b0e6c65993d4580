"""Rounds that imply more variables than the LDS structures of a round hold
(the 256-entry winner table, one frontier record per thread or 128): a
choice atom x that, once true, makes n rule bodies and then n heads true in
single rounds, so the winner table overflows into the global winner keys and
pending map and the next frontier has no LDS records.  Whole solves against
the oracle (verdict, every counter, the trace hash, the answer set) under
both Learning steps and several workgroup widths.
"""
import numpy as np
import pytest

import aspgen
import oracle
from brute import is_stable
from parity import assert_same_stats, STATUS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1909_01786_amd as P
    P.lib()
    return P


def _fanout(n, constrained):
    """x :- not y.  y :- not x.  h_i :- x (i = 1..n); with `constrained`
    also :- h_1, h_n, so that x true leads to a conflict."""
    x, y = 1, 2
    rules = [(x, [-y]), (y, [-x])] + [(2 + i, [x]) for i in range(1, n + 1)]
    if constrained:
        rules.append((0, [3, 2 + n]))
    return aspgen.from_rules(n + 2, rules, name=f"fanout{n}{'c' if constrained else ''}")


@pytest.mark.parametrize("n", [300, 700])
@pytest.mark.parametrize("constrained", [False, True])
@pytest.mark.parametrize("learning", [0, 1])
@pytest.mark.parametrize("threads", [64, 128, 256])
def test_round_overflow_parity(P, n, constrained, learning, threads):
    prog = _fanout(n, constrained)
    rc, m, st = oracle.solve(prog, learning=learning)
    g = P.Program(prog, learning=learning)
    g.bind("cuda", threads=threads)
    grc, gm, gst = g.solve(P.limits(-1, 60000))
    assert grc == STATUS[rc], (prog.name, grc, rc)
    assert_same_stats(st, gst, (prog.name, learning, threads))
    if rc == oracle.SAT:
        assert np.array_equal(gm, m) and is_stable(prog, gm)
