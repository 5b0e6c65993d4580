"""The allocation-free solve (asp_solve_noalloc) against asp_solve.

asp_solve_noalloc runs the same search kernel in the library's own device
array instead of a caller-bound arena.  Its verdict, model, every counter
and the trace hash must equal asp_solve's on the same program, bit for bit,
over consecutive calls that reuse the array with inputs of decreasing size
(what an earlier call left behind must not leak into the next).
"""
import os

import numpy as np
import pytest

import aspgen
import oracle
from parity import assert_same_stats, STATUS

pytestmark = pytest.mark.gpu

LIM_MS = int(os.environ.get("ASP_TEST_MAX_MS", "60000"))
CAPS = dict(learned_cap_ng=4096, learned_cap_lits=1 << 18)
KEYS = ("rounds", "visits", "literal_checks", "propagations", "decisions", "conflicts",
        "learned", "learned_len", "gate_failures", "completes", "trace_hash", "models",
        "restarts", "exhausted")


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1909_01786_amd as P
    P.lib()
    return P


def _both(P, prog, budget, **kw):
    """(noalloc result, asp_solve result) on the same program and limits."""
    lim = P.limits(budget, LIM_MS)
    g = P.Program(prog, **CAPS, **kw)
    na = g.solve_noalloc(lim)
    ref = P.Program(prog, **CAPS, **kw).bind("cuda", threads=256).solve(lim)
    return na, ref


def _same(na, ref, name):
    (rc, m, st), (rrc, rm, rst) = na, ref
    assert rc == rrc, (name, rc, rrc)
    for k in KEYS:
        assert st[k] == rst[k], (name, k, st[k], rst[k])
    if rrc == 1:
        assert np.array_equal(m, rm), name


def test_noalloc_matches_solve_on_shrinking_inputs(P):
    """Three calls in a row, each smaller than the one before: the
    2000-vertex colouring (24k variables), the 200-atom program, a tiny
    one; each equals asp_solve and the oracle."""
    progs = [(aspgen.gnp_coloring(2000), 300), (aspgen.single_random(1001), 30000),
             (aspgen.tiny_program(7, 10, 12), -1)]
    sizes = []
    for prog, budget in progs:
        na, ref = _both(P, prog, budget)
        _same(na, ref, prog.name)
        orc, om, ost = oracle.solve(prog, limits=oracle.make_limits(
            max_conflicts=budget, learned_cap_ng=CAPS["learned_cap_ng"],
            learned_cap_lits=CAPS["learned_cap_lits"]))
        assert na[0] == STATUS[orc], prog.name
        assert_same_stats(ost, na[2], prog.name)
        if orc == oracle.SAT:
            assert np.array_equal(na[1], om)
        sizes.append(P.Program(prog, **CAPS).sizes.device_bytes)
    assert sizes[0] > sizes[1] > sizes[2]


def test_noalloc_other_search_modes(P):
    """Res-learning, several answer sets with restarts, Jeroslow-Wang,
    activity and several conflicts per step through the same array,
    alternating large and small programs."""
    modes = [dict(learning=P.LEARN_RES), dict(max_models=4), dict(decision=P.DECISION_JW),
             dict(decision=P.DECISION_ACTIVITY, restart_every=50), dict(learn_conflicts=4)]
    for i, kw in enumerate(modes):
        for prog in (aspgen.batch_random(i), aspgen.tiny_program(100 + i, 8, 14)):
            na, ref = _both(P, prog, 500, **kw)
            _same(na, ref, f"{prog.name} {kw}")


def test_noalloc_rejects_what_it_cannot_hold(P):
    """Beyond ASP_NOALLOC_MAX_BYTES: a capacity error, nothing launched;
    score-driven Decision: invalid (its scores need a bound arena)."""
    from paper_1909_01786_amd.binding import AspError, E_CAPACITY, E_INVALID, NOALLOC_MAX_BYTES
    prog = aspgen.single_random(1001)
    g = P.Program(prog)                       # default learned-store capacities
    assert g.sizes.device_bytes > NOALLOC_MAX_BYTES
    with pytest.raises(AspError) as e:
        g.solve_noalloc(P.limits(100, LIM_MS))
    assert e.value.status == E_CAPACITY
    with pytest.raises(AspError) as e:
        P.Program(prog, decision=P.DECISION_SCORE, **CAPS).solve_noalloc(P.limits(100, LIM_MS))
    assert e.value.status == E_INVALID
    # the array still serves a valid call afterwards
    na, ref = _both(P, aspgen.tiny_program(3, 6, 10), -1)
    _same(na, ref, "after errors")
