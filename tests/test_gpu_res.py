"""Parity of the HIP library's Res-learning (Alg. 3, first UIP) with the
CPU oracle, through the C ABI: verdicts, models, counters and trace hashes
of whole solves, and the whole state (learned nogoods literal by literal,
in assignment order with the UIP last) after every single step.
"""
import os

import numpy as np
import pytest

import aspgen
import oracle
from brute import is_stable, stable_models
from parity import assert_same_state, assert_same_stats, STATUS

pytestmark = pytest.mark.gpu

LIM_MS = int(os.environ.get("ASP_TEST_MAX_MS", "60000"))
RES = oracle.LEARN_RES


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1909_01786_amd as P
    P.lib()
    assert P.LEARN_RES == oracle.LEARN_RES and P.LEARN_FWD == oracle.LEARN_FWD
    return P


def _check(P, prog, W=1, gate=0, threads=64, max_conflicts=-1):
    rc, m, st = oracle.solve(prog, W=W, gate=gate, limits=oracle.make_limits(max_conflicts),
                             learning=RES)
    g = P.Program(prog, W=W, gate=gate, learning=P.LEARN_RES)
    g.bind("cuda", threads=threads)
    grc, gm, gst = g.solve(P.limits(max_conflicts, LIM_MS))
    assert grc == STATUS[rc], (prog.name, grc, rc)
    assert_same_stats(st, gst, prog.name)
    if rc == oracle.SAT:
        assert np.array_equal(gm, m), prog.name
        assert is_stable(prog, gm)
    return rc, st


@pytest.mark.parametrize("threads", [64, 256])
def test_res_solve_tiny_parity_and_brute_force(P, threads):
    for seed in range(300):
        prog = aspgen.tiny_program(seed, 4, 14)
        rc, _ = _check(P, prog, threads=threads)
        if rc == oracle.UNSAT:
            assert stable_models(prog) == []


def test_res_edge_cases(P):
    cases = [
        aspgen.from_rules(2, [(1, [2]), (2, [1]), (0, [-1])]),
        aspgen.from_rules(2, [(1, [2]), (2, [1])]),
        aspgen.from_rules(1, [(1, []), (0, [])]),
        aspgen.from_rules(1, [(1, []), (0, [1, -1])]),
        aspgen.from_rules(3, []),
        aspgen.from_rules(1, [(1, [-1])]),
        aspgen.coloring(4, [(a, b) for a in range(4) for b in range(a + 1, 4)]),
        aspgen.hamiltonian(5, [(i, (i + 1) % 5) for i in range(5)]),
    ]
    for prog in cases:
        for gate in (0, 1):
            _check(P, prog, gate=gate)


@pytest.mark.parametrize("seed", range(6))
def test_res_solve_random_200x600(P, seed):
    _, st = _check(P, aspgen.single_random(1000 + seed), threads=256)


@pytest.mark.parametrize("seed", range(3))
def test_res_solve_hamiltonian(P, seed):
    _check(P, aspgen.batch_hamiltonian(seed), threads=128, max_conflicts=500)


def test_res_solve_coloring_budget(P):
    """24k variables: resolution chains over many 256-lane chunks."""
    _check(P, aspgen.gnp_coloring(2000), threads=256, max_conflicts=60)


def _walk(P, prog, threads, n):
    o = oracle.Solver(prog, learning=RES)
    g = P.Program(prog, learning=P.LEARN_RES)
    g.bind("cuda", threads=threads)
    for i in range(n):
        k = o.next_step()
        if k == oracle.ST_DONE:
            break
        o.step()
        grc, gst = g.run_steps(1, P.limits(-1, LIM_MS))
        os_ = o.state()
        assert grc == STATUS[os_.status], (prog.name, i, k)
        assert gst["last_step"] == k, (prog.name, i, gst["last_step"], k)
        if os_.status == oracle.RUNNING:
            assert_same_state(os_, g.export_state(), (prog.name, i, k))
        assert_same_stats(o.stats(), gst, (prog.name, i, k))


@pytest.mark.parametrize("seed", range(40))
def test_res_step_by_step_parity(P, seed):
    _walk(P, aspgen.tiny_program(3000 + seed, 6, 20), 64, 3000)


@pytest.mark.parametrize("seed", range(3))
def test_res_step_parity_medium(P, seed):
    _walk(P, aspgen.single_random(1000 + seed), 256, 400)


def test_res_state_import_refused(P):
    from paper_1909_01786_amd import AspError
    prog = aspgen.tiny_program(5, 6, 20)
    g = P.Program(prog, learning=P.LEARN_RES)
    g.bind("cuda", threads=64)
    g.run_steps(2, P.limits(-1, LIM_MS))
    st = g.export_state()
    with pytest.raises(AspError):
        g.import_state(st)


def test_res_batch_parity_and_mixed_learning_refused(P):
    """A batched Res-learning solve over several LDS classes; a batch whose
    programs disagree on the Learning step is refused."""
    from paper_1909_01786_amd import AspError
    progs = [aspgen.tiny_program(s, 4, 20) for s in range(30)]
    progs += [aspgen.single_random(1200 + s) for s in range(3)]
    progs += [aspgen.batch_hamiltonian(s) for s in range(3)]
    progs += [aspgen.batch_random(s, a_lo=100, a_hi=400) for s in range(6)]
    gp = [P.Program(p, learning=P.LEARN_RES) for p in progs]
    b = P.Batch(gp, threads=128, classes=3).bind("cuda")
    b.solve(P.limits(300, LIM_MS))
    verd, models, stats = b.results()
    for i, p in enumerate(progs):
        rc, m, st = oracle.solve(p, limits=oracle.make_limits(300), learning=RES)
        assert verd[i] == STATUS[rc], (i, p.name)
        assert_same_stats(st, stats[i], p.name)
        if rc == oracle.SAT:
            assert np.array_equal(models[i], m)
    mixed = [P.Program(progs[0], learning=P.LEARN_RES), P.Program(progs[1])]
    with pytest.raises(AspError):
        P.Batch(mixed, threads=128)
