"""Parity of the HIP library's Jeroslow-Wang and activity Decision scores
with the CPU oracle, through the C ABI: whole solves (verdicts, models,
counters, trace hashes), every single step, batches, and the combinations
with Res-learning and with several answer sets and restarts.
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
DECISIONS = [oracle.DEC_JW, oracle.DEC_ACTIVITY]


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1909_01786_amd as P
    P.lib()
    assert (P.DECISION_JW, P.DECISION_ACTIVITY) == (oracle.DEC_JW, oracle.DEC_ACTIVITY)
    return P


def _check(P, prog, decision, threads=64, max_conflicts=-1, learning=0, gate=0):
    rc, m, st = oracle.solve(prog, gate=gate, decision=decision, learning=learning,
                             limits=oracle.make_limits(max_conflicts))
    g = P.Program(prog, gate=gate, decision=decision, learning=learning)
    g.bind("cuda", threads=threads)
    grc, gm, gst = g.solve(P.limits(max_conflicts, LIM_MS))
    assert grc == STATUS[rc], (prog.name, grc, rc)
    assert_same_stats(st, gst, prog.name)
    if rc == oracle.SAT:
        assert np.array_equal(gm, m), prog.name
        assert is_stable(prog, gm)
    return rc


@pytest.mark.parametrize("decision", DECISIONS)
@pytest.mark.parametrize("threads", [64, 256])
def test_heur_tiny_parity_and_brute_force(P, decision, threads):
    for seed in range(200):
        prog = aspgen.tiny_program(93000 + seed, 4, 14)
        rc = _check(P, prog, decision, threads=threads, learning=seed % 2, gate=(seed // 2) % 2)
        assert (rc == oracle.SAT) == bool(stable_models(prog))


@pytest.mark.parametrize("decision", DECISIONS)
@pytest.mark.parametrize("seed", range(4))
def test_heur_medium(P, decision, seed):
    _check(P, aspgen.single_random(1000 + seed), decision, threads=256)
    _check(P, aspgen.batch_random(seed, a_lo=100, a_hi=300), decision, threads=128,
           max_conflicts=400, learning=seed % 2)


@pytest.mark.parametrize("decision", DECISIONS)
def test_heur_hamiltonian_and_coloring(P, decision):
    for seed in range(2):
        _check(P, aspgen.batch_hamiltonian(seed), decision, threads=128, max_conflicts=300)
    _check(P, aspgen.gnp_coloring(2000), decision, threads=256, max_conflicts=60)


@pytest.mark.parametrize("decision", DECISIONS)
@pytest.mark.parametrize("seed", range(16))
def test_heur_step_by_step_parity(P, decision, seed):
    prog = aspgen.tiny_program(94000 + seed, 6, 20)
    o = oracle.Solver(prog, decision=decision, learning=seed % 2)
    g = P.Program(prog, decision=decision, learning=seed % 2)
    g.bind("cuda", threads=64)
    for i in range(3000):
        k = o.next_step()
        if k == oracle.ST_DONE:
            break
        o.step()
        grc, gst = g.run_steps(1, P.limits(-1, LIM_MS))
        os_ = o.state()
        assert grc == STATUS[os_.status], (seed, i, k)
        assert gst["last_step"] == k
        if os_.status == oracle.RUNNING:
            assert_same_state(os_, g.export_state(), (seed, i, k))
        assert_same_stats(o.stats(), gst, (seed, i, k))


def test_heur_with_enumeration(P):
    for seed in range(40):
        prog = aspgen.tiny_program(95000 + seed, 4, 14)
        for decision in DECISIONS:
            rc, ms, st, ex = oracle.enumerate_models(prog, max_models=64, restart_every=3,
                                                     decision=decision)
            g = P.Program(prog, decision=decision, max_models=64, restart_every=3)
            g.bind("cuda", threads=64)
            grc, _, gst = g.solve(P.limits(-1, LIM_MS))
            assert grc == STATUS[rc]
            assert_same_stats(st, gst, prog.name)
            gms = g.models()
            assert len(gms) == len(ms) and all(np.array_equal(a, b) for a, b in zip(gms, ms))


@pytest.mark.parametrize("decision", DECISIONS)
def test_heur_batch_parity(P, decision):
    progs = [aspgen.tiny_program(s, 4, 20) for s in range(30)]
    progs += [aspgen.single_random(1500 + s) for s in range(3)]
    progs += [aspgen.batch_random(s, a_lo=100, a_hi=400) for s in range(6)]
    gp = [P.Program(p, decision=decision) for p in progs]
    b = P.Batch(gp, threads=128, classes=3).bind("cuda")
    b.solve(P.limits(300, LIM_MS))
    verd, models, stats = b.results()
    for i, p in enumerate(progs):
        rc, m, st = oracle.solve(p, decision=decision, limits=oracle.make_limits(300))
        assert verd[i] == STATUS[rc], (i, p.name)
        assert_same_stats(st, stats[i], p.name)
        if rc == oracle.SAT:
            assert np.array_equal(models[i], m)
