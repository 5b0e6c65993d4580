"""Parity of the HIP library's lookahead Decision with the CPU oracle,
through the C ABI: whole solves (verdicts, models, counters, trace hashes),
every single step (whole states), batches, and the combinations with the
other Decision scores, several conflicts per step and several answer sets.
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


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1909_01786_amd as P
    P.lib()
    return P


def _check(P, prog, K, threads=64, max_conflicts=-1, gate=0, decision=0, learn_conflicts=1):
    rc, m, st = oracle.solve(prog, gate=gate, decision=decision, lookahead=K,
                             learn_conflicts=learn_conflicts,
                             limits=oracle.make_limits(max_conflicts))
    g = P.Program(prog, gate=gate, decision=decision, lookahead=K,
                  learn_conflicts=learn_conflicts)
    g.bind("cuda", threads=threads)
    grc, gm, gst = g.solve(P.limits(max_conflicts, LIM_MS))
    assert grc == STATUS[rc], (prog.name, grc, rc)
    assert_same_stats(st, gst, prog.name)
    if rc == oracle.SAT:
        assert np.array_equal(gm, m), prog.name
        assert is_stable(prog, gm)
    return rc


@pytest.mark.parametrize("K", [2, 4, 8])
@pytest.mark.parametrize("threads", [64, 256])
def test_lookahead_tiny_parity_and_brute_force(P, K, threads):
    for seed in range(120):
        prog = aspgen.tiny_program(97000 + seed, 4, 14)
        rc = _check(P, prog, K, threads=threads, gate=seed % 2, decision=(0, 2, 3)[seed % 3])
        assert (rc == oracle.SAT) == bool(stable_models(prog))


@pytest.mark.parametrize("seed", range(4))
def test_lookahead_medium(P, seed):
    _check(P, aspgen.single_random(1000 + seed), 4, threads=256)
    _check(P, aspgen.batch_random(seed, a_lo=100, a_hi=300), 4, threads=128, max_conflicts=400)
    _check(P, aspgen.batch_random(seed, a_lo=100, a_hi=300), 3, threads=128, max_conflicts=200,
           learn_conflicts=2)


def test_lookahead_hamiltonian_and_coloring(P):
    for seed in range(2):
        _check(P, aspgen.batch_hamiltonian(seed), 4, threads=128, max_conflicts=300)
    _check(P, aspgen.gnp_coloring(2000), 2, threads=256, max_conflicts=40)


@pytest.mark.parametrize("seed", range(16))
def test_lookahead_step_by_step_parity(P, seed):
    prog = aspgen.tiny_program(97500 + seed, 10, 20)
    kw = dict(lookahead=2 + seed % 3, decision=(3 if seed % 4 == 3 else 0))
    o = oracle.Solver(prog, **kw)
    g = P.Program(prog, **kw)
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


def test_lookahead_with_enumeration_and_scores(P):
    for seed in range(25):
        prog = aspgen.tiny_program(97800 + seed, 4, 14)
        for decision in (0, 2, 3):
            rc, ms, st, ex = oracle.enumerate_models(prog, max_models=64, restart_every=5,
                                                     decision=decision, lookahead=3)
            g = P.Program(prog, decision=decision, max_models=64, restart_every=5, lookahead=3)
            g.bind("cuda", threads=64)
            grc, _, gst = g.solve(P.limits(-1, LIM_MS))
            assert grc == STATUS[rc]
            assert_same_stats(st, gst, prog.name)
            gms = g.models()
            assert len(gms) == len(ms) and all(np.array_equal(a, b) for a, b in zip(gms, ms))


def test_lookahead_learned_scores(P):
    """Scores from the oracle's scorer drive the candidates (with the
    fallback to occurrences)."""
    from oracle import mpnn
    for seed in range(3):
        prog = aspgen.single_random(1300 + seed)
        sc = mpnn.scores(aspgen.mpnn_weights(seed), prog)
        rc, m, st = oracle.solve(prog, scores=sc, fallback_after=10, lookahead=4,
                                 limits=oracle.make_limits(500))
        g = P.Program(prog, decision=P.DECISION_SCORE, fallback_after=10, lookahead=4)
        g.bind("cuda", threads=256)
        g.set_scores(sc)
        grc, gm, gst = g.solve(P.limits(500, LIM_MS))
        assert grc == STATUS[rc]
        assert_same_stats(st, gst, prog.name)


def test_lookahead_batch_parity(P):
    progs = [aspgen.tiny_program(s, 4, 20) for s in range(30)]
    progs += [aspgen.single_random(1700 + s) for s in range(3)]
    progs += [aspgen.batch_random(s, a_lo=100, a_hi=400) for s in range(6)]
    gp = [P.Program(p, lookahead=4) for p in progs]
    b = P.Batch(gp, threads=128, classes=3).bind("cuda")
    b.solve(P.limits(300, LIM_MS))
    verd, models, stats = b.results()
    for i, p in enumerate(progs):
        rc, m, st = oracle.solve(p, lookahead=4, limits=oracle.make_limits(300))
        assert verd[i] == STATUS[rc], (i, p.name)
        assert_same_stats(st, stats[i], p.name)
        if rc == oracle.SAT:
            assert np.array_equal(models[i], m)


def test_lookahead_options_checked(P):
    prog = aspgen.tiny_program(3)
    with pytest.raises(P.AspError):
        P.Program(prog, lookahead=9)
    with pytest.raises(P.AspError):
        P.Program(prog, lookahead=4, learning=P.LEARN_RES)
    assert P.Program(prog, lookahead=1).opt.lookahead == 1
