"""Parity of the HIP library's enumeration of several answer sets (blocking
nogoods and restarts) with the CPU oracle, through the C ABI: the answer sets
in the order found, counters, restarts, trace hashes and the exhausted flag
of whole solves; the whole state after every single step (restarts and the
InitialPropagation over learned units included); batches; closed-form counts.
"""
import math
import os

import numpy as np
import pytest

import aspgen
import oracle
from brute import is_stable, stable_models
from parity import assert_same_state, assert_same_stats, STATUS

pytestmark = pytest.mark.gpu

LIM_MS = int(os.environ.get("ASP_TEST_MAX_MS", "60000"))
STORE = 256


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1909_01786_amd as P
    P.lib()
    return P


def _check(P, prog, max_models=STORE, restart_every=0, learning=0, gate=0, threads=64,
           max_conflicts=-1):
    rc, ms, st, ex = oracle.enumerate_models(prog, max_models=max_models,
                                             restart_every=restart_every, learning=learning,
                                             gate=gate,
                                             limits=oracle.make_limits(max_conflicts))
    g = P.Program(prog, gate=gate, learning=learning, max_models=max_models,
                  restart_every=restart_every)
    g.bind("cuda", threads=threads)
    grc, gm, gst = g.solve(P.limits(max_conflicts, LIM_MS))
    assert grc == STATUS[rc], (prog.name, grc, rc)
    assert_same_stats(st, gst, prog.name)
    assert bool(gst["exhausted"]) == ex, prog.name
    gms = g.models()
    keep = min(len(ms), max(1, max_models))
    assert len(gms) == keep
    for a, b in zip(gms, ms[:keep]):
        assert np.array_equal(a, b), prog.name
    if rc == oracle.SAT:
        assert np.array_equal(gm, ms[0])
    return rc, ms, st, ex


@pytest.mark.parametrize("learning", [0, 1])
def test_enum_tiny_parity_and_brute_force(P, learning):
    for seed in range(150):
        prog = aspgen.tiny_program(60000 + seed, 4, 14)
        for restart_every in (0, 3):
            rc, ms, st, ex = _check(P, prog, learning=learning, restart_every=restart_every,
                                    gate=seed % 2)
            assert ex == bool(ms) and len(ms) == len(stable_models(prog))
            assert all(is_stable(prog, m) for m in ms)


def test_enum_counts_closed_forms(P):
    cases = []
    for n in (4, 5, 7):
        cyc = [(i, (i + 1) % n) for i in range(n)]
        cases.append((aspgen.coloring(n, cyc), 2 ** n + 2 * (-1) ** n))
        cases.append((aspgen.coloring(n + 1, cyc + [(n, i) for i in range(n)]),
                      3 * (1 + (-1) ** n)))
    cases.append((aspgen.coloring(8, [(i, i + 1) for i in range(7)]), 3 * 2 ** 7))
    cases.append((aspgen.coloring(4, [(a, b) for a in range(4) for b in range(a + 1, 4)]), 0))
    for n in (4, 5):
        full = [(u, w) for u in range(n) for w in range(n) if u != w]
        cases.append((aspgen.hamiltonian(n, full), math.factorial(n - 1)))
    for prog, want in cases:
        for learning in (0, 1):
            g = P.Program(prog, learning=learning, max_models=0)
            g.bind("cuda", threads=128)
            grc, _, gst = g.solve(P.limits(-1, LIM_MS))
            assert gst["models"] == want, (prog.name, gst["models"], want)
            assert grc == (P.SAT if want else P.UNSAT)
            assert gst["exhausted"] == (1 if want else 0)
            rc, _, st, _ = oracle.enumerate_models(prog, max_models=0, learning=learning)
            assert_same_stats(st, gst, prog.name)


def test_enum_max_models_and_restarts(P):
    prog = aspgen.coloring(6, [(i, (i + 1) % 6) for i in range(6)])     # 66 colourings
    for k in (1, 2, 17, 66, 67):
        for r in (0, 1, 5):
            _check(P, prog, max_models=k, restart_every=r, threads=128)


@pytest.mark.parametrize("seed", range(3))
def test_enum_medium_budget(P, seed):
    """Larger programs under a conflict budget: every answer set found up
    to the budget, the same on both sides."""
    prog = aspgen.single_random(1300 + seed)
    for learning in (0, 1):
        _check(P, prog, max_models=40, restart_every=50, learning=learning, threads=256,
               max_conflicts=400)


def _walk(P, prog, threads, n, **kw):
    o = oracle.Solver(prog, **kw)
    g = P.Program(prog, **kw)
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
    assert o.next_step() == oracle.ST_DONE


@pytest.mark.parametrize("seed", range(24))
def test_enum_step_by_step_parity(P, seed):
    prog = aspgen.tiny_program(8000 + seed, 5, 14)
    _walk(P, prog, 64, 20000, max_models=0, restart_every=seed % 3,
          learning=seed % 2)


def test_enum_state_import_refused(P):
    from paper_1909_01786_amd import AspError
    g = P.Program(aspgen.tiny_program(5, 6, 20), max_models=3)
    g.bind("cuda", threads=64)
    g.run_steps(2, P.limits(-1, LIM_MS))
    with pytest.raises(AspError):
        g.import_state(g.export_state())


def test_enum_batch_parity(P):
    progs = [aspgen.tiny_program(s, 4, 16) for s in range(30)]
    progs += [aspgen.coloring(5, [(i, (i + 1) % 5) for i in range(5)])]
    progs += [aspgen.batch_random(s, a_lo=100, a_hi=300) for s in range(4)]
    gp = [P.Program(p, max_models=8, restart_every=7) for p in progs]
    b = P.Batch(gp, threads=128, classes=2).bind("cuda")
    b.solve(P.limits(300, LIM_MS))
    verd, models, stats = b.results(all_models=True)
    for i, p in enumerate(progs):
        rc, ms, st, ex = oracle.enumerate_models(p, max_models=8, restart_every=7,
                                                 limits=oracle.make_limits(300))
        assert verd[i] == STATUS[rc], (i, p.name)
        assert_same_stats(st, stats[i], p.name)
        assert bool(stats[i]["exhausted"]) == ex
        assert len(models[i]) == len(ms)
        for a, c in zip(models[i], ms):
            assert np.array_equal(a, c)
