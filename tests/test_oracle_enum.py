"""Pins of the oracle's enumeration of several answer sets and of restarts.

Checked against what the answer-set definition and combinatorics fix: the
set of answer sets found equals the brute-force set (each one once), with and
without restarts, under both Learning steps and both gate modes; counts
equal closed forms -- the chromatic polynomial at 3 for 3-colouring (trees
3*2^(n-1), cycles 2^n + 2(-1)^n, wheels 3(1 + (-1)^n), complete graphs 3!
and 0, disjoint unions multiply) and the number of directed Hamiltonian
cycles ((n-1)! on a complete digraph, 2 on a bidirected cycle, 1 on a
directed cycle); every blocking nogood is the true atoms of the answer set
it follows; asking for one answer set is the plain search, bit for bit.
"""
import math

import numpy as np
import pytest

import aspgen
import oracle
from brute import is_stable, model_to_mask, stable_models


def _as_set(models):
    return {int(model_to_mask(m)) for m in models}


def _check_all(prog, **kw):
    rc, ms, st, ex = oracle.enumerate_models(prog, **kw)
    want = stable_models(prog)
    assert len(ms) == len(_as_set(ms)), "an answer set was found twice"
    assert _as_set(ms) == {int(m) for m in want}, prog.name
    assert rc == (oracle.SAT if want else oracle.UNSAT)
    assert ex == bool(want)
    assert st["models"] == len(want)
    for m in ms:
        assert is_stable(prog, m)
    return st


@pytest.mark.parametrize("chunk", range(4))
def test_all_answer_sets_match_brute_force(chunk):
    for seed in range(chunk * 60, chunk * 60 + 60):
        prog = aspgen.tiny_program(50000 + seed, 4, 14)
        for learning in (oracle.LEARN_FWD, oracle.LEARN_RES):
            for restart_every in (0, 2):
                _check_all(prog, learning=learning, restart_every=restart_every,
                           gate=seed % 2)


def test_restarts_counted_and_hashed():
    prog = aspgen.coloring(6, [(i, (i + 1) % 6) for i in range(6)])
    st0 = _check_all(prog)
    st1 = _check_all(prog, restart_every=1)
    assert st0["restarts"] == st0["models"]          # one per blocked answer set
    assert st1["restarts"] > st0["restarts"]
    assert st0["trace_hash"] != st1["trace_hash"]


def test_max_models_stops_early():
    prog = aspgen.coloring(5, [(i, (i + 1) % 5) for i in range(5)])   # 30 colourings
    for k in (2, 7, 29, 30):
        rc, ms, st, ex = oracle.enumerate_models(prog, max_models=k)
        assert rc == oracle.SAT and len(ms) == k == st["models"]
        assert len(_as_set(ms)) == k and not ex
        assert all(is_stable(prog, m) for m in ms)
    rc, ms, st, ex = oracle.enumerate_models(prog, max_models=31)
    assert len(ms) == 30 and ex


def _count(prog, **kw):
    rc, ms, st, ex = oracle.enumerate_models(prog, **kw)
    assert ex or rc == oracle.UNSAT
    assert len(_as_set(ms)) == len(ms)
    return len(ms)


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_coloring_counts_trees(n):
    path = [(i, i + 1) for i in range(n - 1)]
    star = [(0, i) for i in range(1, n)]
    assert _count(aspgen.coloring(n, path)) == 3 * 2 ** (n - 1)
    assert _count(aspgen.coloring(n, star), restart_every=3) == 3 * 2 ** (n - 1)


@pytest.mark.parametrize("n", [3, 4, 5, 7])
def test_coloring_counts_cycles_and_wheels(n):
    cyc = [(i, (i + 1) % n) for i in range(n)]
    assert _count(aspgen.coloring(n, cyc)) == 2 ** n + 2 * (-1) ** n
    wheel = cyc + [(n, i) for i in range(n)]        # hub n joined to every rim vertex
    assert _count(aspgen.coloring(n + 1, wheel), learning=oracle.LEARN_RES) == 3 * (1 + (-1) ** n)


def test_coloring_counts_complete_and_unions():
    k3 = [(0, 1), (0, 2), (1, 2)]
    k4 = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    assert _count(aspgen.coloring(3, k3)) == 6
    assert _count(aspgen.coloring(4, k4)) == 0
    # a triangle and a path on 3 vertices, disjoint: 6 * 12
    union = k3 + [(3, 4), (4, 5)]
    assert _count(aspgen.coloring(6, union), restart_every=2) == 72


@pytest.mark.parametrize("n", [3, 4, 5])
def test_hamiltonian_cycle_counts(n):
    complete = [(u, w) for u in range(n) for w in range(n) if u != w]
    assert _count(aspgen.hamiltonian(n, complete)) == math.factorial(n - 1)
    bidir = [(i, (i + 1) % n) for i in range(n)] + [((i + 1) % n, i) for i in range(n)]
    assert _count(aspgen.hamiltonian(n, bidir), learning=oracle.LEARN_RES) == 2
    directed = [(i, (i + 1) % n) for i in range(n)]
    assert _count(aspgen.hamiltonian(n, directed)) == 1


def test_empty_answer_set_is_the_only_one():
    prog = aspgen.from_rules(3, [])
    rc, ms, st, ex = oracle.enumerate_models(prog)
    assert rc == oracle.SAT and ex and len(ms) == 1 and not ms[0].any()


def test_blocking_nogoods_walk():
    """After each answer set the newest learned nogood is its true atoms,
    and the next step is InitialPropagation from an empty assignment."""
    prog = aspgen.coloring(4, [(0, 1), (1, 2), (2, 3)])
    s = oracle.Solver(prog, max_models=0)
    seen = 0
    for _ in range(20000):
        k = s.next_step()
        if k == oracle.ST_DONE:
            break
        s.step()
        st = s.stats()
        if k == oracle.ST_GATE and st["models"] > seen:
            seen = st["models"]
            after = s.state()
            if after.status != oracle.RUNNING:
                break
            m = s.models()[-1]
            off, lits = after.ng_off, after.ng_lits
            assert list(lits[off[-2]:off[-1]]) == list(np.nonzero(m)[0] + 1)
            assert s.next_step() == oracle.ST_INIT
            assert not after.val.any() and after.cdl == 1
    assert seen == 24 and s.exhausted()


@pytest.mark.parametrize("seed", range(12))
def test_one_answer_set_is_the_plain_search(seed):
    prog = aspgen.tiny_program(7000 + seed, 6, 20)
    r1 = oracle.solve(prog)
    s = oracle.Solver(prog, max_models=1)
    rc = s.run()
    assert rc == r1[0] and s.stats() == r1[2]
    if rc == oracle.SAT:
        assert np.array_equal(s.model(), r1[1])
    # enumeration finds the plain search's answer set first
    rc2, ms, _, _ = oracle.enumerate_models(prog)
    if rc == oracle.SAT:
        assert np.array_equal(ms[0], r1[1])
    else:
        assert rc2 == oracle.UNSAT and not ms
