"""Pins of the oracle's learning of several conflicts per Learning step.

Checked against what the method and the answer-set definition fix: every
nogood learned in a step is made of literals true at the conflict and
holds in no answer set (brute force over the completion extensions of
every answer set); the step learns as many nogoods as the round had
distinct conflicts, up to K; the backjump goes to the lowest of their
backjump levels, where exactly one literal is asserted and the nogood it
comes from is unit-violated otherwise; verdicts and answer-set counts equal
brute force; K = 1 is the plain search, bit for bit.
"""
import numpy as np
import pytest

import aspgen
import oracle
from brute import is_stable, stable_models
from fullscan import completion_extension, full_scan, lit_val, lit_var, nogoods_list


def _walk(prog, K, learning, max_steps=4000):
    s = oracle.Solver(prog, learning=learning, learn_conflicts=K)
    A = prog.n_atoms
    V = int(s.dims()[0])
    exts = [completion_extension(prog, m, V) for m in stable_models(prog)] if A <= 14 else None
    multi = 0
    for _ in range(max_steps):
        k = s.next_step()
        if k == oracle.ST_DONE:
            break
        before = s.state()
        n_before = len(nogoods_list(before.ng_off, before.ng_lits))
        s.step()
        after = s.state()
        if k != oracle.ST_LEARN or after.status != oracle.RUNNING:
            continue
        ngs = nogoods_list(after.ng_off, after.ng_lits)
        new = ngs[n_before:]
        if before.pend_kind == 1:
            # distinct violated nogoods of the round, up to K of them
            violated = full_scan(nogoods_list(before.ng_off, before.ng_lits), before.val)[0]
            assert 1 <= len(new) <= min(K, len(violated))
            if len(new) > 1:
                multi += 1
        else:
            assert len(new) == 1
        for ng in new:
            assert all(before.val[lit_var(l)] == lit_val(l) for l in ng)
            if exts is not None:
                for e in exts:
                    assert not all(e[lit_var(l)] == lit_val(l) for l in ng)
        # exactly one new assignment, at the lowest backjump level
        assert after.cdl <= before.cdl
        assert len(after.frontier) == 1
        x = int(after.frontier[0])
        assert after.lvl[x] == after.cdl
        units = [ng for ng in new if lit_var(ng[-1]) == x and
                 all(after.val[lit_var(l)] == lit_val(l) for l in ng[:-1]) and
                 after.val[x] == -lit_val(ng[-1])]
        assert units, "the asserted literal comes from a learned nogood"
        for ng in new:
            # no learned nogood is violated after the assertion
            assert not all(after.val[lit_var(l)] == lit_val(l) for l in ng)
    return s, multi


@pytest.mark.parametrize("seed", range(60))
def test_multi_learning_invariants_tiny(seed):
    prog = aspgen.tiny_program(97000 + seed, 5, 14)
    s, _ = _walk(prog, 4, seed % 2)
    assert s.next_step() == oracle.ST_DONE


@pytest.mark.parametrize("learning", [0, 1])
def test_multi_learning_happens(learning):
    total = 0
    for seed in range(3):
        _, m = _walk(aspgen.batch_random(7 + seed, a_lo=100, a_hi=200), 8, learning,
                     max_steps=3000)
        total += m
    assert total > 0, "some steps learn several nogoods"


@pytest.mark.parametrize("K", [2, 8])
def test_multi_learning_verdicts_match_brute_force(K):
    for seed in range(200):
        prog = aspgen.tiny_program(98000 + seed, 4, 16)
        rc, m, _ = oracle.solve(prog, learn_conflicts=K, learning=seed % 2, gate=(seed // 2) % 2)
        want = stable_models(prog)
        assert rc == (oracle.SAT if want else oracle.UNSAT), seed
        if rc == oracle.SAT:
            assert is_stable(prog, m)
        _, ms, _, _ = oracle.enumerate_models(prog, learn_conflicts=K, restart_every=3)
        assert len(ms) == len(want)


@pytest.mark.parametrize("seed", range(12))
def test_one_conflict_is_the_plain_search(seed):
    prog = aspgen.single_random(1600 + seed)
    a = oracle.solve(prog, limits=oracle.make_limits(2000))
    b = oracle.solve(prog, limits=oracle.make_limits(2000), learn_conflicts=1)
    assert a[0] == b[0] and a[2] == b[2]
