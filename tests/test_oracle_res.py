"""Pins of the oracle's Res-learning (Alg. 3, resolution to the first UIP).

Checked against what the method and the answer-set definition fix: every
learned nogood is made of literals true at the conflict, has exactly one
literal at its top level (the first UIP), is asserting after the backjump to
the highest level of its other literals, and holds in no answer set (brute
force over the completion extensions of every answer set); verdicts equal
brute force; gate conflicts and conflicts whose resolution reaches a
CompleteAssignment literal learn the Fwd-learning nogood (decision literals).
"""
import numpy as np
import pytest

import aspgen
import oracle
from fullscan import lit_val, lit_var, nogoods_list, completion_extension
from brute import is_stable, stable_models


def _walk_res(prog, max_steps=4000):
    s = oracle.Solver(prog, learning=oracle.LEARN_RES)
    A = prog.n_atoms
    V = int(s.dims()[0])
    exts = [completion_extension(prog, m, V) for m in stable_models(prog)] if A <= 14 else None
    n_res = 0
    for _ in range(max_steps):
        k = s.next_step()
        if k == oracle.ST_DONE:
            break
        before = s.state()
        s.step()
        after = s.state()
        if k != oracle.ST_LEARN or after.status != oracle.RUNNING:
            continue
        learned = nogoods_list(after.ng_off, after.ng_lits)[-1]
        assert all(before.val[lit_var(l)] == lit_val(l) for l in learned)
        lv = [int(before.lvl[lit_var(l)]) for l in learned]
        top = max(lv)
        is_dec = all(l > 0 and l > A and (l - A - 1) % 3 == 0 and before.dec[before.lvl[l]] == l
                     for l in learned)
        if before.pend_kind == 2:
            assert is_dec, "gate conflicts are learned by Fwd-learning"
        else:
            n_res += 1
        # one literal at the top level, last in the nogood
        assert lv.count(top) == 1 and lv[-1] == top
        bj = max([x for x in lv[:-1]] + [1])
        assert after.cdl == bj
        t = learned[-1]
        assert after.val[lit_var(t)] == -lit_val(t) and after.lvl[lit_var(t)] == bj
        assert all(after.val[lit_var(l)] == lit_val(l) for l in learned[:-1])
        if exts is not None:
            for e in exts:
                assert not all(e[lit_var(l)] == lit_val(l) for l in learned)
    return s, n_res


@pytest.mark.parametrize("seed", range(80))
def test_res_learning_invariants_tiny(seed):
    prog = aspgen.tiny_program(30000 + seed, 4, 12)
    s, _ = _walk_res(prog)
    assert s.next_step() == oracle.ST_DONE


@pytest.mark.parametrize("seed", range(3))
def test_res_learning_invariants_medium(seed):
    s, n_res = _walk_res(aspgen.single_random(1000 + seed), max_steps=600)
    assert n_res > 0


@pytest.mark.parametrize("chunk", range(4))
def test_res_learning_verdicts_match_brute_force(chunk):
    for seed in range(chunk * 100, chunk * 100 + 100):
        prog = aspgen.tiny_program(seed, 4, 16)
        rc, m, _ = oracle.solve(prog, learning=oracle.LEARN_RES)
        models = stable_models(prog)
        assert rc == (oracle.SAT if models else oracle.UNSAT), seed
        if rc == oracle.SAT:
            assert is_stable(prog, m)


def test_res_and_fwd_agree_on_verdicts_medium():
    for seed in range(6):
        prog = aspgen.single_random(1100 + seed)
        r0 = oracle.solve(prog, limits=oracle.make_limits(3000))
        r1 = oracle.solve(prog, limits=oracle.make_limits(3000), learning=oracle.LEARN_RES)
        if r0[0] in (oracle.SAT, oracle.UNSAT) and r1[0] in (oracle.SAT, oracle.UNSAT):
            assert r0[0] == r1[0]
        if r1[0] == oracle.SAT:
            assert is_stable(prog, r1[1])


def test_unfounded_counterexample_res():
    """p <- q. q <- p. <- not p. has no answer set under Res-learning too."""
    prog = aspgen.from_rules(2, [(1, [2]), (2, [1]), (0, [-1])])
    assert oracle.solve(prog, learning=oracle.LEARN_RES)[0] == oracle.UNSAT
