"""Pins of the oracle's Jeroslow-Wang and activity Decision scores.

Jeroslow-Wang and occurrence counts are checked against closed forms read
off the completion's structure (Sect. 2): the head of m rules occurs in m
nogoods {F p, T b_r} and in one nogood of length 1+m; a positive (negative)
body atom of a rule with k+ positive (k- negative) body literals occurs in
one binary nogood and in one of length 1+k+ (1+k-); an atom of a constraint
with k body literals occurs in its nogood of length k.  Activity is checked
along a walk over every step: it starts at the occurrence counts, each
learned nogood adds 8 per literal to the literal's atom (the head of rule r
for the auxiliary variables of r), every 64th learned nogood halves all, and
each decision is the argmax of the head's activity (ties to the lowest
rule).  Verdicts under both scores equal brute force.
"""
import numpy as np
import pytest

import aspgen
import oracle
from fullscan import nogoods_list
from brute import is_stable, stable_models
from test_oracle import norm_rules


def _closed_form(prog):
    A = prog.n_atoms
    occ = np.zeros(A + 1, np.int64)
    jw = np.zeros(A + 1, np.int64)

    def add(p, length):
        occ[p] += 1
        if length <= 16:
            jw[p] += 1 << (16 - length)

    m = np.zeros(A + 1, np.int64)
    for h, pos, neg in norm_rules(prog):
        if h == 0:
            for p in pos + neg:
                add(p, len(pos) + len(neg))
            continue
        m[h] += 1
        add(h, 2)                          # {F h, T b_r}
        for q in pos:
            add(q, 2)                      # {T t_r, F q}
            add(q, 1 + len(pos))           # {F t_r, T q ...}
        for q in neg:
            add(q, 2)                      # {T n_r, T q}
            add(q, 1 + len(neg))           # {F n_r, F q ...}
    for p in range(1, A + 1):
        add(p, 1 + int(m[p]))              # {T p, F b_r ...}
    return occ, jw


@pytest.mark.parametrize("seed", range(60))
def test_occurrence_and_jw_closed_forms(seed):
    prog = aspgen.tiny_program(90000 + seed, 4, 20)
    occ, jw = _closed_form(prog)
    s = oracle.Solver(prog)
    assert np.array_equal(s.atom_scores(0)[1:], occ[1:])
    assert np.array_equal(s.atom_scores(1)[1:], jw[1:])


def test_jw_long_nogoods_contribute_nothing():
    # a constraint of 17 literals and one of 16
    prog = aspgen.from_rules(17, [(0, list(range(1, 18))), (0, list(range(1, 17)))])
    jw = oracle.Solver(prog).atom_scores(1)
    # atom p has no rules: its nogood {T p} gives 2^15; the 16-literal
    # constraint gives 2^0 to atoms 1..16; the 17-literal one nothing
    assert list(jw[1:17]) == [(1 << 15) + 1] * 16 and jw[17] == 1 << 15


def _walk_activity(prog, learning, max_steps=5000):
    s = oracle.Solver(prog, decision=oracle.DEC_ACTIVITY, learning=learning)
    A = prog.n_atoms
    head = [h for h, _, _ in norm_rules(prog) if h != 0]
    act = s.atom_scores(0).astype(np.int64)
    assert np.array_equal(s.atom_scores(2), act)
    n_learned = 0
    for _ in range(max_steps):
        k = s.next_step()
        if k == oracle.ST_DONE:
            break
        before = s.state()
        if k == oracle.ST_DECIDE:
            # the argmax of the head's activity over the applicable rules
            cand = [j for j, p in enumerate(head)
                    if before.val[p] == 0 and before.val[A + 3 * j + 2] == 1
                    and before.val[A + 3 * j + 3] != -1]
            want = min(cand, key=lambda j: (-act[head[j]], j))
        s.step()
        after = s.state()
        if k == oracle.ST_DECIDE:
            assert after.dec[after.cdl] == A + 3 * want + 1
        if k == oracle.ST_LEARN and s.stats()["learned"] > n_learned:
            n_learned = s.stats()["learned"]
            learned = nogoods_list(after.ng_off, after.ng_lits)[-1]
            for l in learned:
                v = abs(l)
                act[v if v <= A else head[(v - A - 1) // 3]] += 8
            if n_learned % 64 == 0:
                act >>= 1
        assert np.array_equal(s.atom_scores(2), act), (k, n_learned)
    return s, n_learned


@pytest.mark.parametrize("seed", range(30))
def test_activity_walk_tiny(seed):
    prog = aspgen.tiny_program(91000 + seed, 6, 20)
    s, _ = _walk_activity(prog, seed % 2)
    assert s.next_step() == oracle.ST_DONE


@pytest.mark.parametrize("learning", [0, 1])
def test_activity_walk_halves(learning):
    """A program with hundreds of conflicts: activities halve several times."""
    _, n = _walk_activity(aspgen.batch_random(7, a_lo=100, a_hi=200), learning,
                          max_steps=12000)
    assert n >= (192 if learning == 0 else 64)


@pytest.mark.parametrize("decision", [oracle.DEC_JW, oracle.DEC_ACTIVITY])
def test_verdicts_match_brute_force(decision):
    for seed in range(200):
        prog = aspgen.tiny_program(92000 + seed, 4, 16)
        rc, m, _ = oracle.solve(prog, decision=decision, learning=seed % 2)
        want = stable_models(prog)
        assert rc == (oracle.SAT if want else oracle.UNSAT), seed
        if rc == oracle.SAT:
            assert is_stable(prog, m)
        # enumeration under the same score finds every answer set
        _, ms, _, _ = oracle.enumerate_models(prog, decision=decision)
        assert len(ms) == len(want)
