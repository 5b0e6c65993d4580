"""Pins of the oracle's Res-learning (Alg. 3, resolution to the first UIP).

Checked against what the method and the answer-set definition fix: every
learned nogood is made of literals true at the conflict, has exactly one
literal at its top level (the first UIP), is asserting after the backjump to
the highest level of its other literals, and holds in no answer set (brute
force over the completion extensions of every answer set); verdicts equal
brute force; gate conflicts and conflicts whose resolution reaches a
CompleteAssignment literal learn the Fwd-learning nogood (decision literals).

The stop of the resolution is pinned separately: the test keeps its own
record of why every literal was assigned (the lowest-id nogood that was unit
on it in the round that assigned it, found by scanning every nogood; the
learned nogood for an asserted literal; none for decisions and
CompleteAssignment literals), builds the implication graph of the
conflict's top level, and checks that the learned nogood's top-level
literal is the immediate dominator of the conflict: the unique implication
point nearest the conflict through which every path from the level's
unexplained literals (its decision, its CompleteAssignment literals) passes.
When only the level's entry dominates, resolution must reach an unexplained
literal and the conflict is learned by Fwd-learning.
"""
from collections import deque

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


# ------------------------------------------------------------ first UIP
def _units(off, lits, val):
    """Every nogood that is unit under `val` (no literal false, exactly one
    open, all others true): {id: open literal}."""
    off = np.asarray(off, np.int64)
    lits = np.asarray(lits, np.int64)
    n = len(off) - 1
    out = {}
    if len(lits) == 0:
        return out
    v = val[np.abs(lits)].astype(np.int64) * np.sign(lits)      # +1 true, -1 false, 0 open
    owner = np.repeat(np.arange(n), np.diff(off))
    false_ = np.bincount(owner, weights=(v < 0), minlength=n)
    open_ = np.bincount(owner, weights=(v == 0), minlength=n)
    for c in np.nonzero((false_ == 0) & (open_ == 1))[0]:
        seg = lits[off[c]:off[c + 1]]
        out[int(c)] = int(seg[v[off[c]:off[c + 1]] == 0][0])
    return out


def _reach(src, succ, removed=None):
    seen, dq = {src}, deque([src])
    while dq:
        a = dq.popleft()
        for b in succ.get(a, ()):
            if b != removed and b not in seen:
                seen.add(b)
                dq.append(b)
    return seen


def _first_uip(before, ngs, reason, conf):
    """Immediate dominator of the conflict in the implication graph of its
    top level T, or None when only the virtual entry dominates it."""
    T = max(int(before.lvl[lit_var(l)]) for l in ngs[conf])
    nodes = [v for v in range(1, before.V + 1) if before.val[v] != 0 and before.lvl[v] == T]
    R, K = "entry", "conflict"
    succ = {}
    for v in nodes:
        r = reason.get(v)
        preds = [] if r is None else sorted({lit_var(l) for l in ngs[r]
                                             if lit_var(l) != v and before.lvl[lit_var(l)] == T})
        if r is not None:
            assert preds, "an explained literal of level T has a level-T antecedent"
        for p in (preds or [R]):
            succ.setdefault(p, []).append(v)
    for l in ngs[conf]:
        if before.lvl[lit_var(l)] == T:
            succ.setdefault(lit_var(l), []).append(K)
    assert K in _reach(R, succ)
    doms = [v for v in nodes if K not in _reach(R, succ, removed=v)]
    if not doms:
        return T, None
    # dominators form a chain; the nearest reaches no other dominator
    near = [d for d in doms if not any(e != d and e in _reach(d, succ) for e in doms)]
    assert len(near) == 1
    return T, near[0]


def _walk_uip(prog, max_steps):
    s = oracle.Solver(prog, learning=oracle.LEARN_RES)
    A = prog.n_atoms
    reason = {}
    checked = fell_back = 0
    for _ in range(max_steps):
        k = s.next_step()
        if k == oracle.ST_DONE:
            break
        before = s.state()
        s.step()
        after = s.state()
        if after.status != oracle.RUNNING:
            break
        ngs = nogoods_list(before.ng_off, before.ng_lits)
        if k == oracle.ST_ROUND:
            un = _units(before.ng_off, before.ng_lits, before.val.astype(np.int64))
            new = [x for x in range(1, before.V + 1) if before.val[x] == 0 and after.val[x] != 0]
            by_var = {}
            for c in sorted(un):
                by_var.setdefault(lit_var(un[c]), c)
            for x in new:
                reason[x] = by_var[x]
                assert after.val[x] == -lit_val(un[by_var[x]])
        elif k in (oracle.ST_DECIDE, oracle.ST_COMPLETE, oracle.ST_INIT):
            for x in range(1, before.V + 1):
                if before.val[x] == 0 and after.val[x] != 0:
                    reason[x] = None
        elif k == oracle.ST_LEARN:
            learned = nogoods_list(after.ng_off, after.ng_lits)[-1]
            if before.pend_kind == 1:
                T, uip = _first_uip(before, ngs, reason, int(before.pend_id))
            # the asserted literal's reason is the nogood just learned
            reason[int(after.frontier[0])] = len(after.ng_off) - 2
            if before.pend_kind != 1 or T <= 1:
                continue
            top = [lit_var(l) for l in learned if before.lvl[lit_var(l)] == T]
            if uip is None:
                fell_back += 1
                assert all(l > A and (l - A - 1) % 3 == 0 for l in learned)
            else:
                checked += 1
                assert top == [uip], (top, uip)
                assert lit_var(learned[-1]) == uip
    return checked, fell_back


@pytest.mark.parametrize("seed", range(60))
def test_res_learning_stops_at_first_uip_tiny(seed):
    _walk_uip(aspgen.tiny_program(31000 + seed, 10, 20), 4000)


@pytest.mark.parametrize("seed", range(4))
def test_res_learning_stops_at_first_uip_medium(seed):
    checked, _ = _walk_uip(aspgen.single_random(1000 + seed), 800)
    assert checked >= 3


@pytest.mark.parametrize("seed", range(4))
def test_res_learning_stops_at_first_uip_batch_family(seed):
    checked, _ = _walk_uip(aspgen.batch_random(seed, a_lo=100, a_hi=200), 1500)
    assert checked >= 5
