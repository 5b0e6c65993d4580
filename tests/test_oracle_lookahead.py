"""Pins of the oracle's lookahead Decision.

Each lookahead Decision step is re-derived from the state before it with
the full-scan rounds of tests/fullscan.py (every nogood classified against
the assignment, not the oracle's frontier-driven visits): the K best
applicable rules by (occurrence count of the head, -r), each trial decision
propagated to a fixpoint or a conflict, the first trial that ends in a
conflict or a total assignment standing, otherwise the candidate whose trial
assigned the most variables decided.  The state after the step (level,
decision literal, every value, the pending conflict) and the rounds and
propagations it added must be the re-derived ones.  Verdicts and answer-set
counts equal brute force; K <= 1 is the plain search, bit for bit.
"""
import numpy as np
import pytest

import aspgen
import oracle
from brute import is_stable, stable_models
from fullscan import expected_round, lit_var, nogoods_list, occurrences


def _candidates(prog, val, occ, K):
    A = prog.n_atoms
    keys = []
    j = 0
    for h, _ in prog.rules():
        if h == 0:
            continue
        t, n = A + 3 * j + 2, A + 3 * j + 3
        if val[h] == 0 and val[t] == 1 and val[n] != -1:
            keys.append(((int(occ[h]), -j), j))
        j += 1
    keys.sort(reverse=True)
    return [j for _, j in keys[:K]]


def _trial(ngs, val, deps, cdl, b, W):
    """Decide T b at level cdl+1 and run full-scan rounds to a fixpoint or a
    conflict: (values, conflict id or -1, rounds, variables assigned)."""
    val = val.copy()
    deps = deps.copy()
    lvl = cdl + 1
    val[b] = 1
    bit = min(lvl - 1, 64 * W - 1)
    deps[b] = 0
    deps[b, bit // 64] = np.uint64(1) << np.uint64(bit % 64)
    assigned, rounds = 1, 0
    while True:
        newval, newdeps, sel = expected_round(ngs, val, deps, lvl)
        rounds += 1
        for x, v in newval.items():
            val[x] = v
            deps[x] = newdeps[x]
        assigned += len(newval)
        if sel >= 0:
            return val, sel, rounds, assigned
        if not newval:
            return val, -1, rounds, assigned


def _walk(prog, K, max_steps=3000):
    s = oracle.Solver(prog, lookahead=K)
    occ = occurrences(nogoods_list(*s.nogoods())[:int(s.dims()[3])], prog.n_atoms)
    V = int(s.dims()[0])
    checked = 0
    for _ in range(max_steps):
        k = s.next_step()
        if k == oracle.ST_DONE:
            break
        before = s.state()
        st0 = s.stats()
        s.step()
        if k != oracle.ST_DECIDE:
            continue
        after = s.state()
        st1 = s.stats()
        ngs = nogoods_list(before.ng_off, before.ng_lits)
        cands = _candidates(prog, before.val, occ, K)
        A = prog.n_atoms
        n_assigned0 = int((before.val != 0).sum()) - int(before.val[0] != 0)
        rounds = props = 0
        stood = None
        counts = []
        if len(cands) > 1:
            for j in cands:
                b = A + 3 * j + 1
                val, conf, r, a = _trial(ngs, before.val, before.deps, before.cdl, b, before.W)
                rounds += r
                props += a - 1
                if conf >= 0 or n_assigned0 + a == V:
                    stood = (j, val, conf)
                    break
                counts.append((a, j))
        if stood is not None:
            j, val, conf = stood
            assert np.array_equal(after.val, val), "the standing trial's assignment"
            assert after.pend_kind == (1 if conf >= 0 else 0)
            if conf >= 0:
                assert after.pend_id == conf
        else:
            if len(cands) > 1:
                best = max(counts, key=lambda t: (t[0], -cands.index(t[1])))[1]
            else:
                best = cands[0]
            j = best
            want = before.val.copy()
            want[A + 3 * j + 1] = 1
            assert np.array_equal(after.val, want), "undone trials leave only the decision"
            assert list(after.frontier) == [A + 3 * j + 1]
        assert after.cdl == before.cdl + 1 and after.dec[after.cdl] == A + 3 * j + 1
        assert st1["decisions"] == st0["decisions"] + 1
        assert st1["rounds"] - st0["rounds"] == rounds
        assert st1["propagations"] - st0["propagations"] == props
        checked += 1
    return checked


@pytest.mark.parametrize("K", [2, 4])
def test_lookahead_steps_rederived_by_full_scan(K):
    checked = 0
    for seed in range(40):
        checked += _walk(aspgen.tiny_program(8000 + seed, 12, 20), K)
    for i in range(12):
        checked += _walk(aspgen.batch_random(i, batch_seed=77, a_lo=30, a_hi=60), K)
    assert checked > 100, checked


@pytest.mark.parametrize("K", [2, 4, 8])
def test_lookahead_verdicts_equal_brute_force(K):
    for seed in range(150):
        prog = aspgen.tiny_program(9000 + seed, 4, 14)
        rc, m, _ = oracle.solve(prog, lookahead=K)
        sms = stable_models(prog)
        if rc == oracle.SAT:
            assert is_stable(prog, m), seed
        else:
            assert rc == oracle.UNSAT and sms == [], seed


def test_lookahead_enumerates_every_answer_set():
    for seed in range(80):
        prog = aspgen.tiny_program(9500 + seed, 4, 12)
        rc, models, _, ex = oracle.enumerate_models(prog, max_models=0, lookahead=4)
        want = sorted(tuple(np.nonzero(np.array([(m >> i) & 1 for i in range(prog.n_atoms)]))[0])
                      for m in stable_models(prog))
        got = sorted(tuple(np.nonzero(x)[0]) for x in models)
        assert got == want, seed


@pytest.mark.parametrize("K", [0, 1])
def test_lookahead_off_is_the_plain_search(K):
    for seed in range(30):
        prog = aspgen.single_random(1000 + seed) if seed % 3 == 0 else aspgen.tiny_program(seed, 6, 20)
        a = oracle.solve(prog)
        b = oracle.solve(prog, lookahead=K)
        assert a[0] == b[0] and a[2] == b[2]


def test_lookahead_needs_fwd_learning():
    with pytest.raises(ValueError):
        oracle.Solver(aspgen.tiny_program(1), lookahead=4, learning=oracle.LEARN_RES)
