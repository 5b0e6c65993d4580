"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
nogood counts of the completion (Sect. 2), brute-force answer sets (the
definition in the Preliminaries), completion models, textbook special cases
(Horn programs, tight programs), chromatic-polynomial and Hamiltonian-cycle
counts, and step-level invariants re-derived by full scans.
"""
import math

import numpy as np
import pytest

import aspgen
import oracle
from fullscan import (completion_extension, decision_choice, expected_round,
                      full_scan, levels_of, lit_val, lit_var, nogoods_list,
                      occurrences, satisfies)
from brute import (completion_models, is_stable, mask_to_model, model_to_mask,
                   stable_models)


def norm_rules(prog):
    """Rules after removing repeated body literals; constraints holding both
    a and not a dropped."""
    out = []
    for h, body in prog.rules():
        seen = []
        for l in body:
            if l not in seen:
                seen.append(l)
        pos = [l for l in seen if l > 0]
        neg = [-l for l in seen if l < 0]
        if h == 0 and set(pos) & set(neg):
            continue
        out.append((h, pos, neg))
    return out


# ------------------------------------------------------------- encoding
@pytest.mark.parametrize("seed", range(40))
def test_encoding_closed_form_counts(seed):
    """|Delta| = sum_r (5+|body r|) + sum_p (|rules p|+1) + #constraints and
    literals = sum_r (9+3|body r|) + sum_p (3|rules p|+1) + sum_c |body c|."""
    prog = aspgen.tiny_program(seed, 4, 20)
    rules = norm_rules(prog)
    A = prog.n_atoms
    nrules = {p: 0 for p in range(1, A + 1)}
    n_ng = n_lit = 0
    for h, pos, neg in rules:
        k = len(pos) + len(neg)
        if h:
            n_ng += 5 + k
            n_lit += 9 + 3 * k
            nrules[h] += 1
        else:
            n_ng += 1
            n_lit += k
    for p in range(1, A + 1):
        n_ng += nrules[p] + 1
        n_lit += 3 * nrules[p] + 1
    s = oracle.Solver(prog)
    off, lits = s.nogoods()
    assert len(off) - 1 == n_ng
    assert len(lits) == n_lit
    lens = np.diff(off)
    assert np.all(np.diff(lens) >= 0), "nogoods must be sorted by length"


def test_encoding_coloring_exact_counts():
    """3-colouring of a graph with E edges and 2000 vertices: 6000 unit,
    36000+3E binary and 12000 ternary nogoods."""
    prog = aspgen.gnp_coloring(2000)
    E = (prog.n_rules - 6000) // 3
    s = oracle.Solver(prog)
    off, _ = s.nogoods()
    lens = np.diff(off)
    assert (lens == 1).sum() == 6000
    assert (lens == 2).sum() == 36000 + 3 * E
    assert (lens == 3).sum() == 12000
    assert len(lens) == 54000 + 3 * E


def test_encoding_first_rule_literal_order():
    """A single rule p <- q, not r: the generation order of Sect. 2 followed by
    the stable length sort fixes every id."""
    prog = aspgen.from_rules(3, [(1, [2, -3])])
    s = oracle.Solver(prog)
    off, lits = s.nogoods()
    ngs = nogoods_list(off, lits)
    b, t, n = 4, 5, 6
    # generation order: {Fb,Tt,Tn},{Tb,Ft},{Tb,Fn},{Tt,Fq},{Tn,Tr},{Ft,Tq},{Fn,Fr},
    # atom 1: {F1,Tb},{T1,Fb}; atom 2: {T2}; atom 3: {T3}
    gen = [[-b, t, n], [b, -t], [b, -n], [t, -2], [n, 3], [-t, 2], [-n, -3],
           [-1, b], [1, -b], [2], [3]]
    expect = sorted(gen, key=len)  # Python's sort is stable
    assert ngs == expect


@pytest.mark.parametrize("seed", range(60))
def test_nogood_solutions_are_completion_models(seed):
    """M is a model of the completion (and the constraints) iff its
    auxiliary extension satisfies Delta; other values of any rule's
    auxiliary atoms violate Delta."""
    prog = aspgen.tiny_program(seed, 3, 9)
    s = oracle.Solver(prog)
    off, lits = s.nogoods()
    ngs = nogoods_list(off, lits)
    V = int(s.dims()[0])
    cm = set(completion_models(prog))
    A = prog.n_atoms
    Rh = int(s.dims()[2])
    for mask in range(1 << A):
        val = completion_extension(prog, mask, V)
        assert satisfies(ngs, val) == (mask in cm), (seed, mask)
        if mask in cm:
            for j in range(Rh):
                base = A + 3 * j + 1
                for combo in range(8):
                    alt = val.copy()
                    for k in range(3):
                        alt[base + k] = 1 if (combo >> k) & 1 else -1
                    if np.array_equal(alt, val):
                        continue
                    assert not satisfies(ngs, alt)


def test_invalid_programs_rejected():
    with pytest.raises(ValueError):
        oracle.Solver(aspgen.from_rules(2, [(3, [1])]))
    with pytest.raises(ValueError):
        oracle.Solver(aspgen.from_rules(2, [(1, [0])]))
    with pytest.raises(ValueError):
        oracle.Solver(aspgen.from_rules(2, [(1, [-5])]))


# ------------------------------------------------------------ verdicts
def _check_verdict(prog, W=1, gate=oracle.GATE_UNFOUNDED):
    rc, m, st = oracle.solve(prog, W=W, gate=gate)
    sm = stable_models(prog)
    if rc == oracle.SAT:
        assert is_stable(prog, m)
        assert model_to_mask(m) in sm
    else:
        assert rc == oracle.UNSAT, rc
        assert sm == []
    return rc, st


@pytest.mark.parametrize("chunk", range(8))
def test_verdicts_match_brute_force(chunk):
    """2400 random programs of 4..14 atoms, with and without constraints."""
    for seed in range(chunk * 300, chunk * 300 + 300):
        _check_verdict(aspgen.tiny_program(seed, 4, 14))


@pytest.mark.parametrize("seed", range(12))
def test_verdicts_match_brute_force_20_atoms(seed):
    _check_verdict(aspgen.tiny_program(100000 + seed, 18, 20))


@pytest.mark.parametrize("seed", range(200))
def test_gate_alldec_same_verdicts(seed):
    prog = aspgen.tiny_program(5000 + seed, 4, 12)
    _check_verdict(prog, gate=oracle.GATE_ALLDEC)


def test_unfounded_counterexample_is_unsat():
    """p <- q.  q <- p.  <- not p.  Propagation alone makes {p, q} total with
    no decision; the least model of the reduct is empty, so there is no
    answer set."""
    prog = aspgen.from_rules(2, [(1, [2]), (2, [1]), (0, [-1])])
    for gate in (oracle.GATE_UNFOUNDED, oracle.GATE_ALLDEC):
        rc, m, st = oracle.solve(prog, gate=gate)
        assert rc == oracle.UNSAT
        assert st["gate_failures"] == 1 and st["decisions"] == 0
    assert stable_models(prog) == []


def test_positive_loop_without_constraint_is_empty_model():
    """p <- q. q <- p.: the only answer set is the empty set."""
    prog = aspgen.from_rules(2, [(1, [2]), (2, [1])])
    rc, m, st = oracle.solve(prog)
    assert rc == oracle.SAT and m.tolist() == [0, 0]


def test_empty_constraint_and_tautology():
    assert oracle.solve(aspgen.from_rules(1, [(1, []), (0, [])]))[0] == oracle.UNSAT
    # <- a, not a can never fire and is dropped
    rc, m, _ = oracle.solve(aspgen.from_rules(1, [(1, []), (0, [1, -1])]))
    assert rc == oracle.SAT and m.tolist() == [1]
    # a <- b, not b never fires
    rc, m, _ = oracle.solve(aspgen.from_rules(2, [(1, [2, -2]), (2, [])]))
    assert rc == oracle.SAT and m.tolist() == [0, 1]


def test_empty_program():
    rc, m, st = oracle.solve(aspgen.from_rules(0, []))
    assert rc == oracle.SAT and len(m) == 0
    rc, m, st = oracle.solve(aspgen.from_rules(3, []))
    assert rc == oracle.SAT and m.tolist() == [0, 0, 0]


def _least_model(prog):
    A = prog.n_atoms
    LM = set()
    changed = True
    while changed:
        changed = False
        for h, body in prog.rules():
            if h and h not in LM and all(b in LM for b in body):
                LM.add(h)
                changed = True
    return np.array([1 if p in LM else 0 for p in range(1, A + 1)], np.uint8)


@pytest.mark.parametrize("seed", range(100))
def test_horn_programs_least_model(seed):
    """A Horn program has exactly one answer set, the least fixpoint of T_Pi."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = int(rng.integers(3, 40))
    prog = aspgen.random_program(rng, A, int(A * rng.uniform(0.5, 3)), 0, 3, p_neg=0.0)
    rc, m, st = oracle.solve(prog)
    assert rc == oracle.SAT
    assert np.array_equal(m, _least_model(prog))


def _tight_program(seed):
    """Positive body atoms are always smaller than the head: the positive
    dependency graph is acyclic."""
    rng = np.random.Generator(np.random.PCG64(90000 + seed))
    A = int(rng.integers(4, 14))
    rules = []
    for _ in range(int(A * rng.uniform(1, 3))):
        h = int(rng.integers(1, A + 1))
        body = []
        for _ in range(int(rng.integers(0, 4))):
            q = int(rng.integers(1, A + 1))
            if rng.random() < 0.5 and q < h:
                body.append(q)
            else:
                body.append(-q)
        rules.append((h, body))
    for _ in range(int(rng.integers(0, 3))):
        rules.append((0, [int(rng.integers(1, A + 1)) * (1 if rng.random() < .5 else -1)]))
    return aspgen.from_rules(A, rules)


@pytest.mark.parametrize("seed", range(200))
def test_tight_programs_never_fail_the_gate(seed):
    """Tight programs: answer sets are the supported models (Fages), so a
    total conflict-free assignment is always stable."""
    prog = _tight_program(seed)
    rc, st = _check_verdict(prog)
    assert st["gate_failures"] == 0
    assert (rc == oracle.SAT) == bool(completion_models(prog))


# ------------------------------------------------------------- families
def _path(n):
    return [(i, i + 1) for i in range(n - 1)]


def _cycle(n):
    return [(i, (i + 1) % n) for i in range(n)]


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_coloring_counts_chromatic_polynomial(n):
    """#answer sets = P(G, 3): a path (tree) on n vertices has 3*2^(n-1), a
    cycle C_n has 2^n + 2(-1)^n; the oracle finds a proper colouring."""
    for edges, count in ((_path(n), 3 * 2 ** (n - 1)),
                         (_cycle(n) if n >= 3 else _path(n),
                          2 ** n + 2 * (-1) ** n if n >= 3 else 3 * 2 ** (n - 1))):
        prog = aspgen.coloring(n, edges)
        assert len(stable_models(prog)) == count
        rc, m, st = oracle.solve(prog)
        assert rc == oracle.SAT and st["gate_failures"] == 0
        col = m.reshape(n, 3)
        assert np.all(col.sum(1) == 1)
        c = col.argmax(1)
        assert all(c[u] != c[w] for u, w in edges)


def test_coloring_k4_unsat():
    edges = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    prog = aspgen.coloring(4, edges)
    assert stable_models(prog) == []
    assert oracle.solve(prog)[0] == oracle.UNSAT


@pytest.mark.parametrize("n", [3, 4, 5])
def test_hamiltonian_directed_cycle_unique(n):
    """The directed n-cycle has exactly one Hamiltonian cycle."""
    edges = _cycle(n)
    prog = aspgen.hamiltonian(n, edges)
    sm = stable_models(prog)
    assert len(sm) == 1
    rc, m, st = oracle.solve(prog)
    assert rc == oracle.SAT and model_to_mask(m) == sm[0]
    E = len(edges)
    assert m[:E].tolist() == [1] * E


def test_hamiltonian_complete_digraph_counts():
    """K_3 as a digraph has (3-1)! = 2 Hamiltonian cycles."""
    edges = [(u, w) for u in range(3) for w in range(3) if u != w]
    prog = aspgen.hamiltonian(3, edges)
    assert len(stable_models(prog)) == math.factorial(2)
    rc, m, _ = oracle.solve(prog)
    assert rc == oracle.SAT and is_stable(prog, m)


def test_hamiltonian_source_vertex_unsat():
    """A vertex with no incoming edge cannot lie on a cycle."""
    edges = [(0, 1), (1, 2), (2, 0), (0, 3), (3, 1)]  # vertex 3 has in-edge (0,3)
    edges2 = [(0, 1), (1, 2), (2, 0), (3, 1)]          # vertex 3 has none
    assert oracle.solve(aspgen.hamiltonian(4, edges))[0] == oracle.SAT
    prog = aspgen.hamiltonian(4, edges2)
    assert oracle.solve(prog)[0] == oracle.UNSAT
    assert stable_models(prog) == []


# --------------------------------------------------------- step invariants
def _stable_extensions(prog, V):
    return [completion_extension(prog, m, V) for m in stable_models(prog)]


def _walk(prog, W=1, max_steps=4000):
    """Step the oracle and check every step against re-derivations."""
    s = oracle.Solver(prog, W=W)
    A = prog.n_atoms
    V = int(s.dims()[0])
    exts = _stable_extensions(prog, V) if A <= 14 else None
    occ_expect = None
    checks = 0
    for _ in range(max_steps):
        k = s.next_step()
        if k == oracle.ST_DONE:
            break
        before = s.state()
        ngs = nogoods_list(before.ng_off, before.ng_lits)
        if occ_expect is None:
            occ_expect = occurrences(ngs[:before.n_static], A)
            assert np.array_equal(s.occ()[1:], occ_expect[1:])
        if k in (oracle.ST_DECIDE, oracle.ST_COMPLETE, oracle.ST_GATE):
            # a fixpoint: nothing is unit and nothing is violated
            viol, unit = full_scan(ngs, before.val)
            assert viol == [] and unit == {}
        if k == oracle.ST_DECIDE or k == oracle.ST_COMPLETE:
            j = decision_choice(prog, before.val, occ_expect)
            assert (j >= 0) == (k == oracle.ST_DECIDE)
        s.step()
        after = s.state()
        st = s.stats()
        if k == oracle.ST_ROUND:
            newval, newdeps, sel = expected_round(ngs, before.val, before.deps, before.cdl)
            assert sorted(newval) == after.frontier.tolist()
            for x, v in newval.items():
                assert after.val[x] == v and after.lvl[x] == before.cdl
                assert np.array_equal(after.deps[x], newdeps[x])
            if sel >= 0:
                assert after.pend_kind == 1 and after.pend_id == sel
            else:
                assert after.pend_kind == 0
            # literal checks: sum of lengths of the nogoods containing each
            # frontier literal
            visits = 0
            for v in before.frontier:
                L = int(v) if before.val[v] > 0 else -int(v)
                visits += sum(len(ng) for ng in ngs if L in ng)
            checks += visits
            assert st["literal_checks"] == checks
        elif k == oracle.ST_DECIDE:
            j = decision_choice(prog, before.val, occ_expect)
            b = A + 3 * j + 1
            assert after.cdl == before.cdl + 1 and after.dec[after.cdl] == b
            assert after.val[b] == 1 and after.frontier.tolist() == [b]
        elif k == oracle.ST_LEARN and after.status == oracle.RUNNING:
            learned = nogoods_list(after.ng_off, after.ng_lits)[-1]
            # only decision literals, by increasing level, unit after backjump
            lv = [int(before.lvl[lit_var(l)]) for l in learned]
            assert lv == sorted(lv) and len(set(lv)) == len(lv)
            assert all(before.dec[l] == lit for l, lit in zip(lv, learned))
            bj = lv[-2] if len(lv) >= 2 else 1
            assert after.cdl == bj
            top = learned[-1]
            assert after.val[lit_var(top)] == -lit_val(top)
            assert all(after.val[lit_var(l)] == lit_val(l) for l in learned[:-1])
        if exts is not None and k != oracle.ST_GATE:
            # soundness of Deps: every answer set holding the decisions of
            # levels(Deps[x]) agrees with x; no answer set holds a learned nogood
            for x in range(1, V + 1):
                if after.val[x] == 0:
                    continue
                lv = levels_of(after.deps[x], after.cdl, W)
                dl = [after.dec[l] for l in lv]
                for e in exts:
                    if all(e[lit_var(d)] == lit_val(d) for d in dl):
                        assert e[x] == after.val[x], (k, x)
            for ng in nogoods_list(after.ng_off, after.ng_lits)[after.n_static:]:
                for e in exts:
                    assert not all(e[lit_var(l)] == lit_val(l) for l in ng)
    return s


@pytest.mark.parametrize("seed", range(120))
def test_step_invariants_tiny(seed):
    prog = aspgen.tiny_program(20000 + seed, 4, 12)
    s = _walk(prog)
    assert s.next_step() == oracle.ST_DONE


@pytest.mark.parametrize("seed", range(4))
def test_step_invariants_medium(seed):
    """Full-scan re-derivation of every round on a 200-atom random program
    (stopped after a bounded number of steps)."""
    _walk(aspgen.single_random(1000 + seed), max_steps=300)


def test_budget_unknown_and_counters():
    """max_conflicts stops the search with UNKNOWN, after exactly that many
    learned nogoods."""
    prog = aspgen.single_random(1000)
    rc, _, st = oracle.solve(prog, limits=oracle.make_limits(max_conflicts=5))
    assert rc == oracle.UNKNOWN and st["conflicts"] == 5 and st["learned"] == 5
    rc, _, st = oracle.solve(prog, limits=oracle.make_limits(learned_cap_ng=3))
    assert rc == oracle.UNKNOWN and st["learned"] == 3


def test_deterministic_trace():
    prog = aspgen.single_random(1003)
    a = oracle.solve(prog)
    b = oracle.solve(prog)
    assert a[0] == b[0] and a[2] == b[2]


def test_saturated_bitmap_deep_search():
    """W=1 on the 2000-vertex colouring: the first conflict comes at a level
    above 63, where levels >= 64 share the last Deps bit; the learned nogood
    must then hold the decision of every level from 64 to cdl, and the
    backjump goes to the second-highest level, cdl-1."""
    prog = aspgen.gnp_coloring(2000)
    s = oracle.Solver(prog, W=1)
    while True:
        k = s.next_step()
        assert k != oracle.ST_DONE
        if k == oracle.ST_LEARN and s.dims()[6] >= 70:
            break
        s.step()
    before = s.state()
    cdl = before.cdl
    s.step()
    after = s.state()
    learned = nogoods_list(after.ng_off, after.ng_lits)[-1]
    tail = [int(before.dec[l]) for l in range(64, cdl + 1)]
    assert learned[-len(tail):] == tail
    assert after.cdl == cdl - 1
    top = learned[-1]
    assert after.val[lit_var(top)] == -lit_val(top)
