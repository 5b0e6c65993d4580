"""Parity of the HIP library (through the C ABI) with the CPU oracle.

Integer and Boolean work throughout, so every comparison is bit-exact:
states after each step (values, levels, Deps bitmaps, frontier, decisions,
learned nogoods), counters, trace hashes, verdicts and models.
"""
import os

import numpy as np
import pytest

import aspgen
import oracle
from brute import is_stable, model_to_mask, stable_models
from parity import assert_same_state, assert_same_stats, to_lib_state, STATUS

pytestmark = pytest.mark.gpu

# device wall-clock guard per launch (a guard, never reached by a passing run)
LIM_MS = int(os.environ.get("ASP_TEST_MAX_MS", "60000"))


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1909_01786_amd as P
    P.lib()
    return P


def _gpu_program(P, prog, W=1, gate=0, threads=64, **kw):
    g = P.Program(prog, W=W, gate=gate, **kw)
    g.bind("cuda", threads=threads)
    return g


def _check_solve(P, prog, W=1, gate=0, threads=64, max_conflicts=-1):
    lim_o = oracle.make_limits(max_conflicts=max_conflicts)
    rc, m, st = oracle.solve(prog, W=W, gate=gate, limits=lim_o)
    g = _gpu_program(P, prog, W, gate, threads)
    grc, gm, gst = g.solve(P.limits(max_conflicts, LIM_MS))
    assert grc == STATUS[rc], (prog.name, grc, rc)
    assert_same_stats(st, gst, prog.name)
    if rc == oracle.SAT:
        assert np.array_equal(gm, m), prog.name
        assert is_stable(prog, gm)
    return rc, g


@pytest.mark.parametrize("threads", [64, 256])
def test_solve_tiny_parity_and_brute_force(P, threads):
    """300 random programs of 4..14 atoms: identical verdict, model and
    counters; SAT models are answer sets, UNSAT programs have none."""
    for seed in range(300):
        prog = aspgen.tiny_program(seed, 4, 14)
        rc, _ = _check_solve(P, prog, threads=threads)
        if rc == oracle.UNSAT:
            assert stable_models(prog) == []


def test_solve_edge_cases(P):
    cases = [
        aspgen.from_rules(2, [(1, [2]), (2, [1]), (0, [-1])]),   # unfounded loop
        aspgen.from_rules(2, [(1, [2]), (2, [1])]),               # empty model
        aspgen.from_rules(1, [(1, []), (0, [])]),                 # empty constraint
        aspgen.from_rules(1, [(1, []), (0, [1, -1])]),            # tautology
        aspgen.from_rules(2, [(1, [2, -2]), (2, [])]),            # never fires
        aspgen.from_rules(3, []),                                 # no rules
        aspgen.from_rules(1, [(1, [-1])]),                        # odd loop: UNSAT
        aspgen.coloring(4, [(a, b) for a in range(4) for b in range(a + 1, 4)]),
        aspgen.hamiltonian(5, [(i, (i + 1) % 5) for i in range(5)]),
    ]
    for prog in cases:
        for gate in (0, 1):
            _check_solve(P, prog, gate=gate)


@pytest.mark.parametrize("seed", range(6))
def test_solve_random_200x600(P, seed):
    """The 200-atom / 600-rule single instance."""
    _check_solve(P, aspgen.single_random(1000 + seed), threads=256)


@pytest.mark.parametrize("W", [1, 2])
def test_solve_coloring_budget(P, W):
    """The 2000-vertex 3-colouring (24k variables, ~66k nogoods) under a
    conflict budget: first frontier of 6000 units spans many 256-lane
    chunks; W=1 saturates the Deps bitmaps."""
    _check_solve(P, aspgen.gnp_coloring(2000), W=W, threads=256, max_conflicts=60)


@pytest.mark.parametrize("seed", range(4))
def test_solve_hamiltonian(P, seed):
    _check_solve(P, aspgen.batch_hamiltonian(seed), threads=128, max_conflicts=500)


@pytest.mark.parametrize("seed", range(40))
def test_step_by_step_parity(P, seed):
    """Every single step from the start: the whole state agrees."""
    prog = aspgen.tiny_program(3000 + seed, 6, 20)
    o = oracle.Solver(prog)
    g = _gpu_program(P, prog, threads=64)
    for i in range(3000):
        k = o.next_step()
        if k == oracle.ST_DONE:
            break
        o.step()
        grc, gst = g.run_steps(1, P.limits(-1, LIM_MS))
        os_ = o.state()
        assert grc == STATUS[os_.status], (seed, i, k)
        assert gst["last_step"] == k, (seed, i, gst["last_step"], k)
        if os_.status == oracle.RUNNING:
            # after a verdict the assignment carries no meaning (the oracle
            # stops its sequential unit pass at the first clash)
            assert_same_state(os_, g.export_state(), (seed, i, k))
        assert_same_stats(o.stats(), gst, (seed, i, k))


@pytest.mark.parametrize("seed", range(3))
def test_step_parity_medium(P, seed):
    prog = aspgen.single_random(1000 + seed)
    o = oracle.Solver(prog)
    g = _gpu_program(P, prog, threads=256)
    for i in range(400):
        if o.next_step() == oracle.ST_DONE:
            break
        o.step()
        grc, gst = g.run_steps(1, P.limits(-1, LIM_MS))
        if o.state().status == oracle.RUNNING:
            assert_same_state(o.state(), g.export_state(), (seed, i))
        assert_same_stats(o.stats(), gst, (seed, i))


def _walk_imports(P, prog, W, threads, max_steps, rounds_only=False):
    """Import the oracle's state before a round (or a learning step), run
    that one step on the GPU through asp_propagate / asp_analyze_conflict,
    and compare with the oracle after it."""
    o = oracle.Solver(prog, W=W)
    g = _gpu_program(P, prog, W=W, threads=threads)
    n_round = n_learn = 0
    for i in range(max_steps):
        k = o.next_step()
        if k == oracle.ST_DONE:
            break
        before = o.state()
        st_before = o.stats()
        if k == oracle.ST_ROUND or (k == oracle.ST_LEARN and before.pend_kind == 1 and not rounds_only):
            g.import_state(to_lib_state(before, st_before))
        o.step()
        after = o.state()
        if k == oracle.ST_ROUND:
            grc, res = g.propagate(1)
            exp = P.CONFLICT if after.pend_kind == 1 else (
                P.FIXPOINT if after.frontier.size == 0 else P.RUNNING)
            assert grc == exp, (i, grc, exp)
            assert res["literal_checks"] == o.stats()["literal_checks"] - st_before["literal_checks"]
            assert_same_state(after, g.export_state(), ("round", i))
            n_round += 1
        elif k == oracle.ST_LEARN and before.pend_kind == 1 and not rounds_only:
            grc, learned, bj = g.analyze_conflict(P.limits(-1, LIM_MS))
            if after.status == oracle.RUNNING:
                assert grc == 0
                off, lits = after.ng_off, after.ng_lits
                assert learned.tolist() == lits[off[-2]:off[-1]].tolist()
                assert bj == after.cdl
                assert_same_state(after, g.export_state(), ("learn", i))
            else:
                assert grc == STATUS[after.status]
            n_learn += 1
    return n_round, n_learn


@pytest.mark.parametrize("seed", range(3))
def test_import_round_and_learn_parity(P, seed):
    nr, nl = _walk_imports(P, aspgen.single_random(1000 + seed), 1, 64, 600)
    assert nr > 10


def test_import_round_parity_wide_deps(P):
    """W=32 on the colouring: 2048-bit Deps per variable."""
    nr, nl = _walk_imports(P, aspgen.gnp_coloring(2000), 32, 256, 120)
    assert nr > 5


def test_determinism(P):
    prog = aspgen.single_random(1003)
    g = _gpu_program(P, prog, threads=128)
    a = g.solve(P.limits(-1, LIM_MS))
    b = g.solve(P.limits(-1, LIM_MS))
    untimed = lambda d: {k: v for k, v in d.items() if not k.startswith("ns_")}
    assert a[0] == b[0] and untimed(a[2]) == untimed(b[2])
    assert (a[1] is None and b[1] is None) or np.array_equal(a[1], b[1])


def test_budget_unknown(P):
    prog = aspgen.single_random(1000)
    g = _gpu_program(P, prog, threads=64)
    rc, _, st = g.solve(P.limits(5, LIM_MS))
    assert rc == P.UNKNOWN and st["conflicts"] == 5
    g2 = _gpu_program(P, prog, threads=64, learned_cap_ng=3)
    rc, _, st = g2.solve(P.limits(-1, LIM_MS))
    orc, _, ost = oracle.solve(prog, limits=oracle.make_limits(learned_cap_ng=3))
    assert rc == P.UNKNOWN == STATUS[orc] and st["learned"] == ost["learned"] == 3


def test_api_errors(P):
    from paper_1909_01786_amd.binding import AspError
    prog = aspgen.single_random(1001)
    g = P.Program(prog)
    with pytest.raises(AspError):
        g.propagate(1)                   # not bound
    g.bind("cuda", threads=64)
    with pytest.raises(AspError):
        g.analyze_conflict()             # nothing pending
    st = g.export_state()
    st.frontier = np.array([5], np.int32)   # unassigned variable in the frontier
    with pytest.raises(AspError):
        g.import_state(st)


@pytest.mark.parametrize("threads", [64, 256])
def test_batch_parity_mixed(P, threads):
    """One batched solve over programs of very different sizes (several LDS
    classes, one workgroup each)."""
    progs = [aspgen.tiny_program(s, 4, 20) for s in range(40)]
    progs += [aspgen.single_random(1000 + s) for s in range(4)]
    progs += [aspgen.batch_hamiltonian(s) for s in range(4)]
    progs += [aspgen.batch_random(s, a_lo=100, a_hi=400) for s in range(8)]
    gp = [P.Program(p) for p in progs]
    b = P.Batch(gp, threads=threads, classes=3).bind("cuda")
    b.solve(P.limits(300, LIM_MS))
    verd, models, stats = b.results()
    for i, p in enumerate(progs):
        rc, m, st = oracle.solve(p, limits=oracle.make_limits(300))
        assert verd[i] == STATUS[rc], (i, p.name)
        assert_same_stats(st, stats[i], p.name)
        if rc == oracle.SAT:
            assert np.array_equal(models[i], m)
    # a second launch on the same arena gives the same results
    b.solve(P.limits(300, LIM_MS))
    verd2, models2, stats2 = b.results()
    untimed = lambda L: [{k: v for k, v in d.items() if not k.startswith("ns_")} for d in L]
    assert np.array_equal(verd, verd2) and untimed(stats) == untimed(stats2)


def test_batch_graph_replays(P):
    """The batched solve as a HIP graph: every replay, with eager device work
    and synchronisations between replays, gives the eager launch's verdicts,
    models and counters; changing the limits re-captures."""
    import torch
    progs = [aspgen.tiny_program(s, 4, 20) for s in range(20)]
    progs += [aspgen.single_random(1500 + s) for s in range(3)]
    progs += [aspgen.batch_random(s, a_lo=100, a_hi=400) for s in range(4)]
    gp = [P.Program(p) for p in progs]
    stream = torch.cuda.Stream()
    b = P.Batch(gp, threads=128, classes=3)
    with torch.cuda.stream(stream):
        b.bind("cuda", stream=stream)
    untimed = lambda L: [{k: v for k, v in d.items() if not k.startswith("ns_")} for d in L]
    for budget in (200, 60):
        lim = P.limits(budget, LIM_MS)
        b.solve(lim)
        torch.cuda.synchronize()
        v0, m0, s0 = b.results()
        for r in range(3):
            x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
            assert float((x * 2).sum()) > 0
            torch.cuda.synchronize()
            b.solve(lim, graph=True)
            torch.cuda.synchronize()
            v, m, st = b.results()
            assert np.array_equal(v, v0), (budget, r)
            assert all(np.array_equal(a, c) for a, c in zip(m, m0)), (budget, r)
            assert untimed(st) == untimed(s0), (budget, r)
        for i in (0, 21, 25):
            rc, _, sto = oracle.solve(progs[i], limits=oracle.make_limits(budget))
            assert v0[i] == STATUS[rc]
            assert_same_stats(sto, s0[i], i)
