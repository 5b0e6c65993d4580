"""Parity of the score-driven Decision and of the learned scorer with the
CPU oracle (through the C ABI).

Both are integer work, so every comparison is bit-exact: the scorer's atom
codes, and the whole search driven by them (states per step, counters,
trace hashes, verdicts, models).  Scores fed to the search come from the
seeded generator or from the oracle's scorer, never from the library.
"""
import os

import numpy as np
import pytest

import aspgen
import oracle
from oracle import mpnn
from brute import is_stable
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


def _scored(P, prog, scores, fallback_after=10, threads=64):
    g = P.Program(prog, decision=P.DECISION_SCORE, fallback_after=fallback_after)
    g.bind("cuda", threads=threads)
    g.set_scores(scores)
    return g


@pytest.mark.parametrize("seed", range(24))
def test_scored_solve_parity(P, seed):
    """Seeded scores (many ties) and several fallback thresholds."""
    prog = aspgen.tiny_program(5000 + seed, 6, 20) if seed < 16 else aspgen.single_random(1200 + seed)
    sc = aspgen.decision_scores(seed, prog.n_atoms, -4, 4)
    fb = [-1, 1, 3, 10][seed % 4]
    rc, m, st = oracle.solve(prog, limits=oracle.make_limits(400), scores=sc, fallback_after=fb)
    g = _scored(P, prog, sc, fb, threads=64 if seed % 2 else 256)
    grc, gm, gst = g.solve(P.limits(400, LIM_MS))
    assert grc == STATUS[rc], (seed, grc, rc)
    assert_same_stats(st, gst, seed)
    if rc == oracle.SAT:
        assert np.array_equal(gm, m) and is_stable(prog, gm)


@pytest.mark.parametrize("seed", range(12))
def test_scored_step_parity(P, seed):
    """Every step agrees, including the fallback state (mode, conflict run)."""
    prog = aspgen.tiny_program(6000 + seed, 8, 20)
    sc = aspgen.decision_scores(100 + seed, prog.n_atoms, -3, 3)
    fb = 1 + seed % 3
    o = oracle.Solver(prog)
    o.set_scores(sc, fb)
    g = _scored(P, prog, sc, fb)
    for i in range(3000):
        k = o.next_step()
        if k == oracle.ST_DONE:
            break
        o.step()
        grc, gst = g.run_steps(1, P.limits(-1, LIM_MS))
        os_ = o.state()
        assert grc == STATUS[os_.status], (seed, i, k)
        if os_.status == oracle.RUNNING:
            gs = g.export_state()
            assert_same_state(os_, gs, (seed, i, k))
            mode, consec = o.score_mode()
            assert gs.score_mode == mode, (seed, i)
            if mode:
                assert gs.consec == consec, (seed, i)
        assert_same_stats(o.stats(), gst, (seed, i, k))


def test_scores_required_and_checked(P):
    prog = aspgen.single_random(1001)
    g = P.Program(prog, decision=P.DECISION_SCORE)
    g.bind("cuda")
    with pytest.raises(P.AspError):
        g.solve(P.limits(10, LIM_MS))
    with pytest.raises(ValueError):
        g.set_scores(np.zeros(prog.n_atoms, np.int32))
    sc = aspgen.decision_scores(1, prog.n_atoms)
    g.set_scores(sc)
    back = g.get_scores()
    assert back[0] == 0 and np.array_equal(back[1:], sc[1:])
    w = aspgen.mpnn_weights(1)
    w["P"] = w["P"].astype(np.float64) + 0.5          # not integer codes
    with pytest.raises(P.AspError):
        g.score(w)


SCORER_PROGS = {
    "random200": lambda: aspgen.single_random(1001),
    "hc": lambda: aspgen.batch_hamiltonian(5),
    "batch": lambda: aspgen.batch_random(11, a_lo=100, a_hi=600),
    "tiny": lambda: aspgen.tiny_program(7, 4, 6),
    "empty_constraint": lambda: aspgen.from_rules(3, [(1, [-2]), (2, [-1]), (0, []), (3, [1, 2, -3])]),
    "unused_atoms": lambda: aspgen.from_rules(6, [(1, [2]), (2, [1])]),
}


@pytest.mark.parametrize("name", sorted(SCORER_PROGS))
@pytest.mark.parametrize("wseed", [0, 1])
def test_scorer_single_exact(P, name, wseed):
    """The device scorer's atom codes equal the oracle's, bit for bit."""
    prog = SCORER_PROGS[name]()
    w = aspgen.mpnn_weights(wseed)
    want = mpnn.scores(w, prog)
    g = P.Program(prog, decision=P.DECISION_SCORE)
    g.bind("cuda")
    got = g.score(w)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (name, bad[:10], got[bad[:10]], want[bad[:10]])


def test_scorer_saturating_weights(P):
    """Largest codes everywhere: activations saturate, sums reach their
    bounds, still exact."""
    prog = aspgen.batch_random(3, a_lo=200, a_hi=400)
    w = aspgen.mpnn_weights(9)
    for k in ("Ev", "Ec", "P", "N", "S", "Q", "R", "T"):
        w[k] = np.full_like(w[k], 127)
    w["wo"] = np.full_like(w["wo"], -127)
    want = mpnn.scores(w, prog)
    g = P.Program(prog)
    g.bind("cuda")
    assert np.array_equal(g.score(w), want)


def _hub(n):
    """Atom 1 in the bodies of n rules: its variable has about n edges of
    one sign, so the scorer's edge sums (up to 255 per edge) need more than
    two base-256 limbs once n exceeds 257."""
    rules = [(i, [1]) for i in range(2, n + 2)] + [(1, [-2])]
    return aspgen.from_rules(n + 1, rules, name=f"hub{n}")


@pytest.mark.parametrize("n", [40, 300, 2000])
@pytest.mark.parametrize("saturate", [False, True])
def test_scorer_wide_edge_sums_exact(P, n, saturate):
    """A variable of high degree (one, two and three limbs of the edge
    sums; saturating weights drive every code to 255): codes equal the
    oracle's bit for bit."""
    prog = _hub(n)
    w = aspgen.mpnn_weights(9)
    if saturate:
        for k in ("Ev", "Ec", "P", "N", "S", "Q", "R", "T"):
            w[k] = np.full_like(w[k], 127)
        w["wo"] = np.full_like(w["wo"], -127)
    want = mpnn.scores(w, prog)
    g = P.Program(prog)
    g.bind("cuda")
    assert np.array_equal(g.score(w), want)


def test_scorer_batch_and_learned_search_end_to_end(P):
    """Batched scorer over uneven programs, then the score-driven batched
    search: every atom code and every search equals the oracle's."""
    progs = [aspgen.tiny_program(s, 4, 20) for s in range(12)]
    progs += [aspgen.single_random(1300 + s) for s in range(3)]
    progs += [aspgen.batch_hamiltonian(s) for s in range(2)]
    progs += [aspgen.batch_random(s, a_lo=100, a_hi=500) for s in range(5)]
    w = aspgen.mpnn_weights(4)
    gp = [P.Program(p, decision=P.DECISION_SCORE, fallback_after=10) for p in progs]
    b = P.Batch(gp, threads=128, classes=3).bind("cuda")
    b.score(w)
    for i, p in enumerate(progs):
        want = mpnn.scores(w, p)
        assert np.array_equal(b.get_scores(i), want), i
    b.solve(P.limits(300, LIM_MS))
    verd, models, stats = b.results()
    for i, p in enumerate(progs):
        rc, m, st = oracle.solve(p, limits=oracle.make_limits(300), scores=mpnn.scores(w, p),
                                 fallback_after=10)
        assert verd[i] == STATUS[rc], (i, p.name)
        assert_same_stats(st, stats[i], p.name)
        if rc == oracle.SAT:
            assert np.array_equal(models[i], m)


def test_batch_scores_required(P):
    progs = [aspgen.tiny_program(s, 4, 10) for s in range(3)]
    gp = [P.Program(p, decision=P.DECISION_SCORE) for p in progs]
    b = P.Batch(gp).bind("cuda")
    b.set_scores(0, aspgen.decision_scores(0, progs[0].n_atoms))
    with pytest.raises(P.AspError):
        b.solve(P.limits(10, LIM_MS))
    for i in (1, 2):
        b.set_scores(i, aspgen.decision_scores(i, progs[i].n_atoms))
    b.solve(P.limits(50, LIM_MS))
    verd, _, stats = b.results()
    for i, p in enumerate(progs):
        rc, _, st = oracle.solve(p, limits=oracle.make_limits(50),
                                 scores=aspgen.decision_scores(i, p.n_atoms))
        assert verd[i] == STATUS[rc]
        assert_same_stats(st, stats[i], i)


def test_readout_training_matches_oracle(P):
    """Device readout training (float32, atomics) against the oracle's
    float64 Adam on the same last-layer codes and labels: losses to 1e-4
    relative, weights to 1e-3 (float32 sums of a few thousand terms move a
    gradient by ~1e-6 relative; Adam's normalised steps keep that small)."""
    progs = [aspgen.tiny_program(s, 8, 20) for s in range(6)]
    progs += [aspgen.single_random(1400 + s) for s in range(2)]
    progs += [aspgen.batch_random(s, a_lo=100, a_hi=300) for s in range(2)]
    w = aspgen.mpnn_weights(0)
    rng = np.random.default_rng(5)
    labels = [rng.integers(-1, 2, size=p.n_atoms).astype(np.int8) for p in progs]
    gp = [P.Program(p) for p in progs]
    b = P.Batch(gp).bind("cuda")
    wb, loss = b.train_readout(w, np.concatenate(labels), steps=40, lr=0.05)
    X, y = [], []
    for p, lab in zip(progs, labels):
        hv = mpnn.last_codes(w, mpnn.graph_of(p))
        sel = np.nonzero(lab >= 0)[0]
        X.append(hv[sel + 1] / 256.0)
        y.append(lab[sel])
    X = np.concatenate(X)
    y = np.concatenate(y).astype(np.float64)
    wr, lr_ = mpnn.train_readout(X, y, 40, 0.05)
    assert np.allclose(loss, lr_, rtol=1e-4, atol=1e-6), (loss[:5], lr_[:5])
    assert np.allclose(wb, wr, rtol=1e-3, atol=1e-3), np.abs(wb - wr).max()
    assert loss[-1] < loss[0]
