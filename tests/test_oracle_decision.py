"""Pins of the oracle's score-driven Decision and of the integer atom scorer.

The Decision of the paper (Sect. 2) takes an applicable rule by a heuristic
score of its head; the learned Decision supplies that score per atom and
falls back to occurrence counting after a run of conflicts.  The scorer is
pinned against two other formulations of the same network (explicit loops
over nodes and edges, and dense incidence matrices), closed forms, and the
exactness premise of its float32 accumulation.
"""
from fractions import Fraction

import numpy as np
import pytest

import aspgen
import oracle
from oracle import mpnn
from brute import is_stable, stable_models


# ------------------------------------------------ score-driven Decision
@pytest.mark.parametrize("seed", range(40))
def test_occ_scores_reproduce_plain_search(seed):
    """Supplying occ(p) itself as the score, with no fallback, is the plain
    occurrence heuristic: same trace hash, same counters, same verdict."""
    prog = aspgen.tiny_program(seed, 4, 20) if seed < 30 else aspgen.single_random(1000 + seed)
    occ = oracle.Solver(prog).occ()
    lim = oracle.make_limits(300)
    r0 = oracle.solve(prog, limits=lim)
    r1 = oracle.solve(prog, limits=lim, scores=occ, fallback_after=-1)
    assert r0[0] == r1[0]
    assert r0[2] == r1[2]


def _applicable(st, prog_A, Rh, heads):
    out = []
    for j in range(Rh):
        p, t, n = heads[j], prog_A + 3 * j + 2, prog_A + 3 * j + 3
        if st.val[p] == 0 and st.val[t] == 1 and st.val[n] != -1:
            out.append(j)
    return out


def _heads(prog):
    return [h for h, _ in prog.rules() if h != 0]


@pytest.mark.parametrize("seed", range(60))
def test_every_decision_is_the_best_applicable_rule(seed):
    """Walk the search: each Decision takes an applicable rule whose head has
    the highest score (occ after the fallback), ties to the lowest rule; and
    the fallback fires exactly when `fallback_after` conflicts came with no
    decision reaching a conflict-free fixpoint in between."""
    prog = aspgen.tiny_program(seed, 8, 20) if seed < 40 else aspgen.single_random(1100 + seed)
    sc = aspgen.decision_scores(seed, prog.n_atoms, -3, 3)   # many ties
    fb = 1 + seed % 4
    s = oracle.Solver(prog)
    s.set_scores(sc, fb)
    occ = s.occ()
    d = s.dims()
    A, Rh = int(d[1]), int(d[2])
    heads = _heads(prog)
    lim = oracle.make_limits(400)
    consec, dec_open, mode, fired = 0, False, 1, False
    for _ in range(20000):
        k = s.next_step()
        if k == oracle.ST_DONE:
            break
        if k in (oracle.ST_DECIDE, oracle.ST_COMPLETE, oracle.ST_GATE) and dec_open:
            consec = 0
        st = s.state()
        if k == oracle.ST_DECIDE:
            cand = _applicable(st, A, Rh, heads)
            table = sc if mode else occ
            best = max(cand, key=lambda j: (table[heads[j]], -j))
        s.step(lim)
        st2 = s.state()
        if k == oracle.ST_DECIDE:
            assert st2.dec[st2.cdl] == A + 3 * best + 1
            dec_open = True
        if k == oracle.ST_LEARN and s.stats()["conflicts"] > 0 and st2.status == oracle.RUNNING:
            consec += 1
            dec_open = False
            if mode and consec >= fb:
                mode, fired = 0, True
        got_mode, got_consec = s.score_mode()
        assert got_mode == mode
        if mode:
            assert got_consec == consec
    assert s.next_step() == oracle.ST_DONE


@pytest.mark.parametrize("seed", range(80))
def test_learned_scores_keep_verdicts(seed):
    """Scores change the search, never the answer: the verdict equals brute
    force and every model is stable."""
    prog = aspgen.tiny_program(seed, 4, 16)
    sc = aspgen.decision_scores(seed + 500, prog.n_atoms)
    rc, m, _ = oracle.solve(prog, scores=sc, fallback_after=2 + seed % 5)
    models = stable_models(prog)
    assert rc == (oracle.SAT if models else oracle.UNSAT)
    if rc == oracle.SAT:
        assert is_stable(prog, m)


def test_scores_rejected_after_start_and_wrong_shape():
    prog = aspgen.single_random(1001)
    s = oracle.Solver(prog)
    with pytest.raises(ValueError):
        s.set_scores(np.zeros(prog.n_atoms, np.int32))
    s.step()
    with pytest.raises(ValueError):
        s.set_scores(np.zeros(prog.n_atoms + 1, np.int32))


# ------------------------------------------------------ integer scorer
def _act(z):
    if z <= 0:
        return 0
    return min(255, (z + 256) // 512)


def _norm(s, n):
    k = 0
    while (1 << k) < max(n, 1):
        k += 1
    return s if k == 0 else (s + (1 << (k - 1))) // (1 << k)


def _loops(w, g):
    """The scorer with explicit loops over nodes and literals (small cases)."""
    x, y, deg = mpnn.features(g)
    V, n = g.V, g.n
    lits = [list(g.lits[g.off[c]:g.off[c + 1]]) for c in range(n)]
    occ = {v: [] for v in range(1, V + 1)}
    for c in range(n):
        for l in lits[c]:
            occ[abs(int(l))].append((c, l > 0))

    def vecmat(v, M):
        return [sum(int(v[i]) * int(M[i][j]) for i in range(len(v))) for j in range(M.shape[1])]

    hv = {v: [_act(z + int(w["ev"][j])) for j, z in enumerate(vecmat(x[v], w["Ev"]))]
          for v in range(1, V + 1)}
    hc = {c: [_act(z + int(w["ec"][j])) for j, z in enumerate(vecmat(y[c], w["Ec"]))]
          for c in range(n)}
    for l in range(mpnn.L):
        new_c = {}
        for c in range(n):
            agg = [0] * 64
            for lit in lits[c]:
                M = w["P"][l] if lit > 0 else w["N"][l]
                m = vecmat(hv[abs(int(lit))], M)
                agg = [a + b for a, b in zip(agg, m)]
            base = vecmat(hc[c], w["S"][l])
            new_c[c] = [_act(base[j] + _norm(agg[j], len(lits[c])) + int(w["bc"][l][j]))
                        for j in range(64)]
        hc = new_c
        new_v = {}
        for v in range(1, V + 1):
            agg = [0] * 64
            for c, positive in occ[v]:
                M = w["Q"][l] if positive else w["R"][l]
                m = vecmat(hc[c], M)
                agg = [a + b for a, b in zip(agg, m)]
            base = vecmat(hv[v], w["T"][l])
            new_v[v] = [_act(base[j] + _norm(agg[j], len(occ[v])) + int(w["bv"][l][j]))
                        for j in range(64)]
        hv = new_v
    return [0] + [sum(hv[v][j] * int(w["wo"][j]) for j in range(64)) + int(w["bo"])
                  for v in range(1, V + 1)]


@pytest.mark.parametrize("seed", range(3))
def test_scorer_equals_explicit_loops(seed):
    prog = aspgen.tiny_program(seed, 4, 6)
    g = mpnn.graph_of(prog)
    w = aspgen.mpnn_weights(seed)
    assert list(mpnn.forward(w, g)) == _loops(w, g)


def _dense(w, g):
    """The scorer through dense incidence matrices: Bp[c, v] = 1 when Tv is in
    c, Bn[c, v] = 1 when Fv is in c; aggregation is Bp (H P) + Bn (H N) and
    its transpose for the variables.  The products run in float64, exact
    here since every value stays below 2^40."""
    x, y, deg = mpnn.features(g)
    Bp = np.zeros((g.n, g.V + 1))
    Bn = np.zeros((g.n, g.V + 1))
    for c in range(g.n):
        for l in g.lits[g.off[c]:g.off[c + 1]]:
            (Bp if l > 0 else Bn)[c, abs(l)] += 1
    lens = (Bp.sum(1) + Bn.sum(1)).astype(np.int64)
    dv = (Bp.sum(0) + Bn.sum(0)).astype(np.int64)
    f = {k: np.asarray(v, np.float64) for k, v in w.items()}

    def exact(a):
        assert np.abs(a).max() < 2.0 ** 40
        return np.rint(a).astype(np.int64)

    hv = mpnn.act(x @ w["Ev"] + w["ev"])
    hv[0] = 0
    hc = mpnn.act(y @ w["Ec"] + w["ec"])
    for l in range(mpnn.L):
        hvf = hv.astype(np.float64)
        hc = mpnn.act(exact(hc @ f["S"][l]) + mpnn.norm(exact(Bp @ hvf @ f["P"][l] + Bn @ hvf @ f["N"][l]),
                                                        lens) + w["bc"][l])
        hcf = hc.astype(np.float64)
        hv = mpnn.act(exact(hv @ f["T"][l]) + mpnn.norm(exact(Bp.T @ hcf @ f["Q"][l] + Bn.T @ hcf @ f["R"][l]),
                                                        dv) + w["bv"][l])
        hv[0] = 0
    out = hv @ w["wo"] + w["bo"]
    out[0] = 0
    return out


@pytest.mark.parametrize("prog", [aspgen.single_random(1001),
                                  aspgen.hamiltonian(8, [(u, (u + d) % 8) for u in range(8)
                                                         for d in (1, 2, 5)]),
                                  aspgen.batch_random(7, a_lo=100, a_hi=150)],
                         ids=["random200", "hc8", "batch"])
def test_scorer_equals_dense_incidence_form(prog):
    g = mpnn.graph_of(prog)
    w = aspgen.mpnn_weights(11)
    assert np.array_equal(mpnn.forward(w, g), _dense(w, g))


def test_scorer_zero_matrices_closed_form():
    """With every matrix zero, each layer's output is act(bias) and every atom
    scores act(bv of the last layer) . wo + bo."""
    prog = aspgen.single_random(1002)
    g = mpnn.graph_of(prog)
    w = aspgen.mpnn_weights(3)
    for k in ("Ev", "Ec", "P", "N", "S", "Q", "R", "T"):
        w[k] = np.zeros_like(w[k])
    s = mpnn.forward(w, g)
    expect = int(np.sum([_act(int(b)) * int(o) for b, o in zip(w["bv"][-1], w["wo"])])) + w["bo"]
    assert (s[1:] == expect).all() and s[0] == 0


def test_scorer_activation_and_normalisation_points():
    """act and norm against their definitions (rounded halves up, floors of
    negative values, saturation) computed with exact fractions."""
    for z in [-10**6, -1, 0, 1, 255, 256, 767, 768, 130559, 130560, 10**9]:
        r = Fraction(z, 512)
        want = 0 if z <= 0 else min(255, int(np.floor(r + Fraction(1, 2))))
        assert int(mpnn.act(z)) == want
    for s in [-7, -3, -2, -1, 0, 1, 2, 3, 5, 1001, -1001]:
        for n in [0, 1, 2, 3, 4, 5, 8, 9, 100]:
            k = 0
            while (1 << k) < max(n, 1):
                k += 1
            want = int(np.floor(Fraction(s, 1 << k) + Fraction(1, 2))) if k else s
            assert int(mpnn.norm(s, n)) == want


def test_scorer_exact_in_float32_accumulation():
    """The premise that makes the network order-independent: the largest
    64-term dot product of activation codes (<= 255) and weight codes
    (|k| <= 127) is below 2^24, so every partial sum is an exactly
    representable float32 integer, and the codes themselves are exact in
    bfloat16 (8 significant bits)."""
    worst = 64 * 255 * 127
    assert worst < 2 ** 24
    assert float(np.float32(worst)) == worst
    for v in list(range(0, 256)) + list(range(-127, 128)):
        f = np.array([v], np.float32).view(np.uint32)[0]
        assert f & 0xFFFF == 0, v          # exact as a bfloat16


def test_scorer_learned_scores_drive_oracle():
    """End to end on the oracle: the scorer's codes are valid Decision input
    and keep the verdict."""
    prog = aspgen.single_random(1003)
    sc = mpnn.scores(aspgen.mpnn_weights(5), prog)
    assert sc.shape == (prog.n_atoms + 1,) and sc.dtype == np.int32
    rc, m, st = oracle.solve(prog, scores=sc)
    rc0, _, _ = oracle.solve(prog)
    assert rc == rc0
    if rc == oracle.SAT:
        assert is_stable(prog, m)


# ------------------------------------------------------ readout training
def _toy_readout(seed, n=400):
    rng = np.random.default_rng(seed)
    X = rng.integers(0, 256, size=(n, 64)).astype(np.float64) / 256.0
    w_true = rng.normal(size=64)
    y = (X @ w_true - np.median(X @ w_true) + rng.normal(scale=0.5, size=n) > 0).astype(np.float64)
    return X, y


def test_readout_gradient_matches_finite_differences():
    X, y = _toy_readout(1)
    wb = np.random.default_rng(2).normal(scale=0.1, size=65)
    f0, g = mpnn.readout_loss_grad(X, y, wb)
    for i in (0, 7, 31, 63, 64):
        e = np.zeros(65)
        e[i] = 1e-6
        fp = mpnn.readout_loss_grad(X, y, wb + e)[0]
        fm = mpnn.readout_loss_grad(X, y, wb - e)[0]
        assert abs((fp - fm) / 2e-6 - g[i]) < 1e-6, i


def test_readout_training_reaches_the_minimiser():
    """The oracle's Adam, run long on the convex loss (with a small ridge
    term, which keeps the minimiser bounded), ends at scipy's minimiser of
    the same objective; without ridge it lowers the loss from the start."""
    from scipy.optimize import minimize
    X, y = _toy_readout(3, 300)
    lam = 1e-2

    def f(wb):
        l, g = mpnn.readout_loss_grad(X, y, wb)
        return l + 0.5 * lam * wb[:64] @ wb[:64], g + lam * np.concatenate([wb[:64], [0]])
    ref = minimize(f, np.zeros(65), jac=True, method="L-BFGS-B", options={"gtol": 1e-10}).x
    wb, losses = mpnn.train_readout(X, y, 6000, 0.01, ridge=lam)
    assert np.abs(wb - ref).max() < 5e-3
    assert abs(losses[-1] - f(ref)[0]) < 1e-5
    _, losses = mpnn.train_readout(X, y, 50, 0.05)
    assert losses[-1] < losses[0] - 0.05
