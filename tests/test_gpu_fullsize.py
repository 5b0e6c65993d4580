"""Full-size parity: the batches at their benchmark sizes, in the launch
configuration the benchmark times.

The 4096-program batch is compared with the oracle instance by instance --
verdict, every search counter, the trace hash and the answer sets -- for the
plain search and for the Jeroslow-Wang, activity, several-conflicts,
several-answer-sets and lookahead searches, against the oracle's stored run of the whole
batch (tests/golden/oracle_batch.py, written by the oracle alone).
Res-learning is compared on a sample stratified by LDS class (the largest
class runs on its 256-thread launch) against the oracle's stored run of it,
the learned Decision on such a sample with the oracle running beside the
test; the learned scorer's atom codes are compared on full-size programs of
every class.  Every returned model is an answer set.
"""
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor, as_completed

import numpy as np
import pytest

import aspgen
import oracle
from oracle import mpnn
from brute import is_stable
from parity import STATUS, assert_same_stats

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
import oracle_batch as ob  # noqa: E402

N, SEED, BUDGET, CAP_NG, CAP_LITS = 4096, ob.SEED, ob.BUDGET, ob.CAP_NG, ob.CAP_LITS
SCHEDULE = dict(threads=128, classes=4, class_threads=[256, 128, 128, 128])
KEYS = ("rounds", "visits", "literal_checks", "propagations", "decisions", "conflicts",
        "learned", "learned_len", "gate_failures", "completes", "trace_hash")
WORKERS = 16


@pytest.fixture(scope="module")
def progs():
    return [aspgen.batch_random(i, batch_seed=SEED) for i in range(N)]


def _log(*a):
    print(*a, flush=True)


def _pool_map(fn, items):
    """fn over items on the host cores, one progress line per result as it
    completes; results in the order of items."""
    out = [None] * len(items)
    with ThreadPoolExecutor(WORKERS) as ex:
        futs = {ex.submit(fn, it): k for k, it in enumerate(items)}
        for n, f in enumerate(as_completed(futs)):
            out[futs[f]] = f.result()
            _log(f"  oracle {n + 1}/{len(items)} done")
    return out


def _solve_batch(progs, budget=BUDGET, cap_ng=CAP_NG, cap_lits=CAP_LITS, scorer=None,
                 all_models=False, **kw):
    import torch
    import paper_1909_01786_amd as P
    _log(f"  batch of {len(progs)} programs, options {kw}")
    with ThreadPoolExecutor(WORKERS) as ex:
        gp = list(ex.map(lambda p: P.Program(p, learned_cap_ng=cap_ng,
                                             learned_cap_lits=cap_lits, **kw), progs))
    b = P.Batch(gp, **SCHEDULE).bind("cuda")
    if scorer is not None:
        b.score(scorer)
    b.solve(P.limits(budget, 150000))
    torch.cuda.synchronize()
    verd, models, stats = b.results(all_models=all_models)
    _log("  batch solved")
    return b, verd, models, stats


def _stratified(progs, per_class, seed=7):
    """per_class programs of each LDS class, drawn at random."""
    rng = np.random.default_rng(seed)
    strata = [[] for _ in range(4)]
    for i in rng.permutation(len(progs)):
        strata[ob.lds_class(progs[int(i)])].append(int(i))
    return [i for st in strata for i in st[:per_class]]


MODES = {
    "plain": {},
    "jw": {"decision": 2},
    "activity": {"decision": 3},
    "multi4": {"learn_conflicts": 4},
    "enum16": {"max_models": 16},
    "look4": {"lookahead": 4},
}


@pytest.mark.parametrize("mode", sorted(MODES))
def test_batch4096_every_instance_equals_oracle(progs, mode):
    """All 4096 instances against the oracle's stored run of the batch."""
    t = time.time()
    rows = ob.load(mode, N)
    assert rows is not None, f"missing {ob.path(mode, N)}: run tests/golden/oracle_batch.py {mode}"
    enum = "max_models" in MODES[mode]
    _, verd, models, stats = _solve_batch(progs, all_models=enum, **MODES[mode])
    assert (verd > 0).all(), "no instance may end in an error"
    bad = []
    for i in range(N):
        r, g = rows[i], stats[i]
        ms = models[i] if enum else ([models[i]] if verd[i] == 1 else [])
        same = int(verd[i]) == r["status"] and all(
            (int(g[k]) & (2 ** 64 - 1)) == r[k] for k in KEYS)
        same = same and ob.models_sha(ms) == r["models_sha"]
        if enum:
            same = same and int(g["models"]) == r["models"] and int(g["exhausted"]) == r["exhausted"]
        if not same:
            bad.append(i)
    assert not bad, f"{len(bad)} instances differ from the oracle, first {bad[:8]}"
    n_models = 0
    for i in np.nonzero(verd == 1)[0]:
        for m in (models[i] if enum else [models[i]]):
            assert is_stable(progs[i], m), i
            n_models += 1
    print(f"{mode}: 4096 instances equal to the oracle, {n_models} answer sets stable, "
          f"{time.time() - t:.0f}s")


def test_batch4096_res_stratified(progs):
    """Res-learning on the whole batch; 4 programs of every LDS class (drawn
    at random; those the oracle finishes in 4 minutes) against the oracle's
    stored run of them: verdict, every counter, the trace hash and the
    answer set."""
    rows = ob.load("res", N)
    assert rows is not None, f"missing {ob.path('res', N)}: run tests/golden/oracle_batch.py res"
    pick = sorted(rows)
    per_class = [sum(1 for i in pick if ob.lds_class(progs[i]) == c) for c in range(4)]
    assert all(n > 0 for n in per_class), per_class
    _, verd, models, stats = _solve_batch(progs, learning=1)
    assert (verd > 0).all()
    for i in pick:
        r, g = rows[i], stats[i]
        assert int(verd[i]) == r["status"], (i, verd[i], r["status"])
        for k in KEYS:
            assert (int(g[k]) & (2 ** 64 - 1)) == r[k], (i, k, g[k], r[k])
        ms = [models[i]] if verd[i] == 1 else []
        assert ob.models_sha(ms) == r["models_sha"], i
        for m in ms:
            assert is_stable(progs[i], m), i
    print(f"res: {len(pick)} sampled instances equal to the oracle "
          f"({[ob.lds_class(progs[i]) for i in pick]} by class)")


def test_batch4096_learned_stratified(progs):
    """The learned Decision on the whole batch (device scorer, trained
    weights): atom codes of 2 programs per LDS class equal the oracle's
    scorer, and their searches equal the oracle's driven by those codes."""
    import paper_1909_01786_amd as P
    from paper_1909_01786_amd import binding as B
    w = B.load_weights()
    pick = _stratified(progs, 2, seed=11)
    b, verd, models, stats = _solve_batch(progs, scorer=P.scorer_weights(w),
                                          decision=P.DECISION_SCORE, fallback_after=10)
    assert (verd > 0).all()
    lim = oracle.make_limits(BUDGET, CAP_NG, CAP_LITS)

    def one(i):
        sc = mpnn.scores(w, progs[i])
        return i, sc, oracle.solve(progs[i], limits=lim, scores=sc, fallback_after=10)

    res = _pool_map(one, pick)
    for i, sc, (rc, m, st) in res:
        got = b.get_scores(i)
        assert np.array_equal(got[1:], sc[1:]), (i, "atom codes differ")
        assert verd[i] == STATUS[rc], (i, verd[i], rc)
        assert_same_stats(st, stats[i], progs[i].name)
        if rc == oracle.SAT:
            assert np.array_equal(models[i], m) and is_stable(progs[i], m)


def test_hamiltonian_batch_512():
    """512 Hamiltonian-cycle programs (recursive reachability), budget 2000;
    every 8th against the oracle."""
    progs = [aspgen.batch_hamiltonian(i) for i in range(512)]
    _, verd, models, stats = _solve_batch(progs)
    assert (verd > 0).all()
    pick = list(range(0, 512, 8))
    lim = oracle.make_limits(BUDGET, CAP_NG, CAP_LITS)
    res = _pool_map(lambda i: (i, oracle.solve(progs[i], limits=lim)), pick)
    for i, (rc, m, st) in res:
        assert verd[i] == STATUS[rc], (i, verd[i], rc)
        assert_same_stats(st, stats[i], progs[i].name)
        if rc == oracle.SAT:
            assert np.array_equal(models[i], m)
    for i in np.nonzero(verd == 1)[0]:
        assert is_stable(progs[i], models[i]), i


def test_coloring_2000_single():
    """The 2000-vertex 3-colouring as a single instance (W=32, 1024 threads),
    compared with the oracle under a conflict budget."""
    import paper_1909_01786_amd as P
    prog = aspgen.gnp_coloring(2002)
    g = P.Program(prog, W=32)
    g.bind("cuda", threads=1024)
    rc, m, st = g.solve(P.limits(4000, 150000))
    orc, om, ost = oracle.solve(prog, W=32, limits=oracle.make_limits(4000))
    assert rc == STATUS[orc]
    assert_same_stats(ost, st, prog.name)
    if orc == oracle.SAT:
        assert np.array_equal(m, om) and is_stable(prog, m)
