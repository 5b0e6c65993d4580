"""Full-size parity: the batches at their benchmark sizes, in the launch
configuration the benchmark times, checked on sampled instances against the
oracle (verdict, model and every counter) and on every returned model
against the answer-set definition."""
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import aspgen
import oracle
from brute import is_stable
from parity import STATUS, assert_same_stats

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _solve_batch(progs, budget, threads, classes, cap_ng, cap_lits):
    import torch
    import paper_1909_01786_amd as P
    with ThreadPoolExecutor(16) as ex:
        gp = list(ex.map(lambda p: P.Program(p, learned_cap_ng=cap_ng,
                                             learned_cap_lits=cap_lits), progs))
    b = P.Batch(gp, threads=threads, classes=classes).bind("cuda")
    b.solve(P.limits(budget, 150000))
    torch.cuda.synchronize()
    return b.results()


def _sample_against_oracle(progs, verd, models, stats, budget, cap_ng, cap_lits,
                           n_sample, max_checks):
    rng = np.random.default_rng(7)
    order = rng.permutation(len(progs))
    pick, acc = [], 0
    for i in order:
        c = int(stats[i]["literal_checks"])
        if acc + c > max_checks and pick:
            continue
        pick.append(int(i))
        acc += c
        if len(pick) >= n_sample:
            break
    lim = oracle.make_limits(budget, cap_ng, cap_lits)
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        res = list(ex.map(lambda i: (i, oracle.solve(progs[i], limits=lim)), pick))
    for i, (rc, m, st) in res:
        assert verd[i] == STATUS[rc], (i, verd[i], rc)
        assert_same_stats(st, stats[i], progs[i].name)
        if rc == oracle.SAT:
            assert np.array_equal(models[i], m)
    return len(pick)


def test_random_batch_4096_bench_configuration():
    """4096 uneven random programs, budget 2000, 128 threads, 4 LDS classes."""
    import bench
    t = time.time()
    progs = bench.make_batch(4096, 3000)
    verd, models, stats = _solve_batch(progs, 2000, 128, 4, 4096, 1 << 18)
    assert (verd > 0).all(), "no instance may end in an error"
    n = _sample_against_oracle(progs, verd, models, stats, 2000, 4096, 1 << 18,
                               n_sample=48, max_checks=int(3e9))
    assert n >= 16
    sat = np.nonzero(verd == 1)[0]
    assert sat.size > 0
    for i in sat:
        assert is_stable(progs[i], models[i]), i
    print(f"4096 batch: {n} sampled instances equal to the oracle, "
          f"{sat.size} models stable, {time.time() - t:.0f}s")


def test_hamiltonian_batch_512():
    """512 Hamiltonian-cycle programs (recursive reachability), budget 2000."""
    progs = [aspgen.batch_hamiltonian(i) for i in range(512)]
    verd, models, stats = _solve_batch(progs, 2000, 128, 4, 4096, 1 << 18)
    assert (verd > 0).all()
    n = _sample_against_oracle(progs, verd, models, stats, 2000, 4096, 1 << 18,
                               n_sample=64, max_checks=int(2e9))
    assert n >= 32
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
