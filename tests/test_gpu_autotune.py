"""The schedule autotuner (paper_1909_01786_amd/autotune.py) on the GPU.

A schedule only lays the batch onto the device, so every candidate -- one to
four LDS classes, 64 to 1024 threads per workgroup -- must give the same
verdicts, counters and trace hashes; the autotuner itself raises when one
does not.  The chosen schedule is then checked against the oracle.
"""
import os

import numpy as np
import pytest

import aspgen
import oracle
from parity import assert_same_stats, STATUS

pytestmark = pytest.mark.gpu

LIM_MS = int(os.environ.get("ASP_TEST_MAX_MS", "60000"))


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1909_01786_amd as P
    P.lib()
    return P


def _mixed():
    """64 programs over every LDS class: small and large random programs of
    the benchmark family, Hamiltonian-cycle programs, 3-colourings."""
    progs = [aspgen.batch_random(i, a_lo=100, a_hi=5000) for i in range(40)]
    progs += [aspgen.batch_random(i, batch_seed=77, a_lo=3500, a_hi=5000) for i in range(8)]
    progs += [aspgen.batch_hamiltonian(i) for i in range(12)]
    progs += [aspgen.gnp_coloring(2000 + s, n=300) for s in range(4)]
    return progs


def test_autotune_candidates_agree_and_match_oracle(P):
    from paper_1909_01786_amd.autotune import autotune
    progs = _mixed()
    gp = [P.Program(p, learned_cap_ng=1024, learned_cap_lits=1 << 16) for p in progs]
    budget = 60
    lim = P.limits(budget, LIM_MS)
    cands = ((4, (256, 128, 128, 64)), (4, (512, 256, 128, 128)), (4, (64, 64, 64, 64)),
             (1, (1024,)), (2, (256, 128)), (3, (128, 128, 128)))
    (classes, cth), table = autotune(gp, lim, candidates=cands)   # raises on any difference
    assert len(table) == len(cands)
    assert all(ms > 0 for _, _, ms in table)
    assert (classes, tuple(cth)) in [(c, tuple(t)) for c, t in cands]
    b = P.Batch(gp, classes=classes, class_threads=list(cth)).bind("cuda")
    b.solve(lim)
    verd, models, stats = b.results()
    lim_o = oracle.make_limits(budget, 1024, 1 << 16)
    for i in range(0, len(progs), 3):
        rc, m, st = oracle.solve(progs[i], limits=lim_o)
        assert verd[i] == STATUS[rc], (i, verd[i], rc)
        assert_same_stats(st, stats[i], progs[i].name)
        if rc == oracle.SAT:
            assert np.array_equal(models[i], m)
