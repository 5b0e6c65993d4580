"""The learned Decision's training kernels against the float reference.

asp_scorer_train runs the float scorer's forward and backward passes on the
matrix cores with bfloat16 operands and float32 accumulation; the reference
(oracle/mpnn_train.py) is the same model in float64 with autograd.  Bfloat16
keeps 8 significant bits, so each product carries a relative error up to
2^-8 and the passes through three layers compound it; clamp masks may flip
for the few pre-activations within that error of 0 or 1.  The comparison is
therefore norm-wise per parameter group: relative L2 error at most 0.05 and
cosine at least 0.995, loss within 1%.  Adam moves every parameter with a
non-zero gradient by about lr whatever the gradient's size, so parameters
whose gradient is within bf16 noise of 0 move either way and two runs'
parameters part after the first step; the Adam arithmetic is therefore
checked on the device's own gradient (to float32 rounding), and the
trajectory on the loss curve.
"""
import os

import numpy as np
import pytest
import torch

import aspgen
import oracle
from oracle import mpnn_train as T
from parity import STATUS

pytestmark = pytest.mark.gpu

torch.set_num_threads(8)


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1909_01786_amd as P
    P.lib()
    return P


def _setup(seed):
    progs = [aspgen.tiny_program(20 + seed, 10, 16), aspgen.single_random(1001 + seed),
             aspgen.batch_hamiltonian(seed + 3)]
    rng = np.random.default_rng(seed)
    labels = [np.where(rng.random(p.n_atoms) < 0.7, rng.integers(0, 2, p.n_atoms), -1).astype(np.float32)
              for p in progs]
    w = aspgen.mpnn_weights(seed, spread=90)
    for k in ("ev", "ec", "bc", "bv"):
        w[k] = w[k] // 4
    return progs, labels, w


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_pass_matches_reference(P, seed):
    from paper_1909_01786_amd import binding as B
    progs, labels, w = _setup(seed)
    vec = B.dequantize(w)
    gp = [P.Program(p) for p in progs]
    _, loss, grad = B.train_scorer(gp, labels, vec, steps=0)
    ref_loss, ref_grad = T.loss_and_grad(vec.astype(np.float64), progs, labels)
    assert abs(loss[0] - ref_loss) <= 0.01 * abs(ref_loss), (loss[0], ref_loss)
    gd, rd = T.split(grad.astype(np.float64)), T.split(ref_grad)
    for name, _ in T.layout():
        a, b = gd[name].reshape(-1), rd[name].reshape(-1)
        nb = np.linalg.norm(b)
        if nb < 1e-9:
            assert np.linalg.norm(a) < 1e-6, name
            continue
        rel = np.linalg.norm(a - b) / nb
        cos = float(a @ b) / (np.linalg.norm(a) * nb + 1e-30)
        assert rel <= 0.05 and cos >= 0.995, (name, rel, cos)


def test_adam_steps_match_reference(P):
    """One step from the device's own gradient is Adam to float32 rounding;
    ten steps follow the reference's loss curve within 2%."""
    from paper_1909_01786_amd import binding as B
    progs, labels, w = _setup(2)
    vec = B.dequantize(w)
    gp = [P.Program(p) for p in progs]
    lr, steps = 2e-3, 10
    one, _, g1 = B.train_scorer(gp, labels, vec, steps=1, lr=lr)
    want, _ = T.adam(vec.astype(np.float64), lambda v: (0.0, g1.astype(np.float64)), 1, lr)
    assert np.abs(one - want).max() <= 1e-6, float(np.abs(one - want).max())
    _, losses, _ = B.train_scorer(gp, labels, vec, steps=steps, lr=lr)
    _, ref_losses = T.adam(vec.astype(np.float64),
                           lambda v: T.loss_and_grad(v, progs, labels), steps, lr)
    assert np.allclose(losses, ref_losses, rtol=0.02), (losses, ref_losses)


def test_training_lowers_the_loss_and_quantizes(P):
    """Labels the network can represent -- an atom is 1 when its occurrence
    count is at least the program's median, which the degree features carry
    -- fall from about ln 2 within 40 steps; the quantized result is a valid
    weight set the integer scorer and the search accept."""
    from paper_1909_01786_amd import binding as B
    progs, _, w = _setup(3)
    labels = []
    for p in progs:
        occ = oracle.Solver(p).occ()[1:].astype(np.float64)
        labels.append((occ >= np.median(occ)).astype(np.float32))
    gp = [P.Program(p) for p in progs]
    vec, losses, _ = B.train_scorer(gp, labels, B.dequantize(w), steps=40, lr=5e-3)
    assert losses[-1] < 0.85 * losses[0] and losses[-1] < 0.6, (losses[0], losses[-1])
    codes = B.quantize(vec)
    g = P.Program(progs[1], decision=P.DECISION_SCORE).bind("cuda")
    sc = g.score(codes)
    from oracle import mpnn
    assert np.array_equal(sc[1:], mpnn.scores(codes, progs[1])[1:])
    rc, m, st = g.solve(P.limits(2000, 60000))
    orc, om, ost = oracle.solve(progs[1], scores=sc, fallback_after=10,
                                limits=oracle.make_limits(2000))
    assert rc == STATUS[orc] and st["trace_hash"] == ost["trace_hash"]


def test_batch_learned_nogoods_are_the_oracles(P):
    """The conflict traces read back from a batch (asp_batch_learned) are
    the oracle's learned nogoods, nogood for nogood."""
    progs = [aspgen.batch_random(i, a_lo=100, a_hi=400) for i in range(12)]
    gp = [P.Program(p, learned_cap_ng=4096, learned_cap_lits=1 << 18) for p in progs]
    b = P.Batch(gp).bind("cuda")
    b.solve(P.limits(300, 60000))
    torch.cuda.synchronize()
    for i, prog in enumerate(progs):
        s = oracle.Solver(prog)
        s.run(oracle.make_limits(300, 4096, 1 << 18))
        st = s.state()
        n0 = st.n_static
        base = int(st.ng_off[n0])
        o_off = (st.ng_off[n0:] - base).astype(np.int32)
        o_lits = st.ng_lits[base:].astype(np.int32)
        off, lits = b.learned(i)
        assert np.array_equal(off, o_off) and np.array_equal(lits, o_lits), i
