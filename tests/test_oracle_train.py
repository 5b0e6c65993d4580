"""Pins of the float training reference (oracle/mpnn_train.py).

The float model is pinned to the integer scorer it is the float form of:
its activations, times 256, stay within the integer model's roundings of
the integer oracle's codes at every layer (a model with the sign matrices
swapped misses by up to 180 codes); its gradient is pinned to central
finite differences of its own loss; its loss to a closed form; and the
library's code <-> float conversions to the scales the reference states.
"""
import numpy as np
import pytest
import torch

import aspgen
from oracle import mpnn
from oracle import mpnn_train as T


# the graphs here are small: one thread avoids oversubscribing the host
torch.set_num_threads(1)

PROGS = {
    "random200": lambda: aspgen.single_random(1001),
    "hc": lambda: aspgen.batch_hamiltonian(5),
    "tiny": lambda: aspgen.tiny_program(7, 8, 12),
}


@pytest.mark.parametrize("name", sorted(PROGS))
@pytest.mark.parametrize("wseed", [0, 1])
def test_float_model_is_the_integer_scorer_over_256(name, wseed):
    """Embedding: within one code (act rounds to nearest, saturates at 255);
    each later layer: within 4 codes (the roundings of act and of the edge
    sums of earlier layers carried through one 64-term product)."""
    prog = PROGS[name]()
    w = aspgen.mpnn_weights(wseed)
    tr = []
    mpnn.forward(w, mpnn.graph_of(prog), tr)
    ft = T.trace(T.from_codes(w), prog)
    assert len(tr) == len(ft) == 4
    for l, ((iv, ic), (fv, fc)) in enumerate(zip(tr, ft)):
        dv = np.abs(iv[1:] - 256.0 * fv).max()
        dc = np.abs(ic - 256.0 * fc).max() if ic.size else 0.0
        bound = 1.0 if l == 0 else 4.0
        assert dv <= bound and dc <= bound, (name, wseed, l, dv, dc)


def test_gradient_matches_finite_differences():
    progs = [aspgen.tiny_program(11, 8, 12), aspgen.batch_hamiltonian(2, n_lo=6, n_hi=8)]
    rng = np.random.default_rng(3)
    w = aspgen.mpnn_weights(5, spread=60)
    for k in ("ev", "ec", "bc", "bv"):
        w[k] = w[k] // 4
    vec = T.from_codes(w)
    labels = [np.where(rng.random(p.n_atoms) < 0.8, rng.integers(0, 2, p.n_atoms), -1).astype(float)
              for p in progs]
    loss, g = T.loss_and_grad(vec, progs, labels)
    assert np.isfinite(loss) and loss > 0
    # coordinates where the gradient is not zero, plus a few at random
    nz = np.nonzero(np.abs(g) > 1e-7)[0]
    idx = np.concatenate([rng.choice(nz, 24, replace=False), rng.choice(T.NPARAM, 8, replace=False)])
    eps = 1e-6
    for i in idx:
        a, b = vec.copy(), vec.copy()
        a[i] += eps
        b[i] -= eps
        fd = (T.loss_and_grad(a, progs, labels)[0] - T.loss_and_grad(b, progs, labels)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 + 1e-4 * abs(g[i]), (i, fd, g[i])


def test_loss_closed_form_with_zero_network():
    """All parameters 0 but bo: every activation is 0, the logit is bo, the
    loss is softplus(bo) - mean(y) bo and d/dbo = sigmoid(bo) - mean(y)."""
    prog = aspgen.tiny_program(4, 6, 9)
    vec = np.zeros(T.NPARAM)
    bo = 0.7
    vec[-1] = bo
    y = (np.arange(prog.n_atoms) % 3 == 0).astype(float)
    y[1] = -1.0
    loss, g = T.loss_and_grad(vec, [prog], [y])
    lab = y[y >= 0]
    want = np.log1p(np.exp(bo)) - lab.mean() * bo
    assert abs(loss - want) < 1e-12
    assert abs(g[-1] - (1 / (1 + np.exp(-bo)) - lab.mean())) < 1e-12
    # wo's gradient is sum of (sigmoid - y) * a with a = 0
    assert np.abs(g[-65:-1]).max() == 0.0


def test_library_code_conversions_match_reference_scales():
    import paper_1909_01786_amd.binding as B
    for seed in range(3):
        w = aspgen.mpnn_weights(seed)
        p = B.dequantize(w)
        assert np.array_equal(p.astype(np.float64), T.from_codes(w).astype(np.float32).astype(np.float64))
        back = B.quantize(p)
        for k in w:
            assert np.array_equal(np.asarray(back[k]), np.asarray(w[k])), k
    # rounding to nearest and clipping to the code ranges
    p = np.zeros(T.NPARAM, np.float32)
    parts = T.split(p)
    parts["P"][0, 0, 0] = 3.0          # beyond 127/128: clipped to 127
    parts["P"][0, 0, 1] = 0.3 / 128    # rounds to 0
    parts["P"][0, 0, 2] = 0.6 / 128    # rounds to 1
    parts["bc"][0, 0] = -1000.0        # beyond 2^24 / 2^17: clipped
    parts["bo"][...] = 1.5 / 32768
    q = B.quantize(p)
    assert q["P"][0, 0, 0] == 127 and q["P"][0, 0, 1] == 0 and q["P"][0, 0, 2] == 1
    assert q["bc"][0, 0] == -(1 << 24) and q["bo"] == 2
