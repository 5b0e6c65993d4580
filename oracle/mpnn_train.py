"""Float reference of the learned Decision scorer's training.

TEST INFRASTRUCTURE ONLY: the test-suite uses it to check the device
training kernels; the product path never does.  It shares no code with the
HIP library.

The integer scorer (oracle/mpnn.py) is trained in its float form: an
activation is its code / 256, a matrix entry its code / 128, a layer or
embedding bias its code / 2^17, the readout bias its code / 2^15.  Dividing
the integer layer act(z) = min(255, (z + 256) >> 9) by 256 then gives,
up to the roundings of act and of the edge-sum normalisation,

    embed    a = clamp(x E / 4 + e, 0, 1)           (x: feature codes / 256)
    layer l  ac = clamp((ac S + (sum_{Tv in c} av P + sum_{Fv in c} av N) / 2^k(|c|)) / 4 + bc, 0, 1)
             av = clamp((av T + (sum_{c with Tv} ac Q + sum_{c with Fv} ac R) / 2^k(deg v)) / 4 + bv, 0, 1)
    logit    s = av wo + bo

with k(n) = ceil(log2 n) (0 for n <= 1), the nogood update using the
variables' previous activations and the variable update the nogoods' new
ones.  The loss is the mean binary cross-entropy of sigmoid(s) against the
labels of the labelled atoms.  This module writes that model with plain
PyTorch CPU operations in float64 and takes its gradient by autograd; the
parameter vector has the layout of the C ABI (asp.h, ASP_SCORER_NPARAM).
Variable 0 does not exist as a row here (it has no edges and code 0).
"""
from __future__ import annotations

import numpy as np

from oracle import mpnn

F, H, L = 8, 64, 3
SCALE_W, SCALE_B, SCALE_BO = 128.0, 131072.0, 32768.0


def layout():
    """(name, shape) of each parameter group, in vector order."""
    return [("Ev", (F, H)), ("Ec", (F, H)), ("ev", (H,)), ("ec", (H,)),
            ("P", (L, H, H)), ("N", (L, H, H)), ("S", (L, H, H)), ("Q", (L, H, H)),
            ("R", (L, H, H)), ("T", (L, H, H)), ("bc", (L, H)), ("bv", (L, H)),
            ("wo", (H,)), ("bo", ())]


NPARAM = sum(int(np.prod(s)) for _, s in layout())


def split(vec):
    """Parameter vector -> dict of views (numpy or torch)."""
    out, o = {}, 0
    for name, shape in layout():
        n = int(np.prod(shape))
        out[name] = vec[o:o + n].reshape(shape)
        o += n
    return out


def from_codes(w: dict) -> np.ndarray:
    """Integer weight codes (aspgen.mpnn_weights layout) -> float vector."""
    parts = []
    for name, shape in layout():
        a = np.asarray(w[name], np.float64).reshape(shape)
        scale = SCALE_BO if name == "bo" else (
            SCALE_B if name in ("ev", "ec", "bc", "bv") else SCALE_W)
        parts.append((a / scale).reshape(-1))
    return np.concatenate(parts)


def log2ceil(n: np.ndarray) -> np.ndarray:
    return mpnn.norm_shift(n)


def graph_tensors(prog):
    """The program's static nogoods as the float model sees them (kept on
    the program object after the first call)."""
    memo = getattr(prog, "_float_graph", None)
    if memo is None:
        g = mpnn.graph_of(prog)
        x, y, deg = mpnn.features(g)
        memo = (g, x[1:].astype(np.float64) / 256.0, y.astype(np.float64) / 256.0, deg[1:])
        prog._float_graph = memo
    return memo


def _forward(W, prog):
    """Float activations (av over variables 1..V, ac over static nogoods)
    after the embedding and after each layer, as torch float64 tensors."""
    import torch
    g, xv, xc, deg = graph_tensors(prog)
    av = torch.clamp(torch.tensor(xv) @ W["Ev"] / 4 + W["ev"], 0, 1)
    ac = torch.clamp(torch.tensor(xc) @ W["Ec"] / 4 + W["ec"], 0, 1)
    out = [(av, ac)]
    var_row = torch.tensor(g.var - 1)
    ng = torch.tensor(g.ng_of_lit)
    pos = torch.tensor(g.pos)
    cscale = torch.tensor(2.0 ** -log2ceil(g.lens).astype(np.float64))
    vscale = torch.tensor(2.0 ** -log2ceil(deg).astype(np.float64))
    for l in range(L):
        mp = av @ W["P"][l]
        mn = av @ W["N"][l]
        src = torch.where(pos[:, None], mp[var_row], mn[var_row])
        agg = torch.zeros((g.n, H), dtype=torch.float64).index_add(0, ng, src)
        ac = torch.clamp((ac @ W["S"][l] + agg * cscale[:, None]) / 4 + W["bc"][l], 0, 1)
        mq = ac @ W["Q"][l]
        mr = ac @ W["R"][l]
        srcv = torch.where(pos[:, None], mq[ng], mr[ng])
        aggv = torch.zeros((g.V, H), dtype=torch.float64).index_add(0, var_row, srcv)
        av = torch.clamp((av @ W["T"][l] + aggv * vscale[:, None]) / 4 + W["bv"][l], 0, 1)
        out.append((av, ac))
    return out


def trace(vec, prog):
    """[(av, ac)] as numpy arrays after the embedding and each layer."""
    import torch
    W = split(torch.tensor(np.asarray(vec, np.float64)))
    return [(a.numpy(), c.numpy()) for a, c in _forward(W, prog)]


def loss_and_grad(vec, progs, labels_per_prog):
    """Mean BCE over the labelled atoms of all programs and its gradient.
    labels_per_prog[i]: float array over atoms 1..A (< 0: no label)."""
    import torch
    p = torch.tensor(np.asarray(vec, np.float64), requires_grad=True)
    W = split(p)
    terms, n_lab = [], 0
    for prog, lab in zip(progs, labels_per_prog):
        av = _forward(W, prog)[-1][0]
        lab = np.asarray(lab, np.float64)
        sel = np.nonzero(lab >= 0)[0]
        if sel.size == 0:
            continue
        z = av[torch.tensor(sel)] @ W["wo"] + W["bo"]
        yl = torch.tensor(np.minimum(lab[sel], 1.0))
        terms.append(torch.clamp(z, min=0) - z * yl + torch.log1p(torch.exp(-torch.abs(z))))
        n_lab += sel.size
    total = torch.cat(terms).sum() / n_lab
    total.backward()
    return float(total.detach()), p.grad.numpy().copy()


def adam(vec, grad_fn, steps: int, lr: float):
    """Full-batch Adam (0.9 / 0.999, eps 1e-8) with the parameters clipped
    after each step to the ranges their codes hold; returns (vec, losses)."""
    p = np.asarray(vec, np.float64).copy()
    lim = np.empty(NPARAM)
    o = 0
    for name, shape in layout():
        n = int(np.prod(shape))
        lim[o:o + n] = 512.0 if name == "bo" else (
            128.0 if name in ("ev", "ec", "bc", "bv") else 127.0 / 128.0)
        o += n
    m = np.zeros(NPARAM)
    v = np.zeros(NPARAM)
    losses = []
    for t in range(1, steps + 1):
        loss, g = grad_fn(p)
        losses.append(loss)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        p = p - lr * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
        p = np.clip(p, -lim, lim)
    return p, losses
