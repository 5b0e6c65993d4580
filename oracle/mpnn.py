"""Plain integer oracle of the learned Decision's atom scorer.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it; the product path never does.  It shares
no code with the HIP library.

The paper's Decision picks an applicable rule by a heuristic score of its
head (Sect. 2, the ASP-computation Decision; occurrence counting is the
heuristic it names first).  The learned Decision replaces that score by the
output of a small message-passing network over the bipartite graph of
variables and static nogoods, whose edges are the nogood literals with their
sign.  The network is quantisation-aware: weights are integer codes in
[-127, 127] and activations integer codes in [0, 255] (both exact in
bfloat16), so each 64-term dot product is an integer below 2^21 and is exact
in a float32 accumulator in any summation order.  The definition, in integer
arithmetic (all sums exact, >> is the arithmetic shift):

  act(z)   = 0 if z <= 0, else min(255, (z + 256) >> 9)
  norm(s, n) = s when n <= 1, else (s + 2^(k-1)) >> k with k = ceil(log2 n)
  embed    hv = act(x Ev + ev),   hc = act(y Ec + ec)
  layer l  hc = act(hc S_l + norm(sum_{Tv in c} (hv P_l) + sum_{Fv in c} (hv N_l), |c|) + bc_l)
           hv = act(hv T_l + norm(sum_{c with Tv} (hc Q_l) + sum_{c with Fv} (hc R_l), deg v) + bv_l)
  readout  score_v = hv wo + bo            (the decision code of atom v <= A)

Features (codes, 32 standing for 1): x_v = [32, 32 if v is an atom, 32 if
v is some b_r, t_r, n_r (three entries), L(#nogoods with Tv),
L(#nogoods with Fv), L(#nogoods with Tv or Fv)]; y_c = [32, r(32, |c|),
32 if |c| = 1, 2, 3, >= 4 (four entries), r(32 #positive literals, |c|), 0],
where L(d) = min(255, 16 * bit length of d) is a saturating log code of a
degree and r(a, b) = (a + b // 2) // b is a / b rounded half up (0 when
b = 0).
"""
from __future__ import annotations

import numpy as np

F, H, L = 8, 64, 3
ACT_MAX = 255
ACT_SHIFT = 9


class Graph:
    """Static nogoods of a program as seen by the scorer."""

    def __init__(self, V: int, A: int, off: np.ndarray, lits: np.ndarray):
        self.V, self.A = int(V), int(A)
        self.off = np.asarray(off, np.int64)
        self.lits = np.asarray(lits, np.int64)
        self.n = len(self.off) - 1
        self.lens = np.diff(self.off)
        self.ng_of_lit = np.repeat(np.arange(self.n), self.lens)
        self.var = np.abs(self.lits)
        self.pos = self.lits > 0


def graph_of(prog) -> Graph:
    """The program's static nogoods, from the oracle's own encoding."""
    from oracle import Solver
    s = Solver(prog)
    d = s.dims()
    V, A, n0 = int(d[0]), int(d[1]), int(d[3])
    off, lits = s.nogoods()
    off = off[: n0 + 1]
    return Graph(V, A, off, lits[: int(off[-1])])


def rdiv(a, b):
    """a / b rounded half up, for a >= 0 and b >= 1 (integers); 0 where b = 0
    (the empty nogood of an empty-body constraint)."""
    a = np.asarray(a, np.int64)
    b = np.asarray(b, np.int64)
    return np.where(b > 0, (a + b // 2) // np.maximum(b, 1), 0)


def act(z):
    z = np.asarray(z, np.int64)
    return np.where(z <= 0, 0, np.minimum(ACT_MAX, (z + (1 << (ACT_SHIFT - 1))) >> ACT_SHIFT))


def norm_shift(n):
    """k = ceil(log2 n) for n >= 1 (0 for n <= 1)."""
    n = np.maximum(np.asarray(n, np.int64), 1)
    k = np.zeros_like(n)
    while True:
        m = (np.int64(1) << k) < n
        if not m.any():
            return k
        k = k + m


def norm(s, n):
    s = np.asarray(s, np.int64)
    k = norm_shift(n)
    while k.ndim < s.ndim:
        k = k[..., None]
    half = np.where(k > 0, np.int64(1) << np.maximum(k - 1, 0), 0)
    return (s + half) >> k


def bitlen(a: np.ndarray) -> np.ndarray:
    """Bit length of non-negative integers (0 for 0), exactly."""
    v = np.asarray(a, np.int64).copy()
    n = np.zeros_like(v)
    while (v > 0).any():
        n += v > 0
        v >>= 1
    return n


def features(g: Graph):
    V, A = g.V, g.A
    dpos = np.bincount(g.var[g.pos], minlength=V + 1).astype(np.int64)
    dneg = np.bincount(g.var[~g.pos], minlength=V + 1).astype(np.int64)
    x = np.zeros((V + 1, F), np.int64)
    x[1:, 0] = 32
    x[1:A + 1, 1] = 32
    aux = np.arange(A + 1, V + 1)
    kind = (aux - A - 1) % 3
    x[aux[kind == 0], 2] = 32
    x[aux[kind == 1], 3] = 32
    x[aux[kind == 2], 4] = 32
    # degrees as saturating log codes: 16 * bit length (the occurrence
    # heuristic ranks by the total degree, column 7)
    x[1:, 5] = np.minimum(255, 16 * bitlen(dpos[1:]))
    x[1:, 6] = np.minimum(255, 16 * bitlen(dneg[1:]))
    x[1:, 7] = np.minimum(255, 16 * bitlen(dpos[1:] + dneg[1:]))
    lens = g.lens.astype(np.int64)
    npos = np.bincount(g.ng_of_lit[g.pos], minlength=g.n).astype(np.int64)
    y = np.zeros((g.n, F), np.int64)
    y[:, 0] = 32
    y[:, 1] = rdiv(32, lens)
    y[:, 2] = 32 * (lens == 1)
    y[:, 3] = 32 * (lens == 2)
    y[:, 4] = 32 * (lens == 3)
    y[:, 5] = 32 * (lens >= 4)
    y[:, 6] = rdiv(32 * npos, lens)
    return x, y, dpos + dneg


def forward(w: dict, g: Graph, trace: list | None = None) -> np.ndarray:
    """Scores of every variable (index 0 is 0), int64.  If ``trace`` is a
    list, the activations (hv, hc) after the embedding and after each layer
    are appended to it."""
    x, y, deg = features(g)
    hv = act(x @ w["Ev"] + w["ev"])
    hv[0] = 0
    hc = act(y @ w["Ec"] + w["ec"])
    if trace is not None:
        trace.append((hv.copy(), hc.copy()))
    for l in range(L):
        mp = hv @ w["P"][l]
        mn = hv @ w["N"][l]
        agg = np.zeros((g.n, H), np.int64)
        np.add.at(agg, g.ng_of_lit[g.pos], mp[g.var[g.pos]])
        np.add.at(agg, g.ng_of_lit[~g.pos], mn[g.var[~g.pos]])
        hc = act(hc @ w["S"][l] + norm(agg, g.lens) + w["bc"][l])
        mq = hc @ w["Q"][l]
        mr = hc @ w["R"][l]
        aggv = np.zeros((g.V + 1, H), np.int64)
        np.add.at(aggv, g.var[g.pos], mq[g.ng_of_lit[g.pos]])
        np.add.at(aggv, g.var[~g.pos], mr[g.ng_of_lit[~g.pos]])
        hv = act(hv @ w["T"][l] + norm(aggv, deg) + w["bv"][l])
        hv[0] = 0
        if trace is not None:
            trace.append((hv.copy(), hc.copy()))
    out = hv @ w["wo"] + int(w["bo"])
    out[0] = 0
    return out


def scores(w: dict, prog) -> np.ndarray:
    """Decision codes of atoms 0..A (index 0 is 0) as int32."""
    g = graph_of(prog)
    s = forward(w, g)[: g.A + 1]
    return s.astype(np.int32)


# ------------------------------------------------------------------ training
def last_codes(w: dict, g: Graph) -> np.ndarray:
    """Activation codes of every variable after the last layer ([V+1, 64])."""
    trace: list = []
    forward(w, g, trace)
    return trace[-1][0]


def readout_loss_grad(X: np.ndarray, y: np.ndarray, wb: np.ndarray):
    """Mean binary cross-entropy of sigmoid(X w + b) against y, and its
    gradient in (w, b).  X: [n, 64] float (codes / 256), y: 0/1."""
    z = X @ wb[:64] + wb[64]
    p = 1.0 / (1.0 + np.exp(-z))
    loss = float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))
    r = (p - y) / len(y)
    return loss, np.concatenate([X.T @ r, [r.sum()]])


def train_readout(X: np.ndarray, y: np.ndarray, steps: int, lr: float, wb0=None,
                  ridge: float = 0.0):
    """Full-batch Adam (beta 0.9 / 0.999, eps 1e-8) on readout_loss_grad
    (plus ridge/2 |w|^2 when ridge > 0; the device trains with none);
    returns the weights after `steps` steps and the loss before each."""
    wb = np.zeros(65) if wb0 is None else np.asarray(wb0, np.float64).copy()
    m = np.zeros(65)
    v = np.zeros(65)
    losses = np.zeros(steps)
    for t in range(steps):
        losses[t], gr = readout_loss_grad(X, y, wb)
        if ridge > 0:
            losses[t] += 0.5 * ridge * float(wb[:64] @ wb[:64])
            gr = gr + ridge * np.concatenate([wb[:64], [0.0]])
        m = 0.9 * m + 0.1 * gr
        v = 0.999 * v + 0.001 * gr * gr
        mh = m / (1.0 - 0.9 ** (t + 1))
        vh = v / (1.0 - 0.999 ** (t + 1))
        wb = wb - lr * mh / (np.sqrt(vh) + 1e-8)
    return wb, losses
