"""Seeded synthetic ground normal programs.

This module only *draws* programs; it holds none of the solving method's
arithmetic (no completion, no nogoods, no propagation).  Both the CPU oracle
and the HIP library read the programs it produces, so it is the one piece of
code the two sides share.

A ground program uses the rule form of the paper's Preliminaries (a head atom
and a body of positive and ``not`` literals; a constraint has no head).  It is
stored as a rule CSR:

* ``n_atoms``  -- atoms are numbered 1..n_atoms,
* ``head``     -- int32[n_rules], head atom id, 0 for a constraint,
* ``body_off`` -- int64[n_rules+1], offsets into ``body_lits``,
* ``body_lits``-- int32, ``+a`` for atom a, ``-a`` for ``not a``.

Workload families (all drawn with numpy ``PCG64``):

* :func:`random_program` -- uniform random normal programs; :func:`single_random`
  is the 200-atom / 600-rule single instance, :func:`batch_random` the batch of
  uneven programs (atoms log-uniform in 100..5000, rules/atoms in 2..4).
* :func:`coloring` -- ground 3-colouring of a graph (choice through even
  negative cycles, one constraint per edge and colour); :func:`gnp_coloring`
  draws the random graph G(n, p).
* :func:`hamiltonian` -- ground Hamiltonian-cycle programs with recursive
  reachability (non-tight); :func:`batch_hamiltonian` draws the random
  directed graphs.
* :func:`tiny_program` -- small programs (4..20 atoms) for brute-force checks.

The paper evaluates on ASP-competition instances that are not available here;
these families stand in for them with the same structure (sparse nogood sets
with 2-3 nogoods per atom, short nogoods, non-tight recursion).
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np

__all__ = [
    "Program", "random_program", "tiny_program", "single_random", "batch_random",
    "coloring", "gnp_coloring", "hamiltonian", "random_digraph",
    "batch_hamiltonian", "from_rules", "save_program", "load_program",
    "MPNN_F", "MPNN_H", "MPNN_L", "mpnn_weights", "decision_scores",
]


@dataclass
class Program:
    n_atoms: int
    head: np.ndarray       # int32[n_rules]
    body_off: np.ndarray   # int64[n_rules + 1]
    body_lits: np.ndarray  # int32[body_off[-1]]
    name: str = ""

    @property
    def n_rules(self) -> int:
        return int(self.head.shape[0])

    def rules(self):
        """Yield (head, [body literals]) in input order."""
        for r in range(self.n_rules):
            a, b = int(self.body_off[r]), int(self.body_off[r + 1])
            yield int(self.head[r]), [int(x) for x in self.body_lits[a:b]]

    def check(self) -> None:
        assert self.head.dtype == np.int32 and self.body_off.dtype == np.int64
        assert self.body_lits.dtype == np.int32
        assert self.body_off.shape[0] == self.n_rules + 1
        assert self.body_off[0] == 0 and self.body_off[-1] == self.body_lits.shape[0]


def from_rules(n_atoms: int, rules, name: str = "") -> Program:
    """Build a Program from a list of (head, [signed body literals])."""
    heads, offs, lits = [], [0], []
    for h, body in rules:
        heads.append(int(h))
        lits.extend(int(x) for x in body)
        offs.append(len(lits))
    return Program(int(n_atoms), np.asarray(heads, dtype=np.int32),
                   np.asarray(offs, dtype=np.int64),
                   np.asarray(lits, dtype=np.int32), name)


def _rng(*seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))


def random_program(rng: np.random.Generator, n_atoms: int, n_rules: int,
                   kmin: int, kmax: int, p_neg: float = 0.5,
                   n_constraints: int = 0, cmin: int = 1, cmax: int = 3,
                   name: str = "") -> Program:
    """Uniform random normal program.

    Each headed rule has a head uniform on 1..n_atoms and a body of k~U{kmin..kmax}
    distinct atoms drawn without replacement, each negated with probability
    ``p_neg``.  Constraints (head 0) are appended after the headed rules with
    bodies of c~U{cmin..cmax} literals drawn the same way.
    """
    A = int(n_atoms)
    heads = rng.integers(1, A + 1, size=n_rules, dtype=np.int64)
    ks = np.minimum(rng.integers(kmin, kmax + 1, size=n_rules, dtype=np.int64), A)
    cks = np.minimum(rng.integers(cmin, cmax + 1, size=n_constraints, dtype=np.int64), A)
    allk = np.concatenate([ks, cks])
    n = allk.shape[0]
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(allk, out=off[1:])
    kw = int(allk.max()) if n else 0
    # distinct atoms per body: draw with replacement, redraw the later copy of
    # any repeated atom until every body is duplicate-free
    M = rng.integers(1, A + 1, size=(n, kw), dtype=np.int64)
    valid = np.arange(kw)[None, :] < allk[:, None]
    while True:
        dup = np.zeros_like(valid)
        for j in range(1, kw):
            for i in range(j):
                dup[:, j] |= (M[:, i] == M[:, j])
        dup &= valid
        if not dup.any():
            break
        M[dup] = rng.integers(1, A + 1, size=int(dup.sum()), dtype=np.int64)
    lits = M[valid]
    neg = rng.random(lits.shape[0]) < p_neg
    lits = np.where(neg, -lits, lits)
    head = np.concatenate([heads, np.zeros(n_constraints, dtype=np.int64)])
    p = Program(A, head.astype(np.int32), off, lits.astype(np.int32), name)
    p.check()
    return p


def tiny_program(seed: int, a_min: int = 4, a_max: int = 20,
                 with_constraints: bool = True) -> Program:
    """Small random program for brute-force checks: 4..20 atoms, rules/atoms
    in 1..4, bodies of 0..4 literals, 0..3 constraints of 1..3 literals."""
    rng = _rng(7, seed)
    A = int(rng.integers(a_min, a_max + 1))
    R = max(1, int(round(A * rng.uniform(1.0, 4.0))))
    C = int(rng.integers(0, 4)) if with_constraints else 0
    return random_program(rng, A, R, 0, 4, 0.5, C, 1, 3, name=f"tiny{seed}")


def single_random(seed: int) -> Program:
    """Single random instance: 200 atoms, 600 rules, bodies of 1..3 literals,
    each negated with p=0.5, no constraints."""
    rng = _rng(1, seed)
    return random_program(rng, 200, 600, 1, 3, 0.5, 0, name=f"rand200x600_s{seed}")


def batch_random(i: int, batch_seed: int = 3000, a_lo: int = 100,
                 a_hi: int = 5000) -> Program:
    """Instance i of the uneven random batch: atoms log-uniform in
    a_lo..a_hi, rules = atoms * U(2, 4), bodies of 1..4 literals, 50% negative."""
    rng = _rng(2, batch_seed, i)
    A = int(round(math.exp(rng.uniform(math.log(a_lo), math.log(a_hi)))))
    R = int(round(A * rng.uniform(2.0, 4.0)))
    return random_program(rng, A, R, 1, 4, 0.5, 0, name=f"batchrand{batch_seed}_{i}")


# ---------------------------------------------------------------- colouring
def coloring(n_vertices: int, edges, k: int = 3, name: str = "") -> Program:
    """Ground k-colouring (k=3 in the workloads).

    Atom col(v, c) = k*v + c + 1.  For each vertex and colour,
    ``col(v,c) <- not col(v,c') for every other colour c'`` (an even negative
    cycle that picks exactly one colour); for each edge {u, w} and colour c,
    the constraint ``<- col(u,c), col(w,c)``.
    """
    A = k * n_vertices
    rules = []
    for v in range(n_vertices):
        for c in range(k):
            body = [-(k * v + c2 + 1) for c2 in range(k) if c2 != c]
            rules.append((k * v + c + 1, body))
    for (u, w) in edges:
        for c in range(k):
            rules.append((0, [k * int(u) + c + 1, k * int(w) + c + 1]))
    return from_rules(A, rules, name or f"col{k}_n{n_vertices}_e{len(edges)}")


def gnp_coloring(seed: int, n: int = 2000, avg_degree: float = 4.2) -> Program:
    """3-colouring of an Erdos-Renyi graph G(n, p = avg_degree/(n-1))."""
    rng = _rng(3, seed)
    p = avg_degree / (n - 1)
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.shape[0]) < p
    edges = list(zip(iu[keep].tolist(), ju[keep].tolist()))
    return coloring(n, edges, 3, name=f"col3_gnp{n}_s{seed}")


# ---------------------------------------------------------- Hamiltonian cycle
def hamiltonian(n: int, edges, s: int = 0, name: str = "") -> Program:
    """Ground Hamiltonian-cycle program on a directed graph.

    Atoms: in(e) = e+1, out(e) = E+e+1, reach(v) = 2E+v+1.  Per edge e=(u,w):
    ``in(e) <- not out(e)``, ``out(e) <- not in(e)``, and
    ``reach(w) <- in(e)`` when u = s, else ``reach(w) <- reach(u), in(e)``.
    Constraints: at most one chosen out-edge per vertex, at most one chosen
    in-edge per vertex, and ``<- not reach(v)`` for every vertex v.
    """
    E = len(edges)
    inn = lambda e: e + 1
    out = lambda e: E + e + 1
    reach = lambda v: 2 * E + v + 1
    rules = []
    for e, (u, w) in enumerate(edges):
        rules.append((inn(e), [-out(e)]))
        rules.append((out(e), [-inn(e)]))
        if u == s:
            rules.append((reach(w), [inn(e)]))
        else:
            rules.append((reach(w), [reach(u), inn(e)]))
    outs = [[] for _ in range(n)]
    ins = [[] for _ in range(n)]
    for e, (u, w) in enumerate(edges):
        outs[u].append(e)
        ins[w].append(e)
    for lst in (outs, ins):
        for v in range(n):
            es = lst[v]
            for a in range(len(es)):
                for b in range(a + 1, len(es)):
                    rules.append((0, [inn(es[a]), inn(es[b])]))
    for v in range(n):
        rules.append((0, [-reach(v)]))
    return from_rules(2 * E + n, rules, name or f"hc_n{n}_e{E}")


def random_digraph(rng: np.random.Generator, n: int, dmin: int, dmax: int):
    """Directed graph: each vertex gets out-degree ~U{dmin..dmax} with distinct
    targets and no self-loops."""
    edges = []
    for u in range(n):
        d = int(rng.integers(dmin, dmax + 1))
        targets = rng.choice(n - 1, size=min(d, n - 1), replace=False)
        for t in targets.tolist():
            edges.append((u, t if t < u else t + 1))
    return edges


def batch_hamiltonian(i: int, batch_seed: int = 4000, n_lo: int = 60,
                      n_hi: int = 200, dmin: int = 3, dmax: int = 6) -> Program:
    """Instance i of the Hamiltonian-cycle batch: n ~ U{60..200} vertices,
    out-degree ~ U{3..6}, start vertex 0."""
    rng = _rng(4, batch_seed, i)
    n = int(rng.integers(n_lo, n_hi + 1))
    edges = random_digraph(rng, n, dmin, dmax)
    return hamiltonian(n, edges, 0, name=f"hc{batch_seed}_{i}")


# ------------------------------------------------------- decision inputs
MPNN_F, MPNN_H, MPNN_L = 8, 64, 3


def mpnn_weights(seed: int, spread: int = 127) -> dict:
    """Seeded integer weight codes for the atom-nogood scorer.

    Matrices (shapes [in, out]) are integers in [-spread, spread], biases
    integers in [-2^17, 2^17], the readout integers in [-127, 127] and its
    bias in [-2^10, 2^10].
    """
    rng = _rng(6, seed)
    F, H, L = MPNN_F, MPNN_H, MPNN_L

    def mat(*shape):
        return rng.integers(-spread, spread + 1, size=shape).astype(np.int64)

    def bias(*shape):
        return rng.integers(-(1 << 17), (1 << 17) + 1, size=shape).astype(np.int64)

    w = {"Ev": mat(F, H), "Ec": mat(F, H)}
    for k in ("P", "N", "S", "Q", "R", "T"):
        w[k] = mat(L, H, H)
    w["ev"], w["ec"] = bias(H), bias(H)
    w["bc"], w["bv"] = bias(L, H), bias(L, H)
    w["wo"] = rng.integers(-127, 128, size=H).astype(np.int64)
    w["bo"] = int(rng.integers(-1024, 1025))
    return w


def decision_scores(seed: int, n_atoms: int, lo: int = -1000, hi: int = 1000) -> np.ndarray:
    """Seeded integer per-atom decision scores (index 0 unused, kept 0)."""
    rng = _rng(7, seed)
    s = rng.integers(lo, hi + 1, size=n_atoms + 1).astype(np.int32)
    s[0] = 0
    return s


# ------------------------------------------------------------------- files
def save_program(path: str, p: Program) -> None:
    np.savez(path, n_atoms=np.int64(p.n_atoms), head=p.head,
             body_off=p.body_off, body_lits=p.body_lits)


def load_program(path: str) -> Program:
    z = np.load(path, allow_pickle=False)
    return Program(int(z["n_atoms"]), z["head"].astype(np.int32),
                   z["body_off"].astype(np.int64), z["body_lits"].astype(np.int32),
                   name=str(path))
