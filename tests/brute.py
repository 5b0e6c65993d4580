"""Brute-force answer sets, independent of both solvers.

Straight from the definitions of the paper's Preliminaries:

* the Gelfond-Lifschitz reduct Pi^M drops every rule whose body- meets M and
  deletes the ``not`` literals of the others (the paper names the reduct
  without defining it; this is the standard one);
* M is an answer set iff M satisfies every constraint and M is the least
  model of Pi^M, computed with the immediate-consequence operator T_Pi
  (whose second condition is read as body-(r) disjoint from I);
* the completion Pi_cc: p <-> OR over rules(p) of (body+ true and body- false).

``stable_models`` enumerates all 2^|atoms| interpretations with numpy bit
masks (|atoms| <= 20); ``is_stable`` checks one interpretation of any size.
"""
from __future__ import annotations

import numpy as np


def _split(prog):
    rules = []
    for h, body in prog.rules():
        pos = sorted({b for b in body if b > 0})
        neg = sorted({-b for b in body if b < 0})
        rules.append((h, pos, neg))
    return rules


def is_stable(prog, model) -> bool:
    """model: 0/1 array over atoms 1..A (index p-1)."""
    A = prog.n_atoms
    M = np.zeros(A + 1, bool)
    M[1:] = np.asarray(model, bool)[:A]
    rules = _split(prog)
    for h, pos, neg in rules:
        if h == 0 and all(M[p] for p in pos) and not any(M[q] for q in neg):
            return False
    # least model of the reduct by counting unsatisfied positive body atoms
    red = [(h, pos) for h, pos, neg in rules if h != 0 and not any(M[q] for q in neg)]
    cnt = [len(pos) for _, pos in red]
    watch = [[] for _ in range(A + 1)]
    for i, (h, pos) in enumerate(red):
        for p in pos:
            watch[p].append(i)
    LM = np.zeros(A + 1, bool)
    queue = []
    for i, (h, pos) in enumerate(red):
        if cnt[i] == 0 and not LM[h]:
            LM[h] = True
            queue.append(h)
    while queue:
        p = queue.pop()
        for i in watch[p]:
            cnt[i] -= 1
            if cnt[i] == 0:
                h = red[i][0]
                if not LM[h]:
                    LM[h] = True
                    queue.append(h)
    return bool(np.array_equal(LM[1:], M[1:]))


def _all_masks(A):
    return np.arange(1 << A, dtype=np.int64)


def _bit(p):
    return np.int64(1) << np.int64(p - 1)


def stable_models(prog):
    """All answer sets as a sorted list of int bit masks (bit p-1 = atom p)."""
    A = prog.n_atoms
    assert A <= 22, "brute force is for tiny programs"
    M = _all_masks(A)
    ok = np.ones(M.shape[0], bool)
    rules = _split(prog)
    for h, pos, neg in rules:
        if h != 0:
            continue
        pm = sum(int(_bit(p)) for p in pos)
        nm = sum(int(_bit(q)) for q in neg)
        viol = ((M & pm) == pm) & ((M & nm) == 0)
        ok &= ~viol
    headed = [(h, sum(int(_bit(p)) for p in pos), sum(int(_bit(q)) for q in neg))
              for h, pos, neg in rules if h != 0]
    LM = np.zeros_like(M)
    while True:
        new = LM.copy()
        for h, pm, nm in headed:
            fire = ((M & nm) == 0) & ((LM & pm) == pm)
            new |= np.where(fire, _bit(h), np.int64(0))
        if np.array_equal(new, LM):
            break
        LM = new
    ok &= LM == M
    return sorted(int(x) for x in M[ok])


def completion_models(prog):
    """Bit masks of all models of the completion Pi_cc that satisfy every
    constraint (supported models)."""
    A = prog.n_atoms
    assert A <= 22
    M = _all_masks(A)
    ok = np.ones(M.shape[0], bool)
    rules = _split(prog)
    support = {p: np.zeros(M.shape[0], bool) for p in range(1, A + 1)}
    for h, pos, neg in rules:
        pm = sum(int(_bit(p)) for p in pos)
        nm = sum(int(_bit(q)) for q in neg)
        body = ((M & pm) == pm) & ((M & nm) == 0)
        if h == 0:
            ok &= ~body
        else:
            support[h] |= body
    for p in range(1, A + 1):
        ok &= ((M & _bit(p)) != 0) == support[p]
    return sorted(int(x) for x in M[ok])


def mask_to_model(mask: int, A: int) -> np.ndarray:
    return np.array([(mask >> (p - 1)) & 1 for p in range(1, A + 1)], np.uint8)


def model_to_mask(model) -> int:
    return int(sum(int(b) << i for i, b in enumerate(np.asarray(model).tolist())))
