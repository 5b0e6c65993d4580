"""Re-derivations used to pin the oracle's steps (test helpers only).

They restate the paper's definitions in the most direct form, without the
frontier-driven shortcuts the solvers use:

* ``full_scan`` classifies *every* nogood against an assignment (Sect. 2:
  violated iff delta is a subset of A; unit iff exactly one literal is open
  and every other literal is in A), instead of only those reached from the
  previous round's assignments;
* ``completion_extension`` extends an interpretation M with the auxiliary
  atoms of the completion (b_r <-> t_r and n_r, t_r <-> body+ true,
  n_r <-> body- false);
* ``decision_choice`` scans every headed rule for applicability.
"""
from __future__ import annotations

import numpy as np


def lit_var(l):
    return abs(int(l))


def lit_val(l):
    return 1 if l > 0 else -1


def nogoods_list(off, lits):
    return [lits[off[i]:off[i + 1]].tolist() for i in range(len(off) - 1)]


def full_scan(ngs, val):
    """Return (violated ids, unit dict id -> open literal)."""
    viol, unit = [], {}
    for i, ng in enumerate(ngs):
        inA, openl, sat = 0, [], False
        for l in ng:
            v = val[lit_var(l)]
            if v == 0:
                openl.append(l)
            elif v == lit_val(l):
                inA += 1
            else:
                sat = True
        if sat:
            continue
        if inA == len(ng):
            viol.append(i)
        elif len(openl) == 1 and inA == len(ng) - 1:
            unit[i] = openl[0]
    return viol, unit


def expected_round(ngs, val, deps, cdl):
    """The round's outcome from a full scan: implied vars with their winner
    (lowest id), values, Deps, and the selected conflict (shortest, lowest id)
    among violated and clash-losing unit nogoods."""
    viol, unit = full_scan(ngs, val)
    winner = {}
    for i in sorted(unit):
        x = lit_var(unit[i])
        if x not in winner:
            winner[x] = i
    conf = list(viol)
    for i, u in unit.items():
        x = lit_var(u)
        if lit_val(unit[winner[x]]) != lit_val(u):
            conf.append(i)
    sel = min(conf, key=lambda i: (len(ngs[i]), i)) if conf else -1
    newval, newdeps = {}, {}
    for x, w in winner.items():
        newval[x] = -lit_val(unit[w])
        d = np.zeros(deps.shape[1], np.uint64)
        for l in ngs[w]:
            y = lit_var(l)
            if y != x:
                d |= deps[y]
        newdeps[x] = d
    return newval, newdeps, sel


def completion_extension(prog, mask, n_vars):
    """Total assignment (val[1..V] in {-1,+1}) of interpretation `mask` with
    the auxiliary atoms set by their definitions."""
    A = prog.n_atoms
    val = np.zeros(n_vars + 1, np.int8)
    for p in range(1, A + 1):
        val[p] = 1 if (mask >> (p - 1)) & 1 else -1
    j = 0
    for h, body in prog.rules():
        if h == 0:
            continue
        pos = [b for b in body if b > 0]
        neg = [-b for b in body if b < 0]
        t = all(val[p] == 1 for p in pos)
        n = all(val[q] == -1 for q in neg)
        b = A + 3 * j + 1
        val[b] = 1 if (t and n) else -1
        val[b + 1] = 1 if t else -1
        val[b + 2] = 1 if n else -1
        j += 1
    return val


def satisfies(ngs, val):
    for ng in ngs:
        if all(val[lit_var(l)] == lit_val(l) for l in ng):
            return False
    return True


def occurrences(ngs, A):
    occ = np.zeros(A + 1, np.int64)
    for ng in ngs:
        for p in {lit_var(l) for l in ng}:
            if p <= A:
                occ[p] += 1
    return occ


def decision_choice(prog, val, occ):
    """Applicable rules (head unassigned, T t_r in A, F n_r not in A) and the
    one with the highest head occurrence count, lowest rule on ties."""
    A = prog.n_atoms
    best, key = -1, None
    j = 0
    for h, _ in prog.rules():
        if h == 0:
            continue
        t, n = A + 3 * j + 2, A + 3 * j + 3
        if val[h] == 0 and val[t] == 1 and val[n] != -1:
            k = (int(occ[h]), -j)
            if key is None or k > key:
                best, key = j, k
        j += 1
    return best


def levels_of(bits_row, cdl, W):
    """Decision levels whose Deps bit is set (bit l-1 for level l, the last
    bit standing for every level >= 64W)."""
    top = 64 * W - 1
    out = []
    for l in range(2, cdl + 1):
        b = min(l - 1, top)
        if (int(bits_row[b // 64]) >> (b % 64)) & 1:
            out.append(l)
    return out
