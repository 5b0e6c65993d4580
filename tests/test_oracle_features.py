"""Pins of the learned Decision scorer's input features (oracle/mpnn.py).

The features are the scorer's only view of a program, so they are checked
here against their written definition on hand-built graphs whose degrees
are chosen around every bit-length boundary (0, 1, 2, 3, 15, 16, 63, 64,
65) and past the saturation of the code (16 times the bit length, capped
at 255), with each expected row computed in the test from Python's exact
``int.bit_length`` and ``fractions.Fraction``, never from the oracle.

Definition (codes, 32 standing for 1):
  x_v = [32, 32 if v is an atom, 32 if v is some b_r / t_r / n_r (three
         columns), L(#positive occurrences of v), L(#negative occurrences),
         L(#occurrences of either sign)],  L(d) = min(255, 16 * bitlen(d));
  y_c = [32, r(32, |c|), 32 if |c| = 1 / 2 / 3 / >= 4 (four columns),
         r(32 * #positive literals of c, |c|), 0],  r(a, b) = a / b rounded
         half up, 0 when b = 0.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

import aspgen
from oracle import mpnn


def _L(d: int) -> int:
    return min(255, 16 * int(d).bit_length())


def _r(a: int, b: int) -> int:
    return 0 if b == 0 else math.floor(Fraction(a, b) + Fraction(1, 2))


def _expected_x(V, A, dpos, dneg):
    rows = [[0] * 8]
    for v in range(1, V + 1):
        kind = (v - A - 1) % 3 if v > A else -1
        rows.append([32, 32 if v <= A else 0, 32 if kind == 0 else 0, 32 if kind == 1 else 0,
                     32 if kind == 2 else 0, _L(dpos[v]), _L(dneg[v]), _L(dpos[v] + dneg[v])])
    return np.array(rows, np.int64)


def _expected_y(nogoods):
    rows = []
    for c in nogoods:
        n, npos = len(c), sum(1 for l in c if l > 0)
        rows.append([32, _r(32, n), 32 * (n == 1), 32 * (n == 2), 32 * (n == 3), 32 * (n >= 4),
                     _r(32 * npos, n), 0])
    return np.array(rows, np.int64)


def _graph_from_degrees(A, degs, extra=()):
    """A graph over V = len(degs) variables where variable v has exactly
    degs[v-1] = (positive, negative) occurrences.  The occurrences are dealt
    round-robin into nogoods of lengths 1..5 (cycling) so that no nogood
    holds a variable twice; `extra` nogoods are appended as given."""
    V = len(degs)
    pending = {v: [v] * p + [-v] * n for v, (p, n) in enumerate(degs, start=1)}
    nogoods, want = [], 1
    while any(pending.values()):
        c = []
        for v in range(1, V + 1):
            if pending[v] and len(c) < want:
                c.append(pending[v].pop())
        nogoods.append(c)
        want = want % 5 + 1
    nogoods.extend(list(c) for c in extra)
    off = np.zeros(len(nogoods) + 1, np.int64)
    off[1:] = np.cumsum([len(c) for c in nogoods])
    lits = np.array([l for c in nogoods for l in c], np.int64)
    return mpnn.Graph(V, A, off, lits), nogoods


BOUNDARY_DEGREES = [(0, 1), (1, 0), (2, 3), (3, 2), (15, 16), (16, 15), (63, 64), (64, 63),
                    (65, 65), (0, 0), (1, 1), (16, 48), (3, 0), (0, 3)]


@pytest.mark.parametrize("A", [0, 5, 14])
def test_variable_features_at_bit_length_boundaries(A):
    g, _ = _graph_from_degrees(A, BOUNDARY_DEGREES)
    x, _, deg = mpnn.features(g)
    dpos = [0] + [p for p, _ in BOUNDARY_DEGREES]
    dneg = [0] + [n for _, n in BOUNDARY_DEGREES]
    assert np.array_equal(x, _expected_x(g.V, A, dpos, dneg))
    assert np.array_equal(deg[1:], np.array(dpos[1:]) + np.array(dneg[1:]))
    # column 7 is the total degree: variables whose negative occurrences
    # change the bit length of the sum differ from a positive-only reading
    assert any(x[v, 7] != _L(dpos[v]) for v in range(1, g.V + 1))


def test_degree_code_saturates():
    """16 * bitlen reaches 256 at 32768 occurrences and is capped at 255;
    32767 occurrences still code to 240."""
    degs = [(32768, 0), (0, 32767), (20000, 20000), (1, 0)]
    g, _ = _graph_from_degrees(2, degs)
    x, _, _ = mpnn.features(g)
    assert x[1].tolist()[5:] == [255, 0, 255]
    assert x[2].tolist()[5:] == [0, 240, 240]
    assert x[3].tolist()[5:] == [240, 240, 255]
    assert x[4].tolist()[5:] == [16, 0, 16]
    assert np.array_equal(x, _expected_x(4, 2, [0] + [p for p, _ in degs], [0] + [n for _, n in degs]))


def test_nogood_features_lengths_and_signs():
    """Every length class (0 -- the empty nogood of an empty-body constraint
    -- then 1..7) and positive shares that round up at one half."""
    extra = [[], [1], [-1], [1, -2], [1, 2], [-1, -2], [1, -2, 3], [1, 2, -3], [1, 2, 3, -4],
             [-1, -2, -3, 4, 5], [1, -2, 3, -4, 5, -6], [1, 2, 3, 4, 5, 6, -7]]
    g, ngs = _graph_from_degrees(3, [(0, 0)] * 7, extra=extra)
    _, y, _ = mpnn.features(g)
    assert np.array_equal(y, _expected_y(ngs))
    # spot values written out by hand: r(32, 3) = 11, r(64, 3) = 21,
    # r(32, 6) = 5, r(96, 6) = 16, r(192, 7) = 27
    byc = {tuple(c): row for c, row in zip(ngs, y.tolist())}
    assert byc[(1, -2, 3)][1] == 11 and byc[(1, -2, 3)][6] == 21
    assert byc[(1, -2, 3, -4, 5, -6)][1] == 5 and byc[(1, -2, 3, -4, 5, -6)][6] == 16
    assert byc[(1, 2, 3, 4, 5, 6, -7)][6] == 27
    assert byc[()] == [32, 0, 0, 0, 0, 0, 0, 0]


@pytest.mark.parametrize("seed", range(4))
def test_features_of_encoded_programs(seed):
    """On real completions: degrees counted directly from the nogood list
    (Python sets per nogood, so a literal is counted once per nogood)."""
    prog = aspgen.tiny_program(seed, 6, 14) if seed < 2 else aspgen.single_random(1000 + seed)
    g = mpnn.graph_of(prog)
    ngs = [[int(l) for l in g.lits[g.off[c]:g.off[c + 1]]] for c in range(g.n)]
    dpos = [0] * (g.V + 1)
    dneg = [0] * (g.V + 1)
    for c in ngs:
        for l in set(c):
            (dpos if l > 0 else dneg)[abs(l)] += 1
    x, y, _ = mpnn.features(g)
    assert np.array_equal(x, _expected_x(g.V, g.A, dpos, dneg))
    assert np.array_equal(y, _expected_y(ngs))
