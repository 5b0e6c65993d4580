"""Host-side checks of libasp that need no GPU: the C ABI loads and exports
every declared symbol, the host encoder reproduces the oracle's nogoods,
input validation, and sizes."""
import ctypes
import os
import re

import numpy as np
import pytest

import aspgen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_1909_01786_amd as P
    P.lib()
    return P


def test_exports_every_declared_symbol(P):
    hdr = open(os.path.join(ROOT, "include", "asp.h")).read()
    declared = set(re.findall(r"^\s*(?:const\s+char\s*\*\s*|int32_t\s+)(asp_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 18
    so = ctypes.CDLL(os.path.join(ROOT, "paper_1909_01786_amd", "libasp.so"))
    for name in sorted(declared):
        assert hasattr(so, name), name
    from paper_1909_01786_amd.binding import EXPORTS
    assert declared == set(EXPORTS)


@pytest.mark.parametrize("family", ["tiny", "c0", "col", "hc", "batch"])
def test_encoder_matches_oracle(P, family):
    progs = {
        "tiny": [aspgen.tiny_program(s, 4, 20) for s in range(200)],
        "c0": [aspgen.single_random(1000 + s) for s in range(5)],
        "col": [aspgen.gnp_coloring(2000)],
        "hc": [aspgen.batch_hamiltonian(s) for s in range(5)],
        "batch": [aspgen.batch_random(s) for s in range(5)],
    }[family]
    for p in progs:
        g = P.Program(p)
        o = oracle.Solver(p)
        off, lits = g.nogoods()
        o_off, o_lits = o.nogoods()
        assert np.array_equal(off, o_off) and np.array_equal(lits, o_lits), p.name
        d = o.dims()
        assert g.sizes.n_vars == d[0] and g.sizes.n_rules_headed == d[2]
        assert g.sizes.n_nogoods == d[3] and g.sizes.n_lits == d[4]
        assert g.sizes.n_constraints == d[14]
        lens = np.diff(off)
        assert g.sizes.n_units == int((lens == 1).sum())


def test_invalid_inputs(P):
    from paper_1909_01786_amd.binding import AspError
    bad = [
        aspgen.from_rules(2, [(3, [1])]),
        aspgen.from_rules(2, [(1, [3])]),
        aspgen.from_rules(2, [(-1, [1])]),
    ]
    for p in bad:
        with pytest.raises(AspError) as e:
            P.Program(p)
        assert e.value.status == -1
    p = aspgen.from_rules(2, [(1, [2])])
    p.body_off = np.array([0, 2], np.int64)   # offsets beyond the literals' count
    p.body_lits = np.array([2, 5], np.int32)
    with pytest.raises(AspError):
        P.Program(p)
    with pytest.raises(AspError):
        P.Program(aspgen.from_rules(2, [(1, [2])]), W=0)
    with pytest.raises(AspError):
        P.Program(aspgen.from_rules(2, [(1, [2])]), W=65)


def test_host_side_argument_checks(P):
    """Refusals that happen before any device call: the allocation-free
    solve's size limit and score mode, training arguments, options."""
    from paper_1909_01786_amd.binding import AspError, NOALLOC_MAX_BYTES, SCORER_NPARAM
    import paper_1909_01786_amd.binding as B
    g = P.Program(aspgen.single_random(1001))        # default learned-store capacities
    assert g.sizes.device_bytes > NOALLOC_MAX_BYTES
    with pytest.raises(AspError) as e:
        g.solve_noalloc(P.limits(10, 1000))
    assert e.value.status == -2
    with pytest.raises(AspError) as e:
        P.Program(aspgen.tiny_program(1), decision=P.DECISION_SCORE).solve_noalloc()
    assert e.value.status == -1
    for kw in (dict(lookahead=9), dict(lookahead=2, learning=P.LEARN_RES)):
        with pytest.raises(AspError):
            P.Program(aspgen.tiny_program(1), **kw)
    bad = np.zeros(SCORER_NPARAM, np.float32)
    bad[5] = np.nan
    with pytest.raises(AspError):
        B.quantize(bad)
    with pytest.raises(ValueError):
        B.quantize(np.zeros(10, np.float32))


def test_status_strings(P):
    from paper_1909_01786_amd.binding import asp_status_str
    assert asp_status_str(1) == "sat" and asp_status_str(-2) == "capacity exceeded"


def test_no_cpu_fallback():
    """The package loads only the HIP library and never imports the oracle."""
    import paper_1909_01786_amd.binding as b
    src = open(b.__file__).read()
    assert "oracle" not in src.replace("the CPU oracle", "")
    for f in os.listdir(os.path.join(ROOT, "paper_1909_01786_amd")):
        if f.endswith(".py"):
            txt = open(os.path.join(ROOT, "paper_1909_01786_amd", f)).read()
            assert "import oracle" not in txt and "from oracle" not in txt, f
