"""ctypes wrapper around the plain C oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it; the product path never does.  It shares
no code with the HIP library.

The oracle runs the conflict-driven solver of the paper one step at a time
(InitialPropagation, PropagateAndCheck round, Fwd-learning + Backjump,
Decision, CompleteAssignment, stability gate), so a test can stop it anywhere
and read its whole state.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

RUNNING, SAT, UNSAT, UNKNOWN = 0, 1, 2, 3
E_INVALID, E_INTERNAL = -1, -5
ST_NONE, ST_INIT, ST_ROUND, ST_LEARN, ST_DECIDE, ST_COMPLETE, ST_GATE, ST_DONE = range(8)
GATE_UNFOUNDED, GATE_ALLDEC = 0, 1
LEARN_FWD, LEARN_RES = 0, 1
DEC_OCC, DEC_SCORE, DEC_JW, DEC_ACTIVITY = 0, 1, 2, 3
STEP_NAMES = {ST_INIT: "init", ST_ROUND: "round", ST_LEARN: "learn", ST_DECIDE: "decide",
              ST_COMPLETE: "complete", ST_GATE: "gate", ST_DONE: "done"}


class Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "rounds", "visits", "literal_checks", "propagations", "decisions", "conflicts",
        "learned", "learned_len", "gate_failures", "completes", "models", "restarts")] + \
        [("trace_hash", C.c_uint64), ("deps_reads", C.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Limits(C.Structure):
    _fields_ = [("max_conflicts", C.c_int64), ("learned_cap_ng", C.c_int64),
                ("learned_cap_lits", C.c_int64)]


def _stale() -> bool:
    return not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2); safe under parallel workers."""
    import fcntl
    if not (force or _stale()):
        return LIB
    with open(os.path.join(HERE, ".build.lock"), "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        if force or _stale():
            tmp = f"{LIB}.tmp{os.getpid()}"
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared",
                                   "-fPIC", "-o", tmp, SRC])
            os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        L.or_create.restype = P
        L.or_create.argtypes = [C.c_int32, C.c_int32, i32p, i64p, i32p, C.c_int32, C.c_int32,
                                C.POINTER(C.c_int32)]
        L.or_free.argtypes = [P]
        L.or_next_step.argtypes = [P]
        L.or_next_step.restype = C.c_int32
        L.or_step.argtypes = [P, C.POINTER(Limits)]
        L.or_step.restype = C.c_int32
        L.or_run.argtypes = [P, C.POINTER(Limits), C.c_int64]
        L.or_run.restype = C.c_int32
        L.or_dims.argtypes = [P, i64p]
        L.or_nogoods.argtypes = [P, i32p, i32p]
        L.or_occ.argtypes = [P, i32p]
        L.or_state.argtypes = [P, np.ctypeslib.ndpointer(np.int8, flags="C"), i32p,
                               np.ctypeslib.ndpointer(np.uint64, flags="C"), i32p, i32p]
        L.or_get_stats.argtypes = [P, C.POINTER(Stats)]
        L.or_model.argtypes = [P, np.ctypeslib.ndpointer(np.uint8, flags="C")]
        L.or_solve.argtypes = [C.c_int32, C.c_int32, i32p, i64p, i32p, C.c_int32, C.c_int32,
                               C.POINTER(Limits), np.ctypeslib.ndpointer(np.uint8, flags="C"),
                               C.POINTER(Stats), C.c_void_p, C.c_int32, C.c_int32, C.c_int64,
                               C.c_int64, C.c_int32, C.c_int32, C.c_int32]
        L.or_set_learn_conflicts.argtypes = [P, C.c_int32]
        L.or_set_learn_conflicts.restype = C.c_int32
        L.or_set_lookahead.argtypes = [P, C.c_int32]
        L.or_set_lookahead.restype = C.c_int32
        L.or_set_decision.argtypes = [P, C.c_int32]
        L.or_set_decision.restype = C.c_int32
        L.or_atom_scores.argtypes = [P, C.c_int32, i32p]
        L.or_set_enum.argtypes = [P, C.c_int64, C.c_int64]
        L.or_set_enum.restype = C.c_int32
        L.or_models.argtypes = [P, np.ctypeslib.ndpointer(np.uint8, flags="C"), C.c_int64]
        L.or_models.restype = C.c_int64
        L.or_set_learning.argtypes = [P, C.c_int32]
        L.or_set_learning.restype = C.c_int32
        L.or_set_scores.argtypes = [P, i32p, C.c_int32]
        L.or_set_scores.restype = C.c_int32
        L.or_score_mode.argtypes = [P, C.POINTER(C.c_int32)]
        L.or_score_mode.restype = C.c_int32
        L.or_solve.restype = C.c_int32
        _lib = L
    return _lib


def make_limits(max_conflicts=-1, learned_cap_ng=-1, learned_cap_lits=-1) -> Limits:
    return Limits(int(max_conflicts), int(learned_cap_ng), int(learned_cap_lits))


@dataclass
class State:
    V: int
    A: int
    Rh: int
    W: int
    cdl: int
    val: np.ndarray        # int8[V+1]
    lvl: np.ndarray        # int32[V+1]
    deps: np.ndarray       # uint64[V+1, W]
    dec: np.ndarray        # int32[cdl+1], dec[l] = decision literal of level l >= 2
    frontier: np.ndarray   # int32, ascending
    ng_off: np.ndarray     # int32, all nogoods (static + learned)
    ng_lits: np.ndarray
    n_static: int
    pend_kind: int         # 0 none, 1 round conflict, 2 gate conflict
    pend_id: int
    status: int
    last_step: int


class Solver:
    """One program in the oracle, steppable."""

    def __init__(self, prog, W: int = 1, gate: int = GATE_UNFOUNDED, learning: int = LEARN_FWD,
                 max_models: int = 1, restart_every: int = 0, decision: int = DEC_OCC,
                 learn_conflicts: int = 1, lookahead: int = 0):
        L = lib()
        err = C.c_int32(0)
        self._h = L.or_create(int(prog.n_atoms), int(prog.n_rules),
                              np.ascontiguousarray(prog.head, np.int32),
                              np.ascontiguousarray(prog.body_off, np.int64),
                              np.ascontiguousarray(prog.body_lits, np.int32),
                              int(W), int(gate), C.byref(err))
        if not self._h:
            raise ValueError(f"oracle rejected the program (status {err.value})")
        self.W = W
        if L.or_set_learning(self._h, int(learning)) != 0:
            raise ValueError("unknown learning mode")
        if L.or_set_enum(self._h, int(max_models), int(restart_every)) != 0:
            raise ValueError("max_models and restart_every must be >= 0")
        if L.or_set_decision(self._h, int(decision)) != 0:
            raise ValueError("decision must be DEC_OCC, DEC_JW or DEC_ACTIVITY")
        if L.or_set_learn_conflicts(self._h, int(learn_conflicts)) != 0:
            raise ValueError("learn_conflicts must be in 1..8")
        if L.or_set_lookahead(self._h, int(lookahead)) != 0:
            raise ValueError("lookahead must be in 0..8, with Fwd-learning")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_free(self._h)
            self._h = None

    def set_scores(self, score, fallback_after: int = 10) -> None:
        """Drive Decision by per-atom integer scores (``score[p]`` for atom p,
        index 0 unused) until ``fallback_after`` consecutive conflicts."""
        sc = np.ascontiguousarray(score, np.int32)
        if sc.shape != (int(self.dims()[1]) + 1,):
            raise ValueError("score must have n_atoms + 1 entries")
        if lib().or_set_scores(self._h, sc, int(fallback_after)) != 0:
            raise ValueError("scores must be set before the first step")

    def score_mode(self):
        """(1 while the scores drive Decision else 0, current conflict run)."""
        c = C.c_int32(0)
        m = lib().or_score_mode(self._h, C.byref(c))
        return int(m), int(c.value)

    def dims(self):
        d = np.zeros(16, np.int64)
        lib().or_dims(self._h, d)
        return d

    def next_step(self) -> int:
        return lib().or_next_step(self._h)

    def step(self, limits: Limits | None = None) -> int:
        return lib().or_step(self._h, C.byref(limits) if limits else None)

    def run(self, limits: Limits | None = None, max_steps: int = -1) -> int:
        return lib().or_run(self._h, C.byref(limits) if limits else None, int(max_steps))

    def stats(self) -> dict:
        s = Stats()
        lib().or_get_stats(self._h, C.byref(s))
        return s.as_dict()

    def model(self) -> np.ndarray:
        A = int(self.dims()[1])
        m = np.zeros(max(A, 1), np.uint8)
        lib().or_model(self._h, m)
        return m[:A]

    def models(self) -> list:
        """The answer sets found so far, in the order found."""
        A = int(self.dims()[1])
        n = int(self.stats()["models"])
        buf = np.zeros(max(n * A, 1), np.uint8)
        lib().or_models(self._h, buf, n)
        return [buf[k * A:(k + 1) * A].copy() for k in range(n)]

    def exhausted(self) -> bool:
        """True once the search has shown that no further answer set exists."""
        return bool(self.dims()[15])

    def nogoods(self):
        d = self.dims()
        n = int(d[3] + d[8])
        nl = int(d[4] + d[9])
        off = np.zeros(n + 1, np.int32)
        lits = np.zeros(max(nl, 1), np.int32)
        lib().or_nogoods(self._h, off, lits)
        return off, lits[:nl]

    def atom_scores(self, kind: int) -> np.ndarray:
        """Per-atom scores (index 0 unused): 0 occurrences, 1 Jeroslow-Wang
        (fixed point), 2 the current activity."""
        A = int(self.dims()[1])
        o = np.zeros(A + 1, np.int32)
        lib().or_atom_scores(self._h, int(kind), o)
        return o

    def occ(self) -> np.ndarray:
        A = int(self.dims()[1])
        o = np.zeros(A + 1, np.int32)
        lib().or_occ(self._h, o)
        return o

    def state(self) -> State:
        d = self.dims()
        V, A, Rh, n0, W, cdl, nf = (int(d[0]), int(d[1]), int(d[2]), int(d[3]), int(d[5]),
                                    int(d[6]), int(d[7]))
        val = np.zeros(V + 1, np.int8)
        lvl = np.zeros(V + 1, np.int32)
        deps = np.zeros((V + 1) * W, np.uint64)
        dec = np.zeros(cdl + 1, np.int32)
        fr = np.zeros(max(nf, 1), np.int32)
        lib().or_state(self._h, val, lvl, deps, dec, fr)
        off, lits = self.nogoods()
        return State(V, A, Rh, W, cdl, val, lvl, deps.reshape(V + 1, W), dec, fr[:nf],
                     off, lits, n0, int(d[10]), int(d[11]), int(d[12]), int(d[13]))


def solve(prog, W: int = 1, gate: int = GATE_UNFOUNDED, limits: Limits | None = None,
          scores=None, fallback_after: int = 10, learning: int = LEARN_FWD,
          max_models: int = 1, restart_every: int = 0, decision: int = DEC_OCC,
          learn_conflicts: int = 1, lookahead: int = 0):
    """Encode and solve in one call; returns (status, model or None, stats).
    ``scores`` (int32[n_atoms + 1]) selects the score-driven Decision; the
    model is the first answer set found."""
    L = lib()
    A = int(prog.n_atoms)
    m = np.zeros(max(A, 1), np.uint8)
    st = Stats()
    sc = None
    if scores is not None:
        sc = np.ascontiguousarray(scores, np.int32)
        if sc.shape != (A + 1,):
            raise ValueError("scores must have n_atoms + 1 entries")
    rc = L.or_solve(A, int(prog.n_rules), np.ascontiguousarray(prog.head, np.int32),
                    np.ascontiguousarray(prog.body_off, np.int64),
                    np.ascontiguousarray(prog.body_lits, np.int32), int(W), int(gate),
                    C.byref(limits) if limits else None, m, C.byref(st),
                    sc.ctypes.data if sc is not None else None, int(fallback_after),
                    int(learning), int(max_models), int(restart_every), int(decision),
                    int(learn_conflicts), int(lookahead))
    return rc, (m[:A].copy() if rc == SAT else None), st.as_dict()


def enumerate_models(prog, max_models: int = 0, restart_every: int = 0, W: int = 1,
                     gate: int = GATE_UNFOUNDED, learning: int = LEARN_FWD,
                     limits: Limits | None = None, decision: int = DEC_OCC,
                     learn_conflicts: int = 1, lookahead: int = 0):
    """Run the search for up to ``max_models`` answer sets (0: all); returns
    (status, list of answer sets in the order found, stats, exhausted)."""
    s = Solver(prog, W=W, gate=gate, learning=learning, max_models=max_models,
               restart_every=restart_every, decision=decision,
               learn_conflicts=learn_conflicts, lookahead=lookahead)
    rc = s.run(limits)
    return rc, s.models(), s.stats(), s.exhausted()
