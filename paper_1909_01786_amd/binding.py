"""Python binding of libasp (``include/asp.h``): argument marshalling only.

Every step of the search runs in the HIP library; torch supplies device
memory (the arena tensors) and streams.  There is no fallback: if
``libasp.so`` is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libasp.so")

OK, SAT, UNSAT, UNKNOWN, FIXPOINT, CONFLICT, RUNNING = 0, 1, 2, 3, 4, 5, 6
E_INVALID, E_CAPACITY, E_DEVICE, E_STATE, E_INTERNAL, E_TIMEOUT = -1, -2, -3, -4, -5, -6
STEP_NONE, STEP_INIT, STEP_ROUND, STEP_LEARN, STEP_DECIDE, STEP_COMPLETE, STEP_GATE, STEP_DONE = range(8)
GATE_UNFOUNDED, GATE_ALLDEC = 0, 1
DECISION_OCC, DECISION_SCORE, DECISION_JW, DECISION_ACTIVITY = 0, 1, 2, 3
LEARN_FWD, LEARN_RES = 0, 1
SCORER_F, SCORER_H, SCORER_L = 8, 64, 3
SCORER_NPARAM = 75329          # ASP_SCORER_NPARAM: float parameters of the trainable scorer
NOALLOC_MAX_BYTES = 64 << 20   # ASP_NOALLOC_MAX_BYTES


class AspError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{asp_status_str(status)} ({status}): {msg}")
        self.status = status


class asp_options(C.Structure):
    _fields_ = [("W", C.c_int32), ("gate", C.c_int32), ("learned_cap_ng", C.c_int64),
                ("learned_cap_lits", C.c_int64), ("decision", C.c_int32),
                ("fallback_after", C.c_int32), ("learning", C.c_int32),
                ("learn_conflicts", C.c_int32),
                ("max_models", C.c_int64), ("restart_every", C.c_int64),
                ("lookahead", C.c_int32), ("reserved", C.c_int32)]


class asp_limits(C.Structure):
    _fields_ = [("max_conflicts", C.c_int64), ("max_ms", C.c_int64)]


class asp_schedule(C.Structure):
    _fields_ = [("threads", C.c_int32), ("classes", C.c_int32),
                ("class_threads", C.c_int32 * 4)]


_STAT_NAMES = ("rounds", "visits", "literal_checks", "propagations", "decisions", "conflicts",
               "learned", "learned_len", "gate_failures", "completes")


class asp_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in _STAT_NAMES] + [
        ("trace_hash", C.c_uint64), ("status", C.c_int32), ("last_step", C.c_int32)] + [
        (n, C.c_int64) for n in ("ns_total", "ns_round", "ns_learn", "ns_decide", "ns_gate")] + [
        ("models", C.c_int64), ("restarts", C.c_int64), ("exhausted", C.c_int32),
        ("reserved", C.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class asp_sizes(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("n_rules_headed", C.c_int32),
                ("n_constraints", C.c_int32), ("n_vars", C.c_int32), ("n_nogoods", C.c_int64),
                ("n_lits", C.c_int64), ("n_units", C.c_int64), ("device_bytes", C.c_uint64)]


class asp_prop_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("conflict_id", C.c_int32), ("rounds", C.c_int64),
                ("implied", C.c_int64), ("visits", C.c_int64), ("literal_checks", C.c_int64)]


class asp_state(C.Structure):
    _fields_ = [("n_vars", C.c_int32), ("W", C.c_int32), ("cdl", C.c_int32),
                ("frontier_len", C.c_int32), ("n_learned", C.c_int32), ("pending", C.c_int32),
                ("learned_lits", C.c_int64), ("initialised", C.c_int32), ("status", C.c_int32),
                ("score_mode", C.c_int32), ("consec", C.c_int32), ("dec_open", C.c_int32),
                ("reserved", C.c_int32), ("val", C.c_void_p), ("lvl", C.c_void_p), ("deps", C.c_void_p),
                ("dec", C.c_void_p), ("frontier", C.c_void_p), ("learned_off", C.c_void_p),
                ("learned", C.c_void_p), ("stats", asp_stats)]


_HH = SCORER_L * SCORER_H * SCORER_H
_FH = SCORER_F * SCORER_H
_LH = SCORER_L * SCORER_H


class asp_scorer_weights(C.Structure):
    _fields_ = [("Ev", C.c_uint16 * _FH), ("Ec", C.c_uint16 * _FH)] + \
        [(k, C.c_uint16 * _HH) for k in ("P", "N", "S", "Q", "R", "T")] + \
        [("ev", C.c_int32 * SCORER_H), ("ec", C.c_int32 * SCORER_H), ("bc", C.c_int32 * _LH),
         ("bv", C.c_int32 * _LH), ("wo", C.c_int32 * SCORER_H), ("bo", C.c_int32),
         ("reserved", C.c_int32 * 63)]


def _bf16_bits(codes) -> np.ndarray:
    """Integer codes (|k| <= 127, exact in bfloat16) as bfloat16 bit patterns."""
    f = np.ascontiguousarray(np.asarray(codes, np.float32).reshape(-1))
    return (f.view(np.uint32) >> 16).astype(np.uint16)


WEIGHTS_PATH = os.path.join(HERE, "weights", "scorer.npz")


def load_weights(path: str = WEIGHTS_PATH) -> dict:
    """Integer weight codes of the scorer, as written by train_scorer.py."""
    z = np.load(path, allow_pickle=False)
    keys = ("Ev", "Ec", "P", "N", "S", "Q", "R", "T", "ev", "ec", "bc", "bv", "wo")
    w = {k: z[k].astype(np.int64) for k in keys}
    w["bo"] = int(z["bo"])
    return w


def scorer_weights(w: dict) -> asp_scorer_weights:
    """Pack a dict of integer weight codes ([in, out] matrices; see asp.h)."""
    out = asp_scorer_weights()
    for k in ("Ev", "Ec", "P", "N", "S", "Q", "R", "T"):
        bits = _bf16_bits(w[k])
        C.memmove(getattr(out, k), bits.ctypes.data, bits.nbytes)
    for k in ("ev", "ec", "bc", "bv", "wo"):
        v = np.ascontiguousarray(np.asarray(w[k], np.int64).reshape(-1).astype(np.int32))
        C.memmove(getattr(out, k), v.ctypes.data, v.nbytes)
    out.bo = int(w["bo"])
    return out


def weights_dict(w: asp_scorer_weights) -> dict:
    """Unpack asp_scorer_weights into integer codes ([in, out] matrices)."""
    def codes(name, shape):
        bits = np.ctypeslib.as_array(getattr(w, name)).astype(np.uint32) << 16
        return bits.view(np.float32).astype(np.int64).reshape(shape)
    out = {"Ev": codes("Ev", (SCORER_F, SCORER_H)), "Ec": codes("Ec", (SCORER_F, SCORER_H))}
    for k in ("P", "N", "S", "Q", "R", "T"):
        out[k] = codes(k, (SCORER_L, SCORER_H, SCORER_H))
    out["ev"] = np.ctypeslib.as_array(w.ev).astype(np.int64).copy()
    out["ec"] = np.ctypeslib.as_array(w.ec).astype(np.int64).copy()
    out["bc"] = np.ctypeslib.as_array(w.bc).astype(np.int64).reshape(SCORER_L, SCORER_H).copy()
    out["bv"] = np.ctypeslib.as_array(w.bv).astype(np.int64).reshape(SCORER_L, SCORER_H).copy()
    out["wo"] = np.ctypeslib.as_array(w.wo).astype(np.int64).copy()
    out["bo"] = int(w.bo)
    return out


def quantize(params) -> dict:
    """Float scorer parameters -> integer weight codes (asp_scorer_quantize)."""
    p = np.ascontiguousarray(params, np.float32)
    if p.shape != (SCORER_NPARAM,):
        raise ValueError(f"expected {SCORER_NPARAM} parameters")
    w = asp_scorer_weights()
    _check(lib().asp_scorer_quantize(_ptr(p), C.byref(w)))
    return weights_dict(w)


def dequantize(w: dict) -> np.ndarray:
    """Integer weight codes -> float scorer parameters (asp_scorer_dequantize)."""
    packed = w if isinstance(w, asp_scorer_weights) else scorer_weights(w)
    p = np.zeros(SCORER_NPARAM, np.float32)
    _check(lib().asp_scorer_dequantize(C.byref(packed), _ptr(p)))
    return p


def train_scorer(programs, labels, params, steps: int, lr: float = 1e-3, device="cuda",
                 stream=None, ws=None):
    """Train the scorer on the device (asp_scorer_train).  labels: one float
    array per program over its atoms 1..A (< 0: no label).  steps = 0: one
    gradient pass.  Returns (params, losses, grad)."""
    progs = list(programs)
    arr = (C.c_void_p * len(progs))(*[p._h.value for p in progs])
    lab = np.ascontiguousarray(np.concatenate([np.asarray(l, np.float32).reshape(-1)
                                               for l in labels]), np.float32)
    if lab.shape[0] != sum(p.n_atoms for p in progs):
        raise ValueError("labels must hold n_atoms entries per program")
    if ws is None:
        nb = C.c_uint64(0)
        _check(lib().asp_scorer_train_workspace(len(progs), C.cast(arr, C.c_void_p), C.byref(nb)))
        ws = _arena(nb.value, device)
    p = np.ascontiguousarray(params, np.float32).copy()
    loss = np.zeros(max(int(steps), 1), np.float32)
    grad = np.zeros(SCORER_NPARAM, np.float32)
    _check(lib().asp_scorer_train(len(progs), C.cast(arr, C.c_void_p), _ptr(lab), _ptr(p),
                                  int(steps), float(lr), C.c_void_p(ws.data_ptr()),
                                  int(ws.numel()), _ptr(loss), _ptr(grad), _stream_ptr(stream)))
    return p, loss, grad


EXPORTS = (
    "asp_load_program", "asp_free_program", "asp_program_nogoods", "asp_bind_device",
    "asp_propagate", "asp_analyze_conflict", "asp_run_steps", "asp_solve",
    "asp_state_export", "asp_state_import", "asp_batch_create", "asp_batch_bind",
    "asp_solve_batch", "asp_batch_results", "asp_batch_last_ms", "asp_batch_free",
    "asp_status_str", "asp_last_error", "asp_set_scores", "asp_get_scores",
    "asp_batch_set_scores", "asp_batch_get_scores", "asp_scorer_workspace",
    "asp_batch_scorer_workspace", "asp_score_program", "asp_score_batch",
    "asp_batch_train_readout", "asp_batch_launch_info", "asp_solve_batch_graph",
    "asp_get_models", "asp_solve_noalloc", "asp_scorer_train_workspace", "asp_scorer_train",
    "asp_scorer_quantize", "asp_scorer_dequantize", "asp_batch_learned",
)

_lib = None


def lib():
    """Load libasp.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1909_01786_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        sig = {
            "asp_load_program": (i32, [i32, i32, P, P, P, C.POINTER(asp_options), C.POINTER(P),
                                       C.POINTER(asp_sizes)]),
            "asp_free_program": (i32, [P]),
            "asp_program_nogoods": (i32, [P, P, P]),
            "asp_bind_device": (i32, [P, P, u64, P, C.POINTER(asp_schedule)]),
            "asp_propagate": (i32, [P, P, i32, C.POINTER(asp_prop_result)]),
            "asp_analyze_conflict": (i32, [P, P, C.POINTER(asp_limits), P, i32, C.POINTER(i32),
                                           C.POINTER(i32)]),
            "asp_run_steps": (i32, [P, P, C.POINTER(asp_limits), i64, C.POINTER(asp_stats)]),
            "asp_solve": (i32, [P, P, C.POINTER(asp_limits), P, C.POINTER(asp_stats)]),
            "asp_solve_noalloc": (i32, [P, P, C.POINTER(asp_limits), P, C.POINTER(asp_stats)]),
            "asp_get_models": (i32, [P, P, P, i64, C.POINTER(i64)]),
            "asp_state_export": (i32, [P, P, C.POINTER(asp_state)]),
            "asp_state_import": (i32, [P, P, C.POINTER(asp_state)]),
            "asp_batch_create": (i32, [i32, P, C.POINTER(asp_schedule), C.POINTER(P),
                                       C.POINTER(u64), C.POINTER(u64)]),
            "asp_batch_bind": (i32, [P, P, u64, P]),
            "asp_solve_batch": (i32, [P, P, C.POINTER(asp_limits)]),
            "asp_solve_batch_graph": (i32, [P, P, C.POINTER(asp_limits)]),
            "asp_batch_results": (i32, [P, P, P, P, P]),
            "asp_batch_last_ms": (i32, [P, C.POINTER(C.c_double)]),
            "asp_batch_launch_info": (i32, [P, C.POINTER(i32), P, P, P, P, P]),
            "asp_batch_free": (i32, [P]),
            "asp_status_str": (C.c_char_p, [i32]),
            "asp_last_error": (i32, [C.c_char_p, u64]),
            "asp_set_scores": (i32, [P, P, P]),
            "asp_get_scores": (i32, [P, P, P]),
            "asp_batch_set_scores": (i32, [P, i32, P, P]),
            "asp_batch_get_scores": (i32, [P, i32, P, P]),
            "asp_scorer_workspace": (i32, [P, C.POINTER(u64)]),
            "asp_batch_scorer_workspace": (i32, [P, C.POINTER(u64)]),
            "asp_score_program": (i32, [P, C.POINTER(asp_scorer_weights), P, u64, P]),
            "asp_score_batch": (i32, [P, C.POINTER(asp_scorer_weights), P, u64, P]),
            "asp_batch_train_readout": (i32, [P, C.POINTER(asp_scorer_weights), P, u64, P, i32,
                                              C.c_float, P, P, P]),
            "asp_scorer_train_workspace": (i32, [i32, P, C.POINTER(u64)]),
            "asp_scorer_train": (i32, [i32, P, P, P, i32, C.c_float, P, u64, P, P, P]),
            "asp_scorer_quantize": (i32, [P, C.POINTER(asp_scorer_weights)]),
            "asp_scorer_dequantize": (i32, [C.POINTER(asp_scorer_weights), P]),
            "asp_batch_learned": (i32, [P, i32, P, i64, P, i64, C.POINTER(i32), C.POINTER(i64), P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def asp_status_str(st: int) -> str:
    return lib().asp_status_str(int(st)).decode()


def last_error() -> str:
    buf = C.create_string_buffer(1024)
    lib().asp_last_error(buf, 1024)
    return buf.value.decode(errors="replace")


def _check(rc: int, allowed=()) -> int:
    if rc < 0 and rc not in allowed:
        raise AspError(rc, last_error())
    return rc


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _arena(nbytes: int, device):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def limits(max_conflicts: int = -1, max_ms: int = 0) -> asp_limits:
    return asp_limits(int(max_conflicts), int(max_ms))


def options(W: int = 1, gate: int = GATE_UNFOUNDED, learned_cap_ng: int = 1 << 20,
            learned_cap_lits: int = 1 << 22, decision: int = DECISION_OCC,
            fallback_after: int = 10, learning: int = LEARN_FWD, max_models: int = 1,
            restart_every: int = 0, learn_conflicts: int = 1, lookahead: int = 0) -> asp_options:
    return asp_options(int(W), int(gate), int(learned_cap_ng), int(learned_cap_lits),
                       int(decision), int(fallback_after), int(learning), int(learn_conflicts),
                       int(max_models), int(restart_every), int(lookahead), 0)


@dataclass
class State:
    n_vars: int
    W: int
    cdl: int
    val: np.ndarray
    lvl: np.ndarray
    deps: np.ndarray
    dec: np.ndarray
    frontier: np.ndarray
    learned_off: np.ndarray
    learned: np.ndarray
    pending: int
    initialised: int
    status: int
    stats: dict
    score_mode: int = 0
    consec: int = 0
    dec_open: int = 0


class Program:
    """A ground program encoded by libasp (asp_load_program)."""

    def __init__(self, prog, W: int = 1, gate: int = GATE_UNFOUNDED,
                 learned_cap_ng: int = 1 << 20, learned_cap_lits: int = 1 << 22,
                 decision: int = DECISION_OCC, fallback_after: int = 10,
                 learning: int = LEARN_FWD, max_models: int = 1, restart_every: int = 0,
                 learn_conflicts: int = 1, lookahead: int = 0):
        self._head = np.ascontiguousarray(prog.head, np.int32)
        self._off = np.ascontiguousarray(prog.body_off, np.int64)
        self._lits = np.ascontiguousarray(prog.body_lits, np.int32)
        self.opt = options(W, gate, learned_cap_ng, learned_cap_lits, decision, fallback_after,
                           learning, max_models, restart_every, learn_conflicts, lookahead)
        self.sizes = asp_sizes()
        h = C.c_void_p()
        _check(lib().asp_load_program(int(prog.n_atoms), int(self._head.shape[0]),
                                      _ptr(self._head), _ptr(self._off), _ptr(self._lits),
                                      C.byref(self.opt), C.byref(h), C.byref(self.sizes)))
        self._h = h
        self.n_atoms = int(prog.n_atoms)
        self.W = int(W)
        self.arena = None
        self.stream = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and h.value and _lib is not None:
            _lib.asp_free_program(h)
            self._h = None

    @property
    def n_vars(self) -> int:
        return int(self.sizes.n_vars)

    def nogoods(self):
        n = int(self.sizes.n_nogoods)
        off = np.zeros(n + 1, np.int32)
        lits = np.zeros(max(int(self.sizes.n_lits), 1), np.int32)
        _check(lib().asp_program_nogoods(self._h, _ptr(off), _ptr(lits)))
        return off, lits[:int(self.sizes.n_lits)]

    def bind(self, device="cuda", threads: int = 256, stream=None):
        """Allocate the arena (torch) and upload the program."""
        self.arena = _arena(self.sizes.device_bytes, device)
        self.stream = stream
        sch = asp_schedule(int(threads), 1, (C.c_int32 * 4)(0, 0, 0, 0))
        _check(lib().asp_bind_device(self._h, C.c_void_p(self.arena.data_ptr()),
                                     int(self.arena.numel()), _stream_ptr(stream), C.byref(sch)))
        return self

    def set_scores(self, scores):
        """Decision scores of atoms 0..n_atoms (index 0 ignored)."""
        sc = np.ascontiguousarray(scores, np.int32)
        if sc.shape != (self.n_atoms + 1,):
            raise ValueError("scores must have n_atoms + 1 entries")
        _check(lib().asp_set_scores(self._h, _ptr(sc), _stream_ptr(self.stream)))

    def get_scores(self) -> np.ndarray:
        out = np.zeros(self.n_atoms + 1, np.int32)
        _check(lib().asp_get_scores(self._h, _ptr(out), _stream_ptr(self.stream)))
        return out

    def score(self, weights: dict, device="cuda"):
        """Run the learned scorer on the device; returns the atom scores."""
        nb = C.c_uint64(0)
        _check(lib().asp_scorer_workspace(self._h, C.byref(nb)))
        ws = _arena(nb.value, device)
        w = scorer_weights(weights)
        _check(lib().asp_score_program(self._h, C.byref(w), C.c_void_p(ws.data_ptr()),
                                       int(ws.numel()), _stream_ptr(self.stream)))
        return self.get_scores()

    def propagate(self, max_rounds: int = 0):
        r = asp_prop_result()
        st = _check(lib().asp_propagate(self._h, _stream_ptr(self.stream), int(max_rounds),
                                        C.byref(r)))
        return st, {n: getattr(r, n) for n, _ in r._fields_}

    def analyze_conflict(self, lim: asp_limits | None = None, cap: int = 1 << 16):
        buf = np.zeros(cap, np.int32)
        ln, bj = C.c_int32(0), C.c_int32(0)
        st = _check(lib().asp_analyze_conflict(self._h, _stream_ptr(self.stream),
                                               C.byref(lim) if lim else None, _ptr(buf), cap,
                                               C.byref(ln), C.byref(bj)))
        return st, buf[:ln.value].copy(), bj.value

    def run_steps(self, n_steps: int, lim: asp_limits | None = None):
        s = asp_stats()
        st = _check(lib().asp_run_steps(self._h, _stream_ptr(self.stream),
                                        C.byref(lim) if lim else None, int(n_steps), C.byref(s)))
        return st, s.as_dict()

    def solve(self, lim: asp_limits | None = None):
        m = np.zeros(max(self.n_atoms, 1), np.uint8)
        s = asp_stats()
        st = _check(lib().asp_solve(self._h, _stream_ptr(self.stream),
                                    C.byref(lim) if lim else None, _ptr(m), C.byref(s)))
        return st, (m[:self.n_atoms].copy() if st == SAT else None), s.as_dict()

    def solve_noalloc(self, lim: asp_limits | None = None, stream=None):
        """asp_solve_noalloc: the same solve in the library's own device
        array (no arena; the program need not be bound)."""
        m = np.zeros(max(self.n_atoms, 1), np.uint8)
        s = asp_stats()
        sp = _stream_ptr(stream) if stream is not None else None   # None: the default stream
        st = _check(lib().asp_solve_noalloc(self._h, sp,
                                            C.byref(lim) if lim else None, _ptr(m), C.byref(s)))
        return st, (m[:self.n_atoms].copy() if st == SAT else None), s.as_dict()

    def models(self) -> list:
        """The answer sets kept from the last search, in the order found
        (at most max(1, max_models) of them)."""
        store = max(1, int(self.opt.max_models))
        found = C.c_int64(0)
        buf = np.zeros(max(store * self.n_atoms, 1), np.uint8)
        _check(lib().asp_get_models(self._h, _stream_ptr(self.stream), _ptr(buf), store,
                                    C.byref(found)))
        n = min(int(found.value), store)
        return [buf[k * self.n_atoms:(k + 1) * self.n_atoms].copy() for k in range(n)]

    def export_state(self) -> State:
        st = asp_state()
        _check(lib().asp_state_export(self._h, _stream_ptr(self.stream), C.byref(st)))
        V, W = st.n_vars, st.W
        val = np.zeros(V + 1, np.int8)
        lvl = np.zeros(V + 1, np.int32)
        deps = np.zeros((V + 1) * W, np.uint64)
        dec = np.zeros(st.cdl + 1, np.int32)
        fr = np.zeros(max(st.frontier_len, 1), np.int32)
        loff = np.zeros(st.n_learned + 1, np.int32)
        lits = np.zeros(max(st.learned_lits, 1), np.int32)
        st.val, st.lvl, st.deps, st.dec = _ptr(val), _ptr(lvl), _ptr(deps), _ptr(dec)
        st.frontier, st.learned_off, st.learned = _ptr(fr), _ptr(loff), _ptr(lits)
        _check(lib().asp_state_export(self._h, _stream_ptr(self.stream), C.byref(st)))
        return State(V, W, st.cdl, val, lvl, deps.reshape(V + 1, W), dec,
                     fr[:st.frontier_len], loff, lits[:st.learned_lits], st.pending,
                     st.initialised, st.status, st.stats.as_dict(), st.score_mode, st.consec,
                     st.dec_open)

    def import_state(self, s: State):
        st = asp_state()
        val = np.ascontiguousarray(s.val, np.int8)
        lvl = np.ascontiguousarray(s.lvl, np.int32)
        deps = np.ascontiguousarray(np.asarray(s.deps, np.uint64).reshape(-1))
        dec = np.ascontiguousarray(s.dec, np.int32)
        fr = np.ascontiguousarray(s.frontier, np.int32)
        loff = np.ascontiguousarray(s.learned_off, np.int32)
        lits = np.ascontiguousarray(s.learned, np.int32)
        st.n_vars, st.W, st.cdl = int(s.n_vars), int(s.W), int(s.cdl)
        st.frontier_len = int(fr.shape[0])
        st.n_learned = int(loff.shape[0]) - 1
        st.pending = int(s.pending)
        st.learned_lits = int(lits.shape[0])
        st.initialised = int(s.initialised)
        st.status = RUNNING
        st.score_mode, st.consec, st.dec_open = int(s.score_mode), int(s.consec), int(s.dec_open)
        st.val, st.lvl, st.deps, st.dec = _ptr(val), _ptr(lvl), _ptr(deps), _ptr(dec)
        st.frontier, st.learned_off, st.learned = _ptr(fr), _ptr(loff), _ptr(lits)
        for k, v in (s.stats or {}).items():
            if hasattr(st.stats, k):
                setattr(st.stats, k, int(v))
        _check(lib().asp_state_import(self._h, _stream_ptr(self.stream), C.byref(st)))


class Batch:
    """Many programs solved together (asp_solve_batch): one workgroup per
    program, one launch per LDS size class."""

    def __init__(self, programs, threads: int = 128, classes: int = 4, class_threads=None):
        self.programs = list(programs)
        arr = (C.c_void_p * len(self.programs))(*[p._h.value for p in self.programs])
        self._arr = arr
        ct = list(class_threads or []) + [0] * 4
        sch = asp_schedule(int(threads), int(classes), (C.c_int32 * 4)(*[int(x) for x in ct[:4]]))
        h = C.c_void_p()
        nb, mb = C.c_uint64(0), C.c_uint64(0)
        _check(lib().asp_batch_create(len(self.programs), C.cast(arr, C.c_void_p), C.byref(sch),
                                      C.byref(h), C.byref(nb), C.byref(mb)))
        self._h = h
        self.device_bytes = int(nb.value)
        self.model_bytes = int(mb.value)
        self.arena = None
        self.stream = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and h.value and _lib is not None:
            _lib.asp_batch_free(h)
            self._h = None

    def bind(self, device="cuda", stream=None):
        self.arena = _arena(self.device_bytes, device)
        self.stream = stream
        _check(lib().asp_batch_bind(self._h, C.c_void_p(self.arena.data_ptr()),
                                    int(self.arena.numel()), _stream_ptr(stream)))
        return self

    def set_scores(self, i: int, scores):
        sc = np.ascontiguousarray(scores, np.int32)
        if sc.shape != (self.programs[i].n_atoms + 1,):
            raise ValueError("scores must have n_atoms + 1 entries")
        _check(lib().asp_batch_set_scores(self._h, int(i), _ptr(sc), _stream_ptr(self.stream)))

    def get_scores(self, i: int) -> np.ndarray:
        out = np.zeros(self.programs[i].n_atoms + 1, np.int32)
        _check(lib().asp_batch_get_scores(self._h, int(i), _ptr(out), _stream_ptr(self.stream)))
        return out

    def scorer_workspace(self, device="cuda"):
        nb = C.c_uint64(0)
        _check(lib().asp_batch_scorer_workspace(self._h, C.byref(nb)))
        return _arena(nb.value, device)

    def score(self, weights, ws=None):
        """Enqueue the learned scorer over every instance (asynchronous).
        ``weights``: a dict of codes or a packed asp_scorer_weights."""
        if ws is None:
            if getattr(self, "_ws", None) is None:
                self._ws = self.scorer_workspace(self.arena.device)
            ws = self._ws
        w = weights if isinstance(weights, asp_scorer_weights) else scorer_weights(weights)
        self._w = w
        _check(lib().asp_score_batch(self._h, C.byref(w), C.c_void_p(ws.data_ptr()),
                                     int(ws.numel()), _stream_ptr(self.stream)))

    def train_readout(self, weights, labels, steps: int = 400, lr: float = 0.05, wb0=None):
        """Train the scorer readout on the device; returns (wb[65], losses)."""
        if getattr(self, "_ws", None) is None:
            self._ws = self.scorer_workspace(self.arena.device)
        w = weights if isinstance(weights, asp_scorer_weights) else scorer_weights(weights)
        lab = np.ascontiguousarray(labels, np.int8)
        if lab.shape != (self.model_bytes,):
            raise ValueError("labels must have one entry per atom of the batch")
        wb = np.zeros(65, np.float32) if wb0 is None else np.ascontiguousarray(wb0, np.float32)
        loss = np.zeros(int(steps), np.float32)
        _check(lib().asp_batch_train_readout(self._h, C.byref(w), C.c_void_p(self._ws.data_ptr()),
                                             int(self._ws.numel()), _ptr(lab), int(steps),
                                             float(lr), _ptr(wb), _ptr(loss),
                                             _stream_ptr(self.stream)))
        return wb, loss

    def solve(self, lim: asp_limits | None = None, graph: bool = False):
        """Enqueue the batched solve on the stream (asynchronous); with
        graph=True as one replay of the captured HIP graph (the batch must be
        bound on a non-default stream)."""
        f = lib().asp_solve_batch_graph if graph else lib().asp_solve_batch
        _check(f(self._h, _stream_ptr(self.stream), C.byref(lim) if lim else None))

    def learned(self, i: int):
        """(offsets, literals) of the nogoods instance i learned in the last
        solve (asp_batch_learned)."""
        n, nl = C.c_int32(0), C.c_int64(0)
        _check(lib().asp_batch_learned(self._h, int(i), None, 0, None, 0, C.byref(n),
                                       C.byref(nl), _stream_ptr(self.stream)))
        off = np.zeros(n.value + 1, np.int32)
        lits = np.zeros(max(nl.value, 1), np.int32)
        _check(lib().asp_batch_learned(self._h, int(i), _ptr(off), off.shape[0], _ptr(lits),
                                       lits.shape[0], C.byref(n), C.byref(nl),
                                       _stream_ptr(self.stream)))
        return off, lits[:nl.value]

    def launch_info(self):
        """[(first, count, threads, ms)] per launch class, and the instance order."""
        n = C.c_int32(0)
        first, count, thr = (C.c_int32 * 4)(), (C.c_int32 * 4)(), (C.c_int32 * 4)()
        ms = (C.c_double * 4)()
        order = np.zeros(len(self.programs), np.int32)
        _check(lib().asp_batch_launch_info(self._h, C.byref(n), first, count, thr, ms, _ptr(order)))
        return [(first[c], count[c], thr[c], ms[c]) for c in range(n.value)], order

    def last_ms(self) -> float:
        ms = C.c_double(0)
        _check(lib().asp_batch_last_ms(self._h, C.byref(ms)))
        return float(ms.value)

    def results(self, all_models: bool = False):
        """(verdicts, models, stats): models[i] is instance i's first answer
        set, or with all_models the list of the answer sets it kept."""
        n = len(self.programs)
        verd = np.zeros(n, np.int32)
        models = np.zeros(max(self.model_bytes, 1), np.uint8)
        stats = (asp_stats * n)()
        _check(lib().asp_batch_results(self._h, _stream_ptr(self.stream), _ptr(verd),
                                       _ptr(models), C.cast(stats, C.c_void_p)))
        sd = [s.as_dict() for s in stats]
        out_models, o = [], 0
        for i, p in enumerate(self.programs):
            store = max(1, int(p.opt.max_models))
            A = p.n_atoms
            if all_models:
                k = min(int(sd[i]["models"]), store)
                out_models.append([models[o + j * A:o + (j + 1) * A].copy() for j in range(k)])
            else:
                out_models.append(models[o:o + A].copy())
            o += A * store
        return verd, out_models, sd
