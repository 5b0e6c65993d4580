"""Write the oracle's results on the 4096-program benchmark batch.

For each search mode this runs the CPU oracle (``oracle/``, nothing else) on
every program of the batch -- 4096 random ground normal programs from
``aspgen.batch_random(i, 3000)``, conflict budget 2000, W = 1, learned store
4096 nogoods / 2^18 literals -- and writes one CSV row per program: verdict,
every search counter, the trace hash and a SHA-256 prefix of the answer sets
found.  The GPU tests and the benchmark compare the library's results on the
same batch with these rows, program by program.

    python tests/golden/oracle_batch.py MODE [--workers N] [--n 4096]

MODE: plain, jw, activity, multi4, enum16, look4, res.  Res-learning's long
learned nogoods make some programs cost the oracle an hour or more, so
"res" covers a sample: programs of every LDS size class (variables above
32767, above 16383, above 4095, the rest) are taken in a seeded random
order and each is run in a child process allowed RES_SECONDS; the first
RES_PER_CLASS of each class that finish are kept.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import aspgen  # noqa: E402
import oracle  # noqa: E402

SEED, BUDGET, CAP_NG, CAP_LITS, W = 3000, 2000, 4096, 1 << 18, 1
MODES = {
    "plain": {},
    "jw": {"decision": oracle.DEC_JW},
    "activity": {"decision": oracle.DEC_ACTIVITY},
    "multi4": {"learn_conflicts": 4},
    "enum16": {"max_models": 16},
    "res": {"learning": oracle.LEARN_RES},
    "look4": {"lookahead": 4},
}
FIELDS = ("i", "status", "rounds", "visits", "literal_checks", "propagations", "decisions",
          "conflicts", "learned", "learned_len", "gate_failures", "completes", "models",
          "restarts", "exhausted", "trace_hash", "models_sha", "deps_reads")


RES_PER_CLASS = 4
RES_SECONDS = 240


def lds_class(prog) -> int:
    """LDS size class of a program by its variable count V = atoms + 3 *
    headed rules (0 holds the largest)."""
    V = int(prog.n_atoms) + 3 * int((np.asarray(prog.head) != 0).sum())
    return 0 if V > 32767 else 1 if V > 16383 else 2 if V > 4095 else 3


def path(mode: str, n: int = 4096) -> str:
    return os.path.join(HERE, f"oracle_batch{SEED}_n{n}_b{BUDGET}_{mode}.csv")


def models_sha(models) -> str:
    """SHA-256 prefix over the answer sets in the order found (one byte per atom)."""
    if not models:
        return "-"
    h = hashlib.sha256()
    for m in models:
        h.update(np.ascontiguousarray(m, np.uint8).tobytes())
        h.update(b"|")
    return h.hexdigest()[:16]


def run_one(i: int, mode: str):
    prog = aspgen.batch_random(i, batch_seed=SEED)
    lim = oracle.make_limits(BUDGET, CAP_NG, CAP_LITS)
    kw = MODES[mode]
    if "max_models" in kw:
        rc, models, st, ex = oracle.enumerate_models(prog, max_models=kw["max_models"], W=W,
                                                     limits=lim)
        if rc in (oracle.UNSAT, oracle.UNKNOWN) and models:
            rc = oracle.SAT                  # a search that found answer sets reports SAT
        exhausted = int(ex)
    else:
        rc, m, st = oracle.solve(prog, W=W, limits=lim, **kw)
        models = [m] if m is not None else []
        exhausted = 0
    row = {"i": i, "status": rc, **{k: int(st[k]) for k in FIELDS[2:14] if k != "exhausted"},
           "exhausted": exhausted, "trace_hash": int(st["trace_hash"]) & (2 ** 64 - 1),
           "models_sha": models_sha(models), "deps_reads": int(st["deps_reads"])}
    return row


def load(mode: str, n: int = 4096):
    """Rows of a written file, by program index (None if absent)."""
    p = path(mode, n)
    if not os.path.exists(p):
        return None
    rows = {}
    with open(p) as fh:
        head = fh.readline().strip().split(",")
        for line in fh:
            v = line.strip().split(",")
            r = dict(zip(head, v))
            rows[int(r["i"])] = {k: (r[k] if k == "models_sha" else int(r[k])) for k in head}
    return rows


def res_sample(workers: int):
    """Rows of the Res-learning sample (see the module docstring)."""
    import json
    import subprocess
    rng = np.random.default_rng(7)
    strata = [[] for _ in range(4)]
    for i in rng.permutation(4096):
        i = int(i)
        strata[lds_class(aspgen.batch_random(i, batch_seed=SEED))].append(i)
    code = ("import sys, json; sys.path.insert(0, %r); sys.path.insert(0, %r); "
            "import oracle_batch as ob; print(json.dumps(ob.run_one(int(sys.argv[1]), 'res')))"
            % (ROOT, HERE))

    def attempt(i):
        try:
            out = subprocess.run([sys.executable, "-c", code, str(i)], capture_output=True,
                                 text=True, timeout=RES_SECONDS)
            return json.loads(out.stdout.strip().splitlines()[-1])
        except subprocess.TimeoutExpired:
            return None

    rows = {}
    for c, st in enumerate(strata):
        got, tried = [], 0
        with ThreadPoolExecutor(workers) as ex:
            while len(got) < RES_PER_CLASS and tried < len(st):
                batch = st[tried:tried + workers]
                tried += len(batch)
                for i, r in zip(batch, ex.map(attempt, batch)):
                    if r is not None and len(got) < RES_PER_CLASS:
                        got.append(i)
                        rows[i] = r
                print(f"res: class {c}: {len(got)} kept of {tried} tried", flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=sorted(MODES))
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--n", type=int, default=4096)
    args = ap.parse_args()
    oracle.build()
    t0 = time.time()
    if args.mode == "res":
        rows = res_sample(args.workers)
    else:
        # largest programs first, so the pool ends together
        sizes = [(aspgen.batch_random(i, batch_seed=SEED).body_lits.size, i) for i in range(args.n)]
        order = [i for _, i in sorted(sizes, reverse=True)]
        rows = {}
        with ThreadPoolExecutor(args.workers) as ex:
            for k, r in enumerate(ex.map(lambda i: run_one(i, args.mode), order)):
                rows[r["i"]] = r
                if (k + 1) % 256 == 0:
                    print(f"{args.mode}: {k + 1}/{args.n} in {time.time() - t0:.0f} s", flush=True)
    tmp = path(args.mode, args.n) + ".tmp"
    with open(tmp, "w") as fh:
        fh.write(",".join(FIELDS) + "\n")
        for i in sorted(rows):
            fh.write(",".join(str(rows[i][k]) for k in FIELDS) + "\n")
    os.replace(tmp, path(args.mode, args.n))
    print(f"{args.mode}: wrote {path(args.mode, args.n)} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
