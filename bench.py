"""Benchmark of the batched GPU search (one MI355X).

One step = one batched solve (asp_solve_batch) that runs the whole
search -- InitialPropagation, PropagateAndCheck rounds, Fwd-learning with
Backjump, Decision / CompleteAssignment and the stability check -- for every
program of a batch of uneven random ground programs (4096 programs, atoms
log-uniform in 100..5000, rules/atoms uniform in 2..4, bodies of 1..4
literals, half of them negated), under a fixed per-instance conflict budget.
Inputs are resident in HBM before the timed region; the step is timed with
HIP events recorded on the launch streams.

Metric: nogood literal checks per second (a visit of nogood d from a
propagated literal counts |d| checks), with decided instances per second
beside it, for the plain (occurrence) Decision; the learned leg reruns the
same batch with the learned scorer (scoring included in its timed step) and
reports its decided instances per second and the ratio to the plain form.

The roofline entry is taken for the dominant launch (the LDS size class
whose launch runs longest): its algorithmic HBM bytes (per visit 4 B map
entry + 8 B nogood offsets + 4 B per literal) over its HIP-event duration.
Its `traffic` is the measured HBM bytes of that launch from the committed
counter summary (profiles/k_search_traffic.json), used only while the
kernel sources are the ones the counters were taken with.

The oracle leg (cpu_baseline) times the plain CPU oracle on a bounded sample
of the same batch with the same budget, one thread per host core.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 4096]
    python bench.py --write-traffic FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
METRIC = "nogood literal checks/s & instances/s, learned vs plain Decision, 1 MI355X"
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "k_search_traffic.json")
KERNEL_SOURCES = ("paper_1909_01786_amd/csrc/solver.hip", "paper_1909_01786_amd/csrc/layout.h")
COPY_BYTES = 1 << 30


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_batch(n: int, seed: int):
    import aspgen
    return [aspgen.batch_random(i, batch_seed=seed) for i in range(n)]


def load_programs(progs, W, cap_ng, cap_lits, workers=16, **kw):
    import paper_1909_01786_amd as P
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda p: P.Program(p, W=W, learned_cap_ng=cap_ng,
                                               learned_cap_lits=cap_lits, **kw), progs))


def host_cpu():
    """Host cores visible to this process and the CPU model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count() or 1, "usable": usable, "model": model}


def lds_class(prog) -> int:
    """The LDS size class (0 = largest) of a program of the batch, by its
    variable count V = atoms + 3 * headed rules (bounds 4095, 16383, 32767)."""
    V = int(prog.n_atoms) + 3 * int((np.asarray(prog.head) != 0).sum())
    return 0 if V > 32767 else 1 if V > 16383 else 2 if V > 4095 else 3


def cpu_baseline(progs, W, budget, cap_ng, cap_lits, target_s, gpu_stats):
    """The oracle on a bounded sample of the batch, stratified by LDS class
    (classes taken in turn, programs drawn at random inside a class, heavy
    programs kept), one thread per usable host core up to the 16 a
    one-GPU job is allotted, largest programs first.  The oracle's C entry
    releases the GIL.  The sampled verdicts and counters are also checked
    against the GPU's."""
    import oracle
    oracle.build()
    n = len(progs)
    host = host_cpu()
    cores = max(1, min(16, host["usable"]))
    rng = np.random.default_rng(12345)
    strata = [[] for _ in range(4)]
    for i in rng.permutation(n):
        strata[lds_class(progs[int(i)])].append(int(i))
    # the sample is bounded by the GPU's own counters at a nominal oracle
    # rate of 3e7 literal checks per second per thread
    checks = np.array([s["literal_checks"] for s in gpu_stats], dtype=np.float64)
    budget_checks = target_s * 3.0e7 * cores
    pick, acc, k = [], 0.0, 0
    while acc < budget_checks and any(strata):
        st = strata[k % 4]
        k += 1
        if not st:
            continue
        i = st.pop()
        pick.append(i)
        acc += checks[i]
    lim = oracle.make_limits(budget, cap_ng, cap_lits)

    def one(i):
        return i, *oracle.solve(progs[i], W=W, limits=lim)

    order = sorted(pick, key=lambda i: -checks[i])
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        res = list(ex.map(one, order))
    wall = time.perf_counter() - t0
    tot_checks = sum(r[3]["literal_checks"] for r in res)
    mism = 0
    for i, rc, _, st in res:
        g = gpu_stats[i]
        same = all(int(g[k]) == int(st[k]) for k in
                   ("literal_checks", "visits", "conflicts", "decisions", "rounds", "trace_hash"))
        mism += int((not same) or rc != g["status"])
    per_class = [sum(1 for i in pick if lds_class(progs[i]) == c) for c in range(4)]
    return {
        "value": tot_checks / wall, "unit": "literal checks/s", "cores": cores,
        "kind": "oracle",
        "sample": f"{len(pick)} of {n} instances of the same batch, stratified by LDS class "
                  f"({per_class} per class, largest first), same conflict budget; "
                  f"{tot_checks} literal checks in {wall:.1f} s wall on {cores} threads",
        "host": host,
        "instances_per_s": len(pick) / wall,
        "sample_mismatches_vs_gpu": int(mism),
    }


def golden_rows(mode, n, seed, budget, W, cap_ng, cap_lits):
    """The oracle's stored results on the whole batch for this mode
    (tests/golden/oracle_batch.py), when they were written for this
    configuration; else None."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import oracle_batch as ob
    if (seed, budget, W, cap_ng, cap_lits) != (ob.SEED, ob.BUDGET, ob.W, ob.CAP_NG, ob.CAP_LITS):
        return None
    return ob.load(mode, n)


def models_sha(models) -> str:
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import oracle_batch as ob
    return ob.models_sha(models)


_ORACLE_KEYS = ("rounds", "visits", "literal_checks", "propagations", "decisions", "conflicts",
                "learned", "learned_len", "gate_failures", "completes", "trace_hash")


def check_against_oracle(rows, verd, model_lists, stats, enum=False):
    """Every instance of the batch against the oracle's stored row:
    verdict, every search counter, the trace hash and the answer sets."""
    if rows is None:
        return None
    n = len(verd)
    bad = []
    for i in range(n):
        r, g = rows.get(i), stats[i]
        if r is None:
            bad.append(i)
            continue
        same = int(verd[i]) == r["status"] and all(
            (int(g[k]) & (2 ** 64 - 1)) == r[k] for k in _ORACLE_KEYS)
        if enum:
            same = same and int(g["models"]) == r["models"] and int(g["exhausted"]) == r["exhausted"]
        same = same and models_sha(model_lists[i]) == r["models_sha"]
        if not same:
            bad.append(i)
    decided = int(((verd == 1) | (verd == 2)).sum())
    dec_bad = sum(1 for i in bad if verd[i] in (1, 2))
    return {"instances": n, "identical_to_oracle": n - len(bad), "decided": decided,
            "decided_identical": decided - dec_bad,
            "verified_fraction": (decided - dec_bad) / n,
            "mismatched": bad[:10],
            "note": "verdict, every counter, trace hash and answer sets of every instance "
                    "against the oracle's stored run (tests/golden); UNKNOWN counts against "
                    "the verified fraction"}


# ------------------------------------------------------------ counters
def _pmc_per_dispatch(path: str, name_part: str):
    agg = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if name_part in r["Kernel_Name"]:
                d = int(r["Dispatch_Id"])
                agg[d] = agg.get(d, 0.0) + float(r["Counter_Value"])
    return [agg[k] for k in sorted(agg)]


def write_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, config):
    """Summarise two FETCH_SIZE / WRITE_SIZE runs of this benchmark (and of
    the 1 GiB copy calibration) into the per-launch traffic file."""
    def one(d):
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith("counter_collection.csv"):
                    return os.path.join(root, f)
        raise FileNotFoundError(d)
    fe = _pmc_per_dispatch(one(fetch_dir), "k_search")
    wr = _pmc_per_dispatch(one(write_dir), "k_search")
    cf = _pmc_per_dispatch(one(copy_fetch_dir), "copyBuffer")
    cw = _pmc_per_dispatch(one(copy_write_dir), "copyBuffer")
    kib = COPY_BYTES / 1024.0
    f_scale = kib / float(np.median(cf))
    w_scale = kib / float(np.median(cw))
    out = {
        "kernel_sha": kernel_hash(), "config": config,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "launch_bytes": [fe[i] * 1024.0 * f_scale + wr[i] * 1024.0 * w_scale
                         for i in range(min(len(fe), len(wr)))],
        "fetch_kib": fe, "write_kib": wr,
        "note": "per k_search dispatch of one eager bench step (--profile-step: the last "
                "len(class_threads) dispatches), in launch order (LDS class 0 first); "
                "scale = copied KiB / counter KiB of a plain 1 GiB device copy",
    }
    nc = len(config.get("class_threads", [])) or 4
    out["launch_bytes"] = out["launch_bytes"][-nc:]
    # one file per kernel sources, one run per schedule measured with them
    runs = []
    try:
        with open(TRAFFIC_JSON) as fh:
            t = json.load(fh)
        if t.get("kernel_sha") == out["kernel_sha"]:
            runs = [r for r in _traffic_runs(t) if r.get("config") != config]
    except OSError:
        pass
    run = {k: v for k, v in out.items() if k != "kernel_sha"}
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump({"kernel_sha": out["kernel_sha"], "runs": runs + [run]}, fh, indent=1)
    print(json.dumps(out))


def _traffic_runs(t):
    """The measured runs of a traffic file (a single run at the top level
    in files written before it held several schedules)."""
    return t["runs"] if "runs" in t else [{k: v for k, v in t.items() if k != "kernel_sha"}]


def traffic_for(config, launch_index):
    """Measured HBM bytes of one launch, when the counters were taken with
    these kernel sources, this batch and budget and the same threads for
    that launch's LDS class; else None."""
    try:
        with open(TRAFFIC_JSON) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("kernel_sha") != kernel_hash():
        return None
    for r in _traffic_runs(t):
        tc = r.get("config", {})
        if any(tc.get(k) != config.get(k) for k in ("n", "seed", "budget", "W", "classes")):
            continue
        a, b = tc.get("class_threads", []), config.get("class_threads", [])
        if launch_index >= len(a) or launch_index >= len(b) or a[launch_index] != b[launch_index]:
            continue
        lb = r.get("launch_bytes", [])
        if launch_index < len(lb):
            return lb[launch_index]
    return None


# ------------------------------------------------------------ runs
def timed_steps(batch, lim, steps, warmup, before=None, graph=False):
    """Warm-up then timed batched solves, each bracketed by device
    synchronisations; with graph=True every solve is one replay of the
    captured HIP graph (the first warm-up captures it)."""
    import torch
    for w in range(warmup):
        if before:
            before()
        batch.solve(lim, graph=graph)
        torch.cuda.synchronize()
        log(f"[bench] warmup {w} {batch.last_ms():.1f} ms")
    ms, walls = [], []
    for s in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if before:
            before()
        batch.solve(lim, graph=graph)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        ms.append(batch.last_ms())
        log(f"[bench] step {s} {'graph' if graph else 'kernel'} {ms[-1]:.1f} ms, "
            f"wall {walls[-1] * 1e3:.1f} ms")
    return ms, walls


def tail(stats):
    ns = np.array([s["ns_total"] for s in stats], np.float64) / 1e6
    return {"p50": float(np.percentile(ns, 50)), "p99": float(np.percentile(ns, 99)),
            "max": float(ns.max())}


def time_split(stats, members=None):
    """Where the device time goes: share of each step kind and the mean
    device time per event (round, conflict, decision) over the instances."""
    sel = [stats[i] for i in (members if members is not None else range(len(stats)))]
    tot = sum(s["ns_total"] for s in sel) or 1
    out = {k: sum(s["ns_" + k] for s in sel) / tot for k in ("round", "learn", "decide", "gate")}
    ev = {"round": "rounds", "learn": "conflicts", "decide": "decisions"}
    for k, n in ev.items():
        cnt = sum(int(s[n]) for s in sel)
        out[f"us_per_{n[:-1]}"] = sum(s["ns_" + k] for s in sel) / 1e3 / max(cnt, 1)
    out["rounds_per_instance"] = sum(int(s["rounds"]) for s in sel) / max(len(sel), 1)
    return out


def search_counters(stats, ms_step):
    """Per-second search counters of a whole step (the quantities the
    paper's Fig. 1 and Fig. 2 compare between Fwd- and Res-learning)."""
    tot = {k: sum(int(s[k]) for s in stats)
           for k in ("propagations", "decisions", "conflicts", "learned", "learned_len")}
    sec = ms_step / 1000.0
    return {"propagations_per_s": tot["propagations"] / sec,
            "decisions_per_s": tot["decisions"] / sec,
            "conflicts_per_s": tot["conflicts"] / sec,
            "learned_per_s": tot["learned"] / sec,
            "avg_learned_len": tot["learned_len"] / max(tot["learned"], 1)}


def verify_models(progs, verd, models):
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from brute import is_stable
    sat = np.nonzero(verd == 1)[0]
    bad = [int(i) for i in sat if not is_stable(progs[i], models[i])]
    return int(sat.size), bad


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=3000)
    ap.add_argument("--budget", type=int, default=2000, help="conflicts per instance")
    ap.add_argument("--W", type=int, default=1)
    ap.add_argument("--threads", type=int, default=128)
    ap.add_argument("--classes", type=int, default=4, help="LDS size classes (launches)")
    ap.add_argument("--class-threads", default="256,128,128,128",
                    help="threads per class, largest first (with --no-autotune)")
    ap.add_argument("--cap-ng", type=int, default=4096)
    ap.add_argument("--cap-lits", type=int, default=1 << 18)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--max-ms", type=int, default=150000, help="device time guard per launch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-steps", type=int, default=3,
                    help="timed steps of the learned leg (its one-step time varies by ~10%%)")
    ap.add_argument("--weights", default=None,
                    help="scorer weight codes (.npz) for the learned legs; default: the trained file")
    ap.add_argument("--no-res", action="store_true", help="skip the Res-learning leg")
    ap.add_argument("--no-enum", action="store_true", help="skip the several-answer-sets leg")
    ap.add_argument("--no-heur", action="store_true",
                    help="skip the Jeroslow-Wang and activity Decision legs")
    ap.add_argument("--no-multi", action="store_true",
                    help="skip the several-conflicts-per-step leg")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the single-instance legs (200-atom programs, 3-colourings)")
    ap.add_argument("--no-hc", action="store_true", help="skip the Hamiltonian-cycle batch legs")
    ap.add_argument("--no-budget-leg", action="store_true",
                    help="skip the larger-budget leg (decided fraction)")
    ap.add_argument("--big-budget", type=int, default=20000)
    ap.add_argument("--budget-restarts", action="store_true",
                    help="also run the larger budget with activity and restarts")
    ap.add_argument("--multi-k", type=int, default=4, help="conflicts learned per step")
    ap.add_argument("--no-lookahead", action="store_true", help="skip the lookahead-Decision leg")
    ap.add_argument("--lookahead", type=int, default=4, help="candidates tried per lookahead Decision")
    ap.add_argument("--enum-models", type=int, default=16, help="answer sets asked per program")
    ap.add_argument("--res-steps", type=int, default=1)
    ap.add_argument("--eager-steps", type=int, default=2,
                    help="eager (stream-launched) solves after the graph-timed steps: per-launch times")
    ap.add_argument("--no-autotune", action="store_true",
                    help="take --classes / --class-threads instead of timing the candidates")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--write-traffic", nargs=4, metavar="DIR",
                    help="summarise FETCH, WRITE, copy FETCH, copy WRITE counter runs")
    ap.add_argument("--profile-step", action="store_true",
                    help="only the headline batch: one warm-up and one eager solve (for counters)")
    args = ap.parse_args()
    cth = [int(x) for x in args.class_threads.split(",") if x]
    config = {"n": args.n, "seed": args.seed, "budget": args.budget, "W": args.W,
              "threads": args.threads, "classes": args.classes, "class_threads": cth}

    if args.write_traffic:
        write_traffic(*args.write_traffic, config)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the batch would shard by instance across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    if args.copy_calibration:
        a = torch.empty(COPY_BYTES, dtype=torch.uint8, device=dev)
        b = torch.empty(COPY_BYTES, dtype=torch.uint8, device=dev)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": COPY_BYTES, "launches": 3}))
        return

    import paper_1909_01786_amd as P

    t0 = time.perf_counter()
    progs = make_batch(args.n, args.seed)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    gp = load_programs(progs, args.W, args.cap_ng, args.cap_lits)
    t_enc = time.perf_counter() - t0
    n_lits = sum(int(g.sizes.n_lits) for g in gp)
    log(f"[bench] generated {args.n} programs in {t_gen:.1f}s, encoded in {t_enc:.1f}s, "
        f"{n_lits} nogood literals")

    lim = P.limits(args.budget, args.max_ms)
    tuned = None
    if not args.no_autotune and not args.profile_step:
        from paper_1909_01786_amd.autotune import autotune
        (args.classes, best), table = autotune(gp, lim, device=dev, log=log)
        cth = list(best)
        tuned = [{"classes": c, "class_threads": list(t), "ms": m} for c, t, m in table]
        config = {"n": args.n, "seed": args.seed, "budget": args.budget, "W": args.W,
                  "threads": args.threads, "classes": args.classes, "class_threads": cth}
    stream = torch.cuda.Stream(device=dev)
    batch = P.Batch(gp, threads=args.threads, classes=args.classes, class_threads=cth)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        batch.bind(dev, stream=stream)
    torch.cuda.synchronize()
    t_bind = time.perf_counter() - t0
    log(f"[bench] arena {batch.device_bytes / 2**30:.2f} GiB bound in {t_bind:.1f}s")

    if args.profile_step:
        timed_steps(batch, lim, 1, 1)
        print(json.dumps({"profile_step": True, "launch_info": batch.launch_info()[0]}))
        return

    # the timed steps are replays of the captured HIP graph of the batched
    # solve; eager solves afterwards give the per-launch times (HIP events on
    # each launch's stream) for the roofline
    ms, walls = timed_steps(batch, lim, args.steps, args.warmup, graph=True)
    verd, models, stats = batch.results()
    ems, ewalls = timed_steps(batch, lim, max(1, args.eager_steps), 0)
    info, order = batch.launch_info()
    everd, _, estats = batch.results()
    same_eager = bool(np.array_equal(everd, verd) and all(
        int(a["trace_hash"]) == int(b["trace_hash"]) and int(a["literal_checks"]) ==
        int(b["literal_checks"]) for a, b in zip(estats, stats)))
    checks = sum(int(s["literal_checks"]) for s in stats)
    visits = sum(int(s["visits"]) for s in stats)
    props = sum(int(s["propagations"]) for s in stats)
    n_sat = int((verd == 1).sum())
    n_unsat = int((verd == 2).sum())
    n_unknown = int((verd == 3).sum())
    n_err = int((verd < 0).sum())
    ms_step = float(np.sum(walls)) * 1000.0 / args.steps

    # every instance against the oracle's stored run of this batch
    rows = golden_rows("plain", args.n, args.seed, args.budget, args.W, args.cap_ng, args.cap_lits)
    oracle_check = check_against_oracle(
        rows, verd, [[models[i]] if verd[i] == 1 else [] for i in range(args.n)], stats)

    # algorithmic bytes: per visit 4 B map entry + 8 B nogood offsets + 4 B
    # per literal; per propagation the Deps words of the winner's other
    # variables (counted by the oracle, identical counters) read and one
    # written, 8 B each, plus 3 B value/level and 4 B trail
    def deps_bytes(members):
        if rows is None:
            return None
        return sum(8 * (rows[i]["deps_reads"] + args.W * int(stats[i]["propagations"])) +
                   7 * int(stats[i]["propagations"]) for i in members)

    def visit_bytes(members):
        return sum(12 * int(stats[i]["visits"]) + 4 * int(stats[i]["literal_checks"])
                   for i in members)

    # dominant launch: the LDS class whose eager launch ran longest
    dom = int(np.argmax([c[3] for c in info]))
    first, count, thr, dom_ms = info[dom]
    members = [int(i) for i in order[first:first + count]]
    vb = visit_bytes(members)
    db = deps_bytes(members)
    dom_bytes = vb + (db or 0)
    achieved = dom_bytes / (dom_ms / 1000.0) / 1e9
    tb = traffic_for(config, dom)
    tl = tail(stats)
    split_all, split_dom = time_split(stats), time_split(stats, members)
    log(f"[bench] launches (first, count, threads, ms): {info}; instance time ms {tl}")
    log(f"[bench] time split, all instances: {split_all}")
    log(f"[bench] time split, dominant launch: {split_dom}")
    all_members = list(range(args.n))
    step_vb, step_db = visit_bytes(all_members), deps_bytes(all_members)

    line = {
        "metric": METRIC,
        "value": checks / (ms_step / 1000.0),
        "unit": "literal checks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": f"batched plain Decision: {args.n} random ground normal programs "
                        f"(atoms log-uniform 100..5000, rules/atoms 2..4, bodies 1..4, 50% negative), "
                        f"conflict budget {args.budget}, W={args.W}",
            "instances": args.n, "nogood_literals": n_lits, "threads_per_wg": args.threads,
            "class_threads": [c[2] for c in info], "lds_classes": args.classes,
            "budget_conflicts": args.budget,
            "schedule": "autotuned" if tuned else "given",
            "timing": "HIP-graph replays of the batched solve (asp_solve_batch_graph), "
                      "inputs resident in HBM",
        },
        "instances_per_s": (n_sat + n_unsat) / (ms_step / 1000.0),
        "verdicts": {"sat": n_sat, "unsat": n_unsat, "unknown": n_unknown, "error": n_err},
        "decided_fraction": (n_sat + n_unsat) / args.n,
        "oracle_verified": oracle_check,
        "literal_checks_per_step": checks,
        "visits_per_step": visits,
        "propagations_per_step": props,
        "algorithmic_bytes_per_step": {"visits": step_vb, "deps": step_db,
                                       "deps_note": "Deps words read for each implied variable "
                                                    "(winner length - 1, W words) and written, "
                                                    "plus value/level/trail bytes"},
        "graph_ms": {"median": float(np.median(ms)), "mean": float(np.mean(ms)),
                     "min": float(np.min(ms)), "max": float(np.max(ms))},
        "eager_ms_per_step": float(np.mean(ems)),
        "eager_same_results_as_graph": same_eager,
        "launch_ms": [c[3] for c in info],
        "instance_ms": tl,
        "time_split": {"all": split_all, "dominant_launch": split_dom},
        "per_class": [{"instances": c[1], "threads": c[2], "launch_ms": c[3],
                       "instance_ms": tail([stats[int(i)] for i in order[c[0]:c[0] + c[1]]]),
                       "us_per_round": time_split(stats, [int(i) for i in order[c[0]:c[0] + c[1]]])["us_per_round"],
                       "rounds_per_instance": time_split(stats, [int(i) for i in order[c[0]:c[0] + c[1]]])["rounds_per_instance"]}
                      for c in info],
        "counters": search_counters(stats, ms_step),
        "host_encode_s": t_enc, "bind_s": t_bind,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": tb,
                     "launch": f"LDS class {dom}: {count} instances, {thr} threads, "
                               f"{dom_ms:.1f} ms (eager launch), {dom_bytes} algorithmic bytes "
                               f"({vb} visits + {db} Deps)"},
    }
    n_sat_checked, bad = verify_models(progs, verd, models)
    line["models_verified"] = {"sat": n_sat_checked, "not_stable": len(bad)}
    if tuned:
        line["autotune"] = tuned

    if not args.no_res:
        log("[bench] Res-learning leg")
        line["res"] = res_leg(args, P, progs, verd, stream, dev, lim, ms_step, cth)
    if not args.no_heur:
        log("[bench] Jeroslow-Wang and activity Decision legs")
        line["heuristics"] = heur_leg(args, P, progs, verd, stream, dev, lim, ms_step, cth)
    if not args.no_multi:
        log("[bench] several-conflicts-per-step leg")
        line["multi_learning"] = multi_leg(args, P, progs, verd, stream, dev, lim, ms_step, cth)
    if not args.no_lookahead:
        log("[bench] lookahead-Decision leg")
        line["lookahead"] = lookahead_leg(args, P, progs, verd, stream, dev, lim, ms_step, cth)
    if not args.no_enum:
        log("[bench] several-answer-sets leg")
        line["enum"] = enum_leg(args, P, progs, verd, stream, dev, lim, cth)
    if not args.no_learned:
        log("[bench] learned Decision leg")
        line["learned"] = learned_leg(args, P, progs, verd, stream, dev, lim, ms_step, cth)
    del batch
    torch.cuda.empty_cache()
    if not args.no_budget_leg:
        log(f"[bench] budget {args.big_budget} leg")
        line["budget_leg"] = budget_leg(args, P, progs, stream, dev, cth)
    if not args.no_hc:
        log("[bench] Hamiltonian-cycle batch legs")
        line["hamiltonian"] = hc_leg(args, P, stream, dev, cth)
    if not args.no_single:
        log("[bench] single-instance legs")
        line["single"] = single_legs(args, P, stream, dev)
    if not args.no_cpu_baseline:
        log("[bench] oracle baseline on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(progs, args.W, args.budget, args.cap_ng,
                                            args.cap_lits, args.cpu_seconds, stats)
    print(json.dumps(line), flush=True)


def res_leg(args, P, progs, fwd_verd, stream, dev, lim, fwd_ms_step, cth):
    """The same batch, budget and schedule with Res-learning (Alg. 3) in
    place of Fwd-learning."""
    import torch
    gp = load_programs(progs, args.W, args.cap_ng, args.cap_lits, learning=P.LEARN_RES)
    batch = P.Batch(gp, threads=args.threads, classes=args.classes, class_threads=cth)
    with torch.cuda.stream(stream):
        batch.bind(dev, stream=stream)
    torch.cuda.synchronize()
    ms, walls = timed_steps(batch, lim, args.res_steps, 1)
    verd, models, stats = batch.results()
    n_sat = int((verd == 1).sum())
    n_unsat = int((verd == 2).sum())
    ms_step = float(np.sum(walls)) * 1000.0 / len(walls)
    contra = int(((verd == 1) & (fwd_verd == 2)).sum() + ((verd == 2) & (fwd_verd == 1)).sum())
    n_sat_checked, bad = verify_models(progs, verd, models)
    ips = (n_sat + n_unsat) / (ms_step / 1000.0)
    fwd_ips = int(((fwd_verd == 1) | (fwd_verd == 2)).sum()) / (fwd_ms_step / 1000.0)
    out = {
        "ms_per_step": ms_step, "instances_per_s": ips,
        "vs_fwd_instances_per_s": ips / fwd_ips if fwd_ips > 0 else None,
        "verdicts": {"sat": n_sat, "unsat": n_unsat, "unknown": int((verd == 3).sum()),
                     "error": int((verd < 0).sum())},
        "verdict_contradictions_vs_fwd": contra,
        "models_verified": {"sat": n_sat_checked, "not_stable": len(bad)},
        "literal_checks_per_s": sum(int(s["literal_checks"]) for s in stats) / (ms_step / 1000.0),
        "counters": search_counters(stats, ms_step),
        "time_split": time_split(stats),
        "instance_ms": tail(stats),
    }
    del batch
    torch.cuda.empty_cache()
    return out


def heur_leg(args, P, progs, plain_verd, stream, dev, lim, plain_ms_step, cth):
    """The same batch, budget and schedule with the Jeroslow-Wang and the
    activity Decision scores in place of occurrence counts."""
    import torch
    plain_ips = int(((plain_verd == 1) | (plain_verd == 2)).sum()) / (plain_ms_step / 1000.0)
    out = {}
    for name, dec in (("jw", P.DECISION_JW), ("activity", P.DECISION_ACTIVITY)):
        gp = load_programs(progs, args.W, args.cap_ng, args.cap_lits, decision=dec)
        batch = P.Batch(gp, threads=args.threads, classes=args.classes, class_threads=cth)
        with torch.cuda.stream(stream):
            batch.bind(dev, stream=stream)
        torch.cuda.synchronize()
        ms, walls = timed_steps(batch, lim, 1, 1)
        verd, models, stats = batch.results()
        ms_step = float(np.sum(walls)) * 1000.0 / len(walls)
        n_sat, n_unsat = int((verd == 1).sum()), int((verd == 2).sum())
        n_sat_checked, bad = verify_models(progs, verd, models)
        ips = (n_sat + n_unsat) / (ms_step / 1000.0)
        out[name] = {
            "ms_per_step": ms_step, "instances_per_s": ips,
            "vs_occurrence_instances_per_s": ips / plain_ips if plain_ips > 0 else None,
            "verdicts": {"sat": n_sat, "unsat": n_unsat, "unknown": int((verd == 3).sum()),
                         "error": int((verd < 0).sum())},
            "verdict_contradictions_vs_occurrence": int(
                ((verd == 1) & (plain_verd == 2)).sum() + ((verd == 2) & (plain_verd == 1)).sum()),
            "models_verified": {"sat": n_sat_checked, "not_stable": len(bad)},
            "oracle_verified": check_against_oracle(
                golden_rows(name, args.n, args.seed, args.budget, args.W, args.cap_ng,
                            args.cap_lits),
                verd, [[models[i]] if verd[i] == 1 else [] for i in range(len(verd))], stats),
            "literal_checks_per_s": sum(int(s["literal_checks"]) for s in stats) / (ms_step / 1000.0),
            "counters": search_counters(stats, ms_step),
        }
        del batch
        torch.cuda.empty_cache()
    return out


def multi_leg(args, P, progs, plain_verd, stream, dev, lim, plain_ms_step, cth):
    """The same batch, budget and schedule learning up to --multi-k of each
    round's conflicts per Learning step."""
    import torch
    gp = load_programs(progs, args.W, args.cap_ng, args.cap_lits, learn_conflicts=args.multi_k)
    batch = P.Batch(gp, threads=args.threads, classes=args.classes, class_threads=cth)
    with torch.cuda.stream(stream):
        batch.bind(dev, stream=stream)
    torch.cuda.synchronize()
    ms, walls = timed_steps(batch, lim, 1, 1)
    verd, models, stats = batch.results()
    ms_step = float(np.sum(walls)) * 1000.0 / len(walls)
    n_sat, n_unsat = int((verd == 1).sum()), int((verd == 2).sum())
    n_sat_checked, bad = verify_models(progs, verd, models)
    ips = (n_sat + n_unsat) / (ms_step / 1000.0)
    plain_ips = int(((plain_verd == 1) | (plain_verd == 2)).sum()) / (plain_ms_step / 1000.0)
    out = {
        "learn_conflicts": args.multi_k, "ms_per_step": ms_step, "instances_per_s": ips,
        "vs_one_conflict_instances_per_s": ips / plain_ips if plain_ips > 0 else None,
        "verdicts": {"sat": n_sat, "unsat": n_unsat, "unknown": int((verd == 3).sum()),
                     "error": int((verd < 0).sum())},
        "verdict_contradictions_vs_one_conflict": int(
            ((verd == 1) & (plain_verd == 2)).sum() + ((verd == 2) & (plain_verd == 1)).sum()),
        "models_verified": {"sat": n_sat_checked, "not_stable": len(bad)},
        "oracle_verified": check_against_oracle(
            golden_rows(f"multi{args.multi_k}", args.n, args.seed, args.budget, args.W,
                        args.cap_ng, args.cap_lits),
            verd, [[models[i]] if verd[i] == 1 else [] for i in range(len(verd))], stats),
        "counters": search_counters(stats, ms_step),
        "time_split": time_split(stats),
    }
    del batch
    torch.cuda.empty_cache()
    return out


def lookahead_leg(args, P, progs, plain_verd, stream, dev, lim, plain_ms_step, cth):
    """The same batch, budget and schedule with the lookahead Decision
    (--lookahead candidates tried by propagation at each Decision)."""
    import torch
    k = args.lookahead
    gp = load_programs(progs, args.W, args.cap_ng, args.cap_lits, lookahead=k)
    batch = P.Batch(gp, threads=args.threads, classes=args.classes, class_threads=cth)
    with torch.cuda.stream(stream):
        batch.bind(dev, stream=stream)
    torch.cuda.synchronize()
    ms, walls = timed_steps(batch, lim, 1, 1)
    verd, models, stats = batch.results()
    ms_step = float(np.sum(walls)) * 1000.0 / len(walls)
    n_sat, n_unsat = int((verd == 1).sum()), int((verd == 2).sum())
    n_sat_checked, bad = verify_models(progs, verd, models)
    ips = (n_sat + n_unsat) / (ms_step / 1000.0)
    plain_ips = int(((plain_verd == 1) | (plain_verd == 2)).sum()) / (plain_ms_step / 1000.0)
    out = {
        "lookahead": k, "ms_per_step": ms_step, "instances_per_s": ips,
        "vs_plain_instances_per_s": ips / plain_ips if plain_ips > 0 else None,
        "verdicts": {"sat": n_sat, "unsat": n_unsat, "unknown": int((verd == 3).sum()),
                     "error": int((verd < 0).sum())},
        "verdict_contradictions_vs_plain": int(
            ((verd == 1) & (plain_verd == 2)).sum() + ((verd == 2) & (plain_verd == 1)).sum()),
        "models_verified": {"sat": n_sat_checked, "not_stable": len(bad)},
        "oracle_verified": check_against_oracle(
            golden_rows(f"look{k}", args.n, args.seed, args.budget, args.W, args.cap_ng,
                        args.cap_lits),
            verd, [[models[i]] if verd[i] == 1 else [] for i in range(len(verd))], stats),
        "counters": search_counters(stats, ms_step),
        "time_split": time_split(stats),
    }
    del batch
    torch.cuda.empty_cache()
    return out


def enum_leg(args, P, progs, plain_verd, stream, dev, lim, cth):
    """The same batch, budget and schedule asking for up to --enum-models
    answer sets per program (blocking nogood and restart after each)."""
    import torch
    k = args.enum_models
    gp = load_programs(progs, args.W, args.cap_ng, args.cap_lits, max_models=k)
    batch = P.Batch(gp, threads=args.threads, classes=args.classes, class_threads=cth)
    with torch.cuda.stream(stream):
        batch.bind(dev, stream=stream)
    torch.cuda.synchronize()
    ms, walls = timed_steps(batch, lim, 1, 1)
    verd, models, stats = batch.results(all_models=True)
    ms_step = float(np.sum(walls)) * 1000.0 / len(walls)
    found = np.array([int(s["models"]) for s in stats])
    exhausted = np.array([int(s["exhausted"]) for s in stats])
    contra = int(((found > 0) & (plain_verd == 2)).sum() + ((found == 0) & (plain_verd == 1)).sum())
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from brute import is_stable
    n_checked = bad = dup = 0
    for i in np.nonzero(found > 0)[0]:
        ms_i = models[i]
        dup += len(ms_i) - len({m.tobytes() for m in ms_i})
        for m in ms_i:
            n_checked += 1
            bad += 0 if is_stable(progs[i], m) else 1
    out = {
        "max_models": k, "ms_per_step": ms_step,
        "answer_sets_per_s": float(found.sum()) / (ms_step / 1000.0),
        "answer_sets": int(found.sum()),
        "instances_with_answer_sets": int((found > 0).sum()),
        "instances_at_max_models": int((found >= k).sum()),
        "instances_exhausted": int(exhausted.sum()),
        "unsat": int((verd == 2).sum()), "unknown": int((verd == 3).sum()),
        "error": int((verd < 0).sum()),
        "restarts": int(sum(int(s["restarts"]) for s in stats)),
        "verdict_contradictions_vs_plain": contra,
        "answer_sets_verified": {"checked": n_checked, "not_stable": bad, "duplicates": dup},
        "oracle_verified": check_against_oracle(
            golden_rows(f"enum{k}", args.n, args.seed, args.budget, args.W, args.cap_ng,
                        args.cap_lits), verd, models, stats, enum=True),
        "counters": search_counters(stats, ms_step),
        "instance_ms": tail(stats),
    }
    del batch
    torch.cuda.empty_cache()
    return out


def learned_leg(args, P, progs, plain_verd, stream, dev, lim, plain_ms_step, cth):
    import torch
    import aspgen
    from paper_1909_01786_amd import binding as B
    wpath = args.weights or B.WEIGHTS_PATH
    if os.path.exists(wpath):
        w, src = B.load_weights(wpath), "trained (" + os.path.relpath(wpath, ROOT) + ")"
    else:
        w, src = aspgen.mpnn_weights(0), "untrained seeded weights (no trained file)"
    gp = load_programs(progs, args.W, args.cap_ng, args.cap_lits, decision=P.DECISION_SCORE,
                       fallback_after=10)
    batch = P.Batch(gp, threads=args.threads, classes=args.classes, class_threads=cth)
    with torch.cuda.stream(stream):
        batch.bind(dev, stream=stream)
        ws = batch.scorer_workspace(dev)
    torch.cuda.synchronize()
    packed = P.scorer_weights(w)
    ms, walls = timed_steps(batch, lim, args.learned_steps, 1, before=lambda: batch.score(packed, ws))
    # the scorer alone (all instances), between device synchronisations
    sc_ms = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.score(packed, ws)
        torch.cuda.synchronize()
        sc_ms.append((time.perf_counter() - t0) * 1e3)
    verd, models, stats = batch.results()
    n_sat = int((verd == 1).sum())
    n_unsat = int((verd == 2).sum())
    ms_step = float(np.sum(walls)) * 1000.0 / len(walls)
    contra = int(((verd == 1) & (plain_verd == 2)).sum() + ((verd == 2) & (plain_verd == 1)).sum())
    n_sat_checked, bad = verify_models(progs, verd, models)
    ips = (n_sat + n_unsat) / (ms_step / 1000.0)
    plain_ips = int(((plain_verd == 1) | (plain_verd == 2)).sum()) / (plain_ms_step / 1000.0)
    return {
        "weights": src, "ms_per_step": ms_step, "scorer_ms": float(np.median(sc_ms)),
        "instances_per_s": ips,
        "vs_plain_instances_per_s": ips / plain_ips if plain_ips > 0 else None,
        "verdicts": {"sat": n_sat, "unsat": n_unsat, "unknown": int((verd == 3).sum()),
                     "error": int((verd < 0).sum())},
        "verdict_contradictions_vs_plain": contra,
        "models_verified": {"sat": n_sat_checked, "not_stable": len(bad)},
        "literal_checks_per_s": sum(int(s["literal_checks"]) for s in stats) / (ms_step / 1000.0),
        "instance_ms": tail(stats),
    }



def budget_leg(args, P, progs, stream, dev, cth):
    """The same batch at a ten times larger conflict budget (learned store
    grown to match): the decided fraction and instances/s, for the
    occurrence Decision and for activity with restarts."""
    import torch
    b = args.big_budget
    cap_ng, cap_lits = max(args.cap_ng, b + 64), 1 << 20
    lim = P.limits(b, max(args.max_ms, 240000))
    out = {"budget_conflicts": b, "learned_cap": [cap_ng, cap_lits]}
    variants = [("occurrence", {})]
    if args.budget_restarts:
        variants.append(("activity_restarts",
                         {"decision": P.DECISION_ACTIVITY, "restart_every": 512}))
    for name, kw in variants:
        gp = load_programs(progs, args.W, cap_ng, cap_lits, **kw)
        batch = P.Batch(gp, threads=args.threads, classes=args.classes, class_threads=cth)
        with torch.cuda.stream(stream):
            batch.bind(dev, stream=stream)
        torch.cuda.synchronize()
        ms, walls = timed_steps(batch, lim, 1, 0)
        verd, models, stats = batch.results()
        n_dec = int(((verd == 1) | (verd == 2)).sum())
        n_sat_checked, bad = verify_models(progs, verd, models)
        sec = float(np.sum(walls))
        out[name] = {
            "ms_per_step": sec * 1000.0, "instances_per_s": n_dec / sec,
            "decided_fraction": n_dec / len(progs),
            "verdicts": {"sat": int((verd == 1).sum()), "unsat": int((verd == 2).sum()),
                         "unknown": int((verd == 3).sum()), "error": int((verd < 0).sum())},
            "models_verified": {"sat": n_sat_checked, "not_stable": len(bad)},
            "literal_checks_per_s": sum(int(s["literal_checks"]) for s in stats) / sec,
            "instance_ms": tail(stats),
        }
        if name == "activity_restarts":
            out[name]["restart_every"] = 512
        del batch
        torch.cuda.empty_cache()
    return out


def hc_leg(args, P, stream, dev, cth, n=512, seed=4000, steps=3):
    """The 512 Hamiltonian-cycle programs (n uniform 60..200 vertices,
    out-degree 3..6, recursive reachability: non-tight) as one batch, plain
    and with the learned Decision; a stratified oracle sample checks the
    plain verdicts and counters."""
    import torch
    import aspgen
    import oracle
    from paper_1909_01786_amd import binding as B
    progs = [aspgen.batch_hamiltonian(i, batch_seed=seed) for i in range(n)]
    lim = P.limits(args.budget, args.max_ms)
    out = {"instances": n, "budget_conflicts": args.budget}
    res = {}
    for name in ("plain", "learned"):
        kw = {} if name == "plain" else {"decision": P.DECISION_SCORE, "fallback_after": 10}
        gp = load_programs(progs, args.W, args.cap_ng, args.cap_lits, **kw)
        batch = P.Batch(gp, threads=args.threads, classes=args.classes, class_threads=cth)
        with torch.cuda.stream(stream):
            batch.bind(dev, stream=stream)
        torch.cuda.synchronize()
        before = None
        if name == "learned":
            wpath = args.weights or B.WEIGHTS_PATH
            w = B.load_weights(wpath) if os.path.exists(wpath) else aspgen.mpnn_weights(0)
            packed = P.scorer_weights(w)
            ws = batch.scorer_workspace(dev)
            before = lambda: batch.score(packed, ws)   # noqa: E731
        ms, walls = timed_steps(batch, lim, steps, 1, before=before)
        verd, models, stats = batch.results()
        sec = float(np.sum(walls)) / len(walls)
        n_dec = int(((verd == 1) | (verd == 2)).sum())
        n_sat_checked, bad = verify_models(progs, verd, models)
        info, _ = batch.launch_info()
        res[name] = (verd, stats)
        out[name] = {
            "ms_per_step": sec * 1000.0, "instances_per_s": n_dec / sec,
            "decided_fraction": n_dec / n,
            "verdicts": {"sat": int((verd == 1).sum()), "unsat": int((verd == 2).sum()),
                         "unknown": int((verd == 3).sum()), "error": int((verd < 0).sum())},
            "models_verified": {"sat": n_sat_checked, "not_stable": len(bad)},
            "literal_checks_per_s": sum(int(s["literal_checks"]) for s in stats) / sec,
            "launch_ms": [c[3] for c in info],
            "time_split": time_split(stats),
            "gate_failures": sum(int(s["gate_failures"]) for s in stats),
        }
        del batch
        torch.cuda.empty_cache()
    pv, ps = res["plain"]
    lv, _ = res["learned"]
    out["learned"]["vs_plain_instances_per_s"] = (
        out["learned"]["instances_per_s"] / out["plain"]["instances_per_s"]
        if out["plain"]["instances_per_s"] > 0 else None)
    out["learned"]["verdict_contradictions_vs_plain"] = int(
        ((lv == 1) & (pv == 2)).sum() + ((lv == 2) & (pv == 1)).sum())
    # oracle on a sample: every 16th program
    cores = max(1, min(16, host_cpu()["usable"]))
    olim = oracle.make_limits(args.budget, args.cap_ng, args.cap_lits)
    pick = list(range(0, n, 16))
    with ThreadPoolExecutor(cores) as ex:
        ores = list(ex.map(lambda i: (i, *oracle.solve(progs[i], W=args.W, limits=olim)), pick))
    same = sum(1 for i, rc, _, st in ores if rc == pv[i] and all(
        (int(ps[i][k]) & (2 ** 64 - 1)) == (int(st[k]) & (2 ** 64 - 1)) for k in _ORACLE_KEYS))
    out["plain"]["oracle_sample"] = {"checked": len(pick), "identical": same,
                                     "sample": "every 16th program"}
    return out


def single_legs(args, P, stream, dev):
    """Single instances on asp_solve (one workgroup): the 200-atom random
    programs (seeds 1000..1099) and the 3-colourings of G(2000, 4.2/1999)
    (seeds 2000..2009).  Device time per solve (the kernel's own clock),
    microseconds per round, literal checks per second; every result is
    compared with the oracle's."""
    import torch
    import aspgen
    import oracle
    cores = max(1, min(16, host_cpu()["usable"]))
    out = {}
    for name, gen, seeds, budget in (
            ("random_200x600", aspgen.single_random, range(1000, 1100), -1),
            ("coloring_2000", aspgen.gnp_coloring, range(2000, 2010), 2000)):
        progs = [gen(s) for s in seeds]
        lim = P.limits(budget, args.max_ms)
        rows = []
        for k, prog in enumerate(progs):
            g = P.Program(prog, W=args.W, learned_cap_ng=1 << 16, learned_cap_lits=1 << 22)
            with torch.cuda.stream(stream):
                g.bind(dev, threads=256, stream=stream)
            if k == 0:
                g.solve(lim)                     # first launch loads the code object
            t0 = time.perf_counter()
            rc, m, st = g.solve(lim)
            rows.append((rc, m, st, time.perf_counter() - t0))
            del g
        olim = oracle.make_limits(budget, 1 << 16, 1 << 22)
        with ThreadPoolExecutor(cores) as ex:
            ores = list(ex.map(lambda p: oracle.solve(p, W=args.W, limits=olim), progs))
        ident = 0
        for (rc, m, st, _), (orc, om, ost) in zip(rows, ores):
            ok = rc == orc and all((int(st[k]) & (2 ** 64 - 1)) == (int(ost[k]) & (2 ** 64 - 1))
                                   for k in _ORACLE_KEYS)
            if ok and orc == 1:
                ok = np.array_equal(m, om)
            ident += int(ok)
        ns = np.array([r[2]["ns_total"] for r in rows], np.float64)
        rounds = np.array([r[2]["rounds"] for r in rows], np.float64)
        chk = np.array([r[2]["literal_checks"] for r in rows], np.float64)
        visits = np.array([r[2]["visits"] for r in rows], np.float64)
        ns_round = np.array([r[2]["ns_round"] for r in rows], np.float64)
        verds = [r[0] for r in rows]
        out[name] = {
            "instances": len(progs), "seeds": [seeds[0], seeds[-1]],
            "budget_conflicts": budget,
            "verdicts": {"sat": verds.count(1), "unsat": verds.count(2),
                         "unknown": verds.count(3)},
            "median_ms_to_solution": float(np.median(ns)) / 1e6,
            "median_wall_ms": float(np.median([r[3] for r in rows])) * 1e3,
            "us_per_round": float(ns_round.sum() / max(rounds.sum(), 1)) / 1e3,
            "visits_per_round": float(visits.sum() / max(rounds.sum(), 1)),
            "rounds_median": float(np.median(rounds)),
            "literal_checks_per_s": float(chk.sum() / max(ns.sum(), 1) * 1e9),
            "oracle_identical": ident,
            "threads": 256,
        }
    return out

if __name__ == "__main__":
    main()
