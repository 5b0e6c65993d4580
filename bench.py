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


def cpu_baseline(progs, W, budget, cap_ng, cap_lits, target_s, gpu_stats):
    """Oracle on a bounded random sample of the batch, one thread per core
    (the oracle's C entry releases the GIL); the sampled verdicts and
    counters are also checked against the GPU's."""
    import oracle
    oracle.build()
    n = len(progs)
    cores = max(1, min(16, os.cpu_count() or 1))
    rng = np.random.default_rng(12345)
    order = rng.permutation(n)
    # bound the sample with the GPU's own counters and a nominal oracle rate
    checks = np.array([s["literal_checks"] for s in gpu_stats], dtype=np.float64)
    budget_checks = target_s * 2.0e7 * cores
    pick, acc = [], 0.0
    for i in order:
        if acc + checks[i] > budget_checks and pick:
            continue
        pick.append(int(i))
        acc += checks[i]
        if acc > 0.8 * budget_checks or len(pick) >= 256:
            break
    lim = oracle.make_limits(budget, cap_ng, cap_lits)

    def one(i):
        return i, *oracle.solve(progs[i], W=W, limits=lim)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        res = list(ex.map(one, pick))
    wall = time.perf_counter() - t0
    tot_checks = sum(r[3]["literal_checks"] for r in res)
    mism = 0
    for i, rc, _, st in res:
        g = gpu_stats[i]
        same = all(int(g[k]) == int(st[k]) for k in
                   ("literal_checks", "visits", "conflicts", "decisions", "rounds", "trace_hash"))
        mism += int((not same) or rc != g["status"])
    return {
        "value": tot_checks / wall, "unit": "literal checks/s", "cores": cores,
        "kind": "oracle",
        "sample": f"{len(pick)} of {n} instances drawn at random from the same batch, "
                  f"same conflict budget; {tot_checks} literal checks in {wall:.1f} s wall "
                  f"on {cores} threads",
        "instances_per_s": len(pick) / wall,
        "sample_mismatches_vs_gpu": int(mism),
    }


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
        files = [f for f in os.listdir(d) if f.endswith("counter_collection.csv")]
        return os.path.join(d, files[0])
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
        "note": "per k_search dispatch of one bench step, in launch order (LDS class 0 first); "
                "scale = copied KiB / counter KiB of a plain 1 GiB device copy",
    }
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def traffic_for(config, launch_index):
    try:
        with open(TRAFFIC_JSON) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("kernel_sha") != kernel_hash() or t.get("config") != config:
        return None
    lb = t.get("launch_bytes", [])
    return lb[launch_index] if launch_index < len(lb) else None


# ------------------------------------------------------------ runs
def timed_steps(batch, lim, steps, warmup, before=None):
    import torch
    for w in range(warmup):
        if before:
            before()
        batch.solve(lim)
        torch.cuda.synchronize()
        log(f"[bench] warmup {w} {batch.last_ms():.1f} ms")
    ms, walls = [], []
    for s in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if before:
            before()
        batch.solve(lim)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        ms.append(batch.last_ms())
        log(f"[bench] step {s} kernel {ms[-1]:.1f} ms, wall {walls[-1] * 1e3:.1f} ms")
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
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=3000)
    ap.add_argument("--budget", type=int, default=2000, help="conflicts per instance")
    ap.add_argument("--W", type=int, default=1)
    ap.add_argument("--threads", type=int, default=128)
    ap.add_argument("--classes", type=int, default=4, help="LDS size classes (launches)")
    ap.add_argument("--class-threads", default="256,128,128,128", help="threads per class, largest first")
    ap.add_argument("--cap-ng", type=int, default=4096)
    ap.add_argument("--cap-lits", type=int, default=1 << 18)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--max-ms", type=int, default=150000, help="device time guard per launch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-steps", type=int, default=2)
    ap.add_argument("--no-res", action="store_true", help="skip the Res-learning leg")
    ap.add_argument("--no-enum", action="store_true", help="skip the several-answer-sets leg")
    ap.add_argument("--no-heur", action="store_true",
                    help="skip the Jeroslow-Wang and activity Decision legs")
    ap.add_argument("--no-multi", action="store_true",
                    help="skip the several-conflicts-per-step leg")
    ap.add_argument("--multi-k", type=int, default=4, help="conflicts learned per step")
    ap.add_argument("--enum-models", type=int, default=16, help="answer sets asked per program")
    ap.add_argument("--res-steps", type=int, default=2)
    ap.add_argument("--graph-steps", type=int, default=2,
                    help="replays of the batched solve as one HIP graph, timed after the eager steps")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the schedule (LDS classes, threads per class) by timing candidates first")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--write-traffic", nargs=4, metavar="DIR",
                    help="summarise FETCH, WRITE, copy FETCH, copy WRITE counter runs")
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
    if args.autotune:
        from paper_1909_01786_amd.autotune import autotune
        (args.classes, best), table = autotune(gp, lim, device=dev, log=log)
        cth = list(best)
        tuned = [{"classes": c, "class_threads": list(t), "ms": m} for c, t, m in table]
    stream = torch.cuda.Stream(device=dev)
    batch = P.Batch(gp, threads=args.threads, classes=args.classes, class_threads=cth)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        batch.bind(dev, stream=stream)
    torch.cuda.synchronize()
    log(f"[bench] arena {batch.device_bytes / 2**30:.2f} GiB bound in {time.perf_counter() - t0:.1f}s")

    ms, walls = timed_steps(batch, lim, args.steps, args.warmup)
    info, order = batch.launch_info()
    verd, models, stats = batch.results()
    checks = sum(int(s["literal_checks"]) for s in stats)
    visits = sum(int(s["visits"]) for s in stats)
    n_sat = int((verd == 1).sum())
    n_unsat = int((verd == 2).sum())
    n_unknown = int((verd == 3).sum())
    n_err = int((verd < 0).sum())
    ms_step = float(np.sum(walls)) * 1000.0 / args.steps
    kern_ms = float(np.mean(ms))

    # dominant launch: the LDS class whose launch ran longest (last step)
    dom = int(np.argmax([c[3] for c in info]))
    first, count, thr, dom_ms = info[dom]
    members = order[first:first + count]
    dom_bytes = sum(12 * int(stats[i]["visits"]) + 4 * int(stats[i]["literal_checks"])
                    for i in members)
    achieved = dom_bytes / (dom_ms / 1000.0) / 1e9
    tb = traffic_for(config, dom)
    tl = tail(stats)
    split_all, split_dom = time_split(stats), time_split(stats, members)
    log(f"[bench] launches (first, count, threads, ms): {info}; instance time ms {tl}")
    log(f"[bench] time split, all instances: {split_all}")
    log(f"[bench] time split, dominant launch: {split_dom}")

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
        },
        "instances_per_s": (n_sat + n_unsat) / (ms_step / 1000.0),
        "verdicts": {"sat": n_sat, "unsat": n_unsat, "unknown": n_unknown, "error": n_err},
        "literal_checks_per_step": checks,
        "visits_per_step": visits,
        "kernel_ms": kern_ms,
        "launch_ms": [c[3] for c in info],
        "instance_ms": tl,
        "time_split": {"all": split_all, "dominant_launch": split_dom},
        "counters": search_counters(stats, ms_step),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": tb,
                     "launch": f"LDS class {dom}: {count} instances, {thr} threads, "
                               f"{dom_ms:.1f} ms, {dom_bytes} algorithmic bytes"},
    }
    n_sat_checked, bad = verify_models(progs, verd, models)
    line["models_verified"] = {"sat": n_sat_checked, "not_stable": len(bad)}
    if tuned:
        line["autotune"] = tuned
    if args.graph_steps > 0:
        gms = []
        for _ in range(args.graph_steps + 1):
            batch.solve(lim, graph=True)
            torch.cuda.synchronize()
            gms.append(batch.last_ms())
        gv, _, gst = batch.results()
        same = np.array_equal(gv, verd) and all(
            int(a[k]) == int(b[k]) for a, b in zip(gst, stats) for k in ("literal_checks", "trace_hash"))
        line["graph"] = {"ms_per_step": float(np.mean(gms[1:])), "replays": args.graph_steps,
                         "same_results_as_eager": bool(same)}

    if not args.no_res:
        log("[bench] Res-learning leg")
        line["res"] = res_leg(args, P, progs, verd, stream, dev, lim, ms_step, cth)
    if not args.no_heur:
        log("[bench] Jeroslow-Wang and activity Decision legs")
        line["heuristics"] = heur_leg(args, P, progs, verd, stream, dev, lim, ms_step, cth)
    if not args.no_multi:
        log("[bench] several-conflicts-per-step leg")
        line["multi_learning"] = multi_leg(args, P, progs, verd, stream, dev, lim, ms_step, cth)
    if not args.no_enum:
        log("[bench] several-answer-sets leg")
        line["enum"] = enum_leg(args, P, progs, verd, stream, dev, lim, cth)
    if not args.no_learned:
        log("[bench] learned Decision leg")
        line["learned"] = learned_leg(args, P, progs, verd, stream, dev, lim, ms_step, cth)
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
    if os.path.exists(B.WEIGHTS_PATH):
        w, src = B.load_weights(), "trained (" + os.path.relpath(B.WEIGHTS_PATH, ROOT) + ")"
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


if __name__ == "__main__":
    main()
