"""Benchmark of the batched GPU search (one MI355X).

One step = one batched solve (asp_solve_batch) that runs the whole
search -- InitialPropagation, PropagateAndCheck rounds, Fwd-learning with
Backjump, Decision / CompleteAssignment and the stability check -- for every
program of a batch of uneven random ground programs (4096 programs, atoms
log-uniform in 100..5000, rules/atoms uniform in 2..4, bodies of 1..4
literals, half of them negated), under a fixed per-instance conflict budget.
Inputs are resident in HBM before the timed region; the step is timed with
HIP events recorded on the launch stream.

Metric: nogood literal checks per second (a visit of nogood d from a
propagated literal counts |d| checks), with decided instances per second
beside it.  The roofline entry prices the kernel's algorithmic HBM bytes:
per visit 4 B map entry + 8 B nogood offsets + 4 B per literal.

The oracle leg (cpu_baseline) times the plain CPU oracle on a bounded sample
of the same batch with the same budget, one thread per host core.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 4096]
"""
from __future__ import annotations

import argparse
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_batch(n: int, seed: int):
    import aspgen
    return [aspgen.batch_random(i, batch_seed=seed) for i in range(n)]


def load_programs(progs, W, cap_ng, cap_lits, workers=16):
    import paper_1909_01786_amd as P
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda p: P.Program(p, W=W, learned_cap_ng=cap_ng,
                                               learned_cap_lits=cap_lits), progs))


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
    ap.add_argument("--cap-ng", type=int, default=4096)
    ap.add_argument("--cap-lits", type=int, default=1 << 18)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--max-ms", type=int, default=150000, help="device time guard per launch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the batch would shard by instance across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    if args.copy_calibration:
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device=dev)
        b = torch.empty(n, dtype=torch.uint8, device=dev)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 3}))
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

    stream = torch.cuda.Stream(device=dev)
    batch = P.Batch(gp, threads=args.threads, classes=args.classes)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        batch.bind(dev, stream=stream)
    torch.cuda.synchronize()
    log(f"[bench] arena {batch.device_bytes / 2**30:.2f} GiB bound in {time.perf_counter() - t0:.1f}s")

    lim = P.limits(args.budget, args.max_ms)
    for w in range(args.warmup):
        batch.solve(lim)
        torch.cuda.synchronize()
        log(f"[bench] warmup {w} {batch.last_ms():.1f} ms")

    ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        batch.solve(lim)
        torch.cuda.synchronize()
        ms.append(batch.last_ms())
        log(f"[bench] step {s} kernel {ms[-1]:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    verd, models, stats = batch.results()
    checks = sum(int(s["literal_checks"]) for s in stats)
    visits = sum(int(s["visits"]) for s in stats)
    n_sat = int((verd == 1).sum())
    n_unsat = int((verd == 2).sum())
    n_unknown = int((verd == 3).sum())
    n_err = int((verd < 0).sum())
    ms_step = wall * 1000.0 / args.steps
    kern_ms = float(np.mean(ms))
    alg_bytes = 12 * visits + 4 * checks
    achieved = alg_bytes / (kern_ms / 1000.0) / 1e9

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
            "lds_classes": args.classes, "budget_conflicts": args.budget,
        },
        "instances_per_s": (n_sat + n_unsat) / (ms_step / 1000.0),
        "verdicts": {"sat": n_sat, "unsat": n_unsat, "unknown": n_unknown, "error": n_err},
        "literal_checks_per_step": checks,
        "visits_per_step": visits,
        "kernel_ms": kern_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
    }
    if not args.no_cpu_baseline:
        log("[bench] oracle baseline on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(progs, args.W, args.budget, args.cap_ng,
                                            args.cap_lits, args.cpu_seconds, stats)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
