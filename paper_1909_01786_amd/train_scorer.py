"""Train the learned Decision's scorer on the device and store its weights.

Training data are decision and conflict traces of the plain solver on
programs drawn like the benchmark batches (uniform random normal programs
and Hamiltonian-cycle programs) from held-out seeds.  The plain batched
search (occurrence Decision, Fwd-learning) solves them under a conflict
budget; its learned nogoods -- each the decision literals T b_r its conflict
depended on -- are read back (asp_batch_learned).  Every atom that heads a
rule is labelled:
  * in a program with an answer set: 1 if true in the answer set found,
    else 0 (deciding it true leads towards that answer set);
  * otherwise: 1 if the decisions on its rules took part in at least the
    q-quantile of conflicts among the program's rule heads (and in at
    least one), else 0 (deciding the most conflict-prone atoms first).
Atoms heading no rule are never decided and get no label.  All layers are
then trained on the device (asp_scorer_train: forward and backward passes on
the matrix cores, full-batch Adam), starting from a seeded initialisation,
and the result is quantised to the integer codes the search uses
(asp_scorer_quantize).

    python -m paper_1909_01786_amd.train_scorer --n-random 512 --n-hc 256
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import aspgen  # noqa: E402
from paper_1909_01786_amd import binding as B  # noqa: E402


def trace_labels(prog, verdict, model, learned_lits, q, sat_only=False):
    """Per-atom labels of one training program from its trace (see the
    module docstring); float32 over atoms 1..A, -1 = no label.  sat_only:
    programs without an answer set get no labels."""
    A = int(prog.n_atoms)
    head = np.asarray(prog.head)
    heads = head[head != 0]                     # headed rule j -> its head
    lab = np.full(A, -1.0, np.float32)
    has_rule = np.zeros(A + 1, bool)
    has_rule[heads] = True
    if verdict == B.SAT:
        lab[has_rule[1:]] = model[has_rule[1:]].astype(np.float32)
        return lab, 0
    if sat_only:
        return lab, 0
    lits = np.asarray(learned_lits, np.int64)
    b = lits[lits > A]                          # decision literals T b_r
    j = (b - A - 1) // 3
    cnt = np.bincount(heads[j], minlength=A + 1).astype(np.float64) if j.size else np.zeros(A + 1)
    c = cnt[1:][has_rule[1:]]
    thr = max(1.0, float(np.quantile(c, q))) if c.size else 1.0
    lab[has_rule[1:]] = (c >= thr).astype(np.float32)
    return lab, int(j.size)


def init_params(seed: int, spread: int) -> np.ndarray:
    """Seeded starting parameters: matrices uniform in +-spread/128, biases
    small, so that the clamped units start in their linear range."""
    w = aspgen.mpnn_weights(seed, spread=spread)
    for k in ("ev", "ec", "bc", "bv"):
        w[k] = w[k] // 8
    return B.dequantize(w)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n-random", type=int, default=512)
    ap.add_argument("--n-hc", type=int, default=256)
    ap.add_argument("--seed", type=int, default=1_000_000, help="training batch seed (held out)")
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--init-spread", type=int, default=24)
    ap.add_argument("--budget", type=int, default=2000)
    ap.add_argument("--quantile", type=float, default=0.8)
    ap.add_argument("--sat-only", action="store_true",
                    help="label only programs with an answer set (answer-set atoms)")
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--out", default=B.WEIGHTS_PATH)
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("training runs on the GPU")
    t0 = time.time()
    progs = [aspgen.batch_random(i, batch_seed=args.seed) for i in range(args.n_random)]
    progs += [aspgen.batch_hamiltonian(i, batch_seed=args.seed) for i in range(args.n_hc)]
    with ThreadPoolExecutor(16) as ex:
        gp = list(ex.map(lambda p: B.Program(p, learned_cap_ng=4096, learned_cap_lits=1 << 18),
                         progs))
    b = B.Batch(gp, threads=128, classes=4).bind("cuda")
    b.solve(B.limits(args.budget, 300000))
    verd, models, stats = b.results()
    print(f"[train] solved {len(progs)} training programs in {time.time() - t0:.1f}s: "
          f"sat {(verd == B.SAT).sum()} unsat {(verd == B.UNSAT).sum()} "
          f"unknown {(verd == B.UNKNOWN).sum()}", flush=True)
    labels, n_dec_lits = [], 0
    for i, p in enumerate(progs):
        _, lits = b.learned(i)
        lab, nd = trace_labels(p, int(verd[i]), models[i], lits, args.quantile, args.sat_only)
        labels.append(lab)
        n_dec_lits += nd
    n_conf = int(sum(int(s["conflicts"]) for s in stats))
    n_dec = int(sum(int(s["decisions"]) for s in stats))
    del b
    torch.cuda.empty_cache()
    lab_all = np.concatenate(labels)
    n_lab = int((lab_all >= 0).sum())
    print(f"[train] traces: {n_dec} decisions, {n_conf} conflicts, {n_dec_lits} decision "
          f"literals in learned nogoods; {n_lab} labelled atoms, positive rate "
          f"{float((lab_all == 1).sum()) / max(n_lab, 1):.3f}", flush=True)
    p0 = init_params(args.init_seed, args.init_spread)
    t1 = time.time()
    params, losses, _ = B.train_scorer(gp, labels, p0, steps=args.steps, lr=args.lr)
    t_train = time.time() - t1
    print(f"[train] {args.steps} Adam steps in {t_train:.1f}s: loss {losses[0]:.4f} -> "
          f"{losses[-1]:.4f}", flush=True)
    w = B.quantize(params)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    meta = {"train_seed": args.seed, "n_random": args.n_random, "n_hc": args.n_hc,
            "budget": args.budget, "quantile": args.quantile, "sat_only": args.sat_only,
            "steps": args.steps,
            "lr": args.lr, "init_seed": args.init_seed, "init_spread": args.init_spread,
            "decisions": n_dec, "conflicts": n_conf, "labelled_atoms": n_lab,
            "positive_rate": float((lab_all == 1).sum() / max(n_lab, 1)),
            "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
            "loss_every_25": [float(x) for x in losses[::25]], "train_s": t_train,
            "trained": "all layers (asp_scorer_train)"}
    np.savez(args.out, **{k: np.asarray(v) for k, v in w.items()}, meta=json.dumps(meta))
    print(json.dumps(meta), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
