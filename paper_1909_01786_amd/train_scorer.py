"""Train the learned Decision's scorer on the device and store its weights.

Training data are programs drawn like the benchmark batches (uniform random
normal programs and Hamiltonian-cycle programs) from held-out seeds.  The
plain batched search (occurrence Decision) solves them; every atom of an
instance with an answer set is labelled 1 if it is true in the answer set
found, else 0.  The message-passing matrices are a fixed seeded projection;
the readout is fitted on the device by logistic regression
(asp_batch_train_readout) and quantised to integer codes: with
k = 127 / max|w|, wo = round(k w) and bo = round(256 k b), so the integer
score is about 256 k times the logit and keeps its order.

    python -m paper_1909_01786_amd.train_scorer --n-random 1536 --n-hc 512
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


def quantise(base: dict, wb: np.ndarray) -> dict:
    w = {k: (np.array(v) if not np.isscalar(v) else v) for k, v in base.items()}
    wf = np.asarray(wb[:64], np.float64)
    bf = float(wb[64])
    k = 127.0 / max(float(np.abs(wf).max()), 1e-12)
    w["wo"] = np.clip(np.rint(wf * k), -127, 127).astype(np.int64)
    w["bo"] = int(np.clip(np.rint(256.0 * k * bf), -(1 << 24), 1 << 24))
    return w


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n-random", type=int, default=1536)
    ap.add_argument("--n-hc", type=int, default=512)
    ap.add_argument("--seed", type=int, default=1_000_000, help="training batch seed (held out)")
    ap.add_argument("--wseed", type=int, default=0, help="seed of the message-passing matrices")
    ap.add_argument("--budget", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--lr", type=float, default=0.05)
    ap.add_argument("--out", default=B.WEIGHTS_PATH)
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("training runs on the GPU")
    t0 = time.time()
    progs = [aspgen.batch_random(i, batch_seed=args.seed) for i in range(args.n_random)]
    progs += [aspgen.batch_hamiltonian(i, batch_seed=args.seed) for i in range(args.n_hc)]
    with ThreadPoolExecutor(16) as ex:
        gp = list(ex.map(lambda p: B.Program(p, learned_cap_ng=4096, learned_cap_lits=1 << 18), progs))
    b = B.Batch(gp, threads=128, classes=4).bind("cuda")
    b.solve(B.limits(args.budget, 300000))
    verd, models, _ = b.results()
    print(f"solved {len(progs)} training programs in {time.time() - t0:.1f}s: "
          f"sat {(verd == B.SAT).sum()} unsat {(verd == B.UNSAT).sum()} "
          f"unknown {(verd == B.UNKNOWN).sum()}", flush=True)
    labels = np.concatenate([m.astype(np.int8) if v == B.SAT else np.full(len(m), -1, np.int8)
                             for v, m in zip(verd, models)])
    n_lab = int((labels >= 0).sum())
    base = aspgen.mpnn_weights(args.wseed)
    wb, loss = b.train_readout(base, labels, steps=args.steps, lr=args.lr)
    w = quantise(base, wb)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    meta = {"train_seed": args.seed, "n_random": args.n_random, "n_hc": args.n_hc,
            "wseed": args.wseed, "budget": args.budget, "steps": args.steps, "lr": args.lr,
            "labelled_atoms": n_lab, "positive_rate": float((labels == 1).sum() / max(n_lab, 1)),
            "loss_first": float(loss[0]), "loss_last": float(loss[-1])}
    np.savez(args.out, **{k: np.asarray(v) for k, v in w.items()}, meta=json.dumps(meta))
    print(json.dumps(meta), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
