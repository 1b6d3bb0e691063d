"""Train the learned warm start on (start, minimum) pairs that the library's
batched L-BFGS produces for synthetic chains, entirely on the GPU, and save
the network.

    python -m paper_1810_03358_amd.train_warmstart --chains 544 --out weights.npz

Chains: sizes log-uniform in [lo, hi]; chain k uses seed 200000 + k, the
compacted (globular) start of the chain generator for even seeds and the
extended one for odd seeds.  The last `--val` fraction of the chains is held
out for the validation loss.  Minima: L-BFGS m = 10, LS_PAR, FP32 pair sums,
|grad E|_inf < 1e-3 or `--max-iter` iterations.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import paper_1810_03358_amd as ff  # noqa: E402
from paper_1810_03358_amd import learn as L  # noqa: E402
from synth import batch_sizes, chain_system  # noqa: E402

TRAIN_SEED0 = 200_000
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warmstart.npz")


def log(msg):
    print(msg, flush=True)


def build_data(sizes, seed0, batch_chains, max_iter, tol, device):
    """(start features, minimum - start) rows of chains seed0 + k, k < len(sizes)."""
    data = L.Dataset(device)
    stats = []
    for b in range(0, len(sizes), batch_chains):
        t = time.time()
        systems = [chain_system(n, seed0 + b + i, compact=(seed0 + b + i) % 2 == 0)
                   for i, n in enumerate(sizes[b:b + batch_chains])]
        tg = time.time() - t
        t = time.time()
        data, res = L.make_pairs(systems, lambda ss: ff.Context(ss), tol=tol, max_iter=max_iter, precision="fp32",
                                 dataset=data, device=device)
        torch.cuda.synchronize()
        conv = sum(r["term"] == ff.FF_CONVERGED for r in res)
        stats += res
        log(f"chains {b}..{b + len(systems) - 1}: generated in {tg:.1f} s, minimized in {time.time() - t:.1f} s, "
            f"converged {conv}/{len(systems)}, iterations max {max(r['iters'] for r in res)}")
    return data.finish(), stats


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--chains", type=int, default=544)
    ap.add_argument("--lo", type=int, default=1000)
    ap.add_argument("--hi", type=int, default=5000)
    ap.add_argument("--val", type=float, default=32 / 544)
    ap.add_argument("--batch-chains", type=int, default=128)
    ap.add_argument("--max-iter", type=int, default=30000)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-final", type=float, default=2e-5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)
    dev = "cuda"
    t0 = time.time()
    sizes = batch_sizes(args.chains, args.lo, args.hi, seed=7)
    n_val = max(1, int(round(args.val * args.chains)))
    train, tstats = build_data(sizes[:-n_val], TRAIN_SEED0, args.batch_chains, args.max_iter, args.tol, dev)
    val, _ = build_data(sizes[-n_val:], TRAIN_SEED0 + args.chains - n_val, args.batch_chains, args.max_iter,
                        args.tol, dev)
    t_data = time.time() - t0
    zero_train = float(train.T.double().pow(2).mean().cpu())
    zero_val = float(val.T.double().pow(2).mean().cpu())
    log(f"rows: train {train.rows}, validation {val.rows}; loss of the zero prediction {zero_train:.4f} / "
        f"{zero_val:.4f}")
    net = L.Net(seed=args.seed, device=dev)
    t = time.time()
    losses = L.train(net, train, epochs=args.epochs, batch=args.batch, lr=args.lr, lr_final=args.lr_final,
                     seed=args.seed, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t
    vloss = L.validation_loss(net, val)
    summary = dict(chains=args.chains, validation_chains=n_val, sizes=[args.lo, args.hi], rows=train.rows,
                   validation_rows=val.rows, epochs=args.epochs, batch=args.batch, adam_steps=net.step,
                   train_loss=losses[-1], validation_loss=vloss, zero_loss_train=zero_train,
                   zero_loss_validation=zero_val, r2_validation=1.0 - vloss / zero_val,
                   converged=sum(r["term"] == ff.FF_CONVERGED for r in tstats), data_seconds=t_data,
                   train_seconds=t_train)
    log(json.dumps(summary))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.savez(args.out, theta=net.params(), summary=np.array(json.dumps(summary)))
    log(f"saved {args.out}")
    return summary


if __name__ == "__main__":
    main()
