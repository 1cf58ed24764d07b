"""Train the U-Net warm start on solver-generated pairs and evaluate it.

Training set: 128^3 grids, box 64 Mpc/h (h = 0.5 Mpc/h, the spacing of the
512^3 / 256 Mpc/h workload), lognormal sigma_delta = 2 plus NFW haloes at the
same number density, seeds 1000..1199, a ~ U[0.5, 1]; symmetron lambda0 = 1,
a_ssb = 0.5; targets are FP64 FAS solutions to relative residual 1e-10.
Held-out set: seeds 2000..2019.  The evaluation reports, per held-out sample,
the relative residual of the prediction and the V-cycles to 1e-8 from the
prediction versus from the cold start.

The solver keeps a prediction only if it cannot cost a V-cycle (its residual
is at most what the first cold-started cycle reaches), so cycles_warm <=
cycles_cold for every sample; the evaluation also reports how many guesses
the judge kept.

Usage: python -m paper_1307_6748_amd.train_warmstart [--pairs 200] [--epochs E]
       [--out paper_1307_6748_amd/data/unet_symmetron_128.npz]
       [--checkpoint PATH [--resume]]   (training state saved after every epoch)
       [--eval-only [--weights PATH]]   (re-evaluate weights, write them to --out)
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import solver as S
from . import warmstart as W


def log(msg):
    print(f"[train {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def evaluate(net: W.WarmStart, n: int, box: float, seeds, model, tol: float = 1e-8,
             a_seed: int = 99) -> dict:
    rng = np.random.default_rng(a_seed)
    solver = S.Solver(n, box, max_cycles=100)
    rows = []
    for sd in seeds:
        a = float(rng.uniform(0.5, 1.0))
        eta = torch.from_numpy(W.training_density(n, box, sd)).cuda()
        _, cold_st = solver.solve(eta, model, a, tol)
        cold = S.cold_start(model, a, eta)
        guess = net.predict(eta, cold, a)
        r_guess = solver.residual(eta, guess, model, a)
        _, st = solver.solve(eta, model, a, tol, phi=guess, use_guess=2)
        rows.append(dict(seed=int(sd), a=a, rel_res_guess=r_guess / cold_st.r_ref,
                         rel_res_first_cold_cycle=cold_st.rel_hist[1],
                         cycles_cold=cold_st.cycles, cycles_warm=st.cycles,
                         used_guess=bool(st.used_guess)))
    saved = [r["cycles_cold"] - r["cycles_warm"] for r in rows]
    return dict(rows=rows, mean_cycles_saved=float(np.mean(saved)),
                median_rel_res_guess=float(np.median([r["rel_res_guess"] for r in rows])),
                used_guess_fraction=float(np.mean([r["used_guess"] for r in rows])))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--box", type=float, default=64.0)
    ap.add_argument("--pairs", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--heldout", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=W.DEFAULT_WEIGHTS)
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--resume", action="store_true")
    ap.add_argument("--eval-only", action="store_true")
    ap.add_argument("--weights", default=W.DEFAULT_WEIGHTS,
                    help="--eval-only: weights to evaluate (written with the new "
                         "evaluation to --out)")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    model = S.symmetron(1.0, 0.5)
    if args.eval_only:
        with np.load(args.weights, allow_pickle=False) as z:
            params = z["params"].copy()
            meta = json.loads(str(z["meta"])) if "meta" in z else {}
        net = W.WarmStart(params=params)
        ev = evaluate(net, args.n, args.box, range(2000, 2000 + args.heldout), model)
        log(f"held-out: mean V-cycles saved {ev['mean_cycles_saved']:.2f}, median rel. residual "
            f"of the guess {ev['median_rel_res_guess']:.3e}, guess used "
            f"{ev['used_guess_fraction']:.2f}")
        meta["eval"] = ev
        net.save(args.out, meta=json.dumps(meta))
        print(json.dumps(dict(mean_cycles_saved=ev["mean_cycles_saved"],
                              median_rel_res_guess=ev["median_rel_res_guess"],
                              used_guess_fraction=ev["used_guess_fraction"])), flush=True)
        return 0
    t0 = time.time()
    pairs = W.make_pairs(args.n, args.box, range(1000, 1000 + args.pairs), model, log=log)
    log(f"{len(pairs)} pairs in {time.time() - t0:.1f}s")
    trainer = None
    if args.resume and args.checkpoint:
        trainer = W.Trainer.load_checkpoint(args.checkpoint)
        net = trainer.net
        log(f"resumed at epoch {trainer.epoch}, step {trainer.k}")
    else:
        net = W.WarmStart(seed=args.seed)
    t1 = time.time()
    losses = W.train(net, pairs, args.epochs, lr=args.lr, lr_final=args.lr_final,
                     seed=args.seed, log=log, checkpoint=args.checkpoint, trainer=trainer)
    train_s = time.time() - t1
    del pairs
    ev = evaluate(net, args.n, args.box, range(2000, 2000 + args.heldout), model)
    log(f"held-out: mean V-cycles saved {ev['mean_cycles_saved']:.2f}, median rel. residual "
        f"of the guess {ev['median_rel_res_guess']:.3e}, guess used {ev['used_guess_fraction']:.2f}")
    meta = dict(n=args.n, box=args.box, pairs=args.pairs, epochs=args.epochs, lr=args.lr,
                lr_final=args.lr_final, train_seconds=train_s, losses=losses, eval=ev)
    net.save(args.out, meta=json.dumps(meta))
    print(json.dumps(dict(train_seconds=train_s, final_loss=losses[-1],
                          mean_cycles_saved=ev["mean_cycles_saved"],
                          median_rel_res_guess=ev["median_rel_res_guess"])), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
