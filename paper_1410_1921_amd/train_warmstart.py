"""Train the warm-start U-Net on solutions of the solver itself, then compare solves
from rest with warm-started solves on held-out geometries.

    python -m paper_1410_1921_amd.train_warmstart --train 400 --epochs 25 \\
        --out paper_1410_1921_amd/weights/unet_warmstart.npz --eval 50 --eval-json eval.json

Training targets are the converged (u, rho - 1, C) of the flow and Knudsen solves from
rest (residual --tol); the held-out comparison runs both forms to residual 1e-7.
"""
import argparse
import json
import os
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=400, help="training geometries (seeds 5000+)")
    ap.add_argument("--epochs", type=int, default=25)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-6, help="residual of the training targets")
    ap.add_argument("--workers", type=int, default=16, help="concurrent solves for the data")
    ap.add_argument("--seed", type=int, default=0, help="weight initialisation")
    ap.add_argument("--out", default=None, help="weights file (.npz)")
    ap.add_argument("--load", default=None, help="start from these weights, skip training")
    ap.add_argument("--finetune", action="store_true",
                    help="train further from the --load weights instead of skipping training")
    ap.add_argument("--first-seed", type=int, default=0, help="index of the first training seed")
    ap.add_argument("--steady", action="store_true",
                    help="targets solved to the steady-state rule (residual 1e-7, flow distance "
                         "1e-3, Knudsen flux spread 5e-4); geometries that miss it are left out")
    ap.add_argument("--kn-cap", type=int, default=None, help="Knudsen step cap of the targets")
    ap.add_argument("--eval", type=int, default=0, help="held-out geometries (seeds 6000+)")
    ap.add_argument("--eval-json", default=None)
    args = ap.parse_args()

    import torch
    from paper_1410_1921_amd import lbm, warmstart as WS, workloads as W
    from paper_1410_1921_amd.unet import UNet

    def log(*a):
        print("[warmstart]", *a, flush=True)

    torch.cuda.set_device(0)
    lbm.load()
    cfg = W.WARMSTART
    report = {"config": {"edge": cfg["edge"], "train": args.train, "epochs": args.epochs,
                         "lr": args.lr, "tol_targets": args.tol}}
    if args.load and not args.finetune:
        net = UNet.load(args.load)
    else:
        net = UNet.load(args.load) if args.load else UNet(n_out=WS.N_OUT, seed=args.seed)
        seeds = list(cfg["train_seeds"])[args.first_seed:args.first_seed + args.train]
        t0 = time.perf_counter()
        if args.steady:
            data = WS.make_dataset(seeds, cfg, tol=1e-7, workers=args.workers, log=log,
                                   steady=(1e-3, 5e-4), kn_cap=args.kn_cap)
        else:
            data = WS.make_dataset(seeds, cfg, tol=args.tol, workers=args.workers, log=log,
                                   kn_cap=args.kn_cap)
        report["samples"] = len(data)
        report["data_s"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        report["loss"] = WS.train(net, data, args.epochs, lr=args.lr, log=log)
        report["train_s"] = time.perf_counter() - t0
        del data
        torch.cuda.empty_cache()
        if args.out:
            os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
            net.save(args.out)
            log("weights ->", args.out)
    if args.eval:
        rows = WS.evaluate(net, list(cfg["test_seeds"])[:args.eval], cfg, log=log)
        report["eval"] = rows
        report["summary"] = WS.summary(rows)
        log("summary", json.dumps(report["summary"]))
    if args.eval_json:
        with open(args.eval_json, "w") as f:
            json.dump(report, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
