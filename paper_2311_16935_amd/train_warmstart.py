"""Train the warm-start U-Net on solves the method generates, then compare
plain and warm-started solves on held-out fields.

    python -m paper_2311_16935_amd.train_warmstart --n 64 --count 512 \
        --steps 3000 --out paper_2311_16935_amd/weights/unet_blobs64.safetensors

Training fields are unit-cube Gaussian-blob gradient fields with 5% noise at
seeds seed_base + i; the targets are the solver's own gauge-fixed answers
(residual tolerance --tol).  Evaluation uses seeds from --eval-seed on
--eval-n^3 grids (network grid = eval-n / factor).
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import torch


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _timed_pair(plan, ws, g, P0, tol, max_iter):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = plan.solve(g, P=P0.clone(), tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    warm = ws.solve(plan, g, P=torch.empty_like(P0), tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return plain, warm, t1 - t0, t2 - t1


def evaluate(net, factor, n, seeds, tol=1e-6, device="cuda:0", max_iter=10**6):
    import synth
    from . import Plan
    from .warmstart import WarmStart

    ws = WarmStart(net, factor)
    rows = []
    plan = None
    for s in seeds:
        w = synth.config_blobs_3d(n, noise=0.05, seed=s, device=device)
        g = [t.float().contiguous() for t in w.grads]
        if plan is None:
            plan = Plan(w.dims, w.spacing)
            vplan = Plan(w.dims, w.spacing, fixed_point=True)
        P0 = torch.zeros(plan.shape, dtype=plan.dtype, device=device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain = plan.solve(g, P=P0, tol=tol, max_iter=max_iter)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P1 = torch.empty_like(P0)
        ws.guess(plan, g, P1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # error of the guess against the converged field, after the mean gauge
        guess_err = float(((P1 - P1.mean()) - plain.P).norm() / plain.P.norm())
        warm = plan.solve(g, P=P1, tol=tol, max_iter=max_iter, warm_start=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        diff = float((warm.P - plain.P).abs().max() / plain.P.pow(2).mean().sqrt())
        vplain, vwarm, vt_plain, vt_warm = _timed_pair(vplan, ws, g, P0, tol, max_iter)
        row = {"seed": s, "plain_outer": plain.info["outer_iters"], "plain_inner": plain.info["inner_iters_total"],
               "plain_s": t1 - t0, "warm_outer": warm.info["outer_iters"],
               "warm_inner": warm.info["inner_iters_total"], "guess_s": t2 - t1, "warm_solve_s": t3 - t2,
               "warm_s": t3 - t1, "guess_rel_err": guess_err, "warm_vs_plain_maxabs_rel": diff,
               "variant_plain_s": vt_plain, "variant_warm_s": vt_warm,
               "variant_plain_inner": vplain.info["inner_iters_total"],
               "variant_warm_inner": vwarm.info["inner_iters_total"]}
        rows.append(row)
        log(f"eval n={n} seed={s}: plain {row['plain_outer']} outer {row['plain_s']:.2f}s | warm "
            f"{row['warm_outer']} outer {row['warm_s']:.2f}s (guess {row['guess_s'] * 1e3:.1f} ms, "
            f"err {guess_err:.3f}); fixed-point CG variant {vt_plain:.3f}s -> {vt_warm:.3f}s")
    plan.close()
    vplan.close()
    return rows


def main(argv=None):
    from .warmstart import UNet, make_dataset, train

    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64, help="training grid side (= network grid)")
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--seed-base", type=int, default=5000)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--out", default="")
    ap.add_argument("--eval-n", type=int, default=256)
    ap.add_argument("--eval-seeds", type=int, default=2)
    ap.add_argument("--eval-seed", type=int, default=90000)
    ap.add_argument("--json", default="")
    ap.add_argument("--fixed-point-data", action="store_true",
                    help="generate the training answers with the fixed-point CG variant (same fixed point)")
    a = ap.parse_args(argv)
    dev = "cuda:0"
    t0 = time.time()
    x, tgt, stats = make_dataset(a.n, a.count, a.seed_base, tol=a.tol, device=dev, log=log,
                                 fixed_point=a.fixed_point_data)
    t_data = time.time() - t0
    net = UNet(base=a.base, levels=a.levels, cin=4, device=dev, seed=0)
    t1 = time.time()
    hist = train(net, x, tgt, a.steps, batch=a.batch, lr=a.lr, log=log)
    t_train = time.time() - t1
    del x, tgt
    net.release()
    torch.cuda.empty_cache()
    if a.out:
        net.save(a.out, {"train_n": a.n, "train_count": a.count, "seed_base": a.seed_base, "tol": a.tol,
                         "steps": a.steps, "batch": a.batch, "lr": a.lr,
                         "data_solver": "fixed-point CG variant" if a.fixed_point_data else "paper iteration"})
        log(f"saved {a.out}")
    rows = evaluate(net, a.eval_n // a.n, a.eval_n, range(a.eval_seed, a.eval_seed + a.eval_seeds), tol=1e-6,
                    device=dev) if a.eval_seeds > 0 else []
    out = {"train_n": a.n, "count": a.count, "data_s": t_data, "train_s": t_train, "steps": a.steps,
           "mean_outer_data": sum(s["outer_iters"] for s in stats) / len(stats), "loss": hist, "eval": rows}
    if a.json:
        with open(a.json, "w") as f:
            json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "loss"}))


if __name__ == "__main__":
    main()
