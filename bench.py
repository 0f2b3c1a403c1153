#!/usr/bin/env python
"""Benchmark: time to momentum residual 1e-6 for one 256^3 solve on one MI355X.

A step is one complete solve -- Algorithm 1 from P^0 = 0 (or from the learned
warm start, reported beside it) until eps_R <= 1e-6 (Eq. ResidualMomentum) --
of a 256^3 field: the gradient of 32 random Gaussian pressure blobs plus 5 %
Gaussian noise, FP32 stencil and vector updates, FP64 iterate, dot products,
residual and gauge.  Inputs are generated on the GPU before the timed region.

Prints one JSON line.  Besides the contract fields it carries
  roofline      HBM roofline of the dominant kernel, its duration measured with
                HIP events on the library's stream (pi_time_kernel)
  kernels       the same for the two kernels of an outer step
  cpu_baseline  the CPU FP64 oracle (route O1, sparse-LU inner solve) on a
                bounded sample, scaled to one 256^3 solve, and the oracle's
                assembled-CSR operator apply timed at the benchmark size
  oracle_check  the same recipe at 96^3 solved by the library and by the
                oracle's route O2-CG: max-abs error over RMS(P) at the
                benchmark tolerance and fully converged
  fp64          one 256^3 solve in FP64 mode (the paper's precision)
The side legs (warm start, variant, FP64) are deterministic and run one
warm-up and at most SIDE_STEPS timed solves each.
"""

from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
# algorithmic bytes per cell per launch (FP32 mode): what each kernel must read
# and write once, neighbour re-reads excluded.  The benchmark grid has no
# mask, so the stencil kernels derive the 4-byte counter code of each cell
# from its coordinates instead of reading it (a masked grid adds 4 bytes to
# the two stencil kernels).
BYTES_PER_CELL = {
    "k_outer": 8 + 4 + 4 + 8 + 8 + 4,   # P, d, p (last CG step folded in), S (FP64) in; P', r out
    "k_cg_step": 4 * 4 + 4 * 4,         # r, q, p, delta in; r', q', p', delta out
}
# a plan whose CG passes evaluate q = M p again (pi_get_cg_recompute) moves
# r, p, delta in and r', p', delta out
CG_RECOMPUTE_BYTES = 3 * 4 + 3 * 4
# the cell-centred kernels always read the 4-byte ring code of each cell
BYTES_PER_CELL_CC = {k: v + 4 for k, v in BYTES_PER_CELL.items()}
TIMED = (("k_outer", 0), ("k_cg_step", 1))  # names and pi_time_kernel ids (PI_K_OUTER, PI_K_INNER)
SIDE_STEPS = 2        # timed solves of each side leg
ORACLE_CHECK_N = 96   # side of the grid the oracle solves beside the library


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="grid side (256 is the benchmark workload)")
    ap.add_argument("--workload", choices=("blobs3d", "lamb2d"), default="blobs3d",
                    help="blobs3d: n^3 Gaussian blobs, 5 %% noise; lamb2d: n^2 Lamb-Oseen pair, 10 %% noise, "
                         "5 %% of cells masked as disks (use --n 2048)")
    ap.add_argument("--chunk-outer-solve", type=int, default=0,
                    help="run each timed solve as calls of at most this many outer steps, continuing from P "
                         "(for solves longer than a few minutes; 0 = one call)")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--seed", type=int, default=9001, help="held out from warm-start training seeds")
    ap.add_argument("--inner", type=int, default=None, help="inner CG iterations per outer step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=28)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--mode", choices=("solve", "kernels", "batched", "flow", "sequence", "unet"), default="solve",
                    help="kernels: only time the outer-step kernels and a copy of known size (for counters); "
                         "batched: the uneven batch of 2-D snapshots and 3-D volumes in one batched solve")
    ap.add_argument("--count2d", type=int, default=512, help="batched mode: 2-D instances")
    ap.add_argument("--count3d", type=int, default=16, help="batched mode: 3-D instances")
    ap.add_argument("--fixed-point", action="store_true", help="batched mode: use the fixed-point CG variant")
    ap.add_argument("--chunk-outer", type=int, default=4000,
                    help="batched mode: outer steps per batched call (unfinished instances continue from P)")
    ap.add_argument("--sequential-sample", type=int, default=8,
                    help="batched mode: instances also solved one by one, to compare")
    ap.add_argument("--no-autotune", action="store_true", help="keep the size-based default tile")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2311_16935_amd", "weights",
                                                      "unet_blobs128.safetensors"),
                    help="trained warm-start network; the warm-started solve is skipped if missing")
    ap.add_argument("--no-warm", action="store_true")
    ap.add_argument("--cell-centered", action="store_true",
                    help="2-D workloads: the cell-centred scheme (9-point stencils) instead of face-crossing")
    ap.add_argument("--snapshots", type=int, default=6, help="sequence mode: snapshots of the 3-D sequence")
    ap.add_argument("--no-pressure", action="store_true",
                    help="flow mode: report the source kernel only, without integrating the pressure")
    ap.add_argument("--no-variant", action="store_true",
                    help="skip the fixed-point CG variant (not the paper's iteration), reported beside it")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip the 96^3 same-recipe comparison with the oracle")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-mode solve")
    return ap.parse_args()


def progress(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def traffic_from_profile(kernel, n, src_hash, workload="blobs"):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}{n}_pmc.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"^source_sha256:\s*(\S+)", txt, re.M)
    m_b = re.search(r"^hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt, re.M)
    if not m_b or not m_hash or m_hash.group(1) != src_hash:
        return None
    return float(m_b.group(1))


def kernel_source_hash(files=("pi_kernels.hip", "pi_common.h")):
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2311_16935_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(n_sample, seed, n_target, tol, workload="blobs3d"):
    """Oracle route O1 on a small grid of the same recipe, timed on this host,
    scaled to the benchmark grid: cost per outer step grows with the cell
    count and the outer-step count with the side length, so the scale factor
    is (n_target / n_sample)^(ndim + 1).  The sparse LU's fill grows faster
    than the cell count in 3-D, so the scaled figure understates the oracle's
    real cost at full size."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle.solve import outer_iteration
    from oracle.system import assemble

    if workload == "lamb2d":
        w = synth.config_lamb_oseen_2d(n_sample, seed=seed)
        ndim, what = 2, "Lamb-Oseen pair, masked"
        mask = np.ones((n_sample,) * 2, np.uint8) if w.mask is None else w.mask.numpy()
    else:
        w = synth.config_blobs_3d(n_sample, seed=seed)
        ndim, what = 3, "blobs"
        mask = np.ones((n_sample,) * 3, np.uint8)
    g = [np.nan_to_num(x.float().double().numpy()) for x in w.grads]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        s = assemble(mask, w.spacing)
        r = outer_iteration(s, s.source(g), tol, 100000)
        t = time.perf_counter() - t0
    scale = (n_target / n_sample) ** (ndim + 1)
    return {
        "value": t * scale,
        "unit": "s per %d^%d solve to eps_R<=%g (extrapolated from the sample)" % (n_target, ndim, tol),
        "extrapolated": True,
        "scale_factor": scale,
        "cores": 1,
        "kind": "oracle",
        "sample": f"route O1 (exact sparse-LU inner solve) on {n_sample}^{ndim} {what}, seed {seed}: "
                  f"{r.outer} outer steps in {t:.2f} s on 1 thread "
                  f"(host affinity {len(os.sched_getaffinity(0))} cores); scaled by (n/{n_sample})^{ndim + 1}",
        "sample_seconds": t,
        "sample_outer_iters": r.outer,
    }


def cpu_spmv_at_size(n, seed, reps=3):
    """The oracle's assembled operator M = [W^{n+1}] (CSR, FP64) applied to
    a vector on the full benchmark grid, timed on one thread of this host:
    the CPU counterpart of the library's operator apply.  Assembly (the
    oracle's own, cell by cell in NumPy) is timed too but is set-up."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle.system import assemble

    w = synth.config_blobs_3d(n, seed=seed)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        s = assemble(np.ones((n, n, n), np.uint8), w.spacing)
        t_asm = time.perf_counter() - t0
        M = s.M
        x = np.random.default_rng(seed).standard_normal(s.n)
        y = M @ x
        t0 = time.perf_counter()
        for _ in range(reps):
            y = M @ x
        t = (time.perf_counter() - t0) / reps
    del s, M, x, y
    return {"n": n, "cells": n**3, "seconds_per_apply": t, "ns_per_cell": t / n**3 * 1e9,
            "assembly_seconds": t_asm, "threads": 1, "reps": reps,
            "what": "oracle CSR FP64 y = M x at the benchmark size (scipy sparse, single-threaded)"}


def oracle_check(pi, n, seed, tol):
    """The benchmark recipe at n^3 (same seed), solved by the library as the
    benchmark runs it (FP32, autotuned tile) at the benchmark tolerance and
    at 1e-10, against the oracle's FP64 fixed point (route O2-CG) of the same
    FP32 gradient values."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_limits

    import synth
    from oracle.solve import fixed_point_cg
    from oracle.system import assemble

    w = synth.config_blobs_3d(n, seed=seed)
    g32 = [x.to(torch.float32).contiguous() for x in w.grads]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        s = assemble(np.ones((n, n, n), np.uint8), w.spacing)
        S = s.source([x.numpy().astype(np.float64) for x in g32])
        ref = fixed_point_cg(s, S, rtol=1e-14, max_iter=20000)
        t_oracle = time.perf_counter() - t0
    rms = float(np.sqrt(np.mean(ref.P**2)))
    plan = pi.Plan(w.dims, w.spacing)
    plan.autotune(reps=3)
    g = [x.to("cuda:0") for x in g32]
    out = {"n": n, "seed": seed, "recipe": "32 Gaussian blobs, 5 % noise (the benchmark's)",
           "oracle": {"route": "O2-CG (FP64 CG on the fixed point, rtol 1e-14)", "iters": ref.iters,
                      "rel_residual": ref.rel_residual, "seconds": t_oracle, "threads": 1}}
    for key, t in (("at_tol", tol), ("converged", 1e-10)):
        r = plan.solve(g, tol=t, max_iter=10**6)
        P = r.P.cpu().numpy().astype(np.float64).ravel()
        out[key] = {"tol": t, "status": r.status, "outer_iters": r.info["outer_iters"], "eps_R": r.info["eps_R"],
                    "maxabs_rel_rms": float(np.abs(P - ref.P).max() / rms)}
    plan.close()
    out["bar_fp32"] = 1e-5
    return out


def fp64_leg(pi, grads, dims, spacing, tol):
    """One solve in FP64 mode (the paper's precision): every vector, the
    stencil and the updates in double."""
    import torch

    plan = pi.Plan(dims, spacing, fp64=True)
    plan.autotune(reps=3)
    g = [x.double() for x in grads]
    P = torch.empty(plan.shape, dtype=torch.float64, device=g[0].device)
    plan.solve(g, P=P, tol=tol, max_iter=8, check=False)   # captures the outer-step graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = plan.solve(g, P=P, tol=tol)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    plan.close()
    del g, P
    return {"s_per_solve": sec, "outer_iters": r.info["outer_iters"], "inner_iters": r.info["inner_iters_total"],
            "eps_R": r.info["eps_R"], "status": r.status, "timed_solves": 1}


def timed_solve(plan, grads, P, tol, chunk, max_iter=10**7):
    """One solve from P^0 = 0; with chunk > 0 as calls of at most `chunk`
    outer steps, each continuing from the P the previous one returned."""
    import paper_2311_16935_amd as pi

    if chunk <= 0:
        r = plan.solve(grads, P=P, tol=tol, max_iter=max_iter)
        return r.info
    P.zero_()
    outer = inner = 0
    first = True
    while True:
        r = plan.solve(grads, P=P, tol=tol, max_iter=chunk, warm_start=not first, check=False)
        first = False
        outer += r.info["outer_iters"]
        inner += r.info["inner_iters_total"]
        progress(f"  ... {outer} outer steps, eps_R {r.info['eps_R']:.2e}")
        if r.status != pi.PI_ERR_NOT_CONVERGED:
            if r.status != pi.PI_OK:
                raise pi.PiError(r.status, "pi_solve")
            info = dict(r.info)
            info.update(outer_iters=outer, inner_iters_total=inner)
            return info


APPLY_TILES = (4, 8, 16, 32)   # segment lengths (planes per wave) tried for pi_apply


def time_apply(pi, plan, reps, code_bytes):
    """y = M x alone (pi_apply, the operator the CG pass applies), timed with
    HIP events on the stream it is launched on.  Algorithmic bytes: x in,
    y out (+ the 4-byte code where the plan reads it).

    pi_apply runs at the plan's tile.  The solve's autotuner picks the tile
    that balances its outer and CG kernels; the apply alone moves 8 bytes
    per cell and needs more waves in flight, so it is timed at its own
    segment length, picked from APPLY_TILES by a short sweep before the
    timed launches.  The plan's tile is restored afterwards."""
    import torch

    x = torch.randn(plan.shape, dtype=plan.dtype, device="cuda:0")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    keep = (pi.pi_get_tile(plan.handle), pi.pi_get_lane_cells(plan.handle))

    def run(n):
        plan.apply(pi.PI_OP_M, x, y, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            plan.apply(pi.PI_OP_M, x, y, stream=stream)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / n

    sweep = {}
    for mseg in APPLY_TILES:
        pi.pi_set_tile(plan.handle, mseg, keep[1])
        sweep[pi.pi_get_tile(plan.handle)] = run(3)
    tile = min(sweep, key=sweep.get)
    pi.pi_set_tile(plan.handle, tile, keep[1])
    ms = run(reps)  # the last reps + 1 launches of k_apply run at this tile
    pi.pi_set_tile(plan.handle, *keep)
    ncell = x.numel()
    alg = (2 * x.element_size() + code_bytes) * ncell
    return {"op": "M = [W^{n+1}]", "avg_ms": ms, "launches": reps + 1, "alg_bytes": alg,
            "achieved_GBs": alg / (ms * 1e-3) / 1e9, "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "tile": tile, "lane_cells": keep[1], "tile_sweep_ms": {str(k): round(v, 5) for k, v in sweep.items()}}


def kernel_mode(args, pi, plan, grads, P, ncell, bytes_per_cell=BYTES_PER_CELL):
    """Few dispatches: fill the workspace with four outer steps, then launch
    each outer-step kernel a few times, then run an element-wise int32 kernel
    over ncell elements (reads and writes 4 * ncell bytes) as the counter
    yardstick."""
    import torch

    plan.solve(grads, P=P, tol=0.0, max_iter=4, check=False)
    res = {}
    for name, kid in TIMED:
        ms = pi.pi_time_kernel(plan.handle, kid, args.kernel_reps)
        res[name] = {"avg_ms": ms, "launches": args.kernel_reps + 1,
                     "alg_bytes": bytes_per_cell[name] * ncell,
                     "achieved_GBs": bytes_per_cell[name] * ncell / (ms * 1e-3) / 1e9}
    res["k_apply"] = time_apply(pi, plan, args.kernel_reps, bytes_per_cell.get("code", 0))
    # yardstick with a kernel name nothing else here uses: reads and writes
    # 4 bytes per element
    x = torch.randint(0, 1 << 30, (ncell,), dtype=torch.int32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(args.kernel_reps):
        torch.bitwise_not(x, out=y)
    torch.cuda.synchronize()
    res["bitwise_not"] = {"bytes_read": 4 * ncell, "bytes_written": 4 * ncell, "launches": args.kernel_reps}
    print(json.dumps({"mode": "kernels", "n": args.n, "cells": ncell, "tile": pi.pi_get_tile(plan.handle),
                      "lane_cells": pi.pi_get_lane_cells(plan.handle),
                      "cg_recompute": pi.pi_get_cg_recompute(plan.handle),
                      "workload": args.workload, "cell_centered": bool(args.cell_centered),
                      "kernels": res, "kernel_source_sha256": kernel_source_hash()}), flush=True)


def warm_start_leg(args, pi, plan, grads, P_plain, n, ws, label):
    """The same solve from a warm start: the guess (network inference --
    gradient RMS, block means, U-Net -- and/or the coarse solve, then
    trilinear upsampling) plus the plain solver finishing from it, timed end
    to end per solve; the converged field is compared with the zero-start
    answer."""
    import torch

    P = torch.empty_like(P_plain)
    steps = min(args.steps, SIDE_STEPS)
    for i in range(min(args.warmup, 1)):
        r = ws.solve(plan, grads, P=P, tol=args.tol)
        progress(f"{label} warmup {i}: {r.info['outer_iters']} outer steps")
    torch.cuda.synchronize()
    infos, t_guess = [], 0.0
    t0 = time.perf_counter()
    for i in range(steps):
        a = time.perf_counter()
        ws.guess(plan, grads, P)
        torch.cuda.synchronize()
        t_guess += time.perf_counter() - a
        r = plan.solve(grads, P=P, tol=args.tol, warm_start=True)
        infos.append(r.info)
        progress(f"{label} step {i}: {r.info['outer_iters']} outer steps")
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / max(1, steps)
    info = infos[-1]
    assert info["status"] == 0 and info["eps_R"] <= args.tol, info
    rms = float(P_plain.double().pow(2).mean().sqrt())
    diff = float((P.double() - P_plain.double()).abs().max()) / rms
    out = {"s_per_solve": sec, "timed_solves": steps, "guess_s": t_guess / max(1, steps),
           "outer_iters": info["outer_iters"], "inner_iters": info["inner_iters_total"], "eps_R": info["eps_R"],
           "factor": ws.factor, "coarse_solve": ws.coarse, "maxabs_vs_plain_rel_rms": diff}
    if ws.coarse:
        out["coarse"] = dict(ws.last, tol=ws.coarse_tol, grid=[d // ws.factor for d in plan.dims],
                             solver="fixed-point CG variant")
    if ws.net is not None:
        out["weights"] = os.path.relpath(args.weights, ROOT)
        out["train"] = {k: ws.net.meta[k] for k in ws.net.meta}
    return out


def warm_start_legs(args, pi, plan, grads, P_plain, n, sec_plain):
    """Three starts beside the zero start: the learned guess with the coarse
    solve (the warm start), the learned guess alone, the coarse solve alone."""
    from paper_2311_16935_amd.warmstart import UNet, WarmStart

    net = UNet.from_file(args.weights)
    factor = n // int(net.meta.get("train_n", 64))
    legs = {}
    for key, ws in (("learned_plus_coarse", WarmStart(net, factor, coarse=True)),
                    ("learned_only", WarmStart(net, factor)),
                    ("coarse_only", WarmStart(None, factor, coarse=True))):
        legs[key] = warm_start_leg(args, pi, plan, grads, P_plain, n, ws, key)
        legs[key]["reduction_vs_plain"] = 1.0 - legs[key]["s_per_solve"] / sec_plain
        ws.close()
    out = dict(legs["learned_plus_coarse"])
    out["legs"] = legs
    return out


def variant_leg(args, pi, grads, P_plain, dims, mask, spacing, weights_ok, cc=False):
    """The PI_FIXED_POINT_CG variant -- CG on the fixed point's operator
    instead of the paper's lagged boundary iteration, same stopping test and
    converged field -- from zero and from the learned guess."""
    import torch

    plan = pi.Plan(dims, spacing, mask=mask, fixed_point=True, cell_centered=cc)
    plan.autotune(reps=5)
    n = dims[0]
    P = torch.empty_like(P_plain)
    out = {"inner_per_outer": None}
    steps = min(args.steps, SIDE_STEPS)
    for i in range(min(args.warmup, 1)):
        r = plan.solve(grads, P=P, tol=args.tol)
    rms = float(P_plain.double().pow(2).mean().sqrt()) if mask is None else \
        float(P_plain.double()[~P_plain.isnan()].pow(2).mean().sqrt())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        r = plan.solve(grads, P=P, tol=args.tol)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / max(1, steps)
    info = r.info
    assert info["status"] == 0 and info["eps_R"] <= args.tol, info
    diff = (P.double() - P_plain.double()).nan_to_num(0.0).abs().max()
    out.update({"s_per_solve": sec, "outer_iters": info["outer_iters"], "inner_iters": info["inner_iters_total"],
                "eps_R": info["eps_R"], "inner_per_outer": info["inner_iters_total"] // max(1, info["outer_iters"]),
                "maxabs_vs_plain_rel_rms": float(diff) / rms})
    progress(f"fixed-point CG variant: {sec:.3f} s per solve, {info['inner_iters_total']} CG iterations")
    if weights_ok:
        from paper_2311_16935_amd.warmstart import UNet, WarmStart

        net = UNet.from_file(args.weights)
        ws = WarmStart(net, n // int(net.meta.get("train_n", 64)))
        ws.solve(plan, grads, P=P, tol=args.tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            r = ws.solve(plan, grads, P=P, tol=args.tol)
        torch.cuda.synchronize()
        wsec = (time.perf_counter() - t0) / max(1, steps)
        out.update({"warm_s_per_solve": wsec, "warm_inner_iters": r.info["inner_iters_total"]})
        progress(f"fixed-point CG variant from the learned guess: {wsec:.3f} s per solve")
    plan.close()
    return out


def batched_mode(args):
    """Uneven batch (2-D Lamb-Oseen snapshots with sides U{128..1024} and
    0-5 % disk masks, 3-D blob volumes with sides U{64..256}, 5 % noise, seeds
    4000 + i) in batched calls of at most --chunk-outer outer steps each;
    instances that are not done continue from their returned P."""
    import torch

    import paper_2311_16935_amd as pi
    import synth

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    works = synth.batched_instances(args.count2d, args.count3d, device=dev)
    progress(f"{len(works)} instances generated ({time.perf_counter() - t0:.1f} s)")
    grads, plans = [], []
    for i, w in enumerate(works):
        grads.append([g.float().contiguous() for g in w.grads])
        mask = None if w.mask is None else w.mask.cpu()
        plans.append(pi.Plan(w.dims, w.spacing, mask=mask, fixed_point=args.fixed_point))
        if args.no_autotune is False:
            plans[-1].autotune(reps=3)
        if (i + 1) % 64 == 0 or i + 1 == len(works):
            progress(f"planned {i + 1}/{len(works)} ({time.perf_counter() - t0:.1f} s)")
    cells = sum(w.ncells for w in works)
    Ps = [torch.zeros(p.shape, dtype=torch.float32, device=dev) for p in plans]
    todo = list(range(len(works)))
    outer = [0] * len(works)
    inner = [0] * len(works)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    first = True
    while todo:
        rc, _, infos = pi.solve_batched([plans[i] for i in todo], [grads[i] for i in todo], [Ps[i] for i in todo],
                                        tol=args.tol, max_iter=args.chunk_outer, warm_start=not first, check=False)
        first = False
        left = []
        for i, info in zip(todo, infos):
            outer[i] += info["outer_iters"]
            inner[i] += info["inner_iters_total"]
            if info["status"] == pi.PI_ERR_NOT_CONVERGED:
                left.append(i)
            elif info["status"] != pi.PI_OK:
                raise pi.PiError(info["status"], f"instance {i}")
        todo = left
        progress(f"batched call: {len(works) - len(todo)}/{len(works)} done, {time.perf_counter() - t1:.1f} s")
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - t1
    # a few instances alone, for the batched-against-sequential comparison
    rng = __import__("random").Random(0)
    sample = sorted(rng.sample(range(len(works)), min(args.sequential_sample, len(works))))
    seq_s = 0.0
    for i in sample:
        P = torch.zeros(plans[i].shape, dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        a = time.perf_counter()
        r = plans[i].solve(grads[i], P=P, tol=args.tol)
        torch.cuda.synchronize()
        seq_s += time.perf_counter() - a
    progress(f"{len(sample)} instances one by one: {seq_s:.1f} s")
    out = {
        "metric": "time-to-residual per uneven batch" + (" (fixed-point CG variant)" if args.fixed_point else ""),
        "value": batch_s, "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f32",
        "reductions_dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batched_{args.count2d}x2d_{args.count3d}x3d", "count2d": args.count2d,
                   "count3d": args.count3d, "cells": cells, "tol_eps_R": args.tol, "seeds": "4000+i",
                   "chunk_outer": args.chunk_outer, "autotuned": not args.no_autotune},
        "outer_iters": {"max": max(outer), "mean": sum(outer) / len(outer)},
        "inner_iters_total": sum(inner),
        "sequential_sample": {"instances": sample, "seconds": seq_s,
                              "estimated_all_one_by_one": seq_s * len(works) / max(1, len(sample))},
    }
    print(json.dumps(out), flush=True)


FLOW_BYTES_PER_CELL = 9 * 4 + 3 * 4   # u, u(t - dt), u(t + dt) in (3 x 3 FP32); f out (3 FP32)


def flow_mode(args):
    """Velocity -> source -> pressure on an n^3 decaying ABC flow (exact
    Navier-Stokes solution, P = -rho |u|^2 / 2): the source kernel timed with
    HIP events on the stream it runs on, against the HBM roofline, then the
    pressure integrated from it (paper iteration and fixed-point CG variant)
    and compared with the analytic pressure."""
    import torch

    import paper_2311_16935_amd as pi
    import synth
    from paper_2311_16935_amd import flow

    dev = torch.device("cuda:0")
    n = args.n
    rho, nu, t, dt = 1.0, 0.5, 0.2, 1e-3
    snaps = []
    for tt in (t, t - dt, t + dt):
        u, P, sp = synth.abc_velocity((n, n, n), t=tt, nu=nu, rho=rho, device=dev)
        snaps.append([c.float().contiguous() for c in u])
        if tt == t:
            P_true = (P - P.mean()).float()
        del u, P
    u, up, un = snaps
    f = [torch.empty_like(u[0]) for _ in range(3)]
    stream = torch.cuda.current_stream()

    def run():
        flow.pi_flow_source(flow.PI_FLOW_NS, u, sp, out=f, u_prev=up, u_next=un, rho=rho, mu=rho * nu, dt=dt,
                            stream=stream)

    for _ in range(args.warmup + 1):
        run()
    stream.synchronize()
    reps = max(1, args.kernel_reps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ncell = n ** 3
    alg = FLOW_BYTES_PER_CELL * ncell
    gbs = alg / (ms * 1e-3) / 1e9
    progress(f"k_flow {n}^3: {ms * 1e3:.1f} us per launch, {gbs:.0f} GB/s")
    # counter yardstick, as in --mode kernels: reads and writes 4 bytes per element
    x = torch.randint(0, 1 << 30, (ncell,), dtype=torch.int32, device=dev)
    torch.bitwise_not(x, out=torch.empty_like(x))
    del x
    legs = {}
    for name, fp in (() if args.no_pressure else (("paper_iteration", False), ("fixed_point_cg_variant", True))):
        plan = pi.Plan((n, n, n), sp, fixed_point=fp)
        P = torch.empty(plan.shape, dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        a = time.perf_counter()
        info = timed_solve(plan, f, P, args.tol, args.chunk_outer_solve)
        torch.cuda.synchronize()
        sec = time.perf_counter() - a
        err = float(torch.sqrt(torch.mean((P.double() - P_true.double()) ** 2)) / P_true.abs().max())
        legs[name] = {"seconds": sec, "outer_iters": info["outer_iters"], "inner_iters": info["inner_iters_total"],
                      "eps_R": info["eps_R"], "rms_err_vs_analytic_over_max": err}
        progress(f"{name}: {sec:.2f} s, {info['outer_iters']} outer steps, error {err:.2e}")
        plan.close()
    out = {
        "metric": f"velocity->source kernel time per {n}^3 snapshot (Navier-Stokes, unsteady, viscous)",
        "value": ms, "unit": "ms", "n_gpus": 1, "steps": reps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64 arithmetic, f32 fields",
        "data": "synthetic",
        "config": {"workload": f"abc_flow_{n}^3", "n": n, "cells": ncell, "rho": rho, "nu": nu, "t": t, "dt": dt},
        "roofline": {"kernel": "k_flow", "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS,
                     "traffic": traffic_from_profile("k_flow", n, kernel_source_hash(("pi_flow.hip",)), "abc"),
                     "bytes_per_cell": FLOW_BYTES_PER_CELL,
                     "cells_per_launch": ncell},
        "pressure_from_source": legs,
    }
    print(json.dumps(out), flush=True)


def sequence_mode(args):
    """Time-resolved sequences, each snapshot solved from zero and from the
    previous snapshot's pressure: (1) n^3 drifting blobs (32 blobs, seed
    --seed, velocities N(0, (1/n)^2) per axis and snapshot, so a blob moves
    about one cell per snapshot; 5 % gradient noise); (2) the Taylor-vortex
    series of the 2-D benchmark section (26 snapshots, 0.05 <= t <= 0.3,
    101^2 on [-3, 3]^2), velocity -> source (pi_flow_source) -> pressure."""
    import numpy as np
    import torch

    import paper_2311_16935_amd as pi
    import synth
    from paper_2311_16935_amd import flow
    from paper_2311_16935_amd.sequence import solve_sequence

    dev = torch.device("cuda:0")
    n = args.n
    snaps = []
    for k in range(args.snapshots):
        _, g, sp = synth.gaussian_blobs((n, n, n), seed=args.seed, device=dev, with_pressure=False, t=float(k),
                                        speed=1.0 / n)
        g = synth.add_noise(g, None, 0.05, args.seed + 1000 + k, device=dev)
        snaps.append([c.float().contiguous() for c in g])
        del g
    progress(f"{len(snaps)} snapshots of {n}^3 drifting blobs generated")
    out_legs = {}
    for name, fp in (("paper_iteration", False), ("fixed_point_cg_variant", True)):
        if fp and args.no_variant:
            continue
        plan = pi.Plan((n, n, n), sp, fixed_point=fp)
        if not args.no_autotune:
            plan.autotune(reps=3)
        leg = {}
        for warm in (False, True):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = solve_sequence(plan, snaps, tol=args.tol, warm=warm)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            assert all(r.status == 0 for r in res), [r.info for r in res]
            leg["warm" if warm else "cold"] = {
                "seconds_per_snapshot": sec / len(snaps),
                "outer_iters": [r.info["outer_iters"] for r in res],
                "inner_iters": [r.info["inner_iters_total"] for r in res]}
            if warm:
                leg["max_diff_warm_vs_cold_over_rms"] = max(
                    float((a.P - b.P).abs().max() / b.P.pow(2).mean().sqrt()) for a, b in zip(res, cold))
            else:
                cold = res
            progress(f"{name} {'warm' if warm else 'cold'}: {sec / len(snaps):.3f} s per snapshot, outer "
                     f"{leg['warm' if warm else 'cold']['outer_iters']}")
        del cold
        plan.close()
        out_legs[name] = leg
    # the paper's 2-D Taylor-vortex series, from velocity
    m, dtv = 101, 1e-4
    srcs = []
    for t in np.linspace(0.05, 0.3, 26):
        u, _, sp2 = synth.taylor_velocity((m, m), t=t, device=dev)
        up = synth.taylor_velocity((m, m), t=t - dtv, device=dev)[0]
        un = synth.taylor_velocity((m, m), t=t + dtv, device=dev)[0]
        f32 = [[c.float().contiguous() for c in v] for v in (u, up, un)]
        srcs.append(flow.pi_flow_source(flow.PI_FLOW_NS, f32[0], sp2, u_prev=f32[1], u_next=f32[2], rho=1.0,
                                        mu=1.0, dt=dtv))
    plan = pi.Plan((m, m), sp2)
    tv = {}
    for warm in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = solve_sequence(plan, srcs, tol=args.tol, warm=warm)
        torch.cuda.synchronize()
        tv["warm" if warm else "cold"] = {"seconds_total": time.perf_counter() - t0,
                                          "outer_iters_total": sum(r.info["outer_iters"] for r in res)}
    plan.close()
    progress(f"taylor vortex series: cold {tv['cold']}, warm {tv['warm']}")
    w, c = out_legs["paper_iteration"]["warm"], out_legs["paper_iteration"]["cold"]
    out = {
        "metric": f"time-to-residual {args.tol:g} per {n}^3 snapshot of a time-resolved sequence, warm-started "
                  "from the previous snapshot",
        "value": w["seconds_per_snapshot"], "unit": "s", "n_gpus": 1, "steps": args.snapshots, "warmup": 0,
        "ms_per_step": w["seconds_per_snapshot"] * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "reductions_dtype": "f64", "data": "synthetic",
        "config": {"workload": f"drifting_blobs3d_{n}^3_x{args.snapshots}", "n": n, "snapshots": args.snapshots,
                   "nblobs": 32, "blob_speed_per_snapshot": 1.0 / n, "noise": 0.05, "seed": args.seed,
                   "tol_eps_R": args.tol},
        "cold_seconds_per_snapshot": c["seconds_per_snapshot"],
        "legs": out_legs,
        "taylor_vortex_series_101": tv,
    }
    print(json.dumps(out), flush=True)


def unet_mode(args):
    """The warm-start network's BF16 matrix-core layers at the training
    shapes 128^3 (batch 4) and 256^3 (batch 1): forward and training-step
    time (HIP events on the current stream) and TFLOP/s against the dense
    BF16 peak, per layer for the 3x3x3 convolutions of each level.  Random
    weights and inputs: the work does not depend on the values."""
    import math

    import torch

    from paper_2311_16935_amd import unet as U
    from paper_2311_16935_amd.warmstart import UNet

    dev = "cuda:0"
    peak = 2500.0
    out = {}
    for res, batch in ((128, 4), (256, 1)):
        net = UNet(device=dev, seed=0)
        B = net.buffers(batch, (res, res, res))
        B["x0"].copy_(torch.randn(B["x0"].shape, device=dev).to(torch.bfloat16))
        tgt = torch.randn((batch, res, res, res), device=dev)
        flops = 0
        for L in net.layers.values():
            if L.kind in ("conv", "up"):
                lvl = int(L.name[3]) if L.kind == "conv" else int(L.name[2]) + 1
                flops += 2 * batch * (res >> lvl) ** 3 * L.cout * L.taps * L.cin

        def timed(fn, n=5):
            for _ in range(2):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(n):
                fn()
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1) / n

        fw = timed(lambda: net.forward(B))
        tr = timed(lambda: net.train_step(B, tgt, 1e-5))
        T, R = U.tensor, B["R"]
        layers = {}
        for name in ("enc0b", "enc1b", "enc2b", "enc3b", "dec0a"):
            L = net.layers[name]
            lvl = int(name[3])
            src = T(B["cat0"]) if name == "dec0a" else T(B[f"t{lvl}"])
            dst = T(B["ua0"]) if name == "dec0a" else (T(B["bot"]) if lvl == 3 else T(B[f"t{lvl}"], 0, L.cout))
            if name in ("enc0b", "enc1b", "enc2b"):
                dst = T(B[f"ua{lvl}"])
            ms = timed(lambda: net._conv(name, src, dst, R[lvl]))
            f = 2 * batch * (res >> lvl) ** 3 * L.cout * 27 * L.cin
            layers[name] = {"ms": ms, "TFLOPs": f / ms / 1e9, "M": batch * (res >> lvl) ** 3, "N": L.cout,
                            "K": 27 * L.cin}
        key = f"{res}^3_batch{batch}"
        out[key] = {"forward_ms": fw, "forward_TFLOPs": flops / fw / 1e9,
                    "forward_frac_of_peak": flops / fw / 1e9 / peak, "train_step_ms": tr,
                    "train_step_TFLOPs": 3 * flops / tr / 1e9, "layers": layers}
        progress(f"{key}: forward {fw:.2f} ms ({flops / fw / 1e9:.0f} TFLOP/s), train step {tr:.1f} ms")
        net.release()
        del net, B, tgt
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "unet", "peak_TFLOPs": peak, "dtype": "bf16 (fp32 accumulate)", "results": out}),
          flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.mode == "batched":
        batched_mode(args)
        return
    if args.mode == "flow":
        flow_mode(args)
        return
    if args.mode == "sequence":
        sequence_mode(args)
        return
    if args.mode == "unet":
        unet_mode(args)
        return
    import torch

    import paper_2311_16935_amd as pi
    import synth

    dev = torch.device("cuda:0")
    n = args.n
    if args.workload == "lamb2d":
        w = synth.config_lamb_oseen_2d(n, device=dev)
        dims = (n, n)
        workload = f"lamb_oseen2d_{n}^2_masked"
    else:
        w = synth.config_blobs_3d(n, seed=args.seed, device=dev, with_pressure=False)
        dims = (n, n, n)
        workload = f"blobs3d_{n}^3"
    mask = None if w.mask is None else w.mask.cpu()
    grads = [g.to(torch.float32).contiguous() for g in w.grads]
    del w.grads[:]
    cc = args.cell_centered and len(dims) == 2
    if cc:
        workload += "_cell_centred"
    plan = pi.Plan(dims, w.spacing, mask=mask, fp64=False, inner_iters=args.inner, cell_centered=cc)
    P = torch.empty(plan.shape, dtype=torch.float32, device=dev)
    ncell = 1
    for v in dims:
        ncell *= v
    # a masked grid reads the 4-byte counter code in both stencil kernels
    bytes_per_cell = dict(BYTES_PER_CELL_CC if cc else BYTES_PER_CELL)
    bytes_per_cell["code"] = 4 if cc else 0
    if mask is not None and not cc:
        bytes_per_cell["k_outer"] += 4
        bytes_per_cell["k_cg_step"] += 4
        bytes_per_cell["code"] = 4
    progress(f"plan ready: {workload}, tile {pi.pi_get_tile(plan.handle)}, "
             f"{plan.workspace_bytes / 2**30:.2f} GiB, {pi.lib.pi_get_lane_cells(plan.handle)} cells per lane")
    tune = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        m = plan.autotune(reps=5)
        tune = {"mseg": m, "lane_cells": pi.pi_get_lane_cells(plan.handle),
                "cg_recompute": pi.pi_get_cg_recompute(plan.handle), "seconds": time.perf_counter() - t0}
        progress(f"autotuned tile: {m} planes per segment ({tune['seconds']:.1f} s, outside the timed region)")
    if pi.pi_get_cg_recompute(plan.handle):
        bytes_per_cell["k_cg_step"] = CG_RECOMPUTE_BYTES + bytes_per_cell["code"]
    if args.mode == "kernels":
        kernel_mode(args, pi, plan, grads, P, ncell, bytes_per_cell)
        return
    for i in range(args.warmup):
        info = timed_solve(plan, grads, P, args.tol, args.chunk_outer_solve)
        progress(f"warmup {i}: {info['outer_iters']} outer steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        info = timed_solve(plan, grads, P, args.tol, args.chunk_outer_solve)
        progress(f"step {i}: {info['outer_iters']} outer steps, {time.perf_counter() - t0:.2f} s so far")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sec = elapsed / max(1, args.steps)
    assert info["status"] == 0 and info["eps_R"] <= args.tol, info
    P_plain = P.clone()
    warm = None
    weights_ok = not args.no_warm and os.path.exists(args.weights) and len(dims) == 3
    if weights_ok:
        warm = warm_start_legs(args, pi, plan, grads, P_plain, n, sec)
    variant = None
    if not args.no_variant:
        variant = variant_leg(args, pi, grads, P_plain, dims, mask, w.spacing, weights_ok, cc)
    fp64 = None
    if not args.no_fp64 and args.workload == "blobs3d" and not args.chunk_outer_solve:
        fp64 = fp64_leg(pi, grads, dims, w.spacing, args.tol)
        progress(f"fp64 mode: {fp64['s_per_solve']:.2f} s, {fp64['outer_iters']} outer steps")

    # kernel durations, measured with HIP events on the library's stream
    src_hash = kernel_source_hash()
    kern = {}
    for name, kid in TIMED:
        ms = pi.pi_time_kernel(plan.handle, kid, args.kernel_reps)
        alg = bytes_per_cell[name] * ncell
        kern[name] = {"avg_ms": ms, "alg_bytes": alg, "achieved_GBs": alg / (ms * 1e-3) / 1e9}
    # one pass per CG iteration; the outer kernel folds in the last one's update
    launches = {"k_outer": info["outer_iters"] + 1, "k_cg_step": info["inner_iters_total"]}
    for name in kern:
        kern[name]["launches_per_solve"] = launches[name]
        kern[name]["share_of_solve"] = launches[name] * kern[name]["avg_ms"] * 1e-3 / sec
    apply = time_apply(pi, plan, args.kernel_reps, bytes_per_cell["code"])
    progress(f"operator apply y = M x: {apply['avg_ms'] * 1e3:.1f} us, {apply['achieved_GBs']:.0f} GB/s "
             f"at {apply['tile']} planes per segment")
    dom = max(kern, key=lambda k: kern[k]["launches_per_solve"] * kern[k]["avg_ms"])
    d = kern[dom]
    if cc:
        kern_names = {"k_outer": "k_outer_cc", "k_cg_step": "k_cg_step_cc"}
        dom_name = kern_names.get(dom, dom)
        traffic = traffic_from_profile(dom_name, n, src_hash, "lamb_cc")
    else:
        # a plan whose CG passes evaluate q again runs them as k_cg_rq
        dom_name = "k_cg_rq" if dom == "k_cg_step" and pi.pi_get_cg_recompute(plan.handle) else dom
        traffic = traffic_from_profile(dom_name, n, src_hash) if args.workload == "blobs3d" else None
    roof = {"kernel": dom_name, "bound": "hbm", "achieved": d["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": d["achieved_GBs"] / HBM_PEAK_GBS, "traffic": traffic,
            "bytes_per_cell": bytes_per_cell[dom], "cells_per_launch": ncell}
    recipe = ({"nblobs": 32, "noise": 0.05, "seed": args.seed} if args.workload == "blobs3d" else
              {"vortices": 2, "core_radius": 0.05, "noise": 0.10, "masked_fraction": 0.05, "seed": 2})
    out = {
        "metric": ("time-to-residual 1e-6 per 256^3 solve, plain vs learned warm start; HBM GB/s"
                   if workload == "blobs3d_256^3" and args.tol == 1e-6 else
                   f"time-to-residual {args.tol:g} per {workload} solve; HBM GB/s"),
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "reductions_dtype": "f64",
        "data": "synthetic",
        "config": dict({"workload": workload, "n": n, "cells": ncell}, **recipe,
                       tol_eps_R=args.tol, start="P0=0 (plain)",
                       inner_cg_iters=info["inner_iters_total"] // max(1, info["outer_iters"]),
                       parallelism="single GPU"),
        "solve": {"outer_iters": info["outer_iters"], "inner_iters": info["inner_iters_total"],
                  "eps_R": info["eps_R"], "eps_P": info["eps_P"],
                  "outer_point_iters_per_s": ncell * info["outer_iters"] / sec,
                  "inner_point_iters_per_s": ncell * info["inner_iters_total"] / sec},
        "warm_start": warm,
        "variant_fixed_point_cg": variant,
        "fp64": fp64,
        "autotune": tune,
        "roofline": roof,
        "kernels": kern,
        "operator_apply": apply,
        "kernel_source_sha256": src_hash,
    }
    plan.close()
    del grads, P
    torch.cuda.empty_cache()
    if not args.no_oracle_check and args.workload == "blobs3d":
        out["oracle_check"] = oracle_check(pi, ORACLE_CHECK_N, args.seed, args.tol)
        progress(f"oracle check at {ORACLE_CHECK_N}^3: {out['oracle_check']['at_tol']['maxabs_rel_rms']:.2e} at "
                 f"tol, {out['oracle_check']['converged']['maxabs_rel_rms']:.2e} converged")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_n if args.workload == "blobs3d" else 96, args.seed, n,
                                           args.tol, args.workload)
        progress(f"cpu baseline sample: {out['cpu_baseline']['sample_seconds']:.1f} s")
        if args.workload == "blobs3d":
            out["cpu_baseline"]["at_size"] = cpu_spmv_at_size(n, args.seed)
            if "oracle_check" in out:
                out["cpu_baseline"]["at_size"]["o2_cg_solve"] = dict(out["oracle_check"]["oracle"], n=ORACLE_CHECK_N)
            progress(f"cpu spmv at {n}^3: {out['cpu_baseline']['at_size']['seconds_per_apply']:.3f} s per apply")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
