"""Benchmark: preconditioned saddle-point solves per second on one MI355X.

Workload: a linearised weak-constraint 4D-Var window shaped like the paper's experiments,
s = 4096 state variables, N = 64 (65 time blocks), p_i = 2048 random observation points,
dense SOAR B (length 0.1), Q_i = 0.1 B, dense SOAR R_i (length 0.05), implicit
advection-diffusion model; 8 right-hand sides (0; d_r; 0) whose innovations share the signal
and redraw the observation noise (perturbed observations).  Inexact-constraint
preconditioner P_I with L_M(3) and the ridge-regression Rhat, flexible GMRES to a 1e-6 true
relative residual, x0 = 0.

Two paths on the same window, right-hand sides, P, k, Rhat and tolerance:
  * plain FP64: one right-hand side per solve, no restart (the reference path);
  * learned + batched (`value`): all 8 right-hand sides in one call, the network
    correction of the Lhat^{-T} sweep (trained beforehand, untimed, on pairs harvested from
    plain solves of other seeds of the same workload), float32 Rhat^{-1} products in P,
    FGMRES restarted every 200 steps (each step's Gram-Schmidt reads the basis of its
    cycle only; measured: 7.0 solves/s against 6.5 without restart).
One step = one batched solve of the 8 right-hand sides.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--plain-only]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Gram-Schmidt passes, C2 x 8 rhs: HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counters
# (fetch scaled by 2.000, write by 1.000 from the calibration map in the same runs) over the
# timed region, divided by the algorithmic bytes per launch of that run (7.0255 GB / 6.9426 GB).
# Valid while k_fg_dot / k_fg_update and their task plan are unchanged.
ORTHO_TRAFFIC_RATIO = 7.0255 / 6.9426
# the same ratio for block Gram-Schmidt (blocks of BLOCK_TRAFFIC_B columns); None until the
# counters have been taken for the current block kernels
BLOCK_TRAFFIC_RATIO = None
BLOCK_TRAFFIC_B = 8
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--k", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="print iterations and time per solve over k, restart length and "
                         "precision (one JSON object) instead of the benchmark line")
    ap.add_argument("--c3", action="store_true",
                    help="Lorenz-96 window (s=2048, N=32): iterations vs k and the 5-iteration "
                         "Gauss-Newton outer loop (one JSON object)")
    ap.add_argument("--c5", type=int, default=0, metavar="W",
                    help="learned-correction mode: train on C5-shaped windows (s=4096, N=32), "
                         "then solve W held-out windows x 8 rhs batched with the network "
                         "against every system one at a time in plain FP64 (one JSON object)")
    ap.add_argument("--c4", type=int, default=0, metavar="W",
                    help="batched mode: W uneven advection-diffusion windows x 8 perturbed-"
                         "observation right-hand sides in one call, against one-at-a-time "
                         "solves of the first two windows (one JSON object)")
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file for the GEMM autotuning cache (--c4 mode)")
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--precision", default="FP64_F32P",
                    help="precision of the learned + batched path")
    ap.add_argument("--block", type=int, default=0,
                    help="s-step FGMRES block size of the learned + batched path (0: one "
                         "column at a time; with the nonlinear network the block basis "
                         "stagnates)")
    ap.add_argument("--c4-learned", action="store_true",
                    help="--c4 mode: also solve the batch with the network trained on the C5 "
                         "shape (FP64_F32P)")
    ap.add_argument("--c4-block", type=int, default=4,
                    help="--c4 mode: also time s-step FGMRES with this block size (0: skip)")
    ap.add_argument("--lb-restart", type=int, default=200,
                    help="FGMRES restart length of the learned + batched path (0: none)")
    ap.add_argument("--plain-block", type=int, default=8,
                    help="also time the batched solve with the plain preconditioner in "
                         "s-step FGMRES with this block size (0: skip)")
    ap.add_argument("--train-windows", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--harvest", type=int, default=300, help="pairs harvested per window")
    ap.add_argument("--plain-only", action="store_true",
                    help="time only the plain FP64 path (no training)")
    ap.add_argument("--n-bound", type=int, default=20,
                    help="later segment starts the network sees (1 + n_bound + k <= 32)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the GEMM autotuning of the batched path")
    ap.add_argument("--patience", type=int, default=20,
                    help="failing FGMRES steps in a row before the network is switched off")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the benchmark, copy a 1 GiB float64 buffer three times (the "
                         "reference kernel for scaling HBM byte counters)")
    ap.add_argument("--cpu-iters", type=int, nargs=2, default=(3, 9),
                    help="oracle iteration counts of the two timed samples")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ortho_bytes(n, iters, restart=0):
    """Algorithmic HBM bytes of the two Gram-Schmidt passes over all iterations: step j of a
    cycle reads j basis vectors twice plus u, w, z and writes Z[j], v_j, u."""
    tot = 0
    for s in range(iters + 1):
        j = s % restart if restart > 0 else s
        tot += (2 * j + 9) * n * 8
    return tot


def block_ortho_bytes(n, iters, b):
    """Algorithmic HBM bytes of the four passes over the basis of block Gram-Schmidt
    (k_bk_dot twice, k_bk_update twice) over all blocks of b columns: a block starting at
    column j reads V_{0..j} in each pass, the projections read the block's b columns and the
    updates read and write them: (4 (j + 1) + 6 b) * 8 n."""
    tot, j = 0, 0
    while j < iters:
        bb = min(b, iters - j)
        tot += (4 * (j + 1) + 6 * bb) * n * 8
        j += bb
    return tot


def gemm_flops(win, iters, applies_a64):
    """Algorithmic flops of the covariance products: per iteration one A (D and R products)
    and one P_I (D and Rhat^{-1} products), plus float64 residual checks (A only)."""
    s, nb, p = win.s, win.nb, int(win.p[0])
    fa = 2.0 * s * s * nb + 2.0 * p * p * nb
    fp = 2.0 * s * s * nb + 2.0 * p * p * nb
    return (iters + 1) * (fa + fp) + applies_a64 * fa


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the library has no "
                                   "multi-GPU path (independent windows would be placed on "
                                   "different GPUs with no communication)"}))
        sys.exit(2)
    import torch

    from paper_2105_06975_amd import svar, workloads as wl
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.c3:
        print(json.dumps(bench_c3(args)), flush=True)
        return
    if args.c4:
        print(json.dumps(bench_c4(args)), flush=True)
        return
    if args.c5:
        print(json.dumps(bench_c5(args)), flush=True)
        return
    t0 = time.time()
    win = wl.make_config_window("c2", seed=0, nrhs=args.nrhs)
    log(f"workload built in {time.time() - t0:.1f}s: n={win.n}, nrhs={args.nrhs}")
    t0 = time.time()
    h = svar.Handle([win], svar.Precond(type="PI", k=args.k, rhat="RR"))
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    log(f"handle set-up {setup_s:.2f}s")
    R = args.nrhs
    rhs_all = torch.from_numpy(np.ascontiguousarray(win.rhs[:R]).reshape(-1)).to(dev)
    rhs1 = [rhs_all[r * win.n:(r + 1) * win.n] for r in range(R)]

    if args.sweep:
        print(json.dumps(sweep(win, rhs1[0], args)), flush=True)
        return

    def timed(fn, steps, warmup, classes=()):
        for _ in range(warmup):
            fn(0)
        for kc in classes:
            h.timing_enable(kc, True)
            h.timing_read(kc, reset=True)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        outs = [fn(i) for i in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - ts
        tm = {}
        for kc in classes:
            tm[kc] = h.timing_read(kc, reset=True)
            h.timing_enable(kc, False)
        return el, outs, tm

    def breakdown(fn):
        # one extra, untimed call with HIP events around every launch of the three kernel
        # classes (events around every launch cost about 3 %, so the timed region records the
        # Gram-Schmidt class only, which the roofline needs)
        for kc in ("GEMM", "ORTHO", "MODEL"):
            h.timing_enable(kc, True)
            h.timing_read(kc, reset=True)
        fn(0)
        torch.cuda.synchronize()
        out = {}
        for kc in ("GEMM", "ORTHO", "MODEL"):
            out[kc] = h.timing_read(kc, reset=True)
            h.timing_enable(kc, False)
        return out

    # ---- plain FP64, one right-hand side per solve (reference path), with its own tuned plans
    if not args.no_autotune:
        h.autotune(1, "FP64", args.tune_cache)
    xs_plain = {}

    def plain(i):
        r = i % R
        x, info, rc = h.solve(rhs1[r], rtol=args.rtol, maxit=1000)
        assert rc == svar.OK, info
        xs_plain[r] = x
        return info[0]
    nplain = max(args.steps, 2)
    el_p, infos_p, tm_p = timed(plain, nplain, args.warmup, ("ORTHO",) if args.plain_only else ())
    sps_plain = nplain / el_p
    it_plain = float(np.mean([i["iters"] for i in infos_p]))
    log(f"plain FP64: {sps_plain:.3f} solves/s, iters {it_plain:.1f}")
    res = {
        "metric": "saddle solves/sec to 1e-6 rel residual; learned+batched vs plain FP64, 1 GPU",
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c2 window with 8 perturbed-observation rhs: s=4096, N=64, "
                               "p_i=2048 random obs, SOAR B l=0.1, Q=0.1B, SOAR R l=0.05, "
                               "implicit advection-diffusion; P_I with L_M(%d) and R_RR; FGMRES "
                               "to a true relative residual of %g" % (args.k, args.rtol),
                   "n_unknowns_per_rhs": int(win.n), "nrhs": R},
        "plain_fp64": {"value": sps_plain, "iters": it_plain, "ms_per_solve": 1e3 / sps_plain,
                       "path": "one rhs per FGMRES solve, every operator float64"},
        "setup_s": setup_s,
    }
    if args.plain_only:
        tm, it_main, ntot_main, steps_main, el_main = tm_p, it_plain, win.n, nplain, el_p
        bd = breakdown(plain)
        res.update(value=sps_plain, ms_per_step=1e3 * el_p / nplain)
        res["config"]["path"] = "plain FP64 only"
    else:
        # ---- training (untimed): pairs from plain solves of other seeds of the workload
        from paper_2105_06975_amd import learned
        t0 = time.time()
        tw = [wl.make_config_window("c2", seed=101 + i) for i in range(args.train_windows)]
        chat, cex = learned.harvest_pairs(tw, args.k, rtol=args.rtol, maxit=1000,
                                          cap=args.harvest, block=args.block)
        del tw
        x, y = svar.make_pairs(chat, cex)
        del chat, cex
        t_h = time.time() - t0
        net = svar.Net(args.k, args.n_bound, "BF16")
        net.set_params(wl.net_init(net.cin, 64, seed=0))
        t0 = time.time()
        hist = learned.train(net, x, y, epochs=args.epochs, batch=64, lr=1e-3, seed=0, log=log)
        torch.cuda.synchronize()
        t_t = time.time() - t0
        npairs = int(x.shape[0])
        del x, y
        torch.cuda.empty_cache()
        log(f"training: {npairs} pairs harvested in {t_h:.1f}s, {args.epochs} epochs in "
            f"{t_t:.1f}s, loss {hist[0]:.4f} -> {hist[-1]:.4f}")
        h.set_net(net)
        t_tune = 0.0
        if not args.no_autotune:
            t0 = time.time()
            h.autotune(R, args.precision, args.tune_cache)
            t_tune = time.time() - t0
            log(f"GEMM autotuning for {R} rhs: {t_tune:.1f}s")
        # ---- learned + batched
        kw = dict(rtol=args.rtol, maxit=700, fallback_patience=args.patience, block=args.block)
        if args.lb_restart > 0:
            kw.update(restart=args.lb_restart, max_outer=100, maxit=2000)
        if args.precision != "FP64":
            kw["precision"] = args.precision

        def batched(i):
            x, infos, rc = h.solve(rhs_all, R, **kw)
            assert rc == svar.OK, infos
            return x, infos
        el_b, outs, tm = timed(batched, args.steps, args.warmup, ("ORTHO",))
        bd = breakdown(batched)
        xb, infos_b = outs[-1]
        sps = R * args.steps / el_b
        it_b = float(np.mean([i["iters"] for i in infos_b]))
        # agreement with the plain float64 solutions (both at the same true residual)
        errs = []
        for r, xp in xs_plain.items():
            a = xb[r * win.n:(r + 1) * win.n]
            errs.append(float(torch.linalg.norm(a - xp) / torch.linalg.norm(xp)))
        log(f"learned+batched: {sps:.3f} solves/s, iters {it_b:.1f}, "
            f"x vs plain {max(errs):.1e}")
        res.update(value=sps, ms_per_step=1e3 * el_b / args.steps)
        res["config"]["path"] = ("learned + batched: 8 rhs per call, network correction of "
                                 "the Lhat^-T sweep (bf16 MFMA), %s, %s"
                                 % (args.precision, ("s-step FGMRES, blocks of %d" % args.block
                                     if args.block >= 2 else "one column per step")
                                    + (", restart %d" % args.lb_restart if args.lb_restart > 0
                                       else "")))
        res["speedup_vs_plain_fp64"] = sps / sps_plain
        res["learned_batched"] = {
            "iters_mean": it_b, "fallbacks": int(sum(i["fallbacks"] for i in infos_b)),
            "relres_true_max": float(max(i["relres_true"] for i in infos_b)),
            "x_rel_diff_vs_plain_fp64_max": max(errs),
            "autotune_s": t_tune, "n_bound": args.n_bound,
            "training": {"pairs": npairs, "windows": args.train_windows, "epochs": args.epochs,
                         "harvest_s": t_h, "train_s": t_t, "loss_first": hist[0],
                         "loss_last": hist[-1]}}
        tm, it_main, ntot_main, steps_main, el_main = tm, it_b, win.n * R, args.steps, el_b
        if args.plain_block >= 2:
            # context, not `value`: the batched solve without the network, s-step FGMRES
            h.set_net(None)
            kwp = dict(rtol=args.rtol, maxit=700, block=args.plain_block)
            if args.precision != "FP64":
                kwp["precision"] = args.precision

            def pblock(i):
                x, infos, rc = h.solve(rhs_all, R, **kwp)
                assert rc == svar.OK, infos
                return infos
            el_pb, outs_pb, _ = timed(pblock, args.steps, 1)
            infos_pb = outs_pb[-1]
            res["plain_batched_block"] = {
                "value": R * args.steps / el_pb, "unit": "solves/s",
                "iters_mean": float(np.mean([i["iters"] for i in infos_pb])),
                "relres_true_max": float(max(i["relres_true"] for i in infos_pb)),
                "path": "plain P_I (no network), 8 rhs per call, %s, s-step FGMRES with blocks "
                        "of %d" % (args.precision, args.plain_block)}
            log(f"plain+batched, blocks of {args.plain_block}: "
                f"{res['plain_batched_block']['value']:.3f} solves/s")
    res["iters"] = it_main
    # roofline of the dominant kernel class (by measured time in the timed region)
    oms, ol = tm["ORTHO"]
    gms, gl = bd["GEMM"]
    res["kernel_time_ms"] = {
        "ortho": oms, "ortho_launches": ol, "timed_region_ms": 1e3 * el_main,
        "one_instrumented_solve": {"gemm": gms, "gemm_launches": gl, "ortho": bd["ORTHO"][0],
                                   "ortho_launches": bd["ORTHO"][1],
                                   "model_and_net": bd["MODEL"][0],
                                   "model_launches": bd["MODEL"][1]},
        "note": "ortho: HIP events around every Gram-Schmidt launch of the timed region; "
                "one_instrumented_solve: one more call of the timed path with events around "
                "every launch of all three classes"}
    blk = args.block if (not args.plain_only and args.block >= 2) else 0
    if bd["ORTHO"][0] >= gms and blk:
        # four timed launches per block: the two projections and the two updates
        byts = block_ortho_bytes(ntot_main, int(round(it_main)), blk) * steps_main
        ach = byts / (oms * 1e-3) / 1e9
        per_launch = byts / max(ol, 1)
        res["roofline"] = {"bound": "hbm",
                           "kernel": "k_bk_dot + k_bk_update (block Gram-Schmidt passes over "
                                     "the basis)",
                           "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS,
                           "traffic": (BLOCK_TRAFFIC_RATIO * per_launch
                                       if BLOCK_TRAFFIC_RATIO and blk == BLOCK_TRAFFIC_B else None),
                           "traffic_note": "HBM bytes per launch: measured/algorithmic ratio of "
                                           "the byte counters (calibrated) times this run's "
                                           "algorithmic bytes per launch",
                           "algorithmic_bytes_per_launch": per_launch,
                           "launches": ol, "avg_ms": oms / max(ol, 1)}
    elif bd["ORTHO"][0] >= gms:
        byts = ortho_bytes(ntot_main, int(round(it_main)),
                           0 if args.plain_only else args.lb_restart) * steps_main
        ach = byts / (oms * 1e-3) / 1e9
        per_launch = byts / max(ol, 1)
        res["roofline"] = {"bound": "hbm", "kernel": "k_fg_dot + k_fg_update (Gram-Schmidt)",
                           "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS,
                           "traffic": ORTHO_TRAFFIC_RATIO * per_launch,
                           "traffic_note": "HBM bytes per launch: measured/algorithmic ratio of the "
                                           "byte counters (calibrated) times this run's "
                                           "algorithmic bytes per launch",
                           "algorithmic_bytes_per_launch": per_launch,
                           "launches": ol, "avg_ms": oms / max(ol, 1)}
    else:
        flops = gemm_flops(win, int(round(it_main)), 2) * (R if ntot_main > win.n else 1)
        ach = flops / (gms * 1e-3) / 1e12
        res["roofline"] = {"bound": "mfma", "kernel": "k_gemm (covariance products)",
                           "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": ach / FP64_PEAK_TFLOPS, "traffic": None,
                           "launches": gl, "avg_ms": gms / max(gl, 1)}
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(win, args, int(round(it_plain)))
    print(json.dumps(res), flush=True)
    if args.calib_copy:
        # reference for the byte counters: an elementwise map that reads 1 GiB and writes 1 GiB
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()


def bench_c3(args):
    """Lorenz-96 configuration: s = 2048, F = 8, RK4 dt = 0.025, 8 steps per observation
    interval, N = 32, every 4th variable observed, Gaussian R (4 cells), B SOAR(0.1), Q = 0.05 B.
    Reports iterations / time of the first inner solve for several k, then the 5-iteration
    Gauss-Newton loop (forecast, right-hand side, solve, update all on the GPU)."""
    import torch

    from paper_2105_06975_amd import svar, workloads as wl
    from paper_2105_06975_amd.gauss_newton import gauss_newton
    t0 = time.time()
    win = wl.make_l96_window(s=2048, N=32, seed=0)
    log(f"c3 workload built in {time.time() - t0:.1f}s, n={win.n}")
    rhs = torch.from_numpy(win.rhs[0]).cuda()
    out = {"workload": "c3 lorenz-96 s=2048 N=32 dt=0.025x8 p=512", "inner": [], "outer": None}
    for k in (3, 8, win.N + 1):
        h = svar.Handle([win], svar.Precond(type="PI", k=k, rhat="RR"))
        h.solve(rhs, rtol=args.rtol, maxit=3000)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, info, rc = h.solve(rhs, rtol=args.rtol, maxit=3000)
        torch.cuda.synchronize()
        r = dict(k=k, rc=rc, iters=info[0]["iters"], ms=1e3 * (time.perf_counter() - t),
                 relres=info[0]["relres_true"])
        out["inner"].append(r)
        log(r)
    h = svar.Handle([win], svar.Precond(type="PI", k=win.N + 1, rhat="RR"))
    torch.cuda.synchronize()
    t = time.perf_counter()
    xg, hist = gauss_newton(h, win, n_outer=5, solve_kw=dict(rtol=args.rtol, maxit=3000))
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    truth = np.asarray(win.meta["truth"])
    err0 = float(np.linalg.norm(np.asarray(win.model["traj"]) - truth) / np.linalg.norm(truth))
    err = float(np.linalg.norm(xg.cpu().numpy().reshape(truth.shape) - truth)
                / np.linalg.norm(truth))
    out["outer"] = dict(k=win.N + 1, seconds=el, iters=[r["iters"] for r in hist],
                        rc=[r["rc"] for r in hist], norm_dx=[r["norm_dx"] for r in hist],
                        norm_rhs=[r["norm_rhs"] for r in hist], rel_err_first_guess=err0,
                        rel_err_analysis=err)
    log(out["outer"])
    return out


def c4_windows(nwin, seed=0, nrhs=8):
    """Uneven windows: s ~ U{256..4096}, N ~ U{8..64}, p = floor(s f) with f ~ U[1/8, 1/2]
    random observation points (fixed in time), SOAR R (0.05, 0.5), 8 right-hand sides whose
    observation noise is redrawn from R."""
    from paper_2105_06975_amd import workloads as wl
    rng = np.random.default_rng(np.random.SeedSequence([seed, 4]))
    wins = []
    for w in range(nwin):
        s = int(rng.integers(256, 4097))
        N = int(rng.integers(8, 65))
        f = float(rng.uniform(1 / 8, 1 / 2))
        p = max(1, int(np.floor(s * f)))
        idx = wl.obs_indices(s, "random", rng, p=p)
        wins.append(wl.make_advdiff_window(s, N, idx, r_len=0.05, r_var=0.5, nrhs=nrhs,
                                           seed=1000 * 4 + w))
    return wins


def train_c5_net(args):
    """The network of the C5 shape (s = 4096, N = 32): pairs from plain solves of seeds
    0..train_windows-1, Adam epochs (untimed)."""
    from paper_2105_06975_amd import learned, svar
    from paper_2105_06975_amd import workloads as wl
    t0 = time.time()
    tw = [wl.make_c5_like(4096, 32, seed=sd) for sd in range(args.train_windows)]
    chat, cex = learned.harvest_pairs(tw, args.k, rtol=args.rtol, maxit=1000, cap=args.harvest)
    del tw
    x, y = svar.make_pairs(chat, cex)
    del chat, cex
    net = svar.Net(args.k, args.n_bound, "BF16")
    net.set_params(wl.net_init(net.cin, 64, seed=0))
    hist = learned.train(net, x, y, epochs=args.epochs, batch=64, lr=1e-3, seed=0)
    t_train = time.time() - t0
    log(f"c5 training: {x.shape[0]} pairs, loss {hist[0]:.4f} -> {hist[-1]:.4f}, {t_train:.1f}s")
    return net, hist, t_train


def bench_c5(args):
    """Learned correction on the C5 shape: training on seeds 0..2 (untimed), evaluation on
    held-out seeds 10^6 + w, 8 rhs each: the learned + batched solve (FP64_F32P, restart as
    the main path) against plain FP64 solves of every system one at a time."""
    import torch

    from paper_2105_06975_amd import svar
    from paper_2105_06975_amd import workloads as wl
    s, N, nrhs = 4096, 32, 8
    net, hist, t_train = train_c5_net(args)
    wins = [wl.make_c5_like(s, N, seed=10**6 + w, nrhs=nrhs) for w in range(args.c5)]
    prec = svar.Precond(type="PI", k=args.k, rhat="RR")
    rhs = torch.from_numpy(np.concatenate([w.rhs.reshape(-1) for w in wins])).cuda()
    # plain FP64, one system at a time (the reference path: no restart)
    one_t, its1 = 0.0, []
    for w in wins:
        hw = svar.Handle([w], prec)
        for r in range(nrhs):
            b = torch.from_numpy(w.rhs[r]).cuda()
            if r == 0:
                hw.solve(b, 1, rtol=args.rtol, maxit=1000)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, inf1, rc1 = hw.solve(b, 1, rtol=args.rtol, maxit=1000)
            torch.cuda.synchronize()
            one_t += time.perf_counter() - t
            assert rc1 == svar.OK, inf1
            its1.append(inf1[0]["iters"])
        hw.close()
    # learned + batched
    h = svar.Handle(wins, prec)
    h.set_net(net)
    kw = dict(rtol=args.rtol, maxit=2000, precision=args.precision,
              fallback_patience=args.patience)
    if args.lb_restart > 0:
        kw.update(restart=args.lb_restart, max_outer=100)
    h.solve(rhs, nrhs, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter()
    xb, infb, rcb = h.solve(rhs, nrhs, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    nsys = len(infb)
    res = {"workload": f"c5: {args.c5} held-out windows (s={s}, N={N}, p=s/2) x {nrhs} rhs",
           "training": {"windows": args.train_windows, "epochs": args.epochs,
                        "loss_first": hist[0], "loss_last": hist[-1], "seconds": t_train},
           "plain_fp64_one_at_a_time": {"systems": len(its1), "solves_per_s": len(its1) / one_t,
                                        "iters_mean": float(np.mean(its1))},
           "learned_batched": {"systems": nsys, "solves_per_s": nsys / el, "rc": rcb,
                               "iters_mean": float(np.mean([i["iters"] for i in infb])),
                               "fallbacks": int(sum(i["fallbacks"] for i in infb)),
                               "relres_max": float(max(i["relres_true"] for i in infb))}}
    res["speedup"] = res["learned_batched"]["solves_per_s"] / \
        res["plain_fp64_one_at_a_time"]["solves_per_s"]
    log(res)
    return res


def bench_c4(args):
    import torch

    from paper_2105_06975_amd import svar
    nrhs = 8
    t0 = time.time()
    wins = c4_windows(args.c4, nrhs=nrhs)
    log(f"c4: {len(wins)} windows built in {time.time() - t0:.1f}s; "
        f"n per rhs: {[w.n for w in wins]}")
    prec = svar.Precond(type="PI", k=args.k, rhat="RR")
    kw = dict(rtol=args.rtol, maxit=3000, restart=args.restart, max_outer=400)
    t0 = time.time()
    h = svar.Handle(wins, prec)
    log(f"c4 set-up {time.time() - t0:.1f}s")
    rhs = torch.from_numpy(np.concatenate([w.rhs.reshape(-1) for w in wins])).cuda()

    def timed_solve(**extra):
        h.solve(rhs, nrhs, **kw, **extra)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, info, rc = h.solve(rhs, nrhs, **kw, **extra)
        torch.cuda.synchronize()
        return time.perf_counter() - t, x, info, rc

    el, x, info, rc = timed_solve()
    its = [i["iters"] for i in info]
    res = {"workload": f"c4 wave: {len(wins)} uneven windows x {nrhs} rhs, restart {args.restart}",
           "batched": {"systems": len(info), "seconds": el, "solves_per_s": len(info) / el,
                       "rc": rc, "iters_mean": float(np.mean(its)), "iters_max": int(max(its)),
                       "relres_max": float(max(i["relres_true"] for i in info)),
                       "n_total": int(sum(w.n for w in wins) * nrhs)}}
    log(res["batched"])
    # the same batch with graph-captured FGMRES step chunks, then with autotuned GEMM plans
    el_g, xg, info_g, rc_g = timed_solve(graph=True)
    res["batched_graph"] = {"seconds": el_g, "solves_per_s": len(info) / el_g, "rc": rc_g,
                            "identical_x": bool(torch.equal(xg, x))}
    log(res["batched_graph"])
    t0 = time.time()
    h.autotune(nrhs, "FP64", args.tune_cache)
    t_tune = time.time() - t0
    el_t, xt, info_t, rc_t = timed_solve(graph=True)
    res["batched_graph_autotuned"] = {"seconds": el_t, "solves_per_s": len(info) / el_t,
                                      "rc": rc_t, "autotune_s": t_tune,
                                      "x_rel_diff": float(torch.linalg.norm(xt - x) /
                                                          torch.linalg.norm(x))}
    log(res["batched_graph_autotuned"])
    if args.c4_block >= 2:
        el_k, xk, info_k, rc_k = timed_solve(block=args.c4_block)
        res["batched_block"] = {"block": args.c4_block, "seconds": el_k,
                                "solves_per_s": len(info) / el_k, "rc": rc_k,
                                "iters_mean": float(np.mean([i["iters"] for i in info_k])),
                                "relres_max": float(max(i["relres_true"] for i in info_k)),
                                "x_rel_diff": float(torch.linalg.norm(xk - x) /
                                                    torch.linalg.norm(x))}
        log(res["batched_block"])
    if args.c4_learned:
        # the network trained on the C5 shape, applied to this batch (a convolution over space
        # with per-block inputs does not depend on s or N)
        net, hist, t_train = train_c5_net(args)
        h.set_net(net)
        el_l, xl, info_l, rc_l = timed_solve(precision=args.precision,
                                             fallback_patience=args.patience)
        h.set_net(None)
        res["learned_batched"] = {"seconds": el_l, "solves_per_s": len(info) / el_l, "rc": rc_l,
                                  "precision": args.precision,
                                  "iters_mean": float(np.mean([i["iters"] for i in info_l])),
                                  "fallbacks": int(sum(i["fallbacks"] for i in info_l)),
                                  "relres_max": float(max(i["relres_true"] for i in info_l)),
                                  "training": {"loss_first": hist[0], "loss_last": hist[-1],
                                               "seconds": t_train}}
        log(res["learned_batched"])
    # one at a time: the first two windows' 16 systems (same preconditioner and restart)
    sub = wins[:2]
    hs = svar.Handle(sub, prec)
    one_t = 0.0
    its1 = []
    for wi, w in enumerate(sub):
        hw = svar.Handle([w], prec)
        for r in range(nrhs):
            b = torch.from_numpy(w.rhs[r]).cuda()
            hw.solve(b, 1, **kw) if r == 0 else None
            torch.cuda.synchronize()
            t = time.perf_counter()
            xx, inf1, rc1 = hw.solve(b, 1, **kw)
            torch.cuda.synchronize()
            one_t += time.perf_counter() - t
            its1.append(inf1[0]["iters"])
    rhs_sub = torch.from_numpy(np.concatenate([w.rhs.reshape(-1) for w in sub])).cuda()
    hs.solve(rhs_sub, nrhs, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter()
    xs, infs, rcs = hs.solve(rhs_sub, nrhs, **kw)
    torch.cuda.synchronize()
    el_sub = time.perf_counter() - t
    res["subset"] = {"systems": 2 * nrhs, "one_at_a_time_s": one_t, "batched_s": el_sub,
                     "batched_speedup": one_t / el_sub, "iters_one": its1,
                     "iters_batched": [i["iters"] for i in infs]}
    if "learned_batched" in res:
        # the whole batch learned + batched against the one-at-a-time plain FP64 rate
        res["learned_batched_vs_one_at_a_time"] = (res["learned_batched"]["solves_per_s"] /
                                                   (2 * nrhs / one_t))
    log(res["subset"])
    return res


def sweep(win, rhs, args):
    """Iterations and time per solve (second of two identical solves) over k, restart length
    and precision on the benchmark window."""
    import torch

    from paper_2105_06975_amd import svar
    out = []

    def one(h, **kw):
        h.solve(rhs, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, info, rc = h.solve(rhs, **kw)
        torch.cuda.synchronize()
        return dict(rc=rc, iters=info[0]["iters"], outer=info[0]["outer"],
                    ms=1e3 * (time.perf_counter() - t), relres=info[0]["relres_true"])

    for k in (1, 2, 3, 4, 6, 8, 16, win.N + 1):
        h = svar.Handle([win], svar.Precond(type="PI", k=k, rhat="RR"))
        r = one(h, rtol=args.rtol, maxit=1500)
        r.update(k=k, restart=0, precision="FP64")
        out.append(r)
        log(r)
        if k in (3, 16):
            for rs in (50, 100, 200):
                r = one(h, rtol=args.rtol, maxit=3000, restart=rs, max_outer=200)
                r.update(k=k, restart=rs, precision="FP64")
                out.append(r)
                log(r)
            for prec, kw in (("FP64_F32P", {}),
                             ("MIXED_FP32", dict(inner_rtol=1e-5, max_outer=6)),
                             ("MIXED_BF16P", dict(inner_rtol=1e-5, max_outer=6))):
                r = one(h, rtol=args.rtol, maxit=3000, precision=prec, **kw)
                r.update(k=k, restart=0, precision=prec)
                out.append(r)
                log(r)
        del h
    return {"sweep": out, "workload": "c2", "rtol": args.rtol}


def cpu_baseline(win, args, gpu_iters):
    """The float64 oracle on the host cores: FGMRES timed for two short iteration counts
    (operator cost a per iteration, Gram-Schmidt cost b per basis vector), extrapolated to
    the GPU's iteration count: T(I) = a I + b I^2 / 2.  Set-up is excluded on both sides."""
    from oracle import svar_oracle as so
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    orc = so.SaddleOracle(win, k=args.k, rhat="RR")
    rhs = win.rhs[0]
    times = []
    m1, m2 = args.cpu_iters
    for m in (m1, m2):
        t = time.perf_counter()
        so.fgmres(orc.apply_A, orc.apply_PI_inv, rhs, 1e-30, m)
        times.append(time.perf_counter() - t)
        log(f"  oracle {m} iterations: {times[-1]:.2f}s")
    # T(m) = a m + b m^2 / 2
    M = np.array([[m1, m1 * m1 / 2.0], [m2, m2 * m2 / 2.0]])
    a, b = np.linalg.solve(M, np.array(times))
    a, b = max(a, 1e-9), max(b, 0.0)
    t_solve = a * gpu_iters + b * gpu_iters ** 2 / 2.0
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle FGMRES timed at {m1} and {m2} iterations on the same window "
                      f"({sum(times):.1f}s), extrapolated to {gpu_iters} iterations",
            "sec_per_solve": t_solve}


if __name__ == "__main__":
    main()
