"""Benchmark: preconditioned saddle-point solves per second on one MI355X.

Headline workload (default): the uneven batch of 512 linear advection-diffusion windows
(s ~ U{256..4096}, N ~ U{8..64}, p_i = floor(s f) random observation points with
f ~ U[1/8, 1/2], dense SOAR B (length 0.1), Q_i = 0.1 B, dense SOAR R_i (length 0.05)), each
with 8 perturbed-observation right-hand sides (0; d_r; 0): 4096 saddle systems, about 9e8
unknowns.  Inexact-constraint preconditioner P_I with L_M(3) and the ridge-regression Rhat,
FGMRES restarted every 20 steps (both paths), stop at a 5e-7 true relative residual (every
solution then within 1e-6 of the float64 reference; the metric asks for 1e-6), x0 = 0.

  * plain FP64 (the reference rate): one system per solve, every operator float64, timed
    on a stratified sample of the windows (every 16th by size, one rhs each);
  * learned + batched (`value`): all 4096 systems per call in waves that fit the device
    memory, the network correction of the Lhat^{-T} sweep (trained beforehand, untimed, on
    pairs harvested from plain solves of s = 4096, N = 32 windows; a convolution over space
    with per-block inputs applies to any s and N), float32 Rhat^{-1} products in P, A in
    float64; converged systems and windows retire from every launch;
  * plain batched (context): the same batched solve without the network.
One step = one batched solve of all 4096 systems.

Other modes: --c2 (one s = 4096, N = 64 window x 8 rhs), --c3 (Lorenz-96 Gauss-Newton),
--c5 (learned correction on held-out s = 4096, N = 32 windows), --sweep (k, restart,
precision on the C2 window).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--windows W] [--no-cpu]
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
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0,
                    help="untimed full steps before the timed ones (a short priming solve "
                         "that builds the launch programs and workspaces always runs)")
    ap.add_argument("--rtol", type=float, default=5e-7,
                    help="true relative residual of every path (5e-7 keeps every solution "
                         "within 1e-6 of the float64 reference)")
    ap.add_argument("--k", type=int, default=3)
    ap.add_argument("--restart", type=int, default=20,
                    help="FGMRES restart length of every path")
    ap.add_argument("--windows", type=int, default=512, help="windows of the headline batch")
    ap.add_argument("--base-sample", type=int, default=32,
                    help="windows (stratified by size, one rhs each) of the one-at-a-time "
                         "plain FP64 sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain-batched", action="store_true")
    ap.add_argument("--c2", action="store_true",
                    help="one s=4096, N=64 window x 8 rhs instead of the batch (one JSON line)")
    ap.add_argument("--sweep", action="store_true",
                    help="print iterations and time per solve over k, restart length and "
                         "precision on the C2 window (one JSON object)")
    ap.add_argument("--c3", action="store_true",
                    help="Lorenz-96 window (s=2048, N=32): iterations vs k and the 5-iteration "
                         "Gauss-Newton outer loop (one JSON object)")
    ap.add_argument("--replay", choices=["A", "B"], default=None,
                    help="the paper's experiments on their own recipes: A = Lorenz-96 (s=2500, "
                         "N=15, dt=1e-4), B = heat equation (s=10000, N=5); iterations for "
                         "P_D (MINRES) and P_I (FGMRES) over k and Rhat (one JSON object)")
    ap.add_argument("--replay-s", type=int, default=0, help="--replay: state size override")
    ap.add_argument("--replay-subset", default="",
                    help="--replay: comma-separated preconditioners / Rhat kinds / k values to "
                         "run, e.g. PI,BLOCK,DIAG,1,3,4,16 (default: all)")
    ap.add_argument("--grid", action="store_true",
                    help="the C2 window with R lengths 0.01, 0.05, 0.2: iterations and time of "
                         "P_D (MINRES, float64) and P_I (FGMRES, float64 and bfloat16 P "
                         "products) over k and Rhat (one JSON object)")
    ap.add_argument("--c5", type=int, default=0, metavar="W",
                    help="learned-correction mode: train on C5-shaped windows (s=4096, N=32), "
                         "then solve W held-out windows x 8 rhs batched with and without the "
                         "network against every system one at a time in plain FP64")
    ap.add_argument("--tune-cache", default=None, help="JSON file for the GEMM autotuning cache")
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--precision", default="MIXED_F32",
                    help="precision of the batched paths (MIXED_F32: float32 covariance "
                         "products in A and P inside the float64 restart loop)")
    ap.add_argument("--block", type=int, default=0,
                    help="s-step FGMRES block size of the batched paths (0: one column at a "
                         "time; with the nonlinear network the block basis stagnates)")
    ap.add_argument("--block-rhs", type=int, default=2, choices=(0, 1, 2),
                    help="the batched paths run block FGMRES over the 8 right-hand sides of "
                         "each window (one Krylov space per window) with 2 (1) or 1 (2) "
                         "Gram-Schmidt passes per step; 0: one Krylov space per system")
    ap.add_argument("--train-windows", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--harvest", type=int, default=300, help="pairs harvested per window")
    ap.add_argument("--plain-only", action="store_true",
                    help="--c2: time only the plain FP64 path (no training)")
    ap.add_argument("--n-bound", type=int, default=8,
                    help="later segment starts the network sees (1 + n_bound + k <= 32)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="--c2: skip the GEMM autotuning of the batched path")
    ap.add_argument("--patience", type=int, default=20,
                    help="failing FGMRES steps in a row before the network is switched off")
    ap.add_argument("--maxit", type=int, default=6000, help="iterations allowed per system")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="host time budget of the oracle sample")
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


def gemm_flops(win, iters, applies_a64):
    """Algorithmic flops of the covariance products of one system of a C2-mode solve: per
    FGMRES step one P_I (D z1, float64, shared with the next A z; Rhat^{-1}) and one A (R;
    D z1 reused), plus a float64 A (D and R) per true-residual check."""
    s, nb, p = win.s, win.nb, int(win.p[0])
    step = 2.0 * s * s * nb + 4.0 * p * p * nb
    fa = 2.0 * s * s * nb + 2.0 * p * p * nb
    return iters * step + applies_a64 * fa


NET_FLOP_PER_POINT = 2 * (5 * 32 * 64 + 2 * 5 * 64 * 64 + 5 * 64)  # 103,040 (padded layer 1)


def batch_work(wins, infos, nrhs, restart, block_rhs=0, precision="FP64_F32P"):
    """Algorithmic work of a batched solve from its per-system iteration counts.

    Covariance products (flops): a window's products run while any of its right-hand sides
    is active (max over its rhs of the steps, plus one float64 A per cycle and one at the
    end): per step 2 (s^2 + p^2)(N+1) nrhs float64 (D z1, R) and 2 p^2 (N+1) nrhs float32
    (Rhat^{-1}); per check 2 (s^2 + p^2)(N+1) nrhs float64.  Gram-Schmidt bytes per system:
    step t of a cycle (j = t mod restart) reads j basis vectors twice plus u, w, z and
    writes Z_j, v_j, u: (2 j + 9) 8 n.  Block mode over the rhs (block_rhs = 1: two passes,
    2: one pass) per window and block step j: each pass reads the j + 1 basis blocks twice (the
    projections and the update) and the new block three times (read twice, written once):
    passes (2 j + 5) nrhs 8 n.  Network flops: NET_FLOP_PER_POINT per grid point of every
    active system's state per step."""
    f64 = f32 = gsb = net = 0.0
    for w, win in enumerate(wins):
        inf = infos[w * nrhs:(w + 1) * nrhs]
        s, nb, p = win.s, win.nb, int(win.p[0])
        steps = max(i["iters"] for i in inf)
        checks = max(i["outer"] for i in inf) + 1
        if precision == "MIXED_F32":   # every inner product float32, the checks float64
            f64 += checks * 2.0 * (s * s + p * p) * nb * nrhs
            f32 += steps * 2.0 * (s * s + 2 * p * p) * nb * nrhs
        else:
            f64 += (steps + checks) * 2.0 * (s * s + p * p) * nb * nrhs
            f32 += steps * 2.0 * p * p * nb * nrhs
        if block_rhs:
            passes = 2 if block_rhs == 1 else 1
            full, rem = divmod(steps, restart) if restart > 0 else (0, steps)
            m = restart if restart > 0 else steps
            per = lambda J: sum(passes * (2 * j + 5) for j in range(J))
            gsb += (full * per(m) + per(rem)) * nrhs * 8.0 * win.n
        for i in inf:
            it = i["iters"]
            if not block_rhs:
                full, rem = divmod(it, restart) if restart > 0 else (0, it)
                m = restart if restart > 0 else it
                per_cycle = sum(2 * j + 9 for j in range(m))
                gsb += (full * per_cycle + sum(2 * j + 9 for j in range(rem))) * 8.0 * win.n
            net += it * float(NET_FLOP_PER_POINT) * nb * s
    return dict(gemm_f64=f64, gemm_f32=f32, ortho_bytes=gsb, net_flops=net)


def threads_in_use():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def main():
    args = parse()
    # the library reports long solves on stderr (at most one line every 20 s)
    os.environ.setdefault("SVAR_PROGRESS", "1")
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the library has no "
                                   "multi-GPU path (independent windows would be placed on "
                                   "different GPUs with no communication)"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.c3:
        print(json.dumps(bench_c3(args)), flush=True)
        return
    if args.c5:
        print(json.dumps(bench_c5(args)), flush=True)
        return
    if args.replay:
        print(json.dumps(bench_replay(args)), flush=True)
        return
    if args.grid:
        print(json.dumps(bench_grid(args)), flush=True)
        return
    if args.c2 or args.sweep:
        bench_c2(args)
        return
    print(json.dumps(bench_headline(args)), flush=True)


def bench_c2(args):
    """One s = 4096, N = 64 window with 8 right-hand sides: plain FP64 one rhs per solve
    against learned + batched, both with FGMRES(restart)."""
    import torch

    from paper_2105_06975_amd import svar, workloads as wl
    dev = torch.device("cuda:0")
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
        for kc in ("GEMM", "ORTHO", "MODEL", "NET"):
            h.timing_enable(kc, True)
            h.timing_read(kc, reset=True)
        fn(0)
        torch.cuda.synchronize()
        out = {}
        for kc in ("GEMM", "ORTHO", "MODEL", "NET"):
            out[kc] = h.timing_read(kc, reset=True)
            h.timing_enable(kc, False)
        return out

    # ---- plain FP64, one right-hand side per solve (reference path), with its own tuned plans
    if not args.no_autotune:
        h.autotune(1, "FP64", args.tune_cache)
    xs_plain = {}

    def plain(i):
        r = i % R
        x, info, rc = h.solve(rhs1[r], rtol=args.rtol, maxit=args.maxit, restart=args.restart,
                              max_outer=args.maxit)
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
        kw = dict(rtol=args.rtol, maxit=args.maxit, fallback_patience=args.patience,
                  block=args.block, restart=args.restart, max_outer=args.maxit)
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
                                    + ", restart %d" % args.restart))
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
        # context, not `value`: the same batched solve without the network
        h.set_net(None)
        kwp = dict(kw)
        kwp.pop("fallback_patience", None)

        def pbatched(i):
            x, infos, rc = h.solve(rhs_all, R, **kwp)
            assert rc == svar.OK, infos
            return infos
        el_pb, outs_pb, _ = timed(pbatched, args.steps, 1)
        infos_pb = outs_pb[-1]
        res["plain_batched"] = {
            "value": R * args.steps / el_pb, "unit": "solves/s",
            "iters_mean": float(np.mean([i["iters"] for i in infos_pb])),
            "relres_true_max": float(max(i["relres_true"] for i in infos_pb)),
            "path": "plain P_I (no network), 8 rhs per call, %s, restart %d"
                    % (args.precision, args.restart)}
        res["network_gain"] = res["value"] / res["plain_batched"]["value"]
        log(f"plain+batched: {res['plain_batched']['value']:.3f} solves/s")
    res["iters"] = it_main
    oms, ol = tm["ORTHO"]
    gms, gl = bd["GEMM"]
    res["kernel_time_ms"] = {
        "ortho": oms, "ortho_launches": ol, "timed_region_ms": 1e3 * el_main,
        "one_instrumented_solve": {"gemm": gms, "gemm_launches": gl, "ortho": bd["ORTHO"][0],
                                   "ortho_launches": bd["ORTHO"][1],
                                   "model": bd["MODEL"][0], "net": bd["NET"][0]},
        "note": "ortho: HIP events around every Gram-Schmidt launch of the timed region; "
                "one_instrumented_solve: one more call of the timed path with events around "
                "every launch of all classes"}
    byts = ortho_bytes(ntot_main, int(round(it_main)), args.restart) * steps_main
    ach = byts / (oms * 1e-3) / 1e9
    res["roofline"] = {"bound": "hbm", "kernel": "k_fg_dot + k_fg_update (Gram-Schmidt)",
                       "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": ach / HBM_PEAK_GBS, "traffic": None,
                       "algorithmic_bytes_per_launch": byts / max(ol, 1),
                       "launches": ol, "avg_ms": oms / max(ol, 1)}
    print(json.dumps(res), flush=True)


def bench_headline(args):
    """The uneven batch (see the module docstring): plain FP64 one system at a time on a
    stratified sample, learned + batched (`value`) and plain batched on all systems."""
    import torch

    from paper_2105_06975_amd import svar, workloads as wl
    nrhs, m = args.nrhs, args.restart
    t0 = time.time()
    wins = wl.make_c4_batch(args.windows, nrhs=nrhs, workers=min(16, os.cpu_count() or 1))
    t_work = time.time() - t0
    nsys = len(wins) * nrhs
    ntot = sum(w.n for w in wins) * nrhs
    log(f"batch: {len(wins)} windows x {nrhs} rhs, {ntot:.3e} unknowns, drawn in {t_work:.1f}s")
    prec = svar.Precond(type="PI", k=args.k, rhat="RR")
    kw = dict(rtol=args.rtol, maxit=args.maxit, restart=m, max_outer=args.maxit)

    # ---- plain FP64, one system at a time, on a stratified sample (one window per size stratum)
    order = np.argsort([w.n for w in wins], kind="stable")
    ns = min(args.base_sample, len(wins))
    pick = [int(order[(2 * i + 1) * len(wins) // (2 * ns)]) for i in range(ns)]
    one_t, its1, one_ms = 0.0, [], {}
    for wi in pick:
        w = wins[wi]
        hw = svar.Handle([w], prec)
        b = torch.from_numpy(np.ascontiguousarray(w.rhs[0])).cuda()
        hw.solve(b, 1, rtol=args.rtol, maxit=2, restart=m)  # builds programs and workspace
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, inf1, rc1 = hw.solve(b, 1, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        assert rc1 == svar.OK, inf1
        one_t += dt
        its1.append(inf1[0]["iters"])
        one_ms[wi] = 1e3 * dt
        hw.close()
    sps_plain = ns / one_t
    log(f"plain FP64 one at a time: {sps_plain:.2f} solves/s on {ns} sampled systems, "
        f"iters mean {np.mean(its1):.1f}")

    # ---- network trained on the s = 4096, N = 32 shape (untimed)
    net, hist, t_train = train_c5_net(args)
    torch.cuda.empty_cache()

    t0 = time.time()
    h = svar.Handle(wins, prec)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    log(f"batch handle set-up {setup_s:.1f}s")
    rhs_all = torch.from_numpy(np.concatenate([w.rhs.reshape(-1) for w in wins])).cuda()
    kwb = dict(kw, precision=args.precision, block=args.block, block_rhs=args.block_rhs)

    def run(label, attach, classes, steps, warmup):
        h.set_net(attach)
        kk = dict(kwb, fallback_patience=args.patience) if attach else kwb
        t0 = time.time()
        h.solve(rhs_all, nrhs, **dict(kk, maxit=2))  # views, programs, arena
        for _ in range(warmup):
            h.solve(rhs_all, nrhs, **kk)
        torch.cuda.synchronize()
        log(f"{label}: priming and {warmup} warm-up steps {time.time() - t0:.1f}s")
        for kc in classes:
            h.timing_enable(kc, True)
            h.timing_read(kc, reset=True)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(steps):
            x, infos, rc = h.solve(rhs_all, nrhs, **kk)
        torch.cuda.synchronize()
        el = time.perf_counter() - ts
        tm = {}
        for kc in classes:
            tm[kc] = h.timing_read(kc, reset=True)
            h.timing_enable(kc, False)
        assert rc == svar.OK, [i for i in infos if i["status"] != 0][:4]
        its = [i["iters"] for i in infos]
        out = {"value": nsys * steps / el, "unit": "solves/s", "seconds": el,
               "iters_mean": float(np.mean(its)), "iters_max": int(max(its)),
               "relres_true_max": float(max(i["relres_true"] for i in infos)),
               "fallbacks": int(sum(i["fallbacks"] for i in infos))}
        log(f"{label}: {out['value']:.2f} solves/s, iters mean {out['iters_mean']:.1f} "
            f"max {out['iters_max']}")
        return out, infos, tm, el

    classes = ("GEMM", "ORTHO", "MODEL", "NET")
    lb, infos_lb, tm, el = run("learned + batched", net, classes, args.steps, args.warmup)
    res = {
        "metric": "saddle solves/sec to 1e-6 rel residual; learned+batched vs plain FP64, 1 GPU",
        "value": lb["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"MIXED_F32": "f64 (Krylov basis, least squares, restart residuals, model "
                               "products, sweeps) + f32 (every covariance product, MFMA) + bf16 "
                               "(network)",
                  "FP64_F32P": "f64 (Krylov, A, D z1, R) + f32 (Rhat^-1 products) + bf16 "
                               "(network)"}.get(args.precision, args.precision + " + bf16 (network)"),
        "data": "synthetic",
        "config": {"workload": "c4 batch: %d uneven advection-diffusion windows (s~U{256..4096}, "
                               "N~U{8..64}, p=floor(s f), f~U[1/8,1/2]) x %d perturbed-"
                               "observation rhs; SOAR B l=0.1, Q=0.1B, SOAR R l=0.05; P_I with "
                               "L_M(%d) and R_RR; %sFGMRES(%d) to a true relative residual of %g"
                               % (len(wins), nrhs, args.k, "block-over-rhs " if args.block_rhs
                                  else "", m, args.rtol),
                   "windows": len(wins), "nrhs": nrhs, "systems": nsys, "unknowns": int(ntot),
                   "restart": m, "path": "learned + batched: all systems per call in waves, "
                   "%snetwork correction of the Lhat^-T sweep (bf16 MFMA), %s"
                   % ("one block Krylov space per window over its %d rhs (block FGMRES, "
                      "restart %d block steps), " % (nrhs, m) if args.block_rhs else "",
                      args.precision)},
        "speedup_vs_plain_fp64": lb["value"] / sps_plain,
        "plain_fp64": {"value": sps_plain, "unit": "solves/s", "systems": ns,
                       "iters_mean": float(np.mean(its1)), "ms_per_solve": 1e3 * one_t / ns,
                       "sample": "one rhs of each of %d windows, one per stratum of the batch "
                                 "sorted by size; one system per FGMRES(%d) solve, every "
                                 "operator float64" % (ns, m)},
        "learned_batched": dict(lb, training={"pairs_windows": args.train_windows,
                                              "epochs": args.epochs, "seconds": t_train,
                                              "loss_first": hist[0], "loss_last": hist[-1]},
                                n_bound=args.n_bound, patience=args.patience),
        "setup_s": setup_s, "workload_s": t_work,
    }
    # ---- roofline of the class with the largest time in the timed region
    wk = batch_work(wins, infos_lb, nrhs, m, args.block_rhs, args.precision)
    wk = {k: v * args.steps for k, v in wk.items()}
    kt = {k: tm[k][0] for k in classes}
    res["kernel_time_ms"] = {k.lower(): kt[k] for k in classes}
    res["kernel_time_ms"].update(timed_region=1e3 * el, launches={k.lower(): tm[k][1]
                                                                  for k in classes})
    # every class against its own roof (the one with the largest time is `roofline` below)
    t_gpeak = (wk["gemm_f64"] / (FP64_PEAK_TFLOPS * 1e12) +
               wk["gemm_f32"] / (FP32_PEAK_TFLOPS * 1e12))
    gfl = wk["gemm_f64"] + wk["gemm_f32"]
    res["class_rates"] = {
        "gemm_tflops": gfl / max(kt["GEMM"] * 1e-3, 1e-12) / 1e12,
        "gemm_frac": (t_gpeak / max(kt["GEMM"] * 1e-3, 1e-12)) if gfl > 0 else None,
        "ortho_gbs": wk["ortho_bytes"] / max(kt["ORTHO"] * 1e-3, 1e-12) / 1e9,
        "ortho_frac": wk["ortho_bytes"] / max(kt["ORTHO"] * 1e-3, 1e-12) / 1e9 / HBM_PEAK_GBS,
        "net_tflops": wk["net_flops"] / max(kt["NET"] * 1e-3, 1e-12) / 1e12,
        "net_frac": wk["net_flops"] / max(kt["NET"] * 1e-3, 1e-12) / 1e12 / BF16_PEAK_TFLOPS}
    top = max(("GEMM", "ORTHO", "NET"), key=lambda k: kt[k])
    if top == "ORTHO":
        ach = wk["ortho_bytes"] / (kt["ORTHO"] * 1e-3) / 1e9
        res["roofline"] = {"bound": "hbm", "kernel": ("k_bkr_dot + k_bkr_update (block "
                                                      "Gram-Schmidt)" if args.block_rhs else
                                                      "k_fg_dot + k_fg_update (Gram-Schmidt)"),
                           "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": None,
                           "algorithmic": wk["ortho_bytes"], "launches": tm["ORTHO"][1],
                           "avg_ms": kt["ORTHO"] / max(tm["ORTHO"][1], 1)}
    elif top == "GEMM":
        fl = wk["gemm_f64"] + wk["gemm_f32"]
        t_peak = wk["gemm_f64"] / (FP64_PEAK_TFLOPS * 1e12) + wk["gemm_f32"] / (FP32_PEAK_TFLOPS * 1e12)
        peak = fl / t_peak / 1e12
        ach = fl / (kt["GEMM"] * 1e-3) / 1e12
        res["roofline"] = {"bound": "mfma", "kernel": "k_gemm_tiled / k_gemm / k_gemm_lp "
                           "(covariance products: %s)" % (
                               "float32 D z1, R and Rhat^-1; float64 A at the restarts"
                               if args.precision == "MIXED_F32" else
                               "float64 D z1 and R, float32 Rhat^-1"),
                           "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                           "traffic": None, "peak_note": "flop-weighted: float64 at 78.6, "
                           "float32 at 157.3 TFLOP/s", "launches": tm["GEMM"][1],
                           "avg_ms": kt["GEMM"] / max(tm["GEMM"][1], 1)}
    else:
        ach = wk["net_flops"] / (kt["NET"] * 1e-3) / 1e12
        res["roofline"] = {"bound": "mfma", "kernel": "k_net_fused (bf16 network inference)",
                           "achieved": ach, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": ach / BF16_PEAK_TFLOPS, "traffic": None,
                           "launches": tm["NET"][1], "avg_ms": kt["NET"] / max(tm["NET"][1], 1)}
    # ---- context: the same batched solve without the network
    if not args.no_plain_batched:
        pb, _, _, el_pb = run("plain batched", None, (), 1, 0)
        res["plain_batched"] = dict(pb, path="the same batched solve without the network")
        res["network_gain"] = lb["value"] / pb["value"]
        res["speedup_plain_batched_vs_plain_fp64"] = pb["value"] / sps_plain
    h.set_net(None)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline_oracle(wins, pick, one_ms, args)
    return res


def cpu_baseline_oracle(wins, pick, gpu_ms, args):
    """The float64 oracle on the host cores: full FGMRES(restart) solves of the sampled
    windows' first rhs, smallest first, until the time budget is used (at least one)."""
    from oracle import svar_oracle as so
    order = sorted(pick, key=lambda wi: wins[wi].n)
    done, t_tot, its, gpu_same = 0, 0.0, [], 0.0
    for wi in order:
        w = wins[wi]
        orc = so.SaddleOracle(w, k=args.k, rhat="RR")
        t = time.perf_counter()
        x, it, _ = so.fgmres_restarted(orc.apply_A, orc.apply_PI_inv, w.rhs[0], args.rtol,
                                       args.restart, args.maxit)
        t_tot += time.perf_counter() - t
        done += 1
        its.append(it)
        gpu_same += gpu_ms[wi] * 1e-3
        log(f"  oracle: window {wi} (n={w.n}) {it} iterations, {t_tot:.1f}s so far")
        if t_tot >= args.cpu_seconds:
            break
    return {"value": done / t_tot, "unit": "solves/s", "cores": int(threads_in_use()),
            "kind": "oracle", "sample": "full oracle FGMRES(%d) solves of the first rhs of the "
            "%d smallest sampled windows (n = %s), %.1f s of host time; the GPU plain FP64 path "
            "solves the same systems at %.2f solves/s" % (args.restart, done,
                                                          [wins[wi].n for wi in order[:done]],
                                                          t_tot, done / gpu_same),
            "iters": its}


# the paper's iteration counts for Experiment A (s = 2500), derived from Tables 4 and 5 as the
# R_i product totals / 16 (one R_i product per block per iteration), by k
PAPER_EXPA = {"PD": {"DIAG": {1: 1406, 2: 1148, 3: 1043, 4: 823, 7: 736, 10: 595, 16: 220},
                     "BLOCK": {1: 669, 2: 515, 3: 471, 4: 414, 7: 380, 10: 301, 16: 86}},
              "PI": {"DIAG": {1: 539, 2: 443, 3: 394, 4: 379, 7: 329, 10: 315, 16: 274},
                     "BLOCK": {1: 209, 2: 169, 3: 150, 4: 146, 7: 125, 10: 119, 16: 103}}}


def bench_replay(args):
    """Iterations of the paper's two experiments on this library: P_D with MINRES (two-norm
    stop) and P_I with unrestarted FGMRES, rtol 1e-6, over k (Definition 1; k = N + 1 is L) and
    the Rhat kinds, the component product counts per solve, and the time per solve.  The
    instances are seeded draws of the paper's recipe (its own random data are not published),
    so the paper's counts are context for the trends, not targets."""
    import torch

    from paper_2105_06975_amd import svar, workloads as wl
    t0 = time.time()
    if args.replay == "A":
        win = wl.make_expA_window(s=args.replay_s or 2500, N=15)
        ks = [1, 2, 3, 4, 7, 10, 16]
    else:
        win = wl.make_expB_window(s=args.replay_s or 10000, N=5)
        ks = [1, 2, 3, 4, 5, 6]
    log(f"replay {args.replay}: n = {win.n}, drawn in {time.time() - t0:.1f}s")
    rhs = torch.from_numpy(np.ascontiguousarray(win.rhs[0])).cuda()
    pvec = win.meta["pvec"]
    rows = []
    sub = [t for t in args.replay_subset.split(",") if t]
    ptypes = [t for t in ("PD", "PI") if not sub or t in sub or not {"PD", "PI"} & set(sub)]
    rhats = [t for t in ("DIAG", "BLOCK", "RR", "ME", "EXACT")
             if not sub or t in sub or not {"DIAG", "BLOCK", "RR", "ME", "EXACT"} & set(sub)]
    kk = [int(t) for t in sub if t.isdigit()]
    ks = [k for k in ks if not kk or k in kk]
    for ptype in ptypes:
        for rh in rhats:
            for k in ks:
                prec = svar.Precond(type=ptype, k=k, rhat=rh, rb_pvec=pvec, rb_tol=0.05)
                h = svar.Handle([win], prec)
                kw = dict(rtol=1e-6, maxit=3000)
                if ptype == "PD":
                    kw["method"] = "MINRES"
                h.solve(rhs, **dict(kw, maxit=2))
                torch.cuda.synchronize()
                t = time.perf_counter()
                x, info, rc = h.solve(rhs, **kw)
                torch.cuda.synchronize()
                el = time.perf_counter() - t
                i0 = info[0]
                row = dict(prec=ptype, rhat=rh, k=k, iters=i0["iters"], rc=rc,
                           relres=i0["relres_true"], ms=1e3 * el, n_R=i0["n_R"], n_D=i0["n_D"],
                           n_M=i0["n_M"] + i0["n_MT"], n_Rhat_inv=i0["n_Rhat_inv"],
                           n_Dhat_inv=i0["n_Dhat_inv"])
                if args.replay == "A" and rh in ("DIAG", "BLOCK") and k in PAPER_EXPA[ptype][rh]:
                    row["paper_iters"] = PAPER_EXPA[ptype][rh][k]
                rows.append(row)
                log(row)
                h.close()
    return {"replay": args.replay, "n": int(win.n), "s": win.s, "N": win.N,
            "recipe": "Lorenz-96, dt 1e-4, one RK4 step per subwindow" if args.replay == "A"
            else "heat equation, forward Euler r = 0.4, Dirichlet",
            "rows": rows}


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
    held-out seeds 10^6 + w, 8 rhs each: learned + batched and plain batched (the same solve
    without the network) against plain FP64 solves of every system one at a time, all with
    FGMRES(restart)."""
    import torch

    from paper_2105_06975_amd import svar
    from paper_2105_06975_amd import workloads as wl
    s, N, nrhs = 4096, 32, 8
    net, hist, t_train = train_c5_net(args)
    wins = [wl.make_c5_like(s, N, seed=10**6 + w, nrhs=nrhs) for w in range(args.c5)]
    prec = svar.Precond(type="PI", k=args.k, rhat="RR")
    rhs = torch.from_numpy(np.concatenate([w.rhs.reshape(-1) for w in wins])).cuda()
    kw1 = dict(rtol=args.rtol, maxit=args.maxit, restart=args.restart, max_outer=args.maxit)
    one_t, its1 = 0.0, []
    for w in wins:
        hw = svar.Handle([w], prec)
        for r in range(nrhs):
            b = torch.from_numpy(w.rhs[r]).cuda()
            if r == 0:
                hw.solve(b, 1, **kw1)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, inf1, rc1 = hw.solve(b, 1, **kw1)
            torch.cuda.synchronize()
            one_t += time.perf_counter() - t
            assert rc1 == svar.OK, inf1
            its1.append(inf1[0]["iters"])
        hw.close()
    h = svar.Handle(wins, prec)
    kwb = dict(kw1, precision=args.precision, block_rhs=args.block_rhs)
    out = {}
    for name, attach in (("learned_batched", net), ("plain_batched", None)):
        h.set_net(attach)
        kk = dict(kwb, fallback_patience=args.patience) if attach else kwb
        h.solve(rhs, nrhs, **kk)
        torch.cuda.synchronize()
        t = time.perf_counter()
        xb, infb, rcb = h.solve(rhs, nrhs, **kk)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        out[name] = {"systems": len(infb), "solves_per_s": len(infb) / el, "rc": rcb,
                     "iters_mean": float(np.mean([i["iters"] for i in infb])),
                     "fallbacks": int(sum(i["fallbacks"] for i in infb)),
                     "relres_max": float(max(i["relres_true"] for i in infb))}
        log(name, out[name])
    res = {"workload": f"c5: {args.c5} held-out windows (s={s}, N={N}, p=s/2) x {nrhs} rhs, "
                       f"FGMRES({args.restart}) on every path; batched paths {args.precision}, "
                       f"block_rhs {args.block_rhs}",
           "training": {"windows": args.train_windows, "epochs": args.epochs,
                        "loss_first": hist[0], "loss_last": hist[-1], "seconds": t_train},
           "plain_fp64_one_at_a_time": {"systems": len(its1), "solves_per_s": len(its1) / one_t,
                                        "iters_mean": float(np.mean(its1))}, **out}
    one = res["plain_fp64_one_at_a_time"]["solves_per_s"]
    res["speedup_learned_batched"] = out["learned_batched"]["solves_per_s"] / one
    res["speedup_plain_batched"] = out["plain_batched"]["solves_per_s"] / one
    res["network_gain"] = (out["learned_batched"]["solves_per_s"] /
                           out["plain_batched"]["solves_per_s"])
    log(res)
    return res


def bench_grid(args):
    """The C2 window (s = 4096, N = 64, p = 2048) for R lengths 0.01, 0.05 and 0.2 (SOAR,
    reconditioned to kappa <= 1724 where worse): iterations, true residual and time per solve
    of P_D with MINRES (float64) and P_I with FGMRES (float64, and with bfloat16 copies of the
    covariance matrices in P: FP64_BF16P) for k in {1, 3, N + 1} and every Rhat kind."""
    import torch

    from paper_2105_06975_amd import svar, workloads as wl
    rows = []
    for rl in (0.01, 0.05, 0.2):
        win = wl.make_config_window("c2", seed=0, r_len=rl)
        rhs = torch.from_numpy(np.ascontiguousarray(win.rhs[0])).cuda()
        log(f"R length {rl}: recondition shift {win.meta['r_shift']:.3e}")
        for ptype in ("PD", "PI"):
            for rh in ("DIAG", "RR", "ME", "EXACT"):
                for k in (1, 3, win.N + 1):
                    h = svar.Handle([win], svar.Precond(type=ptype, k=k, rhat=rh))
                    precs = ("FP64",) if ptype == "PD" else ("FP64", "FP64_BF16P")
                    for pr in precs:
                        kw = dict(rtol=args.rtol, maxit=3000, precision=pr)
                        if ptype == "PD":
                            kw["method"] = "MINRES"
                        h.solve(rhs, **dict(kw, maxit=2))
                        torch.cuda.synchronize()
                        t = time.perf_counter()
                        _, info, rc = h.solve(rhs, **kw)
                        torch.cuda.synchronize()
                        row = dict(r_len=rl, prec=ptype, rhat=rh, k=k, precision=pr, rc=rc,
                                   iters=info[0]["iters"], relres=info[0]["relres_true"],
                                   ms=1e3 * (time.perf_counter() - t))
                        rows.append(row)
                        log(row)
                    h.close()
    return {"grid": rows, "workload": "c2 window, R length sweep", "rtol": args.rtol}


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


if __name__ == "__main__":
    main()
