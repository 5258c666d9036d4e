"""Outer Gauss-Newton loop of incremental weak-constraint 4D-Var around the saddle solve.

§2.1: each outer loop linearises the model and observation operators about the current
trajectory x^(l), solves the saddle system for the increment and sets x^(l+1) = x^(l) + dx.
With x = (x_0..x_N), the right-hand side (b; d; 0) has
    b_0 = x_b - x_0,   b_i = M_i(x_{i-1}) - x_i  (i = 1..N),   d_i = y_i - H_i x_i.
The right-hand side (svar_gn_rhs), the solve and the update x += dx (svar_gn_update) run in
the HIP library; this module is the loop.
"""
from __future__ import annotations

from typing import Optional


def gauss_newton(handle, win, *, n_outer: int = 5, x0=None, solve_kw: Optional[dict] = None,
                 w: int = 0):
    """Run n_outer Gauss-Newton iterations on window `win` (Lorenz-96 model).

    Returns (x, history) with x the final (N+1) s trajectory (torch, device) and history a list
    of per-outer-iteration solver info dicts (plus |dx| and |rhs|)."""
    import numpy as np
    import torch
    s, nb = win.s, win.nb
    dev = torch.device("cuda")
    kw = dict(rtol=1e-6, maxit=1000)
    kw.update(solve_kw or {})
    x = torch.from_numpy(np.ascontiguousarray(win.model["traj"] if x0 is None else x0,
                                              dtype=np.float64).reshape(-1)).to(dev).clone()
    xb = torch.from_numpy(np.asarray(win.meta["xb"], dtype=np.float64)).to(dev)
    y = torch.from_numpy(np.asarray(win.meta["y"], dtype=np.float64).reshape(-1)).to(dev)
    hist = []
    handle.set_trajectory(x, w)
    for _ in range(n_outer):
        rhs = handle.gn_rhs(x, xb, y, w)
        dx, info, rc = handle.solve(rhs, **kw)
        handle.gn_update(x, dx, w)
        rec = dict(info[0])
        rec.update(rc=rc, norm_dx=float(dx[-nb * s:].norm()), norm_rhs=float(rhs.norm()))
        hist.append(rec)
    return x, hist
