"""Lorenz-96 model, tangent linear and adjoint for the oracle (TEST INFRASTRUCTURE ONLY).

§7.1: dx_j/dt = (x_{j+1} - x_{j-2}) x_{j-1} - x_j + F on a periodic ring of s variables,
integrated with the classical fourth-order Runge-Kutta scheme.  M_i, the linearised model of
the window, is the Jacobian of nsteps RK4 steps started from the linearisation state x_{i-1}.

The Jacobian of the right-hand side is assembled as an explicit sparse matrix (four entries per
row), the tangent step follows the chain rule through the four RK4 stages, and the adjoint is the
transpose of that chain (sparse transposes, stages taken in reverse order).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def rhs(x, F):
    """f(x)_j = (x_{j+1} - x_{j-2}) x_{j-1} - x_j + F."""
    return (np.roll(x, -1) - np.roll(x, 2)) * np.roll(x, 1) - x + F


def rk4_step(x, F, dt):
    k1 = rhs(x, F)
    k2 = rhs(x + 0.5 * dt * k1, F)
    k3 = rhs(x + 0.5 * dt * k2, F)
    k4 = rhs(x + dt * k3, F)
    return x + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)


def jacobian(y):
    """Sparse Jacobian of f at y: d f_j / d y_{j+1} = y_{j-1}, / d y_{j-2} = -y_{j-1},
    / d y_{j-1} = y_{j+1} - y_{j-2}, / d y_j = -1 (indices periodic)."""
    s = y.size
    j = np.arange(s)
    rows = np.concatenate([j, j, j, j])
    cols = np.concatenate([(j + 1) % s, (j - 2) % s, (j - 1) % s, j])
    vals = np.concatenate([np.roll(y, 1), -np.roll(y, 1), np.roll(y, -1) - np.roll(y, 2),
                           -np.ones(s)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(s, s))


def stage_states(x, F, dt):
    """The four points at which RK4 evaluates f, and the stage slopes."""
    k1 = rhs(x, F)
    y2 = x + 0.5 * dt * k1
    k2 = rhs(y2, F)
    y3 = x + 0.5 * dt * k2
    k3 = rhs(y3, F)
    y4 = x + dt * k3
    return (x, y2, y3, y4)


class L96Tangent:
    def __init__(self, F, dt, nsteps, traj):
        self.F, self.dt, self.nsteps = float(F), float(dt), int(nsteps)
        self.traj = np.asarray(traj, dtype=np.float64)

    def _states(self, i):
        x = self.traj[i - 1].copy()
        out = []
        for _ in range(self.nsteps):
            out.append(x)
            x = rk4_step(x, self.F, self.dt)
        return out

    def jvp(self, i, d):
        """M_i d: the tangent of each RK4 step by the chain rule through its stages."""
        h = self.dt
        d = np.array(d, dtype=np.float64)
        for x in self._states(i):
            J = [jacobian(y) for y in stage_states(x, self.F, h)]
            d1 = J[0] @ d
            d2 = J[1] @ (d + 0.5 * h * d1)
            d3 = J[2] @ (d + 0.5 * h * d2)
            d4 = J[3] @ (d + h * d3)
            d = d + h / 6.0 * (d1 + 2 * d2 + 2 * d3 + d4)
        return d

    def vjp(self, i, lam):
        """M_i^T lam: the transposed chain, steps and stages in reverse order."""
        h = self.dt
        lam = np.array(lam, dtype=np.float64)
        for x in reversed(self._states(i)):
            JT = [jacobian(y).T.tocsr() for y in stage_states(x, self.F, h)]
            l_out = lam
            l1 = h / 6.0 * l_out
            l2 = h / 3.0 * l_out
            l3 = h / 3.0 * l_out
            l4 = h / 6.0 * l_out
            a4 = JT[3] @ l4            # d4 = J4 (d + h d3)
            l3 = l3 + h * a4
            a3 = JT[2] @ l3            # d3 = J3 (d + h/2 d2)
            l2 = l2 + 0.5 * h * a3
            a2 = JT[1] @ l2            # d2 = J2 (d + h/2 d1)
            l1 = l1 + 0.5 * h * a2
            a1 = JT[0] @ l1            # d1 = J1 d
            lam = l_out + a4 + a3 + a2 + a1
        return lam

    def forecast(self, x):
        """Nonlinear propagation over one observation interval (nsteps RK4 steps)."""
        for _ in range(self.nsteps):
            x = rk4_step(x, self.F, self.dt)
        return x


def forecast_fn(win, traj):
    """The nonlinear model of one observation interval, y = M_i(x_{i-1}) (§2.1): RK4 for a
    Lorenz-96 window, the linear map M for the other model kinds."""
    from oracle import svar_oracle as so
    m = win.model
    if m["kind"] == "l96":
        T = L96Tangent(m["F"], m["dt"], m["nsteps"], traj)
        return lambda i, x: T.forecast(x)
    ops = so.ModelOps(win)
    return lambda i, x: ops.M(i, x)


def gn_rhs(x, xb, y, idx, forecast):
    """Right-hand side (b; d; 0) of the saddle system linearised about x = (x_0..x_N) (§2.1,
    incremental form): b_0 = x_b - x_0, b_i = M_i(x_{i-1}) - x_i, d_i = y_i - H x_i (H picks
    the observed points idx)."""
    nb, s = x.shape
    b = np.zeros((nb, s))
    b[0] = xb - x[0]
    for i in range(1, nb):
        b[i] = forecast(i, x[i - 1]) - x[i]
    d = np.concatenate([y[i] - x[i][idx] for i in range(nb)])
    return np.concatenate([b.ravel(), d, np.zeros(nb * s)])


def cost(win, x, xb, y, idx, forecast):
    """The weak-constraint 4D-Var cost of eq. CostFn at the trajectory x (dense inverses:
    small windows only): 1/2 |x_0 - x_b|^2_{B^-1} + 1/2 sum_i |x_i - M_i(x_{i-1})|^2_{Q_i^-1}
    + 1/2 sum_i |y_i - H x_i|^2_{R_i^-1}."""
    nb = x.shape[0]

    def wnorm(C, v):
        return float(v @ np.linalg.solve(C, v))
    D = [float(win.d_scale[i]) * np.asarray(win.dmats[int(win.d_index[i])]) for i in range(nb)]
    R = [np.asarray(win.rmats[int(win.r_index[i])]) for i in range(nb)]
    J = wnorm(D[0], x[0] - xb)
    for i in range(1, nb):
        J += wnorm(D[i], x[i] - forecast(i, x[i - 1]))
    for i in range(nb):
        J += wnorm(R[i], y[i] - x[i][idx])
    return 0.5 * J


def gauss_newton(win, n_outer, *, k=3, rhat="RR", prec="PI", rtol=1e-12, x0=None,
                 rhs_fn=None):
    """Oracle outer loop (§2.1): linearise about x^(l), solve the saddle system for the
    increment with the oracle FGMRES, x^(l+1) = x^(l) + dx.  The window needs meta["xb"],
    meta["y"] and meta["obs_idx"]; x0 defaults to model["traj"] (Lorenz-96) and must be given
    for the linear kinds.  rhs_fn replaces gn_rhs (tests plant mistakes through it).
    Returns the list of iterates."""
    import copy

    from oracle import svar_oracle as so
    s, nb = win.s, win.N + 1
    m = win.model
    x = np.array(m["traj"] if x0 is None else x0, dtype=np.float64).reshape(nb, s)
    xb = np.asarray(win.meta["xb"])
    y = np.asarray(win.meta["y"])
    idx = np.asarray(win.meta["obs_idx"])
    rhs_fn = gn_rhs if rhs_fn is None else rhs_fn
    out = [x.copy()]
    for _ in range(n_outer):
        w = copy.copy(win)
        if m["kind"] == "l96":
            w.model = dict(m, traj=x.copy())
        orc = so.SaddleOracle(w, k=k, rhat=rhat)
        rhs = rhs_fn(x, xb, y, idx, forecast_fn(w, x))
        sol = so.solve(orc, rhs, prec=prec, rtol=rtol, maxit=orc.n)
        x = x + sol["x"][-nb * s:].reshape(nb, s)
        out.append(x.copy())
    return out
