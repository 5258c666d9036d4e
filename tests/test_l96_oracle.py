"""Pins of the Lorenz-96 tangent linear and adjoint oracle (no GPU)."""
import numpy as np
import pytest

from oracle import l96_oracle as lo
from oracle import svar_oracle as so
from paper_2105_06975_amd import workloads as wl


def small_l96(seed=0, s=40, N=4, nsteps=3):
    return wl.make_l96_window(s=s, N=N, nsteps=nsteps, spinup=200, seed=seed)


def test_tangent_matches_finite_differences():
    """P12: M_i d equals the central difference of the nonlinear RK4 map (O(eps^2) error)."""
    win = small_l96()
    m = win.model
    T = lo.L96Tangent(m["F"], m["dt"], m["nsteps"], m["traj"])
    rng = np.random.default_rng(1)
    d = rng.standard_normal(win.s)
    for i in (1, 3):
        x0 = m["traj"][i - 1]
        eps = 1e-5
        fd = (T.forecast(x0 + eps * d) - T.forecast(x0 - eps * d)) / (2 * eps)
        tl = T.jvp(i, d)
        assert np.linalg.norm(tl - fd) <= 1e-7 * np.linalg.norm(tl)


def test_adjoint_dot_test():
    """P12: <M u, v> = <u, M^T v> to rounding."""
    win = small_l96(seed=2)
    m = win.model
    T = lo.L96Tangent(m["F"], m["dt"], m["nsteps"], m["traj"])
    rng = np.random.default_rng(3)
    for i in (1, 2, 4):
        u, v = rng.standard_normal(win.s), rng.standard_normal(win.s)
        a, b = np.dot(T.jvp(i, u), v), np.dot(u, T.vjp(i, v))
        assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


def test_jacobian_is_the_derivative_of_the_tendency():
    rng = np.random.default_rng(4)
    y = rng.standard_normal(16)
    d = rng.standard_normal(16)
    eps = 1e-6
    fd = (lo.rhs(y + eps * d, 8.0) - lo.rhs(y - eps * d, 8.0)) / (2 * eps)
    assert np.allclose(lo.jacobian(y) @ d, fd, atol=1e-8)


def test_l96_window_saddle_solution_matches_dense():
    """The saddle system with L96 tangent blocks solves to the dense LU solution."""
    win = small_l96(seed=5, s=24, N=3, nsteps=2)
    orc = so.SaddleOracle(win, k=2, rhat="RR")
    rhs = win.rhs[0]
    x_ref = np.linalg.solve(orc.A_dense(), rhs)
    out = so.solve(orc, rhs, prec="PI", rtol=1e-13, maxit=orc.n)
    assert np.linalg.norm(out["x"] - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    # the model is not contractive here (Prop. 2 does not apply, as in §7.1)
    assert np.linalg.norm(orc.model.dense(1), 2) > 1.0


# ------------------------------------------------------------------ Gauss-Newton outer loop
def _linear_gn_window(seed=21, s=12, N=3, p=5):
    """A small linear advection-diffusion window with a background and observations."""
    win = wl.make_small_window(s=s, N=N, p=p, seed=seed)
    rng = np.random.default_rng(seed)
    idx = np.asarray(win.h_cols[0][:, 0])
    win.meta.update(xb=rng.standard_normal(s), y=rng.standard_normal((N + 1, p)), obs_idx=idx)
    return win


def _quadratic_minimiser(win):
    """Minimiser of eq. CostFn for a linear model, from its normal equations written out with
    dense matrices (independent of the saddle oracle): with (L x)_0 = x_0,
    (L x)_i = x_i - M x_{i-1} and btilde = (x_b, 0, .., 0),
        (L^T D^-1 L + H^T R^-1 H) x = L^T D^-1 btilde + H^T R^-1 y."""
    s, nb = win.s, win.N + 1
    m = win.model
    T = np.zeros((s, s))
    for j in range(s):
        T[j, (j - 1) % s] += m["a"]
        T[j, j] += m["b"]
        T[j, (j + 1) % s] += m["c"]
    M = np.linalg.inv(T)
    L = np.eye(nb * s)
    for i in range(1, nb):
        L[i * s:(i + 1) * s, (i - 1) * s:i * s] = -M
    import scipy.linalg as sla
    D = sla.block_diag(*[win.d_scale[i] * win.dmats[win.d_index[i]] for i in range(nb)])
    R = sla.block_diag(*[win.rmats[win.r_index[i]] for i in range(nb)])
    idx = win.meta["obs_idx"]
    H = np.zeros((nb * len(idx), nb * s))
    for i in range(nb):
        H[i * len(idx) + np.arange(len(idx)), i * s + idx] = 1.0
    bt = np.zeros(nb * s)
    bt[:s] = win.meta["xb"]
    Di, Ri = np.linalg.inv(D), np.linalg.inv(R)
    S = L.T @ Di @ L + H.T @ Ri @ H
    return np.linalg.solve(S, L.T @ Di @ bt + H.T @ Ri @ win.meta["y"].ravel()).reshape(nb, s)


def test_gauss_newton_linear_one_step_is_the_minimiser():
    """For a linear model the cost is quadratic: one Gauss-Newton step from any first guess
    reaches its minimiser, and the next increment vanishes."""
    win = _linear_gn_window()
    x0 = np.random.default_rng(5).standard_normal((win.N + 1, win.s))
    xs = lo.gauss_newton(win, 2, k=2, x0=x0)
    xstar = _quadratic_minimiser(win)
    assert np.linalg.norm(xs[1] - xstar) <= 1e-8 * np.linalg.norm(xstar)
    assert np.linalg.norm(xs[2] - xs[1]) <= 1e-8 * np.linalg.norm(xstar)


def _flip_b(x, xb, y, idx, fc):
    r = lo.gn_rhs(x, xb, y, idx, fc)
    nb, s = x.shape
    r[s:nb * s] *= -1.0
    return r


def _forecast_from_own_block(x, xb, y, idx, fc):
    nb, s = x.shape
    r = lo.gn_rhs(x, xb, y, idx, fc)
    for i in range(1, nb):
        r[i * s:(i + 1) * s] = fc(i, x[i]) - x[i]
    return r


def _flip_d(x, xb, y, idx, fc):
    r = lo.gn_rhs(x, xb, y, idx, fc)
    nb, s = x.shape
    r[nb * s:nb * s + nb * len(idx)] *= -1.0
    return r


@pytest.mark.parametrize("mistake", [_flip_b, _forecast_from_own_block, _flip_d])
def test_gauss_newton_pin_catches_planted_mistakes(mistake):
    """A sign flip in b_i, a forecast taken from x_i instead of x_{i-1}, or a flipped d_i in
    the oracle's right-hand side each move the first step off the minimiser."""
    win = _linear_gn_window()
    x0 = np.random.default_rng(5).standard_normal((win.N + 1, win.s))
    xs = lo.gauss_newton(win, 1, k=2, x0=x0, rhs_fn=mistake)
    xstar = _quadratic_minimiser(win)
    assert np.linalg.norm(xs[1] - xstar) > 1e-3 * np.linalg.norm(xstar)


def test_gauss_newton_l96_fixed_point_is_stationary():
    """On a small, short-interval Lorenz-96 window the Gauss-Newton iterates converge to a
    stationary point of eq. CostFn: its central-difference gradient vanishes (relative to the
    gradient at the first guess)."""
    win = wl.make_l96_window(s=12, N=3, dt=0.01, nsteps=2, spinup=300, seed=7, b_len=0.15,
                             q_scale=0.5)
    xb, y, idx = win.meta["xb"], win.meta["y"], win.meta["obs_idx"]
    xs = lo.gauss_newton(win, 14, k=2)
    # Gauss-Newton converges linearly here (the observation residual does not vanish)
    assert np.linalg.norm(xs[-1] - xs[-2]) <= 1e-12 * np.linalg.norm(xs[-1])

    def J(x):
        return lo.cost(win, x, xb, y, idx, lo.forecast_fn(win, x))

    def grad(x, h=1e-5):
        g = np.zeros(x.size)
        for j in range(x.size):
            e = np.zeros(x.size)
            e[j] = h
            g[j] = (J(x + e.reshape(x.shape)) - J(x - e.reshape(x.shape))) / (2 * h)
        return g
    g0, gs = grad(xs[0]), grad(xs[-1])
    assert np.linalg.norm(gs) <= 1e-7 * np.linalg.norm(g0)
    assert J(xs[-1]) < J(xs[0])
