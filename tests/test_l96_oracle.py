"""Pins of the Lorenz-96 tangent linear and adjoint oracle (no GPU)."""
import numpy as np

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
