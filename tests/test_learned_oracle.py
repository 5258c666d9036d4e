"""Pins of the learned-correction oracle against things other than itself.

* the periodic convolution against scipy's correlate1d (wrap mode) and a unit impulse;
* analytic gradients against central differences (weights, biases and inputs);
* Adam against its closed form for a constant gradient;
* the feature map against a worked example written out by hand;
* the exact correction c* - chat against explicit products of the transposed model maps
  and dense solves with L and L_M(k) (the reason for the network's inputs);
* the corrected preconditioners: a zero network gives the plain P exactly, an ideal
  correction gives P with the exact L^{-T} (dense solves);
* the fallback of the flexible GMRES: a useless learned preconditioner triggers it and the
  solve still reaches the dense solution;
* the bfloat16 storage model: the rounding on hand-checked bit patterns (ties to even, the
  float32 step first) and the network on values every step represents exactly.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import learned_oracle as lo
from oracle import svar_oracle as so
from paper_2105_06975_amd import workloads as wl


def test_conv_matches_scipy_correlate_wrap():
    rng = np.random.default_rng(1)
    n, cin, cout, s = 2, 3, 4, 11
    x = rng.standard_normal((n, cin, s))
    W = rng.standard_normal((cout, cin, 5))
    b = rng.standard_normal(cout)
    y = lo.conv_periodic(x, W, b)
    ref = np.zeros_like(y)
    for q in range(n):
        for o in range(cout):
            ref[q, o] = b[o] + sum(ndi.correlate1d(x[q, c], W[o, c], mode="wrap")
                                   for c in range(cin))
    assert np.max(np.abs(y - ref)) < 1e-13


def test_conv_unit_impulse():
    # x = e_q gives y[(q - t + 2) mod s] = W[t]: the taps read back reversed around q
    s, q = 9, 1
    W = np.arange(1.0, 6.0).reshape(1, 1, 5)
    x = np.zeros((1, 1, s))
    x[0, 0, q] = 1.0
    y = lo.conv_periodic(x, W, np.zeros(1))[0, 0]
    expect = np.zeros(s)
    for t in range(5):
        expect[(q - t + 2) % s] = W[0, 0, t]
    assert np.array_equal(y, expect)


def _fd_grad(f, theta, h=1e-6):
    g = np.zeros_like(theta)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        g[i] = (f(tp) - f(tm)) / (2 * h)
    return g


def test_gradients_central_differences():
    rng = np.random.default_rng(2)
    n, cin, C, s = 2, 4, 3, 9
    theta = rng.standard_normal(lo.nparams(cin, C)) * 0.7
    X = rng.standard_normal((n, cin, s))
    Y = rng.standard_normal((n, s))
    loss, g = lo.loss_and_grad(theta, X, Y, C)
    g_fd = _fd_grad(lambda t: lo.loss_and_grad(t, X, Y, C)[0], theta)
    assert np.linalg.norm(g - g_fd) / np.linalg.norm(g) <= 1e-7
    # the loss is the mean squared error of the forward pass
    assert abs(loss - np.mean((lo.forward(theta, X, C) - Y) ** 2)) < 1e-14


def test_input_gradient_central_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 8))
    W = rng.standard_normal((4, 3, 5))
    b = rng.standard_normal(4)
    gy = rng.standard_normal((2, 4, 8))
    gx, gW, gb = lo.conv_periodic_backward(x, W, gy)
    f = lambda xx: float(np.sum(gy * lo.conv_periodic(xx.reshape(x.shape), W, b)))
    gx_fd = _fd_grad(f, x.ravel()).reshape(x.shape)
    assert np.linalg.norm(gx - gx_fd) / np.linalg.norm(gx) <= 1e-7
    fb = lambda bb: float(np.sum(gy * lo.conv_periodic(x, W, bb)))
    assert np.linalg.norm(gb - _fd_grad(fb, b)) / np.linalg.norm(gb) <= 1e-7


def test_adam_constant_gradient_closed_form():
    # with bias correction, a constant gradient g gives mhat = g and vhat = g^2 exactly, so
    # every step moves each parameter by lr * g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 5.0])
    lr, eps = 0.01, 1e-8
    theta = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 6):
        new, m, v = lo.adam_step(theta, g, m, v, t, lr, eps=eps)
        assert np.allclose(theta - new, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
        theta = new


def test_features_worked_example():
    # N = 7, k = 3: segments [0,2], [3,5], [6,7]; S = 2; chat_j = j + 1 everywhere in space
    nb, k, S, s = 8, 3, 2, 2
    chat = np.repeat(np.arange(1.0, nb + 1)[:, None], s, axis=1)
    X = lo.features(chat, k, S)
    # columns: own, start 1, start 2, one-hot of e(i) - i = 0, 1, 2
    expect = np.array([
        [1, 4, 7, 0, 0, 1],
        [2, 4, 7, 0, 1, 0],
        [3, 4, 7, 1, 0, 0],
        [4, 7, 0, 0, 0, 1],
        [5, 7, 0, 0, 1, 0],
        [6, 7, 0, 1, 0, 0],
        [7, 0, 0, 0, 1, 0],
        [8, 0, 0, 1, 0, 0],
    ], dtype=float)
    assert X.shape == (nb, 6, s)
    assert np.array_equal(X[:, :, 0], expect) and np.array_equal(X[:, :, 1], expect)


@pytest.mark.parametrize("k", [2, 3])
def test_exact_correction_is_sum_over_later_segment_starts(k):
    win = wl.with_dense_model(wl.make_small_window(s=6, N=8, p=3, seed=4), seed=5)
    orc = so.SaddleOracle(win, k=k, rhat="RR")
    s, nb, N = win.s, win.nb, win.N
    r = np.random.default_rng(6).standard_normal((nb, s))
    chat = np.linalg.solve(orc.L_dense(k).T, r.ravel()).reshape(nb, s)
    cstar = np.linalg.solve(orc.L_dense().T, r.ravel()).reshape(nb, s)
    mats = win.model["mats"]  # mats[i-1] = M_i

    def P(i, j):  # M_{i+1}^T ... M_j^T
        out = np.eye(s)
        for q in range(i + 1, j + 1):
            out = out @ mats[q - 1].T
        return out

    for i in range(nb):
        e = lo.segment_end(i, k, N)
        corr = np.zeros(s)
        b = e + 1
        while b <= N:
            corr += P(i, b) @ chat[b]
            b += k
        assert np.allclose(cstar[i] - chat[i], corr, rtol=0, atol=1e-12)
    # and the oracle's sweeps agree with the dense solves
    assert np.allclose(orc.LM_invT(r), chat, atol=1e-12)
    assert np.allclose(orc.LM_invT(r, N + 1), cstar, atol=1e-12)


def _small():
    win = wl.make_small_window(s=12, N=6, p=5, seed=7)
    return win, so.SaddleOracle(win, k=3, rhat="RR")


def test_zero_network_gives_plain_preconditioners():
    win, orc = _small()
    C, S = 4, 2
    theta = np.zeros(lo.nparams(lo.n_inputs(3, S), C))
    v = wl.random_vectors(win, 1, seed=8)[0]
    assert np.array_equal(lo.apply_PI_inv_learned(orc, theta, v, C, S), orc.apply_PI_inv(v))
    assert np.array_equal(lo.apply_PD_inv_learned(orc, theta, v, C, S), orc.apply_PD_inv(v))


def test_ideal_correction_gives_exact_backward_factor():
    win, orc = _small()
    s, nb = win.s, win.nb
    v = wl.random_vectors(win, 1, seed=9)[0]
    v1, v2, v3 = orc.split(v)
    Lk, L = orc.L_dense(3), orc.L_dense()
    cstar = np.linalg.solve(L.T, v3.ravel())
    sigma = np.sqrt(np.mean(np.linalg.solve(Lk.T, v3.ravel()) ** 2))

    def ideal(chat_n):  # the exact normalised correction
        return cstar.reshape(nb, s) / sigma - chat_n

    D = np.stack([orc.D_block(i) for i in range(nb)])
    Dc = np.einsum("bij,bj->bi", D, cstar.reshape(nb, s)).ravel()
    z3 = np.linalg.solve(Lk, v1.ravel() - Dc)
    ref = orc.join(cstar, orc.Rhat_inv(v2), z3)
    out = lo.apply_PI_inv_learned(orc, None, v, 0, 0, net_fn=ideal)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-12
    ref_d = orc.join(orc.Dhat_inv(v1), orc.Rhat_inv(v2), np.linalg.solve(Lk, Dc))
    out_d = lo.apply_PD_inv_learned(orc, None, v, 0, 0, net_fn=ideal)
    assert np.linalg.norm(out_d - ref_d) / np.linalg.norm(ref_d) < 1e-12


def test_make_pair_normalisation():
    chat = np.array([[3.0, -4.0]])
    x, y = lo.make_pair(chat, chat + 1.0)
    sigma = np.sqrt((9 + 16) / 2)
    assert np.allclose(x, chat / sigma) and np.allclose(y, 1.0 / sigma)
    x0, y0 = lo.make_pair(np.zeros((1, 2)), np.ones((1, 2)))
    assert not x0.any() and not y0.any()


def test_fallback_rescues_a_useless_learned_preconditioner():
    win, orc = _small()
    rhs = wl.random_vectors(win, 1, seed=10)[0]
    rhs[-win.nb * win.s:] = 0.0
    x_ref = np.linalg.solve(orc.A_dense(), rhs)
    rng = np.random.default_rng(11)
    garbage = lambda v: rng.standard_normal(v.size) * 1e-12  # nearly no progress
    x, it, hist, fb = lo.fgmres_with_fallback(orc.apply_A, garbage, orc.apply_PI_inv, rhs, 1e-10,
                                              400)
    assert fb == 1
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-8
    # with the plain preconditioner in both roles it matches plain FGMRES step for step
    x2, it2, hist2, fb2 = lo.fgmres_with_fallback(orc.apply_A, orc.apply_PI_inv, orc.apply_PI_inv,
                                                  rhs, 1e-10, 400)
    x3, it3, hist3 = so.fgmres(orc.apply_A, orc.apply_PI_inv, rhs, 1e-10, 400)
    assert it2 == it3 and np.allclose(hist2, hist3, rtol=1e-10, atol=0)


def test_fallback_patience_ignores_isolated_plateaus():
    # a preconditioner that is useless on every third call only: each useless step is an
    # isolated plateau, so patience 3 never falls back while patience 1 does at once
    win, orc = _small()
    rhs = wl.random_vectors(win, 1, seed=16)[0]
    rhs[-win.nb * win.s:] = 0.0
    calls = {"n": 0}

    def flaky(v):
        calls["n"] += 1
        return orc.apply_PI_inv(v) if calls["n"] % 3 else np.zeros_like(v) + 1e-14 * v

    _, _, _, fb3 = lo.fgmres_with_fallback(orc.apply_A, flaky, orc.apply_PI_inv, rhs, 1e-8, 400,
                                           patience=3)
    calls["n"] = 0
    _, _, _, fb1 = lo.fgmres_with_fallback(orc.apply_A, flaky, orc.apply_PI_inv, rhs, 1e-8, 400,
                                           patience=1)
    assert fb3 == 0 and fb1 == 1


def test_round_bf16_hand_checked():
    # near 1 the bfloat16 spacing is 2^-7: halfway cases go to the even significand
    cases = [
        (1.0, 1.0),
        (1 + 2**-8, 1.0),                          # tie, 1.0 is even
        (1 + 3 * 2**-8, 1 + 2**-6),                # tie between odd 1+2^-7 and even 1+2^-6
        (1 + 2**-8 + 2**-20, 1 + 2**-7),           # above the tie
        (1 + 2**-8 + 2**-30, 1.0),                 # float32 first drops 2^-30: a tie again
        (-(1 + 3 * 2**-8), -(1 + 2**-6)),
        (3.0, 3.0),
        (255.0, 255.0),                            # 8 significant bits: exact
        (257.0, 256.0),                            # tie between 256 (even) and 258
        (0.0, 0.0),
    ]
    x = np.array([c[0] for c in cases])
    y = lo.round_bf16(x)
    assert np.array_equal(y, np.array([c[1] for c in cases])), y


def test_forward_bf16_exact_on_representable_values():
    # one hidden channel passing channel 0 through (centre tap 1), integer inputs: every
    # value is a small integer, so the bfloat16 model and the exact network agree bit for bit
    rng = np.random.default_rng(17)
    cin, C, s = 3, 1, 10
    parts = [np.zeros(sh) for sh in lo.param_shapes(cin, C)]
    parts[0][0, 0, 2] = 1.0                        # W1: relu(x0)
    parts[2][0, 0, 2] = 1.0                        # W2, W3: identity
    parts[4][0, 0, 2] = 1.0
    parts[6][0, 0, :] = [1.0, -2.0, 0.5, 0.25, 3.0]  # W4 (float32 values, kept as given)
    parts[7][0] = 0.125
    theta = lo.pack(parts)
    X = rng.integers(-8, 9, size=(2, cin, s)).astype(np.float64)
    assert np.array_equal(lo.forward_bf16(theta, X, C), lo.forward(theta, X, C))
    # and on general values it stays within the bfloat16 error of the exact network
    theta_r = rng.standard_normal(lo.nparams(cin, 4)) * 0.5
    Xr = rng.standard_normal((2, cin, s))
    out, ref = lo.forward_bf16(theta_r, Xr, 4), lo.forward(theta_r, Xr, 4)
    assert 0 < np.linalg.norm(out - ref) / np.linalg.norm(ref) < 3e-2
