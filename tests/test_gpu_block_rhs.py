"""Block FGMRES over the right-hand sides of each window (svar_solve_opts.block_rhs) through
the C ABI.

The oracle's block FGMRES (block Arnoldi with block modified Gram-Schmidt and thin QR, per
column least squares) fixes the per-column residual estimates of the first cycle; the GPU's
two block classical Gram-Schmidt passes and Cholesky QR rounds give the same Krylov spaces, so
the estimates agree while they are well above rounding.  Solutions are checked against the
oracle's dense solve, restarted batches of uneven windows against the rtol they were asked
for, and degenerate blocks (a zero column, two equal columns) against their exact answers.
"""
import numpy as np
import pytest

from oracle import svar_oracle as so
from paper_2105_06975_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_06975_amd import svar
    return svar


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def dense_x(orc, rhs):
    return np.linalg.solve(orc.A_dense(), rhs)


@pytest.mark.parametrize("prec,nrhs,rtol", [("PI", 4, 1e-10), ("PD", 3, 1e-8), ("PI", 8, 1e-10)])
def test_first_cycle_matches_oracle_block_fgmres(sv, prec, nrhs, rtol):
    win = wl.make_small_window(s=40, N=6, p=15, seed=90 + nrhs, nrhs=nrhs)
    orc = so.SaddleOracle(win, k=2, rhat="RR")
    RHS = win.rhs.reshape(nrhs, -1).T
    nb = np.linalg.norm(RHS, axis=0)
    pinv = orc.apply_PI_inv if prec == "PI" else orc.apply_PD_inv
    L = 250
    Xo, steps_o, hist_o = so.block_fgmres(orc.apply_A, pinv, RHS, rtol, L)
    h = sv.Handle([win], sv.Precond(type=prec, k=2, rhat="RR"))
    hist = torch.zeros((nrhs, L), dtype=torch.float64, device="cuda")
    x, info, rc = h.solve(dev(win.rhs), nrhs, rtol=rtol, maxit=L, restart=0,
                          block_rhs=True, history=hist)
    assert rc == sv.OK, info
    steps = info[0]["iters"]
    print(f"{prec} nrhs {nrhs}: block steps GPU {steps}, oracle {steps_o}", flush=True)
    assert all(i["iters"] == steps for i in info)
    assert abs(steps - steps_o) <= 2
    hh = host(hist) / nb[:, None]
    ho = np.array(hist_o[1:]).T           # (nrhs, steps_o)
    k = min(steps, steps_o, 40)
    sel = ho[:, :k] > 1e-7
    rel = np.abs(hh[:, :k] - ho[:, :k])[sel] / ho[:, :k][sel]
    print(f"  history: worst relative difference {rel.max():.2e} over {sel.sum()} entries")
    assert rel.max() <= 1e-6
    assert np.all(np.isnan(hh[:, steps:]))
    X = host(x).reshape(nrhs, -1).T
    Xd = dense_x(orc, RHS)
    err = np.linalg.norm(X - Xd, axis=0) / np.linalg.norm(Xd, axis=0)
    erro = np.linalg.norm(Xo - Xd, axis=0) / np.linalg.norm(Xd, axis=0)
    print(f"  solution error GPU {err.max():.2e}, oracle {erro.max():.2e}")
    assert err.max() <= max(10 * erro.max(), 1e-8)
    for i in info:
        assert i["relres_true"] <= rtol


SHAPES = [(24, 3, 9), (40, 6, 15), (17, 2, 6), (64, 5, 30), (33, 7, 11)]


@pytest.mark.parametrize("restart,mode", [(15, 1), (25, 1), (25, 2)])
def test_restarted_uneven_batch(sv, restart, mode):
    """Uneven windows in one call with restarts (mode 2: one Gram-Schmidt pass per step):
    every system meets rtol in the float64 true residual; a window stops as a whole when all
    its columns are below their tolerances."""
    nrhs = 5
    wins = [wl.make_small_window(s=s, N=N, p=p, seed=120 + i, nrhs=nrhs)
            for i, (s, N, p) in enumerate(SHAPES)]
    rhs = np.concatenate([w.rhs.reshape(-1) for w in wins])
    h = sv.Handle(wins, sv.Precond(type="PI", k=2, rhat="RR"))
    off = h.offsets(nrhs)
    x, info, rc = h.solve(dev(rhs), nrhs, rtol=1e-9, maxit=3000, restart=restart,
                          max_outer=3000, block_rhs=mode)
    assert rc == sv.OK, [i for i in info if i["status"]][:3]
    xs = host(x)
    for w, win in enumerate(wins):
        orc = so.SaddleOracle(win, k=2, rhat="RR")
        its = {info[w * nrhs + r]["iters"] for r in range(nrhs)}
        assert len(its) == 1, its   # one block: every column takes the window's steps
        for r in range(nrhs):
            b = win.rhs[r]
            xv = xs[off[w] + r * win.n: off[w] + (r + 1) * win.n]
            res = np.linalg.norm(b - orc.apply_A(xv)) / np.linalg.norm(b)
            assert res <= 1e-9 * 1.01, (w, r, res)
    # the one-at-a-time FGMRES with the same restart (FGMRES(15) stagnates on some of these
    # windows: then its solutions are not compared)
    x1, info1, rc1 = h.solve(dev(rhs), nrhs, rtol=1e-9, maxit=3000, restart=restart,
                             max_outer=3000)
    d = np.linalg.norm(host(x1) - xs) / np.linalg.norm(xs)
    print(f"restart {restart}, mode {mode}: block steps per window "
          f"{[info[w * nrhs]['iters'] for w in range(len(wins))]}, one at a time "
          f"{[max(info1[w * nrhs + r]['iters'] for r in range(nrhs)) for w in range(len(wins))]}"
          f", solution difference {d:.2e} (one at a time: status {rc1})", flush=True)
    if rc1 == sv.OK:
        assert d <= 1e-7


def test_degenerate_columns(sv):
    """A zero right-hand side (solution zero, no iterations needed) and two equal columns
    (deflated in the first QR) beside ordinary ones."""
    nrhs = 4
    win = wl.make_small_window(s=32, N=4, p=12, seed=140, nrhs=nrhs)
    R = win.rhs.reshape(nrhs, -1).copy()
    R[1] = 0.0
    R[3] = R[2]
    orc = so.SaddleOracle(win, k=2, rhat="RR")
    h = sv.Handle([win], sv.Precond(type="PI", k=2, rhat="RR"))
    x, info, rc = h.solve(dev(R), nrhs, rtol=1e-10, maxit=400, restart=0, block_rhs=True)
    assert rc == sv.OK, info
    X = host(x).reshape(nrhs, -1)
    assert np.all(X[1] == 0.0)
    assert info[1]["relres_true"] == 0.0
    Xd = dense_x(orc, R.T).T
    for r in (0, 2, 3):
        assert np.linalg.norm(X[r] - Xd[r]) <= 1e-8 * np.linalg.norm(Xd[r])
    assert np.linalg.norm(X[2] - X[3]) <= 1e-8 * np.linalg.norm(X[2])


def test_waves_match_one_call(sv):
    nrhs = 3
    wins = [wl.make_small_window(s=s, N=N, p=p, seed=150 + i, nrhs=nrhs)
            for i, (s, N, p) in enumerate(SHAPES)]
    rhs = np.concatenate([w.rhs.reshape(-1) for w in wins])
    h = sv.Handle(wins, sv.Precond(type="PI", k=2, rhat="RR"))
    kw = dict(rtol=1e-10, maxit=2000, restart=30, max_outer=2000, block_rhs=True)
    x1, inf1, rc1 = h.solve(dev(rhs), nrhs, **kw)
    lens = [nrhs * w.n for w in wins]
    x2, inf2, rc2 = h.solve(dev(rhs), nrhs, wave_len=max(lens[0] + lens[1], lens[2] + lens[3],
                                                          lens[4]), **kw)
    assert rc1 == sv.OK and rc2 == sv.OK
    assert [i["iters"] for i in inf1] == [i["iters"] for i in inf2]
    d = np.linalg.norm(host(x1) - host(x2)) / np.linalg.norm(host(x1))
    assert d <= 1e-9


def test_block_rhs_rejections(sv):
    win = wl.make_small_window(s=16, N=3, p=6, seed=160, nrhs=9)
    h = sv.Handle([win], sv.Precond(type="PI", k=2, rhat="RR"))
    b = dev(win.rhs)
    with pytest.raises(sv.SvarError):
        h.solve(b, 9, block_rhs=True)                       # more than 8 columns
    with pytest.raises(sv.SvarError):
        h.solve(b[: 2 * win.n], 2, block_rhs=True, block=4)  # with s-step blocks
    with pytest.raises(sv.SvarError):
        h.solve(b[: 2 * win.n], 2, block_rhs=True, method="MINRES")


def test_block_rhs_learned_fallback(sv):
    """The learned correction inside the block: a zero network gives the plain block solve's
    iterations; a garbage network is switched off per window by the decrease test and the
    solve still reaches the dense solution."""
    K, S = 3, 2
    nrhs = 3
    win = wl.make_small_window(s=100, N=10, p=40, seed=170, nrhs=nrhs)
    orc = so.SaddleOracle(win, k=K, rhat="RR")
    RHS = win.rhs.reshape(nrhs, -1)
    Xd = dense_x(orc, RHS.T).T
    h = sv.Handle([win], sv.Precond(type="PI", k=K, rhat="RR"))
    kw = dict(rtol=1e-8, maxit=600, restart=30, max_outer=600, block_rhs=True)
    xp, ip, rcp = h.solve(dev(RHS), nrhs, **kw)
    assert rcp == sv.OK
    net = sv.Net(K, S, "BF16")
    h.set_net(net)                      # zero parameters: the plain preconditioner
    xz, iz, rcz = h.solve(dev(RHS), nrhs, **kw)
    assert rcz == sv.OK
    assert [i["iters"] for i in iz] == [i["iters"] for i in ip]
    rng = np.random.default_rng(171)
    th = wl.net_init(1 + S + K, 64, seed=171)
    net.set_params(np.asarray(30.0 * th + 0.02 * rng.standard_normal(th.size),
                              dtype=np.float32).astype(np.float64))
    xg, ig, rcg = h.solve(dev(RHS), nrhs, **kw)
    print("garbage net in the block:", [(i["iters"], i["fallbacks"]) for i in ig],
          "plain:", ip[0]["iters"], flush=True)
    assert rcg == sv.OK
    assert all(i["fallbacks"] == 1 for i in ig)
    X = host(xg).reshape(nrhs, -1)
    for r in range(nrhs):
        assert np.linalg.norm(X[r] - Xd[r]) <= 1e-6 * np.linalg.norm(Xd[r])
    h.set_net(None)
