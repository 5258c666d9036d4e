"""Parity of the wide-panel paths: the LDS-tiled covariance GEMM (panels of more than 128
columns, i.e. several right-hand sides) and the learned correction at the benchmark's size.

* A v and P^{-1} v for 12 right-hand sides of small uneven windows (tile rows past n, ragged
  column groups) against the oracle, element by element, with float64 matrices and with
  float32 / bfloat16 copies; five windows per launch (the many-problem plan, with and without
  rows that are not 4-element aligned);
* A v at the full C2 size for 3 right-hand sides (195-column panels) against the oracle;
* the learned correction inside P_I at the full C2 size, sampled: three time blocks of one
  right-hand side against the oracle's network on the same blocks.
"""
import numpy as np
import pytest

from oracle import learned_oracle as lo
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("ptype", ["PI", "PD"])
def test_many_rhs_small_windows(sv, ptype):
    wins = [wl.make_small_window(s=100, N=10, p=40, seed=1),
            wl.make_small_window(s=150, N=12, p=70, seed=2)]
    nrhs = 12  # 132 and 156 columns per D product: tiled kernel, ragged tiles
    h = sv.Handle(wins, sv.Precond(type=ptype, k=3, rhat="RR"))
    V = np.concatenate([wl.random_vectors(w, nrhs, seed=5 + i).ravel() for i, w in enumerate(wins)])
    ya = host(h.apply_A(dev(V), nrhs))
    yp = host(h.apply_P(dev(V), nrhs))
    off = h.offsets(nrhs)
    for w, win in enumerate(wins):
        orc = so.SaddleOracle(win, k=3, rhat="RR")
        for r in range(nrhs):
            a = off[w] + r * win.n
            v = V[a:a + win.n]
            assert rel(ya[a:a + win.n], orc.apply_A(v)) < 1e-12, (w, r)
            ref = orc.apply_PI_inv(v) if ptype == "PI" else orc.apply_PD_inv(v)
            assert rel(yp[a:a + win.n], ref) < 1e-10, (w, r)


def test_many_windows_tiled_plans(sv):
    """Five uneven windows x 12 rhs: every covariance launch holds five problems (the
    share-based split plan), with 4-aligned and unaligned rows mixed (the LDS-staged kernel)
    and, for the last three windows alone, aligned rows only (the register path)."""
    shapes = [(122, 10, 45), (98, 11, 37), (152, 12, 64), (200, 10, 80), (136, 11, 52)]
    wins = [wl.make_small_window(s=s, N=N, p=p, seed=40 + i) for i, (s, N, p) in
            enumerate(shapes)]
    nrhs = 12
    for sub in (wins, wins[2:]):
        h = sv.Handle(sub, sv.Precond(type="PI", k=3, rhat="RR"))
        V = np.concatenate([wl.random_vectors(w, nrhs, seed=60 + i).ravel()
                            for i, w in enumerate(sub)])
        ya = host(h.apply_A(dev(V), nrhs))
        yp = host(h.apply_P(dev(V), nrhs))
        off = h.offsets(nrhs)
        for w, win in enumerate(sub):
            orc = so.SaddleOracle(win, k=3, rhat="RR")
            for r in (0, 5, nrhs - 1):
                a = off[w] + r * win.n
                v = V[a:a + win.n]
                assert rel(ya[a:a + win.n], orc.apply_A(v)) < 1e-12, (len(sub), w, r)
                assert rel(yp[a:a + win.n], orc.apply_PI_inv(v)) < 1e-10, (len(sub), w, r)


def test_many_rhs_low_precision_products(sv):
    """float32 and bfloat16 matrix copies in the tiled kernel (ragged tiles, rows of 150 and
    70 entries that take element loads, 100 and 40 that take 4-element loads): errors at the
    level of the storage precision against the float64 oracle, and above float64 rounding."""
    wins = [wl.make_small_window(s=100, N=10, p=40, seed=1),
            wl.make_small_window(s=150, N=12, p=70, seed=2)]
    nrhs = 12
    h = sv.Handle(wins, sv.Precond(type="PI", k=3, rhat="RR"))
    V = np.concatenate([wl.random_vectors(w, nrhs, seed=5 + i).ravel() for i, w in enumerate(wins)])
    ya = host(h.apply_A(dev(V), nrhs, precision="MIXED_FP32"))
    zf = host(h.apply_P(dev(V), nrhs, precision="FP64_F32P"))
    zb = host(h.apply_P(dev(V), nrhs, precision="MIXED_BF16P"))
    off = h.offsets(nrhs)
    worst = [0.0, 0.0, 0.0]
    for w, win in enumerate(wins):
        orc = so.SaddleOracle(win, k=3, rhat="RR")
        for r in range(nrhs):
            a = off[w] + r * win.n
            v = V[a:a + win.n]
            e = (rel(ya[a:a + win.n], orc.apply_A(v)), rel(zf[a:a + win.n], orc.apply_PI_inv(v)),
                 rel(zb[a:a + win.n], orc.apply_PI_inv(v)))
            worst = [max(x, y) for x, y in zip(worst, e)]
            assert 1e-12 < e[0] < 1e-5 and 1e-12 < e[1] < 1e-4 and 1e-9 < e[2] < 5e-2, (w, r, e)
    print("worst relative errors (A float32, P float32, P bfloat16):", worst)


def test_c2_three_rhs_apply_A(sv):
    win = wl.make_config_window("c2", seed=0)
    nrhs = 3
    h = sv.Handle([win], sv.Precond(type="PI", k=3, rhat="RR"))
    V = wl.random_vectors(win, nrhs, seed=7)
    y = host(h.apply_A(dev(V), nrhs)).reshape(nrhs, win.n)
    orc = so.SaddleOracle(win, k=3, rhat="RR")
    for r in range(nrhs):
        assert rel(y[r], orc.apply_A(V[r])) < 1e-12, r


@pytest.mark.parametrize("netprec,tol", [("FP32", 1e-5), ("BF16", 3e-2)])
def test_c2_learned_correction_sampled(sv, netprec, tol):
    win = wl.make_config_window("c2", seed=0)
    K, S, C = 3, 12, 64
    h = sv.Handle([win], sv.Precond(type="PI", k=K, rhat="RR"))
    net = sv.Net(K, S, netprec)
    rng = np.random.default_rng(9)
    th = wl.net_init(net.cin, C, seed=3)
    th = (th + 0.02 * rng.standard_normal(th.size)).astype(np.float32).astype(np.float64)
    net.set_params(th)
    v = wl.random_vectors(win, 1, seed=11)[0]
    zp = host(h.apply_P(dev(v)))
    h.set_net(net)
    zl = host(h.apply_P(dev(v)))
    nb, s = win.nb, win.s
    corr_gpu = (zl - zp)[:nb * s].reshape(nb, s)  # the eta component is c1 in P_I
    orc = so.SaddleOracle(win, k=K, rhat="RR")
    v1, v2, v3 = orc.split(v)
    chat = orc.LM_invT(v3)
    sigma = float(np.sqrt(np.mean(chat * chat)))
    X = lo.features(chat / sigma, K, S)
    blocks = [0, 31, 64]  # first, interior segment start region, last block
    ref = sigma * lo.forward(th, X[blocks], C)
    for i, b in enumerate(blocks):
        e = rel(corr_gpu[b], ref[i])
        print(f"{netprec} block {b}: correction rel err {e:.2e}")
        assert e <= tol, b
