"""Parity of the benchmark's paths at their real shapes (through the C ABI).

* C2 (s = 4096, N = 64, p = 2048) with 8 right-hand sides: A v and P_I^{-1} v on the
  autotuned wide-panel GEMM plans (520 columns per covariance product) against the oracle,
  element by element per block.
* The batched learned path of the headline batch (windows of the uneven batch, 8 rhs,
  bfloat16 network inference, FGMRES(20), two waves): the benchmark's path (one block Krylov
  space per window over its 8 rhs with one Gram-Schmidt pass per step, every covariance product
  float32 inside the float64 restart loop) and the one-column path (FP64 A, float32
  Rhat^{-1}) against reference solutions: float64 FGMRES solves at rtol 1e-12 whose residual
  the oracle's A confirms.  The solution error of every system is reported and bounded.
"""
import numpy as np
import pytest

from blockcheck import assert_blocks, block_errors
from oracle import svar_oracle as so
from paper_2105_06975_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# the benchmark's stopping tolerance (true relative residual) and restart length: at a 1e-6
# residual the solution error of these windows reaches 1.2e-6, so the benchmark stops at
# 5e-7, where every solution is within 1e-6 of the reference
HEADLINE_RTOL = 5e-7
HEADLINE_RESTART = 20


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


def test_c2_eight_rhs_wide_plans(sv):
    win = wl.make_config_window("c2", seed=0)
    nrhs = 8
    h = sv.Handle([win], sv.Precond(type="PI", k=3, rhat="RR"))
    h.autotune(nrhs, "FP64")
    orc = so.SaddleOracle(win, k=3, rhat="RR")
    V = wl.random_vectors(win, nrhs, seed=41)
    print("c2 x 8: A and P_I on the tuned plans", flush=True)
    Y = host(h.apply_A(dev(V), nrhs)).reshape(nrhs, -1)
    Z = host(h.apply_P(dev(V), nrhs)).reshape(nrhs, -1)
    for r in range(nrhs):
        ra, rp = orc.apply_A(V[r]), orc.apply_P_inv(V[r], "PI")
        assert rel(Y[r], ra) < 1e-12 and rel(Z[r], rp) < 1e-10, r
        assert_blocks(win, Y[r], ra, 1e-11, what=f"A rhs {r}")
        assert_blocks(win, Z[r], rp, 1e-9, what=f"P_I rhs {r}")
    h.close()


@pytest.mark.parametrize("block_rhs,precision", [(0, "FP64_F32P"), (2, "MIXED_F32")])
def test_headline_batched_learned_path_solution_error(sv, block_rhs, precision):
    nrhs = 8
    wins = [wl.make_c4_window(w, nrhs=nrhs) for w in (5, 11, 2, 29)]
    print("windows (s, N, p):", [(w.s, w.N, int(w.p[0])) for w in wins], flush=True)
    prec = sv.Precond(type="PI", k=3, rhat="RR")
    h = sv.Handle(wins, prec)
    off = h.offsets(nrhs)
    rhs = np.concatenate([w.rhs.reshape(-1) for w in wins])
    # reference: float64, no network, rtol 1e-12
    xr, infr, rcr = h.solve(dev(rhs), nrhs, rtol=1e-12, maxit=20000, restart=HEADLINE_RESTART,
                            max_outer=20000)
    assert rcr == sv.OK
    XR = host(xr)
    # the network of the benchmark (bfloat16 inference, n_bound = 8); its weights here are
    # the seeded initial ones: the test is about the path's arithmetic, not the gain
    net = sv.Net(3, 8, "BF16")
    net.set_params(wl.net_init(net.cin, 64, seed=0))
    h.set_net(net)
    lens = [nrhs * w.n for w in wins]
    wave_len = max(lens[0] + lens[1], lens[2] + lens[3])
    x, inf, rc = h.solve(dev(rhs), nrhs, rtol=HEADLINE_RTOL, maxit=20000,
                         restart=HEADLINE_RESTART, max_outer=20000, precision=precision,
                         fallback_patience=20, wave_len=wave_len, block_rhs=block_rhs)
    assert rc == sv.OK
    X = host(x)
    worst = 0.0
    for w, win in enumerate(wins):
        orc = so.SaddleOracle(win, k=3, rhat="RR")
        for r in range(nrhs):
            a = off[w] + r * win.n
            b = rhs[a:a + win.n]
            xref = XR[a:a + win.n]
            # the oracle's A confirms the reference
            rr = np.linalg.norm(b - orc.apply_A(xref)) / np.linalg.norm(b)
            assert rr <= 1e-11, (w, r, rr)
            xs = X[a:a + win.n]
            rs = np.linalg.norm(b - orc.apply_A(xs)) / np.linalg.norm(b)
            err = rel(xs, xref)
            blk = max(e for _, e in block_errors(win, xs, xref))
            print(f"window {w} rhs {r}: iters {inf[w * nrhs + r]['iters']}, relres {rs:.2e}, "
                  f"solution error {err:.2e} (worst block {blk:.2e})", flush=True)
            assert rs <= HEADLINE_RTOL * (1 + 1e-6)
            worst = max(worst, err)
    print(f"worst solution error {worst:.2e} at rtol {HEADLINE_RTOL}")
    assert worst <= 1e-6
    h.set_net(None)
    h.close()
