"""The learned correction of the Lhat^{-T} sweep on the GPU, against the float64 oracle.

* network forward (float32 and bfloat16 inference), loss and gradient (float32), one Adam
  step and the pair normalisation, element by element;
* the corrected P_I / P_D through the C ABI, on uneven windows and several rhs; the
  bfloat16 inference also against the oracle's bfloat16 storage model, 300x tighter;
* a zero network reproduces the plain preconditioner exactly; the harvested Arnoldi
  vectors equal the oracle FGMRES's;
* a garbage network trips the fallback and the solve still converges;
* training on harvested pairs, then solves on held-out windows: what the network gains.
"""
import numpy as np
import pytest

from oracle import learned_oracle as lo
from oracle import svar_oracle as so
from paper_2105_06975_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

K, S = 3, 2
CIN = 1 + S + K
C = 64


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
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / (nb if nb > 0 else 1.0))


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def theta_random(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    th = wl.net_init(CIN, C, seed=seed)
    return f32(scale * th + 0.02 * rng.standard_normal(th.size))


def test_net_forward_parity(sv):
    rng = np.random.default_rng(0)
    npair, nb, s = 2, 7, 100  # two tiles per block, the second ragged
    x = f32(rng.standard_normal((npair, nb, s)))
    theta = theta_random(1)
    net = sv.Net(K, S, "FP32")
    net.set_params(theta)
    assert net.nparams == lo.nparams(CIN, C)
    assert np.array_equal(net.get_params().astype(np.float64), theta)
    X = torch.from_numpy(x.astype(np.float32)).cuda()
    ref = np.stack([lo.forward(theta, lo.features(x[p], K, S), C) for p in range(npair)])
    out32 = host(net.forward(X, "FP32"))
    outbf = host(net.forward(X, "BF16"))
    e32, ebf = rel(out32, ref), rel(outbf, ref)
    print(f"forward rel err fp32 {e32:.2e} bf16 {ebf:.2e}")
    assert e32 <= 1e-5
    assert ebf <= 3e-2


def test_net_loss_gradient_and_adam_parity(sv):
    rng = np.random.default_rng(2)
    npair, nb, s = 2, 8, 70
    x = f32(rng.standard_normal((npair, nb, s)))
    y = f32(0.3 * rng.standard_normal((npair, nb, s)))
    theta = theta_random(3)
    net = sv.Net(K, S, "FP32")
    net.set_params(theta)
    X = torch.from_numpy(x.astype(np.float32)).cuda()
    Y = torch.from_numpy(y.astype(np.float32)).cuda()
    samples = np.array([(0, 0), (0, 2), (0, 3), (1, 7), (1, 5), (1, 6), (0, 7)])
    loss, grad = net.train_step(X, Y, samples, adam=None, want_loss=True, want_grad=True)
    Xo = np.stack([lo.features(x[p], K, S)[b] for p, b in samples])
    Yo = np.stack([y[p][b] for p, b in samples])
    loss_ref, g_ref = lo.loss_and_grad(theta, Xo, Yo, C)
    eg = rel(grad, g_ref)
    print(f"loss {loss:.6e} ref {loss_ref:.6e} grad rel err {eg:.2e}")
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    assert eg <= 1e-5
    # the parameters did not move without Adam
    assert np.array_equal(net.get_params().astype(np.float64), theta)
    # one Adam step from fresh moments
    lr = 1e-3
    net.train_step(X, Y, samples, adam=dict(lr=lr), want_loss=False)
    th_ref, _, _ = lo.adam_step(theta, grad.astype(np.float64), np.zeros_like(theta),
                                np.zeros_like(theta), 1, lr)
    th_gpu = net.get_params().astype(np.float64)
    assert rel(th_gpu - theta, th_ref - theta) <= 1e-5


def test_make_pairs_parity(sv):
    rng = np.random.default_rng(4)
    npair, nb, s = 3, 5, 37
    chat = rng.standard_normal((npair, nb, s))
    cex = chat + 0.5 * rng.standard_normal((npair, nb, s))
    chat[1] = 0.0
    x, y = sv.make_pairs(dev(chat).reshape(npair, nb, s), dev(cex).reshape(npair, nb, s))
    x, y = host(x), host(y)
    for p in range(npair):
        xr, yr = lo.make_pair(chat[p], cex[p])
        assert rel(x[p], xr) <= 1e-6 and rel(y[p], yr) <= 1e-6
    assert not x[1].any() and not y[1].any()


def _windows():
    # uneven: s = 100 (ragged tiles), N = 10; s = 64, N = 7 (a short last segment)
    return [wl.make_small_window(s=100, N=10, p=40, seed=5),
            wl.make_small_window(s=64, N=7, p=20, seed=6)]


@pytest.mark.parametrize("ptype", ["PI", "PD"])
@pytest.mark.parametrize("netprec,tol", [("FP32", 1e-5), ("BF16", 3e-2)])
def test_corrected_preconditioner_parity(sv, ptype, netprec, tol):
    wins = _windows()
    nrhs = 2
    theta = theta_random(7)
    h = sv.Handle(wins, sv.Precond(type=ptype, k=K, rhat="RR"))
    off = h.offsets(nrhs)
    V = np.concatenate([wl.random_vectors(w, nrhs, seed=8 + i).ravel() for i, w in enumerate(wins)])
    plain = host(h.apply_P(dev(V), nrhs))
    net = sv.Net(K, S, netprec)
    net.set_params(theta)
    h.set_net(net)
    out = host(h.apply_P(dev(V), nrhs))
    for w, win in enumerate(wins):
        orc = so.SaddleOracle(win, k=K, rhat="RR")
        fn = lo.apply_PI_inv_learned if ptype == "PI" else lo.apply_PD_inv_learned
        for r in range(nrhs):
            a = off[w] + r * win.n
            v = V[a:a + win.n]
            ref = fn(orc, theta, v, C, S)
            ref_plain = orc.apply_PI_inv(v) if ptype == "PI" else orc.apply_PD_inv(v)
            assert rel(plain[a:a + win.n], ref_plain) <= 1e-10
            e = rel(out[a:a + win.n] - plain[a:a + win.n], ref - ref_plain)
            print(f"{ptype} {netprec} window {w} rhs {r}: correction rel err {e:.2e}")
            assert e <= tol
    # detaching restores the plain preconditioner
    h.set_net(None)
    assert np.array_equal(host(h.apply_P(dev(V), nrhs)), plain)


@pytest.mark.parametrize("ptype", ["PI", "PD"])
def test_bf16_inference_matches_bf16_storage_model(sv, ptype):
    # the fused bfloat16 kernel rounds what the model rounds; only float32 accumulation
    # differs (tiles of 128 points: s = 100 is one ragged tile, s = 300 three with wrap)
    wins = _windows() + [wl.make_small_window(s=300, N=5, p=60, seed=21)]
    nrhs = 2
    theta = theta_random(22)
    h = sv.Handle(wins, sv.Precond(type=ptype, k=K, rhat="RR"))
    off = h.offsets(nrhs)
    V = np.concatenate([wl.random_vectors(w, nrhs, seed=23 + i).ravel() for i, w in enumerate(wins)])
    plain = host(h.apply_P(dev(V), nrhs))
    net = sv.Net(K, S, "BF16")
    net.set_params(theta)
    h.set_net(net)
    out = host(h.apply_P(dev(V), nrhs))
    fn = lo.apply_PI_inv_learned if ptype == "PI" else lo.apply_PD_inv_learned
    for w, win in enumerate(wins):
        orc = so.SaddleOracle(win, k=K, rhat="RR")
        model = lambda chat_n: lo.forward_bf16(theta, lo.features(chat_n, K, S), C)
        for r in range(nrhs):
            a = off[w] + r * win.n
            v = V[a:a + win.n]
            ref = fn(orc, theta, v, C, S, net_fn=model)
            ref_plain = orc.apply_PI_inv(v) if ptype == "PI" else orc.apply_PD_inv(v)
            e = rel(out[a:a + win.n] - plain[a:a + win.n], ref - ref_plain)
            print(f"{ptype} window {w} rhs {r}: bf16-model rel err {e:.2e}")
            assert e <= 1e-4  # measured <= 3.5e-6 (against the float64 network: ~5e-3)


def test_zero_network_is_the_plain_preconditioner(sv):
    win = wl.make_small_window(s=100, N=10, p=40, seed=9)
    h = sv.Handle([win], sv.Precond(type="PI", k=K, rhat="RR"))
    v = dev(wl.random_vectors(win, 1, seed=10))
    plain = host(h.apply_P(v))
    net = sv.Net(K, S, "BF16")
    h.set_net(net)
    assert np.array_equal(host(h.apply_P(v)), plain)


def test_harvest_matches_oracle_arnoldi_vectors(sv):
    win = wl.make_small_window(s=40, N=6, p=15, seed=11)
    orc = so.SaddleOracle(win, k=K, rhat="RR")
    rhs = wl.random_vectors(win, 1, seed=12)[0]
    V = []

    def P(v):
        V.append(v.copy())
        return orc.apply_PI_inv(v)

    _, it_ref, _ = so.fgmres(orc.apply_A, P, rhs, 1e-8, 300)
    h = sv.Handle([win], sv.Precond(type="PI", k=K, rhat="RR"))
    L = win.nb * win.s
    cap = it_ref + 10
    buf = torch.zeros((cap, L), dtype=torch.float64, device="cuda")
    _, info, rc = h.solve(dev(rhs), rtol=1e-8, maxit=300, harvest=buf)
    assert rc == sv.OK
    it = info[0]["iters"]
    assert abs(it - it_ref) <= 2
    got = host(buf)
    for j in range(min(8, it)):
        ref = V[j][-L:]
        assert rel(got[j], ref) <= 1e-8, j
    assert not got[it + 4:].any()  # slots after convergence stay untouched


def test_fallback_rescues_a_garbage_network(sv):
    win = wl.make_small_window(s=100, N=10, p=40, seed=13)
    orc = so.SaddleOracle(win, k=K, rhat="RR")
    rhs = wl.random_vectors(win, 1, seed=14)[0]
    rhs[-win.nb * win.s:] = 0.0
    x_ref = np.linalg.solve(orc.A_dense(), rhs)
    h = sv.Handle([win], sv.Precond(type="PI", k=K, rhat="RR"))
    net = sv.Net(K, S, "BF16")
    net.set_params(theta_random(15, scale=30.0))
    h.set_net(net)
    x, info, rc = h.solve(dev(rhs), rtol=1e-8, maxit=600)
    print("garbage net:", info[0])
    assert rc == sv.OK
    assert info[0]["fallbacks"] == 1
    assert rel(host(x), x_ref) <= 1e-6


def test_training_gain_on_held_out_windows(sv):
    """Train on pairs harvested from plain solves, then solve held-out windows with and
    without the network: the learned path must reach the same solution, and fewer
    iterations is the gain it is for."""
    from paper_2105_06975_amd import learned
    s, N = 128, 12
    train_w = [wl.make_c5_like(s, N, seed=sd) for sd in range(6)]
    chat, cex = learned.harvest_pairs(train_w, K, rtol=1e-6, maxit=400, cap=300)
    x, y = sv.make_pairs(chat, cex)
    net = sv.Net(K, S, "BF16")
    net.set_params(wl.net_init(CIN, C, seed=0))
    hist = learned.train(net, x, y, epochs=8, batch=64, lr=1e-3, seed=0)
    print("pairs", x.shape[0], "epoch losses", [round(v, 4) for v in hist])
    assert hist[-1] < 0.5 * hist[0]
    gains = []
    for sd in (1000001, 1000002):
        win = wl.make_c5_like(s, N, seed=sd)
        orc = so.SaddleOracle(win, k=K, rhat="RR")
        x_ref = np.linalg.solve(orc.A_dense(), win.rhs[0])
        h = sv.Handle([win], sv.Precond(type="PI", k=K, rhat="RR"))
        rhs = dev(win.rhs[0])
        xp, ip, rcp = h.solve(rhs, rtol=1e-6, maxit=600)
        h.set_net(net)
        xl, il, rcl = h.solve(rhs, rtol=1e-6, maxit=600)
        _, il0, _ = h.solve(rhs, rtol=1e-6, maxit=600, fallback_drop=0.0)
        print(f"seed {sd}: learned without fallback {il0[0]['iters']} its")
        assert rcp == sv.OK and rcl == sv.OK
        ep, el = rel(host(xp), x_ref), rel(host(xl), x_ref)
        print(f"seed {sd}: plain {ip[0]['iters']} its (err {ep:.1e}), learned {il[0]['iters']}"
              f" its (err {el:.1e}, fallbacks {il[0]['fallbacks']})")
        # both stop at the same true relative residual, so their errors share one bound
        assert el <= max(10 * ep, 1e-6)
        gains.append(ip[0]["iters"] - il[0]["iters"])
    assert min(gains) > 0


def test_train_loop_checkpoint_and_resume(sv, tmp_path):
    """svar_train: two epochs in one call equal one epoch, a checkpoint, and a resumed call
    for the second epoch (bitwise: the sample order of each epoch is rebuilt from the seed and
    the Adam moments and step count come back from the file); svar_load_learned restores the
    parameters and reports the data cursor."""
    rng = np.random.default_rng(31)
    npair, nb, s = 3, 5, 100
    x = torch.from_numpy(f32(rng.standard_normal((npair, nb, s))).astype(np.float32)).cuda()
    y = torch.from_numpy(f32(0.1 * rng.standard_normal((npair, nb, s))).astype(np.float32)).cuda()
    theta0 = theta_random(7, scale=0.5)
    a = sv.Net(K, S, "FP32")
    a.set_params(theta0)
    ha = a.train(x, y, epochs=2, batch=4, lr=1e-3, seed=5, ckpt=tmp_path / "a.ckpt")
    pa = a.get_params()
    b = sv.Net(K, S, "FP32")
    b.set_params(theta0)
    hb1 = b.train(x, y, epochs=1, batch=4, lr=1e-3, seed=5, ckpt=tmp_path / "b.ckpt")
    c = sv.Net(K, S, "FP32")
    c.set_params(np.zeros_like(theta0))
    hc = c.train(x, y, epochs=2, batch=4, lr=1e-3, seed=5, ckpt=tmp_path / "b.ckpt", resume=True)
    pc = c.get_params()
    assert np.array_equal(pa, pc)
    assert hb1[0] == ha[0] and hc[1] == ha[1]
    assert ha[1] < ha[0]
    d = sv.Net(K, S, "FP32")
    cur = d.load(tmp_path / "a.ckpt")
    steps_per_epoch = -(-npair * nb // 4)
    assert cur == (2, 0, 2 * steps_per_epoch)
    assert np.array_equal(d.get_params(), pa)
    e = sv.Net(K, S + 1, "FP32")
    with pytest.raises(sv.SvarError, match="another network shape"):
        e.load(tmp_path / "a.ckpt")
    for n in (a, b, c, d, e):
        n.close()
