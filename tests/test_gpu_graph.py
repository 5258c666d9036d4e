"""FGMRES steps replayed from a captured HIP graph give the step-by-step launches' results.

Every replay chunk runs 4 steps; the solves below run tens of chunks, several cycles
(restart) and repeated solves on the same handle (cache reuse, interleaved with eager
work), and each result is compared bit for bit with the eager solve.
"""
import numpy as np
import pytest

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


def _batch():
    return [wl.make_small_window(s=100, N=10, p=40, seed=1),
            wl.make_small_window(s=64, N=7, p=20, seed=2),
            wl.make_small_window(s=130, N=5, p=60, seed=3)]


@pytest.mark.parametrize("restart,precision", [(0, "FP64"), (12, "FP64"), (0, "MIXED_FP32"),
                                               (0, "FP64_F32P")])
def test_graph_solve_equals_eager(sv, restart, precision):
    wins = _batch()
    nrhs = 2
    h = sv.Handle(wins, sv.Precond(type="PI", k=3, rhat="RR"))
    rhs = np.concatenate([wl.random_vectors(w, nrhs, seed=10 + i).ravel()
                          for i, w in enumerate(wins)])
    kw = dict(rtol=1e-9, maxit=400, restart=restart, max_outer=60, precision=precision,
              inner_rtol=1e-5)
    x0, i0, rc0 = h.solve(dev(rhs), nrhs, **kw)
    x0 = host(x0)
    for rep in range(3):
        x1, i1, rc1 = h.solve(dev(rhs), nrhs, graph=True, **kw)
        assert rc1 == rc0
        assert [a["iters"] for a in i1] == [a["iters"] for a in i0]
        assert np.array_equal(host(x1), x0), rep
        # eager work between replays
        h.apply_A(dev(rhs), nrhs)
    assert max(a["iters"] for a in i0) > 8  # several graph chunks ran


def test_graph_with_learned_correction(sv):
    wins = _batch()[:2]
    h = sv.Handle(wins, sv.Precond(type="PI", k=3, rhat="RR"))
    net = sv.Net(3, 2, "BF16")
    rng = np.random.default_rng(5)
    th = wl.net_init(net.cin, 64, seed=4)
    net.set_params(th + 0.01 * rng.standard_normal(th.size))
    h.set_net(net)
    rhs = np.concatenate([wl.random_vectors(w, 1, seed=20 + i).ravel() for i, w in enumerate(wins)])
    x0, i0, _ = h.solve(dev(rhs), 1, rtol=1e-9, maxit=400, fallback_patience=5)
    for rep in range(2):
        x1, i1, _ = h.solve(dev(rhs), 1, rtol=1e-9, maxit=400, fallback_patience=5, graph=True)
        assert [a["iters"] for a in i1] == [a["iters"] for a in i0]
        assert [a["fallbacks"] for a in i1] == [a["fallbacks"] for a in i0]
        assert np.array_equal(host(x1), host(x0)), rep


def test_autotune_cache_roundtrip(sv, tmp_path):
    wins = _batch()
    nrhs = 4
    rhs = np.concatenate([wl.random_vectors(w, nrhs, seed=30 + i).ravel()
                          for i, w in enumerate(wins)])
    h = sv.Handle(wins, sv.Precond(type="PI", k=3, rhat="RR"))
    x0, i0, _ = h.solve(dev(rhs), nrhs, rtol=1e-9, maxit=400)
    x0 = host(x0)
    path = tmp_path / "tune.json"
    h.autotune(nrhs, "FP64", path)
    text = path.read_text()
    # A and P share their product shapes here (D and R vs D and Rhat^{-1}): one key
    assert '"entries"' in text and text.count('"key"') >= 1
    x1, i1, _ = h.solve(dev(rhs), nrhs, rtol=1e-9, maxit=400)
    x1 = host(x1)
    # another plan changes only the rounding order of the products
    assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) < 1e-8
    assert all(abs(a["iters"] - b["iters"]) <= 2 for a, b in zip(i0, i1))
    h2 = sv.Handle(wins, sv.Precond(type="PI", k=3, rhat="RR"))
    h2.autotune_load(path)
    x2, _, _ = h2.solve(dev(rhs), nrhs, rtol=1e-9, maxit=400)
    assert np.array_equal(host(x2), x1)  # same plans, same results
