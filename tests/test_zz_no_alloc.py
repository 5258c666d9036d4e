"""The allocation-free y = A v entry point (svar_apply_A_noalloc) against svar_apply_A
(collected last: a failure here hides no other test).

Both run the same launch program; the no-alloc variant takes its split-K partial sums from a
static device array instead of the handle's workspace, so the results are bitwise equal.
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


def _windows():
    # two uneven windows (odd s, ragged p) plus a C1-sized one: several GEMM problems
    w1 = wl.make_small_window(s=37, N=5, p=11, seed=3)
    w2 = wl.make_config_window("c1", seed=1)
    w3 = wl.make_small_window(s=64, N=3, p=20, seed=4)
    return [w1, w2, w3]


def test_noalloc_matches_apply_A_two_calls(sv):
    wins = _windows()
    h = sv.Handle(wins, sv.Precond(type="PI", k=2, rhat="RR"))
    rng = np.random.default_rng(7)
    for nrhs in (3, 1):  # the second call with a smaller input
        n = h.space_len("saddle", nrhs)
        v = torch.from_numpy(rng.standard_normal(n)).cuda()
        print(f"noalloc: nrhs={nrhs} n={n}", flush=True)
        y_ref = h.apply_A(v, nrhs)  # builds the program of this nrhs
        y = torch.full_like(v, float("nan"))
        h.apply_A_noalloc(v, y, nrhs)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
    h.close()


def test_noalloc_needs_a_built_program(sv):
    h = sv.Handle([wl.make_small_window(s=16, N=2, p=6, seed=5)], sv.Precond(type="PI", k=1))
    v = torch.zeros(h.space_len("saddle", 2), dtype=torch.float64, device="cuda")
    y = torch.empty_like(v)
    with pytest.raises(sv.SvarError, match="no launch program"):
        h.apply_A_noalloc(v, y, 2)
    h.close()
