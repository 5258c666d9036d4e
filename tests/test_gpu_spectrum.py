"""Spectral diagnostics on the GPU (svar_spectrum, Lanczos in the preconditioner's inner
product) against dense eigenvalues and the paper's closed forms.

* P_D^{-1} A on a tiny window: with n Lanczos steps the extreme Ritz values are the dense
  extreme eigenvalues (Theorem 1's object);
* Rhat^{-1} R at the C2 size (p = 2048): Proposition 3 (R_RR, gamma = lambda_min(R): the
  spectrum is lambda / (lambda + gamma), so its extremes are 1/2 and
  lambda_max / (lambda_max + lambda_min)) and Proposition 4 (R_ME with T = lambda_2: every
  eigenvalue 1 except lambda_1 / lambda_2);
* L_M(k)^{-T} L^T L L_M(k)^{-1} for the contractive advection-diffusion model: the largest
  eigenvalue within Proposition 2's bound, the smallest above 0, both matching dense
  eigenvalues on the C1 window.
"""
import numpy as np
import pytest

from oracle import svar_oracle as so
from oracle import theory as th
from paper_2105_06975_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_06975_amd import svar
    return svar


def test_pd_a_extremes_tiny(sv):
    win = wl.make_small_window(s=10, N=3, p=5, seed=41)
    orc = so.SaddleOracle(win, k=2, rhat="RR")
    h = sv.Handle([win], sv.Precond(type="PD", k=2, rhat="RR"))
    ritz = h.spectrum("PD_A", win.n, seed=1)
    A = orc.A_dense()
    P = orc.operator_dense(lambda v: orc.apply_PD_inv(v))
    ev = np.sort(np.linalg.eigvals(P @ A).real)
    for got, ref in ((ritz[0], ev[0]), (ritz[-1], ev[-1])):
        assert abs(got - ref) <= 1e-8 * max(1.0, abs(ref)), (got, ref)
    # the eigenvalue nearest zero on each side (Theorem 1's inner interval ends)
    neg, pos = ev[ev < 0], ev[ev > 0]
    assert np.min(np.abs(ritz[ritz < 0] - neg.max())) <= 1e-7 * abs(neg.max())
    assert np.min(np.abs(ritz[ritz > 0] - pos.min())) <= 1e-7 * pos.min()


@pytest.fixture(scope="module")
def c2():
    return wl.make_config_window("c2", seed=0)


@pytest.mark.parametrize("rhat", ["RR", "ME"])
def test_rhat_r_closed_forms_at_c2(sv, c2, rhat):
    win = c2
    lam = np.linalg.eigvalsh(win.rmats[0])
    h = sv.Handle([win], sv.Precond(type="PI", k=3, rhat=rhat))
    ritz = h.spectrum("RHAT_R", 300, seed=2)
    if rhat == "RR":
        ref = th.prop3_spectrum(lam, lam[0])
    else:
        ref = th.prop4_spectrum(lam, lam[1])
    print(f"{rhat}: Ritz [{ritz[0]:.10f}, {ritz[-1]:.10f}], closed form [{ref.min():.10f}, "
          f"{ref.max():.10f}]")
    # Ritz values lie inside the spectrum; the clustered small end converges last
    assert -1e-12 <= ritz[0] - ref.min() <= 5e-6 * ref.min()
    assert abs(ritz[-1] - ref.max()) <= 1e-7 * ref.max()


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_lml_bounds(sv, k):
    win = wl.make_config_window("c1", seed=0)
    orc = so.SaddleOracle(win, k=k, rhat="RR")
    h = sv.Handle([win], sv.Precond(type="PI", k=k, rhat="RR"))
    ritz = h.spectrum("LML", 300, seed=3)
    L, Lm = orc.L_dense(), orc.L_dense(k)
    Ti = np.linalg.solve(Lm.T, L.T @ L) @ np.linalg.inv(Lm)
    ev = np.sort(np.linalg.eigvalsh(0.5 * (Ti + Ti.T)))
    assert abs(ritz[-1] - ev[-1]) <= 1e-8 * ev[-1]
    # Ritz values lie inside the spectrum (the smallest converges last)
    assert ritz[0] >= ev[0] * (1 - 1e-9) - 1e-12
    assert ritz[-1] <= th.prop2_bound(k, win.N) * (1 + 1e-12)
    assert ritz[0] > 0
