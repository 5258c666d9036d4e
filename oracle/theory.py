"""Closed-form statements of the paper, used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see the header of svar_oracle.py).  Each function states
one result of Tabeart & Pearson (arXiv 2105.06975) as a formula.
"""
from __future__ import annotations

import math

import numpy as np


def theorem1_intervals(lam_D, Lam_D, lam_R, Lam_R, lam_S, Lam_S, lam_L, Lam_L, kappa_D):
    """Theorem 1 (§3): inclusion intervals for the eigenvalues of P_D^{-1} A.

    With lam_Phi = min(lam_D, lam_R), Lam_Phi = max(Lam_D, Lam_R), the lower bound on the
    Schur-complement ratio phi = lam_S lam_L / kappa(D) and the upper bound
    Phi = Lam_S Lam_L kappa(D), the eigenvalues lie in
      [(l - sqrt(l^2 + 4 U Phi))/2, (U - sqrt(U^2 + 4 l phi))/2]  U  [l, U]
      U [(l + sqrt(l^2 + 4 l phi))/2, (U + sqrt(U^2 + 4 U Phi))/2]
    where l = lam_Phi and U = Lam_Phi.  Returns the three (lo, hi) pairs.
    """
    l = min(lam_D, lam_R)
    U = max(Lam_D, Lam_R)
    phi = lam_S * lam_L / kappa_D
    Phi = Lam_S * Lam_L * kappa_D
    return intervals_from(l, U, phi, Phi)


def intervals_from(l, U, phi, Phi):
    """The generic block-diagonal saddle bound used in the proof of Theorem 1."""
    neg = ((l - math.sqrt(l * l + 4 * U * Phi)) / 2, (U - math.sqrt(U * U + 4 * l * phi)) / 2)
    mid = (l, U)
    pos = ((l + math.sqrt(l * l + 4 * l * phi)) / 2, (U + math.sqrt(U * U + 4 * U * Phi)) / 2)
    return neg, mid, pos


def prop1_unit_eigs(N: int, k: int, s: int) -> int:
    """Proposition 1: L_M^{-T} L^T L L_M^{-1} has at least (N + 1 - 2 floor(N/k)) s unit
    eigenvalues for 2 <= k <= N + 1."""
    return (N + 1 - 2 * (N // k)) * s


def prop2_bound(k: int, N: int) -> float:
    """Proposition 2 and Remark 3: if ||M_i M_i^T||_2 <= 1 for all i, the eigenvalues of
    L_M^{-T} L^T L L_M^{-1} are at most k + 1 + 2 sqrt(k), and at most 1 + k + sqrt(k)
    when k <= N < 2k."""
    if k <= N < 2 * k:
        return 1 + k + math.sqrt(k)
    return k + 1 + 2 * math.sqrt(k)


def prop3_spectrum(lam, gamma):
    """Proposition 3: eigenvalues of R_RR^{-1} R are lam / (lam + gamma)."""
    lam = np.asarray(lam, dtype=np.float64)
    return lam / (lam + gamma)


def prop4_spectrum(lam, T):
    """Proposition 4: eigenvalues of R_ME^{-1} R are 1 where lam > T and lam / T otherwise."""
    lam = np.asarray(lam, dtype=np.float64)
    return lam / np.maximum(T, lam)


def remark1_minres_bound(mu1, mu2, mu3, mu4, ell, r0):
    """Remark 1: after 2 ell MINRES steps, with spectrum in [-mu1,-mu2] U [mu3,mu4] and
    mu1 - mu2 = mu4 - mu3, ||r||_{P^{-1}} <= 2 q^ell ||r0||_{P^{-1}},
    q = (sqrt(mu1 mu4) - sqrt(mu2 mu3)) / (sqrt(mu1 mu4) + sqrt(mu2 mu3))."""
    a = math.sqrt(mu1 * mu4)
    b = math.sqrt(mu2 * mu3)
    return 2.0 * ((a - b) / (a + b)) ** ell * r0


def stretch_intervals(neg, pos):
    """Widen [-mu1,-mu2] U [mu3,mu4] so that mu1 - mu2 = mu4 - mu3 (Remark 1)."""
    mu1, mu2 = -neg[0], -neg[1]
    mu3, mu4 = pos
    w1, w2 = mu1 - mu2, mu4 - mu3
    if w1 < w2:
        mu1 = mu2 + w2
    else:
        mu4 = mu3 + w1
    return mu1, mu2, mu3, mu4


def lemma1_block(Ms, k: int, i: int, j: int, s: int):
    """Lemma 1: the (i, j) block (1-based) of L_M(k)^{-1}.

    I if i = j; the product M_{i-1} M_{i-2} ... M_j (prod_{m=1}^{i-j} M_{i-m}) if
    1 <= i - j <= (i - 1) mod k; zero otherwise.  Ms[m] is M_m for m = 1..N (Ms[0] unused).
    """
    if i == j:
        return np.eye(s)
    d = i - j
    if 1 <= d <= (i - 1) % k:
        out = np.eye(s)
        for m in range(1, d + 1):
            out = out @ Ms[i - m]
        return out
    return np.zeros((s, s))


def definition1_block(Ms, k: int, i: int, j: int, s: int):
    """Definition 1: the (i, j) block (1-based) of L_M(k): I on the diagonal, -M_j at
    (j + 1, j) when k does not divide j, zero elsewhere."""
    if i == j:
        return np.eye(s)
    if i == j + 1 and j % k != 0:
        return -Ms[j]
    return np.zeros((s, s))


def circulant_tridiag_inverse_eigs(a, b, c, s):
    """Eigenvalues of T^{-1} for the periodic tridiagonal T x_j = a x_{j-1} + b x_j + c x_{j+1}:
    1 / (b + a e^{-i theta} + c e^{i theta}), theta = 2 pi m / s."""
    th = 2 * np.pi * np.arange(s) / s
    return 1.0 / (b + a * np.exp(-1j * th) + c * np.exp(1j * th))
