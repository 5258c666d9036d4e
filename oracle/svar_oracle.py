"""FP64 CPU oracle for the preconditioned saddle-point solve of weak-constraint 4D-Var.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
HIP library is checked against.  Only the test suite, the smoke check of the
entry module and the CPU-baseline leg of the benchmark may import it; the
library itself never does, and the two share no code.  Inputs come from the
seeded generators (duck-typed window objects with the attributes listed in
``Window`` of the workloads module); this file never imports them.

Everything is float64.  Paper: Tabeart & Pearson, "Saddle point
preconditioners for weak-constraint 4D-Var" (arXiv 2105.06975).

  * Saddle matrix A = [[D,0,L],[0,R,H],[L^T,H^T,0]]           (§2.1, eq. saddlepointA)
  * L: identity diagonal, -M_i on the block subdiagonal        (§2.1, eq. def:L)
  * L_M(k): L with the couplings into every k-th block removed (§4.1, Definition 1)
  * P_D = blkdiag(Dhat, Rhat, Lhat^T D^{-1} Lhat), P_I         (§2.2, eq. prec)
  * A v, P_D^{-1} v, P_I^{-1} v by block loops                  (§6.2)
  * Rhat in {diag, ridge regression, minimum eigenvalue, R}     (§5, Alg. 1, Alg. 2, §6.1)
  * Dhat = B + 0.01 I, Q + 0.01 I                              (§6.1)
  * FGMRES (right preconditioned, modified Gram-Schmidt, Givens) and
    preconditioned MINRES (Paige-Saunders), x0 = 0               (§7 solver settings)
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

RHAT_KINDS = ("DIAG", "RR", "ME", "EXACT")


# =================================================================== models
class ModelOps:
    """Applies M_i and M_i^T (i = 1..N; M_i maps the state at time i-1 to time i)."""

    def __init__(self, win):
        self.s, self.N = win.s, win.N
        m = win.model
        self.kind = m["kind"]
        if self.kind == "tridiag_inv":
            # periodic tridiagonal T with (T x)_j = a x_{j-1} + b x_j + c x_{j+1}; M = T^{-1}
            s = self.s
            T = np.zeros((s, s))
            for j in range(s):
                T[j, (j - 1) % s] += m["a"]
                T[j, j] += m["b"]
                T[j, (j + 1) % s] += m["c"]
            self.T = T
            self._lu = sla.lu_factor(T)
        elif self.kind == "dense":
            self.mats = [np.asarray(Mi, dtype=np.float64) for Mi in m["mats"]]  # M_1..M_N
        elif self.kind == "band":
            s = self.s
            Mb = np.zeros((s, s))
            for off, w in zip(m["offsets"], m["weights"]):
                for j in range(s):
                    Mb[j, (j + off) % s] += w
            self.mats = [Mb] * self.N
        elif self.kind == "l96":
            from oracle.l96_oracle import L96Tangent
            self.l96 = L96Tangent(m["F"], m["dt"], m["nsteps"], np.asarray(m["traj"]))
        else:
            raise ValueError(self.kind)

    def M(self, i: int, x: np.ndarray) -> np.ndarray:
        """M_i x for i in 1..N (x may be a matrix of columns)."""
        assert 1 <= i <= self.N
        if self.kind == "tridiag_inv":
            return sla.lu_solve(self._lu, x)
        if self.kind == "l96":
            return self.l96.jvp(i, x)
        return self.mats[i - 1] @ x

    def MT(self, i: int, x: np.ndarray) -> np.ndarray:
        assert 1 <= i <= self.N
        if self.kind == "tridiag_inv":
            return sla.lu_solve(self._lu, x, trans=1)
        if self.kind == "l96":
            return self.l96.vjp(i, x)
        return self.mats[i - 1].T @ x

    def dense(self, i: int) -> np.ndarray:
        return self.M(i, np.eye(self.s))


# =================================================================== problem
class SaddleOracle:
    """Operators of one window.  Vectors are laid out (eta_0..eta_N | nu_0..nu_N | x_0..x_N)."""

    def __init__(self, win, *, k: int = 1, rhat: str = "RR", rr_gamma=None, me_T=None,
                 d_ridge: float = 0.01):
        self.win = win
        self.s, self.N, self.nb = win.s, win.N, win.N + 1
        self.p = np.asarray(win.p, dtype=np.int64)
        self.poff = np.concatenate([[0], np.cumsum(self.p)])
        self.P = int(self.poff[-1])
        self.n = 2 * self.nb * self.s + self.P
        if not 1 <= k <= self.nb:
            raise ValueError("k must be in 1..N+1 (Definition 1)")
        self.k = k
        self.model = ModelOps(win)
        self.rhat_kind = rhat
        self.d_ridge = d_ridge
        self._rhat = {}
        self.rhat_params = {}
        for idx, R in enumerate(win.rmats):
            self._rhat[idx] = self._rhat_setup(np.asarray(R), rhat, rr_gamma, me_T, idx)
        self._dhat = {}

    # ---------------------------------------------------------- layout
    def split(self, v):
        s, nb = self.s, self.nb
        v1 = v[: nb * s].reshape(nb, s)
        v2 = v[nb * s: nb * s + self.P]
        v3 = v[nb * s + self.P:].reshape(nb, s)
        return v1, v2, v3

    def join(self, c1, c2, c3):
        return np.concatenate([c1.reshape(-1), c2.reshape(-1), c3.reshape(-1)])

    def obs(self, v2, i):
        return v2[self.poff[i]: self.poff[i + 1]]

    # ---------------------------------------------------------- blocks
    def D_block(self, i: int) -> np.ndarray:
        w = self.win
        return float(w.d_scale[i]) * np.asarray(w.dmats[int(w.d_index[i])])

    def R_block(self, i: int) -> np.ndarray:
        return np.asarray(self.win.rmats[int(self.win.r_index[i])])

    def H_apply(self, i: int, x: np.ndarray) -> np.ndarray:
        cols, vals = self.win.h_cols[i], self.win.h_vals[i]
        return np.sum(vals * x[cols], axis=1)

    def HT_apply(self, i: int, y: np.ndarray) -> np.ndarray:
        cols, vals = self.win.h_cols[i], self.win.h_vals[i]
        out = np.zeros(self.s)
        np.add.at(out, cols.reshape(-1), (vals * y[:, None]).reshape(-1))
        return out

    def H_dense(self, i: int) -> np.ndarray:
        Hi = np.zeros((int(self.p[i]), self.s))
        cols, vals = self.win.h_cols[i], self.win.h_vals[i]
        for r in range(cols.shape[0]):
            for c, w in zip(cols[r], vals[r]):
                Hi[r, c] += w
        return Hi

    # ---------------------------------------------------------- L and L_M(k)
    def L_apply(self, x):
        """(L x)_i = x_i - M_i x_{i-1} (eq. def:L)."""
        out = x.copy()
        for i in range(1, self.nb):
            out[i] -= self.model.M(i, x[i - 1])
        return out

    def LT_apply(self, x):
        """(L^T x)_i = x_i - M_{i+1}^T x_{i+1}."""
        out = x.copy()
        for i in range(self.N):
            out[i] -= self.model.MT(i + 1, x[i + 1])
        return out

    def coupled(self, i: int, k=None) -> bool:
        """Whether L_M(k) keeps the coupling from block i-1 into block i (Definition 1).

        In the paper's 1-based numbering block (i+1, i) holds -M_i unless k divides i; with
        0-based time blocks that is the coupling into block i, dropped when k divides i.
        """
        k = self.k if k is None else k
        return i >= 1 and (i % k) != 0

    def LM_inv(self, v, k=None):
        """L_M(k)^{-1} v: forward recurrence z_i = v_i + M_i z_{i-1} inside each segment."""
        z = v.copy()
        for i in range(1, self.nb):
            if self.coupled(i, k):
                z[i] = v[i] + self.model.M(i, z[i - 1])
        return z

    def LM_invT(self, v, k=None):
        """L_M(k)^{-T} v: backward recurrence w_i = v_i + M_{i+1}^T w_{i+1} inside each segment."""
        w = v.copy()
        for i in range(self.N - 1, -1, -1):
            if self.coupled(i + 1, k):
                w[i] = v[i] + self.model.MT(i + 1, w[i + 1])
        return w

    # ---------------------------------------------------------- covariance products
    def D_apply(self, x):
        return np.stack([self.D_block(i) @ x[i] for i in range(self.nb)])

    def R_apply(self, y):
        return np.concatenate([self.R_block(i) @ self.obs(y, i) for i in range(self.nb)])

    def H_full(self, x):
        return np.concatenate([self.H_apply(i, x[i]) for i in range(self.nb)])

    def HT_full(self, y):
        return np.stack([self.HT_apply(i, self.obs(y, i)) for i in range(self.nb)])

    # ---------------------------------------------------------- A v  (§6.2)
    def apply_A(self, v):
        v1, v2, v3 = self.split(v)
        c1 = self.D_apply(v1) + self.L_apply(v3)
        c2 = self.R_apply(v2) + self.H_full(v3)
        c3 = self.LT_apply(v1) + self.HT_full(v2)
        return self.join(c1, c2, c3)

    # ---------------------------------------------------------- Rhat (§5, §6.1)
    def _rhat_setup(self, R, kind, rr_gamma, me_T, idx):
        if R.shape[0] == 0:  # a matrix used only by blocks without observations
            self.rhat_params[idx] = {}
            return ("diag", np.zeros(0))
        if kind == "DIAG":
            self.rhat_params[idx] = {}
            return ("diag", np.diag(R).copy())
        lam, V = np.linalg.eigh(R)
        if kind == "RR":
            # Alg. 1 with the shift chosen directly: gamma = lambda_min(R_i) (§6.1)
            g = lam[0] if rr_gamma is None or rr_gamma < 0 else float(rr_gamma)
            Rh = R + g * np.eye(R.shape[0])
            self.rhat_params[idx] = dict(gamma=float(g))
        elif kind == "ME":
            # Alg. 2 with the threshold set to the second smallest eigenvalue (§6.1)
            T = lam[1] if me_T is None or me_T < 0 else float(me_T)
            Rh = (V * np.maximum(lam, T)) @ V.T
            self.rhat_params[idx] = dict(T=float(T), lam1=float(lam[0]))
        elif kind == "EXACT":
            Rh = R
            self.rhat_params[idx] = {}
        else:
            raise ValueError(kind)
        return ("chol", sla.cho_factor(Rh, lower=True), Rh)

    def Rhat_dense(self, i):
        f = self._rhat[int(self.win.r_index[i])]
        return np.diag(f[1]) if f[0] == "diag" else f[2]

    def Rhat_inv(self, y):
        out = []
        for i in range(self.nb):
            f = self._rhat[int(self.win.r_index[i])]
            yi = self.obs(y, i)
            out.append(yi / f[1] if f[0] == "diag" else sla.cho_solve(f[1], yi))
        return np.concatenate(out)

    # ---------------------------------------------------------- Dhat (§6.1): B + delta I, Q + delta I
    def Dhat_block(self, i):
        return self.D_block(i) + self.d_ridge * np.eye(self.s)

    def Dhat_inv(self, x):
        out = np.empty_like(x)
        for i in range(self.nb):
            key = (int(self.win.d_index[i]), float(self.win.d_scale[i]))
            if key not in self._dhat:
                self._dhat[key] = sla.cho_factor(self.Dhat_block(i), lower=True)
            out[i] = sla.cho_solve(self._dhat[key], x[i])
        return out

    # ---------------------------------------------------------- preconditioners (§6.2)
    def apply_PD_inv(self, v):
        """(Dhat^{-1} v1, Rhat^{-1} v2, Lhat^{-1} D Lhat^{-T} v3)."""
        v1, v2, v3 = self.split(v)
        z3 = self.LM_inv(self.D_apply(self.LM_invT(v3)))
        return self.join(self.Dhat_inv(v1), self.Rhat_inv(v2), z3)

    def apply_PI_inv(self, v):
        """(c1 = Lhat^{-T} v3, Rhat^{-1} v2, Lhat^{-1}(v1 - D c1))."""
        v1, v2, v3 = self.split(v)
        c1 = self.LM_invT(v3)
        z3 = self.LM_inv(v1 - self.D_apply(c1))
        return self.join(c1, self.Rhat_inv(v2), z3)

    def apply_P_inv(self, v, prec: str):
        if prec == "PD":
            return self.apply_PD_inv(v)
        if prec == "PI":
            return self.apply_PI_inv(v)
        if prec == "NONE":
            return v.copy()
        raise ValueError(prec)

    # ---------------------------------------------------------- dense assembly (tiny instances)
    def L_dense(self, k=None):
        """L_M(k) assembled block by block; k=None gives L itself (= L_M(N+1))."""
        s, nb = self.s, self.nb
        kk = nb if k is None else k
        Lm = np.eye(nb * s)
        for i in range(1, nb):
            if self.coupled(i, kk):
                Lm[i * s:(i + 1) * s, (i - 1) * s: i * s] = -self.model.dense(i)
        return Lm

    def blocks_dense(self):
        s, nb = self.s, self.nb
        D = sla.block_diag(*[self.D_block(i) for i in range(nb)])
        R = sla.block_diag(*[self.R_block(i) for i in range(nb)])
        H = sla.block_diag(*[self.H_dense(i) for i in range(nb)])
        return D, R, H, self.L_dense()

    def A_dense(self):
        D, R, H, L = self.blocks_dense()
        Z = np.zeros
        S, P = D.shape[0], R.shape[0]
        return np.block([[D, Z((S, P)), L], [Z((P, S)), R, H], [L.T, H.T, Z((S, S))]])

    def operator_dense(self, fn):
        """Dense matrix of a linear map given as a function of a saddle vector."""
        n = self.n
        out = np.empty((n, n))
        I = np.eye(n)
        for j in range(n):
            out[:, j] = fn(I[:, j])
        return out

    def xspace_dense(self, fn):
        s, nb = self.s, self.nb
        n = nb * s
        out = np.empty((n, n))
        I = np.eye(n)
        for j in range(n):
            out[:, j] = fn(I[:, j].reshape(nb, s)).reshape(-1)
        return out


# =================================================================== primal form
def primal_solution(orc: SaddleOracle, b, d):
    """Solution of the saddle system through the primal normal equations.

    Eliminating eta and nu from eq. saddlepointsystem (rhs (b; d; 0)) gives
      (L^T D^{-1} L + H^T R^{-1} H) x = L^T D^{-1} b + H^T R^{-1} d,
      eta = D^{-1}(b - L x),  nu = R^{-1}(d - H x),
    with S = L^T D^{-1} L + H^T R^{-1} H the (negative) Schur complement of §2.2.
    """
    D, R, H, L = orc.blocks_dense()
    Di = np.linalg.inv(D)
    Ri = np.linalg.inv(R)
    S = L.T @ Di @ L + H.T @ Ri @ H
    x = np.linalg.solve(S, L.T @ Di @ b + H.T @ Ri @ d)
    eta = Di @ (b - L @ x)
    nu = Ri @ (d - H @ x)
    return np.concatenate([eta, nu, x])


# =================================================================== Krylov
def fgmres(apply_A, apply_Pinv, rhs, rtol: float, maxit: int):
    """Right-preconditioned flexible GMRES, x0 = 0, no restarts, modified Gram-Schmidt.

    Stops when the Givens residual estimate |g_{j+1}| <= rtol * ||rhs||_2 (the relative
    residual in the two norm, §6.2/§7) or at maxit.  Returns (x, iters, hist) where hist[j]
    is the estimated relative residual after j iterations.
    """
    beta = float(np.linalg.norm(rhs))
    n = rhs.size
    if beta == 0.0:
        return np.zeros(n), 0, [0.0]
    V = [rhs / beta]
    Z = []
    H = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    hist = [1.0]
    iters = maxit
    for j in range(maxit):
        z = apply_Pinv(V[j])
        Z.append(z)
        w = apply_A(z)
        for i in range(j + 1):
            H[i, j] = float(np.dot(w, V[i]))
            w = w - H[i, j] * V[i]
        hnext = float(np.linalg.norm(w))
        H[j + 1, j] = hnext
        for i in range(j):
            a, b_ = H[i, j], H[i + 1, j]
            H[i, j] = cs[i] * a + sn[i] * b_
            H[i + 1, j] = -sn[i] * a + cs[i] * b_
        rho = float(np.hypot(H[j, j], H[j + 1, j]))
        cs[j], sn[j] = H[j, j] / rho, H[j + 1, j] / rho
        H[j, j], H[j + 1, j] = rho, 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        hist.append(abs(g[j + 1]) / beta)
        if abs(g[j + 1]) <= rtol * beta or hnext == 0.0:
            iters = j + 1
            break
        V.append(w / hnext)
    y = sla.solve_triangular(H[:iters, :iters], g[:iters])
    x = np.zeros(n)
    for i in range(iters):
        x += y[i] * Z[i]
    return x, iters, hist


def minres(apply_A, apply_Minv, rhs, rtol: float, maxit: int, norm: str = "P"):
    """Preconditioned MINRES (Paige-Saunders) for symmetric A and SPD preconditioner M.

    The Lanczos process runs in the M^{-1} inner product; the tridiagonal least-squares
    problem is solved by Givens rotations.  norm="P": stop when the M^{-1}-norm residual
    estimate phibar <= rtol * beta_1 (hist: the estimate / beta_1).  norm="2": stop when the
    true residual ||rhs - A x||_2 <= rtol ||rhs||_2, recomputed from x after every iteration
    (§7 asks for a residual criterion in the two norm; hist: that relative residual).
    Returns (x, iters, hist).
    """
    if norm not in ("P", "2"):
        raise ValueError(norm)
    nrhs = float(np.linalg.norm(rhs))
    n = rhs.size
    x = np.zeros(n)
    r_prev = np.zeros(n)
    r = rhs.copy()
    y = apply_Minv(r)
    beta1 = float(np.sqrt(max(np.dot(r, y), 0.0)))
    if beta1 == 0.0:
        return x, 0, [0.0]
    beta, beta_old = beta1, 0.0
    phibar = beta1
    c, s = -1.0, 0.0
    dbar, eps = 0.0, 0.0
    w = np.zeros(n)
    w_old = np.zeros(n)
    hist = [1.0]
    iters = maxit
    for k in range(1, maxit + 1):
        v = y / beta
        y = apply_A(v)
        if k >= 2:
            y = y - (beta / beta_old) * r_prev
        alpha = float(np.dot(v, y))
        y = y - (alpha / beta) * r
        r_prev, r = r, y
        y = apply_Minv(r)
        beta_old = beta
        beta = float(np.sqrt(max(np.dot(r, y), 0.0)))
        # apply the previous rotation to the new tridiagonal column, then make a new one
        eps_old = eps
        delta = c * dbar + s * alpha
        gbar = s * dbar - c * alpha
        eps = s * beta
        dbar = -c * beta
        gamma = float(np.hypot(gbar, beta))
        gamma = max(gamma, np.finfo(float).tiny)
        c, s = gbar / gamma, beta / gamma
        phi = c * phibar
        phibar = s * phibar
        w_new = (v - eps_old * w_old - delta * w) / gamma
        w_old, w = w, w_new
        x = x + phi * w
        if norm == "P":
            hist.append(phibar / beta1)
            stop = phibar <= rtol * beta1
        else:
            rel2 = float(np.linalg.norm(rhs - apply_A(x))) / nrhs
            hist.append(rel2)
            stop = rel2 <= rtol
        if stop or beta == 0.0:
            iters = k
            break
    return x, iters, hist


def solve(orc: SaddleOracle, rhs, *, prec="PI", method="FGMRES", rtol=1e-6, maxit=1000,
          minres_norm="2"):
    A = orc.apply_A
    P = lambda v: orc.apply_P_inv(v, prec)  # noqa: E731
    if method == "FGMRES":
        x, it, hist = fgmres(A, P, rhs, rtol, maxit)
    elif method == "MINRES":
        x, it, hist = minres(A, P, rhs, rtol, maxit, norm=minres_norm)
    else:
        raise ValueError(method)
    res = rhs - A(x)
    nr = float(np.linalg.norm(rhs))
    relres = float(np.linalg.norm(res)) / nr if nr > 0 else 0.0
    return dict(x=x, iters=it, hist=hist, relres_true=relres)
