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
  * Rhat in {diag, block, ridge regression, minimum eigenvalue, R}
                                                              (§5, Alg. 1, 2, 3, §6.1)
  * Dhat = B + 0.01 I, Q + 0.01 I                              (§6.1)
  * FGMRES (right preconditioned, modified Gram-Schmidt, Givens) and
    preconditioned MINRES (Paige-Saunders), x0 = 0               (§7 solver settings)
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

RHAT_KINDS = ("DIAG", "RR", "ME", "EXACT")  # plus "BLOCK", which takes its parameters (rblock)


# =================================================================== R_block (§5.1, Alg. 3)
def rblock_partition(R, pvec, tol, maxsize=None, numproc=None):
    """The groups of consecutive blocks that R_block keeps (Alg. 3, Appendix).

    R is split into pn = len(pvec) blocks of sizes pvec.  For every pair of neighbouring
    blocks j, j+1 the scaled Frobenius norm of the super-diagonal block,
        normvec_j = ||R[block j, block j+1]||_F / sqrt(pvec_j pvec_{j+1}),
    is compared with tol; below it, every coupling across the boundary between blocks j and
    j+1 is removed, so R_block is block diagonal over the groups of blocks between removed
    boundaries (inside a group R is kept whole, higher super-diagonals included).  Then, as
    printed, one adjustment each: a group larger than maxsize is split in two; if there are
    more groups than numproc the two smallest adjacent groups are combined, and if there are
    fewer than numproc - 2 the largest group is split.  A split cuts a group at the block
    boundary nearest its middle row (a group of one block is cut at its middle row), so the
    result is a list of (start, stop) row ranges.  Returns (ranges, normvec)."""
    R = np.asarray(R, dtype=np.float64)
    pvec = [int(v) for v in pvec]
    if any(v < 1 for v in pvec) or sum(pvec) != R.shape[0]:
        raise ValueError("pvec must be positive block sizes summing to p")
    pst = np.concatenate([[0], np.cumsum(pvec)]).astype(int)
    pn = len(pvec)
    normvec = np.array([np.linalg.norm(R[pst[j]:pst[j + 1], pst[j + 1]:pst[j + 2]], "fro") /
                        np.sqrt(pvec[j] * pvec[j + 1]) for j in range(pn - 1)])
    # boundaries between groups: block starts where the coupling is dropped
    cuts = [0] + [int(pst[j + 1]) for j in range(pn - 1) if normvec[j] < tol] + [int(pst[-1])]
    bounds = set(int(b) for b in pst)

    def split(lo, hi):
        inner = [b for b in bounds if lo < b < hi]
        mid = (lo + hi) / 2.0
        c = min(inner, key=lambda b: (abs(b - mid), b)) if inner else (lo + hi) // 2
        return [(lo, c), (c, hi)]

    ranges = [(cuts[i], cuts[i + 1]) for i in range(len(cuts) - 1)]
    if maxsize is not None:
        big = max(range(len(ranges)), key=lambda i: (ranges[i][1] - ranges[i][0], -i))
        lo, hi = ranges[big]
        if hi - lo > maxsize and hi - lo > 1:
            ranges[big:big + 1] = split(lo, hi)
    if numproc is not None:
        if len(ranges) > numproc:
            j = min(range(len(ranges) - 1),
                    key=lambda i: (ranges[i][1] - ranges[i][0] + ranges[i + 1][1] -
                                   ranges[i + 1][0], i))
            ranges[j:j + 2] = [(ranges[j][0], ranges[j + 1][1])]
        elif len(ranges) < numproc - 2:
            big = max(range(len(ranges)), key=lambda i: (ranges[i][1] - ranges[i][0], -i))
            lo, hi = ranges[big]
            if hi - lo > 1:
                ranges[big:big + 1] = split(lo, hi)
    return ranges, normvec


def rblock_matrix(R, ranges):
    """R_block: R on the diagonal blocks of the partition, zero elsewhere."""
    R = np.asarray(R, dtype=np.float64)
    out = np.zeros_like(R)
    for lo, hi in ranges:
        out[lo:hi, lo:hi] = R[lo:hi, lo:hi]
    return out


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
        elif self.kind == "band_dirichlet":
            # (M x)_j = sum_t w_t x_{j + o_t}, entries outside the grid zero (Dirichlet), sparse
            import scipy.sparse as sp
            s = self.s
            rows, cols, vals = [], [], []
            for off, w in zip(m["offsets"], m["weights"]):
                j = np.arange(s)
                ok = (j + off >= 0) & (j + off < s)
                rows.append(j[ok])
                cols.append(j[ok] + off)
                vals.append(np.full(int(ok.sum()), float(w)))
            Mb = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows),
                                                       np.concatenate(cols))), shape=(s, s))
            self.mats = [Mb] * self.N
            self.sparse = True
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
                 d_ridge: float = 0.01, rblock=None, lhat: str = "LM"):
        self.win = win
        # Lhat: "LM" = L_M(k) (Definition 1), "LI" = L_I, the -I subdiagonal (§2.2)
        if lhat not in ("LM", "LI"):
            raise ValueError(lhat)
        self.lhat = lhat
        # R_block parameters (Alg. 3): dict(pvec, tol, maxsize, numproc) per distinct R, or one
        # dict for all
        self.rblock = rblock
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

    def LI_inv(self, v):
        """L_I^{-1} v (§2.2: L with every M_i replaced by I): z_i = v_i + z_{i-1}, the running
        sum over the time blocks."""
        return np.cumsum(v, axis=0)

    def LI_invT(self, v):
        """L_I^{-T} v: w_i = v_i + w_{i+1}, the running sum from the last block backwards."""
        return np.cumsum(v[::-1], axis=0)[::-1]

    def Lhat_inv(self, v):
        return self.LI_inv(v) if self.lhat == "LI" else self.LM_inv(v)

    def Lhat_invT(self, v):
        return self.LI_invT(v) if self.lhat == "LI" else self.LM_invT(v)

    def LI_dense(self):
        s, nb = self.s, self.nb
        Li = np.eye(nb * s)
        for i in range(1, nb):
            Li[i * s:(i + 1) * s, (i - 1) * s: i * s] = -np.eye(s)
        return Li

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
        elif kind == "BLOCK":
            prm = self.rblock[idx] if isinstance(self.rblock, (list, tuple)) else self.rblock
            ranges, normvec = rblock_partition(R, prm["pvec"], prm["tol"], prm.get("maxsize"),
                                               prm.get("numproc"))
            Rh = rblock_matrix(R, ranges)
            self.rhat_params[idx] = dict(ranges=ranges, normvec=normvec)
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
        z3 = self.Lhat_inv(self.D_apply(self.Lhat_invT(v3)))
        return self.join(self.Dhat_inv(v1), self.Rhat_inv(v2), z3)

    def apply_PI_inv(self, v):
        """(c1 = Lhat^{-T} v3, Rhat^{-1} v2, Lhat^{-1}(v1 - D c1))."""
        v1, v2, v3 = self.split(v)
        c1 = self.Lhat_invT(v3)
        z3 = self.Lhat_inv(v1 - self.D_apply(c1))
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


def fgmres_restarted(apply_A, apply_Pinv, rhs, rtol: float, m: int, maxit: int):
    """FGMRES(m): cycles of at most m steps of `fgmres` on A d = r, x += d, with the true
    residual r = rhs - A x recomputed before each cycle; stops when ||r||_2 <= rtol ||rhs||_2
    or after maxit steps in total.  Returns (x, iters, cycles)."""
    nb = float(np.linalg.norm(rhs))
    x = np.zeros(rhs.size)
    if nb == 0.0:
        return x, 0, 0
    used, cycles = 0, 0
    r = rhs.copy()
    while used < maxit:
        nr = float(np.linalg.norm(r))
        if nr <= rtol * nb:
            break
        d, it, _ = fgmres(apply_A, apply_Pinv, r, rtol * nb / nr, min(m, maxit - used))
        x = x + d
        used += it
        cycles += 1
        r = rhs - apply_A(x)
    return x, used, cycles


def block_fgmres(apply_A, apply_Pinv, RHS, rtol: float, maxit: int):
    """Block flexible GMRES over the p columns of RHS (n x p), X0 = 0, no restart.

    The block Arnoldi process: RHS = V_0 S_0 (thin QR); at block step j every column of V_j
    goes through the preconditioner, Z_j = [P^{-1} v for the columns v of V_j], W = A Z_j is
    orthogonalised against V_0..V_j by block modified Gram-Schmidt, H_ij = V_i^T W, and
    W = V_{j+1} H_{j+1,j} (thin QR), so that A [Z_0..Z_j] = [V_0..V_{j+1}] Hbar_j with Hbar_j
    block upper Hessenberg.  X = [Z_0..Z_j] Y with Y minimising ||E_1 S_0 - Hbar_j Y||_F,
    which decouples into one least-squares problem per column; column c's residual is that
    column's least-squares residual.  Stops when every column's residual is <= rtol times its
    right-hand side's norm, at maxit block steps, or when the new block loses rank (a Krylov
    space that is invariant up to rounding: the current X is then the solution).

    Returns (X, steps, hist) with hist[j] the per-column relative residuals after j steps."""
    RHS = np.asarray(RHS, dtype=np.float64)
    n, p = RHS.shape
    nb = np.linalg.norm(RHS, axis=0)
    act = nb > 0
    hist = [np.where(act, 1.0, 0.0)]
    X = np.zeros((n, p))
    if not act.any():
        return X, 0, hist
    V0, S0 = np.linalg.qr(RHS)
    V = [V0]
    Z = []
    Hcols = []       # Hcols[j]: ((j + 2) p x p) block column j of Hbar
    steps = maxit
    Y = None
    for j in range(maxit):
        Zj = np.column_stack([apply_Pinv(V[j][:, c]) for c in range(p)])
        Z.append(Zj)
        W = np.column_stack([apply_A(Zj[:, c]) for c in range(p)])
        col = np.zeros(((j + 2) * p, p))
        for i in range(j + 1):
            Hij = V[i].T @ W
            W = W - V[i] @ Hij
            col[i * p:(i + 1) * p] = Hij
        Q, Rn = np.linalg.qr(W)
        col[(j + 1) * p:] = Rn
        Hcols.append(col)
        # least squares over the current space, column by column
        Hbar = np.zeros(((j + 2) * p, (j + 1) * p))
        for c_ in range(j + 1):
            Hbar[:(c_ + 2) * p, c_ * p:(c_ + 1) * p] = Hcols[c_]
        E = np.zeros(((j + 2) * p, p))
        E[:p] = S0
        Y, *_ = np.linalg.lstsq(Hbar, E, rcond=None)
        res = np.linalg.norm(E - Hbar @ Y, axis=0)
        rel = np.where(act, res / np.where(act, nb, 1.0), 0.0)
        hist.append(rel)
        sv = np.linalg.svd(Rn, compute_uv=False)
        if np.all(rel <= rtol) or sv[-1] <= 1e-14 * max(sv[0], 1e-300):
            steps = j + 1
            break
        V.append(Q)
    Zall = np.column_stack(Z)
    X = Zall @ Y
    return X, steps, hist


def block_fgmres_restarted(apply_A, apply_Pinv, RHS, rtol: float, m: int, maxit: int):
    """Block FGMRES(m): cycles of at most m block steps of `block_fgmres` on A D = R, X += D,
    with the true residual block R = RHS - A X recomputed before each cycle (all p columns
    stay in the block); stops when every column's true residual is <= rtol times its
    right-hand side's norm, or after maxit block steps.  Returns (X, steps, cycles)."""
    RHS = np.asarray(RHS, dtype=np.float64)
    n, p = RHS.shape
    nb = np.linalg.norm(RHS, axis=0)
    X = np.zeros((n, p))
    Rb = RHS.copy()
    used, cycles = 0, 0
    while used < maxit:
        nr = np.linalg.norm(Rb, axis=0)
        if np.all(nr <= rtol * nb):
            break
        # the cycle's tolerance, relative to the cycle's right-hand sides: the tightest column
        tol = float(np.min(np.where(nr > 0, rtol * nb / np.where(nr > 0, nr, 1.0), np.inf)))
        D, st, _ = block_fgmres(apply_A, apply_Pinv, Rb, min(tol, 1.0), min(m, maxit - used))
        X = X + D
        used += st
        cycles += 1
        Rb = RHS - np.column_stack([apply_A(X[:, c]) for c in range(p)])
    return X, used, cycles


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
