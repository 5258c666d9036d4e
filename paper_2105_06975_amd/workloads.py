"""Seeded synthetic inputs for the weak-constraint 4D-Var saddle-point solve.

This module only *draws problem data*: covariance matrices, observation
operators, model coefficients and right-hand sides.  It holds none of the
solver's arithmetic (no saddle-point operator, no preconditioner, no Krylov
step), so both the HIP path and the CPU oracle can take their inputs from it.

Problem statement (Tabeart & Pearson, §2.1, eq. saddlepointsystem and
eq. saddlepointA): a window has time blocks i = 0..N, a state of size s per
block, p_i observations at time i, covariances D = blkdiag(B, Q_1..Q_N),
R = blkdiag(R_0..R_N), H = blkdiag(H_i) and the model maps M_i (x_{i-1} -> x_i).

Covariance recipe (paper §6.1 and eq. SOAR, with the readings recorded in the
design notes): second-order auto-regressive correlations sigma^2 (1 + r/l) e^{-r/l}
with the chordal distance r = sin(pi |dx|)/pi on the unit periodic domain (the
arc distance makes SOAR indefinite).  As in §6.1, R_i is kept well conditioned:
when its condition number exceeds KAPPA_R_MAX it is shifted by a multiple of the
identity so that it equals KAPPA_R_MAX (the paper floors lambda_min(R_i) so that
kappa(R_i) stays below about 707/0.41 ~ 1724, Table 2).

Model (advection-diffusion): backward-Euler upwind advection with Courant number
C plus centred diffusion nu on a periodic grid, i.e. T x = x_new with
(T x)_j = -(C+nu) x_{j-1} + (1+C+2 nu) x_j - nu x_{j+1}; M = T^{-1}.  The
generator only reports (a, b, c) = (-(C+nu), 1+C+2nu, -nu).

Right-hand side: the first outer loop of incremental 4D-Var started from a
free model run has b = 0 and d_i = y_i - H_i x_i.  Innovations are drawn
directly as d_i = H_i e_i + R_i^{1/2} eps_i with a smooth signal e_i = B^{1/2} xi_i;
no nature run of the model is made for the linear workloads.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

KAPPA_R_MAX = 1724.0

# Workload descriptions (sizes as in the five configurations this library is
# measured on).  C1 is the small case, C2 the single-window headline shape.
CONFIGS = {
    "c1": dict(s=100, N=10, obs="every", obs_stride=2, r_kind="soar", r_len=0.05, r_var=0.5,
               b_len=0.1, b_var=1.0, q_scale=0.1, courant=0.5, nu=0.1),
    "c2": dict(s=4096, N=64, obs="random", p=2048, r_kind="soar", r_len=0.05, r_var=0.5,
               b_len=0.1, b_var=1.0, q_scale=0.1, courant=0.5, nu=0.1),
    "c5": dict(s=4096, N=32, obs="random", p=2048, r_kind="soar", r_len=0.05, r_var=0.5,
               b_len=0.1, b_var=1.0, q_scale=0.1, courant=0.5, nu=0.1),
}


@dataclass
class Window:
    """One assimilation window, all arrays float64 / int32, row-major."""
    s: int
    N: int
    p: np.ndarray                       # [N+1] observations per block
    dmats: list                         # distinct s x s covariance matrices
    d_index: np.ndarray                 # [N+1] D_i = d_scale[i] * dmats[d_index[i]]
    d_scale: np.ndarray                 # [N+1]
    rmats: list                         # distinct p_i x p_i observation covariances
    r_index: np.ndarray                 # [N+1] R_i = rmats[r_index[i]]
    h_width: int                        # ELL width of each H_i row
    h_cols: list                        # [N+1] int32 arrays (p_i, w), state index per entry
    h_vals: list                        # [N+1] float64 arrays (p_i, w)
    model: dict                         # see module docstring
    rhs: Optional[np.ndarray] = None    # [nrhs, n] saddle right-hand sides (b; d; 0)
    meta: dict = field(default_factory=dict)

    @property
    def nb(self) -> int:
        return self.N + 1

    @property
    def P(self) -> int:
        return int(np.sum(self.p))

    @property
    def n(self) -> int:
        return 2 * self.nb * self.s + self.P


# ---------------------------------------------------------------- covariances
def chordal_distance(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Chordal distance between points x, y of the unit periodic domain."""
    d = np.abs(x[:, None] - y[None, :])
    return np.sin(np.pi * d) / np.pi


def soar_matrix(pos: np.ndarray, length: float, var: float) -> np.ndarray:
    r = chordal_distance(pos, pos) / length
    return var * (1.0 + r) * np.exp(-r)


def gaussian_grid_matrix(idx: np.ndarray, s: int, length_cells: float, var: float) -> np.ndarray:
    """exp(-d^2 / (2 l^2)) with d the periodic grid distance in cells."""
    d = np.abs(idx[:, None] - idx[None, :]).astype(np.float64)
    d = np.minimum(d, s - d)
    return var * np.exp(-d * d / (2.0 * length_cells ** 2))


def recondition(R: np.ndarray, kappa_max: float = KAPPA_R_MAX) -> tuple[np.ndarray, float]:
    """Shift R by a multiple of I so that its condition number is at most kappa_max.

    Returns (R_shifted, shift).  A no-op when R is already that well conditioned.
    """
    lam = np.linalg.eigvalsh(R)
    lmin, lmax = lam[0], lam[-1]
    if lmin > 0 and lmax / lmin <= kappa_max:
        return R, 0.0
    shift = (lmax - kappa_max * lmin) / (kappa_max - 1.0)
    return R + shift * np.eye(R.shape[0]), float(shift)


def _spd_sqrt_factor(C: np.ndarray) -> np.ndarray:
    """A factor F with F F^T = C for drawing correlated samples."""
    try:
        return np.linalg.cholesky(C)
    except np.linalg.LinAlgError:
        lam, V = np.linalg.eigh(C)
        return V * np.sqrt(np.clip(lam, 0.0, None))


# ---------------------------------------------------------------- the paper's own covariances
def modified_soar_row(s: int, L: float, maxval: int, sigma: float) -> np.ndarray:
    """First row of the circulant B / Q of §6.1 (eq. SOAR): entry i (circular index distance
    d = min(i, s - i)) is sigma (1 + r) e^{-r} with r = 2 |sin(d theta / 2)| / L and
    theta = pi / maxval for d <= maxval, zero beyond (maxval fixes the nonzeros per row).
    The printed bracketing puts the exponential inside the factor; the standard SOAR form
    (1 + r) e^{-r} is taken."""
    i = np.arange(s)
    d = np.minimum(i, s - i)
    r = 2.0 * np.abs(np.sin(d * (np.pi / maxval) / 2.0)) / L
    c = sigma * (1.0 + r) * np.exp(-r)
    c[d > maxval] = 0.0
    return c


def modified_soar_matrix(s: int, L: float, maxval: int, sigma: float,
                         rng: np.random.Generator) -> np.ndarray:
    """The circulant B or Q of §6.1 (B: L = 0.6, maxval = 100, sigma = 0.4; Q: 0.5, 120, 0.2):
    when its smallest eigenvalue is negative, |lambda_min| + psi (psi ~ U[0, 0.5]) is added
    to the diagonal."""
    c = modified_soar_row(s, L, maxval, sigma)
    idx = (np.arange(s)[None, :] - np.arange(s)[:, None]) % s
    C = c[idx]
    lam_min = float(np.min(np.fft.fft(c).real))  # eigenvalues of a symmetric circulant
    if lam_min < 0:
        C = C + (abs(lam_min) + rng.uniform(0.0, 0.5)) * np.eye(s)
    return C


def block_obs_covariance(pvec, pcorr, rng: np.random.Generator, density: float = 0.5,
                         lam_min: float = 0.41) -> np.ndarray:
    """An inter-channel observation-error covariance with block structure (§6.1): diagonal
    blocks are the Hadamard product of a sparse random matrix (entries U(0, 1), the given
    density) and a SOAR matrix of the block (eq. SOAR with L = 0.6, maxval = the block size,
    sigma = 1); the off-diagonal block (k, l), k < l, is a sparse random matrix with entries in
    (0, pcorr_m) (m runs over the pairs k < l in row order; pcorr_m = 0: uncorrelated).  The
    diagonal blocks and the upper half are added and symmetrised, and the matrix is shifted by
    a multiple of I so that its smallest eigenvalue is lam_min (0.41 in the paper)."""
    pvec = [int(v) for v in pvec]
    p = sum(pvec)
    pst = np.concatenate([[0], np.cumsum(pvec)])
    A = np.zeros((p, p))
    m = 0
    for k, nk in enumerate(pvec):
        c = modified_soar_row(nk, 0.6, max(1, nk), 1.0)
        idx = (np.arange(nk)[None, :] - np.arange(nk)[:, None]) % nk
        mask = rng.uniform(size=(nk, nk)) < density
        A[pst[k]:pst[k + 1], pst[k]:pst[k + 1]] = c[idx] * mask * rng.uniform(size=(nk, nk))
        for l_ in range(k + 1, len(pvec)):
            nl = pvec[l_]
            pc = float(pcorr[m])
            m += 1
            if pc > 0:
                mask = rng.uniform(size=(nk, nl)) < density
                A[pst[k]:pst[k + 1], pst[l_]:pst[l_ + 1]] = mask * rng.uniform(0.0, pc,
                                                                               size=(nk, nl))
    R = np.triu(A) + np.triu(A, 1).T
    lam = np.linalg.eigvalsh(R)
    return R + (lam_min - lam[0]) * np.eye(p)


# ---------------------------------------------------------------- windows
def advdiff_coeffs(courant: float, nu: float) -> tuple[float, float, float]:
    return (-(courant + nu), 1.0 + courant + 2.0 * nu, -nu)


def obs_indices(s: int, mode: str, rng: np.random.Generator, stride: int = 2,
                p: Optional[int] = None) -> np.ndarray:
    if mode == "every":
        return np.arange(0, s, stride, dtype=np.int32)
    if mode == "random":
        return np.sort(rng.choice(s, size=p, replace=False)).astype(np.int32)
    raise ValueError(mode)


def make_advdiff_window(s: int, N: int, obs_idx: np.ndarray, *, r_kind: str = "soar",
                        r_len: float = 0.05, r_var: float = 0.5, b_len: float = 0.1,
                        b_var: float = 1.0, q_scale: float = 0.1, courant: float = 0.5,
                        nu: float = 0.1, nrhs: int = 1, seed: int = 0,
                        rhs_kind: str = "innovation", model_kind: str = "tridiag_inv",
                        kappa_r_max: float = KAPPA_R_MAX) -> Window:
    """A linear advection-diffusion window with SOAR B, Q = q B and a shared R_i."""
    ss = np.random.SeedSequence(seed)
    rng_sig, rng_obs = [np.random.default_rng(c) for c in ss.spawn(2)]
    grid = np.arange(s, dtype=np.float64) / s
    B = soar_matrix(grid, b_len, b_var)
    obs_idx = np.asarray(obs_idx, dtype=np.int32)
    p = len(obs_idx)
    if r_kind == "soar":
        R = soar_matrix(grid[obs_idx], r_len, r_var)
    elif r_kind == "gaussian":
        R = gaussian_grid_matrix(obs_idx, s, r_len, r_var)
    else:
        raise ValueError(r_kind)
    R, shift = recondition(R, kappa_r_max)
    nb = N + 1
    a, b, c = advdiff_coeffs(courant, nu)
    if model_kind == "tridiag_inv":
        model = dict(kind="tridiag_inv", a=a, b=b, c=c)
    else:
        raise ValueError(model_kind)
    win = Window(
        s=s, N=N, p=np.full(nb, p, dtype=np.int32),
        dmats=[B], d_index=np.zeros(nb, dtype=np.int32),
        d_scale=np.array([1.0] + [q_scale] * N, dtype=np.float64),
        rmats=[R], r_index=np.zeros(nb, dtype=np.int32), h_width=1,
        h_cols=[obs_idx.reshape(p, 1).copy() for _ in range(nb)],
        h_vals=[np.ones((p, 1)) for _ in range(nb)],
        model=model,
        meta=dict(r_shift=shift, seed=seed, r_len=r_len, b_len=b_len, q_scale=q_scale),
    )
    win.rhs = draw_rhs(win, nrhs, rng_sig, rng_obs, kind=rhs_kind)
    return win


def draw_rhs(win: Window, nrhs: int, rng_sig: np.random.Generator,
             rng_obs: np.random.Generator, kind: str = "innovation") -> np.ndarray:
    """Right-hand sides (b; d; 0) of the saddle system, one row per RHS.

    kind="innovation": b = 0, d_i = H_i B^{1/2} xi_i + R_i^{1/2} eps_i, with the
    smooth signal shared by all RHS and the observation noise redrawn per RHS
    (perturbed observations).  kind="random": every component of (b; d; 0)
    standard normal except the last, which is zero (used for parity tests).
    """
    s, nb = win.s, win.nb
    out = np.zeros((nrhs, win.n))
    if kind == "random":
        out[:, : nb * s + win.P] = rng_obs.standard_normal((nrhs, nb * s + win.P))
        return out
    FB = _spd_sqrt_factor(win.dmats[0])
    FR = [_spd_sqrt_factor(R) for R in win.rmats]
    sig = FB @ rng_sig.standard_normal((s, nb))          # smooth signal per block
    off = nb * s
    for i in range(nb):
        pi = int(win.p[i])
        cols, vals = win.h_cols[i], win.h_vals[i]
        hx = np.sum(vals * sig[cols, i], axis=1)
        F = FR[int(win.r_index[i])]
        noise = F @ rng_obs.standard_normal((pi, nrhs))
        out[:, off: off + pi] = hx[None, :] + noise.T
        off += pi
    return out


def soar_circulant(s: int, length: float, var: float) -> np.ndarray:
    """The SOAR matrix of the uniform periodic grid of s points (chordal distance): circulant,
    built from its first row (entry (i, j) depends on (j - i) mod s only)."""
    d = np.arange(s, dtype=np.float64) / s
    r = (np.sin(np.pi * d) / np.pi) / length
    c = var * (1.0 + r) * np.exp(-r)
    idx = (np.arange(s)[None, :] - np.arange(s)[:, None]) % s
    return c[idx]


def circulant_sqrt_apply(first_row: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """C^{1/2} xi for a symmetric circulant C given by its first row (columns of xi), through
    the FFT: C = F^* diag(lambda) F with lambda = fft(first_row) (real, clipped at 0)."""
    lam = np.clip(np.fft.fft(first_row).real, 0.0, None)
    return np.fft.ifft(np.sqrt(lam)[:, None] * np.fft.fft(xi, axis=0), axis=0).real


def make_c4_window(w: int, *, seed: int = 0, nrhs: int = 8, r_len: float = 0.05,
                   r_var: float = 0.5) -> Window:
    """Window w of the uneven batch: s ~ U{256..4096}, N ~ U{8..64}, p = floor(s f) with
    f ~ U[1/8, 1/2] random observation points (fixed in time), SOAR B (0.1, 1) on the grid,
    Q = 0.1 B, SOAR R (r_len, r_var) on the observed points, implicit advection-diffusion,
    nrhs perturbed-observation right-hand sides (observation noise redrawn from R).

    The same recipe as make_advdiff_window, except that the grid SOAR B is built as the
    circulant matrix it is and the smooth signal B^{1/2} xi is drawn through the FFT (the
    batch holds 512 windows with s up to 4096)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 4, w]))
    s = int(rng.integers(256, 4097))
    N = int(rng.integers(8, 65))
    f = float(rng.uniform(1 / 8, 1 / 2))
    p = max(1, int(np.floor(s * f)))
    idx = obs_indices(s, "random", rng, p=p)
    ss = np.random.SeedSequence([seed, 4000 + w])
    rng_sig, rng_obs = [np.random.default_rng(c) for c in ss.spawn(2)]
    B = soar_circulant(s, 0.1, 1.0)
    grid = np.arange(s, dtype=np.float64) / s
    R, shift = recondition(soar_matrix(grid[idx], r_len, r_var))
    nb = N + 1
    a, b, c = advdiff_coeffs(0.5, 0.1)
    win = Window(
        s=s, N=N, p=np.full(nb, p, dtype=np.int32), dmats=[B], d_index=np.zeros(nb, np.int32),
        d_scale=np.array([1.0] + [0.1] * N), rmats=[R], r_index=np.zeros(nb, np.int32),
        h_width=1, h_cols=[idx.reshape(p, 1).copy() for _ in range(nb)],
        h_vals=[np.ones((p, 1)) for _ in range(nb)],
        model=dict(kind="tridiag_inv", a=a, b=b, c=c),
        meta=dict(r_shift=shift, seed=seed, r_len=r_len, b_len=0.1, q_scale=0.1,
                  config="c4", index=w),
    )
    sig = circulant_sqrt_apply(B[0], rng_sig.standard_normal((s, nb)))
    FR = _spd_sqrt_factor(R)
    rhs = np.zeros((nrhs, win.n))
    off = nb * s
    for i in range(nb):
        noise = FR @ rng_obs.standard_normal((p, nrhs))
        rhs[:, off:off + p] = sig[idx, i][None, :] + noise.T
        off += p
    win.rhs = rhs
    return win


def make_c4_batch(nwin: int = 512, *, seed: int = 0, nrhs: int = 8, workers: int = 8) -> list:
    """The uneven batch of nwin windows (make_c4_window), drawn in parallel threads."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max(1, workers)) as ex:
        return list(ex.map(lambda w: make_c4_window(w, seed=seed, nrhs=nrhs), range(nwin)))


def make_config_window(name: str, *, seed: int = 0, nrhs: int = 1, r_len: Optional[float] = None,
                       rhs_kind: str = "innovation") -> Window:
    cfg = dict(CONFIGS[name])
    rng = np.random.default_rng(np.random.SeedSequence([seed, 7]))
    idx = obs_indices(cfg["s"], cfg["obs"], rng, stride=cfg.get("obs_stride", 2), p=cfg.get("p"))
    if r_len is not None:
        cfg["r_len"] = r_len
    win = make_advdiff_window(cfg["s"], cfg["N"], idx, r_kind=cfg["r_kind"], r_len=cfg["r_len"],
                              r_var=cfg["r_var"], b_len=cfg["b_len"], b_var=cfg["b_var"],
                              q_scale=cfg["q_scale"], courant=cfg["courant"], nu=cfg["nu"],
                              nrhs=nrhs, seed=seed, rhs_kind=rhs_kind)
    win.meta["config"] = name
    return win


def make_small_window(s: int = 16, N: int = 4, p: int = 6, *, seed: int = 0, nrhs: int = 1,
                      r_len: float = 0.1, b_len: float = 0.2, q_scale: float = 0.5,
                      rhs_kind: str = "random", h_width: int = 1,
                      kappa_r_max: float = KAPPA_R_MAX) -> Window:
    """Tiny windows for dense cross-checks (random obs positions, optional ELL width > 1)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 11]))
    idx = obs_indices(s, "random", rng, p=p)
    win = make_advdiff_window(s, N, idx, r_len=r_len, b_len=b_len, q_scale=q_scale, nrhs=nrhs,
                              seed=seed, rhs_kind=rhs_kind, kappa_r_max=kappa_r_max)
    if h_width > 1:
        # smoothed observations: each row averages h_width neighbouring state points
        offs = np.arange(h_width) - h_width // 2
        cols = (idx[:, None] + offs[None, :]) % s
        for i in range(win.nb):
            win.h_cols[i] = cols.astype(np.int32)
            win.h_vals[i] = np.full((p, h_width), 1.0 / h_width)
        win.h_width = h_width
        rng2 = np.random.default_rng(seed + 99)
        win.rhs = draw_rhs(win, nrhs, rng2, rng2, kind=rhs_kind)
    return win


def random_vectors(win: Window, nrhs: int, seed: int = 0) -> np.ndarray:
    """Standard normal saddle vectors, shape (nrhs, n)."""
    return np.random.default_rng(seed).standard_normal((nrhs, win.n))


def pack(windows: list, arrays: list) -> np.ndarray:
    """Concatenate per-window arrays of shape (nrhs, n_w) into one packed vector."""
    return np.concatenate([a.reshape(-1) for a in arrays])


def with_dense_model(win: Window, *, seed: int = 0, norm: float = 0.9) -> Window:
    """Replace the model by N distinct random dense maps M_1..M_N with ||M_i||_2 = norm.

    Distinct M_i make every block index visible in cross-checks (the advection-diffusion
    map is the same at every time)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 23]))
    mats = []
    for _ in range(win.N):
        G = rng.standard_normal((win.s, win.s))
        mats.append(norm * G / np.linalg.norm(G, 2))
    win.model = dict(kind="dense", mats=mats)
    return win


# ---------------------------------------------------------------- Lorenz-96 window (nonlinear)
def _l96_tendency(x: np.ndarray, F: float) -> np.ndarray:
    return (np.roll(x, -1) - np.roll(x, 2)) * np.roll(x, 1) - x + F


def _l96_run(x: np.ndarray, F: float, dt: float, nsteps: int) -> np.ndarray:
    """Nature-run integrator (classical RK4) used only to make synthetic data."""
    for _ in range(nsteps):
        a = _l96_tendency(x, F)
        b = _l96_tendency(x + 0.5 * dt * a, F)
        c = _l96_tendency(x + 0.5 * dt * b, F)
        d = _l96_tendency(x + dt * c, F)
        x = x + dt / 6.0 * (a + 2 * b + 2 * c + d)
    return x


def make_l96_window(s: int = 2048, N: int = 32, *, F: float = 8.0, dt: float = 0.025,
                    nsteps: int = 8, obs_stride: int = 4, r_len_cells: float = 4.0,
                    r_var: float = 1.0, b_len: float = 0.1, b_var: float = 1.0,
                    q_scale: float = 0.05, spinup: int = 1000, seed: int = 0,
                    nrhs: int = 1) -> Window:
    """A Lorenz-96 window (§7.1): truth from a spun-up nature run with model error Q^{1/2} eta,
    background x_b = x_0^t + B^{1/2} eps, observations y_i = H x_i^t + R^{1/2} eps_i of every
    obs_stride-th variable, first guess a free run from x_b.  model["traj"] holds the first guess
    (the linearisation states of the first outer loop); meta keeps truth, x_b and y for the outer
    Gauss-Newton loop.  The right-hand side is that of the first outer loop: b = 0, d_i = y_i - H x_i."""
    ss = np.random.SeedSequence([seed, 96])
    rng_init, rng_b, rng_q, rng_o = [np.random.default_rng(c) for c in ss.spawn(4)]
    grid = np.arange(s, dtype=np.float64) / s
    B = soar_matrix(grid, b_len, b_var)
    FB = _spd_sqrt_factor(B)
    idx = np.arange(0, s, obs_stride, dtype=np.int32)
    p = idx.size
    R = gaussian_grid_matrix(idx, s, r_len_cells, r_var)
    R, shift = recondition(R)
    FR = _spd_sqrt_factor(R)
    FQ = np.sqrt(q_scale) * FB
    x = F + 0.01 * rng_init.standard_normal(s)
    x = _l96_run(x, F, dt, spinup)
    truth = np.zeros((N + 1, s))
    truth[0] = x
    for i in range(1, N + 1):
        truth[i] = _l96_run(truth[i - 1], F, dt, nsteps) + FQ @ rng_q.standard_normal(s)
    xb = truth[0] + FB @ rng_b.standard_normal(s)
    y = np.stack([truth[i][idx] + FR @ rng_o.standard_normal(p) for i in range(N + 1)])
    guess = np.zeros((N + 1, s))
    guess[0] = xb
    for i in range(1, N + 1):
        guess[i] = _l96_run(guess[i - 1], F, dt, nsteps)
    nb = N + 1
    win = Window(
        s=s, N=N, p=np.full(nb, p, dtype=np.int32), dmats=[B], d_index=np.zeros(nb, np.int32),
        d_scale=np.array([1.0] + [q_scale] * N), rmats=[R], r_index=np.zeros(nb, np.int32),
        h_width=1, h_cols=[idx.reshape(p, 1).copy() for _ in range(nb)],
        h_vals=[np.ones((p, 1)) for _ in range(nb)],
        model=dict(kind="l96", F=F, dt=dt, nsteps=nsteps, traj=guess.copy()),
        meta=dict(truth=truth, xb=xb, y=y, obs_idx=idx, r_shift=shift, seed=seed, config="c3"),
    )
    rhs = np.zeros((nrhs, win.n))
    off = nb * s
    for i in range(nb):
        rhs[:, off + i * p: off + (i + 1) * p] = (y[i] - guess[i][idx])[None, :]
    win.rhs = rhs
    return win


# ---------------------------------------------------------------- the paper's experiments (§7)
def paper_block_R(p: int, rng: np.random.Generator, block: int = 25,
                  coupling: float = 0.4, weak: float = 0.02) -> tuple[np.ndarray, list]:
    """R_i of §6.1 for the replays: blocks of `block` observations (pvec); neighbouring blocks
    strongly coupled (pcorr = coupling) for a random half of the neighbour pairs and weakly
    (pcorr = weak) for the other half, other pairs uncorrelated (the paper does not print its
    pvec / pcorr), lambda_min = 0.41.  With Alg. 3's tol = 0.05 the weak couplings (scaled
    Frobenius norm about 0.008) are the ones R_block drops, the strong ones (about 0.16) stay."""
    nblk = max(1, p // block)
    pvec = [block] * nblk
    pvec[-1] += p - block * nblk
    pcorr = []
    for k in range(nblk):
        for l_ in range(k + 1, nblk):
            pcorr.append((coupling if rng.uniform() < 0.5 else weak) if l_ == k + 1 else 0.0)
    return block_obs_covariance(pvec, pcorr, rng), pvec


def _paper_D(s, rng):
    B = modified_soar_matrix(s, 0.6, 100, 0.4, rng)
    Q = modified_soar_matrix(s, 0.5, 120, 0.2, rng)
    return B, Q


def make_expA_window(s: int = 2500, N: int = 15, *, dt: float = 1e-4, nsteps: int = 1,
                     seed: int = 0, spinup: int = 2000) -> Window:
    """Experiment A (§7.1, Table 1): Lorenz-96 (F = 8, RK4) with s points, N = 15 subwindows,
    time step 1e-4 (one RK4 step per subwindow: the paper gives the step, not the steps per
    subwindow), observations of every second variable, D from the modified SOAR B and Q of
    eq. SOAR, block R_i (§6.1).  Truth: a spun-up nature run with model error Q^{1/2} eta;
    background x_b = x_0^t + B^{1/2} eps; first guess a free run from x_b (the single outer
    loop is linearised about it); right-hand side b_0 = x_b - x_0 (= 0), b_i = 0, d_i = y_i -
    H x_i."""
    ss = np.random.SeedSequence([seed, 71])
    rng_m, rng_i, rng_b, rng_q, rng_o, rng_r = [np.random.default_rng(c) for c in ss.spawn(6)]
    B, Q = _paper_D(s, rng_m)
    FB, FQ = _spd_sqrt_factor(B), _spd_sqrt_factor(Q)
    idx = np.arange(0, s, 2, dtype=np.int32)
    p = idx.size
    R, pvec = paper_block_R(p, rng_r)
    FR = _spd_sqrt_factor(R)
    x = 8.0 + 0.01 * rng_i.standard_normal(s)
    x = _l96_run(x, 8.0, 0.01, spinup)
    truth = np.zeros((N + 1, s))
    truth[0] = x
    for i in range(1, N + 1):
        truth[i] = _l96_run(truth[i - 1], 8.0, dt, nsteps) + FQ @ rng_q.standard_normal(s)
    xb = truth[0] + FB @ rng_b.standard_normal(s)
    y = np.stack([truth[i][idx] + FR @ rng_o.standard_normal(p) for i in range(N + 1)])
    guess = np.zeros((N + 1, s))
    guess[0] = xb
    for i in range(1, N + 1):
        guess[i] = _l96_run(guess[i - 1], 8.0, dt, nsteps)
    nb = N + 1
    win = Window(
        s=s, N=N, p=np.full(nb, p, dtype=np.int32), dmats=[B, Q],
        d_index=np.array([0] + [1] * N, dtype=np.int32), d_scale=np.ones(nb),
        rmats=[R], r_index=np.zeros(nb, np.int32), h_width=1,
        h_cols=[idx.reshape(p, 1).copy() for _ in range(nb)],
        h_vals=[np.ones((p, 1)) for _ in range(nb)],
        model=dict(kind="l96", F=8.0, dt=dt, nsteps=nsteps, traj=guess.copy()),
        meta=dict(truth=truth, xb=xb, y=y, obs_idx=idx, pvec=pvec, seed=seed, config="expA"),
    )
    rhs = np.zeros((1, win.n))
    off = nb * s
    for i in range(nb):
        rhs[0, off + i * p: off + (i + 1) * p] = y[i] - guess[i][idx]
    win.rhs = rhs
    return win


def make_expB_window(s: int = 10000, N: int = 5, *, r: float = 0.4, seed: int = 0) -> Window:
    """Experiment B (§7.2, Table 1): the heat equation u_t = u_xx on s interior points with
    homogeneous Dirichlet boundaries, forward Euler with r = dt/dx^2 = 0.4 (M: weights r,
    1 - 2r, r on offsets -1, 0, 1), N subwindows (N = 5: 750,000 = 2.5 * 50,000 * (N + 1)),
    every fourth point observed, modified-SOAR D and block R_i.  Truth: a smooth initial
    profile plus B^{1/2} noise, propagated by M with model error; first guess a free run from
    x_b; right-hand side of the first outer loop (b = 0, d = y - H x)."""
    ss = np.random.SeedSequence([seed, 72])
    rng_m, rng_b, rng_q, rng_o, rng_r, rng_t = [np.random.default_rng(c) for c in ss.spawn(6)]
    B, Q = _paper_D(s, rng_m)
    FB, FQ = _spd_sqrt_factor(B), _spd_sqrt_factor(Q)
    idx = np.arange(0, s, 4, dtype=np.int32)
    p = idx.size
    R, pvec = paper_block_R(p, rng_r)
    FR = _spd_sqrt_factor(R)
    offs, wts = [-1, 0, 1], [r, 1.0 - 2.0 * r, r]

    def step(u):
        v = (1.0 - 2.0 * r) * u
        v[1:] += r * u[:-1]
        v[:-1] += r * u[1:]
        return v
    grid = (np.arange(s) + 1.0) / (s + 1.0)
    truth = np.zeros((N + 1, s))
    truth[0] = np.sin(np.pi * grid) + FB @ rng_t.standard_normal(s)
    for i in range(1, N + 1):
        truth[i] = step(truth[i - 1]) + FQ @ rng_q.standard_normal(s)
    xb = truth[0] + FB @ rng_b.standard_normal(s)
    y = np.stack([truth[i][idx] + FR @ rng_o.standard_normal(p) for i in range(N + 1)])
    guess = np.zeros((N + 1, s))
    guess[0] = xb
    for i in range(1, N + 1):
        guess[i] = step(guess[i - 1])
    nb = N + 1
    win = Window(
        s=s, N=N, p=np.full(nb, p, dtype=np.int32), dmats=[B, Q],
        d_index=np.array([0] + [1] * N, dtype=np.int32), d_scale=np.ones(nb),
        rmats=[R], r_index=np.zeros(nb, np.int32), h_width=1,
        h_cols=[idx.reshape(p, 1).copy() for _ in range(nb)],
        h_vals=[np.ones((p, 1)) for _ in range(nb)],
        model=dict(kind="band_dirichlet", offsets=offs, weights=wts),
        meta=dict(truth=truth, xb=xb, y=y, obs_idx=idx, pvec=pvec, seed=seed, config="expB"),
    )
    rhs = np.zeros((1, win.n))
    off = nb * s
    for i in range(nb):
        rhs[0, off + i * p: off + (i + 1) * p] = y[i] - guess[i][idx]
    win.rhs = rhs
    return win


def net_init(cin: int, C: int, seed: int = 0, width: int = 5) -> np.ndarray:
    """Seeded initial parameters of the correction network, flat, float32-representable.

    Layout: W1 (C, cin, width), b1 (C), W2 (C, C, width), b2, W3 (C, C, width), b3,
    W4 (1, C, width), b4 (1).  Weights are uniform in +-sqrt(6 / fan_in) (He), the last
    layer's scaled by 0.1 so that the initial correction is small; biases are zero.
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 23]))
    parts = []
    for li, (co, ci) in enumerate([(C, cin), (C, C), (C, C), (1, C)]):
        a = np.sqrt(6.0 / (ci * width)) * (0.1 if li == 3 else 1.0)
        parts.append(rng.uniform(-a, a, size=(co, ci, width)).ravel())
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def make_c5_like(s: int, N: int, *, seed: int = 0, nrhs: int = 1) -> Window:
    """The learned-correction workload's recipe (advection-diffusion, SOAR B and R with the
    config-5 lengths, p = s/2 random observation points) at a chosen size."""
    cfg = dict(CONFIGS["c5"])
    rng = np.random.default_rng(np.random.SeedSequence([seed, 7]))
    idx = obs_indices(s, "random", rng, p=s // 2)
    win = make_advdiff_window(s, N, idx, r_kind=cfg["r_kind"], r_len=cfg["r_len"],
                              r_var=cfg["r_var"], b_len=cfg["b_len"], b_var=cfg["b_var"],
                              q_scale=cfg["q_scale"], courant=cfg["courant"], nu=cfg["nu"],
                              nrhs=nrhs, seed=seed)
    win.meta["config"] = f"c5-like s={s} N={N}"
    return win
