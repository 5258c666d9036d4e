"""FP64 CPU oracle of the learned correction of the backward L_M(k) sweep.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the entry module and
the CPU-baseline leg of the benchmark may import it; the HIP library never does, and the
two share no code.

What is learned.  Both preconditioners of §2.2/§6.2 apply Lhat^{-T} = L_M(k)^{-T}
(Definition 1) to the third input component v3: P_D inside its Schur-complement
approximation Lhat^{-1} D Lhat^{-T} v3, P_I as its first output component c1 = Lhat^{-T} v3,
which then also feeds the Schur term through D c1.  A small network corrects that sweep
output towards the exact L^{-T} v3 (the k = N+1 sweep):

    c = chat + sigma * NN(features(chat / sigma)),    sigma = rms(chat) over the system.

Why these inputs.  With P(i, j) = M_{i+1}^T ... M_j^T, the exact backward recurrence gives
c*_i = sum_{j >= i} P(i, j) v3_j and the truncated one stops at the end e(i) of block i's
segment, so c*_i - chat_i = sum_m P(i, b_m) chat_{b_m} over the later segment starts
b_m = e(i) + 1 + (m-1) k.  The correction of block i is therefore a function of the sweep
outputs at the following segment starts, and the network sees chat there (S of them),
chat at block i itself, and a one-hot code of e(i) - i.  For a time-invariant
translation-invariant model (the advection-diffusion windows) that function is a spatial
convolution per input, which a periodic 1D conv net can represent.

Network: four periodic 1D convolutions of width 5 over space (cin -> C -> C -> C -> 1),
ReLU after the first three, biases everywhere.  Loss: mean squared error over all outputs.
Optimiser: Adam (Kingma & Ba, 2015) with bias correction.

Flat parameter layout (shared with the library's ABI): W1 (C, cin, 5), b1 (C), W2 (C, C, 5),
b2 (C), W3 (C, C, 5), b3 (C), W4 (1, C, 5), b4 (1), each row-major.
"""
from __future__ import annotations

import numpy as np

WIDTH = 5
HALO = WIDTH // 2


# =================================================================== parameters
def param_shapes(cin: int, C: int):
    return [(C, cin, WIDTH), (C,), (C, C, WIDTH), (C,), (C, C, WIDTH), (C,), (1, C, WIDTH), (1,)]


def nparams(cin: int, C: int) -> int:
    return int(sum(np.prod(sh) for sh in param_shapes(cin, C)))


def unpack(theta: np.ndarray, cin: int, C: int):
    out, o = [], 0
    for sh in param_shapes(cin, C):
        n = int(np.prod(sh))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(sh))
        o += n
    assert o == theta.size
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def n_inputs(k: int, S: int) -> int:
    """Input channels: chat_i, chat at S later segment starts, one-hot of e(i) - i (k)."""
    return 1 + S + k


# =================================================================== features
def segment_end(i: int, k: int, N: int) -> int:
    """Last block of the L_M(k) segment holding block i (segments start at multiples of k)."""
    return min((i // k) * k + k - 1, N)


def features(chat_n: np.ndarray, k: int, S: int) -> np.ndarray:
    """Network input of every block of one system; chat_n is (N+1, s), already divided by sigma.

    Channel 0: chat_i.  Channels 1..S: chat at the segment starts e(i)+1, e(i)+1+k, ...
    (zero past block N).  Channels S+1..S+k: one-hot of e(i) - i.
    """
    nb, s = chat_n.shape
    N = nb - 1
    X = np.zeros((nb, n_inputs(k, S), s))
    for i in range(nb):
        e = segment_end(i, k, N)
        X[i, 0] = chat_n[i]
        for m in range(S):
            b = e + 1 + m * k
            if b <= N:
                X[i, 1 + m] = chat_n[b]
        X[i, 1 + S + (e - i)] = 1.0
    return X


# =================================================================== network
def conv_periodic(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[n, o, j] = b[o] + sum_{c, t} W[o, c, t] x[n, c, (j + t - 2) mod s]."""
    y = np.zeros((x.shape[0], W.shape[0], x.shape[2])) + b[None, :, None]
    for t in range(W.shape[2]):
        xs = np.roll(x, HALO - t, axis=2)  # xs[..., j] = x[..., (j + t - HALO) mod s]
        y += np.einsum("oc,ncj->noj", W[:, :, t], xs)
    return y


def conv_periodic_backward(x, W, gy):
    """Gradients of sum(gy * conv_periodic(x, W, b)) with respect to x, W and b."""
    gW = np.zeros_like(W)
    gx = np.zeros_like(x)
    for t in range(W.shape[2]):
        xs = np.roll(x, HALO - t, axis=2)
        gW[:, :, t] = np.einsum("noj,ncj->oc", gy, xs)
        # x[(j + t - 2)] feeds y[j]: the adjoint shifts gy the other way
        gx += np.einsum("oc,noj->ncj", W[:, :, t], np.roll(gy, t - HALO, axis=2))
    gb = gy.sum(axis=(0, 2))
    return gx, gW, gb


def forward(theta: np.ndarray, X: np.ndarray, C: int, keep: bool = False):
    """Network output (n, s) for inputs X (n, cin, s); with keep, also the activations."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta, X.shape[1], C)
    a0 = X
    z1 = conv_periodic(a0, W1, b1)
    a1 = np.maximum(z1, 0.0)
    z2 = conv_periodic(a1, W2, b2)
    a2 = np.maximum(z2, 0.0)
    z3 = conv_periodic(a2, W3, b3)
    a3 = np.maximum(z3, 0.0)
    out = conv_periodic(a3, W4, b4)[:, 0, :]
    if keep:
        return out, (a0, z1, a1, z2, a2, z3, a3)
    return out


# =================================================================== bfloat16 storage model
def round_bf16(x) -> np.ndarray:
    """Round to float32 (ties to even), then to bfloat16 (8 significant bits, ties to even);
    the storage format of the matrix-core inference.  Returns float64 values."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta: np.ndarray, X: np.ndarray, C: int) -> np.ndarray:
    """The network with bfloat16 storage: inputs, the weights of the three hidden layers and
    the hidden activations rounded to bfloat16, every sum exact (float64), biases and the
    output layer's weights as given (float32 values).  The bfloat16 inference kernels
    accumulate in float32, so they differ from this only by accumulation rounding."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta, X.shape[1], C)
    a = round_bf16(X)
    for W, b in ((W1, b1), (W2, b2), (W3, b3)):
        a = round_bf16(np.maximum(conv_periodic(a, round_bf16(W), b), 0.0))
    return conv_periodic(a, W4, b4)[:, 0, :]


def loss_and_grad(theta: np.ndarray, X: np.ndarray, Y: np.ndarray, C: int):
    """Mean squared error L = sum (out - Y)^2 / Y.size and dL/dtheta (flat layout)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta, X.shape[1], C)
    out, (a0, z1, a1, z2, a2, z3, a3) = forward(theta, X, C, keep=True)
    diff = out - Y
    loss = float(np.sum(diff * diff)) / Y.size
    g4 = (2.0 / Y.size) * diff[:, None, :]
    ga3, gW4, gb4 = conv_periodic_backward(a3, W4, g4)
    gz3 = ga3 * (z3 > 0.0)
    ga2, gW3, gb3 = conv_periodic_backward(a2, W3, gz3)
    gz2 = ga2 * (z2 > 0.0)
    ga1, gW2, gb2 = conv_periodic_backward(a1, W2, gz2)
    gz1 = ga1 * (z1 > 0.0)
    _, gW1, gb1 = conv_periodic_backward(a0, W1, gz1)
    return loss, pack([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4])


# =================================================================== Adam
def adam_step(theta, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step number t >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# =================================================================== training pairs
def make_pair(chat: np.ndarray, cexact: np.ndarray):
    """Normalised input chat / sigma and target (cexact - chat) / sigma of one system."""
    sigma = float(np.sqrt(np.mean(chat * chat)))
    if sigma == 0.0:
        return np.zeros_like(chat), np.zeros_like(chat)
    return chat / sigma, (cexact - chat) / sigma


# =================================================================== corrected preconditioners
def corrected_backward_sweep(orc, theta, v3: np.ndarray, C: int, S: int, net_fn=None):
    """Lhat^{-T} v3 plus the network's correction (v3 of shape (N+1, s)).

    net_fn(chat_n) may replace the network (used by the plumbing checks); it receives the
    normalised sweep output and returns the normalised correction.
    """
    chat = orc.LM_invT(v3)
    sigma = float(np.sqrt(np.mean(chat * chat)))
    if sigma == 0.0:
        return chat
    chat_n = chat / sigma
    if net_fn is not None:
        corr = net_fn(chat_n)
    else:
        corr = forward(theta, features(chat_n, orc.k, S), C)
    return chat + sigma * corr


def apply_PI_inv_learned(orc, theta, v, C: int, S: int, net_fn=None):
    """P_I^{-1} v with c1 = corrected Lhat^{-T} v3; z3 = Lhat^{-1}(v1 - D c1) (§6.2)."""
    v1, v2, v3 = orc.split(v)
    c1 = corrected_backward_sweep(orc, theta, v3, C, S, net_fn)
    z3 = orc.LM_inv(v1 - orc.D_apply(c1))
    return orc.join(c1, orc.Rhat_inv(v2), z3)


def apply_PD_inv_learned(orc, theta, v, C: int, S: int, net_fn=None):
    """P_D^{-1} v with the third component Lhat^{-1} D (corrected Lhat^{-T} v3) (§6.2)."""
    v1, v2, v3 = orc.split(v)
    c = corrected_backward_sweep(orc, theta, v3, C, S, net_fn)
    return orc.join(orc.Dhat_inv(v1), orc.Rhat_inv(v2), orc.LM_inv(orc.D_apply(c)))


def fgmres_with_fallback(apply_A, apply_P_learned, apply_P_plain, rhs, rtol: float,
                         maxit: int, drop: float = 1e-3, patience: int = 3):
    """Flexible GMRES whose preconditioner falls back from the learned to the plain one.

    Step j fails when its least-squares residual is not below (1 - drop) times the one after
    step j-1.  After `patience` failing steps in a row (the last being step j), every
    preconditioner application from step j+2 on is the plain one (step j+1's has already
    been made when the residual of step j is known in a pipelined implementation).  Plain
    FGMRES itself has isolated steps of almost no progress, hence the patience.  Modified
    Gram-Schmidt, Givens rotations, x0 = 0.  Returns (x, iters, hist, fallbacks).
    """
    beta = float(np.linalg.norm(rhs))
    n = rhs.size
    if beta == 0.0:
        return np.zeros(n), 0, [0.0], 0
    V = [rhs / beta]
    Z = []
    H = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    hist = [1.0]
    iters = maxit
    plain_from = None
    fallbacks = 0
    stall = 0
    prev = beta
    for j in range(maxit):
        use_plain = plain_from is not None and j >= plain_from
        z = (apply_P_plain if use_plain else apply_P_learned)(V[j])
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
        res = abs(g[j + 1])
        hist.append(res / beta)
        if plain_from is None:
            stall = 0 if res < (1.0 - drop) * prev else stall + 1
            if stall >= max(1, patience):
                plain_from = j + 2
                fallbacks += 1
        prev = res
        if res <= rtol * beta or hnext == 0.0:
            iters = j + 1
            break
        V.append(w / hnext)
    y = np.linalg.solve(np.triu(H[:iters, :iters]), g[:iters])
    x = np.zeros(n)
    for i in range(iters):
        x += y[i] * Z[i]
    return x, iters, hist, fallbacks
