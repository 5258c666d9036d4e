"""Training driver of the sweep-correction network (argument marshalling and the epoch loop;
every numerical step runs in libsvar).

Pairs: the state component v3 of every preconditioner input of plain FGMRES solves on
training windows (harvested by the solver), its truncated sweep chat = L_M(k)^{-T} v3 and its
exact sweep L^{-T} v3 (k = N+1, Definition 1), normalised by rms(chat).  Training: Adam on
random mini-batches of (pair, block) samples.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from . import svar as sv


def harvest_pairs(windows: Sequence, k: int, rtol: float = 1e-6, maxit: int = 1000,
                  cap: int = 400, rhat: str = "RR", rhs_index: int = 0, block: int = 0):
    """Plain P_I solves of the given windows (s-step FGMRES with the given block size, 0 =
    one column at a time: the inputs the preconditioner sees differ); returns float64 device
    tensors (chat, cexact) of shape (npair, N+1, s).  All windows must share N and s."""
    import torch
    chats: List = []
    cexs: List = []
    for win in windows:
        h = sv.Handle([win], sv.Precond(type="PI", k=k, rhat=rhat))
        hx = sv.Handle([win], sv.Precond(type="PI", k=win.N + 1, rhat=rhat))
        L = win.nb * win.s
        buf = torch.zeros((cap, L), dtype=torch.float64, device="cuda")
        rhs = torch.from_numpy(np.ascontiguousarray(win.rhs[rhs_index])).cuda()
        _, info, _ = h.solve(rhs, rtol=rtol, maxit=maxit, harvest=buf, block=block)
        n = min(cap, info[0]["iters"])
        V = buf[:n].contiguous()
        V = V[V.abs().amax(dim=1) > 0]  # the first input of an innovation right-hand side
        m = V.shape[0]                  # (b = 0) has v3 = 0
        if m == 0:
            continue
        chat = h.apply_op("LHAT_INVT", V.reshape(-1), m).reshape(m, win.nb, win.s)
        cex = hx.apply_op("LHAT_INVT", V.reshape(-1), m).reshape(m, win.nb, win.s)
        chats.append(chat)
        cexs.append(cex)
        h.close()
        hx.close()
    return torch.cat(chats), torch.cat(cexs)


def train(net: "sv.Net", x, y, epochs: int = 10, batch: int = 64, lr: float = 1e-3,
          seed: int = 0, log=None, ckpt=None):
    """Adam epochs over every (pair, block) sample in a shuffled order (svar_train: the loop
    runs in the library); returns the mean loss of each epoch."""
    hist = net.train(x, y, epochs=epochs, batch=batch, lr=lr, seed=seed, ckpt=ckpt)
    if log:
        for ep, v in enumerate(hist):
            log(f"epoch {ep} loss {v:.5f}")
    return list(hist)
