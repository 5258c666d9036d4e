"""Element-wise parity by block: the largest absolute difference inside every (component,
time block) of a packed vector, relative to that block's own largest reference entry, so
that an error confined to a small-magnitude block (one nu_i, one rhs column) cannot hide
under the norm of the others.  A block whose reference entries are all below floor x the
vector's largest entry is compared against that floor instead (rounding of the large
blocks is not a relative error of a near-zero block)."""
import numpy as np


def _spans(win, space):
    s, nb = win.s, win.nb
    P = int(np.sum(win.p))
    poff = np.concatenate([[0], np.cumsum(win.p)]).astype(int)
    out = []
    if space == "saddle":
        for i in range(nb):
            out.append((f"eta{i}", i * s, (i + 1) * s))
        for i in range(nb):
            if win.p[i] > 0:
                out.append((f"nu{i}", nb * s + poff[i], nb * s + poff[i + 1]))
        for i in range(nb):
            out.append((f"x{i}", nb * s + P + i * s, nb * s + P + (i + 1) * s))
    elif space == "state":
        for i in range(nb):
            out.append((f"x{i}", i * s, (i + 1) * s))
    elif space == "obs":
        for i in range(nb):
            if win.p[i] > 0:
                out.append((f"nu{i}", poff[i], poff[i + 1]))
    else:
        raise ValueError(space)
    return out


def block_errors(win, got, ref, space="saddle", floor=1e-2):
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    assert got.shape == ref.shape
    big = float(np.max(np.abs(ref))) if ref.size else 0.0
    errs = []
    for name, a, b in _spans(win, space):
        scale = max(float(np.max(np.abs(ref[a:b]))), floor * big, 1e-300)
        errs.append((name, float(np.max(np.abs(got[a:b] - ref[a:b]))) / scale))
    return errs


def assert_blocks(win, got, ref, tol, space="saddle", floor=1e-2, what=""):
    errs = block_errors(win, got, ref, space, floor)
    name, worst = max(errs, key=lambda e: e[1])
    assert worst <= tol, f"{what} block {name}: max-abs error {worst:.3e} > {tol:.1e}"
    return worst
