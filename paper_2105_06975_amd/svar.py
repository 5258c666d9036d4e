"""ctypes binding of libsvar (declared in include/svar.h).

Argument marshalling only: every step of the solve runs in the HIP library.  Device
vectors are torch float64 tensors on the current CUDA (HIP) device; the current torch
stream is passed to the library.  Importing this module fails loudly when the built
library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvar.so")

OK, E_INVAL, E_NOTSPD, E_NOCONV, E_BREAKDOWN, E_HIP, E_NOMEM = range(7)
STATUS = {0: "OK", 1: "E_INVAL", 2: "E_NOTSPD", 3: "E_NOCONV", 4: "E_BREAKDOWN", 5: "E_HIP",
          6: "E_NOMEM"}
MODEL = {"dense": 0, "band": 1, "tridiag_inv": 2, "l96": 3, "band_dirichlet": 4}
PREC = {"NONE": 0, "PD": 1, "PI": 2}
RHAT = {"DIAG": 0, "RR": 1, "ME": 2, "EXACT": 3, "BLOCK": 4}
METHOD = {"FGMRES": 0, "MINRES": 1}
PRECISION = {"FP64": 0, "MIXED_FP32": 1, "MIXED_BF16P": 2, "FP64_F32P": 3, "FP64_BF16P": 4,
             "MIXED_F32": 5}
OPS = {"L": 0, "LT": 1, "LHAT_INV": 2, "LHAT_INVT": 3, "D": 4, "DHAT_INV": 5, "R": 6,
       "RHAT_INV": 7, "H": 8, "HT": 9}
OP_SPACES = {"L": ("state", "state"), "LT": ("state", "state"), "LHAT_INV": ("state", "state"),
             "LHAT_INVT": ("state", "state"), "D": ("state", "state"),
             "DHAT_INV": ("state", "state"), "R": ("obs", "obs"), "RHAT_INV": ("obs", "obs"),
             "H": ("state", "obs"), "HT": ("obs", "state")}
KCLASS = {"GEMM": 0, "ORTHO": 1, "MODEL": 2, "NET": 3}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class ModelDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dense", C.POINTER(_dp)), ("ntaps", C.c_int32),
                ("offsets", _ip), ("weights", _dp), ("tri_a", C.c_double), ("tri_b", C.c_double),
                ("tri_c", C.c_double), ("l96_F", C.c_double), ("l96_dt", C.c_double),
                ("l96_nsteps", C.c_int32), ("l96_traj", _dp)]


class WindowDesc(C.Structure):
    _fields_ = [("s", C.c_int32), ("N", C.c_int32), ("p", _ip), ("n_dmat", C.c_int32),
                ("dmats", C.POINTER(_dp)), ("d_index", _ip), ("d_scale", _dp),
                ("n_rmat", C.c_int32), ("rmats", C.POINTER(_dp)), ("r_index", _ip),
                ("h_width", C.c_int32), ("h_cols", _ip), ("h_vals", _dp), ("model", ModelDesc)]


class PrecOpts(C.Structure):
    _fields_ = [("type", C.c_int32), ("k", C.c_int32), ("rhat", C.c_int32),
                ("rr_gamma", C.c_double), ("me_T", C.c_double), ("d_ridge", C.c_double),
                ("rb_pvec", C.POINTER(C.c_int32)), ("rb_npvec", C.c_int32),
                ("rb_maxsize", C.c_int32), ("rb_tol", C.c_double), ("rb_numproc", C.c_int32),
                ("lhat", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("method", C.c_int32), ("rtol", C.c_double), ("maxit", C.c_int32),
                ("restart", C.c_int32), ("precision", C.c_int32), ("inner_rtol", C.c_double),
                ("max_outer", C.c_int32), ("fallback_drop", C.c_double),
                ("harvest", C.c_void_p), ("harvest_cap", C.c_int32),
                ("fallback_patience", C.c_int32), ("use_graph", C.c_int32), ("block", C.c_int32),
                ("minres_norm", C.c_int32), ("history", C.c_void_p), ("history_len", C.c_int32),
                ("wave_len", C.c_int64), ("block_rhs", C.c_int32)]


class NetDesc(C.Structure):
    _fields_ = [("k", C.c_int32), ("n_bound", C.c_int32), ("precision", C.c_int32),
                ("pad", C.c_int32)]


class AdamOpts(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double)]


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("adam", AdamOpts),
                ("seed", C.c_uint64), ("checkpoint_every", C.c_int32), ("resume", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer", C.c_int32), ("status", C.c_int32),
                ("fallbacks", C.c_int32), ("relres_true", C.c_double), ("relres_est", C.c_double),
                ("n_M", C.c_int64), ("n_MT", C.c_int64), ("n_D", C.c_int64), ("n_R", C.c_int64),
                ("n_Rhat_inv", C.c_int64), ("n_Dhat_inv", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libsvar.so not built at {path}: run paper_2105_06975_amd.build")
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.svar_create.argtypes = [C.POINTER(WindowDesc), C.c_int32, C.POINTER(PrecOpts),
                                C.POINTER(vp), vp]
    lib.svar_destroy.argtypes = [vp]
    lib.svar_system_size.argtypes = [vp, C.c_int32]
    lib.svar_system_size.restype = C.c_int64
    lib.svar_offsets.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64)]
    for f in (lib.svar_apply_A, lib.svar_apply_P, lib.svar_apply_A_noalloc):
        f.argtypes = [vp, C.c_int32, vp, vp, vp]
    lib.svar_apply_op.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp]
    for f in (lib.svar_apply_A_prec, lib.svar_apply_P_prec):
        f.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp]
    lib.svar_solve.argtypes = [vp, C.POINTER(SolveOpts), C.c_int32, vp, vp, C.POINTER(SolveInfo),
                               vp]
    lib.svar_rhat_params.argtypes = [vp, C.c_int32, _dp, _dp, _dp]
    lib.svar_model_forecast.argtypes = [vp, C.c_int32, vp, vp, vp]
    lib.svar_set_trajectory.argtypes = [vp, C.c_int32, vp, vp]
    lib.svar_gn_rhs.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp]
    lib.svar_gn_update.argtypes = [vp, C.c_int32, vp, vp, vp]
    lib.svar_timing_enable.argtypes = [vp, C.c_int32, C.c_int32]
    lib.svar_timing_read.argtypes = [vp, C.c_int32, _dp, C.POINTER(C.c_int64), C.c_int32]
    lib.svar_net_create.argtypes = [C.POINTER(NetDesc), C.POINTER(vp)]
    lib.svar_net_destroy.argtypes = [vp]
    lib.svar_net_nparams.argtypes = [vp]
    lib.svar_net_nparams.restype = C.c_int64
    lib.svar_net_set_params.argtypes = [vp, C.POINTER(C.c_float)]
    lib.svar_net_get_params.argtypes = [vp, C.POINTER(C.c_float)]
    lib.svar_net_make_pairs.argtypes = [C.c_int32, C.c_int32, C.c_int32, vp, vp, vp, vp, vp]
    lib.svar_net_forward.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp]
    lib.svar_net_train_step.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp, vp, C.c_int32,
                                        _ip, C.POINTER(AdamOpts), _dp, C.POINTER(C.c_float), vp]
    lib.svar_train.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp, vp,
                               C.POINTER(TrainOpts), C.c_char_p, _dp, vp]
    lib.svar_load_learned.argtypes = [vp, C.c_char_p, C.POINTER(C.c_int64)]
    lib.svar_set_net.argtypes = [vp, vp]
    lib.svar_spectrum.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp, _dp, _ip, vp]
    lib.svar_autotune.argtypes = [vp, C.c_int32, C.c_int32, C.c_char_p, vp]
    lib.svar_autotune_load.argtypes = [vp, C.c_char_p]
    lib.svar_last_error.restype = C.c_char_p
    return lib


_LIB: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


class SvarError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise SvarError(rc, lib().svar_last_error().decode())
    return rc


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _vp(t):
    return C.c_void_p(t.data_ptr())


class _Keep:
    """Holds the numpy arrays a descriptor points to until svar_create returns."""

    def __init__(self):
        self.items = []

    def arr(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.items.append(a)
        return a

    def ptr_array(self, mats):
        arrs = [self.arr(m, np.float64) for m in mats]
        P = (_dp * len(arrs))(*[_ptr(a, C.c_double) for a in arrs])
        self.items.append(P)
        return P


def window_desc(win, keep: _Keep) -> WindowDesc:
    d = WindowDesc()
    d.s, d.N = int(win.s), int(win.N)
    d.p = _ptr(keep.arr(win.p, np.int32), C.c_int32)
    d.n_dmat = len(win.dmats)
    d.dmats = keep.ptr_array(win.dmats)
    d.d_index = _ptr(keep.arr(win.d_index, np.int32), C.c_int32)
    d.d_scale = _ptr(keep.arr(win.d_scale, np.float64), C.c_double)
    d.n_rmat = len(win.rmats)
    d.rmats = keep.ptr_array(win.rmats)
    d.r_index = _ptr(keep.arr(win.r_index, np.int32), C.c_int32)
    d.h_width = int(win.h_width)
    cols = np.concatenate([np.asarray(c, np.int32).reshape(-1) for c in win.h_cols]) \
        if len(win.h_cols) else np.zeros(0, np.int32)
    vals = np.concatenate([np.asarray(v, np.float64).reshape(-1) for v in win.h_vals]) \
        if len(win.h_vals) else np.zeros(0)
    d.h_cols = _ptr(keep.arr(cols, np.int32), C.c_int32)
    d.h_vals = _ptr(keep.arr(vals, np.float64), C.c_double)
    m = win.model
    md = ModelDesc()
    md.kind = MODEL[m["kind"]]
    if m["kind"] == "tridiag_inv":
        md.tri_a, md.tri_b, md.tri_c = float(m["a"]), float(m["b"]), float(m["c"])
    elif m["kind"] in ("band", "band_dirichlet"):
        md.ntaps = len(m["offsets"])
        md.offsets = _ptr(keep.arr(m["offsets"], np.int32), C.c_int32)
        md.weights = _ptr(keep.arr(m["weights"], np.float64), C.c_double)
    elif m["kind"] == "dense":
        md.dense = keep.ptr_array(m["mats"])
    elif m["kind"] == "l96":
        md.l96_F, md.l96_dt, md.l96_nsteps = float(m["F"]), float(m["dt"]), int(m["nsteps"])
        md.l96_traj = _ptr(keep.arr(m["traj"], np.float64), C.c_double)
    d.model = md
    return d


@dataclass
class Precond:
    type: str = "PI"
    k: int = 1
    rhat: str = "RR"
    rr_gamma: float = -1.0
    me_T: float = -1.0
    d_ridge: float = 0.01
    rb_pvec: Optional[Sequence[int]] = None   # R_block (Alg. 3): block sizes of R_i
    rb_tol: float = 0.0
    rb_maxsize: int = 0
    rb_numproc: int = 0
    lhat: str = "LM"                          # "LM": L_M(k), "LI": L_I (§2.2)


class Handle:
    """A libsvar handle over one or more windows (same preconditioner options)."""

    def __init__(self, windows: Sequence, prec: Precond = Precond(), stream=None):
        self.windows = list(windows)
        keep = _Keep()
        descs = (WindowDesc * len(self.windows))(*[window_desc(w, keep) for w in self.windows])
        pv = np.ascontiguousarray(prec.rb_pvec if prec.rb_pvec is not None else [],
                                  dtype=np.int32)
        po = PrecOpts(PREC[prec.type], int(prec.k), RHAT[prec.rhat], float(prec.rr_gamma),
                      float(prec.me_T), float(prec.d_ridge),
                      _ptr(pv, C.c_int32) if pv.size else None, int(pv.size),
                      int(prec.rb_maxsize), float(prec.rb_tol), int(prec.rb_numproc),
                      {"LM": 0, "LI": 1}[prec.lhat])
        self.prec = prec
        h = C.c_void_p()
        _check(lib().svar_create(descs, len(self.windows), C.byref(po), C.byref(h), _stream(stream)))
        self._h = h
        del keep

    def close(self):
        if getattr(self, "_h", None):
            lib().svar_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- layout
    def system_size(self, w: int = 0) -> int:
        return int(lib().svar_system_size(self._h, w))

    def offsets(self, nrhs: int = 1) -> np.ndarray:
        off = np.zeros(len(self.windows) + 1, dtype=np.int64)
        _check(lib().svar_offsets(self._h, nrhs, _ptr(off, C.c_int64)))
        return off

    def space_len(self, space: str, nrhs: int = 1) -> int:
        tot = 0
        for w in self.windows:
            n = {"saddle": w.n, "state": w.nb * w.s, "obs": w.P}[space]
            tot += nrhs * n
        return tot

    # ------------------------------------------------------------- operators
    def apply_A(self, v, nrhs: int = 1, out=None, stream=None, precision: str = "FP64"):
        import torch
        out = torch.empty_like(v) if out is None else out
        if precision == "FP64":
            _check(lib().svar_apply_A(self._h, nrhs, _vp(v), _vp(out), _stream(stream)))
        else:
            _check(lib().svar_apply_A_prec(self._h, PRECISION[precision], nrhs, _vp(v), _vp(out),
                                           _stream(stream)))
        return out

    def apply_A_noalloc(self, v, out, nrhs: int = 1, stream=None):
        """y = A v into the caller's `out` without any device allocation (the launch program
        of this nrhs must exist: an earlier apply_A with the same nrhs builds it)."""
        _check(lib().svar_apply_A_noalloc(self._h, nrhs, _vp(v), _vp(out), _stream(stream)))
        return out

    def apply_P(self, v, nrhs: int = 1, out=None, stream=None, precision: str = "FP64"):
        import torch
        out = torch.empty_like(v) if out is None else out
        if precision == "FP64":
            _check(lib().svar_apply_P(self._h, nrhs, _vp(v), _vp(out), _stream(stream)))
        else:
            _check(lib().svar_apply_P_prec(self._h, PRECISION[precision], nrhs, _vp(v), _vp(out),
                                           _stream(stream)))
        return out

    def apply_op(self, op: str, v, nrhs: int = 1, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.space_len(OP_SPACES[op][1], nrhs), dtype=torch.float64,
                              device=v.device)
        _check(lib().svar_apply_op(self._h, OPS[op], nrhs, _vp(v), _vp(out), _stream(stream)))
        return out

    def solve(self, rhs, nrhs: int = 1, *, method="FGMRES", rtol=1e-6, maxit=1000, restart=0,
              precision="FP64", inner_rtol=1e-4, max_outer=1, x=None, stream=None,
              check=False, fallback_drop=1e-3, fallback_patience=3, harvest=None,
              graph=False, block=0, minres_norm="2", history=None, wave_len=0,
              block_rhs=False):
        """Solve A x = rhs; returns (x, [info dicts], status).

        harvest: optional float64 device tensor of shape (cap, state_len): receives the state
        component of the preconditioner input of each FGMRES step.
        block: s-step FGMRES with blocks of this many columns (2..8; 0 = one at a time).
        minres_norm: MINRES stopping rule, "2" (two-norm residual) or "P" (P^{-1}-norm estimate).
        history: optional float64 device tensor (nsys, len): residual-norm estimate per iteration.
        wave_len: FGMRES over windows in contiguous waves of at most this packed length (0: from
        the free device memory).
        block_rhs: block FGMRES over the nrhs (<= 8) right-hand sides of each window (True or
        1: two Gram-Schmidt passes per step; 2: one pass).
        """
        import torch
        x = torch.empty_like(rhs) if x is None else x
        hv, cap = (None, 0) if harvest is None else (C.c_void_p(harvest.data_ptr()),
                                                     int(harvest.shape[0]))
        hp, hl = (None, 0) if history is None else (C.c_void_p(history.data_ptr()),
                                                    int(history.shape[-1]))
        o = SolveOpts(METHOD[method], float(rtol), int(maxit), int(restart), PRECISION[precision],
                      float(inner_rtol), int(max_outer), float(fallback_drop), hv, cap,
                      int(fallback_patience), 1 if graph else 0, int(block),
                      {"2": 0, "P": 1}[minres_norm], hp, hl, int(wave_len),
                      int(block_rhs))
        ninfo = len(self.windows) * nrhs
        infos = (SolveInfo * ninfo)()
        rc = lib().svar_solve(self._h, C.byref(o), nrhs, _vp(rhs), _vp(x), infos, _stream(stream))
        # E_NOCONV / E_BREAKDOWN are solver outcomes reported per system in info
        if rc not in (OK, E_NOCONV, E_BREAKDOWN) or (check and rc != OK):
            _check(rc)
        return x, [i.as_dict() for i in infos], rc

    def spectrum(self, which: str, nsteps: int, w: int = 0, start=None, seed: int = 0,
                 stream=None):
        """Lanczos Ritz values of M^{-1} K (svar_spectrum): which = "PD_A" (P_D^{-1} A),
        "RHAT_R" (Rhat^{-1} R) or "LML" (Lhat^{-T} L^T L Lhat^{-1}); start defaults to a seeded
        standard-normal vector of the operator's space.  Returns the ascending Ritz values."""
        import torch
        win = self.windows[w]
        n = {"PD_A": win.n, "RHAT_R": win.P, "LML": win.nb * win.s}[which]
        if start is None:
            start = torch.from_numpy(np.random.default_rng(seed).standard_normal(n)).cuda()
        ritz = np.zeros(int(nsteps))
        cnt = C.c_int32(0)
        _check(lib().svar_spectrum(self._h, {"PD_A": 0, "RHAT_R": 1, "LML": 2}[which], w,
                                   int(nsteps), _vp(start), _ptr(ritz, C.c_double),
                                   C.byref(cnt), _stream(stream)))
        return ritz[:cnt.value]

    def autotune(self, nrhs: int = 1, precision: str = "FP64", cache_path=None, stream=None):
        """Time the GEMM plan candidates of this handle's A and P programs (svar_autotune)."""
        _check(lib().svar_autotune(self._h, nrhs, PRECISION[precision],
                                   None if cache_path is None else str(cache_path).encode(),
                                   _stream(stream)))

    def autotune_load(self, cache_path):
        _check(lib().svar_autotune_load(self._h, str(cache_path).encode()))

    def set_net(self, net):
        """Attach a Net (or None): the preconditioner then corrects its Lhat^{-T} output."""
        _check(lib().svar_set_net(self._h, None if net is None else net._n))
        self._net = net

    def gn_rhs(self, x, xb, y, w: int = 0, out=None, stream=None):
        """(b; d; 0) of the outer loop about trajectory x (svar_gn_rhs)."""
        import torch
        win = self.windows[w]
        out = torch.empty(win.n, dtype=torch.float64, device=x.device) if out is None else out
        _check(lib().svar_gn_rhs(self._h, w, _vp(x), _vp(xb), _vp(y), _vp(out), _stream(stream)))
        return out

    def gn_update(self, x, sol, w: int = 0, stream=None):
        """x += state component of sol, and the new trajectory (svar_gn_update); in place."""
        _check(lib().svar_gn_update(self._h, w, _vp(x), _vp(sol), _stream(stream)))
        return x

    def model_forecast(self, x, w: int = 0, out=None, stream=None):
        """y_0 = x_0, y_i = M_i(x_{i-1}): one observation interval of the model of window w."""
        import torch
        out = torch.empty_like(x) if out is None else out
        _check(lib().svar_model_forecast(self._h, w, _vp(x), _vp(out), _stream(stream)))
        return out

    def set_trajectory(self, traj, w: int = 0, stream=None):
        _check(lib().svar_set_trajectory(self._h, w, _vp(traj), _stream(stream)))

    def rhat_params(self, w: int = 0):
        n = len(self.windows[w].rmats)
        g, T, l1 = np.zeros(n), np.zeros(n), np.zeros(n)
        _check(lib().svar_rhat_params(self._h, w, _ptr(g, C.c_double), _ptr(T, C.c_double),
                                      _ptr(l1, C.c_double)))
        return dict(gamma=g, T=T, lam1=l1)

    def timing_enable(self, kclass: str, on: bool = True):
        _check(lib().svar_timing_enable(self._h, KCLASS[kclass], 1 if on else 0))

    def timing_read(self, kclass: str, reset: bool = False):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().svar_timing_read(self._h, KCLASS[kclass], C.byref(ms), C.byref(n),
                                      1 if reset else 0))
        return ms.value, n.value


NET_PRECISION = {"FP32": 0, "BF16": 1}


class Net:
    """The sweep-correction network (svar_net_* of include/svar.h)."""

    def __init__(self, k: int, n_bound: int, precision: str = "BF16"):
        self.k, self.n_bound = int(k), int(n_bound)
        self.cin = 1 + self.n_bound + self.k
        d = NetDesc(self.k, self.n_bound, NET_PRECISION[precision], 0)
        h = C.c_void_p()
        _check(lib().svar_net_create(C.byref(d), C.byref(h)))
        self._n = h
        self.nparams = int(lib().svar_net_nparams(self._n))

    def close(self):
        if getattr(self, "_n", None):
            lib().svar_net_destroy(self._n)
            self._n = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.nparams
        _check(lib().svar_net_set_params(self._n, _ptr(a, C.c_float)))

    def get_params(self):
        a = np.zeros(self.nparams, dtype=np.float32)
        _check(lib().svar_net_get_params(self._n, _ptr(a, C.c_float)))
        return a

    def forward(self, x, precision: str = "FP32", out=None, stream=None):
        """x: float32 device tensor (npair, nb, s) of normalised sweep outputs."""
        import torch
        npair, nb, s = x.shape
        out = torch.empty_like(x) if out is None else out
        _check(lib().svar_net_forward(self._n, NET_PRECISION[precision], npair, nb, s, _vp(x),
                                      _vp(out), _stream(stream)))
        return out

    def train_step(self, x, y, samples, adam=None, want_loss=True, want_grad=False,
                   stream=None):
        """samples: int array (nsample, 2) of (pair, block); adam: dict(lr, beta1, beta2, eps)."""
        npair, nb, s = x.shape
        smp = np.ascontiguousarray(samples, dtype=np.int32).reshape(-1)
        ao = None
        if adam is not None:
            ao = AdamOpts(float(adam.get("lr", 1e-3)), float(adam.get("beta1", 0.9)),
                          float(adam.get("beta2", 0.999)), float(adam.get("eps", 1e-8)))
        loss = C.c_double(0.0)
        grad = np.zeros(self.nparams, dtype=np.float32) if want_grad else None
        _check(lib().svar_net_train_step(
            self._n, npair, nb, s, _vp(x), _vp(y), smp.size // 2, _ptr(smp, C.c_int32),
            None if ao is None else C.byref(ao), C.byref(loss) if want_loss else None,
            None if grad is None else _ptr(grad, C.c_float), _stream(stream)))
        return (loss.value if want_loss else None), grad


    def train(self, x, y, epochs: int = 3, batch: int = 64, lr: float = 1e-3, seed: int = 0,
              ckpt=None, checkpoint_every: int = 0, resume: bool = False, beta1=0.9,
              beta2=0.999, eps=1e-8, stream=None):
        """svar_train: the Adam epoch loop over every (pair, block) sample of the pool (x, y),
        with an optional checkpoint file; returns the mean loss of each epoch."""
        npair, nb, s = x.shape
        o = TrainOpts(int(epochs), int(batch), AdamOpts(float(lr), float(beta1), float(beta2),
                                                        float(eps)),
                      int(seed), int(checkpoint_every), 1 if resume else 0)
        hist = np.zeros(int(epochs))
        _check(lib().svar_train(self._n, npair, nb, s, _vp(x), _vp(y), C.byref(o),
                                None if ckpt is None else str(ckpt).encode(),
                                _ptr(hist, C.c_double), _stream(stream)))
        return hist

    def load(self, path):
        """svar_load_learned: parameters and Adam state from a checkpoint; returns the data
        cursor (epoch, position, Adam steps)."""
        cur = np.zeros(3, dtype=np.int64)
        _check(lib().svar_load_learned(self._n, str(path).encode(), _ptr(cur, C.c_int64)))
        return tuple(int(c) for c in cur)


def make_pairs(chat, cexact, stream=None):
    """(chat / sigma, (cexact - chat) / sigma) as float32 tensors; chat: (npair, nb, s) float64."""
    import torch
    npair, nb, s = chat.shape
    x = torch.empty(chat.shape, dtype=torch.float32, device=chat.device)
    y = torch.empty_like(x)
    _check(lib().svar_net_make_pairs(npair, nb, s, _vp(chat), _vp(cexact), _vp(x), _vp(y),
                                     _stream(stream)))
    return x, y
