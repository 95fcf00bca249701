"""Python binding of libcpppl (matrix-free CP-ALS of the CCSD PPL tensor on gfx950).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory (the workspace) and the stream.  The
library must have been built (``python -m paper_2503_10380_amd.build``); if it
is missing, ``load_library`` raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpppl.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "cpppl.h")

FP64, BF16, FP8 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "bf16": BF16, "fp8": FP8}
WS_PLAIN, WS_LEARNED, WS_FIRST_ORDER, WS_NEAR_OPTIMAL = 0, 1, 2, 3
T_CLASSES = ["kr_t2", "y", "z", "m", "g", "h", "solve", "fit", "inv"]

STATUS = {0: "ok", -1: "E_ARG", -2: "E_STATE", -3: "E_HIP", -4: "E_NOMEM", -5: "E_NOT_SPD",
          -6: "E_NONFINITE", -7: "E_UNSUPPORTED"}


class CppplError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Dims(C.Structure):
    _fields_ = [("o", C.c_int64), ("v", C.c_int64), ("nx", C.c_int64), ("rank", C.c_int64),
                ("singles", C.c_int64)]


class AlsOpts(C.Structure):
    _fields_ = [("max_sweeps", C.c_int), ("stop_rule", C.c_int), ("tol", C.c_double),
                ("refine_fp64_sweeps", C.c_int), ("history_cap", C.c_int), ("energy", C.c_int),
                ("timing", C.c_int), ("refine_tol", C.c_double), ("stop_window", C.c_int),
                ("eta", C.c_int), ("near_cache", C.c_int), ("energy_every", C.c_int),
                ("refine_etol", C.c_double)]


class AlsReport(C.Structure):
    _fields_ = [("sweeps_done", C.c_int), ("ridge_retries", C.c_int), ("fit", C.c_double),
                ("loss", C.c_double), ("inner", C.c_double), ("cp_norm2", C.c_double),
                ("eta", C.c_double), ("energy_cp", C.c_double), ("ms_total", C.c_double),
                ("ms_class", C.c_double * 16), ("n_class", C.c_int * 16),
                ("fit_hist", C.POINTER(C.c_double)), ("eta_hist", C.POINTER(C.c_double)),
                ("ms_hist", C.POINTER(C.c_double)), ("refine_done", C.c_int),
                ("energy_hist", C.POINTER(C.c_double)), ("careful_sweeps", C.c_int)]


_lib = None
_P = C.c_void_p
_D = C.POINTER(C.c_double)


def header_symbols():
    """Every function the C header declares."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"CPPPL_API\s+[\w\s\*]+?\b(cpppl_\w+)\s*\(", text)))


def load_library(path: str = LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2503_10380_amd.build`")
    from .build import source_hash
    # One HIP runtime per process: torch ships its own libamdhip64 (same soname
    # as ROCm's).  Importing torch first makes the library bind to that copy, so
    # that torch's streams and device memory are valid handles inside it.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    st = C.c_int
    sig = {
        "cpppl_create": (st, [C.POINTER(Dims), C.c_int, C.c_int, _P, C.POINTER(_P)]),
        "cpppl_workspace_size": (st, [C.POINTER(Dims), C.c_int, C.POINTER(C.c_size_t)]),
        "cpppl_bind_workspace": (st, [_P, _P, C.c_size_t]),
        "cpppl_destroy": (st, [_P]),
        "cpppl_load_t2": (st, [_P, _P, C.c_int]),
        "cpppl_load_df": (st, [_P, _P, C.c_int]),
        "cpppl_load_singles": (st, [_P, _P, _P, C.c_int]),
        "cpppl_load_planted": (st, [_P, _P, _P, _P, _P, _P, C.c_int64, C.c_int]),
        "cpppl_norm_r2": (st, [_P, _D, _D]),
        "cpppl_set_factors": (st, [_P, _P, _P, _P, _P, _P, C.c_int]),
        "cpppl_get_factors": (st, [_P, _P, _P, _P, _P, _P, C.c_int]),
        "cpppl_init_random": (st, [_P, C.c_uint64]),
        "cpppl_als": (st, [_P, C.POINTER(AlsOpts), C.POINTER(AlsReport)]),
        "cpppl_mttkrp": (st, [_P, C.c_int, C.c_int, _P, C.c_int]),
        "cpppl_fit": (st, [_P, _D, _D, _D]),
        "cpppl_energy": (st, [_P, _D]),
        "cpppl_jacobi_step": (st, [_P, _P, _P, _P, C.c_double, _P, C.c_int]),
        "cpppl_reconstruct": (st, [_P, _P, C.c_int, C.c_int]),
        "cpppl_mlp_create": (st, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, C.c_uint64, C.c_int,
                                  C.POINTER(_P)]),
        "cpppl_mlp_destroy": (st, [_P]),
        "cpppl_mlp_num_params": (st, [_P, C.POINTER(C.c_int64)]),
        "cpppl_mlp_get_params": (st, [_P, _P, C.c_int]),
        "cpppl_mlp_set_params": (st, [_P, _P, C.c_int]),
        "cpppl_mlp_forward": (st, [_P, _P, C.c_int64, _P, C.c_int]),
        "cpppl_mlp_grad": (st, [_P, _P, _P, C.c_int64, _P, _P, C.c_int]),
        "cpppl_mlp_add_rows": (st, [_P, _P, _P, C.c_int64, C.c_int]),
        "cpppl_mlp_clear_rows": (st, [_P]),
        "cpppl_mlp_num_rows": (st, [_P, C.POINTER(C.c_int64)]),
        "cpppl_mlp_get_rows": (st, [_P, _P, _P, C.c_int]),
        "cpppl_mlp_train": (st, [_P, C.c_int, C.c_float, C.c_int64, C.c_uint64, _P]),
        "cpppl_mlp_standardize": (st, [_P]),
        "cpppl_mlp_get_standardization": (st, [_P, _P, _P, _P]),
        "cpppl_mlp_save": (st, [_P, C.c_char_p]),
        "cpppl_mlp_load": (st, [_P, C.c_char_p]),
        "cpppl_ws_in_dim": (C.c_int64, [C.POINTER(Dims)]),
        "cpppl_ws_out_dim": (C.c_int64, [C.POINTER(Dims)]),
        "cpppl_warm_start": (st, [_P, _P, C.c_int, C.c_int, _P, C.POINTER(C.c_int)]),
        "cpppl_ws_training_rows": (st, [_P, _P]),
        "cpppl_last_error": (C.c_char_p, [_P]),
        "cpppl_status_str": (C.c_char_p, [C.c_int]),
        "cpppl_build_hash": (C.c_char_p, []),
        "cpppl_mttkrp_noalloc": (st, [C.POINTER(Dims), _P, _P, _P, _P, _P, _P, C.c_int, _P, _P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    built = lib.cpppl_build_hash().decode()
    want = source_hash()
    if built != want:
        raise RuntimeError(f"{path} was built from other sources (hash {built[:16]}, sources "
                           f"{want[:16]}); rebuild with `python -m paper_2503_10380_amd.build`")
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


def _f64_host(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr_host(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Context:
    """A CP-PPL problem on one GPU: inputs, factors, ALS sweeps.

    Arrays may be numpy (host) or torch CUDA tensors (device, float64,
    contiguous); results come back as numpy arrays.
    """

    def __init__(self, o, v, nx, rank, precision="fp64", device=0, stream=None, singles=False):
        torch = _torch()
        self.lib = load_library()
        self.dims = Dims(o, v, nx, rank, 1 if singles else 0)
        self.o, self.v, self.nx, self.rank = o, v, nx, rank
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.device = device
        if stream is None:
            with torch.cuda.device(device):
                stream = torch.cuda.current_stream(device)
        self.stream = stream
        nbytes = C.c_size_t()
        self._check(self.lib.cpppl_workspace_size(C.byref(self.dims), self.precision, C.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=f"cuda:{device}")
        h = _P()
        self._check(self.lib.cpppl_create(C.byref(self.dims), self.precision, device,
                                          _P(stream.cuda_stream), C.byref(h)))
        self.h = h
        self._call("cpppl_bind_workspace", _P(self._ws.data_ptr()), C.c_size_t(self.workspace_bytes))

    # ------------------------------------------------------------------ plumbing
    def _check(self, status, h=None):
        if status != 0:
            msg = ""
            if h is not None:
                m = self.lib.cpppl_last_error(h)
                msg = m.decode() if m else ""
            raise CppplError(status, msg)

    def _call(self, name, *args):
        st = getattr(self.lib, name)(self.h, *args)
        self._check(st, self.h)

    def _arg(self, x, shape, keep):
        """(pointer, on_device) for a host or device float64 array of `shape`."""
        if x is None:
            return None, 0
        if hasattr(x, "is_cuda") and x.is_cuda:
            torch = _torch()
            if x.dtype != torch.float64 or not x.is_contiguous() or tuple(x.shape) != tuple(shape):
                raise ValueError(f"device array must be contiguous float64 of shape {shape}")
            keep.append(x)
            return _P(x.data_ptr()), 1
        a = _f64_host(x)
        if a.shape != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {a.shape}")
        keep.append(a)
        return _ptr_host(a), 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.cpppl_destroy(self.h)
            self.h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ inputs
    def load_t2(self, t):
        keep = []
        p, dev = self._arg(t, (self.o, self.o, self.v, self.v), keep)
        self._call("cpppl_load_t2", p, dev)

    def load_df(self, b):
        keep = []
        p, dev = self._arg(b, (self.nx, self.v, self.v), keep)
        self._call("cpppl_load_df", p, dev)

    def load_singles(self, t1, b_vo):
        """Dress the PPL tensor with singles t1 (o x v) and the DF block
        b_vo (X x v x o); t1=None removes the dressing."""
        keep = []
        if t1 is None:
            self._call("cpppl_load_singles", None, None, 0)
            return
        p1, d1 = self._arg(t1, (self.o, self.v), keep)
        p2, d2 = self._arg(b_vo, (self.nx, self.v, self.o), keep)
        if d1 != d2:
            raise ValueError("t1 and b_vo must both be on the host or both on the device")
        self._call("cpppl_load_singles", p1, p2, d1)

    def load_planted(self, fi, fj, fa, fb, lam=None):
        rp = np.shape(fi)[1]
        keep = []
        ps = [self._arg(x, (n, rp), keep) for x, n in zip((fi, fj, fa, fb),
                                                        (self.o, self.o, self.v, self.v))]
        pl, dl = self._arg(lam, (rp,), keep)
        dev = ps[0][1]
        self._call("cpppl_load_planted", *[q[0] for q in ps], pl, C.c_int64(rp), dev)

    def norm_r2(self):
        n2, e = C.c_double(), C.c_double()
        self._call("cpppl_norm_r2", C.byref(n2), C.byref(e))
        return n2.value, e.value

    # ------------------------------------------------------------------ factors
    def init_random(self, seed):
        """Factors uniform in [-1, 1) from the library's counter-based generator, lambda = 1."""
        self._call("cpppl_init_random", C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF))

    def set_factors(self, fi, fj, fa, fb, lam=None):
        keep = []
        shapes = [(self.o, self.rank), (self.o, self.rank), (self.v, self.rank), (self.v, self.rank)]
        ps = [self._arg(x, s, keep) for x, s in zip((fi, fj, fa, fb), shapes)]
        devs = {q[1] for q in ps}
        if len(devs) != 1:
            raise ValueError("factors must all be on the host or all on the device")
        pl, dl = self._arg(lam, (self.rank,), keep)
        if lam is not None and dl != ps[0][1]:
            raise ValueError("lam must live where the factors live")
        self._call("cpppl_set_factors", *[q[0] for q in ps], pl, ps[0][1])

    def get_factors(self):
        out = [np.empty((n, self.rank)) for n in (self.o, self.o, self.v, self.v)]
        lam = np.empty(self.rank)
        self._call("cpppl_get_factors", *[_ptr_host(a) for a in out], _ptr_host(lam), 0)
        return (*out, lam)

    # ------------------------------------------------------------------ work
    def als(self, sweeps, stop_rule=0, tol=0.0, refine=0, energy=False, timing=False,
            refine_tol=0.0, stop_window=1, eta=False, near_cache=False, energy_every=False,
            refine_etol=0.0):
        cap = sweeps + refine
        opts = AlsOpts(sweeps, stop_rule, tol, refine, cap, int(bool(energy)), int(bool(timing)),
                       refine_tol, stop_window, int(bool(eta)), int(bool(near_cache)),
                       int(bool(energy_every)), refine_etol)
        fit = np.full(cap, np.nan)
        eta_h = np.full(cap, np.nan)
        ms = np.full(cap, np.nan)
        en = np.full(cap, np.nan)
        rep = AlsReport()
        rep.fit_hist = fit.ctypes.data_as(_D)
        rep.eta_hist = eta_h.ctypes.data_as(_D)
        rep.ms_hist = ms.ctypes.data_as(_D)
        rep.energy_hist = en.ctypes.data_as(_D)
        self._call("cpppl_als", C.byref(opts), C.byref(rep))
        n = rep.sweeps_done
        return {
            "sweeps": n, "refine_sweeps": rep.refine_done, "ridge_retries": rep.ridge_retries,
            "careful_sweeps": rep.careful_sweeps,
            "fit": rep.fit, "loss": rep.loss,
            "inner": rep.inner, "cp_norm2": rep.cp_norm2, "eta": rep.eta,
            "energy_cp": rep.energy_cp, "ms_total": rep.ms_total,
            "ms_class": {k: rep.ms_class[i] for i, k in enumerate(T_CLASSES)},
            "n_class": {k: rep.n_class[i] for i, k in enumerate(T_CLASSES)},
            "fit_hist": fit[:n].copy(), "eta_hist": eta_h[:n].copy(), "ms_hist": ms[:n].copy(),
            "energy_hist": en[:n].copy(),
        }

    def inject_alpha_fault(self, sweep):
        """Test hook (cpppl_testing.h): the next als() call sees a failed pivot
        in the W_alpha inverse forked early for sweep `sweep`."""
        fn = self.lib.cpppl_test_inject_alpha_fault
        fn.restype, fn.argtypes = C.c_int, [_P, C.c_int]
        self._check(fn(self.h, int(sweep)), self.h)

    def mttkrp(self, mode, precision=None):
        prec = self.precision if precision is None else PRECISIONS.get(precision, precision)
        n = (self.o, self.o, self.v, self.v)[mode]
        out = np.empty((n, self.rank))
        self._call("cpppl_mttkrp", mode, prec, _ptr_host(out), 0)
        return out

    def fit(self):
        f, i, c = C.c_double(), C.c_double(), C.c_double()
        self._call("cpppl_fit", C.byref(f), C.byref(i), C.byref(c))
        return f.value, i.value, c.value

    def reconstruct(self, symmetrize=False, out=None):
        """The CP tensor (o, o, v, v) in FP64, optionally pair-symmetrised; into
        `out` (a device float64 tensor) when given, else returned as numpy."""
        if out is not None:
            keep = []
            p, dev = self._arg(out, (self.o, self.o, self.v, self.v), keep)
            self._call("cpppl_reconstruct", p, int(bool(symmetrize)), dev)
            return out
        res = np.empty((self.o, self.o, self.v, self.v))
        self._call("cpppl_reconstruct", _ptr_host(res), int(bool(symmetrize)), 0)
        return res

    def jacobi_step(self, w, e_occ, e_vir, scale, out=None):
        """dt of one CCD-like Jacobi step with the pair-symmetrised CP ladder:
        (w + scale R~) / D - t.  Device inputs (torch) give a device dt
        (into `out` when given); host inputs a numpy dt."""
        keep = []
        shape = (self.o, self.o, self.v, self.v)
        pw, dw = self._arg(w, shape, keep)
        po, do = self._arg(e_occ, (self.o,), keep)
        pv, dv = self._arg(e_vir, (self.v,), keep)
        if len({dw, do, dv}) != 1:
            raise ValueError("w, e_occ and e_vir must all be on the host or all on the device")
        if dw:
            torch = _torch()
            if out is None:
                out = torch.empty(shape, dtype=torch.float64, device=w.device)
            po_, _ = self._arg(out, shape, keep)
            self._call("cpppl_jacobi_step", pw, po, pv, C.c_double(scale), po_, 1)
            return out
        res = np.empty(shape)
        self._call("cpppl_jacobi_step", pw, po, pv, C.c_double(scale), _ptr_host(res), 0)
        return res

    def energy(self):
        e = C.c_double()
        self._call("cpppl_energy", C.byref(e))
        return e.value

    # ------------------------------------------------------------------ warm starts
    @property
    def ws_in_dim(self):
        return self.lib.cpppl_ws_in_dim(C.byref(self.dims))

    @property
    def ws_out_dim(self):
        return self.lib.cpppl_ws_out_dim(C.byref(self.dims))

    def warm_start(self, dt, strategy=WS_PLAIN, mlp=None):
        """t <- t + dt and warm-start the factors; returns the strategy chosen."""
        keep = []
        p, dev = self._arg(dt, (self.o, self.o, self.v, self.v), keep)
        chosen = C.c_int(-1)
        self._call("cpppl_warm_start", p, dev, int(strategy), mlp.h if mlp is not None else None,
                   C.byref(chosen))
        return chosen.value

    def training_rows(self, mlp):
        self._call("cpppl_ws_training_rows", mlp.h)


def mttkrp_noalloc(t, b, fi, fj, fa, fb, mode, out=None, stream=None):
    """cpppl_mttkrp_noalloc on torch CUDA float64 tensors (contiguous):
    t (o, o, v, v), b (X, v, v), fi, fj (o, R), fa, fb (v, R); returns (or
    fills) the (n_mode, R) device tensor.  Enqueued on `stream` (default: the
    current stream); nothing is allocated by the library."""
    torch = _torch()
    lib = load_library()
    o, v, nx, rank = t.shape[0], t.shape[2], b.shape[0], fi.shape[1]
    for x in (t, b, fi, fj, fa, fb):
        if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
            raise ValueError("device float64 contiguous tensors expected")
    n = (o, o, v, v)[mode]
    if out is None:
        out = torch.empty((n, rank), dtype=torch.float64, device=t.device)
    if stream is None:
        stream = torch.cuda.current_stream(t.device)
    d = Dims(o, v, nx, rank, 0)
    st = lib.cpppl_mttkrp_noalloc(C.byref(d), *[_P(x.data_ptr()) for x in (t, b, fi, fj, fa, fb)],
                                  int(mode), _P(out.data_ptr()), _P(stream.cuda_stream))
    if st != 0:
        raise CppplError(st, "cpppl_mttkrp_noalloc failed")
    return out


GUESSES = ("random", "optimal", "near_optimal")


def ccd_loop(ctx, w, e_occ, e_vir, scale, steps, guess="optimal", seed=0, tol=1e-3,
             max_sweeps=100, on_step=None):
    """A CCD-like Jacobi iteration with the CP-approximated ladder, as a
    sequence of library calls: per CC step k = 1..steps, ALS (|dfit| < tol, at
    most max_sweeps) on the context's current t, then cpppl_jacobi_step for
    dt, then cpppl_warm_start(dt) with the next step's initial guess --
    "random" (a fresh cpppl_init_random(seed + k + 1) guess), "optimal" (the
    converged factors) or "near_optimal" (the near-optimal cache, kept by the
    ALS calls).  CC step 1 starts from cpppl_init_random(seed + 1).  w, e_occ,
    e_vir: torch CUDA float64 tensors (the driver (ia|jb) and the orbital
    energies); the context must hold t^(0) and B.  Returns one record per CC
    step (sweeps, fit, the guess it started from); on_step(k, dt, record) sees
    each step's dt (device tensor) before it is applied."""
    if guess not in GUESSES:
        raise ValueError(f"guess must be one of {GUESSES}")
    hist = []
    used = "random"
    ctx.init_random(seed + 1)
    for k in range(1, steps + 1):
        rep = ctx.als(max_sweeps, stop_rule=1, tol=tol, near_cache=guess == "near_optimal")
        dt = ctx.jacobi_step(w, e_occ, e_vir, scale)
        rec = {"sweeps": rep["sweeps"], "fit": rep["fit"], "guess": used,
               "ms_als": rep["ms_total"]}
        if on_step is not None:
            on_step(k, dt, rec)
        hist.append(rec)
        if guess == "random":
            ctx.warm_start(dt, WS_PLAIN)
            ctx.init_random(seed + k + 1)
            used = "random"
        elif guess == "near_optimal":
            chosen = ctx.warm_start(dt, WS_NEAR_OPTIMAL)
            used = "near_optimal" if chosen == WS_NEAR_OPTIMAL else "optimal"
        else:
            ctx.warm_start(dt, WS_PLAIN)
            used = "optimal"
    return hist


class MLP:
    """The per-rank-column warm-start network (FP32, trained on the GPU)."""

    def __init__(self, in_dim, out_dim, hidden=256, n_hidden=2, capacity=0, seed=0, device=0):
        _torch()
        self.lib = load_library()
        self.in_dim, self.out_dim = in_dim, out_dim
        h = _P()
        st = self.lib.cpppl_mlp_create(in_dim, hidden, n_hidden, out_dim, capacity, seed, device,
                                       C.byref(h))
        if st != 0:
            raise CppplError(st, "cpppl_mlp_create failed")
        self.h = h
        n = C.c_int64()
        self.lib.cpppl_mlp_num_params(self.h, C.byref(n))
        self.nparams = n.value

    def _check(self, st):
        if st != 0:
            raise CppplError(st, "")

    def close(self):
        if getattr(self, "h", None):
            self.lib.cpppl_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.empty(self.nparams, dtype=np.float32)
        self._check(self.lib.cpppl_mlp_get_params(self.h, out.ctypes.data_as(_P), 0))
        return out

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.nparams
        self._check(self.lib.cpppl_mlp_set_params(self.h, a.ctypes.data_as(_P), 0))

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.empty((x.shape[0], self.out_dim), dtype=np.float32)
        self._check(self.lib.cpppl_mlp_forward(self.h, x.ctypes.data_as(_P), x.shape[0],
                                               y.ctypes.data_as(_P), 0))
        return y

    def grad(self, x, y):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        loss = C.c_float()
        g = np.empty(self.nparams, dtype=np.float32)
        self._check(self.lib.cpppl_mlp_grad(self.h, x.ctypes.data_as(_P), y.ctypes.data_as(_P),
                                            x.shape[0], C.byref(loss), g.ctypes.data_as(_P), 0))
        return loss.value, g

    def add_rows(self, x, y):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        self._check(self.lib.cpppl_mlp_add_rows(self.h, x.ctypes.data_as(_P), y.ctypes.data_as(_P),
                                                x.shape[0], 0))

    def clear_rows(self):
        self._check(self.lib.cpppl_mlp_clear_rows(self.h))

    @property
    def num_rows(self):
        n = C.c_int64()
        self._check(self.lib.cpppl_mlp_num_rows(self.h, C.byref(n)))
        return n.value

    def get_rows(self):
        n = self.num_rows
        x = np.empty((n, self.in_dim), dtype=np.float32)
        y = np.empty((n, self.out_dim), dtype=np.float32)
        self._check(self.lib.cpppl_mlp_get_rows(self.h, x.ctypes.data_as(_P), y.ctypes.data_as(_P), 0))
        return x, y

    def train(self, epochs, lr=1e-3, batch=0, seed=0):
        hist = np.zeros(epochs, dtype=np.float32)
        self._check(self.lib.cpppl_mlp_train(self.h, epochs, C.c_float(lr), batch, seed,
                                             hist.ctypes.data_as(_P)))
        return hist

    def standardize(self):
        """Standardise the stored rows (per-column centring / scaling) and keep
        the map for the learned warm start."""
        self._check(self.lib.cpppl_mlp_standardize(self.h))

    def standardization(self):
        """(x_mu, x_inv, y_sc) of a standardised network."""
        mu = np.empty(self.in_dim, dtype=np.float32)
        inv = np.empty(self.in_dim, dtype=np.float32)
        sc = np.empty(self.out_dim, dtype=np.float32)
        self._check(self.lib.cpppl_mlp_get_standardization(
            self.h, mu.ctypes.data_as(_P), inv.ctypes.data_as(_P), sc.ctypes.data_as(_P)))
        return mu, inv, sc

    def save(self, path):
        self._check(self.lib.cpppl_mlp_save(self.h, str(path).encode()))

    def load(self, path):
        self._check(self.lib.cpppl_mlp_load(self.h, str(path).encode()))
