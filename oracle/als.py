"""Textbook CP-ALS on an explicitly formed tensor (Section "Optimizing the CP-PPL
tensor-network", eq. full_der and the definition of W), plus the fit and the
stopping metrics (eq. cpfit, eq. cp_norm2, eq. N3_stopping).

Readings taken where the paper leaves a choice (each is also followed by the GPU
library):
* sweep order alpha, beta, gamma, rho (modes a, b, i, j);
* after every factor update the new factor's columns are scaled to unit 2-norm
  and the norms become lam (the other factors carry no weight);
* the residual is sqrt(max(||R||^2 - 2<R, CP> + ||CP||^2, 0)) (the printed
  expansion has a sign slip on the last term);
* if the Cholesky factorisation of W fails (a pivot <= 0 or not finite), it is
  retried on W + delta (tr W / R) I with delta = 1e-14 * 100^k, k = 0..4, and
  the update fails after that.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .ppl import mttkrp as _mttkrp_explicit

SWEEP_ORDER = (2, 3, 0, 1)      # alpha, beta, gamma, rho


class NotSPD(RuntimeError):
    pass


def gram_hadamard(factors, mode: int) -> np.ndarray:
    """W = Hadamard product of F_k^T F_k over the three factors k != mode."""
    rank = factors[0].shape[1]
    w = np.ones((rank, rank))
    for k, f in enumerate(factors):
        if k != mode:
            w *= f.T @ f
    return w


def _cholesky_ok(w):
    try:
        c = scipy.linalg.cholesky(w, lower=True, check_finite=True)
    except (np.linalg.LinAlgError, ValueError):
        return None
    if not np.all(np.isfinite(c)) or np.any(np.diag(c) <= 0.0):
        return None
    return c


def solve_normal(m: np.ndarray, w: np.ndarray):
    """F = M W^{-1} by Cholesky, with the ridge retry.  Returns (F, retries)."""
    rank = w.shape[0]
    c = _cholesky_ok(w)
    retries = 0
    if c is None:
        shift = np.trace(w) / rank
        for k in range(5):
            retries = k + 1
            c = _cholesky_ok(w + (1e-14 * 100.0 ** k) * shift * np.eye(rank))
            if c is not None:
                break
        else:
            raise NotSPD("W is not positive definite after 5 ridge retries")
    f = scipy.linalg.cho_solve((c, True), m.T, check_finite=False).T
    return f, retries


def normalize(f: np.ndarray):
    """lam_r = ||F[:, r]||_2; columns with non-zero norm are divided by it."""
    lam = np.linalg.norm(f, axis=0)
    safe = np.where(lam > 0.0, lam, 1.0)
    return f / safe, lam


def als_update(r_tensor, factors, mode: int, mttkrp_fn=None):
    """One ALS block update of factor ``mode`` (eq. full_der solved for that factor).

    Returns (new factors list, lam, M, retries); M is the MTTKRP used.
    """
    mfn = mttkrp_fn or (lambda fs, m: _mttkrp_explicit(r_tensor, fs, m))
    m = mfn(factors, mode)
    w = gram_hadamard(factors, mode)
    f, retries = solve_normal(m, w)
    f, lam = normalize(f)
    out = list(factors)
    out[mode] = f
    return out, lam, m, retries


def sweep_scalars(norm_r2: float, m_last: np.ndarray, factors, lam):
    """(inner, cp2, fit, loss) after a sweep whose last update was rho (mode j)."""
    inner = float(np.sum(lam * np.sum(m_last * factors[1], axis=0)))
    w = np.ones((len(lam), len(lam)))
    for f in factors:
        w *= f.T @ f
    cp2 = float(lam @ w @ lam)
    res2 = norm_r2 - 2.0 * inner + cp2
    fit = 1.0 - np.sqrt(max(res2, 0.0)) / np.sqrt(norm_r2)
    return inner, cp2, fit, 0.5 * res2


def eta(prev_factors, prev_lam, factors, lam) -> float:
    """||CP_n - CP_{n-1}|| / ||CP_{n-1}|| from Gram cross terms (eq. N3_stopping)."""
    def cross(fa, la, fb, lb):
        w = np.ones((len(la), len(lb)))
        for x, y in zip(fa, fb):
            w *= x.T @ y
        return float(la @ w @ lb)
    nn = cross(factors, lam, factors, lam)
    pp = cross(prev_factors, prev_lam, prev_factors, prev_lam)
    npc = cross(factors, lam, prev_factors, prev_lam)
    return float(np.sqrt(max(nn - 2.0 * npc + pp, 0.0)) / np.sqrt(pp))


def cp_als(r_tensor, init, sweeps: int, norm_r2: float | None = None, t=None,
           tol: float = 0.0, stop_rule: int = 0, mttkrp_fn=None, on_sweep=None):
    """Textbook CP-ALS; returns (factors, lam, history dict).

    ``init`` = (gamma, rho, alpha, beta); lam starts at 1.  stop_rule 0 runs all
    sweeps, 1 stops when |fit_n - fit_{n-1}| < tol (eq. canon, with the absolute
    value), 2 stops when eta < tol (eq. N3_stopping).  ``on_sweep(factors, lam)``,
    if given, sees the iterate after every sweep (copies).
    """
    from .ppl import energy_cp
    factors = [np.array(f, dtype=np.float64, copy=True) for f in init]
    lam = np.ones(factors[0].shape[1])
    if norm_r2 is None:
        norm_r2 = float(np.sum(r_tensor * r_tensor))
    hist = {"fit": [], "loss": [], "inner": [], "cp2": [], "eta": [], "energy": [],
            "retries": 0}
    prev_fit = None
    for _ in range(sweeps):
        prev_f, prev_lam = [f.copy() for f in factors], lam.copy()
        m_last = None
        for mode in SWEEP_ORDER:
            factors, lam, m, ret = als_update(r_tensor, factors, mode, mttkrp_fn)
            hist["retries"] += ret
            m_last = m
        inner, cp2, fit, loss = sweep_scalars(norm_r2, m_last, factors, lam)
        hist["fit"].append(fit)
        hist["loss"].append(loss)
        hist["inner"].append(inner)
        hist["cp2"].append(cp2)
        hist["eta"].append(eta(prev_f, prev_lam, factors, lam))
        if t is not None:
            hist["energy"].append(energy_cp(t, factors, lam))
        if on_sweep is not None:
            on_sweep([f.copy() for f in factors], lam.copy())
        if stop_rule == 1 and prev_fit is not None and abs(fit - prev_fit) < tol:
            break
        if stop_rule == 2 and hist["eta"][-1] < tol:
            break
        prev_fit = fit
    return factors, lam, hist
