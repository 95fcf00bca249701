"""A synthetic CCD-like amplitude iteration driven by the CP-approximated
particle-particle ladder (Section "Role of the Initial Guess", with the
reconstruction and pair symmetrisation of Section "The CPD approximation of the
PPL tensor-network").

The doubles equations are cut down to the driver and the ladder term,
    D_ijab t_ijab = w_ijab + s R_ijab(t),   D_ijab = e_i + e_j - e_a - e_b,
with w_ijab = (ia|jb) and R the DF-PPL tensor of eq. dfB, and solved by the
Jacobi iteration the paper's CCSD uses (without DIIS):
    t^(k) = (w + s R~(t^(k-1))) / D,   t^(0) = w / D (the MP2 amplitudes),
where R~ is the pair-symmetrised CP approximation of R(t^(k-1)), fitted by ALS
from one of the paper's three initial guesses:
  * "random": a fresh U[-1, 1] guess every CC step;
  * "optimal": the previous step's converged factors;
  * "near_optimal": the cached factors of an earlier ALS -- if an ALS needs
    n > 5 sweeps the iterate after sweep n - 5 is cached, else the previous
    cache is kept -- and the previous converged factors while no cache exists.
The first CC step always starts from the random guess.  The scale s keeps the
exact iteration contracting (see synth's ccd_scale); the paper's CCSD has no
such factor.  The "energy" followed is E_k = sum_ijab w_ijab t^(k)_ijab.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Pinned in
tests/test_oracle_ccd.py: the exact-ladder fixed point against a direct
solve, the contraction bound, the MP2 limit s = 0, pair symmetry, and the
caching rule.
"""
from __future__ import annotations

import numpy as np

from .als import cp_als
from .ppl import cp_full, form_r, symmetrize_pairs
from .rng import random_guess


def denominators(e_occ, e_vir):
    """D_ijab = e_i + e_j - e_a - e_b."""
    return (e_occ[:, None, None, None] + e_occ[None, :, None, None]
            - e_vir[None, None, :, None] - e_vir[None, None, None, :])


def jacobi_update(w, ladder, e_occ, e_vir, scale):
    """t_new = (w + s ladder) / D."""
    return (w + scale * ladder) / denominators(e_occ, e_vir)


def exact_fixed_point(w, b_vv, e_occ, e_vir, scale):
    """The solution of D t = w + s R(t) without CP: R is linear in t and acts on
    each occupied pair separately, R_ij = g t_ij with g[(a,b),(c,d)] = (ac|bd),
    so every pair is one v^2 x v^2 linear solve (small sizes only)."""
    nx, v, _ = b_vv.shape
    o = w.shape[0]
    g = np.einsum("xac,xbd->abcd", b_vv, b_vv).reshape(v * v, v * v)
    d = denominators(e_occ, e_vir)
    t = np.empty_like(w)
    for i in range(o):
        for j in range(o):
            a = np.diag(d[i, j].reshape(-1)) - scale * g
            t[i, j] = np.linalg.solve(a, w[i, j].reshape(-1)).reshape(v, v)
    return t


def ccd_loop(w, b_vv, e_occ, e_vir, scale, steps, rank, guess="optimal", seed=0, tol=1e-3,
             max_sweeps=100, exact=False):
    """Run `steps` CC steps; returns (t, history).  history[k] holds, for CC
    step k + 1: the ALS sweeps, the fit, the guess used ("random", "optimal",
    "near_optimal"), E = <w, t>, ||t_new - t||.  exact=True takes R itself
    in place of the CP approximation (no ALS).  The random guess of CC step k
    is the SplitMix64 guess of seed + k."""
    o, _, v, _ = w.shape
    t = w / denominators(e_occ, e_vir)
    factors = cache = None
    hist = []
    for k in range(1, steps + 1):
        r = form_r(t, b_vv)
        rec = {}
        if exact:
            ladder = r
        else:
            if k == 1 or guess == "random":
                init, used = random_guess(o, v, rank, seed + k), "random"
            elif guess == "near_optimal" and cache is not None:
                init, used = cache, "near_optimal"
            else:
                init, used = factors, "optimal"
            iterates = []
            factors, lam, h = cp_als(r, init, max_sweeps, norm_r2=float(np.sum(r * r)), tol=tol,
                                     stop_rule=1, on_sweep=lambda f, l: iterates.append(f))
            n = len(h["fit"])
            if guess == "near_optimal" and n > 5:
                cache = iterates[n - 6]
            ladder = symmetrize_pairs(cp_full(factors, lam))
            rec.update({"sweeps": n, "fit": h["fit"][-1], "guess": used})
        t_new = jacobi_update(w, ladder, e_occ, e_vir, scale)
        rec.update({"energy": float(np.sum(w * t_new)),
                    "dt_norm": float(np.linalg.norm(t_new - t))})
        hist.append(rec)
        t = t_new
    return t, hist
