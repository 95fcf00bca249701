"""Seeded, MP2-shaped synthetic inputs for the CP-PPL decomposition.

Recipe (one numpy PCG64 stream per purpose, keyed by a SeedSequence of
``[seed, cfg_id, purpose, k]``):

* purpose 0 -- DF tensor.  For each auxiliary index X, an n x n matrix
  (n = o + v, occupied orbitals first) whose upper triangle including the
  diagonal is N(0, 1)/sqrt(X) and whose lower triangle mirrors it, so that
  B^X_pq = B^X_qp as for real orbitals (the DF factorisation of the Coulomb
  integrals, Section "The Density Fitting approximation", eq. SQG).
* purpose 1 -- orbital energies: occupied ~ U[-1.5, -0.3], virtual ~ U[0.2, 3.0].
  Every MP2 denominator e_i + e_j - e_a - e_b is then <= -1.0.
* First-order (MP2) doubles amplitudes t_ijab = (ia|jb) / (e_i + e_j - e_a - e_b),
  (ia|jb) = sum_X B^X_ia B^X_jb.  No singles (t_i^a = 0), so tau = t.
* purpose 2 -- starting factors, U[-1, 1] (the paper's "random guess"),
  drawn in the order alpha (v x R), beta (v x R), gamma (o x R), rho (o x R).
* purpose 3 -- planted CP factors, N(0, 1), same draw order.
* purpose 4 -- amplitude-sequence perturbation for step k.
* purpose 5 -- rank-one T2 (u_i w_j p_c q_d) for closed-form checks.

Arrays are float64, C-contiguous, and use the index orders
B[X, p, q], t[i, j, a, b], factors (rows = orbital index, columns = rank).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

PURPOSE_DF = 0
PURPOSE_ENERGIES = 1
PURPOSE_INIT = 2
PURPOSE_PLANTED = 3
PURPOSE_PERTURB = 4
PURPOSE_RANK1 = 5
PURPOSE_SINGLES = 6


@dataclass(frozen=True)
class Config:
    name: str
    cfg_id: int
    o: int
    v: int
    nx: int
    rank: int
    sweeps: int


# The five workloads: sizes (o, v, X, R) and default sweep counts.
CONFIGS = {
    "C1": Config("C1", 0, 4, 16, 48, 32, 50),
    "C2": Config("C2", 1, 16, 128, 384, 512, 30),
    "C3": Config("C3", 2, 32, 256, 768, 1024, 30),
    "C4": Config("C4", 3, 24, 192, 576, 768, 30),
    "C5": Config("C5", 4, 48, 384, 1152, 2048, 30),
}


def custom_config(o, v, nx, rank, sweeps=10, cfg_id=99, name=None):
    return Config(name or f"o{o}v{v}X{nx}R{rank}", cfg_id, o, v, nx, rank, sweeps)


def _rng(cfg_id: int, purpose: int, k: int = 0, seed: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, cfg_id, purpose, k])))


@dataclass
class Inputs:
    cfg: Config
    b_full: np.ndarray   # (X, n, n) symmetric in the last two indices
    e_occ: np.ndarray    # (o,)
    e_vir: np.ndarray    # (v,)
    b_vv: np.ndarray     # (X, v, v) = b_full[:, o:, o:]
    t: np.ndarray        # (o, o, v, v)


def make_df(cfg: Config, seed: int = 0) -> np.ndarray:
    o, v, nx = cfg.o, cfg.v, cfg.nx
    n = o + v
    rng = _rng(cfg.cfg_id, PURPOSE_DF, 0, seed)
    b = np.empty((nx, n, n))
    scale = 1.0 / np.sqrt(nx)
    iu = np.triu_indices(n)
    for x in range(nx):
        upper = rng.standard_normal(len(iu[0])) * scale
        m = np.zeros((n, n))
        m[iu] = upper
        m = m + np.triu(m, 1).T
        b[x] = m
    return b


def make_energies(cfg: Config, seed: int = 0):
    rng = _rng(cfg.cfg_id, PURPOSE_ENERGIES, 0, seed)
    e_occ = rng.uniform(-1.5, -0.3, cfg.o)
    e_vir = rng.uniform(0.2, 3.0, cfg.v)
    return e_occ, e_vir


def mp2_amplitudes(b_full: np.ndarray, e_occ: np.ndarray, e_vir: np.ndarray) -> np.ndarray:
    """t_ijab = (ia|jb) / (e_i + e_j - e_a - e_b) with (ia|jb) = sum_X B^X_ia B^X_jb."""
    o, v = len(e_occ), len(e_vir)
    nx = b_full.shape[0]
    bov = np.ascontiguousarray(b_full[:, :o, o:]).reshape(nx, o * v)
    iajb = (bov.T @ bov).reshape(o, v, o, v)
    t = np.ascontiguousarray(iajb.transpose(0, 2, 1, 3))
    denom = (e_occ[:, None, None, None] + e_occ[None, :, None, None]
             - e_vir[None, None, :, None] - e_vir[None, None, None, :])
    t /= denom
    return t


def make_inputs(cfg: Config, seed: int = 0) -> Inputs:
    b_full = make_df(cfg, seed)
    e_occ, e_vir = make_energies(cfg, seed)
    t = mp2_amplitudes(b_full, e_occ, e_vir)
    b_vv = np.ascontiguousarray(b_full[:, cfg.o:, cfg.o:])
    return Inputs(cfg, b_full, e_occ, e_vir, b_vv, t)


def make_singles(inp: "Inputs", seed: int = 0, scale: float = 0.05):
    """Synthetic singles amplitudes t1[i, a] = scale g_ia / (e_i - e_a), g ~ N(0, 1)
    (first-order-like size, |t1| ~ 1e-2), and the DF block B^X_ak (virtual a,
    occupied k) the dressed operand needs.  Returns (t1 (o x v), b_vo (X x v x o))."""
    cfg = inp.cfg
    rng = _rng(cfg.cfg_id, PURPOSE_SINGLES, 0, seed)
    g = rng.standard_normal((cfg.o, cfg.v))
    t1 = scale * g / (inp.e_occ[:, None] - inp.e_vir[None, :])
    b_vo = np.ascontiguousarray(inp.b_full[:, cfg.o:, :cfg.o])
    return t1, b_vo


def rank1_singles(cfg: Config, seed: int = 0):
    """t1 = u p^T with u (o), p (v) ~ N(0, 1): with t2 = 0, tau = u u p p is rank one."""
    rng = _rng(cfg.cfg_id, PURPOSE_SINGLES, 1, seed)
    u = rng.standard_normal(cfg.o)
    p = rng.standard_normal(cfg.v)
    return np.outer(u, p), (u, p)


def init_factors(cfg: Config, rank: int | None = None, seed: int = 0, k: int = 0):
    """U[-1, 1] factors; returned in the order (gamma, rho, alpha, beta) = (i, j, a, b)."""
    r = cfg.rank if rank is None else rank
    rng = _rng(cfg.cfg_id, PURPOSE_INIT, k, seed)
    alpha = rng.uniform(-1.0, 1.0, (cfg.v, r))
    beta = rng.uniform(-1.0, 1.0, (cfg.v, r))
    gamma = rng.uniform(-1.0, 1.0, (cfg.o, r))
    rho = rng.uniform(-1.0, 1.0, (cfg.o, r))
    return gamma, rho, alpha, beta


def planted_factors(cfg: Config, rank: int, seed: int = 0):
    """N(0, 1) factors with unit weights; returned as (gamma, rho, alpha, beta, lam)."""
    rng = _rng(cfg.cfg_id, PURPOSE_PLANTED, 0, seed)
    alpha = rng.standard_normal((cfg.v, rank))
    beta = rng.standard_normal((cfg.v, rank))
    gamma = rng.standard_normal((cfg.o, rank))
    rho = rng.standard_normal((cfg.o, rank))
    return gamma, rho, alpha, beta, np.ones(rank)


def perturbation(cfg: Config, k: int, t: np.ndarray, seed: int = 0) -> np.ndarray:
    """eps_k = 1e-2 ||t|| S(G_k)/||S(G_k)||, S(G)_ijab = (G_ijab + G_jiba)/2, G_k ~ N(0,1)."""
    rng = _rng(cfg.cfg_id, PURPOSE_PERTURB, k, seed)
    g = rng.standard_normal(t.shape)
    s = 0.5 * (g + g.transpose(1, 0, 3, 2))
    return (1e-2 * np.linalg.norm(t) / np.linalg.norm(s)) * s


def amplitude_sequence(cfg: Config, t0: np.ndarray, steps: int, seed: int = 0,
                       period: int | None = None):
    """t^(k+1) = t^(k) + 0.3^k eps_k for k = 0..steps-1 (yields t^(1)..t^(steps)).

    With ``period`` set, the decay exponent is taken as k mod period so that
    later steps see the same perturbation scales as the early ones.
    """
    t = t0.copy()
    for k in range(steps):
        e = k if period is None else (k % period)
        t = t + (0.3 ** e) * perturbation(cfg, k, t, seed)
        yield t


def rank1_t2(cfg: Config, seed: int = 0):
    """u, w (o) and p, q (v) ~ N(0, 1); T2 = u_i w_j p_c q_d."""
    rng = _rng(cfg.cfg_id, PURPOSE_RANK1, 0, seed)
    u = rng.standard_normal(cfg.o)
    w = rng.standard_normal(cfg.o)
    p = rng.standard_normal(cfg.v)
    q = rng.standard_normal(cfg.v)
    t = np.einsum("i,j,c,d->ijcd", u, w, p, q)
    return t, (u, w, p, q)


def exchange_integrals(inp: "Inputs") -> np.ndarray:
    """w[i, j, a, b] = (ia|jb) = sum_X B^X_ia B^X_jb: the driver of the synthetic
    CCD-like iteration (the numerator of the MP2 amplitudes)."""
    cfg = inp.cfg
    o, v, nx = cfg.o, cfg.v, cfg.nx
    bov = np.ascontiguousarray(inp.b_full[:, :o, o:]).reshape(nx, o * v)
    return np.ascontiguousarray((bov.T @ bov).reshape(o, v, o, v).transpose(0, 2, 1, 3))


def ccd_scale(inp: "Inputs") -> float:
    """Scale s of the ladder term in the synthetic CCD-like iteration,
    s = min|D| / (2 sum_X ||B^X_vv||_2^2).  The ladder maps t_ij to
    sum_X B^X t_ij B^X^T, whose norm is at most sum_X ||B^X||_2^2, so the exact
    Jacobi map t -> (w + s R(t)) / D contracts by at least 1/2."""
    o = inp.cfg.o
    d = (inp.e_occ[:, None, None, None] + inp.e_occ[None, :, None, None]
         - inp.e_vir[None, None, :, None] - inp.e_vir[None, None, None, :])
    spec = sum(float(np.linalg.norm(inp.b_full[x, o:, o:], 2)) ** 2 for x in range(inp.cfg.nx))
    return float(np.abs(d).min()) / (2.0 * spec)
