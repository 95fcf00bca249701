"""Explicit (matrix-full) definitions of the PPL tensor and of its MTTKRPs.

Index conventions: the PPL tensor is R[i, j, a, b] (o, o, v, v); the DF tensor
is B[X, p, q]; T2 is t[i, j, c, d]; the CP factors are gamma (o x R, index i),
rho (o x R, index j), alpha (v x R, index a), beta (v x R, index b) with weights
lam (R).  Mode numbers follow the tensor axes: 0 = i, 1 = j, 2 = a, 3 = b.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np


def recompute_t(b_full: np.ndarray, e_occ: np.ndarray, e_vir: np.ndarray) -> np.ndarray:
    """First-order doubles amplitudes from the DF tensor and orbital energies.

    t_ijab = (ia|jb) / (e_i + e_j - e_a - e_b) with (ia|jb) = sum_X B^X_ia B^X_jb
    (the DF form of the integrals, eq. SQG).  Written with einsum so that it is
    an independent route from the input generator's GEMM.
    """
    o = len(e_occ)
    bov = b_full[:, :o, o:]
    iajb = np.einsum("xia,xjb->ijab", bov, bov, optimize=True)
    d = e_occ[:, None, None, None] + e_occ[None, :, None, None] \
        - e_vir[None, None, :, None] - e_vir[None, None, None, :]
    return iajb / d


def df_integrals(b_vv: np.ndarray, a0: int = 0, a1: int | None = None,
                 b_right: np.ndarray | None = None) -> np.ndarray:
    """g[a, b, c, d] = (ac|bd) = sum_X B^X_ac B^X_bd for a in [a0, a1)  (eq. SQG).

    With ``b_right`` (the singles-dressed Dbar of eq. dfB) the second factor
    is b_right^X_bd: g = sum_X B^X_ac Dbar^X_bd."""
    nx, v, _ = b_vv.shape
    a1 = v if a1 is None else a1
    left = b_vv[:, a0:a1, :].reshape(nx, (a1 - a0) * v)      # X x (a, c)
    right = (b_vv if b_right is None else b_right).reshape(nx, v * v)   # X x (b, d)
    g = (left.T @ right).reshape(a1 - a0, v, v, v)            # a, c, b, d
    return g.transpose(0, 2, 1, 3)                            # a, b, c, d


def form_r(t: np.ndarray, b_vv: np.ndarray, block: int | None = None,
           ij_rows: slice | None = None, b_right: np.ndarray | None = None) -> np.ndarray:
    """The DF particle-particle-ladder tensor (eq. dfB).

    R_ijab = sum_cd (sum_X B^X_ac Dbar^X_bd) t_ijcd, computed as
    R_mat (o^2 x v^2) = T_mat (o^2 x v^2) . g_mat^T, with g formed in blocks of a.
    Without singles Dbar = B and t is the doubles amplitude; with singles pass
    tau as ``t`` and Dbar as ``b_right`` (see ``dress``).
    ``ij_rows`` restricts the computation to a slice of the (i, j) pair rows.
    """
    o, _, v, _ = t.shape
    tm = t.reshape(o * o, v * v)
    if ij_rows is not None:
        tm = tm[ij_rows]
    if block is None:
        block = max(1, min(v, (1 << 26) // (v * v * v)))
    out = np.empty((tm.shape[0], v, v))
    for a0 in range(0, v, block):
        a1 = min(v, a0 + block)
        g = df_integrals(b_vv, a0, a1, b_right).reshape((a1 - a0) * v, v * v)
        out[:, a0:a1, :] = (tm @ g.T).reshape(tm.shape[0], a1 - a0, v)
    if ij_rows is None:
        return out.reshape(o, o, v, v)
    return out


def form_r_pairs(t: np.ndarray, b_vv: np.ndarray, occ: int) -> np.ndarray:
    """R restricted to i, j < occ, one occupied pair at a time from eq. dfB
    (no (ac|bd) tensor): U^X = B^X T_ij with T_ij[c, d] = t_ijcd, then
    R_ij[a, b] = sum_{X, d} U^X[a, d] B^X[b, d].  Returns (occ, occ, v, v)."""
    nx, v, _ = b_vv.shape
    bstack = b_vv.reshape(nx * v, v)                        # rows (X, a), cols c
    bperm = b_vv.transpose(1, 0, 2).reshape(v, nx * v)      # rows b, cols (X, d)
    out = np.empty((occ, occ, v, v))
    for i in range(occ):
        for j in range(occ):
            u = (bstack @ t[i, j]).reshape(nx, v, v)          # U[X, a, d]
            ut = u.transpose(1, 0, 2).reshape(v, nx * v)      # rows a, cols (X, d)
            out[i, j] = ut @ bperm.T
    return out


def form_r_einsum(t: np.ndarray, b_vv: np.ndarray, b_right: np.ndarray | None = None) -> np.ndarray:
    """Second route to R (tiny sizes only): one einsum over X, c, d."""
    br = b_vv if b_right is None else b_right
    return np.einsum("xac,xbd,ijcd->ijab", b_vv, br, t, optimize=True)


def dress(t2: np.ndarray, t1: np.ndarray, b_full: np.ndarray):
    """Singles-dressed inputs of the PPL tensor (eq. B, eq. fulldfB and the Dbar
    definition before eq. dfB), restricted closed shell:
    tau_ijcd = t_ijcd + t^c_i t^d_j and Dbar^X_bd = D^X_bd - 2 sum_k D^X_bk t^k_d,
    with t1[i, c] = t^c_i (o x v) and b_full the DF tensor over all n = o + v
    orbitals (occupied first).  Returns (tau, B_vv, Dbar_vv)."""
    o = t1.shape[0]
    b_vv = b_full[:, o:, o:]
    b_vo = b_full[:, o:, :o]                                  # B^X_bk, b virtual, k occupied
    tau = t2 + np.einsum("ic,jd->ijcd", t1, t1)
    dbar = b_vv - 2.0 * np.einsum("xbk,kd->xbd", b_vo, t1)
    return tau, b_vv, dbar


def form_r_fulldf(t2: np.ndarray, t1: np.ndarray, b_full: np.ndarray) -> np.ndarray:
    """R with singles straight from eq. fulldfB (tiny sizes only), without the
    Dbar intermediate: sum_cd sum_X (D^aX_c D^bX_d - 2 sum_k D^aX_c D^bX_k t^k_d) tau_ijcd,
    with the four-index integrals (ac|bd) and (ac|bk) formed explicitly."""
    o = t1.shape[0]
    b_vv = b_full[:, o:, o:]
    b_vo = b_full[:, o:, :o]
    tau = t2 + t1[:, None, :, None] * t1[None, :, None, :]
    g_vvvv = np.einsum("xac,xbd->abcd", b_vv, b_vv)          # (ac|bd)
    g_vvvo = np.einsum("xac,xbk->abck", b_vv, b_vo)          # (ac|bk)
    gbar = g_vvvv - 2.0 * np.einsum("abck,kd->abcd", g_vvvo, t1)
    return np.einsum("abcd,ijcd->ijab", gbar, tau)


def norm_r2_and_energy(r: np.ndarray, t: np.ndarray):
    """||R||^2 (needed by the canonical fit, eq. cpfit) and E_exact = sum R t."""
    return float(np.sum(r * r)), float(np.sum(r * t))


def khatri_rao(*mats: np.ndarray) -> np.ndarray:
    """Column-wise Kronecker product; the last matrix's row index runs fastest."""
    rank = mats[0].shape[1]
    out = np.ones((1, rank))
    for m in mats:
        out = (out[:, None, :] * m[None, :, :]).reshape(-1, rank)
    return out


def unfold(x: np.ndarray, mode: int) -> np.ndarray:
    """Mode-m matricization: rows = axis m, columns = the other axes in order."""
    return np.moveaxis(x, mode, 0).reshape(x.shape[mode], -1)


def mttkrp(r: np.ndarray, factors, mode: int) -> np.ndarray:
    """Textbook MTTKRP: M_m = R_(m) . KR(the other three factors, in axis order).

    ``factors`` = (gamma, rho, alpha, beta).  For mode a this is the numerator
    of the ALS update of alpha in eq. full_der (the sum over c, d, b, i, j).
    """
    others = [f for k, f in enumerate(factors) if k != mode]
    return unfold(r, mode) @ khatri_rao(*others)


def mttkrp_bruteforce(t: np.ndarray, b_vv: np.ndarray, factors, mode: int,
                      b_right: np.ndarray | None = None) -> np.ndarray:
    """Nested loops over every index, straight from R_ijab = sum_cdX B_ac Dbar_bd t_ijcd
    (Dbar = B without singles).

    Pure Python; for tiny sizes only (o, v, X, R of a few).
    """
    br = b_vv if b_right is None else b_right
    gamma, rho, alpha, beta = factors
    o, _, v, _ = t.shape
    nx = b_vv.shape[0]
    rank = gamma.shape[1]
    n_out = (o, o, v, v)[mode]
    out = np.zeros((n_out, rank))
    for r in range(rank):
        for i in range(o):
            for j in range(o):
                for a in range(v):
                    for b in range(v):
                        rv = 0.0
                        for c in range(v):
                            for d in range(v):
                                for x in range(nx):
                                    rv += b_vv[x, a, c] * br[x, b, d] * t[i, j, c, d]
                        w = (gamma[i, r], rho[j, r], alpha[a, r], beta[b, r])
                        prod = 1.0
                        for k in range(4):
                            if k != mode:
                                prod *= w[k]
                        idx = (i, j, a, b)[mode]
                        out[idx, r] += rv * prod
    return out


def mttkrp_chain(t: np.ndarray, b_vv: np.ndarray, factors, mode: int,
                 b_right: np.ndarray | None = None) -> np.ndarray:
    """Matrix-free route in the paper's grouping (eq. distribute and eq. foreachr).

    Modes a and b: tau_r[c, d] = sum_ij gamma_ir rho_jr t_ijcd; the other
    virtual factor is contracted with B first (Dbar^{rX}_d); then the sum over d
    (or c) per r; then the sum over the compound index (X, c).
    Modes i and j (the same idea applied to the occupied factors):
    G_r[c, d] = sum_X (sum_a alpha_ar B^X_ac)(sum_b beta_br B^X_bd),
    H[i, j, r] = sum_cd t_ijcd G_r[c, d], then one occupied factor is summed out.
    With singles the b side carries Dbar (``b_right``) and t is tau.
    """
    gamma, rho, alpha, beta = factors
    br = b_vv if b_right is None else b_right
    if mode in (2, 3):
        tau = np.einsum("ir,jr,ijcd->rcd", gamma, rho, t)
        if mode == 2:
            ybeta = np.einsum("br,xbd->rxd", beta, br)
            z = np.einsum("rxd,rcd->rxc", ybeta, tau)
            return np.einsum("xac,rxc->ar", b_vv, z)
        yalpha = np.einsum("ar,xac->rxc", alpha, b_vv)
        z = np.einsum("rxc,rcd->rxd", yalpha, tau)
        return np.einsum("xbd,rxd->br", br, z)
    yalpha = np.einsum("ar,xac->rxc", alpha, b_vv)
    ybeta = np.einsum("br,xbd->rxd", beta, br)
    g = np.einsum("rxc,rxd->rcd", yalpha, ybeta)
    h = np.einsum("ijcd,rcd->ijr", t, g)
    if mode == 0:
        return np.einsum("ijr,jr->ir", h, rho)
    return np.einsum("ijr,ir->jr", h, gamma)


def cp_full(factors, lam=None) -> np.ndarray:
    """Explicit CP tensor sum_r lam_r gamma_ir rho_jr alpha_ar beta_br (eq. cp-ppl)."""
    gamma, rho, alpha, beta = factors
    if lam is None:
        lam = np.ones(gamma.shape[1])
    return np.einsum("r,ir,jr,ar,br->ijab", lam, gamma, rho, alpha, beta, optimize=True)


def symmetrize_pairs(x: np.ndarray) -> np.ndarray:
    """(X_ijab + X_jiba) / 2: the pair symmetry restored after reconstruction
    (Section "The CPD approximation of the PPL tensor-network")."""
    return 0.5 * (x + x.transpose(1, 0, 3, 2))


def cp_norm2(factors, lam) -> float:
    """||CP||^2 from the Hadamard product of the four Grams (eq. cp_norm2), with weights."""
    w = np.ones((len(lam), len(lam)))
    for f in factors:
        w *= f.T @ f
    return float(lam @ w @ lam)


def cp_inner(m_last: np.ndarray, f_last: np.ndarray, lam: np.ndarray) -> float:
    """<R, CP> = sum_r lam_r sum_n M[n, r] F[n, r] for the MTTKRP of any one mode."""
    return float(np.sum(lam * np.sum(m_last * f_last, axis=0)))


def energy_cp(t: np.ndarray, factors, lam) -> float:
    """E_CP = sum_ijab CP_ijab t_ijab (the PPL energy-like contraction), in FP64."""
    gamma, rho, alpha, beta = factors
    o, _, v, _ = t.shape
    p = t.reshape(o * o, v * v) @ khatri_rao(alpha, beta)     # (ij) x r
    q = khatri_rao(gamma, rho)                                 # (ij) x r
    return float(np.sum(lam * np.sum(p * q, axis=0)))


def rank1_closed_form(u, w, p, q, b_vv, b_right=None):
    """R for T2 (or tau) = u_i w_j p_c q_d, in closed CP form of rank X.

    R_ijab = u_i w_j sum_X (B^X p)_a (Dbar^X q)_b, so R = CP with factors
    (u 1^T, w 1^T, P, Q), P[a, X] = sum_c B^X_ac p_c, Q[b, X] = sum_d Dbar^X_bd q_d
    (Dbar = B without singles).
    """
    nx = b_vv.shape[0]
    pm = np.einsum("xac,c->ax", b_vv, p)
    qm = np.einsum("xbd,d->bx", b_vv if b_right is None else b_right, q)
    return (np.outer(u, np.ones(nx)), np.outer(w, np.ones(nx)), pm, qm)


def planted_mttkrp(true_factors, true_lam, factors, mode: int) -> np.ndarray:
    """MTTKRP of a CP-form tensor without forming it.

    M_m = F_m^true diag(lam^true) (*_{k != m} (F_k^true)^T F_k), with * the
    Hadamard product; O(n R_true R) work, usable at any size.
    """
    cross = np.ones((len(true_lam), factors[0].shape[1]))
    for k in range(4):
        if k != mode:
            cross *= true_factors[k].T @ factors[k]
    return true_factors[mode] @ (true_lam[:, None] * cross)
