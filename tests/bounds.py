"""Tolerances of the parity tests, derived from the arithmetic.

FP64 path.  The GPU chain and the oracle's explicit MTTKRP add the same terms in
different orders, so they agree to a few ulps of the sums of |terms|: element by
element to rtol 1e-10, with atol 1e-10 * max|M| for elements that cancel.

Low-precision paths.  Every term of a low-precision MTTKRP element passes
through a fixed number of bfloat16 roundings (unit roundoff u = 2^-8, round to
nearest even) and through FP32 accumulations (u32 = 2^-24) of K-long sums:

* BF16 contexts, modes a and b: t, B (twice: B^X_ac and B^X_bd), the other
  virtual factor, the Khatri-Rao product gamma_ir rho_jr, and the rounded
  intermediates tau, Y and Z -- 8 roundings.  Modes i and j: alpha, beta, B
  twice, Y_alpha, Y_beta, G and t -- 8 roundings.
* FP8 contexts compared with the oracle's chain on the dequantised inputs: the
  e4m3 values of t and B (times a power of two) are exact in bfloat16, which
  leaves the 5 roundings of the factors and intermediates.

Two bounds follow.
* Element-wise and rigorous (not a first-order estimate): every term carries a
  factor prod_k (1 + d_k), |d_k| <= u, so
      |M_gpu - M| <= ((1 + u)^n (1 + u32)^(sum K) - 1) * M_abs,
  with M_abs the same chain evaluated on |t|, |B| and |factors|.
* Norm-wise and statistical: independent roundings with errors uniform in
  [-u, u] (standard deviation u / sqrt 3) give a relative error of about
  u sqrt(n / 3) per element when the sums do not cancel; the tests allow twice
  that, ||M_gpu - M||_F / ||M||_F <= 2 u sqrt(n / 3) (1.28e-2 for n = 8,
  1.01e-2 for n = 5).  The long sums average the errors further, so the
  measured errors sit well below it (about 2e-3 in modes a and b, 3e-4 in i
  and j).
"""
from __future__ import annotations

import numpy as np

import oracle

U_BF16 = 2.0 ** -8
U_FP32 = 2.0 ** -24
U_E4M3 = 2.0 ** -4
N_ROUND_BF16 = 8
N_ROUND_FP8 = 5


def normwise(n_round: int) -> float:
    return 2.0 * U_BF16 * np.sqrt(n_round / 3.0)


def chain_lengths(o: int, v: int, nx: int, mode: int):
    """Lengths of the FP32-accumulated sums a term of mode `mode` passes through."""
    if mode >= 2:
        return [o * o, v, v, nx * v]      # tau, Y, Z, M
    return [v, v, nx, v * v]              # Y_alpha, Y_beta, G, H


def elementwise_gamma(n_round: int, ks) -> float:
    return (1.0 + U_BF16) ** n_round * (1.0 + U_FP32) ** float(sum(ks)) - 1.0


def abs_chain(t, b, factors, mode, b_right=None):
    """M_abs: the MTTKRP chain on absolute values (oracle, FP64)."""
    return oracle.mttkrp_chain(np.abs(t), np.abs(b), [np.abs(f) for f in factors], mode,
                               b_right=None if b_right is None else np.abs(b_right))


def rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def assert_fp64(got, want, rtol=1e-10):
    """Element-wise FP64 parity: |got - want| <= rtol |want| + rtol max|want|."""
    np.testing.assert_allclose(got, want, rtol=rtol, atol=rtol * float(np.abs(want).max()))


def assert_lowp(got, want, m_abs, n_round, ks, label="", normwise_check=True):
    """Both low-precision bounds: element-wise against M_abs, norm-wise against M
    (the statistical one only where the sums are long enough to average: not
    for the degenerate one-term shapes).  Returns the norm-wise relative error."""
    gamma = elementwise_gamma(n_round, ks)
    diff = np.abs(got - want)
    worst = float(np.max(diff - gamma * m_abs))
    assert worst <= 1e-300 + 1e-13 * float(np.abs(m_abs).max()), \
        f"{label}: element-wise bound exceeded by {worst:.3e} (gamma {gamma:.3e})"
    err = rel(got, want)
    if normwise_check:
        assert err <= normwise(n_round), f"{label}: norm-wise {err:.3e} > {normwise(n_round):.3e}"
    return err
