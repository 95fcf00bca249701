"""Plain FP64 CPU oracle for the CP-PPL decomposition.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never calls it, and it shares no code with the GPU library: it uses numpy and
scipy only, forms the particle-particle-ladder tensor R explicitly, and runs
textbook CP-ALS on it (Kolda & Bader, SIAM Review 51 (2009), Section 3.4).

Parity status of each function is stated in its docstring; every function
here is pinned by a ``-m "not gpu"`` test except where "parity unpinned" is
written.
"""
from .ppl import (  # noqa: F401
    recompute_t,
    df_integrals,
    form_r,
    form_r_einsum,
    form_r_fulldf,
    dress,
    form_r_pairs,
    norm_r2_and_energy,
    khatri_rao,
    unfold,
    mttkrp,
    mttkrp_bruteforce,
    mttkrp_chain,
    cp_full,
    symmetrize_pairs,
    cp_norm2,
    cp_inner,
    energy_cp,
    rank1_closed_form,
    planted_mttkrp,
)
from .als import (  # noqa: F401
    NotSPD,
    gram_hadamard,
    solve_normal,
    als_update,
    cp_als,
    sweep_scalars,
    eta,
)
from . import mlp  # noqa: F401
from . import ccd  # noqa: F401
from . import fp8  # noqa: F401
