"""Pins of the CPU oracle against facts that do not come from the oracle itself:
hand-derived worked examples, brute force, closed forms, identities and
invariants of the definitions (eq. dfB, eq. full_der, eq. cpfit, eq. cp_norm2).
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")
MODE = {"i": 0, "j": 1, "a": 2, "b": 3}


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def _rand_problem(o, v, nx, rank, seed):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((nx, v, v))
    b = 0.5 * (b + b.transpose(0, 2, 1))
    t = rng.standard_normal((o, o, v, v))
    t = 0.5 * (t + t.transpose(1, 0, 3, 2))
    fs = (rng.standard_normal((o, rank)), rng.standard_normal((o, rank)),
          rng.standard_normal((v, rank)), rng.standard_normal((v, rank)))
    return b, t, fs


# ---------------------------------------------------------------- golden cases
@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_worked_example_tensor(case):
    b = np.array(case["B"], dtype=float)
    t = np.array(case["t"], dtype=float)
    r = oracle.form_r(t, b)
    np.testing.assert_allclose(r, np.array(case["R"], dtype=float), atol=1e-14)
    n2, e = oracle.norm_r2_and_energy(r, t)
    assert n2 == pytest.approx(case["norm_r2"], rel=1e-14)
    assert e == pytest.approx(case["energy_exact"], rel=1e-14)


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_worked_example_mttkrp(case):
    b = np.array(case["B"], dtype=float)
    t = np.array(case["t"], dtype=float)
    f = case["factors"]
    fs = tuple(np.array(f[k], dtype=float) for k in ("gamma", "rho", "alpha", "beta"))
    r = oracle.form_r(t, b)
    for name, want in case["mttkrp"].items():
        m = MODE[name]
        want = np.array(want, dtype=float)
        np.testing.assert_allclose(oracle.mttkrp(r, fs, m), want, atol=1e-14)
        np.testing.assert_allclose(oracle.mttkrp_chain(t, b, fs, m), want, atol=1e-14)
        np.testing.assert_allclose(oracle.mttkrp_bruteforce(t, b, fs, m), want, atol=1e-14)


@pytest.mark.parametrize("case", [c for c in _cases() if "rank1_best_fit" in c],
                         ids=lambda c: c["name"])
def test_worked_example_rank1_fit(case):
    b = np.array(case["B"], dtype=float)
    t = np.array(case["t"], dtype=float)
    r = oracle.form_r(t, b)
    o, v = case["o"], case["v"]
    rng = np.random.default_rng(3)
    init = (np.ones((o, 1)), np.ones((o, 1)), rng.uniform(-1, 1, (v, 1)),
            rng.uniform(-1, 1, (v, 1)))
    fs, lam, hist = oracle.cp_als(r, init, 20)
    assert hist["fit"][-1] == pytest.approx(case["rank1_best_fit"], abs=1e-10)


# ---------------------------------------------------------------- MTTKRP routes
@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_mttkrp_three_routes_tiny(seed, mode):
    b, t, fs = _rand_problem(2, 3, 2, 2, seed)
    # no symmetry is assumed anywhere: break it on purpose
    b = b + 0.1 * np.random.default_rng(seed + 7).standard_normal(b.shape)
    t = t + 0.1 * np.random.default_rng(seed + 8).standard_normal(t.shape)
    r = oracle.form_r(t, b)
    brute = oracle.mttkrp_bruteforce(t, b, fs, mode)
    mat = oracle.mttkrp(r, fs, mode)
    chain = oracle.mttkrp_chain(t, b, fs, mode)
    scale = np.linalg.norm(brute)
    assert np.linalg.norm(mat - brute) <= 1e-13 * scale
    assert np.linalg.norm(chain - brute) <= 1e-13 * scale


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_mttkrp_routes_c1(mode):
    cfg = synth.CONFIGS["C1"]
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    r = oracle.form_r(inp.t, inp.b_vv)
    mat = oracle.mttkrp(r, fs, mode)
    chain = oracle.mttkrp_chain(inp.t, inp.b_vv, fs, mode)
    assert np.linalg.norm(mat - chain) <= 1e-13 * np.linalg.norm(mat)


def test_khatri_rao_definition():
    rng = np.random.default_rng(0)
    a, b, c = rng.standard_normal((2, 3)), rng.standard_normal((4, 3)), rng.standard_normal((5, 3))
    kr = oracle.khatri_rao(a, b, c)
    for i in range(2):
        for j in range(4):
            for k in range(5):
                np.testing.assert_allclose(kr[(i * 4 + j) * 5 + k], a[i] * b[j] * c[k])


# ---------------------------------------------------------------- R construction
def test_r_two_routes_and_blocking():
    b, t, _ = _rand_problem(3, 5, 4, 2, 11)
    r1 = oracle.form_r(t, b)
    r2 = oracle.form_r_einsum(t, b)
    r3 = oracle.form_r(t, b, block=2)
    np.testing.assert_allclose(r1, r2, rtol=0, atol=1e-13 * np.abs(r2).max())
    np.testing.assert_allclose(r1, r3, rtol=0, atol=1e-13 * np.abs(r2).max())
    rows = oracle.form_r(t, b, ij_rows=slice(2, 7))
    np.testing.assert_allclose(rows, r1.reshape(9, 5, 5)[2:7], atol=1e-13 * np.abs(r2).max())


def test_r_pairs_route_matches():
    b, t, _ = _rand_problem(4, 6, 5, 2, 13)
    r = oracle.form_r(t, b)
    np.testing.assert_allclose(oracle.form_r_pairs(t, b, 3), r[:3, :3],
                               atol=1e-13 * np.abs(r).max())


def test_r_pair_symmetry_with_symmetric_inputs():
    cfg = synth.CONFIGS["C1"]
    inp = synth.make_inputs(cfg)
    r = oracle.form_r(inp.t, inp.b_vv)
    assert np.abs(r - r.transpose(1, 0, 3, 2)).max() <= 1e-13 * np.abs(r).max()


def test_rank1_t2_closed_form():
    cfg = synth.custom_config(3, 6, 5, 4)
    inp = synth.make_inputs(cfg)
    t, (u, w, p, q) = synth.rank1_t2(cfg)
    r = oracle.form_r(t, inp.b_vv)
    cf = oracle.rank1_closed_form(u, w, p, q, inp.b_vv)
    np.testing.assert_allclose(oracle.cp_full(cf), r, atol=1e-13 * np.abs(r).max())
    fs = synth.init_factors(cfg)
    for mode in range(4):
        want = oracle.mttkrp(r, fs, mode)
        got = oracle.planted_mttkrp(cf, np.ones(cfg.nx), fs, mode)
        assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)


# ---------------------------------------------------------------- CP identities
def test_cp_norm_and_residual_identity():
    b, t, fs = _rand_problem(3, 4, 3, 5, 5)
    r = oracle.form_r(t, b)
    lam = np.abs(np.random.default_rng(1).standard_normal(5)) + 0.1
    cp = oracle.cp_full(fs, lam)
    assert oracle.cp_norm2(fs, lam) == pytest.approx(np.sum(cp * cp), rel=1e-13)
    n2 = np.sum(r * r)
    inner_explicit = np.sum(r * cp)
    for mode in range(4):
        m = oracle.mttkrp(r, fs, mode)
        assert oracle.cp_inner(m, fs[mode], lam) == pytest.approx(inner_explicit, rel=1e-12)
    lhs = np.sum((r - cp) ** 2)
    rhs = n2 - 2 * inner_explicit + oracle.cp_norm2(fs, lam)
    assert lhs == pytest.approx(rhs, rel=1e-11)


def test_energy_cp_explicit_and_symmetrisation_invariance():
    cfg = synth.CONFIGS["C1"]
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    lam = np.linspace(0.5, 2.0, cfg.rank)
    cp = oracle.cp_full(fs, lam)
    e_explicit = np.sum(cp * inp.t)
    assert oracle.energy_cp(inp.t, fs, lam) == pytest.approx(e_explicit, rel=1e-12)
    # half-sum with the pair-transposed tensor (Section CP-PPL, restoring symmetry)
    sym = 0.5 * (cp + cp.transpose(1, 0, 3, 2))
    assert np.sum(sym * inp.t) == pytest.approx(e_explicit, rel=1e-12)


def test_planted_mttkrp_matches_explicit():
    rng = np.random.default_rng(4)
    true = tuple(rng.standard_normal((n, 3)) for n in (3, 3, 4, 5))
    lam = np.array([1.0, 2.0, 0.5])
    r = oracle.cp_full(true, lam)
    fs = tuple(rng.standard_normal((n, 6)) for n in (3, 3, 4, 5))
    for mode in range(4):
        np.testing.assert_allclose(oracle.planted_mttkrp(true, lam, fs, mode),
                                   oracle.mttkrp(r, fs, mode), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- ALS behaviour
def test_als_monotone_and_stationary_c1():
    cfg = synth.CONFIGS["C1"]
    inp = synth.make_inputs(cfg)
    r = oracle.form_r(inp.t, inp.b_vv)
    factors = [np.array(f) for f in synth.init_factors(cfg)]
    n2 = float(np.sum(r * r))
    prev_loss = np.inf
    for sweep in range(15):
        for mode in oracle.als.SWEEP_ORDER:
            factors, lam, m, _ = oracle.als_update(r, factors, mode)
            w = oracle.gram_hadamard(factors, mode)
            # first-order optimality of the block least-squares problem
            resid = m - (factors[mode] * lam) @ w
            assert np.linalg.norm(resid) <= 1e-10 * np.linalg.norm(m)
            cp = oracle.cp_full(factors, lam)
            loss = 0.5 * np.sum((r - cp) ** 2)
            assert loss <= prev_loss * (1 + 1e-12) + 1e-12
            prev_loss = loss
        _, _, fit, loss_id = oracle.sweep_scalars(n2, m, factors, lam)
        assert loss_id == pytest.approx(prev_loss, rel=1e-9)


def test_als_solve_matches_lstsq():
    rng = np.random.default_rng(2)
    fs = [rng.standard_normal((n, 4)) for n in (3, 3, 5, 5)]
    r = rng.standard_normal((3, 3, 5, 5))
    m = oracle.mttkrp(r, fs, 2)
    w = oracle.gram_hadamard(fs, 2)
    f, _ = oracle.solve_normal(m, w)
    kr = oracle.khatri_rao(fs[0], fs[1], fs[3])
    ls = np.linalg.lstsq(kr, oracle.unfold(r, 2).T, rcond=None)[0].T
    np.testing.assert_allclose(f, ls, rtol=1e-10, atol=1e-12)


def test_rank1_planted_exact_after_one_sweep():
    rng = np.random.default_rng(9)
    true = tuple(rng.standard_normal((n, 1)) for n in (3, 4, 5, 6))
    r = oracle.cp_full(true, np.array([3.0]))
    init = tuple(rng.uniform(-1, 1, (n, 1)) for n in (3, 4, 5, 6))
    fs, lam, hist = oracle.cp_als(r, init, 1)
    cp = oracle.cp_full(fs, lam)
    assert np.linalg.norm(r - cp) <= 1e-12 * np.linalg.norm(r)


def test_kruskal_unique_planted_recovery():
    rng = np.random.default_rng(21)
    rank = 3
    true = tuple(rng.standard_normal((n, rank)) for n in (4, 5, 6, 7))
    r = oracle.cp_full(true, np.ones(rank))
    init = tuple(rng.uniform(-1, 1, (n, rank)) for n in (4, 5, 6, 7))
    fs, lam, hist = oracle.cp_als(r, init, 300)
    cp = oracle.cp_full(fs, lam)
    assert 1 - np.linalg.norm(r - cp) / np.linalg.norm(r) >= 1 - 1e-10
    # factor congruence (columns match up to permutation and sign)
    for k in range(4):
        tn = true[k] / np.linalg.norm(true[k], axis=0)
        c = np.abs(tn.T @ fs[k])
        assert np.all(c.max(axis=1) >= 1 - 1e-8)


def test_ridge_retry_on_duplicate_columns():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((4, 3))
    f[:, 2] = f[:, 1]
    fs = [f.copy(), f.copy(), np.vstack([f, f]), np.vstack([f, f])]
    w = oracle.gram_hadamard(fs, 2)
    m = rng.standard_normal((8, 3))
    out, retries = oracle.solve_normal(m, w)
    assert retries >= 1 and np.all(np.isfinite(out))


def test_eta_matches_explicit():
    rng = np.random.default_rng(6)
    f1 = [rng.standard_normal((n, 4)) for n in (3, 3, 4, 4)]
    f2 = [x + 0.1 * rng.standard_normal(x.shape) for x in f1]
    l1, l2 = np.abs(rng.standard_normal(4)), np.abs(rng.standard_normal(4))
    c1, c2 = oracle.cp_full(f1, l1), oracle.cp_full(f2, l2)
    want = np.linalg.norm(c2 - c1) / np.linalg.norm(c1)
    assert oracle.eta(f1, l1, f2, l2) == pytest.approx(want, rel=1e-10)


# ---------------------------------------------------------------- fixtures
def test_fixtures_deterministic_and_shaped():
    cfg = synth.CONFIGS["C1"]
    a, b = synth.make_inputs(cfg), synth.make_inputs(cfg)
    np.testing.assert_array_equal(a.t, b.t)
    np.testing.assert_array_equal(a.b_full, b.b_full)
    assert not np.array_equal(a.t, synth.make_inputs(cfg, seed=1).t)
    assert np.array_equal(a.b_full, a.b_full.transpose(0, 2, 1))
    d = (a.e_occ[:, None, None, None] + a.e_occ[None, :, None, None]
         - a.e_vir[None, None, :, None] - a.e_vir[None, None, None, :])
    assert d.max() <= -1.0
    assert np.abs(a.t - a.t.transpose(1, 0, 3, 2)).max() <= 1e-15 * np.abs(a.t).max()
    t2 = oracle.recompute_t(a.b_full, a.e_occ, a.e_vir)
    np.testing.assert_allclose(a.t, t2, rtol=1e-12, atol=1e-15)
    fs = synth.init_factors(cfg)
    assert [f.shape for f in fs] == [(4, 32), (4, 32), (16, 32), (16, 32)]
    assert all(np.abs(f).max() <= 1.0 for f in fs)


def test_perturbation_scale_and_symmetry():
    cfg = synth.CONFIGS["C1"]
    inp = synth.make_inputs(cfg)
    e = synth.perturbation(cfg, 3, inp.t)
    assert np.linalg.norm(e) == pytest.approx(1e-2 * np.linalg.norm(inp.t), rel=1e-12)
    np.testing.assert_allclose(e, e.transpose(1, 0, 3, 2), atol=1e-18)
