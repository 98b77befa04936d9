"""Pins of the SuperMann / Anderson oracle (oracle/supermann_oracle.py).

What the paper and the mathematics fix, independently of the oracle's code:
  * the least-squares step of Anderson's acceleration (Sec. 5.2, Alg.
    "Anderson's acceleration") is the minimiser NumPy's lstsq returns;
  * <., .>_M is the quadratic form of the dense matrix
    [[I, -alpha L*], [-alpha L, I]] (Sec. 4.1) assembled column by column,
    and it is positive definite when alpha |L| < 1;
  * T is firmly nonexpansive in that norm (the property SuperMann needs):
    |Tu - Tv|_M^2 <= <Tu - Tv, u - v>_M;
  * the accelerated solve reaches the same optimal value as plain CP and as
    the independent NLP solve of the tiny tree, in fewer applications of T.
A planted sign mistake in the M inner product fails the firm
nonexpansiveness check; a dropped alpha fails the dense comparison.
"""
import json
import os

import numpy as np
import pytest

from oracle import spock_oracle as O
from oracle import supermann_oracle as SM
from paper_2505_12078_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_aa_least_squares_matches_lstsq():
    rng = np.random.default_rng(0)
    for n, m in ((50, 3), (400, 3), (30, 5)):
        Y = rng.standard_normal((n, m))
        r = rng.standard_normal(n)
        k = SM.aa_least_squares(Y, r)
        ref = np.linalg.lstsq(Y, r, rcond=None)[0]
        np.testing.assert_allclose(k, ref, rtol=1e-10, atol=1e-12)


def _dense_L(D):
    Y = D.layout
    cols = []
    for k in range(Y.nz):
        e = np.zeros(Y.nz)
        e[k] = 1.0
        cols.append(O.apply_L(D, e))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("seed", [0, 1])
def test_m_inner_is_the_dense_preconditioner(seed):
    p = W.config_problem(0) if seed == 0 else W.random_ragged_problem(3, N=3, nx=2, nu=1, max_children=3)
    D = O.Data(p)
    a = O.step_size(D)
    L = _dense_L(D)
    nz, ne = L.shape[1], L.shape[0]
    M = np.block([[np.eye(nz), -a * L.T], [-a * L, np.eye(ne)]])
    rng = np.random.default_rng(seed)
    for _ in range(3):
        u, v = rng.standard_normal(nz + ne), rng.standard_normal(nz + ne)
        got = SM.m_inner(D, a, u[:nz], u[nz:], v[:nz], v[nz:])
        assert got == pytest.approx(u @ M @ v, rel=1e-12, abs=1e-12)
        assert SM.m_norm(D, a, u[:nz], u[nz:]) == pytest.approx(np.sqrt(u @ M @ u), rel=1e-12)
    # alpha |L| < 1 makes M positive definite: smallest eigenvalue 1 - alpha |L|
    lam = np.linalg.eigvalsh(M)
    assert lam.min() == pytest.approx(1 - a * O.L_norm(D), rel=1e-9)
    assert lam.min() > 0


def _fne_gap(D, F, a, inner, rng):
    """max over random pairs of |Tu - Tv|_M^2 - <Tu - Tv, u - v>_M (<= 0 for
    a firmly nonexpansive T)."""
    nz, ne = D.layout.nz, D.layout.neta
    worst = -np.inf
    for _ in range(6):
        u = rng.standard_normal(nz + ne) * 3
        v = u + rng.standard_normal(nz + ne) * rng.choice([0.01, 0.3, 3.0])
        Tu = np.concatenate(O.cp_step(D, F, u[:nz], u[nz:], a))
        Tv = np.concatenate(O.cp_step(D, F, v[:nz], v[nz:], a))
        d, dT = u - v, Tu - Tv
        lhs = inner(dT[:nz], dT[nz:], dT[:nz], dT[nz:])
        rhs = inner(dT[:nz], dT[nz:], d[:nz], d[nz:])
        worst = max(worst, (lhs - rhs) / max(1.0, abs(rhs)))
    return worst


@pytest.mark.parametrize("name", ["cfg0", "ragged"])
def test_T_is_firmly_nonexpansive_in_the_M_norm(name):
    p = W.config_problem(0) if name == "cfg0" else W.random_ragged_problem(5, N=3, nx=3, nu=2, max_children=3)
    D = O.Data(p)
    F = O.Offline(D)
    a = O.step_size(D)
    gap = _fne_gap(D, F, a, lambda az, ae, bz, be: SM.m_inner(D, a, az, ae, bz, be), np.random.default_rng(7))
    assert gap <= 1e-10


def test_planted_sign_mistake_in_M_fails_firm_nonexpansiveness():
    p = W.config_problem(0)
    D = O.Data(p)
    F = O.Offline(D)
    a = O.step_size(D)

    def flipped(az, ae, bz, be):
        return float(az @ bz + ae @ be + a * (O.apply_L(D, az) @ be + ae @ O.apply_L(D, bz)))

    def no_alpha(az, ae, bz, be):
        return float(az @ bz + ae @ be - (O.apply_L(D, az) @ be + ae @ O.apply_L(D, bz)))

    assert _fne_gap(D, F, a, flipped, np.random.default_rng(7)) > 1e-6
    # a dropped alpha keeps T firmly nonexpansive here, but it is not the
    # dense preconditioner's form
    L = _dense_L(D)
    nz, ne = L.shape[1], L.shape[0]
    M = np.block([[np.eye(nz), -a * L.T], [-a * L, np.eye(ne)]])
    u, v = np.random.default_rng(3).standard_normal((2, nz + ne))
    assert abs(no_alpha(u[:nz], u[nz:], v[:nz], v[nz:]) - u @ M @ v) > 1e-3


@pytest.fixture(scope="module")
def tiny_vstar():
    with open(os.path.join(HERE, "golden", "tiny_tree_vstar.json")) as f:
        return json.load(f)["tiny"][0]["vstar"]


def test_supermann_reaches_the_plain_optimum_with_fewer_T(tiny_vstar):
    p = W.config_problem(0)
    r = SM.solve(p, eps=1e-6, max_iters=20000)
    assert r["status"] == "converged"
    assert abs(r["s0"] - tiny_vstar) <= 10 * 1e-6 * max(1.0, abs(tiny_vstar))
    assert O.nested_cost(p, r["x"], r["u"]) == pytest.approx(r["s0"], rel=1e-5)
    assert O.dynamics_violation(p, r["x"], r["u"]) < 1e-10
    # plain CP needs 3,635 applications of T for the same tolerance
    assert r["counts"]["T"] < 3635
    assert r["counts"]["K0"] + r["counts"]["K1"] + r["counts"]["K2"] == r["iters"]


def test_supermann_risk_neutral_special_case():
    """gamma = 1 with loose bounds: unique (x, u) of the textbook Riccati
    recursion, also through the accelerated iteration."""
    p = W.config_problem(0)
    p["gamma"] = np.ones_like(p["gamma"])
    for k in ("x_lo", "x_hi", "u_lo", "u_hi", "xN_lo", "xN_hi"):
        p[k] = p[k] * 1e3
    V, x, u = O.risk_neutral_lq(p)
    r = SM.solve(p, eps=1e-9, max_iters=20000)
    assert r["status"] == "converged"
    assert r["s0"] == pytest.approx(V, rel=1e-7)
    np.testing.assert_allclose(r["x"], x, atol=1e-6)
    np.testing.assert_allclose(r["u"], u, atol=1e-6)
