"""Parity of the gfx950 library with the FP64 oracle, through the C ABI.

Tolerances (derived in the design doc):
  * L, L*, prox_{alpha g*} in float64: 1e-12 relative to the input scale
    (a handful of rounding errors per entry).
  * One CP step T in float64: 1e-10 relative to max(1, |v|_inf, |T v|_inf)
    (the S1 sweep chains N stages of length-(nx+nu) dot products, and the
    GPU uses the reduced recursion while the oracle runs Alg. 2 with P).
  * One CP step in float32: 2e-4 relative (float32 rounding ~6e-8 amplified
    by the same chains).
  * Solutions: |V*_gpu - V*_oracle| <= 1e-6 max(1, |V*|) with both at
    rel_res <= 1e-6 (float64), and 1e-4 for the mixed form.
"""
import numpy as np
import pytest

from oracle import spock_oracle as O
from paper_2505_12078_amd import spock as S
from paper_2505_12078_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X; none is visible")
    S.load()


def _cases():
    cases = {
        "cfg0": W.config_problem(0),
        "cfg1": W.config_problem(1),
        "ragged_a": W.random_ragged_problem(1, N=4, nx=3, nu=2, max_children=3),
        "ragged_affine": W.random_ragged_problem(2, N=3, nx=5, nu=3, max_children=4, affine=True),
        "ragged_noball": W.random_ragged_problem(3, N=5, nx=4, nu=1, max_children=2, ball=False),
    }
    # single scenario (every node has one child) and the smallest tree
    par, _ = W.tree_from_branching([1, 1, 1, 1])
    cases["chain"] = W.make_problem(par, 3, 2, np.random.default_rng(11), x_ball=6.0, name="chain")
    par, _ = W.tree_from_branching([1])
    cases["two_nodes"] = W.make_problem(par, 2, 1, np.random.default_rng(12), name="two_nodes")
    # extreme risk levels: AV@R_0 = max and AV@R_1 = expectation
    p = W.random_ragged_problem(4, N=3, nx=3, nu=2)
    p["gamma"] = np.where(np.arange(p["gamma"].size) % 2 == 0, 0.0, 1.0)
    cases["gamma_0_1"] = p
    # wide node (many children) and larger dimensions
    par, _ = W.tree_from_branching([7, 2])
    cases["wide"] = W.make_problem(par, 9, 4, np.random.default_rng(13), prob_kind="dirichlet",
                                   gamma=0.6, x_ball=8.0, name="wide")
    # wider than the staged-children limit: per-child inputs read in place
    par, _ = W.tree_from_branching([24, 2])
    cases["very_wide"] = W.make_problem(par, 4, 2, np.random.default_rng(15), prob_kind="dirichlet",
                                        gamma=0.7, x_ball=7.0, name="very_wide")
    # the longest horizon the library takes (512 stages), as a single scenario
    # and with eight scenarios branching off near the root
    par, _ = W.tree_from_branching([1] * 511)
    cases["deep_chain"] = W.make_problem(par, 2, 1, np.random.default_rng(16), x_ball=6.0, name="deep_chain")
    par, _ = W.tree_from_branching([2, 2, 2] + [1] * 300)
    cases["deep_branched"] = W.make_problem(par, 3, 2, np.random.default_rng(17), prob_kind="dirichlet",
                                            gamma=0.8, x_ball=7.0, name="deep_branched")
    # the widest state and input the library takes: nx + nu = 128
    par, _ = W.tree_from_branching([2, 1])
    cases["max_m"] = W.make_problem(par, 96, 32, np.random.default_rng(18), prob_kind="dirichlet",
                                    x_ball=12.0, name="max_m")
    par, _ = W.tree_from_branching([2, 1, 1])
    cases["big_nx"] = W.make_problem(par, 70, 40, np.random.default_rng(14), prob_kind="dirichlet",
                                     x_ball=12.0, name="big_nx")
    # products wider than two 64-column blocks (nx + nu > 128): the
    # networked-control case study's shapes (augmented state 150, input 50,
    # m = 200) with random stable dynamics, the case study's own delay tree
    # (operators only, see ILL_CONDITIONED), a generic nx = 100, nu = 50, and
    # the widest state the library takes (nx = 256)
    par, _ = W.tree_from_branching([4, 1, 1])
    cases["m200"] = W.make_problem(par, 150, 50, np.random.default_rng(21), x_ball=15.0, name="m200")
    cases["delay_m200"] = W.delay_problem([4, 1, 1], nx=100, nu=50)
    par, _ = W.tree_from_branching([2, 2, 1])
    cases["m150"] = W.make_problem(par, 100, 50, np.random.default_rng(19), prob_kind="dirichlet",
                                   x_ball=15.0, name="m150")
    par, _ = W.tree_from_branching([2, 1])
    cases["nx256"] = W.make_problem(par, 256, 6, np.random.default_rng(20), prob_kind="dirichlet",
                                    x_ball=20.0, name="nx256")
    # linear cost terms (Prop. 1 with q != 0): per-edge and per-leaf translations
    cases["linear"] = W.random_ragged_problem(4, N=3, nx=2, nu=1, linear=True)
    cases["linear_big"] = W.random_ragged_problem(8, N=4, nx=12, nu=5, max_children=3, linear=True)
    # per-edge stage costs and per-leaf terminal costs (each edge's own Q^j, R^j)
    cases["edge_costs"] = W.random_ragged_problem(6, N=3, nx=2, nu=1, edge_costs=True)
    cases["edge_costs_lin"] = W.random_ragged_problem(9, N=4, nx=10, nu=4, max_children=4, linear=True,
                                                      edge_costs=True)
    # dense per-edge stage costs and per-leaf terminal costs (symmetric
    # square roots in L and L*): small, with linear terms, more than one row
    # per lane (nx = 100), and an instance of the benchmark case study's random
    # problems (nx = 84, nu = 42: event-dependent dense Q(w), R(w), Q_N = Q_0)
    cases["dense"] = W.random_ragged_problem(5, N=3, nx=3, nu=2, dense_costs=True)
    cases["dense_lin"] = W.random_ragged_problem(10, N=4, nx=12, nu=6, max_children=4, linear=True,
                                                 dense_costs=True)
    par, _ = W.tree_from_branching([2, 2, 1])
    cases["dense_m150"] = W.make_problem(par, 100, 50, np.random.default_rng(22), prob_kind="dirichlet",
                                         x_ball=15.0, dense_costs=True, linear=True, name="dense_m150")
    cases["bench1"] = W.benchmark_problem(1, nu_max=128)
    # general constraint rows (box rows plus coupling rows W_x x + W_u u at
    # non-leaf nodes, W_N x at leaves): small, with dense costs and linear
    # terms, and with 135 rows and 100 columns (more than one row and column
    # per lane)
    cases["general"] = W.random_ragged_problem(7, N=3, nx=3, nu=2, general_con=True)
    cases["general_dense"] = W.random_ragged_problem(11, N=3, nx=6, nu=3, max_children=3, general_con=True,
                                                     dense_costs=True, linear=True)
    par, _ = W.tree_from_branching([2, 2, 1])
    cases["general_big"] = W.make_problem(par, 70, 30, np.random.default_rng(23), prob_kind="dirichlet",
                                          general_con=True, name="general_big")
    # general coherent risks (conic data E, F, b, K per node): the spectral
    # risk w AV@R_g1 + (1 - w) AV@R_g2 (y of 5k + 2 rows, F of 2k columns); a
    # root with 20 children (102 rows of y: two rows per lane, 60 rows of G);
    # one with general constraint rows, dense costs and linear terms; and
    # AV@R itself given as general data
    cases["spectral"] = W.spectral_risk(W.random_ragged_problem(4, N=3, nx=3, nu=2), weight=0.4)
    par, _ = W.tree_from_branching([20, 2, 1])
    cases["spectral_wide"] = W.spectral_risk(W.make_problem(par, 8, 4, np.random.default_rng(24),
                                                            prob_kind="dirichlet", name="spectral_wide"),
                                             weight=0.7, gammas=(0.1, 0.6))
    cases["spectral_mixed"] = W.spectral_risk(W.random_ragged_problem(11, N=3, nx=6, nu=3, max_children=3,
                                                                      general_con=True, dense_costs=True,
                                                                      linear=True))
    cases["avar_general"] = _avar_as_general(W.random_ragged_problem(5, N=3, nx=3, nu=2))
    # the l2-ball ambiguity risk (a second-order cone block in K): small, and
    # a root with 63 children whose cone block's head row sits on the second
    # row of its lane (y of 128 rows)
    cases["l2ball"] = W.l2_ball_risk(W.random_ragged_problem(4, N=3, nx=3, nu=2), r_frac=0.6)
    par, _ = W.tree_from_branching([63, 1])
    cases["l2ball_63"] = W.l2_ball_risk(W.make_problem(par, 4, 2, np.random.default_rng(25), prob_kind="dirichlet",
                                                       name="l2ball_63"), r_frac=0.8)
    # soft upper bound on x_0 at non-leaf nodes (slack inputs and general rows)
    # Prop. 2's l1 input penalty: slack inputs without quadratic cost whose
    # linear term enters the tau rows of L (Prop. 1 with R singular); small,
    # and with per-edge diagonal costs and linear terms on the original inputs
    cases["l1"] = W.l1_input_penalty(W.random_ragged_problem(7, N=2, nx=3, nu=2, ball=False), 2.0)
    cases["l1_edge"] = W.l1_input_penalty(W.random_ragged_problem(12, N=3, nx=4, nu=3, edge_costs=True, linear=True,
                                                                  ball=False), 0.5)
    cases["soft"] = W.soft_state_bounds(W.random_ragged_problem(7, N=2, nx=3, nu=2, ball=False), [0], 0.7,
                                        weight=3.0)
    return cases


def _avar_as_general(prob):
    """AV@R_gamma at every node written out as general conic data (Sec. 3.3):
    E = [gamma I; -I; 1^T], no F, b = (p, 0, 1), K = R_+^{2k} x {0}."""
    parent = np.asarray(prob["parent"])
    p = np.asarray(prob["prob"], float)
    risk = []
    for i in range(int(parent.max()) + 1):
        kids = np.flatnonzero(parent == i)
        k, g = kids.size, float(prob["gamma"][i])
        E = np.vstack([g * np.eye(k), -np.eye(k), np.ones((1, k))])
        risk.append((E, None, np.concatenate([p[kids], np.zeros(k), [1.0]]),
                     np.concatenate([np.zeros(2 * k, int), [1]])))
    return dict(prob, risk=risk)


CASES = _cases()
# The networked-control instance is ill-conditioned beyond float64 (dynamics
# growing 150-fold per stage: cond(C C^T) of the dynamics constraint is 3e18),
# so two exact float64 evaluations of the S1 projection in the oracle itself
# (Alg. 2 and the dense KKT solve) differ by O(1) relative to the iterate
# scale (tests/test_oracle_pins.py); its operators L, L* and prox are compared
# (no Riccati recursion in them), its CP steps are not.
ILL_CONDITIONED = {"delay_m200"}
STEP_CASES = sorted(set(CASES) - ILL_CONDITIONED)


def _pair(name, precondition=True):
    prob = CASES[name]
    D = O.Data(prob, precondition=precondition)
    alpha = O.step_size(D)
    P = S.Problem(prob, S.default_settings(alpha=alpha, precondition=int(precondition)))
    P.set_x0(prob["x0"])
    return prob, D, alpha, P


def _rel(a, b, scale):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / scale)


@pytest.mark.parametrize("name", sorted(CASES))
def test_alpha_and_sizes_match_oracle(name):
    prob, D, alpha, P = _pair(name)
    with P:
        assert P.nz == D.layout.nz and P.neta == D.layout.neta
        # the library's own exact ||L|| (automatic alpha) against the oracle's
        Q = S.Problem(prob)
        assert Q.sizes["L_norm"] == pytest.approx(O.L_norm(D), rel=1e-12)
        assert Q.alpha == pytest.approx(alpha, rel=1e-12)
        Q.close()


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precondition", [True, False])
def test_L_Lt_prox_match_oracle(name, precondition):
    prob, D, alpha, P = _pair(name, precondition)
    rng = np.random.default_rng(5)
    with P:
        z = rng.standard_normal(P.nz) * 2
        e = rng.standard_normal(P.neta) * 2
        # relative to the larger of the input and output scales: dense cost
        # rows sum nx products of entries up to |Q^1/2| |x|
        Lz, Lte = O.apply_L(D, z), O.apply_Lt(D, e)
        sL, sLt = max(2.0, np.abs(Lz).max()), max(2.0, np.abs(Lte).max())
        assert _rel(P.apply_L(z), Lz, sL) < 1e-12
        assert _rel(P.apply_Lt(e), Lte, sLt) < 1e-12
        assert _rel(P.prox_gconj(e), O.prox_gconj(D, e, alpha), 2) < 1e-12
        # float32 kernels
        assert _rel(P.apply_L(z, S.FP32), Lz, sL) < 1e-5
        assert _rel(P.prox_gconj(e, S.FP32), O.prox_gconj(D, e, alpha), 2) < 1e-5


def _random_v(P, rng, scale=2.0):
    return rng.standard_normal(P.nz) * scale, rng.standard_normal(P.neta) * scale


@pytest.mark.parametrize("name", STEP_CASES)
@pytest.mark.parametrize("precondition", [True, False])
def test_T_step_matches_oracle(name, precondition):
    prob, D, alpha, P = _pair(name, precondition)
    F = O.Offline(D)
    rng = np.random.default_rng(17)
    with P:
        for trial in range(2):
            z, e = _random_v(P, rng)
            zo, eo = O.cp_step(D, F, z, e, alpha)
            x1, x2 = O.residuals(D, z, e, zo, eo, alpha)
            zg, eg, xi = P.apply_T(z, e)
            scale = max(1.0, np.abs(z).max(), np.abs(e).max(), np.abs(zo).max(), np.abs(eo).max())
            assert _rel(zg, zo, scale) < 1e-10, (trial, _rel(zg, zo, scale))
            assert _rel(eg, eo, scale) < 1e-10, (trial, _rel(eg, eo, scale))
            assert xi[0] == pytest.approx(np.abs(x1).max(), rel=1e-9)
            assert xi[1] == pytest.approx(np.abs(x2).max(), rel=1e-9)
            zf, ef, xif = P.apply_T(z, e, S.FP32)
            assert _rel(zf, zo, scale) < 2e-4
            assert _rel(ef, eo, scale) < 2e-4
            assert xif[0] == pytest.approx(np.abs(x1).max(), rel=1e-3, abs=1e-3 * scale / alpha)


def test_large_tree_step_matches_oracle():
    """The benchmark's own workload and launch configuration: one CP step of
    the large tree (7,167 nodes, nx = 50, nu = 25: backward products of 64 +
    16 rows with a second column block, forward products of 80 rows, the
    LDS-staged float32 sweeps and the float64 register sweeps, node
    workgroups of 256 threads) against the oracle, every entry, from two
    seeded random iterates."""
    prob = W.config_problem(2)
    D = O.Data(prob)
    F = O.Offline(D)
    alpha = O.step_size(D)
    rng = np.random.default_rng(23)
    with S.Problem(prob, S.default_settings(alpha=alpha)) as P:
        P.set_x0(prob["x0"])
        assert P.sizes["n"] == 7167 and P.sizes["nx"] == 50 and P.sizes["nu"] == 25
        for trial in range(2):
            z, e = _random_v(P, rng)
            zo, eo = O.cp_step(D, F, z, e, alpha)
            x1, x2 = O.residuals(D, z, e, zo, eo, alpha)
            scale = max(1.0, np.abs(z).max(), np.abs(e).max(), np.abs(zo).max(), np.abs(eo).max())
            zg, eg, xi = P.apply_T(z, e)
            assert _rel(zg, zo, scale) < 1e-10, (trial, _rel(zg, zo, scale))
            assert _rel(eg, eo, scale) < 1e-10, (trial, _rel(eg, eo, scale))
            assert xi[0] == pytest.approx(np.abs(x1).max(), rel=1e-9)
            assert xi[1] == pytest.approx(np.abs(x2).max(), rel=1e-9)
            zf, ef, _ = P.apply_T(z, e, S.FP32)
            print("large tree, trial %d: float64 %.2e %.2e, float32 %.2e %.2e" % (
                trial, _rel(zg, zo, scale), _rel(eg, eo, scale), _rel(zf, zo, scale), _rel(ef, eo, scale)))
            assert _rel(zf, zo, scale) < 2e-4, (trial, _rel(zf, zo, scale))
            assert _rel(ef, eo, scale) < 2e-4, (trial, _rel(ef, eo, scale))


@pytest.mark.parametrize("name", ["cfg0", "ragged_a", "wide"])
def test_prox_f_parts(name):
    """With eta = 0 the z part of T is prox_{alpha f}: S1 on (x, u) by Alg. 2,
    S2 on (y, tau, s) and s0 - alpha."""
    prob, D, alpha, P = _pair(name)
    F = O.Offline(D)
    rng = np.random.default_rng(3)
    with P:
        z = rng.standard_normal(P.nz) * 3
        zg, _, _ = P.apply_T(z, np.zeros(P.neta))
        zo = O.prox_f(D, F, z, alpha)
        assert _rel(zg, zo, 3) < 1e-11


@pytest.mark.parametrize("name,steps", [("cfg0", 200), ("cfg1", 60), ("ragged_affine", 100), ("m150", 40),
                                        ("m200", 20), ("linear_big", 60), ("edge_costs_lin", 60),
                                        ("dense_lin", 60), ("bench1", 40), ("general", 100),
                                        ("general_dense", 60), ("general_big", 30), ("spectral", 100),
                                        ("spectral_wide", 40), ("spectral_mixed", 60), ("avar_general", 60),
                                        ("soft", 100), ("l1", 100), ("l1_edge", 60), ("l2ball", 100),
                                        ("l2ball_63", 40)])
def test_trajectory_matches_oracle(name, steps):
    """K plain CP steps from zero: T is firmly nonexpansive, so differences
    cannot amplify along the trajectory."""
    prob, D, alpha, P = _pair(name)
    F = O.Offline(D)
    with P:
        z, e = np.zeros(P.nz), np.zeros(P.neta)
        zg, eg = z.copy(), e.copy()
        for _ in range(steps):
            z, e = O.cp_step(D, F, z, e, alpha)
        P.set_iterate(zg, eg)
        for _ in range(steps):
            zg, eg, _ = P.apply_T(zg, eg)
        scale = max(1.0, np.abs(z).max(), np.abs(e).max())
        assert _rel(zg, z, scale) < steps * 1e-11
        assert _rel(eg, e, scale) < steps * 1e-11


def test_config0_solution_matches_oracle():
    prob = CASES["cfg0"]
    ref = O.solve(prob, eps=1e-6, max_iters=20000)
    with S.Problem(prob, S.default_settings(eps=1e-6, check_every=2)) as P:
        info = P.solve(prob["x0"])
        assert info["code"] == S.SPOCK_OK and info["rel_res"] <= 1e-6
        x, u, s0 = P.solution()
        assert abs(s0 - ref["s0"]) <= 1e-6 * max(1, abs(ref["s0"])) * 10
        assert O.nested_cost(prob, x, u) == pytest.approx(s0, rel=1e-5)
        assert O.dynamics_violation(prob, x, u) < 1e-10
        # the iteration count agrees with the oracle's up to the check interval
        assert abs(info["iters"] - ref["iters"]) <= 2


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)) as f:
        return json.load(f)


def _sampled(snap, z, e):
    st = snap["z_idx_stride"]
    return np.asarray(z[::st]), np.asarray(e[::st]), np.asarray(snap["z"]), np.asarray(snap["eta"])


def test_medium_tree_solve_matches_oracle_golden():
    """The medium tree (229 nodes, nx = 20, nu = 10) solved in float64 to
    rel_res 1e-4 against the oracle's own run to the same tolerance
    (tests/golden/medium_tree_cp.json, written by make_medium_tree_golden.py
    from oracle/ alone).  With a check every 2 steps the GPU stops at the
    same iteration as the oracle (which checks every step), so V*, rel_res
    and the nested risk objective of the returned (x, u) are compared at
    the same iterate: T is nonexpansive, so after K steps the two
    trajectories differ by at most K rounding-sized steps (K 1e-12 relative).
    Plain CP does not reach rel_res 1e-6 on this tree in 3e5 steps; that
    tolerance is the accelerated (SuperMann) method's."""
    g = _golden("medium_tree_cp.json")
    prob = CASES["cfg1"]
    stop = g["stop"]
    K = stop["iters"]
    vs = stop["s0"]
    with S.Problem(prob, S.default_settings(alpha=g["alpha"], eps=g["eps"], max_iters=4 * K, check_every=2)) as P:
        info = P.solve(prob["x0"])
        print("medium tree: GPU iters %d rel_res %.6e s0 %.15g | oracle iters %d rel_res %.6e s0 %.15g" % (
            info["iters"], info["rel_res"], info["s0"], K, stop["rel_res"], vs))
        assert info["code"] == S.SPOCK_OK
        assert info["iters"] == K
        assert abs(info["s0"] - vs) <= 1e-10 * max(1.0, abs(vs))
        assert info["rel_res"] == pytest.approx(stop["rel_res"], rel=1e-8)
        x, u, s0 = P.solution()
        assert O.nested_cost(prob, x, u) == pytest.approx(stop["nested_cost"], rel=1e-9)
        assert O.dynamics_violation(prob, x, u) < 1e-9
        assert np.all(np.abs(x) <= 5 + 1e-3) and np.all(np.abs(u) <= 1 + 1e-3)
        # the trajectory at fixed step counts, every 97th entry
        for snap in g["snapshots"] + [g["final"]]:
            P.set_iterate(np.zeros(P.nz), np.zeros(P.neta))
            P.run_steps(snap["iters"])
            z, e = P.get_iterate()
            zg, eg, zo, eo = _sampled(snap, z, e)
            scale = max(1.0, snap["z_inf"], snap["eta_inf"])
            err = max(_rel(zg, zo, scale), _rel(eg, eo, scale))
            print("  K=%d: max sampled difference %.2e (bound %.1e)" % (snap["iters"], err, snap["iters"] * 1e-12))
            assert err <= snap["iters"] * 1e-12
            assert abs(z[0] - snap["s0"]) <= snap["iters"] * 1e-12 * max(1.0, abs(snap["s0"]))


@pytest.mark.parametrize("name", ["cfg0", "ragged_a"])
def test_mixed_precision_matches_oracle_vstar(name):
    """The mixed form (float32 steps, float64 check and refinement) at
    rel_res 1e-4 against the oracle's V* (plain CP to rel_res 1e-10 / 1e-7,
    tests/golden/tiny_tree_vstar.json): |s0 - V*| <= 10 eps max(1, |V*|).  An
    iterate at rel_res eps lies a few eps from V*: the oracle's own iterate at
    rel_res 1e-4 on the tiny tree is 3.3e-4 relative away (checked on the CPU
    in test_oracle_e2e.py), so 10 eps is the bar a solver at that tolerance
    meets."""
    g = _golden("tiny_tree_vstar.json")
    ref = g["tiny"][0] if name == "cfg0" else g["ragged_a"]
    vs = ref["vstar"]
    prob = CASES[name]
    with S.Problem(prob, S.default_settings(eps=1e-4, precision=S.MIXED)) as PM:
        rm = PM.solve(prob["x0"])
        assert rm["code"] == S.SPOCK_OK and rm["rel_res"] <= 1e-4
        assert rm["precision_used"] == S.FP64  # the accepted step is a float64 one
        x, u, sm = PM.solution()
    print("%s: mixed s0 %.10g, oracle V* %.10g, |diff|/max(1,|V*|) = %.2e (oracle at 1e-4: %.2e)" % (
        name, sm, vs, abs(sm - vs) / max(1.0, abs(vs)), abs(ref["at_1e-4"]["s0"] - vs) / max(1.0, abs(vs))))
    assert abs(sm - vs) <= 10 * 1e-4 * max(1.0, abs(vs))
    assert O.dynamics_violation(prob, x, u) < 1e-9


def test_large_tree_trajectory_matches_oracle():
    """50 plain CP steps from zero on the large tree (7,167 nodes, nx = 50,
    nu = 25) in float64 and in float32, every entry against the oracle.  T is
    nonexpansive, so a trajectory differs from the oracle's by at most the
    sum of the one-step differences: K 1e-12 (float64) and K 2e-4 (float32,
    the one-step bar) relative to the iterate scale."""
    prob = W.config_problem(2)
    D = O.Data(prob)
    F = O.Offline(D)
    alpha = O.step_size(D)
    K = 50
    z, e = np.zeros(D.layout.nz), np.zeros(D.layout.neta)
    for _ in range(K):
        z, e = O.cp_step(D, F, z, e, alpha)
    scale = max(1.0, np.abs(z).max(), np.abs(e).max())
    with S.Problem(prob, S.default_settings(alpha=alpha)) as P:
        P.set_x0(prob["x0"])
        errs = {}
        for prec, bound in ((S.FP64, 1e-12), (S.FP32, 2e-4)):
            P.set_iterate(np.zeros(P.nz), np.zeros(P.neta))
            P.run_steps(K, prec)
            zg, eg = P.get_iterate()
            errs[prec] = max(_rel(zg, z, scale), _rel(eg, e, scale))
            assert errs[prec] <= K * bound, (prec, errs[prec])
        print("large tree, %d steps: float64 %.2e, float32 %.2e relative" % (K, errs[S.FP64], errs[S.FP32]))


def test_large_tree_mixed_solution_error():
    """The benchmark's time-to-tolerance solve (mixed precision, rel_res 1e-4)
    against the plain float64 GPU solve to the same tolerance, and both
    against the oracle's invariants: the nested risk objective of the
    returned (x, u) equals s0 within 10 eps relative and the dynamics hold
    (the float64 trajectory is pinned to the oracle step by step in the
    tests above)."""
    prob = W.config_problem(2)
    eps = 1e-4
    out = {}
    for prec in (S.FP64, S.MIXED):
        with S.Problem(prob, S.default_settings(eps=eps, max_iters=100000, precision=prec)) as P:
            r = P.solve(prob["x0"])
            assert r["code"] == S.SPOCK_OK and r["rel_res"] <= eps, r
            x, u, s0 = P.solution()
            nc = O.nested_cost(prob, x, u)
            dv = O.dynamics_violation(prob, x, u)
            out[prec] = (s0, nc, dv, r["iters"])
            assert abs(nc - s0) <= 10 * eps * max(1.0, abs(s0)), (prec, nc, s0)
            assert dv < 1e-8
    s64, sm = out[S.FP64][0], out[S.MIXED][0]
    print("large tree at rel_res 1e-4: fp64 s0 %.10g (%d it), mixed s0 %.10g (%d it), |diff|/|s0| %.2e; "
          "nested-cost gaps %.2e / %.2e" % (s64, out[S.FP64][3], sm, out[S.MIXED][3], abs(sm - s64) / abs(s64),
                                            abs(out[S.FP64][1] - s64) / abs(s64), abs(out[S.MIXED][1] - sm) / abs(sm)))
    assert abs(sm - s64) <= 10 * eps * max(1.0, abs(s64))


def test_warm_start_and_iterate_roundtrip():
    prob = CASES["cfg0"]
    with S.Problem(prob, S.default_settings(eps=1e-6)) as P:
        a = P.solve(prob["x0"])
        z, e = P.get_iterate()
        b = P.solve(prob["x0"], warm_start=True)
        # already at the fixed point: done at the first check (one check interval)
        assert b["code"] == S.SPOCK_OK and b["iters"] <= P.settings.check_every
        assert b["s0"] == pytest.approx(a["s0"], rel=1e-6)
        P.set_iterate(z, e)
        z2, e2 = P.get_iterate()
        assert np.array_equal(z, z2) and np.array_equal(e, e2)
        assert a["code"] == S.SPOCK_OK


def test_infeasible_x0_and_not_converged():
    prob = CASES["cfg0"]
    with S.Problem(prob, S.default_settings(max_iters=10)) as P:
        with pytest.raises(S.SpockError) as e:
            P.solve(np.array([9.0, 0.0]))
        assert e.value.code == S.SPOCK_E_INFEASIBLE_X0
        r = P.solve(prob["x0"])
        assert r["code"] == S.SPOCK_E_NOT_CONVERGED and r["iters"] >= 10


def test_dense_cost_not_positive_definite_is_rejected():
    """A symmetric dense Q^j with a negative eigenvalue fails at setup with
    SPOCK_E_INVALID (Prop. 1 takes Q > 0); a positive definite one is taken."""
    prob = dict(CASES["dense"])
    Q = prob["Q"].copy()
    w, V = np.linalg.eigh(Q[2])
    Q[2] = (V * np.concatenate([[-0.5], w[1:]])) @ V.T
    Q[2] = 0.5 * (Q[2] + Q[2].T)
    with pytest.raises(S.SpockError) as e:
        S.Problem(dict(prob, Q=Q))
    assert e.value.code == S.SPOCK_E_INVALID and "positive definite" in str(e.value)
    with S.Problem(prob) as P:
        assert P.n == len(prob["parent"])


def test_torch_workspace_and_stream():
    """Device memory and the stream can come from PyTorch."""
    import torch
    prob = CASES["cfg0"]
    nbytes = S.footprint(prob)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    st = torch.cuda.Stream()
    with S.Problem(prob, workspace=ws, stream=st.cuda_stream) as P:
        r = P.solve(prob["x0"])
        assert r["code"] == S.SPOCK_OK
    with S.Problem(prob) as Q:
        r2 = Q.solve(prob["x0"])
    assert r["s0"] == r2["s0"] and r["iters"] == r2["iters"]


def test_run_to_run_bitwise_deterministic():
    prob = CASES["cfg1"]
    out = []
    for _ in range(2):
        with S.Problem(prob, S.default_settings(max_iters=200)) as P:
            P.solve(prob["x0"])
            out.append(P.get_iterate())
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("name", ["cfg0", "cfg1", "ragged_a", "ragged_affine", "wide", "very_wide", "big_nx",
                                  "deep_branched", "m200", "spectral", "spectral_wide", "avar_general", "l2ball",
                                  "l2ball_63"])
def test_project_S1_S2_hooks_match_oracle(name):
    """spock_project_S1 (Alg. 2 through the sweep kernels) against the oracle's
    Alg. 2 with P, and spock_project_S2 against the oracle's dense
    w - G^T (G G^T)^-1 G w, node by node, float64 at 1e-12 of the input scale
    and float32 at 2e-4."""
    prob, D, alpha, P = _pair(name)
    F = O.Offline(D)
    T, Y = D.tree, D.layout
    rng = np.random.default_rng(31)
    with P:
        xbar = rng.standard_normal((T.n, D.nx)) * 3
        ubar = rng.standard_normal((T.n_nl, D.nu)) * 3
        xo, uo = O.project_S1(D, F, xbar, ubar)
        scale = max(3.0, np.abs(xo).max(), np.abs(uo).max())
        xg, ug = P.project_S1(xbar, ubar)
        assert _rel(xg, xo, scale) < 1e-12 and _rel(ug, uo, scale) < 1e-12, (_rel(xg, xo, scale),
                                                                              _rel(ug, uo, scale))
        xf, uf = P.project_S1(xbar, ubar, S.FP32)
        assert _rel(xf, xo, scale) < 2e-4 and _rel(uf, uo, scale) < 2e-4
        ny = Y.yoff[-1]
        y = rng.standard_normal(ny) * 3
        tau = rng.standard_normal(T.n - 1) * 3
        s = rng.standard_normal(T.n - 1) * 3
        yg, tg, sg = P.project_S2(y, tau, s)
        yf, tf, sf = P.project_S2(y, tau, s, S.FP32)
        for i in T.nonleaf:
            kids = T.ch[i]
            w = np.concatenate([y[Y.yoff[i]:Y.yoff[i + 1]], tau[np.asarray(kids) - 1], s[np.asarray(kids) - 1]])
            E, Fm = D.risk[i][0], D.risk[i][1]  # AV@R's E when the node has no general risk
            pw = O.project_S2_block(w, D.gamma[i], len(kids), E, Fm)
            m = Y.ylen[i]
            got = np.concatenate([yg[Y.yoff[i]:Y.yoff[i + 1]], tg[np.asarray(kids) - 1], sg[np.asarray(kids) - 1]])
            gotf = np.concatenate([yf[Y.yoff[i]:Y.yoff[i + 1]], tf[np.asarray(kids) - 1], sf[np.asarray(kids) - 1]])
            assert got.size == pw.size and m + 2 * len(kids) == pw.size
            assert _rel(got, pw, 3.0) < 1e-12, (i, _rel(got, pw, 3.0))
            assert _rel(gotf, pw, 3.0) < 2e-4


@pytest.mark.parametrize("precision", [S.FP64, S.FP32])
def test_nonfinite_iterate_gives_nonfinite_residual(precision):
    """A NaN anywhere in the iterate reaches the residual maxima of Sec. 5.3
    (a plain max would drop it and report a converged solve)."""
    prob, D, alpha, P = _pair("ragged_a")
    rng = np.random.default_rng(41)
    with P:
        for where in ("z_x", "eta"):
            z, e = _random_v(P, rng)
            if where == "z_x":
                z[1 + 3 * D.nx + 1] = np.nan
            else:
                e[P.neta // 2] = np.nan
            _, _, xi = P.apply_T(z, e, precision)
            assert not np.all(np.isfinite(xi)), (where, xi)


@pytest.mark.parametrize("precision", [S.FP64, S.MIXED])
def test_nonfinite_iterate_solve_reports_diverged(precision):
    prob = CASES["ragged_a"]
    with S.Problem(prob, S.default_settings(eps=1e-4, precision=precision)) as P:
        r = P.solve(prob["x0"])
        assert r["code"] == S.SPOCK_OK
        z, e = P.get_iterate()
        z[5] = np.nan
        P.set_iterate(z, e)
        r = P.solve(prob["x0"], warm_start=True)
        assert r["code"] == S.SPOCK_E_DIVERGED, r
        assert not np.isfinite(r["rel_res"])


def test_setup_time_reported():
    prob = CASES["cfg1"]
    with S.Problem(prob, S.default_settings(max_iters=40)) as P:
        r = P.solve(prob["x0"])
        assert 0 < r["t_setup_s"] < 60 and r["t_solve_s"] > 0


@pytest.mark.parametrize("name", ["linear", "dense", "general", "spectral", "soft", "l1"])
def test_linear_cost_solution_matches_oracle(name):
    """A ragged tree with linear stage and terminal cost terms (and ones with
    dense per-edge costs, and with general constraint rows) solved in float64
    to rel_res 1e-6 against the oracle's solve and the nested risk objective
    with the same costs."""
    eps = 1e-6
    prob = CASES[name]
    ref = O.solve(prob, eps=eps, max_iters=60000)
    with S.Problem(prob, S.default_settings(alpha=ref["alpha"], eps=eps, max_iters=200000, check_every=2)) as P:
        r = P.solve(prob["x0"])
        x, u, s0 = P.solution()
        # the oracle's whole trajectory: the same number of steps from zero
        K = ref["iters"]
        P.set_iterate(np.zeros(P.nz), np.zeros(P.neta))
        P.run_steps(K)
        zg, eg = P.get_iterate()
    print("%s: GPU %d it s0 %.10g | oracle %d it s0 %.10g" % (name, r["iters"], s0, ref["iters"], ref["s0"]))
    assert r["code"] == S.SPOCK_OK and ref["status"] == "converged"
    assert abs(s0 - ref["s0"]) <= 10 * eps * max(1.0, abs(ref["s0"]))
    assert O.nested_cost(prob, x, u) == pytest.approx(s0, rel=10 * eps)
    # the residual of plain CP can alternate between even and odd steps, so the
    # two stopping iterations need not agree within the check interval; the
    # iterates at the oracle's stopping iteration do
    scale = max(1.0, np.abs(ref["z"]).max(), np.abs(ref["eta"]).max())
    assert _rel(zg, ref["z"], scale) <= K * 1e-12 and _rel(eg, ref["eta"], scale) <= K * 1e-12


def test_avar_as_general_risk_matches_avar_path():
    """AV@R given as general conic data runs the general-risk code (the node
    kernels built with the general products, the S2 multiplier through
    (G G^T)^-1 instead of the closed form): its iterates after 60 CP steps
    equal those of the AV@R path to rounding, in float64 and float32."""
    prob = CASES["avar_general"]
    base = {k: v for k, v in prob.items() if k != "risk"}
    for prec, tol in ((S.FP64, 1e-12), (S.FP32, 1e-5)):
        out = []
        for p in (base, prob):
            with S.Problem(p) as P:
                P.set_x0(p["x0"])
                P.run_steps(60, prec)
                out.append(P.get_iterate())
        scale = max(1.0, np.abs(out[0][0]).max(), np.abs(out[0][1]).max())
        assert _rel(out[1][0], out[0][0], scale) < tol and _rel(out[1][1], out[0][1], scale) < tol


def test_soft_state_bounds_slacks():
    """Soft state bounds (slack inputs theta with rows theta >= 0 and
    x_0 - theta <= 0.7): the float64 solve's slacks equal max(0, x_0 - 0.7)
    at every non-leaf node, and the bound is exceeded somewhere."""
    prob = CASES["soft"]
    nu0 = prob["nu"] - 1
    with S.Problem(prob, S.default_settings(eps=1e-7, max_iters=200000, check_every=2)) as P:
        r = P.solve(prob["x0"])
        x, u, s0 = P.solution()
    assert r["code"] == S.SPOCK_OK
    nl = u.shape[0]
    pen = np.maximum(0.0, x[:nl, 0] - 0.7)
    assert np.abs(u[:, nu0] - pen).max() <= 1e-3 * max(1.0, np.abs(x).max())
    assert pen.max() > 1e-2


def test_l2_ball_risk_solution_matches_oracle():
    """The l2-ball risk (a second-order cone in K) solved in float64 to
    rel_res 1e-6: the optimal value against the oracle's solve, and the
    iterates at the oracle's stopping iteration against its trajectory."""
    eps = 1e-6
    prob = CASES["l2ball"]
    ref = O.solve(prob, eps=eps, max_iters=60000)
    with S.Problem(prob, S.default_settings(alpha=ref["alpha"], eps=eps, max_iters=200000, check_every=2)) as P:
        r = P.solve(prob["x0"])
        _, _, s0 = P.solution()
        K = ref["iters"]
        P.set_iterate(np.zeros(P.nz), np.zeros(P.neta))
        P.run_steps(K)
        zg, eg = P.get_iterate()
    print("l2ball: GPU %d it s0 %.10g | oracle %d it s0 %.10g" % (r["iters"], s0, ref["iters"], ref["s0"]))
    assert r["code"] == S.SPOCK_OK and ref["status"] == "converged"
    assert abs(s0 - ref["s0"]) <= 10 * eps * max(1.0, abs(ref["s0"]))
    scale = max(1.0, np.abs(ref["z"]).max(), np.abs(ref["eta"]).max())
    assert _rel(zg, ref["z"], scale) <= K * 1e-12 and _rel(eg, ref["eta"], scale) <= K * 1e-12
