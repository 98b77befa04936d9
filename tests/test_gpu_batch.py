"""Batched form: uneven trees in one launch give each member the result it
gets alone (bitwise: the same kernels run the same per-node arithmetic), and
a failing member does not disturb the others."""
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


def _members():
    probs = [W.config_problem(0), W.random_ragged_problem(5, N=4, nx=4, nu=2, max_children=3),
             W.random_ragged_problem(6, N=3, nx=6, nu=3, max_children=4, affine=True)]
    probs += [W.batch_problem(k) for k in range(5)]
    return probs


@pytest.mark.parametrize("precision,eps", [(S.FP64, 1e-5), (S.MIXED, 1e-4)])
def test_batch_equals_alone(precision, eps):
    probs = _members()
    settings = dict(eps=eps, max_iters=60000, precision=precision)
    alone = []
    for p in probs:
        with S.Problem(p, S.default_settings(**settings)) as P:
            info = P.solve(p["x0"])
            alone.append((info, P.solution()))
    handles = [S.Problem(p, S.default_settings(**settings)) for p in probs]
    with S.Batch(handles, S.default_settings(**settings)) as B:
        infos = B.solve([p["x0"] for p in probs])
    for k, (p, h) in enumerate(zip(probs, handles)):
        a_info, (ax, au, as0) = alone[k]
        b_info = infos[k]
        assert b_info["status"] == a_info["code"], (k, b_info, a_info)
        assert b_info["iters"] == a_info["iters"], (k, b_info["iters"], a_info["iters"])
        x, u, s0 = h.solution()
        assert np.array_equal(x, ax) and np.array_equal(u, au) and s0 == as0, k
        if b_info["status"] == S.SPOCK_OK:
            assert O.nested_cost(p, x, u) == pytest.approx(s0, rel=50 * eps)
        h.close()


def test_batch_member_failure_is_isolated():
    probs = _members()[:4]
    handles = [S.Problem(p, S.default_settings(eps=1e-5)) for p in probs]
    x0s = [p["x0"] for p in probs]
    x0s[1] = np.full_like(x0s[1], 100.0)  # outside the root box
    with S.Batch(handles, S.default_settings(eps=1e-5, max_iters=60000)) as B:
        infos = B.solve(x0s)
    assert infos[1]["status"] == S.SPOCK_E_INFEASIBLE_X0
    for k in (0, 2, 3):
        assert infos[k]["status"] == S.SPOCK_OK, infos[k]
        with S.Problem(probs[k], S.default_settings(eps=1e-5)) as P:
            P.solve(probs[k]["x0"])
            assert np.array_equal(P.solution()[0], handles[k].solution()[0])
    for h in handles:
        h.close()


def test_batch_warm_start_after_shift():
    """MPC use: the next request shifts x0 and warm-starts from the resident
    iterate; the warm result equals a cold solve of the shifted problem up to
    the tolerance and takes fewer steps."""
    probs = _members()[:3]
    handles = [S.Problem(p, S.default_settings(eps=1e-5)) for p in probs]
    with S.Batch(handles, S.default_settings(eps=1e-5, max_iters=60000)) as B:
        cold = B.solve([p["x0"] for p in probs])
        x1 = [0.9 * p["x0"] for p in probs]
        warm = B.solve(x1, warm=[1] * len(probs))
    for k, p in enumerate(probs):
        assert warm[k]["status"] == S.SPOCK_OK
        q = dict(p)
        q["x0"] = x1[k]
        with S.Problem(q, S.default_settings(eps=1e-5)) as P:
            ref = P.solve(q["x0"])
        assert warm[k]["s0"] == pytest.approx(ref["s0"], rel=1e-3)
        assert warm[k]["iters"] <= cold[k]["iters"] + 20
    for h in handles:
        h.close()


@pytest.mark.parametrize("wg", [64, 128, 512])
def test_workgroup_sizes_match_oracle(wg):
    """Every launch size the autotuner may pick computes the same CP step."""
    for p in (W.config_problem(1), W.batch_problem(3), W.random_ragged_problem(8, N=3, nx=5, nu=2)):
        D = O.Data(p)
        F = O.Offline(D)
        a = O.step_size(D)
        rng = np.random.default_rng(wg)
        with S.Problem(p, S.default_settings(alpha=a)) as P:
            P.set_x0(p["x0"])
            P.set_launch(wg, S.FP64)
            P.set_launch(wg, S.FP32)
            z, e = rng.standard_normal(P.nz), rng.standard_normal(P.neta)
            zo, eo = O.cp_step(D, F, z, e, a)
            zg, eg, _ = P.apply_T(z, e)
            sc = max(1.0, np.abs(zo).max(), np.abs(eo).max(), np.abs(z).max(), np.abs(e).max())
            assert np.abs(zg - zo).max() / sc < 1e-10 and np.abs(eg - eo).max() / sc < 1e-10
            zf, ef, _ = P.apply_T(z, e, S.FP32)
            assert np.abs(zf - zo).max() / sc < 2e-4 and np.abs(ef - eo).max() / sc < 2e-4


def test_autotuner_picks_a_candidate(tmp_path):
    from paper_2505_12078_amd import tune
    p = W.batch_problem(2)
    with S.Problem(p) as P:
        P.set_x0(p["x0"])
        best, times = tune.tune_problem(P, S.FP32, steps=6, cache_path=str(tmp_path / "t.json"))
        assert best in tune.CANDIDATES and best == min(times, key=times.get)
        assert P.get_launch(S.FP32) == best
        again, _ = tune.tune_problem(P, S.FP32, cache_path=str(tmp_path / "t.json"))
        assert again == best
        P.set_settings(eps=1e-4)
        assert P.solve(p["x0"])["code"] == S.SPOCK_OK


def test_batched_workload_launch_equals_alone_and_oracle():
    """The batched workload's first 40 members (nx 4..32, up to 14,677 nodes,
    54,373 in all) in the launch configuration the benchmark's autotuner picks
    (256-thread node workgroups): after batched steps every member's iterate is
    bitwise the one its own steps give, in both precisions, and the two
    smallest members match the oracle's CP steps from zero."""
    probs = [W.batch_problem(k) for k in range(40)]
    small = sorted(range(len(probs)), key=lambda k: len(probs[k]["parent"]))[:2]
    data = {k: O.Data(probs[k]) for k in small}
    alphas = {k: O.step_size(data[k]) for k in small}

    def handle(k):
        P = S.Problem(probs[k], S.default_settings(alpha=alphas.get(k, 0.0)))
        P.set_x0(probs[k]["x0"])
        return P

    for prec, steps in ((S.FP64, 2), (S.FP32, 4)):
        alone = []
        for k in range(len(probs)):
            with handle(k) as P:
                P.set_launch(256, prec)
                P.run_steps(steps, prec)
                alone.append(P.get_iterate())
        hs = [handle(k) for k in range(len(probs))]
        with S.Batch(hs, S.default_settings()) as B:
            B.set_launch(256, prec)
            B.run_steps(steps, prec)
        for k, h in enumerate(hs):
            z, e = h.get_iterate()
            h.close()
            assert np.array_equal(z, alone[k][0]) and np.array_equal(e, alone[k][1]), (prec, k)
            if k in small:
                D = data[k]
                F = O.Offline(D)
                zo, eo = np.zeros(D.layout.nz), np.zeros(D.layout.neta)
                for _ in range(steps):
                    zo, eo = O.cp_step(D, F, zo, eo, alphas[k])
                scale = max(1.0, np.abs(zo).max(), np.abs(eo).max())
                tol = 1e-10 if prec == S.FP64 else 2e-4
                err = max(np.abs(z - zo).max(), np.abs(e - eo).max()) / scale
                print("member %d (%d nodes) %s: max error / scale %.2e" % (k, len(probs[k]["parent"]),
                      "f64" if prec == S.FP64 else "f32", err), flush=True)
                assert err < tol, (prec, k, err)


def test_batch_with_dense_and_general_members():
    """A batch that mixes plain members with one carrying dense costs, one
    carrying general constraint rows and one with an l1 input penalty runs
    the node kernels built with those products for every member: after
    float64 and float32 steps each member's iterate matches its own steps (the
    same operations in the same order; the other kernel build may fuse
    differently, so to rounding), and the general member matches the oracle."""
    probs = [W.config_problem(0), W.random_ragged_problem(5, N=3, nx=3, nu=2, dense_costs=True),
             W.random_ragged_problem(7, N=3, nx=3, nu=2, general_con=True), W.batch_problem(1),
             W.l1_input_penalty(W.random_ragged_problem(7, N=2, nx=3, nu=2, ball=False), 2.0)]
    D = O.Data(probs[2])
    alpha = O.step_size(D)

    def handle(k):
        P = S.Problem(probs[k], S.default_settings(alpha=alpha if k == 2 else 0.0))
        P.set_x0(probs[k]["x0"])
        return P

    for prec, steps, tol in ((S.FP64, 4, 1e-12), (S.FP32, 4, 1e-5)):
        alone = []
        for k in range(len(probs)):
            with handle(k) as P:
                P.run_steps(steps, prec)
                alone.append(P.get_iterate())
        hs = [handle(k) for k in range(len(probs))]
        with S.Batch(hs, S.default_settings()) as B:
            B.run_steps(steps, prec)
        for k, h in enumerate(hs):
            z, e = h.get_iterate()
            h.close()
            scale = max(1.0, np.abs(alone[k][0]).max(), np.abs(alone[k][1]).max())
            err = max(np.abs(z - alone[k][0]).max(), np.abs(e - alone[k][1]).max()) / scale
            assert err <= tol, (prec, k, err)
        F = O.Offline(D)
        zo, eo = np.zeros(D.layout.nz), np.zeros(D.layout.neta)
        for _ in range(steps):
            zo, eo = O.cp_step(D, F, zo, eo, alpha)
        z2 = alone[2]
        scale = max(1.0, np.abs(zo).max(), np.abs(eo).max())
        err = max(np.abs(z2[0] - zo).max(), np.abs(z2[1] - eo).max()) / scale
        assert err < (1e-10 if prec == S.FP64 else 2e-4), (prec, err)
