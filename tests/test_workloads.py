"""The seeded input generator (no GPU): the dynamics draws keep the node-by-node
order A^1, B^1, A^2, B^2, ... whichever path computes the spectral radii."""
import numpy as np

from paper_2505_12078_amd import workloads as W


def _node_by_node(seed, n, nx, nu):
    rng = np.random.default_rng(seed)
    A = np.zeros((n, nx, nx))
    B = np.zeros((n, nx, nu))
    for j in range(1, n):
        while True:
            G = rng.standard_normal((nx, nx))
            rho = np.max(np.abs(np.linalg.eigvals(G)))
            if rho >= 1e-3:
                A[j] = 0.95 * G / rho
                break
        B[j] = rng.standard_normal((nx, nu))
    return A, B, rng.standard_normal(3)


def test_dynamics_draws_match_node_by_node_order():
    for seed, n, nx, nu in ((1, 15, 2, 1), (2, 40, 7, 3), (3, 1, 4, 2), (4, 2, 1, 1)):
        A0, B0, tail0 = _node_by_node(seed, n, nx, nu)
        rng = np.random.default_rng(seed)
        A, B = W._draw_dynamics(rng, n, nx, nu)
        assert A.tobytes() == A0.tobytes() and B.tobytes() == B0.tobytes()
        # the generator is left where the node-by-node draws leave it
        assert rng.standard_normal(3).tobytes() == tail0.tobytes()


def test_redraw_path_replays_from_the_same_state(monkeypatch):
    # force the stacked radii below the redraw threshold: the node-by-node
    # replay must give exactly the plain order's result
    real = np.linalg.eigvals
    calls = {"stacked": 0}

    def fake(a):
        a = np.asarray(a)
        if a.ndim == 3:
            calls["stacked"] += 1
            return np.zeros(a.shape[:2])
        return real(a)

    A0, B0, tail0 = _node_by_node(5, 20, 3, 2)
    monkeypatch.setattr(W.np.linalg, "eigvals", fake)
    rng = np.random.default_rng(5)
    A, B = W._draw_dynamics(rng, 20, 3, 2)
    assert calls["stacked"] == 1
    assert A.tobytes() == A0.tobytes() and B.tobytes() == B0.tobytes()
    assert rng.standard_normal(3).tobytes() == tail0.tobytes()
