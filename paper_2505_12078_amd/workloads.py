"""Seeded synthetic scenario-tree problems shaped like the paper's workloads.

This module only draws data: trees, conditional probabilities, dynamics,
costs, bounds, risk parameters and initial states.  It holds none of the
method's arithmetic (no projections, no factorisations, no operator L), so
both the FP64 oracle and the HIP path can take their inputs from it.

A problem is a plain dict of NumPy arrays (the "problem description"):

    parent   int32[n]      parent[0] = -1, nodes numbered stage by stage
                           (breadth first), so children of a node are
                           contiguous and every leaf sits at stage N
    prob     float64[n]    conditional probability of a node given its
                           parent (siblings sum to 1), prob[0] = 1
    nx, nu   int           state / input sizes
    A        float64[n,nx,nx]  x^i = A^i x^anc(i) + B^i u^anc(i) + c^i
    B        float64[n,nx,nu]  (entry 0 unused)
    c        float64[n,nx] or None
    Q, R     float64[nx], float64[nu]   diagonal of the edge stage cost
             (or [n,nx], [n,nu]: row j for the edge into node j)
    QN       float64[nx]   diagonal of the leaf cost (or [n,nx]: leaf rows)
    q, r, qN float64[n,nx], [n,nu], [n,nx] (optional) linear cost terms:
                           q^j, r^j on x, u of the parent in the edge into j,
                           qN^j at leaf j
    x_lo, x_hi, u_lo, u_hi, xN_lo, xN_hi   box bounds
    x_ball, xN_ball        Euclidean-ball radius on x (<= 0: none)
    gamma    float64[n_nl] AV@R parameter per non-leaf node
    x0       float64[nx]   initial state

The problem formulation is the scenario-tree RAOCP of the paper's problem
statement section (dynamics, constraints, quadratic costs, AV@R risk).
"""
from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------------------
# trees
# ----------------------------------------------------------------------------


def tree_from_child_counts(counts_by_stage):
    """Breadth-first parent array from per-node child counts.

    ``counts_by_stage[t]`` lists the number of children of each node of stage
    ``t`` in node order.  Returns (parent int32[n], stage int32[n]).
    """
    parent = [-1]
    stage = [0]
    frontier = [0]
    for t, counts in enumerate(counts_by_stage):
        if len(counts) != len(frontier):
            raise ValueError("stage %d: %d counts for %d nodes" % (t, len(counts), len(frontier)))
        nxt = []
        for node, k in zip(frontier, counts):
            if k < 1:
                raise ValueError("every non-leaf node needs at least one child")
            for _ in range(int(k)):
                parent.append(node)
                stage.append(t + 1)
                nxt.append(len(parent) - 1)
        frontier = nxt
    return np.asarray(parent, dtype=np.int32), np.asarray(stage, dtype=np.int32)


def tree_from_branching(branching):
    """Uniform stage branching: ``branching[t]`` children for every node of stage t."""
    counts = []
    width = 1
    for b in branching:
        counts.append([int(b)] * width)
        width *= int(b)
    return tree_from_child_counts(counts)


def children_lists(parent):
    n = len(parent)
    ch = [[] for _ in range(n)]
    for j in range(1, n):
        ch[int(parent[j])].append(j)
    return ch


def draw_cond_probs(parent, rng, kind):
    """Conditional child probabilities, drawn stage-major (node order)."""
    n = len(parent)
    prob = np.zeros(n)
    prob[0] = 1.0
    for i, kids in enumerate(children_lists(parent)):
        if not kids:
            continue
        k = len(kids)
        if kind == "uniform" or k == 1:
            p = np.full(k, 1.0 / k)
        elif kind == "dirichlet":
            p = rng.dirichlet(np.ones(k))
            p = np.maximum(p, 1e-6)
            p /= p.sum()
        else:
            raise ValueError(kind)
        prob[kids] = p
    return prob


# ----------------------------------------------------------------------------
# data
# ----------------------------------------------------------------------------


def _stable_gaussian(rng, nx, radius=0.95):
    while True:
        G = rng.standard_normal((nx, nx))
        rho = np.max(np.abs(np.linalg.eigvals(G)))
        if rho >= 1e-3:
            return radius * G / rho


def _draw_dynamics(rng, n, nx, nu):
    """A^j (scaled to spectral radius 0.95) then B^j for j = 1..n-1, in that
    order.  The spectral radii are computed for all nodes at once; if any draw
    would be redrawn, the draws are replayed node by node from the same state,
    so the result is always that of the node-by-node order."""
    A = np.zeros((n, nx, nx))
    B = np.zeros((n, nx, nu))
    if n <= 1:
        return A, B
    state = rng.bit_generator.state
    for j in range(1, n):
        A[j] = rng.standard_normal((nx, nx))
        B[j] = rng.standard_normal((nx, nu))
    rho = np.max(np.abs(np.linalg.eigvals(A[1:])), axis=1)
    if np.all(rho >= 1e-3):
        A[1:] = 0.95 * A[1:] / rho[:, None, None]
        return A, B
    rng.bit_generator.state = state
    for j in range(1, n):
        A[j] = _stable_gaussian(rng, nx)
        B[j] = rng.standard_normal((nx, nu))
    return A, B


def _guard_x0(x0, parent, A, x_hi, x_ball, xN_hi, xN_ball, n_nl, margin=0.9):
    """Halve x0 until the zero-input rollout keeps a margin inside every box/ball.

    This keeps the drawn instance strictly feasible (Slater), so the conic
    problem has a solution.  Pure simulation of the dynamics, no solver.
    """
    n = len(parent)
    for _ in range(80):
        xs = np.zeros((n, x0.size))
        xs[0] = x0
        ok = True
        for j in range(n):
            if j > 0:
                xs[j] = A[j] @ xs[int(parent[j])]
            hi = x_hi if j < n_nl else xN_hi
            ball = x_ball if j < n_nl else xN_ball
            if np.any(np.abs(xs[j]) > margin * hi):
                ok = False
                break
            if ball > 0 and np.linalg.norm(xs[j]) > margin * ball:
                ok = False
                break
        if ok:
            return x0
        x0 = 0.5 * x0
    raise RuntimeError("could not find a strictly feasible x0")


def make_problem(parent, nx, nu, rng, *, prob_kind="uniform", gamma=0.95,
                 x_box=5.0, u_box=1.0, x_ball=0.0, q=1.0, r=0.1, qn=1.0,
                 affine=False, linear=False, edge_costs=False, dense_costs=False, general_con=False,
                 x0_range=2.0, name="custom"):
    """Draw a full problem on the given tree (draw order: probabilities, then
    A^i and B^i for i = 1..n-1, then x0, then the optional affine terms, then
    the optional linear cost terms q^j, r^j of the edge into j and qN^j of
    leaf j, each N(0, 0.25)), then the optional per-edge and per-leaf cost
    diagonals Q^j = q u, R^j = r u, Q_N^j = qn u with u ~ U[0.5, 2] entrywise),
    then the optional dense per-edge and per-leaf costs
    Q^j = q (I / 2 + W W^T / (2 nx)) with W ~ N(0, 1) entrywise (R^j, Q_N^j alike),
    then the optional general constraints: the box rows of x and u plus
    max(1, nx / 2) coupling rows W_x x + W_u u (entries N(0, 1/nx), N(0, 1/nu))
    at non-leaf nodes and the box rows of x plus as many rows W_N x at leaves,
    each coupling row bounded by +-(1.5 c + 0.5), c its largest magnitude along
    the zero-input rollout from x0 (so the instance stays strictly feasible);
    no ball then."""
    parent = np.asarray(parent, dtype=np.int32)
    n = len(parent)
    n_nl = int(np.sum(np.bincount(parent[1:], minlength=n) > 0))
    prob = draw_cond_probs(parent, rng, prob_kind)
    A, B = _draw_dynamics(rng, n, nx, nu)
    x0 = rng.uniform(-x0_range, x0_range, size=nx)
    c = None
    if affine:
        c = np.zeros((n, nx))
        c[1:] = 0.05 * rng.standard_normal((n - 1, nx))
    x_hi = np.full(nx, float(x_box))
    u_hi = np.full(nu, float(u_box))
    x0 = _guard_x0(x0, parent, A, x_hi, x_ball, x_hi, x_ball, n_nl)
    if np.isscalar(gamma):
        gamma = np.full(n_nl, float(gamma))
    lin = {}
    if linear:
        lin["q"] = 0.5 * rng.standard_normal((n, nx))
        lin["r"] = 0.5 * rng.standard_normal((n, nu))
        lin["qN"] = 0.5 * rng.standard_normal((n, nx))
        for v in lin.values():
            v[0] = 0.0  # node 0 owns no edge and is not a leaf
    Qc, Rc, QNc = np.full(nx, float(q)), np.full(nu, float(r)), np.full(nx, float(qn))
    if edge_costs:
        Qc = float(q) * rng.uniform(0.5, 2.0, size=(n, nx))
        Rc = float(r) * rng.uniform(0.5, 2.0, size=(n, nu))
        QNc = float(qn) * rng.uniform(0.5, 2.0, size=(n, nx))
    if dense_costs:
        def spd(scale, d):
            W = rng.standard_normal((n, d, d))
            return float(scale) * (0.5 * np.eye(d)[None] + np.einsum("nij,nkj->nik", W, W) / (2.0 * d))
        Qc, Rc, QNc = spd(q, nx), spd(r, nu), spd(qn, nx)
    gen = {}
    if general_con:
        ncx = max(1, nx // 2)
        Wx = rng.standard_normal((ncx, nx)) / np.sqrt(nx)
        Wu = rng.standard_normal((ncx, nu)) / np.sqrt(nu)
        WN = rng.standard_normal((ncx, nx)) / np.sqrt(nx)
        xs = np.zeros((n, nx))
        xs[0] = x0
        for j in range(1, n):
            xs[j] = A[j] @ xs[int(parent[j])] + (c[j] if c is not None else 0.0)
        cb = 1.5 * np.abs(xs[:n_nl] @ Wx.T).max(axis=0) + 0.5
        cbN = 1.5 * np.abs(xs[n_nl:] @ WN.T).max(axis=0) + 0.5
        gen = dict(Gamma_x=np.vstack([np.eye(nx), np.zeros((nu, nx)), Wx]),
                   Gamma_u=np.vstack([np.zeros((nx, nu)), np.eye(nu), Wu]),
                   c_lo=np.concatenate([-x_hi, -u_hi, -cb]), c_hi=np.concatenate([x_hi, u_hi, cb]),
                   Gamma_N=np.vstack([np.eye(nx), WN]),
                   cN_lo=np.concatenate([-x_hi, -cbN]), cN_hi=np.concatenate([x_hi, cbN]))
        x_ball = 0.0
    return dict(
        **lin, **gen,
        name=name, parent=parent, prob=prob, nx=int(nx), nu=int(nu), A=A, B=B, c=c,
        Q=Qc, R=Rc, QN=QNc,
        x_lo=-x_hi.copy(), x_hi=x_hi.copy(), u_lo=-u_hi.copy(), u_hi=u_hi.copy(),
        xN_lo=-x_hi.copy(), xN_hi=x_hi.copy(),
        x_ball=float(x_ball), xN_ball=float(x_ball),
        gamma=np.asarray(gamma, dtype=np.float64), x0=x0,
    )


def spectral_risk(prob, weight=0.5, gammas=(0.2, 0.9)):
    """The problem with every non-leaf node's risk replaced by the spectral
    risk weight AV@R_g1 + (1 - weight) AV@R_g2 of its children's costs, as
    general conic data (E, F, b, cone) per node: mu = weight mu1 + (1 - weight)
    mu2 (k rows in {0}), b_l - E_l mu_l in K_l for the two AV@R blocks
    (E_l = [g_l I; -I; 1^T], b_l = (p, 0, 1), K_l = R_+^{2k} x {0}), with
    nu = (mu1, mu2); cone code 0: R_+, 1: {0}."""
    parent = np.asarray(prob["parent"])
    n = len(parent)
    kids = children_lists(parent)
    p_all = np.asarray(prob["prob"], float)
    risk = []
    for i in range(n):
        k = len(kids[i])
        if k == 0:
            break
        p = p_all[kids[i]]
        blocks_E, blocks_F, blocks_b, cones = [np.eye(k)], [np.hstack([-weight * np.eye(k),
                                                                      -(1.0 - weight) * np.eye(k)])], \
            [np.zeros(k)], [np.ones(k, int)]
        for l, g in enumerate(gammas):
            El = np.vstack([g * np.eye(k), -np.eye(k), np.ones((1, k))])
            Fl = np.zeros((2 * k + 1, 2 * k))
            Fl[:, l * k:(l + 1) * k] = El
            blocks_E.append(np.zeros((2 * k + 1, k)))
            blocks_F.append(Fl)
            blocks_b.append(np.concatenate([p, np.zeros(k), [1.0]]))
            cones.append(np.concatenate([np.zeros(2 * k, int), [1]]))
        risk.append((np.vstack(blocks_E), np.vstack(blocks_F), np.concatenate(blocks_b), np.concatenate(cones)))
    return dict(prob, risk=risk, name=prob.get("name", "custom") + "_spectral")


def l2_ball_risk(prob, r_frac=0.5):
    """The problem with every non-leaf node's risk replaced by the worst
    expectation over the probability vectors within Euclidean distance
    r = r_frac * min(p) of the node's conditional probabilities p, as
    conic data with a second-order cone (Sec. 3.3): mu >= 0 (k rows, R_+),
    1^T mu = 1 (one row, {0}) and (r, mu - p) in SOC_{k+1} (a head row,
    code 2, and k tail rows, code 3); no nu.  With r <= min(p) the ball lies
    in the simplex and the risk is p^T Z + r ||Z - mean(Z) 1||."""
    parent = np.asarray(prob["parent"])
    kids = children_lists(parent)
    p_all = np.asarray(prob["prob"], float)
    risk = []
    for i in range(len(parent)):
        k = len(kids[i])
        if k == 0:
            break
        p = p_all[kids[i]]
        r = float(r_frac) * float(p.min())
        E = np.vstack([-np.eye(k), np.ones((1, k)), np.zeros((1, k)), -np.eye(k)])
        b = np.concatenate([np.zeros(k), [1.0], [r], -p])
        cone = np.concatenate([np.zeros(k, int), [1, 2], np.full(k, 3)])
        risk.append((E, None, b, cone))
    return dict(prob, risk=risk, name=prob.get("name", "custom") + "_l2ball")


def soft_state_bounds(prob, idx, x_max, weight=1.0):
    """The problem with the hard upper bounds of the state components idx at
    non-leaf nodes replaced by the quadratic penalty weight *
    ||max(0, x_idx - x_max)||^2 in the stage cost (the soft constraints that
    follow Prop. 2 of Sec. 4.2), written with the paper's relaxation: one slack
    input theta per component (u' = (u, theta), no effect on the dynamics,
    cost weight * theta^T theta on every edge) and the constraint rows
    theta >= 0, x_idx - theta <= x_max, as general rows Gamma_x x + Gamma_u u'
    in a box.  The box of x (other components, and the lower bounds of idx)
    and of u stay as rows; leaves keep their hard bounds.  No ball on x."""
    if float(prob.get("x_ball", 0.0)) > 0 or prob.get("Gamma_x") is not None:
        raise ValueError("soft_state_bounds takes a problem with box constraints only")
    idx = np.asarray(idx, dtype=int)
    x_max = np.broadcast_to(np.asarray(x_max, float), idx.shape)
    nx, nu, ns = int(prob["nx"]), int(prob["nu"]), idx.size
    n = len(prob["parent"])
    nu2 = nu + ns
    B = np.concatenate([np.asarray(prob["B"], float), np.zeros((n, nx, ns))], axis=2)
    R = np.asarray(prob["R"], float)
    w = float(weight)
    if R.ndim == 1:
        R2 = np.concatenate([R, np.full(ns, w)])
    elif R.ndim == 2:
        R2 = np.concatenate([R, np.full((n, ns), w)], axis=1)
    else:
        R2 = np.zeros((n, nu2, nu2))
        R2[:, :nu, :nu] = R
        R2[:, nu:, nu:] = w * np.eye(ns)
    hard_hi = np.asarray(prob["x_hi"], float).copy()
    hard_hi[idx] = np.inf
    Ex = np.zeros((ns, nx))
    Ex[np.arange(ns), idx] = 1.0
    Gx = np.vstack([np.eye(nx), np.zeros((nu, nx)), np.zeros((ns, nx)), Ex])
    Gu = np.vstack([np.zeros((nx, nu2)), np.hstack([np.eye(nu), np.zeros((nu, ns))]),
                    np.hstack([np.zeros((ns, nu)), np.eye(ns)]), np.hstack([np.zeros((ns, nu)), -np.eye(ns)])])
    c_lo = np.concatenate([prob["x_lo"], prob["u_lo"], np.zeros(ns), np.full(ns, -np.inf)])
    c_hi = np.concatenate([hard_hi, prob["u_hi"], np.full(ns, np.inf), x_max])
    out = dict(prob, nu=nu2, B=B, R=R2, Gamma_x=Gx, Gamma_u=Gu, c_lo=c_lo, c_hi=c_hi,
               Gamma_N=np.eye(nx), cN_lo=np.asarray(prob["xN_lo"], float), cN_hi=np.asarray(prob["xN_hi"], float),
               u_lo=np.concatenate([prob["u_lo"], np.zeros(ns)]), u_hi=np.concatenate([prob["u_hi"], np.full(ns, np.inf)]),
               name=prob.get("name", "custom") + "_soft")
    if prob.get("r") is not None:
        out["r"] = np.concatenate([np.asarray(prob["r"], float), np.zeros((n, ns))], axis=1)
    return out


def l1_input_penalty(prob, lam0):
    """The problem with lam0 * ||u||_1 added to every stage cost (Prop. 2 of
    Sec. 4.2, on the inputs), written as the proposition does: slack inputs
    lambda (one per input) and theta, u' = (u, lambda, theta), no effect on
    the dynamics and no quadratic cost (R' = blkdiag(R, 0)), the linear cost
    lam0 * theta on every edge, and the rows -lambda <= u <= lambda,
    sum(lambda) <= theta as general rows next to the box rows of x and u.
    Leaves keep their hard bounds.  No ball on x."""
    if float(prob.get("x_ball", 0.0)) > 0 or prob.get("Gamma_x") is not None:
        raise ValueError("l1_input_penalty takes a problem with box constraints only")
    nx, nu = int(prob["nx"]), int(prob["nu"])
    n = len(prob["parent"])
    ns = nu + 1
    nu2 = nu + ns
    B = np.concatenate([np.asarray(prob["B"], float), np.zeros((n, nx, ns))], axis=2)
    R = np.asarray(prob["R"], float)
    if R.ndim == 1:
        R2 = np.concatenate([R, np.zeros(ns)])
    elif R.ndim == 2:
        R2 = np.concatenate([R, np.zeros((n, ns))], axis=1)
    else:
        raise ValueError("l1_input_penalty takes diagonal input costs")
    r = np.zeros((n, nu)) if prob.get("r") is None else np.asarray(prob["r"], float)
    r2 = np.concatenate([r, np.zeros((n, nu)), np.full((n, 1), float(lam0))], axis=1)
    r2[0] = 0.0  # node 0 owns no edge
    I, Z = np.eye(nu), np.zeros((nu, nu))
    Gx = np.vstack([np.eye(nx), np.zeros((nu, nx)), np.zeros((2 * nu + 1, nx))])
    Gu = np.vstack([np.hstack([np.zeros((nx, nu)), np.zeros((nx, ns))]),
                    np.hstack([I, Z, np.zeros((nu, 1))]),
                    np.hstack([I, -I, np.zeros((nu, 1))]),      # u - lambda <= 0
                    np.hstack([-I, -I, np.zeros((nu, 1))]),     # -u - lambda <= 0
                    np.concatenate([np.zeros(nu), np.ones(nu), [-1.0]])[None, :]])  # sum lambda - theta <= 0
    c_lo = np.concatenate([prob["x_lo"], prob["u_lo"], np.full(2 * nu + 1, -np.inf)])
    c_hi = np.concatenate([prob["x_hi"], prob["u_hi"], np.zeros(2 * nu + 1)])
    out = dict(prob, nu=nu2, B=B, R=R2, r=r2, Gamma_x=Gx, Gamma_u=Gu, c_lo=c_lo, c_hi=c_hi,
               Gamma_N=np.eye(nx), cN_lo=np.asarray(prob["xN_lo"], float), cN_hi=np.asarray(prob["xN_hi"], float),
               u_lo=np.concatenate([prob["u_lo"], np.full(ns, -np.inf)]),
               u_hi=np.concatenate([prob["u_hi"], np.full(ns, np.inf)]),
               name=prob.get("name", "custom") + "_l1")
    if out.get("q") is None:
        out["q"] = np.zeros((n, nx))
    if out.get("qN") is None:
        out["qN"] = np.zeros((n, nx))
    return out


def seeded_rng(config_id, instance_id=0):
    return np.random.default_rng(np.random.SeedSequence([int(config_id), int(instance_id)]))


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------

CONFIGS = {
    0: "tiny: N=3, binary (15 nodes), nx=2, nu=1, box, AV@R_0.95, FP64, eps 1e-6",
    1: "medium: N=10, branching [3,3,3,1x7] (229 nodes), nx=20, nu=10, box+ball, AV@R_0.9, Dirichlet, FP64, eps 1e-6",
    2: "large: N=15, branching [2x10,1x5] (7167 nodes), nx=50, nu=25, box+ball, AV@R_0.95, Dirichlet, mixed, eps 1e-4",
    3: "batched: 256 uneven trees, nx 4..32, nu=nx/2, N 5..20, branching 2..4 for 2..5 stages",
}


def config_problem(config_id, instance_id=0):
    """The single-tree workloads 0, 1, 2."""
    rng = seeded_rng(config_id, instance_id)
    if config_id == 0:
        parent, _ = tree_from_branching([2, 2, 2])
        return make_problem(parent, 2, 1, rng, prob_kind="uniform", gamma=0.95,
                            name="cfg0_N3_b2_nx2_nu1")
    if config_id == 1:
        parent, _ = tree_from_branching([3, 3, 3] + [1] * 7)
        return make_problem(parent, 20, 10, rng, prob_kind="dirichlet", gamma=0.9,
                            x_ball=10.0, name="cfg1_N10_b333_nx20_nu10")
    if config_id == 2:
        parent, _ = tree_from_branching([2] * 10 + [1] * 5)
        return make_problem(parent, 50, 25, rng, prob_kind="dirichlet", gamma=0.95,
                            x_ball=10.0, name="cfg2_N15_b2x10_nx50_nu25")
    raise ValueError("config %r is not a single-tree workload" % (config_id,))


def batch_problem(k, seed=3):
    """Problem k of the batched workload: nx ~ U{4..32}, nu = nx//2, N ~ U{5..20},
    one branching factor b ~ U{2,3,4} for the first n_b ~ U{2..5} stages, then 1;
    Dirichlet probabilities, box + ball, AV@R_0.9."""
    rng = seeded_rng(seed, k)
    nx = int(rng.integers(4, 33))
    nu = max(1, nx // 2)
    N = int(rng.integers(5, 21))
    b = int(rng.integers(2, 5))
    nb = min(int(rng.integers(2, 6)), N)
    parent, _ = tree_from_branching([b] * nb + [1] * (N - nb))
    return make_problem(parent, nx, nu, rng, prob_kind="dirichlet", gamma=0.9,
                        x_ball=10.0, name="batch%d_nx%d_N%d_b%d^%d" % (k, nx, N, b, nb))


def random_ragged_problem(seed, N=4, nx=3, nu=2, max_children=3, ball=True,
                          affine=False, gamma=None, linear=False, edge_costs=False, dense_costs=False,
                          general_con=False):
    """Irregular tree (each non-leaf has 1..max_children children), for tests."""
    rng = np.random.default_rng(np.random.SeedSequence([977, int(seed)]))
    counts = []
    width = 1
    for _ in range(N):
        cs = [int(v) for v in rng.integers(1, max_children + 1, size=width)]
        counts.append(cs)
        width = sum(cs)
    parent, _ = tree_from_child_counts(counts)
    n = len(parent)
    n_nl = n - width
    if gamma is None:
        gamma = rng.uniform(0.05, 1.0, size=n_nl)
    return make_problem(parent, nx, nu, rng, prob_kind="dirichlet", gamma=gamma,
                        x_ball=(6.0 if ball else 0.0), affine=affine, linear=linear, edge_costs=edge_costs,
                        dense_costs=dense_costs, general_con=general_con, name="ragged%d" % seed)


def problem_sizes(p):
    """Counts used for reporting: nodes, non-leaf nodes, leaves, stages."""
    parent = p["parent"]
    n = len(parent)
    n_ch = np.bincount(parent[1:], minlength=n)
    n_nl = int(np.sum(n_ch > 0))
    stage = np.zeros(n, dtype=np.int64)
    for j in range(1, n):
        stage[j] = stage[parent[j]] + 1
    return dict(n=n, n_nl=n_nl, n_leaf=n - n_nl, N=int(stage.max()), max_children=int(n_ch.max()))




# ----------------------------------------------------------------------------
# the benchmark case study (random problems of many sizes)
# ----------------------------------------------------------------------------


def _benchmark_sizes(rng, nu_max):
    """N ~ U{5..15}, then (n_b, n_w, n_u) uniform on the set with
    1 <= n_b <= 3, 2 <= n_w <= 10, 10 <= n_u <= nu_max and
    1e3 <= n_v <= 1e5 (n_v = nx |nodes(0, N)| + nu |nodes(0, N-1)|, nx = 2 nu),
    by rejection."""
    N = int(rng.integers(5, 16))
    while True:
        nb = int(rng.integers(1, 4))
        nw = int(rng.integers(2, 11))
        nu = int(rng.integers(10, nu_max + 1))
        nx = 2 * nu
        widths = [nw ** min(t, nb) for t in range(N + 1)]
        nv = nx * sum(widths) + nu * sum(widths[:-1])
        if 1e3 <= nv <= 1e5:
            return N, nb, nw, nu, nx, nv


def benchmark_problem(k, nu_max=300, seed=1268):
    """Instance k of the benchmark case study's random problems: horizon N,
    a tree that branches into n_w events at each of its first n_b stages
    (children of a branching node take events 1..n_w in order with base
    probabilities pi ~ U(simplex); past stage n_b each node has one child,
    which keeps its parent's event), nx = 2 nu; per event w:
    A(w) = I + A^w, B(w) = B + B^w (A^w, B^w entries ~ N(0, 0.01), B ~ N(0, 1)),
    Q(w) = (Q0 + Q^w)(Q0 + Q^w)^T, R(w) = (R0 + R^w)(R0 + R^w)^T
    (Q0 = diag(U[0, 0.1]), R0 = diag(U[0, 100]), Q^w, R^w entries ~ N(0, 0.01)),
    Q_N = Q0; boxes |x| <= xbar ~ U[1, 2], |u| <= ubar ~ U[0, 0.1]; AV@R_gamma
    with gamma ~ U[0, 1]; x0_i ~ U[-xbar_i / 2, xbar_i / 2].  The edge into
    node j carries its event's matrices.  nu_max caps n_u (the library takes
    nx = 2 nu <= 256)."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), int(k)]))
    N, nb, nw, nu, nx, nv = _benchmark_sizes(rng, nu_max)
    parent, stage = tree_from_branching([nw] * min(nb, N) + [1] * (N - min(nb, N)))
    n = len(parent)
    kids = children_lists(parent)
    pi = rng.dirichlet(np.ones(nw))
    event = np.zeros(n, dtype=np.int64)
    prob = np.zeros(n)
    prob[0] = 1.0
    for i in range(n):
        if len(kids[i]) == nw and nw > 1:
            for w, j in enumerate(kids[i]):
                event[j] = w
                prob[j] = pi[w]
        elif kids[i]:
            event[kids[i][0]] = event[i]
            prob[kids[i][0]] = 1.0
    sd = np.sqrt(0.01)
    B = rng.standard_normal((nx, nu))
    Aw = [np.eye(nx) + sd * rng.standard_normal((nx, nx)) for _ in range(nw)]
    Bw = [B + sd * rng.standard_normal((nx, nu)) for _ in range(nw)]
    q0 = rng.uniform(0.0, 0.1, size=nx)
    r0 = rng.uniform(0.0, 100.0, size=nu)
    Qw, Rw = [], []
    for _ in range(nw):
        M = np.diag(q0) + sd * rng.standard_normal((nx, nx))
        Qw.append(M @ M.T)
        M = np.diag(r0) + sd * rng.standard_normal((nu, nu))
        Rw.append(M @ M.T)
    xbar = rng.uniform(1.0, 2.0, size=nx)
    ubar = rng.uniform(0.0, 0.1, size=nu)
    gamma = float(rng.uniform(0.0, 1.0))
    x0 = rng.uniform(-0.5 * xbar, 0.5 * xbar)
    A = np.zeros((n, nx, nx))
    Bn = np.zeros((n, nx, nu))
    Q = np.zeros((n, nx, nx))
    R = np.zeros((n, nu, nu))
    for j in range(1, n):
        A[j], Bn[j], Q[j], R[j] = Aw[event[j]], Bw[event[j]], Qw[event[j]], Rw[event[j]]
    Q[0], R[0] = Qw[0], Rw[0]
    QN = np.broadcast_to(np.diag(q0), (n, nx, nx)).copy()
    n_nl = int(np.sum(np.bincount(parent[1:], minlength=n) > 0))
    return dict(
        name="bench%d_N%d_nb%d_nw%d_nu%d" % (k, N, nb, nw, nu), parent=parent, prob=prob, nx=nx, nu=nu,
        A=A, B=Bn, c=None, Q=Q, R=R, QN=QN, x_lo=-xbar, x_hi=xbar.copy(), u_lo=-ubar, u_hi=ubar.copy(),
        xN_lo=-xbar, xN_hi=xbar.copy(), x_ball=0.0, xN_ball=0.0, gamma=np.full(n_nl, gamma), x0=x0,
        n_v=nv, events=event)


# ----------------------------------------------------------------------------
# the networked-control case study (delay process on a scenario tree)
# ----------------------------------------------------------------------------


def delay_tree(branching, phi0=0.1, theta=1.0):
    """Scenario tree of the sensor-to-controller delay fraction phi of the
    networked-control case study: the children of a node are equiprobable,
    and a child's phi is the quantile of Beta(theta phi, theta (1 - phi)) (its
    parent's phi) at the centre of the child's equal-length interval of
    [0, 1].  Returns (parent, prob, phi).  phi is kept inside
    [1e-12, 1 - 1e-12] so that the next Beta stays defined (quantiles of a
    Beta with a tiny first parameter underflow to 0)."""
    from scipy.stats import beta as _beta
    parent, _ = tree_from_branching(branching)
    n = len(parent)
    kids = children_lists(parent)
    prob = np.zeros(n)
    prob[0] = 1.0
    phi = np.zeros(n)
    phi[0] = phi0
    for i in range(n):
        k = len(kids[i])
        if not k:
            continue
        centres = (np.arange(k) + 0.5) / k
        q = _beta.ppf(centres, theta * phi[i], theta * (1.0 - phi[i]))
        phi[kids[i]] = np.clip(q, 1e-12, 1.0 - 1e-12)
        prob[kids[i]] = 1.0 / k
    return parent, prob, phi


def delay_problem(branching, nx=100, nu=50, T=5.0, phi0=0.1, theta=1.0, gamma=0.95, seed=0, name=None):
    """The networked-control case study: a plant dx/dt = A_c x + B_c u with
    A_c = I + diag(a), a_i ~ N(0, 0.01), B_c = 0.1 * ones(nx, nu), sampled with
    period T; the input u_k acts after the delay sigma = phi T of its sample,
    so over one period the previous input acts for sigma and the new one for
    T - sigma (zero-order hold).  The state is augmented with the previous
    input, xt = (x, u_prev) in R^(nx + nu), and the edge into node j uses the
    delay of node j:
        A^j = [[e^(A_c T), G1(sigma_j)], [0, 0]],  B^j = [[G0(sigma_j)], [I]],
        G0(s) = int_0^(T - s) e^(A_c r) dr B_c,  G1(s) = int_(T - s)^T e^(A_c r) dr B_c
    (closed forms, A_c being diagonal).  Costs Q = 1e-6 I, R = 0.1 I,
    Q_N = diag(1 (nx), 1e-6 (nu)); |x|_inf <= 3 on the plant state (the
    previous-input part is free), |u|_inf <= 0.9; AV@R_gamma; initial plant
    state 2, previous input 0."""
    parent, prob, phi = delay_tree(branching, phi0, theta)
    n = len(parent)
    rng = np.random.default_rng(np.random.SeedSequence([1385, int(seed)]))
    lam = 1.0 + rng.normal(0.0, 0.1, size=nx)          # diagonal of A_c (variance 0.01)
    Bc = 0.1 * np.ones((nx, nu))
    m = nx + nu
    A = np.zeros((n, m, m))
    B = np.zeros((n, m, nu))
    eT = np.exp(lam * T)
    for j in range(1, n):
        s = phi[j] * T
        g0 = (np.exp(lam * (T - s)) - 1.0) / lam          # int_0^(T-s) e^(lam r) dr
        g1 = (eT - np.exp(lam * (T - s))) / lam           # int_(T-s)^T e^(lam r) dr
        A[j, :nx, :nx] = np.diag(eT)
        A[j, :nx, nx:] = g1[:, None] * Bc
        B[j, :nx, :] = g0[:, None] * Bc
        B[j, nx:, :] = np.eye(nu)
    n_nl = int(np.sum(np.bincount(parent[1:], minlength=n) > 0))
    x_hi = np.concatenate([np.full(nx, 3.0), np.full(nu, np.inf)])
    u_hi = np.full(nu, 0.9)
    x0 = np.concatenate([np.full(nx, 2.0), np.zeros(nu)])
    return dict(
        name=name or "delay_%s_nx%d_nu%d" % ("x".join(str(b) for b in branching[:3]), nx, nu),
        parent=parent, prob=prob, nx=m, nu=int(nu), A=A, B=B, c=None,
        Q=np.full(m, 1e-6), R=np.full(nu, 0.1), QN=np.concatenate([np.ones(nx), np.full(nu, 1e-6)]),
        x_lo=-x_hi.copy(), x_hi=x_hi.copy(), u_lo=-u_hi.copy(), u_hi=u_hi.copy(),
        xN_lo=-x_hi.copy(), xN_hi=x_hi.copy(), x_ball=0.0, xN_ball=0.0,
        gamma=np.full(n_nl, float(gamma)), x0=x0, phi=phi)


def delay_branching(n, N=48, wide_first=True):
    """The two tree shapes of the case study with n^2 scenarios each:
    [n^2, 1, ..., 1] (wide_first) or [n, n, 1, ..., 1], horizon N."""
    return [n * n] + [1] * (N - 1) if wide_first else [n, n] + [1] * (N - 2)
