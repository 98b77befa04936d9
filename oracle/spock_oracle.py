"""FP64 CPU oracle for one Chambolle-Pock (CP) step of SPOCK on a scenario tree.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path
(no kernels, headers, helpers or constants) and imports nothing from it.

Everything is plain NumPy in float64, one node at a time, in the order the
paper states it.  Sections cited are those of arXiv:2505.12078
("GPU-Accelerated SPOCK for Scenario-Based Risk-Averse Optimal Control
Problems"):

* problem statement (scenario tree, dynamics, constraints, quadratic costs,
  AV@R and its conic form, the epigraph problem)   -> Sec. 3
* Prop. 1 (quadratic cost as translated SOC)        -> Sec. 4.2
* sets S1, S2, S3                                   -> Sec. 4.3
* linear operator L                                 -> Sec. 4.4
* splitting f, g                                    -> Sec. 4.5
* CP operator T                                     -> Sec. 4.1, Eq. (CP operator)
* Alg. 1 (offline S1) and Alg. 2 (online S1)        -> Sec. 5.1
* residuals xi1, xi2                                -> Sec. 5.3
* preconditioning                                   -> Sec. 5.4

Readings where the paper is silent or garbled (all listed in the design doc):
  - AV@R parameter gamma is the tail mass (AV@R_1 = E, AV@R_0 = max);
    b^i uses the conditional child probabilities.
  - SOC_d = {(w, t) in R^{d-1} x R : ||w|| <= t}, scalar last; with q = 0 the
    translation of Prop. 1 is a = (0, ..., 0, +1/2, -1/2).
  - Preconditioning: S^x on every non-leaf node (root included), S^u on every
    input, S^x_N on leaves; constraint rows rescaled by 1/a with
    a = max(1, ||Gamma S^-1||_2), at non-leaf nodes and at leaves.
  - Step size alpha = 0.99/||L|| with ||L|| the exact block norm.
  - rel_res = max(|xi1|_inf, |xi2|_inf) / max(1, first-step residuals).

Parity pins for every function here live in tests/test_oracle_*.py.
"""
from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------------------
# scenario tree (Sec. 3.2)
# ----------------------------------------------------------------------------


class Tree:
    """Nodes numbered stage by stage; ``anc``, ``ch``, ``nodes(t)`` as in Sec. 3.2."""

    def __init__(self, parent, cond_prob):
        parent = np.asarray(parent, dtype=np.int64)
        n = parent.size
        if n < 2 or parent[0] != -1:
            raise ValueError("parent[0] must be -1 and the tree needs >= 2 nodes")
        for j in range(1, n):
            if not (0 <= parent[j] < j):
                raise ValueError("nodes must be numbered after their ancestor")
        self.n = n
        self.anc = parent
        self.ch = [[] for _ in range(n)]
        for j in range(1, n):
            self.ch[parent[j]].append(j)
        self.stage = np.zeros(n, dtype=np.int64)
        for j in range(1, n):
            self.stage[j] = self.stage[parent[j]] + 1
        self.N = int(self.stage.max())
        self.nonleaf = [i for i in range(n) if self.ch[i]]
        self.leaves = [j for j in range(n) if not self.ch[j]]
        if self.nonleaf != list(range(len(self.nonleaf))):
            raise ValueError("non-leaf nodes must come first")
        if any(self.stage[j] != self.N for j in self.leaves):
            raise ValueError("every leaf must sit at stage N")
        self.n_nl = len(self.nonleaf)
        self.n_leaf = len(self.leaves)
        self.p = np.asarray(cond_prob, dtype=np.float64)
        for i in self.nonleaf:
            if abs(self.p[self.ch[i]].sum() - 1.0) > 1e-9:
                raise ValueError("children probabilities of node %d do not sum to 1" % i)
        # unconditional probabilities pi^i (sum to 1 per stage)
        self.pi = np.ones(n)
        for j in range(1, n):
            self.pi[j] = self.pi[parent[j]] * self.p[j]

    def nodes(self, t):
        return [i for i in range(self.n) if self.stage[i] == t]


# ----------------------------------------------------------------------------
# AV@R (Sec. 3.3) -- used by the pins and the nested-cost invariant
# ----------------------------------------------------------------------------


def avar_min_form(Z, p, gamma):
    """min_t t + (1/gamma) E^p[Z - t]_+ (gamma > 0); max Z when gamma = 0.

    The objective is convex piecewise linear in the scalar t with kinks at the
    values of Z, so its minimum is attained at one of them.
    """
    Z = np.asarray(Z, float)
    p = np.asarray(p, float)
    if gamma == 0:
        return float(Z.max())
    return float(min(t + np.dot(p, np.maximum(Z - t, 0.0)) / gamma for t in Z))


def avar_ambiguity_form(Z, p, gamma):
    """max mu^T Z over {sum mu = 1, 0 <= mu <= p/gamma}: fill mass on the
    largest costs first (a fractional knapsack)."""
    Z = np.asarray(Z, float)
    p = np.asarray(p, float)
    cap = np.full(Z.size, np.inf) if gamma == 0 else p / gamma
    order = np.argsort(-Z, kind="stable")
    left = 1.0
    val = 0.0
    for k in order:
        m = min(cap[k], left)
        val += m * Z[k]
        left -= m
        if left <= 0:
            break
    return float(val)


def avar_conic_data(p, gamma):
    """b, E of the conic representation of AV@R_gamma (Sec. 3.3), K = R^{2n}_+ x {0}."""
    p = np.asarray(p, float)
    n = p.size
    b = np.concatenate([p, np.zeros(n), [1.0]])
    E = np.vstack([gamma * np.eye(n), -np.eye(n), np.ones((1, n))])
    return b, E


def soc_blocks(cone):
    """The second-order cone blocks of a cone given row by row: code 2 opens
    a block {(t, w): ||w|| <= t} at its head row t, code 3 continues it with
    the rows of w.  Returns (head, tail length) pairs."""
    cone = np.asarray(cone)
    out = []
    r = 0
    while r < cone.size:
        if cone[r] == 2:
            L = 0
            while r + 1 + L < cone.size and cone[r + 1 + L] == 3:
                L += 1
            out.append((r, L))
            r += 1 + L
        else:
            r += 1
    return out


def project_dual_cone(v, cone):
    """Projection onto K* for K given row by row (Sec. 3.3): R_+ rows
    (code 0) are self-dual, {0} rows (code 1) have dual R, and a second-order
    cone block (codes 2, 3...) is self-dual."""
    cone = np.asarray(cone)
    out = np.where(cone == 0, np.maximum(v, 0.0), v)
    for h, L in soc_blocks(cone):
        blk = np.concatenate([v[h + 1:h + 1 + L], [v[h]]])  # (w, t): scalar last
        pb = proj_soc(blk)
        out[h] = pb[-1]
        out[h + 1:h + 1 + L] = pb[:-1]
    return out


def conic_risk_value(Z, E, F, b, cone):
    """rho(Z) = max{mu^T Z : b - E mu - F nu in K} (Sec. 3.3) for a polyhedral
    K given entrywise (cone[r] = 0: R_+, 1: {0}), by an LP (scipy HiGHS)."""
    from scipy.optimize import linprog
    if np.any(np.asarray(cone) >= 2):
        raise NotImplementedError("conic_risk_value evaluates polyhedral cones only")
    E = np.asarray(E, float)
    ny, k = E.shape
    F = np.zeros((ny, 0)) if F is None else np.asarray(F, float)
    nnu = F.shape[1]
    cone = np.asarray(cone)
    A = np.hstack([E, F])  # b - A [mu; nu] in K: A v <= b (R_+ rows), A v = b ({0} rows)
    ineq, eq = cone == 0, cone == 1
    c = -np.concatenate([np.asarray(Z, float), np.zeros(nnu)])
    res = linprog(c, A_ub=A[ineq] if ineq.any() else None, b_ub=np.asarray(b)[ineq] if ineq.any() else None,
                  A_eq=A[eq] if eq.any() else None, b_eq=np.asarray(b)[eq] if eq.any() else None,
                  bounds=[(None, None)] * (k + nnu), method="highs")
    assert res.status == 0, res.message
    return float(-res.fun)


def node_risk(prob, i, p_kids):
    """The conic data (E, F, b, cone) of the risk at non-leaf node i: the
    node's own from prob["risk"][i] when given (general coherent risk,
    Sec. 3.3, polyhedral K), else AV@R_gamma^i."""
    r = prob.get("risk")
    if r is not None:
        E, F, b, cone = r[i]
        return (np.asarray(E, float), None if F is None else np.asarray(F, float), np.asarray(b, float),
                np.asarray(cone, int))
    b, E = avar_conic_data(p_kids, float(prob["gamma"][i]))
    k = len(p_kids)
    return E, None, b, np.concatenate([np.zeros(2 * k, int), [1]])


# ----------------------------------------------------------------------------
# problem data in the iterated (preconditioned) space (Sec. 5.4)
# ----------------------------------------------------------------------------


def cost_matrices(prob, key, n):
    """The cost matrix of every node for prob[key] (Sec. 3.1): one shared
    diagonal [d], one diagonal per node [n][d], or one dense matrix per node
    [n][d][d] (row / matrix j: the edge into node j, or leaf j)."""
    a = np.asarray(prob[key], float)
    if a.ndim == 3:
        return [a[j] for j in range(n)]
    return [np.diag(a[j] if a.ndim == 2 else a) for j in range(n)]


def _sym_sqrt(M):
    w, V = np.linalg.eigh(M)
    return (V * np.sqrt(np.maximum(w, 0.0))) @ V.T


class Data:
    """All matrices of the RAOCP after the change of variables of Sec. 5.4.

    Dense matrices everywhere (the oracle does not exploit the diagonal
    structure of the synthetic workloads).
    """

    def __init__(self, prob, precondition=True):
        self.tree = T = Tree(prob["parent"], prob["prob"])
        nx, nu = int(prob["nx"]), int(prob["nu"])
        self.nx, self.nu = nx, nu
        # stage costs Q^j, R^j of the edge into j and terminal costs Q_N^j of
        # leaf j (Sec. 3.1): one shared diagonal, or one row per node
        n = T.n
        Qs, Rs, QNs = (cost_matrices(prob, k, n) for k in ("Q", "R", "QN"))
        ball = float(prob["x_ball"]) > 0
        ballN = float(prob["xN_ball"]) > 0
        self.has_ball, self.has_ballN = ball, ballN

        # Sec. 5.4 scalings: the largest square root over the edges (leaves)
        if precondition:
            chat = np.sqrt(max(len(T.ch[i]) for i in T.nonleaf))
            edges = range(1, n)
            Sx = chat * np.maximum(1.0, np.sqrt(np.max([np.diag(Qs[j]) for j in edges], axis=0)))
            Su = chat * np.maximum(1.0, np.sqrt(np.max([np.diag(Rs[j]) for j in edges], axis=0)))
            SxN = np.maximum(1.0, np.sqrt(np.max([np.diag(QNs[j]) for j in T.leaves], axis=0)))
        else:
            Sx, Su, SxN = np.ones(nx), np.ones(nu), np.ones(nx)
        self.Sx, self.Su, self.SxN = Sx, Su, SxN

        def S_of(j):
            return Sx if j < T.n_nl else SxN

        self.S_of = S_of
        n = T.n
        A = np.asarray(prob["A"], float)
        B = np.asarray(prob["B"], float)
        c = prob.get("c")
        c = np.zeros((n, nx)) if c is None else np.asarray(c, float)
        # x~ = S x: x~^j = S(j) A S^x^-1 x~^i + S(j) B S^u^-1 u~^i + S(j) c
        self.A = np.zeros_like(A)
        self.B = np.zeros_like(B)
        self.c = np.zeros_like(c)
        for j in range(1, n):
            Sj = S_of(j)
            self.A[j] = (Sj[:, None] * A[j]) / Sx[None, :]
            self.B[j] = (Sj[:, None] * B[j]) / Su[None, :]
            self.c[j] = Sj * c[j]
        # cost square roots in the new variables: ||Q^1/2 x||^2 = x^T Q x, per
        # edge j (Qh_e[j], Rh_e[j]) and per leaf (QNh_l[j])
        self.Qh_e = [_sym_sqrt(Qs[j]) / Sx[None, :] for j in range(n)]
        self.Rh_e = [_sym_sqrt(Rs[j]) / Su[None, :] for j in range(n)]
        self.QNh_l = [_sym_sqrt(QNs[j]) / SxN[None, :] for j in range(n)]

        # non-leaf constraint Gamma_x x + Gamma_u u in C (Sec. 3.1): C a box
        # [c_lo, c_hi] for general Gamma (prob["Gamma_x"], prob["Gamma_u"]),
        # else box(x) x box(u) [x ball(x)]
        Ix, Iu = np.eye(nx), np.eye(nu)
        self.general = prob.get("Gamma_x") is not None
        if self.general:
            ball = False
            Gx = np.asarray(prob["Gamma_x"], float)
            Gu = np.asarray(prob["Gamma_u"], float)
            lo, hi = [np.asarray(prob["c_lo"], float)], [np.asarray(prob["c_hi"], float)]
        else:
            Gx = [Ix, np.zeros((nu, nx))]
            Gu = [np.zeros((nx, nu)), Iu]
            lo = [np.asarray(prob["x_lo"], float), np.asarray(prob["u_lo"], float)]
            hi = [np.asarray(prob["x_hi"], float), np.asarray(prob["u_hi"], float)]
            if ball:
                Gx.append(Ix)
                Gu.append(np.zeros((nx, nu)))
            Gx, Gu = np.vstack(Gx), np.vstack(Gu)
        self.has_ball = ball
        Gx = Gx / Sx[None, :]
        Gu = Gu / Su[None, :]
        a = max(1.0, np.linalg.norm(np.hstack([Gx, Gu]), 2)) if precondition else 1.0
        self.Gx, self.Gu = Gx / a, Gu / a
        self.box_lo = np.concatenate(lo) / a
        self.box_hi = np.concatenate(hi) / a
        self.nbox = self.box_lo.size
        self.ball_r = float(prob["x_ball"]) / a if ball else 0.0
        self.con_scale = a
        # leaf constraint Gamma_N x in C_N: a box [cN_lo, cN_hi] for general
        # Gamma_N (prob["Gamma_N"]), else box(x) [x ball(x)]
        self.generalN = prob.get("Gamma_N") is not None
        if self.generalN:
            ballN = False
            GN = np.asarray(prob["Gamma_N"], float)
            loN, hiN = np.asarray(prob["cN_lo"], float), np.asarray(prob["cN_hi"], float)
        else:
            GN = np.vstack([Ix] + ([Ix] if ballN else []))
            loN, hiN = np.asarray(prob["xN_lo"], float), np.asarray(prob["xN_hi"], float)
        self.has_ballN = ballN
        GN = GN / SxN[None, :]
        aN = max(1.0, np.linalg.norm(GN, 2)) if precondition else 1.0
        self.GN = GN / aN
        self.boxN_lo = loN / aN
        self.boxN_hi = hiN / aN
        self.nboxN = self.boxN_lo.size
        self.ballN_r = float(prob["xN_ball"]) / aN if ballN else 0.0
        self.con_scaleN = aN
        self.nc = self.Gx.shape[0]
        self.ncN = self.GN.shape[0]

        self.gamma = np.asarray(prob["gamma"], float)
        # the risk of every non-leaf node as conic data (E, F, b, K)
        self.risk = [node_risk(prob, i, T.p[T.ch[i]]) for i in range(T.n_nl)]
        self.general_risk = prob.get("risk") is not None
        self.x0 = Sx * np.asarray(prob["x0"], float)
        self.layout = Layout(T, nx, nu, self.nc, self.ncN, [len(r[2]) for r in self.risk])

        # linear cost terms (Prop. 1, Sec. 4.2): q^j, r^j on the edge into j
        # (acting on x^anc(j), u^anc(j)), qN^j at leaf j; in the new variables
        # q~ = S^-1 q, and the translation a of Prop. 1 follows from the factor
        # Q~^1/2 that L uses (Qh, Rh, QNh)
        def lin(key, cols):
            v = prob.get(key)
            return np.zeros((n, cols)) if v is None else np.asarray(v, float).reshape(n, cols)

        self.q_lin = lin("q", nx) / Sx[None, :]
        self.r_lin = lin("r", nu) / Su[None, :]
        self.qN_lin = lin("qN", nx) / SxN[None, :]
        self.has_lin = any(prob.get(k) is not None for k in ("q", "r", "qN"))
        # Prop. 1 with a singular cost matrix: the part of the linear term in
        # ker Q (z' of the proposition) enters the two tau rows of the SOC
        # block, (tau - q_ker^T z) / 2 each; the part in range Q makes the
        # translation.  Per edge j on (x, u) of the parent, per leaf on x.
        def split(F, q):
            # range(F^T F) = range(F^T); q_range its orthogonal projection
            U, sv, _ = np.linalg.svd(F.T)
            r = int(np.sum(sv > 1e-12 * max(1.0, sv.max() if sv.size else 0.0)))
            Ur = U[:, :r]
            q_rng = Ur @ (Ur.T @ q)
            return q_rng, q - q_rng
        self.c_edge = np.zeros((n, nx + nu))
        self.cN_leaf = np.zeros((n, nx))
        self.q_rng = np.zeros((n, nx + nu))
        self.qN_rng = np.zeros((n, nx))
        if self.has_lin:
            for j in range(1, n):
                F = np.zeros((nx + nu, nx + nu))
                F[:nx, :nx], F[nx:, nx:] = self.Qh_e[j], self.Rh_e[j]
                self.q_rng[j], self.c_edge[j] = split(F, np.concatenate([self.q_lin[j], self.r_lin[j]]))
            for j in T.leaves:
                self.qN_rng[j], self.cN_leaf[j] = split(self.QNh_l[j], self.qN_lin[j])
        self.coupled = bool(np.any(self.c_edge != 0) or np.any(self.cN_leaf != 0))

    def unscale(self, x, u):
        T = self.tree
        xs = np.array([x[j] / self.S_of(j) for j in range(T.n)])
        us = np.array([u[i] / self.Su for i in range(T.n_nl)])
        return xs, us


# ----------------------------------------------------------------------------
# canonical vector layout of z and eta
# ----------------------------------------------------------------------------


class Layout:
    """z = (s0, x[0..n), u[non-leaf], y[non-leaf, ragged 2 n_ch + 1],
    tau[1..n), s[1..n)) and eta = (eta_y[ragged], eta_s[non-leaf],
    eta_c[non-leaf], eta_soc[edge j = 1..n-1], eta_cN[leaf], eta_socN[leaf]),
    each block in node order (Sec. 4.3 and Sec. 4.4)."""

    def __init__(self, T, nx, nu, nc, ncN, ylen=None):
        self.T, self.nx, self.nu, self.nc, self.ncN = T, nx, nu, nc, ncN
        n, n_nl, n_l = T.n, T.n_nl, T.n_leaf
        # y^i has one entry per row of the node's conic data (2 n_ch + 1 for AV@R)
        self.ylen = list(ylen) if ylen is not None else [2 * len(T.ch[i]) + 1 for i in range(n_nl)]
        self.yoff = np.concatenate([[0], np.cumsum(self.ylen)]).astype(int)
        ny = int(self.yoff[-1])
        o = 0
        self.z_s0 = o; o += 1
        self.z_x = o; o += n * nx
        self.z_u = o; o += n_nl * nu
        self.z_y = o; o += ny
        self.z_tau = o; o += n - 1
        self.z_s = o; o += n - 1
        self.nz = o
        o = 0
        self.e_y = o; o += ny
        self.e_s = o; o += n_nl
        self.e_c = o; o += n_nl * nc
        self.nsoc = nx + nu + 2
        self.e_soc = o; o += (n - 1) * self.nsoc
        self.e_cN = o; o += n_l * ncN
        self.nsocN = nx + 2
        self.e_socN = o; o += n_l * self.nsocN
        self.neta = o

    # z accessors (views)
    def x(self, z, i): return z[self.z_x + i * self.nx: self.z_x + (i + 1) * self.nx]
    def u(self, z, i): return z[self.z_u + i * self.nu: self.z_u + (i + 1) * self.nu]
    def y(self, z, i): return z[self.z_y + self.yoff[i]: self.z_y + self.yoff[i + 1]]
    def tau(self, z, j): return z[self.z_tau + j - 1: self.z_tau + j]
    def s(self, z, j):
        """s^j for j >= 1; s^0 is the first entry of z."""
        if j == 0:
            return z[self.z_s0: self.z_s0 + 1]
        return z[self.z_s + j - 1: self.z_s + j]

    # eta accessors (views)
    def ey(self, e, i): return e[self.e_y + self.yoff[i]: self.e_y + self.yoff[i + 1]]
    def es(self, e, i): return e[self.e_s + i: self.e_s + i + 1]
    def ec(self, e, i): return e[self.e_c + i * self.nc: self.e_c + (i + 1) * self.nc]
    def esoc(self, e, j): return e[self.e_soc + (j - 1) * self.nsoc: self.e_soc + j * self.nsoc]
    def ecN(self, e, j):
        k = j - self.T.n_nl
        return e[self.e_cN + k * self.ncN: self.e_cN + (k + 1) * self.ncN]
    def esocN(self, e, j):
        k = j - self.T.n_nl
        return e[self.e_socN + k * self.nsocN: self.e_socN + (k + 1) * self.nsocN]


# ----------------------------------------------------------------------------
# operator L and its adjoint (Sec. 4.4)
# ----------------------------------------------------------------------------


def b_vector(D, i):
    """b^i of the risk's conic data at node i: (p^{ch(i)}, 0, 1) for AV@R
    (conditional probabilities), else the given b^i."""
    return D.risk[i][2]


def apply_L(D, z):
    T, Y = D.tree, D.layout
    eta = np.zeros(Y.neta)
    for i in T.nonleaf:
        Y.ey(eta, i)[:] = Y.y(z, i)
        Y.es(eta, i)[:] = Y.s(z, i) - b_vector(D, i) @ Y.y(z, i)
        Y.ec(eta, i)[:] = D.Gx @ Y.x(z, i) + D.Gu @ Y.u(z, i)
    for j in range(1, T.n):
        i = T.anc[j]
        # tau rows (tau - q_ker^T (x, u)) / 2 (Prop. 1; q_ker = 0 unless Q is singular)
        t = Y.tau(z, j)[0] - D.c_edge[j] @ np.concatenate([Y.x(z, i), Y.u(z, i)])
        Y.esoc(eta, j)[:] = np.concatenate([D.Qh_e[j] @ Y.x(z, i), D.Rh_e[j] @ Y.u(z, i), [0.5 * t, 0.5 * t]])
    for j in T.leaves:
        Y.ecN(eta, j)[:] = D.GN @ Y.x(z, j)
        sj = Y.s(z, j)[0] - D.cN_leaf[j] @ Y.x(z, j)
        Y.esocN(eta, j)[:] = np.concatenate([D.QNh_l[j] @ Y.x(z, j), [0.5 * sj, 0.5 * sj]])
    return eta


def apply_Lt(D, eta):
    """Adjoint of apply_L: collects, for every primal entry, the dual blocks
    that depend on it (the sum over siblings in the x/u rows)."""
    T, Y = D.tree, D.layout
    nx, nu = D.nx, D.nu
    z = np.zeros(Y.nz)
    for i in T.nonleaf:
        b = b_vector(D, i)
        es = Y.es(eta, i)[0]
        Y.y(z, i)[:] += Y.ey(eta, i) - b * es
        Y.s(z, i)[:] += es
        Y.x(z, i)[:] += D.Gx.T @ Y.ec(eta, i)
        Y.u(z, i)[:] += D.Gu.T @ Y.ec(eta, i)
    for j in range(1, T.n):
        i = T.anc[j]
        w = Y.esoc(eta, j)
        h = 0.5 * (w[nx + nu] + w[nx + nu + 1])
        Y.x(z, i)[:] += D.Qh_e[j].T @ w[:nx] - h * D.c_edge[j][:nx]
        Y.u(z, i)[:] += D.Rh_e[j].T @ w[nx:nx + nu] - h * D.c_edge[j][nx:]
        Y.tau(z, j)[:] += h
    for j in T.leaves:
        Y.x(z, j)[:] += D.GN.T @ Y.ecN(eta, j)
        w = Y.esocN(eta, j)
        h = 0.5 * (w[nx] + w[nx + 1])
        Y.x(z, j)[:] += D.QNh_l[j].T @ w[:nx] - h * D.cN_leaf[j]
        Y.s(z, j)[:] += h
    return z


def L_norm(D):
    """Exact ||L||: L composed with a permutation is block diagonal (Sec. 4.4);
    its norm is the largest block norm.  Blocks, by primal variable group:
    (x^i, u^i) of a non-leaf node, x^j of a leaf, each tau^j, each leaf s^j and
    (y^i, s^i) of a non-leaf node."""
    T = D.tree
    norms = []
    for i in T.nonleaf:
        rows = [np.hstack([D.Gx, D.Gu])]
        for j in T.ch[i]:
            rows.append(np.hstack([D.Qh_e[j], np.zeros((D.nx, D.nu))]))
            rows.append(np.hstack([np.zeros((D.nu, D.nx)), D.Rh_e[j]]))
        if D.coupled:
            # the tau rows couple (x^i, u^i) with every tau^j of the children:
            # one block over (x^i, u^i, tau^ch(i))
            k = len(T.ch[i])
            blk = [np.hstack([r, np.zeros((r.shape[0], k))]) for r in rows]
            for q, j in enumerate(T.ch[i]):
                tr = np.concatenate([-0.5 * D.c_edge[j], 0.5 * np.eye(k)[q]])
                blk += [tr[None, :], tr[None, :]]
            norms.append(np.linalg.norm(np.vstack(blk), 2))
        else:
            norms.append(np.linalg.norm(np.vstack(rows), 2))
        b = b_vector(D, i)
        m = b.size
        blk = np.zeros((m + 1, m + 1))
        blk[:m, :m] = np.eye(m)
        blk[m, :m] = -b
        blk[m, m] = 1.0
        norms.append(np.linalg.norm(blk, 2))
    for j in T.leaves:
        if D.coupled:  # (x^j, s^j) with the leaf's s rows (s - qN_ker^T x) / 2
            tr = np.concatenate([-0.5 * D.cN_leaf[j], [0.5]])
            blk = np.vstack([np.hstack([D.GN, np.zeros((D.GN.shape[0], 1))]),
                             np.hstack([D.QNh_l[j], np.zeros((D.nx, 1))]), tr, tr])
            norms.append(np.linalg.norm(blk, 2))
        else:
            norms.append(np.linalg.norm(np.vstack([D.GN, D.QNh_l[j]]), 2))
    norms.append(np.sqrt(0.5))  # tau^j and leaf s^j: (1/2, 1/2)
    return float(max(norms))


# ----------------------------------------------------------------------------
# S1: Alg. 1 (offline) and Alg. 2 (online), Sec. 5.1
# ----------------------------------------------------------------------------


class Offline:
    """Alg. 1: P at the leaves is the identity, then stage by stage backwards
    R~ = I + sum B^T P B (and its Cholesky factor), K = -R~^-1 sum B^T P A,
    Abar = A + B K, P = I + K^T K + sum Abar^T P Abar."""

    def __init__(self, D):
        T = D.tree
        nx, nu = D.nx, D.nu
        self.P = [None] * T.n
        self.K = [None] * T.n
        self.Rt = [None] * T.n
        self.Lc = [None] * T.n
        self.Abar = [None] * T.n
        for j in T.leaves:
            self.P[j] = np.eye(nx)
        for t in range(T.N - 1, -1, -1):
            for i in T.nodes(t):
                Pt = {j: D.B[j].T @ self.P[j] for j in T.ch[i]}
                Rt = np.eye(nu) + sum(Pt[j] @ D.B[j] for j in T.ch[i])
                Lc = np.linalg.cholesky(Rt)
                rhs = sum(Pt[j] @ D.A[j] for j in T.ch[i])
                K = -_chol_solve(Lc, rhs)
                for j in T.ch[i]:
                    self.Abar[j] = D.A[j] + D.B[j] @ K
                self.P[i] = np.eye(nx) + K.T @ K + sum(
                    self.Abar[j].T @ self.P[j] @ self.Abar[j] for j in T.ch[i])
                self.K[i], self.Rt[i], self.Lc[i] = K, Rt, Lc


def _chol_solve(Lc, b):
    y = np.linalg.solve(Lc, b)
    return np.linalg.solve(Lc.T, y)


def project_S1(D, F, xbar, ubar):
    """Alg. 2: Euclidean projection of (xbar, ubar) onto the dynamics set S1
    with x^0 fixed to D.x0.  xbar: (n, nx), ubar: (n_nl, nu)."""
    T = D.tree
    q = [None] * T.n
    d = [None] * T.n
    for j in T.leaves:
        q[j] = -xbar[j]
    for t in range(T.N - 1, -1, -1):
        for i in T.nodes(t):
            dbar = sum(D.B[j].T @ (q[j] + F.P[j] @ D.c[j]) for j in T.ch[i])
            d[i] = _chol_solve(F.Lc[i], ubar[i] - dbar)
            qbar = sum(F.Abar[j].T @ (F.P[j] @ (D.B[j] @ d[i] + D.c[j]) + q[j]) for j in T.ch[i])
            q[i] = F.K[i].T @ (d[i] - ubar[i]) - xbar[i] + qbar
    x = np.zeros((T.n, D.nx))
    u = np.zeros((T.n_nl, D.nu))
    x[0] = D.x0
    for t in range(T.N):
        for i in T.nodes(t):
            u[i] = F.K[i] @ x[i] + d[i]
            for j in T.ch[i]:
                x[j] = D.A[j] @ x[i] + D.B[j] @ u[i] + D.c[j]
    return x, u


# ----------------------------------------------------------------------------
# S2: kernel of [E^T -I -I] per non-leaf node (Sec. 4.3, AV@R data of Sec. 3.3)
# ----------------------------------------------------------------------------


def S2_matrix(gamma, nch, E=None, F=None):
    """G with G (y, tau^[i], s^[i]) = (E^T y - tau - s, F^T y) (the kernel of
    Sec. 4.3); AV@R_gamma's E when E is not given (no F)."""
    if E is None:
        _, E = avar_conic_data(np.full(nch, 1.0 / nch), gamma)
    G = np.hstack([E.T, -np.eye(nch), -np.eye(nch)])
    if F is not None and F.shape[1] > 0:
        G = np.vstack([G, np.hstack([F.T, np.zeros((F.shape[1], 2 * nch))])])
    return G


def project_S2_block(w, gamma, nch, E=None, F=None):
    """Orthogonal projection of w onto ker G: w - G^T (G G^T)^-1 G w."""
    G = S2_matrix(gamma, nch, E, F)
    return w - G.T @ np.linalg.solve(G @ G.T, G @ w)


# ----------------------------------------------------------------------------
# S3 cones and Moreau (Sec. 4.3, Sec. 4.1)
# ----------------------------------------------------------------------------


def proj_soc(v):
    """Projection onto SOC = {(w, t): ||w|| <= t} (scalar last)."""
    w, t = v[:-1], v[-1]
    nw = np.linalg.norm(w)
    if nw <= t:
        return v.copy()
    if nw <= -t:
        return np.zeros_like(v)
    a = 0.5 * (nw + t)
    return np.concatenate([a * w / nw, [a]])


def proj_ball(v, r):
    nv = np.linalg.norm(v)
    return v.copy() if nv <= r else v * (r / nv)


def soc_shift(m):
    """Translation a of Prop. 1 for q = 0: (0, ..., 0, +1/2, -1/2), length m."""
    a = np.zeros(m)
    a[-2], a[-1] = 0.5, -0.5
    return a


def soc_shift_lin(Qh, q):
    """Translation a of Prop. 1 (Sec. 4.2):
    (-1/2 Q~^-1/2 q~, -1/8 |q~|^2_{Q~^-1} + 1/2, -1/8 |q~|^2_{Q~^-1} - 1/2),
    where Q~^1/2 is the factor Qh of the cost block of L (Qh^T Qh = Q~), so
    Q~^-1/2 q~ = Qh^-T q~ and |q~|^2_{Q~^-1} = |Qh^-T q~|^2.  For a singular
    Q~, q is its part in range Q~ (the rest enters L's tau rows) and Qh^-T
    is the pseudo-inverse (Qh^T w = q has the solution of least norm, which
    lies in range Qh)."""
    w = np.linalg.lstsq(Qh.T, q, rcond=None)[0]
    c = -0.125 * float(w @ w)
    return np.concatenate([-0.5 * w, [c + 0.5, c - 0.5]])


def edge_shift(D, j):
    """a of the SOC block of the edge into node j: the cost on (x, u) of the
    parent with Q~ = blkdiag(Q~, R~) and q~ = (q~^j, r~^j)."""
    if not D.has_lin:
        return soc_shift(D.nx + D.nu + 2)
    nx, nu = D.nx, D.nu
    F = np.zeros((nx + nu, nx + nu))
    F[:nx, :nx] = D.Qh_e[j]
    F[nx:, nx:] = D.Rh_e[j]
    return soc_shift_lin(F, D.q_rng[j])


def leaf_shift(D, j):
    """a of the SOC block of leaf j (terminal cost Q_N, qN^j)."""
    if not D.has_lin:
        return soc_shift(D.nx + 2)
    return soc_shift_lin(D.QNh_l[j], D.qN_rng[j])


def project_S3(D, eta):
    T, Y = D.tree, D.layout
    nb = D.nbox
    out = np.zeros_like(eta)
    for i in T.nonleaf:
        k = len(T.ch[i])
        v = Y.ey(eta, i)
        # (K^i)*: R_+ where K^i is R_+, R where K^i is {0} (AV@R: R^{2k}_+ x R),
        # a second-order cone where K^i has one
        Y.ey(out, i)[:] = project_dual_cone(v, D.risk[i][3])
        Y.es(out, i)[:] = np.maximum(Y.es(eta, i), 0.0)
        c = Y.ec(eta, i)
        pc = np.clip(c[:nb], D.box_lo, D.box_hi)
        if D.has_ball:
            pc = np.concatenate([pc, proj_ball(c[nb:], D.ball_r)])
        Y.ec(out, i)[:] = pc
    for j in range(1, T.n):
        v = Y.esoc(eta, j)
        a = edge_shift(D, j)
        Y.esoc(out, j)[:] = a + proj_soc(v - a)
    for j in T.leaves:
        c = Y.ecN(eta, j)
        pc = np.clip(c[:D.nboxN], D.boxN_lo, D.boxN_hi)
        if D.has_ballN:
            pc = np.concatenate([pc, proj_ball(c[D.nboxN:], D.ballN_r)])
        Y.ecN(out, j)[:] = pc
        v = Y.esocN(eta, j)
        a = leaf_shift(D, j)
        Y.esocN(out, j)[:] = a + proj_soc(v - a)
    return out


def prox_gconj(D, w, alpha):
    """prox of alpha g* with g = indicator of S3, by Moreau's decomposition:
    w - alpha proj_S3(w / alpha)."""
    return w - alpha * project_S3(D, w / alpha)


# ----------------------------------------------------------------------------
# prox of f and the CP operator T (Sec. 4.5, Sec. 4.1)
# ----------------------------------------------------------------------------


def prox_f(D, F, zbar, alpha):
    """prox of alpha f with f = s0 + delta_S1(z1) + delta_S2(z2)."""
    T, Y = D.tree, D.layout
    z = np.zeros_like(zbar)
    z[Y.z_s0] = zbar[Y.z_s0] - alpha
    xbar = np.array([Y.x(zbar, i) for i in range(T.n)])
    ubar = np.array([Y.u(zbar, i) for i in range(T.n_nl)])
    x, u = project_S1(D, F, xbar, ubar)
    for i in range(T.n):
        Y.x(z, i)[:] = x[i]
    for i in range(T.n_nl):
        Y.u(z, i)[:] = u[i]
    for i in T.nonleaf:
        kids = T.ch[i]
        w = np.concatenate([Y.y(zbar, i),
                            [Y.tau(zbar, j)[0] for j in kids],
                            [Y.s(zbar, j)[0] for j in kids]])
        E, Fm, _, _ = D.risk[i]
        pw = project_S2_block(w, D.gamma[i], len(kids), E, Fm)
        m = Y.ylen[i]
        Y.y(z, i)[:] = pw[:m]
        for k, j in enumerate(kids):
            Y.tau(z, j)[:] = pw[m + k]
            Y.s(z, j)[:] = pw[m + len(kids) + k]
    return z


def cp_step(D, F, z, eta, alpha):
    """One application of the CP operator T (Sec. 4.1):
    z+ = prox_{alpha f}(z - alpha L* eta),
    eta+ = prox_{alpha g*}(eta + alpha L(2 z+ - z))."""
    zp = prox_f(D, F, z - alpha * apply_Lt(D, eta), alpha)
    etap = prox_gconj(D, eta + alpha * apply_L(D, 2.0 * zp - z), alpha)
    return zp, etap


def residuals(D, z, eta, zp, etap, alpha):
    """xi1 = dz/alpha - L* d_eta, xi2 = d_eta/alpha - L dz with
    dz = z - z+, d_eta = eta - eta+ (Sec. 5.3)."""
    dz, de = z - zp, eta - etap
    xi1 = dz / alpha - apply_Lt(D, de)
    xi2 = de / alpha - apply_L(D, dz)
    return xi1, xi2


def step_size(D):
    return 0.99 / L_norm(D)


# ----------------------------------------------------------------------------
# plain CP solve (the iteration that the HIP path accelerates)
# ----------------------------------------------------------------------------


class Result(dict):
    pass


def solve(prob, eps=1e-6, max_iters=20000, precondition=True, alpha=None,
          z0=None, eta0=None, xi_ref=None, record=False):
    """Iterate T from (z0, eta0) (zeros by default) until
    max(|xi1|_inf, |xi2|_inf) <= eps * max(1, |xi1_ref|_inf, |xi2_ref|_inf),
    where the reference residuals are those of the first step from zero."""
    D = Data(prob, precondition)
    F = Offline(D)
    a = step_size(D) if alpha is None else float(alpha)
    Y = D.layout
    z = np.zeros(Y.nz) if z0 is None else np.array(z0, float)
    eta = np.zeros(Y.neta) if eta0 is None else np.array(eta0, float)
    if xi_ref is None:
        zr, er = cp_step(D, F, np.zeros(Y.nz), np.zeros(Y.neta), a)
        x1, x2 = residuals(D, np.zeros(Y.nz), np.zeros(Y.neta), zr, er, a)
        xi_ref = (float(np.abs(x1).max()), float(np.abs(x2).max()))
    scale = max(1.0, xi_ref[0], xi_ref[1])
    hist = []
    status = "max_iters"
    it = 0
    r1 = r2 = np.inf
    for it in range(1, max_iters + 1):
        zp, ep = cp_step(D, F, z, eta, a)
        x1, x2 = residuals(D, z, eta, zp, ep, a)
        r1, r2 = float(np.abs(x1).max()), float(np.abs(x2).max())
        z, eta = zp, ep
        rel = max(r1, r2) / scale
        if record:
            hist.append(rel)
        if not np.isfinite(rel):
            status = "diverged"
            break
        if rel <= eps:
            status = "converged"
            break
    x = np.array([Y.x(z, i) for i in range(D.tree.n)])
    u = np.array([Y.u(z, i) for i in range(D.tree.n_nl)])
    xs, us = D.unscale(x, u)
    return Result(status=status, iters=it, z=z, eta=eta, s0=float(z[Y.z_s0]),
                  x=xs, u=us, xi1=r1, xi2=r2, rel_res=max(r1, r2) / scale,
                  xi_ref=xi_ref, alpha=a, history=hist, data=D)


# ----------------------------------------------------------------------------
# invariants used by the end-to-end pins
# ----------------------------------------------------------------------------


def nested_cost(prob, x, u):
    """Value of the nested risk objective (Sec. 3.5, with the conditional risk mappings of Sec. 3.4) for an unscaled (x, u):
    leaf values x^T Q_N x (+ qN^T x), then per non-leaf node the AV@R over its
    children of (stage cost on the edge, with its linear terms, + child value)."""
    T = Tree(prob["parent"], prob["prob"])
    n, nx, nu = T.n, int(prob["nx"]), int(prob["nu"])
    # cost matrices per node (the edge into j, or leaf j)
    Q, R, QN = (cost_matrices(prob, k, n) for k in ("Q", "R", "QN"))
    q = np.zeros((n, nx)) if prob.get("q") is None else np.asarray(prob["q"], float)
    r = np.zeros((n, nu)) if prob.get("r") is None else np.asarray(prob["r"], float)
    qN = np.zeros((n, nx)) if prob.get("qN") is None else np.asarray(prob["qN"], float)
    val = np.zeros(T.n)
    for j in T.leaves:
        val[j] = x[j] @ QN[j] @ x[j] + qN[j] @ x[j]
    for t in range(T.N - 1, -1, -1):
        for i in T.nodes(t):
            kids = T.ch[i]
            Z = np.array([x[i] @ Q[j] @ x[i] + u[i] @ R[j] @ u[i] + q[j] @ x[i] + r[j] @ u[i] + val[j]
                          for j in kids])
            if prob.get("risk") is not None:
                E, F, b, cone = node_risk(prob, i, T.p[kids])
                val[i] = conic_risk_value(Z, E, F, b, cone)
            else:
                val[i] = avar_ambiguity_form(Z, T.p[kids], float(prob["gamma"][i]))
    return float(val[0])


def dynamics_violation(prob, x, u):
    T = Tree(prob["parent"], prob["prob"])
    A, B = np.asarray(prob["A"]), np.asarray(prob["B"])
    c = prob.get("c")
    err = float(np.abs(x[0] - prob["x0"]).max())
    for j in range(1, T.n):
        i = T.anc[j]
        cj = 0.0 if c is None else c[j]
        err = max(err, float(np.abs(x[j] - A[j] @ x[i] - B[j] @ u[i] - cj).max()))
    return err


def risk_neutral_lq(prob):
    """Probability-weighted Riccati recursion on the tree: the exact solution
    when every AV@R parameter is 1 (AV@R_1 = E) and no constraint is active.
    Returns (V*, x, u) with V* = x0^T P0 x0."""
    T = Tree(prob["parent"], prob["prob"])
    nx, nu = int(prob["nx"]), int(prob["nu"])
    Qd, Rd, QNd = (cost_matrices(prob, k, T.n) for k in ("Q", "R", "QN"))
    A, B = np.asarray(prob["A"]), np.asarray(prob["B"])
    Ph = [None] * T.n
    Kf = [None] * T.n
    for j in T.leaves:
        Ph[j] = QNd[j]
    for t in range(T.N - 1, -1, -1):
        for i in T.nodes(t):
            kids = T.ch[i]
            p = T.p[kids]
            # the stage cost of the edge into child j weighs with p_j
            Huu = sum(pk * (Rd[j] + B[j].T @ Ph[j] @ B[j]) for pk, j in zip(p, kids))
            Hux = sum(pk * B[j].T @ Ph[j] @ A[j] for pk, j in zip(p, kids))
            Hxx = sum(pk * (Qd[j] + A[j].T @ Ph[j] @ A[j]) for pk, j in zip(p, kids))
            Kf[i] = -np.linalg.solve(Huu, Hux)
            Ph[i] = Hxx + Hux.T @ Kf[i]
    x = np.zeros((T.n, A.shape[1]))
    u = np.zeros((T.n_nl, B.shape[2]))
    x[0] = prob["x0"]
    for t in range(T.N):
        for i in T.nodes(t):
            u[i] = Kf[i] @ x[i]
            for j in T.ch[i]:
                x[j] = A[j] @ x[i] + B[j] @ u[i]
    return float(x[0] @ Ph[0] @ x[0]), x, u
