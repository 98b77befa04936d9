"""FP64 CPU oracle of the SPOCK outer method: SuperMann around the CP operator
T with Anderson's acceleration (AA) for the fast directions.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path
and imports nothing from it; the operator T, L and the residuals come from the
CP oracle (spock_oracle.py) of this package.

Sections cited are those of arXiv:2505.12078:
* M-norm of the CP method (preconditioning operator M)   -> Sec. 4.1
* SPOCK algorithm (SuperMann steps K0, K1, K2)            -> Sec. 5.2, Alg. "SPOCK algorithm for RAOCPs"
* Anderson's acceleration, memory m                       -> Sec. 5.2, Alg. "Anderson's acceleration"; Sec. 6.2
* parameters c0 = c1 = c2 = 0.99, beta = 0.5, sigma = 0.1, lambda = 1, m = 3
                                                          -> Sec. 5.2, Sec. 6.2
* termination                                             -> Sec. 5.3

Readings (listed in the design doc):
  - M(z, eta) = (z - alpha L* eta, eta - alpha L z), so
    <a, b>_M = a_z.b_z + a_eta.b_eta - alpha (<L a_z, b_eta> + <a_eta, L b_z>)
    and |r|_M = sqrt(<r, r>_M); T is firmly nonexpansive in this norm.
  - The "2 alpha" in rho of step K2 is twice the averagedness constant of T
    (1/2 for a firmly nonexpansive T), not the CP step size: rho =
    |r~|_M^2 - <r~, v~ - v>_M.  With that, the K2 step is the relaxed
    projection of v onto the half-space that separates v from the fixed
    points, and tau -> 0 gives back the plain CP step.
  - AA direction: psi = -r - (S - Y) kappa with kappa the least-squares
    solution of Y kappa = r, Y the last m residual differences and S the
    matching iterate differences (type-II Anderson, the quasi-Newton form of
    SuperMann's Sec. VI).  The listing stores residuals in M_r and their
    differences in M_d; taken literally (M_r - M_d holds the previous
    residuals in place of the iterate differences) the direction is not a
    quasi-Newton direction; `aa_kind="literal"` keeps that form for
    comparison.  The least squares use the QR factorisation of Y, as the
    paper does.
  - The line search on tau ends by itself (tau -> 0 makes rho = |r|_M^2 >=
    sigma |r|_M^2); after `max_backtracks` halvings the plain CP step (the
    tau = 0 limit of K2 with lambda = 1) is taken.
  - Termination: rel_res of the CP step from v^(k) (Sec. 5.3, same scale as
    the plain method), checked at every k.
"""
from __future__ import annotations

import numpy as np

from . import spock_oracle as O


def m_inner(D, alpha, az, ae, bz, be):
    """<a, b>_M with M(z, eta) = (z - alpha L* eta, eta - alpha L z) (Sec. 4.1)."""
    return float(az @ bz + ae @ be - alpha * (O.apply_L(D, az) @ be + ae @ O.apply_L(D, bz)))


def m_norm(D, alpha, rz, re):
    v = m_inner(D, alpha, rz, re, rz, re)
    return float(np.sqrt(max(v, 0.0)))


class Anderson:
    """Memory of the last m + 1 residuals and iterates; fast direction of
    Alg. "Anderson's acceleration" (type-II form, see the module header)."""

    def __init__(self, m=3, kind="type2"):
        self.m = m
        self.kind = kind
        self.r = []   # residuals, newest first
        self.v = []   # iterates at which they were taken, newest first
        self.k = 0

    def direction(self, v, r):
        self.r.insert(0, r.copy())
        self.v.insert(0, v.copy())
        del self.r[self.m + 1:]
        del self.v[self.m + 1:]
        k = self.k
        self.k += 1
        if k < self.m:   # the first m directions are plain
            return -r
        Y = np.stack([self.r[j] - self.r[j + 1] for j in range(self.m)], axis=1)
        if self.kind == "literal":
            Mr = np.stack(self.r[:self.m], axis=1)
            SmY = Mr - Y
        else:
            S = np.stack([self.v[j] - self.v[j + 1] for j in range(self.m)], axis=1)
            SmY = S - Y
        kappa = aa_least_squares(Y, r)
        return -r - SmY @ kappa


def aa_least_squares(Y, r):
    """kappa = argmin |Y kappa - r|_2 through the QR factorisation of Y:
    R kappa = Q^T r (Alg. "Anderson's acceleration")."""
    Q, R = np.linalg.qr(Y)
    return np.linalg.solve(R, Q.T @ r)


def solve(prob, eps=1e-6, max_iters=20000, precondition=True, alpha=None, m=3, c0=0.99, c1=0.99, c2=0.99,
          beta=0.5, sigma=0.1, lam=1.0, aa_kind="type2", max_backtracks=30, z0=None, eta0=None, xi_ref=None):
    """SPOCK: SuperMann over T with AA directions, from (z0, eta0) (zeros by
    default), until rel_res of the CP step at v^(k) is <= eps.  Returns the
    same fields as the plain CP oracle's solve, plus the counts of K0, K1, K2
    steps and of T applications."""
    D = O.Data(prob, precondition)
    F = O.Offline(D)
    a = O.step_size(D) if alpha is None else float(alpha)
    Y = D.layout
    nz = Y.nz
    z = np.zeros(nz) if z0 is None else np.array(z0, float)
    eta = np.zeros(Y.neta) if eta0 is None else np.array(eta0, float)
    if xi_ref is None:
        zr, er = O.cp_step(D, F, np.zeros(nz), np.zeros(Y.neta), a)
        x1, x2 = O.residuals(D, np.zeros(nz), np.zeros(Y.neta), zr, er, a)
        xi_ref = (float(np.abs(x1).max()), float(np.abs(x2).max()))
    scale = max(1.0, xi_ref[0], xi_ref[1])

    def T(v):
        return np.concatenate(O.cp_step(D, F, v[:nz], v[nz:], a))

    def mnorm(r):
        return m_norm(D, a, r[:nz], r[nz:])

    def minner(p, q):
        return m_inner(D, a, p[:nz], p[nz:], q[:nz], q[nz:])

    v = np.concatenate([z, eta])
    aa = Anderson(m, aa_kind)
    Tv = T(v)
    n_T = 1
    r = v - Tv
    zeta = mnorm(r)
    omega_safe = zeta
    counts = {"K0": 0, "K1": 0, "K2": 0, "T": 0}
    status = "max_iters"
    k = 0
    rel = np.inf
    r1 = r2 = np.inf
    while True:
        # termination on the CP step from v^(k) (Sec. 5.3)
        x1, x2 = O.residuals(D, v[:nz], v[nz:], Tv[:nz], Tv[nz:], a)
        r1, r2 = float(np.abs(x1).max()), float(np.abs(x2).max())
        rel = max(r1, r2) / scale
        if not np.isfinite(rel):
            status = "diverged"
            break
        if rel <= eps:
            status = "converged"
            break
        if k >= max_iters:
            break
        psi = aa.direction(v, r)
        omega = mnorm(r)
        done = None
        if omega <= c0 * zeta:                       # K0: educated step
            v = v + psi
            zeta = omega
            counts["K0"] += 1
        else:
            tau = 1.0
            for _ in range(max_backtracks):
                vt = v + tau * psi
                Tvt = T(vt)
                n_T += 1
                rt = vt - Tvt
                omt = mnorm(rt)
                if omega <= omega_safe and omt <= c1 * omega:   # K1: safeguarded step
                    v = vt
                    omega_safe = omt + c2 ** k
                    counts["K1"] += 1
                    done = "K1"
                    break
                rho = omt ** 2 - minner(rt, vt - v)
                if rho >= sigma * omt * omega:                   # K2: generalized KM step
                    v = v - (lam * rho / omt ** 2) * rt
                    counts["K2"] += 1
                    done = True
                    break
                tau *= beta
            if not done:                                          # tau -> 0 limit of K2
                v = Tv.copy()
                counts["K2"] += 1
        k += 1
        if done == "K1":      # T(v~) is already known
            Tv, r = Tvt, rt
        else:
            Tv = T(v)
            n_T += 1
            r = v - Tv
    counts["T"] = n_T
    z, eta = v[:nz], v[nz:]
    x = np.array([Y.x(z, i) for i in range(D.tree.n)])
    u = np.array([Y.u(z, i) for i in range(D.tree.n_nl)])
    xs, us = D.unscale(x, u)
    return O.Result(status=status, iters=k, z=z, eta=eta, s0=float(z[Y.z_s0]), x=xs, u=us, xi1=r1, xi2=r2,
                    rel_res=rel, xi_ref=xi_ref, alpha=a, counts=counts, data=D)
