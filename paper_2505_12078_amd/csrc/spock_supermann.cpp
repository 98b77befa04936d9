// SuperMann iteration of SPOCK (Sec. 5.2, Alg. "SPOCK algorithm for RAOCPs")
// with Anderson's acceleration for the fast directions (Alg. "Anderson's
// acceleration", memory m; Sec. 6.2), in float64.
//
// Every vector operation runs on the device: T through the CP step kernels
// (the handle's descriptor reads copy 0 = v and writes copy 1 = T(v); a
// second descriptor reads the line-search trial and writes its image), L
// through the operator kernel, and the linear combinations and dot products
// through the vector kernels.  The host keeps only scalars: the m x m Gram
// matrix of the residual differences, the step-acceptance tests and the
// Anderson coefficients.
//
// Readings where the listing is garbled or silent:
//  - M-norm: <a, b>_M = a.b - alpha (<L a_z, b_eta> + <a_eta, L b_z>), the
//    preconditioning operator of Sec. 4.1, in which T is firmly nonexpansive;
//  - rho of step K2 uses twice the averagedness constant of T (1/2), not the
//    CP step size: rho = |r~|_M^2 - <r~, v~ - v>_M;
//  - the Anderson direction is psi = -r - (S - Y) kappa with Y the last m
//    residual differences, S the matching iterate differences and kappa the
//    least-squares solution of Y kappa = r;
//  - the least squares use the Cholesky factor of Y^T Y, which is the R of
//    Y's QR factorisation (Cholesky QR); the m x m Gram matrix is kept up to
//    date with m new dot products per iteration;
//  - after 30 halvings of tau the plain CP step (the tau -> 0 limit of K2)
//    is taken.

#include <cmath>
#include <cstring>
#include <initializer_list>
#include <utility>

#include "spock_internal.h"

namespace {

constexpr double kC0 = 0.99, kC1 = 0.99, kC2 = 0.99, kBeta = 0.5, kSigma = 0.1, kLambda = 1.0;
constexpr int kMaxBacktracks = 30;

// out = sum_i c_i in_i over the whole [z | pad | eta] vector
hipError_t combo(spock_problem* p, double* out, std::initializer_list<std::pair<const double*, double>> terms) {
    spk::VecCombo cb{};
    for (auto& t : terms) {
        cb.in[cb.n_in] = t.first;
        cb.c[cb.n_in] = t.second;
        ++cb.n_in;
    }
    return spk::launch_combo(out, cb, p->nzp + p->neta, p->stream);
}

// Solves G x = b for the symmetric positive definite m x m matrix G (slot
// order); false when G is numerically singular.
bool chol_solve(int m, const double G[8][8], const double* b, double* x) {
    double L[8][8] = {};
    double dmax = 0;
    for (int i = 0; i < m; ++i) dmax = std::max(dmax, G[i][i]);
    if (!(dmax > 0)) return false;
    for (int j = 0; j < m; ++j) {
        double d = G[j][j];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        if (!(d > 1e-13 * dmax)) return false;
        L[j][j] = std::sqrt(d);
        for (int i = j + 1; i < m; ++i) {
            double v = G[i][j];
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            L[i][j] = v / L[j][j];
        }
    }
    double y[8];
    for (int i = 0; i < m; ++i) {
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = v / L[i][i];
    }
    for (int i = m - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < m; ++k) v -= L[k][i] * x[k];
        x[i] = v / L[i][i];
    }
    for (int i = 0; i < m; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

}  // namespace

int32_t supermann_iterate(spock_problem* p, long long budget, spock_info* info) {
    SmWork& w = p->sm;
    DevSet<double>& s = p->s64;
    hipStream_t st = p->stream;
    const long long nzp = p->nzp, ne = p->neta, nv = nzp + ne;
    const int m = p->set.aa_memory;
    const double a = p->alpha;
    const double scale = std::max(1.0, std::max(p->xi_ref[0], p->xi_ref[1]));
    double* C0 = s.h.z[0];  // v
    double* C1 = s.h.z[1];  // T(v)
    double G[8][8] = {};     // Gram matrix of the Y ring, slot order
    int nY = 0;              // valid (S, Y) pairs
    int cur = 0;             // R[cur] holds the current residual
    long long k = 0, nT = 0, nK[3] = {0, 0, 0};
    double zeta = 0, omega_safe = 0;
    double rel = INFINITY, x1 = INFINITY, x2 = INFINITY;
    int32_t status = SPOCK_E_NOT_CONVERGED;
    for (;;) {
        // r_k = v_k - T(v_k); the residual difference r_k - r_{k-1} goes to
        // the slot of the iterate difference the previous update wrote
        HIP_TRY(combo(p, w.R[cur], {{C0, 1.0}, {C1, -1.0}}));
        const int q = k > 0 ? (int)((k - 1) % m) : -1;
        if (q >= 0) HIP_TRY(combo(p, w.Y[q], {{w.R[cur], 1.0}, {w.R[cur ^ 1], -1.0}}));
        HIP_TRY(spk::launch_apply_L<double>(s.d, p->n, w.R[cur], w.LR, st));
        const int nYn = q >= 0 ? std::min(nY + 1, m) : 0;
        spk::DotSet ds{};
        auto add = [&](const double* x, const double* y, long long n) {
            ds.a[ds.count] = x;
            ds.b[ds.count] = y;
            ds.n[ds.count] = n;
            ++ds.count;
        };
        if (q >= 0)
            for (int j = 0; j < nYn; ++j) add(w.Y[q], w.Y[j], nv);  // new row of the Gram matrix
        for (int j = 0; j < nYn; ++j) add(w.Y[j], w.R[cur], nv);    // Y^T r
        add(w.R[cur], w.R[cur], nv);
        add(w.LR, w.R[cur] + nzp, ne);
        HIP_TRY(spk::launch_dots(ds, w.partial, w.dots, st));
        HIP_TRY(hipMemcpyAsync(w.h_dots, w.dots, ds.count * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(w.h_dots + spk::kMaxDots, p->d_res, 2 * spk::kResSlots * sizeof(double),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        res_reduce(reinterpret_cast<const unsigned long long*>(w.h_dots + spk::kMaxDots), &x1, &x2);
        rel = rel_of(x1, x2, scale);
        if (k == 0) nT = 1;  // the step of v_0 was taken by the caller
        if (!std::isfinite(rel)) {
            status = SPOCK_E_DIVERGED;
            break;
        }
        if (rel <= p->set.eps) {
            status = SPOCK_OK;
            break;
        }
        if (k >= budget) break;
        int o = 0;
        if (q >= 0) {
            for (int j = 0; j < nYn; ++j) G[q][j] = G[j][q] = w.h_dots[o++];
            nY = nYn;
        }
        double b[8];
        for (int j = 0; j < nYn; ++j) b[j] = w.h_dots[o++];
        const double rr = w.h_dots[o++], lr = w.h_dots[o++];
        const double omega = std::sqrt(std::max(0.0, rr - 2.0 * a * lr));
        if (k == 0) zeta = omega_safe = omega;
        // Anderson direction (plain -r until m pairs are stored)
        double kap[8];
        if (nY == m && chol_solve(m, G, b, kap)) {
            spk::VecCombo cb{};
            cb.in[0] = w.R[cur];
            cb.c[0] = -1.0;
            cb.n_in = 1;
            for (int j = 0; j < m; ++j) {
                cb.in[cb.n_in] = w.S[j];
                cb.c[cb.n_in++] = -kap[j];
                cb.in[cb.n_in] = w.Y[j];
                cb.c[cb.n_in++] = kap[j];
            }
            HIP_TRY(spk::launch_combo(w.PSI, cb, nv, st));
        } else {
            HIP_TRY(combo(p, w.PSI, {{w.R[cur], -1.0}}));
        }
        double* Snext = w.S[k % m];
        bool stepped = false;  // T(v_{k+1}) already in copy 1
        if (omega <= kC0 * zeta) {
            // K0: educated update
            HIP_TRY(combo(p, C0, {{C0, 1.0}, {w.PSI, 1.0}}));
            HIP_TRY(combo(p, Snext, {{w.PSI, 1.0}}));
            zeta = omega;
            nK[0]++;
        } else {
            HIP_TRY(spk::launch_apply_L<double>(s.d, p->n, w.PSI, w.LPSI, st));
            double tau = 1.0;
            bool done = false;
            for (int bt = 0; bt < kMaxBacktracks; ++bt, tau *= kBeta) {
                HIP_TRY(combo(p, w.VT, {{C0, 1.0}, {w.PSI, tau}}));
                HIP_TRY(spk::launch_step<double>(w.d_trial, s.cfg, 0, 1, st));
                ++nT;
                HIP_TRY(combo(p, w.RT, {{w.VT, 1.0}, {w.TVT, -1.0}}));
                HIP_TRY(spk::launch_apply_L<double>(s.d, p->n, w.RT, w.LRT, st));
                spk::DotSet dt{};
                auto add2 = [&](const double* x, const double* y, long long n) {
                    dt.a[dt.count] = x;
                    dt.b[dt.count] = y;
                    dt.n[dt.count] = n;
                    ++dt.count;
                };
                add2(w.RT, w.RT, nv);
                add2(w.LRT, w.RT + nzp, ne);
                add2(w.RT, w.PSI, nv);
                add2(w.LRT, w.PSI + nzp, ne);
                add2(w.RT + nzp, w.LPSI, ne);
                HIP_TRY(spk::launch_dots(dt, w.partial, w.dots, st));
                HIP_TRY(hipMemcpyAsync(w.h_dots, w.dots, dt.count * sizeof(double), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                const double* h = w.h_dots;
                const double omt = std::sqrt(std::max(0.0, h[0] - 2.0 * a * h[1]));
                if (omega <= omega_safe && omt <= kC1 * omega) {
                    // K1: safeguarded update v <- v~ (its CP step is the trial's)
                    HIP_TRY(hipMemcpyAsync(C0, w.VT, nv * sizeof(double), hipMemcpyDeviceToDevice, st));
                    HIP_TRY(hipMemcpyAsync(C1, w.TVT, nv * sizeof(double), hipMemcpyDeviceToDevice, st));
                    HIP_TRY(combo(p, Snext, {{w.PSI, tau}}));
                    omega_safe = omt + std::pow(kC2, (double)k);
                    stepped = true;
                    nK[1]++;
                    done = true;
                    break;
                }
                const double rho = omt * omt - tau * (h[2] - a * (h[3] + h[4]));
                if (rho >= kSigma * omt * omega && omt > 0) {
                    // K2: generalized Krasnosel'skii-Mann update
                    const double c = kLambda * rho / (omt * omt);
                    HIP_TRY(combo(p, C0, {{C0, 1.0}, {w.RT, -c}}));
                    HIP_TRY(combo(p, Snext, {{w.RT, -c}}));
                    nK[2]++;
                    done = true;
                    break;
                }
            }
            if (!done) {
                // tau -> 0 limit of K2: the plain CP step v <- T(v)
                HIP_TRY(hipMemcpyAsync(C0, C1, nv * sizeof(double), hipMemcpyDeviceToDevice, st));
                HIP_TRY(combo(p, Snext, {{w.R[cur], -1.0}}));
                nK[2]++;
            }
        }
        ++k;
        if (!stepped) {
            HIP_TRY(spk::launch_step<double>(s.d, s.cfg, 0, 1, st));
            ++nT;
        }
        cur ^= 1;
    }
    s.par = 0;
    p->cur = SPOCK_FP64;
    info->iters = k;
    info->rel_res = rel;
    info->xi1_inf = x1;
    info->xi2_inf = x2;
    info->n_T = nT;
    info->n_K0 = nK[0];
    info->n_K1 = nK[1];
    info->n_K2 = nK[2];
    info->status = status;
    return status;
}
