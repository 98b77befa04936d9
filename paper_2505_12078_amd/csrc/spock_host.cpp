// Host side of the SPOCK CP-step library: validation, the diagonal scaling of
// Sec. 5.4, the offline factorisation of Alg. 1 (float64), the exact operator
// norm of L (Sec. 4.4), the device memory plan, the solve loop and the C ABI
// declared in include/spock.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>
#include <unordered_map>
#include <map>

#include "../../include/spock.h"
#include "spock_dev.h"

#include "spock_internal.h"

using spk::ProbDev;

thread_local std::string g_err;

std::recursive_mutex& hip_setup_mutex() {
    static std::recursive_mutex mu;
    return mu;
}

int32_t fail(int32_t code, const std::string& msg) {
    g_err = msg;
    return code;
}

// ---------------------------------------------------------------------------
// small dense float64 kernels for the offline factorisation (row-major)
// ---------------------------------------------------------------------------

// C (M x N) = A (M x K) * B (K x N)  [+ C if acc]
static void mm(int M, int N, int K, const double* A, const double* B, double* C, bool acc) {
    if (!acc) std::fill(C, C + (size_t)M * N, 0.0);
    for (int i = 0; i < M; ++i) {
        double* c = C + (size_t)i * N;
        for (int k = 0; k < K; ++k) {
            const double a = A[(size_t)i * K + k];
            const double* b = B + (size_t)k * N;
            for (int j = 0; j < N; ++j) c[j] += a * b[j];
        }
    }
}

// C (M x N) += A^T * B with A (K x M), B (K x N)
static void mtm_acc(int M, int N, int K, const double* A, const double* B, double* C) {
    for (int k = 0; k < K; ++k) {
        const double* a = A + (size_t)k * M;
        const double* b = B + (size_t)k * N;
        for (int i = 0; i < M; ++i) {
            const double ai = a[i];
            double* c = C + (size_t)i * N;
            for (int j = 0; j < N; ++j) c[j] += ai * b[j];
        }
    }
}

// In-place Cholesky (lower) of an SPD matrix; false if not positive definite.
static bool cholesky(int n, double* A) {
    for (int j = 0; j < n; ++j) {
        double s = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(s > 0)) return false;
        const double l = std::sqrt(s);
        A[(size_t)j * n + j] = l;
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = t / l;
        }
        for (int k = j + 1; k < n; ++k) A[(size_t)j * n + k] = 0.0;
    }
    return true;
}

// inverse of L L^T from the Cholesky factor L
static void chol_inverse(int n, const double* L, double* inv) {
    std::vector<double> Li((size_t)n * n, 0.0);  // L^-1 (lower)
    for (int j = 0; j < n; ++j) {
        Li[(size_t)j * n + j] = 1.0 / L[(size_t)j * n + j];
        for (int i = j + 1; i < n; ++i) {
            double s = 0;
            for (int k = j; k < i; ++k) s -= L[(size_t)i * n + k] * Li[(size_t)k * n + j];
            Li[(size_t)i * n + j] = s / L[(size_t)i * n + i];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = 0;
            for (int k = i; k < n; ++k) s += Li[(size_t)k * n + i] * Li[(size_t)k * n + j];
            inv[(size_t)i * n + j] = s;
            inv[(size_t)j * n + i] = s;
        }
}

// Eigen-decomposition A = V diag(w) V^T of a symmetric n x n matrix by cyclic
// Jacobi rotations (V's columns are the eigenvectors).
static void sym_eig(int n, const double* A, std::vector<double>& w, std::vector<double>& V) {
    std::vector<double> a(A, A + (size_t)n * n);
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double v = a[(size_t)i * n + j] * a[(size_t)i * n + j];
                tot += v;
                if (i != j) off += v;
            }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - sn * akq;
                    a[(size_t)k * n + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - sn * aqk;
                    a[(size_t)q * n + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - sn * vkq;
                    V[(size_t)k * n + q] = sn * vkp + c * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
}

// V diag(f(w)) V^T
template <typename Fn>
static std::vector<double> eig_fn(int n, const std::vector<double>& w, const std::vector<double>& V, Fn f) {
    std::vector<double> out((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k) {
        const double fk = f(w[k]);
        for (int i = 0; i < n; ++i) {
            const double vik = V[(size_t)i * n + k] * fk;
            for (int j = 0; j < n; ++j) out[(size_t)i * n + j] += vik * V[(size_t)j * n + k];
        }
    }
    return out;
}

template <typename F>
static void parallel_for(int n, F f) {
    unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::min<unsigned>(hw ? hw : 1, 32);
    if (n < 4 || nt <= 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    nt = std::min(nt, n);
    std::atomic<int> next(0);
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&] {
            for (int i; (i = next.fetch_add(1)) < n;) f(i);
        });
    for (auto& x : th) x.join();
}

// ---------------------------------------------------------------------------
// memory plan: one arena, 256-byte aligned sub-buffers
// ---------------------------------------------------------------------------

struct Arena {
    char* base;
    size_t off = 0;
    explicit Arena(void* b) : base((char*)b) {}
    template <typename T>
    T* take(long long count) {
        off = (off + 255) & ~(size_t)255;
        T* r = base ? (T*)(base + off) : nullptr;
        off += (size_t)std::max<long long>(count, 1) * sizeof(T);
        return r;
    }
};

template <typename real>
static void carve_set(Arena& a, spock_problem* p, DevSet<real>& s) {
    ProbDev<real>& h = s.h;
    const int n = p->n, nl = p->n_nl, nx = p->nx, nu = p->nu, m = p->m;
    constexpr int V = spk::tile_vec<real>();
    h.T1_stride = spk::tile_elems(nu, nx, V);
    h.T2M_stride = spk::tile_elems(nx, m, V);
    h.T2R_stride = spk::tile_elems(nu, nu, V);
    h.T3_stride = spk::tile_elems(m, nx, V);
    h.T4_stride = spk::tile_elems(nx, nu, V);
    const long long pad = spk::tile_pad_elems<real>();
    h.T1 = a.take<real>((long long)nl * h.T1_stride + pad);
    h.T2M = a.take<real>((long long)n * h.T2M_stride + pad);
    h.T2R = a.take<real>((long long)nl * h.T2R_stride + pad);
    h.T3 = a.take<real>((long long)n * h.T3_stride + pad);
    h.T4 = a.take<real>((long long)nl * h.T4_stride + pad);
    h.c = p->affine ? a.take<real>((long long)n * nx) : nullptr;
    h.Pc = p->affine ? a.take<real>((long long)n * nx) : nullptr;
    h.qh = a.take<real>(nx);
    h.rh = a.take<real>(nu);
    h.qnh = a.take<real>(nx);
    h.gx = a.take<real>(nx);
    h.gu = a.take<real>(nu);
    h.gb = a.take<real>(nx);
    h.gxN = a.take<real>(nx);
    h.gbN = a.take<real>(nx);
    h.lo = a.take<real>(std::max(m, p->nbox));
    h.hi = a.take<real>(std::max(m, p->nbox));
    h.loN = a.take<real>(std::max(nx, p->nboxN));
    h.hiN = a.take<real>(std::max(nx, p->nboxN));
    h.prob = a.take<real>(n);
    h.gamma = a.take<real>(nl);
    h.sa = p->has_lin ? a.take<real>((long long)(n - 1) * (m + 2)) : nullptr;
    h.saN = p->has_lin ? a.take<real>((long long)p->n_leaf * (nx + 2)) : nullptr;
    h.ck = p->coupled ? a.take<real>((long long)n * nu) : nullptr;
    h.qh_e = p->edge_cost ? a.take<real>((long long)n * nx) : nullptr;
    h.rh_e = p->edge_cost ? a.take<real>((long long)n * nu) : nullptr;
    h.qnh_l = p->leaf_cost ? a.take<real>((long long)p->n_leaf * nx) : nullptr;
    h.Hq_e = p->dense_edge ? a.take<real>((long long)n * nx * nx) : nullptr;
    h.Hr_e = p->dense_edge ? a.take<real>((long long)n * nu * nu) : nullptr;
    h.HqN_l = p->dense_leaf ? a.take<real>((long long)p->n_leaf * nx * nx) : nullptr;
    h.Gt = p->gen ? a.take<real>((long long)p->nbox * m) : nullptr;
    h.GtT = p->gen ? a.take<real>((long long)p->nbox * m) : nullptr;
    h.GNt = p->genN ? a.take<real>((long long)p->nboxN * nx) : nullptr;
    h.GNtT = p->genN ? a.take<real>((long long)p->nboxN * nx) : nullptr;
    h.rdata = p->grisk ? a.take<real>((long long)p->rdata.size()) : nullptr;
    h.x0 = a.take<real>(nx);
    // z and eta of one copy are one vector [z | zero pad | eta] (the
    // SuperMann iteration combines whole iterates)
    for (int k = 0; k < 2; ++k) {
        h.z[k] = a.take<real>(p->nzp + p->neta);
        h.eta[k] = h.z[k] + p->nzp;
    }
    h.d = a.take<real>((long long)nl * nu);
    h.e = a.take<real>((long long)n * m);
    h.h0 = a.take<real>((long long)n * nx);
    h.ub = a.take<real>((long long)nl * nu);
    s.d = a.take<ProbDev<real>>(1);
}

static void carve(Arena& a, spock_problem* p) {
    p->d_tree = a.take<int>(3LL * p->n + 4);
    p->d_roff = p->grisk ? a.take<long long>(p->n_nl) : nullptr;
    p->d_rint = p->grisk ? a.take<int>(2LL * p->n_nl) : nullptr;
    p->d_cnt = a.take<int>(p->n);
    p->d_path = a.take<int4>((long long)p->n_leaf * (p->N + 1));
    p->d_top = a.take<int>(p->n_leaf);
    p->d_one = a.take<int>(4);  // [0] constant 1: the problem's active flag
    p->d_tasks = a.take<int2>(p->n_leaf);
    p->n_ntasks = (p->n + spk::kMaxNodeWaves - 1) / spk::kMaxNodeWaves * spk::kMaxNodeWaves;
    p->d_ntasks = a.take<int2>(p->n_ntasks);
    p->d_ninfo = a.take<int4>(p->n_ntasks);
    p->d_res = a.take<unsigned long long>(2 * spk::kResSlots);
    const long long nv = std::max(p->nz, p->neta);
    p->d_stash_z = a.take<double>(nv);
    p->d_stash_e = a.take<double>(nv);
    carve_set(a, p, p->s64);
    carve_set(a, p, p->s32);
    if (p->set.method == SPOCK_SUPERMANN) {
        // float64 vectors of the SuperMann iteration, each [z | pad | eta]
        SmWork& w = p->sm;
        const long long nv = p->nzp + p->neta;
        for (auto& r : w.R) r = a.take<double>(nv);
        w.PSI = a.take<double>(nv);
        w.VT = a.take<double>(nv);
        w.TVT = a.take<double>(nv);
        w.RT = a.take<double>(nv);
        for (int j = 0; j < p->set.aa_memory; ++j) {
            w.Y[j] = a.take<double>(nv);
            w.S[j] = a.take<double>(nv);
        }
        w.LR = a.take<double>(p->neta);
        w.LPSI = a.take<double>(p->neta);
        w.LRT = a.take<double>(p->neta);
        w.partial = a.take<double>((long long)spk::kMaxDots * spk::kDotBlocks);
        w.dots = a.take<double>(spk::kMaxDots);
        w.d_trial = a.take<ProbDev<double>>(1);
    }
}

// ---------------------------------------------------------------------------
// validation and layout
// ---------------------------------------------------------------------------

static bool finite_all(const double* v, long long n) {
    for (long long k = 0; k < n; ++k)
        if (!std::isfinite(v[k])) return false;
    return true;
}

// Cost diagonals of the edge into node j (shared or per edge) and of leaf j.
static double Qd(const spock_problem_desc* d, int j, int k) {
    if (d->Q_dense) return d->Q_dense[((size_t)j * d->nx + k) * d->nx + k];
    return d->Q_edge ? d->Q_edge[(size_t)j * d->nx + k] : d->Q_diag[k];
}
static double Rd(const spock_problem_desc* d, int j, int k) {
    if (d->R_dense) return d->R_dense[((size_t)j * d->nu + k) * d->nu + k];
    return d->R_edge ? d->R_edge[(size_t)j * d->nu + k] : d->R_diag[k];
}
static double QNd(const spock_problem_desc* d, int j, int k) {
    if (d->QN_dense) return d->QN_dense[((size_t)j * d->nx + k) * d->nx + k];
    return d->QN_leaf ? d->QN_leaf[(size_t)j * d->nx + k] : d->QN_diag[k];
}
// The full cost matrix of edge / leaf j (dense, or the diagonal form).
static std::vector<double> cost_mat(const double* dense, int j, int dim, double (*diag)(const spock_problem_desc*, int, int),
                                    const spock_problem_desc* d) {
    std::vector<double> M((size_t)dim * dim, 0.0);
    if (dense) {
        std::copy(dense + (size_t)j * dim * dim, dense + (size_t)(j + 1) * dim * dim, M.begin());
    } else {
        for (int k = 0; k < dim; ++k) M[(size_t)k * dim + k] = diag(d, j, k);
    }
    return M;
}

static int32_t validate_and_layout(const spock_problem_desc* d, spock_problem* p) {
    if (!d) return fail(SPOCK_E_INVALID, "null problem description");
    const int n = d->n_nodes;
    if (n < 2) return fail(SPOCK_E_INVALID, "a tree needs at least two nodes");
    if (d->nx < 1 || d->nu < 1) return fail(SPOCK_E_INVALID, "nx and nu must be >= 1");
    if (!d->parent || !d->cond_prob || !d->A || !d->B || !(d->Q_diag || d->Q_edge || d->Q_dense) ||
        !(d->R_diag || d->R_edge || d->R_dense) || !(d->QN_diag || d->QN_leaf || d->QN_dense) ||
        (!d->Gamma && (!d->x_lo || !d->x_hi || !d->u_lo || !d->u_hi)) ||
        (!d->GammaN && (!d->xN_lo || !d->xN_hi)) || (!d->gamma && !d->risk_ny) ||
        (d->risk_ny && (!d->risk_nnu || !d->risk_E || !d->risk_b || !d->risk_cone)) ||
        (d->Gamma && (!d->con_lo || !d->con_hi)) || (d->GammaN && (!d->conN_lo || !d->conN_hi)))
        return fail(SPOCK_E_INVALID, "missing array in the problem description");
    if (d->parent[0] != -1) return fail(SPOCK_E_INVALID, "parent[0] must be -1");
    p->n = n;
    p->nx = d->nx;
    p->nu = d->nu;
    p->m = d->nx + d->nu;
    p->parent.assign(d->parent, d->parent + n);
    p->n_ch.assign(n, 0);
    p->first_child.assign(n, -1);
    std::vector<int> stage(n, 0);
    for (int j = 1; j < n; ++j) {
        const int i = d->parent[j];
        if (i < 0 || i >= j) return fail(SPOCK_E_INVALID, "parent[j] must lie in [0, j)");
        if (j > 1 && i < d->parent[j - 1])
            return fail(SPOCK_E_INVALID, "nodes must be numbered stage by stage (children contiguous)");
        if (p->n_ch[i] == 0) p->first_child[i] = j;
        p->n_ch[i]++;
        stage[j] = stage[i] + 1;
    }
    int nl = 0;
    while (nl < n && p->n_ch[nl] > 0) ++nl;
    for (int j = nl; j < n; ++j)
        if (p->n_ch[j] != 0) return fail(SPOCK_E_INVALID, "non-leaf nodes must precede all leaves");
    p->n_nl = nl;
    p->n_leaf = n - nl;
    p->N = stage[n - 1];
    for (int j = nl; j < n; ++j)
        if (stage[j] != p->N) return fail(SPOCK_E_INVALID, "every leaf must sit at the last stage");
    if (p->N + 1 > spk::kMaxDepth) return fail(SPOCK_E_INVALID, "horizon too long");
    p->max_ch = *std::max_element(p->n_ch.begin(), p->n_ch.end());
    for (int j = 0; j < n; ++j)
        if (!(d->cond_prob[j] > 0) || !std::isfinite(d->cond_prob[j]))
            return fail(SPOCK_E_INVALID, "probabilities must be positive");
    for (int i = 0; i < nl; ++i) {
        double s = 0;
        for (int c = 0; c < p->n_ch[i]; ++c) s += d->cond_prob[p->first_child[i] + c];
        if (std::fabs(s - 1.0) > 1e-9) return fail(SPOCK_E_INVALID, "children probabilities must sum to 1");
    }
    const int nx = d->nx, nu = d->nu;
    if (!finite_all(d->A + (size_t)nx * nx, (long long)(n - 1) * nx * nx) ||
        !finite_all(d->B + (size_t)nx * nu, (long long)(n - 1) * nx * nu) ||
        (d->c && !finite_all(d->c + nx, (long long)(n - 1) * nx)) || (d->gamma && !finite_all(d->gamma, nl)))
        return fail(SPOCK_E_INVALID, "non-finite problem data");
    // cost diagonals: every edge's Q, R and every leaf's QN positive and finite
    for (int j = 1; j < n; ++j) {
        for (int k = 0; k < nx; ++k) {
            const double v = Qd(d, j, k);
            if (!(v > 0) || !std::isfinite(v)) return fail(SPOCK_E_INVALID, "Q must be finite and > 0");
            if (j >= nl) {
                const double w = QNd(d, j, k);
                if (!(w > 0) || !std::isfinite(w)) return fail(SPOCK_E_INVALID, "QN must be finite and > 0");
            }
        }
        for (int k = 0; k < nu; ++k) {
            // diagonal R may have zero entries (inputs without quadratic cost)
            const double v = Rd(d, j, k);
            if (!(d->R_dense ? v > 0 : v >= 0) || !std::isfinite(v))
                return fail(SPOCK_E_INVALID, "R must be finite and > 0 (diagonal R: >= 0)");
        }
    }
    // linear cost terms: edge rows 1..n-1, leaf rows of qN
    if ((d->q && !finite_all(d->q + nx, (long long)(n - 1) * nx)) ||
        (d->r && !finite_all(d->r + nu, (long long)(n - 1) * nu)) ||
        (d->qN && !finite_all(d->qN + (size_t)nl * nx, (long long)(n - nl) * nx)))
        return fail(SPOCK_E_INVALID, "non-finite linear cost terms");
    p->has_lin = (d->q || d->r || d->qN) ? 1 : 0;
    // Prop. 1 with R singular: a linear term on an input without quadratic cost
    p->coupled = 0;
    if (d->r && !d->R_dense)
        for (int j = 1; j < n && !p->coupled; ++j)
            for (int k = 0; k < nu; ++k)
                if (Rd(d, j, k) == 0.0 && d->r[(size_t)j * nu + k] != 0.0) p->coupled = 1;
    // dense costs: finite and symmetric (definiteness is checked with their
    // eigenvalues when the square roots are taken)
    auto dense_ok = [&](const double* M, int dim, int j0, int j1) {
        if (!M) return true;
        for (int j = j0; j < j1; ++j) {
            const double* A = M + (size_t)j * dim * dim;
            if (!finite_all(A, (long long)dim * dim)) return false;
            for (int a = 0; a < dim; ++a)
                for (int b = 0; b < a; ++b)
                    if (std::fabs(A[a * dim + b] - A[b * dim + a]) > 1e-12 * (std::fabs(A[a * dim + b]) + 1e-300) &&
                        A[a * dim + b] != A[b * dim + a])
                        return false;
        }
        return true;
    };
    if (!dense_ok(d->Q_dense, nx, 1, n) || !dense_ok(d->R_dense, nu, 1, n) || !dense_ok(d->QN_dense, nx, nl, n))
        return fail(SPOCK_E_INVALID, "dense cost matrices must be finite and symmetric");
    p->dense_edge = (d->Q_dense || d->R_dense) ? 1 : 0;
    p->dense_leaf = d->QN_dense ? 1 : 0;
    p->edge_cost = (!p->dense_edge && (d->Q_edge || d->R_edge)) ? 1 : 0;
    p->leaf_cost = (!p->dense_leaf && d->QN_leaf) ? 1 : 0;
    // general constraints: finite rows, bounds lo <= hi (infinite allowed)
    p->gen = d->Gamma ? 1 : 0;
    p->genN = d->GammaN ? 1 : 0;
    auto rows_ok = [&](const double* G, int rows, int cols, const double* lo, const double* hi) {
        if (!finite_all(G, (long long)rows * cols)) return false;
        for (int r = 0; r < rows; ++r)
            if (!(lo[r] <= hi[r])) return false;  // also rejects NaN
        return true;
    };
    if (p->gen && (d->n_con < 1 || d->n_con > 512 || !rows_ok(d->Gamma, d->n_con, p->m, d->con_lo, d->con_hi)))
        return fail(SPOCK_E_INVALID, "general constraints: 1 <= n_con <= 512, finite Gamma, con_lo <= con_hi");
    if (p->genN && (d->n_conN < 1 || d->n_conN > 512 || !rows_ok(d->GammaN, d->n_conN, nx, d->conN_lo, d->conN_hi)))
        return fail(SPOCK_E_INVALID, "general leaf constraints: 1 <= n_conN <= 512, finite GammaN, conN_lo <= conN_hi");
    for (int k = 0; k < nx; ++k) {
        if (!p->gen && (!(d->x_lo[k] <= d->x_hi[k]) || std::isnan(d->x_lo[k])))
            return fail(SPOCK_E_INVALID, "state bounds must satisfy lo <= hi");
        if (!p->genN && (!(d->xN_lo[k] <= d->xN_hi[k]) || std::isnan(d->xN_lo[k])))
            return fail(SPOCK_E_INVALID, "state bounds must satisfy lo <= hi");
    }
    for (int k = 0; k < nu; ++k)
        if (!p->gen && !(d->u_lo[k] <= d->u_hi[k]))
            return fail(SPOCK_E_INVALID, "input bounds must satisfy lo <= hi");
    p->grisk = d->risk_ny ? 1 : 0;
    for (int i = 0; i < nl && !p->grisk; ++i)
        if (!(d->gamma[i] >= 0 && d->gamma[i] <= 1)) return fail(SPOCK_E_INVALID, "gamma must lie in [0, 1]");
    if (p->grisk) {
        // general coherent risks: sizes, finite data, cone codes, and the
        // inverse Gram matrix of G = [E^T -I -I; F^T 0 0] per node (Sec. 4.3)
        p->rny.assign(nl, 0);
        p->rnnu.assign(nl, 0);
        p->roff.assign(nl, 0);
        long long ie = 0, iF = 0, ib = 0, tot = 0;
        for (int i = 0; i < nl; ++i) {
            const int ny = d->risk_ny[i], nnu = d->risk_nnu[i], k = p->n_ch[i];
            if (ny < 1 || ny > 128 || nnu < 0 || k + nnu > 64)
                return fail(SPOCK_E_INVALID, "general risks: 1 <= ny <= 128 and k + nnu <= 64 per node");
            p->rny[i] = ny;
            p->rnnu[i] = nnu;
            p->roff[i] = tot;
            tot += (long long)ny * k + (long long)ny * nnu + 2LL * ny + (long long)(k + nnu) * (k + nnu);
        }
        p->rdata.assign(tot, 0.0);
        for (int i = 0; i < nl; ++i) {
            const int ny = p->rny[i], nnu = p->rnnu[i], k = p->n_ch[i], g = k + nnu;
            double* blk = p->rdata.data() + p->roff[i];
            double* E = blk;
            double* F = E + (size_t)ny * k;
            double* b = F + (size_t)ny * nnu;
            double* cone = b + ny;
            double* M = cone + ny;
            if (!finite_all(d->risk_E + ie, (long long)ny * k) || (nnu > 0 && (!d->risk_F || !finite_all(d->risk_F + iF, (long long)ny * nnu))) ||
                !finite_all(d->risk_b + ib, ny))
                return fail(SPOCK_E_INVALID, "general risks: non-finite E, F or b");
            std::copy(d->risk_E + ie, d->risk_E + ie + (long long)ny * k, E);
            if (nnu > 0) std::copy(d->risk_F + iF, d->risk_F + iF + (long long)ny * nnu, F);
            std::copy(d->risk_b + ib, d->risk_b + ib + ny, b);
            // cone codes: 0 R_+, 1 {0}, 2 the head row t of a second-order cone
            // block {(t, w): ||w|| <= t}, 3 its rows of w; stored for the
            // kernels as 0, 1, 2 and, for a block's w rows, -1 - (head row)
            int head = -1;
            for (int r = 0; r < ny; ++r) {
                const int code = d->risk_cone[ib + r];
                if (code < 0 || code > 3) return fail(SPOCK_E_INVALID, "general risks: cone codes are 0, 1, 2 or 3");
                if (code == 3 && head < 0)
                    return fail(SPOCK_E_INVALID, "general risks: cone code 3 must follow a 2 or a 3");
                if (code == 2) head = r;
                else if (code != 3) head = -1;
                cone[r] = code == 3 ? -1.0 - head : (double)code;
            }
            // G G^T = [E^T E + 2 I, E^T F; F^T E, F^T F]; invert through Cholesky
            std::vector<double> GG((size_t)g * g, 0.0);
            for (int a = 0; a < g; ++a)
                for (int c = 0; c < g; ++c) {
                    double v = 0;
                    for (int r = 0; r < ny; ++r) {
                        const double ga = a < k ? E[(size_t)r * k + a] : F[(size_t)r * nnu + a - k];
                        const double gc = c < k ? E[(size_t)r * k + c] : F[(size_t)r * nnu + c - k];
                        v += ga * gc;
                    }
                    if (a == c && a < k) v += 2.0;
                    GG[(size_t)a * g + c] = v;
                }
            if (!cholesky(g, GG.data())) return fail(SPOCK_E_INVALID, "general risks: G must have full row rank");
            chol_inverse(g, GG.data(), M);
            ie += (long long)ny * k;
            iF += (long long)ny * nnu;
            ib += ny;
        }
    }
    if (std::isnan(d->x_ball) || std::isnan(d->xN_ball)) return fail(SPOCK_E_INVALID, "NaN ball radius");

    p->has_ball = !p->gen && d->x_ball > 0;
    p->has_ballN = !p->genN && d->xN_ball > 0;
    p->affine = d->c != nullptr;
    p->nbox = p->gen ? d->n_con : p->m;
    p->nboxN = p->genN ? d->n_conN : nx;
    p->nc = p->nbox + (p->has_ball ? nx : 0);
    p->ncN = p->nboxN + (p->has_ballN ? nx : 0);
    p->y_off.assign(nl + 1, 0);
    for (int i = 0; i < nl; ++i) p->y_off[i + 1] = p->y_off[i] + (p->grisk ? p->rny[i] : 2 * p->n_ch[i] + 1);
    p->ny = p->y_off[nl];
    long long o = 1;
    p->z_x = o; o += (long long)n * nx;
    p->z_u = o; o += (long long)nl * nu;
    p->z_y = o; o += p->ny;
    p->z_tau = o; o += n - 1;
    p->z_s = o; o += n - 1;
    p->nz = o;
    p->nzp = (o + 63) & ~63LL;
    o = 0;
    p->e_y = o; o += p->ny;
    p->e_s = o; o += nl;
    p->e_c = o; o += (long long)nl * p->nc;
    p->e_soc = o; o += (long long)(n - 1) * (p->m + 2);
    p->e_cN = o; o += (long long)p->n_leaf * p->ncN;
    p->e_socN = o; o += (long long)p->n_leaf * (nx + 2);
    p->neta = o;
    p->M_stride = ((long long)nx * p->m + 31) / 32 * 32;
    p->KR_stride = ((long long)nu * p->m + 31) / 32 * 32;
    // the sweeps keep a vector of nx and of nu entries as 4 entries per lane
    if (p->nx > 256 || p->nu > 256) return fail(SPOCK_E_INVALID, "nx and nu must not exceed 256");
    // stage the per-child inputs of as many children as one wavefront's LDS
    // holds (up to kStageKids); wider nodes read theirs in place
    // (general risks: none staged, their y blocks have other lengths)
    p->stage_kids = p->grisk ? 0 : spk::kStageKids;
    while (p->stage_kids > 0 && node_lds_bytes(p, 64, 8) > 64 * 1024) --p->stage_kids;
    if (node_lds_bytes(p, 64, 8) > 64 * 1024 ||
        spk::sweep_int_bytes(p->N) + spk::sweep_elems(nx, nu) * 8 > 64 * 1024)
        return fail(SPOCK_E_INVALID, "nx + nu or the branching is too large for one wavefront's LDS");
    return SPOCK_OK;
}

// Root-to-leaf path of every leaf, and the first stage of that path whose node
// has the leaf as its leftmost leaf: the forward task of a leaf computes its
// whole path and stores the nodes from that stage down.
static void leaf_paths(const spock_problem* p, std::vector<int>& path, std::vector<int>& top) {
    const int n = p->n, N = p->N;
    std::vector<int> leftmost(n);
    for (int v = n - 1; v >= 0; --v) leftmost[v] = p->n_ch[v] ? leftmost[p->first_child[v]] : v;
    path.assign((size_t)p->n_leaf * (N + 1), 0);
    top.assign(p->n_leaf, 0);
    for (int l = 0; l < p->n_leaf; ++l) {
        int v = p->n_nl + l;
        for (int lev = N; lev >= 0; --lev) {
            path[(size_t)l * (N + 1) + lev] = v;
            v = p->parent[v];
        }
        int L = 0;
        while (leftmost[path[(size_t)l * (N + 1) + L]] != p->n_nl + l) ++L;
        top[l] = L;
    }
}

// ---------------------------------------------------------------------------
// scaling (Sec. 5.4) and exact ||L|| (Sec. 4.4)
// ---------------------------------------------------------------------------

// FNV-1a hash of n doubles' bytes
static uint64_t mat_hash(const std::vector<double>& a) {
    uint64_t h = 1469598103934665603ull;
    const unsigned char* b = reinterpret_cast<const unsigned char*>(a.data());
    for (size_t i = 0; i < a.size() * sizeof(double); ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

// Distinct matrices among items 0..count-1 (mat(i) returns item i's matrix):
// id[i] indexes rep, which holds one item per distinct matrix.
template <typename Mat>
static void distinct_mats(int count, Mat mat, std::vector<int>& id, std::vector<int>& rep) {
    std::unordered_map<uint64_t, std::vector<int>> seen;  // hash -> distinct ids
    id.assign(count, -1);
    rep.clear();
    for (int i = 0; i < count; ++i) {
        const std::vector<double> a = mat(i);
        std::vector<int>& bucket = seen[mat_hash(a)];
        for (int u : bucket)
            if (mat(rep[u]) == a) {
                id[i] = u;
                break;
            }
        if (id[i] < 0) {
            id[i] = (int)rep.size();
            bucket.push_back(id[i]);
            rep.push_back(i);
        }
    }
}

// Dense costs: the symmetric square root H = V diag(w^1/2) V^T of every
// distinct matrix, and V diag(w^-1/2) V^T b for linear terms b (Prop. 1 with a
// dense Q: the translation takes Q^-1/2 q).  Fails unless positive definite.
struct DenseRoots {
    int dim = 0;
    std::vector<int> id, rep;
    std::vector<std::vector<double>> w, V, H;
    template <typename Mat>
    bool build(int count, int dim_, Mat mat) {
        dim = dim_;
        distinct_mats(count, mat, id, rep);
        const int u = (int)rep.size();
        w.assign(u, {});
        V.assign(u, {});
        H.assign(u, {});
        std::vector<int> ok(u, 1);
        parallel_for(u, [&](int k) {
            const std::vector<double> a = mat(rep[k]);
            sym_eig(dim, a.data(), w[k], V[k]);
            double top = 0;
            for (double e : w[k]) top = std::max(top, std::fabs(e));
            for (double e : w[k])
                if (!(e > 1e-14 * top)) ok[k] = 0;
            H[k] = eig_fn(dim, w[k], V[k], [](double e) { return std::sqrt(std::max(e, 0.0)); });
        });
        for (int k = 0; k < u; ++k)
            if (!ok[k]) return false;
        return true;
    }
    // Q^-1/2 b of item i
    void inv_root_apply(int i, const double* b, double* out) const {
        const int k = id[i];
        std::vector<double> t(dim, 0.0);
        for (int e = 0; e < dim; ++e) {
            double s = 0;
            for (int r = 0; r < dim; ++r) s += V[k][(size_t)r * dim + e] * b[r];
            t[e] = s / std::sqrt(w[k][e]);
        }
        for (int r = 0; r < dim; ++r) {
            double s = 0;
            for (int e = 0; e < dim; ++e) s += V[k][(size_t)r * dim + e] * t[e];
            out[r] = s;
        }
    }
};

// Largest eigenvalue of diag(g2) + D (sum of the listed matrices) D, D = diag(dsc)
static double dense_block_norm2(int dim, const std::vector<const std::vector<double>*>& mats,
                                const std::vector<double>& g2, const std::vector<double>& dsc) {
    std::vector<double> M((size_t)dim * dim, 0.0);
    for (const std::vector<double>* a : mats)
        for (size_t e = 0; e < M.size(); ++e) M[e] += (*a)[e];
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c) M[(size_t)r * dim + c] *= dsc[r] * dsc[c];
    for (int r = 0; r < dim; ++r) M[(size_t)r * dim + r] += g2[r];
    std::vector<double> w, V;
    sym_eig(dim, M.data(), w, V);
    double top = 0;
    for (double e : w) top = std::max(top, e);
    return top;
}

static int32_t scale_data(const spock_problem_desc* d, int precondition, spock_problem* p) {
    const int nx = p->nx, nu = p->nu;
    p->Sx.assign(nx, 1.0);
    p->Su.assign(nu, 1.0);
    p->SxN.assign(nx, 1.0);
    if (precondition) {
        // Sec. 5.4: the largest square root over the edges (leaves for S_N)
        const double chat = std::sqrt((double)p->max_ch);
        for (int k = 0; k < nx; ++k) {
            double mq = 0, mqN = 0;
            for (int j = 1; j < p->n; ++j) {
                mq = std::max(mq, Qd(d, j, k));
                if (j >= p->n_nl) mqN = std::max(mqN, QNd(d, j, k));
            }
            p->Sx[k] = chat * std::max(1.0, std::sqrt(mq));
            p->SxN[k] = std::max(1.0, std::sqrt(mqN));
        }
        for (int k = 0; k < nu; ++k) {
            double mr = 0;
            for (int j = 1; j < p->n; ++j) mr = std::max(mr, Rd(d, j, k));
            p->Su[k] = chat * std::max(1.0, std::sqrt(mr));
        }
    }
    // shared square roots (those of edge 1 / the first leaf when they differ
    // per edge; the kernels then read the per-edge ones)
    const int j1 = 1, l1 = p->n_nl;
    p->qh.resize(nx);
    p->rh.resize(nu);
    p->qnh.resize(nx);
    for (int k = 0; k < nx; ++k) {
        p->qh[k] = std::sqrt(Qd(d, j1, k)) / p->Sx[k];
        p->qnh[k] = std::sqrt(QNd(d, l1, k)) / p->SxN[k];
    }
    for (int k = 0; k < nu; ++k) p->rh[k] = std::sqrt(Rd(d, j1, k)) / p->Su[k];
    // dense costs: qh, rh, qnh hold S^-1 and the square roots are per edge / leaf
    DenseRoots dq, dr, dqN;
    const int n = p->n, nl = p->n_nl;
    p->Hq_e.clear();
    p->Hr_e.clear();
    p->HqN_l.clear();
    if (p->dense_edge) {
        for (int k = 0; k < nx; ++k) p->qh[k] = 1.0 / p->Sx[k];
        for (int k = 0; k < nu; ++k) p->rh[k] = 1.0 / p->Su[k];
        // item i is edge i + 1
        if (!dq.build(n - 1, nx, [&](int i) { return cost_mat(d->Q_dense, i + 1, nx, Qd, d); }) ||
            !dr.build(n - 1, nu, [&](int i) { return cost_mat(d->R_dense, i + 1, nu, Rd, d); }))
            return fail(SPOCK_E_INVALID, "dense Q and R must be positive definite");
        p->Hq_e.assign((size_t)n * nx * nx, 0.0);
        p->Hr_e.assign((size_t)n * nu * nu, 0.0);
        for (int j = 1; j < n; ++j) {
            const std::vector<double>& hq = dq.H[dq.id[j - 1]];
            const std::vector<double>& hr = dr.H[dr.id[j - 1]];
            std::copy(hq.begin(), hq.end(), p->Hq_e.begin() + (size_t)j * nx * nx);
            std::copy(hr.begin(), hr.end(), p->Hr_e.begin() + (size_t)j * nu * nu);
        }
    }
    if (p->dense_leaf) {
        for (int k = 0; k < nx; ++k) p->qnh[k] = 1.0 / p->SxN[k];
        if (!dqN.build(p->n_leaf, nx, [&](int l) { return cost_mat(d->QN_dense, nl + l, nx, QNd, d); }))
            return fail(SPOCK_E_INVALID, "dense QN must be positive definite");
        p->HqN_l.assign((size_t)p->n_leaf * nx * nx, 0.0);
        for (int l = 0; l < p->n_leaf; ++l) {
            const std::vector<double>& h = dqN.H[dqN.id[l]];
            std::copy(h.begin(), h.end(), p->HqN_l.begin() + (size_t)l * nx * nx);
        }
    }
    p->qh_e.clear();
    p->rh_e.clear();
    p->qnh_l.clear();
    if (p->edge_cost) {
        p->qh_e.assign((size_t)p->n * nx, 0.0);
        p->rh_e.assign((size_t)p->n * nu, 0.0);
        for (int j = 1; j < p->n; ++j) {
            for (int k = 0; k < nx; ++k) p->qh_e[(size_t)j * nx + k] = std::sqrt(Qd(d, j, k)) / p->Sx[k];
            for (int k = 0; k < nu; ++k) p->rh_e[(size_t)j * nu + k] = std::sqrt(Rd(d, j, k)) / p->Su[k];
        }
    }
    if (p->leaf_cost) {
        p->qnh_l.assign((size_t)p->n_leaf * nx, 0.0);
        for (int l = 0; l < p->n_leaf; ++l)
            for (int k = 0; k < nx; ++k)
                p->qnh_l[(size_t)l * nx + k] = std::sqrt(QNd(d, p->n_nl + l, k)) / p->SxN[k];
    }
    // constraint rows Gamma S^-1 / a with a = max(1, ||Gamma S^-1||_2): the box
    // and ball rows have orthogonal columns (the 2-norm is the largest column
    // norm); general rows take the largest eigenvalue of their Gram matrix
    double a = 1.0, aN = 1.0;
    auto two_norm = [&](const std::vector<double>& G, int rows, int cols) {
        const int k = std::min(rows, cols);
        std::vector<double> M((size_t)k * k, 0.0);
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                double v = 0;
                if (rows <= cols)
                    for (int c = 0; c < cols; ++c) v += G[(size_t)i * cols + c] * G[(size_t)j * cols + c];
                else
                    for (int r = 0; r < rows; ++r) v += G[(size_t)r * cols + i] * G[(size_t)r * cols + j];
                M[(size_t)i * k + j] = v;
            }
        std::vector<double> w, V;
        sym_eig(k, M.data(), w, V);
        double top = 0;
        for (double e : w) top = std::max(top, e);
        return std::sqrt(top);
    };
    std::vector<double> Gs, GNs;  // Gamma S^-1, Gamma_N S_N^-1
    if (p->gen) {
        const int nc = p->nbox, m = p->m;
        Gs.resize((size_t)nc * m);
        for (int r = 0; r < nc; ++r)
            for (int c = 0; c < m; ++c)
                Gs[(size_t)r * m + c] = d->Gamma[(size_t)r * m + c] / (c < nx ? p->Sx[c] : p->Su[c - nx]);
        if (precondition) a = std::max(1.0, two_norm(Gs, nc, m));
    }
    if (p->genN) {
        const int nc = p->nboxN;
        GNs.resize((size_t)nc * nx);
        for (int r = 0; r < nc; ++r)
            for (int c = 0; c < nx; ++c) GNs[(size_t)r * nx + c] = d->GammaN[(size_t)r * nx + c] / p->SxN[c];
        if (precondition) aN = std::max(1.0, two_norm(GNs, nc, nx));
    }
    if (precondition && !p->gen) {
        double mx = 0;
        for (int k = 0; k < nx; ++k) mx = std::max(mx, (1.0 + p->has_ball) / (p->Sx[k] * p->Sx[k]));
        for (int k = 0; k < nu; ++k) mx = std::max(mx, 1.0 / (p->Su[k] * p->Su[k]));
        a = std::max(1.0, std::sqrt(mx));
    }
    if (precondition && !p->genN) {
        double mxN = 0;
        for (int k = 0; k < nx; ++k) mxN = std::max(mxN, (1.0 + p->has_ballN) / (p->SxN[k] * p->SxN[k]));
        aN = std::max(1.0, std::sqrt(mxN));
    }
    p->Gt.clear();
    p->GtT.clear();
    p->GNt.clear();
    p->GNtT.clear();
    if (p->gen) {
        const int nc = p->nbox, m = p->m;
        p->Gt.resize((size_t)nc * m);
        p->GtT.resize((size_t)m * nc);
        for (int r = 0; r < nc; ++r)
            for (int c = 0; c < m; ++c) p->Gt[(size_t)r * m + c] = p->GtT[(size_t)c * nc + r] = Gs[(size_t)r * m + c] / a;
    }
    if (p->genN) {
        const int nc = p->nboxN;
        p->GNt.resize((size_t)nc * nx);
        p->GNtT.resize((size_t)nx * nc);
        for (int r = 0; r < nc; ++r)
            for (int c = 0; c < nx; ++c)
                p->GNt[(size_t)r * nx + c] = p->GNtT[(size_t)c * nc + r] = GNs[(size_t)r * nx + c] / aN;
    }
    p->con_scale = a;
    p->con_scaleN = aN;
    p->gx.resize(nx);
    p->gb.resize(nx);
    p->gu.resize(nu);
    p->gxN.resize(nx);
    p->gbN.resize(nx);
    for (int k = 0; k < nx; ++k) {
        p->gx[k] = 1.0 / (a * p->Sx[k]);
        p->gb[k] = p->has_ball ? 1.0 / (a * p->Sx[k]) : 0.0;
        p->gxN[k] = 1.0 / (aN * p->SxN[k]);
        p->gbN[k] = p->has_ballN ? 1.0 / (aN * p->SxN[k]) : 0.0;
    }
    for (int k = 0; k < nu; ++k) p->gu[k] = 1.0 / (a * p->Su[k]);
    // box bounds of the nbox (nboxN) box rows; at least m (nx) entries, as
    // the node kernels stage that many (zeros past the rows)
    p->lo.assign(std::max(p->m, p->nbox), 0.0);
    p->hi.assign(std::max(p->m, p->nbox), 0.0);
    if (p->gen) {
        for (int r = 0; r < p->nbox; ++r) {
            p->lo[r] = d->con_lo[r] / a;
            p->hi[r] = d->con_hi[r] / a;
        }
    } else {
        for (int k = 0; k < nx; ++k) {
            p->lo[k] = d->x_lo[k] / a;
            p->hi[k] = d->x_hi[k] / a;
        }
        for (int k = 0; k < nu; ++k) {
            p->lo[nx + k] = d->u_lo[k] / a;
            p->hi[nx + k] = d->u_hi[k] / a;
        }
    }
    p->loN.assign(std::max(nx, p->nboxN), 0.0);
    p->hiN.assign(std::max(nx, p->nboxN), 0.0);
    for (int r = 0; r < p->nboxN; ++r) {
        p->loN[r] = (p->genN ? d->conN_lo[r] : d->xN_lo[r]) / aN;
        p->hiN[r] = (p->genN ? d->conN_hi[r] : d->xN_hi[r]) / aN;
    }
    p->ball_r = p->has_ball ? d->x_ball / a : 0.0;
    p->ballN_r = p->has_ballN ? d->xN_ball / aN : 0.0;
    p->prob.assign(d->cond_prob, d->cond_prob + p->n);
    if (p->grisk) p->gamma.assign(p->n_nl, 0.0);  // not read
    else p->gamma.assign(d->gamma, d->gamma + p->n_nl);
    // the root's box and ball for the x0 check (none with general rows)
    if (p->gen) {
        p->x_lo.assign(nx, -INFINITY);
        p->x_hi.assign(nx, INFINITY);
        p->x_ball = 0;
    } else {
        p->x_lo.assign(d->x_lo, d->x_lo + nx);
        p->x_hi.assign(d->x_hi, d->x_hi + nx);
        p->x_ball = d->x_ball;
    }

    // Prop. 1 with a linear term: a = (-Q^-1/2 q / 2, c + 1/2, c - 1/2),
    // c = -|q|^2_{Q^-1} / 8; the change of variables of Sec. 5.4 leaves a
    // unchanged (Q~^-1/2 q~ = Q^-1/2 q for diagonal Q and S)
    p->sa.clear();
    p->saN.clear();
    p->ck.assign(p->coupled ? (size_t)p->n * nu : 0, 0.0);
    if (p->has_lin) {
        const int m = p->m;
        p->sa.assign((size_t)(p->n - 1) * (m + 2), 0.0);
        for (int j = 1; j < p->n; ++j) {
            double* a = p->sa.data() + (size_t)(j - 1) * (m + 2);
            double c = 0;
            std::vector<double> wq(nx, 0.0), wr(nu, 0.0);
            if (d->q && p->dense_edge) dq.inv_root_apply(j - 1, d->q + (size_t)j * nx, wq.data());
            else if (d->q)
                for (int k = 0; k < nx; ++k) wq[k] = d->q[(size_t)j * nx + k] / std::sqrt(Qd(d, j, k));
            if (d->r && p->dense_edge) dr.inv_root_apply(j - 1, d->r + (size_t)j * nu, wr.data());
            else if (d->r)
                for (int k = 0; k < nu; ++k) {
                    // an input without quadratic cost: its linear term lies in
                    // ker R and goes to the tau rows (Prop. 1's z'), not into a
                    const double rk = d->r[(size_t)j * nu + k], Rk = Rd(d, j, k);
                    if (Rk > 0) wr[k] = rk / std::sqrt(Rk);
                    else if (p->coupled) p->ck[(size_t)j * nu + k] = rk / p->Su[k];
                }
            for (int k = 0; k < nx; ++k) {
                a[k] = -0.5 * wq[k];
                c += wq[k] * wq[k];
            }
            for (int k = 0; k < nu; ++k) {
                a[nx + k] = -0.5 * wr[k];
                c += wr[k] * wr[k];
            }
            a[m] = -0.125 * c + 0.5;
            a[m + 1] = -0.125 * c - 0.5;
        }
        p->saN.assign((size_t)p->n_leaf * (nx + 2), 0.0);
        for (int l = 0; l < p->n_leaf; ++l) {
            const int j = p->n_nl + l;
            double* a = p->saN.data() + (size_t)l * (nx + 2);
            double c = 0;
            std::vector<double> wq(nx, 0.0);
            if (d->qN && p->dense_leaf) dqN.inv_root_apply(l, d->qN + (size_t)j * nx, wq.data());
            else if (d->qN)
                for (int k = 0; k < nx; ++k) wq[k] = d->qN[(size_t)j * nx + k] / std::sqrt(QNd(d, j, k));
            for (int k = 0; k < nx; ++k) {
                a[k] = -0.5 * wq[k];
                c += wq[k] * wq[k];
            }
            a[nx] = -0.125 * c + 0.5;
            a[nx + 1] = -0.125 * c - 0.5;
        }
    }

    // ||L||: largest block norm of L composed with a permutation
    double L2 = 0.5;  // tau^j and leaf s^j rows (1/2, 1/2)
    if (p->gen || p->genN) {
        // general constraint rows couple x and u: the (x^i, u^i) block is
        // lambda_max(Gt^T Gt + blockdiag(C_x, C_u)), C the sum over the child
        // edges of the cost rows' Gram matrices (S^-1 Q^j S^-1 dense, or the
        // squared diagonals); the leaf block lambda_max(GNt^T GNt + C_N).
        // Once per distinct C.
        auto gram = [&](const std::vector<double>& G, int rows, int cols) {
            std::vector<double> M((size_t)cols * cols, 0.0);
            for (int r = 0; r < rows; ++r)
                for (int i = 0; i < cols; ++i) {
                    const double gi = G[(size_t)r * cols + i];
                    if (gi == 0.0) continue;
                    for (int j = 0; j < cols; ++j) M[(size_t)i * cols + j] += gi * G[(size_t)r * cols + j];
                }
            return M;
        };
        auto top_of = [&](int dim, const std::vector<double>& base, std::vector<std::vector<double>>& Cs) {
            std::vector<double> top(Cs.size(), 0.0);
            parallel_for((int)Cs.size(), [&](int t) {
                std::vector<double> M = base;
                for (size_t e = 0; e < M.size(); ++e) M[e] += Cs[t][e];
                std::vector<double> w, V;
                sym_eig(dim, M.data(), w, V);
                for (double x : w) top[t] = std::max(top[t], x);
            });
            double best = 0;
            for (double x : top) best = std::max(best, x);
            return best;
        };
        // the cost rows' Gram matrix of edge (leaf) j into C at offset off:
        // S^-1 Q^j S^-1 with dense costs (sc = S^-1), else the squared
        // diagonal (per-row square roots, or the shared ones)
        auto add_cost = [&](std::vector<double>& C, int mm, int off, int dim, bool dense_mode, const double* dense,
                            int j, double (*diag)(const spock_problem_desc*, int, int), const std::vector<double>& sc,
                            const std::vector<double>* per, int per_row) {
            if (dense_mode) {
                const std::vector<double> Qm = cost_mat(dense, j, dim, diag, d);
                for (int a2 = 0; a2 < dim; ++a2)
                    for (int b2 = 0; b2 < dim; ++b2)
                        C[(size_t)(off + a2) * mm + off + b2] += Qm[(size_t)a2 * dim + b2] * sc[a2] * sc[b2];
            } else {
                for (int a2 = 0; a2 < dim; ++a2) {
                    const double h = per ? (*per)[(size_t)per_row * dim + a2] : sc[a2];
                    C[(size_t)(off + a2) * mm + off + a2] += h * h;
                }
            }
        };
        if (p->gen) {
            const int m = p->m;
            const std::vector<double> base = gram(p->Gt, p->nbox, m);
            std::map<std::vector<double>, int> seen;
            std::vector<std::vector<double>> Cs;
            for (int i = 0; i < nl; ++i) {
                std::vector<double> C((size_t)m * m, 0.0);
                for (int c = 0; c < p->n_ch[i]; ++c) {
                    const int j = p->first_child[i] + c;
                    add_cost(C, m, 0, nx, p->dense_edge, d->Q_dense, j, Qd, p->qh, p->edge_cost ? &p->qh_e : nullptr, j);
                    add_cost(C, m, nx, nu, p->dense_edge, d->R_dense, j, Rd, p->rh, p->edge_cost ? &p->rh_e : nullptr,
                             j);
                }
                if (seen.emplace(C, (int)Cs.size()).second) Cs.push_back(C);
            }
            L2 = std::max(L2, top_of(m, base, Cs));
        }
        if (p->genN) {
            const std::vector<double> base = gram(p->GNt, p->nboxN, nx);
            std::map<std::vector<double>, int> seen;
            std::vector<std::vector<double>> Cs;
            for (int l = 0; l < p->n_leaf; ++l) {
                std::vector<double> C((size_t)nx * nx, 0.0);
                add_cost(C, nx, 0, nx, p->dense_leaf, d->QN_dense, nl + l, QNd, p->qnh,
                         p->leaf_cost ? &p->qnh_l : nullptr, l);
                if (seen.emplace(C, (int)Cs.size()).second) Cs.push_back(C);
            }
            L2 = std::max(L2, top_of(nx, base, Cs));
        }
    }
    if (p->dense_edge && !p->gen) {
        // (x^i, u^i) block with dense cost rows: the largest eigenvalue of
        // diag(gx^2 + gb^2) + S^-1 (sum over the child edges of Q^j) S^-1,
        // once per distinct list of children's matrices (likewise for u)
        std::vector<double> gx2(nx), gu2(nu), qd = p->qh, rd = p->rh;
        for (int k = 0; k < nx; ++k) gx2[k] = p->gx[k] * p->gx[k] + p->gb[k] * p->gb[k];
        for (int k = 0; k < nu; ++k) gu2[k] = p->gu[k] * p->gu[k];
        std::vector<std::vector<double>> Qm(dq.rep.size()), Rm(dr.rep.size());
        for (size_t u = 0; u < dq.rep.size(); ++u) Qm[u] = cost_mat(d->Q_dense, dq.rep[u] + 1, nx, Qd, d);
        for (size_t u = 0; u < dr.rep.size(); ++u) Rm[u] = cost_mat(d->R_dense, dr.rep[u] + 1, nu, Rd, d);
        std::map<std::vector<int>, int> keys;
        std::vector<std::vector<int>> klist;
        for (int i = 0; i < nl; ++i) {
            std::vector<int> key;
            for (int c = 0; c < p->n_ch[i]; ++c) key.push_back(dq.id[p->first_child[i] + c - 1]);
            key.push_back(-1);
            for (int c = 0; c < p->n_ch[i]; ++c) key.push_back(dr.id[p->first_child[i] + c - 1]);
            if (keys.emplace(key, (int)klist.size()).second) klist.push_back(key);
        }
        std::vector<double> top(klist.size(), 0.0);
        parallel_for((int)klist.size(), [&](int t) {
            std::vector<const std::vector<double>*> mq, mr;
            size_t e = 0;
            for (; klist[t][e] >= 0; ++e) mq.push_back(&Qm[klist[t][e]]);
            for (++e; e < klist[t].size(); ++e) mr.push_back(&Rm[klist[t][e]]);
            top[t] = std::max(dense_block_norm2(nx, mq, gx2, qd), dense_block_norm2(nu, mr, gu2, rd));
        });
        for (double t : top) L2 = std::max(L2, t);
    }
    if (p->dense_leaf && !p->genN) {
        std::vector<double> g2(nx), qd = p->qnh;
        for (int k = 0; k < nx; ++k) g2[k] = p->gxN[k] * p->gxN[k] + p->gbN[k] * p->gbN[k];
        std::vector<double> top(dqN.rep.size(), 0.0);
        parallel_for((int)dqN.rep.size(), [&](int u) {
            const std::vector<double> QN = cost_mat(d->QN_dense, nl + dqN.rep[u], nx, QNd, d);
            top[u] = dense_block_norm2(nx, {&QN}, g2, qd);
        });
        for (double t : top) L2 = std::max(L2, t);
    }
    for (int i = 0; i < p->n_nl; ++i) {
        // (x^i, u^i) block: constraint rows and every child edge's cost rows
        for (int r = 0; r < ((p->dense_edge || p->gen) ? 0 : nx); ++r) {
            double sq = 0;
            for (int c = 0; c < p->n_ch[i]; ++c) {
                const double h = p->edge_cost ? p->qh_e[(size_t)(p->first_child[i] + c) * nx + r] : p->qh[r];
                sq += h * h;
            }
            L2 = std::max(L2, p->gx[r] * p->gx[r] + p->gb[r] * p->gb[r] + sq);
        }
        for (int r = 0; r < ((p->dense_edge || p->gen) ? 0 : nu); ++r) {
            double sq = 0;
            for (int c = 0; c < p->n_ch[i]; ++c) {
                const double h = p->edge_cost ? p->rh_e[(size_t)(p->first_child[i] + c) * nu + r] : p->rh[r];
                sq += h * h;
            }
            L2 = std::max(L2, p->gu[r] * p->gu[r] + sq);
        }
        double b2 = 0.0;  // ||b^i||^2: (p, 0, 1) for AV@R, else the given b^i
        if (p->grisk) {
            const double* b = p->rdata.data() + p->roff[i] + (size_t)p->rny[i] * (p->n_ch[i] + p->rnnu[i]);
            for (int r = 0; r < p->rny[i]; ++r) b2 += b[r] * b[r];
        } else {
            b2 = 1.0;
            for (int c = 0; c < p->n_ch[i]; ++c) b2 += p->prob[p->first_child[i] + c] * p->prob[p->first_child[i] + c];
        }
        const double beta = std::sqrt(b2);
        const double sig = 0.5 * (beta + std::sqrt(b2 + 4.0));  // [[I, 0], [-b^T, 1]]
        L2 = std::max(L2, sig * sig);
    }
    for (int l = 0; l < ((p->dense_leaf || p->genN) ? 0 : p->leaf_cost ? p->n_leaf : 1); ++l)
        for (int r = 0; r < nx; ++r) {
            const double h = p->leaf_cost ? p->qnh_l[(size_t)l * nx + r] : p->qnh[r];
            L2 = std::max(L2, p->gxN[r] * p->gxN[r] + p->gbN[r] * p->gbN[r] + h * h);
        }
    if (p->coupled) {
        // Prop. 1 with R singular: each child edge's two tau rows carry
        // (tau^j - c_j^T u^i) / 2, which couples (x^i, u^i) with the
        // children's tau.  The block over (x^i, u^i, tau^ch(i)) is
        // [[Gc + C + sum_j c_j c_j^T / 2, -c_j / 2], [-c_j^T / 2, I / 2]]:
        // Gc the constraint rows' Gram matrix, C the cost rows' (dense Q or
        // diagonal).  Once per distinct block.
        const int m = p->m;
        std::vector<double> base((size_t)m * m, 0.0);
        if (p->gen) {
            for (int r = 0; r < p->nbox; ++r)
                for (int a2 = 0; a2 < m; ++a2) {
                    const double ga = p->Gt[(size_t)r * m + a2];
                    if (ga != 0.0)
                        for (int b2 = 0; b2 < m; ++b2) base[(size_t)a2 * m + b2] += ga * p->Gt[(size_t)r * m + b2];
                }
        } else {
            for (int k = 0; k < nx; ++k) base[(size_t)k * m + k] = p->gx[k] * p->gx[k] + p->gb[k] * p->gb[k];
            for (int k = 0; k < nu; ++k) base[(size_t)(nx + k) * m + nx + k] = p->gu[k] * p->gu[k];
        }
        std::map<std::vector<double>, int> seen;
        std::vector<std::pair<int, std::vector<double>>> blocks;
        for (int i = 0; i < nl; ++i) {
            const int k = p->n_ch[i], dim = m + k;
            std::vector<double> M((size_t)dim * dim, 0.0);
            for (int a2 = 0; a2 < m; ++a2)
                for (int b2 = 0; b2 < m; ++b2) M[(size_t)a2 * dim + b2] = base[(size_t)a2 * m + b2];
            for (int q = 0; q < k; ++q) {
                const int j = p->first_child[i] + q;
                if (d->Q_dense) {
                    const std::vector<double> Qm = cost_mat(d->Q_dense, j, nx, Qd, d);
                    for (int a2 = 0; a2 < nx; ++a2)
                        for (int b2 = 0; b2 < nx; ++b2)
                            M[(size_t)a2 * dim + b2] += Qm[(size_t)a2 * nx + b2] * p->qh[a2] * p->qh[b2];
                } else {
                    for (int a2 = 0; a2 < nx; ++a2) {
                        const double h = p->edge_cost ? p->qh_e[(size_t)j * nx + a2] : p->qh[a2];
                        M[(size_t)a2 * dim + a2] += h * h;
                    }
                }
                const double* c = p->ck.data() + (size_t)j * nu;
                for (int a2 = 0; a2 < nu; ++a2) {
                    const double h = p->edge_cost ? p->rh_e[(size_t)j * nu + a2] : p->rh[a2];
                    M[(size_t)(nx + a2) * dim + nx + a2] += h * h;
                    for (int b2 = 0; b2 < nu; ++b2) M[(size_t)(nx + a2) * dim + nx + b2] += 0.5 * c[a2] * c[b2];
                    M[(size_t)(nx + a2) * dim + m + q] = M[(size_t)(m + q) * dim + nx + a2] = -0.5 * c[a2];
                }
                M[(size_t)(m + q) * dim + m + q] = 0.5;
            }
            if (seen.emplace(M, (int)blocks.size()).second) blocks.emplace_back(dim, M);
        }
        std::vector<double> top(blocks.size(), 0.0);
        parallel_for((int)blocks.size(), [&](int t) {
            std::vector<double> w, V;
            sym_eig(blocks[t].first, blocks[t].second.data(), w, V);
            for (double x : w) top[t] = std::max(top[t], x);
        });
        for (double t : top) L2 = std::max(L2, t);
    }
    p->Lnorm = std::sqrt(L2);
    return SPOCK_OK;
}

// ---------------------------------------------------------------------------
// Alg. 1 (offline S1) in float64; fills [Abar|B] per edge and [K | R~^-1] per
// non-leaf node, and P c for affine dynamics.
// ---------------------------------------------------------------------------

static int32_t offline_factor(const spock_problem_desc* d, spock_problem* p, std::vector<double>& M,
                              std::vector<double>& KR, std::vector<double>& cs, std::vector<double>& Pc) {
    const int n = p->n, nx = p->nx, nu = p->nu, m = p->m;
    M.assign((size_t)n * p->M_stride, 0.0);
    KR.assign((size_t)p->n_nl * p->KR_stride, 0.0);
    if (p->affine) {
        cs.assign((size_t)n * nx, 0.0);
        Pc.assign((size_t)n * nx, 0.0);
    }
    // scaled dynamics written straight into M: [A~ | B~] (Abar replaces A~ below)
    auto S_of = [&](int j) -> const std::vector<double>& { return j < p->n_nl ? p->Sx : p->SxN; };
    for (int j = 1; j < n; ++j) {
        const std::vector<double>& Sj = S_of(j);
        double* Mj = M.data() + (size_t)j * p->M_stride;
        const double* A = d->A + (size_t)j * nx * nx;
        const double* B = d->B + (size_t)j * nx * nu;
        for (int r = 0; r < nx; ++r) {
            for (int c = 0; c < nx; ++c) Mj[(size_t)r * m + c] = Sj[r] * A[(size_t)r * nx + c] / p->Sx[c];
            for (int c = 0; c < nu; ++c) Mj[(size_t)r * m + nx + c] = Sj[r] * B[(size_t)r * nu + c] / p->Su[c];
            if (p->affine) cs[(size_t)j * nx + r] = Sj[r] * d->c[(size_t)j * nx + r];
        }
    }
    std::vector<std::vector<double>> P(n);
    std::vector<int> stage_start(p->N + 2, 0);
    {
        std::vector<int> stage(n, 0);
        for (int j = 1; j < n; ++j) stage[j] = stage[p->parent[j]] + 1;
        for (int j = 0; j < n; ++j) stage_start[stage[j] + 1] = j + 1;
        for (int t = 1; t <= p->N + 1; ++t) stage_start[t] = std::max(stage_start[t], stage_start[t - 1]);
    }
    for (int j = p->n_nl; j < n; ++j) {
        P[j].assign((size_t)nx * nx, 0.0);
        for (int r = 0; r < nx; ++r) P[j][(size_t)r * nx + r] = 1.0;
        if (p->affine)
            for (int r = 0; r < nx; ++r) Pc[(size_t)j * nx + r] = cs[(size_t)j * nx + r];
    }
    std::atomic<int> bad(0);
    for (int t = p->N - 1; t >= 0; --t) {
        const int s0 = stage_start[t], s1 = stage_start[t + 1];
        parallel_for(s1 - s0, [&](int q) {
            const int i = s0 + q;
            std::vector<double> Rt((size_t)nu * nu, 0.0), rhs((size_t)nu * nx, 0.0);
            std::vector<double> A((size_t)nx * nx), B((size_t)nx * nu), PB((size_t)nx * nu), PA((size_t)nx * nx);
            for (int r = 0; r < nu; ++r) Rt[(size_t)r * nu + r] = 1.0;
            const int fc = p->first_child[i], k = p->n_ch[i];
            for (int c = 0; c < k; ++c) {
                const int j = fc + c;
                const double* Mj = M.data() + (size_t)j * p->M_stride;
                for (int r = 0; r < nx; ++r) {
                    std::memcpy(&A[(size_t)r * nx], Mj + (size_t)r * m, sizeof(double) * nx);
                    std::memcpy(&B[(size_t)r * nu], Mj + (size_t)r * m + nx, sizeof(double) * nu);
                }
                mm(nx, nu, nx, P[j].data(), B.data(), PB.data(), false);
                mtm_acc(nu, nu, nx, B.data(), PB.data(), Rt.data());  // R~ += B^T P B
                mm(nx, nx, nx, P[j].data(), A.data(), PA.data(), false);
                mtm_acc(nu, nx, nx, B.data(), PA.data(), rhs.data());  // sum B^T P A
            }
            std::vector<double> Lc = Rt, Rinv((size_t)nu * nu), K((size_t)nu * nx);
            if (!cholesky(nu, Lc.data())) {
                bad = 1;
                return;
            }
            chol_inverse(nu, Lc.data(), Rinv.data());
            mm(nu, nx, nu, Rinv.data(), rhs.data(), K.data(), false);
            for (auto& v : K) v = -v;  // K = -R~^-1 sum B^T P A
            std::vector<double> Pi((size_t)nx * nx, 0.0);
            for (int r = 0; r < nx; ++r) Pi[(size_t)r * nx + r] = 1.0;
            mtm_acc(nx, nx, nu, K.data(), K.data(), Pi.data());  // + K^T K
            std::vector<double> BK((size_t)nx * nx), PAb((size_t)nx * nx);
            for (int c = 0; c < k; ++c) {
                const int j = fc + c;
                double* Mj = M.data() + (size_t)j * p->M_stride;
                for (int r = 0; r < nx; ++r) std::memcpy(&B[(size_t)r * nu], Mj + (size_t)r * m + nx, sizeof(double) * nu);
                mm(nx, nx, nu, B.data(), K.data(), BK.data(), false);
                for (int r = 0; r < nx; ++r)
                    for (int cc = 0; cc < nx; ++cc) {
                        const double ab = Mj[(size_t)r * m + cc] + BK[(size_t)r * nx + cc];  // Abar = A + B K
                        Mj[(size_t)r * m + cc] = ab;
                        A[(size_t)r * nx + cc] = ab;
                    }
                mm(nx, nx, nx, P[j].data(), A.data(), PAb.data(), false);
                mtm_acc(nx, nx, nx, A.data(), PAb.data(), Pi.data());  // + Abar^T P Abar
            }
            double* KRi = KR.data() + (size_t)i * p->KR_stride;
            for (int r = 0; r < nu; ++r) {
                std::memcpy(KRi + (size_t)r * m, &K[(size_t)r * nx], sizeof(double) * nx);
                std::memcpy(KRi + (size_t)r * m + nx, &Rinv[(size_t)r * nu], sizeof(double) * nu);
            }
            if (p->affine)
                for (int r = 0; r < nx; ++r) {
                    double s = 0;
                    for (int cc = 0; cc < nx; ++cc) s += Pi[(size_t)r * nx + cc] * cs[(size_t)i * nx + cc];
                    Pc[(size_t)i * nx + r] = s;
                }
            P[i].swap(Pi);
            for (int c = 0; c < k; ++c) std::vector<double>().swap(P[fc + c]);
        });
        if (bad) return fail(SPOCK_E_INVALID, "R~ not positive definite in the offline factorisation");
    }
    return SPOCK_OK;
}

// ---------------------------------------------------------------------------
// upload
// ---------------------------------------------------------------------------

template <typename real>
static hipError_t put(const real* dst, const std::vector<double>& src, hipStream_t st) {
    std::vector<real> tmp(src.begin(), src.end());
    hipError_t e = hipMemcpyAsync((void*)dst, tmp.data(), tmp.size() * sizeof(real), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

// Pack A (K x O, A(k, o) given by `at`) in the lane order of the column-lane
// product out[o] = sum_k A(k, o) v[k] (layout of tile_elems in spock_dev.h).
template <typename real, typename F>
static void tile_pack(real* out, int K, int O, F at) {
    constexpr int V = spk::tile_vec<real>();
    auto block = [&](real* dst, int W, int col0) {
        const int G = 64 / W, rows = spk::tile_rows(K, G, V);
        for (int i = 0; i < rows; ++i)
            for (int l = 0; l < 64; ++l) {
                const int g = l / W, c = l - g * W, k = g + i * G;
                const double val = (g < G && k < K) ? at(k, col0 + c) : 0.0;
                dst[((size_t)(i / V) * 64 + l) * V + i % V] = (real)val;
            }
        return (size_t)rows * 64;
    };
    size_t off = 0;
    for (int b = 0; b < spk::tile_blocks(O); ++b) off += block(out + off, spk::tile_block_width(O, b), 64 * b);
}

// The five packed tile arrays of one precision from the float64 factors.
template <typename real>
static hipError_t put_tiles(const spock_problem* p, const ProbDev<real>& h, const std::vector<double>& M,
                            const std::vector<double>& KR, hipStream_t st) {
    const int n = p->n, nl = p->n_nl, nx = p->nx, nu = p->nu, m = p->m;
    // each array is followed by zero padding (see kTilePadRows)
    auto upload = [&](const real* dst, long long count, long long stride, auto fill) -> hipError_t {
        std::vector<real> buf((size_t)(count * stride + spk::tile_pad_elems<real>()), real(0));
        parallel_for((int)count, [&](int v) { fill(buf.data() + (size_t)v * stride, v); });
        hipError_t e = hipMemcpyAsync((void*)dst, buf.data(), buf.size() * sizeof(real), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(st);
    };
    auto Mj = [&](int j) { return M.data() + (size_t)j * p->M_stride; };
    auto KRi = [&](int i) { return KR.data() + (size_t)i * p->KR_stride; };
    hipError_t e;
    // prep: (K^i)^T ubar, A(k, o) = K[k][o], k < nu, o < nx
    e = upload(h.T1, nl, h.T1_stride, [&](real* t, int i) {
        const double* a = KRi(i);
        tile_pack<real>(t, nu, nx, [&](int k, int o) { return a[(size_t)k * m + o]; });
    });
    if (e != hipSuccess) return e;
    // bsweep: [Abar|B]^T h, A(k, o) = M[k][o], k < nx, o < m
    e = upload(h.T2M, n, h.T2M_stride, [&](real* t, int j) {
        if (j == 0) return;
        const double* a = Mj(j);
        tile_pack<real>(t, nx, m, [&](int k, int o) { return a[(size_t)k * m + o]; });
    });
    if (e != hipSuccess) return e;
    // bsweep: R~^-1 w with R~^-1 made exactly symmetric
    e = upload(h.T2R, nl, h.T2R_stride, [&](real* t, int i) {
        const double* a = KRi(i) + nx;
        tile_pack<real>(t, nu, nu,
                        [&](int k, int o) { return 0.5 * (a[(size_t)k * m + o] + a[(size_t)o * m + k]); });
    });
    if (e != hipSuccess) return e;
    // fsweep: [Abar|B] a, A(k, o) = M[o][k], k < m, o < nx
    e = upload(h.T3, n, h.T3_stride, [&](real* t, int j) {
        if (j == 0) return;
        const double* a = Mj(j);
        tile_pack<real>(t, m, nx, [&](int k, int o) { return a[(size_t)o * m + k]; });
    });
    if (e != hipSuccess) return e;
    // dual: K^i x, A(k, o) = K[o][k], k < nx, o < nu
    return upload(h.T4, nl, h.T4_stride, [&](real* t, int i) {
        const double* a = KRi(i);
        tile_pack<real>(t, nx, nu, [&](int k, int o) { return a[(size_t)o * m + k]; });
    });
}

template <typename real>
static int32_t upload_set(spock_problem* p, DevSet<real>& s, const std::vector<double>& M,
                          const std::vector<double>& KR, const std::vector<double>& cs,
                          const std::vector<double>& Pc) {
    ProbDev<real>& h = s.h;
    h.n = p->n;
    h.n_nl = p->n_nl;
    h.N = p->N;
    h.nx = p->nx;
    h.nu = p->nu;
    h.m = p->m;
    h.nc = p->nc;
    h.ncN = p->ncN;
    h.nbox = p->nbox;
    h.nboxN = p->nboxN;
    h.has_ball = p->has_ball;
    h.has_ballN = p->has_ballN;
    h.affine = p->affine;
    h.max_ch = p->max_ch;
    h.stage_kids = p->stage_kids;
    h.alpha = (real)p->alpha;
    h.ball_r = (real)p->ball_r;
    h.ballN_r = (real)p->ballN_r;
    h.first_child = p->d_tree;
    h.roff = p->d_roff;
    h.rny = p->d_rint;
    h.rnnu = p->d_rint ? p->d_rint + p->n_nl : nullptr;
    h.n_ch = p->d_tree + p->n;
    h.y_off = p->d_tree + 2 * p->n;
    h.z_x = p->z_x; h.z_u = p->z_u; h.z_y = p->z_y; h.z_tau = p->z_tau; h.z_s = p->z_s;
    h.e_y = p->e_y; h.e_s = p->e_s; h.e_c = p->e_c; h.e_soc = p->e_soc; h.e_cN = p->e_cN; h.e_socN = p->e_socN;
    h.nz = p->nz;
    h.neta = p->neta;
    h.cnt = p->d_cnt;
    h.path = p->d_path;
    h.top_owned = p->d_top;
    h.active = p->d_one;
    h.res = p->d_res;
    s.cfg = make_cfg<real>(p, s.cfg.node_wg > 0 ? s.cfg.node_wg : spk::kDefaultWG);
    hipStream_t st = p->stream;
    HIP_TRY(put_tiles<real>(p, h, M, KR, st));
    if (p->affine) {
        HIP_TRY(put<real>(h.c, cs, st));
        HIP_TRY(put<real>(h.Pc, Pc, st));
    }
    HIP_TRY(put<real>(h.qh, p->qh, st));
    HIP_TRY(put<real>(h.rh, p->rh, st));
    HIP_TRY(put<real>(h.qnh, p->qnh, st));
    HIP_TRY(put<real>(h.gx, p->gx, st));
    HIP_TRY(put<real>(h.gu, p->gu, st));
    HIP_TRY(put<real>(h.gb, p->gb, st));
    HIP_TRY(put<real>(h.gxN, p->gxN, st));
    HIP_TRY(put<real>(h.gbN, p->gbN, st));
    HIP_TRY(put<real>(h.lo, p->lo, st));
    HIP_TRY(put<real>(h.hi, p->hi, st));
    HIP_TRY(put<real>(h.loN, p->loN, st));
    HIP_TRY(put<real>(h.hiN, p->hiN, st));
    HIP_TRY(put<real>(h.prob, p->prob, st));
    HIP_TRY(put<real>(h.gamma, p->gamma, st));
    if (p->has_lin) {
        HIP_TRY(put<real>(h.sa, p->sa, st));
        if (p->coupled) HIP_TRY(put<real>(h.ck, p->ck, st));
        HIP_TRY(put<real>(h.saN, p->saN, st));
    }
    if (p->edge_cost) {
        HIP_TRY(put<real>(h.qh_e, p->qh_e, st));
        HIP_TRY(put<real>(h.rh_e, p->rh_e, st));
    }
    if (p->leaf_cost) HIP_TRY(put<real>(h.qnh_l, p->qnh_l, st));
    if (p->dense_edge) {
        HIP_TRY(put<real>(h.Hq_e, p->Hq_e, st));
        HIP_TRY(put<real>(h.Hr_e, p->Hr_e, st));
    }
    if (p->dense_leaf) HIP_TRY(put<real>(h.HqN_l, p->HqN_l, st));
    if (p->gen) {
        HIP_TRY(put<real>(h.Gt, p->Gt, st));
        HIP_TRY(put<real>(h.GtT, p->GtT, st));
    }
    if (p->genN) {
        HIP_TRY(put<real>(h.GNt, p->GNt, st));
        HIP_TRY(put<real>(h.GNtT, p->GNtT, st));
    }
    if (p->grisk) HIP_TRY(put<real>(h.rdata, p->rdata, st));
    for (int k = 0; k < 2; ++k) HIP_TRY(spk::launch_fill<real>(h.z[k], real(0), p->nzp + p->neta, st));
    HIP_TRY(hipMemcpyAsync(s.d, &h, sizeof(h), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SPOCK_OK;
}

// The SuperMann vectors start at zero (their z-to-eta pads stay zero), and the
// trial descriptor is the float64 one reading VT and writing TVT.
static int32_t upload_supermann(spock_problem* p) {
    SmWork& w = p->sm;
    const long long nv = p->nzp + p->neta;
    hipStream_t st = p->stream;
    for (double* v : {w.R[0], w.R[1], w.PSI, w.VT, w.TVT, w.RT}) HIP_TRY(spk::launch_fill<double>(v, 0.0, nv, st));
    for (int j = 0; j < p->set.aa_memory; ++j) {
        HIP_TRY(spk::launch_fill<double>(w.Y[j], 0.0, nv, st));
        HIP_TRY(spk::launch_fill<double>(w.S[j], 0.0, nv, st));
    }
    ProbDev<double> h = p->s64.h;
    h.z[0] = w.VT;
    h.eta[0] = w.VT + p->nzp;
    h.z[1] = w.TVT;
    h.eta[1] = w.TVT + p->nzp;
    HIP_TRY(hipMemcpyAsync(w.d_trial, &h, sizeof(h), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hipHostMalloc((void**)&w.h_dots, (spk::kMaxDots + 2 * spk::kResSlots) * sizeof(double), 0) != hipSuccess)
        return fail(SPOCK_E_HIP, "hipHostMalloc failed");
    return SPOCK_OK;
}

// ---------------------------------------------------------------------------
// stepping
// ---------------------------------------------------------------------------

template <typename real>
int32_t step(spock_problem* p, int check) {
    DevSet<real>& s = set_of<real>(p);
    HIP_TRY(spk::launch_step<real>(s.d, s.cfg, s.par, check, p->stream));
    s.par ^= 1;
    return SPOCK_OK;
}

// `steps` (even) steps, residual check on the last one; replayed as a graph.
template <typename real>
static int32_t chunk(spock_problem* p, int steps) {
    DevSet<real>& s = set_of<real>(p);
    if (p->set.use_graph && (steps & 1) == 0 && steps >= 2) {
        if (s.graph_steps != steps) {
            for (auto& g : s.graph)
                if (g) {
                    (void)hipGraphExecDestroy(g);
                    g = nullptr;
                }
            s.graph_steps = steps;
        }
        hipGraphExec_t& ge = s.graph[s.par];
        if (!ge) {
            std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
            hipGraph_t graph;
            HIP_TRY(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
            int par = s.par;
            for (int k = 0; k < steps; ++k) {
                hipError_t e = spk::launch_step<real>(s.d, s.cfg, par, k == steps - 1, p->stream);
                if (e != hipSuccess) {
                    (void)hipStreamEndCapture(p->stream, &graph);
                    return fail(SPOCK_E_HIP, std::string("capture: ") + hipGetErrorString(e));
                }
                par ^= 1;
            }
            HIP_TRY(hipStreamEndCapture(p->stream, &graph));
            HIP_TRY(hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0));
            HIP_TRY(hipGraphDestroy(graph));
        }
        HIP_TRY(hipGraphLaunch(ge, p->stream));
        return SPOCK_OK;  // parity unchanged after an even number of steps
    }
    for (int k = 0; k < steps; ++k) {
        int32_t r = step<real>(p, k == steps - 1);
        if (r) return r;
    }
    return SPOCK_OK;
}

int32_t read_res(spock_problem* p, double* xi1, double* xi2) {
    HIP_TRY(hipMemcpyAsync(p->h_res, p->d_res, 2 * spk::kResSlots * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    res_reduce(p->h_res, xi1, xi2);
    return SPOCK_OK;
}

// current iterate -> the other precision's copy `par`
int32_t move_iterate(spock_problem* p, int to) {
    if (p->cur == to) return SPOCK_OK;
    if (to == SPOCK_FP64) {
        HIP_TRY(spk::launch_convert<double, float>(p->s64.h.z[0], p->s32.h.z[p->s32.par], p->nz, p->stream));
        HIP_TRY(spk::launch_convert<double, float>(p->s64.h.eta[0], p->s32.h.eta[p->s32.par], p->neta, p->stream));
        p->s64.par = 0;
    } else {
        HIP_TRY(spk::launch_convert<float, double>(p->s32.h.z[0], p->s64.h.z[p->s64.par], p->nz, p->stream));
        HIP_TRY(spk::launch_convert<float, double>(p->s32.h.eta[0], p->s64.h.eta[p->s64.par], p->neta, p->stream));
        p->s32.par = 0;
    }
    p->cur = to;
    return SPOCK_OK;
}

int32_t zero_iterate(spock_problem* p) {
    HIP_TRY(spk::launch_fill<double>(p->s64.h.z[0], 0.0, p->nz, p->stream));
    HIP_TRY(spk::launch_fill<double>(p->s64.h.eta[0], 0.0, p->neta, p->stream));
    p->s64.par = 0;
    p->cur = SPOCK_FP64;
    return SPOCK_OK;
}

int32_t set_x0_device(spock_problem* p, const double* x0, bool check_feasible) {
    if (!x0) return fail(SPOCK_E_INVALID, "null x0");
    if (!finite_all(x0, p->nx)) return fail(SPOCK_E_INVALID, "non-finite x0");
    if (check_feasible) {
        double nrm = 0;
        for (int k = 0; k < p->nx; ++k) {
            if (x0[k] < p->x_lo[k] || x0[k] > p->x_hi[k])
                return fail(SPOCK_E_INFEASIBLE_X0, "x0 violates the state box at the root");
            nrm += x0[k] * x0[k];
        }
        if (p->has_ball && std::sqrt(nrm) > p->x_ball)
            return fail(SPOCK_E_INFEASIBLE_X0, "x0 violates the state ball at the root");
    }
    p->x0s.resize(p->nx);
    for (int k = 0; k < p->nx; ++k) p->x0s[k] = p->Sx[k] * x0[k];
    HIP_TRY(put<double>(p->s64.h.x0, p->x0s, p->stream));
    HIP_TRY(put<float>(p->s32.h.x0, p->x0s, p->stream));
    return SPOCK_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int node_lds_bytes(const spock_problem* p, int node_wg, int real_bytes) {
    const int waves = node_wg / 64;
    return (spk::consts_elems(p->nx, p->nu) +
            waves * spk::node_wave_elems(p->nx, p->nu, p->nc, p->ncN, std::min(p->max_ch, p->stage_kids))) *
           real_bytes;
}

int tile_class(int need) {
    for (int c : spk::kTileClasses)
        if (need <= c) return c;
    // no class holds it: the product runs from the packed tile in global
    // memory, in kernels built for that (a minimal register tile)
    return spk::kWideClass;
}

template <typename real>
spk::LaunchCfg make_cfg(const spock_problem* p, int node_wg) {
    constexpr int V = spk::tile_vec<real>();
    const int nx = p->nx, nu = p->nu, m = p->m;
    // the largest node workgroup (up to node_wg) whose LDS fits 64 KiB
    while (node_wg > 64 && node_lds_bytes(p, node_wg, (int)sizeof(real)) > 64 * 1024) node_wg /= 2;
    spk::LaunchCfg c{};
    c.leaf_tasks = p->d_tasks;
    c.n_leaf_tasks = p->n_leaf;
    c.node_tasks = p->d_ntasks;
    c.node_info = p->d_ninfo;
    c.n_node_tasks = p->n_ntasks;
    c.node_wg = node_wg;
    c.node_lds = node_lds_bytes(p, node_wg, (int)sizeof(real));
    c.wave_elems = spk::node_wave_elems(nx, nu, p->nc, p->ncN, std::min(p->max_ch, p->stage_kids));
    c.cls[0] = tile_class(spk::col_need(nu, nx, V));
    c.cls[1] = tile_class(spk::col_need(nx, m, V));
    c.cls[2] = tile_class(spk::col_need(m, nx, V));
    c.cls[3] = tile_class(spk::col_need(nx, nu, V));
    // node kernel build: 2 with the general formulation's products (general
    // rows, general risks, tau-row coupling; dense costs included), 1 with the
    // dense-cost products only, 0 with neither
    c.dense = (p->gen || p->genN || p->grisk || p->coupled) ? 2 : (p->dense_edge || p->dense_leaf) ? 1 : 0;
    // float sweeps stage their tiles and vectors in LDS
    const int staged = sizeof(real) == 4 ? spk::stage_elems(nx, nu, V, c.cls[1], c.cls[2]) : 0;
    c.sweep_lds = spk::sweep_int_bytes(p->N) + (spk::sweep_elems(nx, nu) + staged) * (int)sizeof(real);
    return c;
}
template spk::LaunchCfg make_cfg<double>(const spock_problem*, int);
template spk::LaunchCfg make_cfg<float>(const spock_problem*, int);

void step_bytes_of(const spock_problem* p, int w, double out[4]) {
    const double n = p->n, nl = p->n_nl, nlf = p->n_leaf, nx = p->nx, nu = p->nu, m = p->m;
    const double nc = p->nc, ncN = p->ncN, ny = (double)p->ny, edges = n - 1;
    const double aff = p->affine ? 1.0 : 0.0;
    // prep: K per non-leaf; z (x, u, y, tau, s), eta (c, soc, y, s, leaf blocks), probabilities, P c
    // in; y, tau, s, h0, ubar out
    out[0] = w * (nl * nu * nx + n * nx + nl * nu + 2 * ny + 2 * edges + nl * nc + edges * (m + 2) + nl +
                  nlf * (ncN + nx + 2) + edges + aff * n * nx + ny + 2 * edges + n * nx + nl * nu);
    // bsweep: [Abar|B] per edge, R~^-1 per non-leaf; h0, ubar, messages in; messages, d out
    out[1] = w * (edges * nx * m + nl * nu * nu + n * nx + nl * nu + 2 * edges * m + nl * nu);
    // fsweep: [Abar|B] per edge; d, c in; x out
    out[2] = w * (edges * m * nx + nl * nu + aff * n * nx + n * nx);
    // dual: K per non-leaf; z old and new, d, eta in; u, eta out
    out[3] = w * (nl * nx * nu + 2 * ((double)p->nz) + nl * nu + 2 * ((double)p->neta) + nl * nu);
}

static bool valid_wg(int wg) { return wg == 64 || wg == 128 || wg == 256 || wg == 512; }

// The iterate of the current precision moved to copy 0 (batched steps keep
// every member at the same parity).
int32_t normalize_parity(spock_problem* p) {
    if (p->cur == SPOCK_FP64 && p->s64.par == 1) {
        HIP_TRY(hipMemcpyAsync(p->s64.h.z[0], p->s64.h.z[1], p->nz * 8, hipMemcpyDeviceToDevice, p->stream));
        HIP_TRY(hipMemcpyAsync(p->s64.h.eta[0], p->s64.h.eta[1], p->neta * 8, hipMemcpyDeviceToDevice, p->stream));
        p->s64.par = 0;
    }
    if (p->cur != SPOCK_FP64 && p->s32.par == 1) {
        HIP_TRY(hipMemcpyAsync(p->s32.h.z[0], p->s32.h.z[1], p->nz * 4, hipMemcpyDeviceToDevice, p->stream));
        HIP_TRY(hipMemcpyAsync(p->s32.h.eta[0], p->s32.h.eta[1], p->neta * 4, hipMemcpyDeviceToDevice, p->stream));
        p->s32.par = 0;
    }
    return SPOCK_OK;
}

// Reference residuals of the first float64 CP step from zero (x0 already on
// the device).  A cold start (warm = false) keeps that step as iteration 1 and
// reports it in *taken; a warm start keeps its iterate untouched.
int32_t ensure_ref(spock_problem* p, bool warm, long long* taken, double* x1, double* x2) {
    *taken = 0;
    if (p->have_ref && warm) return SPOCK_OK;
    if (warm) {
        int32_t r = move_iterate(p, SPOCK_FP64);
        if (r) return r;
        HIP_TRY(hipMemcpyAsync(p->d_stash_z, p->s64.h.z[p->s64.par], p->nz * 8, hipMemcpyDeviceToDevice, p->stream));
        HIP_TRY(hipMemcpyAsync(p->d_stash_e, p->s64.h.eta[p->s64.par], p->neta * 8, hipMemcpyDeviceToDevice,
                               p->stream));
    }
    int32_t r = zero_iterate(p);
    if (!r) r = step<double>(p, 1);
    if (!r) r = read_res(p, x1, x2);
    if (r) return r;
    p->xi_ref[0] = *x1;
    p->xi_ref[1] = *x2;
    p->have_ref = true;
    if (warm) {
        HIP_TRY(hipMemcpyAsync(p->s64.h.z[0], p->d_stash_z, p->nz * 8, hipMemcpyDeviceToDevice, p->stream));
        HIP_TRY(hipMemcpyAsync(p->s64.h.eta[0], p->d_stash_e, p->neta * 8, hipMemcpyDeviceToDevice, p->stream));
        p->s64.par = 0;
        p->cur = SPOCK_FP64;
    } else {
        *taken = 1;
    }
    return SPOCK_OK;
}

extern "C" {

const char* spock_last_error(void) { return g_err.c_str(); }

int32_t spock_default_settings(spock_settings* s) {
    if (!s) return fail(SPOCK_E_INVALID, "null settings");
    s->alpha = 0.0;
    s->eps = 1e-6;
    s->max_iters = 100000;
    s->precision = SPOCK_FP64;
    s->precondition = 1;
    s->check_every = 20;
    s->use_graph = 1;
    s->method = SPOCK_CP;
    s->aa_memory = 3;
    return SPOCK_OK;
}

static int32_t check_settings(const spock_settings* s) {
    if (!s) return fail(SPOCK_E_INVALID, "null settings");
    if (!(s->alpha >= 0) || !std::isfinite(s->alpha)) return fail(SPOCK_E_INVALID, "alpha must be >= 0");
    if (!(s->eps > 0)) return fail(SPOCK_E_INVALID, "eps must be > 0");
    if (s->max_iters < 1) return fail(SPOCK_E_INVALID, "max_iters must be >= 1");
    if (s->precision < SPOCK_FP64 || s->precision > SPOCK_FP32) return fail(SPOCK_E_INVALID, "bad precision");
    if (s->check_every < 2 || (s->check_every & 1)) return fail(SPOCK_E_INVALID, "check_every must be even and >= 2");
    if (s->method != SPOCK_CP && s->method != SPOCK_SUPERMANN) return fail(SPOCK_E_INVALID, "bad method");
    if (s->method == SPOCK_SUPERMANN) {
        if (s->aa_memory < 1 || s->aa_memory > 8) return fail(SPOCK_E_INVALID, "aa_memory must be in 1..8");
        if (s->precision != SPOCK_FP64) return fail(SPOCK_E_INVALID, "SuperMann runs float64 iterations only");
    }
    return SPOCK_OK;
}

int32_t spock_problem_footprint(const spock_problem_desc* desc, const spock_settings* s, size_t* bytes) {
    if (!bytes) return fail(SPOCK_E_INVALID, "null output");
    int32_t r = check_settings(s);
    if (r) return r;
    spock_problem tmp;
    tmp.set = *s;
    r = validate_and_layout(desc, &tmp);
    if (r) return r;
    Arena a(nullptr);
    carve(a, &tmp);
    *bytes = a.off + 256;
    return SPOCK_OK;
}

int32_t spock_problem_create(const spock_problem_desc* desc, const spock_settings* s, void* ws, size_t ws_bytes,
                             void* stream, spock_problem** out) {
    if (!out) return fail(SPOCK_E_INVALID, "null output handle");
    *out = nullptr;
    int32_t r = check_settings(s);
    if (r) return r;
    spock_problem* p = nullptr;
    const double t_create = now_s();
    try {
        p = new spock_problem();
        p->set = *s;
        r = validate_and_layout(desc, p);
        if (r) {
            delete p;
            return r;
        }
        r = scale_data(desc, s->precondition, p);
        if (r) {
            delete p;
            return r;
        }
        p->alpha = s->alpha > 0 ? s->alpha : 0.99 / p->Lnorm;
        std::vector<double> M, KR, cs, Pc;
        r = offline_factor(desc, p, M, KR, cs, Pc);
        if (r) {
            delete p;
            return r;
        }
        Arena dry(nullptr);
        carve(dry, p);
        p->bytes = dry.off + 256;
        std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
        if (hipGetDevice(&p->device) != hipSuccess) {
            delete p;
            return fail(SPOCK_E_HIP, "hipGetDevice failed");
        }
        if (ws) {
            if (ws_bytes < p->bytes) {
                delete p;
                return fail(SPOCK_E_NOMEM, "device workspace smaller than the footprint");
            }
            p->base = ws;
        } else {
            hipError_t e = hipMalloc(&p->base, p->bytes);
            if (e != hipSuccess) {
                delete p;
                return fail(SPOCK_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
            }
            p->owns = true;
        }
        if (stream) {
            p->stream = (hipStream_t)stream;
        } else {
            hipError_t e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                spock_problem_destroy(p);
                return fail(SPOCK_E_HIP, "hipStreamCreate failed");
            }
            p->owns_stream = true;
        }
        if (hipHostMalloc((void**)&p->h_res, 2 * spk::kResSlots * sizeof(unsigned long long), 0) != hipSuccess) {
            spock_problem_destroy(p);
            return fail(SPOCK_E_HIP, "hipHostMalloc failed");
        }
        Arena a(p->base);
        carve(a, p);
        // tree arrays and tasks
        std::vector<int> tree(3 * (size_t)p->n + 4, 0);
        std::copy(p->first_child.begin(), p->first_child.end(), tree.begin());
        std::copy(p->n_ch.begin(), p->n_ch.end(), tree.begin() + p->n);
        std::copy(p->y_off.begin(), p->y_off.end(), tree.begin() + 2 * (size_t)p->n);
        std::vector<int> path, top;
        leaf_paths(p, path, top);
        std::vector<int2> tasks(p->n_leaf);
        for (int k = 0; k < p->n_leaf; ++k) tasks[k] = make_int2(0, k);
        std::vector<int2> ntasks(p->n_ntasks, make_int2(0, -1));
        std::vector<int4> ninfo(p->n_ntasks, make_int4(0, 0, 0, 0));
        for (int v = 0; v < p->n; ++v) {
            ntasks[v] = make_int2(0, v);
            ninfo[v] = make_int4(p->n_ch[v] ? p->first_child[v] : 0, p->n_ch[v], v < p->n_nl ? p->y_off[v] : 0,
                                 p->parent[v]);
        }
        hipError_t e = hipMemcpy(p->d_tree, tree.data(), tree.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess && p->grisk) {
            std::vector<int> rint(p->rny);
            rint.insert(rint.end(), p->rnnu.begin(), p->rnnu.end());
            e = hipMemcpy(p->d_rint, rint.data(), rint.size() * sizeof(int), hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(p->d_roff, p->roff.data(), p->roff.size() * sizeof(long long), hipMemcpyHostToDevice);
        }
        if (e == hipSuccess)
            e = hipMemcpy(p->d_ntasks, ntasks.data(), ntasks.size() * sizeof(int2), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(p->d_ninfo, ninfo.data(), ninfo.size() * sizeof(int4), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(p->d_tasks, tasks.data(), tasks.size() * sizeof(int2), hipMemcpyHostToDevice);
        std::vector<int4> path4(path.size());
        for (size_t q = 0; q < path.size(); ++q) {
            const int v = path[q];
            path4[q] = make_int4(v, p->n_ch[v], p->n_ch[v] ? p->first_child[v] : 0, 0);
        }
        if (e == hipSuccess)
            e = hipMemcpy(p->d_path, path4.data(), path4.size() * sizeof(int4), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(p->d_top, top.data(), top.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            spock_problem_destroy(p);
            return fail(SPOCK_E_HIP, std::string("upload: ") + hipGetErrorString(e));
        }
        // arrival counters and residual slots start at zero; the active flag at one
        e = spk::launch_fill<int>(p->d_cnt, 0, p->n, p->stream);
        if (e == hipSuccess) e = spk::launch_fill<int>(p->d_one, 1, 1, p->stream);
        if (e == hipSuccess) e = spk::launch_fill<unsigned long long>(p->d_res, 0ull, 2 * spk::kResSlots, p->stream);
        if (e != hipSuccess) {
            spock_problem_destroy(p);
            return fail(SPOCK_E_HIP, std::string("init: ") + hipGetErrorString(e));
        }
        r = upload_set<double>(p, p->s64, M, KR, cs, Pc);
        if (!r) r = upload_set<float>(p, p->s32, M, KR, cs, Pc);
        if (!r && p->set.method == SPOCK_SUPERMANN) r = upload_supermann(p);
        if (r) {
            spock_problem_destroy(p);
            return r;
        }
        p->t_setup = now_s() - t_create;
        *out = p;
        return SPOCK_OK;
    } catch (const std::bad_alloc&) {
        if (p) spock_problem_destroy(p);
        return fail(SPOCK_E_NOMEM, "host allocation failed");
    } catch (const std::exception& ex) {
        if (p) spock_problem_destroy(p);
        return fail(SPOCK_E_INVALID, ex.what());
    }
}

int32_t spock_problem_destroy(spock_problem* p) {
    if (!p) return SPOCK_OK;
    std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    for (auto* s : {&p->s64.graph[0], &p->s64.graph[1], &p->s32.graph[0], &p->s32.graph[1]})
        if (*s) (void)hipGraphExecDestroy(*s);
    if (p->h_res) (void)hipHostFree(p->h_res);
    if (p->sm.h_dots) (void)hipHostFree(p->sm.h_dots);
    if (p->owns && p->base) (void)hipFree(p->base);
    if (p->owns_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
    return SPOCK_OK;
}

int32_t spock_problem_sizes(const spock_problem* p, spock_sizes* o) {
    if (!p || !o) return fail(SPOCK_E_INVALID, "null argument");
    o->nz = p->nz;
    o->neta = p->neta;
    o->n = p->n;
    o->n_nl = p->n_nl;
    o->n_leaf = p->n_leaf;
    o->N = p->N;
    o->nx = p->nx;
    o->nu = p->nu;
    o->nc = p->nc;
    o->ncN = p->ncN;
    o->max_children = p->max_ch;
    o->alpha = p->alpha;
    o->L_norm = p->Lnorm;
    o->device_bytes = p->bytes;
    return SPOCK_OK;
}

int32_t spock_set_settings(spock_problem* p, const spock_settings* s) {
    if (!p) return fail(SPOCK_E_INVALID, "null handle");
    int32_t r = check_settings(s);
    if (r) return r;
    if (s->alpha != p->set.alpha && s->alpha > 0 && s->alpha != p->alpha)
        return fail(SPOCK_E_INVALID, "alpha is fixed at create time");
    if (s->precondition != p->set.precondition) return fail(SPOCK_E_INVALID, "precondition is fixed at create time");
    if (s->method != p->set.method) return fail(SPOCK_E_INVALID, "method is fixed at create time");
    if (s->method == SPOCK_SUPERMANN && s->aa_memory != p->set.aa_memory)
        return fail(SPOCK_E_INVALID, "aa_memory is fixed at create time");
    p->set = *s;
    return SPOCK_OK;
}

int32_t spock_set_x0(spock_problem* p, const double* x0) {
    if (!p) return fail(SPOCK_E_INVALID, "null handle");
    return set_x0_device(p, x0, false);
}


// Run chunks in one precision until rel_res <= eps, the step budget is spent,
// or (float32 only) progress stalls.  Returns SPOCK_OK on convergence.
extern "C++" {
template <typename real>
static int32_t iterate(spock_problem* p, long long budget, long long* taken, double* rel, double* x1, double* x2,
                       bool stall_exit) {
    const double scale = std::max(1.0, std::max(p->xi_ref[0], p->xi_ref[1]));
    const int ce = p->set.check_every;
    double best = INFINITY;
    int no_gain = 0, checks = 0;
    *taken = 0;
    while (*taken < budget) {
        int32_t r = chunk<real>(p, ce);
        if (r) return r;
        *taken += ce;
        r = read_res(p, x1, x2);
        if (r) return r;
        *rel = rel_of(*x1, *x2, scale);
        if (!std::isfinite(*rel)) return fail(SPOCK_E_DIVERGED, "non-finite residual");
        if (*rel <= p->set.eps) return SPOCK_OK;
        if (stall_exit) {
            // float32 progress stalls only at its rounding floor; plain CP
            // residuals oscillate, so "no gain" is judged over a window that
            // grows with the run (half of the checks so far, at least 50)
            ++checks;
            if (*rel < 0.99 * best) {
                best = *rel;
                no_gain = 0;
            } else if (++no_gain >= std::max(50, checks / 2)) {
                return SPOCK_E_NOT_CONVERGED;
            }
        }
    }
    return SPOCK_E_NOT_CONVERGED;
}
}  // extern "C++"


// SuperMann solve (Sec. 5.2): float64 iterate in copy 0 with its CP step
// taken, reference residuals of the first CP step from zero, then the
// accelerated iteration.
static int32_t supermann_solve(spock_problem* p, int32_t warm, spock_info* info, double t0) {
    spock_info inf{};
    int32_t r = SPOCK_OK;
    if (!warm) {
        r = zero_iterate(p);
        if (r) return r;
    } else {
        r = move_iterate(p, SPOCK_FP64);
        if (!r) r = normalize_parity(p);
        if (r) return r;
    }
    if (!p->have_ref || !warm) {
        long long taken = 0;
        double x1, x2;
        r = ensure_ref(p, warm != 0, &taken, &x1, &x2);
        if (r) return r;
        // a cold start keeps the reference step: copy 1 holds T(0)
        if (!taken) r = step<double>(p, 1);
    } else {
        r = step<double>(p, 1);
    }
    if (r) return r;
    p->s64.par = 0;  // the SuperMann loop reads v in copy 0 and T(v) in copy 1
    r = supermann_iterate(p, p->set.max_iters, &inf);
    if (r != SPOCK_OK && r != SPOCK_E_NOT_CONVERGED && r != SPOCK_E_DIVERGED) return r;
    p->solved = true;
    double s0 = 0;
    HIP_TRY(hipMemcpyAsync(&s0, p->s64.h.z[0], 8, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    inf.s0 = s0;
    inf.precision_used = SPOCK_FP64;
    inf.t_setup_s = p->t_setup;
    inf.t_solve_s = now_s() - t0;
    if (info) *info = inf;
    if (r == SPOCK_E_NOT_CONVERGED) return fail(r, "max_iters reached before the tolerance");
    if (r == SPOCK_E_DIVERGED) return fail(r, "non-finite residual");
    return SPOCK_OK;
}

int32_t spock_solve(spock_problem* p, const double* x0, int32_t warm, spock_info* info) {
    if (!p) return fail(SPOCK_E_INVALID, "null handle");
    const double t0 = now_s();
    spock_info inf{};
    int32_t r = set_x0_device(p, x0, true);
    if (r) return r;
    if (p->set.method == SPOCK_SUPERMANN) return supermann_solve(p, warm, info, t0);
    long long it = 0, it32 = 0;
    double rel = INFINITY, x1 = INFINITY, x2 = INFINITY;
    const int prec = p->set.precision;
    if (!warm) {
        r = zero_iterate(p);
        if (r) return r;
    }
    if (!p->have_ref || !warm) {
        // reference residuals: the first CP step from zero (float64)
        const bool keep = warm != 0;
        if (keep) {
            r = move_iterate(p, SPOCK_FP64);
            if (r) return r;
            HIP_TRY(hipMemcpyAsync(p->d_stash_z, p->s64.h.z[p->s64.par], p->nz * 8, hipMemcpyDeviceToDevice, p->stream));
            HIP_TRY(hipMemcpyAsync(p->d_stash_e, p->s64.h.eta[p->s64.par], p->neta * 8, hipMemcpyDeviceToDevice, p->stream));
            r = zero_iterate(p);
            if (r) return r;
        }
        r = step<double>(p, 1);
        if (r) return r;
        r = read_res(p, &x1, &x2);
        if (r) return r;
        p->xi_ref[0] = x1;
        p->xi_ref[1] = x2;
        p->have_ref = true;
        if (keep) {
            HIP_TRY(hipMemcpyAsync(p->s64.h.z[0], p->d_stash_z, p->nz * 8, hipMemcpyDeviceToDevice, p->stream));
            HIP_TRY(hipMemcpyAsync(p->s64.h.eta[0], p->d_stash_e, p->neta * 8, hipMemcpyDeviceToDevice, p->stream));
            p->s64.par = 0;
        } else {
            it = 1;
            rel = rel_of(x1, x2, std::max(1.0, std::max(x1, x2)));
        }
    }
    const long long budget = p->set.max_iters;
    int used = SPOCK_FP64;
    int refined = 0;
    long long taken = 0;
    if (prec == SPOCK_FP64) {
        r = move_iterate(p, SPOCK_FP64);
        if (!r && !(it > 0 && rel <= p->set.eps)) r = iterate<double>(p, budget - it, &taken, &rel, &x1, &x2, false);
        it += taken;
    } else {
        r = move_iterate(p, SPOCK_FP32);
        if (r) return r;
        r = iterate<float>(p, budget - it, &taken, &rel, &x1, &x2, prec == SPOCK_MIXED);
        it += taken;
        it32 = taken;
        used = SPOCK_FP32;
        if (prec == SPOCK_MIXED && (r == SPOCK_OK || r == SPOCK_E_NOT_CONVERGED)) {
            // float64 check of the float32 iterate; refine in float64 if needed
            int32_t r2 = move_iterate(p, SPOCK_FP64);
            if (r2) return r2;
            used = SPOCK_FP64;
            r2 = step<double>(p, 1);
            if (!r2) r2 = read_res(p, &x1, &x2);
            if (r2) return r2;
            it += 1;
            rel = rel_of(x1, x2, std::max(1.0, std::max(p->xi_ref[0], p->xi_ref[1])));
            if (rel <= p->set.eps) {
                r = SPOCK_OK;
            } else if (it < budget) {
                refined = 1;
                r = iterate<double>(p, budget - it, &taken, &rel, &x1, &x2, false);
                it += taken;
            } else {
                r = SPOCK_E_NOT_CONVERGED;
            }
        }
    }
    if (r != SPOCK_OK && r != SPOCK_E_NOT_CONVERGED && r != SPOCK_E_DIVERGED) return r;
    p->solved = true;
    inf.iters = it;
    inf.iters_fp32 = it32;
    inf.n_T = it;
    inf.rel_res = rel;
    inf.xi1_inf = x1;
    inf.xi2_inf = x2;
    double s0 = 0;
    if (p->cur == SPOCK_FP64) {
        HIP_TRY(hipMemcpyAsync(&s0, p->s64.h.z[p->s64.par], 8, hipMemcpyDeviceToHost, p->stream));
    } else {
        float f = 0;
        HIP_TRY(hipMemcpyAsync(&f, p->s32.h.z[p->s32.par], 4, hipMemcpyDeviceToHost, p->stream));
        HIP_TRY(hipStreamSynchronize(p->stream));
        s0 = f;
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    inf.s0 = s0;
    inf.status = r;
    inf.precision_used = used;
    inf.refined = refined;
    inf.t_setup_s = p->t_setup;
    inf.t_solve_s = now_s() - t0;
    if (info) *info = inf;
    if (r == SPOCK_E_NOT_CONVERGED) return fail(r, "max_iters reached before the tolerance");
    if (r == SPOCK_E_DIVERGED) return fail(r, "non-finite residual");
    return SPOCK_OK;
}

// float64 copy of the current iterate on the host
static int32_t fetch_iterate(const spock_problem* pc, std::vector<double>& z, std::vector<double>& e) {
    spock_problem* p = const_cast<spock_problem*>(pc);
    z.resize(p->nz);
    e.resize(p->neta);
    if (p->cur == SPOCK_FP64) {
        HIP_TRY(hipMemcpyAsync(z.data(), p->s64.h.z[p->s64.par], p->nz * 8, hipMemcpyDeviceToHost, p->stream));
        HIP_TRY(hipMemcpyAsync(e.data(), p->s64.h.eta[p->s64.par], p->neta * 8, hipMemcpyDeviceToHost, p->stream));
    } else {
        HIP_TRY(spk::launch_convert<double, float>(p->d_stash_z, p->s32.h.z[p->s32.par], p->nz, p->stream));
        HIP_TRY(spk::launch_convert<double, float>(p->d_stash_e, p->s32.h.eta[p->s32.par], p->neta, p->stream));
        HIP_TRY(hipMemcpyAsync(z.data(), p->d_stash_z, p->nz * 8, hipMemcpyDeviceToHost, p->stream));
        HIP_TRY(hipMemcpyAsync(e.data(), p->d_stash_e, p->neta * 8, hipMemcpyDeviceToHost, p->stream));
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    return SPOCK_OK;
}

int32_t spock_get_solution(const spock_problem* p, double* x, double* u, double* s0) {
    if (!p) return fail(SPOCK_E_INVALID, "null handle");
    std::vector<double> z, e;
    int32_t r = fetch_iterate(p, z, e);
    if (r) return r;
    const int nx = p->nx, nu = p->nu;
    if (x)
        for (int j = 0; j < p->n; ++j) {
            const std::vector<double>& S = j < p->n_nl ? p->Sx : p->SxN;
            for (int k = 0; k < nx; ++k) x[(size_t)j * nx + k] = z[p->z_x + (size_t)j * nx + k] / S[k];
        }
    if (u)
        for (int i = 0; i < p->n_nl; ++i)
            for (int k = 0; k < nu; ++k) u[(size_t)i * nu + k] = z[p->z_u + (size_t)i * nu + k] / p->Su[k];
    if (s0) *s0 = z[0];
    return SPOCK_OK;
}

int32_t spock_get_iterate(const spock_problem* p, double* z, double* eta) {
    if (!p) return fail(SPOCK_E_INVALID, "null handle");
    std::vector<double> zz, ee;
    int32_t r = fetch_iterate(p, zz, ee);
    if (r) return r;
    if (z) std::copy(zz.begin(), zz.end(), z);
    if (eta) std::copy(ee.begin(), ee.end(), eta);
    return SPOCK_OK;
}

// host float64 arrays -> copy 0 of the given precision
static int32_t load_iterate(spock_problem* p, const double* z, const double* eta, int prec) {
    if (!z || !eta) return fail(SPOCK_E_INVALID, "null iterate");
    if (prec == SPOCK_FP64) {
        HIP_TRY(hipMemcpyAsync(p->s64.h.z[0], z, p->nz * 8, hipMemcpyHostToDevice, p->stream));
        HIP_TRY(hipMemcpyAsync(p->s64.h.eta[0], eta, p->neta * 8, hipMemcpyHostToDevice, p->stream));
        p->s64.par = 0;
        p->cur = SPOCK_FP64;
    } else {
        HIP_TRY(hipMemcpyAsync(p->d_stash_z, z, p->nz * 8, hipMemcpyHostToDevice, p->stream));
        HIP_TRY(hipMemcpyAsync(p->d_stash_e, eta, p->neta * 8, hipMemcpyHostToDevice, p->stream));
        HIP_TRY(spk::launch_convert<float, double>(p->s32.h.z[0], p->d_stash_z, p->nz, p->stream));
        HIP_TRY(spk::launch_convert<float, double>(p->s32.h.eta[0], p->d_stash_e, p->neta, p->stream));
        p->s32.par = 0;
        p->cur = SPOCK_FP32;
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    return SPOCK_OK;
}

int32_t spock_set_iterate(spock_problem* p, const double* z, const double* eta) {
    if (!p) return fail(SPOCK_E_INVALID, "null handle");
    return load_iterate(p, z, eta, SPOCK_FP64);
}

static int32_t check_prec(int32_t prec) {
    if (prec != SPOCK_FP64 && prec != SPOCK_FP32) return fail(SPOCK_E_INVALID, "hooks take SPOCK_FP64 or SPOCK_FP32");
    return SPOCK_OK;
}

int32_t spock_apply_T(spock_problem* p, const double* z, const double* eta, double* z_out, double* eta_out,
                      int32_t prec, double* xi) {
    if (!p) return fail(SPOCK_E_INVALID, "null handle");
    int32_t r = check_prec(prec);
    if (!r) r = load_iterate(p, z, eta, prec);
    if (!r) r = prec == SPOCK_FP64 ? step<double>(p, 1) : step<float>(p, 1);
    double a = 0, b = 0;
    if (!r) r = read_res(p, &a, &b);
    if (r) return r;
    if (xi) {
        xi[0] = a;
        xi[1] = b;
    }
    std::vector<double> zz, ee;
    r = fetch_iterate(p, zz, ee);
    if (r) return r;
    if (z_out) std::copy(zz.begin(), zz.end(), z_out);
    if (eta_out) std::copy(ee.begin(), ee.end(), eta_out);
    return SPOCK_OK;
}

// The z part of T with eta = 0 is prox_{alpha f}(z) (zbar = z): its (x, u)
// block is the S1 projection (Alg. 2) and its (y, tau, s) block the S2
// projection of every non-leaf node, computed by the step's own kernels.
static int32_t prox_f_only(spock_problem* p, std::vector<double>& z, int32_t prec) {
    std::vector<double> eta(p->neta, 0.0), zo(p->nz, 0.0);
    int32_t r = spock_apply_T(p, z.data(), eta.data(), zo.data(), nullptr, prec, nullptr);
    if (r) return r;
    z.swap(zo);
    return SPOCK_OK;
}

int32_t spock_project_S1(spock_problem* p, const double* xbar, const double* ubar, double* x_out, double* u_out,
                         int32_t prec) {
    if (!p || !xbar || !ubar || !x_out || !u_out) return fail(SPOCK_E_INVALID, "null argument");
    int32_t r = check_prec(prec);
    if (r) return r;
    try {
        std::vector<double> z(p->nz, 0.0);
        std::copy(xbar, xbar + (size_t)p->n * p->nx, z.begin() + p->z_x);
        std::copy(ubar, ubar + (size_t)p->n_nl * p->nu, z.begin() + p->z_u);
        r = prox_f_only(p, z, prec);
        if (r) return r;
        std::copy(z.begin() + p->z_x, z.begin() + p->z_x + (size_t)p->n * p->nx, x_out);
        std::copy(z.begin() + p->z_u, z.begin() + p->z_u + (size_t)p->n_nl * p->nu, u_out);
    } catch (const std::bad_alloc&) {
        return fail(SPOCK_E_NOMEM, "host allocation failed");
    }
    return SPOCK_OK;
}

int32_t spock_project_S2(spock_problem* p, const double* y, const double* tau, const double* s, double* y_out,
                         double* tau_out, double* s_out, int32_t prec) {
    if (!p || !y || !tau || !s || !y_out || !tau_out || !s_out) return fail(SPOCK_E_INVALID, "null argument");
    int32_t r = check_prec(prec);
    if (r) return r;
    try {
        const size_t e = (size_t)p->n - 1;
        std::vector<double> z(p->nz, 0.0);
        std::copy(y, y + p->ny, z.begin() + p->z_y);
        std::copy(tau, tau + e, z.begin() + p->z_tau);
        std::copy(s, s + e, z.begin() + p->z_s);
        r = prox_f_only(p, z, prec);
        if (r) return r;
        std::copy(z.begin() + p->z_y, z.begin() + p->z_y + p->ny, y_out);
        std::copy(z.begin() + p->z_tau, z.begin() + p->z_tau + e, tau_out);
        std::copy(z.begin() + p->z_s, z.begin() + p->z_s + e, s_out);
    } catch (const std::bad_alloc&) {
        return fail(SPOCK_E_NOMEM, "host allocation failed");
    }
    return SPOCK_OK;
}

extern "C++" {
template <typename real>
static int32_t hook(spock_problem* p, int which, const double* in, long long nin, double* out, long long nout) {
    DevSet<real>& s = set_of<real>(p);
    // input -> copy 0 (z or eta as needed), output -> the other buffer kind of copy 1
    real* din = which == 0 ? s.h.z[0] : s.h.eta[0];
    real* dout = which == 1 ? s.h.z[1] : s.h.eta[1];
    HIP_TRY(hipMemcpyAsync(p->d_stash_z, in, nin * 8, hipMemcpyHostToDevice, p->stream));
    if (sizeof(real) == 8) {
        HIP_TRY(hipMemcpyAsync(din, p->d_stash_z, nin * 8, hipMemcpyDeviceToDevice, p->stream));
    } else {
        HIP_TRY(spk::launch_convert<float, double>((float*)din, p->d_stash_z, nin, p->stream));
    }
    HIP_TRY(spk::launch_fill<real>(dout, real(0), nout, p->stream));
    if (which == 0) HIP_TRY(spk::launch_apply_L<real>(s.d, p->n, din, dout, p->stream));
    if (which == 1) HIP_TRY(spk::launch_apply_Lt<real>(s.d, p->n, din, dout, p->stream));
    if (which == 2) HIP_TRY(spk::launch_prox_gconj<real>(s.d, p->n, din, dout, p->stream));
    if (sizeof(real) == 8) {
        HIP_TRY(hipMemcpyAsync(out, dout, nout * 8, hipMemcpyDeviceToHost, p->stream));
    } else {
        HIP_TRY(spk::launch_convert<double, float>(p->d_stash_e, (const float*)dout, nout, p->stream));
        HIP_TRY(hipMemcpyAsync(out, p->d_stash_e, nout * 8, hipMemcpyDeviceToHost, p->stream));
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    return SPOCK_OK;
}
}  // extern "C++"


int32_t spock_apply_L(spock_problem* p, const double* z, double* eta_out, int32_t prec) {
    if (!p || !z || !eta_out) return fail(SPOCK_E_INVALID, "null argument");
    int32_t r = check_prec(prec);
    if (r) return r;
    return prec == SPOCK_FP64 ? hook<double>(p, 0, z, p->nz, eta_out, p->neta)
                              : hook<float>(p, 0, z, p->nz, eta_out, p->neta);
}

int32_t spock_apply_Lt(spock_problem* p, const double* eta, double* z_out, int32_t prec) {
    if (!p || !eta || !z_out) return fail(SPOCK_E_INVALID, "null argument");
    int32_t r = check_prec(prec);
    if (r) return r;
    return prec == SPOCK_FP64 ? hook<double>(p, 1, eta, p->neta, z_out, p->nz)
                              : hook<float>(p, 1, eta, p->neta, z_out, p->nz);
}

int32_t spock_prox_gconj(spock_problem* p, const double* w, double* eta_out, int32_t prec) {
    if (!p || !w || !eta_out) return fail(SPOCK_E_INVALID, "null argument");
    int32_t r = check_prec(prec);
    if (r) return r;
    return prec == SPOCK_FP64 ? hook<double>(p, 2, w, p->neta, eta_out, p->neta)
                              : hook<float>(p, 2, w, p->neta, eta_out, p->neta);
}

extern "C++" {
template <typename real>
static int32_t time_steps(spock_problem* p, int steps, double* ms_total, double ms_k[4]) {
    DevSet<real>& s = set_of<real>(p);
    std::vector<hipEvent_t> ev(4 * (size_t)steps + 1);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    HIP_TRY(hipEventRecord(ev[0], p->stream));
    for (int k = 0; k < steps; ++k) {
        for (int ph = 0; ph < 4; ++ph) {
            HIP_TRY(spk::launch_phase<real>(s.d, s.cfg, ph, s.par, 0, p->stream));
            HIP_TRY(hipEventRecord(ev[4 * k + ph + 1], p->stream));
        }
        s.par ^= 1;
    }
    HIP_TRY(hipEventSynchronize(ev.back()));
    double t[4] = {0, 0, 0, 0};
    for (int k = 0; k < steps; ++k)
        for (int ph = 0; ph < 4; ++ph) {
            float a = 0;
            HIP_TRY(hipEventElapsedTime(&a, ev[4 * k + ph], ev[4 * k + ph + 1]));
            t[ph] += a;
        }
    float tot = 0;
    HIP_TRY(hipEventElapsedTime(&tot, ev[0], ev.back()));
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (ms_total) *ms_total = tot / steps;
    for (int ph = 0; ph < 4; ++ph) ms_k[ph] = t[ph] / steps;
    return SPOCK_OK;
}
}  // extern "C++"


int32_t spock_time_steps(spock_problem* p, int32_t prec, int32_t steps, double* ms_total, double* ms_b,
                         double* ms_f) {
    if (!p || steps < 1) return fail(SPOCK_E_INVALID, "bad argument");
    int32_t r = check_prec(prec);
    if (r) return r;
    r = move_iterate(p, prec);
    if (r) return r;
    double k[4];
    r = prec == SPOCK_FP64 ? time_steps<double>(p, steps, ms_total, k) : time_steps<float>(p, steps, ms_total, k);
    if (r) return r;
    if (ms_b) *ms_b = k[0] + k[1];
    if (ms_f) *ms_f = k[2] + k[3];
    return SPOCK_OK;
}

int32_t spock_time_kernels(spock_problem* p, int32_t prec, int32_t steps, double* ms_total, double* ms_kernels) {
    if (!p || steps < 1 || !ms_kernels) return fail(SPOCK_E_INVALID, "bad argument");
    int32_t r = check_prec(prec);
    if (r) return r;
    r = move_iterate(p, prec);
    if (r) return r;
    return prec == SPOCK_FP64 ? time_steps<double>(p, steps, ms_total, ms_kernels)
                              : time_steps<float>(p, steps, ms_total, ms_kernels);
}

int32_t spock_set_launch(spock_problem* p, int32_t precision, int32_t workgroup) {
    if (!p || !valid_wg(workgroup)) return fail(SPOCK_E_INVALID, "workgroup must be 64, 128, 256 or 512");
    const int bytes = precision == SPOCK_FP64 ? 8 : 4;
    if (node_lds_bytes(p, workgroup, bytes) > 64 * 1024) return fail(SPOCK_E_INVALID, "LDS too large");
    HIP_TRY(hipStreamSynchronize(p->stream));
    auto apply = [&](auto& s, auto cfg) {
        if (s.cfg.node_wg == workgroup) return;
        s.cfg = cfg;
        for (auto& g : s.graph)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
        s.graph_steps = 0;
    };
    if (precision == SPOCK_FP64) apply(p->s64, make_cfg<double>(p, workgroup));
    else apply(p->s32, make_cfg<float>(p, workgroup));
    return SPOCK_OK;
}

int32_t spock_get_launch(const spock_problem* p, int32_t precision, int32_t* workgroup) {
    if (!p || !workgroup) return fail(SPOCK_E_INVALID, "null argument");
    *workgroup = precision == SPOCK_FP64 ? p->s64.cfg.node_wg : p->s32.cfg.node_wg;
    return SPOCK_OK;
}

int32_t spock_run_steps(spock_problem* p, int32_t prec, int32_t steps, int32_t sync) {
    if (!p || steps < 0) return fail(SPOCK_E_INVALID, "bad argument");
    int32_t r = check_prec(prec);
    if (!r) r = move_iterate(p, prec);
    for (int k = 0; !r && k < steps; ++k) r = prec == SPOCK_FP64 ? step<double>(p, 0) : step<float>(p, 0);
    if (r) return r;
    if (sync) HIP_TRY(hipStreamSynchronize(p->stream));
    return SPOCK_OK;
}

int32_t spock_step_bytes(const spock_problem* p, int32_t prec, double* bb, double* bf) {
    if (!p) return fail(SPOCK_E_INVALID, "null handle");
    double k[4];
    step_bytes_of(p, prec == SPOCK_FP64 ? 8 : 4, k);
    if (bb) *bb = k[0] + k[1];
    if (bf) *bf = k[2] + k[3];
    return SPOCK_OK;
}

int32_t spock_kernel_bytes(const spock_problem* p, int32_t prec, double* bytes) {
    if (!p || !bytes) return fail(SPOCK_E_INVALID, "null argument");
    step_bytes_of(p, prec == SPOCK_FP64 ? 8 : 4, bytes);
    return SPOCK_OK;
}

}  // extern "C"

template int32_t step<double>(spock_problem*, int);
template int32_t step<float>(spock_problem*, int);
