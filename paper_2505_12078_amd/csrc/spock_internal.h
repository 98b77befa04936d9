// Internal declarations shared by the host sources of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/spock.h"
#include "spock_dev.h"

namespace spk {
// one CP step: the four launches in order (par: copy holding the iterate,
// check: residuals of this step into res)
template <typename real>
hipError_t launch_step(const ProbDev<real>*, const LaunchCfg&, int par, int check, hipStream_t);
// one of them: 0 prep, 1 bsweep, 2 fsweep, 3 dual
template <typename real>
hipError_t launch_phase(const ProbDev<real>*, const LaunchCfg&, int phase, int par, int check, hipStream_t);
template <typename real>
hipError_t launch_apply_L(const ProbDev<real>*, int, const real*, real*, hipStream_t);
template <typename real>
hipError_t launch_apply_Lt(const ProbDev<real>*, int, const real*, real*, hipStream_t);
template <typename real>
hipError_t launch_prox_gconj(const ProbDev<real>*, int, const real*, real*, hipStream_t);
template <typename D, typename S>
hipError_t launch_convert(D*, const S*, long long, hipStream_t);
template <typename T>
hipError_t launch_fill(T*, T, long long, hipStream_t);
hipError_t launch_combo(double* out, const VecCombo& cb, long long n, hipStream_t);
hipError_t launch_dots(const DotSet& ds, double* partial, double* out, hipStream_t);
}  // namespace spk


// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

extern thread_local std::string g_err;

// Held while a stream is being captured into a graph and while device memory,
// streams and uploads of a problem or a batch are set up or torn down.  The
// runtime invalidates a capture in progress when another thread makes such
// calls at the same time (the server sets up trees on its own thread).
std::recursive_mutex& hip_setup_mutex();
int32_t fail(int32_t code, const std::string& msg);

#define HIP_TRY(...)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (__VA_ARGS__);                                                          \
        if (e_ != hipSuccess)                                                                   \
            return fail(SPOCK_E_HIP, std::string(#__VA_ARGS__ ": ") + hipGetErrorString(e_));    \
    } while (0)

using spk::ProbDev;

// ---------------------------------------------------------------------------
// the handle
// ---------------------------------------------------------------------------

template <typename real>
struct DevSet {
    ProbDev<real> h;           // host mirror of the descriptor
    ProbDev<real>* d = nullptr;  // the descriptor in device memory
    int par = 0;               // which copy holds the current iterate
    spk::LaunchCfg cfg{};      // tasks, LDS and tile classes of the four launches
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // check_every steps from parity 0 / 1
    int graph_steps = 0;
};

// Device vectors of the SuperMann iteration (float64, [z | pad | eta] each
// unless noted), carved from the handle's workspace when the method is
// SuperMann.
struct SmWork {
    double* R[2] = {nullptr, nullptr};  // residual v - T(v): current and previous
    double* PSI = nullptr;              // Anderson direction
    double* VT = nullptr;               // line-search trial v + tau psi
    double* TVT = nullptr;              // T(trial)
    double* RT = nullptr;               // trial residual
    double* Y[8] = {};                  // residual differences (ring of aa_memory)
    double* S[8] = {};                  // iterate differences (ring)
    double* LR = nullptr;               // L r_z, L psi_z, L rt_z (eta-sized)
    double* LPSI = nullptr;
    double* LRT = nullptr;
    double* partial = nullptr;          // dot-product block partials
    double* dots = nullptr;             // dot-product results
    ProbDev<double>* d_trial = nullptr; // float64 descriptor reading VT, writing TVT
    double* h_dots = nullptr;           // pinned readback of dots and residual slots
};

struct spock_problem {
    // sizes
    int n = 0, n_nl = 0, n_leaf = 0, N = 0, nx = 0, nu = 0, m = 0, nc = 0, ncN = 0, max_ch = 0;
    int stage_kids = 16;  // children whose per-child inputs the node kernels stage in LDS
    int has_ball = 0, has_ballN = 0, affine = 0;
    long long ny = 0, nz = 0, neta = 0, nzp = 0;  // nzp: nz rounded up to 64 entries
    long long z_x, z_u, z_y, z_tau, z_s, e_y, e_s, e_c, e_soc, e_cN, e_socN;
    long long M_stride = 0, KR_stride = 0;
    std::vector<int> parent, first_child, n_ch, y_off;
    // scaled problem data
    std::vector<double> Sx, Su, SxN;
    std::vector<double> qh, rh, qnh, gx, gu, gb, gxN, gbN, lo, hi, loN, hiN, prob, gamma;
    // translations a of Prop. 1 with linear cost terms (has_lin): per edge
    // j = 1..n-1 (m + 2 each) and per leaf (nx + 2 each)
    int has_lin = 0;
    std::vector<double> sa, saN;
    // Prop. 1 with a singular R (diagonal R with zero entries): the linear
    // term r_k of an input without quadratic cost enters the edge's two tau
    // rows of L as -(c^T u) / 2 each; ck [n][nu] by edge, in the scaled
    // inputs (r_k / Su_k on those inputs, 0 elsewhere)
    int coupled = 0;
    std::vector<double> ck;
    // per-edge / per-leaf cost square roots in the scaled space (qh_e [n][nx],
    // rh_e [n][nu] by edge, qnh_l [n_leaf][nx] by leaf), used when the
    // description gives per-edge costs (edge_cost) or per-leaf ones (leaf_cost)
    int edge_cost = 0, leaf_cost = 0;
    std::vector<double> qh_e, rh_e, qnh_l;
    // dense costs (dense_edge: Q and R per edge, dense_leaf: QN per leaf):
    // the symmetric square roots Hq_e [n][nx][nx], Hr_e [n][nu][nu] by edge and
    // HqN_l [n_leaf][nx][nx] by leaf; qh, rh (qnh) then hold S_x^-1, S_u^-1
    // (S_xN^-1), so that the cost rows are H (qh o x)
    int dense_edge = 0, dense_leaf = 0;
    std::vector<double> Hq_e, Hr_e, HqN_l;
    // general constraints (gen: non-leaf rows Gamma, genN: leaf rows Gamma_N)
    // in the scaled space: Gt [nc][m] and GtT [m][nc], GNt [ncN][nx] and GNtT
    int gen = 0, genN = 0;
    int nbox = 0, nboxN = 0;
    std::vector<double> Gt, GtT, GNt, GNtT;
    // general coherent risks (grisk): per non-leaf node its y length rny, F
    // columns rnnu and a packed block at roff of rdata: E (ny x k), F
    // (ny x nnu), b (ny), cone codes (ny, 0 or 1), M = (G G^T)^-1 ((k + nnu)^2)
    int grisk = 0;
    std::vector<int> rny, rnnu;
    std::vector<long long> roff;
    std::vector<double> rdata;
    double ball_r = 0, ballN_r = 0, con_scale = 1, con_scaleN = 1;
    double Lnorm = 0, alpha = 0;
    // unscaled root constraint for the x0 check
    std::vector<double> x_lo, x_hi;
    double x_ball = 0;
    std::vector<double> x0s;   // scaled x0 currently on the device
    spock_settings set{};
    // device
    void* base = nullptr;
    bool owns = false;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    int* d_tree = nullptr;
    long long* d_roff = nullptr;  // general risks: per-node block offsets
    int* d_rint = nullptr;        //                y lengths, then F columns
    int* d_cnt = nullptr;
    int4* d_path = nullptr;
    int* d_top = nullptr;
    int* d_one = nullptr;      // constant 1 (active flag of the unbatched form)
    int2* d_tasks = nullptr;   // (0, leaf) per sweep wavefront
    int2* d_ntasks = nullptr;  // (0, node or -1) per node wavefront
    int4* d_ninfo = nullptr;   // first child, children, y offset, parent per node wavefront
    int n_ntasks = 0;
    unsigned long long* d_res = nullptr;
    double* d_stash_z = nullptr;
    double* d_stash_e = nullptr;
    DevSet<double> s64;
    DevSet<float> s32;
    int cur = SPOCK_FP64;      // precision holding the current iterate
    unsigned long long* h_res = nullptr;  // pinned readback: res[2]
    bool have_ref = false;
    double xi_ref[2] = {0, 0};
    bool solved = false;
    double t_setup = 0;        // seconds spock_problem_create took
    int device = 0;            // HIP device current at create
    SmWork sm;                 // SuperMann vectors (method SPOCK_SUPERMANN)
};

template <typename real>
static DevSet<real>& set_of(spock_problem* p);
template <>
inline DevSet<double>& set_of<double>(spock_problem* p) { return p->s64; }
template <>
inline DevSet<float>& set_of<float>(spock_problem* p) { return p->s32; }

// handle operations used by the batched and served forms
template <typename real>
int32_t step(spock_problem* p, int check);
int32_t read_res(spock_problem* p, double* xi1, double* xi2);
int32_t move_iterate(spock_problem* p, int to);
int32_t zero_iterate(spock_problem* p);
int32_t set_x0_device(spock_problem* p, const double* x0, bool check_feasible);
double now_s();
// The residual maxima from kResSlots pairs of float64 bit patterns (the
// unsigned order of non-negative doubles, with a NaN above +inf).
inline void res_reduce(const unsigned long long* h, double* x1, double* x2) {
    unsigned long long a = 0, b = 0;
    for (int s = 0; s < spk::kResSlots; ++s) {
        a = std::max(a, h[2 * s]);
        b = std::max(b, h[2 * s + 1]);
    }
    std::memcpy(x1, &a, 8);
    std::memcpy(x2, &b, 8);
}

// rel_res of Sec. 5.3 from the two residual maxima: NaN when either is NaN
// (std::max would return the other operand and hide it).
inline double rel_of(double x1, double x2, double scale) {
    if (x1 != x1 || x2 != x2) return NAN;
    return std::max(x1, x2) / scale;
}
int32_t normalize_parity(spock_problem* p);
int32_t ensure_ref(spock_problem* p, bool warm, long long* taken, double* x1, double* x2);
// SuperMann iteration (spock_supermann.cpp) from the float64 iterate in copy
// 0, whose CP step (copy 1, residual slots) has been taken; fills info.
int32_t supermann_iterate(spock_problem* p, long long budget, spock_info* info);

// Batched form (spock_batch.cpp).
struct spock_batch {
    std::vector<spock_problem*> probs;
    int n = 0;
    spock_settings set{};
    hipStream_t stream = nullptr;
    void* base = nullptr;
    size_t bytes = 0;
    ProbDev<double>* d64 = nullptr;
    ProbDev<float>* d32 = nullptr;
    int2* tasks = nullptr;
    int n_tasks = 0;
    int2* ntasks = nullptr;
    int4* ninfo = nullptr;
    int n_ntasks = 0;
    int* active = nullptr;
    unsigned long long* res = nullptr;
    spk::LaunchCfg cfg64{}, cfg32{};
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // [0] float64, [1] float32
    int graph_steps[2] = {0, 0};
    unsigned long long* h_res = nullptr;  // pinned: 2n residual slots
    std::vector<int> h_active;
    double bytes_k[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};  // algorithmic bytes per launch, [fp64 / fp32]
};

// State of one problem inside a batched iteration.
struct Member {
    bool live = false;  // iterating in the current phase
    long long iters = 0, iters32 = 0;
    double rel = INFINITY, x1 = INFINITY, x2 = INFINITY;
    double best = INFINITY;
    int no_gain = 0, checks = 0;
    int32_t status = SPOCK_E_NOT_CONVERGED;
    int refined = 0;
};

template <typename real>
int32_t batch_tick(spock_batch* b, std::vector<Member>& m, bool stall_exit);

// Launch configuration of one problem in one precision with node workgroups
// of `node_wg` threads (the tasks are the problem's own).
template <typename real>
spk::LaunchCfg make_cfg(const spock_problem* p, int node_wg);
// Dynamic LDS bytes of a node workgroup of `node_wg` threads for this problem.
int node_lds_bytes(const spock_problem* p, int node_wg, int real_bytes);
// Smallest register tile class that holds a product of `need` rows per lane.
int tile_class(int need);
// Algorithmic bytes of the four launches of one step (prep, bsweep, fsweep,
// dual): every matrix and vector entry the step must read or write, once.
void step_bytes_of(const spock_problem* p, int real_bytes, double out[4]);
