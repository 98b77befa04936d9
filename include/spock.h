/*
 * spock.h -- C ABI of the MI355X (gfx950) library for the Chambolle-Pock (CP)
 * step of SPOCK on scenario trees (arXiv:2505.12078).
 *
 * The library solves the risk-averse optimal control problem (RAOCP) of the
 * paper's problem-statement section (Sec. 3): linear dynamics on a scenario
 * tree, box and Euclidean-ball constraints, quadratic stage and terminal
 * costs, nested AV@R risk.  It iterates the CP operator T of Sec. 4.1 on the
 * conic reformulation of Sec. 4.2-4.5:
 *   z+   = prox_{alpha f}(z - alpha L* eta)       (Alg. 2 sweep + S2 + s0 shift)
 *   eta+ = prox_{alpha g*}(eta + alpha L(2z+ - z)) (S3 cone projections, Moreau)
 * with the offline factorisation of Alg. 1 done once per problem in FP64.
 *
 * Conventions for every entry point:
 *  - Every function returns int32_t status: SPOCK_OK (0) or a negative code.
 *    The message of the last failure on the calling thread is returned by
 *    spock_last_error().  No C++ exception crosses this boundary.
 *  - All pointers named in a description or argument are HOST pointers owned
 *    by the caller, unless the name says "device".  The library copies what it
 *    needs before returning; it keeps no pointer to caller memory.
 *  - Arrays are dense, row-major, float64, in node order.  Nodes are numbered
 *    stage by stage (breadth first): parent[j] < j, children of a node are
 *    consecutive, all non-leaf nodes precede all leaves, every leaf sits at
 *    the last stage N, and 1 <= N <= 511 (at most 512 stages); a description
 *    that breaks any of these is rejected with SPOCK_E_INVALID.
 *  - One problem handle may be used by one host thread at a time.
 *
 * Canonical iterate layout (scaled variables, the space the CP method runs
 * in; used by spock_get_iterate, spock_set_iterate and the operator hooks):
 *   z   = [ s0 | x (n*nx) | u (n_nl*nu) | y (per non-leaf i: 2*n_ch(i)+1)
 *         | tau (nodes 1..n-1) | s (nodes 1..n-1) ]
 *   eta = [ eta_y (as y) | eta_s (n_nl) | eta_c (n_nl*nc) | eta_soc ((n-1)*(nx+nu+2))
 *         | eta_cN (n_leaf*ncN) | eta_socN (n_leaf*(nx+2)) ]
 * with nc = nx+nu (+nx with a ball) and ncN = nx (+nx with a ball); this is
 * the operator L of Sec. 4.4 block by block.
 */
#ifndef SPOCK_MI355X_H
#define SPOCK_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SPOCK_OK 0
#define SPOCK_E_INVALID (-1)         /* malformed tree, data or argument */
#define SPOCK_E_INFEASIBLE_X0 (-2)   /* x0 outside the root constraint set */
#define SPOCK_E_NOT_CONVERGED (-3)   /* max_iters reached; info is filled */
#define SPOCK_E_DIVERGED (-4)        /* non-finite residual */
#define SPOCK_E_HIP (-5)             /* HIP runtime failure */
#define SPOCK_E_CAPACITY (-6)        /* a request larger than the whole budget */
#define SPOCK_E_NOMEM (-7)           /* workspace too small / allocation failed */

/* outer method */
#define SPOCK_CP 0         /* plain Chambolle-Pock iterations v <- T(v) (Sec. 4.1) */
#define SPOCK_SUPERMANN 1  /* SuperMann over T with Anderson directions (Sec. 5.2) */

/* precision of the iteration */
#define SPOCK_FP64 0   /* every step in float64 */
#define SPOCK_MIXED 1  /* float32 steps; float64 final check and refinement */
#define SPOCK_FP32 2   /* float32 steps only (hooks and benchmarks) */

/*
 * Problem data (Sec. 3.1-3.4).  x^j = A^j x^i + B^j u^i + c^j for j with
 * parent i; stage cost of the edge into j: x^iT Q^j x^i + u^iT R^j u^i
 * (+ q^jT x^i + r^jT u^i); leaf cost x^jT QN^j x^j (+ qN^jT x^j); the cost
 * diagonals are shared (Q_diag, R_diag, QN_diag) or given per edge / leaf
 * (Q_edge, R_edge, QN_leaf); constraints lo <= (x, u) <= hi and ||x|| <= x_ball at
 * non-leaf nodes, xN_lo <= x <= xN_hi and ||x|| <= xN_ball at leaves;
 * AV@R_gamma[i] over the children of non-leaf node i with the conditional
 * probabilities cond_prob (AV@R_1 = expectation, AV@R_0 = max).
 */
typedef struct spock_problem_desc {
    int32_t n_nodes;          /* n >= 2 */
    const int32_t* parent;    /* [n], parent[0] = -1 */
    const double* cond_prob;  /* [n], > 0, children of each node sum to 1 */
    int32_t nx, nu;           /* 1 <= nx, nu <= 256 */
    const double* A;          /* [n][nx][nx]; entry 0 ignored */
    const double* B;          /* [n][nx][nu]; entry 0 ignored */
    const double* c;          /* [n][nx] or NULL (= 0) */
    const double* Q_diag;     /* [nx] > 0, shared by all edges (or see Q_edge) */
    const double* R_diag;     /* [nu] >= 0 (or see R_edge; zero entries: see r) */
    const double* QN_diag;    /* [nx] > 0, shared by all leaves (or see QN_leaf) */
    const double* x_lo;       /* [nx], non-leaf state box (may be +-inf) */
    const double* x_hi;
    const double* u_lo;       /* [nu] */
    const double* u_hi;
    const double* xN_lo;      /* [nx], leaf state box */
    const double* xN_hi;
    double x_ball;            /* radius at non-leaf nodes; <= 0: no ball */
    double xN_ball;           /* radius at leaves; <= 0: no ball */
    const double* gamma;      /* [n_nl] in [0, 1] */
    /* Optional linear cost terms (Prop. 1 with q != 0, Sec. 4.2), each NULL
     * for zero: the edge into node j adds q[j]^T x^i + r[j]^T u^i (i its
     * parent), leaf j adds qN[j]^T x^j.  Row-major [n][nx], [n][nu], [n][nx];
     * row 0 (and qN's non-leaf rows) ignored.  Where a diagonal R has a zero
     * entry (an input without quadratic cost, e.g. the slacks of Prop. 2's l1
     * penalty), r's entry lies in ker R and enters the edge's two tau rows of
     * L as -(r_k u_k) / 2 each (Prop. 1 with Q singular) instead of the
     * translation. */
    const double* q;
    const double* r;
    const double* qN;
    /* Optional per-edge stage costs and per-leaf terminal costs (the paper's
     * Q^j, R^j of each event and Q_N^j of each scenario, Sec. 3.1): diagonals
     * [n][nx], [n][nu] (row j: the edge into node j; row 0 ignored) and
     * [n][nx] (leaf rows).  A non-NULL array replaces Q_diag, R_diag or
     * QN_diag, which may then be NULL; every used entry must be > 0 (R's:
     * >= 0). */
    const double* Q_edge;
    const double* R_edge;
    const double* QN_leaf;
    /* Optional dense per-edge / per-leaf cost matrices (symmetric positive
     * definite; Prop. 1 with S = I): [n][nx][nx], [n][nu][nu] (matrix j: the
     * edge into node j; matrix 0 ignored) and [n][nx][nx] (leaf matrices).  A
     * non-NULL array replaces the corresponding diagonal form.  The SOC block
     * of an edge then carries Q^1/2 x (the symmetric square root). */
    const double* Q_dense;
    const double* R_dense;
    const double* QN_dense;
    /* Optional general constraints (Sec. 3.1, the set C a box): at every
     * non-leaf node Gamma_x x + Gamma_u u in [con_lo, con_hi], Gamma the
     * n_con x (nx + nu) row-major matrix [Gamma_x | Gamma_u]; at every leaf
     * Gamma_N x in [conN_lo, conN_hi], GammaN n_conN x nx.  Bounds may be
     * infinite (one-sided rows), never NaN, and lo <= hi.  A non-NULL Gamma
     * replaces x_lo, x_hi, u_lo, u_hi and x_ball at non-leaf nodes (the root
     * x0 is then not checked against them); a non-NULL GammaN replaces xN_lo,
     * xN_hi and xN_ball.  1 <= n_con, n_conN <= 512. */
    int32_t n_con;
    const double* Gamma;
    const double* con_lo;
    const double* con_hi;
    int32_t n_conN;
    const double* GammaN;
    const double* conN_lo;
    const double* conN_hi;
    /* Optional general coherent risks (Sec. 3.3; K a product of R_+, {0}
     * and second-order cones, given row by row): the risk at non-leaf node i
     * (k_i children) is max{mu^T Z : b - E mu - F nu in K} over the
     * children's costs Z, with y^i of risk_ny[i] entries (the
     * rows of E, F, b) and nu of risk_nnu[i] (the columns of F).  Concatenated
     * in node order: risk_E (ny x k_i, row-major), risk_F (ny x nnu), risk_b
     * (ny), risk_cone (ny codes: 0 for R_+, 1 for {0}, 2 for the head row t
     * of a second-order cone block {(t, w): ||w|| <= t} and 3 for each of
     * its rows of w, which follow the head).  A non-NULL risk_ny
     * replaces AV@R (gamma is then not read); 1 <= ny <= 128,
     * k_i + nnu <= 64, and [E^T -I -I; F^T 0 0] must have full row rank. */
    const int32_t* risk_ny;
    const int32_t* risk_nnu;
    const double* risk_E;
    const double* risk_F;
    const double* risk_b;
    const int32_t* risk_cone;
} spock_problem_desc;

typedef struct spock_settings {
    double alpha;          /* CP step; 0 = automatic 0.99/||L|| (exact block norm) */
    double eps;            /* tolerance on rel_res (default 1e-6) */
    int64_t max_iters;     /* CP steps (default 100000) */
    int32_t precision;     /* SPOCK_FP64 / SPOCK_MIXED / SPOCK_FP32 */
    int32_t precondition;  /* 1 = diagonal scaling of Sec. 5.4 (default), 0 = off */
    int32_t check_every;   /* steps between residual checks, even (default 20) */
    int32_t use_graph;     /* 1 = replay check_every steps as one hipGraph (default) */
    int32_t method;        /* SPOCK_CP (default) or SPOCK_SUPERMANN; fixed at create time.
                              SuperMann runs float64 iterations (precision SPOCK_FP64), checks
                              the residuals at every iteration, and is available to
                              spock_solve only (not to the batched and served forms) */
    int32_t aa_memory;     /* Anderson memory m of SuperMann, 1..8 (default 3) */
} spock_settings;

/*
 * Per-solve report.  rel_res = max(|xi1|_inf, |xi2|_inf) / max(1, |xi1_ref|_inf,
 * |xi2_ref|_inf) with the residuals xi1, xi2 of Sec. 5.3 and the reference
 * residuals of the first CP step from zero (kept with the handle).  With
 * SPOCK_SUPERMANN, iters counts SuperMann iterations and the residuals are
 * those of the CP step from the returned iterate.
 */
typedef struct spock_info {
    int64_t iters;          /* CP steps taken in this solve */
    int64_t iters_fp32;     /* of which in float32 */
    double rel_res, xi1_inf, xi2_inf;
    double s0;              /* objective value s^0 (= V* at convergence) */
    double t_setup_s;       /* wall time spock_problem_create took for this handle
                               (validation, scaling, Alg. 1, exact ||L||, upload) */
    double t_solve_s;       /* wall time of the solve call */
    int32_t status;         /* the same code the call returned */
    int32_t precision_used; /* precision of the final accepted step */
    int32_t refined;        /* 1 if float64 steps had to follow float32 ones */
    int64_t n_T;            /* applications of T (plain CP: iters) */
    int64_t n_K0, n_K1, n_K2;  /* SuperMann: educated, safeguarded and generalized-KM steps */
} spock_info;

typedef struct spock_sizes {
    int64_t nz, neta;       /* canonical iterate lengths */
    int32_t n, n_nl, n_leaf, N, nx, nu, nc, ncN, max_children;
    double alpha, L_norm;
    size_t device_bytes;    /* device memory held by the handle */
} spock_sizes;

typedef struct spock_problem spock_problem;

/* Message of the last failed call on this thread ("" if none). */
const char* spock_last_error(void);

/* Defaults listed in spock_settings. */
int32_t spock_default_settings(spock_settings* out);

/* Device bytes spock_problem_create would need for this problem (pure; no
 * device access).  Used for admission by footprint. */
int32_t spock_problem_footprint(const spock_problem_desc* desc, const spock_settings* s,
                                size_t* device_bytes);

/*
 * Validate the data, apply the scaling of Sec. 5.4, run Alg. 1 (offline S1
 * factorisation, Sec. 5.1) in float64 on the host, compute the exact ||L||
 * (Sec. 4.4) and upload everything to the current HIP device.
 * device_workspace: device pointer of >= spock_problem_footprint bytes that
 * the caller keeps alive until destroy, or NULL to let the library allocate.
 * stream: hipStream_t to launch on, or NULL for the default stream.
 * Errors: SPOCK_E_INVALID, SPOCK_E_NOMEM, SPOCK_E_HIP.
 */
int32_t spock_problem_create(const spock_problem_desc* desc, const spock_settings* s,
                             void* device_workspace, size_t workspace_bytes, void* stream,
                             spock_problem** out);

int32_t spock_problem_destroy(spock_problem* p);

int32_t spock_problem_sizes(const spock_problem* p, spock_sizes* out);

/* Replace the settings used by later solves (alpha changes need a new handle). */
int32_t spock_set_settings(spock_problem* p, const spock_settings* s);

/*
 * Solve from initial state x0 ([nx], unscaled).  warm_start = 0 starts from
 * z = 0, eta = 0; 1 starts from the iterate left by the previous solve (or
 * spock_set_iterate).  Stops when rel_res <= eps (checked every check_every
 * steps) or after max_iters steps.
 * Errors: SPOCK_E_INFEASIBLE_X0 (x0 outside the root box/ball),
 * SPOCK_E_NOT_CONVERGED, SPOCK_E_DIVERGED, SPOCK_E_HIP.  info may be NULL.
 */
int32_t spock_solve(spock_problem* p, const double* x0, int32_t warm_start, spock_info* info);

/* Unscaled solution of the last solve: x [n][nx], u [n_nl][nu], s0 (each may be NULL). */
int32_t spock_get_solution(const spock_problem* p, double* x, double* u, double* s0);

/* Current iterate (float64 copy) in the canonical layout, scaled space. */
int32_t spock_get_iterate(const spock_problem* p, double* z, double* eta);
int32_t spock_set_iterate(spock_problem* p, const double* z, const double* eta);

/* Set the initial state used by the operator hooks below ([nx], unscaled). */
int32_t spock_set_x0(spock_problem* p, const double* x0);

/*
 * Operator hooks on caller iterates (canonical layout, scaled space, host
 * arrays).  precision selects the float64 or float32 kernels.
 *  spock_apply_T: (z_out, eta_out) = T(z, eta) (Sec. 4.1); with eta = 0 the z
 *    part is prox_{alpha f}(z): the S1 projection of Alg. 2 on (x, u), the S2
 *    projection on (y, tau, s) and s0 - alpha.  xi (nullable, [2]) receives
 *    |xi1|_inf and |xi2|_inf of this step (Sec. 5.3).
 *  spock_apply_L: eta_out = L z (Sec. 4.4).
 *  spock_apply_Lt: z_out = L* eta.
 *  spock_prox_gconj: eta_out = w - alpha proj_S3(w / alpha) (Moreau).
 */
int32_t spock_apply_T(spock_problem* p, const double* z, const double* eta, double* z_out,
                      double* eta_out, int32_t precision, double* xi);
int32_t spock_apply_L(spock_problem* p, const double* z, double* eta_out, int32_t precision);

/*
 * The two parts of prox_{alpha f} (Sec. 4.5) on their own, host arrays, scaled
 * space, float64 or float32 kernels as precision says.
 *  spock_project_S1: Euclidean projection of (xbar, ubar) onto the dynamics
 *    set S1 of Sec. 4.3 with x^0 fixed to the handle's initial state
 *    (spock_set_x0), computed by the online sweep of Alg. 2 (Sec. 5.1).
 *    xbar [n][nx] (row 0 is ignored: x^0 is fixed), ubar [n_nl][nu];
 *    x_out [n][nx], u_out [n_nl][nu].
 *  spock_project_S2: orthogonal projection of every non-leaf node's block
 *    (y^i, tau^[i], s^[i]) onto the kernel of [E^T -I -I; F^T 0 0] of
 *    Sec. 4.3 (E of AV@R, Sec. 3.3, and no F unless general risks are given).
 *    y in the canonical y layout (per non-leaf node 2 n_ch + 1 entries for
 *    AV@R, risk_ny[i] for a general risk), tau and s per node 1..n-1; the
 *    outputs have the same shapes.
 * Errors: SPOCK_E_INVALID (null pointer, bad precision), SPOCK_E_HIP.
 */
int32_t spock_project_S1(spock_problem* p, const double* xbar, const double* ubar, double* x_out, double* u_out,
                         int32_t precision);
int32_t spock_project_S2(spock_problem* p, const double* y, const double* tau, const double* s, double* y_out,
                         double* tau_out, double* s_out, int32_t precision);
int32_t spock_apply_Lt(spock_problem* p, const double* eta, double* z_out, int32_t precision);
int32_t spock_prox_gconj(spock_problem* p, const double* w, double* eta_out, int32_t precision);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one CP step
 * T, as spock_apply_T computes it, on caller DEVICE iterates, with every
 * scratch buffer of the step's kernels (the step's descriptor, d, the backward
 * messages, h0, ubar, the arrival counters, the residual slots) in a static
 * device array of the library of SPOCK_NOALLOC_SCRATCH_BYTES per GPU, which
 * each GPU the library runs on holds until the process ends.  The call makes
 * no device or host allocation.
 *  z, eta: device arrays [nz], [neta] (canonical layout, scaled space) of
 *    float64 for precision SPOCK_FP64 or float32 for SPOCK_FP32; read only.
 *  z_out, eta_out: device arrays of the same type and sizes, distinct from
 *    the inputs and from each other; every entry is written.
 *  xi (host, nullable, [2]) receives |xi1|_inf and |xi2|_inf of the step.
 * The kernels run on the handle's stream with the handle's device current,
 * and the call waits for them.  Scratch need, 256-byte aligned regions:
 * descriptor + w (n_nl nu + n (nx + nu) + n nx + n_nl nu) + 4 n + 512 bytes,
 * w = 8 or 4; a problem that needs more fails with SPOCK_E_CAPACITY.  Every
 * call on one GPU shares that GPU's array and leaves its contents behind:
 * calls that overlap on one GPU (other streams or threads) race.
 * Errors: SPOCK_E_INVALID (null or aliased pointer, bad precision, another
 * device current), SPOCK_E_CAPACITY, SPOCK_E_HIP.
 */
#define SPOCK_NOALLOC_SCRATCH_BYTES (16u << 20)
int32_t spock_apply_T_noalloc(spock_problem* p, const void* z, const void* eta, void* z_out, void* eta_out,
                              int32_t precision, double* xi);

/*
 * Timing hook: run `steps` CP steps from the current device iterate in the
 * given precision (no residual checks, no readback) and report mean device
 * durations measured with HIP events on the handle's stream around every
 * launch.  A step is four launches: prep (node-parallel: z - alpha L* eta, the
 * S2 projection and the children-independent part of Alg. 2's backward
 * recursion, Sec. 4.1-4.4), bsweep (leaves -> root: the dependent part of the
 * backward recursion), fsweep (root -> leaves: x^j = Abar^j x^i + B^j d^i + c^j)
 * and dual (node-parallel: u = K x + d and prox_{alpha g*} with the S3
 * projections, Sec. 4.1, 5.3).  spock_time_steps reports ms_backward =
 * prep + bsweep and ms_forward = fsweep + dual (each nullable);
 * spock_time_kernels fills ms_kernels[4] in launch order.
 */
int32_t spock_time_steps(spock_problem* p, int32_t precision, int32_t steps, double* ms_total,
                         double* ms_backward, double* ms_forward);
int32_t spock_time_kernels(spock_problem* p, int32_t precision, int32_t steps, double* ms_total,
                           double* ms_kernels);

/* Launch `steps` CP steps from the current device iterate in the given
 * precision (SPOCK_FP64 or SPOCK_FP32), without residual checks or readback;
 * sync = 1 waits for them to finish.  For throughput measurement. */
int32_t spock_run_steps(spock_problem* p, int32_t precision, int32_t steps, int32_t sync);

/* Workgroup size (64, 128, 256 or 512 threads, i.e. 1-8 nodes per workgroup)
 * of the node-parallel kernels of one precision; picked by the autotuner
 * (default 256; lowered automatically when the LDS of a larger workgroup would
 * exceed 64 KiB).  Results do not depend on it. */
int32_t spock_set_launch(spock_problem* p, int32_t precision, int32_t workgroup);
int32_t spock_get_launch(const spock_problem* p, int32_t precision, int32_t* workgroup);

/* Bytes one CP step must move at minimum (every factor matrix and iterate
 * entry a launch reads or writes, once) in the given precision; for roofline
 * reporting.  spock_step_bytes: prep + bsweep and fsweep + dual;
 * spock_kernel_bytes: bytes[4] per launch, in launch order. */
int32_t spock_step_bytes(const spock_problem* p, int32_t precision, double* bytes_backward,
                         double* bytes_forward);
int32_t spock_kernel_bytes(const spock_problem* p, int32_t precision, double* bytes);

/*
 * Batched form: one CP step of the batch is the same four launches over every
 * member tree (uneven trees of any shapes and sizes share each launch; one
 * sweep wavefront per leaf and one node wavefront per node of every member).
 *
 * spock_batch_create groups problems created on the current device.  The
 * problems stay owned by the caller, must outlive the batch, and must not be
 * used on their own while a batch call runs.  s gives eps, max_iters,
 * precision (SPOCK_FP64 / SPOCK_MIXED / SPOCK_FP32), check_every, use_graph for
 * every member (alpha and precondition are the members' own).
 * Errors: SPOCK_E_INVALID, SPOCK_E_NOMEM, SPOCK_E_HIP.
 */
typedef struct spock_batch spock_batch;
int32_t spock_batch_create(spock_problem* const* probs, int32_t n, const spock_settings* s, spock_batch** out);
int32_t spock_batch_destroy(spock_batch* b);
int32_t spock_batch_size(const spock_batch* b, int32_t* n_problems, int32_t* n_tasks, size_t* device_bytes);

/*
 * Solve every member from x0s[k] (host [nx_k], unscaled); warm (nullable)
 * selects warm starts per member.  Members that converge leave the launch
 * (their tasks exit at once) while the others continue; each member's result is
 * in infos[k] (status: SPOCK_OK, SPOCK_E_NOT_CONVERGED, SPOCK_E_DIVERGED or
 * SPOCK_E_INFEASIBLE_X0 for that member only).  Returns SPOCK_OK unless the
 * batch itself failed (SPOCK_E_HIP).  Solutions are read per member with
 * spock_get_solution.
 */
int32_t spock_batch_solve(spock_batch* b, const double* const* x0s, const int32_t* warm, spock_info* infos);

/* Measurement: `steps` (even) batched steps of every member; mean durations
 * with HIP events (backward = prep + bsweep, forward = fsweep + dual, or the
 * four launches in ms_kernels[4]); algorithmic bytes of one batched step. */
int32_t spock_batch_run_steps(spock_batch* b, int32_t precision, int32_t steps, int32_t sync);
int32_t spock_batch_time_steps(spock_batch* b, int32_t precision, int32_t steps, double* ms_total,
                               double* ms_backward, double* ms_forward);
int32_t spock_batch_time_kernels(spock_batch* b, int32_t precision, int32_t steps, double* ms_total,
                                 double* ms_kernels);
int32_t spock_batch_step_bytes(const spock_batch* b, int32_t precision, double* bytes_backward,
                               double* bytes_forward);
int32_t spock_batch_kernel_bytes(const spock_batch* b, int32_t precision, double* bytes);
/* Workgroup size of the batch's node-parallel kernels for one precision (autotuner). */
int32_t spock_batch_set_launch(spock_batch* b, int32_t precision, int32_t workgroup);

/*
 * Served form: continuous batching of MPC requests.
 *
 * A server owns a worker thread that drives the current HIP device.  Trees
 * are registered once (the description is copied; its device footprint is
 * computed without touching the device).  Requests (tree, x0) may be submitted
 * from any thread at any time; a request starts as soon as its tree has no
 * other request in flight and the tree is resident or fits in hbm_budget
 * bytes (idle trees are evicted least recently used first).  A resident tree
 * keeps its offline factors and its last iterate: its next request warm-starts
 * from it.  All requests in flight advance together, one batched chunk of
 * check_every CP steps per tick; requests that arrive in between join at the
 * next tick.  Each request's result equals the result of the same sequence of
 * spock_solve calls on that tree alone.
 */
typedef struct spock_server spock_server;

typedef struct spock_result {
    uint64_t req_id;
    int64_t tree_id;
    int32_t status;          /* SPOCK_OK, SPOCK_E_NOT_CONVERGED, SPOCK_E_DIVERGED, SPOCK_E_INFEASIBLE_X0 */
    int32_t warm;            /* 1: started from the tree's resident iterate */
    spock_info info;         /* iters, residuals, s0 (t_solve_s = admission to completion) */
    double t_submit, t_admit, t_done;  /* spock_now() clock, seconds */
} spock_result;

typedef struct spock_server_stats {
    uint64_t submitted, completed, created, evicted, ticks;
    size_t resident_bytes, budget_bytes, pending, in_flight;
} spock_server_stats;

/* Errors: SPOCK_E_INVALID. */
int32_t spock_server_create(size_t hbm_budget, const spock_settings* s, spock_server** out);
/* SPOCK_E_CAPACITY if the tree alone exceeds the budget; SPOCK_E_INVALID for bad data. */
int32_t spock_server_add_tree(spock_server* srv, const spock_problem_desc* desc, int64_t* tree_id);
/* Thread-safe; x0 is copied ([nx] of the tree, unscaled). */
int32_t spock_server_submit(spock_server* srv, int64_t tree_id, const double* x0, uint64_t req_id);
/* Thread-safe, non-blocking: moves up to max finished results to out. */
int32_t spock_server_poll(spock_server* srv, spock_result* out, int32_t max, int32_t* n_out);
/* Block until nothing is pending or in flight (SPOCK_E_NOT_CONVERGED on timeout). */
int32_t spock_server_wait_idle(spock_server* srv, double timeout_s);
int32_t spock_server_get_stats(spock_server* srv, spock_server_stats* out);
/* Unscaled solution of the tree's last request (tree idle and resident). */
int32_t spock_server_solution(spock_server* srv, int64_t tree_id, double* x, double* u, double* s0);
/* Stops the worker and frees every resident tree. */
int32_t spock_server_destroy(spock_server* srv);
/* The monotonic clock of the t_* fields. */
double spock_now(void);

#ifdef __cplusplus
}
#endif

#endif /* SPOCK_MI355X_H */
