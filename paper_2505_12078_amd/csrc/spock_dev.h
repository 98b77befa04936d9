// Device-side description of one scenario-tree problem, shared by the host
// set-up code and the gfx950 kernels.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spk {

// Threads per workgroup of the sweep kernels (a launch parameter: 64, 128,
// 256 or 512, picked per problem or batch); the default is four wave64s.
constexpr int kDefaultWG = 256;
// Longest root-to-leaf path a forward task may walk (stages + 1).
constexpr int kMaxDepth = 512;

// One problem in one precision.  Every pointer is a device address inside the
// problem's workspace.  Node j >= 1 owns the edge (anc(j), j).
template <typename real>
struct ProbDev {
    // sizes
    int n, n_nl, N;          // nodes, non-leaf nodes, horizon
    int nx, nu, m;           // m = nx + nu
    int nc, ncN, nbox;       // constraint rows at non-leaf / leaf nodes, nbox = nx + nu
    int has_ball, has_ballN, affine, max_ch;
    real alpha, ball_r, ballN_r;

    // tree (breadth-first numbering, children contiguous)
    const int* parent;
    const int* first_child;
    const int* n_ch;
    const int* y_off;        // start of y^i inside the y block, per non-leaf node
    const int* path;         // per leaf l: node at each stage 0..N on the root-to-leaf path
    const int* top_owned;    // per leaf l: first stage whose path node has l as leftmost leaf

    // Offline factors (Alg. 1, reduced online form):
    //   M[j]  = [Abar^j | B^j]  (nx x m, row-major), node j >= 1
    //   KR[i] = [K^i | R~^i^-1] (nu x m, row-major), non-leaf node i
    const real* M;
    long long M_stride;
    const real* KR;
    long long KR_stride;
    const real* c;           // affine term c^j (nx per node) or null
    const real* Pc;          // P^j c^j (nx per node) or null

    // diagonal data in the scaled space (Sec. 5.4)
    const real* qh;          // Q^1/2 S_x^-1, nx
    const real* rh;          // R^1/2 S_u^-1, nu
    const real* qnh;         // Q_N^1/2 S_xN^-1, nx
    const real* gx;          // constraint rows on x, u, ball rows on x (non-leaf)
    const real* gu;
    const real* gb;
    const real* gxN;         // leaf rows on x and ball rows on x
    const real* gbN;
    const real* lo;          // box bounds of the nbox box rows (non-leaf)
    const real* hi;
    const real* loN;         // leaf box bounds, nx
    const real* hiN;
    const real* prob;        // conditional probability per node
    const real* gamma;       // AV@R parameter per non-leaf node
    const real* x0;          // scaled initial state

    // iterates, two copies each; a step reads copy `par` and writes `par ^ 1`
    real* z[2];
    real* eta[2];
    long long z_x, z_u, z_y, z_tau, z_s;
    long long e_y, e_s, e_c, e_soc, e_cN, e_socN;
    long long nz, neta;

    // scratch
    real* d;                 // d^i of Alg. 2, nu per non-leaf node
    real* e;                 // backward message [Abar|B]^T h of node j, m per node
    int* cnt;                // backward arrival counters, per node
    int* flag;               // forward claim/done flags, per node
    int* err;                // device wait timeout
    const int* active;       // 0: this problem sits out the launch (batched form)
    unsigned long long* res; // |xi1|_inf, |xi2|_inf as float64 bit patterns
};

// Children whose per-child inputs are staged in LDS; a wider node reads them
// from global memory directly (same contiguous layout).
constexpr int kStageKids = 16;

// Elements of one wavefront's staging array for a dual block in the forward sweep.
__host__ __device__ inline int blk_elems(int nx, int nu, int /*max_ch*/) {
    const int m = nx + nu;
    int b = 2 * nx + nu;
    if (m + 2 > b) b = m + 2;
    return b;
}

// Elements of the LDS area that stages one node's vector inputs.
__host__ __device__ inline int stage_elems(int nx, int nu, int nc, int max_ch) {
    const int m = nx + nu;
    const int kc = max_ch < kStageKids ? max_ch : kStageKids;
    return 3 * nx + 2 * nu + nc + kc * (2 * m + nx + 12) + 16;
}

// Number of `real` elements of dynamic LDS a sweep workgroup of `wg` threads
// needs (the larger of the backward and the forward partitions).
__host__ __device__ inline int lds_elems(int nx, int nu, int max_ch, int wg) {
    const int m = nx + nu;
    const int nc = m + nx;  // the larger constraint block (with a ball)
    const int waves = wg / 64;
    const int common = wg + 10 * nx + 4 * nu + stage_elems(nx, nu, nc, max_ch);
    const int bwd = common + 2 * m + nx + 2 * nu + max_ch;
    const int fwd = common + m + nx + nu + waves * (nx + nu) + 2 * waves * blk_elems(nx, nu, max_ch);
    return (bwd > fwd ? bwd : fwd) + 8;
}

}  // namespace spk
