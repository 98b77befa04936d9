// Device-side description of one scenario-tree problem, shared by the host
// set-up code and the gfx950 kernels.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spk {

// Threads per workgroup of the node-parallel kernels (a launch parameter: 64,
// 128, 256 or 512, i.e. one to eight nodes per workgroup, one wavefront each).
constexpr int kDefaultWG = 256;
constexpr int kMaxNodeWaves = 8;
// Longest root-to-leaf path (stages + 1).
constexpr int kMaxDepth = 512;

// One problem in one precision.  Every pointer is a device address inside the
// problem's workspace.  Node j >= 1 owns the edge (anc(j), j).
template <typename real>
struct ProbDev {
    // sizes
    int n, n_nl, N;          // nodes, non-leaf nodes, horizon
    int nx, nu, m;           // m = nx + nu
    int nc, ncN, nbox;       // constraint rows at non-leaf / leaf nodes; box rows among the nc (nx + nu,
                             // or nc with general constraints; the rest are ball rows)
    int nboxN;               // box rows among the ncN (nx, or ncN with general leaf constraints)
    int has_ball, has_ballN, affine, max_ch;
    int stage_kids;          // nodes with at most this many children stage their per-child inputs in LDS
    real alpha, ball_r, ballN_r;

    // tree (breadth-first numbering, children contiguous)
    const int* first_child;
    const int* n_ch;
    const int* y_off;        // start of y^i inside the y block, per non-leaf node
    const int4* path;        // per leaf l, stage 0..N of its root-to-leaf path: (node, children,
                             // first child, 0), children 0 at the leaf
    const int* top_owned;    // per leaf l: first stage whose path node has l as leftmost leaf
                             // (the forward sweep of l stores x from that stage on)

    // Offline factors (Alg. 1, reduced online form), each packed in the lane
    // order of the product that reads it (tile_pack):
    //   T1[i]  = K^i              read as (K^i)^T ubar          prep, non-leaf i
    //   T2M[j] = [Abar^j | B^j]   read as [Abar|B]^T h          bsweep, node j >= 1
    //   T2R[i] = R~^i^-1          (symmetric)                   bsweep, non-leaf i
    //   T3[j]  = [Abar^j | B^j]^T read as [Abar|B] [x; d]       fsweep, node j >= 1
    //   T4[i]  = (K^i)^T          read as K^i x                 dual, non-leaf i
    const real* T1;
    long long T1_stride;
    const real* T2M;
    long long T2M_stride;
    const real* T2R;
    long long T2R_stride;
    const real* T3;
    long long T3_stride;
    const real* T4;
    long long T4_stride;
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
    // translations a of Prop. 1 with linear cost terms: per edge j (m + 2,
    // at (j - 1) (m + 2)) and per leaf (nx + 2); null without linear terms,
    // then a = (0, ..., 0, 1/2, -1/2)
    const real* sa;
    const real* saN;
    const real* ck;  // tau-row coupling of the inputs per edge [n][nu] (null unless R is singular)
    // per-edge cost square roots (Q^j^1/2 S_x^-1 at j nx, R^j^1/2 S_u^-1 at
    // j nu, edge j = 1..n-1) and per-leaf terminal ones (at (j - n_nl) nx);
    // null when every edge shares qh, rh and every leaf qnh
    const real* qh_e;
    const real* rh_e;
    const real* qnh_l;
    // dense costs (null unless the costs are dense): the symmetric square
    // roots H = Q^j^1/2 (nx x nx at j nx^2), R^j^1/2 (nu x nu at j nu^2) per
    // edge and Q_N^j^1/2 per leaf (at (j - n_nl) nx^2); the cost rows of L are
    // then H (qh o x) (qh, rh, qnh hold S^-1) and those of L* qh o (H w)
    const real* Hq_e;
    const real* Hr_e;
    const real* HqN_l;
    // general constraints (null unless given): Gamma S^-1 / a row-major
    // (nc x m, Gt, read by L*) and transposed (m x nc, GtT, read by L); at the
    // leaves Gamma_N S_N^-1 / a_N (ncN x nx, GNt) and transposed (GNtT).  The
    // box bounds lo, hi (loN, hiN) then hold nc (ncN) rows.
    const real* Gt;
    const real* GtT;
    const real* GNt;
    const real* GNtT;
    // general coherent risks (null unless given): per non-leaf node i, y^i has
    // rny[i] entries and nu rnnu[i]; at rdata + roff[i]: E (ny x k, row-major),
    // F (ny x nnu), b (ny), cone codes (ny: 0 for R_+, 1 for {0}), and
    // M = (G G^T)^-1 ((k + nnu) x (k + nnu)) of G = [E^T -I -I; F^T 0 0]
    const long long* roff;
    const int* rny;
    const int* rnnu;
    const real* rdata;
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
    real* h0;                // -xbar - K^T ubar (+ P c): h of node j before its children's messages, nx
    real* ub;                // ubar of non-leaf node i, nu
    int* cnt;                // backward arrival counters, per node
    const int* active;       // 0: this problem sits out the launch (batched form)
    unsigned long long* res; // kResSlots pairs (|xi1|_inf, |xi2|_inf) as float64 bit patterns:
                             // a node wavefront records into the pair of its workgroup
                             // (mod kResSlots); the residuals are the maxima over the pairs
};

// Residual slot pairs per problem: spreading the atomic maxima of thousands of
// node wavefronts over many addresses keeps them from serializing on one.
constexpr int kResSlots = 32;

// Children whose per-child inputs are staged in LDS (at most; fewer when a
// node's blocks are wide, so that a wavefront's LDS stays within 64 KiB); a
// wider node reads them from global memory directly (same contiguous layout).
constexpr int kStageKids = 16;
// LDS scratch of one wavefront for cross-lane partial sums.
constexpr int kRed = 128;
// Vector entries per lane the forward sweep keeps in registers (nx, nu <= 64 kVecPL).
constexpr int kVecPL = 4;

__host__ __device__ inline int imax(int a, int b) { return a > b ? a : b; }
__host__ __device__ inline int round4(int a) { return (a + 3) & ~3; }

// Per-problem diagonal data staged once per node workgroup.
__host__ __device__ inline int consts_elems(int nx, int nu) { return round4(10 * nx + 4 * nu); }

// Largest dual block of a node (constraint block with a ball, an SOC block).
__host__ __device__ inline int blk_elems(int nx, int nu, int nc, int ncN) {
    return imax(imax(nc, nx + nu + 2), imax(ncN, nx + 2));
}

// Staged vector inputs of one node in the prep and dual kernels.
__host__ __device__ inline int node_stage_elems(int nx, int nu, int nc, int ncN, int max_ch) {
    const int m = nx + nu;
    const int kk = max_ch < kStageKids ? max_ch : kStageKids;
    const int prep = 2 * nx + nu + nc + kk * (m + 2) + 2 * (2 * kk + 1) + 1 + 3 * kk + kk * (nx + 2);
    const int dual = 2 * nx + 2 * nu + nc + kk * (m + 2) + 3 * (2 * kk + 1) + 3 + 3 * kk;
    const int leaf = 3 * nx + ncN + 4;
    return imax(imax(prep, dual), leaf);
}

// LDS elements of one wavefront of the prep / dual kernels:
//   prep: red | xbar (nx) | ubar (nu) | K^T ubar (nx) | stage
//   dual: red | u (nu) | L* d_eta on x (nx) and u (nu) | blk | dblk | stage
__host__ __device__ inline int node_head_elems(int nx, int nu, int nc, int ncN) {
    return round4(imax(2 * round4(nx) + round4(nu), 2 * nu + nx + 2 * blk_elems(nx, nu, nc, ncN)));
}
__host__ __device__ inline int node_wave_elems(int nx, int nu, int nc, int ncN, int max_ch) {
    return round4(kRed + node_head_elems(nx, nu, nc, ncN) + node_stage_elems(nx, nu, nc, ncN, max_ch));
}

// LDS bytes of the sweep kernels (one wavefront per workgroup): path node ids,
// child counts and first children (ints), then red | h / a | g / x | w | d.
// Every vector region holds at least kVecPad entries: the products read the
// full register class of v (zero past the vector's length).
constexpr int kVecPad = 80;
__host__ __device__ inline int sweep_vec(int n) { return round4(imax(n, kVecPad)); }
__host__ __device__ inline int sweep_int_bytes(int N) { return ((3 * (N + 1) * 4) + 15) & ~15; }
__host__ __device__ inline int sweep_elems(int nx, int nu) {
    const int m = nx + nu;
    return kRed + 2 * sweep_vec(m) + 2 * sweep_vec(nu);
}

// What one launch of a CP step needs besides the problem descriptors.
struct LaunchCfg {
    const int2* leaf_tasks;  // (problem, leaf) per sweep wavefront
    int n_leaf_tasks;
    const int2* node_tasks;  // (problem, node or -1) per node wavefront, kMaxNodeWaves-padded per problem
    const int4* node_info;   // per node task: first child, children, y offset, parent
    int n_node_tasks;
    int node_wg;             // threads per node workgroup (64, 128, 256, 512)
    int node_lds;            // dynamic LDS bytes of a node workgroup
    int wave_elems;          // LDS elements of one node wavefront
    int sweep_lds;           // dynamic LDS bytes of a sweep wavefront
    int cls[4];              // register tile class of prep, bsweep, fsweep, dual
    int dense;               // node kernel build: 0 plain, 1 dense costs, 2 the general formulation (max over problems)
};

// Packed tiles of the column-lane products out[o] = sum_k A[k][o] v[k]
// (K rows, O columns; the register forms below take O <= 128).  Block 1 holds columns 0..min(O,64)-1 with
// G1 = 64 / min(O,64) row groups, block 2 the columns from 64 on with
// G2 = 64 / (O - 64).  Lane l = g W + c of a block holds rows g, g + G, ... of
// column c; rows per lane are padded to the 16-byte vector width V, and the
// element of (row slot i, lane l) sits at ((i / V) * 64 + l) * V + i % V.
template <typename real>
__host__ __device__ constexpr int tile_vec() { return 16 / (int)sizeof(real); }
__host__ __device__ inline int tile_rows(int K, int G, int V) { return ((K + G - 1) / G + V - 1) / V * V; }
// Wider products (O > 128) continue the same way: block b holds the columns
// 64 b .. min(O, 64 (b + 1)) - 1, every block but the last with one row group.
__host__ __device__ inline int tile_blocks(int O) { return (O + 63) / 64; }
__host__ __device__ inline int tile_block_width(int O, int b) { return O - 64 * b < 64 ? O - 64 * b : 64; }
__host__ __device__ inline long long tile_elems(int K, int O, int V) {
    if (O < 1) return 0;
    long long e = 0;
    for (int b = 0; b < tile_blocks(O); ++b) e += (long long)tile_rows(K, 64 / tile_block_width(O, b), V) * 64;
    return e;
}

// Zero rows (of 64 lanes x V) after every packed tile array: a wavefront
// loads the full rows of its register class from every tile, so reads run up
// to (80 + 20) rows past the start of the last tile.
constexpr int kTilePadRows = 128;
template <typename real>
__host__ __device__ constexpr long long tile_pad_elems() { return (long long)kTilePadRows * 64 * tile_vec<real>(); }

// Register tile classes of the column-lane products (rows per lane); a
// product that does not fit its class runs from global memory instead.
// kWideClass: the launch's product fits no class; its kernels keep a minimal
// register tile and read every product from global memory with several row
// groups in flight.
constexpr int kTileClasses[4] = {16, 32, 64, 80};
constexpr int kWideClass = 8;

// Register rows a column-lane product needs: block 1 rows, and block 2 rows
// times 4 (block 2 has a quarter of the class).
__host__ __device__ inline int col_need(int K, int O, int V) {
    if (O > 128 || O < 1) return 1 << 20;
    const int W1 = O < 64 ? O : 64, G1 = 64 / W1;
    int need = tile_rows(K, G1, V);
    if (O > 64) {
        const int W2 = O - 64, G2 = 64 / W2;
        need = imax(need, 4 * tile_rows(K, G2, V));
    }
    return need;
}

// Staged sweeps (float): each level's tiles and vectors are copied global ->
// LDS a level ahead.  A vector slot holds kVecSlot entries (the vector, then
// copies of its last entry); a tile occupies its own 1 KiB lane groups, with at least
// one group for block 2 (0 when the shape does not fit class R: that product
// runs from global memory).
constexpr int kVecSlot = 64 * kVecPL;
__host__ __device__ inline int stage_groups(int K, int O, int V, int R) {
    if (col_need(K, O, V) > R) return 0;
    const int W1 = O < 64 ? O : 64, G1 = 64 / W1;
    int g = tile_rows(K, G1, V) / V;
    if (O > 64) {
        const int W2 = O - 64, G2 = 64 / W2;
        g += tile_rows(K, G2, V) / V;
    } else {
        g += 1;
    }
    return g;
}
// LDS elements of a staged sweep wavefront after the vectors: four vector
// slots and the stage of the larger sweep (bsweep: [Abar|B] and R~^-1 tiles,
// fsweep: [Abar|B]^T tile), for classes rb (bsweep) and rf (fsweep).
__host__ __device__ inline int stage_elems(int nx, int nu, int V, int rb, int rf) {
    const int m = nx + nu;
    const int gb = stage_groups(nx, m, V, rb) + stage_groups(nu, nu, V, 16);
    const int gf = stage_groups(m, nx, V, rf);
    return 4 * kVecSlot + imax(gb, gf) * 64 * V;
}

// Vector algebra of the SuperMann iteration (float64, iterate-sized vectors).
// out = sum_i c[i] in[i] entrywise; an input may be the output itself.
constexpr int kMaxCombo = 17;  // 2 m + 1 inputs for the Anderson direction, m <= 8
struct VecCombo {
    const double* in[kMaxCombo];
    double c[kMaxCombo];
    int n_in;
};
// A batch of dot products sum_k a[j][k] b[j][k], k < n[j], reduced in a fixed
// order (kDotBlocks block partials, then one wavefront).
constexpr int kMaxDots = 20;  // 2 m + 2 for the Anderson update, m <= 8
constexpr int kDotBlocks = 512;
struct DotSet {
    const double* a[kMaxDots];
    const double* b[kMaxDots];
    long long n[kMaxDots];
    int count;
};

}  // namespace spk
