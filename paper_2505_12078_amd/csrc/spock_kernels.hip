// gfx950 kernels of one Chambolle-Pock (CP) step of SPOCK on a scenario tree.
//
// One CP step (Sec. 4.1) is two launches over the tree:
//
//  backward  leaves -> root.  Per node: zbar = z - alpha L* eta for the node's
//            (x, u) (adjoint of L, Sec. 4.4), the backward recursion of Alg. 2
//            in reduced form, the S2 projection of the node's (y, tau, s) block
//            (Sec. 4.3) and, at the root, the prox of s0.  One workgroup starts
//            at every leaf and walks up; at a node with several children only
//            the last child to arrive continues (atomic arrival counter), so no
//            workgroup ever waits and the launch cannot deadlock.
//
//  forward   root -> leaves.  Per node: x^j = [Abar^j | B^j] [x^i; d^i] + c^j,
//            u^j = K^j x^j + d^j (Alg. 2 forward), then every dual block the
//            node owns: eta+ = prox_{alpha g*}(eta + alpha L(2 z+ - z)) with the
//            S3 cone projections and Moreau's identity, and on request the
//            residuals xi1, xi2 of Sec. 5.3.  One workgroup per leaf walks its
//            root-to-leaf path; the first workgroup to reach a node claims and
//            computes it, the others wait on its done flag.  A workgroup only
//            waits on a node claimed by a running workgroup whose own inputs
//            are already complete, so the wait always ends; a bounded spin
//            turns an unexpected stall into an error flag instead of a hang.
//
// Reduced S1 recursion (algebraically equal to Alg. 2, using
// sum_j Abar^jT P^j B^j = -K^iT, which follows from the definition of K in
// Alg. 1):  with h^j = q^j + P^j c^j and g = sum_{j in ch(i)} [Abar^j|B^j]^T h^j,
//   q^i = -xbar^i - K^iT ubar^i + g_x,   d^i = R~^i^-1 (ubar^i - g_u),
// and forward u^i = K^i x^i + d^i, x^j = Abar^j x^i + B^j d^i + c^j.
// Only [Abar|B] per edge and [K | R~^-1] per non-leaf node are read online.
//
// Every matrix is a contiguous row-major block per node, read once per
// kernel with coalesced loads straight into registers (no LDS staging): the
// transposed product (backward) maps consecutive lanes to consecutive columns;
// the plain product (forward) maps a power-of-two lane segment to a row and
// reduces it with cross-lane shuffles.  LDS only holds node vectors.

#include <hip/hip_runtime.h>

#include "spock_dev.h"

namespace spk {

constexpr int kHookWG = 256;  // workgroup size of the per-node hook kernels

#define SPK_DEV __device__ __forceinline__

// ---------------------------------------------------------------------------
// workgroup helpers
// ---------------------------------------------------------------------------

template <typename T>
SPK_DEV T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T>
SPK_DEV T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// Sum over the workgroup, same value returned to every thread; deterministic.
template <int kWG, typename T>
SPK_DEV T block_sum(T v, T* red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = 0;
#pragma unroll
    for (int k = 0; k < kWG / 64; ++k) s += red[k];
    return s;
}

template <int kWG, typename T>
SPK_DEV T block_max(T v, T* red) {
    v = wave_max(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = red[0];
#pragma unroll
    for (int k = 1; k < kWG / 64; ++k) s = red[k] > s ? red[k] : s;
    return s;
}

// out[c] = sum_r A[r*ld + c] * (c < split ? va[r] : vb[r]),  r < R, c < C.
// A in global memory, vectors and out in LDS.  Threads (g, c): lanes run along
// the columns of a row, so each load instruction covers a contiguous row
// segment; G row groups split the rows and are summed through LDS.
template <int kWG, typename real>
SPK_DEV void mat_t_vec(const real* __restrict__ A, int R, int C, long long ld, int split,
                       const real* va, const real* vb, real* out, real* red) {
    const int t = threadIdx.x;
    for (int c0 = 0; c0 < C; c0 += kWG) {
        const int Cc = (C - c0) < kWG ? (C - c0) : kWG;
        const int G = kWG / Cc;
        const int g = t / Cc, c = t - g * Cc;
        real acc = 0;
        if (g < G) {
            const real* v = (c0 + c < split) ? va : vb;
            const real* a = A + c0 + c;
#pragma unroll 4
            for (int r = g; r < R; r += G) acc += a[(long long)r * ld] * v[r];
        }
        __syncthreads();
        red[t] = acc;
        __syncthreads();
        if (t < Cc) {
            real s = 0;
            for (int k = 0; k < G; ++k) s += red[k * Cc + t];
            out[c0 + t] = s;
        }
        __syncthreads();
    }
}

// out[r] = sum_c A[r*ld + c] * v[c],  r < R, c < C.  A power-of-two segment of
// W lanes (W <= 64) owns a row: lanes stride the row, then reduce by xor
// shuffles inside the segment.
template <int kWG, typename real>
SPK_DEV void mat_vec(const real* __restrict__ A, int R, int C, long long ld, const real* v,
                     real* out) {
    int W = 1;
    while (W < C && W < 64) W <<= 1;
    const int t = threadIdx.x;
    const int nseg = kWG / W;
    const int seg = t / W, k = t - seg * W;
    for (int r0 = 0; r0 < R; r0 += nseg) {
        const int r = r0 + seg;
        real acc = 0;
        if (r < R) {
            const real* a = A + (long long)r * ld;
#pragma unroll 4
            for (int c = k; c < C; c += W) acc += a[c] * v[c];
        }
        for (int o = W >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, W);
        if (k == 0 && r < R) out[r] = acc;
    }
    __syncthreads();
}

// Register-prefetched forms of the two products.  The loads of a node's
// matrices do not depend on the sweep's vectors, so they are issued as soon as
// the node is known and consumed after the vectors are ready: one memory
// latency per node instead of one per batch of dependent loads.

// Transposed product, thread (g, c) with G = kWG / C row groups (needs C <= kWG):
// rows g + i G for i < RB live in registers, any further rows are read directly.
template <typename real, int RB>
struct TTile {
    real a[RB];
};

template <int kWG, typename real, int RB>
SPK_DEV void t_load(TTile<real, RB>& T, const real* __restrict__ A, int R, int C, long long ld) {
    const int t = threadIdx.x, G = kWG / C, g = t / C, c = t - g * C;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        const int r = g + i * G;
        T.a[i] = (g < G && r < R) ? A[(long long)r * ld + c] : real(0);
    }
}

// out[c] = sum_r A[r][c] (c < split ? va[r] : vb[r]) from a loaded tile.
template <int kWG, typename real, int RB>
SPK_DEV void t_apply(const TTile<real, RB>& T, const real* __restrict__ A, int R, int C, long long ld, int split,
                     const real* va, const real* vb, real* out, real* red) {
    const int t = threadIdx.x, G = kWG / C, g = t / C, c = t - g * C;
    real acc = 0;
    if (g < G) {
        const real* v = c < split ? va : vb;
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int r = g + i * G;
            if (r < R) acc += T.a[i] * v[r];
        }
        for (int r = g + RB * G; r < R; r += G) acc += A[(long long)r * ld + c] * v[r];
    }
    __syncthreads();
    red[t] = acc;
    __syncthreads();
    if (t < C) {
        real s = 0;
        for (int k = 0; k < G; ++k) s += red[k * C + t];
        out[t] = s;
    }
    __syncthreads();
}

// Plain product, a power-of-two segment of W lanes per row: rows seg + i nseg
// for i < RB and columns k + j W for j < CB live in registers.
template <typename real, int RB, int CB>
struct PTile {
    real a[RB][CB];
};

SPK_DEV int seg_width(int C) {
    int W = 1;
    while (W < C && W < 64) W <<= 1;
    return W;
}

template <int kWG, typename real, int RB, int CB>
SPK_DEV void p_load(PTile<real, RB, CB>& T, const real* __restrict__ A, int R, int C, long long ld) {
    const int W = seg_width(C), t = threadIdx.x, nseg = kWG / W, seg = t / W, k = t - seg * W;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        const int r = seg + i * nseg;
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            const int c = k + j * W;
            T.a[i][j] = (r < R && c < C) ? A[(long long)r * ld + c] : real(0);
        }
    }
}

template <int kWG, typename real, int RB, int CB>
SPK_DEV void p_apply(const PTile<real, RB, CB>& T, const real* __restrict__ A, int R, int C, long long ld,
                     const real* v, real* out) {
    const int W = seg_width(C), t = threadIdx.x, nseg = kWG / W, seg = t / W, k = t - seg * W;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        if (i * nseg >= R) break;  // uniform over the workgroup
        const int r = seg + i * nseg;
        real acc = 0;
        if (r < R) {
#pragma unroll
            for (int j = 0; j < CB; ++j)
                if (k + j * W < C) acc += T.a[i][j] * v[k + j * W];
            for (int c = k + CB * W; c < C; c += W) acc += A[(long long)r * ld + c] * v[c];
        }
        for (int o = W >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, W);
        if (k == 0 && r < R) out[r] = acc;
    }
    for (int r0 = RB * nseg; r0 < R; r0 += nseg) {
        const int r = r0 + seg;
        real acc = 0;
        if (r < R)
            for (int c = k; c < C; c += W) acc += A[(long long)r * ld + c] * v[c];
        for (int o = W >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, W);
        if (k == 0 && r < R) out[r] = acc;
    }
    __syncthreads();
}

// Register tile sizes (rows per thread kept in registers).
constexpr int kRBM = 20;  // [Abar|B]^T in the backward sweep
constexpr int kRBK = 12;  // [K|R~^-1]^T in the backward sweep
constexpr int kRBP = 16;  // [Abar|B] rows in the forward sweep (two column chunks)
constexpr int kRBQ = 8;   // K rows in the forward sweep

// Exchange between workgroups of one launch.  A value that another workgroup
// reads while the launch runs is stored and loaded at device scope: the store
// is written through to the level of the memory hierarchy that all XCDs share,
// and the load skips the XCD-private caches.  Before the barrier that precedes
// the counter or flag update, every wavefront drains its vector memory counter,
// so its device-scope stores are complete.  Release/acquire fences would do the
// same job, but at device scope they write back or invalidate the whole L2 of
// the XCD, and that costs tens of microseconds per node when many workgroups
// have stores in flight.
template <typename real>
SPK_DEV void st_dev(real* p, real v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename real>
SPK_DEV real ld_dev(const real* p) {
    return __hip_atomic_load(const_cast<real*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Every store this wavefront issued has completed (s_waitcnt vmcnt(0)); the
// workgroup fence keeps the compiler from sinking stores below it.
SPK_DEV void drain_stores() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0x0F70);
}

// Wait until a node's forward result is published; false on timeout.
SPK_DEV bool wait_done(int* flag) {
    const uint64_t t0 = wall_clock64();
    unsigned spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 2) {
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 1023u) == 0 && wall_clock64() - t0 > 200000000ull) return false;  // ~2 s
    }
    return true;
}

template <typename real>
SPK_DEV void record_max(unsigned long long* slot, real v) {
    const double d = (double)v;
    atomicMax(slot, (unsigned long long)__double_as_longlong(d));
}

// ---------------------------------------------------------------------------
// node input staging
// ---------------------------------------------------------------------------

// A node's vector inputs come from several arrays (z, eta, d, messages, ...).
// They are gathered into LDS in one pass: thread 0 writes a table of
// (source, length) segments, then every thread issues its share of the loads
// back to back before storing any of them, so a node costs one memory round
// trip for its vectors (issued together with its matrix tiles).
constexpr int kMaxSeg = 16;
constexpr int kGatherE = 4;  // loads in flight per thread per pass

template <typename real>
struct SegTable {
    const real* src[kMaxSeg];
    int off[kMaxSeg + 1];
    int n;
};

template <typename real>
SPK_DEV void seg_reset(SegTable<real>& T) {
    T.n = 0;
    T.off[0] = 0;
}

template <typename real>
SPK_DEV void seg_add(SegTable<real>& T, const real* src, int len) {
    T.src[T.n] = src;
    T.off[T.n + 1] = T.off[T.n] + len;
    T.n++;
}

template <int kWG, typename real>
SPK_DEV void seg_gather(const SegTable<real>& T, real* st, bool dev = false) {
    const int nseg = T.n;
    const int total = T.off[nseg];
    int off[kMaxSeg + 1];  // segment ends in registers: no dependent LDS reads per element
#pragma unroll
    for (int q = 0; q <= kMaxSeg; ++q) off[q] = q <= nseg ? T.off[q] : total;
    for (int base = 0; base < total; base += kGatherE * kWG) {
        real v[kGatherE];
#pragma unroll
        for (int j = 0; j < kGatherE; ++j) {
            const int e = base + j * kWG + (int)threadIdx.x;
            v[j] = 0;
            if (e < total) {
                int s = 0;
#pragma unroll
                for (int q = 1; q <= kMaxSeg; ++q) s += e >= off[q];
                const real* src = T.src[s] + (e - T.off[s]);
                v[j] = dev ? ld_dev(src) : *src;
            }
        }
#pragma unroll
        for (int j = 0; j < kGatherE; ++j) {
            const int e = base + j * kWG + (int)threadIdx.x;
            if (e < total) st[e] = v[j];
        }
    }
}

// Per-problem diagonal data staged once per workgroup.
template <typename real>
struct Consts {
    const real *qh, *rh, *qnh, *gx, *gu, *gb, *gxN, *gbN, *lo, *hi, *loN, *hiN;
};

SPK_DEV int consts_elems(int nx, int nu) { return 10 * nx + 4 * nu; }

template <typename real>
SPK_DEV void consts_table(const ProbDev<real>* __restrict__ P, SegTable<real>& T) {
    const int nx = P->nx, nu = P->nu, m = P->m;
    seg_reset(T);
    seg_add(T, P->qh, nx);
    seg_add(T, P->rh, nu);
    seg_add(T, P->qnh, nx);
    seg_add(T, P->gx, nx);
    seg_add(T, P->gu, nu);
    seg_add(T, P->gb, nx);
    seg_add(T, P->gxN, nx);
    seg_add(T, P->gbN, nx);
    seg_add(T, P->lo, m);
    seg_add(T, P->hi, m);
    seg_add(T, P->loN, nx);
    seg_add(T, P->hiN, nx);
}

template <typename real>
SPK_DEV Consts<real> consts_at(const real* c, int nx, int nu) {
    const int m = nx + nu;
    Consts<real> C;
    C.qh = c;
    C.rh = C.qh + nx;
    C.qnh = C.rh + nu;
    C.gx = C.qnh + nx;
    C.gu = C.gx + nx;
    C.gb = C.gu + nu;
    C.gxN = C.gb + nx;
    C.gbN = C.gxN + nx;
    C.lo = C.gbN + nx;
    C.hi = C.lo + m;
    C.loN = C.hi + m;
    C.hiN = C.loN + nx;
    return C;
}

// Root-to-leaf path nodes, their child counts and first children (LDS).
template <int kWG, typename real>
SPK_DEV void load_path(const ProbDev<real>* __restrict__ P, int leaf, int from, int* s_node, int* s_nch,
                       int* s_fc) {
    const int N = P->N;
    const int* path = P->path + (long long)leaf * (N + 1);
    for (int q = from + (int)threadIdx.x; q <= N; q += kWG) {
        const int v = path[q];
        s_node[q] = v;
        s_nch[q] = v < P->n_nl ? P->n_ch[v] : 0;
        s_fc[q] = v < P->n_nl ? P->first_child[v] : 0;
    }
}

// ---------------------------------------------------------------------------
// backward sweep
// ---------------------------------------------------------------------------

template <typename real, int kWG>
__global__ __launch_bounds__(kWG) void k_backward(const ProbDev<real>* __restrict__ probs,
                                                  const int2* __restrict__ tasks, int* __restrict__ ticket,
                                                  int par, int check) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_node[kMaxDepth], s_nch[kMaxDepth], s_fc[kMaxDepth];
    __shared__ SegTable<real> s_seg;
    __shared__ int s_last;
    real* sm = reinterpret_cast<real*>(smem_raw);
    const int2 tk = tasks[blockIdx.x];
    const ProbDev<real>* __restrict__ P = probs + tk.x;
    if (*P->active == 0) return;
    const int nx = P->nx, nu = P->nu, m = P->m, N = P->N, nc = P->nc, ncN = P->ncN, nbox = P->nbox;
    const int n_nl = P->n_nl;
    const real alpha = P->alpha;
    const real* __restrict__ zin = P->z[par];
    const real* __restrict__ ein = P->eta[par];
    real* __restrict__ zout = P->z[par ^ 1];
    const int t = threadIdx.x;

    real* red = sm;
    real* cst = red + kWG;
    real* st = cst + consts_elems(nx, nu);
    real* xb = st + stage_elems(nx, nu, nc, P->max_ch);  // xbar, then h = q + P c
    real* ub = xb + nx;                                  // ubar
    real* g = ub + nu;                                   // sum of children messages
    real* w2 = g + m;                                    // ubar - g_u
    real* o = w2 + nu;                                   // product outputs
    real* lam = o + m;                                   // S2 multipliers

    load_path<kWG>(P, tk.y, 0, s_node, s_nch, s_fc);
    if (t == 0) consts_table(P, s_seg);
    __syncthreads();
    seg_gather<kWG>(s_seg, cst);
    const Consts<real> C = consts_at<real>(cst, nx, nu);
    const bool tiles = m <= kWG;  // one column tile: register-prefetched products

    // ---- leaf: q = -xbar, message [Abar|B]^T (q + P c) ----
    int j = s_node[N];
    {
        TTile<real, kRBM> TM;
        if (tiles) t_load<kWG>(TM, P->M + j * P->M_stride, nx, m, m);
        const long long lf = j - n_nl;
        __syncthreads();  // constants gathered, table free
        if (t == 0) {
            seg_reset(s_seg);
            seg_add(s_seg, zin + P->z_x + (long long)j * nx, nx);
            seg_add(s_seg, ein + P->e_cN + lf * ncN, ncN);
            seg_add(s_seg, ein + P->e_socN + lf * (nx + 2), nx + 2);
            if (P->affine) seg_add(s_seg, P->Pc + (long long)j * nx, nx);
            P->flag[j] = 0;
        }
        __syncthreads();
        seg_gather<kWG>(s_seg, st);
        __syncthreads();
        const real* sx = st;
        const real* sc = sx + nx;
        const real* ss = sc + ncN;
        const real* spc = ss + nx + 2;
        for (int k = t; k < nx; k += kWG) {
            real lt = C.gxN[k] * sc[k] + C.qnh[k] * ss[k];
            if (P->has_ballN) lt += C.gbN[k] * sc[nx + k];
            real h = -(sx[k] - alpha * lt);
            if (P->affine) h += spc[k];
            xb[k] = h;
        }
        __syncthreads();
        if (tiles) t_apply<kWG>(TM, P->M + j * P->M_stride, nx, m, m, m, xb, xb, o, red);
        else mat_t_vec<kWG>(P->M + j * P->M_stride, nx, m, m, m, xb, xb, o, red);
    }

    // ---- walk up ----
    for (int lev = N - 1; lev >= 0; --lev) {
        const int i = s_node[lev];
        const int k = s_nch[lev], fc = s_fc[lev];
        if (k > 1) {
            for (int c = t; c < m; c += kWG) st_dev(P->e + (long long)j * m + c, o[c]);
            // every wave completes its own message stores before the arrival
            // is counted (a barrier alone does not wait for them)
            drain_stores();
            __syncthreads();
            if (t == 0) {
                const int prev =
                    __hip_atomic_fetch_add(&P->cnt[i], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int last = (prev == k - 1);
                if (last) P->cnt[i] = 0;  // the next launch reuses the counter
                s_last = last;
            }
            __syncthreads();
            if (!s_last) return;
        }
        TTile<real, kRBK> TK;
        TTile<real, kRBM> TM;
        if (tiles) {
            t_load<kWG>(TK, P->KR + i * P->KR_stride, nu, m, m);
            if (i > 0) t_load<kWG>(TM, P->M + i * P->M_stride, nx, m, m);
        }
        const bool leafkids = fc >= n_nl;
        const bool sk = k <= kStageKids;  // per-child inputs staged, else read in place
        const int kk = sk ? k : 0;
        const int cs_len = leafkids ? kk * (nx + 2) : kk;
        const long long yo = P->y_off[i];
        // staged inputs of node i (offsets into st)
        const int oX = 0, oU = oX + nx, oEC = oU + nu, oSOC = oEC + nc, oEY = oSOC + kk * (m + 2);
        const int oES = oEY + (sk ? 2 * k + 1 : 0), oZY = oES + 1, oZT = oZY + (sk ? 2 * k + 1 : 0);
        const int oZS = oZT + kk, oCS = oZS + kk, oP = oCS + cs_len, oMSG = oP + kk;
        const int oPC = oMSG + (k > 1 ? kk * m : 0);
        const real* g_soc = ein + P->e_soc + (long long)(fc - 1) * (m + 2);
        const real* g_cs = leafkids ? ein + P->e_socN + (long long)(fc - n_nl) * (nx + 2) : ein + P->e_s + fc;
        if (t == 0) {
            seg_reset(s_seg);
            seg_add(s_seg, zin + P->z_x + (long long)i * nx, nx);
            seg_add(s_seg, zin + P->z_u + (long long)i * nu, nu);
            seg_add(s_seg, ein + P->e_c + (long long)i * nc, nc);
            if (sk) {
                seg_add(s_seg, g_soc, k * (m + 2));
                seg_add(s_seg, ein + P->e_y + yo, 2 * k + 1);
            }
            seg_add(s_seg, ein + P->e_s + i, 1);
            if (sk) {
                seg_add(s_seg, zin + P->z_y + yo, 2 * k + 1);
                seg_add(s_seg, zin + P->z_tau + fc - 1, k);
                seg_add(s_seg, zin + P->z_s + fc - 1, k);
                seg_add(s_seg, g_cs, cs_len);
                seg_add(s_seg, P->prob + fc, k);
                if (k > 1) seg_add(s_seg, P->e + (long long)fc * m, k * m);
            }
            if (P->affine && i > 0) seg_add(s_seg, P->Pc + (long long)i * nx, nx);
            P->flag[i] = 0;
        }
        __syncthreads();
        seg_gather<kWG>(s_seg, st, k > 1);  // messages: device scope
        __syncthreads();
        // per-child inputs: staged copies or the arrays themselves
        const real* soc = sk ? st + oSOC : g_soc;
        const real* ey = sk ? st + oEY : ein + P->e_y + yo;
        const real* zy = sk ? st + oZY : zin + P->z_y + yo;
        const real* zt = sk ? st + oZT : zin + P->z_tau + fc - 1;
        const real* zs = sk ? st + oZS : zin + P->z_s + fc - 1;
        const real* cs = sk ? st + oCS : g_cs;
        const real* pr = sk ? st + oP : P->prob + fc;
        const real* msg = sk ? st + oMSG : P->e + (long long)fc * m;

        for (int c = t; c < m; c += kWG) {
            if (k > 1) {
                real s = 0;
                if (sk) {
                    for (int q = 0; q < k; ++q) s += msg[q * m + c];
                } else {
                    for (int q = 0; q < k; ++q) s += ld_dev(msg + q * m + c);
                }
                g[c] = s;
            } else {
                g[c] = o[c];
            }
        }
        // zbar for (x^i, u^i): L* gathers the constraint rows and the SOC rows of
        // every child edge (Sec. 4.4)
        for (int r = t; r < nx; r += kWG) {
            real s = 0;
            for (int q = 0; q < k; ++q) s += soc[q * (m + 2) + r];
            real lt = C.gx[r] * st[oEC + r] + C.qh[r] * s;
            if (P->has_ball) lt += C.gb[r] * st[oEC + nbox + r];
            xb[r] = st[oX + r] - alpha * lt;
        }
        for (int r = t; r < nu; r += kWG) {
            real s = 0, gu = 0;
            for (int q = 0; q < k; ++q) s += soc[q * (m + 2) + nx + r];
            if (k > 1) {
                if (sk) {
                    for (int q = 0; q < k; ++q) gu += msg[q * m + nx + r];
                } else {
                    for (int q = 0; q < k; ++q) gu += ld_dev(msg + q * m + nx + r);
                }
            } else {
                gu = o[nx + r];
            }
            const real lt = C.gu[r] * st[oEC + nx + r] + C.rh[r] * s;
            const real u = st[oU + r] - alpha * lt;
            ub[r] = u;
            w2[r] = u - gu;
        }
        // S2 projection (Sec. 4.3) of node i's block (y^i, tau^[i], s^[i]) after
        // the z - alpha L* eta shift, on the last wavefront.  Kernel of
        // G = [E^T, -I, -I] with E = [gamma I; -I; 1^T] (AV@R, Sec. 3.3);
        // G G^T = (gamma^2 + 3) I + 1 1^T, so with rho = G w the multiplier is
        // lambda = (rho - (1^T rho / (c + n)) 1) / c, c = gamma^2 + 3
        // (Sherman-Morrison), and w - G^T lambda is the projection.
        if ((t >> 6) == (kWG / 64) - 1) {
            const int lane = t & 63;
            const real gam = P->gamma[i], cc = gam * gam + real(3);
            const real es = st[oES];
            const real yb3 = zy[2 * k] - alpha * (ey[2 * k] - es);
            auto shifted = [&](int c, real& yb1, real& yb2, real& tb, real& sb) {
                yb1 = zy[c] - alpha * (ey[c] - pr[c] * es);
                yb2 = zy[k + c] - alpha * ey[k + c];
                tb = zt[c] - alpha * real(0.5) * (soc[c * (m + 2) + m] + soc[c * (m + 2) + m + 1]);
                const real lts = leafkids ? real(0.5) * (cs[c * (nx + 2) + nx] + cs[c * (nx + 2) + nx + 1]) : cs[c];
                sb = zs[c] - alpha * lts;
            };
            real rsum = 0;
            for (int c = lane; c < k; c += 64) {
                real yb1, yb2, tb, sb;
                shifted(c, yb1, yb2, tb, sb);
                const real rho = gam * yb1 - yb2 + yb3 - tb - sb;
                lam[c] = rho;
                rsum += rho;
            }
            rsum = wave_sum(rsum);
            real lsum = 0;
            for (int c = lane; c < k; c += 64) {
                real yb1, yb2, tb, sb;
                shifted(c, yb1, yb2, tb, sb);
                const real l = (lam[c] - rsum / (cc + real(k))) / cc;
                lsum += l;
                zout[P->z_y + yo + c] = yb1 - gam * l;
                zout[P->z_y + yo + k + c] = yb2 + l;
                zout[P->z_tau + fc + c - 1] = tb + l;
                zout[P->z_s + fc + c - 1] = sb + l;
            }
            lsum = wave_sum(lsum);
            if (lane == 0) zout[P->z_y + yo + 2 * k] = yb3 - lsum;
        }
        __syncthreads();
        // [K^T ubar ; R~^-1 (ubar - g_u)] in one pass over [K | R~^-1]
        if (tiles) t_apply<kWG>(TK, P->KR + i * P->KR_stride, nu, m, m, nx, ub, w2, o, red);
        else mat_t_vec<kWG>(P->KR + i * P->KR_stride, nu, m, m, nx, ub, w2, o, red);
        for (int r = t; r < nx; r += kWG) {
            real h = -xb[r] - o[r] + g[r];
            if (P->affine && i > 0) h += st[oPC + r];
            xb[r] = h;
        }
        for (int r = t; r < nu; r += kWG) P->d[(long long)i * nu + r] = o[nx + r];
        if (i == 0) {
            if (t == 0) {
                zout[0] = zin[0] - alpha * st[oES] - alpha;  // prox of alpha * s0
                ticket[0] = 0;                              // forward tickets restart
                if (check) {
                    P->res[0] = 0ull;
                    P->res[1] = 0ull;
                }
            }
            return;
        }
        __syncthreads();
        if (tiles) t_apply<kWG>(TM, P->M + i * P->M_stride, nx, m, m, m, xb, xb, o, red);
        else mat_t_vec<kWG>(P->M + i * P->M_stride, nx, m, m, m, xb, xb, o, red);
        j = i;
    }
}

// ---------------------------------------------------------------------------
// forward sweep
// ---------------------------------------------------------------------------

// eta+ = prox_{alpha g*}(etabar) for a box row: etabar - clamp(etabar, alpha lo, alpha hi)
template <typename real>
SPK_DEV real moreau_box(real eb, real alpha, real lo, real hi) {
    real p = eb < alpha * lo ? alpha * lo : eb;
    p = p > alpha * hi ? alpha * hi : p;
    return eb - p;
}

// Translated SOC (Prop. 1 with q = 0, a = (0,..,0, 1/2, -1/2), scalar last):
// with v = etabar - alpha a, eta+ = v - proj_SOC(v).  `nw2` is ||v_w||^2 over
// all entries but the last, `vt` the last entry.  Returns the factor applied
// to the w part and the value of the t entry.
template <typename real>
SPK_DEV void soc_moreau_coef(real nw2, real vt, real& cw, real& ct) {
    const real nw = sqrt(nw2);
    if (nw <= vt) {  // inside: proj = v, eta+ = 0
        cw = 0;
        ct = 0;
    } else if (nw <= -vt) {  // polar: proj = 0, eta+ = v
        cw = 1;
        ct = vt;
    } else {
        const real a = real(0.5) * (nw + vt);
        cw = real(1) - a / nw;
        ct = vt - a;
    }
}

// What the dual-block updates of one node read (LDS) and where they write.
template <typename real>
struct FwdNode {
    Consts<real> C;
    const real* xn;  // x+ of the node
    const real* un;  // u+
    const real* xo;  // x of the previous iterate (staged)
    const real* uo;
    real* blk;       // this wavefront's staging: etabar
    real* dblk;      //                            L dz, then eta - eta+
    real* lxw;       // this wavefront's share of (L* d_eta) on x
    real* luw;       //                                    on u
};

// eta_c of non-leaf node v: C^i = box x ball (one wavefront).  ec: staged eta_c.
template <typename real>
SPK_DEV void fwd_block_c(const ProbDev<real>* __restrict__ P, int v, const real* ec, real* __restrict__ eout,
                         const FwdNode<real>& V, int check, real& r2) {
    const int lane = threadIdx.x & 63;
    const int nx = P->nx, nbox = P->nbox, nc = P->nc;
    const real alpha = P->alpha, ialpha = real(1) / alpha;
    const long long off = P->e_c + (long long)v * nc;
    real nb2 = 0;
    for (int r = lane; r < nc; r += 64) {
        real wn, wo;
        if (r < nx) {
            wn = V.C.gx[r] * V.xn[r];
            wo = V.C.gx[r] * V.xo[r];
        } else if (r < nbox) {
            wn = V.C.gu[r - nx] * V.un[r - nx];
            wo = V.C.gu[r - nx] * V.uo[r - nx];
        } else {
            wn = V.C.gb[r - nbox] * V.xn[r - nbox];
            wo = V.C.gb[r - nbox] * V.xo[r - nbox];
        }
        const real eb = ec[r] + alpha * (real(2) * wn - wo);
        V.blk[r] = eb;
        V.dblk[r] = wo - wn;
        if (r >= nbox) nb2 += eb * eb;
    }
    real cb = 0;
    if (P->has_ball) {
        nb2 = wave_sum(nb2);
        const real nrm = sqrt(nb2);
        const real rad = alpha * P->ball_r;
        cb = nrm > rad ? real(1) - rad / nrm : real(0);
    }
    for (int r = lane; r < nc; r += 64) {
        const real eb = V.blk[r];
        const real ep = r < nbox ? moreau_box(eb, alpha, V.C.lo[r], V.C.hi[r]) : eb * cb;
        eout[off + r] = ep;
        const real de = ec[r] - ep;
        if (check) r2 = fmax(r2, fabs(de * ialpha - V.dblk[r]));
        V.dblk[r] = de;
    }
    if (check) {
        __builtin_amdgcn_wave_barrier();
        for (int r = lane; r < nx; r += 64) {
            real s = V.C.gx[r] * V.dblk[r];
            if (P->has_ball) s += V.C.gb[r] * V.dblk[nbox + r];
            V.lxw[r] += s;
        }
        for (int r = lane; r < P->nu; r += 64) V.luw[r] += V.C.gu[r] * V.dblk[nx + r];
    }
}

// eta_y in (K^i)* = R^{2k}_+ x R and eta_s in R_+ (one wavefront), from staged
// eta_y (ey), eta_s (es), new and old y (yn, yv) and s (sn, sv), probabilities p.
template <typename real>
SPK_DEV void fwd_block_risk(const ProbDev<real>* __restrict__ P, int v, int k, const real* ey, real es,
                            const real* yn, const real* yv, real sn, real sv, const real* p,
                            real* __restrict__ eout, int check, real& r1, real& r2) {
    const int lane = threadIdx.x & 63;
    const real alpha = P->alpha, ialpha = real(1) / alpha;
    const long long yo = P->y_off[v];
    real bn = 0, bo = 0;  // b^T y with b = (p, 0, 1)
    for (int c = lane; c < k; c += 64) {
        bn += p[c] * yn[c];
        bo += p[c] * yv[c];
    }
    bn = wave_sum(bn) + yn[2 * k];
    bo = wave_sum(bo) + yv[2 * k];
    const real wsn = sn - bn, wso = sv - bo;
    const real ebs = es + alpha * (real(2) * wsn - wso);
    const real eps_ = ebs < 0 ? ebs : real(0);
    const real des = es - eps_;
    if (lane == 0) eout[P->e_s + v] = eps_;
    for (int c = lane; c < 2 * k + 1; c += 64) {
        const real eb = ey[c] + alpha * (real(2) * yn[c] - yv[c]);
        const real ep = c < 2 * k ? (eb < 0 ? eb : real(0)) : real(0);
        eout[P->e_y + yo + c] = ep;
        if (check) {
            const real de = ey[c] - ep;
            const real dy = yv[c] - yn[c];
            r2 = fmax(r2, fabs(de * ialpha - dy));
            const real bc = c < k ? p[c] : (c == 2 * k ? real(1) : real(0));
            r1 = fmax(r1, fabs(dy * ialpha - (de - bc * des)));
        }
    }
    if (check && lane == 0) {
        r2 = fmax(r2, fabs(des * ialpha - (wso - wsn)));
        r1 = fmax(r1, fabs((sv - sn) * ialpha - des));
    }
}

// SOC block of the edge into child j of non-leaf node v:
// (Q^1/2 x^v, R^1/2 u^v, tau^j / 2, tau^j / 2) in SOC + a (one wavefront);
// es: staged eta_soc of that edge, tn / tv: new / old tau^j.
template <typename real>
SPK_DEV void fwd_block_soc(const ProbDev<real>* __restrict__ P, int j, const real* es, real tn, real tv,
                           real* __restrict__ eout, const FwdNode<real>& V, int check, real& r1, real& r2) {
    const int lane = threadIdx.x & 63;
    const int nx = P->nx, m = P->m;
    const real alpha = P->alpha, ialpha = real(1) / alpha;
    const long long off = P->e_soc + (long long)(j - 1) * (m + 2);
    real nw2 = 0;
    for (int r = lane; r < m + 2; r += 64) {
        real wn, wo;
        if (r < nx) {
            wn = V.C.qh[r] * V.xn[r];
            wo = V.C.qh[r] * V.xo[r];
        } else if (r < m) {
            wn = V.C.rh[r - nx] * V.un[r - nx];
            wo = V.C.rh[r - nx] * V.uo[r - nx];
        } else {
            wn = real(0.5) * tn;
            wo = real(0.5) * tv;
        }
        real eb = es[r] + alpha * (real(2) * wn - wo);
        if (r == m) eb -= real(0.5) * alpha;  // v = etabar - alpha a
        if (r == m + 1) eb += real(0.5) * alpha;
        V.blk[r] = eb;
        V.dblk[r] = wo - wn;
        if (r <= m) nw2 += eb * eb;
    }
    nw2 = wave_sum(nw2);
    __builtin_amdgcn_wave_barrier();
    real cw, ct;
    soc_moreau_coef(nw2, V.blk[m + 1], cw, ct);
    for (int r = lane; r < m + 2; r += 64) {
        const real ep = r <= m ? V.blk[r] * cw : ct;
        eout[off + r] = ep;
        const real de = es[r] - ep;
        if (check) r2 = fmax(r2, fabs(de * ialpha - V.dblk[r]));
        V.dblk[r] = de;
    }
    if (check) {
        __builtin_amdgcn_wave_barrier();
        for (int r = lane; r < nx; r += 64) V.lxw[r] += V.C.qh[r] * V.dblk[r];
        for (int r = lane; r < P->nu; r += 64) V.luw[r] += V.C.rh[r] * V.dblk[nx + r];
        if (lane == 0) r1 = fmax(r1, fabs((tv - tn) * ialpha - real(0.5) * (V.dblk[m] + V.dblk[m + 1])));
    }
}

// Leaf v: eta_cN (box x ball) for which = 0, eta_socN (Q_N^1/2 x, s/2, s/2) for
// which = 1 (one wavefront each); ec / es: the staged blocks.
template <typename real>
SPK_DEV void fwd_block_leaf(const ProbDev<real>* __restrict__ P, int v, int which, const real* ec,
                            const real* es, real sn, real sv, real* __restrict__ eout, const FwdNode<real>& V,
                            int check, real& r1, real& r2) {
    const int lane = threadIdx.x & 63;
    const int nx = P->nx;
    const real alpha = P->alpha, ialpha = real(1) / alpha;
    const long long lf = v - P->n_nl;
    if (which == 0) {
        const long long off = P->e_cN + lf * P->ncN;
        real nb2 = 0;
        for (int r = lane; r < P->ncN; r += 64) {
            real wn, wo;
            if (r < nx) {
                wn = V.C.gxN[r] * V.xn[r];
                wo = V.C.gxN[r] * V.xo[r];
            } else {
                wn = V.C.gbN[r - nx] * V.xn[r - nx];
                wo = V.C.gbN[r - nx] * V.xo[r - nx];
            }
            const real eb = ec[r] + alpha * (real(2) * wn - wo);
            V.blk[r] = eb;
            V.dblk[r] = wo - wn;
            if (r >= nx) nb2 += eb * eb;
        }
        real cb = 0;
        if (P->has_ballN) {
            nb2 = wave_sum(nb2);
            const real nrm = sqrt(nb2);
            const real rad = alpha * P->ballN_r;
            cb = nrm > rad ? real(1) - rad / nrm : real(0);
        }
        for (int r = lane; r < P->ncN; r += 64) {
            const real eb = V.blk[r];
            const real ep = r < nx ? moreau_box(eb, alpha, V.C.loN[r], V.C.hiN[r]) : eb * cb;
            eout[off + r] = ep;
            const real de = ec[r] - ep;
            if (check) r2 = fmax(r2, fabs(de * ialpha - V.dblk[r]));
            V.dblk[r] = de;
        }
        if (check) {
            __builtin_amdgcn_wave_barrier();
            for (int r = lane; r < nx; r += 64) {
                real s = V.C.gxN[r] * V.dblk[r];
                if (P->has_ballN) s += V.C.gbN[r] * V.dblk[nx + r];
                V.lxw[r] += s;
            }
        }
    } else {
        const long long off = P->e_socN + lf * (nx + 2);
        real nw2 = 0;
        for (int r = lane; r < nx + 2; r += 64) {
            real wn, wo;
            if (r < nx) {
                wn = V.C.qnh[r] * V.xn[r];
                wo = V.C.qnh[r] * V.xo[r];
            } else {
                wn = real(0.5) * sn;
                wo = real(0.5) * sv;
            }
            real eb = es[r] + alpha * (real(2) * wn - wo);
            if (r == nx) eb -= real(0.5) * alpha;
            if (r == nx + 1) eb += real(0.5) * alpha;
            V.blk[r] = eb;
            V.dblk[r] = wo - wn;
            if (r <= nx) nw2 += eb * eb;
        }
        nw2 = wave_sum(nw2);
        __builtin_amdgcn_wave_barrier();
        real cw, ct;
        soc_moreau_coef(nw2, V.blk[nx + 1], cw, ct);
        for (int r = lane; r < nx + 2; r += 64) {
            const real ep = r <= nx ? V.blk[r] * cw : ct;
            eout[off + r] = ep;
            const real de = es[r] - ep;
            if (check) r2 = fmax(r2, fabs(de * ialpha - V.dblk[r]));
            V.dblk[r] = de;
        }
        if (check) {
            __builtin_amdgcn_wave_barrier();
            for (int r = lane; r < nx; r += 64) V.lxw[r] += V.C.qnh[r] * V.dblk[r];
            if (lane == 0) r1 = fmax(r1, fabs((sv - sn) * ialpha - real(0.5) * (V.dblk[nx] + V.dblk[nx + 1])));
        }
    }
}

template <typename real, int kWG>
__global__ __launch_bounds__(kWG) void k_forward(const ProbDev<real>* __restrict__ probs,
                                                 const int2* __restrict__ tasks, int* __restrict__ ticket,
                                                 int par, int check) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_node[kMaxDepth], s_nch[kMaxDepth], s_fc[kMaxDepth];
    __shared__ SegTable<real> s_seg;
    __shared__ int s_task, s_ok;
    real* sm = reinterpret_cast<real*>(smem_raw);
    const int t = threadIdx.x, w = t >> 6;
    // Tickets hand out tasks in start order, so a workgroup only ever waits on
    // a workgroup that started before it.
    if (t == 0) s_task = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int2 tk = tasks[s_task];
    const ProbDev<real>* __restrict__ P = probs + tk.x;
    if (*P->active == 0) return;
    const int nx = P->nx, nu = P->nu, m = P->m, N = P->N, nc = P->nc, ncN = P->ncN;
    const int n_nl = P->n_nl;
    const real ialpha = real(1) / P->alpha;
    const real* __restrict__ zin = P->z[par];
    const real* __restrict__ ein = P->eta[par];
    real* __restrict__ zout = P->z[par ^ 1];
    real* __restrict__ eout = P->eta[par ^ 1];
    const int bmax = blk_elems(nx, nu, P->max_ch);
    constexpr int kWaves = kWG / 64;

    real* red = sm;
    real* cst = red + kWG;
    real* st = cst + consts_elems(nx, nu);
    real* xa = st + stage_elems(nx, nu, nc, P->max_ch);  // [x^anc ; d^anc]
    real* xn = xa + m;
    real* un = xn + nx;
    real* lxw = un + nu;             // kWaves x nx
    real* luw = lxw + kWaves * nx;   // kWaves x nu
    real* blk = luw + kWaves * nu;   // kWaves x bmax
    real* dblk = blk + kWaves * bmax;

    // this task computes the path nodes from stage L down to its leaf; the
    // node above them belongs to the task of its leftmost leaf
    const int L = P->top_owned[tk.y];
    load_path<kWG>(P, tk.y, L > 0 ? L - 1 : 0, s_node, s_nch, s_fc);
    if (t == 0) consts_table(P, s_seg);
    __syncthreads();
    seg_gather<kWG>(s_seg, cst);
    const Consts<real> C = consts_at<real>(cst, nx, nu);
    if (t == 0) {
        int ok = 1;
        if (L > 0 && !wait_done(&P->flag[s_node[L - 1]])) {
            atomicExch(P->err, 1);
            ok = 0;
        }
        s_ok = ok;
    }
    __syncthreads();
    if (!s_ok) return;
    if (L > 0) {
        const int pn = s_node[L - 1];
        for (int r = t; r < nx; r += kWG) xa[r] = ld_dev(zout + P->z_x + (long long)pn * nx + r);
        for (int r = t; r < nu; r += kWG) xa[nx + r] = P->d[(long long)pn * nu + r];
    }

    real r1 = 0, r2 = 0;  // residual maxima of this thread
    for (int lev = L; lev <= N; ++lev) {
        const int v = s_node[lev];
        const int k = s_nch[lev], fc = s_fc[lev];
        const bool nonleaf = v < n_nl;
        PTile<real, kRBP, 2> TM;
        PTile<real, kRBQ, 1> TK;
        if (v > 0) p_load<kWG>(TM, P->M + v * P->M_stride, nx, m, m);
        if (nonleaf) p_load<kWG>(TK, P->KR + v * P->KR_stride, nu, nx, m);
        // staged inputs of node v (offsets into st)
        const long long yo = nonleaf ? P->y_off[v] : 0;
        const long long soff = (v == 0) ? 0 : P->z_s + v - 1;
        const bool sk = k <= kStageKids;  // per-child inputs staged, else read in place
        const int kk = sk ? k : 0, ky = sk ? 2 * k + 1 : 0;
        int oD = 0, oXO = 0, oUO = 0, oEC = 0, oSOC = 0, oEY = 0, oES = 0, oYN = 0, oYO = 0, oSN = 0, oSO = 0;
        int oTN = 0, oTO = 0, oP = 0, oC = 0, oECN = 0, oSOCN = 0;
        if (nonleaf) {
            oD = 0; oXO = oD + nu; oUO = oXO + nx; oEC = oUO + nu; oSOC = oEC + nc; oEY = oSOC + kk * (m + 2);
            oES = oEY + ky; oYN = oES + 1; oYO = oYN + ky; oSN = oYO + ky; oSO = oSN + 1;
            oTN = oSO + 1; oTO = oTN + kk; oP = oTO + kk; oC = oP + kk;
        } else {
            oXO = 0; oECN = oXO + nx; oSOCN = oECN + ncN; oSN = oSOCN + nx + 2; oSO = oSN + 1; oC = oSO + 1;
        }
        __syncthreads();  // previous stage data consumed, table free
        if (t == 0) {
            seg_reset(s_seg);
            if (nonleaf) {
                seg_add(s_seg, P->d + (long long)v * nu, nu);
                seg_add(s_seg, zin + P->z_x + (long long)v * nx, nx);
                seg_add(s_seg, zin + P->z_u + (long long)v * nu, nu);
                seg_add(s_seg, ein + P->e_c + (long long)v * nc, nc);
                if (sk) {
                    seg_add(s_seg, ein + P->e_soc + (long long)(fc - 1) * (m + 2), k * (m + 2));
                    seg_add(s_seg, ein + P->e_y + yo, 2 * k + 1);
                }
                seg_add(s_seg, ein + P->e_s + v, 1);
                if (sk) {
                    seg_add(s_seg, zout + P->z_y + yo, 2 * k + 1);
                    seg_add(s_seg, zin + P->z_y + yo, 2 * k + 1);
                }
                seg_add(s_seg, zout + soff, 1);
                seg_add(s_seg, zin + soff, 1);
                if (sk) {
                    seg_add(s_seg, zout + P->z_tau + fc - 1, k);
                    seg_add(s_seg, zin + P->z_tau + fc - 1, k);
                    seg_add(s_seg, P->prob + fc, k);
                }
            } else {
                seg_add(s_seg, zin + P->z_x + (long long)v * nx, nx);
                seg_add(s_seg, ein + P->e_cN + (long long)(v - n_nl) * ncN, ncN);
                seg_add(s_seg, ein + P->e_socN + (long long)(v - n_nl) * (nx + 2), nx + 2);
                seg_add(s_seg, zout + soff, 1);
                seg_add(s_seg, zin + soff, 1);
            }
            if (P->affine && v > 0) seg_add(s_seg, P->c + (long long)v * nx, nx);
        }
        __syncthreads();
        seg_gather<kWG>(s_seg, st);
        __syncthreads();

        // ---- state: x^v = [Abar|B] [x^anc; d^anc] + c ----
        if (v == 0) {
            for (int r = t; r < nx; r += kWG) xn[r] = P->x0[r];
            __syncthreads();
        } else {
            p_apply<kWG>(TM, P->M + v * P->M_stride, nx, m, m, xa, xn);
            if (P->affine) {
                for (int r = t; r < nx; r += kWG) xn[r] += st[oC + r];
                __syncthreads();
            }
        }
        if (nonleaf && k > 1) {
            // children owned by other tasks read x^v (and d^v): publish now
            for (int r = t; r < nx; r += kWG) st_dev(zout + P->z_x + (long long)v * nx + r, xn[r]);
            drain_stores();
            __syncthreads();
            if (t == 0) st_dev(P->flag + v, 2);
        } else {
            for (int r = t; r < nx; r += kWG) zout[P->z_x + (long long)v * nx + r] = xn[r];
        }
        if (nonleaf) {
            // ---- input: u^v = K^v x^v + d^v ----
            p_apply<kWG>(TK, P->KR + v * P->KR_stride, nu, nx, m, xn, un);
            for (int r = t; r < nu; r += kWG) {
                const real u = un[r] + st[oD + r];
                un[r] = u;
                zout[P->z_u + (long long)v * nu + r] = u;
            }
        }
        if (check) {
            for (int r = t & 63; r < nx; r += 64) lxw[w * nx + r] = 0;
            for (int r = t & 63; r < nu; r += 64) luw[w * nu + r] = 0;
        }
        __syncthreads();
        // ---- dual blocks, one wavefront each ----
        const FwdNode<real> V{C, xn, un, st + oXO, st + oUO, blk + w * bmax, dblk + w * bmax,
                              lxw + w * nx, luw + w * nu};
        if (nonleaf) {
            // per-child inputs: staged copies or the arrays themselves
            const real* soc = sk ? st + oSOC : ein + P->e_soc + (long long)(fc - 1) * (m + 2);
            const real* ey = sk ? st + oEY : ein + P->e_y + yo;
            const real* yn = sk ? st + oYN : zout + P->z_y + yo;
            const real* yv = sk ? st + oYO : zin + P->z_y + yo;
            const real* tn = sk ? st + oTN : zout + P->z_tau + fc - 1;
            const real* tv = sk ? st + oTO : zin + P->z_tau + fc - 1;
            const real* pr = sk ? st + oP : P->prob + fc;
            for (int b = w; b < k + 2; b += kWaves) {
                if (b == 0) {
                    fwd_block_c(P, v, st + oEC, eout, V, check, r2);
                } else if (b == 1) {
                    fwd_block_risk(P, v, k, ey, st[oES], yn, yv, st[oSN], st[oSO], pr, eout, check, r1, r2);
                } else {
                    const int q = b - 2;
                    fwd_block_soc(P, fc + q, soc + q * (m + 2), tn[q], tv[q], eout, V, check, r1, r2);
                }
            }
        } else {
            for (int b = w; b < 2; b += kWaves)
                fwd_block_leaf(P, v, b, st + oECN, st + oSOCN, st[oSN], st[oSO], eout, V, check, r1, r2);
        }
        if (check) {
            __syncthreads();
            for (int r = t; r < nx; r += kWG) {
                real s = 0;
                for (int q = 0; q < kWaves; ++q) s += lxw[q * nx + r];
                r1 = fmax(r1, fabs((st[oXO + r] - xn[r]) * ialpha - s));
            }
            if (nonleaf)
                for (int r = t; r < nu; r += kWG) {
                    real s = 0;
                    for (int q = 0; q < kWaves; ++q) s += luw[q * nu + r];
                    r1 = fmax(r1, fabs((st[oUO + r] - un[r]) * ialpha - s));
                }
        }
        // ---- next stage input [x^v ; d^v] ----
        if (lev < N) {
            __syncthreads();
            for (int r = t; r < nx; r += kWG) xa[r] = xn[r];
            for (int r = t; r < nu; r += kWG) xa[nx + r] = st[oD + r];
        }
    }
    if (check) {
        r1 = block_max<kWG>(r1, red);
        r2 = block_max<kWG>(r2, red);
        if (t == 0) {
            record_max(&P->res[0], r1);
            record_max(&P->res[1], r2);
        }
    }
}

// ---------------------------------------------------------------------------
// operator hooks: one workgroup per node, plain code paths
// ---------------------------------------------------------------------------

// eta = L z for the blocks node v owns (Sec. 4.4).
template <typename real>
__global__ __launch_bounds__(kHookWG) void k_apply_L(const ProbDev<real>* __restrict__ P,
                                                 const real* __restrict__ z, real* __restrict__ eta) {
    __shared__ real red[kHookWG];
    const int v = blockIdx.x, t = threadIdx.x;
    const int nx = P->nx, nu = P->nu, m = P->m, nbox = P->nbox;
    const real* x = z + P->z_x + (long long)v * nx;
    if (v < P->n_nl) {
        const real* u = z + P->z_u + (long long)v * nu;
        for (int r = t; r < P->nc; r += kHookWG) {
            real w;
            if (r < nx) w = P->gx[r] * x[r];
            else if (r < nbox) w = P->gu[r - nx] * u[r - nx];
            else w = P->gb[r - nbox] * x[r - nbox];
            eta[P->e_c + (long long)v * P->nc + r] = w;
        }
        const int k = P->n_ch[v], fc = P->first_child[v];
        const long long yo = P->y_off[v];
        const real* y = z + P->z_y + yo;
        real b = 0;
        for (int c = t; c < k; c += kHookWG) b += P->prob[fc + c] * y[c];
        b = block_sum<kHookWG>(b, red) + y[2 * k];
        const real s = (v == 0) ? z[0] : z[P->z_s + v - 1];
        if (t == 0) eta[P->e_s + v] = s - b;
        for (int c = t; c < 2 * k + 1; c += kHookWG) eta[P->e_y + yo + c] = y[c];
        for (int q = 0; q < k; ++q) {
            const int j = fc + q;
            const real tau = z[P->z_tau + j - 1];
            real* o = eta + P->e_soc + (long long)(j - 1) * (m + 2);
            for (int r = t; r < m + 2; r += kHookWG)
                o[r] = r < nx ? P->qh[r] * x[r] : (r < m ? P->rh[r - nx] * u[r - nx] : real(0.5) * tau);
        }
    } else {
        const long long lf = v - P->n_nl;
        for (int r = t; r < P->ncN; r += kHookWG)
            eta[P->e_cN + lf * P->ncN + r] = r < nx ? P->gxN[r] * x[r] : P->gbN[r - nx] * x[r - nx];
        const real s = z[P->z_s + v - 1];
        for (int r = t; r < nx + 2; r += kHookWG)
            eta[P->e_socN + lf * (nx + 2) + r] = r < nx ? P->qnh[r] * x[r] : real(0.5) * s;
    }
}

// z = L* eta for the primal entries node v owns (adjoint of k_apply_L).
template <typename real>
__global__ __launch_bounds__(kHookWG) void k_apply_Lt(const ProbDev<real>* __restrict__ P,
                                                  const real* __restrict__ eta, real* __restrict__ z) {
    const int v = blockIdx.x, t = threadIdx.x;
    const int nx = P->nx, nu = P->nu, m = P->m, nbox = P->nbox;
    real* x = z + P->z_x + (long long)v * nx;
    if (v < P->n_nl) {
        const int k = P->n_ch[v], fc = P->first_child[v];
        const real* ec = eta + P->e_c + (long long)v * P->nc;
        for (int r = t; r < nx; r += kHookWG) {
            real s = 0;
            for (int q = 0; q < k; ++q) s += eta[P->e_soc + (long long)(fc + q - 1) * (m + 2) + r];
            real w = P->gx[r] * ec[r] + P->qh[r] * s;
            if (P->has_ball) w += P->gb[r] * ec[nbox + r];
            x[r] = w;
        }
        for (int r = t; r < nu; r += kHookWG) {
            real s = 0;
            for (int q = 0; q < k; ++q) s += eta[P->e_soc + (long long)(fc + q - 1) * (m + 2) + nx + r];
            z[P->z_u + (long long)v * nu + r] = P->gu[r] * ec[nx + r] + P->rh[r] * s;
        }
        const long long yo = P->y_off[v];
        const real es = eta[P->e_s + v];
        for (int c = t; c < 2 * k + 1; c += kHookWG) {
            const real bc = c < k ? P->prob[fc + c] : (c == 2 * k ? real(1) : real(0));
            z[P->z_y + yo + c] = eta[P->e_y + yo + c] - bc * es;
        }
        if (t == 0) {
            if (v == 0) z[0] = es;
            else z[P->z_s + v - 1] = es;
        }
        for (int q = t; q < k; q += kHookWG) {
            const int j = fc + q;
            const real* o = eta + P->e_soc + (long long)(j - 1) * (m + 2);
            z[P->z_tau + j - 1] = real(0.5) * (o[m] + o[m + 1]);
        }
    } else {
        const long long lf = v - P->n_nl;
        const real* ecN = eta + P->e_cN + lf * P->ncN;
        const real* esN = eta + P->e_socN + lf * (nx + 2);
        for (int r = t; r < nx; r += kHookWG) {
            real w = P->gxN[r] * ecN[r] + P->qnh[r] * esN[r];
            if (P->has_ballN) w += P->gbN[r] * ecN[nx + r];
            x[r] = w;
        }
        if (t == 0) z[P->z_s + v - 1] = real(0.5) * (esN[nx] + esN[nx + 1]);
    }
}

// eta = w - alpha proj_S3(w / alpha) for the blocks node v owns.
template <typename real>
__global__ __launch_bounds__(kHookWG) void k_prox_gconj(const ProbDev<real>* __restrict__ P,
                                                    const real* __restrict__ w, real* __restrict__ eta) {
    __shared__ real red[kHookWG];
    const int v = blockIdx.x, t = threadIdx.x;
    const int nx = P->nx, m = P->m, nbox = P->nbox;
    const real alpha = P->alpha;
    auto soc = [&](long long off, int len) {
        real nw2 = 0;
        for (int r = t; r < len - 1; r += kHookWG) {
            real e = w[off + r];
            if (r == len - 2) e -= real(0.5) * alpha;
            nw2 += e * e;
        }
        nw2 = block_sum<kHookWG>(nw2, red);
        const real vt = w[off + len - 1] + real(0.5) * alpha;
        real cw, ct;
        soc_moreau_coef(nw2, vt, cw, ct);
        for (int r = t; r < len; r += kHookWG) {
            real e = w[off + r];
            if (r == len - 2) e -= real(0.5) * alpha;
            eta[off + r] = r < len - 1 ? e * cw : ct;
        }
    };
    auto ballbox = [&](long long off, int nb, int ntot, const real* lo, const real* hi, real r_ball) {
        real nb2 = 0;
        for (int r = nb + t; r < ntot; r += kHookWG) nb2 += w[off + r] * w[off + r];
        real cb = 0;
        if (ntot > nb) {
            nb2 = block_sum<kHookWG>(nb2, red);
            const real nrm = sqrt(nb2), rad = alpha * r_ball;
            cb = nrm > rad ? real(1) - rad / nrm : real(0);
        }
        for (int r = t; r < ntot; r += kHookWG)
            eta[off + r] = r < nb ? moreau_box(w[off + r], alpha, lo[r], hi[r]) : w[off + r] * cb;
    };
    if (v < P->n_nl) {
        const int k = P->n_ch[v], fc = P->first_child[v];
        const long long yo = P->y_off[v];
        for (int c = t; c < 2 * k + 1; c += kHookWG) {
            const real e = w[P->e_y + yo + c];
            eta[P->e_y + yo + c] = c < 2 * k ? (e < 0 ? e : real(0)) : real(0);
        }
        if (t == 0) {
            const real e = w[P->e_s + v];
            eta[P->e_s + v] = e < 0 ? e : real(0);
        }
        ballbox(P->e_c + (long long)v * P->nc, nbox, P->nc, P->lo, P->hi, P->ball_r);
        for (int q = 0; q < k; ++q) soc(P->e_soc + (long long)(fc + q - 1) * (m + 2), m + 2);
    } else {
        const long long lf = v - P->n_nl;
        ballbox(P->e_cN + lf * P->ncN, nx, P->ncN, P->loN, P->hiN, P->ballN_r);
        soc(P->e_socN + lf * (nx + 2), nx + 2);
    }
}

// dst = (real) src over n entries (precision conversion of iterates)
template <typename D, typename S>
__global__ void k_convert(D* __restrict__ dst, const S* __restrict__ src, long long n) {
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        dst[k] = (D)src[k];
}

template <typename T>
__global__ void k_fill(T* __restrict__ dst, T val, long long n) {
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        dst[k] = val;
}

// ---------------------------------------------------------------------------
// launchers (host side)
// ---------------------------------------------------------------------------

template <typename real, int WG>
static hipError_t launch_sweep(bool backward, const ProbDev<real>* probs, const int2* tasks, int* ticket,
                               int n_tasks, int lds_bytes, int par, int check, hipStream_t st) {
    if (backward)
        hipLaunchKernelGGL((k_backward<real, WG>), dim3(n_tasks), dim3(WG), lds_bytes, st, probs, tasks, ticket,
                           par, check);
    else
        hipLaunchKernelGGL((k_forward<real, WG>), dim3(n_tasks), dim3(WG), lds_bytes, st, probs, tasks, ticket,
                           par, check);
    return hipGetLastError();
}

template <typename real>
static hipError_t launch_wg(bool backward, const ProbDev<real>* probs, const int2* tasks, int* ticket,
                            int n_tasks, int lds_bytes, int par, int check, int wg, hipStream_t st) {
    switch (wg) {
        case 64: return launch_sweep<real, 64>(backward, probs, tasks, ticket, n_tasks, lds_bytes, par, check, st);
        case 128: return launch_sweep<real, 128>(backward, probs, tasks, ticket, n_tasks, lds_bytes, par, check, st);
        case 256: return launch_sweep<real, 256>(backward, probs, tasks, ticket, n_tasks, lds_bytes, par, check, st);
        case 512: return launch_sweep<real, 512>(backward, probs, tasks, ticket, n_tasks, lds_bytes, par, check, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename real>
hipError_t launch_backward(const ProbDev<real>* probs, const int2* tasks, int* ticket, int n_tasks,
                           int lds_bytes, int par, int check, int wg, hipStream_t st) {
    return launch_wg<real>(true, probs, tasks, ticket, n_tasks, lds_bytes, par, check, wg, st);
}

template <typename real>
hipError_t launch_forward(const ProbDev<real>* probs, const int2* tasks, int* ticket, int n_tasks,
                          int lds_bytes, int par, int check, int wg, hipStream_t st) {
    return launch_wg<real>(false, probs, tasks, ticket, n_tasks, lds_bytes, par, check, wg, st);
}

template <typename real>
hipError_t launch_step(const ProbDev<real>* probs, const int2* tasks, int* ticket, int n_tasks, int lds_bytes,
                       int par, int check, int wg, hipStream_t st) {
    hipError_t e = launch_backward<real>(probs, tasks, ticket, n_tasks, lds_bytes, par, check, wg, st);
    if (e != hipSuccess) return e;
    return launch_forward<real>(probs, tasks, ticket, n_tasks, lds_bytes, par, check, wg, st);
}

template <typename real>
hipError_t launch_apply_L(const ProbDev<real>* P, int n, const real* z, real* eta, hipStream_t st) {
    hipLaunchKernelGGL(k_apply_L<real>, dim3(n), dim3(kHookWG), 0, st, P, z, eta);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_apply_Lt(const ProbDev<real>* P, int n, const real* eta, real* z, hipStream_t st) {
    hipLaunchKernelGGL(k_apply_Lt<real>, dim3(n), dim3(kHookWG), 0, st, P, eta, z);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_prox_gconj(const ProbDev<real>* P, int n, const real* w, real* eta, hipStream_t st) {
    hipLaunchKernelGGL(k_prox_gconj<real>, dim3(n), dim3(kHookWG), 0, st, P, w, eta);
    return hipGetLastError();
}

template <typename D, typename S>
hipError_t launch_convert(D* dst, const S* src, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_convert<D, S>), dim3((unsigned)blocks), dim3(256), 0, st, dst, src, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* dst, T val, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, st, dst, val, n);
    return hipGetLastError();
}

#define SPK_INSTANTIATE(real)                                                                              \
    template hipError_t launch_step<real>(const ProbDev<real>*, const int2*, int*, int, int, int, int, int,  \
                                          hipStream_t);                                                    \
    template hipError_t launch_backward<real>(const ProbDev<real>*, const int2*, int*, int, int, int, int, \
                                              int, hipStream_t);                                           \
    template hipError_t launch_forward<real>(const ProbDev<real>*, const int2*, int*, int, int, int, int,  \
                                             int, hipStream_t);                                            \
    template hipError_t launch_apply_L<real>(const ProbDev<real>*, int, const real*, real*, hipStream_t);   \
    template hipError_t launch_apply_Lt<real>(const ProbDev<real>*, int, const real*, real*, hipStream_t);  \
    template hipError_t launch_prox_gconj<real>(const ProbDev<real>*, int, const real*, real*, hipStream_t); \
    template hipError_t launch_fill<real>(real*, real, long long, hipStream_t);

SPK_INSTANTIATE(float)
SPK_INSTANTIATE(double)
template hipError_t launch_convert<float, double>(float*, const double*, long long, hipStream_t);
template hipError_t launch_convert<double, float>(double*, const float*, long long, hipStream_t);
template hipError_t launch_fill<int>(int*, int, long long, hipStream_t);
template hipError_t launch_fill<unsigned long long>(unsigned long long*, unsigned long long, long long,
                                                    hipStream_t);

}  // namespace spk
