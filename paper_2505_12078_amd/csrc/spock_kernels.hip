// gfx950 kernels of one Chambolle-Pock (CP) step of SPOCK on a scenario tree.
//
// One CP step (Sec. 4.1), z+ = prox_{alpha f}(z - alpha L* eta) and
// eta+ = prox_{alpha g*}(eta + alpha L(2 z+ - z)), is four launches:
//
//  prep    one wavefront per node, every node at once.  zbar = z - alpha L* eta
//          on the node's (x, u) (adjoint of L, Sec. 4.4), the S2 projection of
//          the node's (y, tau, s) block (Sec. 4.3), the prox of s0 at the root,
//          and the parts of the reduced S1 recursion that do not depend on the
//          children: h0 = -xbar - K^T ubar (+ P c) and ubar.
//  bsweep  one wavefront per leaf, leaves -> root: the sequential part of the
//          backward recursion of Alg. 2.  g = sum of the children's messages,
//          h = h0 + g_x, d = R~^-1 (ubar - g_u), message [Abar|B]^T h to the
//          parent.  At a node with several children only the wavefront that
//          arrives last continues (atomic counter), so nothing ever waits.
//  fsweep  one wavefront per leaf, root -> leaves: x^j = [Abar^j|B^j][x^i; d^i] + c^j
//          along the whole root-to-leaf path.  Paths share their upper nodes:
//          every wavefront through a node computes the same x^v (same data,
//          same order), and only the one whose leaf is the node's leftmost
//          leaf stores it, so no wavefront waits for another (the shared
//          tiles are read from cache).
//  dual    one wavefront per node: u = K x + d, then every dual block the node
//          owns, eta+ = prox_{alpha g*}(eta + alpha L(2 z+ - z)) with the S3
//          cone projections and Moreau's identity, and on request the
//          residuals xi1, xi2 of Sec. 5.3.
//
// Reduced S1 recursion (algebraically equal to Alg. 2, using
// sum_j Abar^jT P^j B^j = -K^iT, which follows from the definition of K in
// Alg. 1):  with h^j = q^j + P^j c^j and g = sum_{j in ch(i)} [Abar^j|B^j]^T h^j,
//   q^i = -xbar^i - K^iT ubar^i + g_x,   d^i = R~^i^-1 (ubar^i - g_u),
// and forward u^i = K^i x^i + d^i, x^j = Abar^j x^i + B^j d^i + c^j.  Only the
// messages and x pass between tree levels, so the sweeps carry one matrix-vector
// product per level and everything else runs node-parallel.
//
// Matrix products are "column-lane": out[o] = sum_k A[k][o] v[k], each lane
// holding its rows of one output column in registers.  The host packs every
// node matrix in the lane order of its product (one copy per product), so a
// wavefront reads a tile with contiguous 16-byte-per-lane loads.  LDS holds
// node vectors only.

#include <hip/hip_runtime.h>

#include "spock_dev.h"

namespace spk {

constexpr int kHookWG = 256;  // workgroup size of the per-node hook kernels

#define SPK_DEV __device__ __forceinline__

// ---------------------------------------------------------------------------
// wavefront and workgroup helpers
// ---------------------------------------------------------------------------

// Cross-lane moves inside rows of 16 lanes (DPP): CTRL 0xB1 / 0x4E swap lanes
// 1 / 2 apart within quads, 0x141 mirrors each half row, 0x140 each row.
// Every lane of the wavefront must be active.
template <int CTRL>
SPK_DEV float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
SPK_DEV double dpp(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Lane l's value (uniform result).
SPK_DEV float lane_value(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
SPK_DEV double lane_value(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the wavefront in a fixed order, the same value in every lane:
// quads, half rows and rows by DPP, then the four row sums.  Every lane of the
// wavefront must be active.
template <typename T>
SPK_DEV T wave_sum(T v) {
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    v += dpp<0x141>(v);
    v += dpp<0x140>(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Maximum that keeps a NaN from either side (fmax would drop it), so that a
// non-finite iterate gives a non-finite residual and stops the solve.
template <typename T>
SPK_DEV T nmax(T a, T b) {
    return (b > a || b != b) ? b : a;
}

template <typename T>
SPK_DEV T wave_max(T v) {
    v = nmax(v, dpp<0xB1>(v));
    v = nmax(v, dpp<0x4E>(v));
    v = nmax(v, dpp<0x141>(v));
    v = nmax(v, dpp<0x140>(v));
    return nmax(nmax(lane_value(v, 0), lane_value(v, 16)), nmax(lane_value(v, 32), lane_value(v, 48)));
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

// LDS exchange between lanes of one wavefront: the hardware keeps a
// wavefront's LDS accesses in order; this keeps the compiler from moving them.
SPK_DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

SPK_DEV int lane_id() { return (int)(threadIdx.x & 63); }

// The dispatcher hands workgroups to the 8 XCDs in turn (workgroup w to XCD
// w mod 8).  The sweeps renumber them so that each XCD takes one contiguous run
// of the leaf table: neighbouring leaves (one subtree) then share an L2, and the
// tiles of the nodes above them are fetched from HBM once per XCD rather than
// by every XCD.  A bijection of [0, g) for any g.
SPK_DEV int xcd_order(int w, int g) {
    const int per = g >> 3, rem = g & 7, x = w & 7, j = w >> 3;
    return x * per + (x < rem ? x : rem) + j;
}

// Exchange between workgroups of one launch.  A value that another workgroup
// reads while the launch runs is stored and loaded at device scope: the store
// is written through to the level of the memory hierarchy that all XCDs share,
// and the load skips the XCD-private caches.  Before the barrier that precedes
// the counter or flag update, every wavefront drains its vector memory counter,
// so its device-scope stores are complete.  Release/acquire fences would do the
// same job, but at device scope they write back or invalidate the whole L2 of
// the XCD, and that costs tens of microseconds per node when many workgroups
// have stores in flight.
// Global-address-space views: accesses through them compile to global (not
// flat) memory instructions, which only count against the vector memory
// counter, so waits for them stay precise.
template <typename T>
SPK_DEV __attribute__((address_space(1))) T* gm(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}
template <typename T>
SPK_DEV const __attribute__((address_space(1))) T* gm(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}

template <typename T>
SPK_DEV const __attribute__((address_space(3))) T* lds(const T* p) {
    return (const __attribute__((address_space(3))) T*)p;
}

// sum_c H[c][r] x(c) for a symmetric n x n H in global memory: with r the
// lane's row, consecutive lanes read consecutive addresses of row c of H
// (used only by the node kernels built for dense costs, so the loads in
// flight cost the other kernels no registers)
template <typename real, typename X>
SPK_DEV real sym_col_dot(const real* H, int n, int r, X x) {
    real s = 0;
#pragma unroll 16
    for (int c = 0; c < n; ++c) s += gm(H)[(long long)c * n + r] * x(c);
    return s;
}

// the same for two vectors in one pass over H
template <typename real, typename X, typename Y>
SPK_DEV void sym_col_dot2(const real* H, int n, int r, X x, Y y, real& sx, real& sy) {
    real a = 0, b = 0;
#pragma unroll 16
    for (int c = 0; c < n; ++c) {
        const real h = gm(H)[(long long)c * n + r];
        a += h * x(c);
        b += h * y(c);
    }
    sx = a;
    sy = b;
}

template <typename real>
SPK_DEV void st_dev(real* p, real v) {
    __hip_atomic_store(gm(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename real>
SPK_DEV real ld_dev(const real* p) {
    return __hip_atomic_load(gm(const_cast<real*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Every store this wavefront issued has completed (s_waitcnt vmcnt(0)); the
// workgroup fence keeps the compiler from sinking stores below it.
SPK_DEV void drain_stores() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0x0F70);
}

// v >= 0 or NaN: the float64 bit patterns of non-negative values order as the
// values, and a NaN with a clear sign bit orders above +inf, so the slot keeps
// a NaN once any wavefront records one.
template <typename real>
SPK_DEV void record_max(unsigned long long* slot, real v) {
    const double d = v != v ? __longlong_as_double(0x7FF8000000000000LL) : (double)v;
    atomicMax(slot, (unsigned long long)__double_as_longlong(d));
}

// Per-problem diagonal data staged once per workgroup.
template <typename real>
struct Consts {
    const real *qh, *rh, *qnh, *gx, *gu, *gb, *gxN, *gbN, *lo, *hi, *loN, *hiN;
};


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

// ---------------------------------------------------------------------------
// input staging
// ---------------------------------------------------------------------------

// A node's vector inputs come from several arrays (z, eta, probabilities, ...).
// They are copied into LDS with global-to-LDS loads (no registers involved):
// every wavefront issues all of its copies back to back and waits once, so a
// node costs one memory round trip for its vectors, overlapped with the loads
// of its matrix tile.  Slots have fixed positions (uniform values); an empty
// slot has length 0.
template <typename real, int NS>
struct Stage {
    const real* src[NS];
    int len[NS];
    SPK_DEV void set(int q, const real* p, int n) {
        src[q] = p;
        len[q] = n;
    }
};

// Copy n dwords from global memory to LDS, one wavefront; dst uniform.
SPK_DEV void lds_copy(const void* src, void* dst, int ndw) {
    const int lane = lane_id();
    const unsigned* s = static_cast<const unsigned*>(src);
    unsigned* d = static_cast<unsigned*>(dst);
    for (int c = 0; c < ndw; c += 64)
        if (c + lane < ndw)
            __builtin_amdgcn_global_load_lds(s + c + lane, (__attribute__((address_space(3))) void*)(d + c), 4, 0, 0);
}

// Wait for this wavefront's outstanding global loads (global-to-LDS included).
SPK_DEV void wait_loads() {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    wave_sync();
}

// Copy the slots back to back into st (one wavefront); off[q] receives the
// start of slot q.  Completion needs wait_loads().
template <typename real, int NS>
SPK_DEV void gather(const Stage<real, NS>& S, real* st, int* off) {
    int o = 0;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        off[q] = o;
        if (S.len[q] > 0) lds_copy(S.src[q], st + o, S.len[q] * (int)(sizeof(real) / 4));
        o += S.len[q];
    }
}

// The 12 diagonal data arrays of a problem, staged by the whole workgroup.
template <typename real>
SPK_DEV void stage_consts(const ProbDev<real>* __restrict__ P, real* cst) {
    const int nx = P->nx, nu = P->nu, m = P->m;
    Stage<real, 12> S{};
    S.set(0, P->qh, nx);
    S.set(1, P->rh, nu);
    S.set(2, P->qnh, nx);
    S.set(3, P->gx, nx);
    S.set(4, P->gu, nu);
    S.set(5, P->gb, nx);
    S.set(6, P->gxN, nx);
    S.set(7, P->gbN, nx);
    S.set(8, P->lo, m);
    S.set(9, P->hi, m);
    S.set(10, P->loN, nx);
    S.set(11, P->hiN, nx);
    // wavefront w copies the slots q = w, w + waves, ...
    const int waves = (int)(blockDim.x >> 6), w = (int)(threadIdx.x >> 6);
    int o = 0;
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        if (q % waves == w) lds_copy(S.src[q], cst + o, S.len[q] * (int)(sizeof(real) / 4));
        o += S.len[q];
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wavefront's copies are in LDS
    __syncthreads();
}

// ---------------------------------------------------------------------------
// column-lane products (one wavefront)
// ---------------------------------------------------------------------------

// out[o] = sum_{k<K} A[k][o] v[k] for o < O.  Block 1 covers the
// columns 0..W1-1 (W1 = min(O, 64)) with G1 = 64 / W1 row groups: lane
// l = g W1 + c keeps rows g, g + G1, ... of column c.  Block 2 covers the
// columns 64..O-1 the same way with G2 = 64 / (O - 64).  The host stores every
// such matrix pre-packed in exactly that lane order (tile_pack), so a lane
// reads its rows with 16-byte loads at fixed offsets and a wavefront's load
// covers 1 KiB of contiguous memory.  Group partial sums meet in LDS and are
// added in group order (deterministic).
// Wider products (O > 128, more blocks of 64 columns) run from global memory
// (col_direct); W2, G2 and rows2 then describe the full second block.
struct ColShape {
    int K, O, W1, G1, W2, G2, rows1, rows2;  // rows per lane, padded to the vector width
};

template <typename real>
SPK_DEV ColShape col_shape(int K, int O) {
    ColShape s;
    s.K = K;
    s.O = O;
    s.W1 = O < 64 ? O : 64;
    s.G1 = 64 / s.W1;
    s.W2 = O > 64 ? (O - 64 < 64 ? O - 64 : 64) : 0;
    s.G2 = s.W2 > 0 ? 64 / s.W2 : 1;
    s.rows1 = tile_rows(K, s.G1, tile_vec<real>());
    s.rows2 = s.W2 > 0 ? tile_rows(K, s.G2, tile_vec<real>()) : 0;
    // uniform by construction; say so, so that what derives from it stays scalar
    s.K = __builtin_amdgcn_readfirstlane(s.K);
    s.O = __builtin_amdgcn_readfirstlane(s.O);
    s.W1 = __builtin_amdgcn_readfirstlane(s.W1);
    s.G1 = __builtin_amdgcn_readfirstlane(s.G1);
    s.W2 = __builtin_amdgcn_readfirstlane(s.W2);
    s.G2 = __builtin_amdgcn_readfirstlane(s.G2);
    s.rows1 = __builtin_amdgcn_readfirstlane(s.rows1);
    s.rows2 = __builtin_amdgcn_readfirstlane(s.rows2);
    return s;
}

template <typename real, int R>
struct ColTile {
    real a[R];
    real b[R / 4];
};

// 16 bytes as tile_vec<real>() values
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename real>
SPK_DEV void unpack16(u32x4 u, real* dst);
template <>
SPK_DEV void unpack16<float>(u32x4 u, float* dst) {
    dst[0] = __uint_as_float(u.x);
    dst[1] = __uint_as_float(u.y);
    dst[2] = __uint_as_float(u.z);
    dst[3] = __uint_as_float(u.w);
}
template <>
SPK_DEV void unpack16<double>(u32x4 u, double* dst) {
    dst[0] = __hiloint2double((int)u.y, (int)u.x);
    dst[1] = __hiloint2double((int)u.w, (int)u.z);
}

// Every lane loads the full register class unconditionally: the loads past
// the tile's own 1 KiB lane groups repeat its last group (the same addresses,
// so no extra memory traffic), and col_apply masks every row past K.  With no
// conditional loads the compiler can count the loads in flight, so a later
// level's prefetch does not force a wait for everything.
template <typename real, int R>
SPK_DEV void col_load(ColTile<real, R>& T, const real* __restrict__ tile, const ColShape& s) {
    constexpr int V = 16 / (int)sizeof(real);
    const __attribute__((address_space(1))) u32x4* p =
        (const __attribute__((address_space(1))) u32x4*)tile + lane_id();
    const int l1 = s.rows1 / V - 1, l2 = s.rows2 > 0 ? s.rows2 / V - 1 : 0;
#pragma unroll
    for (int q = 0; q < R / V; ++q) {
        const u32x4 u = p[(q < l1 ? q : l1) * 64];
        unpack16<real>(u, T.a + q * V);
    }
    // block 2 (when there is none, the group after block 1, unused)
    p += (s.rows1 / V) * 64;
#pragma unroll
    for (int q = 0; q < R / 4 / V; ++q) {
        const u32x4 u = p[(q < l2 ? q : l2) * 64];
        unpack16<real>(u, T.b + q * V);
    }
}

// 16 bytes of LDS as tile_vec<real>() values
template <typename real>
SPK_DEV void lds16(const real* p, real* dst) {
    const u32x4 u = *reinterpret_cast<const u32x4*>(p);
    unpack16<real>(u, dst);
}

// v: K entries (LDS, 16-byte aligned), out: O entries (LDS), red: kRed
// entries of scratch (LDS).  Rows past the tile's own (rows1 / rows2) repeat
// its last lane group (finite data) and are masked; inside them, entries of
// rows past K and of idle lanes are zero.  kPadded: v is zero from K up to R
// entries, so the one-group block needs no masks (rows past the tile meet
// zeros of v; tile data is finite).  The v values a lane needs are read into
// registers before the products, so the LDS reads issue back to back.
template <bool kPadded, typename real, int R>
SPK_DEV void col_apply(const ColTile<real, R>& T, const ColShape& s, const real* v, real* out, real* red) {
    constexpr int V = 16 / (int)sizeof(real);
    const int lane = lane_id();
    const int km = s.K - 1;
    real acc = 0;
    if (s.G1 == 1) {
        // every lane needs v[i]: broadcast reads
        real x[R];
        if constexpr (kPadded) {
#pragma unroll
            for (int i = 0; i < R; i += V) lds16(v + i, x + i);  // V rows per read
#pragma unroll
            for (int i = 0; i < R; ++i) acc += T.a[i] * x[i];
        } else {
#pragma unroll
            for (int i = 0; i < R; ++i) x[i] = v[i < km ? i : km];
#pragma unroll
            for (int i = 0; i < R; ++i) acc += (i < s.rows1 ? T.a[i] : real(0)) * x[i];
        }
    } else {
        const int g1 = lane / s.W1;
        real x[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int k = g1 + i * s.G1;
            x[i] = v[k < km ? k : km];
        }
#pragma unroll
        for (int i = 0; i < R; ++i) acc += (i < s.rows1 ? T.a[i] : real(0)) * x[i];
    }
    real acc2 = 0;
    if (s.W2 > 0) {
        const int g2 = lane / s.W2;
        real x[R / 4];
#pragma unroll
        for (int i = 0; i < R / 4; ++i) {
            const int k = g2 + i * s.G2;
            x[i] = v[k < km ? k : km];
        }
#pragma unroll
        for (int i = 0; i < R / 4; ++i) acc2 += (i < s.rows2 ? T.b[i] : real(0)) * x[i];
    }
    red[lane] = acc;
    red[64 + lane] = acc2;
    wave_sync();
    if (lane < s.W1) {
        real t = 0;
        for (int g = 0; g < s.G1; ++g) t += red[g * s.W1 + lane];
        out[lane] = t;
    }
    if (lane < s.W2) {
        real t = 0;
        for (int g = 0; g < s.G2; ++g) t += red[64 + g * s.W2 + lane];
        out[64 + lane] = t;
    }
    wave_sync();
}

// The same product read from the packed tile in global memory (shapes beyond
// the register class, and products of any width: one 64-column block after
// the other, block b at columns 64 b ..).  kWide (the launches of problems whose
// products fit no register class): a lane keeps kU = 16 16-byte row groups of its
// column in flight; otherwise one row at a time, four in flight, so that the
// fallback adds few registers to kernels that rarely take it.  Both sum a
// lane's rows in row order.
template <bool kWide, typename real>
SPK_DEV void col_direct(const real* __restrict__ tile, const ColShape& s, const real* v, real* out, real* red) {
    constexpr int V = 16 / (int)sizeof(real);
    const int lane = lane_id();
    auto part = [&](const real* blk, int rows, int W, int G) {
        const int g = lane / W;
        real acc = 0;
        if constexpr (kWide) {
            constexpr int kU = 16;
            const int nv = rows / V;  // rows are a multiple of V
            const __attribute__((address_space(1))) u32x4* p =
                (const __attribute__((address_space(1))) u32x4*)blk + lane;
            for (int q0 = 0; q0 < nv; q0 += kU) {
                real buf[kU * V];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int q = q0 + u < nv ? q0 + u : nv - 1;  // stays inside the block
                    unpack16<real>(p[(long long)q * 64], buf + u * V);
                }
#pragma unroll
                for (int e = 0; e < kU * V; ++e) {
                    const int i = q0 * V + e, k = g + i * G;
                    if (i < rows && k < s.K) acc += buf[e] * v[k];
                }
            }
        } else {
#pragma unroll 4
            for (int i = 0; i < rows; ++i) {
                const int k = g + i * G;
                if (k < s.K) acc += blk[((i / V) * 64 + lane) * V + (i % V)] * v[k];
            }
        }
        return acc;
    };
    const int nb = tile_blocks(s.O);
    const real* blk = tile;
    for (int b = 0; b < nb; ++b) {
        const int W = tile_block_width(s.O, b), G = 64 / W, rows = tile_rows(s.K, G, V);
        red[lane] = part(blk, rows, W, G);
        wave_sync();
        if (lane < W) {
            real t = 0;
            for (int g = 0; g < G; ++g) t += red[g * W + lane];
            out[64 * b + lane] = t;
        }
        wave_sync();
        blk += (long long)rows * 64;
    }
}

// A tile of class R if the shape fits it, else the product runs from the
// packed tile in global memory.
template <typename real, int R>
struct ColProd {
    ColTile<real, R> T;
    ColShape s;
    const real* tile;
    bool fit;
    SPK_DEV void load(const real* t, const ColShape& sh) {
        tile = t;
        s = sh;
        fit = sh.O <= 128 && sh.rows1 <= R && sh.rows2 <= R / 4;
        col_load(T, t, sh);  // unconditional (see col_load); unused when !fit
    }
    // staged form: the tile from LDS (st) once its copy has landed
    SPK_DEV void take(const real* t, const ColShape& sh, const real* st) {
        tile = t;
        s = sh;
        fit = sh.O <= 128 && sh.rows1 <= R && sh.rows2 <= R / 4;
        if (fit) col_take(T, st, sh);
    }
    // kPadded: v is zero from K up to kVecPad entries (see col_apply)
    template <bool kPadded = false>
    SPK_DEV void apply(const real* v, real* out, real* red) const {
        if (fit) col_apply<kPadded>(T, s, v, out, red);
        else col_direct<R == kWideClass>(tile, s, v, out, red);
    }
};

// ---------------------------------------------------------------------------
// dual blocks
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

// Entry r of the translation a of Prop. 1 for an SOC block of length len:
// the stored per-block vector with linear cost terms, else (0, .., 1/2, -1/2).
template <typename real>
SPK_DEV real soc_shift_at(const real* a, int r, int len) {
    if (a) return a[r];
    return r == len - 2 ? real(0.5) : (r == len - 1 ? real(-0.5) : real(0));
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

// General constraint rows G [x; u] in a box (one wavefront): G S^-1 / a as
// Gt (rows) and GtT (columns), ncol = nx + nu columns, or ncol = nx at a leaf
// (u unused); the box bounds in global memory.  lxw, luw gather G^T of the
// dual change for the residual.
template <typename real>
SPK_DEV void fwd_block_gen(const real* Gt, const real* GtT, int nr, int nx, int ncol, const real* lo,
                           const real* hi, long long off, const real* ec, const real* xn, const real* xo,
                           const real* un, const real* uo, real alpha, real* dblk, real* lxw, real* luw,
                           real* __restrict__ eout, int check, real& r2) {
    const int lane = threadIdx.x & 63;
    const real ialpha = real(1) / alpha;
    for (int r = lane; r < nr; r += 64) {
        real wn = 0, wo = 0;
#pragma unroll 4
        for (int c = 0; c < ncol; ++c) {
            const real g = gm(GtT)[(long long)c * nr + r];
            wn += g * (c < nx ? xn[c] : un[c - nx]);
            wo += g * (c < nx ? xo[c] : uo[c - nx]);
        }
        const real eb = ec[r] + alpha * (real(2) * wn - wo);
        const real ep = moreau_box(eb, alpha, gm(lo)[r], gm(hi)[r]);
        gm(eout)[off + r] = ep;
        const real de = ec[r] - ep;
        if (check) r2 = nmax(r2, fabs(de * ialpha - (wo - wn)));
        dblk[r] = de;
    }
    if (check) {
        wave_sync();
        for (int c = lane; c < ncol; c += 64) {
            real s = 0;
#pragma unroll 4
            for (int r = 0; r < nr; ++r) s += gm(Gt)[(long long)r * ncol + c] * dblk[r];
            if (c < nx) lxw[c] += s;
            else luw[c - nx] += s;
        }
    }
}

// eta_c of non-leaf node v: C^i = box x ball (one wavefront).  ec: staged eta_c.
template <typename real, int kMode>
SPK_DEV void fwd_block_c(const ProbDev<real>* __restrict__ P, int v, const real* ec, real* __restrict__ eout,
                         const FwdNode<real>& V, int check, real& r2) {
    const int lane = threadIdx.x & 63;
    const int nx = P->nx, nbox = P->nbox, nc = P->nc;
    const real alpha = P->alpha, ialpha = real(1) / alpha;
    const long long off = P->e_c + (long long)v * nc;
    if (kMode == 2 && P->Gt) {
        fwd_block_gen(P->Gt, P->GtT, nc, nx, P->m, P->lo, P->hi, off, ec, V.xn, V.xo, V.un, V.uo, alpha, V.dblk,
                      V.lxw, V.luw, eout, check, r2);
        return;
    }
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
        gm(eout)[off + r] = ep;
        const real de = ec[r] - ep;
        if (check) r2 = nmax(r2, fabs(de * ialpha - V.dblk[r]));
        V.dblk[r] = de;
    }
    if (check) {
        wave_sync();
        for (int r = lane; r < nx; r += 64) {
            real s = V.C.gx[r] * V.dblk[r];
            if (P->has_ball) s += V.C.gb[r] * V.dblk[nbox + r];
            V.lxw[r] += s;
        }
        for (int r = lane; r < P->nu; r += 64) V.luw[r] += V.C.gu[r] * V.dblk[nx + r];
    }
}

// eta_y in (K^i)* = R^{2k}_+ x R and eta_s in R_+ (one wavefront), from staged
// eta_y (ey), eta_s (es), new and old y (yn, yv) and s (sn, sv), probabilities p;
// yo: start of y^v in the y block.
template <typename real, typename PT>
SPK_DEV void fwd_block_risk(const ProbDev<real>* __restrict__ P, int v, long long yo, int k, PT ey, real es,
                            PT yn, PT yv, real sn, real sv, PT p,
                            real* __restrict__ eout, int check, real& r1, real& r2) {
    const int lane = threadIdx.x & 63;
    const real alpha = P->alpha, ialpha = real(1) / alpha;
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
    if (lane == 0) gm(eout)[P->e_s + v] = eps_;
    for (int c = lane; c < 2 * k + 1; c += 64) {
        const real eb = ey[c] + alpha * (real(2) * yn[c] - yv[c]);
        const real ep = c < 2 * k ? (eb < 0 ? eb : real(0)) : real(0);
        gm(eout)[P->e_y + yo + c] = ep;
        if (check) {
            const real de = ey[c] - ep;
            const real dy = yv[c] - yn[c];
            r2 = nmax(r2, fabs(de * ialpha - dy));
            const real bc = c < k ? p[c] : (c == 2 * k ? real(1) : real(0));
            r1 = nmax(r1, fabs(dy * ialpha - (de - bc * des)));
        }
    }
    if (check && lane == 0) {
        r2 = nmax(r2, fabs(des * ialpha - (wso - wsn)));
        r1 = nmax(r1, fabs((sv - sn) * ialpha - des));
    }
}

// The conic data of a general coherent risk at non-leaf node v (Sec. 3.3, K
// polyhedral): y^v has ny entries, nu^v has nnu; the node's packed block holds
// E (ny x k, row-major), F (ny x nnu), b (ny), the cone codes of K's rows (ny;
// 0: R_+, 1: {0}) and M = (G G^T)^-1 ((k + nnu)^2) of G = [E^T -I -I; F^T 0 0].
template <typename real>
struct RiskData {
    int ny, nnu;
    const real *E, *F, *b, *cone, *M;
};
template <typename real>
SPK_DEV RiskData<real> risk_data(const ProbDev<real>* __restrict__ P, int v, int k) {
    RiskData<real> d;
    d.ny = P->rny[v];
    d.nnu = P->rnnu[v];
    d.E = P->rdata + P->roff[v];
    d.F = d.E + (long long)d.ny * k;
    d.b = d.F + (long long)d.ny * d.nnu;
    d.cone = d.b + d.ny;
    d.M = d.cone + d.ny;
    return d;
}

// fwd_block_risk for a general coherent risk: eta_y in (K^v)* row by row (R_+
// where K^v is R_+, R where it is {0}) and eta_s in R_+, with the node's b.
template <typename real, typename PT>
SPK_DEV void fwd_block_risk_gen(const ProbDev<real>* __restrict__ P, int v, long long yo, int k, PT ey, real es,
                                PT yn, PT yv, real sn, real sv, real* __restrict__ eout, int check, real& r1,
                                real& r2) {
    const int lane = threadIdx.x & 63;
    const real alpha = P->alpha, ialpha = real(1) / alpha;
    const RiskData<real> D = risk_data(P, v, k);
    real bn = 0, bo = 0;
    for (int c = lane; c < D.ny; c += 64) {
        const real bc = gm(D.b)[c];
        bn += bc * yn[c];
        bo += bc * yv[c];
    }
    bn = wave_sum(bn);
    bo = wave_sum(bo);
    const real wsn = sn - bn, wso = sv - bo;
    const real ebs = es + alpha * (real(2) * wsn - wso);
    const real eps_ = ebs < 0 ? ebs : real(0);
    const real des = es - eps_;
    if (lane == 0) gm(eout)[P->e_s + v] = eps_;
    // eta_y+ = ebar - P_{K*}(ebar) on the rows of y (lanes r and r + 64):
    // R_+ rows min(ebar, 0), {0} rows 0, and each second-order cone block
    // (head row code 2, its w rows coded -1 - head) ebar minus its projection
    // onto the (self-dual) cone
    real eb[2], cd[2], ep[2];
    for (int h = 0; h < 2; ++h) {
        const int c = lane + 64 * h;
        eb[h] = c < D.ny ? ey[c] + alpha * (real(2) * yn[c] - yv[c]) : real(0);
        cd[h] = c < D.ny ? gm(D.cone)[c] : real(1);
        ep[h] = cd[h] == real(0) ? (eb[h] < 0 ? eb[h] : real(0)) : real(0);
    }
    for (int half = 0; half < 2; ++half) {
        unsigned long long heads = __ballot(cd[half] == real(2));
        while (heads) {
            const int hr = 64 * half + __ffsll((long long)heads) - 1;
            heads &= heads - 1;
            const real tag = real(-1 - hr);
            real w2 = 0;
            for (int h = 0; h < 2; ++h)
                if (cd[h] == tag) w2 += eb[h] * eb[h];
            w2 = wave_sum(w2);
            const real t = lane_value(half ? eb[1] : eb[0], hr & 63), nw = sqrt(w2);
            real ct, cw;  // projection: head ct, w rows cw * w
            if (nw <= t) {
                ct = t;
                cw = real(1);
            } else if (nw <= -t) {
                ct = real(0);
                cw = real(0);
            } else {
                ct = real(0.5) * (t + nw);
                cw = ct / nw;
            }
            for (int h = 0; h < 2; ++h) {
                if (lane + 64 * h == hr) ep[h] = eb[h] - ct;
                else if (cd[h] == tag) ep[h] = eb[h] - cw * eb[h];
            }
        }
    }
    for (int h = 0; h < 2; ++h) {
        const int c = lane + 64 * h;
        if (c >= D.ny) continue;
        gm(eout)[P->e_y + yo + c] = ep[h];
        if (check) {
            const real de = ey[c] - ep[h];
            const real dy = yv[c] - yn[c];
            r2 = nmax(r2, fabs(de * ialpha - dy));
            r1 = nmax(r1, fabs(dy * ialpha - (de - gm(D.b)[c] * des)));
        }
    }
    if (check && lane == 0) {
        r2 = nmax(r2, fabs(des * ialpha - (wso - wsn)));
        r1 = nmax(r1, fabs((sv - sn) * ialpha - des));
    }
}

// SOC block of the edge into child j of non-leaf node v:
// (Q^1/2 x^v, R^1/2 u^v, tau^j / 2, tau^j / 2) in SOC + a (one wavefront);
// es: staged eta_soc of that edge, tn / tv: new / old tau^j.
template <typename real, int kMode, typename PT>
SPK_DEV void fwd_block_soc(const ProbDev<real>* __restrict__ P, int j, PT es, real tn, real tv,
                           real* __restrict__ eout, const FwdNode<real>& V, int check, real& r1, real& r2) {
    const int lane = threadIdx.x & 63;
    const int nx = P->nx, m = P->m;
    const real alpha = P->alpha, ialpha = real(1) / alpha;
    const long long off = P->e_soc + (long long)(j - 1) * (m + 2);
    const real* aj = P->sa ? P->sa + (long long)(j - 1) * (m + 2) : nullptr;
    // the edge's cost square roots: its own, or the shared ones staged in LDS
    const real* qe = P->qh_e ? P->qh_e + (long long)j * nx : nullptr;
    const real* re = P->rh_e ? P->rh_e + (long long)j * P->nu : nullptr;
    auto qh = [&](int r) { return qe ? gm(qe)[r] : V.C.qh[r]; };
    auto rh = [&](int r) { return re ? gm(re)[r] : V.C.rh[r]; };
    // dense costs: the cost rows H (S^-1 x) of the new and old iterate, first
    // into blk / dblk
    const real* Hq = kMode >= 1 && P->Hq_e ? P->Hq_e + (long long)j * nx * nx : nullptr;
    const real* Hr = kMode >= 1 && P->Hr_e ? P->Hr_e + (long long)j * P->nu * P->nu : nullptr;
    if (Hq) {
        wave_sync();
        for (int r = lane; r < nx; r += 64)
            sym_col_dot2(
                Hq, nx, r, [&](int c) { return V.C.qh[c] * V.xn[c]; }, [&](int c) { return V.C.qh[c] * V.xo[c]; },
                V.blk[r], V.dblk[r]);
        for (int r = lane; r < P->nu; r += 64)
            sym_col_dot2(
                Hr, P->nu, r, [&](int c) { return V.C.rh[c] * V.un[c]; },
                [&](int c) { return V.C.rh[c] * V.uo[c]; }, V.blk[nx + r], V.dblk[nx + r]);
        wave_sync();
    }
    // Prop. 1 with R singular: the tau rows are (tau - c_j^T u) / 2
    real cun = 0, cuo = 0;
    if (kMode == 2 && P->ck) {
        const real* cj = P->ck + (long long)j * P->nu;
        for (int r = lane; r < P->nu; r += 64) {
            cun += gm(cj)[r] * V.un[r];
            cuo += gm(cj)[r] * V.uo[r];
        }
        cun = wave_sum(cun);
        cuo = wave_sum(cuo);
    }
    real nw2 = 0;
    for (int r = lane; r < m + 2; r += 64) {
        real wn, wo;
        if (Hq && r < m) {
            wn = V.blk[r];
            wo = V.dblk[r];
        } else if (r < nx) {
            wn = qh(r) * V.xn[r];
            wo = qh(r) * V.xo[r];
        } else if (r < m) {
            wn = rh(r - nx) * V.un[r - nx];
            wo = rh(r - nx) * V.uo[r - nx];
        } else {
            wn = real(0.5) * (tn - cun);
            wo = real(0.5) * (tv - cuo);
        }
        real eb = es[r] + alpha * (real(2) * wn - wo);
        eb -= alpha * soc_shift_at(aj, r, m + 2);  // v = etabar - alpha a
        V.blk[r] = eb;
        V.dblk[r] = wo - wn;
        if (r <= m) nw2 += eb * eb;
    }
    nw2 = wave_sum(nw2);
    wave_sync();
    real cw, ct;
    soc_moreau_coef(nw2, V.blk[m + 1], cw, ct);
    for (int r = lane; r < m + 2; r += 64) {
        const real ep = r <= m ? V.blk[r] * cw : ct;
        gm(eout)[off + r] = ep;
        const real de = es[r] - ep;
        if (check) r2 = nmax(r2, fabs(de * ialpha - V.dblk[r]));
        V.dblk[r] = de;
    }
    if (check) {
        wave_sync();
        if (Hq) {
            for (int r = lane; r < nx; r += 64)
                V.lxw[r] += V.C.qh[r] * sym_col_dot(Hq, nx, r, [&](int c) { return V.dblk[c]; });
            for (int r = lane; r < P->nu; r += 64)
                V.luw[r] += V.C.rh[r] * sym_col_dot(Hr, P->nu, r, [&](int c) { return V.dblk[nx + c]; });
        } else {
            for (int r = lane; r < nx; r += 64) V.lxw[r] += qh(r) * V.dblk[r];
            for (int r = lane; r < P->nu; r += 64) V.luw[r] += rh(r) * V.dblk[nx + r];
        }
        if (kMode == 2 && P->ck) {
            const real h = real(0.5) * (V.dblk[m] + V.dblk[m + 1]);
            for (int r = lane; r < P->nu; r += 64) V.luw[r] -= gm(P->ck)[(long long)j * P->nu + r] * h;
        }
        if (lane == 0) r1 = nmax(r1, fabs((tv - tn) * ialpha - real(0.5) * (V.dblk[m] + V.dblk[m + 1])));
    }
}

// Leaf v: eta_cN (box x ball) for which = 0, eta_socN (Q_N^1/2 x, s/2, s/2) for
// which = 1 (one wavefront each); ec / es: the staged blocks.
template <typename real, int kMode>
SPK_DEV void fwd_block_leaf(const ProbDev<real>* __restrict__ P, int v, int which, const real* ec,
                            const real* es, real sn, real sv, real* __restrict__ eout, const FwdNode<real>& V,
                            int check, real& r1, real& r2) {
    const int lane = threadIdx.x & 63;
    const int nx = P->nx;
    const real alpha = P->alpha, ialpha = real(1) / alpha;
    const long long lf = v - P->n_nl;
    if (which == 0) {
        const long long off = P->e_cN + lf * P->ncN;
        if (kMode == 2 && P->GNt) {
            fwd_block_gen(P->GNt, P->GNtT, P->ncN, nx, nx, P->loN, P->hiN, off, ec, V.xn, V.xo, V.xn, V.xo,
                          alpha, V.dblk, V.lxw, V.lxw, eout, check, r2);
            return;
        }
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
            gm(eout)[off + r] = ep;
            const real de = ec[r] - ep;
            if (check) r2 = nmax(r2, fabs(de * ialpha - V.dblk[r]));
            V.dblk[r] = de;
        }
        if (check) {
            wave_sync();
            for (int r = lane; r < nx; r += 64) {
                real s = V.C.gxN[r] * V.dblk[r];
                if (P->has_ballN) s += V.C.gbN[r] * V.dblk[nx + r];
                V.lxw[r] += s;
            }
        }
    } else {
        const long long off = P->e_socN + lf * (nx + 2);
        const real* aj = P->saN ? P->saN + lf * (nx + 2) : nullptr;
        const real* qe = P->qnh_l ? P->qnh_l + lf * nx : nullptr;
        auto qnh = [&](int r) { return qe ? gm(qe)[r] : V.C.qnh[r]; };
        const real* Hq = kMode >= 1 && P->HqN_l ? P->HqN_l + lf * nx * nx : nullptr;
        if (Hq) {
            for (int r = lane; r < nx; r += 64)
                sym_col_dot2(
                    Hq, nx, r, [&](int c) { return V.C.qnh[c] * V.xn[c]; },
                    [&](int c) { return V.C.qnh[c] * V.xo[c]; }, V.blk[r], V.dblk[r]);
        }
        real nw2 = 0;
        for (int r = lane; r < nx + 2; r += 64) {
            real wn, wo;
            if (Hq && r < nx) {
                wn = V.blk[r];
                wo = V.dblk[r];
            } else if (r < nx) {
                wn = qnh(r) * V.xn[r];
                wo = qnh(r) * V.xo[r];
            } else {
                wn = real(0.5) * sn;
                wo = real(0.5) * sv;
            }
            real eb = es[r] + alpha * (real(2) * wn - wo);
            eb -= alpha * soc_shift_at(aj, r, nx + 2);
            V.blk[r] = eb;
            V.dblk[r] = wo - wn;
            if (r <= nx) nw2 += eb * eb;
        }
        nw2 = wave_sum(nw2);
        wave_sync();
        real cw, ct;
        soc_moreau_coef(nw2, V.blk[nx + 1], cw, ct);
        for (int r = lane; r < nx + 2; r += 64) {
            const real ep = r <= nx ? V.blk[r] * cw : ct;
            gm(eout)[off + r] = ep;
            const real de = es[r] - ep;
            if (check) r2 = nmax(r2, fabs(de * ialpha - V.dblk[r]));
            V.dblk[r] = de;
        }
        if (check) {
            wave_sync();
            for (int r = lane; r < nx; r += 64)
                V.lxw[r] += Hq ? V.C.qnh[r] * sym_col_dot(Hq, nx, r, [&](int c) { return V.dblk[c]; })
                               : qnh(r) * V.dblk[r];
            if (lane == 0) r1 = nmax(r1, fabs((sv - sn) * ialpha - real(0.5) * (V.dblk[nx] + V.dblk[nx + 1])));
        }
    }
}

// ---------------------------------------------------------------------------
// prep: node-parallel part of the backward half-step
// ---------------------------------------------------------------------------

// One wavefront per node; the workgroup's wavefronts take consecutive entries
// of the node task table, which never mixes problems inside one workgroup
// (entries with node -1 pad a problem to a multiple of kMaxNodeWaves).
template <typename real, int R, int kMode>
__global__ __launch_bounds__(512) void k_prep(const ProbDev<real>* __restrict__ probs,
                                              const int2* __restrict__ ntasks, const int4* __restrict__ ninfo,
                                              int wave_elems, int par, int check) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real* sm = reinterpret_cast<real*>(smem_raw);
    const int waves = (int)(blockDim.x >> 6), w = (int)(threadIdx.x >> 6), lane = lane_id();
    const int2 t0 = ntasks[blockIdx.x * waves];
    // this wavefront's node and its first child, children, y offset (loaded
    // with the task, not after it)
    const int v = ntasks[blockIdx.x * waves + w].y;
    const int4 ni = ninfo[blockIdx.x * waves + w];
    const ProbDev<real>* __restrict__ P = probs + t0.x;
    if (*P->active == 0) return;  // uniform over the workgroup
    const int nx = P->nx, nu = P->nu, m = P->m, nc = P->nc, ncN = P->ncN, nbox = P->nbox, n_nl = P->n_nl;
    real* cst = sm;
    stage_consts(P, cst);
    if (v < 0) return;
    const Consts<real> C = consts_at<real>(cst, nx, nu);
    const real alpha = P->alpha;
    const real* __restrict__ zin = P->z[par];
    const real* __restrict__ ein = P->eta[par];
    real* __restrict__ zout = P->z[par ^ 1];
    real* red = cst + consts_elems(nx, nu) + w * wave_elems;
    real* xb = red + kRed;
    real* ub = xb + round4(nx);  // 16-byte aligned: the K^T ubar product reads it in vectors
    real* tk = ub + round4(nu);
    real* st = red + kRed + node_head_elems(nx, nu, nc, ncN);
    // vectors are read in 16-byte groups: their padding must hold finite values
    for (int e = lane; e < kRed + node_head_elems(nx, nu, nc, ncN); e += 64) red[e] = real(0);
    wave_sync();

    if (v < n_nl) {
        const int fc = ni.x, k = ni.y;
        const long long yo = ni.z;
        const bool leafkids = fc >= n_nl;
        const bool sk = k <= kStageKids && k <= P->stage_kids;  // per-child inputs staged, else read in place
        const int kk = sk ? k : 0;
        // K^T ubar: rows r < nu of [K | R~^-1], columns c < nx
        ColProd<real, R> TK;
        TK.load(P->T1 + v * P->T1_stride, col_shape<real>(nu, nx));
        const real* g_soc = ein + P->e_soc + (long long)(fc - 1) * (m + 2);
        const real* g_cs = leafkids ? ein + P->e_socN + (long long)(fc - n_nl) * (nx + 2) : ein + P->e_s + fc;
        Stage<real, 12> S{};
        S.set(0, zin + P->z_x + (long long)v * nx, nx);
        S.set(1, zin + P->z_u + (long long)v * nu, nu);
        S.set(2, ein + P->e_c + (long long)v * nc, nc);
        S.set(3, g_soc, kk * (m + 2));
        S.set(4, ein + P->e_y + yo, sk ? 2 * k + 1 : 0);
        S.set(5, ein + P->e_s + v, 1);
        S.set(6, zin + P->z_y + yo, sk ? 2 * k + 1 : 0);
        S.set(7, zin + P->z_tau + fc - 1, kk);
        S.set(8, zin + P->z_s + fc - 1, kk);
        S.set(9, g_cs, leafkids ? kk * (nx + 2) : kk);
        S.set(10, P->prob + fc, kk);
        S.set(11, P->affine ? P->Pc + (long long)v * nx : nullptr, (P->affine && v > 0) ? nx : 0);
        int off[12];
        gather(S, st, off);
        wait_loads();
        const real* sx = st + off[0];
        const real* su = st + off[1];
        const real* ec = st + off[2];
        const real es = st[off[5]];
        const real* spc = st + off[11];
        // per-child inputs: the staged copies, or for a wide node the arrays
        // themselves, each through a pointer of its own address space
        auto per_child = [&](auto soc, auto ey, auto zy, auto zt, auto zs, auto cs, auto pr) {
        // zbar on (x^v, u^v): L* gathers the constraint rows and the SOC rows
        // of every child edge (Sec. 4.4)
        for (int r = lane; r < nx; r += 64) {
            real s = 0;
            if (kMode >= 1 && P->Hq_e) {  // dense: S^-1 sum over child edges of H^j eta^j
                for (int q = 0; q < k; ++q)
                    s += sym_col_dot(P->Hq_e + (long long)(fc + q) * nx * nx, nx, r,
                                     [&](int c) { return soc[q * (m + 2) + c]; });
                s *= C.qh[r];
            } else if (P->qh_e) {  // each child edge's own Q^1/2
                for (int q = 0; q < k; ++q) s += gm(P->qh_e)[(long long)(fc + q) * nx + r] * soc[q * (m + 2) + r];
            } else {
                for (int q = 0; q < k; ++q) s += soc[q * (m + 2) + r];
                s *= C.qh[r];
            }
            real lt;
            if (kMode == 2 && P->Gt) {  // general rows: (G^T eta_c) on x
                lt = s;
                for (int q = 0; q < nc; ++q) lt += gm(P->Gt)[(long long)q * m + r] * ec[q];
            } else {
                lt = C.gx[r] * ec[r] + s;
                if (P->has_ball) lt += C.gb[r] * ec[nbox + r];
            }
            xb[r] = sx[r] - alpha * lt;
        }
        for (int r = lane; r < nu; r += 64) {
            real s = 0;
            if (kMode >= 1 && P->Hr_e) {
                for (int q = 0; q < k; ++q)
                    s += sym_col_dot(P->Hr_e + (long long)(fc + q) * nu * nu, nu, r,
                                     [&](int c) { return soc[q * (m + 2) + nx + c]; });
                s *= C.rh[r];
            } else if (P->rh_e) {
                for (int q = 0; q < k; ++q)
                    s += gm(P->rh_e)[(long long)(fc + q) * nu + r] * soc[q * (m + 2) + nx + r];
            } else {
                for (int q = 0; q < k; ++q) s += soc[q * (m + 2) + nx + r];
                s *= C.rh[r];
            }
            if (kMode == 2 && P->ck)  // each child edge's tau rows: -(c_j^T u) / 2 twice
                for (int q = 0; q < k; ++q)
                    s -= real(0.5) * gm(P->ck)[(long long)(fc + q) * nu + r] *
                         (soc[q * (m + 2) + m] + soc[q * (m + 2) + m + 1]);
            real lt;
            if (kMode == 2 && P->Gt) {
                lt = s;
                for (int q = 0; q < nc; ++q) lt += gm(P->Gt)[(long long)q * m + nx + r] * ec[q];
            } else {
                lt = C.gu[r] * ec[nx + r] + s;
            }
            ub[r] = su[r] - alpha * lt;
        }
        // S2 projection (Sec. 4.3) of (y^v, tau^[v], s^[v]) after the
        // z - alpha L* eta shift, general coherent risk: G w = (E^T y - tau - s,
        // F^T y) with one row per lane (k + nnu <= 64), lambda = M G w, and
        // w - G^T lambda = (y - E lambda_E - F lambda_F, tau + lambda_E, s + lambda_E).
        // Rows of y sit on lanes r and r + 64 (ny <= 128); every sum over rows
        // or multipliers runs in index order with the other side broadcast.
        if (kMode == 2 && P->rdata) {
            const RiskData<real> D = risk_data(P, v, k);
            const int g = k + D.nnu;
            real ybh[2];
            for (int h = 0; h < 2; ++h) {
                const int r = lane + 64 * h;
                ybh[h] = r < D.ny ? zy[r] - alpha * (ey[r] - gm(D.b)[r] * es) : real(0);
            }
            real tb = 0, sb = 0;
            if (lane < k) {
                tb = zt[lane] - alpha * real(0.5) * (soc[lane * (m + 2) + m] + soc[lane * (m + 2) + m + 1]);
                const real lts = leafkids ? real(0.5) * (cs[lane * (nx + 2) + nx] + cs[lane * (nx + 2) + nx + 1])
                                          : cs[lane];
                sb = zs[lane] - alpha * lts;
            }
            real rho = 0;
            for (int r = 0; r < D.ny; ++r) {
                const real yr = lane_value(r < 64 ? ybh[0] : ybh[1], r & 63);
                if (lane < k) rho += gm(D.E)[(long long)r * k + lane] * yr;
                else if (lane < g) rho += gm(D.F)[(long long)r * D.nnu + lane - k] * yr;
            }
            if (lane < k) rho -= tb + sb;
            real lam = 0;
            for (int d = 0; d < g; ++d) {
                const real rd = lane_value(rho, d);
                if (lane < g) lam += gm(D.M)[(long long)d * g + lane] * rd;  // M is symmetric
            }
            if (lane < k) {
                gm(zout)[P->z_tau + fc + lane - 1] = tb + lam;
                gm(zout)[P->z_s + fc + lane - 1] = sb + lam;
            }
            real acc[2] = {ybh[0], ybh[1]};
            for (int c = 0; c < g; ++c) {
                const real lc = lane_value(lam, c);
                for (int h = 0; h < 2; ++h) {
                    const int r = lane + 64 * h;
                    if (r < D.ny)
                        acc[h] -= (c < k ? gm(D.E)[(long long)r * k + c] : gm(D.F)[(long long)r * D.nnu + c - k]) * lc;
                }
            }
            for (int h = 0; h < 2; ++h) {
                const int r = lane + 64 * h;
                if (r < D.ny) gm(zout)[P->z_y + yo + r] = acc[h];
            }
        } else
        // AV@R: the kernel of G = [E^T, -I, -I] with
        // E = [gamma I; -I; 1^T] (AV@R, Sec. 3.3); G G^T = (gamma^2 + 3) I + 1 1^T,
        // so with rho = G w the multiplier is lambda = (rho - (1^T rho / (c + n)) 1) / c,
        // c = gamma^2 + 3 (Sherman-Morrison), and w - G^T lambda is the projection.
        {
            const real gam = P->gamma[v], cc = gam * gam + real(3);
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
                rsum += gam * yb1 - yb2 + yb3 - tb - sb;
            }
            rsum = wave_sum(rsum);
            real lsum = 0;
            for (int c = lane; c < k; c += 64) {
                real yb1, yb2, tb, sb;
                shifted(c, yb1, yb2, tb, sb);
                const real rho = gam * yb1 - yb2 + yb3 - tb - sb;
                const real l = (rho - rsum / (cc + real(k))) / cc;
                lsum += l;
                gm(zout)[P->z_y + yo + c] = yb1 - gam * l;
                gm(zout)[P->z_y + yo + k + c] = yb2 + l;
                gm(zout)[P->z_tau + fc + c - 1] = tb + l;
                gm(zout)[P->z_s + fc + c - 1] = sb + l;
            }
            lsum = wave_sum(lsum);
            if (lane == 0) gm(zout)[P->z_y + yo + 2 * k] = yb3 - lsum;
        }
        };
        if (sk)
            per_child(lds(st + off[3]), lds(st + off[4]), lds(st + off[6]), lds(st + off[7]), lds(st + off[8]),
                      lds(st + off[9]), lds(st + off[10]));
        else
            per_child(gm(g_soc), gm(ein + P->e_y + yo), gm(zin + P->z_y + yo), gm(zin + P->z_tau + fc - 1),
                      gm(zin + P->z_s + fc - 1), gm(g_cs), gm(P->prob + fc));
        wave_sync();
        // h0 = -xbar - K^T ubar (+ P c)
        TK.apply(ub, tk, red);
        for (int r = lane; r < nx; r += 64) {
            real h = -xb[r] - tk[r];
            if (P->affine && v > 0) h += spc[r];
            gm(P->h0)[(long long)v * nx + r] = h;
        }
        for (int r = lane; r < nu; r += 64) gm(P->ub)[(long long)v * nu + r] = ub[r];
        if (v == 0 && lane == 0) gm(zout)[0] = zin[0] - alpha * es - alpha;  // prox of alpha * s0
        if (v == 0 && check)
            for (int e = lane; e < 2 * kResSlots; e += 64) gm(P->res)[e] = 0ull;
    } else {
        // leaf: h0 = -xbar (+ P c) with xbar = x - alpha L* eta on x
        const long long lf = v - n_nl;
        Stage<real, 4> S{};
        S.set(0, zin + P->z_x + (long long)v * nx, nx);
        S.set(1, ein + P->e_cN + lf * ncN, ncN);
        S.set(2, ein + P->e_socN + lf * (nx + 2), nx + 2);
        S.set(3, P->affine ? P->Pc + (long long)v * nx : nullptr, P->affine ? nx : 0);
        int off[4];
        gather(S, st, off);
        wait_loads();
        const real* sx = st + off[0];
        const real* sc = st + off[1];
        const real* ss = st + off[2];
        const real* spc = st + off[3];
        for (int r = lane; r < nx; r += 64) {
            const real cost = kMode >= 1 && P->HqN_l ? C.qnh[r] * sym_col_dot(P->HqN_l + lf * nx * nx, nx, r,
                                                                 [&](int c) { return ss[c]; })
                                       : (P->qnh_l ? gm(P->qnh_l)[lf * nx + r] : C.qnh[r]) * ss[r];
            real lt;
            if (kMode == 2 && P->GNt) {
                lt = cost;
                for (int q = 0; q < ncN; ++q) lt += gm(P->GNt)[(long long)q * nx + r] * sc[q];
            } else {
                lt = C.gxN[r] * sc[r] + cost;
                if (P->has_ballN) lt += C.gbN[r] * sc[nx + r];
            }
            real h = -(sx[r] - alpha * lt);
            if (P->affine) h += spc[r];
            gm(P->h0)[(long long)v * nx + r] = h;
        }
    }
}

// ---------------------------------------------------------------------------
// bsweep: leaves -> root
// ---------------------------------------------------------------------------

// base[r] for r = lane + 64 q (q < kVecPL), r clamped to n - 1: every load is
// issued unconditionally (the consumer ignores r >= n).
template <typename real>
SPK_DEV void vec_load(const real* __restrict__ base, int n, real* out) {
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < kVecPL; ++q) {
        const int r = lane + 64 * q;
        out[q] = gm(base)[r < n ? r : n - 1];
    }
}

// Children whose messages the backward sweep reads in one batch of loads.
constexpr int kMsgFast = 4;

// What one backward level needs from memory: its two tiles and h0, ubar.
template <typename real, int R>
struct BLevel {
    ColProd<real, R> TM;
    ColProd<real, R == kWideClass ? kWideClass : 16> TR;
    real h0r[kVecPL], ubr[kVecPL];
};

template <typename real, int R>
__global__ __launch_bounds__(64) void k_bsweep(const ProbDev<real>* __restrict__ probs,
                                               const int2* __restrict__ tasks) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = lane_id();
    const int2 tk = tasks[xcd_order(blockIdx.x, gridDim.x)];
    const ProbDev<real>* __restrict__ P = probs + tk.x;
    if (*P->active == 0) return;
    const int N = P->N, nx = P->nx, nu = P->nu, m = P->m, n_nl = P->n_nl;
    int* s_node = reinterpret_cast<int*>(smem_raw);
    int* s_nch = s_node + (N + 1);
    int* s_fc = s_nch + (N + 1);
    real* red = reinterpret_cast<real*>(smem_raw + sweep_int_bytes(N));
    real* hv = red + kRed;          // h of the current node (nx)
    real* gv = hv + sweep_vec(m);   // message (m)
    real* wv = gv + sweep_vec(m);   // ubar - g_u (nu)
    real* dv = wv + sweep_vec(nu);  // d (nu)
    // vectors are read in 16-byte groups: their padding must hold finite values
    for (int e = lane; e < sweep_elems(nx, nu); e += 64) red[e] = real(0);

    // (node, children, first child) of every stage of the path, one load each
    const auto* path = gm(reinterpret_cast<const int*>(P->path + (long long)tk.y * (N + 1)));
    for (int q = lane; q <= N; q += 64) {
        s_node[q] = path[4 * q];
        s_nch[q] = path[4 * q + 1];
        s_fc[q] = path[4 * q + 2];
    }
    wave_sync();
    const ColShape sM = col_shape<real>(nx, m), sR = col_shape<real>(nu, nu);
    // every load unconditional (the root reads node 1's [Abar|B] tile unused)
    auto load_level = [&](BLevel<real, R>& L, int i) {
        L.TM.load(P->T2M + (i > 0 ? i : 1) * P->T2M_stride, sM);
        L.TR.load(P->T2R + i * P->T2R_stride, sR);
        vec_load(P->h0 + (long long)i * nx, nx, L.h0r);
        vec_load(P->ub + (long long)i * nu, nu, L.ubr);
    };
    // Double-buffered levels (the next level's tiles load during this one)
    // where the registers allow it.
    constexpr bool kDB = sizeof(real) == 4 || R <= 32;
    BLevel<real, R> A, B;
    int j = s_node[N];
    {   // message of the leaf: [Abar^j|B^j]^T h0^j; the parent's data is
        // prefetched when the leaf is its only child
        ColProd<real, R> TM;
        TM.load(P->T2M + j * P->T2M_stride, sM);
        for (int r = lane; r < nx; r += 64) hv[r] = gm(P->h0)[(long long)j * nx + r];
        if constexpr (kDB) load_level(A, s_node[N - 1]);
        wave_sync();
        TM.template apply<true>(hv, gv, red);
    }
    // d of the node below is computed once the next level has begun (its
    // R~^-1 tile in the data set `prv`, its ubar - g_u in wv): off the message
    // chain, while the arrival at the next node is being counted
    int pend = -1;
    auto finish_d = [&](BLevel<real, R>& prv) {
        prv.TR.template apply<true>(wv, dv, red);  // d^pend = R~^-1 (ubar - g_u)
        for (int r = lane; r < nu; r += 64) gm(P->d)[(long long)pend * nu + r] = dv[r];
        pend = -1;
    };
    // one level with the data set `cur`; prefetches the next level into `nxt`
    // (`prv`: the previous level's set); false: another child continues
    auto level = [&](BLevel<real, R>& cur, BLevel<real, R>& nxt, BLevel<real, R>& prv, int lev) -> bool {
        const int i = s_node[lev], k = s_nch[lev], fc = s_fc[lev];
        if (k > 1) {
            for (int c = lane; c < m; c += 64) st_dev(P->e + (long long)j * m + c, gv[c]);
            // the message stores complete before the arrival is counted
            drain_stores();
            int prev = 0;
            if (lane == 0) prev = __hip_atomic_fetch_add(gm(P->cnt) + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (pend >= 0) finish_d(prv);
            prev = __builtin_amdgcn_readfirstlane(prev);
            if (prev != k - 1) return false;
            // the siblings' message loads below stay after the arrival count
            // (an ordering the compiler must keep; no cache action at wavefront scope)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane == 0) gm(P->cnt)[i] = 0;  // the next launch reuses the counter
        } else if (pend >= 0) {
            finish_d(prv);
        }
        // the children's messages (up to kMsgFast in registers, issued before
        // the prefetch so that waiting for them does not wait for it)
        real mv[kMsgFast][2];
        if (k > 1 && k <= kMsgFast) {
#pragma unroll
            for (int q = 0; q < kMsgFast; ++q) {
                const real* e = P->e + (long long)(fc + (q < k ? q : k - 1)) * m;
                mv[q][0] = ld_dev(e + (lane < m ? lane : m - 1));
                mv[q][1] = ld_dev(e + (64 + lane < m ? 64 + lane : m - 1));
            }
        }
        if constexpr (kDB) {
            // the next level's data, also where another child may take over
            // (then it is read in vain)
            load_level(nxt, s_node[lev > 0 ? lev - 1 : 0]);
        } else {
            load_level(cur, i);
        }
        if (k > 1) {
            // summed in child order
            if (k <= kMsgFast) {
                real s0 = 0, s1 = 0;
#pragma unroll
                for (int q = 0; q < kMsgFast; ++q)
                    if (q < k) {
                        s0 += mv[q][0];
                        s1 += mv[q][1];
                    }
                if (lane < m) gv[lane] = s0;
                if (64 + lane < m) gv[64 + lane] = s1;
                for (int c = 128 + lane; c < m; c += 64) {
                    real sum = 0;
                    for (int q = 0; q < k; ++q) sum += ld_dev(P->e + (long long)(fc + q) * m + c);
                    gv[c] = sum;
                }
            } else {
                for (int c = lane; c < m; c += 64) {
                    real sum = 0;
                    for (int q = 0; q < k; ++q) sum += ld_dev(P->e + (long long)(fc + q) * m + c);
                    gv[c] = sum;
                }
            }
            wave_sync();
        }
#pragma unroll
        for (int q = 0; q < kVecPL; ++q) {
            const int r = lane + 64 * q;
            if (r < nx) hv[r] = cur.h0r[q] + gv[r];
            if (r < nu) wv[r] = cur.ubr[q] - gv[nx + r];
        }
        wave_sync();
        if (i > 0) cur.TM.template apply<true>(hv, gv, red);  // message of i: [Abar^i|B^i]^T h^i
        pend = i;
        j = i;
        return true;
    };
    if constexpr (kDB) {
        int lev = N - 1;
        for (; lev >= 0; lev -= 2) {
            if (!level(A, B, B, lev)) return;
            if (lev == 0) break;
            if (!level(B, A, A, lev - 1)) return;
        }
        finish_d(lev == 0 ? A : B);  // the root's
    } else {
        for (int lev = N - 1; lev >= 0; --lev)
            if (!level(A, A, A, lev)) return;
        finish_d(A);  // the root's
    }
}

// ---------------------------------------------------------------------------
// fsweep: root -> leaves
// ---------------------------------------------------------------------------

// What one forward level needs from memory: its tile, c^v and d^v.
template <typename real, int R>
struct FLevel {
    ColProd<real, R> TM;
    real cr[kVecPL], dr[kVecPL];
};

template <typename real, int R>
__global__ __launch_bounds__(64) void k_fsweep(const ProbDev<real>* __restrict__ probs,
                                               const int2* __restrict__ tasks, int par) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = lane_id();
    const int2 tk = tasks[xcd_order(blockIdx.x, gridDim.x)];
    const ProbDev<real>* __restrict__ P = probs + tk.x;
    if (*P->active == 0) return;
    const int N = P->N, nx = P->nx, nu = P->nu, m = P->m, n_nl = P->n_nl;
    real* __restrict__ zout = P->z[par ^ 1];
    int* s_node = reinterpret_cast<int*>(smem_raw);
    real* red = reinterpret_cast<real*>(smem_raw + sweep_int_bytes(N));
    real* av = red + kRed;          // [x^anc ; d^anc] (m)
    real* xv = av + sweep_vec(m);   // x of the current node (nx)
    for (int e = lane; e < sweep_elems(nx, nu); e += 64) red[e] = real(0);

    // This task computes its whole root-to-leaf path and stores the nodes it
    // owns (stages L..N, those whose leftmost leaf it is); every other task
    // through a node computes the same x^v, bit for bit, and drops it.
    const int L = gm(P->top_owned)[tk.y];
    const auto* path = gm(reinterpret_cast<const int*>(P->path + (long long)tk.y * (N + 1)));
    for (int q = lane; q <= N; q += 64) s_node[q] = path[4 * q];
    wave_sync();
    const ColShape sT = col_shape<real>(m, nx);
    // every load unconditional: without an affine term c is read from x0 and
    // a leaf reads the last non-leaf d, both unused
    auto load_level = [&](FLevel<real, R>& F, int v) {
        F.TM.load(P->T3 + v * P->T3_stride, sT);
        vec_load(P->affine ? P->c + (long long)v * nx : P->x0, nx, F.cr);
        vec_load(P->d + (long long)(v < n_nl ? v : n_nl - 1) * nu, nu, F.dr);
    };
    // Double-buffered levels (the next level's data loads during this one)
    // where the registers allow it.
    constexpr bool kDB = (sizeof(real) == 4 && R <= 64) || R <= 32;
    FLevel<real, R> A, B;
    // the root's state is the initial state
    for (int r = lane; r < nx; r += 64) {
        const real x = gm(P->x0)[r];
        av[r] = x;
        if (L == 0) gm(zout)[P->z_x + r] = x;
    }
    for (int r = lane; r < nu; r += 64) av[nx + r] = gm(P->d)[r];
    if (N >= 1) load_level(A, s_node[1]);
    wave_sync();
    // one level with the data set `cur`, the next level's data loading into `nxt`
    auto level = [&](FLevel<real, R>& cur, FLevel<real, R>& nxt, int lv) {
        const int v = s_node[lv];
        if (kDB) load_level(nxt, s_node[lv < N ? lv + 1 : N]);
        if (!kDB && lv > 1) load_level(cur, v);
        cur.TM.template apply<true>(av, xv, red);  // x^v = [Abar^v | B^v] [x^anc; d^anc]
#pragma unroll
        for (int q = 0; q < kVecPL; ++q) {
            const int r = lane + 64 * q;
            if (r < nx) {
                const real x = xv[r] + (P->affine ? cur.cr[q] : real(0));
                av[r] = x;
                if (lv >= L) gm(zout)[P->z_x + (long long)v * nx + r] = x;
            }
            if (r < nu) av[nx + r] = cur.dr[q];
        }
        wave_sync();
    };
    int lev = 1;
    if constexpr (kDB) {
        for (; lev <= N; lev += 2) {
            level(A, B, lev);
            if (lev + 1 > N) break;
            level(B, A, lev + 1);
        }
    } else {
        for (; lev <= N; ++lev) level(A, A, lev);
    }
}

// ---------------------------------------------------------------------------
// staged sweeps (float): global -> LDS copies a level ahead
// ---------------------------------------------------------------------------
//
// Same recursions as k_bsweep / k_fsweep.  Every tile and vector a level
// needs is copied to LDS with global-to-LDS loads while the level before it
// runs, and moved into registers (tiles) only when the level starts, so one
// tile is ever held in registers and no prefetch waits on register pressure.
// The copies are written in assembly: the compiler neither counts nor waits
// for them, and each consumer waits for them explicitly (vm_wait).  No load
// that the compiler waits for is issued after a copy that is still wanted in
// flight (its wait would cover the copy too).

// LDS byte address of a pointer into dynamic LDS.
SPK_DEV unsigned lds_off(const void* p) {
    return (unsigned)(size_t)(const __attribute__((address_space(3))) void*)p;
}

// A uniform value or address, held in scalar registers.
SPK_DEV unsigned uni(unsigned x) { return (unsigned)__builtin_amdgcn_readfirstlane((int)x); }
SPK_DEV const void* uni(const void* p) {
    const unsigned long long a = (unsigned long long)p;
    return (const void*)(((unsigned long long)uni((unsigned)(a >> 32)) << 32) | uni((unsigned)a));
}

// Global-to-LDS loads: lane l reads 16 (dma16) or 4 (dma4) bytes at
// base + voff (+ k KiB) and writes them at lds + 16 l (+ 4 l) (+ k KiB);
// base and lds are uniform.  M0 carries lds and is restored.  dma16x4 copies
// four consecutive 1 KiB lane groups with one address set-up.
SPK_DEV void dma16(const void* base, unsigned voff, unsigned lds) {
    unsigned save;
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %3\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %1, %2\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(save)
        : "v"(voff), "s"(uni(base)), "s"(uni(lds))
        : "memory");
}
SPK_DEV void dma16x4(const void* base, unsigned voff, unsigned lds) {
    unsigned save;
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %3\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %1, %2\n\t"
        "global_load_lds_dwordx4 %1, %2 offset:1024\n\t"
        "global_load_lds_dwordx4 %1, %2 offset:2048\n\t"
        "global_load_lds_dwordx4 %1, %2 offset:3072\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(save)
        : "v"(voff), "s"(uni(base)), "s"(uni(lds))
        : "memory");
}
SPK_DEV void dma4(const void* base, unsigned voff, unsigned lds) {
    unsigned save;
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %3\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dword %1, %2\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(save)
        : "v"(voff), "s"(uni(base)), "s"(uni(lds))
        : "memory");
}

// Wait until at most N of this wavefront's vector memory operations are in
// flight (they complete in issue order), then order the LDS accesses after it.
template <int N>
SPK_DEV void vm_wait() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
    wave_sync();
}
// Wait for this wavefront's LDS reads (before a copy overwrites what they read).
SPK_DEV void lgkm_wait() {
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    wave_sync();
}

// The tile's own lane groups to LDS, in the same layout (block 2, or one
// group after block 1 when there is none, follows block 1).  Nothing is
// copied when the shape does not fit class R (or has more than two blocks).
template <typename real, int R>
SPK_DEV void col_dma(const real* __restrict__ tile, const ColShape& s, real* st) {
    constexpr int V = 16 / (int)sizeof(real);
    if (s.O > 128 || s.rows1 > R || s.rows2 > R / 4) return;
    const int G = s.rows1 / V + (s.rows2 > 0 ? s.rows2 / V : 1);
    const unsigned voff = (unsigned)lane_id() * 16;
    const char* t = reinterpret_cast<const char*>(tile);
    const unsigned base = lds_off(st);
    int g = 0;
    for (; g + 4 <= G; g += 4) dma16x4(t + (long long)g * 1024, voff, base + g * 1024);
    for (; g < G; ++g) dma16(t + (long long)g * 1024, voff, base + g * 1024);
}

// A staged tile from LDS into registers (the layout of col_load).
template <typename real, int R>
SPK_DEV void col_take(ColTile<real, R>& T, const real* st, const ColShape& s) {
    constexpr int V = 16 / (int)sizeof(real);
    const int lane = lane_id();
    const int g1 = s.rows1 / V, l1 = g1 - 1, l2 = s.rows2 > 0 ? s.rows2 / V - 1 : 0;
#pragma unroll
    for (int q = 0; q < R / V; ++q) lds16(st + ((q < l1 ? q : l1) * 64 + lane) * V, T.a + q * V);
    st += g1 * 64 * V;
#pragma unroll
    for (int q = 0; q < R / 4 / V; ++q) lds16(st + ((q < l2 ? q : l2) * 64 + lane) * V, T.b + q * V);
}

// n >= 1 entries of src into an LDS slot (entries past n up to the next
// multiple of 256 bytes: copies of the last dword).
template <typename real>
SPK_DEV void vec_dma(const real* src, int n, real* dst) {
    const int lane = lane_id();
    const unsigned base = lds_off(dst);
    const int nd = n * (int)(sizeof(real) / 4);
    for (int q = 0; q * 64 < nd; ++q) {
        const int e = q * 64 + lane;
        dma4(src, (unsigned)(e < nd ? e : nd - 1) * 4, base + q * 256);
    }
}

template <typename real, int R>
__global__ __launch_bounds__(64) void k_bsweep_st(const ProbDev<real>* __restrict__ probs,
                                                  const int2* __restrict__ tasks) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int V = tile_vec<real>();
    const int lane = lane_id();
    const int2 tk = tasks[xcd_order(blockIdx.x, gridDim.x)];
    const ProbDev<real>* __restrict__ P = probs + tk.x;
    if (*P->active == 0) return;
    const int N = P->N, nx = P->nx, nu = P->nu, m = P->m;
    int* s_node = reinterpret_cast<int*>(smem_raw);
    int* s_nch = s_node + (N + 1);
    int* s_fc = s_nch + (N + 1);
    real* red = reinterpret_cast<real*>(smem_raw + sweep_int_bytes(N));
    real* hv = red + kRed;          // h of the current node (nx)
    real* gv = hv + sweep_vec(m);   // message (m)
    real* wv = gv + sweep_vec(m);   // ubar - g_u (nu)
    real* dv = wv + sweep_vec(nu);  // d (nu)
    real* vs = red + sweep_elems(nx, nu);
    real* h0s[2] = {vs, vs + 2 * kVecSlot};  // h0 of the level, two slots
    real* ubs[2] = {vs + kVecSlot, vs + 3 * kVecSlot};
    const ColShape sM = col_shape<real>(nx, m), sR = col_shape<real>(nu, nu);
    real* stM = vs + 4 * kVecSlot;  // staged [Abar|B] tile
    real* stR = stM + stage_groups(nx, m, V, R) * 64 * V;  // staged R~^-1 tile
    for (int e = lane; e < sweep_elems(nx, nu); e += 64) red[e] = real(0);

    // (node, children, first child) of every stage of the path, one load each
    const auto* path = gm(reinterpret_cast<const int*>(P->path + (long long)tk.y * (N + 1)));
    for (int q = lane; q <= N; q += 64) {
        s_node[q] = path[4 * q];
        s_nch[q] = path[4 * q + 1];
        s_fc[q] = path[4 * q + 2];
    }
    wave_sync();
    ColProd<real, R> TM;
    ColProd<real, R == kWideClass ? kWideClass : 16> TR;
    // level data of node i into slot b (the root stages node 1's [Abar|B], unused)
    auto stage = [&](int i, int b) {
        col_dma<real, R>(P->T2M + (i > 0 ? i : 1) * P->T2M_stride, sM, stM);
        col_dma<real, 16>(P->T2R + i * P->T2R_stride, sR, stR);
        vec_dma(P->h0 + (long long)i * nx, nx, h0s[b]);
        vec_dma(P->ub + (long long)i * nu, nu, ubs[b]);
    };
    int j = s_node[N];
    // the leaf's message [Abar^j|B^j]^T h0^j (its h0 through slot 1)
    col_dma<real, R>(P->T2M + j * P->T2M_stride, sM, stM);
    vec_dma(P->h0 + (long long)j * nx, nx, h0s[1]);
    vm_wait<0>();
    TM.take(P->T2M + j * P->T2M_stride, sM, stM);
    for (int r = lane; r < nx; r += 64) hv[r] = h0s[1][r];
    lgkm_wait();
    if (N >= 1) stage(s_node[N - 1], 0);
    TM.template apply<true>(hv, gv, red);
    // d of the node below is computed once the next level has begun (its R~^-1
    // tile stays in registers, its ubar - g_u in wv): off the message chain,
    // while the arrival at the next node is being counted
    int pend = -1;
    auto finish_d = [&]() {
        TR.template apply<true>(wv, dv, red);  // d^pend = R~^-1 (ubar - g_u)
        for (int r = lane; r < nu; r += 64) gm(P->d)[(long long)pend * nu + r] = dv[r];
        pend = -1;
    };
    int b = 0;
    for (int lev = N - 1; lev >= 0; --lev, b ^= 1) {
        const int i = s_node[lev], k = s_nch[lev], fc = s_fc[lev];
        real mv[kMsgFast][2];
        if (k > 1) {
            for (int c = lane; c < m; c += 64) st_dev(P->e + (long long)j * m + c, gv[c]);
            // the message stores (and every copy issued so far) complete
            // before the arrival is counted
            drain_stores();
            int prev = 0;
            if (lane == 0) prev = __hip_atomic_fetch_add(gm(P->cnt) + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (pend >= 0) finish_d();
            prev = __builtin_amdgcn_readfirstlane(prev);
            if (prev != k - 1) return;
            // the siblings' message loads below stay after the arrival count
            // (an ordering the compiler must keep; no cache action at wavefront scope)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane == 0) gm(P->cnt)[i] = 0;  // the next launch reuses the counter
            if (k <= kMsgFast) {
#pragma unroll
                for (int q = 0; q < kMsgFast; ++q) {
                    const real* e = P->e + (long long)(fc + (q < k ? q : k - 1)) * m;
                    mv[q][0] = ld_dev(e + (lane < m ? lane : m - 1));
                    mv[q][1] = ld_dev(e + (64 + lane < m ? 64 + lane : m - 1));
                }
            }
        } else if (lev == N - 1) {
            vm_wait<0>();
        } else {
            finish_d();
            // only the previous level's d store (at least one) may be younger
            // than this level's copies
            vm_wait<1>();
        }
        TM.take(P->T2M + (i > 0 ? i : 1) * P->T2M_stride, sM, stM);
        TR.take(P->T2R + i * P->T2R_stride, sR, stR);
        lgkm_wait();
        // the next level's copies: right away on a single-child level, after
        // the messages arrived otherwise (their wait would cover the copies)
        if (k == 1 && lev > 0) stage(s_node[lev - 1], b ^ 1);
        if (k > 1) {
            // summed in child order
            if (k <= kMsgFast) {
                real s0 = 0, s1 = 0;
#pragma unroll
                for (int q = 0; q < kMsgFast; ++q)
                    if (q < k) {
                        s0 += mv[q][0];
                        s1 += mv[q][1];
                    }
                if (lane < m) gv[lane] = s0;
                if (64 + lane < m) gv[64 + lane] = s1;
                for (int c = 128 + lane; c < m; c += 64) {
                    real sum = 0;
                    for (int q = 0; q < k; ++q) sum += ld_dev(P->e + (long long)(fc + q) * m + c);
                    gv[c] = sum;
                }
            } else {
                for (int c = lane; c < m; c += 64) {
                    real sum = 0;
                    for (int q = 0; q < k; ++q) sum += ld_dev(P->e + (long long)(fc + q) * m + c);
                    gv[c] = sum;
                }
            }
            wave_sync();
            if (lev > 0) stage(s_node[lev - 1], b ^ 1);
        }
        for (int r = lane; r < nx; r += 64) hv[r] = h0s[b][r] + gv[r];
        for (int r = lane; r < nu; r += 64) wv[r] = ubs[b][r] - gv[nx + r];
        wave_sync();
        if (i > 0) TM.template apply<true>(hv, gv, red);  // message of i: [Abar^i|B^i]^T h^i
        pend = i;
        j = i;
    }
    finish_d();  // the root's
    vm_wait<0>();  // no copy outlives the wavefront
}

template <typename real, int R>
__global__ __launch_bounds__(64) void k_fsweep_st(const ProbDev<real>* __restrict__ probs,
                                                  const int2* __restrict__ tasks, int par) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = lane_id();
    const int2 tk = tasks[xcd_order(blockIdx.x, gridDim.x)];
    const ProbDev<real>* __restrict__ P = probs + tk.x;
    if (*P->active == 0) return;
    const int N = P->N, nx = P->nx, nu = P->nu, m = P->m, n_nl = P->n_nl;
    real* __restrict__ zout = P->z[par ^ 1];
    int* s_node = reinterpret_cast<int*>(smem_raw);
    real* red = reinterpret_cast<real*>(smem_raw + sweep_int_bytes(N));
    real* av = red + kRed;          // [x^anc ; d^anc] (m)
    real* xv = av + sweep_vec(m);   // x of the current node (nx)
    real* vs = red + sweep_elems(nx, nu);
    real* cs[2] = {vs, vs + 2 * kVecSlot};  // c of the level, two slots
    real* ds[2] = {vs + kVecSlot, vs + 3 * kVecSlot};  // d of the level
    real* stT = vs + 4 * kVecSlot;  // staged [Abar|B]^T tile
    for (int e = lane; e < sweep_elems(nx, nu); e += 64) red[e] = real(0);

    // the whole root-to-leaf path, stores from stage L on (see k_fsweep)
    const int L = gm(P->top_owned)[tk.y];
    const auto* path = gm(reinterpret_cast<const int*>(P->path + (long long)tk.y * (N + 1)));
    for (int q = lane; q <= N; q += 64) s_node[q] = path[4 * q];
    const ColShape sT = col_shape<real>(m, nx);
    ColProd<real, R> TM;
    // level data of node v into slot b (a leaf stages an unused d)
    auto stage = [&](int v, int b) {
        col_dma<real, R>(P->T3 + v * P->T3_stride, sT, stT);
        if (P->affine) vec_dma(P->c + (long long)v * nx, nx, cs[b]);
        vec_dma(P->d + (long long)(v < n_nl ? v : n_nl - 1) * nu, nu, ds[b]);
    };
    // the root's state is the initial state (read before any copy)
    for (int r = lane; r < nx; r += 64) {
        const real x = gm(P->x0)[r];
        av[r] = x;
        if (L == 0) gm(zout)[P->z_x + r] = x;
    }
    for (int r = lane; r < nu; r += 64) av[nx + r] = gm(P->d)[r];
    wave_sync();
    if (N >= 1) stage(s_node[1], 0);
    for (int lev = 1, b = 0; lev <= N; ++lev, b ^= 1) {
        const int v = s_node[lev];
        // this level's copies have landed (the previous level's stores of x,
        // if any, may still be in flight)
        if (lev > 1 && lev - 1 >= L) vm_wait<1>();
        else vm_wait<0>();
        TM.take(P->T3 + v * P->T3_stride, sT, stT);
        lgkm_wait();
        if (lev < N) stage(s_node[lev + 1], b ^ 1);
        TM.template apply<true>(av, xv, red);  // x^v = [Abar^v | B^v] [x^anc; d^anc]
        for (int r = lane; r < nx; r += 64) {
            const real x = xv[r] + (P->affine ? cs[b][r] : real(0));
            av[r] = x;
            if (lev >= L) gm(zout)[P->z_x + (long long)v * nx + r] = x;
        }
        for (int r = lane; r < nu; r += 64) av[nx + r] = ds[b][r];
        wave_sync();
    }
    vm_wait<0>();  // no copy outlives the wavefront
}

// ---------------------------------------------------------------------------
// dual: node-parallel forward half-step
// ---------------------------------------------------------------------------

template <typename real, int R, int kMode>
__global__ __launch_bounds__(512) void k_dual(const ProbDev<real>* __restrict__ probs,
                                              const int2* __restrict__ ntasks, const int4* __restrict__ ninfo,
                                              int wave_elems, int par, int check) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real* sm = reinterpret_cast<real*>(smem_raw);
    const int waves = (int)(blockDim.x >> 6), w = (int)(threadIdx.x >> 6), lane = lane_id();
    const int2 t0 = ntasks[blockIdx.x * waves];
    const int v = ntasks[blockIdx.x * waves + w].y;
    const int4 ni = ninfo[blockIdx.x * waves + w];
    const ProbDev<real>* __restrict__ P = probs + t0.x;
    if (*P->active == 0) return;
    const int nx = P->nx, nu = P->nu, m = P->m, nc = P->nc, ncN = P->ncN, n_nl = P->n_nl;
    real* cst = sm;
    stage_consts(P, cst);
    if (v < 0) return;
    const Consts<real> C = consts_at<real>(cst, nx, nu);
    const real ialpha = real(1) / P->alpha;
    const real* __restrict__ zin = P->z[par];
    const real* __restrict__ ein = P->eta[par];
    real* __restrict__ zout = P->z[par ^ 1];
    real* __restrict__ eout = P->eta[par ^ 1];
    const int bmax = blk_elems(nx, nu, nc, ncN);
    real* red = cst + consts_elems(nx, nu) + w * wave_elems;
    real* un = red + kRed;
    real* lxw = un + nu;
    real* luw = lxw + nx;
    real* blk = luw + nu;
    real* dblk = blk + bmax;
    real* st = red + kRed + node_head_elems(nx, nu, nc, ncN);
    const long long soff = (v == 0) ? 0 : P->z_s + v - 1;
    real r1 = 0, r2 = 0;  // residual maxima of this lane

    if (v < n_nl) {
        const int fc = ni.x, k = ni.y;
        const long long yo = ni.z;
        const bool sk = k <= kStageKids && k <= P->stage_kids;
        const int kk = sk ? k : 0, ky = sk ? 2 * k + 1 : 0;
        ColProd<real, R> TK;  // u = K x + d
        TK.load(P->T4 + v * P->T4_stride, col_shape<real>(nx, nu));
        Stage<real, 15> S{};
        S.set(0, zout + P->z_x + (long long)v * nx, nx);
        S.set(1, zin + P->z_x + (long long)v * nx, nx);
        S.set(2, zin + P->z_u + (long long)v * nu, nu);
        S.set(3, P->d + (long long)v * nu, nu);
        S.set(4, ein + P->e_c + (long long)v * nc, nc);
        S.set(5, ein + P->e_soc + (long long)(fc - 1) * (m + 2), kk * (m + 2));
        S.set(6, ein + P->e_y + yo, ky);
        S.set(7, ein + P->e_s + v, 1);
        S.set(8, zout + P->z_y + yo, ky);
        S.set(9, zin + P->z_y + yo, ky);
        S.set(10, zout + soff, 1);
        S.set(11, zin + soff, 1);
        S.set(12, zout + P->z_tau + fc - 1, kk);
        S.set(13, zin + P->z_tau + fc - 1, kk);
        S.set(14, P->prob + fc, kk);
        int off[15];
        gather(S, st, off);
        wait_loads();
        const real* xn = st + off[0];
        const real* xo = st + off[1];
        const real* uo = st + off[2];
        const real* dd = st + off[3];
        // ---- input: u^v = K^v x^v + d^v ----
        TK.apply(xn, un, red);
        for (int r = lane; r < nu; r += 64) {
            const real u = un[r] + dd[r];
            un[r] = u;
            gm(zout)[P->z_u + (long long)v * nu + r] = u;
        }
        if (check) {
            for (int r = lane; r < nx; r += 64) lxw[r] = 0;
            for (int r = lane; r < nu; r += 64) luw[r] = 0;
        }
        wave_sync();
        const FwdNode<real> V{C, xn, un, xo, uo, blk, dblk, lxw, luw};
        fwd_block_c<real, kMode>(P, v, st + off[4], eout, V, check, r2);
        wave_sync();
        // per-child inputs: the staged copies, or for a wide node the arrays
        // themselves, each through a pointer of its own address space
        auto per_child = [&](auto soc, auto ey, auto yn, auto yv, auto tn, auto tv, auto pr) {
            if (kMode == 2 && P->rdata)
                fwd_block_risk_gen(P, v, yo, k, ey, st[off[7]], yn, yv, st[off[10]], st[off[11]], eout, check, r1,
                                   r2);
            else
                fwd_block_risk(P, v, yo, k, ey, st[off[7]], yn, yv, st[off[10]], st[off[11]], pr, eout, check, r1,
                               r2);
            wave_sync();
            for (int q = 0; q < k; ++q) {
                fwd_block_soc<real, kMode>(P, fc + q, soc + q * (m + 2), tn[q], tv[q], eout, V, check, r1, r2);
                wave_sync();
            }
        };
        if (sk)
            per_child(lds(st + off[5]), lds(st + off[6]), lds(st + off[8]), lds(st + off[9]), lds(st + off[12]),
                      lds(st + off[13]), lds(st + off[14]));
        else
            per_child(gm(ein + P->e_soc + (long long)(fc - 1) * (m + 2)), gm(ein + P->e_y + yo),
                      gm(static_cast<const real*>(zout + P->z_y + yo)), gm(zin + P->z_y + yo),
                      gm(static_cast<const real*>(zout + P->z_tau + fc - 1)), gm(zin + P->z_tau + fc - 1),
                      gm(P->prob + fc));
        if (check) {
            for (int r = lane; r < nx; r += 64) r1 = nmax(r1, fabs((xo[r] - xn[r]) * ialpha - lxw[r]));
            for (int r = lane; r < nu; r += 64) r1 = nmax(r1, fabs((uo[r] - un[r]) * ialpha - luw[r]));
        }
    } else {
        const long long lf = v - n_nl;
        Stage<real, 6> S{};
        S.set(0, zout + P->z_x + (long long)v * nx, nx);
        S.set(1, zin + P->z_x + (long long)v * nx, nx);
        S.set(2, ein + P->e_cN + lf * ncN, ncN);
        S.set(3, ein + P->e_socN + lf * (nx + 2), nx + 2);
        S.set(4, zout + soff, 1);
        S.set(5, zin + soff, 1);
        int off[6];
        gather(S, st, off);
        wait_loads();
        if (check)
            for (int r = lane; r < nx; r += 64) lxw[r] = 0;
        wave_sync();
        const real* xn = st + off[0];
        const real* xo = st + off[1];
        const FwdNode<real> V{C, xn, un, xo, xo, blk, dblk, lxw, luw};
        fwd_block_leaf<real, kMode>(P, v, 0, st + off[2], st + off[3], st[off[4]], st[off[5]], eout, V, check, r1, r2);
        wave_sync();
        fwd_block_leaf<real, kMode>(P, v, 1, st + off[2], st + off[3], st[off[4]], st[off[5]], eout, V, check, r1, r2);
        wave_sync();
        if (check)
            for (int r = lane; r < nx; r += 64) r1 = nmax(r1, fabs((xo[r] - xn[r]) * ialpha - lxw[r]));
    }
    if (check) {
        r1 = wave_max(r1);
        r2 = wave_max(r2);
        if (lane == 0) {
            const int slot = (int)(blockIdx.x % kResSlots);
            record_max(&P->res[2 * slot], r1);
            record_max(&P->res[2 * slot + 1], r2);
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
            if (P->Gt) {
                w = 0;
                for (int c = 0; c < m; ++c) w += P->Gt[(long long)r * m + c] * (c < nx ? x[c] : u[c - nx]);
            } else if (r < nx) {
                w = P->gx[r] * x[r];
            } else if (r < nbox) {
                w = P->gu[r - nx] * u[r - nx];
            } else {
                w = P->gb[r - nbox] * x[r - nbox];
            }
            eta[P->e_c + (long long)v * P->nc + r] = w;
        }
        const int k = P->n_ch[v], fc = P->first_child[v];
        const long long yo = P->y_off[v];
        const real* y = z + P->z_y + yo;
        // b^T y with b = (p, 0, 1) for AV@R, else the node's own b
        const real* bg = P->rdata ? risk_data(P, v, k).b : nullptr;
        const int ny = bg ? P->rny[v] : 2 * k + 1;
        real b = 0;
        if (bg) {
            for (int c = t; c < ny; c += kHookWG) b += bg[c] * y[c];
            b = block_sum<kHookWG>(b, red);
        } else {
            for (int c = t; c < k; c += kHookWG) b += P->prob[fc + c] * y[c];
            b = block_sum<kHookWG>(b, red) + y[2 * k];
        }
        const real s = (v == 0) ? z[0] : z[P->z_s + v - 1];
        if (t == 0) eta[P->e_s + v] = s - b;
        for (int c = t; c < ny; c += kHookWG) eta[P->e_y + yo + c] = y[c];
        for (int q = 0; q < k; ++q) {
            const int j = fc + q;
            real tau = z[P->z_tau + j - 1];
            if (P->ck) {  // tau rows (tau - c_j^T u) / 2 (Prop. 1 with R singular)
                real cu = 0;
                for (int c = t; c < nu; c += kHookWG) cu += P->ck[(long long)j * nu + c] * u[c];
                tau -= block_sum<kHookWG>(cu, red);
            }
            real* o = eta + P->e_soc + (long long)(j - 1) * (m + 2);
            for (int r = t; r < m + 2; r += kHookWG) {
                if (P->Hq_e && r < m) {
                    real a = 0;
                    if (r < nx)
                        for (int c = 0; c < nx; ++c) a += P->Hq_e[((long long)j * nx + r) * nx + c] * P->qh[c] * x[c];
                    else
                        for (int c = 0; c < nu; ++c)
                            a += P->Hr_e[((long long)j * nu + r - nx) * nu + c] * P->rh[c] * u[c];
                    o[r] = a;
                    continue;
                }
                o[r] = r < nx ? (P->qh_e ? P->qh_e[(long long)j * nx + r] : P->qh[r]) * x[r]
                              : (r < m ? (P->rh_e ? P->rh_e[(long long)j * nu + r - nx] : P->rh[r - nx]) * u[r - nx]
                                       : real(0.5) * tau);
            }
        }
    } else {
        const long long lf = v - P->n_nl;
        for (int r = t; r < P->ncN; r += kHookWG) {
            real w;
            if (P->GNt) {
                w = 0;
                for (int c = 0; c < nx; ++c) w += P->GNt[(long long)r * nx + c] * x[c];
            } else {
                w = r < nx ? P->gxN[r] * x[r] : P->gbN[r - nx] * x[r - nx];
            }
            eta[P->e_cN + lf * P->ncN + r] = w;
        }
        const real s = z[P->z_s + v - 1];
        for (int r = t; r < nx + 2; r += kHookWG) {
            real w;
            if (P->HqN_l && r < nx) {
                w = 0;
                for (int c = 0; c < nx; ++c) w += P->HqN_l[(lf * nx + r) * nx + c] * P->qnh[c] * x[c];
            } else {
                w = r < nx ? (P->qnh_l ? P->qnh_l[lf * nx + r] : P->qnh[r]) * x[r] : real(0.5) * s;
            }
            eta[P->e_socN + lf * (nx + 2) + r] = w;
        }
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
            for (int q = 0; q < k; ++q) {
                const real* o = eta + P->e_soc + (long long)(fc + q - 1) * (m + 2);
                if (P->Hq_e) {
                    real a = 0;
                    for (int c = 0; c < nx; ++c) a += P->Hq_e[((long long)(fc + q) * nx + r) * nx + c] * o[c];
                    s += P->qh[r] * a;
                } else {
                    s += (P->qh_e ? P->qh_e[(long long)(fc + q) * nx + r] : P->qh[r]) * o[r];
                }
            }
            real w = s;
            if (P->Gt) {
                for (int q = 0; q < P->nc; ++q) w += P->Gt[(long long)q * m + r] * ec[q];
            } else {
                w += P->gx[r] * ec[r];
                if (P->has_ball) w += P->gb[r] * ec[nbox + r];
            }
            x[r] = w;
        }
        for (int r = t; r < nu; r += kHookWG) {
            real s = 0;
            for (int q = 0; q < k; ++q) {
                const real* o = eta + P->e_soc + (long long)(fc + q - 1) * (m + 2) + nx;
                if (P->Hr_e) {
                    real a = 0;
                    for (int c = 0; c < nu; ++c) a += P->Hr_e[((long long)(fc + q) * nu + r) * nu + c] * o[c];
                    s += P->rh[r] * a;
                } else {
                    s += (P->rh_e ? P->rh_e[(long long)(fc + q) * nu + r] : P->rh[r]) * o[r];
                }
                if (P->ck) s -= real(0.5) * P->ck[(long long)(fc + q) * nu + r] * (o[m - nx] + o[m - nx + 1]);
            }
            real w = s;
            if (P->Gt) {
                for (int q = 0; q < P->nc; ++q) w += P->Gt[(long long)q * m + nx + r] * ec[q];
            } else {
                w += P->gu[r] * ec[nx + r];
            }
            z[P->z_u + (long long)v * nu + r] = w;
        }
        const long long yo = P->y_off[v];
        const real es = eta[P->e_s + v];
        const real* bg = P->rdata ? risk_data(P, v, k).b : nullptr;
        const int ny = bg ? P->rny[v] : 2 * k + 1;
        for (int c = t; c < ny; c += kHookWG) {
            const real bc = bg ? bg[c] : c < k ? P->prob[fc + c] : (c == 2 * k ? real(1) : real(0));
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
            real cost;
            if (P->HqN_l) {
                cost = 0;
                for (int c = 0; c < nx; ++c) cost += P->HqN_l[(lf * nx + r) * nx + c] * esN[c];
                cost *= P->qnh[r];
            } else {
                cost = (P->qnh_l ? P->qnh_l[lf * nx + r] : P->qnh[r]) * esN[r];
            }
            real w = cost;
            if (P->GNt) {
                for (int q = 0; q < P->ncN; ++q) w += P->GNt[(long long)q * nx + r] * ecN[q];
            } else {
                w += P->gxN[r] * ecN[r];
                if (P->has_ballN) w += P->gbN[r] * ecN[nx + r];
            }
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
    // v = w - alpha a, eta = v - proj_SOC(v) (a: the block's translation)
    auto soc = [&](long long off, int len, const real* a) {
        real nw2 = 0;
        for (int r = t; r < len - 1; r += kHookWG) {
            const real e = w[off + r] - alpha * soc_shift_at(a, r, len);
            nw2 += e * e;
        }
        nw2 = block_sum<kHookWG>(nw2, red);
        const real vt = w[off + len - 1] - alpha * soc_shift_at(a, len - 1, len);
        real cw, ct;
        soc_moreau_coef(nw2, vt, cw, ct);
        for (int r = t; r < len; r += kHookWG) {
            const real e = w[off + r] - alpha * soc_shift_at(a, r, len);
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
        // rows where K is R_+ keep min(e, 0), rows where K is {0} (dual R) give 0
        const real* cg = P->rdata ? risk_data(P, v, k).cone : nullptr;
        const int ny = cg ? P->rny[v] : 2 * k + 1;
        for (int c = t; c < ny; c += kHookWG) {
            const real e = w[P->e_y + yo + c];
            const bool pos = cg ? cg[c] == real(0) : c < 2 * k;
            eta[P->e_y + yo + c] = pos ? (e < 0 ? e : real(0)) : real(0);
        }
        // second-order cone blocks of a general risk: e minus its projection
        // onto the cone (head row code 2, its w rows coded -1 - head)
        for (int hr = 0; cg && hr < ny; ++hr) {
            if (cg[hr] != real(2)) continue;
            const real tag = real(-1 - hr);
            real w2 = 0;
            for (int c = t; c < ny; c += kHookWG)
                if (cg[c] == tag) w2 += w[P->e_y + yo + c] * w[P->e_y + yo + c];
            const real nw = sqrt(block_sum<kHookWG>(w2, red)), th = w[P->e_y + yo + hr];
            const real ct = nw <= th ? th : (nw <= -th ? real(0) : real(0.5) * (th + nw));
            const real cw = nw <= th ? real(1) : (nw <= -th ? real(0) : ct / nw);
            for (int c = t; c < ny; c += kHookWG) {
                const real e = w[P->e_y + yo + c];
                if (c == hr) eta[P->e_y + yo + c] = e - ct;
                else if (cg[c] == tag) eta[P->e_y + yo + c] = e - cw * e;
            }
        }
        if (t == 0) {
            const real e = w[P->e_s + v];
            eta[P->e_s + v] = e < 0 ? e : real(0);
        }
        ballbox(P->e_c + (long long)v * P->nc, nbox, P->nc, P->lo, P->hi, P->ball_r);
        for (int q = 0; q < k; ++q)
            soc(P->e_soc + (long long)(fc + q - 1) * (m + 2), m + 2,
                P->sa ? P->sa + (long long)(fc + q - 1) * (m + 2) : nullptr);
    } else {
        const long long lf = v - P->n_nl;
        ballbox(P->e_cN + lf * P->ncN, P->nboxN, P->ncN, P->loN, P->hiN, P->ballN_r);
        soc(P->e_socN + lf * (nx + 2), nx + 2, P->saN ? P->saN + lf * (nx + 2) : nullptr);
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
// vector algebra of the SuperMann iteration (float64)
// ---------------------------------------------------------------------------

// out = sum_i c_i in_i, inputs summed in index order; every entry is read
// before it is written, so out may be one of the inputs.
__global__ __launch_bounds__(256) void k_combo(double* out, VecCombo cb, long long n) {
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        double s = 0.0;
        for (int i = 0; i < cb.n_in; ++i) s += cb.c[i] * cb.in[i][k];
        out[k] = s;
    }
}

// The same for 16-byte aligned vectors and a fixed number of inputs (the
// common one to three): two entries per lane and pass, every input's load
// issued before the sums (in input order, as above); an odd last entry is
// taken by the first lane.
template <int NIN>
__global__ __launch_bounds__(256) void k_combo2(double* out, VecCombo cb, long long n) {
    const long long n2 = n >> 1;
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n2; k += (long long)gridDim.x * 256) {
        double2 v[NIN];
#pragma unroll
        for (int i = 0; i < NIN; ++i) v[i] = reinterpret_cast<const double2*>(cb.in[i])[k];
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
            sx += cb.c[i] * v[i].x;
            sy += cb.c[i] * v[i].y;
        }
        reinterpret_cast<double2*>(out)[k] = make_double2(sx, sy);
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < NIN; ++i) s += cb.c[i] * cb.in[i][n - 1];
        out[n - 1] = s;
    }
}

// Block partial sums of every dot product of the set; each block strides
// over the whole vector with a fixed assignment, so the result does not
// depend on timing.  (One pass per product: a fused pass over all products
// of a set, which reads a shared vector once, measured slower.)
__global__ __launch_bounds__(256) void k_dots(DotSet ds, double* partial) {
    __shared__ double red[4];
    for (int j = 0; j < ds.count; ++j) {
        const double* a = ds.a[j];
        const double* b = ds.b[j];
        double s = 0.0;
        for (long long k = blockIdx.x * 256LL + threadIdx.x; k < ds.n[j]; k += (long long)gridDim.x * 256)
            s += a[k] * b[k];
        s = block_sum<256>(s, red);
        if (threadIdx.x == 0) partial[j * gridDim.x + blockIdx.x] = s;
    }
}

// The same for 16-byte aligned vectors: two entries per lane and load, two
// loads of each vector in flight, partial sums in a fixed assignment.
__global__ __launch_bounds__(256) void k_dots2(DotSet ds, double* partial) {
    __shared__ double red[4];
    const long long st = (long long)gridDim.x * 256;
    for (int j = 0; j < ds.count; ++j) {
        const double2* a = reinterpret_cast<const double2*>(ds.a[j]);
        const double2* b = reinterpret_cast<const double2*>(ds.b[j]);
        const long long n2 = ds.n[j] >> 1;
        double s0 = 0.0, s1 = 0.0;
        long long k = blockIdx.x * 256LL + threadIdx.x;
        for (; k + st < n2; k += 2 * st) {
            const double2 x0 = a[k], y0 = b[k], x1 = a[k + st], y1 = b[k + st];
            s0 += x0.x * y0.x;
            s0 += x0.y * y0.y;
            s1 += x1.x * y1.x;
            s1 += x1.y * y1.y;
        }
        if (k < n2) {
            const double2 x0 = a[k], y0 = b[k];
            s0 += x0.x * y0.x;
            s0 += x0.y * y0.y;
        }
        double s = s0 + s1;
        if ((ds.n[j] & 1) && blockIdx.x == 0 && threadIdx.x == 0) s += ds.a[j][ds.n[j] - 1] * ds.b[j][ds.n[j] - 1];
        s = block_sum<256>(s, red);
        if (threadIdx.x == 0) partial[j * gridDim.x + blockIdx.x] = s;
    }
}

// Wavefront j adds the block partials of dot product j in a fixed order.
__global__ __launch_bounds__(64) void k_dots_final(const double* partial, int blocks, double* out) {
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < blocks; b += 64) s += partial[j * blocks + b];
    s = wave_sum(s);
    if (threadIdx.x == 0) out[j] = s;
}

// ---------------------------------------------------------------------------
// launchers (host side)
// ---------------------------------------------------------------------------

template <typename real, int R>
static hipError_t launch_phase_r(const ProbDev<real>* probs, const LaunchCfg& c, int phase, int par, int check,
                                 hipStream_t st) {
    const int waves = c.node_wg / 64;
    switch (phase) {
        case 0:
            if (c.dense == 2)
                hipLaunchKernelGGL((k_prep<real, R, 2>), dim3(c.n_node_tasks / waves), dim3(c.node_wg),
                                   c.node_lds, st, probs, c.node_tasks, c.node_info, c.wave_elems, par, check);
            else if (c.dense == 1)
                hipLaunchKernelGGL((k_prep<real, R, 1>), dim3(c.n_node_tasks / waves), dim3(c.node_wg),
                                   c.node_lds, st, probs, c.node_tasks, c.node_info, c.wave_elems, par, check);
            else
                hipLaunchKernelGGL((k_prep<real, R, 0>), dim3(c.n_node_tasks / waves), dim3(c.node_wg),
                                   c.node_lds, st, probs, c.node_tasks, c.node_info, c.wave_elems, par, check);
            break;
        case 1:
            if constexpr (sizeof(real) == 4)
                hipLaunchKernelGGL((k_bsweep_st<real, R>), dim3(c.n_leaf_tasks), dim3(64), c.sweep_lds, st, probs,
                                   c.leaf_tasks);
            else
                hipLaunchKernelGGL((k_bsweep<real, R>), dim3(c.n_leaf_tasks), dim3(64), c.sweep_lds, st, probs,
                                   c.leaf_tasks);
            break;
        case 2:
            if constexpr (sizeof(real) == 4)
                hipLaunchKernelGGL((k_fsweep_st<real, R>), dim3(c.n_leaf_tasks), dim3(64), c.sweep_lds, st, probs,
                                   c.leaf_tasks, par);
            else
                hipLaunchKernelGGL((k_fsweep<real, R>), dim3(c.n_leaf_tasks), dim3(64), c.sweep_lds, st, probs,
                                   c.leaf_tasks, par);
            break;
        default:
            if (c.dense == 2)
                hipLaunchKernelGGL((k_dual<real, R, 2>), dim3(c.n_node_tasks / waves), dim3(c.node_wg),
                                   c.node_lds, st, probs, c.node_tasks, c.node_info, c.wave_elems, par, check);
            else if (c.dense == 1)
                hipLaunchKernelGGL((k_dual<real, R, 1>), dim3(c.n_node_tasks / waves), dim3(c.node_wg),
                                   c.node_lds, st, probs, c.node_tasks, c.node_info, c.wave_elems, par, check);
            else
                hipLaunchKernelGGL((k_dual<real, R, 0>), dim3(c.n_node_tasks / waves), dim3(c.node_wg),
                                   c.node_lds, st, probs, c.node_tasks, c.node_info, c.wave_elems, par, check);
            break;
    }
    return hipGetLastError();
}

// One of the four launches of a CP step (0 prep, 1 bsweep, 2 fsweep, 3 dual).
template <typename real>
hipError_t launch_phase(const ProbDev<real>* probs, const LaunchCfg& c, int phase, int par, int check,
                        hipStream_t st) {
    if (phase < 0 || phase > 3 || c.n_leaf_tasks <= 0 || c.n_node_tasks <= 0) return hipErrorInvalidValue;
    if (c.node_wg != 64 && c.node_wg != 128 && c.node_wg != 256 && c.node_wg != 512) return hipErrorInvalidValue;
    switch (c.cls[phase]) {
        case kWideClass: return launch_phase_r<real, kWideClass>(probs, c, phase, par, check, st);
        case 16: return launch_phase_r<real, 16>(probs, c, phase, par, check, st);
        case 32: return launch_phase_r<real, 32>(probs, c, phase, par, check, st);
        case 64: return launch_phase_r<real, 64>(probs, c, phase, par, check, st);
        case 80: return launch_phase_r<real, 80>(probs, c, phase, par, check, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename real>
hipError_t launch_step(const ProbDev<real>* probs, const LaunchCfg& c, int par, int check, hipStream_t st) {
    for (int phase = 0; phase < 4; ++phase) {
        const hipError_t e = launch_phase<real>(probs, c, phase, par, check, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
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

hipError_t launch_combo(double* out, const VecCombo& cb, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (cb.n_in < 1 || cb.n_in > kMaxCombo) return hipErrorInvalidValue;
    bool aligned = (reinterpret_cast<uintptr_t>(out) & 15) == 0 && cb.n_in <= 3;
    for (int i = 0; i < cb.n_in; ++i) aligned = aligned && (reinterpret_cast<uintptr_t>(cb.in[i]) & 15) == 0;
    long long blocks = ((aligned ? (n + 1) / 2 : n) + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    const dim3 g((unsigned)blocks), b(256);
    if (!aligned) hipLaunchKernelGGL(k_combo, g, b, 0, st, out, cb, n);
    else if (cb.n_in == 1) hipLaunchKernelGGL(k_combo2<1>, g, b, 0, st, out, cb, n);
    else if (cb.n_in == 2) hipLaunchKernelGGL(k_combo2<2>, g, b, 0, st, out, cb, n);
    else hipLaunchKernelGGL(k_combo2<3>, g, b, 0, st, out, cb, n);
    return hipGetLastError();
}

// out[j] = <a_j, b_j> for the set; partial holds kMaxDots * kDotBlocks doubles.
hipError_t launch_dots(const DotSet& ds, double* partial, double* out, hipStream_t st) {
    if (ds.count < 1 || ds.count > kMaxDots) return hipErrorInvalidValue;
    bool aligned = true;
    for (int j = 0; j < ds.count; ++j)
        aligned = aligned && (reinterpret_cast<uintptr_t>(ds.a[j]) & 15) == 0 &&
                  (reinterpret_cast<uintptr_t>(ds.b[j]) & 15) == 0;
    if (aligned)
        hipLaunchKernelGGL(k_dots2, dim3(kDotBlocks), dim3(256), 0, st, ds, partial);
    else
        hipLaunchKernelGGL(k_dots, dim3(kDotBlocks), dim3(256), 0, st, ds, partial);
    hipLaunchKernelGGL(k_dots_final, dim3(ds.count), dim3(64), 0, st, (const double*)partial, kDotBlocks, out);
    return hipGetLastError();
}

#define SPK_INSTANTIATE(real)                                                                              \
    template hipError_t launch_step<real>(const ProbDev<real>*, const LaunchCfg&, int, int, hipStream_t);   \
    template hipError_t launch_phase<real>(const ProbDev<real>*, const LaunchCfg&, int, int, int,           \
                                           hipStream_t);                                                   \
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
