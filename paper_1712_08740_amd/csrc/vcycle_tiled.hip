// Temporally blocked V-cycle legs: one kernel per level and direction.
//
//   down (level l -> l+1):  x1 = w D^{-1} b,  x2 = x1 + w D^{-1}(b - M x1),
//                           r = b - M x2,     b_c = R r
//   up   (level l+1 -> l):  x' = x2 + P e,    x3 = x' + w D^{-1}(b - M x'),
//                           x4 = x3 + w D^{-1}(b - M x3)
//
// A block owns a tile and stages the data of the tile plus the halo the
// sweeps need in LDS: each sweep shrinks the region by one node, so the
// intermediate iterates never touch global memory. Nodes of the region that
// lie outside the grid hold 0 and have no coupling to grid nodes.
//
// The operator of a level is a policy: Fine5 (level 0: the matrix-free
// 5-point stencil of M with absorbing rows, coefficients from m^2) or Coarse9
// (Galerkin levels: 9 complex coefficient planes).
// Every tile shape must give the same bits: the node arithmetic below uses
// explicit fused multiply-adds, and nothing else in this file is contracted.
#pragma clang fp contract(off)
#include "hh_internal.h"

namespace hh {

namespace {

constexpr int NT = 128;    // threads per block

__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// a b
template <class C>
__device__ __forceinline__ C xmul(C a, C b) {
    C r;
    r.x = fmad(a.x, b.x, -(a.y * b.y));
    r.y = fmad(a.x, b.y, a.y * b.x);
    return r;
}
// acc + a b
template <class C>
__device__ __forceinline__ C xmuladd(C acc, C a, C b) {
    C r;
    r.x = fmad(a.x, b.x, fmad(-a.y, b.y, acc.x));
    r.y = fmad(a.x, b.y, fmad(a.y, b.x, acc.y));
    return r;
}
// acc + s a (s real)
template <class C, class T>
__device__ __forceinline__ C xaxpy(C acc, C a, T s) {
    C r;
    r.x = fmad(a.x, s, acc.x);
    r.y = fmad(a.y, s, acc.y);
    return r;
}
// one Jacobi update of a node: x + (b - (A x)) w
template <class C>
__device__ __forceinline__ C jacobi(C x, C b, C ax, C w) {
    return xmuladd(x, csub(b, ax), w);
}

// The flag may be cleared by a Givens step running as another workgroup of
// the same launch (the fine down leg hosts it): read it atomically. Blocks
// that still see it set do work the solver then ignores.
__device__ __forceinline__ bool inactive(const int* active) {
    return active && __hip_atomic_load(const_cast<int*>(active), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT) == 0;
}

// Row of the 5-point fine operator: a_p = diag, couplings -cx (x) and -cz (z).
template <class T>
struct Row5 {
    typename Cx<T>::type diag;
    T cx, cz;
};

template <class T>
struct Fine5 {
    typedef T real;
    typedef typename Cx<T>::type C;
    typedef Row5<T> Row;
    FineOpT<T> op;
    __host__ __device__ int nz() const { return op.nz; }
    __host__ __device__ int nx() const { return op.nx; }
    __device__ __forceinline__ Row row(int iz, int ix) const {
        const Coef5T<T> c = fine_coefs(op, iz, ix, op.m2[(int64_t)iz * op.nx + ix]);
        Row r;
        r.diag = c.diag;
        r.cx = c.cx;
        r.cz = c.cz;
        return r;
    }
    __device__ __forceinline__ C wd(int iz, int ix) const {
        return op.wdinv[(int64_t)iz * op.nx + ix];
    }
    // the stored data of row p (m^2), and the row built from it
    typedef T Raw;
    __device__ __forceinline__ Raw load_raw(int64_t p) const { return op.m2[p]; }
    __device__ __forceinline__ Row make_row(const Raw& m2p, int iz, int ix) const {
        const Coef5T<T> c = fine_coefs(op, iz, ix, m2p);
        Row r;
        r.diag = c.diag;
        r.cx = c.cx;
        r.cz = c.cz;
        return r;
    }
    __device__ __forceinline__ C wd_at(int64_t p) const { return op.wdinv[p]; }
    __device__ __forceinline__ static Row zero_row() {
        Row r;
        r.diag = cconv<C>(mk(1.0, 0.0));
        r.cx = r.cz = 0;
        return r;
    }
    // (A x)_q from the node value c and the sums of its x and z neighbours
    __device__ __forceinline__ static C apply5(const Row& r, C c, C sx, C sz) {
        return xaxpy(xaxpy(xmul(r.diag, c), sx, -r.cx), sz, -r.cz);
    }
    // (A x)_q from an LDS field s with row stride ld at local index i
    __device__ __forceinline__ C apply(const Row& r, const C* s, int i, int ld) const {
        return apply5(r, s[i], cadd(s[i - 1], s[i + 1]), cadd(s[i - ld], s[i + ld]));
    }
};

// Row of a 9-point Galerkin operator: coefficient t = (dz+1)*3 + (dx+1).
template <class T>
struct Row9 {
    typename Cx<T>::type a[9];
};

template <class T>
struct Coarse9 {
    typedef T real;
    typedef typename Cx<T>::type C;
    typedef Row9<T> Row;
    CoarseOpT<T> op;
    __host__ __device__ int nz() const { return op.nz; }
    __host__ __device__ int nx() const { return op.nx; }
    __device__ __forceinline__ Row row(int iz, int ix) const {
        const int64_t N = (int64_t)op.nz * op.nx;
        const int64_t p = (int64_t)iz * op.nx + ix;
        Row r;
#pragma unroll
        for (int t = 0; t < 9; ++t) r.a[t] = op.C[t * N + p];
        return r;
    }
    __device__ __forceinline__ C wd(int iz, int ix) const {
        return op.wdinv[(int64_t)iz * op.nx + ix];
    }
    // the stored data of row p (its 9 coefficients) is the row
    typedef Row Raw;
    __device__ __forceinline__ Raw load_raw(int64_t p) const {
        const int64_t N = (int64_t)op.nz * op.nx;
        Row r;
#pragma unroll
        for (int t = 0; t < 9; ++t) r.a[t] = op.C[t * N + p];
        return r;
    }
    __device__ __forceinline__ Row make_row(const Raw& raw, int, int) const { return raw; }
    __device__ __forceinline__ C wd_at(int64_t p) const { return op.wdinv[p]; }
    __device__ __forceinline__ static Row zero_row() {
        Row r;
#pragma unroll
        for (int t = 0; t < 9; ++t) r.a[t] = czero<C>();
        r.a[4] = cconv<C>(mk(1.0, 0.0));
        return r;
    }
    __device__ __forceinline__ C apply(const Row& r, const C* s, int i, int ld) const {
        C acc = czero<C>();
#pragma unroll
        for (int t = 0; t < 9; ++t) acc = xmuladd(acc, r.a[t], s[i + (t / 3 - 1) * ld + (t % 3 - 1)]);
        return acc;
    }
};

__device__ __forceinline__ bool in_grid(int z, int x, int nz, int nx) {
    return z >= 0 && z < nz && x >= 0 && x < nx;
}

// ---------------------------------------------------------------------------
// down leg. A block owns a TCX x TCZ tile of coarse nodes. Along a halved
// axis the fine region of the residual is [2c0 - 1, 2(c0 + TC) - 1], along
// an unhalved axis [c0, c0 + TC - 1]; x2 needs one more node on each side,
// x1 (and b, D) two more.
// ---------------------------------------------------------------------------
// SC is the type of src: complex128 on the fine level (the Krylov vector)
// whatever the precision of the cycle, the level's own type below.
template <class OP, class SC, int TCX, int TCZ>
__global__ void __launch_bounds__(NT) k_down(OP A, const SC* __restrict__ src,
                                             typename OP::C* __restrict__ x2out,
                                             int hz, int hx, CGrid cg,
                                             typename OP::C* __restrict__ bc, double rscale,
                                             const int* __restrict__ active, int ntx, int ntiles,
                                             int64_t bs) {
    typedef typename OP::C C;
    typedef typename OP::real T;
    constexpr int W1X = 2 * TCX + 5, W1Z = 2 * TCZ + 5;   // largest x1 region
    constexpr int TRASH = W1X * W1Z;                        // slot for stores past the region
    __shared__ C sb[W1X * W1Z + 1];
    __shared__ C sw[W1X * W1Z + 1];                         // omega_J / diag
    __shared__ C s1[W1X * W1Z + 1];
    __shared__ C s2[W1X * W1Z];
    __shared__ typename OP::Row srow[W1X * W1Z + 1];       // rows of the x1 region
    const int rb = blockIdx.y;                             // right-hand side
    active = rhs_at(active, rb, bs);
    if (inactive(active)) return;
    src = rhs_nn(src, rb, bs);
    x2out = rhs_nn(x2out, rb, bs);
    bc = rhs_nn(bc, rb, bs);
    const int tile = xcd_tile(blockIdx.x, ntiles);
    const int nz = A.nz(), nx = A.nx();
    const int cx0 = (tile % ntx) * TCX, cz0 = (tile / ntx) * TCZ;
    const int rlx = hx ? 2 * cx0 - 1 : cx0, rhx = hx ? 2 * (cx0 + TCX) - 1 : cx0 + TCX - 1;
    const int rlz = hz ? 2 * cz0 - 1 : cz0, rhz = hz ? 2 * (cz0 + TCZ) - 1 : cz0 + TCZ - 1;
    const int ox = rlx - 2, oz = rlz - 2;                  // origin of the x1 region
    const int wx = rhx - rlx + 5, wz = rhz - rlz + 5;      // x1 region size (row stride wx)
    const int olx = hx ? 2 * cx0 : cx0, ohx = hx ? 2 * (cx0 + TCX) - 1 : cx0 + TCX - 1;
    const int olz = hz ? 2 * cz0 : cz0, ohz = hz ? 2 * (cz0 + TCZ) - 1 : cz0 + TCZ - 1;
    const int n1 = wx * wz;
    constexpr int SL1 = (W1X * W1Z + NT - 1) / NT;
    // phase 1: b, the operator rows and x1 on the x1 region (the only global
    // reads). Every load of the thread is issued before any value is used:
    // nodes outside the grid or the region read node 0 and take zero values by
    // selection, and stores past the region go to a spare slot, so no load or
    // use sits under a branch (which made the loads of each node wait for the
    // previous node's).
    SC lb[SL1];
    C lw[SL1];
    typename OP::Raw lr[SL1];
#pragma unroll
    for (int k = 0; k < SL1; ++k) {
        const int i = threadIdx.x + k * NT;
        const int qz = oz + i / wx, qx = ox + i % wx;
        const bool ok = i < n1 && in_grid(qz, qx, nz, nx);
        const int64_t q = ok ? (int64_t)qz * nx + qx : 0;
        lb[k] = src[q];
        lw[k] = A.wd_at(q);
        lr[k] = A.load_raw(q);
    }
#pragma unroll
    for (int k = 0; k < SL1; ++k) {
        const int i = threadIdx.x + k * NT;
        const int qz = oz + i / wx, qx = ox + i % wx;
        const bool ok = i < n1 && in_grid(qz, qx, nz, nx);
        const C bq = ok ? cconv<C>(lb[k]) : czero<C>();
        const C wq = ok ? lw[k] : czero<C>();
        const typename OP::Row r = ok ? A.make_row(lr[k], qz, qx) : OP::zero_row();
        const int d = i < n1 ? i : TRASH;
        sb[d] = bq;
        sw[d] = wq;
        srow[d] = r;
        s1[d] = xmul(bq, wq);
    }
    __syncthreads();
    // phase 2: x2 on the x1 region shrunk by one node (stored at the same local index)
    const int w2x = wx - 2, n2 = w2x * (wz - 2);
#pragma unroll
    for (int k = 0; k < SL1; ++k) {
        const int j = threadIdx.x + k * NT;
        if (j < n2) {
            const int lz = 1 + j / w2x, lx = 1 + j % w2x;
            const int i = lz * wx + lx;
            const int qz = oz + lz, qx = ox + lx;
            C x2 = czero<C>();
            if (in_grid(qz, qx, nz, nx)) {
                const typename OP::Row& r = srow[i];
                const C ax = A.apply(r, s1, i, wx);
                x2 = jacobi(s1[i], sb[i], ax, sw[i]);
                if (qz >= olz && qz <= ohz && qx >= olx && qx <= ohx)
                    x2out[(int64_t)qz * nx + qx] = x2;
            }
            s2[i] = x2;
        }
    }
    __syncthreads();
    // phase 3: residual on the region shrunk by two nodes (into s1, no longer needed)
    const int w3x = wx - 4, n3 = w3x * (wz - 4);
#pragma unroll
    for (int k = 0; k < SL1; ++k) {
        const int j = threadIdx.x + k * NT;
        if (j < n3) {
            const int lz = 2 + j / w3x, lx = 2 + j % w3x;
            const int i = lz * wx + lx;
            const int qz = oz + lz, qx = ox + lx;
            C r = czero<C>();
            if (in_grid(qz, qx, nz, nx)) r = csub(sb[i], A.apply(srow[i], s2, i, wx));
            s1[i] = r;
        }
    }
    __syncthreads();
    // phase 4: b_c = R r for the tile's coarse nodes
    for (int t = threadIdx.x; t < TCX * TCZ; t += NT) {
        const int Iz = cz0 + t / TCX, Ix = cx0 + t % TCX;
        if (Iz >= cg.nz || Ix >= cg.nx) continue;
        const int lz = (hz ? 2 * Iz : Iz) - oz, lx = (hx ? 2 * Ix : Ix) - ox;
        C acc = czero<C>();
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if ((dz != 0 && !hz) || (dx != 0 && !hx)) continue;
                const T w = (dz == 0 ? (T)1 : (T)0.5) * (dx == 0 ? (T)1 : (T)0.5);
                acc = xaxpy(acc, s1[(lz + dz) * wx + (lx + dx)], w);
            }
        }
        bc[cg.at(Iz, Ix)] = cscale(acc, (T)rscale);
    }
}

// ---------------------------------------------------------------------------
// down leg of the fine 5-point level marching along z (both axes halved): one
// wavefront per block, its 64 lanes the fine columns x0 - 3 .. x0 + 60 of a
// strip whose 58 middle columns it owns, over the 8 rows z0 .. z0 + 7 it owns
// plus 3 rows above and 2 below. Every load of the block is issued first;
// x-neighbours come from the adjacent lanes (shuffles), z-neighbours from the
// lane's own registers, so there is no LDS and no barrier. Each node is
// computed with the same operations in the same order as in k_down: the two
// give the same bits.
constexpr int ZM_COLS = 58, ZM_ROWS = 8;

template <class T>
__device__ __forceinline__ typename Cx<T>::type lane_c(typename Cx<T>::type v, int src) {
    typename Cx<T>::type r;
    r.x = __shfl(v.x, src, 64);
    r.y = __shfl(v.y, src, 64);
    return r;
}

template <class T, class SC>
__global__ void __launch_bounds__(64) k_down_zmarch(FineOpT<T> op, const SC* __restrict__ src,
                                                    typename Cx<T>::type* __restrict__ x2out,
                                                    CGrid cg, typename Cx<T>::type* __restrict__ bc,
                                                    double rscale, const int* __restrict__ active,
                                                    int nstrips, int64_t bs) {
    typedef typename Cx<T>::type C;
    typedef Fine5<T> OP;
    constexpr int NR = ZM_ROWS + 5;                  // rows z0 - 3 .. z0 + ZM_ROWS + 1
    const int rb = blockIdx.y;
    active = rhs_at(active, rb, bs);
    if (inactive(active)) return;
    src = rhs_nn(src, rb, bs);
    x2out = rhs_nn(x2out, rb, bs);
    bc = rhs_nn(bc, rb, bs);
    const int lane = threadIdx.x;
    const int x0 = (blockIdx.x % nstrips) * ZM_COLS, z0 = (blockIdx.x / nstrips) * ZM_ROWS;
    const int x = x0 - 3 + lane;
    const int nz = op.nz, nx = op.nx;
    OP A;
    A.op = op;
    SC lb[NR];
    typename OP::Raw lr[NR];
    C lw[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int z = z0 - 3 + k;
        const bool ok = in_grid(z, x, nz, nx);
        const int64_t q = ok ? (int64_t)z * nx + x : 0;
        lb[k] = src[q];
        lr[k] = A.load_raw(q);
        lw[k] = A.wd_at(q);
    }
    const int lw1 = lane > 0 ? lane - 1 : 0, le1 = lane < 63 ? lane + 1 : 63;
    C b[NR], w[NR], x1[NR], x2[NR], r[NR];
    typename OP::Row rw[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int z = z0 - 3 + k;
        const bool ok = in_grid(z, x, nz, nx);
        b[k] = ok ? cconv<C>(lb[k]) : czero<C>();
        w[k] = ok ? lw[k] : czero<C>();
        rw[k] = ok ? A.make_row(lr[k], z, x) : OP::zero_row();
        x1[k] = xmul(b[k], w[k]);
    }
    // x2 on rows 1 .. NR - 2 (lanes 1 .. 62 hold valid values)
#pragma unroll
    for (int k = 1; k < NR - 1; ++k) {
        const int z = z0 - 3 + k;
        const bool ok = in_grid(z, x, nz, nx);
        const C sx = cadd(lane_c<T>(x1[k], lw1), lane_c<T>(x1[k], le1));
        const C ax = OP::apply5(rw[k], x1[k], sx, cadd(x1[k - 1], x1[k + 1]));
        x2[k] = ok ? jacobi(x1[k], b[k], ax, w[k]) : czero<C>();
        if (ok && k >= 3 && k < 3 + ZM_ROWS && lane >= 3 && lane < 3 + ZM_COLS)
            x2out[(int64_t)z * nx + x] = x2[k];
    }
    // residual on rows 2 .. NR - 3 (lanes 2 .. 61)
#pragma unroll
    for (int k = 2; k < NR - 2; ++k) {
        const int z = z0 - 3 + k;
        const bool ok = in_grid(z, x, nz, nx);
        const C sx = cadd(lane_c<T>(x2[k], lw1), lane_c<T>(x2[k], le1));
        r[k] = ok ? csub(b[k], OP::apply5(rw[k], x2[k], sx, cadd(x2[k - 1], x2[k + 1])))
                  : czero<C>();
    }
    // b_c = R r: coarse row z0/2 + i at fine row k = 3 + 2i, coarse column at lane 3 + 2j
    const bool own = lane >= 3 && lane < 3 + ZM_COLS && ((lane - 3) & 1) == 0;
#pragma unroll
    for (int i = 0; i < ZM_ROWS / 2; ++i) {
        const int k = 3 + 2 * i;
        const int I = (z0 >> 1) + i, J = (x0 >> 1) + ((lane - 3) >> 1);
        C rv[3][3];                                       // [dz + 1][dx + 1]
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            rv[d][0] = lane_c<T>(r[k - 1 + d], lw1);
            rv[d][1] = r[k - 1 + d];
            rv[d][2] = lane_c<T>(r[k - 1 + d], le1);
        }
        if (own && I < cg.nz && J < cg.nx) {
            C acc = czero<C>();
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const T wv = (dz == 0 ? (T)1 : (T)0.5) * (dx == 0 ? (T)1 : (T)0.5);
                    acc = xaxpy(acc, rv[dz + 1][dx + 1], wv);
                }
            }
            bc[cg.at(I, J)] = cscale(acc, (T)rscale);
        }
    }
}

// ---------------------------------------------------------------------------
// up leg. A block owns a TX x TZ tile of fine nodes: x' on the tile plus two
// nodes, x3 on the tile plus one, x4 on the tile.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void interp2(int q, int halved, int& J0, int& J1, T& w0, T& w1) {
    if (!halved) { J0 = J1 = q; w0 = 1; w1 = 0; return; }
    if ((q & 1) == 0) { J0 = J1 = q >> 1; w0 = 1; w1 = 0; return; }
    J0 = (q - 1) >> 1; J1 = J0 + 1; w0 = w1 = (T)0.5;
}

// SB is the type of b: complex128 on the fine level (the Krylov vector).
template <class OP, class SB, int TX, int TZ>
__global__ void __launch_bounds__(NT) k_up(OP A, int hz, int hx,
                                           const SB* __restrict__ b,
                                           const typename OP::C* __restrict__ x2,
                                           const typename OP::C* __restrict__ e, CGrid cg,
                                           typename OP::C* __restrict__ out,
                                           const int* __restrict__ active, int ntx, int ntiles,
                                           int64_t bs) {
    typedef typename OP::C C;
    typedef typename OP::real T;
    const int rb = blockIdx.y;                             // right-hand side
    active = rhs_at(active, rb, bs);
    if (inactive(active)) return;
    b = rhs_nn(b, rb, bs);
    x2 = rhs_nn(x2, rb, bs);
    e = rhs_nn(e, rb, bs);
    out = rhs_nn(out, rb, bs);
    constexpr int WX = TX + 4, WZ = TZ + 4;
    constexpr int W3X = TX + 2, W3Z = TZ + 2;
    constexpr int TRASH = WX * WZ, TRASH3 = W3X * W3Z;   // slots for stores past the regions
    __shared__ C sp[WX * WZ + 1];                     // x' (tile + 2)
    __shared__ C s3[WX * WZ];                         // x3 (tile + 1)
    __shared__ C sbb[W3X * W3Z + 1];                  // b on the tile + 1
    __shared__ C sw[W3X * W3Z + 1];                   // omega_J / diag on the tile + 1
    __shared__ typename OP::Row srow[W3X * W3Z + 1];  // rows on the tile + 1
    const int nz = A.nz(), nx = A.nx();
    const int tile = xcd_tile(blockIdx.x, ntiles);
    const int fx0 = (tile % ntx) * TX, fz0 = (tile / ntx) * TZ;
    const int ox = fx0 - 2, oz = fz0 - 2;
    constexpr int SL = (WX * WZ + NT - 1) / NT;
    constexpr int SL3 = (W3X * W3Z + NT - 1) / NT;
    // phase 1: x' = x2 + P e on the tile + 2; b and rows on the tile + 1.
    // Every load of the thread is issued before any value is used (nodes
    // outside the grid or the regions read node 0 and take zero values by
    // selection; stores past a region go to a spare slot).
    C le[SL][4], lx[SL];
    SB lb[SL3];
    C lw[SL3];
    typename OP::Raw lr[SL3];
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int i = threadIdx.x + k * NT;
        const int qz = oz + i / WX, qx = ox + i % WX;
        const bool ok = i < WX * WZ && in_grid(qz, qx, nz, nx);
        int z0, z1, x0, x1;
        T wz0, wz1, wx0, wx1;
        interp2(qz, hz, z0, z1, wz0, wz1);
        interp2(qx, hx, x0, x1, wx0, wx1);
        le[k][0] = e[ok ? cg.at(z0, x0) : 0];
        le[k][1] = e[ok ? cg.at(z0, x1) : 0];
        le[k][2] = e[ok ? cg.at(z1, x0) : 0];
        le[k][3] = e[ok ? cg.at(z1, x1) : 0];
        lx[k] = x2[ok ? (int64_t)qz * nx + qx : 0];
    }
#pragma unroll
    for (int k = 0; k < SL3; ++k) {
        const int j = threadIdx.x + k * NT;
        const int qz = fz0 - 1 + j / W3X, qx = fx0 - 1 + j % W3X;
        const bool ok = j < W3X * W3Z && in_grid(qz, qx, nz, nx);
        const int64_t q = ok ? (int64_t)qz * nx + qx : 0;
        lb[k] = b[q];
        lw[k] = A.wd_at(q);
        lr[k] = A.load_raw(q);
    }
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int i = threadIdx.x + k * NT;
        const int qz = oz + i / WX, qx = ox + i % WX;
        const bool ok = i < WX * WZ && in_grid(qz, qx, nz, nx);
        int z0, z1, x0, x1;
        T wz0, wz1, wx0, wx1;
        interp2(qz, hz, z0, z1, wz0, wz1);
        interp2(qx, hx, x0, x1, wx0, wx1);
        const C pe = xaxpy(xaxpy(xaxpy(cscale(le[k][0], wz0 * wx0), le[k][1], wz0 * wx1),
                                 le[k][2], wz1 * wx0), le[k][3], wz1 * wx1);
        sp[i < WX * WZ ? i : TRASH] = ok ? cadd(lx[k], pe) : czero<C>();
    }
#pragma unroll
    for (int k = 0; k < SL3; ++k) {
        const int j = threadIdx.x + k * NT;
        const int qz = fz0 - 1 + j / W3X, qx = fx0 - 1 + j % W3X;
        const bool ok = j < W3X * W3Z && in_grid(qz, qx, nz, nx);
        const int d = j < W3X * W3Z ? j : TRASH3;
        srow[d] = ok ? A.make_row(lr[k], qz, qx) : OP::zero_row();
        sbb[d] = ok ? cconv<C>(lb[k]) : czero<C>();
        sw[d] = ok ? lw[k] : czero<C>();
    }
    __syncthreads();
    // phase 2: x3 on the tile plus one node
#pragma unroll
    for (int k = 0; k < SL3; ++k) {
        const int j = threadIdx.x + k * NT;
        if (j < W3X * W3Z) {
            const int lz = 1 + j / W3X, lx = 1 + j % W3X;
            const int i = lz * WX + lx;
            const int qz = oz + lz, qx = ox + lx;
            C v = czero<C>();
            if (in_grid(qz, qx, nz, nx)) {
                const typename OP::Row& r = srow[j];
                const C ax = A.apply(r, sp, i, WX);
                v = jacobi(sp[i], sbb[j], ax, sw[j]);
            }
            s3[i] = v;
        }
    }
    __syncthreads();
    // phase 3: x4 on the tile
    constexpr int SL4 = (TX * TZ + NT - 1) / NT;
#pragma unroll
    for (int k = 0; k < SL4; ++k) {
        const int t = threadIdx.x + k * NT;
        if (t < TX * TZ) {
            const int lz = 2 + t / TX, lx = 2 + t % TX;
            const int i = lz * WX + lx;
            const int j = (lz - 1) * W3X + (lx - 1);
            const int qz = oz + lz, qx = ox + lx;
            if (in_grid(qz, qx, nz, nx)) {
                const typename OP::Row& r = srow[j];
                const C ax = A.apply(r, s3, i, WX);
                out[(int64_t)qz * nx + qx] = jacobi(s3[i], sbb[j], ax, sw[j]);
            }
        }
    }
}

inline double inv2dc(int hz, int hx) { return 1.0 / (double)((hz ? 2 : 1) * (hx ? 2 : 1)); }

// the up leg on 5-point grids of at least this many nodes takes large tiles
constexpr int64_t kBigLevel = 200000;

template <class OP>
bool big_tiles(const OP& A) {
    if constexpr (sizeof(typename OP::Row) <= 32)
        return (int64_t)A.nz() * A.nx() >= kBigLevel;
    return false;
}

template <class OP, class SC, int TCX, int TCZ>
hipError_t down_launch(const OP& A, const SC* src, typename OP::C* x2, int hz, int hx, CGrid cg,
                       typename OP::C* bc, const int* active, hipStream_t s,
                       const Batch& bt) {
    const int ntx = (cg.nx + TCX - 1) / TCX, ntz = (cg.nz + TCZ - 1) / TCZ;
    const int ntiles = ntx * ntz;
    HH_LAUNCH((k_down<OP, SC, TCX, TCZ>), dim3(ntiles, bt.n), dim3(NT), 0, s, A, src, x2, hz, hx,
              cg, bc, inv2dc(hz, hx), active, ntx, ntiles, bt.bs);
    return hipGetLastError();
}

// Tile shapes of the down leg (coarse nodes): 0 = 4 x 4 (an 8 x 8 fine block
// and its halo), 1 = 8 x 4, 2 = the fine level marching along z (k_down_zmarch;
// other levels, or a fine level not halved in both axes, take 4 x 4). The
// default (tile < 0): 4 x 4 tiles, which beat larger ones up to a few 100k
// nodes (more blocks in flight against the latency, measured on the 401 x 201
// and 1201 x 401 hierarchies), except on 5-point fine grids of at least
// kBigLevel nodes, where marching along z is faster (1201 x 401: 16.0 -> 13.1 us
// in complex128, 11.4 -> 8.3 us in complex64; slower on 401 x 201). Every shape
// computes every node with the same arithmetic: the choice changes speed, not
// results.
template <class OP, class SC>
hipError_t down_dispatch(const OP& A, const SC* src, typename OP::C* x2, int hz, int hx, CGrid cg,
                         typename OP::C* bc, const int* active, hipStream_t s,
                         const Batch& bt, int tile) {
    if constexpr (sizeof(typename OP::Row) <= 32) {      // the fine 5-point level
        if (tile < 0) tile = big_tiles(A) ? 2 : 0;
        if (tile == 2 && hz && hx) {
            const int nstrips = (A.nx() + ZM_COLS - 1) / ZM_COLS;
            const int nchunks = (A.nz() + ZM_ROWS - 1) / ZM_ROWS;
            HH_LAUNCH((k_down_zmarch<typename OP::real, SC>), dim3(nstrips * nchunks, bt.n),
                      dim3(64), 0, s, A.op, src, x2, cg, bc, inv2dc(hz, hx), active, nstrips,
                      bt.bs);
            return hipGetLastError();
        }
    }
    if (tile == 1) return down_launch<OP, SC, 8, 4>(A, src, x2, hz, hx, cg, bc, active, s, bt);
    return down_launch<OP, SC, 4, 4>(A, src, x2, hz, hx, cg, bc, active, s, bt);
}

template <class OP, class SB, int TX, int TZ>
hipError_t up_launch(const OP& A, int hz, int hx, const SB* b, const typename OP::C* x2,
                     const typename OP::C* e, CGrid cg, typename OP::C* out, const int* active,
                     hipStream_t s, const Batch& bt) {
    const int ntx = (A.nx() + TX - 1) / TX, ntz = (A.nz() + TZ - 1) / TZ;
    HH_LAUNCH((k_up<OP, SB, TX, TZ>), dim3(ntx * ntz, bt.n), dim3(NT), 0, s, A, hz, hx, b, x2, e,
              cg, out, active, ntx, ntx * ntz, bt.bs);
    return hipGetLastError();
}

// Tile shapes of the up leg (fine nodes): 0 = 8 x 4, 1 = 16 x 8, 2 = 32 x 8.
// The default (tile < 0) is 8 x 4, and 32 x 8 (less halo work) on large
// 5-point grids. Results do not depend on the choice.
template <class OP, class SB>
hipError_t up_dispatch(const OP& A, int hz, int hx, const SB* b, const typename OP::C* x2,
                       const typename OP::C* e, CGrid cg, typename OP::C* out, const int* active,
                       hipStream_t s, const Batch& bt, int tile) {
    if (tile < 0) tile = big_tiles(A) ? 2 : 0;
    if (tile == 2) return up_launch<OP, SB, 32, 8>(A, hz, hx, b, x2, e, cg, out, active, s, bt);
    if (tile == 1) return up_launch<OP, SB, 16, 8>(A, hz, hx, b, x2, e, cg, out, active, s, bt);
    return up_launch<OP, SB, 8, 4>(A, hz, hx, b, x2, e, cg, out, active, s, bt);
}

template <class T>
Fine5<T> fine5(const FineOpT<T>& op) {
    Fine5<T> A;
    A.op = op;
    return A;
}
template <class T>
Coarse9<T> coarse9(const CoarseOpT<T>& op) {
    Coarse9<T> A;
    A.op = op;
    return A;
}

}  // namespace

hipError_t launch_vc_fine_down(const FineOp& op, const cplx* src, cplx* x2, int hz, int hx,
                               CGrid cg, cplx* bc, const int* active, hipStream_t s,
                               const Batch& bt, int tile) {
    return down_dispatch(fine5(op), src, x2, hz, hx, cg, bc, active, s, bt, tile);
}
hipError_t launch_vc_fine_down(const FineOpT<float>& op, const cplx* src, cplxf* x2, int hz,
                               int hx, CGrid cg, cplxf* bc, const int* active,
                               hipStream_t s, const Batch& bt, int tile) {
    return down_dispatch(fine5(op), src, x2, hz, hx, cg, bc, active, s, bt, tile);
}

hipError_t launch_vc_coarse_down(const CoarseOp& op, const cplx* b, cplx* x2, int hz, int hx,
                                 CGrid cg, cplx* bc, const int* active, hipStream_t s,
                                 const Batch& bt, int tile) {
    return down_dispatch(coarse9(op), b, x2, hz, hx, cg, bc, active, s, bt, tile);
}
hipError_t launch_vc_coarse_down(const CoarseOpT<float>& op, const cplxf* b, cplxf* x2, int hz,
                                 int hx, CGrid cg, cplxf* bc, const int* active,
                                 hipStream_t s, const Batch& bt, int tile) {
    return down_dispatch(coarse9(op), b, x2, hz, hx, cg, bc, active, s, bt, tile);
}

hipError_t launch_vc_fine_up(const FineOp& op, int hz, int hx, const cplx* b, const cplx* x2,
                             const cplx* e, CGrid cg, cplx* out, const int* active, hipStream_t s,
                             const Batch& bt, int tile) {
    return up_dispatch(fine5(op), hz, hx, b, x2, e, cg, out, active, s, bt, tile);
}
hipError_t launch_vc_fine_up(const FineOpT<float>& op, int hz, int hx, const cplx* b,
                             const cplxf* x2, const cplxf* e, CGrid cg, cplxf* out,
                             const int* active, hipStream_t s, const Batch& bt, int tile) {
    return up_dispatch(fine5(op), hz, hx, b, x2, e, cg, out, active, s, bt, tile);
}

hipError_t launch_vc_coarse_up(const CoarseOp& op, int hz, int hx, const cplx* b, const cplx* x2,
                               const cplx* e, CGrid cg, cplx* out, const int* active,
                               hipStream_t s, const Batch& bt, int tile) {
    return up_dispatch(coarse9(op), hz, hx, b, x2, e, cg, out, active, s, bt, tile);
}
hipError_t launch_vc_coarse_up(const CoarseOpT<float>& op, int hz, int hx, const cplxf* b,
                               const cplxf* x2, const cplxf* e, CGrid cg, cplxf* out,
                               const int* active, hipStream_t s, const Batch& bt, int tile) {
    return up_dispatch(coarse9(op), hz, hx, b, x2, e, cg, out, active, s, bt, tile);
}

namespace {
__global__ void __launch_bounds__(256) k_wdinv_fine(FineOp op, double wj, cplx* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)op.nz * op.nx) return;
    const int iz = (int)(p / op.nx), ix = (int)(p - (int64_t)iz * op.nx);
    out[p] = cscale(crecip(fine_coefs(op, iz, ix, op.m2[p]).diag), wj);
}
__global__ void __launch_bounds__(256) k_wdinv_coarse(CoarseOp op, double wj,
                                                      cplx* __restrict__ out) {
    const int64_t N = (int64_t)op.nz * op.nx;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= N) return;
    out[p] = cscale(crecip(op.C[4 * N + p]), wj);
}
}  // namespace

hipError_t launch_wdinv_fine(const FineOp& op, double wj, cplx* wdinv, hipStream_t s) {
    const int64_t n = (int64_t)op.nz * op.nx;
    HH_LAUNCH(k_wdinv_fine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, op, wj, wdinv);
    return hipGetLastError();
}

hipError_t launch_wdinv_coarse(const CoarseOp& op, double wj, cplx* wdinv, hipStream_t s) {
    const int64_t n = (int64_t)op.nz * op.nx;
    HH_LAUNCH(k_wdinv_coarse, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, op, wj, wdinv);
    return hipGetLastError();
}

}  // namespace hh
