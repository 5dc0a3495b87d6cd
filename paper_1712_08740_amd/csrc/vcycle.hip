// Fused kernels of one V(2,2) omega-Jacobi multigrid cycle on the shifted
// Laplacian (the approximate M^{-1} of Eq. 6-7). Per level four launches:
//
//   presmooth      x2 = two sweeps from x = 0:  x1 = w D^{-1} b,
//                  x2 = x1 + w D^{-1} (b - M x1)          (x1 recomputed at the
//                  neighbours, never stored)
//   resid_restrict b_c = R (b - M x2)                     (residual recomputed at
//                  the fine nodes of R's support, never stored)
//   prolong_post1  x3 = x' + w D^{-1} (b - M x'),  x' = x2 + P e_c
//   post2          x4 = x3 + w D^{-1} (b - M x3)
//
// Level 0 is the matrix-free 5-point operator M itself; coarser levels are the
// 9-point Galerkin operators (coefficient planes C[t*N + p]).
//
// The level-0 presmooth also normalises the Arnoldi vector: it reads the
// unnormalised w and the scale 1/||w|| from device memory and writes v = w/||w||
// into the Krylov basis. Every kernel takes an optional device flag `active`;
// when it reads 0 the kernel returns at once, which lets the host enqueue
// Arnoldi steps ahead of the convergence decision.
#include "hh_internal.h"

namespace hh {

namespace {

constexpr int BX = 64;
constexpr int BZ = 4;

dim3 grid2(int nz, int nx) { return dim3((nx + BX - 1) / BX, (nz + BZ - 1) / BZ); }

__device__ __forceinline__ bool inactive(const int* active) { return active && *active == 0; }

// Linear interpolation along one axis at fine index q: always two coarse
// nodes (J0, J1) with weights (w0, w1); unused slots repeat J0 with weight 0,
// so the loads are straight-line.
__device__ __forceinline__ void interp2(int q, int halved, int& J0, int& J1, double& w0,
                                        double& w1) {
    if (!halved) { J0 = J1 = q; w0 = 1.0; w1 = 0.0; return; }
    if ((q & 1) == 0) { J0 = J1 = q >> 1; w0 = 1.0; w1 = 0.0; return; }
    J0 = (q - 1) >> 1; J1 = J0 + 1; w0 = w1 = 0.5;
}

// (P e)_q at fine node (qz, qx)
__device__ __forceinline__ cplx prolong_at(const cplx* e, int nxc, int hz, int hx, int qz, int qx) {
    int z0, z1, x0, x1;
    double wz0, wz1, wx0, wx1;
    interp2(qz, hz, z0, z1, wz0, wz1);
    interp2(qx, hx, x0, x1, wx0, wx1);
    const cplx e00 = e[(int64_t)z0 * nxc + x0], e01 = e[(int64_t)z0 * nxc + x1];
    const cplx e10 = e[(int64_t)z1 * nxc + x0], e11 = e[(int64_t)z1 * nxc + x1];
    return cadd(cadd(cscale(e00, wz0 * wx0), cscale(e01, wz0 * wx1)),
                cadd(cscale(e10, wz1 * wx0), cscale(e11, wz1 * wx1)));
}

// ---------------------------------------------------------------------------
// level 0: 5-point operator. Neighbours in the order W, E, N, S; a neighbour
// outside the grid is replaced by the node itself with coupling 0.
// ---------------------------------------------------------------------------
struct Nbr5 {
    int64_t q[4];
    int qz[4], qx[4];
    double c[4];           // coupling magnitude (entry is -c), 0 outside the grid
};

__device__ __forceinline__ Nbr5 nbrs5(const FineOp& op, const Coef5& cp, int iz, int ix,
                                      int64_t p) {
    Nbr5 r;
    const bool w = ix > 0, e = ix < op.nx - 1, n = iz > 0, s = iz < op.nz - 1;
    r.q[0] = w ? p - 1 : p;      r.qz[0] = iz;            r.qx[0] = w ? ix - 1 : ix; r.c[0] = w ? cp.cx : 0.0;
    r.q[1] = e ? p + 1 : p;      r.qz[1] = iz;            r.qx[1] = e ? ix + 1 : ix; r.c[1] = e ? cp.cx : 0.0;
    r.q[2] = n ? p - op.nx : p;  r.qz[2] = n ? iz - 1 : iz; r.qx[2] = ix;            r.c[2] = n ? cp.cz : 0.0;
    r.q[3] = s ? p + op.nx : p;  r.qz[3] = s ? iz + 1 : iz; r.qx[3] = ix;            r.c[3] = s ? cp.cz : 0.0;
    return r;
}

__global__ void __launch_bounds__(256) k_fine_presmooth(FineOp op, double wj,
                                                        const cplx* __restrict__ src,
                                                        const double* __restrict__ scale,
                                                        cplx* __restrict__ bout,
                                                        cplx* __restrict__ xo,
                                                        const int* __restrict__ active) {
    if (inactive(active)) return;
    const int ix = blockIdx.x * BX + threadIdx.x;
    const int iz = blockIdx.y * BZ + threadIdx.y;
    if (ix >= op.nx || iz >= op.nz) return;
    const int64_t p = (int64_t)iz * op.nx + ix;
    const double s = scale ? scale[0] : 1.0;
    const Coef5 cp = fine_coefs(op, iz, ix, op.m2[p]);
    const Nbr5 nb = nbrs5(op, cp, iz, ix, p);
    cplx sq[4];
    double mq[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        sq[t] = src[nb.q[t]];
        mq[t] = op.m2[nb.q[t]];
    }
    const cplx bp = cscale(src[p], s);
    if (bout) bout[p] = bp;
    const cplx x1p = cscale(cdiv(bp, cp.diag), wj);
    cplx ax = cmul(cp.diag, x1p);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const Coef5 cq = fine_coefs(op, nb.qz[t], nb.qx[t], mq[t]);
        const cplx x1q = cscale(cdiv(cscale(sq[t], s), cq.diag), wj);
        ax = csub(ax, cscale(x1q, nb.c[t]));
    }
    xo[p] = cadd(x1p, cscale(cdiv(csub(bp, ax), cp.diag), wj));
}

// b_c = R (b - M x)
__global__ void __launch_bounds__(256) k_fine_resid_restrict(FineOp op, int hz, int hx,
                                                             const cplx* __restrict__ b,
                                                             const cplx* __restrict__ x,
                                                             int nzc, int nxc,
                                                             cplx* __restrict__ bc,
                                                             double scale,
                                                             const int* __restrict__ active) {
    if (inactive(active)) return;
    const int Ix = blockIdx.x * BX + threadIdx.x;
    const int Iz = blockIdx.y * BZ + threadIdx.y;
    if (Ix >= nxc || Iz >= nzc) return;
    const int fz = hz ? 2 * Iz : Iz;
    const int fx = hx ? 2 * Ix : Ix;
    cplx acc = mk(0.0, 0.0);
#pragma unroll 1
    for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int qz0 = fz + dz, qx0 = fx + dx;
            const bool in = (dz == 0 || hz) && (dx == 0 || hx) && qz0 >= 0 && qz0 < op.nz &&
                            qx0 >= 0 && qx0 < op.nx;
            const int qz = in ? qz0 : fz, qx = in ? qx0 : fx;
            const int64_t q = (int64_t)qz * op.nx + qx;
            const Coef5 c = fine_coefs(op, qz, qx, op.m2[q]);
            const Nbr5 nb = nbrs5(op, c, qz, qx, q);
            cplx ax = cmul(c.diag, x[q]);
#pragma unroll
            for (int t = 0; t < 4; ++t) ax = csub(ax, cscale(x[nb.q[t]], nb.c[t]));
            const double w = in ? (dz == 0 ? 1.0 : 0.5) * (dx == 0 ? 1.0 : 0.5) : 0.0;
            acc = cadd(acc, cscale(csub(b[q], ax), w));
        }
    }
    bc[(int64_t)Iz * nxc + Ix] = cscale(acc, scale);
}

// x3 = x' + w D^{-1} (b - M x'),  x' = x + P e
__global__ void __launch_bounds__(256) k_fine_prolong_post1(FineOp op, double wj, int hz, int hx,
                                                            const cplx* __restrict__ b,
                                                            const cplx* __restrict__ x,
                                                            const cplx* __restrict__ e,
                                                            int nxc, cplx* __restrict__ xo,
                                                            const int* __restrict__ active) {
    if (inactive(active)) return;
    const int ix = blockIdx.x * BX + threadIdx.x;
    const int iz = blockIdx.y * BZ + threadIdx.y;
    if (ix >= op.nx || iz >= op.nz) return;
    const int64_t p = (int64_t)iz * op.nx + ix;
    const Coef5 cp = fine_coefs(op, iz, ix, op.m2[p]);
    const Nbr5 nb = nbrs5(op, cp, iz, ix, p);
    const cplx xp = cadd(x[p], prolong_at(e, nxc, hz, hx, iz, ix));
    cplx ax = cmul(cp.diag, xp);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const cplx xq = cadd(x[nb.q[t]], prolong_at(e, nxc, hz, hx, nb.qz[t], nb.qx[t]));
        ax = csub(ax, cscale(xq, nb.c[t]));
    }
    xo[p] = cadd(xp, cscale(cdiv(csub(b[p], ax), cp.diag), wj));
}

__global__ void __launch_bounds__(256) k_fine_post2(FineOp op, double wj,
                                                    const cplx* __restrict__ b,
                                                    const cplx* __restrict__ x,
                                                    cplx* __restrict__ xo,
                                                    const int* __restrict__ active) {
    if (inactive(active)) return;
    const int ix = blockIdx.x * BX + threadIdx.x;
    const int iz = blockIdx.y * BZ + threadIdx.y;
    if (ix >= op.nx || iz >= op.nz) return;
    const int64_t p = (int64_t)iz * op.nx + ix;
    const Coef5 cp = fine_coefs(op, iz, ix, op.m2[p]);
    const Nbr5 nb = nbrs5(op, cp, iz, ix, p);
    const cplx xp = x[p];
    cplx ax = cmul(cp.diag, xp);
#pragma unroll
    for (int t = 0; t < 4; ++t) ax = csub(ax, cscale(x[nb.q[t]], nb.c[t]));
    xo[p] = cadd(xp, cscale(cdiv(csub(b[p], ax), cp.diag), wj));
}

// ---------------------------------------------------------------------------
// coarse levels: 9-point Galerkin operators. Coefficients towards neighbours
// outside the grid are exactly 0, so those neighbours are read at the clamped
// (in-grid) index and contribute nothing.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t clamp_nbr(const CoarseOp& op, int iz, int ix, int dz, int dx) {
    int qz = iz + dz, qx = ix + dx;
    qz = qz < 0 ? 0 : (qz >= op.nz ? op.nz - 1 : qz);
    qx = qx < 0 ? 0 : (qx >= op.nx ? op.nx - 1 : qx);
    return (int64_t)qz * op.nx + qx;
}

__device__ __forceinline__ cplx coarse_row(const CoarseOp& op, const cplx* x, int iz, int ix,
                                           int64_t p, int64_t N) {
    cplx acc = mk(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int64_t q = clamp_nbr(op, iz, ix, t / 3 - 1, t % 3 - 1);
        acc = cadd(acc, cmul(op.C[t * N + p], x[q]));
    }
    return acc;
}

__global__ void __launch_bounds__(256) k_coarse_presmooth(CoarseOp op, double wj,
                                                          const cplx* __restrict__ b,
                                                          cplx* __restrict__ xo,
                                                          const int* __restrict__ active) {
    if (inactive(active)) return;
    const int ix = blockIdx.x * BX + threadIdx.x;
    const int iz = blockIdx.y * BZ + threadIdx.y;
    if (ix >= op.nx || iz >= op.nz) return;
    const int64_t N = (int64_t)op.nz * op.nx;
    const int64_t p = (int64_t)iz * op.nx + ix;
    const cplx dp = op.C[4 * N + p];
    const cplx bp = b[p];
    const cplx x1p = cscale(cdiv(bp, dp), wj);
    cplx ax = mk(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int64_t q = clamp_nbr(op, iz, ix, t / 3 - 1, t % 3 - 1);
        const cplx x1q = (t == 4) ? x1p : cscale(cdiv(b[q], op.C[4 * N + q]), wj);
        ax = cadd(ax, cmul(op.C[t * N + p], x1q));
    }
    xo[p] = cadd(x1p, cscale(cdiv(csub(bp, ax), dp), wj));
}

__global__ void __launch_bounds__(256) k_coarse_resid_restrict(CoarseOp op, int hz, int hx,
                                                               const cplx* __restrict__ b,
                                                               const cplx* __restrict__ x,
                                                               int nzc, int nxc,
                                                               cplx* __restrict__ bc,
                                                               double scale,
                                                               const int* __restrict__ active) {
    if (inactive(active)) return;
    const int Ix = blockIdx.x * BX + threadIdx.x;
    const int Iz = blockIdx.y * BZ + threadIdx.y;
    if (Ix >= nxc || Iz >= nzc) return;
    const int64_t N = (int64_t)op.nz * op.nx;
    const int fz = hz ? 2 * Iz : Iz;
    const int fx = hx ? 2 * Ix : Ix;
    cplx acc = mk(0.0, 0.0);
#pragma unroll 1
    for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int qz0 = fz + dz, qx0 = fx + dx;
            const bool in = (dz == 0 || hz) && (dx == 0 || hx) && qz0 >= 0 && qz0 < op.nz &&
                            qx0 >= 0 && qx0 < op.nx;
            const int qz = in ? qz0 : fz, qx = in ? qx0 : fx;
            const int64_t q = (int64_t)qz * op.nx + qx;
            const cplx r = csub(b[q], coarse_row(op, x, qz, qx, q, N));
            const double w = in ? (dz == 0 ? 1.0 : 0.5) * (dx == 0 ? 1.0 : 0.5) : 0.0;
            acc = cadd(acc, cscale(r, w));
        }
    }
    bc[(int64_t)Iz * nxc + Ix] = cscale(acc, scale);
}

__global__ void __launch_bounds__(256) k_coarse_prolong_post1(CoarseOp op, double wj, int hz,
                                                              int hx, const cplx* __restrict__ b,
                                                              const cplx* __restrict__ x,
                                                              const cplx* __restrict__ e,
                                                              int nxc, cplx* __restrict__ xo,
                                                              const int* __restrict__ active) {
    if (inactive(active)) return;
    const int ix = blockIdx.x * BX + threadIdx.x;
    const int iz = blockIdx.y * BZ + threadIdx.y;
    if (ix >= op.nx || iz >= op.nz) return;
    const int64_t N = (int64_t)op.nz * op.nx;
    const int64_t p = (int64_t)iz * op.nx + ix;
    cplx ax = mk(0.0, 0.0);
    cplx xp = mk(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        int qz = iz + t / 3 - 1, qx = ix + t % 3 - 1;
        qz = qz < 0 ? 0 : (qz >= op.nz ? op.nz - 1 : qz);
        qx = qx < 0 ? 0 : (qx >= op.nx ? op.nx - 1 : qx);
        const int64_t q = (int64_t)qz * op.nx + qx;
        const cplx xq = cadd(x[q], prolong_at(e, nxc, hz, hx, qz, qx));
        if (t == 4) xp = xq;
        ax = cadd(ax, cmul(op.C[t * N + p], xq));
    }
    xo[p] = cadd(xp, cscale(cdiv(csub(b[p], ax), op.C[4 * N + p]), wj));
}

__global__ void __launch_bounds__(256) k_coarse_post2(CoarseOp op, double wj,
                                                      const cplx* __restrict__ b,
                                                      const cplx* __restrict__ x,
                                                      cplx* __restrict__ xo,
                                                      const int* __restrict__ active) {
    if (inactive(active)) return;
    const int ix = blockIdx.x * BX + threadIdx.x;
    const int iz = blockIdx.y * BZ + threadIdx.y;
    if (ix >= op.nx || iz >= op.nz) return;
    const int64_t N = (int64_t)op.nz * op.nx;
    const int64_t p = (int64_t)iz * op.nx + ix;
    const cplx ax = coarse_row(op, x, iz, ix, p, N);
    xo[p] = cadd(x[p], cscale(cdiv(csub(b[p], ax), op.C[4 * N + p]), wj));
}

// y = A x for the coarsest dense inverse; one 256-thread block per row
__global__ void __launch_bounds__(256) k_gemv_pred(int n, const cplx* __restrict__ A,
                                                   const cplx* __restrict__ x,
                                                   cplx* __restrict__ y,
                                                   const int* __restrict__ active) {
    if (inactive(active)) return;
    __shared__ cplx sh[4];
    const int i = blockIdx.x;
    const int tid = threadIdx.x;
    const cplx* row = A + (int64_t)i * n;
    cplx acc = mk(0.0, 0.0);
    for (int j = tid; j < n; j += 256) acc = cadd(acc, cmul(row[j], x[j]));
    for (int off = 32; off > 0; off >>= 1) {
        acc.x += __shfl_down(acc.x, off, 64);
        acc.y += __shfl_down(acc.y, off, 64);
    }
    if ((tid & 63) == 0) sh[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) y[i] = cadd(cadd(sh[0], sh[1]), cadd(sh[2], sh[3]));
}

inline double inv2dc(int hz, int hx) { return 1.0 / (double)((hz ? 2 : 1) * (hx ? 2 : 1)); }

}  // namespace

hipError_t launch_vc_fine_presmooth(const FineOp& op, double wj, const cplx* src,
                                    const double* scale, cplx* bout, cplx* xo, const int* active,
                                    hipStream_t s) {
    HH_LAUNCH(k_fine_presmooth, grid2(op.nz, op.nx), dim3(BX, BZ), 0, s, op, wj, src,
                       scale, bout, xo, active);
    return hipGetLastError();
}
hipError_t launch_vc_fine_resid_restrict(const FineOp& op, int hz, int hx, const cplx* b,
                                         const cplx* x, int nzc, int nxc, cplx* bc,
                                         const int* active, hipStream_t s) {
    HH_LAUNCH(k_fine_resid_restrict, grid2(nzc, nxc), dim3(BX, BZ), 0, s, op, hz, hx, b,
                       x, nzc, nxc, bc, inv2dc(hz, hx), active);
    return hipGetLastError();
}
hipError_t launch_vc_fine_prolong_post1(const FineOp& op, double wj, int hz, int hx,
                                        const cplx* b, const cplx* x, const cplx* e, int nxc,
                                        cplx* xo, const int* active, hipStream_t s) {
    HH_LAUNCH(k_fine_prolong_post1, grid2(op.nz, op.nx), dim3(BX, BZ), 0, s, op, wj, hz,
                       hx, b, x, e, nxc, xo, active);
    return hipGetLastError();
}
hipError_t launch_vc_fine_post2(const FineOp& op, double wj, const cplx* b, const cplx* x,
                                cplx* xo, const int* active, hipStream_t s) {
    HH_LAUNCH(k_fine_post2, grid2(op.nz, op.nx), dim3(BX, BZ), 0, s, op, wj, b, x, xo,
                       active);
    return hipGetLastError();
}
hipError_t launch_vc_coarse_presmooth(const CoarseOp& op, double wj, const cplx* b, cplx* xo,
                                      const int* active, hipStream_t s) {
    HH_LAUNCH(k_coarse_presmooth, grid2(op.nz, op.nx), dim3(BX, BZ), 0, s, op, wj, b, xo,
                       active);
    return hipGetLastError();
}
hipError_t launch_vc_coarse_resid_restrict(const CoarseOp& op, int hz, int hx, const cplx* b,
                                           const cplx* x, int nzc, int nxc, cplx* bc,
                                           const int* active, hipStream_t s) {
    HH_LAUNCH(k_coarse_resid_restrict, grid2(nzc, nxc), dim3(BX, BZ), 0, s, op, hz, hx,
                       b, x, nzc, nxc, bc, inv2dc(hz, hx), active);
    return hipGetLastError();
}
hipError_t launch_vc_coarse_prolong_post1(const CoarseOp& op, double wj, int hz, int hx,
                                          const cplx* b, const cplx* x, const cplx* e, int nxc,
                                          cplx* xo, const int* active, hipStream_t s) {
    HH_LAUNCH(k_coarse_prolong_post1, grid2(op.nz, op.nx), dim3(BX, BZ), 0, s, op, wj,
                       hz, hx, b, x, e, nxc, xo, active);
    return hipGetLastError();
}
hipError_t launch_vc_coarse_post2(const CoarseOp& op, double wj, const cplx* b, const cplx* x,
                                  cplx* xo, const int* active, hipStream_t s) {
    HH_LAUNCH(k_coarse_post2, grid2(op.nz, op.nx), dim3(BX, BZ), 0, s, op, wj, b, x, xo,
                       active);
    return hipGetLastError();
}
hipError_t launch_vc_gemv(int n, const cplx* A, const cplx* x, cplx* y, const int* active,
                          hipStream_t s) {
    HH_LAUNCH(k_gemv_pred, dim3(n), dim3(256), 0, s, n, A, x, y, active);
    return hipGetLastError();
}

}  // namespace hh
