// Matrix-free operator kernels: the fine-grid 5-point (2D) / 3-point (1D)
// stencil of A_sigma with absorbing boundary rows (Eq. 2-3 and Eq. 6), and
// the 9-point Galerkin operators of the coarse multigrid levels.
//
// One thread per grid node; 2D blocks are 64 x 4 so that a wavefront covers 64
// consecutive x nodes (one 1 KiB coalesced complex128 row segment); the x
// neighbours come from the same cache lines and the z neighbours from the rows
// above and below, which the block's other wavefronts load.
#include "hh_internal.h"

namespace hh {

namespace {

constexpr int BX = 64;
constexpr int BZ = 4;
constexpr int B1 = 256;

// sum of (A x) off-diagonal part with the sign folded in: -cx (xW + xE) - cz (xN + xS)
template <int NDIM>
__device__ __forceinline__ cplx fine_offdiag(const FineOp& op, const Coef5& c, const cplx* x,
                                             int iz, int ix, int64_t p) {
    cplx sx = mk(0.0, 0.0);
    if (ix > 0) sx = cadd(sx, x[p - 1]);
    if (ix < op.nx - 1) sx = cadd(sx, x[p + 1]);
    cplx r = cscale(sx, -c.cx);
    if (NDIM == 2) {
        cplx sz = mk(0.0, 0.0);
        if (iz > 0) sz = cadd(sz, x[p - op.nx]);
        if (iz < op.nz - 1) sz = cadd(sz, x[p + op.nx]);
        r = cadd(r, cscale(sz, -c.cz));
    }
    return r;
}

template <int NDIM>
__device__ __forceinline__ bool node_of_thread(const FineOp& op, int& iz, int& ix) {
    if (NDIM == 2) {
        ix = blockIdx.x * BX + threadIdx.x;
        iz = blockIdx.y * BZ + threadIdx.y;
    } else {
        ix = blockIdx.x * B1 + threadIdx.x;
        iz = 0;
    }
    return ix < op.nx && iz < op.nz;
}

template <int NDIM>
__global__ void __launch_bounds__(256) k_fine_apply(FineOp op, const cplx* __restrict__ x,
                                                    cplx* __restrict__ y) {
    int iz, ix;
    if (!node_of_thread<NDIM>(op, iz, ix)) return;
    const int64_t p = (int64_t)iz * op.nx + ix;
    const Coef5 c = fine_coefs(op, iz, ix, op.m2[p]);
    y[p] = cadd(cmul(c.diag, x[p]), fine_offdiag<NDIM>(op, c, x, iz, ix, p));
}

// ---- 9-point coarse operators ---------------------------------------------
__device__ __forceinline__ bool coarse_node(const CoarseOp& op, int& iz, int& ix) {
    ix = blockIdx.x * BX + threadIdx.x;
    iz = blockIdx.y * BZ + threadIdx.y;
    return ix < op.nx && iz < op.nz;
}

__device__ __forceinline__ cplx coarse_row(const CoarseOp& op, const cplx* x, int iz, int ix,
                                           int64_t p, cplx* diag_out) {
    const int64_t N = (int64_t)op.nz * op.nx;
    cplx acc = mk(0.0, 0.0);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
        const int qz = iz + dz;
        if (qz < 0 || qz >= op.nz) continue;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int qx = ix + dx;
            if (qx < 0 || qx >= op.nx) continue;
            const int t = (dz + 1) * 3 + (dx + 1);
            const cplx a = op.C[t * N + p];
            if (t == 4 && diag_out) *diag_out = a;
            acc = cadd(acc, cmul(a, x[(int64_t)qz * op.nx + qx]));
        }
    }
    return acc;
}

__global__ void __launch_bounds__(256) k_coarse_apply(CoarseOp op, const cplx* __restrict__ x,
                                                      cplx* __restrict__ y) {
    int iz, ix;
    if (!coarse_node(op, iz, ix)) return;
    const int64_t p = (int64_t)iz * op.nx + ix;
    y[p] = coarse_row(op, x, iz, ix, p, nullptr);
}

dim3 grid2(int nz, int nx) { return dim3((nx + BX - 1) / BX, (nz + BZ - 1) / BZ); }

}  // namespace

#define HH_FINE_LAUNCH(KERNEL, ...)                                                        \
    do {                                                                                   \
        if (op.ndim == 2)                                                                  \
            HH_LAUNCH(KERNEL<2>, grid2(op.nz, op.nx), dim3(BX, BZ), 0, s,         \
                               __VA_ARGS__);                                               \
        else                                                                               \
            HH_LAUNCH(KERNEL<1>, dim3((op.nx + B1 - 1) / B1), dim3(B1), 0, s,     \
                               __VA_ARGS__);                                               \
        return hipGetLastError();                                                          \
    } while (0)

hipError_t launch_fine_apply(const FineOp& op, const cplx* x, cplx* y, hipStream_t s) {
    HH_FINE_LAUNCH(k_fine_apply, op, x, y);
}
hipError_t launch_coarse_apply(const CoarseOp& op, const cplx* x, cplx* y, hipStream_t s) {
    HH_LAUNCH(k_coarse_apply, grid2(op.nz, op.nx), dim3(BX, BZ), 0, s, op, x, y);
    return hipGetLastError();
}
}  // namespace hh
