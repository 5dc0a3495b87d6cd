// Multigrid transfer and set-up kernels for the approximate shifted-Laplace
// inverse (Eq. 6-7): full-weighting restriction R = P^T / 2^{d_c}, (bi)linear
// prolongation P, Galerkin coarse operators R M P (9-point), and the dense
// matrix of the coarsest operator (inverted by LU in the set-up).
#include "hh_internal.h"

namespace hh {

namespace {

constexpr int BX = 64;
constexpr int BZ = 4;

dim3 grid2(int nz, int nx) { return dim3((nx + BX - 1) / BX, (nz + BZ - 1) / BZ); }

// Coarse nodes J with P[q, J] != 0 along one axis, and their weights.
__device__ __forceinline__ int interp_nodes(int q, int halved, int* J, double* w) {
    if (!halved) { J[0] = q; w[0] = 1.0; return 1; }
    if ((q & 1) == 0) { J[0] = q >> 1; w[0] = 1.0; return 1; }
    J[0] = (q - 1) >> 1; w[0] = 0.5;
    J[1] = (q + 1) >> 1; w[1] = 0.5;
    return 2;
}

// Accumulate R[I,p] * A[p,q] * P[q,J] over the fine rows p of R's support and
// the entries q of row p; row p is produced by the functor `row(pz, px, emit)`.
template <class RowFn>
__device__ __forceinline__ void galerkin_node(int Iz, int Ix, int nzf, int nxf, int hz, int hx,
                                              double inv2dc, RowFn row, cplx acc[9]) {
    for (int t = 0; t < 9; ++t) acc[t] = mk(0.0, 0.0);
    const int fz = hz ? 2 * Iz : Iz;
    const int fx = hx ? 2 * Ix : Ix;
    const int rz = hz ? 1 : 0, rx = hx ? 1 : 0;
    for (int dz = -rz; dz <= rz; ++dz) {
        const int pz = fz + dz;
        if (pz < 0 || pz >= nzf) continue;
        for (int dx = -rx; dx <= rx; ++dx) {
            const int px = fx + dx;
            if (px < 0 || px >= nxf) continue;
            const double rw = (dz == 0 ? 1.0 : 0.5) * (dx == 0 ? 1.0 : 0.5) * inv2dc;
            row(pz, px, [&](int qz, int qx, cplx a) {
                int Jz[2], Jx[2];
                double wz[2], wx[2];
                const int nzj = interp_nodes(qz, hz, Jz, wz);
                const int nxj = interp_nodes(qx, hx, Jx, wx);
                for (int u = 0; u < nzj; ++u)
                    for (int v = 0; v < nxj; ++v) {
                        const int t = (Jz[u] - Iz + 1) * 3 + (Jx[v] - Ix + 1);
                        acc[t] = cadd(acc[t], cscale(a, rw * wz[u] * wx[v]));
                    }
            });
        }
    }
}

__global__ void __launch_bounds__(256) k_galerkin_from_fine(FineOp op, int hz, int hx, int nzc,
                                                            int nxc, cplx* __restrict__ Cc) {
    const int Ix = blockIdx.x * BX + threadIdx.x;
    const int Iz = blockIdx.y * BZ + threadIdx.y;
    if (Ix >= nxc || Iz >= nzc) return;
    const double inv2dc = 1.0 / (double)((hz ? 2 : 1) * (hx ? 2 : 1));
    cplx acc[9];
    auto row = [&](int pz, int px, auto emit) {
        const int64_t p = (int64_t)pz * op.nx + px;
        const Coef5 c = fine_coefs(op, pz, px, op.m2[p]);
        emit(pz, px, c.diag);
        if (px > 0) emit(pz, px - 1, mk(-c.cx, 0.0));
        if (px < op.nx - 1) emit(pz, px + 1, mk(-c.cx, 0.0));
        if (pz > 0) emit(pz - 1, px, mk(-c.cz, 0.0));
        if (pz < op.nz - 1) emit(pz + 1, px, mk(-c.cz, 0.0));
    };
    galerkin_node(Iz, Ix, op.nz, op.nx, hz, hx, inv2dc, row, acc);
    const int64_t Nc = (int64_t)nzc * nxc;
    const int64_t P = (int64_t)Iz * nxc + Ix;
    for (int t = 0; t < 9; ++t) Cc[t * Nc + P] = acc[t];
}

__global__ void __launch_bounds__(256) k_galerkin_from_coarse(CoarseOp op, int hz, int hx,
                                                              int nzc, int nxc,
                                                              cplx* __restrict__ Cc) {
    const int Ix = blockIdx.x * BX + threadIdx.x;
    const int Iz = blockIdx.y * BZ + threadIdx.y;
    if (Ix >= nxc || Iz >= nzc) return;
    const double inv2dc = 1.0 / (double)((hz ? 2 : 1) * (hx ? 2 : 1));
    const int64_t Nf = (int64_t)op.nz * op.nx;
    cplx acc[9];
    auto row = [&](int pz, int px, auto emit) {
        const int64_t p = (int64_t)pz * op.nx + px;
        for (int sz = -1; sz <= 1; ++sz) {
            const int qz = pz + sz;
            if (qz < 0 || qz >= op.nz) continue;
            for (int sx = -1; sx <= 1; ++sx) {
                const int qx = px + sx;
                if (qx < 0 || qx >= op.nx) continue;
                emit(qz, qx, op.C[((sz + 1) * 3 + (sx + 1)) * Nf + p]);
            }
        }
    };
    galerkin_node(Iz, Ix, op.nz, op.nx, hz, hx, inv2dc, row, acc);
    const int64_t Nc = (int64_t)nzc * nxc;
    const int64_t P = (int64_t)Iz * nxc + Ix;
    for (int t = 0; t < 9; ++t) Cc[t * Nc + P] = acc[t];
}

// Dense row-major n x n matrix of a level operator (A must be zeroed first).
__global__ void __launch_bounds__(256) k_dense_from_fine(FineOp op, cplx* __restrict__ A) {
    const int ix = blockIdx.x * BX + threadIdx.x;
    const int iz = blockIdx.y * BZ + threadIdx.y;
    if (ix >= op.nx || iz >= op.nz) return;
    const int64_t n = (int64_t)op.nz * op.nx;
    const int64_t p = (int64_t)iz * op.nx + ix;
    const Coef5 c = fine_coefs(op, iz, ix, op.m2[p]);
    cplx* row = A + p * n;
    row[p] = c.diag;
    if (ix > 0) row[p - 1] = mk(-c.cx, 0.0);
    if (ix < op.nx - 1) row[p + 1] = mk(-c.cx, 0.0);
    if (op.ndim == 2) {
        if (iz > 0) row[p - op.nx] = mk(-c.cz, 0.0);
        if (iz < op.nz - 1) row[p + op.nx] = mk(-c.cz, 0.0);
    }
}

__global__ void __launch_bounds__(256) k_dense_from_coarse(CoarseOp op, cplx* __restrict__ A) {
    const int ix = blockIdx.x * BX + threadIdx.x;
    const int iz = blockIdx.y * BZ + threadIdx.y;
    if (ix >= op.nx || iz >= op.nz) return;
    const int64_t n = (int64_t)op.nz * op.nx;
    const int64_t p = (int64_t)iz * op.nx + ix;
    cplx* row = A + p * n;
    for (int sz = -1; sz <= 1; ++sz) {
        const int qz = iz + sz;
        if (qz < 0 || qz >= op.nz) continue;
        for (int sx = -1; sx <= 1; ++sx) {
            const int qx = ix + sx;
            if (qx < 0 || qx >= op.nx) continue;
            row[(int64_t)qz * op.nx + qx] = op.C[((sz + 1) * 3 + (sx + 1)) * n + p];
        }
    }
}

}  // namespace

hipError_t launch_galerkin_from_fine(const FineOp& fine, int hz, int hx, int nzc, int nxc,
                                     cplx* Cc, hipStream_t s) {
    HH_LAUNCH(k_galerkin_from_fine, grid2(nzc, nxc), dim3(BX, BZ), 0, s, fine, hz, hx,
                       nzc, nxc, Cc);
    return hipGetLastError();
}

hipError_t launch_galerkin_from_coarse(const CoarseOp& fine, int hz, int hx, int nzc, int nxc,
                                       cplx* Cc, hipStream_t s) {
    HH_LAUNCH(k_galerkin_from_coarse, grid2(nzc, nxc), dim3(BX, BZ), 0, s, fine, hz, hx,
                       nzc, nxc, Cc);
    return hipGetLastError();
}

hipError_t launch_dense_from_fine(const FineOp& op, cplx* A, hipStream_t s) {
    const size_t n = (size_t)op.nz * op.nx;
    hipError_t e = hipMemsetAsync(A, 0, n * n * sizeof(cplx), s);
    if (e != hipSuccess) return e;
    HH_LAUNCH(k_dense_from_fine, grid2(op.nz, op.nx), dim3(BX, BZ), 0, s, op, A);
    return hipGetLastError();
}

hipError_t launch_dense_from_coarse(const CoarseOp& op, cplx* A, hipStream_t s) {
    const size_t n = (size_t)op.nz * op.nx;
    hipError_t e = hipMemsetAsync(A, 0, n * n * sizeof(cplx), s);
    if (e != hipSuccess) return e;
    HH_LAUNCH(k_dense_from_coarse, grid2(op.nz, op.nx), dim3(BX, BZ), 0, s, op, A);
    return hipGetLastError();
}

}  // namespace hh
