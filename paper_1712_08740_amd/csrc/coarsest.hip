// Coarsest-level solve of the V-cycle: z = A^{-1} b with the explicit inverse
// computed at set-up, as a dense complex matrix-vector product with a
// fixed-order reduction.
#include "helmholtz.h"
#include "hh_internal.h"

namespace hh {

namespace {

// One 256-thread workgroup per row; each thread keeps its loads of the row and
// of x in flight together (n <= HH_MAX_COARSE = 16 * 256).
constexpr int GEMV_SLOTS = HH_MAX_COARSE / 256;

// C: matrix and result type; X: type of x (complex128 when the fine grid is
// itself the coarsest level and x is the Krylov vector). Accumulates in C.
template <class C, class X>
__global__ void __launch_bounds__(256) k_gemv_pred(int n, const C* __restrict__ A,
                                                   const X* __restrict__ x,
                                                   C* __restrict__ y,
                                                   const int* __restrict__ active) {
    if (active && *active == 0) return;
    __shared__ C sh[4];
    const int tid = threadIdx.x;
    const C* a = A + (int64_t)blockIdx.x * n;
    C acc = czero<C>();
    for (int j0 = 0; j0 < n; j0 += 256 * 8) {
        C av[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + u * 256 + tid;
            av[u] = j < n ? a[j] : czero<C>();
            xv[u] = j < n ? cconv<C>(x[j]) : czero<C>();
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = cadd(acc, cmul(av[u], xv[u]));
    }
    for (int off = 32; off > 0; off >>= 1) {
        acc.x += __shfl_down(acc.x, off, 64);
        acc.y += __shfl_down(acc.y, off, 64);
    }
    if ((tid & 63) == 0) sh[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) y[blockIdx.x] = cadd(cadd(sh[0], sh[1]), cadd(sh[2], sh[3]));
}

// Several right-hand sides: one workgroup per (row, group of GR right-hand
// sides) keeps its slice of the row in registers and applies it to each
// right-hand side of the group (x, y and the predicate in that right-hand
// side's workspace, bs bytes apart), so the inverse is read once per group.
constexpr int GR = 8;

template <class C, class X>
__global__ void __launch_bounds__(256) k_gemm_pred(int n, const C* __restrict__ A,
                                                   const X* __restrict__ x, C* __restrict__ y,
                                                   const int* __restrict__ active, int nrhs,
                                                   int64_t bs) {
    __shared__ C sh[4];
    const int tid = threadIdx.x;
    const C* a = A + (int64_t)blockIdx.x * n;
    C av[GEMV_SLOTS];
#pragma unroll
    for (int u = 0; u < GEMV_SLOTS; ++u) {
        const int j = u * 256 + tid;
        av[u] = j < n ? a[j] : czero<C>();
    }
    const int r0 = blockIdx.y * GR;
    for (int r = r0; r < r0 + GR && r < nrhs; ++r) {
        const int* act = rhs_at(active, r, bs);
        if (act && *act == 0) continue;                 // uniform over the block
        const X* xr = rhs_nn(x, r, bs);
        C acc = czero<C>();
#pragma unroll
        for (int u = 0; u < GEMV_SLOTS; ++u) {
            const int j = u * 256 + tid;
            if (j < n) acc = cadd(acc, cmul(av[u], cconv<C>(xr[j])));
        }
        for (int off = 32; off > 0; off >>= 1) {
            acc.x += __shfl_down(acc.x, off, 64);
            acc.y += __shfl_down(acc.y, off, 64);
        }
        if ((tid & 63) == 0) sh[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0) rhs_nn(y, r, bs)[blockIdx.x] = cadd(cadd(sh[0], sh[1]), cadd(sh[2], sh[3]));
        __syncthreads();
    }
}

template <class C, class X>
hipError_t gemv(int n, const C* A, const X* x, C* y, const int* active, hipStream_t s,
                const Batch& bt) {
    if (n > HH_MAX_COARSE) return hipErrorInvalidValue;
    if (bt.n == 1) {
        HH_LAUNCH((k_gemv_pred<C, X>), dim3(n), dim3(256), 0, s, n, A, x, y, active);
    } else {
        HH_LAUNCH((k_gemm_pred<C, X>), dim3(n, (bt.n + GR - 1) / GR), dim3(256), 0, s, n, A, x, y,
                  active, bt.n, bt.bs);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_vc_gemv(int n, const cplx* A, const cplx* x, cplx* y, const int* active,
                          hipStream_t s, const Batch& bt) {
    return gemv(n, A, x, y, active, s, bt);
}
hipError_t launch_vc_gemv(int n, const cplxf* A, const cplxf* x, cplxf* y, const int* active,
                          hipStream_t s, const Batch& bt) {
    return gemv(n, A, x, y, active, s, bt);
}
hipError_t launch_vc_gemv(int n, const cplxf* A, const cplx* x, cplxf* y, const int* active,
                          hipStream_t s, const Batch& bt) {
    return gemv(n, A, x, y, active, s, bt);
}

}  // namespace hh
