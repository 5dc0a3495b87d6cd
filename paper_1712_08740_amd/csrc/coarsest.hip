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

template <class C, class X>
hipError_t gemv(int n, const C* A, const X* x, C* y, const int* active, hipStream_t s) {
    if (n > HH_MAX_COARSE) return hipErrorInvalidValue;
    HH_LAUNCH((k_gemv_pred<C, X>), dim3(n), dim3(256), 0, s, n, A, x, y, active);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_vc_gemv(int n, const cplx* A, const cplx* x, cplx* y, const int* active,
                          hipStream_t s) {
    return gemv(n, A, x, y, active, s);
}
hipError_t launch_vc_gemv(int n, const cplxf* A, const cplxf* x, cplxf* y, const int* active,
                          hipStream_t s) {
    return gemv(n, A, x, y, active, s);
}
hipError_t launch_vc_gemv(int n, const cplxf* A, const cplx* x, cplxf* y, const int* active,
                          hipStream_t s) {
    return gemv(n, A, x, y, active, s);
}

}  // namespace hh
