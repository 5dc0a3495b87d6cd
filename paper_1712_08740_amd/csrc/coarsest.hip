// Coarsest-level solve of the V-cycle: z = A^{-1} b with the explicit inverse
// computed at set-up, as a dense complex matrix-vector product. One
// 256-thread workgroup per row, fixed-order reduction.
#include "hh_internal.h"

namespace hh {

namespace {

__global__ void __launch_bounds__(256) k_gemv_pred(int n, const cplx* __restrict__ A,
                                                   const cplx* __restrict__ x,
                                                   cplx* __restrict__ y,
                                                   const int* __restrict__ active) {
    if (active && *active == 0) return;
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

}  // namespace

hipError_t launch_vc_gemv(int n, const cplx* A, const cplx* x, cplx* y, const int* active,
                          hipStream_t s) {
    HH_LAUNCH(k_gemv_pred, dim3(n), dim3(256), 0, s, n, A, x, y, active);
    return hipGetLastError();
}

}  // namespace hh
