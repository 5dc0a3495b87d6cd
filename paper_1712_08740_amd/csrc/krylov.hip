// Krylov-side kernels of right-preconditioned flexible GMRES (Eq. 7): the
// classical Gram-Schmidt passes of the Arnoldi step as multi-vector complex
// dot products and fused multi-AXPYs, norms, the Givens least-squares update
// of the Hessenberg matrix, back substitution and the solution update.
//
// Reductions are two-stage with a fixed summation order (per-block partial
// sums, then one pass over the partials), so results are bitwise
// reproducible from run to run.
#include "hh_internal.h"

namespace hh {

namespace {

constexpr int RB = 256;    // threads per reduction block
constexpr int EB = 256;    // threads per elementwise block

// Sum over a 256-thread block; the result is valid in thread 0.
__device__ __forceinline__ cplx block_sum(cplx v, cplx* sh) {
    for (int off = 32; off > 0; off >>= 1) {
        v.x += __shfl_down(v.x, off, 64);
        v.y += __shfl_down(v.y, off, 64);
    }
    const int tid = threadIdx.x;
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    cplx r = mk(0.0, 0.0);
    if (tid == 0) r = cadd(cadd(sh[0], sh[1]), cadd(sh[2], sh[3]));
    return r;
}

__global__ void __launch_bounds__(RB) k_dot_partials(const cplx* __restrict__ V, int64_t n,
                                                     const cplx* __restrict__ w,
                                                     cplx* __restrict__ partial, int nb) {
    __shared__ cplx sh[RB / 64];
    const int i = blockIdx.y;
    const cplx* vi = V + (int64_t)i * n;
    cplx acc = mk(0.0, 0.0);
    for (int64_t p = (int64_t)blockIdx.x * RB + threadIdx.x; p < n; p += (int64_t)nb * RB)
        acc = cadd(acc, cmulc(vi[p], w[p]));
    const cplx s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)i * nb + blockIdx.x] = s;
}

__global__ void __launch_bounds__(64) k_reduce_partials(const cplx* __restrict__ partial, int nb,
                                                        cplx* __restrict__ out) {
    const int i = blockIdx.x;
    const cplx* pi = partial + (int64_t)i * nb;
    cplx acc = mk(0.0, 0.0);
    for (int t = threadIdx.x; t < nb; t += 64) acc = cadd(acc, pi[t]);
    for (int off = 32; off > 0; off >>= 1) {
        acc.x += __shfl_down(acc.x, off, 64);
        acc.y += __shfl_down(acc.y, off, 64);
    }
    if (threadIdx.x == 0) out[i] = acc;
}

__global__ void __launch_bounds__(EB) k_multi_axpy(const cplx* __restrict__ V, int64_t n, int k,
                                                   const cplx* __restrict__ h,
                                                   cplx* __restrict__ w) {
    const int64_t p = (int64_t)blockIdx.x * EB + threadIdx.x;
    if (p >= n) return;
    cplx acc = w[p];
    for (int i = 0; i < k; ++i) acc = csub(acc, cmul(V[(int64_t)i * n + p], h[i]));
    w[p] = acc;
}

__global__ void __launch_bounds__(EB) k_scale_dev(const cplx* x,
                                                  const double* __restrict__ scale,
                                                  cplx* y, int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * EB + threadIdx.x;
    if (p >= n) return;
    y[p] = cscale(x[p], scale[0]);
}

__global__ void __launch_bounds__(EB) k_weight_rhs(FineOp op, const cplx* __restrict__ f,
                                                   cplx* __restrict__ b) {
    const int64_t p = (int64_t)blockIdx.x * EB + threadIdx.x;
    const int64_t n = (int64_t)op.nz * op.nx;
    if (p >= n) return;
    const int ix = (int)(p % op.nx);
    const int iz = (int)(p / op.nx);
    double w = (ix == 0 || ix == op.nx - 1) ? 0.5 : 1.0;
    if (op.ndim == 2 && (iz == 0 || iz == op.nz - 1)) w *= 0.5;
    b[p] = cscale(f[p], w);
}

__global__ void __launch_bounds__(EB) k_update_x(const cplx* __restrict__ Z, int64_t n, int k,
                                                 const cplx* __restrict__ y,
                                                 cplx* __restrict__ x) {
    const int64_t p = (int64_t)blockIdx.x * EB + threadIdx.x;
    if (p >= n) return;
    cplx acc = x[p];
    for (int i = 0; i < k; ++i) acc = cadd(acc, cmul(Z[(int64_t)i * n + p], y[i]));
    x[p] = acc;
}

__global__ void __launch_bounds__(RB) k_check_slowness(const double* __restrict__ m, int64_t n,
                                                       double* __restrict__ m2,
                                                       int* __restrict__ flag,
                                                       double* __restrict__ partial, int nb) {
    __shared__ double sh[RB / 64];
    double mx = 0.0;
    int bad = 0;
    for (int64_t p = (int64_t)blockIdx.x * RB + threadIdx.x; p < n; p += (int64_t)nb * RB) {
        const double v = m[p];
        if (!(isfinite(v) && v > 0.0)) bad = 1;
        m2[p] = v * v;
        mx = fmax(mx, v);
    }
    if (bad) atomicOr(flag, 1);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// One Givens step on column j (single thread; j <= m is small).
__global__ void k_givens(GivensState* st, const cplx* __restrict__ h1,
                         const cplx* __restrict__ h2, const cplx* __restrict__ nrm2,
                         cplx* __restrict__ R, double* __restrict__ cs, cplx* __restrict__ sn,
                         cplx* __restrict__ g) {
    if (threadIdx.x != 0) return;
    const int j = st->j;
    const int ld = st->m + 1;
    cplx* col = R + (int64_t)j * ld;
    for (int i = 0; i <= j; ++i) col[i] = cadd(h1[i], h2[i]);
    const double hn = sqrt(nrm2[0].x);
    col[j + 1] = mk(hn, 0.0);
    for (int i = 0; i < j; ++i) {           // previous rotations
        const cplx p = col[i], q = col[i + 1];
        col[i] = cadd(cscale(p, cs[i]), cmul(sn[i], q));
        col[i + 1] = csub(cscale(q, cs[i]), cmulc(sn[i], p));
    }
    const cplx a = col[j];
    double c;
    cplx s;
    if (hn == 0.0) {
        c = 1.0; s = mk(0.0, 0.0);
    } else if (a.x == 0.0 && a.y == 0.0) {
        c = 0.0; s = mk(1.0, 0.0);
    } else {
        const double aa = sqrt(cabs2(a));
        const double t = sqrt(aa * aa + hn * hn);
        c = aa / t;
        s = cscale(mk(a.x / aa, a.y / aa), hn / t);
    }
    cs[j] = c;
    sn[j] = s;
    col[j] = cadd(cscale(a, c), cscale(s, hn));
    col[j + 1] = mk(0.0, 0.0);
    const cplx gj = g[j];
    g[j + 1] = csub(mk(0.0, 0.0), cmulc(s, gj));
    g[j] = cscale(gj, c);
    const double est = sqrt(cabs2(g[j + 1])) / st->beta0;
    st->est = est;
    st->hn = hn;
    st->inv_hn = hn > 0.0 ? 1.0 / hn : 0.0;
    st->breakdown = hn == 0.0;
    st->bad = !(isfinite(est) && isfinite(hn));
    st->j = j + 1;
}

__global__ void k_backsub(int k, int m, const cplx* __restrict__ R, const cplx* __restrict__ g,
                          cplx* __restrict__ y) {
    if (threadIdx.x != 0) return;
    const int ld = m + 1;
    for (int i = k - 1; i >= 0; --i) {
        cplx acc = g[i];
        for (int l = i + 1; l < k; ++l) acc = csub(acc, cmul(R[i + (int64_t)l * ld], y[l]));
        y[i] = cdiv(acc, R[i + (int64_t)i * ld]);
    }
}

__global__ void k_cycle_init(GivensState* st, int m, double beta0, const cplx* __restrict__ nrm2,
                             cplx* __restrict__ g, double* __restrict__ inv_beta) {
    const double beta = sqrt(nrm2[0].x);
    for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = mk(i == 0 ? beta : 0.0, 0.0);
    if (threadIdx.x == 0) {
        inv_beta[0] = 1.0 / beta;
        st->j = 0;
        st->m = m;
        st->beta0 = beta0;
        st->est = beta / beta0;
        st->hn = 0.0;
        st->inv_hn = 0.0;
        st->breakdown = 0;
        st->bad = 0;
    }
}

inline unsigned eblocks(int64_t n) { return (unsigned)((n + EB - 1) / EB); }

}  // namespace

int reduce_blocks(int64_t n) {
    int64_t nb = (n + 2047) / 2048;
    if (nb < 1) nb = 1;
    if (nb > 512) nb = 512;
    return (int)nb;
}

hipError_t launch_dot_partials(const cplx* V, int64_t n, int k, const cplx* w, cplx* partial,
                               int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partials, dim3(nb, k), dim3(RB), 0, s, V, n, w, partial, nb);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const cplx* partial, int nb, int k, cplx* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(k), dim3(64), 0, s, partial, nb, out);
    return hipGetLastError();
}

hipError_t launch_multi_axpy(const cplx* V, int64_t n, int k, const cplx* h, cplx* w,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_multi_axpy, dim3(eblocks(n)), dim3(EB), 0, s, V, n, k, h, w);
    return hipGetLastError();
}

hipError_t launch_scale_dev(const cplx* x, const double* scale, cplx* y, int64_t n,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_scale_dev, dim3(eblocks(n)), dim3(EB), 0, s, x, scale, y, n);
    return hipGetLastError();
}

hipError_t launch_weight_rhs(const FineOp& op, const cplx* f, cplx* b, hipStream_t s) {
    const int64_t n = (int64_t)op.nz * op.nx;
    hipLaunchKernelGGL(k_weight_rhs, dim3(eblocks(n)), dim3(EB), 0, s, op, f, b);
    return hipGetLastError();
}

hipError_t launch_update_x(const cplx* Z, int64_t n, int k, const cplx* y, cplx* x,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_update_x, dim3(eblocks(n)), dim3(EB), 0, s, Z, n, k, y, x);
    return hipGetLastError();
}

hipError_t launch_check_slowness(const double* m, int64_t n, double* m2, int* flag,
                                 double* mmax_partial, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_check_slowness, dim3(nb), dim3(RB), 0, s, m, n, m2, flag, mmax_partial,
                       nb);
    return hipGetLastError();
}

hipError_t launch_givens(GivensState* st, const cplx* h1, const cplx* h2, const cplx* nrm2,
                         cplx* R, double* cs, cplx* sn, cplx* g, hipStream_t s) {
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, s, st, h1, h2, nrm2, R, cs, sn, g);
    return hipGetLastError();
}

hipError_t launch_backsub(int k, int m, const cplx* R, const cplx* g, cplx* y, hipStream_t s) {
    hipLaunchKernelGGL(k_backsub, dim3(1), dim3(64), 0, s, k, m, R, g, y);
    return hipGetLastError();
}

hipError_t launch_cycle_init(GivensState* st, int m, double beta0, const cplx* nrm2, cplx* g,
                             double* inv_beta, hipStream_t s) {
    hipLaunchKernelGGL(k_cycle_init, dim3(1), dim3(64), 0, s, st, m, beta0, nrm2, g, inv_beta);
    return hipGetLastError();
}

}  // namespace hh
