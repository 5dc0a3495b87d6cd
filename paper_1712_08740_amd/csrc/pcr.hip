// Exact 1D shifted-Laplace solve z = M^{-1} d (Eq. 6-7 in 1D, where M is
// tridiagonal) by parallel cyclic reduction in one workgroup.
//
// Row i of M: sub a_i = -1/h^2 (i > 0), super c_i = -1/h^2 (i < n-1), diagonal
// from the shared operator row. Step s (s = 1, 2, 4, ...) eliminates the
// couplings to rows i-s and i+s:
//   k1 = a_i / b_{i-s},  k2 = c_i / b_{i+s}
//   a_i' = -k1 a_{i-s},  c_i' = -k2 c_{i+s}
//   b_i' = b_i - k1 c_{i-s} - k2 a_{i+s},  d_i' = d_i - k1 d_{i-s} - k2 d_{i+s}
// until s >= n, when every row reads b_i z_i = d_i. With Im M > 0 (beta2 > 0)
// every principal submatrix is nonsingular, so no pivoting is needed.
// The whole system lives in LDS (4 complex arrays of n entries).
#include "hh_internal.h"

namespace hh {

namespace {

constexpr int PCR_THREADS = 1024;
constexpr int PCR_MAXN = 1024;

// x = M^{-1} src in the operator's precision T (src stays complex128).
// Returns at once when *active == 0.
template <class T>
__global__ void __launch_bounds__(PCR_THREADS) k_pcr(FineOpT<T> op, const cplx* __restrict__ src,
                                                     typename Cx<T>::type* __restrict__ x_out,
                                                     const int* __restrict__ active, int64_t bs) {
    typedef typename Cx<T>::type C;
    const int rb = blockIdx.x;                 // right-hand side
    active = rhs_at(active, rb, bs);
    if (active && *active == 0) return;
    src = rhs_nn(src, rb, bs);
    x_out = rhs_nn(x_out, rb, bs);
    __shared__ C sa[PCR_MAXN], sb[PCR_MAXN], sc[PCR_MAXN], sd[PCR_MAXN];
    const int n = op.nx;
    const int i = threadIdx.x;
    const C zero = czero<C>();
    if (i < n) {
        const Coef5T<T> c = fine_coefs(op, 0, i, op.m2[i]);
        C lo = zero, up = zero;
        lo.x = i > 0 ? -c.cx : (T)0;
        up.x = i < n - 1 ? -c.cx : (T)0;
        sa[i] = lo;
        sc[i] = up;
        sb[i] = c.diag;
        sd[i] = cconv<C>(src[i]);
    }
    __syncthreads();
    for (int s = 1; s < n; s <<= 1) {
        C na = zero, nb = zero, nc = zero, nd = zero;
        if (i < n) {
            const C ai = sa[i], ci = sc[i];
            nb = sb[i];
            nd = sd[i];
            if (i - s >= 0) {
                const C k1 = cdiv(ai, sb[i - s]);
                na = csub(zero, cmul(k1, sa[i - s]));
                nb = csub(nb, cmul(k1, sc[i - s]));
                nd = csub(nd, cmul(k1, sd[i - s]));
            }
            if (i + s < n) {
                const C k2 = cdiv(ci, sb[i + s]);
                nc = csub(zero, cmul(k2, sc[i + s]));
                nb = csub(nb, cmul(k2, sa[i + s]));
                nd = csub(nd, cmul(k2, sd[i + s]));
            }
        }
        __syncthreads();
        if (i < n) {
            sa[i] = na;
            sb[i] = nb;
            sc[i] = nc;
            sd[i] = nd;
        }
        __syncthreads();
    }
    if (i < n) x_out[i] = cdiv(sd[i], sb[i]);
}

template <class T>
hipError_t pcr(const FineOpT<T>& op, const cplx* src, typename Cx<T>::type* x, const int* active,
               hipStream_t s, const Batch& bt) {
    if (op.ndim != 1 || op.nx > PCR_MAXN) return hipErrorInvalidValue;
    HH_LAUNCH((k_pcr<T>), dim3(bt.n), dim3(PCR_THREADS), 0, s, op, src, x, active, bt.bs);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pcr_solve(const FineOp& op, const cplx* d, cplx* x, hipStream_t s) {
    return launch_pcr(op, d, x, nullptr, s);
}

hipError_t launch_pcr(const FineOp& op, const cplx* src, cplx* x, const int* active,
                      hipStream_t s, const Batch& bt) {
    return pcr(op, src, x, active, s, bt);
}
hipError_t launch_pcr(const FineOpT<float>& op, const cplx* src, cplxf* x, const int* active,
                      hipStream_t s, const Batch& bt) {
    return pcr(op, src, x, active, s, bt);
}

}  // namespace hh
