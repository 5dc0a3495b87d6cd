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
// The multipliers k1, k2 of every step and the final b depend on M only: they
// are computed once per shift (k_pcr_factor) and each application updates d
// alone (k_pcr_apply: two multiply-adds and one barrier per step, no
// division but the last), with the same operations in the same order.
#include "hh_internal.h"

namespace hh {

namespace {

constexpr int PCR_THREADS = 1024;
constexpr int PCR_MAXN = 1024;
constexpr int PCR_MAXL = 10;                    // steps for n <= 1024

// The reduction of a, b, c in LDS, recording k1, k2 of every step:
// K[(2 l) n + i] = k1, K[(2 l + 1) n + i] = k2 (0 where the coupling is absent),
// bfin[i] = the final diagonal.
template <class T>
__global__ void __launch_bounds__(PCR_THREADS) k_pcr_factor(FineOpT<T> op,
                                                            typename Cx<T>::type* __restrict__ K,
                                                            typename Cx<T>::type* __restrict__ bfin) {
    typedef typename Cx<T>::type C;
    __shared__ C sa[PCR_MAXN], sb[PCR_MAXN], sc[PCR_MAXN];
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
    }
    __syncthreads();
    int l = 0;
    for (int s = 1; s < n; s <<= 1, ++l) {
        C na = zero, nb = zero, nc = zero, k1 = zero, k2 = zero;
        if (i < n) {
            const C ai = sa[i], ci = sc[i];
            nb = sb[i];
            if (i - s >= 0) {
                k1 = cdiv(ai, sb[i - s]);
                na = csub(zero, cmul(k1, sa[i - s]));
                nb = csub(nb, cmul(k1, sc[i - s]));
            }
            if (i + s < n) {
                k2 = cdiv(ci, sb[i + s]);
                nc = csub(zero, cmul(k2, sc[i + s]));
                nb = csub(nb, cmul(k2, sa[i + s]));
            }
            K[(int64_t)(2 * l) * n + i] = k1;
            K[(int64_t)(2 * l + 1) * n + i] = k2;
        }
        __syncthreads();
        if (i < n) {
            sa[i] = na;
            sb[i] = nb;
            sc[i] = nc;
        }
        __syncthreads();
    }
    if (i < n) bfin[i] = sb[i];
}

// x = M^{-1} src for every right-hand side (one workgroup each), from the
// factors; src stays complex128, x in the factors' precision. The factors of
// all steps are loaded up front; d is double buffered in LDS (one barrier per
// step). Returns at once when *active == 0.
template <class T>
__global__ void __launch_bounds__(PCR_THREADS) k_pcr_apply(int n, int levels,
                                                           const typename Cx<T>::type* __restrict__ K,
                                                           const typename Cx<T>::type* __restrict__ bfin,
                                                           const cplx* __restrict__ src,
                                                           typename Cx<T>::type* __restrict__ x_out,
                                                           const int* __restrict__ active, int64_t bs) {
    typedef typename Cx<T>::type C;
    const int rb = blockIdx.x;                 // right-hand side
    active = rhs_at(active, rb, bs);
    if (active && *active == 0) return;
    src = rhs_nn(src, rb, bs);
    x_out = rhs_nn(x_out, rb, bs);
    __shared__ C sd[2][PCR_MAXN];
    const int i = threadIdx.x;
    const bool ok = i < n;
    const int ic = ok ? i : 0;
    C k1[PCR_MAXL], k2[PCR_MAXL];
#pragma unroll
    for (int l = 0; l < PCR_MAXL; ++l) {
        const bool lv = l < levels;
        k1[l] = K[lv ? (int64_t)(2 * l) * n + ic : 0];
        k2[l] = K[lv ? (int64_t)(2 * l + 1) * n + ic : 0];
    }
    const C bi = bfin[ic];
    sd[0][ic] = cconv<C>(src[ic]);
    __syncthreads();
#pragma unroll
    for (int l = 0; l < PCR_MAXL; ++l) {
        if (l < levels) {
            const int s = 1 << l;
            const C* d = sd[l & 1];
            C nd = d[ic];
            if (i - s >= 0) nd = csub(nd, cmul(k1[l], d[i - s]));
            if (i + s < n) nd = csub(nd, cmul(k2[l], d[i + s]));
            if (ok) sd[(l + 1) & 1][i] = nd;
            __syncthreads();
        }
    }
    if (ok) x_out[i] = cdiv(sd[levels & 1][i], bi);
}

}  // namespace

int pcr_levels(int n) {
    int l = 0;
    for (int s = 1; s < n; s <<= 1) ++l;
    return l;
}

size_t pcr_factor_elems(int n) { return (size_t)(2 * pcr_levels(n) + 1) * n; }

template <class T>
static hipError_t pcr_factor(const FineOpT<T>& op, typename Cx<T>::type* f, hipStream_t s) {
    if (op.ndim != 1 || op.nx > PCR_MAXN) return hipErrorInvalidValue;
    const int n = op.nx;
    HH_LAUNCH((k_pcr_factor<T>), dim3(1), dim3(PCR_THREADS), 0, s, op, f,
              f + (size_t)2 * pcr_levels(n) * n);
    return hipGetLastError();
}

template <class T>
static hipError_t pcr_apply(int n, const typename Cx<T>::type* f, const cplx* src,
                            typename Cx<T>::type* x, const int* active, hipStream_t s,
                            const Batch& bt) {
    if (n > PCR_MAXN) return hipErrorInvalidValue;
    const int L = pcr_levels(n);
    HH_LAUNCH((k_pcr_apply<T>), dim3(bt.n), dim3(PCR_THREADS), 0, s, n, L, f,
              f + (size_t)2 * L * n, src, x, active, bt.bs);
    return hipGetLastError();
}

hipError_t launch_pcr_factor(const FineOp& op, cplx* f, hipStream_t s) {
    return pcr_factor(op, f, s);
}
hipError_t launch_pcr_factor(const FineOpT<float>& op, cplxf* f, hipStream_t s) {
    return pcr_factor(op, f, s);
}
hipError_t launch_pcr(int n, const cplx* f, const cplx* src, cplx* x, const int* active,
                      hipStream_t s, const Batch& bt) {
    return pcr_apply<double>(n, f, src, x, active, s, bt);
}
hipError_t launch_pcr(int n, const cplxf* f, const cplx* src, cplxf* x, const int* active,
                      hipStream_t s, const Batch& bt) {
    return pcr_apply<float>(n, f, src, x, active, s, bt);
}

}  // namespace hh
