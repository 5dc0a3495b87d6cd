// Coarsest-level solve of the V-cycle: z = A^{-1} b with the explicit inverse
// computed at set-up, as a dense complex matrix-vector product with a
// fixed-order reduction; for a batch of sources, as one complex matrix product
// on the matrix cores (k_coarsest_mfma).
#include "helmholtz.h"
#include "hh_internal.h"

namespace hh {

namespace {

// One 256-thread workgroup per row; each thread keeps 8 loads of the row and
// of x in flight together.

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

// Several right-hand sides with x of another precision than A (the fine grid
// is itself the coarsest level and x is the complex128 Krylov vector): one
// workgroup per (row, right-hand side). The same-precision batched product
// is k_coarsest_mfma below.
template <class C, class X>
__global__ void __launch_bounds__(256) k_gemv_batch(int n, const C* __restrict__ A,
                                                    const X* __restrict__ x, C* __restrict__ y,
                                                    const int* __restrict__ active, int64_t bs) {
    const int rb = blockIdx.y;
    const int* act = rhs_at(active, rb, bs);
    if (act && *act == 0) return;
    x = rhs_nn(x, rb, bs);
    y = rhs_nn(y, rb, bs);
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

// Y = A X for a batch of right-hand sides (the coarsest solve of every source
// at once) on the matrix cores: A row-major n x n, column b of X and Y in
// right-hand side b's workspace (bs bytes after column b - 1).
//
// With A's complex entries stored as interleaved (re, im) pairs, A is a real
// n x 2n matrix A_r, and for x = X(:, b)
//   Re Y(:, b) = A_r [Re x_0, -Im x_0, Re x_1, -Im x_1, ...]^T,
//   Im Y(:, b) = A_r [Im x_0,  Re x_0, Im x_1,  Re x_1, ...]^T,
// so one real product with 2n terms gives both parts of every output.
//
// k_coarsest_mfma: a block of four waves owns 128 rows (32 per wave: two
// 16-row tiles), 32 right-hand sides (group blockIdx.y: two 16-column tiles,
// each for the real and the imaginary part) and one of KS contiguous ranges of
// k (blockIdx.z), stepping 16 complex k at a time. A is loaded once, straight
// into registers; X comes from the L2 (it is read by every row block).
// MFMA 16x16x4 (f32 or f64): lane l supplies A(l%16, l/16) and B(l/16, l%16)
// and receives in accumulator r the entry of column l%16 and row 4(l/16)+r
// (f32) or l/16+4r (f64). Lane (i, q) of a tile holds
// complex entries 4u + q (u = 0..3) of its row (or column) in the step, so one
// load instruction reads 4 consecutive entries per row; each u is fed as two
// k-slices (real parts, then imaginary parts). The order of the terms is fixed:
// every result depends only on A and its own column.
// k_coarsest_sum adds the KS partial sums in order.
constexpr int MF_TM = 128, MF_TN = 32, MF_KC = 16;

typedef float mfma_f4 __attribute__((ext_vector_type(4)));
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <class R> struct Mfma;
template <> struct Mfma<float> {
    typedef mfma_f4 acc;
    // row of D held by lane group q (= lane / 16) in accumulator r
    static __device__ __forceinline__ int row(int q, int r) { return 4 * q + r; }
    static __device__ __forceinline__ acc fma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    typedef mfma_d4 acc;
    static __device__ __forceinline__ int row(int q, int r) { return q + 4 * r; }
    static __device__ __forceinline__ acc fma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// WIDE (complex64 with n even, so every row of A starts on 16 bytes): each
// load instruction takes two consecutive entries per lane, entries 8v + 2q and
// 8v + 2q + 1 of the step (v = 0, 1) standing in the places u = 2v, 2v + 1 of
// the k order (half the load instructions: measured 72 -> 88 TFLOP/s at
// n = 7676).
template <class R, bool WIDE>
__global__ void __launch_bounds__(256) k_coarsest_mfma(int n, const typename Cx<R>::type* __restrict__ A,
                                                       const typename Cx<R>::type* __restrict__ X,
                                                       int nrhs, int64_t bs, int chunks_per_split,
                                                       typename Cx<R>::type* __restrict__ part) {
    typedef typename Cx<R>::type C;
    typedef typename Mfma<R>::acc Acc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, q = lane >> 4;
    const int row0 = blockIdx.x * MF_TM + wave * 32;
    const int col0 = blockIdx.y * MF_TN;
    const int nchunks = (n + MF_KC - 1) / MF_KC;
    const int kc0 = blockIdx.z * chunks_per_split;
    const int kc1 = min(nchunks, kc0 + chunks_per_split);
    // rows and columns past the end read row/column 0; their results are not stored
    const C* pa[2];
    const C* px[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int row = row0 + 16 * t + li, col = col0 + 16 * t + li;
        pa[t] = A + (int64_t)(row < n ? row : 0) * n;
        px[t] = rhs_nn(X, col < nrhs ? col : 0, bs);
    }
    Acc acc[2][2][2];                       // [row tile][column tile][re, im]
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[t][c][p][r] = (R)0;
    // Steps below n / MF_KC lie inside the matrix and load without a mask; the
    // one partial step at the end loads entry 0 in place of entries k >= n and
    // zeroes their A values (A is finite). No load sits under a branch.
    auto load = [&](int kc, C (&ra)[2][4], C (&rx)[2][4]) {
        if constexpr (WIDE) {
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int k = kc * MF_KC + 8 * v + 2 * q;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const float4 a4 = *reinterpret_cast<const float4*>(pa[t] + k);
                    const float4 x4 = *reinterpret_cast<const float4*>(px[t] + k);
                    ra[t][2 * v].x = a4.x;
                    ra[t][2 * v].y = a4.y;
                    ra[t][2 * v + 1].x = a4.z;
                    ra[t][2 * v + 1].y = a4.w;
                    rx[t][2 * v].x = x4.x;
                    rx[t][2 * v].y = x4.y;
                    rx[t][2 * v + 1].x = x4.z;
                    rx[t][2 * v + 1].y = x4.w;
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = kc * MF_KC + 4 * u + q;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    ra[t][u] = pa[t][k];
                    rx[t][u] = px[t][k];
                }
            }
        }
    };
    auto step = [&](const C (&ra)[2][4], const C (&rx)[2][4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const R xr = rx[c][u].x, xi = rx[c][u].y;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    acc[t][c][0] = Mfma<R>::fma(ra[t][u].x, xr, acc[t][c][0]);
                    acc[t][c][1] = Mfma<R>::fma(ra[t][u].x, xi, acc[t][c][1]);
                    acc[t][c][0] = Mfma<R>::fma(ra[t][u].y, -xi, acc[t][c][0]);
                    acc[t][c][1] = Mfma<R>::fma(ra[t][u].y, xr, acc[t][c][1]);
                }
            }
        }
    };
    // one register buffer: the waves sharing a SIMD (5 in complex64, 3 in
    // complex128) hide each other's load latency (measured faster than a
    // second buffer, or than 64 rows per wave, both of which cost occupancy)
    const int nfull = n / MF_KC;              // steps that lie inside the matrix
    const int kf = max(kc0, min(kc1, nfull)); // this range's unmasked steps: [kc0, kf)
    C a0[2][4], x0[2][4];
    for (int kc = kc0; kc < kf; ++kc) {
        load(kc, a0, x0);
        step(a0, x0);
    }
    if (nfull >= kc0 && nfull < kc1) {        // the partial last step, in this range
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = nfull * MF_KC + (WIDE ? 8 * (u >> 1) + 2 * q + (u & 1) : 4 * u + q);
            const int kk = k < n ? k : 0;
            const R m = k < n ? (R)1 : (R)0;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const C va = pa[t][kk];
                a0[t][u].x = va.x * m;
                a0[t][u].y = va.y * m;
                x0[t][u] = px[t][kk];
            }
        }
        step(a0, x0);
    }
    const int ncol = gridDim.y * MF_TN;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int col = col0 + 16 * c + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + 16 * t + Mfma<R>::row(q, r);
                if (row < n) {
                    C v;
                    v.x = acc[t][c][0][r];
                    v.y = acc[t][c][1][r];
                    part[((int64_t)blockIdx.z * ncol + col) * n + row] = v;
                }
            }
        }
}

template <class C>
__global__ void __launch_bounds__(256) k_coarsest_sum(int n, int nrhs, int64_t bs, int ks,
                                                      int ncol, const C* __restrict__ part,
                                                      C* __restrict__ Y) {
    const int col = blockIdx.y;
    const int row = blockIdx.x * 256 + threadIdx.x;
    if (row >= n || col >= nrhs) return;
    C acc = part[(int64_t)col * n + row];
    for (int z = 1; z < ks; ++z) acc = cadd(acc, part[((int64_t)z * ncol + col) * n + row]);
    rhs_nn(Y, col, bs)[row] = acc;
}

// split of k: about three resident blocks per CU in one round (a second,
// partly filled round of blocks measured slower), at least 4 steps per split
int gemm_splits(int n, int nrhs) {
    const int nchunks = (n + MF_KC - 1) / MF_KC;
    const int blocks = ((n + MF_TM - 1) / MF_TM) * ((nrhs + MF_TN - 1) / MF_TN);
    int ks = 768 / blocks;
    if (ks > nchunks / 4) ks = nchunks / 4;
    return ks < 1 ? 1 : ks;
}

template <class R>
hipError_t gemm(int n, const typename Cx<R>::type* A, const typename Cx<R>::type* x,
                typename Cx<R>::type* y, typename Cx<R>::type* part, hipStream_t s,
                const Batch& bt) {
    typedef typename Cx<R>::type C;
    if (n > HH_MAX_COARSE_LIMIT) return hipErrorInvalidValue;
    const int groups = (bt.n + MF_TN - 1) / MF_TN;
    const int ks = gemm_splits(n, bt.n);
    const int nchunks = (n + MF_KC - 1) / MF_KC;
    const int cps = (nchunks + ks - 1) / ks;
    const dim3 grid((n + MF_TM - 1) / MF_TM, groups, ks);
    // with n even, A and X on 16 bytes and a per-source stride that is a
    // multiple of 16 (the workspace layout keeps 256), every row of A and every
    // X entry pair 2i, 2i + 1 is 16-byte aligned
    if (sizeof(C) == 8 && n % 2 == 0 && bt.bs % 16 == 0 &&
        reinterpret_cast<uintptr_t>(x) % 16 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0)
        HH_LAUNCH((k_coarsest_mfma<R, sizeof(C) == 8>), grid, dim3(256), 0, s, n, A, x, bt.n,
                  bt.bs, cps, part);
    else
        HH_LAUNCH((k_coarsest_mfma<R, false>), grid, dim3(256), 0, s, n, A, x, bt.n, bt.bs, cps,
                  part);
    HH_LAUNCH((k_coarsest_sum<C>), dim3((n + 255) / 256, bt.n), dim3(256), 0, s, n, bt.n, bt.bs,
              ks, groups * MF_TN, (const C*)part, y);
    return hipGetLastError();
}

template <class C, class X>
hipError_t gemv(int n, const C* A, const X* x, C* y, const int* active, hipStream_t s,
                const Batch& bt) {
    if (n > HH_MAX_COARSE_LIMIT) return hipErrorInvalidValue;
    if (bt.n == 1) {
        HH_LAUNCH((k_gemv_pred<C, X>), dim3(n), dim3(256), 0, s, n, A, x, y, active);
    } else {
        HH_LAUNCH((k_gemv_batch<C, X>), dim3(n, bt.n), dim3(256), 0, s, n, A, x, y, active,
                  bt.bs);
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
size_t vc_gemm_scratch_bytes(int n, int nrhs) {
    const int groups = (nrhs + MF_TN - 1) / MF_TN;
    return (size_t)gemm_splits(n, nrhs) * groups * MF_TN * n * sizeof(cplx);
}
hipError_t launch_vc_gemm(int n, const cplx* A, const cplx* x, cplx* y, void* scratch,
                          hipStream_t s, const Batch& bt) {
    return gemm<double>(n, A, x, y, static_cast<cplx*>(scratch), s, bt);
}
hipError_t launch_vc_gemm(int n, const cplxf* A, const cplxf* x, cplxf* y, void* scratch,
                          hipStream_t s, const Batch& bt) {
    return gemm<float>(n, A, x, y, static_cast<cplxf*>(scratch), s, bt);
}

}  // namespace hh
