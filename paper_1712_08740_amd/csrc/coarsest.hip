// Coarsest-level solve of the V-cycle: z = A^{-1} b with the explicit inverse
// computed at set-up, as a dense complex matrix-vector product with a
// fixed-order reduction.
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
// goes to a library GEMM in the solve driver.
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
// at once): A row-major n x n, column b of X and Y in right-hand side b's
// workspace (bs bytes after column b - 1).
//
// k_coarsest_gemm: a block owns 64 rows, 32 right-hand sides (group
// blockIdx.y) and one of KS contiguous ranges of k (blockIdx.z), streamed
// through LDS in chunks of 32 (the next chunk's loads are issued before the
// current chunk is consumed). Thread (r, g) owns row r and right-hand sides
// 8g..8g+7 and sums its k range in increasing order into part[z][col][row].
// k_coarsest_sum adds the KS partial sums in order: every result depends only
// on A and its own column, in a fixed order. A is read once per group of 32
// right-hand sides; X once per 64 rows.
constexpr int GM_TM = 64, GM_TK = 32, GM_TN = 32;

template <class C>
__global__ void __launch_bounds__(256) k_coarsest_gemm(int n, const C* __restrict__ A,
                                                       const C* __restrict__ X, int nrhs,
                                                       int64_t bs, int chunks_per_split,
                                                       C* __restrict__ part) {
    constexpr int TM = GM_TM, TK = GM_TK, TN = GM_TN;
    constexpr int CPT = TN / (256 / TM);      // 8 right-hand sides per thread
    constexpr int LA = TM * TK / 256, LX = TK * TN / 256;
    __shared__ C As[TM][TK + 1];
    __shared__ C Xs[TK][TN];
    const int tid = threadIdx.x;
    const int r = tid % TM, g = tid / TM;
    const int r0 = blockIdx.x * TM, c0 = blockIdx.y * TN;
    const int nchunks = (n + TK - 1) / TK;
    const int kc0 = blockIdx.z * chunks_per_split;
    const int kc1 = min(nchunks, kc0 + chunks_per_split);
    C acc[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) acc[c] = czero<C>();
    C ra[LA], rx[LX];
    auto load = [&](int kc) {
        const int k0 = kc * TK;
#pragma unroll
        for (int i = 0; i < LA; ++i) {            // A tile, coalesced along k
            const int e = tid + 256 * i;
            const int row = r0 + e / TK, k = k0 + e % TK;
            ra[i] = (row < n && k < n) ? A[(int64_t)row * n + k] : czero<C>();
        }
#pragma unroll
        for (int i = 0; i < LX; ++i) {            // X tile, coalesced along k
            const int e = tid + 256 * i;
            const int col = c0 + e / TK, k = k0 + e % TK;
            rx[i] = (col < nrhs && k < n) ? rhs_nn(X, col, bs)[k] : czero<C>();
        }
    };
    if (kc0 < kc1) load(kc0);
    for (int kc = kc0; kc < kc1; ++kc) {
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int e = tid + 256 * i;
            As[e / TK][e % TK] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < LX; ++i) {
            const int e = tid + 256 * i;
            Xs[e % TK][e / TK] = rx[i];
        }
        __syncthreads();
        if (kc + 1 < kc1) load(kc + 1);          // in flight while this chunk is consumed
#pragma unroll 8
        for (int kk = 0; kk < TK; ++kk) {
            const C a = As[r][kk];
#pragma unroll
            for (int c = 0; c < CPT; ++c) acc[c] = cadd(acc[c], cmul(a, Xs[kk][g * CPT + c]));
        }
        __syncthreads();
    }
    const int ncol = gridDim.y * TN;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int col = c0 + g * CPT + c;
        if (r0 + r < n)
            part[((int64_t)blockIdx.z * ncol + col) * n + r0 + r] = acc[c];
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

// split of k: enough blocks to give every CU a few, at least 4 chunks per split
int gemm_splits(int n, int nrhs) {
    const int nchunks = (n + GM_TK - 1) / GM_TK;
    const int blocks = ((n + GM_TM - 1) / GM_TM) * ((nrhs + GM_TN - 1) / GM_TN);
    int ks = (1024 + blocks - 1) / blocks;
    if (ks > nchunks / 4) ks = nchunks / 4;
    return ks < 1 ? 1 : ks;
}

template <class C>
hipError_t gemm(int n, const C* A, const C* x, C* y, C* part, hipStream_t s, const Batch& bt) {
    if (n > HH_MAX_COARSE_LIMIT) return hipErrorInvalidValue;
    const int groups = (bt.n + GM_TN - 1) / GM_TN;
    const int ks = gemm_splits(n, bt.n);
    const int nchunks = (n + GM_TK - 1) / GM_TK;
    const int cps = (nchunks + ks - 1) / ks;
    HH_LAUNCH((k_coarsest_gemm<C>), dim3((n + GM_TM - 1) / GM_TM, groups, ks), dim3(256), 0, s, n,
              A, x, bt.n, bt.bs, cps, part);
    HH_LAUNCH((k_coarsest_sum<C>), dim3((n + 255) / 256, bt.n), dim3(256), 0, s, n, bt.n, bt.bs,
              ks, groups * GM_TN, (const C*)part, y);
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
    const int groups = (nrhs + GM_TN - 1) / GM_TN;
    return (size_t)gemm_splits(n, nrhs) * groups * GM_TN * n * sizeof(cplx);
}
hipError_t launch_vc_gemm(int n, const cplx* A, const cplx* x, cplx* y, void* scratch,
                          hipStream_t s, const Batch& bt) {
    return gemm(n, A, x, y, static_cast<cplx*>(scratch), s, bt);
}
hipError_t launch_vc_gemm(int n, const cplxf* A, const cplxf* x, cplxf* y, void* scratch,
                          hipStream_t s, const Batch& bt) {
    return gemm(n, A, x, y, static_cast<cplxf*>(scratch), s, bt);
}

}  // namespace hh
