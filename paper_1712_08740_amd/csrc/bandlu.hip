// Explicit inverse of the coarsest multigrid operator through a banded LU
// factorisation (set-up of the direct coarsest solve).
//
// The coarsest operator is a 9-point (Galerkin) or 5-point stencil on an
// nz x nx grid: numbered with the shorter dimension fastest it is banded with
// half-bandwidth b = min(nz, nx) + 1, so the factorisation costs n b^2 instead
// of n^3 and the n solves for the columns of the inverse cost 2 n^2 b.
// Gaussian elimination runs without pivoting: the operator is complex
// symmetric with a positive definite imaginary part (the damping and shift
// terms of Eq. 6 with beta2 > 0, and the absorbing rows), so every leading
// principal submatrix is nonsingular (x^H A x has a positive imaginary part);
// a zero or non-finite pivot is reported.
//
// We factor the transpose A'^T of the renumbered matrix A' = Pi A Pi^T: its
// unit vectors solve to the rows of A'^{-1}, which are rows of A^{-1} with
// permuted columns, written straight into the row-major inverse.
#include "hh_internal.h"

namespace hh {

namespace {

constexpr int LU_THREADS = 1024;
constexpr int SOLVE_COLS = 16;      // columns of the inverse per solve workgroup
constexpr int SOLVE_W = 256;        // circular window of the solve (> b)

struct Numbering {
    int nz, nx;
    bool zfast;                     // renumber with z fastest (nz < nx)
    __host__ __device__ int64_t orig(int64_t q) const {   // pi^{-1}(q)
        if (!zfast) return q;
        const int64_t ix = q / nz, iz = q - ix * nz;
        return iz * nx + ix;
    }
};

// AB[i][d] = A'^T(i, i + d - b) = A(orig(i + d - b), orig(i)), |d - b| <= b
__global__ void __launch_bounds__(256) k_band_extract(const cplx* __restrict__ A, int64_t n, int b,
                                                      Numbering num, cplx* __restrict__ AB) {
    const int w = 2 * b + 1;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * w) return;
    const int64_t i = e / w;
    const int d = (int)(e - i * w);
    const int64_t j = i + d - b;
    cplx v = mk(0.0, 0.0);
    if (j >= 0 && j < n) v = A[num.orig(j) * n + num.orig(i)];
    AB[e] = v;
}

// In-place LU without pivoting of the band (one workgroup; step k: scale the
// column of L below the pivot, then the rank-1 update of the b x b trailing
// window). flag[0] = 1 on a zero or non-finite pivot.
__global__ void __launch_bounds__(LU_THREADS) k_band_lu(cplx* __restrict__ AB, int n, int b,
                                                        int* __restrict__ flag) {
    const int w = 2 * b + 1;
    const int tid = threadIdx.x;
    __shared__ cplx srow[2 * 256 + 1];             // U row k (columns k+1..k+b)
    __shared__ cplx scol[2 * 256 + 1];             // L column k (rows k+1..k+b)
    for (int k = 0; k < n; ++k) {
        const cplx piv = AB[(int64_t)k * w + b];
        const int m = min(b, n - 1 - k);           // rows / columns in the window
        if (tid == 0 && !(isfinite(piv.x) && isfinite(piv.y) && (piv.x != 0.0 || piv.y != 0.0)))
            *flag = 1;
        for (int t = tid; t < m; t += LU_THREADS) {
            cplx* lp = &AB[(int64_t)(k + 1 + t) * w + (b - 1 - t)];
            const cplx l = cdiv(*lp, piv);
            *lp = l;
            scol[t] = l;
            srow[t] = AB[(int64_t)k * w + b + 1 + t];
        }
        __syncthreads();
        for (int e = tid; e < m * m; e += LU_THREADS) {
            const int ti = e / m, tj = e - ti * m;
            cplx* a = &AB[(int64_t)(k + 1 + ti) * w + (b + tj - ti)];
            *a = csub(*a, cmul(scol[ti], srow[tj]));
        }
        __syncthreads();
    }
}

// Lc[i][t] = L(i+1+t, i), Uc[i][t] = U(i-1-t, i) (0 outside), Ud[i] = U(i, i)
__global__ void __launch_bounds__(256) k_band_split(const cplx* __restrict__ AB, int64_t n, int b,
                                                    cplx* __restrict__ Lc, cplx* __restrict__ Uc,
                                                    cplx* __restrict__ Ud) {
    const int w = 2 * b + 1;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * b) return;
    const int64_t i = e / b;
    const int t = (int)(e - i * b);
    const int64_t rl = i + 1 + t, ru = i - 1 - t;
    Lc[e] = rl < n ? AB[rl * w + (b - 1 - t)] : mk(0.0, 0.0);
    Uc[e] = ru >= 0 ? AB[ru * w + (b + 1 + t)] : mk(0.0, 0.0);
    if (t == 0) Ud[i] = AB[i * w + b];
}

// Columns c0 .. c0+SOLVE_COLS-1 of (A'^T)^{-1}: forward with unit L from e_c,
// backward with U, both right-looking over a circular window in LDS; the
// result (row orig(c) of A^{-1}) is written into Ainv, which holds the forward
// result in between. The next row's factor entries (and, backward, the
// forward results) are loaded one step ahead.
__global__ void __launch_bounds__(64) k_band_solve(const cplx* __restrict__ Lc,
                                                   const cplx* __restrict__ Uc,
                                                   const cplx* __restrict__ Ud, int n, int b,
                                                   Numbering num, cplx* __restrict__ Ainv) {
    constexpr int C = SOLVE_COLS, W = SOLVE_W, SLOTS = SOLVE_W / 64;
    __shared__ cplx win[C][W];
    const int lane = threadIdx.x;
    const int c0 = blockIdx.x * C;
    const int nc = min(C, n - c0);
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) win[c][lane + 64 * s] = mk(0.0, 0.0);
    __syncthreads();
    if (lane < nc) win[lane][(c0 + lane) % W] = mk(1.0, 0.0);
    const int64_t myrow = lane < nc ? num.orig(c0 + lane) : 0;
    __syncthreads();
    auto load_band = [&](const cplx* F, int i, cplx* out) {
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int t = lane + 64 * s;
            out[s] = (i >= 0 && i < n && t < b) ? F[(int64_t)i * b + t] : mk(0.0, 0.0);
        }
    };
    // forward: y = L^{-1} e_c (rows before c are zero)
    cplx l[SLOTS], ln[SLOTS];
    load_band(Lc, c0, l);
    for (int i = c0; i < n; ++i) {
        load_band(Lc, i + 1, ln);
        cplx yi[C];
#pragma unroll
        for (int c = 0; c < C; ++c) yi[c] = c < nc ? win[c][i % W] : mk(0.0, 0.0);
        __syncthreads();
        if (lane < nc) {
            Ainv[myrow * n + num.orig(i)] = yi[lane];
            win[lane][i % W] = mk(0.0, 0.0);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (c >= nc) continue;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const int t = lane + 64 * s;
                if (t < b) {
                    cplx& y = win[c][(i + 1 + t) % W];
                    y = csub(y, cmul(l[s], yi[c]));
                }
            }
        }
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) l[s] = ln[s];
        __syncthreads();
    }
    // backward: x = U^{-1} y, accumulating the updates of later rows in the window
    cplx u[SLOTS], un[SLOTS];
    load_band(Uc, n - 1, u);
    cplx d = Ud[n - 1];
    // lane c < nc keeps its own column's forward value of the current row
    cplx yv = (lane < nc && n - 1 >= c0 + lane) ? Ainv[myrow * n + num.orig(n - 1)]
                                                : mk(0.0, 0.0);
    for (int i = n - 1; i >= 0; --i) {
        load_band(Uc, i - 1, un);
        const cplx dn = i > 0 ? Ud[i - 1] : mk(1.0, 0.0);
        const cplx yvn = (lane < nc && i > 0 && i - 1 >= c0 + lane)
                             ? Ainv[myrow * n + num.orig(i - 1)] : mk(0.0, 0.0);
        // x_i for every column: lane c computes its own, then all lanes read them
        if (lane < nc) {
            const cplx xi = cdiv(cadd(yv, win[lane][i % W]), d);
            Ainv[myrow * n + num.orig(i)] = xi;
            win[lane][i % W] = xi;                 // slot i is free after this step: stage x_i
        }
        __syncthreads();
        cplx xi[C];
#pragma unroll
        for (int c = 0; c < C; ++c) xi[c] = c < nc ? win[c][i % W] : mk(0.0, 0.0);
        __syncthreads();
        if (lane < nc) win[lane][i % W] = mk(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (c >= nc) continue;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const int t = lane + 64 * s;
                if (t < b && i - 1 - t >= 0) {
                    cplx& z = win[c][(i - 1 - t + W) % W];
                    z = csub(z, cmul(u[s], xi[c]));
                }
            }
        }
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) u[s] = un[s];
        d = dn;
        yv = yvn;
        __syncthreads();
    }
}

}  // namespace

int band_halfwidth(int nz, int nx) { return (nz < nx ? nz : nx) + 1; }

size_t band_scratch_bytes(int nz, int nx) {
    const int64_t n = (int64_t)nz * nx;
    const int b = band_halfwidth(nz, nx);
    return (size_t)(n * (2 * b + 1) + 2 * n * b + n) * sizeof(cplx);
}

hipError_t band_invert(int nz, int nx, cplx* A, void* scratch, int* flag, hipStream_t s) {
    const int64_t n = (int64_t)nz * nx;
    const int b = band_halfwidth(nz, nx);
    if (b >= SOLVE_W || b > 256) return hipErrorInvalidValue;
    Numbering num{nz, nx, nz < nx};
    cplx* AB = static_cast<cplx*>(scratch);
    cplx* Lc = AB + n * (2 * b + 1);
    cplx* Uc = Lc + n * b;
    cplx* Ud = Uc + n * b;
    HH_LAUNCH(k_band_extract, dim3((unsigned)((n * (2 * b + 1) + 255) / 256)), dim3(256), 0, s, A,
              n, b, num, AB);
    HH_LAUNCH(k_band_lu, dim3(1), dim3(LU_THREADS), 0, s, AB, (int)n, b, flag);
    HH_LAUNCH(k_band_split, dim3((unsigned)((n * b + 255) / 256)), dim3(256), 0, s, AB, n, b, Lc,
              Uc, Ud);
    HH_LAUNCH(k_band_solve, dim3((unsigned)((n + SOLVE_COLS - 1) / SOLVE_COLS)), dim3(64), 0, s, Lc,
              Uc, Ud, (int)n, b, num, A);
    return hipGetLastError();
}

}  // namespace hh
