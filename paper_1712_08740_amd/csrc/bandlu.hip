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

// 1 / z as conj(z) / |z|^2, the real reciprocal from the hardware estimate
// refined by two Newton steps (exact division when |z|^2 is not a normal
// number well inside the range)
__device__ __forceinline__ cplx crecip(cplx z) {
    const double d = z.x * z.x + z.y * z.y;
    if (!(d > 1e-290 && d < 1e290)) return cdiv(mk(1.0, 0.0), z);
    double r = __builtin_amdgcn_rcp(d);
    r = r * (2.0 - d * r);
    r = r * (2.0 - d * r);
    return mk(z.x * r, -z.y * r);
}

// a -= l y with four fused multiply-adds
__device__ __forceinline__ void msub4(cplx& a, cplx l, cplx y) {
    a.x = fma(-l.x, y.x, a.x);
    a.x = fma(l.y, y.y, a.x);
    a.y = fma(-l.x, y.y, a.y);
    a.y = fma(-l.y, y.x, a.y);
}

// Blocked right-looking LU without pivoting of the band (one workgroup of
// LU_T threads). Columns are taken LU_P at a time. The panel (rows k0 ..
// k0+kp+b-1 of those columns) and the block U12 of U to its right (rows k0 ..
// k0+kp-1, the b columns after the panel) are factored in registers: thread i
// holds panel row i, thread nr + j column j of U12. At each column the pivot
// row and the column below the pivot are published in LDS (double buffered:
// one barrier per column), every panel row scales its entry and updates the
// rest of its row, every U12 column updates its entries below the pivot.
// Then the trailing b x b block takes the rank-kp update L21 U12 from global
// memory, each thread a 4 x 4 tile in registers. Entries outside the band are
// zero and stay zero. flag[0] = 1 on a zero or non-finite pivot.
// LDS: 2 b LU_P + 4 LU_P complex.
constexpr int LU_P = 16;
constexpr int LU_T = 512;

__host__ __device__ inline size_t lu_blk_lds(int b) {
    return (size_t)(2 * b * LU_P + 4 * LU_P) * sizeof(cplx);
}

__global__ void __launch_bounds__(LU_T) k_band_lu_blk(cplx* __restrict__ AB, int n, int b,
                                                      int* __restrict__ flag) {
    extern __shared__ cplx lds[];
    const int w = 2 * b + 1;
    const int tid = threadIdx.x;
    cplx* l21 = lds;                             // [b][LU_P]: panel rows below the top block
    cplx* u12 = lds + b * LU_P;                  // [LU_P][b]
    cplx* brow = u12 + LU_P * b;                 // [2][LU_P]: pivot row
    cplx* bcol = brow + 2 * LU_P;                // [2][LU_P]: column below the pivot, top block
    auto at = [&](int r, int c) -> cplx* { return AB + (int64_t)r * w + (c - r + b); };
    for (int k0 = 0; k0 < n; k0 += LU_P) {
        const int kp = min(LU_P, n - k0);
        const int nr = min(kp + b, n - k0);          // panel rows
        const int nc = min(b, n - k0 - kp);          // columns of U12 and of the trailing block
        const bool isrow = tid < nr, iscol = !isrow && tid < nr + nc;
        const int j = tid - nr;
        // every load is issued (from entry 0 when out of range) and masked: loads
        // under branches would each be waited for before the next is issued
        cplx v[LU_P];
#pragma unroll
        for (int t = 0; t < LU_P; ++t) {
            const bool okr = isrow && t < kp && tid - t <= b && t - tid <= b;
            const bool okc = iscol && t < kp && kp + j - t <= b;
            const cplx* q = okr ? at(k0 + tid, k0 + t) : okc ? at(k0 + t, k0 + kp + j) : AB;
            v[t] = cscale(*q, (okr || okc) ? 1.0 : 0.0);
        }
#pragma unroll
        for (int c = 0; c < LU_P; ++c) {
            if (c < kp) {                        // uniform: kp < LU_P only for the last panel
            const int par = c & 1;
            if (isrow && tid == c) {
#pragma unroll
                for (int t = c; t < LU_P; ++t) brow[par * LU_P + t] = v[t];
            }
            if (isrow && tid > c && tid < kp) bcol[par * LU_P + tid] = v[c];
            __syncthreads();
            const cplx piv = brow[par * LU_P + c];
            if (tid == 0 && !(isfinite(piv.x) && isfinite(piv.y) && (piv.x != 0.0 || piv.y != 0.0)))
                *flag = 1;
            const cplx ip = crecip(piv);
            if (isrow && tid > c) {
                const cplx l = cmul(v[c], ip);
                v[c] = l;
#pragma unroll
                for (int t = c + 1; t < LU_P; ++t) msub4(v[t], l, brow[par * LU_P + t]);
            }
            if (iscol) {
                const cplx uc = v[c];
#pragma unroll
                for (int i = c + 1; i < LU_P; ++i)
                    if (i < kp) msub4(v[i], cmul(bcol[par * LU_P + i], ip), uc);
            }
            }
        }
        // factors out; L21 and U12 into LDS for the trailing update
        if (isrow) {
#pragma unroll
            for (int t = 0; t < LU_P; ++t) {
                if (t < kp && tid - t <= b && t - tid <= b) *at(k0 + tid, k0 + t) = v[t];
                if (tid >= kp) l21[(tid - kp) * LU_P + t] = v[t];
            }
        }
        if (iscol) {
#pragma unroll
            for (int t = 0; t < LU_P; ++t) {
                if (t < kp && kp + j - t <= b) *at(k0 + t, k0 + kp + j) = v[t];
                u12[t * b + j] = v[t];
            }
        }
        __syncthreads();
        // trailing block: rows and columns k0+kp .. (nr - kp rows, nc columns)
        const int r22 = nr - kp;
        const int tr = (r22 + 3) / 4, tc = (nc + 3) / 4;
        for (int e = tid; e < tr * tc; e += LU_T) {
            const int r0 = 4 * (e / tc), c0 = 4 * (e % tc);
            cplx acc[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool ok = r0 + a < r22 && c0 + q < nc;
                    acc[a][q] = cscale(*(ok ? at(k0 + kp + r0 + a, k0 + kp + c0 + q) : AB),
                                       ok ? 1.0 : 0.0);
                }
            for (int t = 0; t < kp; ++t) {
                cplx l[4], u[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) l[a] = r0 + a < r22 ? l21[(r0 + a) * LU_P + t] : mk(0.0, 0.0);
#pragma unroll
                for (int q = 0; q < 4; ++q) u[q] = c0 + q < nc ? u12[t * b + c0 + q] : mk(0.0, 0.0);
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int q = 0; q < 4; ++q) msub4(acc[a][q], l[a], u[q]);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (r0 + a < r22 && c0 + q < nc) *at(k0 + kp + r0 + a, k0 + kp + c0 + q) = acc[a][q];
        }
        __syncthreads();
    }
}

// Lc[i][t] = L(i+1+t, i), Uc[i][t] = U(i-1-t, i) (0 outside), Ui[i] = 1 / U(i, i)
__global__ void __launch_bounds__(256) k_band_split(const cplx* __restrict__ AB, int64_t n, int b,
                                                    cplx* __restrict__ Lc, cplx* __restrict__ Uc,
                                                    cplx* __restrict__ Ui) {
    const int w = 2 * b + 1;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * b) return;
    const int64_t i = e / b;
    const int t = (int)(e - i * b);
    const int64_t rl = i + 1 + t, ru = i - 1 - t;
    Lc[e] = rl < n ? AB[rl * w + (b - 1 - t)] : mk(0.0, 0.0);
    Uc[e] = ru >= 0 ? AB[ru * w + (b + 1 + t)] : mk(0.0, 0.0);
    if (t == 0) Ui[i] = cdiv(mk(1.0, 0.0), AB[i * w + b]);
}

// Columns c0 .. c0+C-1 of M^{-1} (M = L U, the transposed renumbered operator)
// by forward substitution with the unit lower factor from e_c, then backward
// substitution with U, both right-looking, by one wavefront. The lanes form
// 64/R groups of R; group g takes CG of the columns and lane r of a group the
// rows r, r + R, ... of the current block of R rows and of the SLOTS - 1 blocks
// after it (the rows the current row can still update: at most b away), in
// registers. At each row the lanes that own it pass their values to their
// group through LDS; when a block is done its slot is written out and the
// slots shift by one. Factor entries are loaded D rows ahead. The forward
// result is kept in `out` and read back by the backward pass.
//
// out receives row c0+c of A'^{-1} (A' = M^T): at (c0+c) n + q in the band
// numbering, or at orig(c0+c) n + orig(q) (the natural numbering of A^{-1})
// when `natural` is set. flag[0] |= 2 for a non-finite entry of the inverse.
// a -= l y with four fused multiply-adds
__device__ __forceinline__ void msub(cplx& a, cplx l, cplx y) {
    a.x = fma(-l.x, y.x, a.x);
    a.x = fma(l.y, y.y, a.x);
    a.y = fma(-l.x, y.y, a.y);
    a.y = fma(-l.y, y.x, a.y);
}

template <int R, int SLOTS, int CG, int D>
__global__ void __launch_bounds__(64) k_band_inv(const cplx* __restrict__ Lc,
                                                 const cplx* __restrict__ Uc,
                                                 const cplx* __restrict__ Ui, int n, int b,
                                                 Numbering num, int natural,
                                                 cplx* __restrict__ out, int* __restrict__ flag) {
    static_assert(64 % R == 0 && R % D == 0, "R divides the wavefront, D divides R");
    constexpr int C = CG * (64 / R);
    const int rl = threadIdx.x % R;                // row lane
    const int cb = (threadIdx.x / R) * CG;         // first column of this lane's group
    const int c0 = blockIdx.x * C;
    const int nc = min(C, n - c0);
    __shared__ cplx ybuf[2][C];
    auto at = [&](int c, int64_t q) -> int64_t {
        return natural ? num.orig(c0 + c) * (int64_t)n + num.orig(q) : (int64_t)(c0 + c) * n + q;
    };
    cplx acc[SLOTS][CG];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s)
#pragma unroll
        for (int k = 0; k < CG; ++k) {
            const int c = cb + k;
            acc[s][k] = mk((c < nc && s == c / R && rl == c % R) ? 1.0 : 0.0, 0.0);
        }

    // ---- forward: y = L^{-1} e_c, rows c0 .. n-1 (the rows above c0 are zero)
    // L(row, i) = Lc[i][row - i - 1] for the row of slot s in the block at base
    // Every load is issued (from entry 0 when out of range, a finite factor
    // entry) and scaled by 0 or 1: a load under a branch makes the compiler wait
    // for all outstanding loads before its first use, defeating the prefetch.
    auto lval = [&](int i, int base, int s) -> cplx {
        const int row = base + R * s + rl;
        const int t = row - i - 1;
        const bool ok = i < n && t >= 0 && t < b && row < n;
        return cscale(Lc[ok ? (int64_t)i * b + t : 0], ok ? 1.0 : 0.0);
    };
    cplx fv[D][SLOTS];
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) fv[d][s] = lval(c0 + d, c0, s);
    for (int base = c0; base < n; base += R) {
        for (int g = 0; g < R && base + g < n; g += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int i = base + g + d;
                if (i < n) {
                    if (rl == g + d) {
#pragma unroll
                        for (int k = 0; k < CG; ++k) ybuf[i & 1][cb + k] = acc[0][k];
                    }
                    __syncthreads();
                    cplx l[SLOTS];
                    const int bn = (g + d + D >= R) ? base + R : base;     // block of row i + D
#pragma unroll
                    for (int s = 0; s < SLOTS; ++s) {
                        l[s] = fv[d][s];
                        fv[d][s] = lval(i + D, bn, s);
                    }
#pragma unroll
                    for (int k = 0; k < CG; ++k) {
                        const cplx y = ybuf[i & 1][cb + k];
#pragma unroll
                        for (int s = 0; s < SLOTS; ++s) msub(acc[s][k], l[s], y);
                    }
                }
            }
        }
        const int row = base + rl;
        if (row < n) {
#pragma unroll
            for (int k = 0; k < CG; ++k)
                if (cb + k < nc) out[at(cb + k, row)] = acc[0][k];
        }
#pragma unroll
        for (int s = 0; s + 1 < SLOTS; ++s)
#pragma unroll
            for (int k = 0; k < CG; ++k) acc[s][k] = acc[s + 1][k];
#pragma unroll
        for (int k = 0; k < CG; ++k) acc[SLOTS - 1][k] = mk(0.0, 0.0);
    }
    // the forward results are read back by other lanes: complete the stores and
    // read them past the first-level cache
    __threadfence();
    __syncthreads();
    auto yval = [&](int row, int k) -> cplx {
        const bool ok = row >= c0 && cb + k < nc;
        double* q = reinterpret_cast<double*>(out + (ok ? at(cb + k, row) : 0));
        const cplx v = mk(__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                          __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        return ok ? v : mk(0.0, 0.0);
    };

    // ---- backward: x = U^{-1} y, rows n-1 .. 0; row top - R s - rl in slot s
    auto uval = [&](int i, int top, int s) -> cplx {
        const int row = top - R * s - rl;
        const int t = i - 1 - row;
        const bool ok = i >= 0 && t >= 0 && t < b && row >= 0;
        return cscale(Uc[ok ? (int64_t)i * b + t : 0], ok ? 1.0 : 0.0);
    };
    auto uinv = [&](int row) -> cplx {
        return cscale(Ui[row >= 0 ? row : 0], row >= 0 ? 1.0 : 0.0);
    };
    const int top0 = n - 1;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s)
#pragma unroll
        for (int k = 0; k < CG; ++k) acc[s][k] = yval(top0 - R * s - rl, k);
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) fv[d][s] = uval(top0 - d, top0, s);
    cplx dinv = uinv(top0 - rl);
    bool bad = false;
    for (int top = top0; top >= 0; top -= R) {
        // the slot entering after this block, and the diagonal of the next block
        cplx ynext[CG];
        const int rn = top - R * SLOTS - rl;
#pragma unroll
        for (int k = 0; k < CG; ++k) ynext[k] = yval(rn, k);
        const cplx dnext = uinv(top - R - rl);
        for (int g = 0; g < R && top - g >= 0; g += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int i = top - g - d;
                if (i >= 0) {
                    if (rl == g + d) {
#pragma unroll
                        for (int k = 0; k < CG; ++k) {
                            acc[0][k] = cmul(acc[0][k], dinv);
                            ybuf[i & 1][cb + k] = acc[0][k];
                        }
                    }
                    __syncthreads();
                    cplx u[SLOTS];
                    const int tn = (g + d + D >= R) ? top - R : top;       // block of row i - D
#pragma unroll
                    for (int s = 0; s < SLOTS; ++s) {
                        u[s] = fv[d][s];
                        fv[d][s] = uval(i - D, tn, s);
                    }
#pragma unroll
                    for (int k = 0; k < CG; ++k) {
                        const cplx x = ybuf[i & 1][cb + k];
#pragma unroll
                        for (int s = 0; s < SLOTS; ++s) msub(acc[s][k], u[s], x);
                    }
                }
            }
        }
        const int row = top - rl;
        if (row >= 0) {
#pragma unroll
            for (int k = 0; k < CG; ++k)
                if (cb + k < nc) {
                    const cplx v = acc[0][k];
                    bad = bad || !(isfinite(v.x) && isfinite(v.y));
                    out[at(cb + k, row)] = v;
                }
        }
#pragma unroll
        for (int s = 0; s + 1 < SLOTS; ++s)
#pragma unroll
            for (int k = 0; k < CG; ++k) acc[s][k] = acc[s + 1][k];
#pragma unroll
        for (int k = 0; k < CG; ++k) acc[SLOTS - 1][k] = ynext[k];
        dinv = dnext;
    }
    if (bad) atomicOr(flag, 2);
}

}  // namespace

int band_halfwidth(int nz, int nx) { return (nz < nx ? nz : nx) + 1; }

bool band_renumbered(int nz, int nx) { return nz < nx; }

size_t band_scratch_bytes(int nz, int nx) {
    const int64_t n = (int64_t)nz * nx;
    const int b = band_halfwidth(nz, nx);
    return (size_t)(n * (2 * b + 1) + 2 * n * b + n) * sizeof(cplx);
}

template <int R, int SLOTS, int CG, int D>
static void inv_launch(const cplx* Lc, const cplx* Uc, const cplx* Ui, int n, int b, Numbering num,
                       int natural, cplx* A, int* flag, hipStream_t s) {
    constexpr int C = CG * (64 / R);
    HH_LAUNCH((k_band_inv<R, SLOTS, CG, D>), dim3((unsigned)((n + C - 1) / C)), dim3(64), 0, s, Lc,
              Uc, Ui, n, b, num, natural, A, flag);
}

hipError_t band_invert(int nz, int nx, cplx* A, void* scratch, int* flag, bool natural,
                       hipStream_t s) {
    const int64_t n = (int64_t)nz * nx;
    const int b = band_halfwidth(nz, nx);
    if (b > 255) return hipErrorInvalidValue;
    Numbering num{nz, nx, band_renumbered(nz, nx)};
    cplx* AB = static_cast<cplx*>(scratch);
    cplx* Lc = AB + n * (2 * b + 1);
    cplx* Uc = Lc + n * b;
    cplx* Ui = Uc + n * b;
    HH_LAUNCH(k_band_extract, dim3((unsigned)((n * (2 * b + 1) + 255) / 256)), dim3(256), 0, s, A,
              n, b, num, AB);
    const size_t lu_lds = lu_blk_lds(b);
    if (lu_lds <= 65536)                          // b <= 125
        HH_LAUNCH(k_band_lu_blk, dim3(1), dim3(LU_T), lu_lds, s, AB, (int)n, b, flag);
    else
        HH_LAUNCH(k_band_lu, dim3(1), dim3(LU_THREADS), 0, s, AB, (int)n, b, flag);
    HH_LAUNCH(k_band_split, dim3((unsigned)((n * b + 255) / 256)), dim3(256), 0, s, AB, n, b, Lc,
              Uc, Ui);
    // the window of a block of R rows reaches b rows further: 1 + ceil(b / R) slots
    const int nat = natural || !num.zfast ? 1 : 0;
    if (b <= 16)
        inv_launch<16, 2, 4, 8>(Lc, Uc, Ui, (int)n, b, num, nat, A, flag, s);
    else if (b <= 32)
        inv_launch<16, 3, 4, 8>(Lc, Uc, Ui, (int)n, b, num, nat, A, flag, s);
    else if (b <= 64)
        inv_launch<16, 5, 4, 4>(Lc, Uc, Ui, (int)n, b, num, nat, A, flag, s);
    else if (b <= 96)
        inv_launch<16, 7, 4, 2>(Lc, Uc, Ui, (int)n, b, num, nat, A, flag, s);
    else if (b <= 128)
        inv_launch<16, 9, 4, 2>(Lc, Uc, Ui, (int)n, b, num, nat, A, flag, s);
    else
        inv_launch<64, 5, 4, 4>(Lc, Uc, Ui, (int)n, b, num, nat, A, flag, s);
    return hipGetLastError();
}

}  // namespace hh
