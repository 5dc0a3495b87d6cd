// Krylov-side kernels of right-preconditioned flexible GMRES (Eq. 7): the
// classical Gram-Schmidt passes of the Arnoldi step as multi-vector complex
// dot products and fused multi-AXPYs, norms, the Givens least-squares update
// of the Hessenberg matrix, back substitution and the solution update.
//
// Reductions are two-stage with a fixed summation order (per-block partial
// sums, then one pass over the partials), so results are bitwise
// reproducible from run to run.
#include "givens.h"

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

__global__ void __launch_bounds__(EB) k_weight_rhs(FineOp op, const cplx* __restrict__ f,
                                                   cplx* __restrict__ b, int64_t bs, int64_t fs) {
    const int rb = blockIdx.y;
    f += rb * fs;
    b = rhs_nn(b, rb, bs);
    const int64_t p = (int64_t)blockIdx.x * EB + threadIdx.x;
    const int64_t n = (int64_t)op.nz * op.nx;
    if (p >= n) return;
    const int ix = (int)(p % op.nx);
    const int iz = (int)(p / op.nx);
    double w = (ix == 0 || ix == op.nx - 1) ? 0.5 : 1.0;
    if (op.ndim == 2 && (iz == 0 || iz == op.nz - 1)) w *= 0.5;
    b[p] = cscale(f[p], w);
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

// ---------------------------------------------------------------------------
// Fused Arnoldi kernels (device-side control: every kernel returns at once
// when st->active == 0, so the host may enqueue ahead of the decision).
// ---------------------------------------------------------------------------
constexpr int KC = 8;   // projections reduced per LDS pass

// Block reduction of KC complex values per thread (256 threads, linear tid):
// out[c] (valid in thread (c * 32)) = sum over threads, fixed order.
__device__ __forceinline__ void block_multi_sum(const cplx v[KC], cplx* lds, int tid,
                                                cplx* out_c, int* out_idx) {
    for (int c = 0; c < KC; ++c) lds[c * 256 + tid] = v[c];
    __syncthreads();
    const int g = tid >> 5, l = tid & 31;
    cplx acc = mk(0.0, 0.0);
    for (int r = 0; r < 8; ++r) acc = cadd(acc, lds[g * 256 + l + 32 * r]);
    for (int off = 16; off > 0; off >>= 1) {
        acc.x += __shfl_down(acc.x, off, 32);
        acc.y += __shfl_down(acc.y, off, 32);
    }
    *out_c = acc;
    *out_idx = (l == 0) ? g : -1;
    __syncthreads();
}

// partial[i*nb + blk] = sum over the block's nodes of conj(V_i[p]) w_p, i < k
__device__ __forceinline__ void block_dots(const cplx* V, int64_t n, int k, bool valid, int64_t p,
                                           cplx wp, cplx* partial, int nb, int blk, cplx* lds,
                                           int tid) {
    for (int c0 = 0; c0 < k; c0 += KC) {
        cplx v[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            const int i = c0 + c;
            v[c] = (valid && i < k) ? cmulc(V[(int64_t)i * n + p], wp) : mk(0.0, 0.0);
        }
        cplx sum;
        int idx;
        block_multi_sum(v, lds, tid, &sum, &idx);
        if (idx >= 0 && c0 + idx < k) partial[(int64_t)(c0 + idx) * nb + blk] = sum;
    }
}

__device__ __forceinline__ bool off(const int* active) { return active && *active == 0; }

// One recursive-halving step over lane bit 4H (H = 2, 1): each lane keeps
// the lower (bit clear) or upper half of its 2H values, sends the other half
// to the partner lane and adds what it receives.
template <int H>
__device__ __forceinline__ void halve(cplx (&v)[16], int lane) {
    const bool hi = (lane & (4 * H)) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const cplx keep = hi ? v[H + i] : v[i];
        const cplx send = hi ? v[i] : v[H + i];
        v[i] = cadd(keep, mk(__shfl_xor(send.x, 4 * H, 64), __shfl_xor(send.y, 4 * H, 64)));
    }
}

// The same step over lane bits 5 and 4 with the gfx950 lane swaps (no
// selects, no LDS crossbar): v_permlane32_swap exchanges the upper half of a
// with the lower half of b, so afterwards a + b holds a_l + a_{l+32} in lanes
// below 32 and b_{l-32} + b_l above; v_permlane16_swap does the same for the
// odd 16-lane rows of a and the even rows of b.
template <bool ROWS16>
__device__ __forceinline__ double swap_add(double a, double b) {
    const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    const unsigned alo = (unsigned)ua, ahi = (unsigned)(ua >> 32);
    const unsigned blo = (unsigned)ub, bhi = (unsigned)(ub >> 32);
    unsigned xlo, ylo, xhi, yhi;
    if (ROWS16) {
        const auto l = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
        xlo = l[0]; ylo = l[1]; xhi = h[0]; yhi = h[1];
    } else {
        const auto l = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
        xlo = l[0]; ylo = l[1]; xhi = h[0]; yhi = h[1];
    }
    return __longlong_as_double((long long)(((unsigned long long)xhi << 32) | xlo)) +
           __longlong_as_double((long long)(((unsigned long long)yhi << 32) | ylo));
}

// Sum over the 64 lanes of a wavefront of 16 complex values per lane:
// recursive halving over lane bits 5..2, then a butterfly over bits 1..0.
// Every lane returns the total of value (lane >> 2) & 15; the order of the
// additions is fixed.
__device__ __forceinline__ cplx wave_sum16(cplx (&v)[16], int lane) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
        v[i] = mk(swap_add<false>(v[i].x, v[8 + i].x), swap_add<false>(v[i].y, v[8 + i].y));
#pragma unroll
    for (int i = 0; i < 4; ++i)
        v[i] = mk(swap_add<true>(v[i].x, v[4 + i].x), swap_add<true>(v[i].y, v[4 + i].y));
    halve<2>(v, lane);
    halve<1>(v, lane);
    cplx a = v[0];
    a = cadd(a, mk(__shfl_xor(a.x, 1, 64), __shfl_xor(a.y, 1, 64)));
    a = cadd(a, mk(__shfl_xor(a.x, 2, 64), __shfl_xor(a.y, 2, 64)));
    return a;
}

// w = H z (fine operator) and the projections of the Arnoldi step with
// delayed reorthogonalisation: with u = V_{k-1} (the new, not yet
// reorthogonalised vector), partial[i] = block sums of conj(V_i) u and
// partial[k + i] = block sums of conj(V_i) w, i < k. A block of 256 threads
// takes AD_NPT runs of 256 consecutive nodes; each thread sums its nodes'
// products, then the sums are reduced over each wavefront (wave_sum16) and
// over the four wavefronts in LDS. For k <= KMAX the basis values of a node
// are loaded up front (all in flight together); beyond, in chunks of 8.
// Two nodes per thread halve the reductions where the launch is small enough
// for them to matter; on large launches one node per thread keeps two
// wavefronts per SIMD in flight (ad_npt, of the nodes over all right-hand
// sides: a batch of sources on a small grid is a large launch).
inline int ad_npt(int64_t nodes) { return nodes < 262144 ? 2 : 1; }

template <int NDIM, int KMAX, class ZC, int AD_NPT>
__global__ void __launch_bounds__(256) k_apply_dot(FineOp op, const ZC* __restrict__ z,
                                                   cplx* __restrict__ w,
                                                   const cplx* __restrict__ V, int k,
                                                   cplx* __restrict__ partial,
                                                   const int* __restrict__ active, int64_t bs) {
    const int rb = blockIdx.y;
    active = rhs_at(active, rb, bs);
    if (off(active)) return;
    z = rhs_nn(z, rb, bs);
    w = rhs_nn(w, rb, bs);
    V = rhs_nn(V, rb, bs);
    partial = rhs_nn(partial, rb, bs);
    constexpr int NS = (KMAX > 0 ? KMAX : 8) * 2;          // staged sums per wavefront
    __shared__ cplx wsum[4 * NS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = gridDim.x, blk = blockIdx.x;
    const int64_t n = (int64_t)op.nz * op.nx;
    int64_t pr[AD_NPT];
    bool ok[AD_NPT];
    cplx ur[AD_NPT], wr[AD_NPT];
    // w = H z on the block's nodes
#pragma unroll
    for (int r = 0; r < AD_NPT; ++r) {
        const int64_t p0 = ((int64_t)blk * AD_NPT + r) * 256 + tid;
        ok[r] = p0 < n;
        const int64_t p = ok[r] ? p0 : 0;
        pr[r] = p;
        ur[r] = ok[r] ? V[(int64_t)(k - 1) * n + p] : mk(0.0, 0.0);
        cplx wp = mk(0.0, 0.0);
        if (ok[r]) {
            const int iz = NDIM == 2 ? (int)(p / op.nx) : 0;
            const int ix = NDIM == 2 ? (int)(p - (int64_t)iz * op.nx) : (int)p;
            const Coef5 c = fine_coefs(op, iz, ix, op.m2[p]);
            const cplx zW = cconv<cplx>(z[ix > 0 ? p - 1 : p]);
            const cplx zE = cconv<cplx>(z[ix < op.nx - 1 ? p + 1 : p]);
            const cplx zp = cconv<cplx>(z[p]);
            const cplx sx = cadd(ix > 0 ? zW : mk(0.0, 0.0), ix < op.nx - 1 ? zE : mk(0.0, 0.0));
            wp = csub(cmul(c.diag, zp), cscale(sx, c.cx));
            if (NDIM == 2) {
                const cplx zN = cconv<cplx>(z[iz > 0 ? p - op.nx : p]);
                const cplx zS = cconv<cplx>(z[iz < op.nz - 1 ? p + op.nx : p]);
                const cplx sz = cadd(iz > 0 ? zN : mk(0.0, 0.0), iz < op.nz - 1 ? zS : mk(0.0, 0.0));
                wp = csub(wp, cscale(sz, c.cz));
            }
            w[p] = wp;
        }
        wr[r] = wp;
    }
    if (KMAX > 0) {
        cplx acc[2][KMAX > 0 ? KMAX : 1];
#pragma unroll
        for (int i = 0; i < KMAX; ++i) acc[0][i] = acc[1][i] = mk(0.0, 0.0);
#pragma unroll
        for (int r = 0; r < AD_NPT; ++r) {
            cplx v[KMAX > 0 ? KMAX : 1];
#pragma unroll
            for (int i = 0; i < KMAX; ++i)
                v[i] = (ok[r] && i < k) ? V[(int64_t)i * n + pr[r]] : mk(0.0, 0.0);
#pragma unroll
            for (int i = 0; i < KMAX; ++i) {
                acc[0][i] = cadd(acc[0][i], cmulc(v[i], ur[r]));
                acc[1][i] = cadd(acc[1][i], cmulc(v[i], wr[r]));
            }
        }
        // chunks of 8 basis vectors: values 0..7 against u, 8..15 against w
#pragma unroll
        for (int c0 = 0; c0 < KMAX; c0 += 8) {
            if (c0 >= k) break;
            cplx d[16];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                d[c] = acc[0][c0 + c];
                d[8 + c] = acc[1][c0 + c];
            }
            const cplx t = wave_sum16(d, lane);
            if ((lane & 3) == 0) wsum[wave * NS + c0 * 2 + (lane >> 2)] = t;
        }
        __syncthreads();
        for (int t = tid; t < 2 * k; t += 256) {
            const int set = t >= k, i = t - set * k;
            const int slot = (i & ~7) * 2 + set * 8 + (i & 7);
            cplx a = wsum[slot];
#pragma unroll
            for (int q = 1; q < 4; ++q) a = cadd(a, wsum[q * NS + slot]);
            partial[(int64_t)t * nb + blk] = a;
        }
    } else {
        for (int c0 = 0; c0 < k; c0 += 8) {
            cplx d[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) d[c] = mk(0.0, 0.0);
#pragma unroll
            for (int r = 0; r < AD_NPT; ++r) {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const cplx v = (ok[r] && c0 + c < k) ? V[(int64_t)(c0 + c) * n + pr[r]]
                                                         : mk(0.0, 0.0);
                    d[c] = cadd(d[c], cmulc(v, ur[r]));
                    d[8 + c] = cadd(d[8 + c], cmulc(v, wr[r]));
                }
            }
            const cplx t = wave_sum16(d, lane);
            if ((lane & 3) == 0) wsum[wave * NS + (lane >> 2)] = t;
            __syncthreads();
            if (tid < 16) {
                const int set = tid >= 8, i = c0 + (tid & 7);
                cplx a = wsum[tid];
#pragma unroll
                for (int q = 1; q < 4; ++q) a = cadd(a, wsum[q * NS + tid]);
                if (i < k) partial[(int64_t)(set * k + i) * nb + blk] = a;
            }
            __syncthreads();
        }
    }
}

// plain projections V^H w (for the stand-alone orthogonalisation entry point)
__global__ void __launch_bounds__(256) k_dot_blocks(const cplx* __restrict__ V, int64_t n, int k,
                                                    const cplx* __restrict__ w,
                                                    cplx* __restrict__ partial, int64_t bs) {
    __shared__ cplx lds[KC * 256];
    const int rb = blockIdx.y;
    V = rhs_nn(V, rb, bs);
    w = rhs_nn(w, rb, bs);
    partial = rhs_nn(partial, rb, bs);
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * 256 + tid;
    const bool valid = p < n;
    const cplx wp = valid ? w[p] : mk(0.0, 0.0);
    block_dots(V, n, k, valid, valid ? p : 0, wp, partial, gridDim.x, blockIdx.x, lds, tid);
}

// w -= V h with the basis loads issued KC at a time (independent loads in
// flight rather than one dependent round trip per vector)
__device__ __forceinline__ cplx axpy_chunked(const cplx* V, int64_t n, int k, const cplx* h,
                                             int64_t p, cplx wp) {
    for (int c0 = 0; c0 < k; c0 += KC) {
        cplx v[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) v[c] = (c0 + c < k) ? V[(int64_t)(c0 + c) * n + p] : mk(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < KC; ++c)
            if (c0 + c < k) wp = csub(wp, cmul(v[c], h[c0 + c]));
    }
    return wp;
}

// w -= V h, then the second projections V^H w. For k <= KMAX the basis
// values stay in registers between the update and the projections.
template <int KMAX>
__global__ void __launch_bounds__(256) k_axpy_dot(const cplx* __restrict__ V, int64_t n, int k,
                                                  const cplx* __restrict__ h,
                                                  cplx* __restrict__ w,
                                                  cplx* __restrict__ partial,
                                                  const int* __restrict__ active, int64_t bs) {
    const int rb = blockIdx.y;
    active = rhs_at(active, rb, bs);
    if (off(active)) return;
    V = rhs_nn(V, rb, bs);
    h = rhs_nn(h, rb, bs);
    w = rhs_nn(w, rb, bs);
    partial = rhs_nn(partial, rb, bs);
    __shared__ cplx lds[KC * 256];
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * 256 + tid;
    const bool valid = p < n;
    const int64_t pp = valid ? p : 0;
    const int nb = gridDim.x, blk = blockIdx.x;
    if (KMAX > 0 && k <= KMAX) {
        cplx v[KMAX > 0 ? KMAX : 1];
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
            v[i] = (valid && i < k) ? V[(int64_t)i * n + pp] : mk(0.0, 0.0);
        cplx wp = valid ? w[pp] : mk(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
            if (i < k) wp = csub(wp, cmul(v[i], h[i]));
        if (valid) w[pp] = wp;
#pragma unroll
        for (int c0 = 0; c0 < KMAX; c0 += KC) {
            if (c0 >= k) break;
            cplx d[KC];
#pragma unroll
            for (int c = 0; c < KC; ++c) d[c] = cmulc(v[c0 + c], wp);
            cplx sum;
            int idx;
            block_multi_sum(d, lds, tid, &sum, &idx);
            if (idx >= 0 && c0 + idx < k) partial[(int64_t)(c0 + idx) * nb + blk] = sum;
        }
    } else {
        cplx wp = mk(0.0, 0.0);
        if (valid) {
            wp = axpy_chunked(V, n, k, h, pp, w[pp]);
            w[pp] = wp;
        }
        block_dots(V, n, k, valid, pp, wp, partial, nb, blk, lds, tid);
    }
}

// Second pass of the Arnoldi step with delayed reorthogonalisation (one pass
// over the basis): from the reduced projections red = [V^H u, V^H w] (u =
// V_j, 2(j+1) values) every block derives (dcgs_coeffs) nu = ||u - V a||, the
// new Hessenberg entry h_jj = v_j^H w and c = b - a h_jj / nu, then
//   V_j     <- (u - sum_i a_i V_i) / nu          (the reorthogonalised v_j)
//   V_{j+1} <- (w - sum_i c_i V_i - (h_jj / nu) u) / nu
// (w projected once: the next u). The division by nu keeps the scale of the
// stored u (and of z = M^{-1} u) that of one Hessenberg column: without it
// the scales of consecutive steps multiply over a cycle and overflow complex64
// within a few tens of steps. The Hessenberg entries carried to the next
// column are divided by nu as well, and z_j enters the update as z_j / nu.
// With giv.st set, one extra workgroup performs the Givens step of column j-1
// (which needed this step's reorthogonalisation coefficients).
// LDS (dynamic): 3 (j + 2) complex + (j + 2) doubles.
template <int KMAX>
__global__ void __launch_bounds__(256) k_axpy_dcgs(cplx* __restrict__ V, int64_t n, int j,
                                                   const cplx* __restrict__ red,
                                                   const cplx* __restrict__ w,
                                                   const int* __restrict__ active, int64_t bs,
                                                   int nbn, GivensArgs giv) {
    extern __shared__ cplx dsm[];
    cplx* sa = dsm;
    cplx* sc = dsm + (j + 2);
    const int rb = blockIdx.y;
    if ((int)blockIdx.x == nbn) {                 // the hosted Givens step (column j - 1)
        givens_dcgs(giv, rb, false, sa, sc, dsm + 2 * (j + 2),
                    reinterpret_cast<double*>(dsm + 3 * (j + 2)));
        return;
    }
    // read atomically: the Givens workgroup of this launch may clear it
    active = rhs_at(active, rb, bs);
    if (active && __hip_atomic_load(const_cast<int*>(active), __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT) == 0)
        return;
    V = rhs_nn(V, rb, bs);
    red = rhs_nn(red, rb, bs);
    w = rhs_nn(w, rb, bs);
    const int tid = threadIdx.x;
    __shared__ double s_inv_nu, s_nu;
    __shared__ cplx s_d, s_h;
    // a_i, c_i and the scalars, identical in every block (fixed-order sums)
    dcgs_coeffs(red, j, sa, sc, &s_inv_nu, &s_d, &s_h, &s_nu);
    __syncthreads();
    const double inv_nu = s_inv_nu;
    const cplx dd = s_d;
    const int64_t p = (int64_t)blockIdx.x * 256 + tid;
    if (p >= n) return;
    const cplx up = V[(int64_t)j * n + p];
    const cplx wp = w[p];
    cplx acc_v = up, acc_u = csub(wp, cmul(dd, up));
    if (KMAX > 0 && j <= KMAX) {
        cplx v[KMAX > 0 ? KMAX : 1];
#pragma unroll
        for (int i = 0; i < KMAX; ++i) v[i] = i < j ? V[(int64_t)i * n + p] : mk(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (i < j) {
                acc_v = csub(acc_v, cmul(sa[i], v[i]));
                acc_u = csub(acc_u, cmul(sc[i], v[i]));
            }
        }
    } else {
        for (int c0 = 0; c0 < j; c0 += KC) {
            cplx v[KC];
#pragma unroll
            for (int c = 0; c < KC; ++c)
                v[c] = (c0 + c < j) ? V[(int64_t)(c0 + c) * n + p] : mk(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                if (c0 + c < j) {
                    acc_v = csub(acc_v, cmul(sa[c0 + c], v[c]));
                    acc_u = csub(acc_u, cmul(sc[c0 + c], v[c]));
                }
            }
        }
    }
    V[(int64_t)j * n + p] = cscale(acc_v, inv_nu);
    V[(int64_t)(j + 1) * n + p] = cscale(acc_u, inv_nu);
}

// w -= V h, then ||w||^2 per block. At most kNormBlocks blocks (grid-stride
// over the nodes): the partials are summed again by every consumer of the
// norm, so their number is kept small.
__global__ void __launch_bounds__(256) k_axpy_norm(const cplx* __restrict__ V, int64_t n, int k,
                                                   const cplx* __restrict__ h,
                                                   cplx* __restrict__ w,
                                                   cplx* __restrict__ partial,
                                                   const int* __restrict__ active, int64_t bs) {
    const int rb = blockIdx.y;
    active = rhs_at(active, rb, bs);
    if (off(active)) return;
    V = rhs_nn(V, rb, bs);
    h = rhs_nn(h, rb, bs);
    w = rhs_nn(w, rb, bs);
    partial = rhs_nn(partial, rb, bs);
    __shared__ cplx sh[4];
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * 256) {
        const cplx wp = axpy_chunked(V, n, k, h, p, w[p]);
        w[p] = wp;
        acc += cabs2(wp);
    }
    const cplx s = block_sum(mk(acc, 0.0), sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// predicated fixed-order reduction of partial sums (k blocks of 64 threads)
__global__ void __launch_bounds__(64) k_reduce_pred(const cplx* __restrict__ partial, int nb,
                                                    cplx* __restrict__ out,
                                                    const int* __restrict__ active, int64_t bs) {
    const int rb = blockIdx.y;
    active = rhs_at(active, rb, bs);
    if (off(active)) return;
    partial = rhs_nn(partial, rb, bs);
    out = rhs_nn(out, rb, bs);
    const int i = blockIdx.x;
    const cplx* pi = partial + (int64_t)i * nb;
    // eight loads in flight per lane (issued from a clamped index and masked,
    // so that no load waits behind a branch), summed in a fixed order
    cplx acc = mk(0.0, 0.0);
    for (int t0 = threadIdx.x; t0 < nb; t0 += 64 * 8) {
        cplx v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0 + 64 * u;
            v[u] = cscale(pi[t < nb ? t : 0], t < nb ? 1.0 : 0.0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = cadd(acc, v[u]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        acc.x += __shfl_down(acc.x, o, 64);
        acc.y += __shfl_down(acc.y, o, 64);
    }
    if (threadIdx.x == 0) out[i] = acc;
}

// r = b - H u (true residual) with ||r||^2 per block; predicated on !done
template <int NDIM>
__global__ void __launch_bounds__(256) k_residual_norm(FineOp op, const cplx* __restrict__ b,
                                                       const cplx* __restrict__ u,
                                                       cplx* __restrict__ r,
                                                       cplx* __restrict__ partial,
                                                       const int* __restrict__ done, int64_t bs,
                                                       int64_t fs) {
    const int rb = blockIdx.z;
    done = rhs_at(done, rb, bs);
    if (*done) return;
    b = rhs_nn(b, rb, bs);
    u += rb * fs;
    r = rhs_nn(r, rb, bs);
    partial = rhs_nn(partial, rb, bs);
    __shared__ cplx sh[4];
    int ix, iz;
    if (NDIM == 2) {
        ix = blockIdx.x * 64 + threadIdx.x;
        iz = blockIdx.y * 4 + threadIdx.y;
    } else {
        ix = blockIdx.x * 256 + threadIdx.x;
        iz = 0;
    }
    cplx acc = mk(0.0, 0.0);
    if (ix < op.nx && iz < op.nz) {
        const int64_t p = (int64_t)iz * op.nx + ix;
        const Coef5 c = fine_coefs(op, iz, ix, op.m2[p]);
        cplx sx = mk(0.0, 0.0);
        if (ix > 0) sx = cadd(sx, u[p - 1]);
        if (ix < op.nx - 1) sx = cadd(sx, u[p + 1]);
        cplx au = csub(cmul(c.diag, u[p]), cscale(sx, c.cx));
        if (NDIM == 2) {
            cplx sz = mk(0.0, 0.0);
            if (iz > 0) sz = cadd(sz, u[p - op.nx]);
            if (iz < op.nz - 1) sz = cadd(sz, u[p + op.nx]);
            au = csub(au, cscale(sz, c.cz));
        }
        const cplx rp = csub(b[p], au);
        r[p] = rp;
        acc = mk(cabs2(rp), 0.0);
    }
    // block of 256 threads (linear id)
    const int tid = NDIM == 2 ? threadIdx.y * 64 + threadIdx.x : threadIdx.x;
    for (int o = 32; o > 0; o >>= 1) acc.x += __shfl_down(acc.x, o, 64);
    if ((tid & 63) == 0) sh[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        const int blk = blockIdx.y * gridDim.x + blockIdx.x;
        partial[blk] = mk(sh[0].x + sh[1].x + sh[2].x + sh[3].x, 0.0);
    }
}

// fixed-order sum of nb real partials (x components) by one 256-thread block
__device__ __forceinline__ double block_sum_partials(const cplx* partial, int nb, double* sh) {
    double acc = 0.0;
    for (int t = threadIdx.x; t < nb; t += 256) acc += partial[t].x;
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Start of a restart cycle: beta = ||b - H u||; decide whether the solve is
// finished; otherwise reset the least-squares state and open the cycle. From
// a given initial guess (warm), the first cycle's relative residual is the
// history's first entry.
__global__ void __launch_bounds__(256) k_cycle_start(SolveState* st, const cplx* __restrict__ partial,
                                                     int nb, cplx* __restrict__ g,
                                                     HostRecord* rec, int64_t bs, double* hist,
                                                     int64_t hist_stride, int warm) {
    const int rb = blockIdx.x;
    st = rhs_nn(st, rb, bs);
    partial = rhs_nn(partial, rb, bs);
    g = rhs_nn(g, rb, bs);
    rec += rb;
    hist += (int64_t)rb * hist_stride;
    if (st->done) return;
    __shared__ double sh[4];
    const double beta = sqrt(block_sum_partials(partial, nb, sh));
    if (threadIdx.x != 0) return;
    const double rel = beta / st->beta0;
    st->rel = rel;
    if (warm && st->it == 0) hist[0] = rel;
    int done = 0, status = 0;
    if (!isfinite(rel)) { done = 1; status = -4; }
    else if (rel <= st->tol) { done = 1; status = 0; }
    else if (st->it >= st->max_iters) { done = 1; status = 1; }
    st->k = 0;
    st->j = 0;
    if (done) {
        st->done = 1;
        st->active = 0;
        st->status = status;
    } else {
        st->active = 1;
        g[0] = mk(beta, 0.0);
        for (int i = 1; i <= st->m; ++i) g[i] = mk(0.0, 0.0);
    }
    rec->rel = rel;
    rec->status = status;
    rec->it = st->it;
    rec->jstep = 0;
    __threadfence_system();
    rec->cycles += 1;
    rec->done = st->done;
    rec->seq += 1;
    __threadfence_system();
}

// Givens step that closes a full cycle (column m - 1), from the projections of
// the last vector u = V_m on the basis (red = [V_0..V_{m-1}^H u, u^H u]).
__global__ void __launch_bounds__(256) k_givens_tail(GivensArgs a) {
    __shared__ cplx sa[kMaxColumns + 2], scol[kMaxColumns + 2], sc[kMaxColumns + 2];
    __shared__ double scs[kMaxColumns + 2];
    givens_dcgs(a, blockIdx.x, true, sa, sc, scol, scs);
}

// y = R^{-1} g (k = st->k columns), then u += Z y; one block of 256 threads
// solves the triangle (column-oriented, g kept in LDS), the update is separate.
__global__ void __launch_bounds__(256) k_backsub_pred(const SolveState* st,
                                                      const cplx* __restrict__ R,
                                                      const cplx* __restrict__ g,
                                                      const double* __restrict__ zs,
                                                      cplx* __restrict__ y, int64_t bs) {
    const int rb = blockIdx.x;
    st = rhs_nn(st, rb, bs);
    R = rhs_nn(R, rb, bs);
    g = rhs_nn(g, rb, bs);
    zs = rhs_nn(zs, rb, bs);
    y = rhs_nn(y, rb, bs);
    const int k = st->k;
    if (k == 0) return;
    const int ld = st->m + 1;
    __shared__ cplx gs[1025];
    for (int i = threadIdx.x; i < k; i += 256) gs[i] = g[i];
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        const cplx yi = cdiv(gs[i], R[i + (int64_t)i * ld]);
        __syncthreads();
        for (int l = threadIdx.x; l < i; l += 256)
            gs[l] = csub(gs[l], cmul(R[l + (int64_t)i * ld], yi));
        if (threadIdx.x == 0) y[i] = cscale(yi, zs[i]);
        __syncthreads();
    }
}

// The same for k <= 32 columns by one wavefront: lane l holds g_l and the
// entries R[l, i] of every column (loaded up front, off the recurrence) and
// forms 1 / R[l, l] before it starts; column i then costs two broadcasts and
// one multiply-add per lane, with no barrier.
constexpr int BS_MAX = 32;

__device__ __forceinline__ cplx bcast(cplx v, int src) {
    return mk(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

__global__ void __launch_bounds__(64) k_backsub_wave(const SolveState* st,
                                                     const cplx* __restrict__ R,
                                                     const cplx* __restrict__ g,
                                                     const double* __restrict__ zs,
                                                     cplx* __restrict__ y, int64_t bs) {
    const int rb = blockIdx.x;
    st = rhs_nn(st, rb, bs);
    R = rhs_nn(R, rb, bs);
    g = rhs_nn(g, rb, bs);
    zs = rhs_nn(zs, rb, bs);
    y = rhs_nn(y, rb, bs);
    const int k = st->k;
    if (k == 0) return;
    const int ld = st->m + 1;
    const int lane = threadIdx.x;
    const bool mine = lane < k;
    const int lc = mine ? lane : 0;
    cplx r[BS_MAX];
#pragma unroll
    for (int i = 0; i < BS_MAX; ++i) {
        const bool ok = i < k && lane < i;
        r[i] = cscale(R[ok ? lane + (int64_t)i * ld : 0], ok ? 1.0 : 0.0);
    }
    cplx gl = cscale(g[lc], mine ? 1.0 : 0.0);
    const cplx dl = R[lc + (int64_t)lc * ld];
    const cplx rinv = cdiv(mk(1.0, 0.0), dl);
    const double zl = zs[lc];
#pragma unroll
    for (int i = BS_MAX - 1; i >= 0; --i) {
        if (i < k) {
            const cplx yi = cmul(bcast(gl, i), bcast(rinv, i));
            gl = csub(gl, cmul(r[i], yi));
            if (lane == i) y[i] = cscale(yi, zl);
        }
    }
}

template <class ZC>
__global__ void __launch_bounds__(256) k_update_pred(const SolveState* st,
                                                     const ZC* __restrict__ Z, int64_t n,
                                                     const cplx* __restrict__ y,
                                                     cplx* __restrict__ x, int64_t bs,
                                                     int64_t fs) {
    const int rb = blockIdx.y;
    st = rhs_nn(st, rb, bs);
    Z = rhs_nn(Z, rb, bs);
    y = rhs_nn(y, rb, bs);
    x += rb * fs;
    const int k = st->k;
    if (k == 0) return;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    cplx acc = x[p];
    for (int c0 = 0; c0 < k; c0 += KC) {
        cplx v[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c)
            v[c] = (c0 + c < k) ? cconv<cplx>(Z[(int64_t)(c0 + c) * n + p]) : mk(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < KC; ++c)
            if (c0 + c < k) acc = cadd(acc, cmul(v[c], y[c0 + c]));
    }
    x[p] = acc;
}

// after the update of a cycle: mark k = 0 so a repeated end-of-cycle is a no-op
__global__ void k_cycle_end(SolveState* st, int64_t bs) {
    if (threadIdx.x == 0) rhs_at(st, (int)blockIdx.x, bs)->k = 0;
}

// solve prologue: beta0 = ||b|| from partials; sets done when b == 0 or not
// finite. b == 0 has the solution u = 0, also from a given initial guess
// (u_warm: the guess, zeroed here in that case; null when u starts at 0).
__global__ void __launch_bounds__(256) k_solve_init(SolveState* st, const cplx* __restrict__ partial,
                                                    int nb, int m, int max_iters, double tol,
                                                    HostRecord* rec, double* hist, int64_t bs,
                                                    int64_t hist_stride, cplx* u_warm, int64_t n,
                                                    int64_t fs) {
    const int rb = blockIdx.x;
    st = rhs_nn(st, rb, bs);
    partial = rhs_nn(partial, rb, bs);
    rec += rb;
    hist += (int64_t)rb * hist_stride;
    __shared__ double sh[4];
    const double b2 = block_sum_partials(partial, nb, sh);
    if (u_warm && b2 == 0.0) {
        cplx* u = u_warm + (int64_t)rb * fs;
        for (int64_t p = threadIdx.x; p < n; p += 256) u[p] = mk(0.0, 0.0);
    }
    if (threadIdx.x != 0) return;
    const double beta0 = sqrt(b2);
    st->beta0 = beta0;
    st->m = m;
    st->max_iters = max_iters;
    st->tol = tol;
    st->it = 0;
    st->j = 0;
    st->k = 0;
    st->active = 0;
    st->rel = 0.0;
    st->done = 0;
    st->status = 0;
    if (!isfinite(beta0)) { st->done = 1; st->status = -4; st->rel = beta0; }
    else if (beta0 == 0.0) { st->done = 1; st->status = 0; }
    hist[0] = 1.0;
    rec->it = 0;
    rec->est = 1.0;
    rec->rel = st->rel;
    rec->status = st->status;
    rec->cycles = 0;
    rec->jstep = 0;
    rec->stops = 0;
    __threadfence_system();
    rec->done = st->done;
    rec->seq = 1;
    __threadfence_system();
}

inline unsigned eblocks(int64_t n) { return (unsigned)((n + EB - 1) / EB); }

}  // namespace

hipError_t launch_weight_rhs(const FineOp& op, const cplx* f, cplx* b, hipStream_t s,
                             const Batch& bt) {
    const int64_t n = (int64_t)op.nz * op.nx;
    HH_LAUNCH(k_weight_rhs, dim3(eblocks(n), bt.n), dim3(EB), 0, s, op, f, b, bt.bs, bt.fs);
    return hipGetLastError();
}

hipError_t launch_check_slowness(const double* m, int64_t n, double* m2, int* flag,
                                 double* mmax_partial, int nb, hipStream_t s) {
    HH_LAUNCH(k_check_slowness, dim3(nb), dim3(RB), 0, s, m, n, m2, flag, mmax_partial,
                       nb);
    return hipGetLastError();
}

template <int NDIM, class ZC, int NPT>
static void apply_dot_dispatch(dim3 g, dim3 b, const FineOp& op, const ZC* z, cplx* w,
                               const cplx* V, int k, cplx* partial, const int* active,
                               int64_t bs, hipStream_t s) {
    if (k <= 8)
        HH_LAUNCH((k_apply_dot<NDIM, 8, ZC, NPT>), g, b, 0, s, op, z, w, V, k, partial, active, bs);
    else if (k <= 16)
        HH_LAUNCH((k_apply_dot<NDIM, 16, ZC, NPT>), g, b, 0, s, op, z, w, V, k, partial, active,
                  bs);
    else if (k <= 32)
        HH_LAUNCH((k_apply_dot<NDIM, 32, ZC, NPT>), g, b, 0, s, op, z, w, V, k, partial, active,
                  bs);
    else if (k <= 48)
        HH_LAUNCH((k_apply_dot<NDIM, 48, ZC, NPT>), g, b, 0, s, op, z, w, V, k, partial, active,
                  bs);
    else
        HH_LAUNCH((k_apply_dot<NDIM, 0, ZC, NPT>), g, b, 0, s, op, z, w, V, k, partial, active, bs);
}

template <class ZC>
hipError_t apply_dot(const FineOp& op, const ZC* z, cplx* w, const cplx* V, int k, cplx* partial,
                     const int* active, hipStream_t s, const Batch& bt) {
    const dim3 g(apply_blocks(op, bt.n), bt.n), b(256);
    const bool two = ad_npt((int64_t)op.nz * op.nx * bt.n) == 2;
    if (op.ndim == 2 && two)
        apply_dot_dispatch<2, ZC, 2>(g, b, op, z, w, V, k, partial, active, bt.bs, s);
    else if (op.ndim == 2)
        apply_dot_dispatch<2, ZC, 1>(g, b, op, z, w, V, k, partial, active, bt.bs, s);
    else
        apply_dot_dispatch<1, ZC, 2>(g, b, op, z, w, V, k, partial, active, bt.bs, s);
    return hipGetLastError();
}

hipError_t launch_apply_dot(const FineOp& op, const cplx* z, cplx* w, const cplx* V, int k,
                            cplx* partial, const int* active, hipStream_t s, const Batch& bt) {
    return apply_dot(op, z, w, V, k, partial, active, s, bt);
}
hipError_t launch_apply_dot(const FineOp& op, const cplxf* z, cplx* w, const cplx* V, int k,
                            cplx* partial, const int* active, hipStream_t s, const Batch& bt) {
    return apply_dot(op, z, w, V, k, partial, active, s, bt);
}

int residual_blocks(const FineOp& op) {
    return op.ndim == 2 ? ((op.nx + 63) / 64) * ((op.nz + 3) / 4) : (op.nx + 255) / 256;
}
int apply_blocks(const FineOp& op, int nrhs) {
    const int64_t n = (int64_t)op.nz * op.nx;
    const int npt = ad_npt(n * nrhs);
    return (int)((n + 256 * npt - 1) / (256 * npt));
}
int node_blocks(int64_t n) { return (int)((n + 255) / 256); }
int norm_blocks(int64_t n) { return node_blocks(n) < kNormBlocks ? node_blocks(n) : kNormBlocks; }
hipError_t launch_dot_blocks(const cplx* V, int64_t n, int k, const cplx* w, cplx* partial,
                             hipStream_t s, const Batch& bt) {
    HH_LAUNCH(k_dot_blocks, dim3(node_blocks(n), bt.n), dim3(256), 0, s, V, n, k, w, partial,
              bt.bs);
    return hipGetLastError();
}
hipError_t launch_axpy_dot(const cplx* V, int64_t n, int k, const cplx* h, cplx* w, cplx* partial,
                           const int* active, hipStream_t s, const Batch& bt) {
    const dim3 g(node_blocks(n), bt.n), b(256);
    const int64_t bs = bt.bs;
    if (k <= 8)
        HH_LAUNCH(k_axpy_dot<8>, g, b, 0, s, V, n, k, h, w, partial, active, bs);
    else if (k <= 16)
        HH_LAUNCH(k_axpy_dot<16>, g, b, 0, s, V, n, k, h, w, partial, active, bs);
    else if (k <= 32)
        HH_LAUNCH(k_axpy_dot<32>, g, b, 0, s, V, n, k, h, w, partial, active, bs);
    else if (k <= 48)
        HH_LAUNCH(k_axpy_dot<48>, g, b, 0, s, V, n, k, h, w, partial, active, bs);
    else
        HH_LAUNCH(k_axpy_dot<0>, g, b, 0, s, V, n, k, h, w, partial, active, bs);
    return hipGetLastError();
}
hipError_t launch_axpy_norm(const cplx* V, int64_t n, int k, const cplx* h, cplx* w, cplx* partial,
                            const int* active, hipStream_t s, const Batch& bt) {
    HH_LAUNCH(k_axpy_norm, dim3(norm_blocks(n), bt.n), dim3(256), 0, s, V, n, k, h, w, partial,
              active, bt.bs);
    return hipGetLastError();
}
hipError_t launch_reduce_pred(const cplx* partial, int nb, int k, cplx* out, const int* active,
                              hipStream_t s, const Batch& bt) {
    HH_LAUNCH(k_reduce_pred, dim3(k, bt.n), dim3(64), 0, s, partial, nb, out, active, bt.bs);
    return hipGetLastError();
}
hipError_t launch_residual_norm(const FineOp& op, const cplx* b, const cplx* u, cplx* r,
                                cplx* partial, const int* done, hipStream_t s, const Batch& bt) {
    if (op.ndim == 2)
        HH_LAUNCH(k_residual_norm<2>, dim3((op.nx + 63) / 64, (op.nz + 3) / 4, bt.n),
                  dim3(64, 4), 0, s, op, b, u, r, partial, done, bt.bs, bt.fs);
    else
        HH_LAUNCH(k_residual_norm<1>, dim3((op.nx + 255) / 256, 1, bt.n), dim3(256), 0, s, op,
                  b, u, r, partial, done, bt.bs, bt.fs);
    return hipGetLastError();
}
hipError_t launch_cycle_start(SolveState* st, const cplx* partial, int nb, cplx* g,
                              HostRecord* rec, double* hist, int64_t hist_stride, bool warm,
                              hipStream_t s, const Batch& bt) {
    HH_LAUNCH(k_cycle_start, dim3(bt.n), dim3(256), 0, s, st, partial, nb, g, rec, bt.bs, hist,
              hist_stride, warm ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_givens_tail(const GivensArgs& a, hipStream_t s, const Batch& bt) {
    HH_LAUNCH(k_givens_tail, dim3(bt.n), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_axpy_dcgs(cplx* V, int64_t n, int j, const cplx* red, const cplx* w,
                            const int* active, const GivensArgs* giv, hipStream_t s,
                            const Batch& bt) {
    const int nbn = node_blocks(n);
    const GivensArgs none{};
    const GivensArgs& g = giv ? *giv : none;
    const dim3 grid(nbn + (giv ? 1 : 0), bt.n), b(256);
    const size_t shm = 3 * (size_t)(j + 2) * sizeof(cplx) + (size_t)(j + 2) * sizeof(double);
    if (j <= 8)
        HH_LAUNCH(k_axpy_dcgs<8>, grid, b, shm, s, V, n, j, red, w, active, bt.bs, nbn, g);
    else if (j <= 16)
        HH_LAUNCH(k_axpy_dcgs<16>, grid, b, shm, s, V, n, j, red, w, active, bt.bs, nbn, g);
    else if (j <= 32)
        HH_LAUNCH(k_axpy_dcgs<32>, grid, b, shm, s, V, n, j, red, w, active, bt.bs, nbn, g);
    else if (j <= 48)
        HH_LAUNCH(k_axpy_dcgs<48>, grid, b, shm, s, V, n, j, red, w, active, bt.bs, nbn, g);
    else
        HH_LAUNCH(k_axpy_dcgs<0>, grid, b, shm, s, V, n, j, red, w, active, bt.bs, nbn, g);
    return hipGetLastError();
}
template <class ZC>
hipError_t cycle_finish(SolveState* st, int m, const cplx* R, const cplx* g, const double* zs,
                        cplx* y, const ZC* Z, int64_t n, cplx* x, hipStream_t s,
                        const Batch& bt) {
    // k <= restart: one wavefront when the restart length allows it
    if (m <= BS_MAX)
        HH_LAUNCH(k_backsub_wave, dim3(bt.n), dim3(64), 0, s, st, R, g, zs, y, bt.bs);
    else
        HH_LAUNCH(k_backsub_pred, dim3(bt.n), dim3(256), 0, s, st, R, g, zs, y, bt.bs);
    HH_LAUNCH(k_update_pred<ZC>, dim3(node_blocks(n), bt.n), dim3(256), 0, s, st, Z, n, y, x,
              bt.bs, bt.fs);
    HH_LAUNCH(k_cycle_end, dim3(bt.n), dim3(64), 0, s, st, bt.bs);
    return hipGetLastError();
}
hipError_t launch_cycle_finish(SolveState* st, int m, const cplx* R, const cplx* g,
                               const double* zs, cplx* y, const cplx* Z, int64_t n, cplx* x,
                               hipStream_t s, const Batch& bt) {
    return cycle_finish(st, m, R, g, zs, y, Z, n, x, s, bt);
}
hipError_t launch_cycle_finish(SolveState* st, int m, const cplx* R, const cplx* g,
                               const double* zs, cplx* y, const cplxf* Z, int64_t n, cplx* x,
                               hipStream_t s, const Batch& bt) {
    return cycle_finish(st, m, R, g, zs, y, Z, n, x, s, bt);
}
hipError_t launch_solve_init(SolveState* st, const cplx* partial, int nb, int m, int max_iters,
                             double tol, HostRecord* rec, double* hist, int64_t hist_stride,
                             cplx* u_warm, int64_t n, hipStream_t s, const Batch& bt) {
    HH_LAUNCH(k_solve_init, dim3(bt.n), dim3(256), 0, s, st, partial, nb, m, max_iters, tol,
              rec, hist, bt.bs, hist_stride, u_warm, n, bt.fs);
    return hipGetLastError();
}

namespace {
__global__ void __launch_bounds__(256) k_to_f32(const double* __restrict__ a, float* __restrict__ b,
                                                int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < n) b[p] = (float)a[p];
}
__global__ void __launch_bounds__(256) k_to_c64(const cplx* __restrict__ a, cplxf* __restrict__ b,
                                                int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < n) b[p] = cconv<cplxf>(a[p]);
}
}  // namespace

hipError_t launch_to_f32(const double* a, float* b, int64_t n, hipStream_t s) {
    HH_LAUNCH(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}
hipError_t launch_to_c64(const cplx* a, cplxf* b, int64_t n, hipStream_t s) {
    HH_LAUNCH(k_to_c64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}
}  // namespace hh
