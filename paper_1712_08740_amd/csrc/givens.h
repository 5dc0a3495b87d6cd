// Device-side pieces of the Givens least-squares update shared by the
// stand-alone Givens kernel and the V-cycle kernel that hosts the step as one
// extra workgroup (so the update overlaps the next step's first leg instead
// of taking a launch of its own).
#pragma once

#include "hh_internal.h"

namespace hh {

// Sum of partial[t].x for t < nb, computed by the 64 lanes of one wavefront in
// a fixed order (lane-strided sums, then an xor butterfly, so every lane ends
// with the same bits). Callers that must agree on a norm (the Givens step and
// the kernel that normalises the next basis vector) both use this.
__device__ __forceinline__ double wave_sum_re(const cplx* __restrict__ partial, int nb, int lane) {
    double acc = 0.0;
    for (int t = lane; t < nb; t += 64) acc += partial[t].x;
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    return acc;
}

// 1 / ||w|| from the sum of squares, 0 for a zero vector (breakdown)
__device__ __forceinline__ double inv_norm(double sumsq) {
    return sumsq > 0.0 ? 1.0 / sqrt(sumsq) : 0.0;
}

struct GivensArgs {
    SolveState* st;           // nullptr: no Givens step in this launch
    const cplx* h1;           // first projections of the column
    const cplx* h2;           // second projections
    const cplx* partial;      // per-block sums of |w|^2 (first nb entries, .x)
    int nb;
    cplx* R;                  // (m + 1) x m triangular factor, column-major
    double* cs;               // rotations
    cplx* sn;
    cplx* g;                  // rotated right-hand side
    HostRecord* rec;          // progress records in pinned host memory (one per right-hand side)
    double* hist;             // residual estimates, pinned host memory
    int64_t bs;               // bytes between the workspaces of consecutive right-hand sides
    int64_t hist_stride;      // entries between the histories of consecutive right-hand sides
};

// Capacity (in columns) of LDS staging a caller provides: scol holds
// cap + 2 complex values, scs and ssn cap values each.
//
// Givens step on column j of the Hessenberg matrix (the least-squares part of
// GMRES, Eq. 7's outer solver): column = h1 + h2 with h_{j+1,j} = ||w||, the
// previous rotations applied, a new rotation that zeroes h_{j+1,j}, the rotated
// right-hand side, the residual estimate |g_{j+1}| / beta0 and the decision to
// stop the cycle. Called by every thread of one workgroup (blockDim >= 64)
// for right-hand side rb.
__device__ inline void givens_body(const GivensArgs& ga, int rb, cplx* scol, double* scs,
                                   cplx* ssn) {
    GivensArgs a = ga;                 // this right-hand side's state
    a.st = rhs_nn(ga.st, rb, ga.bs);
    a.h1 = rhs_nn(ga.h1, rb, ga.bs);
    a.h2 = rhs_nn(ga.h2, rb, ga.bs);
    a.partial = rhs_nn(ga.partial, rb, ga.bs);
    a.R = rhs_nn(ga.R, rb, ga.bs);
    a.cs = rhs_nn(ga.cs, rb, ga.bs);
    a.sn = rhs_nn(ga.sn, rb, ga.bs);
    a.g = rhs_nn(ga.g, rb, ga.bs);
    a.rec = ga.rec + rb;
    a.hist = ga.hist + (int64_t)rb * ga.hist_stride;
    SolveState* st = a.st;
    if (__hip_atomic_load(&st->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nt = blockDim.x * blockDim.y;
    const int j = st->j;
    double hn2 = 0.0;
    if (tid < 64) hn2 = wave_sum_re(a.partial, a.nb, tid);
    for (int i = tid; i <= j; i += nt) scol[i] = cadd(a.h1[i], a.h2[i]);
    for (int i = tid; i < j; i += nt) {
        scs[i] = a.cs[i];
        ssn[i] = a.sn[i];
    }
    __syncthreads();
    if (tid != 0) return;
    const int ld = st->m + 1;
    cplx* col = scol;
    const double hn = sqrt(hn2);
    col[j + 1] = mk(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        const cplx p = col[i], q = col[i + 1];
        col[i] = cadd(cscale(p, scs[i]), cmul(ssn[i], q));
        col[i + 1] = csub(cscale(q, scs[i]), cmulc(ssn[i], p));
    }
    const cplx av = col[j];
    double c;
    cplx s;
    if (hn == 0.0) {
        c = 1.0;
        s = mk(0.0, 0.0);
    } else if (av.x == 0.0 && av.y == 0.0) {
        c = 0.0;
        s = mk(1.0, 0.0);
    } else {
        const double aa = sqrt(cabs2(av));
        const double t = sqrt(aa * aa + hn * hn);
        c = aa / t;
        s = cscale(mk(av.x / aa, av.y / aa), hn / t);
    }
    a.cs[j] = c;
    a.sn[j] = s;
    col[j] = cadd(cscale(av, c), cscale(s, hn));
    col[j + 1] = mk(0.0, 0.0);
    cplx* Rcol = a.R + (int64_t)j * ld;
    for (int i = 0; i <= j + 1; ++i) Rcol[i] = col[i];
    const cplx gj = a.g[j];
    a.g[j + 1] = csub(mk(0.0, 0.0), cmulc(s, gj));
    a.g[j] = cscale(gj, c);
    const double est = sqrt(cabs2(a.g[j + 1])) / st->beta0;
    const int it = st->it + 1;
    const int bad = !(isfinite(est) && isfinite(hn));
    const int stop = bad || hn == 0.0 || est <= st->tol || it >= st->max_iters || j + 1 >= st->m;
    st->it = it;
    st->j = j + 1;
    st->k = j + 1;
    st->scale = inv_norm(hn2);
    if (stop) __hip_atomic_store(&st->active, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (bad) {
        st->done = 1;
        st->status = -4;
    }
    HostRecord* rec = a.rec;
    a.hist[it] = est;
    rec->it = it;
    rec->est = est;
    rec->jstep = j + 1;
    rec->status = st->status;
    __threadfence_system();          // the fields above are visible before the flags
    if (stop) rec->stops += 1;
    rec->done = st->done;
    rec->seq += 1;
}

}  // namespace hh
