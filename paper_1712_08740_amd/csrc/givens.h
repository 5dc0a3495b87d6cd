// Device-side pieces of the Arnoldi step with delayed reorthogonalisation and
// of the Givens least-squares update, shared by the kernel that hosts the
// Givens step as one extra workgroup and the stand-alone kernel that closes a
// cycle.
#pragma once

#include "hh_internal.h"

namespace hh {

struct GivensArgs {
    SolveState* st;           // nullptr: no Givens step in this launch
    const cplx* red;          // reduced projections of this step: [V^H u, V^H w]
    cplx* hprev;              // previous step's projections of w and h_jj
    cplx* R;                  // (m + 1) x m triangular factor, column-major
    double* cs;               // rotations
    cplx* sn;
    cplx* g;                  // rotated right-hand side
    HostRecord* rec;          // progress records in pinned host memory (one per right-hand side)
    double* hist;             // residual estimates, pinned host memory
    int64_t bs;               // bytes between the workspaces of consecutive right-hand sides
    int64_t hist_stride;      // entries between the histories of consecutive right-hand sides
    double* zs;               // 1 / nu_j: the update coefficient of z_j is y_j / nu_j
};

// Sum over i < n of f(i) by the 64 lanes of wavefront 0 in a fixed order
// (lane-strided partial sums, then an xor butterfly: every lane of wave 0
// ends with the same bits).
template <class F>
__device__ __forceinline__ cplx wave_csum(int n, int lane, F f) {
    cplx acc = mk(0.0, 0.0);
    for (int i = lane; i < n; i += 64) acc = cadd(acc, f(i));
    for (int o = 32; o > 0; o >>= 1) {
        acc.x += __shfl_xor(acc.x, o, 64);
        acc.y += __shfl_xor(acc.y, o, 64);
    }
    return acc;
}

// Coefficients of the Arnoldi step with delayed reorthogonalisation, from the
// reduced projections red = [a_0..a_{j-1}, alpha, b_0..b_{j-1}, gamma] of
// u = V_j (a = V^H u, alpha = u^H u, b = V^H w, gamma = u^H w over the
// previous basis V_0..V_{j-1}; w = A z_j):
//   nu   = ||u - V a|| = sqrt(alpha - |a|^2)        (Pythagoras)
//   h_jj = v_j^H w = (gamma - a^H b) / nu
//   c    = b - a h_jj / nu,  d = h_jj / nu
// Every block computes them in the same fixed order. sa[i] = a_i,
// sc[i] = c_i; *inv_nu = 1/nu (0 when nu = 0), *d, *h = h_jj (thread 0).
__device__ inline void dcgs_coeffs(const cplx* red, int j, cplx* sa, cplx* sc, double* inv_nu,
                                   cplx* d, cplx* h, double* nu_out) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nt = blockDim.x * blockDim.y;
    for (int i = tid; i < j; i += nt) sa[i] = red[i];
    __syncthreads();
    if (tid < 64) {
        const cplx saa = wave_csum(j, tid, [&](int i) { return mk(cabs2(sa[i]), 0.0); });
        const cplx sab = wave_csum(j, tid, [&](int i) { return cmulc(sa[i], red[j + 1 + i]); });
        if (tid == 0) {
            const double nu2 = red[j].x - saa.x;
            const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
            const double inu = nu > 0.0 ? 1.0 / nu : 0.0;
            const cplx hh = cscale(csub(red[2 * j + 1], sab), inu);
            *inv_nu = inu;
            *h = hh;
            *d = cscale(hh, inu);
            *nu_out = nu;
        }
    }
    __syncthreads();
    const cplx dd = *d;
    for (int i = tid; i < j; i += nt) sc[i] = csub(red[j + 1 + i], cmul(sa[i], dd));
}

// Givens step of the delayed-reorthogonalisation Arnoldi process (the
// least-squares part of GMRES, Eq. 7's outer solver), run at step j by every
// thread of one workgroup for right-hand side rb. Column j-1 of the Hessenberg
// matrix becomes known here: entries i <= j-1 are the previous step's
// projections (hprev) plus this step's reorthogonalisation coefficients a_i,
// and the subdiagonal is nu. The previous rotations are applied, a new one
// zeroes the subdiagonal, and g, the residual estimate |g_j| / beta0 and the
// stop decision follow (estimate at tol, budget spent, breakdown, non-finite).
// At j = 0 there is no column yet: g_0 = nu (the cycle's initial residual).
// With tail set (after the last step of a cycle, red holding only
// [V^H u, u^H u]) column j-1 is the last of the cycle and the cycle stops.
// LDS: sa, sc of j+2 complex each, scol of j+2 complex, scs of j+2 doubles.
__device__ inline void givens_dcgs(const GivensArgs& ga, int rb, bool tail, cplx* sa, cplx* sc,
                                   cplx* scol, double* scs) {
    GivensArgs a = ga;                 // this right-hand side's state
    a.st = rhs_nn(ga.st, rb, ga.bs);
    a.red = rhs_nn(ga.red, rb, ga.bs);
    a.hprev = rhs_nn(ga.hprev, rb, ga.bs);
    a.R = rhs_nn(ga.R, rb, ga.bs);
    a.cs = rhs_nn(ga.cs, rb, ga.bs);
    a.sn = rhs_nn(ga.sn, rb, ga.bs);
    a.g = rhs_nn(ga.g, rb, ga.bs);
    a.zs = rhs_nn(ga.zs, rb, ga.bs);
    a.rec = ga.rec + rb;
    a.hist = ga.hist + (int64_t)rb * ga.hist_stride;
    SolveState* st = a.st;
    if (__hip_atomic_load(&st->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nt = blockDim.x * blockDim.y;
    const int j = st->j;
    __shared__ double s_inv_nu, s_nu;
    __shared__ cplx s_d, s_h;
    if (tail) {
        // red = [a_0..a_{j-1}, alpha] only
        for (int i = tid; i < j; i += nt) sa[i] = a.red[i];
        __syncthreads();
        if (tid < 64) {
            const cplx saa = wave_csum(j, tid, [&](int i) { return mk(cabs2(sa[i]), 0.0); });
            if (tid == 0) {
                const double nu2 = a.red[j].x - saa.x;
                s_nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
            }
        }
        __syncthreads();
    } else {
        dcgs_coeffs(a.red, j, sa, sc, &s_inv_nu, &s_d, &s_h, &s_nu);
    }
    // stage column j-1 and the previous rotations
    for (int i = tid; i < j; i += nt) scol[i] = cadd(a.hprev[i], sa[i]);
    for (int i = tid; i + 1 < j; i += nt) scs[i] = a.cs[i];
    // (sc is free once its c_i are no longer needed: the sines go there)
    __syncthreads();
    cplx* ssn = sc;
    if (!tail) {
        // keep this step's w-projections and h_jj for the next column, divided
        // by nu (u_{j+1} is stored divided by nu: see k_axpy_dcgs)
        for (int i = tid; i < j; i += nt) a.hprev[i] = cscale(a.red[j + 1 + i], s_inv_nu);
    }
    __syncthreads();
    for (int i = tid; i + 1 < j; i += nt) ssn[i] = a.sn[i];
    __syncthreads();
    if (tid != 0) return;
    const double hn = s_nu;
    if (!tail) {
        a.hprev[j] = cscale(s_h, s_inv_nu);
        a.zs[j] = s_inv_nu;
    }
    if (j == 0) {                      // first step of the cycle: no column yet
        a.g[0] = mk(hn, 0.0);
        st->j = 1;
        st->k = 0;
        HostRecord* rec = a.rec;
        rec->jstep = 1;
        rec->seq += 1;
        return;
    }
    const int col = j - 1;             // the column completed at this step
    const int ld = st->m + 1;
    scol[j] = mk(hn, 0.0);
    // previous rotations; the entry carried from one rotation to the next stays
    // in registers, so only the carry is a dependent chain (the other operands
    // are loaded ahead)
    cplx carry = scol[0];
    for (int i = 0; i < col; ++i) {
        const cplx q = scol[i + 1];
        const double c = scs[i];
        const cplx sn = ssn[i];
        scol[i] = cadd(cscale(carry, c), cmul(sn, q));
        carry = csub(cscale(q, c), cmulc(sn, carry));
    }
    const cplx av = carry;
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
    a.cs[col] = c;
    a.sn[col] = s;
    scol[col] = cadd(cscale(av, c), cscale(s, hn));
    scol[col + 1] = mk(0.0, 0.0);
    cplx* Rcol = a.R + (int64_t)col * ld;
    for (int i = 0; i <= col + 1; ++i) Rcol[i] = scol[i];
    const cplx gj = a.g[col];
    a.g[col + 1] = csub(mk(0.0, 0.0), cmulc(s, gj));
    a.g[col] = cscale(gj, c);
    const double est = sqrt(cabs2(a.g[col + 1])) / st->beta0;
    const int it = st->it + 1;
    const int bad = !(isfinite(est) && isfinite(hn));
    const int stop = tail || bad || hn == 0.0 || est <= st->tol || it >= st->max_iters;
    st->it = it;
    st->j = j + 1;
    st->k = col + 1;
    if (stop) __hip_atomic_store(&st->active, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (bad) {
        st->done = 1;
        st->status = -4;
    }
    HostRecord* rec = a.rec;
    a.hist[it] = est;
    rec->it = it;
    rec->est = est;
    rec->jstep = tail ? j : j + 1;
    rec->status = st->status;
    if (stop) {
        // the host reads the fields above once it sees the cycle stopped: make
        // them visible first (a step that goes on needs no ordering)
        __threadfence_system();
        rec->stops += 1;
        rec->done = st->done;
    }
    rec->seq += 1;
}

}  // namespace hh
