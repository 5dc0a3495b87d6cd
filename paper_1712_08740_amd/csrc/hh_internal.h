// Internal declarations shared by the library's HIP sources: complex helpers,
// grid/level descriptors and the host-side kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace hh {

// ---------------------------------------------------------------------------
// complex128 as double2 (x = re, y = im)
// ---------------------------------------------------------------------------
typedef double2 cplx;

__host__ __device__ inline cplx mk(double re, double im) { cplx c; c.x = re; c.y = im; return c; }
__host__ __device__ inline cplx cadd(cplx a, cplx b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cplx csub(cplx a, cplx b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cplx cmul(cplx a, cplx b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ inline cplx cmulc(cplx a, cplx b) {
    return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline cplx cscale(cplx a, double s) { return mk(a.x * s, a.y * s); }
__host__ __device__ inline double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }
// a / b, by scaling with the larger component of b (Smith's method)
__host__ __device__ inline cplx cdiv(cplx a, cplx b) {
    if (fabs(b.x) >= fabs(b.y)) {
        double r = b.y / b.x, d = b.x + b.y * r;
        return mk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    } else {
        double r = b.x / b.y, d = b.y + b.x * r;
        return mk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
    }
}
__host__ __device__ inline cplx crecip(cplx b) { return cdiv(mk(1.0, 0.0), b); }

// ---------------------------------------------------------------------------
// Fine-grid operator A_sigma (matrix-free 5-point / 3-point stencil):
//   row p:  sum_a (prod_{b!=a} w_b)/h_a^2 sum_{q a-nbr}(u_p - u_q)
//         + j k_p sum_a e_a (prod_{b!=a} w_b)/h_a u_p - sigma k_p^2 prod_a w_a u_p
// w = 1/2 and e = 1 on the end nodes of an axis; 1D has no z axis.
// ---------------------------------------------------------------------------
struct FineOp {
    int nz, nx;          // nz = 1 in 1D
    int ndim;
    double ihx2, ihz2;   // 1/hx^2, 1/hz^2
    double ihx, ihz;     // 1/hx, 1/hz
    double omega;        // rad/s
    double omega2;       // omega^2
    double sr, si;       // sigma = sr + j si
    const double* m2;    // slowness squared, nz*nx
};

struct Coef5 {
    double cx;   // x-neighbour coupling (entry is -cx)
    double cz;   // z-neighbour coupling (entry is -cz)
    cplx diag;
};

// Row p = (iz, ix) of the fine operator.
__device__ __forceinline__ Coef5 fine_coefs(const FineOp& op, int iz, int ix, double m2p) {
    Coef5 c;
    const bool bx = (ix == 0) || (ix == op.nx - 1);
    const double wx = bx ? 0.5 : 1.0;
    bool bz = false;
    double wz = 1.0;
    if (op.ndim == 2) {
        bz = (iz == 0) || (iz == op.nz - 1);
        wz = bz ? 0.5 : 1.0;
    }
    c.cx = wz * op.ihx2;
    c.cz = wx * op.ihz2;
    double re = (double)((ix > 0) + (ix < op.nx - 1)) * c.cx;
    if (op.ndim == 2) re += (double)((iz > 0) + (iz < op.nz - 1)) * c.cz;
    const double k2 = op.omega2 * m2p;
    const double ww = wx * wz;
    double im = 0.0;
    if (bx || bz) {
        const double k = op.omega * sqrt(m2p);
        im = k * ((bx ? wz * op.ihx : 0.0) + (bz ? wx * op.ihz : 0.0));
    }
    re -= op.sr * k2 * ww;
    im -= op.si * k2 * ww;
    c.diag = mk(re, im);
    return c;
}

// Galerkin 9-point operator on a coarse level: coefficient t = (dz+1)*3+(dx+1)
// of node p is C[t*N + p]; coefficients of neighbours outside the grid are 0.
struct CoarseOp {
    int nz, nx;
    const cplx* C;
};

struct Level {
    int nz, nx;
    double hz, hx;
    int halve_z, halve_x;    // whether the NEXT coarser level halves z / x
};

// ---------------------------------------------------------------------------
// launchers (stencil.hip)
// ---------------------------------------------------------------------------
// y = A x (fine operator)
hipError_t launch_fine_apply(const FineOp& op, const cplx* x, cplx* y, hipStream_t s);
// r = b - A x
hipError_t launch_fine_residual(const FineOp& op, const cplx* b, const cplx* x, cplx* r,
                                hipStream_t s);
// x_out = omega_j D^{-1} b            (first sweep from x = 0)
hipError_t launch_fine_jacobi0(const FineOp& op, double wj, const cplx* b, cplx* xo,
                               hipStream_t s);
// x_out = x_in + omega_j D^{-1} (b - A x_in)
hipError_t launch_fine_jacobi(const FineOp& op, double wj, const cplx* b, const cplx* xi,
                              cplx* xo, hipStream_t s);
hipError_t launch_coarse_apply(const CoarseOp& op, const cplx* x, cplx* y, hipStream_t s);
hipError_t launch_coarse_residual(const CoarseOp& op, const cplx* b, const cplx* x, cplx* r,
                                  hipStream_t s);
hipError_t launch_coarse_jacobi0(const CoarseOp& op, double wj, const cplx* b, cplx* xo,
                                 hipStream_t s);
hipError_t launch_coarse_jacobi(const CoarseOp& op, double wj, const cplx* b, const cplx* xi,
                                cplx* xo, hipStream_t s);

// ---------------------------------------------------------------------------
// launchers (mg.hip)
// ---------------------------------------------------------------------------
// b_c = R r_f, R = P^T / 2^{d_c}
hipError_t launch_restrict(int nzf, int nxf, int hz, int hx, const cplx* rf, int nzc, int nxc,
                           cplx* bc, hipStream_t s);
// x_f += P e_c
hipError_t launch_prolong_add(int nzf, int nxf, int hz, int hx, const cplx* ec, int nzc,
                              int nxc, cplx* xf, hipStream_t s);
// Galerkin coarse operator from the fine operator (src level 0) or from a
// coarse 9-point operator
hipError_t launch_galerkin_from_fine(const FineOp& fine, int hz, int hx, int nzc, int nxc,
                                     cplx* Cc, hipStream_t s);
hipError_t launch_galerkin_from_coarse(const CoarseOp& fine, int hz, int hx, int nzc, int nxc,
                                       cplx* Cc, hipStream_t s);
// dense row-major matrix of a level operator
hipError_t launch_dense_from_fine(const FineOp& op, cplx* A, hipStream_t s);
hipError_t launch_dense_from_coarse(const CoarseOp& op, cplx* A, hipStream_t s);
// in-place inverse by Gauss-Jordan elimination with partial pivoting;
// scratch: 3n complex + n ints
hipError_t dense_invert(int n, cplx* A, cplx* scratch, int* perm, hipStream_t s);
// y = A x, A dense n x n row-major
hipError_t launch_dense_gemv(int n, const cplx* A, const cplx* x, cplx* y, hipStream_t s);

// ---------------------------------------------------------------------------
// launchers (pcr.hip): exact solve of the 1D tridiagonal shifted Laplacian
// ---------------------------------------------------------------------------
hipError_t launch_pcr_solve(const FineOp& op, const cplx* d, cplx* x, hipStream_t s);

// ---------------------------------------------------------------------------
// launchers (krylov.hip)
// ---------------------------------------------------------------------------
// number of partial-sum blocks used for a length-n reduction
int reduce_blocks(int64_t n);
// partial[i*nb + blk] = sum over the block's share of conj(V_i) w,  i < k
hipError_t launch_dot_partials(const cplx* V, int64_t n, int k, const cplx* w, cplx* partial,
                               int nb, hipStream_t s);
// out[i] = sum_blk partial[i*nb + blk], summed in a fixed order
hipError_t launch_reduce_partials(const cplx* partial, int nb, int k, cplx* out,
                                  hipStream_t s);
// w -= sum_i V_i h_i
hipError_t launch_multi_axpy(const cplx* V, int64_t n, int k, const cplx* h, cplx* w,
                             hipStream_t s);
// y = a * x with a read from device (real); a = *scale
hipError_t launch_scale_dev(const cplx* x, const double* scale, cplx* y, int64_t n,
                            hipStream_t s);
// b = W f
hipError_t launch_weight_rhs(const FineOp& op, const cplx* f, cplx* b, hipStream_t s);
// x += sum_i Z_i y_i
hipError_t launch_update_x(const cplx* Z, int64_t n, int k, const cplx* y, cplx* x,
                           hipStream_t s);
// validation of the slowness: flags[0] |= any non-finite or <= 0, mmax[0] = max
hipError_t launch_check_slowness(const double* m, int64_t n, double* m2, int* flag,
                                 double* mmax_partial, int nb, hipStream_t s);

// Device-side GMRES least-squares state (one restart cycle).
struct GivensState {
    int j;                // current column
    int m;                // restart length
    double beta0;         // ||b||
    double est;           // last residual estimate |g_{j+1}| / beta0
    double hn;            // h_{j+1,j}
    double inv_hn;        // 1 / h_{j+1,j}
    int breakdown;        // h_{j+1,j} == 0
    int bad;              // NaN/Inf seen
};
// Givens step on column j = st->j: the column is h1 + h2 (the two CGS2
// passes) with h_{j+1,j} = sqrt(nrm2[0].x); R is (m+1) x m column-major.
hipError_t launch_givens(GivensState* st, const cplx* h1, const cplx* h2, const cplx* nrm2,
                         cplx* R, double* cs, cplx* sn, cplx* g, hipStream_t s);
// y = R(1:k,1:k)^{-1} g(1:k)
hipError_t launch_backsub(int k, int m, const cplx* R, const cplx* g, cplx* y, hipStream_t s);
// state init for a new cycle: g = [beta, 0...], st->j = 0
hipError_t launch_cycle_init(GivensState* st, int m, double beta0, const cplx* nrm2, cplx* g,
                             double* inv_beta, hipStream_t s);

}  // namespace hh
