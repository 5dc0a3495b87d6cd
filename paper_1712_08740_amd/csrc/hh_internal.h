// Internal declarations shared by the library's HIP sources: complex helpers,
// grid/level descriptors and the host-side kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace hh {

// When set (by the solve driver, for the one kernel class being timed), the
// next launch goes through hipExtLaunchKernelGGL with these events, which the
// runtime stamps at the dispatch's own start and end.
struct LaunchEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};
extern thread_local LaunchEvents g_launch_events;

#define HH_LAUNCH(KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                                  \
    do {                                                                                    \
        if (::hh::g_launch_events.start) {                                                  \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM,                       \
                                  ::hh::g_launch_events.start, ::hh::g_launch_events.stop,  \
                                  0, __VA_ARGS__);                                          \
            ::hh::g_launch_events = ::hh::LaunchEvents();                                   \
        } else {                                                                            \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);            \
        }                                                                                   \
    } while (0)

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

// complex64 as float2, for the single-precision preconditioner
typedef float2 cplxf;

__host__ __device__ inline cplxf mkf(float re, float im) { cplxf c; c.x = re; c.y = im; return c; }
__host__ __device__ inline cplxf cadd(cplxf a, cplxf b) { return mkf(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cplxf csub(cplxf a, cplxf b) { return mkf(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cplxf cmul(cplxf a, cplxf b) {
    return mkf(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline cplxf cmulc(cplxf a, cplxf b) {
    return mkf(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline cplxf cscale(cplxf a, float s) { return mkf(a.x * s, a.y * s); }
__host__ __device__ inline float cabs2(cplxf a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline cplxf cdiv(cplxf a, cplxf b) {
    if (fabsf(b.x) >= fabsf(b.y)) {
        float r = b.y / b.x, d = b.x + b.y * r;
        return mkf((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    } else {
        float r = b.x / b.y, d = b.y + b.x * r;
        return mkf((a.x * r + a.y) / d, (a.y * r - a.x) / d);
    }
}
__host__ __device__ inline cplxf crecip(cplxf b) { return cdiv(mkf(1.0f, 0.0f), b); }

// Complex type of a real type, and conversions between the two precisions
// (double -> float rounds to nearest even).
template <class T> struct Cx;
template <> struct Cx<double> { typedef cplx type; };
template <> struct Cx<float> { typedef cplxf type; };

template <class C> __host__ __device__ inline C cconv(cplx a);
template <class C> __host__ __device__ inline C cconv(cplxf a);
template <> __host__ __device__ inline cplx cconv<cplx>(cplx a) { return a; }
template <> __host__ __device__ inline cplxf cconv<cplxf>(cplx a) {
    return mkf((float)a.x, (float)a.y);
}
template <> __host__ __device__ inline cplx cconv<cplx>(cplxf a) {
    return mk((double)a.x, (double)a.y);
}
template <> __host__ __device__ inline cplxf cconv<cplxf>(cplxf a) { return a; }
template <class C> __host__ __device__ inline C czero() { return cconv<C>(mk(0.0, 0.0)); }

// ---------------------------------------------------------------------------
// Fine-grid operator A_sigma (matrix-free 5-point / 3-point stencil):
//   row p:  sum_a (prod_{b!=a} w_b)/h_a^2 sum_{q a-nbr}(u_p - u_q)
//         + j k_p sum_a e_a (prod_{b!=a} w_b)/h_a u_p - sigma k_p^2 prod_a w_a u_p
// w = 1/2 and e = 1 on the end nodes of an axis; 1D has no z axis.
// ---------------------------------------------------------------------------
template <class T>
struct FineOpT {
    typedef T real;
    typedef typename Cx<T>::type C;
    int nz, nx;          // nz = 1 in 1D
    int ndim;
    T ihx2, ihz2;        // 1/hx^2, 1/hz^2
    T ihx, ihz;          // 1/hx, 1/hz
    T omega;             // rad/s
    T omega2;            // omega^2
    T sr, si;            // sigma = sr + j si
    const T* m2;         // slowness squared, nz*nx
    const C* wdinv;      // omega_J / diag per node (V-cycle smoother), or nullptr
};
typedef FineOpT<double> FineOp;

template <class T>
struct Coef5T {
    T cx;                        // x-neighbour coupling (entry is -cx)
    T cz;                        // z-neighbour coupling (entry is -cz)
    typename Cx<T>::type diag;
};
typedef Coef5T<double> Coef5;

// Row p = (iz, ix) of the fine operator, in the operator's precision.
template <class T>
__device__ __forceinline__ Coef5T<T> fine_coefs(const FineOpT<T>& op, int iz, int ix, T m2p) {
    Coef5T<T> c;
    const T half = (T)0.5, one = (T)1;
    const bool bx = (ix == 0) || (ix == op.nx - 1);
    const T wx = bx ? half : one;
    bool bz = false;
    T wz = one;
    if (op.ndim == 2) {
        bz = (iz == 0) || (iz == op.nz - 1);
        wz = bz ? half : one;
    }
    c.cx = wz * op.ihx2;
    c.cz = wx * op.ihz2;
    T re = (T)((ix > 0) + (ix < op.nx - 1)) * c.cx;
    if (op.ndim == 2) re += (T)((iz > 0) + (iz < op.nz - 1)) * c.cz;
    const T k2 = op.omega2 * m2p;
    const T ww = wx * wz;
    T im = 0;
    if (bx || bz) {
        const T k = op.omega * sqrt(m2p);
        im = k * ((bx ? wz * op.ihx : (T)0) + (bz ? wx * op.ihz : (T)0));
    }
    re -= op.sr * k2 * ww;
    im -= op.si * k2 * ww;
    c.diag.x = re;
    c.diag.y = im;
    return c;
}

// Galerkin 9-point operator on a coarse level: coefficient t = (dz+1)*3+(dx+1)
// of node p is C[t*N + p]; coefficients of neighbours outside the grid are 0.
template <class T>
struct CoarseOpT {
    typedef T real;
    typedef typename Cx<T>::type Cv;
    int nz, nx;
    const Cv* C;
    const Cv* wdinv;     // omega_J / diag per node (V-cycle smoother)
};
typedef CoarseOpT<double> CoarseOp;

// Largest restart length (columns of the least-squares problem)
constexpr int kMaxColumns = 1024;

// Several right-hand sides solved together share the operators; each has its
// own copy of the solver workspace (same layout), `bs` bytes apart, and its
// source / wavefield `fs` elements apart in the caller's arrays. Kernels take
// the right-hand side from a grid dimension. One right-hand side: n = 1.
struct Batch {
    int n = 1;
    int64_t bs = 0;       // bytes between the workspaces of consecutive right-hand sides
    int64_t fs = 0;       // elements between consecutive sources / wavefields
};

// p advanced by `rb` strides of `bytes` (null stays null). Pointer arithmetic
// (not an integer round trip) keeps the pointer's provenance, so the compiler
// still knows it addresses global memory and emits global, not flat, accesses.
template <class T>
__host__ __device__ __forceinline__ T* rhs_at(T* p, int rb, int64_t bytes) {
    typedef typename std::conditional<std::is_const<T>::value, const char, char>::type B;
    return p ? reinterpret_cast<T*>(reinterpret_cast<B*>(p) + (int64_t)rb * bytes) : p;
}
// the same for a pointer that is never null (no select: keeps the compiler's
// proof that read-only arguments are not clobbered, so uniform values are
// fetched with scalar loads)
template <class T>
__host__ __device__ __forceinline__ T* rhs_nn(T* p, int rb, int64_t bytes) {
    typedef typename std::conditional<std::is_const<T>::value, const char, char>::type B;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(p) + (int64_t)rb * bytes);
}

// Workgroups of a launch are handed to the 8 XCDs round-robin by linear id.
// Map the linear id w (< n) to a logical tile index so that each XCD runs a
// contiguous range of tiles: neighbouring tiles then share halo data in the
// same L2.
__device__ __forceinline__ int xcd_tile(int w, int n) {
    const int x = w & 7, loc = w >> 3;
    const int q = n >> 3, r = n & 7;
    return x < r ? x * (q + 1) + loc : r * (q + 1) + (x - r) * q + loc;
}

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
hipError_t launch_coarse_apply(const CoarseOp& op, const cplx* x, cplx* y, hipStream_t s);

// Galerkin coarse operator from the fine operator (src level 0) or from a
// coarse 9-point operator
hipError_t launch_galerkin_from_fine(const FineOp& fine, int hz, int hx, int nzc, int nxc,
                                     cplx* Cc, hipStream_t s);
hipError_t launch_galerkin_from_coarse(const CoarseOp& fine, int hz, int hx, int nzc, int nxc,
                                       cplx* Cc, hipStream_t s);
// dense row-major matrix of a level operator
hipError_t launch_dense_from_fine(const FineOp& op, cplx* A, hipStream_t s);
hipError_t launch_dense_from_coarse(const CoarseOp& op, cplx* A, hipStream_t s);

// explicit inverse of the coarsest operator (bandlu.hip): A (row-major dense
// nz*nx x nz*nx, a 5- or 9-point stencil) is replaced by its inverse; scratch
// of band_scratch_bytes(nz, nx). The factorisation numbers the grid with z
// fastest when band_renumbered(nz, nx) (nz < nx); the inverse is then stored in
// that numbering (entry (q1, q2) for grid nodes q = ix nz + iz) unless
// `natural` is set. flag[0] |= 1 on a zero/non-finite pivot, |= 2 on a
// non-finite entry of the inverse (clear it first).
int band_halfwidth(int nz, int nx);
bool band_renumbered(int nz, int nx);
size_t band_scratch_bytes(int nz, int nx);
hipError_t band_invert(int nz, int nx, cplx* A, void* scratch, int* flag, bool natural,
                       hipStream_t s);

// ---------------------------------------------------------------------------
// launchers (krylov.hip): right-hand side, Arnoldi steps, solve control
// ---------------------------------------------------------------------------

// b = W f
hipError_t launch_weight_rhs(const FineOp& op, const cplx* f, cplx* b, hipStream_t s,
                             const Batch& bt = Batch());
// validation of the slowness: flags[0] |= any non-finite or <= 0, mmax[0] = max
hipError_t launch_check_slowness(const double* m, int64_t n, double* m2, int* flag,
                                 double* mmax_partial, int nb, hipStream_t s);

// Device-side control of a solve: every Arnoldi-step kernel reads `active`
// and returns at once when it is 0; the solve-level kernels read `done`.
struct SolveState {
    int active;      // a restart cycle is open: Arnoldi steps run
    int done;        // the solve has finished
    int status;      // 0 converged, 1 budget spent, -4 non-finite
    int j;           // steps taken in the current cycle
    int k;           // columns of the current least-squares problem
    int m;           // restart length
    int it;          // Arnoldi steps taken in the solve
    int max_iters;
    double tol;
    double beta0;    // ||W f||
    double rel;      // last recomputed relative residual
};

// Progress record in pinned host memory, written by the device, polled by the
// host to decide how far ahead to enqueue.
struct HostRecord {
    int seq;         // bumped by every record write
    int done;
    int status;
    int it;
    int cycles;      // restart cycles opened (or closed as done) so far
    int jstep;       // steps finished in the current cycle
    int stops;       // cycles closed by a step (converged estimate, full basis, budget)
    int pad;
    double est;      // last residual estimate
    double rel;      // last recomputed relative residual
};


// ---- fused, predicated Arnoldi kernels (krylov.hip) -----------------------
// w = H z and, with u = V_{k-1}, partial[i*nb + blk] = block sums of conj(V_i) u
// and partial[(k+i)*nb + blk] = block sums of conj(V_i) w, i < k (nb = apply_blocks(op, nrhs))
hipError_t launch_apply_dot(const FineOp& op, const cplx* z, cplx* w, const cplx* V, int k,
                            cplx* partial, const int* active, hipStream_t s,
                            const Batch& bt = Batch());
hipError_t launch_apply_dot(const FineOp& op, const cplxf* z, cplx* w, const cplx* V, int k,
                            cplx* partial, const int* active, hipStream_t s,
                            const Batch& bt = Batch());
int apply_blocks(const FineOp& op, int nrhs);
// partials of launch_residual_norm (one per 64 x 4 tile in 2D)
int residual_blocks(const FineOp& op);
int node_blocks(int64_t n);
// blocks of the norm kernel (its partial sums are re-read by each consumer)
constexpr int kNormBlocks = 512;
int norm_blocks(int64_t n);
hipError_t launch_dot_blocks(const cplx* V, int64_t n, int k, const cplx* w, cplx* partial,
                             hipStream_t s, const Batch& bt = Batch());
// w -= V h; partial = block sums of conj(V_i) w (nb = node_blocks(n))
hipError_t launch_axpy_dot(const cplx* V, int64_t n, int k, const cplx* h, cplx* w, cplx* partial,
                           const int* active, hipStream_t s, const Batch& bt = Batch());
// w -= V h; partial[blk].x = block sums of |w|^2 (nb = norm_blocks(n))
hipError_t launch_axpy_norm(const cplx* V, int64_t n, int k, const cplx* h, cplx* w, cplx* partial,
                            const int* active, hipStream_t s, const Batch& bt = Batch());
hipError_t launch_reduce_pred(const cplx* partial, int nb, int k, cplx* out, const int* active,
                              hipStream_t s, const Batch& bt = Batch());
// r = b - H u; partial[blk].x = block sums of |r|^2 (skipped when *done)
hipError_t launch_residual_norm(const FineOp& op, const cplx* b, const cplx* u, cplx* r,
                                cplx* partial, const int* done, hipStream_t s,
                                const Batch& bt = Batch());
// warm: the solve started from a given guess; the first cycle records its
// relative residual as hist[0]
hipError_t launch_cycle_start(SolveState* st, const cplx* partial, int nb, cplx* g,
                              HostRecord* rec, double* hist, int64_t hist_stride, bool warm,
                              hipStream_t s, const Batch& bt = Batch());
struct GivensArgs;
// Arnoldi step with delayed reorthogonalisation, second pass (see krylov.hip):
// V_j <- reorthogonalised, normalised u = V_j; V_{j+1} <- w projected once;
// red = the reduced [V_{0..j}^H u, V_{0..j}^H w]; with giv, one extra
// workgroup per right-hand side runs the Givens step of column j - 1
hipError_t launch_axpy_dcgs(cplx* V, int64_t n, int j, const cplx* red, const cplx* w,
                            const int* active, const GivensArgs* giv, hipStream_t s,
                            const Batch& bt = Batch());
// the Givens step closing a full cycle (red = [V_{0..m-1}^H V_m, V_m^H V_m])
hipError_t launch_givens_tail(const GivensArgs& a, hipStream_t s, const Batch& bt = Batch());
// y = R^{-1} g, x += Z y for the st->k columns of the cycle, then st->k = 0
// (m: the restart length, an upper bound of the columns st->k)
hipError_t launch_cycle_finish(SolveState* st, int m, const cplx* R, const cplx* g,
                               const double* zs, cplx* y, const cplx* Z, int64_t n, cplx* x,
                               hipStream_t s, const Batch& bt = Batch());
hipError_t launch_cycle_finish(SolveState* st, int m, const cplx* R, const cplx* g,
                               const double* zs, cplx* y, const cplxf* Z, int64_t n, cplx* x,
                               hipStream_t s, const Batch& bt = Batch());
// u_warm: the caller's initial guesses (zeroed for a zero right-hand side), or
// null when the solve starts from zero; n nodes per wavefield
hipError_t launch_solve_init(SolveState* st, const cplx* partial, int nb, int m, int max_iters,
                             double tol, HostRecord* rec, double* hist, int64_t hist_stride,
                             cplx* u_warm, int64_t n, hipStream_t s, const Batch& bt = Batch());

// ---- V-cycle kernels (vcycle_tiled.hip, coarsest.hip) ------------------------
// coarsest level: y = A x (one right-hand side), or for every right-hand side
// of a batch (x, y and the predicate in each right-hand side's workspace)
hipError_t launch_vc_gemv(int n, const cplx* A, const cplx* x, cplx* y, const int* active,
                          hipStream_t s, const Batch& bt = Batch());
hipError_t launch_vc_gemv(int n, const cplxf* A, const cplxf* x, cplxf* y, const int* active,
                          hipStream_t s, const Batch& bt = Batch());
hipError_t launch_vc_gemv(int n, const cplxf* A, const cplx* x, cplxf* y, const int* active,
                          hipStream_t s, const Batch& bt = Batch());
// the same product for every right-hand side of a batch at once (Y = A X, the
// inverse read once per 32 right-hand sides); not predicated: the columns of
// sources whose cycle has stopped are computed too and not used
// (split over k for parallelism; scratch holds the partial sums, at least
// vc_gemm_scratch_bytes(n, bt.n) bytes)
size_t vc_gemm_scratch_bytes(int n, int nrhs);
hipError_t launch_vc_gemm(int n, const cplx* A, const cplx* x, cplx* y, void* scratch,
                          hipStream_t s, const Batch& bt);
hipError_t launch_vc_gemm(int n, const cplxf* A, const cplxf* x, cplxf* y, void* scratch,
                          hipStream_t s, const Batch& bt);
// temporally blocked legs (vcycle_tiled.hip): down = two pre-sweeps from zero,
// residual and restriction; up = prolongation and two post-sweeps
// (the smoother weight enters through op.wdinv = omega_J / diag).
// tile: the leg's tile shape, HH_TILE_* ids of helmholtz.h (-1: the default
// for the level); every shape gives the same bits.
// The next coarser grid: its shape, and whether its vectors are stored x-major
// (node (iz, ix) at ix nz + iz: the band numbering of the coarsest inverse)
// instead of z-major.
struct CGrid {
    int nz, nx, xmajor;
    __host__ __device__ int64_t at(int iz, int ix) const {
        return xmajor ? (int64_t)ix * nz + iz : (int64_t)iz * nx + ix;
    }
};
hipError_t launch_vc_fine_down(const FineOp& op, const cplx* src, cplx* x2, int hz, int hx,
                               CGrid cg, cplx* bc, const int* active, hipStream_t s,
                               const Batch& bt = Batch(), int tile = -1);
// single-precision cycle: the Krylov vector src stays complex128
hipError_t launch_vc_fine_down(const FineOpT<float>& op, const cplx* src, cplxf* x2, int hz,
                               int hx, CGrid cg, cplxf* bc, const int* active,
                               hipStream_t s, const Batch& bt = Batch(), int tile = -1);
hipError_t launch_vc_coarse_down(const CoarseOpT<float>& op, const cplxf* b, cplxf* x2, int hz,
                                 int hx, CGrid cg, cplxf* bc, const int* active,
                                 hipStream_t s, const Batch& bt = Batch(), int tile = -1);
hipError_t launch_vc_fine_up(const FineOpT<float>& op, int hz, int hx, const cplx* b,
                             const cplxf* x2, const cplxf* e, CGrid cg, cplxf* out,
                             const int* active, hipStream_t s, const Batch& bt = Batch(), int tile = -1);
hipError_t launch_vc_coarse_up(const CoarseOpT<float>& op, int hz, int hx, const cplxf* b,
                               const cplxf* x2, const cplxf* e, CGrid cg, cplxf* out,
                               const int* active, hipStream_t s, const Batch& bt = Batch(), int tile = -1);
hipError_t launch_vc_coarse_down(const CoarseOp& op, const cplx* b, cplx* x2, int hz,
                                 int hx, CGrid cg, cplx* bc, const int* active,
                                 hipStream_t s, const Batch& bt = Batch(), int tile = -1);
hipError_t launch_vc_fine_up(const FineOp& op, int hz, int hx, const cplx* b,
                             const cplx* x2, const cplx* e, CGrid cg, cplx* out, const int* active,
                             hipStream_t s, const Batch& bt = Batch(), int tile = -1);
hipError_t launch_vc_coarse_up(const CoarseOp& op, int hz, int hx, const cplx* b,
                               const cplx* x2, const cplx* e, CGrid cg, cplx* out,
                               const int* active, hipStream_t s, const Batch& bt = Batch(), int tile = -1);
// wdinv = wj / diag of a level operator (set-up)
hipError_t launch_wdinv_fine(const FineOp& op, double wj, cplx* wdinv, hipStream_t s);
hipError_t launch_wdinv_coarse(const CoarseOp& op, double wj, cplx* wdinv, hipStream_t s);
// 1D preconditioner x = M^{-1} src by parallel cyclic reduction (pcr.hip):
// the multipliers of every step and the final diagonal of M (op), computed
// once per shift into f (pcr_factor_elems(n) values), then applied per
// right-hand side, predicated on *active
int pcr_levels(int n);
size_t pcr_factor_elems(int n);
hipError_t launch_pcr_factor(const FineOp& op, cplx* f, hipStream_t s);
hipError_t launch_pcr_factor(const FineOpT<float>& op, cplxf* f, hipStream_t s);
hipError_t launch_pcr(int n, const cplx* f, const cplx* src, cplx* x, const int* active,
                      hipStream_t s, const Batch& bt = Batch());
hipError_t launch_pcr(int n, const cplxf* f, const cplx* src, cplxf* x, const int* active,
                      hipStream_t s, const Batch& bt = Batch());

// precision conversions (set-up of the single-precision preconditioner), RNE
hipError_t launch_to_f32(const double* a, float* b, int64_t n, hipStream_t s);
hipError_t launch_to_c64(const cplx* a, cplxf* b, int64_t n, hipStream_t s);

}  // namespace hh
