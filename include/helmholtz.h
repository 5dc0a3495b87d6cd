/*
 * helmholtz.h -- C ABI of the MI355X (gfx950) shifted-Laplace preconditioned
 * Helmholtz solver.
 *
 * The library solves the constant-density damped Helmholtz equation
 *     -Lap u - omega^2 m^2 (1 - j alpha) u = f                     (Eq. 2)
 * with a first-order absorbing boundary, discretised as H u = W f (Eq. 3),
 * by right-preconditioned flexible GMRES,
 *     H M^{-1} z = W f,  u = M^{-1} z                               (Eq. 5-7)
 * with the shifted Laplacian M = -Lap - (beta1 - j beta2) omega^2 m^2 of Eq. 6
 * as preconditioner (Kazemi, arXiv:1712.08740, Section "Data modelling").
 *
 * Discretisation (the paper prints none): second-order centred differences
 * (3-point in 1D, 5-point in 2D); boundary condition du/dn + j k u = 0 with
 * k = omega m, eliminated through a centred ghost node; every boundary row is
 * multiplied by 1/2 per boundary axis, and the right-hand side by the same row
 * weights W, which makes H and M exactly complex-symmetric. M^{-1} is applied
 * exactly in 1D (tridiagonal solve by parallel cyclic reduction) and
 * approximately in 2D by one V(2,2) multigrid cycle: omega-Jacobi smoothing
 * (weight 0.8, or 0.5 on levels with omega * max(m) * max(h) >= 2),
 * full-weighting restriction R = P^T / 2^{d_c}, bilinear prolongation P,
 * Galerkin coarse operators R M P, and a direct (explicit inverse) solve on the
 * coarsest grid. A dimension of n nodes and spacing h is coarsened to
 * (n-1)/2+1 nodes when n-1 is even, (n-1)/2 >= 2, and either
 * omega * max(m) * 2h <= pi (two or more nodes per shortest wavelength) or the
 * grid still has more than the dense limit (HH_MAX_COARSE nodes unless changed
 * by hh_set_max_coarse). The coarsest inverse comes from an LU factorisation
 * with partial pivoting (rocSOLVER) at set-up.
 *
 * Layout: real arrays are float64; complex arrays are complex128 stored as
 * interleaved (re, im) pairs. 1D grids have n nodes; 2D grids are stored
 * (nz, nx) row-major with x fastest.
 *
 * Pointers named *_dev are device pointers on the current HIP device; the
 * caller owns them. "stream" is a hipStream_t (NULL = the null stream). All
 * entry points return an hh_status; nothing aborts or throws across the ABI.
 * On error, hh_last_error() returns a message (thread-local, valid until the
 * next call on the same thread). A problem handle is not thread-safe; distinct
 * handles may be used concurrently from distinct threads on distinct streams.
 */
#ifndef HH_HELMHOLTZ_H
#define HH_HELMHOLTZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hh_problem_s* hh_problem;

enum hh_status {
    HH_OK            =  0,  /* converged / done                                   */
    HH_NOT_CONVERGED =  1,  /* iteration budget spent; u holds the last iterate   */
    HH_EINVAL        = -1,  /* invalid argument; nothing was launched             */
    HH_ENOMEM        = -2,  /* device allocation failed                           */
    HH_EDEVICE       = -3,  /* a HIP runtime call failed                          */
    HH_ENUMERIC      = -4,  /* NaN/Inf in a residual norm or breakdown quantity   */
    HH_EUNSUPPORTED  = -5   /* valid input outside what the library implements   */
};

/* hh_solve flags */
#define HH_NO_PRECOND 1u    /* plain GMRES on H (the paper's comparison, Fig. 3b/4) */
#define HH_PRECOND_F32 2u   /* the preconditioner M^{-1} in complex64 arithmetic: m^2,
                               smoother weights, Galerkin operators and coarsest inverse
                               rounded to single precision (round to nearest even), the
                               stored preconditioned vectors Z in complex64; the outer
                               flexible GMRES (Arnoldi basis, Hessenberg least squares,
                               residual recomputation, solution update) stays complex128.
                               Flexible GMRES takes any fixed preconditioner, so the
                               tolerance is met in full precision. Excludes HH_NO_PRECOND. */
#define HH_INITIAL_GUESS 4u /* u_dev holds the initial guess x0 on entry (default x0 = 0).
                               GMRES restarts from the iterate alone, so a solve that
                               stopped with HH_NOT_CONVERGED resumes from its returned u:
                               stopped at the end of a cycle (max_iters a multiple of
                               restart), the resumed solve gives the same bits as one
                               uninterrupted solve. hist[0] is then ||W f - H x0|| / ||W f||;
                               W f = 0 still returns u = 0. */

/* Default largest coarsest-grid size (unknowns) inverted densely, and the
 * largest that hh_set_max_coarse accepts (a 32768^2 complex128 inverse is 17 GB). */
#define HH_MAX_COARSE 4096
#define HH_MAX_COARSE_LIMIT 32768
/* Largest 1D grid handled by the single-workgroup tridiagonal solve. */
#define HH_MAX_1D 1024
/* Most right-hand sides in one hh_solve_batch call. */
#define HH_MAX_BATCH 1024

/*
 * hh_create_problem -- set up H for one model and frequency (Eq. 2-3).
 *   m_dev  : slowness 1/c (s/m), float64, n (1D) or nz*nx (2D) values, finite
 *            and > 0 (checked on the device; EINVAL otherwise). Copied: the
 *            caller may free it after the call returns.
 *   ndim   : 1 or 2.   shape: {n} or {nz, nx}; every entry >= 3; 1D n <= HH_MAX_1D.
 *   omega  : angular frequency 2 pi f (rad/s), > 0.
 *   alpha  : damping of Eq. 2, >= 0.
 *   h      : grid spacing (m), equal in x and z, > 0.
 *   stream : stream for the set-up work; the call returns after it completes.
 *   out    : receives the handle. The default shift (beta1, beta2) = (1, 0.5) is
 *            applied (hh_set_shift).
 * Returns EINVAL on bad arguments, EUNSUPPORTED when the coarsest multigrid grid
 * would exceed HH_MAX_COARSE unknowns, ENOMEM/EDEVICE on runtime failure.
 */
int hh_create_problem(const double* m_dev, int ndim, const int64_t* shape, double omega,
                      double alpha, double h, void* stream, hh_problem* out);

/* hh_create_problem with the dense limit of the coarsest grid given at once
 * (1..HH_MAX_COARSE_LIMIT; see hh_set_max_coarse), saving a rebuild. */
int hh_create_problem_ex(const double* m_dev, int ndim, const int64_t* shape, double omega,
                         double alpha, double h, int max_coarse, void* stream, hh_problem* out);

/*
 * hh_set_max_coarse -- rebuild the multigrid hierarchy with a different dense
 * limit for the coarsest grid (1..HH_MAX_COARSE_LIMIT unknowns; default
 * HH_MAX_COARSE). A larger limit stops the coarsening earlier, at the level
 * that still keeps two nodes per wavelength when that level fits, so the cycle
 * is a better preconditioner at the price of a larger dense inverse
 * (limit^2 * 16 bytes at most, plus a complex64 copy) read once per
 * preconditioner application (once per step for a whole batch of sources).
 * The shift in force is re-applied. 2D only (1D is solved exactly).
 */
int hh_set_max_coarse(hh_problem p, int max_coarse);

/*
 * Tile shapes of the multigrid legs. Each level l = 0 .. nlevels-2 has a down
 * leg (two pre-smoothing sweeps, residual, restriction; tiles of coarse nodes)
 * and an up leg (prolongation, two post-smoothing sweeps; tiles of level-l
 * nodes), one kernel each. Every shape computes every node with the same
 * arithmetic, so the choice changes the speed of a solve, never its bits.
 * HH_TILE_DOWN_ZMARCH is not a tile: on the fine level (when both axes halve)
 * each block marches along z over a strip of columns; on other levels it
 * means 4 x 4. HH_TILE_DEFAULT (-1) is a fixed rule: down 4 x 4 (z-marching on
 * a fine grid of at least 200000 nodes), up 8 x 4 (32 x 8 on such a fine
 * grid). A rebuilt hierarchy starts from the default.
 */
#define HH_TILE_DEFAULT (-1)
#define HH_TILE_DOWN_4X4 0
#define HH_TILE_DOWN_8X4 1
#define HH_TILE_DOWN_ZMARCH 2
#define HH_TILE_DOWN_COUNT 3
#define HH_TILE_UP_8X4 0
#define HH_TILE_UP_16X8 1
#define HH_TILE_UP_32X8 2
#define HH_TILE_UP_COUNT 3

/*
 * hh_autotune -- times every tile shape of every leg on this problem's
 * hierarchy and keeps per leg the fastest, where a shape replaces the default
 * only when it runs more than 3% faster (a project-side tuner for the
 * multigrid cycle of Sec. 3; not part of the paper's method).
 *   flags     : 0 (complex128 cycle) or HH_PRECOND_F32 (complex64 cycle).
 *   nrhs      : sources per batch the choice is made for (1..HH_MAX_BATCH).
 *   workspace_dev / workspace_bytes : at least hh_workspace_bytes_batch(p, 1,
 *               nrhs) bytes; overwritten (zeroed, then the legs' outputs).
 *   reps      : launches per timing (1..1000); each shape is timed three
 *               times and the shortest counts.
 * The call synchronises the stream. 1D problems and single-level hierarchies
 * have no legs: HH_OK, nothing tuned.
 */
int hh_autotune(hh_problem p, unsigned flags, int nrhs, void* workspace_dev,
                size_t workspace_bytes, int reps, void* stream);

/* Tile shapes of level `level`'s legs (HH_TILE_*; -1: default); read, or set
 * (for example from a cache of earlier hh_autotune results). HH_EINVAL for a
 * level without legs or an unknown shape. */
int hh_get_tiles(hh_problem p, int level, int* tile_down, int* tile_up);
int hh_set_tiles(hh_problem p, int level, int tile_down, int tile_up);

/*
 * hh_set_shift -- choose the shifted-Laplace preconditioner of Eq. 6,
 * M = -Lap - (beta1 - j beta2) omega^2 m^2 (same absorbing rows as H).
 * Rebuilds the multigrid hierarchy (Galerkin operators and coarsest inverse,
 * 2D) or the tridiagonal coefficients (1D) on the device. beta1, beta2 finite.
 * beta = (1, alpha) gives M = H.
 */
int hh_set_shift(hh_problem p, double beta1, double beta2);

/*
 * hh_footprint_bytes -- device memory a solve will need, before anything is
 * created (host-side planning only; for admission control by HBM footprint):
 * *problem_b = what hh_create_problem (+ hh_set_max_coarse(max_coarse)) would
 * allocate for the operators, *workspace_b = the workspace of hh_solve_batch
 * with nrhs sources (nrhs = 1: hh_solve) plus the batched coarsest product's
 * scratch. max_slowness = max(m) decides the coarsening (as in the solve).
 * flags as for hh_solve (the estimate is the complex128 one, an upper bound).
 */
int hh_footprint_bytes(int ndim, const int64_t* shape, double omega, double max_slowness,
                       double h, int max_coarse, int restart, int nrhs, unsigned flags,
                       size_t* problem_b, size_t* workspace_b);

/* Bytes of device workspace hh_solve needs for a given restart length. */
int hh_workspace_bytes(hh_problem p, int restart, size_t* bytes);

/*
 * hh_solve -- right-preconditioned FGMRES(restart) on H u = W f, x0 = 0 (or u_dev on
 *   entry with HH_INITIAL_GUESS).
 *   f_dev     : complex128 source, grid-shaped (not modified).
 *   tol       : relative tolerance in (0, 1) on ||W f - H u||_2 / ||W f||_2.
 *   restart   : Krylov basis length per cycle, 1..1024.
 *   max_iters : budget of preconditioned operator applications, >= 1.
 *   flags     : 0, HH_NO_PRECOND or HH_PRECOND_F32, each with or without
 *               HH_INITIAL_GUESS.
 *   workspace_dev / workspace_bytes : caller-owned device scratch of at least
 *               hh_workspace_bytes(p, restart) bytes; contents are overwritten.
 *   u_dev     : complex128 output wavefield, grid-shaped (caller-owned); the
 *               initial guess on entry with HH_INITIAL_GUESS.
 *   iterations: number of Arnoldi steps taken (may be NULL).
 *   true_rel_res : recomputed ||W f - H u|| / ||W f|| at exit (may be NULL).
 *   hist_host : host array; hist[0] = 1, hist[k] = Givens residual estimate
 *               after step k; at most hist_cap entries written (may be NULL).
 *   hist_len  : entries available (iterations + 1) (may be NULL).
 *   stream    : stream for the solve; the call returns after it completes.
 * Returns HH_OK when the recomputed residual meets tol (a happy breakdown counts),
 * HH_NOT_CONVERGED when max_iters is spent (u = last iterate), HH_ENUMERIC on
 * NaN/Inf. W f = 0 returns u = 0 and HH_OK with zero iterations.
 */
int hh_solve(hh_problem p, const void* f_dev, double tol, int restart, int max_iters,
             unsigned flags, void* workspace_dev, size_t workspace_bytes, void* u_dev,
             int* iterations, double* true_rel_res, double* hist_host, int hist_cap,
             int* hist_len, void* stream);

/* Bytes of device workspace hh_solve_batch needs: nrhs copies of the
 * single-solve workspace (any flags). */
int hh_workspace_bytes_batch(hh_problem p, int restart, int nrhs, size_t* bytes);

/*
 * hh_solve_batch -- hh_solve for nrhs sources of the same problem (same model,
 * frequency and shift; several sources per frequency in the paper's modelling
 * use), solved together: every kernel of an Arnoldi step covers all of them,
 * the operators and multigrid hierarchy are shared, and each source keeps its
 * own Krylov basis, least-squares problem and convergence test (a source whose
 * cycle has stopped takes no further work in it; cycles close when every source
 * has stopped). Each result is the one hh_solve gives for that source alone.
 *   nrhs      : 1..HH_MAX_BATCH.
 *   f_dev     : complex128 sources, nrhs grids back to back (not modified).
 *   u_dev     : complex128 wavefields, nrhs grids back to back (caller-owned;
 *               the initial guesses on entry with HH_INITIAL_GUESS).
 *   workspace : at least hh_workspace_bytes_batch(p, restart, nrhs) bytes.
 *   iterations, true_rel_res, status : host arrays of nrhs entries (may be NULL);
 *               status[i] is HH_OK, HH_NOT_CONVERGED or HH_ENUMERIC for source i.
 *   hist_host : host array of nrhs * hist_cap entries (source i at i * hist_cap,
 *               laid out as in hh_solve), or NULL with hist_cap = 0.
 * Returns HH_OK when every source converged, HH_NOT_CONVERGED when any spent
 * max_iters, HH_ENUMERIC when any met a non-finite value, or an error code.
 */
int hh_solve_batch(hh_problem p, int nrhs, const void* f_dev, double tol, int restart,
                   int max_iters, unsigned flags, void* workspace_dev, size_t workspace_bytes,
                   void* u_dev, int* iterations, double* true_rel_res, int* status,
                   double* hist_host, int hist_cap, void* stream);

/* Releases every device allocation of the handle. NULL is accepted. */
int hh_destroy_problem(hh_problem p);

/* Static description of a status code (thread-safe). */
const char* hh_status_string(int status);

/* Message of the last error on the calling thread ("" if none). */
const char* hh_last_error(void);

/* ---------------------------------------------------------------------------
 * Single steps of the solve, exported so that each can be checked on its own.
 * ------------------------------------------------------------------------- */

/* Number of multigrid levels (1 for 1D problems) and one level's grid:
 * shape2 = {nz, nx} (1D: {1, n}), spacing2 = {hz, hx}. */
int hh_num_levels(hh_problem p, int* nlevels);
int hh_level_info(hh_problem p, int level, int64_t* shape2, double* spacing2);

/*
 * hh_apply_operator -- y = A x on the fine grid, where which = 0 selects H
 * (Eq. 2-3) and which = 1 the shifted Laplacian M (Eq. 6). x_dev, y_dev:
 * complex128, grid-shaped, distinct. Matrix-free stencil kernel.
 */
int hh_apply_operator(hh_problem p, int which, const void* x_dev, void* y_dev, void* stream);

/*
 * hh_apply_level_operator -- y = M_l x on multigrid level l (l = 0 is M; l >= 1
 * the Galerkin operator R M_{l-1} P). Sizes are the level's grid.
 */
int hh_apply_level_operator(hh_problem p, int level, const void* x_dev, void* y_dev,
                            void* stream);

/*
 * hh_apply_precond -- z = M^{-1} v as used inside the solve (Eq. 7): the exact
 * tridiagonal solve in 1D, one V(2,2) cycle in 2D. v_dev, z_dev complex128,
 * grid-shaped, distinct; workspace as for hh_solve (any restart >= 1).
 */
int hh_apply_precond(hh_problem p, const void* v_dev, void* z_dev, void* workspace_dev,
                     size_t workspace_bytes, void* stream);

/*
 * hh_apply_precond_f32 -- the same preconditioner in complex64 (HH_PRECOND_F32):
 * v_dev complex128 (read, rounded inside), z_dev complex64 (written),
 * grid-shaped; workspace as for hh_solve.
 */
int hh_apply_precond_f32(hh_problem p, const void* v_dev, void* z_dev, void* workspace_dev,
                         size_t workspace_bytes, void* stream);

/*
 * hh_orthogonalize -- one classical Gram-Schmidt step with reorthogonalisation
 * (CGS2), the Arnoldi step of GMRES: given k orthonormal complex128 vectors of
 * length n stored contiguously (V_dev, vector i at V_dev + i*n) and w_dev,
 * computes h = V^H w, w -= V h, h2 = V^H w, w -= V h2, returns h + h2 in
 * h_host (k complex128 values, interleaved) and ||w||_2 in *norm_host.
 * 1 <= k <= 1024; scratch_dev must hold hh_orthogonalize_scratch_bytes(n, k).
 */
int hh_orthogonalize_scratch_bytes(int64_t n, int k, size_t* bytes);
int hh_orthogonalize(const void* V_dev, int64_t n, int k, void* w_dev, void* scratch_dev,
                     size_t scratch_bytes, double* h_host, double* norm_host, void* stream);

/* ---------------------------------------------------------------------------
 * Kernel timing (measurement support). After hh_kernel_timer_start(p, id),
 * every launch of that kernel class inside hh_solve on this handle is made
 * with hipExtLaunchKernelGGL and a pair of HIP events that the runtime stamps
 * at the dispatch's own start and end, on the solve's stream. Durations and
 * the algorithmic bytes of each launch (the kernel's byte model: the data it
 * must read and write once; k = number of basis vectors touched) are summed
 * over the launches that did work until read. HH_KERNEL_NONE switches it off.
 * ------------------------------------------------------------------------- */
enum hh_kernel_id {
    HH_KERNEL_NONE       = 0,
    HH_KERNEL_APPLY_DOT  = 1,  /* w = H z and the first projections V^H w: (40 + 16k) B/node */
    HH_KERNEL_AXPY_DOT   = 2,  /* w -= V h and the second projections: (k + 2) * 16 B/node   */
    HH_KERNEL_AXPY_NORM  = 3,  /* w -= V h and ||w||^2: (k + 2) * 16 B/node                  */
    HH_KERNEL_VC_DOWN    = 4,  /* fine-grid V-cycle down leg (2 sweeps, residual, restriction):
                                  72 B/node (w, m^2, omega/diag in; v, x2 out) + 16 B per
                                  coarse node                                              */
    HH_KERNEL_VC_UP      = 5,  /* fine-grid V-cycle up leg (prolongation, 2 sweeps):
                                  72 B/node (x2, v, m^2, omega/diag in; z out) + 16 B per
                                  coarse node                                              */
    HH_KERNEL_GEMV       = 6,  /* coarsest dense inverse times vector: (n^2 + 2n) * 16 B     */
    HH_KERNEL_PCR        = 7,  /* 1D tridiagonal solve: 56 B/node                            */
    HH_KERNEL_VC_DOWN_COARSE = 8,  /* coarse-level down legs: 192 B/node (b, 9 coefficients,
                                      omega/diag in; x2 out) + 16 B per next-level node    */
    HH_KERNEL_VC_UP_COARSE   = 9,  /* coarse-level up legs: 208 B/node (x2, b, 9 coefficients,
                                      omega/diag in; x out) + 16 B per next-level node     */
    HH_KERNEL_REDUCE     = 10, /* fixed-order sums of the projection partials:
                                  16 B per partial + 16 B per result                       */
    HH_KERNEL_GIVENS     = 11  /* Givens step (reads the norm partials; one block)         */
};
int hh_kernel_timer_start(hh_problem p, int kernel_id);
int hh_kernel_timer_read(hh_problem p, int64_t* launches, double* total_ms,
                         double* total_bytes);

#ifdef __cplusplus
}
#endif
#endif /* HH_HELMHOLTZ_H */
