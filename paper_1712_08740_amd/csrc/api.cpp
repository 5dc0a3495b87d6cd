// C ABI of the solver (include/helmholtz.h): problem set-up, the
// shifted-Laplace preconditioner hierarchy, and the right-preconditioned
// flexible GMRES driver (Eq. 5-7). The host only sequences kernels and reads
// back the scalars that decide convergence; every arithmetic step runs on
// the device.
#include "helmholtz.h"
#include "hh_internal.h"

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

using namespace hh;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(e_ == hipErrorOutOfMemory ? HH_ENOMEM : HH_EDEVICE,              \
                        std::string(#expr) + ": " + hipGetErrorString(e_));              \
    } while (0)

#define CHK(expr)                       \
    do {                                \
        int r_ = (expr);                \
        if (r_ != HH_OK) return r_;     \
    } while (0)

constexpr double kJacobiWeight = 0.8;
constexpr int kMaxRestart = 1024;

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct LevelData {
    int nz = 0, nx = 0;
    double hz = 0, hx = 0;
    int halve_z = 0, halve_x = 0;   // halving flags towards the next coarser level
    cplx* C = nullptr;              // 9-point Galerkin operator (levels >= 1)
    int64_t size() const { return (int64_t)nz * nx; }
};

}  // namespace

struct hh_problem_s {
    int ndim = 0;
    int nz = 1, nx = 0;
    int64_t N = 0;
    double omega = 0, alpha = 0, h = 0;
    double beta1 = 1.0, beta2 = 0.5;
    double mmax = 0;
    double* m2 = nullptr;
    std::vector<LevelData> levels;
    cplx* cinv = nullptr;           // explicit inverse of the coarsest operator
    int nc = 0;
    cplx* gj_scratch = nullptr;
    int* gj_perm = nullptr;
    int* dflag = nullptr;           // device scratch for checks
    double* dpartial = nullptr;
    GivensState* st_host = nullptr; // pinned
    cplx* nrm2_host = nullptr;      // pinned
    hipStream_t stream = nullptr;
    // per-launch event timing of one kernel class (hh_kernel_timer_*)
    struct {
        int kid = HH_KERNEL_NONE;
        std::vector<hipEvent_t> pool;
        int used = 0;
        std::vector<double> pending_bytes;
        int64_t launches = 0;
        double total_ms = 0.0, total_bytes = 0.0;
    } kt;
};

namespace {

FineOp fine_op(const hh_problem_s* p, double sr, double si) {
    FineOp op;
    op.nz = p->nz;
    op.nx = p->nx;
    op.ndim = p->ndim;
    op.ihx2 = 1.0 / (p->h * p->h);
    op.ihz2 = op.ihx2;
    op.ihx = 1.0 / p->h;
    op.ihz = op.ihx;
    op.omega = p->omega;
    op.omega2 = p->omega * p->omega;
    op.sr = sr;
    op.si = si;
    op.m2 = p->m2;
    return op;
}
FineOp op_H(const hh_problem_s* p) { return fine_op(p, 1.0, -p->alpha); }
FineOp op_M(const hh_problem_s* p) { return fine_op(p, p->beta1, -p->beta2); }
CoarseOp coarse_op(const LevelData& L) {
    CoarseOp op;
    op.nz = L.nz;
    op.nx = L.nx;
    op.C = L.C;
    return op;
}

// ---------------------------------------------------------------------------
// kernel timer
// ---------------------------------------------------------------------------
int kt_begin(hh_problem_s* p, int kid, hipStream_t s) {
    if (p->kt.kid != kid) return HH_OK;
    while ((int)p->kt.pool.size() < p->kt.used + 2) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        p->kt.pool.push_back(e);
    }
    HIPCHK(hipEventRecord(p->kt.pool[p->kt.used], s));
    return HH_OK;
}

int kt_end(hh_problem_s* p, int kid, hipStream_t s, double bytes) {
    if (p->kt.kid != kid) return HH_OK;
    HIPCHK(hipEventRecord(p->kt.pool[p->kt.used + 1], s));
    p->kt.pending_bytes.push_back(bytes);
    p->kt.used += 2;
    return HH_OK;
}

// after a stream synchronisation: fold the completed event pairs in
int kt_harvest(hh_problem_s* p) {
    for (int i = 0; i < p->kt.used / 2; ++i) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, p->kt.pool[2 * i], p->kt.pool[2 * i + 1]));
        p->kt.total_ms += ms;
        p->kt.total_bytes += p->kt.pending_bytes[i];
        p->kt.launches += 1;
    }
    p->kt.used = 0;
    p->kt.pending_bytes.clear();
    return HH_OK;
}

#define TIMED(KID, BYTES, EXPR)                     \
    do {                                            \
        CHK(kt_begin(p, (KID), s));                 \
        HIPCHK(EXPR);                               \
        CHK(kt_end(p, (KID), s, (double)(BYTES)));  \
    } while (0)

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
struct Layout {
    size_t V, Z, b, partial, h1, h2, nrm2, R, cs, sn, g, y, inv_beta, st, total;
    std::vector<size_t> t, r, bc, ec;   // per level
    int nb;
};

Layout layout(const hh_problem_s* p, int m) {
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t c = sizeof(cplx);
    const size_t N = (size_t)p->N;
    L.V = take((size_t)(m + 1) * N * c);
    L.Z = take((size_t)m * N * c);
    L.b = take(N * c);
    const int nl = (int)p->levels.size();
    L.t.assign(nl, 0);
    L.r.assign(nl, 0);
    L.bc.assign(nl, 0);
    L.ec.assign(nl, 0);
    if (p->ndim == 2) {
        for (int l = 0; l < nl; ++l) {
            const size_t n = (size_t)p->levels[l].size();
            if (l < nl - 1) {
                L.t[l] = take(n * c);
                L.r[l] = take(n * c);
            }
            if (l >= 1) {
                L.bc[l] = take(n * c);
                L.ec[l] = take(n * c);
            }
        }
    }
    L.nb = reduce_blocks(p->N);
    const int kmax = m + 1 > 1 ? m + 1 : 1;
    L.partial = take((size_t)L.nb * kmax * c);
    L.h1 = take((size_t)kmax * c);
    L.h2 = take((size_t)kmax * c);
    L.nrm2 = take(c);
    L.R = take((size_t)(m + 1) * m * c);
    L.cs = take((size_t)m * sizeof(double));
    L.sn = take((size_t)m * c);
    L.g = take((size_t)(m + 1) * c);
    L.y = take((size_t)m * c);
    L.inv_beta = take(sizeof(double));
    L.st = take(sizeof(GivensState));
    L.total = off;
    return L;
}

template <class T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// ||x||^2 into out[0].x
int norm2_async(const cplx* x, int64_t n, cplx* partial, int nb, cplx* out, hipStream_t s) {
    HIPCHK(launch_dot_partials(x, n, 1, x, partial, nb, s));
    HIPCHK(launch_reduce_partials(partial, nb, 1, out, s));
    return HH_OK;
}

// ---------------------------------------------------------------------------
// preconditioner
// ---------------------------------------------------------------------------
// One V(2,2) cycle on level l: out = V(l, b). b and out are distinct.
int vcycle(hh_problem_s* p, const Layout& L, void* ws, int l, const cplx* b, cplx* out,
           hipStream_t s) {
    const int nl = (int)p->levels.size();
    const LevelData& lv = p->levels[l];
    if (l == nl - 1) {
        const double nc = p->nc;
        TIMED(HH_KERNEL_GEMV, (nc * nc + 2 * nc) * sizeof(cplx),
              launch_dense_gemv(p->nc, p->cinv, b, out, s));
        return HH_OK;
    }
    cplx* t = at<cplx>(ws, L.t[l]);
    cplx* r = at<cplx>(ws, L.r[l]);
    const LevelData& nx = p->levels[l + 1];
    cplx* bc = at<cplx>(ws, L.bc[l + 1]);
    cplx* ec = at<cplx>(ws, L.ec[l + 1]);
    const double jac_bytes = 56.0 * (double)lv.size();
    if (l == 0) {
        const FineOp M = op_M(p);
        HIPCHK(launch_fine_jacobi0(M, kJacobiWeight, b, t, s));
        TIMED(HH_KERNEL_JACOBI, jac_bytes, launch_fine_jacobi(M, kJacobiWeight, b, t, out, s));
        HIPCHK(launch_fine_residual(M, b, out, r, s));
    } else {
        const CoarseOp A = coarse_op(lv);
        HIPCHK(launch_coarse_jacobi0(A, kJacobiWeight, b, t, s));
        HIPCHK(launch_coarse_jacobi(A, kJacobiWeight, b, t, out, s));
        HIPCHK(launch_coarse_residual(A, b, out, r, s));
    }
    HIPCHK(launch_restrict(lv.nz, lv.nx, lv.halve_z, lv.halve_x, r, nx.nz, nx.nx, bc, s));
    CHK(vcycle(p, L, ws, l + 1, bc, ec, s));
    HIPCHK(launch_prolong_add(lv.nz, lv.nx, lv.halve_z, lv.halve_x, ec, nx.nz, nx.nx, out, s));
    if (l == 0) {
        const FineOp M = op_M(p);
        TIMED(HH_KERNEL_JACOBI, jac_bytes, launch_fine_jacobi(M, kJacobiWeight, b, out, t, s));
        TIMED(HH_KERNEL_JACOBI, jac_bytes, launch_fine_jacobi(M, kJacobiWeight, b, t, out, s));
    } else {
        const CoarseOp A = coarse_op(lv);
        HIPCHK(launch_coarse_jacobi(A, kJacobiWeight, b, out, t, s));
        HIPCHK(launch_coarse_jacobi(A, kJacobiWeight, b, t, out, s));
    }
    return HH_OK;
}

int precond(hh_problem_s* p, const Layout& L, void* ws, const cplx* v, cplx* z,
            hipStream_t s) {
    if (p->ndim == 1) {
        TIMED(HH_KERNEL_PCR, 40.0 * (double)p->N, launch_pcr_solve(op_M(p), v, z, s));
        return HH_OK;
    }
    return vcycle(p, L, ws, 0, v, z, s);
}

// ---------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------
void free_levels(hh_problem_s* p) {
    for (auto& l : p->levels)
        if (l.C) {
            (void)hipFree(l.C);
            l.C = nullptr;
        }
}

int build_hierarchy(hh_problem_s* p) {
    p->levels.clear();
    LevelData L0;
    L0.nz = p->nz;
    L0.nx = p->nx;
    L0.hz = p->h;
    L0.hx = p->h;
    p->levels.push_back(L0);
    if (p->ndim == 1) {
        p->nc = 0;
        return HH_OK;
    }
    const double kmax = p->omega * p->mmax;
    for (;;) {
        LevelData& cur = p->levels.back();
        auto halves = [&](int n, double h) {
            return (n - 1) % 2 == 0 && (n - 1) / 2 >= 2 && kmax * 2.0 * h <= M_PI;
        };
        const int hz = halves(cur.nz, cur.hz), hx = halves(cur.nx, cur.hx);
        if (!hz && !hx) break;
        cur.halve_z = hz;
        cur.halve_x = hx;
        LevelData nxt;
        nxt.nz = hz ? (cur.nz - 1) / 2 + 1 : cur.nz;
        nxt.nx = hx ? (cur.nx - 1) / 2 + 1 : cur.nx;
        nxt.hz = hz ? 2.0 * cur.hz : cur.hz;
        nxt.hx = hx ? 2.0 * cur.hx : cur.hx;
        p->levels.push_back(nxt);
    }
    const int64_t nc = p->levels.back().size();
    if (nc > HH_MAX_COARSE)
        return fail(HH_EUNSUPPORTED,
                    "coarsest multigrid grid has " + std::to_string(nc) +
                        " unknowns (more than HH_MAX_COARSE = " +
                        std::to_string(HH_MAX_COARSE) + ")");
    p->nc = (int)nc;
    for (size_t l = 1; l < p->levels.size(); ++l)
        HIPCHK(hipMalloc(&p->levels[l].C, 9 * (size_t)p->levels[l].size() * sizeof(cplx)));
    HIPCHK(hipMalloc(&p->cinv, (size_t)nc * nc * sizeof(cplx)));
    HIPCHK(hipMalloc(&p->gj_scratch, 3 * (size_t)nc * sizeof(cplx)));
    HIPCHK(hipMalloc(&p->gj_perm, (size_t)nc * sizeof(int)));
    return HH_OK;
}

int apply_shift(hh_problem_s* p) {
    if (p->ndim == 1) return HH_OK;
    hipStream_t s = p->stream;
    const int nl = (int)p->levels.size();
    const FineOp M = op_M(p);
    for (int l = 1; l < nl; ++l) {
        const LevelData& f = p->levels[l - 1];
        LevelData& c = p->levels[l];
        if (l == 1)
            HIPCHK(launch_galerkin_from_fine(M, f.halve_z, f.halve_x, c.nz, c.nx, c.C, s));
        else
            HIPCHK(launch_galerkin_from_coarse(coarse_op(f), f.halve_z, f.halve_x, c.nz, c.nx,
                                               c.C, s));
    }
    if (nl == 1)
        HIPCHK(launch_dense_from_fine(M, p->cinv, s));
    else
        HIPCHK(launch_dense_from_coarse(coarse_op(p->levels.back()), p->cinv, s));
    HIPCHK(dense_invert(p->nc, p->cinv, p->gj_scratch, p->gj_perm, s));
    // the inverse must be finite: ||cinv||^2 over the whole matrix
    const int64_t nn = (int64_t)p->nc * p->nc;
    const int nb = reduce_blocks(nn);
    cplx* partial = reinterpret_cast<cplx*>(p->dpartial);
    std::vector<cplx> tmp(1);
    cplx* out = partial + nb;
    CHK(norm2_async(p->cinv, nn, partial, nb, out, s));
    HIPCHK(hipMemcpyAsync(p->nrm2_host, out, sizeof(cplx), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!std::isfinite(p->nrm2_host->x))
        return fail(HH_ENUMERIC, "coarsest-level operator is singular for this shift");
    return HH_OK;
}

void destroy(hh_problem_s* p) {
    if (!p) return;
    free_levels(p);
    if (p->m2) (void)hipFree(p->m2);
    if (p->cinv) (void)hipFree(p->cinv);
    if (p->gj_scratch) (void)hipFree(p->gj_scratch);
    if (p->gj_perm) (void)hipFree(p->gj_perm);
    if (p->dflag) (void)hipFree(p->dflag);
    if (p->dpartial) (void)hipFree(p->dpartial);
    if (p->st_host) (void)hipHostFree(p->st_host);
    if (p->nrm2_host) (void)hipHostFree(p->nrm2_host);
    for (hipEvent_t e : p->kt.pool) (void)hipEventDestroy(e);
    delete p;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_vec_args(const void* a, const char* name) {
    if (!a) return fail(HH_EINVAL, std::string(name) + " is NULL");
    return HH_OK;
}

}  // namespace

extern "C" {

const char* hh_status_string(int status) {
    switch (status) {
        case HH_OK: return "ok";
        case HH_NOT_CONVERGED: return "not converged within the iteration budget";
        case HH_EINVAL: return "invalid argument";
        case HH_ENOMEM: return "device out of memory";
        case HH_EDEVICE: return "HIP runtime error";
        case HH_ENUMERIC: return "non-finite value in the iteration";
        case HH_EUNSUPPORTED: return "unsupported problem size";
        default: return "unknown status";
    }
}

const char* hh_last_error(void) { return g_err.c_str(); }

int hh_create_problem(const double* m_dev, int ndim, const int64_t* shape, double omega,
                      double alpha, double h, void* stream, hh_problem* out) {
    g_err.clear();
    if (!out) return fail(HH_EINVAL, "out is NULL");
    *out = nullptr;
    if (!m_dev) return fail(HH_EINVAL, "m_dev is NULL");
    if (ndim != 1 && ndim != 2) return fail(HH_EINVAL, "ndim must be 1 or 2");
    if (!shape) return fail(HH_EINVAL, "shape is NULL");
    for (int d = 0; d < ndim; ++d)
        if (shape[d] < 3 || shape[d] > (1 << 24))
            return fail(HH_EINVAL, "every grid dimension must be in [3, 2^24]");
    if (ndim == 1 && shape[0] > HH_MAX_1D)
        return fail(HH_EUNSUPPORTED, "1D grids are limited to HH_MAX_1D nodes");
    if (!finite_pos(omega)) return fail(HH_EINVAL, "omega must be finite and > 0");
    if (!(std::isfinite(alpha) && alpha >= 0.0)) return fail(HH_EINVAL, "alpha must be >= 0");
    if (!finite_pos(h)) return fail(HH_EINVAL, "h must be finite and > 0");

    hh_problem_s* p = new hh_problem_s();
    p->ndim = ndim;
    p->nz = ndim == 2 ? (int)shape[0] : 1;
    p->nx = ndim == 2 ? (int)shape[1] : (int)shape[0];
    p->N = (int64_t)p->nz * p->nx;
    p->omega = omega;
    p->alpha = alpha;
    p->h = h;
    p->stream = static_cast<hipStream_t>(stream);
    auto bail = [&](int code) {
        destroy(p);
        return code;
    };
    const int nb = reduce_blocks(p->N);
    hipError_t e;
    if ((e = hipMalloc(&p->m2, p->N * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&p->dflag, sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&p->dpartial, 4096 * sizeof(cplx))) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void**>(&p->st_host), sizeof(GivensState))) !=
            hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void**>(&p->nrm2_host), 64 * sizeof(cplx))) !=
            hipSuccess)
        return bail(fail(e == hipErrorOutOfMemory ? HH_ENOMEM : HH_EDEVICE,
                         std::string("allocation: ") + hipGetErrorString(e)));
    hipStream_t s = p->stream;
    double* mpart = p->dpartial;
    std::vector<double> hpart(nb);
    int hflag = 0;
    if ((e = hipMemsetAsync(p->dflag, 0, sizeof(int), s)) != hipSuccess ||
        (e = launch_check_slowness(m_dev, p->N, p->m2, p->dflag, mpart, nb, s)) != hipSuccess ||
        (e = hipMemcpyAsync(hpart.data(), mpart, nb * sizeof(double), hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipMemcpyAsync(&hflag, p->dflag, sizeof(int), hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return bail(fail(HH_EDEVICE, std::string("set-up: ") + hipGetErrorString(e)));
    if (hflag) return bail(fail(HH_EINVAL, "slowness must be finite and > 0 everywhere"));
    p->mmax = 0.0;
    for (double v : hpart) p->mmax = std::fmax(p->mmax, v);
    int rc = build_hierarchy(p);
    if (rc != HH_OK) return bail(rc);
    rc = apply_shift(p);
    if (rc != HH_OK) return bail(rc);
    *out = p;
    return HH_OK;
}

int hh_set_shift(hh_problem p, double beta1, double beta2) {
    g_err.clear();
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    if (!std::isfinite(beta1) || !std::isfinite(beta2))
        return fail(HH_EINVAL, "beta1 and beta2 must be finite");
    p->beta1 = beta1;
    p->beta2 = beta2;
    return apply_shift(p);
}

int hh_workspace_bytes(hh_problem p, int restart, size_t* bytes) {
    g_err.clear();
    if (!p || !bytes) return fail(HH_EINVAL, "NULL argument");
    if (restart < 1 || restart > kMaxRestart) return fail(HH_EINVAL, "restart must be in [1, 1024]");
    *bytes = layout(p, restart).total;
    return HH_OK;
}

int hh_destroy_problem(hh_problem p) {
    g_err.clear();
    destroy(p);
    return HH_OK;
}

int hh_num_levels(hh_problem p, int* nlevels) {
    if (!p || !nlevels) return fail(HH_EINVAL, "NULL argument");
    *nlevels = (int)p->levels.size();
    return HH_OK;
}

int hh_level_info(hh_problem p, int level, int64_t* shape2, double* spacing2) {
    if (!p || !shape2 || !spacing2) return fail(HH_EINVAL, "NULL argument");
    if (level < 0 || level >= (int)p->levels.size()) return fail(HH_EINVAL, "level out of range");
    const LevelData& L = p->levels[level];
    shape2[0] = L.nz;
    shape2[1] = L.nx;
    spacing2[0] = p->ndim == 2 ? L.hz : 0.0;
    spacing2[1] = L.hx;
    return HH_OK;
}

int hh_apply_operator(hh_problem p, int which, const void* x_dev, void* y_dev, void* stream) {
    g_err.clear();
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    CHK(check_vec_args(x_dev, "x_dev"));
    CHK(check_vec_args(y_dev, "y_dev"));
    if (x_dev == y_dev) return fail(HH_EINVAL, "x_dev and y_dev must be distinct");
    if (which != 0 && which != 1) return fail(HH_EINVAL, "which must be 0 (H) or 1 (M)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const FineOp op = which == 0 ? op_H(p) : op_M(p);
    HIPCHK(launch_fine_apply(op, static_cast<const cplx*>(x_dev), static_cast<cplx*>(y_dev), s));
    HIPCHK(hipStreamSynchronize(s));
    return HH_OK;
}

int hh_apply_level_operator(hh_problem p, int level, const void* x_dev, void* y_dev,
                            void* stream) {
    g_err.clear();
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    CHK(check_vec_args(x_dev, "x_dev"));
    CHK(check_vec_args(y_dev, "y_dev"));
    if (x_dev == y_dev) return fail(HH_EINVAL, "x_dev and y_dev must be distinct");
    if (level < 0 || level >= (int)p->levels.size()) return fail(HH_EINVAL, "level out of range");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const cplx* x = static_cast<const cplx*>(x_dev);
    cplx* y = static_cast<cplx*>(y_dev);
    if (level == 0)
        HIPCHK(launch_fine_apply(op_M(p), x, y, s));
    else
        HIPCHK(launch_coarse_apply(coarse_op(p->levels[level]), x, y, s));
    HIPCHK(hipStreamSynchronize(s));
    return HH_OK;
}

int hh_apply_precond(hh_problem p, const void* v_dev, void* z_dev, void* workspace_dev,
                     size_t workspace_bytes, void* stream) {
    g_err.clear();
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    CHK(check_vec_args(v_dev, "v_dev"));
    CHK(check_vec_args(z_dev, "z_dev"));
    CHK(check_vec_args(workspace_dev, "workspace_dev"));
    if (v_dev == z_dev) return fail(HH_EINVAL, "v_dev and z_dev must be distinct");
    const Layout L = layout(p, 1);
    if (workspace_bytes < L.total) return fail(HH_EINVAL, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    CHK(precond(p, L, workspace_dev, static_cast<const cplx*>(v_dev), static_cast<cplx*>(z_dev),
                s));
    HIPCHK(hipStreamSynchronize(s));
    return HH_OK;
}

int hh_orthogonalize_scratch_bytes(int64_t n, int k, size_t* bytes) {
    if (!bytes || n < 1 || k < 1 || k > kMaxRestart + 1) return fail(HH_EINVAL, "bad argument");
    const int nb = reduce_blocks(n);
    *bytes = align_up((size_t)nb * k * sizeof(cplx)) + 3 * align_up((size_t)k * sizeof(cplx));
    return HH_OK;
}

int hh_orthogonalize(const void* V_dev, int64_t n, int k, void* w_dev, void* scratch_dev,
                     size_t scratch_bytes, double* h_host, double* norm_host, void* stream) {
    g_err.clear();
    size_t need = 0;
    CHK(hh_orthogonalize_scratch_bytes(n, k, &need));
    if (!V_dev || !w_dev || !scratch_dev || !h_host || !norm_host)
        return fail(HH_EINVAL, "NULL argument");
    if (scratch_bytes < need) return fail(HH_EINVAL, "scratch too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nb = reduce_blocks(n);
    cplx* partial = static_cast<cplx*>(scratch_dev);
    cplx* h1 = at<cplx>(scratch_dev, align_up((size_t)nb * k * sizeof(cplx)));
    cplx* h2 = h1 + align_up((size_t)k * sizeof(cplx)) / sizeof(cplx);
    cplx* nr = h2 + align_up((size_t)k * sizeof(cplx)) / sizeof(cplx);
    const cplx* V = static_cast<const cplx*>(V_dev);
    cplx* w = static_cast<cplx*>(w_dev);
    HIPCHK(launch_dot_partials(V, n, k, w, partial, nb, s));
    HIPCHK(launch_reduce_partials(partial, nb, k, h1, s));
    HIPCHK(launch_multi_axpy(V, n, k, h1, w, s));
    HIPCHK(launch_dot_partials(V, n, k, w, partial, nb, s));
    HIPCHK(launch_reduce_partials(partial, nb, k, h2, s));
    HIPCHK(launch_multi_axpy(V, n, k, h2, w, s));
    CHK(norm2_async(w, n, partial, nb, nr, s));
    std::vector<cplx> a(k), b(k);
    cplx nrm;
    HIPCHK(hipMemcpyAsync(a.data(), h1, k * sizeof(cplx), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(b.data(), h2, k * sizeof(cplx), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&nrm, nr, sizeof(cplx), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < k; ++i) {
        h_host[2 * i] = a[i].x + b[i].x;
        h_host[2 * i + 1] = a[i].y + b[i].y;
    }
    *norm_host = std::sqrt(nrm.x);
    return HH_OK;
}

int hh_solve(hh_problem p, const void* f_dev, double tol, int restart, int max_iters,
             unsigned flags, void* workspace_dev, size_t workspace_bytes, void* u_dev,
             int* iterations, double* true_rel_res, double* hist_host, int hist_cap,
             int* hist_len, void* stream) {
    g_err.clear();
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    CHK(check_vec_args(f_dev, "f_dev"));
    CHK(check_vec_args(u_dev, "u_dev"));
    CHK(check_vec_args(workspace_dev, "workspace_dev"));
    if (!(tol > 0.0 && tol < 1.0)) return fail(HH_EINVAL, "tol must be in (0, 1)");
    if (restart < 1 || restart > kMaxRestart) return fail(HH_EINVAL, "restart must be in [1, 1024]");
    if (max_iters < 1) return fail(HH_EINVAL, "max_iters must be >= 1");
    if (flags & ~HH_NO_PRECOND) return fail(HH_EINVAL, "unknown flag");
    if (hist_cap < 0 || (hist_cap > 0 && !hist_host)) return fail(HH_EINVAL, "bad history buffer");
    if (f_dev == u_dev) return fail(HH_EINVAL, "f_dev and u_dev must be distinct");
    const int m = restart;
    const Layout L = layout(p, m);
    if (workspace_bytes < L.total) return fail(HH_EINVAL, "workspace too small");
    const bool no_prec = (flags & HH_NO_PRECOND) != 0;

    hipStream_t s = static_cast<hipStream_t>(stream);
    void* ws = workspace_dev;
    const int64_t N = p->N;
    const size_t vbytes = (size_t)N * sizeof(cplx);
    cplx* V = at<cplx>(ws, L.V);
    cplx* Z = at<cplx>(ws, L.Z);
    cplx* b = at<cplx>(ws, L.b);
    cplx* partial = at<cplx>(ws, L.partial);
    cplx* h1 = at<cplx>(ws, L.h1);
    cplx* h2 = at<cplx>(ws, L.h2);
    cplx* nrm2 = at<cplx>(ws, L.nrm2);
    cplx* R = at<cplx>(ws, L.R);
    double* cs = at<double>(ws, L.cs);
    cplx* sn = at<cplx>(ws, L.sn);
    cplx* g = at<cplx>(ws, L.g);
    cplx* y = at<cplx>(ws, L.y);
    double* inv_beta = at<double>(ws, L.inv_beta);
    GivensState* st = at<GivensState>(ws, L.st);
    cplx* u = static_cast<cplx*>(u_dev);
    const FineOp H = op_H(p);
    const int nb = L.nb;

    std::vector<double> hist;
    hist.push_back(1.0);
    int it = 0;
    int status = HH_OK;
    double rel = 0.0;
    auto finish = [&](int code) {
        if (iterations) *iterations = it;
        if (true_rel_res) *true_rel_res = rel;
        if (hist_len) *hist_len = (int)hist.size();
        for (int i = 0; i < (int)hist.size() && i < hist_cap; ++i) hist_host[i] = hist[i];
        return code;
    };

    HIPCHK(launch_weight_rhs(H, static_cast<const cplx*>(f_dev), b, s));
    CHK(norm2_async(b, N, partial, nb, nrm2, s));
    HIPCHK(hipMemcpyAsync(p->nrm2_host, nrm2, sizeof(cplx), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemsetAsync(u, 0, vbytes, s));
    HIPCHK(hipStreamSynchronize(s));
    const double beta0 = std::sqrt(p->nrm2_host->x);
    if (!std::isfinite(beta0)) return finish(fail(HH_ENUMERIC, "source is not finite"));
    if (beta0 == 0.0) return finish(HH_OK);

    for (;;) {
        // true residual r = b - H u into v_1
        HIPCHK(launch_fine_residual(H, b, u, V, s));
        CHK(norm2_async(V, N, partial, nb, nrm2, s));
        HIPCHK(hipMemcpyAsync(p->nrm2_host, nrm2, sizeof(cplx), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        CHK(kt_harvest(p));
        const double beta = std::sqrt(p->nrm2_host->x);
        rel = beta / beta0;
        if (!std::isfinite(rel)) return finish(fail(HH_ENUMERIC, "residual is not finite"));
        if (rel <= tol) return finish(HH_OK);
        if (it >= max_iters) return finish(HH_NOT_CONVERGED);
        HIPCHK(launch_cycle_init(st, m, beta0, nrm2, g, inv_beta, s));
        HIPCHK(launch_scale_dev(V, inv_beta, V, N, s));
        int k = 0;
        for (int j = 0; j < m; ++j) {
            cplx* vj = V + (size_t)j * N;
            cplx* w = V + (size_t)(j + 1) * N;
            const cplx* zj = vj;
            if (!no_prec) {
                cplx* zz = Z + (size_t)j * N;
                CHK(precond(p, L, ws, vj, zz, s));
                zj = zz;
            }
            TIMED(HH_KERNEL_STENCIL, 40.0 * (double)N, launch_fine_apply(H, zj, w, s));
            // CGS2 against v_1..v_{j+1}
            const int kk = j + 1;
            const double dot_bytes = (kk + 1) * 16.0 * (double)N;
            const double axpy_bytes = (kk + 2) * 16.0 * (double)N;
            TIMED(HH_KERNEL_DOT, dot_bytes, launch_dot_partials(V, N, kk, w, partial, nb, s));
            HIPCHK(launch_reduce_partials(partial, nb, kk, h1, s));
            TIMED(HH_KERNEL_AXPY, axpy_bytes, launch_multi_axpy(V, N, kk, h1, w, s));
            TIMED(HH_KERNEL_DOT, dot_bytes, launch_dot_partials(V, N, kk, w, partial, nb, s));
            HIPCHK(launch_reduce_partials(partial, nb, kk, h2, s));
            TIMED(HH_KERNEL_AXPY, axpy_bytes, launch_multi_axpy(V, N, kk, h2, w, s));
            CHK(norm2_async(w, N, partial, nb, nrm2, s));
            HIPCHK(launch_givens(st, h1, h2, nrm2, R, cs, sn, g, s));
            HIPCHK(launch_scale_dev(w, &st->inv_hn, w, N, s));
            HIPCHK(hipMemcpyAsync(p->st_host, st, sizeof(GivensState), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            CHK(kt_harvest(p));
            ++it;
            const GivensState gs = *p->st_host;
            hist.push_back(gs.est);
            k = j + 1;
            if (gs.bad) {
                rel = NAN;
                return finish(fail(HH_ENUMERIC, "non-finite value in the Arnoldi step"));
            }
            if (gs.breakdown || gs.est <= tol || it >= max_iters) break;
        }
        HIPCHK(launch_backsub(k, m, R, g, y, s));
        HIPCHK(launch_update_x(no_prec ? V : Z, N, k, y, u, s));
    }
    return finish(status);
}

int hh_kernel_timer_start(hh_problem p, int kernel_id) {
    g_err.clear();
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    if (kernel_id < HH_KERNEL_NONE || kernel_id > HH_KERNEL_PCR)
        return fail(HH_EINVAL, "unknown kernel id");
    p->kt.kid = kernel_id;
    p->kt.used = 0;
    p->kt.pending_bytes.clear();
    p->kt.launches = 0;
    p->kt.total_ms = 0.0;
    p->kt.total_bytes = 0.0;
    return HH_OK;
}

int hh_kernel_timer_read(hh_problem p, int64_t* launches, double* total_ms,
                         double* total_bytes) {
    g_err.clear();
    if (!p || !launches || !total_ms || !total_bytes) return fail(HH_EINVAL, "NULL argument");
    *launches = p->kt.launches;
    *total_ms = p->kt.total_ms;
    *total_bytes = p->kt.total_bytes;
    return HH_OK;
}

}  // extern "C"
