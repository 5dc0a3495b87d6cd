// C ABI of the solver (include/helmholtz.h): problem set-up, the
// shifted-Laplace preconditioner hierarchy, and the right-preconditioned
// flexible GMRES driver (Eq. 5-7).
//
// Control flow of a solve lives on the device: the Givens kernel decides when
// a restart cycle stops, the cycle-start kernel decides when the solve is
// done, and every Arnoldi-step kernel returns at once when its cycle is
// closed. The host enqueues work a bounded number of steps ahead and paces
// itself on a progress record that the device writes into pinned host memory;
// it never waits on the stream inside the iteration.
#include "helmholtz.h"
#include "givens.h"

#include <immintrin.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace hh {
thread_local LaunchEvents g_launch_events;
}

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

constexpr double kJacobiWeight = 0.8;         // resolved levels
constexpr double kJacobiWeightCoarse = 0.5;   // levels with omega*max(m)*max(h) >= kKhSmooth
constexpr double kKhSmooth = 2.0;
constexpr int kMaxRestart = 1024;
constexpr int kLookahead = 2;          // Arnoldi steps enqueued ahead of the device
constexpr double kStallSeconds = 120.0;

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct LevelData {
    int nz = 0, nx = 0;
    double hz = 0, hx = 0;
    int halve_z = 0, halve_x = 0;   // halving flags towards the next coarser level
    double wj = kJacobiWeight;      // Jacobi weight of this level's smoother
    cplx* C = nullptr;              // 9-point Galerkin operator (levels >= 1)
    cplx* wd = nullptr;             // wj / diag per node (smoothing levels)
    cplxf* Cf = nullptr;            // the same, rounded to complex64
    cplxf* wdf = nullptr;
    int tile_down = -1;             // tile shapes of this level's legs (HH_TILE_*, -1: default)
    int tile_up = -1;
    int64_t size() const { return (int64_t)nz * nx; }
};

struct PendingTime {
    int cycle, j;                   // Arnoldi step that made the launch
    double bytes;                   // per working right-hand side
    double shared;                  // once per launch (operator data read for all of them)
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
    float* m2f = nullptr;           // m^2 rounded to float (single-precision preconditioner)
    std::vector<LevelData> levels;
    cplx* cinv = nullptr;           // explicit inverse of the coarsest operator
    cplxf* cinvf = nullptr;         // ... rounded to complex64
    cplx* pcr = nullptr;            // 1D: reduction multipliers of M (pcr_factor_elems)
    cplxf* pcrf = nullptr;          // ... of the complex64 operator
    int nc = 0;
    int max_coarse = HH_MAX_COARSE; // largest coarsest grid inverted densely
    void* band = nullptr;           // banded LU scratch of the coarsest inverse
    void* gemm_part = nullptr;      // partial sums of the batched coarsest product
    size_t gemm_part_bytes = 0;
    int* dflag = nullptr;           // device scratch for checks
    double* dpartial = nullptr;
    cplx* nrm2_host = nullptr;      // pinned
    HostRecord* rec = nullptr;      // pinned, written by the device (one per right-hand side)
    int rec_cap = 0;
    double* hist = nullptr;         // pinned, written by the device
    int64_t hist_cap = 0;           // entries
    int64_t hist_stride = 0;        // entries per right-hand side
    hipStream_t stream = nullptr;
    // dispatch-stamped timing of one kernel class (hh_kernel_timer_*)
    struct {
        int kid = HH_KERNEL_NONE;
        std::vector<hipEvent_t> pool;
        std::vector<PendingTime> pending;
        int64_t launches = 0;
        double total_ms = 0.0, total_bytes = 0.0;
        int cycle = 0, j = 0;       // step being enqueued
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
    op.wdinv = nullptr;
    return op;
}
FineOp op_H(const hh_problem_s* p) { return fine_op(p, 1.0, -p->alpha); }
FineOp op_M(const hh_problem_s* p) {
    FineOp op = fine_op(p, p->beta1, -p->beta2);
    op.wdinv = p->levels.empty() ? nullptr : p->levels[0].wd;
    return op;
}
CoarseOp coarse_op(const LevelData& L) {
    CoarseOp op;
    op.nz = L.nz;
    op.nx = L.nx;
    op.C = L.C;
    op.wdinv = L.wd;
    return op;
}

// The preconditioner in complex64: the same operator with its parameters,
// m^2, smoother weights, Galerkin planes and coarsest inverse rounded to
// single precision (the double-precision set-up is done first).
FineOpT<float> op_Mf(const hh_problem_s* p) {
    const FineOp d = op_M(p);
    FineOpT<float> op;
    op.nz = d.nz;
    op.nx = d.nx;
    op.ndim = d.ndim;
    op.ihx2 = (float)d.ihx2;
    op.ihz2 = (float)d.ihz2;
    op.ihx = (float)d.ihx;
    op.ihz = (float)d.ihz;
    op.omega = (float)d.omega;
    op.omega2 = (float)d.omega2;
    op.sr = (float)d.sr;
    op.si = (float)d.si;
    op.m2 = p->m2f;
    op.wdinv = p->levels.empty() ? nullptr : p->levels[0].wdf;
    return op;
}
CoarseOpT<float> coarse_opf(const LevelData& L) {
    CoarseOpT<float> op;
    op.nz = L.nz;
    op.nx = L.nx;
    op.C = L.Cf;
    op.wdinv = L.wdf;
    return op;
}

// precision-generic access to the preconditioner's data
template <class T> struct Prec;
template <> struct Prec<double> {
    static FineOp fine(const hh_problem_s* p) { return op_M(p); }
    static CoarseOp coarse(const LevelData& L) { return coarse_op(L); }
    static const cplx* cinv(const hh_problem_s* p) { return p->cinv; }
    static const cplx* pcr(const hh_problem_s* p) { return p->pcr; }
};
template <> struct Prec<float> {
    static FineOpT<float> fine(const hh_problem_s* p) { return op_Mf(p); }
    static CoarseOpT<float> coarse(const LevelData& L) { return coarse_opf(L); }
    static const cplxf* cinv(const hh_problem_s* p) { return p->cinvf; }
    static const cplxf* pcr(const hh_problem_s* p) { return p->pcrf; }
};

// ---------------------------------------------------------------------------
// kernel timer
// ---------------------------------------------------------------------------
bool kt_arm(hh_problem_s* p, int kid) {
    if (p->kt.kid == HH_KERNEL_NONE || p->kt.kid != kid) return false;
    const size_t used = 2 * p->kt.pending.size();
    while (p->kt.pool.size() < used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return false;
        p->kt.pool.push_back(e);
    }
    g_launch_events.start = p->kt.pool[used];
    g_launch_events.stop = p->kt.pool[used + 1];
    return true;
}

void kt_done(hh_problem_s* p, double bytes, double shared) {
    p->kt.pending.push_back(PendingTime{p->kt.cycle, p->kt.j, bytes, shared});
}

// After the stream is idle: keep the launches of steps that did work, with
// the byte model times the number of right-hand sides that did the step
// (executed[c][b] = steps right-hand side b took in cycle c + 1).
int kt_harvest(hh_problem_s* p, const std::vector<std::vector<int>>& executed) {
    for (size_t i = 0; i < p->kt.pending.size(); ++i) {
        const PendingTime& t = p->kt.pending[i];
        int working = 0;
        if (t.cycle >= 1 && t.cycle <= (int)executed.size())
            for (int e : executed[t.cycle - 1]) working += t.j < e;
        if (working == 0) continue;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, p->kt.pool[2 * i], p->kt.pool[2 * i + 1]));
        p->kt.total_ms += ms;
        p->kt.total_bytes += t.bytes * working + t.shared;
        p->kt.launches += 1;
    }
    p->kt.pending.clear();
    return HH_OK;
}

// Launch EXPR; when kernel class KID is being timed, stamp it and record its
// algorithmic bytes: BYTES per right-hand side that did the step, SHARED once.
#define TIMED2(KID, BYTES, SHARED, EXPR)                             \
    do {                                                             \
        const bool armed_ = kt_arm(p, (KID));                        \
        const hipError_t e2_ = (EXPR);                               \
        g_launch_events = LaunchEvents();                            \
        HIPCHK(e2_);                                                 \
        if (armed_) kt_done(p, (double)(BYTES), (double)(SHARED));   \
    } while (0)
#define TIMED(KID, BYTES, EXPR) TIMED2(KID, BYTES, 0.0, EXPR)



// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
struct Layout {
    size_t V, Z, b, w, partial, h1, h2, R, cs, sn, g, y, zs, st, total;
    std::vector<size_t> t, bc, ec;   // per level
    int nbA, nbN, nbR, nbmax;   // partials of apply_dot, node kernels, the residual norm
};

// es: bytes per complex value of Z and the V-cycle vectors (16, or 8 when
// the preconditioner runs in complex64; the 16-byte layout is the larger).
Layout layout(const hh_problem_s* p, int m, size_t es = sizeof(cplx)) {
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
    L.Z = take((size_t)m * N * es);
    L.b = take(N * c);
    L.w = take(N * c);
    const int nl = (int)p->levels.size();
    L.t.assign(nl, 0);
    L.bc.assign(nl, 0);
    L.ec.assign(nl, 0);
    if (p->ndim == 2) {
        for (int l = 0; l < nl; ++l) {
            const size_t n = (size_t)p->levels[l].size();
            if (l < nl - 1) L.t[l] = take(n * es);
            if (l >= 1) {
                L.bc[l] = take(n * es);
                L.ec[l] = take(n * es);
            }
        }
    }
    L.nbA = apply_blocks(op_H(p), 1);   // a batch resets it (solve_impl)
    L.nbN = node_blocks(p->N);
    L.nbR = residual_blocks(op_H(p));
    L.nbmax = std::max(std::max(L.nbA, L.nbN), L.nbR);
    L.partial = take((size_t)L.nbmax * 2 * (m + 1) * c);
    L.h1 = take((size_t)2 * (m + 1) * c);
    L.h2 = take((size_t)(m + 1) * c);
    L.R = take((size_t)(m + 1) * m * c);
    L.cs = take((size_t)m * sizeof(double));
    L.sn = take((size_t)m * c);
    L.g = take((size_t)(m + 1) * c);
    L.y = take((size_t)m * c);
    L.zs = take((size_t)m * sizeof(double));
    L.st = take(sizeof(SolveState));
    L.total = off;
    return L;
}

template <class T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// ---------------------------------------------------------------------------
// preconditioner
// ---------------------------------------------------------------------------
// Grid of level l >= 1 as the legs of level l - 1 see it: the vectors of the
// coarsest level are in the band numbering of its inverse.
CGrid coarse_grid(const hh_problem_s* p, int l) {
    const LevelData& lv = p->levels[l];
    const bool last = l + 1 == (int)p->levels.size();
    return CGrid{lv.nz, lv.nx, last && band_renumbered(lv.nz, lv.nx) ? 1 : 0};
}

// One V(2,2) cycle on level l >= 1: ec_l = V(l, bc_l), one kernel per leg,
// in precision T, for every right-hand side of the batch.
template <class T>
int vcycle_coarse(hh_problem_s* p, const Layout& L, void* ws, int l, const int* active,
                  hipStream_t s, const Batch& bt) {
    typedef typename Cx<T>::type C;
    const double es = (double)sizeof(C);
    const int nl = (int)p->levels.size();
    C* b = at<C>(ws, L.bc[l]);
    C* x = at<C>(ws, L.ec[l]);
    if (l == nl - 1) {
        const double nc = p->nc;
        if (bt.n > 1)
            TIMED2(HH_KERNEL_GEMV, 2 * nc * es, nc * nc * es * ((bt.n + 31) / 32),
                   launch_vc_gemm(p->nc, Prec<T>::cinv(p), b, x, p->gemm_part, s, bt));
        else
            TIMED2(HH_KERNEL_GEMV, 2 * nc * es, nc * nc * es,
                   launch_vc_gemv(p->nc, Prec<T>::cinv(p), b, x, active, s, bt));
        return HH_OK;
    }
    const LevelData& lv = p->levels[l];
    const LevelData& nx = p->levels[l + 1];
    const auto A = Prec<T>::coarse(lv);
    C* x2 = at<C>(ws, L.t[l]);
    const double nl_ = (double)lv.size(), nn_ = (double)nx.size();
    // down: b in, x2 out, the coarser right-hand side out; up: x2, b in, x out,
    // the coarser correction in; both read the 9 coefficients and omega/diag
    TIMED2(HH_KERNEL_VC_DOWN_COARSE, 2.0 * es * nl_ + es * nn_, 10.0 * es * nl_,
           launch_vc_coarse_down(A, b, x2, lv.halve_z, lv.halve_x, coarse_grid(p, l + 1),
                                 at<C>(ws, L.bc[l + 1]), active, s, bt, lv.tile_down));
    CHK(vcycle_coarse<T>(p, L, ws, l + 1, active, s, bt));
    TIMED2(HH_KERNEL_VC_UP_COARSE, 3.0 * es * nl_ + es * nn_, 10.0 * es * nl_,
           launch_vc_coarse_up(A, lv.halve_z, lv.halve_x, b, x2, at<C>(ws, L.ec[l + 1]),
                               coarse_grid(p, l + 1), x, active, s, bt, lv.tile_up));
    return HH_OK;
}

// z = M^{-1} v in precision T (v stays complex128), for every right-hand side
// of the batch; every kernel is predicated on *active (NULL: unconditional).
template <class T>
int precond(hh_problem_s* p, const Layout& L, void* ws, const cplx* src, const int* active,
            typename Cx<T>::type* z, hipStream_t s, const Batch& bt = Batch()) {
    typedef typename Cx<T>::type C;
    const double es = (double)sizeof(C), rs = (double)sizeof(T);
    const double N = (double)p->N;
    const auto M = Prec<T>::fine(p);
    if (p->ndim == 1) {
        // v in, z out; m^2 shared
        TIMED2(HH_KERNEL_PCR, (16.0 + es) * N, rs * N,
               launch_pcr((int)p->N, Prec<T>::pcr(p), src, z, active, s, bt));
        return HH_OK;
    }
    const int nl = (int)p->levels.size();
    if (nl == 1) {   // the fine grid is the coarsest: dense inverse only
        const double nc = p->nc;
        TIMED2(HH_KERNEL_GEMV, 2 * nc * es, nc * nc * es,
               launch_vc_gemv(p->nc, Prec<T>::cinv(p), src, z, active, s, bt));
        return HH_OK;
    }
    const LevelData& lv = p->levels[0];
    const LevelData& nx = p->levels[1];
    C* x2 = at<C>(ws, L.t[0]);
    const double N1 = (double)nx.size();
    // down: v in (complex128), x2 out, the coarse right-hand side out; up: v in,
    // x2 in, z out, the coarse correction in; both read m^2 and omega/diag
    // (shared by the right-hand sides)
    TIMED2(HH_KERNEL_VC_DOWN, (16.0 + es) * N + es * N1, (rs + es) * N,
           launch_vc_fine_down(M, src, x2, lv.halve_z, lv.halve_x, coarse_grid(p, 1),
                               at<C>(ws, L.bc[1]), active, s, bt, lv.tile_down));
    CHK(vcycle_coarse<T>(p, L, ws, 1, active, s, bt));
    TIMED2(HH_KERNEL_VC_UP, (16.0 + 2.0 * es) * N + es * N1, (rs + es) * N,
           launch_vc_fine_up(M, lv.halve_z, lv.halve_x, src, x2, at<C>(ws, L.ec[1]),
                             coarse_grid(p, 1), z, active, s, bt, lv.tile_up));
    return HH_OK;
}

// ---------------------------------------------------------------------------
// tile autotuner
// ---------------------------------------------------------------------------
// Launch configuration to keep: -1 (the default) unless one of 0 .. count-1
// runs more than 3% faster than it (a margin above the timing noise, so that
// the choice departs from the default only for a clear gain). Each runs once
// to warm up, then three times `reps` back-to-back launches between two
// events; the shortest of the three counts.
template <class F>
int fastest(F&& launch, int count, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
            int* best) {
    float best_ms = 0.0f;
    *best = -1;
    for (int c = -1; c < count; ++c) {
        HIPCHK(launch(c));
        float tmin = 0.0f;
        for (int trial = 0; trial < 3; ++trial) {
            HIPCHK(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) HIPCHK(launch(c));
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (trial == 0 || ms < tmin) tmin = ms;
        }
        if (c == -1 || tmin < 0.97f * best_ms) {
            best_ms = tmin;
            *best = c;
        }
    }
    return HH_OK;
}

// Times every tile shape of the down and up legs of levels 0 .. nl-2 in
// precision T on the workspace's own vectors (inputs zero, every kernel
// unconditional) and keeps per leg the choice of fastest() in the level data.
template <class T>
int tune_legs(hh_problem_s* p, const Layout& L, void* ws, int reps, hipStream_t s,
              const Batch& bt, hipEvent_t e0, hipEvent_t e1) {
    typedef typename Cx<T>::type C;
    const int nl = (int)p->levels.size();
    const cplx* src = at<cplx>(ws, L.V);
    C* z = at<C>(ws, L.Z);
    for (int l = 0; l + 1 < nl; ++l) {
        LevelData& lv = p->levels[l];
        const CGrid cg = coarse_grid(p, l + 1);
        C* x2 = at<C>(ws, L.t[l]);
        C* bcn = at<C>(ws, L.bc[l + 1]);
        C* ecn = at<C>(ws, L.ec[l + 1]);
        auto down = [&](int tile) -> hipError_t {
            if (l == 0)
                return launch_vc_fine_down(Prec<T>::fine(p), src, x2, lv.halve_z, lv.halve_x, cg,
                                           bcn, nullptr, s, bt, tile);
            return launch_vc_coarse_down(Prec<T>::coarse(lv), at<C>(ws, L.bc[l]), x2, lv.halve_z,
                                         lv.halve_x, cg, bcn, nullptr, s, bt, tile);
        };
        auto up = [&](int tile) -> hipError_t {
            if (l == 0)
                return launch_vc_fine_up(Prec<T>::fine(p), lv.halve_z, lv.halve_x, src, x2, ecn,
                                         cg, z, nullptr, s, bt, tile);
            return launch_vc_coarse_up(Prec<T>::coarse(lv), lv.halve_z, lv.halve_x,
                                       at<C>(ws, L.bc[l]), x2, ecn, cg, at<C>(ws, L.ec[l]),
                                       nullptr, s, bt, tile);
        };
        int best = 0;
        CHK(fastest(down, HH_TILE_DOWN_COUNT, reps, s, e0, e1, &best));
        lv.tile_down = best;
        CHK(fastest(up, HH_TILE_UP_COUNT, reps, s, e0, e1, &best));
        lv.tile_up = best;
    }
    return HH_OK;
}

// ---------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------
// releases the level operators and the coarsest-level data
void free_levels(hh_problem_s* p) {
    for (auto& l : p->levels) {
        if (l.C) (void)hipFree(l.C);
        if (l.wd) (void)hipFree(l.wd);
        if (l.Cf) (void)hipFree(l.Cf);
        if (l.wdf) (void)hipFree(l.wdf);
        l.C = nullptr;
        l.wd = nullptr;
        l.Cf = nullptr;
        l.wdf = nullptr;
    }
    p->levels.clear();
    if (p->cinv) (void)hipFree(p->cinv);
    if (p->cinvf) (void)hipFree(p->cinvf);
    if (p->pcr) (void)hipFree(p->pcr);
    if (p->pcrf) (void)hipFree(p->pcrf);
    if (p->band) (void)hipFree(p->band);
    p->cinv = nullptr;
    p->cinvf = nullptr;
    p->pcr = nullptr;
    p->pcrf = nullptr;
    p->band = nullptr;
}


// Level grids, spacings, halving flags and smoother weights (host only; no
// device memory). EUNSUPPORTED when the coarsest grid exceeds the dense limit.
int plan_levels(hh_problem_s* p) {
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
        cur.wj = kmax * std::fmax(cur.hz, cur.hx) < kKhSmooth ? kJacobiWeight : kJacobiWeightCoarse;
        // keep two nodes per shortest wavelength, unless the grid is still too
        // large for the direct coarsest solve
        const bool big = cur.size() > p->max_coarse;
        auto halves = [&](int n, double h) {
            return (n - 1) % 2 == 0 && (n - 1) / 2 >= 2 && (kmax * 2.0 * h <= M_PI || big);
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
    if (nc > p->max_coarse)
        return fail(HH_EUNSUPPORTED,
                    "coarsest multigrid grid has " + std::to_string(nc) +
                        " unknowns (more than the dense limit " +
                        std::to_string(p->max_coarse) + ")");
    p->nc = (int)nc;
    return HH_OK;
}

// Device bytes the handle owns for its operators (levels, coarsest inverse
// and the band factorisation scratch, m^2 in both precisions),
// from a planned hierarchy.
size_t problem_bytes(const hh_problem_s* p) {
    size_t b = align_up((size_t)p->N * (sizeof(double) + sizeof(float))) + align_up(sizeof(int)) +
               align_up(4096 * sizeof(cplx));
    const size_t nl = p->levels.size();
    for (size_t l = 0; l < nl; ++l) {
        const size_t n = (size_t)p->levels[l].size();
        if (l >= 1) b += align_up(9 * n * sizeof(cplx)) + align_up(9 * n * sizeof(cplxf));
        if (l + 1 < nl) b += align_up(n * sizeof(cplx)) + align_up(n * sizeof(cplxf));
    }
    if (p->ndim == 2) {
        const size_t nc = (size_t)p->nc;
        const LevelData& lc = p->levels.back();
        b += align_up(nc * nc * sizeof(cplx)) + align_up(nc * nc * sizeof(cplxf)) +
             align_up(band_scratch_bytes(lc.nz, lc.nx));
    } else {
        const size_t e = pcr_factor_elems((int)p->N);
        b += align_up(e * sizeof(cplx)) + align_up(e * sizeof(cplxf));
    }
    return b;
}

int build_hierarchy(hh_problem_s* p) {
    free_levels(p);
    CHK(plan_levels(p));
    const int64_t nc = p->nc;
    if (p->ndim == 1) {
        const size_t e = pcr_factor_elems((int)p->N);
        HIPCHK(hipMalloc(&p->pcr, e * sizeof(cplx)));
        HIPCHK(hipMalloc(&p->pcrf, e * sizeof(cplxf)));
        return HH_OK;
    }
    for (size_t l = 1; l < p->levels.size(); ++l) {
        HIPCHK(hipMalloc(&p->levels[l].C, 9 * (size_t)p->levels[l].size() * sizeof(cplx)));
        HIPCHK(hipMalloc(&p->levels[l].Cf, 9 * (size_t)p->levels[l].size() * sizeof(cplxf)));
    }
    for (size_t l = 0; l + 1 < p->levels.size(); ++l) {
        HIPCHK(hipMalloc(&p->levels[l].wd, (size_t)p->levels[l].size() * sizeof(cplx)));
        HIPCHK(hipMalloc(&p->levels[l].wdf, (size_t)p->levels[l].size() * sizeof(cplxf)));
    }
    HIPCHK(hipMalloc(&p->cinv, (size_t)nc * nc * sizeof(cplx)));
    HIPCHK(hipMalloc(&p->cinvf, (size_t)nc * nc * sizeof(cplxf)));
    const LevelData& lc = p->levels.back();
    HIPCHK(hipMalloc(&p->band, band_scratch_bytes(lc.nz, lc.nx)));
    return HH_OK;
}

int apply_shift(hh_problem_s* p) {
    hipStream_t s = p->stream;
    if (p->ndim == 1) {                 // the reduction multipliers of M in both precisions
        HIPCHK(launch_pcr_factor(op_M(p), p->pcr, s));
        HIPCHK(launch_pcr_factor(op_Mf(p), p->pcrf, s));
        HIPCHK(hipStreamSynchronize(s));
        return HH_OK;
    }
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
    for (int l = 0; l + 1 < nl; ++l) {
        const LevelData& lv = p->levels[l];
        if (l == 0)
            HIPCHK(launch_wdinv_fine(op_M(p), lv.wj, lv.wd, s));
        else
            HIPCHK(launch_wdinv_coarse(coarse_op(lv), lv.wj, lv.wd, s));
    }
    if (nl == 1)
        HIPCHK(launch_dense_from_fine(M, p->cinv, s));
    else
        HIPCHK(launch_dense_from_coarse(coarse_op(p->levels.back()), p->cinv, s));
    // explicit inverse from a banded LU (the coarsest operator is a stencil); with
    // a coarser level the inverse stays in the band numbering, and the legs of the
    // level above read and write the coarsest vectors in that numbering
    const LevelData& lc = p->levels.back();
    HIPCHK(hipMemsetAsync(p->dflag, 0, sizeof(int), s));
    HIPCHK(band_invert(lc.nz, lc.nx, p->cinv, p->band, p->dflag, nl == 1, s));
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, p->dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad) return fail(HH_ENUMERIC, "coarsest-level operator is singular for this shift");
    const int64_t nn = (int64_t)p->nc * p->nc;
    // complex64 copies for the single-precision preconditioner
    for (int l = 0; l < nl; ++l) {
        const LevelData& lv = p->levels[l];
        if (lv.C) HIPCHK(launch_to_c64(lv.C, lv.Cf, 9 * lv.size(), s));
        if (lv.wd) HIPCHK(launch_to_c64(lv.wd, lv.wdf, lv.size(), s));
    }
    HIPCHK(launch_to_c64(p->cinv, p->cinvf, nn, s));
    HIPCHK(hipStreamSynchronize(s));
    return HH_OK;
}

void destroy(hh_problem_s* p) {
    if (!p) return;
    free_levels(p);
    if (p->m2) (void)hipFree(p->m2);
    if (p->m2f) (void)hipFree(p->m2f);
    if (p->gemm_part) (void)hipFree(p->gemm_part);
    if (p->dflag) (void)hipFree(p->dflag);
    if (p->dpartial) (void)hipFree(p->dpartial);
    if (p->nrm2_host) (void)hipHostFree(p->nrm2_host);
    if (p->rec) (void)hipHostFree(p->rec);
    if (p->hist) (void)hipHostFree(p->hist);
    for (hipEvent_t e : p->kt.pool) (void)hipEventDestroy(e);
    delete p;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_ptr(const void* a, const char* name) {
    if (!a) return fail(HH_EINVAL, std::string(name) + " is NULL");
    return HH_OK;
}

// pinned, device-visible memory written by kernels and polled by the host:
// one progress record and one history of max_iters + 1 entries per right-hand side
int ensure_host_buffers(hh_problem_s* p, int max_iters, int nrhs) {
    if (p->rec_cap < nrhs) {
        if (p->rec) HIPCHK(hipHostFree(p->rec));
        p->rec = nullptr;
        p->rec_cap = 0;
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&p->rec), (size_t)nrhs * sizeof(HostRecord),
                             hipHostMallocCoherent | hipHostMallocMapped));
        p->rec_cap = nrhs;
    }
    const int64_t per = max_iters + 1 > 1024 ? max_iters + 1 : 1024;
    if (p->hist_cap < per * nrhs) {
        if (p->hist) HIPCHK(hipHostFree(p->hist));
        p->hist = nullptr;
        p->hist_cap = 0;
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&p->hist),
                             (size_t)(per * nrhs) * sizeof(double),
                             hipHostMallocCoherent | hipHostMallocMapped));
        p->hist_cap = per * nrhs;
    }
    p->hist_stride = per;
    return HH_OK;
}

// ---------------------------------------------------------------------------
// host pacing on the device-written record
// ---------------------------------------------------------------------------
struct RecView {
    int done, cycles, jstep, stops;
};

RecView read_rec(const HostRecord* r) {
    const volatile HostRecord* v = r;
    RecView o;
    o.stops = v->stops;
    o.done = v->done;
    o.cycles = v->cycles;
    _mm_lfence();
    o.jstep = v->jstep;
    return o;
}

// Spin until pred holds for the record of every right-hand side; fails when
// the stream drained without it (lost progress), on a stream error, or after
// kStallSeconds.
template <class Pred>
int wait_for(const hh_problem_s* p, int nrhs, hipStream_t s, Pred pred) {
    auto all = [&]() {
        for (int b = 0; b < nrhs; ++b)
            if (!pred(read_rec(p->rec + b))) return false;
        return true;
    };
    auto t0 = std::chrono::steady_clock::now();
    for (unsigned spin = 0;; ++spin) {
        if (all()) return HH_OK;
        if ((spin & 1023) == 1023) {
            const hipError_t q = hipStreamQuery(s);
            if (q == hipSuccess) {
                if (all()) return HH_OK;
                return fail(HH_EDEVICE, "device stopped without reaching the awaited state");
            }
            if (q != hipErrorNotReady)
                return fail(HH_EDEVICE, std::string("stream error: ") + hipGetErrorString(q));
            const double el =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (el > kStallSeconds) return fail(HH_EDEVICE, "no progress for too long");
        }
        _mm_pause();
    }
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
    return hh_create_problem_ex(m_dev, ndim, shape, omega, alpha, h, HH_MAX_COARSE, stream, out);
}

int hh_create_problem_ex(const double* m_dev, int ndim, const int64_t* shape, double omega,
                         double alpha, double h, int max_coarse, void* stream, hh_problem* out) {
    g_err.clear();
    if (max_coarse < 1 || max_coarse > HH_MAX_COARSE_LIMIT)
        return fail(HH_EINVAL, "max_coarse must be in [1, HH_MAX_COARSE_LIMIT]");
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
    if (ndim == 2 && shape[0] * shape[1] > (int64_t(1) << 31))
        return fail(HH_EUNSUPPORTED, "grids are limited to 2^31 nodes");
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
    p->max_coarse = max_coarse;
    auto bail = [&](int code) {
        destroy(p);
        return code;
    };
    int nb = (int)((p->N + 2047) / 2048);
    if (nb > 512) nb = 512;
    hipError_t e;
    if ((e = hipMalloc(&p->m2, p->N * sizeof(double))) != hipSuccess ||

        (e = hipMalloc(&p->m2f, p->N * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&p->dflag, sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&p->dpartial, 4096 * sizeof(cplx))) != hipSuccess ||
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
        (e = launch_to_f32(p->m2, p->m2f, p->N, s)) != hipSuccess ||
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

int hh_footprint_bytes(int ndim, const int64_t* shape, double omega, double max_slowness,
                       double h, int max_coarse, int restart, int nrhs, unsigned flags,
                       size_t* problem_b, size_t* workspace_b) {
    g_err.clear();
    if (!shape || !problem_b || !workspace_b) return fail(HH_EINVAL, "NULL argument");
    if (ndim != 1 && ndim != 2) return fail(HH_EINVAL, "ndim must be 1 or 2");
    for (int d = 0; d < ndim; ++d)
        if (shape[d] < 3 || shape[d] > (1 << 24))
            return fail(HH_EINVAL, "every grid dimension must be in [3, 2^24]");
    if (!finite_pos(omega) || !finite_pos(max_slowness) || !finite_pos(h))
        return fail(HH_EINVAL, "omega, max_slowness and h must be finite and > 0");
    if (max_coarse < 1 || max_coarse > HH_MAX_COARSE_LIMIT)
        return fail(HH_EINVAL, "max_coarse must be in [1, HH_MAX_COARSE_LIMIT]");
    if (restart < 1 || restart > kMaxRestart) return fail(HH_EINVAL, "restart must be in [1, 1024]");
    if (nrhs < 1 || nrhs > HH_MAX_BATCH) return fail(HH_EINVAL, "nrhs must be in [1, HH_MAX_BATCH]");
    if (flags & ~(HH_NO_PRECOND | HH_PRECOND_F32 | HH_INITIAL_GUESS))
        return fail(HH_EINVAL, "unknown flag");
    hh_problem_s q;                 // host-side plan only: nothing is allocated
    q.ndim = ndim;
    q.nz = ndim == 2 ? (int)shape[0] : 1;
    q.nx = ndim == 2 ? (int)shape[1] : (int)shape[0];
    q.N = (int64_t)q.nz * q.nx;
    q.omega = omega;
    q.h = h;
    q.mmax = max_slowness;
    q.max_coarse = max_coarse;
    CHK(plan_levels(&q));
    *problem_b = problem_bytes(&q);
    *workspace_b = (size_t)nrhs * layout(&q, restart).total;
    if (nrhs > 1 && ndim == 2 && q.levels.size() >= 2)
        *workspace_b += align_up(vc_gemm_scratch_bytes(q.nc, nrhs));
    return HH_OK;
}

int hh_set_max_coarse(hh_problem p, int max_coarse) {
    g_err.clear();
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    if (max_coarse < 1 || max_coarse > HH_MAX_COARSE_LIMIT)
        return fail(HH_EINVAL, "max_coarse must be in [1, HH_MAX_COARSE_LIMIT]");
    if (p->ndim != 2) return fail(HH_EINVAL, "the dense coarsest limit applies to 2D problems");
    const int old = p->max_coarse;
    p->max_coarse = max_coarse;
    int rc = build_hierarchy(p);
    if (rc == HH_OK) rc = apply_shift(p);
    if (rc != HH_OK) {   // restore a working hierarchy with the previous limit
        const std::string why = g_err;
        p->max_coarse = old;
        if (build_hierarchy(p) == HH_OK) (void)apply_shift(p);
        g_err = why;
    }
    return rc;
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

int hh_autotune(hh_problem p, unsigned flags, int nrhs, void* workspace_dev,
                size_t workspace_bytes, int reps, void* stream) {
    g_err.clear();
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    CHK(check_ptr(workspace_dev, "workspace_dev"));
    if (flags & ~HH_PRECOND_F32) return fail(HH_EINVAL, "flags must be 0 or HH_PRECOND_F32");
    if (nrhs < 1 || nrhs > HH_MAX_BATCH) return fail(HH_EINVAL, "nrhs must be in [1, HH_MAX_BATCH]");
    if (reps < 1 || reps > 1000) return fail(HH_EINVAL, "reps must be in [1, 1000]");
    const bool f32 = (flags & HH_PRECOND_F32) != 0;
    const Layout L = layout(p, 1, f32 ? sizeof(cplxf) : sizeof(cplx));
    if (workspace_bytes < (size_t)nrhs * L.total) return fail(HH_EINVAL, "workspace too small");
    if (p->ndim != 2 || p->levels.size() < 2) return HH_OK;   // no multigrid legs
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Batch bt{nrhs, (int64_t)L.total, p->N};
    HIPCHK(hipMemsetAsync(workspace_dev, 0, (size_t)nrhs * L.total, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    hipError_t ee = hipEventCreate(&e1);
    int rc = ee == hipSuccess ? HH_OK : fail(HH_EDEVICE, hipGetErrorString(ee));
    if (rc == HH_OK)
        rc = f32 ? tune_legs<float>(p, L, workspace_dev, reps, s, bt, e0, e1)
                 : tune_legs<double>(p, L, workspace_dev, reps, s, bt, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

int hh_get_tiles(hh_problem p, int level, int* tile_down, int* tile_up) {
    g_err.clear();
    if (!p || !tile_down || !tile_up) return fail(HH_EINVAL, "NULL argument");
    if (p->ndim != 2 || level < 0 || level + 1 >= (int)p->levels.size())
        return fail(HH_EINVAL, "level has no multigrid legs");
    *tile_down = p->levels[level].tile_down;
    *tile_up = p->levels[level].tile_up;
    return HH_OK;
}

int hh_set_tiles(hh_problem p, int level, int tile_down, int tile_up) {
    g_err.clear();
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    if (p->ndim != 2 || level < 0 || level + 1 >= (int)p->levels.size())
        return fail(HH_EINVAL, "level has no multigrid legs");
    if (tile_down < -1 || tile_down >= HH_TILE_DOWN_COUNT || tile_up < -1 ||
        tile_up >= HH_TILE_UP_COUNT)
        return fail(HH_EINVAL, "unknown tile shape");
    p->levels[level].tile_down = tile_down;
    p->levels[level].tile_up = tile_up;
    return HH_OK;
}

int hh_apply_operator(hh_problem p, int which, const void* x_dev, void* y_dev, void* stream) {
    g_err.clear();
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    CHK(check_ptr(x_dev, "x_dev"));
    CHK(check_ptr(y_dev, "y_dev"));
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
    CHK(check_ptr(x_dev, "x_dev"));
    CHK(check_ptr(y_dev, "y_dev"));
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
    CHK(check_ptr(v_dev, "v_dev"));
    CHK(check_ptr(z_dev, "z_dev"));
    CHK(check_ptr(workspace_dev, "workspace_dev"));
    if (v_dev == z_dev) return fail(HH_EINVAL, "v_dev and z_dev must be distinct");
    const Layout L = layout(p, 1);
    if (workspace_bytes < L.total) return fail(HH_EINVAL, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    CHK(precond<double>(p, L, workspace_dev, static_cast<const cplx*>(v_dev), nullptr,
                        static_cast<cplx*>(z_dev), s));
    HIPCHK(hipStreamSynchronize(s));
    return HH_OK;
}

int hh_apply_precond_f32(hh_problem p, const void* v_dev, void* z_dev, void* workspace_dev,
                         size_t workspace_bytes, void* stream) {
    g_err.clear();
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    CHK(check_ptr(v_dev, "v_dev"));
    CHK(check_ptr(z_dev, "z_dev"));
    CHK(check_ptr(workspace_dev, "workspace_dev"));
    if (v_dev == z_dev) return fail(HH_EINVAL, "v_dev and z_dev must be distinct");
    const Layout L = layout(p, 1, sizeof(cplxf));
    if (workspace_bytes < L.total) return fail(HH_EINVAL, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    CHK(precond<float>(p, L, workspace_dev, static_cast<const cplx*>(v_dev), nullptr,
                       static_cast<cplxf*>(z_dev), s));
    HIPCHK(hipStreamSynchronize(s));
    return HH_OK;
}

int hh_orthogonalize_scratch_bytes(int64_t n, int k, size_t* bytes) {
    if (!bytes || n < 1 || k < 1 || k > kMaxRestart + 1) return fail(HH_EINVAL, "bad argument");
    const int nb = node_blocks(n);
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
    const int nb = node_blocks(n);
    cplx* partial = static_cast<cplx*>(scratch_dev);
    cplx* h1 = at<cplx>(scratch_dev, align_up((size_t)nb * k * sizeof(cplx)));
    cplx* h2 = h1 + align_up((size_t)k * sizeof(cplx)) / sizeof(cplx);
    cplx* nr = h2 + align_up((size_t)k * sizeof(cplx)) / sizeof(cplx);
    const cplx* V = static_cast<const cplx*>(V_dev);
    cplx* w = static_cast<cplx*>(w_dev);
    HIPCHK(launch_dot_blocks(V, n, k, w, partial, s));
    HIPCHK(launch_reduce_pred(partial, nb, k, h1, nullptr, s));
    HIPCHK(launch_axpy_dot(V, n, k, h1, w, partial, nullptr, s));
    HIPCHK(launch_reduce_pred(partial, nb, k, h2, nullptr, s));
    HIPCHK(launch_axpy_norm(V, n, k, h2, w, partial, nullptr, s));
    HIPCHK(launch_reduce_pred(partial, norm_blocks(n), 1, nr, nullptr, s));
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

}  // extern "C"

namespace {

// Right-preconditioned FGMRES(restart) for nrhs right-hand sides of one
// problem, each with its own Krylov basis, least-squares problem and
// convergence (the kernels of a step cover all of them; a right-hand side
// whose cycle has stopped returns at once). Steps advance together; a cycle
// closes when every right-hand side has stopped it.
int solve_impl(hh_problem_s* p, int nrhs, const cplx* f, double tol, int restart, int max_iters,
               unsigned flags, void* workspace_dev, size_t workspace_bytes, cplx* u,
               int* iterations, double* true_rel_res, int* status, double* hist_host,
               int hist_cap, int* hist_len, hipStream_t s) {
    const int m = restart;
    const bool no_prec = (flags & HH_NO_PRECOND) != 0;
    const bool f32 = (flags & HH_PRECOND_F32) != 0;
    const bool warm = (flags & HH_INITIAL_GUESS) != 0;
    Layout L = layout(p, m, f32 ? sizeof(cplxf) : sizeof(cplx));
    // blocks of the fused apply for this many sources: never more than
    // node_blocks(N), which sized the partial sums
    L.nbA = apply_blocks(op_H(p), nrhs);
    if (workspace_bytes < (size_t)nrhs * L.total) return fail(HH_EINVAL, "workspace too small");
    CHK(ensure_host_buffers(p, max_iters, nrhs));
    if (nrhs > 1 && p->ndim == 2 && p->levels.size() >= 2) {
        const size_t need = vc_gemm_scratch_bytes(p->nc, nrhs);
        if (p->gemm_part_bytes < need) {
            if (p->gemm_part) HIPCHK(hipFree(p->gemm_part));
            p->gemm_part = nullptr;
            p->gemm_part_bytes = 0;
            HIPCHK(hipMalloc(&p->gemm_part, need));
            p->gemm_part_bytes = need;
        }
    }
    const int64_t N = p->N;
    const Batch bt{nrhs, (int64_t)L.total, N};

    void* ws = workspace_dev;
    cplx* V = at<cplx>(ws, L.V);
    cplx* Z = at<cplx>(ws, L.Z);
    cplxf* Zf = at<cplxf>(ws, L.Z);
    cplx* b = at<cplx>(ws, L.b);
    cplx* w = at<cplx>(ws, L.w);
    cplx* partial = at<cplx>(ws, L.partial);
    cplx* h1 = at<cplx>(ws, L.h1);
    cplx* h2 = at<cplx>(ws, L.h2);
    cplx* R = at<cplx>(ws, L.R);
    double* cs = at<double>(ws, L.cs);
    cplx* sn = at<cplx>(ws, L.sn);
    cplx* g = at<cplx>(ws, L.g);
    cplx* y = at<cplx>(ws, L.y);
    double* zs = at<double>(ws, L.zs);
    SolveState* st = at<SolveState>(ws, L.st);
    const int* active = &st->active;
    const FineOp H = op_H(p);
    double* dhist = nullptr;
    HostRecord* drec = nullptr;
    HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&dhist), p->hist, 0));
    HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&drec), p->rec, 0));
    std::memset(p->rec, 0, (size_t)nrhs * sizeof(HostRecord));
    p->kt.pending.clear();

    // prologue: b = W f, ||b||, u = 0 (or the caller's initial guess)
    HIPCHK(launch_weight_rhs(H, f, b, s, bt));
    HIPCHK(launch_dot_blocks(b, N, 1, b, partial, s, bt));
    HIPCHK(launch_solve_init(st, partial, L.nbN, m, max_iters, tol, drec, dhist, p->hist_stride,
                             warm ? u : nullptr, N, s, bt));
    if (!warm) HIPCHK(hipMemsetAsync(u, 0, (size_t)nrhs * N * sizeof(cplx), s));

    // Arnoldi with delayed reorthogonalisation: step j preconditions and applies
    // H to u_j = V_j (projected once, not yet normalised), reduces the
    // projections of u_j and w = H z_j on V_0..V_j in one pass, then one pass
    // over the basis normalises v_j and projects w into V_{j+1}; the Givens
    // step of column j - 1 runs as an extra workgroup of that pass (column j - 1
    // needs step j's reorthogonalisation coefficients). A full cycle ends with
    // the projections of u_m and the Givens step of column m - 1.
    const GivensArgs giv{st, h1, h2, R, cs, sn, g, drec, dhist, (int64_t)L.total,
                         p->hist_stride, zs};
    cplx* red = h1;

    std::vector<std::vector<int>> executed;   // Arnoldi steps that did work, per cycle and RHS
    double min_est = 1.0;
    auto est_of = [&](int rb) { return ((const volatile HostRecord*)(p->rec + rb))->est; };
    for (int cycle = 1;; ++cycle) {
        p->kt.cycle = cycle;
        HIPCHK(launch_residual_norm(H, b, u, V, partial, &st->done, s, bt));   // u_0 = r
        HIPCHK(launch_cycle_start(st, partial, L.nbR, g, drec, dhist, p->hist_stride, warm, s,
                                  bt));
        // close to convergence: learn whether this cycle opens before enqueuing it
        if (min_est <= tol)
            CHK(wait_for(p, nrhs, s,
                         [&](const RecView& r) { return r.done || r.cycles >= cycle; }));
        bool closed = false;
        for (int j = 0; j < m; ++j) {
            if (j >= kLookahead)
                CHK(wait_for(p, nrhs, s, [&](const RecView& r) {
                    return r.done || r.stops >= cycle ||
                           (r.cycles >= cycle && r.jstep >= j - kLookahead + 1);
                }));
            bool all_stopped = true;
            for (int rb = 0; rb < nrhs && all_stopped; ++rb) {
                const RecView r = read_rec(p->rec + rb);
                all_stopped = r.done || r.stops >= cycle;
            }
            if (all_stopped) {
                closed = true;
                break;
            }
            p->kt.j = j;
            const int kk = j + 1;
            cplx* uj = V + (size_t)j * N;
            if (no_prec) {
                // z_j = u_j: kept in Z (V_j is normalised in place below)
                cplx* zz = Z + (size_t)j * N;
                HIPCHK(hipMemcpy2DAsync(zz, L.total, uj, L.total, (size_t)N * sizeof(cplx), nrhs,
                                        hipMemcpyDeviceToDevice, s));
                TIMED2(HH_KERNEL_APPLY_DOT, (32.0 + 16.0 * kk) * (double)N, 8.0 * (double)N,
                       launch_apply_dot(H, zz, w, V, kk, partial, active, s, bt));
            } else if (f32) {
                cplxf* zz = Zf + (size_t)j * N;
                CHK(precond<float>(p, L, ws, uj, active, zz, s, bt));
                TIMED2(HH_KERNEL_APPLY_DOT, (24.0 + 16.0 * kk) * (double)N, 8.0 * (double)N,
                       launch_apply_dot(H, zz, w, V, kk, partial, active, s, bt));
            } else {
                cplx* zz = Z + (size_t)j * N;
                CHK(precond<double>(p, L, ws, uj, active, zz, s, bt));
                TIMED2(HH_KERNEL_APPLY_DOT, (32.0 + 16.0 * kk) * (double)N, 8.0 * (double)N,
                       launch_apply_dot(H, zz, w, V, kk, partial, active, s, bt));
            }
            TIMED(HH_KERNEL_REDUCE, 16.0 * 2 * kk * (L.nbA + 1),
                  launch_reduce_pred(partial, L.nbA, 2 * kk, red, active, s, bt));
            // V_0..V_{j-1}, u_j and w in; v_j and u_{j+1} out
            TIMED(HH_KERNEL_AXPY_DOT, (j + 4) * 16.0 * (double)N,
                  launch_axpy_dcgs(V, N, j, red, w, active, &giv, s, bt));
        }
        if (!closed) {
            // a full cycle: projections of u_m on the basis and its norm, then
            // the Givens step of the last column
            TIMED(HH_KERNEL_AXPY_NORM, (m + 2) * 16.0 * (double)N,
                  launch_dot_blocks(V, N, m + 1, V + (size_t)m * N, partial, s, bt));
            TIMED(HH_KERNEL_REDUCE, 16.0 * (m + 1) * (L.nbN + 1),
                  launch_reduce_pred(partial, L.nbN, m + 1, red, active, s, bt));
            TIMED(HH_KERNEL_GIVENS, 16.0 * (m + 1), launch_givens_tail(giv, s, bt));
        }
        // the cycle closes on a step for every right-hand side (or they ended at its start)
        CHK(wait_for(p, nrhs, s, [&](const RecView& r) { return r.done || r.stops >= cycle; }));
        std::vector<int> ex(nrhs, 0);
        bool any_stopped = false, all_done = true;
        min_est = 1.0;
        for (int rb = 0; rb < nrhs; ++rb) {
            const RecView r = read_rec(p->rec + rb);
            ex[rb] = r.stops >= cycle ? r.jstep : 0;
            any_stopped = any_stopped || r.stops >= cycle;
            all_done = all_done && r.done;
            if (!r.done) min_est = std::fmin(min_est, est_of(rb));
        }
        executed.push_back(ex);
        if (!any_stopped) break;                    // every right-hand side finished at the start
        if (f32)
            HIPCHK(launch_cycle_finish(st, m, R, g, zs, y, Zf, N, u, s, bt));
        else
            HIPCHK(launch_cycle_finish(st, m, R, g, zs, y, Z, N, u, s, bt));
        if (all_done) break;                        // non-finite values inside the cycle
    }
    HIPCHK(hipStreamSynchronize(s));
    std::vector<SolveState> fin(nrhs);
    HIPCHK(hipMemcpy2D(fin.data(), sizeof(SolveState), st, L.total, sizeof(SolveState), nrhs,
                       hipMemcpyDeviceToHost));
    CHK(kt_harvest(p, executed));
    bool any_bad = false, any_nc = false;
    for (int rb = 0; rb < nrhs; ++rb) {
        const SolveState& q = fin[rb];
        if (iterations) iterations[rb] = q.it;
        if (true_rel_res) true_rel_res[rb] = q.rel;
        const int code = q.status == -4 ? HH_ENUMERIC : q.status == 1 ? HH_NOT_CONVERGED : HH_OK;
        if (status) status[rb] = code;
        any_bad = any_bad || code == HH_ENUMERIC;
        any_nc = any_nc || code == HH_NOT_CONVERGED;
        if (hist_host)
            for (int i = 0; i <= q.it && i < hist_cap; ++i)
                hist_host[(int64_t)rb * hist_cap + i] = p->hist[rb * p->hist_stride + i];
    }
    if (hist_len) *hist_len = fin[0].it + 1;
    if (any_bad) return fail(HH_ENUMERIC, "non-finite value in the iteration");
    return any_nc ? HH_NOT_CONVERGED : HH_OK;
}

int check_solve_args(hh_problem p, const void* f_dev, const void* u_dev, const void* ws,
                     double tol, int restart, int max_iters, unsigned flags) {
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    CHK(check_ptr(f_dev, "f_dev"));
    CHK(check_ptr(u_dev, "u_dev"));
    CHK(check_ptr(ws, "workspace_dev"));
    if (!(tol > 0.0 && tol < 1.0)) return fail(HH_EINVAL, "tol must be in (0, 1)");
    if (restart < 1 || restart > kMaxRestart) return fail(HH_EINVAL, "restart must be in [1, 1024]");
    if (max_iters < 1 || max_iters > (1 << 28)) return fail(HH_EINVAL, "max_iters must be in [1, 2^28]");
    if (flags & ~(HH_NO_PRECOND | HH_PRECOND_F32 | HH_INITIAL_GUESS))
        return fail(HH_EINVAL, "unknown flag");
    if ((flags & HH_NO_PRECOND) && (flags & HH_PRECOND_F32))
        return fail(HH_EINVAL, "HH_NO_PRECOND and HH_PRECOND_F32 exclude each other");
    if (f_dev == u_dev) return fail(HH_EINVAL, "f_dev and u_dev must be distinct");
    return HH_OK;
}

}  // namespace

extern "C" {

int hh_solve(hh_problem p, const void* f_dev, double tol, int restart, int max_iters,
             unsigned flags, void* workspace_dev, size_t workspace_bytes, void* u_dev,
             int* iterations, double* true_rel_res, double* hist_host, int hist_cap,
             int* hist_len, void* stream) {
    g_err.clear();
    CHK(check_solve_args(p, f_dev, u_dev, workspace_dev, tol, restart, max_iters, flags));
    if (hist_cap < 0 || (hist_cap > 0 && !hist_host)) return fail(HH_EINVAL, "bad history buffer");
    return solve_impl(p, 1, static_cast<const cplx*>(f_dev), tol, restart, max_iters, flags,
                      workspace_dev, workspace_bytes, static_cast<cplx*>(u_dev), iterations,
                      true_rel_res, nullptr, hist_host, hist_cap, hist_len,
                      static_cast<hipStream_t>(stream));
}

int hh_workspace_bytes_batch(hh_problem p, int restart, int nrhs, size_t* bytes) {
    g_err.clear();
    if (!p || !bytes) return fail(HH_EINVAL, "NULL argument");
    if (restart < 1 || restart > kMaxRestart) return fail(HH_EINVAL, "restart must be in [1, 1024]");
    if (nrhs < 1 || nrhs > HH_MAX_BATCH) return fail(HH_EINVAL, "nrhs must be in [1, HH_MAX_BATCH]");
    *bytes = (size_t)nrhs * layout(p, restart).total;
    return HH_OK;
}

int hh_solve_batch(hh_problem p, int nrhs, const void* f_dev, double tol, int restart,
                   int max_iters, unsigned flags, void* workspace_dev, size_t workspace_bytes,
                   void* u_dev, int* iterations, double* true_rel_res, int* status,
                   double* hist_host, int hist_cap, void* stream) {
    g_err.clear();
    CHK(check_solve_args(p, f_dev, u_dev, workspace_dev, tol, restart, max_iters, flags));
    if (nrhs < 1 || nrhs > HH_MAX_BATCH) return fail(HH_EINVAL, "nrhs must be in [1, HH_MAX_BATCH]");
    if (hist_cap < 0 || (hist_cap > 0 && !hist_host)) return fail(HH_EINVAL, "bad history buffer");
    return solve_impl(p, nrhs, static_cast<const cplx*>(f_dev), tol, restart, max_iters, flags,
                      workspace_dev, workspace_bytes, static_cast<cplx*>(u_dev), iterations,
                      true_rel_res, status, hist_host, hist_cap, nullptr,
                      static_cast<hipStream_t>(stream));
}

int hh_kernel_timer_start(hh_problem p, int kernel_id) {
    g_err.clear();
    if (!p) return fail(HH_EINVAL, "problem is NULL");
    if (kernel_id < HH_KERNEL_NONE || kernel_id > HH_KERNEL_GIVENS)
        return fail(HH_EINVAL, "unknown kernel id");
    p->kt.kid = kernel_id;
    p->kt.pending.clear();
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
