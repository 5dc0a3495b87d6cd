// Host-side driver for the sanitizer test: calls every entry point that does
// its work on the host before touching a device (argument validation, null
// handles, status strings, footprint planning over a sweep of grids and
// limits), so that the library's host code runs under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU. Exit 0 and "ok" when
// every call returned what the header documents.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "helmholtz.h"

static int fails = 0;

static void expect(bool ok, const char* what) {
    if (!ok) {
        std::printf("FAIL: %s\n", what);
        ++fails;
    }
}

int main() {
    // status strings: static, non-empty, also for unknown codes
    for (int st = -8; st <= 3; ++st) {
        const char* s = hh_status_string(st);
        expect(s && *s, "status string");
    }
    expect(hh_status_string(99) && *hh_status_string(99), "unknown status string");

    // creation is refused before any device work
    const double* fake = reinterpret_cast<const double*>(0x1000);   // never dereferenced
    hh_problem out = nullptr;
    const int64_t shape[2] = {9, 11}, small[2] = {2, 11}, big1d[2] = {HH_MAX_1D + 1, 0};
    const double w = 2 * M_PI * 10.0;
    expect(hh_create_problem(fake, 3, shape, w, 0.01, 10.0, nullptr, &out) == HH_EINVAL, "ndim");
    expect(hh_create_problem(nullptr, 2, shape, w, 0.01, 10.0, nullptr, &out) == HH_EINVAL, "m");
    expect(hh_create_problem(fake, 2, nullptr, w, 0.01, 10.0, nullptr, &out) == HH_EINVAL,
           "shape");
    expect(hh_create_problem(fake, 2, shape, -1.0, 0.01, 10.0, nullptr, &out) == HH_EINVAL,
           "omega");
    expect(hh_create_problem(fake, 2, shape, NAN, 0.01, 10.0, nullptr, &out) == HH_EINVAL,
           "omega nan");
    expect(hh_create_problem(fake, 2, shape, w, -0.1, 10.0, nullptr, &out) == HH_EINVAL, "alpha");
    expect(hh_create_problem(fake, 2, shape, w, 0.01, 0.0, nullptr, &out) == HH_EINVAL, "h");
    expect(hh_create_problem(fake, 2, small, w, 0.01, 10.0, nullptr, &out) == HH_EINVAL, "small");
    expect(hh_create_problem(fake, 2, shape, w, 0.01, 10.0, nullptr, nullptr) == HH_EINVAL,
           "out");
    expect(hh_create_problem(fake, 1, big1d, w, 0.01, 10.0, nullptr, &out) == HH_EUNSUPPORTED,
           "1D limit");
    expect(hh_last_error() && std::strstr(hh_last_error(), "1D"), "last error");
    expect(hh_create_problem_ex(fake, 2, shape, w, 0.01, 10.0, 0, nullptr, &out) == HH_EINVAL,
           "max_coarse 0");
    expect(hh_create_problem_ex(fake, 2, shape, w, 0.01, 10.0, HH_MAX_COARSE_LIMIT + 1, nullptr,
                                &out) == HH_EINVAL,
           "max_coarse limit");
    expect(out == nullptr, "no handle on failure");

    // null handles
    size_t n = 0;
    int a = 0, b = 0;
    expect(hh_workspace_bytes(nullptr, 30, &n) == HH_EINVAL, "workspace null");
    expect(hh_workspace_bytes_batch(nullptr, 30, 4, &n) == HH_EINVAL, "workspace batch null");
    expect(hh_set_shift(nullptr, 1.0, 0.5) == HH_EINVAL, "shift null");
    expect(hh_set_max_coarse(nullptr, 100) == HH_EINVAL, "max coarse null");
    expect(hh_get_tiles(nullptr, 0, &a, &b) == HH_EINVAL, "tiles null");
    expect(hh_set_tiles(nullptr, 0, 0, 0) == HH_EINVAL, "set tiles null");
    expect(hh_num_levels(nullptr, &a) == HH_EINVAL, "levels null");
    expect(hh_solve(nullptr, fake, 1e-6, 30, 100, 0, nullptr, 0, nullptr, nullptr, nullptr,
                    nullptr, 0, nullptr, nullptr) == HH_EINVAL,
           "solve null");
    expect(hh_destroy_problem(nullptr) == HH_OK, "destroy null");
    expect(hh_orthogonalize_scratch_bytes(1000, 0, &n) == HH_EINVAL, "orth k 0");
    for (int64_t len : {int64_t(1), int64_t(1000), int64_t(1) << 24})
        for (int k : {1, 7, 64, 1024}) {
            n = 0;
            expect(hh_orthogonalize_scratch_bytes(len, k, &n) == HH_OK && n > 0, "orth bytes");
        }

    // footprint planning: a sweep of grids, frequencies, limits, restarts and batch sizes
    const int64_t sizes[] = {3, 4, 5, 9, 17, 33, 64, 101, 201, 401, 801, 1201, 1601};
    const double freqs[] = {2.0, 10.0, 30.0};
    const int limits[] = {1, 100, HH_MAX_COARSE, 16384};
    const int restarts[] = {1, 30, 1024};
    const int batches[] = {1, 32, HH_MAX_BATCH};
    long calls = 0;
    for (int64_t nz : sizes)
        for (int64_t nx : sizes)
            for (double f : freqs)
                for (int mc : limits)
                    for (int r : restarts)
                        for (int nb : batches)
                            for (unsigned fl : {0u, HH_PRECOND_F32}) {
                                const int64_t s2[2] = {nz, nx};
                                size_t pb = 0, wb = 0;
                                const int st = hh_footprint_bytes(2, s2, 2 * M_PI * f, 1 / 1500.0,
                                                                  10.0, mc, r, nb, fl, &pb, &wb);
                                expect(st == HH_OK || st == HH_EUNSUPPORTED, "footprint status");
                                if (st == HH_OK) expect(pb > 0 && wb > 0, "footprint bytes");
                                ++calls;
                            }
    for (int64_t len : {int64_t(3), int64_t(100), int64_t(1001), int64_t(HH_MAX_1D)})
        for (int r : restarts) {
            const int64_t s1[2] = {len, 0};
            size_t pb = 0, wb = 0;
            expect(hh_footprint_bytes(1, s1, w, 1 / 1500.0, 5.0, HH_MAX_COARSE, r, 1, 0, &pb,
                                      &wb) == HH_OK && pb > 0 && wb > 0,
                   "footprint 1D");
        }
    const int64_t s2[2] = {201, 401};
    size_t pb = 0, wb = 0;
    expect(hh_footprint_bytes(2, s2, w, 1 / 1500.0, 10.0, HH_MAX_COARSE, 0, 1, 0, &pb, &wb) ==
               HH_EINVAL,
           "footprint restart 0");
    expect(hh_footprint_bytes(2, s2, w, 1 / 1500.0, 10.0, HH_MAX_COARSE, 30, HH_MAX_BATCH + 1, 0,
                              &pb, &wb) == HH_EINVAL,
           "footprint batch");
    expect(hh_footprint_bytes(2, s2, w, 1 / 1500.0, -1.0, HH_MAX_COARSE, 30, 1, 0, &pb, &wb) ==
               HH_EINVAL,
           "footprint h");
    std::printf("%ld footprint plans, %d failures\n", calls, fails);
    if (fails == 0) std::printf("ok\n");
    return fails ? 1 : 0;
}
