// Host-logic driver for the AddressSanitizer / UndefinedBehaviorSanitizer
// build of the library (tests/test_host_sanitizers.py builds both).  It runs
// the entry points that need no GPU: the segment schedules of the two- and
// one-site parallel steps (Sec. III B) over many partitions, the
// sum-of-exponentials fit (Sec. II C) over exponents, term counts and
// ranges, with and without refinement, and the argument checks of those and
// of the context calls.  Any sanitizer report aborts the process; the
// driver itself only checks the results' basic invariants.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "tdvp.h"

static int fails = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                                    \
        }                                                               \
    } while (0)

using Sched = int (*)(int, const int*, double, int, int, int*, int*, int*, double*, int*);

static void schedules(Sched f, int min_inner) {
    std::mt19937 g(7);
    for (int trial = 0; trial < 400; ++trial) {
        const int nseg = 1 + (int)(g() % 40);
        std::vector<int> sz(nseg);
        int N = 0;
        for (int i = 0; i < nseg; ++i) {
            sz[i] = min_inner - 1 + (int)(g() % 10);
            N += sz[i];
        }
        for (int first = 0; first < 2; ++first) {
            int n = -1;
            // size query (max_ops = 0 reports the count with TDVP_E_SHAPE),
            // then the real call, then a buffer one too small
            const int rc = f(nseg, sz.data(), 0.01, first, 0, nullptr, nullptr, nullptr, nullptr, &n);
            CHECK(rc != TDVP_OK);
            if (n <= 0) continue;  // a partition the schedule refuses
            std::vector<int> ph(n), kind(n), site(n);
            std::vector<double> tau(n);
            int m = 0;
            CHECK(f(nseg, sz.data(), 0.01, first, n, ph.data(), kind.data(), site.data(), tau.data(), &m) == TDVP_OK);
            CHECK(m == n);
            for (int i = 0; i < m; ++i) {
                CHECK(site[i] >= 0 && site[i] < N);
                CHECK(ph[i] >= 0 && std::isfinite(tau[i]));
            }
            if (n > 1) {
                int m2 = 0;
                CHECK(f(nseg, sz.data(), 0.01, first, n - 1, ph.data(), kind.data(), site.data(), tau.data(), &m2) !=
                      TDVP_OK);
            }
        }
    }
    int n = 0;
    const int bad[2] = {3, -1};
    CHECK(f(2, bad, 0.01, 1, 0, nullptr, nullptr, nullptr, nullptr, &n) != TDVP_OK);
    CHECK(f(0, bad, 0.01, 1, 0, nullptr, nullptr, nullptr, nullptr, &n) != TDVP_OK);
    CHECK(f(1, nullptr, 0.01, 1, 0, nullptr, nullptr, nullptr, nullptr, &n) != TDVP_OK);
}

static void fits() {
    const double alphas[] = {0.75, 1.5, 3.0};
    for (double a : alphas)
        for (int K : {1, 4, 6})
            for (int R : {2 * K, 31, 64})
                for (int refine = 0; refine < 2; ++refine) {
                    if (R < 2 * K) continue;
                    std::vector<double> c(2 * K), lam(2 * K);
                    double err = -1.0;
                    const int rc = tdvp_fit_power_law(a, K, R, refine, c.data(), lam.data(), &err);
                    CHECK(rc == TDVP_OK || rc == TDVP_E_NUMERIC);
                    if (rc == TDVP_OK) CHECK(std::isfinite(err) && err >= 0.0);
                }
    // exact sums are recovered; bad sizes and samples are refused
    std::vector<double> f(40), c(8), lam(8);
    for (int r = 1; r <= 40; ++r) f[r - 1] = 0.7 * std::pow(0.5, r) + 0.2 * std::pow(-0.3, r);
    double err = -1.0;
    CHECK(tdvp_fit_exponentials(f.data(), 40, 2, 0, c.data(), lam.data(), &err) == TDVP_OK);
    CHECK(err < 1e-10);
    CHECK(tdvp_fit_exponentials(f.data(), 3, 2, 0, c.data(), lam.data(), &err) != TDVP_OK);
    CHECK(tdvp_fit_exponentials(f.data(), 40, 0, 0, c.data(), lam.data(), &err) != TDVP_OK);
    CHECK(tdvp_fit_exponentials(nullptr, 40, 2, 0, c.data(), lam.data(), &err) != TDVP_OK);
    f[5] = NAN;
    CHECK(tdvp_fit_exponentials(f.data(), 40, 2, 0, c.data(), lam.data(), &err) != TDVP_OK);
}

static void contexts() {
    CHECK(tdvp_ctx_destroy(nullptr) != TDVP_OK);
    CHECK(tdvp_ctx_sync(nullptr) != TDVP_OK);
    CHECK(tdvp_version() != nullptr);
    CHECK(tdvp_ctx_create(0, nullptr, nullptr, nullptr, nullptr, nullptr) != TDVP_OK);
}

int main() {
    schedules(seg_schedule, 2);
    schedules(seg_schedule1, 3);
    fits();
    contexts();
    std::printf("sanitize driver: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
