// Drives the plan builder's host code through the C ABI (plan creation in 2D and 3D with and
// without influence coefficients, constraints, broken-bond lists valid and invalid, crack
// segments to bonds, surface factors, per-case coefficients, bond read-back) so that
// AddressSanitizer and UndefinedBehaviorSanitizer see every host path of plan.cpp.  Exit
// status 0 when every call returned what it should; a sanitizer report aborts the run.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/msbfm.h"

static int fails = 0;
#define EXPECT(cond)                                                             \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "%s:%d: failed: %s\n", __FILE__, __LINE__, #cond); \
            ++fails;                                                             \
        }                                                                        \
    } while (0)

static msb_problem_desc desc2(int nx, int ny, int M, int nk, const double *infl, int batch) {
    msb_problem_desc d;
    std::memset(&d, 0, sizeof(d));
    d.dim = 2;
    d.n[0] = nx;
    d.n[1] = ny;
    d.n[2] = 1;
    d.h = 1.0 / nx;
    d.M = M;
    d.alpha = 9.0 / (M_PI * std::pow(M * d.h, 3));
    d.n_infl = nk;
    d.infl = infl;
    d.rho = 1.0;
    d.batch = batch;
    return d;
}

int main() {
    const double infl[4] = {0.3, 0.5, 0.1, 0.7};
    // 2D plans of several sizes and horizons, with a crack, constraints and surface factors
    for (int M = 1; M <= 4; ++M) {
        for (int nk : {0, 4}) {
            msb_problem_desc d = desc2(23 + M, 17 + 2 * M, M, nk, nk ? infl : nullptr, 2);
            msb_plan p = nullptr;
            EXPECT(msb_plan_create(&d, &p) == MSB_OK && p);
            const int64_t N = d.n[0] * d.n[1];
            std::vector<uint8_t> fixed(2 * N, 0);
            for (int64_t i = 0; i < N; i += 7) fixed[i] = 1;
            EXPECT(msb_plan_set_constraints(p, fixed.data()) == MSB_OK);
            const double seg[8] = {0.2, 0.25, 0.8, 0.7, 0.5, 0.1, 0.55, 0.9};
            int64_t nb = 0;
            // a count query: capacity 0 is too small, the status says so and the count is set
            EXPECT(msb_crack_to_bonds(&d, seg, 2, nullptr, 0, &nb) == MSB_EINVAL && nb > 0);
            std::vector<int64_t> pq(2 * nb);
            int64_t nb2 = 0;
            EXPECT(msb_crack_to_bonds(&d, seg, 2, pq.data(), nb, &nb2) == MSB_OK && nb2 == nb);
            EXPECT(msb_plan_set_bonds(p, pq.data(), nb) == MSB_OK);
            std::vector<int64_t> back(2 * nb);
            int64_t cnt = 0;
            EXPECT(msb_plan_get_bonds(p, back.data(), nb, &cnt) == MSB_OK && cnt == nb);
            EXPECT(back == pq);
            // invalid lists are rejected and leave the old list
            const int64_t bad_range[2] = {0, N};
            const int64_t bad_far[2] = {0, (int64_t)(M + 1)};
            std::vector<int64_t> dup(pq.begin(), pq.begin() + 2);
            dup.insert(dup.end(), pq.begin(), pq.begin() + 2);
            const int64_t rev_dup[4] = {pq[0], pq[1], pq[1], pq[0]};   // one pair in both orders
            EXPECT(msb_plan_set_bonds(p, bad_range, 1) == MSB_EINVAL);
            EXPECT(msb_plan_set_bonds(p, bad_far, 1) == MSB_EINVAL);
            EXPECT(msb_plan_set_bonds(p, dup.data(), 2) == MSB_EINVAL);
            EXPECT(msb_plan_set_bonds(p, rev_dup, 2) == MSB_EINVAL);
            int64_t L[3], Nn = 0, nbp = 0;
            EXPECT(msb_plan_info(p, L, &Nn, &nbp) == MSB_OK && nbp == nb && Nn == N);
            std::vector<double> nu(N);
            EXPECT(msb_surface_volume_factors(p, nu.data()) == MSB_OK);
            for (double x : nu) EXPECT(x >= 1.0 && std::isfinite(x));
            EXPECT(msb_plan_set_surface(p, nu.data()) == MSB_OK);
            EXPECT(msb_plan_set_surface(p, nullptr) == MSB_OK);
            if (nk) {
                const double pc[8] = {0.2, 0.4, 0.6, 0.8, 0.9, 0.1, 0.3, 0.5};
                EXPECT(msb_plan_set_infl(p, pc, 4, 1) == MSB_OK);
                EXPECT(msb_plan_set_infl(p, infl, 4, 0) == MSB_OK);
            }
            EXPECT(msb_plan_set_bonds(p, nullptr, 0) == MSB_OK);
            EXPECT(msb_plan_set_constraints(p, nullptr) == MSB_OK);
            msb_plan_destroy(p);
        }
    }
    // 3D plans
    for (int M = 1; M <= 3; ++M) {
        msb_problem_desc d;
        std::memset(&d, 0, sizeof(d));
        d.dim = 3;
        d.n[0] = 11;
        d.n[1] = 9;
        d.n[2] = 8;
        d.h = 1.0 / 11;
        d.M = M;
        d.alpha = 12.0 / (M_PI * std::pow(M * d.h, 4));
        d.n_infl = 2;
        d.infl = infl;
        d.rho = 1.0;
        d.batch = 1;
        msb_plan p = nullptr;
        EXPECT(msb_plan_create(&d, &p) == MSB_OK && p);
        const int64_t N = 11 * 9 * 8;
        std::vector<uint8_t> fixed(3 * N, 0);
        for (int64_t i = 0; i < 3 * 11 * 9; ++i) fixed[i] = 1;
        EXPECT(msb_plan_set_constraints(p, fixed.data()) == MSB_OK);
        const int64_t pair[2] = {0, 1};
        EXPECT(msb_plan_set_bonds(p, pair, 1) == MSB_OK);
        msb_plan_destroy(p);
    }
    // descriptions rejected before any allocation
    msb_problem_desc d = desc2(10, 10, 0, 0, nullptr, 1);
    msb_plan p = nullptr;
    EXPECT(msb_plan_create(&d, &p) == MSB_EINVAL && !p);
    d = desc2(10, 10, 3, 0, nullptr, 0);
    EXPECT(msb_plan_create(&d, &p) == MSB_EINVAL && !p);
    EXPECT(msb_plan_create(nullptr, &p) == MSB_EINVAL);
    std::printf("plan host driver: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
