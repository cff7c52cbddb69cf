// Host-side checks of the library's C-ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (test infrastructure; built by
// tests/test_host_sanitized.py with the sanitizers on host code only).
// Every call here runs on the host: circuit creation (with distant pairs),
// the compiled circuit, light cones, cut bounds, validation errors, the
// all-outputs count query.  No device is needed.
#include <cmath>
#include <cstdio>
#include <vector>

#include "lofp.h"

static int failures = 0;
#define CHECK(cond)                                                            \
    do {                                                                       \
        if (!(cond)) {                                                         \
            std::printf("check failed at line %d: %s\n", __LINE__, #cond);     \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

int main()
{
    // a 16-mode, depth-8 brickwork
    const int m = 16, D = 8;
    std::vector<lofp_bs> bs;
    std::vector<int32_t> lens;
    for (int l = 0; l < D; ++l) {
        int k = 0;
        for (int a = l % 2; a + 1 < m; a += 2, ++k) bs.push_back({a, a + 1, 0.3 + 0.01 * a, 1.1 * l});
        lens.push_back(k);
    }
    lofp_circuit c = nullptr;
    CHECK(lofp_circuit_create(m, D, lens.data(), bs.data(), &c) == LOFP_OK);
    std::vector<int32_t> S(m, 0), T(m, 0);
    for (int i = 0; i < m; i += 2) S[i] = 1;
    for (int i = 1; i < m; i += 2) T[i] = 1;
    std::vector<int32_t> lo((D + 1) * (m - 1)), hi(lo.size());
    int32_t feasible = -1;
    CHECK(lofp_bounds(c, S.data(), T.data(), lo.data(), hi.data(), &feasible) == LOFP_OK);
    CHECK(feasible == 1);
    for (size_t i = 0; i < lo.size(); ++i) CHECK(lo[i] <= hi[i]);
    int32_t pl, ph, fl, fh;
    CHECK(lofp_light_cone(c, 4, 7, &pl, &ph, &fl, &fh) == LOFP_OK);
    CHECK(pl <= 7 && ph >= 7 && fl <= 7 && fh >= 7);
    int64_t count = 0;
    CHECK(lofp_all_outputs(c, S.data(), 0, nullptr, nullptr, &count, nullptr) == LOFP_OK);
    CHECK(count == 490314);
    int32_t nl = 0;
    CHECK(lofp_circuit_compiled(c, &nl, nullptr, nullptr, 0) == LOFP_OK && nl == D);
    CHECK(lofp_circuit_destroy(c) == LOFP_OK);

    // distant pairs, compiled; host queries of layers refuse them
    std::vector<lofp_bs> far = {{0, 3, 0.4, 0.2}, {1, 2, 0.5, 0.1}, {4, 7, 0.6, 0.3}};
    std::vector<int32_t> flen = {3};
    CHECK(lofp_circuit_create(8, 1, flen.data(), far.data(), &c) == LOFP_OK);
    CHECK(lofp_circuit_compiled(c, &nl, nullptr, nullptr, 0) == LOFP_OK && nl == 11);
    std::vector<int32_t> clen(nl);
    std::vector<lofp_bs> cbs(64);
    CHECK(lofp_circuit_compiled(c, &nl, clen.data(), cbs.data(), 64) == LOFP_OK);
    int tot = 0;
    for (int l = 0; l < nl; ++l) tot += clen[l];
    CHECK(tot == 3 + 2 * 2 + 2 * 2);
    for (int g = 0; g < tot; ++g) CHECK(cbs[g].b == cbs[g].a + 1);
    CHECK(lofp_light_cone(c, 0, 0, &pl, &ph, &fl, &fh) == LOFP_ENOTSUP);
    CHECK(lofp_circuit_destroy(c) == LOFP_OK);

    // validation
    CHECK(lofp_circuit_create(1, 0, nullptr, nullptr, &c) == LOFP_EINVAL);
    std::vector<lofp_bs> clash = {{0, 1, 0.1, 0.1}, {1, 2, 0.1, 0.1}};
    std::vector<int32_t> clen2 = {2};
    CHECK(lofp_circuit_create(4, 1, clen2.data(), clash.data(), &c) == LOFP_EINVAL);
    CHECK(lofp_circuit_create(40, 0, nullptr, nullptr, &c) == LOFP_ENOTSUP);
    CHECK(lofp_last_error()[0] != 0);
    std::printf("host checks: %d failures\n", failures);
    return failures ? 1 : 0;
}
