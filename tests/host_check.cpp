// Host-side checks of the C ABI for a sanitizer build (AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of plan.hip).  Every call here
// returns before any device work: argument validation, the extension
// arithmetic, status strings and error details, the rejection and cleanup
// paths of plans, batches, workspaces and the solve cache.  Without a GPU
// the plan and batch creations fail at the device query and must unwind
// without leaks.  Exit status 0 when every expectation holds.
#include <cstdio>
#include <cstring>
#include <vector>

#include "ipoisson.h"

static int g_fail = 0;

static void expect(bool ok, const char *what)
{
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what);
        ++g_fail;
    }
}

int main()
{
    const int64_t n3[3] = {9, 10, 11};
    const double h3[3] = {0.1, 0.12, 0.09};
    ips_plan p = nullptr;
    // validation of every argument
    expect(ips_plan_create(&p, 0, n3, h3, 6, 0, 0) == IPS_E_INVALID_ARG, "d = 0");
    expect(ips_plan_create(&p, 4, n3, h3, 6, 0, 0) == IPS_E_INVALID_ARG, "d = 4");
    expect(ips_plan_create(&p, 3, nullptr, h3, 6, 0, 0) == IPS_E_INVALID_ARG, "NULL n");
    expect(ips_plan_create(&p, 3, n3, nullptr, 6, 0, 0) == IPS_E_INVALID_ARG, "NULL h");
    expect(ips_plan_create(nullptr, 3, n3, h3, 6, 0, 0) == IPS_E_INVALID_ARG, "NULL out");
    expect(ips_plan_create(&p, 3, n3, h3, 5, 0, 0) == IPS_E_INVALID_ARG, "order 5");
    expect(ips_plan_create(&p, 3, n3, h3, 6, 7, 0) == IPS_E_INVALID_ARG, "precision 7");
    expect(ips_plan_create(&p, 3, n3, h3, 6, 0, 1u << 12) == IPS_E_INVALID_ARG, "unknown flag");
    expect(ips_plan_create(&p, 1, n3, h3, 6, 1, 0) == IPS_E_UNSUPPORTED, "1D mixed");
    expect(ips_plan_create(&p, 3, n3, h3, 6, 1, IPS_FLAG_SCREENING) == IPS_E_UNSUPPORTED, "screening mixed");
    expect(ips_plan_create(&p, 3, n3, h3, 6, 0, IPS_FLAG_SCREENING | IPS_FLAG_ADJOINT) == IPS_E_UNSUPPORTED,
           "screening adjoint");
    expect(ips_plan_create(&p, 3, n3, h3, 6, 0, IPS_FLAG_SCREEN_DIRECT) == IPS_E_INVALID_ARG,
           "direct surface sums without screening");
    const int64_t small[3] = {9, 6, 9};
    expect(ips_plan_create(&p, 3, small, h3, 4, 0, IPS_FLAG_SCREENING) == IPS_E_INVALID_ARG, "screening n < 7");
    const int64_t seven[3] = {9, 7, 9};
    expect(ips_plan_create(&p, 3, seven, h3, 6, 0, 0) == IPS_E_INVALID_ARG, "order 6 with n < 8");
    const int64_t huge[3] = {9, 9, 1026};
    expect(ips_plan_create(&p, 3, huge, h3, 6, 0, 0) == IPS_E_UNSUPPORTED, "3D too long");
    const double hbad[3] = {0.1, -0.1, 0.1};
    expect(ips_plan_create(&p, 3, n3, hbad, 6, 0, 0) == IPS_E_INVALID_ARG, "negative h");
    expect(p == nullptr, "no plan returned on errors");
    // the calls that pass validation stop at the device query here (no GPU)
    // or succeed on a GPU: either way they must unwind cleanly
    int rc = ips_plan_create(&p, 3, n3, h3, 6, 0, 0);
    if (rc == IPS_OK) {
        expect(p != nullptr, "plan on success");
        ips_plan_destroy(p);
        p = nullptr;
    } else {
        expect(rc == IPS_E_DEVICE && p == nullptr, "plan creation without a device");
    }
    // error details: truncation, NULL buffer, long messages
    char buf[4];
    ips_plan_create(&p, 0, n3, h3, 6, 0, 0);
    expect(ips_last_error_detail(buf, sizeof buf) == IPS_OK && std::strlen(buf) == 3, "detail truncation");
    expect(ips_last_error_detail(nullptr, 8) == IPS_E_INVALID_ARG, "detail NULL");
    expect(ips_last_error_detail(buf, 0) == IPS_OK, "detail empty buffer");
    for (int s = -6; s <= 1; ++s) expect(ips_status_string(s) && *ips_status_string(s), "status string");
    for (int s = -1; s <= IPS_STAGE_COUNT; ++s) expect(ips_stage_name(s) != nullptr, "stage name");
    // extension arithmetic over many sizes
    for (int64_t n = 3; n < 600; n += 7) {
        const int64_t nn[3] = {n, n + 1, n + 2}, mg[3] = {0, 3, 17};
        int64_t ne[3], off[3];
        expect(ips_extension(3, nn, mg, ne, off) == IPS_OK, "extension");
        for (int a = 0; a < 3; ++a) {
            expect(ne[a] >= nn[a] + 2 * mg[a] && off[a] >= mg[a] && off[a] + nn[a] <= ne[a], "extension bounds");
            int64_t m = ne[a] - 1;
            for (int64_t q : {2, 3, 5})
                while (m % q == 0) m /= q;
            expect(m == 1, "extension 5-smooth");
        }
    }
    int64_t ne[3], off[3];
    const int64_t neg[3] = {-1, 0, 0};
    expect(ips_extension(3, n3, neg, ne, off) == IPS_E_INVALID_ARG, "negative margin");
    expect(ips_extension(3, n3, nullptr, ne, off) == IPS_E_INVALID_ARG, "NULL margin");
    expect(ips_plan_create_extended(&p, 3, n3, h3, 6, 0, 0, neg) == IPS_E_INVALID_ARG, "extended bad margin");
    // NULL plans and arrays everywhere
    size_t sz = 0;
    expect(ips_execute(nullptr, nullptr, nullptr, nullptr) == IPS_E_INVALID_ARG, "execute NULL");
    expect(ips_execute_static(nullptr, nullptr, nullptr, nullptr) == IPS_E_INVALID_ARG, "static NULL");
    expect(ips_execute_adjoint(nullptr, nullptr, nullptr, nullptr) == IPS_E_INVALID_ARG, "adjoint NULL");
    expect(ips_plan_workspace_size(nullptr, &sz) == IPS_E_INVALID_ARG, "workspace size NULL");
    expect(ips_plan_table_size(nullptr, &sz) == IPS_E_INVALID_ARG, "table size NULL");
    expect(ips_plan_set_workspace(nullptr, nullptr, 0) == IPS_E_INVALID_ARG, "set workspace NULL");
    expect(ips_plan_destroy(nullptr) == IPS_OK, "destroy NULL");
    expect(ips_solve(3, n3, h3, nullptr, 6, nullptr) == IPS_E_INVALID_ARG, "solve NULL arrays");
    expect(ips_solve_ex(3, n3, h3, nullptr, 6, 9, nullptr) == IPS_E_INVALID_ARG, "solve bad precision");
    expect(ips_solve_cache_size(&sz) == IPS_OK && sz == 0, "cache size");
    expect(ips_solve_release_cache() == IPS_OK, "cache release");
    expect(ips_live_device_bytes(&sz) == IPS_OK, "live bytes");
    // batches: bad descriptions, and creations that unwind at the device query
    ips_batch b = nullptr;
    const int dd[2] = {3, 3};
    const int64_t nb[2][3] = {{9, 10, 11}, {12, 9, 10}};
    const double hb[2][3] = {{0.1, 0.1, 0.1}, {0.1, 0.2, 0.1}};
    expect(ips_batch_create(&b, 0, dd, nb, hb, 6, 0, 0) == IPS_E_INVALID_ARG, "empty batch");
    expect(ips_batch_create(&b, 2, nullptr, nb, hb, 6, 0, 0) == IPS_E_INVALID_ARG, "batch NULL d");
    expect(ips_batch_create(&b, 2, dd, nb, hb, 6, 0, IPS_FLAG_BATCH_SMOOTH | IPS_FLAG_SCREENING) ==
               IPS_E_UNSUPPORTED,
           "smooth screening batch");
    for (unsigned fl : {0u, (unsigned)IPS_FLAG_BATCH_SMOOTH, (unsigned)IPS_FLAG_BATCH_EAGER}) {
        rc = ips_batch_create(&b, 2, dd, nb, hb, 6, 0, fl);
        if (rc == IPS_OK) {
            ips_batch_destroy(b);
            b = nullptr;
        } else {
            expect(b == nullptr, "no batch on errors");
        }
    }
    expect(ips_batch_execute(nullptr, nullptr, nullptr, nullptr) == IPS_E_INVALID_ARG, "batch execute NULL");
    expect(ips_batch_destroy(nullptr) == IPS_OK, "batch destroy NULL");
    if (g_fail) {
        std::fprintf(stderr, "%d host checks failed\n", g_fail);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
