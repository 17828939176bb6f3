// Host-code check under AddressSanitizer and UndefinedBehaviorSanitizer: the
// host analysis of a context (sightline supports, nested dissection,
// multifrontal layout) through ep_plan, on valid and invalid inputs.  Built
// and run by tests/test_host_sanitizers.py; no GPU is touched.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ep.h"

namespace ep {
static std::string g_err;
void set_last_error(const std::string& m) { g_err = m; }
}  // namespace ep

static ep_config make_cfg(int n, double box) {
    ep_config c;
    std::memset(&c, 0, sizeof c);
    c.n = n;
    c.box_pc = box;
    c.observer_pc[0] = box / 2;
    c.observer_pc[1] = 0.0;
    c.observer_pc[2] = box / 2;
    c.prior_mean = -7.0;
    c.prior_var = 1.0;
    c.outer_scale_pc = 100.0;
    c.support_pc = 150.0;
    c.los_step_pc = 2.0;
    c.damping = 1.0;
    c.leaf_size = 64;
    return c;
}

static std::vector<double> stars(int64_t count, double box, uint64_t seed) {
    std::vector<double> x((size_t)(3 * count));
    uint64_t s = seed;
    for (auto& v : x) {
        s = s * 6364136223846793005ULL + 1442695040888963407ULL;
        v = box * (0.001 + 0.998 * (double)(s >> 11) / 9007199254740992.0);
    }
    return x;
}

int main() {
    int bad = 0;
    struct Case { int n; double box; int64_t count; };
    for (const Case& k : {Case{16, 1000.0, 1000}, Case{24, 1500.0, 6000}, Case{12, 700.0, 0}}) {
        ep_config c = make_cfg(k.n, k.box);
        std::vector<double> x = stars(k.count, k.box, 17 + k.n);
        ep_plan_stats p;
        const int rc = ep_plan(&c, k.count, x.data(), &p);
        std::printf("n=%d stars=%lld rc=%d fronts=%lld nnz_L=%lld front_elems=%lld\n", k.n, (long long)k.count, rc,
                    (long long)p.n_fronts, (long long)p.nnz_L, (long long)p.front_elems);
        if (rc != 0 || !(p.nnz_L > 0) || p.nnz_L > p.front_elems) bad++;
    }
    // invalid inputs are refused before any analysis
    ep_config c = make_cfg(16, 1000.0);
    std::vector<double> x = stars(10, 1000.0, 3);
    ep_plan_stats p;
    x[5] = 5000.0;   // outside the cube
    if (ep_plan(&c, 10, x.data(), &p) != EP_ERR_INVALID_ARG) bad++;
    x[5] = std::nan("");
    if (ep_plan(&c, 10, x.data(), &p) != EP_ERR_INVALID_ARG) bad++;
    x[3] = 500.0; x[4] = 0.0; x[5] = 500.0;   // at the observer
    if (ep_plan(&c, 10, x.data(), &p) != EP_ERR_INVALID_ARG) bad++;
    c.n = 1;
    if (ep_plan(&c, 0, nullptr, &p) != EP_ERR_INVALID_ARG) bad++;
    std::printf(bad ? "FAILED %d\n" : "OK\n", bad);
    return bad ? 1 : 0;
}
