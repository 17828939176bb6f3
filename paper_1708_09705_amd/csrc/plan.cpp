// ep_plan: the structure, work and memory of a configuration from the host
// analysis alone (sightline supports, nested dissection, multifrontal
// layout), without a device.  The same analysis ep_init runs; what ep_init
// would then allocate is counted instead of allocated.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/ep.h"
#include "kernels.h"
#include "symbolic.h"

namespace ep {
void set_last_error(const std::string& m);   // api.cpp
}

using namespace ep;

extern "C" int ep_plan(const ep_config* c, int64_t S, const double* xyz, ep_plan_stats* out) {
    if (!c || !out || S < 0 || (S > 0 && !xyz)) {
        set_last_error("ep_plan: bad arguments");
        return EP_ERR_INVALID_ARG;
    }
    if (c->n < 2 || c->n > 1290 || !(c->box_pc > 0) || !(c->support_pc > 0) || !(c->los_step_pc > 0)) {
        set_last_error("ep_plan: n must be in [2, 1290] and box_pc, support_pc, los_step_pc > 0");
        return EP_ERR_INVALID_ARG;
    }
    for (int a = 0; a < 3; a++)
        if (!(c->observer_pc[a] >= 0 && c->observer_pc[a] <= c->box_pc)) {
            set_last_error("ep_plan: observer must lie in the cube");
            return EP_ERR_INVALID_ARG;
        }
    for (int64_t s = 0; s < S; s++) {
        double d2 = 0;
        for (int a = 0; a < 3; a++) {
            const double x = xyz[3 * s + a];
            if (!std::isfinite(x) || x < 0 || x > c->box_pc) {
                set_last_error("ep_plan: star " + std::to_string(s) + " lies outside the cube or is not finite");
                return EP_ERR_INVALID_ARG;
            }
            d2 += (x - c->observer_pc[a]) * (x - c->observer_pc[a]);
        }
        if (!(std::sqrt(d2) > 1e-9 * c->box_pc)) {
            set_last_error("ep_plan: star " + std::to_string(s) + " coincides with the observer");
            return EP_ERR_INVALID_ARG;
        }
    }
    GridGeom g;
    g.n = c->n;
    g.L = c->box_pc;
    g.h = c->box_pc / (c->n - 1);
    for (int a = 0; a < 3; a++) g.obs[a] = c->observer_pc[a];
    g.step = c->los_step_pc;
    const double rho = c->vecchia_radius_pc > 0 ? c->vecchia_radius_pc : c->support_pc;
    Stencil st;
    build_stencil(g, rho, st);
    Supports sup;
    build_supports(g, S, xyz, sup);
    int64_t max_support = 0;
    for (int64_t s = 0; s < S; s++) max_support = std::max<int64_t>(max_support, sup.ptr[s + 1] - sup.ptr[s]);
    OrderingOpts opt;
    opt.leaf_size = c->leaf_size > 0 ? c->leaf_size : 512;
    opt.sep_halfwidth = std::max(rho, std::sqrt(3.0) * g.h) * (1.0 + 1e-9);
    opt.tile = TS;
    opt.panel_tiles = PW;
    Symbolic sym;
    const int rc = analyse(g, st, sup, opt, sym);
    if (rc != 0) {
        set_last_error("ep_plan: symbolic analysis failed (" + std::to_string(rc) + ")");
        return EP_ERR_STATE;
    }
    const int64_t N = g.N(), nnz = (int64_t)sup.nodes.size();
    ep_plan_stats p{};
    p.n_nodes = N;
    p.n_stars = S;
    p.nnz_g = nnz;
    p.max_support = max_support;
    p.n_fronts = (int64_t)sym.fronts.size();
    p.n_levels = sym.nlevels;
    p.max_front = sym.max_m;
    p.front_elems = sym.total_elems;
    p.factor_flops = sym.factor_flops;
    p.selinv_flops = sym.selinv_flops;
    p.trail_flops = sym.trail_flops;
    // per level: the selected inversion's scratch W holds R x V of every front
    std::vector<int64_t> wlev(sym.nlevels, 0);
    int64_t sep_max = 0;
    for (const Front& f : sym.fronts) {
        const int64_t T = f.m / TS;
        p.front_elems_lower += (int64_t)TS * TS * T * (T + 1) / 2;
        p.nnz_L += (int64_t)f.nv * (f.nv + 1) / 2 + (int64_t)f.nv * f.nr;
        p.x_elems += (int64_t)f.nvpad * f.nvpad;
        wlev[f.level] += (int64_t)TS * ((f.nr + TS - 1) / TS) * f.nvpad;
        sep_max = std::max<int64_t>(sep_max, f.nv);
    }
    p.max_separator = sep_max;
    for (int64_t w : wlev) p.w_elems = std::max(p.w_elems, w);
    // what ep_init allocates beside the fronts, X and W: every dense buffer's
    // read pad, the stars' CSR rows (node, local row, slot order, g), their
    // per-star state, the clique assembly's incidences, the node vectors, the
    // prior's rows and the Q0 scatter list (its entries on the factor's
    // pattern, about half the stencil per node); the GEMM task lists are not
    // counted
    const int64_t pad = 256 * sym.max_m + 256;
    const int64_t dense = 8 * (sym.total_elems + p.x_elems + p.w_elems + 3 * pad);
    // the clique assembly's (star, tile) incidences: a star whose slots fall
    // in r runs of 64 local rows has r (r + 1) / 2 of them, 16 bytes each,
    // plus at most 32 bytes each of partial tiles; its sorted local rows and g
    int64_t incid = 0;
    {
        std::vector<int32_t> loc;
        for (int64_t s = 0; s < S; s++) {
            loc.assign(sym.star_loc.begin() + sup.ptr[s], sym.star_loc.begin() + sup.ptr[s + 1]);
            std::sort(loc.begin(), loc.end());
            int64_t r = 0;
            for (size_t k = 0; k < loc.size(); k++)
                if (k == 0 || loc[k] / TS != loc[k - 1] / TS) r++;
            incid += r * (r + 1) / 2;
        }
    }
    const int64_t stars = nnz * (8 + 3 * 4) + S * 30 * 8 + incid * (16 + 32) + nnz * 12;
    const int64_t vectors = N * 24 * 8 + N * (int64_t)(st.full.size() / 3) * 8;
    p.device_bytes = dense + stars + vectors;
    p.device_bytes_mixed = p.device_bytes + 4 * (sym.total_elems + pad);
    *out = p;
    return EP_OK;
}
