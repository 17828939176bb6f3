// Host-side structure of the EP posterior precision: sightline supports, a
// nested-dissection ordering that is valid for both the prior stencil and
// the sightline cliques, and the multifrontal layout of the Cholesky factor.
//
// Why the ordering is special.  Every star contributes the rank-one term
// tau_n g_n g_n^T (the Gaussian site of the per-star EP factor, Sec. 4.1),
// so all nodes on one sightline form a clique, and every sightline starts
// at the observer.  A separator must therefore avoid cutting sightlines:
// planes through the observer never do, whatever their orientation, while
// planes elsewhere are only valid in parts of the volume no sightline
// reaches.  The recursion tries both kinds and keeps the smallest valid
// separator.
#include "symbolic.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

namespace ep {

static int hw_threads() {
    unsigned t = std::thread::hardware_concurrency();
    if (t == 0) t = 4;
    if (t > 32) t = 32;
    return (int)t;
}

template <class F>
static void parallel_for(int64_t n, F&& f) {
    int T = hw_threads();
    if (n < 256 || T == 1) {
        for (int64_t i = 0; i < n; i++) f(i);
        return;
    }
    std::vector<std::thread> th;
    std::atomic<int64_t> next{0};
    for (int t = 0; t < T; t++)
        th.emplace_back([&]() {
            for (;;) {
                int64_t s = next.fetch_add(64);
                if (s >= n) break;
                int64_t e = std::min<int64_t>(n, s + 64);
                for (int64_t i = s; i < e; i++) f(i);
            }
        });
    for (auto& x : th) x.join();
}

// ---------------------------------------------------------------------------
// Sightline supports.  Sample t of star n sits at o + (t/T)(x_n - o),
// T = max(1, ceil(d_n / step)); each sample touches the 8 corners of its
// grid cell (cell index clamped to [0, n-2] per axis).
// ---------------------------------------------------------------------------
static inline int64_t cell1(double s, double h, int n) {
    double c = std::floor(s / h);
    if (c < 0) c = 0;
    if (c > n - 2) c = n - 2;
    return (int64_t)c;
}

static void star_support(const GridGeom& g, const double* x, std::vector<int32_t>& out, int32_t& T) {
    double dv[3] = {x[0] - g.obs[0], x[1] - g.obs[1], x[2] - g.obs[2]};
    double d = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    double tt = std::ceil(d / g.step);
    if (tt < 1) tt = 1;
    T = (int32_t)tt;
    out.clear();
    int64_t last = -1;
    int n = g.n;
    for (int64_t t = 0; t <= T; t++) {
        double f = (double)t / (double)T;
        int64_t ci = cell1(g.obs[0] + f * dv[0], g.h, n);
        int64_t cj = cell1(g.obs[1] + f * dv[1], g.h, n);
        int64_t ck = cell1(g.obs[2] + f * dv[2], g.h, n);
        int64_t cid = ci + (int64_t)n * (cj + (int64_t)n * ck);
        if (cid == last) continue;
        last = cid;
        for (int c = 0; c < 8; c++)
            out.push_back((int32_t)((ci + (c & 1)) + (int64_t)n * ((cj + ((c >> 1) & 1)) + (int64_t)n * (ck + ((c >> 2) & 1)))));
    }
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
}

void build_supports(const GridGeom& g, int64_t n_stars, const double* xyz, Supports& sup) {
    std::vector<std::vector<int32_t>> per(n_stars);
    sup.nsamp.assign(n_stars, 0);
    parallel_for(n_stars, [&](int64_t s) { star_support(g, xyz + 3 * s, per[s], sup.nsamp[s]); });
    sup.ptr.assign(n_stars + 1, 0);
    for (int64_t s = 0; s < n_stars; s++) sup.ptr[s + 1] = sup.ptr[s] + (int64_t)per[s].size();
    sup.nodes.resize(sup.ptr[n_stars]);
    parallel_for(n_stars, [&](int64_t s) {
        std::copy(per[s].begin(), per[s].end(), sup.nodes.begin() + sup.ptr[s]);
    });
}

// ---------------------------------------------------------------------------
// Prior stencil.  A node's Vecchia conditioning set holds the earlier nodes
// (lexicographic order) within rho; Q0 = (I-B)^T D^{-1} (I-B) couples every
// two nodes that appear together in one conditioning row.
// ---------------------------------------------------------------------------
void build_stencil(const GridGeom& g, double rho, Stencil& st) {
    int R = (int)std::floor(rho / g.h) + 1;
    if (R > g.n) R = g.n;
    st.R = R;
    st.half.clear();
    double lim = rho * rho * (1.0 + 1e-9);
    for (int dk = -R; dk <= 0; dk++)
        for (int dj = -R; dj <= R; dj++)
            for (int di = -R; di <= R; di++) {
                bool neg = dk < 0 || (dk == 0 && (dj < 0 || (dj == 0 && di < 0)));
                if (!neg) continue;
                double m2 = (double)(di * di + dj * dj + dk * dk) * g.h * g.h;
                if (m2 <= lim) { st.half.push_back(di); st.half.push_back(dj); st.half.push_back(dk); }
            }
    // full stencil: differences of members of H u {0}
    std::vector<int> hz = st.half;
    hz.push_back(0); hz.push_back(0); hz.push_back(0);
    int W = 4 * R + 1;
    std::vector<char> seen((size_t)W * W * W, 0);
    st.full.clear();
    for (size_t a = 0; a < hz.size(); a += 3)
        for (size_t b = 0; b < hz.size(); b += 3) {
            int di = hz[a] - hz[b], dj = hz[a + 1] - hz[b + 1], dk = hz[a + 2] - hz[b + 2];
            size_t key = ((size_t)(dk + 2 * R) * W + (dj + 2 * R)) * W + (di + 2 * R);
            if (seen[key]) continue;
            seen[key] = 1;
            st.full.push_back(di); st.full.push_back(dj); st.full.push_back(dk);
        }
    st.pattern = st.full;
    for (int dk = -2; dk <= 2; dk++)
        for (int dj = -2; dj <= 2; dj++)
            for (int di = -2; di <= 2; di++) {   // R >= 1, so the block lies inside seen's range
                size_t key = ((size_t)(dk + 2 * R) * W + (dj + 2 * R)) * W + (di + 2 * R);
                if (seen[key]) continue;
                seen[key] = 1;
                st.pattern.push_back(di); st.pattern.push_back(dj); st.pattern.push_back(dk);
            }
}

// ---------------------------------------------------------------------------
// Nested dissection.
// ---------------------------------------------------------------------------
namespace {

struct ND {
    const GridGeom& g;
    const Supports& sup;
    const OrderingOpts& opt;
    std::vector<int32_t> stamp;
    int32_t next_stamp = 1;
    std::vector<int8_t> side;
    std::vector<int32_t> order;                    // emitted original ids, in new order
    std::vector<std::pair<int64_t, int32_t>> blocks;  // (first new index, count)

    ND(const GridGeom& g_, const Supports& s_, const OrderingOpts& o_)
        : g(g_), sup(s_), opt(o_), stamp(g_.N(), 0), side(g_.N(), 0) {}

    void coords(int32_t p, double* x) const {
        int n = g.n;
        x[0] = g.h * (double)(p % n);
        x[1] = g.h * (double)((p / n) % n);
        x[2] = g.h * (double)(p / ((int64_t)n * n));
    }

    void emit(std::vector<int32_t>& nodes) {
        if (nodes.empty()) return;
        std::sort(nodes.begin(), nodes.end());
        blocks.emplace_back((int64_t)order.size(), (int32_t)nodes.size());
        order.insert(order.end(), nodes.begin(), nodes.end());
    }

    // Evaluate the separator of plane {x : (x - pt) . nrm = 0}.
    // Returns |S| or -1 if invalid/unbalanced.
    int64_t try_plane(const std::vector<int32_t>& nodes, const std::vector<int32_t>& stars,
                      int32_t st_region, const double* pt, const double* nrm, int64_t& na, int64_t& nb) {
        double w = opt.sep_halfwidth;
        na = nb = 0;
        int64_t ns = 0;
        for (int32_t p : nodes) {
            double x[3];
            coords(p, x);
            double d = (x[0] - pt[0]) * nrm[0] + (x[1] - pt[1]) * nrm[1] + (x[2] - pt[2]) * nrm[2];
            int8_t s = (d < -w) ? 0 : (d > w ? 2 : 1);
            side[p] = s;
            if (s == 0) na++; else if (s == 2) nb++; else ns++;
        }
        int64_t tot = na + nb;
        if (na == 0 || nb == 0) return -1;
        if (std::min(na, nb) < (int64_t)(0.15 * (double)tot)) return -1;
        for (int32_t s : stars) {
            bool ha = false, hb = false;
            for (int64_t e = sup.ptr[s]; e < sup.ptr[s + 1]; e++) {
                int32_t q = sup.nodes[e];
                if (stamp[q] != st_region) continue;
                if (side[q] == 0) ha = true; else if (side[q] == 2) hb = true;
                if (ha && hb) return -1;
            }
        }
        return ns;
    }

    static double median(std::vector<double>& v) {
        size_t m = v.size() / 2;
        std::nth_element(v.begin(), v.begin() + m, v.end());
        return v[m];
    }

    void run(std::vector<int32_t>& nodes, std::vector<int32_t>& stars) {
        if ((int64_t)nodes.size() <= opt.leaf_size) { emit(nodes); return; }
        int32_t st = next_stamp++;
        for (int32_t p : nodes) stamp[p] = st;
        // candidate planes
        struct Cand { double pt[3], nrm[3]; };
        std::vector<Cand> cands;
        std::vector<double> vals(nodes.size());
        for (int a = 0; a < 3; a++) {
            for (size_t i = 0; i < nodes.size(); i++) { double x[3]; coords(nodes[i], x); vals[i] = x[a]; }
            double med = median(vals);
            double c = (std::floor(med / g.h) + 0.5) * g.h;
            Cand cd{};
            cd.pt[a] = c;
            cd.nrm[a] = 1.0;
            cands.push_back(cd);
        }
        // planes through the observer: rotate about z, about x and about y
        const int ax[3][2] = {{0, 1}, {1, 2}, {0, 2}};
        for (int r = 0; r < 3; r++) {
            int u = ax[r][0], v = ax[r][1];
            for (size_t i = 0; i < nodes.size(); i++) {
                double x[3];
                coords(nodes[i], x);
                vals[i] = std::atan2(x[v] - g.obs[v], x[u] - g.obs[u]);
            }
            double th = median(vals);
            Cand cd{};
            for (int k = 0; k < 3; k++) cd.pt[k] = g.obs[k];
            cd.nrm[u] = -std::sin(th);
            cd.nrm[v] = std::cos(th);
            cands.push_back(cd);
        }
        int best = -1;
        int64_t bestS = -1;
        for (size_t c = 0; c < cands.size(); c++) {
            int64_t na, nb;
            int64_t s = try_plane(nodes, stars, st, cands[c].pt, cands[c].nrm, na, nb);
            if (s < 0) continue;
            if (best < 0 || s < bestS) { best = (int)c; bestS = s; }
        }
        if (best < 0) { emit(nodes); return; }
        int64_t na, nb;
        try_plane(nodes, stars, st, cands[best].pt, cands[best].nrm, na, nb);
        std::vector<int32_t> A, B, S;
        A.reserve(na); B.reserve(nb); S.reserve(bestS);
        for (int32_t p : nodes) {
            if (side[p] == 0) A.push_back(p); else if (side[p] == 2) B.push_back(p); else S.push_back(p);
        }
        std::vector<int32_t> sA, sB;
        for (int32_t s : stars) {
            bool ha = false, hb = false;
            for (int64_t e = sup.ptr[s]; e < sup.ptr[s + 1]; e++) {
                int32_t q = sup.nodes[e];
                if (stamp[q] != st) continue;
                if (side[q] == 0) ha = true; else if (side[q] == 2) hb = true;
            }
            if (ha) sA.push_back(s);
            if (hb) sB.push_back(s);
        }
        std::vector<int32_t>().swap(nodes);
        std::vector<int32_t>().swap(stars);
        run(A, sA);
        run(B, sB);
        emit(S);
    }
};

}  // namespace

static inline int32_t front_local(const Symbolic& sym, const Front& f, int64_t newidx) {
    if (newidx >= f.first && newidx < f.first + f.nv) return (int32_t)(newidx - f.first);
    const int64_t* b = sym.rrows.data() + f.rptr;
    const int64_t* e = b + f.nr;
    const int64_t* it = std::lower_bound(b, e, newidx);
    if (it == e || *it != newidx) return -1;
    return f.nvpad + (int32_t)(it - b);
}

int analyse(const GridGeom& g, const Stencil& st, const Supports& sup, const OrderingOpts& opt, Symbolic& sym) {
    const int64_t N = g.N();
    const int64_t S = (int64_t)sup.ptr.size() - 1;
    const int T = opt.tile;
    sym.tile = T;
    // ---- ordering ----
    ND nd(g, sup, opt);
    {
        std::vector<int32_t> all(N), stars(S);
        std::iota(all.begin(), all.end(), 0);
        std::iota(stars.begin(), stars.end(), 0);
        nd.run(all, stars);
    }
    if ((int64_t)nd.order.size() != N) return -1;
    sym.perm = nd.order;
    sym.iperm.assign(N, 0);
    for (int64_t i = 0; i < N; i++) sym.iperm[sym.perm[i]] = (int32_t)i;
    const int64_t nf = (int64_t)nd.blocks.size();
    sym.fronts.assign(nf, Front{});
    sym.snode.assign(N, 0);
    for (int64_t f = 0; f < nf; f++) {
        sym.fronts[f].first = nd.blocks[f].first;
        sym.fronts[f].nv = nd.blocks[f].second;
        sym.fronts[f].nvpad = (nd.blocks[f].second + T - 1) / T * T;
        for (int32_t k = 0; k < nd.blocks[f].second; k++) sym.snode[nd.blocks[f].first + k] = (int32_t)f;
    }
    // ---- stars: the front of each clique's first node ----
    sym.star_front.assign(S, 0);
    std::vector<std::vector<int32_t>> stars_of(nf);
    for (int64_t s = 0; s < S; s++) {
        int64_t mn = INT64_MAX;
        for (int64_t e = sup.ptr[s]; e < sup.ptr[s + 1]; e++) mn = std::min<int64_t>(mn, sym.iperm[sup.nodes[e]]);
        int32_t f = (sup.ptr[s + 1] > sup.ptr[s]) ? sym.snode[mn] : 0;
        sym.star_front[s] = f;
        stars_of[f].push_back((int32_t)s);
    }
    // ---- symbolic multifrontal: R_s, parents ----
    std::vector<std::vector<int64_t>> pending(nf);
    std::vector<std::vector<int64_t>> R(nf);
    std::vector<int64_t> mark(N, -1);
    const int n = g.n;
    for (int64_t f = 0; f < nf; f++) {
        Front& F = sym.fronts[f];
        int64_t last = F.first + F.nv - 1;
        std::vector<int64_t> cand;
        cand.swap(pending[f]);
        auto add = [&](int64_t x) {
            if (x > last && mark[x] != f) { mark[x] = f; cand.push_back(x); }
        };
        {   // dedupe what the children passed up
            std::vector<int64_t> c2;
            c2.swap(cand);
            for (int64_t x : c2) add(x);
        }
        for (int32_t k = 0; k < F.nv; k++) {
            int32_t p = sym.perm[F.first + k];
            int i = p % n, j = (p / n) % n, l = p / (n * n);
            for (size_t o = 0; o < st.pattern.size(); o += 3) {
                int ii = i + st.pattern[o], jj = j + st.pattern[o + 1], ll = l + st.pattern[o + 2];
                if (ii < 0 || jj < 0 || ll < 0 || ii >= n || jj >= n || ll >= n) continue;
                add(sym.iperm[ii + (int64_t)n * (jj + (int64_t)n * ll)]);
            }
        }
        for (int32_t s : stars_of[f])
            for (int64_t e = sup.ptr[s]; e < sup.ptr[s + 1]; e++) add(sym.iperm[sup.nodes[e]]);
        std::sort(cand.begin(), cand.end());
        R[f].swap(cand);
        F.nr = (int32_t)R[f].size();
        if (F.nr > 0) {
            int32_t p = sym.snode[R[f][0]];
            F.parent = p;
            const Front& P = sym.fronts[p];
            for (int64_t x : R[f])
                if (x >= P.first + P.nv) pending[p].push_back(x);
        } else {
            F.parent = -1;
        }
    }
    // ---- layout ----
    int64_t off = 0, rp = 0;
    sym.total_elems = 0;
    sym.factor_flops = sym.selinv_flops = sym.trail_flops = 0;
    const int64_t panel_cols = (int64_t)opt.tile * opt.panel_tiles;
    sym.max_m = 0;
    for (int64_t f = 0; f < nf; f++) {
        Front& F = sym.fronts[f];
        F.m = F.nvpad + (F.nr + T - 1) / T * T;
        F.off = off;
        off += (int64_t)F.m * F.m;
        F.rptr = rp;
        rp += F.nr;
        double nv = F.nv, mm = F.nv + F.nr, nr = F.nr;
        sym.factor_flops += (mm * mm * mm - (mm - nv) * (mm - nv) * (mm - nv)) / 3.0;
        sym.selinv_flops += 2.0 * nv * nv * nv / 3.0 + 2.0 * nr * nv * nv + 2.0 * nr * nr * nv;
        // trailing update after each panel of panel_cols pivot columns: the
        // lower triangle of the remaining R x R block, rank w
        for (int64_t c0 = 0; c0 < F.nv; c0 += panel_cols) {
            const double w = (double)(std::min<int64_t>(F.nv, c0 + panel_cols) - c0);
            const double R = mm - (double)std::min<int64_t>(F.nv, c0 + panel_cols);
            sym.trail_flops += w * R * (R + 1.0);
        }
        sym.max_m = std::max<int64_t>(sym.max_m, F.m);
    }
    sym.total_elems = off;
    sym.rrows.resize(rp);
    for (int64_t f = 0; f < nf; f++)
        std::copy(R[f].begin(), R[f].end(), sym.rrows.begin() + sym.fronts[f].rptr);
    // levels (children have lower indices than parents)
    sym.nlevels = 0;
    for (int64_t f = 0; f < nf; f++) {
        Front& F = sym.fronts[f];
        if (F.parent >= 0) {
            Front& P = sym.fronts[F.parent];
            P.level = std::max(P.level, F.level + 1);
        }
        sym.nlevels = std::max(sym.nlevels, F.level + 1);
    }
    // relative maps into the parent
    sym.relmap.assign(rp, -1);
    for (int64_t f = 0; f < nf; f++) {
        const Front& F = sym.fronts[f];
        if (F.parent < 0) continue;
        const Front& P = sym.fronts[F.parent];
        for (int32_t k = 0; k < F.nr; k++) {
            int32_t l = front_local(sym, P, sym.rrows[F.rptr + k]);
            if (l < 0) return -2;   // structure is not closed: a bug
            sym.relmap[F.rptr + k] = l;
        }
    }
    // star local rows
    sym.star_loc.assign(sup.nodes.size(), 0);
    int bad = 0;
    for (int64_t s = 0; s < S; s++) {
        const Front& F = sym.fronts[sym.star_front[s]];
        for (int64_t e = sup.ptr[s]; e < sup.ptr[s + 1]; e++) {
            int32_t l = front_local(sym, F, sym.iperm[sup.nodes[e]]);
            if (l < 0) bad = 1;
            sym.star_loc[e] = l;
        }
    }
    if (bad) return -3;
    return 0;
}

}  // namespace ep
