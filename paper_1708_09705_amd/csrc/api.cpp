// C ABI of the EP library: context set-up (host analysis + device upload),
// the sweep driver and the outputs.  Every numerical step of the sweep runs
// in the HIP kernels of kernels.hip; the host only enqueues them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <unordered_map>
#include <map>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/ep.h"
#include "kernels.h"
#include "pitc.h"
#include "task_order.h"
#include "prior.h"
#include "surrogate.h"
#include "symbolic.h"

using namespace ep;

namespace {
// roctx range over a host-side scope (visible with rocprofv3 --marker-trace)
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};
}  // namespace

static thread_local std::string g_tls_err = "no error";
namespace ep {
void set_last_error(const std::string& m) { g_tls_err = m; }
}

namespace {

struct Launch {   // a batch of implicitly enumerated tile tasks
    int64_t be_off = 0;
    int nbe = 0;
    int64_t ntasks = 0;
};
struct FList {
    int64_t off = 0;
    int n = 0;
};
struct TaskRange {
    int64_t off = 0;
    int64_t n = 0;
    bool a32 = false;   // some task reads its A operand from the FP32 factor copy
};
struct LevelPlan {
    std::vector<FList> potrf;   // per pivot step
    std::vector<Launch> trsm, inner;
    std::vector<TaskRange> trail32;   // FP32 levels: after a panel ending at step k, its trailing update (FP32 tasks)
    // FP64 levels, left-looking by panel, as 256 x 128 GEMM tasks:
    // panelT[k]: before step k (a panel start), the panel's columns take the
    //            updates of every earlier panel;
    // finalT[k]: after step k (a front's last pivot step), the update block
    //            takes the updates of all pivot columns.
    std::vector<TaskRange> panelT, finalT;
    Launch extend;              // also the Sigma-gather enumeration
    std::vector<Launch> extend_groups;   // the same fronts, at most one child per parent in each group
    Launch conv;                // FP64 -> FP32 copy of the level's fronts (mixed precision)
    Launch fwd_xv, fwd_r, bwd_t, bwd_x;
    FList fronts;
    TaskRange selW, selS21, selS11;
};

}  // namespace

struct ep_ctx {
    ep_config cfg{};
    GridGeom g;
    PriorParams pp;
    Stencil st;
    Vecchia vec;
    Supports sup;
    Symbolic sym;
    int64_t S = 0;
    int max_support = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err = "no error";
    int64_t dev_bytes = 0;
    std::vector<void*> allocs;
    int64_t n_cu = 256;   // compute units of the device (the GEMM schedules' round size)
    // clique assembly by tile owner: incidences, chunks, multi-chunk tiles,
    // partial tiles, local rows in each star's sorted slot order, and g in
    // that order (refreshed every sweep)
    TileInc* d_tinc = nullptr;
    TileChunk* d_tch = nullptr;
    TileRed* d_tred = nullptr;
    double *d_tpart = nullptr, *d_gsort = nullptr;
    int32_t* d_lsort = nullptr;
    int64_t n_tch = 0, n_tred = 0;
    // deterministic mode: right-hand-side node lists, the forward solve's
    // per-level update lists and their staging vector
    int32_t* d_nstar = nullptr;
    int64_t *d_nptr = nullptr, *d_nslot = nullptr;
    double* d_stage = nullptr;
    struct DetLevel {
        int64_t n = 0;
        int32_t* tgt = nullptr;
        int64_t *tptr = nullptr, *src = nullptr;
    };
    std::vector<DetLevel> det_lv;

    std::vector<int64_t> xoff;   // X block offset per front
    double *d_fronts = nullptr, *d_X = nullptr, *d_W = nullptr;
    int64_t W_elems = 0, X_elems = 0;
    int64_t *d_off = nullptr, *d_first = nullptr, *d_rptr = nullptr, *d_xoff = nullptr;
    int32_t *d_m = nullptr, *d_nv = nullptr, *d_nvpad = nullptr, *d_nr = nullptr, *d_parent = nullptr;
    int32_t *d_rrows = nullptr, *d_relmap = nullptr, *d_perm = nullptr, *d_snode = nullptr;
    int64_t *d_q0_dest = nullptr, *d_pad_dest = nullptr;
    double* d_q0_val = nullptr;
    int64_t n_q0 = 0, n_pad = 0;
    int32_t* d_flists = nullptr;
    BatchEnt* d_batches = nullptr;
    GemmTask* d_tasks = nullptr;
    int* d_err = nullptr;
    double *d_xyz = nullptr, *d_A = nullptr, *d_sigma = nullptr, *d_g = nullptr, *d_lnA = nullptr, *d_c = nullptr;
    double *d_tau = nullptr, *d_nu = nullptr, *d_cmu = nullptr, *d_cvar = nullptr, *d_lnZ = nullptr;
    double *d_tmean = nullptr, *d_tvar = nullptr, *d_dtau = nullptr;
    double *d_tau_bak = nullptr, *d_nu_bak = nullptr;
    int64_t* d_sptr = nullptr;
    int32_t *d_snodes = nullptr, *d_sloc = nullptr, *d_sord = nullptr, *d_sfront = nullptr, *d_nsamp = nullptr;
    int32_t* d_status = nullptr;
    double *d_fhat = nullptr, *d_b0 = nullptr, *d_borig = nullptr, *d_y = nullptr, *d_x = nullptr, *d_t = nullptr;
    double *d_mu = nullptr, *d_var = nullptr;
    // mixed precision: FP32 copy of the fronts, prior factor for the residual
    float* d_f32 = nullptr;
    int64_t *d_brp = nullptr;
    int32_t* d_bcol = nullptr;
    double *d_bval = nullptr, *d_bd = nullptr, *d_u = nullptr, *d_w = nullptr, *d_r = nullptr, *d_dx = nullptr;
    int ir_iters = 0;
    double ir_res = 0;
    // tilted-moment surrogate
    float* d_mlp_P = nullptr;
    short* d_mlp_bf = nullptr;
    int32_t *d_fb_list = nullptr, *d_fb_count = nullptr;
    // map prediction (allocated at first use)
    int32_t *d_iperm = nullptr, *d_mapT = nullptr;
    double *d_cellS = nullptr, *d_s1 = nullptr, *d_s2 = nullptr, *d_mapmean = nullptr;
    double* d_pts = nullptr;
    int64_t pts_cap = 0;
    int* d_mapbad = nullptr;
    bool mlp_loaded = false;
    int64_t fallbacks = 0;
    // inferred prior-mean parameters (mean_fn DISC_BUMP): M = 5, else 0
    int M = 0;
    double mu0[NTHETA] = {}, s0sq[NTHETA] = {};   // hyperprior of phi = ln theta
    double phihat[NTHETA] = {};                   // mean linearisation point
    BorderDev border{};                           // mu_phi, phihat, Sigma_phiphi of the last border solve
    double *d_mhat = nullptr, *d_J = nullptr, *d_h = nullptr, *d_R = nullptr, *d_Wb = nullptr, *d_part = nullptr;
    // unknown distances (likelihood GMM): per-star mixtures (ep_set_gmm) and the
    // largest sample count of the sightlines extended to the cube's face
    int32_t* d_order = nullptr;   // clique kernels' star order (XCD pieces)
    int64_t n_order = 0;
    int gmm_K = 0;
    double* d_gmm = nullptr;
    int64_t gmm_kcap = 0;
    // multi-vector solves (border columns, batches of posterior draws): MR_MAX x N each, at first use
    double *d_ymr = nullptr, *d_tmr = nullptr, *d_xmr = nullptr, *d_omr = nullptr;
    // PITC sub-catalogue pass (ep_pitc_setup)
    PitcState* pitc = nullptr;

    std::vector<LevelPlan> levels;
    Launch zero_lower;                       // lower tiles of all fronts
    std::vector<TaskRange> trtri1, trtri1f, trtri2;   // per doubling stage (1f: FP32 factor copy)
    bool linearised = false;                 // g, c valid for the current fhat (frozen modes)
    std::vector<hipEvent_t> kt_ev;           // per-launch timing events (profile_kernels)
    size_t kt_used = 0;
    std::vector<int> kt_kind;                // EP_KK_* of each timed launch

    FrontsDev F{};
    StarsDev SD{};
    GridDev GD{};
};

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ctx->err = std::string("HIP error ") + hipGetErrorString(e_) + " at " #expr; \
            return EP_ERR_DEVICE;                                                        \
        }                                                                                \
    } while (0)

#define TRY(x)                      \
    do {                            \
        int r_ = (x);               \
        if (r_ != EP_OK) return r_; \
    } while (0)

template <class T>
static int dev_alloc(ep_ctx* ctx, T** p, int64_t count) {
    int64_t bytes = std::max<int64_t>(count, 1) * (int64_t)sizeof(T);
    if (ctx->cfg.hbm_cap_bytes > 0 && ctx->dev_bytes + bytes > ctx->cfg.hbm_cap_bytes) {
        ctx->err = "device allocation of " + std::to_string(bytes) + " bytes exceeds hbm_cap_bytes";
        return EP_ERR_OOM;
    }
    hipError_t e = hipMalloc((void**)p, (size_t)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ctx->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
        return EP_ERR_OOM;
    }
    ctx->dev_bytes += bytes;
    ctx->allocs.push_back((void*)*p);
    return EP_OK;
}

template <class T>
static int upload(ep_ctx* ctx, T** p, const std::vector<T>& v) {
    TRY(dev_alloc(ctx, p, (int64_t)v.size()));
    if (!v.empty()) HIPCHK(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return EP_OK;
}

static int32_t front_local(const Symbolic& sym, const Front& f, int64_t newidx) {
    if (newidx >= f.first && newidx < f.first + f.nv) return (int32_t)(newidx - f.first);
    const int64_t* b = sym.rrows.data() + f.rptr;
    const int64_t* e = b + f.nr;
    const int64_t* it = std::lower_bound(b, e, newidx);
    if (it == e || *it != newidx) return -1;
    return f.nvpad + (int32_t)(it - b);
}

static bool is_f32_level(const ep_ctx* ctx, int level) {
    return ctx->cfg.precision == EP_PREC_MIXED && level < ctx->sym.nlevels - ctx->cfg.mixed_fp64_levels;
}

static GemmSeg mkseg(int bufA, int64_t a, int64_t sa, int lda, bool ta, bool neg, int bufB, int64_t b, int64_t sb,
                     int ldb, bool tb, int nk) {
    GemmSeg s{};
    s.a = a;
    s.sa = sa;
    s.lda = lda;
    s.b = b;
    s.sb = sb;
    s.ldb = ldb;
    s.nk = nk;
    s.flags = (ta ? 1 : 0) | (tb ? 2 : 0) | (neg ? 4 : 0) | (bufA << 8) | (bufB << 10);
    return s;
}

static void balance_range(std::vector<GemmTask>& tasks, TaskRange& r) { balance_xcd(tasks, r.off, r.n); }

// ---------------------------------------------------------------------------
// Schedules.  All tile addresses are absolute element offsets into their
// buffer (fronts, X = diagonal-block inverses, W = scratch).
//   front f, tile (i, j):       off_f + 64 i + 64 j m_f
//   X block of f, tile (i, j):  xoff_f + 64 i + 64 j nvpad_f
// ---------------------------------------------------------------------------
static int build_plans(ep_ctx* ctx, std::vector<int32_t>& flists, std::vector<BatchEnt>& batches,
                       std::vector<GemmTask>& tasks) {
    const Symbolic& sym = ctx->sym;
    const int64_t nf = (int64_t)sym.fronts.size();
    const int L = sym.nlevels;
    // where each front's factor lives: FP32 copy in mixed precision, except
    // in the top mixed_fp64_levels levels of the dissection tree
    auto Lbuf_of = [&](int f) { return is_f32_level(ctx, sym.fronts[f].level) ? (int)BUF_F32 : (int)BUF_FRONTS; };
    // X layout
    ctx->xoff.assign(nf, 0);
    int64_t xo = 0;
    for (int64_t f = 0; f < nf; f++) {
        ctx->xoff[f] = xo;
        xo += (int64_t)sym.fronts[f].nvpad * sym.fronts[f].nvpad;
    }
    ctx->X_elems = std::max<int64_t>(xo, 1);
    std::vector<std::vector<int32_t>> lv(L);
    for (int64_t f = 0; f < nf; f++) lv[sym.fronts[f].level].push_back((int32_t)f);
    auto P_of = [&](int f) { return sym.fronts[f].nvpad / TS; };
    auto M_of = [&](int f) { return sym.fronts[f].m / TS; };
    auto MR_of = [&](int f) { return (sym.fronts[f].nr + TS - 1) / TS; };
    auto mk_launch = [&](const std::vector<std::pair<int, int64_t>>& fc) {
        Launch l;
        l.be_off = (int64_t)batches.size();
        int64_t base = 0;
        for (auto& x : fc) {
            if (x.second <= 0) continue;
            BatchEnt e{};
            e.front = x.first;
            e.base = base;
            batches.push_back(e);
            base += x.second;
        }
        l.nbe = (int)((int64_t)batches.size() - l.be_off);
        l.ntasks = base;
        return l;
    };
    ctx->levels.assign(L, LevelPlan{});
    int64_t Wmax = 0;
    for (int l = 0; l < L; l++) {
        LevelPlan& P = ctx->levels[l];
        int Pmax = 0;
        for (int f : lv[l]) Pmax = std::max(Pmax, P_of(f));
        // Blocked partial Cholesky, panels of PW tiles:
        //   step k: diagonal tile, column below it, then column k + 1 of the
        //   panel takes the updates of the panel's pivots up to k (K = k + 1
        //   - panel start); the columns of later panels take their updates
        //   in GEMM tasks.
        for (int k = 0; k < Pmax; k++) {
            FList fl;
            fl.off = (int64_t)flists.size();
            std::vector<std::pair<int, int64_t>> tr, in;
            const int g = k / PW;
            for (int f : lv[l]) {
                const int Pf = P_of(f), M = M_of(f);
                if (Pf <= k) continue;
                flists.push_back(f);
                tr.emplace_back(f, (int64_t)(M - k - 1));
                const int gend = std::min(PW * (g + 1), Pf);
                in.emplace_back(f, k + 1 < gend ? (int64_t)(M - k - 1) : 0);
            }
            fl.n = (int)((int64_t)flists.size() - fl.off);
            P.potrf.push_back(fl);
            P.trsm.push_back(mk_launch(tr));
            P.inner.push_back(mk_launch(in));

            // left-looking updates as 256 x 128 block tasks (four row tiles x
            // two column tiles), C(i, j) -= sum over K of L(i, kk) L(j, kk)^T
            // for j <= i < M; blocks straddling the diagonal store only their
            // lower quadrants
            // split > 1 cuts K into that many pieces that add into C
            // atomically (used when a launch has too few blocks to fill the
            // GPU)
            auto lower_count = [&](int f, int j0, int j1) {
                const int M = M_of(f);
                int64_t c = 0;
                for (int i = j0; i < M; i += 4)
                    for (int j = j0; j < j1 && j <= i + 3; j += 2) c++;
                return c;
            };
            auto lower_tasks = [&](int f, int j0, int j1, int kk0, int kk1, int split, int buf = BUF_FRONTS) {
                const Front& Fr = sym.fronts[f];
                const int M = M_of(f);
                const int64_t m = Fr.m;
                const int nk = kk1 - kk0;
                for (int i = j0; i < M; i += 4)
                    for (int j = j0; j < j1 && j <= i + 3; j += 2)
                        for (int sp = 0; sp < split; sp++) {
                            const int a0 = kk0 + (int)((int64_t)nk * sp / split);
                            const int a1 = kk0 + (int)((int64_t)nk * (sp + 1) / split);
                            if (a1 <= a0) continue;
                            GemmTask t{};
                            t.c = Fr.off + TS * i + TS * j * m;
                            t.ldc = (int32_t)m;
                            t.flags = (split > 1 ? 2 : 0) | (1 << 4) | (buf << 8) |
                                      gt_shape(std::min(4, M - i), j + 1 < j1, true, i - j, false);
                            t.s[0] = mkseg(buf, Fr.off + TS * i + TS * a0 * m, TS * m, (int)m, false, true, buf,
                                           Fr.off + TS * j + TS * a0 * m, TS * m, (int)m, true, a1 - a0);
                            tasks.push_back(t);
                        }
            };
            // K pieces per block: the launch's blocks are dealt to the CUs in
            // rounds (one block per CU at a time), so with equal tasks its
            // time is rounds x (per-task start and store + K tiles per
            // piece); the start and store cost about two K tiles.  Pieces of
            // at least 4 tiles; none in the deterministic mode (the pieces add
            // atomically).
            const bool nosplit = ctx->cfg.deterministic != 0;
            const int64_t ncu = ctx->n_cu;
            auto split_for = [nosplit, ncu](int64_t nblocks, int nk) {
                if (nblocks <= 0 || nosplit) return 1;
                int best = 1;
                double tbest = 1e300;
                for (int sp = 1; sp <= std::max(1, nk / 4); sp++) {
                    const int64_t rounds = (nblocks * sp + ncu - 1) / ncu;
                    const double t = (double)rounds * (2.0 + (double)((nk + sp - 1) / sp));
                    if (t < tbest * (1.0 - 1e-9)) {
                        tbest = t;
                        best = sp;
                    }
                }
                return best;
            };
            TaskRange pt, ft;
            pt.off = (int64_t)tasks.size();
            if (!is_f32_level(ctx, l)) {
                int64_t nb = 0;
                for (int f : lv[l]) {
                    const int Pf = P_of(f);
                    if (Pf <= k || k % PW != 0 || k == 0) continue;
                    nb += lower_count(f, k, std::min(k + PW, Pf));
                }
                const int sp = split_for(nb, k);
                for (int f : lv[l]) {
                    const int Pf = P_of(f);
                    if (Pf <= k || k % PW != 0 || k == 0) continue;
                    lower_tasks(f, k, std::min(k + PW, Pf), 0, k, sp);
                }
            }
            pt.n = (int64_t)tasks.size() - pt.off;
            balance_range(tasks, pt);
            P.panelT.push_back(pt);
            ft.off = (int64_t)tasks.size();
            if (!is_f32_level(ctx, l)) {
                int64_t nb = 0;
                int nkmin = 1 << 30;
                for (int f : lv[l]) {
                    const int Pf = P_of(f), M = M_of(f);
                    if (Pf - 1 != k || M == Pf) continue;
                    nb += lower_count(f, Pf, M);
                    nkmin = std::min(nkmin, Pf);
                }
                const int sp = nb > 0 ? split_for(nb, nkmin) : 1;
                for (int f : lv[l]) {
                    const int Pf = P_of(f), M = M_of(f);
                    if (Pf - 1 != k || M == Pf) continue;
                    lower_tasks(f, Pf, M, 0, Pf, sp);
                }
            }
            ft.n = (int64_t)tasks.size() - ft.off;
            balance_range(tasks, ft);
            P.finalT.push_back(ft);
            // FP32 levels, right-looking by panel: after the panel ending at
            // step k, its trailing update as FP32 MFMA block tasks
            TaskRange t32;
            t32.off = (int64_t)tasks.size();
            if (is_f32_level(ctx, l))
                for (int f : lv[l]) {
                    const int Pf = P_of(f), M = M_of(f);
                    if (Pf <= k) continue;
                    const int gend = std::min(PW * (k / PW + 1), Pf);
                    if (gend - 1 == k && M > gend) lower_tasks(f, gend, M, PW * (k / PW), gend, 1, BUF_F32);
                }
            t32.n = (int64_t)tasks.size() - t32.off;
            balance_range(tasks, t32);
            P.trail32.push_back(t32);
        }
        std::vector<std::pair<int, int64_t>> ea, fx, fr;
        for (int f : lv[l]) {
            int64_t MR = MR_of(f);
            if (sym.fronts[f].parent >= 0) ea.emplace_back(f, MR * (MR + 1) / 2);
            fx.emplace_back(f, P_of(f));
            fr.emplace_back(f, MR);
        }
        // the in-panel update of step k factors step k + 1's diagonal tiles
        // inside a panel: its launch must hold exactly that step's fronts
        for (int k = 0; k + 1 < (int)P.potrf.size(); k++) {
            if ((k + 1) % PW == 0) continue;
            const Launch& in = P.inner[k];
            const FList& nx = P.potrf[k + 1];
            if (in.nbe != nx.n) return EP_ERR_INVALID_ARG;
            for (int q = 0; q < in.nbe; q++)
                if (batches[in.be_off + q].front != flists[nx.off + q]) return EP_ERR_INVALID_ARG;
        }
        P.extend = mk_launch(ea);
        {   // group r: the r-th child (in this level) of every parent
            std::map<int, int> rank;
            std::vector<std::vector<std::pair<int, int64_t>>> groups;
            for (auto& x : ea) {
                const int r = rank[sym.fronts[x.first].parent]++;
                if ((int)groups.size() <= r) groups.resize(r + 1);
                groups[r].push_back(x);
            }
            for (auto& gv : groups) P.extend_groups.push_back(mk_launch(gv));
        }
        std::vector<std::pair<int, int64_t>> cv;
        for (int f : lv[l]) cv.emplace_back(f, M_of(f));
        P.conv = mk_launch(cv);
        P.fwd_xv = mk_launch(fx);
        P.fwd_r = mk_launch(fr);
        P.bwd_t = mk_launch(fx);
        P.bwd_x = mk_launch(fx);
        P.fronts.off = (int64_t)flists.size();
        for (int f : lv[l]) flists.push_back(f);
        P.fronts.n = (int)lv[l].size();

        // ---- selected inversion of the level's fronts ----
        //   W    = L21 X                  (R x V, scratch)
        //   S21  = -S22 W                 (overwrites L21)
        //   S11  = X^T X - W^T S21        (overwrites L11)
        std::vector<int64_t> wbase(lv[l].size());
        int64_t wb = 0;
        for (size_t q = 0; q < lv[l].size(); q++) {
            wbase[q] = wb;
            wb += (int64_t)TS * MR_of(lv[l][q]) * (int64_t)sym.fronts[lv[l][q]].nvpad;
        }
        Wmax = std::max(Wmax, wb);
        // Tasks are 256 x 128 blocks: four row tiles x two column tiles.
        // Where a block's later tiles lie in the upper triangle of a
        // lower-triangular operand, that operand is zero there (X holds zeros
        // above its diagonal), so a block shares its first tile's K range.
        P.selW.off = (int64_t)tasks.size();
        for (size_t q = 0; q < lv[l].size(); q++) {
            const int f = lv[l][q];
            const Front& Fr = sym.fronts[f];
            const int Pf = P_of(f), MR = MR_of(f);
            const int64_t ldw = (int64_t)TS * MR, m = Fr.m, xb = ctx->xoff[f], nvp = Fr.nvpad;
            for (int i = 0; i < MR; i += 4)
                for (int k = 0; k < Pf; k += 2) {
                    GemmTask t{};
                    t.c = wbase[q] + TS * i + TS * k * ldw;
                    t.ldc = (int32_t)ldw;
                    t.flags = 1 | (1 << 4) | (BUF_W << 8) | gt_shape(std::min(4, MR - i), k + 1 < Pf, false, 0, false);
                    // sum_{j=k}^{P-1} L(R_i, j) X(j, k)
                    t.s[0] = mkseg(Lbuf_of(f), Fr.off + nvp + TS * i + TS * k * m, TS * m, (int)m, false, false, BUF_X,
                                   xb + TS * k + TS * k * nvp, TS, (int)nvp, false, Pf - k);
                    tasks.push_back(t);
                }
        }
        P.selW.n = (int64_t)tasks.size() - P.selW.off;
        P.selW.a32 = is_f32_level(ctx, l);
        balance_range(tasks, P.selW);
        // S21 = -S22 W, computed transposed: S21^T(k, i) = -sum_l W(l, k) S22(l, i),
        // four pivot tiles k x two update tiles i per block, stored transposed
        P.selS21.off = (int64_t)tasks.size();
        for (size_t q = 0; q < lv[l].size(); q++) {
            const int f = lv[l][q];
            const Front& Fr = sym.fronts[f];
            const int Pf = P_of(f), MR = MR_of(f);
            const int64_t ldw = (int64_t)TS * MR, m = Fr.m, nvp = Fr.nvpad;
            for (int k = 0; k < Pf; k += 4)
                for (int i = 0; i < MR; i += 2) {
                    GemmTask t{};
                    t.c = Fr.off + nvp + TS * i + TS * k * m;
                    t.ldc = (int32_t)m;
                    int nseg = 0;
                    // l <= i: S22(l, i) = tile (i, l) as stored, transposed
                    t.s[nseg++] = mkseg(BUF_W, wbase[q] + TS * k * ldw, TS, (int)ldw, true, true, BUF_FRONTS,
                                        Fr.off + nvp + TS * i + nvp * m, TS * m, (int)m, true, i + 1);
                    // l > i: tiles (l, i), (l, i+1) as stored; at l = i+1 the
                    // second is the (symmetric, fully stored) diagonal tile
                    if (i + 1 < MR)
                        t.s[nseg++] = mkseg(BUF_W, wbase[q] + TS * (i + 1) + TS * k * ldw, TS, (int)ldw, true, true,
                                            BUF_FRONTS, Fr.off + nvp + TS * (i + 1) + (nvp + TS * i) * m, TS, (int)m,
                                            false, MR - i - 1);
                    t.flags = 1 | (nseg << 4) | (BUF_FRONTS << 8) |
                              gt_shape(std::min(4, Pf - k), i + 1 < MR, false, 0, true);
                    tasks.push_back(t);
                }
        }
        P.selS21.n = (int64_t)tasks.size() - P.selS21.off;
        balance_range(tasks, P.selS21);
        P.selS11.off = (int64_t)tasks.size();
        for (size_t q = 0; q < lv[l].size(); q++) {
            const int f = lv[l][q];
            const Front& Fr = sym.fronts[f];
            const int Pf = P_of(f), MR = MR_of(f);
            const int64_t ldw = (int64_t)TS * MR, m = Fr.m, xb = ctx->xoff[f], nvp = Fr.nvpad;
            for (int k = 0; k < Pf; k += 4)
                for (int j = 0; j < Pf && j <= k + 3; j += 2) {
                    GemmTask t{};
                    t.c = Fr.off + TS * k + TS * j * m;
                    t.ldc = (int32_t)m;
                    int nseg = 0;
                    // sum_{r=k}^{P-1} X(r, k)^T X(r, j)
                    t.s[nseg++] = mkseg(BUF_X, xb + TS * k + TS * k * nvp, TS, (int)nvp, true, false, BUF_X,
                                        xb + TS * k + TS * j * nvp, TS, (int)nvp, false, Pf - k);
                    // - sum_i W(i, k)^T S21(i, j)
                    if (MR > 0)
                        t.s[nseg++] = mkseg(BUF_W, wbase[q] + TS * k * ldw, TS, (int)ldw, true, true, BUF_FRONTS,
                                            Fr.off + nvp + TS * j * m, TS, (int)m, false, MR);
                    t.flags = 1 | (nseg << 4) | (BUF_FRONTS << 8) |
                              gt_shape(std::min(4, Pf - k), j + 1 < Pf, true, k - j, false);
                    tasks.push_back(t);
                }
        }
        P.selS11.n = (int64_t)tasks.size() - P.selS11.off;
        balance_range(tasks, P.selS11);
    }
    // ---- inverse of each L11 by doubling over all fronts ----
    // blocks [t0, b0) (top, inverted) and [b0, b1) (bottom, inverted):
    //   T   = L(bot, top) X(top, top)        (scratch W)
    //   X21 = - X(bot, bot) T
    int64_t Tmax = 0;
    int Pall = 0;
    for (int64_t f = 0; f < nf; f++) Pall = std::max(Pall, P_of((int)f));
    for (int b = 1; b < Pall; b *= 2) {
        std::vector<std::tuple<int, int, int, int, int64_t>> pairs;
        int64_t tb = 0;
        for (int64_t f = 0; f < nf; f++) {
            const int Pf = P_of((int)f);
            for (int t0 = 0; t0 + b < Pf; t0 += 2 * b) {
                const int b0 = t0 + b, b1 = std::min(t0 + 2 * b, Pf);
                pairs.emplace_back((int)f, t0, b0, b1, tb);
                tb += (int64_t)(b1 - b0) * TS * (int64_t)b * TS;
            }
        }
        Tmax = std::max(Tmax, tb);
        TaskRange r1, r1f, r2;
        // T = L(bot, top) X(top, top): FP64 and FP32 factor copies in
        // separate launches
        for (int pass = 0; pass < 2; pass++) {
            TaskRange& rr = pass == 0 ? r1 : r1f;
            rr.off = (int64_t)tasks.size();
            rr.a32 = pass == 1;
            for (auto& pr : pairs) {
                int f, t0, b0, b1;
                int64_t tbase;
                std::tie(f, t0, b0, b1, tbase) = pr;
                if ((Lbuf_of(f) == BUF_F32) != (pass == 1)) continue;
                const Front& Fr = sym.fronts[f];
                const int64_t ldt = (int64_t)TS * (b1 - b0), m = Fr.m, xb = ctx->xoff[f], nvp = Fr.nvpad;
                for (int i = b0; i < b1; i += 4)
                    for (int k = t0; k < b0; k += 2) {
                        GemmTask t{};
                        t.c = tbase + TS * (i - b0) + TS * (k - t0) * ldt;
                        t.ldc = (int32_t)ldt;
                        t.flags = 1 | (1 << 4) | (BUF_W << 8) | gt_shape(std::min(4, b1 - i), k + 1 < b0, false, 0, false);
                        // sum_{j=k}^{b0-1} L(i, j) X(j, k)
                        t.s[0] = mkseg(Lbuf_of(f), Fr.off + TS * i + TS * k * m, TS * m, (int)m, false, false, BUF_X,
                                       xb + TS * k + TS * k * nvp, TS, (int)nvp, false, b0 - k);
                        tasks.push_back(t);
                    }
            }
            rr.n = (int64_t)tasks.size() - rr.off;
            balance_range(tasks, rr);
        }
        r2.off = (int64_t)tasks.size();
        for (auto& pr : pairs) {
            int f, t0, b0, b1;
            int64_t tbase;
            std::tie(f, t0, b0, b1, tbase) = pr;
            const Front& Fr = sym.fronts[f];
            const int64_t ldt = (int64_t)TS * (b1 - b0), xb = ctx->xoff[f], nvp = Fr.nvpad;
            for (int i = b0; i < b1; i += 4)
                for (int k = t0; k < b0; k += 2) {
                    const int nq = std::min(4, b1 - i);
                    GemmTask t{};
                    t.c = xb + TS * i + TS * k * nvp;
                    t.ldc = (int32_t)nvp;
                    t.flags = 1 | (1 << 4) | (BUF_X << 8) | gt_shape(nq, k + 1 < b0, false, 0, false);
                    // - sum_{j=b0}^{i + nq - 1} X(i, j) T(j, k)
                    t.s[0] = mkseg(BUF_X, xb + TS * i + TS * b0 * nvp, TS * nvp, (int)nvp, false, true, BUF_W,
                                   tbase + TS * (k - t0) * ldt, TS, (int)ldt, false, i + nq - b0);
                    tasks.push_back(t);
                }
        }
        r2.n = (int64_t)tasks.size() - r2.off;
        balance_range(tasks, r2);
        ctx->trtri1f.push_back(r1f);
        ctx->trtri1.push_back(r1);
        ctx->trtri2.push_back(r2);
    }
    ctx->W_elems = std::max<int64_t>(std::max(Wmax, Tmax), 1);
    {   // the lower-triangular 64 x 64 tiles of every front (the assembly's zeroing)
        std::vector<std::pair<int, int64_t>> zl;
        for (int f = 0; f < (int)sym.fronts.size(); f++) zl.emplace_back(f, (int64_t)M_of(f) * (M_of(f) + 1) / 2);
        ctx->zero_lower = mk_launch(zl);
    }
    return EP_OK;
}

// ---------------------------------------------------------------------------
// init
// ---------------------------------------------------------------------------
static int validate(const ep_config* c, int64_t S, const double* xyz, const double* A, const double* sig,
                    std::string& err) {
    if (!c) { err = "cfg is NULL"; return EP_ERR_INVALID_ARG; }
    if (c->n < 2 || c->n > 1290) { err = "n must be in [2, 1290]"; return EP_ERR_INVALID_ARG; }
    if (!(c->box_pc > 0)) { err = "box_pc must be > 0"; return EP_ERR_INVALID_ARG; }
    if (!(c->prior_var > 0) || !(c->outer_scale_pc > 0) || !(c->support_pc > 0)) {
        err = "prior_var, outer_scale_pc and support_pc must be > 0";
        return EP_ERR_INVALID_ARG;
    }
    if (!(c->los_step_pc > 0)) { err = "los_step_pc must be > 0"; return EP_ERR_INVALID_ARG; }
    if (!(c->damping > 0 && c->damping <= 1)) { err = "damping must be in (0, 1]"; return EP_ERR_INVALID_ARG; }
    if (!(c->relin_step > 0 && c->relin_step <= 1)) { err = "relin_step must be in (0, 1]"; return EP_ERR_INVALID_ARG; }
    if (c->deterministic != 0 && c->deterministic != 1) { err = "deterministic must be 0 or 1"; return EP_ERR_INVALID_ARG; }
    if (c->deterministic && (c->precision != EP_PREC_FP64 || c->mean_fn != EP_MEAN_CONSTANT)) {
        err = "deterministic needs precision FP64 and mean_fn CONSTANT";
        return EP_ERR_INVALID_ARG;
    }
    if (c->likelihood != EP_LIK_EXTINCTION && c->likelihood != EP_LIK_GAUSS_LINEAR && c->likelihood != EP_LIK_GMM) {
        err = "unknown likelihood";
        return EP_ERR_INVALID_ARG;
    }
    if (c->precision != EP_PREC_FP64 && c->precision != EP_PREC_MIXED && c->precision != EP_PREC_SELINV32) {
        err = "unknown precision";
        return EP_ERR_INVALID_ARG;
    }
    if (c->pointers_on_device != 0 && c->pointers_on_device != 1) { err = "pointers_on_device must be 0 or 1"; return EP_ERR_INVALID_ARG; }
    if (c->mean_fn != EP_MEAN_CONSTANT && c->mean_fn != EP_MEAN_DISC_BUMP) { err = "unknown mean_fn"; return EP_ERR_INVALID_ARG; }
    if (c->mean_fn == EP_MEAN_DISC_BUMP) {
        for (int j = 0; j < 5; j++)
            if (!(c->theta_prior[j] > 0) || !std::isfinite(c->theta_prior[j])) {
                err = "theta_prior must be finite and > 0";
                return EP_ERR_INVALID_ARG;
            }
        if (!(c->sun_radius_pc > 0) || !std::isfinite(c->sun_radius_pc) || !(c->bump_width_pc > 0) ||
            !std::isfinite(c->bump_width_pc)) {
            err = "sun_radius_pc and bump_width_pc must be finite and > 0";
            return EP_ERR_INVALID_ARG;
        }
        if (c->precision != EP_PREC_FP64) { err = "mean_fn DISC_BUMP needs precision FP64"; return EP_ERR_INVALID_ARG; }
    }
    if (c->mixed_fp64_levels < 0) { err = "mixed_fp64_levels must be >= 0"; return EP_ERR_INVALID_ARG; }
    if (c->moments != EP_MOM_QUADRATURE && c->moments != EP_MOM_SURROGATE) { err = "unknown moments mode"; return EP_ERR_INVALID_ARG; }
    if (c->moments == EP_MOM_SURROGATE && !(c->surrogate_tol > 0)) { err = "surrogate_tol must be > 0"; return EP_ERR_INVALID_ARG; }
    for (int a = 0; a < 3; a++)
        if (!(c->observer_pc[a] >= 0 && c->observer_pc[a] <= c->box_pc)) {
            err = "observer must lie in the cube";
            return EP_ERR_INVALID_ARG;
        }
    const bool gmm = c->likelihood == EP_LIK_GMM;   // the mixtures come later (ep_set_gmm); A_obs, sigma unused
    if (gmm && c->moments != EP_MOM_QUADRATURE) { err = "the distance mixture needs moments QUADRATURE"; return EP_ERR_INVALID_ARG; }
    if (S < 0 || (S > 0 && (!xyz || (!gmm && (!A || !sig))))) { err = "bad star arrays"; return EP_ERR_INVALID_ARG; }
    for (int64_t s = 0; s < S; s++) {
        for (int a = 0; a < 3; a++)
            if (!std::isfinite(xyz[3 * s + a]) || xyz[3 * s + a] < 0 || xyz[3 * s + a] > c->box_pc) {
                err = "star " + std::to_string(s) + " lies outside the cube or is not finite";
                return EP_ERR_INVALID_ARG;
            }
        {
            double d2 = 0;
            for (int a = 0; a < 3; a++) d2 += (xyz[3 * s + a] - c->observer_pc[a]) * (xyz[3 * s + a] - c->observer_pc[a]);
            if (!(std::sqrt(d2) > 1e-9 * c->box_pc)) {
                err = "star " + std::to_string(s) + " coincides with the observer (zero sightline)";
                return EP_ERR_INVALID_ARG;
            }
        }
        if (gmm) continue;
        if (!std::isfinite(A[s])) { err = "A_obs of star " + std::to_string(s) + " is not finite"; return EP_ERR_INVALID_ARG; }
        if (!(sig[s] > 0) || !std::isfinite(sig[s])) {
            err = "sigma of star " + std::to_string(s) + " must be finite and > 0";
            return EP_ERR_INVALID_ARG;
        }
    }
    return EP_OK;
}

static void geom_from_cfg(const ep_config* c, GridGeom& g, PriorParams& p) {
    g.n = c->n;
    g.L = c->box_pc;
    g.h = c->box_pc / (c->n - 1);
    for (int a = 0; a < 3; a++) g.obs[a] = c->observer_pc[a];
    g.step = c->los_step_pc;
    p.mean = c->prior_mean;
    p.var = c->prior_var;
    p.ell = c->outer_scale_pc;
    p.support = c->support_pc;
    p.rho = c->vecchia_radius_pc > 0 ? c->vecchia_radius_pc : c->support_pc;
}

// the disc + bump mean function at theta = exp(phihat)
static MeanDev mean_params(const ep_ctx* ctx) {
    MeanDev P{};
    for (int j = 0; j < NTHETA; j++) P.theta[j] = std::exp(ctx->phihat[j]);
    P.R0 = ctx->cfg.sun_radius_pc;
    P.w = ctx->cfg.bump_width_pc;
    return P;
}
static void enqueue_mean(ep_ctx* ctx) {
    launch_mean_fn(ctx->stream, ctx->GD, mean_params(ctx), ctx->d_mhat, ctx->d_J, ctx->g.N());
}
static Phi5 phi5(const double* v) {
    Phi5 p{};
    for (int j = 0; j < NTHETA; j++) p.v[j] = v[j];
    return p;
}

// Clique assembly by tile owner (host, once).  A star's slots, sorted by
// local row in its front, fall into runs by 64-row tile; every pair of runs
// (u >= v) is an incidence of tile (run u's tile, run v's tile).  The
// incidences are grouped by tile (star order inside a tile) and cut into
// chunks of bounded work for one wave each; a tile with several chunks gets
// partial tiles that a second launch sums in chunk order.  Chunks are
// launched heaviest first.  Work of an incidence: its 8 x 8 pair blocks and
// the staging of its slots.
constexpr int64_t TILE_CHUNK_WORK = 4096;
static int build_tile_assembly(ep_ctx* ctx, const std::vector<int32_t>& sord) {
    const Symbolic& sym = ctx->sym;
    const int64_t S = ctx->S;
    const auto& ptr = ctx->sup.ptr;
    const int64_t nslots = (int64_t)ctx->sup.nodes.size();
    std::vector<int32_t> lsort((size_t)nslots);
    for (int64_t st = 0; st < S; st++)
        for (int64_t q = ptr[st]; q < ptr[st + 1]; q++) lsort[q] = sym.star_loc[ptr[st] + sord[q]];
    const int64_t nf = (int64_t)sym.fronts.size();
    std::vector<int64_t> tbase((size_t)nf + 1, 0);
    for (int64_t f = 0; f < nf; f++) {
        const int64_t M = sym.fronts[f].m / TS;
        tbase[f + 1] = tbase[f] + M * (M + 1) / 2;
    }
    const int64_t ntiles = tbase[nf];
    // runs of one star: (tile, first sorted position, count)
    auto runs = [&](int64_t st, std::vector<std::array<int64_t, 3>>& r) {
        r.clear();
        for (int64_t q = ptr[st]; q < ptr[st + 1]; q++) {
            const int64_t t = lsort[q] / TS;
            if (r.empty() || r.back()[0] != t) r.push_back({t, q, 0});
            r.back()[2]++;
        }
    };
    auto tile_id = [&](int64_t f, int64_t tu, int64_t tv) { return tbase[f] + tu * (tu + 1) / 2 + tv; };
    std::vector<int64_t> cnt((size_t)ntiles + 1, 0);
    std::vector<std::array<int64_t, 3>> r;
    for (int64_t st = 0; st < S; st++) {
        runs(st, r);
        const int64_t f = sym.star_front[st];
        for (size_t u = 0; u < r.size(); u++)
            for (size_t v = 0; v <= u; v++) cnt[tile_id(f, r[u][0], r[v][0]) + 1]++;
    }
    for (int64_t t = 0; t < ntiles; t++) cnt[t + 1] += cnt[t];
    const int64_t ninc = cnt[ntiles];
    std::vector<TileInc> incs((size_t)ninc);
    {
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        for (int64_t st = 0; st < S; st++) {
            runs(st, r);
            const int64_t f = sym.star_front[st];
            for (size_t u = 0; u < r.size(); u++)
                for (size_t v = 0; v <= u; v++) {
                    TileInc& I = incs[(size_t)fill[tile_id(f, r[u][0], r[v][0])]++];
                    I.star = (int32_t)st;
                    I.r0 = (uint16_t)(r[u][1] - ptr[st]);
                    I.c0 = (uint16_t)(r[v][1] - ptr[st]);
                    I.nr = (uint16_t)r[u][2];
                    I.nc = (uint16_t)r[v][2];
                    I.rlo = (uint8_t)(lsort[(size_t)r[u][1]] % TS);
                    I.rhi = (uint8_t)(lsort[(size_t)(r[u][1] + r[u][2] - 1)] % TS);
                    I.pad = 0;
                }
        }
    }
    std::vector<TileChunk> chunks;
    std::vector<int64_t> work;
    std::vector<TileRed> reds;
    int32_t nparts = 0;
    for (int64_t f = 0; f < nf; f++) {
        const int64_t M = sym.fronts[f].m / TS;
        for (int64_t ti = 0; ti < M; ti++)
            for (int64_t tj = 0; tj <= ti; tj++) {
                const int64_t id = tile_id(f, ti, tj);
                if (cnt[id + 1] == cnt[id]) continue;
                const size_t c0 = chunks.size();
                int64_t e = cnt[id];
                while (e < cnt[id + 1]) {
                    TileChunk C{};
                    C.i0 = e;
                    C.f = (int32_t)f;
                    C.ti = (int32_t)ti;
                    C.tj = (int32_t)tj;
                    C.part = -1;
                    int64_t w = 0;
                    while (e < cnt[id + 1] && (w == 0 || w < TILE_CHUNK_WORK)) {
                        const TileInc& I = incs[(size_t)e];
                        w += 2 + (int64_t)((I.nr + 7) / 8) * ((I.nc + 7) / 8);
                        e++;
                    }
                    C.n = (int32_t)(e - C.i0);
                    chunks.push_back(C);
                    work.push_back(w);
                }
                const int np = (int)(chunks.size() - c0);
                if (np > 1) {
                    TileRed R{};
                    R.f = (int32_t)f;
                    R.ti = (int32_t)ti;
                    R.tj = (int32_t)tj;
                    R.p0 = nparts;
                    R.np = np;
                    reds.push_back(R);
                    for (int q = 0; q < np; q++) chunks[c0 + q].part = nparts++;
                }
            }
    }
    std::vector<int64_t> ord(chunks.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return work[a] > work[b]; });
    std::vector<TileChunk> sorted(chunks.size());
    for (size_t q = 0; q < ord.size(); q++) sorted[q] = chunks[(size_t)ord[q]];
    ctx->n_tch = (int64_t)sorted.size();
    ctx->n_tred = (int64_t)reds.size();
    TRY(upload(ctx, &ctx->d_lsort, lsort));
    TRY(upload(ctx, &ctx->d_tinc, incs));
    TRY(upload(ctx, &ctx->d_tch, sorted));
    TRY(upload(ctx, &ctx->d_tred, reds));
    TRY(dev_alloc(ctx, &ctx->d_tpart, (int64_t)nparts * TS * TS));
    TRY(dev_alloc(ctx, &ctx->d_gsort, nslots));
    return EP_OK;
}

// The deterministic mode's fixed summation orders (host, once):
//  * right-hand side: for every node, its slots in star order;
//  * forward solve: for every level, every updated row with the positions
//    (rptr + local row) of the level's fronts that update it, in front order.
static int build_deterministic(ep_ctx* ctx) {
    const Symbolic& sym = ctx->sym;
    const int64_t S = ctx->S, N = ctx->g.N();
    const auto& ptr = ctx->sup.ptr;
    {
        std::vector<int64_t> nptr((size_t)N + 1, 0);
        for (int64_t q = 0; q < (int64_t)ctx->sup.nodes.size(); q++) nptr[(size_t)ctx->sup.nodes[q] + 1]++;
        for (int64_t p = 0; p < N; p++) nptr[p + 1] += nptr[p];
        std::vector<int64_t> fill(nptr.begin(), nptr.end() - 1), nslot(ctx->sup.nodes.size());
        std::vector<int32_t> nstar(ctx->sup.nodes.size());
        for (int64_t st = 0; st < S; st++)
            for (int64_t q = ptr[st]; q < ptr[st + 1]; q++) {
                const int64_t at = fill[ctx->sup.nodes[q]]++;
                nslot[at] = q;
                nstar[at] = (int32_t)st;
            }
        TRY(upload(ctx, &ctx->d_nptr, nptr));
        TRY(upload(ctx, &ctx->d_nslot, nslot));
        TRY(upload(ctx, &ctx->d_nstar, nstar));
    }
    {
        ctx->det_lv.assign(sym.nlevels, ep_ctx::DetLevel{});
        std::vector<std::vector<int32_t>> lv(sym.nlevels);
        for (int32_t f = 0; f < (int32_t)sym.fronts.size(); f++) lv[sym.fronts[f].level].push_back(f);
        for (int l = 0; l < sym.nlevels; l++) {
            std::map<int64_t, std::vector<int64_t>> rows;   // updated row -> stage positions, front order
            for (int32_t f : lv[l]) {
                const Front& Fr = sym.fronts[f];
                for (int a = 0; a < Fr.nr; a++) rows[sym.rrows[Fr.rptr + a]].push_back(Fr.rptr + a);
            }
            std::vector<int32_t> tgt;
            std::vector<int64_t> tptr(1, 0), src;
            for (const auto& kv : rows) {
                tgt.push_back((int32_t)kv.first);
                src.insert(src.end(), kv.second.begin(), kv.second.end());
                tptr.push_back((int64_t)src.size());
            }
            ep_ctx::DetLevel& D = ctx->det_lv[l];
            D.n = (int64_t)tgt.size();
            TRY(upload(ctx, &D.tgt, tgt));
            TRY(upload(ctx, &D.tptr, tptr));
            TRY(upload(ctx, &D.src, src));
        }
        TRY(dev_alloc(ctx, &ctx->d_stage, (int64_t)sym.rrows.size()));
    }
    return EP_OK;
}

static int init_impl(ep_ctx* ctx, const double* xyz, const double* A, const double* sig) {
    const ep_config& c = ctx->cfg;
    geom_from_cfg(&c, ctx->g, ctx->pp);
    HIPCHK(hipSetDevice(c.device));
    if (c.stream) {
        ctx->stream = (hipStream_t)c.stream;
    } else {
        HIPCHK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    const GridGeom& g = ctx->g;
    const int64_t N = g.N();
    const int64_t S = ctx->S;
    build_stencil(g, ctx->pp.rho, ctx->st);
    if (build_vecchia(g, ctx->pp, ctx->st, ctx->vec) != 0) {
        ctx->err = "Vecchia conditional covariance is not positive definite";
        return EP_ERR_NUMERIC;
    }
    build_supports(g, S, xyz, ctx->sup);
    ctx->max_support = 0;
    for (int64_t s = 0; s < S; s++)
        ctx->max_support = std::max<int>(ctx->max_support, (int)(ctx->sup.ptr[s + 1] - ctx->sup.ptr[s]));
    if (ctx->max_support > 1300) {
        ctx->err = "a sightline touches more than 1300 nodes";
        return EP_ERR_INVALID_ARG;
    }
    OrderingOpts opt;
    opt.leaf_size = c.leaf_size > 0 ? c.leaf_size : 512;
    // a separator slab is at least as wide as the longest pattern offset:
    // the prior stencil reaches 2 rho, the {-2..2}^3 block 2 sqrt(3) h
    opt.sep_halfwidth = std::max(ctx->pp.rho, std::sqrt(3.0) * g.h) * (1.0 + 1e-9);
    opt.tile = TS;
    opt.panel_tiles = PW;
    int rc = analyse(g, ctx->st, ctx->sup, opt, ctx->sym);
    if (rc != 0) {
        ctx->err = "symbolic analysis failed (" + std::to_string(rc) + ")";
        return EP_ERR_STATE;
    }
    const Symbolic& sym = ctx->sym;
    const int64_t nf = (int64_t)sym.fronts.size();
    // schedules
    std::vector<int32_t> flists;
    std::vector<BatchEnt> batches;
    std::vector<GemmTask> tasks;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device) == hipSuccess && cus > 0)
            ctx->n_cu = cus;
    }
    TRY(build_plans(ctx, flists, batches, tasks));
    // Q0 entries -> front positions
    Q0Table q0;
    build_q0(g, ctx->st, ctx->vec, q0);
    std::vector<int64_t> q0dest;
    std::vector<double> q0val;
    q0dest.reserve((size_t)N * q0.nlower / 2);
    q0val.reserve((size_t)N * q0.nlower / 2);
    const int n = g.n;
    for (int64_t p = 0; p < N; p++) {
        int64_t i = p % n, j = (p / n) % n, k = p / ((int64_t)n * n);
        for (int o = 0; o < q0.nlower; o++) {
            double v = q0.val[(size_t)p * q0.nlower + o];
            if (v == 0.0) continue;
            int64_t ii = i + q0.lower[3 * o], jj = j + q0.lower[3 * o + 1], kk = k + q0.lower[3 * o + 2];
            if (ii < 0 || jj < 0 || kk < 0 || ii >= n || jj >= n || kk >= n) continue;
            int64_t q = ii + (int64_t)n * (jj + (int64_t)n * kk);
            int64_t a = sym.iperm[p], b = sym.iperm[q];
            int64_t lo = std::min(a, b), hi = std::max(a, b);
            const Front& Fr = sym.fronts[sym.snode[lo]];
            int32_t row = front_local(sym, Fr, hi);
            if (row < 0) {
                ctx->err = "prior stencil entry outside the front structure";
                return EP_ERR_STATE;
            }
            q0dest.push_back(Fr.off + row + (lo - Fr.first) * (int64_t)Fr.m);
            q0val.push_back(v);
        }
    }
    std::vector<int64_t> paddest;
    for (int64_t f = 0; f < nf; f++) {
        const Front& Fr = sym.fronts[f];
        for (int l = Fr.nv; l < Fr.nvpad; l++) paddest.push_back(Fr.off + l + (int64_t)l * Fr.m);
    }
    ctx->n_q0 = (int64_t)q0dest.size();
    ctx->n_pad = (int64_t)paddest.size();
    std::vector<double> b0;
    if (c.mean_fn == EP_MEAN_DISC_BUMP) {
        // the latent field is delta = f - m(phi), of prior mean 0; phi = ln theta
        // has independent log-normal hyperpriors whose sd equals their mean
        ctx->M = NTHETA;
        b0.assign((size_t)N, 0.0);
        for (int j = 0; j < NTHETA; j++) {
            ctx->s0sq[j] = std::log(2.0);
            ctx->mu0[j] = std::log(c.theta_prior[j]) - 0.5 * ctx->s0sq[j];
            ctx->phihat[j] = ctx->mu0[j];
        }
    } else {
        q0_times_const(g, ctx->vec, ctx->pp.mean, b0);
    }
    // per-star slot order by local row
    std::vector<int32_t> sord(ctx->sup.nodes.size());
    for (int64_t s = 0; s < S; s++) {
        int64_t p0 = ctx->sup.ptr[s];
        int cnt = (int)(ctx->sup.ptr[s + 1] - p0);
        std::vector<int32_t> idx(cnt);
        std::iota(idx.begin(), idx.end(), 0);
        std::sort(idx.begin(), idx.end(), [&](int a, int b) { return sym.star_loc[p0 + a] < sym.star_loc[p0 + b]; });
        std::copy(idx.begin(), idx.end(), sord.begin() + p0);
    }
    // ---- device upload ----
    std::vector<int64_t> off(nf), first(nf), rptr(nf);
    std::vector<int32_t> m(nf), nv(nf), nvpad(nf), nr(nf), parent(nf);
    for (int64_t f = 0; f < nf; f++) {
        const Front& Fr = sym.fronts[f];
        off[f] = Fr.off; first[f] = Fr.first; rptr[f] = Fr.rptr;
        m[f] = Fr.m; nv[f] = Fr.nv; nvpad[f] = Fr.nvpad; nr[f] = Fr.nr; parent[f] = Fr.parent;
    }
    std::vector<int32_t> rrows(sym.rrows.begin(), sym.rrows.end());
    TRY(upload(ctx, &ctx->d_off, off));
    TRY(upload(ctx, &ctx->d_first, first));
    TRY(upload(ctx, &ctx->d_rptr, rptr));
    TRY(upload(ctx, &ctx->d_xoff, ctx->xoff));
    TRY(upload(ctx, &ctx->d_m, m));
    TRY(upload(ctx, &ctx->d_nv, nv));
    TRY(upload(ctx, &ctx->d_nvpad, nvpad));
    TRY(upload(ctx, &ctx->d_nr, nr));
    TRY(upload(ctx, &ctx->d_parent, parent));
    TRY(upload(ctx, &ctx->d_rrows, rrows));
    TRY(upload(ctx, &ctx->d_relmap, sym.relmap));
    TRY(upload(ctx, &ctx->d_perm, sym.perm));
    TRY(upload(ctx, &ctx->d_snode, sym.snode));
    TRY(upload(ctx, &ctx->d_q0_dest, q0dest));
    TRY(upload(ctx, &ctx->d_q0_val, q0val));
    TRY(upload(ctx, &ctx->d_pad_dest, paddest));
    TRY(upload(ctx, &ctx->d_flists, flists));
    TRY(upload(ctx, &ctx->d_batches, batches));
    TRY(upload(ctx, &ctx->d_tasks, tasks));
    // The GEMM tasks load whole 256 x 128 footprints, also the row quarters
    // and column halves a task does not have (their results are discarded):
    // every dense buffer ends in a pad of 256 leading dimensions (any leading
    // dimension is at most the largest front order) so those loads stay in
    // the allocation.
    const int64_t pad = 256 * (int64_t)sym.max_m + 256;
    TRY(dev_alloc(ctx, &ctx->d_fronts, sym.total_elems + pad));
    TRY(dev_alloc(ctx, &ctx->d_X, ctx->X_elems + pad));
    // X tiles above the diagonal are never written and must read as zero
    // (a task runs its row and column tiles over the first tile's K range)
    launch_fill(ctx->stream, ctx->d_X, ctx->X_elems, 0.0);
    TRY(dev_alloc(ctx, &ctx->d_W, ctx->W_elems + pad));
    TRY(dev_alloc(ctx, &ctx->d_err, 1));
    if (c.precision == EP_PREC_MIXED) TRY(dev_alloc(ctx, &ctx->d_f32, sym.total_elems + pad));
    TRY(upload(ctx, &ctx->d_brp, ctx->vec.rowptr));
    TRY(upload(ctx, &ctx->d_bcol, ctx->vec.col));
    TRY(upload(ctx, &ctx->d_bval, ctx->vec.val));
    TRY(upload(ctx, &ctx->d_bd, ctx->vec.d));
    for (double** p : {&ctx->d_u, &ctx->d_w, &ctx->d_r, &ctx->d_dx}) TRY(dev_alloc(ctx, p, N));
    // stars
    const bool gmm = c.likelihood == EP_LIK_GMM;   // A_obs and sigma unused (may be NULL)
    std::vector<double> vx(xyz, xyz + 3 * S), vA((size_t)S, 0.0), vs((size_t)S, 1.0);
    if (!gmm) {
        std::copy(A, A + S, vA.begin());
        std::copy(sig, sig + S, vs.begin());
    } else {
        for (int64_t s = 0; s < S; s++)
            ctx->gmm_kcap = std::max(ctx->gmm_kcap, gmm_ray_samples(xyz + 3 * s, g.obs, ctx->sup.nsamp[s], c.box_pc,
                                                                    c.los_step_pc) + 1);
    }
    TRY(upload(ctx, &ctx->d_xyz, vx));
    TRY(upload(ctx, &ctx->d_A, vA));
    TRY(upload(ctx, &ctx->d_sigma, vs));
    TRY(upload(ctx, &ctx->d_sptr, ctx->sup.ptr));
    TRY(upload(ctx, &ctx->d_snodes, ctx->sup.nodes));
    TRY(upload(ctx, &ctx->d_sloc, sym.star_loc));
    TRY(upload(ctx, &ctx->d_sord, sord));
    {   // processing order of the clique kernels: stars grouped by the front
        // that holds their clique and, inside it, by their first local row,
        // so that stars reading the same part of a front run together; the
        // order is cut into eight contiguous pieces, one per XCD (block b runs
        // on XCD b mod 8), four stars per block, -1 padding
        std::vector<int32_t> byf((size_t)S);
        std::iota(byf.begin(), byf.end(), 0);
        auto first_loc = [&](int32_t s) {
            const int64_t p0 = ctx->sup.ptr[s];
            return ctx->sup.ptr[s + 1] > p0 ? sym.star_loc[p0 + sord[p0]] : INT32_MAX;
        };
        std::stable_sort(byf.begin(), byf.end(), [&](int32_t a, int32_t b) {
            const int32_t fa = sym.star_front[a], fb = sym.star_front[b];
            return fa != fb ? fa < fb : first_loc(a) < first_loc(b);
        });
        const int64_t piece = (S + 7) / 8, per = (piece + 3) / 4;   // stars and blocks per XCD
        std::vector<int32_t> order((size_t)(32 * per), -1);
        for (int64_t q = 0; q < S; q++) {
            const int64_t x = q / piece, j = q % piece;              // XCD x, its j-th star
            order[(size_t)(((j / 4) * 8 + x) * 4 + j % 4)] = byf[q];
        }
        ctx->n_order = (int64_t)order.size();
        TRY(upload(ctx, &ctx->d_order, order));
    }
    TRY(upload(ctx, &ctx->d_sfront, sym.star_front));
    TRY(upload(ctx, &ctx->d_nsamp, ctx->sup.nsamp));
    TRY(build_tile_assembly(ctx, sord));
    if (c.deterministic) TRY(build_deterministic(ctx));
    const int64_t nG = (int64_t)ctx->sup.nodes.size();
    TRY(dev_alloc(ctx, &ctx->d_g, nG));
    double** sarr[] = {&ctx->d_lnA, &ctx->d_c, &ctx->d_tau, &ctx->d_nu, &ctx->d_cmu, &ctx->d_cvar, &ctx->d_lnZ,
                       &ctx->d_tmean, &ctx->d_tvar, &ctx->d_dtau, &ctx->d_tau_bak, &ctx->d_nu_bak};
    for (auto p : sarr) {
        TRY(dev_alloc(ctx, p, S));
        launch_fill(ctx->stream, *p, S, 0.0);
    }
    TRY(dev_alloc(ctx, &ctx->d_status, S));
    TRY(upload(ctx, &ctx->d_b0, b0));
    double** varr[] = {&ctx->d_fhat, &ctx->d_borig, &ctx->d_y, &ctx->d_x, &ctx->d_t, &ctx->d_mu, &ctx->d_var};
    for (auto p : varr) TRY(dev_alloc(ctx, p, N));
    launch_fill(ctx->stream, ctx->d_fhat, N, ctx->pp.mean);
    HIPCHK(set_gauss_legendre(ctx->stream));
    HIPCHK(set_gauss_hermite(ctx->stream));
    TRY(dev_alloc(ctx, &ctx->d_mlp_P, MLP_NPARAM));
    TRY(dev_alloc(ctx, &ctx->d_mlp_bf, 2 * 128 * 128));
    TRY(dev_alloc(ctx, &ctx->d_fb_list, S));
    TRY(dev_alloc(ctx, &ctx->d_fb_count, 1));

    FrontsDev& F = ctx->F;
    F.off = ctx->d_off; F.m = ctx->d_m; F.nv = ctx->d_nv; F.nvpad = ctx->d_nvpad; F.nr = ctx->d_nr;
    F.first = ctx->d_first; F.rptr = ctx->d_rptr; F.parent = ctx->d_parent; F.xoff = ctx->d_xoff;
    F.rrows = ctx->d_rrows; F.relmap = ctx->d_relmap;
    StarsDev& SD = ctx->SD;
    SD.n = S; SD.xyz = ctx->d_xyz; SD.A = ctx->d_A; SD.sigma = ctx->d_sigma; SD.ptr = ctx->d_sptr;
    SD.nodes = ctx->d_snodes; SD.loc = ctx->d_sloc; SD.sord = ctx->d_sord; SD.front = ctx->d_sfront;
    SD.order = ctx->d_order; SD.norder = ctx->n_order;
    SD.nsamp = ctx->d_nsamp; SD.g = ctx->d_g; SD.lnA = ctx->d_lnA; SD.c = ctx->d_c; SD.tau = ctx->d_tau;
    SD.nu = ctx->d_nu; SD.cav_mu = ctx->d_cmu; SD.cav_var = ctx->d_cvar; SD.lnZ = ctx->d_lnZ;
    SD.tmean = ctx->d_tmean; SD.tvar = ctx->d_tvar; SD.status = ctx->d_status; SD.dtau = ctx->d_dtau;
    GridDev& GD = ctx->GD;
    GD.n = g.n; GD.h = g.h; GD.ox = g.obs[0]; GD.oy = g.obs[1]; GD.oz = g.obs[2];
    if (ctx->M) {
        TRY(dev_alloc(ctx, &ctx->d_mhat, N));
        TRY(dev_alloc(ctx, &ctx->d_J, NTHETA * N));
        TRY(dev_alloc(ctx, &ctx->d_h, NTHETA * std::max<int64_t>(S, 1)));
        TRY(dev_alloc(ctx, &ctx->d_R, NTHETA * N));
        TRY(dev_alloc(ctx, &ctx->d_Wb, (NTHETA + 1) * N));
        TRY(dev_alloc(ctx, &ctx->d_part, DOT_BLOCKS * (NTHETA * (NTHETA + 1) + NTHETA * (NTHETA + 1) / 2 + NTHETA)));
        launch_fill(ctx->stream, ctx->d_h, NTHETA * S, 0.0);
        // fhat = m(phihat) + deltahat with deltahat = 0
        enqueue_mean(ctx);
        HIPCHK(hipMemcpyAsync(ctx->d_fhat, ctx->d_mhat, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
    // free host-side bulk no longer needed
    std::vector<double>().swap(ctx->vec.val);
    std::vector<int32_t>().swap(ctx->vec.col);
    std::vector<int64_t>().swap(ctx->vec.rowptr);
    return EP_OK;
}

// ---------------------------------------------------------------------------
// sweep pieces
// ---------------------------------------------------------------------------
static Bufs bufs(ep_ctx* ctx) { return Bufs{ctx->d_fronts, ctx->d_X, ctx->d_W, ctx->d_f32}; }
// buffers for the solves of one level: the FP32 factor copy only where that level was factored in FP32
static Bufs level_bufs(ep_ctx* ctx, int lvl) {
    Bufs b = bufs(ctx);
    if (!is_f32_level(ctx, lvl)) b.F32 = nullptr;
    return b;
}

static bool frozen(const ep_ctx* ctx) {
    return ctx->cfg.likelihood == EP_LIK_GAUSS_LINEAR || ctx->cfg.relinearize == 0;
}

// sightlines at fhat; with an inferred mean also the border projections
// h_n = J^T g_n and c'_n (the mean linearised about phihat)
static void enqueue_linearise(ep_ctx* ctx) {
    const double* field = ctx->d_fhat;
    if (frozen(ctx)) {
        if (ctx->linearised) return;
        // freeze at the prior mean (m(mu0) with an inferred mean, held in fhat)
        if (!ctx->M) {
            launch_fill(ctx->stream, ctx->d_t, ctx->g.N(), ctx->pp.mean);
            field = ctx->d_t;
        }
    }
    launch_los(ctx->stream, ctx->GD, ctx->SD, field, ctx->max_support);
    if (ctx->M) launch_star_border(ctx->stream, ctx->SD, ctx->d_mhat, ctx->d_J, phi5(ctx->phihat), ctx->d_h, ctx->g.N());
    ctx->linearised = true;
}

// Optional per-launch timing of the MFMA tile kernels and the sparse kernels
// (cfg.profile_kernels).
static void kt_begin(ep_ctx* ctx, int64_t ntasks) {
    if (!ctx->cfg.profile_kernels || ntasks <= 0) return;
    if (ctx->kt_used + 2 > ctx->kt_ev.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
        ctx->kt_ev.push_back(a);
        ctx->kt_ev.push_back(b);
        ctx->kt_kind.push_back(0);
    }
    (void)hipEventRecord(ctx->kt_ev[ctx->kt_used], ctx->stream);
}
static void kt_end(ep_ctx* ctx, int64_t ntasks, int kind) {
    if (!ctx->cfg.profile_kernels || ntasks <= 0 || ctx->kt_used + 2 > ctx->kt_ev.size()) return;
    (void)hipEventRecord(ctx->kt_ev[ctx->kt_used + 1], ctx->stream);
    ctx->kt_kind[ctx->kt_used / 2] = kind;
    ctx->kt_used += 2;
}

static int enqueue_assemble(ep_ctx* ctx) {
    hipStream_t st = ctx->stream;
    // Only the lower-triangular tiles of a front are assembled, accumulated
    // into or read; the strictly upper tiles are left as they are.
    kt_begin(ctx, ctx->zero_lower.ntasks);
    launch_zero_lower(st, ctx->d_batches + ctx->zero_lower.be_off, ctx->zero_lower.nbe, ctx->zero_lower.ntasks, ctx->F,
                      ctx->d_fronts);
    kt_end(ctx, ctx->zero_lower.ntasks, EP_KK_ZERO);
    launch_scatter_set(st, ctx->d_fronts, ctx->d_q0_dest, ctx->d_q0_val, ctx->n_q0);
    launch_scatter_const(st, ctx->d_fronts, ctx->d_pad_dest, ctx->n_pad, 1.0);
    StarsDev sd = ctx->SD;
    sd.order = nullptr;
    kt_begin(ctx, ctx->S);
    launch_sort_g(st, sd, ctx->d_gsort, (int64_t)ctx->sup.nodes.size());
    launch_assemble_tiles(st, ctx->d_tch, ctx->n_tch, ctx->d_tinc, ctx->d_sptr, ctx->d_tau, ctx->d_gsort,
                          ctx->d_lsort, ctx->F, ctx->d_fronts, ctx->d_tpart);
    launch_tiles_reduce(st, ctx->d_tred, ctx->n_tred, ctx->d_tpart, ctx->F, ctx->d_fronts);
    kt_end(ctx, ctx->S, EP_KK_ASSEMBLE);
    HIPCHK(hipMemcpyAsync(ctx->d_borig, ctx->d_b0, sizeof(double) * ctx->g.N(), hipMemcpyDeviceToDevice, st));
    if (ctx->cfg.deterministic) {
        launch_assemble_b_nodes(st, sd, ctx->d_nptr, ctx->d_nslot, ctx->d_nstar, ctx->d_borig, ctx->g.N());
        return EP_OK;
    }
    launch_assemble_b(st, sd, ctx->d_borig);
    return EP_OK;
}

static void enqueue_factor(ep_ctx* ctx) {
    hipStream_t st = ctx->stream;
    Bufs b = bufs(ctx);
    for (int lvl = 0; lvl < (int)ctx->levels.size(); lvl++) {
        auto& P = ctx->levels[lvl];
        if (is_f32_level(ctx, lvl)) {
            launch_to_f32(st, ctx->d_batches + P.conv.be_off, P.conv.nbe, P.conv.ntasks, ctx->F, b);
            for (size_t k = 0; k < P.potrf.size(); k++) {
                launch_potrf32(st, ctx->d_flists + P.potrf[k].off, P.potrf[k].n, (int)k, ctx->F, b, ctx->d_err);
                const Launch& t = P.trsm[k];
                kt_begin(ctx, t.ntasks);
                launch_trsm32(st, ctx->d_batches + t.be_off, t.nbe, t.ntasks, (int)k, ctx->F, b);
                kt_end(ctx, t.ntasks, EP_KK_TRSM);
                const Launch& s = P.inner[k];
                kt_begin(ctx, s.ntasks);
                launch_syrk_inner32(st, ctx->d_batches + s.be_off, s.nbe, s.ntasks, (int)k, ctx->F, b);
                kt_end(ctx, s.ntasks, EP_KK_INNER);
                const TaskRange& r = P.trail32[k];
                kt_begin(ctx, r.n);
                launch_gemm_tasks_f32(st, ctx->d_tasks + r.off, r.n, ctx->d_f32);
                kt_end(ctx, r.n, EP_KK_TRAIL);
            }
            const Launch& e = P.extend;
            launch_extend_add32(st, ctx->d_batches + e.be_off, e.nbe, e.ntasks, ctx->F, b);
            continue;
        }
        for (size_t k = 0; k < P.potrf.size(); k++) {
            const TaskRange& pu = P.panelT[k];
            kt_begin(ctx, pu.n);
            launch_gemm_tasks(st, ctx->d_tasks + pu.off, pu.n, b, false);
            kt_end(ctx, pu.n, EP_KK_TRAIL);
            // inside a panel the diagonal tile of step k was factored by step
            // k - 1's in-panel update, whose launch holds the same fronts
            if (k % PW == 0)
                launch_potrf(st, ctx->d_flists + P.potrf[k].off, P.potrf[k].n, (int)k, ctx->F, b, ctx->d_err);
            const Launch& t = P.trsm[k];
            kt_begin(ctx, t.ntasks);
            launch_trsm_step(st, ctx->d_batches + t.be_off, t.nbe, t.ntasks, (int)k, ctx->F, b);
            kt_end(ctx, t.ntasks, EP_KK_TRSM);
            const Launch& s = P.inner[k];
            const bool factor_next = (k + 1) % PW != 0 && k + 1 < P.potrf.size();
            kt_begin(ctx, s.ntasks);
            launch_syrk_inner(st, ctx->d_batches + s.be_off, s.nbe, s.ntasks, (int)k, ctx->F, b,
                              factor_next ? ctx->d_err : nullptr);
            kt_end(ctx, s.ntasks, EP_KK_INNER);
            const TaskRange& fu = P.finalT[k];
            kt_begin(ctx, fu.n);
            launch_gemm_tasks(st, ctx->d_tasks + fu.off, fu.n, b, false);
            kt_end(ctx, fu.n, EP_KK_TRAIL);
        }
        for (const Launch& e : P.extend_groups) {
            kt_begin(ctx, e.ntasks);
            launch_extend_add_plain(st, ctx->d_batches + e.be_off, e.nbe, e.ntasks, ctx->F, b);
            kt_end(ctx, e.ntasks, EP_KK_EXTEND);
        }
    }
    for (size_t s = 0; s < ctx->trtri1.size(); s++) {
        for (const TaskRange* r : {&ctx->trtri1[s], &ctx->trtri1f[s]}) {
            kt_begin(ctx, r->n);
            launch_gemm_tasks(st, ctx->d_tasks + r->off, r->n, b, r->a32);
            kt_end(ctx, r->n, EP_KK_GEMM);
        }
        kt_begin(ctx, ctx->trtri2[s].n);
        launch_gemm_tasks(st, ctx->d_tasks + ctx->trtri2[s].off, ctx->trtri2[s].n, b, false);
        kt_end(ctx, ctx->trtri2[s].n, EP_KK_GEMM);
    }
}

// L L^T x = y for y (elimination order) in d_y, consumed; x to out (node order)
static void enqueue_tri_solve(ep_ctx* ctx, double* out) {
    hipStream_t st = ctx->stream;
    for (int lvl = 0; lvl < (int)ctx->levels.size(); lvl++) {
        auto& P = ctx->levels[lvl];
        Bufs b = level_bufs(ctx, lvl);
        kt_begin(ctx, P.fwd_xv.ntasks);
        launch_fwd_xv(st, ctx->d_batches + P.fwd_xv.be_off, P.fwd_xv.nbe, P.fwd_xv.ntasks, ctx->F, b, ctx->d_y,
                      ctx->d_t);
        kt_end(ctx, P.fwd_xv.ntasks, EP_KK_SOLVE);
        kt_begin(ctx, P.fwd_r.ntasks);
        const bool det = ctx->cfg.deterministic != 0;
        launch_fwd_r(st, ctx->d_batches + P.fwd_r.be_off, P.fwd_r.nbe, P.fwd_r.ntasks, ctx->F, b, ctx->d_t,
                     ctx->d_y, det ? ctx->d_stage : nullptr);
        if (det) {
            const ep_ctx::DetLevel& D = ctx->det_lv[lvl];
            launch_gather_sub(st, D.tgt, D.tptr, D.src, D.n, ctx->d_stage, ctx->d_y);
        }
        kt_end(ctx, P.fwd_r.ntasks, EP_KK_SOLVE);
        launch_copy_v(st, ctx->d_flists + P.fronts.off, P.fronts.n, ctx->F, ctx->d_t, ctx->d_y);
    }
    for (int l = (int)ctx->levels.size() - 1; l >= 0; l--) {
        auto& P = ctx->levels[l];
        Bufs b = level_bufs(ctx, l);
        kt_begin(ctx, P.bwd_t.ntasks);
        launch_bwd_t(st, ctx->d_batches + P.bwd_t.be_off, P.bwd_t.nbe, P.bwd_t.ntasks, ctx->F, b, ctx->d_y, ctx->d_x,
                     ctx->d_t);
        kt_end(ctx, P.bwd_t.ntasks, EP_KK_SOLVE);
        kt_begin(ctx, P.bwd_x.ntasks);
        launch_bwd_x(st, ctx->d_batches + P.bwd_x.be_off, P.bwd_x.nbe, P.bwd_x.ntasks, ctx->F, b, ctx->d_t,
                     ctx->d_x);
        kt_end(ctx, P.bwd_x.ntasks, EP_KK_SOLVE);
    }
    launch_scatter_perm(st, ctx->d_perm, ctx->d_x, out, ctx->g.N());
}

static int ensure_mr(ep_ctx* ctx) {
    if (ctx->d_ymr) return EP_OK;
    const int64_t N = ctx->g.N();
    for (double** p : {&ctx->d_ymr, &ctx->d_tmr, &ctx->d_xmr, &ctx->d_omr}) TRY(dev_alloc(ctx, p, MR_MAX * N));
    return EP_OK;
}

// backward half for nrhs <= MR_MAX vectors: x = L^{-T} z with the columns of
// z (elimination order, leading dimension N) in d_ymr; x to out (node order,
// leading dimension N).  Each tile of the factor is read once per batch.
static void enqueue_bwd_mr(ep_ctx* ctx, int nrhs, double* out) {
    hipStream_t st = ctx->stream;
    const int64_t N = ctx->g.N();
    for (int l = (int)ctx->levels.size() - 1; l >= 0; l--) {
        auto& P = ctx->levels[l];
        Bufs b = level_bufs(ctx, l);
        launch_bwd_t_mr(st, ctx->d_batches + P.bwd_t.be_off, P.bwd_t.nbe, P.bwd_t.ntasks, ctx->F, b, ctx->d_ymr,
                        ctx->d_xmr, ctx->d_tmr, nrhs, N);
        launch_bwd_x_mr(st, ctx->d_batches + P.bwd_x.be_off, P.bwd_x.nbe, P.bwd_x.ntasks, ctx->F, b, ctx->d_tmr,
                        ctx->d_xmr, nrhs, N);
    }
    launch_scatter_perm_mr(st, ctx->d_perm, ctx->d_xmr, N, out, N, nrhs, N);
}

// L L^T X = Y for nrhs <= MR_MAX columns of Y in d_ymr (elimination order,
// consumed); X to out (node order), leading dimension N throughout
static void enqueue_tri_solve_mr(ep_ctx* ctx, int nrhs, double* out) {
    hipStream_t st = ctx->stream;
    const int64_t N = ctx->g.N();
    for (int lvl = 0; lvl < (int)ctx->levels.size(); lvl++) {
        auto& P = ctx->levels[lvl];
        Bufs b = level_bufs(ctx, lvl);
        launch_fwd_xv_mr(st, ctx->d_batches + P.fwd_xv.be_off, P.fwd_xv.nbe, P.fwd_xv.ntasks, ctx->F, b, ctx->d_ymr,
                         ctx->d_tmr, nrhs, N);
        launch_fwd_r_mr(st, ctx->d_batches + P.fwd_r.be_off, P.fwd_r.nbe, P.fwd_r.ntasks, ctx->F, b, ctx->d_tmr,
                        ctx->d_ymr, nrhs, N);
        launch_copy_v_mr(st, ctx->d_flists + P.fronts.off, P.fronts.n, ctx->F, ctx->d_tmr, ctx->d_ymr, nrhs, N);
    }
    enqueue_bwd_mr(ctx, nrhs, out);
}

static double host_norm(const std::vector<double>& v) {
    double s = 0;
    for (double x : v) s += x * x;
    return std::sqrt(s);
}

// Posterior mean mu = Q^{-1} b into d_mu.  With the FP32 factor (mixed
// precision) the FP64 residual r = b - Q mu is solved again with the factor
// and added back until ||r|| <= 1e-12 ||b|| (at most 10 rounds).
static int run_solve(ep_ctx* ctx) {
    hipStream_t st = ctx->stream;
    const int64_t N = ctx->g.N();
    launch_gather_perm(st, ctx->d_perm, ctx->d_borig, ctx->d_y, N);
    enqueue_tri_solve(ctx, ctx->d_mu);
    ctx->ir_iters = 0;
    ctx->ir_res = 0;
    if (ctx->cfg.precision != EP_PREC_MIXED) return EP_OK;
    std::vector<double> hb(N), hr(N);
    HIPCHK(hipMemcpyAsync(hb.data(), ctx->d_borig, sizeof(double) * N, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double bn = std::max(host_norm(hb), 1e-300);
    for (int it = 0; it <= 10; it++) {
        launch_residual(st, N, ctx->d_brp, ctx->d_bcol, ctx->d_bval, ctx->d_bd, ctx->SD, ctx->d_borig, ctx->d_mu,
                        ctx->d_u, ctx->d_w, ctx->d_r);
        HIPCHK(hipMemcpyAsync(hr.data(), ctx->d_r, sizeof(double) * N, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        ctx->ir_res = host_norm(hr) / bn;
        if (!(ctx->ir_res > 1e-12) || it == 10) break;
        launch_gather_perm(st, ctx->d_perm, ctx->d_r, ctx->d_y, N);
        enqueue_tri_solve(ctx, ctx->d_dx);
        launch_add(st, N, ctx->d_mu, ctx->d_dx);
        ctx->ir_iters = it + 1;
    }
    return EP_OK;
}

// Small dense SPD inverse (the border's Schur complement); false if not PD.
static bool spd_inverse(int n, const double* A, double* inv) {
    double L[NTHETA * NTHETA] = {};
    for (int j = 0; j < n; j++) {
        double d = A[j * n + j];
        for (int k = 0; k < j; k++) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0) || !std::isfinite(d)) return false;
        L[j * n + j] = std::sqrt(d);
        for (int i = j + 1; i < n; i++) {
            double v = A[i * n + j];
            for (int k = 0; k < j; k++) v -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = v / L[j * n + j];
        }
    }
    for (int c = 0; c < n; c++) {   // solve L L^T x = e_c
        double y[NTHETA];
        for (int i = 0; i < n; i++) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; k++) v -= L[i * n + k] * y[k];
            y[i] = v / L[i * n + i];
        }
        for (int i = n - 1; i >= 0; i--) {
            double v = y[i];
            for (int k = i + 1; k < n; k++) v -= L[k * n + i] * inv[k * n + c];
            inv[i * n + c] = v / L[i * n + i];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < i; j++) inv[i * n + j] = inv[j * n + i] = 0.5 * (inv[i * n + j] + inv[j * n + i]);
    return true;
}

// The border of the inferred mean parameters, after run_solve left
// y = Q_dd^{-1} b_d in d_mu: W = Q_dd^{-1} R (five solves), the Schur
// complement S = S0^{-1} + H^T T H - R^T W, mu_phi = S^{-1} (b_phi - R^T y),
// Sigma_phiphi = S^{-1}; then d_mu <- mu_delta = y - W mu_phi.  Partial sums
// come back per block and are added on the host in block order.
static int border_solve(ep_ctx* ctx) {
    hipStream_t st = ctx->stream;
    const int64_t N = ctx->g.N();
    constexpr int NP = NTHETA * (NTHETA + 1), NS = NTHETA * (NTHETA + 1) / 2 + NTHETA;
    launch_fill(st, ctx->d_R, NTHETA * N, 0.0);
    launch_border_rhs(st, ctx->SD, ctx->d_h, ctx->d_R, N);
    static_assert(NTHETA <= MR_MAX, "the border columns are solved as one batch");
    TRY(ensure_mr(ctx));
    launch_gather_perm_mr(st, ctx->d_perm, ctx->d_R, N, ctx->d_ymr, N, NTHETA, N);
    enqueue_tri_solve_mr(ctx, NTHETA, ctx->d_Wb);
    double* y = ctx->d_Wb + NTHETA * N;
    HIPCHK(hipMemcpyAsync(y, ctx->d_mu, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    launch_dots_5x6(st, ctx->d_R, ctx->d_Wb, N, ctx->d_part);
    launch_star_sums(st, ctx->SD, ctx->d_h, ctx->d_part + DOT_BLOCKS * NP);
    std::vector<double> part((size_t)DOT_BLOCKS * (NP + NS));
    HIPCHK(hipMemcpyAsync(part.data(), ctx->d_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double dots[NP] = {}, sums[NS] = {};
    for (int b = 0; b < DOT_BLOCKS; b++) {
        for (int i = 0; i < NP; i++) dots[i] += part[(size_t)b * NP + i];
        for (int i = 0; i < NS; i++) sums[i] += part[(size_t)DOT_BLOCKS * NP + (size_t)b * NS + i];
    }
    // dots[i * 6 + k] = R_i . W_k (k < 5), R_i . y (k = 5); sums: tau h_j h_k
    // (j <= k, row by row), then (nu - tau c') h_j
    double S[NTHETA * NTHETA], rhs[NTHETA];
    int q = 0;
    for (int j = 0; j < NTHETA; j++)
        for (int k = j; k < NTHETA; k++, q++) {
            const double rw = 0.5 * (dots[j * (NTHETA + 1) + k] + dots[k * (NTHETA + 1) + j]);
            S[j * NTHETA + k] = S[k * NTHETA + j] = (j == k ? 1.0 / ctx->s0sq[j] : 0.0) + sums[q] - rw;
        }
    for (int j = 0; j < NTHETA; j++)
        rhs[j] = ctx->mu0[j] / ctx->s0sq[j] + sums[q + j] - dots[j * (NTHETA + 1) + NTHETA];
    BorderDev& B = ctx->border;
    if (!spd_inverse(NTHETA, S, B.sinv)) {
        ctx->err = "the Schur complement of the mean parameters is not positive definite";
        return EP_ERR_NOT_PD;
    }
    for (int j = 0; j < NTHETA; j++) {
        double v = 0;
        for (int k = 0; k < NTHETA; k++) v += B.sinv[j * NTHETA + k] * rhs[k];
        if (!std::isfinite(v)) {
            ctx->err = "posterior mean of the mean parameters is not finite";
            return EP_ERR_NUMERIC;
        }
        B.mu_phi[j] = v;
        B.phihat[j] = ctx->phihat[j];
    }
    launch_minus_w(st, y, ctx->d_Wb, phi5(B.mu_phi), ctx->d_mu, N);
    return EP_OK;
}

static void enqueue_selinv(ep_ctx* ctx) {
    hipStream_t st = ctx->stream;
    Bufs b = bufs(ctx);
    for (int l = (int)ctx->levels.size() - 1; l >= 0; l--) {
        auto& P = ctx->levels[l];
        kt_begin(ctx, P.extend.ntasks);
        launch_sigma_gather(st, ctx->d_batches + P.extend.be_off, P.extend.nbe, P.extend.ntasks, ctx->F, b);
        kt_end(ctx, P.extend.ntasks, EP_KK_GATHER);
        for (const TaskRange* r : {&P.selW, &P.selS21, &P.selS11}) {
            kt_begin(ctx, r->n);
            if (ctx->cfg.precision == EP_PREC_SELINV32)
                launch_gemm_tasks_x32(st, ctx->d_tasks + r->off, r->n, b);
            else
                launch_gemm_tasks(st, ctx->d_tasks + r->off, r->n, b, r->a32);
            kt_end(ctx, r->n, EP_KK_GEMM);
        }
    }
}

static int check_pivots(ep_ctx* ctx) {
    int e = 0;
    HIPCHK(hipMemcpyAsync(&e, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
    if (e != 0) {
        ctx->err = "posterior precision is not positive definite (front " + std::to_string(e - 1) + ")";
        return EP_ERR_NOT_PD;
    }
    return EP_OK;
}

// linearise + assemble + factor (+ inverse of the diagonal blocks)
static int run_factor(ep_ctx* ctx, hipEvent_t* ev) {
    hipStream_t st = ctx->stream;
    HIPCHK(hipMemsetAsync(ctx->d_err, 0, sizeof(int), st));
    if (ev) HIPCHK(hipEventRecord(ev[0], st));
    enqueue_linearise(ctx);
    if (ev) HIPCHK(hipEventRecord(ev[1], st));
    TRY(enqueue_assemble(ctx));
    if (ev) HIPCHK(hipEventRecord(ev[2], st));
    enqueue_factor(ctx);
    if (ev) HIPCHK(hipEventRecord(ev[3], st));
    return check_pivots(ctx);
}

static double ev_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return ms;
}

static int sweep_impl(ep_ctx* ctx, ep_sweep_stats* stats) {
    hipStream_t st = ctx->stream;
    if (ctx->cfg.moments == EP_MOM_SURROGATE && !ctx->mlp_loaded) {
        ctx->err = "surrogate moments need network weights (ep_mlp_load)";
        return EP_ERR_STATE;
    }
    if (ctx->cfg.likelihood == EP_LIK_GMM && !ctx->gmm_K) {
        ctx->err = "the distance-mixture likelihood needs the per-star mixtures (ep_set_gmm)";
        return EP_ERR_STATE;
    }
    const int64_t N = ctx->g.N(), S = ctx->S;
    hipEvent_t ev[8];
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard() { for (int i = 0; i < 8; i++) (void)hipEventDestroy(e[i]); }
    } guard{ev};
    ctx->kt_used = 0;
    {
        Range r("ep: linearise, assemble, factor");
        TRY(run_factor(ctx, ev));
    }
    {
        Range r("ep: solve");
        TRY(run_solve(ctx));
        if (ctx->M) TRY(border_solve(ctx));
    }
    HIPCHK(hipEventRecord(ev[4], st));
    {
        Range r("ep: selected inversion");
        enqueue_selinv(ctx);
    }
    HIPCHK(hipEventRecord(ev[5], st));
    // non-finite posterior mean -> NUMERIC, nothing changed (with an
    // inferred mean: the mean of f = mhat + J (mu_phi - phihat) + mu_delta)
    std::vector<double> mu(N), fh(N);
    if (ctx->M) launch_f_mean(st, ctx->d_mhat, ctx->d_J, ctx->d_mu, ctx->border, ctx->d_t, N);
    HIPCHK(hipMemcpyAsync(mu.data(), ctx->M ? ctx->d_t : ctx->d_mu, sizeof(double) * N, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(fh.data(), ctx->d_fhat, sizeof(double) * N, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double dmu = 0;
    for (int64_t i = 0; i < N; i++) {
        if (!std::isfinite(mu[i])) {
            ctx->err = "posterior mean is not finite";
            return EP_ERR_NUMERIC;
        }
        dmu = std::max(dmu, std::fabs(mu[i] - fh[i]));
    }
    // per-star phase: cavity -> tilted -> site update
    Range star_range("ep: cavity, tilted moments, site update");
    HIPCHK(hipMemcpyAsync(ctx->d_tau_bak, ctx->d_tau, sizeof(double) * S, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(ctx->d_nu_bak, ctx->d_nu, sizeof(double) * S, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipEventRecord(ev[6], st));
    kt_begin(ctx, ctx->S);
    launch_cavity(st, ctx->SD, ctx->F, ctx->d_fronts, ctx->d_mu, ctx->max_support);
    kt_end(ctx, ctx->S, EP_KK_CAVITY);
    if (ctx->M) launch_cavity_border(st, ctx->SD, ctx->d_Wb, ctx->d_h, ctx->border, N);
    EpParams p{ctx->cfg.likelihood == EP_LIK_GAUSS_LINEAR ? 1 : 0, ctx->cfg.damping, ctx->cfg.cavity_var_floor};
    ctx->fallbacks = 0;
    if (ctx->cfg.likelihood == EP_LIK_GMM) {
        // the extinction curves at the point the sightlines were linearised
        // about: fhat, or the constant prior mean when frozen
        p.mode = 2;
        const double* field = ctx->d_fhat;
        if (frozen(ctx) && !ctx->M) {
            launch_fill(st, ctx->d_t, N, ctx->pp.mean);
            field = ctx->d_t;
        }
        launch_gmm_ray(st, ctx->GD, ctx->SD, p, field, ctx->d_gmm, ctx->gmm_K, ctx->cfg.box_pc, ctx->cfg.los_step_pc,
                       (int)ctx->gmm_kcap);
    } else if (ctx->cfg.moments == EP_MOM_SURROGATE && p.mode == 0) {
        // gated surrogate for every star, quadrature for the rejected ones
        HIPCHK(hipMemsetAsync(ctx->d_fb_count, 0, sizeof(int32_t), st));
        launch_mlp_tilted(st, ctx->SD, p, ctx->d_mlp_P, ctx->d_mlp_bf, ctx->cfg.surrogate_tol, ctx->d_fb_list,
                          ctx->d_fb_count, nullptr, nullptr, nullptr);
        int32_t nfb = 0;
        HIPCHK(hipMemcpyAsync(&nfb, ctx->d_fb_count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        ctx->fallbacks = nfb;
        launch_tilted_update(st, ctx->SD, p, ctx->d_fb_list, nfb);
    } else {
        launch_tilted_update(st, ctx->SD, p);
    }
    HIPCHK(hipEventRecord(ev[7], st));
    HIPCHK(hipGetLastError());
    std::vector<int32_t> status(S);
    std::vector<double> dtau(S), tau(S), nu(S);
    HIPCHK(hipMemcpyAsync(status.data(), ctx->d_status, sizeof(int32_t) * S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(dtau.data(), ctx->d_dtau, sizeof(double) * S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(tau.data(), ctx->d_tau, sizeof(double) * S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(nu.data(), ctx->d_nu, sizeof(double) * S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int64_t s = 0; s < S; s++)
        if (!std::isfinite(tau[s]) || !std::isfinite(nu[s])) {
            HIPCHK(hipMemcpyAsync(ctx->d_tau, ctx->d_tau_bak, sizeof(double) * S, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(ctx->d_nu, ctx->d_nu_bak, sizeof(double) * S, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            ctx->err = "non-finite site after the update";
            return EP_ERR_NUMERIC;
        }
    if (!frozen(ctx)) {
        const double r = ctx->cfg.relin_step;
        if (ctx->M) {
            // relinearise: deltahat <- (1 - r) deltahat + r mu_delta (deltahat =
            // fhat - m(phihat)), phihat <- (1 - r) phihat + r mu_phi, then
            // fhat = m(phihat) + deltahat; r = 1: fhat = m(mu_phi) + mu_delta
            if (r == 1.0) {
                for (int j = 0; j < NTHETA; j++) ctx->phihat[j] = ctx->border.mu_phi[j];
                enqueue_mean(ctx);
                launch_sum2(st, ctx->d_mhat, ctx->d_mu, ctx->d_fhat, N);
            } else {
                launch_relin_step(st, ctx->d_fhat, ctx->d_mhat, ctx->d_mu, r, ctx->d_t, N);
                for (int j = 0; j < NTHETA; j++)
                    ctx->phihat[j] = (1.0 - r) * ctx->phihat[j] + r * ctx->border.mu_phi[j];
                enqueue_mean(ctx);
                launch_sum2(st, ctx->d_mhat, ctx->d_t, ctx->d_fhat, N);
            }
        } else if (r == 1.0) {
            HIPCHK(hipMemcpyAsync(ctx->d_fhat, ctx->d_mu, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
        } else {
            launch_relin_step(st, ctx->d_fhat, nullptr, ctx->d_mu, r, ctx->d_fhat, N);
        }
    } else if (ctx->M && ctx->cfg.relinearize) {
        // Gaussian mode: the sightlines stay at the prior mean (the observation
        // model), and the mean's linearisation point takes a damped
        // Gauss-Newton step to the posterior mean of phi; the border rows
        // h_n, c'_n are recomputed with it before the next use
        const double d = ctx->cfg.damping;
        for (int j = 0; j < NTHETA; j++) ctx->phihat[j] = (1.0 - d) * ctx->phihat[j] + d * ctx->border.mu_phi[j];
        enqueue_mean(ctx);
        ctx->linearised = false;
    }
    HIPCHK(hipStreamSynchronize(st));
    if (stats) {
        stats->ms_linearise = ev_ms(ev[0], ev[1]);
        stats->ms_assemble = ev_ms(ev[1], ev[2]);
        stats->ms_factor = ev_ms(ev[2], ev[3]);
        stats->ms_solve = ev_ms(ev[3], ev[4]);
        stats->ms_selinv = ev_ms(ev[4], ev[5]);
        stats->ms_star = ev_ms(ev[6], ev[7]);
        stats->ms_total = ev_ms(ev[0], ev[7]);
        stats->updated = stats->skipped_cavity = stats->skipped_negsite = 0;
        stats->max_dtau = 0;
        for (int64_t s = 0; s < S; s++) {
            if (status[s] == 0) stats->updated++;
            else if (status[s] == 1) stats->skipped_cavity++;
            else stats->skipped_negsite++;
            stats->max_dtau = std::max(stats->max_dtau, dtau[s]);
        }
        stats->max_dmu = dmu;
        stats->mfma_ms = 0;
        stats->mfma_launches = (int64_t)(ctx->kt_used / 2);
        for (int k = 0; k < EP_KK_COUNT; k++) {
            stats->kernel_ms[k] = 0;
            stats->kernel_launches[k] = 0;
        }
        stats->refine_iters = ctx->ir_iters;
        stats->refine_residual = ctx->ir_res;
        stats->surrogate_fallbacks = ctx->fallbacks;
        stats->mfma_launches = 0;
        for (size_t i = 0; i + 1 < ctx->kt_used; i += 2) {
            const double ms = ev_ms(ctx->kt_ev[i], ctx->kt_ev[i + 1]);
            const int kind = ctx->kt_kind[i / 2];
            if (kind < EP_KK_MFMA) {
                stats->mfma_ms += ms;
                stats->mfma_launches++;
            }
            stats->kernel_ms[kind] += ms;
            stats->kernel_launches[kind]++;
        }
    }
    return EP_OK;
}

// ---------------------------------------------------------------------------
// Map prediction: buffers and the posterior they read
// ---------------------------------------------------------------------------
static int ensure_maps(ep_ctx* ctx) {
    if (ctx->d_iperm) return EP_OK;
    const int64_t N = ctx->g.N();
    const int n = ctx->g.n;
    // trapezoid step count of the observer's sightline to every node, by the
    // same rule as the stars' (0 at the observer)
    std::vector<int32_t> T(N);
    for (int64_t p = 0; p < N; p++) {
        const double x[3] = {(double)(p % n) * ctx->g.h, (double)((p / n) % n) * ctx->g.h,
                             (double)(p / ((int64_t)n * n)) * ctx->g.h};
        const double dv[3] = {x[0] - ctx->g.obs[0], x[1] - ctx->g.obs[1], x[2] - ctx->g.obs[2]};
        const double d = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        if (!(d > 0)) {
            T[p] = 0;
            continue;
        }
        double tt = std::ceil(d / ctx->g.step);
        if (tt < 1) tt = 1;
        T[p] = (int32_t)tt;
    }
    TRY(upload(ctx, &ctx->d_mapT, T));
    TRY(upload(ctx, &ctx->d_iperm, ctx->sym.iperm));
    const int64_t ncell = (int64_t)(n - 1) * (n - 1) * (n - 1);
    TRY(dev_alloc(ctx, &ctx->d_cellS, 36 * ncell));
    for (double** q : {&ctx->d_s1, &ctx->d_s2, &ctx->d_mapmean}) TRY(dev_alloc(ctx, q, N));
    TRY(dev_alloc(ctx, &ctx->d_mapbad, 1));
    return EP_OK;
}

// mu (node order, d_mu) from the current sites at the current
// linearisation point; the fronts hold the factor afterwards
static int maps_factor_and_mean(ep_ctx* ctx) {
    TRY(run_factor(ctx, nullptr));
    TRY(run_solve(ctx));
    return EP_OK;
}

// Sigma on the fronts (selected inversion of the current factor), then the
// packed Sigma blocks of every cell's corners; STATE if an entry is
// non-finite (an off-pattern pair reads as NaN, which the pattern's
// {-2..2}^3 block rules out)
static int maps_sigma(ep_ctx* ctx, bool cells) {
    enqueue_selinv(ctx);
    if (!cells) return EP_OK;
    HIPCHK(hipMemsetAsync(ctx->d_mapbad, 0, sizeof(int), ctx->stream));
    launch_cell_sigma(ctx->stream, ctx->GD, ctx->F, ctx->d_fronts, ctx->d_iperm, ctx->d_snode, ctx->d_cellS,
                      ctx->d_mapbad);
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, ctx->d_mapbad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (bad) {
        ctx->err = "non-finite Sigma in a cell's corner block";
        return EP_ERR_STATE;
    }
    return EP_OK;
}

// ---------------------------------------------------------------------------
// Caller arrays: host memory, or device memory on cfg.device when
// cfg.pointers_on_device = 1.
// ---------------------------------------------------------------------------
static hipMemcpyKind kind_out(const ep_ctx* c) {
    return c->cfg.pointers_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}
// The caller's array as host memory (itself, or a copy staged in buf) for
// the checks and host-side work that read it.
template <class T>
static hipError_t host_view(bool on_device, const T*& p, int64_t n, std::vector<T>& buf) {
    if (!on_device || !p || n <= 0) return hipSuccess;
    buf.resize((size_t)n);
    hipError_t e = hipMemcpy(buf.data(), p, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost);
    p = buf.data();
    return e;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void ep_config_default(ep_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->n = 16;
    c->box_pc = 1000.0;
    c->observer_pc[0] = 500.0;
    c->observer_pc[1] = 0.0;
    c->observer_pc[2] = 500.0;
    c->prior_mean = -7.0;
    c->prior_var = 1.0;
    c->outer_scale_pc = 100.0;
    c->support_pc = 150.0;
    c->vecchia_radius_pc = 0.0;
    c->los_step_pc = 2.0;
    const double tp[5] = {3000.0, 150.0, 7.5e-4, 2000.0, 0.1};   // Sec. 5 hyperprior means
    for (int j = 0; j < 5; j++) c->theta_prior[j] = tp[j];
    c->sun_radius_pc = 8000.0;
    c->bump_width_pc = 400.0;
    c->likelihood = EP_LIK_EXTINCTION;
    c->precision = EP_PREC_FP64;
    c->moments = EP_MOM_QUADRATURE;
    c->damping = 1.0;
    c->cavity_var_floor = 0.0;
    c->relinearize = 1;
    c->relin_step = 1.0;
    c->deterministic = 0;
    c->device = 0;
    c->stream = nullptr;
    c->leaf_size = 0;
    c->hbm_cap_bytes = 0;
    c->profile_kernels = 0;
    c->mixed_fp64_levels = 0;
    c->surrogate_tol = 1e-4;
}

void ep_free(ep_ctx* ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    pitc_free(ctx->pitc);
    for (void* p : ctx->allocs) (void)hipFree(p);
    for (hipEvent_t e : ctx->kt_ev) (void)hipEventDestroy(e);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

int ep_init(const ep_config* cfg, int64_t n_stars, const double* xyz, const double* A_obs, const double* sigma,
            ep_ctx** out) {
    if (!out) { g_tls_err = "out is NULL"; return EP_ERR_INVALID_ARG; }
    *out = nullptr;
    std::string err;
    std::vector<double> hx, ha, hs;
    if (cfg && cfg->pointers_on_device == 1 && n_stars > 0) {
        if (hipSetDevice(cfg->device) != hipSuccess || host_view(true, xyz, 3 * n_stars, hx) != hipSuccess ||
            host_view(true, A_obs, n_stars, ha) != hipSuccess || host_view(true, sigma, n_stars, hs) != hipSuccess) {
            g_tls_err = "copying the star arrays from the device failed";
            return EP_ERR_DEVICE;
        }
    }
    int rc = validate(cfg, n_stars, xyz, A_obs, sigma, err);
    if (rc) { g_tls_err = err; return rc; }
    ep_ctx* ctx = new ep_ctx();
    ctx->cfg = *cfg;
    ctx->S = n_stars;
    try {
        rc = init_impl(ctx, xyz, A_obs, sigma);
    } catch (const std::bad_alloc&) {
        ctx->err = "host allocation failed";
        rc = EP_ERR_OOM;
    }
    if (rc) {
        g_tls_err = ctx->err;
        ep_free(ctx);
        return rc;
    }
    *out = ctx;
    return EP_OK;
}

int ep_sweep(ep_ctx* ctx, ep_sweep_stats* stats) {
    if (!ctx) { g_tls_err = "ctx is NULL"; return EP_ERR_INVALID_ARG; }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    Range r("ep_sweep");
    return sweep_impl(ctx, stats);
}

int ep_posterior_mean(ep_ctx* ctx, double* out) {
    if (!ctx || !out) { g_tls_err = "NULL argument"; return EP_ERR_INVALID_ARG; }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    TRY(run_factor(ctx, nullptr));
    TRY(run_solve(ctx));
    const double* src = ctx->d_mu;
    if (ctx->M) {
        TRY(border_solve(ctx));
        launch_f_mean(ctx->stream, ctx->d_mhat, ctx->d_J, ctx->d_mu, ctx->border, ctx->d_t, ctx->g.N());
        src = ctx->d_t;
    }
    HIPCHK(hipMemcpyAsync(out, src, sizeof(double) * ctx->g.N(), kind_out(ctx), ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
    return EP_OK;
}

int ep_marginal_var(ep_ctx* ctx, double* out) {
    if (!ctx || !out) { g_tls_err = "NULL argument"; return EP_ERR_INVALID_ARG; }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    TRY(run_factor(ctx, nullptr));
    if (ctx->M) {
        TRY(run_solve(ctx));
        TRY(border_solve(ctx));
    }
    enqueue_selinv(ctx);
    launch_diag(ctx->stream, ctx->d_perm, ctx->d_snode, ctx->F, ctx->d_fronts, ctx->d_var, ctx->g.N());
    if (ctx->M) launch_f_var(ctx->stream, ctx->d_Wb, ctx->d_J, ctx->border, ctx->d_var, ctx->g.N());
    HIPCHK(hipMemcpyAsync(out, ctx->d_var, sizeof(double) * ctx->g.N(), kind_out(ctx), ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
    return EP_OK;
}

int ep_theta(ep_ctx* ctx, double* mean, double* cov) {
    if (!ctx || !mean) { g_tls_err = "NULL argument"; return EP_ERR_INVALID_ARG; }
    if (!ctx->M) {
        ctx->err = "ep_theta: the context has no inferred mean parameters (mean_fn CONSTANT)";
        return EP_ERR_STATE;
    }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    TRY(run_factor(ctx, nullptr));
    TRY(run_solve(ctx));
    TRY(border_solve(ctx));
    const hipMemcpyKind k = ctx->cfg.pointers_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
    HIPCHK(hipMemcpyAsync(mean, ctx->border.mu_phi, sizeof(double) * NTHETA, k, ctx->stream));
    if (cov) HIPCHK(hipMemcpyAsync(cov, ctx->border.sinv, sizeof(double) * NTHETA * NTHETA, k, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return EP_OK;
}

const char* ep_last_error(const ep_ctx* ctx) { return ctx ? ctx->err.c_str() : g_tls_err.c_str(); }

int ep_ordering(const ep_ctx* ctx, int32_t* perm) {
    if (!ctx || !perm) { g_tls_err = "NULL argument"; return EP_ERR_INVALID_ARG; }
    if (ctx->cfg.pointers_on_device) {
        if (hipSetDevice(ctx->cfg.device) != hipSuccess ||
            hipMemcpy(perm, ctx->sym.perm.data(), sizeof(int32_t) * ctx->sym.perm.size(), hipMemcpyHostToDevice) !=
                hipSuccess) {
            g_tls_err = "copying the ordering to the device failed";
            return EP_ERR_DEVICE;
        }
    } else {
        std::copy(ctx->sym.perm.begin(), ctx->sym.perm.end(), perm);
    }
    return EP_OK;
}

int ep_density_moments(ep_ctx* ctx, double* mean, double* var) {
    if (!ctx || !mean || !var) { g_tls_err = "NULL argument"; return EP_ERR_INVALID_ARG; }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    TRY(maps_factor_and_mean(ctx));
    const int64_t N = ctx->g.N();
    const double* fmean = ctx->d_mu;
    if (ctx->M) {
        TRY(border_solve(ctx));
        launch_f_mean(ctx->stream, ctx->d_mhat, ctx->d_J, ctx->d_mu, ctx->border, ctx->d_y, N);
        fmean = ctx->d_y;
    }
    enqueue_selinv(ctx);
    launch_diag(ctx->stream, ctx->d_perm, ctx->d_snode, ctx->F, ctx->d_fronts, ctx->d_var, ctx->g.N());
    if (ctx->M) launch_f_var(ctx->stream, ctx->d_Wb, ctx->d_J, ctx->border, ctx->d_var, N);
    // the two outputs go through d_x and d_t
    launch_density(ctx->stream, fmean, ctx->d_var, ctx->d_x, ctx->d_t, N);
    HIPCHK(hipMemcpyAsync(mean, ctx->d_x, sizeof(double) * N, kind_out(ctx), ctx->stream));
    HIPCHK(hipMemcpyAsync(var, ctx->d_t, sizeof(double) * N, kind_out(ctx), ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
    return EP_OK;
}

int ep_extinction_map(ep_ctx* ctx, int32_t n_samples, const double* z, double* mean, double* var) {
    if (!ctx || !mean || n_samples < 0 || (var && (n_samples < 2 || !z))) {
        g_tls_err = "ep_extinction_map: bad arguments";
        if (ctx) ctx->err = g_tls_err;
        return EP_ERR_INVALID_ARG;
    }
    const int64_t N = ctx->g.N();
    HIPCHK(hipSetDevice(ctx->cfg.device));
    std::vector<double> hz;
    if (var) HIPCHK(host_view(ctx->cfg.pointers_on_device != 0, z, (int64_t)n_samples * N, hz));
    if (z && var)
        for (int64_t i = 0; i < (int64_t)n_samples * N; i++)
            if (!std::isfinite(z[i])) {
                ctx->err = "ep_extinction_map: z must be finite";
                return EP_ERR_INVALID_ARG;
            }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    if (ctx->M) {
        ctx->err = "ep_extinction_map: not available with an inferred prior mean (mean_fn DISC_BUMP)";
        return EP_ERR_STATE;
    }
    TRY(ensure_maps(ctx));
    TRY(maps_factor_and_mean(ctx));
    // Posterior draws f = mu + L^{-T} z need the factor, so they come before
    // the selected inversion overwrites it with Sigma.  Their A are summed as
    // deviations from a centre, A at f = mu (the shifted sums give the
    // sample variance exactly for any centre, with less cancellation).
    const bool sample = var != nullptr;
    if (sample) {
        launch_ext_plugin(ctx->stream, ctx->GD, ctx->d_mapT, ctx->d_mu, ctx->d_mapmean, N);
        launch_fill(ctx->stream, ctx->d_s1, N, 0.0);
        launch_fill(ctx->stream, ctx->d_s2, N, 0.0);
        TRY(ensure_mr(ctx));
        for (int k0 = 0; k0 < n_samples; k0 += MR_MAX) {
            const int nb = std::min(MR_MAX, n_samples - k0);
            HIPCHK(hipMemcpyAsync(ctx->d_ymr, z + (int64_t)k0 * N, sizeof(double) * N * nb, hipMemcpyHostToDevice,
                                  ctx->stream));   // z is host memory here (staged if need be)
            enqueue_bwd_mr(ctx, nb, ctx->d_omr);
            for (int q = 0; q < nb; q++) {
                double* fk = ctx->d_omr + (int64_t)q * N;
                launch_sum2(ctx->stream, fk, ctx->d_mu, fk, N);
                launch_ext_sample(ctx->stream, ctx->GD, ctx->d_mapT, fk, ctx->d_mapmean, ctx->d_s1, ctx->d_s2, N);
            }
        }
        launch_sample_var(ctx->stream, ctx->d_s1, ctx->d_s2, ctx->d_t, n_samples, N);
        HIPCHK(hipMemcpyAsync(var, ctx->d_t, sizeof(double) * N, kind_out(ctx), ctx->stream));
    }
    TRY(maps_sigma(ctx, true));
    launch_ext_mean(ctx->stream, ctx->GD, ctx->d_mapT, ctx->d_mu, ctx->d_cellS, ctx->d_mapmean, N);
    HIPCHK(hipMemcpyAsync(mean, ctx->d_mapmean, sizeof(double) * N, kind_out(ctx), ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
    return EP_OK;
}

int ep_point_predict(ep_ctx* ctx, int64_t n_pairs, const double* xyz2, double* out5) {
    if (!ctx || n_pairs < 0 || (n_pairs > 0 && (!xyz2 || !out5))) {
        g_tls_err = "ep_point_predict: bad arguments";
        if (ctx) ctx->err = g_tls_err;
        return EP_ERR_INVALID_ARG;
    }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    std::vector<double> hp;
    HIPCHK(host_view(ctx->cfg.pointers_on_device != 0, xyz2, 6 * n_pairs, hp));
    for (int64_t i = 0; i < 6 * n_pairs; i++)
        if (!std::isfinite(xyz2[i]) || xyz2[i] < 0 || xyz2[i] > ctx->g.L) {
            ctx->err = "ep_point_predict: points must lie in the cube";
            return EP_ERR_INVALID_ARG;
        }
    // the two cells must touch (the forward model's cell rule), which keeps
    // all 16 corners pairwise on the factor's pattern
    for (int64_t i = 0; i < n_pairs; i++)
        for (int a = 0; a < 3; a++) {
            auto cell = [&](double s) { return std::min<double>(std::max<double>(std::floor(s / ctx->g.h), 0), ctx->g.n - 2); };
            if (std::fabs(cell(xyz2[6 * i + a]) - cell(xyz2[6 * i + 3 + a])) > 1) {
                ctx->err = "ep_point_predict: the two points of a pair must lie in the same or touching cells";
                return EP_ERR_INVALID_ARG;
            }
        }
    if (n_pairs == 0) return EP_OK;
    HIPCHK(hipSetDevice(ctx->cfg.device));
    if (ctx->M) {
        ctx->err = "ep_point_predict: not available with an inferred prior mean (mean_fn DISC_BUMP)";
        return EP_ERR_STATE;
    }
    TRY(ensure_maps(ctx));
    if (ctx->pts_cap < n_pairs) {
        TRY(dev_alloc(ctx, &ctx->d_pts, 11 * n_pairs));
        ctx->pts_cap = n_pairs;
    }
    TRY(maps_factor_and_mean(ctx));
    TRY(maps_sigma(ctx, false));
    HIPCHK(hipMemcpyAsync(ctx->d_pts, xyz2, sizeof(double) * 6 * n_pairs, hipMemcpyHostToDevice, ctx->stream));
    // (xyz2 is host memory here, staged if need be)
    HIPCHK(hipMemsetAsync(ctx->d_mapbad, 0, sizeof(int), ctx->stream));
    launch_point_pred(ctx->stream, ctx->GD, ctx->F, ctx->d_fronts, ctx->d_iperm, ctx->d_snode, ctx->d_mu, ctx->d_pts,
                      ctx->d_pts + 6 * n_pairs, n_pairs, ctx->d_mapbad);
    int bad = 0;
    HIPCHK(hipMemcpyAsync(out5, ctx->d_pts + 6 * n_pairs, sizeof(double) * 5 * n_pairs, kind_out(ctx),
                          ctx->stream));
    HIPCHK(hipMemcpyAsync(&bad, ctx->d_mapbad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
    if (bad) {
        ctx->err = "non-finite Sigma among the corners of a pair of points";
        return EP_ERR_STATE;
    }
    return EP_OK;
}

int ep_get_sites(ep_ctx* ctx, double* tau, double* nu) {
    if (!ctx) { g_tls_err = "ctx is NULL"; return EP_ERR_INVALID_ARG; }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    if (tau) HIPCHK(hipMemcpyAsync(tau, ctx->d_tau, sizeof(double) * ctx->S, kind_out(ctx), ctx->stream));
    if (nu) HIPCHK(hipMemcpyAsync(nu, ctx->d_nu, sizeof(double) * ctx->S, kind_out(ctx), ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return EP_OK;
}

int ep_set_sites(ep_ctx* ctx, const double* tau, const double* nu) {
    if (!ctx || !tau || !nu) { g_tls_err = "NULL argument"; return EP_ERR_INVALID_ARG; }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    std::vector<double> ht, hn;
    HIPCHK(host_view(ctx->cfg.pointers_on_device != 0, tau, ctx->S, ht));
    HIPCHK(host_view(ctx->cfg.pointers_on_device != 0, nu, ctx->S, hn));
    for (int64_t s = 0; s < ctx->S; s++)
        if (!std::isfinite(tau[s]) || !std::isfinite(nu[s])) {
            ctx->err = "sites must be finite";
            return EP_ERR_INVALID_ARG;
        }
    HIPCHK(hipMemcpyAsync(ctx->d_tau, tau, sizeof(double) * ctx->S, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->d_nu, nu, sizeof(double) * ctx->S, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return EP_OK;
}

int ep_set_gmm(ep_ctx* ctx, int32_t K, const double* comps) {
    if (!ctx || (ctx->S > 0 && !comps) || K < 1 || K > 8) {
        g_tls_err = "ep_set_gmm: bad arguments";
        if (ctx) ctx->err = g_tls_err;
        return EP_ERR_INVALID_ARG;
    }
    if (ctx->cfg.likelihood != EP_LIK_GMM) {
        ctx->err = "ep_set_gmm: the context's likelihood is not GMM";
        return EP_ERR_STATE;
    }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    const int64_t n = ctx->S * K * 6;
    std::vector<double> hc;
    HIPCHK(host_view(ctx->cfg.pointers_on_device != 0, comps, n, hc));
    for (int64_t s = 0; s < ctx->S; s++) {
        double wsum = 0;
        for (int z = 0; z < K; z++) {
            const double* c = comps + (s * K + z) * 6;
            for (int k = 0; k < 6; k++)
                if (!std::isfinite(c[k])) { ctx->err = "ep_set_gmm: non-finite component"; return EP_ERR_INVALID_ARG; }
            const bool ok = c[0] >= 0 && c[5] > 0 && c[3] >= 0 &&
                            (c[3] * c[5] - c[4] * c[4] > 0 || (c[3] == 0 && c[4] == 0));
            if (!ok) {
                ctx->err = "ep_set_gmm: star " + std::to_string(s) +
                           " needs weights >= 0 and covariances with C_bb > 0 that are positive definite";
                return EP_ERR_INVALID_ARG;
            }
            wsum += c[0];
        }
        if (!(wsum > 0)) { ctx->err = "ep_set_gmm: star " + std::to_string(s) + " has no positive weight"; return EP_ERR_INVALID_ARG; }
    }
    if (gmm_lds_doubles(ctx->gmm_kcap, K) * (int64_t)sizeof(double) > 65536) {
        ctx->err = "ep_set_gmm: the sightlines extended to the cube's face have " + std::to_string(ctx->gmm_kcap) +
                   " samples; with " + std::to_string(K) + " components they exceed the 64 KB the kernel keeps in LDS";
        return EP_ERR_INVALID_ARG;
    }
    if (ctx->gmm_K != K) {
        if (ctx->d_gmm) {   // resize: the old buffer stays in the context's list until ep_free
            ctx->d_gmm = nullptr;
        }
        TRY(dev_alloc(ctx, &ctx->d_gmm, n));
    }
    if (n > 0) HIPCHK(hipMemcpyAsync(ctx->d_gmm, comps, sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->gmm_K = K;
    return EP_OK;
}

int ep_get_linpoint(ep_ctx* ctx, double* f) {
    if (!ctx || !f) { g_tls_err = "NULL argument"; return EP_ERR_INVALID_ARG; }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    const int64_t N = ctx->g.N();
    HIPCHK(hipMemcpyAsync(f, ctx->d_fhat, sizeof(double) * N, kind_out(ctx), ctx->stream));
    if (ctx->M)   // then phihat
        HIPCHK(hipMemcpyAsync(f + N, ctx->phihat, sizeof(double) * NTHETA,
                              ctx->cfg.pointers_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return EP_OK;
}

int ep_set_linpoint(ep_ctx* ctx, const double* f) {
    if (!ctx || !f) { g_tls_err = "NULL argument"; return EP_ERR_INVALID_ARG; }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    std::vector<double> hf;
    const int64_t N = ctx->g.N(), n = N + ctx->M;
    HIPCHK(host_view(ctx->cfg.pointers_on_device != 0, f, n, hf));
    for (int64_t i = 0; i < n; i++)
        if (!std::isfinite(f[i])) { ctx->err = "linearisation point must be finite"; return EP_ERR_INVALID_ARG; }
    HIPCHK(hipMemcpyAsync(ctx->d_fhat, f, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream));
    if (ctx->M) {
        for (int j = 0; j < NTHETA; j++) ctx->phihat[j] = f[N + j];
        enqueue_mean(ctx);
        ctx->linearised = false;   // the border rows h_n, c'_n follow the mean's linearisation
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return EP_OK;
}

int ep_star_state(ep_ctx* ctx, double* lnA, double* cav_mu, double* cav_var, double* lnZ, double* tmean,
                  double* tvar) {
    if (!ctx) { g_tls_err = "ctx is NULL"; return EP_ERR_INVALID_ARG; }
    const size_t b = sizeof(double) * ctx->S;
    hipStream_t st = ctx->stream;
    const hipMemcpyKind k = kind_out(ctx);
    HIPCHK(hipSetDevice(ctx->cfg.device));
    if (lnA) HIPCHK(hipMemcpyAsync(lnA, ctx->d_lnA, b, k, st));
    if (cav_mu) HIPCHK(hipMemcpyAsync(cav_mu, ctx->d_cmu, b, k, st));
    if (cav_var) HIPCHK(hipMemcpyAsync(cav_var, ctx->d_cvar, b, k, st));
    if (lnZ) HIPCHK(hipMemcpyAsync(lnZ, ctx->d_lnZ, b, k, st));
    if (tmean) HIPCHK(hipMemcpyAsync(tmean, ctx->d_tmean, b, k, st));
    if (tvar) HIPCHK(hipMemcpyAsync(tvar, ctx->d_tvar, b, k, st));
    HIPCHK(hipStreamSynchronize(st));
    return EP_OK;
}

int ep_mlp_load(ep_ctx* ctx, const float* weights) {
    if (!ctx || !weights) { g_tls_err = "NULL argument"; return EP_ERR_INVALID_ARG; }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    std::vector<float> hw;
    HIPCHK(host_view(ctx->cfg.pointers_on_device != 0, weights, MLP_NPARAM, hw));
    for (int i = 0; i < MLP_NPARAM; i++)
        if (!std::isfinite(weights[i])) { ctx->err = "network weights must be finite"; return EP_ERR_INVALID_ARG; }
    for (int k = 0; k < 7; k++)
        if (!(weights[MLP_NTRAIN + 4 + (k < 4 ? k : k + 3)] > 0)) {
            ctx->err = "standardisation scales must be > 0";
            return EP_ERR_INVALID_ARG;
        }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    HIPCHK(hipMemcpyAsync(ctx->d_mlp_P, weights, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, ctx->stream));
    mlp_make_bf16(ctx->stream, ctx->d_mlp_P, ctx->d_mlp_bf);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
    ctx->mlp_loaded = true;
    return EP_OK;
}

int ep_structure(const ep_ctx* ctx, ep_structure_stats* out) {
    if (!ctx || !out) { g_tls_err = "NULL argument"; return EP_ERR_INVALID_ARG; }
    out->n_nodes = ctx->g.N();
    out->n_stars = ctx->S;
    out->nnz_g = (int64_t)ctx->sup.nodes.size();
    out->n_fronts = (int64_t)ctx->sym.fronts.size();
    out->n_levels = ctx->sym.nlevels;
    out->front_elems = ctx->sym.total_elems;
    out->max_front = ctx->sym.max_m;
    out->factor_flops = ctx->sym.factor_flops;
    out->selinv_flops = ctx->sym.selinv_flops;
    out->trail_flops = ctx->sym.trail_flops;
    out->device_bytes = ctx->dev_bytes;
    out->front_elems_lower = 0;
    out->update_elems = out->offdiag_elems = out->x_elems = 0;
    for (const Front& f : ctx->sym.fronts) {
        const int64_t T = f.m / TS;
        out->front_elems_lower += (int64_t)TS * TS * T * (T + 1) / 2;
        out->update_elems += (int64_t)f.nr * (f.nr + 1) / 2;
        out->offdiag_elems += (int64_t)f.nr * f.nv;
        out->x_elems += (int64_t)f.nvpad * f.nvpad;
    }
    out->clique_pairs = 0;
    for (int64_t s = 0; s < ctx->S; s++) {
        const int64_t c = ctx->sup.ptr[s + 1] - ctx->sup.ptr[s];
        out->clique_pairs += c * (c + 1) / 2;
    }
    return EP_OK;
}

int ep_tilted_moments(int32_t mode, int64_t n, const double* mu_c, const double* v_c, const double* A,
                      const double* sigma, double* lnZ, double* mean, double* var, int32_t device) {
    if (n < 0 || (n > 0 && (!mu_c || !v_c || !A || !sigma || !lnZ || !mean || !var))) {
        g_tls_err = "bad arguments";
        return EP_ERR_INVALID_ARG;
    }
    if (mode != 0 && mode != 1) { g_tls_err = "unknown mode"; return EP_ERR_INVALID_ARG; }
    for (int64_t i = 0; i < n; i++)
        if (!(v_c[i] > 0) || !(sigma[i] > 0) || !std::isfinite(mu_c[i]) || !std::isfinite(A[i]) ||
            !std::isfinite(v_c[i]) || !std::isfinite(sigma[i])) {
            g_tls_err = "inputs must be finite with v_c > 0 and sigma > 0";
            return EP_ERR_INVALID_ARG;
        }
    if (n == 0) return EP_OK;
    if (hipSetDevice(device) != hipSuccess) { g_tls_err = "hipSetDevice failed"; return EP_ERR_DEVICE; }
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        g_tls_err = "stream creation failed";
        return EP_ERR_DEVICE;
    }
    if (set_gauss_legendre(st) != hipSuccess) {
        g_tls_err = "quadrature table upload failed";
        (void)hipStreamDestroy(st);
        return EP_ERR_DEVICE;
    }
    double* d = nullptr;
    const size_t b = sizeof(double) * n;
    int rc = EP_OK;
    if (hipMalloc((void**)&d, 7 * b) != hipSuccess) {
        g_tls_err = "device allocation failed";
        (void)hipStreamDestroy(st);
        return EP_ERR_OOM;
    }
    hipError_t e = hipSuccess;
    auto keep = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    keep(hipMemcpyAsync(d, mu_c, b, hipMemcpyHostToDevice, st));
    keep(hipMemcpyAsync(d + n, v_c, b, hipMemcpyHostToDevice, st));
    keep(hipMemcpyAsync(d + 2 * n, A, b, hipMemcpyHostToDevice, st));
    keep(hipMemcpyAsync(d + 3 * n, sigma, b, hipMemcpyHostToDevice, st));
    if (e == hipSuccess) launch_tilted_batch(st, mode, n, d, d + n, d + 2 * n, d + 3 * n, d + 4 * n, d + 5 * n, d + 6 * n);
    keep(hipMemcpyAsync(lnZ, d + 4 * n, b, hipMemcpyDeviceToHost, st));
    keep(hipMemcpyAsync(mean, d + 5 * n, b, hipMemcpyDeviceToHost, st));
    keep(hipMemcpyAsync(var, d + 6 * n, b, hipMemcpyDeviceToHost, st));
    keep(hipStreamSynchronize(st));
    keep(hipGetLastError());
    if (e != hipSuccess) {
        g_tls_err = "tilted-moment kernel failed";
        rc = EP_ERR_DEVICE;
    }
    (void)hipFree(d);
    (void)hipStreamDestroy(st);
    return rc;
}

int ep_simulate(const ep_config* cfg, int64_t n_stars, const double* xyz, const double* sigma, const double* eps,
                const double* xi, double* f_true, double* A_obs) {
    std::vector<double> ones(std::max<int64_t>(n_stars, 1), 0.0);
    std::string err;
    std::vector<double> sg(sigma ? sigma : ones.data(), (sigma ? sigma : ones.data()) + n_stars);
    for (auto& v : sg) if (!(v > 0)) v = 1.0;
    int rc = validate(cfg, n_stars, xyz, ones.data(), sg.data(), err);
    if (rc) { g_tls_err = err; return rc; }
    if (!xi || (n_stars > 0 && (!sigma || !eps))) { g_tls_err = "NULL argument"; return EP_ERR_INVALID_ARG; }
    GridGeom g;
    PriorParams pp;
    geom_from_cfg(cfg, g, pp);
    Stencil st;
    build_stencil(g, pp.rho, st);
    Vecchia v;
    if (build_vecchia(g, pp, st, v) != 0) { g_tls_err = "Vecchia prior not positive definite"; return EP_ERR_NUMERIC; }
    const int64_t N = g.N();
    const bool disc = cfg->mean_fn == EP_MEAN_DISC_BUMP;
    std::vector<double> f(N);
    prior_draw(g, v, disc ? 0.0 : pp.mean, xi, f.data());
    if (!disc) {
        if (f_true) std::copy(f.begin(), f.end(), f_true);
        if (!A_obs || n_stars == 0) return EP_OK;
    }
    // the disc + bump mean at theta_prior, and the line-of-sight integrals,
    // on the GPU with the library's kernels
    ep_config c2 = *cfg;
    ep_ctx* ctx = new ep_ctx();
    ctx->cfg = c2;
    ctx->S = n_stars;
    ctx->g = g;
    ctx->pp = pp;
    struct Del {
        ep_ctx* c;
        ~Del() { ep_free(c); }
    } del{ctx};
    HIPCHK(hipSetDevice(c2.device));
    HIPCHK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    ctx->own_stream = true;
    GridDev GD{g.n, g.h, g.obs[0], g.obs[1], g.obs[2]};
    std::vector<double> mfield((size_t)N, pp.mean);
    if (disc) {
        TRY(dev_alloc(ctx, &ctx->d_mhat, N));
        TRY(dev_alloc(ctx, &ctx->d_J, NTHETA * N));
        MeanDev P{};
        for (int j = 0; j < NTHETA; j++) P.theta[j] = cfg->theta_prior[j];
        P.R0 = cfg->sun_radius_pc;
        P.w = cfg->bump_width_pc;
        launch_mean_fn(ctx->stream, GD, P, ctx->d_mhat, ctx->d_J, N);
        HIPCHK(hipMemcpyAsync(mfield.data(), ctx->d_mhat, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        HIPCHK(hipGetLastError());
        for (int64_t i = 0; i < N; i++) f[i] += mfield[i];
        if (f_true) std::copy(f.begin(), f.end(), f_true);
        if (!A_obs || n_stars == 0) return EP_OK;
    }
    build_supports(g, n_stars, xyz, ctx->sup);
    int cap = 0;
    for (int64_t s = 0; s < n_stars; s++) cap = std::max<int>(cap, (int)(ctx->sup.ptr[s + 1] - ctx->sup.ptr[s]));
    if (cap > 1300) { g_tls_err = "a sightline touches more than 1300 nodes"; return EP_ERR_INVALID_ARG; }
    std::vector<double> vx(xyz, xyz + 3 * n_stars);
    TRY(upload(ctx, &ctx->d_xyz, vx));
    TRY(upload(ctx, &ctx->d_sptr, ctx->sup.ptr));
    TRY(upload(ctx, &ctx->d_snodes, ctx->sup.nodes));
    TRY(upload(ctx, &ctx->d_nsamp, ctx->sup.nsamp));
    TRY(dev_alloc(ctx, &ctx->d_g, (int64_t)ctx->sup.nodes.size()));
    TRY(dev_alloc(ctx, &ctx->d_lnA, n_stars));
    TRY(dev_alloc(ctx, &ctx->d_c, n_stars));
    std::vector<double> field(N);
    const bool gauss = cfg->likelihood == EP_LIK_GAUSS_LINEAR;
    field = gauss ? mfield : f;   // the Gaussian mode's observation operator is frozen at the prior mean
    TRY(upload(ctx, &ctx->d_fhat, field));
    StarsDev SD{};
    SD.n = n_stars; SD.xyz = ctx->d_xyz; SD.ptr = ctx->d_sptr; SD.nodes = ctx->d_snodes; SD.nsamp = ctx->d_nsamp;
    SD.g = ctx->d_g; SD.lnA = ctx->d_lnA; SD.c = ctx->d_c;
    launch_los(ctx->stream, GD, SD, ctx->d_fhat, cap);
    std::vector<double> lnA(n_stars), cc(n_stars), gv(ctx->sup.nodes.size());
    HIPCHK(hipMemcpyAsync(lnA.data(), ctx->d_lnA, sizeof(double) * n_stars, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(cc.data(), ctx->d_c, sizeof(double) * n_stars, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(gv.data(), ctx->d_g, sizeof(double) * gv.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
    for (int64_t s = 0; s < n_stars; s++) {
        double base;
        if (gauss) {
            base = cc[s];
            for (int64_t e = ctx->sup.ptr[s]; e < ctx->sup.ptr[s + 1]; e++) base += gv[e] * f[ctx->sup.nodes[e]];
        } else {
            base = std::exp(lnA[s]);
        }
        A_obs[s] = base + sigma[s] * eps[s];
    }
    return EP_OK;
}

// ---------------------------------------------------------------------------
// PITC sub-catalogue EP and the PIC predictive (pitc.cpp)
// ---------------------------------------------------------------------------
// the sightlines at the constant prior mean (the PITC pass with the
// extinction likelihood linearises there, as the Gaussian pass does)
static void linearise_at_prior_mean(ep_ctx* ctx) {
    launch_fill(ctx->stream, ctx->d_t, ctx->g.N(), ctx->pp.mean);
    launch_los(ctx->stream, ctx->GD, ctx->SD, ctx->d_t, ctx->max_support);
    ctx->linearised = false;
}

static PitcBorrow pitc_borrow(ep_ctx* ctx) {
    PitcBorrow b{};
    b.ext = ctx->cfg.likelihood == EP_LIK_EXTINCTION;
    b.d_tau = ctx->d_tau;
    b.d_nu = ctx->d_nu;
    b.d_qmean = ctx->d_cmu;
    b.d_qvar = ctx->d_cvar;
    b.st = ctx->stream;
    b.g = &ctx->g;
    b.pp = &ctx->pp;
    b.S = ctx->S;
    b.h_sptr = ctx->sup.ptr.data();
    b.h_snodes = ctx->sup.nodes.data();
    b.d_sptr = ctx->d_sptr;
    b.d_g = ctx->d_g;
    b.d_c = ctx->d_c;
    b.d_A = ctx->d_A;
    b.d_sigma = ctx->d_sigma;
    b.M = ctx->M;
    b.d_mhat = ctx->d_mhat;
    b.d_J = ctx->d_J;
    b.d_h = ctx->d_h;
    for (int j = 0; j < ctx->M; j++) {
        b.s0sq[j] = ctx->s0sq[j];
        b.phihat[j] = ctx->phihat[j];
    }
    // what hbm_cap_bytes leaves after the context's own allocations
    b.cap_bytes = ctx->cfg.hbm_cap_bytes > 0 ? std::max<int64_t>(ctx->cfg.hbm_cap_bytes - ctx->dev_bytes, 1) : 0;
    return b;
}

static int pitc_status(ep_ctx* ctx, int rc, const std::string& err) {
    if (rc != EP_OK) {
        ctx->err = err;
        g_tls_err = err;
    }
    return rc;
}

// The PITC pass with the mean parameters reads the context's mean and border
// rows linearised at the hyperprior mean (its oracle's reading).  Grid sweeps
// in the Gaussian mode move that linearisation; then the pass refuses.
static int pitc_mean_at_prior(ep_ctx* ctx, const char* who) {
    for (int j = 0; j < ctx->M; j++)
        if (ctx->phihat[j] != ctx->mu0[j]) {
            ctx->err = std::string(who) +
                       ": the mean parameters' linearisation has moved from the hyperprior mean (grid sweeps "
                       "re-linearise it); the PITC pass linearises at the hyperprior mean: use a fresh context or "
                       "relinearize = 0";
            return EP_ERR_STATE;
        }
    return EP_OK;
}

int ep_pitc_setup(ep_ctx* ctx, int32_t n_blocks, const int32_t* star_block, int64_t n_inducing,
                  const int32_t* inducing, const int32_t* node_block) {
    if (!ctx) {
        g_tls_err = "ep_pitc_setup: null context";
        return EP_ERR_INVALID_ARG;
    }
    if (ctx->cfg.likelihood != EP_LIK_GAUSS_LINEAR && ctx->cfg.likelihood != EP_LIK_EXTINCTION) {
        ctx->err = "ep_pitc_setup: needs likelihood GAUSS_LINEAR or EXTINCTION";
        return EP_ERR_INVALID_ARG;
    }
    if (ctx->cfg.likelihood == EP_LIK_EXTINCTION && ctx->M) {
        ctx->err = "ep_pitc_setup: with the extinction likelihood the pass takes mean_fn CONSTANT";
        return EP_ERR_INVALID_ARG;
    }
    if (n_blocks < 1 || n_inducing < 1 || !star_block || !inducing || !node_block) {
        ctx->err = "ep_pitc_setup: bad arguments";
        return EP_ERR_INVALID_ARG;
    }
    TRY(pitc_mean_at_prior(ctx, "ep_pitc_setup"));
    HIPCHK(hipSetDevice(ctx->cfg.device));
    std::vector<int32_t> hb, hu, hn;
    const bool dev = ctx->cfg.pointers_on_device != 0;
    HIPCHK(host_view(dev, star_block, ctx->S, hb));
    HIPCHK(host_view(dev, inducing, n_inducing, hu));
    HIPCHK(host_view(dev, node_block, ctx->g.N(), hn));
    HIPCHK(hipSetDevice(ctx->cfg.device));
    if (ctx->cfg.likelihood == EP_LIK_EXTINCTION)
        linearise_at_prior_mean(ctx);
    else
        enqueue_linearise(ctx);   // the frozen sightline weights (and h_n) at the prior mean
    HIPCHK(hipStreamSynchronize(ctx->stream));
    pitc_free(ctx->pitc);
    ctx->pitc = nullptr;
    std::string err;
    PitcState* s = nullptr;
    const int rc = pitc_setup(&s, pitc_borrow(ctx), n_blocks, star_block, n_inducing, inducing, node_block, err);
    if (rc == EP_OK) ctx->pitc = s;
    return pitc_status(ctx, rc, err);
}

int ep_pitc_sweep(ep_ctx* ctx, double damping, double* lnZ) {
    if (!ctx || !ctx->pitc) {
        if (ctx) ctx->err = "ep_pitc_sweep: no ep_pitc_setup";
        return ctx ? EP_ERR_STATE : EP_ERR_INVALID_ARG;
    }
    TRY(pitc_mean_at_prior(ctx, "ep_pitc_sweep"));
    HIPCHK(hipSetDevice(ctx->cfg.device));
    std::string err;
    double lz = 0;
    const bool ext = ctx->cfg.likelihood == EP_LIK_EXTINCTION;
    // grid sweeps re-linearise the context's sightlines; the pass takes them
    // at the prior mean
    if (ext) linearise_at_prior_mean(ctx);
    const int rc = pitc_sweep(ctx->pitc, pitc_borrow(ctx), damping, &lz, err);
    if (rc == EP_OK && ext) {
        // the pass left every star's posterior marginal of a_n in the cavity
        // arrays: cavity, tilted moments and damped site update as on the grid
        EpParams p{0, damping, ctx->cfg.cavity_var_floor};
        launch_tilted_update(ctx->stream, ctx->SD, p);
        HIPCHK(hipStreamSynchronize(ctx->stream));
        HIPCHK(hipGetLastError());
    }
    if (rc == EP_OK && lnZ) *lnZ = lz;
    return pitc_status(ctx, rc, err);
}

int ep_pitc_inducing(ep_ctx* ctx, double* mean, double* cov) {
    if (!ctx || !ctx->pitc) {
        if (ctx) ctx->err = "ep_pitc_inducing: no ep_pitc_setup";
        return ctx ? EP_ERR_STATE : EP_ERR_INVALID_ARG;
    }
    TRY(pitc_mean_at_prior(ctx, "ep_pitc_inducing"));
    HIPCHK(hipSetDevice(ctx->cfg.device));
    std::string err;
    if (ctx->cfg.likelihood == EP_LIK_EXTINCTION) linearise_at_prior_mean(ctx);
    return pitc_status(ctx, pitc_inducing(ctx->pitc, pitc_borrow(ctx), mean, cov, kind_out(ctx), err), err);
}

int ep_pitc_theta(ep_ctx* ctx, double* mean, double* cov) {
    if (!ctx || !ctx->pitc) {
        if (ctx) ctx->err = "ep_pitc_theta: no ep_pitc_setup";
        return ctx ? EP_ERR_STATE : EP_ERR_INVALID_ARG;
    }
    TRY(pitc_mean_at_prior(ctx, "ep_pitc_theta"));
    HIPCHK(hipSetDevice(ctx->cfg.device));
    std::string err;
    return pitc_status(ctx, pitc_theta(ctx->pitc, pitc_borrow(ctx), mean, cov, kind_out(ctx), err), err);
}

int ep_pitc_predict(ep_ctx* ctx, double* mean, double* var) {
    if (!ctx || !ctx->pitc) {
        if (ctx) ctx->err = "ep_pitc_predict: no ep_pitc_setup";
        return ctx ? EP_ERR_STATE : EP_ERR_INVALID_ARG;
    }
    TRY(pitc_mean_at_prior(ctx, "ep_pitc_predict"));
    HIPCHK(hipSetDevice(ctx->cfg.device));
    std::string err;
    if (ctx->cfg.likelihood == EP_LIK_EXTINCTION) linearise_at_prior_mean(ctx);
    return pitc_status(ctx, pitc_predict(ctx->pitc, pitc_borrow(ctx), mean, var, kind_out(ctx), err), err);
}

int ep_pitc_info(const ep_ctx* ctx, ep_pitc_stats* out) {
    if (!ctx || !out) {
        g_tls_err = "ep_pitc_info: bad arguments";
        return EP_ERR_INVALID_ARG;
    }
    if (!ctx->pitc) {
        g_tls_err = "ep_pitc_info: no ep_pitc_setup";
        return EP_ERR_STATE;
    }
    pitc_stats(ctx->pitc, out);
    return EP_OK;
}

}  // extern "C"
