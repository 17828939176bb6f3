// Host side of the PITC / PIC block pass: the plan (every sub-catalogue's
// node sets, work arrays, covariance fills, dense products and block
// Cholesky schedule) and its enqueueing.
//
// Each sub-catalogue k (N_k stars, V_k = the nodes its sightlines touch, P_k
// = the nodes it predicts) works in whitened inducing coordinates
// u = m + L_C v, C = K_uu = L_C L_C^T:
//   Z_k   = rho_k L_C^{-T}                  rho_k = G_k K(V_k, u)
//   B_k   = Sigma_k + S_k - Z_k Z_k^T       Sigma_k = G_k K(V_k, V_k) G_k^T
//   [W_Z | w_r | E] = L_B^{-1} [Z_k | r_k | D_k],  r_k = a~_k - mu_k,
//   D_k = G_k K(V_k, P_k) - Z_k L_C^{-1} K(u, P_k)
// so that B_k^{-1} and p(a~_k | u) = N(mu_k + Z_k v, B_k) give the block's
// site on v: precision W_Z^T W_Z, shift W_Z^T w_r (the natural parameters of
// p(u | a~_k) / p(u), App. B).  B_k, its factor and the W's come out of one
// partial Cholesky of the front [B_k; Z_k^T; r_k^T; D_k^T] (the right-hand
// sides ride along as extra rows), so every sub-catalogue is one front of
// the same batched factorization the sweep uses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/ep.h"
#include "kernels.h"
#include "pitc.h"
#include "task_order.h"

namespace ep {

namespace {

inline int64_t pad64(int64_t x) { return (x + TS - 1) / TS * TS; }

struct Range {
    int64_t off = 0, n = 0;
};
struct TrsmLaunch {
    int64_t be_off = 0;
    int nbe = 0;
    int64_t ntasks = 0;
};
struct FactorPlan {
    std::vector<Range> upd, potrf;
    std::vector<TrsmLaunch> trsm;
};
struct Op {
    int64_t off;
    int ld;
    bool t;
};

struct Blk {
    int nst = 0, nv = 0, np = 0;
    int64_t star0 = 0, v0 = 0, p0 = 0;     // offsets into the star list / id list
    int npad = 0, vpad = 0, ppad = 0;
    int64_t G = 0, KV = 0, KuP = 0, M1 = 0, F = 0, Kt = 0, At = 0, SAt = 0;
    int64_t ZM = 0, TM = 0, TV = 0, CD = 0;   // extinction likelihood only
    int m = 0;
};

}  // namespace

struct PitcState {
    int K = 0, R = 0, rpad = 0;
    int M = 0, xdim = 0;   // mean parameters in the sites; posterior variables x = (v, psi), padded
    int64_t u0 = 0;        // the inducing nodes in d_ids
    PitcMeanDev mean{};
    PitcPriorDev prior{};
    Phi5 phihat{};
    double ln_det_s0 = 0;
    int64_t offT = 0;
    int64_t S = 0, N = 0;
    std::vector<Blk> blk;
    int64_t ws_n = 0, wx_n = 0;
    double *ws = nullptr, *wx = nullptr;
    int64_t offKt = 0, offAt = 0, nKt = 0;
    int64_t offC = 0, offQ = 0, offE = 0, offSnew = 0, offSsites = 0, offSig = 0, offMu = 0, offT1 = 0, offSigU = 0,
            offMuU = 0, offLam = 0, offLnz = 0, offG = 0, nG = 0;
    int mC = 0, mQ = 0, mE = 0;
    int32_t *d_ids = nullptr, *d_stars = nullptr, *d_flist = nullptr, *d_fm = nullptr, *d_fnvpad = nullptr;
    int64_t *d_gdest = nullptr, *d_jobbase = nullptr, *d_predbase = nullptr, *d_foff = nullptr, *d_fxoff = nullptr;
    int64_t nslots = 0, ntiles = 0, npred_tasks = 0;
    int njobs = 0;
    PitcKJob* d_jobs = nullptr;
    PitcBlockDev* d_blk = nullptr;
    BatchEnt* d_be = nullptr;
    GemmTask* d_tasks = nullptr;
    double* d_table = nullptr;
    double *d_mean = nullptr, *d_var = nullptr, *d_theta = nullptr;
    int* d_err = nullptr;
    PitcCovDev cov{};
    FrontsDev F{};
    FactorPlan facC, facB, facQE;
    Range tM1, tZt, tB, tKt, tD, tLam, tSig, tMu, tT1, tSigU, tMuU, tAt, tSAt, tPW, tTM;
    bool ext = false;   // extinction likelihood: star sites under the PITC prior
    std::vector<void*> allocs;
    double m0 = 0, k0 = 0;
    bool swept = false;
    double flops_sweep = 0, flops_pred = 0;
    int64_t dev_bytes = 0, cap_bytes = 0;
};

namespace {

template <typename T>
int dalloc(PitcState* s, T** p, int64_t n, std::string& err) {
    const int64_t bytes = (int64_t)sizeof(T) * std::max<int64_t>(n, 1);
    if (s->cap_bytes > 0 && s->dev_bytes + bytes > s->cap_bytes) {
        err = "pitc: device allocation of " + std::to_string(bytes) + " bytes exceeds hbm_cap_bytes";
        return EP_ERR_OOM;
    }
    void* q = nullptr;
    if (hipMalloc(&q, (size_t)bytes) != hipSuccess) {
        (void)hipGetLastError();
        err = "pitc: hipMalloc of " + std::to_string(bytes) + " bytes failed";
        return EP_ERR_OOM;
    }
    s->allocs.push_back(q);
    s->dev_bytes += bytes;
    *p = (T*)q;
    return EP_OK;
}
template <typename T>
int dupload(PitcState* s, T** p, const std::vector<T>& v, std::string& err) {
    int rc = dalloc(s, p, (int64_t)v.size(), err);
    if (rc) return rc;
    if (!v.empty() && hipMemcpy(*p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess) {
        err = "pitc: upload failed";
        return EP_ERR_DEVICE;
    }
    return EP_OK;
}

// C (M x N, padded sizes; real sizes mr x nr x kr for the flop count)
// [+]= up to two segments +-op(A) op(B), as 256 x 128 block tasks of
// k_gemm_tasks; with lower, only the quadrants on or below the diagonal
// are stored; with tstore, element (i, j) goes to C[j + i ldc].
// Rows [r0, r1) of the K dimension that can be non-zero for one 128-column
// output block (the taper zeroes the rest); real = its non-padding columns.
struct Win {
    int64_t r0 = 0, r1 = 0;
    int real = 0;
};

struct Gemm {
    std::vector<GemmTask>& T;
    double& flops;
    const std::vector<Win>* win = nullptr;   // K windows of the first segment, per 128-column block
    void operator()(int64_t c, int ldc, int M, int N, bool over, bool lower, bool tstore, Op A, Op B, int K, bool neg,
                    const Op* A2, const Op* B2, int K2, bool neg2, double mr, double nr, double kr, double kr2) {
        for (int i0 = 0; i0 < M; i0 += 256)
            for (int j0 = 0; j0 < N; j0 += 128) {
                const int nq = std::min(4, (M - i0) / TS);
                const bool cols2 = N - j0 > TS;
                const int d = (i0 - j0) / TS;
                if (lower && d + 3 < 0) continue;
                GemmTask t{};
                t.c = tstore ? c + j0 + (int64_t)i0 * ldc : c + i0 + (int64_t)j0 * ldc;
                t.ldc = ldc;
                int nseg = 0;
                auto seg = [&](Op a, Op b, int k, bool ng) {
                    GemmSeg g{};
                    g.a = a.t ? a.off + (int64_t)i0 * a.ld : a.off + i0;
                    g.sa = a.t ? TS : (int64_t)TS * a.ld;
                    g.lda = a.ld;
                    g.b = b.t ? b.off + j0 : b.off + (int64_t)j0 * b.ld;
                    g.sb = b.t ? (int64_t)TS * b.ld : TS;
                    g.ldb = b.ld;
                    g.nk = k / TS;
                    g.flags = (a.t ? 1 : 0) | (b.t ? 2 : 0) | (ng ? 4 : 0) | (BUF_FRONTS << 8) | (BUF_FRONTS << 10);
                    t.s[nseg++] = g;
                };
                if (K > 0) {
                    if (win) {
                        // every K tile outside the window multiplies zeros; keep at least one tile so that an
                        // overwriting task still writes its (zero) block
                        const Win& w = (*win)[j0 / 128];
                        const int t0 = (int)std::min<int64_t>(w.r0 / TS, K / TS - 1);
                        const int t1 = (int)std::max<int64_t>(std::min<int64_t>((w.r1 + TS - 1) / TS, K / TS), t0 + 1);
                        Op a = A, b = B;
                        a.off += a.t ? (int64_t)TS * t0 : (int64_t)TS * t0 * a.ld;
                        b.off += b.t ? (int64_t)TS * t0 * b.ld : (int64_t)TS * t0;
                        seg(a, b, TS * (t1 - t0), neg);
                    } else {
                        seg(A, B, K, neg);
                    }
                }
                if (A2 && K2 > 0) seg(*A2, *B2, K2, neg2);
                if (nseg == 0) continue;
                t.flags = (over ? 1 : 0) | (nseg << 4) | (BUF_FRONTS << 8) | gt_shape(nq, cols2, lower, d, tstore);
                T.push_back(t);
            }
        const double area = lower ? 0.5 * mr * (mr + 1.0) : mr * nr;
        if (win) {
            for (const Win& w : *win) flops += 2.0 * mr * w.real * (double)(w.r1 - w.r0);
            flops += 2.0 * area * kr2;
        } else {
            flops += 2.0 * area * (kr + kr2);
        }
    }
};

// Right-looking-by-column Cholesky of the listed fronts' first nvpad
// columns (all rows): before pivot column j, column j takes the updates of
// columns 0..j-1 (one product, K = 64 j); then the diagonal tile's factor
// and inverse, then the tiles below it.
void plan_factor(const std::vector<int>& fronts, const std::vector<int64_t>& off, const std::vector<int>& m,
                 const std::vector<int>& nvpad, std::vector<GemmTask>& tasks, std::vector<int32_t>& flists,
                 std::vector<BatchEnt>& be, FactorPlan& P, double& flops) {
    int Tmax = 0;
    for (int f : fronts) Tmax = std::max(Tmax, nvpad[f] / TS);
    (void)flops;
    for (int j = 0; j < Tmax; j++) {
        Range u;
        u.off = (int64_t)tasks.size();
        if (j > 0) {
            // late columns have few row blocks and a long K: cut K into
            // pieces of at least 8 tiles that add into the column atomically
            // until the launch has ~512 blocks
            int64_t nb = 0;
            for (int f : fronts)
                if (nvpad[f] / TS > j) nb += (m[f] - TS * j + 255) / 256;
            const int split = (int)std::max<int64_t>(1, std::min<int64_t>((512 + nb - 1) / std::max<int64_t>(nb, 1),
                                                                          std::max(1, j / 8)));
            for (int f : fronts) {
                if (nvpad[f] / TS <= j) continue;
                const int64_t o = off[f], mf = m[f];
                for (int i0 = TS * j; i0 < mf; i0 += 256)
                    for (int sp = 0; sp < split; sp++) {
                        const int a0 = (int)((int64_t)j * sp / split), a1 = (int)((int64_t)j * (sp + 1) / split);
                        if (a1 <= a0) continue;
                        GemmTask t{};
                        t.c = o + i0 + (int64_t)TS * j * mf;
                        t.ldc = (int32_t)mf;
                        t.flags = (split > 1 ? 2 : 0) | (1 << 4) | (BUF_FRONTS << 8) |
                                  gt_shape((int)std::min<int64_t>(4, (mf - i0) / TS), false, false, 0, false);
                        GemmSeg g{};
                        g.a = o + i0 + (int64_t)TS * a0 * mf;   // L(i0.., a0..)
                        g.sa = (int64_t)TS * mf;
                        g.lda = (int32_t)mf;
                        g.b = o + TS * j + (int64_t)TS * a0 * mf;   // L(j, a0..)^T
                        g.sb = (int64_t)TS * mf;
                        g.ldb = (int32_t)mf;
                        g.nk = a1 - a0;
                        g.flags = 2 | 4 | (BUF_FRONTS << 8) | (BUF_FRONTS << 10);
                        t.s[0] = g;
                        tasks.push_back(t);
                    }
            }
        }
        u.n = (int64_t)tasks.size() - u.off;
        P.upd.push_back(u);
        Range fl;
        fl.off = (int64_t)flists.size();
        TrsmLaunch tr;
        tr.be_off = (int64_t)be.size();
        int64_t base = 0;
        for (int f : fronts) {
            if (nvpad[f] / TS <= j) continue;
            flists.push_back(f);
            const int64_t cnt = m[f] / TS - j - 1;
            if (cnt <= 0) continue;
            BatchEnt e{};
            e.front = f;
            e.base = base;
            be.push_back(e);
            base += cnt;
        }
        fl.n = (int64_t)flists.size() - fl.off;
        tr.nbe = (int)((int64_t)be.size() - tr.be_off);
        tr.ntasks = base;
        P.potrf.push_back(fl);
        P.trsm.push_back(tr);
    }
}

void enqueue_factor(PitcState* s, hipStream_t st, const FactorPlan& P) {
    Bufs b{s->ws, s->wx, nullptr, nullptr};
    for (size_t j = 0; j < P.upd.size(); j++) {
        launch_gemm_tasks(st, s->d_tasks + P.upd[j].off, P.upd[j].n, b, false);
        launch_potrf(st, s->d_flist + P.potrf[j].off, (int)P.potrf[j].n, (int)j, s->F, b, s->d_err);
        launch_trsm_step(st, s->d_be + P.trsm[j].be_off, P.trsm[j].nbe, P.trsm[j].ntasks, (int)j, s->F, b);
    }
}

void gemm_range(PitcState* s, hipStream_t st, const Range& r) {
    launch_gemm_tasks(st, s->d_tasks + r.off, r.n, Bufs{s->ws, s->wx, nullptr, nullptr}, false);
}

#define PCHK(x)                                                      \
    do {                                                             \
        hipError_t e_ = (x);                                         \
        if (e_ != hipSuccess) {                                      \
            err = std::string("pitc: ") + hipGetErrorString(e_);     \
            return EP_ERR_DEVICE;                                    \
        }                                                            \
    } while (0)
#define PTRY(x)                    \
    do {                           \
        int r_ = (x);              \
        if (r_ != EP_OK) return r_; \
    } while (0)

}  // namespace

void pitc_stats(const PitcState* s, ep_pitc_stats* out) {
    *out = ep_pitc_stats{};
    out->n_blocks = s->K;
    out->n_inducing = s->R;
    for (const Blk& B : s->blk) {
        out->max_block_stars = std::max<int64_t>(out->max_block_stars, B.nst);
        out->max_block_nodes = std::max<int64_t>(out->max_block_nodes, B.nv);
    }
    out->sweep_flops = s->flops_sweep;
    out->predict_flops = s->flops_pred;
    out->device_bytes = s->dev_bytes;
}

void pitc_free(PitcState* s) {
    if (!s) return;
    for (void* p : s->allocs) (void)hipFree(p);
    delete s;
}

int pitc_setup(PitcState** out, const PitcBorrow& b, int32_t n_blocks, const int32_t* star_block, int64_t R,
               const int32_t* inducing, const int32_t* node_block, std::string& err) {
    const int64_t N = b.g->N(), S = b.S;
    if (n_blocks < 1 || R < 1 || R > N || !star_block || !inducing || !node_block) {
        err = "pitc_setup: need n_blocks >= 1, 1 <= n_inducing <= n^3 and all three arrays";
        return EP_ERR_INVALID_ARG;
    }
    std::vector<int64_t> cnt(n_blocks, 0);
    for (int64_t n = 0; n < S; n++) {
        if (star_block[n] < 0 || star_block[n] >= n_blocks) {
            err = "pitc_setup: star_block out of range";
            return EP_ERR_INVALID_ARG;
        }
        cnt[star_block[n]]++;
    }
    for (int k = 0; k < n_blocks; k++)
        if (cnt[k] == 0) {
            err = "pitc_setup: every sub-catalogue needs at least one star";
            return EP_ERR_INVALID_ARG;
        }
    std::vector<int32_t> mark(N, -1);
    for (int64_t r = 0; r < R; r++) {
        if (inducing[r] < 0 || inducing[r] >= N || mark[inducing[r]] >= 0) {
            err = "pitc_setup: inducing nodes must be distinct node ids";
            return EP_ERR_INVALID_ARG;
        }
        mark[inducing[r]] = 0;
    }
    for (int64_t p = 0; p < N; p++)
        if (node_block[p] < 0 || node_block[p] >= n_blocks) {
            err = "pitc_setup: node_block out of range";
            return EP_ERR_INVALID_ARG;
        }
    std::fill(mark.begin(), mark.end(), -1);

    PitcState* s = new PitcState;
    auto fail = [&](int rc) {
        pitc_free(s);
        return rc;
    };
    s->cap_bytes = b.cap_bytes;
    s->ext = b.ext;
    s->K = n_blocks;
    s->R = (int)R;
    s->rpad = (int)pad64(R);
    s->S = S;
    s->N = N;
    s->m0 = b.pp->mean;
    const int rpad = s->rpad;
    s->M = b.M;
    const int hb = b.M > 0 ? TS : 0;   // the tile of the mean parameters' rows
    s->xdim = rpad + hb;
    const int xdim = s->xdim;
    const int64_t e1 = xdim + TS;
    s->prior.M = b.M;
    for (int j = 0; j < b.M; j++) {
        s->prior.s0inv[j] = 1.0 / b.s0sq[j];
        s->ln_det_s0 += std::log(b.s0sq[j]);
        s->phihat.v[j] = b.phihat[j];
    }

    // stars by block (ascending ids), node sets, prediction nodes
    std::vector<int32_t> stars;
    stars.reserve(S);
    s->blk.assign(n_blocks, Blk{});
    {
        std::vector<std::vector<int32_t>> by(n_blocks);
        for (int64_t n = 0; n < S; n++) by[star_block[n]].push_back((int32_t)n);
        for (int k = 0; k < n_blocks; k++) {
            s->blk[k].star0 = (int64_t)stars.size();
            s->blk[k].nst = (int)by[k].size();
            stars.insert(stars.end(), by[k].begin(), by[k].end());
        }
    }
    std::vector<int32_t> ids;   // V lists, then u, then P lists
    std::vector<std::vector<int32_t>> plist(n_blocks);
    for (int64_t p = 0; p < N; p++) plist[node_block[p]].push_back((int32_t)p);
    std::vector<int64_t> gdest(b.h_sptr[S], -1);
    for (int k = 0; k < n_blocks; k++) {
        Blk& B = s->blk[k];
        std::vector<int32_t> V;
        for (int i = 0; i < B.nst; i++) {
            const int32_t n = stars[B.star0 + i];
            for (int64_t q = b.h_sptr[n]; q < b.h_sptr[n + 1]; q++) {
                const int32_t node = b.h_snodes[q];
                if (mark[node] != k) {
                    mark[node] = k;
                    V.push_back(node);
                }
            }
        }
        std::sort(V.begin(), V.end());
        B.v0 = (int64_t)ids.size();
        B.nv = (int)V.size();
        ids.insert(ids.end(), V.begin(), V.end());
        B.np = (int)plist[k].size();
        B.npad = (int)pad64(B.nst);
        B.vpad = (int)pad64(B.nv);
        B.ppad = (int)pad64(std::max(B.np, 1));
    }
    const int64_t u0 = (int64_t)ids.size();
    s->u0 = u0;
    ids.insert(ids.end(), inducing, inducing + R);
    for (int k = 0; k < n_blocks; k++) {
        s->blk[k].p0 = (int64_t)ids.size();
        ids.insert(ids.end(), plist[k].begin(), plist[k].end());
    }

    // workspace layout (doubles, every offset a multiple of 64)
    int64_t w = 0;
    int maxld = 2 * xdim + TS;
    s->offG = w;
    for (auto& B : s->blk) {
        B.G = w;
        w += (int64_t)B.npad * B.vpad;
    }
    s->nG = w - s->offG;
    for (auto& B : s->blk) {
        B.m = B.npad + rpad + hb + TS + B.ppad + (s->ext ? B.npad : 0);
        maxld = std::max({maxld, B.m, B.vpad, B.npad, B.ppad});
        if (s->ext) {
            B.ZM = w;
            w += (int64_t)B.npad * rpad;
            B.TM = w;
            w += (int64_t)B.npad * rpad;
            B.TV = w;
            w += B.npad;
            B.CD = w;
            w += B.npad;
        }
        B.KV = w;
        w += (int64_t)B.vpad * (B.vpad + rpad + B.ppad);
        B.KuP = w;
        w += (int64_t)rpad * B.ppad;
        B.M1 = w;
        w += (int64_t)B.npad * (B.vpad + rpad);
        B.F = w;
        w += (int64_t)B.m * B.npad;
    }
    // K~^T, A^T and (Sigma~ A)^T of all blocks as three regions with the same
    // block offsets, so that A^T starts as one copy of K~^T
    for (int q = 0; q < 3; q++) {
        if (q == 0) s->offKt = w;
        if (q == 1) s->offAt = w;
        for (auto& B : s->blk) {
            (q == 0 ? B.Kt : (q == 1 ? B.At : B.SAt)) = w;
            w += (int64_t)B.ppad * xdim;
        }
    }
    s->nKt = s->offAt - s->offKt;
    s->offLam = w;
    w += (int64_t)n_blocks * e1 * e1;
    s->mC = 2 * rpad;
    s->mQ = 2 * xdim + TS;
    s->mE = xdim + TS;
    s->offC = w;
    w += (int64_t)s->mC * rpad;
    s->offQ = w;
    w += (int64_t)s->mQ * xdim;
    s->offE = w;
    w += (int64_t)s->mE * xdim;
    for (int64_t* o : {&s->offSnew, &s->offSsites}) {
        *o = w;
        w += e1 * e1;
    }
    s->offSig = w;
    w += (int64_t)xdim * xdim;
    for (int64_t* o : {&s->offT, &s->offT1}) {
        *o = w;
        w += (int64_t)rpad * xdim;
    }
    s->offSigU = w;
    w += (int64_t)rpad * rpad;
    s->offMu = w;
    w += (int64_t)xdim * TS;
    s->offMuU = w;
    w += (int64_t)rpad * TS;
    s->offLnz = w;
    w += TS;
    // the product kernel stages whole 256 x 128 blocks: a pad of 256 leading
    // dimensions keeps its reads of absent quadrants inside the allocation
    s->ws_n = w + 256 * (int64_t)maxld + 4096;

    // fronts: blocks 0..K-1, then C, Q, E; X = the diagonal tiles' inverses
    const int nf = n_blocks + 3;
    std::vector<int64_t> foff(nf), fxoff(nf);
    std::vector<int> fm(nf), fnv(nf);
    int64_t xo = 0;
    for (int k = 0; k < nf; k++) {
        if (k < n_blocks) {
            foff[k] = s->blk[k].F;
            fm[k] = s->blk[k].m;
            fnv[k] = s->blk[k].npad;
        } else {
            const int q = k - n_blocks;
            foff[k] = q == 0 ? s->offC : (q == 1 ? s->offQ : s->offE);
            fm[k] = q == 0 ? s->mC : (q == 1 ? s->mQ : s->mE);
            fnv[k] = q == 0 ? rpad : xdim;
        }
        fxoff[k] = xo;
        xo += (int64_t)fnv[k] * fnv[k];
    }
    s->wx_n = xo + 4096;

    // slot -> G entry
    for (int k = 0; k < n_blocks; k++) {
        const Blk& B = s->blk[k];
        std::vector<int32_t>& col = mark;   // reuse as node -> local column
        for (int i = 0; i < B.nv; i++) col[ids[B.v0 + i]] = i;
        for (int i = 0; i < B.nst; i++) {
            const int32_t n = stars[B.star0 + i];
            for (int64_t q = b.h_sptr[n]; q < b.h_sptr[n + 1]; q++)
                gdest[q] = B.G + i + (int64_t)col[b.h_snodes[q]] * B.npad;
        }
    }
    s->nslots = b.h_sptr[S];

    // covariance fills
    std::vector<PitcKJob> jobs;
    auto job = [&](int64_t out_, int ld, int64_t rows, int nrows, int rp, int64_t cols, int ncols, int cp, bool lower) {
        PitcKJob J{};
        J.out = out_;
        J.ld = ld;
        J.rows = rows;
        J.nrows = nrows;
        J.rpad = rp;
        J.cols = cols;
        J.ncols = ncols;
        J.cpad = cp;
        J.lower = lower ? 1 : 0;
        jobs.push_back(J);
    };
    for (const Blk& B : s->blk) {
        job(B.KV, B.vpad, B.v0, B.nv, B.vpad, B.v0, B.nv, B.vpad, false);
        job(B.KV + (int64_t)B.vpad * B.vpad, B.vpad, B.v0, B.nv, B.vpad, u0, (int)R, rpad, false);
        job(B.KV + (int64_t)B.vpad * (B.vpad + rpad), B.vpad, B.v0, B.nv, B.vpad, B.p0, B.np, B.ppad, false);
        job(B.KuP, rpad, u0, (int)R, rpad, B.p0, B.np, B.ppad, false);
    }
    job(s->offC, s->mC, u0, (int)R, rpad, u0, (int)R, rpad, true);
    std::vector<int64_t> jobbase(jobs.size());
    int64_t tiles = 0;
    for (size_t j = 0; j < jobs.size(); j++) {
        jobbase[j] = tiles;
        tiles += (int64_t)(jobs[j].rpad / TS) * (jobs[j].cpad / TS);
    }
    s->njobs = (int)jobs.size();
    s->ntiles = tiles;

    // covariance table over offsets
    const double h = b.g->h;
    int wmax = (int)std::ceil(b.pp->support / h);
    wmax = std::min(wmax, b.g->n - 1);
    std::vector<double> table((size_t)(wmax + 1) * (wmax + 1) * (wmax + 1));
    for (int a = 0; a <= wmax; a++)
        for (int c = 0; c <= wmax; c++)
            for (int e = 0; e <= wmax; e++)
                table[((size_t)a * (wmax + 1) + c) * (wmax + 1) + e] =
                    cov_tapered(*b.pp, h * std::sqrt((double)(a * a + c * c + e * e)));
    s->k0 = table[0];

    // dense products and factorizations
    std::vector<GemmTask> tasks;
    std::vector<int32_t> flists;
    std::vector<BatchEnt> be;
    double fs = 0, fp = 0;
    Gemm gs{tasks, fs}, gp{tasks, fp};
    auto begin = [&](Range& r) { r.off = (int64_t)tasks.size(); };
    auto end = [&](Range& r) { r.n = (int64_t)tasks.size() - r.off; };
    const Op XCt{s->offC + rpad, s->mC, false}, XCtT{s->offC + rpad, s->mC, true};   // L_C^{-T}, its transpose
    {
        std::vector<int> one{n_blocks};
        plan_factor(one, foff, fm, fnv, tasks, flists, be, s->facC, fs);
    }
    fs += (double)R * R * R / 3.0 + (double)R * R * R;
    // K windows: rows of V_k (ascending ids) that can lie within the taper of
    // a column block's nodes (node ids within w n^2 + w n + w of them)
    const int64_t nn = b.g->n, dwin = (int64_t)wmax * (nn * nn + nn + 1);
    auto windows = [&](const Blk& B, const std::vector<int32_t>& col) {
        std::vector<Win> out;
        const int32_t* V = ids.data() + B.v0;
        for (size_t j0 = 0; j0 < col.size(); j0 += 128) {
            int64_t lo = INT64_MAX, hi = INT64_MIN;
            Win wd;
            for (size_t q = j0; q < std::min(col.size(), j0 + 128); q++)
                if (col[q] >= 0) {
                    lo = std::min<int64_t>(lo, col[q]);
                    hi = std::max<int64_t>(hi, col[q]);
                    wd.real++;
                }
            if (wd.real) {
                wd.r0 = std::lower_bound(V, V + B.nv, lo - dwin) - V;
                wd.r1 = std::upper_bound(V, V + B.nv, hi + dwin) - V;
            }
            out.push_back(wd);
        }
        return out;
    };
    begin(s->tM1);
    for (const Blk& B : s->blk) {   // [G K_VV | rho] = G [K_VV | K_Vu]
        std::vector<int32_t> col((size_t)B.vpad + rpad, -1);
        std::copy(ids.begin() + B.v0, ids.begin() + B.v0 + B.nv, col.begin());
        std::copy(inducing, inducing + R, col.begin() + B.vpad);
        const std::vector<Win> w = windows(B, col);
        gs.win = &w;
        gs(B.M1, B.npad, B.npad, B.vpad + rpad, true, false, false, Op{B.G, B.npad, false}, Op{B.KV, B.vpad, false},
           B.vpad, false, nullptr, nullptr, 0, false, B.nst, B.nv + R, B.nv, 0);
        gs.win = nullptr;
    }
    end(s->tM1);
    balance_xcd(tasks, s->tM1.off, s->tM1.n);
    begin(s->tZt);
    for (const Blk& B : s->blk)   // Z^T = L_C^{-1} rho^T
        gs(B.F + B.npad, B.m, rpad, B.npad, true, false, false, XCtT, Op{B.M1 + (int64_t)B.vpad * B.npad, B.npad, true},
           rpad, false, nullptr, nullptr, 0, false, R, B.nst, R, 0);
    end(s->tZt);
    balance_xcd(tasks, s->tZt.off, s->tZt.n);
    begin(s->tB);
    for (const Blk& B : s->blk) {   // B = (G K_VV) G^T - Z Z^T (lower tiles)
        const Op Zt{B.F + B.npad, B.m, true}, Zn{B.F + B.npad, B.m, false};
        gs(B.F, B.m, B.npad, B.npad, true, true, false, Op{B.M1, B.npad, false}, Op{B.G, B.npad, true}, B.vpad, false,
           &Zt, &Zn, rpad, true, B.nst, B.nst, B.nv, R);
    }
    end(s->tB);
    balance_xcd(tasks, s->tB.off, s->tB.n);
    begin(s->tKt);
    for (const Blk& B : s->blk)   // Kt = (L_C^{-1} K_uP)^T = K_uP^T L_C^{-T}
        gs(B.Kt, B.ppad, B.ppad, rpad, true, false, false, Op{B.KuP, rpad, true}, XCt, rpad, false, nullptr, nullptr,
           0, false, B.np, R, R, 0);
    end(s->tKt);
    balance_xcd(tasks, s->tKt.off, s->tKt.n);
    begin(s->tD);
    for (const Blk& B : s->blk) {   // D = G K_VP - Z (L_C^{-1} K_uP), stored transposed under the residual tile
        const Op Zt{B.F + B.npad, B.m, true}, KtT{B.Kt, B.ppad, true};
        std::vector<int32_t> col((size_t)B.ppad, -1);
        std::copy(ids.begin() + B.p0, ids.begin() + B.p0 + B.np, col.begin());
        const std::vector<Win> w = windows(B, col);
        gs.win = &w;
        gs(B.F + B.npad + rpad + hb + TS, B.m, B.npad, B.ppad, true, false, true, Op{B.G, B.npad, false},
           Op{B.KV + (int64_t)B.vpad * (B.vpad + rpad), B.vpad, false}, B.vpad, false, &Zt, &KtT, rpad, true, B.nst,
           B.np, B.nv, R);
        gs.win = nullptr;
    }
    end(s->tD);
    balance_xcd(tasks, s->tD.off, s->tD.n);
    {
        std::vector<int> blks(n_blocks);
        std::iota(blks.begin(), blks.end(), 0);
        double ff = 0;
        plan_factor(blks, foff, fm, fnv, tasks, flists, be, s->facB, ff);
        for (const Blk& B : s->blk)
            fs += (double)B.nst * B.nst * B.nst / 3.0 + (double)B.nst * B.nst * (R + b.M + 1 + B.np);
    }
    begin(s->tLam);
    for (int k = 0; k < n_blocks; k++) {   // [W_Z | w_r]^T [W_Z | w_r]
        const Blk& B = s->blk[k];
        gs(s->offLam + (int64_t)k * e1 * e1, (int)e1, (int)e1, (int)e1, true, false, false,
           Op{B.F + B.npad, B.m, false}, Op{B.F + B.npad, B.m, true}, B.npad, false, nullptr, nullptr, 0, false,
           R + b.M + 1, R + b.M + 1, B.nst, 0);
    }
    end(s->tLam);
    balance_xcd(tasks, s->tLam.off, s->tLam.n);
    {
        std::vector<int> qe{n_blocks + 1, n_blocks + 2};
        double ff = 0;
        plan_factor(qe, foff, fm, fnv, tasks, flists, be, s->facQE, ff);
        const double X = R + b.M;
        fs += 2.0 * (X * X * X / 3.0) + X * X * (X + 2);
    }
    begin(s->tSig);   // Sigma~ = L_q^{-T} L_q^{-1}
    gs(s->offSig, xdim, xdim, xdim, true, false, false, Op{s->offQ + xdim, s->mQ, false},
       Op{s->offQ + xdim, s->mQ, true}, xdim, false, nullptr, nullptr, 0, false, R + b.M, R + b.M, R + b.M, 0);
    end(s->tSig);
    begin(s->tMu);    // mu~ = L_q^{-T} (L_q^{-1} h)
    gs(s->offMu, xdim, xdim, TS, true, false, false, Op{s->offQ + xdim, s->mQ, false},
       Op{s->offQ + 2 * xdim, s->mQ, true}, xdim, false, nullptr, nullptr, 0, false, R + b.M, 1, R + b.M, 0);
    end(s->tMu);
    double fi = 0;
    Gemm gi{tasks, fi};
    begin(s->tT1);
    const Op Tn{s->offT, rpad, false}, Tt{s->offT, rpad, true};   // T = [L_C | J_u], u = m(phihat) + T x
    gi(s->offT1, rpad, rpad, xdim, true, false, false, Tn, Op{s->offSig, xdim, false}, xdim, false, nullptr, nullptr,
       0, false, R, R + b.M, R + b.M, 0);
    end(s->tT1);
    begin(s->tSigU);
    gi(s->offSigU, rpad, rpad, rpad, true, false, false, Op{s->offT1, rpad, false}, Tt, xdim, false, nullptr, nullptr,
       0, false, R, R, R + b.M, 0);
    end(s->tSigU);
    begin(s->tMuU);
    gi(s->offMuU, rpad, rpad, TS, true, false, false, Tn, Op{s->offMu, xdim, false}, xdim, false, nullptr, nullptr, 0,
       false, R, 1, R, 0);
    end(s->tMuU);
    begin(s->tAt);
    for (const Blk& B : s->blk) {   // A^T = K~^T - E^T W_Z (A^T holds a copy of K~^T)
        const Op Ed{B.F + B.npad + rpad + hb + TS, B.m, false}, WZ{B.F + B.npad, B.m, true};
        gp(B.At, B.ppad, B.ppad, xdim, false, false, false, Ed, WZ, B.npad, true, nullptr, nullptr, 0, false, B.np,
           R + b.M, B.nst, 0);
    }
    end(s->tAt);
    balance_xcd(tasks, s->tAt.off, s->tAt.n);
    begin(s->tSAt);
    for (const Blk& B : s->blk)   // (Sigma~ A)^T = A^T Sigma~
        gp(B.SAt, B.ppad, B.ppad, xdim, true, false, false, Op{B.At, B.ppad, false}, Op{s->offSig, xdim, false}, xdim,
           false, nullptr, nullptr, 0, false, B.np, R + b.M, R + b.M, 0);
    end(s->tSAt);
    balance_xcd(tasks, s->tSAt.off, s->tSAt.n);
    if (s->ext) {
        // the marginals of a: M = Z - P^T W_Z (zm holds Z), P = L_B^{-1} S C
        // in the extra rows, W_Z^T in the Z^T rows; then M Sigma~
        begin(s->tPW);
        for (const Blk& B : s->blk) {
            const int crow = B.npad + rpad + hb + TS + B.ppad;
            gs(B.ZM, B.npad, B.npad, rpad, false, false, false, Op{B.F + crow, B.m, false}, Op{B.F + B.npad, B.m, true},
               B.npad, true, nullptr, nullptr, 0, false, B.nst, R, B.nst, 0);
        }
        end(s->tPW);
        balance_xcd(tasks, s->tPW.off, s->tPW.n);
        begin(s->tTM);
        for (const Blk& B : s->blk)
            gs(B.TM, B.npad, B.npad, rpad, true, false, false, Op{B.ZM, B.npad, false}, Op{s->offSig, xdim, false}, rpad,
               false, nullptr, nullptr, 0, false, B.nst, R, R, 0);
        end(s->tTM);
        balance_xcd(tasks, s->tTM.off, s->tTM.n);
    }
    s->flops_sweep = fs;
    s->flops_pred = fp;

    // device arrays
    std::vector<PitcBlockDev> bd(n_blocks);
    std::vector<int64_t> predbase(n_blocks);
    int64_t pt = 0;
    for (int k = 0; k < n_blocks; k++) {
        const Blk& B = s->blk[k];
        PitcBlockDev& d = bd[k];
        d.front = B.F;
        d.kt = B.Kt;
        d.at = B.At;
        d.sat = B.SAt;
        d.m = B.m;
        d.npad = B.npad;
        d.rpad = rpad;
        d.xdim = xdim;
        d.rrow = B.npad + rpad + hb;
        d.drow = B.npad + rpad + hb + TS;
        d.ppad = B.ppad;
        d.nstars = B.nst;
        d.npred = B.np;
        d.star0 = B.star0;
        d.pred0 = B.p0;
        d.crow = B.npad + rpad + hb + TS + B.ppad;
        d.zm = B.ZM;
        d.tm = B.TM;
        d.tv = B.TV;
        d.cd = B.CD;
        predbase[k] = pt;
        pt += B.np;
    }
    s->npred_tasks = pt;
    std::vector<int32_t> fm32(fm.begin(), fm.end()), fnv32(fnv.begin(), fnv.end());
    int rc;
    if ((rc = dalloc(s, &s->ws, s->ws_n, err)) || (rc = dalloc(s, &s->wx, s->wx_n, err)) ||
        (rc = dupload(s, &s->d_ids, ids, err)) || (rc = dupload(s, &s->d_stars, stars, err)) ||
        (rc = dupload(s, &s->d_gdest, gdest, err)) || (rc = dupload(s, &s->d_jobs, jobs, err)) ||
        (rc = dupload(s, &s->d_jobbase, jobbase, err)) || (rc = dupload(s, &s->d_blk, bd, err)) ||
        (rc = dupload(s, &s->d_predbase, predbase, err)) || (rc = dupload(s, &s->d_tasks, tasks, err)) ||
        (rc = dupload(s, &s->d_flist, flists, err)) || (rc = dupload(s, &s->d_be, be, err)) ||
        (rc = dupload(s, &s->d_foff, foff, err)) || (rc = dupload(s, &s->d_fxoff, fxoff, err)) ||
        (rc = dupload(s, &s->d_fm, fm32, err)) || (rc = dupload(s, &s->d_fnvpad, fnv32, err)) ||
        (rc = dupload(s, &s->d_table, table, err)) || (rc = dalloc(s, &s->d_mean, N, err)) ||
        (rc = dalloc(s, &s->d_var, N, err)) || (rc = dalloc(s, &s->d_err, 1, err)) ||
        (rc = dalloc(s, &s->d_theta, 8 + 64, err)))
        return fail(rc);
    // the whole workspace starts at zero (padding rows and columns are read
    // as operands)
    if (hipMemset(s->ws, 0, sizeof(double) * s->ws_n) != hipSuccess ||
        hipMemset(s->wx, 0, sizeof(double) * s->wx_n) != hipSuccess || hipMemset(s->d_err, 0, sizeof(int)) != hipSuccess) {
        err = "pitc: memset failed";
        return fail(EP_ERR_DEVICE);
    }
    s->mean.mhat = b.M > 0 ? b.d_mhat : nullptr;
    s->mean.J = b.d_J;
    s->mean.h = b.d_h;
    s->mean.m0 = s->m0;
    s->mean.N = N;
    for (int j = 0; j < b.M; j++) s->mean.phihat[j] = b.phihat[j];
    s->cov.table = s->d_table;
    s->cov.n = b.g->n;
    s->cov.w = wmax;
    s->F.off = s->d_foff;
    s->F.m = s->d_fm;
    s->F.nvpad = s->d_fnvpad;
    s->F.nv = s->d_fnvpad;
    s->F.xoff = s->d_fxoff;
    *out = s;
    return EP_OK;
}

// Everything of a pass up to q(x) = N(mu~, Sigma~): the covariance fills,
// the fronts of C and of every sub-catalogue, the sites on x (damped by
// 'damping' for the Gaussian likelihood; recomputed whole from the star
// sites for the extinction likelihood), the factor of the posterior
// precision; lnZ for the Gaussian likelihood.
static int pass_posterior(PitcState* s, const PitcBorrow& b, double damping, std::string& err) {
    hipStream_t st = b.st;
    const int rpad = s->rpad;
    PCHK(hipMemsetAsync(s->d_err, 0, sizeof(int), st));
    launch_fill(st, s->ws + s->offG, s->nG, 0.0);
    launch_scatter_set(st, s->ws, s->d_gdest, b.d_g, s->nslots);
    launch_pitc_kfill(st, s->d_jobs, s->d_jobbase, s->njobs, s->ntiles, s->cov, s->d_ids, s->ws);
    launch_pitc_cfront_prep(st, s->ws + s->offC, s->mC, s->R, rpad);
    enqueue_factor(s, st, s->facC);
    for (const Range* r : {&s->tM1, &s->tZt, &s->tB, &s->tKt}) gemm_range(s, st, *r);
    if (s->M) launch_pitc_kt_j(st, s->d_blk, s->d_predbase, s->K, s->npred_tasks, s->d_ids, s->mean, s->ws);
    gemm_range(s, st, s->tD);
    if (s->ext)
        launch_pitc_ext_prep(st, s->d_blk, s->K, s->d_stars, b.d_sptr, b.d_g, b.d_c, b.d_tau, b.d_nu, s->m0, s->ws);
    else
        launch_pitc_block_prep(st, s->d_blk, s->K, s->d_stars, b.d_sptr, b.d_g, b.d_c, b.d_A, b.d_sigma, s->mean,
                               s->ws);
    enqueue_factor(s, st, s->facB);
    gemm_range(s, st, s->tLam);
    const int64_t e1 = s->xdim + TS;
    launch_pitc_sum_blocks(st, s->ws + s->offLam, s->K, e1 * e1, s->ws + s->offSnew);
    // with the extinction likelihood the sub-catalogues' terms on x follow
    // from the star sites and are taken whole (the star sites are damped)
    launch_pitc_sites_fronts(st, s->ws + s->offSnew, s->ws + s->offSsites, s->ext ? 1.0 : damping, s->ext || !s->swept,
                             s->ws + s->offQ, s->mQ, s->ws + s->offE, s->mE, rpad, s->xdim, s->prior);
    enqueue_factor(s, st, s->facQE);
    gemm_range(s, st, s->tSig);
    gemm_range(s, st, s->tMu);
    if (!s->ext)
        launch_pitc_lnz(st, s->d_blk, s->K, s->ws, s->ws + s->offE, s->mE, s->xdim, s->ws + s->offSnew, s->S,
                        s->ln_det_s0, s->ws + s->offLnz);
    int bad = 0;
    PCHK(hipMemcpyAsync(&bad, s->d_err, sizeof(int), hipMemcpyDeviceToHost, st));
    PCHK(hipStreamSynchronize(st));
    PCHK(hipGetLastError());
    if (bad) {
        err = "pitc: a sub-catalogue or inducing covariance is not positive definite";
        return EP_ERR_NOT_PD;
    }
    return EP_OK;
}

int pitc_sweep(PitcState* s, const PitcBorrow& b, double damping, double* lnZ, std::string& err) {
    if (!(damping > 0.0) || damping > 1.0) {
        err = "pitc_sweep: damping must lie in (0, 1]";
        return EP_ERR_INVALID_ARG;
    }
    hipStream_t st = b.st;
    const int rc = pass_posterior(s, b, damping, err);
    if (rc != EP_OK) return rc;
    double lz = std::nan("");
    if (s->ext) {
        // the posterior marginal of every star's a_n, for the caller's site update
        launch_pitc_ext_mean(st, s->d_blk, s->K, s->d_stars, b.d_sptr, b.d_g, b.d_c, s->m0, s->ws + s->offMu, s->ws,
                             b.d_qmean);
        gemm_range(s, st, s->tPW);
        gemm_range(s, st, s->tTM);
        launch_pitc_ext_var(st, s->d_blk, s->K, s->d_stars, s->ws, b.d_qvar);
    } else {
        PCHK(hipMemcpyAsync(&lz, s->ws + s->offLnz, sizeof(double), hipMemcpyDeviceToHost, st));
    }
    PCHK(hipStreamSynchronize(st));
    PCHK(hipGetLastError());
    s->swept = true;
    if (lnZ) *lnZ = lz;
    return EP_OK;
}

int pitc_inducing(PitcState* s, const PitcBorrow& b, double* mean, double* cov, hipMemcpyKind kind, std::string& err) {
    if (!s->swept) {
        err = "pitc_inducing: no sweep yet";
        return EP_ERR_STATE;
    }
    hipStream_t st = b.st;
    if (s->ext) {   // q(x) from the current star sites
        const int rc = pass_posterior(s, b, 1.0, err);
        if (rc != EP_OK) return rc;
    }
    launch_pitc_build_t(st, s->ws + s->offC, s->mC, s->d_ids + s->u0, s->R, s->rpad, s->xdim, s->mean,
                        s->ws + s->offT);
    for (const Range* r : {&s->tT1, &s->tSigU, &s->tMuU}) gemm_range(s, st, *r);
    launch_pitc_add_mean(st, s->ws + s->offMuU, s->d_ids + s->u0, s->R, s->mean);
    const size_t R = (size_t)s->R;
    if (mean) PCHK(hipMemcpyAsync(mean, s->ws + s->offMuU, sizeof(double) * R, kind, st));
    if (cov)
        PCHK(hipMemcpy2DAsync(cov, sizeof(double) * R, s->ws + s->offSigU, sizeof(double) * s->rpad,
                              sizeof(double) * R, R, kind, st));
    PCHK(hipStreamSynchronize(st));
    PCHK(hipGetLastError());
    return EP_OK;
}

int pitc_theta(PitcState* s, const PitcBorrow& b, double* mean, double* cov, hipMemcpyKind kind, std::string& err) {
    if (!s->swept) {
        err = "pitc_theta: no sweep yet";
        return EP_ERR_STATE;
    }
    if (!s->M) {
        err = "pitc_theta: the context has no inferred mean parameters (mean_fn CONSTANT)";
        return EP_ERR_STATE;
    }
    hipStream_t st = b.st;
    launch_pitc_theta_out(st, s->ws + s->offMu, s->ws + s->offSig, s->xdim, s->rpad, s->M, s->phihat, s->d_theta);
    if (mean) PCHK(hipMemcpyAsync(mean, s->d_theta, sizeof(double) * s->M, kind, st));
    if (cov) PCHK(hipMemcpyAsync(cov, s->d_theta + s->M, sizeof(double) * s->M * s->M, kind, st));
    PCHK(hipStreamSynchronize(st));
    PCHK(hipGetLastError());
    return EP_OK;
}

int pitc_predict(PitcState* s, const PitcBorrow& b, double* mean, double* var, hipMemcpyKind kind, std::string& err) {
    if (!s->swept) {
        err = "pitc_predict: no sweep yet";
        return EP_ERR_STATE;
    }
    hipStream_t st = b.st;
    if (s->ext) {   // q(x) and the scaled fronts from the current star sites
        const int rc = pass_posterior(s, b, 1.0, err);
        if (rc != EP_OK) return rc;
    }
    PCHK(hipMemcpyAsync(s->ws + s->offAt, s->ws + s->offKt, sizeof(double) * s->nKt, hipMemcpyDeviceToDevice, st));
    gemm_range(s, st, s->tAt);
    gemm_range(s, st, s->tSAt);
    launch_pitc_predict(st, s->d_blk, s->d_predbase, s->K, s->npred_tasks, s->ws, s->d_ids, s->ws + s->offMu, s->mean,
                        s->k0, s->d_mean, s->d_var);
    if (mean) PCHK(hipMemcpyAsync(mean, s->d_mean, sizeof(double) * s->N, kind, st));
    if (var) PCHK(hipMemcpyAsync(var, s->d_var, sizeof(double) * s->N, kind, st));
    PCHK(hipStreamSynchronize(st));
    PCHK(hipGetLastError());
    return EP_OK;
}

}  // namespace ep
