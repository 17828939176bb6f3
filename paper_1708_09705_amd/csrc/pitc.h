// PITC / PIC block pass: the paper's sub-catalogue EP over the values u of
// the field at inducing nodes (Sec. 4.1, App. A.1, App. B) and the PIC
// predictive at the grid nodes (App. C), on the sightlines and observations
// of an EP context in the gauss_linear likelihood.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "kernels.h"
#include "prior.h"
#include "symbolic.h"

struct ep_pitc_stats;

namespace ep {

// Covariance between grid nodes from a table over absolute offsets.
struct PitcCovDev {
    const double* table;   // (w + 1)^3, index (|di| (w + 1) + |dj|) (w + 1) + |dk|
    int n;                 // nodes per axis
    int w;                 // largest offset with a non-zero entry
};

// A dense covariance fill: out[r + c ld] = K(ids[rows + r], ids[cols + c])
// for r < nrows, c < ncols, zero elsewhere in rpad x cpad (and in the
// strictly upper 64 x 64 tiles if lower).
struct PitcKJob {
    int64_t out;
    int64_t rows, cols;
    int32_t nrows, ncols, rpad, cpad;
    int32_t ld, lower;
};

// One sub-catalogue's front and work arrays (element offsets into the
// workspace).  Front (m x npad, column-major, ld m): rows [0, npad) the
// block's B = Sigma_k + S_k - Z Z^T, then rpad rows Z^T, with inferred mean
// parameters one 64-row tile H^T (rows 0..4), then one 64-row tile with the
// residual in its first row (at rrow), then ppad rows D^T (from drow).  The
// posterior variables x = (v, psi) are the first xdim = rpad (+ 64) rows
// after B.
struct PitcBlockDev {
    int64_t front, kt, at, sat;
    int32_t m, npad, rpad, ppad, xdim, rrow, drow;
    int32_t nstars, npred;
    int64_t star0, pred0;
    // extinction likelihood: npad more front rows from crow holding (S C)^T
    // (C = Sigma_k - Z Z^T, S = diag sqrt(tau)), the unscaled Z (zm, then
    // Z - P^T W_Z; npad x rpad), T = (Z - P^T W_Z) Sigma~ (tm), a vector of
    // npad (tv: sqrt(tau), then w_r - W_Z mu~) and diag C (cd)
    int32_t crow;
    int64_t zm, tm, tv, cd;
};

// The prior mean of the field: constant m0, or (with the mean parameters in
// the sites) mhat + J psi, J column-major N x 5, h_n = J^T g_n per star; the
// stars' c then hold c'_n = c_n + g_n . mhat - h_n . phihat, so that the
// prior mean of a_n is c'_n + h_n . phihat.
struct PitcMeanDev {
    const double* mhat;   // null: constant m0
    const double* J;
    const double* h;
    double m0;
    int64_t N;
    double phihat[8];
};

void launch_pitc_kfill(hipStream_t st, const PitcKJob* jobs, const int64_t* base, int njobs, int64_t ntiles,
                       PitcCovDev cov, const int32_t* ids, double* ws);
void launch_pitc_block_prep(hipStream_t st, const PitcBlockDev* blk, int nblk, const int32_t* stars, const int64_t* sptr,
                            const double* g, const double* c, const double* A, const double* sigma, PitcMeanDev mean,
                            double* ws);
void launch_pitc_cfront_prep(hipStream_t st, double* F, int64_t m, int R, int rpad);
void launch_pitc_sum_blocks(hipStream_t st, const double* lam, int nblk, int64_t E, double* out);
// The prior precision of x = (v, psi): 1 on v and on padding, 1/s0^2 on the
// M mean-parameter slots (rows rpad .. rpad + M - 1).
struct PitcPriorDev {
    double s0inv[8];
    int M;
};
void launch_pitc_sites_fronts(hipStream_t st, const double* Snew, double* Ssites, double damp, bool first, double* Fq,
                              int64_t mq, double* Fe, int64_t me, int rpad, int xdim, PitcPriorDev prior);
void launch_pitc_lnz(hipStream_t st, const PitcBlockDev* blk, int nblk, const double* ws, const double* Fe, int64_t me,
                     int xdim, const double* Snew, int64_t S, double ln_det_s0, double* out);
void launch_pitc_predict(hipStream_t st, const PitcBlockDev* blk, const int64_t* base, int nblk, int64_t ntasks,
                         const double* ws, const int32_t* pnodes, const double* mu_t, PitcMeanDev mean, double k0,
                         double* out_mean, double* out_var);
// Kt's mean-parameter columns: J at each block's prediction nodes
void launch_pitc_kt_j(hipStream_t st, const PitcBlockDev* blk, const int64_t* base, int nblk, int64_t ntasks,
                      const int32_t* pnodes, PitcMeanDev mean, double* ws);
// T = [L_C | J_u]: rpad x xdim (ld rpad) from the C front and J at the inducing nodes
void launch_pitc_build_t(hipStream_t st, const double* Cf, int64_t mC, const int32_t* unodes, int R, int rpad, int xdim,
                         PitcMeanDev mean, double* T);
// out[r] += mean at inducing node r (r < R)
void launch_pitc_add_mean(hipStream_t st, double* out, const int32_t* unodes, int R, PitcMeanDev mean);
// phi = phihat + mu~[rpad .. rpad + M), then Sigma~ of those slots (row-major): out (M + M^2)
void launch_pitc_theta_out(hipStream_t st, const double* mu_t, const double* sig_t, int xdim, int rpad, int M,
                           Phi5 phihat, double* out);
// Extinction likelihood (sites tau, nu per star; constant prior mean m0):
// copy (S C)^T into the extra rows, diag C and the unscaled Z^T, sqrt(tau)
// into tv; then scale B (I + S C S), Z^T, D^T by S and set the residual
// r~ = (nu - tau mu_a) / sqrt(tau) (0 without a site).
void launch_pitc_ext_prep(hipStream_t st, const PitcBlockDev* blk, int nblk, const int32_t* stars, const int64_t* sptr,
                          const double* g, const double* c, const double* tau, const double* nu, double m0,
                          double* ws);
// After q(v): the posterior mean of every star's a_n (before zm turns into
// Z - P^T W_Z), then (after that product and T) its variance.
void launch_pitc_ext_mean(hipStream_t st, const PitcBlockDev* blk, int nblk, const int32_t* stars, const int64_t* sptr,
                          const double* g, const double* c, double m0, const double* mu_t, double* ws, double* qmean);
void launch_pitc_ext_var(hipStream_t st, const PitcBlockDev* blk, int nblk, const int32_t* stars, const double* ws,
                         double* qvar);

// What the block pass borrows from the EP context.
struct PitcBorrow {
    hipStream_t st;
    const GridGeom* g;
    const PriorParams* pp;
    int64_t S;
    const int64_t* h_sptr;     // host: sightline supports (CSR over stars)
    const int32_t* h_snodes;
    const int64_t* d_sptr;     // device: the same, and per slot weights g,
    const double* d_g;         // per star c, observed a~ and sigma
    const double* d_c;
    const double* d_A;
    const double* d_sigma;
    int64_t cap_bytes;         // device bytes the pass may allocate (0: no cap)
    // the inferred mean parameters (M = 5), or M = 0 for the constant mean
    int M;
    const double* d_mhat;
    const double* d_J;
    const double* d_h;
    double s0sq[8];
    double phihat[8];
    // extinction likelihood: the pass reads the star sites and writes the
    // posterior marginals of every a_n (the grid path's cavity arrays)
    bool ext = false;
    const double* d_tau = nullptr;
    const double* d_nu = nullptr;
    double* d_qmean = nullptr;
    double* d_qvar = nullptr;
};

struct PitcState;
// Each returns 0 (EP_OK) or a negative ep_status with err set.
int pitc_setup(PitcState** out, const PitcBorrow& b, int32_t n_blocks, const int32_t* star_block, int64_t R,
               const int32_t* inducing, const int32_t* node_block, std::string& err);
int pitc_sweep(PitcState* s, const PitcBorrow& b, double damping, double* lnZ, std::string& err);
int pitc_inducing(PitcState* s, const PitcBorrow& b, double* mean, double* cov, hipMemcpyKind kind, std::string& err);
int pitc_predict(PitcState* s, const PitcBorrow& b, double* mean, double* var, hipMemcpyKind kind, std::string& err);
int pitc_theta(PitcState* s, const PitcBorrow& b, double* mean, double* cov, hipMemcpyKind kind, std::string& err);
void pitc_stats(const PitcState* s, ep_pitc_stats* out);
void pitc_free(PitcState* s);

}  // namespace ep
