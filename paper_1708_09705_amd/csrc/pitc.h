// PITC / PIC block pass: the paper's sub-catalogue EP over the values u of
// the field at inducing nodes (Sec. 4.1, App. A.1, App. B) and the PIC
// predictive at the grid nodes (App. C), on the sightlines and observations
// of an EP context in the gauss_linear likelihood.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

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
// block's B = Sigma_k + S_k - Z Z^T, then rpad rows Z^T, one 64-row tile
// with the residual in its first row, ppad rows D^T.
struct PitcBlockDev {
    int64_t front, kt, at, sat;
    int32_t m, npad, rpad, ppad;
    int32_t nstars, npred;
    int64_t star0, pred0;
};

void launch_pitc_kfill(hipStream_t st, const PitcKJob* jobs, const int64_t* base, int njobs, int64_t ntiles,
                       PitcCovDev cov, const int32_t* ids, double* ws);
void launch_pitc_block_prep(hipStream_t st, const PitcBlockDev* blk, int nblk, const int32_t* stars, const int64_t* sptr,
                            const double* g, const double* c, const double* A, const double* sigma, double m0,
                            double* ws);
void launch_pitc_cfront_prep(hipStream_t st, double* F, int64_t m, int R, int rpad);
void launch_pitc_sum_blocks(hipStream_t st, const double* lam, int nblk, int64_t E, double* out);
void launch_pitc_sites_fronts(hipStream_t st, const double* Snew, double* Ssites, double damp, bool first, double* Fq,
                              int64_t mq, double* Fe, int64_t me, int rpad);
void launch_pitc_lnz(hipStream_t st, const PitcBlockDev* blk, int nblk, const double* ws, const double* Fe, int64_t me,
                     int rpad, const double* Snew, int64_t S, double* out);
void launch_pitc_predict(hipStream_t st, const PitcBlockDev* blk, const int64_t* base, int nblk, int64_t ntasks,
                         const double* ws, const int32_t* pnodes, const double* mu_t, double m0, double k0, int rpad,
                         double* mean, double* var);
void launch_pitc_add_const(hipStream_t st, double* p, int64_t n, double c);

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
};

struct PitcState;
// Each returns 0 (EP_OK) or a negative ep_status with err set.
int pitc_setup(PitcState** out, const PitcBorrow& b, int32_t n_blocks, const int32_t* star_block, int64_t R,
               const int32_t* inducing, const int32_t* node_block, std::string& err);
int pitc_sweep(PitcState* s, const PitcBorrow& b, double damping, double* lnZ, std::string& err);
int pitc_inducing(PitcState* s, const PitcBorrow& b, double* mean, double* cov, hipMemcpyKind kind, std::string& err);
int pitc_predict(PitcState* s, const PitcBorrow& b, double* mean, double* var, hipMemcpyKind kind, std::string& err);
void pitc_stats(const PitcState* s, ep_pitc_stats* out);
void pitc_free(PitcState* s);

}  // namespace ep
