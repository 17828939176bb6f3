// Device kernels of the EP sweep (gfx950) and their launch wrappers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ep {

constexpr int TS = 64;   // dense tile edge (doubles)
constexpr int PW = 8;    // factorization panel width in tiles

// Base buffers a tile task may address.
enum Buf : int { BUF_FRONTS = 0, BUF_X = 1, BUF_W = 2, BUF_F32 = 3 };

// One K-segment of a tile product: sum_t op(A_t) op(B_t), A_t = A + t*sa.
struct GemmSeg {
    int64_t a, b, sa, sb;
    int32_t lda, ldb, nk;
    int32_t flags;   // 1 transA, 2 transB, 4 negate; bits 8-9 buffer of A, 10-11 buffer of B
};
// C (256 x 128, column-major, ldc) = [C +] sum over segments.  The block is
// eight 64 x 64 quadrants (four 64-row quarters x two 64-column halves):
// only the first gt_rows(flags) row quarters and, with GT_COLS2, the second
// column half are present (their operand rows / columns are neither read
// nor written when absent).  With GT_LOWER, quadrant (r, c) is stored only
// when d + r - c >= 0, d = gt_diag(flags) the block's row tile minus column
// tile (a lower-triangular output).  With GT_TSTORE the block is stored
// transposed: element (i, j) to C[j + i ldc].  A segment's nk counts 64-deep
// K tiles; sa, sb step one of them.  A task without segments is padding and
// does nothing.
struct GemmTask {
    int64_t c;
    int32_t ldc;
    int32_t flags;   // 1 overwrite, 2 atomic add (else accumulate); bits 4-5 nseg; bits 8-9 buffer of C; bits 12-14 row
                     // quarters present; GT_COLS2, GT_LOWER (+ bits 17-19 d + 4), GT_TSTORE
    GemmSeg s[2];
};
constexpr int32_t GT_COLS2 = 1 << 15;    // columns 64..127 present
constexpr int32_t GT_LOWER = 1 << 16;    // store only quadrants on or below the diagonal
constexpr int32_t GT_TSTORE = 1 << 20;   // store the block transposed
__host__ __device__ inline int32_t gt_rows(int32_t flags) { return (flags >> 12) & 7; }
__host__ __device__ inline int32_t gt_diag(int32_t flags) { return ((flags >> 17) & 7) - 4; }
// flags for a block with nq row quarters, an optional second column half,
// optionally lower-triangular with row tile - column tile = d, optionally
// stored transposed
inline int32_t gt_shape(int nq, bool cols2, bool lower, int d, bool tstore) {
    int32_t f = (nq << 12) | (cols2 ? GT_COLS2 : 0) | (tstore ? GT_TSTORE : 0);
    if (lower) f |= GT_LOWER | ((d < -4 ? 0 : (d > 1 ? 5 : d + 4)) << 17);
    return f;
}

// Front metadata (structure of arrays, device pointers).
struct FrontsDev {
    const int64_t* off;     // element offset of the front block
    const int32_t* m;       // padded front order (leading dimension)
    const int32_t* nv;
    const int32_t* nvpad;
    const int32_t* nr;
    const int64_t* first;   // first new index of V
    const int64_t* rptr;    // offset into rrows / relmap
    const int32_t* parent;
    const int64_t* xoff;    // offset of the nvpad x nvpad inverse block in X
    const int32_t* rrows;   // R rows as new indices
    const int32_t* relmap;  // R rows as local rows of the parent front
};

// Clique assembly by tile owner.  A star's clique entries that fall in one
// 64 x 64 tile of its front form an incidence: the star's slots, sorted by
// local row, whose rows lie in the tile's row range (nr of them, from rpos)
// and those whose rows lie in its column range (nc, from cpos).
struct TileInc {
    int32_t star;
    uint16_t r0, c0;   // first row slot, first column slot: positions in the star's sorted slots
    uint16_t nr, nc;
    uint8_t rlo, rhi;  // tile rows of the first and the last row slot
    uint16_t pad;
};
// A run of one tile's incidences, applied in order by one wave.
struct TileChunk {
    int64_t i0;     // first incidence
    int32_t n;      // incidences
    int32_t f;      // front
    int32_t ti, tj; // tile row and column in the front (ti >= tj)
    int32_t part;   // -1: the tile has this chunk only and it adds into the front; else its partial-tile slot
    int32_t pad;
};
// A tile assembled in several chunks: their partial tiles, summed in order.
struct TileRed {
    int32_t f, ti, tj;
    int32_t p0, np;
    int32_t pad;
};

// Per-front task batch entry for implicitly enumerated tile tasks.
struct BatchEnt {
    int32_t front;
    int32_t pad;
    int64_t base;   // first task index of this front in the launch
};

struct Bufs {
    double* fronts;   // FP64 fronts: assembly, FP64 factor, selected inverse
    double* X;        // L11^{-1} of every front
    double* W;        // scratch
    float* F32;       // FP32 copy of the fronts for the mixed-precision factor (or null)
};

// ---- launch wrappers (all asynchronous on 'st') ----
void launch_fill(hipStream_t st, double* p, int64_t n, double v);
void launch_scatter_set(hipStream_t st, double* base, const int64_t* dest, const double* val, int64_t n);
void launch_scatter_const(hipStream_t st, double* base, const int64_t* dest, int64_t n, double v);

void launch_gemm_tasks(hipStream_t st, const GemmTask* t, int64_t n, Bufs b, bool a32);
// the same layout in FP32 on the FP32 copy of the fronts (every offset into F32)
void launch_gemm_tasks_f32(hipStream_t st, const GemmTask* t, int64_t n, float* F32);
// the FP64-buffer tasks of launch_gemm_tasks computed in FP32 arithmetic
void launch_gemm_tasks_x32(hipStream_t st, const GemmTask* t, int64_t n, Bufs b);
void launch_potrf(hipStream_t st, const int32_t* flist, int nf, int k, FrontsDev F, Bufs b, int* err);
void launch_trsm_step(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, int k, FrontsDev F, Bufs b);
// factor_err non-null: the launch also factors the diagonal tile of column
// kk + 1 of every front in it (the next step's potrf), errors as launch_potrf
void launch_syrk_inner(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, int kk, FrontsDev F, Bufs b,
                       int* factor_err = nullptr);
void launch_extend_add(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b);
// the same with at most one child per parent in the launch: no atomics
void launch_extend_add_plain(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b);
void launch_sigma_gather(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b);
// zero the lower-triangular 64 x 64 tiles of the listed fronts
void launch_zero_lower(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, double* fronts);

// solves (vectors in the new node order)
void launch_fwd_xv(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                   const double* y, double* t);
void launch_fwd_r(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                  const double* t, double* y, double* stage = nullptr);
// y[tgt[i]] -= stage[src[e]] for e in [tptr[i], tptr[i+1]), in that order
void launch_gather_sub(hipStream_t st, const int32_t* tgt, const int64_t* tptr, const int64_t* src, int64_t n,
                       const double* stage, double* y);
void launch_copy_v(hipStream_t st, const int32_t* flist, int nf, FrontsDev F, const double* t, double* y);
void launch_bwd_t(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                  const double* y, const double* x, double* t);
void launch_bwd_x(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                  const double* t, double* x);
// the same for nrhs <= MR_MAX vectors at once, column q at q * ld
constexpr int MR_MAX = 8;
void launch_fwd_xv_mr(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                      const double* y, double* t, int nrhs, int64_t ld);
void launch_fwd_r_mr(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                     const double* t, double* y, int nrhs, int64_t ld);
void launch_copy_v_mr(hipStream_t st, const int32_t* flist, int nf, FrontsDev F, const double* t, double* y, int nrhs,
                      int64_t ld);
void launch_bwd_t_mr(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                     const double* y, const double* x, double* t, int nrhs, int64_t ld);
void launch_bwd_x_mr(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                     const double* t, double* x, int nrhs, int64_t ld);
void launch_gather_perm_mr(hipStream_t st, const int32_t* perm, const double* src, int64_t lds, double* dst,
                           int64_t ldd, int nrhs, int64_t n);
void launch_scatter_perm_mr(hipStream_t st, const int32_t* perm, const double* src, int64_t lds, double* dst,
                            int64_t ldd, int nrhs, int64_t n);

// star kernels
struct StarsDev {
    int64_t n;
    const double* xyz;
    const double* A;
    const double* sigma;
    const int64_t* ptr;
    const int32_t* nodes;    // original node ids, sorted per star
    const int32_t* loc;      // local row in the star's front, per slot
    const int32_t* sord;     // slot order by ascending loc, per star (slot indices)
    const int32_t* front;    // front per star
    const int32_t* nsamp;    // trapezoid intervals per star
    double* g;               // per slot
    double* lnA;
    double* c;
    double* tau;
    double* nu;
    double* cav_mu;
    double* cav_var;
    double* lnZ;
    double* tmean;
    double* tvar;
    int32_t* status;         // per star: 0 updated, 1 cavity skip, 2 negative site
    double* dtau;            // per star |delta tau|
    // processing order of the clique kernels (assembly, cavity): slot i of a
    // launch (block i / 4, wave i % 4) takes star order[i] (-1: none); NULL
    // takes star i
    const int32_t* order;
    int64_t norder;
};
struct GridDev {
    int n;
    double h;
    double ox, oy, oz;
};
void launch_los(hipStream_t st, GridDev g, StarsDev s, const double* f, int max_support);

// ---- inferred prior-mean parameters (theta.hip) ----
constexpr int NTHETA = 5;        // (L, H, rho kappa_0, s_bump, A_bump)
constexpr int DOT_BLOCKS = 256;  // blocks of the partial-sum kernels
struct MeanDev {                 // disc + bump mean function at theta
    double theta[NTHETA];
    double R0, w;                // Galactocentric radius of the observer; bump width
};
struct Phi5 { double v[NTHETA]; };
struct BorderDev {
    double mu_phi[NTHETA];
    double phihat[NTHETA];
    double sinv[NTHETA * NTHETA];  // Sigma_phiphi = S^-1, row-major
};
void launch_mean_fn(hipStream_t st, GridDev g, MeanDev P, double* mhat, double* J, int64_t N);
void launch_star_border(hipStream_t st, StarsDev s, const double* mhat, const double* J, Phi5 phihat, double* h,
                        int64_t N);
void launch_border_rhs(hipStream_t st, StarsDev s, const double* h, double* R, int64_t N);
void launch_dots_5x6(hipStream_t st, const double* A, const double* B, int64_t n, double* part);
void launch_star_sums(hipStream_t st, StarsDev s, const double* h, double* part);
void launch_minus_w(hipStream_t st, const double* y, const double* W, Phi5 c, double* out, int64_t N);
void launch_cavity_border(hipStream_t st, StarsDev s, const double* W, const double* h, BorderDev b, int64_t N);
void launch_f_mean(hipStream_t st, const double* mhat, const double* J, const double* mu_d, BorderDev b, double* out,
                   int64_t N);
void launch_f_var(hipStream_t st, const double* W, const double* J, BorderDev b, double* var, int64_t N);
// clique assembly: g in the sorted slot order, then the tile chunks, then
// the sums of the tiles assembled in several chunks (fixed orders throughout)
void launch_sort_g(hipStream_t st, StarsDev s, double* gs, int64_t nslots);
void launch_assemble_tiles(hipStream_t st, const TileChunk* ch, int64_t nch, const TileInc* inc, const int64_t* ptr,
                           const double* tau, const double* gs, const int32_t* ls, FrontsDev F, double* fronts,
                           double* parts);
void launch_tiles_reduce(hipStream_t st, const TileRed* red, int64_t nred, const double* parts, FrontsDev F,
                         double* fronts);
void launch_assemble_b(hipStream_t st, StarsDev s, double* b);
// deterministic form of the above (fixed summation order, no atomics)
void launch_assemble_b_nodes(hipStream_t st, StarsDev s, const int64_t* nptr, const int64_t* nslot,
                             const int32_t* nstar, double* b, int64_t N);
void launch_gather_perm(hipStream_t st, const int32_t* perm, const double* src, double* dst, int64_t n);
void launch_scatter_perm(hipStream_t st, const int32_t* perm, const double* src, double* dst, int64_t n);
void launch_diag(hipStream_t st, const int32_t* perm, const int32_t* snode, FrontsDev F, const double* fronts,
                 double* var, int64_t n);
void launch_cavity(hipStream_t st, StarsDev s, FrontsDev F, const double* fronts, const double* mu,
                   int max_support);
struct EpParams {
    int mode;          // 0 extinction, 1 gaussian, 2 distance mixture
    double damping;
    double vfloor;
};
// unknown distances (gmm.hip): the tilted moments with the distance
// marginalised along each sightline extended to the cube's face, and the site
// update.  gmm_ray_samples: samples of one star's extended sightline (host);
// gmm_lds_doubles: the kernel's LDS per star, kcap >= every star's samples.
int64_t gmm_ray_samples(const double* xyz, const double* obs, int32_t T, double box, double step);
int64_t gmm_lds_doubles(int64_t kcap, int K);
void launch_gmm_ray(hipStream_t st, GridDev g, StarsDev s, EpParams p, const double* f, const double* comps, int K,
                    double box, double step, int kcap);
// list: optional subset of stars (nlist entries)
void launch_tilted_update(hipStream_t st, StarsDev s, EpParams p, const int32_t* list = nullptr, int64_t nlist = 0);
void launch_tilted_batch(hipStream_t st, int mode, int64_t n, const double* mu, const double* v, const double* A,
                         const double* sig, double* lnZ, double* mean, double* var);
hipError_t set_gauss_legendre(hipStream_t st);
void gauss_legendre16(double* x, double* w);   // nodes and weights on [-1, 1]

// mixed precision factor (FP32 storage and MFMA, FP64 diagonal pivots)
void launch_to_f32(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b);
void launch_potrf32(hipStream_t st, const int32_t* flist, int nf, int k, FrontsDev F, Bufs b, int* err);
void launch_trsm32(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, int k, FrontsDev F, Bufs b);
void launch_syrk_inner32(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, int kk, FrontsDev F, Bufs b);
void launch_extend_add32(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b);
// r = b - Q x in FP64 (Q = Vecchia prior precision + star sites), for refinement
void launch_residual(hipStream_t st, int64_t N, const int64_t* rp, const int32_t* col, const double* val,
                     const double* d, StarsDev s, const double* b, const double* x, double* u, double* w, double* r);
void launch_add(hipStream_t st, int64_t n, double* x, const double* dx);
void launch_maxabs_diff(hipStream_t st, const double* a, const double* b, int64_t n, double* out);

// Map prediction (maps.hip).  S: (n-1)^3 cells x 36 packed Sigma entries of
// the cell's 8 corners.  T: per node, the trapezoid step count of the
// observer's sightline to it (0 for the observer's own node).
void launch_cell_sigma(hipStream_t st, GridDev g, FrontsDev F, const double* fronts, const int32_t* iperm,
                       const int32_t* snode, double* S, int* bad);
void launch_ext_mean(hipStream_t st, GridDev g, const int32_t* T, const double* mu, const double* S, double* mean,
                     int64_t N);
void launch_ext_sample(hipStream_t st, GridDev g, const int32_t* T, const double* f, const double* mean, double* s1,
                       double* s2, int64_t N);
void launch_ext_plugin(hipStream_t st, GridDev g, const int32_t* T, const double* f, double* centre, int64_t N);
void launch_sum2(hipStream_t st, const double* a, const double* b, double* out, int64_t n);
// out = (1 - r) (f - m) + r mu (m may be null); out may alias f
void launch_relin_step(hipStream_t st, const double* f, const double* m, const double* mu, double r, double* out,
                       int64_t n);
void launch_sample_var(hipStream_t st, const double* s1, const double* s2, double* var, int K, int64_t n);
void launch_density(hipStream_t st, const double* mu, const double* var, double* m, double* v, int64_t n);
void launch_point_pred(hipStream_t st, GridDev g, FrontsDev F, const double* fronts, const int32_t* iperm,
                       const int32_t* snode, const double* mu, const double* xyz2, double* out, int64_t np, int* bad);

}  // namespace ep
