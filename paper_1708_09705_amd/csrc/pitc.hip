// Kernels of the PITC / PIC block pass (the sub-catalogue EP of Sec. 4.1,
// App. B, and the PIC predictive of App. C): covariance fills from the
// per-offset table, front set-up, the site combination and the per-node
// predictive reductions.  The dense products run in k_gemm_tasks and the
// block Cholesky in k_potrf / k_trsm_step.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"
#include "pitc.h"

namespace ep {

namespace {

__device__ __forceinline__ int64_t find_job(const int64_t* base, int n, int64_t t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Covariance of two nodes from the table over absolute offsets (0..w)^3
__device__ __forceinline__ double kcov(const PitcCovDev& c, int32_t a, int32_t b) {
    const int n = c.n;
    const int ai = a % n, aj = (a / n) % n, ak = a / (n * n);
    const int bi = b % n, bj = (b / n) % n, bk = b / (n * n);
    const int di = abs(ai - bi), dj = abs(aj - bj), dk = abs(ak - bk);
    if (di > c.w || dj > c.w || dk > c.w) return 0.0;
    return c.table[(di * (c.w + 1) + dj) * (c.w + 1) + dk];
}

// One 64 x 64 tile of a covariance fill per block (256 threads, 16 entries
// each); entries outside the job's rows / columns are zero, and so are the
// strictly upper tiles of a lower-only job.
__global__ __launch_bounds__(256) void k_kfill(const PitcKJob* __restrict__ jobs, const int64_t* __restrict__ base,
                                               int njobs, int64_t ntiles, PitcCovDev cov,
                                               const int32_t* __restrict__ ids, double* __restrict__ ws) {
    const int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int j = (int)find_job(base, njobs, t);
    const PitcKJob J = jobs[j];
    const int64_t local = t - base[j];
    const int tr = (int)(local % (J.rpad / TS)), tc = (int)(local / (J.rpad / TS));
    const int r = TS * tr + (threadIdx.x & 63);
    const int32_t* rows = ids + J.rows;
    const int32_t* cols = ids + J.cols;
    const bool zero_tile = J.lower && tr < tc;
#pragma unroll 4
    for (int q = 0; q < 16; q++) {
        const int c = TS * tc + (threadIdx.x >> 6) + 4 * q;
        double v = 0.0;
        if (!zero_tile && r < J.nrows && c < J.ncols) v = kcov(cov, rows[r], cols[c]);
        ws[J.out + r + (int64_t)c * J.ld] = v;
    }
}

// Per block: sigma^2 onto the diagonal of B, 1 on its padding diagonal;
// with mean parameters the H tile (rows 0..4: h_n = J^T g_n); the residual
// tile (row 0: a~_n minus its prior mean, c_n + m0 sum_i g_ni, or c'_n +
// h_n . phihat with mean parameters; rows 1..63: 0).
__global__ __launch_bounds__(256) void k_block_prep(const PitcBlockDev* __restrict__ blk, const int32_t* __restrict__ stars,
                                                    const int64_t* __restrict__ sptr,
                                                    const double* __restrict__ g, const double* __restrict__ c,
                                                    const double* __restrict__ A, const double* __restrict__ sigma,
                                                    PitcMeanDev mean, double* __restrict__ ws) {
    const PitcBlockDev B = blk[blockIdx.x];
    double* F = ws + B.front;
    const int64_t m = B.m;
    double* rt = F + B.rrow;                            // residual tile
    double* ht = B.xdim > B.rpad ? F + B.npad + B.rpad : nullptr;   // H tile
    for (int n = threadIdx.x; n < B.npad; n += blockDim.x) {
        double* d = F + n + (int64_t)n * m;
        if (n < B.nstars) {
            const int32_t s = stars[B.star0 + n];
            double sg = 0.0;
            if (mean.mhat) {
                for (int j = 0; j < NTHETA; j++) sg += mean.h[(int64_t)NTHETA * s + j] * mean.phihat[j];
            } else {
                for (int64_t q = sptr[s]; q < sptr[s + 1]; q++) sg += g[q];
                sg *= mean.m0;
            }
            *d += sigma[s] * sigma[s];
            rt[(int64_t)n * m] = A[s] - c[s] - sg;
            if (ht)
                for (int r = 0; r < TS; r++) ht[r + (int64_t)n * m] = r < NTHETA ? mean.h[(int64_t)NTHETA * s + r] : 0.0;
        } else {
            *d = 1.0;
            rt[(int64_t)n * m] = 0.0;
            if (ht)
                for (int r = 0; r < TS; r++) ht[r + (int64_t)n * m] = 0.0;
        }
        for (int r = 1; r < TS; r++) rt[r + (int64_t)n * m] = 0.0;
    }
}

// The front of p(u)'s covariance C = K_uu: identity in the right-hand-side
// rows [rpad, 2 rpad), 1 on the padding diagonal of the C part.
__global__ void k_cfront_prep(double* __restrict__ F, int64_t m, int R, int rpad) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)rpad * rpad;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % rpad), j = (int)(e / rpad);
        F[rpad + i + (int64_t)j * m] = (i == j) ? 1.0 : 0.0;
        if (i == j && i >= R) F[i + (int64_t)i * m] = 1.0;
    }
}

// S_new = sum over blocks of the per-block products, in block order
__global__ void k_sum_blocks(const double* __restrict__ lam, int nblk, int64_t E, double* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < nblk; k++) s += lam[(int64_t)k * E + e];
        out[e] = s;
    }
}

// Sites (damped) and the two fronts over x (xdim): Fq = [P0 + S_sites; I;
// h_sites^T], Fe = [P0 + S_new; h_new^T] (lower triangles; upper tiles
// zero), P0 the prior precision of x.  S_* are E1 x E1 with E1 = xdim + 64:
// the x block, then the residual row xdim.
__global__ void k_sites_fronts(const double* __restrict__ Snew, double* __restrict__ Ssites, double damp, int first,
                               double* __restrict__ Fq, int64_t mq, double* __restrict__ Fe, int64_t me, int rpad,
                               int xdim, PitcPriorDev prior) {
    const int64_t e1 = xdim + TS;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < e1 * e1; e += (int64_t)gridDim.x * blockDim.x) {
        const double s = first ? damp * Snew[e] : (1.0 - damp) * Ssites[e] + damp * Snew[e];
        Ssites[e] = s;
        const int i = (int)(e % e1), j = (int)(e / e1);
        if (j >= xdim) continue;
        if (i < xdim) {
            double d = 0.0;
            if (i == j) d = (i >= rpad && i < rpad + prior.M) ? prior.s0inv[i - rpad] : 1.0;
            Fq[i + (int64_t)j * mq] = i >= j ? d + s : 0.0;
            Fe[i + (int64_t)j * me] = i >= j ? d + Snew[e] : 0.0;
            Fq[xdim + i + (int64_t)j * mq] = (i == j) ? 1.0 : 0.0;
        } else {
            Fq[2 * xdim + (i - xdim) + (int64_t)j * mq] = (i == xdim) ? s : 0.0;
            Fe[xdim + (i - xdim) + (int64_t)j * me] = (i == xdim) ? Snew[e] : 0.0;
        }
    }
}

// ln p(a~) = -1/2 [S ln 2 pi + sum_k ln|B_k| + sum_k r_k^T B_k^{-1} r_k
//            + ln|S0| + ln|P0 + S_new| - |L_e^{-1} h_new|^2]; one block of 256
__global__ __launch_bounds__(256) void k_lnz(const PitcBlockDev* __restrict__ blk, int nblk, const double* __restrict__ ws,
                                             const double* __restrict__ Fe, int64_t me, int xdim,
                                             const double* __restrict__ Snew, int64_t S, double ln_det_s0,
                                             double* __restrict__ out) {
    __shared__ double part[256];
    double s = 0.0;
    for (int k = 0; k < nblk; k++) {
        const PitcBlockDev B = blk[k];
        const double* F = ws + B.front;
        for (int n = threadIdx.x; n < B.nstars; n += blockDim.x) s += 2.0 * log(F[n + (int64_t)n * B.m]);
    }
    for (int i = threadIdx.x; i < xdim; i += blockDim.x) {
        s += 2.0 * log(Fe[i + (int64_t)i * me]);
        const double v = Fe[xdim + (int64_t)i * me];
        s -= v * v;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t e1 = xdim + TS;
        const double rr = Snew[xdim + (int64_t)xdim * e1];
        out[0] = -0.5 * ((double)S * 1.8378770664093453 + part[0] + rr + ln_det_s0);
    }
}

// PIC predictive at the nodes of each block, one thread per node:
//   mean = m(x_p) + a^T mu~ + e^T w_r
//   var  = k0 - |k~|^2 - |e|^2 + a^T Sigma~ a
// with k~ = L_C^{-1} K(u, p) (the first rpad entries of Kt's row; with mean
// parameters its next entries are J_p), e = L_B^{-1} d (row of the front's
// D part), a = Kt row - W_x^T e (row of At), Sigma~ a (row of SAt); x-space
// vectors have xdim entries.
__global__ __launch_bounds__(256) void k_predict(const PitcBlockDev* __restrict__ blk, const int64_t* __restrict__ base,
                                                 int nblk, int64_t ntasks, const double* __restrict__ ws,
                                                 const int32_t* __restrict__ pnodes, const double* __restrict__ mu_t,
                                                 PitcMeanDev mean, double k0, double* __restrict__ out_mean,
                                                 double* __restrict__ out_var) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ntasks) return;
    const int k = (int)find_job(base, nblk, t);
    const PitcBlockDev B = blk[k];
    const int p = (int)(t - base[k]);
    if (p >= B.npred) return;
    const double* F = ws + B.front;
    const double* Erow = F + B.drow + p;   // e_n at Erow[n m]
    const double* wr = F + B.rrow;         // w_r,n at wr[n m]
    const int64_t ldp = B.ppad;
    const double* kt = ws + B.kt + p;
    const double* at = ws + B.at + p;
    const double* sat = ws + B.sat + p;
    const int32_t node = pnodes[B.pred0 + p];
    double mn = mean.mhat ? mean.mhat[node] : mean.m0, v = k0;
    for (int n = 0; n < B.nstars; n++) {
        const double e = Erow[(int64_t)n * B.m];
        mn += e * wr[(int64_t)n * B.m];
        v -= e * e;
    }
    for (int r = 0; r < B.xdim; r++) {
        const double a = at[r * ldp];
        mn += a * mu_t[r];
        v += a * sat[r * ldp];
        if (r < B.rpad) {
            const double kk = kt[r * ldp];
            v -= kk * kk;
        }
    }
    out_mean[node] = mn;
    out_var[node] = v;
}

// Kt columns rpad .. rpad + 4: J at the block's prediction nodes
__global__ void k_kt_j(const PitcBlockDev* __restrict__ blk, const int64_t* __restrict__ base, int nblk, int64_t ntasks,
                       const int32_t* __restrict__ pnodes, PitcMeanDev mean, double* __restrict__ ws) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ntasks) return;
    const int k = (int)find_job(base, nblk, t);
    const PitcBlockDev B = blk[k];
    const int p = (int)(t - base[k]);
    if (p >= B.npred) return;
    const int32_t node = pnodes[B.pred0 + p];
    double* kt = ws + B.kt + p;
    for (int j = 0; j < NTHETA; j++) kt[(int64_t)(B.rpad + j) * B.ppad] = mean.J[node + (int64_t)j * mean.N];
}

// T = [L_C | J_u] (rpad x xdim, ld rpad): the C front's lower triangle (its
// strictly upper tiles are zero and its diagonal tiles zero above the
// diagonal), then J at the inducing nodes
__global__ void k_build_t(const double* __restrict__ Cf, int64_t mC, const int32_t* __restrict__ unodes, int R, int rpad,
                          int xdim, PitcMeanDev mean, double* __restrict__ T) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)rpad * xdim;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % rpad), j = (int)(e / rpad);
        double v = 0.0;
        if (j < rpad) v = Cf[i + (int64_t)j * mC];
        else if (j - rpad < NTHETA && i < R) v = mean.J[unodes[i] + (int64_t)(j - rpad) * mean.N];
        T[e] = v;
    }
}

__global__ void k_add_mean(double* out, const int32_t* __restrict__ unodes, int R, PitcMeanDev mean) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += gridDim.x * blockDim.x)
        out[r] += mean.mhat ? mean.mhat[unodes[r]] : mean.m0;
}

__global__ void k_theta_out(const double* __restrict__ mu_t, const double* __restrict__ sig_t, int xdim, int rpad, int M,
                            Phi5 phihat, double* __restrict__ out) {
    const int t = threadIdx.x;
    if (t < M) out[t] = phihat.v[t] + mu_t[rpad + t];
    if (t < M * M) out[M + t] = sig_t[(rpad + t / M) + (int64_t)(rpad + t % M) * xdim];
}

unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}


// ---- the extinction likelihood: star sites under the PITC prior ----------
// The prior mean of a_n, c_n + m0 sum_q g_nq.
__device__ __forceinline__ double ext_prior_mean(const int64_t* sptr, const double* g, const double* c, double m0,
                                                 int32_t s) {
    double sg = 0.0;
    for (int64_t q = sptr[s]; q < sptr[s + 1]; q++) sg += g[q];
    return c[s] + m0 * sg;
}

// Before the scaling (one block of threads per sub-catalogue, a thread per
// front column i): the extra rows get column i of (S C)^T, i.e. row j holds
// s_i C_ij, with C read from the lower tiles of the unscaled B region; diag
// C, the unscaled Z^T (transposed into zm: element (n, r) at n + r npad) and
// s into tv.
__global__ __launch_bounds__(256) void k_ext_copy(const PitcBlockDev* __restrict__ blk,
                                                  const int32_t* __restrict__ stars,
                                                  const double* __restrict__ tau, double* __restrict__ ws) {
    const PitcBlockDev B = blk[blockIdx.x];
    double* F = ws + B.front;
    const int64_t m = B.m;
    for (int i = threadIdx.x; i < B.npad; i += blockDim.x) {
        const bool real = i < B.nstars;
        const double si = real ? sqrt(tau[stars[B.star0 + i]]) : 0.0;
        for (int j = 0; j < B.npad; j++) {
            const double cij = j >= i ? F[j + (int64_t)i * m] : F[i + (int64_t)j * m];
            F[B.crow + j + (int64_t)i * m] = (real && j < B.nstars) ? si * cij : 0.0;
        }
        ws[B.cd + i] = real ? F[i + (int64_t)i * m] : 0.0;
        ws[B.tv + i] = si;
        for (int r = 0; r < B.rpad; r++) ws[B.zm + i + (int64_t)r * B.npad] = F[B.npad + r + (int64_t)i * m];
    }
}

// The scaling, a thread per front column n: B <- I + S B S (the lower tiles
// and the padding diagonal), Z^T and D^T columns times s_n, the residual
// r~_n = (nu_n - tau_n mu_n) / s_n (0 where s_n = 0) in the residual row.
__global__ __launch_bounds__(256) void k_ext_scale(const PitcBlockDev* __restrict__ blk,
                                                   const int32_t* __restrict__ stars, const int64_t* __restrict__ sptr,
                                                   const double* __restrict__ g, const double* __restrict__ c,
                                                   const double* __restrict__ tau, const double* __restrict__ nu,
                                                   double m0, double* __restrict__ ws) {
    const PitcBlockDev B = blk[blockIdx.x];
    double* F = ws + B.front;
    const int64_t m = B.m;
    const double* sv = ws + B.tv;
    double* rt = F + B.rrow;
    for (int n = threadIdx.x; n < B.npad; n += blockDim.x) {
        const double sn = sv[n];
        double* col = F + (int64_t)n * m;
        for (int i = 0; i < B.npad; i++) col[i] = (i == n ? 1.0 : 0.0) + sv[i] * sn * col[i];
        for (int r = 0; r < B.rpad; r++) col[B.npad + r] *= sn;
        for (int p = 0; p < B.ppad; p++) col[B.drow + p] *= sn;
        double res = 0.0;
        if (n < B.nstars && sn > 0.0) {
            const int32_t s = stars[B.star0 + n];
            res = (nu[s] - tau[s] * ext_prior_mean(sptr, g, c, m0, s)) / sn;
        }
        rt[(int64_t)n * m] = res;
        for (int r = 1; r < TS; r++) rt[r + (int64_t)n * m] = 0.0;
    }
}

// tv <- w_r - W_Z mu~ (rows i of the factored front: w_r in the residual row,
// W_Z^T in the Z^T rows), a thread per row.
__global__ __launch_bounds__(256) void k_ext_tvec(const PitcBlockDev* __restrict__ blk, const double* __restrict__ mu_t,
                                                  double* __restrict__ ws) {
    const PitcBlockDev B = blk[blockIdx.x];
    const double* F = ws + B.front;
    const int64_t m = B.m;
    for (int i = threadIdx.x; i < B.npad; i += blockDim.x) {
        const double* col = F + (int64_t)i * m;
        double t = col[B.rrow];
        for (int r = 0; r < B.rpad; r++) t -= col[B.npad + r] * mu_t[r];
        ws[B.tv + i] = t;
    }
}

// E[a_n] = mu_n + Z_n . mu~ + sum_i P_in t_i, a thread per star (P_in at
// row crow + n of column i).
__global__ __launch_bounds__(256) void k_ext_mean(const PitcBlockDev* __restrict__ blk,
                                                  const int32_t* __restrict__ stars, const int64_t* __restrict__ sptr,
                                                  const double* __restrict__ g, const double* __restrict__ c, double m0,
                                                  const double* __restrict__ mu_t, const double* __restrict__ ws,
                                                  double* __restrict__ qmean) {
    const PitcBlockDev B = blk[blockIdx.x];
    const double* F = ws + B.front;
    const int64_t m = B.m;
    for (int n = threadIdx.x; n < B.nstars; n += blockDim.x) {
        const int32_t s = stars[B.star0 + n];
        double v = ext_prior_mean(sptr, g, c, m0, s);
        for (int r = 0; r < B.rpad; r++) v += ws[B.zm + n + (int64_t)r * B.npad] * mu_t[r];
        for (int i = 0; i < B.npad; i++) v += F[B.crow + n + (int64_t)i * m] * ws[B.tv + i];
        qmean[s] = v;
    }
}

// Var[a_n] = C_nn - |P_.n|^2 + (M Sigma~)_n . M_n with M = Z - P^T W_Z in zm
// and M Sigma~ in tm, a thread per star.
__global__ __launch_bounds__(256) void k_ext_var(const PitcBlockDev* __restrict__ blk, const int32_t* __restrict__ stars,
                                                 const double* __restrict__ ws, double* __restrict__ qvar) {
    const PitcBlockDev B = blk[blockIdx.x];
    const double* F = ws + B.front;
    const int64_t m = B.m;
    for (int n = threadIdx.x; n < B.nstars; n += blockDim.x) {
        double v = ws[B.cd + n];
        for (int i = 0; i < B.npad; i++) {
            const double p = F[B.crow + n + (int64_t)i * m];
            v -= p * p;
        }
        for (int r = 0; r < B.rpad; r++)
            v += ws[B.tm + n + (int64_t)r * B.npad] * ws[B.zm + n + (int64_t)r * B.npad];
        qvar[stars[B.star0 + n]] = v;
    }
}

}  // namespace

void launch_pitc_kfill(hipStream_t st, const PitcKJob* jobs, const int64_t* base, int njobs, int64_t ntiles,
                       PitcCovDev cov, const int32_t* ids, double* ws) {
    if (ntiles > 0) hipLaunchKernelGGL(k_kfill, dim3((unsigned)ntiles), dim3(256), 0, st, jobs, base, njobs, ntiles, cov, ids, ws);
}
void launch_pitc_block_prep(hipStream_t st, const PitcBlockDev* blk, int nblk, const int32_t* stars, const int64_t* sptr,
                            const double* g, const double* c, const double* A, const double* sigma, PitcMeanDev mean,
                            double* ws) {
    if (nblk > 0)
        hipLaunchKernelGGL(k_block_prep, dim3(nblk), dim3(256), 0, st, blk, stars, sptr, g, c, A, sigma, mean, ws);
}
void launch_pitc_cfront_prep(hipStream_t st, double* F, int64_t m, int R, int rpad) {
    hipLaunchKernelGGL(k_cfront_prep, dim3(grid_for((int64_t)rpad * rpad)), dim3(256), 0, st, F, m, R, rpad);
}
void launch_pitc_sum_blocks(hipStream_t st, const double* lam, int nblk, int64_t E, double* out) {
    hipLaunchKernelGGL(k_sum_blocks, dim3(grid_for(E)), dim3(256), 0, st, lam, nblk, E, out);
}
void launch_pitc_sites_fronts(hipStream_t st, const double* Snew, double* Ssites, double damp, bool first, double* Fq,
                              int64_t mq, double* Fe, int64_t me, int rpad, int xdim, PitcPriorDev prior) {
    const int64_t e1 = xdim + TS;
    hipLaunchKernelGGL(k_sites_fronts, dim3(grid_for(e1 * e1)), dim3(256), 0, st, Snew, Ssites, damp, first ? 1 : 0, Fq,
                       mq, Fe, me, rpad, xdim, prior);
}
void launch_pitc_lnz(hipStream_t st, const PitcBlockDev* blk, int nblk, const double* ws, const double* Fe, int64_t me,
                     int xdim, const double* Snew, int64_t S, double ln_det_s0, double* out) {
    hipLaunchKernelGGL(k_lnz, dim3(1), dim3(256), 0, st, blk, nblk, ws, Fe, me, xdim, Snew, S, ln_det_s0, out);
}
void launch_pitc_predict(hipStream_t st, const PitcBlockDev* blk, const int64_t* base, int nblk, int64_t ntasks,
                         const double* ws, const int32_t* pnodes, const double* mu_t, PitcMeanDev mean, double k0,
                         double* out_mean, double* out_var) {
    if (ntasks > 0)
        hipLaunchKernelGGL(k_predict, dim3((unsigned)((ntasks + 255) / 256)), dim3(256), 0, st, blk, base, nblk, ntasks,
                           ws, pnodes, mu_t, mean, k0, out_mean, out_var);
}
void launch_pitc_kt_j(hipStream_t st, const PitcBlockDev* blk, const int64_t* base, int nblk, int64_t ntasks,
                      const int32_t* pnodes, PitcMeanDev mean, double* ws) {
    if (ntasks > 0)
        hipLaunchKernelGGL(k_kt_j, dim3((unsigned)((ntasks + 255) / 256)), dim3(256), 0, st, blk, base, nblk, ntasks,
                           pnodes, mean, ws);
}
void launch_pitc_build_t(hipStream_t st, const double* Cf, int64_t mC, const int32_t* unodes, int R, int rpad, int xdim,
                         PitcMeanDev mean, double* T) {
    hipLaunchKernelGGL(k_build_t, dim3(grid_for((int64_t)rpad * xdim)), dim3(256), 0, st, Cf, mC, unodes, R, rpad, xdim,
                       mean, T);
}
void launch_pitc_theta_out(hipStream_t st, const double* mu_t, const double* sig_t, int xdim, int rpad, int M,
                           Phi5 phihat, double* out) {
    hipLaunchKernelGGL(k_theta_out, dim3(1), dim3(64), 0, st, mu_t, sig_t, xdim, rpad, M, phihat, out);
}
void launch_pitc_add_mean(hipStream_t st, double* out, const int32_t* unodes, int R, PitcMeanDev mean) {
    if (R > 0) hipLaunchKernelGGL(k_add_mean, dim3(grid_for(R)), dim3(256), 0, st, out, unodes, R, mean);
}
void launch_pitc_ext_prep(hipStream_t st, const PitcBlockDev* blk, int nblk, const int32_t* stars, const int64_t* sptr,
                          const double* g, const double* c, const double* tau, const double* nu, double m0,
                          double* ws) {
    if (nblk <= 0) return;
    hipLaunchKernelGGL(k_ext_copy, dim3(nblk), dim3(256), 0, st, blk, stars, tau, ws);
    hipLaunchKernelGGL(k_ext_scale, dim3(nblk), dim3(256), 0, st, blk, stars, sptr, g, c, tau, nu, m0, ws);
}
void launch_pitc_ext_mean(hipStream_t st, const PitcBlockDev* blk, int nblk, const int32_t* stars, const int64_t* sptr,
                          const double* g, const double* c, double m0, const double* mu_t, double* ws, double* qmean) {
    if (nblk <= 0) return;
    hipLaunchKernelGGL(k_ext_tvec, dim3(nblk), dim3(256), 0, st, blk, mu_t, ws);
    hipLaunchKernelGGL(k_ext_mean, dim3(nblk), dim3(256), 0, st, blk, stars, sptr, g, c, m0, mu_t, ws, qmean);
}
void launch_pitc_ext_var(hipStream_t st, const PitcBlockDev* blk, int nblk, const int32_t* stars, const double* ws,
                         double* qvar) {
    if (nblk > 0) hipLaunchKernelGGL(k_ext_var, dim3(nblk), dim3(256), 0, st, blk, stars, ws, qvar);
}

}  // namespace ep
