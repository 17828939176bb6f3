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

// Per block: sigma^2 onto the diagonal of B, 1 on its padding diagonal, and
// the residual tile (row 0: a~_n - c_n - m0 sum_i g_ni; rows 1..63: 0).
__global__ __launch_bounds__(256) void k_block_prep(const PitcBlockDev* __restrict__ blk, const int32_t* __restrict__ stars,
                                                    const int64_t* __restrict__ sptr, const double* __restrict__ g,
                                                    const double* __restrict__ c, const double* __restrict__ A,
                                                    const double* __restrict__ sigma, double m0, double* __restrict__ ws) {
    const PitcBlockDev B = blk[blockIdx.x];
    double* F = ws + B.front;
    const int64_t m = B.m;
    double* rt = F + B.npad + B.rpad;   // residual tile, rows npad + rpad .. + 63
    for (int n = threadIdx.x; n < B.npad; n += blockDim.x) {
        double* d = F + n + (int64_t)n * m;
        if (n < B.nstars) {
            const int32_t s = stars[B.star0 + n];
            double sg = 0.0;
            for (int64_t q = sptr[s]; q < sptr[s + 1]; q++) sg += g[q];
            *d += sigma[s] * sigma[s];
            rt[(int64_t)n * m] = A[s] - c[s] - m0 * sg;
        } else {
            *d = 1.0;
            rt[(int64_t)n * m] = 0.0;
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

// Sites (damped) and the two R x R fronts: Fq = [I + S_sites; I; h_sites^T],
// Fe = [I + S_new; h_new^T] (lower triangles; upper tiles zero).
__global__ void k_sites_fronts(const double* __restrict__ Snew, double* __restrict__ Ssites, double damp, int first,
                               double* __restrict__ Fq, int64_t mq, double* __restrict__ Fe, int64_t me, int rpad) {
    const int64_t e1 = rpad + TS;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < e1 * e1; e += (int64_t)gridDim.x * blockDim.x) {
        const double s = first ? damp * Snew[e] : (1.0 - damp) * Ssites[e] + damp * Snew[e];
        Ssites[e] = s;
        const int i = (int)(e % e1), j = (int)(e / e1);
        if (j >= rpad) continue;
        if (i < rpad) {
            const double d = (i == j) ? 1.0 : 0.0;
            Fq[i + (int64_t)j * mq] = i >= j ? d + s : 0.0;
            Fe[i + (int64_t)j * me] = i >= j ? d + Snew[e] : 0.0;
            Fq[rpad + i + (int64_t)j * mq] = d;
        } else {
            Fq[2 * rpad + (i - rpad) + (int64_t)j * mq] = (i == rpad) ? s : 0.0;
            Fe[rpad + (i - rpad) + (int64_t)j * me] = (i == rpad) ? Snew[e] : 0.0;
        }
    }
}

// ln p(a~) = -1/2 [S ln 2 pi + sum_k ln|B_k| + sum_k r_k^T B_k^{-1} r_k
//            + ln|I + S_new| - |L_e^{-1} h_new|^2]; one block of 256
__global__ __launch_bounds__(256) void k_lnz(const PitcBlockDev* __restrict__ blk, int nblk, const double* __restrict__ ws,
                                             const double* __restrict__ Fe, int64_t me, int rpad,
                                             const double* __restrict__ Snew, int64_t S, double* __restrict__ out) {
    __shared__ double part[256];
    double s = 0.0;
    for (int k = 0; k < nblk; k++) {
        const PitcBlockDev B = blk[k];
        const double* F = ws + B.front;
        for (int n = threadIdx.x; n < B.nstars; n += blockDim.x) s += 2.0 * log(F[n + (int64_t)n * B.m]);
    }
    for (int i = threadIdx.x; i < rpad; i += blockDim.x) {
        s += 2.0 * log(Fe[i + (int64_t)i * me]);
        const double v = Fe[rpad + (int64_t)i * me];
        s -= v * v;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t e1 = rpad + TS;
        const double rr = Snew[rpad + (int64_t)rpad * e1];
        out[0] = -0.5 * ((double)S * 1.8378770664093453 + part[0] + rr);
    }
}

// PIC predictive at the nodes of each block, one thread per node:
//   mean = m0 + a^T mu~ + e^T w_r
//   var  = k0 - |k~|^2 - |e|^2 + a^T Sigma~ a
// with k~ = X_C K_u* (row of Kt), e = L_B^{-1} d (row of the front's D part),
// a = k~ - W_Z^T e (row of At), Sigma~ a (row of SAt).
__global__ __launch_bounds__(256) void k_predict(const PitcBlockDev* __restrict__ blk, const int64_t* __restrict__ base,
                                                 int nblk, int64_t ntasks, const double* __restrict__ ws,
                                                 const int32_t* __restrict__ pnodes, const double* __restrict__ mu_t,
                                                 double m0, double k0, int rpad, double* __restrict__ mean,
                                                 double* __restrict__ var) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ntasks) return;
    const int k = (int)find_job(base, nblk, t);
    const PitcBlockDev B = blk[k];
    const int p = (int)(t - base[k]);
    if (p >= B.npred) return;
    const double* F = ws + B.front;
    const double* Erow = F + B.npad + B.rpad + TS + p;   // e_n at Erow[n m]
    const double* wr = F + B.npad + B.rpad;             // w_r,n at wr[n m]
    const int64_t ldp = B.ppad;
    const double* kt = ws + B.kt + p;
    const double* at = ws + B.at + p;
    const double* sat = ws + B.sat + p;
    double mn = m0, v = k0;
    for (int n = 0; n < B.nstars; n++) {
        const double e = Erow[(int64_t)n * B.m];
        mn += e * wr[(int64_t)n * B.m];
        v -= e * e;
    }
    for (int r = 0; r < rpad; r++) {
        const double a = at[r * ldp], kk = kt[r * ldp];
        mn += a * mu_t[r];
        v += a * sat[r * ldp] - kk * kk;
    }
    const int32_t node = pnodes[B.pred0 + p];
    mean[node] = mn;
    var[node] = v;
}

__global__ void k_add_const(double* p, int64_t n, double c) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] += c;
}

unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

void launch_pitc_kfill(hipStream_t st, const PitcKJob* jobs, const int64_t* base, int njobs, int64_t ntiles,
                       PitcCovDev cov, const int32_t* ids, double* ws) {
    if (ntiles > 0) hipLaunchKernelGGL(k_kfill, dim3((unsigned)ntiles), dim3(256), 0, st, jobs, base, njobs, ntiles, cov, ids, ws);
}
void launch_pitc_block_prep(hipStream_t st, const PitcBlockDev* blk, int nblk, const int32_t* stars, const int64_t* sptr,
                            const double* g, const double* c, const double* A, const double* sigma, double m0,
                            double* ws) {
    if (nblk > 0)
        hipLaunchKernelGGL(k_block_prep, dim3(nblk), dim3(256), 0, st, blk, stars, sptr, g, c, A, sigma, m0, ws);
}
void launch_pitc_cfront_prep(hipStream_t st, double* F, int64_t m, int R, int rpad) {
    hipLaunchKernelGGL(k_cfront_prep, dim3(grid_for((int64_t)rpad * rpad)), dim3(256), 0, st, F, m, R, rpad);
}
void launch_pitc_sum_blocks(hipStream_t st, const double* lam, int nblk, int64_t E, double* out) {
    hipLaunchKernelGGL(k_sum_blocks, dim3(grid_for(E)), dim3(256), 0, st, lam, nblk, E, out);
}
void launch_pitc_sites_fronts(hipStream_t st, const double* Snew, double* Ssites, double damp, bool first, double* Fq,
                              int64_t mq, double* Fe, int64_t me, int rpad) {
    const int64_t e1 = rpad + TS;
    hipLaunchKernelGGL(k_sites_fronts, dim3(grid_for(e1 * e1)), dim3(256), 0, st, Snew, Ssites, damp, first ? 1 : 0, Fq,
                       mq, Fe, me, rpad);
}
void launch_pitc_lnz(hipStream_t st, const PitcBlockDev* blk, int nblk, const double* ws, const double* Fe, int64_t me,
                     int rpad, const double* Snew, int64_t S, double* out) {
    hipLaunchKernelGGL(k_lnz, dim3(1), dim3(256), 0, st, blk, nblk, ws, Fe, me, rpad, Snew, S, out);
}
void launch_pitc_predict(hipStream_t st, const PitcBlockDev* blk, const int64_t* base, int nblk, int64_t ntasks,
                         const double* ws, const int32_t* pnodes, const double* mu_t, double m0, double k0, int rpad,
                         double* mean, double* var) {
    if (ntasks > 0)
        hipLaunchKernelGGL(k_predict, dim3((unsigned)((ntasks + 255) / 256)), dim3(256), 0, st, blk, base, nblk, ntasks,
                           ws, pnodes, mu_t, m0, k0, rpad, mean, var);
}
void launch_pitc_add_const(hipStream_t st, double* p, int64_t n, double c) {
    if (n > 0) hipLaunchKernelGGL(k_add_const, dim3(grid_for(n)), dim3(256), 0, st, p, n, c);
}

}  // namespace ep
