// Triangular solves with the fronts for up to MR_MAX right-hand sides at
// once (the five border columns of the inferred mean parameters; batches of
// posterior draws for the extinction map).  The single-vector kernels read
// each tile of the factor once per vector; these read it once per batch and
// apply it to every vector, so the solve stays bound by one pass over the
// factor.  Vectors are column q of an N x nrhs block with leading
// dimension ld, in the new node order.
//   forward : z_V = X y_V ; y_R -= L21 z_V ; y_V = z_V
//   backward: t_V = y_V - L21^T x_R ; x_V = X^T t_V
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ep {

namespace {

constexpr int LDT = TS + 1;

__device__ __forceinline__ int64_t find_batch(const BatchEnt* be, int nbe, int64_t t) {
    int lo = 0, hi = nbe - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (be[mid].base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// v[q][l] = src[q ld + off + l] for l < lim (0 beyond), q < nrhs
__device__ __forceinline__ void load_vecs(double (*v)[TS], const double* src, int64_t ld, int64_t off, int lim,
                                          int nrhs) {
    for (int idx = threadIdx.x; idx < nrhs * TS; idx += blockDim.x) {
        const int q = idx / TS, l = idx % TS;
        v[q][l] = l < lim ? src[q * ld + off + l] : 0.0;
    }
}

// out[q][c] of one block: reduce the four row groups' partial sums
__device__ __forceinline__ void reduce_parts(double (*part)[MR_MAX][TS], const double* acc, int nrhs) {
    const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;
    for (int q = 0; q < nrhs; q++) part[cg][q][r] = acc[q];
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_fwd_xv_mr(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                                   FrontsDev F, Bufs bufs, const double* __restrict__ y,
                                                   double* __restrict__ tout, int nrhs, int64_t ld) {
    __shared__ double v[MR_MAX][TS];
    __shared__ double part[4][MR_MAX][TS];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)find_batch(be, nbe, t);
    const int f = be[e].front;
    const int i = (int)(t - be[e].base);
    const int nv = F.nv[f], ldx = F.nvpad[f];
    const int64_t first = F.first[f];
    const double* Xb = bufs.X + F.xoff[f];
    const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;
    double acc[MR_MAX] = {};
    for (int k = 0; k <= i; k++) {
        __syncthreads();
        load_vecs(v, y, ld, first + TS * k, nv - TS * k, nrhs);
        __syncthreads();
        const double* T = Xb + (int64_t)TS * i + (int64_t)TS * k * ldx;
#pragma unroll
        for (int c = 0; c < 16; c++) {
            const double tv = T[r + (int64_t)(cg * 16 + c) * ldx];
#pragma unroll
            for (int q = 0; q < MR_MAX; q++)
                if (q < nrhs) acc[q] += tv * v[q][cg * 16 + c];
        }
    }
    reduce_parts(part, acc, nrhs);
    for (int idx = threadIdx.x; idx < nrhs * TS; idx += blockDim.x) {
        const int q = idx / TS, l = idx % TS;
        const double s = part[0][q][l] + part[1][q][l] + part[2][q][l] + part[3][q][l];
        if (TS * i + l < nv) tout[q * ld + first + TS * i + l] = s;
    }
}

template <typename LT>
__global__ __launch_bounds__(256) void k_fwd_r_mr(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                                  FrontsDev F, const LT* __restrict__ Lbuf,
                                                  const double* __restrict__ z, double* __restrict__ y, int nrhs,
                                                  int64_t ld) {
    __shared__ double v[MR_MAX][TS];
    __shared__ double part[4][MR_MAX][TS];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)find_batch(be, nbe, t);
    const int f = be[e].front;
    const int i = (int)(t - be[e].base);
    const int nv = F.nv[f], nvp = F.nvpad[f], m = F.m[f], nr = F.nr[f];
    const int64_t first = F.first[f];
    const LT* base = Lbuf + F.off[f];
    const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;
    double acc[MR_MAX] = {};
    const int P = nvp / TS;
    for (int k = 0; k < P; k++) {
        __syncthreads();
        load_vecs(v, z, ld, first + TS * k, nv - TS * k, nrhs);
        __syncthreads();
        const LT* T = base + nvp + (int64_t)TS * i + (int64_t)TS * k * m;
#pragma unroll
        for (int c = 0; c < 16; c++) {
            const double tv = (double)T[r + (int64_t)(cg * 16 + c) * m];
#pragma unroll
            for (int q = 0; q < MR_MAX; q++)
                if (q < nrhs) acc[q] += tv * v[q][cg * 16 + c];
        }
    }
    reduce_parts(part, acc, nrhs);
    for (int idx = threadIdx.x; idx < nrhs * TS; idx += blockDim.x) {
        const int q = idx / TS, l = idx % TS;
        const double s = part[0][q][l] + part[1][q][l] + part[2][q][l] + part[3][q][l];
        const int a = TS * i + l;
        if (a < nr) atomicAdd(y + q * ld + F.rrows[F.rptr[f] + a], -s);
    }
}

__global__ void k_copy_v_mr(const int32_t* __restrict__ flist, FrontsDev F, const double* __restrict__ src,
                            double* __restrict__ dst, int nrhs, int64_t ld) {
    const int f = flist[blockIdx.x];
    const int64_t first = F.first[f];
    const int nv = F.nv[f];
    for (int q = 0; q < nrhs; q++)
        for (int l = threadIdx.x; l < nv; l += blockDim.x) dst[q * ld + first + l] = src[q * ld + first + l];
}

// the 64 x 64 tile T (leading dimension ld) to LDS, transposed access later
template <typename LT>
__device__ __forceinline__ void tile_to_lds(double* sT, const LT* T, int64_t ld) {
    const int tid = threadIdx.x;
    __syncthreads();
    const int r = tid & 63;
#pragma unroll
    for (int q = 0; q < 16; q++) {
        const int c = (tid >> 6) + 4 * q;
        sT[c * LDT + r] = (double)T[r + (int64_t)c * ld];
    }
}

// acc[q] += sum_r T[r][c] v[q][r], c = lane, rows of group rg
__device__ __forceinline__ void tgemv_mr(const double* sT, const double (*v)[TS], double* acc, int nrhs) {
    const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const double tv = sT[c * LDT + rg * 16 + k];
#pragma unroll
        for (int q = 0; q < MR_MAX; q++)
            if (q < nrhs) acc[q] += tv * v[q][rg * 16 + k];
    }
}

template <typename LT>
__global__ __launch_bounds__(256) void k_bwd_t_mr(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                                  FrontsDev F, const LT* __restrict__ Lbuf,
                                                  const double* __restrict__ y, const double* __restrict__ x,
                                                  double* __restrict__ tout, int nrhs, int64_t ld) {
    __shared__ double sT[TS * LDT];
    __shared__ double v[MR_MAX][TS];
    __shared__ double part[4][MR_MAX][TS];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)find_batch(be, nbe, t);
    const int f = be[e].front;
    const int k = (int)(t - be[e].base);
    const int nv = F.nv[f], nvp = F.nvpad[f], m = F.m[f], nr = F.nr[f];
    const int64_t first = F.first[f];
    const LT* base = Lbuf + F.off[f];
    const int32_t* rows = F.rrows + F.rptr[f];
    const int MR = (nr + TS - 1) / TS;
    double acc[MR_MAX] = {};
    for (int i = 0; i < MR; i++) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < nrhs * TS; idx += blockDim.x) {
            const int q = idx / TS, l = idx % TS, a = TS * i + l;
            v[q][l] = a < nr ? x[q * ld + rows[a]] : 0.0;
        }
        tile_to_lds(sT, base + nvp + (int64_t)TS * i + (int64_t)TS * k * m, m);
        __syncthreads();
        tgemv_mr(sT, v, acc, nrhs);
    }
    __syncthreads();
    reduce_parts(part, acc, nrhs);
    for (int idx = threadIdx.x; idx < nrhs * TS; idx += blockDim.x) {
        const int q = idx / TS, l = idx % TS, a = TS * k + l;
        const double s = part[0][q][l] + part[1][q][l] + part[2][q][l] + part[3][q][l];
        if (a < nv) tout[q * ld + first + a] = y[q * ld + first + a] - s;
    }
}

__global__ __launch_bounds__(256) void k_bwd_x_mr(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                                  FrontsDev F, Bufs bufs, const double* __restrict__ tin,
                                                  double* __restrict__ x, int nrhs, int64_t ld) {
    __shared__ double sT[TS * LDT];
    __shared__ double v[MR_MAX][TS];
    __shared__ double part[4][MR_MAX][TS];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)find_batch(be, nbe, t);
    const int f = be[e].front;
    const int k = (int)(t - be[e].base);
    const int nv = F.nv[f], nvp = F.nvpad[f];
    const int64_t first = F.first[f];
    const double* Xb = bufs.X + F.xoff[f];
    const int P = nvp / TS;
    double acc[MR_MAX] = {};
    for (int i = k; i < P; i++) {
        __syncthreads();
        load_vecs(v, tin, ld, first + TS * i, nv - TS * i, nrhs);
        tile_to_lds(sT, Xb + (int64_t)TS * i + (int64_t)TS * k * nvp, nvp);
        __syncthreads();
        tgemv_mr(sT, v, acc, nrhs);
    }
    __syncthreads();
    reduce_parts(part, acc, nrhs);
    for (int idx = threadIdx.x; idx < nrhs * TS; idx += blockDim.x) {
        const int q = idx / TS, l = idx % TS, a = TS * k + l;
        const double s = part[0][q][l] + part[1][q][l] + part[2][q][l] + part[3][q][l];
        if (a < nv) x[q * ld + first + a] = s;
    }
}

__global__ void k_gather_perm_mr(const int32_t* __restrict__ perm, const double* __restrict__ src, int64_t lds,
                                 double* __restrict__ dst, int64_t ldd, int nrhs, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = perm[i];
        for (int q = 0; q < nrhs; q++) dst[q * ldd + i] = src[q * lds + p];
    }
}

__global__ void k_scatter_perm_mr(const int32_t* __restrict__ perm, const double* __restrict__ src, int64_t lds,
                                  double* __restrict__ dst, int64_t ldd, int nrhs, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = perm[i];
        for (int q = 0; q < nrhs; q++) dst[q * ldd + p] = src[q * lds + i];
    }
}

unsigned grid_of(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

void launch_fwd_xv_mr(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                      const double* y, double* t, int nrhs, int64_t ld) {
    if (ntasks <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_fwd_xv_mr, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F, b, y, t, nrhs, ld);
}
void launch_fwd_r_mr(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                     const double* t, double* y, int nrhs, int64_t ld) {
    if (ntasks <= 0 || nrhs <= 0) return;
    if (b.F32)
        hipLaunchKernelGGL(k_fwd_r_mr<float>, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F,
                           (const float*)b.F32, t, y, nrhs, ld);
    else
        hipLaunchKernelGGL(k_fwd_r_mr<double>, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F,
                           (const double*)b.fronts, t, y, nrhs, ld);
}
void launch_copy_v_mr(hipStream_t st, const int32_t* flist, int nf, FrontsDev F, const double* t, double* y, int nrhs,
                      int64_t ld) {
    if (nf <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_copy_v_mr, dim3(nf), dim3(256), 0, st, flist, F, t, y, nrhs, ld);
}
void launch_bwd_t_mr(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                     const double* y, const double* x, double* t, int nrhs, int64_t ld) {
    if (ntasks <= 0 || nrhs <= 0) return;
    if (b.F32)
        hipLaunchKernelGGL(k_bwd_t_mr<float>, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F,
                           (const float*)b.F32, y, x, t, nrhs, ld);
    else
        hipLaunchKernelGGL(k_bwd_t_mr<double>, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F,
                           (const double*)b.fronts, y, x, t, nrhs, ld);
}
void launch_bwd_x_mr(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                     const double* t, double* x, int nrhs, int64_t ld) {
    if (ntasks <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_bwd_x_mr, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F, b, t, x, nrhs, ld);
}
void launch_gather_perm_mr(hipStream_t st, const int32_t* perm, const double* src, int64_t lds, double* dst,
                           int64_t ldd, int nrhs, int64_t n) {
    if (n > 0 && nrhs > 0)
        hipLaunchKernelGGL(k_gather_perm_mr, dim3(grid_of(n)), dim3(256), 0, st, perm, src, lds, dst, ldd, nrhs, n);
}
void launch_scatter_perm_mr(hipStream_t st, const int32_t* perm, const double* src, int64_t lds, double* dst,
                            int64_t ldd, int nrhs, int64_t n) {
    if (n > 0 && nrhs > 0)
        hipLaunchKernelGGL(k_scatter_perm_mr, dim3(grid_of(n)), dim3(256), 0, st, perm, src, lds, dst, ldd, nrhs, n);
}

}  // namespace ep
