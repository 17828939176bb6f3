// Map prediction from the EP posterior q(f) = N(mu, Sigma) (Sec. 5: maps of
// extinction and of the pseudo-density rho kappa = e^f).
//
// * Density at the nodes: rho kappa = e^f is lognormal under q.
// * Extinction to every node x: A(x) is the line-of-sight integral of e^F
//   from the observer to x with the forward model of the sightlines
//   (trapezoid, trilinear F).  Its posterior mean is exact: each sample point
//   s contributes w e^{m(s) + v(s)/2}, m = phi . mu and v = phi^T Sigma_c phi
//   with Sigma_c the 8 x 8 block of the point's cell, which lies on the
//   factor's pattern.  Its variance needs Sigma between distant cells, which
//   the selected inversion does not hold, so it is estimated from posterior
//   draws f = mu + L^{-T} z.
// * Two points x, x' (e.g. 10 pc apart): the joint lognormal moments of
//   (rho kappa(x), rho kappa(x')) from the Sigma entries among their cells'
//   corners.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace ep {

namespace {

__device__ __forceinline__ double wave_sum_m(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sigma(p, q) for grid nodes p, q after the selected inversion, read from
// the front of whichever is eliminated first; NaN when the pair is not on
// the factor's pattern.
__device__ double sigma_pair(const FrontsDev& F, const double* fronts, const int32_t* iperm,
                             const int32_t* snode, int p, int q) {
    int a = iperm[p], b = iperm[q];
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
    const int f = snode[a];
    const int64_t first = F.first[f];
    const int la = (int)(a - first);
    int lb;
    if (b < first + F.nv[f]) {
        lb = (int)(b - first);
    } else {
        const int32_t* r = F.rrows + F.rptr[f];
        int lo = 0, hi = F.nr[f] - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (r[mid] < b) lo = mid + 1; else hi = mid;
        }
        if (F.nr[f] == 0 || r[lo] != b) return __builtin_nan("");
        lb = F.nvpad[f] + lo;
    }
    return fronts[F.off[f] + lb + (int64_t)la * F.m[f]];
}

// corner c8 of cell (ci, cj, ck): bit 0 -> +i, bit 1 -> +j, bit 2 -> +k
__device__ __forceinline__ int corner(int n, int ci, int cj, int ck, int c8) {
    return (ci + (c8 & 1)) + n * ((cj + ((c8 >> 1) & 1)) + n * (ck + ((c8 >> 2) & 1)));
}

// packed index of (a, b), a <= b, in an 8 x 8 symmetric block
__device__ __forceinline__ int pk(int a, int b) { return a * 8 - a * (a - 1) / 2 + (b - a); }

// cell and trilinear weights of a point (the forward model's rule:
// cell = clamp(floor(s/h), 0, n-2) per axis)
__device__ __forceinline__ void locate(const GridDev& g, const double p[3], int cc[3], double phi[8]) {
    double wv[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double c = floor(p[a] / g.h);
        c = c < 0 ? 0 : (c > g.n - 2 ? g.n - 2 : c);
        cc[a] = (int)c;
        wv[a] = p[a] / g.h - c;
    }
#pragma unroll
    for (int c8 = 0; c8 < 8; c8++) {
        const int bi = c8 & 1, bj = (c8 >> 1) & 1, bk = (c8 >> 2) & 1;
        phi[c8] = (bi ? wv[0] : 1.0 - wv[0]) * (bj ? wv[1] : 1.0 - wv[1]) * (bk ? wv[2] : 1.0 - wv[2]);
    }
}

__global__ void k_cell_sigma(GridDev g, FrontsDev F, const double* __restrict__ fronts, const int32_t* iperm,
                             const int32_t* snode, double* S, int* bad) {
    const int nc = g.n - 1;
    const int64_t ncell = (int64_t)nc * nc * nc;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(c % nc), cj = (int)((c / nc) % nc), ck = (int)(c / ((int64_t)nc * nc));
        int nd[8];
#pragma unroll
        for (int a = 0; a < 8; a++) nd[a] = corner(g.n, ci, cj, ck, a);
        for (int a = 0; a < 8; a++)
            for (int b = a; b < 8; b++) {
                const double v = sigma_pair(F, fronts, iperm, snode, nd[a], nd[b]);
                if (!isfinite(v)) atomicExch(bad, 1);
                S[c * 36 + pk(a, b)] = v;
            }
    }
}

// One wave per target node.  MODE 0: the exact posterior mean of A(node)
// (f = mu, S the cells' Sigma blocks).  MODE 1: A(node) for one posterior
// draw f, accumulated as its deviation from a centre: s1 += A - centre,
// s2 += (A - centre)^2 (the centre in mean).  MODE 2: A(node) at f, written
// to mean (the centre).
template <int MODE>
__global__ __launch_bounds__(256) void k_ext(GridDev g, const int32_t* __restrict__ T, const double* __restrict__ f,
                                             const double* __restrict__ S, double* mean, double* s1, double* s2,
                                             int64_t N) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + w;
    if (p >= N) return;
    const int n = g.n;
    const double x = (double)(p % n) * g.h, y = (double)((p / n) % n) * g.h, z = (double)(p / ((int64_t)n * n)) * g.h;
    const double dx = x - g.ox, dy = y - g.oy, dz = z - g.oz;
    const int Tn = T[p];
    double acc = 0.0;
    if (Tn > 0) {
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        const double delta = d / (double)Tn;
        for (int t = lane; t <= Tn; t += 64) {
            const double fr = (double)t / (double)Tn;
            const double pt[3] = {g.ox + fr * dx, g.oy + fr * dy, g.oz + fr * dz};
            int cc[3];
            double phi[8];
            locate(g, pt, cc, phi);
            const double wt = (t == 0 || t == Tn) ? 0.5 * delta : delta;
            double F = 0.0;
#pragma unroll
            for (int a = 0; a < 8; a++) F += phi[a] * f[corner(n, cc[0], cc[1], cc[2], a)];
            if (MODE != 0) {
                acc += wt * exp(F);
            } else {
                const int64_t cell = cc[0] + (int64_t)(n - 1) * (cc[1] + (int64_t)(n - 1) * cc[2]);
                const double* Sc = S + cell * 36;
                double v = 0.0;
#pragma unroll
                for (int a = 0; a < 8; a++) {
                    v += phi[a] * phi[a] * Sc[pk(a, a)];
#pragma unroll
                    for (int b = a + 1; b < 8; b++) v += 2.0 * phi[a] * phi[b] * Sc[pk(a, b)];
                }
                acc += wt * exp(F + 0.5 * v);
            }
        }
    }
    acc = wave_sum_m(acc);
    if (lane != 0) return;
    if (MODE != 1) {
        mean[p] = acc;
    } else {
        const double dlt = acc - mean[p];
        s1[p] += dlt;
        s2[p] += dlt * dlt;
    }
}

__global__ void k_axpy_add(const double* a, const double* b, double* out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] + b[i];
}

// out = (1 - r) (f - m) + r mu, m optional (null: 0)
__global__ void k_relin_step(const double* f, const double* m, const double* mu, double r, double* out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (1.0 - r) * (f[i] - (m ? m[i] : 0.0)) + r * mu[i];
}

__global__ void k_sample_var(const double* s1, const double* s2, double* var, int K, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        var[i] = (s2[i] - s1[i] * s1[i] / K) / (K - 1);
}

__global__ void k_density(const double* mu, const double* var, double* m, double* v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double e = exp(mu[i] + 0.5 * var[i]);
        m[i] = e;
        v[i] = expm1(var[i]) * e * e;
    }
}

// cell (clamp rule) and fractional coordinates of a point
__device__ __forceinline__ void cell_frac(const GridDev& g, const double* p, int cc[3], double wv[3]) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double c = floor(p[a] / g.h);
        c = c < 0 ? 0 : (c > g.n - 2 ? g.n - 2 : c);
        cc[a] = (int)c;
        wv[a] = p[a] / g.h - c;
    }
}

__device__ __forceinline__ double tri_weight(const double wv[3], int c8) {
    return ((c8 & 1) ? wv[0] : 1.0 - wv[0]) * (((c8 >> 1) & 1) ? wv[1] : 1.0 - wv[1]) *
           (((c8 >> 2) & 1) ? wv[2] : 1.0 - wv[2]);
}

// One wave per pair of points (x, x'): lane (a, b) = (lane / 8, lane % 8)
// takes the corner pair (a, b) of the three 8 x 8 blocks (x with x, x' with
// x', x with x'), and lanes 0-7 the means; wave sums give the Gaussian
// moments of (F(x), F(x')), then the lognormal moments of
// (e^F(x), e^F(x')): E, E', Var, Var', Cov.
__global__ __launch_bounds__(256) void k_point_pred(GridDev g, FrontsDev F, const double* __restrict__ fronts,
                                                    const int32_t* iperm, const int32_t* snode,
                                                    const double* __restrict__ mu, const double* __restrict__ xyz2,
                                                    double* out, int64_t np, int* bad) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + w;
    if (i >= np) return;
    int ca[3], cb[3];
    double wa[3], wb[3];
    cell_frac(g, xyz2 + 6 * i, ca, wa);
    cell_frac(g, xyz2 + 6 * i + 3, cb, wb);
    const int a = lane >> 3, b = lane & 7;
    const int na = corner(g.n, ca[0], ca[1], ca[2], a), nb = corner(g.n, cb[0], cb[1], cb[2], b);
    const int naa = corner(g.n, ca[0], ca[1], ca[2], b), nbb = corner(g.n, cb[0], cb[1], cb[2], a);
    const double pa = tri_weight(wa, a), pb = tri_weight(wb, b);
    double va = pa * tri_weight(wa, b) * sigma_pair(F, fronts, iperm, snode, na, naa);
    double vb = tri_weight(wb, a) * pb * sigma_pair(F, fronts, iperm, snode, nbb, nb);
    double cab = pa * pb * sigma_pair(F, fronts, iperm, snode, na, nb);
    double ma = 0.0, mb = 0.0;
    if (lane < 8) {
        ma = tri_weight(wa, lane) * mu[corner(g.n, ca[0], ca[1], ca[2], lane)];
        mb = tri_weight(wb, lane) * mu[corner(g.n, cb[0], cb[1], cb[2], lane)];
    }
    va = wave_sum_m(va);
    vb = wave_sum_m(vb);
    cab = wave_sum_m(cab);
    ma = wave_sum_m(ma);
    mb = wave_sum_m(mb);
    if (lane != 0) return;
    if (!isfinite(va) || !isfinite(vb) || !isfinite(cab)) atomicExch(bad, 1);
    const double ea = exp(ma + 0.5 * va), eb = exp(mb + 0.5 * vb);
    double* o = out + 5 * i;
    o[0] = ea;
    o[1] = eb;
    o[2] = expm1(va) * ea * ea;
    o[3] = expm1(vb) * eb * eb;
    o[4] = expm1(cab) * ea * eb;
}

unsigned grid_n(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

void launch_cell_sigma(hipStream_t st, GridDev g, FrontsDev F, const double* fronts, const int32_t* iperm,
                       const int32_t* snode, double* S, int* bad) {
    const int64_t nc = (int64_t)(g.n - 1) * (g.n - 1) * (g.n - 1);
    hipLaunchKernelGGL(k_cell_sigma, dim3(grid_n(nc)), dim3(256), 0, st, g, F, fronts, iperm, snode, S, bad);
}

void launch_ext_mean(hipStream_t st, GridDev g, const int32_t* T, const double* mu, const double* S, double* mean,
                     int64_t N) {
    if (N > 0)
        hipLaunchKernelGGL(k_ext<0>, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, st, g, T, mu, S, mean,
                           (double*)nullptr, (double*)nullptr, N);
}

void launch_ext_plugin(hipStream_t st, GridDev g, const int32_t* T, const double* f, double* centre, int64_t N) {
    if (N > 0)
        hipLaunchKernelGGL(k_ext<2>, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, st, g, T, f, (const double*)nullptr,
                           centre, (double*)nullptr, (double*)nullptr, N);
}

void launch_ext_sample(hipStream_t st, GridDev g, const int32_t* T, const double* f, const double* mean, double* s1,
                       double* s2, int64_t N) {
    if (N > 0)
        hipLaunchKernelGGL(k_ext<1>, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, st, g, T, f, (const double*)nullptr,
                           (double*)mean, s1, s2, N);
}

void launch_sum2(hipStream_t st, const double* a, const double* b, double* out, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_axpy_add, dim3(grid_n(n)), dim3(256), 0, st, a, b, out, n);
}

void launch_relin_step(hipStream_t st, const double* f, const double* m, const double* mu, double r, double* out,
                       int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_relin_step, dim3(grid_n(n)), dim3(256), 0, st, f, m, mu, r, out, n);
}

void launch_sample_var(hipStream_t st, const double* s1, const double* s2, double* var, int K, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_sample_var, dim3(grid_n(n)), dim3(256), 0, st, s1, s2, var, K, n);
}

void launch_density(hipStream_t st, const double* mu, const double* var, double* m, double* v, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_density, dim3(grid_n(n)), dim3(256), 0, st, mu, var, m, v, n);
}

void launch_point_pred(hipStream_t st, GridDev g, FrontsDev F, const double* fronts, const int32_t* iperm,
                       const int32_t* snode, const double* mu, const double* xyz2, double* out, int64_t np, int* bad) {
    if (np > 0)
        hipLaunchKernelGGL(k_point_pred, dim3((unsigned)((np + 3) / 4)), dim3(256), 0, st, g, F, fronts, iperm, snode,
                           mu, xyz2, out, np, bad);
}

}  // namespace ep
