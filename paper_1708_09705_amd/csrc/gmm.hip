// Unknown distances (Sec. 4.2, general case): each star's likelihood is a
// Gaussian mixture over components z in (l, b) = (ln s, log-extinction
// implied at distance s), and the distance is marginalised in the tilted
// distribution together with z.
//
// The site variable stays a_n = ln A to the star's catalogue position at
// distance s~.  The log-extinction at another distance is linearised in
// l = ln s about l~ = ln s~ with the current field: a(s) ~ a_n + beta_n (l - l~),
// beta_n = d ln A / d ln s = s~ e^{F(x_n)} / A_n.  A component then gives the
// likelihood N(a_n; m_b - beta (m_l - l~), C_bb - 2 beta C_lb + beta^2 C_ll)
// (the density of b - beta (l - l~) under (l, b) ~ N(m, C)), so the tilted
// distribution is a Gaussian mixture with closed-form normaliser and
// moments, one star per thread.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace ep {

namespace {

// beta_n = d_n exp(F(x_n) - ln A_n), F trilinear with the forward model's
// cell rule, at the field f the sightlines were linearised at
__global__ void k_beta(GridDev g, StarsDev s, const double* __restrict__ f, double* __restrict__ beta) {
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < s.n; n += (int64_t)gridDim.x * blockDim.x) {
        const double p[3] = {s.xyz[3 * n], s.xyz[3 * n + 1], s.xyz[3 * n + 2]};
        const double o[3] = {g.ox, g.oy, g.oz};
        int cc[3];
        double wv[3], d2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            double c = floor(p[a] / g.h);
            c = c < 0 ? 0 : (c > g.n - 2 ? g.n - 2 : c);
            cc[a] = (int)c;
            wv[a] = p[a] / g.h - c;
            d2 += (p[a] - o[a]) * (p[a] - o[a]);
        }
        double F = 0.0;
#pragma unroll
        for (int c8 = 0; c8 < 8; c8++) {
            const int bi = c8 & 1, bj = (c8 >> 1) & 1, bk = (c8 >> 2) & 1;
            const double phi = (bi ? wv[0] : 1.0 - wv[0]) * (bj ? wv[1] : 1.0 - wv[1]) * (bk ? wv[2] : 1.0 - wv[2]);
            F += phi * f[(cc[0] + bi) + (int64_t)g.n * ((cc[1] + bj) + (int64_t)g.n * (cc[2] + bk))];
        }
        beta[n] = sqrt(d2) * exp(F - s.lnA[n]);
    }
}

// Cavity, mixture tilted moments and the damped site update with the skip
// rules of the quadrature path, one star per thread.  comps: per star K rows
// of (w, m_l, m_b, C_ll, C_lb, C_bb).
__global__ void k_gmm_update(StarsDev s, EpParams P, const double* __restrict__ comps, int K,
                             const double* __restrict__ beta, const double* __restrict__ lref) {
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < s.n; n += (int64_t)gridDim.x * blockDim.x) {
        const double qm = s.cav_mu[n], qv = s.cav_var[n];
        const double tau = s.tau[n], nu = s.nu[n];
        double tau_c = 1.0 / qv - tau, nu_c = qm / qv - nu;
        if (!(tau_c > 0.0)) {
            s.status[n] = 1;
            s.dtau[n] = 0.0;
            continue;
        }
        double v_c = 1.0 / tau_c;
        if (v_c < P.vfloor) v_c = P.vfloor;
        const double mu_c = nu_c / tau_c;
        tau_c = 1.0 / v_c;
        nu_c = mu_c / v_c;
        const double b = beta[n], dl = lref[n];
        const double* cp = comps + (int64_t)n * K * 6;
        // pass 1: the largest log weight; pass 2: the normalised sums
        double top = -INFINITY;
        for (int z = 0; z < K; z++) {
            const double* c = cp + 6 * z;
            if (!(c[0] > 0.0)) continue;
            const double m = c[2] - b * (c[1] - dl), v = c[5] - 2.0 * b * c[4] + b * b * c[3], sv = v_c + v;
            const double lz = log(c[0]) - 0.5 * log(6.283185307179586 * sv) - 0.5 * (m - mu_c) * (m - mu_c) / sv;
            top = fmax(top, lz);
        }
        double Z = 0.0, s1 = 0.0;
        for (int z = 0; z < K; z++) {
            const double* c = cp + 6 * z;
            if (!(c[0] > 0.0)) continue;
            const double m = c[2] - b * (c[1] - dl), v = c[5] - 2.0 * b * c[4] + b * b * c[3], sv = v_c + v;
            const double r = exp(log(c[0]) - 0.5 * log(6.283185307179586 * sv) - 0.5 * (m - mu_c) * (m - mu_c) / sv - top);
            const double vz = v_c * v / sv, mz = vz * (mu_c / v_c + m / v);
            Z += r;
            s1 += r * mz;
        }
        const double mh = s1 / Z;
        double vh = 0.0;
        for (int z = 0; z < K; z++) {
            const double* c = cp + 6 * z;
            if (!(c[0] > 0.0)) continue;
            const double m = c[2] - b * (c[1] - dl), v = c[5] - 2.0 * b * c[4] + b * b * c[3], sv = v_c + v;
            const double r = exp(log(c[0]) - 0.5 * log(6.283185307179586 * sv) - 0.5 * (m - mu_c) * (m - mu_c) / sv - top);
            const double vz = v_c * v / sv, mz = vz * (mu_c / v_c + m / v);
            vh += r * (vz + (mz - mh) * (mz - mh));
        }
        vh /= Z;
        s.cav_mu[n] = mu_c;
        s.cav_var[n] = v_c;
        s.lnZ[n] = top + log(Z);
        s.tmean[n] = mh;
        s.tvar[n] = vh;
        const double tn = 1.0 / vh - tau_c, nn = mh / vh - nu_c;
        if (!(tn >= 0.0) || !isfinite(tn) || !isfinite(nn)) {
            s.status[n] = 2;
            s.dtau[n] = 0.0;
        } else {
            const double d = P.damping, t2 = (1.0 - d) * tau + d * tn;
            s.status[n] = 0;
            s.dtau[n] = fabs(t2 - tau);
            s.tau[n] = t2;
            s.nu[n] = (1.0 - d) * nu + d * nn;
        }
    }
}

unsigned blocks_of(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

void launch_beta(hipStream_t st, GridDev g, StarsDev s, const double* f, double* beta) {
    if (s.n > 0) hipLaunchKernelGGL(k_beta, dim3(blocks_of(s.n)), dim3(256), 0, st, g, s, f, beta);
}
void launch_gmm_update(hipStream_t st, StarsDev s, EpParams p, const double* comps, int K, const double* beta,
                       const double* lref) {
    if (s.n > 0) hipLaunchKernelGGL(k_gmm_update, dim3(blocks_of(s.n)), dim3(256), 0, st, s, p, comps, K, beta, lref);
}

}  // namespace ep
