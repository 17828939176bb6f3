// Unknown distances (Sec. 4.2, general case): each star's likelihood is a
// Gaussian mixture over components z in (l, b) = (ln s, log-extinction to
// distance s), and the tilted distribution sums over z and integrates over
// the distance s.
//
// The site variable is a_n = ln A(s~), the log-extinction to the catalogue
// position at distance s~.  The log-extinction at another distance s on the
// sightline is a_n + delta(s), delta(s) = ln A(s; fhat) - ln A(s~; fhat), with
// A(s) the forward model at the linearisation point extended past the star:
// samples t_k = k s~/T for k <= T (the star's own steps), then
// t_k = s~ + (k - T) step out to the last one inside the cube; A(s) is the
// trapezoid sum up to the last sample t_K <= s plus the partial trapezoid
// (s - t_K)(e^{F(t_K)} + e^{F(s)})/2.  For one component and one distance the
// likelihood in a_n is N(l; m_l, C_ll) N(a_n + delta(l); mu_b(l), v_b)
// (mu_b = m_b + C_lb/C_ll (l - m_l), v_b = C_bb - C_lb^2/C_ll), so against the
// cavity its normaliser and moments are closed form; the integral over l is
// a composite Gauss-Legendre rule (GMM_PANELS panels of 16 nodes over
// m_l +- GMM_WIDTH sd, cut at the cube's face).  C_ll = C_lb = 0 is a known
// distance: one node at l = m_l.
//
// One wave per star: the lanes evaluate e^F at the samples and keep the
// running sums in LDS, then take the distance nodes of every component, and
// three wave reductions (largest log term, normaliser and mean, variance)
// give the tilted moments; lane 0 writes the damped site.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace ep {

namespace {

constexpr int GMM_PANELS = 16;
constexpr int GMM_NODES = GMM_PANELS * 16;   // per component with a distance spread
constexpr double GMM_WIDTH = 8.0;

struct GL16 {
    double x[16], w[16];
};

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// trilinear F at o + fr (x - o), cell clamp(floor(p / h), 0, n - 2)
__device__ __forceinline__ double field_at(const GridDev& g, const double* __restrict__ f, double fr, double dx,
                                           double dy, double dz) {
    const double p[3] = {g.ox + fr * dx, g.oy + fr * dy, g.oz + fr * dz};
    int cc[3];
    double wv[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double c = floor(p[a] / g.h);
        c = c < 0 ? 0 : (c > g.n - 2 ? g.n - 2 : c);
        cc[a] = (int)c;
        wv[a] = p[a] / g.h - c;
    }
    double F = 0.0;
#pragma unroll
    for (int c8 = 0; c8 < 8; c8++) {
        const int bi = c8 & 1, bj = (c8 >> 1) & 1, bk = (c8 >> 2) & 1;
        const double phi = (bi ? wv[0] : 1.0 - wv[0]) * (bj ? wv[1] : 1.0 - wv[1]) * (bk ? wv[2] : 1.0 - wv[2]);
        F += phi * f[(cc[0] + bi) + (int64_t)g.n * ((cc[1] + bj) + (int64_t)g.n * (cc[2] + bk))];
    }
    return F;
}

struct Ray {
    GridDev g;
    const double* f;
    const double* sC;   // running sums of e^F over the samples (LDS)
    double dx, dy, dz, sref, del, step, E0, ET, AT;
    int T, Kmax;

    __device__ double frac(int k) const {
        return k <= T ? (double)k / (double)T : 1.0 + (double)(k - T) * step / sref;
    }
    __device__ double E(int k) const { return exp(field_at(g, f, frac(k), dx, dy, dz)); }
    // trapezoid sum over the samples 0..k
    __device__ double Alat(int k, double Ek) const {
        if (k == 0) return 0.0;
        if (k <= T) return del * (sC[k] - 0.5 * (E0 + Ek));
        return AT + step * (sC[k] - sC[T - 1] - 0.5 * (ET + Ek));
    }
    __device__ double A(double s) const {
        int K;
        if (s <= sref) {
            const double q = floor(s / del);
            K = q > (double)T ? T : (int)q;
        } else {
            const double q = floor((s - sref) / step);
            K = T + (q > (double)(Kmax - T) ? Kmax - T : (int)q);
        }
        if (K < 0) K = 0;
        const double tK = K <= T ? K * del : sref + (K - T) * step;
        const double EK = E(K);
        return Alat(K, EK) + 0.5 * (s - tK) * (EK + exp(field_at(g, f, s / sref, dx, dy, dz)));
    }
};

// one node of one component: log weight of the node, E[a | l], Var[a | l]
struct Comp {
    double lw, ml, mb, cll, clb, cbb, lo, h;
    int known, J;
};

__device__ __forceinline__ void node_lw(const Comp& c, const GL16& gl, int j, double& l, double& lW) {
    if (c.known) {
        l = c.ml;
        lW = 0.0;
    } else {
        const int p = j >> 4, i = j & 15;
        l = c.lo + c.h * (p + 0.5 * (1.0 + gl.x[i]));
        lW = log(0.5 * c.h * gl.w[i]);
    }
}

__device__ __forceinline__ void node_terms(const Comp& c, double l, double lW, double dlt, double mu_c, double v_c,
                                           double& lt, double& m, double& vz) {
    double mub, vb, lN;
    if (c.known) {
        mub = c.mb;
        vb = c.cbb;
        lN = 0.0;
    } else {
        mub = c.mb + (c.clb / c.cll) * (l - c.ml);
        vb = c.cbb - c.clb * c.clb / c.cll;
        lN = -0.5 * log(6.283185307179586 * c.cll) - 0.5 * (l - c.ml) * (l - c.ml) / c.cll;
    }
    const double y = mub - dlt, S = v_c + vb;
    lt = c.lw + lW + lN - 0.5 * log(6.283185307179586 * S) - 0.5 * (y - mu_c) * (y - mu_c) / S;
    m = (vb * mu_c + v_c * y) / S;
    vz = v_c * vb / S;
}

__device__ __forceinline__ bool comp_setup(const double* cp, double lnx, Comp& c) {
    if (!(cp[0] > 0.0)) return false;
    c.lw = log(cp[0]);
    c.ml = cp[1];
    c.mb = cp[2];
    c.cll = cp[3];
    c.clb = cp[4];
    c.cbb = cp[5];
    if (c.cll == 0.0) {
        c.known = 1;
        c.J = 1;
        c.lo = c.h = 0.0;
        return c.ml <= lnx;
    }
    c.known = 0;
    const double sd = sqrt(c.cll);
    c.lo = c.ml - GMM_WIDTH * sd;
    const double hi = fmin(c.ml + GMM_WIDTH * sd, lnx);
    if (!(hi > c.lo)) return false;
    c.h = (hi - c.lo) / GMM_PANELS;
    c.J = GMM_NODES;
    return true;
}

__global__ __launch_bounds__(64) void k_gmm_ray(GridDev g, StarsDev s, EpParams P, const double* __restrict__ f,
                                                const double* __restrict__ comps, int K, double L, double step,
                                                GL16 gl, int kcap) {
    extern __shared__ double smem[];
    double* sC = smem;          // kcap running sums
    double* sD = smem + kcap;   // delta at the nodes, GMM_NODES per component
    const int lane = threadIdx.x;
    const int64_t n = blockIdx.x;
    if (n >= s.n) return;
    const double qm = s.cav_mu[n], qv = s.cav_var[n];
    const double tau = s.tau[n], nu = s.nu[n];
    double tau_c = 1.0 / qv - tau, nu_c = qm / qv - nu;
    if (!(tau_c > 0.0)) {
        if (lane == 0) {
            s.status[n] = 1;
            s.dtau[n] = 0.0;
        }
        return;
    }
    double v_c = 1.0 / tau_c;
    if (v_c < P.vfloor) v_c = P.vfloor;
    const double mu_c = nu_c / tau_c;
    tau_c = 1.0 / v_c;
    nu_c = mu_c / v_c;

    Ray r;
    r.g = g;
    r.f = f;
    r.sC = sC;
    r.dx = s.xyz[3 * n] - g.ox;
    r.dy = s.xyz[3 * n + 1] - g.oy;
    r.dz = s.xyz[3 * n + 2] - g.oz;
    r.sref = sqrt(r.dx * r.dx + r.dy * r.dy + r.dz * r.dz);
    r.T = s.nsamp[n];
    r.del = r.sref / (double)r.T;
    r.step = step;
    {
        const double u[3] = {r.dx / r.sref, r.dy / r.sref, r.dz / r.sref};
        const double o[3] = {g.ox, g.oy, g.oz};
        double sx = INFINITY;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (u[a] > 0) sx = fmin(sx, (L - o[a]) / u[a]);
            else if (u[a] < 0) sx = fmin(sx, -o[a] / u[a]);
        }
        sx = fmax(sx, r.sref);
        int km = r.T + (int)floor((sx - r.sref) / step);
        r.Kmax = km < kcap - 1 ? km : kcap - 1;   // kcap is sized on the host for every star
        // e^F at the samples and their running sums (wave scans of 64)
        double carry = 0.0;
        for (int base = 0; base <= r.Kmax; base += 64) {
            const int k = base + lane;
            double v = k <= r.Kmax ? r.E(k) : 0.0;
#pragma unroll
            for (int o2 = 1; o2 < 64; o2 <<= 1) {
                const double t = __shfl_up(v, o2, 64);
                if (lane >= o2) v += t;
            }
            if (k <= r.Kmax) sC[k] = carry + v;
            carry += __shfl(v, 63, 64);
        }
        __syncthreads();
        r.E0 = sC[0];
        r.ET = r.E(r.T);
        r.AT = r.del * (sC[r.T] - 0.5 * (r.E0 + r.ET));
        const double lnx = log(sx), lnAref = log(r.AT);
        const double* cp = comps + n * (int64_t)K * 6;
        // pass 1: delta at every node (kept in LDS) and the largest log term
        double top = -INFINITY;
        for (int z = 0; z < K; z++) {
            Comp c;
            if (!comp_setup(cp + 6 * z, lnx, c)) continue;
            for (int j = lane; j < c.J; j += 64) {
                double l, lW, lt, m, vz;
                node_lw(c, gl, j, l, lW);
                const double dlt = log(r.A(exp(l))) - lnAref;
                sD[z * GMM_NODES + j] = dlt;
                node_terms(c, l, lW, dlt, mu_c, v_c, lt, m, vz);
                top = fmax(top, lt);
            }
        }
        top = wmax(top);
        __syncthreads();
        double Z = 0.0, M1 = 0.0;
        if (top > -INFINITY) {
            for (int z = 0; z < K; z++) {
                Comp c;
                if (!comp_setup(cp + 6 * z, lnx, c)) continue;
                for (int j = lane; j < c.J; j += 64) {
                    double l, lW, lt, m, vz;
                    node_lw(c, gl, j, l, lW);
                    node_terms(c, l, lW, sD[z * GMM_NODES + j], mu_c, v_c, lt, m, vz);
                    const double w = exp(lt - top);
                    Z += w;
                    M1 += w * m;
                }
            }
        }
        Z = wsum(Z);
        M1 = wsum(M1);
        const double mh = M1 / Z;
        double V = 0.0;
        if (top > -INFINITY) {
            for (int z = 0; z < K; z++) {
                Comp c;
                if (!comp_setup(cp + 6 * z, lnx, c)) continue;
                for (int j = lane; j < c.J; j += 64) {
                    double l, lW, lt, m, vz;
                    node_lw(c, gl, j, l, lW);
                    node_terms(c, l, lW, sD[z * GMM_NODES + j], mu_c, v_c, lt, m, vz);
                    V += exp(lt - top) * (vz + (m - mh) * (m - mh));
                }
            }
        }
        V = wsum(V);
        if (lane != 0) return;
        const bool any = top > -INFINITY;
        const double vh = any ? V / Z : NAN, mean = any ? mh : NAN;
        s.cav_mu[n] = mu_c;
        s.cav_var[n] = v_c;
        s.lnZ[n] = any ? top + log(Z) : -INFINITY;
        s.tmean[n] = mean;
        s.tvar[n] = vh;
        const double tn = 1.0 / vh - tau_c, nn = mean / vh - nu_c;
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

}  // namespace

// Samples on the sightline extended to the cube's face (the forward model
// above) for a star at xyz with T trapezoid steps: K_max + 1.
int64_t gmm_ray_samples(const double* xyz, const double* obs, int32_t T, double box, double step) {
    const double dv[3] = {xyz[0] - obs[0], xyz[1] - obs[1], xyz[2] - obs[2]};
    const double sref = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    double sx = INFINITY;
    for (int a = 0; a < 3; a++) {
        const double u = dv[a] / sref;
        if (u > 0) sx = std::fmin(sx, (box - obs[a]) / u);
        else if (u < 0) sx = std::fmin(sx, -obs[a] / u);
    }
    sx = std::fmax(sx, sref);
    return (int64_t)T + (int64_t)std::floor((sx - sref) / step) + 1;
}

int64_t gmm_lds_doubles(int64_t kcap, int K) { return kcap + (int64_t)K * GMM_NODES; }

void launch_gmm_ray(hipStream_t st, GridDev g, StarsDev s, EpParams p, const double* f, const double* comps, int K,
                    double box, double step, int kcap) {
    if (s.n <= 0) return;
    GL16 gl;
    gauss_legendre16(gl.x, gl.w);
    const size_t sh = sizeof(double) * (size_t)gmm_lds_doubles(kcap, K);
    hipLaunchKernelGGL(k_gmm_ray, dim3((unsigned)s.n), dim3(64), sh, st, g, s, p, f, comps, K, box, step, gl, kcap);
}

}  // namespace ep
