// Tilted-moment surrogate: a 4-128-128-128-3 SiLU network that predicts
// corrections to a Gaussian baseline of the per-star tilted distribution
// (Sec. 4.1 tilted distribution; App. A.2 moment matching).
//
// Baseline: the likelihood N(A | e^a, s^2) linearised in a at
// a0 = ln max(A, s) is Gaussian in a; times the cavity it gives (m0, v0) and
// a normaliser Z0.  Outputs (after de-standardisation):
//   y1 = (mean - m0)/sqrt(v0), y2 = ln(var/v0), y3 = ln Z - ln Z0.
// Features: (mu_c, ln v_c, A e^{-mu_c}, ln s - mu_c), standardised.
//
// Training: FP32 forward, backward and Adam kernels.  Inference: BF16
// operands on v_mfma_f32_16x16x16bf16_1k with FP32 accumulation, fused with
// the gate: a 20-node Gauss-Hermite rule centred at the predicted mean and
// standard deviation computes the moments of the true integrand, and a
// 32-node rule re-centred at those moments checks them; the star is accepted
// when the two passes agree to the tolerance, a bound on the tails beyond
// 8 sd is below it, and the prediction is within a factor 4 of the variance;
// the second pass's moments are used.
// Rejected stars go to the quadrature.  Without a network the rule is
// centred at the baseline (the reference for what the network gains).
#include <hip/hip_runtime.h>

#include <vector>

#include <cmath>

#include "kernels.h"
#include "surrogate.h"

namespace ep {

constexpr int HD = 128;

// parameter blob offsets (floats)
constexpr int O_W1 = 0, O_B1 = O_W1 + 4 * HD, O_W2 = O_B1 + HD, O_B2 = O_W2 + HD * HD, O_W3 = O_B2 + HD,
              O_B3 = O_W3 + HD * HD, O_W4 = O_B3 + HD, O_B4 = O_W4 + HD * 3, O_XM = O_B4 + 3, O_XS = O_XM + 4,
              O_YM = O_XS + 4, O_YS = O_YM + 3, O_END = O_YS + 3;
static_assert(O_END == MLP_NPARAM, "blob layout");
static_assert(O_XM == MLP_NTRAIN, "trainable prefix");

__device__ __forceinline__ float silu_f(float x) { return x / (1.0f + expf(-x)); }
__device__ __forceinline__ float dsilu_f(float x) {
    float s = 1.0f / (1.0f + expf(-x));
    return s * (1.0f + x * (1.0f - s));
}

// ---------------------------------------------------------------------------
// Training (FP32).  Batch rows are gathered through idx (a shuffled order).
// ---------------------------------------------------------------------------
// layer 1: z1 = x W1 + b1, h1 = silu(z1); one thread per (sample, unit)
__global__ void k_mlp_fwd1(int B, const int32_t* idx, const float* X, const float* P, float* z1, float* h1) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * HD) return;
    const int b = (int)(t / HD), o = (int)(t % HD);
    const float* x = X + 4 * (int64_t)idx[b];
    float z = P[O_B1 + o];
#pragma unroll
    for (int k = 0; k < 4; k++) z += x[k] * P[O_W1 + k * HD + o];
    z1[t] = z;
    h1[t] = silu_f(z);
}

// dense 128 -> 128: out[b][o] = sum_k in[b][k] W[k][o] (+ b[o]); 64 samples per block.
// transposed: out[b][k] = sum_o in[b][o] W[k][o] (back-propagation through W).
// act: z = out (+bias); h = silu(z)  (forward)   |  dz = out * dsilu(zprev)  (backward)
template <bool BWD>
__global__ __launch_bounds__(256) void k_mlp_dense(int B, const float* in, const float* W, const float* bias,
                                                   const float* zaux, float* zout, float* hout) {
    __shared__ float sW[HD * (HD + 1)];
    __shared__ float sx[64 * HD];
    const int b0 = blockIdx.x * 64;
    for (int q = threadIdx.x; q < HD * HD; q += 256) {
        int k = q / HD, o = q % HD;
        if (BWD) sW[o * (HD + 1) + k] = W[q];   // sW[o][k] = W[k][o]: rows of W^T
        else sW[k * (HD + 1) + o] = W[q];
    }
    for (int q = threadIdx.x; q < 64 * HD; q += 256) {
        int b = b0 + q / HD;
        sx[q] = b < B ? in[(int64_t)b * HD + q % HD] : 0.0f;
    }
    __syncthreads();
    const int sb = threadIdx.x >> 2, og = (threadIdx.x & 3) * 32;
    float acc[32];
#pragma unroll
    for (int j = 0; j < 32; j++) acc[j] = 0.0f;
    for (int k = 0; k < HD; k++) {
        const float xv = sx[sb * HD + k];
#pragma unroll
        for (int j = 0; j < 32; j++) acc[j] += xv * sW[k * (HD + 1) + og + j];
    }
    const int b = b0 + sb;
    if (b >= B) return;
#pragma unroll
    for (int j = 0; j < 32; j++) {
        const int64_t q = (int64_t)b * HD + og + j;
        if (!BWD) {
            const float z = acc[j] + bias[og + j];
            zout[q] = z;
            hout[q] = silu_f(z);
        } else {
            zout[q] = acc[j] * dsilu_f(zaux[q]);
        }
    }
}

// output layer, loss and its gradient: out = h3 W4 + b4; d = out - y;
// dout = 2 d / B; loss += sum d^2 / B
__global__ void k_mlp_out(int B, const int32_t* idx, const float* h3, const float* P, const float* Y, float* dout,
                          double* loss) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (b < B) {
        const float* y = Y + 3 * (int64_t)idx[b];
        for (int c = 0; c < 3; c++) {
            float o = P[O_B4 + c];
            for (int k = 0; k < HD; k++) o += h3[(int64_t)b * HD + k] * P[O_W4 + k * 3 + c];
            const float d = o - y[c];
            dout[3 * (int64_t)b + c] = 2.0f * d / (float)B;
            l += (double)d * d / B;
        }
    }
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss, l);
}

// dz3 = (dout W4^T) * dsilu(z3)
__global__ void k_mlp_bwd_out(int B, const float* dout, const float* P, const float* z3, float* dz3) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * HD) return;
    const int b = (int)(t / HD), k = (int)(t % HD);
    float s = 0.0f;
    for (int c = 0; c < 3; c++) s += dout[3 * (int64_t)b + c] * P[O_W4 + k * 3 + c];
    dz3[t] = s * dsilu_f(z3[t]);
}

// weight gradient G[k][o] += sum_b A[b][k] D[b][o] over a chunk of the batch;
// bias gradient when k == KA (A implicitly 1).  KA rows of A, NO columns of D.
__global__ __launch_bounds__(256) void k_mlp_wgrad(int B, int KA, int NO, const float* A, const int32_t* idx,
                                                   const float* Xin, const float* D, float* G, float* Gb) {
    // grid: x = output tile over (KA+1) x NO in 16x16 tiles... simple form: one thread per (k, o)
    const int chunk = 512;
    const int b0 = blockIdx.y * chunk;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)(KA + 1) * NO) return;
    const int k = (int)(t / NO), o = (int)(t % NO);
    float s = 0.0f;
    const int b1 = min(B, b0 + chunk);
    for (int b = b0; b < b1; b++) {
        float a;
        if (k == KA) a = 1.0f;
        else if (Xin) a = Xin[4 * (int64_t)idx[b] + k];
        else a = A[(int64_t)b * KA + k];
        s += a * D[(int64_t)b * NO + o];
    }
    if (k == KA) atomicAdd(Gb + o, s);
    else atomicAdd(G + k * NO + o, s);
}

__global__ void k_mlp_adam(int n, float* P, const float* G, float* m, float* v, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_zero_f(float* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

static unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// one forward + backward pass; G (MLP_NTRAIN floats) must be zero on entry
void mlp_fwd_bwd(hipStream_t st, const MlpWork& w, int B, const int32_t* idx, const float* X, const float* Y,
                 const float* P, float* G, double* loss) {
    hipLaunchKernelGGL(k_mlp_fwd1, dim3(nblk((int64_t)B * HD)), dim3(256), 0, st, B, idx, X, P, w.z1, w.h1);
    hipLaunchKernelGGL(k_mlp_dense<false>, dim3(nblk(B, 64)), dim3(256), 0, st, B, w.h1, P + O_W2, P + O_B2,
                       (const float*)nullptr, w.z2, w.h2);
    hipLaunchKernelGGL(k_mlp_dense<false>, dim3(nblk(B, 64)), dim3(256), 0, st, B, w.h2, P + O_W3, P + O_B3,
                       (const float*)nullptr, w.z3, w.h3);
    hipLaunchKernelGGL(k_mlp_out, dim3(nblk(B)), dim3(256), 0, st, B, idx, w.h3, P, Y, w.dout, loss);
    const unsigned nch = (unsigned)((B + 511) / 512);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(nblk((HD + 1) * 3), nch), dim3(256), 0, st, B, HD, 3, w.h3, idx,
                       (const float*)nullptr, w.dout, G + O_W4, G + O_B4);
    hipLaunchKernelGGL(k_mlp_bwd_out, dim3(nblk((int64_t)B * HD)), dim3(256), 0, st, B, w.dout, P, w.z3, w.dz3);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(nblk((HD + 1) * HD), nch), dim3(256), 0, st, B, HD, HD, w.h2, idx,
                       (const float*)nullptr, w.dz3, G + O_W3, G + O_B3);
    hipLaunchKernelGGL(k_mlp_dense<true>, dim3(nblk(B, 64)), dim3(256), 0, st, B, w.dz3, P + O_W3,
                       (const float*)nullptr, w.z2, w.dz2, (float*)nullptr);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(nblk((HD + 1) * HD), nch), dim3(256), 0, st, B, HD, HD, w.h1, idx,
                       (const float*)nullptr, w.dz2, G + O_W2, G + O_B2);
    hipLaunchKernelGGL(k_mlp_dense<true>, dim3(nblk(B, 64)), dim3(256), 0, st, B, w.dz2, P + O_W2,
                       (const float*)nullptr, w.z1, w.dz1, (float*)nullptr);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(nblk(5 * HD), nch), dim3(256), 0, st, B, 4, HD, (const float*)nullptr, idx,
                       X, w.dz1, G + O_W1, G + O_B1);
}

void mlp_zero(hipStream_t st, float* p, int64_t n) {
    hipLaunchKernelGGL(k_zero_f, dim3(nblk(n) > 4096 ? 4096 : nblk(n)), dim3(256), 0, st, p, n);
}

void mlp_adam(hipStream_t st, float* P, const float* G, float* m, float* v, float lr, int step) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3(nblk(MLP_NTRAIN)), dim3(256), 0, st, MLP_NTRAIN, P, G, m, v, lr, b1, b2,
                       1e-8f, c1, c2);
}

// ---------------------------------------------------------------------------
// Inference with BF16 MFMA, fused with the gate and the site update.
// One block of 256 threads per 64 stars.
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

// Gauss-Hermite rules of the gate: a 20-node rule for the first pass and a
// 32-node rule for the second.  Nodes, then ln(weight) + node^2, per rule.
constexpr int NGH1 = 20, NGH2 = 32;
__constant__ double c_gh1[2 * NGH1];
__constant__ double c_gh2[2 * NGH2];

// Moments (ln Z, mean, var) of cavity(a) x N(A | e^a, s^2) by an N-node
// Gauss-Hermite rule with centre c and scale sqrt(cv); one streaming pass
// with a running maximum of the log-terms, moments taken about c.
template <int N>
__device__ __forceinline__ void gh_moments(const double* rule, double mu, double v, double A, double s, double c,
                                           double cv, double& lnZ, double& mean, double& var) {
    const double h = 1.4142135623730951 * sqrt(cv), s2 = s * s;
    const double cst = -0.5 * log(6.283185307179586 * v) - 0.5 * log(6.283185307179586 * s2);
    double mx = -1e300, Z = 0.0, M1 = 0.0, M2 = 0.0;
    for (int i = 0; i < N; i++) {
        const double d = h * rule[i];
        const double a = c + d, ea = exp(a);
        const double lg = -(a - mu) * (a - mu) / (2.0 * v) - (A - ea) * (A - ea) / (2.0 * s2) + rule[N + i];
        if (lg > mx) {
            const double r = exp(mx - lg);
            Z *= r;
            M1 *= r;
            M2 *= r;
            mx = lg;
        }
        const double e = exp(lg - mx);
        Z += e;
        M1 += e * d;
        M2 += e * d * d;
    }
    const double m1 = M1 / Z;
    mean = c + m1;
    var = M2 / Z - m1 * m1;
    lnZ = log(Z) + mx + cst + log(h);
}

// Upper bounds, relative to Z, on the mass and on the second moment about c
// of the tilted density beyond c - K sd and c + K sd.  On each tail the
// likelihood is bounded by its value at the cut when it is monotone there
// (e^a below A on the left, above A on the right), else by its maximum, and
// the cavity's partial moments are closed-form.  Mass the rules cannot see
// is bounded this way; the agreement of the two passes does not see it.
__device__ __forceinline__ void tail_bounds(double mu, double v, double A, double s, double c, double var,
                                            double lnZ, double& t0, double& t2) {
    constexpr double K = 8.0;
    const double sd = sqrt(var), sv = sqrt(v), s2 = s * s;
    const double lmax = -0.5 * log(6.283185307179586 * s2) - lnZ;
    const double aL = c - K * sd, aR = c + K * sd;
    const double eL = exp(aL), eR = exp(aR);
    const double fL = exp(lmax - (eL <= A ? (A - eL) * (A - eL) / (2.0 * s2) : 0.0));
    const double fR = exp(lmax - (eR >= A ? (A - eR) * (A - eR) / (2.0 * s2) : 0.0));
    const double tL = (aL - mu) / sv, tR = (mu - aR) / sv, d = mu - c;
    const double PL = 0.5 * erfc(-tL * 0.7071067811865476), PR = 0.5 * erfc(-tR * 0.7071067811865476);
    const double pL = 0.3989422804014327 * exp(-0.5 * tL * tL), pR = 0.3989422804014327 * exp(-0.5 * tR * tR);
    t0 = fL * PL + fR * PR;
    t2 = fL * (v * (PL - tL * pL) - 2.0 * d * sv * pL + d * d * PL) +
         fR * (v * (PR - tR * pR) + 2.0 * d * sv * pR + d * d * PR);
}

__device__ __forceinline__ short to_bf16(float x) {   // round to nearest even
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// Gaussian baseline of the tilted distribution
__device__ __forceinline__ void baseline_dev(double mu, double v, double A, double s, double& m0, double& v0,
                                             double& lnZ0) {
    const double y0 = A > s ? A : s;
    const double ml = log(y0) + (A - y0) / y0;
    const double vl = (s / y0) * (s / y0);
    v0 = 1.0 / (1.0 / v + 1.0 / vl);
    m0 = v0 * (mu / v + ml / vl);
    const double tv = v + vl;
    lnZ0 = -0.5 * log(6.283185307179586 * tv) - 0.5 * (ml - mu) * (ml - mu) / tv - log(y0);
}

// 16 x 128 strip (rows r0..r0+15) of h (bf16, [64][HD+8]) times W (bf16,
// [HD][HD+8] as W[k][o]) -> 8 MFMA blocks of 16 x 16 in acc[8]
__device__ __forceinline__ void strip_mma(f4 acc[8], const short* h, const short* W, int r0) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = 4 * (lane >> 4);
#pragma unroll
    for (int j = 0; j < 8; j++) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < HD; k0 += 16) {
        s4 a;
#pragma unroll
        for (int q = 0; q < 4; q++) a[q] = h[(r0 + li) * (HD + 8) + k0 + lk + q];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            s4 b;
#pragma unroll
            for (int q = 0; q < 4; q++) b[q] = W[(k0 + lk + q) * (HD + 8) + 16 * j + li];
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
        }
    }
}

__global__ __launch_bounds__(256) void k_mlp_tilted(StarsDev s, EpParams prm, const float* __restrict__ P,
                                                    const short* __restrict__ Wbf, double tol, int32_t* fb_list,
                                                    int32_t* fb_count, int32_t* accepted, double* errest,
                                                    double* out3) {
    __shared__ short sW2[HD * (HD + 8)];
    __shared__ short sW3[HD * (HD + 8)];
    __shared__ short sh[64 * (HD + 8)];
    __shared__ float sh3[64 * (HD + 1)];
    __shared__ double sin4[64][4];
    __shared__ double scav[64][4];   // mu_c, v_c, tau_c, nu_c
    __shared__ int sok[64];
    const int tid = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * 64;
    if (P)
        for (int q = tid; q < HD * HD; q += 256) {
            sW2[(q / HD) * (HD + 8) + q % HD] = Wbf[q];
            sW3[(q / HD) * (HD + 8) + q % HD] = Wbf[HD * HD + q];
        }
    // per star: cavity from the q-marginal, skip rules, features
    if (tid < 64) {
        const int64_t star = s0 + tid;
        int ok = 0;
        double mu_c = 0, v_c = 1, tau_c = 1, nu_c = 0, A = 1, sg = 1;
        if (star < s.n) {
            const double qm = s.cav_mu[star], qv = s.cav_var[star];
            tau_c = 1.0 / qv - s.tau[star];
            nu_c = qm / qv - s.nu[star];
            A = s.A[star];
            sg = s.sigma[star];
            if (tau_c > 0.0) {
                v_c = 1.0 / tau_c;
                if (v_c < prm.vfloor) v_c = prm.vfloor;
                mu_c = nu_c / tau_c;
                tau_c = 1.0 / v_c;
                nu_c = mu_c / v_c;
                ok = 1;
            } else {
                ok = -1;   // cavity skip
            }
        }
        sok[tid] = ok;
        scav[tid][0] = mu_c;
        scav[tid][1] = v_c;
        scav[tid][2] = tau_c;
        scav[tid][3] = nu_c;
        sin4[tid][0] = A;
        sin4[tid][1] = sg;
        // standardised features
        const double f0 = mu_c, f1 = log(v_c), f2 = A * exp(-mu_c), f3 = log(sg) - mu_c;
        if (!P) goto no_net;
        {
        float x[4] = {(float)((f0 - P[O_XM]) / P[O_XS]), (float)((f1 - P[O_XM + 1]) / P[O_XS + 1]),
                      (float)((f2 - P[O_XM + 2]) / P[O_XS + 2]), (float)((f3 - P[O_XM + 3]) / P[O_XS + 3])};
        // layer 1 in FP32, stored as bf16
        for (int o = 0; o < HD; o++) {
            float z = P[O_B1 + o];
#pragma unroll
            for (int k = 0; k < 4; k++) z += x[k] * P[O_W1 + k * HD + o];
            sh[tid * (HD + 8) + o] = to_bf16(silu_f(z));
        }
        }
    no_net:;
    }
    __syncthreads();
    const int w = tid >> 6, lane = tid & 63;
    const int r0 = 16 * w;   // each wave owns 16 of the 64 stars
    f4 acc[8];
    if (P) {
    // layer 2
    strip_mma(acc, sh, sW2, r0);
    __syncthreads();   // every wave has read sh
#pragma unroll
    for (int j = 0; j < 8; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            // v_mfma_f32_16x16x16bf16_1k output: lane l, item r -> row 4(l/16) + r, column l%16
            const int row = r0 + 4 * (lane >> 4) + r, col = 16 * j + (lane & 15);
            sh[row * (HD + 8) + col] = to_bf16(silu_f(acc[j][r] + P[O_B2 + col]));
        }
    __syncthreads();
    // layer 3 (kept in FP32 for the output layer)
    strip_mma(acc, sh, sW3, r0);
#pragma unroll
    for (int j = 0; j < 8; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int row = r0 + 4 * (lane >> 4) + r, col = 16 * j + (lane & 15);
            sh3[row * (HD + 1) + col] = silu_f(acc[j][r] + P[O_B3 + col]);
        }
    }
    __syncthreads();
    if (tid >= 64) return;
    const int64_t star = s0 + tid;
    if (star >= s.n || sok[tid] == 0) return;
    if (sok[tid] < 0) {   // improper cavity: skip (as the quadrature path)
        if (accepted) accepted[star] = 0;
        if (s.status) { s.status[star] = 1; s.dtau[star] = 0.0; }
        return;
    }
    float y[3] = {0.f, 0.f, 0.f};
    if (P)
        for (int c = 0; c < 3; c++) {
            float o = P[O_B4 + c];
            for (int k = 0; k < HD; k++) o += sh3[tid * (HD + 1) + k] * P[O_W4 + k * 3 + c];
            y[c] = o * P[O_YS + c] + P[O_YM + c];
        }
    const double mu_c = scav[tid][0], v_c = scav[tid][1], A = sin4[tid][0], sg = sin4[tid][1];
    double m0, v0, lnZ0;
    baseline_dev(mu_c, v_c, A, sg, m0, v0, lnZ0);
    double pm, pv, plz;
    if (P) {
        pm = m0 + sqrt(v0) * (double)y[0];
        pv = v0 * exp((double)y[1]);
        plz = lnZ0 + (double)y[2];
    } else {   // no network: centre the check at the analytic baseline
        pm = m0;
        pv = v0;
        plz = lnZ0;
    }
    // gate: moments of the true integrand by the 20-node rule centred at the
    // prediction, then by the 32-node rule re-centred at those moments; the
    // second pass is the more accurate, so the difference of the two bounds
    // the first pass's error and, conservatively, the second's.  Added to it:
    // the bounds on the tails beyond 8 sd (the Cauchy-Schwarz bound for the
    // mean).  Accept when within tol and the predicted variance is within a
    // factor 4.
    double glz1, gm1, gv1, glz, gm, gv;
    gh_moments<NGH1>(c_gh1, mu_c, v_c, A, sg, pm, pv, glz1, gm1, gv1);
    gh_moments<NGH2>(c_gh2, mu_c, v_c, A, sg, gm1, gv1 > 0.0 ? gv1 : pv, glz, gm, gv);
    double t0, t2;
    tail_bounds(mu_c, v_c, A, sg, gm, gv, glz, t0, t2);
    const double scale = fmax(fabs(gm), sqrt(fabs(gv)));
    double err = fabs(glz - glz1) + t0;
    err = fmax(err, (fabs(gm - gm1) + sqrt(t0 * t2)) / scale);
    err = fmax(err, fabs(gv / gv1 - 1.0) + t2 / gv);
    if (!isfinite(err) || !(gv > 0.0) || !(pv > 0.25 * gv && pv < 4.0 * gv)) err = 1e300;
    const bool acc_ok = err <= tol;
    if (errest) errest[star] = err;
    if (accepted) accepted[star] = acc_ok ? 1 : 0;
    if (out3) {
        out3[3 * star] = acc_ok ? glz : plz;
        out3[3 * star + 1] = acc_ok ? gm : pm;
        out3[3 * star + 2] = acc_ok ? gv : pv;
    }
    if (!s.status) return;   // batch evaluation: no EP state
    if (!acc_ok) {
        fb_list[atomicAdd(fb_count, 1)] = (int32_t)star;
        return;
    }
    const double tau_c = scav[tid][2], nu_c = scav[tid][3];
    const double tau = s.tau[star], nu = s.nu[star];
    s.cav_mu[star] = mu_c;
    s.cav_var[star] = v_c;
    s.lnZ[star] = glz;
    s.tmean[star] = gm;
    s.tvar[star] = gv;
    const double tn = 1.0 / gv - tau_c, nn = gm / gv - nu_c;
    if (!(tn >= 0.0) || !isfinite(tn) || !isfinite(nn)) {
        s.status[star] = 2;
        s.dtau[star] = 0.0;
    } else {
        const double d = prm.damping;
        const double t2 = (1.0 - d) * tau + d * tn;
        s.status[star] = 0;
        s.dtau[star] = fabs(t2 - tau);
        s.tau[star] = t2;
        s.nu[star] = (1.0 - d) * nu + d * nn;
    }
}

__global__ void k_to_bf16(const float* P, short* Wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < HD * HD) {
        Wbf[i] = to_bf16(P[O_W2 + i]);
        Wbf[HD * HD + i] = to_bf16(P[O_W3 + i]);
    }
}

void mlp_make_bf16(hipStream_t st, const float* P, short* Wbf) {
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(HD * HD)), dim3(256), 0, st, P, Wbf);
}

void launch_mlp_tilted(hipStream_t st, StarsDev s, EpParams p, const float* P, const short* Wbf, double tol,
                       int32_t* fb_list, int32_t* fb_count, int32_t* accepted, double* errest, double* out3) {
    if (s.n <= 0) return;
    hipLaunchKernelGGL(k_mlp_tilted, dim3((unsigned)((s.n + 63) / 64)), dim3(256), 0, st, s, p, P, Wbf, tol, fb_list,
                       fb_count, accepted, errest, out3);
}

// n-node Gauss-Hermite rule (weight e^{-x^2}): Newton's iteration on the
// orthonormal Hermite recurrence from the published asymptotic first guesses
// for the largest nodes and extrapolation from the previous two for the
// rest (Press et al., Numerical Recipes, Sec. 4.5).
// Writes the nodes to out[0..n) and ln(weight) + node^2 to out[n..2n).
static void gauss_hermite_rule(int n, double* out) {
    std::vector<double> x(n), w(n);
    const double pi4 = 0.7511255444649425;   // pi^{-1/4}
    double z = 0;
    for (int i = 0; i < (n + 1) / 2; i++) {
        if (i == 0) z = sqrt(2.0 * n + 1) - 1.85575 * pow(2.0 * n + 1, -0.16667);
        else if (i == 1) z -= 1.14 * pow((double)n, 0.426) / z;
        else if (i == 2) z = 1.86 * z - 0.86 * x[0];
        else if (i == 3) z = 1.91 * z - 0.91 * x[1];
        else z = 2.0 * z - x[i - 2];
        double pp = 0;
        for (int it = 0; it < 100; it++) {
            double p1 = pi4, p2 = 0.0;
            for (int j = 1; j <= n; j++) {
                double p3 = p2;
                p2 = p1;
                p1 = z * sqrt(2.0 / j) * p2 - sqrt((double)(j - 1) / j) * p3;
            }
            pp = sqrt(2.0 * n) * p2;
            double dz = p1 / pp;
            z -= dz;
            if (fabs(dz) < 1e-15) break;
        }
        x[i] = z;
        x[n - 1 - i] = -z;
        w[i] = 2.0 / (pp * pp);
        w[n - 1 - i] = w[i];
    }
    for (int i = 0; i < n; i++) {
        out[i] = x[i];
        out[n + i] = log(w[i]) + x[i] * x[i];
    }
}

hipError_t set_gauss_hermite(hipStream_t st) {
    double r1[2 * NGH1], r2[2 * NGH2];
    gauss_hermite_rule(NGH1, r1);
    gauss_hermite_rule(NGH2, r2);
    hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_gh1), r1, sizeof(r1), 0, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_gh2), r2, sizeof(r2), 0, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

}  // namespace ep
