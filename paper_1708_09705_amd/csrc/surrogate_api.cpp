// C ABI of the tilted-moment surrogate: training, gated prediction and a
// gradient hook.  The network, its baseline and its gate are described in
// surrogate.hip; every numerical step runs in those kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "../../include/ep.h"
#include "kernels.h"
#include "surrogate.h"

using namespace ep;

namespace ep {
void set_last_error(const std::string& m);   // api.cpp
}

namespace {

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

template <class T>
bool dalloc(DevBuf& b, int64_t n) {
    if (hipMalloc(&b.p, std::max<int64_t>(n, 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return true;
}

// Gaussian baseline of the tilted distribution (see surrogate.hip)
void baseline(double mu, double v, double A, double s, double& m0, double& v0, double& lnZ0) {
    const double y0 = A > s ? A : s;
    const double ml = std::log(y0) + (A - y0) / y0;
    const double vl = (s / y0) * (s / y0);
    v0 = 1.0 / (1.0 / v + 1.0 / vl);
    m0 = v0 * (mu / v + ml / vl);
    const double tv = v + vl;
    lnZ0 = -0.5 * std::log(6.283185307179586 * tv) - 0.5 * (ml - mu) * (ml - mu) / tv - std::log(y0);
}

void features(const double* in, double* f) {
    const double mu = in[0], v = in[1], A = in[2], s = in[3];
    f[0] = mu;
    f[1] = std::log(v);
    f[2] = A * std::exp(-mu);
    f[3] = std::log(s) - mu;
}

}  // namespace

extern "C" {

int ep_mlp_train(const ep_mlp_hyper* hp, int64_t n, const double* inputs, const double* targets, float* weights_out,
                 double* loss_per_epoch, int32_t device) {
    if (!hp || n <= 0 || !inputs || !targets || !weights_out || hp->epochs <= 0 || hp->batch <= 0 ||
        !(hp->lr > 0)) {
        set_last_error("ep_mlp_train: bad arguments");
        return EP_ERR_INVALID_ARG;
    }
    // features and baseline-relative targets; drop rows that are not finite
    std::vector<double> F, T;
    F.reserve(4 * n);
    T.reserve(3 * n);
    for (int64_t i = 0; i < n; i++) {
        const double* in = inputs + 4 * i;
        const double* tg = targets + 3 * i;
        if (!(in[1] > 0) || !(in[3] > 0) || !(tg[2] > 0)) continue;
        double f[4], m0, v0, lz0;
        features(in, f);
        baseline(in[0], in[1], in[2], in[3], m0, v0, lz0);
        const double t[3] = {(tg[1] - m0) / std::sqrt(v0), std::log(tg[2] / v0), tg[0] - lz0};
        bool ok = true;
        for (double x : f) ok &= std::isfinite(x);
        for (double x : t) ok &= std::isfinite(x);
        if (!ok) continue;
        F.insert(F.end(), f, f + 4);
        T.insert(T.end(), t, t + 3);
    }
    const int64_t m = (int64_t)T.size() / 3;
    const int B = hp->batch;
    if (m < B) {
        set_last_error("ep_mlp_train: fewer valid rows than one batch");
        return EP_ERR_INVALID_ARG;
    }
    // standardisation
    double xm[4] = {0}, xs[4] = {0}, ym[3] = {0}, ys[3] = {0};
    for (int64_t i = 0; i < m; i++) {
        for (int k = 0; k < 4; k++) xm[k] += F[4 * i + k];
        for (int k = 0; k < 3; k++) ym[k] += T[3 * i + k];
    }
    for (int k = 0; k < 4; k++) xm[k] /= m;
    for (int k = 0; k < 3; k++) ym[k] /= m;
    for (int64_t i = 0; i < m; i++) {
        for (int k = 0; k < 4; k++) xs[k] += (F[4 * i + k] - xm[k]) * (F[4 * i + k] - xm[k]);
        for (int k = 0; k < 3; k++) ys[k] += (T[3 * i + k] - ym[k]) * (T[3 * i + k] - ym[k]);
    }
    for (int k = 0; k < 4; k++) xs[k] = std::max(std::sqrt(xs[k] / m), 1e-12);
    for (int k = 0; k < 3; k++) ys[k] = std::max(std::sqrt(ys[k] / m), 1e-12);
    std::vector<float> X(4 * m), Y(3 * m);
    for (int64_t i = 0; i < m; i++) {
        for (int k = 0; k < 4; k++) X[4 * i + k] = (float)((F[4 * i + k] - xm[k]) / xs[k]);
        for (int k = 0; k < 3; k++) Y[3 * i + k] = (float)((T[3 * i + k] - ym[k]) / ys[k]);
    }
    // Glorot-uniform initialisation, zero biases
    std::vector<float> P(MLP_NPARAM, 0.0f);
    std::mt19937_64 rng(hp->seed);
    auto glorot = [&](int off, int fin, int fout) {
        const double a = std::sqrt(6.0 / (fin + fout));
        std::uniform_real_distribution<double> U(-a, a);
        for (int i = 0; i < fin * fout; i++) P[off + i] = (float)U(rng);
    };
    const int H = 128;
    int o = 0;
    glorot(o, 4, H);
    o += 4 * H + H;
    glorot(o, H, H);
    o += H * H + H;
    glorot(o, H, H);
    o += H * H + H;
    glorot(o, H, 3);
    o += 3 * H + 3;
    for (int k = 0; k < 4; k++) { P[o + k] = (float)xm[k]; P[o + 4 + k] = (float)xs[k]; }
    for (int k = 0; k < 3; k++) { P[o + 8 + k] = (float)ym[k]; P[o + 11 + k] = (float)ys[k]; }
    if (hipSetDevice(device) != hipSuccess) { set_last_error("hipSetDevice failed"); return EP_ERR_DEVICE; }
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        set_last_error("stream creation failed");
        return EP_ERR_DEVICE;
    }
    struct SG {
        hipStream_t s;
        ~SG() { (void)hipStreamDestroy(s); }
    } sg{st};
    DevBuf dX, dY, dP, dG, dM, dV, dIdx, dW, dL;
    if (!dalloc<float>(dX, 4 * m) || !dalloc<float>(dY, 3 * m) || !dalloc<float>(dP, MLP_NPARAM) ||
        !dalloc<float>(dG, MLP_NPARAM) || !dalloc<float>(dM, MLP_NPARAM) || !dalloc<float>(dV, MLP_NPARAM) ||
        !dalloc<int32_t>(dIdx, m) || !dalloc<float>(dW, (int64_t)B * H * 9 + (int64_t)B * 3) ||
        !dalloc<double>(dL, 1)) {
        set_last_error("ep_mlp_train: device allocation failed");
        return EP_ERR_OOM;
    }
    (void)hipMemcpyAsync(dX.p, X.data(), 4 * m * sizeof(float), hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(dY.p, Y.data(), 3 * m * sizeof(float), hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(dP.p, P.data(), MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, st);
    mlp_zero(st, (float*)dM.p, MLP_NPARAM);
    mlp_zero(st, (float*)dV.p, MLP_NPARAM);
    float* wb = (float*)dW.p;
    MlpWork w{};
    float** parts[] = {&w.z1, &w.h1, &w.z2, &w.h2, &w.z3, &w.h3, &w.dz3, &w.dz2, &w.dz1};
    for (int i = 0; i < 9; i++) *parts[i] = wb + (int64_t)i * B * H;
    w.dout = wb + (int64_t)9 * B * H;
    std::vector<int32_t> idx(m);
    std::iota(idx.begin(), idx.end(), 0);
    const int64_t steps = m / B;
    const int64_t total = steps * hp->epochs;
    int64_t step = 0;
    for (int e = 0; e < hp->epochs; e++) {
        std::shuffle(idx.begin(), idx.end(), rng);
        (void)hipMemcpyAsync(dIdx.p, idx.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, st);
        (void)hipMemsetAsync(dL.p, 0, sizeof(double), st);
        for (int64_t q = 0; q < steps; q++) {
            step++;
            const float lr = (float)(hp->lr * 0.5 * (1.0 + std::cos(3.141592653589793 * (step - 1) / total)));
            mlp_zero(st, (float*)dG.p, MLP_NTRAIN);
            mlp_fwd_bwd(st, w, B, (int32_t*)dIdx.p + q * B, (float*)dX.p, (float*)dY.p, (float*)dP.p, (float*)dG.p,
                        (double*)dL.p);
            mlp_adam(st, (float*)dP.p, (float*)dG.p, (float*)dM.p, (float*)dV.p, lr, (int)step);
        }
        double L = 0;
        (void)hipMemcpyAsync(&L, dL.p, sizeof(double), hipMemcpyDeviceToHost, st);
        if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) {
            set_last_error("ep_mlp_train: kernel failure");
            return EP_ERR_DEVICE;
        }
        if (loss_per_epoch) loss_per_epoch[e] = L / steps;
    }
    (void)hipMemcpyAsync(weights_out, dP.p, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, st);
    if (hipStreamSynchronize(st) != hipSuccess) { set_last_error("copy failed"); return EP_ERR_DEVICE; }
    return EP_OK;
}

int ep_mlp_loss_grad(const float* weights, int64_t n, const float* xstd, const float* ystd, double* loss, float* grad,
                     int32_t device) {
    if (!weights || n <= 0 || n > (1 << 20) || !xstd || !ystd || !loss || !grad) {
        set_last_error("ep_mlp_loss_grad: bad arguments");
        return EP_ERR_INVALID_ARG;
    }
    if (hipSetDevice(device) != hipSuccess) { set_last_error("hipSetDevice failed"); return EP_ERR_DEVICE; }
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) { set_last_error("stream"); return EP_ERR_DEVICE; }
    struct SG {
        hipStream_t s;
        ~SG() { (void)hipStreamDestroy(s); }
    } sg{st};
    const int H = 128;
    DevBuf dX, dY, dP, dG, dIdx, dW, dL;
    if (!dalloc<float>(dX, 4 * n) || !dalloc<float>(dY, 3 * n) || !dalloc<float>(dP, MLP_NPARAM) ||
        !dalloc<float>(dG, MLP_NPARAM) || !dalloc<int32_t>(dIdx, n) || !dalloc<float>(dW, n * H * 9 + n * 3) ||
        !dalloc<double>(dL, 1)) {
        set_last_error("ep_mlp_loss_grad: allocation failed");
        return EP_ERR_OOM;
    }
    std::vector<int32_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    (void)hipMemcpyAsync(dX.p, xstd, 4 * n * sizeof(float), hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(dY.p, ystd, 3 * n * sizeof(float), hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(dP.p, weights, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(dIdx.p, idx.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, st);
    (void)hipMemsetAsync(dL.p, 0, sizeof(double), st);
    mlp_zero(st, (float*)dG.p, MLP_NPARAM);
    float* wb = (float*)dW.p;
    MlpWork w{};
    float** parts[] = {&w.z1, &w.h1, &w.z2, &w.h2, &w.z3, &w.h3, &w.dz3, &w.dz2, &w.dz1};
    for (int i = 0; i < 9; i++) *parts[i] = wb + (int64_t)i * n * H;
    w.dout = wb + (int64_t)9 * n * H;
    mlp_fwd_bwd(st, w, (int)n, (int32_t*)dIdx.p, (float*)dX.p, (float*)dY.p, (float*)dP.p, (float*)dG.p,
                (double*)dL.p);
    (void)hipMemcpyAsync(loss, dL.p, sizeof(double), hipMemcpyDeviceToHost, st);
    (void)hipMemcpyAsync(grad, dG.p, MLP_NTRAIN * sizeof(float), hipMemcpyDeviceToHost, st);
    if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) {
        set_last_error("ep_mlp_loss_grad: kernel failure");
        return EP_ERR_DEVICE;
    }
    return EP_OK;
}

int ep_mlp_predict(const float* weights, int64_t n, const double* inputs, double tol, double* out3, double* errest,
                   int32_t* accepted, int32_t device) {
    if (n < 0 || (n > 0 && (!inputs || !out3)) || !(tol > 0)) {
        set_last_error("ep_mlp_predict: bad arguments");
        return EP_ERR_INVALID_ARG;
    }
    for (int64_t i = 0; i < n; i++)
        if (!(inputs[4 * i + 1] > 0) || !(inputs[4 * i + 3] > 0) || !std::isfinite(inputs[4 * i]) ||
            !std::isfinite(inputs[4 * i + 2])) {
            set_last_error("ep_mlp_predict: inputs must be finite with v_c > 0 and sigma > 0");
            return EP_ERR_INVALID_ARG;
        }
    if (n == 0) return EP_OK;
    if (hipSetDevice(device) != hipSuccess) { set_last_error("hipSetDevice failed"); return EP_ERR_DEVICE; }
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) { set_last_error("stream"); return EP_ERR_DEVICE; }
    struct SG {
        hipStream_t s;
        ~SG() { (void)hipStreamDestroy(s); }
    } sg{st};
    if (set_gauss_hermite(st) != hipSuccess) { set_last_error("quadrature table upload failed"); return EP_ERR_DEVICE; }
    std::vector<double> mu(n), v(n), A(n), s(n), zero(n, 0.0);
    for (int64_t i = 0; i < n; i++) {
        mu[i] = inputs[4 * i];
        v[i] = inputs[4 * i + 1];
        A[i] = inputs[4 * i + 2];
        s[i] = inputs[4 * i + 3];
    }
    DevBuf dmu, dv, dA, ds, dz, dP, dBf, dO, dE, dAc;
    if (!dalloc<double>(dmu, n) || !dalloc<double>(dv, n) || !dalloc<double>(dA, n) || !dalloc<double>(ds, n) ||
        !dalloc<double>(dz, n) || !dalloc<float>(dP, MLP_NPARAM) || !dalloc<short>(dBf, 2 * 128 * 128) ||
        !dalloc<double>(dO, 3 * n) || !dalloc<double>(dE, n) || !dalloc<int32_t>(dAc, n)) {
        set_last_error("ep_mlp_predict: allocation failed");
        return EP_ERR_OOM;
    }
    const size_t b = n * sizeof(double);
    (void)hipMemcpyAsync(dmu.p, mu.data(), b, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(dv.p, v.data(), b, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(dA.p, A.data(), b, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(ds.p, s.data(), b, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(dz.p, zero.data(), b, hipMemcpyHostToDevice, st);
    if (weights) {
        (void)hipMemcpyAsync(dP.p, weights, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, st);
        mlp_make_bf16(st, (float*)dP.p, (short*)dBf.p);
    }
    StarsDev S{};
    S.n = n;
    S.A = (double*)dA.p;
    S.sigma = (double*)ds.p;
    S.cav_mu = (double*)dmu.p;    // the q-marginal with zero sites is the cavity itself
    S.cav_var = (double*)dv.p;
    S.tau = (double*)dz.p;
    S.nu = (double*)dz.p;
    EpParams p{0, 1.0, 0.0};
    launch_mlp_tilted(st, S, p, weights ? (float*)dP.p : nullptr, (short*)dBf.p, tol, nullptr, nullptr,
                      (int32_t*)dAc.p, (double*)dE.p, (double*)dO.p);
    (void)hipMemcpyAsync(out3, dO.p, 3 * b, hipMemcpyDeviceToHost, st);
    if (errest) (void)hipMemcpyAsync(errest, dE.p, b, hipMemcpyDeviceToHost, st);
    if (accepted) (void)hipMemcpyAsync(accepted, dAc.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) {
        set_last_error("ep_mlp_predict: kernel failure");
        return EP_ERR_DEVICE;
    }
    return EP_OK;
}

}  // extern "C"
