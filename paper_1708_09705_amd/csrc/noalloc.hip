// ep_mlp_predict_noalloc: the gated surrogate moments of ep_mlp_predict for
// callers that cannot allocate device memory.  Inputs, weights and outputs
// are the caller's device buffers; everything else the kernels need (the
// BF16 copy of the two hidden layers, the per-tuple inputs split into one
// array per field, a zero site array and an error counter) lives in one
// file-scope device array, `scratch`, that each GPU holds for the life of the
// process.  Its device address is looked up once per device with
// hipGetSymbolAddress; host code uses only that address.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/ep.h"
#include "kernels.h"
#include "surrogate.h"

namespace ep {
void set_last_error(const std::string& m);   // api.cpp
}

namespace {

constexpr int64_t NMAX = EP_NOALLOC_MAX_TUPLES;
constexpr int HD = 128;
constexpr size_t HDR_D = 32;                                      // 256 B: the error counter
constexpr size_t BF_D = 2 * HD * HD * sizeof(short) / sizeof(double);   // BF16 W2 and W3
constexpr size_t SCRATCH_D = HDR_D + BF_D + 5 * (size_t)NMAX;       // mu, v, A, sigma, zero sites

__device__ __align__(256) double scratch[SCRATCH_D];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_scratch[MAX_DEVICES] = {};   // device address of `scratch`, per device

__global__ void k_na_clear(int32_t* count) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = 0;
}

// Split the n x 4 tuples into one array per field, zero the site arrays and
// count tuples that fail the argument checks of ep_mlp_predict.
__global__ void k_na_split(int64_t n, const double* __restrict__ in, double* mu, double* v, double* A, double* s,
                           double* zero, int32_t* bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a0 = in[4 * i], a1 = in[4 * i + 1], a2 = in[4 * i + 2], a3 = in[4 * i + 3];
    mu[i] = a0;
    v[i] = a1;
    A[i] = a2;
    s[i] = a3;
    zero[i] = 0.0;
    if (!(a1 > 0) || !(a3 > 0) || !isfinite(a0) || !isfinite(a2)) atomicAdd(bad, 1);
}

// Look the array up on the current device (once per device).
int scratch_for(int device, double** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            ep::set_last_error(std::string("ep_mlp_predict_noalloc: hipGetSymbolAddress failed: ") +
                               hipGetErrorString(e));
            return EP_ERR_DEVICE;
        }
        // the Gauss-Hermite tables of the gate are module constants: upload
        // them once per device as well
        hipStream_t null_stream = nullptr;
        if (ep::set_gauss_hermite(null_stream) != hipSuccess) {
            (void)hipGetLastError();
            ep::set_last_error("ep_mlp_predict_noalloc: quadrature table upload failed");
            return EP_ERR_DEVICE;
        }
        g_scratch[device] = (double*)p;
    }
    *out = g_scratch[device];
    return EP_OK;
}

}  // namespace

extern "C" int ep_mlp_predict_noalloc(const float* weights, int64_t n, const double* inputs, double tol,
                                      double* out3, double* errest, int32_t* accepted, int32_t device,
                                      void* stream) {
    if (n > NMAX) {
        char m[160];
        std::snprintf(m, sizeof m, "ep_mlp_predict_noalloc: n = %lld exceeds the maximum of %lld tuples per call",
                      (long long)n, (long long)NMAX);
        ep::set_last_error(m);
        return EP_ERR_INVALID_ARG;
    }
    if (n < 0 || (n > 0 && (!inputs || !out3)) || !(tol > 0)) {
        ep::set_last_error("ep_mlp_predict_noalloc: bad arguments");
        return EP_ERR_INVALID_ARG;
    }
    if (device < 0 || device >= MAX_DEVICES) {
        ep::set_last_error("ep_mlp_predict_noalloc: device ordinal out of range");
        return EP_ERR_INVALID_ARG;
    }
    if (n == 0) return EP_OK;
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        ep::set_last_error("ep_mlp_predict_noalloc: hipSetDevice failed");
        return EP_ERR_DEVICE;
    }
    double* base = nullptr;
    if (int rc = scratch_for(device, &base)) return rc;
    hipStream_t st = (hipStream_t)stream;
    int32_t* bad = (int32_t*)base;
    short* Wbf = (short*)(base + HDR_D);
    double* mu = base + HDR_D + BF_D;
    double* v = mu + NMAX;
    double* A = v + NMAX;
    double* s = A + NMAX;
    double* zero = s + NMAX;

    hipLaunchKernelGGL(k_na_clear, dim3(1), dim3(64), 0, st, bad);
    hipLaunchKernelGGL(k_na_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, inputs, mu, v, A, s,
                       zero, bad);
    int32_t nbad = 0;
    if (hipMemcpyAsync(&nbad, bad, sizeof nbad, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        ep::set_last_error("ep_mlp_predict_noalloc: input staging failed");
        return EP_ERR_DEVICE;
    }
    if (nbad) {
        ep::set_last_error("ep_mlp_predict_noalloc: inputs must be finite with v_c > 0 and sigma > 0");
        return EP_ERR_INVALID_ARG;
    }
    if (weights) ep::mlp_make_bf16(st, weights, Wbf);
    ep::StarsDev S{};
    S.n = n;
    S.A = A;
    S.sigma = s;
    S.cav_mu = mu;   // with zero sites the q-marginal is the cavity itself
    S.cav_var = v;
    S.tau = zero;
    S.nu = zero;
    ep::EpParams p{0, 1.0, 0.0};
    ep::launch_mlp_tilted(st, S, p, weights, Wbf, tol, nullptr, nullptr, accepted, errest, out3);
    if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) {
        ep::set_last_error("ep_mlp_predict_noalloc: kernel failure");
        return EP_ERR_DEVICE;
    }
    return EP_OK;
}
