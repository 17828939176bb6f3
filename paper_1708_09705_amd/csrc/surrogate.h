// Tilted-moment surrogate network: training and gated inference kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace ep {

constexpr int MLP_NPARAM = 34065;   // W1 b1 W2 b2 W3 b3 W4 b4 | x mean, x std, y mean, y std
constexpr int MLP_NTRAIN = 34051;   // the trainable prefix (weights and biases)

// activations of one batch (B x 128 each, dout B x 3)
struct MlpWork {
    float *z1, *h1, *z2, *h2, *z3, *h3, *dz3, *dz2, *dz1, *dout;
};

void mlp_fwd_bwd(hipStream_t st, const MlpWork& w, int B, const int32_t* idx, const float* X, const float* Y,
                 const float* P, float* G, double* loss);
void mlp_zero(hipStream_t st, float* p, int64_t n);
void mlp_adam(hipStream_t st, float* P, const float* G, float* m, float* v, float lr, int step);
void mlp_make_bf16(hipStream_t st, const float* P, short* Wbf);
hipError_t set_gauss_hermite(hipStream_t st);
// gated surrogate moments for every star; stars whose check fails are
// appended to fb_list.  With s.status == nullptr it only evaluates
// (out3 / errest / accepted may be null).
void launch_mlp_tilted(hipStream_t st, StarsDev s, EpParams p, const float* P, const short* Wbf, double tol,
                       int32_t* fb_list, int32_t* fb_count, int32_t* accepted, double* errest, double* out3);

}  // namespace ep
