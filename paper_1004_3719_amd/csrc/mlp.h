// The selector network's kernels (mlp.hip) and model object (selector.cpp).
#pragma once

#include "ffx_impl.h"

namespace ffx {

constexpr int MLP_NPARAM = 6662;
constexpr int MLP_NIN = 32;
constexpr int MLP_NOUT = 6;

hipError_t mlp_predict(const float* theta, const float* mean, const float* scale, const float* X, int64_t n, float* out,
                       hipStream_t st);
// gradient of the masked squared error over n samples; act (n * mlp_act_floats()), del
// (n * mlp_del_floats()) and sqerr (n) are workspace; *sse receives the sum of squared errors
hipError_t mlp_gradient(const float* theta, const float* mean, const float* scale, const float* X, const float* T,
                        const float* M, int64_t n, float* act, float* del, float* sqerr, float* grad, float* sse,
                        hipStream_t st);
hipError_t mlp_adam(float* theta, float* m, float* v, const float* g, float lr, int64_t t, hipStream_t st);
size_t mlp_act_floats();
size_t mlp_del_floats();

}  // namespace ffx
