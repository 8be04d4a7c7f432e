// Internal declarations of the surrogate-network kernels (tsne_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tsne {

// Workspace of the surrogate network for batches of up to Bpad rows.
struct MlpLayout {
  int d_in = 0, H = 0;
  int64_t Bpad = 0;
  size_t w1b = 0, w2b = 0, w2tb = 0, xb = 0, h1b = 0, h2 = 0, loss_part = 0;
  size_t xbt = 0, yb = 0, h1 = 0, h1t = 0, dout = 0, dh2 = 0, dh2b = 0, dh2t = 0, dh1 = 0,
         dh1t = 0, gw1 = 0, colpart = 0;
  size_t total = 0;
};

MlpLayout make_mlp_layout(int d_in, int H, int64_t Bpad, bool train);

// Size of the device-resident scratch of tsne_mlp_forward_noalloc, and its
// address on the current device (looked up on the first call per device).
constexpr size_t kNoAllocScratchBytes = 512 * 1024;
hipError_t noalloc_scratch(void **out);

hipError_t launch_mlp_forward(const MlpLayout &L, const float *params, const float *mean,
                              const float *invstd, const float *x, int64_t n, float *out, void *ws,
                              hipStream_t stream);
hipError_t launch_mlp_gradient(const MlpLayout &L, const float *params, const float *mean,
                               const float *invstd, const float *x, const float *y,
                               const int32_t *idx, int64_t B, float *grad, double *loss,
                               void *ws, hipStream_t stream);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr,
                       float beta1, float beta2, float eps, int32_t t, hipStream_t stream);

}  // namespace tsne
