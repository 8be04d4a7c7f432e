// Perplexity-adaptive kernel density estimate of a 2-D map (paKDE, section
// "Perplexity-adaptive Kernel Density Estimation"): every map point gets the
// precision beta_j of the same perplexity search as the input affinities, run
// on the map's squared distances; the density is the sample smoothing
// estimator with bivariate Gaussian kernels of bandwidth h_j^2 = 1 / beta_j,
//   f(c) = (S / n) sum_j (beta_j / pi) exp(-beta_j |c - y_j|^2),
// evaluated at the centres of a regular raster with cells of area S.
#include <hip/hip_runtime.h>
#include <math.h>

#include "../../include/tsne355.h"
#include "tsne_internal.h"

namespace {

constexpr int kKdeThreads = 256;
constexpr int kKdeCells = 4;  // cells per thread (consecutive along x)
constexpr double kLog2e = 1.4426950408889634074;
constexpr double kInvPi = 0.31830988618379067154;

// One thread: kKdeCells consecutive cells of one raster row. Points pass
// through LDS in chunks of 256 as {x, y, beta log2(e), beta / pi}; each cell
// sums a chunk in FP32 and the chunk sums in FP64.
__global__ __launch_bounds__(kKdeThreads) void k_kde_raster(const float2 *__restrict__ y,
                                                            const double *__restrict__ beta,
                                                            int64_t n, tsne_raster g,
                                                            float *__restrict__ out) {
  __shared__ float4 pts[kKdeThreads];
  const int64_t per_row = (g.gx + kKdeCells - 1) / kKdeCells;
  const int64_t slot = (int64_t)blockIdx.x * kKdeThreads + threadIdx.x;
  const int64_t v = slot / per_row, u0 = (slot - v * per_row) * kKdeCells;
  const bool live = v < g.gy;
  const float cy = g.y0 + ((float)v + 0.5f) * g.cy;
  float cx[kKdeCells];
#pragma unroll
  for (int k = 0; k < kKdeCells; ++k) cx[k] = g.x0 + ((float)(u0 + k) + 0.5f) * g.cx;
  double acc[kKdeCells] = {};
  for (int64_t j0 = 0; j0 < n; j0 += kKdeThreads) {
    __syncthreads();
    const int64_t j = j0 + threadIdx.x;
    if (j < n) {
      const float2 p = y[j];
      const double b = beta[j];
      pts[threadIdx.x] = make_float4(p.x, p.y, (float)(b * kLog2e), (float)(b * kInvPi));
    } else {
      pts[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);  // weight 0
    }
    __syncthreads();
    const int cnt = (int)((n - j0) < kKdeThreads ? (n - j0) : kKdeThreads);
    float s[kKdeCells] = {};
    for (int q = 0; q < cnt; ++q) {
      const float4 p = pts[q];
      const float dy = cy - p.y, dy2 = dy * dy;
#pragma unroll
      for (int k = 0; k < kKdeCells; ++k) {
        const float dx = cx[k] - p.x;
        const float r2 = fmaf(dx, dx, dy2);
        s[k] = fmaf(p.w, __builtin_amdgcn_exp2f(-p.z * r2), s[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < kKdeCells; ++k) acc[k] += (double)s[k];
  }
  if (!live) return;
  const double scale = (double)g.cx * (double)g.cy / (double)n;
#pragma unroll
  for (int k = 0; k < kKdeCells; ++k)
    if (u0 + k < g.gx) out[v * g.gx + u0 + k] = (float)(acc[k] * scale);
}

}  // namespace

namespace tsne {

hipError_t launch_kde_raster(const float *y, int64_t n, const double *beta, const tsne_raster &g,
                             float *out, hipStream_t st) {
  const int64_t slots = (int64_t)g.gy * ((g.gx + kKdeCells - 1) / kKdeCells);
  hipLaunchKernelGGL(k_kde_raster, dim3((unsigned)((slots + kKdeThreads - 1) / kKdeThreads)),
                     dim3(kKdeThreads), 0, st, reinterpret_cast<const float2 *>(y), beta, n, g,
                     out);
  return hipGetLastError();
}

}  // namespace tsne
