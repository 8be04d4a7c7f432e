// Input affinities P on the GPU (section "Similarities in the input space",
// Eqs. 1-3 of the bigMap paper):
//   1. centre X (distances are translation invariant) and form row norms;
//   2. per block of T rows: squared distances to all points on MFMA
//      (d_ij = |x_i|^2 + |x_j|^2 - 2 x_i.x_j), a per-row bracketed search on
//      the Gaussian precision beta_i so that the entropy of p_{.|i} equals
//      ln(perplexity), and a copy of the block's upper-triangle tiles into
//      the P store;
//   3. in place over the stored tiles: p_ij = (p_{j|i} + p_{i|j}) / (2n).
#include <float.h>
#include <math.h>

#include "tsne_internal.h"

namespace tsne {

namespace {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;
constexpr float kBig = 3.0e38f;  // stands for an excluded entry (self pair)

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline void flag_error(Hdr *h, uint32_t bit) { atomicOr(&h->err, bit); }

// Implicit P: the kernels of a pass run only on a workspace whose header
// records implicit affinities for the same n, d and distance mode (its layout,
// hence every offset these kernels use, depends on all three); key is
// implicit_key(d, mode).
__device__ inline bool implicit_ready(const Hdr *h, int64_t n, int32_t key) {
  return h->magic == kMagic && h->n == n && implicit_key(h->d, h->mode) == key && h->ready == 2;
}

// ----------------------------------------------------------------------------
// Wave / block reductions (fixed order, hence deterministic)
// ----------------------------------------------------------------------------
__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_min_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}

// ----------------------------------------------------------------------------
// 0. Header
// ----------------------------------------------------------------------------
__global__ void k_init_hdr(Hdr *h, int64_t n, int32_t d, int32_t mode, double perplexity) {
  if (threadIdx.x == 0) {
    h->magic = kMagic;
    h->n = n;
    h->d = d;
    h->ready = 0;
    h->err = 0;
    h->mode = mode;
    h->perplexity = perplexity;
    h->z = 0.0;
    h->c_p = 0.0;
    h->p_sum = 0.0;
    h->xmax = 0.f;
  }
}

// ----------------------------------------------------------------------------
// 1. Column means (FP64) and centred, transposed X with FP64 row norms
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_colmean(const float *__restrict__ x, int64_t n, int32_t d,
                                                 double *__restrict__ mean) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)x[i * d + k];
  s = wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) mean[k] = (red[0] + red[1] + red[2] + red[3]) / (double)n;
}

__global__ __launch_bounds__(256) void k_centre(const float *__restrict__ x, int64_t n, int32_t d,
                                                int64_t npad, int32_t dpad,
                                                const double *__restrict__ mean,
                                                double *__restrict__ xcT,
                                                double *__restrict__ norms, Hdr *h) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npad) return;
  double nrm = 0.0;
  bool bad = false;
  float amax = 0.f;
  for (int k = 0; k < dpad; ++k) {
    double v = 0.0;
    if (i < n && k < d) {
      float xv = x[i * d + k];
      bad |= !isfinite(xv);
      v = (double)xv - mean[k];
    }
    xcT[(int64_t)k * npad + i] = v;
    nrm += v * v;
    amax = fmaxf(amax, fabsf((float)v));
  }
  norms[i] = nrm;
  if (bad) flag_error(h, kErrNonFinite);
  // max |centred x| over the wave, then one atomic per wave (non-negative
  // floats order like their bit patterns)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  if ((threadIdx.x & 63) == 0 && isfinite(amax))
    atomicMax(reinterpret_cast<unsigned int *>(&h->xmax), __float_as_uint(amax));
}

// ----------------------------------------------------------------------------
// 2a. Distance block on FP64 MFMA: rows b*T .. b*T+T-1 against all columns.
//
// v_mfma_f64_16x16x4f64 computes a 16x16 block of A(16x4) B(4x16). Lane l
// supplies A[l%16][l/16] and B[l/16][l%16] and receives D[l/16 + 4r][l%16]
// in accumulator element r (rows interleaved by 4, unlike the FP32/BF16
// 16x16 variants, whose element r holds row 4(l/16) + r). X is stored transposed (k-major), so the 16
// lanes that share a k read 16 consecutive doubles. A wave computes a
// 64 x 16 kDistCT block (4 x kDistCT MFMA tiles, small enough for two waves
// per SIMD); a workgroup of 4 waves covers 64 rows x 64 kDistCT columns.
// ----------------------------------------------------------------------------
constexpr int kDistCT = 2;  // 16-column MFMA tiles per wave (a wave covers 64 x 16 kDistCT)
// the implicit tile kernel's width: two 16-column tiles per wave, so that a
// lane's two columns are neighbours in the tile layout
constexpr int kTileCT = 2;

// With P given, the block row's tiles (J >= b) also go straight to their
// place in the packed buffer, in the layout k_stage writes, as in k_dist_x3:
// for each of its rows a lane holds columns cl + li and cl + 16 + li of the
// tile (cl = 128 h + 32 w, h the half of the tile this workgroup covers),
// the two consecutive elements 2 (w mod 2) and 2 (w mod 2) + 1 of one float4
// there. The column strips are rotated so that the diagonal tile's are
// dispatched first.
static_assert(kDistCT == 2, "the packed stores assume 32 columns per wave");
__global__ __launch_bounds__(256) void k_dist_f64(const double *__restrict__ xcT,
                                                  const double *__restrict__ norms, int64_t npad,
                                                  int32_t dpad, int32_t b,
                                                  float *__restrict__ dblock,
                                                  float4 *__restrict__ P, int32_t nb) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int xs = (int)((blockIdx.x + 2u * (unsigned)b) % gridDim.x);  // column strip
  const int J = xs >> 1, cl = 128 * (xs & 1) + 32 * w;
  const int64_t col0 = (int64_t)xs * (64 * kDistCT) + w * (16 * kDistCT);
  const int row0_loc = blockIdx.y * 64;
  const int64_t row0 = (int64_t)b * T + row0_loc;
  const int li = l & 15, lk = l >> 4;
  v4d acc[4][kDistCT];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < kDistCT; ++c) acc[a][c] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < dpad; k0 += 4) {
    const double *xk = xcT + (int64_t)(k0 + lk) * npad;
    double av[4], bv[kDistCT];
#pragma unroll
    for (int a = 0; a < 4; ++a) av[a] = xk[row0 + a * 16 + li];
#pragma unroll
    for (int c = 0; c < kDistCT; ++c) bv[c] = xk[col0 + c * 16 + li];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < kDistCT; ++c)
        acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[a][c], 0, 0, 0);
  }
  // every norm is loaded before the first store, so no store waits on a load
  double ni[4][4], nj[kDistCT];
#pragma unroll
  for (int c = 0; c < kDistCT; ++c) nj[c] = norms[col0 + c * 16 + li];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) ni[a][r] = norms[(int64_t)b * T + row0_loc + a * 16 + lk + 4 * r];
  float *pt = (P != nullptr && J > b)
                  ? reinterpret_cast<float *>(P + (size_t)(tile_start(b, nb) + (J - b)) * TT4)
                  : nullptr;
  float *pd = (P != nullptr && J == b) ? reinterpret_cast<float *>(P + (size_t)tile_start(b, nb) * TT4)
                                       : nullptr;
  auto packed = [](int i, int j) {  // float of (row i, column j) of a tile
    return 4 * ((4 * (i >> 4) + (j >> 6)) * 256 + 16 * (i & 15) + (j & 15)) + ((j >> 4) & 3);
  };
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int il = row0_loc + a * 16 + lk + 4 * r;
      float v[kDistCT];
#pragma unroll
      for (int c = 0; c < kDistCT; ++c) {
        const int64_t j = col0 + c * 16 + li;
        double dd = ni[a][r] + nj[c] - 2.0 * acc[a][c][r];
        v[c] = (float)fmax(dd, 0.0);
        dblock[(int64_t)il * npad + j] = v[c];
      }
      if (pt) {
        *reinterpret_cast<float2 *>(pt + packed(il, cl + li)) = make_float2(v[0], v[1]);
      } else if (pd) {
#pragma unroll
        for (int c = 0; c < kDistCT; ++c) {
          const int jl = cl + 16 * c + li;  // column within the tile
          if (jl >= il) {
            pd[packed(il, jl)] = v[c];
            if (jl > il) pd[packed(jl, il)] = v[c];
          }
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// 2a'. Reduced-precision distance contraction (the precision path).
//
// FP32 mode: the FP64-centred X rounded to FP32, v_mfma_f32_16x16x4f32, norms
// of the rounded points, d = (n_i + n_j) - 2 x.y in FP32.
// BF16 / FP16 modes: operands rounded to 16 bits, v_mfma_f32_16x16x32_{bf16,f16}
// with FP32 accumulation, and the norms of the rounded operands, so that d is
// the exact squared distance of two slightly moved points (never negative, no
// cancellation blow-up of the dot-product error). FP16 operands are scaled by
// a power of two so that max |x| maps to <= 256 (exact, undone after the
// contraction).
// These three keep the cancellation of |x|^2 + |y|^2 - 2 x.y: near pairs
// have d ~ 200 against |x|^2 ~ 1,350 on the benchmark data, so an FP32
// rounding of the large terms moves d by ~1e-4. The x3 modes (2a'' below)
// remove it.
// 16x16x32 layout: lane l supplies A[l%16][8(l/16) .. 8(l/16)+7] and the
// matching B column slice, and receives D[4(l/16) + r][l%16] in element r.
// ----------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

__device__ inline float fp16_scale(const Hdr *h) {
  // 2^(8 - ceil(log2 xmax)); 1 if xmax is 0
  const float xm = h->xmax;
  if (!(xm > 0.f)) return 1.f;
  int e;
  frexpf(xm, &e);  // xm = f 2^e, f in [0.5, 1)
  return ldexpf(1.f, 8 - e);
}

__global__ __launch_bounds__(256) void k_prep_f32(const double *__restrict__ xcT, int64_t npad,
                                                  int32_t dpad, float *__restrict__ xfT,
                                                  float *__restrict__ norms32) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npad) return;
  double nrm = 0.0;
  for (int k = 0; k < dpad; ++k) {
    const float v = (float)xcT[(int64_t)k * npad + i];
    xfT[(int64_t)k * npad + i] = v;
    nrm += (double)v * (double)v;
  }
  norms32[i] = (float)nrm;
}

template <typename H, bool SCALE>
__global__ __launch_bounds__(256) void k_prep_lp(const double *__restrict__ xcT, int64_t npad,
                                                 int32_t d, int32_t k32, H *__restrict__ xa,
                                                 float *__restrict__ norms32, const Hdr *h) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npad) return;
  const float s = SCALE ? fp16_scale(h) : 1.f;
  H *ra = xa + i * k32;
  double nrm = 0.0;
  for (int k = 0; k < k32; ++k) {
    const float v = (k < d) ? (float)xcT[(int64_t)k * npad + i] : 0.f;
    const H hi = (H)(v * s);
    ra[k] = hi;
    const double hv = (double)(float)hi / (double)s;
    nrm += hv * hv;
  }
  norms32[i] = (float)nrm;
}

__global__ __launch_bounds__(256) void k_dist_f32(const float *__restrict__ xfT,
                                                  const float *__restrict__ norms, int64_t npad,
                                                  int32_t dpad, int32_t b,
                                                  float *__restrict__ dblock) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t col0 = (int64_t)blockIdx.x * 256 + w * 64;
  const int row0_loc = blockIdx.y * 64;
  const int64_t row0 = (int64_t)b * T + row0_loc;
  const int li = l & 15, lk = l >> 4;
  v4f acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < dpad; k0 += 4) {
    const float *xk = xfT + (int64_t)(k0 + lk) * npad;
    float av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) av[a] = xk[row0 + a * 16 + li];
#pragma unroll
    for (int c = 0; c < 4; ++c) bv[c] = xk[col0 + c * 16 + li];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[c], acc[a][c], 0, 0, 0);
  }
  // every norm is loaded before the first store, so no store waits on a load
  float ni[4][4], nj[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) nj[c] = norms[col0 + c * 16 + li];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) ni[a][r] = norms[(int64_t)b * T + row0_loc + a * 16 + 4 * lk + r];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int il = row0_loc + a * 16 + 4 * lk + r;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t j = col0 + c * 16 + li;
        const float dd = (ni[a][r] + nj[c]) - 2.f * acc[a][c][r];
        dblock[(int64_t)il * npad + j] = fmaxf(dd, 0.f);
      }
    }
  }
}

template <typename H, typename V8, bool SCALE>
__global__ __launch_bounds__(256) void k_dist_lp(const H *__restrict__ xa,
                                                 const float *__restrict__ norms, int64_t npad,
                                                 int32_t kk, int32_t b, float *__restrict__ dblock,
                                                 const Hdr *h) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t col0 = (int64_t)blockIdx.x * 256 + w * 64;
  const int row0_loc = blockIdx.y * 64;
  const int64_t row0 = (int64_t)b * T + row0_loc;
  const int li = l & 15, lk = l >> 4;
  float inv_s2 = 1.f;
  if (SCALE) {
    const float s = fp16_scale(h);
    inv_s2 = 1.f / (s * s);
  }
  v4f acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < kk; k0 += 32) {
    V8 av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      av[a] = *reinterpret_cast<const V8 *>(xa + (row0 + a * 16 + li) * kk + k0 + 8 * lk);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      bv[c] = *reinterpret_cast<const V8 *>(xa + (col0 + c * 16 + li) * kk + k0 + 8 * lk);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if constexpr (sizeof(H) == 2 && __is_same(H, __bf16))
          acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[c], acc[a][c], 0, 0, 0);
        else
          acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[a], bv[c], acc[a][c], 0, 0, 0);
      }
  }
  // every norm is loaded before the first store, so no store waits on a load
  float ni[4][4], nj[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) nj[c] = norms[col0 + c * 16 + li];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) ni[a][r] = norms[(int64_t)b * T + row0_loc + a * 16 + 4 * lk + r];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int il = row0_loc + a * 16 + 4 * lk + r;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t j = col0 + c * 16 + li;
        const float dd = (ni[a][r] + nj[c]) - 2.f * (acc[a][c][r] * inv_s2);
        dblock[(int64_t)il * npad + j] = fmaxf(dd, 0.f);
      }
    }
  }
}

// ----------------------------------------------------------------------------
// 2a''. The x3 modes: exact-accumulate slices and a compensated FP32 combine.
//
// Every centred coordinate is cut on one grid for the whole data set,
//   x = sigma (h1 + 2^-b h2 + 2^-2b h3) + r,  sigma = 2^(E - b), max |x| < 2^E,
// rounding to the nearest integer at each level (|h1| <= 2^b, |h2|, |h3| <=
// 2^(b-1), |r| <= sigma 2^(-2b-1)). b is the largest value with
// 2b + log2(K) <= 24 (K = d rounded up to 32), at most 10 for FP16 and 8 for
// BF16, so each slice is exact in 16 bits and
//   A0 = sum_k h1 h1'
// is an integer below 2^24: the MFMA's FP32 accumulation adds it exactly, in
// whatever order it works. The rest of the contraction, scaled by 2^b,
//   R = sum_k (h1 h2' + h2 h1') + 2^-b (h1 h3' + h2 h2' + h3 h1')
//       + 2^-2b (h2 h3' + h3 h2'),
// is 2^-b smaller and is allowed to round. Its operands are stored as four
// slices per point, [h1 | h2 | 2^-b h2 | 2^-b h3] (all normal numbers in
// both formats), so R takes seven MFMA products and A0 one. Then
//   x.y = sigma^2 (A0 + 2^-b R);
// the product left out (h3 h3') is below sigma^2 2^-4b K 2^2b.
// The norms are FP32 pairs (hi, lo) of the FP64 norm of the represented point
// sigma (h1 + 2^-b h2 + 2^-2b h3). d = n_i + n_j - 2 x.y cancels most of its
// operands, so it is formed with error-free transformations: TwoSum of the
// two hi parts, the exact difference of that sum and 2 sigma^2 A0, then the
// small terms (the TwoSum error, the lo parts and 2 sigma^2 2^-b R) added to
// the leading difference. d then carries about one FP32 rounding of d
// itself instead of one of |x|^2.
// Operand layout: per point, per block of 32 values of k, the four slices'
// 32 values in a row ([point][k / 32][slice][32]), so that the four
// fragments a lane loads for one MFMA step sit in one 256-byte segment.
// ----------------------------------------------------------------------------
__host__ __device__ inline int x3_bits(int32_t k32, bool bf16) {
  int lk = 0;
  while ((1 << lk) < k32) ++lk;
  const int b = (24 - lk) / 2;
  const int bmax = bf16 ? 8 : 10;
  return b < bmax ? b : bmax;
}

// E with max |x| < 2^E (0 for an all-zero input)
__device__ inline int x3_exp(const Hdr *h) {
  const float xm = h->xmax;
  if (!(xm > 0.f)) return 0;
  int e;
  frexpf(xm, &e);
  return e;
}

template <typename H>
__global__ __launch_bounds__(256) void k_prep_x3(const double *__restrict__ xcT, int64_t npad,
                                                 int32_t d, int32_t k32, int32_t b,
                                                 H *__restrict__ xs, float2 *__restrict__ nhl,
                                                 const Hdr *h) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npad) return;
  const int E = x3_exp(h);
  H *row = xs + i * (4 * (int64_t)k32);
  double nrm = 0.0;
  for (int k = 0; k < k32; ++k) {
    const double v = (k < d) ? xcT[(int64_t)k * npad + i] : 0.0;
    const double q = ldexp(v, b - E);
    const double h1 = rint(q);
    double r = ldexp(q - h1, b);
    const double h2 = rint(r);
    r = ldexp(r - h2, b);
    const double h3 = rint(r);
    H *blk = row + (k >> 5) * 128 + (k & 31);
    blk[0] = (H)(float)h1;
    blk[32] = (H)(float)h2;
    blk[64] = (H)(float)ldexp(h2, -b);
    blk[96] = (H)(float)ldexp(h3, -b);
    const double xr = ldexp(h1 + ldexp(h2 + ldexp(h3, -b), -b), E - b);
    nrm += xr * xr;
  }
  const float hi = (float)nrm;
  nhl[i] = make_float2(hi, (float)(nrm - (double)hi));
}

template <typename H, typename V8>
__device__ __forceinline__ v4f mfma16x32(V8 a, V8 b, v4f c) {
  if constexpr (__is_same(H, __bf16))
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// The two sums A0 and R of a 64 x 64 block (4 x 4 MFMA tiles): rows ra .. ra+63
// against columns cb .. cb+63. Stored and recomputed P call this same routine,
// so their sums agree bit for bit.
template <typename H, typename V8>
__device__ __forceinline__ void x3_contract(const H *__restrict__ xs, int32_t k32, int64_t ra,
                                            int64_t cb, int li, int lk, v4f (&A0)[4][4],
                                            v4f (&R)[4][4]) {
  const int64_t kk = 4 * (int64_t)k32;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      A0[t][c] = (v4f){0.f, 0.f, 0.f, 0.f};
      R[t][c] = A0[t][c];
    }
  for (int k0 = 0; k0 < k32; k0 += 32) {
    const int64_t off = (int64_t)(k0 >> 5) * 128 + 8 * lk;
    V8 a[4][4];  // [slice][row tile]: h1, h2, 2^-b h2, 2^-b h3
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        a[q][t] = *reinterpret_cast<const V8 *>(xs + (ra + 16 * t + li) * kk + off + 32 * q);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      V8 bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        bv[q] = *reinterpret_cast<const V8 *>(xs + (cb + 16 * c + li) * kk + off + 32 * q);
#pragma unroll
      for (int t = 0; t < 4; ++t) A0[t][c] = mfma16x32<H, V8>(a[0][t], bv[0], A0[t][c]);
#pragma unroll
      for (int t = 0; t < 4; ++t) R[t][c] = mfma16x32<H, V8>(a[0][t], bv[1], R[t][c]);
#pragma unroll
      for (int t = 0; t < 4; ++t) R[t][c] = mfma16x32<H, V8>(a[1][t], bv[0], R[t][c]);
#pragma unroll
      for (int t = 0; t < 4; ++t) R[t][c] = mfma16x32<H, V8>(a[0][t], bv[3], R[t][c]);
#pragma unroll
      for (int t = 0; t < 4; ++t) R[t][c] = mfma16x32<H, V8>(a[1][t], bv[2], R[t][c]);
#pragma unroll
      for (int t = 0; t < 4; ++t) R[t][c] = mfma16x32<H, V8>(a[3][t], bv[0], R[t][c]);
#pragma unroll
      for (int t = 0; t < 4; ++t) R[t][c] = mfma16x32<H, V8>(a[2][t], bv[3], R[t][c]);
#pragma unroll
      for (int t = 0; t < 4; ++t) R[t][c] = mfma16x32<H, V8>(a[3][t], bv[2], R[t][c]);
    }
  }
}

// 2 sigma^2 and 2 sigma^2 2^-b
struct X3Scale {
  float s0, s1;
};
__device__ inline X3Scale x3_scale(const Hdr *h, int b) {
  const int e = 2 * (x3_exp(h) - b) + 1;
  return X3Scale{ldexpf(1.f, e), ldexpf(1.f, e - b)};
}

// d = n_i + n_j - 2 x.y from (hi, lo) norms and the two sums. The sum of the
// hi parts is taken with TwoSum (its rounding error e is kept); the leading
// difference t = s - 2 sigma^2 A0 needs no correction: the product is exact,
// and where the operands cancel (2 sigma^2 A0 >= s / 2, i.e. d below about
// s / 2) the subtraction is exact by Sterbenz's lemma, while elsewhere its
// rounding is below one FP32 ulp of d itself.
__device__ __forceinline__ float x3_combine(float2 ni, float2 nj, float a0, float r,
                                            const X3Scale &sc) {
  const float s = __fadd_rn(ni.x, nj.x);
  const float bs = __fsub_rn(s, ni.x);
  const float e = __fadd_rn(__fsub_rn(ni.x, __fsub_rn(s, bs)), __fsub_rn(nj.x, bs));
  const float t = __fsub_rn(s, __fmul_rn(sc.s0, a0));  // a0: an integer below 2^24
  const float low = __fsub_rn(__fadd_rn(e, __fadd_rn(ni.y, nj.y)), __fmul_rn(sc.s1, r));
  return fmaxf(__fadd_rn(t, low), 0.f);
}

// Distance block of the x3 modes: a workgroup covers 64 rows x 256 columns,
// as k_dist_lp. With P given, the block row's tiles (J >= b) also go
// straight to their place in the packed buffer, in the layout k_stage
// writes, so that no staging pass follows: lane (li, lk) of wave w holds,
// for each of its rows tr + 16 k of a tile, columns li + 16 (4 w + c),
// c = 0 .. 3, which is the float4 4 k + w of thread 16 tr + li there.
template <typename H, typename V8>
__global__ __launch_bounds__(256, 2) void k_dist_x3(const H *__restrict__ xs,
                                                 const float2 *__restrict__ nhl, int64_t npad,
                                                 int32_t k32, int32_t bits, int32_t b,
                                                 float *__restrict__ dblock, const Hdr *h,
                                                 float4 *__restrict__ P, int32_t nb) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  // column tile, rotated so that the diagonal one (the workgroups with the
  // most stores) is dispatched first
  const int J = (int)((blockIdx.x + (unsigned)b) % gridDim.x);
  const int64_t col0 = (int64_t)J * 256 + w * 64;
  const int row0_loc = blockIdx.y * 64;
  const int64_t row0 = (int64_t)b * T + row0_loc;
  const int li = l & 15, lk = l >> 4;
  v4f A0[4][4], R[4][4];
  x3_contract<H, V8>(xs, k32, row0, col0, li, lk, A0, R);
  const X3Scale sc = x3_scale(h, bits);
  // every norm is loaded before the first store, so no store waits on a load
  float2 nj[4], ni[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) nj[c] = nhl[col0 + c * 16 + li];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) ni[t][r] = nhl[(int64_t)b * T + row0_loc + t * 16 + 4 * lk + r];
  float4 *pt = (P != nullptr && J > b) ? P + (size_t)(tile_start(b, nb) + (J - b)) * TT4 : nullptr;
  // the diagonal tile is symmetrised as k_stage does it: each value of the
  // upper triangle (diagonal included) goes to its own place and to the
  // mirrored one, one float at a time
  float *pd = (P != nullptr && J == b) ? reinterpret_cast<float *>(P + (size_t)tile_start(b, nb) * TT4)
                                       : nullptr;
  // float of (row i, column j) of a tile in that layout
  auto packed = [](int i, int j) {
    return 4 * ((4 * (i >> 4) + (j >> 6)) * 256 + 16 * (i & 15) + (j & 15)) + ((j >> 4) & 3);
  };
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int il = row0_loc + t * 16 + 4 * lk + r;
      float v[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t j = col0 + c * 16 + li;
        v[c] = x3_combine(ni[t][r], nj[c], A0[t][c][r], R[t][c][r], sc);
        dblock[(int64_t)il * npad + j] = v[c];
      }
      if (pt) {
        pt[((il >> 4) * 4 + w) * 256 + 16 * (il & 15) + li] = make_float4(v[0], v[1], v[2], v[3]);
      } else if (pd) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int jl = 64 * w + 16 * c + li;  // column within the tile
          if (jl >= il) {
            pd[packed(il, jl)] = v[c];
            if (jl > il) pd[packed(jl, il)] = v[c];
          }
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// 2b. Per-row search for beta (Eqs. 1-2).
//
// One workgroup of 1024 threads per row, one launch for the rows of a group
// of consecutive row blocks (their distances side by side in the scratch;
// b is the group's first block), so that rows needing more passes than
// others are spread over the compute units instead of setting the length of
// every block's launch. The row's distances, shifted by the row minimum m,
// are held in registers (VPT per thread) when they fit, else re-read from
// the scratch on every pass. Each pass forms, with FP32
// exponentials and FP32 per-thread partial sums combined in FP64,
//   S = sum_j exp(-beta (d_j - m)),  T = sum_j (d_j - m) exp(-beta (d_j - m)),
//   Q = sum_j (d_j - m)^2 exp(-beta (d_j - m)),
//   H = ln S + beta T / S,  dH/dbeta = -beta (Q / S - (T / S)^2),
// where beta is the FP32-rounded precision actually applied. The paper
// leaves the search to a supplement it does not include; H decreases in
// beta, so any bracketed search that reaches the tolerance finds the same
// root. Bracket logic: start with [0, inf) at the beta of the same position
// in the row block before the group (a nearby point in the locality order;
// 1 for the first group); each pass moves one end of the bracket to beta, then takes
// the Newton step if it lands inside the bracket, else doubles beta (no
// upper end yet) or bisects. Stops at |H - ln u| <= tol_h, at a bracket
// narrower than FP32 resolution, or after max_bisect passes (then the row is
// flagged as not converged).
// The per-wave FP64 partial sums meet in LDS (double-buffered by pass
// parity); every wave then reduces them in the same fixed order and takes
// the same step, so one barrier per pass suffices and no thread waits for
// another's serial arithmetic.
// ----------------------------------------------------------------------------
constexpr int kCalThreads = 1024;

struct CalOut {
  double *beta, *S, *H;
  float *m, *a, *r;
  int32_t *evals;
};

// sum over the 16 lanes of each DPP row group, the same in every lane of the
// group (xor butterfly of exactly commutative additions)
__device__ inline double sum16_d(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int VPT>
__global__ __launch_bounds__(kCalThreads) void k_calibrate(const float *__restrict__ dblock,
                                                           int64_t n, int64_t npad, int32_t b,
                                                           double logu, int max_bisect,
                                                           double tol_h, CalOut out, Hdr *h) {
  constexpr int NW = kCalThreads / 64;
  static_assert(NW == 16, "one partial per lane of a 16-lane group");
  __shared__ double sred[2][3][NW];
  __shared__ float smin[NW];
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const int64_t i = (int64_t)b * T + blockIdx.x;
  if (i >= n) return;
  const float *row = dblock + (int64_t)blockIdx.x * npad;

  // row minimum over j != i, j < n
  float mn = INFINITY;
  float v[VPT > 0 ? VPT : 1];
  if constexpr (VPT > 0) {
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      int64_t j = (int64_t)q * kCalThreads + tid;
      float dv = (j < n && j != i) ? row[j] : INFINITY;
      v[q] = dv;
      mn = fminf(mn, dv);
    }
  } else {
    for (int64_t j = tid; j < n; j += kCalThreads)
      if (j != i) mn = fminf(mn, row[j]);
  }
  mn = wave_min_f(mn);
  if (ln == 0) smin[wv] = mn;
  __syncthreads();
  float m = smin[0];
#pragma unroll
  for (int q = 1; q < NW; ++q) m = fminf(m, smin[q]);
  if constexpr (VPT > 0) {
#pragma unroll
    for (int q = 0; q < VPT; ++q) v[q] = (v[q] == INFINITY) ? kBig : v[q] - m;
  }

  double beta = 1.0;
  if (b > 0) {
    const double bp = out.beta[(int64_t)(b - 1) * T + (blockIdx.x & (T - 1))];
    if (bp > 0.0 && isfinite(bp)) beta = bp;
  }
  double lo = 0.0, hi = INFINITY, S = 0.0, H = 0.0;
  float a = 0.f;
  int it = 0, done = 0;
  for (;;) {
    ++it;
    a = fmaxf((float)(beta * kLog2e), 1e-30f);
    float s0 = 0.f, s1 = 0.f, t0 = 0.f, t1 = 0.f, q0 = 0.f, q1 = 0.f;
    if constexpr (VPT > 0) {
#pragma unroll
      for (int q = 0; q < VPT; q += 2) {
        const float e0 = __builtin_amdgcn_exp2f(-a * v[q]);
        const float ve0 = v[q] * e0;  // 0 for an excluded entry (e = 0)
        s0 += e0;
        t0 += ve0;
        q0 = fmaf(v[q], ve0, q0);
        if (q + 1 < VPT) {
          const float e1 = __builtin_amdgcn_exp2f(-a * v[q + 1]);
          const float ve1 = v[q + 1] * e1;
          s1 += e1;
          t1 += ve1;
          q1 = fmaf(v[q + 1], ve1, q1);
        }
      }
    } else {
      for (int64_t j = tid; j < n; j += kCalThreads) {
        const float dm = (j == i) ? kBig : row[j] - m;
        const float e = __builtin_amdgcn_exp2f(-a * dm);
        const float ve = dm * e;
        s0 += e;
        t0 += ve;
        q0 = fmaf(dm, ve, q0);
      }
    }
    const int par = it & 1;
    const double ds = wave_sum_d((double)(s0 + s1)), dt = wave_sum_d((double)(t0 + t1)),
                 dq = wave_sum_d((double)(q0 + q1));
    if (ln == 0) {
      sred[par][0][wv] = ds;
      sred[par][1][wv] = dt;
      sred[par][2][wv] = dq;
    }
    __syncthreads();
    // every wave: the 16 wave partials, summed in one fixed order
    const int k16 = ln & 15;
    const double SS = sum16_d(sred[par][0][k16]), TT = sum16_d(sred[par][1][k16]),
                 QQ = sum16_d(sred[par][2][k16]);
    const double beff = (double)a * kLn2;
    S = SS;
    const double mean = TT / SS;
    H = log(SS) + beff * mean;
    if (fabs(H - logu) <= tol_h) {
      done = 1;
    } else if (isfinite(hi) && (hi - lo) <= hi * 0x1p-24) {
      done = 1;
    } else if (it >= max_bisect) {
      done = 2;
    } else {
      // H falls with beta (dH/dbeta = -beta Var(d)): shrink the bracket of
      // FP64 iterates, then take the Newton step if it lands inside it,
      // else bisect (H was taken at beff, within 2^-24 of beta)
      if (H > logu)
        lo = beta;
      else
        hi = beta;
      const double var = QQ / SS - mean * mean;
      const double nb = beta + (H - logu) / (beff * var);
      if (var > 0.0 && nb > lo && nb < hi && isfinite(nb))
        beta = nb;
      else
        beta = isinf(hi) ? 2.0 * beta : 0.5 * (lo + hi);
    }
    if (done) break;
  }
  if (tid == 0) {
    const double beff = (double)a * kLn2;
    const bool ok = (done == 1);
    out.beta[i] = beff;
    out.S[i] = S;
    out.H[i] = H;
    out.m[i] = m;
    out.a[i] = a;
    out.r[i] = (float)(1.0 / (2.0 * (double)n * S));
    out.evals[i] = ok ? it : -it;
    if (!ok) flag_error(h, kErrNoConv);
    if (!isfinite(H) || !isfinite(S)) flag_error(h, kErrNonFinite);
  }
}

// ----------------------------------------------------------------------------
// 2c. Copy the block's tiles (b, J >= b) into the P store in consumer order.
// The diagonal tile holds both orders of each pair; both take the distance
// of the upper element so that the stored P is exactly symmetric.
// ----------------------------------------------------------------------------
// Grid (nb - b, kStageSplit).
constexpr int kStageSplit = 4;
__global__ __launch_bounds__(256) void k_stage(const float *__restrict__ dblock, int64_t npad,
                                               int32_t nb, int32_t b, float4 *__restrict__ P) {
  const int J = b + blockIdx.x;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int tc = l & 15, tr = (l >> 4) + 4 * w;
  float4 *dst = P + (size_t)tile_start(b, nb) * TT4 + (size_t)blockIdx.x * TT4;
  const float *src = dblock + (int64_t)J * T;
  // workgroup y of the tile copies float4 rows s0 .. s1 - 1 of its 64
  const int s0 = blockIdx.y * (64 / kStageSplit), s1 = s0 + 64 / kStageSplit;
  if (J != b) {
#pragma unroll 4
    for (int s = s0; s < s1; ++s) {
      const int k = s >> 2, mq = s & 3;
      const float *rp = src + (int64_t)(tr + 16 * k) * npad + tc + 64 * mq;
      dst[s * 256 + t] = make_float4(rp[0], rp[16], rp[32], rp[48]);
    }
  } else {
    for (int s = s0; s < s1; ++s) {
      const int k = s >> 2, mq = s & 3;
      const int il = tr + 16 * k;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int jl = tc + 16 * (4 * mq + e);
        const int lo = il < jl ? il : jl, hi = il < jl ? jl : il;
        v[e] = src[(int64_t)lo * npad + hi];
      }
      dst[s * 256 + t] = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
}

// ----------------------------------------------------------------------------
// 2d. Implicit P: distances straight into the tile buffer. One launch covers
// the tiles tile0 .. tile0 + gridDim.x - 1 (whole block rows) and writes each
// tile's distances in the layout k_stage produces (float4 s * 256 + t of a
// tile holds rows tr + 16 (s / 4), columns tc + 64 (s % 4) + 16 e), so the
// pack and force kernels read them as before. The contraction of an element
// is the one the per-block-row kernels form for it (same operands, same
// MFMA sequence); a diagonal tile takes the upper element for both orders of
// a pair, as k_stage does, so P stays bitwise symmetric and bitwise that of
// the stored path. skip: the zero tiles are known and are left alone.
// ----------------------------------------------------------------------------
// p_ij of Eq. 3 from the distance and both rows' statistics (a = beta
// log2(e), m = row minimum, r = 1 / (2 n S)). No contraction into an FMA, so
// that the two orders of a pair give bitwise equal sums.
__device__ __forceinline__ float pair_p(float d, float ai, float mi, float ri, float aj, float mj,
                                        float rj) {
#pragma clang fp contract(off)
  const float pi = __builtin_amdgcn_exp2f(-ai * (d - mi)) * ri;
  const float pj = __builtin_amdgcn_exp2f(-aj * (d - mj)) * rj;
  return pi + pj;
}

__device__ __forceinline__ int64_t tile_pos(int il, int jl) {
  const int tr = il & 15, k = il >> 4, tc = jl & 15, mq = jl >> 6, e = (jl >> 4) & 3;
  const int t = 64 * (tr >> 2) + 16 * (tr & 3) + tc;
  return ((int64_t)(4 * k + mq) * 256 + t) * 4 + e;
}

__device__ __forceinline__ void put_d(float *__restrict__ tp, bool diag, int il, int jl,
                                      float v) {
  if (!diag) {
    tp[tile_pos(il, jl)] = v;
  } else if (il < jl) {
    tp[tile_pos(il, jl)] = v;
    tp[tile_pos(jl, il)] = v;
  } else if (il == jl) {
    tp[tile_pos(il, il)] = v;
  }
}

// Statistics (a, m, r) of one point for the PACK epilogue; ok = false for a
// padding point (its pairs are stored as 0).
struct PtStat {
  float a, m, r;
  bool ok;
};

template <bool PACK>
__device__ __forceinline__ PtStat pt_stat(int64_t g, int64_t n, const float *__restrict__ a,
                                          const float *__restrict__ m,
                                          const float *__restrict__ r) {
  PtStat p{0.f, 0.f, 0.f, false};
  if (PACK && g < n) p = PtStat{a[g], m[g], r[g], true};
  return p;
}

// The stored value of one element: the distance, or with PACK its p_ij (the
// packed value k_pack would write: zero on the diagonal, for padding points
// and below FP32's normal range).
template <bool PACK>
__device__ __forceinline__ float tile_value(float d, bool diag, int il, int jl, const PtStat &si,
                                            const PtStat &sj) {
  if (!PACK) return d;
  if ((diag && il == jl) || !si.ok || !sj.ok) return 0.f;
  const float v = pair_p(d, si.a, si.m, si.r, sj.a, sj.m, sj.r);
  return v < FLT_MIN ? 0.f : v;
}

// Common start: header check (a workspace prepared for another n, d or mode
// is flagged and left alone), zero-tile skip, tile coordinates. Returns false
// if the workgroup has nothing to do.
__device__ __forceinline__ bool tdist_begin(const Hdr *guard, int64_t gn, int32_t gkey,
                                            const uint8_t *__restrict__ nz, bool skip,
                                            int64_t tile, int32_t nb, int &I, int &J) {
  if (!implicit_ready(guard, gn, gkey)) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
      flag_error(const_cast<Hdr *>(guard), kErrState);
    return false;
  }
  if (skip && !nz[tile]) return false;
  tile_coords(tile, nb, I, J);
  return true;
}

// FP64 mode: a workgroup covers 64 rows x 128 columns of a tile (grid y: 4
// row groups x 2 column groups), as k_dist_f64. a, m, r: the row statistics
// (read with PACK only).
template <bool PACK>
__global__ __launch_bounds__(256) void k_tdist_f64(const double *__restrict__ xcT,
                                                   const double *__restrict__ norms, int64_t npad,
                                                   int32_t dpad, int32_t nb, int64_t tile0,
                                                   int64_t tile_base, float *__restrict__ Pb,
                                                   const Hdr *guard, int64_t gn, int32_t gkey,
                                                   const uint8_t *__restrict__ nz, bool skip,
                                                   const float *__restrict__ ra,
                                                   const float *__restrict__ rm,
                                                   const float *__restrict__ rr) {
  const int64_t tile = tile0 + blockIdx.x;
  int I, J;
  if (!tdist_begin(guard, gn, gkey, nz, skip, tile, nb, I, J)) return;
  const int ry = blockIdx.y & 3, cx = blockIdx.y >> 2;
  const bool diag = (I == J);
  if (diag && 64 * ry >= 64 * kTileCT * (cx + 1)) return;  // wholly below the diagonal
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int cl0 = 64 * kTileCT * cx + w * (16 * kTileCT);  // first column in the tile
  const int64_t col0 = (int64_t)J * T + cl0;
  const int row0_loc = 64 * ry;
  const int64_t row0 = (int64_t)I * T + row0_loc;
  const int li = l & 15, lk = l >> 4;
  v4d acc[4][kTileCT];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < kTileCT; ++c) acc[a][c] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < dpad; k0 += 4) {
    const double *xk = xcT + (int64_t)(k0 + lk) * npad;
    double av[4], bv[kTileCT];
#pragma unroll
    for (int a = 0; a < 4; ++a) av[a] = xk[row0 + a * 16 + li];
#pragma unroll
    for (int c = 0; c < kTileCT; ++c) bv[c] = xk[col0 + c * 16 + li];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < kTileCT; ++c)
        acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[a][c], 0, 0, 0);
  }
  float *tp = Pb + (size_t)(tile - tile_base) * T * T;
  PtStat sc[kTileCT];
#pragma unroll
  for (int c = 0; c < kTileCT; ++c)
    sc[c] = pt_stat<PACK>((int64_t)J * T + cl0 + c * 16 + li, gn, ra, rm, rr);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int il = row0_loc + a * 16 + lk + 4 * r;
      const double ni = norms[(int64_t)I * T + il];
      const PtStat si = pt_stat<PACK>((int64_t)I * T + il, gn, ra, rm, rr);
      float v[kTileCT];
#pragma unroll
      for (int c = 0; c < kTileCT; ++c) {
        const int jl = cl0 + c * 16 + li;
        const double dd = ni + norms[(int64_t)J * T + jl] - 2.0 * acc[a][c][r];
        v[c] = tile_value<PACK>((float)fmax(dd, 0.0), diag, il, jl, si, sc[c]);
      }
      // the lane's columns are consecutive elements (e, e + 1) of one float4
      // slot of the tile layout: one 8-byte store off the diagonal
      static_assert(kTileCT == 2, "two columns per lane");
      if (!diag) {
        *reinterpret_cast<float2 *>(tp + tile_pos(il, cl0 + li)) = make_float2(v[0], v[1]);
      } else {
#pragma unroll
        for (int c = 0; c < kTileCT; ++c) put_d(tp, true, il, cl0 + c * 16 + li, v[c]);
      }
    }
  }
}

// FP32 mode: a workgroup covers 64 rows x 256 columns (grid y: 4 row groups),
// as k_dist_f32.
template <bool PACK>
__global__ __launch_bounds__(256) void k_tdist_f32(const float *__restrict__ xfT,
                                                   const float *__restrict__ norms, int64_t npad,
                                                   int32_t dpad, int32_t nb, int64_t tile0,
                                                   int64_t tile_base, float *__restrict__ Pb,
                                                   const Hdr *guard, int64_t gn, int32_t gkey,
                                                   const uint8_t *__restrict__ nz, bool skip,
                                                   const float *__restrict__ ra,
                                                   const float *__restrict__ rm,
                                                   const float *__restrict__ rr) {
  const int64_t tile = tile0 + blockIdx.x;
  int I, J;
  if (!tdist_begin(guard, gn, gkey, nz, skip, tile, nb, I, J)) return;
  const bool diag = (I == J);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int cl0 = w * 64;
  const int64_t col0 = (int64_t)J * T + cl0;
  const int row0_loc = blockIdx.y * 64;
  const int64_t row0 = (int64_t)I * T + row0_loc;
  const int li = l & 15, lk = l >> 4;
  v4f acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < dpad; k0 += 4) {
    const float *xk = xfT + (int64_t)(k0 + lk) * npad;
    float av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) av[a] = xk[row0 + a * 16 + li];
#pragma unroll
    for (int c = 0; c < 4; ++c) bv[c] = xk[col0 + c * 16 + li];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[c], acc[a][c], 0, 0, 0);
  }
  float *tp = Pb + (size_t)(tile - tile_base) * T * T;
  PtStat sc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
    sc[c] = pt_stat<PACK>((int64_t)J * T + cl0 + c * 16 + li, gn, ra, rm, rr);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int il = row0_loc + a * 16 + 4 * lk + r;
      const float ni = norms[(int64_t)I * T + il];
      const PtStat si = pt_stat<PACK>((int64_t)I * T + il, gn, ra, rm, rr);
      float v[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int jl = cl0 + c * 16 + li;
        const float dd = (ni + norms[(int64_t)J * T + jl]) - 2.f * acc[a][c][r];
        v[c] = tile_value<PACK>(fmaxf(dd, 0.f), diag, il, jl, si, sc[c]);
      }
      // the lane's four columns are the four elements of one float4 slot of
      // the tile layout: one 16-byte store off the diagonal
      if (!diag) {
        *reinterpret_cast<float4 *>(tp + tile_pos(il, cl0 + li)) =
            make_float4(v[0], v[1], v[2], v[3]);
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) put_d(tp, true, il, cl0 + c * 16 + li, v[c]);
      }
    }
  }
}

// 16-bit modes: as k_dist_lp, a workgroup covers 64 rows x 256 columns.
template <typename H, typename V8, bool SCALE, bool PACK>
__global__ __launch_bounds__(256) void k_tdist_lp(const H *__restrict__ xa,
                                                  const float *__restrict__ norms, int32_t kk,
                                                  int32_t nb, int64_t tile0, int64_t tile_base,
                                                  float *__restrict__ Pb, const Hdr *guard,
                                                  int64_t gn, int32_t gkey,
                                                  const uint8_t *__restrict__ nz, bool skip,
                                                  const float *__restrict__ ra,
                                                  const float *__restrict__ rm,
                                                  const float *__restrict__ rr) {
  const int64_t tile = tile0 + blockIdx.x;
  int I, J;
  if (!tdist_begin(guard, gn, gkey, nz, skip, tile, nb, I, J)) return;
  const bool diag = (I == J);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int cl0 = w * 64;
  const int64_t col0 = (int64_t)J * T + cl0;
  const int row0_loc = blockIdx.y * 64;
  const int64_t row0 = (int64_t)I * T + row0_loc;
  const int li = l & 15, lk = l >> 4;
  float inv_s2 = 1.f;
  if (SCALE) {
    const float s = fp16_scale(guard);
    inv_s2 = 1.f / (s * s);
  }
  v4f acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < kk; k0 += 32) {
    V8 av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      av[a] = *reinterpret_cast<const V8 *>(xa + (row0 + a * 16 + li) * kk + k0 + 8 * lk);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      bv[c] = *reinterpret_cast<const V8 *>(xa + (col0 + c * 16 + li) * kk + k0 + 8 * lk);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if constexpr (sizeof(H) == 2 && __is_same(H, __bf16))
          acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[c], acc[a][c], 0, 0, 0);
        else
          acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[a], bv[c], acc[a][c], 0, 0, 0);
      }
  }
  float *tp = Pb + (size_t)(tile - tile_base) * T * T;
  PtStat sc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
    sc[c] = pt_stat<PACK>((int64_t)J * T + cl0 + c * 16 + li, gn, ra, rm, rr);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int il = row0_loc + a * 16 + 4 * lk + r;
      const float ni = norms[(int64_t)I * T + il];
      const PtStat si = pt_stat<PACK>((int64_t)I * T + il, gn, ra, rm, rr);
      float v[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int jl = cl0 + c * 16 + li;
        const float dd = (ni + norms[(int64_t)J * T + jl]) - 2.f * (acc[a][c][r] * inv_s2);
        v[c] = tile_value<PACK>(fmaxf(dd, 0.f), diag, il, jl, si, sc[c]);
      }
      // the lane's four columns are the four elements of one float4 slot of
      // the tile layout: one 16-byte store off the diagonal
      if (!diag) {
        *reinterpret_cast<float4 *>(tp + tile_pos(il, cl0 + li)) =
            make_float4(v[0], v[1], v[2], v[3]);
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) put_d(tp, true, il, cl0 + c * 16 + li, v[c]);
      }
    }
  }
}

// x3 modes: as k_tdist_lp, a workgroup covers 64 rows x 256 columns of the
// tile; the sums come from the same routine as the stored path's.
template <typename H, typename V8, bool PACK>
__global__ __launch_bounds__(256, 2) void k_tdist_x3(const H *__restrict__ xs,
                                                  const float2 *__restrict__ nhl, int32_t k32,
                                                  int32_t bits, int32_t nb, int64_t tile0,
                                                  int64_t tile_base, float *__restrict__ Pb,
                                                  const Hdr *guard, int64_t gn, int32_t gkey,
                                                  const uint8_t *__restrict__ nz, bool skip,
                                                  const float *__restrict__ ra,
                                                  const float *__restrict__ rm,
                                                  const float *__restrict__ rr) {
  const int64_t tile = tile0 + blockIdx.x;
  int I, J;
  if (!tdist_begin(guard, gn, gkey, nz, skip, tile, nb, I, J)) return;
  const bool diag = (I == J);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int cl0 = w * 64;
  const int64_t col0 = (int64_t)J * T + cl0;
  const int row0_loc = blockIdx.y * 64;
  const int64_t row0 = (int64_t)I * T + row0_loc;
  const int li = l & 15, lk = l >> 4;
  v4f A0[4][4], R[4][4];
  x3_contract<H, V8>(xs, k32, row0, col0, li, lk, A0, R);
  const X3Scale sc = x3_scale(guard, bits);
  float *tp = Pb + (size_t)(tile - tile_base) * T * T;
  PtStat scs[4];
  float2 nj[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    scs[c] = pt_stat<PACK>(col0 + c * 16 + li, gn, ra, rm, rr);
    nj[c] = nhl[col0 + c * 16 + li];
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int il = row0_loc + t * 16 + 4 * lk + r;
      const float2 ni = nhl[(int64_t)I * T + il];
      const PtStat si = pt_stat<PACK>((int64_t)I * T + il, gn, ra, rm, rr);
      float v[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int jl = cl0 + c * 16 + li;
        const float dd = x3_combine(ni, nj[c], A0[t][c][r], R[t][c][r], sc);
        v[c] = tile_value<PACK>(dd, diag, il, jl, si, scs[c]);
      }
      if (!diag) {
        *reinterpret_cast<float4 *>(tp + tile_pos(il, cl0 + li)) =
            make_float4(v[0], v[1], v[2], v[3]);
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) put_d(tp, true, il, cl0 + c * 16 + li, v[c]);
      }
    }
  }
}

// ----------------------------------------------------------------------------
// 3. Symmetrise and normalise in place (Eq. 3):
//    p_ij = exp2(-a_i (d - m_i)) r_i + exp2(-a_j (d - m_j)) r_j,  r = 1/(2 n S).
// Also per tile: sum p and sum p ln p over ordered pairs (off-diagonal tiles
// stand for both (i, j) and (j, i)).
// ----------------------------------------------------------------------------
__device__ __forceinline__ void pack_tile(float4 *__restrict__ P, const float *__restrict__ a,
                                          const float *__restrict__ m,
                                          const float *__restrict__ r, int64_t n, int32_t nb,
                                          double2 *__restrict__ ppart,
                                          uint8_t *__restrict__ nzflag, int2 *__restrict__ tmap,
                                          int64_t tile, int64_t pslot) {
  __shared__ double red[2][4];
  __shared__ float srow[3][T];  // a, m, r of the tile's rows (0 past n)
  int I, J;
  tile_coords(tile, nb, I, J);
  if (threadIdx.x == 0) tmap[tile] = make_int2(I, J);
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int tc = l & 15, tr = (l >> 4) + 4 * w;
  const bool diag = (I == J);
  {
    const int64_t i = (int64_t)I * T + t;
    const bool ok = i < n;
    srow[0][t] = ok ? a[i] : 0.f;
    srow[1][t] = ok ? m[i] : 0.f;
    srow[2][t] = ok ? r[i] : 0.f;
  }
  float ac[16], mc[16], rc[16];
  uint32_t rvalid = 0, cvalid = 0;  // bit k: row tr+16k (column tc+16k) is a real point
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    rvalid |= ((int64_t)I * T + tr + 16 * k < n) ? (1u << k) : 0u;
    const int64_t j = (int64_t)J * T + tc + 16 * k;
    const bool ok = j < n;
    cvalid |= ok ? (1u << k) : 0u;
    ac[k] = ok ? a[j] : 0.f;
    mc[k] = ok ? m[j] : 0.f;
    rc[k] = ok ? r[j] : 0.f;
  }
  __syncthreads();
  float4 *tp = P + (size_t)pslot * TT4;
  float psum = 0.f, plp = 0.f;
  bool any = false;
  // row k of the thread's block is four float4 (one per column quarter mq);
  // rows alternate between two register buffers, so the next row's four
  // loads are in flight while a row is converted
  auto convert_row = [&](int k, const float4 (&dv)[4]) {
    const int row = tr + 16 * k;
    const float ark = srow[0][row], mrk = srow[1][row], rrk = srow[2][row];
#pragma unroll
    for (int mq = 0; mq < 4; ++mq) {
      const float dd[4] = {dv[mq].x, dv[mq].y, dv[mq].z, dv[mq].w};
      float pv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int mm = 4 * mq + e;
        float p = pair_p(dd[e], ark, mrk, rrk, ac[mm], mc[mm], rc[mm]);
        if (diag && tr == tc && k == mm) p = 0.f;
        if (!((rvalid >> k) & (cvalid >> mm) & 1u)) p = 0.f;
        // values below the normal FP32 range are stored as 0 (they change no
        // sum by more than 1e-38); a tile whose entries are all 0 is skipped
        // by the attractive part of the force pass
        if (p < FLT_MIN) p = 0.f;
        any |= p > 0.f;
        pv[e] = p;
        psum += p;
        // denormal p (< FLT_MIN) contribute below 1e-36 and are skipped: the
        // hardware log flushes them to zero
        plp += (p >= FLT_MIN) ? p * __builtin_amdgcn_logf(p) : 0.f;
      }
      tp[(k * 4 + mq) * 256 + t] = make_float4(pv[0], pv[1], pv[2], pv[3]);
    }
  };
  float4 ba[4], bb[4];
#pragma unroll
  for (int mq = 0; mq < 4; ++mq) ba[mq] = tp[mq * 256 + t];
#pragma unroll 1
  for (int k = 0; k < 16; k += 2) {
#pragma unroll
    for (int mq = 0; mq < 4; ++mq) bb[mq] = tp[((k + 1) * 4 + mq) * 256 + t];
    convert_row(k, ba);
    if (k + 2 < 16) {
#pragma unroll
      for (int mq = 0; mq < 4; ++mq) ba[mq] = tp[((k + 2) * 4 + mq) * 256 + t];
    }
    convert_row(k + 1, bb);
  }
  double ds = wave_sum_d((double)psum), dl = wave_sum_d((double)plp);
  if (l == 0) {
    red[0][w] = ds;
    red[1][w] = dl;
  }
  const int tile_any = __syncthreads_or(any ? 1 : 0);
  if (t == 0) {
    nzflag[tile] = tile_any ? 1 : 0;
    double mult = diag ? 1.0 : 2.0;
    double S = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    double Lg = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    ppart[tile] = make_double2(mult * S, mult * Lg * kLn2);
  }
}

__global__ __launch_bounds__(256) void k_pack(float4 *__restrict__ P, const float *__restrict__ a,
                                              const float *__restrict__ m,
                                              const float *__restrict__ r, int64_t n, int32_t nb,
                                              double2 *__restrict__ ppart,
                                              uint8_t *__restrict__ nzflag,
                                              int2 *__restrict__ tmap) {
  pack_tile(P, a, m, r, n, nb, ppart, nzflag, tmap, blockIdx.x, blockIdx.x);
}

__device__ __forceinline__ void pack_reduce_wg(const double2 *__restrict__ ppart, int64_t nt,
                                               Hdr *h, int32_t ready = 1) {
  __shared__ double red[2][16];
  double s = 0.0, lg = 0.0;
  for (int64_t q = threadIdx.x; q < nt; q += 1024) {
    s += ppart[q].x;
    lg += ppart[q].y;
  }
  s = wave_sum_d(s);
  lg = wave_sum_d(lg);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s;
    red[1][threadIdx.x >> 6] = lg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double S = 0.0, Lg = 0.0;
    for (int q = 0; q < 16; ++q) {
      S += red[0][q];
      Lg += red[1][q];
    }
    h->p_sum = S;
    h->c_p = Lg;
    if (!isfinite(S) || !isfinite(Lg)) atomicOr(&h->err, kErrNonFinite);
    h->ready = ready;
  }
}

__global__ __launch_bounds__(1024) void k_pack_reduce(const double2 *__restrict__ ppart,
                                                      int64_t nt, Hdr *h) {
  pack_reduce_wg(ppart, nt, h);
}

// ----------------------------------------------------------------------------
// 4. Locality reordering (not part of the method: it only changes the order
// in which P is stored and summed).
//
// Points whose affinities are nonzero lie close in the input space, so an
// order in which nearby points are contiguous concentrates the nonzero p_ij in
// few tiles and leaves the rest all-zero (skipped by the attractive part of
// every force pass). The order is a principal-direction bisection tree with
// tile-aligned leaves: at level l the internal positions split into 2^l
// segments [floor(s nb / 2^l) T, floor((s + 1) nb / 2^l) T); each segment is
// sorted by the projection of its centred points on their leading principal
// direction (a few power iterations from a fixed start), so that its two
// halves at the next level are the two sides of that direction. Every step is
// deterministic (fixed reduction orders, a fixed sorting network).
// ----------------------------------------------------------------------------
constexpr int kTreeThreads = 256;
constexpr int kTreeMaxD = 2048;
constexpr int kTreePowerIters = 4;
constexpr int kTreeTargetGroups = 1024;  // workgroups per level at the shallow levels
constexpr int kSortBlock = 4096;         // keys per workgroup in the LDS sorting stages

// Given dissimilarities (any measure may enter, section "ptSNE: parallelized
// t-SNE"): the squares of rows b*T .. b*T + T - 1 of the n x n matrix into the
// distance block, in place of the contraction. Grid (npad / 256, T / 16):
// workgroup (c, g) covers columns 256 c .. 256 c + 255 of rows 16 g .. 16 g + 15.
__global__ __launch_bounds__(256) void k_dissim_block(const float *__restrict__ dis, int64_t n,
                                                      int64_t npad, int32_t b,
                                                      float *__restrict__ dblock, Hdr *h) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool bad = false;
  for (int r = 16 * blockIdx.y; r < 16 * (blockIdx.y + 1); ++r) {
    const int64_t i = (int64_t)b * T + r;
    float v = 0.f;
    if (i < n && j < n) {
      const float dv = dis[i * n + j];
      bad |= !(dv >= 0.f && dv < INFINITY) && j != i;
      v = dv * dv;
    }
    dblock[(int64_t)r * npad + j] = v;
  }
  if (bad) flag_error(h, kErrNonFinite);
}

__global__ void k_reorder_init(int64_t n, int64_t npad, int32_t *__restrict__ perm,
                               int32_t *__restrict__ inv) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npad) return;
  perm[i] = (int32_t)i;
  inv[i] = (int32_t)i;
}

// Segment s of level `level`: internal positions [lo, hi).
struct TreeSeg {
  int64_t lo, hi;
};

__device__ inline TreeSeg tree_segment(int64_t s, int level, int32_t nb, int64_t n) {
  TreeSeg g;
  g.lo = ((s * nb) >> level) * T;
  g.hi = (((s + 1) * nb) >> level) * T;
  if (g.lo > n) g.lo = n;
  if (g.hi > n) g.hi = n;
  return g;
}

// Sum of acc[0..7] over the workgroup into out[0..7] (LDS), in a fixed order.
__device__ inline void tree_block_sum8(double (&acc)[8], double (*red)[8], double *out) {
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = wave_sum_d(acc[q]);
  if (l == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) red[w][q] = acc[q];
  }
  __syncthreads();
  if (t < 8) {
    double s = 0.0;
    for (int g = 0; g < kTreeThreads / 64; ++g) s += red[g][t];
    out[t] = s;
  }
  __syncthreads();
}

__device__ inline uint32_t orderable_f32(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Partial sums of one chunk (workgroup blockIdx.x = s * C + c) of a segment:
//   MODE 0: sum_r x_r                       (for the mean)
//   MODE 1: sum_r (x_r - mean) w_r, w_r = (x_r - mean) . v   (power iteration)
// into part[blockIdx.x][0 .. d). Each thread keeps w_r of its own rows in
// wbuf and reads back only what it wrote.
template <int MODE>
__global__ __launch_bounds__(kTreeThreads) void k_tree_partial(
    const double *__restrict__ xcT, int64_t npad, int32_t d, int64_t n, int32_t nb, int level,
    int32_t C, const int32_t *__restrict__ perm, const double *__restrict__ segmean,
    const double *__restrict__ segv, double *__restrict__ wbuf, double *__restrict__ part) {
  __shared__ double mean[MODE ? kTreeMaxD : 1], v[MODE ? kTreeMaxD : 1];
  __shared__ double red[kTreeThreads / 64][8];
  __shared__ double out8[8];
  const int t = threadIdx.x;
  const int64_t s = blockIdx.x / C, c = blockIdx.x % C;
  const TreeSeg g = tree_segment(s, level, nb, n);
  if (g.hi - g.lo <= T) return;  // leaves are not split
  const int64_t len = g.hi - g.lo;
  const int64_t r0 = g.lo + len * c / C, r1 = g.lo + len * (c + 1) / C;
  double *out = part + (int64_t)blockIdx.x * d;
  if (MODE == 1) {
    for (int k = t; k < d; k += kTreeThreads) {
      mean[k] = segmean[s * d + k];
      v[k] = segv[s * d + k];
    }
    __syncthreads();
    for (int64_t r = r0 + t; r < r1; r += kTreeThreads) {
      const int64_t i = perm[r];
      double wsum = 0.0;
      for (int k = 0; k < d; ++k) wsum += (xcT[(int64_t)k * npad + i] - mean[k]) * v[k];
      wbuf[r] = wsum;
    }
  }
  for (int k0 = 0; k0 < d; k0 += 8) {
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    for (int64_t r = r0 + t; r < r1; r += kTreeThreads) {
      const int64_t i = perm[r];
      const double wr = MODE ? wbuf[r] : 1.0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (k0 + q < d) {
          const double xv = xcT[(int64_t)(k0 + q) * npad + i];
          acc[q] += MODE ? (xv - mean[MODE ? k0 + q : 0]) * wr : xv;
        }
    }
    tree_block_sum8(acc, red, out8);
    if (t < 8 && k0 + t < d) out[k0 + t] = out8[t];
  }
}

// Per segment: MODE 0 turns the chunk sums into the mean and sets the fixed
// start vector; MODE 1 turns them into the next (normalised) direction.
template <int MODE>
__global__ __launch_bounds__(kTreeThreads) void k_tree_reduce(const double *__restrict__ part,
                                                              int32_t d, int64_t n, int32_t nb,
                                                              int level, int32_t C,
                                                              double *__restrict__ segmean,
                                                              double *__restrict__ segv) {
  __shared__ double red[kTreeThreads / 64];
  __shared__ double scale;
  const int t = threadIdx.x;
  const int64_t s = blockIdx.x;
  const TreeSeg g = tree_segment(s, level, nb, n);
  if (g.hi - g.lo <= T) return;
  double ss = 0.0;
  for (int k = t; k < d; k += kTreeThreads) {
    double sum = 0.0;
    for (int c = 0; c < C; ++c) sum += part[(s * C + c) * d + k];
    if (MODE == 0) {
      segmean[s * d + k] = sum / (double)(g.hi - g.lo);
      const uint32_t hsh = (uint32_t)(k + 1) * 2654435761u;
      segv[s * d + k] = 0.5 + (double)(hsh >> 8) * (1.0 / 16777216.0);
    } else {
      segv[s * d + k] = sum;
      ss += sum * sum;
    }
  }
  if (MODE == 0) return;
  ss = wave_sum_d(ss);
  if ((t & 63) == 0) red[t >> 6] = ss;
  __syncthreads();
  if (t == 0) {
    double tot = 0.0;
    for (int q = 0; q < kTreeThreads / 64; ++q) tot += red[q];
    scale = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;  // coincident points: projections all 0
  }
  __syncthreads();
  for (int k = t; k < d; k += kTreeThreads) segv[s * d + k] *= scale;
}

// Sort keys (segment << 32 | projection on the segment's direction) and the
// caller indices of the positions; leaves keep their order.
__global__ __launch_bounds__(kTreeThreads) void k_tree_keys(
    const double *__restrict__ xcT, int64_t npad, int32_t d, int64_t n, int32_t nb, int level,
    int32_t C, const int32_t *__restrict__ perm, const double *__restrict__ segmean,
    const double *__restrict__ segv, uint64_t *__restrict__ keys, int32_t *__restrict__ vals) {
  __shared__ double mean[kTreeMaxD], v[kTreeMaxD];
  const int t = threadIdx.x;
  const int64_t s = blockIdx.x / C, c = blockIdx.x % C;
  const TreeSeg g = tree_segment(s, level, nb, n);
  const int64_t len = g.hi - g.lo;
  const int64_t r0 = g.lo + len * c / C, r1 = g.lo + len * (c + 1) / C;
  const uint64_t seg = (uint64_t)s << 32;
  if (len <= T) {
    for (int64_t r = r0 + t; r < r1; r += kTreeThreads) {
      keys[r] = seg | (uint64_t)(r - g.lo);
      vals[r] = perm[r];
    }
    return;
  }
  for (int k = t; k < d; k += kTreeThreads) {
    mean[k] = segmean[s * d + k];
    v[k] = segv[s * d + k];
  }
  __syncthreads();
  for (int64_t r = r0 + t; r < r1; r += kTreeThreads) {
    const int64_t i = perm[r];
    double p = 0.0;
    for (int k = 0; k < d; ++k) p += (xcT[(int64_t)k * npad + i] - mean[k]) * v[k];
    keys[r] = seg | (uint64_t)orderable_f32((float)p);
    vals[r] = perm[r];
  }
}

// Keys of positions beyond n sort last.
__global__ void k_tree_pad(int64_t n, int64_t npow2, uint64_t *__restrict__ keys,
                           int32_t *__restrict__ vals) {
  const int64_t r = n + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= npow2) return;
  keys[r] = ~0ull;
  vals[r] = (int32_t)(r < INT32_MAX ? r : INT32_MAX);
}

// Bitonic sort (ascending) of (key, value) pairs over npow2 entries.
// Global stage: one compare-exchange distance j >= kSortBlock / 2 ... of
// merge size k.
__global__ void k_bitonic(uint64_t *__restrict__ keys, int32_t *__restrict__ vals, int64_t npow2,
                          int64_t j, int64_t k) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npow2) return;
  const int64_t l = i ^ j;
  if (l <= i) return;
  const uint64_t a = keys[i], b = keys[l];
  const bool up = (i & k) == 0;
  if ((a > b) == up) {
    keys[i] = b;
    keys[l] = a;
    const int32_t va = vals[i];
    vals[i] = vals[l];
    vals[l] = va;
  }
}

// LDS stages on blocks of `blk` consecutive entries (blk a power of two, at
// most kSortBlock): with k0 = 0, every merge size k = 2 .. blk and all its
// distances (a full sort of each block in the global direction pattern);
// otherwise the distances blk / 2 .. 1 of merge size k0.
__global__ __launch_bounds__(1024) void k_bitonic_local(uint64_t *__restrict__ keys,
                                                        int32_t *__restrict__ vals, int64_t blk,
                                                        int64_t k0) {
  __shared__ uint64_t sk[kSortBlock];
  __shared__ int32_t sv[kSortBlock];
  const int64_t base = (int64_t)blockIdx.x * blk;
  for (int64_t e = threadIdx.x; e < blk; e += 1024) {
    sk[e] = keys[base + e];
    sv[e] = vals[base + e];
  }
  __syncthreads();
  const int64_t kfirst = k0 ? k0 : 2, klast = k0 ? k0 : blk;
  for (int64_t k = kfirst; k <= klast; k <<= 1) {
    for (int64_t j = (k0 ? blk : k) >> 1; j > 0; j >>= 1) {
      for (int64_t e = threadIdx.x; e < blk; e += 1024) {
        const int64_t l = e ^ j;
        if (l > e) {
          const uint64_t a = sk[e], b = sk[l];
          const bool up = ((base + e) & k) == 0;
          if ((a > b) == up) {
            sk[e] = b;
            sk[l] = a;
            const int32_t va = sv[e];
            sv[e] = sv[l];
            sv[l] = va;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int64_t e = threadIdx.x; e < blk; e += 1024) {
    keys[base + e] = sk[e];
    vals[base + e] = sv[e];
  }
}

__global__ void k_tree_apply(const int32_t *__restrict__ vals, int64_t n,
                             int32_t *__restrict__ perm) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r < n) perm[r] = vals[r];
}

__global__ void k_inverse(const int32_t *__restrict__ perm, int64_t npad,
                          int32_t *__restrict__ inv) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r < npad) inv[perm[r]] = (int32_t)r;
}

// Centred X and its norms in the internal order (padding rows stay zero).
__global__ __launch_bounds__(256) void k_permute_x(const double *__restrict__ xcT,
                                                   const double *__restrict__ norms,
                                                   const int32_t *__restrict__ perm, int64_t n,
                                                   int64_t npad, int32_t dpad,
                                                   double *__restrict__ xcT2,
                                                   double *__restrict__ norms2) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= npad) return;
  const int64_t i = r < n ? perm[r] : -1;
  for (int k = 0; k < dpad; ++k) xcT2[(int64_t)k * npad + r] = i >= 0 ? xcT[(int64_t)k * npad + i] : 0.0;
  norms2[r] = i >= 0 ? norms[i] : 0.0;
}

// ----------------------------------------------------------------------------
// Exports (test hooks)
// ----------------------------------------------------------------------------
__device__ inline bool state_ok(const Hdr *h, int64_t n) {
  return h->magic == kMagic && h->n == n && h->ready == 1;
}

__global__ __launch_bounds__(256) void k_export_rows(const float4 *__restrict__ P, int64_t n,
                                                     int32_t nb, int64_t row0, int64_t nrows,
                                                     const int32_t *__restrict__ inv,
                                                     float *__restrict__ out, Hdr *h) {
  if (!state_ok(h, n)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) flag_error(h, kErrState);
    return;
  }
  // one thread per output element (row rr, column j)
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= nrows * n) return;
  const int64_t rr = idx / n, j = idx % n;
  int64_t i = inv[row0 + rr], jj = inv[j];  // internal positions of the caller's (row, column)
  if (i / T > jj / T) {  // lower triangle: read the mirrored entry
    int64_t tmp = i;
    i = jj;
    jj = tmp;
  }
  const int I = (int)(i / T), J = (int)(jj / T);
  const int il = (int)(i % T), jl = (int)(jj % T);
  const int tr = il & 15, k = il >> 4, tc = jl & 15, mmi = jl >> 4;
  const int mq = mmi >> 2, e = mmi & 3;
  const int th = (tr >> 2) * 64 + (tr & 3) * 16 + tc;
  const int s = k * 4 + mq;
  const float *tile = reinterpret_cast<const float *>(P + (size_t)tile_start(I, nb) * TT4 +
                                                      (size_t)(J - I) * TT4);
  out[idx] = tile[((size_t)s * 256 + th) * 4 + e];
}

__global__ void k_export_stats(int64_t n, const double *__restrict__ beta,
                               const float *__restrict__ m, const double *__restrict__ S,
                               const double *__restrict__ H, const int32_t *__restrict__ ev,
                               const int32_t *__restrict__ inv, double *ob, float *om, double *oS,
                               double *oH, int32_t *oe, Hdr *h) {
  // affinities for this n complete (stored or implicit P): the order exists
  if (!(h->magic == kMagic && h->n == n && (h->ready == 1 || h->ready == 2))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) flag_error(h, kErrState);
    return;
  }
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t r = inv[i];
  if (ob) ob[i] = beta[r];
  if (om) om[i] = m[r];
  if (oS) oS[i] = S[r];
  if (oH) oH[i] = H[r];
  if (oe) oe[i] = ev[r];
}

// The internal order and the zero-tile flags, after checking that the
// workspace holds affinities for this n.
__global__ __launch_bounds__(256) void k_export_order(const Hdr *h, int64_t n, int64_t nt,
                                                      const int32_t *__restrict__ perm,
                                                      const uint8_t *__restrict__ nz,
                                                      int32_t *__restrict__ operm,
                                                      uint8_t *__restrict__ oflags) {
  if (!(h->magic == kMagic && h->n == n && (h->ready == 1 || h->ready == 2))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) flag_error(const_cast<Hdr *>(h), kErrState);
    return;
  }
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (operm && i < n) operm[i] = perm[i];
  // the flags exist only where P is stored
  if (oflags && h->ready == 1 && i < nt) oflags[i] = nz[i];
}

__global__ void k_export_scalars(int64_t n, const Hdr *h, double *out) {
  if (threadIdx.x != 0) return;
  const bool ok = h->magic == kMagic && h->n == n;
  out[0] = ok ? h->p_sum : NAN;
  out[1] = ok ? h->c_p : NAN;
  out[2] = ok ? h->z : NAN;
  out[3] = ok ? h->perplexity : NAN;
}

// Tile lists for the force pass: all-zero tiles in ascending order, then the
// others in ascending order (one workgroup; ballot prefix counts in a fixed
// order).
__device__ __forceinline__ void tile_lists_wg(const uint8_t *__restrict__ nz, int64_t nt,
                                              int32_t *__restrict__ tlist,
                                              int32_t *__restrict__ tcount) {
  __shared__ int32_t wz[16], wn[16];
  __shared__ int32_t zbase, nbase, zeros;
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  // pass 1: number of all-zero tiles
  int32_t cnt = 0;
  for (int64_t q = t; q < nt; q += 1024) cnt += nz[q] == 0;
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if (l == 0) wz[w] = cnt;
  __syncthreads();
  if (t == 0) {
    int32_t z = 0;
    for (int q = 0; q < 16; ++q) z += wz[q];
    zeros = z;
    zbase = 0;
    nbase = z;
  }
  __syncthreads();
  // pass 2: positions
  for (int64_t q0 = 0; q0 < nt; q0 += 1024) {
    const int64_t q = q0 + t;
    const bool valid = q < nt;
    const bool isz = valid && nz[q] == 0, isn = valid && nz[q] != 0;
    const uint64_t mz = __ballot(isz), mn = __ballot(isn);
    const uint64_t below = (l == 0) ? 0ull : (~0ull >> (64 - l));
    if (l == 0) {
      wz[w] = __popcll(mz);
      wn[w] = __popcll(mn);
    }
    __syncthreads();
    int32_t oz = zbase, on = nbase;
    for (int k = 0; k < w; ++k) {
      oz += wz[k];
      on += wn[k];
    }
    if (isz) tlist[oz + __popcll(mz & below)] = (int32_t)q;
    if (isn) tlist[on + __popcll(mn & below)] = (int32_t)q;
    __syncthreads();
    if (t == 0) {
      for (int k = 0; k < 16; ++k) {
        zbase += wz[k];
        nbase += wn[k];
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    tcount[0] = zeros;
    tcount[1] = (int32_t)(nt - zeros);
  }
}

__global__ __launch_bounds__(1024) void k_tile_lists(const uint8_t *__restrict__ nz, int64_t nt,
                                                     int32_t *__restrict__ tlist,
                                                     int32_t *__restrict__ tcount) {
  tile_lists_wg(nz, nt, tlist, tcount);
}

// Per row block b, the slots s (tiles (b, s) or (s, b)) whose P is not all
// zero, in increasing s: the update reads the attractive partial sums of
// these slots only. One workgroup per block; a fixed-order prefix count.
__device__ __forceinline__ void slot_list_wg(const uint8_t *__restrict__ nz, int32_t nb,
                                             int32_t *__restrict__ slots,
                                             int32_t *__restrict__ nslots, int b) {
  __shared__ int32_t wsum[4];
  __shared__ int32_t base;
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  if (t == 0) base = 0;
  __syncthreads();
  for (int s0 = 0; s0 < nb; s0 += 256) {
    const int s = s0 + t;
    int f = 0;
    if (s < nb) {
      const int64_t tile = s >= b ? tile_start(b, nb) + (s - b) : tile_start(s, nb) + (b - s);
      f = nz[tile] != 0;
    }
    const uint64_t mask = __ballot(f);
    const int before = __popcll(mask & ((l == 0) ? 0ull : (~0ull >> (64 - l))));
    if (l == 0) wsum[w] = __popcll(mask);
    __syncthreads();
    int off = base;
    for (int q = 0; q < w; ++q) off += wsum[q];
    if (f) slots[(int64_t)b * nb + off + before] = s;
    __syncthreads();
    if (t == 0) base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
  if (t == 0) nslots[b] = base;
}

__global__ __launch_bounds__(256) void k_slot_lists(const uint8_t *__restrict__ nz, int32_t nb,
                                                    int32_t *__restrict__ slots,
                                                    int32_t *__restrict__ nslots) {
  slot_list_wg(nz, nb, slots, nslots, blockIdx.x);
}

// ----------------------------------------------------------------------------
// 5. Many small problems at once (the partial problems of the parallel
// scheme). Same method as above with one wave per row: the row's squared
// distances (FP64 direct differences, rounded to FP32 like the distance
// block of the large path) stay in registers for the bisection, whose sums
// are wave reductions, so no workgroup barrier sits inside the search. The
// rows of a workgroup belong to one problem and share the staging of
// the other points' coordinates in LDS. The distances of tiles (I, J >= I)
// go straight into the P store in consumer order; the pack, reduction and
// list steps are the same device code as the single-problem path.
// ----------------------------------------------------------------------------

__device__ inline int small_find(const SmallEntry *tab, int count, int64_t key, int which) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t start = which == 0 ? tab[mid].wg0 : which == 1 ? tab[mid].tile0 : tab[mid].blk0;
    if (start <= key)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Position of element (il, jl) of a tile in the consumer order of the P store
// (the order the stage and pack kernels use), as a float index in the tile.
__device__ inline int small_pos(int il, int jl) {
  const int tr = il & 15, k = il >> 4, tc = jl & 15, mm = jl >> 4;
  const int s = k * 4 + (mm >> 2), t = 64 * (tr >> 2) + tc + 16 * (tr & 3);
  return (s * 256 + t) * 4 + (mm & 3);
}

// Header and identity order of every problem: one workgroup per row block.
__global__ __launch_bounds__(256) void k_small_init(const SmallEntry *__restrict__ tab, int count) {
  const int p = small_find(tab, count, blockIdx.x, 2);
  const SmallEntry &e = tab[p];
  const int64_t b = (int64_t)blockIdx.x - e.blk0;
  if (b < 0 || b >= e.nb) return;
  if (b == 0 && threadIdx.x == 0) {
    Hdr *h = e.h;
    h->magic = kMagic;
    h->n = e.n;
    h->d = e.d;
    h->ready = 0;
    h->err = 0;
    h->mode = TSNE_DIST_FP64;
    h->perplexity = e.perplexity;
    h->z = 0.0;
    h->c_p = 0.0;
    h->p_sum = 0.0;
    h->xmax = 0.f;
  }
  const int64_t i = b * T + threadIdx.x;
  e.perm[i] = (int32_t)i;
  e.inv[i] = (int32_t)i;
}

template <int VPT>
__global__ __launch_bounds__(kSmallRows * 64) void k_small_calibrate(
    const SmallEntry *__restrict__ tab, int count, int32_t dstride, int max_bisect,
    double tol_h) {
  // LDS (FP64, converted once): two buffers of 64 points ([64][dstride]
  // each), then the own rows
  extern __shared__ double sx[];
  constexpr int kThr = kSmallRows * 64;
  constexpr int kPre = 64 * kSmallMaxD / kThr;  // prefetch registers per thread
  const int p = small_find(tab, count, blockIdx.x, 0);
  const SmallEntry &e = tab[p];
  const int64_t n = e.n;
  const int32_t d = e.d;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x - e.wg0) * kSmallRows;
  const int64_t i = r0 + w;
  const bool row_ok = i < n;
  double *own = sx + 2 * 64 * dstride;
  for (int q = threadIdx.x; q < kSmallRows * d; q += kThr) {
    const int rr = q / d, k = q - rr * d;
    own[rr * dstride + k] = (r0 + rr) < n ? (double)e.x[(r0 + rr) * d + k] : 0.0;
  }
  const int nchunk = (int)((n + 63) / 64);
  // chunk c holds points 64c .. 64c + 63 as rows of d floats (contiguous in x)
  auto fetch = [&](int c, float (&pre)[kPre]) {
    const int64_t base = (int64_t)c * 64 * d, lim = (n - (int64_t)c * 64) * d;
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int idx = threadIdx.x + u * kThr;
      pre[u] = (idx < 64 * d && idx < lim) ? e.x[base + idx] : 0.f;
    }
  };
  auto put = [&](int c, const float (&pre)[kPre]) {
    double *buf = sx + (c & 1) * 64 * dstride;
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int idx = threadIdx.x + u * kThr;
      if (idx < 64 * d) {
        const int rr = idx / d, k = idx - rr * d;
        buf[rr * dstride + k] = (double)pre[u];
      }
    }
  };
  float pre[kPre];
  fetch(0, pre);
  put(0, pre);
  __syncthreads();
  const int I = (int)(i / T), il = (int)(i - (int64_t)I * T);
  float v[VPT];
  bool bad = false;
#pragma unroll
  for (int q = 0; q < VPT; ++q) {
    v[q] = INFINITY;
    if (q < nchunk) {  // uniform over the workgroup
      if (q + 1 < nchunk) fetch(q + 1, pre);  // in flight while this chunk is used
      const int64_t j = (int64_t)q * 64 + l;
      if (row_ok && j < n) {
        double acc = 0.0;
        const double *xj = sx + (q & 1) * 64 * dstride + l * dstride, *xi = own + w * dstride;
        for (int k = 0; k < d; ++k) {
          const double df = xj[k] - xi[k];
          acc = fma(df, df, acc);
        }
        const float dv = (float)acc;
        bad |= !isfinite(dv);
        const int J = (int)(j / T);
        if (J >= I) {
          const int jl = (int)(j - (int64_t)J * T);
          float *tp = reinterpret_cast<float *>(e.P + (size_t)(tile_start(I, e.nb) + (J - I)) * TT4);
          tp[small_pos(il, jl)] = dv;
        }
        if (j != i) v[q] = dv;
      }
      if (q + 1 < nchunk) put(q + 1, pre);  // the other buffer: last read two chunks ago
      __syncthreads();
    }
  }
  if (!row_ok) return;  // no barrier below this point
  float mn = INFINITY;
#pragma unroll
  for (int q = 0; q < VPT; ++q) mn = fminf(mn, v[q]);
  const float m = wave_min_f(mn);
#pragma unroll
  for (int q = 0; q < VPT; ++q) v[q] = (v[q] == INFINITY) ? kBig : v[q] - m;
  const double logu = log(e.perplexity);
  double beta = 1.0, lo = 0.0, hi = INFINITY, S = 0.0, H = 0.0;
  float a = 0.f;
  int it = 0, done = 0;
  while (!done) {
    ++it;
    a = fmaxf((float)(beta * kLog2e), 1e-30f);
    float s = 0.f, tt = 0.f, qq = 0.f;
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      const float ex = __builtin_amdgcn_exp2f(-a * v[q]);
      const float ve = v[q] * ex;  // 0 for an excluded entry (ex = 0)
      s += ex;
      tt += ve;
      qq = fmaf(v[q], ve, qq);
    }
    // butterfly sums: every lane holds the same totals, so the search below
    // takes the same branch in every lane
    const double SS = wave_sum_d((double)s), TT = wave_sum_d((double)tt);
    const double QQ = wave_sum_d((double)qq);
    const double beff = (double)a * kLn2;
    S = SS;
    const double mean = TT / SS;
    H = log(SS) + beff * mean;
    if (fabs(H - logu) <= tol_h) {
      done = 1;
    } else if (isfinite(hi) && (hi - lo) <= hi * 0x1p-24) {
      done = 1;
    } else if (it >= max_bisect) {
      done = 2;
    } else {
      // H falls with beta (dH/dbeta = -beta Var(d)): shrink the bracket,
      // then take the Newton step if it lands inside it, else bisect
      // (the bracket holds the FP64 iterates; H was taken at their FP32
      // rounding beff, within 2^-24 of beta)
      if (H > logu)
        lo = beta;
      else
        hi = beta;
      const double var = QQ / SS - mean * mean;
      const double nb = beta + (H - logu) / (beff * var);
      if (var > 0.0 && nb > lo && nb < hi && isfinite(nb))
        beta = nb;
      else
        beta = isinf(hi) ? 2.0 * beta : 0.5 * (lo + hi);
    }
  }
  bad = __any(bad);
  if (l == 0) {
    e.beta[i] = (double)a * kLn2;
    e.S[i] = S;
    e.H[i] = H;
    e.m[i] = m;
    e.a[i] = a;
    e.r[i] = (float)(1.0 / (2.0 * (double)n * S));
    e.evals[i] = done == 1 ? it : -it;
    if (done != 1) flag_error(e.h, kErrNoConv);
    if (bad || !isfinite(H) || !isfinite(S)) flag_error(e.h, kErrNonFinite);
  }
}

__global__ __launch_bounds__(256) void k_small_pack(const SmallEntry *__restrict__ tab,
                                                    int count) {
  const int p = small_find(tab, count, blockIdx.x, 1);
  const SmallEntry &e = tab[p];
  const int64_t tile = (int64_t)blockIdx.x - e.tile0;
  if (tile < 0 || tile >= e.nt) return;
  pack_tile(e.P, e.a, e.m, e.r, e.n, e.nb, e.ppart, e.nz, e.tmap, tile, tile);
}

__global__ __launch_bounds__(256) void k_small_slots(const SmallEntry *__restrict__ tab,
                                                     int count) {
  const int p = small_find(tab, count, blockIdx.x, 2);
  const SmallEntry &e = tab[p];
  const int64_t b = (int64_t)blockIdx.x - e.blk0;
  if (b < 0 || b >= e.nb) return;
  slot_list_wg(e.nz, e.nb, e.slots, e.nslots, (int)b);
}

// One workgroup per problem: the sums of P (marks the problem ready), then
// the tile lists.
__global__ __launch_bounds__(1024) void k_small_lists(const SmallEntry *__restrict__ tab) {
  const SmallEntry &e = tab[blockIdx.x];
  pack_reduce_wg(e.ppart, e.nt, e.h);
  __syncthreads();
  tile_lists_wg(e.nz, e.nt, e.tlist, e.tcount);
}

// ----------------------------------------------------------------------------
// 6. Implicit P: the workspace keeps a buffer of whole block rows of tiles
// (at most 2,048 tiles, at least one block row); every pass recomputes the
// distances of each block b of the rows in the buffer (the same MFMA kernel as
// the affinity stage, from the centred X in the internal order) and stages
// its tiles (b, b .. nb - 1), then packs the buffer, slot x holding tile
// base + x. The arithmetic is that of the stored P, so the values
// are bitwise the same.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pack_range(float4 *__restrict__ Pb,
                                                    const float *__restrict__ a,
                                                    const float *__restrict__ m,
                                                    const float *__restrict__ r, int64_t n,
                                                    int32_t nb, double2 *__restrict__ ppart,
                                                    uint8_t *__restrict__ nzflag,
                                                    int2 *__restrict__ tmap, int64_t tile0,
                                                    int64_t tile_base, const Hdr *guard,
                                                    int32_t gkey) {
  if (!implicit_ready(guard, n, gkey)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) flag_error(const_cast<Hdr *>(guard), kErrState);
    return;
  }
  const int64_t tile = tile0 + blockIdx.x;
  pack_tile(Pb, a, m, r, n, nb, ppart, nzflag, tmap, tile, tile - tile_base);
}

// After all blocks of a pass: sums of P (the header keeps ready = 2).
__global__ __launch_bounds__(1024) void k_implicit_sums(const double2 *__restrict__ ppart,
                                                        int64_t nt, int64_t n, int32_t key,
                                                        Hdr *h) {
  if (!implicit_ready(h, n, key)) return;
  pack_reduce_wg(ppart, nt, h, 2);
}

// End of an implicit affinity stage: no tile flagged nonzero and empty slot
// lists until the first pass builds them, then the mode in the header.
__global__ __launch_bounds__(256) void k_implicit_init(uint8_t *__restrict__ nz, int64_t nt,
                                                       int32_t *__restrict__ nslots, int32_t nb,
                                                       Hdr *h) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < nt) nz[i] = 0;
  if (i < nb) nslots[i] = 0;
}

__global__ void k_set_ready(Hdr *h, int32_t ready) {
  if (threadIdx.x == 0) h->ready = ready;
}

}  // namespace

// ----------------------------------------------------------------------------
// Host-side sequencing
// ----------------------------------------------------------------------------

// Distances of row block b against all columns into dblock (its slot of the
// group scratch), in the workspace's distance mode. xc, nrm: the centred X and its norms for the
// FP64 mode (the reduced modes read their prepared operands).
// P: the packed buffer, for the modes whose distance kernel stages the block
// row's tiles itself (FP64 and the x3 modes), else nullptr. Returns whether
// it did.
static bool launch_dist(const Layout &L, void *ws, int b, const double *xc, const double *nrm,
                        float *dblock, float4 *P, hipStream_t st) {
  const Hdr *h = at<const Hdr>(ws, L.hdr);
  const float *norms32 = at<const float>(ws, L.norms32);
  const dim3 dgrid((unsigned)(L.npad / 256), T / 64);
  switch (L.mode) {
    case TSNE_DIST_FP32:
      hipLaunchKernelGGL(k_dist_f32, dgrid, dim3(256), 0, st, at<const float>(ws, L.xfT), norms32,
                         L.npad, L.dpad, b, dblock);
      break;
    case TSNE_DIST_BF16:
      hipLaunchKernelGGL((k_dist_lp<__bf16, v8bf, false>), dgrid, dim3(256), 0, st,
                         at<const __bf16>(ws, L.xa), norms32, L.npad,
                         L.kk, b, dblock, h);
      break;
    case TSNE_DIST_FP16:
      hipLaunchKernelGGL((k_dist_lp<_Float16, v8h, true>), dgrid, dim3(256), 0, st,
                         at<const _Float16>(ws, L.xa), norms32,
                         L.npad, L.kk, b, dblock, h);
      break;
    case TSNE_DIST_BF16X3:
      hipLaunchKernelGGL((k_dist_x3<__bf16, v8bf>), dgrid, dim3(256), 0, st,
                         at<const __bf16>(ws, L.xa), at<const float2>(ws, L.norms32), L.npad,
                         L.kk / 4, x3_bits(L.kk / 4, true), b, dblock, h, P, L.nb);
      return P != nullptr;
    case TSNE_DIST_FP16X3:
      hipLaunchKernelGGL((k_dist_x3<_Float16, v8h>), dgrid, dim3(256), 0, st,
                         at<const _Float16>(ws, L.xa), at<const float2>(ws, L.norms32), L.npad,
                         L.kk / 4, x3_bits(L.kk / 4, false), b, dblock, h, P, L.nb);
      return P != nullptr;
    default:
      hipLaunchKernelGGL(k_dist_f64, dim3((unsigned)(L.npad / (64 * kDistCT)), T / 64), dim3(256),
                         0, st, xc, nrm, L.npad, L.dpad, b, dblock, P, L.nb);
      return P != nullptr;
  }
  return false;
}

hipError_t launch_affinities(const Layout &L, const float *x, const float *dis, double perplexity,
                             int max_bisect, double tol_h, int reorder, void *ws, hipStream_t st,
                             bool stats_only, bool implicit) {
  Hdr *h = at<Hdr>(ws, L.hdr);
  hipLaunchKernelGGL(k_init_hdr, dim3(1), dim3(64), 0, st, h, L.n, L.d, L.mode, perplexity);
  double *mean = at<double>(ws, L.xmean);
  double *xcT = at<double>(ws, L.xcT);
  double *norms = at<double>(ws, L.norms);
  float *dblock = at<float>(ws, L.dblock);
  float4 *P = at<float4>(ws, L.P);
  int32_t *perm = at<int32_t>(ws, L.perm), *inv = at<int32_t>(ws, L.inv);
  const unsigned pgrid = (unsigned)((L.npad + 255) / 256);
  if (!dis) {
    hipLaunchKernelGGL(k_colmean, dim3(L.d), dim3(256), 0, st, x, L.n, L.d, mean);
    hipLaunchKernelGGL(k_centre, dim3(pgrid), dim3(256), 0, st, x, L.n, L.d, L.npad, L.dpad,
                       mean, xcT, norms, h);
  }
  hipLaunchKernelGGL(k_reorder_init, dim3(pgrid), dim3(256), 0, st, L.n, L.npad, perm, inv);
  CalOut co{at<double>(ws, L.beta), at<double>(ws, L.S), at<double>(ws, L.H),
            at<float>(ws, L.m),     at<float>(ws, L.a),  at<float>(ws, L.r),
            at<int32_t>(ws, L.evals)};
  const double logu = log(perplexity);
  const int64_t vpt_need = (L.n + kCalThreads - 1) / kCalThreads;
  const int32_t k32 = (L.d + 31) / 32 * 32;
  float *norms32 = at<float>(ws, L.norms32);
  float *xfT = at<float>(ws, L.xfT);
  __bf16 *xa_b = at<__bf16>(ws, L.xa);
  _Float16 *xa_h = at<_Float16>(ws, L.xa);
  float2 *nhl = at<float2>(ws, L.norms32);
  double2 *ppart = at<double2>(ws, L.ppart);
  uint8_t *nz = at<uint8_t>(ws, L.nz);

  // Reduced-precision operands of the contraction, from centred X in the
  // current order.
  auto prep = [&](const double *xc) {
    switch (L.mode) {
      case TSNE_DIST_FP32:
        hipLaunchKernelGGL(k_prep_f32, dim3(pgrid), dim3(256), 0, st, xc, L.npad, L.dpad, xfT,
                           norms32);
        break;
      case TSNE_DIST_BF16:
        hipLaunchKernelGGL((k_prep_lp<__bf16, false>), dim3(pgrid), dim3(256), 0, st, xc, L.npad,
                           L.d, k32, xa_b, norms32, h);
        break;
      case TSNE_DIST_BF16X3:
        hipLaunchKernelGGL(k_prep_x3<__bf16>, dim3(pgrid), dim3(256), 0, st, xc, L.npad, L.d, k32,
                           x3_bits(k32, true), xa_b, nhl, h);
        break;
      case TSNE_DIST_FP16:
        hipLaunchKernelGGL((k_prep_lp<_Float16, true>), dim3(pgrid), dim3(256), 0, st, xc,
                           L.npad, L.d, k32, xa_h, norms32, h);
        break;
      case TSNE_DIST_FP16X3:
        hipLaunchKernelGGL(k_prep_x3<_Float16>, dim3(pgrid), dim3(256), 0, st, xc, L.npad, L.d,
                           k32, x3_bits(k32, false), xa_h, nhl, h);
        break;
      default:
        break;
    }
  };
  // Row blocks are handled in groups of L.cal_group: block b's distances go
  // to slot b - b0 of the scratch (b0 the group's first block).
  auto slot = [&](int b) { return dblock + (size_t)(b % L.cal_group) * T * L.npad; };
  auto group_end = [&](int b0) { return b0 + L.cal_group < L.nb ? b0 + L.cal_group : L.nb; };
  // Distances of row block b (into its slot), all columns.
  // Whether the distance kernel staged the block row's tiles itself.
  bool staged = false;
  auto dist = [&](int b, const double *xc, const double *nrm) {
    staged = launch_dist(L, ws, b, xc, nrm, slot(b), (stats_only || implicit) ? nullptr : P, st);
  };
  // The search over every row of the group starting at block b.
  auto calibrate = [&](int b) {
    const int64_t left = L.n - (int64_t)b * T, span = (int64_t)L.cal_group * T;
    const int rows = (int)(left < span ? left : span);
    dim3 g(rows), blk(kCalThreads);
    if (vpt_need <= 1)
      hipLaunchKernelGGL(k_calibrate<1>, g, blk, 0, st, dblock, L.n, L.npad, b, logu, max_bisect,
                         tol_h, co, h);
    else if (vpt_need <= 2)
      hipLaunchKernelGGL(k_calibrate<2>, g, blk, 0, st, dblock, L.n, L.npad, b, logu, max_bisect,
                         tol_h, co, h);
    else if (vpt_need <= 4)
      hipLaunchKernelGGL(k_calibrate<4>, g, blk, 0, st, dblock, L.n, L.npad, b, logu, max_bisect,
                         tol_h, co, h);
    else if (vpt_need <= 8)
      hipLaunchKernelGGL(k_calibrate<8>, g, blk, 0, st, dblock, L.n, L.npad, b, logu, max_bisect,
                         tol_h, co, h);
    else if (vpt_need <= 16)
      hipLaunchKernelGGL(k_calibrate<16>, g, blk, 0, st, dblock, L.n, L.npad, b, logu,
                         max_bisect, tol_h, co, h);
    else if (vpt_need <= 32)
      hipLaunchKernelGGL(k_calibrate<32>, g, blk, 0, st, dblock, L.n, L.npad, b, logu,
                         max_bisect, tol_h, co, h);
    else if (vpt_need <= 64)
      hipLaunchKernelGGL(k_calibrate<64>, g, blk, 0, st, dblock, L.n, L.npad, b, logu,
                         max_bisect, tol_h, co, h);
    else
      hipLaunchKernelGGL(k_calibrate<0>, g, blk, 0, st, dblock, L.n, L.npad, b, logu, max_bisect,
                         tol_h, co, h);
  };
  auto pack = [&]() {
    hipLaunchKernelGGL(k_pack, dim3((unsigned)L.nt), dim3(256), 0, st, P, co.a, co.m, co.r, L.n,
                       L.nb, ppart, nz, at<int2>(ws, L.tmap));
    hipLaunchKernelGGL(k_pack_reduce, dim3(1), dim3(1024), 0, st, ppart, L.nt, h);
    hipLaunchKernelGGL(k_slot_lists, dim3(L.nb), dim3(256), 0, st, nz, L.nb,
                       at<int32_t>(ws, L.slots), at<int32_t>(ws, L.nslots));
    hipLaunchKernelGGL(k_tile_lists, dim3(1), dim3(1024), 0, st, nz, L.nt,
                       at<int32_t>(ws, L.tlist), at<int32_t>(ws, L.tcount));
  };

  if (dis) {
    // given dissimilarities: no coordinates, so no ordering tree; the squared
    // rows take the place of the contraction
    for (int b0 = 0; b0 < L.nb; b0 += L.cal_group) {
      for (int b = b0; b < group_end(b0); ++b)
        hipLaunchKernelGGL(k_dissim_block, dim3((unsigned)(L.npad / 256), T / 16), dim3(256), 0,
                           st, dis, L.n, L.npad, b, slot(b), h);
      calibrate(b0);
      for (int b = b0; b < group_end(b0); ++b)
        hipLaunchKernelGGL(k_stage, dim3(L.nb - b, kStageSplit), dim3(256), 0, st, slot(b),
                           L.npad, L.nb, b, P);
    }
    pack();
    return hipGetLastError();
  }
  const double *xc = xcT, *nrm = norms;
  if (reorder && !stats_only && L.nb >= 2 && L.d <= kTreeMaxD) {
    // Internal order: bisection tree over the centred X, then X in that order.
    uint64_t *keys = at<uint64_t>(ws, L.keys);
    int32_t *vals = at<int32_t>(ws, L.vals);
    // tree scratch in the (still idle) distance block: w per row, chunk
    // partial sums, segment means and directions (each at most nb x d)
    double *wbuf = reinterpret_cast<double *>(dblock);
    double *part = wbuf + L.npad;
    double *segmean = part + (size_t)L.nb * L.d;
    double *segv = segmean + (size_t)L.nb * L.d;
    const unsigned ngrid = (unsigned)((L.n + 255) / 256);
    const int64_t blk = L.npow2 < kSortBlock ? L.npow2 : kSortBlock;
    int levels = 0;
    while ((1 << levels) < L.nb) ++levels;
    for (int lev = 0; lev < levels; ++lev) {
      const int32_t S = 1 << lev;
      int32_t C = kTreeTargetGroups / S;
      if (C > L.nb / S) C = L.nb / S;  // at least a tile of rows per chunk on average
      if (C < 1) C = 1;
      const dim3 chunks((unsigned)(S * C)), segs((unsigned)S), tb(kTreeThreads);
      hipLaunchKernelGGL(k_tree_partial<0>, chunks, tb, 0, st, xcT, L.npad, L.d, L.n, L.nb, lev, C,
                         perm, segmean, segv, wbuf, part);
      hipLaunchKernelGGL(k_tree_reduce<0>, segs, tb, 0, st, part, L.d, L.n, L.nb, lev, C, segmean,
                         segv);
      for (int it = 0; it < kTreePowerIters; ++it) {
        hipLaunchKernelGGL(k_tree_partial<1>, chunks, tb, 0, st, xcT, L.npad, L.d, L.n, L.nb, lev,
                           C, perm, segmean, segv, wbuf, part);
        hipLaunchKernelGGL(k_tree_reduce<1>, segs, tb, 0, st, part, L.d, L.n, L.nb, lev, C,
                           segmean, segv);
      }
      hipLaunchKernelGGL(k_tree_keys, chunks, tb, 0, st, xcT, L.npad, L.d, L.n, L.nb, lev, C, perm,
                         segmean, segv, keys, vals);
      if (L.npow2 > L.n)
        hipLaunchKernelGGL(k_tree_pad, dim3((unsigned)((L.npow2 - L.n + 255) / 256)), dim3(256),
                           0, st, L.n, L.npow2, keys, vals);
      const unsigned nblk = (unsigned)(L.npow2 / blk);
      hipLaunchKernelGGL(k_bitonic_local, dim3(nblk), dim3(1024), 0, st, keys, vals, blk,
                         (int64_t)0);
      for (int64_t k = 2 * blk; k <= L.npow2; k <<= 1) {
        for (int64_t j = k >> 1; j >= blk; j >>= 1)
          hipLaunchKernelGGL(k_bitonic, dim3((unsigned)(L.npow2 / 256)), dim3(256), 0, st, keys,
                             vals, L.npow2, j, k);
        hipLaunchKernelGGL(k_bitonic_local, dim3(nblk), dim3(1024), 0, st, keys, vals, blk, k);
      }
      hipLaunchKernelGGL(k_tree_apply, dim3(ngrid), dim3(256), 0, st, vals, L.n, perm);
    }
    hipLaunchKernelGGL(k_inverse, dim3(pgrid), dim3(256), 0, st, perm, L.npad, inv);
    double *xcT2 = at<double>(ws, L.xcT2), *norms2 = at<double>(ws, L.norms2);
    hipLaunchKernelGGL(k_permute_x, dim3(pgrid), dim3(256), 0, st, xcT, norms, perm, L.n, L.npad,
                       L.dpad, xcT2, norms2);
    xc = xcT2;
    nrm = norms2;
  }
  // Distances, calibration and staging block by block, then P.
  prep(xc);
  for (int b0 = 0; b0 < L.nb; b0 += L.cal_group) {
    for (int b = b0; b < group_end(b0); ++b) dist(b, xc, nrm);
    calibrate(b0);
    if (!stats_only && !implicit && !staged)
      for (int b = b0; b < group_end(b0); ++b)
        hipLaunchKernelGGL(k_stage, dim3(L.nb - b, kStageSplit), dim3(256), 0, st, slot(b),
                           L.npad, L.nb, b, P);
  }
  if (implicit) {
    // every pass rebuilds P from the contraction operands in the internal
    // order: the prepared ones of a reduced mode stay where prep() wrote
    // them; the FP64 mode reads the centred X from the second buffer (the
    // identity order copies it there)
    if (L.mode == TSNE_DIST_FP64 && xc != at<double>(ws, L.xcT2))
      hipLaunchKernelGGL(k_permute_x, dim3(pgrid), dim3(256), 0, st, xcT, norms, perm, L.n,
                         L.npad, L.dpad, at<double>(ws, L.xcT2), at<double>(ws, L.norms2));
    const int64_t m = L.nt > L.nb ? L.nt : L.nb;
    hipLaunchKernelGGL(k_implicit_init, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                       at<uint8_t>(ws, L.nz), L.nt, at<int32_t>(ws, L.nslots), L.nb, h);
    hipLaunchKernelGGL(k_set_ready, dim3(1), dim3(64), 0, st, h, 2);
    hipError_t e = launch_implicit_discover(L, ws, st);
    if (e != hipSuccess) return e;
  } else if (!stats_only) {
    pack();
  }
  return hipGetLastError();
}

template <bool PACK>
static void launch_tdist(const Layout &L, void *ws, int64_t tile0, int64_t count,
                         int64_t tile_base, bool skip_zero, hipStream_t st) {
  const Hdr *h = at<const Hdr>(ws, L.hdr);
  const int32_t key = implicit_key(L.d, L.mode);
  const uint8_t *nz = at<const uint8_t>(ws, L.nz);
  float *Pb = at<float>(ws, L.P);
  const float *norms32 = at<const float>(ws, L.norms32);
  const float *ra = at<const float>(ws, L.a), *rm = at<const float>(ws, L.m),
              *rr = at<const float>(ws, L.r);
  const dim3 g4((unsigned)count, T / 64);
  switch (L.mode) {
    case TSNE_DIST_FP32:
      hipLaunchKernelGGL(k_tdist_f32<PACK>, g4, dim3(256), 0, st, at<const float>(ws, L.xfT),
                         norms32, L.npad, L.dpad, L.nb, tile0, tile_base, Pb, h, L.n, key, nz,
                         skip_zero, ra, rm, rr);
      break;
    case TSNE_DIST_BF16:
      hipLaunchKernelGGL((k_tdist_lp<__bf16, v8bf, false, PACK>), g4, dim3(256), 0, st,
                         at<const __bf16>(ws, L.xa), norms32, L.kk,
                         L.nb, tile0, tile_base, Pb, h, L.n, key, nz, skip_zero, ra, rm, rr);
      break;
    case TSNE_DIST_FP16:
      hipLaunchKernelGGL((k_tdist_lp<_Float16, v8h, true, PACK>), g4, dim3(256), 0, st,
                         at<const _Float16>(ws, L.xa), norms32,
                         L.kk, L.nb, tile0, tile_base, Pb, h, L.n, key, nz, skip_zero, ra, rm, rr);
      break;
    case TSNE_DIST_BF16X3:
      hipLaunchKernelGGL((k_tdist_x3<__bf16, v8bf, PACK>), g4, dim3(256), 0, st,
                         at<const __bf16>(ws, L.xa), at<const float2>(ws, L.norms32), L.kk / 4,
                         x3_bits(L.kk / 4, true), L.nb, tile0, tile_base, Pb, h, L.n, key, nz,
                         skip_zero, ra, rm, rr);
      break;
    case TSNE_DIST_FP16X3:
      hipLaunchKernelGGL((k_tdist_x3<_Float16, v8h, PACK>), g4, dim3(256), 0, st,
                         at<const _Float16>(ws, L.xa), at<const float2>(ws, L.norms32), L.kk / 4,
                         x3_bits(L.kk / 4, false), L.nb, tile0, tile_base, Pb, h, L.n, key, nz,
                         skip_zero, ra, rm, rr);
      break;
    default:
      hipLaunchKernelGGL(k_tdist_f64<PACK>,
                         dim3((unsigned)count, (T / 64) * (T / (64 * kTileCT))), dim3(256), 0, st,
                         at<const double>(ws, L.xcT2), at<const double>(ws, L.norms2), L.npad,
                         L.dpad, L.nb, tile0, tile_base, Pb, h, L.n, key, nz, skip_zero, ra, rm,
                         rr);
  }
}

hipError_t launch_implicit_tiles(const Layout &L, void *ws, int64_t tile0, int64_t count,
                                 int64_t tile_base, bool skip_zero, bool pack, hipStream_t st) {
  if (pack)
    launch_tdist<true>(L, ws, tile0, count, tile_base, skip_zero, st);
  else
    launch_tdist<false>(L, ws, tile0, count, tile_base, skip_zero, st);
  return hipGetLastError();
}

// Pack (Eq. 3) the tiles tile0 .. tile0 + count - 1 of the buffer, with their
// sums, flags and coordinates.
static hipError_t launch_implicit_pack(const Layout &L, void *ws, int64_t tile0, int64_t count,
                                       int64_t tile_base, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_range, dim3((unsigned)count), dim3(256), 0, st, at<float4>(ws, L.P),
                     at<const float>(ws, L.a), at<const float>(ws, L.m), at<const float>(ws, L.r),
                     L.n, L.nb, at<double2>(ws, L.ppart), at<uint8_t>(ws, L.nz),
                     at<int2>(ws, L.tmap), tile0, tile_base, at<const Hdr>(ws, L.hdr),
                     implicit_key(L.d, L.mode));
  return hipGetLastError();
}

// The end of the affinity stage of implicit P: one pass over every tile
// (distances, stage, pack) finds the zero tiles, the sums of P and the tile
// coordinates; P is the same in every later pass, so those passes recompute
// only the nonzero tiles and take the all-zero ones with the repulsion-only
// body, as the stored path does.
hipError_t launch_implicit_discover(const Layout &L, void *ws, hipStream_t st) {
  const int64_t cap = implicit_capacity(L);
  for (int b0 = 0; b0 < L.nb;) {
    int b1 = b0 + 1;
    while (b1 < L.nb && tile_start(b1 + 1, L.nb) - tile_start(b0, L.nb) <= cap) ++b1;
    const int64_t base = tile_start(b0, L.nb), count = tile_start(b1, L.nb) - base;
    hipError_t e = launch_implicit_tiles(L, ws, base, count, base, false, false, st);
    if (e != hipSuccess) return e;
    e = launch_implicit_pack(L, ws, base, count, base, st);
    if (e != hipSuccess) return e;
    b0 = b1;
  }
  uint8_t *nz = at<uint8_t>(ws, L.nz);
  hipLaunchKernelGGL(k_implicit_sums, dim3(1), dim3(1024), 0, st, at<const double2>(ws, L.ppart),
                     L.nt, L.n, implicit_key(L.d, L.mode), at<Hdr>(ws, L.hdr));
  hipLaunchKernelGGL(k_slot_lists, dim3(L.nb), dim3(256), 0, st, nz, L.nb,
                     at<int32_t>(ws, L.slots), at<int32_t>(ws, L.nslots));
  hipLaunchKernelGGL(k_tile_lists, dim3(1), dim3(1024), 0, st, nz, L.nt,
                     at<int32_t>(ws, L.tlist), at<int32_t>(ws, L.tcount));
  return hipGetLastError();
}

void small_entry(const Layout &L, void *ws, const float *x, double perplexity, SmallEntry &e) {
  e.x = x;
  e.n = L.n;
  e.nt = L.nt;
  e.d = L.d;
  e.nb = L.nb;
  e.perplexity = perplexity;
  e.h = at<Hdr>(ws, L.hdr);
  e.a = at<float>(ws, L.a);
  e.m = at<float>(ws, L.m);
  e.r = at<float>(ws, L.r);
  e.beta = at<double>(ws, L.beta);
  e.S = at<double>(ws, L.S);
  e.H = at<double>(ws, L.H);
  e.evals = at<int32_t>(ws, L.evals);
  e.P = at<float4>(ws, L.P);
  e.ppart = at<double2>(ws, L.ppart);
  e.nz = at<uint8_t>(ws, L.nz);
  e.tmap = at<int2>(ws, L.tmap);
  e.tlist = at<int32_t>(ws, L.tlist);
  e.tcount = at<int32_t>(ws, L.tcount);
  e.slots = at<int32_t>(ws, L.slots);
  e.nslots = at<int32_t>(ws, L.nslots);
  e.perm = at<int32_t>(ws, L.perm);
  e.inv = at<int32_t>(ws, L.inv);
}

hipError_t launch_affinities_small(const SmallEntry *tab, int count, int64_t wgs, int64_t tiles,
                                   int64_t blocks, int64_t nmax, int32_t dmax, int max_bisect,
                                   double tol_h, hipStream_t st) {
  if (nmax > kSmallMaxN || dmax > kSmallMaxD || count < 1) return hipErrorInvalidValue;
  const int32_t dstride = dmax | 1;  // odd row stride: conflict-free LDS reads
  const size_t lds = (size_t)(2 * 64 + kSmallRows) * dstride * sizeof(double);
  hipLaunchKernelGGL(k_small_init, dim3((unsigned)blocks), dim3(256), 0, st, tab, count);
  const dim3 g((unsigned)wgs), b(kSmallRows * 64);
  const int vpt = (int)((nmax + 63) / 64);
  if (vpt <= 4)
    hipLaunchKernelGGL(k_small_calibrate<4>, g, b, lds, st, tab, count, dstride, max_bisect, tol_h);
  else if (vpt <= 8)
    hipLaunchKernelGGL(k_small_calibrate<8>, g, b, lds, st, tab, count, dstride, max_bisect, tol_h);
  else if (vpt <= 16)
    hipLaunchKernelGGL(k_small_calibrate<16>, g, b, lds, st, tab, count, dstride, max_bisect,
                       tol_h);
  else if (vpt <= 32)
    hipLaunchKernelGGL(k_small_calibrate<32>, g, b, lds, st, tab, count, dstride, max_bisect,
                       tol_h);
  else
    hipLaunchKernelGGL(k_small_calibrate<64>, g, b, lds, st, tab, count, dstride, max_bisect,
                       tol_h);
  hipLaunchKernelGGL(k_small_pack, dim3((unsigned)tiles), dim3(256), 0, st, tab, count);
  hipLaunchKernelGGL(k_small_slots, dim3((unsigned)blocks), dim3(256), 0, st, tab, count);
  hipLaunchKernelGGL(k_small_lists, dim3((unsigned)count), dim3(1024), 0, st, tab);
  return hipGetLastError();
}

hipError_t launch_export_p_rows(const Layout &L, void *ws, int64_t row0, int64_t nrows,
                                float *out, hipStream_t st) {
  const int64_t total = nrows * L.n;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_export_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     at<const float4>(ws, L.P), L.n, L.nb, row0, nrows,
                     at<const int32_t>(ws, L.inv), out, at<Hdr>(ws, L.hdr));
  return hipGetLastError();
}

hipError_t launch_export_rowstats(const Layout &L, void *ws, double *beta, float *m, double *S,
                                  double *H, int32_t *evals, hipStream_t st) {
  hipLaunchKernelGGL(k_export_stats, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, st, L.n,
                     at<const double>(ws, L.beta), at<const float>(ws, L.m),
                     at<const double>(ws, L.S), at<const double>(ws, L.H),
                     at<const int32_t>(ws, L.evals), at<const int32_t>(ws, L.inv), beta, m, S, H,
                     evals, at<Hdr>(ws, L.hdr));
  return hipGetLastError();
}

hipError_t launch_export_order(const Layout &L, void *ws, int32_t *perm, uint8_t *flags,
                               hipStream_t st) {
  const int64_t m = L.n > L.nt ? L.n : L.nt;
  hipLaunchKernelGGL(k_export_order, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                     at<const Hdr>(ws, L.hdr), L.n, L.nt, at<const int32_t>(ws, L.perm),
                     at<const uint8_t>(ws, L.nz), perm, flags);
  return hipGetLastError();
}

hipError_t launch_export_scalars(const Layout &L, void *ws, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_export_scalars, dim3(1), dim3(64), 0, st, L.n, at<const Hdr>(ws, L.hdr),
                     out);
  return hipGetLastError();
}

}  // namespace tsne
