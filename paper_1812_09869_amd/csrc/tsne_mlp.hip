// Surrogate network on the GPU: 50 -> 256 -> 256 -> 2 (d_in -> H -> H -> 2),
// ReLU, trained by mean squared error to map input points to their t-SNE
// embedding, with BF16 MFMA contractions (FP32 accumulation) for the two wide
// layers and FP32 VALU for the 2-wide output layer.
//
// Packed FP32 parameters: W1 [H][d_in], b1 [H], W2 [H][H], b2 [H], W3 [2][H],
// b3 [2]. Inputs are standardised ((x - mean) * invstd) and rounded to BF16;
// W1 and W2 are rounded to BF16 copies before each pass; hidden activations
// are kept in FP32 and rounded to BF16 where they feed a contraction.
#include <math.h>

#include <mutex>

#include "tsne_internal.h"
#include "tsne_mlp.h"

namespace tsne {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kK1 = 64;  // d_in rounded up to the MFMA K step (d_in <= 64)

// ----------------------------------------------------------------------------
// Generic C[M][N] = sum_k A[m][k] B[n][k] on v_mfma_f32_16x16x32_bf16 with a
// fused epilogue. One wave computes a 64 x 64 block (4 x 4 MFMA tiles); lane l
// supplies rows l%16 of A and B with k-slice 8(l/16) .. 8(l/16)+7 and receives
// D[4(l/16) + r][l%16] in element r. M, N multiples of 64, K of 32.
// ----------------------------------------------------------------------------
struct Epi {
  const float *bias;   // per column n, or null
  int relu;            // max(v, 0)
  const float *mask;   // keep v only where mask[m * ldm + n] > 0, or null
  int ldm;
  float *outF;         // FP32 result [m * ldf + n] for n < nvalid, or null
  int ldf, nvalid;
  __bf16 *outB;        // BF16 result [m * ldb + n], or null
  int ldb;
  __bf16 *outBT;       // BF16 transposed result [n * ldt + m], or null
  int ldt;
};

// KW waves per workgroup split K evenly (K / KW a multiple of 32); their
// 64 x 64 partial results meet in LDS and wave 0 adds them in wave order
// (a fixed order) before the epilogue.
template <int KW>
__global__ __launch_bounds__(64 * KW) void k_gemm_bf16(const __bf16 *__restrict__ A, int lda,
                                                       const __bf16 *__restrict__ Bm, int ldbm,
                                                       int K, Epi e) {
  __shared__ v4f red[KW > 1 ? KW - 1 : 1][16][64];
  const int64_t m0 = (int64_t)blockIdx.x * 64;
  const int n0 = blockIdx.y * 64;
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, li = l & 15, lk = l >> 4;
  v4f acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = (v4f){0.f, 0.f, 0.f, 0.f};
  const int kpw = K / KW;
  for (int k0 = wv * kpw; k0 < (wv + 1) * kpw; k0 += 32) {
    v8bf av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      av[a] = *reinterpret_cast<const v8bf *>(A + (m0 + a * 16 + li) * lda + k0 + 8 * lk);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      bv[c] = *reinterpret_cast<const v8bf *>(Bm + (int64_t)(n0 + c * 16 + li) * ldbm + k0 +
                                              8 * lk);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[c], acc[a][c], 0, 0, 0);
  }
  if (KW > 1) {
    if (wv > 0) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) red[wv - 1][4 * a + c][l] = acc[a][c];
    }
    __syncthreads();
    if (wv > 0) return;
    for (int w = 0; w < KW - 1; ++w)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] += red[w][4 * a + c][l];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + a * 16 + 4 * lk + r;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int n = n0 + c * 16 + li;
        float v = acc[a][c][r];
        if (e.bias) v += e.bias[n];
        if (e.relu) v = fmaxf(v, 0.f);
        if (e.mask && !(e.mask[m * e.ldm + n] > 0.f)) v = 0.f;
        if (e.outF && n < e.nvalid) e.outF[m * e.ldf + n] = v;
        if (e.outB) e.outB[m * e.ldb + n] = (__bf16)v;
        if (e.outBT) e.outBT[(int64_t)n * e.ldt + m] = (__bf16)v;
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Fused inference. A persistent workgroup of W waves keeps the weights in
// registers and runs tiles of kInferRows rows through the whole network:
//
//   wave w owns hidden units [H/W w, H/W (w + 1)) of both wide layers: its
//   row slices of W1 and W2 (the A operands of the two transposed layers)
//   stay in registers for the life of the workgroup;
//   the standardised BF16 input tile and the BF16 first-layer output tile
//   live in LDS, shared by the W waves;
//   the output layer's partial sums of the W waves meet in LDS.
//
// Both wide layers are computed transposed, H1^T = W1 X^T and H2^T = W2 H1^T
// (M = hidden, N = rows). The B operand of either is one 16-byte LDS read of
// eight consecutive inputs of one row, and lane l = 16g + c receives
// H^T[h0 + 16i + 4g + r][16a + c]: four consecutive hidden units of row
// 16a + c. The first layer's four go to LDS as one 8-byte write; the second
// layer's are summed into the output layer in place, so the sum over a wave's
// hidden units needs only the four lanes of a column (two cross-lane steps).
//
// The next tile's inputs are loaded into registers at the start of a tile and
// written to LDS after its second layer, so the loads have most of a tile's
// time to arrive; the second layer's LDS reads run one K step ahead of its
// MFMAs (explicit double buffer plus scheduling groups of one read per TW
// MFMAs).
// ----------------------------------------------------------------------------
constexpr int kInferRows = 64;   // rows per tile
constexpr int kXPitch = kK1 + 8;  // BF16 elements per LDS row of the input tile

typedef __bf16 v4bf __attribute__((ext_vector_type(4)));

__device__ inline float row16_sum_f(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x124, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x122, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x121, 0xf, 0xf, true));
  return v;
}

// v + (v of lane l ^ 32) and v + (v of lane l ^ 16) in every lane, with the
// gfx950 lane-swap instructions (VALU, no LDS crossbar): permlane32_swap(v, v)
// leaves the two halves of the wave in its two results, permlane16_swap(v, v)
// the even and odd rows of 16.
__device__ inline float add_xor32(float v) {
  const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                  false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
__device__ inline float add_xor16(float v) {
  const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                  false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}

template <int H, int W>
__global__ __launch_bounds__(64 * W, 1) void k_mlp_infer(
    const float *__restrict__ x, int64_t n, int d_in, const float *__restrict__ mean,
    const float *__restrict__ invstd, const __bf16 *__restrict__ w1b,
    const float *__restrict__ b1, const __bf16 *__restrict__ w2b, const float *__restrict__ b2,
    const float *__restrict__ w3, const float *__restrict__ b3, float *__restrict__ out) {
  constexpr int NT = 64 * W;         // threads
  constexpr int HW = H / W;          // hidden units per wave
  constexpr int TW = HW / 16;        // hidden tiles per wave
  constexpr int KS = H / 32;         // K steps of layer 2
  constexpr int RA = kInferRows / 16;  // row tiles
  constexpr int HPitch = H + 8;      // BF16 elements per LDS row of the hidden tile
  __shared__ __bf16 xs[kInferRows][kXPitch];
  __shared__ __bf16 hs[kInferRows][HPitch];
  __shared__ float po[W][kInferRows][2];
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int c = l & 15, g = l >> 4;
  const int h0 = w * HW;  // first hidden unit of this wave
  v8bf wa[TW][2];  // W1 rows h0 + 16i + c, inputs 32s + 8g .. + 7
#pragma unroll
  for (int i = 0; i < TW; ++i)
#pragma unroll
    for (int st = 0; st < 2; ++st)
      wa[i][st] = *reinterpret_cast<const v8bf *>(w1b + (h0 + 16 * i + c) * kK1 + 32 * st + 8 * g);
  v8bf wb[TW][KS];  // W2 rows h0 + 16e + c, inputs 32s + 8g .. + 7
#pragma unroll
  for (int e = 0; e < TW; ++e)
#pragma unroll
    for (int st = 0; st < KS; ++st)
      wb[e][st] = *reinterpret_cast<const v8bf *>(w2b + (int64_t)(h0 + 16 * e + c) * H + 32 * st + 8 * g);
  float bias1[TW][4], bias2[TW][4], u0[TW][4], u1[TW][4];
#pragma unroll
  for (int i = 0; i < TW; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = h0 + 16 * i + 4 * g + r;
      bias1[i][r] = b1[j];
      bias2[i][r] = b2[j];
      u0[i][r] = w3[j];
      u1[i][r] = w3[H + j];
    }
  const float c0 = b3[0], c1 = b3[1];
  const int64_t ntiles = (n + kInferRows - 1) / kInferRows;
  // the input tile: each thread loads two adjacent columns (xk, xk + 1) of
  // XM rows and stores them as one 32-bit LDS write
  constexpr int XM = kInferRows * kK1 / NT / 2;
  constexpr int RS = NT / (kK1 / 2);  // rows covered per step
  const int xk = 2 * (t & (kK1 / 2 - 1)), xr = t / (kK1 / 2);
  const bool kin0 = xk < d_in, kin1 = xk + 1 < d_in;
  const int xkc0 = kin0 ? xk : d_in - 1, xkc1 = kin1 ? xk + 1 : d_in - 1;  // padding lanes load a real element and store 0
  const float xmean0 = kin0 ? mean[xk] : 0.f, xinv0 = kin0 ? invstd[xk] : 0.f;
  const float xmean1 = kin1 ? mean[xk + 1] : 0.f, xinv1 = kin1 ? invstd[xk + 1] : 0.f;
  float xv[XM][2];
  auto load_x = [&](int64_t tl) {
    if (tl >= ntiles) return;
    const float *xt = x + tl * kInferRows * d_in;  // uniform tile base
    const int64_t lim = n - tl * kInferRows;       // rows of this tile that exist
    if (lim >= kInferRows) {
#pragma unroll
      for (int m = 0; m < XM; ++m) {
        xv[m][0] = xt[(xr + RS * m) * d_in + xkc0];
        xv[m][1] = xt[(xr + RS * m) * d_in + xkc1];
      }
    } else {
#pragma unroll
      for (int m = 0; m < XM; ++m) {
        const int rl = xr + RS * m;
        xv[m][0] = rl < lim ? xt[rl * d_in + xkc0] : 0.f;
        xv[m][1] = rl < lim ? xt[rl * d_in + xkc1] : 0.f;
      }
    }
  };
  auto store_x = [&]() {
#pragma unroll
    for (int m = 0; m < XM; ++m) {
      typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
      v2bf pr;
      pr[0] = (__bf16)((xv[m][0] - xmean0) * xinv0);  // 0 in padding lanes
      pr[1] = (__bf16)((xv[m][1] - xmean1) * xinv1);
      *reinterpret_cast<v2bf *>(&xs[xr + RS * m][xk]) = pr;
    }
  };
  load_x(blockIdx.x);
  store_x();
  __syncthreads();
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * kInferRows;
    load_x(tile + gridDim.x);
    v4f acc1[TW][RA];
#pragma unroll
    for (int i = 0; i < TW; ++i)
#pragma unroll
      for (int a = 0; a < RA; ++a) acc1[i][a] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int a = 0; a < RA; ++a) {
        const v8bf xb = *reinterpret_cast<const v8bf *>(&xs[16 * a + c][32 * st + 8 * g]);
#pragma unroll
        for (int i = 0; i < TW; ++i)
          acc1[i][a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[i][st], xb, acc1[i][a], 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < TW; ++i)
#pragma unroll
      for (int a = 0; a < RA; ++a) {
        v4bf hv;
#pragma unroll
        for (int r = 0; r < 4; ++r) hv[r] = (__bf16)fmaxf(acc1[i][a][r] + bias1[i][r], 0.f);
        *reinterpret_cast<v4bf *>(&hs[16 * a + c][h0 + 16 * i + 4 * g]) = hv;
      }
    __syncthreads();
    // layer 2, transposed: acc2[e][a] = H2^T[h0 + 16e + 4g + r][16a + c]
    v4f acc2[TW][RA];
#pragma unroll
    for (int e = 0; e < TW; ++e)
#pragma unroll
      for (int a = 0; a < RA; ++a) acc2[e][a] = (v4f){0.f, 0.f, 0.f, 0.f};
    v8bf hb[2][RA];
#pragma unroll
    for (int a = 0; a < RA; ++a) hb[0][a] = *reinterpret_cast<const v8bf *>(&hs[16 * a + c][8 * g]);
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      if (st + 1 < KS) {
#pragma unroll
        for (int a = 0; a < RA; ++a)
          hb[(st + 1) & 1][a] = *reinterpret_cast<const v8bf *>(&hs[16 * a + c][32 * (st + 1) + 8 * g]);
      }
#pragma unroll
      for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int e = 0; e < TW; ++e)
          acc2[e][a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[e][st], hb[st & 1][a], acc2[e][a], 0, 0, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x100, RA, 0);
#pragma unroll
    for (int q = 0; q < (KS - 1) * RA; ++q) {
      __builtin_amdgcn_sched_group_barrier(0x008, TW, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, TW * RA, 0);
    // output layer: lane (c, g) holds 4 TW hidden units of row 16a + c
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int e = 0; e < TW; ++e)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float hh = fmaxf(acc2[e][a][r] + bias2[e][r], 0.f);
          s0 = fmaf(u0[e][r], hh, s0);
          s1 = fmaf(u1[e][r], hh, s1);
        }
      s0 = add_xor32(s0);
      s1 = add_xor32(s1);
      s0 = add_xor16(s0);
      s1 = add_xor16(s1);
      po[w][16 * a + c][0] = s0;  // the four lanes of a column hold the same sums
      po[w][16 * a + c][1] = s1;
    }
    __builtin_amdgcn_sched_barrier(0);
    store_x();
    __syncthreads();
    if (t < kInferRows * 2) {
      const int rr = t >> 1, o = t & 1;
      const int64_t row = row0 + rr;
      float sum = 0.f;
#pragma unroll
      for (int q = 0; q < W; ++q) sum += po[q][rr][o];
      if (row < n) out[2 * row + o] = sum + (o ? c1 : c0);
    }
  }
}


// BF16 copies of W1 (zero-padded to [H][kK1]), W2 and W2 transposed.
__global__ void k_mlp_cast(const float *__restrict__ p, int d_in, int H, __bf16 *__restrict__ w1b,
                           __bf16 *__restrict__ w2b, __bf16 *__restrict__ w2tb) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const float *w1 = p, *w2 = p + (int64_t)H * d_in + H;
  if (i < (int64_t)H * kK1) {
    const int j = (int)(i / kK1), k = (int)(i % kK1);
    w1b[i] = (__bf16)(k < d_in ? w1[(int64_t)j * d_in + k] : 0.f);
  }
  if (i < (int64_t)H * H) {
    const int j = (int)(i / H), k = (int)(i % H);
    const __bf16 v = (__bf16)w2[i];
    w2b[i] = v;
    w2tb[(int64_t)k * H + j] = v;
  }
}

// Standardised BF16 inputs for a batch (rows idx[b] of x, or rows row0 + b).
__global__ void k_mlp_gather(const float *__restrict__ x, int d_in, const float *__restrict__ mean,
                             const float *__restrict__ invstd, const int32_t *__restrict__ idx,
                             int64_t row0, int64_t B, int64_t Bpad, const float *__restrict__ y,
                             __bf16 *__restrict__ xb, __bf16 *__restrict__ xbt,
                             float *__restrict__ yb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;  // one (row, input) element
  if (e >= Bpad * kK1) return;
  const int64_t b = e / kK1;
  const int k = (int)(e % kK1);
  const bool ok = b < B;
  const int64_t r = ok ? (idx ? (int64_t)idx[b] : row0 + b) : 0;
  float v = 0.f;
  if (ok && k < d_in) v = (x[r * d_in + k] - mean[k]) * invstd[k];
  const __bf16 hv = (__bf16)v;
  xb[e] = hv;
  if (xbt) xbt[(int64_t)k * Bpad + b] = hv;
  if (yb && k < 2) yb[2 * b + k] = ok ? y[2 * r + k] : 0.f;
}

// Output layer of a training batch and its backward pass: out = W3 h2 + b3
// (FP32), dout = (out - y) / B_total, per-row loss 0.5 |out - y|^2 summed per
// workgroup, dh2 = (W3^T dout) masked by h2 > 0 (FP32, BF16 and BF16
// transposed). Sixteen threads per row, each covering H / 16 consecutive
// hidden units; the two outputs are summed over the 16 lanes of a DPP row.
__global__ __launch_bounds__(256) void k_mlp_head(
    const float *__restrict__ h2, int H, const float *__restrict__ w3, const float *__restrict__ b3,
    int64_t B, int64_t Bpad, const float *__restrict__ yb, double inv_batch,
    float *__restrict__ dout, float *__restrict__ dh2, __bf16 *__restrict__ dh2b,
    __bf16 *__restrict__ dh2t, double *__restrict__ loss_part) {
  __shared__ double red[4];
  const int t = threadIdx.x, p = t & 15;
  const int64_t b = (int64_t)blockIdx.x * 16 + (t >> 4);  // < Bpad: the grid is Bpad / 16
  const int per = H / 16, k0 = p * per;
  const float *hr = h2 + b * H + k0;
  float o0 = 0.f, o1 = 0.f;
  for (int j = 0; j < per; ++j) {
    const float h = hr[j];
    o0 = fmaf(w3[k0 + j], h, o0);
    o1 = fmaf(w3[H + k0 + j], h, o1);
  }
  o0 = row16_sum_f(o0) + b3[0];
  o1 = row16_sum_f(o1) + b3[1];
  float d0 = 0.f, d1 = 0.f;
  double lsum = 0.0;
  if (b < B) {
    const float e0 = o0 - yb[2 * b], e1 = o1 - yb[2 * b + 1];
    if (p == 0) lsum = 0.5 * ((double)e0 * e0 + (double)e1 * e1);
    d0 = (float)(e0 * inv_batch);
    d1 = (float)(e1 * inv_batch);
  }
  if (p == 0) {
    dout[2 * b] = d0;
    dout[2 * b + 1] = d1;
  }
  for (int j = 0; j < per; ++j) {
    const int k = k0 + j;
    float g = fmaf(d0, w3[k], d1 * w3[H + k]);
    if (!(hr[j] > 0.f)) g = 0.f;
    dh2[b * H + k] = g;
    dh2b[b * H + k] = (__bf16)g;
    dh2t[(int64_t)k * Bpad + b] = (__bf16)g;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
  if ((t & 63) == 0) red[t >> 6] = lsum;
  __syncthreads();
  if (t == 0) loss_part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Column sums over the batch, out[n] = sum_b wgt(b) D[b][n] with wgt(b) = 1
// or w[b * wstride]: kColChunks chunks of rows summed in parallel (four
// independent accumulators per thread), then the chunks added in order.
// Several independent sums share one launch (blockIdx.z picks the job).
constexpr int kColChunks = 32;
constexpr int kColJobs = 4;

struct ColJob {
  const float *D;
  const float *w;
  float *part;  // [kColChunks][N]
  float *out;   // [N]
  int ldd, wstride, N;
};
struct ColJobs {
  ColJob j[kColJobs];
};

__global__ __launch_bounds__(256) void k_colsum_part(ColJobs jobs, int64_t B) {
  const ColJob &jb = jobs.j[blockIdx.z];
  const int n = blockIdx.x * 256 + threadIdx.x, ch = blockIdx.y;
  if (!jb.D || n >= jb.N) return;
  const int64_t b0 = B * ch / kColChunks, b1 = B * (ch + 1) / kColChunks;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  int64_t b = b0;
  for (; b + 3 < b1; b += 4) {
    const float d0 = jb.D[b * jb.ldd + n], d1 = jb.D[(b + 1) * jb.ldd + n];
    const float d2 = jb.D[(b + 2) * jb.ldd + n], d3 = jb.D[(b + 3) * jb.ldd + n];
    if (jb.w) {
      s0 = fmaf(jb.w[b * jb.wstride], d0, s0);
      s1 = fmaf(jb.w[(b + 1) * jb.wstride], d1, s1);
      s2 = fmaf(jb.w[(b + 2) * jb.wstride], d2, s2);
      s3 = fmaf(jb.w[(b + 3) * jb.wstride], d3, s3);
    } else {
      s0 += d0;
      s1 += d1;
      s2 += d2;
      s3 += d3;
    }
  }
  for (; b < b1; ++b) {
    const float d = jb.D[b * jb.ldd + n];
    s0 = jb.w ? fmaf(jb.w[b * jb.wstride], d, s0) : s0 + d;
  }
  jb.part[(int64_t)ch * jb.N + n] = (s0 + s1) + (s2 + s3);
}

__global__ __launch_bounds__(256) void k_colsum_fin(ColJobs jobs) {
  const ColJob &jb = jobs.j[blockIdx.z];
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (!jb.D || n >= jb.N) return;
  float s = 0.f;
  for (int ch = 0; ch < kColChunks; ++ch) s += jb.part[(int64_t)ch * jb.N + n];
  jb.out[n] = s;
}

__global__ void k_loss_reduce(const double *__restrict__ part, int nparts, double inv_batch,
                              double *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < nparts; ++q) s += part[q];
    *out = s * inv_batch;
  }
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t count, float lr, float beta1, float beta2,
                       float eps, float inv_c1, float inv_c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * inv_c1) / (sqrtf(vi * inv_c2) + eps);
}

}  // namespace

// ----------------------------------------------------------------------------
// Workspace layout for a batch of up to Bpad rows (Bpad multiple of 64)
// ----------------------------------------------------------------------------
MlpLayout make_mlp_layout(int d_in, int H, int64_t Bpad, bool train) {
  MlpLayout L;
  L.d_in = d_in;
  L.H = H;
  L.Bpad = Bpad;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = (o + bytes + 255) / 256 * 256;
    return at;
  };
  const size_t B = (size_t)Bpad, Hs = (size_t)H;
  L.w1b = take(Hs * kK1 * 2);
  L.w2b = take(Hs * Hs * 2);
  L.w2tb = take(Hs * Hs * 2);
  L.xb = take(B * kK1 * 2);
  L.h1b = take(B * Hs * 2);
  L.h2 = take(B * Hs * 4);
  L.loss_part = take((B / 16 + 1) * 8);
  if (train) {
    L.xbt = take(B * kK1 * 2);
    L.yb = take(B * 2 * 4);
    L.h1 = take(B * Hs * 4);
    L.h1t = take(B * Hs * 2);
    L.dout = take(B * 2 * 4);
    L.dh2 = take(B * Hs * 4);
    L.dh2b = take(B * Hs * 2);
    L.dh2t = take(B * Hs * 2);
    L.dh1 = take(B * Hs * 4);
    L.dh1t = take(B * Hs * 2);
    L.gw1 = take(Hs * kK1 * 4);
    L.colpart = take((size_t)kColChunks * (4 * Hs + 2) * 4);
  }
  L.total = o;
  return L;
}

static Epi epi() {
  Epi e{};
  e.nvalid = 1 << 30;
  return e;
}

// C = A B^T on (M / 64) x (N / 64) workgroups, splitting K over as many waves
// (8, 4, 2 or 1) as divide its 32-wide steps, so that short grids with long
// K still have enough loads in flight.
static void gemm(int64_t M, int N, const __bf16 *A, int lda, const __bf16 *Bm, int ldb, int K,
                 const Epi &e, hipStream_t st) {
  const dim3 grid((unsigned)(M / 64), (unsigned)(N / 64));
  const int steps = K / 32;
  const int64_t tiles = M / 64 * (N / 64);
  const int want = tiles >= 256 ? 1 : (tiles >= 64 ? 4 : 8);
  if (want >= 8 && steps % 8 == 0)
    hipLaunchKernelGGL(k_gemm_bf16<8>, grid, dim3(512), 0, st, A, lda, Bm, ldb, K, e);
  else if (want >= 4 && steps % 4 == 0)
    hipLaunchKernelGGL(k_gemm_bf16<4>, grid, dim3(256), 0, st, A, lda, Bm, ldb, K, e);
  else if (want >= 2 && steps % 2 == 0)
    hipLaunchKernelGGL(k_gemm_bf16<2>, grid, dim3(128), 0, st, A, lda, Bm, ldb, K, e);
  else
    hipLaunchKernelGGL(k_gemm_bf16<1>, grid, dim3(64), 0, st, A, lda, Bm, ldb, K, e);
}

// Forward pass of rows [row0, row0 + B) (or idx[0..B)) of x into out.
hipError_t launch_mlp_cast(const MlpLayout &L, const float *params, void *ws, hipStream_t st) {
  const int64_t cnt = (int64_t)L.H * (L.H > kK1 ? L.H : kK1);
  hipLaunchKernelGGL(k_mlp_cast, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, params,
                     L.d_in, L.H, at<__bf16>(ws, L.w1b), at<__bf16>(ws, L.w2b),
                     at<__bf16>(ws, L.w2tb));
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpLayout &L, const float *params, const float *mean,
                              const float *invstd, const float *x, int64_t n, float *out, void *ws,
                              hipStream_t st) {
  hipError_t e = launch_mlp_cast(L, params, ws, st);
  if (e != hipSuccess) return e;
  const int H = L.H;
  const float *b1 = params + (int64_t)H * L.d_in, *b2 = b1 + H + (int64_t)H * H;
  const float *w3 = b2 + H, *b3 = w3 + 2 * H;
  const __bf16 *w1b = at<const __bf16>(ws, L.w1b), *w2b = at<const __bf16>(ws, L.w2b);
  // persistent: at most one workgroup per compute unit (the weights fill the
  // registers of a wave per SIMD), fewer when there are fewer tiles
  const int64_t ntiles = (n + kInferRows - 1) / kInferRows;
  const dim3 grid((unsigned)(ntiles < 256 ? ntiles : 256));
  switch (H) {
    case 64:
      hipLaunchKernelGGL((k_mlp_infer<64, 4>), grid, dim3(256), 0, st, x, n, L.d_in, mean, invstd,
                         w1b, b1, w2b, b2, w3, b3, out);
      break;
    case 128:
      hipLaunchKernelGGL((k_mlp_infer<128, 8>), grid, dim3(512), 0, st, x, n, L.d_in, mean,
                         invstd, w1b, b1, w2b, b2, w3, b3, out);
      break;
    case 192:
      hipLaunchKernelGGL((k_mlp_infer<192, 4>), grid, dim3(256), 0, st, x, n, L.d_in, mean,
                         invstd, w1b, b1, w2b, b2, w3, b3, out);
      break;
    default:
      hipLaunchKernelGGL((k_mlp_infer<256, 8>), grid, dim3(512), 0, st, x, n, L.d_in, mean,
                         invstd, w1b, b1, w2b, b2, w3, b3, out);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Scratch of the allocation-free forward entry point: the BF16 weight copies
// of a forward pass (the whole 64-row forward layout, under 0.4 MiB for every
// supported d_in and H). One copy per device, held until the process ends and
// shared by every call on that device. Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol): the
// device address is looked up once per device, with that device current, and
// kept here.
// ----------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};
}  // namespace

hipError_t noalloc_scratch(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_mlp_gradient(const MlpLayout &L, const float *params, const float *mean,
                               const float *invstd, const float *x, const float *y,
                               const int32_t *idx, int64_t B, float *grad, double *loss,
                               void *ws, hipStream_t st) {
  const int H = L.H, d_in = L.d_in;
  const int64_t Bpad = (B + 63) / 64 * 64;
  const float *b1 = params + (int64_t)H * d_in, *b2 = b1 + H + (int64_t)H * H;
  const float *w3 = b2 + H, *b3 = w3 + 2 * H;
  float *g_w1 = grad, *g_b1 = g_w1 + (int64_t)H * d_in, *g_w2 = g_b1 + H,
        *g_b2 = g_w2 + (int64_t)H * H, *g_w3 = g_b2 + H, *g_b3 = g_w3 + 2 * H;
  __bf16 *xb = at<__bf16>(ws, L.xb), *xbt = at<__bf16>(ws, L.xbt), *h1b = at<__bf16>(ws, L.h1b),
         *h1t = at<__bf16>(ws, L.h1t), *dh2b = at<__bf16>(ws, L.dh2b),
         *dh2t = at<__bf16>(ws, L.dh2t), *dh1t = at<__bf16>(ws, L.dh1t);
  float *yb = at<float>(ws, L.yb), *h1 = at<float>(ws, L.h1), *h2 = at<float>(ws, L.h2),
        *dout = at<float>(ws, L.dout), *dh2 = at<float>(ws, L.dh2), *dh1 = at<float>(ws, L.dh1);
  double *lp = at<double>(ws, L.loss_part);
  hipError_t err = launch_mlp_cast(L, params, ws, st);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_mlp_gather, dim3((unsigned)(Bpad * kK1 / 256)), dim3(256), 0, st, x, d_in,
                     mean, invstd, idx, 0, B, Bpad, y, xb, xbt, yb);
  // forward
  Epi e1 = epi();
  e1.bias = b1;
  e1.relu = 1;
  e1.outF = h1;
  e1.ldf = H;
  e1.outB = h1b;
  e1.ldb = H;
  e1.outBT = h1t;
  e1.ldt = (int)Bpad;
  gemm(Bpad, H, xb, kK1, at<const __bf16>(ws, L.w1b), kK1, kK1, e1, st);
  Epi e2 = epi();
  e2.bias = b2;
  e2.relu = 1;
  e2.outF = h2;
  e2.ldf = H;
  gemm(Bpad, H, h1b, H, at<const __bf16>(ws, L.w2b), H, H, e2, st);
  const unsigned hgrid = (unsigned)(Bpad / 16);
  hipLaunchKernelGGL(k_mlp_head, dim3(hgrid), dim3(256), 0, st, h2, H, w3, b3, B, Bpad, yb,
                     1.0 / (double)B, dout, dh2, dh2b, dh2t, lp);
  hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(64), 0, st, lp, (int)hgrid, 1.0 / (double)B,
                     loss);
  // output layer gradients and db2: dW3[c][k] = sum_b dout[b][c] h2[b][k],
  // db3[c] = sum_b dout[b][c], db2 = colsum(dh2)
  float *cpart = at<float>(ws, L.colpart);
  const size_t cstride = (size_t)kColChunks * H;
  ColJobs jh{};
  jh.j[0] = ColJob{h2, dout, cpart, g_w3, H, 2, H};
  jh.j[1] = ColJob{h2, dout + 1, cpart + cstride, g_w3 + H, H, 2, H};
  jh.j[2] = ColJob{dh2, nullptr, cpart + 2 * cstride, g_b2, H, 0, H};
  jh.j[3] = ColJob{dout, nullptr, cpart + 4 * cstride, g_b3, 2, 0, 2};
  const unsigned cgx = (unsigned)((H + 255) / 256);
  hipLaunchKernelGGL(k_colsum_part, dim3(cgx, kColChunks, 4), dim3(256), 0, st, jh, Bpad);
  // second layer: dW2 = dh2^T h1, dh1 = (dh2 W2) masked by h1 > 0
  Epi ew2 = epi();
  ew2.outF = g_w2;
  ew2.ldf = H;
  gemm(H, H, dh2t, (int)Bpad, h1t, (int)Bpad, (int)Bpad, ew2, st);
  Epi ed1 = epi();
  ed1.mask = h1;
  ed1.ldm = H;
  ed1.outF = dh1;
  ed1.ldf = H;
  ed1.outBT = dh1t;
  ed1.ldt = (int)Bpad;
  gemm(Bpad, H, dh2b, H, at<const __bf16>(ws, L.w2tb), H, H, ed1, st);
  // first layer: dW1 = dh1^T xh (columns beyond d_in dropped), db1 = colsum(dh1)
  Epi ew1 = epi();
  ew1.outF = g_w1;
  ew1.ldf = d_in;
  ew1.nvalid = d_in;
  gemm(H, kK1, dh1t, (int)Bpad, xbt, (int)Bpad, (int)Bpad, ew1, st);
  ColJobs j1{};
  j1.j[0] = ColJob{dh1, nullptr, cpart + 3 * cstride, g_b1, H, 0, H};
  hipLaunchKernelGGL(k_colsum_part, dim3(cgx, kColChunks, 1), dim3(256), 0, st, j1, Bpad);
  ColJobs jf = jh;
  jf.j[3] = j1.j[0];
  ColJobs jb3{};
  jb3.j[0] = jh.j[3];
  hipLaunchKernelGGL(k_colsum_fin, dim3(cgx, 1, 4), dim3(256), 0, st, jf);
  hipLaunchKernelGGL(k_colsum_fin, dim3(1, 1, 1), dim3(256), 0, st, jb3);
  return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr,
                       float beta1, float beta2, float eps, int32_t t, hipStream_t st) {
  const double c1 = 1.0 - pow((double)beta1, t), c2 = 1.0 - pow((double)beta2, t);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, g, m, v,
                     count, lr, beta1, beta2, eps, (float)(1.0 / c1), (float)(1.0 / c2));
  return hipGetLastError();
}

}  // namespace tsne
