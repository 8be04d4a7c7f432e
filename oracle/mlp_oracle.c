/*
 * FP64 CPU oracle of the surrogate network (not part of the paper; the
 * learned map from input points to their t-SNE embedding).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite to check the GPU's forward
 * and backward passes and the optimiser step. Shares nothing with the HIP
 * library.
 *
 * Network: 50 -> 256 -> 256 -> 2 (d_in -> H -> H -> 2 in general), ReLU:
 *   xh = (x - mean) * invstd
 *   h1 = relu(W1 xh + b1),  h2 = relu(W2 h1 + b2),  out = W3 h2 + b3
 * Loss over a batch of B rows: L = (1 / (2B)) sum_b |out_b - y_b|^2.
 * Packed parameters: W1 [H][d_in], b1 [H], W2 [H][H], b2 [H], W3 [2][H], b3 [2].
 *
 * With emulate = 1 the operands of the two wide layers are rounded to
 * bfloat16 (round to nearest even, through float) exactly where the GPU
 * rounds them: xh, W1, W2, h1 in the forward pass; dh2, h1, W2, dh1, xh in
 * the backward pass; xh, dh2 and dh1 are first rounded to float, as the GPU
 * holds them in FP32. Sums stay in double, so a GPU comparison isolates its
 * FP32 accumulation. With emulate = 0 everything is plain double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

static double bf16r(double v) {
  float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan unchanged */
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

static double rd(double v, int emulate) { return emulate ? bf16r(v) : v; }

/* Elementwise bfloat16 rounding (through float), exposed for its pin test. */
ORC_API void orc_bf16_round(const double *in, int64_t count, double *out) {
  for (int64_t i = 0; i < count; ++i) out[i] = bf16r(in[i]);
}

/* With emulation, values the GPU holds in FP32 before rounding them to
 * bfloat16 are first rounded to float. */
static double rf(double v, int emulate) { return emulate ? (double)(float)v : v; }

ORC_API int64_t orc_mlp_param_count(int d_in, int H) {
  return (int64_t)H * d_in + H + (int64_t)H * H + H + 2 * H + 2;
}

typedef struct {
  const double *w1, *b1, *w2, *b2, *w3, *b3;
} net_t;

static net_t unpack(const double *p, int d_in, int H) {
  net_t n;
  n.w1 = p;
  n.b1 = n.w1 + (int64_t)H * d_in;
  n.w2 = n.b1 + H;
  n.b2 = n.w2 + (int64_t)H * H;
  n.w3 = n.b2 + H;
  n.b3 = n.w3 + 2 * H;
  return n;
}

/* Forward pass of one row; fills xh (d_in), h1 (H), h2 (H), out (2). */
static void fwd_row(const net_t *n, int d_in, int H, const double *x, const double *mean,
                    const double *invstd, int emulate, double *xh, double *h1, double *h2,
                    double *out) {
  for (int k = 0; k < d_in; ++k) xh[k] = rf((x[k] - mean[k]) * invstd[k], emulate);
  for (int j = 0; j < H; ++j) {
    double s = 0.0;
    for (int k = 0; k < d_in; ++k) s += rd(n->w1[(int64_t)j * d_in + k], emulate) * rd(xh[k], emulate);
    s += n->b1[j];
    h1[j] = s > 0.0 ? s : 0.0;
  }
  for (int j = 0; j < H; ++j) {
    double s = 0.0;
    for (int k = 0; k < H; ++k) s += rd(n->w2[(int64_t)j * H + k], emulate) * rd(h1[k], emulate);
    s += n->b2[j];
    h2[j] = s > 0.0 ? s : 0.0;
  }
  for (int c = 0; c < 2; ++c) {
    double s = 0.0;
    for (int k = 0; k < H; ++k) s += n->w3[c * H + k] * h2[k];
    out[c] = s + n->b3[c];
  }
}

ORC_API void orc_mlp_forward(const double *params, int d_in, int H, const double *mean,
                             const double *invstd, const double *x, int64_t B, int emulate,
                             double *out) {
  net_t n = unpack(params, d_in, H);
#pragma omp parallel
  {
    double *xh = (double *)malloc(sizeof(double) * d_in);
    double *h1 = (double *)malloc(sizeof(double) * H);
    double *h2 = (double *)malloc(sizeof(double) * H);
#pragma omp for schedule(static)
    for (int64_t b = 0; b < B; ++b)
      fwd_row(&n, d_in, H, x + b * d_in, mean, invstd, emulate, xh, h1, h2, out + 2 * b);
    free(xh);
    free(h1);
    free(h2);
  }
}

/*
 * Gradient of L with respect to all packed parameters (grad has the packed
 * layout) and the loss value. Plain backpropagation through the network
 * above, one row at a time, accumulated over the batch in row order.
 */
ORC_API double orc_mlp_gradient(const double *params, int d_in, int H, const double *mean,
                                const double *invstd, const double *x, const double *y,
                                int64_t B, int emulate, double *grad) {
  net_t n = unpack(params, d_in, H);
  const int64_t np = orc_mlp_param_count(d_in, H);
  memset(grad, 0, sizeof(double) * np);
  double *g_w1 = grad, *g_b1 = g_w1 + (int64_t)H * d_in, *g_w2 = g_b1 + H,
         *g_b2 = g_w2 + (int64_t)H * H, *g_w3 = g_b2 + H, *g_b3 = g_w3 + 2 * H;
  double *xh = (double *)malloc(sizeof(double) * d_in);
  double *h1 = (double *)malloc(sizeof(double) * H);
  double *h2 = (double *)malloc(sizeof(double) * H);
  double *dh2 = (double *)malloc(sizeof(double) * H);
  double *dh1 = (double *)malloc(sizeof(double) * H);
  double loss = 0.0;
  for (int64_t b = 0; b < B; ++b) {
    double out[2];
    fwd_row(&n, d_in, H, x + b * d_in, mean, invstd, emulate, xh, h1, h2, out);
    double dout[2];
    for (int c = 0; c < 2; ++c) {
      double e = out[c] - y[2 * b + c];
      loss += 0.5 * e * e;
      dout[c] = e / (double)B;
    }
    /* output layer (plain precision on the GPU too) */
    for (int c = 0; c < 2; ++c) {
      g_b3[c] += dout[c];
      for (int k = 0; k < H; ++k) g_w3[c * H + k] += dout[c] * h2[k];
    }
    for (int k = 0; k < H; ++k) {
      double s = dout[0] * n.w3[k] + dout[1] * n.w3[H + k];
      dh2[k] = h2[k] > 0.0 ? rf(s, emulate) : 0.0;
    }
    /* second layer */
    for (int j = 0; j < H; ++j) {
      g_b2[j] += dh2[j];
      for (int k = 0; k < H; ++k) g_w2[(int64_t)j * H + k] += rd(dh2[j], emulate) * rd(h1[k], emulate);
    }
    for (int k = 0; k < H; ++k) {
      double s = 0.0;
      for (int j = 0; j < H; ++j) s += rd(dh2[j], emulate) * rd(n.w2[(int64_t)j * H + k], emulate);
      dh1[k] = h1[k] > 0.0 ? rf(s, emulate) : 0.0;
    }
    /* first layer */
    for (int j = 0; j < H; ++j) {
      g_b1[j] += dh1[j];
      for (int k = 0; k < d_in; ++k)
        g_w1[(int64_t)j * d_in + k] += rd(dh1[j], emulate) * rd(xh[k], emulate);
    }
  }
  free(xh);
  free(h1);
  free(h2);
  free(dh2);
  free(dh1);
  return loss / (double)B;
}

/* Adam step t (1-based) on packed parameters, in place on p, m, v. */
ORC_API void orc_adam(double *p, const double *g, double *m, double *v, int64_t count, double lr,
                      double beta1, double beta2, double eps, int t) {
  const double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
  for (int64_t i = 0; i < count; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
    const double mh = m[i] / c1, vh = v[i] / c2;
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}
