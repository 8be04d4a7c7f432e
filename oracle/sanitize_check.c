/*
 * TEST INFRASTRUCTURE ONLY: a driver that runs every exported function of the
 * FP64 oracle once on tiny inputs, for a build with the address and
 * undefined-behaviour sanitizers (tests/test_oracle_sanitized.py builds it
 * with gcc and checks that it runs clean). It prints one line per function.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_sqdist(const double *X, int64_t n, int32_t d, double *D);
void orc_calibrate(const double *X, int64_t n, int32_t d, double perplexity, const int64_t *rows,
                   int64_t nrows, int max_iter, double tol, double *beta, double *m, double *S,
                   double *H, int32_t *iters);
void orc_joint_p(const double *X, int64_t n, int32_t d, const double *beta, const double *m,
                 const double *S, double *P);
void orc_calibrate_dissim(const double *Dl, int64_t n, double perplexity, int max_iter,
                          double tol, double *beta, double *m, double *S, double *H,
                          int32_t *iters);
void orc_joint_p_dissim(const double *Dl, int64_t n, const double *beta, const double *m,
                        const double *S, double *P);
void orc_p_entries(const double *X, int64_t n, int32_t d, const int64_t *ii, const int64_t *jj,
                   int64_t cnt, const double *beta_i, const double *m_i, const double *S_i,
                   const double *beta_j, const double *m_j, const double *S_j, double *out);
void orc_p_rows(const double *X, int64_t n, int32_t d, const int64_t *rows, int64_t nrows,
                const double *beta, const double *m, const double *S, double *out);
double orc_p_entropy_term(const double *P, int64_t n);
double orc_z(const double *Y, int64_t n);
void orc_gradient(const double *P, int64_t n, const double *Y, double alpha, double *g,
                  double *Z_out);
void orc_repulsion_rows(const double *Y, int64_t n, const int64_t *rows, int64_t nrows, double Z,
                        double *out);
void orc_gradient_rows(const double *Prows, int64_t n, const double *Y, const int64_t *rows,
                       int64_t nrows, double alpha, double Z, double *out);
void orc_kl_rows(const double *Prows, int64_t n, const double *Y, const int64_t *rows,
                 int64_t nrows, double Z, double *out);
void orc_cost(const double *P, int64_t n, const double *Y, double *kl, double *cnorm);
void orc_step(const double *P, int64_t n, double *Y, double *U, double *G, double alpha,
              double mu, double eta, double min_gain, int recentre, double *g_out, double *Z_out);
double orc_adaptive_eta(const double *Y, int64_t n);
double orc_embedding_size(const double *Y, int64_t n);
void orc_step_range(const double *P, int64_t n, double *Y, double *U, double alpha, double mu,
                    int recentre, double *g_out, double *Z_out, double *eta_out);
double orc_knn_overlap(const double *X, int64_t n, int32_t d, const double *Y,
                       const int64_t *rows, int64_t nrows, int k);
int64_t orc_mlp_param_count(int d_in, int H);
void orc_bf16_round(const double *in, int64_t count, double *out);
void orc_mlp_forward(const double *params, int d_in, int H, const double *mean,
                     const double *invstd, const double *x, int64_t B, int emulate, double *out);
double orc_mlp_gradient(const double *params, int d_in, int H, const double *mean,
                        const double *invstd, const double *x, const double *y, int64_t B,
                        int emulate, double *grad);
void orc_adam(double *p, const double *g, double *m, double *v, int64_t count, double lr,
              double beta1, double beta2, double eps, int t);

/* deterministic pseudo-random values in [-1, 1) */
static double rnd(uint64_t *s) {
  *s = *s * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(*s >> 11) / 4503599627370496.0 - 1.0;
}

int main(void) {
  enum { N = 37, D = 5 };
  uint64_t s = 7;
  double X[N * D], Y[N * 2], U[N * 2] = {0}, G[N * 2], Dm[N * N], P[N * N], Pd[N * N];
  double beta[N], m[N], S[N], H[N], g[N * 2], out[N * 2], kl, cn, z;
  int32_t it[N];
  for (int i = 0; i < N * D; ++i) X[i] = 3.0 * rnd(&s);
  for (int i = 0; i < N * 2; ++i) { Y[i] = 0.5 * rnd(&s); G[i] = 1.0; }
  orc_sqdist(X, N, D, Dm);
  orc_calibrate(X, N, D, 8.0, NULL, N, 200, 1e-12, beta, m, S, H, it);
  orc_joint_p(X, N, D, beta, m, S, P);
  for (int i = 0; i < N * N; ++i) Dm[i] = sqrt(Dm[i]);
  double bd[N], md[N], Sd[N], Hd[N];
  orc_calibrate_dissim(Dm, N, 8.0, 200, 1e-12, bd, md, Sd, Hd, it);
  orc_joint_p_dissim(Dm, N, bd, md, Sd, Pd);
  int64_t ii[3] = {0, 5, 36}, jj[3] = {1, 5, 2}, rows[3] = {0, 17, 36};
  double pe[3], prow[3 * N], gr[3 * 2], klr[3];
  orc_p_entries(X, N, D, ii, jj, 3, beta, m, S, beta, m, S, pe);
  orc_p_rows(X, N, D, rows, 3, beta, m, S, prow);
  double cp = orc_p_entropy_term(P, N);
  z = orc_z(Y, N);
  orc_gradient(P, N, Y, 12.0, g, &z);
  orc_repulsion_rows(Y, N, rows, 3, z, out);
  orc_gradient_rows(prow, N, Y, rows, 3, 1.0, z, gr);
  orc_kl_rows(prow, N, Y, rows, 3, z, klr);
  orc_cost(P, N, Y, &kl, &cn);
  orc_step(P, N, Y, U, G, 12.0, 0.5, 200.0, 0.01, 1, g, &z);
  double eta = orc_adaptive_eta(Y, N), size = orc_embedding_size(Y, N), e2;
  orc_step_range(P, N, Y, U, 1.0, 0.8, 1, g, &z, &e2);
  double ov = orc_knn_overlap(X, N, D, Y, rows, 3, 4);
  printf("affinities: beta[0] %.6g, sum p ln p %.6g\n", beta[0], cp);
  printf("iteration: KL %.6g, C_norm %.6g, Z %.6g, eta %.6g, size %.6g, knn %.3f\n", kl, cn, z,
         eta, size, ov);
  enum { DI = 3, HH = 4, B = 6 };
  int64_t np = orc_mlp_param_count(DI, HH);
  double *prm = malloc(sizeof(double) * np), *gm = malloc(sizeof(double) * np);
  double *mm = calloc(np, sizeof(double)), *vv = calloc(np, sizeof(double));
  double xs[B * DI], ys[B * 2], mean[DI] = {0}, inv[DI] = {1, 1, 1}, o[B * 2], r[B * 2];
  for (int64_t i = 0; i < np; ++i) prm[i] = 0.4 * rnd(&s);
  for (int i = 0; i < B * DI; ++i) xs[i] = rnd(&s);
  for (int i = 0; i < B * 2; ++i) ys[i] = rnd(&s);
  orc_bf16_round(ys, B * 2, r);
  orc_mlp_forward(prm, DI, HH, mean, inv, xs, B, 1, o);
  double loss = orc_mlp_gradient(prm, DI, HH, mean, inv, xs, ys, B, 1, gm);
  orc_adam(prm, gm, mm, vv, np, 1e-3, 0.9, 0.999, 1e-8, 1);
  printf("network: loss %.6g, out[0] %.6g\n", loss, o[0]);
  free(prm);
  free(gm);
  free(mm);
  free(vv);
  return 0;
}
