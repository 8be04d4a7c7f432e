/*
 * FP64 CPU oracle for the exact t-SNE hot path (bigMap / ptSNE, arXiv 1812.09869).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct
 * reference that the GPU path is checked against. Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it. It shares no
 * code, header, table or constant with the HIP library and includes nothing
 * from it.
 *
 * Everything is double precision, written as plain loops in the order the
 * paper states the method:
 *   - squared Euclidean input similarities        (section "Similarities in the
 *     input (high dimensional) space", first paragraph)
 *   - conditional Gaussian affinities p_{j|i}      (Eq. 1, conditional probability)
 *   - precision beta_i and perplexity 2^H          (Eq. 2 and the text around it;
 *     the search procedure itself is in a supplement the paper does not
 *     include, so it is a bisection on beta: reading documented with the tests)
 *   - symmetric joint P                             (Eq. 3)
 *   - Student-t joint Q and its normaliser Z        (Eq. 4)
 *   - KL cost                                       (Eq. 5)
 *   - exact gradient                                (Eq. 6)
 *   - pseudo-normalised cost H(P,Q)/H(P,U)          (Eq. 9, section
 *     "Pseudo-normalized cost function")
 *   - mapping update with momentum, learning rate,
 *     adaptive gains and early exaggeration         (Eq. 10 and the paragraph
 *     after it, section "Internal parametric configuration")
 *   - the paper's own learning rate from the extent
 *     of the map, and the embedding size            (Eq. 11; section
 *     "Comparison of t-SNE and ptSNE" for the size as the diagonal)
 *
 * Readings of points where the paper is silent or garbled:
 *   - entropy in nats; the target is ln(perplexity), identical to Eq. 2's
 *     base-2 form because 2^{H_bits} = e^{H_nats};
 *   - self terms p_{i|i}, p_ii, q_ii are zero and Z excludes i = j (the k != i
 *     and k != l restrictions of Eqs. 1 and 4);
 *   - early exaggeration multiplies p_ij in the gradient only;
 *   - the update descends: U <- mu U - eta G.g, Y <- Y + U (Eq. 10 prints a
 *     plus sign in front of the gradient term);
 *   - gains: +0.2 where sign(g) differs from sign(U), x0.8 otherwise, floor
 *     min_gain; (g > 0) is compared with (U > 0);
 *   - the map is re-centred to zero mean after every update (optional);
 *   - Eq. 11's Y_max - Y_min is the larger of the two coordinate ranges of
 *     the map the gradient is taken at, ln is the natural logarithm, and the
 *     rule replaces the gains (eta is the only internal parameter).
 *
 * Parallel loops run over rows with OpenMP; every reduction is written into a
 * per-row array first and summed afterwards in row order, so results do not
 * depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------- */
/* Input similarities: squared Euclidean distance in direct-difference form. */
/* ------------------------------------------------------------------------- */

static double sqdist(const double *a, const double *b, int32_t d) {
  double s = 0.0;
  for (int32_t k = 0; k < d; ++k) {
    double t = a[k] - b[k];
    s += t * t;
  }
  return s;
}

/* D[i*n + j] = ||x_i - x_j||^2, D[i*n + i] = 0. */
ORC_API void orc_sqdist(const double *X, int64_t n, int32_t d, double *D) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j)
      D[i * n + j] = (i == j) ? 0.0 : sqdist(X + i * d, X + j * d, d);
}

/* ------------------------------------------------------------------------- */
/* Calibration of one row (Eqs. 1-2).                                         */
/* ------------------------------------------------------------------------- */

/*
 * Normaliser S and entropy H (nats) of p_{.|i} at precision beta. Distances
 * are shifted by the row minimum m: exp(-beta d) / sum exp(-beta d) is
 * unchanged by the shift, and the shifted exponentials stay in (0, 1].
 *   S = sum_{j != i} exp(-beta (d_ij - m))
 *   H = -sum p ln p = ln S + beta * sum_j (d_ij - m) exp(-beta (d_ij - m)) / S
 */
static void row_entropy(const double *drow, int64_t n, int64_t i, double m, double beta,
                        double *S_out, double *H_out) {
  double S = 0.0, T = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    double e = exp(-beta * (drow[j] - m));
    S += e;
    T += (drow[j] - m) * e;
  }
  *S_out = S;
  *H_out = log(S) + beta * T / S;
}

static double ulp_of(double x) { return nextafter(x, INFINITY) - x; }

/*
 * Bisection on beta for H_i(beta) = ln(perplexity). H is non-increasing in
 * beta (dH/dbeta = -beta Var_p(d) <= 0), maximal (ln(n-1)) at beta = 0.
 * Start at beta = 1 with the bracket [0, +inf): while no upper end is known,
 * a too-high entropy doubles beta; afterwards each pass halves the bracket.
 * Stops at |H - ln u| <= tol, at a bracket no wider than 4 ulp, or after
 * max_iter evaluations. The returned beta is the last one evaluated, with
 * its own S and H. Returns the number of evaluations, negated if the row did
 * not converge.
 */
static int calibrate_row(const double *drow, int64_t n, int64_t i, double logu, int max_iter,
                         double tol, double *beta_o, double *m_o, double *S_o, double *H_o) {
  double m = INFINITY;
  for (int64_t j = 0; j < n; ++j)
    if (j != i && drow[j] < m) m = drow[j];
  double beta = 1.0, lo = 0.0, hi = INFINITY, S = 0.0, H = 0.0;
  int it = 0, ok = 0;
  for (;;) {
    ++it;
    row_entropy(drow, n, i, m, beta, &S, &H);
    if (fabs(H - logu) <= tol) { ok = 1; break; }
    if (isfinite(hi) && hi - lo <= 4.0 * ulp_of(hi)) { ok = 1; break; }
    if (it >= max_iter) break;
    if (H > logu) {
      lo = beta;
      beta = isinf(hi) ? 2.0 * beta : 0.5 * (beta + hi);
    } else {
      hi = beta;
      beta = 0.5 * (lo + beta);
    }
  }
  *beta_o = beta;
  *m_o = m;
  *S_o = S;
  *H_o = H;
  return ok ? it : -it;
}

/*
 * Calibrate the rows listed in rows[0..nrows) (all rows if rows == NULL, then
 * nrows must equal n). Distances of each row are recomputed from X; nothing
 * of size n^2 is stored. Outputs are indexed by position in the list.
 */
ORC_API void orc_calibrate(const double *X, int64_t n, int32_t d, double perplexity,
                           const int64_t *rows, int64_t nrows, int max_iter, double tol,
                           double *beta, double *m, double *S, double *H, int32_t *iters) {
  const double logu = log(perplexity);
#pragma omp parallel
  {
    double *drow = (double *)malloc((size_t)n * sizeof(double));
#pragma omp for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; ++r) {
      int64_t i = rows ? rows[r] : r;
      for (int64_t j = 0; j < n; ++j)
        drow[j] = (j == i) ? 0.0 : sqdist(X + i * d, X + j * d, d);
      iters[r] = calibrate_row(drow, n, i, logu, max_iter, tol, beta + r, m + r, S + r, H + r);
    }
    free(drow);
  }
}

/* ------------------------------------------------------------------------- */
/* Joint input affinities (Eq. 3).                                            */
/* ------------------------------------------------------------------------- */

/* p_{j|i} from the calibrated statistics of row i (Eq. 1). */
static double cond_p(double dij, double beta_i, double m_i, double S_i) {
  return exp(-beta_i * (dij - m_i)) / S_i;
}

/* Full square P: P[i*n+j] = (p_{j|i} + p_{i|j}) / (2n), P[i*n+i] = 0. */
ORC_API void orc_joint_p(const double *X, int64_t n, int32_t d, const double *beta,
                         const double *m, const double *S, double *P) {
  const double inv2n = 1.0 / (2.0 * (double)n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < n; ++j) {
      if (i == j) { P[i * n + j] = 0.0; continue; }
      double dij = sqdist(X + i * d, X + j * d, d);
      P[i * n + j] = (cond_p(dij, beta[i], m[i], S[i]) + cond_p(dij, beta[j], m[j], S[j])) * inv2n;
    }
  }
}

/*
 * Affinities from given dissimilarities (section "ptSNE: parallelized t-SNE":
 * any measure of similarity may enter; the dwt1005 set gives shortest-path
 * distances). The dissimilarity delta_ij takes the place of ||x_i - x_j||, so
 * Eq. 1 uses delta_ij^2. Dl is the n x n matrix (row-major, symmetric; the
 * diagonal is ignored). Row i is calibrated from its own row of delta^2.
 */
ORC_API void orc_calibrate_dissim(const double *Dl, int64_t n, double perplexity, int max_iter,
                                  double tol, double *beta, double *m, double *S, double *H,
                                  int32_t *iters) {
  const double logu = log(perplexity);
#pragma omp parallel
  {
    double *drow = (double *)malloc((size_t)n * sizeof(double));
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t j = 0; j < n; ++j) drow[j] = (j == i) ? 0.0 : Dl[i * n + j] * Dl[i * n + j];
      iters[i] = calibrate_row(drow, n, i, logu, max_iter, tol, beta + i, m + i, S + i, H + i);
    }
    free(drow);
  }
}

/* Full square P of Eq. 3 from given dissimilarities: p_{j|i} from row i's
 * delta_ij^2 and p_{i|j} from row j's delta_ji^2. */
ORC_API void orc_joint_p_dissim(const double *Dl, int64_t n, const double *beta, const double *m,
                                const double *S, double *P) {
  const double inv2n = 1.0 / (2.0 * (double)n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < n; ++j) {
      if (i == j) { P[i * n + j] = 0.0; continue; }
      const double dij = Dl[i * n + j] * Dl[i * n + j], dji = Dl[j * n + i] * Dl[j * n + i];
      P[i * n + j] = (cond_p(dij, beta[i], m[i], S[i]) + cond_p(dji, beta[j], m[j], S[j])) * inv2n;
    }
  }
}

/* Single entries P_{i_k j_k} from the statistics of rows i_k and j_k. */
ORC_API void orc_p_entries(const double *X, int64_t n, int32_t d, const int64_t *ii,
                           const int64_t *jj, int64_t cnt, const double *beta_i,
                           const double *m_i, const double *S_i, const double *beta_j,
                           const double *m_j, const double *S_j, double *out) {
  const double inv2n = 1.0 / (2.0 * (double)n);
  for (int64_t k = 0; k < cnt; ++k) {
    if (ii[k] == jj[k]) { out[k] = 0.0; continue; }
    double dij = sqdist(X + ii[k] * d, X + jj[k] * d, d);
    out[k] = (cond_p(dij, beta_i[k], m_i[k], S_i[k]) + cond_p(dij, beta_j[k], m_j[k], S_j[k])) *
             inv2n;
  }
}

/*
 * Whole rows of P (Eq. 3) for the listed rows, from the statistics of every
 * row (beta, m, S indexed by point): out[r*n + j] = p_{rows[r], j}. Needs
 * O(nrows * n) memory, so rows of P can be formed at sizes where the full
 * square cannot be stored.
 */
ORC_API void orc_p_rows(const double *X, int64_t n, int32_t d, const int64_t *rows,
                        int64_t nrows, const double *beta, const double *m, const double *S,
                        double *out) {
  const double inv2n = 1.0 / (2.0 * (double)n);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = rows[r];
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) { out[r * n + j] = 0.0; continue; }
      double dij = sqdist(X + i * d, X + j * d, d);
      out[r * n + j] =
          (cond_p(dij, beta[i], m[i], S[i]) + cond_p(dij, beta[j], m[j], S[j])) * inv2n;
    }
  }
}

/* sum_{i != j, p > 0} p_ij ln p_ij: the constant part of the KL cost. */
ORC_API double orc_p_entropy_term(const double *P, int64_t n) {
  double *row = (double *)malloc((size_t)n * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j)
      if (j != i && P[i * n + j] > 0.0) s += P[i * n + j] * log(P[i * n + j]);
    row[i] = s;
  }
  double t = 0.0;
  for (int64_t i = 0; i < n; ++i) t += row[i];
  free(row);
  return t;
}

/* ------------------------------------------------------------------------- */
/* Output similarities, cost and gradient (Eqs. 4-6, 9).                      */
/* ------------------------------------------------------------------------- */

/* Unnormalised Student-t kernel w_ij = (1 + ||y_i - y_j||^2)^{-1}, 2-D map. */
static double wker(const double *Y, int64_t i, int64_t j) {
  double dx = Y[2 * i] - Y[2 * j], dy = Y[2 * i + 1] - Y[2 * j + 1];
  return 1.0 / (1.0 + dx * dx + dy * dy);
}

/* Z = sum_{k != l} w_kl over ordered pairs (denominator of Eq. 4). */
ORC_API double orc_z(const double *Y, int64_t n) {
  double *row = (double *)malloc((size_t)n * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j)
      if (j != i) s += wker(Y, i, j);
    row[i] = s;
  }
  double z = 0.0;
  for (int64_t i = 0; i < n; ++i) z += row[i];
  free(row);
  return z;
}

/*
 * Gradient of Eq. 6 with q_ij = w_ij / Z and early exaggeration alpha applied
 * to p_ij:  g_i = 4 sum_{j != i} (alpha p_ij - w_ij / Z) w_ij (y_i - y_j).
 * P is the full square (row-major n x n). Writes g (n x 2) and Z.
 */
ORC_API void orc_gradient(const double *P, int64_t n, const double *Y, double alpha, double *g,
                          double *Z_out) {
  const double Z = orc_z(Y, n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double gx = 0.0, gy = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double w = wker(Y, i, j);
      double c = (alpha * P[i * n + j] - w / Z) * w;
      gx += c * (Y[2 * i] - Y[2 * j]);
      gy += c * (Y[2 * i + 1] - Y[2 * j + 1]);
    }
    g[2 * i] = 4.0 * gx;
    g[2 * i + 1] = 4.0 * gy;
  }
  if (Z_out) *Z_out = Z;
}

/*
 * The repulsive part of Eq. 6 alone (alpha = 0) for the listed rows:
 *   r_i = -4 sum_{j != i} w_ij^2 (y_i - y_j) / Z.
 * Needs only the map, so it can be evaluated row by row at any n.
 */
ORC_API void orc_repulsion_rows(const double *Y, int64_t n, const int64_t *rows, int64_t nrows,
                                double Z, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t i = rows[r];
    double gx = 0.0, gy = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double w = wker(Y, i, j);
      gx += w * w * (Y[2 * i] - Y[2 * j]);
      gy += w * w * (Y[2 * i + 1] - Y[2 * j + 1]);
    }
    out[2 * r] = -4.0 * gx / Z;
    out[2 * r + 1] = -4.0 * gy / Z;
  }
}

/*
 * Eq. 6 for the listed rows only, from their rows of P (Prows[r*n + j] =
 * p_{rows[r], j}) and a given Z (the sum over all ordered pairs, Eq. 4):
 *   g_i = 4 sum_{j != i} (alpha p_ij - w_ij / Z) w_ij (y_i - y_j).
 * The same loop as the whole-map gradient, so rows of P that cannot all be
 * stored still give exact gradient rows.
 */
ORC_API void orc_gradient_rows(const double *Prows, int64_t n, const double *Y,
                               const int64_t *rows, int64_t nrows, double alpha, double Z,
                               double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = rows[r];
    double gx = 0.0, gy = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double w = wker(Y, i, j);
      double c = (alpha * Prows[r * n + j] - w / Z) * w;
      gx += c * (Y[2 * i] - Y[2 * j]);
      gy += c * (Y[2 * i + 1] - Y[2 * j + 1]);
    }
    out[2 * r] = 4.0 * gx;
    out[2 * r + 1] = 4.0 * gy;
  }
}

/*
 * The listed rows' share of the KL of Eq. 5, from their rows of P and a
 * given Z:  kl_i = sum_{j != i, p_ij > 0} p_ij (ln p_ij - ln w_ij + ln Z).
 * Summed over every row this is the KL itself.
 */
ORC_API void orc_kl_rows(const double *Prows, int64_t n, const double *Y, const int64_t *rows,
                         int64_t nrows, double Z, double *out) {
  const double lz = log(Z);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = rows[r];
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      const double p = Prows[r * n + j];
      if (j == i || !(p > 0.0)) continue;
      s += p * (log(p) - log(wker(Y, i, j)) + lz);
    }
    out[r] = s;
  }
}

/*
 * KL(P||Q) of Eq. 5 and the pseudo-normalised cost of Eq. 9, using
 * ln q_ij = ln w_ij - ln Z:
 *   KL     = sum p ln p - sum p ln w + (sum p) ln Z
 *   C_norm = (-sum p ln w + (sum p) ln Z) / (ln n + ln(n-1))
 * The true P is used (no exaggeration).
 */
ORC_API void orc_cost(const double *P, int64_t n, const double *Y, double *kl, double *cnorm) {
  const double Z = orc_z(Y, n);
  double *plp = (double *)malloc((size_t)n * sizeof(double));
  double *plw = (double *)malloc((size_t)n * sizeof(double));
  double *ps = (double *)malloc((size_t)n * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double p = P[i * n + j];
      if (p > 0.0) a += p * log(p);
      b += p * log(wker(Y, i, j));
      c += p;
    }
    plp[i] = a;
    plw[i] = b;
    ps[i] = c;
  }
  double A = 0.0, B = 0.0, C = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    A += plp[i];
    B += plw[i];
    C += ps[i];
  }
  free(plp);
  free(plw);
  free(ps);
  double cross = -B + C * log(Z); /* H(P, Q) */
  if (kl) *kl = A + cross;
  if (cnorm) *cnorm = cross / (log((double)n) + log((double)n - 1.0));
}

/* ------------------------------------------------------------------------- */
/* Mapping update (Eq. 10 and the following paragraph).                       */
/* ------------------------------------------------------------------------- */

/*
 * One iteration from state (Y, U, G), all n x 2:
 *   g = gradient(P, Y, alpha)
 *   G <- (g > 0) != (U > 0) ? G + 0.2 : 0.8 G;  G <- max(G, min_gain)
 *   U <- mu U - eta G g
 *   Y <- Y + U;  Y <- Y - mean(Y) if recentre
 * Optionally returns g and Z.
 */
ORC_API void orc_step(const double *P, int64_t n, double *Y, double *U, double *G, double alpha,
                      double mu, double eta, double min_gain, int recentre, double *g_out,
                      double *Z_out) {
  double *g = (double *)malloc((size_t)n * 2 * sizeof(double));
  double Z = 0.0;
  orc_gradient(P, n, Y, alpha, g, &Z);
  for (int64_t k = 0; k < 2 * n; ++k) {
    double gain = ((g[k] > 0.0) != (U[k] > 0.0)) ? G[k] + 0.2 : G[k] * 0.8;
    G[k] = gain < min_gain ? min_gain : gain;
    U[k] = mu * U[k] - eta * G[k] * g[k];
    Y[k] += U[k];
  }
  if (recentre) {
    double mx = 0.0, my = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      mx += Y[2 * i];
      my += Y[2 * i + 1];
    }
    mx /= (double)n;
    my /= (double)n;
    for (int64_t i = 0; i < n; ++i) {
      Y[2 * i] -= mx;
      Y[2 * i + 1] -= my;
    }
  }
  if (g_out) memcpy(g_out, g, (size_t)n * 2 * sizeof(double));
  if (Z_out) *Z_out = Z;
  free(g);
}

/* Extent of a 2-D map: range of each coordinate, max_i y_ic - min_i y_ic. */
static void map_ranges(const double *Y, int64_t n, double *rx, double *ry) {
  double lox = Y[0], hix = Y[0], loy = Y[1], hiy = Y[1];
  for (int64_t i = 1; i < n; ++i) {
    if (Y[2 * i] < lox) lox = Y[2 * i];
    if (Y[2 * i] > hix) hix = Y[2 * i];
    if (Y[2 * i + 1] < loy) loy = Y[2 * i + 1];
    if (Y[2 * i + 1] > hiy) hiy = Y[2 * i + 1];
  }
  *rx = hix - lox;
  *ry = hiy - loy;
}

/* Learning rate of Eq. 11: eta = ln(n - 1) * (Y_max - Y_min) / 2, with
 * Y_max - Y_min the larger coordinate range of the map. */
ORC_API double orc_adaptive_eta(const double *Y, int64_t n) {
  double rx, ry;
  map_ranges(Y, n, &rx, &ry);
  return log((double)n - 1.0) * (rx > ry ? rx : ry) / 2.0;
}

/* Embedding size: length of the diagonal of the box spanned by the map. */
ORC_API double orc_embedding_size(const double *Y, int64_t n) {
  double rx, ry;
  map_ranges(Y, n, &rx, &ry);
  return sqrt(rx * rx + ry * ry);
}

/*
 * One iteration with the paper's own optimiser (Eqs. 10 and 11, descent
 * reading, no gains):
 *   g = gradient(P, Y, alpha);  eta = orc_adaptive_eta(Y) at the same Y
 *   U <- mu U - eta g;  Y <- Y + U;  Y <- Y - mean(Y) if recentre
 * Optionally returns g, Z and eta.
 */
ORC_API void orc_step_range(const double *P, int64_t n, double *Y, double *U, double alpha,
                            double mu, int recentre, double *g_out, double *Z_out,
                            double *eta_out) {
  double *g = (double *)malloc((size_t)n * 2 * sizeof(double));
  double Z = 0.0;
  orc_gradient(P, n, Y, alpha, g, &Z);
  const double eta = orc_adaptive_eta(Y, n);
  for (int64_t k = 0; k < 2 * n; ++k) {
    U[k] = mu * U[k] - eta * g[k];
    Y[k] += U[k];
  }
  if (recentre) {
    double mx = 0.0, my = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      mx += Y[2 * i];
      my += Y[2 * i + 1];
    }
    mx /= (double)n;
    my /= (double)n;
    for (int64_t i = 0; i < n; ++i) {
      Y[2 * i] -= mx;
      Y[2 * i + 1] -= my;
    }
  }
  if (g_out) memcpy(g_out, g, (size_t)n * 2 * sizeof(double));
  if (Z_out) *Z_out = Z;
  if (eta_out) *eta_out = eta;
  free(g);
}

/* ------------------------------------------------------------------------- */
/* Neighbourhood preservation (evaluation of an embedding).                   */
/* ------------------------------------------------------------------------- */

/* Indices of the k nearest neighbours of row q among all n rows (self
 * excluded), by squared distance, ties broken by the lower index. */
static void knn_row(const double *A, int64_t n, int32_t d, int64_t q, int k, int64_t *nb,
                    double *nd) {
  int cnt = 0;
  for (int64_t j = 0; j < n; ++j) {
    if (j == q) continue;
    double dist = sqdist(A + q * d, A + j * d, d);
    if (cnt == k && !(dist < nd[k - 1])) continue;
    int pos = cnt < k ? cnt++ : k - 1;
    while (pos > 0 && dist < nd[pos - 1]) {
      nd[pos] = nd[pos - 1];
      nb[pos] = nb[pos - 1];
      --pos;
    }
    nd[pos] = dist;
    nb[pos] = j;
  }
}

/*
 * Mean over the query rows of |kNN_k^X(q) intersect kNN_k^Y(q)| / k.
 * X is n x d, Y is n x 2; queries = rows[0..nrows).
 */
ORC_API double orc_knn_overlap(const double *X, int64_t n, int32_t d, const double *Y,
                               const int64_t *rows, int64_t nrows, int k) {
  double *frac = (double *)malloc((size_t)nrows * sizeof(double));
#pragma omp parallel
  {
    int64_t *a = (int64_t *)malloc((size_t)k * sizeof(int64_t));
    int64_t *b = (int64_t *)malloc((size_t)k * sizeof(int64_t));
    double *da = (double *)malloc((size_t)k * sizeof(double));
    double *db = (double *)malloc((size_t)k * sizeof(double));
#pragma omp for schedule(dynamic, 8)
    for (int64_t r = 0; r < nrows; ++r) {
      knn_row(X, n, d, rows[r], k, a, da);
      knn_row(Y, n, 2, rows[r], k, b, db);
      int common = 0;
      for (int u = 0; u < k; ++u)
        for (int v = 0; v < k; ++v)
          if (a[u] == b[v]) { ++common; break; }
      frac[r] = (double)common / (double)k;
    }
    free(a);
    free(b);
    free(da);
    free(db);
  }
  double s = 0.0;
  for (int64_t r = 0; r < nrows; ++r) s += frac[r];
  free(frac);
  return nrows ? s / (double)nrows : 0.0;
}
