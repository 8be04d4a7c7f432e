// C ABI of libtsne355: argument validation, workspace layout and launch
// sequencing. Device work lives in tsne_affinity.hip and tsne_iterate.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/tsne355.h"
#include "tsne_internal.h"
#include "tsne_mlp.h"

namespace tsne {

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

Layout make_layout(int64_t n, int32_t d, int32_t mode, bool stats_only, bool implicit) {
  Layout L;
  L.n = n;
  L.d = d;
  L.mode = mode;
  L.nb = (int32_t)((n + T - 1) / T);
  L.npad = (int64_t)L.nb * T;
  L.nt = (int64_t)L.nb * (L.nb + 1) / 2;
  L.dpad = (d + 3) / 4 * 4;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  // stats_only: the row statistics and the distance stage only (no P, no
  // iteration state, no ordering tree)
  const size_t sz = stats_only ? 0 : 1;
  const size_t np = (size_t)L.npad;
  L.hdr = take(256);
  L.beta = take(np * 8);
  L.S = take(np * 8);
  L.H = take(np * 8);
  L.m = take(np * 4);
  L.a = take(np * 4);
  L.r = take(np * 4);
  L.evals = take(np * 4);
  L.part = take(sz * (size_t)L.nb * L.nb * T * 16);
  L.zpart = take(sz * (size_t)L.nt * 8);
  L.cpart = take(sz * (size_t)L.nt * 16);
  L.ppart = take(sz * (size_t)L.nt * 16);
  L.meanpart = take(sz * (size_t)L.nb * kMeanPartsPerBlock * 16);
  L.nz = take(sz * (size_t)L.nt);
  L.tmap = take(sz * (size_t)L.nt * 8);
  L.tlist = take(sz * (size_t)L.nt * 4);
  L.tcount = take(8);
  L.slots = take(sz * (size_t)L.nb * L.nb * 4);
  L.nslots = take(sz * (size_t)L.nb * 4);
  L.perm = take(np * 4);
  L.inv = take(np * 4);
  L.yp = take(sz * np * 8);
  L.extent = take(sz * (size_t)L.nb * 16);
  // P last: every array above has the same offset whether P is stored (nt
  // tiles) or recomputed per pass (a buffer of whole block rows), so the entry
  // points of either mode stay inside the other's workspace and find its
  // header, order and statistics
  {
    const int64_t cap = L.nb > kImplicitTiles ? L.nb : kImplicitTiles;
    const int64_t tiles = implicit ? (cap < L.nt ? cap : L.nt) : L.nt;
    L.P = take(sz * (size_t)tiles * T * T * 4);
  }
  L.iter_end = o;
  // affinity-stage scratch (only needed inside tsne_affinities)
  L.xmean = take((size_t)L.dpad * 8);
  L.xcT = take((size_t)L.dpad * np * 8);
  L.norms = take(np * 8);
  L.cal_group = L.nb < kCalGroup ? L.nb : kCalGroup;
  L.dblock = take((size_t)L.cal_group * T * np * 4);
  L.npow2 = 1;
  while (L.npow2 < n) L.npow2 <<= 1;
  L.xcT2 = take(sz * (size_t)L.dpad * np * 8);
  L.norms2 = take(sz * np * 8);
  L.keys = take(sz * (size_t)L.npow2 * 8);
  L.vals = take(sz * (size_t)L.npow2 * 4);
  if (mode == TSNE_DIST_FP32) {
    L.xfT = take((size_t)L.dpad * np * 4);
    L.norms32 = take(np * 4);
  } else if (mode != TSNE_DIST_FP64) {
    // 16-bit operands; the x3 modes keep four slice vectors per point and
    // (hi, lo) FP32 norm pairs
    const int32_t k32 = (d + 31) / 32 * 32;
    const bool split = (mode == TSNE_DIST_BF16X3 || mode == TSNE_DIST_FP16X3);
    L.kk = split ? 4 * k32 : k32;
    L.xa = take(np * (size_t)L.kk * 2);
    L.norms32 = take(np * (split ? 8 : 4));
  }
  L.total = o;
  return L;
}

}  // namespace tsne

using tsne::Layout;

static thread_local char g_err[512];

static int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

static int ok() {
  g_err[0] = '\0';
  return TSNE_OK;
}

static int hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) return fail(TSNE_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return ok();
}

static bool valid_n(int64_t n) { return n >= 2 && n <= (int64_t)1 << 30; }

static bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

extern "C" {

size_t tsne_workspace_bytes(int64_t n, int32_t d, int32_t dist_mode) {
  if (!valid_n(n) || d < 1 || d > 65536 || dist_mode < TSNE_DIST_FP64 ||
      dist_mode > TSNE_DIST_FP16X3)
    return 0;
  return tsne::make_layout(n, d, dist_mode).total;
}

int tsne_affinities(const float *x, int64_t n, int32_t d, double perplexity,
                    const tsne_aff_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  tsne_aff_opts o = {TSNE_DIST_FP64, 200, 1e-6, 1, 0};
  if (opts) o = *opts;
  if (!x || !ws) return fail(TSNE_E_ARG, "tsne_affinities: null pointer");
  if (!valid_n(n)) return fail(TSNE_E_ARG, "tsne_affinities: n = %lld out of range", (long long)n);
  if (d < 1 || d > 65536) return fail(TSNE_E_ARG, "tsne_affinities: d = %d out of range", d);
  if (o.dist_mode < TSNE_DIST_FP64 || o.dist_mode > TSNE_DIST_FP16X3)
    return fail(TSNE_E_ARG, "tsne_affinities: unknown distance mode %d", o.dist_mode);
  if (o.max_bisect < 1 || !(o.tol_h > 0.0) || (o.implicit_p != 0 && o.implicit_p != 1))
    return fail(TSNE_E_ARG, "tsne_affinities: max_bisect >= 1, tol_h > 0, implicit_p 0 or 1 required");
  if (!(perplexity > 1.0) || !(perplexity < (double)(n - 1)))
    return fail(TSNE_E_PERPLEXITY, "tsne_affinities: perplexity %g not in (1, n-1 = %lld)",
                perplexity, (long long)(n - 1));
  if (!aligned(ws, 256)) return fail(TSNE_E_WORKSPACE, "tsne_affinities: ws not 256-byte aligned");
  const Layout L = tsne::make_layout(n, d, o.dist_mode, false, o.implicit_p != 0);
  if (ws_bytes < L.total)
    return fail(TSNE_E_WORKSPACE, "tsne_affinities: workspace %zu bytes, need %zu", ws_bytes,
                L.total);
  return hip_check(tsne::launch_affinities(L, x, nullptr, perplexity, o.max_bisect, o.tol_h,
                                           o.reorder != 0, ws, (hipStream_t)stream, false,
                                           o.implicit_p != 0),
                   "tsne_affinities");
}

int tsne_affinities_dissim(const float *dis, int64_t n, double perplexity,
                           const tsne_aff_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  tsne_aff_opts o = {TSNE_DIST_FP64, 200, 1e-6, 0, 0};
  if (opts) o = *opts;
  if (!dis || !ws) return fail(TSNE_E_ARG, "tsne_affinities_dissim: null pointer");
  if (!valid_n(n))
    return fail(TSNE_E_ARG, "tsne_affinities_dissim: n = %lld out of range", (long long)n);
  if (o.max_bisect < 1 || !(o.tol_h > 0.0) || o.implicit_p != 0)
    return fail(TSNE_E_ARG,
                "tsne_affinities_dissim: max_bisect >= 1, tol_h > 0, implicit_p = 0 required");
  if (!(perplexity > 1.0) || !(perplexity < (double)(n - 1)))
    return fail(TSNE_E_PERPLEXITY, "tsne_affinities_dissim: perplexity %g not in (1, n-1 = %lld)",
                perplexity, (long long)(n - 1));
  if (!aligned(ws, 256))
    return fail(TSNE_E_WORKSPACE, "tsne_affinities_dissim: ws not 256-byte aligned");
  const Layout L = tsne::make_layout(n, 1, TSNE_DIST_FP64);
  if (ws_bytes < L.total)
    return fail(TSNE_E_WORKSPACE, "tsne_affinities_dissim: workspace %zu bytes, need %zu",
                ws_bytes, L.total);
  return hip_check(tsne::launch_affinities(L, nullptr, dis, perplexity, o.max_bisect, o.tol_h, 0,
                                           ws, (hipStream_t)stream),
                   "tsne_affinities_dissim");
}

static int check_params(const char *fn, const tsne_step_params *prm) {
  if (!(prm->learning_rate >= 0.f) || !(prm->min_gain >= 0.f) || !isfinite(prm->momentum) ||
      !isfinite(prm->exaggeration))
    return fail(TSNE_E_ARG, "%s: invalid parameters", fn);
  if (prm->lr_rule != TSNE_LR_GAINS && prm->lr_rule != TSNE_LR_RANGE)
    return fail(TSNE_E_ARG, "%s: unknown lr_rule %d", fn, (int)prm->lr_rule);
  return TSNE_OK;
}

static int check_iter_args(const char *fn, void *ws, int64_t n) {
  if (!ws) return fail(TSNE_E_ARG, "%s: null workspace", fn);
  if (!valid_n(n)) return fail(TSNE_E_ARG, "%s: n = %lld out of range", fn, (long long)n);
  if (!aligned(ws, 256)) return fail(TSNE_E_WORKSPACE, "%s: ws not 256-byte aligned", fn);
  return TSNE_OK;
}

int tsne_step(void *ws, int64_t n, float *y, float *u, float *g, const tsne_step_params *prm,
              float *grad_out, double *z_out, void *stream) {
  if (int rc = check_iter_args("tsne_step", ws, n)) return rc;
  if (!y || !u || !prm || (!g && prm->lr_rule != TSNE_LR_RANGE))
    return fail(TSNE_E_ARG, "tsne_step: null pointer");
  if (int rc = check_params("tsne_step", prm)) return rc;
  const Layout L = tsne::make_layout(n, 1, TSNE_DIST_FP64);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = tsne::launch_force(L, ws, y, st);
  if (e == hipSuccess)
    e = tsne::launch_update(L, ws, y, u, g, prm->exaggeration, prm->momentum, prm->learning_rate,
                            prm->min_gain, prm->recentre, prm->lr_rule, grad_out, z_out, st);
  return hip_check(e, "tsne_step");
}

int tsne_forces(void *ws, int64_t n, const float *y, void *stream) {
  if (int rc = check_iter_args("tsne_forces", ws, n)) return rc;
  if (!y) return fail(TSNE_E_ARG, "tsne_forces: null pointer");
  const Layout L = tsne::make_layout(n, 1, TSNE_DIST_FP64);
  return hip_check(tsne::launch_force(L, ws, y, (hipStream_t)stream), "tsne_forces");
}

int tsne_update(void *ws, int64_t n, float *y, float *u, float *g, const tsne_step_params *prm,
                float *grad_out, double *z_out, void *stream) {
  if (int rc = check_iter_args("tsne_update", ws, n)) return rc;
  if (!y || !u || !prm || (!g && prm->lr_rule != TSNE_LR_RANGE))
    return fail(TSNE_E_ARG, "tsne_update: null pointer");
  if (int rc = check_params("tsne_update", prm)) return rc;
  const Layout L = tsne::make_layout(n, 1, TSNE_DIST_FP64);
  return hip_check(tsne::launch_update(L, ws, y, u, g, prm->exaggeration, prm->momentum,
                                       prm->learning_rate, prm->min_gain, prm->recentre,
                                       prm->lr_rule, grad_out, z_out, (hipStream_t)stream),
                   "tsne_update");
}

int tsne_gradient(void *ws, int64_t n, const float *y, float alpha, float *grad_out,
                  double *z_out, void *stream) {
  if (int rc = check_iter_args("tsne_gradient", ws, n)) return rc;
  if (!y || !grad_out) return fail(TSNE_E_ARG, "tsne_gradient: null pointer");
  if (!isfinite(alpha)) return fail(TSNE_E_ARG, "tsne_gradient: non-finite alpha");
  const Layout L = tsne::make_layout(n, 1, TSNE_DIST_FP64);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = tsne::launch_force(L, ws, y, st);
  if (e == hipSuccess) e = tsne::launch_gradient_only(L, ws, alpha, grad_out, z_out, st);
  return hip_check(e, "tsne_gradient");
}

int tsne_cost(void *ws, int64_t n, const float *y, double *out, void *stream) {
  if (int rc = check_iter_args("tsne_cost", ws, n)) return rc;
  if (!y || !out) return fail(TSNE_E_ARG, "tsne_cost: null pointer");
  const Layout L = tsne::make_layout(n, 1, TSNE_DIST_FP64);
  return hip_check(tsne::launch_cost(L, ws, y, out, (hipStream_t)stream), "tsne_cost");
}

size_t tsne_workspace_bytes_implicit(int64_t n, int32_t d, int32_t dist_mode) {
  if (!valid_n(n) || d < 1 || d > 65536 || dist_mode < TSNE_DIST_FP64 ||
      dist_mode > TSNE_DIST_FP16X3)
    return 0;
  return tsne::make_layout(n, d, dist_mode, false, true).total;
}

// The iteration entry points on a workspace whose P is recomputed per pass
// (the layout of tsne_workspace_bytes_implicit, filled by tsne_affinities
// with implicit_p = 1).
static int check_implicit(const char *fn, void *ws, int64_t n, int32_t d, int32_t mode) {
  if (int rc = check_iter_args(fn, ws, n)) return rc;
  if (d < 1 || d > 65536) return fail(TSNE_E_ARG, "%s: d = %d out of range", fn, d);
  if (mode < TSNE_DIST_FP64 || mode > TSNE_DIST_FP16X3)
    return fail(TSNE_E_ARG, "%s: unknown distance mode %d", fn, mode);
  return TSNE_OK;
}

int tsne_step_implicit(void *ws, int64_t n, int32_t d, int32_t dist_mode, float *y, float *u,
                       float *g, const tsne_step_params *prm, float *grad_out, double *z_out,
                       void *stream) {
  if (int rc = check_implicit("tsne_step_implicit", ws, n, d, dist_mode)) return rc;
  if (!y || !u || !prm || (!g && prm->lr_rule != TSNE_LR_RANGE))
    return fail(TSNE_E_ARG, "tsne_step_implicit: null pointer");
  if (int rc = check_params("tsne_step_implicit", prm)) return rc;
  const Layout L = tsne::make_layout(n, d, dist_mode, false, true);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = tsne::launch_force_implicit(L, ws, y, st);
  if (e == hipSuccess)
    e = tsne::launch_update(L, ws, y, u, g, prm->exaggeration, prm->momentum, prm->learning_rate,
                            prm->min_gain, prm->recentre, prm->lr_rule, grad_out, z_out, st);
  return hip_check(e, "tsne_step_implicit");
}

int tsne_gradient_implicit(void *ws, int64_t n, int32_t d, int32_t dist_mode, const float *y,
                           float alpha, float *grad_out, double *z_out, void *stream) {
  if (int rc = check_implicit("tsne_gradient_implicit", ws, n, d, dist_mode)) return rc;
  if (!y || !grad_out) return fail(TSNE_E_ARG, "tsne_gradient_implicit: null pointer");
  if (!isfinite(alpha)) return fail(TSNE_E_ARG, "tsne_gradient_implicit: non-finite alpha");
  const Layout L = tsne::make_layout(n, d, dist_mode, false, true);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = tsne::launch_force_implicit(L, ws, y, st);
  if (e == hipSuccess) e = tsne::launch_gradient_only(L, ws, alpha, grad_out, z_out, st);
  return hip_check(e, "tsne_gradient_implicit");
}

int tsne_cost_implicit(void *ws, int64_t n, int32_t d, int32_t dist_mode, const float *y,
                       double *out, void *stream) {
  if (int rc = check_implicit("tsne_cost_implicit", ws, n, d, dist_mode)) return rc;
  if (!y || !out) return fail(TSNE_E_ARG, "tsne_cost_implicit: null pointer");
  const Layout L = tsne::make_layout(n, d, dist_mode, false, true);
  return hip_check(tsne::launch_cost_implicit(L, ws, y, out, (hipStream_t)stream),
                   "tsne_cost_implicit");
}

int tsne_sync_status(void *ws, void *stream) {
  if (!ws) return fail(TSNE_E_ARG, "tsne_sync_status: null workspace");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_check(e, "tsne_sync_status: synchronize");
  tsne::Hdr h;
  e = hipMemcpy(&h, ws, sizeof h, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_check(e, "tsne_sync_status: copy");
  if (h.err & tsne::kErrState)
    return fail(TSNE_E_STATE, "workspace holds no affinities for this n");
  if (h.err & tsne::kErrNonFinite) return fail(TSNE_E_NONFINITE, "non-finite value on device");
  if (h.err & tsne::kErrNoConv)
    return fail(TSNE_E_NOCONV, "a row's bisection stopped at max_bisect");
  return ok();
}

const char *tsne_last_error(void) { return g_err; }

int tsne_export_rowstats(void *ws, int64_t n, double *beta, float *m, double *S, double *H,
                         int32_t *evals, void *stream) {
  if (int rc = check_iter_args("tsne_export_rowstats", ws, n)) return rc;
  const Layout L = tsne::make_layout(n, 1, TSNE_DIST_FP64);
  return hip_check(tsne::launch_export_rowstats(L, ws, beta, m, S, H, evals, (hipStream_t)stream),
                   "tsne_export_rowstats");
}

int tsne_export_scalars(void *ws, int64_t n, double *out, void *stream) {
  if (int rc = check_iter_args("tsne_export_scalars", ws, n)) return rc;
  if (!out) return fail(TSNE_E_ARG, "tsne_export_scalars: null pointer");
  const Layout L = tsne::make_layout(n, 1, TSNE_DIST_FP64);
  return hip_check(tsne::launch_export_scalars(L, ws, out, (hipStream_t)stream),
                   "tsne_export_scalars");
}

int tsne_export_p_rows(void *ws, int64_t n, int64_t row0, int64_t nrows, float *out,
                       void *stream) {
  if (int rc = check_iter_args("tsne_export_p_rows", ws, n)) return rc;
  if (!out) return fail(TSNE_E_ARG, "tsne_export_p_rows: null pointer");
  if (row0 < 0 || nrows < 0 || row0 + nrows > n)
    return fail(TSNE_E_ARG, "tsne_export_p_rows: rows out of range");
  const Layout L = tsne::make_layout(n, 1, TSNE_DIST_FP64);
  return hip_check(tsne::launch_export_p_rows(L, ws, row0, nrows, out, (hipStream_t)stream),
                   "tsne_export_p_rows");
}

int tsne_export_order(void *ws, int64_t n, int32_t *perm, uint8_t *flags, void *stream) {
  if (int rc = check_iter_args("tsne_export_order", ws, n)) return rc;
  const Layout L = tsne::make_layout(n, 1, TSNE_DIST_FP64);
  return hip_check(tsne::launch_export_order(L, ws, perm, flags, (hipStream_t)stream),
                   "tsne_export_order");
}

size_t tsne_batch_workspace_bytes(int32_t count) {
  if (count < 1 || count > (1 << 20)) return 0;
  return tsne::kBatchHdrBytes + (size_t)count * sizeof(tsne::BatchEntry);
}

static int batch_totals(const char *fn, const tsne_batch_problem *pr, int32_t count,
                        int64_t &tiles, int64_t &blocks) {
  if (!pr || count < 1) return fail(TSNE_E_ARG, "%s: no problems", fn);
  tiles = 0;
  blocks = 0;
  for (int32_t p = 0; p < count; ++p) {
    if (!pr[p].ws || !pr[p].y || !pr[p].u || !pr[p].g)
      return fail(TSNE_E_ARG, "%s: null pointer in problem %d", fn, p);
    if (!valid_n(pr[p].n)) return fail(TSNE_E_ARG, "%s: problem %d: bad n", fn, p);
    if (!aligned(pr[p].ws, 256))
      return fail(TSNE_E_WORKSPACE, "%s: problem %d: ws not 256-byte aligned", fn, p);
    const tsne::Layout L = tsne::make_layout(pr[p].n, 1, TSNE_DIST_FP64);
    tiles += L.nt;
    blocks += L.nb;
  }
  if (tiles >= ((int64_t)1 << 31) || blocks >= ((int64_t)1 << 31))
    return fail(TSNE_E_ARG, "%s: batch too large for one launch", fn);
  return TSNE_OK;
}

int tsne_batch_plan(const tsne_batch_problem *problems, int32_t count, void *batch_ws,
                    size_t batch_ws_bytes, void *stream) {
  int64_t tiles, blocks;
  if (int rc = batch_totals("tsne_batch_plan", problems, count, tiles, blocks)) return rc;
  if (!batch_ws || !aligned(batch_ws, 256))
    return fail(TSNE_E_WORKSPACE, "tsne_batch_plan: batch_ws null or misaligned");
  const size_t need = tsne_batch_workspace_bytes(count);
  if (batch_ws_bytes < need)
    return fail(TSNE_E_WORKSPACE, "tsne_batch_plan: batch workspace %zu bytes, need %zu",
                batch_ws_bytes, need);
  char *host = (char *)calloc(1, need);
  if (!host) return fail(TSNE_E_DEVICE, "tsne_batch_plan: host allocation failed");
  tsne::BatchHdr *bh = reinterpret_cast<tsne::BatchHdr *>(host);
  bh->magic = tsne::kBatchMagic;
  bh->count = count;
  bh->total_tiles = tiles;
  bh->total_blocks = blocks;
  tsne::BatchEntry *tab = reinterpret_cast<tsne::BatchEntry *>(host + tsne::kBatchHdrBytes);
  int64_t t0 = 0;
  int32_t b0 = 0;
  for (int32_t p = 0; p < count; ++p) {
    const tsne::Layout L = tsne::make_layout(problems[p].n, 1, TSNE_DIST_FP64);
    void *ws = problems[p].ws;
    tsne::BatchEntry &e = tab[p];
    e.P = tsne::at<const float4>(ws, L.P);
    e.Y = reinterpret_cast<float2 *>(problems[p].y);
    e.U = reinterpret_cast<float2 *>(problems[p].u);
    e.G = reinterpret_cast<float2 *>(problems[p].g);
    e.part = tsne::at<float4>(ws, L.part);
    e.zpart = tsne::at<float>(ws, L.zpart);
    e.meanpart = tsne::at<double2>(ws, L.meanpart);
    e.extent = tsne::at<float4>(ws, L.extent);
    e.cpart = tsne::at<double2>(ws, L.cpart);
    e.nz = tsne::at<const uint8_t>(ws, L.nz);
    e.slots = tsne::at<const int32_t>(ws, L.slots);
    e.tmap = tsne::at<const int2>(ws, L.tmap);
    e.tlist = tsne::at<const int32_t>(ws, L.tlist);
    e.tcount = tsne::at<const int32_t>(ws, L.tcount);
    e.nslots = tsne::at<const int32_t>(ws, L.nslots);
    e.perm = tsne::at<const int32_t>(ws, L.perm);
    e.yp = tsne::at<float2>(ws, L.yp);
    e.h = tsne::at<tsne::Hdr>(ws, L.hdr);
    e.n = L.n;
    e.nt = L.nt;
    e.nb = L.nb;
    e.tile0 = t0;
    e.blk0 = b0;
    t0 += L.nt;
    b0 += L.nb;
  }
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(batch_ws, host, need, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  free(host);
  return hip_check(e, "tsne_batch_plan");
}

int tsne_batch_step(const tsne_batch_problem *problems, int32_t count, const void *batch_ws,
                    const tsne_step_params *prm, void *stream) {
  int64_t tiles, blocks;
  if (int rc = batch_totals("tsne_batch_step", problems, count, tiles, blocks)) return rc;
  if (!batch_ws || !prm) return fail(TSNE_E_ARG, "tsne_batch_step: null pointer");
  if (int rc = check_params("tsne_batch_step", prm)) return rc;
  return hip_check(tsne::launch_batch_step(batch_ws, count, tiles, blocks, prm->exaggeration,
                                           prm->momentum, prm->learning_rate, prm->min_gain,
                                           prm->recentre, prm->lr_rule, (hipStream_t)stream),
                   "tsne_batch_step");
}

int tsne_batch_cost(const tsne_batch_problem *problems, int32_t count, const void *batch_ws,
                    double *out, void *stream) {
  int64_t tiles, blocks;
  if (int rc = batch_totals("tsne_batch_cost", problems, count, tiles, blocks)) return rc;
  if (!batch_ws || !out) return fail(TSNE_E_ARG, "tsne_batch_cost: null pointer");
  return hip_check(tsne::launch_batch_cost(batch_ws, count, tiles, blocks, out,
                                           (hipStream_t)stream),
                   "tsne_batch_cost");
}

size_t tsne_kde_workspace_bytes(int64_t n) {
  if (n < 3 || n > ((int64_t)1 << 30)) return 0;
  return tsne::make_layout(n, 2, TSNE_DIST_FP64, true).total;
}

int tsne_kde_bandwidths(const float *y, int64_t n, double perplexity, double *beta, void *ws,
                        size_t ws_bytes, void *stream) {
  if (!y || !ws || !beta) return fail(TSNE_E_ARG, "tsne_kde_bandwidths: null pointer");
  if (n < 3 || n > ((int64_t)1 << 30))
    return fail(TSNE_E_ARG, "tsne_kde_bandwidths: n = %lld out of range", (long long)n);
  if (!(perplexity > 1.0) || !(perplexity < (double)(n - 1)))
    return fail(TSNE_E_PERPLEXITY, "tsne_kde_bandwidths: perplexity %g not in (1, n-1 = %lld)",
                perplexity, (long long)(n - 1));
  if (!aligned(ws, 256)) return fail(TSNE_E_WORKSPACE, "tsne_kde_bandwidths: ws not aligned");
  const Layout L = tsne::make_layout(n, 2, TSNE_DIST_FP64, true);
  if (ws_bytes < L.total)
    return fail(TSNE_E_WORKSPACE, "tsne_kde_bandwidths: workspace %zu bytes, need %zu",
                ws_bytes, L.total);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = tsne::launch_affinities(L, y, nullptr, perplexity, 200, 1e-6, 0, ws, st, true);
  // no reordering: the row statistics are in the caller's order
  if (e == hipSuccess)
    e = hipMemcpyAsync(beta, tsne::at<double>(ws, L.beta), (size_t)n * sizeof(double),
                       hipMemcpyDeviceToDevice, st);
  return hip_check(e, "tsne_kde_bandwidths");
}

int tsne_kde_raster(const float *y, int64_t n, const double *beta, const tsne_raster *grid,
                    float *out, void *stream) {
  if (!y || !beta || !grid || !out) return fail(TSNE_E_ARG, "tsne_kde_raster: null pointer");
  if (n < 1 || n > ((int64_t)1 << 30))
    return fail(TSNE_E_ARG, "tsne_kde_raster: n = %lld out of range", (long long)n);
  const tsne_raster g = *grid;
  if (g.gx < 1 || g.gy < 1 || (int64_t)g.gx * g.gy > ((int64_t)1 << 30) || !(g.cx > 0.f) ||
      !(g.cy > 0.f) || !isfinite(g.x0) || !isfinite(g.y0) || !isfinite(g.cx) || !isfinite(g.cy))
    return fail(TSNE_E_ARG, "tsne_kde_raster: invalid raster");
  return hip_check(tsne::launch_kde_raster(y, n, beta, g, out, (hipStream_t)stream),
                   "tsne_kde_raster");
}

static bool mlp_dims_ok(int32_t d_in, int32_t hidden) {
  return d_in >= 1 && d_in <= 64 && hidden >= 64 && hidden <= 256 && hidden % 64 == 0;
}

int64_t tsne_mlp_param_count(int32_t d_in, int32_t hidden) {
  if (!mlp_dims_ok(d_in, hidden)) return 0;
  return (int64_t)hidden * d_in + hidden + (int64_t)hidden * hidden + hidden + 2 * hidden + 2;
}

size_t tsne_mlp_workspace_bytes(int32_t d_in, int32_t hidden, int64_t batch, int32_t train) {
  if (!mlp_dims_ok(d_in, hidden) || batch < 1 || batch > ((int64_t)1 << 28)) return 0;
  return tsne::make_mlp_layout(d_in, hidden, (batch + 63) / 64 * 64, train != 0).total;
}

// Largest batch (multiple of 64) whose layout fits in ws_bytes, or 0.
static int64_t mlp_capacity(int32_t d_in, int32_t hidden, size_t ws_bytes, bool train) {
  if (tsne::make_mlp_layout(d_in, hidden, 64, train).total > ws_bytes) return 0;
  int64_t lo = 64, hi = 128;
  while (hi <= ((int64_t)1 << 28) && tsne::make_mlp_layout(d_in, hidden, hi, train).total <= ws_bytes)
    hi *= 2;
  while (hi - lo > 64) {
    int64_t mid = (lo + hi) / 2 / 64 * 64;
    if (mid <= lo) break;
    if (tsne::make_mlp_layout(d_in, hidden, mid, train).total <= ws_bytes)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

int tsne_mlp_forward(const float *params, int32_t d_in, int32_t hidden, const float *mean,
                     const float *invstd, const float *x, int64_t n, float *out, void *ws,
                     size_t ws_bytes, void *stream) {
  if (!params || !mean || !invstd || !x || !out || !ws)
    return fail(TSNE_E_ARG, "tsne_mlp_forward: null pointer");
  if (!mlp_dims_ok(d_in, hidden) || n < 1)
    return fail(TSNE_E_ARG, "tsne_mlp_forward: unsupported d_in %d / hidden %d / n %lld", d_in,
                hidden, (long long)n);
  if (!aligned(ws, 256)) return fail(TSNE_E_WORKSPACE, "tsne_mlp_forward: ws not 256-byte aligned");
  const int64_t cap = mlp_capacity(d_in, hidden, ws_bytes, false);
  if (cap == 0) return fail(TSNE_E_WORKSPACE, "tsne_mlp_forward: workspace too small");
  const tsne::MlpLayout L = tsne::make_mlp_layout(d_in, hidden, cap, false);
  return hip_check(tsne::launch_mlp_forward(L, params, mean, invstd, x, n, out, ws,
                                            (hipStream_t)stream),
                   "tsne_mlp_forward");
}

int tsne_mlp_forward_noalloc(const float *params, int32_t d_in, int32_t hidden,
                             const float *mean, const float *invstd, const float *x, int64_t n,
                             float *out, void *stream) {
  if (!params || !mean || !invstd || !x || !out)
    return fail(TSNE_E_ARG, "tsne_mlp_forward_noalloc: null pointer");
  if (!mlp_dims_ok(d_in, hidden) || n < 1)
    return fail(TSNE_E_ARG, "tsne_mlp_forward_noalloc: unsupported d_in %d / hidden %d / n %lld",
                d_in, hidden, (long long)n);
  const tsne::MlpLayout L = tsne::make_mlp_layout(d_in, hidden, 64, false);
  if (L.total > tsne::kNoAllocScratchBytes)
    return fail(TSNE_E_WORKSPACE,
                "tsne_mlp_forward_noalloc: needs %zu bytes of scratch, the library holds %zu",
                L.total, tsne::kNoAllocScratchBytes);
  void *scr = nullptr;
  hipError_t e = tsne::noalloc_scratch(&scr);
  if (e != hipSuccess) return hip_check(e, "tsne_mlp_forward_noalloc: scratch address");
  return hip_check(tsne::launch_mlp_forward(L, params, mean, invstd, x, n, out, scr,
                                            (hipStream_t)stream),
                   "tsne_mlp_forward_noalloc");
}

int tsne_mlp_gradient(const float *params, int32_t d_in, int32_t hidden, const float *mean,
                      const float *invstd, const float *x, const float *y, const int32_t *idx,
                      int64_t batch, float *grad, double *loss, void *ws, size_t ws_bytes,
                      void *stream) {
  if (!params || !mean || !invstd || !x || !y || !grad || !loss || !ws)
    return fail(TSNE_E_ARG, "tsne_mlp_gradient: null pointer");
  if (!mlp_dims_ok(d_in, hidden) || batch < 1)
    return fail(TSNE_E_ARG, "tsne_mlp_gradient: unsupported d_in %d / hidden %d / batch %lld",
                d_in, hidden, (long long)batch);
  if (!aligned(ws, 256))
    return fail(TSNE_E_WORKSPACE, "tsne_mlp_gradient: ws not 256-byte aligned");
  const int64_t bpad = (batch + 63) / 64 * 64;
  const tsne::MlpLayout L = tsne::make_mlp_layout(d_in, hidden, bpad, true);
  if (L.total > ws_bytes)
    return fail(TSNE_E_WORKSPACE, "tsne_mlp_gradient: workspace %zu bytes, need %zu", ws_bytes,
                L.total);
  return hip_check(tsne::launch_mlp_gradient(L, params, mean, invstd, x, y, idx, batch, grad, loss,
                                             ws, (hipStream_t)stream),
                   "tsne_mlp_gradient");
}

int tsne_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t count, float lr,
                  float beta1, float beta2, float eps, int32_t t, void *stream) {
  if (!params || !grad || !m || !v) return fail(TSNE_E_ARG, "tsne_mlp_adam: null pointer");
  if (count < 1 || t < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(TSNE_E_ARG, "tsne_mlp_adam: invalid arguments");
  return hip_check(tsne::launch_adam(params, grad, m, v, count, lr, beta1, beta2, eps, t,
                                     (hipStream_t)stream),
                   "tsne_mlp_adam");
}

}  // extern "C"
