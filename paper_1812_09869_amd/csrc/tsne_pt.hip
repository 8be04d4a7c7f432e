// Parallel scheme (ptSNE, section "Parallelized implementation"): the n points
// are split into `threads` chunks of a per-epoch order; partial t-SNE k runs on
// chunks k .. k+layers-1 (cyclic), each chunk entering at its points' layer-l
// positions, l its place in the thread; after a short run every partial
// result is written back to the layer it was read from.
//
// Device work per epoch, all on the caller's stream (the per-thread
// affinities fan out over side streams and join back):
//   mix      one launch: the rows of every partial problem (X rows, start map
//            from the layers, zero momentum) gathered into pooled buffers;
//   P        the affinities of every partial problem (Eqs. 1-3);
//   iterate  the batched iteration of all partial problems at once, with the
//            paper's learning rate (Eq. 11) and no exaggeration;
//   monitor  each partial problem's pseudo-normalised cost (Eq. 9), then one
//            launch pools the maps back into the layers, and two more form
//            the mean partial cost and the mean layer size.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/tsne355.h"
#include "tsne_internal.h"

namespace {

constexpr uint32_t kPtMagic = 0x70745331u;
constexpr int kPtStreams = 4;
constexpr int kExtBlocks = 64;  // partial extents per layer

struct PtHdr {
  uint32_t magic;
  int32_t status;  // TSNE_OK, or TSNE_E_ARG for an order entry out of range
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Host-side layout of the ptSNE workspace; recomputed identically on every call.
struct PtLayout {
  int64_t n = 0, rows = 0;
  int32_t d = 0, T = 0, L = 0, mode = 0;
  std::vector<int64_t> z, row0;  // thread sizes and first pooled row
  std::vector<size_t> ws;        // offset of each partial problem's workspace
  std::vector<size_t> wsb;       // its size
  size_t hdr = 0, rowtab = 0, xk = 0, yk = 0, uk = 0, gk = 0, src = 0, lay = 0, costs = 0,
         ext = 0, batch = 0, batch_bytes = 0, smalltab = 0, total = 0;
  int64_t zmin = 0, zmax = 0;
  // totals of the batched small-problem affinity path (used when `small`)
  bool small = false;
  int64_t small_wgs = 0, small_tiles = 0, small_blocks = 0;
};

int64_t chunk_size(int64_t n, int32_t T, int32_t c) { return n / T + (c < n % T ? 1 : 0); }

bool make_pt_layout(int64_t n, int32_t d, const tsne_pt_opts &o, PtLayout &P) {
  P.n = n;
  P.d = d;
  P.T = o.threads;
  P.L = o.layers;
  P.mode = o.dist_mode;
  P.z.assign(P.T, 0);
  P.row0.assign(P.T + 1, 0);
  for (int32_t k = 0; k < P.T; ++k) {
    int64_t s = 0;
    for (int32_t l = 0; l < P.L; ++l) s += chunk_size(n, P.T, (k + l) % P.T);
    P.z[k] = s;
    P.row0[k + 1] = P.row0[k] + s;
  }
  P.rows = P.row0[P.T];
  P.zmin = P.z[0];
  P.zmax = P.z[0];
  for (int64_t s : P.z) {
    P.zmin = s < P.zmin ? s : P.zmin;
    P.zmax = s > P.zmax ? s : P.zmax;
  }
  // every partial problem small enough for the batched one-wave-per-row path
  P.small = o.dist_mode == TSNE_DIST_FP64 && o.reorder == 0 && P.zmax <= tsne::kSmallMaxN &&
            d <= tsne::kSmallMaxD;
  if (P.small) {
    for (int64_t s : P.z) {
      const tsne::Layout L = tsne::make_layout(s, d, TSNE_DIST_FP64);
      P.small_wgs += (s + tsne::kSmallRows - 1) / tsne::kSmallRows;
      P.small_tiles += L.nt;
      P.small_blocks += L.nb;
    }
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  P.hdr = take(256);
  P.rowtab = take((size_t)(P.T + 1) * 8);
  P.xk = take((size_t)P.rows * d * 4);
  P.yk = take((size_t)P.rows * 8);
  P.uk = take((size_t)P.rows * 8);
  P.gk = take((size_t)P.rows * 8);
  P.src = take((size_t)P.rows * 4);
  P.lay = take((size_t)P.rows * 4);
  P.costs = take((size_t)P.T * 16);
  P.ext = take((size_t)P.L * kExtBlocks * 16);
  P.batch_bytes = tsne_batch_workspace_bytes(P.T);
  if (P.batch_bytes == 0) return false;
  P.batch = take(P.batch_bytes);
  P.smalltab = take((size_t)P.T * sizeof(tsne::SmallEntry));
  P.ws.resize(P.T);
  P.wsb.resize(P.T);
  for (int32_t k = 0; k < P.T; ++k) {
    const size_t b = tsne_workspace_bytes(P.z[k], d, o.dist_mode);
    if (b == 0) return false;
    P.wsb[k] = b;
    P.ws[k] = take(b);
  }
  P.total = off;
  return true;
}

template <class U>
U *at(void *base, size_t off) {
  return reinterpret_cast<U *>(static_cast<char *>(base) + off);
}

thread_local char g_pt_err[512];

int pt_fail(int code, const char *msg, long long a = 0, long long b = 0) {
  snprintf(g_pt_err, sizeof g_pt_err, msg, a, b);
  return code;
}

// A failure of a call into the single-problem API: its message is kept.
int nested_fail(int rc, const char *what, long long k) {
  snprintf(g_pt_err, sizeof g_pt_err, "%s (partial problem %lld): %s", what, k, tsne_last_error());
  return rc;
}

int hip_fail(hipError_t e, const char *what) {
  snprintf(g_pt_err, sizeof g_pt_err, "%s: %s", what, hipGetErrorString(e));
  return TSNE_E_DEVICE;
}

// Argument checks shared by every entry point.
int check_pt(int64_t n, int32_t d, const tsne_pt_opts *o, PtLayout &P) {
  if (!o) return pt_fail(TSNE_E_ARG, "tsne_pt: null options");
  if (n < 2 || n > ((int64_t)1 << 30)) return pt_fail(TSNE_E_ARG, "tsne_pt: n = %lld out of range", n);
  if (d < 1 || d > 65536) return pt_fail(TSNE_E_ARG, "tsne_pt: d = %lld out of range", d);
  if (o->threads < 1 || o->threads > n)
    return pt_fail(TSNE_E_ARG, "tsne_pt: threads = %lld not in [1, n]", o->threads);
  if (o->layers < 1 || o->layers > o->threads)
    return pt_fail(TSNE_E_ARG, "tsne_pt: layers = %lld not in [1, threads]", o->layers);
  if (o->dist_mode < TSNE_DIST_FP64 || o->dist_mode > TSNE_DIST_FP16X3)
    return pt_fail(TSNE_E_ARG, "tsne_pt: unknown distance mode %lld", o->dist_mode);
  if (!isfinite(o->momentum) || o->reserved != 0)
    return pt_fail(TSNE_E_ARG, "tsne_pt: momentum must be finite and reserved 0");
  if (!make_pt_layout(n, d, *o, P)) return pt_fail(TSNE_E_ARG, "tsne_pt: thread problem too small");
  if (P.zmin < 2) return pt_fail(TSNE_E_ARG, "tsne_pt: a partial problem has %lld points", P.zmin);
  if (!(o->perplexity > 1.0) || !(o->perplexity < (double)(P.zmin - 1)))
    return pt_fail(TSNE_E_PERPLEXITY,
                   "tsne_pt: perplexity must lie in (1, smallest thread size - 1 = %lld)",
                   P.zmin - 1);
  return TSNE_OK;
}

int check_ws(void *ws, size_t bytes, const PtLayout &P) {
  if (!ws || ((uintptr_t)ws % 256) != 0)
    return pt_fail(TSNE_E_WORKSPACE, "tsne_pt: workspace null or not 256-byte aligned");
  if (bytes < P.total)
    return pt_fail(TSNE_E_WORKSPACE, "tsne_pt: workspace %lld bytes, need %lld", (long long)bytes,
                   (long long)P.total);
  return TSNE_OK;
}

// Prefix offsets of the small-problem table (first workgroup of kSmallRows rows,
// first tile, first row block of each problem); the totals are the layout's.
void small_prefix(std::vector<tsne::SmallEntry> &tab) {
  int64_t w = 0, t = 0, b = 0;
  for (auto &e : tab) {
    e.wg0 = w;
    e.tile0 = t;
    e.blk0 = b;
    w += (e.n + tsne::kSmallRows - 1) / tsne::kSmallRows;
    t += e.nt;
    b += e.nb;
  }
}

std::vector<tsne_batch_problem> problems_of(const PtLayout &P, void *ws) {
  std::vector<tsne_batch_problem> pr(P.T);
  for (int32_t k = 0; k < P.T; ++k) {
    pr[k].ws = at<char>(ws, P.ws[k]);
    pr[k].n = P.z[k];
    pr[k].y = at<float>(ws, P.yk) + 2 * P.row0[k];
    pr[k].u = at<float>(ws, P.uk) + 2 * P.row0[k];
    pr[k].g = at<float>(ws, P.gk) + 2 * P.row0[k];
  }
  return pr;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Mix: one wave per pooled row r. The thread k of the row is found by binary
// search on the first rows; its place s within the thread gives the chunk
// (k + l) mod T and the layer l; the point is order[start of chunk + offset].
__global__ __launch_bounds__(256) void k_pt_mix(const float *__restrict__ x, int64_t n, int32_t d,
                                                int32_t T, int32_t L,
                                                const int32_t *__restrict__ order,
                                                const float2 *__restrict__ maps,
                                                const int64_t *__restrict__ row0, int64_t rows,
                                                float *__restrict__ xk, float2 *__restrict__ yk,
                                                float2 *__restrict__ uk, float2 *__restrict__ gk,
                                                int32_t *__restrict__ src,
                                                int32_t *__restrict__ lay, PtHdr *hdr) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  int lo = 0, hi = T - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (row0[mid] <= r)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int k = lo;
  int64_t s = r - row0[k];
  const int64_t q = n / T, rem = n % T;
  int l = 0;
  int64_t start = 0;
  for (; l < L; ++l) {
    const int64_t c = (k + l) % T;
    const int64_t sz = q + (c < rem ? 1 : 0);
    if (s < sz) {
      start = c * q + (c < rem ? c : rem);
      break;
    }
    s -= sz;
  }
  int64_t i = (l < L) ? (int64_t)order[start + s] : -1;
  const bool ok = i >= 0 && i < n;
  if (!ok) {
    if (lane == 0) hdr->status = TSNE_E_ARG;
    i = 0;
  }
  if (l >= L) l = 0;
  for (int j = lane; j < d; j += 64) xk[r * d + j] = x[i * d + j];
  if (lane == 0) {
    yk[r] = maps[(int64_t)l * n + i];
    uk[r] = make_float2(0.f, 0.f);
    gk[r] = make_float2(1.f, 1.f);
    src[r] = (int32_t)i;
    lay[r] = l;
  }
}

// Pool: every pooled row back to the layer and point it was read from.
__global__ __launch_bounds__(256) void k_pt_pool(const float2 *__restrict__ yk,
                                                 const int32_t *__restrict__ src,
                                                 const int32_t *__restrict__ lay, int64_t rows,
                                                 int64_t n, float2 *__restrict__ maps) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r < rows) maps[(int64_t)lay[r] * n + src[r]] = yk[r];
}

__device__ inline float4 ext_merge(float4 a, float4 b) {
  return make_float4(fminf(a.x, b.x), fmaxf(a.y, b.y), fminf(a.z, b.z), fmaxf(a.w, b.w));
}

__device__ inline float4 ext_wave(float4 e) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
    e = ext_merge(e, make_float4(__shfl_xor(e.x, o), __shfl_xor(e.y, o), __shfl_xor(e.z, o),
                                 __shfl_xor(e.w, o)));
  return e;
}

// Extents of each layer: grid (kExtBlocks, L), strided over the points.
__global__ __launch_bounds__(256) void k_pt_extent(const float2 *__restrict__ maps, int64_t n,
                                                   float4 *__restrict__ part) {
  __shared__ float4 red[4];
  const int l = blockIdx.y;
  float4 e = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kExtBlocks * 256) {
    const float2 v = maps[(int64_t)l * n + i];
    e = ext_merge(e, make_float4(v.x, v.x, v.y, v.y));
  }
  e = ext_wave(e);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0)
    part[l * kExtBlocks + blockIdx.x] = ext_merge(ext_merge(red[0], red[1]),
                                                  ext_merge(red[2], red[3]));
}

// Monitors: out[0] = mean over threads of the partial C_norm, out[1] = mean
// over layers of the diagonal of the layer's box. One wave, fixed order.
__global__ __launch_bounds__(64) void k_pt_monitor(const double2 *__restrict__ costs, int32_t T,
                                                   const float4 *__restrict__ part, int32_t L,
                                                   double *__restrict__ out) {
  const int lane = threadIdx.x;
  double c = 0.0;
  for (int k = lane; k < T; k += 64) c += costs[k].y;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  double size = 0.0;
  for (int l = 0; l < L; ++l) {
    float4 e = part[l * kExtBlocks + lane];  // kExtBlocks == 64: one partial per lane
    e = ext_wave(e);
    const double rx = (double)e.y - (double)e.x, ry = (double)e.w - (double)e.z;
    size += sqrt(rx * rx + ry * ry);
  }
  if (lane == 0) {
    out[0] = c / (double)T;
    out[1] = size / (double)L;
  }
}

__global__ void k_pt_hdr(PtHdr *h) {
  h->magic = kPtMagic;
  h->status = TSNE_OK;
}

static_assert(kExtBlocks == 64, "the monitor kernel reads one extent partial per lane");

// Side streams for the per-thread affinity and cost calls (default priority).
struct PtStreams {
  hipStream_t s[kPtStreams] = {};
  hipEvent_t fork = nullptr, join[kPtStreams] = {};
};
std::mutex g_pt_mu;
PtStreams g_pt[64];

hipError_t pt_streams(PtStreams *&out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  PtStreams &p = g_pt[dev];
  if (!p.fork) {
    for (int i = 0; i < kPtStreams; ++i) {
      if ((e = hipStreamCreateWithFlags(&p.s[i], hipStreamNonBlocking)) != hipSuccess) return e;
      if ((e = hipEventCreateWithFlags(&p.join[i], hipEventDisableTiming)) != hipSuccess) return e;
    }
    if ((e = hipEventCreateWithFlags(&p.fork, hipEventDisableTiming)) != hipSuccess) return e;
  }
  out = &p;
  return hipSuccess;
}

hipError_t fork_streams(PtStreams &p, hipStream_t st) {
  hipError_t e = hipEventRecord(p.fork, st);
  for (int i = 0; e == hipSuccess && i < kPtStreams; ++i) e = hipStreamWaitEvent(p.s[i], p.fork, 0);
  return e;
}

hipError_t join_streams(PtStreams &p, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int i = 0; e == hipSuccess && i < kPtStreams; ++i) {
    e = hipEventRecord(p.join[i], p.s[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, p.join[i], 0);
  }
  return e;
}

}  // namespace

extern "C" {

TSNE_API const char *tsne_pt_last_error(void) { return g_pt_err; }

TSNE_API size_t tsne_pt_workspace_bytes(int64_t n, int32_t d, const tsne_pt_opts *opts) {
  PtLayout P;
  if (check_pt(n, d, opts, P) != TSNE_OK) return 0;
  return P.total;
}

TSNE_API int32_t tsne_pt_iterations(int64_t n, const tsne_pt_opts *opts) {
  if (!opts || opts->threads < 1 || opts->layers < 1 || n < 2) return 0;
  if (opts->iters > 0) return opts->iters;
  const double z = (double)n * opts->layers / opts->threads;
  return (int32_t)ceil(sqrt(z) - 1e-12);
}

TSNE_API int tsne_pt_init(int64_t n, int32_t d, const tsne_pt_opts *opts, void *ws, size_t bytes,
                          void *stream) {
  PtLayout P;
  if (int rc = check_pt(n, d, opts, P)) return rc;
  if (int rc = check_ws(ws, bytes, P)) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_pt_hdr, dim3(1), dim3(1), 0, st, at<PtHdr>(ws, P.hdr));
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(at<char>(ws, P.rowtab), P.row0.data(), (size_t)(P.T + 1) * 8,
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host table must outlive the copy
  if (e != hipSuccess) return hip_fail(e, "tsne_pt_init");
  std::vector<tsne_batch_problem> pr = problems_of(P, ws);
  int rc = tsne_batch_plan(pr.data(), P.T, at<char>(ws, P.batch), P.batch_bytes, stream);
  if (rc != TSNE_OK) return nested_fail(rc, "tsne_pt_init: batch plan", -1);
  if (P.small) {
    std::vector<tsne::SmallEntry> tab(P.T);
    for (int32_t k = 0; k < P.T; ++k) {
      const tsne::Layout L = tsne::make_layout(P.z[k], d, TSNE_DIST_FP64);
      tsne::small_entry(L, at<char>(ws, P.ws[k]), at<float>(ws, P.xk) + P.row0[k] * d,
                        opts->perplexity, tab[k]);
    }
    small_prefix(tab);
    e = hipMemcpyAsync(at<char>(ws, P.smalltab), tab.data(), tab.size() * sizeof(tab[0]),
                       hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "tsne_pt_init (small table)");
  }
  g_pt_err[0] = '\0';
  return TSNE_OK;
}

TSNE_API int tsne_pt_epoch(const float *x, int64_t n, int32_t d, const tsne_pt_opts *opts,
                           const int32_t *order, float *maps, void *ws, size_t bytes,
                           double *monitors, void *stream) {
  PtLayout P;
  if (int rc = check_pt(n, d, opts, P)) return rc;
  if (int rc = check_ws(ws, bytes, P)) return rc;
  if (!x || !order || !maps) return pt_fail(TSNE_E_ARG, "tsne_pt_epoch: null pointer");
  hipStream_t st = (hipStream_t)stream;
  const int32_t iters = tsne_pt_iterations(n, opts);
  float *xk = at<float>(ws, P.xk);
  float2 *yk = at<float2>(ws, P.yk);
  int32_t *src = at<int32_t>(ws, P.src), *lay = at<int32_t>(ws, P.lay);
  double *costs = at<double>(ws, P.costs);

  // mix
  hipLaunchKernelGGL(k_pt_mix, dim3((unsigned)((P.rows + 3) / 4)), dim3(256), 0, st, x, n, d, P.T,
                     P.L, order, reinterpret_cast<const float2 *>(maps),
                     at<const int64_t>(ws, P.rowtab), P.rows, xk, yk, at<float2>(ws, P.uk),
                     at<float2>(ws, P.gk), src, lay, at<PtHdr>(ws, P.hdr));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "tsne_pt_epoch (mix)");

  std::vector<tsne_batch_problem> pr = problems_of(P, ws);
  const tsne_aff_opts ao = {opts->dist_mode, 200, 1e-6, opts->reorder, 0};
  if (P.small) {
    // all partial problems in one launch per phase
    e = tsne::launch_affinities_small(at<const tsne::SmallEntry>(ws, P.smalltab), P.T, P.small_wgs,
                                      P.small_tiles, P.small_blocks, P.zmax, d, ao.max_bisect,
                                      ao.tol_h, st);
    if (e != hipSuccess) return hip_fail(e, "tsne_pt_epoch (affinities)");
  } else {
    // affinities of every partial problem, spread over the side streams
    std::lock_guard<std::mutex> lock(g_pt_mu);
    PtStreams *ps = nullptr;
    if ((e = pt_streams(ps)) != hipSuccess || (e = fork_streams(*ps, st)) != hipSuccess)
      return hip_fail(e, "tsne_pt_epoch (streams)");
    for (int32_t k = 0; k < P.T; ++k) {
      int rc = tsne_affinities(xk + P.row0[k] * d, P.z[k], d, opts->perplexity, &ao, pr[k].ws,
                               P.wsb[k], ps->s[k % kPtStreams]);
      if (rc != TSNE_OK) {
        (void)join_streams(*ps, st);
        return nested_fail(rc, "tsne_pt_epoch: affinities", k);
      }
    }
    if ((e = join_streams(*ps, st)) != hipSuccess) return hip_fail(e, "tsne_pt_epoch (join)");
  }
  // iterate: Eqs. 10-11, no exaggeration, no re-centring
  const tsne_step_params prm = {1.0f, opts->momentum, 0.0f, 0.0f, 0, TSNE_LR_RANGE};
  for (int32_t t = 0; t < iters; ++t) {
    int rc = tsne_batch_step(pr.data(), P.T, at<char>(ws, P.batch), &prm, stream);
    if (rc != TSNE_OK) return nested_fail(rc, "tsne_pt_epoch: batched step", -1);
  }
  // monitors of the partial problems (one batched cost), then pool and summarise
  {
    int rc = tsne_batch_cost(pr.data(), P.T, at<char>(ws, P.batch), costs, stream);
    if (rc != TSNE_OK) return nested_fail(rc, "tsne_pt_epoch: batched cost", -1);
  }
  hipLaunchKernelGGL(k_pt_pool, dim3((unsigned)((P.rows + 255) / 256)), dim3(256), 0, st, yk, src,
                     lay, P.rows, n, reinterpret_cast<float2 *>(maps));
  float4 *ext = at<float4>(ws, P.ext);
  hipLaunchKernelGGL(k_pt_extent, dim3(kExtBlocks, (unsigned)P.L), dim3(256), 0, st,
                     reinterpret_cast<const float2 *>(maps), n, ext);
  if (monitors)
    hipLaunchKernelGGL(k_pt_monitor, dim3(1), dim3(64), 0, st,
                       reinterpret_cast<const double2 *>(costs), P.T, ext, P.L, monitors);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "tsne_pt_epoch (pool)");
  g_pt_err[0] = '\0';
  return TSNE_OK;
}

TSNE_API int tsne_pt_sync_status(int64_t n, int32_t d, const tsne_pt_opts *opts, void *ws,
                                 size_t bytes, void *stream) {
  PtLayout P;
  if (int rc = check_pt(n, d, opts, P)) return rc;
  if (int rc = check_ws(ws, bytes, P)) return rc;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "tsne_pt_sync_status");
  PtHdr h;
  e = hipMemcpy(&h, at<char>(ws, P.hdr), sizeof h, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "tsne_pt_sync_status");
  if (h.magic != kPtMagic) return pt_fail(TSNE_E_WORKSPACE, "tsne_pt: workspace not initialised");
  if (h.status != TSNE_OK) return pt_fail(h.status, "tsne_pt: order entry out of range");
  for (int32_t k = 0; k < P.T; ++k) {
    int rc = tsne_sync_status(at<char>(ws, P.ws[k]), stream);
    if (rc != TSNE_OK) return nested_fail(rc, "tsne_pt: device condition", k);
  }
  return TSNE_OK;
}

TSNE_API int tsne_pt_partial(int64_t n, int32_t d, const tsne_pt_opts *opts, void *ws,
                             size_t bytes, int32_t k, void **ws_k, int64_t *n_k) {
  PtLayout P;
  if (int rc = check_pt(n, d, opts, P)) return rc;
  if (int rc = check_ws(ws, bytes, P)) return rc;
  if (k < 0 || k >= P.T || !ws_k || !n_k)
    return pt_fail(TSNE_E_ARG, "tsne_pt_partial: partial problem %lld out of range", k);
  *ws_k = at<char>(ws, P.ws[k]);
  *n_k = P.z[k];
  g_pt_err[0] = '\0';
  return TSNE_OK;
}

}  // extern "C"
