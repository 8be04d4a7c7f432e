// Internal definitions shared by the HIP translation units of libtsne355:
// workspace layout, tile geometry, device helpers and launch wrappers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/tsne355.h"

namespace tsne {

// ---------------------------------------------------------------------------
// Tile geometry
//
// The n x n pair matrix is cut into T x T tiles; only tiles (I, J) with I <= J
// are stored ("upper triangle"), enumerated row by row. Inside a tile the
// 256 threads of a workgroup are laid out as a 16 x 16 grid (tr, tc): thread
// t = 64 w + l (wave w, lane l) has tc = l % 16, tr = l / 16 + 4 w, and owns
// rows tr + 16 k and columns tc + 16 m (k, m in 0..15). P is stored in the
// order in which these threads consume it: float4 number s * 256 + t of a
// tile holds the pairs (row tr + 16 (s / 4), column tc + 16 (4 (s % 4) + e)),
// e = 0..3, so every wave-wide float4 load is one contiguous 1 KiB segment.
// ---------------------------------------------------------------------------
constexpr int kMeanPartsPerBlock = 2;  // re-centring partial sums per row block
constexpr int64_t kImplicitTiles = 2048;  // implicit P: tiles recomputed per force launch (at least)
constexpr int T = 256;             // tile edge
constexpr int TT4 = T * T / 4;     // float4 per tile
constexpr int kThreads = 256;      // threads per tile workgroup
constexpr int kCalGroup = 4;       // row blocks per launch of the per-row search
constexpr uint64_t kMagic = 0x74534E4533353501ull;

// Error bits of the device flag word.
constexpr uint32_t kErrNonFinite = 1u;
constexpr uint32_t kErrNoConv = 2u;
constexpr uint32_t kErrState = 4u;

// Header at the start of the workspace (device memory).
struct Hdr {
  uint64_t magic;
  int64_t n;
  int32_t d;
  int32_t ready;
  uint32_t err;
  int32_t mode;
  double perplexity;
  double z;        // Z of the last force pass
  double c_p;      // sum_{i != j} p_ij ln p_ij
  double p_sum;    // sum_{i != j} p_ij
  float xmax;      // max |centred x| (operand scaling of the FP16 modes)
  float pad0;
  double pad[7];
};
static_assert(sizeof(Hdr) <= 256, "header must fit its slot");

struct Layout {
  int64_t n = 0, npad = 0, nt = 0;
  int32_t nb = 0, d = 0, dpad = 0, mode = 0;
  // byte offsets from the workspace base
  size_t hdr = 0, beta = 0, S = 0, H = 0, m = 0, a = 0, r = 0, evals = 0;
  size_t P = 0, part = 0, zpart = 0, cpart = 0, ppart = 0, meanpart = 0;
  size_t nz = 0;    // per tile: 1 if any stored p_ij of the tile is nonzero
  size_t tmap = 0;    // int2 [nt]: (I, J) of every tile, written by the pack
  size_t tlist = 0;   // int32 [nt]: all-zero tiles ascending, then the others ascending
  size_t tcount = 0;  // int32 [2]: number of all-zero tiles, number of the others
  size_t slots = 0;   // int32 [nb][nb]: per row block, its slots with nonzero P, in order
  size_t nslots = 0;  // int32 [nb]: how many
  size_t perm = 0;  // int32 [npad]: internal position -> caller's index
  size_t inv = 0;   // int32 [npad]: caller's index -> internal position
  size_t yp = 0;    // float2 [npad]: the map in the internal order (per force pass)
  size_t extent = 0;  // float4 [nb]: per-block {min x, max x, min y, max y} of that map
  size_t iter_end = 0;  // end of the part that tsne_step needs
  int32_t kk = 0;  // 16-bit operand values per point (d rounded up to 32; four slices in the x3 modes)
  int32_t cal_group = 1;  // row blocks per search launch (their distance blocks side by side)
  size_t xmean = 0, xcT = 0, norms = 0, dblock = 0;
  size_t xcT2 = 0, norms2 = 0, keys = 0, vals = 0;  // reordering
  int64_t npow2 = 0;
  size_t xfT = 0, norms32 = 0, xa = 0;  // reduced-precision operands and norms
  size_t total = 0;
};

// stats_only: a layout holding only what the per-row search needs (header,
// row statistics, order, centred X and the distance block).
// implicit: P is not stored; a buffer of whole block rows holds the P that every
// pass recomputes (FP64 distances only).
Layout make_layout(int64_t n, int32_t d, int32_t mode, bool stats_only = false,
                   bool implicit = false);

// Upper-triangle tile enumeration: row I holds tiles (I, I..nb-1).
__host__ __device__ inline int64_t tile_start(int64_t I, int64_t nb) {
  return I * nb - I * (I - 1) / 2;
}

__device__ inline void tile_coords(int64_t t, int nb, int &I, int &J) {
  double b = 2.0 * nb + 1.0;
  int i = (int)((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
  if (i < 0) i = 0;
  if (i > nb - 1) i = nb - 1;
  while (i > 0 && tile_start(i, nb) > t) --i;
  while (i < nb - 1 && tile_start(i + 1, nb) <= t) ++i;
  I = i;
  J = i + (int)(t - tile_start(i, nb));
}

// One problem of a batched iteration (device table entry).
struct BatchEntry {
  const float4 *P;
  float2 *Y, *U, *G;
  float4 *part;
  float *zpart;
  double2 *meanpart;
  float4 *extent;
  double2 *cpart;
  const uint8_t *nz;
  const int32_t *slots, *nslots;
  const int2 *tmap;
  const int32_t *tlist, *tcount;
  const int32_t *perm;
  float2 *yp;  // positions in the internal order (refreshed by every force pass)
  Hdr *h;
  int64_t n, nt, tile0;  // tile0: first global tile index of this problem
  int32_t nb, blk0;      // blk0: first global row-block index of this problem
};

// Header of a batch workspace, followed by `count` BatchEntry records.
// Affinities of many small problems at once (n <= kSmallMaxN, d <=
// kSmallMaxD, FP64 distances, the caller's order): one launch per phase for
// all of them. Device table entry of one problem; wg0, tile0 and blk0 are
// the problem's first workgroup (kSmallRows rows each), tile and row block.
constexpr int64_t kSmallMaxN = 4096;
constexpr int32_t kSmallMaxD = 64;
constexpr int kSmallRows = 8;  // rows (one wave each) per workgroup of the search
struct SmallEntry {
  const float *x;
  int64_t n, nt, wg0, tile0, blk0;
  int32_t d, nb;
  double perplexity;
  Hdr *h;
  float *a, *m, *r;
  double *beta, *S, *H;
  int32_t *evals;
  float4 *P;
  double2 *ppart;
  uint8_t *nz;
  int2 *tmap;
  int32_t *tlist, *tcount, *slots, *nslots, *perm, *inv;
};

constexpr uint64_t kBatchMagic = 0x7453424154434801ull;
struct BatchHdr {
  uint64_t magic;
  int32_t count;
  int32_t pad;
  int64_t total_tiles, total_blocks;
};
constexpr size_t kBatchHdrBytes = 256;

template <typename P>
inline P *at(void *ws, size_t off) {
  return reinterpret_cast<P *>(reinterpret_cast<char *>(ws) + off);
}

// ---------------------------------------------------------------------------
// Launch wrappers (all asynchronous on `stream`)
// ---------------------------------------------------------------------------
// Exactly one of x (n x d points) and dis (n x n dissimilarities) is non-null.
hipError_t launch_affinities(const Layout &L, const float *x, const float *dis, double perplexity,
                             int max_bisect, double tol_h, int reorder, void *ws,
                             hipStream_t stream, bool stats_only = false, bool implicit = false);
// Implicit P: recompute block b's distances and stage its tiles into the
// buffer; pack a range of staged tiles; after all blocks, the P sums and the
// slot lists.
// Implicit P: the passes check the workspace header against the shape their
// layout was computed for, n and one word holding d (below 2^20) and the
// distance mode (the mode decides which contraction operands exist).
inline __host__ __device__ int32_t implicit_key(int32_t d, int32_t mode) {
  return d | (mode << 20);
}
// Implicit P buffer capacity in tiles: at least one block row, at most the
// whole triangle.
inline int64_t implicit_capacity(const Layout &L) {
  const int64_t c = L.nb > kImplicitTiles ? L.nb : kImplicitTiles;
  return c < L.nt ? c : L.nt;
}
// Block rows [b0, b1) fill the buffer: tile t of them sits at slot
// t - tile_start(b0). The distances of the tiles tile0 .. tile0 + count - 1,
// written into the buffer in the staged layout, or with pack their packed
// P (Eq. 3, the values launch_implicit_pack would leave). skip_zero: the zero
// tiles are known (every pass after the affinity stage) and are left alone.
hipError_t launch_implicit_tiles(const Layout &L, void *ws, int64_t tile0, int64_t count,
                                 int64_t tile_base, bool skip_zero, bool pack,
                                 hipStream_t stream);
// The affinity stage's pass over every tile: zero flags, tile coordinates,
// the sums of P, slot and tile lists.
hipError_t launch_implicit_discover(const Layout &L, void *ws, hipStream_t stream);
hipError_t launch_force_implicit(const Layout &L, void *ws, const float *y, hipStream_t stream);
hipError_t launch_cost_implicit(const Layout &L, void *ws, const float *y, double *out,
                                hipStream_t stream);
// Fills the table entry of a problem whose workspace has layout L.
void small_entry(const Layout &L, void *ws, const float *x, double perplexity, SmallEntry &e);
// tab: device copy of `count` entries with prefix offsets filled in; wgs,
// tiles, blocks: their totals; nmax, dmax: the largest n and d.
hipError_t launch_affinities_small(const SmallEntry *tab, int count, int64_t wgs, int64_t tiles,
                                   int64_t blocks, int64_t nmax, int32_t dmax, int max_bisect,
                                   double tol_h, hipStream_t stream);
hipError_t launch_kde_raster(const float *y, int64_t n, const double *beta, const tsne_raster &g,
                             float *out, hipStream_t stream);
hipError_t launch_force(const Layout &L, void *ws, const float *y, hipStream_t stream);
hipError_t launch_update(const Layout &L, void *ws, float *y, float *u, float *g, float alpha,
                         float mu, float eta, float min_gain, int recentre, int lr_rule,
                         float *grad_out, double *z_out, hipStream_t stream);
hipError_t launch_gradient_only(const Layout &L, void *ws, float alpha, float *grad_out,
                                double *z_out, hipStream_t stream);
hipError_t launch_cost(const Layout &L, void *ws, const float *y, double *out,
                       hipStream_t stream);
hipError_t launch_batch_cost(const void *batch_ws, int count, int64_t total_tiles,
                             int64_t total_blocks, double *out, hipStream_t stream);
hipError_t launch_batch_step(const void *batch_ws, int count, int64_t total_tiles,
                             int64_t total_blocks, float alpha, float mu, float eta,
                             float min_gain, int recentre, int lr_rule, hipStream_t stream);
hipError_t launch_export_p_rows(const Layout &L, void *ws, int64_t row0, int64_t nrows,
                                float *out, hipStream_t stream);
hipError_t launch_export_scalars(const Layout &L, void *ws, double *out, hipStream_t stream);
hipError_t launch_export_order(const Layout &L, void *ws, int32_t *perm, uint8_t *flags,
                               hipStream_t stream);
hipError_t launch_export_rowstats(const Layout &L, void *ws, double *beta, float *m, double *S,
                                  double *H, int32_t *evals, hipStream_t stream);

}  // namespace tsne
