// Exact gradient iteration (Eqs. 4-6 and 10 of the bigMap paper) and the KL
// cost (Eqs. 5 and 9).
//
// Force pass over the stored upper-triangle tiles. For every unordered pair
// (i, j) of a tile, with d = y_i - y_j and w = 1 / (1 + |d|^2):
//   Z   += 2 w                     (ordered pairs, denominator of Eq. 4)
//   A_i += p w d,  A_j -= p w d     (attraction, Eq. 6 numerator with p)
//   R_i += w^2 d,  R_j -= w^2 d     (repulsion, Eq. 6 with q = w / Z)
// so that g_i = 4 (alpha A_i - R_i / Z) once Z is known. A diagonal tile
// holds both orders of each pair and accumulates the row side only.
//
// Each tile writes its row-side partials into the slot (I, J) of block I and
// its column-side partials into the slot (J, I) of block J; every slot is
// written exactly once per pass and the update sums the slots of a row in a
// fixed order in FP64, so results are bitwise reproducible. The partial-sum
// buffer holds two float2 arrays of nb x nb x T: the repulsive sums (R_x,
// R_y) of every slot, then the attractive sums (A_x, A_y), written and read
// only for slots whose tile holds nonzero P.
#include <math.h>

#include <mutex>

#include "tsne_internal.h"

namespace tsne {

namespace {

constexpr double kLn2 = 0.69314718055994530942;

__device__ inline float2 *part_rep(float4 *part) { return reinterpret_cast<float2 *>(part); }
__device__ inline float2 *part_att(float4 *part, int32_t nb) {
  return reinterpret_cast<float2 *>(part) + (size_t)nb * nb * T;
}
__device__ inline const float2 *part_rep(const float4 *part) {
  return reinterpret_cast<const float2 *>(part);
}
__device__ inline const float2 *part_att(const float4 *part, int32_t nb) {
  return reinterpret_cast<const float2 *>(part) + (size_t)nb * nb * T;
}

__device__ inline void flag_error(Hdr *h, uint32_t bit) { atomicOr(&h->err, bit); }

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the 16 lanes of a DPP row (rotations by 8, 4, 2, 1); every lane of
// the row ends with the total. A rotation reads no lane outside the row, so
// bound_ctrl does not change the result; setting it lets the compiler fold
// each move into its add (one v_add_f32 with a DPP operand).
__device__ inline float row16_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x124, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x122, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x121, 0xf, 0xf, true));
  return v;
}

// Bit k set when position off + 16 k of a tile is a real row (or column):
// rem = n - (first index of the tile's block), which may exceed T.
__device__ inline uint32_t valid_bits(int64_t rem, int off) {
  if (rem >= T) return 0xFFFFu;
  const int64_t c = rem - off;
  if (c <= 0) return 0u;
  const int64_t cnt = (c + 15) / 16;
  return cnt >= 16 ? 0xFFFFu : ((1u << cnt) - 1u);
}

// FP32 sum over the wave: the 16-lane DPP sum, then the four rows (a fixed
// pattern, so the result is reproducible).
__device__ inline float wave_sum_f(float v) {
  v = row16_sum(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Header check shared by the iteration kernels: the workspace must hold
// affinities for exactly this n.
// The workspace holds affinities for n points: ready is 1 when P is stored,
// 2 when P is recomputed in every pass (implicit P). Kernels that read the
// stored P accept only 1, those of the implicit pass only 2.
__device__ inline bool state_ok(Hdr *h, int64_t n) {
  return h->magic == kMagic && h->n == n && (h->ready == 1 || h->ready == 2);
}
__device__ inline bool ready_is(Hdr *h, int64_t n, int32_t ready) {
  return h->magic == kMagic && h->n == n && h->ready == ready;
}

// One row (k) of a thread's 16 x 16 block against its 16 columns.
template <bool DIAG, bool EDGE>
__device__ __forceinline__ float4 force_row(const float4 (&pv4)[4], float2 yi, const float2 yc[16],
                                            uint32_t rvalid, uint32_t cvalid, int k, int tr, int tc,
                                            float4 colacc[16], float &z) {
  float ax = 0.f, ay = 0.f, rx = 0.f, ry = 0.f;
#pragma unroll
  for (int mq = 0; mq < 4; ++mq) {
    const float pp[4] = {pv4[mq].x, pv4[mq].y, pv4[mq].z, pv4[mq].w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = 4 * mq + e;
      const float dx = yi.x - yc[m].x, dy = yi.y - yc[m].y;
      const float q = fmaf(dx, dx, fmaf(dy, dy, 1.0f));
      float w = __builtin_amdgcn_rcpf(q);
      if (DIAG) {
        if (tr == tc && k == m) w = 0.f;
      }
      if (EDGE) {
        if (!((rvalid >> k) & (cvalid >> m) & 1u)) w = 0.f;
      }
      z += w;
      const float pw = pp[e] * w, w2 = w * w;
      ax = fmaf(pw, dx, ax);
      ay = fmaf(pw, dy, ay);
      rx = fmaf(w2, dx, rx);
      ry = fmaf(w2, dy, ry);
      if (!DIAG) {
        colacc[m].x = fmaf(-pw, dx, colacc[m].x);
        colacc[m].y = fmaf(-pw, dy, colacc[m].y);
        colacc[m].z = fmaf(-w2, dx, colacc[m].z);
        colacc[m].w = fmaf(-w2, dy, colacc[m].w);
      }
    }
  }
  return make_float4(ax, ay, rx, ry);
}

// Totals of four rows' per-lane sums r0 .. r3 over the 16 lanes of a DPP
// row, one kept per lane: lane tc ends with the total of r(2 b3 + b2), b3 and
// b2 being bits 3 and 2 of tc.
// The additions are row16_sum's, in the same order: pairs of lanes at
// distance 8, then 4, 2 and 1 (after the first level every lane of a row
// holds a function of tc mod 8, so row16_sum's rotations by 4, 2 and 1 add
// the same operands as the exchanges used here), hence each total is bitwise
// row16_sum's. Choosing the kept quantity after the first two levels drops
// the additions every lane would repeat for totals it does not keep: 11
// instructions for four totals instead of 16.
__device__ __forceinline__ float row16_sum4(float r0, float r1, float r2, float r3, bool b3,
                                            bool b2) {
  // distance 8: a rotation by 8 inside the row exchanges its halves
  const float x0 = r0 + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(r0), 0x128, 0xf, 0xf, true));
  const float x1 = r1 + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(r1), 0x128, 0xf, 0xf, true));
  const float x2 = r2 + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(r2), 0x128, 0xf, 0xf, true));
  const float x3 = r3 + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(r3), 0x128, 0xf, 0xf, true));
  const float sa = b3 ? x2 : x0;  // r0 or r2
  const float sb = b3 ? x3 : x1;  // r1 or r3
  // distance 4: a lane with bit 2 clear reads lane + 4 (row shift left),
  // one with bit 2 set reads lane - 4 (row shift right); the lanes whose
  // shifted read leaves the row take the other operand
  const float ya = sa + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(sa), 0x104, 0xf, 0xf, true));
  const float yb = sb + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(sb), 0x114, 0xf, 0xf, true));
  float s = b2 ? yb : ya;
  // distances 2 and 1 inside each group of four lanes (quad permutations)
  s += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s), 0x4E, 0xf, 0xf, true));
  s += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s), 0xB1, 0xf, 0xf, true));
  return s;
}

// ---------------------------------------------------------------------------
// P streaming through LDS. Each wave owns a ring of kStages row slots in LDS;
// a slot holds the four float4 per lane that one row (k) of the thread's
// 16 x 16 block needs. Rows are fetched kStages - 1 ahead with
// global_load_lds_dwordx4 (global memory straight into LDS, no registers in
// flight) and the wave waits on its own vector-memory counter for the row it
// is about to use. The ring is read with ds_read_b128 inside an asm block
// that also waits for the read, so the compiler neither reorders it nor adds
// a blanket wait on all outstanding loads in front of it.
// ---------------------------------------------------------------------------
constexpr int kStages = 4;
typedef __attribute__((address_space(3))) void lds_void_t;

// s_waitcnt immediate that waits until at most n vector-memory operations are
// outstanding (expcnt and lgkmcnt left unconstrained).
constexpr int vmcnt_imm(int n) { return (n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8); }

__device__ __forceinline__ void fetch_row(const float4 *__restrict__ tp, int k, int t,
                                          float4 *ring_slot /* this wave's slot base */) {
#pragma unroll
  for (int mq = 0; mq < 4; ++mq)
    __builtin_amdgcn_global_load_lds((const void *)(tp + (k * 4 + mq) * 256 + t),
                                     (lds_void_t *)(ring_slot + mq * 64), 16, 0, 0);
}

// The four float4 of this lane in one ring slot (LDS byte address of the
// lane's first float4; the others follow at 1 KiB strides) and the position
// of the row (LDS byte address of a float2).
__device__ __forceinline__ void read_row(uint32_t p_addr, uint32_t y_addr, float4 (&v)[4],
                                         float2 &yi) {
  asm volatile(
      "ds_read_b128 %0, %5\n\t"
      "ds_read_b128 %1, %5 offset:1024\n\t"
      "ds_read_b128 %2, %5 offset:2048\n\t"
      "ds_read_b128 %3, %5 offset:3072\n\t"
      "ds_read_b64 %4, %6\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=v"(v[0]), "=v"(v[1]), "=v"(v[2]), "=v"(v[3]), "=v"(yi)
      : "v"(p_addr), "v"(y_addr)
      : "memory");
}

// ---------------------------------------------------------------------------
// Force pass: one workgroup per tile. Each wave streams its share of the
// tile's P through its LDS ring (rows fetched kStages - 1 ahead) and keeps the
// 16 column positions of its threads in registers.
//   row side    16-lane DPP sums, one row per thread, written to slot (I, J);
//   column side the 16 row groups' partial sums meet in LDS (the buffer
//               overlays the ring, which is idle by then), written to slot
//               (J, I);
//   Z           FP32 per thread, FP64 across the workgroup, one value per tile.
// ---------------------------------------------------------------------------

struct ForceSmem {
  union {
    float4 colbuf[16][T + 4];        // [row group tr][column], padded rows
    float2 colbuf2[16][T + 4];       // the same for the repulsive pair only
    float4 ring[4][kStages][4][64];  // [wave][slot][float4 of the row][lane]
  };
  float2 yrow[T];                    // positions of the tile's rows
  double zred[4];
};

template <bool DIAG, bool EDGE>
__device__ __forceinline__ void tile_rows(const float4 *__restrict__ tp, float4 *wring,
                                          uint32_t lane_addr, uint32_t yrow_addr,
                                          const float2 yc[16], uint32_t rvalid, uint32_t cvalid,
                                          int t, int tr, int tc, float4 &myrow, float4 colacc[16],
                                          float &z) {
#pragma unroll
  for (int r = 0; r < kStages - 1; ++r) fetch_row(tp, r, t, wring + r * 256);
#pragma unroll 1
  for (int k = 0; k < 16; ++k) {
    if (k + kStages - 1 < 16) {
      fetch_row(tp, k + kStages - 1, t, wring + ((k + kStages - 1) % kStages) * 256);
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(4 * (kStages - 1)));
    } else {
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    }
    float4 pv[4];
    float2 yi;
    read_row(lane_addr + (uint32_t)(k % kStages) * 4096u, yrow_addr + (uint32_t)(16 * k) * 8u, pv,
             yi);
    float4 r = force_row<DIAG, EDGE>(pv, yi, yc, rvalid, cvalid, k, tr, tc, colacc, z);
    r.x = row16_sum(r.x);
    r.y = row16_sum(r.y);
    r.z = row16_sum(r.z);
    r.w = row16_sum(r.w);
    if (tc == k) myrow = r;
  }
}

// Row of the thread's 16 x 16 block whose total the all-zero tile body keeps
// in lane tc: rows are summed four at a time (4 j .. 4 j + 3) and lane tc
// keeps row 4 j + (tc >> 2) of group j = tc & 3.
__device__ __forceinline__ int zero_row_of_lane(int tc) { return 4 * (tc & 3) + (tc >> 2); }

// A tile whose stored P is all zero: only the repulsive sums and Z, no P
// traffic. Row positions come from LDS (no ring is in use here). Rows are
// taken in order (so Z and the column sums accumulate as row by row), four
// per pass of the loop, and reduced over the lanes together.
template <bool DIAG, bool EDGE>
__device__ __forceinline__ void tile_rows_zero(const float2 *yrow, const float2 yc[16],
                                               uint32_t rvalid, uint32_t cvalid, int tr, int tc,
                                               float2 &myrow, float2 colrep[16], float &z) {
  const bool b3 = (tc & 8) != 0, b2 = (tc & 4) != 0;
#pragma unroll 1
  for (int j = 0; j < 4; ++j) {
    float rx[4], ry[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int k = 4 * j + g;
      const float2 yi = yrow[tr + 16 * k];
      rx[g] = 0.f;
      ry[g] = 0.f;
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const float dx = yi.x - yc[m].x, dy = yi.y - yc[m].y;
        const float q = fmaf(dx, dx, fmaf(dy, dy, 1.0f));
        float w = __builtin_amdgcn_rcpf(q);
        if (DIAG) {
          if (tr == tc && k == m) w = 0.f;
        }
        if (EDGE) {
          if (!((rvalid >> k) & (cvalid >> m) & 1u)) w = 0.f;
        }
        z += w;
        const float w2 = w * w;
        rx[g] = fmaf(w2, dx, rx[g]);
        ry[g] = fmaf(w2, dy, ry[g]);
        if (!DIAG) {
          colrep[m].x = fmaf(-w2, dx, colrep[m].x);
          colrep[m].y = fmaf(-w2, dy, colrep[m].y);
        }
      }
    }
    const float sx = row16_sum4(rx[0], rx[1], rx[2], rx[3], b3, b2);
    const float sy = row16_sum4(ry[0], ry[1], ry[2], ry[3], b3, b2);
    if ((tc & 3) == j) myrow = make_float2(sx, sy);
  }
}

// The map in the internal order, zero-padded to whole tiles (read by the
// force and cost passes, so that their loads are contiguous).
// Gathers the rows of block b into the internal order and writes the block's
// extent of the map, {min x, max x, min y, max y}, for the adaptive learning
// rate (exact: the order of min and max does not matter).
__device__ __forceinline__ void gather_rows(const float2 *__restrict__ Y,
                                            const int32_t *__restrict__ perm, int64_t n,
                                            float2 *__restrict__ Yp, float4 *__restrict__ extent,
                                            int64_t b) {
  __shared__ float4 red[T / 64];
  const int64_t r = b * T + threadIdx.x;
  const bool ok = r < n;
  const float2 v = ok ? Y[perm[r]] : make_float2(0.f, 0.f);
  Yp[r] = v;
  float lox = ok ? v.x : INFINITY, hix = ok ? v.x : -INFINITY;
  float loy = ok ? v.y : INFINITY, hiy = ok ? v.y : -INFINITY;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lox = fminf(lox, __shfl_xor(lox, o));
    hix = fmaxf(hix, __shfl_xor(hix, o));
    loy = fminf(loy, __shfl_xor(loy, o));
    hiy = fmaxf(hiy, __shfl_xor(hiy, o));
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_float4(lox, hix, loy, hiy);
  __syncthreads();
  if (threadIdx.x == 0) {
    float4 e = red[0];
#pragma unroll
    for (int w = 1; w < T / 64; ++w) {
      e.x = fminf(e.x, red[w].x);
      e.y = fmaxf(e.y, red[w].y);
      e.z = fminf(e.z, red[w].z);
      e.w = fmaxf(e.w, red[w].w);
    }
    extent[b] = e;
  }
}

__global__ __launch_bounds__(256) void k_gather_y(const float2 *__restrict__ Y,
                                                  const int32_t *__restrict__ perm, int64_t n,
                                                  float2 *__restrict__ Yp,
                                                  float4 *__restrict__ extent, Hdr *h) {
  if (!state_ok(h, n)) return;  // the layout of another n: touch nothing
  gather_rows(Y, perm, n, Yp, extent, blockIdx.x);
}

// LDS of the all-zero-tile kernel: no P ring, so four workgroups fit a CU.
constexpr int64_t kFullGrid = 512;  // persistent workgroups of the nonzero-tile kernel (at most)

struct ZeroSmem {
  float2 colbuf2[16][T + 4];
  float2 yrow[T];
  double zred[4];
};

// Set-up shared by both tile bodies: coordinates, valid-row masks, the
// column positions in registers and the row positions in LDS.
struct TileCtx {
  int I, J, t, w, l, tc, tr;
  uint32_t rvalid, cvalid;
  bool edge;
  size_t rslot, cslot;
};

template <class Smem>
__device__ __forceinline__ TileCtx tile_begin(const float2 *__restrict__ Y, int64_t n, int32_t nb,
                                              const int2 *__restrict__ tmap, int64_t tile,
                                              float2 (&yc)[16], Smem &sm) {
  TileCtx c;
  const int2 ij = tmap[tile];
  c.I = ij.x;
  c.J = ij.y;
  c.t = threadIdx.x;
  c.w = c.t >> 6;
  c.l = c.t & 63;
  c.tc = c.l & 15;
  c.tr = (c.l >> 4) + 4 * c.w;
  // Y is the zero-padded internal-order copy, so whole tiles load unguarded
  c.rvalid = valid_bits(n - (int64_t)c.I * T, c.tr);
  c.cvalid = valid_bits(n - (int64_t)c.J * T, c.tc);
#pragma unroll
  for (int k = 0; k < 16; ++k) yc[k] = Y[(int64_t)c.J * T + c.tc + 16 * k];
  sm.yrow[c.t] = Y[(int64_t)c.I * T + c.t];
  c.edge = ((int64_t)(c.J + 1) * T > n);
  c.rslot = ((size_t)c.I * nb + c.J) * T + c.tr + 16 * c.tc;  // row tr + 16 tc
  c.cslot = ((size_t)c.J * nb + c.I) * T + c.t;               // column t
  __syncthreads();
  return c;
}

// A tile whose stored P is all zero: repulsion and Z only, no P traffic,
// float2 accumulators. Ends with a workgroup barrier.
template <class Smem>
__device__ __forceinline__ void zero_tile_body(const TileCtx &c, const float2 (&yc)[16],
                                               float4 *__restrict__ part,
                                               float *__restrict__ zpart, int64_t tile,
                                               Smem &sm) {
  float2 *prep = part_rep(part);
  float z = 0.f;
  float2 myrow = make_float2(0.f, 0.f);
  float2 colrep[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) colrep[m] = make_float2(0.f, 0.f);
  if (c.I == c.J) {
    if (c.edge)
      tile_rows_zero<true, true>(sm.yrow, yc, c.rvalid, c.cvalid, c.tr, c.tc, myrow, colrep, z);
    else
      tile_rows_zero<true, false>(sm.yrow, yc, c.rvalid, c.cvalid, c.tr, c.tc, myrow, colrep, z);
  } else {
    if (c.edge)
      tile_rows_zero<false, true>(sm.yrow, yc, c.rvalid, c.cvalid, c.tr, c.tc, myrow, colrep, z);
    else
      tile_rows_zero<false, false>(sm.yrow, yc, c.rvalid, c.cvalid, c.tr, c.tc, myrow, colrep,
                                   z);
  }
  // this lane holds the total of row tr + 16 zero_row_of_lane(tc), not of
  // row tr + 16 tc as in c.rslot
  prep[(int64_t)c.rslot + 16 * (zero_row_of_lane(c.tc) - c.tc)] = myrow;
  // column side: the 16 row groups' sums meet in LDS
  if (c.I != c.J) {
#pragma unroll
    for (int m = 0; m < 16; ++m) sm.colbuf2[c.tr][c.tc + 16 * m] = colrep[m];
  }
  const double zd = (double)wave_sum_f(z);
  if (c.l == 0) sm.zred[c.w] = zd;
  __syncthreads();
  if (c.I != c.J) {
    float2 s2 = sm.colbuf2[0][c.t];
#pragma unroll
    for (int g = 1; g < 16; ++g) {
      const float2 v = sm.colbuf2[g][c.t];
      s2.x += v.x;
      s2.y += v.y;
    }
    prep[c.cslot] = s2;
  }
  if (c.t == 0)
    zpart[tile] =
        (float)((sm.zred[0] + sm.zred[1] + sm.zred[2] + sm.zred[3]) * (c.I == c.J ? 1.0 : 2.0));
}

// A tile with nonzero P: attraction and repulsion, P streamed through the
// per-wave LDS rings. Ends with a workgroup barrier.
__device__ __forceinline__ void full_tile_body(const TileCtx &c, const float2 (&yc)[16],
                                               const float4 *__restrict__ P,
                                               float4 *__restrict__ part, int32_t nb,
                                               float *__restrict__ zpart, int64_t tile,
                                               int64_t pslot, ForceSmem &sm) {
  float2 *prep = part_rep(part), *patt = part_att(part, nb);
  float z = 0.f;
  float4 *wring = &sm.ring[c.w][0][0][0];
  const uint32_t lane_addr = (uint32_t)(size_t)((lds_void_t *)wring) + (uint32_t)c.l * 16u;
  const uint32_t yrow_addr = (uint32_t)(size_t)((lds_void_t *)(sm.yrow + c.tr));
  const float4 *tp = P + (size_t)pslot * TT4;
  float4 myrow = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 colacc[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) colacc[m] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (c.I == c.J) {
    if (c.edge)
      tile_rows<true, true>(tp, wring, lane_addr, yrow_addr, yc, c.rvalid, c.cvalid, c.t, c.tr,
                            c.tc, myrow, colacc, z);
    else
      tile_rows<true, false>(tp, wring, lane_addr, yrow_addr, yc, c.rvalid, c.cvalid, c.t, c.tr,
                             c.tc, myrow, colacc, z);
  } else {
    if (c.edge)
      tile_rows<false, true>(tp, wring, lane_addr, yrow_addr, yc, c.rvalid, c.cvalid, c.t, c.tr,
                             c.tc, myrow, colacc, z);
    else
      tile_rows<false, false>(tp, wring, lane_addr, yrow_addr, yc, c.rvalid, c.cvalid, c.t,
                              c.tr, c.tc, myrow, colacc, z);
  }
  prep[c.rslot] = make_float2(myrow.z, myrow.w);
  patt[c.rslot] = make_float2(myrow.x, myrow.y);
  // column side: the 16 row groups' sums meet in LDS (colbuf overlays the P
  // ring, so every wave must be done with its ring first)
  __syncthreads();
  if (c.I != c.J) {
#pragma unroll
    for (int m = 0; m < 16; ++m) sm.colbuf[c.tr][c.tc + 16 * m] = colacc[m];
  }
  const double zd = (double)wave_sum_f(z);
  if (c.l == 0) sm.zred[c.w] = zd;
  __syncthreads();
  if (c.I != c.J) {
    float4 s4 = sm.colbuf[0][c.t];
#pragma unroll
    for (int g = 1; g < 16; ++g) {
      const float4 v = sm.colbuf[g][c.t];
      s4.x += v.x;
      s4.y += v.y;
      s4.z += v.z;
      s4.w += v.w;
    }
    prep[c.cslot] = make_float2(s4.z, s4.w);
    patt[c.cslot] = make_float2(s4.x, s4.y);
  }
  if (c.t == 0)
    zpart[tile] =
        (float)((sm.zred[0] + sm.zred[1] + sm.zred[2] + sm.zred[3]) * (c.I == c.J ? 1.0 : 2.0));
}

// Force kernels of a single problem, one per kind of tile, over the tile
// lists built after the pack (zero tiles in ascending order at the front of
// the list, then the nonzero tiles). They write disjoint slots and may run
// concurrently. The all-zero kernel runs one tile per workgroup (launched
// over every tile; workgroups past the count exit at once) with four
// workgroups per CU; the full kernel is persistent.
__global__ __launch_bounds__(256, 4) void k_force_zero(const float2 *__restrict__ Y, int64_t n,
                                                       int32_t nb, float4 *__restrict__ part,
                                                       float *__restrict__ zpart,
                                                       const int32_t *__restrict__ tlist,
                                                       const int32_t *__restrict__ tcount,
                                                       const int2 *__restrict__ tmap, Hdr *h,
                                                       int32_t ready) {
  __shared__ ZeroSmem sm;
  // the header check comes first: with a workspace for another n, the lists
  // are not where this layout puts them. ready: 1 stored P, 2 implicit P
  // (the lists and tile coordinates of its affinity stage; nothing here
  // depends on d or the distance mode)
  if (!ready_is(h, n, ready)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) flag_error(h, kErrState);
    return;
  }
  if ((int32_t)blockIdx.x >= tcount[0]) return;
  const int64_t tile = tlist[blockIdx.x];
  float2 yc[16];
  const TileCtx c = tile_begin(Y, n, nb, tmap, tile, yc, sm);
  zero_tile_body(c, yc, part, zpart, tile, sm);
}

__global__ __launch_bounds__(256, 2) void k_force_full(const float4 *__restrict__ P,
                                                       const float2 *__restrict__ Y, int64_t n,
                                                       int32_t nb, float4 *__restrict__ part,
                                                       float *__restrict__ zpart,
                                                       const int32_t *__restrict__ tlist,
                                                       const int32_t *__restrict__ tcount,
                                                       const int2 *__restrict__ tmap, Hdr *h) {
  __shared__ ForceSmem sm;
  if (!ready_is(h, n, 1)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) flag_error(h, kErrState);
    return;
  }
  const int32_t count = tcount[1], first = tcount[0];
  // one workgroup per CU leaves room for the all-zero kernel beside it; when
  // most tiles hold P, two per CU keep enough of P in flight
  const int32_t active = (int32_t)min((int64_t)gridDim.x, count > first ? kFullGrid : kFullGrid / 2);
  if ((int32_t)blockIdx.x >= active) return;
  for (int32_t i = blockIdx.x; i < count; i += active) {
    const int64_t tile = tlist[first + i];
    float2 yc[16];
    const TileCtx c = tile_begin(Y, n, nb, tmap, tile, yc, sm);
    full_tile_body(c, yc, P, part, nb, zpart, tile, tile, sm);
  }
}

// Implicit P: the nonzero tiles among tile0 .. tile0 + gridDim.x - 1 (whole
// block rows), whose P was just recomputed into the buffer Pb (tile
// tile0 + x at slot x); the all-zero ones are k_force_zero's.
__global__ __launch_bounds__(256, 2) void k_force_range(const float4 *__restrict__ Pb,
                                                        const float2 *__restrict__ Y, int64_t n,
                                                        int32_t nb, float4 *__restrict__ part,
                                                        float *__restrict__ zpart,
                                                        const int2 *__restrict__ tmap,
                                                        const uint8_t *__restrict__ nz,
                                                        int64_t tile0, int32_t key, Hdr *h) {
  __shared__ ForceSmem sm;
  if (!ready_is(h, n, 2) || implicit_key(h->d, h->mode) != key) {
    if (blockIdx.x == 0 && threadIdx.x == 0) flag_error(h, kErrState);
    return;
  }
  const int64_t tile = tile0 + blockIdx.x;
  if (!nz[tile]) return;
  float2 yc[16];
  const TileCtx c = tile_begin(Y, n, nb, tmap, tile, yc, sm);
  full_tile_body(c, yc, Pb, part, nb, zpart, tile, blockIdx.x, sm);
}

// ----------------------------------------------------------------------------
// Reduce + update. kUpdPerBlock workgroups of kUpd threads per block of T
// rows; thread (r, q) of a workgroup sums the slots s = q, q + kUpdSplit, ...
// of its row r in order, and the kUpdSplit partial sums meet in LDS in q
// order (a fixed order). Every workgroup also forms Z from the tile partials
// in the same fixed order (so all of them hold the same value) instead of a
// separate launch; workgroup 0 stores it.
// ----------------------------------------------------------------------------
constexpr int kUpd = 1024;
constexpr int kUpdRows = 128;                 // rows per workgroup
constexpr int kUpdPerBlock = T / kUpdRows;    // workgroups per row block
static_assert(kUpdPerBlock == kMeanPartsPerBlock, "one re-centring partial per update workgroup");
constexpr int kUpdSplit = kUpd / kUpdRows;    // threads per row
constexpr int kSlotLds = 4096;                // nonzero-slot list entries staged in LDS
constexpr int kUpdBatch = 8;                  // repulsive-slot loads in flight per thread

struct UpdSmem {
  double4 part[kUpdSplit - 1][kUpdRows];
  double red[2][kUpd / 64];
  double z;
  float eta;
  int32_t slots[kSlotLds];
};

// Z = sum of the tile partials (FP32 per tile, FP64 sums): four strided
// sums per thread (loads in flight), the wave sums, then the 16 wave results
// in order.
__device__ inline double z_total(const float *__restrict__ zpart, int64_t nt, UpdSmem &sm) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t q = threadIdx.x;
  for (; q + 7 * kUpd < nt; q += 8 * kUpd) {  // two rounds of four, loads first
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = zpart[q + u * kUpd];
    s0 += v[0];
    s1 += v[1];
    s2 += v[2];
    s3 += v[3];
    s0 += v[4];
    s1 += v[5];
    s2 += v[6];
    s3 += v[7];
  }
  for (; q + 3 * kUpd < nt; q += 4 * kUpd) {
    s0 += zpart[q];
    s1 += zpart[q + kUpd];
    s2 += zpart[q + 2 * kUpd];
    s3 += zpart[q + 3 * kUpd];
  }
  for (; q < nt; q += kUpd) s0 += zpart[q];
  double s = wave_sum_d((s0 + s1) + (s2 + s3));
  if ((threadIdx.x & 63) == 0) sm.red[0][threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double Z = 0.0;
    for (int w = 0; w < kUpd / 64; ++w) Z += sm.red[0][w];
    sm.z = Z;
  }
  __syncthreads();
  return sm.z;
}

// Row sums (A_x, A_y, R_x, R_y) of row r (0 .. T-1) of block b from its nb
// slots; every thread of the workgroup must call it, the result is valid for
// q == 0.
__device__ inline double4 row_sums(const float4 *__restrict__ part,
                                   const int32_t *__restrict__ slots,
                                   const int32_t *__restrict__ nslots, int32_t nb, int b, int r,
                                   int q, UpdSmem &sm) {
  // the block's list of slots with nonzero P (attractive sums exist only
  // there); count and entries are clamped to the block's nb slots, so a list
  // that was never built cannot send the reads outside the partial sums
  const int cnt = min(max(nslots[b], 0), (int)nb);
  const int32_t *gl = slots + (int64_t)b * nb;
  for (int m = threadIdx.x; m < cnt && m < kSlotLds; m += kUpd) sm.slots[m] = gl[m];
  __syncthreads();
  double ax = 0.0, ay = 0.0, rx = 0.0, ry = 0.0;
  const float2 *pr = part_rep(part) + (size_t)b * nb * T + r;
  const float2 *pa = part_att(part, nb) + (size_t)b * nb * T + r;
  // batches of kUpdBatch slots: all loads of a batch are issued before the
  // first add, and the adds keep ascending slot order
  int s = q;
  for (; s + (kUpdBatch - 1) * kUpdSplit < nb; s += kUpdBatch * kUpdSplit) {
    float2 v[kUpdBatch];
#pragma unroll
    for (int u = 0; u < kUpdBatch; ++u) v[u] = pr[(size_t)(s + u * kUpdSplit) * T];
#pragma unroll
    for (int u = 0; u < kUpdBatch; ++u) {
      rx += v[u].x;
      ry += v[u].y;
    }
  }
  for (; s < nb; s += kUpdSplit) {
    const float2 v = pr[(size_t)s * T];
    rx += v.x;
    ry += v.y;
  }
  int m = q;
  for (; m + 3 * kUpdSplit < cnt; m += 4 * kUpdSplit) {
    float2 a[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int mu = m + u * kUpdSplit;
      const int su = mu < kSlotLds ? sm.slots[mu] : gl[mu];
      ok[u] = su >= 0 && su < nb;
      a[u] = ok[u] ? pa[(size_t)su * T] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (ok[u]) {
        ax += a[u].x;
        ay += a[u].y;
      }
    }
  }
  for (; m < cnt; m += kUpdSplit) {
    const int su = m < kSlotLds ? sm.slots[m] : gl[m];
    if (su < 0 || su >= nb) continue;
    const float2 a = pa[(size_t)su * T];
    ax += a.x;
    ay += a.y;
  }
  const int rl = r % kUpdRows;
  if (q > 0) sm.part[q - 1][rl] = make_double4(ax, ay, rx, ry);
  __syncthreads();
  if (q == 0) {
#pragma unroll
    for (int g = 0; g < kUpdSplit - 1; ++g) {
      const double4 v = sm.part[g][rl];
      ax += v.x;
      ay += v.y;
      rx += v.z;
      ry += v.w;
    }
  }
  return make_double4(ax, ay, rx, ry);
}

// The paper's learning rate (Eq. 11): eta = ln(n - 1) (Y_max - Y_min) / 2,
// with Y_max - Y_min the larger of the two coordinate ranges of the map the
// gradient is taken at (the extents its gather wrote per block). One wave
// reduces the block extents; the result is published by the next barrier.
__device__ inline void adaptive_eta(const float4 *__restrict__ extent, int32_t nb, int64_t n,
                                    UpdSmem &sm) {
  if (threadIdx.x >= 64) return;
  float lox = INFINITY, hix = -INFINITY, loy = INFINITY, hiy = -INFINITY;
  for (int b = threadIdx.x; b < nb; b += 64) {
    const float4 e = extent[b];
    lox = fminf(lox, e.x);
    hix = fmaxf(hix, e.y);
    loy = fminf(loy, e.z);
    hiy = fmaxf(hiy, e.w);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lox = fminf(lox, __shfl_xor(lox, o));
    hix = fmaxf(hix, __shfl_xor(hix, o));
    loy = fminf(loy, __shfl_xor(loy, o));
    hiy = fmaxf(hiy, __shfl_xor(hiy, o));
  }
  if (threadIdx.x == 0) {
    const double range = fmax((double)hix - (double)lox, (double)hiy - (double)loy);
    sm.eta = (float)(log((double)(n - 1)) * range * 0.5);
  }
}

// g = 4 (alpha A - R / Z)
__device__ inline float2 gradient_of(double4 s, double alpha, double Z) {
  return make_float2((float)(4.0 * (alpha * s.x - s.z / Z)), (float)(4.0 * (alpha * s.y - s.w / Z)));
}

// Update (Eq. 10, descent): gains, momentum, position; per-workgroup sums of
// the new positions for the re-centring. Workgroup wg of the problem covers
// rows (wg % kUpdPerBlock) * kUpdRows ... of block wg / kUpdPerBlock.
// lr_rule 0: the given eta with adaptive gains; lr_rule 1: eta of Eq. 11 and
// no gains (G is neither read nor written).
__device__ __forceinline__ void update_wg(const float4 *__restrict__ part,
                                          const int32_t *__restrict__ slots,
                                          const int32_t *__restrict__ nslots,
                                          const float *__restrict__ zpart, int64_t nt,
                                          int64_t n, int32_t nb, const int32_t *__restrict__ perm,
                                          float2 *__restrict__ Y, float2 *__restrict__ U,
                                          float2 *__restrict__ G, float alpha, float mu, float eta,
                                          float min_gain, int lr_rule,
                                          const float4 *__restrict__ extent,
                                          float2 *__restrict__ grad_out,
                                          double *__restrict__ z_out,
                                          double2 *__restrict__ meanpart, Hdr *h, int wg,
                                          UpdSmem &sm) {
  if (!state_ok(h, n)) return;
  if (lr_rule) adaptive_eta(extent, nb, n, sm);
  const int b = wg / kUpdPerBlock;
  const int t = threadIdx.x, q = t / kUpdRows;
  const int r = (wg % kUpdPerBlock) * kUpdRows + t % kUpdRows;  // row within the block
  const int64_t ir = (int64_t)b * T + r;                         // internal position
  // odd workgroups sum their rows before Z, even ones after, so that the
  // HBM-bound row sums of one half overlap the cached Z reads of the other
  // (both results are the same in either order); the barriers of either
  // also publish sm.eta
  double Z;
  double4 rs;
  if (wg & 1) {
    rs = row_sums(part, slots, nslots, nb, b, r, q, sm);
    Z = z_total(zpart, nt, sm);
  } else {
    Z = z_total(zpart, nt, sm);
    rs = row_sums(part, slots, nslots, nb, b, r, q, sm);
  }
  if (lr_rule) eta = sm.eta;
  if (wg == 0 && t == 0) {
    h->z = Z;
    if (z_out) *z_out = Z;
    if (!isfinite(Z) || !(Z > 0.0)) flag_error(h, kErrNonFinite);
  }
  const float2 g = gradient_of(rs, (double)alpha, Z);
  double sx = 0.0, sy = 0.0;
  bool bad = false;
  if (q == 0 && ir < n) {
    const int64_t i = perm[ir];
    if (grad_out) grad_out[i] = g;
    float2 u = U[i], y = Y[i];
    if (lr_rule) {
      u.x = mu * u.x - eta * g.x;
      u.y = mu * u.y - eta * g.y;
    } else {
      float2 gn = G[i];
      gn.x = ((g.x > 0.f) != (u.x > 0.f)) ? gn.x + 0.2f : gn.x * 0.8f;
      gn.y = ((g.y > 0.f) != (u.y > 0.f)) ? gn.y + 0.2f : gn.y * 0.8f;
      gn.x = fmaxf(gn.x, min_gain);
      gn.y = fmaxf(gn.y, min_gain);
      u.x = mu * u.x - eta * (gn.x * g.x);
      u.y = mu * u.y - eta * (gn.y * g.y);
      G[i] = gn;
    }
    y.x += u.x;
    y.y += u.y;
    U[i] = u;
    Y[i] = y;
    sx = y.x;
    sy = y.y;
    bad = !(isfinite(g.x) && isfinite(g.y) && isfinite(y.x) && isfinite(y.y));
  }
  if (bad) flag_error(h, kErrNonFinite);
  sx = wave_sum_d(sx);
  sy = wave_sum_d(sy);
  if ((t & 63) == 0) {
    sm.red[0][t >> 6] = sx;
    sm.red[1][t >> 6] = sy;
  }
  __syncthreads();
  if (t == 0) {  // the waves of q == 0 hold the rows
    double mx = 0.0, my = 0.0;
    for (int w = 0; w < kUpdRows / 64; ++w) {
      mx += sm.red[0][w];
      my += sm.red[1][w];
    }
    meanpart[wg] = make_double2(mx, my);
  }
}

__global__ __launch_bounds__(kUpd) void k_update(
    const float4 *__restrict__ part, const int32_t *__restrict__ slots,
    const int32_t *__restrict__ nslots, const float *__restrict__ zpart, int64_t nt, int64_t n,
    int32_t nb, const int32_t *__restrict__ perm, float2 *__restrict__ Y, float2 *__restrict__ U,
    float2 *__restrict__ G, float alpha, float mu, float eta, float min_gain, int lr_rule,
    const float4 *__restrict__ extent, float2 *__restrict__ grad_out, double *__restrict__ z_out,
    double2 *__restrict__ meanpart, Hdr *h) {
  __shared__ UpdSmem sm;
  update_wg(part, slots, nslots, zpart, nt, n, nb, perm, Y, U, G, alpha, mu, eta, min_gain,
            lr_rule, extent, grad_out, z_out, meanpart, h, blockIdx.x, sm);
}

// Subtract the mean of the map from the rows of block `blk`.
__device__ __forceinline__ void recentre_wg(const double2 *__restrict__ meanpart, int64_t n,
                                            int32_t nb, float2 *__restrict__ Y, Hdr *h, int blk,
                                            float2 &smean) {
  __shared__ double2 wred[4];
  if (!state_ok(h, n)) return;
  // strided partial sums over the 256 threads, the wave sums, then the four
  // wave results in order (a fixed order)
  double mx = 0.0, my = 0.0;
  for (int b = threadIdx.x; b < nb * kUpdPerBlock; b += 256) {
    mx += meanpart[b].x;
    my += meanpart[b].y;
  }
  mx = wave_sum_d(mx);
  my = wave_sum_d(my);
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = make_double2(mx, my);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double sx = (wred[0].x + wred[1].x) + (wred[2].x + wred[3].x);
    const double sy = (wred[0].y + wred[1].y) + (wred[2].y + wred[3].y);
    smean = make_float2((float)(sx / (double)n), (float)(sy / (double)n));
  }
  __syncthreads();
  const int64_t i = (int64_t)blk * 256 + threadIdx.x;
  if (i < n) {
    float2 y = Y[i];
    y.x -= smean.x;
    y.y -= smean.y;
    Y[i] = y;
  }
}

__global__ __launch_bounds__(256) void k_recentre(const double2 *__restrict__ meanpart, int64_t n,
                                                  int32_t nb, float2 *__restrict__ Y, Hdr *h) {
  __shared__ float2 smean;
  recentre_wg(meanpart, n, nb, Y, h, blockIdx.x, smean);
}

// ----------------------------------------------------------------------------
// Batched iteration: many independent problems (each with its own workspace
// and map) in one launch per phase. A device table lists the problems in
// order with prefix sums of their tile and row-block counts; workgroup w
// finds its problem by binary search and runs the single-problem code on it
// (the nonzero-tile kernel is persistent and walks the problems' lists in
// turn), so every problem's result is bitwise the same as a separate launch.
// ----------------------------------------------------------------------------
__device__ inline int find_entry(const BatchEntry *tab, int count, int64_t key, bool by_tile) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t start = by_tile ? tab[mid].tile0 : tab[mid].blk0;
    if (start <= key)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// The launch must match the plan held in the batch workspace.
__device__ inline bool batch_ok(const BatchHdr *bh, int count, int64_t tiles, int64_t blocks) {
  return bh->magic == kBatchMagic && bh->count == count && bh->total_tiles == tiles &&
         bh->total_blocks == blocks;
}

__device__ inline const BatchEntry *batch_table(const BatchHdr *bh) {
  return reinterpret_cast<const BatchEntry *>(reinterpret_cast<const char *>(bh) +
                                              kBatchHdrBytes);
}

// All-zero tiles of the batch: launched over every tile of every problem
// (the problem found by binary search on its first tile); a workgroup whose
// position within its problem is past the count of all-zero tiles exits at
// once.
__global__ __launch_bounds__(256, 4) void k_force_zero_batched(const BatchHdr *__restrict__ bh,
                                                               int count, int64_t tiles,
                                                               int64_t blocks) {
  __shared__ ZeroSmem sm;
  if (!batch_ok(bh, count, tiles, blocks)) return;
  const BatchEntry *tab = batch_table(bh);
  const int p = find_entry(tab, count, blockIdx.x, true);
  const BatchEntry &e = tab[p];
  const int64_t i = (int64_t)blockIdx.x - e.tile0;
  if (i < 0 || i >= e.nt) return;
  if (!ready_is(e.h, e.n, 1)) {
    if (i == 0 && threadIdx.x == 0) flag_error(e.h, kErrState);
    return;
  }
  if (i >= e.tcount[0]) return;
  const int64_t tile = e.tlist[i];
  float2 yc[16];
  const TileCtx c = tile_begin(e.yp, e.n, e.nb, e.tmap, tile, yc, sm);
  zero_tile_body(c, yc, e.part, e.zpart, tile, sm);
}

// The nonzero tiles of every problem form one list (problem by problem, each
// in the order of its own list), dealt round-robin to a persistent grid as in
// the single-problem kernel: position g of the list goes to workgroup
// g % active. A problem whose workspace is not ready is skipped here (the
// all-zero kernel flags it). Counts are clamped to the problem's tile list.
__device__ inline void full_range(const BatchEntry &e, int64_t &first, int64_t &cnt) {
  first = min(max((int64_t)e.tcount[0], (int64_t)0), e.nt);
  cnt = min(max((int64_t)e.tcount[1], (int64_t)0), e.nt - first);
}

// Problems whose list offsets a workgroup of the nonzero-tile kernel keeps in
// LDS (larger batches walk the table serially).
constexpr int kBatchLds = 1024;

__global__ __launch_bounds__(256, 2) void k_force_full_batched(const BatchHdr *__restrict__ bh,
                                                               int count, int64_t tiles,
                                                               int64_t blocks) {
  __shared__ ForceSmem sm;
  __shared__ int64_t pre[kBatchLds + 1];  // list position of problem p's first nonzero tile
  __shared__ int64_t nzero_s;
  if (!batch_ok(bh, count, tiles, blocks)) return;
  const BatchEntry *tab = batch_table(bh);
  const int t = threadIdx.x;
  if (count <= kBatchLds) {
    // one wave: lane l sums the nonzero and all-zero counts of problems
    // 16 l .. 16 l + 15 (loads in flight together), then an inclusive scan
    // over the lanes gives every problem's offset
    if (t < 64) {
      constexpr int kPer = kBatchLds / 64;
      int64_t c[kPer], zs = 0, run = 0;
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int p = kPer * t + u;
        c[u] = 0;
        if (p < count) {
          const BatchEntry &e = tab[p];
          if (ready_is(e.h, e.n, 1)) {
            int64_t first, cnt;
            full_range(e, first, cnt);
            c[u] = cnt;
            zs += first;
          }
        }
        run += c[u];
      }
      int64_t inc = run;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int64_t v = __shfl_up(inc, o, 64);
        if (t >= o) inc += v;
      }
      int64_t off = inc - run;  // exclusive prefix of this lane's problems
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int p = kPer * t + u;
        if (p < count) pre[p] = off;
        off += c[u];
      }
      if (t == 63) pre[count] = inc;
      for (int o = 32; o > 0; o >>= 1) zs += __shfl_xor(zs, o, 64);
      if (t == 0) nzero_s = zs;
    }
    __syncthreads();
    const int64_t nfull = pre[count], nzero = nzero_s;
    // one workgroup per CU beside the all-zero kernel; two when most tiles
    // hold P
    const int64_t active = min((int64_t)gridDim.x, nfull > nzero ? kFullGrid : kFullGrid / 2);
    if ((int64_t)blockIdx.x >= active) return;
    for (int64_t g = blockIdx.x; g < nfull; g += active) {
      int lo = 0, hi = count - 1;  // last problem with pre[p] <= g
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= g)
          lo = mid;
        else
          hi = mid - 1;
      }
      const BatchEntry &e = tab[lo];
      int64_t first, cnt;
      full_range(e, first, cnt);
      const int64_t i = g - pre[lo];
      if (i >= cnt) continue;  // not reached: pre counts exactly cnt positions
      const int64_t tile = e.tlist[first + i];
      float2 yc[16];
      const TileCtx c = tile_begin(e.yp, e.n, e.nb, e.tmap, tile, yc, sm);
      full_tile_body(c, yc, e.P, e.part, e.nb, e.zpart, tile, tile, sm);
    }
    return;
  }
  int64_t nfull = 0, nzero = 0;
  for (int p = 0; p < count; ++p) {
    const BatchEntry &e = tab[p];
    if (!ready_is(e.h, e.n, 1)) continue;
    int64_t first, cnt;
    full_range(e, first, cnt);
    nzero += first;
    nfull += cnt;
  }
  const int64_t active = min((int64_t)gridDim.x, nfull > nzero ? kFullGrid : kFullGrid / 2);
  if ((int64_t)blockIdx.x >= active) return;
  int64_t base = 0;  // list position of the problem's first nonzero tile
  for (int p = 0; p < count; ++p) {
    const BatchEntry &e = tab[p];
    if (!ready_is(e.h, e.n, 1)) continue;
    int64_t first, cnt;
    full_range(e, first, cnt);
    int64_t i = ((int64_t)blockIdx.x - base) % active;
    if (i < 0) i += active;
    for (; i < cnt; i += active) {
      const int64_t tile = e.tlist[first + i];
      float2 yc[16];
      const TileCtx c = tile_begin(e.yp, e.n, e.nb, e.tmap, tile, yc, sm);
      full_tile_body(c, yc, e.P, e.part, e.nb, e.zpart, tile, tile, sm);
    }
    base += cnt;
  }
}

__global__ __launch_bounds__(256) void k_gather_batched(const BatchHdr *__restrict__ bh,
                                                        int count, int64_t tiles,
                                                        int64_t blocks) {
  if (!batch_ok(bh, count, tiles, blocks)) return;
  const BatchEntry *tab = batch_table(bh);
  const int p = find_entry(tab, count, blockIdx.x, false);
  const BatchEntry &e = tab[p];
  const int64_t b = (int64_t)blockIdx.x - e.blk0;
  if (b < 0 || b >= e.nb) return;
  if (!state_ok(e.h, e.n)) return;
  gather_rows(e.Y, e.perm, e.n, e.yp, e.extent, b);
}

__global__ __launch_bounds__(kUpd) void k_update_batched(const BatchHdr *__restrict__ bh,
                                                        int count, int64_t tiles, int64_t blocks,
                                                        float alpha, float mu, float eta,
                                                        float min_gain, int lr_rule) {
  __shared__ UpdSmem sm;
  if (!batch_ok(bh, count, tiles, blocks)) return;
  const BatchEntry *tab = batch_table(bh);
  const int64_t gb = (int64_t)blockIdx.x / kUpdPerBlock;  // global row block
  const int p = find_entry(tab, count, gb, false);
  const BatchEntry &e = tab[p];
  const int64_t b = gb - e.blk0;
  if (b < 0 || b >= e.nb) return;
  update_wg(e.part, e.slots, e.nslots, e.zpart, e.nt, e.n, e.nb, e.perm, e.Y, e.U, e.G, alpha, mu,
            eta, min_gain, lr_rule, e.extent, nullptr, nullptr, e.meanpart, e.h,
            (int)(b * kUpdPerBlock + blockIdx.x % kUpdPerBlock), sm);
}

__global__ __launch_bounds__(256) void k_recentre_batched(const BatchHdr *__restrict__ bh,
                                                          int count, int64_t tiles,
                                                          int64_t blocks) {
  __shared__ float2 smean;
  if (!batch_ok(bh, count, tiles, blocks)) return;
  const BatchEntry *tab = batch_table(bh);
  const int p = find_entry(tab, count, blockIdx.x, false);
  const BatchEntry &e = tab[p];
  const int64_t b = (int64_t)blockIdx.x - e.blk0;
  if (b < 0 || b >= e.nb) return;
  recentre_wg(e.meanpart, e.n, e.nb, e.Y, e.h, (int)b, smean);
}

__global__ __launch_bounds__(kUpd) void k_grad_only(
    const float4 *__restrict__ part, const int32_t *__restrict__ slots,
    const int32_t *__restrict__ nslots, const float *__restrict__ zpart, int64_t nt, int64_t n,
    int32_t nb, const int32_t *__restrict__ perm, float alpha, float2 *__restrict__ grad_out,
    double *__restrict__ z_out, Hdr *h) {
  __shared__ UpdSmem sm;
  if (!state_ok(h, n)) return;
  const int wg = blockIdx.x, b = wg / kUpdPerBlock, t = threadIdx.x, q = t / kUpdRows;
  const int r = (wg % kUpdPerBlock) * kUpdRows + t % kUpdRows;
  const int64_t ir = (int64_t)b * T + r;
  const double Z = z_total(zpart, nt, sm);
  if (wg == 0 && t == 0) {
    h->z = Z;
    if (z_out) *z_out = Z;
    if (!isfinite(Z) || !(Z > 0.0)) flag_error(h, kErrNonFinite);
  }
  const float2 g = gradient_of(row_sums(part, slots, nslots, nb, b, r, q, sm), (double)alpha, Z);
  if (q == 0 && ir < n) {
    grad_out[perm[ir]] = g;
    if (!(isfinite(g.x) && isfinite(g.y))) flag_error(h, kErrNonFinite);
  }
}

// ----------------------------------------------------------------------------
// Cost: per tile sum p log2(1 + |d|^2) and Z, then
//   KL = C_P + ln2 sum p log2(1 + |d|^2) + (sum p) ln Z,
//   C_norm = (ln2 sum p log2(1 + |d|^2) + (sum p) ln Z) / (ln n + ln(n - 1)).
// ----------------------------------------------------------------------------
template <bool DIAG, bool EDGE>
__device__ __forceinline__ void cost_tile(const float4 *__restrict__ tp,
                                          const float2 *__restrict__ yrow, const float2 yc[16],
                                          uint32_t rvalid, uint32_t cvalid, int t, int tr, int tc,
                                          float &plq, float &z) {
#pragma unroll 1
  for (int k = 0; k < 16; ++k) {
    const float2 yi = ((rvalid >> k) & 1u) ? yrow[16 * k] : make_float2(0.f, 0.f);
#pragma unroll
    for (int mq = 0; mq < 4; ++mq) {
      const float4 pv = tp[(k * 4 + mq) * 256 + t];
      const float pp[4] = {pv.x, pv.y, pv.z, pv.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = 4 * mq + e;
        const float dx = yi.x - yc[m].x, dy = yi.y - yc[m].y;
        const float q = fmaf(dx, dx, fmaf(dy, dy, 1.0f));
        float w = __builtin_amdgcn_rcpf(q);
        bool keep = true;
        if (DIAG) keep = !(tr == tc && k == m);
        if (EDGE) keep = keep && ((rvalid >> k) & (cvalid >> m) & 1u);
        if (!keep) w = 0.f;
        z += w;
        plq = fmaf(pp[e], __builtin_amdgcn_logf(q), plq);
      }
    }
  }
}

__device__ __forceinline__ void cost_wg(const float4 *__restrict__ P,
                                        const float2 *__restrict__ Y, int64_t n, int32_t nb,
                                        double2 *__restrict__ cpart,
                                        const uint8_t *__restrict__ nz, Hdr *h, int64_t tile,
                                        int64_t pslot, int32_t ready) {
  __shared__ double red[2][4];
  if (!ready_is(h, n, ready)) {
    if (tile == 0 && threadIdx.x == 0) flag_error(h, kErrState);
    return;
  }
  int I, J;
  tile_coords(tile, nb, I, J);
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int tc = l & 15, tr = (l >> 4) + 4 * w;
  const uint32_t rvalid = valid_bits(n - (int64_t)I * T, tr);
  const uint32_t cvalid = valid_bits(n - (int64_t)J * T, tc);
  float2 yc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) yc[k] = Y[(int64_t)J * T + tc + 16 * k];
  const float2 *yrow = Y + (int64_t)I * T + tr;
  const bool edge = ((int64_t)(J + 1) * T > n);
  const float4 *tp = P + (size_t)pslot * TT4;
  float plq = 0.f, z = 0.f;
  if (!nz[tile]) {
    // no p_ij in this tile: only Z
#pragma unroll 1
    for (int k = 0; k < 16; ++k) {
      const float2 yi = ((rvalid >> k) & 1u) ? yrow[16 * k] : make_float2(0.f, 0.f);
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const float dx = yi.x - yc[m].x, dy = yi.y - yc[m].y;
        float w = __builtin_amdgcn_rcpf(fmaf(dx, dx, fmaf(dy, dy, 1.0f)));
        bool keep = (I != J) || !(tr == tc && k == m);
        keep = keep && ((rvalid >> k) & (cvalid >> m) & 1u);
        z += keep ? w : 0.f;
      }
    }
  } else if (I == J) {
    if (edge)
      cost_tile<true, true>(tp, yrow, yc, rvalid, cvalid, t, tr, tc, plq, z);
    else
      cost_tile<true, false>(tp, yrow, yc, rvalid, cvalid, t, tr, tc, plq, z);
  } else {
    if (edge)
      cost_tile<false, true>(tp, yrow, yc, rvalid, cvalid, t, tr, tc, plq, z);
    else
      cost_tile<false, false>(tp, yrow, yc, rvalid, cvalid, t, tr, tc, plq, z);
  }
  double a = wave_sum_d((double)plq), c = wave_sum_d((double)z);
  if (l == 0) {
    red[0][w] = a;
    red[1][w] = c;
  }
  __syncthreads();
  if (t == 0) {
    const double mult = (I == J) ? 1.0 : 2.0;
    cpart[tile] = make_double2(mult * (red[0][0] + red[0][1] + red[0][2] + red[0][3]),
                                     mult * (red[1][0] + red[1][1] + red[1][2] + red[1][3]));
  }
}

__global__ __launch_bounds__(256, 2) void k_cost(const float4 *__restrict__ P,
                                                 const float2 *__restrict__ Y, int64_t n,
                                                 int32_t nb, double2 *__restrict__ cpart,
                                                 const uint8_t *__restrict__ nz, Hdr *h) {
  cost_wg(P, Y, n, nb, cpart, nz, h, blockIdx.x, blockIdx.x, 1);
}

// Implicit P: the cost terms of the tiles in the buffer (see k_force_range).
__global__ __launch_bounds__(256, 2) void k_cost_range(const float4 *__restrict__ Pb,
                                                       const float2 *__restrict__ Y, int64_t n,
                                                       int32_t nb, double2 *__restrict__ cpart,
                                                       const uint8_t *__restrict__ nz, Hdr *h,
                                                       int64_t tile0) {
  cost_wg(Pb, Y, n, nb, cpart, nz, h, tile0 + blockIdx.x, blockIdx.x, 2);
}

__device__ __forceinline__ void cost_reduce_wg(const double2 *__restrict__ cpart, int64_t nt,
                                               int64_t n, Hdr *h, double *out) {
  __shared__ double red[2][16];
  if (!state_ok(h, n)) return;
  double a = 0.0, c = 0.0;
  for (int64_t q = threadIdx.x; q < nt; q += 1024) {
    a += cpart[q].x;
    c += cpart[q].y;
  }
  a = wave_sum_d(a);
  c = wave_sum_d(c);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double A = 0.0, Z = 0.0;
    for (int q = 0; q < 16; ++q) {
      A += red[0][q];
      Z += red[1][q];
    }
    const double cross = kLn2 * A + h->p_sum * log(Z);  // H(P, Q)
    out[0] = h->c_p + cross;
    out[1] = cross / (log((double)n) + log((double)n - 1.0));
    if (!isfinite(out[0])) flag_error(h, kErrNonFinite);
  }
}

__global__ __launch_bounds__(1024) void k_cost_reduce(const double2 *__restrict__ cpart,
                                                      int64_t nt, int64_t n, Hdr *h,
                                                      double *out) {
  cost_reduce_wg(cpart, nt, n, h, out);
}

// Cost of every problem of a batch: one workgroup per tile, then one per
// problem (out: device double[2 count], {KL, C_norm} per problem).
__global__ __launch_bounds__(256, 2) void k_cost_batched(const BatchHdr *__restrict__ bh,
                                                         int count, int64_t tiles,
                                                         int64_t blocks) {
  if (!batch_ok(bh, count, tiles, blocks)) return;
  const BatchEntry *tab = batch_table(bh);
  const int p = find_entry(tab, count, blockIdx.x, true);
  const BatchEntry &e = tab[p];
  const int64_t i = (int64_t)blockIdx.x - e.tile0;
  if (i < 0 || i >= e.nt) return;
  cost_wg(e.P, e.yp, e.n, e.nb, e.cpart, e.nz, e.h, i, i, 1);
}

__global__ __launch_bounds__(1024) void k_cost_reduce_batched(const BatchHdr *__restrict__ bh,
                                                              int count, int64_t tiles,
                                                              int64_t blocks, double *out) {
  if (!batch_ok(bh, count, tiles, blocks)) return;
  const BatchEntry &e = batch_table(bh)[blockIdx.x];
  cost_reduce_wg(e.cpart, e.nt, e.n, e.h, out + 2 * (int64_t)blockIdx.x);
}

}  // namespace

// ----------------------------------------------------------------------------
// Host-side sequencing
// ----------------------------------------------------------------------------
// A second stream per device for the all-zero-tile kernel, forked from and
// joined back into the caller's stream with events, so that the two force
// kernels share the GPU (the nonzero-tile one is bound by its P stream, the
// all-zero one by the vector ALUs). Default priority. The enqueue sequence is
// serialised by a mutex, so concurrent callers never interleave on the
// shared events.
namespace {
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_side_mu;
SideStream g_side[64];

hipError_t side_stream(SideStream *&out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  SideStream &ss = g_side[dev];
  if (!ss.s) {
    if ((e = hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&ss.join, hipEventDisableTiming)) != hipSuccess) return e;
  }
  out = &ss;
  return hipSuccess;
}
}  // namespace

hipError_t launch_force(const Layout &L, void *ws, const float *y, hipStream_t st) {
  Hdr *h = at<Hdr>(ws, L.hdr);
  float2 *yp = at<float2>(ws, L.yp);
  hipLaunchKernelGGL(k_gather_y, dim3(L.nb), dim3(256), 0, st, reinterpret_cast<const float2 *>(y),
                     at<const int32_t>(ws, L.perm), L.n, yp, at<float4>(ws, L.extent), h);
  const int32_t *tl = at<const int32_t>(ws, L.tlist), *tc = at<const int32_t>(ws, L.tcount);
  const int2 *tm = at<const int2>(ws, L.tmap);
  float4 *part = at<float4>(ws, L.part);
  float *zp = at<float>(ws, L.zpart);
  const unsigned full_grid = (unsigned)(L.nt < kFullGrid ? L.nt : kFullGrid);
  std::lock_guard<std::mutex> lock(g_side_mu);
  SideStream *ss = nullptr;
  hipError_t e = side_stream(ss);
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(ss->fork, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_force_full, dim3(full_grid), dim3(256), 0, st, at<const float4>(ws, L.P),
                     (const float2 *)yp, L.n, L.nb, part, zp, tl, tc, tm, h);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(ss->s, ss->fork, 0)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_force_zero, dim3((unsigned)L.nt), dim3(256), 0, ss->s, (const float2 *)yp,
                     L.n, L.nb, part, zp, tl, tc, tm, h, 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipEventRecord(ss->join, ss->s)) != hipSuccess) return e;
  return hipStreamWaitEvent(st, ss->join, 0);
}

// Implicit P: the all-zero tiles (known since the affinity stage) in one
// repulsion-only launch on the side stream, as in the stored path; beside it,
// per buffer of block rows, the nonzero tiles' packed P recomputed by one
// tile-distance launch (zero tiles skipped) and the full tile body on them.
// The two write disjoint partial-sum slots. The slot lists and the sums of P
// are those of the affinity stage.
hipError_t launch_force_implicit(const Layout &L, void *ws, const float *y, hipStream_t st) {
  Hdr *h = at<Hdr>(ws, L.hdr);
  float2 *yp = at<float2>(ws, L.yp);
  hipLaunchKernelGGL(k_gather_y, dim3(L.nb), dim3(256), 0, st, reinterpret_cast<const float2 *>(y),
                     at<const int32_t>(ws, L.perm), L.n, yp, at<float4>(ws, L.extent), h);
  float4 *part = at<float4>(ws, L.part);
  float *zp = at<float>(ws, L.zpart);
  const int2 *tm = at<const int2>(ws, L.tmap);
  std::lock_guard<std::mutex> lock(g_side_mu);
  SideStream *ss = nullptr;
  hipError_t e = side_stream(ss);
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(ss->fork, st)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(ss->s, ss->fork, 0)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_force_zero, dim3((unsigned)L.nt), dim3(256), 0, ss->s, (const float2 *)yp,
                     L.n, L.nb, part, zp, at<const int32_t>(ws, L.tlist),
                     at<const int32_t>(ws, L.tcount), tm, h, 2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipEventRecord(ss->join, ss->s)) != hipSuccess) return e;
  const int64_t cap = implicit_capacity(L);
  for (int b0 = 0; b0 < L.nb;) {
    // the block rows whose tiles fill the buffer (at least one)
    int b1 = b0 + 1;
    while (b1 < L.nb && tile_start(b1 + 1, L.nb) - tile_start(b0, L.nb) <= cap) ++b1;
    const int64_t base = tile_start(b0, L.nb), count = tile_start(b1, L.nb) - base;
    // the nonzero tiles' P, packed as the distances are formed
    if ((e = launch_implicit_tiles(L, ws, base, count, base, true, true, st)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_force_range, dim3((unsigned)count), dim3(256), 0, st,
                       at<const float4>(ws, L.P), (const float2 *)yp, L.n, L.nb, part, zp, tm,
                       at<const uint8_t>(ws, L.nz), base, implicit_key(L.d, L.mode), h);
    b0 = b1;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipStreamWaitEvent(st, ss->join, 0);
}

hipError_t launch_cost_implicit(const Layout &L, void *ws, const float *y, double *out,
                                hipStream_t st) {
  Hdr *h = at<Hdr>(ws, L.hdr);
  double2 *cp = at<double2>(ws, L.cpart);
  float2 *yp = at<float2>(ws, L.yp);
  hipLaunchKernelGGL(k_gather_y, dim3(L.nb), dim3(256), 0, st, reinterpret_cast<const float2 *>(y),
                     at<const int32_t>(ws, L.perm), L.n, yp, at<float4>(ws, L.extent), h);
  const int64_t cap = implicit_capacity(L);
  for (int b0 = 0; b0 < L.nb;) {
    int b1 = b0 + 1;
    while (b1 < L.nb && tile_start(b1 + 1, L.nb) - tile_start(b0, L.nb) <= cap) ++b1;
    const int64_t base = tile_start(b0, L.nb), count = tile_start(b1, L.nb) - base;
    {
      // the nonzero tiles' P, packed as the distances are formed
      hipError_t e = launch_implicit_tiles(L, ws, base, count, base, true, true, st);
      if (e != hipSuccess) return e;
    }
    // every tile: the all-zero ones add to Z without reading P
    hipLaunchKernelGGL(k_cost_range, dim3((unsigned)count), dim3(256), 0, st,
                       at<const float4>(ws, L.P), (const float2 *)yp, L.n, L.nb, cp,
                       at<const uint8_t>(ws, L.nz), h, base);
    b0 = b1;
  }
  hipLaunchKernelGGL(k_cost_reduce, dim3(1), dim3(1024), 0, st, cp, L.nt, L.n, h, out);
  return hipGetLastError();
}

hipError_t launch_update(const Layout &L, void *ws, float *y, float *u, float *g, float alpha,
                         float mu, float eta, float min_gain, int recentre, int lr_rule,
                         float *grad_out, double *z_out, hipStream_t st) {
  Hdr *h = at<Hdr>(ws, L.hdr);
  double2 *mp = at<double2>(ws, L.meanpart);
  hipLaunchKernelGGL(k_update, dim3((unsigned)(L.nb * kUpdPerBlock)), dim3(kUpd), 0, st,
                     at<const float4>(ws, L.part), at<const int32_t>(ws, L.slots),
                     at<const int32_t>(ws, L.nslots), at<const float>(ws, L.zpart), L.nt, L.n,
                     L.nb, at<const int32_t>(ws, L.perm), reinterpret_cast<float2 *>(y),
                     reinterpret_cast<float2 *>(u), reinterpret_cast<float2 *>(g), alpha, mu, eta,
                     min_gain, lr_rule, at<const float4>(ws, L.extent),
                     reinterpret_cast<float2 *>(grad_out), z_out, mp, h);
  if (recentre)
    hipLaunchKernelGGL(k_recentre, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, st, mp, L.n,
                       L.nb, reinterpret_cast<float2 *>(y), h);
  return hipGetLastError();
}

hipError_t launch_gradient_only(const Layout &L, void *ws, float alpha, float *grad_out,
                                double *z_out, hipStream_t st) {
  Hdr *h = at<Hdr>(ws, L.hdr);
  hipLaunchKernelGGL(k_grad_only, dim3((unsigned)(L.nb * kUpdPerBlock)), dim3(kUpd), 0, st,
                     at<const float4>(ws, L.part), at<const int32_t>(ws, L.slots),
                     at<const int32_t>(ws, L.nslots), at<const float>(ws, L.zpart), L.nt, L.n,
                     L.nb, at<const int32_t>(ws, L.perm), alpha,
                     reinterpret_cast<float2 *>(grad_out), z_out, h);
  return hipGetLastError();
}

hipError_t launch_cost(const Layout &L, void *ws, const float *y, double *out, hipStream_t st) {
  Hdr *h = at<Hdr>(ws, L.hdr);
  double2 *cp = at<double2>(ws, L.cpart);
  float2 *yp = at<float2>(ws, L.yp);
  hipLaunchKernelGGL(k_gather_y, dim3(L.nb), dim3(256), 0, st, reinterpret_cast<const float2 *>(y),
                     at<const int32_t>(ws, L.perm), L.n, yp, at<float4>(ws, L.extent), h);
  hipLaunchKernelGGL(k_cost, dim3((unsigned)L.nt), dim3(256), 0, st, at<const float4>(ws, L.P), yp,
                     L.n, L.nb, cp, at<const uint8_t>(ws, L.nz), h);
  hipLaunchKernelGGL(k_cost_reduce, dim3(1), dim3(1024), 0, st, cp, L.nt, L.n, h, out);
  return hipGetLastError();
}

hipError_t launch_batch_cost(const void *batch_ws, int count, int64_t total_tiles,
                             int64_t total_blocks, double *out, hipStream_t st) {
  const BatchHdr *bh = reinterpret_cast<const BatchHdr *>(batch_ws);
  hipLaunchKernelGGL(k_gather_batched, dim3((unsigned)total_blocks), dim3(256), 0, st, bh, count,
                     total_tiles, total_blocks);
  hipLaunchKernelGGL(k_cost_batched, dim3((unsigned)total_tiles), dim3(256), 0, st, bh, count,
                     total_tiles, total_blocks);
  hipLaunchKernelGGL(k_cost_reduce_batched, dim3((unsigned)count), dim3(1024), 0, st, bh, count,
                     total_tiles, total_blocks, out);
  return hipGetLastError();
}

hipError_t launch_batch_step(const void *batch_ws, int count, int64_t total_tiles,
                             int64_t total_blocks, float alpha, float mu, float eta,
                             float min_gain, int recentre, int lr_rule, hipStream_t st) {
  const BatchHdr *bh = reinterpret_cast<const BatchHdr *>(batch_ws);
  hipLaunchKernelGGL(k_gather_batched, dim3((unsigned)total_blocks), dim3(256), 0, st, bh, count,
                     total_tiles, total_blocks);
  {
    std::lock_guard<std::mutex> lock(g_side_mu);
    SideStream *ss = nullptr;
    hipError_t e = side_stream(ss);
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(ss->fork, st)) != hipSuccess) return e;
    const unsigned full_grid = (unsigned)(total_tiles < kFullGrid ? total_tiles : kFullGrid);
    hipLaunchKernelGGL(k_force_full_batched, dim3(full_grid), dim3(256), 0, st, bh, count,
                       total_tiles, total_blocks);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(ss->s, ss->fork, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_force_zero_batched, dim3((unsigned)total_tiles), dim3(256), 0, ss->s, bh,
                       count, total_tiles, total_blocks);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipEventRecord(ss->join, ss->s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(st, ss->join, 0)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_update_batched, dim3((unsigned)(total_blocks * kUpdPerBlock)), dim3(kUpd),
                     0, st, bh, count,
                     total_tiles, total_blocks, alpha, mu, eta, min_gain, lr_rule);
  if (recentre)
    hipLaunchKernelGGL(k_recentre_batched, dim3((unsigned)total_blocks), dim3(256), 0, st, bh,
                       count, total_tiles, total_blocks);
  return hipGetLastError();
}

}  // namespace tsne
