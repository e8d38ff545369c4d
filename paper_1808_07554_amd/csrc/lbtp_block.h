// Register-resident temporal blocking of the plain D2Q5 pressure sweep: the
// work of one workgroup, shared by the single-context kernel
// (lbtp_block.hip) and the ensemble kernel (lbtp_batch.hip).
//
// A workgroup of W wavefronts runs H consecutive sweeps (eq. 3-1) over a
// region of 64 columns x (W * RW) rows held in registers: each lane of a wavefront owns one column, each
// wavefront RW consecutive rows.  The x-streamed populations move between
// adjacent lanes (lane shuffles), the y-streamed ones between the rows of a
// lane's registers, and across wavefronts through a small LDS exchange (one
// barrier per sweep).  Only the tile, the nodes at least H links from any cut
// edge of the region, is written back; the halo around it is recomputed by
// the neighbouring workgroups.  Walls and periodic faces are handled where the
// region meets them, with the same rules as the one-sweep kernels.  The
// sweeps are plain, except that single contexts may make the first one
// re-base (a chunk's first sweep), so that the re-basing sweep needs no
// launch of its own.
//
// Arithmetic and its order are those of sweep_cell (lbtp_device.h) for each
// mode, so float32 storage gives bitwise the same populations and bases as H
// single sweeps.  16-bit storage rounds to the storage format only when the
// tile is written back (once per launch instead of once per sweep).
//
// H must be odd: a launch reads one population buffer and writes the other,
// which is where H single sweeps would leave the state.
#ifndef LBTP_BLOCK_H
#define LBTP_BLOCK_H

#include "lbtp_device.h"

namespace lbtp {

constexpr int kBX = 64;        // region columns: one per lane
constexpr int kBWmax = 16;     // most wavefronts per workgroup
// The launch shapes of single contexts: 8 wavefronts of 9 rows (a 64 x 72
// region) without a pressure source (grids of few tiles may take 8 rows, see
// block_rows_per_wave in lbtp_block.hip) and of 8 rows (64 x 64) with one, so
// that two workgroups fit a compute unit (at most 128 registers a lane) and
// one loads while the other sweeps (measured on the 4096^2 injection problem
// against 16 x 6, 16 x 8, 8 x 6, 8 x 8 and 8 x 10; 9 rows and a source need
// 130 registers, 10 rows 134).
constexpr int kUseW = 8, kUseRW = 8, kUseRWPlain = 9;

__device__ inline int blk_wrap(int v, int n) {
  const int r = v % n;
  return r < 0 ? r + n : r;
}

// Anti-bounce-back / bounce-back value of the population arriving through a
// wall face at node (x, y) whose opposite population is o.  The sweep also
// applies it at region rows and columns beyond the wall, which hold no node
// (their values are never read by a node of the domain); the coordinates are
// clamped so that the wall data are read within their arrays there too.
__device__ inline float blk_wall_rule(const KC &kc, int face, int x, int y, float pb, float o) {
  x = min(max(x, 0), kc.nx - 1);
  y = min(max(y, 0), kc.ny - 1);
  return kc.bc_f[face] == LBTP_BC_DIRICHLET ? 2.0f * kc.w1 * (wall_P(kc, face, x, y, 0, 1, 0) - pb) - o : o;
}

// Element i of an array, addressed by a 32-bit byte offset from its base
// (a context holds fewer than 2^31 populations, so no array reaches 4 GiB).
template <typename T>
__device__ inline T *blk_at(T *p, uint32_t i) {
  return (T *)((char *)p + i * (uint32_t)sizeof(T));
}
template <typename T>
__device__ inline const T *blk_at(const T *p, uint32_t i) {
  return (const T *)((const char *)p + i * (uint32_t)sizeof(T));
}

// State of one lane: RW rows of its column.
template <int RW, bool HAS_FP>
struct BlkRows {
  float d[RW][4];              // deviations
  float pb[RW + 2];            // base of rows -1 .. RW
  float pbl[RW], pbr[RW];      // base of the x-neighbours
  float it[RW];                // 1 / tau_f
  float fp[HAS_FP ? RW : 1];   // dt wbar F_p
};

// One sweep of the lane's rows.  PASS 0: plain (eq. 3-1); 1: also re-base
// every node to its new P and keep the new bases in place of the old ones
// (the pass reads the old ones throughout).  Rows are updated in place from
// the bottom up; the old +y population of the row below, which the next row
// still pulls, is kept aside.
template <int W, int RW, bool HAS_FP, int PASS>
__device__ inline void blk_pass(const KC &kc, BlkRows<RW, HAS_FP> &r, float prev1, float above, int gx, int uy0,
                                bool wall_l, bool wall_r, bool pery, bool walls) {
  float pn[PASS == 1 ? RW : 1];
#pragma unroll
  for (int t = 0; t < RW; ++t) {
    const float p = r.pb[t + 1];
    const float v0 = lane_from_left(r.d[t][0]);
    const float v2 = lane_from_right(r.d[t][2]);
    const float v3 = t < RW - 1 ? r.d[t + 1][3] : above;
    float e[4];
    e[0] = v0 + kc.w1 * (r.pbl[t] - p);
    e[1] = prev1 + kc.w1 * (r.pb[t] - p);
    e[2] = v2 + kc.w1 * (r.pbr[t] - p);
    // w (P_b(y+1) - P_b(y)) is minus the term row t + 1 adds to its e[1]
    // (exactly: negation commutes with the subtraction and the product),
    // so inner rows reuse that value instead of holding one of their own
    e[3] = t < RW - 1 ? v3 - kc.w1 * (r.pb[t + 1] - r.pb[t + 2]) : v3 + kc.w1 * (r.pb[t + 2] - p);
    if (walls) {
      // the row index is made opaque here so that the compiler forms the
      // wall rows' coordinates (a modulo on a periodic axis) inside this
      // branch, in the regions that hold wall nodes, instead of hoisting
      // them for every region and row out of the sweep loop
      int uy = uy0 + t;
      asm volatile("" : "+v"(uy));
      const int wy = pery ? blk_wrap(uy, kc.ny) : uy;
      if (wall_l) e[0] = blk_wall_rule(kc, 0, 0, wy, p, r.d[t][2]);
      if (wall_r) e[2] = blk_wall_rule(kc, 1, kc.nx - 1, wy, p, r.d[t][0]);
      if (!pery && uy == 0) e[1] = blk_wall_rule(kc, 2, gx, 0, p, r.d[t][3]);
      if (!pery && uy == kc.ny - 1) e[3] = blk_wall_rule(kc, 3, gx, kc.ny - 1, p, r.d[t][1]);
    }
    const float sum = dsum<2>(e);
    const float wdP = sum * kc.w1_1mw0;
    // with a source, keep = 1 - 1/tau_f is formed again every sweep: held
    // for all rows it would cost 8 registers and one wavefront per SIMD
    float it = r.it[t];
    if (HAS_FP) asm volatile("" : "+v"(it));
    const float keep = 1.0f - it, gain = wdP * it;
    // the terms added after the relaxation, formed as the one-sweep kernels
    // form them (source first, then the re-basing shift)
    float add = HAS_FP ? r.fp[t] : 0.0f;
    if (PASS == 1) {
      const float dP = sum * kc.inv_1mw0;
      const float P = p + dP;
      add += kc.w1 * (p - P);
      pn[t] = P;
    }
    prev1 = r.d[t][1];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float o = bgk_relax(e[j], keep, gain);
      if (HAS_FP || PASS == 1) o += add;
      r.d[t][j] = o;
    }
  }
  if (PASS == 1) {
#pragma unroll
    for (int t = 0; t < RW; ++t) r.pb[t + 1] = pn[t];
  }
}

// H sweeps of the region.  walls: the region holds wall nodes (uniform over
// the workgroup, so regions inside the domain skip every wall test).  FIRST:
// the first sweep re-bases (pass 1); after it the new bases of the rows next
// to a wavefront's own come through the LDS and those of the neighbouring
// columns by lane shuffles.  The region's outermost rows and columns keep
// their old bases, which only nodes outside the tile's dependence cone read.
template <int W, int RW, bool HAS_FP, int FIRST>
__device__ inline void blk_sweep_rows(const KC &kc, BlkRows<RW, HAS_FP> &r, float (*xup)[kBWmax][kBX],
                                      float (*xdn)[kBWmax][kBX], float (*pbx)[kBWmax][kBX], int H, int lane,
                                      int wv, int ux, int gx, int uy0, bool perx, bool pery, bool walls) {
  const bool wall_l = !perx && ux == 0, wall_r = !perx && ux == kc.nx - 1;
  // the neighbouring wavefronts' rows (garbage at the region's outer rows,
  // which are cut edges or walls)
  auto from_below = [&](int rd) { return wv > 0 ? xup[rd][wv - 1][lane] : 0.0f; };
  auto from_above = [&](int rd) { return wv < W - 1 ? xdn[rd][wv + 1][lane] : 0.0f; };
  // the +y population of the last row and the -y one of the first row for
  // the neighbouring wavefronts' next sweep
  auto exchange = [&](int s) {
    xup[s & 1][wv][lane] = r.d[RW - 1][1];
    xdn[s & 1][wv][lane] = r.d[0][3];
  };
  int s = 1;
  if (FIRST) {
    blk_pass<W, RW, HAS_FP, 1>(kc, r, from_below(0), from_above(0), gx, uy0, wall_l, wall_r, pery, walls);
    exchange(1);
    pbx[0][wv][lane] = r.pb[1];
    pbx[1][wv][lane] = r.pb[RW];
    __syncthreads();
    if (wv > 0) r.pb[0] = pbx[1][wv - 1][lane];
    if (wv < W - 1) r.pb[RW + 1] = pbx[0][wv + 1][lane];
#pragma unroll
    for (int t = 0; t < RW; ++t) {
      r.pbl[t] = lane_from_left(r.pb[t + 1]);
      r.pbr[t] = lane_from_right(r.pb[t + 1]);
    }
    s = 2;
  }
  for (; s <= H; ++s) {
    const int rd = (s - 1) & 1;
    blk_pass<W, RW, HAS_FP, 0>(kc, r, from_below(rd), from_above(rd), gx, uy0, wall_l, wall_r, pery, walls);
    if (s == H) break;
    exchange(s);
    __syncthreads();
  }
}

// The work of one workgroup (kBX * W threads): H sweeps of the region of
// tile (tile_x, tile_y) of a context, reading fin and writing the tile to
// fout; plain sweeps unless FIRST makes the first one re-base (reading the
// bases Pb and writing the tile's new ones to Pb_out).
template <typename T, bool HAS_FP, int W, int RW, int FIRST = 0>
__device__ inline void block_region(const KC &kc, const FP<T> &fin, const FP<T> &fout, const float *__restrict__ Pb,
                                    const float *__restrict__ itau, const float *__restrict__ Fp, int H, int tile_x,
                                    int tile_y, float *__restrict__ Pb_out = nullptr) {
  constexpr int kBY = W * RW;     // region rows
  // boundary rows exchanged between wavefronts, two copies (sweep s reads
  // copy (s - 1) & 1): the +y population of each wavefront's last row and
  // the -y population of its first row
  __shared__ float xup[2][kBWmax][kBX];
  __shared__ float xdn[2][kBWmax][kBX];
  // after a re-basing first sweep: each wavefront's new first- and last-row bases
  __shared__ float pbx[FIRST ? 2 : 1][kBWmax][kBX];
  const float is = kc.inv_dev_scale;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tcols = kBX - 2 * H, trows = kBY - 2 * H;
  const int gx0 = tile_x * tcols - H;   // global coordinates of region node (0, 0)
  const int gy0 = tile_y * trows - H;
  const bool perx = kc.bc_f[0] == LBTP_BC_PERIODIC, pery = kc.bc_f[2] == LBTP_BC_PERIODIC;
  const int ux = gx0 + lane;                                // this lane's column (unwrapped)
  const bool colin = perx || (ux >= 0 && ux < kc.nx);
  const int gx = perx ? blk_wrap(ux, kc.nx) : ux;
  const int uy0 = gy0 + wv * RW;                            // this wavefront's first row (unwrapped)

  auto row_in = [&](int uy) { return pery || (uy >= 0 && uy < kc.ny); };
  auto gidx = [&](int uy) { return (pery ? blk_wrap(uy, kc.ny) : uy) * kc.nx + gx; };

  // a region one node or more inside the domain on every side (most of a
  // large grid) wraps no index, holds no wall node and needs no row or column
  // test; its loads take 32-bit offsets from the arrays' uniform base
  // addresses, one offset per row shared by every array
  const bool interior = gx0 >= 1 && gx0 + kBX <= kc.nx - 1 && gy0 >= 1 && gy0 + kBY <= kc.ny - 1;
  BlkRows<RW, HAS_FP> r;
  if (interior) {
    const uint32_t rs = (uint32_t)kc.nx, n0 = (uint32_t)uy0 * rs + (uint32_t)ux;
#pragma unroll
    for (int t = 0; t < RW + 2; ++t) r.pb[t] = *blk_at(Pb, n0 + (uint32_t)t * rs - rs);
#pragma unroll
    for (int t = 0; t < RW; ++t) {
      const uint32_t c = n0 + (uint32_t)t * rs;
#pragma unroll
      for (int j = 0; j < 4; ++j) r.d[t][j] = Storage<T>::load(blk_at(fin.p[j], c), 0, is);
      r.it[t] = *blk_at(itau, c);
      if (HAS_FP) r.fp[t] = kc.dt * kc.wbar * *blk_at(Fp, c);
    }
  } else {
#pragma unroll
    for (int t = 0; t < RW + 2; ++t) {
      const int uy = uy0 + t - 1;
      r.pb[t] = (colin && row_in(uy)) ? Pb[gidx(uy)] : 0.0f;
    }
#pragma unroll
    for (int t = 0; t < RW; ++t) {
      const int uy = uy0 + t;
      const bool in = colin && row_in(uy);
      const int c = in ? gidx(uy) : 0;
      // every load is issued (from node 0 outside the domain) and the value
      // selected afterwards: a load made conditional on the row would make
      // the compiler wait for each one before issuing the next
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float v = Storage<T>::load(fin.p[j], c, is);
        r.d[t][j] = in ? v : 0.0f;
      }
      r.it[t] = in ? itau[c] : 0.0f;
      if (HAS_FP) r.fp[t] = in ? kc.dt * kc.wbar * Fp[c] : 0.0f;
    }
  }
  // the x-neighbours' bases by lane shifts (the outermost lanes get 0: they
  // are columns outside the tile's dependence cone, or beyond a wall)
#pragma unroll
  for (int t = 0; t < RW; ++t) {
    r.pbl[t] = lane_from_left(r.pb[t + 1]);
    r.pbr[t] = lane_from_right(r.pb[t + 1]);
  }
  xup[0][wv][lane] = r.d[RW - 1][1];
  xdn[0][wv][lane] = r.d[0][3];
  __syncthreads();

  // wall nodes in the region: x = 0 or nx - 1 on a walled x axis, likewise y
  const bool walls = (!perx && (gx0 <= 0 || gx0 + kBX > kc.nx - 1)) || (!pery && (gy0 <= 0 || gy0 + kBY > kc.ny - 1));
  blk_sweep_rows<W, RW, HAS_FP, FIRST>(kc, r, xup, xdn, pbx, H, lane, wv, ux, gx, uy0, perx, pery, walls);

  // the tile: columns and rows [H, extent - H) of the region inside the domain
  const bool tcol = lane >= H && lane < kBX - H && ux < kc.nx;
  auto trow = [&](int t) {
    const int ry = wv * RW + t;
    return ry >= H && ry < kBY - H && uy0 + t < kc.ny;
  };
  if (!tcol) return;
#pragma unroll
  for (int t = 0; t < RW; ++t) {
    if (!trow(t)) continue;
    const uint32_t c = (uint32_t)(uy0 + t) * (uint32_t)kc.nx + (uint32_t)ux;
#pragma unroll
    for (int j = 0; j < 4; ++j) Storage<T>::store(blk_at(fout.p[j], c), 0, r.d[t][j], kc.dev_scale);
    if (FIRST) *blk_at(Pb_out, c) = r.pb[t + 1];
  }
}

// Tiles of a context per axis for block length H and regions of `rows` rows.
__host__ __device__ inline void block_tile_counts_rows(const KC &kc, int H, int rows, int *tx, int *ty) {
  const int tcols = kBX - 2 * H, trows = rows - 2 * H;
  *tx = (kc.nx + tcols - 1) / tcols;
  *ty = (kc.ny + trows - 1) / trows;
}

// Region shapes the ensemble autotuner chooses from: W wavefronts of RW rows.
// Every one keeps the region in registers; they differ in region height
// (the halo share and the ragged last tile of a small member) and in the
// number of workgroups a compute unit holds.
constexpr int kBatchShapes = 5;
__host__ __device__ constexpr int batch_shape_w(int s) { return s == 0 ? 8 : s == 1 ? 8 : s == 2 ? 16 : s == 3 ? 4 : 8; }
__host__ __device__ constexpr int batch_shape_rw(int s) { return s == 0 ? 8 : s == 1 ? 6 : s == 2 ? 4 : s == 3 ? 8 : 9; }
__host__ __device__ constexpr int batch_shape_rows(int s) { return batch_shape_w(s) * batch_shape_rw(s); }

}  // namespace lbtp

#endif  // LBTP_BLOCK_H
