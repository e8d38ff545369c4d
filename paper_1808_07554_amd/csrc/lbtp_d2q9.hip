// D2Q9 kernels (gfx950): the paper's own lattice (Section 3, eq. 3-5, 3-6)
// for both distributions, one node per thread.
//
// Layout and forms are those of the D2Q5 / D3Q7 kernels (lbtp_kernels.hip):
// the pressure lattice stores the deviations d_i = f_i - w_i P_b of its eight
// moving populations in a pull-form ping-pong (local form right after
// initialisation), the saturation lattice stores g_0..g_8 as float and
// pushes after the collision.  What changes with D2Q9:
//   - directions j = 0..7 (population i = j + 1, the order of eq. 3-6):
//     +x, +y, -x, -y, then (1,1), (-1,1), (-1,-1), (1,-1); weights 1/9 on
//     the axes and 1/36 on the diagonals (eq. 3-5), c_s^2 = c^2/3 (eq. 3-6a),
//     source weights bar-omega_i = 1/8 (eq. 3-5a);
//   - g^eq is eq. 3-4 with C = (beta - phi) I, so every g_i^eq depends on the
//     local porosity:  Gamma_i = g_i^eq / S = w_i (phi + (beta - phi)
//     (|c_i|^2 - 2 c_s^2) / (2 c_s^2)), i.e. w_0 (2 phi - beta) at rest,
//     w_1 (phi + beta) / 2 on the axes, w_2 (2 beta - phi) on the diagonals;
//   - a diagonal link can cross an x face and a y face at once (corner
//     nodes); the rule of the y face then applies, and a link that crosses
//     one periodic and one wall face is reflected by the wall.
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "lbtp_d2q9.h"

namespace lbtp {
namespace {

// ------------------------------------------------------------ pressure sweep
// One iteration of eq. 3-1 per node (q9_sweep_cell).
template <typename T, bool LOCAL, int MODE, bool HAS_FP>
__global__ __launch_bounds__(kThreads) void q9_f_sweep_kernel(KC kc, FPtrs fin_, FPtrs fout_,
                                                              const float *__restrict__ Pb_in,
                                                              float *__restrict__ Pb_out,
                                                              const float *__restrict__ itau,
                                                              const float *__restrict__ Fp,
                                                              double *__restrict__ partials,
                                                              const Ctl *__restrict__ ctl, long long k) {
  if (ctl->done || k > ctl->kmax) return;
  const int c = blockIdx.x * kThreads + threadIdx.x;
  double acc[2] = {0.0, 0.0};
  if (c < kc.ncell)
    q9_sweep_cell<T, LOCAL, MODE, HAS_FP>(kc, typed<T>(fin_), typed<T>(fout_), Pb_in, Pb_out, itau, Fp, c, acc);
  if (MODE == 2) block_sum<2>(acc, partials);
}

template <typename T, int MODE, bool HAS_FP>
__global__ __launch_bounds__(kThreads) void q9_f_sweep_vec_kernel(KC kc, FPtrs fin_, FPtrs fout_,
                                                                  const float *__restrict__ Pb_in,
                                                                  float *__restrict__ Pb_out,
                                                                  const float *__restrict__ itau,
                                                                  const float *__restrict__ Fp,
                                                                  double *__restrict__ partials,
                                                                  const Ctl *__restrict__ ctl, long long k) {
  if (ctl->done || k > ctl->kmax) return;
  double acc[2] = {0.0, 0.0};
  q9_sweep_quad<T, MODE, HAS_FP>(kc, typed<T>(fin_), typed<T>(fout_), Pb_in, Pb_out, itau, Fp,
                                 blockIdx.x * kThreads + threadIdx.x, acc);
  if (MODE == 2) block_sum<2>(acc, partials);
}

// ------------------------------------------------ blocked plain sweeps
// H plain sweeps per launch with the region held in registers, as the D2Q5
// blocked kernel (lbtp_block.h) does: each lane owns one column of a
// 64-column region, each of the kQ9W wavefronts RW consecutive rows (5 for
// the BGK kernel without a source on grids of many tiles, 126 registers;
// kQ9RW = 4 otherwise).
// Populations moving along x or diagonally come from the adjacent lanes
// (shuffles), those moving along y from the lane's own rows or, across
// wavefronts, through an LDS exchange of the three populations that leave a
// row upwards (j = 1, 4, 5) or downwards (j = 3, 6, 7).  Only the tile at
// least H links from every cut edge of the region is written back.  The
// arithmetic is that of q9_f_sweep_kernel for a plain sweep (bitwise the
// same populations with float32 storage); walls follow q9_load_e, with the
// y face's priority at corners and per-link conditions.  H odd: a launch
// reads one population buffer and writes the other.
constexpr int kQ9BX = 64, kQ9W = 16, kQ9RW = 4;

__device__ inline int q9_wrap_any(int v, int n) {
  const int r = v % n;
  return r < 0 ? r + n : r;
}

// Element i of an array, addressed by a 32-bit byte offset from its base.
template <typename T>
__device__ inline T *q9_at(T *p, uint32_t i) {
  return (T *)((char *)p + i * (uint32_t)sizeof(T));
}

// BGK_ONLY: the collision is BGK, so the sweep loop carries no MRT code (4 %
// of its time); otherwise kc.mrt chooses at run time (a fixed MRT would
// need more than 128 registers).
template <typename T, bool HAS_FP, bool BGK_ONLY, int RW>
__global__ __launch_bounds__(kQ9BX * kQ9W) void q9_f_block_kernel(KC kc, FPtrs fin_, FPtrs fout_,
                                                                  const float *__restrict__ Pb,
                                                                  const float *__restrict__ itau,
                                                                  const float *__restrict__ Fp,
                                                                  const Ctl *__restrict__ ctl, long long k, int H,
                                                                  int tiles_x) {
  if (ctl->done || k > ctl->kmax) return;
  constexpr int W = kQ9W, BY = W * RW;
  // two copies (sweep s reads copy (s - 1) & 1): the upward populations of
  // each wavefront's last row, the downward ones of its first row
  __shared__ float xup[2][3][W][kQ9BX];
  __shared__ float xdn[2][3][W][kQ9BX];
  const FP<T> fin = typed<T>(fin_), fout = typed<T>(fout_);
  const float is = kc.inv_dev_scale;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tcols = kQ9BX - 2 * H, trows = BY - 2 * H;
  int tile_x, tile_y;
  // bands 8 tiles wide (on 4096^2 faster than rows, or bands of 4, 16, 32)
  band_tile(xcd_tile((int)blockIdx.x, (int)gridDim.x), tiles_x, (int)gridDim.x / tiles_x, 8, &tile_x, &tile_y);
  const int gx0 = tile_x * tcols - H;   // global coordinates of region node (0, 0)
  const int gy0 = tile_y * trows - H;
  const bool perx = kc.bc_f[0] == LBTP_BC_PERIODIC, pery = kc.bc_f[2] == LBTP_BC_PERIODIC;
  const int ux = gx0 + lane;                                // this lane's column (unwrapped)
  const bool colin = perx || (ux >= 0 && ux < kc.nx);
  const int gx = perx ? q9_wrap_any(ux, kc.nx) : ux;
  const int uy0 = gy0 + wv * RW;                            // this wavefront's first row (unwrapped)
  auto row_in = [&](int uy) { return pery || (uy >= 0 && uy < kc.ny); };
  auto gidx = [&](int uy) { return (pery ? q9_wrap_any(uy, kc.ny) : uy) * kc.nx + gx; };

  float d[RW][8], it[RW];
  float fpv[HAS_FP ? RW : 1];
  float pb[RW + 2], pbl[RW + 2], pbr[RW + 2];   // base of rows -1 .. RW at x, x - 1, x + 1
  // a region one node or more inside the domain on every side wraps no
  // index, holds no wall node and needs no row or column test; its loads take
  // 32-bit offsets from the arrays' uniform base addresses (a context holds
  // fewer than 2^31 populations, so no array reaches 4 GiB)
  const bool interior = gx0 >= 1 && gx0 + kQ9BX <= kc.nx - 1 && gy0 >= 1 && gy0 + BY <= kc.ny - 1;
  if (interior) {
    const uint32_t rs = (uint32_t)kc.nx, n0 = (uint32_t)uy0 * rs + (uint32_t)ux;
#pragma unroll
    for (int t = 0; t < RW + 2; ++t) pb[t] = *q9_at(Pb, n0 + (uint32_t)t * rs - rs);
#pragma unroll
    for (int t = 0; t < RW; ++t) {
      const uint32_t c = n0 + (uint32_t)t * rs;
#pragma unroll
      for (int j = 0; j < 8; ++j) d[t][j] = Storage<T>::load(q9_at(fin.p[j], c), 0, is);
      it[t] = *q9_at(itau, c);
      if (HAS_FP) fpv[t] = kc.dt * kc.wbar * *q9_at(Fp, c);
    }
  } else {
#pragma unroll
    for (int t = 0; t < RW + 2; ++t) {
      const int uy = uy0 + t - 1;
      pb[t] = (colin && row_in(uy)) ? Pb[gidx(uy)] : 0.0f;
    }
#pragma unroll
    for (int t = 0; t < RW; ++t) {
      const int uy = uy0 + t;
      const bool in = colin && row_in(uy);
      const int c = in ? gidx(uy) : 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {   // unconditional loads, selected afterwards (as in block_region)
        const float v = Storage<T>::load(fin.p[j], c, is);
        d[t][j] = in ? v : 0.0f;
      }
      it[t] = in ? itau[c] : 0.0f;
      if (HAS_FP) fpv[t] = in ? kc.dt * kc.wbar * Fp[c] : 0.0f;
    }
  }
  // the x-neighbours' bases by lane shifts (the outermost lanes get 0: they
  // are columns outside the tile's dependence cone, or beyond a wall)
#pragma unroll
  for (int t = 0; t < RW + 2; ++t) {
    pbl[t] = lane_from_left(pb[t]);
    pbr[t] = lane_from_right(pb[t]);
  }
  xup[0][0][wv][lane] = d[RW - 1][1];
  xup[0][1][wv][lane] = d[RW - 1][4];
  xup[0][2][wv][lane] = d[RW - 1][5];
  xdn[0][0][wv][lane] = d[0][3];
  xdn[0][1][wv][lane] = d[0][6];
  xdn[0][2][wv][lane] = d[0][7];

  // wall nodes in the region: x = 0 or nx - 1 on a walled x axis, likewise y
  const bool walls = (!perx && (gx0 <= 0 || gx0 + kQ9BX > kc.nx - 1)) || (!pery && (gy0 <= 0 || gy0 + BY > kc.ny - 1));
  const bool wall_l = !perx && ux == 0, wall_r = !perx && ux == kc.nx - 1;
  // The wall rules of q9_load_e as e = c + m o per link arriving through a
  // wall (m = -1, c = 2 w (P_w - P_b) for anti-bounce-back; m = 1, c = 0 for
  // bounce-back); fixed while no sweep re-bases.  Three links per face and
  // node: x faces per region row, y faces per column.
  __shared__ float wc_x[2][BY][3], wm_x[2][BY][3], wc_y[2][kQ9BX][3], wm_y[2][kQ9BX][3];
  if (walls) {
    auto rule = [&](int face, int j, int along_x, int along_y, float p, float &c, float &m) {
      const int slot = q9_wall_slot(face, q9x(j), q9y(j));
      if (q9_link_bc(kc.bc_f, kc.wtF, face, face < 2 ? along_y : along_x, slot) == LBTP_BC_DIRICHLET) {
        c = 2.0f * q9w(kc, j) * (wall_P(kc, face, along_x, along_y, 0, 3, slot) - p);
        m = -1.0f;
      } else {
        c = 0.0f;
        m = 1.0f;
      }
    };
    const int jl[3] = {0, 4, 7}, jr[3] = {2, 5, 6}, jb[3] = {1, 4, 5}, jt[3] = {3, 6, 7};
#pragma unroll
    for (int t = 0; t < RW; ++t) {
      const int uy = uy0 + t, ry = wv * RW + t;
      const bool in = row_in(uy) && colin;
      const int wy = pery ? q9_wrap_any(uy, kc.ny) : uy;
      const float p = pb[t + 1];
      if (in && wall_l)
        for (int k = 0; k < 3; ++k) rule(0, jl[k], 0, wy, p, wc_x[0][ry][k], wm_x[0][ry][k]);
      if (in && wall_r)
        for (int k = 0; k < 3; ++k) rule(1, jr[k], kc.nx - 1, wy, p, wc_x[1][ry][k], wm_x[1][ry][k]);
      if (in && !pery && uy == 0)
        for (int k = 0; k < 3; ++k) rule(2, jb[k], gx, 0, p, wc_y[0][lane][k], wm_y[0][lane][k]);
      if (in && !pery && uy == kc.ny - 1)
        for (int k = 0; k < 3; ++k) rule(3, jt[k], gx, kc.ny - 1, p, wc_y[1][lane][k], wm_y[1][lane][k]);
    }
  }
  __syncthreads();
  for (int s = 1; s <= H; ++s) {
    const int rd = (s - 1) & 1;
    // the row below the first and the row above the last (garbage at the
    // region's outer rows, which are cut edges or walls)
    float p1 = wv > 0 ? xup[rd][0][wv - 1][lane] : 0.0f;
    float p4 = wv > 0 ? xup[rd][1][wv - 1][lane] : 0.0f;
    float p5 = wv > 0 ? xup[rd][2][wv - 1][lane] : 0.0f;
    const float a3 = wv < W - 1 ? xdn[rd][0][wv + 1][lane] : 0.0f;
    const float a6 = wv < W - 1 ? xdn[rd][1][wv + 1][lane] : 0.0f;
    const float a7 = wv < W - 1 ? xdn[rd][2][wv + 1][lane] : 0.0f;
#pragma unroll
    for (int t = 0; t < RW; ++t) {
      // rows are updated in place from the bottom up: p1, p4, p5 hold the old
      // upward populations of the row below, the row above is still old
      const float q3 = t < RW - 1 ? d[t + 1][3] : a3;
      const float q6 = t < RW - 1 ? d[t + 1][6] : a6;
      const float q7 = t < RW - 1 ? d[t + 1][7] : a7;
      const float p = pb[t + 1];
      float e[8];
      e[0] = lane_from_left(d[t][0]) + kc.w1 * (pbl[t + 1] - p);     // from (x - 1, y)
      e[1] = p1 + kc.w1 * (pb[t] - p);                               // (x, y - 1)
      e[2] = lane_from_right(d[t][2]) + kc.w1 * (pbr[t + 1] - p);    // (x + 1, y)
      e[3] = q3 + kc.w1 * (pb[t + 2] - p);                           // (x, y + 1)
      e[4] = lane_from_left(p4) + kc.w2 * (pbl[t] - p);              // (x - 1, y - 1)
      e[5] = lane_from_right(p5) + kc.w2 * (pbr[t] - p);             // (x + 1, y - 1)
      e[6] = lane_from_right(q6) + kc.w2 * (pbr[t + 2] - p);         // (x + 1, y + 1)
      e[7] = lane_from_left(q7) + kc.w2 * (pbl[t + 2] - p);          // (x - 1, y + 1)
      if (walls) {
        // links whose pull source lies beyond a wall: e = c + m o with the
        // node's old opposite population o (tables filled at load); x faces
        // first, then y faces, so the y face decides at corners
        const int ry = wv * RW + t, uy = uy0 + t;
        if (wall_l) {
          e[0] = wc_x[0][ry][0] + wm_x[0][ry][0] * d[t][2];
          e[4] = wc_x[0][ry][1] + wm_x[0][ry][1] * d[t][6];
          e[7] = wc_x[0][ry][2] + wm_x[0][ry][2] * d[t][5];
        }
        if (wall_r) {
          e[2] = wc_x[1][ry][0] + wm_x[1][ry][0] * d[t][0];
          e[5] = wc_x[1][ry][1] + wm_x[1][ry][1] * d[t][7];
          e[6] = wc_x[1][ry][2] + wm_x[1][ry][2] * d[t][4];
        }
        if (!pery && uy == 0) {
          e[1] = wc_y[0][lane][0] + wm_y[0][lane][0] * d[t][3];
          e[4] = wc_y[0][lane][1] + wm_y[0][lane][1] * d[t][6];
          e[5] = wc_y[0][lane][2] + wm_y[0][lane][2] * d[t][7];
        }
        if (!pery && uy == kc.ny - 1) {
          e[3] = wc_y[1][lane][0] + wm_y[1][lane][0] * d[t][1];
          e[6] = wc_y[1][lane][1] + wm_y[1][lane][1] * d[t][4];
          e[7] = wc_y[1][lane][2] + wm_y[1][lane][2] * d[t][5];
        }
      }
      float oc[8];
      q9_collide(kc, BGK_ONLY ? false : kc.mrt, e, q9_dsum(e), it[t], oc);
      p1 = d[t][1];
      p4 = d[t][4];
      p5 = d[t][5];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        float o = oc[j];
        if (HAS_FP) o += fpv[t];
        d[t][j] = o;
      }
    }
    if (s == H) break;
    xup[s & 1][0][wv][lane] = d[RW - 1][1];
    xup[s & 1][1][wv][lane] = d[RW - 1][4];
    xup[s & 1][2][wv][lane] = d[RW - 1][5];
    xdn[s & 1][0][wv][lane] = d[0][3];
    xdn[s & 1][1][wv][lane] = d[0][6];
    xdn[s & 1][2][wv][lane] = d[0][7];
    __syncthreads();
  }

  // the tile: columns and rows [H, extent - H) of the region inside the domain
  if (lane < H || lane >= kQ9BX - H || ux >= kc.nx) return;
#pragma unroll
  for (int t = 0; t < RW; ++t) {
    const int ry = wv * RW + t, uy = uy0 + t;
    if (ry < H || ry >= BY - H || uy >= kc.ny) continue;
    const uint32_t c = (uint32_t)uy * (uint32_t)kc.nx + (uint32_t)ux;
#pragma unroll
    for (int j = 0; j < 8; ++j) Storage<T>::store(q9_at(fout.p[j], c), 0, d[t][j], kc.dev_scale);
  }
}

// ------------------------------------------------------------------ moments
template <bool HAS_FS, typename TG>
__global__ __launch_bounds__(kThreads) void q9_moments_kernel(KC kc, GPtrs g, const float *__restrict__ K,
                                                              const float *__restrict__ phi,
                                                              const float *__restrict__ Fs,
                                                              float *__restrict__ S, float *__restrict__ itau,
                                                              double *__restrict__ partials, int write_coef) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  double acc[1] = {0.0};
  if (c < kc.ncell) acc[0] = q9_moments_cell<HAS_FS, TG>(kc, g, K, phi, Fs, S, itau, c, write_coef);
  block_sum<1>(acc, partials);
}

// ---------------------------------------------------------- saturation sweep
// One saturation step per node (q9_g_sweep_cell); block partials of the net
// flux through reflected links.
template <typename T, bool FLOCAL, bool HAS_FS>
__global__ __launch_bounds__(kThreads) void q9_g_sweep_kernel(KC kc, GPtrs gin, GPtrs gout, FPtrs f_,
                                                              const float *__restrict__ Pb,
                                                              const float *__restrict__ itau,
                                                              const float *__restrict__ K,
                                                              const float *__restrict__ phi,
                                                              const float *__restrict__ Fs,
                                                              const float *__restrict__ Sn,
                                                              double *__restrict__ partials) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  double acc[1] = {0.0};
  if (c < kc.ncell)
    acc[0] = q9_g_sweep_cell<T, FLOCAL, HAS_FS>(kc, gin, gout, typed<T>(f_), Pb, itau, K, phi, Fs, Sn, c);
  block_sum<1>(acc, partials);
}

// ------------------------------------------------------------ initialisation
// f_i = w_i P0 - tau_f dt w_i c_i . grad P0 (deviations against P_b = P0) and
// g_i = g_i^eq(S0) - tau_g dt [(Gamma_i/phi - w_i(1 - 1/(2 tau_g))) F_s
//       + Gamma_i c_i . grad S0 - gamma w_i c_i . grad P0 / tau_g]  (eq. gini, gneq).
template <typename T>
__global__ __launch_bounds__(kThreads) void q9_init_kernel(KC kc, const float *__restrict__ P0,
                                                           const float *__restrict__ S0,
                                                           const float *__restrict__ dP0,
                                                           const float *__restrict__ dS0,
                                                           const float *__restrict__ K,
                                                           const float *__restrict__ phi,
                                                           const float *__restrict__ Fs, int neq, FPtrs f_,
                                                           float *__restrict__ Pb, GPtrs g_) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const FP<T> f = typed<T>(f_);
  const GP<T> g = gtyped<T>(g_);
  const Cell q = cell_of(c, kc);
  const float P = P0[c], S = S0[c], ph = phi[c];
  const float fs = Fs ? Fs[c] : 0.0f;
  float gp[2] = {0.f, 0.f}, gs[2] = {0.f, 0.f};
  if (neq) {
    const float inv2dx = 0.5f / (kc.c * kc.dt);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      gp[a] = dP0 ? dP0[a * kc.ncell + c] : cdiff(P0, q, a, kc, inv2dx);
      gs[a] = dS0 ? dS0[a * kc.ncell + c] : cdiff(S0, q, a, kc, inv2dx);
    }
  }
  const float tau_f = 1.0f / inv_tau_f_of(S, K[c], kc);
  const float gamma = -lwk_of(S, K[c], kc) * kc.inv_cs2dt;
  const float itg = kc.cap_B > 0.0f ? inv_tau_g_of(S, K[c], kc) : kc.inv_tau_g;
  const float tau_g = 1.0f / itg;
  const float wsrc = 1.0f - 0.5f * itg;
  Pb[c] = P;
  {
    const float G0 = q9_gamma0(kc, ph);
    float v = G0 * S;
    if (neq) v -= tau_g * kc.dt * ((G0 / ph - kc.w0 * wsrc) * fs);
    if (gdev<T>()) g.B[c] = S;
    gstore(g.p[0], c, v, gdev<T>() ? q9_geq(kc, 0, S, ph) : 0.0f, kc);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float w = q9w(kc, j);
    const float cdp = kc.c * ((float)q9x(j) * gp[0] + (float)q9y(j) * gp[1]);
    const float cds = kc.c * ((float)q9x(j) * gs[0] + (float)q9y(j) * gs[1]);
    Storage<T>::store(f.p[j], c, neq ? -tau_f * kc.dt * w * cdp : 0.0f, kc.dev_scale);
    const float G = q9_gamma(kc, j, ph);
    float v = G * S;
    if (neq) v -= tau_g * kc.dt * ((G / ph - w * wsrc) * fs + G * cds - gamma * w * cdp * itg);
    gstore(g.p[j + 1], c, v, gdev<T>() ? q9_geq(kc, j + 1, S, ph) : 0.0f, kc);
  }
}

// ----------------------------------------------------------------- outputs
template <typename T, bool LOCAL>
__global__ __launch_bounds__(kThreads) void q9_pressure_kernel(KC kc, FPtrs f_, const float *__restrict__ Pb,
                                                               float *__restrict__ P) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const int y = c / kc.nx, x = c - y * kc.nx;
  const float pb = Pb[c];
  float e[8];
  q9_load_e<T, LOCAL>(typed<T>(f_), Pb, c, x, y, kc, pb, e);
  P[c] = pb + q9_dpressure(e, kc);
}

template <typename T, bool LOCAL>
__global__ __launch_bounds__(kThreads) void q9_grad_kernel(KC kc, FPtrs f_, const float *__restrict__ Pb,
                                                           const float *__restrict__ itau,
                                                           const float *__restrict__ K,
                                                           const float *__restrict__ S, int velocity,
                                                           float *__restrict__ out) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const int y = c / kc.nx, x = c - y * kc.nx;
  float e[8];
  q9_load_e<T, LOCAL>(typed<T>(f_), Pb, c, x, y, kc, Pb[c], e);
  float m1[2];
  q9_moment(e, kc, m1);
  float scale = -itau[c] * kc.inv_cs2dt;
  if (velocity) scale = -dp_of(S[c], K[c], kc) * scale;   // u = -D_p grad P
  out[c] = scale * m1[0];
  out[kc.ncell + c] = scale * m1[1];
}

template <bool HAS_FS, typename TG>
__global__ __launch_bounds__(kThreads) void q9_saturation_kernel(KC kc, GPtrs g_, const float *__restrict__ phi,
                                                                 const float *__restrict__ Fs,
                                                                 float *__restrict__ S) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const GP<TG> g = gtyped<TG>(g_);
  const float ph = phi[c], B = gdev<TG>() ? g.B[c] : 0.0f;
  float gv[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) gv[i] = gload(g.p[i], c, gdev<TG>() ? q9_geq(kc, i, B, ph) : 0.0f, kc);
  S[c] = saturation_of(q9_sum_g(gv), HAS_FS ? Fs[c] : 0.0f, ph, kc);
}

template <typename TG>
__global__ __launch_bounds__(kThreads) void q9_gpop_kernel(KC kc, GPtrs g_, const float *__restrict__ phi,
                                                           float *__restrict__ out) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const GP<TG> g = gtyped<TG>(g_);
  const float ph = phi[c], B = gdev<TG>() ? g.B[c] : 0.0f;
#pragma unroll
  for (int i = 0; i < 9; ++i)
    out[(size_t)i * kc.ncell + c] = gload(g.p[i], c, gdev<TG>() ? q9_geq(kc, i, B, ph) : 0.0f, kc);
}

template <typename T, bool LOCAL>
__global__ __launch_bounds__(kThreads) void q9_populations_kernel(KC kc, FPtrs f_, const float *__restrict__ Pb,
                                                                  float *__restrict__ out) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const int y = c / kc.nx, x = c - y * kc.nx;
  const float pb = Pb[c];
  float e[8];
  q9_load_e<T, LOCAL>(typed<T>(f_), Pb, c, x, y, kc, pb, e);
#pragma unroll
  for (int j = 0; j < 8; ++j) out[j * kc.ncell + c] = q9w(kc, j) * pb + e[j];
}

// Calls fn with the storage type (as a null pointer of that type) and the
// local flag as compile-time values.
template <typename Fn>
void q9_dispatch(int storage, int local, Fn &&fn) {
  auto by_local = [&](auto t) {
    if (local) fn(t, std::true_type{});
    else fn(t, std::false_type{});
  };
  if (storage == LBTP_FP16_DEV) by_local((_Float16 *)nullptr);
  else if (storage == LBTP_BF16_DEV) by_local((bf16_t *)nullptr);
  else by_local((float *)nullptr);
}

#define Q9_GRID(kc) dim3(nblocks((kc).ncell)), dim3(kThreads), 0, s

}  // namespace

hipError_t launch_f_sweep_q9(int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb_in, float *Pb_out,
                             const float *itau, const float *Fp, double *partials, const Ctl *ctl, long long k,
                             int local, int mode, hipStream_t s) {
  q9_dispatch(storage, local, [&](auto t, auto l) {
    using T = std::remove_pointer_t<decltype(t)>;
    constexpr bool L = decltype(l)::value;
#define Q9_SWEEP(M, HF)                                                                                   \
  do {                                                                                                    \
    if (!L && kc.nx % 4 == 0)                                                                             \
      hipLaunchKernelGGL((q9_f_sweep_vec_kernel<T, M, HF>), dim3(nblocks(kc.ncell / 4)), dim3(kThreads), 0, s, \
                         kc, fin, fout, Pb_in, Pb_out, itau, Fp, partials, ctl, k);                        \
    else                                                                                                  \
      hipLaunchKernelGGL((q9_f_sweep_kernel<T, L, M, HF>), Q9_GRID(kc), kc, fin, fout, Pb_in, Pb_out, itau, \
                         Fp, partials, ctl, k);                                                           \
  } while (0)
    if (Fp) {
      if (mode == 0) Q9_SWEEP(0, true);
      else if (mode == 1) Q9_SWEEP(1, true);
      else Q9_SWEEP(2, true);
    } else {
      if (mode == 0) Q9_SWEEP(0, false);
      else if (mode == 1) Q9_SWEEP(1, false);
      else Q9_SWEEP(2, false);
    }
#undef Q9_SWEEP
  });
  return hipGetLastError();
}

int block_sweeps_supported_q9(int H) { return H >= 3 && H % 2 == 1 && kQ9BX - 2 * H >= 16 && kQ9W * kQ9RW - 2 * H >= 16; }

hipError_t launch_f_block_q9(int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, const float *itau,
                             const float *Fp, const Ctl *ctl, long long k, int H, hipStream_t s) {
  // 5 rows per wavefront (an 80-row region) for the BGK kernel without a
  // source, 4 (64 rows) where a source or MRT leaves too few registers; on a
  // grid of few tiles (fewer than two rounds of resident workgroups, one per
  // compute unit, at 4 rows) 5 only if it needs no more rounds x rows
  const int tcols = kQ9BX - 2 * H, tx = (kc.nx + tcols - 1) / tcols;
  auto tiles = [&](int rw) { return (long long)tx * ((kc.ny + kQ9W * rw - 2 * H - 1) / (kQ9W * rw - 2 * H)); };
  const long long cus = device_cus();
  const bool rows5 = !Fp && !kc.mrt &&
                     (tiles(4) >= 2 * cus || (tiles(5) + cus - 1) / cus * 5 <= (tiles(4) + cus - 1) / cus * 4);
  const int ty = (int)(tiles(rows5 ? 5 : kQ9RW) / tx);
  q9_dispatch(storage, 0, [&](auto t, auto) {
    using T = std::remove_pointer_t<decltype(t)>;
    auto go = [&](auto kernel) {
      hipLaunchKernelGGL(kernel, dim3(tx * ty), dim3(kQ9BX * kQ9W), 0, s, kc, fin, fout, Pb, itau, Fp, ctl, k, H, tx);
    };
    if (Fp) {
      if (kc.mrt) go(q9_f_block_kernel<T, true, false, 4>);
      else go(q9_f_block_kernel<T, true, true, 4>);
    } else {
      if (kc.mrt) go(q9_f_block_kernel<T, false, false, 4>);
      else if (rows5) go(q9_f_block_kernel<T, false, true, 5>);
      else go(q9_f_block_kernel<T, false, true, 4>);
    }
  });
  return hipGetLastError();
}

hipError_t launch_moments_q9(const KC &kc, GPtrs g, const float *K, const float *phi, const float *Fs, float *S,
                             float *itau, double *partials, int write_coef, hipStream_t s) {
  q9_dispatch(g.storage, 0, [&](auto t, auto) {
    using TG = std::remove_pointer_t<decltype(t)>;
    if (Fs)
      hipLaunchKernelGGL((q9_moments_kernel<true, TG>), Q9_GRID(kc), kc, g, K, phi, Fs, S, itau, partials,
                         write_coef);
    else
      hipLaunchKernelGGL((q9_moments_kernel<false, TG>), Q9_GRID(kc), kc, g, K, phi, Fs, S, itau, partials,
                         write_coef);
  });
  return hipGetLastError();
}

hipError_t launch_g_sweep_q9(int storage, const KC &kc, GPtrs gin, GPtrs gout, FPtrs f, int f_local,
                             const float *Pb, const float *itau, const float *K, const float *phi, const float *Fs,
                             const float *Sn, double *partials, hipStream_t s) {
  q9_dispatch(storage, f_local, [&](auto t, auto l) {
    using T = std::remove_pointer_t<decltype(t)>;
    constexpr bool L = decltype(l)::value;
    if (Fs)
      hipLaunchKernelGGL((q9_g_sweep_kernel<T, L, true>), Q9_GRID(kc), kc, gin, gout, f, Pb, itau, K, phi, Fs, Sn,
                         partials);
    else
      hipLaunchKernelGGL((q9_g_sweep_kernel<T, L, false>), Q9_GRID(kc), kc, gin, gout, f, Pb, itau, K, phi, Fs, Sn,
                         partials);
  });
  return hipGetLastError();
}

hipError_t launch_init_q9(int storage, const KC &kc, const float *P0, const float *S0, const float *dP0,
                          const float *dS0, const float *K, const float *phi, const float *Fs, int neq, FPtrs f,
                          float *Pb, GPtrs g, hipStream_t s) {
  q9_dispatch(storage, 0, [&](auto t, auto) {
    using T = std::remove_pointer_t<decltype(t)>;
    hipLaunchKernelGGL((q9_init_kernel<T>), Q9_GRID(kc), kc, P0, S0, dP0, dS0, K, phi, Fs, neq, f, Pb, g);
  });
  return hipGetLastError();
}

hipError_t launch_pressure_q9(int storage, const KC &kc, FPtrs f, int f_local, const float *Pb, float *P,
                              hipStream_t s) {
  q9_dispatch(storage, f_local, [&](auto t, auto l) {
    using T = std::remove_pointer_t<decltype(t)>;
    hipLaunchKernelGGL((q9_pressure_kernel<T, decltype(l)::value>), Q9_GRID(kc), kc, f, Pb, P);
  });
  return hipGetLastError();
}

hipError_t launch_grad_q9(int storage, const KC &kc, FPtrs f, int f_local, const float *Pb, const float *itau,
                          const float *K, const float *S, int velocity, float *out, hipStream_t s) {
  q9_dispatch(storage, f_local, [&](auto t, auto l) {
    using T = std::remove_pointer_t<decltype(t)>;
    hipLaunchKernelGGL((q9_grad_kernel<T, decltype(l)::value>), Q9_GRID(kc), kc, f, Pb, itau, K, S, velocity, out);
  });
  return hipGetLastError();
}

hipError_t launch_saturation_q9(const KC &kc, GPtrs g, const float *phi, const float *Fs, float *S, hipStream_t s) {
  q9_dispatch(g.storage, 0, [&](auto t, auto) {
    using TG = std::remove_pointer_t<decltype(t)>;
    if (Fs) hipLaunchKernelGGL((q9_saturation_kernel<true, TG>), Q9_GRID(kc), kc, g, phi, Fs, S);
    else hipLaunchKernelGGL((q9_saturation_kernel<false, TG>), Q9_GRID(kc), kc, g, phi, Fs, S);
  });
  return hipGetLastError();
}

hipError_t launch_g_populations_q9(const KC &kc, GPtrs g, const float *phi, float *out, hipStream_t s) {
  q9_dispatch(g.storage, 0, [&](auto t, auto) {
    using TG = std::remove_pointer_t<decltype(t)>;
    hipLaunchKernelGGL((q9_gpop_kernel<TG>), Q9_GRID(kc), kc, g, phi, out);
  });
  return hipGetLastError();
}

hipError_t launch_populations_q9(int storage, const KC &kc, FPtrs f, int f_local, const float *Pb, float *out,
                                 hipStream_t s) {
  q9_dispatch(storage, f_local, [&](auto t, auto l) {
    using T = std::remove_pointer_t<decltype(t)>;
    hipLaunchKernelGGL((q9_populations_kernel<T, decltype(l)::value>), Q9_GRID(kc), kc, f, Pb, out);
  });
  return hipGetLastError();
}

}  // namespace lbtp
