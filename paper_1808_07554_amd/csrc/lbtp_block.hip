// Temporal blocking of the plain D2Q5 pressure sweep (gfx950).
//
// The pressure lattice is iterated many times per coupled step (eq. 3-1
// "iterated to a steady state", Section 3), and a plain sweep (one that
// neither re-bases nor evaluates the stopping rule) only needs the previous
// state within one link.  So one launch here runs H consecutive plain sweeps:
// each workgroup loads a square region of kBR x kBR nodes (its tile of
// kBR - 2H nodes per side plus a halo of H) into LDS, sweeps it H times
// between two LDS copies, and writes back only the tile, whose nodes lie at least H links
// from any cut edge of the region and so never see the stale halo.  Walls
// and periodic faces are handled where the region meets them, with the same
// rules as the one-sweep kernels.
//
// Arithmetic and its order are those of sweep_cell (lbtp_device.h) for a
// plain sweep, so float32 storage gives bitwise the same populations as H
// single sweeps.  16-bit storage rounds to the storage format only when the
// tile is written back (once per launch instead of once per sweep).
//
// H must be odd: the launch reads one population buffer and writes the
// other, which is where H single sweeps would leave the state.
#include <math.h>
#include <stdint.h>

#include "lbtp_device.h"

namespace lbtp {
namespace {

constexpr int kBR = 64;                          // region side (tile + 2 H)
constexpr int kBN = kBR * kBR;                   // region nodes
constexpr int kBT = 1024;                        // threads per workgroup
constexpr int kBPer = kBN / kBT;                 // region nodes per thread
static_assert(kBN % kBT == 0, "whole region rows per pass");

__device__ inline int wrap_mod(int v, int n) {
  const int r = v % n;
  return r < 0 ? r + n : r;
}

template <typename T, bool HAS_FP>
__global__ __launch_bounds__(kBT) void f_block_kernel(KC kc, FPtrs fin_, FPtrs fout_, const float *__restrict__ Pb,
                                                      const float *__restrict__ itau, const float *__restrict__ Fp,
                                                      const Ctl *__restrict__ ctl, long long k, int H,
                                                      int tiles_x) {
  if (ctl->done || k > ctl->kmax) return;
  // deviations d_j of the region (against the base of their node), two
  // copies: sweep s reads copy (s - 1) & 1 and writes the other
  __shared__ float sd[2][4][kBN];
  __shared__ float sp[kBN];       // base pressure P_b of the region
  __shared__ float st[kBN];       // 1 / tau_f of the region
  const FP<T> fin = typed<T>(fin_), fout = typed<T>(fout_);
  const float is = kc.inv_dev_scale;
  const int tile = kBR - 2 * H;
  const int gx0 = (int)(blockIdx.x % tiles_x) * tile - H;   // global coordinates of region node (0, 0)
  const int gy0 = (int)(blockIdx.x / tiles_x) * tile - H;
  const bool perx = kc.bc_f[0] == LBTP_BC_PERIODIC, pery = kc.bc_f[2] == LBTP_BC_PERIODIC;
  // region nodes inside the domain: [lo, hi) per axis (all of them on a periodic axis)
  const int xlo = perx ? 0 : max(0, -gx0), xhi = perx ? kBR : min(kBR, kc.nx - gx0);
  const int ylo = pery ? 0 : max(0, -gy0), yhi = pery ? kBR : min(kBR, kc.ny - gy0);
  // a region edge that cuts through the domain (not a wall) loses one valid
  // node row per sweep
  const bool cut_l = perx || gx0 > 0, cut_r = perx || gx0 + kBR < kc.nx;
  const bool cut_b = pery || gy0 > 0, cut_t = pery || gy0 + kBR < kc.ny;
  const int rx = threadIdx.x % kBR;               // each thread keeps one column
  const int ry0 = threadIdx.x / kBR;              // and every (kBT / kBR)-th row from ry0

  float fpv[HAS_FP ? kBPer : 1];
#pragma unroll
  for (int t = 0; t < kBPer; ++t) {
    const int ry = ry0 + t * (kBT / kBR);
    const int idx = ry * kBR + rx;
    if (HAS_FP) fpv[t] = 0.0f;
    if (rx < xlo || rx >= xhi || ry < ylo || ry >= yhi) continue;
    const int gx = perx ? wrap_mod(gx0 + rx, kc.nx) : gx0 + rx;
    const int gy = pery ? wrap_mod(gy0 + ry, kc.ny) : gy0 + ry;
    const int c = gy * kc.nx + gx;
#pragma unroll
    for (int j = 0; j < 4; ++j) sd[0][j][idx] = Storage<T>::load(fin.p[j], c, is);
    sp[idx] = Pb[c];
    st[idx] = itau[c];
    if (HAS_FP) fpv[t] = kc.dt * kc.wbar * Fp[c];
  }
  __syncthreads();

  const int ux = gx0 + rx;                        // global x (unwrapped)
  for (int s = 1; s <= H; ++s) {
    const int wxl = cut_l ? s : xlo, wxh = cut_r ? kBR - s : xhi;
    const int wyl = cut_b ? s : ylo, wyh = cut_t ? kBR - s : yhi;
    const int rd = (s - 1) & 1;
    const bool last = s == H;
    if (rx >= wxl && rx < wxh) {
#pragma unroll
      for (int t = 0; t < kBPer; ++t) {
        const int ry = ry0 + t * (kBT / kBR);
        if (ry < wyl || ry >= wyh) continue;
        const int idx = ry * kBR + rx;
        const int uy = gy0 + ry;
        const float pb = sp[idx];
        float e[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int a = dir_axis(j), sg = dir_sign(j);
          // walls only on non-periodic axes, where the coordinates need no wrapping
          const bool out = (a == 0) ? (!perx && (sg > 0 ? ux == 0 : ux == kc.nx - 1))
                                    : (!pery && (sg > 0 ? uy == 0 : uy == kc.ny - 1));
          if (!out) {
            const int src = idx - sg * (a == 0 ? 1 : kBR);
            e[j] = sd[rd][j][src] + kc.w1 * (sp[src] - pb);
          } else {
            const int face = 2 * a + (sg > 0 ? 0 : 1);
            const float o = sd[rd][dir_opp(j)][idx];
            if (kc.bc_f[face] == LBTP_BC_DIRICHLET) {
              // the coordinate along the wall may run over a periodic axis
              const int wx = perx ? wrap_mod(ux, kc.nx) : ux, wy = pery ? wrap_mod(uy, kc.ny) : uy;
              e[j] = 2.0f * kc.w1 * (wall_P(kc, face, wx, wy, 0, 1, 0) - pb) - o;
            } else {
              e[j] = o;
            }
          }
        }
        const float dP = dpressure<2>(e, kc);
        const float wdP = kc.w1 * dP;
        const float it = st[idx];
        float o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          o[j] = e[j] + (wdP - e[j]) * it;
          if (HAS_FP) o[j] += fpv[t];
        }
        if (!last) {
#pragma unroll
          for (int j = 0; j < 4; ++j) sd[rd ^ 1][j][idx] = o[j];
        } else if (rx >= H && rx < H + tile && ry >= H && ry < H + tile && ux < kc.nx && uy < kc.ny) {
          // the tile (region nodes [H, H + tile) per axis inside the domain)
          // goes from the last sweep straight to global memory
          const int c = uy * kc.nx + ux;
#pragma unroll
          for (int j = 0; j < 4; ++j) Storage<T>::store(fout.p[j], c, o[j], kc.dev_scale);
        }
      }
    }
    if (!last) __syncthreads();
  }
}

template <typename T>
void block_launch(const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, const float *itau, const float *Fp,
                  const Ctl *ctl, long long k, int H, hipStream_t s) {
  const int tile = kBR - 2 * H;
  const int tx = (kc.nx + tile - 1) / tile, ty = (kc.ny + tile - 1) / tile;
  if (Fp)
    hipLaunchKernelGGL((f_block_kernel<T, true>), dim3(tx * ty), dim3(kBT), 0, s, kc, fin, fout, Pb, itau, Fp, ctl, k,
                       H, tx);
  else
    hipLaunchKernelGGL((f_block_kernel<T, false>), dim3(tx * ty), dim3(kBT), 0, s, kc, fin, fout, Pb, itau, Fp, ctl,
                       k, H, tx);
}

}  // namespace

int block_sweeps_supported(int dim, const KC &kc, int H) {
  return dim == 2 && kc.nz == 1 && H >= 3 && H % 2 == 1 && kBR - 2 * H >= 16;
}

hipError_t launch_f_block(int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, const float *itau,
                          const float *Fp, const Ctl *ctl, long long k, int H, hipStream_t s) {
  switch (storage) {
    case LBTP_FP16_DEV: block_launch<_Float16>(kc, fin, fout, Pb, itau, Fp, ctl, k, H, s); break;
    case LBTP_BF16_DEV: block_launch<bf16_t>(kc, fin, fout, Pb, itau, Fp, ctl, k, H, s); break;
    default: block_launch<float>(kc, fin, fout, Pb, itau, Fp, ctl, k, H, s); break;
  }
  return hipGetLastError();
}

}  // namespace lbtp
