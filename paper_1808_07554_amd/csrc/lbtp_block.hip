// Temporal blocking of the plain D2Q5 pressure sweep, single contexts
// (gfx950): H plain sweeps per launch, one workgroup per tile; the
// workgroup's work is block_region (lbtp_block.h).
#include <math.h>
#include <stdint.h>

#include "lbtp_block.h"

namespace lbtp {
namespace {

template <typename T, bool HAS_FP, int W, int RW>
__global__ __launch_bounds__(kBX * W) void f_block_kernel(
    KC kc, FPtrs fin_, FPtrs fout_, const float *__restrict__ Pb, const float *__restrict__ itau,
    const float *__restrict__ Fp, const Ctl *__restrict__ ctl, long long k, int H, int tiles_x) {
  if (ctl->done || k > ctl->kmax) return;
  // tiles row by row (measured faster here than in bands)
  const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  block_region<T, HAS_FP, W, RW>(kc, typed<T>(fin_), typed<T>(fout_), Pb, itau, Fp, H, t % tiles_x, t / tiles_x);
}

// The same with a re-basing first sweep (a chunk's first), which reads the
// bases Pb and writes the tile's new ones to Pb_out.
template <typename T, bool HAS_FP, int W, int RW>
__global__ __launch_bounds__(kBX * W) void f_block_first_kernel(
    KC kc, FPtrs fin_, FPtrs fout_, const float *__restrict__ Pb, const float *__restrict__ itau,
    const float *__restrict__ Fp, const Ctl *__restrict__ ctl, long long k, int H, int tiles_x,
    float *__restrict__ Pb_out) {
  if (ctl->done || k > ctl->kmax) return;
  const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  block_region<T, HAS_FP, W, RW, 1>(kc, typed<T>(fin_), typed<T>(fout_), Pb, itau, Fp, H, t % tiles_x, t / tiles_x,
                                    Pb_out);
}

// Rows per wavefront of a launch: 9 (a 64 x 72 region, less halo per node)
// without a pressure source, 8 with one.  On a grid of few tiles (fewer
// than two rounds of resident workgroups, two per compute unit, at 8 rows)
// 9 rows are taken only if they need no more rounds x rows than 8: there
// more and shorter workgroups finish sooner.
inline int block_rows_per_wave(const KC &kc, int H, bool has_fp) {
  if (has_fp) return kUseRW;
  const long long slots = 2LL * device_cus();
  long long tiles[2];
  const int rws[2] = {kUseRW, kUseRWPlain};
  for (int i = 0; i < 2; ++i) {
    int tx, ty;
    block_tile_counts_rows(kc, H, kUseW * rws[i], &tx, &ty);
    tiles[i] = (long long)tx * ty;
  }
  if (tiles[0] >= 2 * slots) return kUseRWPlain;
  return (tiles[1] + slots - 1) / slots * rws[1] <= (tiles[0] + slots - 1) / slots * rws[0] ? kUseRWPlain : kUseRW;
}

template <typename T, int RW>
void block_launch_rw(const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, float *Pb_out, const float *itau,
                     const float *Fp, const Ctl *ctl, long long k, int H, hipStream_t s) {
  constexpr int W = kUseW;
  int tx, ty;
  block_tile_counts_rows(kc, H, W * RW, &tx, &ty);
  const dim3 grid(tx * ty), block(kBX * W);
  if (Pb_out) {
    if (Fp)
      hipLaunchKernelGGL((f_block_first_kernel<T, true, W, RW>), grid, block, 0, s, kc, fin, fout, Pb, itau, Fp,
                         ctl, k, H, tx, Pb_out);
    else
      hipLaunchKernelGGL((f_block_first_kernel<T, false, W, RW>), grid, block, 0, s, kc, fin, fout, Pb, itau, Fp,
                         ctl, k, H, tx, Pb_out);
  } else {
    if (Fp)
      hipLaunchKernelGGL((f_block_kernel<T, true, W, RW>), grid, block, 0, s, kc, fin, fout, Pb, itau, Fp, ctl, k,
                         H, tx);
    else
      hipLaunchKernelGGL((f_block_kernel<T, false, W, RW>), grid, block, 0, s, kc, fin, fout, Pb, itau, Fp, ctl, k,
                         H, tx);
  }
}

template <typename T>
void block_launch(const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, float *Pb_out, const float *itau,
                  const float *Fp, const Ctl *ctl, long long k, int H, hipStream_t s) {
  if (Fp || block_rows_per_wave(kc, H, false) == kUseRW)
    block_launch_rw<T, kUseRW>(kc, fin, fout, Pb, Pb_out, itau, Fp, ctl, k, H, s);
  else
    block_launch_rw<T, kUseRWPlain>(kc, fin, fout, Pb, Pb_out, itau, Fp, ctl, k, H, s);
}

hipError_t block_launch_storage(int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, float *Pb_out,
                                const float *itau, const float *Fp, const Ctl *ctl, long long k, int H,
                                hipStream_t s) {
  switch (storage) {
    case LBTP_FP16_DEV: block_launch<_Float16>(kc, fin, fout, Pb, Pb_out, itau, Fp, ctl, k, H, s); break;
    case LBTP_BF16_DEV: block_launch<bf16_t>(kc, fin, fout, Pb, Pb_out, itau, Fp, ctl, k, H, s); break;
    default: block_launch<float>(kc, fin, fout, Pb, Pb_out, itau, Fp, ctl, k, H, s); break;
  }
  return hipGetLastError();
}

}  // namespace

int block_sweeps_supported(int dim, const KC &kc, int H) {
  if (dim == kD2Q9) return block_sweeps_supported_q9(H);
  if (dim == 3) return block_sweeps_supported_3d(H);
  return dim == 2 && kc.nz == 1 && H >= 3 && H % 2 == 1 && kBX - 2 * H >= 16 && kUseW * kUseRW - 2 * H >= 16;
}

hipError_t launch_f_block(int dim, int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb,
                          const float *itau, const float *Fp, const Ctl *ctl, long long k, int H, hipStream_t s) {
  if (dim == kD2Q9) return launch_f_block_q9(storage, kc, fin, fout, Pb, itau, Fp, ctl, k, H, s);
  if (dim == 3) return launch_f_block_3d(storage, kc, fin, fout, Pb, itau, Fp, ctl, k, H, s);
  return block_launch_storage(storage, kc, fin, fout, Pb, nullptr, itau, Fp, ctl, k, H, s);
}

int block_first_supported(int dim, const KC &kc, int H) {
  return dim == 2 && kc.nz == 1 && block_sweeps_supported(dim, kc, H);
}

hipError_t launch_f_block_first(int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, float *Pb_out,
                                const float *itau, const float *Fp, const Ctl *ctl, long long k, int H,
                                hipStream_t s) {
  if (!Pb_out || Pb_out == Pb) return hipErrorInvalidValue;
  return block_launch_storage(storage, kc, fin, fout, Pb, Pb_out, itau, Fp, ctl, k, H, s);
}

}  // namespace lbtp
