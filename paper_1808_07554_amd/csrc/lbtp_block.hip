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

template <typename T, int W, int RW>
void block_launch(const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, const float *itau, const float *Fp,
                  const Ctl *ctl, long long k, int H, hipStream_t s) {
  static_assert(W == kUseW && RW == kUseRW, "the tile counts assume the launch shape in use");
  int tx, ty;
  block_tile_counts(kc, H, &tx, &ty);
  if (Fp)
    hipLaunchKernelGGL((f_block_kernel<T, true, W, RW>), dim3(tx * ty), dim3(kBX * W), 0, s, kc, fin, fout, Pb,
                       itau, Fp, ctl, k, H, tx);
  else
    hipLaunchKernelGGL((f_block_kernel<T, false, W, RW>), dim3(tx * ty), dim3(kBX * W), 0, s, kc, fin, fout, Pb,
                       itau, Fp, ctl, k, H, tx);
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
  switch (storage) {
    case LBTP_FP16_DEV: block_launch<_Float16, kUseW, kUseRW>(kc, fin, fout, Pb, itau, Fp, ctl, k, H, s); break;
    case LBTP_BF16_DEV: block_launch<bf16_t, kUseW, kUseRW>(kc, fin, fout, Pb, itau, Fp, ctl, k, H, s); break;
    default: block_launch<float, kUseW, kUseRW>(kc, fin, fout, Pb, itau, Fp, ctl, k, H, s); break;
  }
  return hipGetLastError();
}

}  // namespace lbtp
