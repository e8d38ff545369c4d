// Ensembles: many independent realisations (grids of different sizes, each
// with its own K, phi, boundary values) advanced together.
//
// Every per-step kernel covers all members in one launch.  Work is cut into
// tiles of 4*NT nodes (NT threads of four nodes each); a table maps each block
// to (member, tile), so small and large members share one grid.  Each member
// has a device control block (convergence flag, iteration base, active
// pressure-base buffer); members that have converged return at once, so one
// launch sequence serves members whose pressure solves need different
// iteration counts.  A chunk of m sweeps plus the stopping-rule reduction is
// captured once in a HIP graph and replayed until every member has stopped;
// the host reads one counter per chunk, one chunk behind the GPU.  Inside a
// chunk the plain sweeps run blocked as in a single context (several sweeps
// per launch over a second (member, tile) table; block_region of
// lbtp_block.h).
//
// The pressure state of every member is always in buffer 0 between solves:
// sweep k reads buffer k & 1, the residual stride m is even and solves stop
// on multiples of m.  Member arithmetic is the single-realisation arithmetic
// (the same device functions), so a member's results are bit-identical to a
// lbtp_ctx run of that member with the same sweeps per launch.
#include <string.h>

#include <vector>

#include "../../include/lbtp.h"
#include "lbtp_block.h"
#include "lbtp_d2q9.h"
#include "lbtp_device.h"

namespace lbtp {

namespace {

template <int NT>
__device__ inline void tile_of(const int *__restrict__ tmember, const int *__restrict__ tindex, int &m, int &t) {
  m = tmember[blockIdx.x];
  t = tindex[blockIdx.x];
}

// Pressure sweep j of a chunk (or the first sweep, j = 0) over all members.
template <int DIM, typename T, int MODE, bool LOCAL, int NT>
__global__ __launch_bounds__(NT) void batch_sweep_kernel(const Member *__restrict__ mem, const BCtl *__restrict__ ctl,
                                                         const int *__restrict__ tmember,
                                                         const int *__restrict__ tindex, double *__restrict__ partials,
                                                         int j) {
  int m, t;
  tile_of<NT>(tmember, tindex, m, t);
  const BCtl &bc = ctl[m];
  if (bc.done || bc.kbase + j > bc.kmax) return;
  const Member &M = mem[m];
  const KC &kc = M.kc;
  const int in = j & 1;
  const FP<T> fin = typed<T>(M.f[in]), fout = typed<T>(M.f[in ^ 1]);
  const float *Pb_in = M.Pb[bc.pb];
  float *Pb_out = M.Pb[bc.pb ^ 1];
  double acc[2] = {0.0, 0.0};
  if (LOCAL) {
    // initial state in local form: one node per thread, four passes
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = t * 4 * NT + i * NT + threadIdx.x;
      if (c < kc.ncell) {
        if constexpr (DIM == kD2Q9) {
          if (M.Fp) q9_sweep_cell<T, true, MODE, true>(kc, fin, fout, Pb_in, Pb_out, M.itau, M.Fp, c, acc);
          else q9_sweep_cell<T, true, MODE, false>(kc, fin, fout, Pb_in, Pb_out, M.itau, M.Fp, c, acc);
        } else {
          if (M.Fp) sweep_cell<DIM, T, true, MODE, true>(kc, fin, fout, Pb_in, Pb_out, M.itau, M.Fp, c, acc);
          else sweep_cell<DIM, T, true, MODE, false>(kc, fin, fout, Pb_in, Pb_out, M.itau, M.Fp, c, acc);
        }
      }
    }
  } else {
    const int qi = t * NT + threadIdx.x;
    if constexpr (DIM == kD2Q9) {
      if (M.Fp) q9_sweep_quad<T, MODE, true>(kc, fin, fout, Pb_in, Pb_out, M.itau, M.Fp, qi, acc);
      else q9_sweep_quad<T, MODE, false>(kc, fin, fout, Pb_in, Pb_out, M.itau, M.Fp, qi, acc);
    } else {
      if (M.Fp) sweep_quad<DIM, T, MODE, true>(kc, fin, fout, Pb_in, Pb_out, M.itau, M.Fp, qi, acc);
      else sweep_quad<DIM, T, MODE, false>(kc, fin, fout, Pb_in, Pb_out, M.itau, M.Fp, qi, acc);
    }
  }
  if (MODE == 2) block_sum<2, NT>(acc, partials);
}

// Plain sweeps j .. j + H - 1 of the members of one size class, blocked
// (block_region of lbtp_block.h, D2Q5, regions of W wavefronts x RW rows):
// one workgroup per (member, tile) of the class's blocked tiling.  Members
// with a pressure source run in the HAS_FP launch, the others in the plain
// one.
template <typename T, bool HAS_FP, int W, int RW>
__global__ __launch_bounds__(kBX * W) void batch_block_kernel(const Member *__restrict__ mem,
                                                              const BCtl *__restrict__ ctl,
                                                              const int *__restrict__ tmember,
                                                              const int *__restrict__ tindex, int j, int H) {
  const int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int m = tmember[b], t = tindex[b];
  const BCtl &bc = ctl[m];
  if (bc.done || bc.kbase + j > bc.kmax) return;
  const Member &M = mem[m];
  if ((M.Fp != nullptr) != HAS_FP) return;
  // the member's launch constants as a local copy: read once into scalar
  // registers instead of from memory inside the sweep loop
  const KC kc = M.kc;
  int tx, ty;
  block_tile_counts_rows(kc, H, W * RW, &tx, &ty);
  const int in = j & 1;
  block_region<T, HAS_FP, W, RW>(kc, typed<T>(M.f[in]), typed<T>(M.f[in ^ 1]), M.Pb[bc.pb], M.itau, M.Fp, H,
                                 t % tx, t / tx);
}

template <typename T, int W, int RW>
void batch_block_launch_shape(bool has_fp, int nblk, const Member *mem, const BCtl *ctl, const int *tm,
                              const int *ti, int j, int H, hipStream_t s) {
  if (has_fp)
    hipLaunchKernelGGL((batch_block_kernel<T, true, W, RW>), dim3(nblk), dim3(kBX * W), 0, s, mem, ctl, tm, ti, j, H);
  else
    hipLaunchKernelGGL((batch_block_kernel<T, false, W, RW>), dim3(nblk), dim3(kBX * W), 0, s, mem, ctl, tm, ti, j,
                       H);
}

template <typename T>
void batch_block_launch(int shape, bool has_fp, int nblk, const Member *mem, const BCtl *ctl, const int *tm,
                        const int *ti, int j, int H, hipStream_t s) {
  static_assert(batch_shape_rows(0) == kUseW * kUseRW && batch_shape_rows(4) == kUseW * kUseRWPlain,
                "shapes 0 and 4 are the single-context launch shapes");
  switch (shape) {
    case 4: batch_block_launch_shape<T, batch_shape_w(4), batch_shape_rw(4)>(has_fp, nblk, mem, ctl, tm, ti, j, H, s); break;
    case 1: batch_block_launch_shape<T, batch_shape_w(1), batch_shape_rw(1)>(has_fp, nblk, mem, ctl, tm, ti, j, H, s); break;
    case 2: batch_block_launch_shape<T, batch_shape_w(2), batch_shape_rw(2)>(has_fp, nblk, mem, ctl, tm, ti, j, H, s); break;
    case 3: batch_block_launch_shape<T, batch_shape_w(3), batch_shape_rw(3)>(has_fp, nblk, mem, ctl, tm, ti, j, H, s); break;
    default: batch_block_launch_shape<T, batch_shape_w(0), batch_shape_rw(0)>(has_fp, nblk, mem, ctl, tm, ti, j, H, s); break;
  }
}

// Stopping rule of every member (one block each) after the check sweep j = m of
// a chunk; advances the iteration base or stops the member.
__global__ __launch_bounds__(256) void batch_finish_kernel(const Member *__restrict__ mem, BCtl *ctl,
                                                           const double *__restrict__ partials, int m,
                                                           int *__restrict__ active) {
  __shared__ double sa[256], sb[256];
  const int mb = blockIdx.x;
  BCtl &bc = ctl[mb];
  const int t0 = mem[mb].tstart_s, nt = mem[mb].ntiles_s;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nt; i += 256) {
    a += partials[2 * (t0 + i)];
    b += partials[2 * (t0 + i) + 1];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (bc.done) return;
  const long long k = bc.kbase + m;
  if (k > bc.kmax) return;
  const double num = sqrt(sa[0]), den = sqrt(sb[0]);
  const double r = den > 0.0 ? num / ((double)m * den) : num / (double)m;
  bc.resid = r;
  if (!isfinite(r)) {
    bc.done = 1;
    bc.status = LBTP_EUNSTABLE;
    bc.K = k;
  } else if (r <= bc.tol) {
    bc.done = 1;
    bc.status = LBTP_OK;
    bc.K = k;
  } else if (k == bc.kmax) {
    bc.done = 1;
    bc.status = LBTP_NOT_CONVERGED;
    bc.K = k;
  } else {
    bc.pb ^= 1;          // the check sweep re-based into the other buffer
    bc.kbase = k;
  }
  if (!bc.done) atomicAdd(active, 1);
}

__global__ void batch_reset_kernel(BCtl *ctl, int n, long long kmax, double tol, int *active) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *active = 0;
  if (i >= n) return;
  ctl[i].done = 0;
  ctl[i].status = LBTP_OK;
  ctl[i].kbase = 0;
  ctl[i].kmax = kmax;
  ctl[i].K = 0;
  ctl[i].tol = tol;
  ctl[i].resid = -1.0;
}

// After the first sweep (which re-based every member), flip the base buffer.
__global__ void batch_flip_kernel(BCtl *ctl, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ctl[i].pb ^= 1;
}

__global__ void zero_int_kernel(int *p) { *p = 0; }

// Moments of every member (S, 1/tau_f, mass partials per tile).
template <int DIM, int NT, typename TG>
__global__ __launch_bounds__(NT) void batch_moments_kernel(const Member *__restrict__ mem,
                                                           const int *__restrict__ tmember,
                                                           const int *__restrict__ tindex,
                                                           double *__restrict__ partials, int gs, int write_coef) {
  int m, t;
  tile_of<NT>(tmember, tindex, m, t);
  const Member &M = mem[m];
  double acc[1] = {0.0};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = t * 4 * NT + i * NT + threadIdx.x;
    if (c < M.kc.ncell) {
      if constexpr (DIM == kD2Q9) {
        if (M.Fs) acc[0] += q9_moments_cell<true, TG>(M.kc, M.g[gs], M.K, M.phi, M.Fs, M.S, M.itau, c, write_coef);
        else acc[0] += q9_moments_cell<false, TG>(M.kc, M.g[gs], M.K, M.phi, M.Fs, M.S, M.itau, c, write_coef);
      } else {
        if (M.Fs) acc[0] += moments_cell<DIM, true, TG>(M.kc, M.g[gs], M.K, M.phi, M.Fs, M.S, M.itau, c, write_coef);
        else acc[0] += moments_cell<DIM, false, TG>(M.kc, M.g[gs], M.K, M.phi, M.Fs, M.S, M.itau, c, write_coef);
      }
    }
  }
  block_sum<1, NT>(acc, partials);
}

// Saturation step of every member; flux partials per tile.
template <int DIM, typename T, bool FLOCAL, int NT>
__global__ __launch_bounds__(NT) void batch_gsweep_kernel(const Member *__restrict__ mem, const BCtl *__restrict__ ctl,
                                                          const int *__restrict__ tmember,
                                                          const int *__restrict__ tindex,
                                                          double *__restrict__ partials, int gs) {
  int m, t;
  tile_of<NT>(tmember, tindex, m, t);
  const Member &M = mem[m];
  const FP<T> f = typed<T>(M.f[0]);
  const float *Pb = M.Pb[ctl[m].pb];
  double acc[1] = {0.0};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = t * 4 * NT + i * NT + threadIdx.x;
    if (c < M.kc.ncell) {
      if constexpr (DIM == kD2Q9) {
        if (M.Fs)
          acc[0] += q9_g_sweep_cell<T, FLOCAL, true>(M.kc, M.g[gs], M.g[gs ^ 1], f, Pb, M.itau, M.K, M.phi, M.Fs,
                                                     M.S, c);
        else
          acc[0] += q9_g_sweep_cell<T, FLOCAL, false>(M.kc, M.g[gs], M.g[gs ^ 1], f, Pb, M.itau, M.K, M.phi, M.Fs,
                                                      M.S, c);
      } else {
        if (M.Fs)
          acc[0] += g_sweep_cell<DIM, T, FLOCAL, true>(M.kc, M.g[gs], M.g[gs ^ 1], f, Pb, M.itau, M.K, M.phi, M.Fs,
                                                       M.S, c);
        else
          acc[0] += g_sweep_cell<DIM, T, FLOCAL, false>(M.kc, M.g[gs], M.g[gs ^ 1], f, Pb, M.itau, M.K, M.phi, M.Fs,
                                                        M.S, c);
      }
    }
  }
  block_sum<1, NT>(acc, partials);
}

// Per-member fixed-order sum of tile partials into the control block
// (mass: overwrite; ledger: accumulate).
__global__ __launch_bounds__(256) void batch_sum_kernel(const Member *__restrict__ mem, BCtl *ctl,
                                                        const double *__restrict__ partials, int ledger) {
  __shared__ double sa[256];
  const int mb = blockIdx.x;
  const int t0 = mem[mb].tstart_c, nt = mem[mb].ntiles_c;
  double a = 0.0;
  for (int i = threadIdx.x; i < nt; i += 256) a += partials[t0 + i];
  sa[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sa[threadIdx.x] += sa[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (ledger) ctl[mb].ledger += sa[0];
    else ctl[mb].mass = sa[0];
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers
template <int DIM, typename T, int NT>
static void sweep_launch(int mode, int local, int nblk, const Member *mem, const BCtl *ctl, const int *tm,
                         const int *ti, double *part, int j, hipStream_t s) {
  const dim3 g(nblk), b(NT);
  if (local) {
    if (mode == 1) hipLaunchKernelGGL((batch_sweep_kernel<DIM, T, 1, true, NT>), g, b, 0, s, mem, ctl, tm, ti, part, j);
    else if (mode == 2) hipLaunchKernelGGL((batch_sweep_kernel<DIM, T, 2, true, NT>), g, b, 0, s, mem, ctl, tm, ti, part, j);
    else hipLaunchKernelGGL((batch_sweep_kernel<DIM, T, 0, true, NT>), g, b, 0, s, mem, ctl, tm, ti, part, j);
  } else {
    if (mode == 1) hipLaunchKernelGGL((batch_sweep_kernel<DIM, T, 1, false, NT>), g, b, 0, s, mem, ctl, tm, ti, part, j);
    else if (mode == 2) hipLaunchKernelGGL((batch_sweep_kernel<DIM, T, 2, false, NT>), g, b, 0, s, mem, ctl, tm, ti, part, j);
    else hipLaunchKernelGGL((batch_sweep_kernel<DIM, T, 0, false, NT>), g, b, 0, s, mem, ctl, tm, ti, part, j);
  }
}

template <int DIM, int NT>
static void sweep_by_storage(int storage, int mode, int local, int nblk, const Member *mem, const BCtl *ctl,
                             const int *tm, const int *ti, double *part, int j, hipStream_t s) {
  if (storage == LBTP_FP16_DEV) sweep_launch<DIM, _Float16, NT>(mode, local, nblk, mem, ctl, tm, ti, part, j, s);
  else if (storage == LBTP_BF16_DEV) sweep_launch<DIM, bf16_t, NT>(mode, local, nblk, mem, ctl, tm, ti, part, j, s);
  else sweep_launch<DIM, float, NT>(mode, local, nblk, mem, ctl, tm, ti, part, j, s);
}

template <int NT>
static void sweep_by_dim(int dim, int storage, int mode, int local, int nblk, const Member *mem, const BCtl *ctl,
                         const int *tm, const int *ti, double *part, int j, hipStream_t s) {
  if (dim == 2) sweep_by_storage<2, NT>(storage, mode, local, nblk, mem, ctl, tm, ti, part, j, s);
  else if (dim == 3) sweep_by_storage<3, NT>(storage, mode, local, nblk, mem, ctl, tm, ti, part, j, s);
  else sweep_by_storage<kD2Q9, NT>(storage, mode, local, nblk, mem, ctl, tm, ti, part, j, s);
}

hipError_t batch_launch_sweep(int nt, int dim, int storage, int mode, int local, int nblk, const Member *mem,
                              const BCtl *ctl, const int *tm, const int *ti, double *part, int j, hipStream_t s) {
  switch (nt) {
    case 64: sweep_by_dim<64>(dim, storage, mode, local, nblk, mem, ctl, tm, ti, part, j, s); break;
    case 128: sweep_by_dim<128>(dim, storage, mode, local, nblk, mem, ctl, tm, ti, part, j, s); break;
    case 512: sweep_by_dim<512>(dim, storage, mode, local, nblk, mem, ctl, tm, ti, part, j, s); break;
    default: sweep_by_dim<256>(dim, storage, mode, local, nblk, mem, ctl, tm, ti, part, j, s); break;
  }
  return hipGetLastError();
}

template <int DIM, int NT, typename TG>
static void moments_launch(int nblk, const Member *mem, const int *tm, const int *ti, double *part, int gs,
                           int write_coef, hipStream_t s) {
  hipLaunchKernelGGL((batch_moments_kernel<DIM, NT, TG>), dim3(nblk), dim3(NT), 0, s, mem, tm, ti, part, gs,
                     write_coef);
}

template <int DIM>
static void moments_by_storage(int storage, int nblk, const Member *mem, const int *tm, const int *ti, double *part,
                               int gs, int write_coef, hipStream_t s) {
  if (storage == LBTP_FP16_DEV) moments_launch<DIM, 256, _Float16>(nblk, mem, tm, ti, part, gs, write_coef, s);
  else if (storage == LBTP_BF16_DEV) moments_launch<DIM, 256, bf16_t>(nblk, mem, tm, ti, part, gs, write_coef, s);
  else moments_launch<DIM, 256, float>(nblk, mem, tm, ti, part, gs, write_coef, s);
}

hipError_t batch_launch_block(int storage, int shape, bool has_fp, int nblk, const Member *mem, const BCtl *ctl,
                              const int *tm, const int *ti, int j, int H, hipStream_t s) {
  switch (storage) {
    case LBTP_FP16_DEV: batch_block_launch<_Float16>(shape, has_fp, nblk, mem, ctl, tm, ti, j, H, s); break;
    case LBTP_BF16_DEV: batch_block_launch<bf16_t>(shape, has_fp, nblk, mem, ctl, tm, ti, j, H, s); break;
    default: batch_block_launch<float>(shape, has_fp, nblk, mem, ctl, tm, ti, j, H, s); break;
  }
  return hipGetLastError();
}

hipError_t batch_launch_moments(int dim, int storage, int nblk, const Member *mem, const int *tm, const int *ti,
                                double *part, int gs, int write_coef, hipStream_t s) {
  // moments and the saturation step use tiles of kCellTile nodes (256 threads x 4)
  if (dim == 2) moments_by_storage<2>(storage, nblk, mem, tm, ti, part, gs, write_coef, s);
  else if (dim == 3) moments_by_storage<3>(storage, nblk, mem, tm, ti, part, gs, write_coef, s);
  else moments_by_storage<kD2Q9>(storage, nblk, mem, tm, ti, part, gs, write_coef, s);
  return hipGetLastError();
}

template <int DIM, typename T>
static void gsweep_launch(int local, int nblk, const Member *mem, const BCtl *ctl, const int *tm, const int *ti,
                          double *part, int gs, hipStream_t s) {
  if (local)
    hipLaunchKernelGGL((batch_gsweep_kernel<DIM, T, true, 256>), dim3(nblk), dim3(256), 0, s, mem, ctl, tm, ti, part, gs);
  else
    hipLaunchKernelGGL((batch_gsweep_kernel<DIM, T, false, 256>), dim3(nblk), dim3(256), 0, s, mem, ctl, tm, ti, part, gs);
}

hipError_t batch_launch_gsweep(int dim, int storage, int local, int nblk, const Member *mem, const BCtl *ctl,
                               const int *tm, const int *ti, double *part, int gs, hipStream_t s) {
  if (dim == 2) {
    if (storage == LBTP_FP16_DEV) gsweep_launch<2, _Float16>(local, nblk, mem, ctl, tm, ti, part, gs, s);
    else if (storage == LBTP_BF16_DEV) gsweep_launch<2, bf16_t>(local, nblk, mem, ctl, tm, ti, part, gs, s);
    else gsweep_launch<2, float>(local, nblk, mem, ctl, tm, ti, part, gs, s);
  } else if (dim == 3) {
    if (storage == LBTP_FP16_DEV) gsweep_launch<3, _Float16>(local, nblk, mem, ctl, tm, ti, part, gs, s);
    else if (storage == LBTP_BF16_DEV) gsweep_launch<3, bf16_t>(local, nblk, mem, ctl, tm, ti, part, gs, s);
    else gsweep_launch<3, float>(local, nblk, mem, ctl, tm, ti, part, gs, s);
  } else {
    if (storage == LBTP_FP16_DEV) gsweep_launch<kD2Q9, _Float16>(local, nblk, mem, ctl, tm, ti, part, gs, s);
    else if (storage == LBTP_BF16_DEV) gsweep_launch<kD2Q9, bf16_t>(local, nblk, mem, ctl, tm, ti, part, gs, s);
    else gsweep_launch<kD2Q9, float>(local, nblk, mem, ctl, tm, ti, part, gs, s);
  }
  return hipGetLastError();
}

hipError_t batch_launch_finish(int n, const Member *mem, BCtl *ctl, const double *part, int m, int *active,
                               hipStream_t s) {
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, active);
  hipLaunchKernelGGL(batch_finish_kernel, dim3(n), dim3(256), 0, s, mem, ctl, part, m, active);
  return hipGetLastError();
}

hipError_t batch_launch_reset(int n, BCtl *ctl, long long kmax, double tol, int *active, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ctl, n, kmax, tol, active);
  return hipGetLastError();
}

hipError_t batch_launch_flip(int n, BCtl *ctl, hipStream_t s) {
  hipLaunchKernelGGL(batch_flip_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ctl, n);
  return hipGetLastError();
}

hipError_t batch_launch_sum(int n, const Member *mem, BCtl *ctl, const double *part, int ledger, hipStream_t s) {
  hipLaunchKernelGGL(batch_sum_kernel, dim3(n), dim3(256), 0, s, mem, ctl, part, ledger);
  return hipGetLastError();
}

}  // namespace lbtp
