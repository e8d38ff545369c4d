// HIP kernels (gfx950) of the double-distribution lattice Boltzmann model
// (Chai, Liang, Du, Shi, arXiv:1808.07554) on D2Q5 / D3Q7.
//
// Data layout: structure of arrays, one array per population and per scalar
// field, x fastest (index = x + nx*(y + ny*z)).
//
// Pressure lattice.  Populations are kept as deviations from a per-node base
// equilibrium, d_i(x) = f_i(x) - w_i P_b(x), stored as float, fp16 or bf16
// (type T) in a two-buffer ping-pong in "pull" form: the buffer holds the
// post-collision deviations of the previous sweep, and a sweep at node y
// reads d_i(y - c_i) (streaming, eq. 3-1), re-expressed against its own
// base:  e_i(y) = f_i(y) - w_i P_b(y) = d_i(y - c_i) + w_i (P_b(y - c_i) - P_b(y)).
// Where y - c_i lies beyond a wall the Section 4 rules apply:
//   anti-bounce-back f_i = -f_opp^+ + 2 w P_w  ->  e_i = -d_opp(y) + 2 w (P_w - P_b(y)),
//   bounce-back      f_i =  f_opp^+            ->  e_i =  d_opp(y).
// With w_0 + sum_{i>=1} w_i = 1 the moment eq. 3-9a becomes
// P - P_b = sum_i e_i / (1 - w_0), and the BGK collision (eq. 2-1b a) acts on
// the deviations unchanged: e_i^+ = e_i + (w_i (P - P_b) - e_i) / tau_f.
// Every quantity the sweep rounds is therefore of the size of the
// non-equilibrium part, not of P.  The base is reset to the current P at the
// first sweep of a solve and at every residual check (re-basing shifts the
// stored deviations by w (P_b,old - P_b,new), an exact difference), so the
// stopping-rule numerator P^k - P^{k-m} is the deviation itself.
// Right after initialisation the buffer holds pre-collision deviations read
// in place ("local" form).  The rest population of f never affects an output
// and is not stored.
//
// Saturation lattice: float pre-collision g, pushed to x + c_i after the
// collision (eq. 3-2).
//
// Cell kernels run one thread per node, kThreads per block; reductions are
// float64, per wavefront (shuffles), per block (LDS), then over blocks in a
// fixed order by a single-block kernel, so every result is deterministic.
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "lbtp_device.h"

namespace lbtp {
namespace {

// ------------------------------------------------------------- pressure sweep
// One iteration of eq. 3-1: stream, P (eq. 3-9a), BGK collision with the local
// 1/tau_f (eq. 2-1b a) and the source dt wbar_i F_p, store at node y.
// MODE 0: plain; 1: also reset the base to P (first sweep of a solve);
// 2: reset the base and accumulate sum (P - P_b)^2 and sum P^2 (stopping rule);
// 3: a probe, which only accumulates those sums and writes nothing else.
template <int DIM, typename T, bool LOCAL, int MODE, bool HAS_FP>
__global__ __launch_bounds__(kThreads) void f_sweep_kernel(KC kc, FPtrs fin_, FPtrs fout_,
                                                           const float *__restrict__ Pb_in,
                                                           float *__restrict__ Pb_out,
                                                           const float *__restrict__ itau,
                                                           const float *__restrict__ Fp,
                                                           double *__restrict__ partials,
                                                           const Ctl *__restrict__ ctl, long long k) {
  // a converged (or finished) solve turns the remaining queued sweeps into no-ops
  if (ctl->done || k > ctl->kmax) return;
  const int c = blockIdx.x * kThreads + threadIdx.x;
  double acc[2] = {0.0, 0.0};
  if (c < kc.ncell)
    sweep_cell<DIM, T, LOCAL, MODE, HAS_FP>(kc, typed<T>(fin_), typed<T>(fout_), Pb_in, Pb_out, itau, Fp, c, acc);
  if (MODE >= 2) block_sum<2>(acc, partials);
}

template <int DIM, typename T, int MODE, bool HAS_FP>
__global__ __launch_bounds__(kThreads) void f_sweep_vec_kernel(KC kc, FPtrs fin_, FPtrs fout_,
                                                               const float *__restrict__ Pb_in,
                                                               float *__restrict__ Pb_out,
                                                               const float *__restrict__ itau,
                                                               const float *__restrict__ Fp,
                                                               double *__restrict__ partials,
                                                               const Ctl *__restrict__ ctl, long long k) {
  if (ctl->done || k > ctl->kmax) return;
  double acc[2] = {0.0, 0.0};
  sweep_quad<DIM, T, MODE, HAS_FP>(kc, typed<T>(fin_), typed<T>(fout_), Pb_in, Pb_out, itau, Fp,
                                   blockIdx.x * kThreads + threadIdx.x, acc);
  if (MODE >= 2) block_sum<2>(acc, partials);
}

// Stopping rule r = ||P^k - P^{k-m}|| / (m ||P^k||) from the block partials.
__global__ __launch_bounds__(1024) void finish_residual_kernel(const double *__restrict__ partials,
                                                               int nblk, Ctl *ctl, int m) {
  __shared__ double sa[1024], sb[1024];
  double a = 0.0, b = 0.0;
  int i = threadIdx.x;
  // eight partials in flight, added in the same order as one at a time
  for (; i + 7 * 1024 < nblk; i += 8 * 1024) {
    double va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      va[u] = partials[2 * (i + 1024 * u)];
      vb[u] = partials[2 * (i + 1024 * u) + 1];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a += va[u];
      b += vb[u];
    }
  }
  for (; i < nblk; i += 1024) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (ctl->done) return;
    const long long k = ctl->kcheck + m;     // the iteration this check follows
    ctl->kcheck = k;
    if (k > ctl->kmax) return;
    const double num = sqrt(sa[0]), den = sqrt(sb[0]);
    const double r = den > 0.0 ? num / ((double)m * den) : num / (double)m;
    ctl->resid = r;
    ctl->last_check = k;
    if (!isfinite(r)) {
      ctl->done = 1;
      ctl->status = LBTP_EUNSTABLE;
      ctl->K = k;
    } else if (r <= ctl->tol) {
      ctl->done = 1;
      ctl->status = LBTP_OK;
      ctl->K = k;
    }
  }
}

__global__ void ctl_reset_kernel(Ctl *ctl, long long kmax, double tol) {
  ctl->kcheck = 0;
  ctl->done = 0;
  ctl->status = LBTP_OK;
  ctl->K = -1;
  ctl->kmax = kmax;
  ctl->tol = tol;
  ctl->resid = -1.0;
  ctl->last_check = -1;
}

// Fixed-order sum of nblk partials into *dst (or += when accumulate).
__global__ __launch_bounds__(1024) void finish_sum_kernel(const double *__restrict__ partials, int nblk,
                                                          double *dst, int accumulate, double *copy_to) {
  __shared__ double sa[1024];
  double a = 0.0;
  int i = threadIdx.x;
  // eight partials in flight, added in the same order as one at a time
  for (; i + 7 * 1024 < nblk; i += 8 * 1024) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = partials[i + 1024 * u];
#pragma unroll
    for (int u = 0; u < 8; ++u) a += v[u];
  }
  for (; i < nblk; i += 1024) a += partials[i];
  sa[threadIdx.x] = a;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) sa[threadIdx.x] += sa[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (copy_to) *copy_to = sa[0];
    *dst = accumulate ? (*dst + sa[0]) : sa[0];
  }
}

// ------------------------------------------------------------------ moments
// S^n (eq. 3-9b) and 1/tau_f (eq. 3-11a, 2-9, 2-16) of the coupled step, and
// the block partials of the mass sum_x (sum_i g_i + dt F_s / 2) = sum phi S.
template <int DIM, bool HAS_FS, typename TG>
__global__ __launch_bounds__(kThreads) void moments_kernel(KC kc, GPtrs g, const float *__restrict__ K,
                                                           const float *__restrict__ phi,
                                                           const float *__restrict__ Fs, float *__restrict__ S,
                                                           float *__restrict__ itau,
                                                           double *__restrict__ partials, int write_coef) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  double acc[1] = {0.0};
  if (c < kc.ncell) acc[0] = moments_cell<DIM, HAS_FS, TG>(kc, g, K, phi, Fs, S, itau, c, write_coef);
  block_sum<1>(acc, partials);
}

// ---------------------------------------------------------- saturation sweep
// One step of eq. 3-2 with g^eq of eq. 3-4b, the local grad P of eq. 3-10a
// (from the pressure lattice, read as in the pressure sweep) and
// gamma = -lambda_w K / (c_s^2 dt) (eq. 3-8); post-collision values are
// pushed to x + c_i, or reflected at walls (Section 4).  Block partials of
// the net flux through reflected links.
template <int DIM, typename T, bool FLOCAL, bool HAS_FS>
__global__ __launch_bounds__(kThreads) void g_sweep_kernel(KC kc, GPtrs gin, GPtrs gout, FPtrs f_,
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
    acc[0] = g_sweep_cell<DIM, T, FLOCAL, HAS_FS>(kc, gin, gout, typed<T>(f_), Pb, itau, K, phi, Fs, Sn, c);
  block_sum<1>(acc, partials);
}

// The D2Q5 saturation step four nodes per thread (pull form, nx % 4 == 0).
template <typename T, bool HAS_FS>
__global__ __launch_bounds__(kThreads) void g_sweep_quad_kernel(KC kc, GPtrs gin, GPtrs gout, FPtrs f_,
                                                                const float *__restrict__ Pb,
                                                                const float *__restrict__ itau,
                                                                const float *__restrict__ K,
                                                                const float *__restrict__ phi,
                                                                const float *__restrict__ Fs,
                                                                const float *__restrict__ Sn,
                                                                double *__restrict__ partials) {
  double acc[1] = {g_sweep_quad<T, HAS_FS>(kc, gin, gout, typed<T>(f_), Pb, itau, K, phi, Fs, Sn,
                                           blockIdx.x * kThreads + threadIdx.x)};
  block_sum<1>(acc, partials);
}

template <int DIM, typename T>
__global__ __launch_bounds__(kThreads) void init_kernel(KC kc, const float *__restrict__ P0,
                                                        const float *__restrict__ S0,
                                                        const float *__restrict__ dP0,
                                                        const float *__restrict__ dS0,
                                                        const float *__restrict__ K,
                                                        const float *__restrict__ phi,
                                                        const float *__restrict__ Fs, int neq, FPtrs f_,
                                                        float *__restrict__ Pb, GPtrs g) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c < kc.ncell) init_cell<DIM, T>(kc, P0, S0, dP0, dS0, K, phi, Fs, neq, typed<T>(f_), Pb, g, c);
}

// ----------------------------------------------------------------- outputs
template <int DIM, typename T, bool LOCAL>
__global__ __launch_bounds__(kThreads) void pressure_kernel(KC kc, FPtrs f_, const float *__restrict__ Pb,
                                                            float *__restrict__ P) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const Cell q = cell_of(c, kc);
  const float pb = Pb[c];
  float e[2 * DIM];
  load_e<DIM, T, LOCAL>(typed<T>(f_), Pb, q, kc, pb, e);
  P[c] = pb + dpressure<DIM>(e, kc);
}

// grad P (eq. 3-10a) or u = -K lambda_t grad P (eq. 3-10b), component-major.
template <int DIM, typename T, bool LOCAL>
__global__ __launch_bounds__(kThreads) void grad_kernel(KC kc, FPtrs f_, const float *__restrict__ Pb,
                                                        const float *__restrict__ itau,
                                                        const float *__restrict__ K,
                                                        const float *__restrict__ S, int velocity,
                                                        float *__restrict__ out) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const Cell q = cell_of(c, kc);
  float e[2 * DIM];
  load_e<DIM, T, LOCAL>(typed<T>(f_), Pb, q, kc, Pb[c], e);
  float m1[3];
  moment_c<DIM>(e, kc, m1);
  float scale = -itau[c] * kc.inv_cs2dt;
  if (velocity) scale = -dp_of(S[c], K[c], kc) * scale;   // u = -D_p grad P
#pragma unroll
  for (int a = 0; a < DIM; ++a) out[a * kc.ncell + c] = scale * m1[a];
}

template <int DIM, bool HAS_FS, typename TG>
__global__ __launch_bounds__(kThreads) void saturation_kernel(KC kc, GPtrs g_, const float *__restrict__ phi,
                                                              const float *__restrict__ Fs,
                                                              float *__restrict__ S) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const GP<TG> g = gtyped<TG>(g_);
  const float ph = phi[c], B = gdev<TG>() ? g.B[c] : 0.0f;
  float gv[2 * DIM + 1];
#pragma unroll
  for (int i = 0; i <= 2 * DIM; ++i) gv[i] = gload(g.p[i], c, gdev<TG>() ? geq_odd(kc, i, B, ph) : 0.0f, kc);
  S[c] = saturation_of(sum_g<DIM>(gv), HAS_FS ? Fs[c] : 0.0f, ph, kc);
}

// The saturation populations as float32 (component-major), reconstructed
// from 16-bit deviations where they are stored so.
template <int DIM, typename TG>
__global__ __launch_bounds__(kThreads) void gpop_kernel(KC kc, GPtrs g_, const float *__restrict__ phi,
                                                        float *__restrict__ out) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const GP<TG> g = gtyped<TG>(g_);
  const float ph = phi[c], B = gdev<TG>() ? g.B[c] : 0.0f;
#pragma unroll
  for (int i = 0; i <= 2 * DIM; ++i)
    out[(size_t)i * kc.ncell + c] = gload(g.p[i], c, gdev<TG>() ? geq_odd(kc, i, B, ph) : 0.0f, kc);
}

// Phase velocities (eq. 2-12, 2-13) from the total velocity u (component-
// major, dim x ncell) and S^n: with the constant D_s of the model,
// D_s = -K lambda_n f_w P_c' (eq. 2-16) turns K lambda_n grad P_c into
// -(D_s / f_w) grad S, so u_w = f_w u - D_s grad S, u_n = f_n u + D_s grad S,
// f_w = lambda_w K / D_p (eq. 2-10); grad S by second-order central
// differences (one-sided at walls).
__global__ __launch_bounds__(kThreads) void phase_kernel(KC kc, int dim, const float *__restrict__ u,
                                                         const float *__restrict__ S, const float *__restrict__ K,
                                                         float Ds, float *__restrict__ uw, float *__restrict__ un) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const Cell q = cell_of(c, kc);
  const float Sv = S[c], Kv = K[c];
  const float fw = lwk_of(Sv, Kv, kc) / dp_of(Sv, Kv, kc);
  const float inv2dx = 0.5f / (kc.c * kc.dt);
  for (int a = 0; a < dim; ++a) {
    const float gs = cdiff(S, q, a, kc, inv2dx);
    const float ua = u[a * kc.ncell + c];
    uw[a * kc.ncell + c] = fw * ua - Ds * gs;
    un[a * kc.ncell + c] = (1.0f - fw) * ua + Ds * gs;
  }
}

// Pre-collision populations f_i = w_i P_b + e_i (float) for inspection.
template <int DIM, typename T, bool LOCAL>
__global__ __launch_bounds__(kThreads) void populations_kernel(KC kc, FPtrs f_, const float *__restrict__ Pb,
                                                               float *__restrict__ out) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const Cell q = cell_of(c, kc);
  const float pb = Pb[c];
  float e[2 * DIM];
  load_e<DIM, T, LOCAL>(typed<T>(f_), Pb, q, kc, pb, e);
#pragma unroll
  for (int j = 0; j < 2 * DIM; ++j) out[j * kc.ncell + c] = kc.w1 * pb + e[j];
}

// Plain copy of n4 16-byte words: the known-size reference that calibrates
// the HBM byte counters (FETCH_SIZE / WRITE_SIZE) of the sweep kernels.
__global__ __launch_bounds__(kThreads) void copy_probe_kernel(const float4 *__restrict__ src,
                                                              float4 *__restrict__ dst, long long n4) {
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n4; i += (long long)gridDim.x * kThreads)
    dst[i] = src[i];
}

}  // namespace

// ---------------------------------------------------------------- launchers
#define LBTP_GRID(kc) dim3(nblocks((kc).ncell)), dim3(kThreads), 0, s

// Dispatch on lattice (2-D / 3-D), storage type and the local flag.
template <template <int, typename, bool> class Fn, typename... A>
static void dispatch(int dim, int storage, int local, A &&...args) {
  auto go = [&](auto d, auto t) {
    constexpr int D = decltype(d)::value;
    using T = typename decltype(t)::type;
    if (local) Fn<D, T, true>::run(args...);
    else Fn<D, T, false>::run(args...);
  };
  struct F32 { using type = float; };
  struct F16 { using type = _Float16; };
  struct B16 { using type = bf16_t; };
  using D2 = std::integral_constant<int, 2>;
  using D3 = std::integral_constant<int, 3>;
  if (dim == 2) {
    if (storage == LBTP_FP16_DEV) go(D2{}, F16{});
    else if (storage == LBTP_BF16_DEV) go(D2{}, B16{});
    else go(D2{}, F32{});
  } else {
    if (storage == LBTP_FP16_DEV) go(D3{}, F16{});
    else if (storage == LBTP_BF16_DEV) go(D3{}, B16{});
    else go(D3{}, F32{});
  }
}

template <int DIM, typename T, bool LOCAL>
struct SweepLaunch {
  static void run(const KC &kc, FPtrs fin, FPtrs fout, const float *Pb_in, float *Pb_out, const float *itau,
                  const float *Fp, double *partials, const Ctl *ctl, long long k, int mode, hipStream_t s) {
#define LBTP_SWEEP(M, HF)                                                                                     \
  do {                                                                                                        \
    if (!LOCAL && kc.nx % 4 == 0)                                                                             \
      hipLaunchKernelGGL((f_sweep_vec_kernel<DIM, T, M, HF>), dim3(nblocks(kc.ncell / 4)), dim3(kThreads), 0, \
                         s, kc, fin, fout, Pb_in, Pb_out, itau, Fp, partials, ctl, k);                        \
    else                                                                                                      \
      hipLaunchKernelGGL((f_sweep_kernel<DIM, T, LOCAL, M, HF>), LBTP_GRID(kc), kc, fin, fout, Pb_in, Pb_out,  \
                         itau, Fp, partials, ctl, k);                                                         \
  } while (0)
    if (mode == 3) {
      LBTP_SWEEP(3, false);   // P does not depend on the source
    } else if (Fp) {
      if (mode == 0) LBTP_SWEEP(0, true);
      else if (mode == 1) LBTP_SWEEP(1, true);
      else LBTP_SWEEP(2, true);
    } else {
      if (mode == 0) LBTP_SWEEP(0, false);
      else if (mode == 1) LBTP_SWEEP(1, false);
      else LBTP_SWEEP(2, false);
    }
#undef LBTP_SWEEP
  }
};

hipError_t launch_f_sweep(int dim, int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb_in,
                          float *Pb_out, const float *itau, const float *Fp, double *partials, const Ctl *ctl,
                          long long k, int local, int mode, hipStream_t s) {
  if (dim == kD2Q9)
    return launch_f_sweep_q9(storage, kc, fin, fout, Pb_in, Pb_out, itau, Fp, partials, ctl, k, local, mode, s);
  dispatch<SweepLaunch>(dim, storage, local, kc, fin, fout, Pb_in, Pb_out, itau, Fp, partials, ctl, k, mode, s);
  return hipGetLastError();
}

hipError_t launch_finish_residual(const double *partials, int nblk, Ctl *ctl, int m, hipStream_t s) {
  hipLaunchKernelGGL(finish_residual_kernel, dim3(1), dim3(1024), 0, s, partials, nblk, ctl, m);
  return hipGetLastError();
}

hipError_t launch_ctl_reset(Ctl *ctl, long long kmax, double tol, hipStream_t s) {
  hipLaunchKernelGGL(ctl_reset_kernel, dim3(1), dim3(1), 0, s, ctl, kmax, tol);
  return hipGetLastError();
}

hipError_t launch_finish_sum(const double *partials, int nblk, double *dst, int accumulate, double *copy_to,
                             hipStream_t s) {
  hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(1024), 0, s, partials, nblk, dst, accumulate, copy_to);
  return hipGetLastError();
}

template <int DIM, typename TG, bool LOCAL_UNUSED>
struct MomentsLaunch {
  static void run(const KC &kc, GPtrs g, const float *K, const float *phi, const float *Fs, float *S, float *itau,
                  double *partials, int write_coef, hipStream_t s) {
    if (Fs)
      hipLaunchKernelGGL((moments_kernel<DIM, true, TG>), LBTP_GRID(kc), kc, g, K, phi, Fs, S, itau, partials,
                         write_coef);
    else
      hipLaunchKernelGGL((moments_kernel<DIM, false, TG>), LBTP_GRID(kc), kc, g, K, phi, Fs, S, itau, partials,
                         write_coef);
  }
};

hipError_t launch_moments(int dim, const KC &kc, GPtrs g, const float *K, const float *phi, const float *Fs,
                          float *S, float *itau, double *partials, int write_coef, hipStream_t s) {
  if (dim == kD2Q9) return launch_moments_q9(kc, g, K, phi, Fs, S, itau, partials, write_coef, s);
  dispatch<MomentsLaunch>(dim, g.storage, 0, kc, g, K, phi, Fs, S, itau, partials, write_coef, s);
  return hipGetLastError();
}

template <int DIM, typename T, bool LOCAL>
struct GSweepLaunch {
  static void run(const KC &kc, GPtrs gin, GPtrs gout, FPtrs f, const float *Pb, const float *itau, const float *K,
                  const float *phi, const float *Fs, const float *Sn, double *partials, hipStream_t s) {
    if (g_sweep_quads(DIM, kc, LOCAL)) {
      const dim3 grid(nblocks(kc.ncell / 4)), block(kThreads);
      if (Fs)
        hipLaunchKernelGGL((g_sweep_quad_kernel<T, true>), grid, block, 0, s, kc, gin, gout, f, Pb, itau, K, phi,
                           Fs, Sn, partials);
      else
        hipLaunchKernelGGL((g_sweep_quad_kernel<T, false>), grid, block, 0, s, kc, gin, gout, f, Pb, itau, K, phi,
                           Fs, Sn, partials);
      return;
    }
    if (Fs)
      hipLaunchKernelGGL((g_sweep_kernel<DIM, T, LOCAL, true>), LBTP_GRID(kc), kc, gin, gout, f, Pb, itau, K, phi,
                         Fs, Sn, partials);
    else
      hipLaunchKernelGGL((g_sweep_kernel<DIM, T, LOCAL, false>), LBTP_GRID(kc), kc, gin, gout, f, Pb, itau, K, phi,
                         Fs, Sn, partials);
  }
};

hipError_t launch_g_sweep(int dim, int storage, const KC &kc, GPtrs gin, GPtrs gout, FPtrs f, int f_local,
                          const float *Pb, const float *itau, const float *K, const float *phi, const float *Fs,
                          const float *Sn, double *partials, hipStream_t s) {
  if (dim == kD2Q9)
    return launch_g_sweep_q9(storage, kc, gin, gout, f, f_local, Pb, itau, K, phi, Fs, Sn, partials, s);
  dispatch<GSweepLaunch>(dim, storage, f_local, kc, gin, gout, f, Pb, itau, K, phi, Fs, Sn, partials, s);
  return hipGetLastError();
}

template <int DIM, typename T, bool LOCAL_UNUSED>
struct InitLaunch {
  static void run(const KC &kc, const float *P0, const float *S0, const float *dP0, const float *dS0,
                  const float *K, const float *phi, const float *Fs, int neq, FPtrs f, float *Pb, GPtrs g,
                  hipStream_t s) {
    hipLaunchKernelGGL((init_kernel<DIM, T>), LBTP_GRID(kc), kc, P0, S0, dP0, dS0, K, phi, Fs, neq, f, Pb, g);
  }
};

hipError_t launch_init(int dim, int storage, const KC &kc, const float *P0, const float *S0, const float *dP0,
                       const float *dS0, const float *K, const float *phi, const float *Fs, int neq, FPtrs f,
                       float *Pb, GPtrs g, hipStream_t s) {
  if (dim == kD2Q9) return launch_init_q9(storage, kc, P0, S0, dP0, dS0, K, phi, Fs, neq, f, Pb, g, s);
  dispatch<InitLaunch>(dim, storage, 0, kc, P0, S0, dP0, dS0, K, phi, Fs, neq, f, Pb, g, s);
  return hipGetLastError();
}

template <int DIM, typename T, bool LOCAL>
struct PressureLaunch {
  static void run(const KC &kc, FPtrs f, const float *Pb, float *P, hipStream_t s) {
    hipLaunchKernelGGL((pressure_kernel<DIM, T, LOCAL>), LBTP_GRID(kc), kc, f, Pb, P);
  }
};

hipError_t launch_pressure(int dim, int storage, const KC &kc, FPtrs f, int f_local, const float *Pb, float *P,
                           hipStream_t s) {
  if (dim == kD2Q9) return launch_pressure_q9(storage, kc, f, f_local, Pb, P, s);
  dispatch<PressureLaunch>(dim, storage, f_local, kc, f, Pb, P, s);
  return hipGetLastError();
}

template <int DIM, typename T, bool LOCAL>
struct GradLaunch {
  static void run(const KC &kc, FPtrs f, const float *Pb, const float *itau, const float *K, const float *S,
                  int velocity, float *out, hipStream_t s) {
    hipLaunchKernelGGL((grad_kernel<DIM, T, LOCAL>), LBTP_GRID(kc), kc, f, Pb, itau, K, S, velocity, out);
  }
};

hipError_t launch_grad(int dim, int storage, const KC &kc, FPtrs f, int f_local, const float *Pb,
                       const float *itau, const float *K, const float *S, int velocity, float *out, hipStream_t s) {
  if (dim == kD2Q9) return launch_grad_q9(storage, kc, f, f_local, Pb, itau, K, S, velocity, out, s);
  dispatch<GradLaunch>(dim, storage, f_local, kc, f, Pb, itau, K, S, velocity, out, s);
  return hipGetLastError();
}

template <int DIM, typename TG, bool LOCAL_UNUSED>
struct SaturationLaunch {
  static void run(const KC &kc, GPtrs g, const float *phi, const float *Fs, float *S, hipStream_t s) {
    if (Fs) hipLaunchKernelGGL((saturation_kernel<DIM, true, TG>), LBTP_GRID(kc), kc, g, phi, Fs, S);
    else hipLaunchKernelGGL((saturation_kernel<DIM, false, TG>), LBTP_GRID(kc), kc, g, phi, Fs, S);
  }
};

hipError_t launch_saturation(int dim, const KC &kc, GPtrs g, const float *phi, const float *Fs, float *S,
                             hipStream_t s) {
  if (dim == kD2Q9) return launch_saturation_q9(kc, g, phi, Fs, S, s);
  dispatch<SaturationLaunch>(dim, g.storage, 0, kc, g, phi, Fs, S, s);
  return hipGetLastError();
}

template <int DIM, typename TG, bool LOCAL_UNUSED>
struct GPopLaunch {
  static void run(const KC &kc, GPtrs g, const float *phi, float *out, hipStream_t s) {
    hipLaunchKernelGGL((gpop_kernel<DIM, TG>), LBTP_GRID(kc), kc, g, phi, out);
  }
};

hipError_t launch_g_populations(int dim, const KC &kc, GPtrs g, const float *phi, float *out, hipStream_t s) {
  if (dim == kD2Q9) return launch_g_populations_q9(kc, g, phi, out, s);
  dispatch<GPopLaunch>(dim, g.storage, 0, kc, g, phi, out, s);
  return hipGetLastError();
}

template <int DIM, typename T, bool LOCAL>
struct PopulationsLaunch {
  static void run(const KC &kc, FPtrs f, const float *Pb, float *out, hipStream_t s) {
    hipLaunchKernelGGL((populations_kernel<DIM, T, LOCAL>), LBTP_GRID(kc), kc, f, Pb, out);
  }
};

hipError_t launch_populations(int dim, int storage, const KC &kc, FPtrs f, int f_local, const float *Pb,
                              float *out, hipStream_t s) {
  if (dim == kD2Q9) return launch_populations_q9(storage, kc, f, f_local, Pb, out, s);
  dispatch<PopulationsLaunch>(dim, storage, f_local, kc, f, Pb, out, s);
  return hipGetLastError();
}

hipError_t launch_phase(int dim, const KC &kc, const float *u, const float *S, const float *K, float Ds, float *uw,
                        float *un, hipStream_t s) {
  hipLaunchKernelGGL(phase_kernel, LBTP_GRID(kc), kc, dim, u, S, K, Ds, uw, un);
  return hipGetLastError();
}

hipError_t launch_copy_probe(const void *src, void *dst, long long n4, hipStream_t s) {
  const long long want = (n4 + kThreads - 1) / kThreads;
  const int grid = (int)(want < 65536 ? want : 65536);
  hipLaunchKernelGGL(copy_probe_kernel, dim3(grid), dim3(kThreads), 0, s, (const float4 *)src, (float4 *)dst, n4);
  return hipGetLastError();
}

}  // namespace lbtp
