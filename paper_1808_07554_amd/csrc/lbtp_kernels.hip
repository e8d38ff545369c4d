// HIP kernels (gfx950) of the double-distribution lattice Boltzmann model
// (Chai, Liang, Du, Shi, arXiv:1808.07554) on D2Q5 / D3Q7.
//
// Data layout: structure of arrays, one float32 array per population and per
// scalar field, x fastest (index = x + nx*(y + ny*z)).  The pressure lattice
// is a two-buffer ping-pong in "pull" form: the buffer holds post-collision
// values f_i^+ of the previous sweep, and a sweep at node x reads
// f_i^+(x - c_i) (streaming, eq. 3-1) or, where x - c_i lies beyond a wall,
// the Section 4 rule: -f_opp^+(x) + 2 w P_b (anti-bounce-back) or f_opp^+(x)
// (bounce-back).  Right after initialisation the buffer instead holds
// pre-collision values read in place ("local" form).  The saturation lattice
// keeps pre-collision g and pushes post-collision values to the neighbours.
//
// Every cell kernel runs one thread per node, kThreads per block; all
// reductions are float64, first per wavefront (shuffles), then per block
// (LDS), then over blocks by a single-block finishing kernel in a fixed
// order, so every result is deterministic.
#include <math.h>

#include "lbtp_internal.h"

namespace lbtp {
namespace {

struct Cell {
  int c, x, y, z;
};

__device__ inline Cell cell_of(int c, const KC &kc) {
  Cell r;
  r.c = c;
  int row = c / kc.nx;
  r.x = c - row * kc.nx;
  r.z = row / kc.ny;
  r.y = row - r.z * kc.ny;
  return r;
}

__device__ inline int coord(const Cell &q, int a) { return a == 0 ? q.x : (a == 1 ? q.y : q.z); }
__device__ inline int extent(const KC &kc, int a) { return a == 0 ? kc.nx : (a == 1 ? kc.ny : kc.nz); }
__device__ inline int stride_of(const KC &kc, int a) { return a == 0 ? 1 : (a == 1 ? kc.nx : kc.nx * kc.ny); }

// Pre-collision f_j at node q (moving directions only).
template <int DIM, bool LOCAL>
__device__ inline void load_f(const FPtrs &fin, const Cell &q, const KC &kc, float *f) {
#pragma unroll
  for (int j = 0; j < 2 * DIM; ++j) {
    if (LOCAL) {
      f[j] = fin.p[j][q.c];
      continue;
    }
    const int a = dir_axis(j), s = dir_sign(j);
    const int x = coord(q, a), n = extent(kc, a), st = stride_of(kc, a);
    const bool out = (s > 0) ? (x == 0) : (x == n - 1);
    if (!out) {
      f[j] = fin.p[j][q.c - s * st];
    } else {
      const int face = 2 * a + (s > 0 ? 0 : 1);
      const int bc = kc.bc_f[face];
      if (bc == LBTP_BC_PERIODIC) {
        f[j] = fin.p[j][q.c - s * st + s * n * st];
      } else {
        const float o = fin.p[dir_opp(j)][q.c];
        f[j] = (bc == LBTP_BC_DIRICHLET) ? (kc.abbP[face] - o) : o;
      }
    }
  }
}

template <int DIM>
__device__ inline float moment_p(const float *f, const KC &kc) {
  float s = f[0];
#pragma unroll
  for (int j = 1; j < 2 * DIM; ++j) s += f[j];
  return s * kc.inv_1mw0;   // eq. 3-9a
}

// First moment sum_i c_i f_i along each axis.
template <int DIM>
__device__ inline void moment_c(const float *f, const KC &kc, float *m1) {
  m1[0] = kc.c * (f[0] - f[2]);
  m1[1] = kc.c * (f[1] - f[3]);
  if (DIM == 3) m1[2] = kc.c * (f[4] - f[5]);
}

template <int DIM>
__device__ inline float sum_g(const float *g) {
  float s = g[0];
#pragma unroll
  for (int i = 1; i <= 2 * DIM; ++i) s += g[i];
  return s;
}

// eq. 3-9b
__device__ inline float saturation_of(float gsum, float Fs, float phi, const KC &kc) {
  return (gsum + kc.half_dt * Fs) / phi;
}

// 1/tau_f from eq. 3-11a with D_p = K lambda_t (eq. 2-9, 2-16).
__device__ inline float inv_tau_f_of(float S, float K, const KC &kc) {
  const float lw = S * S * kc.inv_mu_w;
  const float ln = (1.0f - S) * (1.0f - S) * kc.inv_mu_n;
  const float Dp = K * (lw + ln);
  return 1.0f / (0.5f + Dp * kc.inv_cs2dt);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum of NV doubles, written by thread 0 to out[NV*blockIdx.x + v].
template <int NV>
__device__ inline void block_sum(double *v, double *out) {
  __shared__ double sh[NV][kThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[i][wid] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double t = 0.0;
      for (int w = 0; w < kThreads / 64; ++w) t += sh[i][w];
      out[NV * blockIdx.x + i] = t;
    }
  }
}

// ------------------------------------------------------------- pressure sweep
// One iteration of eq. 3-1: read (stream) f, P (eq. 3-9a), BGK collision with
// the local 1/tau_f (eq. 2-1b a), write f^+ in place of node x.
// SNAP: 0 nothing, 1 store P in the snapshot, 2 also accumulate
// sum (P - P_snap)^2 and sum P^2 for the stopping rule.
template <int DIM, bool LOCAL, int SNAP, bool HAS_FP>
__global__ __launch_bounds__(kThreads) void f_sweep_kernel(KC kc, FPtrs fin, FPtrs fout,
                                                           const float *__restrict__ itau,
                                                           const float *__restrict__ Fp,
                                                           float *__restrict__ Psnap,
                                                           double *__restrict__ partials,
                                                           const Ctl *__restrict__ ctl, long long k) {
  // a converged (or finished) solve turns the remaining queued sweeps into no-ops
  if (ctl->done || k > ctl->kmax) return;
  double acc[2] = {0.0, 0.0};
  const int stride = gridDim.x * kThreads;
  for (int c = blockIdx.x * kThreads + threadIdx.x; c < kc.ncell; c += stride) {
    const Cell q = cell_of(c, kc);
    float f[2 * DIM];
    load_f<DIM, LOCAL>(fin, q, kc, f);
    const float P = moment_p<DIM>(f, kc);
    const float wP = kc.w1 * P;
    const float it = itau[c];
    const float src = HAS_FP ? kc.dt * kc.wbar * Fp[c] : 0.0f;
#pragma unroll
    for (int j = 0; j < 2 * DIM; ++j) {
      float o = f[j] + (wP - f[j]) * it;
      if (HAS_FP) o += src;
      fout.p[j][c] = o;
    }
    if (SNAP == 2) {
      const double d = (double)P - (double)Psnap[c];
      acc[0] += d * d;
      acc[1] += (double)P * (double)P;
    }
    if (SNAP >= 1) Psnap[c] = P;
  }
  if (SNAP == 2) block_sum<2>(acc, partials);
}

// Stopping rule r = ||P^k - P^{k-m}|| / (m ||P^k||) from the block partials.
__global__ __launch_bounds__(1024) void finish_residual_kernel(const double *__restrict__ partials,
                                                               int nblk, Ctl *ctl, long long k, int m) {
  __shared__ double sa[1024], sb[1024];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 1024) {
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
    if (ctl->done || k > ctl->kmax) return;
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
  for (int i = threadIdx.x; i < nblk; i += 1024) a += partials[i];
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
template <int DIM, bool HAS_FS>
__global__ __launch_bounds__(kThreads) void moments_kernel(KC kc, GPtrs g, const float *__restrict__ K,
                                                           const float *__restrict__ phi,
                                                           const float *__restrict__ Fs, float *__restrict__ S,
                                                           float *__restrict__ itau,
                                                           double *__restrict__ partials, int write_coef) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  double acc[1] = {0.0};
  if (c < kc.ncell) {
    float gv[2 * DIM + 1];
    double dm = 0.0;
#pragma unroll
    for (int i = 0; i <= 2 * DIM; ++i) {
      gv[i] = g.p[i][c];
      dm += (double)gv[i];
    }
    const float fs = HAS_FS ? Fs[c] : 0.0f;
    const float Sv = saturation_of(sum_g<DIM>(gv), fs, phi[c], kc);
    if (write_coef) {
      S[c] = Sv;
      itau[c] = inv_tau_f_of(Sv, K[c], kc);
    }
    if (HAS_FS) dm += 0.5 * (double)kc.dt * (double)fs;
    acc[0] = dm;
  }
  block_sum<1>(acc, partials);
}

// ---------------------------------------------------------- saturation sweep
// One step of eq. 3-2 with g^eq of eq. 3-4b, the local grad P of eq. 3-10a
// (from the pressure lattice, read as in the pressure sweep) and
// gamma = -lambda_w K / (c_s^2 dt) (eq. 3-8); post-collision values are
// pushed to x + c_i, or reflected at walls (Section 4).  Block partials of
// the net flux through reflected links.
template <int DIM, bool FLOCAL, bool HAS_FS>
__global__ __launch_bounds__(kThreads) void g_sweep_kernel(KC kc, GPtrs gin, GPtrs gout, FPtrs f,
                                                           const float *__restrict__ itau,
                                                           const float *__restrict__ K,
                                                           const float *__restrict__ phi,
                                                           const float *__restrict__ Fs,
                                                           double *__restrict__ partials) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  double acc[1] = {0.0};
  if (c < kc.ncell) {
    const Cell q = cell_of(c, kc);
    float gv[2 * DIM + 1];
#pragma unroll
    for (int i = 0; i <= 2 * DIM; ++i) gv[i] = gin.p[i][c];
    const float fs = HAS_FS ? Fs[c] : 0.0f;
    const float ph = phi[c];
    const float Sv = saturation_of(sum_g<DIM>(gv), fs, ph, kc);
    float fv[2 * DIM];
    load_f<DIM, FLOCAL>(f, q, kc, fv);
    float m1[3];
    moment_c<DIM>(fv, kc, m1);
    const float gscale = -itau[c] * kc.inv_cs2dt;      // grad P = gscale * m1
    const float lw = Sv * Sv * kc.inv_mu_w;
    const float gamma = -lw * K[c] * kc.inv_cs2dt;
    const float conv = gamma * kc.dt * kc.w1 * kc.inv_tau_g * kc.c * gscale;  // times s * m1[a]
    const float srcw = kc.src_g * fs;
    // rest population
    {
      const float geq = (kc.geq0_phi + ph) * Sv;
      float o = gv[0] + (geq - gv[0]) * kc.inv_tau_g;
      if (HAS_FS) o += kc.w0 * srcw;
      gout.p[0][c] = o;
    }
    const float geq = kc.w1beta * Sv;
    double flux = 0.0;
#pragma unroll
    for (int j = 0; j < 2 * DIM; ++j) {
      const int a = dir_axis(j), s = dir_sign(j);
      float o = gv[j + 1] + (geq - gv[j + 1]) * kc.inv_tau_g;
      if (HAS_FS) o += kc.w1 * srcw;
      o += conv * (float)s * m1[a];
      const int x = coord(q, a), n = extent(kc, a), st = stride_of(kc, a);
      const bool out = (s > 0) ? (x == n - 1) : (x == 0);
      if (!out) {
        gout.p[j + 1][c + s * st] = o;
      } else {
        const int face = 2 * a + (s > 0 ? 1 : 0);
        const int bc = kc.bc_g[face];
        if (bc == LBTP_BC_PERIODIC) {
          gout.p[j + 1][c + s * st - s * n * st] = o;
        } else {
          float r;
          if (bc == LBTP_BC_NOFLUX) r = o;
          else if (bc == LBTP_BC_DIRICHLET) r = kc.abbS[face] - o;
          else r = 2.0f * kc.w1beta * Sv - o;    // outflow: S_wb = S of this node
          gout.p[dir_opp(j) + 1][c] = r;
          flux += (double)r - (double)o;
        }
      }
    }
    acc[0] = flux;
  }
  block_sum<1>(acc, partials);
}

// ------------------------------------------------------------ initialisation
// Central difference of u along axis a (one-sided second order at walls).
template <int DIM>
__device__ inline float cdiff(const float *__restrict__ u, const Cell &q, int a, const KC &kc, float inv2dx) {
  const int x = coord(q, a), n = extent(kc, a), st = stride_of(kc, a);
  const bool periodic = kc.bc_f[2 * a] == LBTP_BC_PERIODIC;
  const int c = q.c;
  if (periodic) {
    const int cp = (x == n - 1) ? c - (n - 1) * st : c + st;
    const int cm = (x == 0) ? c + (n - 1) * st : c - st;
    return (u[cp] - u[cm]) * inv2dx;
  }
  if (x == 0) return (-3.0f * u[c] + 4.0f * u[c + st] - u[c + 2 * st]) * inv2dx;
  if (x == n - 1) return (3.0f * u[c] - 4.0f * u[c - st] + u[c - 2 * st]) * inv2dx;
  return (u[c + st] - u[c - st]) * inv2dx;
}

// f_i = w_i P0 - tau_f dt w_i c_i . grad P0 (i >= 1); g_i = g_i^eq(S0) + eps g_i^(1)
// with eps g_i^(1) = -tau_g dt [(Gamma_i/phi - w_i(1 - 1/(2 tau_g))) F_s
//                               + Gamma_i c_i . grad S0 - gamma w_i c_i . grad P0 / tau_g]
// (eq. gini, gneq), Gamma_i = g_i^eq / S.  f is written in local form.
template <int DIM>
__global__ __launch_bounds__(kThreads) void init_kernel(KC kc, const float *__restrict__ P0,
                                                        const float *__restrict__ S0,
                                                        const float *__restrict__ dP0,
                                                        const float *__restrict__ dS0,
                                                        const float *__restrict__ K,
                                                        const float *__restrict__ phi,
                                                        const float *__restrict__ Fs, int neq, FPtrs f,
                                                        GPtrs g) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const Cell q = cell_of(c, kc);
  const float P = P0[c], S = S0[c], ph = phi[c];
  const float fs = Fs ? Fs[c] : 0.0f;
  float gp[3] = {0.f, 0.f, 0.f}, gs[3] = {0.f, 0.f, 0.f};
  if (neq) {
    const float inv2dx = 0.5f / (kc.c * kc.dt);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      gp[a] = dP0 ? dP0[a * kc.ncell + c] : cdiff<DIM>(P0, q, a, kc, inv2dx);
      gs[a] = dS0 ? dS0[a * kc.ncell + c] : cdiff<DIM>(S0, q, a, kc, inv2dx);
    }
  }
  const float itf = inv_tau_f_of(S, K[c], kc);
  const float tau_f = 1.0f / itf;
  const float lw = S * S * kc.inv_mu_w;
  const float gamma = -lw * K[c] * kc.inv_cs2dt;
  const float tau_g = 1.0f / kc.inv_tau_g;
  const float wsrc = 1.0f - 0.5f * kc.inv_tau_g;
  const float wP = kc.w1 * P;
#pragma unroll
  for (int j = 0; j < 2 * DIM; ++j) {
    const int a = dir_axis(j), s = dir_sign(j);
    const float cdp = (float)s * kc.c * gp[a];
    f.p[j][c] = neq ? wP - tau_f * kc.dt * kc.w1 * cdp : wP;
  }
  // rest population: Gamma_0 = (w0 - 1) beta + phi, c_0 = 0
  {
    const float G0 = kc.geq0_phi + ph;
    float v = G0 * S;
    if (neq) v -= tau_g * kc.dt * ((G0 / ph - kc.w0 * wsrc) * fs);
    g.p[0][c] = v;
  }
  const float G = kc.w1beta;
#pragma unroll
  for (int j = 0; j < 2 * DIM; ++j) {
    const int a = dir_axis(j), s = dir_sign(j);
    float v = G * S;
    if (neq) {
      const float cdp = (float)s * kc.c * gp[a];
      const float cds = (float)s * kc.c * gs[a];
      v -= tau_g * kc.dt * ((G / ph - kc.w1 * wsrc) * fs + G * cds - gamma * kc.w1 * cdp * kc.inv_tau_g);
    }
    g.p[j + 1][c] = v;
  }
}

// ----------------------------------------------------------------- outputs
template <int DIM, bool LOCAL>
__global__ __launch_bounds__(kThreads) void pressure_kernel(KC kc, FPtrs f, float *__restrict__ P) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const Cell q = cell_of(c, kc);
  float fv[2 * DIM];
  load_f<DIM, LOCAL>(f, q, kc, fv);
  P[c] = moment_p<DIM>(fv, kc);
}

// grad P (eq. 3-10a) or u = -K lambda_t grad P (eq. 3-10b), component-major.
template <int DIM, bool LOCAL>
__global__ __launch_bounds__(kThreads) void grad_kernel(KC kc, FPtrs f, const float *__restrict__ itau,
                                                        const float *__restrict__ K,
                                                        const float *__restrict__ S, int velocity,
                                                        float *__restrict__ out) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const Cell q = cell_of(c, kc);
  float fv[2 * DIM];
  load_f<DIM, LOCAL>(f, q, kc, fv);
  float m1[3];
  moment_c<DIM>(fv, kc, m1);
  float scale = -itau[c] * kc.inv_cs2dt;
  if (velocity) {
    const float Sv = S[c];
    const float lt = Sv * Sv * kc.inv_mu_w + (1.0f - Sv) * (1.0f - Sv) * kc.inv_mu_n;
    scale = -K[c] * lt * scale;
  }
#pragma unroll
  for (int a = 0; a < DIM; ++a) out[a * kc.ncell + c] = scale * m1[a];
}

template <int DIM, bool HAS_FS>
__global__ __launch_bounds__(kThreads) void saturation_kernel(KC kc, GPtrs g, const float *__restrict__ phi,
                                                              const float *__restrict__ Fs,
                                                              float *__restrict__ S) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  float gv[2 * DIM + 1];
#pragma unroll
  for (int i = 0; i <= 2 * DIM; ++i) gv[i] = g.p[i][c];
  S[c] = saturation_of(sum_g<DIM>(gv), HAS_FS ? Fs[c] : 0.0f, phi[c], kc);
}

template <int DIM, bool LOCAL>
__global__ __launch_bounds__(kThreads) void materialize_kernel(KC kc, FPtrs fin, FPtrs fout) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= kc.ncell) return;
  const Cell q = cell_of(c, kc);
  float fv[2 * DIM];
  load_f<DIM, LOCAL>(fin, q, kc, fv);
#pragma unroll
  for (int j = 0; j < 2 * DIM; ++j) fout.p[j][c] = fv[j];
}

}  // namespace

// ---------------------------------------------------------------- launchers
#define LBTP_GRID(kc) dim3(nblocks((kc).ncell)), dim3(kThreads), 0, s
#define LBTP_SWEEP_GRID(kc) dim3(sweep_blocks((kc).ncell)), dim3(kThreads), 0, s

template <int DIM, bool LOCAL, int SNAP>
static void f_sweep_fp(const KC &kc, FPtrs fin, FPtrs fout, const float *itau, const float *Fp,
                       float *Psnap, double *partials, const Ctl *ctl, long long k, hipStream_t s) {
  if (Fp)
    hipLaunchKernelGGL((f_sweep_kernel<DIM, LOCAL, SNAP, true>), LBTP_SWEEP_GRID(kc), kc, fin, fout, itau, Fp,
                       Psnap, partials, ctl, k);
  else
    hipLaunchKernelGGL((f_sweep_kernel<DIM, LOCAL, SNAP, false>), LBTP_SWEEP_GRID(kc), kc, fin, fout, itau, Fp,
                       Psnap, partials, ctl, k);
}

template <int DIM, bool LOCAL>
static void f_sweep_snap(const KC &kc, FPtrs fin, FPtrs fout, const float *itau, const float *Fp,
                         float *Psnap, double *partials, const Ctl *ctl, long long k, int snap, hipStream_t s) {
  if (snap == 0) f_sweep_fp<DIM, LOCAL, 0>(kc, fin, fout, itau, Fp, Psnap, partials, ctl, k, s);
  else if (snap == 1) f_sweep_fp<DIM, LOCAL, 1>(kc, fin, fout, itau, Fp, Psnap, partials, ctl, k, s);
  else f_sweep_fp<DIM, LOCAL, 2>(kc, fin, fout, itau, Fp, Psnap, partials, ctl, k, s);
}

hipError_t launch_f_sweep(int dim, const KC &kc, FPtrs fin, FPtrs fout, const float *itau, const float *Fp,
                          float *Psnap, double *partials, const Ctl *ctl, long long k, int local, int snap,
                          hipStream_t s) {
  if (dim == 2) {
    if (local) f_sweep_snap<2, true>(kc, fin, fout, itau, Fp, Psnap, partials, ctl, k, snap, s);
    else f_sweep_snap<2, false>(kc, fin, fout, itau, Fp, Psnap, partials, ctl, k, snap, s);
  } else {
    if (local) f_sweep_snap<3, true>(kc, fin, fout, itau, Fp, Psnap, partials, ctl, k, snap, s);
    else f_sweep_snap<3, false>(kc, fin, fout, itau, Fp, Psnap, partials, ctl, k, snap, s);
  }
  return hipGetLastError();
}

hipError_t launch_finish_residual(const double *partials, int nblk, Ctl *ctl, long long k, int m, hipStream_t s) {
  hipLaunchKernelGGL(finish_residual_kernel, dim3(1), dim3(1024), 0, s, partials, nblk, ctl, k, m);
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

hipError_t launch_moments(int dim, const KC &kc, GPtrs g, const float *K, const float *phi, const float *Fs,
                          float *S, float *itau, double *partials, int write_coef, hipStream_t s) {
  if (dim == 2) {
    if (Fs) hipLaunchKernelGGL((moments_kernel<2, true>), LBTP_GRID(kc), kc, g, K, phi, Fs, S, itau, partials, write_coef);
    else hipLaunchKernelGGL((moments_kernel<2, false>), LBTP_GRID(kc), kc, g, K, phi, Fs, S, itau, partials, write_coef);
  } else {
    if (Fs) hipLaunchKernelGGL((moments_kernel<3, true>), LBTP_GRID(kc), kc, g, K, phi, Fs, S, itau, partials, write_coef);
    else hipLaunchKernelGGL((moments_kernel<3, false>), LBTP_GRID(kc), kc, g, K, phi, Fs, S, itau, partials, write_coef);
  }
  return hipGetLastError();
}

template <int DIM, bool FLOCAL>
static void g_sweep_fs(const KC &kc, GPtrs gin, GPtrs gout, FPtrs f, const float *itau, const float *K,
                       const float *phi, const float *Fs, double *partials, hipStream_t s) {
  if (Fs) hipLaunchKernelGGL((g_sweep_kernel<DIM, FLOCAL, true>), LBTP_GRID(kc), kc, gin, gout, f, itau, K, phi, Fs, partials);
  else hipLaunchKernelGGL((g_sweep_kernel<DIM, FLOCAL, false>), LBTP_GRID(kc), kc, gin, gout, f, itau, K, phi, Fs, partials);
}

hipError_t launch_g_sweep(int dim, const KC &kc, GPtrs gin, GPtrs gout, FPtrs f, int f_local, const float *itau,
                          const float *K, const float *phi, const float *Fs, double *partials, hipStream_t s) {
  if (dim == 2) {
    if (f_local) g_sweep_fs<2, true>(kc, gin, gout, f, itau, K, phi, Fs, partials, s);
    else g_sweep_fs<2, false>(kc, gin, gout, f, itau, K, phi, Fs, partials, s);
  } else {
    if (f_local) g_sweep_fs<3, true>(kc, gin, gout, f, itau, K, phi, Fs, partials, s);
    else g_sweep_fs<3, false>(kc, gin, gout, f, itau, K, phi, Fs, partials, s);
  }
  return hipGetLastError();
}

hipError_t launch_init(int dim, const KC &kc, const float *P0, const float *S0, const float *dP0, const float *dS0,
                       const float *K, const float *phi, const float *Fs, int neq, FPtrs f, GPtrs g, hipStream_t s) {
  if (dim == 2) hipLaunchKernelGGL((init_kernel<2>), LBTP_GRID(kc), kc, P0, S0, dP0, dS0, K, phi, Fs, neq, f, g);
  else hipLaunchKernelGGL((init_kernel<3>), LBTP_GRID(kc), kc, P0, S0, dP0, dS0, K, phi, Fs, neq, f, g);
  return hipGetLastError();
}

hipError_t launch_pressure(int dim, const KC &kc, FPtrs f, int f_local, float *P, hipStream_t s) {
  if (dim == 2) {
    if (f_local) hipLaunchKernelGGL((pressure_kernel<2, true>), LBTP_GRID(kc), kc, f, P);
    else hipLaunchKernelGGL((pressure_kernel<2, false>), LBTP_GRID(kc), kc, f, P);
  } else {
    if (f_local) hipLaunchKernelGGL((pressure_kernel<3, true>), LBTP_GRID(kc), kc, f, P);
    else hipLaunchKernelGGL((pressure_kernel<3, false>), LBTP_GRID(kc), kc, f, P);
  }
  return hipGetLastError();
}

hipError_t launch_grad(int dim, const KC &kc, FPtrs f, int f_local, const float *itau, const float *K,
                       const float *S, int velocity, float *out, hipStream_t s) {
  if (dim == 2) {
    if (f_local) hipLaunchKernelGGL((grad_kernel<2, true>), LBTP_GRID(kc), kc, f, itau, K, S, velocity, out);
    else hipLaunchKernelGGL((grad_kernel<2, false>), LBTP_GRID(kc), kc, f, itau, K, S, velocity, out);
  } else {
    if (f_local) hipLaunchKernelGGL((grad_kernel<3, true>), LBTP_GRID(kc), kc, f, itau, K, S, velocity, out);
    else hipLaunchKernelGGL((grad_kernel<3, false>), LBTP_GRID(kc), kc, f, itau, K, S, velocity, out);
  }
  return hipGetLastError();
}

hipError_t launch_saturation(int dim, const KC &kc, GPtrs g, const float *phi, const float *Fs, float *S,
                             hipStream_t s) {
  if (dim == 2) {
    if (Fs) hipLaunchKernelGGL((saturation_kernel<2, true>), LBTP_GRID(kc), kc, g, phi, Fs, S);
    else hipLaunchKernelGGL((saturation_kernel<2, false>), LBTP_GRID(kc), kc, g, phi, Fs, S);
  } else {
    if (Fs) hipLaunchKernelGGL((saturation_kernel<3, true>), LBTP_GRID(kc), kc, g, phi, Fs, S);
    else hipLaunchKernelGGL((saturation_kernel<3, false>), LBTP_GRID(kc), kc, g, phi, Fs, S);
  }
  return hipGetLastError();
}

hipError_t launch_materialize_f(int dim, const KC &kc, FPtrs fin, int f_local, FPtrs fout, hipStream_t s) {
  if (dim == 2) {
    if (f_local) hipLaunchKernelGGL((materialize_kernel<2, true>), LBTP_GRID(kc), kc, fin, fout);
    else hipLaunchKernelGGL((materialize_kernel<2, false>), LBTP_GRID(kc), kc, fin, fout);
  } else {
    if (f_local) hipLaunchKernelGGL((materialize_kernel<3, true>), LBTP_GRID(kc), kc, fin, fout);
    else hipLaunchKernelGGL((materialize_kernel<3, false>), LBTP_GRID(kc), kc, fin, fout);
  }
  return hipGetLastError();
}

}  // namespace lbtp
