// Device functions shared by the single-realisation kernels (lbtp_kernels.hip)
// and the ensemble kernels (lbtp_batch.hip).  See lbtp_kernels.hip for the
// data layout and the deviation form of the pressure lattice.
#pragma once
#include <math.h>
#include <stdint.h>

#include <type_traits>

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

// ------------------------------------------------------------ storage types
// bf16 is kept as raw 16-bit words (round to nearest even on store).
struct bf16_t {
  uint16_t u;
};

template <typename T>
struct Storage;

template <>
struct Storage<float> {
  static __device__ inline float load(const float *p, int i, float) { return p[i]; }
  static __device__ inline void store(float *p, int i, float v, float) { p[i] = v; }
};

// fp16 values are scaled by a power of two (kc.dev_scale) to keep the
// deviations in the normal range.
template <>
struct Storage<_Float16> {
  static __device__ inline float load(const _Float16 *p, int i, float inv_s) { return (float)p[i] * inv_s; }
  static __device__ inline void store(_Float16 *p, int i, float v, float s) { p[i] = (_Float16)(v * s); }
};

template <>
struct Storage<bf16_t> {
  static __device__ inline float load(const bf16_t *p, int i, float) {
    return __uint_as_float((uint32_t)p[i].u << 16);
  }
  static __device__ inline void store(bf16_t *p, int i, float v, float) {
    const uint32_t u = __float_as_uint(v);
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    bf16_t b;
    b.u = (uint16_t)(r >> 16);
    p[i] = b;
  }
};

template <typename T>
struct FP {
  T *p[8];
};

template <typename T>
__host__ __device__ inline FP<T> typed(const FPtrs &f) {
  FP<T> r;
  for (int j = 0; j < 8; ++j) r.p[j] = (T *)f.p[j];
  return r;
}

// Typed view of a saturation buffer (GPtrs).
template <typename T>
struct GP {
  T *p[9];
  float *B;
};
template <typename T>
__host__ __device__ inline GP<T> gtyped(const GPtrs &g) {
  GP<T> r;
  for (int i = 0; i < 9; ++i) r.p[i] = (T *)g.p[i];
  r.B = g.B;
  return r;
}

// g_i^eq(B) of eq. 3-4b on D2Q5 / D3Q7: [(w0 - 1) beta + phi] B for the rest
// population, w1 beta B for the moving ones.
__device__ inline float geq_odd(const KC &kc, int i, float B, float phi) {
  return i == 0 ? (kc.geq0_phi + phi) * B : kc.w1beta * B;
}

// Saturation population i at node c: stored as is (float32), or as the
// 16-bit deviation from geq (the caller's g_i^eq(B) of the node, from the
// buffer's base B) in FP32 arithmetic.
template <typename T>
__device__ inline float gload(const T *p, int c, float geq, const KC &kc) {
  if constexpr (std::is_same<T, float>::value) return p[c];
  else return Storage<T>::load(p, c, kc.inv_g_scale) + geq;
}
template <typename T>
__device__ inline void gstore(T *p, int c, float v, float geq, const KC &kc) {
  if constexpr (std::is_same<T, float>::value) p[c] = v;
  else Storage<T>::store(p, c, v - geq, kc.g_scale);
}
template <typename T>
constexpr bool gdev() { return !std::is_same<T, float>::value; }

// Node index within the wall-value arrays of a face: y + ny z (x faces),
// x + nx z (y faces), x + nx y (z faces).
__device__ inline int face_index(const KC &kc, int face, int x, int y, int z) {
  return face < 2 ? y + kc.ny * z : (face < 4 ? x + kc.nx * z : x + kc.nx * y);
}

// Dirichlet pressure / saturation of the link k (L per node) arriving at node
// (x, y, z) through face: the per-link data if set, else the face constant.
__device__ inline float wall_P(const KC &kc, int face, int x, int y, int z, int L, int k) {
  const float *a = kc.wP[face];
  return a ? a[face_index(kc, face, x, y, z) * L + k] : kc.Pw[face];
}
__device__ inline float wall_S(const KC &kc, int face, int x, int y, int z, int L, int k) {
  const float *a = kc.wS[face];
  return a ? a[face_index(kc, face, x, y, z) * L + k] : kc.Sw[face];
}

// Pre-collision deviations e_j at node q (moving directions) against P_b(q).
template <int DIM, typename T, bool LOCAL>
__device__ inline void load_e(const FP<T> &fin, const float *__restrict__ Pb, const Cell &q, const KC &kc,
                              float pb, float *e) {
#pragma unroll
  for (int j = 0; j < 2 * DIM; ++j) {
    if (LOCAL) {
      e[j] = Storage<T>::load(fin.p[j], q.c, kc.inv_dev_scale);
      continue;
    }
    const int a = dir_axis(j), s = dir_sign(j);
    const int x = coord(q, a), n = extent(kc, a), st = stride_of(kc, a);
    const bool out = (s > 0) ? (x == 0) : (x == n - 1);
    if (!out) {
      const int src = q.c - s * st;
      e[j] = Storage<T>::load(fin.p[j], src, kc.inv_dev_scale) + kc.w1 * (Pb[src] - pb);
    } else {
      const int face = 2 * a + (s > 0 ? 0 : 1);
      const int bc = kc.bc_f[face];
      if (bc == LBTP_BC_PERIODIC) {
        const int src = q.c - s * st + s * n * st;
        e[j] = Storage<T>::load(fin.p[j], src, kc.inv_dev_scale) + kc.w1 * (Pb[src] - pb);
      } else {
        const float o = Storage<T>::load(fin.p[dir_opp(j)], q.c, kc.inv_dev_scale);
        e[j] = (bc == LBTP_BC_DIRICHLET) ? (2.0f * kc.w1 * (wall_P(kc, face, q.x, q.y, q.z, 1, 0) - pb) - o) : o;
      }
    }
  }
}

// Sum of the deviations of the moving directions; P - P_b is this sum over
// 1 - w0 (eq. 3-9a), and w1 (P - P_b) this sum times w1 / (1 - w0) (one
// product, 1/4 on D2Q5).
template <int DIM>
__device__ inline float dsum(const float *e) {
  float s = e[0];
#pragma unroll
  for (int j = 1; j < 2 * DIM; ++j) s += e[j];
  return s;
}

// P - P_b from the deviations (eq. 3-9a).
template <int DIM>
__device__ inline float dpressure(const float *e, const KC &kc) {
  return dsum<DIM>(e) * kc.inv_1mw0;
}

// First moment sum_i c_i f_i = sum_i c_i e_i along each axis (the base part cancels).
template <int DIM>
__device__ inline void moment_c(const float *e, const KC &kc, float *m1) {
  m1[0] = kc.c * (e[0] - e[2]);
  m1[1] = kc.c * (e[1] - e[3]);
  if (DIM == 3) m1[2] = kc.c * (e[4] - e[5]);
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

// D_p and lambda_w K of the coefficient model: K lambda_t and K k_rw/mu_w with
// k_rw = S^2, k_rn = (1-S)^2 (eq. 2-9, 2-16), or given as rational functions
// of S (the form Sections 4.1 and 4.2 use).
__device__ inline float dp_of(float S, float K, const KC &kc) {
  if (kc.coef == LBTP_COEF_RATIONAL) return K * (kc.cf[0] + kc.cf[1] * S) / (kc.cf[4] + kc.cf[5] * S);
  const float lw = S * S * kc.inv_mu_w;
  const float ln = (1.0f - S) * (1.0f - S) * kc.inv_mu_n;
  return K * (lw + ln);
}
__device__ inline float lwk_of(float S, float K, const KC &kc) {
  if (kc.coef == LBTP_COEF_RATIONAL) return K * (kc.cf[2] + kc.cf[3] * S) / (kc.cf[4] + kc.cf[5] * S);
  return S * S * kc.inv_mu_w * K;
}

// 1/tau_f from eq. 3-11a.
__device__ inline float inv_tau_f_of(float S, float K, const KC &kc) {
  return 1.0f / (0.5f + dp_of(S, K, kc) * kc.inv_cs2dt);
}

// 1/tau_g (eq. 3-11b) with D_s = Ds + cap_B K lambda_n f_w, K lambda_n =
// D_p - lambda_w K and f_w = lambda_w K / D_p (eq. 2-10, 2-16).
__device__ inline float inv_tau_g_of(float S, float K, const KC &kc) {
  const float dp = dp_of(S, K, kc), lwk = lwk_of(S, K, kc);
  const float Ds = kc.Ds + kc.cap_B * (dp - lwk) * (lwk / dp);
  return 1.0f / (0.5f + Ds * kc.inv_bcs2dt);
}

// The value of the lane one below (from_left) or one above (from_right) in
// the wavefront, moved by the data-parallel primitives' wavefront shift
// (a VALU operation, no LDS round trip).  Lane 0, respectively lane 63, gets
// 0: callers use these only where the edge lanes hold halo columns whose
// values are never kept.
__device__ inline float lane_from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));   // wave_shr:1
}
__device__ inline float lane_from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));   // wave_shl:1
}

// Tile handled by workgroup b of a launch over n tiles.  Workgroups are dealt
// to the 8 XCDs in turn (b % 8); this gives each XCD a contiguous run of
// tiles, so that the halos neighbouring tiles share stay in that XCD's L2.
__device__ inline int xcd_tile(int b, int n) {
  constexpr int kXcd = 8;
  const int q = n / kXcd, r = n % kXcd, x = b % kXcd;
  return x * q + (x < r ? x : r) + b / kXcd;
}

// Position (tile_x, tile_y) of tile t of a tiles_x x tiles_y grid taken in
// bands of `band` tiles' width, each band row by row: runs of consecutive
// tiles form patches that overlap in x and y.
__host__ __device__ inline void band_tile(int t, int tiles_x, int tiles_y, int band, int *tile_x, int *tile_y) {
  const int full = tiles_x / band, b = t / (band * tiles_y);
  const int w = b < full ? band : tiles_x - full * band;
  const int r = t - b * band * tiles_y;
  *tile_x = b * band + r % w;
  *tile_y = r / w;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum of NV doubles, written by thread 0 to out[NV*blockIdx.x + v].
template <int NV, int NT = kThreads>
__device__ inline void block_sum(double *v, double *out) {
  __shared__ double sh[NV][NT / 64];
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
      for (int w = 0; w < NT / 64; ++w) t += sh[i][w];
      out[NV * blockIdx.x + i] = t;
    }
  }
}

// BGK relaxation of one deviation (eq. 2-1b a), e + (w dP - e) / tau_f,
// evaluated as e (1 - 1/tau_f) + (w dP) / tau_f: keep = 1 - 1/tau_f and
// gain = (w dP) / tau_f once per node, then one fused multiply-add per
// population.  Every D2Q5 / D3Q7 pressure kernel relaxes through this
// function, so all of them round alike.
__device__ inline float bgk_relax(float e, float keep, float gain) { return __builtin_fmaf(e, keep, gain); }

// One node of the pressure sweep (eq. 3-1): stream (pull, or in place in
// the local form), P (eq. 3-9a), BGK collision with 1/tau_f (eq. 2-1b a) and
// the source dt wbar_i F_p.  MODE as in f_sweep_kernel; the stopping-rule
// terms are added to acc.
template <int DIM, typename T, bool LOCAL, int MODE, bool HAS_FP>
__device__ inline void sweep_cell(const KC &kc, const FP<T> &fin, const FP<T> &fout, const float *__restrict__ Pb_in,
                                  float *__restrict__ Pb_out, const float *__restrict__ itau,
                                  const float *__restrict__ Fp, int c, double *acc) {
  const Cell q = cell_of(c, kc);
  const float pb = Pb_in[c];
  float e[2 * DIM];
  load_e<DIM, T, LOCAL>(fin, Pb_in, q, kc, pb, e);
  const float sum = dsum<DIM>(e);
  const float dP = sum * kc.inv_1mw0, wdP = sum * kc.w1_1mw0;
  if (MODE == 3) {        // probe: the stopping-rule terms only
    const float P = pb + dP;
    acc[0] += (double)dP * (double)dP;
    acc[1] += (double)P * (double)P;
    return;
  }
  const float it = itau[c];
  const float keep = 1.0f - it, gain = wdP * it;
  float add = HAS_FP ? kc.dt * kc.wbar * Fp[c] : 0.0f;
  if (MODE >= 1) {
    const float P = pb + dP;
    add += kc.w1 * (pb - P);          // re-base to P_b = P (exact difference)
    Pb_out[c] = P;
    if (MODE == 2) {
      acc[0] += (double)dP * (double)dP;
      acc[1] += (double)P * (double)P;
    }
  }
#pragma unroll
  for (int j = 0; j < 2 * DIM; ++j) {
    float o = bgk_relax(e[j], keep, gain);
    if (HAS_FP || MODE >= 1) o += add;
    Storage<T>::store(fout.p[j], c, o, kc.dev_scale);
  }
}

// ------------------------------------------------- pressure sweep, 4 nodes / thread
// The same sweep with each thread owning four consecutive nodes of a row
// (nx % 4 == 0), so populations, base and 1/tau_f move as 16-byte (float) or
// 8-byte (16-bit) vectors.  The x-streamed populations and the x-neighbour
// bases come from the adjacent lane of the wavefront (a lane shuffle) or, at a
// wavefront edge, from one scalar load; rows at walls use the Section 4 rules.
template <typename T>
struct Vec4;

// Stores are non-temporal: a sweep's output is only read by the next sweep,
// after the whole grid has passed, so keeping it in the caches only evicts
// the neighbour rows the current sweep still reads.
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef uint32_t uint2_t __attribute__((ext_vector_type(2)));

template <>
struct Vec4<float> {
  static __device__ inline float4 load(const float *p, int i, float) { return *(const float4 *)(p + i); }
  static __device__ inline void store(float *p, int i, float4 v, float) {
    const float4_t w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, (float4_t *)(p + i));
  }
};

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

template <>
struct Vec4<_Float16> {
  static __device__ inline float4 load(const _Float16 *p, int i, float inv_s) {
    const half4_t h = *(const half4_t *)(p + i);
    return make_float4((float)h.x * inv_s, (float)h.y * inv_s, (float)h.z * inv_s, (float)h.w * inv_s);
  }
  static __device__ inline void store(_Float16 *p, int i, float4 v, float s) {
    half4_t h;
    h.x = (_Float16)(v.x * s);
    h.y = (_Float16)(v.y * s);
    h.z = (_Float16)(v.z * s);
    h.w = (_Float16)(v.w * s);
    __builtin_nontemporal_store(h, (half4_t *)(p + i));
  }
};

__device__ inline uint32_t bf16_round(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

template <>
struct Vec4<bf16_t> {
  static __device__ inline float4 load(const bf16_t *p, int i, float) {
    const uint2 w = *(const uint2 *)(p + i);
    return make_float4(__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xFFFF0000u),
                       __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xFFFF0000u));
  }
  static __device__ inline void store(bf16_t *p, int i, float4 v, float) {
    uint2_t w;
    w.x = bf16_round(v.x) | (bf16_round(v.y) << 16);
    w.y = bf16_round(v.z) | (bf16_round(v.w) << 16);
    __builtin_nontemporal_store(w, (uint2_t *)(p + i));
  }
};

__device__ inline float f4get(const float4 &v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w)); }
__device__ inline void f4set(float4 &v, int i, float x) {
  if (i == 0) v.x = x;
  else if (i == 1) v.y = x;
  else if (i == 2) v.z = x;
  else v.w = x;
}

// +x (e0) and -x (e2) deviations of the quad at node c (first node x0):
// from the thread's own vectors, the adjacent lanes (shuffles), one scalar
// load at a wavefront edge, or the x-face rules.  Every lane of the
// wavefront must call it (the shuffles).
template <typename T>
__device__ inline void pull_x_quad(const KC &kc, const FP<T> &fin, const float *__restrict__ Pb_in, int c, int x0,
                                   int y, int z, const float4 &pb, float4 &e0, float4 &e2) {
  const int lane = threadIdx.x & 63;
  const float is = kc.inv_dev_scale;
  // +x (j = 0) pulls from x - 1, -x (j = 2) from x + 1
  const float4 A = Vec4<T>::load(fin.p[0], c, is);
  const float4 B = Vec4<T>::load(fin.p[2], c, is);
  float a_left = __shfl_up(A.w, 1, 64), pb_left = __shfl_up(pb.w, 1, 64);
  float b_right = __shfl_down(B.x, 1, 64), pb_right = __shfl_down(pb.x, 1, 64);
  // +x for nodes 1..3 from the own vector, node 0 from the left neighbour
  e0 = make_float4(0.f, A.x + kc.w1 * (pb.x - pb.y), A.y + kc.w1 * (pb.y - pb.z), A.z + kc.w1 * (pb.z - pb.w));
  e2 = make_float4(B.y + kc.w1 * (pb.y - pb.x), B.z + kc.w1 * (pb.z - pb.y), B.w + kc.w1 * (pb.w - pb.z), 0.f);
  if (x0 == 0) {
    const int bc = kc.bc_f[0];
    if (bc == LBTP_BC_PERIODIC) {
      const int src = c + kc.nx - 1;
      e0.x = Storage<T>::load(fin.p[0], src, is) + kc.w1 * (Pb_in[src] - pb.x);
    } else {
      e0.x = (bc == LBTP_BC_DIRICHLET) ? (2.0f * kc.w1 * (wall_P(kc, 0, 0, y, z, 1, 0) - pb.x) - B.x) : B.x;
    }
  } else {
    if (lane == 0) {
      a_left = Storage<T>::load(fin.p[0], c - 1, is);
      pb_left = Pb_in[c - 1];
    }
    e0.x = a_left + kc.w1 * (pb_left - pb.x);
  }
  if (x0 + 4 == kc.nx) {
    const int bc = kc.bc_f[1];
    if (bc == LBTP_BC_PERIODIC) {
      const int src = c + 3 - (kc.nx - 1);
      e2.w = Storage<T>::load(fin.p[2], src, is) + kc.w1 * (Pb_in[src] - pb.w);
    } else {
      e2.w = (bc == LBTP_BC_DIRICHLET) ? (2.0f * kc.w1 * (wall_P(kc, 1, x0 + 3, y, z, 1, 0) - pb.w) - A.w) : A.w;
    }
  } else {
    if (lane == 63) {
      b_right = Storage<T>::load(fin.p[2], c + 4, is);
      pb_right = Pb_in[c + 4];
    }
    e2.w = b_right + kc.w1 * (pb_right - pb.w);
  }
}

// Whether the +a pull at coordinate coordv reads a node (inside, or across a
// periodic face), and likewise the -a pull; otherwise a wall rule applies.
__device__ inline bool reads_lo(const KC &kc, int a, int coordv) {
  return coordv != 0 || kc.bc_f[2 * a] == LBTP_BC_PERIODIC;
}
__device__ inline bool reads_hi(const KC &kc, int a, int coordv, int n) {
  return coordv != n - 1 || kc.bc_f[2 * a + 1] == LBTP_BC_PERIODIC;
}

// Deviations streamed along axis a >= 1 (+a into ep, -a into em) for the quad
// at node c with coordinate coordv along a (extent n, stride st): whole
// vectors from the neighbouring row or plane, or the face rules.  pbm and pbp
// are the bases of the rows the +a and -a pulls read (used only when they
// read one).
// Per-link Dirichlet data of the four nodes at face (x0.., other) (other = z
// for a y face, y for a z face), or the face constant.
__device__ inline float4 wall_P4(const KC &kc, int face, int x0, int other) {
  const float *a = kc.wP[face];
  if (a) return *(const float4 *)(a + x0 + kc.nx * other);
  const float pw = kc.Pw[face];
  return make_float4(pw, pw, pw, pw);
}

template <typename T>
__device__ inline void pull_axis_quad(const KC &kc, const FP<T> &fin, int c, int a, int coordv, int n, int st,
                                      int x0, int other, const float4 &pb, const float4 &pbm, const float4 &pbp,
                                      float4 &ep, float4 &em) {
  const float is = kc.inv_dev_scale;
  const int jp = (a == 1) ? 1 : 4, jm = (a == 1) ? 3 : 5;   // +a and -a directions
  // +a pulls from coord - 1
  if (reads_lo(kc, a, coordv)) {
    const int src = coordv == 0 ? c + (n - 1) * st : c - st;
    const float4 v = Vec4<T>::load(fin.p[jp], src, is);
    ep = make_float4(v.x + kc.w1 * (pbm.x - pb.x), v.y + kc.w1 * (pbm.y - pb.y), v.z + kc.w1 * (pbm.z - pb.z),
                     v.w + kc.w1 * (pbm.w - pb.w));
  } else {
    const float4 o = Vec4<T>::load(fin.p[jm], c, is);
    if (kc.bc_f[2 * a] == LBTP_BC_DIRICHLET) {
      const float4 pw = wall_P4(kc, 2 * a, x0, other);
      ep = make_float4(2.0f * kc.w1 * (pw.x - pb.x) - o.x, 2.0f * kc.w1 * (pw.y - pb.y) - o.y,
                       2.0f * kc.w1 * (pw.z - pb.z) - o.z, 2.0f * kc.w1 * (pw.w - pb.w) - o.w);
    } else {
      ep = o;
    }
  }
  // -a pulls from coord + 1
  if (reads_hi(kc, a, coordv, n)) {
    const int src = coordv == n - 1 ? c - (n - 1) * st : c + st;
    const float4 v = Vec4<T>::load(fin.p[jm], src, is);
    em = make_float4(v.x + kc.w1 * (pbp.x - pb.x), v.y + kc.w1 * (pbp.y - pb.y), v.z + kc.w1 * (pbp.z - pb.z),
                     v.w + kc.w1 * (pbp.w - pb.w));
  } else {
    const float4 o = Vec4<T>::load(fin.p[jp], c, is);
    if (kc.bc_f[2 * a + 1] == LBTP_BC_DIRICHLET) {
      const float4 pw = wall_P4(kc, 2 * a + 1, x0, other);
      em = make_float4(2.0f * kc.w1 * (pw.x - pb.x) - o.x, 2.0f * kc.w1 * (pw.y - pb.y) - o.y,
                       2.0f * kc.w1 * (pw.z - pb.z) - o.z, 2.0f * kc.w1 * (pw.w - pb.w) - o.w);
    } else {
      em = o;
    }
  }
}

// Bases of the rows the +a / -a pulls read, from memory (only those read).
__device__ inline void load_pb_axis(const KC &kc, const float *__restrict__ Pb_in, int c, int a, int coordv, int n,
                                    int st, float4 &pbm, float4 &pbp) {
  if (reads_lo(kc, a, coordv)) pbm = *(const float4 *)(Pb_in + (coordv == 0 ? c + (n - 1) * st : c - st));
  if (reads_hi(kc, a, coordv, n)) pbp = *(const float4 *)(Pb_in + (coordv == n - 1 ? c - (n - 1) * st : c + st));
}

// P (eq. 3-9a), collision (eq. 2-1b a), source, re-basing and stopping-rule
// terms of the four nodes of a quad, then the stores (active quads only).
template <int DIM, typename T, int MODE, bool HAS_FP>
__device__ inline void collide_quad(const KC &kc, const float4 *e, const float4 &pb, const float4 &it,
                                    const float4 &fp, const FP<T> &fout, float *__restrict__ Pb_out, int c,
                                    bool active, double *acc) {
  float4 o[2 * DIM];
  float4 pnew;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float ev[2 * DIM];
#pragma unroll
    for (int j = 0; j < 2 * DIM; ++j) ev[j] = f4get(e[j], i);
    const float sum = dsum<DIM>(ev);
    const float dP = sum * kc.inv_1mw0, wdP = sum * kc.w1_1mw0;
    const float t = f4get(it, i);
    const float keep = 1.0f - t, gain = wdP * t;
    float add = HAS_FP ? kc.dt * kc.wbar * f4get(fp, i) : 0.0f;
    if (MODE >= 1) {
      const float pbi = f4get(pb, i);
      const float P = pbi + dP;
      add += kc.w1 * (pbi - P);
      f4set(pnew, i, P);
      if (MODE == 2 && active) {
        acc[0] += (double)dP * (double)dP;
        acc[1] += (double)P * (double)P;
      }
    }
#pragma unroll
    for (int j = 0; j < 2 * DIM; ++j) {
      float v = bgk_relax(ev[j], keep, gain);
      if (HAS_FP || MODE >= 1) v += add;
      f4set(o[j], i, v);
    }
  }
  if (active) {
#pragma unroll
    for (int j = 0; j < 2 * DIM; ++j) Vec4<T>::store(fout.p[j], c, o[j], kc.dev_scale);
    if (MODE >= 1) *(float4 *)(Pb_out + c) = pnew;
  }
}

// Four nodes starting at quad qi of one realisation; adds the stopping-rule
// terms of the active quad to acc.  Shared by the single-realisation kernel
// and the batched (ensemble) kernel, so both compute bit-identical results.
template <int DIM, typename T, int MODE, bool HAS_FP>
__device__ inline void sweep_quad(const KC &kc, const FP<T> &fin, const FP<T> &fout, const float *__restrict__ Pb_in,
                                  float *__restrict__ Pb_out, const float *__restrict__ itau,
                                  const float *__restrict__ Fp, int qi, double *acc) {
  const int n4 = kc.ncell >> 2;
  const bool active = qi < n4;
  const int c = (active ? qi : n4 - 1) << 2;     // first of the four nodes
  const int row = c / kc.nx;
  const int x0 = c - row * kc.nx;
  const int z = row / kc.ny;
  const int y = row - z * kc.ny;

  const float4 pb = *(const float4 *)(Pb_in + c);
  float4 e[2 * DIM];
  pull_x_quad<T>(kc, fin, Pb_in, c, x0, y, z, pb, e[0], e[2]);
#pragma unroll
  for (int a = 1; a < DIM; ++a) {
    const int coordv = (a == 1) ? y : z;
    const int n = (a == 1) ? kc.ny : kc.nz;
    const int st = (a == 1) ? kc.nx : kc.nx * kc.ny;
    float4 pbm = pb, pbp = pb;
    load_pb_axis(kc, Pb_in, c, a, coordv, n, st, pbm, pbp);
    pull_axis_quad<T>(kc, fin, c, a, coordv, n, st, x0, (a == 1) ? z : y, pb, pbm, pbp, e[a == 1 ? 1 : 4],
                      e[a == 1 ? 3 : 5]);
  }
  if (MODE == 3) {        // probe: the stopping-rule terms only, as collide_quad forms them
    if (active) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float ev[2 * DIM];
#pragma unroll
        for (int j = 0; j < 2 * DIM; ++j) ev[j] = f4get(e[j], i);
        const float dP = dsum<DIM>(ev) * kc.inv_1mw0;
        const float P = f4get(pb, i) + dP;
        acc[0] += (double)dP * (double)dP;
        acc[1] += (double)P * (double)P;
      }
    }
    return;
  }
  const float4 it = *(const float4 *)(itau + c);
  float4 fp = make_float4(0.f, 0.f, 0.f, 0.f);
  if (HAS_FP) fp = *(const float4 *)(Fp + c);
  collide_quad<DIM, T, MODE, HAS_FP>(kc, e, pb, it, fp, fout, Pb_out, c, active, acc);
}

// S^n (eq. 3-9b) and 1/tau_f (eq. 3-11a, 2-9, 2-16) at node c; returns the
// node's mass sum_i g_i + dt F_s / 2 (= phi S) in float64.
template <int DIM, bool HAS_FS, typename TG>
__device__ inline double moments_cell(const KC &kc, const GPtrs &g_, const float *__restrict__ K,
                                      const float *__restrict__ phi, const float *__restrict__ Fs,
                                      float *__restrict__ S, float *__restrict__ itau, int c, int write_coef) {
  const GP<TG> g = gtyped<TG>(g_);
  const float ph = phi[c];
  const float B = gdev<TG>() ? g.B[c] : 0.0f;
  float gv[2 * DIM + 1];
  double dm = 0.0;
#pragma unroll
  for (int i = 0; i <= 2 * DIM; ++i) {
    gv[i] = gload(g.p[i], c, gdev<TG>() ? geq_odd(kc, i, B, ph) : 0.0f, kc);
    dm += (double)gv[i];
  }
  const float fs = HAS_FS ? Fs[c] : 0.0f;
  const float Sv = saturation_of(sum_g<DIM>(gv), fs, ph, kc);
  if (write_coef) {
    S[c] = Sv;
    itau[c] = inv_tau_f_of(Sv, K[c], kc);
    if (kc.itg) kc.itg[c] = inv_tau_g_of(Sv, K[c], kc);
  }
  if (HAS_FS) dm += 0.5 * (double)kc.dt * (double)fs;
  return dm;
}

// Push of the post-collision moving population j of node q (value o) to
// x + c_j, or its reflection at a wall (Section 4: bounce-back, anti-bounce-back
// with S_wb, or the zero-gradient outlet with S_wb = Sv, the node's S);
// periodic faces wrap.  16-bit storage writes the deviation from g^eq of the
// node written, from S^n (Sn; Snc at q).  Returns the reflected link's flux.
template <typename T>
__device__ inline double g_push(const KC &kc, const GP<T> &gout, const float *__restrict__ Sn, const Cell &q, int j,
                                float o, float Sv, float Snc) {
  const int a = dir_axis(j), s = dir_sign(j);
  const int c = q.c;
  const int x = coord(q, a), n = extent(kc, a), st = stride_of(kc, a);
  const bool out = (s > 0) ? (x == n - 1) : (x == 0);
  if (!out) {
    const int d = c + s * st;
    gstore(gout.p[j + 1], d, o, gdev<T>() ? kc.w1beta * Sn[d] : 0.0f, kc);
    return 0.0;
  }
  const int face = 2 * a + (s > 0 ? 1 : 0);
  const int bc = kc.bc_g[face];
  if (bc == LBTP_BC_PERIODIC) {
    const int d = c + s * st - s * n * st;
    gstore(gout.p[j + 1], d, o, gdev<T>() ? kc.w1beta * Sn[d] : 0.0f, kc);
    return 0.0;
  }
  float r;
  if (bc == LBTP_BC_NOFLUX) r = o;
  else if (bc == LBTP_BC_DIRICHLET)
    r = (kc.wS[face] ? 2.0f * kc.w1beta * wall_S(kc, face, q.x, q.y, q.z, 1, 0) : kc.abbS[face]) - o;
  else r = 2.0f * kc.w1beta * Sv - o;    // outflow: S_wb = S of this node
  gstore(gout.p[dir_opp(j) + 1], c, r, gdev<T>() ? kc.w1beta * Snc : 0.0f, kc);
  return (double)r - (double)o;
}

// One node of the saturation step (eq. 3-2 with g^eq of eq. 3-4b, the local
// grad P of eq. 3-10a read from the pressure lattice as in the pressure sweep,
// gamma = -lambda_w K / (c_s^2 dt), eq. 3-8): collide and push to x + c_i, or
// reflect at walls (Section 4).  Returns the net flux through reflected links.
// With 16-bit storage (T) both lattices are stored in 16 bits: the
// saturation populations are read against the input buffer's base and
// written as deviations from g^eq(S^n) of the node they land on (Sn, the
// saturation of this coupled step, which becomes the output buffer's base).
template <int DIM, typename T, bool FLOCAL, bool HAS_FS>
__device__ inline double g_sweep_cell(const KC &kc, const GPtrs &gin_, const GPtrs &gout_, const FP<T> &f,
                                      const float *__restrict__ Pb, const float *__restrict__ itau,
                                      const float *__restrict__ K, const float *__restrict__ phi,
                                      const float *__restrict__ Fs, const float *__restrict__ Sn, int c) {
  const Cell q = cell_of(c, kc);
  const GP<T> gin = gtyped<T>(gin_), gout = gtyped<T>(gout_);
  const float ph = phi[c];
  const float Bc = gdev<T>() ? gin.B[c] : 0.0f;
  float gv[2 * DIM + 1];
#pragma unroll
  for (int i = 0; i <= 2 * DIM; ++i) gv[i] = gload(gin.p[i], c, gdev<T>() ? geq_odd(kc, i, Bc, ph) : 0.0f, kc);
  const float fs = HAS_FS ? Fs[c] : 0.0f;
  const float Snc = gdev<T>() ? Sn[c] : 0.0f;
  if (gdev<T>()) gout.B[c] = Snc;
  const float Sv = saturation_of(sum_g<DIM>(gv), fs, ph, kc);
  float e[2 * DIM];
  load_e<DIM, T, FLOCAL>(f, Pb, q, kc, Pb[c], e);
  float m1[3];
  moment_c<DIM>(e, kc, m1);
  const float gscale = -itau[c] * kc.inv_cs2dt;      // grad P = gscale * m1
  const float gamma = -lwk_of(Sv, K[c], kc) * kc.inv_cs2dt;
  // 1/tau_g and the source weight dt (1 - 1/(2 tau_g)): uniform, or per node
  const float itg = kc.itg ? kc.itg[c] : kc.inv_tau_g;
  const float srcg = kc.itg ? kc.dt * (1.0f - 0.5f * itg) : kc.src_g;
  const float conv = gamma * kc.dt * kc.w1 * itg * kc.c * gscale;  // times s * m1[a]
  const float srcw = srcg * fs;
  // rest population
  {
    const float geq = (kc.geq0_phi + ph) * Sv;
    float o = gv[0] + (geq - gv[0]) * itg;
    if (HAS_FS) o += kc.w0 * srcw;
    gstore(gout.p[0], c, o, gdev<T>() ? geq_odd(kc, 0, Snc, ph) : 0.0f, kc);
  }
  const float geq = kc.w1beta * Sv;
  double flux = 0.0;
#pragma unroll
  for (int j = 0; j < 2 * DIM; ++j) {
    const int a = dir_axis(j), s = dir_sign(j);
    float o = gv[j + 1] + (geq - gv[j + 1]) * itg;
    if (HAS_FS) o += kc.w1 * srcw;
    o += conv * (float)s * m1[a];
    flux += g_push<T>(kc, gout, Sn, q, j, o, Sv, Snc);
  }
  return flux;
}

// The saturation step of the four nodes x0 .. x0 + 3 of a row (D2Q5, the
// pressure lattice in pull form, nx % 4 == 0; thread qi): per node the
// arithmetic of g_sweep_cell, with the pressure deviations pulled by the quad
// functions of the pressure sweep (the same values as load_e), the node data
// read and the rest and y-moving populations written as 4-wide vectors; the
// x-moving populations, and the y-moving ones of a row at a y face, go
// through g_push.  Every lane of the wavefront must call it (the pulls
// shuffle between lanes).
template <typename T, bool HAS_FS>
__device__ inline double g_sweep_quad(const KC &kc, const GPtrs &gin_, const GPtrs &gout_, const FP<T> &f,
                                      const float *__restrict__ Pb, const float *__restrict__ itau,
                                      const float *__restrict__ K, const float *__restrict__ phi,
                                      const float *__restrict__ Fs, const float *__restrict__ Sn, int qi) {
  const int n4 = kc.ncell >> 2;
  const bool active = qi < n4;
  const int c = (active ? qi : n4 - 1) << 2;     // first of the four nodes
  const int y = c / kc.nx;
  const int x0 = c - y * kc.nx;
  const float4 pb = *(const float4 *)(Pb + c);
  float4 e4[4];
  pull_x_quad<T>(kc, f, Pb, c, x0, y, 0, pb, e4[0], e4[2]);
  {
    float4 pbm = pb, pbp = pb;
    load_pb_axis(kc, Pb, c, 1, y, kc.ny, kc.nx, pbm, pbp);
    pull_axis_quad<T>(kc, f, c, 1, y, kc.ny, kc.nx, x0, 0, pb, pbm, pbp, e4[1], e4[3]);
  }
  if (!active) return 0.0;
  const GP<T> gin = gtyped<T>(gin_), gout = gtyped<T>(gout_);
  const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
  const float4 ph4 = *(const float4 *)(phi + c);
  const float4 B4 = gdev<T>() ? *(const float4 *)(gin.B + c) : zero;
  float4 g4[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) g4[i] = Vec4<T>::load(gin.p[i], c, kc.inv_g_scale);
  const float4 fs4 = HAS_FS ? *(const float4 *)(Fs + c) : zero;
  const float4 Sn4 = gdev<T>() ? *(const float4 *)(Sn + c) : zero;
  if (gdev<T>()) *(float4 *)(gout.B + c) = Sn4;
  const float4 it4 = *(const float4 *)(itau + c);
  const float4 K4 = *(const float4 *)(K + c);
  const float4 itg4 = kc.itg ? *(const float4 *)(kc.itg + c) : zero;
  // both y pushes land on rows of the domain (else g_push applies the y faces)
  const bool yin = y > 0 && y < kc.ny - 1;
  float4 Snm = zero, Snp = zero;
  if (gdev<T>() && yin) {
    Snm = *(const float4 *)(Sn + c - kc.nx);
    Snp = *(const float4 *)(Sn + c + kc.nx);
  }
  float4 out0 = zero, outp = zero, outm = zero;   // rest, +y, -y: what the vectors store
  double flux = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float ph = f4get(ph4, k), Bc = f4get(B4, k);
    float gv[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const float v = f4get(g4[i], k);
      gv[i] = gdev<T>() ? v + geq_odd(kc, i, Bc, ph) : v;
    }
    const float fs = HAS_FS ? f4get(fs4, k) : 0.0f;
    const float Snc = gdev<T>() ? f4get(Sn4, k) : 0.0f;
    const float Sv = saturation_of(sum_g<2>(gv), fs, ph, kc);
    const float e[4] = {f4get(e4[0], k), f4get(e4[1], k), f4get(e4[2], k), f4get(e4[3], k)};
    float m1[3];
    moment_c<2>(e, kc, m1);
    const float gscale = -f4get(it4, k) * kc.inv_cs2dt;
    const float gamma = -lwk_of(Sv, f4get(K4, k), kc) * kc.inv_cs2dt;
    const float itg = kc.itg ? f4get(itg4, k) : kc.inv_tau_g;
    const float srcg = kc.itg ? kc.dt * (1.0f - 0.5f * itg) : kc.src_g;
    const float conv = gamma * kc.dt * kc.w1 * itg * kc.c * gscale;
    const float srcw = srcg * fs;
    {
      const float geq = (kc.geq0_phi + ph) * Sv;
      float o = gv[0] + (geq - gv[0]) * itg;
      if (HAS_FS) o += kc.w0 * srcw;
      f4set(out0, k, gdev<T>() ? o - geq_odd(kc, 0, Snc, ph) : o);
    }
    const float geq = kc.w1beta * Sv;
    Cell q;
    q.c = c + k;
    q.x = x0 + k;
    q.y = y;
    q.z = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = dir_axis(j), s = dir_sign(j);
      float o = gv[j + 1] + (geq - gv[j + 1]) * itg;
      if (HAS_FS) o += kc.w1 * srcw;
      o += conv * (float)s * m1[a];
      if (a == 1 && yin) {
        if (s > 0) f4set(outp, k, gdev<T>() ? o - kc.w1beta * f4get(Snp, k) : o);
        else f4set(outm, k, gdev<T>() ? o - kc.w1beta * f4get(Snm, k) : o);
      } else {
        flux += g_push<T>(kc, gout, Sn, q, j, o, Sv, Snc);
      }
    }
  }
  Vec4<T>::store(gout.p[0], c, out0, kc.g_scale);
  if (yin) {
    Vec4<T>::store(gout.p[2], c + kc.nx, outp, kc.g_scale);   // +y (j = 1)
    Vec4<T>::store(gout.p[4], c - kc.nx, outm, kc.g_scale);   // -y (j = 3)
  }
  return flux;
}

// Central difference of u along axis a (one-sided second order at walls).
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

// f_i = w_i P0 - tau_f dt w_i c_i . grad P0 (i >= 1): base P_b = P0 and local
// deviations e_i = -tau_f dt w_i c_i . grad P0.
// g_i = g_i^eq(S0) + eps g_i^(1) with
// eps g_i^(1) = -tau_g dt [(Gamma_i/phi - w_i(1 - 1/(2 tau_g))) F_s
//                          + Gamma_i c_i . grad S0 - gamma w_i c_i . grad P0 / tau_g]
// (eq. gini, gneq), Gamma_i = g_i^eq / S.
template <int DIM, typename T>
__device__ inline void init_cell(const KC &kc, const float *__restrict__ P0, const float *__restrict__ S0,
                                 const float *__restrict__ dP0, const float *__restrict__ dS0,
                                 const float *__restrict__ K, const float *__restrict__ phi,
                                 const float *__restrict__ Fs, int neq, const FP<T> &f, float *__restrict__ Pb,
                                 const GPtrs &g_, int c) {
  const Cell q = cell_of(c, kc);
  const GP<T> g = gtyped<T>(g_);
  const float P = P0[c], S = S0[c], ph = phi[c];
  const float fs = Fs ? Fs[c] : 0.0f;
  float gp[3] = {0.f, 0.f, 0.f}, gs[3] = {0.f, 0.f, 0.f};
  if (neq) {
    const float inv2dx = 0.5f / (kc.c * kc.dt);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      gp[a] = dP0 ? dP0[a * kc.ncell + c] : cdiff(P0, q, a, kc, inv2dx);
      gs[a] = dS0 ? dS0[a * kc.ncell + c] : cdiff(S0, q, a, kc, inv2dx);
    }
  }
  const float itf = inv_tau_f_of(S, K[c], kc);
  const float tau_f = 1.0f / itf;
  const float gamma = -lwk_of(S, K[c], kc) * kc.inv_cs2dt;
  const float itg = kc.cap_B > 0.0f ? inv_tau_g_of(S, K[c], kc) : kc.inv_tau_g;
  const float tau_g = 1.0f / itg;
  const float wsrc = 1.0f - 0.5f * itg;
  Pb[c] = P;
#pragma unroll
  for (int j = 0; j < 2 * DIM; ++j) {
    const int a = dir_axis(j), s = dir_sign(j);
    const float cdp = (float)s * kc.c * gp[a];
    Storage<T>::store(f.p[j], c, neq ? -tau_f * kc.dt * kc.w1 * cdp : 0.0f, kc.dev_scale);
  }
  // rest population: Gamma_0 = (w0 - 1) beta + phi, c_0 = 0
  {
    const float G0 = kc.geq0_phi + ph;
    float v = G0 * S;
    if (neq) v -= tau_g * kc.dt * ((G0 / ph - kc.w0 * wsrc) * fs);
    if (gdev<T>()) g.B[c] = S;
    gstore(g.p[0], c, v, gdev<T>() ? geq_odd(kc, 0, S, ph) : 0.0f, kc);
  }
  const float G = kc.w1beta;
#pragma unroll
  for (int j = 0; j < 2 * DIM; ++j) {
    const int a = dir_axis(j), s = dir_sign(j);
    float v = G * S;
    if (neq) {
      const float cdp = (float)s * kc.c * gp[a];
      const float cds = (float)s * kc.c * gs[a];
      v -= tau_g * kc.dt * ((G / ph - kc.w1 * wsrc) * fs + G * cds - gamma * kc.w1 * cdp * itg);
    }
    gstore(g.p[j + 1], c, v, gdev<T>() ? kc.w1beta * S : 0.0f, kc);
  }
}

}  // namespace
}  // namespace lbtp
