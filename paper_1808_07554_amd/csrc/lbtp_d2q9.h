// Device functions of the D2Q9 lattice (the paper's own, Section 3, eq. 3-5,
// 3-6), shared by the single-context kernels (lbtp_d2q9.hip) and the
// ensemble kernels (lbtp_batch.hip): the lattice tables, the pulls with their
// wall rules, the collisions, the per-node and four-node pressure sweeps, the
// moments and the saturation step of one node.  Conventions as in
// lbtp_d2q9.hip.
#ifndef LBTP_D2Q9_H
#define LBTP_D2Q9_H

#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "lbtp_device.h"

namespace lbtp {
namespace {

__device__ constexpr int q9x(int j) { return (j == 0 || j == 4 || j == 7) ? 1 : ((j == 2 || j == 5 || j == 6) ? -1 : 0); }
__device__ constexpr int q9y(int j) { return (j == 1 || j == 4 || j == 5) ? 1 : ((j == 3 || j == 6 || j == 7) ? -1 : 0); }
__device__ constexpr int q9opp(int j) { return j < 4 ? (j + 2) & 3 : 4 + ((j - 2) & 3); }
__device__ inline float q9w(const KC &kc, int j) { return j < 4 ? kc.w1 : kc.w2; }

// Gamma_j = g^eq / S of moving direction j (eq. 3-4 with C = (beta - phi) I).
__device__ inline float q9_gamma(const KC &kc, int j, float phi) {
  return j < 4 ? kc.w1 * (phi + 0.5f * (kc.beta - phi)) : kc.w2 * (phi + 2.0f * (kc.beta - phi));
}
__device__ inline float q9_gamma0(const KC &kc, float phi) { return kc.w0 * (phi - (kc.beta - phi)); }

// Face a link leaving node (x, y) along (ex, ey) crosses (push view, faces
// -x, +x, -y, +y = 0..3), or -1 if it stays inside or wraps across periodic
// faces.  Where it leaves through both an x and a y face the y face counts.
__device__ inline int q9_exit_face(const KC &kc, const int *bc, int x, int y, int ex, int ey) {
  const bool outy = ey > 0 ? y == kc.ny - 1 : (ey < 0 ? y == 0 : false);
  const bool outx = ex > 0 ? x == kc.nx - 1 : (ex < 0 ? x == 0 : false);
  const int fy = ey > 0 ? 3 : 2, fx = ex > 0 ? 1 : 0;
  if (outy && bc[fy] != LBTP_BC_PERIODIC) return fy;
  if (outx && bc[fx] != LBTP_BC_PERIODIC) return fx;
  return -1;
}

__device__ inline int q9_wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Slot of a link in the per-link wall data of a face (three per node): 0 for
// the normal link, 1 / 2 for the diagonal whose arriving population has
// tangential velocity -1 / +1.
__device__ inline int q9_wall_slot(int face, int ax, int ay) {
  const int t = face < 2 ? ay : ax;
  return t == 0 ? 0 : (t < 0 ? 1 : 2);
}

// Condition of one link of a face: the per-link list if one is set
// (lbtp_set_wall_types), else the face's own.  along = y on the x faces, x
// on the y faces; slot as in q9_wall_slot.
__device__ inline int q9_link_bc(const int *bc, const int *const *wt, int face, int along, int slot) {
  const int *t = wt[face];
  return t ? t[along * 3 + slot] : bc[face];
}

// Pre-collision deviations e_j at node c = (x, y) against P_b(c) = pb:
// streamed from (x - e_x, y - e_y) (eq. 3-1) and re-expressed against the
// node's base, or the Section 4 rule of the wall the link comes through:
// anti-bounce-back e_j = 2 w_j (P_w - pb) - d_opp(c), bounce-back d_opp(c).
template <typename T, bool LOCAL>
__device__ inline void q9_load_e(const FP<T> &fin, const float *__restrict__ Pb, int c, int x, int y, const KC &kc,
                                 float pb, float *e) {
  const float is = kc.inv_dev_scale;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (LOCAL) {
      e[j] = Storage<T>::load(fin.p[j], c, is);
      continue;
    }
    const int ex = q9x(j), ey = q9y(j);
    // the pull source lies beyond the face the opposite link leaves through
    const int face = q9_exit_face(kc, kc.bc_f, x, y, -ex, -ey);
    const float w = q9w(kc, j);
    if (face < 0) {
      const int src = q9_wrap(y - ey, kc.ny) * kc.nx + q9_wrap(x - ex, kc.nx);
      e[j] = Storage<T>::load(fin.p[j], src, is) + w * (Pb[src] - pb);
    } else {
      const float o = Storage<T>::load(fin.p[q9opp(j)], c, is);
      const int slot = q9_wall_slot(face, ex, ey);
      e[j] = (q9_link_bc(kc.bc_f, kc.wtF, face, face < 2 ? y : x, slot) == LBTP_BC_DIRICHLET)
                 ? (2.0f * w * (wall_P(kc, face, x, y, 0, 3, slot) - pb) - o)
                 : o;
    }
  }
}

// Sum of the deviations of the moving directions; P - P_b is this sum over
// 1 - w0 (eq. 3-9a).
__device__ inline float q9_dsum(const float *e) {
  float s = e[0];
#pragma unroll
  for (int j = 1; j < 8; ++j) s += e[j];
  return s;
}

__device__ inline float q9_dpressure(const float *e, const KC &kc) { return q9_dsum(e) * kc.inv_1mw0; }

// sum_j c_j e_j (the base part cancels: sum_j w_j c_j = 0)
__device__ inline void q9_moment(const float *e, const KC &kc, float *m1) {
  float mx = 0.f, my = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (q9x(j)) mx += (float)q9x(j) * e[j];
    if (q9y(j)) my += (float)q9y(j) * e[j];
  }
  m1[0] = kc.c * mx;
  m1[1] = kc.c * my;
}

__device__ inline float q9_sum_g(const float *g) {
  float s = g[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) s += g[i];
  return s;
}

// Collision of the pressure lattice: o_j = e_j minus the relaxation of the
// non-equilibrium part n_j = e_j - w_j dP (the base part of f^eq cancels in
// the deviation form).  BGK: n_j / tau_f.  MRT: M^-1 S M n with the
// orthogonal D2Q9 basis (rows rho, e, epsilon, j_x, q_x, j_y, q_y, p_xx,
// p_xy; squared norms 9, 36, 36, 6, 12, 6, 12, 4, 4).  With rho, e and epsilon
// at one rate s0, M^-1 S M = s0 I + M^-1 (S - s0 I) M, and the second term
// only involves the flux and stress moments, none of which sees the rest
// population; it is written out here moment by moment.
__device__ inline void q9_collide(const KC &kc, bool mrt, const float *e, float sum, float it, float *o) {
  if (!mrt) {
    // e_j + (w_j dP - e_j) / tau_f as e_j (1 - 1/tau_f) + (w_j dP) / tau_f,
    // one fused multiply-add per population (every sweep kernel calls this);
    // w_j dP is the sum of the deviations times w_j / (1 - w0)
    const float keep = 1.0f - it;
    const float g1 = (sum * (kc.w1 * kc.inv_1mw0)) * it, g2 = (sum * (kc.w2 * kc.inv_1mw0)) * it;
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = __builtin_fmaf(e[j], keep, j < 4 ? g1 : g2);
    return;
  }
  const float dP = sum * kc.inv_1mw0;
  float n[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) n[j] = e[j] - q9w(kc, j) * dP;
  // directions j = 0..7: +x, +y, -x, -y, (1,1), (-1,1), (-1,-1), (1,-1)
  const float jx = n[0] - n[2] + n[4] - n[5] - n[6] + n[7];
  const float qx = -2.0f * n[0] + 2.0f * n[2] + n[4] - n[5] - n[6] + n[7];
  const float jy = n[1] - n[3] + n[4] + n[5] - n[6] - n[7];
  const float qy = -2.0f * n[1] + 2.0f * n[3] + n[4] + n[5] - n[6] - n[7];
  const float pxx = n[0] - n[1] + n[2] - n[3];
  const float pxy = n[4] - n[5] + n[6] - n[7];
  const float s0 = kc.ms0;
  const float ajx = (it - s0) * jx * (1.0f / 6.0f), ajy = (it - s0) * jy * (1.0f / 6.0f);
  const float aqx = (kc.msq - s0) * qx * (1.0f / 12.0f), aqy = (kc.msq - s0) * qy * (1.0f / 12.0f);
  const float apxx = (kc.msp - s0) * pxx * 0.25f, apxy = (kc.msp - s0) * pxy * 0.25f;
  float d[8];
  d[0] = ajx - 2.0f * aqx + apxx;
  d[1] = ajy - 2.0f * aqy - apxx;
  d[2] = -ajx + 2.0f * aqx + apxx;
  d[3] = -ajy + 2.0f * aqy - apxx;
  d[4] = ajx + aqx + ajy + aqy + apxy;
  d[5] = -ajx - aqx + ajy + aqy - apxy;
  d[6] = -ajx - aqx - ajy - aqy + apxy;
  d[7] = ajx + aqx - ajy - aqy - apxy;
#pragma unroll
  for (int j = 0; j < 8; ++j) o[j] = e[j] - (s0 * n[j] + d[j]);
}

// ------------------------------------------------------------ pressure sweep
// One iteration of eq. 3-1 at node c; MODE as in the D2Q5 sweeps (0 plain,
// 1 re-base, 2 re-base and stopping-rule terms, added to acc).
template <typename T, bool LOCAL, int MODE, bool HAS_FP>
__device__ inline void q9_sweep_cell(const KC &kc, const FP<T> &fin, const FP<T> &fout,
                                     const float *__restrict__ Pb_in, float *__restrict__ Pb_out,
                                     const float *__restrict__ itau, const float *__restrict__ Fp, int c,
                                     double *acc) {
  const int y = c / kc.nx, x = c - y * kc.nx;
  const float pb = Pb_in[c];
  float e[8];
  q9_load_e<T, LOCAL>(fin, Pb_in, c, x, y, kc, pb, e);
  const float sum = q9_dsum(e), dP = sum * kc.inv_1mw0;
  const float it = itau[c];
  const float add = HAS_FP ? kc.dt * kc.wbar * Fp[c] : 0.0f;
  float rb = 0.0f;
  if (MODE >= 1) {
    const float P = pb + dP;
    rb = pb - P;                      // re-base to P_b = P (exact difference)
    Pb_out[c] = P;
    if (MODE == 2) {
      acc[0] += (double)dP * (double)dP;
      acc[1] += (double)P * (double)P;
    }
  }
  float oc[8];
  q9_collide(kc, kc.mrt, e, sum, it, oc);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float w = q9w(kc, j);
    float o = oc[j];
    if (HAS_FP) o += add;
    if (MODE >= 1) o += w * rb;
    Storage<T>::store(fout.p[j], c, o, kc.dev_scale);
  }
}

// ------------------------------------------- pressure sweep, 4 nodes / thread
// The same sweep with each thread owning four consecutive nodes of a row
// (nx % 4 == 0): every population and base row moves as one vector; values
// from x - 1 / x + 1 come from the adjacent lane (shuffles) or, at a
// wavefront edge, from one scalar load.  Every lane runs every shuffle.

// 4-vector of the node-wise Dirichlet pressures of a y face for slot k.
__device__ inline float4 q9_wall_P4(const KC &kc, int face, int x0, int k) {
  const float *a = kc.wP[face];
  if (!a) {
    const float pw = kc.Pw[face];
    return make_float4(pw, pw, pw, pw);
  }
  return make_float4(a[(x0 + 0) * 3 + k], a[(x0 + 1) * 3 + k], a[(x0 + 2) * 3 + k], a[(x0 + 3) * 3 + k]);
}

// Source rows of the y-moving populations of the quad at (x0, y): ey = +1
// pulls from row y - 1, ey = -1 from row y + 1 (wrapped across a periodic
// face); *_has = false means the row lies beyond a wall (the y-face rule).
struct Q9Rows {
  bool lo_has, hi_has;
  int c_lo, c_hi;   // first node of the quad in the source rows
};

__device__ inline Q9Rows q9_rows(const KC &kc, int x0, int y) {
  Q9Rows r;
  const bool lo_in = y > 0, hi_in = y < kc.ny - 1;
  r.lo_has = lo_in || kc.bc_f[2] == LBTP_BC_PERIODIC;
  r.hi_has = hi_in || kc.bc_f[3] == LBTP_BC_PERIODIC;
  r.c_lo = (lo_in ? y - 1 : kc.ny - 1) * kc.nx + x0;
  r.c_hi = (hi_in ? y + 1 : 0) * kc.nx + x0;
  return r;
}

// The quad's update given its base pb and the bases of its source rows.
template <typename T, int MODE, bool HAS_FP>
__device__ inline void q9_quad_core(const KC &kc, const FP<T> &fin, const FP<T> &fout,
                                    const float *__restrict__ Pb_in, float *__restrict__ Pb_out,
                                    const float *__restrict__ itau, const float *__restrict__ Fp, int c, int x0,
                                    int y, bool active, const Q9Rows &R, const float4 &pb, const float4 &pb_lo,
                                    const float4 &pb_hi, double *acc) {
  const int lane = threadIdx.x & 63;
  const float is = kc.inv_dev_scale;
  const bool lo_has = R.lo_has, hi_has = R.hi_has;
  const int c_lo = R.c_lo, c_hi = R.c_hi;
  float4 e[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int ex = q9x(j), ey = q9y(j);
    const float w = q9w(kc, j);
    const bool has = ey == 0 ? true : (ey > 0 ? lo_has : hi_has);
    const int cs = ey == 0 ? c : (ey > 0 ? c_lo : c_hi);
    const float4 P = ey == 0 ? pb : (ey > 0 ? pb_lo : pb_hi);
    // the source row as loaded by this lane (a valid address for every lane)
    const float4 V = Vec4<T>::load(fin.p[j], has ? cs : c, is);
    // elements at x - 1 (ex = +1) or x + 1 (ex = -1) of the neighbouring lanes
    float vn = 0.f, pn = 0.f;
    if (ex > 0) {
      vn = __shfl_up(V.w, 1, 64);
      pn = __shfl_up(P.w, 1, 64);
      if (lane == 0 && x0 > 0 && has) {
        vn = Storage<T>::load(fin.p[j], cs - 1, is);
        pn = Pb_in[cs - 1];
      }
    } else if (ex < 0) {
      vn = __shfl_down(V.x, 1, 64);
      pn = __shfl_down(P.x, 1, 64);
      if (lane == 63 && x0 + 4 < kc.nx && has) {
        vn = Storage<T>::load(fin.p[j], cs + 4, is);
        pn = Pb_in[cs + 4];
      }
    }
    if (!has) {
      // the whole quad takes the y-face rule (it also wins at the corners)
      const int face = ey > 0 ? 2 : 3;
      const int slot = q9_wall_slot(face, ex, ey);
      const float4 o = Vec4<T>::load(fin.p[q9opp(j)], c, is);
      if (kc.wtF[face]) {
        // conditions link by link
        const float4 pw = q9_wall_P4(kc, face, x0, slot);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool abb = kc.wtF[face][(x0 + i) * 3 + slot] == LBTP_BC_DIRICHLET;
          f4set(e[j], i, abb ? 2.0f * w * (f4get(pw, i) - f4get(pb, i)) - f4get(o, i) : f4get(o, i));
        }
      } else if (kc.bc_f[face] == LBTP_BC_DIRICHLET) {
        const float4 pw = q9_wall_P4(kc, face, x0, slot);
        e[j] = make_float4(2.0f * w * (pw.x - pb.x) - o.x, 2.0f * w * (pw.y - pb.y) - o.y,
                           2.0f * w * (pw.z - pb.z) - o.z, 2.0f * w * (pw.w - pb.w) - o.w);
      } else {
        e[j] = o;
      }
      continue;
    }
    float4 src, psrc;
    if (ex == 0) {
      src = V;
      psrc = P;
    } else if (ex > 0) {
      src = make_float4(vn, V.x, V.y, V.z);
      psrc = make_float4(pn, P.x, P.y, P.z);
    } else {
      src = make_float4(V.y, V.z, V.w, vn);
      psrc = make_float4(P.y, P.z, P.w, pn);
    }
    e[j] = make_float4(src.x + w * (psrc.x - pb.x), src.y + w * (psrc.y - pb.y), src.z + w * (psrc.z - pb.z),
                       src.w + w * (psrc.w - pb.w));
    // x faces: node 0 (ex = +1, x0 == 0) or node 3 (ex = -1, x0 + 4 == nx)
    if (ex > 0 && x0 == 0) {
      if (kc.bc_f[0] == LBTP_BC_PERIODIC) {
        const int s0 = cs + kc.nx - 1;
        e[j].x = Storage<T>::load(fin.p[j], s0, is) + w * (Pb_in[s0] - pb.x);
      } else {
        const float o = Storage<T>::load(fin.p[q9opp(j)], c, is);
        const int slot = q9_wall_slot(0, ex, ey);
        e[j].x = q9_link_bc(kc.bc_f, kc.wtF, 0, y, slot) == LBTP_BC_DIRICHLET
                     ? 2.0f * w * (wall_P(kc, 0, 0, y, 0, 3, slot) - pb.x) - o
                     : o;
      }
    } else if (ex < 0 && x0 + 4 == kc.nx) {
      if (kc.bc_f[1] == LBTP_BC_PERIODIC) {
        const int s3 = cs + 3 - (kc.nx - 1);
        e[j].w = Storage<T>::load(fin.p[j], s3, is) + w * (Pb_in[s3] - pb.w);
      } else {
        const float o = Storage<T>::load(fin.p[q9opp(j)], c + 3, is);
        const int slot = q9_wall_slot(1, ex, ey);
        e[j].w = q9_link_bc(kc.bc_f, kc.wtF, 1, y, slot) == LBTP_BC_DIRICHLET
                     ? 2.0f * w * (wall_P(kc, 1, kc.nx - 1, y, 0, 3, slot) - pb.w) - o
                     : o;
      }
    }
  }
  // collision, re-basing and stopping-rule terms, as in the one-node kernel
  const float4 it = *(const float4 *)(itau + c);
  float4 fp = make_float4(0.f, 0.f, 0.f, 0.f);
  if (HAS_FP) fp = *(const float4 *)(Fp + c);
  float4 o[8];
  float4 pnew;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float ev[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) ev[j] = f4get(e[j], i);
    const float sum = q9_dsum(ev), dP = sum * kc.inv_1mw0;
    const float t = f4get(it, i);
    const float add = HAS_FP ? kc.dt * kc.wbar * f4get(fp, i) : 0.0f;
    float rb = 0.0f;
    if (MODE >= 1) {
      const float pbi = f4get(pb, i);
      const float P = pbi + dP;
      rb = pbi - P;
      f4set(pnew, i, P);
      if (MODE == 2 && active) {
        acc[0] += (double)dP * (double)dP;
        acc[1] += (double)P * (double)P;
      }
    }
    float oc[8];
    q9_collide(kc, kc.mrt, ev, sum, t, oc);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float w = q9w(kc, j);
      float v = oc[j];
      if (HAS_FP) v += add;
      if (MODE >= 1) v += w * rb;
      f4set(o[j], i, v);
    }
  }
  if (active) {
#pragma unroll
    for (int j = 0; j < 8; ++j) Vec4<T>::store(fout.p[j], c, o[j], kc.dev_scale);
    if (MODE >= 1) *(float4 *)(Pb_out + c) = pnew;
  }
}

template <typename T, int MODE, bool HAS_FP>
__device__ inline void q9_sweep_quad(const KC &kc, const FP<T> &fin, const FP<T> &fout,
                                     const float *__restrict__ Pb_in, float *__restrict__ Pb_out,
                                     const float *__restrict__ itau, const float *__restrict__ Fp, int qi,
                                     double *acc) {
  const int n4 = kc.ncell >> 2;
  const bool active = qi < n4;
  const int c = (active ? qi : n4 - 1) << 2;
  const int y = c / kc.nx;
  const int x0 = c - y * kc.nx;
  const Q9Rows R = q9_rows(kc, x0, y);
  const float4 pb = *(const float4 *)(Pb_in + c);
  const float4 pb_lo = R.lo_has ? *(const float4 *)(Pb_in + R.c_lo) : pb;
  const float4 pb_hi = R.hi_has ? *(const float4 *)(Pb_in + R.c_hi) : pb;
  q9_quad_core<T, MODE, HAS_FP>(kc, fin, fout, Pb_in, Pb_out, itau, Fp, c, x0, y, active, R, pb, pb_lo, pb_hi,
                                acc);
}

// ------------------------------------------------------------------ moments
// g_i^eq(B) of eq. 3-4 for population i (0 rest, j + 1 moving) at porosity phi.
__device__ inline float q9_geq(const KC &kc, int i, float B, float phi) {
  return (i == 0 ? q9_gamma0(kc, phi) : q9_gamma(kc, i - 1, phi)) * B;
}

// S^n (eq. 3-9b) and 1/tau_f at node c; returns the node's mass in float64.
template <bool HAS_FS, typename TG>
__device__ inline double q9_moments_cell(const KC &kc, const GPtrs &g_, const float *__restrict__ K,
                                         const float *__restrict__ phi, const float *__restrict__ Fs,
                                         float *__restrict__ S, float *__restrict__ itau, int c, int write_coef) {
  const GP<TG> g = gtyped<TG>(g_);
  const float ph = phi[c], B = gdev<TG>() ? g.B[c] : 0.0f;
  float gv[9];
  double dm = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    gv[i] = gload(g.p[i], c, gdev<TG>() ? q9_geq(kc, i, B, ph) : 0.0f, kc);
    dm += (double)gv[i];
  }
  const float fs = HAS_FS ? Fs[c] : 0.0f;
  const float Sv = saturation_of(q9_sum_g(gv), fs, ph, kc);
  if (write_coef) {
    S[c] = Sv;
    itau[c] = inv_tau_f_of(Sv, K[c], kc);
    if (kc.itg) kc.itg[c] = inv_tau_g_of(Sv, K[c], kc);
  }
  if (HAS_FS) dm += 0.5 * (double)kc.dt * (double)fs;
  return dm;
}

// ---------------------------------------------------------- saturation sweep
// eq. 3-2 with g^eq of eq. 3-4, the local grad P of eq. 3-10a and
// gamma = -lambda_w K / (c_s^2 dt) at node c; push to x + c_i or reflect at
// walls (anti-bounce-back with g^eq(S_b, phi(x)), S_b the face value or, for
// an outflow face, S of the node; bounce-back for no-flux faces).  With
// 16-bit storage the populations are read against the input's base and
// written as deviations from g^eq(S^n, phi) of the node written (Sn; the
// output's base).  Returns the net flux through reflected links.
template <typename T, bool FLOCAL, bool HAS_FS>
__device__ inline double q9_g_sweep_cell(const KC &kc, const GPtrs &gin_, const GPtrs &gout_, const FP<T> &f,
                                         const float *__restrict__ Pb, const float *__restrict__ itau,
                                         const float *__restrict__ K, const float *__restrict__ phi,
                                         const float *__restrict__ Fs, const float *__restrict__ Sn, int c) {
  const int y = c / kc.nx, x = c - y * kc.nx;
  const GP<T> gin = gtyped<T>(gin_), gout = gtyped<T>(gout_);
  const float ph = phi[c];
  const float Bc = gdev<T>() ? gin.B[c] : 0.0f;
  float gv[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) gv[i] = gload(gin.p[i], c, gdev<T>() ? q9_geq(kc, i, Bc, ph) : 0.0f, kc);
  const float fs = HAS_FS ? Fs[c] : 0.0f;
  const float Snc = gdev<T>() ? Sn[c] : 0.0f;
  if (gdev<T>()) gout.B[c] = Snc;
  const float Sv = saturation_of(q9_sum_g(gv), fs, ph, kc);
  float e[8];
  q9_load_e<T, FLOCAL>(f, Pb, c, x, y, kc, Pb[c], e);
  float m1[2];
  q9_moment(e, kc, m1);
  const float gscale = -itau[c] * kc.inv_cs2dt;       // grad P = gscale * m1
  const float gx = gscale * m1[0], gy = gscale * m1[1];
  const float gamma = -lwk_of(Sv, K[c], kc) * kc.inv_cs2dt;
  const float itg = kc.itg ? kc.itg[c] : kc.inv_tau_g;
  const float srcg = kc.itg ? kc.dt * (1.0f - 0.5f * itg) : kc.src_g;
  const float conv = gamma * kc.dt * itg;     // times w_i c_i . grad P
  const float srcw = srcg * fs;
  {
    const float geq = q9_gamma0(kc, ph) * Sv;
    float o = gv[0] + (geq - gv[0]) * itg;
    if (HAS_FS) o += kc.w0 * srcw;
    gstore(gout.p[0], c, o, gdev<T>() ? q9_geq(kc, 0, Snc, ph) : 0.0f, kc);
  }
  double flux = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int ex = q9x(j), ey = q9y(j);
    const float w = q9w(kc, j);
    const float G = q9_gamma(kc, j, ph);
    float o = gv[j + 1] + (G * Sv - gv[j + 1]) * itg;
    if (HAS_FS) o += w * srcw;
    o += conv * w * (kc.c * ((float)ex * gx + (float)ey * gy));
    const int face = q9_exit_face(kc, kc.bc_g, x, y, ex, ey);
    if (face < 0) {
      const int d = q9_wrap(y + ey, kc.ny) * kc.nx + q9_wrap(x + ex, kc.nx);
      gstore(gout.p[j + 1], d, o, gdev<T>() ? q9_geq(kc, j + 1, Sn[d], phi[d]) : 0.0f, kc);
    } else {
      const int slot = q9_wall_slot(face, -ex, -ey);
      const int bc = q9_link_bc(kc.bc_g, kc.wtG, face, face < 2 ? y : x, slot);
      float r;
      if (bc == LBTP_BC_NOFLUX) r = o;
      else if (bc == LBTP_BC_DIRICHLET) r = 2.0f * G * wall_S(kc, face, x, y, 0, 3, slot) - o;
      else r = 2.0f * G * Sv - o;      // outflow: S_b = S of this node
      gstore(gout.p[q9opp(j) + 1], c, r, gdev<T>() ? q9_geq(kc, q9opp(j) + 1, Snc, ph) : 0.0f, kc);
      flux += (double)r - (double)o;
    }
  }
  return flux;
}

}  // namespace
}  // namespace lbtp

#endif  // LBTP_D2Q9_H
