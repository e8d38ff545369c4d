// Temporal blocking of the plain D3Q7 pressure sweep (gfx950): H plain sweeps
// (eq. 3-1, no re-basing, no stopping-rule terms) per launch, streaming along z.
//
// A workgroup of kZW wavefronts owns a column of the box, 64 x-columns (one
// per lane) by kZW y-rows (one per wavefront), and walks it along a segment
// of z with the H sweep levels pipelined.  At each step it takes one new
// plane of the state before the launch (level 0), and level s turns planes
// p - 1, p, p + 1 of level s - 1 into plane p = z - (2s - 1) of level s,
// where z is the plane just taken.  A level reads only planes that earlier
// steps made (the levels are skewed by two planes), so the H levels of a step
// are independent of each other.  The x-moving populations come from the
// adjacent lanes (wavefront shifts), the y-moving ones from the adjacent
// wavefronts through LDS (one exchange and one barrier per step), the
// z-moving ones from the lane's own registers.  Per level a lane keeps the
// plane the level sweeps next, the +z population of the plane below it and
// the plane above it; the per-plane constants (the base differences
// w (P_b(src) - P_b(node)) along -x, +-y and -z, 1/tau_f, P_b) sit in rings
// of 2H planes (the y-neighbours' bases come through LDS with the populations),
// and the step loop is unrolled by 2H so that every
// ring slot is named at compile time.  Only the nodes at least H links from
// the column's cut x and y edges, in the planes of the workgroup's own
// segment, are written; the neighbouring columns and segments recompute the
// halo.  Walls on any face are applied where they are met, with the rules of
// the one-sweep kernel (anti-bounce-back with the face's or the link's
// pressure, bounce-back).
//
// A register-resident region (the D2Q5 design) does not carry over to 3-D:
// a region that fits the registers of a workgroup keeps too small a share of
// its nodes after H sweeps when it is cut on four faces instead of two.
//
// Arithmetic and its order are those of sweep_cell (lbtp_device.h) for a
// plain sweep: float32 storage gives bitwise the populations of H single
// sweeps.  16-bit storage rounds to its format once per launch.
#include <math.h>
#include <stdint.h>

#include <atomic>

#include "lbtp_device.h"

namespace lbtp {
namespace {

constexpr int kZW = 16;     // wavefronts (y-rows) per workgroup
constexpr int kZBX = 64;    // x-columns: one per lane
constexpr int kZPF = 2;     // planes loaded ahead of the one being taken

struct ZGeom {
  int tiles_x, tiles_y, segs, seg;
};

__device__ inline int z_wrap(int v, int n) {
  const int r = v % n;
  return r < 0 ? r + n : r;
}
__device__ inline int z_clamp(int v, int n) { return v < 0 ? 0 : (v > n - 1 ? n - 1 : v); }
// Element i of an array, addressed by a 32-bit byte offset from its base (a
// context holds fewer than 2^31 populations, so no array reaches 4 GiB).
template <typename T>
__device__ inline T *z_at(T *p, uint32_t i) {
  return (T *)((char *)p + i * (uint32_t)sizeof(T));
}
template <typename T>
__device__ inline const T *z_at(const T *p, uint32_t i) {
  return (const T *)((const char *)p + i * (uint32_t)sizeof(T));
}

// Anti-bounce-back / bounce-back value of the population arriving through
// wall face `face` at the node whose opposite population is o (load_e).
__device__ inline float z_wall_rule(const KC &kc, int face, int x, int y, int z, float pb, float o) {
  return kc.bc_f[face] == LBTP_BC_DIRICHLET ? 2.0f * kc.w1 * (wall_P(kc, face, x, y, z, 1, 0) - pb) - o : o;
}

template <typename T, bool HAS_FP, int H>
__global__ __launch_bounds__(kZBX * kZW) void f_zstream_kernel(KC kc, FPtrs fin_, FPtrs fout_,
                                                               const float *__restrict__ Pb,
                                                               const float *__restrict__ itau,
                                                               const float *__restrict__ Fp,
                                                               const Ctl *__restrict__ ctl, long long k, ZGeom g) {
  constexpr int M = 2 * H;   // ring length
  constexpr int PF = kZPF;
  static_assert(H % 2 == 1 && M % PF == 0, "H odd, the prefetch period divides the ring");
  static_assert(kZW - 2 * H >= 2, "rows left after the halo");
  if (ctl->done || k > ctl->kmax) return;   // uniform over the grid
  __shared__ float xup[2][H][kZW][kZBX];    // +y population of each row, per level (step parity)
  __shared__ float xdn[2][H][kZW][kZBX];    // -y population
  __shared__ float xpb[2][kZW][kZBX];       // P_b of the plane just taken
  const FP<T> fin = typed<T>(fin_), fout = typed<T>(fout_);
  const float is = kc.inv_dev_scale;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nx = kc.nx, ny = kc.ny, nz = kc.nz;
  int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int tx = t % g.tiles_x;
  t /= g.tiles_x;
  const int ty = t % g.tiles_y, seg = t / g.tiles_y;
  const bool perx = kc.bc_f[0] == LBTP_BC_PERIODIC, pery = kc.bc_f[2] == LBTP_BC_PERIODIC,
             perz = kc.bc_f[4] == LBTP_BC_PERIODIC;
  const int ux = tx * (kZBX - 2 * H) - H + lane;   // this lane's column (unwrapped)
  const int uy = ty * (kZW - 2 * H) - H + wv;      // this wavefront's row (unwrapped)
  const int gx = perx ? z_wrap(ux, nx) : z_clamp(ux, nx);
  const int gy = pery ? z_wrap(uy, ny) : z_clamp(uy, ny);
  const int zs = seg * g.seg, ze = min(zs + g.seg, nz);
  const int z0 = zs - H;                                   // plane taken at step 0 (unwrapped)
  const int nsteps = (ze - zs + 3 * H - 1 + M - 1) / M * M;
  const bool keep_node = lane >= H && lane < kZBX - H && ux < nx && wv >= H && wv < kZW - H && uy < ny;
  // wall nodes: x faces per lane (and whether the column holds any), y faces per wavefront
  const bool wall_l = !perx && ux == 0, wall_r = !perx && ux == nx - 1;
  const int ux0 = tx * (kZBX - 2 * H) - H;
  const bool xwalls = !perx && (ux0 <= 0 || ux0 + kZBX > nx - 1);
  const bool wall_b = !pery && uy == 0, wall_t = !pery && uy == ny - 1;
  const float wsrc = kc.dt * kc.wbar;
  const int plane = nx * ny;

  // one plane of the state before the launch at this lane's (x, y): every
  // load is issued (clamped to the box where the lane, row or plane lies
  // outside a walled axis; such values never reach a node of the box)
  // plane index of unwrapped plane uz on a periodic z axis; the value is made
  // opaque so that the modulo is formed only where it is used (periodic z,
  // wall planes), not for every plane and level
  auto zwrap = [&](int uz) {
    asm volatile("" : "+s"(uz));
    return z_wrap(uz, nz);
  };
  const uint32_t col = (uint32_t)(gy * nx + gx);
  auto load_plane = [&](int uz, float (&d)[6], float &pb, float &it) {
    const int gz = perz ? zwrap(uz) : z_clamp(uz, nz);
    const uint32_t c = (uint32_t)gz * (uint32_t)plane + col;
#pragma unroll
    for (int j = 0; j < 6; ++j) d[j] = Storage<T>::load(z_at(fin.p[j], c), 0, is);
    pb = *z_at(Pb, c);
    it = *z_at(itau, c);
  };

  float cur[H + 1][6];   // level s: plane p_s of level s - 1 (p_s = the plane level s sweeps next)
  float up[H + 1];       // level s: +z population of plane p_s - 1 of level s - 1
  float fr[H + 1][6];    // level s >= 2: plane p_s + 1 of level s - 1, made at the previous step
  // per-plane constants: w (P_b(x-1) - P_b), w (P_b(y-1) - P_b), w (P_b(y+1) - P_b),
  // w (P_b(z-1) - P_b), 1/tau_f, P_b (the source, if any, is read where it is added)
  float apx[M], apym[M], apyp[M], apz[M], itr[M], pbr[M];
  float pfd[PF][6], pfpb[PF], pfit[PF];
#pragma unroll
  for (int s = 0; s <= H; ++s) {
    up[s] = 0.0f;
#pragma unroll
    for (int j = 0; j < 6; ++j) cur[s][j] = fr[s][j] = 0.0f;
  }
#pragma unroll
  for (int j = 0; j < M; ++j) {
    apx[j] = apym[j] = apyp[j] = apz[j] = itr[j] = pbr[j] = 0.0f;
  }
#pragma unroll
  for (int q = 0; q < PF; ++q) load_plane(z0 + q, pfd[q], pfpb[q], pfit[q]);
  float pbprev = 0.0f;

  for (int base = 0; base < nsteps; base += M) {
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int uz = z0 + base + j;   // plane taken at this step
      const int q = j % PF, par = j & 1;
      float fresh[6];
#pragma unroll
      for (int jj = 0; jj < 6; ++jj) fresh[jj] = pfd[q][jj];
      const float pbv = pfpb[q], itv = pfit[q];
      load_plane(uz + PF, pfd[q], pfpb[q], pfit[q]);
      apx[j] = kc.w1 * (lane_from_left(pbv) - pbv);
      apz[j] = kc.w1 * (pbprev - pbv);
      itr[j] = itv;
      pbr[j] = pbv;
      pbprev = pbv;
      // the y-moving populations of every level's plane and the new plane's
      // base, for the rows above and below (two copies by step parity: one
      // barrier per step)
#pragma unroll
      for (int s = 1; s <= H; ++s) {
        xup[par][s - 1][wv][lane] = cur[s][1];
        xdn[par][s - 1][wv][lane] = cur[s][3];
      }
      xpb[par][wv][lane] = pbv;
      __syncthreads();
      // w (P_b(y -+ 1) - P_b(y)) of the new plane (first used at the next
      // step); the outer rows of the column get 0, which reaches no kept node
      apym[j] = wv > 0 ? kc.w1 * (xpb[par][wv - 1][lane] - pbv) : 0.0f;
      apyp[j] = wv < kZW - 1 ? kc.w1 * (xpb[par][wv + 1][lane] - pbv) : 0.0f;
      // levels from H down to 1: level s reads fr[s] before level s - 1 replaces it
#pragma unroll
      for (int s = H; s >= 1; --s) {
        const int rs = (j - (2 * s - 1) + 2 * M) % M;   // slot of plane p = uz - (2s - 1)
        const int rs1 = (j - (2 * s - 2) + 2 * M) % M;  // slot of plane p + 1
        const int pz = uz - (2 * s - 1);
        float in[6];
#pragma unroll
        for (int jj = 0; jj < 6; ++jj) in[jj] = s == 1 ? fresh[jj] : fr[s][jj];
        const float nb1 = wv > 0 ? xup[par][s - 1][wv - 1][lane] : 0.0f;
        const float nb3 = wv < kZW - 1 ? xdn[par][s - 1][wv + 1][lane] : 0.0f;
        float e[6];
        e[0] = lane_from_left(cur[s][0]) + apx[rs];
        e[1] = nb1 + apym[rs];
        // w (P_b(x + 1) - P_b(x)) is minus the -x term of the lane to the
        // right (exactly), so the difference is formed there and moved
        e[2] = lane_from_right(cur[s][2] - apx[rs]);
        e[3] = nb3 + apyp[rs];
        e[4] = up[s] + apz[rs];
        // likewise w (P_b(z + 1) - P_b(z)) is minus the term of plane p + 1
        e[5] = in[5] - apz[rs1];
        if (xwalls) {
          const int wz = perz ? zwrap(pz) : z_clamp(pz, nz);
          if (wall_l) e[0] = z_wall_rule(kc, 0, 0, gy, wz, pbr[rs], cur[s][2]);
          if (wall_r) e[2] = z_wall_rule(kc, 1, nx - 1, gy, wz, pbr[rs], cur[s][0]);
        }
        if (wall_b || wall_t) {
          const int wz = perz ? zwrap(pz) : z_clamp(pz, nz);
          if (wall_b) e[1] = z_wall_rule(kc, 2, gx, 0, wz, pbr[rs], cur[s][3]);
          if (wall_t) e[3] = z_wall_rule(kc, 3, gx, ny - 1, wz, pbr[rs], cur[s][1]);
        }
        if (!perz && pz == 0) e[4] = z_wall_rule(kc, 4, gx, gy, 0, pbr[rs], cur[s][5]);
        if (!perz && pz == nz - 1) e[5] = z_wall_rule(kc, 5, gx, gy, nz - 1, pbr[rs], cur[s][4]);
        const float wdP = dsum<3>(e) * kc.w1_1mw0;
        const float it = itr[rs];
        const float keep = 1.0f - it, gain = wdP * it;
        float fp = 0.0f;
        if (HAS_FP) fp = wsrc * Fp[(perz ? z_wrap(pz, nz) : z_clamp(pz, nz)) * plane + gy * nx + gx];
        up[s] = cur[s][4];
        float o[6];
#pragma unroll
        for (int jj = 0; jj < 6; ++jj) {
          cur[s][jj] = in[jj];
          o[jj] = bgk_relax(e[jj], keep, gain);
          if (HAS_FP) o[jj] += fp;
        }
        if (s < H) {
#pragma unroll
          for (int jj = 0; jj < 6; ++jj) fr[s + 1][jj] = o[jj];
        } else if (keep_node && pz >= zs && pz < ze) {
          // plane uz - (2H - 1) after H sweeps
          const uint32_t c = (uint32_t)pz * (uint32_t)plane + (uint32_t)(uy * nx + ux);
#pragma unroll
          for (int jj = 0; jj < 6; ++jj) Storage<T>::store(z_at(fout.p[jj], c), 0, o[jj], kc.dev_scale);
        }
      }
    }
  }
}

}  // namespace

// Compute units of the current device (queried once per device).
int device_cus() {
  static std::atomic<int> cus[64];   // 0 = not queried yet (a repeated query writes the same value)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int n = cus[dev].load(std::memory_order_relaxed);
  if (!n) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cus[dev].store(n, std::memory_order_relaxed);
  }
  return n;
}

namespace {


// Columns of 64 - 2H x 16 - 2H output nodes; the number of z segments is the
// one that minimises rounds of resident workgroups x planes walked per
// workgroup (its segment plus the 3H - 1 planes of pipeline fill), over
// segments of at least 16 planes.
ZGeom zgeom(const KC &kc, int H) {
  ZGeom g;
  g.tiles_x = (kc.nx + kZBX - 2 * H - 1) / (kZBX - 2 * H);
  g.tiles_y = (kc.ny + kZW - 2 * H - 1) / (kZW - 2 * H);
  const long long cols = (long long)g.tiles_x * g.tiles_y;
  const int cus = device_cus();
  int most = (kc.nz + 15) / 16;
  if (most < 1) most = 1;
  long long best = -1;
  g.segs = 1;
  for (int segs = 1; segs <= most; ++segs) {
    const int seg = (kc.nz + segs - 1) / segs;
    const long long rounds = (cols * segs + cus - 1) / cus;
    const long long cost = rounds * (seg + 3 * H - 1);
    if (best < 0 || cost < best) {
      best = cost;
      g.segs = segs;
    }
  }
  g.seg = (kc.nz + g.segs - 1) / g.segs;
  g.segs = (kc.nz + g.seg - 1) / g.seg;
  return g;
}

template <typename T, int H>
void zstream_launch(const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, const float *itau, const float *Fp,
                    const Ctl *ctl, long long k, hipStream_t s) {
  const ZGeom g = zgeom(kc, H);
  const dim3 grid((unsigned)(g.tiles_x * g.tiles_y * g.segs)), block(kZBX * kZW);
  if (Fp)
    hipLaunchKernelGGL((f_zstream_kernel<T, true, H>), grid, block, 0, s, kc, fin, fout, Pb, itau, Fp, ctl, k, g);
  else
    hipLaunchKernelGGL((f_zstream_kernel<T, false, H>), grid, block, 0, s, kc, fin, fout, Pb, itau, Fp, ctl, k, g);
}

}  // namespace

// H = 3 only: at H = 5 the ten-plane rings and five levels do not fit the
// 128 registers a lane has with 16 wavefronts per workgroup.
int block_sweeps_supported_3d(int H) { return H == 3; }

hipError_t launch_f_block_3d(int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, const float *itau,
                             const float *Fp, const Ctl *ctl, long long k, int H, hipStream_t s) {
  if (!block_sweeps_supported_3d(H)) return hipErrorInvalidValue;
  switch (storage) {
    case LBTP_FP16_DEV: zstream_launch<_Float16, 3>(kc, fin, fout, Pb, itau, Fp, ctl, k, s); break;
    case LBTP_BF16_DEV: zstream_launch<bf16_t, 3>(kc, fin, fout, Pb, itau, Fp, ctl, k, s); break;
    default: zstream_launch<float, 3>(kc, fin, fout, Pb, itau, Fp, ctl, k, s); break;
  }
  return hipGetLastError();
}

}  // namespace lbtp
