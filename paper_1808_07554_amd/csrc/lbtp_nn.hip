// Warm-start network for the pressure iteration: a convolutional
// encoder-decoder mapping (lnK, S, wall proximity) on an H x W grid to a
// pressure estimate P = (1 - (x + 1/2)/W) + (scale / W) * net(.), where the
// wall proximity is exp(-d/16) with d the distance (in nodes) to the nearer
// Dirichlet wall; inputs and output are per node, so a network trained on one
// grid size applies to others.  P is used as the initial pressure of the
// lattice Boltzmann solve (the solve itself is unchanged and still runs to its
// tolerance).  Architecture: `levels` levels, base*2^l channels at level l,
// two 3x3 convolutions + ReLU per level on each side, 2x2 average pooling
// down, nearest 2x upsampling up, skip connections by channel concatenation
// [upsampled, skip], and a 3x3 head without activation.
//
// Tensors are [N][H][W][C] with C padded to a multiple of 16, activations in
// bf16, accumulation in float32.  The 3x3 convolution is an implicit GEMM on
// the bf16 matrix cores (16x16x32 MFMA): a workgroup stages a block of input
// pixels with its halo and the block's weights in LDS, and each wavefront
// computes several 16-pixel x 16-channel products per fragment it reads, with
// K running over the nine taps and the input channels.
// The backward-data pass is the same kernel with the weights rotated by 180
// degrees and input/output channels swapped; the weight gradient is a second
// MFMA GEMM with the pixels as K, split into chunks whose partial sums are
// added in a fixed order (deterministic).  Master weights, gradients and the
// Adam moments are float32.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/lbtp_nn.h"
#include "lbtp_internal.h"

namespace lbtp {
namespace {

typedef uint16_t bf16;
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ inline float bf2f(bf16 h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline bf16 f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (bf16)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ------------------------------------------------------------------ convolution
// out[n,y,x,co] = act(bias[co] + sum_{ky,kx,ci} w[co][ky][kx][ci] in[n, y+ky-1, x+kx-1, ci])
//
// Implicit GEMM on the 16x16x32 bf16 matrix cores, D[co][pixel] += W[co][k] X[k][pixel]
// with k = (tap, input channel).  A workgroup (4 waves) computes a TR x TC block
// of output pixels for TN output channels.  Input channels are
// taken CK at a time: the block's input pixels with a one-pixel halo,
// (TR+2) x (TC+2) x CK, and the TN x 9 x CK weights are staged in LDS with a
// pitch of CK + 8 bf16 per pixel / per weight row, which puts 16 consecutive
// pixels (or output channels) of one 16-byte column on 16 distinct groups of
// four banks.  Every wave then runs the nine taps out of LDS: wave v owns
// SPW = TR*TC/64 runs of 16 consecutive pixels of a row; per tap it reads
// TN/16 weight fragments and SPW input fragments and issues SPW * TN/16 MFMAs,
// so each fragment read from LDS feeds several products.  With CK = 16 (an
// input of 16 channels) one MFMA covers two taps: lanes 0-31 the even tap,
// lanes 32-63 the odd one; the tenth tap is zero.  The result of a lane is
// four consecutive output channels of one pixel, stored as one 8-byte (bf16)
// or 16-byte (float) write.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ inline f32x4_t mfma_16x16x32(const uint4 &a, const uint4 &b, const f32x4_t &c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                 0, 0, 0);
}

__device__ inline uint32_t pack_bf16x2(float lo, float hi) {
  return (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16);
}

// Tile of P = 256 pixels, TR x TC with TC = 2^tcs
// of 8, 16, 32 or 64 columns: the images of the batch are taken as one stack
// of N*H rows, so a tile may span images; a lane masks the rows above and
// below its output pixel where they belong to another image (the column halo
// is zero where it leaves the grid).
constexpr int conv_halo_max(int P) {
  int best = 0;
  for (int tc = 8; tc <= 64; tc *= 2) {
    const int h = (P / tc + 2) * (tc + 2);
    best = h > best ? h : best;
  }
  return best;
}

template <int TN, int CK>
__global__ __launch_bounds__(256, 2) void conv3x3_kernel(const bf16 *__restrict__ in, const bf16 *__restrict__ w,
                                                         const float *__restrict__ bias, void *__restrict__ out,
                                                         int NH, int H, int W, int Ci, int Co, int tcs, int relu,
                                                         int out_f32) {
  constexpr int P = 256;                   // pixels per tile
  constexpr int CKP = CK + 8;              // LDS pitch (bf16) of one pixel and of one weight row
  constexpr int SPW = P / 64;              // 16-pixel runs per wave
  constexpr int NB = TN / 16;              // 16-channel output blocks
  constexpr int Q = CK / 8;                // 16-byte pieces per pixel of a chunk
  constexpr int KSTEPS = CK == 32 ? 9 : 5;
  static_assert(CK == 16 || CK == 32, "chunk of 16 or 32 channels");
  __shared__ __align__(16) bf16 sx[conv_halo_max(P) * CKP];
  __shared__ __align__(16) bf16 sw[TN * 9 * CKP];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
  const int TC = 1 << tcs, TR = P >> tcs, HC = TC + 2, HR = TR + 2;
  const uint32_t hc_magic = 0xFFFFFFFFu / (uint32_t)HC + 1u;  // p / HC = umulhi(p, magic) for p < 2^16
  const int ntx = (W + TC - 1) >> tcs;
  const int tx0 = (int)(blockIdx.x % (unsigned)ntx) << tcs;
  const int ty0 = (int)(blockIdx.x / (unsigned)ntx) * TR;  // first stacked row
  const int co0 = blockIdx.y * TN;
  const uint4 z4 = {0u, 0u, 0u, 0u};
  // the wave's runs: LDS offset of the output pixel's halo origin, and whether
  // the rows above / below it belong to its image
  int base[SPW];
  bool up_ok[SPW], dn_ok[SPW];
#pragma unroll
  for (int i = 0; i < SPW; ++i) {
    const int pi = (wave * SPW + i) * 16 + m;
    const int r = pi >> tcs, c = pi & (TC - 1);
    const int y = (ty0 + r) % H;
    base[i] = r * HC + c;
    up_ok[i] = y > 0;
    dn_ok[i] = y < H - 1;
  }
  f32x4_t acc[SPW][NB];
#pragma unroll
  for (int i = 0; i < SPW; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  // The next chunk's input (and, below 64 output channels, its weights) is
  // loaded into registers while the current one is swept, and written to LDS
  // between two barriers; at 64 channels the weights, which every workgroup
  // reads and so come from L2, are loaded there (registers for both would
  // spill).
  constexpr bool PREW = TN < 64;
  constexpr int NXI = (conv_halo_max(P) * Q + 255) / 256, NWI = (TN * 9 * Q + 255) / 256;
  uint4 px[NXI], pw[PREW ? NWI : 1];
  const int nhalo = HR * HC * Q;
  // staging piece idx -> (row, piece), rows being pixels or weight rows:
  // with 4 pieces per row the 16 lanes of a group take rows a, a+4, a+8,
  // a+12 of a run of 16, which (80 bytes apart) start 16 banks apart, so the
  // group's writes fill the 64 banks once (weight rows come in multiples of
  // 16); with 2 pieces per row the plain order does
  auto stage_pixel = [&](int idx) {
    if constexpr (Q == 4) {
      const int u = (idx >> 2) & 15;
      return (idx >> 6) * 16 + ((u & 3) << 2) + (u >> 2);
    } else {
      return idx / Q;
    }
  };
  auto fetch = [&](int c0) {
#pragma unroll
    for (int k = 0; k < NXI; ++k) {
      const int idx = tid + 256 * k;
      const int q = idx % Q, p = stage_pixel(idx);
      const int r = (int)__umulhi((uint32_t)p, hc_magic);
      const int ys = ty0 + r - 1, gx = tx0 + (p - r * HC) - 1;
      px[k] = make_uint4(0u, 0u, 0u, 0u);
      if (p < nhalo / Q && ys >= 0 && ys < NH && gx >= 0 && gx < W)
        px[k] = *(const uint4 *)(in + ((size_t)ys * W + gx) * Ci + c0 + 8 * q);
    }
    if constexpr (PREW) {
#pragma unroll
      for (int k = 0; k < NWI; ++k) {
        const int idx = tid + 256 * k;
        const int q = idx % Q, row = stage_pixel(idx);  // row = local output channel * 9 + tap
        pw[k] = make_uint4(0u, 0u, 0u, 0u);
        if (idx < TN * 9 * Q) pw[k] = *(const uint4 *)(w + ((size_t)co0 * 9 + row) * Ci + c0 + 8 * q);
      }
    }
  };
  fetch(0);
  for (int c0 = 0; c0 < Ci; c0 += CK) {
    __syncthreads();  // the previous chunk's fragments have been read
#pragma unroll
    for (int k = 0; k < NXI; ++k) {
      const int idx = tid + 256 * k;
      const int p = stage_pixel(idx);
      if (p < nhalo / Q) *(uint4 *)(sx + p * CKP + 8 * (idx % Q)) = px[k];
    }
    if constexpr (PREW) {
#pragma unroll
      for (int k = 0; k < NWI; ++k) {
        const int idx = tid + 256 * k;
        if (idx < TN * 9 * Q) *(uint4 *)(sw + stage_pixel(idx) * CKP + 8 * (idx % Q)) = pw[k];
      }
    } else {
      for (int idx = tid; idx < TN * 9 * Q; idx += 256) {
        const int q = idx % Q, row = stage_pixel(idx);
        *(uint4 *)(sw + row * CKP + 8 * q) = *(const uint4 *)(w + ((size_t)co0 * 9 + row) * Ci + c0 + 8 * q);
      }
    }
    __syncthreads();
    if (c0 + CK < Ci) fetch(c0 + CK);
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) {
      const int tap = CK == 32 ? s : 2 * s + (g >> 1);
      const int ch = CK == 32 ? 8 * g : 8 * (g & 1);
      const bool live = tap < 9;
      const int ky = live ? tap / 3 : 0, kx = live ? tap % 3 : 0;
      uint4 a[NB], x[SPW];
#pragma unroll
      for (int j = 0; j < NB; ++j) a[j] = live ? *(const uint4 *)(sw + ((16 * j + m) * 9 + tap) * CKP + ch) : z4;
#pragma unroll
      for (int i = 0; i < SPW; ++i) {
        const bool ok = live && (ky != 0 || up_ok[i]) && (ky != 2 || dn_ok[i]);
        x[i] = ok ? *(const uint4 *)(sx + (base[i] + ky * HC + kx) * CKP + ch) : z4;
      }
#pragma unroll
      for (int i = 0; i < SPW; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = mfma_16x16x32(a[j], x[i], acc[i][j]);
    }
  }
  // lane holds D[4 g + r][m]: output channel co0 + 16 j + 4 g + r of pixel m of each run
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int co = co0 + 16 * j + 4 * g;
    float bv[4] = {0.f, 0.f, 0.f, 0.f};
    if (bias) {
#pragma unroll
      for (int r = 0; r < 4; ++r) bv[r] = bias[co + r];
    }
#pragma unroll
    for (int i = 0; i < SPW; ++i) {
      const int pi = (wave * SPW + i) * 16 + m;
      const int ys = ty0 + (pi >> tcs), x = tx0 + (pi & (TC - 1));
      if (ys < NH && x < W) {
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          v[r] = acc[i][j][r] + bv[r];
          if (relu) v[r] = fmaxf(v[r], 0.0f);
        }
        const size_t o = ((size_t)ys * W + x) * Co + co;
        if (out_f32) *(float4 *)((float *)out + o) = make_float4(v[0], v[1], v[2], v[3]);
        else *(uint2 *)((bf16 *)out + o) = make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
      }
    }
  }
}

// Transpose of an 8 x 8 block of bf16: v[p] holds channels 0..7 of pixel p,
// o[c] receives pixels 0..7 of channel c.
__device__ inline uint32_t dword_of(const uint4 &v, int d) { return d == 0 ? v.x : d == 1 ? v.y : d == 2 ? v.z : v.w; }

__device__ inline void transpose8x8(const uint4 (&v)[8], uint4 (&o)[8]) {
#pragma unroll
  for (int d = 0; d < 4; ++d) {  // channels 2d, 2d+1 sit in dword d of every pixel
    uint32_t lo[4], hi[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t a = dword_of(v[2 * e], d), b = dword_of(v[2 * e + 1], d);
      lo[e] = (a & 0xFFFFu) | (b << 16);
      hi[e] = (a >> 16) | (b & 0xFFFF0000u);
    }
    o[2 * d] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
    o[2 * d + 1] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
  }
}

// Weight gradient, an implicit GEMM with the pixels as K:
// part[slice][co][tap][ci] = sum over the slice's pixels p of dy[p][co] x[p shifted by tap][ci].
// A workgroup owns COT output x CIT input channels and a run of TR x TC pixel
// tiles.  Per tile it stages dy (COT channels x TR*TC pixels) and the input
// with one halo row above and below and eight columns either side
// (CIT x (TR+2) x (TC+16)) in LDS, channel-major: the pixel-major tensors are
// transposed 8 x 8 in registers on the way, so the eight K values of a lane
// (eight consecutive pixels of a row) are one aligned 16-byte read.  The three
// horizontal taps come out of the same three aligned reads per input row,
// shifted by one bf16 with v_alignbyte.  Wave v takes input-channel block
// v % (CIT/16) and every KS-th K step (KS = 64/CIT); its 16x16 products for
// all COT/16 output blocks and the nine taps stay in registers over the whole
// tile run, and it writes them as its own slice (chunk * KS + v / (CIT/16)),
// so the fixed-order sum over the slices is deterministic.  The waves of input
// block 0 also form the bias gradient, sum_p dy[p][co], as a product of the
// same dy fragments with a matrix of ones, into bpart[slice][co].
template <int TR, int TC, int COT, int CIT>
__global__ __launch_bounds__(256, 2) void conv3x3_wgrad_kernel(const bf16 *__restrict__ dy,
                                                               const bf16 *__restrict__ x, float *__restrict__ part,
                                                               float *__restrict__ bpart, int N, int H, int W, int Ci,
                                                               int Co, int tiles_per_chunk) {
  constexpr int NA = COT / 16, NCB = CIT / 16, KS = 4 / NCB;
  constexpr int TP = TR * TC, DYP = TP + 8;                    // pixels per tile; LDS pitch of a dy channel
  constexpr int HR = TR + 2, HCW = TC + 16, HB = HCW / 8;      // halo rows, columns, 8-column blocks
  constexpr int XP = HR * HCW + 8;                             // LDS pitch of an input channel
  constexpr int RUNS = TP / 8, RPR = TC / 8, KSTEPS = RUNS / 4;
  static_assert(TC % 8 == 0 && RUNS % 4 == 0, "whole K steps per tile");
  static_assert((DYP / 8) % 2 == 1 && (XP / 8) % 2 == 1, "odd multiples of 16 bytes spread the 16 rows over the banks");
  __shared__ __align__(16) bf16 sdy[COT * DYP];
  __shared__ __align__(16) bf16 sx[CIT * XP];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
  const int cb = wave % NCB, ks = wave / NCB;
  const int ncit = Ci / CIT;
  const int co0 = (blockIdx.x / ncit) * COT, ci0 = (blockIdx.x % ncit) * CIT;
  const int ntx = (W + TC - 1) / TC, nty = (H + TR - 1) / TR;
  const int ntiles = N * ntx * nty;
  const int t0 = blockIdx.y * tiles_per_chunk;
  const int t1 = t0 + tiles_per_chunk < ntiles ? t0 + tiles_per_chunk : ntiles;
  const bool do_bias = (blockIdx.x % ncit) == 0 && cb == 0;
  const uint4 ones = make_uint4(0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u);  // bf16 1.0
  f32x4_t acc[NA][9], bacc[NA];
#pragma unroll
  for (int ia = 0; ia < NA; ++ia) {
    bacc[ia] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[ia][t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  }
  for (int t = t0; t < t1; ++t) {
    const int tx0 = (t % ntx) * TC, ty0 = ((t / ntx) % nty) * TR, n = t / (ntx * nty);
    __syncthreads();  // the previous tile's fragments have been read
    for (int it = tid; it < RUNS * (COT / 8); it += 256) {
      const int cg = it % (COT / 8), run = it / (COT / 8);
      const int y = ty0 + run / RPR, xb = tx0 + (run % RPR) * 8;
      uint4 v[8], o[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        v[j] = make_uint4(0u, 0u, 0u, 0u);
        if (y < H && xb + j < W) v[j] = *(const uint4 *)(dy + (((size_t)n * H + y) * W + xb + j) * Co + co0 + 8 * cg);
      }
      transpose8x8(v, o);
#pragma unroll
      for (int c = 0; c < 8; ++c) *(uint4 *)(sdy + (8 * cg + c) * DYP + run * 8) = o[c];
    }
    for (int it = tid; it < HR * HB * (CIT / 8); it += 256) {
      const int cg = it % (CIT / 8), rb = it / (CIT / 8);
      const int hr = rb / HB, hb = rb % HB;
      const int y = ty0 + hr - 1, xb = tx0 - 8 + hb * 8;
      uint4 v[8], o[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        v[j] = make_uint4(0u, 0u, 0u, 0u);
        if (y >= 0 && y < H && xb + j >= 0 && xb + j < W)
          v[j] = *(const uint4 *)(x + (((size_t)n * H + y) * W + xb + j) * Ci + ci0 + 8 * cg);
      }
      transpose8x8(v, o);
#pragma unroll
      for (int c = 0; c < 8; ++c) *(uint4 *)(sx + (8 * cg + c) * XP + hr * HCW + hb * 8) = o[c];
    }
    __syncthreads();
    for (int k = ks; k < KSTEPS; k += KS) {
      const int run = 4 * k + g;
      const int r = run / RPR, c8 = run % RPR;
      uint4 a[NA];
#pragma unroll
      for (int ia = 0; ia < NA; ++ia) a[ia] = *(const uint4 *)(sdy + (16 * ia + m) * DYP + run * 8);
      if (do_bias) {
#pragma unroll
        for (int ia = 0; ia < NA; ++ia) bacc[ia] = mfma_16x16x32(a[ia], ones, bacc[ia]);
      }
      // halo column 8 (c8 + 1) + j holds the input under tile column 8 c8 + j
      const bf16 *xr = sx + (16 * cb + m) * XP + r * HCW + c8 * 8;
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        const uint4 b0 = *(const uint4 *)(xr + ky * HCW);
        const uint4 b1 = *(const uint4 *)(xr + ky * HCW + 8);
        const uint4 b2 = *(const uint4 *)(xr + ky * HCW + 16);
        const uint32_t s1 = __builtin_amdgcn_alignbyte(b1.y, b1.x, 2), s2 = __builtin_amdgcn_alignbyte(b1.z, b1.y, 2),
                       s3 = __builtin_amdgcn_alignbyte(b1.w, b1.z, 2);
        const uint4 left = make_uint4(__builtin_amdgcn_alignbyte(b1.x, b0.w, 2), s1, s2, s3);   // columns - 1
        const uint4 right = make_uint4(s1, s2, s3, __builtin_amdgcn_alignbyte(b2.x, b1.w, 2));  // columns + 1
#pragma unroll
        for (int ia = 0; ia < NA; ++ia) {
          acc[ia][3 * ky] = mfma_16x16x32(a[ia], left, acc[ia][3 * ky]);
          acc[ia][3 * ky + 1] = mfma_16x16x32(a[ia], b1, acc[ia][3 * ky + 1]);
          acc[ia][3 * ky + 2] = mfma_16x16x32(a[ia], right, acc[ia][3 * ky + 2]);
        }
      }
    }
  }
  // lane holds D[4 g + r][m]: output channel co0 + 16 ia + 4 g + r, input channel ci0 + 16 cb + m
  const size_t slice = (size_t)blockIdx.y * KS + ks;
  const int ci = ci0 + 16 * cb + m;
#pragma unroll
  for (int ia = 0; ia < NA; ++ia)
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        part[((slice * Co + co0 + 16 * ia + 4 * g + r) * 9 + tap) * Ci + ci] = acc[ia][tap][r];
  if (do_bias && m == 0) {
#pragma unroll
    for (int ia = 0; ia < NA; ++ia)
#pragma unroll
      for (int r = 0; r < 4; ++r) bpart[slice * Co + co0 + 16 * ia + 4 * g + r] = bacc[ia][r];
  }
}

// dw[i] = sum over chunks of part[chunk][i] in a fixed order: lane l (of four
// per column) adds chunks l, l + 4, l + 8, ... in turn, eight loads in flight,
// and the four lane sums are added in lane order.  Block 256 = 64 columns x 4.
__global__ __launch_bounds__(256) void sum_chunks_kernel(const float *__restrict__ part, float *__restrict__ dw,
                                                         long long n, int nchunk) {
  __shared__ float sh[4][64];
  const int tx = threadIdx.x & 63, l = threadIdx.x >> 6;
  const long long i = (long long)blockIdx.x * 64 + tx;
  float s = 0.0f;
  if (i < n) {
    int c = l;
    for (; c + 28 < nchunk; c += 32) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(c + 4 * u) * n + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < nchunk; c += 4) s += part[(size_t)c * n + i];
  }
  sh[l][tx] = s;
  __syncthreads();
  if (l == 0 && i < n) dw[i] = ((sh[0][tx] + sh[1][tx]) + sh[2][tx]) + sh[3][tx];
}

// ------------------------------------------------------------ element-wise
#define GRID1(n) dim3((unsigned)(((n) + 255) / 256)), dim3(256)

__global__ void relu_mask_kernel(bf16 *__restrict__ dy, const bf16 *__restrict__ y, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n && !(bf2f(y[i]) > 0.0f)) dy[i] = 0;
}

// [N,H,W,C] -> [N,H/2,W/2,C], mean of 2x2
__global__ void pool_kernel(const bf16 *__restrict__ in, bf16 *__restrict__ out, int N, int H, int W, int C) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const int Ho = H / 2, Wo = W / 2;
  if (i >= (long long)N * Ho * Wo * C) return;
  const int c = (int)(i % C);
  long long r = i / C;
  const int xo = (int)(r % Wo);
  r /= Wo;
  const int yo = (int)(r % Ho);
  const long long n = r / Ho;
  const size_t b = (((size_t)n * H + 2 * yo) * W + 2 * xo) * C + c;
  const float s = bf2f(in[b]) + bf2f(in[b + C]) + bf2f(in[b + (size_t)W * C]) + bf2f(in[b + (size_t)W * C + C]);
  out[i] = f2bf(0.25f * s);
}

// adjoint of pool: [N,H/2,W/2,C] -> [N,H,W,C]
__global__ void pool_bwd_kernel(const bf16 *__restrict__ dout, bf16 *__restrict__ din, int N, int H, int W, int C) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long long)N * H * W * C) return;
  const int c = (int)(i % C);
  long long r = i / C;
  const int x = (int)(r % W);
  r /= W;
  const int y = (int)(r % H);
  const long long n = r / H;
  din[i] = f2bf(0.25f * bf2f(dout[(((size_t)n * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c]));
}

// nearest 2x: [N,H,W,C] -> [N,2H,2W,C]
__global__ void up_kernel(const bf16 *__restrict__ in, bf16 *__restrict__ out, int N, int H, int W, int C) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const int Ho = 2 * H, Wo = 2 * W;
  if (i >= (long long)N * Ho * Wo * C) return;
  const int c = (int)(i % C);
  long long r = i / C;
  const int x = (int)(r % Wo);
  r /= Wo;
  const int y = (int)(r % Ho);
  const long long n = r / Ho;
  out[i] = in[(((size_t)n * H + y / 2) * W + x / 2) * C + c];
}

// adjoint of up: [N,2H,2W,C] -> [N,H,W,C], sum of 2x2
__global__ void up_bwd_kernel(const bf16 *__restrict__ dout, bf16 *__restrict__ din, int N, int H, int W, int C) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long long)N * H * W * C) return;
  const int c = (int)(i % C);
  long long r = i / C;
  const int x = (int)(r % W);
  r /= W;
  const int y = (int)(r % H);
  const long long n = r / H;
  const int W2 = 2 * W;
  const size_t b = (((size_t)n * 2 * H + 2 * y) * W2 + 2 * x) * C + c;
  const float s = bf2f(dout[b]) + bf2f(dout[b + C]) + bf2f(dout[b + (size_t)W2 * C]) +
                  bf2f(dout[b + (size_t)W2 * C + C]);
  din[i] = f2bf(s);
}

// out[p, 0:Ca] = a[p], out[p, Ca:Ca+Cb] = b[p]
__global__ void concat_kernel(const bf16 *__restrict__ a, const bf16 *__restrict__ b, bf16 *__restrict__ out,
                              long long npix, int Ca, int Cb) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const int C = Ca + Cb;
  if (i >= npix * C) return;
  const int c = (int)(i % C);
  const long long p = i / C;
  out[i] = c < Ca ? a[p * Ca + c] : b[p * Cb + (c - Ca)];
}

__global__ void split_kernel(const bf16 *__restrict__ in, bf16 *__restrict__ a, bf16 *__restrict__ b, long long npix,
                             int Ca, int Cb) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const int C = Ca + Cb;
  if (i >= npix * C) return;
  const int c = (int)(i % C);
  const long long p = i / C;
  if (c < Ca) a[p * Ca + c] = in[i];
  else b[p * Cb + (c - Ca)] = in[i];
}

__global__ void add_kernel(bf16 *__restrict__ a, const bf16 *__restrict__ b, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) a[i] = f2bf(bf2f(a[i]) + bf2f(b[i]));
}

// network input [N,H,W,16]: lnK, S, wall proximity exp(-d/16), zeros
__global__ void pack_input_kernel(const float *__restrict__ lnK, const float *__restrict__ S, bf16 *__restrict__ x,
                                  long long npix, int W) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  const float xc = (float)(p % W) + 0.5f;
  const float d = fminf(xc, (float)W - xc);
  bf16 *o = x + p * 16;
  o[0] = f2bf(lnK[p]);
  o[1] = f2bf(S[p]);
  o[2] = f2bf(expf(-d / 16.0f));
  for (int c = 3; c < 16; ++c) o[c] = 0;
}

// P = (1 - (x + 1/2)/W) + (scale / W) * head[..., 0]
__global__ void head_out_kernel(const float *__restrict__ head, float *__restrict__ P, long long npix, int W,
                                float scale) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  const int xq = (int)(p % W);
  P[p] = (1.0f - ((float)xq + 0.5f) / (float)W) + (scale / (float)W) * head[p * 16];
}

// Block mean over f x f nodes: out[n][Y][X] = f^-2 sum in[n][fY + j][fX + i]
// (sum in row-major order of (j, i)), for lnK and S together.
__global__ void coarsen_kernel(const float *__restrict__ a, const float *__restrict__ b, float *__restrict__ ac,
                               float *__restrict__ bc, long long ncoarse, int Hc, int Wc, int f) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= ncoarse) return;
  const int X = (int)(q % Wc);
  const long long r = q / Wc;
  const int Y = (int)(r % Hc);
  const long long n = r / Hc;
  const long long W = (long long)Wc * f;
  const long long base = (n * Hc * f + (long long)Y * f) * W + (long long)X * f;
  float sa = 0.f, sb = 0.f;
  for (int j = 0; j < f; ++j)
    for (int i = 0; i < f; ++i) {
      sa += a[base + j * W + i];
      sb += b[base + j * W + i];
    }
  const float inv = 1.0f / (float)(f * f);
  ac[q] = sa * inv;
  bc[q] = sb * inv;
}

// Fine pressure from the coarse network output: the coarse deviation
// D = (scale / Wc) * head is interpolated bilinearly to the fine node centres
// (coarse coordinate u = (x + 1/2)/f - 1/2, indices clamped to the grid) and
// added to the fine linear profile 1 - (x + 1/2)/W.
__global__ void upsample_kernel(const float *__restrict__ head, float *__restrict__ P, long long npix, int H, int W,
                                int f, float dscale) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  const int x = (int)(p % W);
  const long long r = p / W;
  const int y = (int)(r % H);
  const long long n = r / H;
  const int Hc = H / f, Wc = W / f;
  const float inv_f = 1.0f / (float)f;
  const float u = ((float)x + 0.5f) * inv_f - 0.5f, v = ((float)y + 0.5f) * inv_f - 0.5f;
  const float fu = floorf(u), fv = floorf(v);
  const float tu = u - fu, tv = v - fv;
  const int x0 = min(max((int)fu, 0), Wc - 1), x1 = min(max((int)fu + 1, 0), Wc - 1);
  const int y0 = min(max((int)fv, 0), Hc - 1), y1 = min(max((int)fv + 1, 0), Hc - 1);
  const float *h = head + n * Hc * Wc * 16;
  const float d00 = h[((long long)y0 * Wc + x0) * 16], d01 = h[((long long)y0 * Wc + x1) * 16];
  const float d10 = h[((long long)y1 * Wc + x0) * 16], d11 = h[((long long)y1 * Wc + x1) * 16];
  const float d0 = d00 + tu * (d01 - d00), d1 = d10 + tu * (d11 - d10);
  P[p] = (1.0f - ((float)x + 0.5f) / (float)W) + dscale * (d0 + tv * (d1 - d0));
}

// loss partial sums and d(loss)/d(head) for L = mean w_n (P - T)^2, with a
// weight per sample (wts NULL: all 1) and hw nodes per sample
__global__ __launch_bounds__(256) void mse_kernel(const float *__restrict__ P, const float *__restrict__ T,
                                                  const float *__restrict__ wts, bf16 *__restrict__ dhead,
                                                  double *__restrict__ partial, long long npix, long long hw,
                                                  float scale) {
  __shared__ double sh[256];
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (p < npix) {
    const float r = P[p] - T[p];
    const float wn = wts ? wts[p / hw] : 1.0f;
    l = (double)wn * (double)r * (double)r;
    bf16 *o = dhead + p * 16;
    o[0] = f2bf(scale * 2.0f * wn * r / (float)npix);
    for (int c = 1; c < 16; ++c) o[c] = 0;
  }
  sh[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void sum_double_kernel(const double *__restrict__ part, int n, double *out, double scale) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0] * scale;
}

// flat float weights [co][3][3][ci] + bias -> padded bf16 w [cop][9][cip], float bias [cop],
// and the rotated copy wt [cip][9][cop] (wt[ci][8 - tap][co] = w[co][tap][ci]) for backward-data
__global__ void pack_layer_kernel(const float *__restrict__ flat, int ci, int co, int cip, int cop,
                                  bf16 *__restrict__ w, bf16 *__restrict__ wt, float *__restrict__ b) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long n = (long long)cop * 9 * cip;
  if (i < cop) b[i] = i < co ? flat[(size_t)co * 9 * ci + i] : 0.0f;
  if (i >= n) return;
  const int c = (int)(i % cip);
  const long long r = i / cip;
  const int tap = (int)(r % 9);
  const int o = (int)(r / 9);
  const float v = (c < ci && o < co) ? flat[((size_t)o * 9 + tap) * ci + c] : 0.0f;
  const bf16 h = f2bf(v);
  w[i] = h;
  wt[((size_t)c * 9 + (8 - tap)) * cop + o] = h;
}

// padded dw [cop][9][cip] and db [cop] -> flat gradient of one layer
__global__ void unpack_grad_kernel(const float *__restrict__ dw, const float *__restrict__ db, int ci, int co,
                                   int cip, float *__restrict__ flat) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long nw = (long long)co * 9 * ci;
  if (i < nw) {
    const int c = (int)(i % ci);
    const long long r = i / ci;
    const int tap = (int)(r % 9);
    const int o = (int)(r / 9);
    flat[i] = dw[((size_t)o * 9 + tap) * cip + c];
  } else if (i < nw + co) {
    flat[i] = db[i - nw];
  }
}

__global__ void adam_kernel(float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace
}  // namespace lbtp

// =========================================================== host driver
using namespace lbtp;

namespace {

struct NNLayer {
  int ci, co, cip, cop;
  bool relu;
  size_t off;          // offset of the layer's weights in the flat parameter vector
  bf16 *w, *wt;        // padded [cop][9][cip] and rotated [cip][9][cop]
  float *b;            // [cop]
  float *dw, *db;      // padded gradients
};

struct Tensor {
  bf16 *p = nullptr;
  size_t cap = 0;
};

int pad16(int c) { return (c + 15) / 16 * 16; }

}  // namespace

namespace {
// Bump allocation from a caller-independent device buffer (the no-allocation
// predict): offsets aligned to 256 bytes, never beyond cap.
struct Arena {
  char *base = nullptr;
  size_t cap = 0, used = 0;
};

void *arena_take(Arena *a, size_t bytes, int *rc) {
  const size_t off = (a->used + 255) & ~(size_t)255;
  if (off > a->cap || bytes > a->cap - off) {
    *rc = LBTP_ENOMEM;
    return nullptr;
  }
  a->used = off + bytes;
  return a->base + off;
}
}  // namespace

struct lbtp_nn {
  int base = 32, levels = 4;
  float scale = 1.0f;
  hipStream_t stream = nullptr;
  std::vector<NNLayer> L;
  size_t np = 0;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  long long adam_t = 0;
  // activations of the last forward pass (training keeps them for backward)
  std::vector<Tensor> act;     // pool of tensors, reused across calls
  float *part = nullptr;       // weight-gradient chunk partials
  size_t part_cap = 0;
  float *head = nullptr;
  size_t head_cap = 0;
  float *head_cur = nullptr;   // head output of the last forward pass
  Arena *arena = nullptr;      // set: forward takes its buffers from here
  int device = -1;             // HIP device current at creation
  double *lpart = nullptr, *dloss = nullptr;
  size_t lpart_cap = 0;
};

namespace {

#define NN_TRY(x)                          \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) return LBTP_EHIP; \
  } while (0)

int ensure(void **p, size_t *cap, size_t bytes) {
  if (*cap >= bytes) return LBTP_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  if (hipMalloc(p, bytes) != hipSuccess) return LBTP_ENOMEM;
  *cap = bytes;
  return LBTP_OK;
}

bf16 *tensor(lbtp_nn *nn, int slot, size_t elems, int *rc) {
  if (nn->arena) return (bf16 *)arena_take(nn->arena, elems * sizeof(bf16), rc);
  if ((int)nn->act.size() <= slot) nn->act.resize(slot + 1);
  Tensor &t = nn->act[slot];
  if (ensure((void **)&t.p, &t.cap, elems * sizeof(bf16))) *rc = LBTP_ENOMEM;
  return t.p;
}

template <int TN, int CK>
void conv_launch(hipStream_t st, const bf16 *in, const bf16 *w, const float *b, void *out, int N, int H, int W,
                 int Ci, int Co, bool relu, bool f32) {
  // tile width: of 8, 16, 32 and 64 columns the one that wastes the fewest, the wider on a tie
  int tcs = 6, waste = (W + 63) / 64 * 64 - W;
  for (int t = 5; t >= 3; --t) {
    const int wt = ((W + (1 << t) - 1) >> t << t) - W;
    if (wt < waste) {
      waste = wt;
      tcs = t;
    }
  }
  const int P = 256;
  const int ntx = (W + (1 << tcs) - 1) >> tcs, nty = (N * H + (P >> tcs) - 1) / (P >> tcs);
  const dim3 g((unsigned)(ntx * nty), (unsigned)(Co / TN));
  hipLaunchKernelGGL((conv3x3_kernel<TN, CK>), g, dim3(256), 0, st, in, w, b, out, N * H, H, W, Ci, Co, tcs,
                     (int)relu, (int)f32);
}

// 64 output channels per workgroup where they divide Co, else 32, else 16;
// input channels in chunks of 32, or of 16 when Ci is an odd multiple of 16.
template <int CK>
void conv_dispatch(hipStream_t st, const bf16 *in, const bf16 *w, const float *b, void *out, int N, int H, int W,
                   int Ci, int Co, bool relu, bool f32) {
  if (Co % 64 == 0) conv_launch<64, CK>(st, in, w, b, out, N, H, W, Ci, Co, relu, f32);
  else if (Co % 32 == 0) conv_launch<32, CK>(st, in, w, b, out, N, H, W, Ci, Co, relu, f32);
  else conv_launch<16, CK>(st, in, w, b, out, N, H, W, Ci, Co, relu, f32);
}

int conv_fwd(lbtp_nn *nn, const bf16 *in, const bf16 *w, const float *b, void *out, int N, int H, int W, int Ci,
             int Co, bool relu, bool f32) {
  if (Ci <= 0 || Ci % 16 || Co <= 0 || Co % 16) return LBTP_EINVAL;
  if (Ci % 32 == 0) conv_dispatch<32>(nn->stream, in, w, b, out, N, H, W, Ci, Co, relu, f32);
  else conv_dispatch<16>(nn->stream, in, w, b, out, N, H, W, Ci, Co, relu, f32);
  NN_TRY(hipGetLastError());
  return LBTP_OK;
}

int pack_params(lbtp_nn *nn) {
  for (NNLayer &l : nn->L) {
    const long long n = (long long)l.cop * 9 * l.cip;
    hipLaunchKernelGGL(pack_layer_kernel, GRID1(n > l.cop ? n : l.cop), 0, nn->stream, nn->theta + l.off, l.ci, l.co,
                       l.cip, l.cop, l.w, l.wt, l.b);
    NN_TRY(hipGetLastError());
  }
  return LBTP_OK;
}

// Tape of one forward pass: per conv the input and output tensors.
struct Tape {
  std::vector<const bf16 *> x, y;
  std::vector<int> H, W;
};

// Slots in nn->act: 0 input; per conv i: output slot 1 + i; pooled inputs,
// upsampled and concatenated tensors after that.
int forward(lbtp_nn *nn, const float *lnK, const float *S, int N, int H, int W, Tape *tape) {
  int rc = LBTP_OK;
  const long long npix = (long long)N * H * W;
  const int nconv = (int)nn->L.size();
  int slot = 0;
  bf16 *x = tensor(nn, slot++, (size_t)npix * 16, &rc);
  if (rc) return rc;
  hipLaunchKernelGGL(pack_input_kernel, GRID1(npix), 0, nn->stream, lnK, S, x, npix, W);
  NN_TRY(hipGetLastError());
  int li = 0, h = H, wd = W;
  const bf16 *cur = x;
  std::vector<const bf16 *> skips(nn->levels);
  auto conv = [&](const bf16 *in) -> const bf16 * {
    const NNLayer &l = nn->L[li];
    bf16 *o = tensor(nn, slot++, (size_t)N * h * wd * l.cop, &rc);
    if (rc) return nullptr;
    if ((rc = conv_fwd(nn, in, l.w, l.b, o, N, h, wd, l.cip, l.cop, l.relu, false))) return nullptr;
    if (tape) {
      tape->x.push_back(in);
      tape->y.push_back(o);
      tape->H.push_back(h);
      tape->W.push_back(wd);
    }
    ++li;
    return o;
  };
  for (int lv = 0; lv < nn->levels; ++lv) {
    if (lv > 0) {
      const int C = nn->L[li - 1].cop;
      bf16 *p = tensor(nn, slot++, (size_t)N * (h / 2) * (wd / 2) * C, &rc);
      if (rc) return rc;
      hipLaunchKernelGGL(pool_kernel, GRID1((long long)N * (h / 2) * (wd / 2) * C), 0, nn->stream, cur, p, N, h, wd, C);
      NN_TRY(hipGetLastError());
      h /= 2;
      wd /= 2;
      cur = p;
    }
    cur = conv(cur);
    if (!cur) return rc;
    cur = conv(cur);
    if (!cur) return rc;
    skips[lv] = cur;
  }
  for (int lv = nn->levels - 2; lv >= 0; --lv) {
    const int Cu = nn->L[li - 1].cop, Cs = nn->L[2 * lv + 1].cop;
    bf16 *u = tensor(nn, slot++, (size_t)N * (2 * h) * (2 * wd) * Cu, &rc);
    if (rc) return rc;
    hipLaunchKernelGGL(up_kernel, GRID1((long long)N * 4 * h * wd * Cu), 0, nn->stream, cur, u, N, h, wd, Cu);
    NN_TRY(hipGetLastError());
    h *= 2;
    wd *= 2;
    bf16 *k = tensor(nn, slot++, (size_t)N * h * wd * (Cu + Cs), &rc);
    if (rc) return rc;
    hipLaunchKernelGGL(concat_kernel, GRID1((long long)N * h * wd * (Cu + Cs)), 0, nn->stream, u, skips[lv], k,
                       (long long)N * h * wd, Cu, Cs);
    NN_TRY(hipGetLastError());
    cur = conv(k);
    if (!cur) return rc;
    cur = conv(cur);
    if (!cur) return rc;
  }
  // head (float output)
  const NNLayer &hl = nn->L[nconv - 1];
  if (nn->arena) {
    nn->head_cur = (float *)arena_take(nn->arena, (size_t)npix * 16 * sizeof(float), &rc);
    if (rc) return rc;
  } else {
    if ((rc = ensure((void **)&nn->head, &nn->head_cap, (size_t)npix * 16 * sizeof(float)))) return rc;
    nn->head_cur = nn->head;
  }
  if (tape) {
    tape->x.push_back(cur);
    tape->y.push_back(nullptr);
    tape->H.push_back(h);
    tape->W.push_back(wd);
  }
  if ((rc = conv_fwd(nn, cur, hl.w, hl.b, nn->head_cur, N, h, wd, hl.cip, hl.cop, false, true))) return rc;
  return LBTP_OK;
}

template <int TR, int TC, int COT, int CIT>
int wgrad_launch(lbtp_nn *nn, const bf16 *dy, const bf16 *x, int N, int H, int W, int Ci, int Co, int *slices) {
  const int ntiles = N * ((H + TR - 1) / TR) * ((W + TC - 1) / TC);
  const int pairs = (Co / COT) * (Ci / CIT);
  // about 512 workgroups, each over at least 4 tiles
  int nchunk = 512 / pairs;
  if (nchunk > ntiles / 4) nchunk = ntiles / 4;
  if (nchunk < 1) nchunk = 1;
  const int tpc = (ntiles + nchunk - 1) / nchunk;
  nchunk = (ntiles + tpc - 1) / tpc;
  const int ks = 64 / CIT;
  *slices = nchunk * ks;
  const size_t nw = (size_t)Co * 9 * Ci;
  // weight partials [slices][nw], then bias partials [slices][Co]
  int rc = ensure((void **)&nn->part, &nn->part_cap, (size_t)*slices * (nw + Co) * sizeof(float));
  if (rc) return rc;
  hipLaunchKernelGGL((conv3x3_wgrad_kernel<TR, TC, COT, CIT>), dim3((unsigned)pairs, (unsigned)nchunk), dim3(256), 0,
                     nn->stream, dy, x, nn->part, nn->part + (size_t)*slices * nw, N, H, W, Ci, Co, tpc);
  NN_TRY(hipGetLastError());
  return LBTP_OK;
}

template <int TR, int TC, int COT>
int wgrad_ci(lbtp_nn *nn, const bf16 *dy, const bf16 *x, int N, int H, int W, int Ci, int Co, int *slices) {
  if (Ci % 64 == 0) return wgrad_launch<TR, TC, COT, 64>(nn, dy, x, N, H, W, Ci, Co, slices);
  if (Ci % 32 == 0) return wgrad_launch<TR, TC, COT, 32>(nn, dy, x, N, H, W, Ci, Co, slices);
  return wgrad_launch<TR, TC, COT, 16>(nn, dy, x, N, H, W, Ci, Co, slices);
}

template <int TR, int TC>
int wgrad_co(lbtp_nn *nn, const bf16 *dy, const bf16 *x, int N, int H, int W, int Ci, int Co, int *slices) {
  if (Co % 64 == 0) return wgrad_ci<TR, TC, 64>(nn, dy, x, N, H, W, Ci, Co, slices);
  if (Co % 32 == 0) return wgrad_ci<TR, TC, 32>(nn, dy, x, N, H, W, Ci, Co, slices);
  return wgrad_ci<TR, TC, 16>(nn, dy, x, N, H, W, Ci, Co, slices);
}

// Weight- and bias-gradient partials of one convolution into nn->part: *slices
// weight slices, then *slices bias slices.
// Tiles of 128 pixels: 2 x 64 on grids at least 64 wide, 8 x 16 on narrower ones.
int wgrad(lbtp_nn *nn, const bf16 *dy, const bf16 *x, int N, int H, int W, int Ci, int Co, int *slices) {
  if (Ci <= 0 || Ci % 16 || Co <= 0 || Co % 16) return LBTP_EINVAL;
  if (W >= 64) return wgrad_co<2, 64>(nn, dy, x, N, H, W, Ci, Co, slices);
  return wgrad_co<8, 16>(nn, dy, x, N, H, W, Ci, Co, slices);
}

// Gradient of one convolution: given d(output) after the activation in dy (may
// be modified), accumulate dw/db and return d(input) in dx (if non-null).
int conv_bwd(lbtp_nn *nn, int li, const Tape &tp, bf16 *dy, bf16 *dx, int N) {
  const NNLayer &l = nn->L[li];
  const int H = tp.H[li], W = tp.W[li];
  const long long npix = (long long)N * H * W;
  if (l.relu) {
    hipLaunchKernelGGL(relu_mask_kernel, GRID1(npix * l.cop), 0, nn->stream, dy, tp.y[li], npix * l.cop);
    NN_TRY(hipGetLastError());
  }
  // weight and bias gradients: partial sums per (pixel chunk, K slice), added in a fixed order
  const size_t nw = (size_t)l.cop * 9 * l.cip;
  int slices = 0;
  int rc = wgrad(nn, dy, tp.x[li], N, H, W, l.cip, l.cop, &slices);
  if (rc) return rc;
  hipLaunchKernelGGL(sum_chunks_kernel, dim3((unsigned)((nw + 63) / 64)), dim3(256), 0, nn->stream, nn->part, l.dw,
                     (long long)nw, slices);
  NN_TRY(hipGetLastError());
  hipLaunchKernelGGL(sum_chunks_kernel, dim3((unsigned)((l.cop + 63) / 64)), dim3(256), 0, nn->stream,
                     nn->part + (size_t)slices * nw, l.db, (long long)l.cop, slices);
  NN_TRY(hipGetLastError());
  if (dx) {
    if ((rc = conv_fwd(nn, dy, l.wt, nullptr, dx, N, H, W, l.cop, l.cip, false, false))) return rc;
  }
  return LBTP_OK;
}

// Backward pass of the tape; gradients land in nn->grad (flat).
int backward(lbtp_nn *nn, const Tape &tp, int N, int H, int W, bf16 *dhead) {
  int rc = LBTP_OK;
  const int nconv = (int)nn->L.size();
  int slot = 1000;   // gradient tensors live after the forward slots
  auto grad_tensor = [&](size_t elems) { return tensor(nn, slot++, elems, &rc); };
  int li = nconv - 1;
  // head
  {
    const NNLayer &l = nn->L[li];
    bf16 *dx = grad_tensor((size_t)N * tp.H[li] * tp.W[li] * l.cip);
    if (rc) return rc;
    if ((rc = conv_bwd(nn, li, tp, dhead, dx, N))) return rc;
    dhead = dx;
    --li;
  }
  bf16 *dh = dhead;
  std::vector<bf16 *> dskip(nn->levels, nullptr);
  for (int lv = 0; lv <= nn->levels - 2; ++lv) {
    for (int r = 0; r < 2; ++r) {
      const NNLayer &l = nn->L[li];
      bf16 *dx = grad_tensor((size_t)N * tp.H[li] * tp.W[li] * l.cip);
      if (rc) return rc;
      if ((rc = conv_bwd(nn, li, tp, dh, dx, N))) return rc;
      dh = dx;
      --li;
    }
    // dh is d(concat) at this level: split into d(up) and d(skip)
    const NNLayer &l = nn->L[li + 1];
    const int h = tp.H[li + 1], w = tp.W[li + 1];
    const int Cs = nn->L[2 * lv + 1].cop;
    const int Cu = l.cip - Cs;
    bf16 *du = grad_tensor((size_t)N * h * w * Cu);
    bf16 *ds = grad_tensor((size_t)N * h * w * Cs);
    if (rc) return rc;
    hipLaunchKernelGGL(split_kernel, GRID1((long long)N * h * w * (Cu + Cs)), 0, nn->stream, dh, du, ds,
                       (long long)N * h * w, Cu, Cs);
    NN_TRY(hipGetLastError());
    dskip[lv] = ds;
    bf16 *dd = grad_tensor((size_t)N * (h / 2) * (w / 2) * Cu);
    if (rc) return rc;
    hipLaunchKernelGGL(up_bwd_kernel, GRID1((long long)N * (h / 2) * (w / 2) * Cu), 0, nn->stream, du, dd, N, h / 2,
                       w / 2, Cu);
    NN_TRY(hipGetLastError());
    dh = dd;
  }
  for (int lv = nn->levels - 1; lv >= 0; --lv) {
    const NNLayer &top = nn->L[2 * lv + 1];
    const int h = tp.H[2 * lv + 1], w = tp.W[2 * lv + 1];
    if (dskip[lv]) {
      hipLaunchKernelGGL(add_kernel, GRID1((long long)N * h * w * top.cop), 0, nn->stream, dh, dskip[lv],
                         (long long)N * h * w * top.cop);
      NN_TRY(hipGetLastError());
    }
    for (int r = 0; r < 2; ++r) {
      const int idx = 2 * lv + 1 - r;
      const NNLayer &l = nn->L[idx];
      const bool need_dx = !(lv == 0 && r == 1);
      bf16 *dx = need_dx ? grad_tensor((size_t)N * tp.H[idx] * tp.W[idx] * l.cip) : nullptr;
      if (rc) return rc;
      if ((rc = conv_bwd(nn, idx, tp, dh, dx, N))) return rc;
      dh = dx;
    }
    if (lv > 0) {
      const int C = nn->L[2 * lv].cip;
      bf16 *dp = grad_tensor((size_t)N * (2 * h) * (2 * w) * C);
      if (rc) return rc;
      hipLaunchKernelGGL(pool_bwd_kernel, GRID1((long long)N * 4 * h * w * C), 0, nn->stream, dh, dp, N, 2 * h, 2 * w,
                         C);
      NN_TRY(hipGetLastError());
      dh = dp;
    }
  }
  for (NNLayer &l : nn->L) {
    const long long n = (long long)l.co * 9 * l.ci + l.co;
    hipLaunchKernelGGL(unpack_grad_kernel, GRID1(n), 0, nn->stream, l.dw, l.db, l.ci, l.co, l.cip, nn->grad + l.off);
    NN_TRY(hipGetLastError());
  }
  return LBTP_OK;
}

int loss_grad(lbtp_nn *nn, const float *lnK, const float *S, const float *T, const float *wts, int N, int H, int W,
              double *loss) {
  Tape tp;
  int rc = forward(nn, lnK, S, N, H, W, &tp);
  if (rc) return rc;
  const long long npix = (long long)N * H * W;
  float *P = nullptr;
  size_t pcap = 0;
  // predicted pressure in a scratch tensor (float) placed after the head
  if ((rc = ensure((void **)&P, &pcap, (size_t)npix * sizeof(float)))) return rc;
  hipLaunchKernelGGL(head_out_kernel, GRID1(npix), 0, nn->stream, nn->head_cur, P, npix, W, nn->scale);
  int nb = (int)((npix + 255) / 256);
  if ((rc = ensure((void **)&nn->lpart, &nn->lpart_cap, (size_t)(nb + 1) * sizeof(double)))) {
    (void)hipFree(P);
    return rc;
  }
  bf16 *dhead = tensor(nn, 999, (size_t)npix * 16, &rc);
  if (rc) {
    (void)hipFree(P);
    return rc;
  }
  hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, nn->stream, P, T, wts, dhead, nn->lpart, npix,
                     (long long)H * W, nn->scale / W);
  hipLaunchKernelGGL(sum_double_kernel, dim3(1), dim3(256), 0, nn->stream, nn->lpart, nb, nn->lpart + nb,
                     1.0 / (double)npix);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) rc = backward(nn, tp, N, H, W, dhead);
  else rc = LBTP_EHIP;
  if (!rc && loss) {
    e = hipMemcpyAsync(loss, nn->lpart + nb, sizeof(double), hipMemcpyDeviceToHost, nn->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(nn->stream);
    if (e != hipSuccess) rc = LBTP_EHIP;
  }
  (void)hipStreamSynchronize(nn->stream);
  (void)hipFree(P);
  return rc;
}

int check_shape(const lbtp_nn *nn, int N, int H, int W) {
  const int f = 1 << (nn->levels - 1);
  if (N < 1 || H < f || W < f || H % f || W % f) return LBTP_EINVAL;
  return LBTP_OK;
}

// Stage a caller field of n floats on the device (returns the device pointer).
const float *stage(lbtp_nn *nn, const float *p, size_t n, int on_device, std::vector<void *> &tmp, int *rc) {
  if (on_device || !p) return p;
  void *d = nullptr;
  if (hipMalloc(&d, n * sizeof(float)) != hipSuccess) {
    *rc = LBTP_ENOMEM;
    return nullptr;
  }
  tmp.push_back(d);
  if (hipMemcpyAsync(d, p, n * sizeof(float), hipMemcpyHostToDevice, nn->stream) != hipSuccess) *rc = LBTP_EHIP;
  return (const float *)d;
}

void free_tmp(lbtp_nn *nn, std::vector<void *> &tmp) {
  (void)hipStreamSynchronize(nn->stream);
  for (void *p : tmp) (void)hipFree(p);
  tmp.clear();
}

// Device scratch of the no-allocation predict: the activations, the head
// output and the coarsened inputs of one forward pass.  Each device holds its
// own copy from module load until the process ends.  Host code must use the
// address hipGetSymbolAddress returns for the current device, never the
// array's name.
constexpr size_t kNNScratchBytes = (size_t)LBTP_NN_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char nn_scratch[kNNScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Address of nn_scratch on the current device (looked up once per device).
int scratch_of_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LBTP_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(nn_scratch)) != hipSuccess || !p) return LBTP_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LBTP_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes forward() takes from an arena for N x H x W (the same sequence of
// buffers, each rounded up to 256 bytes as arena_take places them).
size_t forward_bytes(const lbtp_nn *nn, int N, int H, int W) {
  const size_t npix = (size_t)N * H * W;
  size_t b = align256(npix * 16 * sizeof(bf16));
  size_t h = H, w = W;
  int li = 0;
  for (int lv = 0; lv < nn->levels; ++lv) {
    if (lv > 0) {
      b += align256((size_t)N * (h / 2) * (w / 2) * nn->L[li - 1].cop * sizeof(bf16));
      h /= 2;
      w /= 2;
    }
    for (int k = 0; k < 2; ++k, ++li) b += align256((size_t)N * h * w * nn->L[li].cop * sizeof(bf16));
  }
  for (int lv = nn->levels - 2; lv >= 0; --lv) {
    const size_t Cu = nn->L[li - 1].cop, Cs = nn->L[2 * lv + 1].cop;
    b += align256((size_t)N * (2 * h) * (2 * w) * Cu * sizeof(bf16));
    h *= 2;
    w *= 2;
    b += align256((size_t)N * h * w * (Cu + Cs) * sizeof(bf16));
    for (int k = 0; k < 2; ++k, ++li) b += align256((size_t)N * h * w * nn->L[li].cop * sizeof(bf16));
  }
  return b + align256(npix * 16 * sizeof(float));
}

}  // namespace

extern "C" {

int lbtp_nn_create(int base, int levels, double scale, void *stream, lbtp_nn **out) {
  if (!out || base < 1 || levels < 1 || levels > 6 || !(scale > 0)) return LBTP_EINVAL;
  *out = nullptr;
  lbtp_nn *nn = new lbtp_nn();
  nn->base = base;
  nn->levels = levels;
  nn->scale = (float)scale;
  nn->stream = (hipStream_t)stream;
  if (hipGetDevice(&nn->device) != hipSuccess) {
    delete nn;
    return LBTP_EHIP;
  }
  {
    // the device scratch of lbtp_nn_predict_noalloc, looked up at set-up
    void *scratch = nullptr;
    if (scratch_of_current_device(&scratch) != LBTP_OK) {
      delete nn;
      return LBTP_EHIP;
    }
  }
  // layer list (same order as the flat parameter vector)
  std::vector<int> c(levels);
  for (int l = 0; l < levels; ++l) c[l] = base << l;
  std::vector<std::pair<int, int>> io;
  std::vector<bool> relu;
  int prev = 3;
  for (int l = 0; l < levels; ++l) {
    io.push_back({prev, c[l]});
    io.push_back({c[l], c[l]});
    relu.push_back(true);
    relu.push_back(true);
    prev = c[l];
  }
  for (int l = levels - 2; l >= 0; --l) {
    io.push_back({c[l + 1] + c[l], c[l]});
    io.push_back({c[l], c[l]});
    relu.push_back(true);
    relu.push_back(true);
  }
  io.push_back({c[0], 1});
  relu.push_back(false);
  size_t off = 0;
  for (size_t i = 0; i < io.size(); ++i) {
    NNLayer l{};
    l.ci = io[i].first;
    l.co = io[i].second;
    l.cip = pad16(l.ci);
    l.cop = pad16(l.co);
    l.relu = relu[i];
    l.off = off;
    off += (size_t)l.co * 9 * l.ci + l.co;
    nn->L.push_back(l);
  }
  nn->np = off;
  bool ok = hipMalloc((void **)&nn->theta, off * 4) == hipSuccess && hipMalloc((void **)&nn->grad, off * 4) == hipSuccess &&
            hipMalloc((void **)&nn->m, off * 4) == hipSuccess && hipMalloc((void **)&nn->v, off * 4) == hipSuccess;
  for (NNLayer &l : nn->L) {
    const size_t nw = (size_t)l.cop * 9 * l.cip;
    ok = ok && hipMalloc((void **)&l.w, nw * 2) == hipSuccess && hipMalloc((void **)&l.wt, nw * 2) == hipSuccess &&
         hipMalloc((void **)&l.b, l.cop * 4) == hipSuccess && hipMalloc((void **)&l.dw, nw * 4) == hipSuccess &&
         hipMalloc((void **)&l.db, l.cop * 4) == hipSuccess;
  }
  if (!ok || hipMemsetAsync(nn->theta, 0, off * 4, nn->stream) != hipSuccess ||
      hipMemsetAsync(nn->m, 0, off * 4, nn->stream) != hipSuccess ||
      hipMemsetAsync(nn->v, 0, off * 4, nn->stream) != hipSuccess || pack_params(nn) != LBTP_OK ||
      hipStreamSynchronize(nn->stream) != hipSuccess) {
    lbtp_nn_destroy(nn);
    return ok ? LBTP_EHIP : LBTP_ENOMEM;
  }
  *out = nn;
  return LBTP_OK;
}

void lbtp_nn_destroy(lbtp_nn *nn) {
  if (!nn) return;
  void *bufs[] = {nn->theta, nn->grad, nn->m, nn->v, nn->part, nn->head, nn->lpart};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  for (NNLayer &l : nn->L) {
    void *lb[] = {l.w, l.wt, l.b, l.dw, l.db};
    for (void *p : lb)
      if (p) (void)hipFree(p);
  }
  for (Tensor &t : nn->act)
    if (t.p) (void)hipFree(t.p);
  delete nn;
}

long long lbtp_nn_num_params(lbtp_nn *nn) { return nn ? (long long)nn->np : LBTP_EINVAL; }

int lbtp_nn_set_params(lbtp_nn *nn, const float *theta, int on_device) {
  if (!nn || !theta) return LBTP_EINVAL;
  NN_TRY(hipMemcpyAsync(nn->theta, theta, nn->np * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        nn->stream));
  NN_TRY(hipMemsetAsync(nn->m, 0, nn->np * 4, nn->stream));
  NN_TRY(hipMemsetAsync(nn->v, 0, nn->np * 4, nn->stream));
  nn->adam_t = 0;
  int rc = pack_params(nn);
  if (rc) return rc;
  NN_TRY(hipStreamSynchronize(nn->stream));
  return LBTP_OK;
}

int lbtp_nn_get_params(lbtp_nn *nn, float *theta, int on_device) {
  if (!nn || !theta) return LBTP_EINVAL;
  NN_TRY(hipMemcpyAsync(theta, nn->theta, nn->np * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        nn->stream));
  NN_TRY(hipStreamSynchronize(nn->stream));
  return LBTP_OK;
}

int lbtp_nn_predict(lbtp_nn *nn, const float *lnK, const float *S, int N, int H, int W, int factor, float *P,
                    int on_device) {
  if (!nn || !lnK || !S || !P || factor < 1 || H % factor || W % factor) return LBTP_EINVAL;
  const int Hc = H / factor, Wc = W / factor;
  int rc = check_shape(nn, N, Hc, Wc);
  if (rc) return rc;
  const size_t npix = (size_t)N * H * W, ncoarse = (size_t)N * Hc * Wc;
  std::vector<void *> tmp;
  const float *dK = stage(nn, lnK, npix, on_device, tmp, &rc);
  const float *dS = stage(nn, S, npix, on_device, tmp, &rc);
  float *dP = P;
  if (!rc && !on_device) {
    if (hipMalloc((void **)&dP, npix * 4) != hipSuccess) rc = LBTP_ENOMEM;
    else tmp.push_back(dP);
  }
  const float *cK = dK, *cS = dS;
  if (!rc && factor > 1) {
    float *c = nullptr;
    if (hipMalloc((void **)&c, 2 * ncoarse * 4) != hipSuccess) rc = LBTP_ENOMEM;
    else {
      tmp.push_back(c);
      hipLaunchKernelGGL(coarsen_kernel, GRID1((long long)ncoarse), 0, nn->stream, dK, dS, c, c + ncoarse,
                         (long long)ncoarse, Hc, Wc, factor);
      cK = c;
      cS = c + ncoarse;
    }
  }
  if (!rc) rc = forward(nn, cK, cS, N, Hc, Wc, nullptr);
  if (!rc) {
    if (factor == 1)
      hipLaunchKernelGGL(head_out_kernel, GRID1((long long)npix), 0, nn->stream, nn->head_cur, dP, (long long)npix, W,
                         nn->scale);
    else
      hipLaunchKernelGGL(upsample_kernel, GRID1((long long)npix), 0, nn->stream, nn->head_cur, dP, (long long)npix, H,
                         W, factor, nn->scale / (float)Wc);
    if (hipGetLastError() != hipSuccess) rc = LBTP_EHIP;
  }
  if (!rc && !on_device &&
      hipMemcpyAsync(P, dP, npix * 4, hipMemcpyDeviceToHost, nn->stream) != hipSuccess)
    rc = LBTP_EHIP;
  free_tmp(nn, tmp);
  return rc;
}

int lbtp_nn_predict_noalloc(lbtp_nn *nn, const float *lnK, const float *S, int N, int H, int W, int factor,
                            float *P) {
  if (!nn || !lnK || !S || !P || factor < 1 || H < 1 || W < 1 || H % factor || W % factor) return LBTP_EINVAL;
  const int Hc = H / factor, Wc = W / factor;
  int rc = check_shape(nn, N, Hc, Wc);
  if (rc) return rc;
  const size_t npix = (size_t)N * H * W, ncoarse = (size_t)N * Hc * Wc;
  const size_t need = forward_bytes(nn, N, Hc, Wc) + (factor > 1 ? align256(2 * ncoarse * sizeof(float)) : 0);
  if (need > kNNScratchBytes) return LBTP_EINVAL;
  void *scratch = nullptr;
  if ((rc = scratch_of_current_device(&scratch))) return rc;
  Arena arena;
  arena.base = (char *)scratch;
  arena.cap = kNNScratchBytes;
  const float *cK = lnK, *cS = S;
  if (factor > 1) {
    float *c = (float *)arena_take(&arena, 2 * ncoarse * sizeof(float), &rc);
    if (rc) return rc;
    hipLaunchKernelGGL(coarsen_kernel, GRID1((long long)ncoarse), 0, nn->stream, lnK, S, c, c + ncoarse,
                       (long long)ncoarse, Hc, Wc, factor);
    if (hipGetLastError() != hipSuccess) return LBTP_EHIP;
    cK = c;
    cS = c + ncoarse;
  }
  nn->arena = &arena;
  rc = forward(nn, cK, cS, N, Hc, Wc, nullptr);
  nn->arena = nullptr;
  if (rc) return rc;
  if (factor == 1)
    hipLaunchKernelGGL(head_out_kernel, GRID1((long long)npix), 0, nn->stream, nn->head_cur, P, (long long)npix, W,
                       nn->scale);
  else
    hipLaunchKernelGGL(upsample_kernel, GRID1((long long)npix), 0, nn->stream, nn->head_cur, P, (long long)npix, H,
                       W, factor, nn->scale / (float)Wc);
  nn->head_cur = nullptr;
  return hipGetLastError() == hipSuccess ? LBTP_OK : LBTP_EHIP;
}

int lbtp_nn_loss_grad(lbtp_nn *nn, const float *lnK, const float *S, const float *P, const float *weight, int N,
                      int H, int W, double *loss, float *grad, int on_device) {
  if (!nn || !lnK || !S || !P) return LBTP_EINVAL;
  int rc = check_shape(nn, N, H, W);
  if (rc) return rc;
  const size_t npix = (size_t)N * H * W;
  std::vector<void *> tmp;
  const float *dK = stage(nn, lnK, npix, on_device, tmp, &rc);
  const float *dS = stage(nn, S, npix, on_device, tmp, &rc);
  const float *dT = stage(nn, P, npix, on_device, tmp, &rc);
  const float *dW = stage(nn, weight, (size_t)N, on_device, tmp, &rc);
  if (!rc) rc = loss_grad(nn, dK, dS, dT, dW, N, H, W, loss);
  if (!rc && grad &&
      hipMemcpyAsync(grad, nn->grad, nn->np * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                     nn->stream) != hipSuccess)
    rc = LBTP_EHIP;
  free_tmp(nn, tmp);
  return rc;
}

int lbtp_nn_train_step(lbtp_nn *nn, const float *lnK, const float *S, const float *P, const float *weight, int N,
                       int H, int W, double lr, double *loss, int on_device) {
  if (!nn || !lnK || !S || !P || !(lr > 0)) return LBTP_EINVAL;
  int rc = check_shape(nn, N, H, W);
  if (rc) return rc;
  const size_t npix = (size_t)N * H * W;
  std::vector<void *> tmp;
  const float *dK = stage(nn, lnK, npix, on_device, tmp, &rc);
  const float *dS = stage(nn, S, npix, on_device, tmp, &rc);
  const float *dT = stage(nn, P, npix, on_device, tmp, &rc);
  const float *dW = stage(nn, weight, (size_t)N, on_device, tmp, &rc);
  if (!rc) rc = loss_grad(nn, dK, dS, dT, dW, N, H, W, loss);
  if (!rc) {
    nn->adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - pow(b1, (double)nn->adam_t)), c2 = (float)(1.0 - pow(b2, (double)nn->adam_t));
    hipLaunchKernelGGL(adam_kernel, GRID1((long long)nn->np), 0, nn->stream, nn->theta, nn->grad, nn->m, nn->v,
                       (long long)nn->np, (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2);
    if (hipGetLastError() != hipSuccess) rc = LBTP_EHIP;
  }
  if (!rc) rc = pack_params(nn);
  free_tmp(nn, tmp);
  return rc;
}

}  // extern "C"
