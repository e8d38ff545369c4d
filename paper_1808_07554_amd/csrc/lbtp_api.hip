// Host side of liblbtp: the C ABI declared in include/lbtp.h.
//
// A context owns the device buffers of one realisation and drives the
// kernels of lbtp_kernels.hip on one stream.  The pressure solve enqueues
// sweeps in chunks of m (the residual stride); the first sweep of every
// chunk evaluates the stopping rule into a device control block, and later
// sweeps of a converged solve return at once, so the host only reads the
// control block one chunk behind the GPU and never stalls it.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/lbtp_probe.h"
#include "lbtp_block.h"
#include "lbtp_internal.h"

using namespace lbtp;

struct lbtp_ctx {
  lbtp_params p;
  int dim = 2, Q = 5, nf = 4;
  int lk = 2;   // lattice kind of the launchers: 2 (D2Q5), 3 (D3Q7), kD2Q9
  long long ncell = 0;
  hipStream_t stream = nullptr;
  KC kc;
  void *fbuf[2] = {nullptr, nullptr};    // nf * ncell deviations of the storage type each
  void *gbuf[2] = {nullptr, nullptr};    // Q * ncell of the storage type each
  float *gB[2] = {nullptr, nullptr};     // 16-bit storage: base saturation of each g buffer
  float *Pb[2] = {nullptr, nullptr};     // base pressure of the f deviations
  int fs = 0, gs = 0, pbs = 0;           // index of the state buffers
  int f_local = 1;                       // state buffer holds pre-collision values
  float *K = nullptr, *phi = nullptr, *Fp = nullptr, *Fs = nullptr;
  int has_Fp = 0, has_Fs = 0;
  float *S = nullptr, *itau = nullptr, *scratch = nullptr;
  float *wallP[6] = {}, *wallS[6] = {};   // per-link Dirichlet data (lbtp_set_wall_values)
  int *wallTF[4] = {}, *wallTG[4] = {};     // per-link conditions, D2Q9 (lbtp_set_wall_types)
  float *itg = nullptr;                    // 1/tau_g per node (cap_B > 0)
  double *partials = nullptr;
  int nblk = 0;
  Ctl *ctl = nullptr;       // device
  Ctl *ctl_host = nullptr;  // pinned mirror
  Ctl *ctl_ring = nullptr;  // pinned, two slots for lookahead polling
  hipEvent_t ev[2] = {nullptr, nullptr};
  long long step = 0;
  int have_fields = 0, have_state = 0, have_coef = 0;
  // captured chunks of m sweeps (+ the check), by (buffer parity, base
  // buffer, checks, F_p); kc_ver counts changes of the launch constants
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t chunk[64] = {};
  int chunk_ver[64] = {};
  int kc_ver = 1;
  int sweep_block = 0;      // plain sweeps per launch inside chunks (0 or 1: one)
};

namespace {

#define HIP_TRY(x)                         \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) return LBTP_EHIP; \
  } while (0)

FPtrs fptrs(const lbtp_ctx *c, void *base) {
  FPtrs r{};
  const size_t es = storage_bytes(c->p.storage);
  for (int j = 0; j < c->nf; ++j) r.p[j] = (char *)base + (size_t)j * c->ncell * es;
  return r;
}
GPtrs gptrs(const lbtp_ctx *c, int idx) {
  GPtrs r{};
  const size_t es = storage_bytes(c->p.storage);
  for (int i = 0; i < c->Q; ++i) r.p[i] = (char *)c->gbuf[idx] + (size_t)i * c->ncell * es;
  r.B = c->gB[idx];
  r.storage = c->p.storage;
  return r;
}

// Lattice constants: D2Q9 of eq. 3-5 / 3-6a; D2Q5 and D3Q7 with c_s^2 = 2 w_1 c^2
// (the moment conditions eq. 3-7 on an axis-aligned lattice).
double weight_rest(int lattice) {
  return lattice == LBTP_D2Q5 ? 1.0 / 3.0 : (lattice == LBTP_D3Q7 ? 1.0 / 4.0 : 4.0 / 9.0);
}
double weight_move(int lattice) {   // axis directions
  return lattice == LBTP_D2Q5 ? 1.0 / 6.0 : (lattice == LBTP_D3Q7 ? 1.0 / 8.0 : 1.0 / 9.0);
}
double cs2_over_c2(int lattice) { return lattice == LBTP_D3Q7 ? 1.0 / 4.0 : 1.0 / 3.0; }
int lattice_dim(int lattice) { return lattice == LBTP_D3Q7 ? 3 : 2; }
int lattice_q(int lattice) { return lattice == LBTP_D2Q5 ? 5 : (lattice == LBTP_D3Q7 ? 7 : 9); }

int validate(const lbtp_params *p) {
  if (!p) return LBTP_EINVAL;
  if (p->lattice != LBTP_D2Q5 && p->lattice != LBTP_D3Q7 && p->lattice != LBTP_D2Q9) return LBTP_EINVAL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return LBTP_EINVAL;
  if (p->lattice != LBTP_D3Q7 && p->nz != 1) return LBTP_EINVAL;
  const long long n = (long long)p->nx * p->ny * p->nz;
  const int Q = lattice_q(p->lattice);
  if ((long long)Q * n >= (1LL << 31)) return LBTP_EINVAL;   // 32-bit cell indexing
  if (!(p->dx > 0) || !(p->dt > 0) || !(p->beta > 0) || !(p->Ds > 0)) return LBTP_EINVAL;
  if (p->coef_model != LBTP_COEF_QUADRATIC_KR && p->coef_model != LBTP_COEF_RATIONAL) return LBTP_EINVAL;
  if (!(p->cap_B >= 0.0) || !isfinite(p->cap_B)) return LBTP_EINVAL;
  if (p->coef_model == LBTP_COEF_QUADRATIC_KR && (!(p->mu_w > 0) || !(p->mu_n > 0))) return LBTP_EINVAL;
  if (p->sweep_block < 0 || (p->sweep_block > 1 && p->sweep_block % 2 == 0)) return LBTP_EINVAL;
  if (p->lattice == LBTP_D3Q7 && p->sweep_block > 1 && !block_sweeps_supported_3d(p->sweep_block)) return LBTP_EINVAL;
  if (p->collision != LBTP_COLLISION_BGK && p->collision != LBTP_COLLISION_MRT) return LBTP_EINVAL;
  if (p->collision == LBTP_COLLISION_MRT) {
    if (p->lattice != LBTP_D2Q9) return LBTP_EINVAL;
    for (int i = 0; i < 3; ++i)
      if (!(p->mrt_rates[i] > 0.0 && p->mrt_rates[i] < 2.0)) return LBTP_EINVAL;
  }
  if (p->coef_model == LBTP_COEF_RATIONAL) {
    for (int i = 0; i < 6; ++i)
      if (!isfinite(p->coef[i])) return LBTP_EINVAL;
    if (p->coef[4] == 0.0 && p->coef[5] == 0.0) return LBTP_EINVAL;
  }
  if (p->storage != LBTP_FP32 && p->storage != LBTP_FP16_DEV && p->storage != LBTP_BF16_DEV) return LBTP_EINVAL;
  if (p->residual_stride < 1) return LBTP_EINVAL;
  const int dim = lattice_dim(p->lattice);
  const double c = p->dx / p->dt;
  const double cs2 = cs2_over_c2(p->lattice) * c * c;
  const double tau_g = 0.5 + p->Ds / (p->beta * cs2 * p->dt);   // eq. 3-11b
  if (!(tau_g > 0.5) || !isfinite(tau_g)) return LBTP_EINVAL;
  for (int a = 0; a < dim; ++a) {
    const int f0 = p->bc_f[2 * a], f1 = p->bc_f[2 * a + 1], g0 = p->bc_g[2 * a], g1 = p->bc_g[2 * a + 1];
    const int per = (f0 == LBTP_BC_PERIODIC) + (f1 == LBTP_BC_PERIODIC) + (g0 == LBTP_BC_PERIODIC) +
                    (g1 == LBTP_BC_PERIODIC);
    if (per != 0 && per != 4) return LBTP_EINVAL;
    for (int s = 0; s < 2; ++s) {
      const int bf = p->bc_f[2 * a + s], bg = p->bc_g[2 * a + s];
      if (bf < 0 || bf > LBTP_BC_NOFLUX) return LBTP_EINVAL;
      if (bg < 0 || bg > LBTP_BC_OUTFLOW) return LBTP_EINVAL;
    }
    const int n = a == 0 ? p->nx : (a == 1 ? p->ny : p->nz);
    if (per == 0 && n < 3) return LBTP_EINVAL;   // one-sided differences at walls
  }
  return LBTP_OK;
}

void fill_kc(lbtp_ctx *c) {
  const lbtp_params &p = c->p;
  KC &k = c->kc;
  memset(&k, 0, sizeof(k));
  k.nx = p.nx;
  k.ny = p.ny;
  k.nz = p.nz;
  k.ncell = (int)c->ncell;
  const double cc = p.dx / p.dt;
  const double cs2 = cs2_over_c2(p.lattice) * cc * cc;
  const double w0 = weight_rest(p.lattice), w1 = weight_move(p.lattice);
  const double tau_g = 0.5 + p.Ds / (p.beta * cs2 * p.dt);
  k.c = (float)cc;
  k.dt = (float)p.dt;
  k.cs2 = (float)cs2;
  k.w0 = (float)w0;
  k.w1 = (float)w1;
  k.w2 = (float)(1.0 / 36.0);
  k.inv_1mw0 = (float)(1.0 / (1.0 - w0));
  k.w1_1mw0 = (float)(w1 / (1.0 - w0));
  k.wbar = (float)(1.0 / c->nf);      // bar-omega_i = 1/(Q-1) for every moving direction
  k.beta = (float)p.beta;
  k.inv_tau_g = (float)(1.0 / tau_g);
  k.src_g = (float)(p.dt * (1.0 - 0.5 / tau_g));
  k.inv_mu_w = p.mu_w > 0 ? (float)(1.0 / p.mu_w) : 0.0f;
  k.inv_mu_n = p.mu_n > 0 ? (float)(1.0 / p.mu_n) : 0.0f;
  k.coef = p.coef_model;
  for (int i = 0; i < 6; ++i) k.cf[i] = (float)p.coef[i];
  k.mrt = p.collision == LBTP_COLLISION_MRT;
  k.ms0 = (float)p.mrt_rates[0];
  k.msq = (float)p.mrt_rates[1];
  k.msp = (float)p.mrt_rates[2];
  k.Ds = (float)p.Ds;
  k.cap_B = (float)p.cap_B;
  k.inv_bcs2dt = (float)(1.0 / (p.beta * cs2 * p.dt));
  k.itg = c->itg;
  k.inv_cs2dt = (float)(1.0 / (cs2 * p.dt));
  k.geq0_phi = (float)((w0 - 1.0) * p.beta);
  k.w1beta = (float)(w1 * p.beta);
  k.half_dt = (float)(0.5 * p.dt);
  k.dev_scale = 1.0f;
  k.inv_dev_scale = 1.0f;
  // fp16 saturation deviations: about one step's change of S times the
  // equilibrium weights, so 2^10 keeps them out of the subnormal range and
  // far below the fp16 maximum
  k.g_scale = p.storage == LBTP_FP16_DEV ? 1024.0f : 1.0f;
  k.inv_g_scale = 1.0f / k.g_scale;
  for (int f = 0; f < 6; ++f) {
    const bool used = f < 2 * c->dim;
    k.bc_f[f] = used ? p.bc_f[f] : LBTP_BC_PERIODIC;
    k.bc_g[f] = used ? p.bc_g[f] : LBTP_BC_PERIODIC;
    k.Pw[f] = (float)p.bc_P[f];
    k.abbS[f] = (float)(2.0 * w1 * p.beta * p.bc_S[f]);
    k.Sw[f] = (float)p.bc_S[f];
  }
}

// Copy n floats from a caller pointer to device memory dst.
int upload(lbtp_ctx *c, float *dst, const float *src, size_t n, int on_device) {
  HIP_TRY(hipMemcpyAsync(dst, src, n * sizeof(float), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         c->stream));
  if (!on_device) HIP_TRY(hipStreamSynchronize(c->stream));
  return LBTP_OK;
}

int download(lbtp_ctx *c, float *dst, const float *src, size_t n, int on_device) {
  HIP_TRY(hipMemcpyAsync(dst, src, n * sizeof(float), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBTP_OK;
}

// Host copy of a caller field (for validation).
int fetch_host(lbtp_ctx *c, const float *src, int on_device, std::vector<float> &out) {
  out.resize(c->ncell);
  if (on_device) {
    HIP_TRY(hipMemcpyAsync(out.data(), src, c->ncell * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  } else {
    memcpy(out.data(), src, c->ncell * sizeof(float));
  }
  return LBTP_OK;
}

bool fully_periodic(const lbtp_ctx *c) {
  for (int f = 0; f < 2 * c->dim; ++f)
    if (c->p.bc_f[f] != LBTP_BC_PERIODIC) return false;
  return true;
}

int set_sources_impl(lbtp_ctx *c, const float *Fp, const float *Fs, int on_device) {
  if (Fp && fully_periodic(c)) {
    // a periodic Poisson problem has a solution only if sum F_p = 0
    std::vector<float> h;
    int rc = fetch_host(c, Fp, on_device, h);
    if (rc) return rc;
    double s = 0.0, a = 0.0;
    for (float v : h) {
      s += v;
      a += fabs((double)v);
    }
    if (fabs(s) > 1e-6 * a + 1e-30) return LBTP_EINVAL;
  }
  if (Fp) {
    int rc = upload(c, c->Fp, Fp, c->ncell, on_device);
    if (rc) return rc;
  }
  if (Fs) {
    int rc = upload(c, c->Fs, Fs, c->ncell, on_device);
    if (rc) return rc;
  }
  c->has_Fp = Fp != nullptr;
  c->has_Fs = Fs != nullptr;
  return LBTP_OK;
}

const float *Fp_or_null(const lbtp_ctx *c) { return c->has_Fp ? c->Fp : nullptr; }
const float *Fs_or_null(const lbtp_ctx *c) { return c->has_Fs ? c->Fs : nullptr; }

int read_ctl(lbtp_ctx *c) {
  HIP_TRY(hipMemcpyAsync(c->ctl_host, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBTP_OK;
}

}  // namespace

extern "C" {

void lbtp_default_params(lbtp_params *p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->lattice = LBTP_D2Q5;
  p->nx = p->ny = p->nz = 1;
  p->dx = p->dt = 1.0;
  p->beta = 1.0;
  p->Ds = 0.0;
  p->mu_w = p->mu_n = 1.0;
  p->storage = LBTP_FP32;
  p->residual_stride = 64;
  p->init_neq = 1;
  p->stream = nullptr;
}

const char *lbtp_strerror(int s) {
  switch (s) {
    case LBTP_OK: return "ok";
    case LBTP_NOT_CONVERGED: return "not converged: iteration limit reached";
    case LBTP_EINVAL: return "invalid argument";
    case LBTP_ENOMEM: return "device allocation failed";
    case LBTP_EHIP: return "HIP runtime error";
    case LBTP_EUNSTABLE: return "unstable: non-finite residual or mass";
    case LBTP_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

void lbtp_destroy(lbtp_ctx *c) {
  if (!c) return;
  void *bufs[] = {c->fbuf[0], c->fbuf[1], c->gbuf[0], c->gbuf[1], c->gB[0], c->gB[1], c->Pb[0], c->Pb[1],
                  c->K, c->phi, c->Fp, c->Fs, c->S, c->itau, c->scratch, c->itg};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  for (int f = 0; f < 6; ++f) {
    if (c->wallP[f]) (void)hipFree(c->wallP[f]);
    if (c->wallS[f]) (void)hipFree(c->wallS[f]);
  }
  for (int f = 0; f < 4; ++f) {
    if (c->wallTF[f]) (void)hipFree(c->wallTF[f]);
    if (c->wallTG[f]) (void)hipFree(c->wallTG[f]);
  }
  if (c->partials) (void)hipFree(c->partials);
  if (c->ctl) (void)hipFree(c->ctl);
  if (c->ctl_host) (void)hipHostFree(c->ctl_host);
  if (c->ctl_ring) (void)hipHostFree(c->ctl_ring);
  for (int i = 0; i < 2; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  for (hipGraphExec_t g : c->chunk)
    if (g) (void)hipGraphExecDestroy(g);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

int lbtp_init(const lbtp_params *p, lbtp_ctx **out) {
  if (!out) return LBTP_EINVAL;
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  lbtp_ctx *c = new lbtp_ctx();
  c->p = *p;
  c->dim = lattice_dim(p->lattice);
  c->Q = lattice_q(p->lattice);
  c->nf = c->Q - 1;
  c->lk = p->lattice == LBTP_D2Q9 ? kD2Q9 : c->dim;
  c->ncell = (long long)p->nx * p->ny * p->nz;
  c->stream = (hipStream_t)p->stream;
  c->nblk = nblocks(c->ncell);
  fill_kc(c);
  {
    const int H = p->sweep_block == 0 ? (p->lattice == LBTP_D3Q7 ? 3 : 9) : p->sweep_block;
    if (H > 1) {
      if (!block_sweeps_supported(c->lk, c->kc, H)) {
        delete c;
        return LBTP_EINVAL;
      }
      c->sweep_block = H;
    }
  }
  const size_t n = (size_t)c->ncell;
  const size_t fbytes = n * c->nf * storage_bytes(p->storage);
  struct {
    void **ptr;
    size_t bytes;
  } allocs[] = {{&c->fbuf[0], fbytes},
                {&c->fbuf[1], fbytes},
                {(void **)&c->gbuf[0], n * c->Q * storage_bytes(p->storage)},
                {(void **)&c->gbuf[1], n * c->Q * storage_bytes(p->storage)},
                {(void **)&c->gB[0], p->storage == LBTP_FP32 ? 0 : n * 4},
                {(void **)&c->gB[1], p->storage == LBTP_FP32 ? 0 : n * 4},
                {(void **)&c->Pb[0], n * 4},
                {(void **)&c->Pb[1], n * 4},
                {(void **)&c->K, n * 4},
                {(void **)&c->phi, n * 4},
                {(void **)&c->Fp, n * 4},
                {(void **)&c->Fs, n * 4},
                {(void **)&c->S, n * 4},
                {(void **)&c->itau, n * 4},
                {(void **)&c->scratch, n * 3 * 4},
                {(void **)&c->itg, p->cap_B > 0.0 ? n * 4 : 0}};
  for (auto &a : allocs) {
    if (a.bytes && hipMalloc(a.ptr, a.bytes) != hipSuccess) {
      lbtp_destroy(c);
      return LBTP_ENOMEM;
    }
  }
  c->kc.itg = c->itg;
  if (hipMalloc((void **)&c->partials, (size_t)c->nblk * 2 * sizeof(double)) != hipSuccess ||
      hipMalloc((void **)&c->ctl, sizeof(Ctl)) != hipSuccess) {
    lbtp_destroy(c);
    return LBTP_ENOMEM;
  }
  if (hipHostMalloc((void **)&c->ctl_host, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&c->ctl_ring, 2 * sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
    lbtp_destroy(c);
    return LBTP_ENOMEM;
  }
  memset(c->ctl_host, 0, sizeof(Ctl));
  memset(c->ctl_ring, 0, 2 * sizeof(Ctl));
  for (int i = 0; i < 2; ++i) {
    if (hipEventCreateWithFlags(&c->ev[i], hipEventDisableTiming) != hipSuccess) {
      lbtp_destroy(c);
      return LBTP_EHIP;
    }
  }
  if (hipMemcpyAsync(c->ctl, c->ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    lbtp_destroy(c);
    return LBTP_EHIP;
  }
  *out = c;
  return LBTP_OK;
}

int lbtp_set_stream(lbtp_ctx *c, void *stream) {
  if (!c) return LBTP_EINVAL;
  c->stream = (hipStream_t)stream;
  c->p.stream = stream;
  return LBTP_OK;
}

int lbtp_set_fields(lbtp_ctx *c, const float *K, const float *phi, const float *Fp, const float *Fs,
                    int on_device) {
  if (!c || !K || !phi) return LBTP_EINVAL;
  std::vector<float> hK, hphi;
  int rc = fetch_host(c, K, on_device, hK);
  if (rc) return rc;
  rc = fetch_host(c, phi, on_device, hphi);
  if (rc) return rc;
  double phimin = INFINITY, phimax = 0.0;
  for (long long i = 0; i < c->ncell; ++i) {
    if (!(hK[i] > 0.0f) || !isfinite(hK[i])) return LBTP_EINVAL;
    if (!(hphi[i] > 0.0f) || !isfinite(hphi[i])) return LBTP_EINVAL;
    phimin = fmin(phimin, (double)hphi[i]);
    phimax = fmax(phimax, (double)hphi[i]);
  }
  if (c->p.lattice == LBTP_D2Q9) {
    // eq. 3-4: phi/2 <= beta <= 2 phi keeps every g^eq non-negative
    if (c->p.beta < 0.5 * phimax * (1.0 - 1e-12) || c->p.beta > 2.0 * phimin * (1.0 + 1e-12)) return LBTP_EINVAL;
  } else {
    // eq. 3-4b: 0 <= beta <= phi / (1 - w0) keeps every g^eq non-negative
    if (c->p.beta > phimin / (1.0 - weight_rest(c->p.lattice)) * (1.0 + 1e-12)) return LBTP_EINVAL;
  }
  rc = upload(c, c->K, K, c->ncell, on_device);
  if (rc) return rc;
  rc = upload(c, c->phi, phi, c->ncell, on_device);
  if (rc) return rc;
  rc = set_sources_impl(c, Fp, Fs, on_device);
  if (rc) return rc;
  c->have_fields = 1;
  return LBTP_OK;
}

int lbtp_set_sources(lbtp_ctx *c, const float *Fp, const float *Fs, int on_device) {
  if (!c) return LBTP_EINVAL;
  if (!c->have_fields) return LBTP_ESTATE;
  return set_sources_impl(c, Fp, Fs, on_device);
}

int lbtp_set_wall_values(lbtp_ctx *c, int face, const float *P, const float *S, int on_device) {
  if (!c || face < 0 || face >= 2 * c->dim) return LBTP_EINVAL;
  // Dirichlet faces, and faces whose links carry their own conditions
  const bool mixed_f = face < 4 && c->wallTF[face], mixed_g = face < 4 && c->wallTG[face];
  if (P && c->p.bc_f[face] != LBTP_BC_DIRICHLET && !mixed_f) return LBTP_EINVAL;
  if (S && c->p.bc_g[face] != LBTP_BC_DIRICHLET && !mixed_g) return LBTP_EINVAL;
  const int a = face / 2;
  const long long nface = c->ncell / (a == 0 ? c->p.nx : (a == 1 ? c->p.ny : c->p.nz));
  const size_t n = (size_t)nface * (c->p.lattice == LBTP_D2Q9 ? 3 : 1);
  float **dst[2] = {&c->wallP[face], &c->wallS[face]};
  const float *src[2] = {P, S};
  for (int i = 0; i < 2; ++i) {
    if (!src[i]) continue;
    if (!*dst[i] && hipMalloc((void **)dst[i], n * sizeof(float)) != hipSuccess) return LBTP_ENOMEM;
    int rc = upload(c, *dst[i], src[i], n, on_device);
    if (rc) return rc;
  }
  c->kc.wP[face] = c->wallP[face];
  c->kc.wS[face] = c->wallS[face];
  c->kc_ver += 1;
  return LBTP_OK;
}

int lbtp_set_wall_types(lbtp_ctx *c, int face, const int *f_types, const int *g_types, int on_device) {
  if (!c || c->p.lattice != LBTP_D2Q9 || face < 0 || face >= 4) return LBTP_EINVAL;
  if (f_types && c->p.bc_f[face] == LBTP_BC_PERIODIC) return LBTP_EINVAL;
  if (g_types && c->p.bc_g[face] == LBTP_BC_PERIODIC) return LBTP_EINVAL;
  const size_t n = (size_t)(face < 2 ? c->p.ny : c->p.nx) * 3;
  int **dst[2] = {&c->wallTF[face], &c->wallTG[face]};
  const int *src[2] = {f_types, g_types};
  std::vector<int> h[2];
  // validate every list before changing anything
  for (int i = 0; i < 2; ++i) {
    if (!src[i]) continue;
    h[i].resize(n);
    if (on_device) {
      HIP_TRY(hipMemcpyAsync(h[i].data(), src[i], n * sizeof(int), hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
    } else {
      memcpy(h[i].data(), src[i], n * sizeof(int));
    }
    for (int t : h[i]) {
      const bool ok = t == LBTP_BC_DIRICHLET || t == LBTP_BC_NOFLUX || (i == 1 && t == LBTP_BC_OUTFLOW);
      if (!ok) return LBTP_EINVAL;
    }
  }
  for (int i = 0; i < 2; ++i) {
    if (!src[i]) continue;
    if (!*dst[i] && hipMalloc((void **)dst[i], n * sizeof(int)) != hipSuccess) return LBTP_ENOMEM;
    HIP_TRY(hipMemcpyAsync(*dst[i], h[i].data(), n * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  c->kc.wtF[face] = c->wallTF[face];
  c->kc.wtG[face] = c->wallTG[face];
  c->kc_ver += 1;
  return LBTP_OK;
}

int lbtp_set_state(lbtp_ctx *c, const float *P0, const float *S0, const float *dP0, const float *dS0,
                   int on_device) {
  if (!c || !P0 || !S0) return LBTP_EINVAL;
  if (!c->have_fields) return LBTP_ESTATE;
  const size_t n = (size_t)c->ncell;
  if (c->p.storage == LBTP_FP16_DEV) {
    // fp16 deviations are scaled so that w_1 max|P| maps to about 1024: the
    // deviations (at most a few w_1 |P|) stay below the fp16 maximum and the
    // typical ones stay out of the subnormal range
    std::vector<float> h;
    int rc = fetch_host(c, P0, on_device, h);
    if (rc) return rc;
    double pmax = 0.0;
    for (float v : h) pmax = fmax(pmax, fabs((double)v));
    for (int f = 0; f < 2 * c->dim; ++f)
      if (c->p.bc_f[f] == LBTP_BC_DIRICHLET) pmax = fmax(pmax, fabs(c->p.bc_P[f]));
    if (!(pmax > 0.0) || !isfinite(pmax)) pmax = 1.0;
    const int e2 = (int)floor(log2(1024.0 / (weight_move(c->p.lattice) * pmax)));
    c->kc.dev_scale = (float)ldexp(1.0, e2 < -60 ? -60 : (e2 > 60 ? 60 : e2));
    c->kc.inv_dev_scale = 1.0f / c->kc.dev_scale;
    c->kc_ver += 1;
  }
  // stage P0 in the second base buffer, S0 in S, dP0 in scratch and dS0 in
  // the second f buffer (at least dim floats per node for every storage)
  int rc = upload(c, c->Pb[1], P0, n, on_device);
  if (rc) return rc;
  rc = upload(c, c->S, S0, n, on_device);
  if (rc) return rc;
  const float *dP = nullptr, *dS = nullptr;
  if (dP0) {
    rc = upload(c, c->scratch, dP0, n * c->dim, on_device);
    if (rc) return rc;
    dP = c->scratch;
  }
  if (dS0) {
    rc = upload(c, (float *)c->fbuf[1], dS0, n * c->dim, on_device);
    if (rc) return rc;
    dS = (const float *)c->fbuf[1];
  }
  HIP_TRY(launch_init(c->lk, c->p.storage, c->kc, c->Pb[1], c->S, dP, dS, c->K, c->phi, Fs_or_null(c),
                      c->p.init_neq, fptrs(c, c->fbuf[0]), c->Pb[0], gptrs(c, 0), c->stream));
  c->fs = 0;
  c->gs = 0;
  c->pbs = 0;
  c->f_local = 1;
  c->step = 0;
  c->ctl_host->ledger = 0.0;
  HIP_TRY(hipMemcpyAsync(&c->ctl->ledger, &c->ctl_host->ledger, sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->have_state = 1;
  c->have_coef = 0;
  return LBTP_OK;
}

int lbtp_update_coefficients(lbtp_ctx *c) {
  if (!c) return LBTP_EINVAL;
  if (!c->have_state) return LBTP_ESTATE;
  HIP_TRY(launch_moments(c->lk, c->kc, gptrs(c, c->gs), c->K, c->phi, Fs_or_null(c), c->S, c->itau,
                         c->partials, 1, c->stream));
  HIP_TRY(launch_finish_sum(c->partials, c->nblk, &c->ctl->mass, 0, nullptr, c->stream));
  c->have_coef = 1;
  return LBTP_OK;
}

namespace {
// Launch lengths covering n consecutive sweeps with blocked launches only
// (D2Q5): odd lengths (a launch must end in the buffer n single sweeps
// would), as few launches as the supported lengths allow near the configured
// length H, the longer ones first.  Returns the number of launches, or 0
// where chunks keep their one-sweep launches.
int fused_plan(const lbtp_ctx *c, int n, int *len, int cap) {
  const int H = c->sweep_block;
  if (H < 3 || n < 3 || !block_first_supported(c->lk, c->kc, 3)) return 0;
  int hmax = 0;
  for (int h = 3; h <= 63; h += 2)
    if (block_first_supported(c->lk, c->kc, h)) hmax = h;
  int b = n / H;
  if (b < 1) b = 1;
  if ((b & 1) != (n & 1)) b = b > 1 ? b - 1 : b + 1;
  while (b <= cap && n > b * hmax) b += 2;
  if (b > cap) return 0;
  int q = n / b;
  if (!(q & 1)) --q;
  if (q < 3) return 0;
  int d = n - b * q;     // even: n and b * q have b's parity
  for (int i = 0; i < b; ++i) len[i] = q;
  for (int i = 0; d > 0; i = (i + 1) % b, d -= 2) len[i] += 2;
  for (int i = 0; i < b; ++i)
    if (len[i] > hmax) return 0;
  return b;
}

constexpr int kMaxLaunches = 64;

// The launches of one chunk: m sweeps with one re-basing sweep and, with
// checks, one evaluation of the stopping rule.  kChunkOneSweep: sweeps
// k0+1 .. k0+m, blocked where the lattice allows and one per launch
// otherwise, sweep k0+m re-basing and checking in a launch of its own.
// kChunkFused (D2Q5, blocked launches only): sweeps k0 .. k0+m-1, the first
// launch performing the re-basing sweep k0 as its first sweep; with checks a
// probe of sweep k0+m (a one-sweep launch that only forms P and the
// stopping-rule sums) follows.  The re-basing sweep k0+m opens the next
// chunk, so the state a check passes on (the one sweep k0+m reads) is the
// one in memory.  kChunkFusedAfterLocal: the same for chunk 1 after a
// one-sweep local sweep 0, sweeps 1 .. m-1 and the probe of m.  With m even
// the buffer parities of a chunk depend only on fs.
enum ChunkKind { kChunkOneSweep = 0, kChunkFused = 1, kChunkFusedAfterLocal = 2 };

hipError_t enqueue_chunk(lbtp_ctx *c, long long k0, int pb, bool checks, int kind, hipStream_t s) {
  const int m = c->p.residual_stride;
  if (kind != kChunkOneSweep) {
    const bool first = kind == kChunkFused;
    int len[kMaxLaunches];
    const int nb = fused_plan(c, first ? m : m - 1, len, kMaxLaunches);
    if (nb <= 0) return hipErrorInvalidValue;   // callers ask for it only where the plan exists
    long long k = first ? k0 : k0 + 1;
    int cur = pb;
    for (int b = 0; b < nb; ++b) {
      const int parity = (int)((c->fs + k) & 1);
      const hipError_t e =
          (first && b == 0)
              ? launch_f_block_first(c->p.storage, c->kc, fptrs(c, c->fbuf[parity]), fptrs(c, c->fbuf[parity ^ 1]),
                                     c->Pb[cur], c->Pb[cur ^ 1], c->itau, Fp_or_null(c), c->ctl, k, len[b], s)
              : launch_f_block(c->lk, c->p.storage, c->kc, fptrs(c, c->fbuf[parity]), fptrs(c, c->fbuf[parity ^ 1]),
                               c->Pb[cur], c->itau, Fp_or_null(c), c->ctl, k, len[b], s);
      if (e != hipSuccess) return e;
      if (first && b == 0) cur ^= 1;
      k += len[b];
    }
    if (!checks) return hipSuccess;
    const int parity = (int)((c->fs + k) & 1);
    hipError_t e = launch_f_sweep(c->lk, c->p.storage, c->kc, fptrs(c, c->fbuf[parity]),
                                  fptrs(c, c->fbuf[parity ^ 1]), c->Pb[cur], c->Pb[cur ^ 1], c->itau, Fp_or_null(c),
                                  c->partials, c->ctl, k, 0, 3, s);
    if (e == hipSuccess) e = launch_finish_residual(c->partials, sweep_blocks(c->kc, 0), c->ctl, m, s);
    return e;
  }
  int i = 1;
  // plain sweeps in blocks of H (H odd: a block ends in the buffer where H
  // single sweeps would), the rest one by one
  const int H = c->sweep_block;
  for (; H > 1 && i + H - 1 <= m - 1; i += H) {
    const long long k = k0 + i;
    const int parity = (int)((c->fs + k) & 1);
    const hipError_t e = launch_f_block(c->lk, c->p.storage, c->kc, fptrs(c, c->fbuf[parity]),
                                        fptrs(c, c->fbuf[parity ^ 1]), c->Pb[pb], c->itau, Fp_or_null(c), c->ctl,
                                        k, H, s);
    if (e != hipSuccess) return e;
  }
  for (; i <= m; ++i) {
    const long long k = k0 + i;
    const int parity = (int)((c->fs + k) & 1);
    const int mode = i < m ? 0 : (checks ? 2 : 1);
    hipError_t e = launch_f_sweep(c->lk, c->p.storage, c->kc, fptrs(c, c->fbuf[parity]),
                                  fptrs(c, c->fbuf[parity ^ 1]), c->Pb[pb], c->Pb[pb ^ 1], c->itau, Fp_or_null(c),
                                  c->partials, c->ctl, k, 0, mode, s);
    if (e == hipSuccess && mode == 2)
      e = launch_finish_residual(c->partials, sweep_blocks(c->kc, 0), c->ctl, m, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The executable graph of a full chunk in the current configuration,
// captured on first use (on a private stream: the caller's may be the null
// stream) and again after the launch constants change.  The sweeps' own
// iteration arguments are those of the first chunk; they only guard against
// sweeps beyond the iteration limit, which a full chunk never reaches, and
// the check counts iterations on the device.
hipError_t chunk_graph(lbtp_ctx *c, int pb, bool checks, int kind, hipGraphExec_t *out) {
  const int key = (c->fs & 1) | (pb << 1) | ((checks ? 1 : 0) << 2) | ((c->has_Fp ? 1 : 0) << 3) | (kind << 4);
  if (c->chunk[key] && c->chunk_ver[key] == c->kc_ver) {
    *out = c->chunk[key];
    return hipSuccess;
  }
  if (c->chunk[key]) {
    (void)hipGraphExecDestroy(c->chunk[key]);
    c->chunk[key] = nullptr;
  }
  hipError_t e = hipSuccess;
  if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  // the fs of the first chunk of a solve: sweeps 1..m read (fs + k) & 1
  const hipError_t el = enqueue_chunk(c, 0, pb, checks, kind, c->cap_stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->cap_stream, &g);
  if (el != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return el != hipSuccess ? el : e;
  }
  e = hipGraphInstantiate(&c->chunk[key], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->chunk[key] = nullptr;
    return e;
  }
  c->chunk_ver[key] = c->kc_ver;
  *out = c->chunk[key];
  return hipSuccess;
}
}  // namespace

int lbtp_pressure_solve(lbtp_ctx *c, double tol, long long max_iters, long long *iters, double *resid) {
  if (!c || max_iters < 0) return LBTP_EINVAL;
  if (!c->have_coef) return LBTP_ESTATE;
  const int m = c->p.residual_stride;
  const bool checks = tol >= 0.0;
  HIP_TRY(launch_ctl_reset(c->ctl, max_iters, tol, c->stream));
  // Sweep k reads buffer (fs + k) & 1 and computes P^k; sweep k < max_iters
  // also produces f^{k+1}.  With checks on, sweeps k = 0, m, 2m, ... <=
  // max_iters handle the snapshot and the stopping rule.
  long long last = max_iters - 1;   // last sweep whose output is needed
  if (checks) last = (max_iters / m) * m > last ? (max_iters / m) * m : last;
  // Sweep k reads the deviations of buffer (fs + k) & 1 against base pb and
  // writes the other buffer.  Sweep 0 and every sweep with k % m == 0 reset
  // the base to the current P (writing the other base buffer); with checks on,
  // those with k > 0 also evaluate the stopping rule.
  int pb = c->pbs;
  long long probed = -1;     // a sweep whose check a fused chunk's probe has made
  auto sweep = [&](long long k) -> hipError_t {
    const int parity = (int)((c->fs + k) & 1);
    const int mode = (k % m != 0) ? 0 : ((k == 0 || !checks || k == probed) ? 1 : 2);
    const int local = (k == 0) && c->f_local;
    hipError_t e = launch_f_sweep(c->lk, c->p.storage, c->kc, fptrs(c, c->fbuf[parity]),
                                  fptrs(c, c->fbuf[parity ^ 1]), c->Pb[pb], c->Pb[pb ^ 1], c->itau,
                                  Fp_or_null(c), c->partials, c->ctl, k, local, mode, c->stream);
    if (e == hipSuccess && mode == 2)
      e = launch_finish_residual(c->partials, sweep_blocks(c->kc, local), c->ctl, m, c->stream);
    if (mode >= 1) pb ^= 1;
    return e;
  };
  // full chunks run as captured graphs (m even: the parities repeat)
  const bool graphs = m % 2 == 0 && m > 1;
  // fused chunks (enqueue_chunk): chunk j is sweeps (j-1)m .. jm-1 and the
  // probe of jm; after a local sweep 0, chunk 1 is sweeps 1 .. m-1 and the
  // probe of m
  int plan[kMaxLaunches];
  const bool fused = graphs && fused_plan(c, m, plan, kMaxLaunches) > 0 &&
                     (!c->f_local || fused_plan(c, m - 1, plan, kMaxLaunches) > 0);
  // Chunk 0 is sweep 0 (snapshot of P^0) where it runs alone; chunk j >= 1
  // ends with the check at jm.  The first check is waited for at once (warm
  // steps usually stop there); later ones are read one chunk behind so the
  // GPU never idles while the host decides.
  long long k = 0;
  if (last >= 0 && (!fused || c->f_local)) {
    HIP_TRY(sweep(0));
    k = 1;
  }
  int slot = 0, last_copy = -1;   // ring slot of the control block copied after the last enqueued work
  bool pending[2] = {false, false};
  bool stop = false;
  for (long long j = 1; k <= last; ++j) {
    last_copy = -1;
    const long long kend = (j * m < last) ? j * m : last;
    // a fused chunk ends at sweep jm - 1 (the probe of jm only with checks
    // on), so without checks it also serves a solve that stops there
    const bool full = graphs && (kend == j * m || (fused && !checks && kend == j * m - 1));
    if (full && fused && (k == (j - 1) * m || (j == 1 && k == 1))) {
      const bool first = k == (j - 1) * m;     // the chunk performs the re-basing sweep (j-1)m
      hipGraphExec_t g = nullptr;
      HIP_TRY(chunk_graph(c, pb, checks, first ? kChunkFused : kChunkFusedAfterLocal, &g));
      HIP_TRY(hipGraphLaunch(g, c->stream));
      if (first) pb ^= 1;
      // sweep jm, re-basing, opens the next chunk; its output is needed only
      // below max_iters (with checks on, its check is made)
      k = j * m < max_iters ? j * m : last + 1;
      if (checks) probed = j * m;
    } else if (full && !fused && k == (j - 1) * m + 1) {
      hipGraphExec_t g = nullptr;
      HIP_TRY(chunk_graph(c, pb, checks, kChunkOneSweep, &g));
      HIP_TRY(hipGraphLaunch(g, c->stream));
      pb ^= 1;
      k = kend + 1;
    } else {
      for (; k <= kend; ++k) HIP_TRY(sweep(k));
    }
    if (!checks || k > last) continue;
    HIP_TRY(hipMemcpyAsync(&c->ctl_ring[slot], c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipEventRecord(c->ev[slot], c->stream));
    pending[slot] = true;
    last_copy = slot;
    const int prev = slot ^ 1;
    int wait = -1;
    if (j == 1) wait = slot;
    else if (pending[prev]) wait = prev;
    if (wait >= 0) {
      HIP_TRY(hipEventSynchronize(c->ev[wait]));
      pending[wait] = false;
      stop = c->ctl_ring[wait].done != 0;
    }
    slot = prev;
    if (stop) break;
  }
  if (stop && last_copy >= 0) {
    // the copy behind the last enqueued work is the final control block (work
    // queued after a stop only exits early and leaves it as it is)
    if (pending[last_copy]) HIP_TRY(hipEventSynchronize(c->ev[last_copy]));
    pending[last_copy] = false;
    *c->ctl_host = c->ctl_ring[last_copy];
  } else {
    const int rc = read_ctl(c);
    if (rc) return rc;
  }
  const Ctl &h = *c->ctl_host;
  long long K;
  int status;
  if (h.done) {
    K = h.K;
    status = h.status;
  } else {
    K = max_iters;
    status = checks ? LBTP_NOT_CONVERGED : LBTP_OK;
  }
  if (K > 0) {
    // the state is the buffer sweep K read, against the base sweep K read:
    // sweeps 0 and k % m == 0 (k < K) reset the base
    const long long flips = 1 + (K - 1) / m;
    c->fs = (int)((c->fs + K) & 1);
    c->pbs = (int)((c->pbs + flips) & 1);
    c->f_local = 0;
  }
  if (iters) *iters = K;
  if (resid) *resid = h.resid;
  if (!checks && status == LBTP_OK && max_iters > 0) status = LBTP_NOT_CONVERGED;
  return status;
}

int lbtp_probe_sweeps(lbtp_ctx *c, long long launches) {
  if (!c || launches < 0) return LBTP_EINVAL;
  if (!c->have_coef || c->f_local) return LBTP_ESTATE;
  const int H = c->sweep_block > 1 ? c->sweep_block : 1;
  // no stopping rule: clear a finished solve's flag so the sweeps run
  HIP_TRY(launch_ctl_reset(c->ctl, 1LL << 62, -1.0, c->stream));
  for (long long i = 0; i < launches; ++i) {
    const int parity = c->fs & 1;
    if (H > 1) {
      HIP_TRY(launch_f_block(c->lk, c->p.storage, c->kc, fptrs(c, c->fbuf[parity]), fptrs(c, c->fbuf[parity ^ 1]),
                             c->Pb[c->pbs], c->itau, Fp_or_null(c), c->ctl, 1, H, c->stream));
    } else {
      HIP_TRY(launch_f_sweep(c->lk, c->p.storage, c->kc, fptrs(c, c->fbuf[parity]), fptrs(c, c->fbuf[parity ^ 1]),
                             c->Pb[c->pbs], c->Pb[c->pbs ^ 1], c->itau, Fp_or_null(c), c->partials, c->ctl, 1, 0, 0,
                             c->stream));
    }
    c->fs ^= 1;       // H is odd: every launch leaves the state in the other buffer
  }
  return H;
}

int lbtp_saturation_step(lbtp_ctx *c) {
  if (!c) return LBTP_EINVAL;
  if (!c->have_coef) return LBTP_ESTATE;
  HIP_TRY(launch_g_sweep(c->lk, c->p.storage, c->kc, gptrs(c, c->gs), gptrs(c, c->gs ^ 1),
                         fptrs(c, c->fbuf[c->fs]), c->f_local, c->Pb[c->pbs], c->itau, c->K, c->phi, Fs_or_null(c),
                         c->S, c->partials, c->stream));
  HIP_TRY(launch_finish_sum(c->partials, g_sweep_blocks(c->lk, c->kc, c->f_local), &c->ctl->ledger, 1,
                            &c->ctl->last_flux, c->stream));
  c->gs ^= 1;
  c->step += 1;
  c->have_coef = 0;
  return LBTP_OK;
}

int lbtp_step(lbtp_ctx *c, long long nsteps, double tol, long long max_iters, long long *iters) {
  if (!c || nsteps < 0) return LBTP_EINVAL;
  if (!c->have_state) return LBTP_ESTATE;
  int worst = LBTP_OK;
  for (long long n = 0; n < nsteps; ++n) {
    int rc = lbtp_update_coefficients(c);
    if (rc) return rc;
    long long k = 0;
    rc = lbtp_pressure_solve(c, tol, max_iters, &k, nullptr);
    if (iters) iters[n] = k;
    if (rc < 0) return rc;
    if (rc == LBTP_NOT_CONVERGED && tol >= 0.0) worst = LBTP_NOT_CONVERGED;
    rc = lbtp_saturation_step(c);
    if (rc) return rc;
  }
  return worst;
}

int lbtp_pressure(lbtp_ctx *c, float *P, int on_device) {
  if (!c || !P) return LBTP_EINVAL;
  if (!c->have_state) return LBTP_ESTATE;
  HIP_TRY(launch_pressure(c->lk, c->p.storage, c->kc, fptrs(c, c->fbuf[c->fs]), c->f_local, c->Pb[c->pbs],
                          c->scratch, c->stream));
  return download(c, P, c->scratch, c->ncell, on_device);
}

static int grad_common(lbtp_ctx *c, float *out, int on_device, int velocity) {
  if (!c || !out) return LBTP_EINVAL;
  if (!c->have_state) return LBTP_ESTATE;
  if (!c->have_coef && c->step == 0) {
    // coefficients of the initial state
    int rc = lbtp_update_coefficients(c);
    if (rc) return rc;
  }
  HIP_TRY(launch_grad(c->lk, c->p.storage, c->kc, fptrs(c, c->fbuf[c->fs]), c->f_local, c->Pb[c->pbs], c->itau,
                      c->K, c->S, velocity, c->scratch, c->stream));
  return download(c, out, c->scratch, (size_t)c->ncell * c->dim, on_device);
}

int lbtp_velocity(lbtp_ctx *c, float *u, int on_device) { return grad_common(c, u, on_device, 1); }
int lbtp_grad_p(lbtp_ctx *c, float *g, int on_device) { return grad_common(c, g, on_device, 0); }

int lbtp_saturation(lbtp_ctx *c, float *S, int on_device) {
  if (!c || !S) return LBTP_EINVAL;
  if (!c->have_state) return LBTP_ESTATE;
  HIP_TRY(launch_saturation(c->lk, c->kc, gptrs(c, c->gs), c->phi, Fs_or_null(c), c->scratch,
                            c->stream));
  return download(c, S, c->scratch, c->ncell, on_device);
}

int lbtp_mass(lbtp_ctx *c, double *mass, double *ledger) {
  if (!c) return LBTP_EINVAL;
  if (!c->have_state) return LBTP_ESTATE;
  HIP_TRY(launch_moments(c->lk, c->kc, gptrs(c, c->gs), c->K, c->phi, Fs_or_null(c), nullptr, nullptr,
                         c->partials, 0, c->stream));
  HIP_TRY(launch_finish_sum(c->partials, c->nblk, &c->ctl->mass, 0, nullptr, c->stream));
  int rc = read_ctl(c);
  if (rc) return rc;
  if (mass) *mass = c->ctl_host->mass;
  if (ledger) *ledger = c->ctl_host->ledger;
  if (!isfinite(c->ctl_host->mass)) return LBTP_EUNSTABLE;
  return LBTP_OK;
}

int lbtp_phase_velocities(lbtp_ctx *c, float *uw, float *un, int on_device) {
  if (!c || !uw || !un) return LBTP_EINVAL;
  if (!c->have_coef) return LBTP_ESTATE;
  const size_t nv = (size_t)c->ncell * c->dim;
  HIP_TRY(launch_grad(c->lk, c->p.storage, c->kc, fptrs(c, c->fbuf[c->fs]), c->f_local, c->Pb[c->pbs], c->itau,
                      c->K, c->S, 1, c->scratch, c->stream));
  float *dw = uw, *dn = un;
  if (!on_device) {
    if (hipMalloc((void **)&dw, 2 * nv * sizeof(float)) != hipSuccess) return LBTP_ENOMEM;
    dn = dw + nv;
  }
  hipError_t e = launch_phase(c->dim, c->kc, c->scratch, c->S, c->K, (float)c->p.Ds, dw, dn, c->stream);
  if (e == hipSuccess && !on_device) {
    e = hipMemcpyAsync(uw, dw, nv * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(un, dn, nv * sizeof(float), hipMemcpyDeviceToHost, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (!on_device) (void)hipFree(dw);
  return e == hipSuccess ? LBTP_OK : LBTP_EHIP;
}

int lbtp_populations(lbtp_ctx *c, float *f, float *g, int on_device) {
  if (!c) return LBTP_EINVAL;
  if (!c->have_state) return LBTP_ESTATE;
  const size_t n = (size_t)c->ncell;
  if (f) {
    float *dst = f;
    if (!on_device && hipMalloc((void **)&dst, n * c->nf * sizeof(float)) != hipSuccess) return LBTP_ENOMEM;
    hipError_t e = launch_populations(c->lk, c->p.storage, c->kc, fptrs(c, c->fbuf[c->fs]), c->f_local,
                                      c->Pb[c->pbs], dst, c->stream);
    if (e == hipSuccess && !on_device)
      e = hipMemcpyAsync(f, dst, n * c->nf * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (!on_device) (void)hipFree(dst);
    if (e != hipSuccess) return LBTP_EHIP;
  }
  if (g) {
    if (c->p.storage == LBTP_FP32) {
      int rc = download(c, g, (const float *)c->gbuf[c->gs], n * c->Q, on_device);
      if (rc) return rc;
    } else {
      // 16-bit deviations: reconstruct g_i = e_i + g_i^eq(B) in float32
      float *dst = g;
      if (!on_device && hipMalloc((void **)&dst, n * c->Q * sizeof(float)) != hipSuccess) return LBTP_ENOMEM;
      hipError_t e = launch_g_populations(c->lk, c->kc, gptrs(c, c->gs), c->phi, dst, c->stream);
      if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(g, dst, n * c->Q * sizeof(float), hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (!on_device) (void)hipFree(dst);
      if (e != hipSuccess) return LBTP_EHIP;
    }
  }
  return LBTP_OK;
}

namespace {
struct CkptHeader {
  uint32_t magic, version;
  int32_t lattice, nx, ny, nz, storage, f_local;
  int64_t step;
  double ledger;
  float dev_scale, inv_dev_scale;
};
constexpr uint32_t kCkptMagic = 0x5054424Cu;   // "LBTP"

size_t ckpt_parts(const lbtp_ctx *c, size_t *fb, size_t *pb, size_t *gb) {
  const size_t n = (size_t)c->ncell;
  *fb = n * c->nf * storage_bytes(c->p.storage);
  *pb = n * sizeof(float);
  // g populations of the storage type, and with 16-bit storage their base
  // saturation (float32) after them
  *gb = n * c->Q * storage_bytes(c->p.storage) + (c->p.storage == LBTP_FP32 ? 0 : n * sizeof(float));
  return sizeof(CkptHeader) + *fb + *pb + *gb;
}

int copy_bytes(lbtp_ctx *c, void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, kind, c->stream));
  return LBTP_OK;
}
}  // namespace

long long lbtp_checkpoint_size(lbtp_ctx *c) {
  if (!c) return LBTP_EINVAL;
  size_t fb, pb, gb;
  return (long long)ckpt_parts(c, &fb, &pb, &gb);
}

int lbtp_get_state(lbtp_ctx *c, void *buf, long long nbytes, int on_device) {
  if (!c || !buf) return LBTP_EINVAL;
  if (!c->have_state) return LBTP_ESTATE;
  size_t fb, pb, gb;
  if (nbytes < (long long)ckpt_parts(c, &fb, &pb, &gb)) return LBTP_EINVAL;
  int rc = read_ctl(c);
  if (rc) return rc;
  CkptHeader h{};
  h.magic = kCkptMagic;
  h.version = 2;
  h.lattice = c->p.lattice;
  h.nx = c->p.nx;
  h.ny = c->p.ny;
  h.nz = c->p.nz;
  h.storage = c->p.storage;
  h.f_local = c->f_local;
  h.step = c->step;
  h.ledger = c->ctl_host->ledger;
  h.dev_scale = c->kc.dev_scale;
  h.inv_dev_scale = c->kc.inv_dev_scale;
  char *out = (char *)buf;
  const hipMemcpyKind d2x = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (on_device) {
    rc = copy_bytes(c, out, &h, sizeof(h), hipMemcpyHostToDevice);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
  } else {
    memcpy(out, &h, sizeof(h));
  }
  out += sizeof(h);
  if ((rc = copy_bytes(c, out, c->fbuf[c->fs], fb, d2x))) return rc;
  if ((rc = copy_bytes(c, out + fb, c->Pb[c->pbs], pb, d2x))) return rc;
  const size_t gpop = (size_t)c->ncell * c->Q * storage_bytes(c->p.storage);
  if ((rc = copy_bytes(c, out + fb + pb, c->gbuf[c->gs], gpop, d2x))) return rc;
  if (gb > gpop && (rc = copy_bytes(c, out + fb + pb + gpop, c->gB[c->gs], gb - gpop, d2x))) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBTP_OK;
}

int lbtp_put_state(lbtp_ctx *c, const void *buf, long long nbytes, int on_device) {
  if (!c || !buf) return LBTP_EINVAL;
  if (!c->have_fields) return LBTP_ESTATE;
  size_t fb, pb, gb;
  if (nbytes < (long long)ckpt_parts(c, &fb, &pb, &gb)) return LBTP_EINVAL;
  CkptHeader h;
  const char *in = (const char *)buf;
  if (on_device) {
    HIP_TRY(hipMemcpyAsync(&h, in, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  } else {
    memcpy(&h, in, sizeof(h));
  }
  if (h.magic != kCkptMagic || h.version != 2 || h.lattice != c->p.lattice || h.nx != c->p.nx ||
      h.ny != c->p.ny || h.nz != c->p.nz || h.storage != c->p.storage)
    return LBTP_EINVAL;
  in += sizeof(h);
  const hipMemcpyKind x2d = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  int rc;
  if ((rc = copy_bytes(c, c->fbuf[0], in, fb, x2d))) return rc;
  if ((rc = copy_bytes(c, c->Pb[0], in + fb, pb, x2d))) return rc;
  const size_t gpop = (size_t)c->ncell * c->Q * storage_bytes(c->p.storage);
  if ((rc = copy_bytes(c, c->gbuf[0], in + fb + pb, gpop, x2d))) return rc;
  if (gb > gpop && (rc = copy_bytes(c, c->gB[0], in + fb + pb + gpop, gb - gpop, x2d))) return rc;
  c->ctl_host->ledger = h.ledger;
  if ((rc = copy_bytes(c, &c->ctl->ledger, &c->ctl_host->ledger, sizeof(double), hipMemcpyHostToDevice))) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->fs = 0;
  c->gs = 0;
  c->pbs = 0;
  c->f_local = h.f_local;
  c->step = h.step;
  c->kc.dev_scale = h.dev_scale;
  c->kc.inv_dev_scale = h.inv_dev_scale;
  c->kc_ver += 1;
  c->have_state = 1;
  c->have_coef = 0;
  return LBTP_OK;
}

int lbtp_copy_probe(void *dst, const void *src, long long bytes, void *stream) {
  if (!dst || !src || bytes <= 0 || bytes % 16 != 0) return LBTP_EINVAL;
  if ((((uintptr_t)dst) | ((uintptr_t)src)) % 16 != 0) return LBTP_EINVAL;
  HIP_TRY(launch_copy_probe(src, dst, bytes / 16, (hipStream_t)stream));
  return LBTP_OK;
}

}  // extern "C"

// ======================================================================
// Ensembles.  A batch owns one lbtp_ctx per member (so every per-member call
// reuses the single-realisation code and buffers) plus the tables that let
// one launch cover all members.
// ======================================================================
struct lbtp_batch {
  int n = 0, dim = 2, storage = 0, m = 64, nt = 256;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<lbtp_ctx *> ctx;
  Member *d_mem = nullptr;
  BCtl *d_ctl = nullptr, *h_ctl = nullptr;      // h_ctl pinned
  int *d_tm_s = nullptr, *d_ti_s = nullptr;     // sweep tiling (4*nt nodes per tile)
  int *d_tm_c = nullptr, *d_ti_c = nullptr;     // cell tiling (kCellTile nodes per tile)
  int ntiles_s = 0, ntiles_c = 0, tiles_cap = 0;
  int H = 1;                                    // plain sweeps per launch before tuning (blocked if > 1)
  // members of one grid size share a class: its blocked tiling (region
  // shape and block length, chosen by lbtp_batch_autotune) and tile tables
  struct Class {
    int nx = 0, ny = 0, nz = 0;
    int shape = 0, H = 1;
    int *d_tm = nullptr, *d_ti = nullptr;
    int ntiles = 0, cap = 0;
    bool any_fp = false, any_nofp = false;
  };
  std::vector<Class> cls;
  std::vector<int> mclass;                      // class of each member
  bool any_fp = false, any_nofp = false;        // members with / without a pressure source
  double *partials = nullptr;
  int *d_active = nullptr, *h_active = nullptr;  // h_active: pinned, two slots
  hipEvent_t ev[2] = {nullptr, nullptr};
  // captured chunk sequences: graph k runs 2^k chunks back to back (members
  // that stop return at once from the rest), so the host reads the active
  // count once per 2^k chunks
  static constexpr int kGraphs = 5;
  hipGraphExec_t chunk[kGraphs] = {};
  long long last_chunks = 1;                    // chunks the slowest member needed in the last step
  int gs = 0, f_local = 1;
  long long step = 0;
};

namespace {

void batch_drop_graphs(lbtp_batch *b) {
  for (auto &g : b->chunk) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

void batch_free(lbtp_batch *b) {
  if (!b) return;
  batch_drop_graphs(b);
  void *bufs[] = {b->d_mem, b->d_ctl, b->d_tm_s, b->d_ti_s, b->d_tm_c, b->d_ti_c, b->partials, b->d_active};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  for (auto &k : b->cls) {
    if (k.d_tm) (void)hipFree(k.d_tm);
    if (k.d_ti) (void)hipFree(k.d_ti);
  }
  if (b->h_ctl) (void)hipHostFree(b->h_ctl);
  if (b->h_active) (void)hipHostFree(b->h_active);
  for (int i = 0; i < 2; ++i)
    if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
  for (lbtp_ctx *c : b->ctx) lbtp_destroy(c);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

// (Re)build the member table and both tile tables for sweep width nt.
int batch_tables(lbtp_batch *b, int nt) {
  std::vector<Member> mem(b->n);
  std::vector<int> tm_s, ti_s, tm_c, ti_c;
  std::vector<std::vector<int>> tm_b(b->cls.size()), ti_b(b->cls.size());
  const int tile_s = 4 * nt;
  b->any_fp = b->any_nofp = false;
  for (auto &k : b->cls) k.any_fp = k.any_nofp = false;
  for (int i = 0; i < b->n; ++i) {
    lbtp_ctx *c = b->ctx[i];
    Member &M = mem[i];
    memset(&M, 0, sizeof(M));
    M.kc = c->kc;
    M.f[0] = fptrs(c, c->fbuf[0]);
    M.f[1] = fptrs(c, c->fbuf[1]);
    M.g[0] = gptrs(c, 0);
    M.g[1] = gptrs(c, 1);
    M.Pb[0] = c->Pb[0];
    M.Pb[1] = c->Pb[1];
    M.K = c->K;
    M.phi = c->phi;
    M.S = c->S;
    M.itau = c->itau;
    M.Fp = c->has_Fp ? c->Fp : nullptr;
    M.Fs = c->has_Fs ? c->Fs : nullptr;
    const int ns = (int)((c->ncell + tile_s - 1) / tile_s);
    const int nc = (int)((c->ncell + kCellTile - 1) / kCellTile);
    M.tstart_s = (int)tm_s.size();
    M.ntiles_s = ns;
    M.tstart_c = (int)tm_c.size();
    M.ntiles_c = nc;
    for (int t = 0; t < ns; ++t) {
      tm_s.push_back(i);
      ti_s.push_back(t);
    }
    for (int t = 0; t < nc; ++t) {
      tm_c.push_back(i);
      ti_c.push_back(t);
    }
    lbtp_batch::Class &k = b->cls[b->mclass[i]];
    if (k.H > 1) {
      int tx, ty;
      block_tile_counts_rows(c->kc, k.H, batch_shape_rows(k.shape), &tx, &ty);
      for (int t = 0; t < tx * ty; ++t) {
        tm_b[b->mclass[i]].push_back(i);
        ti_b[b->mclass[i]].push_back(t);
      }
    }
    (M.Fp ? b->any_fp : b->any_nofp) = true;
    (M.Fp ? k.any_fp : k.any_nofp) = true;
  }
  for (size_t ci = 0; ci < b->cls.size(); ++ci) {
    lbtp_batch::Class &k = b->cls[ci];
    if ((int)tm_b[ci].size() > k.cap) {
      for (int **p : {&k.d_tm, &k.d_ti}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
        if (hipMalloc((void **)p, tm_b[ci].size() * sizeof(int)) != hipSuccess) return LBTP_ENOMEM;
      }
      k.cap = (int)tm_b[ci].size();
    }
    k.ntiles = (int)tm_b[ci].size();
    if (k.ntiles) {
      HIP_TRY(hipMemcpyAsync(k.d_tm, tm_b[ci].data(), k.ntiles * sizeof(int), hipMemcpyHostToDevice, b->stream));
      HIP_TRY(hipMemcpyAsync(k.d_ti, ti_b[ci].data(), k.ntiles * sizeof(int), hipMemcpyHostToDevice, b->stream));
    }
  }
  const int need = (int)(tm_s.size() > tm_c.size() ? tm_s.size() : tm_c.size());
  if (need > b->tiles_cap) {
    for (int **p : {&b->d_tm_s, &b->d_ti_s, &b->d_tm_c, &b->d_ti_c}) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
      if (hipMalloc((void **)p, need * sizeof(int)) != hipSuccess) return LBTP_ENOMEM;
    }
    if (b->partials) (void)hipFree(b->partials);
    b->partials = nullptr;
    if (hipMalloc((void **)&b->partials, (size_t)need * 2 * sizeof(double)) != hipSuccess) return LBTP_ENOMEM;
    b->tiles_cap = need;
  }
  b->ntiles_s = (int)tm_s.size();
  b->ntiles_c = (int)tm_c.size();
  b->nt = nt;
  HIP_TRY(hipMemcpyAsync(b->d_mem, mem.data(), b->n * sizeof(Member), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_tm_s, tm_s.data(), tm_s.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_ti_s, ti_s.data(), ti_s.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_tm_c, tm_c.data(), tm_c.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_ti_c, ti_c.data(), ti_c.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  batch_drop_graphs(b);
  return LBTP_OK;
}

// Enqueue one chunk: sweeps j = 1 .. m (the last one evaluates the stopping
// rule and re-bases), then the per-member finish.
int batch_enqueue_chunk(lbtp_batch *b) {
  // plain sweeps of each size class in blocks of its H (H odd: a block ends
  // in the buffer where H single sweeps would); every class ends its blocks
  // at the same sweep (one shared H, or tuned H that divide m - 1), and the
  // rest run one by one over all members
  int jend = -1;
  for (const auto &k : b->cls) {
    int j = 1;
    for (; k.H > 1 && j + k.H - 1 <= b->m - 1; j += k.H)
      for (int fp = 0; fp < 2; ++fp)
        if (fp ? k.any_fp : k.any_nofp)
          HIP_TRY(batch_launch_block(b->storage, k.shape, fp != 0, k.ntiles, b->d_mem, b->d_ctl, k.d_tm, k.d_ti, j,
                                     k.H, b->stream));
    if (jend >= 0 && j != jend) return LBTP_EINVAL;
    jend = j;
  }
  for (int j = jend < 1 ? 1 : jend; j <= b->m; ++j) {
    const int mode = (j == b->m) ? 2 : 0;
    HIP_TRY(batch_launch_sweep(b->nt, b->dim, b->storage, mode, 0, b->ntiles_s, b->d_mem, b->d_ctl, b->d_tm_s,
                               b->d_ti_s, b->partials, j, b->stream));
  }
  HIP_TRY(batch_launch_finish(b->n, b->d_mem, b->d_ctl, b->partials, b->m, b->d_active, b->stream));
  return LBTP_OK;
}

// Graph k: 2^k chunks.
int batch_capture(lbtp_batch *b, int k) {
  if (b->chunk[k]) return LBTP_OK;
  HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  int rc = LBTP_OK;
  for (int i = 0; i < (1 << k) && !rc; ++i) rc = batch_enqueue_chunk(b);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return LBTP_EHIP;
  e = hipGraphInstantiate(&b->chunk[k], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->chunk[k] = nullptr;
    return LBTP_EHIP;
  }
  return LBTP_OK;
}

// Tuned blocked tilings, kept for the life of the process: (nx, ny,
// storage, m) -> (region shape, block length).
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, std::pair<int, int>> g_tuned;

bool batch_ready(const lbtp_batch *b) {
  for (lbtp_ctx *c : b->ctx)
    if (!c->have_state) return false;
  return true;
}

}  // namespace

extern "C" {

int lbtp_batch_init(const lbtp_params *members, int n, lbtp_batch **out) {
  if (!out || !members || n < 1) return LBTP_EINVAL;
  *out = nullptr;
  const lbtp_params &p0 = members[0];
  if (p0.residual_stride < 2 || p0.residual_stride % 2) return LBTP_EINVAL;
  for (int i = 0; i < n; ++i) {
    const lbtp_params &p = members[i];
    if (p.lattice != p0.lattice || p.storage != p0.storage || p.residual_stride != p0.residual_stride ||
        p.stream != p0.stream || p.sweep_block != p0.sweep_block)
      return LBTP_EINVAL;
    if (p.nx % 4) return LBTP_EINVAL;   // the ensemble sweep runs four nodes per thread
    int rc = validate(&p);
    if (rc) return rc;
  }
  lbtp_batch *b = new lbtp_batch();
  b->n = n;
  // lattice kind of the ensemble launchers: 2 (D2Q5), 3 (D3Q7), kD2Q9
  b->dim = p0.lattice == LBTP_D2Q5 ? 2 : (p0.lattice == LBTP_D3Q7 ? 3 : kD2Q9);
  b->storage = p0.storage;
  b->m = p0.residual_stride;
  if (p0.stream) {
    b->stream = (hipStream_t)p0.stream;
  } else {
    // graph capture needs a stream other than the null stream
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return LBTP_EHIP;
    }
    b->own_stream = true;
  }
  for (int i = 0; i < n; ++i) {
    lbtp_params p = members[i];
    p.stream = b->stream;
    lbtp_ctx *c = nullptr;
    int rc = lbtp_init(&p, &c);
    if (rc) {
      batch_free(b);
      return rc;
    }
    b->ctx.push_back(c);
  }
  if (hipMalloc((void **)&b->d_mem, n * sizeof(Member)) != hipSuccess ||
      hipMalloc((void **)&b->d_ctl, n * sizeof(BCtl)) != hipSuccess ||
      hipMalloc((void **)&b->d_active, sizeof(int)) != hipSuccess ||
      hipHostMalloc((void **)&b->h_ctl, n * sizeof(BCtl), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&b->h_active, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    batch_free(b);
    return LBTP_ENOMEM;
  }
  memset(b->h_ctl, 0, n * sizeof(BCtl));
  for (int i = 0; i < 2; ++i) {
    if (hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming) != hipSuccess) {
      batch_free(b);
      return LBTP_EHIP;
    }
  }
  if (hipMemcpyAsync(b->d_ctl, b->h_ctl, n * sizeof(BCtl), hipMemcpyHostToDevice, b->stream) != hipSuccess) {
    batch_free(b);
    return LBTP_EHIP;
  }
  // blocked plain sweeps: D2Q5 ensembles (D2Q9 and D3Q7 members sweep one
  // sweep per launch, four nodes per thread on D2Q9)
  b->H = (b->dim == 2 && b->ctx[0]->sweep_block > 1) ? b->ctx[0]->sweep_block : 1;
  // size classes; a blocked tiling tuned earlier in the process for a
  // class's size, storage and m is taken over
  for (int i = 0; i < n; ++i) {
    const lbtp_params &p = members[i];
    int ci = 0;
    while (ci < (int)b->cls.size() &&
           !(b->cls[ci].nx == p.nx && b->cls[ci].ny == p.ny && b->cls[ci].nz == p.nz))
      ++ci;
    if (ci == (int)b->cls.size()) {
      lbtp_batch::Class k;
      k.nx = p.nx;
      k.ny = p.ny;
      k.nz = p.nz;
      k.H = b->H;
      b->cls.push_back(k);
    }
    b->mclass.push_back(ci);
  }
  if (b->H > 1) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    bool all = true;
    for (const auto &k : b->cls) all = all && g_tuned.count(std::make_tuple(k.nx, k.ny, b->storage, b->m)) > 0;
    if (all)
      for (auto &k : b->cls) {
        const auto v = g_tuned[std::make_tuple(k.nx, k.ny, b->storage, b->m)];
        k.shape = v.first;
        k.H = v.second;
      }
  }
  int rc = batch_tables(b, 256);
  if (rc) {
    batch_free(b);
    return rc;
  }
  *out = b;
  return LBTP_OK;
}

void lbtp_batch_destroy(lbtp_batch *b) { batch_free(b); }

int lbtp_batch_size(lbtp_batch *b) { return b ? b->n : LBTP_EINVAL; }

int lbtp_batch_set_fields(lbtp_batch *b, int i, const float *K, const float *phi, const float *Fp, const float *Fs,
                          int on_device) {
  if (!b || i < 0 || i >= b->n) return LBTP_EINVAL;
  int rc = lbtp_set_fields(b->ctx[i], K, phi, Fp, Fs, on_device);
  if (rc) return rc;
  return batch_tables(b, b->nt);   // source pointers may have appeared or gone
}

int lbtp_batch_set_state(lbtp_batch *b, int i, const float *P0, const float *S0, const float *dP0,
                         const float *dS0, int on_device) {
  if (!b || i < 0 || i >= b->n) return LBTP_EINVAL;
  int rc = lbtp_set_state(b->ctx[i], P0, S0, dP0, dS0, on_device);
  if (rc) return rc;
  // a fresh state: base buffer 0, no ledger, local form (all members are
  // (re)initialised before the first ensemble step)
  BCtl h{};
  h.pb = 0;
  HIP_TRY(hipMemcpyAsync(&b->d_ctl[i], &h, sizeof(BCtl), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->gs = 0;
  b->f_local = 1;
  b->step = 0;
  return batch_tables(b, b->nt);   // dev_scale of fp16 members is set by set_state
}

int lbtp_batch_set_threads(lbtp_batch *b, int nt) {
  if (!b || (nt != 64 && nt != 128 && nt != 256 && nt != 512)) return LBTP_EINVAL;
  return batch_tables(b, nt);
}

int lbtp_batch_step(lbtp_batch *b, long long nsteps, double tol, long long max_iters, long long *iters) {
  if (!b || nsteps < 0 || max_iters < b->m || max_iters % b->m) return LBTP_EINVAL;
  if (!batch_ready(b)) return LBTP_ESTATE;
  int worst = LBTP_OK;
  for (long long s = 0; s < nsteps; ++s) {
    // coefficients of every member
    HIP_TRY(batch_launch_moments(b->dim, b->storage, b->ntiles_c, b->d_mem, b->d_tm_c, b->d_ti_c, b->partials,
                                 b->gs, 1, b->stream));
    HIP_TRY(batch_launch_sum(b->n, b->d_mem, b->d_ctl, b->partials, 0, b->stream));
    // pressure solve of every member: first sweep (re-base), then chunks
    HIP_TRY(batch_launch_reset(b->n, b->d_ctl, max_iters, tol, b->d_active, b->stream));
    HIP_TRY(batch_launch_sweep(b->nt, b->dim, b->storage, 1, b->f_local, b->ntiles_s, b->d_mem, b->d_ctl, b->d_tm_s,
                               b->d_ti_s, b->partials, 0, b->stream));
    HIP_TRY(batch_launch_flip(b->n, b->d_ctl, b->stream));
    // chunks in graphs of 2^k: as many as the slowest member needed in the
    // last step at first (one in the first step), then doubling; the host
    // reads the active count after each graph, one graph behind
    int slot = 0;
    bool pending[2] = {false, false};
    const long long max_chunks = max_iters / b->m;
    long long done = 0, want = b->last_chunks;
    for (int launch = 0;; ++launch) {
      int k = 0;
      while (k + 1 < lbtp_batch::kGraphs && (2LL << k) <= want && done + (2LL << k) <= max_chunks) ++k;
      int rc = batch_capture(b, k);
      if (rc) return rc;
      HIP_TRY(hipGraphLaunch(b->chunk[k], b->stream));
      done += 1LL << k;
      want = want > (1LL << k) ? want - (1LL << k) : 2 * (1LL << k);
      HIP_TRY(hipMemcpyAsync(&b->h_active[slot], b->d_active, sizeof(int), hipMemcpyDeviceToHost, b->stream));
      HIP_TRY(hipEventRecord(b->ev[slot], b->stream));
      pending[slot] = true;
      const int prev = slot ^ 1;
      int wait = launch == 0 ? slot : (pending[prev] ? prev : -1);
      bool stop = done >= max_chunks;
      if (wait >= 0) {
        HIP_TRY(hipEventSynchronize(b->ev[wait]));
        pending[wait] = false;
        if (b->h_active[wait] == 0) stop = true;
      }
      slot = prev;
      if (stop) break;
    }
    // saturation step of every member, then its flux into the ledger
    HIP_TRY(batch_launch_gsweep(b->dim, b->storage, 0, b->ntiles_c, b->d_mem, b->d_ctl, b->d_tm_c, b->d_ti_c,
                                b->partials, b->gs, b->stream));
    HIP_TRY(batch_launch_sum(b->n, b->d_mem, b->d_ctl, b->partials, 1, b->stream));
    HIP_TRY(hipMemcpyAsync(b->h_ctl, b->d_ctl, b->n * sizeof(BCtl), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->gs ^= 1;
    b->f_local = 0;
    b->step += 1;
    long long slowest = 1;
    for (int i = 0; i < b->n; ++i) slowest = std::max(slowest, (b->h_ctl[i].K + b->m - 1) / b->m);
    b->last_chunks = slowest;
    for (int i = 0; i < b->n; ++i) {
      const BCtl &h = b->h_ctl[i];
      if (iters) iters[s * b->n + i] = h.K;
      if (h.status == LBTP_EUNSTABLE) return LBTP_EUNSTABLE;
      if (h.status == LBTP_NOT_CONVERGED && tol >= 0.0) worst = LBTP_NOT_CONVERGED;
      // keep the member contexts consistent with the ensemble state
      lbtp_ctx *c = b->ctx[i];
      c->fs = 0;
      c->pbs = h.pb;
      c->gs = b->gs;
      c->f_local = 0;
      c->step = b->step;
      c->have_coef = 0;
    }
  }
  return worst;
}

int lbtp_batch_pressure(lbtp_batch *b, int i, float *P, int on_device) {
  if (!b || i < 0 || i >= b->n) return LBTP_EINVAL;
  return lbtp_pressure(b->ctx[i], P, on_device);
}

int lbtp_batch_saturation(lbtp_batch *b, int i, float *S, int on_device) {
  if (!b || i < 0 || i >= b->n) return LBTP_EINVAL;
  return lbtp_saturation(b->ctx[i], S, on_device);
}

int lbtp_batch_velocity(lbtp_batch *b, int i, float *u, int on_device) {
  if (!b || i < 0 || i >= b->n) return LBTP_EINVAL;
  return lbtp_velocity(b->ctx[i], u, on_device);
}

int lbtp_batch_mass(lbtp_batch *b, int i, double *mass, double *ledger) {
  if (!b || i < 0 || i >= b->n) return LBTP_EINVAL;
  double m = 0.0;
  int rc = lbtp_mass(b->ctx[i], &m, nullptr);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(&b->h_ctl[i], &b->d_ctl[i], sizeof(BCtl), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (mass) *mass = m;
  if (ledger) *ledger = b->h_ctl[i].ledger;
  return LBTP_OK;
}

int lbtp_batch_autotune(lbtp_batch *b, int sweeps, int *threads) {
  if (!b || sweeps < 1) return LBTP_EINVAL;
  if (!batch_ready(b)) return LBTP_ESTATE;
  // time plain sweeps of every member (state untouched: sweeps read buffer 0,
  // write buffer 1) for each block width and keep the fastest
  hipEvent_t t0, t1;
  HIP_TRY(hipEventCreate(&t0));
  HIP_TRY(hipEventCreate(&t1));
  const int cand[4] = {64, 128, 256, 512};
  int best = b->nt;
  float best_ms = 1e30f;
  int rc = LBTP_OK;
  HIP_TRY(batch_launch_reset(b->n, b->d_ctl, 1LL << 60, -1.0, b->d_active, b->stream));
  for (int ci = 0; ci < 4 && !rc; ++ci) {
    rc = batch_tables(b, cand[ci]);
    if (rc) break;
    for (int w = 0; w < 2 && !rc; ++w)
      if (batch_launch_sweep(b->nt, b->dim, b->storage, 0, b->f_local, b->ntiles_s, b->d_mem, b->d_ctl, b->d_tm_s,
                             b->d_ti_s, b->partials, 0, b->stream) != hipSuccess)
        rc = LBTP_EHIP;
    if (rc) break;
    if (hipEventRecord(t0, b->stream) != hipSuccess) rc = LBTP_EHIP;
    for (int r = 0; r < sweeps && !rc; ++r)
      if (batch_launch_sweep(b->nt, b->dim, b->storage, 0, b->f_local, b->ntiles_s, b->d_mem, b->d_ctl, b->d_tm_s,
                             b->d_ti_s, b->partials, 0, b->stream) != hipSuccess)
        rc = LBTP_EHIP;
    if (!rc && (hipEventRecord(t1, b->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess)) rc = LBTP_EHIP;
    float ms = 0.f;
    if (!rc && hipEventElapsedTime(&ms, t0, t1) != hipSuccess) rc = LBTP_EHIP;
    if (!rc && ms < best_ms) {
      best_ms = ms;
      best = cand[ci];
    }
  }
  if (rc) {
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    return rc;
  }
  rc = batch_tables(b, best);
  // the blocked plain sweeps, class by class: every region shape and every
  // odd block length H >= 3 that divides the m - 1 plain sweeps of a chunk
  // and leaves tiles of at least 16 x 16 nodes; timed over the launches of
  // one chunk (reading buffer 0, writing buffer 1: the state is untouched)
  if (!rc && b->H > 1) {
    std::vector<std::pair<int, int>> cands;
    for (int sh = 0; sh < kBatchShapes; ++sh)
      for (int H = 3; H <= b->m - 1; H += 2)
        if ((b->m - 1) % H == 0 && kBX - 2 * H >= 16 && batch_shape_rows(sh) - 2 * H >= 16) cands.push_back({sh, H});
    for (size_t ci = 0; ci < b->cls.size() && !rc && !cands.empty(); ++ci) {
      lbtp_batch::Class &k = b->cls[ci];
      float kbest_ms = 1e30f;
      std::pair<int, int> kbest = cands[0];
      for (const auto &cd : cands) {
        k.shape = cd.first;
        k.H = cd.second;
        if ((rc = batch_tables(b, b->nt))) break;
        const int nl = (b->m - 1) / k.H;
        auto run = [&]() {
          for (int l = 0; l < nl && !rc; ++l)
            for (int fp = 0; fp < 2 && !rc; ++fp)
              if ((fp ? k.any_fp : k.any_nofp) &&
                  batch_launch_block(b->storage, k.shape, fp != 0, k.ntiles, b->d_mem, b->d_ctl, k.d_tm, k.d_ti, 0,
                                     k.H, b->stream) != hipSuccess)
                rc = LBTP_EHIP;
        };
        run();   // warm-up
        if (!rc && hipEventRecord(t0, b->stream) != hipSuccess) rc = LBTP_EHIP;
        for (int r = 0; r < sweeps && !rc; ++r) run();
        if (!rc && (hipEventRecord(t1, b->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess))
          rc = LBTP_EHIP;
        float ms = 0.f;
        if (!rc && hipEventElapsedTime(&ms, t0, t1) != hipSuccess) rc = LBTP_EHIP;
        if (!rc && ms < kbest_ms) {
          kbest_ms = ms;
          kbest = cd;
        }
      }
      k.shape = kbest.first;
      k.H = kbest.second;
    }
    if (!rc) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      for (const auto &k : b->cls) g_tuned[std::make_tuple(k.nx, k.ny, b->storage, b->m)] = {k.shape, k.H};
    }
    if (!rc) rc = batch_tables(b, b->nt);
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (rc) return rc;
  if (threads) *threads = best;
  return LBTP_OK;
}

int lbtp_batch_tiling(lbtp_batch *b, int member, int *waves, int *rows_per_wave, int *sweeps_per_launch) {
  if (!b || member < 0 || member >= b->n) return LBTP_EINVAL;
  const lbtp_batch::Class &k = b->cls[b->mclass[member]];
  if (waves) *waves = k.H > 1 ? batch_shape_w(k.shape) : 0;
  if (rows_per_wave) *rows_per_wave = k.H > 1 ? batch_shape_rw(k.shape) : 0;
  if (sweeps_per_launch) *sweeps_per_launch = k.H;
  return LBTP_OK;
}

}  // extern "C"
