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

#include <vector>

#include "lbtp_internal.h"

using namespace lbtp;

struct lbtp_ctx {
  lbtp_params p;
  int dim = 2, Q = 5, nf = 4;
  long long ncell = 0;
  hipStream_t stream = nullptr;
  KC kc;
  float *fbuf[2] = {nullptr, nullptr};   // nf * ncell each
  float *gbuf[2] = {nullptr, nullptr};   // Q * ncell each
  int fs = 0, gs = 0;                    // index of the state buffer
  int f_local = 1;                       // state buffer holds pre-collision values
  float *K = nullptr, *phi = nullptr, *Fp = nullptr, *Fs = nullptr;
  int has_Fp = 0, has_Fs = 0;
  float *S = nullptr, *itau = nullptr, *Psnap = nullptr, *scratch = nullptr;
  double *partials = nullptr;
  int nblk = 0;
  Ctl *ctl = nullptr;       // device
  Ctl *ctl_host = nullptr;  // pinned mirror
  Ctl *ctl_ring = nullptr;  // pinned, two slots for lookahead polling
  hipEvent_t ev[2] = {nullptr, nullptr};
  long long step = 0;
  int have_fields = 0, have_state = 0, have_coef = 0;
};

namespace {

#define HIP_TRY(x)                         \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) return LBTP_EHIP; \
  } while (0)

FPtrs fptrs(const lbtp_ctx *c, float *base) {
  FPtrs r{};
  for (int j = 0; j < c->nf; ++j) r.p[j] = base + (size_t)j * c->ncell;
  return r;
}
GPtrs gptrs(const lbtp_ctx *c, float *base) {
  GPtrs r{};
  for (int i = 0; i < c->Q; ++i) r.p[i] = base + (size_t)i * c->ncell;
  return r;
}

double weight_rest(int lattice) { return lattice == LBTP_D2Q5 ? 1.0 / 3.0 : 1.0 / 4.0; }
double weight_move(int lattice) { return lattice == LBTP_D2Q5 ? 1.0 / 6.0 : 1.0 / 8.0; }
double cs2_over_c2(int lattice) { return lattice == LBTP_D2Q5 ? 1.0 / 3.0 : 1.0 / 4.0; }

int validate(const lbtp_params *p) {
  if (!p) return LBTP_EINVAL;
  if (p->lattice != LBTP_D2Q5 && p->lattice != LBTP_D3Q7) return LBTP_EINVAL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return LBTP_EINVAL;
  if (p->lattice == LBTP_D2Q5 && p->nz != 1) return LBTP_EINVAL;
  const long long n = (long long)p->nx * p->ny * p->nz;
  const int Q = p->lattice == LBTP_D2Q5 ? 5 : 7;
  if ((long long)Q * n >= (1LL << 31)) return LBTP_EINVAL;   // 32-bit cell indexing
  if (!(p->dx > 0) || !(p->dt > 0) || !(p->beta > 0) || !(p->Ds > 0)) return LBTP_EINVAL;
  if (!(p->mu_w > 0) || !(p->mu_n > 0)) return LBTP_EINVAL;
  if (p->storage != LBTP_FP32) return LBTP_EINVAL;
  if (p->residual_stride < 1) return LBTP_EINVAL;
  const int dim = p->lattice == LBTP_D2Q5 ? 2 : 3;
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
  k.inv_1mw0 = (float)(1.0 / (1.0 - w0));
  k.wbar = (float)(1.0 / (2 * c->dim));
  k.beta = (float)p.beta;
  k.inv_tau_g = (float)(1.0 / tau_g);
  k.src_g = (float)(p.dt * (1.0 - 0.5 / tau_g));
  k.inv_mu_w = (float)(1.0 / p.mu_w);
  k.inv_mu_n = (float)(1.0 / p.mu_n);
  k.inv_cs2dt = (float)(1.0 / (cs2 * p.dt));
  k.geq0_phi = (float)((w0 - 1.0) * p.beta);
  k.w1beta = (float)(w1 * p.beta);
  k.half_dt = (float)(0.5 * p.dt);
  for (int f = 0; f < 6; ++f) {
    const bool used = f < 2 * c->dim;
    k.bc_f[f] = used ? p.bc_f[f] : LBTP_BC_PERIODIC;
    k.bc_g[f] = used ? p.bc_g[f] : LBTP_BC_PERIODIC;
    k.abbP[f] = (float)(2.0 * w1 * p.bc_P[f]);
    k.abbS[f] = (float)(2.0 * w1 * p.beta * p.bc_S[f]);
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
  float *bufs[] = {c->fbuf[0], c->fbuf[1], c->gbuf[0], c->gbuf[1], c->K, c->phi, c->Fp, c->Fs,
                   c->S, c->itau, c->Psnap, c->scratch};
  for (float *b : bufs)
    if (b) (void)hipFree(b);
  if (c->partials) (void)hipFree(c->partials);
  if (c->ctl) (void)hipFree(c->ctl);
  if (c->ctl_host) (void)hipHostFree(c->ctl_host);
  if (c->ctl_ring) (void)hipHostFree(c->ctl_ring);
  for (int i = 0; i < 2; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  delete c;
}

int lbtp_init(const lbtp_params *p, lbtp_ctx **out) {
  if (!out) return LBTP_EINVAL;
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  lbtp_ctx *c = new lbtp_ctx();
  c->p = *p;
  c->dim = p->lattice == LBTP_D2Q5 ? 2 : 3;
  c->Q = 2 * c->dim + 1;
  c->nf = 2 * c->dim;
  c->ncell = (long long)p->nx * p->ny * p->nz;
  c->stream = (hipStream_t)p->stream;
  c->nblk = nblocks(c->ncell);
  fill_kc(c);
  const size_t n = (size_t)c->ncell;
  struct {
    float **ptr;
    size_t count;
  } allocs[] = {{&c->fbuf[0], n * c->nf}, {&c->fbuf[1], n * c->nf}, {&c->gbuf[0], n * c->Q},
                {&c->gbuf[1], n * c->Q},  {&c->K, n},               {&c->phi, n},
                {&c->Fp, n},              {&c->Fs, n},              {&c->S, n},
                {&c->itau, n},            {&c->Psnap, n},           {&c->scratch, n * 3}};
  for (auto &a : allocs) {
    if (hipMalloc((void **)a.ptr, a.count * sizeof(float)) != hipSuccess) {
      lbtp_destroy(c);
      return LBTP_ENOMEM;
    }
  }
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
  double phimin = INFINITY;
  for (long long i = 0; i < c->ncell; ++i) {
    if (!(hK[i] > 0.0f) || !isfinite(hK[i])) return LBTP_EINVAL;
    if (!(hphi[i] > 0.0f) || !isfinite(hphi[i])) return LBTP_EINVAL;
    phimin = fmin(phimin, (double)hphi[i]);
  }
  // eq. 3-4b: 0 <= beta <= phi / (1 - w0) keeps every g^eq non-negative
  if (c->p.beta > phimin / (1.0 - weight_rest(c->p.lattice)) * (1.0 + 1e-12)) return LBTP_EINVAL;
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

int lbtp_set_state(lbtp_ctx *c, const float *P0, const float *S0, const float *dP0, const float *dS0,
                   int on_device) {
  if (!c || !P0 || !S0) return LBTP_EINVAL;
  if (!c->have_fields) return LBTP_ESTATE;
  const size_t n = (size_t)c->ncell;
  // stage P0 in Psnap, S0 in S, gradients in scratch (dP0) and the second f buffer (dS0)
  int rc = upload(c, c->Psnap, P0, n, on_device);
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
    rc = upload(c, c->fbuf[1], dS0, n * c->dim, on_device);
    if (rc) return rc;
    dS = c->fbuf[1];
  }
  HIP_TRY(launch_init(c->dim, c->kc, c->Psnap, c->S, dP, dS, c->K, c->phi, Fs_or_null(c), c->p.init_neq,
                      fptrs(c, c->fbuf[0]), gptrs(c, c->gbuf[0]), c->stream));
  c->fs = 0;
  c->gs = 0;
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
  HIP_TRY(launch_moments(c->dim, c->kc, gptrs(c, c->gbuf[c->gs]), c->K, c->phi, Fs_or_null(c), c->S, c->itau,
                         c->partials, 1, c->stream));
  HIP_TRY(launch_finish_sum(c->partials, c->nblk, &c->ctl->mass, 0, nullptr, c->stream));
  c->have_coef = 1;
  return LBTP_OK;
}

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
  auto sweep = [&](long long k) -> hipError_t {
    const int parity = (int)((c->fs + k) & 1);
    const int snap = !checks ? 0 : (k % m != 0 ? 0 : (k == 0 ? 1 : 2));
    const int local = (k == 0) && c->f_local;
    hipError_t e = launch_f_sweep(c->dim, c->kc, fptrs(c, c->fbuf[parity]), fptrs(c, c->fbuf[parity ^ 1]),
                                  c->itau, Fp_or_null(c), c->Psnap, c->partials, c->ctl, k, local, snap, c->stream);
    if (e == hipSuccess && snap == 2)
      e = launch_finish_residual(c->partials, sweep_blocks(c->ncell), c->ctl, k, m, c->stream);
    return e;
  };
  // Chunk 0 is sweep 0 (snapshot of P^0); chunk j >= 1 is sweeps
  // (j-1)m+1 .. jm and ends with the check at jm.  The first check is waited
  // for at once (warm steps usually stop there); later ones are read one
  // chunk behind so the GPU never idles while the host decides.
  long long k = 0;
  if (last >= 0) {
    HIP_TRY(sweep(0));
    k = 1;
  }
  int slot = 0;
  bool pending[2] = {false, false};
  for (long long j = 1; k <= last; ++j) {
    const long long kend = (j * m < last) ? j * m : last;
    for (; k <= kend; ++k) HIP_TRY(sweep(k));
    if (!checks || k > last) continue;
    HIP_TRY(hipMemcpyAsync(&c->ctl_ring[slot], c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipEventRecord(c->ev[slot], c->stream));
    pending[slot] = true;
    const int prev = slot ^ 1;
    int wait = -1;
    if (j == 1) wait = slot;
    else if (pending[prev]) wait = prev;
    bool stop = false;
    if (wait >= 0) {
      HIP_TRY(hipEventSynchronize(c->ev[wait]));
      pending[wait] = false;
      stop = c->ctl_ring[wait].done != 0;
    }
    slot = prev;
    if (stop) break;
  }
  int rc = read_ctl(c);
  if (rc) return rc;
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
    c->fs = (int)((c->fs + K) & 1);
    c->f_local = 0;
  }
  if (iters) *iters = K;
  if (resid) *resid = h.resid;
  if (!checks && status == LBTP_OK && max_iters > 0) status = LBTP_NOT_CONVERGED;
  return status;
}

int lbtp_saturation_step(lbtp_ctx *c) {
  if (!c) return LBTP_EINVAL;
  if (!c->have_coef) return LBTP_ESTATE;
  HIP_TRY(launch_g_sweep(c->dim, c->kc, gptrs(c, c->gbuf[c->gs]), gptrs(c, c->gbuf[c->gs ^ 1]),
                         fptrs(c, c->fbuf[c->fs]), c->f_local, c->itau, c->K, c->phi, Fs_or_null(c), c->partials,
                         c->stream));
  HIP_TRY(launch_finish_sum(c->partials, c->nblk, &c->ctl->ledger, 1, &c->ctl->last_flux, c->stream));
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
  HIP_TRY(launch_pressure(c->dim, c->kc, fptrs(c, c->fbuf[c->fs]), c->f_local, c->scratch, c->stream));
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
  HIP_TRY(launch_grad(c->dim, c->kc, fptrs(c, c->fbuf[c->fs]), c->f_local, c->itau, c->K, c->S, velocity,
                      c->scratch, c->stream));
  return download(c, out, c->scratch, (size_t)c->ncell * c->dim, on_device);
}

int lbtp_velocity(lbtp_ctx *c, float *u, int on_device) { return grad_common(c, u, on_device, 1); }
int lbtp_grad_p(lbtp_ctx *c, float *g, int on_device) { return grad_common(c, g, on_device, 0); }

int lbtp_saturation(lbtp_ctx *c, float *S, int on_device) {
  if (!c || !S) return LBTP_EINVAL;
  if (!c->have_state) return LBTP_ESTATE;
  HIP_TRY(launch_saturation(c->dim, c->kc, gptrs(c, c->gbuf[c->gs]), c->phi, Fs_or_null(c), c->scratch,
                            c->stream));
  return download(c, S, c->scratch, c->ncell, on_device);
}

int lbtp_mass(lbtp_ctx *c, double *mass, double *ledger) {
  if (!c) return LBTP_EINVAL;
  if (!c->have_state) return LBTP_ESTATE;
  HIP_TRY(launch_moments(c->dim, c->kc, gptrs(c, c->gbuf[c->gs]), c->K, c->phi, Fs_or_null(c), nullptr, nullptr,
                         c->partials, 0, c->stream));
  HIP_TRY(launch_finish_sum(c->partials, c->nblk, &c->ctl->mass, 0, nullptr, c->stream));
  int rc = read_ctl(c);
  if (rc) return rc;
  if (mass) *mass = c->ctl_host->mass;
  if (ledger) *ledger = c->ctl_host->ledger;
  if (!isfinite(c->ctl_host->mass)) return LBTP_EUNSTABLE;
  return LBTP_OK;
}

int lbtp_get_state(lbtp_ctx *c, float *f, float *g, long long *step, int on_device) {
  if (!c) return LBTP_EINVAL;
  if (!c->have_state) return LBTP_ESTATE;
  const size_t n = (size_t)c->ncell;
  if (f) {
    // materialise the pre-collision f into the other buffer's space is not
    // allowed (it may be needed); use the caller buffer directly when it is
    // on the device, else a staging copy through scratch one population at a time
    if (on_device) {
      HIP_TRY(launch_materialize_f(c->dim, c->kc, fptrs(c, c->fbuf[c->fs]), c->f_local, fptrs(c, f), c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
    } else {
      float *tmp = nullptr;
      if (hipMalloc((void **)&tmp, n * c->nf * sizeof(float)) != hipSuccess) return LBTP_ENOMEM;
      hipError_t e = launch_materialize_f(c->dim, c->kc, fptrs(c, c->fbuf[c->fs]), c->f_local, fptrs(c, tmp), c->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(f, tmp, n * c->nf * sizeof(float), hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      (void)hipFree(tmp);
      if (e != hipSuccess) return LBTP_EHIP;
    }
  }
  if (g) {
    int rc = download(c, g, c->gbuf[c->gs], n * c->Q, on_device);
    if (rc) return rc;
  }
  if (step) *step = c->step;
  return LBTP_OK;
}

int lbtp_put_state(lbtp_ctx *c, const float *f, const float *g, long long step, int on_device) {
  if (!c || !f || !g) return LBTP_EINVAL;
  if (!c->have_fields) return LBTP_ESTATE;
  const size_t n = (size_t)c->ncell;
  int rc = upload(c, c->fbuf[0], f, n * c->nf, on_device);
  if (rc) return rc;
  rc = upload(c, c->gbuf[0], g, n * c->Q, on_device);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->fs = 0;
  c->gs = 0;
  c->f_local = 1;
  c->step = step;
  c->have_state = 1;
  c->have_coef = 0;
  return LBTP_OK;
}

}  // extern "C"
