// Internal declarations shared by the kernels and the host side of liblbtp.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbtp.h"

namespace lbtp {

// Stored moving directions j = 0..2*DIM-1 (population i = j + 1):
//   0:+x 1:+y 2:-x 3:-y 4:+z 5:-z
// axis, sign and opposite of each.
__host__ __device__ constexpr int dir_axis(int j) { return (j == 0 || j == 2) ? 0 : (j == 1 || j == 3) ? 1 : 2; }
__host__ __device__ constexpr int dir_sign(int j) { return (j == 0 || j == 1 || j == 4) ? 1 : -1; }
__host__ __device__ constexpr int dir_opp(int j) { return j == 0 ? 2 : j == 1 ? 3 : j == 2 ? 0 : j == 3 ? 1 : j == 4 ? 5 : 4; }

constexpr int kThreads = 256;       // threads per block of every cell kernel

// Lattice constants and boundary data passed by value to every cell kernel.
struct KC {
  int nx, ny, nz;
  int ncell;
  float c;          // dx / dt
  float dt;
  float cs2;        // c_s^2
  float w0, w1;     // rest and moving weights (D2Q9: w1 of the axis directions)
  float w2;         // D2Q9: weight of the diagonal directions
  float inv_1mw0;   // 1 / (1 - w0)
  float w1_1mw0;    // w1 / (1 - w0): w1 (P - P_b) from the sum of the deviations
  float wbar;       // source weight of a moving direction (eq. 3-5a pattern)
  float beta;
  float inv_tau_g;  // 1 / tau_g
  float src_g;      // dt (1 - 1/(2 tau_g)): weight of F_s in eq. 3-2
  float inv_mu_w, inv_mu_n;
  float inv_cs2dt;  // 1 / (c_s^2 dt)
  float geq0_phi;   // (w0 - 1) beta: g_0^eq = (geq0_phi + phi) S
  float w1beta;     // w1 beta: g_i^eq = w1 beta S
  float half_dt;    // dt / 2
  float dev_scale;      // storage scale of 16-bit float deviations (a power of two)
  float inv_dev_scale;  // its inverse
  float g_scale, inv_g_scale;   // the same for the saturation deviations
  int bc_f[6];
  float Pw[6];      // Dirichlet pressure of a face
  int bc_g[6];
  float abbS[6];    // 2 w1 beta S_b of a Dirichlet saturation face
  float Sw[6];      // Dirichlet saturation of a face
  int coef;         // lbtp_coef_model
  float cf[6];      // RATIONAL: a0, a1, c0, c1, b0, b1
  // Dirichlet data per link of a face (lbtp_set_wall_values), or null for
  // the face constants above
  const float *wP[6];
  const float *wS[6];
  // D2Q9: condition per link of a face (lbtp_set_wall_types; three per face
  // node, the layout of the wall data), or null where the face condition
  // above holds for every link
  const int *wtF[4];
  const int *wtG[4];
  // pressure-lattice collision: 0 BGK, 1 MRT (D2Q9) with rates s0 (rho, e,
  // epsilon), sq (energy fluxes), sp (stresses); the fluxes relax at 1/tau_f
  int mrt;
  float ms0, msq, msp;
  // saturation diffusivity D_s(x) = Ds + cap_B K lambda_n f_w (eq. 2-16 with
  // the capillary curve P_c = cap_B (1 - S)); itg holds 1/tau_g per node
  // when cap_B > 0 (written with the coefficients), else null
  float Ds, cap_B, inv_bcs2dt;   // inv_bcs2dt = 1 / (beta c_s^2 dt)
  float *itg;
};

// Device-side control block of a pressure solve and the float64 reductions.
struct Ctl {
  int done;          // set once the solve has stopped (converged or unstable)
  int status;        // LBTP_OK or LBTP_EUNSTABLE when done
  long long K;       // iteration at which it stopped
  long long kmax;    // sweeps with index > kmax do nothing
  double tol;
  double resid;      // last evaluated residual
  long long last_check;
  double mass;       // last mass reduction
  double ledger;     // accumulated boundary-link flux of g
  double last_flux;  // flux of the last saturation step
  long long kcheck;  // iteration of the last stopping-rule check (advanced by m per check)
};

// ----------------------------------------------------------------- launchers
// Each returns the hipError_t of the launch.  Pointer arrays hold one base
// pointer per stored population.
struct FPtrs { void *p[8]; };
// Saturation populations: Q arrays of the storage type.  With 16-bit
// storage they hold deviations e_i = g_i - g_i^eq(B) from the equilibrium
// (eq. 3-4b, or eq. 3-4 on D2Q9) of a per-node base saturation B, the
// saturation the buffer was written against; B is null for float32 storage,
// where the arrays hold g_i itself.
struct GPtrs {
  void *p[9];
  float *B;
  int storage;   // lbtp_storage of the arrays
};

// Lattice kind passed to the launchers: 2 = D2Q5, 3 = D3Q7 (the spatial
// dimension of those), kD2Q9 = D2Q9.
constexpr int kD2Q9 = 9;

// One pressure sweep per launch; mode as f_sweep_kernel's (3, the probe
// that only evaluates the stopping-rule sums, on D2Q5 and D3Q7).
hipError_t launch_f_sweep(int dim, int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb_in,
                          float *Pb_out, const float *itau, const float *Fp, double *partials, const Ctl *ctl,
                          long long k, int local, int mode, hipStream_t s);
// H consecutive plain pressure sweeps (no re-basing, no stopping-rule terms)
// in one launch, sweeps k .. k + H - 1 (temporal blocking: the region in
// registers on D2Q5 and D2Q9, streaming along z on D3Q7; H odd); fin holds
// the state before sweep k, fout receives it after.  dim is the lattice kind
// (2, 3 or kD2Q9).
int block_sweeps_supported(int dim, const KC &kc, int H);
hipError_t launch_f_block(int dim, int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb,
                          const float *itau, const float *Fp, const Ctl *ctl, long long k, int H, hipStream_t s);
// The same on D2Q5 with the first sweep, k, re-basing (as f_sweep_kernel's
// mode 1: a chunk's first sweep): the launch reads bases Pb and writes the
// new ones to Pb_out (another buffer).
int block_first_supported(int dim, const KC &kc, int H);
hipError_t launch_f_block_first(int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, float *Pb_out,
                                const float *itau, const float *Fp, const Ctl *ctl, long long k, int H,
                                hipStream_t s);
// Compute units of the current device (queried once per device).
int device_cus();
int block_sweeps_supported_q9(int H);
int block_sweeps_supported_3d(int H);
hipError_t launch_f_block_3d(int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, const float *itau,
                             const float *Fp, const Ctl *ctl, long long k, int H, hipStream_t s);
hipError_t launch_f_block_q9(int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb, const float *itau,
                             const float *Fp, const Ctl *ctl, long long k, int H, hipStream_t s);
// Check of the stopping rule at iteration ctl->kcheck + m (device-side
// count, so a captured chunk serves every position in the solve).
hipError_t launch_finish_residual(const double *partials, int nblk, Ctl *ctl, int m, hipStream_t s);
hipError_t launch_ctl_reset(Ctl *ctl, long long kmax, double tol, hipStream_t s);
hipError_t launch_moments(int dim, const KC &kc, GPtrs g, const float *K, const float *phi,
                          const float *Fs, float *S, float *itau, double *partials, int write_coef,
                          hipStream_t s);
hipError_t launch_finish_sum(const double *partials, int nblk, double *dst, int accumulate,
                             double *copy_to, hipStream_t s);
hipError_t launch_g_sweep(int dim, int storage, const KC &kc, GPtrs gin, GPtrs gout, FPtrs f, int f_local,
                          const float *Pb, const float *itau, const float *K, const float *phi,
                          const float *Fs, const float *Sn, double *partials, hipStream_t s);
hipError_t launch_init(int dim, int storage, const KC &kc, const float *P0, const float *S0, const float *dP0,
                       const float *dS0, const float *K, const float *phi, const float *Fs, int neq, FPtrs f,
                       float *Pb, GPtrs g, hipStream_t s);
hipError_t launch_pressure(int dim, int storage, const KC &kc, FPtrs f, int f_local, const float *Pb, float *P,
                           hipStream_t s);
hipError_t launch_grad(int dim, int storage, const KC &kc, FPtrs f, int f_local, const float *Pb,
                       const float *itau, const float *K, const float *S, int velocity, float *out,
                       hipStream_t s);
hipError_t launch_saturation(int dim, const KC &kc, GPtrs g, const float *phi, const float *Fs,
                             float *S, hipStream_t s);
// The saturation populations as float32 (Q x ncell, component-major).
hipError_t launch_g_populations(int dim, const KC &kc, GPtrs g, const float *phi, float *out, hipStream_t s);
hipError_t launch_g_populations_q9(const KC &kc, GPtrs g, const float *phi, float *out, hipStream_t s);
hipError_t launch_populations(int dim, int storage, const KC &kc, FPtrs f, int f_local, const float *Pb,
                              float *out, hipStream_t s);

hipError_t launch_copy_probe(const void *src, void *dst, long long n4, hipStream_t s);
// dim = spatial dimension (any lattice); u: dim x ncell total velocity
hipError_t launch_phase(int dim, const KC &kc, const float *u, const float *S, const float *K, float Ds, float *uw,
                        float *un, hipStream_t s);

// D2Q9 (lbtp_d2q9.hip): the same operations, one node per thread.
hipError_t launch_f_sweep_q9(int storage, const KC &kc, FPtrs fin, FPtrs fout, const float *Pb_in, float *Pb_out,
                             const float *itau, const float *Fp, double *partials, const Ctl *ctl, long long k,
                             int local, int mode, hipStream_t s);
hipError_t launch_moments_q9(const KC &kc, GPtrs g, const float *K, const float *phi, const float *Fs, float *S,
                             float *itau, double *partials, int write_coef, hipStream_t s);
hipError_t launch_g_sweep_q9(int storage, const KC &kc, GPtrs gin, GPtrs gout, FPtrs f, int f_local,
                             const float *Pb, const float *itau, const float *K, const float *phi, const float *Fs,
                             const float *Sn, double *partials, hipStream_t s);
hipError_t launch_init_q9(int storage, const KC &kc, const float *P0, const float *S0, const float *dP0,
                          const float *dS0, const float *K, const float *phi, const float *Fs, int neq, FPtrs f,
                          float *Pb, GPtrs g, hipStream_t s);
hipError_t launch_pressure_q9(int storage, const KC &kc, FPtrs f, int f_local, const float *Pb, float *P,
                              hipStream_t s);
hipError_t launch_grad_q9(int storage, const KC &kc, FPtrs f, int f_local, const float *Pb, const float *itau,
                          const float *K, const float *S, int velocity, float *out, hipStream_t s);
hipError_t launch_saturation_q9(const KC &kc, GPtrs g, const float *phi, const float *Fs, float *S, hipStream_t s);
hipError_t launch_populations_q9(int storage, const KC &kc, FPtrs f, int f_local, const float *Pb, float *out,
                                 hipStream_t s);

inline size_t storage_bytes(int storage) { return storage == LBTP_FP32 ? 4 : 2; }

// ------------------------------------------------------------------ ensembles
// One member of an ensemble: its lattice constants and device buffers, and
// its tile ranges in the sweep tiling (4*NT nodes per tile) and the cell
// tiling (1024 nodes per tile).
struct Member {
  KC kc;
  FPtrs f[2];
  GPtrs g[2];
  float *Pb[2];
  float *K, *phi, *S, *itau, *Fp, *Fs;
  int tstart_s, ntiles_s, tstart_c, ntiles_c;
};

// Device control block of one member's pressure solve and reductions.
struct BCtl {
  int done;          // the member's current solve has stopped
  int status;        // LBTP_OK, LBTP_NOT_CONVERGED or LBTP_EUNSTABLE
  int pb;            // base buffer of the member's pressure state
  int pad;
  long long kbase;   // iteration index before the current chunk
  long long kmax;
  long long K;       // iterations of the last solve
  double tol;
  double resid;
  double mass;
  double ledger;
};

constexpr int kCellTile = 1024;   // nodes per tile of the ensemble cell kernels

// Plain sweeps j .. j + H - 1 of every member through the blocked tiling
// (tables tm / ti of (member, tile)), members with a pressure source or without.
hipError_t batch_launch_block(int storage, int shape, bool has_fp, int nblk, const Member *mem, const BCtl *ctl,
                              const int *tm, const int *ti, int j, int H, hipStream_t s);
hipError_t batch_launch_sweep(int nt, int dim, int storage, int mode, int local, int nblk, const Member *mem,
                              const BCtl *ctl, const int *tm, const int *ti, double *part, int j, hipStream_t s);
hipError_t batch_launch_moments(int dim, int storage, int nblk, const Member *mem, const int *tm, const int *ti, double *part,
                                int gs, int write_coef, hipStream_t s);
hipError_t batch_launch_gsweep(int dim, int storage, int local, int nblk, const Member *mem, const BCtl *ctl,
                               const int *tm, const int *ti, double *part, int gs, hipStream_t s);
hipError_t batch_launch_finish(int n, const Member *mem, BCtl *ctl, const double *part, int m, int *active,
                               hipStream_t s);
hipError_t batch_launch_reset(int n, BCtl *ctl, long long kmax, double tol, int *active, hipStream_t s);
hipError_t batch_launch_flip(int n, BCtl *ctl, hipStream_t s);
hipError_t batch_launch_sum(int n, const Member *mem, BCtl *ctl, const double *part, int ledger, hipStream_t s);

inline int nblocks(long long n);

// Blocks of a pull-form pressure sweep (and so its residual partials): rows
// with nx % 4 == 0 run four nodes per thread.
inline int sweep_blocks(const KC &kc, int local) {
  return (!local && kc.nx % 4 == 0) ? nblocks(kc.ncell / 4) : nblocks(kc.ncell);
}

inline int nblocks(long long n) { return (int)((n + kThreads - 1) / kThreads); }
// Whether the saturation step of a context runs four nodes per thread (D2Q5,
// the pressure lattice in pull form, nx % 4 == 0), and its blocks (partials).
inline bool g_sweep_quads(int lk, const KC &kc, int local) { return lk == 2 && !local && kc.nx % 4 == 0 && kc.nz == 1; }
inline int g_sweep_blocks(int lk, const KC &kc, int local) {
  return g_sweep_quads(lk, kc, local) ? nblocks(kc.ncell / 4) : nblocks(kc.ncell);
}

}  // namespace lbtp
