/*
 * lbtp.h -- C ABI of an MI355X (gfx950) implementation of the
 * double-distribution lattice Boltzmann model for two-phase flow in porous
 * media of Chai, Liang, Du and Shi (arXiv:1808.07554).
 *
 * Problem solved (Section 2): the global-pressure Poisson equation
 *     div(D_p grad P) + F_p = 0,                  D_p = K lambda_t   (eq. 2-15, 2-16)
 * and the saturation equation with convection written as a source
 *     phi dS/dt = div(D_s grad S) + F_s + div(lambda_w K grad P)   (eq. 2-18)
 * with lambda_a = k_ra / mu_a (eq. 2-9), k_rw = S^2, k_rn = (1-S)^2
 * (Section 4.3), on a box of nx x ny (x nz) nodes.
 *
 * Method (Section 3): a pressure lattice f_i iterated in pseudo time to a
 * steady state (eq. 3-1, 3-3) and a saturation lattice g_i advanced in
 * physical time (eq. 3-2), on D2Q5 or D3Q7 (equilibrium eq. 3-4b, Remark V)
 * or on the paper's D2Q9 (eq. 3-4, 3-5, 3-6).  The pressure
 * gradient and velocity come from the local first moment of f (eq. 3-10);
 * the relaxation times follow from D_p and D_s (eq. 3-11).  Dirichlet
 * boundaries use anti-bounce-back, no-flux boundaries bounce-back
 * (Section 4).
 *
 * Conventions
 *   - Lattice units of the caller: dx, dt given; c = dx/dt; c_s^2 = c^2/3
 *     (D2Q5, D2Q9) or c^2/4 (D3Q7).  Weights: D2Q5 1/3, 1/6; D3Q7 1/4, 1/8;
 *     D2Q9 4/9, 1/9 (axes), 1/36 (diagonals) (eq. 3-5).
 *   - Scalar fields are float32 arrays of nx*ny*nz values, x fastest:
 *     index = x + nx*(y + ny*z).  Vector fields are component-major:
 *     component a of cell c at a*ncell + c.
 *   - Population order: i = 0 rest, then +x, +y, -x, -y (D2Q5), followed by
 *     +z, -z (D3Q7) or by the diagonals (1,1), (-1,1), (-1,-1), (1,-1)
 *     (D2Q9, eq. 3-6).  On D2Q9 a diagonal link that crosses an x and a y face
 *     at a corner takes the y face's rule.  The rest population of the pressure lattice never
 *     influences any output (P sums i >= 1, eq. 3-9a; c_0 = 0 in eq. 3-10;
 *     bar-omega_0 = 0; walls act on moving populations only), so it is not
 *     stored; f arrays hold Q-1 populations, g arrays hold Q.
 *   - on_device: 1 if a pointer is device memory of the current HIP device
 *     (e.g. a torch tensor's data_ptr), 0 if it is host memory.
 *   - Ownership: the context owns all device memory it allocates.  Caller
 *     pointers are only read or written during the call; none is retained.
 *   - Streams: every device operation is enqueued on params.stream (a
 *     hipStream_t; NULL = the null stream).  Calls that return host values
 *     synchronise that stream.  A context is not thread-safe; use one per
 *     stream.
 *   - Return codes: 0 ok; > 0 warning; < 0 error (see lbtp_status).  On an
 *     error no device state has been changed unless stated.
 */
#ifndef LBTP_H
#define LBTP_H

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define LBTP_API __attribute__((visibility("default")))
#else
#define LBTP_API
#endif

typedef struct lbtp_ctx lbtp_ctx;

/* D2Q9 plain pressure sweeps run blocked (several per launch) or four nodes per thread. */
enum lbtp_lattice { LBTP_D2Q5 = 0, LBTP_D3Q7 = 1, LBTP_D2Q9 = 2 };

/* Storage of the populations of both lattices.  The pressure lattice stores
 * the deviation of f_i from a per-node base equilibrium, f_i - w_i P_b, where
 * P_b is the pressure at the start of the solve or at the last residual
 * check: FP32 as float, FP16_DEV as (power-of-two scaled) fp16, BF16_DEV as
 * bf16.  The saturation lattice stores g_i itself as float under FP32, and
 * under FP16_DEV / BF16_DEV the deviation g_i - g_i^eq(S_b) (eq. 3-4b) from
 * the equilibrium of a per-node base saturation S_b, the saturation of the
 * step that wrote it, in the same 16-bit format.  Collision arithmetic is
 * float32 in every form, and the residual / mass reductions are float64. */
enum lbtp_storage { LBTP_FP32 = 0, LBTP_FP16_DEV = 1, LBTP_BF16_DEV = 2 };

/* Boundary condition of one face (faces ordered -x, +x, -y, +y, -z, +z).
 * DIRICHLET: anti-bounce-back with the face value (Section 4).
 * NOFLUX:    bounce-back (Section 4).
 * OUTFLOW:   saturation lattice only: anti-bounce-back with S_wb equal to the
 *            current saturation of the boundary node (zero-gradient outlet).
 * PERIODIC must be set on both faces of an axis, for f and for g. */
enum lbtp_bc { LBTP_BC_PERIODIC = 0, LBTP_BC_DIRICHLET = 1, LBTP_BC_NOFLUX = 2, LBTP_BC_OUTFLOW = 3 };

/* Coefficient model.  QUADRATIC_KR: lambda_a = k_ra/mu_a with k_rw = S^2,
 * k_rn = (1-S)^2 (eq. 2-9, Section 4.3), D_p = K lambda_t (eq. 2-16),
 * lambda_w K.  RATIONAL: D_p and lambda_w K given directly, as Sections 4.1
 * and 4.2 do:  D_p = K (a0 + a1 S) / (b0 + b1 S),
 * lambda_w K = K (c0 + c1 S) / (b0 + b1 S), coef = {a0, a1, c0, c1, b0, b1}
 * (Section 4.1: a0 = c0 = 1e-3, b0 = 1, others 0, K = 1; Section 4.2:
 * a0 = 1, c1 = 1, b0 = 0.5, b1 = -0.2, others 0, K = 1).  The velocity is
 * u = -D_p grad P in both. */
enum lbtp_coef_model { LBTP_COEF_QUADRATIC_KR = 0, LBTP_COEF_RATIONAL = 1 };

/* Collision of the pressure lattice.  BGK: eq. 3-1 as the paper states it.
 * MRT (D2Q9 only): the multiple-relaxation-time form the paper says the
 * model extends to (Section 3), f^+ = f - M^-1 S M (f - f^eq) with the
 * orthogonal D2Q9 moment basis of Lallemand and Luo (rows rho, e, epsilon,
 * j_x, q_x, j_y, q_y, p_xx, p_xy), the fluxes j relaxed at 1/tau_f (eq. 3-11a,
 * which keeps D_p) and the other rates from params.mrt_rates = {s0 (rho, e and
 * epsilon, one rate so the rest population stays decoupled), s_q, s_p}, each
 * in (0, 2).  The saturation lattice keeps BGK. */
enum lbtp_collision { LBTP_COLLISION_BGK = 0, LBTP_COLLISION_MRT = 1 };

enum lbtp_status {
  LBTP_OK = 0,
  LBTP_NOT_CONVERGED = 1,   /* max_iters reached before the residual met tol */
  LBTP_EINVAL = -1,         /* invalid argument or parameter; nothing done */
  LBTP_ENOMEM = -2,         /* device allocation failed */
  LBTP_EHIP = -3,           /* a HIP runtime call failed */
  LBTP_EUNSTABLE = -4,      /* non-finite residual or mass */
  LBTP_ESTATE = -5          /* call out of order (e.g. step before set_state) */
};

typedef struct lbtp_params {
  int lattice;                 /* lbtp_lattice */
  int nx, ny, nz;              /* nodes per axis; nz = 1 for D2Q5 and D2Q9 */
  double dx, dt;               /* lattice spacing and time step */
  double beta;                 /* equilibrium parameter: 0 <= beta <= min(phi)/(1-w_0) (eq. 3-4b), or
                                  max(phi)/2 <= beta <= 2 min(phi) on D2Q9 (eq. 3-4) */
  double Ds;                   /* saturation diffusivity; tau_g = 1/2 + Ds/(beta c_s^2 dt) (eq. 3-11b) */
  double mu_w, mu_n;           /* phase viscosities (eq. 2-9) */
  int storage;                 /* lbtp_storage */
  int residual_stride;         /* m >= 1: the stopping rule compares P^k with P^(k-m) */
  int bc_f[6];                 /* pressure-lattice face conditions (PERIODIC, DIRICHLET, NOFLUX) */
  double bc_P[6];              /* Dirichlet pressure per face */
  int bc_g[6];                 /* saturation-lattice face conditions (any lbtp_bc) */
  double bc_S[6];              /* Dirichlet saturation per face */
  int init_neq;                /* 1: lbtp_set_state adds the first-order non-equilibrium parts */
  void *stream;                /* hipStream_t for all device work; NULL = null stream */
  int coef_model;              /* lbtp_coef_model */
  double coef[6];              /* RATIONAL: a0, a1, c0, c1, b0, b1 (unused otherwise) */
  double cap_B;                /* >= 0: capillary curve P_c = cap_B (1 - S), which adds
                                  cap_B K lambda_n f_w to Ds (eq. 2-16), so D_s and tau_g
                                  vary with S and K from node to node; 0 = constant Ds. */
  int sweep_block;             /* plain pressure sweeps fused into one launch inside the
                                  captured chunks of m sweeps (temporal blocking: the region
                                  in registers on D2Q5 and D2Q9, streaming along z on D3Q7;
                                  float32 results bitwise unchanged; 16-bit storage rounds
                                  once per launch): 0 = library default (9 on D2Q5 and D2Q9,
                                  3 on D3Q7), 1 = one sweep per launch, or an odd number
                                  3..23 (D3Q7: 3); LBTP_EINVAL otherwise */
  int collision;               /* lbtp_collision of the pressure lattice */
  double mrt_rates[3];         /* MRT: s0, s_q, s_p (unused for BGK) */
} lbtp_params;

/* Fill *p with defaults: D2Q5, 1x1x1, dx = dt = 1, beta = 1, Ds = 0, mu = 1,
 * FP32, m = 64, periodic faces, init_neq = 1, null stream, QUADRATIC_KR,
 * sweep_block = 0, BGK collision. */
LBTP_API void lbtp_default_params(lbtp_params *p);

/* Validate *p (tau_g > 1/2, beta >= 0, periodicity consistent, sizes > 0,
 * at least three nodes along every walled axis -- the one-sided differences
 * of the initial gradients need them; a periodic axis may have any length --
 * storage/lattice known) and allocate all device buffers of a context.
 * Returns LBTP_EINVAL, LBTP_ENOMEM or LBTP_EHIP on failure (*out = NULL). */
LBTP_API int lbtp_init(const lbtp_params *p, lbtp_ctx **out);

/* Release every device buffer of ctx; ctx may be NULL. */
LBTP_API void lbtp_destroy(lbtp_ctx *ctx);

/* Follow another stream from now on (hipStream_t, NULL = null stream). */
LBTP_API int lbtp_set_stream(lbtp_ctx *ctx, void *stream);

/* The medium and the sources of eq. 2-15/2-18 (Section 2): absolute
 * permeability K > 0, porosity phi > 0, F_p = q_w/rho_w + q_n/rho_n and
 * F_s = q_w/rho_w (eq. 2-17).  Fp / Fs may be NULL for zero.  Fails with
 * LBTP_EINVAL if K or phi is not positive and finite, if beta violates the
 * non-negativity bound of eq. 3-4b for the smallest phi, or if a fully
 * periodic pressure problem has sum(F_p) != 0 (no solution). */
LBTP_API int lbtp_set_fields(lbtp_ctx *ctx, const float *K, const float *phi,
                    const float *Fp, const float *Fs, int on_device);

/* Replace F_p and F_s only (time-dependent sources); NULL = zero. */
LBTP_API int lbtp_set_sources(lbtp_ctx *ctx, const float *Fp, const float *Fs, int on_device);

/* Dirichlet data that vary along a face (and in time: call again before the
 * solve or step they apply to), for the anti-bounce-back rules of Section 4:
 * P (pressure lattice) and / or S (saturation lattice) at the midpoint of
 * every link that crosses the face, x_node - c_i dt / 2 for the population
 * i arriving at the boundary node.  Layout: face nodes in the order
 * y + ny z (faces -x, +x), x + nx z (-y, +y), x + nx y (-z, +z), and per
 * node L values, L = 1 on D2Q5 / D3Q7 (the normal link) and L = 3 on D2Q9:
 * the normal link, then the diagonal links whose arriving population has
 * tangential velocity -1 and +1 (at a corner the diagonal link crossing
 * both faces takes the value of the y face).  NULL keeps the current data
 * of that lattice; the face constants of params apply until data are set.
 * The face's condition must be DIRICHLET for the lattice whose data are
 * given, or the face must carry per-link conditions in that lattice
 * (lbtp_set_wall_types); LBTP_EINVAL otherwise. */
LBTP_API int lbtp_set_wall_values(lbtp_ctx *ctx, int face, const float *P, const float *S, int on_device);

/* D2Q9 only: a condition per link of a face, so that one wall can hold
 * Dirichlet segments (wells) between no-flux stretches, as the five-spot
 * problem of Section 4.3 needs.  f_types (pressure lattice: DIRICHLET or
 * NOFLUX) and g_types (saturation lattice: DIRICHLET, NOFLUX or OUTFLOW)
 * hold one lbtp_bc value per link in the layout of lbtp_set_wall_values
 * (three per face node: normal link, then the diagonals with tangential
 * velocity -1 and +1; at a corner the y face decides a link that crosses
 * both faces).  A DIRICHLET link takes the per-link data of
 * lbtp_set_wall_values if set, else the face constant of params.  NULL
 * keeps that lattice's current list; until a list is set the face condition
 * holds for every link.  The face must not be periodic in that lattice.
 * LBTP_EINVAL for another lattice, a bad face or an unknown value (nothing
 * is changed then).  Device lists are read back to the host for checking. */
LBTP_API int lbtp_set_wall_types(lbtp_ctx *ctx, int face, const int *f_types, const int *g_types, int on_device);

/* Initial populations (initialisation paragraph of Section 4):
 *   g_i = g_i^eq(S0) + eps g_i^(1) with eps g_i^(1) of eq. (gneq),
 *   f_i = w_i P0 - tau_f dt w_i c_i . grad P0   (i >= 1, Appendix A order 1).
 * dP0 / dS0 are component-major gradient fields (dim x ncell) or NULL, in
 * which case second-order central differences of P0 / S0 are used
 * (one-sided at walls).  With params.init_neq = 0 both are pure equilibria.
 * Resets the step counter and the mass ledger. */
LBTP_API int lbtp_set_state(lbtp_ctx *ctx, const float *P0, const float *S0,
                   const float *dP0, const float *dS0, int on_device);

/* Coefficients of the current coupled step: S^n (eq. 3-9b), D_p and
 * lambda_w K of the coefficient model, 1/tau_f (eq. 3-11a), and the mass
 * M^n = sum phi S^n in float64. */
LBTP_API int lbtp_update_coefficients(lbtp_ctx *ctx);

/* Iterate the pressure lattice (eq. 3-1) with the current coefficients.
 * Stopping rule: r_k = ||P^k - P^(k-m)||_2 / (m ||P^k||_2) (float64 sums),
 * tested when k is a positive multiple of m; stops at the first r_k <= tol
 * or after max_iters iterations (tol < 0: exactly max_iters iterations).
 * *iters receives the iteration count, *resid the last tested r (or -1 if
 * none).  Returns LBTP_OK, LBTP_NOT_CONVERGED or LBTP_EUNSTABLE. */
LBTP_API int lbtp_pressure_solve(lbtp_ctx *ctx, double tol, long long max_iters,
                        long long *iters, double *resid);

/* One step of the saturation lattice (eq. 3-2, 3-4b) with S^n, the local
 * gradient of the current pressure lattice (eq. 3-10a) and the current F_s;
 * accumulates the net boundary-link flux into the mass ledger and advances
 * the step counter. */
LBTP_API int lbtp_saturation_step(lbtp_ctx *ctx);

/* nsteps coupled steps, each = update_coefficients + pressure_solve(tol,
 * max_iters) + saturation_step.  iters (may be NULL) receives nsteps
 * iteration counts.  Stops early with the first error or LBTP_EUNSTABLE;
 * a step that does not converge continues (returns LBTP_NOT_CONVERGED at
 * the end). */
LBTP_API int lbtp_step(lbtp_ctx *ctx, long long nsteps, double tol, long long max_iters,
              long long *iters);

/* Outputs on the current state.  pressure: eq. 3-9a of the pre-collision f.
 * velocity: u = D_p sum_i c_i f_i / (tau_f dt c_s^2) (eq. 3-10b), dim
 * components, with the coefficients of the last update_coefficients.
 * grad_p: eq. 3-10a.  saturation: eq. 3-9b with the current F_s. */
LBTP_API int lbtp_pressure(lbtp_ctx *ctx, float *P, int on_device);
LBTP_API int lbtp_velocity(lbtp_ctx *ctx, float *u, int on_device);
LBTP_API int lbtp_grad_p(lbtp_ctx *ctx, float *gradP, int on_device);
LBTP_API int lbtp_saturation(lbtp_ctx *ctx, float *S, int on_device);

/* Phase velocities of eq. 2-12 / 2-13 (dim x ncell each, component-major)
 * with the coefficients of the last update_coefficients: with the constant
 * D_s of the model, D_s = -K lambda_n f_w dP_c/dS (eq. 2-16), so
 *   u_w = f_w u - D_s grad S,   u_n = f_n u + D_s grad S,
 * f_w = lambda_w K / D_p (eq. 2-10), u of lbtp_velocity and grad S^n by
 * second-order central differences (one-sided at walls).  LBTP_ESTATE before
 * the first update_coefficients. */
LBTP_API int lbtp_phase_velocities(lbtp_ctx *ctx, float *uw, float *un, int on_device);

/* Mass M = sum_x phi S (float64, current g and F_s) and the accumulated net
 * flux of g through Dirichlet/outflow links since lbtp_set_state.  Exactly,
 * M^{n+1} = M^n + dt/2 sum(F_s^n + F_s^{n+1}) + flux_n. */
LBTP_API int lbtp_mass(lbtp_ctx *ctx, double *mass, double *ledger);

/* Pre-collision populations of the current state as float32, population-
 * major: f (Q-1) x ncell for i = 1..Q-1 (the rest population of f is not
 * stored), g Q x ncell.  Either pointer may be NULL. */
LBTP_API int lbtp_populations(lbtp_ctx *ctx, float *f, float *g, int on_device);

/* Checkpoint of the full device state (raw stored populations in their
 * storage type, the pressure base, g, step counter, mass ledger) as an opaque
 * byte image of lbtp_checkpoint_size() bytes.  put_state needs a context with
 * the same lattice, size and storage (LBTP_EINVAL otherwise) that has had
 * lbtp_set_fields; a run resumed from a checkpoint is bitwise identical to
 * the uninterrupted run. */
LBTP_API long long lbtp_checkpoint_size(lbtp_ctx *ctx);
LBTP_API int lbtp_get_state(lbtp_ctx *ctx, void *buf, long long nbytes, int on_device);
LBTP_API int lbtp_put_state(lbtp_ctx *ctx, const void *buf, long long nbytes, int on_device);

/* ------------------------------------------------------------------------
 * Ensembles: n independent realisations (their own size, K, phi, boundary
 * values and sources) advanced together, every coupled step covering all
 * members with one launch per kernel (the blocked plain sweeps of D2Q5: one
 * per size class of members).  Each member's pressure solve stops on its
 * own, on a device-side flag; members that stopped drop out of the
 * remaining sweeps.  Chunks of m sweeps run as captured HIP graphs of 1, 2,
 * 4, 8 or 16 chunks, sized from the iterations the slowest member needed in
 * the previous step, and the host reads the number of active members once
 * per graph.  The members' numbers are bit-identical to separate lbtp_ctx
 * runs with the same parameters (float32; with 16-bit storage, with the
 * same sweeps per launch).  Lattices D2Q5, D3Q7 and D2Q9 (D2Q9 and D3Q7
 * members run one pressure sweep per launch), constant or capillary D_s.
 * All members share lattice, storage, stream and the residual stride m,
 * which must be even; nx % 4 == 0 for every member; max_iters of a step must
 * be a positive multiple of m.  A NULL stream makes the ensemble use a
 * stream of its own (HIP graphs cannot be captured on the null stream).
 * ------------------------------------------------------------------------ */
typedef struct lbtp_batch lbtp_batch;

LBTP_API int lbtp_batch_init(const lbtp_params *members, int n, lbtp_batch **out);
LBTP_API void lbtp_batch_destroy(lbtp_batch *b);
LBTP_API int lbtp_batch_size(lbtp_batch *b);
/* Per-member versions of lbtp_set_fields / lbtp_set_state (member in [0, n)). */
LBTP_API int lbtp_batch_set_fields(lbtp_batch *b, int member, const float *K, const float *phi,
                                   const float *Fp, const float *Fs, int on_device);
LBTP_API int lbtp_batch_set_state(lbtp_batch *b, int member, const float *P0, const float *S0,
                                  const float *dP0, const float *dS0, int on_device);
/* nsteps coupled steps of every member (as lbtp_step).  iters (may be NULL)
 * receives nsteps x n iteration counts, step-major. */
LBTP_API int lbtp_batch_step(lbtp_batch *b, long long nsteps, double tol, long long max_iters,
                             long long *iters);
/* Per-member outputs, as lbtp_pressure / lbtp_saturation / lbtp_velocity /
 * lbtp_mass (the ledger is the ensemble's record of the member's flux). */
LBTP_API int lbtp_batch_pressure(lbtp_batch *b, int member, float *P, int on_device);
LBTP_API int lbtp_batch_saturation(lbtp_batch *b, int member, float *S, int on_device);
LBTP_API int lbtp_batch_velocity(lbtp_batch *b, int member, float *u, int on_device);
LBTP_API int lbtp_batch_mass(lbtp_batch *b, int member, double *mass, double *ledger);
/* Block width of the ensemble pressure sweep: 64, 128, 256 (default) or 512
 * threads of four nodes each.  lbtp_batch_autotune times `sweeps` plain
 * sweeps of the whole ensemble for each width (leaving the state unchanged)
 * and keeps the fastest; *threads receives it.  With blocked plain sweeps
 * (D2Q5, sweep_block > 1) it then tunes, for each size class of members (one
 * grid size), the region shape of the blocked kernel (8 x 8, 8 x 6, 16 x 4,
 * 4 x 8 or 8 x 9 wavefronts x rows) and the sweeps per launch (an odd divisor >= 3 of
 * the m - 1 plain sweeps of a chunk), timing `sweeps` chunks' worth of
 * blocked launches per candidate, and keeps the fastest per class; the
 * choice is remembered for the process (by grid size, storage and m) and
 * taken by later ensembles whose every size was tuned. */
LBTP_API int lbtp_batch_set_threads(lbtp_batch *b, int threads);
LBTP_API int lbtp_batch_autotune(lbtp_batch *b, int sweeps, int *threads);
/* The blocked tiling a member's size class runs: regions of `waves`
 * wavefronts x `rows_per_wave` rows (64 columns) and `sweeps_per_launch`
 * plain sweeps per launch (1: one sweep per launch, waves = 0). */
LBTP_API int lbtp_batch_tiling(lbtp_batch *b, int member, int *waves, int *rows_per_wave, int *sweeps_per_launch);

/* Static description of a status code. */
LBTP_API const char *lbtp_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* LBTP_H */
