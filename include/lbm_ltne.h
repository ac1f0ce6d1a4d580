/*
 * lbm_ltne.h -- C ABI of the MI355X (gfx950) implementation of one fused time
 * step of the REV-scale multiple-relaxation-time lattice Boltzmann model for
 * convection in porous media under local thermal non-equilibrium
 * (Q. Liu, Y.-L. He, arXiv:1608.04118).
 *
 * The step (Sec. 3) couples
 *   - a D2Q9 lattice for the flow: MRT collision in moment space (Eq. 10)
 *     with the transform M (Eq. 13), equilibrium moments (Eq. 15), the
 *     generalized non-Darcy force (Eq. 5) with Boussinesq buoyancy (Eq. 6),
 *     the explicit velocity (Eqs. 20-22) and its moment-space forcing
 *     (Eq. 12, S~ = M S);
 *   - two D2Q5 lattices for the fluid and solid temperatures: MRT collisions
 *     (Eqs. 32, 33) with the transform N (Eq. 36), equilibria (Eqs. 37, 38),
 *     the interphase source terms (Eqs. 29-31) and the explicit temperatures
 *     (Eqs. 43-46);
 *   - streaming (Eqs. 11, 34, 35) and non-equilibrium extrapolation walls
 *     (the boundary scheme named in Sec. 4).
 *
 * Conventions
 *   - Lattice units, delta_x = delta_t = 1.  Node (x, y), x in [0, nx),
 *     y in [0, ny); host fields are row-major doubles, index y * nx + x.
 *   - Velocities in the order of Eq. 8: 0 rest, 1 +x, 2 +y, 3 -x, 4 -y,
 *     5 (+,+), 6 (-,+), 7 (-,-), 8 (+,-); D2Q5 uses 0..4.
 *   - A non-periodic axis has walls on its first and last node, so the
 *     characteristic length defaults to n - 1.  Gravity points along -y.
 *   - Wall index w: 0 left (x = 0), 1 right (x = nx-1), 2 bottom (y = 0),
 *     3 top (y = ny-1).
 *   - Every entry point returns LBM_OK (0) or a negative LBM_E* code and never
 *     throws.  lbm_ltne_strerror() names the code; lbm_ltne_last_error()
 *     gives the last detailed message of the calling thread.
 *   - Handles are not thread-safe.  Work is queued on the stream given at
 *     creation; entry points that return host data synchronize that stream.
 *
 * Time convention: the state is always the post-collision populations of the
 * current time t; creating a handle performs the boundary treatment and the
 * collision of t = 0, so lbm_ltne_macros() is valid right after creation.
 */
#ifndef LBM_LTNE_H
#define LBM_LTNE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_LTNE_ABI_VERSION 3

/* Return codes. */
#define LBM_OK 0
#define LBM_EINVAL (-1)       /* invalid argument or physically invalid parameters */
#define LBM_ENOMEM (-2)       /* device allocation failed or caller pool too small */
#define LBM_EHIP (-3)         /* a HIP runtime call failed (message in last_error) */
#define LBM_EDIVERGED (-4)    /* non-finite mass or energy detected (diagnostics, or the check of diag_every) */
#define LBM_EUNSUPPORTED (-5) /* valid request the library does not implement */
#define LBM_ENODEV (-6)       /* no gfx950 device is available */

/* Storage / arithmetic forms. */
#define LBM_FP64 0  /* binary64 storage and arithmetic */
#define LBM_FP32 1  /* binary32 storage of shifted populations; binary32 flow arithmetic, binary64 temperature
                       arithmetic with stochastic rounding of the temperature populations on store */
#define LBM_FP16S 2 /* binary16 storage of shifted, power-of-two scaled populations; binary32 arithmetic,
                       stochastic rounding on store */
#define LBM_FP32SR 3 /* binary32 storage of shifted populations; binary64 arithmetic, stochastic rounding
                        on store (rounding errors average out instead of repeating on slowly changing fields) */

/* Thermal wall conditions. */
#define LBM_WALL_DIRICHLET 0
#define LBM_WALL_ADIABATIC 1

typedef struct lbm_ltne *lbm_ltne_t;
typedef struct lbm_ltne_batch *lbm_ltne_batch_t;

/*
 * Problem statement.  The physical inputs are the groups of Sec. 2
 * (Ra, Pr, Da, J_e, gamma_sf, sigma, H_v) plus the porosity phi (the paper's
 * epsilon), the Forchheimer coefficient F_phi and the internal heat sources;
 * the free relaxation rates and varpi are those of Eqs. 17, 39, 40 and the
 * D2Q5 weights.  lbm_ltne_default_params() fills the setup of Sec. 4.
 */
typedef struct lbm_ltne_params {
  int32_t nx, ny;          /* nodes, walls included; >= 4 on a walled axis, >= 3 on a periodic one */
  int32_t precision;       /* LBM_FP64, LBM_FP32, LBM_FP16S or LBM_FP32SR */
  int32_t periodic_x;      /* 1: periodic along x, 0: walls at x = 0 and x = nx-1 */
  int32_t periodic_y;      /* 1: periodic along y, 0: walls at y = 0 and y = ny-1 */
  int32_t wall_thermal[4]; /* LBM_WALL_* for walls 0..3 (ignored on periodic axes) */
  int32_t nu_wall;         /* wall of the reported Nusselt number; -1: hottest Dirichlet wall */
  int32_t thermal_correction; /* 1: add the correction term of Sec. 3.2 to the fluid D2Q5 equation, 0: off */
  double T_wall[4];        /* Dirichlet temperature of walls 0..3 (both phases) */
  double T0;               /* Boussinesq reference temperature T_0 (Eq. 6) */
  double T_init_f, T_init_s; /* uniform initial temperatures when no field is given */
  double L;                /* characteristic length; <= 0: nx-1 if x is walled, else ny-1 */
  double dT;               /* temperature scale; <= 0: spread of the Dirichlet wall temperatures (1 if none) */
  double phi;              /* porosity in (0, 1) (per-node field may replace it) */
  double Da;               /* Darcy number K / L^2 (Sec. 2) */
  double F_phi;            /* Forchheimer coefficient (Eq. 5); < 0: Ergun relation of Eq. 7 at the local phi */
  double Ra, Pr, Je;       /* Rayleigh, Prandtl numbers, viscosity ratio nu_e / nu_f */
  double gamma_sf;         /* solid-to-fluid conductivity ratio k_s / k_f */
  double sigma;            /* solid-to-fluid heat capacity ratio (rho c_p)_s / (rho c_p)_f */
  double Hv;               /* interphase coefficient h_v L^2 / k_f (per-node field may replace it) */
  double Qf, Qs;           /* q'''/(rho c_p) of each phase in lattice units (Eq. 45) */
  double Ma;               /* buoyancy Mach number u_c / c_s, u_c = sqrt(g beta dT L); used when nu_f <= 0 */
  double nu_f;             /* fluid viscosity in lattice units; > 0 takes precedence over Ma */
  double body_force[2];    /* constant body acceleration G_b added to the buoyancy G of Eq. 6 */
  double varpi;            /* D2Q5 weight parameter in (0, 1); cs_T^2 = varpi / 2 */
  double s_e, s_eps, s_q;  /* free D2Q9 rates of Eq. 17 (s_nu follows from nu_e, Eq. 23) */
  double zeta_e, zeta_nu;  /* free fluid D2Q5 rates of Eq. 39 (zeta_alpha follows from alpha_f, Eq. 49) */
  double eta_e, eta_nu;    /* free solid D2Q5 rates of Eq. 40 (eta_alpha follows from alpha_s) */
  double rho0;             /* initial density; also the population shift reference */
  double T_ref;            /* temperature shift reference of the FP32/FP16 forms; NaN: midpoint of the wall and initial temperatures */
  double fp16_scale_f;     /* power-of-two storage scale of shifted D2Q9 populations (LBM_FP16S); 0: automatic */
  double fp16_scale_g;     /* same for the D2Q5 populations; 0: automatic */
  double pore_size;        /* D_p / L; > 0: h_v of every node from the correlation of Eq. 52 with the
                              local Reynolds number |j| D_p / (rho nu_f) (Hv and an H_v field are then
                              not used); 0: h_v from Hv or the H_v field */
  int32_t diag_every;      /* > 0: lbm_ltne_step checks every diag_every-th step (steps whose number
                              is a multiple of it) for non-finite mass or energy (binary64 sums of the
                              macroscopic fields of that step, on the device); the next synchronizing
                              call then returns LBM_EDIVERGED.  0: no check.  Single lattices only. */
} lbm_ltne_params;

/* Lattice values derived from a parameter set (uniform phi and H_v). */
typedef struct lbm_ltne_derived {
  double L, dT;            /* characteristic length and temperature scale */
  double cs2, csT2;        /* 1/3 and varpi/2 */
  double gbeta;            /* g beta in lattice units */
  double u_c;              /* buoyancy velocity sqrt(g beta dT L) */
  double nu_f, nu_e;       /* viscosities */
  double s_nu, tau_nu;     /* Eq. 23 */
  double alpha_f, alpha_s; /* thermal diffusivities */
  double zeta_a, eta_a;    /* Eq. 49 */
  double tau_Tf, tau_Ts;   /* 1/zeta_a, 1/eta_a */
  double K;                /* permeability Da L^2 */
  double F_phi;            /* Forchheimer coefficient at the uniform phi */
  double l0, l1;           /* Eq. 22 at the uniform phi */
  double d0, d1;           /* Eq. 46 at the uniform phi and H_v */
  double T_ref;            /* resolved temperature shift */
  double scale_f, scale_g; /* resolved FP16 storage scales (1 for other forms) */
} lbm_ltne_derived;

/* Fills the cavity setup of Sec. 4 (varpi = 2/5, s_e = s_eps = 1.1,
 * s_q = 1.2, zeta_e = zeta_nu = eta_e = eta_nu = 1.1, J_e = 1, sigma = 1,
 * Pr = 1) on a 64 x 64 lattice with a hot left and a cold right wall,
 * adiabatic top and bottom, Ma = 0.1, FP64.  p must not be NULL. */
int lbm_ltne_default_params(lbm_ltne_params *p);

/* Validates p and maps it to lattice units (host only, no device use).
 * Rejects with LBM_EINVAL: sizes out of range, phi not in (0, 1), Da <= 0,
 * Pr <= 0, Je <= 0, sigma <= 0, gamma_sf < 0, Hv < 0, varpi not in (0, 1),
 * any rate not in (0, 2), no usable scale (nu_f <= 0 and Ma or Ra <= 0),
 * a derived relaxation time <= 1/2, a non-finite input.  d may be NULL. */
int lbm_ltne_derive(const lbm_ltne_params *p, lbm_ltne_derived *d);

/* Bytes of device memory lbm_ltne_create needs for p when a caller pool is
 * used (has_phi / has_Hv: whether those fields will be passed).  0 on
 * invalid parameters. */
size_t lbm_ltne_pool_bytes(const lbm_ltne_params *p, int has_phi, int has_Hv);

/*
 * Creates a lattice, initialises it (fluid at rest with density rho0,
 * temperatures T_init or the given fields, populations g = g^eq - w~ Sr / 2
 * so that Eqs. 43-44 return the initial temperatures) and performs the
 * collision of t = 0.
 *   phi_field, Hv_field, Tf_init, Ts_init: optional host arrays of nx*ny
 *     doubles (NULL: uniform p->phi, p->Hv, p->T_init_f, p->T_init_s);
 *     copied, the caller keeps ownership.  phi must lie in (0, 1), Hv >= 0;
 *     an Hv_field with p->pore_size > 0 (the correlation of Eq. 52) is
 *     refused with LBM_EINVAL.
 *   hip_stream: a hipStream_t to queue all work on (borrowed; NULL: the
 *     default stream of the current device).
 *   device_pool, pool_bytes: optional caller-owned device memory of at least
 *     lbm_ltne_pool_bytes() bytes (borrowed, must outlive the handle); NULL:
 *     the library allocates and frees its own.
 *   out: receives the handle.
 * Errors: LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_ENODEV. */
int lbm_ltne_create(const lbm_ltne_params *p, const double *phi_field, const double *Hv_field,
                    const double *Tf_init, const double *Ts_init, void *hip_stream,
                    void *device_pool, size_t pool_bytes, lbm_ltne_t *out);

/* Advances nsteps >= 0 time steps (asynchronous).  Each step is one fused
 * launch: pull streaming, wall reconstruction, macros, the three collisions,
 * store.  In the FP32 and FP64 forms, on lattices that yield at least 1024
 * (FP32) or 2560 (FP64) strips of 62 (periodic x) or 61 columns by 8 rows,
 * the steps of a call advance in pairs, two steps per launch with the
 * intermediate time level kept on chip (an odd last step, and the steps
 * checked under diag_every, alone); the result equals single steps bit for
 * bit.  Small lattices run their steps in recorded sequences of launches (a
 * HIP graph).  The macros of the last step are kept for
 * lbm_ltne_macros, lbm_ltne_nusselt and lbm_ltne_diagnostics; the residual
 * compares them with the macros kept by the previous call that advanced the
 * lattice (a call with nsteps = 0 changes nothing).  With diag_every > 0 a
 * non-finite mass or energy at a checked step is recorded on the device and
 * reported as LBM_EDIVERGED by lbm_ltne_macros, lbm_ltne_nusselt,
 * lbm_ltne_diagnostics and lbm_ltne_save (which still fill their outputs)
 * until a state is loaded. */
int lbm_ltne_step(lbm_ltne_t h, int64_t nsteps);

/* Steps taken since creation (or since the state loaded by lbm_ltne_load). */
int64_t lbm_ltne_steps_done(lbm_ltne_t h);

/* Copies the macroscopic fields of the current time to host arrays of nx*ny
 * doubles: rho (Eq. 18), u (Eq. 20), T_f, T_s (Eqs. 43-44); wall nodes report
 * their prescribed values.  Any pointer may be NULL.  Synchronizes. */
int lbm_ltne_macros(lbm_ltne_t h, double *rho, double *ux, double *uy, double *Tf, double *Ts);

/* Mean Nusselt numbers of the fluid and solid phase over wall p->nu_wall:
 * Nu = (L / dT) <-dT/dn>, dT/dn by the one-sided second-order difference
 * (-3 T_0 + 4 T_1 - T_2) / 2 along the inward normal, averaged by the
 * trapezoid rule along a walled wall (plain mean along a periodic one).
 * Binary64 reduction in a fixed order.  Synchronizes.  LBM_EINVAL if no wall
 * is selected. */
int lbm_ltne_nusselt(lbm_ltne_t h, double *Nu_f, double *Nu_s);

/* Binary64 reductions in a fixed order: total mass sum(rho), thermal energy
 * sum(phi T_f + (1 - phi) sigma T_s), and the relative change
 * max over (u, T_f, T_s) of sum|a - a_prev| / sum|a| between the macros of
 * the last two step calls.  Any pointer may be NULL.  Returns LBM_EDIVERGED
 * (after filling the outputs) if mass or energy is not finite.  Synchronizes. */
int lbm_ltne_diagnostics(lbm_ltne_t h, double *mass, double *energy, double *residual);

/* Checkpoint: bytes of a saved state, save to and load from a caller-owned
 * host buffer (populations, macros, step count).  load requires a handle
 * created with the same nx, ny and precision, and clears a recorded
 * divergence.  Synchronize. */
size_t lbm_ltne_state_bytes(lbm_ltne_t h);
int lbm_ltne_save(lbm_ltne_t h, void *host_buf, size_t bytes);
int lbm_ltne_load(lbm_ltne_t h, const void *host_buf, size_t bytes);

/*
 * Discrete adjoint (reverse-time) of the time stepping.  Advances the lattice
 * by nsteps >= 1 steps from its current state exactly as lbm_ltne_step does,
 * and returns the loss L = mean hot-wall Nusselt number of the fluid phase
 * (lbm_ltne_nusselt) at the final time, with dL/dphi and dL/dH_v at every
 * node (host arrays of nx*ny doubles, row-major; either may be NULL).  The
 * gradient is that of the discrete map actually computed: every step,
 * the wall reconstruction and, when the handle is still at t = 0, the
 * initialisation.  Checkpoints of the state are kept every ckpt_every steps
 * (< 1: one segment) and each segment is recomputed once while its
 * per-node sums are recorded, on a second stream of the library's own that
 * runs the recompute of one segment while the handle's stream sweeps the
 * next one back.  Work memory of about (nsteps/ckpt_every + 2) state copies
 * + 40 x ckpt_every bytes per node (binary32; two recording buffers, or one
 * with 20 x ckpt_every bytes per node when two do not fit, and then the
 * recompute and the sweep alternate) is allocated for the call.  FP64, FP32 and FP32SR forms
 * (LBM_EUNSUPPORTED for FP16 storage, and for a lattice with the correlation
 * of Eq. 52; the correction term of Sec. 3.2 is covered).  Synchronizes.  On an error the
 * lattice is left at its state on entry (unless the device itself failed).
 */
int lbm_ltne_adjoint(lbm_ltne_t h, int64_t nsteps, int64_t ckpt_every, double *loss, double *dL_dphi,
                     double *dL_dHv);

/* Derived lattice values of a live handle. */
int lbm_ltne_get_derived(lbm_ltne_t h, lbm_ltne_derived *d);

/* Releases the handle and the device memory it owns (never a caller pool).
 * NULL is accepted. */
int lbm_ltne_destroy(lbm_ltne_t h);

/*
 * Batched lattices: n independent lattices of uneven size and parameters
 * (one precision per batch) advanced together.  By default (mode 0) a batch
 * step is one launch over the combined tile list of all lattices (FP32
 * batches of at least 1024 strips of 8 rows: pairs of steps per launch, as in
 * lbm_ltne_step, with per-lattice chunk heights, 16 rows by default); mode 1
 * runs all steps of a call in one persistent cooperative launch with a
 * grid-wide barrier between steps (every barrier wait is bounded; a timeout
 * is reported as LBM_EHIP by the next synchronizing call).  Every lattice
 * evolves exactly as a single lattice with the same parameters would.
 *   ps: n parameter sets (diag_every must be 0: LBM_EUNSUPPORTED otherwise);
 *   phi_fields, Hv_fields: NULL, or n pointers each NULL or nx*ny doubles
 *   (copied).  The batch owns its device memory.
 */
int lbm_ltne_batch_create(int32_t n, const lbm_ltne_params *ps, const double *const *phi_fields,
                          const double *const *Hv_fields, void *hip_stream, lbm_ltne_batch_t *out);
int lbm_ltne_batch_step(lbm_ltne_batch_t b, int64_t nsteps);
int64_t lbm_ltne_batch_steps_done(lbm_ltne_batch_t b);
/* Macros of lattice i (host arrays of nx*ny doubles, any may be NULL). */
int lbm_ltne_batch_macros(lbm_ltne_batch_t b, int32_t i, double *rho, double *ux, double *uy,
                          double *Tf, double *Ts);
/* Mean Nusselt numbers of lattice i (definition of lbm_ltne_nusselt). */
int lbm_ltne_batch_nusselt(lbm_ltne_batch_t b, int32_t i, double *Nu_f, double *Nu_s);
/* 0: one launch per step (default), 1: persistent cooperative launch (LBM_EUNSUPPORTED if the
 * device cannot keep a grid resident). */
int lbm_ltne_batch_set_mode(lbm_ltne_batch_t b, int32_t persistent);
/* Total nodes, tiles, persistent grid size (workgroups) and current mode. */
int lbm_ltne_batch_info(lbm_ltne_batch_t b, int64_t *nodes, int32_t *tiles, int32_t *grid,
                        int32_t *persistent);
/* Tile width of each lattice as log2 (6, 7, 8 = 64, 128, 256 nodes wide; 0 = default). */
int lbm_ltne_batch_set_tiles(lbm_ltne_batch_t b, const int32_t *tile_shift);
int lbm_ltne_batch_get_tiles(lbm_ltne_batch_t b, int32_t *tile_shift);
/* Chunk height (rows) of each lattice's wavefronts in the two-step launches
 * of an FP32 batch: 8, 12, 16, 24 or 32 (0 = default 16). */
int lbm_ltne_batch_set_chunks(lbm_ltne_batch_t b, const int32_t *rows);
int lbm_ltne_batch_get_chunks(lbm_ltne_batch_t b, int32_t *rows);
/* Autotuner: for each size class (lattices of equal nx) tries tile widths
 * 64/128/256 by timing reps single-step launches, then (FP32 batches that
 * run two steps per launch) chunk heights 8..32 by timing 2 reps steps of
 * two-step launches, then the launch mode (one launch per step or pair of
 * steps, or one persistent launch; skipped when the device has no resident
 * grid for it) by timing 2 reps steps of each, every trial from a snapshot
 * of the state (restored afterwards), and keeps the fastest of each;
 * ms_per_step (may be NULL) receives the time per step of the chosen
 * configuration on the path the batch runs (two-step launches where they
 * apply).  Allocates a snapshot of the populations for the call. */
int lbm_ltne_batch_autotune(lbm_ltne_batch_t b, int32_t reps, double *ms_per_step);
int lbm_ltne_batch_destroy(lbm_ltne_batch_t b);

/*
 * Binary64 sums of macroscopic fields held by the caller, computed without
 * any allocation -- for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The sums are those of lbm_ltne_diagnostics, in the same fixed
 * order (bit-identical for the same fields): total mass, thermal energy and
 * the residual between mac and prev.
 *   p: nx, ny; precision selects the compute type of the fields (double for
 *     LBM_FP64 and LBM_FP32SR, float for LBM_FP32 and LBM_FP16S); phi (used
 *     when phi_field is NULL) and sigma weight the energy.
 *   mac, prev: device addresses of 5 planes of nx*ny values each (rho, u_x,
 *     u_y, T_f, T_s; node (x, y) at y * nx + x), the current and the
 *     previous macros; borrowed, read only.
 *   phi_field: device address of nx*ny porosities in the compute type, or NULL.
 *   hip_stream: the stream to queue on (NULL: default stream); synchronized.
 * Scratch: a file-scope device array of about 66 KB per GPU, held until the
 * process ends; calls that overlap on one GPU race on it.  Lattices of up
 * to 2^30 nodes.  Errors: LBM_EINVAL (NULL field pointer, empty or oversized
 * lattice, unknown precision, phi or sigma out of range), LBM_EHIP,
 * LBM_EUNSUPPORTED (device index above 63), LBM_EDIVERGED (a non-finite mass
 * or energy; the outputs are filled).
 */
int lbm_ltne_macro_sums_noalloc(const lbm_ltne_params *p, const void *mac, const void *prev,
                                const void *phi_field, void *hip_stream, double *mass, double *energy,
                                double *residual);

/* Static description of a return code. */
const char *lbm_ltne_strerror(int code);

/* Last detailed error message of the calling thread ("" if none). */
const char *lbm_ltne_last_error(void);

/* LBM_LTNE_ABI_VERSION of the library. */
int lbm_ltne_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_LTNE_H */
