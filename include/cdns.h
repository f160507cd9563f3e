/*
 * cdns.h -- C ABI of the MI355X library for the right-hand side and
 * low-storage RK3 step of the compressible Navier-Stokes equations as
 * discretised in "STREAmS: a high-fidelity accelerated solver for direct
 * numerical simulation of compressible turbulent flows" (arXiv 2004.02276).
 *
 * Equations (Sec. 2, eqs. mass/momentum/energy): conservation of mass,
 * momentum and total energy of a perfect heat-conducting gas with Newtonian
 * stresses, Fourier heat flux, Sutherland viscosity, k = c_p mu / Pr, and an
 * optional streamwise body force f with power f u (constant mass flow).
 * Convective terms (Sec. 2.1, eqs. num_flux, avg_operator, encflux):
 * kinetic-energy-preserving central flux in split form of order 2L (fourth
 * order by default, L = 1..3 selectable), replaced at interfaces flagged by
 * the Ducros sensor (eq. sensor) with WENO reconstruction (fifth order by
 * default, third and seventh selectable) of Lax-Friedrichs-split
 * characteristic fluxes.  Viscous terms in Laplacian form with formulas of
 * the same order 2L.  Time integration (Sec. 2.2, eq. RK): Wray's
 * three-stage low-storage scheme.
 *
 * Conventions
 *  - Every function returns a cdns_status; nothing aborts or throws across
 *    the ABI.  On error the context's message is available from
 *    cdns_last_error().
 *  - Device memory is owned by the caller (allocated, e.g., by PyTorch).
 *    The library never frees caller memory and calls no device allocator
 *    on the stepping path.
 *  - State layout: double w[5][nz][ny][nx] (x fastest) holding
 *    (rho, rho u, rho v, rho w, rho E); same layout for right-hand sides.
 *  - Non-dimensional variables: the gas constant R_gas sets the reference
 *    Mach number (R = 1/(gamma M^2) with unit reference density,
 *    velocity and temperature); c_v = R/(gamma-1), c_p = gamma R/(gamma-1).
 *  - Grid: x and z uniform (dx = lx/nx, dz = lz/nz); y given by the metric
 *    of a mapping y(eta) sampled at the nodes, d_eta = 1/ny.  With walls
 *    the nodes sit at eta_j = (j+1/2)/ny so the walls fall half-way
 *    between the last node and the first ghost (staggered wall, Sec. 3.1).
 *  - All work is enqueued on the hip stream given at creation and is
 *    asynchronous, except cdns_diagnostics(), the export hooks,
 *    cdns_time_phases() and cdns_stats_export(), which synchronise that
 *    stream.
 */
#ifndef CDNS_H
#define CDNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cdns_status;
enum {
  CDNS_OK = 0,
  CDNS_EINVAL = -1,  /* invalid argument or unsupported combination of values */
  CDNS_ENOMEM = -2,  /* workspace too small */
  CDNS_EHIP = -3,    /* a HIP runtime call failed */
  CDNS_ESTATE = -4,  /* device detected a non-finite or non-positive state */
  CDNS_EUNSUP = -5,  /* boundary condition not supported on that face */
  CDNS_EBUSY = -6    /* batch full / slot in use */
};

/* Arithmetic of the flux evaluation.  CDNS_FP32_FLUX evaluates the central
 * and shock-capturing fluxes and the viscous terms in single precision; the
 * stored state, the RK accumulation, the shock sensor and every reduction
 * stay double precision. */
enum { CDNS_FP64 = 0, CDNS_FP32_FLUX = 1 };

/* Shock sensor mode: central flux only; hybrid (sensor-driven switch);
 * shock-capturing flux at every interior interface. */
enum { CDNS_SENSOR_OFF = 0, CDNS_SENSOR_HYBRID = 1, CDNS_SENSOR_WENO_ALL = 2 };

/* Boundary conditions (faces 0..5 = x-, x+, y-, y+, z-, z+).  Ghost nodes
 * (3 per face) are filled x faces first, then y faces over the x-extended
 * range; z must be periodic.
 *  PERIODIC        both faces of an axis; no parameters.
 *  WALL_ISOTHERMAL y faces; params[0] = wall temperature T_w.  No-slip
 *                  staggered wall: ghost s mirrors interior node s-1 with
 *                  u -> -u, p -> p, T -> 2 T_w - T; the wall interface
 *                  carries no convective flux, only pressure (Sec. 3.1).
 *  WALL_ADIABATIC  y faces; as above with T -> T.
 *  DIRICHLET       x faces; params = primitive profile (rho,u,v,w,p) as
 *                  5 rows of ny values (row-major [5][ny]) imposed at the
 *                  ghost nodes (inflow).
 *  OUTFLOW_CHAR    x and y faces; characteristic extrapolation: the wave
 *                  amplitudes of (w_b - w_{b-1}) travelling out of the
 *                  domain are extrapolated linearly, incoming ones are held
 *                  (Sec. 3.2: non-reflecting treatment by characteristic
 *                  decomposition normal to the boundary; the exact form is a
 *                  reading, the paper gives no formula).
 *  SHOCK_TOP       y faces; params = {i_shock, rho1,u1,v1,w1,p1,
 *                  rho2,u2,v2,w2,p2}: ghost nodes take state 1 for
 *                  i < i_shock and state 2 otherwise (imposed inviscid
 *                  oblique-shock solution, Sec. 3.3).
 *  DF_INFLOW       x- face only; synthetic inflow turbulence by digital
 *                  filtering (Sec. 3.2).  params = {n_y, n_z, T, seed,
 *                  mean (rho,u,v,w,p) [5][ny], Reynolds stresses (R11,
 *                  R22, R33, R12, R13, R23) [6][ny]} (4 + 11 ny values):
 *                  n_y, n_z are the integral lengths of the inflow
 *                  turbulence in grid spacings (y: the caller's mean
 *                  spacing), T its Lagrangian time scale.  The library
 *                  derives the Gaussian filter coefficients b_l ~
 *                  exp(-pi l^2/(2 n^2)), |l| <= N = max(1, ceil(2 n)) <= ny
 *                  (resp. nz), unit sum of squares, and the lower
 *                  triangular factor a a^T = R (Lund's transformation).
 *                  Deviates uniform on [-sqrt 3, sqrt 3) from SplitMix64
 *                  (output n of the generator seeded with `seed`, n = 1 +
 *                  (((key*3 + c)*nz + k)*(ny + 2 N_y) + jj) for component
 *                  c, plane k, extended row jj; key 0 for the initial plane
 *                  made by this call, key s + 1 at the start of step s);
 *                  filtered along y then z (periodic); time correlation
 *                  psi = psi E + psi_hat sqrt(1 - E^2), E = exp(-pi dt/(2T));
 *                  fluctuations u'_i = a_ij psi_j; T' = -u_mean u'/c_p at
 *                  constant pressure (strong Reynolds analogy).  The plane
 *                  is refreshed once per RK step and imposed on the ghost
 *                  layers.  Not accepted by batches. */
enum {
  CDNS_BC_PERIODIC = 0,
  CDNS_BC_WALL_ISOTHERMAL = 1,
  CDNS_BC_WALL_ADIABATIC = 2,
  CDNS_BC_DIRICHLET = 3,
  CDNS_BC_OUTFLOW_CHAR = 4,
  CDNS_BC_SHOCK_TOP = 5,
  CDNS_BC_DF_INFLOW = 6
};

typedef struct {
  int32_t nx, ny, nz;         /* interior nodes, each >= 4 */
  double lx, lz;              /* periodic lengths / extents of the uniform axes */
  const double* y_eta;        /* host array [ny]: dy/deta at the nodes (copied) */
  const double* y_etaeta;     /* host array [ny]: d2y/deta2 at the nodes (copied) */
} cdns_grid;

typedef struct {
  double gamma;               /* ratio of specific heats */
  double Pr;                  /* Prandtl number */
  double R_gas;               /* gas constant */
  double mu_ref, T_ref, S_suth; /* Sutherland: mu = mu_ref t^1.5 (1+S)/(t+S), t = T/T_ref */
  int32_t viscous;            /* 0: Euler equations, 1: Navier-Stokes */
  int32_t sensor_mode;        /* CDNS_SENSOR_* */
  double theta_star;          /* node flag when theta > theta_star */
  double sensor_eps;          /* regulariser of the sensor denominator, (u0/L0)^2 */
  int32_t forcing;            /* constant streamwise mass flow (bulk force f) */
} cdns_phys;

/* Diagnostics (volume integrals use dV = dx dz d_eta y_eta). */
typedef struct {
  double dt;                  /* last time step used */
  double time;                /* accumulated time */
  double mass, mom[3], energy, kinetic;
  double rho_min, p_min, mach_max;
  double forcing_f;           /* bulk force of the last stage evaluated */
  double weno_frac[3];        /* shock-capturing share of interfaces, last stage */
  int64_t step;               /* completed RK steps */
  int64_t nonfinite;          /* non-finite conserved values */
  int32_t status;             /* device status bits (0 = healthy) */
} cdns_diag;

typedef struct cdns_ctx cdns_ctx;
typedef struct cdns_batch cdns_batch;

/* Bytes of device workspace cdns_create needs for this grid and precision.
 * Returns 0 for an invalid grid. */
size_t cdns_workspace_bytes(const cdns_grid* grid, int32_t precision);

/* Create a solver instance.  state_dev: caller-owned device array
 * [5][nz][ny][nx] holding w^n; it is read and updated in place by the
 * stepping calls.  workspace_dev: caller-owned device memory of at least
 * cdns_workspace_bytes() bytes, 256-byte aligned, used for stage states,
 * residual registers, ghost planes, flags, lists and reductions.
 * hip_stream: a hipStream_t (NULL = default stream).  All faces start
 * periodic.  On success *out receives the context. */
cdns_status cdns_create(const cdns_grid* grid, const cdns_phys* phys, int32_t precision,
                        double* state_dev, void* workspace_dev, size_t workspace_bytes,
                        void* hip_stream, cdns_ctx** out);

/* Set the boundary condition of one face (CDNS_BC_*, see above).  params
 * is a host array of nparams doubles (copied).  Both faces of an axis must
 * be periodic or both non-periodic; combinations not listed above return
 * CDNS_EUNSUP.  Call before stepping; CDNS_EBUSY while the context is
 * attached to a batch (as for cdns_set_tiling and cdns_set_scheme). */
cdns_status cdns_set_bc(cdns_ctx* ctx, int32_t face, int32_t kind, const double* params,
                        int64_t nparams);

/* Debugging hook: fills every double-precision work region of the
 * workspace that the stepping path writes before reading it (stage states,
 * residual registers, shock-capturing fluxes, sensor values, ghost planes,
 * inflow-generator fields, reduction partials) with NaN, so that a read of
 * memory no kernel has written shows up as a NaN in the results.  The
 * digital-filter inflow's initial plane is regenerated.  Synchronises;
 * CDNS_EBUSY while attached to a batch. */
cdns_status cdns_poison_workspace(cdns_ctx* ctx);

/* Tile shape of the fused right-hand-side kernel: (tile_x, tile_y) must be
 * one of the compiled variants (64x4, 32x8, 64x2, 128x2, 64x8), kz >= 1
 * planes per block.  Results are bitwise independent of the choice except
 * for the rounding of the bulk-force sum, whose per-tile partial sums follow
 * the tiling.  Returns CDNS_EINVAL for other shapes, CDNS_EUNSUP for a
 * shape other than 64x4 when the central order is not 4. */
cdns_status cdns_set_tiling(cdns_ctx* ctx, int32_t tile_x, int32_t tile_y, int32_t kz);

/* Scheme orders (Sec. 2.1; eq. encflux gives the central flux of order 2L
 * for any L, the viscous formulas use first and second derivatives of the
 * same order; the WENO scheme is cited without its order).  central_order
 * in {2, 4, 6} (L = 1, 2, 3): the split-form flux over the pairs
 * (i-m, i-m+l), l = 1..L, m < l, and the Laplacian-form viscous terms;
 * interface i+1/2 switches to the shock-capturing flux when a node of
 * i-L+1..i+L is flagged.  weno_order in {3, 5, 7}: Jiang-Shu reconstruction
 * from r = 2, 3, 4 candidate stencils (smoothness indicators are the
 * integrals of the squared candidate derivatives, eps = 1e-6), the
 * Lax-Friedrichs constant taken over the 2r stencil nodes.  The shock
 * sensor keeps fourth-order derivatives, and the viscous time-step bound
 * uses the largest magnitude of the order-2L second-derivative symbol (4,
 * 16/3, 272/45).  Defaults: 4 and 5.  Orders other than 4 run the fused
 * kernel in the 64x4 tile only (the tiling is reset to the default if it
 * differs) and need nz >= central_order.  With a digital-filter inflow the
 * initial inflow plane is regenerated.  Call before stepping.  Returns
 * CDNS_EINVAL for other orders or too small a grid. */
cdns_status cdns_set_scheme(cdns_ctx* ctx, int32_t central_order, int32_t weno_order);

/* Copy a state w [5][nz][ny][nx] (the conserved vector of Sec. 2.2) into
 * the context's state array (from_host != 0: w is host memory and the call
 * returns after the copy; else w is device memory and the copy is
 * stream-ordered), or the state out of it (to_host != 0: synchronous copy
 * to host memory; else stream-ordered to device memory).  The state array
 * is the caller's own allocation; these calls are conveniences for callers
 * that do not address it directly. */
cdns_status cdns_set_state(cdns_ctx* ctx, const double* w, int32_t from_host);
cdns_status cdns_get_state(cdns_ctx* ctx, double* w, int32_t to_host);

/* Full right-hand side R(w) of dw/dt = R(w) (Sec. 2.2) for the device
 * array w_dev [5][nz][ny][nx], written to r_dev (same layout), including
 * boundary conditions, sensor switching and bulk forcing. */
cdns_status cdns_rhs(cdns_ctx* ctx, const double* w_dev, double* r_dev);

/* One RK3 step of the state.  dt_fixed > 0 sets the step; otherwise
 * dt = cfl * min(1/max sum_d (|u_d|+c)/dx_d, 2.5/max[max(4/3,gamma/Pr)
 * (mu/rho) s2 sum_d dx_d^-2]) is computed on the device from w^n, s2 the
 * largest magnitude of the central second-derivative symbol (16/3 at
 * fourth order); with the hybrid sensor (and no digital-filter inflow) the
 * first stage's sensor kernel reduces the two maxima.  In the default 64x4
 * tiling each stage's update is done by the right-hand-side kernel as it
 * finishes a point (the same rounding as the separate update kernel used
 * otherwise): the whole update without bulk forcing; with forcing the
 * rho, rho v and rho w components, rho u and rho E following in an update
 * kernel once the force is reduced. */
cdns_status cdns_rk_step(cdns_ctx* ctx, double cfl, double dt_fixed);

/* n RK3 steps, replayed from one captured HIP graph per step. */
cdns_status cdns_advance_n(cdns_ctx* ctx, int32_t n, double cfl, double dt_fixed);

/* Volume integrals, extrema and status of the current state; synchronises
 * the stream.  Returns CDNS_ESTATE if the device flagged a bad state (an RK
 * stage produced a point with rho <= 0, p <= 0 or a non-finite energy;
 * with bulk forcing in the default tiling this is detected when the next
 * stage reads the point) or the current state has rho_min <= 0,
 * p_min <= 0 or non-finite values. */
cdns_status cdns_diagnostics(cdns_ctx* ctx, cdns_diag* out);

/* For callers that cannot allocate memory or synchronise (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the volume integrals and extrema of cdns_diagnostics, computed on the
 * device and written to the device array out_dev[CDNS_NDIAG_DEV] in the
 * order of the CDNS_DV_* slots (the non-finite count as a double).  w_dev is
 * a device state [5][nz][ny][nx] of the context's grid, or NULL for the
 * context's state array.  Enqueued on the context's stream; no host
 * synchronisation, no allocation, no use of the context's workspace.  The
 * per-block partial sums live in one static device array per GPU (8192
 * blocks x 16 doubles = 1 MiB, one block per 4096 points), held until the
 * process ends: grids of more than CDNS_NOALLOC_MAX_POINTS points return
 * CDNS_EINVAL.  All calls on one GPU share that array, so calls that overlap
 * in time on one GPU (different streams, or different host threads) race;
 * calls ordered on one stream do not.  The sums are grouped differently from
 * cdns_diagnostics (rounding differs in the last bits; extrema and counts are
 * identical).  Status checks of the state are left to the caller. */
enum { CDNS_DV_MASS = 0, CDNS_DV_MOMX, CDNS_DV_MOMY, CDNS_DV_MOMZ, CDNS_DV_ENERGY, CDNS_DV_KINETIC,
       CDNS_DV_RHOMIN, CDNS_DV_PMIN, CDNS_DV_MACHMAX, CDNS_DV_NONFINITE, CDNS_NDIAG_DEV };
#define CDNS_NOALLOC_MAX_POINTS 33554432LL
cdns_status cdns_diagnostics_noalloc(cdns_ctx* ctx, const double* w_dev, double* out_dev);

/* Running statistics for mean profiles and turbulent stresses (the
 * quantities of Sec. 4's validation figures; the paper does not describe
 * how they are gathered).  cdns_stats_accumulate adds, for every (i, j)
 * column, the spanwise sums (k ascending) over the current state of
 * CDNS_NSTAT products to a per-context accumulator [CDNS_NSTAT][ny][nx]
 * and counts one sample (asynchronous, no host synchronisation);
 * cdns_stats_export copies the accumulator to host memory (caller-owned,
 * CDNS_NSTAT*ny*nx doubles) and the sample count to *samples
 * (synchronises); cdns_stats_reset zeroes both.  Quantities, with
 * u = (rho u)/rho, T = (E/rho - |u|^2/2)/c_v, p = rho R T: */
enum { CDNS_ST_RHO = 0, CDNS_ST_RHOU, CDNS_ST_RHOV, CDNS_ST_RHOW, CDNS_ST_RHOUU,
       CDNS_ST_RHOVV, CDNS_ST_RHOWW, CDNS_ST_RHOUV, CDNS_ST_U, CDNS_ST_UU, CDNS_ST_T,
       CDNS_ST_RHOT, CDNS_ST_TT, CDNS_ST_P, CDNS_ST_PP, CDNS_ST_RHORHO, CDNS_NSTAT };
cdns_status cdns_stats_accumulate(cdns_ctx* ctx);
cdns_status cdns_stats_export(cdns_ctx* ctx, double* host_out, int64_t* samples);
cdns_status cdns_stats_reset(cdns_ctx* ctx);

/* Mean fields of the accumulated statistics, written on the device to
 * out_dev [CDNS_NMEAN][ny][nx], or [CDNS_NMEAN][ny] with average_x != 0
 * (the x sums taken i ascending); asynchronous.  With m the sums divided by
 * samples * nz (* nx): Reynolds mean density, Favre mean velocities
 * m(rho u_i)/rho, Favre stresses m(rho u_i u_j)/rho - u~_i u~_j for ij = 11,
 * 22, 33, 12, the Reynolds mean u and its rms, mean T, Favre mean T
 * m(rho T)/rho, rms of T, mean p and its rms, rms of rho (each rms from the
 * second moment, clipped at zero).  CDNS_EINVAL when no sample was
 * accumulated. */
enum { CDNS_MN_RHO = 0, CDNS_MN_U_FAVRE, CDNS_MN_V_FAVRE, CDNS_MN_W_FAVRE, CDNS_MN_R11,
       CDNS_MN_R22, CDNS_MN_R33, CDNS_MN_R12, CDNS_MN_U, CDNS_MN_U_RMS, CDNS_MN_T,
       CDNS_MN_T_FAVRE, CDNS_MN_T_RMS, CDNS_MN_P, CDNS_MN_P_RMS, CDNS_MN_RHO_RMS, CDNS_NMEAN };
cdns_status cdns_stats_means(cdns_ctx* ctx, int32_t average_x, double* out_dev);

/* Test hooks: node sensor value theta, node flags and interface flags
 * (bit d: interface i+1/2 in direction d is shock-capturing) of the last
 * right-hand side evaluated by cdns_rhs (device arrays [nz][ny][nx]).
 * theta_dev may be NULL. */
cdns_status cdns_export_sensor(cdns_ctx* ctx, double* theta_dev, uint8_t* nflags_dev,
                               uint8_t* iflags_dev);

/* Test hooks for the sensor switch (eq. sensor): cdns_export_flags copies
 * the node flags (theta > theta*) of the last cdns_rhs into the device
 * array flags_dev [nz][ny][nx] (bytes 0/1); cdns_import_flags copies such a
 * mask in and makes the next cdns_rhs use it instead of evaluating the
 * sensor (hybrid mode only, CDNS_EINVAL otherwise; the interface flags and
 * lists are rebuilt from it; theta is not recomputed; stepping calls
 * always evaluate the sensor and drop a pending import).  For comparing runs whose sensor decisions
 * differ only where theta is within round-off of the threshold. */
cdns_status cdns_export_flags(cdns_ctx* ctx, uint8_t* flags_dev);
cdns_status cdns_import_flags(cdns_ctx* ctx, const uint8_t* flags_dev);

/* Test hook: shock-capturing interface fluxes of direction dir (0..2) from
 * the last cdns_rhs, interface i+1/2 at node i, layout [5][nz][ny][nx]
 * (device); entries of interfaces that were not flagged are undefined. */
cdns_status cdns_export_iface_flux(cdns_ctx* ctx, int32_t dir, double* out_dev);

/* Profiling hook: nsteps RK3 steps launched kernel by kernel, with a pair
 * of HIP events recorded on the context's stream around every phase.
 * ms_out[CDNS_NPHASES] receives the mean duration (ms) of one launch of
 * each phase, launches_out[CDNS_NPHASES] (may be NULL) the number of
 * launches timed, weno_ifaces_out (may be NULL) the total number of
 * shock-capturing interfaces (all directions) processed by the timed WENO
 * launches.  Where the update runs inside the right-hand-side kernel (see
 * cdns_rk_step), CDNS_PH_RHS covers both and CDNS_PH_RK times only the
 * completion of a forced update; where the first stage's sensor reduces
 * the time-step bounds, CDNS_PH_SENSOR covers both and CDNS_PH_DT has no
 * launches.
 * Advances the state like cdns_rk_step; synchronises. */
enum { CDNS_PH_DT = 0, CDNS_PH_GHOSTS, CDNS_PH_SENSOR, CDNS_PH_IFLAGS, CDNS_PH_WENO,
       CDNS_PH_RHS, CDNS_PH_FORCE, CDNS_PH_RK, CDNS_NPHASES };
cdns_status cdns_time_phases(cdns_ctx* ctx, int32_t nsteps, double cfl, double dt_fixed,
                             double* ms_out, int32_t* launches_out, int64_t* weno_ifaces_out);

/* Last error message of the context (valid until the next call on it). */
const char* cdns_last_error(const cdns_ctx* ctx);

/* Destroy the context (does not free caller memory). */
cdns_status cdns_destroy(cdns_ctx* ctx);

/* ---------------------------------------------------------------- batching
 * Many independent instances advanced together: every stage phase is one
 * kernel launch over a device work table of (instance, tile) items for all
 * attached instances; the stage sequence is captured once as a HIP graph
 * and replayed, membership changes only rewrite the table.  Each instance
 * keeps its own time step, forcing and reductions (fixed order per
 * instance), so its results do not depend on what else is attached. */
cdns_status cdns_batch_create(int32_t max_slots, void* workspace_dev, size_t workspace_bytes,
                              void* hip_stream, cdns_batch** out);
size_t cdns_batch_workspace_bytes(int32_t max_slots);
/* Attach a context (its tile shape and precision must match the batch's);
 * *slot receives its slot.  CDNS_EBUSY: already attached or no free slot;
 * CDNS_EUNSUP: the context uses digital-filter inflow or scheme orders
 * other than the defaults. */
cdns_status cdns_batch_attach(cdns_batch* b, cdns_ctx* ctx, int32_t* slot);
cdns_status cdns_batch_detach(cdns_batch* b, int32_t slot);
/* nsteps RK3 steps of every attached instance; each uses its own cfl /
 * dt_fixed as given to cdns_batch_set_step. */
cdns_status cdns_batch_set_step(cdns_batch* b, int32_t slot, double cfl, double dt_fixed);
cdns_status cdns_batch_step(cdns_batch* b, int32_t nsteps);
cdns_status cdns_batch_destroy(cdns_batch* b);

/* Library version string. */
const char* cdns_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CDNS_H */
