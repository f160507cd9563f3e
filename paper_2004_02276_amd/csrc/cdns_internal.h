// cdns_internal.h -- device descriptor of one solver instance and the host
// launchers of the HIP kernels (library-internal, not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cdns {

constexpr int kHalo = 4;          // ghost planes stored (WENO7 stencil i-3..i+4); Desc::hw
                                  // of them are filled, as many as the stencils reach
constexpr int kRedBlocks = 1024;  // partial-sum slots of the generic reductions

// Boundary kinds (same values as the C ABI).
enum { BC_PERIODIC = 0, BC_WALL_ISO = 1, BC_WALL_ADIA = 2, BC_DIRICHLET = 3,
       BC_OUTFLOW = 4, BC_SHOCK_TOP = 5, BC_DF_INFLOW = 6 };

// Device status bits.
enum { ST_BAD_STATE = 1u, ST_BAD_GHOST = 2u };

// Scalar slots in Desc::scal.
enum { SC_DT = 0, SC_FORCE = 1, SC_TIME = 2, SC_STEP = 3, SC_WACC = 4, SC_COUNT = 8 };

// Diagnostics slots in Desc::diag.
enum { DG_MASS = 0, DG_MX, DG_MY, DG_MZ, DG_E, DG_K, DG_RHOMIN, DG_PMIN, DG_MACHMAX,
       DG_NONFINITE, DG_COUNT = 16 };

// Everything a kernel needs about one instance.  Passed by value as a kernel
// argument for single-instance launches and stored in a device array for
// batched launches.
struct Desc {
  int nx, ny, nz, nxg;            // nxg = nx + 2*kHalo (row length of y ghost planes)
  long long N;                    // nx*ny*nz
  double rnx, rny;                // 1/nx, 1/ny (node index decomposition)
  double dx, dz, deta;
  double idx, idz, ideta, idx2, idz2, ideta2;
  const double* y_eta;            // [ny]
  const double* y_etaeta;         // [ny]
  const double* iy;               // [ny] 1/(deta*y_eta)
  const double* iye2;             // [ny] 1/y_eta^2
  double gamma, gm1, R, cv, icv, cp, Pr, mu_ref, iTref, S, muc, kfac;
  double theta_star, eps_s, vol_den;
  double vfac;                    // max(4/3, gamma/Pr) for the viscous time-step bound
  double rho2;                    // largest |symbol| of the second derivative in use
  int cl, wr, hw;                 // central half-width L (order 2L), WENO stencils r
                                  // (order 2r-1), ghost layers filled max(2, L, r)
  int viscous, sensor_mode, forcing, precision;
  int per_x, per_y;
  int bc[6];
  const double* bcp[6];
  int wall_lo, wall_hi;
  // stage buffers: index 0..2 = RK stages, 3 = standalone right-hand side
  const double* win[4];
  double* wout[4];
  double* rcur[4];
  const double* rprev[4];
  // work arrays
  uint8_t* nflag;                 // [N]
  int* slot[3];                   // [N] per direction: position of interface i+1/2 in the
                                  // direction's list if it is shock-capturing, else -1
  double* theta;                  // [N] optional sensor export (may be null)
  double* Fw[3];                  // [5][N] shock-capturing interface fluxes per direction,
                                  // compacted: entry e belongs to node list[d][e]
  int* list[3];                   // [N] compacted interface lists per direction
  unsigned* count;                // [4] list lengths
  double* gx[2];                  // [5][kHalo][nz][ny] x-face ghost planes
  double* stats;                  // [NSTAT][ny][nx] spanwise sums of the running statistics
  double* dfpsi;                  // [3][nz][ny] filtered inflow field (digital filter)
  double* dffy;                   // [3][nz][ny] inflow deviates filtered along y
  double* gy[2];                  // [5][kHalo][nz][nxg] y-face ghost planes
  double* part;                   // [npart] right-hand-side block partial sums (forcing)
  int npart;
  double* red;                    // [2*kRedBlocks] generic reduction partials
  double* redd;                   // [DG_COUNT*kRedBlocks] diagnostics partials
  double* scal;                   // [SC_COUNT]
  unsigned* status;               // [1]
  unsigned long long* dtmax;      // [2] largest convective and viscous time-step bounds of
                                  // the step as ordered bit patterns (non-negative doubles),
                                  // zero between steps
  double* diag;                   // [DG_COUNT]
  // launch geometry of the fused right-hand-side kernel
  int tile_x, tile_y, kz, tiles_x, tiles_y, zchunks;
  // stepping
  double cfl, dt_fixed;
};

// Host launchers (cdns_kernels.hip).  All enqueue on `st`.
hipError_t launch_stage_begin(const Desc& D, hipStream_t st);
bool ghosts_needed(const Desc& D);  // does launch_ghosts launch anything
hipError_t launch_ghosts(const Desc& D, int stage, hipStream_t st);
// with_dt: the first stage of a step, whose sensor also reduces the time-step
// bounds (dt_in_sensor(D)); the stage's launch_iflags(set_dt) then sets the
// step (they replace launch_dt)
hipError_t launch_sensor(const Desc& D, int stage, bool export_theta, hipStream_t st,
                         bool with_dt = false);
bool dt_in_sensor(const Desc& D);
// set_dt: also set the step's time step from the first stage's sensor maxima
hipError_t launch_iflags(const Desc& D, hipStream_t st, bool set_dt = false);
hipError_t launch_weno(const Desc& D, int stage, hipStream_t st);
// fuse_rk: the RK update of the stage in the same pass (rk_fused(D) only)
hipError_t launch_rhs(const Desc& D, int stage, hipStream_t st, bool fuse_rk = false);
bool rk_fused(const Desc& D);
// completion of a fused update under bulk forcing (after launch_force)
hipError_t launch_rk_forced(const Desc& D, int stage, hipStream_t st);
hipError_t launch_force(const Desc& D, hipStream_t st);
hipError_t launch_apply_force(const Desc& D, int stage, hipStream_t st);
hipError_t launch_rk(const Desc& D, int stage, hipStream_t st);
hipError_t launch_dt(const Desc& D, hipStream_t st);
hipError_t launch_diag(const Desc& D, hipStream_t st);
// No-allocation diagnostics: partials in a static per-device array of
// kNoallocBlocks * DG_COUNT doubles (one block per kNoallocPoints points,
// so grids of at most kNoallocBlocks * kNoallocPoints points).
constexpr int kMaxDevices = 64;
constexpr int kNoallocBlocks = 8192;
constexpr long long kNoallocPoints = 4096;
hipError_t noalloc_scratch(int dev, double** out);  // device address of the array on dev
long long noalloc_diag_blocks(long long N);
hipError_t launch_diag_noalloc(const Desc& D, const double* w, double* part, double* out,
                               int nout, hipStream_t st);
hipError_t launch_export_iflags(const Desc& D, uint8_t* out, hipStream_t st);
hipError_t launch_count_iface(const Desc& D, bool reset, hipStream_t st);  // scal[SC_WACC]
// digital-filter inflow: the initial plane (key 0), or the update at the
// start of the current step (key = scal[SC_STEP], dt = scal[SC_DT])
hipError_t launch_df(const Desc& D, bool initial, hipStream_t st);
constexpr int kNStat = 16;  // running-statistics products (CDNS_NSTAT)
hipError_t launch_stats(const Desc& D, hipStream_t st);
// mean fields [kNStat][ny][nx] (or [kNStat][ny] averaged along x) from the
// accumulated sums, count = samples * nz (* nx when averaged)
hipError_t launch_stats_means(const Desc& D, bool avg, double count, double* out, hipStream_t st);
hipError_t launch_export_iface(const Desc& D, int dir, double* out, hipStream_t st);
bool rhs_tile_supported(int tx, int ty);
int rhs_blocks(const Desc& D);

// ---------------------------------------------------------------- batching
// Work table of a batch: the active instances (indices into the device
// descriptor array) and, per phase kind, prefix sums of the number of work
// items (blocks) of each active instance.  Persistent kernels walk the
// flattened item range with a grid stride and locate the instance by a
// search over the prefix sums, so membership changes rewrite this table only.
constexpr int kMaxSlots = 64;
enum { WK_PTS = 0, WK_RHS, WK_GX, WK_GY, WK_DT, WK_IFL, WK_SEN, WK_RK, WK_COUNT };
struct BatchTable {
  int ninst;
  int inst[kMaxSlots];
  int pre[WK_COUNT][kMaxSlots + 1];
};
enum { BPH_BEGIN = 0, BPH_DT_PART, BPH_DT_FINAL, BPH_GHOST_X, BPH_GHOST_Y, BPH_SENSOR, BPH_IFLAGS,
       BPH_WENO, BPH_RHS, BPH_FORCE, BPH_RK };
// Items of one instance per work kind (blocks of the single-instance kernels).
int batch_items(const Desc& D, int kind);
hipError_t launch_batch_phase(int phase, const Desc* descs_dev, const BatchTable* tab_dev,
                              int stage, int tile_x, int tile_y, int precision, hipStream_t st);

}  // namespace cdns
