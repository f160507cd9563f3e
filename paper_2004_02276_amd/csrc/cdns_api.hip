// cdns_api.hip -- host side of the C ABI declared in include/cdns.h:
// argument validation, workspace carving, stage sequencing, HIP graph
// capture of whole RK steps, diagnostics and the batched runner.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cdns.h"
#include "cdns_internal.h"

using cdns::Desc;

struct cdns_ctx {
  Desc D;
  hipStream_t stream = nullptr;     // caller's stream (work is enqueued here)
  hipStream_t cap = nullptr;        // private stream used only for graph capture
  std::string err;
  int precision = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<double> h_yeta, h_yetaeta, h_iy, h_iye2;
  std::vector<double> h_bcp[6];
  double* bcp_dev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  size_t bcp_cap = 0;
  size_t part_cap = 0;
  hipGraphExec_t gexec = nullptr;
  double g_cfl = -1.0, g_dt = -1.0;
  bool last_rhs_valid = false;
  bool flags_imported = false;        // next cdns_rhs uses the imported node flags
  int batch_refs = 0;
  int64_t stat_samples = 0;           // samples in the statistics accumulator
  int device = 0;                     // device current at creation
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t metric, bcp, w1, w2, ra, rb, nflag, slot, theta, fw, list, count, sync, gx, gy, df, stats, part, red,
      redd, scal, status, diag, total;
  size_t bcp_cap, part_cap;
};

bool grid_ok(const cdns_grid* g) {
  return g && g->nx >= 4 && g->ny >= 4 && g->nz >= 4 && g->lx > 0 && g->lz > 0 && g->y_eta &&
         g->y_etaeta && (long long)g->nx * g->ny * g->nz < (1LL << 31);
}

Layout layout_of(const cdns_grid* g) {
  Layout L{};
  const size_t nx = g->nx, ny = g->ny, nz = g->nz;
  const size_t N = nx * ny * nz;
  const size_t nxg = nx + 2 * cdns::kHalo;
  // largest parameter set: the digital-filter inflow, 4 + (2 Ny + 1) +
  // (2 Nz + 1) + 11 ny values with filter half-widths Ny <= ny, Nz <= nz
  L.bcp_cap = std::max<size_t>(16, 5 * std::max(nx, ny));
  L.bcp_cap = std::max<size_t>(L.bcp_cap, 6 + 13 * ny + 2 * nz);
  // largest number of fused-kernel blocks over the compiled tile shapes (kz >= 1)
  L.part_cap = ((nx + 31) / 32) * ((ny + 1) / 2) * nz;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.metric = take(4 * ny * sizeof(double));
  L.bcp = take(6 * L.bcp_cap * sizeof(double));
  L.w1 = take(5 * N * sizeof(double));
  L.w2 = take(5 * N * sizeof(double));
  L.ra = take(5 * N * sizeof(double));
  L.rb = take(5 * N * sizeof(double));
  L.nflag = take(N);
  L.slot = take(3 * N * sizeof(int));
  L.theta = take(N * sizeof(double));
  L.fw = take(3 * 5 * N * sizeof(double));
  L.list = take(3 * N * sizeof(int));
  L.count = take(4 * sizeof(unsigned));
  L.sync = take(4 * sizeof(unsigned long long));
  L.gx = take(2 * 5 * cdns::kHalo * nz * ny * sizeof(double));
  L.gy = take(2 * 5 * cdns::kHalo * nz * nxg * sizeof(double));
  L.df = take(2 * 3 * nz * ny * sizeof(double));
  L.stats = take((size_t)cdns::kNStat * ny * nx * sizeof(double));
  L.part = take(L.part_cap * sizeof(double));
  L.red = take(2 * cdns::kRedBlocks * sizeof(double));
  L.redd = take((size_t)cdns::DG_COUNT * cdns::kRedBlocks * sizeof(double));
  L.scal = take(cdns::SC_COUNT * sizeof(double));
  L.status = take(sizeof(unsigned) * 4);
  L.diag = take(cdns::DG_COUNT * sizeof(double));
  L.total = o;
  return L;
}

cdns_status fail(cdns_ctx* c, cdns_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

cdns_status hip_fail(cdns_ctx* c, hipError_t e, const char* what) {
  return fail(c, CDNS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void invalidate_graph(cdns_ctx* c) {
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
}

void set_tiling_desc(Desc& D, int tx, int ty, int kz) {
  D.tile_x = tx;
  D.tile_y = ty;
  D.kz = kz < 1 ? 1 : (kz > D.nz ? D.nz : kz);
  D.tiles_x = (D.nx + tx - 1) / tx;
  D.tiles_y = (D.ny + ty - 1) / ty;
  D.zchunks = (D.nz + D.kz - 1) / D.kz;
  D.npart = D.tiles_x * D.tiles_y * D.zchunks;
}

// Scheme orders: central half-width L (order 2L), WENO stencils r (order
// 2r-1); ghost layers in use max(2, L, r) (the sensor reaches two); the
// largest |symbol| of the order-2L second derivative for the time step.
void set_orders(Desc& D, int L, int r) {
  D.cl = L;
  D.wr = r;
  D.hw = std::max(2, std::max(L, r));
  D.rho2 = L == 1 ? 4.0 : (L == 2 ? 16.0 / 3.0 : 272.0 / 45.0);
}

// Default tiling: enough blocks to give each of the 256 CUs two.
void default_tiling(Desc& D) {
  int tx = 64, ty = 4;
  int kz = 32;  // deep z chunks amortise the 4-plane pipeline start
  long long tiles = (long long)((D.nx + tx - 1) / tx) * ((D.ny + ty - 1) / ty);
  while (kz > 4 && tiles * ((D.nz + kz - 1) / kz) < 512) kz /= 2;
  set_tiling_desc(D, tx, ty, kz);
}

// Enqueue the right-hand-side phases of one stage (ghosts .. forcing sum).
// keep_flags: use the node flags already in place (imported) instead of
// running the sensor.
// with_dt: the sensor also reduces the step's time-step bounds and the flag
// kernel sets the step (first stage of a step, dt_in_sensor(D)).
hipError_t enqueue_rhs_phases(const Desc& D, int stage, bool export_theta, hipStream_t st,
                              bool keep_flags = false, bool fuse_rk = false,
                              bool with_dt = false) {
  hipError_t e;
  // list counters: reset by the sensor kernel in hybrid mode, else here
  if ((D.sensor_mode == 2 || keep_flags) && (e = cdns::launch_stage_begin(D, st)) != hipSuccess)
    return e;
  if ((e = cdns::launch_ghosts(D, stage, st)) != hipSuccess) return e;
  if (D.sensor_mode == 1 && !keep_flags &&
      (e = cdns::launch_sensor(D, stage, export_theta, st, with_dt)) != hipSuccess)
    return e;
  if (D.sensor_mode > 0) {
    if ((e = cdns::launch_iflags(D, st, with_dt)) != hipSuccess) return e;
    if ((e = cdns::launch_weno(D, stage, st)) != hipSuccess) return e;
  }
  if ((e = cdns::launch_rhs(D, stage, st, fuse_rk)) != hipSuccess) return e;
  if (D.forcing && (e = cdns::launch_force(D, st)) != hipSuccess) return e;
  return hipSuccess;
}

// One RK step; the time step is reduced by the first stage's sensor, or by
// its own kernels.
hipError_t enqueue_step(const Desc& D, hipStream_t st) {
  hipError_t e;
  const bool dt_sen = cdns::dt_in_sensor(D);
  if (!dt_sen && (e = cdns::launch_dt(D, st)) != hipSuccess) return e;
  // inflow plane of this step (needs the step's dt and counter)
  if (D.bc[0] == cdns::BC_DF_INFLOW && (e = cdns::launch_df(D, false, st)) != hipSuccess) return e;
  const bool fuse = cdns::rk_fused(D);  // update inside the right-hand-side pass
  for (int stage = 0; stage < 3; ++stage) {
    if ((e = enqueue_rhs_phases(D, stage, false, st, false, fuse, dt_sen && stage == 0)) !=
        hipSuccess)
      return e;
    if (!fuse) e = cdns::launch_rk(D, stage, st);
    else if (D.forcing) e = cdns::launch_rk_forced(D, stage, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

const char* cdns_version(void) { return "cdns 0.1 (gfx950)"; }

size_t cdns_workspace_bytes(const cdns_grid* grid, int32_t precision) {
  if (!grid_ok(grid) || (precision != CDNS_FP64 && precision != CDNS_FP32_FLUX)) return 0;
  return layout_of(grid).total;
}

cdns_status cdns_create(const cdns_grid* grid, const cdns_phys* phys, int32_t precision,
                        double* state_dev, void* workspace_dev, size_t workspace_bytes,
                        void* hip_stream, cdns_ctx** out) {
  if (!out) return CDNS_EINVAL;
  *out = nullptr;
  if (!grid_ok(grid) || !phys || !state_dev || !workspace_dev) return CDNS_EINVAL;
  if (precision != CDNS_FP64 && precision != CDNS_FP32_FLUX) return CDNS_EINVAL;
  if (!(phys->gamma > 1.0) || !(phys->R_gas > 0.0) || !(phys->Pr > 0.0) || !(phys->T_ref > 0.0) ||
      !(phys->mu_ref >= 0.0) || !(phys->S_suth >= 0.0) || phys->sensor_mode < 0 ||
      phys->sensor_mode > 2 || !(phys->sensor_eps >= 0.0))
    return CDNS_EINVAL;
  if (((uintptr_t)workspace_dev) % kAlign != 0) return CDNS_EINVAL;
  Layout L = layout_of(grid);
  if (workspace_bytes < L.total) return CDNS_ENOMEM;
  for (int j = 0; j < grid->ny; ++j)
    if (!(grid->y_eta[j] > 0.0)) return CDNS_EINVAL;

  cdns_ctx* c = new cdns_ctx();
  c->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
  c->precision = precision;
  c->ws = (char*)workspace_dev;
  c->ws_bytes = workspace_bytes;
  c->bcp_cap = L.bcp_cap;
  c->part_cap = L.part_cap;
  Desc& D = c->D;
  std::memset(&D, 0, sizeof(D));
  const int nx = grid->nx, ny = grid->ny, nz = grid->nz;
  D.nx = nx; D.ny = ny; D.nz = nz;
  D.nxg = nx + 2 * cdns::kHalo;
  D.N = (long long)nx * ny * nz;
  D.rnx = 1.0 / nx;
  D.rny = 1.0 / ny;
  D.dx = grid->lx / nx;
  D.dz = grid->lz / nz;
  D.deta = 1.0 / ny;
  D.idx = 1.0 / D.dx;
  D.idz = 1.0 / D.dz;
  D.ideta = 1.0 / D.deta;
  D.idx2 = D.idx * D.idx;
  D.idz2 = D.idz * D.idz;
  D.ideta2 = D.ideta * D.ideta;
  c->h_yeta.assign(grid->y_eta, grid->y_eta + ny);
  c->h_yetaeta.assign(grid->y_etaeta, grid->y_etaeta + ny);
  c->h_iy.resize(ny);
  c->h_iye2.resize(ny);
  double ysum = 0.0;
  for (int j = 0; j < ny; ++j) {
    c->h_iy[j] = 1.0 / (D.deta * c->h_yeta[j]);
    c->h_iye2[j] = 1.0 / (c->h_yeta[j] * c->h_yeta[j]);
    ysum += c->h_yeta[j];
  }
  D.vol_den = ysum * (double)nx * (double)nz;
  D.gamma = phys->gamma;
  D.gm1 = phys->gamma - 1.0;
  D.R = phys->R_gas;
  D.cv = phys->R_gas / (phys->gamma - 1.0);
  D.icv = 1.0 / D.cv;
  D.cp = phys->gamma * phys->R_gas / (phys->gamma - 1.0);
  D.Pr = phys->Pr;
  D.mu_ref = phys->mu_ref;
  D.iTref = 1.0 / phys->T_ref;
  D.S = phys->S_suth;
  D.muc = phys->mu_ref * (1.0 + phys->S_suth);
  D.kfac = D.cp / phys->Pr;
  D.vfac = std::max(4.0 / 3.0, phys->gamma / phys->Pr);
  set_orders(D, 2, 3);
  D.theta_star = phys->theta_star;
  D.eps_s = phys->sensor_eps;
  D.viscous = phys->viscous ? 1 : 0;
  D.sensor_mode = phys->sensor_mode;
  D.forcing = phys->forcing ? 1 : 0;
  D.precision = precision;
  D.per_x = 1;
  D.per_y = 1;
  for (int f = 0; f < 6; ++f) D.bc[f] = cdns::BC_PERIODIC;

  char* ws = c->ws;
  double* metric = (double*)(ws + L.metric);
  D.y_eta = metric;
  D.y_etaeta = metric + ny;
  D.iy = metric + 2 * ny;
  D.iye2 = metric + 3 * ny;
  for (int f = 0; f < 6; ++f) {
    c->bcp_dev[f] = (double*)(ws + L.bcp) + (size_t)f * L.bcp_cap;
    D.bcp[f] = c->bcp_dev[f];
  }
  double* w1 = (double*)(ws + L.w1);
  double* w2 = (double*)(ws + L.w2);
  double* ra = (double*)(ws + L.ra);
  double* rb = (double*)(ws + L.rb);
  D.win[0] = state_dev; D.wout[0] = w1; D.rcur[0] = ra; D.rprev[0] = nullptr;
  D.win[1] = w1; D.wout[1] = w2; D.rcur[1] = rb; D.rprev[1] = ra;
  D.win[2] = w2; D.wout[2] = state_dev; D.rcur[2] = ra; D.rprev[2] = rb;
  D.win[3] = state_dev; D.wout[3] = nullptr; D.rcur[3] = ra; D.rprev[3] = nullptr;
  D.nflag = (uint8_t*)(ws + L.nflag);
  D.theta = (double*)(ws + L.theta);
  for (int d = 0; d < 3; ++d) {
    D.Fw[d] = (double*)(ws + L.fw) + (size_t)d * 5 * D.N;
    D.list[d] = (int*)(ws + L.list) + (size_t)d * D.N;
    D.slot[d] = (int*)(ws + L.slot) + (size_t)d * D.N;
  }
  D.count = (unsigned*)(ws + L.count);
  D.dtmax = (unsigned long long*)(ws + L.sync);
  const size_t gxs = (size_t)5 * cdns::kHalo * nz * ny;
  const size_t gys = (size_t)5 * cdns::kHalo * nz * D.nxg;
  D.gx[0] = (double*)(ws + L.gx);
  D.gx[1] = D.gx[0] + gxs;
  D.stats = (double*)(ws + L.stats);
  D.dfpsi = (double*)(ws + L.df);
  D.dffy = D.dfpsi + (size_t)3 * nz * ny;
  D.gy[0] = (double*)(ws + L.gy);
  D.gy[1] = D.gy[0] + gys;
  D.part = (double*)(ws + L.part);
  D.red = (double*)(ws + L.red);
  D.redd = (double*)(ws + L.redd);
  D.scal = (double*)(ws + L.scal);
  D.status = (unsigned*)(ws + L.status);
  D.diag = (double*)(ws + L.diag);
  default_tiling(D);
  D.cfl = 0.8;
  D.dt_fixed = 0.0;

  hipError_t e;
  if ((e = hipMemcpyAsync(metric, c->h_yeta.data(), ny * sizeof(double), hipMemcpyHostToDevice,
                          c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(metric + ny, c->h_yetaeta.data(), ny * sizeof(double),
                          hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(metric + 2 * ny, c->h_iy.data(), ny * sizeof(double),
                          hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(metric + 3 * ny, c->h_iye2.data(), ny * sizeof(double),
                          hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
      (e = hipMemsetAsync(ws + L.count, 0, align_up(4 * sizeof(unsigned)), c->stream)) != hipSuccess ||
      (e = hipMemsetAsync(ws + L.sync, 0, 4 * sizeof(unsigned long long), c->stream)) != hipSuccess ||
      (e = hipMemsetAsync(ws + L.scal, 0, cdns::SC_COUNT * sizeof(double), c->stream)) != hipSuccess ||
      (e = hipMemsetAsync(ws + L.status, 0, 4 * sizeof(unsigned), c->stream)) != hipSuccess ||
      (e = hipMemsetAsync(ws + L.slot, 0xFF, 3 * D.N * sizeof(int), c->stream)) != hipSuccess ||
      (e = hipMemsetAsync(ws + L.nflag, 0, D.N, c->stream)) != hipSuccess ||
      (e = hipMemsetAsync(ws + L.stats, 0, (size_t)cdns::kNStat * ny * nx * sizeof(double),
                          c->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(c->stream)) != hipSuccess) {
    delete c;
    return CDNS_EHIP;
  }
  if ((e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking)) != hipSuccess) {
    delete c;
    return CDNS_EHIP;
  }
  *out = c;
  return CDNS_OK;
}

// Digital-filter inflow (Sec. 3.2): half-width of the Gaussian filter of a
// length of n grid spacings, N = max(1, ceil(2 n)).
static int df_half_width(double n) {
  const double N = std::ceil(2.0 * n);
  return N < 1.0 ? 1 : (N > 1e9 ? 1000000000 : (int)N);
}

// Expands the caller's parameters [n_y, n_z, T, seed, mean[5][ny],
// R11, R22, R33, R12, R13, R23 [6][ny]] into the block the generator
// kernels read: [N_y, N_z, T, seed, b_y[2N_y+1], b_z[2N_z+1], mean[5][ny],
// a11, a21, a22, a31, a32, a33 [6][ny]] with the Gaussian coefficients
// b_l ~ exp(-pi l^2/(2 n^2)) of unit sum of squares and the lower triangular
// factor a a^T = R of the stresses (Lund's transformation; a zero diagonal
// entry zeroes the column below it).
static void df_derive(int ny, const double* p, std::vector<double>& out) {
  const int Ny = df_half_width(p[0]), Nz = df_half_width(p[1]);
  out.assign(4 + (2 * (size_t)Ny + 1) + (2 * (size_t)Nz + 1) + 11 * (size_t)ny, 0.0);
  out[0] = Ny;
  out[1] = Nz;
  out[2] = p[2];
  out[3] = p[3];
  double* b = out.data() + 4;
  for (int f = 0; f < 2; ++f) {
    const double n = p[f];
    const int N = f == 0 ? Ny : Nz;
    double ss = 0.0;
    for (int l = -N; l <= N; ++l) {
      b[l + N] = std::exp(-M_PI * (double)l * (double)l / (2.0 * n * n));
      ss += b[l + N] * b[l + N];
    }
    const double inv = 1.0 / std::sqrt(ss);
    for (int l = 0; l <= 2 * N; ++l) b[l] *= inv;
    b += 2 * N + 1;
  }
  std::memcpy(b, p + 4, 5 * (size_t)ny * sizeof(double));
  double* a = b + 5 * (size_t)ny;
  const double* R = p + 4 + 5 * (size_t)ny;
  for (int j = 0; j < ny; ++j) {
    const double r11 = R[j], r22 = R[ny + j], r33 = R[2 * ny + j];
    const double r12 = R[3 * ny + j], r13 = R[4 * ny + j], r23 = R[5 * ny + j];
    const double a11 = std::sqrt(std::fmax(r11, 0.0));
    const double a21 = a11 > 0.0 ? r12 / a11 : 0.0;
    const double a31 = a11 > 0.0 ? r13 / a11 : 0.0;
    const double a22 = std::sqrt(std::fmax(r22 - a21 * a21, 0.0));
    const double a32 = a22 > 0.0 ? (r23 - a21 * a31) / a22 : 0.0;
    const double a33 = std::sqrt(std::fmax(r33 - a31 * a31 - a32 * a32, 0.0));
    a[j] = a11;
    a[ny + j] = a21;
    a[2 * ny + j] = a22;
    a[3 * ny + j] = a31;
    a[4 * ny + j] = a32;
    a[5 * ny + j] = a33;
  }
}

cdns_status cdns_poison_workspace(cdns_ctx* c) {
  if (!c) return CDNS_EINVAL;
  if (c->batch_refs > 0) return fail(c, CDNS_EBUSY, "context attached to a batch");
  const Desc& D = c->D;
  cdns_grid g{};
  g.nx = D.nx;
  g.ny = D.ny;
  g.nz = D.nz;
  const Layout L = layout_of(&g);
  // every double-precision work region the stepping path must write before
  // it reads (0xFF bytes are a NaN in every double)
  const size_t N = (size_t)D.N, nz = D.nz, ny = D.ny;
  const size_t regions[][2] = {
      {L.w1, 5 * N * sizeof(double)},
      {L.w2, 5 * N * sizeof(double)},
      {L.ra, 5 * N * sizeof(double)},
      {L.rb, 5 * N * sizeof(double)},
      {L.theta, N * sizeof(double)},
      {L.fw, 3 * 5 * N * sizeof(double)},
      {L.gx, 2 * 5 * cdns::kHalo * nz * ny * sizeof(double)},
      {L.gy, 2 * 5 * cdns::kHalo * nz * (size_t)D.nxg * sizeof(double)},
      {L.df, 2 * 3 * nz * ny * sizeof(double)},
      {L.part, L.part_cap * sizeof(double)},
      {L.red, 2 * cdns::kRedBlocks * sizeof(double)},
      {L.redd, (size_t)cdns::DG_COUNT * cdns::kRedBlocks * sizeof(double)},
      {L.diag, cdns::DG_COUNT * sizeof(double)}};
  hipError_t e = hipSuccess;
  for (const auto& r : regions)
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + r[0], 0xFF, r[1], c->stream);
  // the inflow generator's state is set up with the boundary: again
  if (e == hipSuccess && D.bc[0] == cdns::BC_DF_INFLOW) e = cdns::launch_df(D, true, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "workspace poisoning");
  c->last_rhs_valid = false;
  invalidate_graph(c);
  return CDNS_OK;
}

cdns_status cdns_set_bc(cdns_ctx* c, int32_t face, int32_t kind, const double* params,
                        int64_t nparams) {
  if (!c) return CDNS_EINVAL;
  if (c->batch_refs > 0) return fail(c, CDNS_EBUSY, "context attached to a batch");
  if (face < 0 || face > 5) return fail(c, CDNS_EINVAL, "face out of range");
  if (kind < 0 || kind > 6) return fail(c, CDNS_EINVAL, "unknown boundary kind");
  if (nparams < 0 || (nparams > 0 && !params)) return fail(c, CDNS_EINVAL, "bad parameters");
  const int ax = face / 2;
  Desc& D = c->D;
  if (kind != cdns::BC_PERIODIC) {
    if (ax == 2) return fail(c, CDNS_EUNSUP, "z faces must be periodic");
    if (ax == 0 && !(kind == cdns::BC_DIRICHLET || kind == cdns::BC_OUTFLOW ||
                     (kind == cdns::BC_DF_INFLOW && face == 0)))
      return fail(c, CDNS_EUNSUP,
                  "x faces accept periodic, Dirichlet, characteristic outflow or (x-) digital-filter inflow");
    if (ax == 1 && !(kind == cdns::BC_WALL_ISO || kind == cdns::BC_WALL_ADIA ||
                     kind == cdns::BC_SHOCK_TOP || kind == cdns::BC_OUTFLOW))
      return fail(c, CDNS_EUNSUP,
                  "y faces accept periodic, walls, an imposed shock state or characteristic outflow");
    if (kind == cdns::BC_DF_INFLOW) {
      if (nparams != 4 + 11LL * D.ny)
        return fail(c, CDNS_EINVAL, "digital-filter inflow needs 4 + 11*ny parameters");
      const double ly = params[0], lz = params[1];
      if (!(ly > 0.0 && df_half_width(ly) <= D.ny && lz > 0.0 && df_half_width(lz) <= D.nz) ||
          !(params[2] > 0.0) || !(params[3] >= 0.0) || params[3] != (double)(uint64_t)params[3])
        return fail(c, CDNS_EINVAL, "digital-filter lengths, time scale or seed invalid");
    }
    if (kind == cdns::BC_DIRICHLET && nparams != 5LL * D.ny)
      return fail(c, CDNS_EINVAL, "Dirichlet profile needs 5*ny values");
    if (kind == cdns::BC_WALL_ISO && (nparams != 1 || !(params[0] > 0.0)))
      return fail(c, CDNS_EINVAL, "isothermal wall needs one positive temperature");
    if (kind == cdns::BC_SHOCK_TOP && nparams != 11)
      return fail(c, CDNS_EINVAL, "shock state needs 11 values");
  }
  std::vector<double> block;
  if (kind == cdns::BC_DF_INFLOW) df_derive(D.ny, params, block);
  else block.assign(params, params + nparams);
  if (block.size() > c->bcp_cap) return fail(c, CDNS_EINVAL, "too many parameters");
  c->h_bcp[face].swap(block);
  if (!c->h_bcp[face].empty()) {
    hipError_t e = hipMemcpyAsync(c->bcp_dev[face], c->h_bcp[face].data(),
                                  c->h_bcp[face].size() * sizeof(double), hipMemcpyHostToDevice,
                                  c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "sync");
  }
  D.bc[face] = kind;
  D.per_x = D.bc[0] == cdns::BC_PERIODIC && D.bc[1] == cdns::BC_PERIODIC;
  D.per_y = D.bc[2] == cdns::BC_PERIODIC && D.bc[3] == cdns::BC_PERIODIC;
  D.wall_lo = D.bc[2] == cdns::BC_WALL_ISO || D.bc[2] == cdns::BC_WALL_ADIA;
  D.wall_hi = D.bc[3] == cdns::BC_WALL_ISO || D.bc[3] == cdns::BC_WALL_ADIA;
  invalidate_graph(c);
  if (kind == cdns::BC_DF_INFLOW) {
    // the initial inflow plane (generator key 0)
    hipError_t e = cdns::launch_df(D, true, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "inflow generator");
  }
  return CDNS_OK;
}

static cdns_status check_bcs(cdns_ctx* c) {
  const Desc& D = c->D;
  for (int a = 0; a < 3; ++a) {
    const bool p0 = D.bc[2 * a] == cdns::BC_PERIODIC, p1 = D.bc[2 * a + 1] == cdns::BC_PERIODIC;
    if (p0 != p1) return fail(c, CDNS_EINVAL, "both faces of an axis must be periodic or neither");
  }
  return CDNS_OK;
}

cdns_status cdns_set_tiling(cdns_ctx* c, int32_t tx, int32_t ty, int32_t kz) {
  if (!c) return CDNS_EINVAL;
  if (c->batch_refs > 0) return fail(c, CDNS_EBUSY, "context attached to a batch");
  if (!cdns::rhs_tile_supported(tx, ty) || kz < 1)
    return fail(c, CDNS_EINVAL, "unsupported tile shape");
  if (c->D.cl != 2 && (tx != 64 || ty != 4))
    return fail(c, CDNS_EUNSUP, "central orders other than 4 use the 64x4 tile only");
  Desc t = c->D;
  set_tiling_desc(t, tx, ty, kz);
  if ((size_t)t.npart > c->part_cap) return fail(c, CDNS_EINVAL, "too many tiles");
  c->D = t;
  invalidate_graph(c);
  return CDNS_OK;
}

cdns_status cdns_set_scheme(cdns_ctx* c, int32_t central_order, int32_t weno_order) {
  if (!c) return CDNS_EINVAL;
  if (c->batch_refs > 0) return fail(c, CDNS_EBUSY, "context attached to a batch");
  if (central_order != 2 && central_order != 4 && central_order != 6)
    return fail(c, CDNS_EINVAL, "central order must be 2, 4 or 6");
  if (weno_order != 3 && weno_order != 5 && weno_order != 7)
    return fail(c, CDNS_EINVAL, "WENO order must be 3, 5 or 7");
  const int L = central_order / 2, r = (weno_order + 1) / 2;
  if (c->D.nz < 2 * L) return fail(c, CDNS_EINVAL, "nz is below the central stencil width");
  Desc t = c->D;
  set_orders(t, L, r);
  if (L != 2 && (t.tile_x != 64 || t.tile_y != 4)) default_tiling(t);
  c->D = t;
  invalidate_graph(c);
  if (t.bc[0] == cdns::BC_DF_INFLOW) {
    // the ghost layers in use may have changed: the initial plane again
    hipError_t e = cdns::launch_df(t, true, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "inflow generator");
  }
  return CDNS_OK;
}

cdns_status cdns_rhs(cdns_ctx* c, const double* w_dev, double* r_dev) {
  if (!c || !w_dev || !r_dev) return c ? fail(c, CDNS_EINVAL, "null array") : CDNS_EINVAL;
  cdns_status s = check_bcs(c);
  if (s) return s;
  Desc D = c->D;
  D.win[3] = w_dev;
  D.rcur[3] = r_dev;
  const bool keep = c->flags_imported && D.sensor_mode == 1;
  c->flags_imported = false;
  hipError_t e = enqueue_rhs_phases(D, 3, true, c->stream, keep);
  if (e == hipSuccess && D.forcing) e = cdns::launch_apply_force(D, 3, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "rhs launch");
  c->last_rhs_valid = true;
  return CDNS_OK;
}

cdns_status cdns_set_state(cdns_ctx* c, const double* w, int32_t from_host) {
  if (!c || !w) return c ? fail(c, CDNS_EINVAL, "null state") : CDNS_EINVAL;
  const size_t bytes = (size_t)5 * (size_t)c->D.N * sizeof(double);
  hipError_t e = hipMemcpyAsync((void*)c->D.win[0], w, bytes,
                                from_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                                c->stream);
  if (e == hipSuccess && from_host) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "set_state copy");
  return CDNS_OK;
}

cdns_status cdns_get_state(cdns_ctx* c, double* w, int32_t to_host) {
  if (!c || !w) return c ? fail(c, CDNS_EINVAL, "null output") : CDNS_EINVAL;
  const size_t bytes = (size_t)5 * (size_t)c->D.N * sizeof(double);
  hipError_t e = hipMemcpyAsync(w, c->D.win[0], bytes,
                                to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && to_host) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "get_state copy");
  return CDNS_OK;
}

cdns_status cdns_export_flags(cdns_ctx* c, uint8_t* flags_dev) {
  if (!c || !flags_dev) return c ? fail(c, CDNS_EINVAL, "null output") : CDNS_EINVAL;
  if (!c->last_rhs_valid) return fail(c, CDNS_EINVAL, "no right-hand side evaluated yet");
  hipError_t e = hipMemcpyAsync(flags_dev, c->D.nflag, (size_t)c->D.N, hipMemcpyDeviceToDevice,
                                c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "export_flags copy");
  return CDNS_OK;
}

cdns_status cdns_import_flags(cdns_ctx* c, const uint8_t* flags_dev) {
  if (!c || !flags_dev) return c ? fail(c, CDNS_EINVAL, "null flags") : CDNS_EINVAL;
  if (c->D.sensor_mode != 1) return fail(c, CDNS_EINVAL, "node flags are used in hybrid mode only");
  hipError_t e = hipMemcpyAsync(c->D.nflag, flags_dev, (size_t)c->D.N, hipMemcpyDeviceToDevice,
                                c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "import_flags copy");
  c->flags_imported = true;
  return CDNS_OK;
}

cdns_status cdns_rk_step(cdns_ctx* c, double cfl, double dt_fixed) {
  if (!c) return CDNS_EINVAL;
  if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return fail(c, CDNS_EINVAL, "need cfl > 0 or dt > 0");
  cdns_status s = check_bcs(c);
  if (s) return s;
  c->flags_imported = false;  // the step's sensor overwrites the node flags
  Desc D = c->D;
  D.cfl = cfl;
  D.dt_fixed = dt_fixed > 0.0 ? dt_fixed : 0.0;
  hipError_t e = enqueue_step(D, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "step launch");
  return CDNS_OK;
}

cdns_status cdns_advance_n(cdns_ctx* c, int32_t n, double cfl, double dt_fixed) {
  if (!c) return CDNS_EINVAL;
  if (n < 0) return fail(c, CDNS_EINVAL, "negative step count");
  if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return fail(c, CDNS_EINVAL, "need cfl > 0 or dt > 0");
  cdns_status s = check_bcs(c);
  if (s) return s;
  if (n == 0) return CDNS_OK;
  c->flags_imported = false;  // the steps' sensor overwrites the node flags
  const double dtf = dt_fixed > 0.0 ? dt_fixed : 0.0;
  hipError_t e;
  if (!c->gexec || c->g_cfl != cfl || c->g_dt != dtf) {
    invalidate_graph(c);
    Desc D = c->D;
    D.cfl = cfl;
    D.dt_fixed = dtf;
    hipGraph_t g = nullptr;
    if ((e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(c, e, "begin capture");
    hipError_t le = enqueue_step(D, c->cap);
    e = hipStreamEndCapture(c->cap, &g);
    if (le != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(c, le, "capture launch");
    }
    if (e != hipSuccess) return hip_fail(c, e, "end capture");
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->gexec = nullptr;
      return hip_fail(c, e, "graph instantiate");
    }
    c->g_cfl = cfl;
    c->g_dt = dtf;
  }
  for (int s2 = 0; s2 < n; ++s2) {
    if ((e = hipGraphLaunch(c->gexec, c->stream)) != hipSuccess)
      return hip_fail(c, e, "graph launch");
  }
  return CDNS_OK;
}

cdns_status cdns_diagnostics(cdns_ctx* c, cdns_diag* out) {
  if (!c || !out) return c ? fail(c, CDNS_EINVAL, "null output") : CDNS_EINVAL;
  Desc D = c->D;
  hipError_t e = cdns::launch_diag(D, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "diag launch");
  double dg[cdns::DG_COUNT], sc[cdns::SC_COUNT];
  unsigned st[4], cnt[4];
  if ((e = hipMemcpyAsync(dg, D.diag, sizeof(dg), hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(sc, D.scal, sizeof(sc), hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(st, D.status, sizeof(st), hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(cnt, D.count, sizeof(cnt), hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(c->stream)) != hipSuccess)
    return hip_fail(c, e, "diag copy");
  std::memset(out, 0, sizeof(*out));
  out->dt = sc[cdns::SC_DT];
  out->time = sc[cdns::SC_TIME];
  out->step = (int64_t)llround(sc[cdns::SC_STEP]);
  out->forcing_f = sc[cdns::SC_FORCE];
  out->mass = dg[cdns::DG_MASS];
  out->mom[0] = dg[cdns::DG_MX];
  out->mom[1] = dg[cdns::DG_MY];
  out->mom[2] = dg[cdns::DG_MZ];
  out->energy = dg[cdns::DG_E];
  out->kinetic = dg[cdns::DG_K];
  out->rho_min = dg[cdns::DG_RHOMIN];
  out->p_min = dg[cdns::DG_PMIN];
  out->mach_max = dg[cdns::DG_MACHMAX];
  out->nonfinite = (int64_t)llround(dg[cdns::DG_NONFINITE]);
  const double nif[3] = {(double)(D.per_x ? D.nx : D.nx - 1) * D.ny * D.nz,
                         (double)D.nx * (D.per_y ? D.ny : D.ny - 1) * D.nz, (double)D.N};
  for (int d = 0; d < 3; ++d) out->weno_frac[d] = D.sensor_mode > 0 ? cnt[d] / nif[d] : 0.0;
  out->status = (int32_t)st[0];
  if (st[0] != 0 || out->nonfinite != 0 || !(out->rho_min > 0.0) || !(out->p_min > 0.0))
    return fail(c, CDNS_ESTATE, "device flagged a bad state");
  return CDNS_OK;
}

cdns_status cdns_diagnostics_noalloc(cdns_ctx* c, const double* w_dev, double* out_dev) {
  if (!c) return CDNS_EINVAL;
  if (!out_dev) return fail(c, CDNS_EINVAL, "null output");
  const Desc& D = c->D;
  if (D.N > CDNS_NOALLOC_MAX_POINTS)
    return fail(c, CDNS_EINVAL,
                "grid of " + std::to_string(D.N) + " points exceeds the " +
                    std::to_string((long long)CDNS_NOALLOC_MAX_POINTS) +
                    "-point maximum of cdns_diagnostics_noalloc");
  static_assert(CDNS_NOALLOC_MAX_POINTS == (long long)cdns::kNoallocBlocks * cdns::kNoallocPoints,
                "header maximum must match the scratch array");
  static_assert(CDNS_NDIAG_DEV <= cdns::DG_COUNT, "output slots");
  double* part = nullptr;
  hipError_t e = cdns::noalloc_scratch(c->device, &part);
  if (e != hipSuccess) return hip_fail(c, e, "scratch address");
  e = cdns::launch_diag_noalloc(D, w_dev ? w_dev : D.win[0], part, out_dev, CDNS_NDIAG_DEV,
                                 c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "diag launch");
  return CDNS_OK;
}

cdns_status cdns_export_sensor(cdns_ctx* c, double* theta_dev, uint8_t* nflags_dev,
                               uint8_t* iflags_dev) {
  if (!c) return CDNS_EINVAL;
  if (!c->last_rhs_valid) return fail(c, CDNS_EINVAL, "no right-hand side evaluated yet");
  const Desc& D = c->D;
  hipError_t e = hipSuccess;
  if (theta_dev && D.sensor_mode == 1)
    e = hipMemcpyAsync(theta_dev, D.theta, D.N * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  else if (theta_dev)
    e = hipMemsetAsync(theta_dev, 0, D.N * sizeof(double), c->stream);
  if (e == hipSuccess && nflags_dev) {
    if (D.sensor_mode == 1)
      e = hipMemcpyAsync(nflags_dev, D.nflag, D.N, hipMemcpyDeviceToDevice, c->stream);
    else
      e = hipMemsetAsync(nflags_dev, 0, D.N, c->stream);
  }
  if (e == hipSuccess && iflags_dev) {
    if (D.sensor_mode > 0)
      e = cdns::launch_export_iflags(D, iflags_dev, c->stream);
    else
      e = hipMemsetAsync(iflags_dev, 0, D.N, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "export");
  return CDNS_OK;
}

cdns_status cdns_export_iface_flux(cdns_ctx* c, int32_t dir, double* out_dev) {
  if (!c) return CDNS_EINVAL;
  if (dir < 0 || dir > 2 || !out_dev) return fail(c, CDNS_EINVAL, "bad direction or pointer");
  if (!c->last_rhs_valid) return fail(c, CDNS_EINVAL, "no right-hand side evaluated yet");
  const Desc& D = c->D;
  hipError_t e = cdns::launch_export_iface(D, dir, out_dev, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "export");
  return CDNS_OK;
}

cdns_status cdns_time_phases(cdns_ctx* c, int32_t nsteps, double cfl, double dt_fixed,
                             double* ms_out, int32_t* launches_out, int64_t* weno_ifaces_out) {
  if (!c) return CDNS_EINVAL;
  if (nsteps < 1 || !ms_out) return fail(c, CDNS_EINVAL, "need nsteps >= 1 and an output array");
  if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return fail(c, CDNS_EINVAL, "need cfl > 0 or dt > 0");
  cdns_status s = check_bcs(c);
  if (s) return s;
  c->flags_imported = false;  // the steps' sensor overwrites the node flags
  Desc D = c->D;
  D.cfl = cfl;
  D.dt_fixed = dt_fixed > 0.0 ? dt_fixed : 0.0;
  hipStream_t st = c->stream;
  // every launch is bracketed by its own event pair; durations are summed per phase
  struct Rec { int ph; hipEvent_t a, b; };
  std::vector<Rec> recs;
  hipError_t e = hipSuccess;
  auto timed = [&](int ph, auto&& fn) {
    if (e != hipSuccess) return;
    Rec r{ph, nullptr, nullptr};
    if ((e = hipEventCreate(&r.a)) != hipSuccess) return;
    if ((e = hipEventCreate(&r.b)) != hipSuccess) { (void)hipEventDestroy(r.a); return; }
    recs.push_back(r);
    if ((e = hipEventRecord(r.a, st)) != hipSuccess) return;
    if ((e = fn()) != hipSuccess) return;
    e = hipEventRecord(r.b, st);
  };
  if (D.sensor_mode > 0) e = cdns::launch_count_iface(D, true, st);
  const bool dt_sen = cdns::dt_in_sensor(D);
  for (int step = 0; step < nsteps && e == hipSuccess; ++step) {
    if (!dt_sen) timed(CDNS_PH_DT, [&] { return cdns::launch_dt(D, st); });
    if (D.bc[0] == cdns::BC_DF_INFLOW)
      timed(CDNS_PH_GHOSTS, [&] { return cdns::launch_df(D, false, st); });
    for (int stage = 0; stage < 3; ++stage) {
      if (D.sensor_mode == 2 && e == hipSuccess) e = cdns::launch_stage_begin(D, st);
      if (cdns::ghosts_needed(D))
        timed(CDNS_PH_GHOSTS, [&] { return cdns::launch_ghosts(D, stage, st); });
      if (D.sensor_mode == 1)
        timed(CDNS_PH_SENSOR,
              [&] { return cdns::launch_sensor(D, stage, false, st, dt_sen && stage == 0); });
      if (D.sensor_mode > 0) {
        timed(CDNS_PH_IFLAGS,
              [&] { return cdns::launch_iflags(D, st, dt_sen && stage == 0); });
        timed(CDNS_PH_WENO, [&] { return cdns::launch_weno(D, stage, st); });
        if (e == hipSuccess) e = cdns::launch_count_iface(D, false, st);  // outside the events
      }
      const bool fuse = cdns::rk_fused(D);
      timed(CDNS_PH_RHS, [&] { return cdns::launch_rhs(D, stage, st, fuse); });
      if (D.forcing) timed(CDNS_PH_FORCE, [&] { return cdns::launch_force(D, st); });
      if (!fuse) timed(CDNS_PH_RK, [&] { return cdns::launch_rk(D, stage, st); });
      else if (D.forcing) timed(CDNS_PH_RK, [&] { return cdns::launch_rk_forced(D, stage, st); });
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  double tot[CDNS_NPHASES] = {0};
  int cnt[CDNS_NPHASES] = {0};
  for (auto& r : recs) {
    float ms = 0.0f;
    if (e == hipSuccess && r.b) e = hipEventElapsedTime(&ms, r.a, r.b);
    tot[r.ph] += ms;
    cnt[r.ph] += 1;
    (void)hipEventDestroy(r.a);
    if (r.b) (void)hipEventDestroy(r.b);
  }
  if (e != hipSuccess) return hip_fail(c, e, "timed step");
  for (int p = 0; p < CDNS_NPHASES; ++p) {
    ms_out[p] = cnt[p] ? tot[p] / cnt[p] : 0.0;
    if (launches_out) launches_out[p] = cnt[p];
  }
  if (weno_ifaces_out) {
    double acc = 0.0;
    if (D.sensor_mode > 0 &&
        ((e = hipMemcpyAsync(&acc, D.scal + cdns::SC_WACC, sizeof(double), hipMemcpyDeviceToHost,
                             st)) != hipSuccess ||
         (e = hipStreamSynchronize(st)) != hipSuccess))
      return hip_fail(c, e, "interface count");
    *weno_ifaces_out = (int64_t)acc;
  }
  return CDNS_OK;
}

cdns_status cdns_stats_accumulate(cdns_ctx* c) {
  if (!c) return CDNS_EINVAL;
  hipError_t e = cdns::launch_stats(c->D, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "statistics launch");
  c->stat_samples += 1;
  return CDNS_OK;
}

cdns_status cdns_stats_export(cdns_ctx* c, double* host_out, int64_t* samples) {
  if (!c || !host_out || !samples) return c ? fail(c, CDNS_EINVAL, "null output") : CDNS_EINVAL;
  const Desc& D = c->D;
  const size_t bytes = (size_t)cdns::kNStat * D.ny * D.nx * sizeof(double);
  hipError_t e = hipMemcpyAsync(host_out, D.stats, bytes, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "statistics export");
  *samples = c->stat_samples;
  return CDNS_OK;
}

cdns_status cdns_stats_means(cdns_ctx* c, int32_t average_x, double* out_dev) {
  if (!c) return CDNS_EINVAL;
  if (!out_dev) return fail(c, CDNS_EINVAL, "null output");
  if (c->stat_samples <= 0) return fail(c, CDNS_EINVAL, "no statistics accumulated");
  const Desc& D = c->D;
  const double count = (double)c->stat_samples * D.nz * (average_x ? D.nx : 1);
  hipError_t e = cdns::launch_stats_means(D, average_x != 0, count, out_dev, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "statistics means");
  return CDNS_OK;
}

cdns_status cdns_stats_reset(cdns_ctx* c) {
  if (!c) return CDNS_EINVAL;
  const Desc& D = c->D;
  hipError_t e = hipMemsetAsync(D.stats, 0, (size_t)cdns::kNStat * D.ny * D.nx * sizeof(double),
                                c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "statistics reset");
  c->stat_samples = 0;
  return CDNS_OK;
}

const char* cdns_last_error(const cdns_ctx* c) { return c ? c->err.c_str() : "null context"; }

cdns_status cdns_destroy(cdns_ctx* c) {
  if (!c) return CDNS_EINVAL;
  if (c->batch_refs > 0) return fail(c, CDNS_EBUSY, "context attached to a batch");
  invalidate_graph(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
  return CDNS_OK;
}

}  // extern "C"

// Accessors used by the batched runner (cdns_batch.hip).
namespace cdns {
const Desc& ctx_desc(const cdns_ctx* c) { return c->D; }
int& ctx_batch_refs(cdns_ctx* c) { return c->batch_refs; }
hipStream_t ctx_stream(const cdns_ctx* c) { return c->stream; }
}  // namespace cdns
