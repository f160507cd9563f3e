/*
 * cdns_oracle.c -- plain, slow FP64 CPU reference of the compressible
 * Navier-Stokes right-hand side and the low-storage RK3 step of
 * "STREAmS: a high-fidelity accelerated solver for direct numerical
 * simulation of compressible turbulent flows" (arXiv 2004.02276).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -std=c11 -fPIC -shared -lm
 * (no contraction to fused multiply-add, t^{3/2} as t*sqrt(t)).
 *
 * Data layout of the caller's arrays: w[5][nz][ny][nx], x fastest.
 * Internally every field lives on a padded grid with a halo of H = 4 nodes
 * on each side; the hw = max(2, L, r) ghost layers that the schemes reach
 * (L: half-width of the central stencils, r: WENO stencil size) are filled
 * explicitly (x faces, then y faces over the x-extended range, then z faces
 * over the x,y-extended range) and every operator then reads plain
 * neighbours.  This is deliberately the most direct form of the
 * discretisation, not a fast one.
 *
 * Parity status of each function is stated beside it; all are pinned by
 * the CPU tests (closed forms, invariants, exact solutions, convergence).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define H 4

enum { BC_PERIODIC = 0, BC_WALL_ISO = 1, BC_WALL_ADIA = 2, BC_DIRICHLET = 3,
       BC_OUTFLOW = 4, BC_SHOCK_TOP = 5, BC_DF_INFLOW = 6 };
enum { T_CONV = 1, T_PRES = 2, T_VISC = 4, T_FORCE = 8, T_ALL = 15 };
enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_ENOMEM = -2, ORA_ESTATE = -4, ORA_EUNSUP = -5 };

typedef struct {
  int32_t nx, ny, nz;
  double lx, lz;
  const double* y_eta;     /* [ny] */
  const double* y_etaeta;  /* [ny] */
  double gamma, Pr, R_gas, mu_ref, T_ref, S_suth;
  int32_t viscous, sensor_mode;
  double theta_star, sensor_eps;
  int32_t forcing;
  int32_t terms;           /* bit mask of T_* (T_ALL for the full operator) */
  int32_t bc_kind[6];
  const double* bc_params[6];
  int32_t bc_nparams[6];
  /* digital-filter inflow plane to use (conserved [5][nz][ny]); NULL: the
   * initial plane of the generator (see df_plane) */
  const double* df_plane;
  /* scheme orders (Sec. 2.1): central flux and viscous derivatives of order
   * 2L (L = 1, 2, 3; 0 selects L = 2), WENO reconstruction of order 2r - 1
   * from r candidate stencils (r = 2, 3, 4; 0 selects r = 3) */
  int32_t central_L, weno_r;
} ora_problem;

/* Standard central finite-difference coefficients of order 2L (Sec. 2.1),
 * rows L = 1, 2, 3: first derivative f'_i ~ (1/h) sum_{l=1}^{L} a_l
 * (f_{i+l} - f_{i-l}); second derivative f''_i ~ (1/h^2) (b_0 f_i +
 * sum_{l=1}^{L} b_l (f_{i+l} + f_{i-l})). */
static const double ACOEF[4][3] = {{0.0, 0.0, 0.0},
                                   {1.0 / 2.0, 0.0, 0.0},
                                   {2.0 / 3.0, -1.0 / 12.0, 0.0},
                                   {3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0}};
static const double BCOEF[4][4] = {{0.0, 0.0, 0.0, 0.0},
                                   {-2.0, 1.0, 0.0, 0.0},
                                   {-5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0, 0.0},
                                   {-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0}};
/* largest magnitude of the symbol of the order-2L second derivative
 * (reached at the grid Nyquist wavenumber): |b_0 + 2 sum_l (-1)^l b_l| */
static const double D2RHO[4] = {0.0, 4.0, 16.0 / 3.0, 272.0 / 45.0};

/* Wray's low-storage RK3 (Sec. 2.2, eq. RK).  The second alpha is printed
 * with a plus sign; only -17/60 makes the scheme consistent (weights sum to
 * one) and third-order, so that is the reading used. */
static const double RK_ALPHA[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
static const double RK_BETA[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};

typedef struct {
  int nx, ny, nz, nxp, nyp, nzp;
  int L, r, hw;   /* central half-width, WENO stencil size, ghost layers used */
  size_t np;
  double dx, dz, deta;
  double cv, cp, icv;
} geom;

static void make_geom(const ora_problem* P, geom* g) {
  g->nx = P->nx; g->ny = P->ny; g->nz = P->nz;
  g->nxp = P->nx + 2 * H; g->nyp = P->ny + 2 * H; g->nzp = P->nz + 2 * H;
  g->np = (size_t)g->nxp * g->nyp * g->nzp;
  g->dx = P->lx / P->nx; g->dz = P->lz / P->nz; g->deta = 1.0 / P->ny;
  g->cv = P->R_gas / (P->gamma - 1.0);
  g->icv = 1.0 / g->cv;
  g->cp = P->gamma * P->R_gas / (P->gamma - 1.0);
  g->L = P->central_L ? P->central_L : 2;
  g->r = P->weno_r ? P->weno_r : 3;
  g->hw = 2;  /* the shock sensor's fourth-order derivatives */
  if (g->L > g->hw) g->hw = g->L;
  if (g->r > g->hw) g->hw = g->r;
}

static inline size_t pidx(const geom* g, int i, int j, int k) {
  return ((size_t)(k + H) * g->nyp + (size_t)(j + H)) * g->nxp + (size_t)(i + H);
}
static inline size_t uidx(const geom* g, int i, int j, int k) {
  return ((size_t)k * g->ny + (size_t)j) * g->nx + (size_t)i;
}

/* ------------------------------------------------------------ thermodynamics
 * Perfect gas (Sec. 2): E = c_v T + |u|^2/2, p = rho R T, H = E + p/rho;
 * Sutherland viscosity mu = mu_ref t^{3/2} (1+S)/(t+S), t = T/T_ref;
 * conductivity k = c_p mu / Pr. */
typedef struct { double rho, u, v, w, p, T, Ht, mu; } prim_t;

static prim_t to_prim(const ora_problem* P, const geom* g, const double q[5]) {
  /* one reciprocal of the density, then products; T from the internal
   * energy per unit mass, p from the gas law, H = E + p/rho */
  prim_t s;
  double ir = 1.0 / q[0];
  s.rho = q[0];
  s.u = q[1] * ir;
  s.v = q[2] * ir;
  s.w = q[3] * ir;
  double ke = 0.5 * (s.u * s.u + s.v * s.v + s.w * s.w);
  double E = q[4] * ir;
  s.T = (E - ke) * g->icv;
  s.p = s.rho * P->R_gas * s.T;
  s.Ht = E + s.p * ir;
  double t = s.T * (1.0 / P->T_ref);
  s.mu = P->mu_ref * t * sqrt(t) * (1.0 + P->S_suth) / (t + P->S_suth);
  return s;
}

static void from_prim(const ora_problem* P, double rho, double u, double v, double w,
                      double p, double q[5]) {
  q[0] = rho;
  q[1] = rho * u;
  q[2] = rho * v;
  q[3] = rho * w;
  q[4] = p / (P->gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
}

/* ------------------------------------------------------------ eigenvectors
 * Right/left eigenvectors of the Euler flux Jacobian in direction d, written
 * for components permuted so that the normal momentum comes first:
 * (rho, rho u_n, rho u_t1, rho u_t2, rho E).  Inputs are the state's normal
 * and tangential velocities, total enthalpy and sound speed.  Used for the
 * Lax-Friedrichs characteristic splitting of Sec. 2.1. */
static void eigvecs_perm(double gm1, double un, double ut1, double ut2, double Ht, double c,
                         double Rm[5][5], double Lm[5][5]) {
  double q2 = un * un + ut1 * ut1 + ut2 * ut2;
  double b1 = gm1 / (c * c);
  double b2 = 0.5 * q2 * b1;
  /* columns of R */
  double R_[5][5] = {
      {1.0, 1.0, 0.0, 0.0, 1.0},
      {un - c, un, 0.0, 0.0, un + c},
      {ut1, ut1, 1.0, 0.0, ut1},
      {ut2, ut2, 0.0, 1.0, ut2},
      {Ht - un * c, 0.5 * q2, ut1, ut2, Ht + un * c}};
  double L_[5][5] = {
      {0.5 * (b2 + un / c), -0.5 * (b1 * un + 1.0 / c), -0.5 * b1 * ut1, -0.5 * b1 * ut2, 0.5 * b1},
      {1.0 - b2, b1 * un, b1 * ut1, b1 * ut2, -b1},
      {-ut1, 0.0, 1.0, 0.0, 0.0},
      {-ut2, 0.0, 0.0, 1.0, 0.0},
      {0.5 * (b2 - un / c), -0.5 * (b1 * un - 1.0 / c), -0.5 * b1 * ut1, -0.5 * b1 * ut2, 0.5 * b1}};
  memcpy(Rm, R_, sizeof(R_));
  memcpy(Lm, L_, sizeof(L_));
}

/* permutation: component index in permuted order -> natural component index */
static void perm_of_dir(int d, int pm[5]) {
  pm[0] = 0; pm[4] = 4;
  if (d == 0) { pm[1] = 1; pm[2] = 2; pm[3] = 3; }
  else if (d == 1) { pm[1] = 2; pm[2] = 3; pm[3] = 1; }
  else { pm[1] = 3; pm[2] = 1; pm[3] = 2; }
}

/* exported for tests: eigenvectors in natural component order for direction d */
void ora_eigenvectors(double gamma, int d, double u, double v, double w, double Ht,
                      double* Rout, double* Lout) {
  int pm[5];
  perm_of_dir(d, pm);
  double vel[3] = {u, v, w};
  double un = vel[d], ut1 = vel[(d + 1) % 3], ut2 = vel[(d + 2) % 3];
  double c = sqrt((gamma - 1.0) * (Ht - 0.5 * (u * u + v * v + w * w)));
  double Rm[5][5], Lm[5][5];
  eigvecs_perm(gamma - 1.0, un, ut1, ut2, Ht, c, Rm, Lm);
  /* natural R[row=component][col=wave] ; natural L[row=wave][col=component] */
  for (int a = 0; a < 5; ++a)
    for (int b = 0; b < 5; ++b) {
      Rout[pm[a] * 5 + b] = Rm[a][b];
      Lout[b * 5 + pm[a]] = Lm[b][a];
    }
}

/* ------------------------------------------------------------ WENO-JS
 * Jiang-Shu weighted reconstruction of order 2r - 1 at the right face of
 * cell i from the r candidate stencils S_k = {i-r+1+k, ..., i+k}
 * (k = 0..r-1).  v[0..2r-2] holds cells i-r+1..i+r-1.  ora_weno_parts gives
 * each candidate's polynomial value at the face, q_k, and its smoothness
 * indicator beta_k (sum over the derivatives m = 1..r-1 of the squared m-th
 * derivative of the candidate polynomial integrated over cell i, scaled by
 * h^(2m-1)); ora_weno combines them with the nonlinear weights
 * d_k/(eps + beta_k)^2, eps = 1e-6, normalised.  Linear weights d_k:
 * r = 2: (1/3, 2/3); r = 3: (1/10, 6/10, 3/10); r = 4: (1/35, 12/35, 18/35,
 * 4/35).  (Sec. 2.1 cites the Jiang-Shu scheme without its order; the
 * default is r = 3, fifth order.) */
void ora_weno_parts(int r, const double* v, double* q, double* beta) {
  const double* c = v + (r - 1);  /* c[0] = cell i */
  if (r == 2) {
    q[0] = (-c[-1] + 3.0 * c[0]) / 2.0;
    q[1] = (c[0] + c[1]) / 2.0;
    beta[0] = (c[0] - c[-1]) * (c[0] - c[-1]);
    beta[1] = (c[1] - c[0]) * (c[1] - c[0]);
  } else if (r == 3) {
    double vm2 = c[-2], vm1 = c[-1], v0 = c[0], vp1 = c[1], vp2 = c[2];
    q[0] = (2.0 * vm2 - 7.0 * vm1 + 11.0 * v0) / 6.0;
    q[1] = (-vm1 + 5.0 * v0 + 2.0 * vp1) / 6.0;
    q[2] = (2.0 * v0 + 5.0 * vp1 - vp2) / 6.0;
    /* squared second and first differences of each candidate */
    double c0 = vm2 - 2.0 * vm1 + v0, e0 = vm2 - 4.0 * vm1 + 3.0 * v0;
    double c1 = vm1 - 2.0 * v0 + vp1, e1 = vm1 - vp1;
    double c2 = v0 - 2.0 * vp1 + vp2, e2 = 3.0 * v0 - 4.0 * vp1 + vp2;
    beta[0] = 13.0 / 12.0 * (c0 * c0) + 0.25 * (e0 * e0);
    beta[1] = 13.0 / 12.0 * (c1 * c1) + 0.25 * (e1 * e1);
    beta[2] = 13.0 / 12.0 * (c2 * c2) + 0.25 * (e2 * e2);
  } else {
    double a = c[-3], b = c[-2], d = c[-1], e = c[0], f = c[1], g = c[2], h = c[3];
    q[0] = (-3.0 * a + 13.0 * b - 23.0 * d + 25.0 * e) / 12.0;
    q[1] = (b - 5.0 * d + 13.0 * e + 3.0 * f) / 12.0;
    q[2] = (-d + 7.0 * e + 7.0 * f - g) / 12.0;
    q[3] = (3.0 * e + 13.0 * f - 5.0 * g + h) / 12.0;
    /* the indicators as quadratic forms of the four stencil values
     * (Balsara and Shu's seventh-order scheme), divided by 240 */
    beta[0] = (a * (547.0 * a - 3882.0 * b + 4642.0 * d - 1854.0 * e) +
               b * (7043.0 * b - 17246.0 * d + 7042.0 * e) + d * (11003.0 * d - 9402.0 * e) +
               2107.0 * e * e) / 240.0;
    beta[1] = (b * (267.0 * b - 1642.0 * d + 1602.0 * e - 494.0 * f) +
               d * (2843.0 * d - 5966.0 * e + 1922.0 * f) + e * (3443.0 * e - 2522.0 * f) +
               547.0 * f * f) / 240.0;
    beta[2] = (d * (547.0 * d - 2522.0 * e + 1922.0 * f - 494.0 * g) +
               e * (3443.0 * e - 5966.0 * f + 1602.0 * g) + f * (2843.0 * f - 1642.0 * g) +
               267.0 * g * g) / 240.0;
    beta[3] = (e * (2107.0 * e - 9402.0 * f + 7042.0 * g - 1854.0 * h) +
               f * (11003.0 * f - 17246.0 * g + 4642.0 * h) + g * (7043.0 * g - 3882.0 * h) +
               547.0 * h * h) / 240.0;
  }
}

double ora_weno(int r, const double* v) {
  static const double DLIN[5][4] = {{0, 0, 0, 0}, {0, 0, 0, 0},
                                    {1.0 / 3.0, 2.0 / 3.0, 0, 0},
                                    {0.1, 0.6, 0.3, 0},
                                    {1.0 / 35.0, 12.0 / 35.0, 18.0 / 35.0, 4.0 / 35.0}};
  double q[4], beta[4];
  ora_weno_parts(r, v, q, beta);
  const double eps = 1e-6;
  double num = 0.0, sum = 0.0;
  for (int k = 0; k < r; ++k) {
    double ak = DLIN[r][k] / ((eps + beta[k]) * (eps + beta[k]));
    num += ak * q[k];
    sum += ak;
  }
  return num / sum;
}

/* fifth-order case, kept as its own entry point for the tests */
double ora_weno5(const double* v) { return ora_weno(3, v); }

/* ------------------------------------------------------------ inflow turbulence
 * Synthetic inflow turbulence by digital filtering (Sec. 3.2: the DF method
 * with the filtering split into one-dimensional convolutions and the
 * strong Reynolds analogy for the thermodynamic fluctuations).  Readings
 * (the paper gives the method, not its constants):
 *  - deviates: zero mean, unit variance, uniform on [-sqrt 3, sqrt 3) from
 *    the counter-based SplitMix64 generator (output n of the generator
 *    seeded with `seed`), n = 1 + (((key*3 + c)*nz + k)*(ny + 2 Ny) + jj)
 *    for velocity component c, plane k, extended row jj, and key = 0 for
 *    the initial plane, key = s + 1 at the start of step s;
 *  - filters: for a filter length of n grid spacings, the Gaussian
 *    coefficients b_l proportional to exp(-pi l^2 / (2 n^2)), l = -N..N
 *    with N = max(1, ceil(2 n)), normalised to unit sum of squares;
 *    applied along y (over the extended rows) and then along z (periodic),
 *    each as a sum in increasing l;
 *  - time correlation: psi = psi E + psi_hat sqrt(1 - E^2) with
 *    E = exp(-pi dt / (2 T)); the initial plane takes psi = psi_hat;
 *  - fluctuations u'_i = a_ij psi_j with a the lower triangular factor of
 *    the Reynolds stress tensor R = a a^T (Lund's transformation: a11 =
 *    sqrt R11, a21 = R21/a11, a22 = sqrt(R22 - a21^2), a31 = R31/a11,
 *    a32 = (R32 - a21 a31)/a22, a33 = sqrt(R33 - a31^2 - a32^2); a zero
 *    diagonal entry zeroes the entries below it), temperature from the
 *    strong Reynolds analogy with constant total enthalpy, T' = -u_mean u'/c_p,
 *    constant pressure, so rho = p/(R (T_mean + T')).
 * Parameters (face x-): [n_y, n_z (filter lengths in grid spacings), T,
 * seed, mean rho, u, v, w, p [5][ny], R11, R22, R33, R12, R13, R23 [6][ny]]. */
uint64_t ora_splitmix64(uint64_t seed, uint64_t n) {
  uint64_t z = seed + n * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static double df_deviate(uint64_t seed, uint64_t n) {
  const double u = (double)(ora_splitmix64(seed, n) >> 11) * 0x1.0p-53;
  return (2.0 * u - 1.0) * 1.7320508075688772;
}

static int df_half_width(double n) {
  const int N = (int)ceil(2.0 * n);
  return N < 1 ? 1 : N;
}

static int df_layout(const ora_problem* P, int* Ny, int* Nz) {
  const double* pr = P->bc_params[0];
  if (P->bc_nparams[0] != 4 + 11 * P->ny) return ORA_EINVAL;
  if (!(pr[0] > 0.0) || !(pr[1] > 0.0) || !(pr[2] > 0.0)) return ORA_EINVAL;
  *Ny = df_half_width(pr[0]);
  *Nz = df_half_width(pr[1]);
  return ORA_OK;
}

/* Gaussian filter coefficients b[0..2N] (l = -N..N) for a length of n
 * grid spacings, unit sum of squares. */
static void df_filter(double n, int N, double* b) {
  double ss = 0.0;
  for (int l = -N; l <= N; ++l) {
    b[l + N] = exp(-3.141592653589793 * (double)(l * l) / (2.0 * n * n));
    ss += b[l + N] * b[l + N];
  }
  const double nrm = sqrt(ss);
  for (int l = 0; l <= 2 * N; ++l) b[l] /= nrm;
}

/* Lower triangular a with a a^T = R for R = (R11, R22, R33, R12, R13, R23);
 * a = (a11, a21, a22, a31, a32, a33). */
static void df_cholesky(const double R[6], double a[6]) {
  const double a11 = sqrt(fmax(R[0], 0.0));
  const double a21 = a11 > 0.0 ? R[3] / a11 : 0.0;
  const double a31 = a11 > 0.0 ? R[4] / a11 : 0.0;
  const double a22 = sqrt(fmax(R[1] - a21 * a21, 0.0));
  const double a32 = a22 > 0.0 ? (R[5] - a21 * a31) / a22 : 0.0;
  const double a33 = sqrt(fmax(R[2] - a31 * a31 - a32 * a32, 0.0));
  a[0] = a11; a[1] = a21; a[2] = a22; a[3] = a31; a[4] = a32; a[5] = a33;
}

/* The derived inflow-generator coefficients of a problem: half-widths,
 * by[2 Ny + 1], bz[2 Nz + 1] (each array at least 2 * ny + 1, resp.
 * 2 * nz + 1, long) and the factor chol[6][ny]. */
int ora_df_coeffs(const ora_problem* P, int* Ny, int* Nz, double* by, double* bz, double* chol) {
  int st = df_layout(P, Ny, Nz);
  if (st) return st;
  const double* pr = P->bc_params[0];
  df_filter(pr[0], *Ny, by);
  df_filter(pr[1], *Nz, bz);
  const double* rs = pr + 4 + 5 * P->ny;
  for (int j = 0; j < P->ny; ++j) {
    double R[6], a[6];
    for (int m = 0; m < 6; ++m) R[m] = rs[m * P->ny + j];
    df_cholesky(R, a);
    for (int m = 0; m < 6; ++m) chol[m * P->ny + j] = a[m];
  }
  return ORA_OK;
}

/* One update of the filtered field psi[3][nz][ny] (first: psi = psi_hat)
 * and the resulting conserved inflow plane[5][nz][ny]; fl (may be NULL)
 * receives the velocity fluctuations [3][nz][ny]. */
int ora_df_update(const ora_problem* P, uint64_t key, double dt, int first, double* psi,
                  double* plane, double* fl) {
  int Ny, Nz;
  int st = df_layout(P, &Ny, &Nz);
  if (st) return st;
  const int ny = P->ny, nz = P->nz, nyr = ny + 2 * Ny;
  const double* pr = P->bc_params[0];
  const double TL = pr[2];
  const uint64_t seed = (uint64_t)pr[3];
  const double* mean = pr + 4;
  double* by = malloc((size_t)(2 * Ny + 1) * sizeof(double));
  double* bz = malloc((size_t)(2 * Nz + 1) * sizeof(double));
  double* chol = malloc((size_t)6 * ny * sizeof(double));
  double* fy = malloc((size_t)3 * nz * ny * sizeof(double));
  if (!by || !bz || !chol || !fy) {
    free(by); free(bz); free(chol); free(fy);
    return ORA_ENOMEM;
  }
  ora_df_coeffs(P, &Ny, &Nz, by, bz, chol);
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j) {
        double acc = 0.0;
        for (int l = -Ny; l <= Ny; ++l) {
          uint64_t n = 1 + (((key * 3 + (uint64_t)c) * (uint64_t)nz + (uint64_t)k) * (uint64_t)nyr +
                            (uint64_t)(j + l + Ny));
          acc += by[l + Ny] * df_deviate(seed, n);
        }
        fy[((size_t)c * nz + k) * ny + j] = acc;
      }
  const double E = exp(-3.141592653589793 * dt / (2.0 * TL));
  const double F = sqrt(1.0 - E * E);
  const double cp = P->gamma * P->R_gas / (P->gamma - 1.0);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) {
      double ps[3];
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int m = -Nz; m <= Nz; ++m) {
          int kk = ((k + m) % nz + nz) % nz;
          acc += bz[m + Nz] * fy[((size_t)c * nz + kk) * ny + j];
        }
        size_t q = ((size_t)c * nz + k) * ny + j;
        psi[q] = first ? acc : psi[q] * E + acc * F;
        ps[c] = psi[q];
      }
      const double a11 = chol[j], a21 = chol[ny + j], a22 = chol[2 * ny + j];
      const double a31 = chol[3 * ny + j], a32 = chol[4 * ny + j], a33 = chol[5 * ny + j];
      const double du = a11 * ps[0];
      const double dv = a21 * ps[0] + a22 * ps[1];
      const double dw = a31 * ps[0] + a32 * ps[1] + a33 * ps[2];
      const double rm = mean[j], um = mean[ny + j], vm = mean[2 * ny + j], wm = mean[3 * ny + j];
      const double pm = mean[4 * ny + j];
      const double Tm = pm / (rm * P->R_gas);
      const double T = Tm - um * du / cp;
      double qc[5];
      from_prim(P, pm / (P->R_gas * T), um + du, vm + dv, wm + dw, pm, qc);
      for (int m = 0; m < 5; ++m) plane[((size_t)m * nz + k) * ny + j] = qc[m];
      if (fl) {
        fl[((size_t)0 * nz + k) * ny + j] = du;
        fl[((size_t)1 * nz + k) * ny + j] = dv;
        fl[((size_t)2 * nz + k) * ny + j] = dw;
      }
    }
  free(by); free(bz); free(chol); free(fy);
  return ORA_OK;
}

/* Characteristic extrapolation through a face (Sec. 3.2, non-reflecting
 * boundaries): only waves leaving the domain are extrapolated from the two
 * nodes next to the face, incoming ones are held; d is the face normal,
 * qb the boundary node, qi its interior neighbour, out[s-1] ghost s. */
static void char_ghosts(const ora_problem* P, const geom* g, int d, int hi, const double qb[5],
                        const double qi[5], double out[H][5]) {
  const int hw = g->hw;
  double dq[5];
  for (int m = 0; m < 5; ++m) dq[m] = qb[m] - qi[m];
  prim_t s0 = to_prim(P, g, qb);
  double c = sqrt(P->gamma * s0.p / s0.rho);
  double Rn[25], Ln[25];
  ora_eigenvectors(P->gamma, d, s0.u, s0.v, s0.w, s0.Ht, Rn, Ln);
  double un = d == 0 ? s0.u : (d == 1 ? s0.v : s0.w);
  double lam[5] = {un - c, un, un, un, un + c};
  double dv[5];
  for (int a = 0; a < 5; ++a) {
    double acc = 0.0;
    for (int b = 0; b < 5; ++b) acc += Ln[a * 5 + b] * dq[b];
    int outgoing = hi ? (lam[a] > 0.0) : (lam[a] < 0.0);
    dv[a] = outgoing ? acc : 0.0;
  }
  for (int s = 1; s <= hw; ++s)
    for (int m = 0; m < 5; ++m) {
      double acc = 0.0;
      for (int a = 0; a < 5; ++a) acc += Rn[m * 5 + a] * dv[a];
      out[s - 1][m] = qb[m] + (double)s * acc;
    }
}

/* ------------------------------------------------------------ ghost nodes */
static int fill_ghosts(const ora_problem* P, const geom* g, double* W[5]) {
  const int nx = g->nx, ny = g->ny, nz = g->nz, hw = g->hw;
  int bad = 0;
  /* x faces (interior j, k) */
  for (int side = 0; side < 2; ++side) {
    int kind = P->bc_kind[side];
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j) {
        if (kind == BC_PERIODIC) {
          for (int s = 1; s <= hw; ++s) {
            int gi = side == 0 ? -s : nx - 1 + s;
            int si = side == 0 ? nx - s : s - 1;
            for (int m = 0; m < 5; ++m) W[m][pidx(g, gi, j, k)] = W[m][pidx(g, si, j, k)];
          }
        } else if (kind == BC_DIRICHLET) {
          const double* pr = P->bc_params[side];
          double q[5];
          from_prim(P, pr[0 * ny + j], pr[1 * ny + j], pr[2 * ny + j], pr[3 * ny + j],
                    pr[4 * ny + j], q);
          for (int s = 1; s <= hw; ++s) {
            int gi = side == 0 ? -s : nx - 1 + s;
            for (int m = 0; m < 5; ++m) W[m][pidx(g, gi, j, k)] = q[m];
          }
        } else if (kind == BC_OUTFLOW) {
          int ib = side == 0 ? 0 : nx - 1;
          int ii = side == 0 ? 1 : nx - 2;
          double qb[5], qi[5], gq[H][5];
          for (int m = 0; m < 5; ++m) {
            qb[m] = W[m][pidx(g, ib, j, k)];
            qi[m] = W[m][pidx(g, ii, j, k)];
          }
          char_ghosts(P, g, 0, side, qb, qi, gq);
          for (int s = 1; s <= hw; ++s) {
            int gi = side == 0 ? -s : nx - 1 + s;
            for (int m = 0; m < 5; ++m) W[m][pidx(g, gi, j, k)] = gq[s - 1][m];
          }
        } else if (kind == BC_DF_INFLOW && side == 0) {
          /* the inflow plane of the current step, the same on every layer */
          if (!P->df_plane) return ORA_EINVAL;
          for (int s = 1; s <= hw; ++s)
            for (int m = 0; m < 5; ++m)
              W[m][pidx(g, -s, j, k)] = P->df_plane[((size_t)m * nz + k) * ny + j];
        } else {
          return ORA_EUNSUP;
        }
      }
  }
  /* y faces over the x-extended range, interior k */
  for (int side = 0; side < 2; ++side) {
    int kind = P->bc_kind[2 + side];
    for (int k = 0; k < nz; ++k)
      for (int i = -hw; i < nx + hw; ++i) {
        for (int s = 1; s <= hw; ++s) {
          int gj = side == 0 ? -s : ny - 1 + s;
          double q[5];
          if (kind == BC_PERIODIC) {
            int sj = side == 0 ? ny - s : s - 1;
            for (int m = 0; m < 5; ++m) q[m] = W[m][pidx(g, i, sj, k)];
          } else if (kind == BC_WALL_ISO || kind == BC_WALL_ADIA) {
            /* mirror about the wall, which lies half-way between node 0 and
             * ghost -1 (staggered wall, Sec. 3.1): ghost s <-> interior s-1 */
            int mj = side == 0 ? s - 1 : ny - s;
            double qm[5];
            for (int m = 0; m < 5; ++m) qm[m] = W[m][pidx(g, i, mj, k)];
            prim_t sm = to_prim(P, g, qm);
            double Tg = kind == BC_WALL_ISO ? 2.0 * P->bc_params[2 + side][0] - sm.T : sm.T;
            if (!(Tg > 0.0)) bad = 1;
            double rg = sm.p / (P->R_gas * Tg);
            from_prim(P, rg, -sm.u, -sm.v, -sm.w, sm.p, q);
          } else if (kind == BC_SHOCK_TOP) {
            const double* pr = P->bc_params[2 + side];
            int ish = (int)pr[0];
            const double* st = i < ish ? pr + 1 : pr + 6;
            from_prim(P, st[0], st[1], st[2], st[3], st[4], q);
          } else if (kind == BC_OUTFLOW) {
            int jb = side == 0 ? 0 : ny - 1;
            int ji = side == 0 ? 1 : ny - 2;
            double qb[5], qi[5], gq[H][5];
            for (int m = 0; m < 5; ++m) {
              qb[m] = W[m][pidx(g, i, jb, k)];
              qi[m] = W[m][pidx(g, i, ji, k)];
            }
            char_ghosts(P, g, 1, side, qb, qi, gq);
            for (int m = 0; m < 5; ++m) q[m] = gq[s - 1][m];
          } else {
            return ORA_EUNSUP;
          }
          for (int m = 0; m < 5; ++m) W[m][pidx(g, i, gj, k)] = q[m];
        }
      }
  }
  /* z faces over the x,y-extended range: only periodic is accepted */
  if (P->bc_kind[4] != BC_PERIODIC || P->bc_kind[5] != BC_PERIODIC) return ORA_EUNSUP;
  for (int j = -hw; j < ny + hw; ++j)
    for (int i = -hw; i < nx + hw; ++i)
      for (int s = 1; s <= hw; ++s)
        for (int m = 0; m < 5; ++m) {
          W[m][pidx(g, i, j, -s)] = W[m][pidx(g, i, j, nz - s)];
          W[m][pidx(g, i, j, nz - 1 + s)] = W[m][pidx(g, i, j, s - 1)];
        }
  return bad ? ORA_ESTATE : ORA_OK;
}

static int validate(const ora_problem* P) {
  if (P->nx < 4 || P->ny < 4 || P->nz < 4) return ORA_EINVAL;
  for (int a = 0; a < 3; ++a) {
    int k0 = P->bc_kind[2 * a], k1 = P->bc_kind[2 * a + 1];
    if ((k0 == BC_PERIODIC) != (k1 == BC_PERIODIC)) return ORA_EINVAL;
  }
  for (int f = 0; f < 6; ++f) {
    int k = P->bc_kind[f];
    int ax = f / 2;
    if (k == BC_PERIODIC) continue;
    if (ax == 2) return ORA_EUNSUP;
    if (ax == 0 && !(k == BC_DIRICHLET || k == BC_OUTFLOW || (k == BC_DF_INFLOW && f == 0)))
      return ORA_EUNSUP;
    if (ax == 1 && !(k == BC_WALL_ISO || k == BC_WALL_ADIA || k == BC_SHOCK_TOP || k == BC_OUTFLOW))
      return ORA_EUNSUP;
    if (k == BC_DF_INFLOW) {
      int Ny, Nz;
      if (df_layout(P, &Ny, &Nz)) return ORA_EINVAL;
    }
    if (k == BC_DIRICHLET && P->bc_nparams[f] != 5 * P->ny) return ORA_EINVAL;
    if (k == BC_WALL_ISO && P->bc_nparams[f] != 1) return ORA_EINVAL;
    if (k == BC_SHOCK_TOP && P->bc_nparams[f] != 11) return ORA_EINVAL;
  }
  if (P->sensor_mode < 0 || P->sensor_mode > 2) return ORA_EINVAL;
  if (P->central_L < 0 || P->central_L > 3) return ORA_EINVAL;
  if (P->weno_r != 0 && (P->weno_r < 2 || P->weno_r > 4)) return ORA_EINVAL;
  return ORA_OK;
}

/* ------------------------------------------------------------ work arrays */
typedef struct {
  geom g;
  double* W[5];               /* padded conserved */
  double *rho, *u, *v, *w, *p, *T, *Ht, *mu;   /* padded primitives */
  unsigned char* nflag;       /* padded node flags */
  unsigned char* iflag[3];    /* padded interface flags, interface i+1/2 at node i */
} work_t;

static void work_free(work_t* a) {
  for (int m = 0; m < 5; ++m) free(a->W[m]);
  free(a->rho); free(a->u); free(a->v); free(a->w); free(a->p); free(a->T); free(a->Ht);
  free(a->mu); free(a->nflag);
  for (int d = 0; d < 3; ++d) free(a->iflag[d]);
}

static int work_alloc(const ora_problem* P, work_t* a) {
  memset(a, 0, sizeof(*a));
  make_geom(P, &a->g);
  size_t n = a->g.np;
  int ok = 1;
  for (int m = 0; m < 5; ++m) ok &= (a->W[m] = calloc(n, sizeof(double))) != NULL;
  ok &= (a->rho = calloc(n, sizeof(double))) != NULL;
  ok &= (a->u = calloc(n, sizeof(double))) != NULL;
  ok &= (a->v = calloc(n, sizeof(double))) != NULL;
  ok &= (a->w = calloc(n, sizeof(double))) != NULL;
  ok &= (a->p = calloc(n, sizeof(double))) != NULL;
  ok &= (a->T = calloc(n, sizeof(double))) != NULL;
  ok &= (a->Ht = calloc(n, sizeof(double))) != NULL;
  ok &= (a->mu = calloc(n, sizeof(double))) != NULL;
  ok &= (a->nflag = calloc(n, 1)) != NULL;
  for (int d = 0; d < 3; ++d) ok &= (a->iflag[d] = calloc(n, 1)) != NULL;
  if (!ok) { work_free(a); return ORA_ENOMEM; }
  return ORA_OK;
}

/* load state, fill ghosts, compute primitives everywhere */
static int prepare(const ora_problem* P, const double* w, work_t* a) {
  const geom* g = &a->g;
  for (int m = 0; m < 5; ++m)
    for (int k = 0; k < g->nz; ++k)
      for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i)
          a->W[m][pidx(g, i, j, k)] = w[(size_t)m * g->nx * g->ny * g->nz + uidx(g, i, j, k)];
  int st = fill_ghosts(P, g, a->W);
  if (st != ORA_OK && st != ORA_ESTATE) return st;
  int bad = st == ORA_ESTATE;
  const int hw = g->hw;  /* layers beyond hw stay unset and unused */
#pragma omp parallel for reduction(| : bad)
  for (int k = -hw; k < g->nz + hw; ++k)
    for (int j = -hw; j < g->ny + hw; ++j)
      for (int i = -hw; i < g->nx + hw; ++i) {
        size_t q = pidx(g, i, j, k);
        double s5[5] = {a->W[0][q], a->W[1][q], a->W[2][q], a->W[3][q], a->W[4][q]};
        prim_t s = to_prim(P, g, s5);
        a->rho[q] = s.rho; a->u[q] = s.u; a->v[q] = s.v; a->w[q] = s.w;
        a->p[q] = s.p; a->T[q] = s.T; a->Ht[q] = s.Ht; a->mu[q] = s.mu;
        if (!(s.rho > 0.0) || !(s.T > 0.0) || !(s.p > 0.0)) bad = 1;
      }
  return bad ? ORA_ESTATE : ORA_OK;
}

/* ------------------------------------------------------------ derivatives
 * First and second derivatives of order 2L (Sec. 2.1).  The y direction
 * uses the computational coordinate eta with the analytic metric:
 * d/dy = (1/y_eta) d/deta,  d2/dy2 = (d2/deta2 - y_etaeta d/dy)/y_eta^2. */
static inline double d1(const double* f, size_t q, size_t s, double inv, int L) {
  double acc = 0.0;
  for (int l = 1; l <= L; ++l) acc += ACOEF[L][l - 1] * (f[q + l * s] - f[q - l * s]);
  return inv * acc;
}
static inline double d2(const double* f, size_t q, size_t s, double inv2, int L) {
  double acc = BCOEF[L][0] * f[q];
  for (int l = 1; l <= L; ++l) acc += BCOEF[L][l] * (f[q + l * s] + f[q - l * s]);
  return inv2 * acc;
}

/* ------------------------------------------------------------ shock sensor
 * Ducros sensor (Sec. 2.1, eq. sensor):
 * theta = max(-div u / sqrt(div^2 + |curl u|^2 + eps_s), 0), with the
 * regulariser eps_s = (u0/L0)^2 given per case (the printed form is read as
 * a squared inverse time scale).  Its velocity derivatives are of fourth
 * order whatever the order of the fluxes (the paper ties the sensor to no
 * scheme order). */
static void sensor_theta(const ora_problem* P, work_t* a, double* theta /* [N] or NULL */) {
  const geom* g = &a->g;
  size_t sx = 1, sy = (size_t)g->nxp, sz = (size_t)g->nxp * g->nyp;
#pragma omp parallel for
  for (int k = 0; k < g->nz; ++k)
    for (int j = 0; j < g->ny; ++j) {
      double iy = 1.0 / (g->deta * P->y_eta[j]);
      for (int i = 0; i < g->nx; ++i) {
        size_t q = pidx(g, i, j, k);
        double ux = d1(a->u, q, sx, 1.0 / g->dx, 2), uy = d1(a->u, q, sy, iy, 2);
        double uz = d1(a->u, q, sz, 1.0 / g->dz, 2);
        double vx = d1(a->v, q, sx, 1.0 / g->dx, 2), vy = d1(a->v, q, sy, iy, 2);
        double vz = d1(a->v, q, sz, 1.0 / g->dz, 2);
        double wx = d1(a->w, q, sx, 1.0 / g->dx, 2), wy = d1(a->w, q, sy, iy, 2);
        double wz = d1(a->w, q, sz, 1.0 / g->dz, 2);
        double div = ux + vy + wz;
        double ox = wy - vz, oy = uz - wx, oz = vx - uy;
        double den = sqrt(div * div + (ox * ox + oy * oy + oz * oz) + P->sensor_eps);
        double th = -div / den;
        if (th < 0.0) th = 0.0;
        if (theta) theta[uidx(g, i, j, k)] = th;
        a->nflag[q] = th > P->theta_star;
      }
    }
}

/* flags of ghost nodes: copies under periodicity, unflagged otherwise */
static void wrap_flags(const ora_problem* P, work_t* a) {
  const geom* g = &a->g;
  int per[3] = {P->bc_kind[0] == BC_PERIODIC, P->bc_kind[2] == BC_PERIODIC,
                P->bc_kind[4] == BC_PERIODIC};
  for (int k = -H; k < g->nz + H; ++k)
    for (int j = -H; j < g->ny + H; ++j)
      for (int i = -H; i < g->nx + H; ++i) {
        int ii = i, jj = j, kk = k, ghost = 0;
        if (i < 0 || i >= g->nx) { if (per[0]) ii = (i + g->nx) % g->nx; else ghost = 1; }
        if (j < 0 || j >= g->ny) { if (per[1]) jj = (j + g->ny) % g->ny; else ghost = 1; }
        if (k < 0 || k >= g->nz) { if (per[2]) kk = (k + g->nz) % g->nz; else ghost = 1; }
        if (ii == i && jj == j && kk == k) continue;
        a->nflag[pidx(g, i, j, k)] = ghost ? 0 : a->nflag[pidx(g, ii, jj, kk)];
      }
}

/* Interface flags: interface i+1/2 in direction d uses the shock-capturing
 * flux when the sensor mode forces it everywhere, or when any of the nodes
 * i-L+1..i+L (the stencil of the central flux of order 2L) is flagged.  The two boundary
 * interfaces of a non-periodic direction (walls and open boundaries) always
 * use the central flux. */
static void interface_flags(const ora_problem* P, work_t* a) {
  const geom* g = &a->g;
  int n[3] = {g->nx, g->ny, g->nz};
  size_t st[3] = {1, (size_t)g->nxp, (size_t)g->nxp * g->nyp};
  for (int d = 0; d < 3; ++d) {
    int per = P->bc_kind[2 * d] == BC_PERIODIC;
    for (int k = 0; k < g->nz; ++k)
      for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
          int id[3] = {i, j, k};
          size_t q = pidx(g, i, j, k);
          unsigned char f = 0;
          if (!per && id[d] == n[d] - 1) f = 0;
          else if (P->sensor_mode == 2) f = 1;
          else if (P->sensor_mode == 1)
            for (int o = 1 - g->L; o <= g->L; ++o)
              f |= a->nflag[(size_t)((ptrdiff_t)q + (ptrdiff_t)o * (ptrdiff_t)st[d])];
          a->iflag[d][q] = f;
        }
  }
}

/* ------------------------------------------------------------ Euler fluxes
 * The three-point average operator of Sec. 2.1 (eq. avg_operator),
 * (1/8)(F_a + F_b)(G_a + G_b)(H_a + H_b), appears below with F = rho,
 * G = u_n and H = phi. */

/* Energy-preserving central flux of order 2L at interface i+1/2, node i at
 * padded index q, stride s along the direction d (eq. encflux):
 *   f = 2 sum_{l=1}^{L} a_l sum_{m=0}^{l-1} avg(rho, u_n, phi)_{i-m,l},
 * phi = 1, u, v, w, H, with the average operator of eq. avg_operator,
 *   avg(F, G, H)_{i,l} = (1/8)(F_i + F_{i+l})(G_i + G_{i+l})(H_i + H_{i+l}).
 * The pressure term of the momentum equation is put in the same
 * conservative form with two-point averages,
 *   2 sum_l a_l sum_m (p_{i-m} + p_{i-m+l})/2.
 * Written out as the formula reads: each average is the product of its
 * three pair sums times 1/8, taken left to right; the inner sum runs over
 * m ascending, the outer over l ascending, plain additions throughout (the
 * file is compiled without contraction).  Output in natural component
 * order; conv/pres select the two parts (both for the full operator). */
static void central_flux(const work_t* a, size_t q, size_t s, int d, int conv, int pres,
                         double f[5]) {
  const double* un = d == 0 ? a->u : (d == 1 ? a->v : a->w);
  const double* r = a->rho;
  const double* phis[5] = {NULL, a->u, a->v, a->w, a->Ht};
  const int L = a->g.L;
  for (int c = 0; c < 5; ++c) {
    double outer = 0.0;
    for (int l = 1; l <= L; ++l) {
      double inner = 0.0;
      for (int m = 0; m < l; ++m) {
        size_t ia = q - (size_t)m * s, ib = q + (size_t)(l - m) * s;
        double phi_sum = c == 0 ? 1.0 + 1.0 : phis[c][ia] + phis[c][ib];
        inner += 0.125 * (r[ia] + r[ib]) * (un[ia] + un[ib]) * phi_sum;
      }
      outer += ACOEF[L][l - 1] * inner;
    }
    f[c] = conv ? 2.0 * outer : 0.0;
  }
  if (pres) {
    double outer = 0.0;
    for (int l = 1; l <= L; ++l) {
      double inner = 0.0;
      for (int m = 0; m < l; ++m) {
        size_t ia = q - (size_t)m * s, ib = q + (size_t)(l - m) * s;
        inner += (a->p[ia] + a->p[ib]) / 2.0;
      }
      outer += ACOEF[L][l - 1] * inner;
    }
    f[1 + d] += 2.0 * outer;
  }
}

/* Splitting constants of the local Lax-Friedrichs flux at interface i+1/2
 * (Sec. 2.1): for each characteristic field k (wave order u_n - c, u_n,
 * u_n, u_n, u_n + c) the largest |lambda_k| over the 2r stencil nodes
 * i-r+1..i+r, with the sound speed of each node. */
static void lf_alpha(const ora_problem* P, const work_t* a, size_t q, size_t s, int d,
                     double alpha[5]) {
  const double* un_all = d == 0 ? a->u : (d == 1 ? a->v : a->w);
  const int rw = a->g.r;
  for (int k = 0; k < 5; ++k) alpha[k] = 0.0;
  for (int t = 0; t < 2 * rw; ++t) {
    size_t qs = q + (size_t)((long)(t - rw + 1) * (long)s);
    double un = un_all[qs];
    double cs = sqrt(P->gamma * a->p[qs] / a->rho[qs]);
    double lam[5] = {fabs(un - cs), fabs(un), fabs(un), fabs(un), fabs(un + cs)};
    for (int k = 0; k < 5; ++k)
      if (lam[k] > alpha[k]) alpha[k] = lam[k];
  }
}

/* Shock-capturing flux at interface i+1/2 (Sec. 2.1): Lax-Friedrichs flux
 * vector splitting of the characteristic fields, each split flux
 * reconstructed with the WENO scheme of order 2r - 1 (the positive part
 * from cells i-r+1..i+r-1, the negative part mirrored about the interface
 * from cells i+r..i-r+2).  Eigenvectors at the Roe average of nodes i and
 * i+1; splitting constants from lf_alpha (local Lax-Friedrichs). */
static void weno_flux(const ora_problem* P, const work_t* a, size_t q, size_t s, int d,
                      double f[5]) {
  int pm[5];
  perm_of_dir(d, pm);
  const double* vel[3] = {a->u, a->v, a->w};
  /* Roe average */
  size_t qL = q, qR = q + s;
  double sl = sqrt(a->rho[qL]), sr = sqrt(a->rho[qR]);
  double uroe[3];
  for (int c = 0; c < 3; ++c) uroe[c] = (sl * vel[c][qL] + sr * vel[c][qR]) / (sl + sr);
  double Hroe = (sl * a->Ht[qL] + sr * a->Ht[qR]) / (sl + sr);
  double q2 = uroe[0] * uroe[0] + uroe[1] * uroe[1] + uroe[2] * uroe[2];
  double croe = sqrt((P->gamma - 1.0) * (Hroe - 0.5 * q2));
  double Rm[5][5], Lm[5][5];
  eigvecs_perm(P->gamma - 1.0, uroe[d], uroe[(d + 1) % 3], uroe[(d + 2) % 3], Hroe, croe, Rm, Lm);
  double alpha[5];
  lf_alpha(P, a, q, s, d, alpha);
  /* characteristic projections of the state and of the Euler flux (with
   * pressure) at the stencil nodes, node i-r+1+t */
  const int rw = a->g.r, ns = 2 * rw;
  double gp[8][5], gmn[8][5];
  double vch[8][5], gch[8][5];
  for (int t = 0; t < ns; ++t) {
    size_t qs = q + (size_t)((long)(t - rw + 1) * (long)s);
    double wn[5], fn[5];
    for (int c = 0; c < 5; ++c) wn[c] = a->W[pm[c]][qs];
    double un = vel[d][qs];
    fn[0] = a->rho[qs] * un;
    fn[1] = a->rho[qs] * un * un + a->p[qs];
    fn[2] = a->rho[qs] * un * vel[(d + 1) % 3][qs];
    fn[3] = a->rho[qs] * un * vel[(d + 2) % 3][qs];
    fn[4] = un * (a->W[4][qs] + a->p[qs]);
    for (int k = 0; k < 5; ++k) {
      double av = 0.0, ag = 0.0;
      for (int c = 0; c < 5; ++c) { av += Lm[k][c] * wn[c]; ag += Lm[k][c] * fn[c]; }
      vch[t][k] = av;
      gch[t][k] = ag;
    }
  }
  double ghat[5];
  for (int k = 0; k < 5; ++k) {
    for (int t = 0; t < ns; ++t) {
      gp[t][k] = 0.5 * (gch[t][k] + alpha[k] * vch[t][k]);
      gmn[t][k] = 0.5 * (gch[t][k] - alpha[k] * vch[t][k]);
    }
    double sp[7], sm[7];
    for (int t = 0; t < ns - 1; ++t) {
      sp[t] = gp[t][k];            /* i-r+1..i+r-1 */
      sm[t] = gmn[ns - 1 - t][k];  /* i+r..i-r+2 */
    }
    ghat[k] = ora_weno(rw, sp) + ora_weno(rw, sm);
  }
  for (int c = 0; c < 5; ++c) {
    double acc = 0.0;
    for (int k = 0; k < 5; ++k) acc += Rm[c][k] * ghat[k];
    f[pm[c]] = acc;
  }
}

static void euler_terms(const ora_problem* P, work_t* a, double* r) {
  const geom* g = &a->g;
  int conv = (P->terms & T_CONV) != 0, pres = (P->terms & T_PRES) != 0;
  size_t N = (size_t)g->nx * g->ny * g->nz;
  size_t st[3] = {1, (size_t)g->nxp, (size_t)g->nxp * g->nyp};
  int n[3] = {g->nx, g->ny, g->nz};
  for (int d = 0; d < 3; ++d) {
    int wall_lo = d == 1 && (P->bc_kind[2] == BC_WALL_ISO || P->bc_kind[2] == BC_WALL_ADIA);
    int wall_hi = d == 1 && (P->bc_kind[3] == BC_WALL_ISO || P->bc_kind[3] == BC_WALL_ADIA);
    /* lines along d */
    int o1 = (d + 1) % 3, o2 = (d + 2) % 3;
#pragma omp parallel for collapse(2)
    for (int b2 = 0; b2 < n[o2]; ++b2)
      for (int b1 = 0; b1 < n[o1]; ++b1) {
        double (*F)[5] = malloc(sizeof(double[5]) * (size_t)(n[d] + 1));
        for (int ii = -1; ii < n[d]; ++ii) {
          int id[3];
          id[d] = ii; id[o1] = b1; id[o2] = b2;
          size_t q = pidx(g, id[0], id[1], id[2]);
          double f[5];
          int boundary = (ii == -1) || (ii == n[d] - 1);
          int use_weno = 0;
          if (P->sensor_mode > 0 && ii >= 0) use_weno = a->iflag[d][q];
          if (P->sensor_mode > 0 && ii == -1) {
            /* interface -1/2 is the periodic image of n-1/2 */
            int idw[3] = {id[0], id[1], id[2]};
            idw[d] = n[d] - 1;
            use_weno = a->iflag[d][pidx(g, idw[0], idw[1], idw[2])];
          }
          (void)boundary;
          if (use_weno) weno_flux(P, a, q, st[d], d, f);
          else central_flux(a, q, st[d], d, conv, pres, f);
          if ((ii == -1 && wall_lo) || (ii == n[d] - 1 && wall_hi)) {
            /* staggered wall: convective fluxes vanish, only pressure acts */
            double fp[5];
            central_flux(a, q, st[d], d, 0, pres, fp);
            for (int c = 0; c < 5; ++c) f[c] = fp[c];
          }
          for (int c = 0; c < 5; ++c) F[ii + 1][c] = f[c];
        }
        for (int ii = 0; ii < n[d]; ++ii) {
          int id[3];
          id[d] = ii; id[o1] = b1; id[o2] = b2;
          /* flux difference times the inverse local spacing (eq. num_flux) */
          double inv = d == 0 ? 1.0 / g->dx : (d == 2 ? 1.0 / g->dz : 1.0 / (g->deta * P->y_eta[id[1]]));
          size_t u = uidx(g, id[0], id[1], id[2]);
          for (int c = 0; c < 5; ++c) r[(size_t)c * N + u] -= (F[ii + 1][c] - F[ii][c]) * inv;
        }
        free(F);
      }
  }
}

/* ------------------------------------------------------------ viscous terms
 * Laplacian form (Sec. 2.1): d/dx_j (mu du/dx_j) = dmu/dx_j du/dx_j +
 * mu d2u/dx_j2 with first and second derivatives of order 2L; the stress
 * divergence expands to
 *   F_i = mu (lap u_i + (1/3) d_i div) + d_j mu (d_j u_i + d_i u_j) - (2/3) d_i mu div,
 * the energy equation receives u_i F_i + sigma_ij d_j u_i (the work of the
 * stresses) plus k lap T + d_j k d_j T (heat conduction, k = c_p mu/Pr).
 * Mixed derivatives are first derivatives of first derivatives:
 * d_x d_y f = D_y(D_x f), d_x d_z f = D_z(D_x f), d_y d_z f = D_z(D_y f). */
static void viscous_terms(const ora_problem* P, work_t* a, double* r) {
  const geom* g = &a->g;
  size_t N = (size_t)g->nx * g->ny * g->nz;
  size_t sx = 1, sy = (size_t)g->nxp, sz = (size_t)g->nxp * g->nyp;
  double ix = 1.0 / g->dx, iz = 1.0 / g->dz;
  double ix2 = ix * ix, iz2 = iz * iz, ie2 = 1.0 / (g->deta * g->deta);
  double kfac = g->cp / P->Pr;
  const int L = g->L;
#pragma omp parallel for
  for (int k = 0; k < g->nz; ++k)
    for (int j = 0; j < g->ny; ++j) {
      double ye = P->y_eta[j], yee = P->y_etaeta[j];
      double iy = 1.0 / (g->deta * ye);
      for (int i = 0; i < g->nx; ++i) {
        size_t q = pidx(g, i, j, k);
        const double* fld[4] = {a->u, a->v, a->w, a->T};
        double gx[4], gy[4], gz[4], lap[4];
        for (int f = 0; f < 4; ++f) {
          gx[f] = d1(fld[f], q, sx, ix, L);
          gy[f] = d1(fld[f], q, sy, iy, L);
          gz[f] = d1(fld[f], q, sz, iz, L);
          double fxx = d2(fld[f], q, sx, ix2, L);
          double fyy = (d2(fld[f], q, sy, ie2, L) - yee * gy[f]) / (ye * ye);
          double fzz = d2(fld[f], q, sz, iz2, L);
          lap[f] = fxx + fyy + fzz;
        }
        double uxx = d2(a->u, q, sx, ix2, L);
        double vyy = (d2(a->v, q, sy, ie2, L) - yee * gy[1]) / (ye * ye);
        double wzz = d2(a->w, q, sz, iz2, L);
        /* mixed derivatives as compositions of first derivatives; the
         * windows hold the inner derivative at offsets -L..L */
        double ux_at[7], vx_at[7], ux_z[7], wx_z[7], vy_z[7], wy_z[7];
        for (int l = -L; l <= L; ++l) {
          size_t qy = q + (size_t)((long)l * (long)sy);
          ux_at[l + L] = d1(a->u, qy, sx, ix, L);
          vx_at[l + L] = d1(a->v, qy, sx, ix, L);
          size_t qz = q + (size_t)((long)l * (long)sz);
          ux_z[l + L] = d1(a->u, qz, sx, ix, L);
          wx_z[l + L] = d1(a->w, qz, sx, ix, L);
          vy_z[l + L] = d1(a->v, qz, sy, iy, L);
          wy_z[l + L] = d1(a->w, qz, sy, iy, L);
        }
        double uxy = d1(ux_at, L, 1, iy, L), vxy = d1(vx_at, L, 1, iy, L);
        double uxz = d1(ux_z, L, 1, iz, L), wxz = d1(wx_z, L, 1, iz, L);
        double vyz = d1(vy_z, L, 1, iz, L), wyz = d1(wy_z, L, 1, iz, L);
        double mux = d1(a->mu, q, sx, ix, L), muy = d1(a->mu, q, sy, iy, L);
        double muz = d1(a->mu, q, sz, iz, L);
        double mu = a->mu[q];
        double ux = gx[0], uy = gy[0], uz = gz[0];
        double vx = gx[1], vy = gy[1], vz = gz[1];
        double wx = gx[2], wy = gy[2], wz = gz[2];
        double div = ux + vy + wz;
        double ddx = uxx + vxy + wxz;  /* d/dx div */
        double ddy = uxy + vyy + wyz;  /* d/dy div */
        double ddz = uxz + vyz + wzz;  /* d/dz div */
        double Fx = mu * (lap[0] + ddx / 3.0) + mux * (ux + ux) + muy * (uy + vx) + muz * (uz + wx)
                    - 2.0 / 3.0 * mux * div;
        double Fy = mu * (lap[1] + ddy / 3.0) + mux * (vx + uy) + muy * (vy + vy) + muz * (vz + wy)
                    - 2.0 / 3.0 * muy * div;
        double Fz = mu * (lap[2] + ddz / 3.0) + mux * (wx + uz) + muy * (wy + vz) + muz * (wz + wz)
                    - 2.0 / 3.0 * muz * div;
        /* sigma_ij d_j u_i */
        double sxx = mu * (2.0 * ux - 2.0 / 3.0 * div);
        double syy = mu * (2.0 * vy - 2.0 / 3.0 * div);
        double szz = mu * (2.0 * wz - 2.0 / 3.0 * div);
        double sxy = mu * (uy + vx), sxz = mu * (uz + wx), syz = mu * (vz + wy);
        double phi = sxx * ux + syy * vy + szz * wz + sxy * (uy + vx) + sxz * (uz + wx) + syz * (vz + wy);
        double kk = kfac * mu;
        double heat = kk * lap[3] + kfac * (mux * gx[3] + muy * gy[3] + muz * gz[3]);
        size_t uq = uidx(g, i, j, k);
        double uu = a->u[q], vv = a->v[q], ww = a->w[q];
        r[1 * N + uq] += Fx;
        r[2 * N + uq] += Fy;
        r[3 * N + uq] += Fz;
        r[4 * N + uq] += uu * Fx + vv * Fy + ww * Fz + phi + heat;
      }
    }
}

/* ------------------------------------------------------------ bulk forcing
 * Constant mass flow (Sec. 2): a uniform streamwise body force f chosen so
 * that the volume integral of the streamwise momentum residual vanishes,
 * f = -sum(R_rhou dV)/sum(dV) with dV proportional to y_eta; its power f u
 * enters the energy equation.  Applied at every stage evaluation.  The sum
 * runs in a fixed serial order. */
static double apply_forcing(const ora_problem* P, const work_t* a, double* r) {
  const geom* g = &a->g;
  size_t N = (size_t)g->nx * g->ny * g->nz;
  double num = 0.0, den = 0.0;
  for (int k = 0; k < g->nz; ++k)
    for (int j = 0; j < g->ny; ++j)
      for (int i = 0; i < g->nx; ++i) {
        num += r[1 * N + uidx(g, i, j, k)] * P->y_eta[j];
        den += P->y_eta[j];
      }
  double f = -num / den;
  for (int k = 0; k < g->nz; ++k)
    for (int j = 0; j < g->ny; ++j)
      for (int i = 0; i < g->nx; ++i) {
        size_t u = uidx(g, i, j, k);
        r[1 * N + u] += f;
        r[4 * N + u] += f * a->u[pidx(g, i, j, k)];
      }
  return f;
}

/* ------------------------------------------------------------ entry points */
static int rhs_core(const ora_problem* P, const double* w, double* r, double* theta,
                    unsigned char* nflags, unsigned char* iflags, double* fout) {
  int st = validate(P);
  if (st) return st;
  work_t a;
  if (work_alloc(P, &a)) return ORA_ENOMEM;
  st = prepare(P, w, &a);
  if (st) { work_free(&a); return st; }
  const geom* g = &a.g;
  size_t N = (size_t)g->nx * g->ny * g->nz;
  if (P->sensor_mode == 1) {
    sensor_theta(P, &a, theta);
    wrap_flags(P, &a);
  } else if (theta) {
    memset(theta, 0, N * sizeof(double));
  }
  interface_flags(P, &a);
  if (nflags || iflags)
    for (int k = 0; k < g->nz; ++k)
      for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
          size_t q = pidx(g, i, j, k), u = uidx(g, i, j, k);
          if (nflags) nflags[u] = a.nflag[q];
          if (iflags)
            iflags[u] = (unsigned char)(a.iflag[0][q] | (a.iflag[1][q] << 1) | (a.iflag[2][q] << 2));
        }
  memset(r, 0, 5 * N * sizeof(double));
  euler_terms(P, &a, r);
  if (P->viscous && (P->terms & T_VISC)) viscous_terms(P, &a, r);
  double f = 0.0;
  if (P->forcing && (P->terms & T_FORCE)) f = apply_forcing(P, &a, r);
  if (fout) *fout = f;
  work_free(&a);
  return ORA_OK;
}

/* Full right-hand side R(w) of the semi-discrete system dw/dt = R(w)
 * (Sec. 2.2).  theta (node sensor values), nflags (node flags) and iflags
 * (bit d set when interface i+1/2 in direction d is shock-capturing) are
 * optional outputs; forcing_out receives the bulk force. */
/* A copy Q of the problem whose digital-filter inflow (if any, and without
 * a plane of its own) uses the generator's initial plane (key 0), held in
 * *buf until the caller frees it. */
static int with_inflow_plane(const ora_problem* P, ora_problem* Q, double** buf) {
  *Q = *P;
  *buf = NULL;
  if (P->bc_kind[0] != BC_DF_INFLOW || P->df_plane) return ORA_OK;
  int st = validate(P);
  if (st) return st;
  size_t np = (size_t)P->nz * P->ny;
  double* psi = malloc(3 * np * sizeof(double));
  double* plane = malloc(5 * np * sizeof(double));
  if (!psi || !plane) { free(psi); free(plane); return ORA_ENOMEM; }
  st = ora_df_update(P, 0, 0.0, 1, psi, plane, NULL);
  free(psi);
  if (st) { free(plane); return st; }
  Q->df_plane = plane;
  *buf = plane;
  return ORA_OK;
}

int ora_rhs(const ora_problem* P, const double* w, double* r, double* theta,
            unsigned char* nflags, unsigned char* iflags, double* forcing_out) {
  ora_problem Q;
  double* plane;
  int st = with_inflow_plane(P, &Q, &plane);
  if (!st) st = rhs_core(&Q, w, r, theta, nflags, iflags, forcing_out);
  free(plane);
  return st;
}

/* Time step (the paper gives no rule): dt = CFL * min(1/max_i sum_d (|u_d|+c)/dx_d,
 * 2.5/max_i [max(4/3, gamma/Pr) (mu/rho) rho_2 sum_d dx_d^-2]); 2.5 is about
 * the real-axis stability bound of the RK3 scheme and rho_2 the largest
 * magnitude of the symbol of the second derivative in use (4, 16/3 and
 * 272/45 for orders 2, 4 and 6). */
int ora_dt(const ora_problem* P, const double* w, double cfl, double* dt_out) {
  int st = validate(P);
  if (st) return st;
  geom g;
  make_geom(P, &g);
  size_t N = (size_t)g.nx * g.ny * g.nz;
  double cmax = 0.0, vmax = 0.0;
  double vf = 4.0 / 3.0 > P->gamma / P->Pr ? 4.0 / 3.0 : P->gamma / P->Pr;
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j) {
      double dy = g.deta * P->y_eta[j];
      for (int i = 0; i < g.nx; ++i) {
        size_t u = uidx(&g, i, j, k);
        double q[5] = {w[u], w[N + u], w[2 * N + u], w[3 * N + u], w[4 * N + u]};
        prim_t s = to_prim(P, &g, q);
        double c = sqrt(P->gamma * s.p / s.rho);
        double conv = (fabs(s.u) + c) / g.dx + (fabs(s.v) + c) / dy + (fabs(s.w) + c) / g.dz;
        if (conv > cmax) cmax = conv;
        if (P->viscous) {
          double vis = vf * (s.mu / s.rho) * (1.0 / (g.dx * g.dx) + 1.0 / (dy * dy) + 1.0 / (g.dz * g.dz));
          if (vis > vmax) vmax = vis;
        }
      }
    }
  double dt = 1.0 / cmax;
  if (P->viscous && vmax > 0.0) {
    double dv = 2.5 / (D2RHO[g.L] * vmax);
    if (dv < dt) dt = dv;
  }
  *dt_out = cfl * dt;
  return ORA_OK;
}

/* One low-storage stage: out = w + dt (alpha_l rprev + beta_l r). */
void ora_rk_stage(size_t n, const double* w, const double* r, const double* rprev, double dt,
                  int l, double* out) {
  for (size_t i = 0; i < n; ++i) {
    double acc = RK_BETA[l] * r[i];
    if (l > 0) acc += RK_ALPHA[l] * rprev[i];
    out[i] = w[i] + dt * acc;
  }
}

/* Advance nsteps RK3 steps in place.  dt_fixed > 0 overrides the CFL rule;
 * otherwise dt is taken from the state at the start of each step.  dts (if
 * not NULL, length nsteps) receives the steps used.  With digital-filter
 * inflow the generator starts from its initial plane (key 0) and is
 * updated at the start of every step s with key s + 1, so one call of
 * nsteps steps is the reference for a fresh GPU context. */
int ora_advance(const ora_problem* P, double* w, int nsteps, double cfl, double dt_fixed,
                double* dts) {
  int st = validate(P);
  if (st) return st;
  size_t N = (size_t)P->nx * P->ny * P->nz, n5 = 5 * N;
  double* r = malloc(n5 * sizeof(double));
  double* rp = malloc(n5 * sizeof(double));
  double* ws = malloc(n5 * sizeof(double));
  const int df = P->bc_kind[0] == BC_DF_INFLOW;
  size_t np = (size_t)P->nz * P->ny;
  double* psi = df ? malloc(3 * np * sizeof(double)) : NULL;
  double* plane = df ? malloc(5 * np * sizeof(double)) : NULL;
  if (!r || !rp || !ws || (df && (!psi || !plane))) {
    free(r); free(rp); free(ws); free(psi); free(plane);
    return ORA_ENOMEM;
  }
  ora_problem Q = *P;
  if (df) {
    st = ora_df_update(P, 0, 0.0, 1, psi, plane, NULL);
    Q.df_plane = plane;
  }
  for (int step = 0; step < nsteps && st == ORA_OK; ++step) {
    double dt = dt_fixed;
    if (!(dt_fixed > 0.0)) {
      st = ora_dt(P, w, cfl, &dt);
      if (st) break;
    }
    if (dts) dts[step] = dt;
    if (df && (st = ora_df_update(P, (uint64_t)step + 1, dt, 0, psi, plane, NULL))) break;
    for (int l = 0; l < 3; ++l) {
      st = rhs_core(&Q, w, r, NULL, NULL, NULL, NULL);
      if (st) break;
      ora_rk_stage(n5, w, r, rp, dt, l, ws);
      memcpy(w, ws, n5 * sizeof(double));
      double* t = rp; rp = r; r = t;
    }
  }
  free(r); free(rp); free(ws); free(psi); free(plane);
  return st;
}

/* Volume-weighted totals (dV = dx dz deta y_eta): mass, momentum x,y,z,
 * total energy and kinetic energy. */
int ora_totals(const ora_problem* P, const double* w, double* out6) {
  geom g;
  make_geom(P, &g);
  size_t N = (size_t)g.nx * g.ny * g.nz;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j) {
      double dv = g.dx * g.dz * g.deta * P->y_eta[j];
      for (int i = 0; i < g.nx; ++i) {
        size_t u = uidx(&g, i, j, k);
        for (int m = 0; m < 5; ++m) acc[m] += w[m * N + u] * dv;
        acc[5] += 0.5 * (w[N + u] * w[N + u] + w[2 * N + u] * w[2 * N + u] + w[3 * N + u] * w[3 * N + u])
                  / w[u] * dv;
      }
    }
  for (int m = 0; m < 6; ++m) out6[m] = acc[m];
  return ORA_OK;
}

/* Extrema of the state: out4 = {min rho, min p, max |u|/c, number of
 * non-finite conserved values}, with the primitives of the perfect gas
 * (Sec. 2) and the sound speed c = sqrt(gamma p / rho).  Points holding a
 * non-finite value are counted and left out of the extrema. */
int ora_extrema(const ora_problem* P, const double* w, double* out4) {
  geom g;
  make_geom(P, &g);
  size_t N = (size_t)g.nx * g.ny * g.nz;
  double rmin = INFINITY, pmin = INFINITY, mmax = 0.0, bad = 0.0;
  for (size_t n = 0; n < N; ++n) {
    double q[5];
    int fin = 1;
    for (int m = 0; m < 5; ++m) {
      q[m] = w[m * N + n];
      if (!isfinite(q[m])) {
        bad += 1.0;
        fin = 0;
      }
    }
    if (!fin) continue;
    prim_t s = to_prim(P, &g, q);
    if (s.rho < rmin) rmin = s.rho;
    if (s.p < pmin) pmin = s.p;
    double c = sqrt(P->gamma * s.p / s.rho);
    double mach = sqrt(s.u * s.u + s.v * s.v + s.w * s.w) / c;
    if (mach > mmax) mmax = mach;
  }
  out4[0] = rmin;
  out4[1] = pmin;
  out4[2] = mmax;
  out4[3] = bad;
  return ORA_OK;
}

/* Running statistics (the quantities behind the mean profiles and stresses
 * of Sec. 4): for every (i, j) column, the spanwise sums (k ascending) of
 * rho, rho u, rho v, rho w, rho u u, rho v v, rho w w, rho u v, u, u u, T,
 * rho T, T T, p, p p, rho rho are added to acc[16][ny][nx], with
 * u = (rho u)/rho, T = (E/rho - |u|^2/2)/c_v, p = rho R T. */
int ora_stats(const ora_problem* P, const double* w, double* acc) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const size_t N = (size_t)nx * ny * nz, plane = (size_t)nx * ny;
  const double icv = (P->gamma - 1.0) / P->R_gas;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double a[16] = {0};
      for (int k = 0; k < nz; ++k) {
        size_t n = (size_t)k * plane + (size_t)j * nx + i;
        double r = w[n], ir = 1.0 / r;
        double u = w[N + n] * ir, v = w[2 * N + n] * ir, ww = w[3 * N + n] * ir;
        double T = (w[4 * N + n] * ir - 0.5 * (u * u + v * v + ww * ww)) * icv;
        double p = r * P->R_gas * T;
        double ru = w[N + n], rv = w[2 * N + n], rw = w[3 * N + n];
        double q[16] = {r, ru, rv, rw, ru * u, rv * v, rw * ww, ru * v, u, u * u, T, r * T,
                        T * T, p, p * p, r * r};
        for (int m = 0; m < 16; ++m) a[m] += q[m];
      }
      for (int m = 0; m < 16; ++m) acc[(size_t)m * plane + (size_t)j * nx + i] += a[m];
    }
  return ORA_OK;
}

/* Mean fields from the accumulated sums acc[16][ny][nx] of `samples`
 * states: with m = sums / (samples nz), or the x sums (i ascending) divided
 * by samples nz nx when average_x, out[16][ny][nx] (or [16][ny]) holds the
 * Reynolds mean density, the Favre mean velocities, the Favre stresses
 * R11, R22, R33, R12, u and its rms, T, the Favre mean T, the rms of T,
 * p and its rms, and the rms of rho; the rms values from the second
 * moments, clipped at zero (Favre average: rho-weighted mean; Favre
 * stress: rho-weighted mean of the product of the fluctuations about the
 * Favre means). */
int ora_stats_means(const ora_problem* P, const double* acc, long samples, int average_x,
                    double* out) {
  if (samples <= 0) return ORA_EINVAL;
  const int nx = P->nx, ny = P->ny;
  const size_t plane = (size_t)nx * ny;
  const int ncol = average_x ? ny : nx * ny;
  const double cnt = (double)samples * P->nz * (average_x ? nx : 1);
  for (int c = 0; c < ncol; ++c) {
    double m[16];
    for (int q = 0; q < 16; ++q) {
      double s = 0.0;
      if (average_x)
        for (int i = 0; i < nx; ++i) s += acc[(size_t)q * plane + (size_t)c * nx + i];
      else
        s = acc[(size_t)q * plane + (size_t)c];
      m[q] = s / cnt;
    }
    const double rho = m[0];
    const double uf = m[1] / rho, vf = m[2] / rho, wf = m[3] / rho;
    const double o[16] = {rho, uf, vf, wf,
                          m[4] / rho - uf * uf, m[5] / rho - vf * vf, m[6] / rho - wf * wf,
                          m[7] / rho - uf * vf,
                          m[8], sqrt(fmax(m[9] - m[8] * m[8], 0.0)),
                          m[10], m[11] / rho, sqrt(fmax(m[12] - m[10] * m[10], 0.0)),
                          m[13], sqrt(fmax(m[14] - m[13] * m[13], 0.0)),
                          sqrt(fmax(m[15] - rho * rho, 0.0))};
    for (int q = 0; q < 16; ++q) out[(size_t)q * ncol + c] = o[q];
  }
  return ORA_OK;
}

int ora_num_threads(void) {
  int n = 1;
#ifdef _OPENMP
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
#endif
  return n;
}

/* Thread count of the following parallel loops (n >= 1; a no-op without
 * OpenMP); returns the previous count.  For timing only: every result is
 * independent of the thread count. */
int ora_set_threads(int n) {
  int prev = ora_num_threads();
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
  return prev;
}

/* Test hook: the interface fluxes of direction d exactly as used by the
 * right-hand side (central, shock-capturing or wall), interface i+1/2
 * stored at node i, layout out[5][nz][ny][nx]. */
int ora_iface_flux(const ora_problem* P, const double* w, int d, double* out) {
  int st = validate(P);
  if (st) return st;
  if (P->bc_kind[0] == BC_DF_INFLOW && !P->df_plane) {
    ora_problem Q;
    double* plane;
    st = with_inflow_plane(P, &Q, &plane);
    if (!st) st = ora_iface_flux(&Q, w, d, out);
    free(plane);
    return st;
  }
  work_t a;
  if (work_alloc(P, &a)) return ORA_ENOMEM;
  st = prepare(P, w, &a);
  if (st) { work_free(&a); return st; }
  const geom* g = &a.g;
  size_t N = (size_t)g->nx * g->ny * g->nz;
  if (P->sensor_mode == 1) { sensor_theta(P, &a, NULL); wrap_flags(P, &a); }
  interface_flags(P, &a);
  size_t stv[3] = {1, (size_t)g->nxp, (size_t)g->nxp * g->nyp};
  int wall_hi = d == 1 && (P->bc_kind[3] == BC_WALL_ISO || P->bc_kind[3] == BC_WALL_ADIA);
  int n[3] = {g->nx, g->ny, g->nz};
  for (int k = 0; k < g->nz; ++k)
    for (int j = 0; j < g->ny; ++j)
      for (int i = 0; i < g->nx; ++i) {
        size_t q = pidx(g, i, j, k);
        int id[3] = {i, j, k};
        double f[5];
        if (P->sensor_mode > 0 && a.iflag[d][q]) weno_flux(P, &a, q, stv[d], d, f);
        else central_flux(&a, q, stv[d], d, 1, 1, f);
        if (wall_hi && id[d] == n[d] - 1) central_flux(&a, q, stv[d], d, 0, 1, f);
        for (int c = 0; c < 5; ++c) out[(size_t)c * N + uidx(g, i, j, k)] = f[c];
      }
  work_free(&a);
  return ORA_OK;
}

/* Test hook: the ghost layers of a y face (2: y-, 3: y+) as filled for the
 * right-hand side, out[5][hw][nz][nx + 2 hw] (conserved variables; layer
 * s-1 holds ghost s, i.e. row -s below or row ny-1+s above, over the
 * x-extended range i = -hw..nx+hw-1); *hw_out receives hw. */
int ora_ghosts_y(const ora_problem* P, const double* w, int face, double* out, int* hw_out) {
  int st = validate(P);
  if (st) return st;
  if (face != 2 && face != 3) return ORA_EINVAL;
  if (P->bc_kind[0] == BC_DF_INFLOW && !P->df_plane) {
    ora_problem Q;
    double* plane;
    st = with_inflow_plane(P, &Q, &plane);
    if (!st) st = ora_ghosts_y(&Q, w, face, out, hw_out);
    free(plane);
    return st;
  }
  work_t a;
  if (work_alloc(P, &a)) return ORA_ENOMEM;
  st = prepare(P, w, &a);
  if (st != ORA_OK && st != ORA_ESTATE) { work_free(&a); return st; }
  const geom* g = &a.g;
  const int hw = g->hw, nxe = g->nx + 2 * hw;
  for (int m = 0; m < 5; ++m)
    for (int s = 1; s <= hw; ++s)
      for (int k = 0; k < g->nz; ++k)
        for (int i = -hw; i < g->nx + hw; ++i) {
          int j = face == 2 ? -s : g->ny - 1 + s;
          out[(((size_t)m * hw + (s - 1)) * g->nz + k) * nxe + (i + hw)] = a.W[m][pidx(g, i, j, k)];
        }
  *hw_out = hw;
  work_free(&a);
  return st;
}

/* Test hook: the Lax-Friedrichs splitting constants used by the
 * shock-capturing flux at interface i+1/2 of direction d (node (i, j, k)). */
int ora_lf_alpha(const ora_problem* P, const double* w, int d, int i, int j, int k,
                 double* alpha) {
  int st = validate(P);
  if (st) return st;
  if (P->bc_kind[0] == BC_DF_INFLOW && !P->df_plane) {
    ora_problem Q;
    double* plane;
    st = with_inflow_plane(P, &Q, &plane);
    if (!st) st = ora_lf_alpha(&Q, w, d, i, j, k, alpha);
    free(plane);
    return st;
  }
  if (d < 0 || d > 2 || i < 0 || i >= P->nx || j < 0 || j >= P->ny || k < 0 || k >= P->nz)
    return ORA_EINVAL;
  work_t a;
  if (work_alloc(P, &a)) return ORA_ENOMEM;
  st = prepare(P, w, &a);
  if (st) { work_free(&a); return st; }
  size_t stv[3] = {1, (size_t)a.g.nxp, (size_t)a.g.nxp * a.g.nyp};
  lf_alpha(P, &a, pidx(&a.g, i, j, k), stv[d], d, alpha);
  work_free(&a);
  return ORA_OK;
}
