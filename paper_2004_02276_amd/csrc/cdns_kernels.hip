// cdns_kernels.hip -- HIP kernels (gfx950) for the right-hand side and the
// low-storage RK3 step of the compressible Navier-Stokes equations following
// Sec. 2 of "STREAmS" (arXiv 2004.02276).
//
// Per stage (all on one stream, no host synchronisation):
//   ghosts   x-face then y-face ghost planes of non-periodic faces
//   sensor   Ducros sensor in FP64 with the node flag theta > theta*
//   iflags   interface flags (OR over the central stencil), compaction
//            into one node-ordered list of interfaces per direction and a
//            per-node slot (list position or -1)
//   weno     Lax-Friedrichs characteristic WENO flux (order 3, 5 or 7) on
//            the listed interfaces, stored compacted at the list position
//   rhs      fused central convective + pressure flux in x, y, z and
//            Laplacian-form viscous/heat terms (order 2L = 2, 4 or 6),
//            2.5-D tiling: an (x,y) tile with an L-node halo is staged in
//            LDS plane by plane while each thread keeps its own z column in
//            registers; flagged interfaces take the compacted WENO flux
//            through their slot
//   force    bulk force from the per-block partial sums (fixed order)
//   rk       w' = w + dt (alpha R_prev + beta R), forcing applied here
//
// State layout: w[5][nz][ny][nx] (x fastest); every kernel reads and writes
// x-contiguous rows, so a wavefront touches 512 contiguous bytes per field.
#include <hip/hip_runtime.h>

#include <mutex>
#include <utility>

#include "cdns_internal.h"

namespace cdns {

// Central finite-difference coefficients of order 2L (Sec. 2.1), L = 1..3:
// first derivative a_l (l = 1..L), second derivative b_l (l = 0..L).
__host__ __device__ constexpr double coef_a(int L, int l) {
  return L == 1 ? 0.5
       : L == 2 ? (l == 1 ? 2.0 / 3.0 : -1.0 / 12.0)
                : (l == 1 ? 3.0 / 4.0 : (l == 2 ? -3.0 / 20.0 : 1.0 / 60.0));
}
// Fourth-order first-derivative weights of the shock sensor (its order does
// not follow the flux order).
#define CA1 (2.0 / 3.0)
#define CA2 (-1.0 / 12.0)

__host__ __device__ constexpr double coef_b(int L, int l) {
  return L == 1 ? (l == 0 ? -2.0 : 1.0)
       : L == 2 ? (l == 0 ? -5.0 / 2.0 : (l == 1 ? 4.0 / 3.0 : -1.0 / 12.0))
                : (l == 0 ? -49.0 / 18.0 : (l == 1 ? 3.0 / 2.0 : (l == 2 ? -3.0 / 20.0 : 1.0 / 90.0)));
}

// consecutive logical tiles land on the same XCD (blocks are dealt
// round-robin over the 8 XCDs), so neighbouring tiles share an L2
__device__ __forceinline__ int xcd_swizzle_blk(int b, int nb) {
  return (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
}

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// periodic wrap of an index within one period of the range: -n <= i < 2n
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// q = n / d and rem = n % d for 0 <= n < 2^31, d >= 1, rd = 1/d: the double
// estimate is within 2^-21 of the exact quotient, so truncation is off by at
// most one and one correction step makes it exact.
__device__ __forceinline__ int qdiv(int n, int d, double rd, int& rem) {
  int q = (int)((double)n * rd);
  int r = n - q * d;
  if (r < 0) {
    --q;
    r += d;
  } else if (r >= d) {
    ++q;
    r -= d;
  }
  rem = r;
  return q;
}

__device__ __forceinline__ size_t nidx(const Desc& D, int i, int j, int k) {
  return ((size_t)k * D.ny + (size_t)j) * D.nx + (size_t)i;
}

// 32-bit node index (the point count is below 2^31, checked at creation)
__device__ __forceinline__ int nidx32(const Desc& D, int i, int j, int k) {
  return (k * D.ny + j) * D.nx + i;
}

__device__ __forceinline__ void from_prim(const Desc& D, double r, double u, double v, double w,
                                          double p, double q[5]) {
#pragma clang fp contract(off)
  q[0] = r;
  q[1] = r * u;
  q[2] = r * v;
  q[3] = r * w;
  q[4] = p / D.gm1 + 0.5 * r * (u * u + v * v + w * w);
}

// Ghost node of a staggered wall (y face `side`) from its mirror image qm:
// velocity reversed, pressure copied, temperature 2 T_w - T (isothermal) or
// T (adiabatic).  A non-positive ghost temperature is reported in the
// status word.  Without contraction, so that its bits do not depend on the
// kernel that evaluates it (single and batched ghost fills).
__device__ __forceinline__ void wall_ghost(const Desc& D, int kind, int side, const double qm[5],
                                           double q[5]) {
#pragma clang fp contract(off)
  const double rr = qm[0], ir = 1.0 / rr;
  const double u = qm[1] * ir, v = qm[2] * ir, ww = qm[3] * ir;
  const double T = (qm[4] * ir - 0.5 * (u * u + v * v + ww * ww)) * D.icv;
  const double p = rr * D.R * T;
  const double Tg = kind == BC_WALL_ISO ? 2.0 * D.bcp[2 + side][0] - T : T;
  if (!(Tg > 0.0)) atomicOr(D.status, (unsigned)ST_BAD_GHOST);
  from_prim(D, p / (D.R * Tg), -u, -v, -ww, p, q);
}

__host__ __device__ __forceinline__ bool is_wall(int kind) {
  return kind == BC_WALL_ISO || kind == BC_WALL_ADIA;
}

// Conserved variables at any node index (interior, periodic image or ghost
// plane).  Resolution order follows the ghost fill order: z (periodic), then
// y ghost planes (which already hold the x-extended range), then x.
__device__ __forceinline__ void load_node(const Desc& D, const double* __restrict__ w, int i,
                                          int j, int k, double q[5]) {
  k = wrapi(k, D.nz);
  if (j < 0 || j >= D.ny) {
    if (D.per_y) {
      j = wrapi(j, D.ny);
    } else {
      const int side = j < 0 ? 0 : 1;
      int s = j < 0 ? -j : j - D.ny + 1;
      s = s > kHalo ? kHalo : s;
      int ii = i < -kHalo ? -kHalo : (i > D.nx + kHalo - 1 ? D.nx + kHalo - 1 : i);
      const double* g = D.gy[side];
      const size_t mst = (size_t)kHalo * D.nz * D.nxg;
      const size_t b = ((size_t)(s - 1) * D.nz + k) * D.nxg + (size_t)(ii + kHalo);
#pragma unroll
      for (int m = 0; m < 5; ++m) q[m] = g[m * mst + b];
      return;
    }
  }
  if (i < 0 || i >= D.nx) {
    if (D.per_x) {
      i = wrapi(i, D.nx);
    } else {
      const int side = i < 0 ? 0 : 1;
      int s = i < 0 ? -i : i - D.nx + 1;
      s = s > kHalo ? kHalo : s;
      const double* g = D.gx[side];
      const size_t mst = (size_t)kHalo * D.nz * D.ny;
      const size_t b = ((size_t)(s - 1) * D.nz + k) * D.ny + (size_t)j;
#pragma unroll
      for (int m = 0; m < 5; ++m) q[m] = g[m * mst + b];
      return;
    }
  }
  const size_t b = nidx(D, i, j, k);
#pragma unroll
  for (int m = 0; m < 5; ++m) q[m] = w[(size_t)m * D.N + b];
}

// Reciprocal for the shock-capturing flux and the viscosity: in FP64 the
// hardware estimate refined by two Newton steps (within one ulp of 1/x for
// normal x, not correctly rounded), in FP32 the ordinary division.
template <typename F>
__device__ __forceinline__ F wrcp(F x) {
  return F(1) / x;
}
template <>
__device__ __forceinline__ double wrcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Square root of a positive normal x for the shock-capturing flux and the
// viscosity: the hardware reciprocal-square-root estimate (relative error
// about 2^-24) refined by one coupled Newton step and a final residual
// correction, within one ulp (measured over 2^20 arguments in [1e-6, 1e6]:
// a second coupled step changes nothing); no scaling for denormals or
// infinities, which a valid state never produces here; a negative argument
// gives NaN like sqrt.  FP32: the ordinary square root.
template <typename F>
__device__ __forceinline__ F wsqrt(F x) {
  return sqrt(x);
}
template <>
__device__ __forceinline__ double wsqrt<double>(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}

// Primitive variables in the flux arithmetic F.
template <typename F>
struct PV {
  F r, u, v, w, p, h, t, mu;
};

template <typename F>
__device__ __forceinline__ void to_prim(const Desc& D, const double q[5], PV<F>& s) {
  const F r = (F)q[0];
  const F ir = F(1) / r;
  s.r = r;
  s.u = (F)q[1] * ir;
  s.v = (F)q[2] * ir;
  s.w = (F)q[3] * ir;
  const F E = (F)q[4] * ir;
  const F ke = F(0.5) * (s.u * s.u + s.v * s.v + s.w * s.w);
  s.t = (E - ke) * (F)D.icv;
  s.p = r * (F)D.R * s.t;
  s.h = E + s.p * ir;
  const F tt = s.t * (F)D.iTref;
  s.mu = (F)D.muc * tt * sqrt(tt) / (tt + (F)D.S);
}

// FP64 primitives in a fixed evaluation order without contraction: the
// pressure and enthalpy feed fluxes that are differenced across a cell, so
// at low Mach number (p >> rho u^2) their rounding dominates the residual;
// keeping the order fixed keeps results reproducible against the reference.
template <>
__device__ __forceinline__ void to_prim<double>(const Desc& D, const double q[5], PV<double>& s) {
#pragma clang fp contract(off)
  const double ir = 1.0 / q[0];
  s.r = q[0];
  s.u = q[1] * ir;
  s.v = q[2] * ir;
  s.w = q[3] * ir;
  const double ke = 0.5 * (s.u * s.u + s.v * s.v + s.w * s.w);
  const double E = q[4] * ir;
  s.t = (E - ke) * D.icv;
  s.p = s.r * D.R * s.t;
  s.h = E + s.p * ir;
  const double tt = s.t * D.iTref;
  // viscosity: enters only the viscous terms, whose rounding is far below
  // the tolerance, so the refined estimates are used here
  s.mu = D.mu_ref * tt * wsqrt<double>(tt) * (1.0 + D.S) * wrcp<double>(tt + D.S);
}

// Energy-preserving central flux of order 2L (eq. encflux) at the interface
// between nodes nd[L-1] and nd[L] of the 2L consecutive nodes nd[0..2L-1]
// along direction DIR.  The pairs (i-m, i-m+l) are taken with l ascending
// and m ascending within l; the pressure is put in the same conservative
// form with two-point averages.
template <int DIR, typename F>
__device__ __forceinline__ F normal_vel(const PV<F>& s) {
  return DIR == 0 ? s.u : (DIR == 1 ? s.v : s.w);
}

template <typename F, int DIR, int L>
__device__ __forceinline__ void central_flux(const PV<F>* nd, F f[5]) {
  constexpr int NP = L * (L + 1) / 2;
  F c[NP];
  F pf = F(0);
  {
    int t = 0;
#pragma unroll
    for (int l = 1; l <= L; ++l) {
      F ps = F(0);
#pragma unroll
      for (int m = 0; m < l; ++m, ++t) {
        const PV<F>& A = nd[L - 1 - m];
        const PV<F>& B = nd[L - 1 - m + l];
        c[t] = F(0.25 * coef_a(L, l)) * ((A.r + B.r) * (normal_vel<DIR>(A) + normal_vel<DIR>(B)));
        ps = m == 0 ? (A.p + B.p) : ps + (A.p + B.p);
      }
      pf = l == 1 ? F(coef_a(L, 1)) * ps : pf + F(coef_a(L, l)) * ps;
    }
  }
  F s0 = c[0], s1 = F(0), s2 = F(0), s3 = F(0), s4 = F(0);
  {
    int t = 0;
#pragma unroll
    for (int l = 1; l <= L; ++l)
#pragma unroll
      for (int m = 0; m < l; ++m, ++t) {
        const PV<F>& A = nd[L - 1 - m];
        const PV<F>& B = nd[L - 1 - m + l];
        if (t > 0) s0 = s0 + c[t];
        const F a1 = c[t] * (A.u + B.u), a2 = c[t] * (A.v + B.v);
        const F a3 = c[t] * (A.w + B.w), a4 = c[t] * (A.h + B.h);
        s1 = t == 0 ? a1 : s1 + a1;
        s2 = t == 0 ? a2 : s2 + a2;
        s3 = t == 0 ? a3 : s3 + a3;
        s4 = t == 0 ? a4 : s4 + a4;
      }
  }
  f[0] = F(2) * s0;
  f[1] = s1;
  f[2] = s2;
  f[3] = s3;
  f[4] = s4;
  f[1 + DIR] += pf;
}

// Pressure part of the central flux, 2 sum_l a_l sum_m (p_{i-m} + p_{i-m+l})/2,
// in FP64 without contraction, m ascending inside l, l ascending.
template <int L>
__device__ __forceinline__ double comp_pressure_f64(const PV<double>* nd) {
#pragma clang fp contract(off)
  double outer = 0.0;
#pragma unroll
  for (int l = 1; l <= L; ++l) {
    double inner = 0.0;
#pragma unroll
    for (int m = 0; m < l; ++m) {
      const double term = (nd[L - 1 - m].p + nd[L - 1 - m + l].p) * 0.5;
      inner = m == 0 ? term : inner + term;
    }
    outer = l == 1 ? coef_a(L, 1) * inner : outer + coef_a(L, l) * inner;
  }
  return 2.0 * outer;
}

// FP64 version, evaluated as eq. encflux reads, without contraction: per
// pair (l, m) the average (1/8)(rho_a + rho_b)(u_a + u_b)(phi_a + phi_b),
// taken left to right (its first two factors are shared by the five
// components); the averages summed over m ascending, each inner sum
// weighted by a_l and summed over l ascending, the total doubled; the
// pressure part 2 sum_l a_l sum_m (p_a + p_b)/2 the same way.
template <int DIR, int L>
__device__ __forceinline__ void central_flux_f64(const PV<double>* nd, double f[5]) {
#pragma clang fp contract(off)
  constexpr int NP = L * (L + 1) / 2;
  double M[NP];
  {
    int t = 0;
#pragma unroll
    for (int l = 1; l <= L; ++l)
#pragma unroll
      for (int m = 0; m < l; ++m, ++t) {
        const PV<double>& A = nd[L - 1 - m];
        const PV<double>& B = nd[L - 1 - m + l];
        M[t] = 0.125 * (A.r + B.r) * (normal_vel<DIR>(A) + normal_vel<DIR>(B));
      }
  }
  // 2 sum_l a_l sum_m M_t (phi_a + phi_b)_t for one component
  auto comp = [&](auto phi) {
    double outer = 0.0;
    int t = 0;
#pragma unroll
    for (int l = 1; l <= L; ++l) {
      double inner = 0.0;
#pragma unroll
      for (int m = 0; m < l; ++m, ++t) {
        const double term = M[t] * phi(nd[L - 1 - m], nd[L - 1 - m + l]);
        inner = m == 0 ? term : inner + term;
      }
      outer = l == 1 ? coef_a(L, 1) * inner : outer + coef_a(L, l) * inner;
    }
    return 2.0 * outer;
  };
  f[0] = comp([](const PV<double>&, const PV<double>&) { return 2.0; });
  f[1] = comp([](const PV<double>& A, const PV<double>& B) { return A.u + B.u; });
  f[2] = comp([](const PV<double>& A, const PV<double>& B) { return A.v + B.v; });
  f[3] = comp([](const PV<double>& A, const PV<double>& B) { return A.w + B.w; });
  f[4] = comp([](const PV<double>& A, const PV<double>& B) { return A.h + B.h; });
  f[1 + DIR] = f[1 + DIR] + comp_pressure_f64<L>(nd);
}

// Pressure-only flux at a staggered wall (convective fluxes vanish there).
template <typename F, int DIR, int L>
__device__ __forceinline__ void wall_flux(const PV<F>* nd, F f[5]) {
  f[0] = f[1] = f[2] = f[3] = f[4] = F(0);
  F pf = F(0);
#pragma unroll
  for (int l = 1; l <= L; ++l) {
    F ps = F(0);
#pragma unroll
    for (int m = 0; m < l; ++m) ps = m == 0 ? (nd[L - 1 - m].p + nd[L - 1 - m + l].p)
                                            : ps + (nd[L - 1 - m].p + nd[L - 1 - m + l].p);
    pf = l == 1 ? F(coef_a(L, 1)) * ps : pf + F(coef_a(L, l)) * ps;
  }
  f[1 + DIR] = pf;
}

template <int DIR, int L>
__device__ __forceinline__ void wall_flux_f64(const PV<double>* nd, double f[5]) {
  f[0] = f[1] = f[2] = f[3] = f[4] = 0.0;
  f[1 + DIR] = comp_pressure_f64<L>(nd);
}

// Dispatch: FP64 uses the fixed-order forms above.  nd points at node i-L+1.
template <typename F, int DIR, int L>
__device__ __forceinline__ void cflux(const PV<F>* nd, F f[5]) {
  if constexpr (sizeof(F) == 8) central_flux_f64<DIR, L>(nd, f);
  else central_flux<F, DIR, L>(nd, f);
}
template <typename F, int DIR, int L>
__device__ __forceinline__ void wflux(const PV<F>* nd, F f[5]) {
  if constexpr (sizeof(F) == 8) wall_flux_f64<DIR, L>(nd, f);
  else wall_flux<F, DIR, L>(nd, f);
}

// The shock-capturing flux code below (reconstructions, node quantities,
// flux) is evaluated without automatic contraction and with its fused
// multiply-adds written out, so that every kernel that runs it (single
// instances, batched instances) computes the same bits whatever the code
// around it.

// WENO5-JS reconstruction at i+1/2 from v_{i-2..i+2}.  The argument `eps4`
// is four times the regulariser: the callers pass twice the split fluxes
// (the factor 1/2 of the splitting is applied once to the sum), and
// scaling the inputs by 2 scales the smoothness indicators by exactly 4,
// so the weights are those of the unscaled reconstruction.  The indicators
// are formed times 12/13 (d^2 + (3/13) e^2 + (12/13) eps): a common factor
// of the three cancels in the normalised weights.  The reconstruction is
// num / (6 den); the caller divides (half_sum folds the 6).
template <typename F>
__device__ __forceinline__ void weno5(F vm2, F vm1, F v0, F vp1, F vp2, F eps4, F& num, F& den) {
#pragma clang fp contract(off)
  // candidate reconstructions, times 6 (the 1/6 is applied with the weights)
  const F q0 = fma(F(11), v0, fma(F(-7), vm1, F(2) * vm2));
  const F q1 = fma(F(2), vp1, fma(F(5), v0, -vm1));
  const F q2 = fma(F(5), vp1, fma(F(2), v0, -vp2));
  const F d0 = fma(F(-2), vm1, vm2 + v0), e0 = fma(F(3), v0, fma(F(-4), vm1, vm2));
  const F d1 = fma(F(-2), v0, vm1 + vp1), e1 = vm1 - vp1;
  const F d2 = fma(F(-2), vp1, v0 + vp2), e2 = fma(F(3), v0, fma(F(-4), vp1, vp2));
  const F c3 = F(3.0 / 13.0), ce = F(12.0 / 13.0) * eps4;
  const F s0 = fma(d0, d0, fma(c3 * e0, e0, ce));
  const F s1 = fma(d1, d1, fma(c3 * e1, e1, ce));
  const F s2 = fma(d2, d2, fma(c3 * e2, e2, ce));
  // weights d_k/(eps+beta_k)^2 normalised, with numerator and denominator
  // multiplied by 10 times the product of the three squares (d = 0.1, 0.6,
  // 0.3 become 1, 6, 3): a = (t1 t2, 6 t0 t2, 3 t0 t1), one reciprocal
  const F t0 = s0 * s0, t1 = s1 * s1, t2 = s2 * s2;
  const F P = t1 * t2, B = F(3) * t1, C = F(6) * t2;
  num = fma(P, q0, t0 * fma(C, q1, B * q2));
  den = fma(t0, C + B, P);
}

// WENO3-JS (two candidate stencils, linear weights 1/3, 2/3) at i+1/2 from
// v_{i-1..i+1}, same input scaling as weno5; numerator and denominator are
// multiplied by 3 t0 t1 (a = (t1, 2 t0)) and the candidates by 2: the
// reconstruction is num / (2 den).
template <typename F>
__device__ __forceinline__ void weno3(F vm1, F v0, F vp1, F eps4, F& num, F& den) {
#pragma clang fp contract(off)
  const F q0 = fma(F(3), v0, -vm1);
  const F q1 = v0 + vp1;
  const F d0 = v0 - vm1, d1 = vp1 - v0;
  const F s0 = fma(d0, d0, eps4), s1 = fma(d1, d1, eps4);
  const F t0 = s0 * s0, t1 = s1 * s1;
  num = fma(t1, q0, (F(2) * t0) * q1);
  den = fma(F(2), t0, t1);
}

// WENO7-JS (four candidate stencils, linear weights (1, 12, 18, 4)/35) at
// i+1/2 from v[0..6] = v_{i-3..i+3}, same input scaling as weno5.  The
// smoothness indicators are Balsara and Shu's quadratic forms divided by
// 240 (which makes them the integrals of the squared derivatives of the
// candidate polynomials over the cell, as for the other orders), here
// formed times 240 with the regulariser likewise (the common factor cancels
// in the normalised weights); the candidates are multiplied by 12 and the
// weights formed with one reciprocal each (a product form would overflow in
// FP32).  The reconstruction is num / (12 den).
template <typename F>
__device__ __forceinline__ void weno7(const F* v, F eps4, F& num, F& den) {
#pragma clang fp contract(off)
  const F a = v[0], b = v[1], d = v[2], e = v[3], f = v[4], g = v[5], h = v[6];
  const F q0 = fma(F(25), e, fma(F(-23), d, fma(F(13), b, F(-3) * a)));
  const F q1 = fma(F(3), f, fma(F(13), e, fma(F(-5), d, b)));
  const F q2 = fma(F(7), f, fma(F(7), e, -d)) - g;
  const F q3 = fma(F(3), e, fma(F(13), f, fma(F(-5), g, h)));
  // sum of x_k times a linear form, the last term a square
  const F b0 = fma(a, fma(F(-1854), e, fma(F(4642), d, fma(F(-3882), b, F(547) * a))),
                   fma(b, fma(F(7042), e, fma(F(-17246), d, F(7043) * b)),
                       fma(d, fma(F(-9402), e, F(11003) * d), (F(2107) * e) * e)));
  const F b1 = fma(b, fma(F(-494), f, fma(F(1602), e, fma(F(-1642), d, F(267) * b))),
                   fma(d, fma(F(1922), f, fma(F(-5966), e, F(2843) * d)),
                       fma(e, fma(F(-2522), f, F(3443) * e), (F(547) * f) * f)));
  const F b2 = fma(d, fma(F(-494), g, fma(F(1922), f, fma(F(-2522), e, F(547) * d))),
                   fma(e, fma(F(1602), g, fma(F(-5966), f, F(3443) * e)),
                       fma(f, fma(F(-1642), g, F(2843) * f), (F(267) * g) * g)));
  const F b3 = fma(e, fma(F(-1854), h, fma(F(7042), g, fma(F(-9402), f, F(2107) * e))),
                   fma(f, fma(F(4642), h, fma(F(-17246), g, F(11003) * f)),
                       fma(g, fma(F(-3882), h, F(7043) * g), (F(547) * h) * h)));
  const F e240 = F(240) * eps4;
  const F s0 = e240 + b0, s1 = e240 + b1, s2 = e240 + b2, s3 = e240 + b3;
  const F w0 = wrcp<F>(s0 * s0), w1 = F(12) * wrcp<F>(s1 * s1);
  const F w2 = F(18) * wrcp<F>(s2 * s2), w3 = F(4) * wrcp<F>(s3 * s3);
  num = fma(w0, q0, fma(w1, q1, fma(w2, q2, w3 * q3)));
  den = ((w0 + w1) + w2) + w3;
}

// Reconstruction of order 2R-1 at i+1/2 from v[0..2R-2] = v_{i-R+1..i+R-1},
// as num / (wden<R>() den).
template <typename F, int R>
__device__ __forceinline__ void wrec(const F* v, F eps4, F& num, F& den) {
  if constexpr (R == 2) weno3<F>(v[0], v[1], v[2], eps4, num, den);
  else if constexpr (R == 3) weno5<F>(v[0], v[1], v[2], v[3], v[4], eps4, num, den);
  else weno7<F>(v, eps4, num, den);
}
template <int R>
__host__ __device__ constexpr double wden() { return R == 2 ? 2.0 : (R == 3 ? 6.0 : 12.0); }

// Half the sum of the two reconstructions np/(c dp) + nm/(c dm), c =
// wden<R>().  In FP64 with one reciprocal, (np dm + nm dp) / (2 c dp dm):
// the denominators are products of up to four squared indicators (each at
// least the regulariser), so their product stays far inside the FP64
// range; FP32 takes one reciprocal each.
template <typename F, int R>
__device__ __forceinline__ F half_sum(F np, F dp, F nm, F dm) {
#pragma clang fp contract(off)
  if constexpr (sizeof(F) == 8)
    return fma(np, dm, nm * dp) * wrcp<F>(F(2.0 * wden<R>()) * (dp * dm));
  else return F(0.5 / wden<R>()) * fma(np, wrcp<F>(dp), nm * wrcp<F>(dm));
}

// Quantities of one stencil node of the shock-capturing flux along DIR: the
// conserved state in the permuted order (rho, m_n, m_t1, m_t2, E), the
// normal velocity, the pressure (gamma-1)(E - m.u/2) and the sound speed.
template <typename F>
struct WNode {
  F r, mn, m1, m2, E, un, p, c;
};

template <typename F, int DIR>
__device__ __forceinline__ void weno_node(const Desc& D, const double q[5], WNode<F>& n) {
#pragma clang fp contract(off)
  constexpr int PN = 1 + DIR, P1 = 1 + (DIR + 1) % 3, P2 = 1 + (DIR + 2) % 3;
  const F gm1 = (F)D.gm1, gam = (F)D.gamma;
  const F hgm1 = F(0.5) * gm1;
  n.r = (F)q[0];
  n.mn = (F)q[PN];
  n.m1 = (F)q[P1];
  n.m2 = (F)q[P2];
  n.E = (F)q[4];
  const F ir = wrcp<F>(n.r);
  n.un = n.mn * ir;
  const F t1 = n.m1 * ir, t2 = n.m2 * ir;
  n.p = fma(-hgm1, fma(n.mn, n.un, fma(n.m1, t1, n.m2 * t2)), gm1 * n.E);
  n.c = wsqrt<F>((gam * n.p) * ir);
}

// Lax-Friedrichs split characteristic WENO flux of order 2R-1 at interface
// i+1/2 along DIR from the 2R nodes i-R+1..i+R (stencil index s = 0..2R-1,
// node(s, n) gives node s's quantities; Sec. 2.1).  Eigenvectors at the
// Roe average of nodes i, i+1; splitting constant per field from the
// largest |eigenvalue| over the stencil.
template <typename F, int DIR, int R, typename NodeGet>
__device__ __forceinline__ void weno_flux(const Desc& D, NodeGet&& node, F out[5]) {
#pragma clang fp contract(off)
  constexpr int NS = 2 * R;
  constexpr int PN = 1 + DIR, P1 = 1 + (DIR + 1) % 3, P2 = 1 + (DIR + 2) % 3;
  const F gm1 = (F)D.gm1;
  // Roe average of nodes i (s=R-1) and i+1 (s=R)
  F ur, vr, wr, Hr;
  {
    WNode<F> a, b;
    node(R - 1, a);
    node(R, b);
    const F ira = wrcp<F>(a.r), irb = wrcp<F>(b.r);
    const F t1a = a.m1 * ira, t2a = a.m2 * ira;
    const F t1b = b.m1 * irb, t2b = b.m2 * irb;
    const F Ha = (a.E + a.p) * ira, Hb = (b.E + b.p) * irb;
    const F sl = wsqrt<F>(a.r), sr = wsqrt<F>(b.r);
    const F iw = wrcp<F>(sl + sr);
    ur = fma(sl, a.un, sr * b.un) * iw;
    vr = fma(sl, t1a, sr * t1b) * iw;
    wr = fma(sl, t2a, sr * t2b) * iw;
    Hr = fma(sl, Ha, sr * Hb) * iw;
  }
  const F q2 = fma(ur, ur, fma(vr, vr, wr * wr));
  const F cr = wsqrt<F>(gm1 * fma(F(-0.5), q2, Hr));
  const F ic = wrcp<F>(cr);
  const F b1 = (gm1 * ic) * ic;
  const F b2 = (F(0.5) * q2) * b1;
  // Projection on the left eigenvectors (permuted order rho, m_n, m_t1,
  // m_t2, E).  With X = b2 q0 - b1 (u q1 + v q2 + w q3) + b1 q4 and
  // Y = (u q0 - q1)/c the rows are: (X + Y)/2, q0 - X, q2 - v q0,
  // q3 - w q0, (X - Y)/2.
  // (evaluated with X/2 and Y/2, which saves the two halvings)
  const F hb1 = F(0.5) * b1, hb2 = F(0.5) * b2, hic = F(0.5) * ic;
  auto project = [&](const F* q, F out[5]) {
    const F m = fma(ur, q[1], fma(vr, q[2], wr * q[3]));
    const F Xh = fma(hb1, q[4], fma(-hb1, m, hb2 * q[0]));
    const F Yh = fma(ur, q[0], -q[1]) * hic;
    out[0] = Xh + Yh;
    out[1] = fma(F(-2), Xh, q[0]);
    out[2] = fma(-vr, q[0], q[2]);
    out[3] = fma(-wr, q[0], q[3]);
    out[4] = Xh - Yh;
  };
  // stencil nodes: physical flux, eigenvalue bounds, characteristic projections
  F v[NS][5], g[NS][5];
  F am0 = F(0), am1 = F(0), am4 = F(0);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    WNode<F> nd;
    node(s, nd);
    const F un = nd.un, p = nd.p, c = nd.c;
    const F wq[5] = {nd.r, nd.mn, nd.m1, nd.m2, nd.E};
    project(wq, v[s]);
    // the flux is f = u_n w + p (0, 1, 0, 0, u_n), so its projection is
    // u_n (L w) + p L(0, 1, 0, 0, u_n), whose rows are p (X + Y, -2 X,
    // 0, 0, X - Y) with X = b1 (u_n - u)/2 and Y = -1/(2c)
    const F pX = p * (hb1 * (un - ur)), pY = p * hic;
    g[s][0] = fma(un, v[s][0], pX - pY);
    g[s][1] = fma(F(-2), pX, un * v[s][1]);
    g[s][2] = un * v[s][2];
    g[s][3] = un * v[s][3];
    g[s][4] = fma(un, v[s][4], pX + pY);
    am0 = fmax(am0, fabs(un - c));
    am1 = fmax(am1, fabs(un));
    am4 = fmax(am4, fabs(un + c));
  }
  const F alpha[5] = {am0, am1, am1, am1, am4};
  const F eps4 = F(4) * F(1e-6);  // exact power-of-two multiple of the regulariser
  F gh[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const F a = alpha[k];
    // twice the Lax-Friedrichs split characteristic fluxes g+- = (g +- a v)/2
    F vp[NS - 1], vm[NS - 1];
#pragma unroll
    for (int t = 0; t < NS - 1; ++t) {
      vp[t] = fma(a, v[t][k], g[t][k]);                    // i-R+1..i+R-1
      vm[t] = fma(-a, v[NS - 1 - t][k], g[NS - 1 - t][k]);  // i+R..i-R+2 (mirrored)
    }
    F np, dp, nm, dm;
    wrec<F, R>(vp, eps4, np, dp);
    wrec<F, R>(vm, eps4, nm, dm);
    gh[k] = half_sum<F, R>(np, dp, nm, dm);
  }
  // right eigenvectors applied to the reconstructed characteristic flux
  const F sg = (gh[0] + gh[1]) + gh[4];
  const F urc = ur * cr;
  const F f0 = sg;
  const F f1 = fma(ur - cr, gh[0], fma(ur, gh[1], (ur + cr) * gh[4]));
  const F f2 = fma(vr, sg, gh[2]);
  const F f3 = fma(wr, sg, gh[3]);
  const F f4 = fma(Hr - urc, gh[0],
                   fma(F(0.5) * q2, gh[1], fma(vr, gh[2], fma(wr, gh[3], (Hr + urc) * gh[4]))));
  out[0] = f0;
  out[PN] = f1;
  out[P1] = f2;
  out[P2] = f3;
  out[4] = f4;
}

// ------------------------------------------------------------------ stage begin
__global__ void k_stage_begin(Desc D) {
  if (threadIdx.x < 4) D.count[threadIdx.x] = 0u;
}

// ------------------------------------------------------------------ ghost planes

// Characteristic extrapolation through a face with normal DIR (Sec. 3.2,
// non-reflecting boundaries): the amplitudes of (q_b - q_i) on the waves
// leaving the domain are extrapolated linearly, incoming ones are held.
// qb is the boundary node, qi its interior neighbour, hi the upper face;
// gq[s] receives ghost layer s+1.
template <int DIR>
__device__ __forceinline__ void char_ghosts(const Desc& D, const double qb[5], const double qi[5],
                                            bool hi, double gq[kHalo][5]) {
  constexpr int PN = 1 + DIR, P1 = 1 + (DIR + 1) % 3, P2 = 1 + (DIR + 2) % 3;
  const double r = qb[0], ir = 1.0 / r;
  const double u = qb[PN] * ir, v = qb[P1] * ir, ww = qb[P2] * ir;  // normal, tangential
  const double p = D.gm1 * (qb[4] - 0.5 * r * (u * u + v * v + ww * ww));
  const double c = sqrt(D.gamma * p * ir);
  const double H = (qb[4] + p) * ir;
  const double q2 = u * u + v * v + ww * ww;
  const double ic = 1.0 / c, b1 = D.gm1 * ic * ic, b2 = 0.5 * q2 * b1;
  // differences in the permuted order (rho, m_n, m_t1, m_t2, E)
  const double d0 = qb[0] - qi[0], d1 = qb[PN] - qi[PN], d2 = qb[P1] - qi[P1];
  const double d3 = qb[P2] - qi[P2], d4 = qb[4] - qi[4];
  double a0 = 0.5 * (b2 + u * ic) * d0 - 0.5 * (b1 * u + ic) * d1 - 0.5 * b1 * v * d2 -
              0.5 * b1 * ww * d3 + 0.5 * b1 * d4;
  double a1 = (1.0 - b2) * d0 + b1 * u * d1 + b1 * v * d2 + b1 * ww * d3 - b1 * d4;
  double a2 = -v * d0 + d2;
  double a3 = -ww * d0 + d3;
  double a4 = 0.5 * (b2 - u * ic) * d0 - 0.5 * (b1 * u - ic) * d1 - 0.5 * b1 * v * d2 -
              0.5 * b1 * ww * d3 + 0.5 * b1 * d4;
  const double lam0 = u - c, lam1 = u, lam4 = u + c;
  if (!(hi ? lam0 > 0.0 : lam0 < 0.0)) a0 = 0.0;
  if (!(hi ? lam1 > 0.0 : lam1 < 0.0)) { a1 = 0.0; a2 = 0.0; a3 = 0.0; }
  if (!(hi ? lam4 > 0.0 : lam4 < 0.0)) a4 = 0.0;
  double dr[5];
  dr[0] = a0 + a1 + a4;
  dr[PN] = (u - c) * a0 + u * a1 + (u + c) * a4;
  dr[P1] = v * (a0 + a1 + a4) + a2;
  dr[P2] = ww * (a0 + a1 + a4) + a3;
  dr[4] = (H - u * c) * a0 + 0.5 * q2 * a1 + v * a2 + ww * a3 + (H + u * c) * a4;
#pragma unroll
  for (int s = 0; s < kHalo; ++s)
    for (int m = 0; m < 5; ++m) gq[s][m] = qb[m] + (double)(s + 1) * dr[m];
}

__device__ __forceinline__ void ghost_x_body(const Desc& D, const double* __restrict__ w, long long t) {
  // t over 2 * ny * nz (side, k, j)
  const long long per_side = (long long)D.ny * D.nz;
  const int side = (int)(t / per_side);
  const long long r = t - side * per_side;
  const int k = (int)(r / D.ny), j = (int)(r - (long long)k * D.ny);
  const int kind = D.bc[side];
  if (kind == BC_DF_INFLOW) return;  // planes written by the inflow generator once per step
  double* g = D.gx[side];
  const size_t mst = (size_t)kHalo * D.nz * D.ny;
  double gq[kHalo][5];
  if (kind == BC_DIRICHLET) {
    const double* pr = D.bcp[side];
    double q[5];
    from_prim(D, pr[j], pr[D.ny + j], pr[2 * D.ny + j], pr[3 * D.ny + j], pr[4 * D.ny + j], q);
#pragma unroll
    for (int s = 0; s < kHalo; ++s)
      for (int m = 0; m < 5; ++m) gq[s][m] = q[m];
  } else {  // characteristic outflow
    const int ib = side == 0 ? 0 : D.nx - 1;
    const int ii = side == 0 ? 1 : D.nx - 2;
    double qb[5], qi[5];
    const size_t nb = nidx(D, ib, j, k), ni = nidx(D, ii, j, k);
    for (int m = 0; m < 5; ++m) {
      qb[m] = w[(size_t)m * D.N + nb];
      qi[m] = w[(size_t)m * D.N + ni];
    }
    char_ghosts<0>(D, qb, qi, side == 1, gq);
  }
  // only the D.hw layers the stencils reach are written
#pragma unroll
  for (int s = 0; s < kHalo; ++s)
    if (s < D.hw)
      for (int m = 0; m < 5; ++m) g[m * mst + ((size_t)s * D.nz + k) * D.ny + j] = gq[s][m];
}

__device__ __forceinline__ void ghost_y_body(const Desc& D, const double* __restrict__ w, long long t) {
  // t over 2 * nz * nxg (side, k, ii)
  const long long per_side = (long long)D.nz * D.nxg;
  const int side = (int)(t / per_side);
  const long long r = t - side * per_side;
  const int k = (int)(r / D.nxg);
  const int i = (int)(r - (long long)k * D.nxg) - kHalo;
  if (i < -D.hw || i >= D.nx + D.hw) return;  // x range of the layers in use
  const int kind = D.bc[2 + side];
  double* g = D.gy[side];
  const size_t mst = (size_t)kHalo * D.nz * D.nxg;
  double gq[kHalo][5];
  if (kind == BC_OUTFLOW) {
    double qb[5], qi[5];
    load_node(D, w, i, side == 0 ? 0 : D.ny - 1, k, qb);
    load_node(D, w, i, side == 0 ? 1 : D.ny - 2, k, qi);
    char_ghosts<1>(D, qb, qi, side == 1, gq);
  }
#pragma unroll
  for (int s = 1; s <= kHalo; ++s) {
    if (s > D.hw) break;  // only the layers the stencils reach
    double q[5];
    if (is_wall(kind)) {
      double qm[5];
      load_node(D, w, i, side == 0 ? s - 1 : D.ny - s, k, qm);
      wall_ghost(D, kind, side, qm, q);
    } else if (kind == BC_OUTFLOW) {
      for (int m = 0; m < 5; ++m) q[m] = gq[s - 1][m];
    } else {  // imposed shock state
      const double* pr = D.bcp[2 + side];
      const int ish = (int)pr[0];
      const double* st = i < ish ? pr + 1 : pr + 6;
      from_prim(D, st[0], st[1], st[2], st[3], st[4], q);
    }
    for (int m = 0; m < 5; ++m)
      g[m * mst + ((size_t)(s - 1) * D.nz + k) * D.nxg + (size_t)(i + kHalo)] = q[m];
  }
}

// ------------------------------------------------------------------ inflow turbulence
// Synthetic inflow turbulence by digital filtering (Sec. 3.2), parameters
// D.bcp[0] = {Ny, Nz, T, seed, b_y[2Ny+1], b_z[2Nz+1], mean (rho,u,v,w,p)
// [5][ny], Cholesky (a11,a21,a22,a31,a32,a33)[6][ny]}.  Deviates are
// uniform on [-sqrt 3, sqrt 3) from SplitMix64 (output n of the generator
// seeded with `seed`), filtered along y and then z (periodic), correlated
// in time, mapped by the Cholesky factor and completed by the strong
// Reynolds analogy; one plane per RK step on the three x- ghost layers.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t n) {
  uint64_t z = seed + n * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t df_key(const Desc& D, int initial) {
  return initial ? 0ULL : (uint64_t)llround(D.scal[SC_STEP]);  // step s (0-based): s + 1
}

// fy[c][k][j] = sum_l b_y[l] r(c, k, j + l), the deviates made on the fly
__global__ void k_df_filter_y(Desc D, int initial) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ny = D.ny, nz = D.nz;
  if (t >= 3LL * nz * ny) return;
  const int c = (int)(t / ((long long)nz * ny));
  const int rem = (int)(t - (long long)c * nz * ny);
  const int k = rem / ny, j = rem - k * ny;
  const double* pr = D.bcp[0];
  const int Ny = (int)pr[0];
  const uint64_t seed = (uint64_t)pr[3];
  const double* by = pr + 4;
  const uint64_t key = df_key(D, initial);
  const uint64_t nyr = (uint64_t)(ny + 2 * Ny);
  const uint64_t row = 1 + ((key * 3 + (uint64_t)c) * (uint64_t)nz + (uint64_t)k) * nyr;
  double acc = 0.0;
  for (int l = -Ny; l <= Ny; ++l) {
    const uint64_t z = splitmix64_at(seed, row + (uint64_t)(j + l + Ny));
    const double u = (double)(z >> 11) * 0x1.0p-53;
    acc += by[l + Ny] * ((2.0 * u - 1.0) * 1.7320508075688772);
  }
  D.dffy[t] = acc;
}

// psi_hat = sum_m b_z[m] fy(k + m); psi update; fluctuations; ghost planes
__global__ void k_df_plane(Desc D, int initial) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ny = D.ny, nz = D.nz;
  if (t >= (long long)nz * ny) return;
  const int k = (int)(t / ny), j = (int)(t - (long long)k * ny);
  const double* pr = D.bcp[0];
  const int Ny = (int)pr[0], Nz = (int)pr[1];
  const double TL = pr[2];
  const double* bz = pr + 4 + 2 * Ny + 1;
  const double* mean = bz + 2 * Nz + 1;
  const double* chol = mean + 5 * ny;
  const double dt = D.scal[SC_DT];
  const double E = exp(-3.141592653589793 * dt / (2.0 * TL));
  const double F = sqrt(1.0 - E * E);
  const size_t plane = (size_t)nz * ny;
  double ps[3];
  for (int c = 0; c < 3; ++c) {
    double acc = 0.0;
    for (int m = -Nz; m <= Nz; ++m) {
      int kk = (k + m) % nz;
      kk = kk < 0 ? kk + nz : kk;
      acc += bz[m + Nz] * D.dffy[(size_t)c * plane + (size_t)kk * ny + j];
    }
    const size_t q = (size_t)c * plane + (size_t)t;
    const double v = initial ? acc : D.dfpsi[q] * E + acc * F;
    D.dfpsi[q] = v;
    ps[c] = v;
  }
  const double a11 = chol[j], a21 = chol[ny + j], a22 = chol[2 * ny + j];
  const double a31 = chol[3 * ny + j], a32 = chol[4 * ny + j], a33 = chol[5 * ny + j];
  const double du = a11 * ps[0];
  const double dv = a21 * ps[0] + a22 * ps[1];
  const double dw = a31 * ps[0] + a32 * ps[1] + a33 * ps[2];
  const double rm = mean[j], um = mean[ny + j], vm = mean[2 * ny + j], wm = mean[3 * ny + j];
  const double pm = mean[4 * ny + j];
  const double Tm = pm / (rm * D.R);
  const double T = Tm - um * du / D.cp;
  double q[5];
  from_prim(D, pm / (D.R * T), um + du, vm + dv, wm + dw, pm, q);
  double* g = D.gx[0];
  const size_t mst = (size_t)kHalo * nz * ny;
  for (int s = 0; s < D.hw; ++s)
    for (int m = 0; m < 5; ++m) g[m * mst + ((size_t)s * nz + k) * ny + j] = q[m];
}

__global__ void k_ghost_x(Desc D, int stage) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 2LL * D.ny * D.nz) ghost_x_body(D, D.win[stage], t);
}
__global__ void k_ghost_y(Desc D, int stage) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 2LL * D.nz * D.nxg) ghost_y_body(D, D.win[stage], t);
}

// ------------------------------------------------------------------ time-step bounds
// Largest convective and viscous time-step bounds of one node (conserved
// state q at row j), folded into cm and vm.  Evaluated without contraction,
// so that every kernel that takes the bound (the reduction kernel, the first
// stage's sensor, the batched kernels) gets the same bits for a node and the
// maxima, which do not depend on the order of the nodes, agree exactly.
__device__ __forceinline__ void dt_node(const Desc& D, const double q[5], int j, double& cm,
                                        double& vm) {
#pragma clang fp contract(off)
  const double r = q[0], ir = 1.0 / r;
  const double u = q[1] * ir, v = q[2] * ir, ww = q[3] * ir;
  const double T = (q[4] * ir - 0.5 * (u * u + v * v + ww * ww)) * D.icv;
  const double p = r * D.R * T;
  const double c = sqrt(D.gamma * p * ir);
  const double dy = D.deta * D.y_eta[j];
  const double conv = (fabs(u) + c) * D.idx + (fabs(v) + c) / dy + (fabs(ww) + c) * D.idz;
  cm = fmax(cm, conv);
  if (D.viscous) {
    const double t = T * D.iTref;
    const double mu = D.muc * t * sqrt(t) / (t + D.S);
    const double vis = D.vfac * (mu * ir) * (D.idx2 + 1.0 / (dy * dy) + D.idz2);
    vm = fmax(vm, vis);
  }
}

// Time step of the step from the largest bounds (CFL and viscous limits),
// or the fixed step; advances the step's time and counter.
__device__ __forceinline__ void dt_set(const Desc& D, double cm, double vm) {
  double dt;
  if (D.dt_fixed > 0.0) {
    dt = D.dt_fixed;
  } else {
    dt = 1.0 / cm;
    if (D.viscous && vm > 0.0) {
      const double dv = 2.5 / (D.rho2 * vm);
      if (dv < dt) dt = dv;
    }
    dt *= D.cfl;
  }
  D.scal[SC_DT] = dt;
  D.scal[SC_TIME] += dt;
  D.scal[SC_STEP] += 1.0;
}

// ------------------------------------------------------------------ sensor
// Ducros sensor (eq. sensor), FP64, operations in the order of the
// definition and without contraction, so that the flag decision is
// reproducible: theta = max(-div / sqrt(div^2 + |curl|^2 + eps), 0).
// 2.5-D tiling: a 64x4 tile of velocities with a 2-node cross-shaped halo
// is staged in LDS plane by plane; each thread keeps its own column's
// velocities for planes c-2..c+2 in registers.
constexpr int kSenTX = 64, kSenTY = 4;

// z planes per sensor block: 16, or 32 where that still leaves at least
// 2,048 blocks (eight per CU), which halves the share of the four planes
// each block loads only to fill its z window
__host__ __device__ inline int sensor_kz(const Desc& D) {
  const int t = ((D.nx + kSenTX - 1) / kSenTX) * ((D.ny + kSenTY - 1) / kSenTY);
  return t * ((D.nz + 31) / 32) >= 2048 ? 32 : 16;
}

// two plane buffers, used alternately: a plane's staging never waits for
// the previous plane's readers (one barrier per plane)
struct SenSmem {
  double v[2][3][kSenTY + 4][kSenTX + 4];
};

int sensor_tiles(const Desc& D) {
  return ((D.nx + kSenTX - 1) / kSenTX) * ((D.ny + kSenTY - 1) / kSenTY) *
         ((D.nz + sensor_kz(D) - 1) / sensor_kz(D));
}

// DT: the tile also folds its nodes' time-step bounds into cm and vm (the
// step's first stage, whose input is the state the step starts from).
template <bool DT = false>
__device__ __forceinline__ void sensor_tile(const Desc& D, const double* __restrict__ w, int lb, SenSmem& S,
                            bool export_theta, double* cm = nullptr, double* vm = nullptr) {
  constexpr int LX = kSenTX + 4;
  const int stx = (D.nx + kSenTX - 1) / kSenTX, sty = (D.ny + kSenTY - 1) / kSenTY;
  const int txi = lb % stx, rem = lb / stx;
  const int tyi = rem % sty, zc = rem / sty;
  const int i0 = txi * kSenTX, j0 = tyi * kSenTY;
  const int kz = sensor_kz(D);
  const int kb = zc * kz, ke = min(kb + kz, D.nz);
  const int tid = threadIdx.x, tx = tid % kSenTX, ty = tid / kSenTX;
  const int i = i0 + tx, j = j0 + ty;
  const bool valid = i < D.nx && j < D.ny;
  const bool tile_in = i0 >= 2 && i0 + kSenTX + 2 <= D.nx && j0 >= 2 && j0 + kSenTY + 2 <= D.ny;
  const size_t N = (size_t)D.N;
  const double iy = D.iy[j < D.ny ? j : D.ny - 1];
  double U[5], V[5], W[5];
  // raw (rho, rho u, rho v, rho w) of a node
  auto fetch = [&](int gi, int gj, int plane, bool fast, double q[4]) {
    if (fast) {
      const size_t b = nidx(D, gi, gj, wrap1(plane, D.nz));  // plane in [-2, nz+2]
#pragma unroll
      for (int m = 0; m < 4; ++m) q[m] = w[(size_t)m * N + b];
    } else {
      double qq[5];
      load_node(D, w, gi, gj, plane, qq);
#pragma unroll
      for (int m = 0; m < 4; ++m) q[m] = qq[m];
    }
  };
  auto vel = [&](const double q[4], double& u, double& v, double& ww) {
    const double ir = 1.0 / q[0];
    u = q[1] * ir;
    v = q[2] * ir;
    ww = q[3] * ir;
  };
  constexpr int NHS = 4 * kSenTX + 4 * kSenTY;  // halo nodes of a plane
  constexpr int HPS = (NHS + 255) / 256;        // per thread
  auto halo_pos = [&](int h, int& lx, int& ly) {
    if (h < 4 * kSenTX) {  // two rows below and two above the tile
      const int r = h / kSenTX;
      ly = r < 2 ? r : kSenTY + r;
      lx = 2 + h - r * kSenTX;
    } else {               // two columns left and two right of the tile
      const int hh = h - 4 * kSenTX;
      ly = 2 + hh / 4;
      const int cc = hh & 3;
      lx = cc < 2 ? cc : kSenTX + cc;
    }
  };
  auto fetch_halo = [&](int plane, double qh[HPS][4]) {
#pragma unroll
    for (int r = 0; r < HPS; ++r) {
      const int h = tid + r * 256;
      if (h < NHS) {
        int lx, ly;
        halo_pos(h, lx, ly);
        fetch(i0 - 2 + lx, j0 - 2 + ly, plane, tile_in, qh[r]);
      }
    }
  };
  // own column: (rho, rho u, rho v, rho w), and rho E for the time step
  constexpr int NQC = DT ? 5 : 4;
  auto fetch_col = [&](int plane, double q[NQC]) {
    if (valid) {
      const size_t b = nidx(D, i, j, wrap1(plane, D.nz));
#pragma unroll
      for (int m = 0; m < NQC; ++m) q[m] = w[(size_t)m * N + b];
    } else {
      double qq[5];
      load_node(D, w, i, j, plane, qq);
#pragma unroll
      for (int m = 0; m < NQC; ++m) q[m] = qq[m];
    }
  };
  const bool dt_on = DT && valid && !(D.dt_fixed > 0.0);
  auto bound = [&](int plane, const double q[NQC]) {
    if constexpr (DT) {
      if (dt_on && plane >= kb && plane < ke) dt_node(D, q, j, *cm, *vm);
    }
  };
  double qc[NQC], qh[HPS][4];
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    fetch_col(kb - 2 + sl, qc);
    vel(qc, U[sl], V[sl], W[sl]);
    bound(kb - 2 + sl, qc);
  }
  // the loads of plane c+1 (own column c+3, halo c+1) are issued during
  // plane c, before its closing barrier
  fetch_col(kb + 2, qc);
  fetch_halo(kb, qh);
  for (int c = kb; c < ke; ++c) {
    // this plane's buffer was last read in plane c-2, which every thread
    // finished before passing plane c-1's barrier: no barrier before the
    // writes
    double(&V3)[3][kSenTY + 4][kSenTX + 4] = S.v[(c - kb) & 1];
    vel(qc, U[4], V[4], W[4]);
    V3[0][ty + 2][tx + 2] = U[2];
    V3[1][ty + 2][tx + 2] = V[2];
    V3[2][ty + 2][tx + 2] = W[2];
#pragma unroll
    for (int r = 0; r < HPS; ++r) {
      const int h = tid + r * 256;
      if (h < NHS) {
        int lx, ly;
        halo_pos(h, lx, ly);
        double u, v, ww;
        vel(qh[r], u, v, ww);
        V3[0][ly][lx] = u;
        V3[1][ly][lx] = v;
        V3[2][ly][lx] = ww;
      }
    }
    // (after the halo conversion, when its registers are free)
    bound(c + 2, qc);
    if (c + 1 < ke) {
      fetch_col(c + 3, qc);
      fetch_halo(c + 1, qh);
    }
    __syncthreads();
    if (valid) {
#pragma clang fp contract(off)
      const int ly = ty + 2, lx = tx + 2;
      double g[3][3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        g[q][0] = D.idx * (CA1 * (V3[q][ly][lx + 1] - V3[q][ly][lx - 1]) +
                           CA2 * (V3[q][ly][lx + 2] - V3[q][ly][lx - 2]));
        g[q][1] = iy * (CA1 * (V3[q][ly + 1][lx] - V3[q][ly - 1][lx]) +
                        CA2 * (V3[q][ly + 2][lx] - V3[q][ly - 2][lx]));
      }
      g[0][2] = D.idz * (CA1 * (U[3] - U[1]) + CA2 * (U[4] - U[0]));
      g[1][2] = D.idz * (CA1 * (V[3] - V[1]) + CA2 * (V[4] - V[0]));
      g[2][2] = D.idz * (CA1 * (W[3] - W[1]) + CA2 * (W[4] - W[0]));
      const double div = g[0][0] + g[1][1] + g[2][2];
      const double ox = g[2][1] - g[1][2], oy = g[0][2] - g[2][0], oz = g[1][0] - g[0][1];
      const double den = sqrt(div * div + (ox * ox + oy * oy + oz * oz) + D.eps_s);
      double th = -div / den;
      if (th < 0.0) th = 0.0;
      const size_t n = nidx(D, i, j, c);
      D.nflag[n] = th > D.theta_star ? 1 : 0;
      if (export_theta) D.theta[n] = th;
    }
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      U[sl] = U[sl + 1];
      V[sl] = V[sl + 1];
      W[sl] = W[sl + 1];
    }
  }
  __syncthreads();  // the buffers are free for the block's next tile
}

// DT (first stage of a step): the kernel also folds the nodes' time-step
// bounds into D.dtmax, one atomic maximum per block on the bit patterns
// (ordered like the values for non-negative doubles, so the result is the
// exact maximum whatever the order); the stage's k_iflags turns them into
// the step.
template <bool DT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DT ? 3 : 4))) k_sensor(Desc D, int stage, int export_theta) {
  __shared__ SenSmem S;
  // the list counters of this stage start at zero (the previous stage's
  // lists were consumed before this kernel starts)
  if (blockIdx.x == 0 && threadIdx.x < 4) D.count[threadIdx.x] = 0u;
  double cm = 0.0, vm = 0.0;
  sensor_tile<DT>(D, D.win[stage], xcd_swizzle_blk(blockIdx.x, gridDim.x), S, export_theta != 0,
                  &cm, &vm);
  if constexpr (DT) {
    __shared__ double red[2][4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      cm = fmax(cm, __shfl_xor(cm, off));
      vm = fmax(vm, __shfl_xor(vm, off));
    }
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = cm;
      red[1][threadIdx.x >> 6] = vm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      cm = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
      vm = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
      atomicMax(&D.dtmax[0], (unsigned long long)__double_as_longlong(cm));
      atomicMax(&D.dtmax[1], (unsigned long long)__double_as_longlong(vm));
    }
  }
}

// ------------------------------------------------------------------ interface flags + lists
// Node flag at (i, j, k), each index within one period of its range (the
// callers reach at most L <= 3 nodes beyond a face and every dimension is
// at least 4), so the periodic images need no integer division.
__device__ __forceinline__ uint8_t node_flag(const Desc& D, int i, int j, int k) {
  if (i < 0 || i >= D.nx) {
    if (!D.per_x) return 0;
    i = wrap1(i, D.nx);
  }
  if (j < 0 || j >= D.ny) {
    if (!D.per_y) return 0;
    j = wrap1(j, D.ny);
  }
  k = wrap1(k, D.nz);
  return D.nflag[nidx(D, i, j, k)];
}

// Exclusive prefix sum over the 256 threads of a block (fixed order); returns
// the thread's offset and writes the block total to *tot.
__device__ __forceinline__ unsigned block_scan256(unsigned v, unsigned* sm, unsigned* tot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  unsigned x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sm[wv] = x;
  __syncthreads();
  unsigned pre = 0, all = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < wv) pre += sm[q];
    all += sm[q];
  }
  __syncthreads();
  *tot = all;
  return pre + x - v;
}

// 16 node flags (bytes 0/1) of one 128-bit word -> 16-bit mask.
__device__ __forceinline__ unsigned flag_mask16(uint4 v) {
  auto m4 = [](unsigned x) { return (x | (x >> 7) | (x >> 14) | (x >> 21)) & 0xFu; };
  return m4(v.x) | (m4(v.y) << 4) | (m4(v.z) << 8) | (m4(v.w) << 12);
}

// Interface-flag masks (bit r = node n0+r) of 16 consecutive nodes that lie
// in one x-row starting at i0 (row (j, k)); the node flags are read as
// 128-bit words.  Interface i+1/2 is flagged when a node of the central
// stencil i-L+1..i+L is.
template <int L>
__device__ __forceinline__ void iface_masks_row(const Desc& D, int n0, int i0, int j, int k,
                                                unsigned& mx, unsigned& my, unsigned& mz) {
  const uint4* nf = reinterpret_cast<const uint4*>(D.nflag);
  const unsigned mc = flag_mask16(nf[n0 >> 4]);
  const int rowstep = D.nx, plane = D.nx * D.ny;
  // x: bit t of e is node i0-L+1+t; neighbours beyond the word singly
  unsigned e = mc << (L - 1);
#pragma unroll
  for (int t = 0; t < L - 1; ++t) e |= (unsigned)node_flag(D, i0 - L + 1 + t, j, k) << t;
#pragma unroll
  for (int t = 0; t < L; ++t) e |= (unsigned)node_flag(D, i0 + 16 + t, j, k) << (L + 15 + t);
  unsigned ox = e;
#pragma unroll
  for (int t = 1; t < 2 * L; ++t) ox |= e >> t;
  mx = ox & 0xFFFFu;
  if (!D.per_x && i0 + 16 == D.nx) mx &= 0x7FFFu;  // last x interface is a boundary
  // y: rows j-L+1..j+L (non-periodic rows beyond the walls are unflagged)
  unsigned oy = mc;
#pragma unroll
  for (int o = 1 - L; o <= L; ++o) {
    if (o == 0) continue;
    int t = j + o;
    if (t < 0 || t >= D.ny) {
      if (!D.per_y) continue;
      t = wrapi(t, D.ny);
    }
    oy |= flag_mask16(nf[(n0 + (t - j) * rowstep) >> 4]);
  }
  my = (!D.per_y && j == D.ny - 1) ? 0u : oy;
  // z: planes k-L+1..k+L (periodic)
  unsigned oz = mc;
#pragma unroll
  for (int o = 1 - L; o <= L; ++o) {
    if (o == 0) continue;
    const int t = wrapi(k + o, D.nz);
    oz |= flag_mask16(nf[(n0 + (t - k) * plane) >> 4]);
  }
  mz = oz;
}

// Interface flags of a range of kIflagsPer*256 nodes and their compaction
// into the per-direction lists: one atomic per direction and block reserves
// the block's segment; each thread owns kIflagsPer consecutive nodes, the
// block stages its entries in LDS and writes the segment with coalesced
// stores, so the segment is in node order and the shock-capturing kernel
// reading the list touches consecutive nodes in consecutive lanes; the
// per-node list positions go through LDS too and leave as the block's
// contiguous range.
constexpr int kIflagsPer = 16;

// The step's time step from the maxima the first stage's sensor folded into
// D.dtmax, which are cleared for the next step (one thread).
__device__ __forceinline__ void dt_from_max(const Desc& D) {
  const double cm = __longlong_as_double((long long)D.dtmax[0]);
  const double vm = __longlong_as_double((long long)D.dtmax[1]);
  dt_set(D, cm, vm);
  D.dtmax[0] = 0ull;
  D.dtmax[1] = 0ull;
}

template <int L>
__device__ __forceinline__ void iflags_body(const Desc& D, long long blk) {
  __shared__ unsigned sm[4];
  __shared__ unsigned base[3];
  __shared__ uint16_t seg[3][256 * kIflagsPer];  // entries as offsets from the block start
  __shared__ int4 sst[256 * kIflagsPer / 4];      // the block's slots of one direction
  const int N = (int)D.N;  // below 2^31 (checked at creation)
  const int nb = (int)blk * (256 * kIflagsPer);
  const int n0 = nb + (int)threadIdx.x * kIflagsPer;
  unsigned mx = 0u, my = 0u, mz = 0u;
  if (n0 < N) {
    const int i0 = n0 % D.nx;
    const int rr = n0 / D.nx;
    int j = rr % D.ny, k = rr / D.ny;
    if (D.sensor_mode == 1 && D.nx % kIflagsPer == 0 && n0 + kIflagsPer <= N) {
      iface_masks_row<L>(D, n0, i0, j, k, mx, my, mz);
    } else {
      // general shape: walk the nodes with incremental indices.  An
      // interface is shock-capturing when a node of its central stencil is
      // flagged; boundary interfaces of non-periodic directions never are.
      int i = i0;
      for (int r = 0; r < kIflagsPer && n0 + r < N; ++r) {
        uint8_t f;
        const bool bx = !D.per_x && i == D.nx - 1, by = !D.per_y && j == D.ny - 1;
        if (D.sensor_mode == 2) {
          f = (uint8_t)((bx ? 0 : 1) | (by ? 0 : 2) | 4);
        } else {
          uint8_t ox = 0, oy = 0, oz = 0;
#pragma unroll
          for (int o = 1 - L; o <= L; ++o) {
            ox |= node_flag(D, i + o, j, k);
            oy |= node_flag(D, i, j + o, k);
            oz |= node_flag(D, i, j, k + o);
          }
          f = (uint8_t)((!bx && ox ? 1 : 0) | (!by && oy ? 2 : 0) | (oz ? 4 : 0));
        }
        mx |= (unsigned)(f & 1) << r;
        my |= (unsigned)((f >> 1) & 1) << r;
        mz |= (unsigned)((f >> 2) & 1) << r;
        if (++i == D.nx) {
          i = 0;
          if (++j == D.ny) {
            j = 0;
            ++k;
          }
        }
      }
    }
  }
  const unsigned msk[3] = {mx, my, mz};
  unsigned off[3], tot[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) off[d] = block_scan256((unsigned)__popc(msk[d]), sm, &tot[d]);
  if (threadIdx.x < 3) base[threadIdx.x] = tot[threadIdx.x] ? atomicAdd(&D.count[threadIdx.x], tot[threadIdx.x]) : 0u;
  const uint16_t loc = (uint16_t)(threadIdx.x * kIflagsPer);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    unsigned m = msk[d], p = off[d];
    while (m) {
      const int r = __ffs(m) - 1;
      m &= m - 1u;
      seg[d][p++] = (uint16_t)(loc + r);
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int* __restrict__ out = D.list[d] + base[d];
    for (unsigned e = threadIdx.x; e < tot[d]; e += 256u) out[e] = nb + (int)seg[d][e];
    // list position of every flagged node of the thread, -1 for the others
    int sl[kIflagsPer];
    int p = (int)(base[d] + off[d]);
#pragma unroll
    for (int r = 0; r < kIflagsPer; ++r) sl[r] = ((msk[d] >> r) & 1u) ? p++ : -1;
    // staged in LDS, then stored as the block's contiguous range (each
    // wave instruction writes 1 KiB of consecutive slots)
    if (d > 0) __syncthreads();  // the previous direction's slots are read
#pragma unroll
    for (int q = 0; q < kIflagsPer / 4; ++q)
      sst[threadIdx.x * (kIflagsPer / 4) + q] =
          make_int4(sl[4 * q], sl[4 * q + 1], sl[4 * q + 2], sl[4 * q + 3]);
    __syncthreads();
    if (nb + 256 * kIflagsPer <= N) {
      int4* o4 = reinterpret_cast<int4*>(D.slot[d] + nb);
#pragma unroll
      for (int q = 0; q < kIflagsPer / 4; ++q) o4[threadIdx.x + 256 * q] = sst[threadIdx.x + 256 * q];
    } else {
      const int* si = reinterpret_cast<const int*>(sst);
      for (int e = threadIdx.x; nb + e < N; e += 256) D.slot[d][nb + e] = si[e];
    }
  }
  __syncthreads();
}

// set_dt (first stage of a step whose sensor reduced the time-step bounds):
// one thread also sets the step's time step, which no earlier kernel of the
// stage reads.
template <int L>
__global__ void __launch_bounds__(256) k_iflags(Desc D, int set_dt) {
  if (set_dt && blockIdx.x == 0 && threadIdx.x == 0) dt_from_max(D);
  iflags_body<L>(D, blockIdx.x);
}

// ------------------------------------------------------------------ WENO on lists
template <typename F, int DIR, int R>
__device__ __forceinline__ void weno_entry(const Desc& D, const double* __restrict__ w, int n, unsigned e) {
  constexpr int NS = 2 * R;
  int i, j;
  const int k = qdiv(qdiv(n, D.nx, D.rnx, i), D.ny, D.rny, j);
  // all 10 R loads are issued before any arithmetic (latency-bound kernel)
  double qn[NS][5];
  const int c = DIR == 0 ? i : (DIR == 1 ? j : k);
  const int nd = DIR == 0 ? D.nx : (DIR == 1 ? D.ny : D.nz);
  if (c >= R - 1 && c + R < nd) {  // stencil inside the interior: direct addressing
    const long long st = DIR == 0 ? 1LL : (DIR == 1 ? (long long)D.nx : (long long)D.nx * D.ny);
    const double* __restrict__ b = w + (n - (R - 1) * st);
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int m = 0; m < 5; ++m) qn[s][m] = b[m * D.N + s * st];
  } else if (DIR == 2 || (DIR == 0 ? D.per_x : D.per_y)) {
    // periodic direction: the stencil wraps (|offset| < nd), still direct
    const int st = DIR == 0 ? 1 : (DIR == 1 ? D.nx : D.nx * D.ny);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int ns = n + (wrap1(c + s - (R - 1), nd) - c) * st;
#pragma unroll
      for (int m = 0; m < 5; ++m) qn[s][m] = w[(size_t)m * D.N + ns];
    }
  } else {  // a wall or open boundary within reach: ghost planes
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int o = s - (R - 1);
      load_node(D, w, i + (DIR == 0 ? o : 0), j + (DIR == 1 ? o : 0), k + (DIR == 2 ? o : 0),
                qn[s]);
    }
  }
  auto node = [&](int s, WNode<F>& nd) { weno_node<F, DIR>(D, qn[s], nd); };
  F f[5];
  weno_flux<F, DIR, R>(D, node, f);
  double* out = D.Fw[DIR];
#pragma unroll
  for (int m = 0; m < 5; ++m) out[(size_t)m * D.N + e] = (double)f[m];
}

template <typename F, int R>
__global__ void __launch_bounds__(256) k_weno(Desc D, const double* __restrict__ w) {
  const int dir = blockIdx.y;
  const unsigned cnt = D.count[dir];
  // The list is cut into chunks of 256 entries (one per block and pass, so
  // every wave but the list's last is full) and the chunks into eight equal
  // contiguous ranges, one per XCD; the blocks of an XCD take consecutive
  // chunks in each pass, so neighbouring interfaces share stencil nodes in
  // that XCD's L2.
  const unsigned G = gridDim.x;
  const unsigned lb = (unsigned)xcd_swizzle_blk(blockIdx.x, G);
  const unsigned groups = G % 8u == 0u ? 8u : 1u, per_g = G / groups;
  const unsigned g = lb / per_g, q = lb - g * per_g;
  const unsigned chunks = (cnt + 255u) / 256u;
  const unsigned c0 = (unsigned)((unsigned long long)chunks * g / groups);
  const unsigned c1 = (unsigned)((unsigned long long)chunks * (g + 1u) / groups);
  for (unsigned ch = c0 + q; ch < c1; ch += per_g) {
    const unsigned e = ch * 256u + threadIdx.x;
    if (e >= cnt) break;
    const int n = D.list[dir][e];
    if (dir == 0) weno_entry<F, 0, R>(D, w, n, e);
    else if (dir == 1) weno_entry<F, 1, R>(D, w, n, e);
    else weno_entry<F, 2, R>(D, w, n, e);
  }
}

// ------------------------------------------------------------------ reductions
template <int NT>
__device__ double block_sum(double v, double* sm) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < NT / 64; ++q) t += sm[q];
  __syncthreads();
  return t;
}

template <int NT>
__device__ double block_max(double v, double* sm) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = sm[0];
  if (threadIdx.x == 0)
    for (int q = 1; q < NT / 64; ++q) t = fmax(t, sm[q]);
  __syncthreads();
  return t;
}

template <int NT>
__device__ double block_min(double v, double* sm) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = sm[0];
  if (threadIdx.x == 0)
    for (int q = 1; q < NT / 64; ++q) t = fmin(t, sm[q]);
  __syncthreads();
  return t;
}

// Bulk force from the fused kernel's per-block partial sums of R_rhou dV,
// reduced by one wave without barriers: lane l sums partials l, l+64, ...
// in order, then a butterfly of exchanges adds the lanes' sums.  Each step
// adds the same two values in every lane of a pair (x + y and y + x are the
// same number), so every lane, wave and kernel gets the same bits.
__device__ __forceinline__ double force_wave(const Desc& D) {
  const int lane = threadIdx.x & 63;
  double v = 0.0;
  for (int q = lane; q < D.npart; q += 64) v += D.part[q];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return -v / D.vol_den;
}

__device__ __forceinline__ void force_body(const Desc& D, double* sm) {
  (void)sm;
  const double f = force_wave(D);
  if (threadIdx.x == 0) D.scal[SC_FORCE] = f;
}

// ------------------------------------------------------------------ fused right-hand side
// Quantity slots in the LDS plane.
enum { QR = 0, QU, QV, QW, QP, QH, QT, QM, NQ };

// Shared memory of one block of the fused kernel for central half-width L.
template <typename F, int TX, int TY, int L>
struct RhsSmem {
  F q[NQ][TY + 2 * L][TX + 2 * L];    // current plane with an L-node halo
  F zr[2 * L][3][TX * TY];            // per-thread ring of (rho, p, H) of planes c-L+1..c+L
  double pend[L][5][TX * TY];         // per-thread residuals awaiting their z-mixed terms
  double red[TX * TY / 64];
};

// First and second central derivatives of order 2L from an accessor
// at(o) = f_{i+o}: inv * sum_l a_l (f_{+l} - f_{-l}) and
// inv2 * (b_0 f_0 + sum_l b_l (f_{+l} + f_{-l})), each written as one
// expression summed left to right (l ascending).
template <typename F, int L, typename At, int... I>
__device__ __forceinline__ F d1_sum(At& at, std::integer_sequence<int, I...>) {
  return (... + (F(coef_a(L, I + 1)) * (at(I + 1) - at(-(I + 1)))));
}
template <typename F, int L, typename At, int... I>
__device__ __forceinline__ F d2_sum(At& at, F ctr, std::integer_sequence<int, I...>) {
  return ((F(coef_b(L, 0)) * ctr) + ... + (F(coef_b(L, I + 1)) * (at(I + 1) + at(-(I + 1)))));
}
template <typename F, int L, typename At>
__device__ __forceinline__ F d1g(At&& at, F inv) {
  return inv * d1_sum<F, L>(at, std::make_integer_sequence<int, L>{});
}
template <typename F, int L, typename At>
__device__ __forceinline__ F d2g(At&& at, F ctr, F inv2) {
  return inv2 * d2_sum<F, L>(at, ctr, std::make_integer_sequence<int, L>{});
}

template <typename F, int TX, int TY, int L>
__device__ __forceinline__ void lds_prim(const RhsSmem<F, TX, TY, L>& S, int ly, int lx, PV<F>& s) {
  s.r = S.q[QR][ly][lx]; s.u = S.q[QU][ly][lx]; s.v = S.q[QV][ly][lx]; s.w = S.q[QW][ly][lx];
  s.p = S.q[QP][ly][lx]; s.h = S.q[QH][ly][lx]; s.t = S.q[QT][ly][lx]; s.mu = S.q[QM][ly][lx];
}

template <typename F, int TX, int TY, int L>
__device__ __forceinline__ void lds_store(RhsSmem<F, TX, TY, L>& S, int ly, int lx, const PV<F>& s) {
  S.q[QR][ly][lx] = s.r; S.q[QU][ly][lx] = s.u; S.q[QV][ly][lx] = s.v; S.q[QW][ly][lx] = s.w;
  S.q[QP][ly][lx] = s.p; S.q[QH][ly][lx] = s.h; S.q[QT][ly][lx] = s.t; S.q[QM][ly][lx] = s.mu;
}

// x mod P in [0, P) for x >= -P and a compile-time period P (a mask for
// powers of two, which is exact for any x)
template <int P>
__device__ __forceinline__ int modp(int x) {
  if constexpr ((P & (P - 1)) == 0) return x & (P - 1);
  else return (int)((unsigned)(x + P) % (unsigned)P);
}

// Low-storage RK3 update of one point (Sec. 2.2, eq. RK) from its finished
// right-hand side r: the same arithmetic as k_rk, done where r is produced.
// Without bulk forcing (SPLIT false) all five components are updated, R is
// stored for the next stage (stages 0 and 1) and non-physical results set
// `bad`.  With forcing (SPLIT true) the force is not yet known: R is stored
// unforced by the caller and only rho, rho v, rho w are updated here; the
// update of rho u, rho E and the state check follow in k_rk_forced once
// the force has been reduced.
template <bool SPLIT>
__device__ __forceinline__ void rk_point(const Desc& D, int stage, double dt,
                                         const double* __restrict__ w, int no, const double r[5],
                                         bool& bad) {
  const double alpha = stage == 0 ? 0.0 : (stage == 1 ? -17.0 / 60.0 : -5.0 / 12.0);
  const double beta = stage == 0 ? 8.0 / 15.0 : (stage == 1 ? 5.0 / 12.0 : 3.0 / 4.0);
  const size_t N = (size_t)D.N;
  const double* __restrict__ Rp = D.rprev[stage];
  double* __restrict__ Rc = D.rcur[stage];
  double* __restrict__ wo = D.wout[stage];
  double q[5], rp[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    if (SPLIT && (m == 1 || m == 4)) continue;
    q[m] = w[m * N + no];
    rp[m] = stage > 0 ? Rp[m * N + no] : 0.0;
  }
  if (!SPLIT && stage < 2) {
#pragma unroll
    for (int m = 0; m < 5; ++m) Rc[m * N + no] = r[m];
  }
  double o[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    if (SPLIT && (m == 1 || m == 4)) continue;
    double acc = beta * r[m];
    if (stage > 0) acc = fma(alpha, rp[m], acc);
    o[m] = fma(dt, acc, q[m]);
    wo[m * N + no] = o[m];
  }
  if constexpr (!SPLIT) {
    const double ke = 0.5 * (o[1] * o[1] + o[2] * o[2] + o[3] * o[3]) / o[0];
    const double pe = o[4] - ke;
    bad |= !(o[0] > 0.0) || !(pe > 0.0) || !(fabs(o[4]) < 1e300);
  }
}

// One block of the fused kernel: tile (tile index lb) of the instance D,
// central stencils of half-width L (order 2L).  Each thread owns one (i, j)
// column of the tile and walks its z chunk; plane c is staged in LDS with an
// L-node halo for the in-plane derivatives and fluxes, the column's own
// planes c-L..c+L stay in a register window for the z terms, and the
// z-mixed viscous terms of plane c-L are completed once the in-plane
// derivatives of plane c are known.  VISC_ON false compiles the viscous
// terms out (inviscid problems: fewer registers); true evaluates them when
// the instance is viscous.
// RKM: 0 stores R for the update kernel; 1 (no bulk forcing) does the
// point's RK update of stage rk_stage in the same pass; 2 (bulk forcing)
// stores R and does the part of the update that does not involve the force;
// 3 chooses between 1 and 2 by the instance's forcing (batched instances).
template <typename F, int TX, int TY, bool VISC_ON, int L, int RKM = 0>
__device__ __forceinline__ void rhs_body(const Desc& D, const double* __restrict__ w, double* __restrict__ R,
                         int lb, RhsSmem<F, TX, TY, L>& S, int rk_stage = -1) {
  constexpr int LX = TX + 2 * L, LY = TY + 2 * L;
  constexpr int NT = TX * TY;
  constexpr int NH = LX * LY - TX * TY;
  constexpr int NW = 2 * L + 1;  // window planes c-L..c+L
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int txi = lb % D.tiles_x;
  const int rem = lb / D.tiles_x;
  const int tyi = rem % D.tiles_y;
  const int zc = rem / D.tiles_y;
  const int i0 = txi * TX, j0 = tyi * TY;
  const int kb = zc * D.kz;
  const int ke = min(kb + D.kz, D.nz);
  const int i = i0 + tx, j = j0 + ty;
  const bool valid = i < D.nx && j < D.ny;
  const bool col_in = valid;
  const bool tile_in = i0 >= L && i0 + TX + L <= D.nx && j0 >= L && j0 + TY + L <= D.ny;
  const size_t N = (size_t)D.N;
  const int jc = j < D.ny ? j : D.ny - 1;
  const F idx = (F)D.idx, idz = (F)D.idz, idx2 = (F)D.idx2, idz2 = (F)D.idz2;
  const F iy = (F)D.iy[jc], iye2 = (F)D.iye2[jc], yee = (F)D.y_etaeta[jc];
  const F ideta2 = (F)D.ideta2;
  const F kfac = (F)D.kfac;
  const bool visc = VISC_ON && D.viscous != 0;
  const bool hybrid = D.sensor_mode != 0;
  const bool wall_lo = D.wall_lo && j == 0;
  const bool wall_hi = D.wall_hi && j == D.ny - 1;

  // own-column register window, slots 0..2L = planes c-L..c+L
  PV<F> win[NW];
  // (rho, p, H) of the column live in the LDS ring S.zr; the other fields
  // of the window stay in registers.
  // deferred mixed-derivative windows (planes c-2L..c)
  F Sw[NW], Tw[NW], Qw[NW];
  double Ra0[5];
  F Fzm[5];
#pragma unroll
  for (int s = 0; s < NW; ++s) {
    win[s] = PV<F>{F(0), F(0), F(0), F(0), F(0), F(0), F(0), F(0)};
    Sw[s] = Tw[s] = Qw[s] = F(0);
  }
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    Ra0[m] = 0.0;
    Fzm[m] = F(0);
  }
  double fsum = 0.0;
  const double dt_rk = RKM ? D.scal[SC_DT] : 0.0;
  bool bad_state = false;  // a non-physical update result (or input, RKM 2)

  // list positions of the interfaces of plane c (x i+-1/2, y j+-1/2, z
  // c+1/2; -1: central flux), loaded one plane ahead so that their latency
  // overlaps a whole plane instead of delaying the flux loads behind them
  int sxr, sxl, syr, syl, szr;
  auto load_slots = [&](int cp, int& xr, int& xl, int& yr, int& yl, int& zr) {
    xr = xl = yr = yl = zr = -1;
    if (!hybrid || !valid) return;
    if (cp >= kb - 1 && cp < ke) zr = D.slot[2][nidx32(D, i, j, wrap1(cp, D.nz))];
    if (cp >= kb && cp < ke) {
      const int n0 = nidx32(D, i, j, cp);
      xr = D.slot[0][n0];
      if (i > 0 || D.per_x) xl = D.slot[0][i > 0 ? n0 - 1 : n0 + (D.nx - 1)];
      yr = D.slot[1][n0];
      if (j > 0 || D.per_y) yl = D.slot[1][j > 0 ? n0 - D.nx : n0 + (D.ny - 1) * D.nx];
    }
  };
  load_slots(kb - L, sxr, sxl, syr, syl, szr);

  // the column's conserved state at `plane` (issue), then its primitives
  // into the window slot s and (rho, p, H) into the ring (complete)
  auto issue_col = [&](int plane, double q[5]) {
    if (col_in) {
      const int b = nidx32(D, i, j, wrap1(plane, D.nz));  // plane in [-L, nz+2L-1], nz >= 2L
#pragma unroll
      for (int m = 0; m < 5; ++m) q[m] = w[(size_t)m * N + b];
    } else {
      load_node(D, w, i, j, plane, q);
    }
  };
  auto finish_col = [&](int plane, const double q[5], PV<F>& s) {
    to_prim<F>(D, q, s);
    // split update: the previous update's result is checked here, once per
    // point (the block's own planes), with the test the update kernels
    // apply to their results
    if constexpr (RKM >= 2) {
      if ((RKM == 2 || D.forcing) && valid && plane >= kb && plane < ke) {
        const double kq = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
        bad_state |= !(q[0] > 0.0) || !(q[4] - kq > 0.0) || !(fabs(q[4]) < 1e300);
      }
    }
    const int slot = modp<2 * L>(plane);
    S.zr[slot][0][tid] = s.r;
    S.zr[slot][1][tid] = s.p;
    S.zr[slot][2][tid] = s.h;
  };
  auto load_col = [&](int plane, PV<F>& s) {
    double q[5];
    issue_col(plane, q);
    finish_col(plane, q, s);
  };
  // window slot with (rho, p, H) restored from the ring
  auto full = [&](int ws, int plane) {
    PV<F> s = win[ws];
    const int slot = modp<2 * L>(plane);
    s.r = S.zr[slot][0][tid];
    s.p = S.zr[slot][1][tid];
    s.h = S.zr[slot][2][tid];
    return s;
  };

#pragma unroll
  for (int s = 0; s < L; ++s) load_col(kb - L + s, win[L + 1 + s]);

  for (int c = kb - L; c <= ke + L - 1; ++c) {
#pragma unroll
    for (int s = 0; s < 2 * L; ++s) win[s] = win[s + 1];
    int nxr, nxl, nyr, nyl, nzr;
    load_slots(c + 1, nxr, nxl, nyr, nyl, nzr);
    // the column's plane c+L is loaded while the halo of plane c is staged
    double qcol[5];
    issue_col(c + L, qcol);
    // stage plane c into LDS: interior from the window, halo cooperatively
    lds_store<F, TX, TY, L>(S, ty + L, tx + L, full(L, c));
    {
      const int kk = wrap1(c, D.nz);
      for (int h = tid; h < NH; h += NT) {
        int lx, ly;
        if (h < L * LX) {
          ly = h / LX; lx = h - ly * LX;
        } else if (h < 2 * L * LX) {
          const int hh = h - L * LX;
          ly = TY + L + hh / LX; lx = hh - (hh / LX) * LX;
        } else {
          const int hh = h - 2 * L * LX;
          ly = L + hh / (2 * L);
          const int cc = modp<2 * L>(hh);
          lx = cc < L ? cc : TX + cc;
        }
        const int gi = i0 - L + lx, gj = j0 - L + ly;
        double q[5];
        if (tile_in) {
          const int b = nidx32(D, gi, gj, kk);
#pragma unroll
          for (int m = 0; m < 5; ++m) q[m] = w[(size_t)m * N + b];
        } else {
          load_node(D, w, gi, gj, kk, q);
        }
        PV<F> s;
        to_prim<F>(D, q, s);
        lds_store<F, TX, TY, L>(S, ly, lx, s);
      }
    }
    finish_col(c + L, qcol, win[2 * L]);
    __syncthreads();
    const int ly = ty + L, lx = tx + L;
    // in-plane first derivatives feeding the z-mixed terms
#pragma unroll
    for (int s = 0; s < 2 * L; ++s) { Sw[s] = Sw[s + 1]; Tw[s] = Tw[s + 1]; Qw[s] = Qw[s + 1]; }
    if (visc) {
      const F wx = d1g<F, L>([&](int o) { return S.q[QW][ly][lx + o]; }, idx);
      const F wy = d1g<F, L>([&](int o) { return S.q[QW][ly + o][lx]; }, iy);
      const F ux = d1g<F, L>([&](int o) { return S.q[QU][ly][lx + o]; }, idx);
      const F vy = d1g<F, L>([&](int o) { return S.q[QV][ly + o][lx]; }, iy);
      Sw[2 * L] = wx; Tw[2 * L] = wy; Qw[2 * L] = ux + vy;
    }
    // z-direction interface flux at c+1/2 (own column)
    F Fzp[5] = {F(0), F(0), F(0), F(0), F(0)};
    if (c >= kb - 1 && c < ke && valid) {
      const int ez = szr;
      if (ez >= 0) {
#pragma unroll
        for (int m = 0; m < 5; ++m) Fzp[m] = (F)D.Fw[2][(size_t)m * N + ez];
      } else {
        PV<F> zn[2 * L];
#pragma unroll
        for (int s = 0; s < 2 * L; ++s) zn[s] = full(s + 1, c - L + 1 + s);
        cflux<F, 2, L>(zn, Fzp);
      }
    }
    if (c >= kb && c < ke && valid) {
      const double didx = D.idx, diy = D.iy[j], didz = D.idz;
      double acc[5];
      const int n0 = nidx32(D, i, j, c);
      // x direction: interfaces i-1/2, i+1/2 from the LDS row
      {
        F fr[5], fl[5];
        PV<F> nd[2 * L + 1];
#pragma unroll
        for (int s = 0; s <= 2 * L; ++s) lds_prim<F, TX, TY, L>(S, ly, lx - L + s, nd[s]);
        cflux<F, 0, L>(nd + 1, fr);
        cflux<F, 0, L>(nd, fl);
        if (hybrid) {
          const int er = sxr, el = sxl;
          if (er >= 0) {
#pragma unroll
            for (int m = 0; m < 5; ++m) fr[m] = (F)D.Fw[0][(size_t)m * N + er];
          }
          if (el >= 0) {
#pragma unroll
            for (int m = 0; m < 5; ++m) fl[m] = (F)D.Fw[0][(size_t)m * N + el];
          }
        }
#pragma unroll
        for (int m = 0; m < 5; ++m) {
#pragma clang fp contract(off)
          acc[m] = 0.0 - (double)(fr[m] - fl[m]) * didx;
        }
      }
      // y direction (stretched): interfaces j-1/2, j+1/2 from the LDS column
      {
        F fr[5], fl[5];
        PV<F> nd[2 * L + 1];
#pragma unroll
        for (int s = 0; s <= 2 * L; ++s) lds_prim<F, TX, TY, L>(S, ly - L + s, lx, nd[s]);
        if (wall_hi) wflux<F, 1, L>(nd + 1, fr);
        else cflux<F, 1, L>(nd + 1, fr);
        if (wall_lo) wflux<F, 1, L>(nd, fl);
        else cflux<F, 1, L>(nd, fl);
        if (hybrid) {
          const int er = syr, el = syl;
          if (er >= 0) {
#pragma unroll
            for (int m = 0; m < 5; ++m) fr[m] = (F)D.Fw[1][(size_t)m * N + er];
          }
          if (el >= 0) {
#pragma unroll
            for (int m = 0; m < 5; ++m) fl[m] = (F)D.Fw[1][(size_t)m * N + el];
          }
        }
#pragma unroll
        for (int m = 0; m < 5; ++m) {
#pragma clang fp contract(off)
          acc[m] = acc[m] - (double)(fr[m] - fl[m]) * diy;
        }
      }
      // z direction from the register window (flux at c+1/2 computed above)
#pragma unroll
      for (int m = 0; m < 5; ++m) {
#pragma clang fp contract(off)
        Ra0[m] = acc[m] - (double)(Fzp[m] - Fzm[m]) * didz;
      }
      if (visc) {
        const PV<F>& o = win[L];
#define SQ(qq, dy, dx) S.q[qq][ly + (dy)][lx + (dx)]
#define DX1(q) d1g<F, L>([&](int t_) { return SQ(q, 0, t_); }, idx)
#define DY1(q) d1g<F, L>([&](int t_) { return SQ(q, t_, 0); }, iy)
#define DX2(q, ctr) d2g<F, L>([&](int t_) { return SQ(q, 0, t_); }, ctr, idx2)
#define DY2(q, ctr, dy1) \
  ((d2g<F, L>([&](int t_) { return SQ(q, t_, 0); }, ctr, ideta2) - yee * (dy1)) * iye2)
#define DZ1(fld) d1g<F, L>([&](int t_) { return win[L + t_].fld; }, idz)
#define DZ2(fld) d2g<F, L>([&](int t_) { return win[L + t_].fld; }, o.fld, idz2)
        // velocity gradient
        const F ux = DX1(QU), uy = DY1(QU), uz = DZ1(u);
        const F vx = DX1(QV), vy = DY1(QV), vz = DZ1(v);
        const F wx = DX1(QW), wy = DY1(QW), wz = DZ1(w);
        const F div = ux + vy + wz;
        const F mx = DX1(QM), my = DY1(QM), mz = DZ1(mu);
        const F mu = o.mu;
        const F third = F(1.0 / 3.0), twoth = F(2.0 / 3.0);
        // in-plane mixed derivatives d_y(d_x f), metric of the outer (y) operator
        auto dxrow = [&](int q, int dy) {
          return d1g<F, L>([&](int t_) { return S.q[q][ly + dy][lx + t_]; }, idx);
        };
        const F uxy = d1g<F, L>([&](int t_) { return dxrow(QU, t_); }, iy);
        const F vxy = d1g<F, L>([&](int t_) { return dxrow(QV, t_); }, iy);
        const F uxx = DX2(QU, o.u);
        const F vyy = DY2(QV, o.v, vy);
        const F wzz = DZ2(w);
        const F Fx = mu * (uxx + DY2(QU, o.u, uy) + DZ2(u) + third * (uxx + vxy)) + mx * (ux + ux) +
                     my * (uy + vx) + mz * (uz + wx) - twoth * mx * div;
        const F Fy = mu * (DX2(QV, o.v) + vyy + DZ2(v) + third * (uxy + vyy)) + mx * (vx + uy) +
                     my * (vy + vy) + mz * (vz + wy) - twoth * my * div;
        const F Fz = mu * (DX2(QW, o.w) + DY2(QW, o.w, wy) + wzz + third * wzz) + mx * (wx + uz) +
                     my * (wy + vz) + mz * (wz + wz) - twoth * mz * div;
        const F sxy = uy + vx, sxz = uz + wx, syz = vz + wy;
        const F phi = mu * (F(2) * (ux * ux + vy * vy + wz * wz) + sxy * sxy + sxz * sxz +
                            syz * syz - twoth * div * div);
        const F Ty = DY1(QT);
        const F heat = kfac * (mu * (DX2(QT, o.t) + DY2(QT, o.t, Ty) + DZ2(t)) + mx * DX1(QT) +
                               my * Ty + mz * DZ1(t));
#undef SQ
#undef DX1
#undef DY1
#undef DX2
#undef DY2
#undef DZ1
#undef DZ2
        Ra0[1] += (double)Fx;
        Ra0[2] += (double)Fy;
        Ra0[3] += (double)Fz;
        Ra0[4] += (double)(o.u * Fx + o.v * Fy + o.w * Fz + phi + heat);
      }
    }
    if (c >= kb - 1 && c < ke) {
#pragma unroll
      for (int m = 0; m < 5; ++m) Fzm[m] = Fzp[m];
    }
    // finish plane c-L: z-mixed viscous parts, store, forcing partial sum
    // (plane c-L and plane c share the slot c mod L of the pending ring:
    // the older one is read before the newer one is written)
    const int pslot = modp<L>(c);
    if (c >= kb + L && valid) {
      const int m2 = c - L;
      double Ra2[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) Ra2[m] = S.pend[pslot][m][tid];
      if (visc) {
        const F dS = d1g<F, L>([&](int t_) { return Sw[L + t_]; }, idz);  // d_x d_z w
        const F dT = d1g<F, L>([&](int t_) { return Tw[L + t_]; }, idz);  // d_y d_z w
        const F dQ = d1g<F, L>([&](int t_) { return Qw[L + t_]; }, idz);  // d_z (d_x u + d_y v)
        const PV<F>& o2 = win[0];
        const F t3 = F(1.0 / 3.0) * o2.mu;
        const F ax = t3 * dS, ay = t3 * dT, az = t3 * dQ;
        Ra2[1] += (double)ax;
        Ra2[2] += (double)ay;
        Ra2[3] += (double)az;
        Ra2[4] += (double)(o2.u * ax + o2.v * ay + o2.w * az);
      }
      const int no = nidx32(D, i, j, m2);
      if (RKM == 1 || (RKM == 3 && !D.forcing)) {
        rk_point<false>(D, rk_stage, dt_rk, w, no, Ra2, bad_state);
      } else {
#pragma unroll
        for (int m = 0; m < 5; ++m) R[(size_t)m * N + no] = Ra2[m];
        fsum += Ra2[1] * D.y_eta[j];
        if constexpr (RKM >= 2) rk_point<true>(D, rk_stage, dt_rk, w, no, Ra2, bad_state);
      }
    }
    if (c >= kb && c < ke && valid) {
#pragma unroll
      for (int m = 0; m < 5; ++m) S.pend[pslot][m][tid] = Ra0[m];
    }
    sxr = nxr; sxl = nxl; syr = nyr; syl = nyl; szr = nzr;
    __syncthreads();
  }
  if (bad_state) atomicOr(D.status, (unsigned)ST_BAD_STATE);
  // block partial sum of R_rhou dV (fixed order)
  if (RKM != 1 && D.forcing) {
    double v = fsum;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    if ((tid & 63) == 0) S.red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int q = 0; q < NT / 64; ++q) t += S.red[q];
      D.part[lb] = t;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int xcd_swizzle(int b, int nb) {
  // consecutive logical tiles land on the same XCD (blocks are dealt
  // round-robin over the 8 XCDs), so neighbouring tiles share an L2
  return (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
}

// Sixth-order stencils need more shared memory than two blocks of a CU can
// hold, so that variant runs one block per CU with the full register file.
template <typename F, int TX, int TY, bool VISC_ON, int L, int RKM = 0>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(L == 3 ? 1 : 2)))
k_rhs(Desc D, const double* __restrict__ w, double* __restrict__ R, int rk_stage) {
  __shared__ RhsSmem<F, TX, TY, L> S;
  const int lb = xcd_swizzle(blockIdx.x, gridDim.x);
  rhs_body<F, TX, TY, VISC_ON, L, RKM>(D, w, R, lb, S, rk_stage);
}

__global__ void __launch_bounds__(256) k_force(Desc D) {
  __shared__ double sm[4];
  force_body(D, sm);
}

__global__ void k_apply_force(Desc D, int stage) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= D.N) return;
  const double f = D.scal[SC_FORCE];
  const double* w = D.win[stage];
  double* R = D.rcur[stage];
  R[D.N + n] += f;
  R[4 * D.N + n] += f * (w[D.N + n] * (1.0 / w[n]));
}

// ------------------------------------------------------------------ RK3 update
// Low-storage RK3 stage (Sec. 2.2): w' = w + dt (beta_s R_s + alpha_s R_{s-1}),
// with the bulk force (reduced beforehand) added to R_s, which is stored
// back for the next stage.  Every load of the thread's points is issued
// before any store, so the loads of all three input streams are in flight
// together.
constexpr int kRkPer = 2;  // points per thread of the update kernel

template <int stage>
__device__ __forceinline__ void rk_block_s(const Desc& D, long long blk) {
  const double f = D.forcing ? D.scal[SC_FORCE] : 0.0;  // reduced by the forcing kernel
  const double alpha = stage == 0 ? 0.0 : (stage == 1 ? -17.0 / 60.0 : -5.0 / 12.0);
  const double beta = stage == 0 ? 8.0 / 15.0 : (stage == 1 ? 5.0 / 12.0 : 3.0 / 4.0);
  const double* __restrict__ w = D.win[stage];
  double* __restrict__ wo = D.wout[stage];
  double* __restrict__ R = D.rcur[stage];
  const double* __restrict__ Rp = D.rprev[stage];
  const size_t N = (size_t)D.N;
  const double dt = D.scal[SC_DT];
  long long n[kRkPer];
  double q[kRkPer][5], r[kRkPer][5], rp[kRkPer][5];
#pragma unroll
  for (int p = 0; p < kRkPer; ++p) {
    n[p] = (blk * kRkPer + p) * 256 + threadIdx.x;
    // points past the end load the last point (unconditional loads stay
    // in flight together) and store nothing
    const size_t c = (size_t)(n[p] < D.N ? n[p] : D.N - 1);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      q[p][m] = w[m * N + c];
      r[p][m] = R[m * N + c];
      if (stage > 0) rp[p][m] = Rp[m * N + c];
    }
  }
  bool bad = false;
#pragma unroll
  for (int p = 0; p < kRkPer; ++p) {
    if (n[p] >= D.N) continue;
    if (D.forcing) {
      r[p][1] += f;
      r[p][4] = fma(f, q[p][1] * (1.0 / q[p][0]), r[p][4]);
      if (stage < 2) {
        R[1 * N + n[p]] = r[p][1];
        R[4 * N + n[p]] = r[p][4];
      }
    }
    double o[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      // explicit fused multiply-adds: rounded as in rk_point, the update
      // done inside the flux kernel
      double acc = beta * r[p][m];
      if (stage > 0) acc = fma(alpha, rp[p][m], acc);
      o[m] = fma(dt, acc, q[p][m]);
      wo[m * N + n[p]] = o[m];
    }
    const double ke = 0.5 * (o[1] * o[1] + o[2] * o[2] + o[3] * o[3]) / o[0];
    const double pe = o[4] - ke;
    bad |= !(o[0] > 0.0) || !(pe > 0.0) || !(fabs(o[4]) < 1e300);
  }
  if (bad) atomicOr(D.status, (unsigned)ST_BAD_STATE);
}

__device__ __forceinline__ void rk_block(const Desc& D, int stage, long long blk, double* sm) {
  (void)sm;
  if (stage == 0) rk_block_s<0>(D, blk);
  else if (stage == 1) rk_block_s<1>(D, blk);
  else rk_block_s<2>(D, blk);
}

__global__ void __launch_bounds__(256) k_rk(Desc D, int stage) {
  __shared__ double sm[8];
  rk_block(D, stage, blockIdx.x, sm);
}

// Completion of a split update (bulk forcing, rk_point<true> in the flux
// kernel): adds the reduced force to R_rhou and R_rhoE, stores them for the
// next stage and updates rho u and rho E with the arithmetic of k_rk.  The
// new state is checked where it is next read: by the flux kernel of the
// next stage (every input point) or, after the last stage, by the next
// step's flux kernel and by the diagnostics.
template <int stage>
__device__ __forceinline__ void rk_forced_block_s(const Desc& D, long long blk) {
  const double f = D.scal[SC_FORCE];  // reduced by the forcing kernel
  const double alpha = stage == 0 ? 0.0 : (stage == 1 ? -17.0 / 60.0 : -5.0 / 12.0);
  const double beta = stage == 0 ? 8.0 / 15.0 : (stage == 1 ? 5.0 / 12.0 : 3.0 / 4.0);
  const double* __restrict__ w = D.win[stage];
  double* __restrict__ wo = D.wout[stage];
  double* __restrict__ R = D.rcur[stage];
  const double* __restrict__ Rp = D.rprev[stage];
  const size_t N = (size_t)D.N;
  const double dt = D.scal[SC_DT];
  long long n[kRkPer];
  double q0[kRkPer], q1[kRkPer], q4[kRkPer], r1[kRkPer], r4[kRkPer], p1[kRkPer], p4[kRkPer];
#pragma unroll
  for (int p = 0; p < kRkPer; ++p) {
    n[p] = (blk * kRkPer + p) * 256 + threadIdx.x;
    const size_t c = (size_t)(n[p] < D.N ? n[p] : D.N - 1);
    q0[p] = w[c];
    q1[p] = w[N + c];
    q4[p] = w[4 * N + c];
    r1[p] = R[N + c];
    r4[p] = R[4 * N + c];
    if (stage > 0) {
      p1[p] = Rp[N + c];
      p4[p] = Rp[4 * N + c];
    }
  }
#pragma unroll
  for (int p = 0; p < kRkPer; ++p) {
    if (n[p] >= D.N) continue;
    const double fr1 = r1[p] + f;
    const double fr4 = fma(f, q1[p] * (1.0 / q0[p]), r4[p]);
    if (stage < 2) {
      R[1 * N + n[p]] = fr1;
      R[4 * N + n[p]] = fr4;
    }
    double a1 = beta * fr1, a4 = beta * fr4;
    if (stage > 0) {
      a1 = fma(alpha, p1[p], a1);
      a4 = fma(alpha, p4[p], a4);
    }
    const double o1 = fma(dt, a1, q1[p]);
    const double o4 = fma(dt, a4, q4[p]);
    wo[1 * N + n[p]] = o1;
    wo[4 * N + n[p]] = o4;
  }
}

__device__ __forceinline__ void rk_forced_block(const Desc& D, int stage, long long blk) {
  if (stage == 0) rk_forced_block_s<0>(D, blk);
  else if (stage == 1) rk_forced_block_s<1>(D, blk);
  else rk_forced_block_s<2>(D, blk);
}

__global__ void __launch_bounds__(256) k_rk_forced(Desc D, int stage) {
  rk_forced_block(D, stage, blockIdx.x);
}

// ------------------------------------------------------------------ time step
__device__ __forceinline__ void dt_part_body(const Desc& D, int b, int nb, double* sm) {
  const double* w = D.win[0];
  const size_t N = (size_t)D.N;
  double cm = 0.0, vm = 0.0;
  for (long long n = (long long)b * 256 + threadIdx.x; n < D.N; n += (long long)nb * 256) {
    const int j = (int)((n / D.nx) % D.ny);
    double q[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) q[m] = w[m * N + n];
    dt_node(D, q, j, cm, vm);
  }
  cm = block_max<256>(cm, sm);
  vm = block_max<256>(vm, sm);
  if (threadIdx.x == 0) {
    D.red[2 * b] = cm;
    D.red[2 * b + 1] = vm;
  }
}

__global__ void __launch_bounds__(256) k_dt_part(Desc D) {
  __shared__ double sm[4];
  dt_part_body(D, blockIdx.x, gridDim.x, sm);
}

__device__ __forceinline__ void dt_final_body(const Desc& D, int nb, double* sm) {
  double cm = 0.0, vm = 0.0;
  if (!(D.dt_fixed > 0.0)) {
    for (int q = threadIdx.x; q < nb; q += 256) {
      cm = fmax(cm, D.red[2 * q]);
      vm = fmax(vm, D.red[2 * q + 1]);
    }
    cm = block_max<256>(cm, sm);
    vm = block_max<256>(vm, sm);
  }
  if (threadIdx.x == 0) dt_set(D, cm, vm);
}

__global__ void __launch_bounds__(256) k_dt_final(Desc D, int nb) {
  __shared__ double sm[4];
  dt_final_body(D, nb, sm);
}


// ------------------------------------------------------------------ diagnostics
// Per-block partials of the volume integrals and extrema of the state w,
// written to part[blockIdx.x][DG_COUNT]; k_diag_final reduces nb of them in
// block order into res[0..nres-1] (nres <= DG_COUNT).
__global__ void __launch_bounds__(256) k_diag_part(Desc D, const double* __restrict__ w,
                                                   double* __restrict__ part) {
  __shared__ double sm[4];
  const size_t N = (size_t)D.N;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  double rmin = 1e300, pmin = 1e300, mmax = 0.0, nonf = 0.0;
  const double dv0 = D.dx * D.dz * D.deta;
  for (long long n = (long long)blockIdx.x * 256 + threadIdx.x; n < D.N;
       n += (long long)gridDim.x * 256) {
    const int j = (int)((n / D.nx) % D.ny);
    const double dv = dv0 * D.y_eta[j];
    double q[5];
    for (int m = 0; m < 5; ++m) {
      q[m] = w[m * N + n];
      if (!(fabs(q[m]) < 1e300)) nonf += 1.0;
      acc[m] += q[m] * dv;
    }
    const double ir = 1.0 / q[0];
    const double ke = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) * ir;
    acc[5] += ke * dv;
    const double p = D.gm1 * (q[4] - ke);
    rmin = fmin(rmin, q[0]);
    pmin = fmin(pmin, p);
    const double c = sqrt(fabs(D.gamma * p * ir));
    mmax = fmax(mmax, sqrt(2.0 * ke * ir) / c);
  }
  double* out = part + (size_t)blockIdx.x * DG_COUNT;
  for (int m = 0; m < 6; ++m) {
    const double t = block_sum<256>(acc[m], sm);
    if (threadIdx.x == 0) out[m] = t;
  }
  double t = block_min<256>(rmin, sm);
  if (threadIdx.x == 0) out[DG_RHOMIN] = t;
  t = block_min<256>(pmin, sm);
  if (threadIdx.x == 0) out[DG_PMIN] = t;
  t = block_max<256>(mmax, sm);
  if (threadIdx.x == 0) out[DG_MACHMAX] = t;
  t = block_sum<256>(nonf, sm);
  if (threadIdx.x == 0) out[DG_NONFINITE] = t;
}

__global__ void __launch_bounds__(256) k_diag_final(const double* __restrict__ part, int nb,
                                                    double* __restrict__ res, int nres) {
  __shared__ double sm[4];
  for (int m = 0; m < nres; ++m) {
    double v;
    if (m == DG_RHOMIN || m == DG_PMIN) {
      v = 1e300;
      for (int q = threadIdx.x; q < nb; q += 256) v = fmin(v, part[(size_t)q * DG_COUNT + m]);
      v = block_min<256>(v, sm);
    } else if (m == DG_MACHMAX) {
      v = 0.0;
      for (int q = threadIdx.x; q < nb; q += 256) v = fmax(v, part[(size_t)q * DG_COUNT + m]);
      v = block_max<256>(v, sm);
    } else if (m <= DG_NONFINITE) {
      v = 0.0;
      for (int q = threadIdx.x; q < nb; q += 256) v += part[(size_t)q * DG_COUNT + m];
      v = block_sum<256>(v, sm);
    } else {
      v = 0.0;
    }
    if (threadIdx.x == 0) res[m] = v;
  }
}

// ------------------------------------------------------------------ launchers
static inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_stage_begin(const Desc& D, hipStream_t st) {
  k_stage_begin<<<1, 64, 0, st>>>(D);
  return hipGetLastError();
}

bool ghosts_needed(const Desc& D) { return !D.per_x || !D.per_y; }

// ------------------------------------------------------------------ running statistics
// One thread per (i, j) column: spanwise sums (k ascending) of the
// statistics products of the current state, added to the accumulator.
__global__ void k_stats(Desc D) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)D.nx * D.ny) return;
  const double* w = D.win[0];
  const size_t N = (size_t)D.N, plane = (size_t)D.nx * D.ny;
  double acc[kNStat];
#pragma unroll
  for (int q = 0; q < kNStat; ++q) acc[q] = 0.0;
  for (int k = 0; k < D.nz; ++k) {
#pragma clang fp contract(off)
    const size_t n = (size_t)k * plane + (size_t)t;
    const double r = w[n], ir = 1.0 / r;
    const double u = w[N + n] * ir, v = w[2 * N + n] * ir, ww = w[3 * N + n] * ir;
    const double T = (w[4 * N + n] * ir - 0.5 * (u * u + v * v + ww * ww)) * D.icv;
    const double p = r * D.R * T;
    const double ru = w[N + n], rv = w[2 * N + n], rw = w[3 * N + n];
    acc[0] += r;
    acc[1] += ru;
    acc[2] += rv;
    acc[3] += rw;
    acc[4] += ru * u;
    acc[5] += rv * v;
    acc[6] += rw * ww;
    acc[7] += ru * v;
    acc[8] += u;
    acc[9] += u * u;
    acc[10] += T;
    acc[11] += r * T;
    acc[12] += T * T;
    acc[13] += p;
    acc[14] += p * p;
    acc[15] += r * r;
  }
#pragma unroll
  for (int q = 0; q < kNStat; ++q) D.stats[(size_t)q * plane + (size_t)t] += acc[q];
}

// Mean fields from the accumulated sums S (count samples x nz, times nx
// when averaged along x, the x sums taken i ascending): with m = S/count,
// rho, Favre means m(rho u_i)/rho, Favre stresses m(rho u_i u_j)/rho -
// u~_i u~_j (11, 22, 33, 12), u, u_rms, T, T~ = m(rho T)/rho, T_rms, p,
// p_rms, rho_rms (rms from the second moments, clipped at zero).  One
// thread per output column (j, i), or per row j when averaged.
__global__ void k_stats_means(Desc D, int avg, double count, double* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ncol = avg ? (long long)D.ny : (long long)D.nx * D.ny;
  if (t >= ncol) return;
  const size_t plane = (size_t)D.nx * D.ny;
  double m[kNStat];
#pragma unroll
  for (int q = 0; q < kNStat; ++q) {
    double s = 0.0;
    if (avg) {
      for (int i = 0; i < D.nx; ++i) s += D.stats[(size_t)q * plane + (size_t)t * D.nx + i];
    } else {
      s = D.stats[(size_t)q * plane + (size_t)t];
    }
    m[q] = s / count;
  }
  const double rho = m[0], ir = 1.0 / rho;
  const double uf = m[1] * ir, vf = m[2] * ir, wf = m[3] * ir;
  auto rms = [](double sq, double mean) { return sqrt(fmax(sq - mean * mean, 0.0)); };
  const double o[kNStat] = {rho, uf, vf, wf,
                            m[4] * ir - uf * uf, m[5] * ir - vf * vf, m[6] * ir - wf * wf,
                            m[7] * ir - uf * vf,
                            m[8], rms(m[9], m[8]), m[10], m[11] * ir, rms(m[12], m[10]),
                            m[13], rms(m[14], m[13]), rms(m[15], rho)};
  const size_t stride = (size_t)ncol;
#pragma unroll
  for (int q = 0; q < kNStat; ++q) out[(size_t)q * stride + (size_t)t] = o[q];
}

hipError_t launch_stats_means(const Desc& D, bool avg, double count, double* out, hipStream_t st) {
  const long long ncol = avg ? (long long)D.ny : (long long)D.nx * D.ny;
  k_stats_means<<<nblk(ncol, 128), 128, 0, st>>>(D, avg ? 1 : 0, count, out);
  return hipGetLastError();
}

hipError_t launch_stats(const Desc& D, hipStream_t st) {
  k_stats<<<nblk((long long)D.nx * D.ny, 256), 256, 0, st>>>(D);
  return hipGetLastError();
}

hipError_t launch_df(const Desc& D, bool initial, hipStream_t st) {
  k_df_filter_y<<<nblk(3LL * D.nz * D.ny, 256), 256, 0, st>>>(D, initial ? 1 : 0);
  k_df_plane<<<nblk((long long)D.nz * D.ny, 256), 256, 0, st>>>(D, initial ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_ghosts(const Desc& D, int stage, hipStream_t st) {
  if (!D.per_x) k_ghost_x<<<nblk(2LL * D.ny * D.nz, 128), 128, 0, st>>>(D, stage);
  if (!D.per_y) k_ghost_y<<<nblk(2LL * D.nz * D.nxg, 128), 128, 0, st>>>(D, stage);
  return hipGetLastError();
}

hipError_t launch_sensor(const Desc& D, int stage, bool export_theta, hipStream_t st, bool with_dt) {
  if (with_dt) k_sensor<true><<<sensor_tiles(D), 256, 0, st>>>(D, stage, export_theta ? 1 : 0);
  else k_sensor<false><<<sensor_tiles(D), 256, 0, st>>>(D, stage, export_theta ? 1 : 0);
  return hipGetLastError();
}

bool dt_in_sensor(const Desc& D) { return D.sensor_mode == 1 && D.bc[0] != BC_DF_INFLOW; }

__global__ void k_export_iflags(Desc D, uint8_t* __restrict__ out) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= D.N) return;
  out[n] = (uint8_t)((D.slot[0][n] >= 0 ? 1 : 0) | (D.slot[1][n] >= 0 ? 2 : 0) |
                     (D.slot[2][n] >= 0 ? 4 : 0));
}

__global__ void k_export_iface(Desc D, int dir, double* __restrict__ out) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= D.N) return;
  const int e = D.slot[dir][n];
  for (int m = 0; m < 5; ++m) out[(size_t)m * D.N + n] = e >= 0 ? D.Fw[dir][(size_t)m * D.N + e] : 0.0;
}

// Running total of listed interfaces (profiling): adds the three list
// lengths of the current stage to scal[SC_WACC] (or restarts it).
__global__ void k_count_iface(Desc D, int reset) {
  if (threadIdx.x != 0) return;
  const double prev = reset ? 0.0 : D.scal[SC_WACC];
  D.scal[SC_WACC] = reset ? 0.0 : prev + (double)D.count[0] + (double)D.count[1] + (double)D.count[2];
}

hipError_t launch_count_iface(const Desc& D, bool reset, hipStream_t st) {
  k_count_iface<<<1, 64, 0, st>>>(D, reset ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_export_iflags(const Desc& D, uint8_t* out, hipStream_t st) {
  k_export_iflags<<<nblk(D.N, 256), 256, 0, st>>>(D, out);
  return hipGetLastError();
}

hipError_t launch_export_iface(const Desc& D, int dir, double* out, hipStream_t st) {
  k_export_iface<<<nblk(D.N, 256), 256, 0, st>>>(D, dir, out);
  return hipGetLastError();
}

hipError_t launch_iflags(const Desc& D, hipStream_t st, bool set_dt) {
  const unsigned nb = nblk(D.N, 256 * kIflagsPer);
  const int sd = set_dt ? 1 : 0;
  if (D.cl == 1) k_iflags<1><<<nb, 256, 0, st>>>(D, sd);
  else if (D.cl == 3) k_iflags<3><<<nb, 256, 0, st>>>(D, sd);
  else k_iflags<2><<<nb, 256, 0, st>>>(D, sd);
  return hipGetLastError();
}

hipError_t launch_weno(const Desc& D, int stage, hipStream_t st) {
  // a few passes per block: fewer, longer-lived blocks (the WENO5 kernels,
  // at three (FP64) and four (FP32) waves per SIMD, measured fastest with
  // 512 per direction)
  const long long cap = D.wr == 3 ? 512 : 1024;
  long long b = nblk(D.N, 256);
  if (b > cap) b = cap;
  dim3 grid((unsigned)b, 3);
  const double* w = D.win[stage];
  if (D.precision == 1) {
    if (D.wr == 2) k_weno<float, 2><<<grid, 256, 0, st>>>(D, w);
    else if (D.wr == 4) k_weno<float, 4><<<grid, 256, 0, st>>>(D, w);
    else k_weno<float, 3><<<grid, 256, 0, st>>>(D, w);
  } else {
    if (D.wr == 2) k_weno<double, 2><<<grid, 256, 0, st>>>(D, w);
    else if (D.wr == 4) k_weno<double, 4><<<grid, 256, 0, st>>>(D, w);
    else k_weno<double, 3><<<grid, 256, 0, st>>>(D, w);
  }
  return hipGetLastError();
}

int rhs_blocks(const Desc& D) { return D.tiles_x * D.tiles_y * D.zchunks; }

bool rhs_tile_supported(int tx, int ty) {
  return (tx == 64 && ty == 4) || (tx == 32 && ty == 8) || (tx == 64 && ty == 2) ||
         (tx == 128 && ty == 2) || (tx == 64 && ty == 8);
}

// The fourth-order kernel comes in every supported tile shape; the second-
// and sixth-order ones in the 64x4 tile only (the scheme setter enforces it).
// The RK update joins the right-hand-side pass in the default 64x4 tile:
// whole without bulk forcing; with forcing the rho, rho v, rho w part,
// the rest following in k_rk_forced once the force is reduced.
bool rk_fused(const Desc& D) { return D.tile_x == 64 && D.tile_y == 4; }

template <typename F, bool VISC_ON>
static hipError_t launch_rhs_v(const Desc& D, int stage, bool fuse, hipStream_t st) {
  const unsigned nb = (unsigned)rhs_blocks(D);
  const double* w = D.win[stage];
  double* R = D.rcur[stage];
  if (fuse && D.forcing) {
    if (D.cl == 1) k_rhs<F, 64, 4, VISC_ON, 1, 2><<<nb, 256, 0, st>>>(D, w, R, stage);
    else if (D.cl == 3) k_rhs<F, 64, 4, VISC_ON, 3, 2><<<nb, 256, 0, st>>>(D, w, R, stage);
    else k_rhs<F, 64, 4, VISC_ON, 2, 2><<<nb, 256, 0, st>>>(D, w, R, stage);
  } else if (fuse) {
    if (D.cl == 1) k_rhs<F, 64, 4, VISC_ON, 1, 1><<<nb, 256, 0, st>>>(D, w, R, stage);
    else if (D.cl == 3) k_rhs<F, 64, 4, VISC_ON, 3, 1><<<nb, 256, 0, st>>>(D, w, R, stage);
    else k_rhs<F, 64, 4, VISC_ON, 2, 1><<<nb, 256, 0, st>>>(D, w, R, stage);
  } else if (D.cl != 2) {
    if (D.tile_x != 64 || D.tile_y != 4) return hipErrorInvalidValue;
    if (D.cl == 1) k_rhs<F, 64, 4, VISC_ON, 1><<<nb, 256, 0, st>>>(D, w, R, -1);
    else k_rhs<F, 64, 4, VISC_ON, 3><<<nb, 256, 0, st>>>(D, w, R, -1);
  } else if (D.tile_x == 64 && D.tile_y == 4) k_rhs<F, 64, 4, VISC_ON, 2><<<nb, 256, 0, st>>>(D, w, R, -1);
  else if (D.tile_x == 32 && D.tile_y == 8) k_rhs<F, 32, 8, VISC_ON, 2><<<nb, 256, 0, st>>>(D, w, R, -1);
  else if (D.tile_x == 64 && D.tile_y == 2) k_rhs<F, 64, 2, VISC_ON, 2><<<nb, 128, 0, st>>>(D, w, R, -1);
  else if (D.tile_x == 128 && D.tile_y == 2) k_rhs<F, 128, 2, VISC_ON, 2><<<nb, 256, 0, st>>>(D, w, R, -1);
  else if (D.tile_x == 64 && D.tile_y == 8) k_rhs<F, 64, 8, VISC_ON, 2><<<nb, 512, 0, st>>>(D, w, R, -1);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename F>
static hipError_t launch_rhs_t(const Desc& D, int stage, bool fuse, hipStream_t st) {
  return D.viscous ? launch_rhs_v<F, true>(D, stage, fuse, st)
                   : launch_rhs_v<F, false>(D, stage, fuse, st);
}

hipError_t launch_rhs(const Desc& D, int stage, hipStream_t st, bool fuse_rk) {
  if (fuse_rk && (stage > 2 || !rk_fused(D))) return hipErrorInvalidValue;
  return D.precision == 1 ? launch_rhs_t<float>(D, stage, fuse_rk, st)
                          : launch_rhs_t<double>(D, stage, fuse_rk, st);
}

hipError_t launch_force(const Desc& D, hipStream_t st) {
  k_force<<<1, 256, 0, st>>>(D);
  return hipGetLastError();
}

hipError_t launch_apply_force(const Desc& D, int stage, hipStream_t st) {
  k_apply_force<<<nblk(D.N, 256), 256, 0, st>>>(D, stage);
  return hipGetLastError();
}

hipError_t launch_rk(const Desc& D, int stage, hipStream_t st) {
  k_rk<<<nblk(D.N, 256 * kRkPer), 256, 0, st>>>(D, stage);
  return hipGetLastError();
}

hipError_t launch_rk_forced(const Desc& D, int stage, hipStream_t st) {
  if (!D.forcing || stage > 2) return hipErrorInvalidValue;
  k_rk_forced<<<nblk(D.N, 256 * kRkPer), 256, 0, st>>>(D, stage);
  return hipGetLastError();
}

hipError_t launch_dt(const Desc& D, hipStream_t st) {
  int nb = (int)nblk(D.N, 256);
  if (nb > kRedBlocks) nb = kRedBlocks;
  if (!(D.dt_fixed > 0.0)) k_dt_part<<<nb, 256, 0, st>>>(D);
  k_dt_final<<<1, 256, 0, st>>>(D, nb);
  return hipGetLastError();
}

hipError_t launch_diag(const Desc& D, hipStream_t st) {
  int nb = (int)nblk(D.N, 256);
  if (nb > kRedBlocks) nb = kRedBlocks;
  k_diag_part<<<nb, 256, 0, st>>>(D, D.win[0], D.redd);
  k_diag_final<<<1, 256, 0, st>>>(D.redd, nb, D.diag, DG_COUNT);
  return hipGetLastError();
}

// ------------------------------------------------------------------ no-allocation diagnostics
// Partials of the no-allocation diagnostics live in this file-scope device
// array (one copy per GPU, alive until the process ends).  Host code never
// passes the array's name to a kernel: it uses the device address obtained
// once per device with hipGetSymbolAddress (the name is only a host-side
// stand-in).  All calls on one GPU share the array, so calls that overlap in
// time on one GPU race.
static __device__ __align__(256) double scratch[kNoallocBlocks * DG_COUNT];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    double* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

long long noalloc_diag_blocks(long long N) { return (N + kNoallocPoints - 1) / kNoallocPoints; }

hipError_t launch_diag_noalloc(const Desc& D, const double* w, double* part, double* out,
                               int nout, hipStream_t st) {
  if (nout < 1 || nout > DG_COUNT || noalloc_diag_blocks(D.N) > kNoallocBlocks)
    return hipErrorInvalidValue;
  const int nb = (int)noalloc_diag_blocks(D.N);
  k_diag_part<<<nb, 256, 0, st>>>(D, w, part);
  k_diag_final<<<1, 256, 0, st>>>(part, nb, out, nout);
  return hipGetLastError();
}

// ------------------------------------------------------------------ batched kernels
// Persistent kernels over all attached instances.  Every instance is
// processed with exactly the per-item arithmetic of its single-instance
// kernels (same tiles, same reduction slots), so its results are the same
// alone and in any mix.  Batched instances use the default scheme orders
// (fourth-order central, fifth-order WENO); attaching others is refused.
int batch_items(const Desc& D, int kind) {
  switch (kind) {
    case WK_PTS: return (int)nblk(D.N, 256);
    case WK_IFL: return (int)nblk(D.N, 256 * kIflagsPer);
    case WK_SEN: return sensor_tiles(D);
    case WK_RK: return (int)nblk(D.N, 256 * kRkPer);
    case WK_RHS: return rhs_blocks(D);
    case WK_GX: return D.per_x ? 0 : (int)nblk(2LL * D.ny * D.nz, 256);
    case WK_GY: return D.per_y ? 0 : (int)nblk(2LL * D.nz * D.nxg, 256);
    case WK_DT: {
      int nb = (int)nblk(D.N, 256);
      return nb > kRedBlocks ? kRedBlocks : nb;
    }
  }
  return 0;
}

__device__ __forceinline__ int find_inst(const BatchTable* T, int kind, int b) {
  int lo = 0, hi = T->ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (T->pre[kind][mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

#define BATCH_FOR(KIND)                                                  \
  const int total_ = T->pre[KIND][T->ninst];                             \
  for (int b_ = blockIdx.x; b_ < total_; b_ += gridDim.x) {              \
    const int a_ = find_inst(T, KIND, b_);                               \
    const Desc& D = descs[T->inst[a_]];                                  \
    const int local = b_ - T->pre[KIND][a_];                             \
    const int litems = T->pre[KIND][a_ + 1] - T->pre[KIND][a_];          \
    (void)litems;
#define BATCH_END }

__global__ void k_b_begin(const Desc* __restrict__ descs, const BatchTable* __restrict__ T) {
  for (int a = threadIdx.x; a < T->ninst; a += blockDim.x) {
    unsigned* c = descs[T->inst[a]].count;
    c[0] = c[1] = c[2] = c[3] = 0u;
  }
}

__global__ void __launch_bounds__(256) k_b_dt_part(const Desc* __restrict__ descs,
                                                   const BatchTable* __restrict__ T) {
  __shared__ double sm[4];
  BATCH_FOR(WK_DT)
  if (!(D.dt_fixed > 0.0)) dt_part_body(D, local, litems, sm);
  BATCH_END
}

__global__ void __launch_bounds__(256) k_b_dt_final(const Desc* __restrict__ descs,
                                                    const BatchTable* __restrict__ T) {
  __shared__ double sm[4];
  for (int a = blockIdx.x; a < T->ninst; a += gridDim.x) {
    const Desc& D = descs[T->inst[a]];
    dt_final_body(D, T->pre[WK_DT][a + 1] - T->pre[WK_DT][a], sm);
  }
}

__global__ void __launch_bounds__(256) k_b_ghost_x(const Desc* __restrict__ descs,
                                                   const BatchTable* __restrict__ T, int stage) {
  BATCH_FOR(WK_GX)
  const long long t = (long long)local * 256 + threadIdx.x;
  if (t < 2LL * D.ny * D.nz) ghost_x_body(D, D.win[stage], t);
  BATCH_END
}

__global__ void __launch_bounds__(256) k_b_ghost_y(const Desc* __restrict__ descs,
                                                   const BatchTable* __restrict__ T, int stage) {
  BATCH_FOR(WK_GY)
  const long long t = (long long)local * 256 + threadIdx.x;
  if (t < 2LL * D.nz * D.nxg) ghost_y_body(D, D.win[stage], t);
  BATCH_END
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_b_sensor(const Desc* __restrict__ descs,
                                                  const BatchTable* __restrict__ T, int stage) {
  __shared__ SenSmem S;
  BATCH_FOR(WK_SEN)
  if (D.sensor_mode == 1) sensor_tile<false>(D, D.win[stage], local, S, false);
  BATCH_END
}

__global__ void __launch_bounds__(256) k_b_iflags(const Desc* __restrict__ descs,
                                                  const BatchTable* __restrict__ T) {
  BATCH_FOR(WK_IFL)
  if (D.sensor_mode > 0) iflags_body<2>(D, local);
  BATCH_END
}

template <typename F>
__global__ void __launch_bounds__(256) k_b_weno(const Desc* __restrict__ descs,
                                                const BatchTable* __restrict__ T, int stage) {
  for (int a = 0; a < T->ninst; ++a) {
    const Desc& D = descs[T->inst[a]];
    if (D.sensor_mode == 0) continue;
    const double* w = D.win[stage];
    for (int dir = 0; dir < 3; ++dir) {
      const unsigned cnt = D.count[dir];
      for (unsigned e = blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += gridDim.x * blockDim.x) {
        const int n = D.list[dir][e];
        if (dir == 0) weno_entry<F, 0, 3>(D, w, n, e);
        else if (dir == 1) weno_entry<F, 1, 3>(D, w, n, e);
        else weno_entry<F, 2, 3>(D, w, n, e);
      }
    }
  }
}

template <typename F, int TX, int TY>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(2))) k_b_rhs(const Desc* __restrict__ descs,
                                                  const BatchTable* __restrict__ T, int stage) {
  __shared__ RhsSmem<F, TX, TY, 2> S;
  BATCH_FOR(WK_RHS)
  // the 64x4 tiling does each instance's stage update here (whole, or the
  // part without the force), as for a single instance
  rhs_body<F, TX, TY, true, 2, (TX == 64 && TY == 4) ? 3 : 0>(D, D.win[stage], D.rcur[stage],
                                                              local, S, stage);
  BATCH_END
}

__global__ void __launch_bounds__(256) k_b_force(const Desc* __restrict__ descs,
                                                 const BatchTable* __restrict__ T) {
  __shared__ double sm[4];
  for (int a = blockIdx.x; a < T->ninst; a += gridDim.x) {
    const Desc& D = descs[T->inst[a]];
    if (D.forcing) force_body(D, sm);
  }
}

// fused: the right-hand-side kernel did the update (64x4 tiling); only the
// completion of forced instances remains
__global__ void __launch_bounds__(256) k_b_rk(const Desc* __restrict__ descs,
                                              const BatchTable* __restrict__ T, int stage,
                                              int fused) {
  __shared__ double sm[8];
  BATCH_FOR(WK_RK)
  if (!fused) rk_block(D, stage, local, sm);
  else if (D.forcing) rk_forced_block(D, stage, local);
  BATCH_END
}

template <typename F>
static hipError_t launch_b_rhs(const Desc* d, const BatchTable* t, int stage, int tx, int ty,
                               hipStream_t st) {
  const unsigned g = 1024;
  if (tx == 64 && ty == 4) k_b_rhs<F, 64, 4><<<g, 256, 0, st>>>(d, t, stage);
  else if (tx == 32 && ty == 8) k_b_rhs<F, 32, 8><<<g, 256, 0, st>>>(d, t, stage);
  else if (tx == 64 && ty == 2) k_b_rhs<F, 64, 2><<<g, 128, 0, st>>>(d, t, stage);
  else if (tx == 128 && ty == 2) k_b_rhs<F, 128, 2><<<g, 256, 0, st>>>(d, t, stage);
  else if (tx == 64 && ty == 8) k_b_rhs<F, 64, 8><<<g, 512, 0, st>>>(d, t, stage);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_batch_phase(int phase, const Desc* d, const BatchTable* t, int stage, int tx,
                              int ty, int precision, hipStream_t st) {
  switch (phase) {
    case BPH_BEGIN: k_b_begin<<<1, 64, 0, st>>>(d, t); break;
    case BPH_DT_PART: k_b_dt_part<<<2048, 256, 0, st>>>(d, t); break;
    case BPH_DT_FINAL: k_b_dt_final<<<kMaxSlots, 256, 0, st>>>(d, t); break;
    case BPH_GHOST_X: k_b_ghost_x<<<512, 256, 0, st>>>(d, t, stage); break;
    case BPH_GHOST_Y: k_b_ghost_y<<<512, 256, 0, st>>>(d, t, stage); break;
    case BPH_SENSOR: k_b_sensor<<<4096, 256, 0, st>>>(d, t, stage); break;
    case BPH_IFLAGS: k_b_iflags<<<4096, 256, 0, st>>>(d, t); break;
    case BPH_WENO:
      if (precision == 1) k_b_weno<float><<<2048, 256, 0, st>>>(d, t, stage);
      else k_b_weno<double><<<2048, 256, 0, st>>>(d, t, stage);
      break;
    case BPH_RHS:
      return precision == 1 ? launch_b_rhs<float>(d, t, stage, tx, ty, st)
                            : launch_b_rhs<double>(d, t, stage, tx, ty, st);
    case BPH_FORCE: k_b_force<<<kMaxSlots, 256, 0, st>>>(d, t); break;
    case BPH_RK: k_b_rk<<<4096, 256, 0, st>>>(d, t, stage, tx == 64 && ty == 4 ? 1 : 0); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace cdns
