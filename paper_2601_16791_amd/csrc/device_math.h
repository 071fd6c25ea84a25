// Device-side mathematics of the hybrid step for gfx950 (FP64 VALU).
//
// Everything here is inline __device__ code used by the kernels of the step:
// the changeover weight of the direct force (Sect. 2.1.3), the gas drag of
// Sect. 3.1 (Eqs. 1-7), the universal-variable Kepler drift, the Hermite
// minimum-separation test of the encounter search, and fixed-order block
// reductions (run-to-run bitwise determinism: no floating-point atomics).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mx_internal.h"

namespace mxd {

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrt2Pi = 2.5066282746310002;   // sqrt(2 pi)
constexpr double kSqrt8OverPi = 1.5957691216057308; // sqrt(8 / pi)

// Full-precision reciprocal square root: the hardware estimate (about 2^-24
// relative) corrected by one third-order step y (1 + e/2 + 3e^2/8), e = 1 - x y^2.
__device__ __forceinline__ double rsqrt_full(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

// Pair weight inside the changeover zone (s2 < rc2): K(s)/s^3 with the
// branches of the direct-force routine; rc2 = rc*rc.
__device__ __forceinline__ double changeover_weight_slow(double s2, double rc, double rc2) {
  if (s2 <= 0.01 * rc2) return 0.0;
  double s = sqrt(s2);
  double si = 1.0 / s;
  double q = (s - 0.1 * rc) / (0.9 * rc);
  double q2 = q * q, q3 = q * q2, q4 = q2 * q2, q5 = q2 * q3;
  return (10.0 * q3 - 15.0 * q4 + 6.0 * q5) * si * si * si;
}

// K itself (0..1) for the complementary force of the encounter integrator.
__device__ __forceinline__ double changeover_k(double s2, double rc) {
  double rc2 = rc * rc;
  if (s2 >= rc2) return 1.0;
  if (s2 <= 0.01 * rc2) return 0.0;
  double s = sqrt(s2);
  double q = (s - 0.1 * rc) / (0.9 * rc);
  double q2 = q * q, q3 = q * q2, q4 = q2 * q2, q5 = q2 * q3;
  return 10.0 * q3 - 15.0 * q4 + 6.0 * q5;
}

// ------------------------------------------------------------------ gas drag
// Drag acceleration of one massless body (Sect. 3.1): midplane gas density
// Sigma/(sqrt(2 pi) h) (Eq. 4) with Sigma of Eq. 1, gas velocity v_k sqrt(1-2eta)
// along phi-hat (Eq. 5), C_D of Eq. 7 with Ma = |dv|/c_s and Re = 2 r_p |dv| / nu,
// nu = sqrt(8/pi) c_s lambda / 3, and F_D of Eq. 3 directed against dv.
// (vx, vy, vz) is the heliocentric velocity.  Returns a zero vector where the
// gas density vanishes or dv = 0.
// DragConst and make_drag_const live in mx_internal.h (host and device).

__device__ __forceinline__ double pow_kexp(double b, double kexp) {
  if (kexp == -2.0) return 1.0 / (b * b);
  if (kexp == -1.0) return 1.0 / b;
  return pow(b, kexp);
}

// Sound speed, midplane density and gas speed of the general disk (c.ext): c_s
// from T(R) = T0 (R/1AU)^-beta (Eq. 2) or h_over_r v_K; scale height c_s/Omega;
// the density factor of the gaps (Eqs. 8-9); eta fixed or eta(R) of Eq. 6; and the
// disk gravity of Eqs. 10-12 (signed radial, positive away from the star) into
// (gx, gy).
__device__ __noinline__ void gas_general(const DragConst& c, double X, double Y, double R,
                                         double inv_R, double vk, double sig, double& cs,
                                         double& rhog, double& vg, double& gx, double& gy) {
  if (c.cs2_1au > 0.0) cs = sqrt(c.cs2_1au * pow(R, -c.beta));
  else cs = c.h_over_r * vk;
  // rho_g = Sigma / (sqrt(2 pi) c_s / Omega) = Sigma v_K / (sqrt(2 pi) c_s R)
  rhog = sig * vk * inv_R / (kSqrt2Pi * cs);
  // the gaps of the massive bodies (dens_factor of Sect. 3.1.1): the open gap of
  // the highest index with R strictly inside it scales the density
  for (int i = 0; i < c.gap_n; ++i) {
    const double* g = c.gaps + 4 * i;
    if (g[3] != 0.0 && R < g[0] + g[1] && R > g[0] - g[1]) rhog = sig * vk * inv_R / (kSqrt2Pi * cs) * g[2];
  }
  double eta = c.eta;
  if (c.eta6_fac != 0.0) {
    const double m = cs / vk;
    eta = c.eta6_fac * m * m;
  }
  vg = vk * sqrt(1.0 - 2.0 * eta);
  gx = gy = 0.0;
  if (c.dg_fac != 0.0) {
    const double g = c.dg_edge ? c.dg_fac * sig * inv_R : c.dg_fac * sig;
    gx = g * X * inv_R;
    gy = g * Y * inv_R;
  }
}

// The part of the drag that depends only on the position (X, Y): the disk's
// surface density, sound speed, gas density and velocity and the disk gravity
// at R.  A body closed and opened at the same position (the closing kick of one
// step and the opening kick of the next) can evaluate it once.  on = 0: no gas
// there (R = 0, inside the inner edge, or Sigma = 0): no drag, no disk gravity.
// Written with few divisions (each is a long dependent chain in FP64):
// c_s = (H/r) v_k; rho_g = Sigma / (sqrt(2 pi) (H/r) R).
struct GasSite {
  double X, Y, inv_R, cs, rhog, vg, gx, gy;
  int on;
};

__device__ __forceinline__ GasSite gas_site(const DragConst& c, double X, double Y) {
  GasSite g;
  g.on = 0;
  g.X = X;
  g.Y = Y;
  g.gx = g.gy = 0.0;
  double R2 = X * X + Y * Y;
  double R = sqrt(R2);
  if (!(R > 0.0) || R < c.r_in) return g;
  double inv_R = 1.0 / R;
  double vk = sqrt(c.mu0 * inv_R);
  double sig;
  if (c.gamma == 1.0) sig = c.sigma1_unit * inv_R;
  else sig = c.sigma1_unit * pow(R, -c.gamma);
  if (c.r_c > 0.0) sig *= exp(c.rc_norm - pow(R * c.inv_rc, 2.0 - c.gamma));
  if (!(sig > 0.0)) return g;
  double cs, rhog, vg, gx, gy;
  if (__builtin_expect(c.ext != 0, 0)) {
    // the outputs start at zero only on this branch: the call takes their
    // addresses, so the plain disk stores nothing to private memory
    gx = gy = 0.0;
    gas_general(c, X, Y, R, inv_R, vk, sig, cs, rhog, vg, gx, gy);
  } else {
    cs = c.h_over_r * vk;
    rhog = sig * inv_R * c.rho_fac;
    vg = vk * c.vg_fac;
    gx = gy = 0.0;
  }
  g.inv_R = inv_R;
  g.cs = cs;
  g.rhog = rhog;
  g.vg = vg;
  g.gx = gx;
  g.gy = gy;
  g.on = 1;
  return g;
}

// Drag (and disk gravity) at site g on a body of radius r_p and density rho_p
// moving at (vx, vy, vz): Re = 2 r_p dv / nu with nu = sqrt(8/pi) c_s (mfp /
// rho_g) / 3, i.e. Re = re_fac r_p dv rho_g / c_s;
// 1 / (24/Re + 40/(10 + Re)) = Re (10 + Re) / (240 + 64 Re).
__device__ __forceinline__ void gas_drag_at(const DragConst& c, const GasSite& g, double vx,
                                            double vy, double vz, double r_p, double rho_p,
                                            double& ax, double& ay, double& az) {
  ax = ay = az = 0.0;
  if (!g.on) return;
  ax = g.gx;
  ay = g.gy;
  double dvx = vx + g.vg * g.Y * g.inv_R;
  double dvy = vy - g.vg * g.X * g.inv_R;
  double dvz = vz;
  double dv = sqrt(dvx * dvx + dvy * dvy + dvz * dvz);
  if (!(dv > 0.0)) return;
  double inv_cs = 1.0 / g.cs;
  double ma = dv * inv_cs;
  double re = c.re_fac * r_p * dv * g.rhog * inv_cs;
  double k = re < 1.0e5 ? 0.4 : 0.2;
  double inner = re * (10.0 + re) / fma(64.0, re, 240.0) + 0.23 * ma;
  double cd = pow_kexp(inner, c.kexp) + 2.0 * (0.8 * k + ma) / (1.6 + ma);
  double f = -0.375 * cd * g.rhog * dv / (r_p * rho_p);
  ax = fma(f, dvx, g.gx);
  ay = fma(f, dvy, g.gy);
  az = f * dvz;
}

__device__ __forceinline__ void gas_drag(const DragConst& c, double X, double Y, double vx,
                                         double vy, double vz, double r_p, double rho_p,
                                         double& ax, double& ay, double& az) {
  const GasSite g = gas_site(c, X, Y);
  gas_drag_at(c, g, vx, vy, vz, r_p, rho_p, ax, ay, az);
}

// ------------------------------------------------------------ Kepler drift
// Stumpff functions c0..c3 of z: the defining series on |z| <= 0.5, reached by
// quartering z, then the quadruplication identities
//   c0(4z) = 2 c0^2 - 1,  c1(4z) = c0 c1,  c2(4z) = c1^2 / 2,
//   c3(4z) = (c2 + c0 c3) / 4.
__device__ __forceinline__ void stumpff(double z, double& c0, double& c1, double& c2,
                                        double& c3) {
  int n = 0;
  while (fabs(z) > 0.5 && n < 60) {
    z *= 0.25;
    ++n;
  }
  // c2 = sum (-z)^k / (2k+2)!,  c3 = sum (-z)^k / (2k+3)!,  k = 0..8
  c2 = fma(z, fma(z, fma(z, fma(z, fma(z, fma(z, fma(z, -1.0 / 6402373705728000.0,
       1.0 / 20922789888000.0), -1.0 / 87178291200.0), 1.0 / 479001600.0),
       -1.0 / 3628800.0), 1.0 / 40320.0), -1.0 / 720.0), 1.0 / 24.0);
  c2 = fma(-z, c2, 0.5);
  c3 = fma(z, fma(z, fma(z, fma(z, fma(z, fma(z, fma(z, -1.0 / 121645100408832000.0,
       1.0 / 355687428096000.0), -1.0 / 1307674368000.0), 1.0 / 6227020800.0),
       -1.0 / 39916800.0), 1.0 / 362880.0), -1.0 / 5040.0), 1.0 / 120.0);
  c3 = fma(-z, c3, 1.0 / 6.0);
  c1 = fma(-z, c3, 1.0);
  c0 = fma(-z, c2, 1.0);
  for (int i = 0; i < n; ++i) {
    c3 = 0.25 * fma(c0, c3, c2);
    c2 = 0.5 * c1 * c1;
    c1 = c0 * c1;
    c0 = fma(2.0 * c0, c0, -1.0);
  }
}

// Advance (x, v) on the two-body orbit about mu over h.  Universal variable s
// with beta = 2 mu / r0 - v0^2:  h = r0 s + eta0 G2 + zeta0 G3,
// G_k = s^k c_k(beta s^2), eta0 = x0.v0, zeta0 = mu - beta r0, solved by Halley's
// method inside a bisection bracket (the time equation is increasing in s, its
// derivative being r); then the Lagrange functions f = 1 - mu G2 / r0,
// g = h - mu G3, fdot = -mu G1 / (r r0), gdot = 1 - mu G2 / r.  A bound orbit is
// first advanced by whole periods (h reduced to |h| <= P/2), which brackets s in
// [-S, S] with S = 2 pi / sqrt(beta) the s-length of one period.  Returns false if
// the iteration did not converge (state left unchanged).
__device__ __forceinline__ void kepler_eval(double beta, double r0, double eta, double zeta,
                                            double s, double& c0, double& G1, double& G2,
                                            double& G3) {
  double c1, c2, c3;
  stumpff(beta * s * s, c0, c1, c2, c3);
  G1 = s * c1;
  G2 = s * s * c2;
  G3 = s * s * s * c3;
}

__device__ __forceinline__ bool kepler_drift(double mu, double h, double& x, double& y,
                                             double& z, double& vx, double& vy, double& vz) {
  if (h == 0.0) return true;
  double r0 = sqrt(x * x + y * y + z * z);
  double v2 = vx * vx + vy * vy + vz * vz;
  double eta = x * vx + y * vy + z * vz;
  double inv_r0 = 1.0 / r0;
  double beta = 2.0 * mu * inv_r0 - v2;
  double zeta = mu - beta * r0;
  double c0, G1, G2, G3;
  double lo, hi;
  if (beta > 0.0) {
    double isb = 1.0 / sqrt(beta);
    double S = 2.0 * kPi * isb;
    double P = S * mu * (isb * isb);   // 2 pi mu / beta^(3/2)
    if (fabs(h) > 0.5 * P) h -= rint(h / P) * P;
    lo = -S;
    hi = S;
  } else {
    // outward doubling from h / r0 until the time equation changes sign
    double sg = h > 0.0 ? 1.0 : -1.0;
    lo = 0.0;
    hi = h * inv_r0;
    for (int it = 0; it < 200; ++it) {
      kepler_eval(beta, r0, eta, zeta, hi, c0, G1, G2, G3);
      double F = fma(r0, hi, fma(eta, G2, fma(zeta, G3, -h)));
      if (sg * F >= 0.0) break;
      lo = hi;
      hi *= 2.0;
    }
    if (sg < 0.0) {
      double t = lo; lo = hi; hi = t;
    }
  }
  double s = h * inv_r0 - 0.5 * h * h * eta * inv_r0 * inv_r0 * inv_r0;
  if (!(s > lo && s < hi)) s = 0.5 * (lo + hi);
  bool ok = false;
  // A Halley step that leaves the bracket, or (after the first steps) does not at
  // least halve the previous correction, is replaced by a bisection of the
  // bracket, so stiff cases (near-radial orbits through a close pericentre) still
  // converge within the cap.
  double ds_prev = hi - lo;
  for (int it = 0; it < 120; ++it) {
    kepler_eval(beta, r0, eta, zeta, s, c0, G1, G2, G3);
    double F = fma(r0, s, fma(eta, G2, fma(zeta, G3, -h)));
    double Fp = fma(eta, G1, fma(zeta, G2, r0));
    double Fpp = fma(eta, c0, zeta * G1);
    if (F == 0.0) {
      ok = true;
      break;
    }
    if (F < 0.0) lo = s;
    else hi = s;
    double sn = s - F * Fp / fma(Fp, Fp, -0.5 * F * Fpp);  // Halley step
    if (fabs(sn - s) <= 1e-13 * fabs(sn)) {
      s = sn;
      ok = true;
      break;
    }
    if (!(sn > lo && sn < hi) || (it >= 4 && fabs(sn - s) > 0.5 * ds_prev))
      sn = 0.5 * (lo + hi);
    double ds = sn - s;
    ds_prev = fabs(ds);
    s = sn;
    if (fabs(ds) <= 1e-13 * fabs(s) || lo == hi) {
      ok = true;
      break;
    }
  }
  if (!ok) return false;
  kepler_eval(beta, r0, eta, zeta, s, c0, G1, G2, G3);
  double r = fma(eta, G1, fma(zeta, G2, r0));
  double f = 1.0 - mu * G2 * inv_r0;
  double g = h - mu * G3;
  double inv_r = 1.0 / r;
  double fd = -mu * G1 * inv_r * inv_r0;
  double gd = 1.0 - mu * G2 * inv_r;
  double nx = f * x + g * vx, ny = f * y + g * vy, nz = f * z + g * vz;
  double nvx = fd * x + gd * vx, nvy = fd * y + gd * vy, nvz = fd * z + gd * vz;
  x = nx; y = ny; z = nz;
  vx = nvx; vy = nvy; vz = nvz;
  return true;
}

// ---------------------------------------------------- encounter separation
// Minimum squared separation over the step of the cubic Hermite interpolant
// of the relative position (end values r0, r1 and rates w0, w1 over [0, h]):
// the end points plus each interior minimum of |r|^2 located by a sign change
// (negative to non-negative) of d|r|^2/dtau on a 16-interval grid, refined by
// 40 bisection steps.  The derivative (halved) is r . r', a quintic in tau
// whose coefficient of tau^m is the sum of j c_i . c_j over i + j = m + 1
// (c_0..c_3 the cubic's coefficients), evaluated by Horner's rule.  Evaluated
// without contraction so that it is the plain sequence of IEEE operations of
// its definition.
#pragma clang fp contract(off)
__device__ __noinline__ double hermite_dmin2(double r0x, double r0y, double r0z, double w0x,
                                             double w0y, double w0z, double r1x, double r1y,
                                             double r1z, double w1x, double w1y, double w1z,
                                             double h) {
  double c[4][3];
  double r0[3] = {r0x, r0y, r0z}, r1[3] = {r1x, r1y, r1z};
  double w0[3] = {w0x, w0y, w0z}, w1[3] = {w1x, w1y, w1z};
  for (int k = 0; k < 3; ++k) {
    c[0][k] = r0[k];
    c[1][k] = h * w0[k];
    c[2][k] = 3.0 * (r1[k] - r0[k]) - h * (2.0 * w0[k] + w1[k]);
    c[3][k] = 2.0 * (r0[k] - r1[k]) + h * (w0[k] + w1[k]);
  }
  auto dot3 = [&](int i, int j) {
    return c[i][0] * c[j][0] + c[i][1] * c[j][1] + c[i][2] * c[j][2];
  };
  double a[6];
  a[0] = dot3(0, 1);
  a[1] = dot3(1, 1) + 2.0 * dot3(0, 2);
  a[2] = 3.0 * dot3(0, 3) + 3.0 * dot3(1, 2);
  a[3] = 4.0 * dot3(1, 3) + 2.0 * dot3(2, 2);
  a[4] = 5.0 * dot3(2, 3);
  a[5] = 3.0 * dot3(3, 3);
  double d0 = r0x * r0x + r0y * r0y + r0z * r0z;
  double d1 = r1x * r1x + r1y * r1y + r1z * r1z;
  double best = d0 < d1 ? d0 : d1;
  auto dd = [&](double t) {
    return a[0] + t * (a[1] + t * (a[2] + t * (a[3] + t * (a[4] + t * a[5]))));
  };
  // the 17 grid values are independent: evaluate them all first
  constexpr int NG = 16;
  double g[NG + 1];
#pragma unroll
  for (int k = 0; k <= NG; ++k) g[k] = dd((double)k / NG);
  // intervals holding a sign change, as a bit mask: the lanes of a wave then
  // refine their first, second, ... roots together whatever their intervals
  uint32_t roots = 0;
#pragma unroll
  for (int k = 0; k < NG; ++k) roots |= (g[k] < 0.0 && g[k + 1] >= 0.0) ? (1u << k) : 0u;
  while (roots != 0) {
    const int k = __builtin_ctz(roots);
    roots &= roots - 1;
    {
      double lo = (double)k / NG, hi = (double)(k + 1) / NG;
      // 40 bisection steps taken two at a time: the midpoint and both possible
      // next midpoints are evaluated together, then the two decisions are
      // made in order (the same points and decisions as one step at a time)
      for (int it = 0; it < 20; ++it) {
        const double mid = 0.5 * (lo + hi);
        const double qa = 0.5 * (lo + mid), qb = 0.5 * (mid + hi);
        const double fm = dd(mid), fa = dd(qa), fb = dd(qb);
        if (fm < 0.0) {
          lo = mid;
          if (fb < 0.0) lo = qb;
          else hi = qb;
        } else {
          hi = mid;
          if (fa < 0.0) lo = qa;
          else hi = qa;
        }
      }
      double t = 0.5 * (lo + hi);
      double r[3];
      for (int q = 0; q < 3; ++q) r[q] = c[0][q] + t * (c[1][q] + t * (c[2][q] + t * c[3][q]));
      double d = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      if (d < best) best = d;
    }
  }
  return best;
}
#pragma clang fp contract(on)

// ---------------------------------------------------------- reductions
// Sum over the 64 lanes of a wave (all lanes active), the same bits on every
// lane and for every caller.  Within each row of 16 lanes, DPP moves pair lane i
// with i ^ 1, i ^ 2, then 7 - i within eight and 15 - i within sixteen: each
// step adds the same two partial sums on both lanes of a pair (in either
// order, which IEEE addition does not distinguish), so every lane of a row ends
// with the row's sum; the four row sums are then added as (r0 + r1) + (r2 + r3).
template <int CTRL>
__device__ __forceinline__ double dpp_move_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}

__device__ __forceinline__ double wave_sum_fixed(double v) {
  v += dpp_move_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move_f64<0x141>(v);  // row_half_mirror
  v += dpp_move_f64<0x140>(v);  // row_mirror
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Fixed-order sum over a block of BS threads (power of two): each thread's value
// lands in LDS, then a binary tree with a fixed pairing.  Every block that runs
// the same reduction on the same data gets the same bits.
template <int BS, int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* sh) {
  const int tid = threadIdx.x;
  for (int k = 0; k < K; ++k) sh[k * BS + tid] = v[k];
  __syncthreads();
  for (int w = BS / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int k = 0; k < K; ++k) sh[k * BS + tid] += sh[k * BS + tid + w];
    __syncthreads();
  }
  for (int k = 0; k < K; ++k) v[k] = sh[k * BS];
  __syncthreads();
}

// Fixed-order sum over a block of BS threads (a multiple of 64, at most 1024):
// each wave sums its lanes by the fixed DPP reduction, then every thread adds
// the waves' sums from LDS as a pairwise tree (one barrier instead of one per
// level).  Every block that runs it on the same data gets the same bits.
template <int BS, int K>
__device__ __forceinline__ void block_sum_waves(double (&v)[K], double* sh) {
  constexpr int W = BS / 64;
  static_assert(W >= 1 && (W & (W - 1)) == 0 && W <= 16, "waves per block");
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum_fixed(v[k]);
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < K; ++k) sh[k * W + w] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t[W];
#pragma unroll
    for (int i = 0; i < W; ++i) t[i] = sh[k * W + i];
#pragma unroll
    for (int span = 1; span < W; span <<= 1)
#pragma unroll
      for (int i = 0; i + span < W; i += 2 * span) t[i] = t[i] + t[i + span];
    v[k] = t[0];
  }
  __syncthreads();
}

}  // namespace mxd
