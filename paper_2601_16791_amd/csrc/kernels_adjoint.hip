// Reverse-mode adjoint of the hybrid step for systems with n_big <= 64
// (gfx950, FP64).
//
// The forward step (half kick with gravity and gas drag, jump by the massive-body
// momentum, Kepler drift or Bulirsch-Stoer for the encounter subsystems, jump,
// half kick with the new gravity) is differentiated sub-step by sub-step in
// reverse order.  lx, lu hold the adjoint of the DH state (x, u), lmu the
// adjoint of the massive-body mu = G m.  The changeover radii are constants of
// the map (not differentiated).
//
//   k_adj_kick      : vector-Jacobian product of one half kick: the pair term of
//                     the changeover-weighted gravity (mu f(r) d with
//                     f = K(r)/r^3, Jacobian f I + f'(r)/r d d^T), its mass term,
//                     and the drag Jacobian (forward-mode over the drag formula,
//                     drag regime fixed); source-side sums reduced per wave
//   k_adj_reduce_apply : fixed-order sums of the per-wave partials, applied to
//                     the massive bodies by the block that ends last, with the
//                     momentum terms of the jump and of the heliocentric
//                     velocity that the drag sees
//   k_adj_drift     : transposed Jacobian of the Kepler map per body, by
//                     forward-mode evaluation at the solved universal variable,
//                     whose tangent comes from the solved time equation
//   k_adj_bs        : tangents of the Bulirsch-Stoer map of a subsystem along
//                     the accepted step sizes and columns of the forward run, one
//                     input direction and column per thread, contracted with the
//                     adjoint of the kept members
//   k_adj_bs_apply  : those contributions added in a fixed order
//   k_adj_sum3      : per-wave sums of an adjoint over all bodies, whose
//                     momentum term (jumps, DH <-> heliocentric) the reduction
//                     above applies
//   k_adj_copy, k_adj_record : saved states, and the per-step record (state,
//                     subsystem table, accepted Bulirsch-Stoer steps) kept for
//                     the reverse pass
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "mx_internal.h"

namespace {

constexpr int kBlock = 256;

// ------------------------------------------------------------------ duals
template <int N>
struct Dn {
  double v;
  double d[N];
};

template <int N>
__device__ __forceinline__ Dn<N> dconst(double v) {
  Dn<N> r;
  r.v = v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = 0.0;
  return r;
}

template <int N>
__device__ __forceinline__ Dn<N> dseed(double v, int k) {
  Dn<N> r = dconst<N>(v);
  r.d[k] = 1.0;
  return r;
}

template <int N>
__device__ __forceinline__ Dn<N> operator+(const Dn<N>& a, const Dn<N>& b) {
  Dn<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator-(const Dn<N>& a, const Dn<N>& b) {
  Dn<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator-(const Dn<N>& a) {
  Dn<N> r;
  r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator*(const Dn<N>& a, const Dn<N>& b) {
  Dn<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator/(const Dn<N>& a, const Dn<N>& b) {
  Dn<N> r;
  r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator+(const Dn<N>& a, double b) {
  Dn<N> r = a;
  r.v += b;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator+(double b, const Dn<N>& a) {
  return a + b;
}
template <int N>
__device__ __forceinline__ Dn<N> operator-(const Dn<N>& a, double b) {
  Dn<N> r = a;
  r.v -= b;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator-(double b, const Dn<N>& a) {
  Dn<N> r = -a;
  r.v += b;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator*(const Dn<N>& a, double b) {
  Dn<N> r;
  r.v = a.v * b;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator*(double b, const Dn<N>& a) {
  return a * b;
}
template <int N>
__device__ __forceinline__ Dn<N> operator/(const Dn<N>& a, double b) {
  return a * (1.0 / b);
}
template <int N>
__device__ __forceinline__ Dn<N> operator/(double a, const Dn<N>& b) {
  Dn<N> r;
  r.v = a / b.v;
  const double k = -r.v / b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = k * b.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> chain(const Dn<N>& a, double fv, double dfv) {
  Dn<N> r;
  r.v = fv;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * dfv;
  return r;
}
template <int N>
__device__ __forceinline__ Dn<N> dsqrt(const Dn<N>& a) {
  const double s = sqrt(a.v);
  return chain(a, s, 0.5 / s);
}
template <int N>
__device__ __forceinline__ Dn<N> dexp(const Dn<N>& a) {
  const double e = exp(a.v);
  return chain(a, e, e);
}
template <int N>
__device__ __forceinline__ Dn<N> dpowc(const Dn<N>& a, double p) {
  return chain(a, pow(a.v, p), p * pow(a.v, p - 1.0));
}

// ------------------------------------------------------------------ drag
// Jacobian-transpose product of the gas drag (Sect. 3.1, Eqs. 1, 3, 4, 5, 7) of
// one massless body: inputs (X, Y, vx, vy, vz) with v the heliocentric
// velocity; returns (g . da/dX, g . da/dY, g . da/dv).  The drag regime (the k
// switch of Eq. 7, a vanishing density) is taken at the value.
__device__ void drag_vjp(const mxd::DragConst& c, double X0, double Y0, double vx0, double vy0,
                         double vz0, double r_p, double rho_p, const double (&g)[3],
                         double (&out)[5]) {
  typedef Dn<5> T;
  for (int i = 0; i < 5; ++i) out[i] = 0.0;
  const T X = dseed<5>(X0, 0), Y = dseed<5>(Y0, 1);
  const T vx = dseed<5>(vx0, 2), vy = dseed<5>(vy0, 3), vz = dseed<5>(vz0, 4);
  const T R = dsqrt(X * X + Y * Y);
  if (!(R.v > 0.0) || R.v < c.r_in) return;
  const T inv_R = 1.0 / R;
  const T vk = dsqrt(c.mu0 * inv_R);
  const T om = vk * inv_R;
  const T hg = c.h_over_r * R;
  const T cs = hg * om;
  T sig = c.gamma == 1.0 ? c.sigma1_unit * inv_R : c.sigma1_unit * dpowc(R, -c.gamma);
  if (c.r_c > 0.0) sig = sig * dexp(c.rc_norm - dpowc(R * c.inv_rc, 2.0 - c.gamma));
  if (!(sig.v > 0.0)) return;
  const T rhog = sig / (mxd::kSqrt2Pi * hg);
  const T vg = vk * c.vg_fac;
  const T dvx = vx + vg * Y * inv_R;
  const T dvy = vy - vg * X * inv_R;
  const T dvz = vz;
  const T dv = dsqrt(dvx * dvx + dvy * dvy + dvz * dvz);
  if (!(dv.v > 0.0)) return;
  const T ma = dv / cs;
  const T lam = c.mfp_coef / rhog;
  const T nu = ((1.0 / 3.0) * mxd::kSqrt8OverPi) * cs * lam;
  const T re = (2.0 * r_p) * dv / nu;
  const double k = re.v < 1.0e5 ? 0.4 : 0.2;
  const T inner = 1.0 / (24.0 / re + 40.0 / (10.0 + re)) + 0.23 * ma;
  const T cd = dpowc(inner, c.kexp) + 2.0 * (0.8 * k + ma) / (1.6 + ma);
  const T f = (-0.375 / r_p / rho_p) * cd * rhog * dv;
  const T ax = f * dvx, ay = f * dvy, az = f * dvz;
  for (int i = 0; i < 5; ++i) out[i] = g[0] * ax.d[i] + g[1] * ay.d[i] + g[2] * az.d[i];
}

// ------------------------------------------------------------------ Kepler
// Stumpff functions c0..c3 of a dual argument: the series after quartering the
// value of z to |z| <= 0.5, then the quadruplication identities.
template <int N>
__device__ void dstumpff(const Dn<N>& z0, Dn<N>& c0, Dn<N>& c1, Dn<N>& c2, Dn<N>& c3) {
  int q = 0;
  Dn<N> z = z0;
  while (fabs(z.v) > 0.5 && q < 64) {
    z = z * 0.25;
    ++q;
  }
  // c2 = sum (-z)^k / (2k+2)!, c3 = sum (-z)^k / (2k+3)!, k = 0..10
  double a2[11], a3[11];
  double f2 = 2.0, f3 = 6.0;
  for (int k = 0; k < 11; ++k) {
    a2[k] = (k & 1 ? -1.0 : 1.0) / f2;
    a3[k] = (k & 1 ? -1.0 : 1.0) / f3;
    f2 *= (2.0 * k + 3.0) * (2.0 * k + 4.0);
    f3 *= (2.0 * k + 4.0) * (2.0 * k + 5.0);
  }
  c2 = dconst<N>(a2[10]);
  c3 = dconst<N>(a3[10]);
  for (int k = 9; k >= 0; --k) {
    c2 = c2 * z + a2[k];
    c3 = c3 * z + a3[k];
  }
  c1 = 1.0 - z * c3;
  c0 = 1.0 - z * c2;
  for (int i = 0; i < q; ++i) {
    c3 = 0.25 * (c0 * c3 + c2);
    c2 = 0.5 * c1 * c1;
    c1 = c0 * c1;
    c0 = 2.0 * c0 * c0 - 1.0;
  }
}

// The universal variable s of the drift (value only) and the number of whole
// periods removed from h; same equation and bracket as the forward solver.
__device__ bool kepler_solve_s(double mu, double h, const double (&x)[3], const double (&v)[3],
                               double& s_out, double& nper) {
  const double r0 = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double eta = x[0] * v[0] + x[1] * v[1] + x[2] * v[2];
  const double inv_r0 = 1.0 / r0;
  const double beta = 2.0 * mu * inv_r0 - v2;
  const double zeta = mu - beta * r0;
  double lo, hi, c0, G1, G2, G3;
  nper = 0.0;
  if (beta > 0.0) {
    const double sb = sqrt(beta);
    const double S = 2.0 * mxd::kPi / sb;
    const double P = S * mu / beta;
    if (fabs(h) > 0.5 * P) {
      nper = rint(h / P);
      h -= nper * P;
    }
    lo = -S;
    hi = S;
  } else {
    const double sg = h > 0.0 ? 1.0 : -1.0;
    lo = 0.0;
    hi = h * inv_r0;
    for (int it = 0; it < 200; ++it) {
      mxd::kepler_eval(beta, r0, eta, zeta, hi, c0, G1, G2, G3);
      double F = fma(r0, hi, fma(eta, G2, fma(zeta, G3, -h)));
      if (sg * F >= 0.0) break;
      lo = hi;
      hi *= 2.0;
    }
    if (sg < 0.0) {
      double t = lo;
      lo = hi;
      hi = t;
    }
  }
  double s = h * inv_r0 - 0.5 * h * h * eta * inv_r0 * inv_r0 * inv_r0;
  if (!(s > lo && s < hi)) s = 0.5 * (lo + hi);
  for (int it = 0; it < 80; ++it) {
    mxd::kepler_eval(beta, r0, eta, zeta, s, c0, G1, G2, G3);
    double F = fma(r0, s, fma(eta, G2, fma(zeta, G3, -h)));
    double Fp = fma(eta, G1, fma(zeta, G2, r0));
    double Fpp = fma(eta, c0, zeta * G1);
    if (F == 0.0) {
      s_out = s;
      return true;
    }
    if (F < 0.0) lo = s;
    else hi = s;
    double sn = s - F / (Fp - 0.5 * F * Fpp / Fp);
    if (fabs(sn - s) <= 1e-13 * fabs(sn)) {
      s_out = sn;
      return true;
    }
    if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
    double ds = sn - s;
    s = sn;
    if (fabs(ds) <= 1e-13 * fabs(s) || lo == hi) {
      s_out = s;
      return true;
    }
  }
  return false;
}

// (lx0, lv0) = J^T (lx1, lv1) for the Kepler map (x0, v0) -> (x1, v1) over h.
// The map is evaluated in dual arithmetic at the solved s; the tangent of s is
// minus the tangent of the time equation over its s-derivative r.  Whole
// periods removed from h enter through the derivative of the period.
__device__ bool kepler_vjp(double mu, double h, const double (&x0)[3], const double (&v0)[3],
                           const double (&lx1)[3], const double (&lv1)[3], double (&lx0)[3],
                           double (&lv0)[3]) {
  typedef Dn<6> T;
  if (h == 0.0) {
    for (int c = 0; c < 3; ++c) {
      lx0[c] = lx1[c];
      lv0[c] = lv1[c];
    }
    return true;
  }
  double s, nper;
  if (!kepler_solve_s(mu, h, x0, v0, s, nper)) return false;
  T X[3], V[3];
  for (int c = 0; c < 3; ++c) {
    X[c] = dseed<6>(x0[c], c);
    V[c] = dseed<6>(v0[c], 3 + c);
  }
  const T r0 = dsqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
  const T v2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
  const T eta = X[0] * V[0] + X[1] * V[1] + X[2] * V[2];
  const T beta = 2.0 * mu / r0 - v2;
  const T zeta = mu - beta * r0;
  T hr = dconst<6>(h);
  if (nper != 0.0) {
    // P = 2 pi mu beta^(-3/2)
    const T P = (2.0 * mxd::kPi * mu) * dpowc(beta, -1.5);
    hr = h - nper * P;
  }
  T c0, c1, c2, c3;
  // tangent of s from the time equation at fixed s
  T sd = dconst<6>(s);
  dstumpff(beta * (s * s), c0, c1, c2, c3);
  {
    const T G2 = (s * s) * c2, G3 = (s * s * s) * c3, G1 = s * c1;
    const T F = r0 * s + eta * G2 + zeta * G3 - hr;
    const double r = (r0 + eta * G1 + zeta * G2).v;
    for (int i = 0; i < 6; ++i) sd.d[i] = -F.d[i] / r;
  }
  dstumpff(beta * sd * sd, c0, c1, c2, c3);
  const T G1 = sd * c1, G2 = sd * sd * c2, G3 = sd * sd * sd * c3;
  const T r = r0 + eta * G1 + zeta * G2;
  const T f = 1.0 - mu * G2 / r0;
  const T g = hr - mu * G3;
  const T fd = -mu * G1 / (r * r0);
  const T gd = 1.0 - mu * G2 / r;
  for (int i = 0; i < 3; ++i) lx0[i] = lv0[i] = 0.0;
  for (int c = 0; c < 3; ++c) {
    const T x1 = f * X[c] + g * V[c];
    const T v1 = fd * X[c] + gd * V[c];
    for (int i = 0; i < 3; ++i) {
      lx0[i] += x1.d[i] * lx1[c] + v1.d[i] * lv1[c];
      lv0[i] += x1.d[3 + i] * lx1[c] + v1.d[3 + i] * lv1[c];
    }
  }
  return true;
}

// ------------------------------------------------------------------ helpers
// Fixed-order sum over the 64 lanes of a wave by DPP row moves (all lanes active).
__device__ __forceinline__ double wave_sum(double v) { return mxd::wave_sum_fixed(v); }

// f(r) = K(r)/r^3 and F1 = f'(r)/r of the changeover-weighted pair force
__device__ __forceinline__ void pair_f(double s2, double rc, double& f, double& F1) {
  const double rc2 = rc * rc;
  const double ir = mxd::rsqrt_full(s2), r = s2 * ir, ir2 = ir * ir, ir3 = ir2 * ir;
  if (s2 >= rc2) {
    f = ir3;
    F1 = -3.0 * ir3 * ir2;
    return;
  }
  if (s2 <= 0.01 * rc2) {
    f = 0.0;
    F1 = 0.0;
    return;
  }
  const double q = (r - 0.1 * rc) / (0.9 * rc);
  const double q2 = q * q;
  const double K = q2 * q * fma(q, fma(q, 6.0, -15.0), 10.0);
  const double Kp = 30.0 * q2 * (1.0 - q) * (1.0 - q) / (0.9 * rc);
  f = K * ir3;
  F1 = (Kp * ir3 - 3.0 * K * ir3 * ir) * ir;
}

// ------------------------------------------------------------------ kick
// Arguments of the massive-body step that follows a reduction: uref is the
// velocity the momentum is taken of, lx is touched by the kick only.
struct AdjApply {
  int n, nb;
  double coef;
  const double* mu;
  const double* uref;
  double* lx;
  double* lu;
  double* lmu;
};

// Partials per wave: [4 nb] source terms (3 position, 1 mass), [3] sum of the
// updated lx over the wave's bodies, [3] momentum term of the drag.
__host__ __device__ __forceinline__ int part_stride(int nb) { return 4 * nb + 6; }

// One half kick u' = u + hh (a(x) + ad(x, u + P/mu0)) taken back: g = lu (the
// adjoint of u'); x: positions of the kick; up: velocities before it.
__global__ __launch_bounds__(kBlock) void k_adj_kick(
    int n, int nb, double mu0, double hh, mxd::DragConst dc, int gas_on,
    const double* __restrict__ x, const double* __restrict__ up, const double* __restrict__ mu,
    const double* __restrict__ rcrit, const double* __restrict__ r_p,
    const double* __restrict__ rho_p, double* __restrict__ lx, double* __restrict__ lu,
    double* __restrict__ part) {
  __shared__ double bx[3][kSmallBig], bmu[kSmallBig], brc[kSmallBig];
  const int tid = threadIdx.x;
  double P[3] = {0.0, 0.0, 0.0};  // massive momentum: every wave sums it the same way
  if ((tid & 63) < nb) {
    const int k = tid & 63;
    P[0] = mu[k] * up[k];
    P[1] = mu[k] * up[n + k];
    P[2] = mu[k] * up[2 * n + k];
  }
  for (int c = 0; c < 3; ++c) P[c] = wave_sum(P[c]);
  if (tid < nb) {
    for (int c = 0; c < 3; ++c) bx[c][tid] = x[c * n + tid];
    bmu[tid] = mu[tid];
    brc[tid] = rcrit[tid];
  }
  __syncthreads();
  const int t = blockIdx.x * kBlock + tid;
  const bool live = t < n;
  const int lane = tid & 63;
  const int wave = t >> 6;
  const int S = part_stride(nb);
  double* pw = part + (size_t)wave * S;
  double g[3] = {0.0, 0.0, 0.0}, p[3] = {0.0, 0.0, 0.0};
  if (live)
    for (int c = 0; c < 3; ++c) {
      g[c] = lu[c * n + t];
      p[c] = x[c * n + t];
    }
  const double rct = live && t < nb ? brc[t] : 0.0;
  double tx[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < nb; ++s) {
    double vec[3] = {0.0, 0.0, 0.0}, fm = 0.0;
    if (live && s != t) {
      double d[3];
      for (int c = 0; c < 3; ++c) d[c] = bx[c][s] - p[c];
      const double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      double f, F1;
      pair_f(s2, fmax(brc[s], rct), f, F1);
      const double dg = d[0] * g[0] + d[1] * g[1] + d[2] * g[2];
      for (int c = 0; c < 3; ++c) vec[c] = hh * bmu[s] * (f * g[c] + F1 * dg * d[c]);
      fm = hh * f * dg;
      for (int c = 0; c < 3; ++c) tx[c] -= vec[c];
    }
    for (int c = 0; c < 3; ++c) vec[c] = wave_sum(vec[c]);
    fm = wave_sum(fm);
    if (lane == 0) {
      for (int c = 0; c < 3; ++c) pw[4 * s + c] = vec[c];
      pw[4 * s + 3] = fm;
    }
  }
  double lP[3] = {0.0, 0.0, 0.0};
  double lxn[3] = {0.0, 0.0, 0.0};
  if (live) {
    double lun[3] = {g[0], g[1], g[2]};
    for (int c = 0; c < 3; ++c) lxn[c] = lx[c * n + t] + tx[c];
    if (t >= nb && gas_on) {
      const int j = t - nb;
      double o[5];
      const double hg[3] = {hh * g[0], hh * g[1], hh * g[2]};
      drag_vjp(dc, p[0], p[1], up[t] + P[0] / mu0, up[n + t] + P[1] / mu0,
               up[2 * n + t] + P[2] / mu0, r_p[j], rho_p[j], hg, o);
      lxn[0] += o[0];
      lxn[1] += o[1];
      for (int c = 0; c < 3; ++c) {
        lun[c] += o[2 + c];
        lP[c] = o[2 + c] / mu0;
      }
    }
    for (int c = 0; c < 3; ++c) {
      lx[c * n + t] = lxn[c];
      lu[c * n + t] = lun[c];
    }
  }
  for (int c = 0; c < 3; ++c) {
    const double a = wave_sum(lxn[c]);
    const double b = wave_sum(lP[c]);
    if (lane == 0) {
      pw[4 * nb + c] = a;
      pw[4 * nb + 3 + c] = b;
    }
  }
}

// Fixed-order sum over the nw waves of value v of the wave partials (stride S):
// lane l adds waves l, l + 64, ... in order, then a fixed butterfly.
__global__ __launch_bounds__(64) void k_adj_reduce(const double* __restrict__ part, int nw, int S,
                                                   double* __restrict__ tot) {
  const int v = blockIdx.x;
  double a = 0.0;
  for (int w = threadIdx.x; w < nw; w += 64) a += part[(size_t)w * S + v];
  a = wave_sum(a);
  if (threadIdx.x == 0) tot[v] = a;
}
// The massive bodies' part of a kick taken back (tid < nb): the source terms
// tot[4 k + {0,1,2,3}], and the momentum of the jump before the kick (coef =
// hh / mu0, else 0) and of the drag, from the summed lx tot[4 nb + c] and drag
// term tot[4 nb + 3 + c].
__device__ __forceinline__ void kick_apply(int tid, const AdjApply& ap, const double* tot) {
  const int n = ap.n, nb = ap.nb;
  double lP[3];
  for (int c = 0; c < 3; ++c) {
    double sx = tot[4 * nb + c];
    for (int s = 0; s < nb; ++s) sx += tot[4 * s + c];
    lP[c] = ap.coef * sx + tot[4 * nb + 3 + c];
  }
  double dm = tot[4 * tid + 3];
  for (int c = 0; c < 3; ++c) {
    ap.lx[c * n + tid] += tot[4 * tid + c];
    ap.lu[c * n + tid] += ap.mu[tid] * lP[c];
    dm += ap.uref[c * n + tid] * lP[c];
  }
  ap.lmu[tid] += dm;
}

// lP = coef * sum_t a_t (tot[c]); lu_k += mu_k lP; lmu_k += uref_k . lP
__device__ __forceinline__ void momentum_apply(int tid, const AdjApply& ap, const double* tot) {
  const int n = ap.n;
  double dm = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double lP = ap.coef * tot[c];
    ap.lu[c * n + tid] += ap.mu[tid] * lP;
    dm += ap.uref[c * n + tid] * lP;
  }
  ap.lmu[tid] += dm;
}

// Block v sums column v of the per-wave partials into tot[v]; the block that
// finishes last (counted in *ctr, which it sets back to zero) applies the sums
// to the massive bodies.  Release and acquire fences at device scope order the
// sums before the count and the count before their reads.
template <bool kKick>
__global__ __launch_bounds__(64) void k_adj_reduce_apply(const double* __restrict__ part, int nw,
                                                         int S, double* __restrict__ tot,
                                                         unsigned* __restrict__ ctr, AdjApply ap) {
  __shared__ int last;
  __shared__ double sums[4 * kSmallBig + 6];
  const int v = blockIdx.x, tid = threadIdx.x;
  double a = 0.0;
  for (int w = tid; w < nw; w += 64) a += part[(size_t)w * S + v];
  a = wave_sum(a);
  if (tid == 0) {
    tot[v] = a;
    __threadfence();
    last = atomicAdd(ctr, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (tid == 0) *ctr = 0;
  for (int i = tid; i < S; i += 64) sums[i] = tot[i];  // all loads in flight at once
  __syncthreads();
  if (tid >= ap.nb) return;
  if (kKick) kick_apply(tid, ap, sums);
  else momentum_apply(tid, ap, sums);
}

// Kick totals applied: source terms to the massive bodies (lx, lmu); the
// momentum adjoint lP = jump_coef * (sum of the updated lx over all bodies) +
// (drag term) feeds lu and lmu of the massive bodies through P = sum mu_k up_k.
__global__ __launch_bounds__(kBlock) void k_adj_sum3(int n, const double* __restrict__ a,
                                                     double* __restrict__ part) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (t < n)
    for (int c = 0; c < 3; ++c) v[c] = a[c * n + t];
  for (int c = 0; c < 3; ++c) {
    const double s = wave_sum(v[c]);
    if ((threadIdx.x & 63) == 0) part[(size_t)(t >> 6) * 3 + c] = s;
  }
}

// lP = coef * tot[0..2]; lu_k += mu_k lP, lmu_k += uref_k . lP

// ------------------------------------------------------------------ drift
// (lx, lu) <- J_Kepler^T (lx, lu) at the pre-drift state for bodies that drifted;
// zero for the kept members of encounter subsystems (their part comes from the
// Bulirsch-Stoer tangents)
__global__ __launch_bounds__(kBlock) void k_adj_drift(int n, double mu0, double h,
                                                      const double* __restrict__ x0,
                                                      const double* __restrict__ u0,
                                                      const int32_t* __restrict__ kept,
                                                      double* __restrict__ lx,
                                                      double* __restrict__ lu,
                                                      int32_t* __restrict__ err) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  if (kept[t]) {
    for (int c = 0; c < 3; ++c) lx[c * n + t] = lu[c * n + t] = 0.0;
    return;
  }
  double xa[3], va[3], l1[3], m1[3], l0[3], m0[3];
  for (int c = 0; c < 3; ++c) {
    xa[c] = x0[c * n + t];
    va[c] = u0[c * n + t];
    l1[c] = lx[c * n + t];
    m1[c] = lu[c * n + t];
  }
  if (!kepler_vjp(mu0, h, xa, va, l1, m1, l0, m0)) {
    atomicOr(err, MXE_NOCONV);
    return;
  }
  for (int c = 0; c < 3; ++c) {
    lx[c * n + t] = l0[c];
    lu[c * n + t] = m0[c];
  }
}

// ------------------------------------------------------------------ BS
// Tangent Stoermer sequence of an M-member subsystem in one-direction dual
// arithmetic (the lane's input direction), the forward rule's operations.
typedef Dn<1> D1;

template <int M>
__device__ __forceinline__ void tforce(uint32_t pmask, const D1 (&mu)[M], const double (&rc)[M],
                                       double mu0, const D1 (&pos)[3 * M], D1 (&acc)[3 * M]) {
  // r^-3 and its derivative from y = 1/sqrt(r^2) (the corrected hardware
  // estimate): d(r^-3)/d(r^2) = -1.5 y^5, no division on the dual chain
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const D1 r2 = pos[3 * k] * pos[3 * k] + pos[3 * k + 1] * pos[3 * k + 1] +
                  pos[3 * k + 2] * pos[3 * k + 2];
    const double y = mxd::rsqrt_full(r2.v), y2 = y * y, y3 = y2 * y;
    D1 f;
    f.v = -mu0 * y3;
    f.d[0] = (1.5 * mu0) * (y3 * y2) * r2.d[0];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[3 * k + c] = f * pos[3 * k + c];
  }
  int bit = 0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
#pragma unroll
    for (int b = a + 1; b < M; ++b, ++bit) {
      if (!((pmask >> bit) & 1u)) continue;
      D1 d[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) d[c] = pos[3 * b + c] - pos[3 * a + c];
      const D1 s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const double rcp = fmax(rc[a], rc[b]);
      const double rc2 = rcp * rcp;
      D1 w = dconst<1>(0.0);
      if (s2.v < rc2 && s2.v > 0.0) {
        const double y = mxd::rsqrt_full(s2.v), y2 = y * y, y3 = y2 * y;
        w.v = y3;  // 1/s^3
        w.d[0] = -1.5 * (y3 * y2) * s2.d[0];
        if (s2.v > 0.01 * rc2) {
          D1 sd;  // s = s2 y, ds/ds2 = y/2
          sd.v = s2.v * y;
          sd.d[0] = 0.5 * y * s2.d[0];
          const D1 q = (sd - 0.1 * rcp) * (1.0 / (0.9 * rcp));
          const D1 K = q * q * q * (10.0 + q * (-15.0 + 6.0 * q));
          w = w * (1.0 - K);
        }
      }
      const D1 wa = mu[b] * w, wb = mu[a] * w;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[3 * a + c] = acc[3 * a + c] + wa * d[c];
        acc[3 * b + c] = acc[3 * b + c] - wb * d[c];
      }
    }
  }
}

template <int M>
__device__ __forceinline__ void tstoermer(int ns, double H, uint32_t pmask, const D1 (&mu)[M],
                          const double (&rc)[M], double mu0, const D1 (&xs)[3 * M],
                          const D1 (&vs)[3 * M], D1 (&xo)[3 * M], D1 (&vo)[3 * M]) {
  constexpr int NN = 3 * M;
  D1 acc[NN], d[NN];
  const double dt = H / ns;
#pragma unroll
  for (int i = 0; i < NN; ++i) xo[i] = xs[i];
  tforce<M>(pmask, mu, rc, mu0, xo, acc);
#pragma unroll
  for (int i = 0; i < NN; ++i) {
    d[i] = dt * (vs[i] + (0.5 * dt) * acc[i]);
    xo[i] = xo[i] + d[i];
  }
  for (int k = 1; k < ns; ++k) {
    tforce<M>(pmask, mu, rc, mu0, xo, acc);
#pragma unroll
    for (int i = 0; i < NN; ++i) {
      d[i] = d[i] + (dt * dt) * acc[i];
      xo[i] = xo[i] + d[i];
    }
  }
  tforce<M>(pmask, mu, rc, mu0, xo, acc);
#pragma unroll
  for (int i = 0; i < NN; ++i) vo[i] = d[i] / dt + (0.5 * dt) * acc[i];
}

// One block per subsystem: thread t carries input direction t % 32 (member
// positions 3M, velocities 3M, masses M; directions >= 7M idle along) and
// Stoermer column t / 32.  The state is advanced along the accepted steps of the
// forward run; the columns 0..a of one accepted step run side by side, their
// results meet in LDS, and the step's result is their polynomial extrapolation to
// zero step, the Lagrange combination sum_k w_k T_k with
// w_k = prod_{j != k} n_k^2/(n_k^2-n_j^2), summed in column order.
constexpr int kAdjBsDirs = 32;
constexpr int kAdjBsThreads = kAdjBsDirs * kBsColumns;

struct AdjBsShared {
  double cv[kBsColumns][24];              // each column's result, primal (x then v)
  double cd[kBsColumns][24][kAdjBsDirs];  // and its tangent per direction
  double sv[24];                          // state after the accepted step, primal
  double sd[24][kAdjBsDirs];              // and tangent per direction
  double xs[12], vs[12], mum[4], rcm[4], lxo[12], luo[12];
  double w[kBsColumns][kBsColumns];  // w[a][k]: weight of column k when column a is accepted
  double sched[2 * kBsMaxSched];     // the subsystem's accepted steps (H, a)
  uint32_t pmask;                    // pairs of members that interact
};

template <int M>
__device__ void bs_tangent_block(AdjBsShared& sh, const Subsystem& S, int nsched, double mu0,
                                 double* out) {
  constexpr int NN = 3 * M, NC = 6 * M;
  const int dir = threadIdx.x % kAdjBsDirs, col = threadIdx.x / kAdjBsDirs;
  D1 xs[NN], vs[NN], mu[M];
  double rc[M];
#pragma unroll
  for (int i = 0; i < NN; ++i) {
    xs[i] = dconst<1>(sh.xs[i]);
    vs[i] = dconst<1>(sh.vs[i]);
    if (dir == i) xs[i].d[0] = 1.0;
    if (dir == NN + i) vs[i].d[0] = 1.0;
  }
#pragma unroll
  for (int k = 0; k < M; ++k) {
    mu[k] = dconst<1>(sh.mum[k]);
    if (dir == 2 * NN + k) mu[k].d[0] = 1.0;
    rc[k] = sh.rcm[k];
  }
  const uint32_t pmask = sh.pmask;
  for (int j = 0; j < nsched; ++j) {
    const double H = sh.sched[2 * j];
    const int acc = min((int)sh.sched[2 * j + 1], kBsColumns - 1);  // columns the LDS holds
    if (col <= acc) {
      D1 xo[NN], vo[NN];
      tstoermer<M>(2 * (col + 1), H, pmask, mu, rc, mu0, xs, vs, xo, vo);
#pragma unroll
      for (int i = 0; i < NN; ++i) {
        sh.cd[col][i][dir] = xo[i].d[0];
        sh.cd[col][NN + i][dir] = vo[i].d[0];
      }
      if (dir == 0) {
#pragma unroll
        for (int i = 0; i < NN; ++i) {
          sh.cv[col][i] = xo[i].v;
          sh.cv[col][NN + i] = vo[i].v;
        }
      }
    }
    __syncthreads();
    for (int c = col; c < NC; c += kBsColumns) {
      D1 sum = dconst<1>(0.0);
      for (int k = 0; k <= acc; ++k) {
        D1 t;
        t.v = sh.cv[k][c];
        t.d[0] = sh.cd[k][c][dir];
        sum = sum + sh.w[acc][k] * t;
      }
      sh.sd[c][dir] = sum.d[0];
      if (dir == 0) sh.sv[c] = sum.v;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NN; ++i) {
      xs[i].v = sh.sv[i];
      xs[i].d[0] = sh.sd[i][dir];
      vs[i].v = sh.sv[NN + i];
      vs[i].d[0] = sh.sd[NN + i][dir];
    }
  }
  if (col != 0 || dir >= 7 * M) return;
  double acc = 0.0;
  const int keep_from = S.keep_from;
#pragma unroll
  for (int k = 0; k < M; ++k) {  // static indices keep the state in registers
    if (k < keep_from) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      acc += xs[3 * k + c].d[0] * sh.lxo[3 * k + c] + vs[3 * k + c].d[0] * sh.luo[3 * k + c];
  }
  out[dir] = acc;
}

// One block per subsystem: contributions contrib[b][i] = d(kept outputs)/d(input
// i) . adjoint of the kept outputs, i over positions, velocities, masses; the
// kept members are marked in kept[] for the drift kernel that follows.
__global__ __launch_bounds__(kAdjBsThreads) void k_adj_bs(int n, int nb, double mu0,
                                                          const double* __restrict__ x0s,
                                                          const double* __restrict__ u0s,
                                                          const double* __restrict__ mu,
                                                          const double* __restrict__ rcrit,
                                                          const Subsystem* __restrict__ subs,
                                                          const int32_t* __restrict__ n_sub,
                                                          const double* __restrict__ sched,
                                                          const int32_t* __restrict__ nsched,
                                                          const double* __restrict__ lx,
                                                          const double* __restrict__ lu,
                                                          double* __restrict__ contrib,
                                                          int32_t* __restrict__ kept,
                                                          int32_t* __restrict__ err) {
  __shared__ AdjBsShared sh;
  const int t = threadIdx.x;
  const int nsub = *n_sub;
  if (t < kBsColumns * kBsColumns) {  // Lagrange weights of column k among columns 0..a
    const int a = t / kBsColumns, k = t % kBsColumns;
    const double nk = 2.0 * (k + 1);
    double w = 1.0;
    for (int jj = 0; jj <= a; ++jj) {
      if (jj == k) continue;
      const double nj = 2.0 * (jj + 1);
      w *= nk * nk / (nk * nk - nj * nj);
    }
    sh.w[a][k] = w;
  }
  for (int b = blockIdx.x; b < nsub; b += gridDim.x) {
    const Subsystem& S = subs[b];
    const int m = S.m;
    if (t >= S.keep_from && t < m) kept[S.mem[t]] = 1;  // read by k_adj_drift
    if (m == 0) continue;
    if (m > 4 || nsched[b] > kBsMaxSched) {
      if (t == 0) atomicOr(err, MXE_ADJOINT);
      continue;
    }
    __syncthreads();
    if (t < 3 * m) {
      const int k = t / 3, c = t - 3 * (t / 3);
      const int body = S.mem[k];
      sh.xs[t] = x0s[(size_t)c * n + body];
      sh.vs[t] = u0s[(size_t)c * n + body];
      sh.lxo[t] = lx[(size_t)c * n + body];
      sh.luo[t] = lu[(size_t)c * n + body];
    }
    if (t < m) {
      const int body = S.mem[t];
      sh.mum[t] = body < nb ? mu[body] : 0.0;
      sh.rcm[t] = body < nb ? rcrit[body] : 0.0;
    }
    const int ns = nsched[b];
    if (t < 2 * ns) sh.sched[t] = sched[(size_t)b * kBsMaxSched * 2 + t];
    if (t == 0) sh.pmask = 0;
    __syncthreads();
    if (t < S.np) {  // bit of pair (a, b), a < b, in row-major order of the upper triangle
      const int a = S.pl[t][0], c = S.pl[t][1];
      atomicOr(&sh.pmask, 1u << (a * (2 * m - a - 1) / 2 + (c - a - 1)));
    }
    __syncthreads();
    double* out = contrib + (size_t)b * 28;
    switch (m) {
      case 1:
        if (t < 7) out[t] = 0.0;  // cannot occur: subsystems have two or more members
        break;
      case 2: bs_tangent_block<2>(sh, S, ns, mu0, out); break;
      case 3: bs_tangent_block<3>(sh, S, ns, mu0, out); break;
      default: bs_tangent_block<4>(sh, S, ns, mu0, out); break;
    }
  }
}

// Adds the subsystem contributions.  Massive body k < nb gets wave k: lane l
// sums subsystems l, l + 64, ... in order and the 64 partials meet in a fixed
// tree, so the sum is the same on every run.  The remaining threads take the
// massless members, each of which belongs to one subsystem only, and clear the
// marks k_adj_bs set.
constexpr int kAdjApplyMassless = 1024;  // threads beyond the massive bodies' waves

__global__ __launch_bounds__(256) void k_adj_bs_apply(int n, int nb,
                                                      const Subsystem* __restrict__ subs,
                                                      const int32_t* __restrict__ n_sub,
                                                      const double* __restrict__ contrib,
                                                      double* __restrict__ lx,
                                                      double* __restrict__ lu,
                                                      double* __restrict__ lmu,
                                                      int32_t* __restrict__ kept) {
  const int nsub = *n_sub;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  if (wave < nb) {
    double a[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = lane; b < nsub; b += 64) {
      const Subsystem& S = subs[b];
      const int m = S.m;
      if (m < 2 || m > 4) continue;
      const double* c = contrib + (size_t)b * 28;
      for (int k = 0; k < m; ++k) {
        if (S.mem[k] != wave) continue;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          a[q] += c[3 * k + q];
          a[3 + q] += c[3 * m + 3 * k + q];
        }
        a[6] += c[6 * m + k];
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int i = 0; i < 7; ++i) a[i] += __shfl_down(a[i], off);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        lx[q * n + wave] += a[q];
        lu[q * n + wave] += a[3 + q];
      }
      lmu[wave] += a[6];
    }
    return;
  }
  const int stride = gridDim.x * blockDim.x - 64 * nb;
  for (int b = tid - 64 * nb; b < nsub; b += stride) {
    const Subsystem& S = subs[b];
    const int m = S.m;
    for (int k = S.keep_from; k < m; ++k) kept[S.mem[k]] = 0;
    if (m < 2 || m > 4) continue;
    const double* c = contrib + (size_t)b * 28;
    for (int k = 0; k < m; ++k) {
      const int body = S.mem[k];
      if (body < nb) continue;
      for (int q = 0; q < 3; ++q) {
        lx[q * n + body] += c[3 * k + q];
        lu[q * n + body] += c[3 * m + 3 * k + q];
      }
    }
  }
}

// ------------------------------------------------------------------ init
// Heliocentric -> DH at start-up taken back: u = v - V, V = sum m v / (m0 + M)
// over the massive bodies.  lu_sum (device [3]) is the sum of lu over all
// bodies; gm[k] = dL/dm_k = G lmu_k + the mass term of V; gv = lu + the V term.
__global__ __launch_bounds__(64) void k_adj_h2dh(int n, int nb, double G, double m0,
                                                 const double* __restrict__ tot,
                                                 const double* __restrict__ m_big,
                                                 const double* __restrict__ v_h,
                                                 const double* __restrict__ lmu,
                                                 double* __restrict__ gm,
                                                 double* __restrict__ gv) {
  __shared__ double lV[3], Vc[3], Mt;
  const int tid = threadIdx.x;
  if (tid == 0) {
    double M = m0;
    for (int k = 0; k < nb; ++k) M += m_big[k];
    Mt = M;
    for (int c = 0; c < 3; ++c) {
      double pv = 0.0;
      for (int k = 0; k < nb; ++k) pv += m_big[k] * v_h[c * n + k];
      lV[c] = -tot[c];
      Vc[c] = pv / M;
    }
  }
  __syncthreads();
  if (tid < nb) {
    double dm = G * lmu[tid];
    for (int c = 0; c < 3; ++c) {
      gv[c * n + tid] += m_big[tid] / Mt * lV[c];
      dm += (v_h[c * n + tid] - Vc[c]) * lV[c] / Mt;
    }
    gm[tid] = dm;
  }
}

// Copies of the step state in one launch: up to four arrays of given lengths
// packed one after another in dst (or unpacked from src when unpack != 0).
struct CopyList {
  double* ptr[4];
  int64_t len[4];
};

__global__ __launch_bounds__(kBlock) void k_adj_copy(CopyList l, double* __restrict__ packed,
                                                     int unpack) {
  int64_t off = 0;
  for (int a = 0; a < 4; ++a) {
    const int64_t m = l.len[a];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
      if (unpack) l.ptr[a][i] = packed[off + i];
      else packed[off + i] = l.ptr[a][i];
    }
    off += m;
  }
}

// One step's record in one launch.  Blocks below ncopy pack the arrays of l
// (the pre-drift state and the velocities after the drift) into `packed`; the
// other blocks copy the subsystem table of the step (its n_sub entries), n_sub,
// and the accepted Bulirsch-Stoer steps of those subsystems.
constexpr int kTapeBlocks = 64;

__global__ __launch_bounds__(kBlock) void k_adj_record(
    CopyList l, double* __restrict__ packed, int ncopy, const Subsystem* __restrict__ subs,
    const DevScalars* __restrict__ dsc, const double* __restrict__ sched,
    const int32_t* __restrict__ nsched, Subsystem* __restrict__ dsubs,
    int32_t* __restrict__ n_sub_out, double* __restrict__ dsched, int32_t* __restrict__ dnsched) {
  if ((int)blockIdx.x < ncopy) {
    int64_t off = 0;
    for (int a = 0; a < 4; ++a) {
      const int64_t m = l.len[a];
      for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
           i += (int64_t)ncopy * kBlock)
        packed[off + i] = l.ptr[a][i];
      off += m;
    }
    return;
  }
  const int nsub = dsc->n_sub;
  const int words = (int)(sizeof(Subsystem) / 4);
  const int32_t* src = reinterpret_cast<const int32_t*>(subs);
  int32_t* out = reinterpret_cast<int32_t*>(dsubs);
  const int64_t stride = (int64_t)(gridDim.x - ncopy) * kBlock;
  const int64_t i0 = (int64_t)(blockIdx.x - ncopy) * kBlock + threadIdx.x;
  for (int64_t i = i0; i < (int64_t)nsub * words; i += stride) out[i] = src[i];
  for (int64_t i = i0; i < (int64_t)nsub * kBsMaxSched * 2; i += stride) dsched[i] = sched[i];
  for (int64_t i = i0; i < nsub; i += stride) dnsched[i] = nsched[i];
  if (i0 == 0) *n_sub_out = nsub;
}

int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }

}  // namespace

namespace mxk {

// tot holds the part_stride(kSmallBig) sums, then one word that counts the
// blocks of a reduction (zero between launches)
unsigned* tot_counter(double* tot) {
  return reinterpret_cast<unsigned*>(tot + part_stride(kSmallBig));
}

hipError_t adj_reduce(hipStream_t st, const double* part, int nw, int S, double* tot) {
  hipLaunchKernelGGL(k_adj_reduce, dim3(S), dim3(64), 0, st, part, nw, S, tot);
  return hipGetLastError();
}

// adjoint of the closing (jump_coef = hh / mu0: with the jump before it) or
// opening (0) half kick of a step
hipError_t adj_kick(hipStream_t st, int n, int nb, double mu0, double hh,
                    const mxd::DragConst& dc, int gas_on, const double* x, const double* up,
                    const double* mu, const double* rcrit, const double* r_p,
                    const double* rho_p, double* lx, double* lu, double* lmu, double* part,
                    double* tot, double jump_coef) {
  if (nb > kSmallBig) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_adj_kick, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, nb, mu0, hh, dc,
                     gas_on, x, up, mu, rcrit, r_p, rho_p, lx, lu, part);
  const AdjApply ap{n, nb, jump_coef, mu, up, lx, lu, lmu};
  hipLaunchKernelGGL(k_adj_reduce_apply<true>, dim3(part_stride(nb)), dim3(64), 0, st, part,
                     (n + 63) / 64, part_stride(nb), tot, tot_counter(tot), ap);
  return hipGetLastError();
}

// lP = coef * sum_t a_t; lu_k += mu_k lP; lmu_k += uref_k . lP
hipError_t adj_momentum(hipStream_t st, int n, int nb, const double* a, double coef,
                        const double* mu, const double* uref, double* lu, double* lmu,
                        double* part, double* tot) {
  hipLaunchKernelGGL(k_adj_sum3, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, a, part);
  const AdjApply ap{n, nb, coef, mu, uref, nullptr, lu, lmu};
  hipLaunchKernelGGL(k_adj_reduce_apply<false>, dim3(3), dim3(64), 0, st, part, (n + 63) / 64, 3,
                     tot, tot_counter(tot), ap);
  return hipGetLastError();
}

// adjoint of the drift and encounter integration of a step (tape: pre-drift
// state x0, u0, the step's subsystem table and count, the accepted BS steps)
hipError_t adj_drift(hipStream_t st, int n, int nb, double mu0, double h, const double* x0,
                     const double* u0, const double* mu, const double* rcrit,
                     const Subsystem* subs, const int32_t* n_sub, const double* sched,
                     const int32_t* nsched, int32_t* kept, double* contrib, double* lx,
                     double* lu, double* lmu, int32_t* err) {
  hipLaunchKernelGGL(k_adj_bs, dim3(256), dim3(kAdjBsThreads), 0, st, n, nb, mu0, x0, u0, mu,
                     rcrit, subs, n_sub, sched, nsched, lx, lu, contrib, kept, err);
  hipLaunchKernelGGL(k_adj_drift, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, mu0, h, x0, u0,
                     kept, lx, lu, err);
  const int apply_blocks = (64 * nb + kAdjApplyMassless + 255) / 256;
  hipLaunchKernelGGL(k_adj_bs_apply, dim3(apply_blocks), dim3(256), 0, st, n, nb, subs, n_sub,
                     contrib, lx, lu, lmu, kept);
  return hipGetLastError();
}

// gradients with respect to the heliocentric start state and masses from the
// adjoint of the DH start state: gx = lx, gv = lu + V term, gm
hipError_t adj_h2dh(hipStream_t st, int n, int nb, double G, double m0, const double* m_big,
                    const double* v_h, const double* lu, const double* lmu, double* gm,
                    double* gv, double* part, double* tot) {
  hipLaunchKernelGGL(k_adj_sum3, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, lu, part);
  hipError_t e = adj_reduce(st, part, (n + 63) / 64, 3, tot);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(gv, lu, sizeof(double) * 3 * (size_t)n, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adj_h2dh, dim3(1), dim3(64), 0, st, n, nb, G, m0, tot, m_big, v_h, lmu,
                     gm, gv);
  return hipGetLastError();
}

// pack (unpack != 0: unpack) up to four arrays into / from one buffer
hipError_t adj_copy(hipStream_t st, double* const* ptr, const int64_t* len, int count,
                    double* packed, int unpack) {
  CopyList l;
  int64_t tot = 0;
  for (int a = 0; a < 4; ++a) {
    l.ptr[a] = a < count ? ptr[a] : nullptr;
    l.len[a] = a < count ? len[a] : 0;
    tot += l.len[a];
  }
  int64_t blocks = (tot / 4 + kBlock - 1) / kBlock;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_adj_copy, dim3((unsigned)blocks), dim3(kBlock), 0, st, l, packed, unpack);
  return hipGetLastError();
}

hipError_t adj_record(hipStream_t st, double* const* ptr, const int64_t* len, int count,
                      double* packed, const Subsystem* subs, const DevScalars* dsc,
                      const double* sched, const int32_t* nsched, Subsystem* dsubs,
                      int32_t* n_sub_out, double* dsched, int32_t* dnsched) {
  CopyList l;
  int64_t tot = 0;
  for (int a = 0; a < 4; ++a) {
    l.ptr[a] = a < count ? ptr[a] : nullptr;
    l.len[a] = a < count ? len[a] : 0;
    tot += l.len[a];
  }
  int64_t ncopy = (tot / 4 + kBlock - 1) / kBlock;
  if (ncopy < 1) ncopy = 1;
  if (ncopy > 4096) ncopy = 4096;
  hipLaunchKernelGGL(k_adj_record, dim3((unsigned)ncopy + kTapeBlocks), dim3(kBlock), 0, st, l,
                     packed, (int)ncopy, subs, dsc, sched, nsched, dsubs, n_sub_out, dsched,
                     dnsched);
  return hipGetLastError();
}

}  // namespace mxk
