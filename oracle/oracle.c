/*
 * CPU oracle of the hybrid symplectic step -- TEST INFRASTRUCTURE ONLY.
 *
 * Written from the paper (Mercury-Arxes: Sect. 2 "Mercury+, the n-body engine",
 * Sect. 3.1 "Protoplanetary disks and dynamical effects of gas", Sect. 3.2
 * "Growth of the forming planets", Sect. 3.4 "Planetesimal disk"), and from
 * textbook celestial mechanics where the paper defers to its references.
 * Every loop is written in the plain order of the definition; double precision
 * throughout.  Only tests, the smoke check and the benchmark's CPU-baseline leg
 * may use this file.  It shares nothing with the HIP library.
 *
 * Readings of the paper that this file fixes (the paper is silent on them):
 *  - sub-step order of the hybrid step: kick(h/2) jump(h/2) drift(h)+encounters
 *    jump(h/2) kick(h/2), the order of the democratic-heliocentric split that the
 *    paper's integrator inherits from Mercury 6;
 *  - gas drag is evaluated at the current state immediately before each half kick;
 *  - the Kepler drift uses mu0 = G*m0 for every body (the DH Kepler term);
 *  - the minimum pair separation inside a step comes from the cubic Hermite
 *    interpolant of the relative position (see or_pair_dmin2);
 *  - Bulirsch-Stoer subsystems: connected big-body components, and each flagged
 *    small body together with copies of the big components it touches.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

struct or_sys {
  or_params p;
  int n, nb, ns;
  double mu0;
  double *x, *u, *ag;               /* [3][n] state and FSAL gravity */
  double *mu, *mu_init;             /* [nb] */
  double *rcrit, *rcrit_init;       /* [nb] */
  double *r_p, *rho_p;              /* [ns]; rho_p in Msun/AU^3 */
  double *growth;                   /* [nb][3] (G*M0, G*Mc, tau_c) or NULL */
  long step;
  int32_t* pairs;
  int npairs, cap_pairs;
  double *x0, *u0, *x1, *u1, *ad;   /* scratch [3][n] */
  double *x1k, *u1k;                /* last step's post-drift state before BS [3][n] */
  /* time-dependent physics (or_set_physics) */
  or_planet* phys;                  /* [nb] or NULL */
  double *radius, *rad_c;           /* [nb] planet radius; radius at the start of the runaway */
  double* gaps;                     /* [nb][3] gap centre R, half width, density factor; */
  int* gap_on;                      /* [nb] 1 while the gap is open */
  double time, h;                   /* time at the start of the next step; current step */
  double a_switch, a_min;           /* step switch (a_switch <= 0: none) */
  int switched;
  /* body removal: status (0 alive, -2 central-body encounter, -3 ejected), radial
   * direction at the previous check (-1 inward, +1 outward, 0 none yet) */
  int32_t* stat;
  int8_t* rsign;
};

/* ------------------------------------------------------------------ */
/* Changeover function of the direct-force routine (Sect. 2.1.3, the
 * mfo_drct listing): K = 1 for s >= rc, 0 for s^2 <= 0.01 rc^2, else the
 * quintic 10q^3 - 15q^4 + 6q^5 with q = (s - 0.1 rc)/(0.9 rc).            */
static double kfun(double s2, double rc) {
  double rc2 = rc * rc;
  if (s2 >= rc2) return 1.0;
  if (s2 <= 0.01 * rc2) return 0.0;
  double s = sqrt(s2);
  double q = (s - 0.1 * rc) / (0.9 * rc);
  double q2 = q * q, q3 = q * q2, q4 = q2 * q2, q5 = q2 * q3;
  return 10.0 * q3 - 15.0 * q4 + 6.0 * q5;
}

double or_changeover(double s, double rc) { return kfun(s * s, rc); }

/* Weight w such that the pair acceleration is mu_s * w * (x_s - x_t):
 * K(s)/s^3 with the three branches of the listing.                      */
static double pair_weight(double s2, double rc) {
  double rc2 = rc * rc;
  if (s2 >= rc2) {
    double si = 1.0 / sqrt(s2);
    return si * si * si;
  }
  if (s2 <= 0.01 * rc2) return 0.0;
  double s = sqrt(s2);
  double si = 1.0 / s;
  double q = (s - 0.1 * rc) / (0.9 * rc);
  double q2 = q * q, q3 = q * q2, q4 = q2 * q2, q5 = q2 * q3;
  return (10.0 * q3 - 15.0 * q4 + 6.0 * q5) * si * si * si;
}

/* Rectangular changeover-weighted gravity (the parallel branch of the
 * mfo_drct listing): every target t against every massive source s != t,
 * rc = max(rcrit_s, rcrit_t), sources summed in ascending order.          */
void or_gravity(int n, int nb, const double* x, const double* mu, const double* rcrit,
                double* a) {
#pragma omp parallel for schedule(static)
  for (int t = 0; t < n; ++t) {
    double rct = t < nb ? rcrit[t] : 0.0;
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int s = 0; s < nb; ++s) {
      if (s == t) continue;
      double dx = x[s] - x[t];
      double dy = x[n + s] - x[n + t];
      double dz = x[2 * n + s] - x[2 * n + t];
      double s2 = dx * dx + dy * dy + dz * dz;
      double rc = rcrit[s] > rct ? rcrit[s] : rct;
      double w = mu[s] * pair_weight(s2, rc);
      ax += w * dx;
      ay += w * dy;
      az += w * dz;
    }
    a[t] = ax;
    a[n + t] = ay;
    a[2 * n + t] = az;
  }
}

/* ------------------------------------------------------------------ */
/* Drag coefficient, Eq. 7 (Tanigawa et al. form): the first bracket is
 * raised to the exponent kexp (printed as -2); k = 0.4 for Re < 1e5 and 0.2
 * otherwise.                                                              */
double or_drag_cd(double re, double ma, double kexp) {
  double k = re < 1.0e5 ? 0.4 : 0.2;
  double inner = 1.0 / (24.0 / re + 40.0 / (10.0 + re)) + 0.23 * ma;
  return pow(inner, kexp) + 2.0 * (0.8 * k + ma) / (1.6 + ma);
}

/* Gas surface density of Eq. 1 (Sect. 3.1) in g cm^-2 at cylindrical radius R
 * [AU]: Sigma0 (R/R_C)^-gamma exp[-(R/R_C)^(2-gamma)], with Sigma0 chosen so
 * that Sigma(1 AU) = sigma1 (the configuration gives the density at 1 AU);
 * without a taper radius (r_c = 0) the exponential is dropped.  Zero inward
 * of the inner edge r_in.                                                  */
double or_gas_sigma(const or_params* p, double R) {
  if (!(R > 0.0) || R < p->r_in) return 0.0;
  double sig = p->sigma1 * pow(R, -p->gamma);
  if (p->r_c > 0.0) {
    double at1 = pow(1.0 / p->r_c, 2.0 - p->gamma);
    double atR = pow(R / p->r_c, 2.0 - p->gamma);
    sig *= exp(at1 - atR);
  }
  return sig;
}

/* Disk gravity, leading term of the axisymmetric thin-disk treatment (Sect. 3.1,
 * Eqs. 10-12).  For gamma != 1 the radial force is 2 pi G Sigma(R) S(gamma) with
 *   S(gamma) = sum_{n>=0} A_n (1-gamma)(4n+1) / ((2n+2-gamma)(2n-1+gamma)),
 *   A_n = [(2n)! / (2^{2n} (n!)^2)]^2   (Eq. 10);
 * for gamma = 1 the leading term of the inner-edge series, 2 pi G Sigma(R) R_in/R
 * (Eqs. 11-12).  The series is summed term by term for n < 2^20 (A_n from
 * A_{n-1} by the factor ((2n-1)/(2n))^2) and the rest is added from the large-n
 * form of its terms, (1-gamma)/(pi n^2) (1 - 1/(2n) + O(n^-2)), whose sum from N
 * on is (1-gamma)/pi (1/N + 1/(4N^2)) + O(N^-3).                            */
double or_dg_series(double gamma) {
  const long N = 1L << 20;
  double A = 1.0, sum = 0.0;
  for (long n = 0; n < N; ++n) {
    if (n > 0) {
      double r = (2.0 * n - 1.0) / (2.0 * n);
      A *= r * r;
    }
    double t = A * (1.0 - gamma) * (4.0 * n + 1.0) /
               ((2.0 * n + 2.0 - gamma) * (2.0 * n - 1.0 + gamma));
    sum += t;
  }
  double Nd = (double)N;
  return sum + (1.0 - gamma) / PI * (1.0 / Nd + 1.0 / (4.0 * Nd * Nd));
}

/* The printed F_DG read as the signed cylindrical-radial acceleration, positive
 * away from the star, in AU day^-2 for Sigma of Eq. 1 (zero inside r_in): the
 * gamma -> 1 limit of the Eq. 10 series is -1, the inward pull 2 pi G Sigma of
 * an infinite disk with Sigma ~ 1/R, which fixes the sign.                  */
static double dg_cached_gamma = -1e300, dg_cached_S = 0.0;

static double dg_series_cached(double gamma) {
  if (gamma != dg_cached_gamma) {
    dg_cached_S = or_dg_series(gamma);
    dg_cached_gamma = gamma;
  }
  return dg_cached_S;
}

double or_disk_gravity(const or_params* p, double R) {
  double sig = or_gas_sigma(p, R) * (p->rho_unit / p->au_cm); /* Msun/AU^2 */
  if (!(sig > 0.0)) return 0.0;
  double f = 2.0 * PI * p->G * sig;
  if (p->gamma == 1.0) return f * p->r_in / R;
  return f * dg_series_cached(p->gamma);
}

/* Gas acceleration of the massless bodies (Sect. 3.1, Eqs. 1-7 and 10-12),
 * applied to bodies nbig+1..nbod only: the drag of Eq. 3, plus the disk gravity
 * when dg_mode is set.  Midplane density at every height; the velocity relative
 * to the gas uses the heliocentric velocity u + P/mu0.  The sound speed is
 * h_over_r v_K, or with a temperature profile sqrt(cs2_per_k T(R)) (Eq. 2); the
 * scale height is c_s/Omega; eta is fixed or from Eq. 6 with gamma_C = 7/5.    */

void or_drag(const or_params* p, int n, int nb, const double* x, const double* u,
             const double* mu, const double* r_p, const double* rho_p, double* a) {
  or_drag_gaps(p, n, nb, x, u, mu, r_p, rho_p, NULL, NULL, a);
}

/* gaps, gap_on: the open gaps of the massive bodies (or NULL).  A massless body
 * at cylindrical R strictly inside (R_gap - w, R_gap + w) of an open gap sees the
 * gas density times that gap's factor, the gap of the highest index winning (the
 * dens_factor loop of Sect. 3.1.1); the factor multiplies the midplane density of
 * the drag only.                                                               */
void or_drag_gaps(const or_params* p, int n, int nb, const double* x, const double* u,
                  const double* mu, const double* r_p, const double* rho_p, const double* gaps,
                  const int* gap_on, double* a) {
  double mu0 = p->G * p->m0;
  double px = 0, py = 0, pz = 0;
  for (int k = 0; k < nb; ++k) {
    px += mu[k] * u[k];
    py += mu[k] * u[n + k];
    pz += mu[k] * u[2 * n + k];
  }
  double sx = px / mu0, sy = py / mu0, sz = pz / mu0;
  double sigma_unit = p->rho_unit / p->au_cm; /* Msun/AU^2 per g/cm^2 */
  if (p->dg_mode && p->gas_on && p->gamma != 1.0) dg_series_cached(p->gamma);
#pragma omp parallel for schedule(static)
  for (int t = 0; t < n; ++t) {
    a[t] = a[n + t] = a[2 * n + t] = 0.0;
    if (t < nb || !p->gas_on) continue;
    int j = t - nb;
    double X = x[t], Y = x[n + t];
    double R = sqrt(X * X + Y * Y);
    if (!(R > 0.0) || R < p->r_in) continue;
    double sig = or_gas_sigma(p, R) * sigma_unit;
    if (!(sig > 0.0)) continue;
    if (p->dg_mode) {
      double g = or_disk_gravity(p, R);
      a[t] += g * X / R;
      a[n + t] += g * Y / R;
    }
    double vk = sqrt(mu0 / R);
    double om = vk / R;
    double cs;
    if (p->temp_1au > 0.0)
      cs = sqrt(p->cs2_per_k * p->temp_1au * pow(R, -p->temp_beta));
    else
      cs = p->h_over_r * vk;
    double hg = cs / om;
    double eta = p->eta;
    if (p->eta_mode)
      eta = (p->gamma + 0.5 * p->temp_beta + 1.5) / (2.0 * 1.4) * (cs / vk) * (cs / vk);
    double rhog = sig / (sqrt(2.0 * PI) * hg);
    if (gaps) {
      for (int i = 0; i < nb; ++i)
        if (gap_on[i] && R < gaps[3 * i] + gaps[3 * i + 1] && R > gaps[3 * i] - gaps[3 * i + 1])
          rhog = sig / (sqrt(2.0 * PI) * hg) * gaps[3 * i + 2];
    }
    double vg = vk * sqrt(1.0 - 2.0 * eta);
    double gx = -vg * Y / R, gy = vg * X / R;
    double dvx = u[t] + sx - gx;
    double dvy = u[n + t] + sy - gy;
    double dvz = u[2 * n + t] + sz;
    double dv = sqrt(dvx * dvx + dvy * dvy + dvz * dvz);
    if (!(dv > 0.0)) continue;
    double ma = dv / cs;
    double lam = p->mfp_coef / rhog;
    double nu = (1.0 / 3.0) * sqrt(8.0 / PI) * cs * lam;
    double re = 2.0 * r_p[j] * dv / nu;
    double cd = or_drag_cd(re, ma, p->kdrag_exp);
    double f = -(3.0 / 8.0) * (cd / r_p[j]) * (rhog / rho_p[j]) * dv;
    a[t] += f * dvx;
    a[n + t] += f * dvy;
    a[2 * n + t] += f * dvz;
  }
}

/* ------------------------------------------------------------------ */
/* Kepler drift.  The paper's code hands the drift to a Kepler solver; this
 * oracle uses the textbook difference forms of Kepler's equation in the
 * eccentric (elliptic) and hyperbolic anomaly, with a Newton iteration kept
 * inside a bisection bracket, and the universal variable only for orbits
 * within |alpha r0| <= 1e-6 of parabolic.  The Lagrange f, g functions carry
 * the state over the interval h.                                           */

static double x_minus_sin(double x) {
  if (fabs(x) < 0.5) {
    double x2 = x * x, term = x * x2 / 6.0, sum = 0.0;
    for (int k = 1; k < 40 && fabs(term) > 1e-40; ++k) {
      sum += term;
      term *= -x2 / ((2.0 * k + 2.0) * (2.0 * k + 3.0));
    }
    return sum;
  }
  return x - sin(x);
}

static double sinh_minus_x(double x) {
  if (fabs(x) < 0.5) {
    double x2 = x * x, term = x * x2 / 6.0, sum = 0.0;
    for (int k = 1; k < 40 && fabs(term) > 1e-40; ++k) {
      sum += term;
      term *= x2 / ((2.0 * k + 2.0) * (2.0 * k + 3.0));
    }
    return sum;
  }
  return sinh(x) - x;
}

/* Stumpff functions c0..c3 by their defining series (small |z|) or closed form. */
static void stumpff(double z, double c[4]) {
  if (fabs(z) < 0.5) {
    for (int k = 0; k < 4; ++k) {
      double fact = 1.0;
      for (int m = 2; m <= k; ++m) fact *= m;
      double term = 1.0 / fact, sum = 0.0;
      for (int j = 0; j < 60; ++j) {
        sum += term;
        term *= -z / ((2.0 * j + k + 1.0) * (2.0 * j + k + 2.0));
        if (fabs(term) < 1e-40) break;
      }
      c[k] = sum;
    }
  } else if (z > 0) {
    double sz = sqrt(z);
    c[0] = cos(sz);
    c[1] = sin(sz) / sz;
    c[2] = 2.0 * sin(0.5 * sz) * sin(0.5 * sz) / z;
    c[3] = x_minus_sin(sz) / (z * sz);
  } else {
    double sz = sqrt(-z);
    c[0] = cosh(sz);
    c[1] = sinh(sz) / sz;
    c[2] = -2.0 * sinh(0.5 * sz) * sinh(0.5 * sz) / z;
    c[3] = sinh_minus_x(sz) / (-z * sz);
  }
}

static int converged(double dx, double x) {
  return fabs(dx) <= 4.0 * 2.220446049250313e-16 * fabs(x) || fabs(dx) < 1e-300;
}

int or_drift(double mu, const double x0[3], const double v0[3], double h, double x1[3],
             double v1[3]) {
  double r0 = sqrt(x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2]);
  double vv = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
  double sig = x0[0] * v0[0] + x0[1] * v0[1] + x0[2] * v0[2];
  double alpha = 2.0 / r0 - vv / mu;
  double f, g, fd, gd;
  if (h == 0.0) {
    for (int c = 0; c < 3; ++c) { x1[c] = x0[c]; v1[c] = v0[c]; }
    return OR_OK;
  }
  if (alpha * r0 > 1e-6) {
    /* elliptic: solve dM = dE - c sin dE + s (1 - cos dE) */
    double a = 1.0 / alpha;
    double n = sqrt(mu * alpha * alpha * alpha);
    double c = 1.0 - r0 * alpha;
    double s = sig * sqrt(alpha / mu);
    double dm = n * h;
    double lo = dm - 2.0, hi = dm + 2.0, E = dm;
    int it, ok = 0;
    for (it = 0; it < 100; ++it) {
      double F = E - c * sin(E) + s * (1.0 - cos(E)) - dm;
      double Fp = 1.0 - c * cos(E) + s * sin(E);
      if (F == 0.0) { ok = 1; break; }
      if (F < 0) lo = E; else hi = E;
      double En = E - F / Fp;
      if (converged(En - E, En)) { E = En; ok = 1; break; }
      if (!(En > lo && En < hi)) En = 0.5 * (lo + hi);
      double d = En - E;
      E = En;
      if (converged(d, E)) { ok = 1; break; }
    }
    if (!ok) return OR_ENOCONV;
    double sE = sin(E);
    double omc = 2.0 * sin(0.5 * E) * sin(0.5 * E); /* 1 - cos E */
    double r = a * (1.0 - c * cos(E) + s * sE);
    f = 1.0 - (a / r0) * omc;
    g = h - x_minus_sin(E) / n;
    fd = -sqrt(mu * a) * sE / (r * r0);
    gd = 1.0 - (a / r) * omc;
  } else if (alpha * r0 < -1e-6) {
    /* hyperbolic: solve dN = c sinh dH + s (cosh dH - 1) - dH */
    double a = 1.0 / alpha; /* negative */
    double n = sqrt(-mu * alpha * alpha * alpha);
    double c = 1.0 - r0 * alpha;
    double s = sig * sqrt(-alpha / mu);
    double dn = n * h;
#define HF(x) (c * sinh(x) + s * (cosh(x) - 1.0) - (x) - dn)
    double lo, hi;
    if (dn >= 0) {
      lo = 0.0; hi = 1.0;
      while (HF(hi) < 0) { lo = hi; hi *= 2.0; if (hi > 1e4) return OR_ENOCONV; }
    } else {
      hi = 0.0; lo = -1.0;
      while (HF(lo) > 0) { hi = lo; lo *= 2.0; if (lo < -1e4) return OR_ENOCONV; }
    }
    double H = 0.5 * (lo + hi);
    int it, ok = 0;
    for (it = 0; it < 100; ++it) {
      double F = HF(H);
      double Fp = c * cosh(H) + s * sinh(H) - 1.0;
      if (F == 0.0) { ok = 1; break; }
      if (F < 0) lo = H; else hi = H;
      double Hn = H - F / Fp;
      if (converged(Hn - H, Hn)) { H = Hn; ok = 1; break; }
      if (!(Hn > lo && Hn < hi)) Hn = 0.5 * (lo + hi);
      double d = Hn - H;
      H = Hn;
      if (converged(d, H)) { ok = 1; break; }
    }
#undef HF
    if (!ok) return OR_ENOCONV;
    double shH = sinh(H);
    double chm1 = 2.0 * sinh(0.5 * H) * sinh(0.5 * H); /* cosh H - 1 */
    double r = a * (1.0 - c * cosh(H) - s * shH);
    f = 1.0 + (a / r0) * chm1;
    g = h - sinh_minus_x(H) / n;
    fd = -sqrt(-mu * a) * shH / (r * r0);
    gd = 1.0 + (a / r) * chm1;
  } else {
    /* near-parabolic: universal variable s, h = r0 G1 + sig G2 + mu G3 */
    double beta = mu * alpha;
    double cc[4];
#define UF(S, out, rr)                                                       \
  do {                                                                       \
    double _s = (S);                                                         \
    stumpff(beta * _s * _s, cc);                                             \
    double G1 = _s * cc[1], G2 = _s * _s * cc[2], G3 = _s * _s * _s * cc[3]; \
    (out) = r0 * G1 + sig * G2 + mu * G3 - h;                                \
    (rr) = r0 * cc[0] + sig * G1 + mu * G2;                                  \
  } while (0)
    double lo, hi, F, rr;
    if (h >= 0) {
      lo = 0.0; hi = h / r0;
      UF(hi, F, rr);
      while (F < 0) { lo = hi; hi *= 2.0; UF(hi, F, rr); if (hi > 1e12) return OR_ENOCONV; }
    } else {
      hi = 0.0; lo = h / r0;
      UF(lo, F, rr);
      while (F > 0) { hi = lo; lo *= 2.0; UF(lo, F, rr); if (lo < -1e12) return OR_ENOCONV; }
    }
    double S = 0.5 * (lo + hi);
    int ok = 0;
    for (int it = 0; it < 100; ++it) {
      UF(S, F, rr);
      if (F == 0.0) { ok = 1; break; }
      if (F < 0) lo = S; else hi = S;
      double Sn = S - F / rr;
      if (converged(Sn - S, Sn)) { S = Sn; ok = 1; break; }
      if (!(Sn > lo && Sn < hi)) Sn = 0.5 * (lo + hi);
      double d = Sn - S;
      S = Sn;
      if (converged(d, S)) { ok = 1; break; }
    }
#undef UF
    if (!ok) return OR_ENOCONV;
    stumpff(beta * S * S, cc);
    double G1 = S * cc[1], G2 = S * S * cc[2], G3 = S * S * S * cc[3];
    double r = r0 * cc[0] + sig * G1 + mu * G2;
    f = 1.0 - mu * G2 / r0;
    g = h - mu * G3;
    fd = -mu * G1 / (r * r0);
    gd = 1.0 - mu * G2 / r;
  }
  for (int c = 0; c < 3; ++c) {
    x1[c] = f * x0[c] + g * v0[c];
    v1[c] = fd * x0[c] + gd * v0[c];
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Minimum squared separation of a pair inside the step (the encounter test of
 * the mce_snif region, Sect. 2.1.2; the paper does not print how the minimum
 * is found, so this is the reading the whole oracle uses).  Over the step,
 * tau = t/h in [0,1], the relative position is the cubic Hermite interpolant
 * that takes the value r0 and the slope h*w0 at tau = 0 and r1, h*w1 at tau = 1:
 *   r(tau) = H00(tau) r0 + H10(tau) h w0 + H01(tau) r1 + H11(tau) h w1,
 *   H00 = (1 + 2 tau)(1 - tau)^2,  H10 = tau (1 - tau)^2,
 *   H01 = tau^2 (3 - 2 tau),       H11 = tau^2 (tau - 1).
 * |r|^2 is minimised over the two end points and over the interior zeros of
 * its derivative 2 r.r' at which the derivative passes from negative to
 * non-negative between neighbouring points of a fixed grid of 16 intervals;
 * such a zero is located by 40 halvings of its interval and |r|^2 taken at
 * the final midpoint.                                                       */
static void herm_at(const double r0[3], const double p0[3], const double r1[3],
                    const double p1[3], double tau, double r[3], double dr[3]) {
  double s = 1.0 - tau;
  double h00 = (1.0 + 2.0 * tau) * s * s;
  double h10 = tau * s * s;
  double h01 = tau * tau * (3.0 - 2.0 * tau);
  double h11 = tau * tau * (tau - 1.0);
  double g00 = 6.0 * tau * (tau - 1.0); /* dH00/dtau; dH01/dtau = -g00 */
  double g10 = s * (1.0 - 3.0 * tau);
  double g11 = tau * (3.0 * tau - 2.0);
  for (int k = 0; k < 3; ++k) {
    r[k] = h00 * r0[k] + h10 * p0[k] + h01 * r1[k] + h11 * p1[k];
    dr[k] = g00 * (r0[k] - r1[k]) + g10 * p0[k] + g11 * p1[k];
  }
}

/* sign-deciding half derivative r . dr/dtau, and |r|^2 */
static double herm_slope(const double r0[3], const double p0[3], const double r1[3],
                         const double p1[3], double tau, double* d2) {
  double r[3], dr[3];
  herm_at(r0, p0, r1, p1, tau, r, dr);
  if (d2) *d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  return r[0] * dr[0] + r[1] * dr[1] + r[2] * dr[2];
}

double or_pair_dmin2(const double r0[3], const double w0[3], const double r1[3],
                     const double w1[3], double h) {
  double p0[3], p1[3];
  for (int k = 0; k < 3; ++k) {
    p0[k] = h * w0[k];
    p1[k] = h * w1[k];
  }
  double d0 = r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2];
  double d1 = r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2];
  double best = d0 < d1 ? d0 : d1;
  const int NG = 16;
  double s_lo = herm_slope(r0, p0, r1, p1, 0.0, NULL);
  for (int k = 0; k < NG; ++k) {
    double lo = (double)k / NG, hi = (double)(k + 1) / NG;
    double s_hi = herm_slope(r0, p0, r1, p1, hi, NULL);
    int falls = s_lo < 0.0 && !(s_hi < 0.0);
    s_lo = s_hi;
    if (!falls) continue;
    for (int it = 0; it < 40; ++it) {
      double mid = 0.5 * (lo + hi);
      if (herm_slope(r0, p0, r1, p1, mid, NULL) < 0.0) lo = mid;
      else hi = mid;
    }
    double d;
    herm_slope(r0, p0, r1, p1, 0.5 * (lo + hi), &d);
    if (d < best) best = d;
  }
  return best;
}

/* Encounter flagging (the mce_snif critical region): every unordered pair
 * {big i, body j > i} whose minimum separation over the step is <= rc,
 * rc = max(rcrit_i, rcrit_j), inclusive.  Pairs come out sorted by (i, j):
 * for each i the tests of all j are taken first (independently, so they may
 * run in parallel) and the flagged j are then listed in increasing order.   */
int or_flag(int n, int nb, const double* rcrit, const double* x0, const double* u0,
            const double* x1, const double* u1, double h, int32_t* pairs, int cap,
            int* n_pairs) {
  int np = 0;
  unsigned char* hit = (unsigned char*)malloc(n > 0 ? (size_t)n : 1);
  if (!hit) { *n_pairs = 0; return OR_ENOMEM; }
  for (int i = 0; i < nb; ++i) {
#pragma omp parallel for schedule(static)
    for (int j = i + 1; j < n; ++j) {
      double rcj = j < nb ? rcrit[j] : 0.0;
      double rc = rcrit[i] > rcj ? rcrit[i] : rcj;
      double r0[3], r1[3], w0[3], w1[3];
      for (int k = 0; k < 3; ++k) {
        r0[k] = x0[k * n + j] - x0[k * n + i];
        r1[k] = x1[k * n + j] - x1[k * n + i];
        w0[k] = u0[k * n + j] - u0[k * n + i];
        w1[k] = u1[k * n + j] - u1[k * n + i];
      }
      hit[j] = or_pair_dmin2(r0, w0, r1, w1, h) <= rc * rc;
    }
    for (int j = i + 1; j < n; ++j) {
      if (!hit[j]) continue;
      if (np < cap) {
        pairs[2 * np] = i;
        pairs[2 * np + 1] = j;
      }
      ++np;
    }
  }
  free(hit);
  *n_pairs = np;
  return np <= cap ? OR_OK : OR_EINVAL;
}

/* ------------------------------------------------------------------ */
/* Bulirsch-Stoer on one subsystem ("BS for conservative forces").  The
 * members feel the star (mu0) and, for each flagged pair in the subsystem,
 * the complementary part (1-K) of the pair force.  Each BS step runs the
 * Stoermer (velocity-Verlet) rule with n = 2,4,...,16 substeps, extrapolates
 * polynomially in (H/n)^2 (Aitken-Neville), and accepts when
 * max_members,coords max(dx^2 xscal, dv^2 vscal) <= tol^2 with
 * xscal = 1/|x|^2, vscal = 1/|v|^2 at the BS step start (the xscal/vscal
 * loop of Sect. 2.1.1).  Otherwise H halves; an acceptance at column <= 5
 * doubles H.  More than 30 consecutive halvings is a failure.
 * xs, vs: [m][3] member-major; pl: local member indices of each pair.       */
static void bs_force(int m, const double* mu_m, const double* rc_m, int np,
                     const int32_t* pl, double mu0, const double* xs, double* as) {
  for (int k = 0; k < m; ++k) {
    const double* p = xs + 3 * k;
    double r2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    double r = sqrt(r2);
    double f = -mu0 / (r2 * r);
    as[3 * k] = f * p[0];
    as[3 * k + 1] = f * p[1];
    as[3 * k + 2] = f * p[2];
  }
  for (int q = 0; q < np; ++q) {
    int a = pl[2 * q], b = pl[2 * q + 1];
    double d[3];
    for (int c = 0; c < 3; ++c) d[c] = xs[3 * b + c] - xs[3 * a + c];
    double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double rc = rc_m[a] > rc_m[b] ? rc_m[a] : rc_m[b];
    double w = s2 > 0.0 ? (1.0 / (s2 * sqrt(s2))) * (1.0 - kfun(s2, rc)) : 0.0;
    for (int c = 0; c < 3; ++c) {
      as[3 * a + c] += mu_m[b] * w * d[c];
      as[3 * b + c] -= mu_m[a] * w * d[c];
    }
  }
}

static void stoermer(int m, const double* mu_m, const double* rc_m, int np, const int32_t* pl,
                     double mu0, const double* x0, const double* v0, double H, int nsub,
                     double* xo, double* vo, double* acc, double* d) {
  double dt = H / nsub;
  int nn = 3 * m;
  for (int i = 0; i < nn; ++i) xo[i] = x0[i];
  bs_force(m, mu_m, rc_m, np, pl, mu0, xo, acc);
  for (int i = 0; i < nn; ++i) {
    d[i] = dt * (v0[i] + 0.5 * dt * acc[i]);
    xo[i] += d[i];
  }
  for (int k = 1; k < nsub; ++k) {
    bs_force(m, mu_m, rc_m, np, pl, mu0, xo, acc);
    for (int i = 0; i < nn; ++i) {
      d[i] += dt * dt * acc[i];
      xo[i] += d[i];
    }
  }
  bs_force(m, mu_m, rc_m, np, pl, mu0, xo, acc);
  for (int i = 0; i < nn; ++i) vo[i] = d[i] / dt + 0.5 * dt * acc[i];
}


int or_bs(int m, const double* mu_m, const double* rc_m, int np, const int32_t* pl, double mu0,
          double h, double tol, double* xs, double* vs) {
  enum { KMAX = 8 };
  const int nn = 3 * m;
  /* T[k][j] holds the extrapolation table entry (x then v), k, j < KMAX */
  double* T = (double*)malloc(sizeof(double) * KMAX * KMAX * 2 * nn);
  double* wk = (double*)malloc(sizeof(double) * 4 * nn);
  double* scal = (double*)malloc(sizeof(double) * 2 * m);
  if (!T || !wk || !scal) { free(T); free(wk); free(scal); return OR_ENOMEM; }
#define TAB(k, j) (T + ((size_t)(k) * KMAX + (j)) * 2 * nn)
  double* xo = wk;
  double* vo = wk + nn;
  double* acc = wk + 2 * nn;
  double* dd = wk + 3 * nn;
  double done = 0.0, H = h;
  int fails = 0, status = OR_OK;
  while (fabs(h - done) > 1e-14 * fabs(h)) {
    double rem = h - done;
    if (fabs(H) > fabs(rem)) H = rem;
    for (int k = 0; k < m; ++k) {
      const double* p = xs + 3 * k;
      const double* q = vs + 3 * k;
      scal[k] = 1.0 / (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
      scal[m + k] = 1.0 / (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    }
    int accepted = -1;
    for (int k = 0; k < KMAX; ++k) {
      int nk = 2 * (k + 1);
      stoermer(m, mu_m, rc_m, np, pl, mu0, xs, vs, H, nk, xo, vo, acc, dd);
      double* t0 = TAB(k, 0);
      for (int i = 0; i < nn; ++i) { t0[i] = xo[i]; t0[nn + i] = vo[i]; }
      for (int j = 1; j <= k; ++j) {
        double ratio = (double)nk / (double)(2 * (k - j + 1));
        double den = ratio * ratio - 1.0;
        double* cur = TAB(k, j);
        double* left = TAB(k, j - 1);
        double* up = TAB(k - 1, j - 1);
        for (int i = 0; i < 2 * nn; ++i) cur[i] = left[i] + (left[i] - up[i]) / den;
      }
      if (k >= 1) {
        double* best = TAB(k, k);
        double* prev = TAB(k, k - 1);
        double err = 0.0;
        for (int b = 0; b < m; ++b) {
          for (int c = 0; c < 3; ++c) {
            double ex = best[3 * b + c] - prev[3 * b + c];
            double ev = best[nn + 3 * b + c] - prev[nn + 3 * b + c];
            double e1 = ex * ex * scal[b];
            double e2 = ev * ev * scal[m + b];
            if (e1 > err) err = e1;
            if (e2 > err) err = e2;
          }
        }
        if (err <= tol * tol) { accepted = k; break; }
      }
    }
    if (accepted >= 0) {
      double* best = TAB(accepted, accepted);
      for (int i = 0; i < nn; ++i) { xs[i] = best[i]; vs[i] = best[nn + i]; }
      done += H;
      fails = 0;
      if (accepted <= 4) H = 2.0 * H; /* columns are counted from 1: column <= 5 */
    } else {
      H = 0.5 * H;
      if (++fails > 30) { status = OR_EBS; break; }
    }
  }
#undef TAB
  free(T); free(wk); free(scal);
  return status;
}

/* ------------------------------------------------------------------ */
/* Subsystem decomposition of the flagged pairs and the BS hand-off.
 * Big-big pairs join big bodies into connected components; a component of
 * two or more bodies is integrated as one subsystem and all its members keep
 * the result.  Each flagged small body is integrated with copies of the big
 * components it touches; only the small body keeps its result.  Every
 * subsystem starts from the pre-drift state (x0, u0) and overwrites (x1, u1). */
static int find_root(int* par, int a) {
  while (par[a] != a) a = par[a];
  return a;
}

static int cmp_int(const void* a, const void* b) {
  int x = *(const int*)a, y = *(const int*)b;
  return (x > y) - (x < y);
}

static int run_subsystem(const or_sys* s, int m, const int* mem, int np, const int32_t* pl,
                         int keep_from, double h) {
  int n = s->n;
  double* buf = (double*)malloc(sizeof(double) * (8 * (size_t)m + 1));
  if (!buf) return OR_ENOMEM;
  double* xs = buf;
  double* vs = buf + 3 * m;
  double* mu_m = buf + 6 * m;
  double* rc_m = buf + 7 * m;
  for (int k = 0; k < m; ++k) {
    int b = mem[k];
    for (int c = 0; c < 3; ++c) {
      xs[3 * k + c] = s->x0[c * n + b];
      vs[3 * k + c] = s->u0[c * n + b];
    }
    mu_m[k] = b < s->nb ? s->mu[b] : 0.0;
    rc_m[k] = b < s->nb ? s->rcrit[b] : 0.0;
  }
  int st = or_bs(m, mu_m, rc_m, np, pl, s->mu0, h, s->p.bs_tol, xs, vs);
  if (st == OR_OK) {
    for (int k = keep_from; k < m; ++k) {
      int b = mem[k];
      for (int c = 0; c < 3; ++c) {
        s->x1[c * n + b] = xs[3 * k + c];
        s->u1[c * n + b] = vs[3 * k + c];
      }
    }
  }
  free(buf);
  return st;
}

static int local_index(const int* mem, int m, int b) {
  for (int k = 0; k < m; ++k)
    if (mem[k] == b) return k;
  return -1;
}

static int encounter_bs(or_sys* s, double h) {
  int nb = s->nb, np = s->npairs;
  const int32_t* P = s->pairs;
  if (np == 0) return OR_OK;
  int* par = (int*)malloc(sizeof(int) * (nb > 0 ? nb : 1));
  int* mem = (int*)malloc(sizeof(int) * (nb + 1));
  int32_t* pl = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(np + 1));
  int* inbig = (int*)calloc(nb > 0 ? nb : 1, sizeof(int));
  if (!par || !mem || !pl || !inbig) { free(par); free(mem); free(pl); free(inbig); return OR_ENOMEM; }
  for (int i = 0; i < nb; ++i) par[i] = i;
  for (int q = 0; q < np; ++q) {
    int i = P[2 * q], j = P[2 * q + 1];
    if (j < nb) {
      int ri = find_root(par, i), rj = find_root(par, j);
      if (ri != rj) { if (ri < rj) par[rj] = ri; else par[ri] = rj; }
      inbig[i] = inbig[j] = 1;
    }
  }
  int status = OR_OK;
  /* big components with two or more members, in order of their smallest index */
  for (int r = 0; r < nb && status == OR_OK; ++r) {
    if (!inbig[r] || find_root(par, r) != r) continue;
    int m = 0;
    for (int b = 0; b < nb; ++b)
      if (inbig[b] && find_root(par, b) == r) mem[m++] = b;
    int npl = 0;
    for (int q = 0; q < np; ++q) {
      int i = P[2 * q], j = P[2 * q + 1];
      if (j < nb && find_root(par, i) == r) {
        pl[2 * npl] = local_index(mem, m, i);
        pl[2 * npl + 1] = local_index(mem, m, j);
        ++npl;
      }
    }
    status = run_subsystem(s, m, mem, npl, pl, 0, h);
  }
  /* flagged small bodies, ascending */
  int* smalls = (int*)malloc(sizeof(int) * (size_t)np);
  int nsm = 0;
  if (!smalls) status = OR_ENOMEM;
  for (int q = 0; q < np && smalls; ++q)
    if (P[2 * q + 1] >= nb) smalls[nsm++] = P[2 * q + 1];
  if (smalls) qsort(smalls, nsm, sizeof(int), cmp_int);
  for (int t = 0; t < nsm && status == OR_OK; ++t) {
    int j = smalls[t];
    if (t > 0 && smalls[t - 1] == j) continue;
    /* big members: the whole component of every big body flagged with j */
    int m = 0;
    for (int q = 0; q < np; ++q) {
      if (P[2 * q + 1] != j) continue;
      int i = P[2 * q];
      int r = find_root(par, i);
      for (int b = 0; b < nb; ++b) {
        int same = (b == i) || (inbig[i] && inbig[b] && find_root(par, b) == r);
        if (same && local_index(mem, m, b) < 0) mem[m++] = b;
      }
    }
    qsort(mem, m, sizeof(int), cmp_int);
    int nbig_mem = m;
    mem[m++] = j;
    int npl = 0;
    for (int q = 0; q < np; ++q) {
      int a = P[2 * q], b = P[2 * q + 1];
      if (b < nb) {
        int la = local_index(mem, nbig_mem, a), lb = local_index(mem, nbig_mem, b);
        if (la >= 0 && lb >= 0) { pl[2 * npl] = la; pl[2 * npl + 1] = lb; ++npl; }
      } else if (b == j) {
        pl[2 * npl] = local_index(mem, nbig_mem, a);
        pl[2 * npl + 1] = nbig_mem;
        ++npl;
      }
    }
    status = run_subsystem(s, m, mem, npl, pl, nbig_mem, h);
  }
  free(smalls);
  free(par); free(mem); free(pl); free(inbig);
  return status;
}

/* ------------------------------------------------------------------ */
/* Orbital elements from a state (textbook two-body relations); el =
 * (a, e, i, q, |h|, energy).  Used for the Hill radius at start-up and by
 * tests.                                                                  */
void or_x2el(double gm, const double x[3], const double v[3], double el[6]) {
  double hx = x[1] * v[2] - x[2] * v[1];
  double hy = x[2] * v[0] - x[0] * v[2];
  double hz = x[0] * v[1] - x[1] * v[0];
  double h2 = hx * hx + hy * hy + hz * hz;
  double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  double en = 0.5 * vv - gm / r;
  double ex = (v[1] * hz - v[2] * hy) / gm - x[0] / r;
  double ey = (v[2] * hx - v[0] * hz) / gm - x[1] / r;
  double ez = (v[0] * hy - v[1] * hx) / gm - x[2] / r;
  double e = sqrt(ex * ex + ey * ey + ez * ez);
  el[0] = -gm / (2.0 * en);
  el[1] = e;
  el[2] = acos(hz / sqrt(h2));
  el[3] = h2 / (gm * (1.0 + e));
  el[4] = sqrt(h2);
  el[5] = en;
}

/* Mass schedule of the core-growth phase, Eq. 13, held at Mc after tau_c. */
static void apply_growth(or_sys* s, double t) {
  if (!s->growth) return;
  const double E = 2.718281828459045235;
  for (int k = 0; k < s->nb; ++k) {
    double m0 = s->growth[3 * k], mc = s->growth[3 * k + 1], tau = s->growth[3 * k + 2];
    if (!(tau > 0.0)) continue;
    double mu = t >= tau ? mc : m0 + (E / (E - 1.0)) * (mc - m0) * (1.0 - exp(-t / tau));
    s->mu[k] = mu;
    s->rcrit[k] = s->rcrit_init[k] * cbrt(mu / s->mu_init[k]);
  }
}

static void momentum(const or_sys* s, const double* u, double P[3]);

/* Sound speed of the disk at cylindrical radius R (as in the drag). */
static double disk_cs(const or_params* p, double mu0, double R) {
  if (p->temp_1au > 0.0) return sqrt(p->cs2_per_k * p->temp_1au * pow(R, -p->temp_beta));
  return p->h_over_r * sqrt(mu0 / R);
}

/* Planet radius during the solid/atmosphere phase, Eq. 14 (Sect. 3.2):
 * R_p = G M / (c_s^2 / k1 + G M / (k2 R_H)), k1 = 1, k2 = 1/4.              */
static double radius_core(double gm, double cs, double rhill) {
  return gm / (cs * cs / 1.0 + gm / (0.25 * rhill));
}

/* The time-dependent physics of the massive bodies at the start of a step (time
 * t = s->time), held through the step:
 *  - mass: Eq. 13 for t < tau_c; for t >= tau_c, Eq. 15 (runaway gas accretion)
 *    when tau_g > 0, else M_c; the changeover radius follows the Hill radius,
 *    rcrit = rcrit_init (M / M_init)^(1/3);
 *  - radius: Eq. 14 before tau_c with the disk's c_s at the planet's cylindrical
 *    distance and its Hill radius r (M / 3 m0)^(1/3) at its distance r from the
 *    star; from tau_c on (with tau_g > 0), Eq. 16 with R_c the Eq. 14 radius at the
 *    first step of the runaway and Delta R = R_c - R_I;
 *  - migration: a velocity change along the planet's heliocentric velocity of
 *    Eq. 17 for t < tau1 and of Eq. 18 for t >= tau1, with a_p the osculating
 *    semi-major axis (gm = G(m0 + m)) and v_k = sqrt(G (m0 + m) / a_p);
 *  - gap: open after tau_c (tau_g > 0, gap_C > 0), centred on the planet's
 *    cylindrical distance, half width gap_C R_H (Eq. 8), density factor
 *    exp(-(t - tau_c)/tau_g) (Eq. 9);
 *  - step switch (Sect. 3.6): once a migrating planet's a_p <= a_switch, the step
 *    becomes 1/25 of the orbital period at a_min, from this step on.          */
static void apply_physics(or_sys* s) {
  const double E = 2.718281828459045235;
  int n = s->n, nb = s->nb;
  double t = s->time, G = s->p.G, mu0 = s->mu0;
  for (int k = 0; k < nb; ++k) {
    const or_planet* q = &s->phys[k];
    if (!(q->tau_c > 0.0)) continue;
    double m;
    if (t < q->tau_c)
      m = q->M0 + (E / (E - 1.0)) * (q->Mc - q->M0) * (1.0 - exp(-t / q->tau_c));
    else if (q->tau_g > 0.0)
      m = q->Mc + (q->Mf - q->Mc) * (1.0 - exp(-(t - q->tau_c) / q->tau_g));
    else
      m = q->Mc;
    s->mu[k] = G * m;
    s->rcrit[k] = s->rcrit_init[k] * cbrt(s->mu[k] / s->mu_init[k]);
  }
  /* heliocentric states and osculating semi-major axes at the step start */
  double P[3];
  momentum(s, s->u, P);
  double* ap = (double*)malloc(sizeof(double) * 5 * (size_t)nb);
  if (!ap) return;
  double* rr = ap + nb;      /* distance from the star */
  double* Rc = ap + 2 * nb;  /* cylindrical distance */
  double* vn = ap + 3 * nb;  /* |v| heliocentric */
  double* rh = ap + 4 * nb;  /* Hill radius */
  int inside = 0;
  for (int k = 0; k < nb; ++k) {
    const or_planet* q = &s->phys[k];
    double x[3] = {s->x[k], s->x[n + k], s->x[2 * n + k]};
    double v[3];
    for (int c = 0; c < 3; ++c) v[c] = s->u[c * n + k] + P[c] / mu0;
    double el[6];
    or_x2el(mu0 + s->mu[k], x, v, el);
    ap[k] = el[0];
    rr[k] = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    Rc[k] = sqrt(x[0] * x[0] + x[1] * x[1]);
    vn[k] = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    rh[k] = rr[k] * cbrt(s->mu[k] / (3.0 * mu0));
    if ((q->tau1 > 0.0 || q->tau2 > 0.0) && s->a_switch > 0.0 && ap[k] > 0.0 &&
        ap[k] <= s->a_switch)
      inside = 1;
  }
  if (inside && !s->switched) {
    s->h = 2.0 * PI * sqrt(s->a_min * s->a_min * s->a_min / mu0) / 25.0;
    s->switched = 1;
  }
  for (int k = 0; k < nb; ++k) {
    const or_planet* q = &s->phys[k];
    /* radius */
    double cs = disk_cs(&s->p, mu0, Rc[k]);
    if (q->tau_c > 0.0 && q->tau_g > 0.0 && t >= q->tau_c) {
      if (s->rad_c[k] == 0.0) s->rad_c[k] = radius_core(s->mu[k], cs, rh[k]);
      double R0 = s->rad_c[k];
      s->radius[k] = R0 - (R0 - q->R_I) * (1.0 - exp(-(t - q->tau_c) / q->tau_g));
    } else {
      s->radius[k] = radius_core(s->mu[k], cs, rh[k]);
    }
    /* gap */
    s->gap_on[k] = q->gap_C > 0.0 && q->tau_c > 0.0 && q->tau_g > 0.0 && t > q->tau_c;
    s->gaps[3 * k] = Rc[k];
    s->gaps[3 * k + 1] = q->gap_C * rh[k];
    s->gaps[3 * k + 2] = s->gap_on[k] ? exp(-(t - q->tau_c) / q->tau_g) : 1.0;
    /* migration: velocity change along the heliocentric velocity */
    if ((q->tau1 > 0.0 || q->tau2 > 0.0) && ap[k] > 0.0) {
      double vk = sqrt((mu0 + s->mu[k]) / ap[k]);
      double t1 = q->tau1 > 0.0 ? q->tau1 : 0.0;
      double dv = 0.0;
      if (q->tau1 > 0.0 && t < q->tau1)
        dv = 0.5 * (q->da1 / ap[k]) * (s->h / q->tau1) * vk;
      else if (q->tau2 > 0.0)
        dv = 0.5 * (q->da2 / ap[k]) * (s->h / q->tau2) * exp(-(t - t1) / q->tau2) * vk;
      for (int c = 0; c < 3; ++c) {
        double vc = s->u[c * n + k] + P[c] / mu0;
        s->u[c * n + k] += dv * vc / vn[k];
      }
    }
  }
  free(ap);
}

static void momentum(const or_sys* s, const double* u, double P[3]) {
  int n = s->n;
  P[0] = P[1] = P[2] = 0.0;
  for (int k = 0; k < s->nb; ++k) {
    P[0] += s->mu[k] * u[k];
    P[1] += s->mu[k] * u[n + k];
    P[2] += s->mu[k] * u[2 * n + k];
  }
}

static void refresh_fsal(or_sys* s) { or_gravity(s->n, s->nb, s->x, s->mu, s->rcrit, s->ag); }

or_sys* or_create(const or_params* p, const double* x_h, const double* v_h, const double* m_big,
                  const double* r_p, const double* rho_p, const double* growth, int* status) {
  int n = p->n_big + p->n_small;
  *status = OR_EINVAL;
  if (p->n_big < 0 || p->n_small < 0 || n <= 0 || !(p->G > 0) || !(p->m0 > 0)) return NULL;
  if (p->gas_on && p->n_small > 0 && (!r_p || !rho_p)) return NULL;
  for (int k = 0; k < p->n_big; ++k)
    if (!(m_big[k] > 0.0)) return NULL;
  or_sys* s = (or_sys*)calloc(1, sizeof(or_sys));
  *status = OR_ENOMEM;
  if (!s) return NULL;
  s->p = *p;
  s->n = n;
  s->nb = p->n_big;
  s->ns = p->n_small;
  s->mu0 = p->G * p->m0;
  size_t v3 = sizeof(double) * 3 * (size_t)n;
  s->x = (double*)malloc(v3); s->u = (double*)malloc(v3); s->ag = (double*)malloc(v3);
  s->x0 = (double*)malloc(v3); s->u0 = (double*)malloc(v3);
  s->x1 = (double*)malloc(v3); s->u1 = (double*)malloc(v3); s->ad = (double*)malloc(v3);
  s->x1k = (double*)calloc(1, v3); s->u1k = (double*)calloc(1, v3);
  size_t nbs = sizeof(double) * (s->nb > 0 ? s->nb : 1);
  s->mu = (double*)malloc(nbs); s->mu_init = (double*)malloc(nbs);
  s->rcrit = (double*)malloc(nbs); s->rcrit_init = (double*)malloc(nbs);
  size_t nss = sizeof(double) * (s->ns > 0 ? s->ns : 1);
  s->r_p = (double*)calloc(1, nss); s->rho_p = (double*)calloc(1, nss);
  s->cap_pairs = 1 << 20;
  s->pairs = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)s->cap_pairs);
  if (!s->x || !s->u || !s->ag || !s->x0 || !s->u0 || !s->x1 || !s->u1 || !s->ad || !s->mu ||
      !s->x1k || !s->u1k ||
      !s->mu_init || !s->rcrit || !s->rcrit_init || !s->r_p || !s->rho_p || !s->pairs) {
    or_destroy(s);
    return NULL;
  }
  if (growth) {
    s->growth = (double*)malloc(sizeof(double) * 3 * (size_t)s->nb);
    if (!s->growth) { or_destroy(s); return NULL; }
    for (int k = 0; k < s->nb; ++k) {
      s->growth[3 * k] = p->G * growth[3 * k];
      s->growth[3 * k + 1] = p->G * growth[3 * k + 1];
      s->growth[3 * k + 2] = growth[3 * k + 2];
    }
  }
  double mtot = s->mu0, P[3] = {0, 0, 0};
  for (int k = 0; k < s->nb; ++k) {
    s->mu[k] = s->mu_init[k] = p->G * m_big[k];
    mtot += s->mu[k];
    for (int c = 0; c < 3; ++c) P[c] += s->mu[k] * v_h[c * n + k];
  }
  /* heliocentric -> democratic heliocentric: u = v - (sum m v)/(m0 + sum m) */
  for (int c = 0; c < 3; ++c) {
    double V = P[c] / mtot;
    for (int t = 0; t < n; ++t) {
      s->x[c * n + t] = x_h[c * n + t];
      s->u[c * n + t] = v_h[c * n + t] - V;
    }
  }
  /* changeover radius: rcrit_hill Hill radii with the osculating a at start */
  for (int k = 0; k < s->nb; ++k) {
    double xk[3] = {x_h[k], x_h[n + k], x_h[2 * n + k]};
    double vk[3] = {v_h[k], v_h[n + k], v_h[2 * n + k]};
    double el[6];
    or_x2el(s->mu0 + s->mu[k], xk, vk, el);
    double a = el[0];
    if (!(a > 0.0) || !isfinite(a)) a = sqrt(xk[0] * xk[0] + xk[1] * xk[1] + xk[2] * xk[2]);
    s->rcrit[k] = s->rcrit_init[k] = p->rcrit_hill * a * cbrt(s->mu[k] / (3.0 * s->mu0));
  }
  for (int j = 0; j < s->ns; ++j) {
    if (r_p) s->r_p[j] = r_p[j];
    if (rho_p) s->rho_p[j] = rho_p[j] * p->rho_unit;
  }
  s->step = 0;
  s->time = 0.0;
  s->h = p->dt;
  refresh_fsal(s);
  *status = OR_OK;
  return s;
}

void or_destroy(or_sys* s) {
  if (!s) return;
  free(s->x); free(s->u); free(s->ag); free(s->x0); free(s->u0); free(s->x1); free(s->u1);
  free(s->ad); free(s->x1k); free(s->u1k); free(s->mu);
  free(s->phys); free(s->radius); free(s->rad_c); free(s->gaps); free(s->gap_on);
  free(s->stat); free(s->rsign); free(s->mu_init); free(s->rcrit); free(s->rcrit_init);
  free(s->r_p); free(s->rho_p); free(s->growth); free(s->pairs);
  free(s);
}

static void half_kick(or_sys* s, double hh) {
  int n = s->n;
  or_drag_gaps(&s->p, n, s->nb, s->x, s->u, s->mu, s->r_p, s->rho_p,
               s->phys ? s->gaps : NULL, s->gap_on, s->ad);
  for (int i = 0; i < 3 * n; ++i) s->u[i] += hh * (s->ag[i] + s->ad[i]);
}

/* jump: x += (h/2) P/mu0 with P over the massive bodies only */
static void jump(or_sys* s, double hh) {
  int n = s->n;
  double P[3];
  momentum(s, s->u, P);
  for (int c = 0; c < 3; ++c) {
    double d = hh * P[c] / s->mu0;
    for (int t = 0; t < n; ++t) s->x[c * n + t] += d;
  }
}

/* One hybrid step (Sect. 2; the kick listing of Sect. 2.1.2 with angf = 0). */
static int one_step(or_sys* s) {
  int n = s->n;
  if (s->phys) apply_physics(s);
  else apply_growth(s, s->step * s->p.dt);
  double h = s->h, hh = 0.5 * h;
  half_kick(s, hh);
  jump(s, hh);
  memcpy(s->x0, s->x, sizeof(double) * 3 * n);
  memcpy(s->u0, s->u, sizeof(double) * 3 * n);
  int bad = OR_OK;
#pragma omp parallel for schedule(static) reduction(min : bad)
  for (int t = 0; t < n; ++t) {
    double a[3] = {s->x0[t], s->x0[n + t], s->x0[2 * n + t]};
    double b[3] = {s->u0[t], s->u0[n + t], s->u0[2 * n + t]};
    double c[3], d[3];
    int st = or_drift(s->mu0, a, b, h, c, d);
    if (st < bad) bad = st;
    for (int k = 0; k < 3; ++k) { s->x1[k * n + t] = c[k]; s->u1[k * n + t] = d[k]; }
  }
  if (bad != OR_OK) return bad;
  memcpy(s->x1k, s->x1, sizeof(double) * 3 * n);
  memcpy(s->u1k, s->u1, sizeof(double) * 3 * n);
  int np = 0;
  or_flag(n, s->nb, s->rcrit, s->x0, s->u0, s->x1, s->u1, h, s->pairs, s->cap_pairs, &np);
  if (np > s->cap_pairs) return OR_EINVAL;
  s->npairs = np;
  int st = encounter_bs(s, h);
  if (st != OR_OK) return st;
  memcpy(s->x, s->x1, sizeof(double) * 3 * n);
  memcpy(s->u, s->u1, sizeof(double) * 3 * n);
  jump(s, hh);
  refresh_fsal(s);
  half_kick(s, hh);
  s->step += 1;
  s->time += h;
  return OR_OK;
}

int or_step(or_sys* s, int n_steps) {
  for (int k = 0; k < n_steps; ++k) {
    int st = one_step(s);
    if (st != OR_OK) return st;
  }
  return OR_OK;
}

/* Energy with the potential over massive bodies only (the mxx_en change of
 * Sect. 2.1.3), and total angular momentum, both in Msun AU^2 day^-k units. */
void or_energy(const or_sys* s, double* E, double L[3]) {
  int n = s->n, nb = s->nb;
  const double* x = s->x;
  const double* u = s->u;
  double ke = 0.0, pe = 0.0, P[3];
  momentum(s, u, P);
  L[0] = L[1] = L[2] = 0.0;
  for (int k = 0; k < nb; ++k) {
    double xk = x[k], yk = x[n + k], zk = x[2 * n + k];
    double ux = u[k], uy = u[n + k], uz = u[2 * n + k];
    ke += 0.5 * s->mu[k] * (ux * ux + uy * uy + uz * uz);
    pe -= s->mu0 * s->mu[k] / sqrt(xk * xk + yk * yk + zk * zk);
    L[0] += s->mu[k] * (yk * uz - zk * uy);
    L[1] += s->mu[k] * (zk * ux - xk * uz);
    L[2] += s->mu[k] * (xk * uy - yk * ux);
  }
  ke += (P[0] * P[0] + P[1] * P[1] + P[2] * P[2]) / (2.0 * s->mu0);
  for (int i = 0; i < nb; ++i)
    for (int j = i + 1; j < nb; ++j) {
      double dx = x[j] - x[i], dy = x[n + j] - x[n + i], dz = x[2 * n + j] - x[2 * n + i];
      pe -= s->mu[i] * s->mu[j] / sqrt(dx * dx + dy * dy + dz * dz);
    }
  *E = (ke + pe) / s->p.G;
  for (int c = 0; c < 3; ++c) L[c] /= s->p.G;
}

int or_encounters(const or_sys* s, int32_t* pairs, int cap) {
  int m = s->npairs < cap ? s->npairs : cap;
  for (int i = 0; i < 2 * m; ++i) pairs[i] = s->pairs[i];
  return s->npairs;
}

void or_get_state(const or_sys* s, double* x_h, double* v_h) {
  int n = s->n;
  double P[3];
  momentum(s, s->u, P);
  for (int c = 0; c < 3; ++c)
    for (int t = 0; t < n; ++t) {
      x_h[c * n + t] = s->x[c * n + t];
      v_h[c * n + t] = s->u[c * n + t] + P[c] / s->mu0;
    }
}

void or_get_dh(const or_sys* s, double* x, double* u) {
  memcpy(x, s->x, sizeof(double) * 3 * s->n);
  memcpy(u, s->u, sizeof(double) * 3 * s->n);
}

/* Replace the state; the masses in force are those of the step before
 * step_index (the end-of-step force of a continuous run used them), and the
 * FSAL force is recomputed from the new positions.                        */
void or_set_dh(or_sys* s, const double* x, const double* u, long step_index) {
  memcpy(s->x, x, sizeof(double) * 3 * s->n);
  memcpy(s->u, u, sizeof(double) * 3 * s->n);
  s->step = step_index;
  s->time = (double)step_index * s->p.dt;
  s->h = s->p.dt;
  s->switched = 0;
  if (s->phys) {
    for (int k = 0; k < s->nb; ++k) s->rad_c[k] = 0.0;
    if (step_index > 0) {
      /* masses of the step before (the end-of-step force of a continuous run) */
      double keep_t = s->time;
      double* ukeep = (double*)malloc(sizeof(double) * 3 * (size_t)s->n);
      if (ukeep) memcpy(ukeep, s->u, sizeof(double) * 3 * (size_t)s->n);
      s->time = (double)(step_index - 1) * s->p.dt;
      apply_physics(s);
      if (ukeep) { memcpy(s->u, ukeep, sizeof(double) * 3 * (size_t)s->n); free(ukeep); }
      s->time = keep_t;
      s->h = s->p.dt;
      s->switched = 0;
      for (int k = 0; k < s->nb; ++k) s->rad_c[k] = 0.0;  /* re-latched after a restart */
    } else {
      for (int k = 0; k < s->nb; ++k) { s->mu[k] = s->mu_init[k]; s->rcrit[k] = s->rcrit_init[k]; }
    }
  } else if (s->growth) {
    if (step_index > 0) {
      apply_growth(s, (step_index - 1) * s->p.dt);
    } else {
      for (int k = 0; k < s->nb; ++k) { s->mu[k] = s->mu_init[k]; s->rcrit[k] = s->rcrit_init[k]; }
    }
  }
  s->npairs = 0;
  refresh_fsal(s);
}

void or_get_accel(const or_sys* s, double* a) { memcpy(a, s->ag, sizeof(double) * 3 * s->n); }

/* Replace the changeover radii (massive bodies; the value at the current mass,
 * also kept as the reference radius of the growth law) and refresh the FSAL
 * force.  Used to hold the radii fixed while masses or orbits are perturbed. */
void or_set_rcrit(or_sys* s, const double* rcrit) {
  for (int k = 0; k < s->nb; ++k) {
    s->rcrit[k] = rcrit[k];
    s->rcrit_init[k] = rcrit[k] * cbrt(s->mu_init[k] / s->mu[k]);
  }
  refresh_fsal(s);
}

void or_get_mu(const or_sys* s, double* mu, double* rcrit) {
  for (int k = 0; k < s->nb; ++k) { mu[k] = s->mu[k]; rcrit[k] = s->rcrit[k]; }
}

long or_step_index(const or_sys* s) { return s->step; }

/* Threads the loops over bodies run on (1 without OpenMP). */
int or_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* The deciding quantity of the last step's encounter test for the pair (i, j):
 * its minimum squared separation over the step (or_pair_dmin2) from the
 * pre-drift state and the Kepler-drifted state before the encounter
 * integrator, and the squared changeover radius it was compared with.      */
double or_last_pair_dmin2(const or_sys* s, int i, int j, double* rc2) {
  int n = s->n, nb = s->nb;
  double r0[3], w0[3], r1[3], w1[3];
  for (int k = 0; k < 3; ++k) {
    r0[k] = s->x0[k * n + j] - s->x0[k * n + i];
    w0[k] = s->u0[k * n + j] - s->u0[k * n + i];
    r1[k] = s->x1k[k * n + j] - s->x1k[k * n + i];
    w1[k] = s->u1k[k * n + j] - s->u1k[k * n + i];
  }
  double rci = i < nb ? s->rcrit[i] : 0.0, rcj = j < nb ? s->rcrit[j] : 0.0;
  double rc = rci > rcj ? rci : rcj;
  if (rc2) *rc2 = rc * rc;
  return or_pair_dmin2(r0, w0, r1, w1, s->p.dt);
}


/* Install the time-dependent physics of the massive bodies (replaces a growth
 * schedule given at creation).  pl: [nb]; a_switch > 0 enables the step switch to
 * 1/25 of the period at a_min.                                               */
int or_set_physics(or_sys* s, const or_planet* pl, double a_switch, double a_min) {
  int nb = s->nb;
  if (nb <= 0 || !pl || (a_switch > 0.0 && !(a_min > 0.0))) return OR_EINVAL;
  free(s->phys); free(s->radius); free(s->rad_c); free(s->gaps); free(s->gap_on);
  free(s->stat); free(s->rsign);
  s->phys = (or_planet*)malloc(sizeof(or_planet) * (size_t)nb);
  s->radius = (double*)calloc((size_t)nb, sizeof(double));
  s->rad_c = (double*)calloc((size_t)nb, sizeof(double));
  s->gaps = (double*)calloc(3 * (size_t)nb, sizeof(double));
  s->gap_on = (int*)calloc((size_t)nb, sizeof(int));
  if (!s->phys || !s->radius || !s->rad_c || !s->gaps || !s->gap_on) return OR_ENOMEM;
  memcpy(s->phys, pl, sizeof(or_planet) * (size_t)nb);
  /* the masses given at creation are the ones in force before the first step
   * (M0 for a growing body) */
  s->a_switch = a_switch;
  s->a_min = a_min;
  s->switched = 0;
  s->h = s->p.dt;
  refresh_fsal(s);
  return OR_OK;
}

void or_get_radii(const or_sys* s, double* radius) {
  for (int k = 0; k < s->nb; ++k) radius[k] = s->radius ? s->radius[k] : 0.0;
}

double or_time(const or_sys* s) { return s->time; }
double or_step_size(const or_sys* s) { return s->h; }

/* The gaps of the current step: [nb][4] = centre R, half width, density factor,
 * open (1) or not (0). */
void or_get_gaps(const or_sys* s, double* g) {
  for (int k = 0; k < s->nb; ++k) {
    g[4 * k] = s->gaps ? s->gaps[3 * k] : 0.0;
    g[4 * k + 1] = s->gaps ? s->gaps[3 * k + 1] : 0.0;
    g[4 * k + 2] = s->gaps ? s->gaps[3 * k + 2] : 1.0;
    g[4 * k + 3] = s->gap_on ? (double)s->gap_on[k] : 0.0;
  }
}

/* Replace positions and velocities only (time, step size, masses and the physics
 * state are kept) and refresh the stored end-of-step force.                   */
void or_set_xu(or_sys* s, const double* x, const double* u) {
  memcpy(s->x, x, sizeof(double) * 3 * (size_t)s->n);
  memcpy(s->u, u, sizeof(double) * 3 * (size_t)s->n);
  refresh_fsal(s);
}

static void* dup_bytes(const void* src, size_t bytes) {
  if (!src) return NULL;
  void* d = malloc(bytes ? bytes : 1);
  if (d) memcpy(d, src, bytes);
  return d;
}

/* A deep copy of a system (state, masses, clock and physics state), for re-running a
 * step from the same point. */
or_sys* or_clone(const or_sys* s) {
  or_sys* c = (or_sys*)malloc(sizeof(or_sys));
  if (!c) return NULL;
  *c = *s;
  size_t v3 = sizeof(double) * 3 * (size_t)s->n;
  size_t nbs = sizeof(double) * (s->nb > 0 ? s->nb : 1);
  size_t nss = sizeof(double) * (s->ns > 0 ? s->ns : 1);
  c->x = dup_bytes(s->x, v3); c->u = dup_bytes(s->u, v3); c->ag = dup_bytes(s->ag, v3);
  c->x0 = dup_bytes(s->x0, v3); c->u0 = dup_bytes(s->u0, v3); c->x1 = dup_bytes(s->x1, v3);
  c->u1 = dup_bytes(s->u1, v3); c->ad = dup_bytes(s->ad, v3);
  c->x1k = dup_bytes(s->x1k, v3); c->u1k = dup_bytes(s->u1k, v3);
  c->mu = dup_bytes(s->mu, nbs); c->mu_init = dup_bytes(s->mu_init, nbs);
  c->rcrit = dup_bytes(s->rcrit, nbs); c->rcrit_init = dup_bytes(s->rcrit_init, nbs);
  c->r_p = dup_bytes(s->r_p, nss); c->rho_p = dup_bytes(s->rho_p, nss);
  c->growth = dup_bytes(s->growth, 3 * nbs);
  c->pairs = dup_bytes(s->pairs, sizeof(int32_t) * 2 * (size_t)s->cap_pairs);
  c->phys = dup_bytes(s->phys, sizeof(or_planet) * (size_t)(s->nb > 0 ? s->nb : 1));
  c->radius = dup_bytes(s->radius, nbs); c->rad_c = dup_bytes(s->rad_c, nbs);
  c->gaps = dup_bytes(s->gaps, 3 * nbs);
  c->gap_on = dup_bytes(s->gap_on, sizeof(int) * (size_t)(s->nb > 0 ? s->nb : 1));
  c->stat = dup_bytes(s->stat, sizeof(int32_t) * (size_t)s->n);
  c->rsign = dup_bytes(s->rsign, (size_t)s->n);
  return c;
}

/* Body removal.  The ejection criterion of Sect. 3.5: a body whose osculating
 * orbit about the star is unbound, e >= 1 (gm = G(m0 + m) for massive bodies,
 * G m0 for massless ones; heliocentric position and velocity), is flagged
 * stat = -3 and its mass set to zero.  Central-body encounters (the mce_cent
 * routine, whose test the paper does not print): with r_cen > 0 a body is flagged
 * stat = -2 when its distance from the star is <= r_cen, or when it passed
 * pericentre since the previous check (radial velocity inward then, outward or
 * zero now) on an orbit of perihelion distance q = |h|^2 / (gm (1 + e)) <= r_cen.
 * A flagged massive body keeps its place with zero mass, zero changeover radius
 * and its growth, migration and gap switched off; or_compact removes flagged
 * massless bodies.  Returns ejcount, the number of bodies with stat < 0 (the
 * workshare count of Sect. 2.1.2).                                            */
static int ensure_status(or_sys* s) {
  if (s->stat) return OR_OK;
  s->stat = (int32_t*)calloc((size_t)s->n, sizeof(int32_t));
  s->rsign = (int8_t*)calloc((size_t)s->n, 1);
  return s->stat && s->rsign ? OR_OK : OR_ENOMEM;
}

int or_check_removal(or_sys* s, double r_cen) {
  if (ensure_status(s) != OR_OK) return OR_ENOMEM;
  int n = s->n, nb = s->nb;
  double P[3];
  momentum(s, s->u, P);
  int count = 0;
  for (int t = 0; t < n; ++t) {
    if (s->stat[t] < 0) { ++count; continue; }
    double x[3] = {s->x[t], s->x[n + t], s->x[2 * n + t]};
    double v[3];
    for (int c = 0; c < 3; ++c) v[c] = s->u[c * n + t] + P[c] / s->mu0;
    double gm = s->mu0 + (t < nb ? s->mu[t] : 0.0);
    double el[6];
    or_x2el(gm, x, v, el);
    double e = el[1], q = el[3];
    double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    double rdot = x[0] * v[0] + x[1] * v[1] + x[2] * v[2];
    int st = 0;
    if (e >= 1.0) st = -3;
    else if (r_cen > 0.0 && (r <= r_cen || (s->rsign[t] < 0 && rdot >= 0.0 && q <= r_cen)))
      st = -2;
    s->rsign[t] = rdot < 0.0 ? -1 : 1;
    if (st < 0) {
      s->stat[t] = st;
      ++count;
      if (t < nb) {
        s->mu[t] = 0.0;
        s->rcrit[t] = 0.0;
        if (s->growth) s->growth[3 * t + 2] = 0.0;
        if (s->phys) memset(&s->phys[t], 0, sizeof(or_planet));
      }
    }
  }
  return count;
}

void or_get_status(const or_sys* s, int32_t* stat) {
  for (int t = 0; t < s->n; ++t) stat[t] = s->stat ? s->stat[t] : 0;
}

int or_n_bodies(const or_sys* s) { return s->n; }

/* Remove the flagged massless bodies, keeping the order of the others (massive
 * bodies keep their places).  index_map (or NULL): [n before] new index of each
 * body, -1 if removed.  Returns the number removed; the end-of-step force is kept
 * (the survivors' entries).                                                   */
int or_compact(or_sys* s, int32_t* index_map) {
  if (!s->stat) {
    if (index_map)
      for (int t = 0; t < s->n; ++t) index_map[t] = t;
    return 0;
  }
  int n = s->n, nb = s->nb, m = 0;
  int32_t* map = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!map) return OR_ENOMEM;
  for (int t = 0; t < n; ++t) map[t] = (t < nb || s->stat[t] >= 0) ? m++ : -1;
  int removed = n - m;
  double* arrs[] = {s->x, s->u, s->ag};
  for (int a = 0; a < 3; ++a) {
    double* A = arrs[a];
    for (int c = 0; c < 3; ++c)
      for (int t = 0; t < n; ++t)
        if (map[t] >= 0) A[c * m + map[t]] = A[c * n + t];
  }
  for (int t = nb; t < n; ++t)
    if (map[t] >= 0) {
      s->r_p[map[t] - nb] = s->r_p[t - nb];
      s->rho_p[map[t] - nb] = s->rho_p[t - nb];
    }
  for (int t = 0; t < n; ++t)
    if (map[t] >= 0) {
      s->stat[map[t]] = s->stat[t];
      s->rsign[map[t]] = s->rsign[t];
    }
  if (index_map) memcpy(index_map, map, sizeof(int32_t) * (size_t)n);
  free(map);
  s->n = m;
  s->ns = m - nb;
  s->p.n_small = s->ns;
  s->npairs = 0;
  return removed;
}
