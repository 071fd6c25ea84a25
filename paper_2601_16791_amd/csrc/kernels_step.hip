// Kernels of the hybrid step that stream over bodies (gfx950, FP64 VALU).
//
//   growth            : core-growth mass schedule of Eq. 13 at the step start
//   kick_jump_drift   : half kick (gravity + gas drag), jump by the massive-body
//                       momentum, Kepler drift; keeps the pre-drift state
//   jump_pack         : second jump; packs the massive bodies for the force
//   force_kick        : changeover-weighted gravity (rectangular, Sect. 2.1.3)
//                       plus gas drag and the closing half kick
//
// Layout: SoA [3][n] FP64 in HBM, big bodies first.  Sources of the force sum
// are read through wave-uniform (scalar) loads of packed 64-byte records, so
// every lane of a wave holds one target and all lanes walk the same source.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "force_sum.h"
#include "mx_internal.h"

namespace {

constexpr int kBlock = 256;

using mxd::DragConst;
using mxd::make_drag_const;


// ------------------------------------------------------------------ growth
// M(t) = M0 + e/(e-1) (Mc - M0) (1 - exp(-t/tau_c)) for t < tau_c, Mc after
// (body k grows when its tau_c = growth[3 k + 2] > 0); rcrit scales with the
// cube root of the mass (Hill radius).
__device__ __forceinline__ double grown_mass(const double* __restrict__ growth, int k, double t) {
  const double E = 2.718281828459045235;
  const double tau = growth[3 * k + 2];
  const double m0 = growth[3 * k], mc = growth[3 * k + 1];
  return t >= tau ? mc : m0 + (E / (E - 1.0)) * (mc - m0) * (1.0 - exp(-t / tau));
}

__global__ void k_growth(int nb, double dt, const double* __restrict__ growth,
                         const double* __restrict__ mu_init,
                         const double* __restrict__ rcrit_init, double* __restrict__ mu,
                         double* __restrict__ rcrit, const DevScalars* __restrict__ dsc) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  if (!(growth[3 * k + 2] > 0.0)) return;
  const double m = grown_mass(growth, k, (double)dsc->step * dt);
  mu[k] = m;
  rcrit[k] = rcrit_init[k] * cbrt(m / mu_init[k]);
}

// ------------------------------------------------- time-dependent physics
// Sect. 3.2 (Eqs. 13-16), Sect. 3.3 (Eqs. 17-18), the gaps of Sect. 3.1 (Eqs. 8-9)
// and the step switch of Sect. 3.6, at the start of a step (one wave; n_big <= 64,
// lane k = massive body k).  masses_only: only the masses and changeover radii at
// time t_fix (restarts).  Otherwise at t = the step's start time: masses; the
// massive-body momentum P (summed in index order) for the heliocentric velocities;
// osculating semi-major axes; the step switch; radii; gap records; the migration
// velocity changes (written to u and to the step-start snapshot); the clock
// advanced by the step taken.
__device__ __forceinline__ double planet_radius_core(double gm, double cs, double rhill) {
  return gm / (cs * cs + gm / (0.25 * rhill));  // k1 = 1, k2 = 1/4
}

__global__ __launch_bounds__(64) void k_physics(
    int n, int nb, double G, double mu0, DragConst dc, const PlanetPhys* __restrict__ ph,
    const double* __restrict__ mu_init, const double* __restrict__ rcrit_init,
    double* __restrict__ mu, double* __restrict__ rcrit, const double* __restrict__ x,
    double* __restrict__ u, double* __restrict__ bigsnap, double* __restrict__ radius,
    double* __restrict__ rad_c, double* __restrict__ gaps, DevScalars* __restrict__ dsc,
    SysDesc* __restrict__ desc, double a_switch, double a_min, int masses_only, double t_fix) {
  __shared__ double smu[64 * 3];
  __shared__ double sP[3];
  const int k = threadIdx.x;
  const double t = masses_only ? t_fix : dsc->time;
  PlanetPhys q{};
  if (k < nb) q = ph[k];
  double m_k = 0.0;
  if (k < nb) {
    m_k = mu[k];
    if (q.tau_c > 0.0) {
      const double E = 2.718281828459045235;
      double m;
      if (t < q.tau_c) m = q.M0 + (E / (E - 1.0)) * (q.Mc - q.M0) * (1.0 - exp(-t / q.tau_c));
      else if (q.tau_g > 0.0) m = q.Mc + (q.Mf - q.Mc) * (1.0 - exp(-(t - q.tau_c) / q.tau_g));
      else m = q.Mc;
      m_k = G * m;
      mu[k] = m_k;
      rcrit[k] = rcrit_init[k] * cbrt(m_k / mu_init[k]);
    }
  }
  if (masses_only) return;
  double v[3] = {0.0, 0.0, 0.0}, p[3] = {0.0, 0.0, 0.0};
  if (k < nb) {
    for (int c = 0; c < 3; ++c) {
      p[c] = x[c * n + k];
      v[c] = u[c * n + k];
      smu[3 * k + c] = m_k * v[c];
    }
  }
  __syncthreads();
  if (k == 0) {
    double P0 = 0.0, P1 = 0.0, P2 = 0.0;
    for (int j = 0; j < nb; ++j) {
      P0 += smu[3 * j];
      P1 += smu[3 * j + 1];
      P2 += smu[3 * j + 2];
    }
    sP[0] = P0;
    sP[1] = P1;
    sP[2] = P2;
  }
  __syncthreads();
  double vh[3], ap = 0.0, r = 0.0, Rc = 0.0, vn = 0.0, rh = 0.0;
  bool inside = false;
  const bool migrates = k < nb && (q.tau1 > 0.0 || q.tau2 > 0.0);
  if (k < nb) {
    for (int c = 0; c < 3; ++c) vh[c] = v[c] + sP[c] / mu0;
    r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    Rc = sqrt(p[0] * p[0] + p[1] * p[1]);
    const double vv = vh[0] * vh[0] + vh[1] * vh[1] + vh[2] * vh[2];
    vn = sqrt(vv);
    const double gm = mu0 + m_k;
    ap = gm / (2.0 * gm / r - vv);  // osculating semi-major axis (negative if unbound)
    rh = r * cbrt(m_k / (3.0 * mu0));
    inside = migrates && a_switch > 0.0 && ap > 0.0 && ap <= a_switch;
  }
  const bool any_inside = __builtin_amdgcn_ballot_w64(inside) != 0;
  double h = desc->h;
  if (any_inside && !dsc->switched) {
    h = 2.0 * mxd::kPi * sqrt(a_min * a_min * a_min / mu0) / 25.0;
    if (k == 0) {
      desc->h = h;
      dsc->switched = 1;
    }
  }
  if (k < nb) {
    // radius: Eq. 14 with the disk's sound speed at the cylindrical distance
    const double cs = dc.cs2_1au > 0.0 ? sqrt(dc.cs2_1au * pow(Rc, -dc.beta))
                                       : dc.h_over_r * sqrt(mu0 / Rc);
    if (q.tau_c > 0.0 && q.tau_g > 0.0 && t >= q.tau_c) {
      double R0 = rad_c[k];
      if (R0 == 0.0) {
        R0 = planet_radius_core(m_k, cs, rh);
        rad_c[k] = R0;
      }
      radius[k] = R0 - (R0 - q.R_I) * (1.0 - exp(-(t - q.tau_c) / q.tau_g));
    } else {
      radius[k] = planet_radius_core(m_k, cs, rh);
    }
    // gap (Eqs. 8-9)
    const bool open = q.gap_C > 0.0 && q.tau_c > 0.0 && q.tau_g > 0.0 && t > q.tau_c;
    gaps[4 * k] = Rc;
    gaps[4 * k + 1] = q.gap_C * rh;
    gaps[4 * k + 2] = open ? exp(-(t - q.tau_c) / q.tau_g) : 1.0;
    gaps[4 * k + 3] = open ? 1.0 : 0.0;
    // migration (Eqs. 17-18) along the heliocentric velocity
    if (migrates && ap > 0.0) {
      const double vk = sqrt((mu0 + m_k) / ap);
      const double t1 = q.tau1 > 0.0 ? q.tau1 : 0.0;
      double dv = 0.0;
      if (q.tau1 > 0.0 && t < q.tau1) dv = 0.5 * (q.da1 / ap) * (h / q.tau1) * vk;
      else if (q.tau2 > 0.0) dv = 0.5 * (q.da2 / ap) * (h / q.tau2) * exp(-(t - t1) / q.tau2) * vk;
      for (int c = 0; c < 3; ++c) {
        const double w = v[c] + dv * vh[c] / vn;
        u[c * n + k] = w;
        bigsnap[(3 + c) * nb + k] = w;
      }
    }
  }
  if (k == 0) dsc->time = t + h;
}

// clock restart: time t, the initial step, the step switch undone, R_c forgotten
__global__ void k_physics_reset(int nb, double t, double dt, double* __restrict__ rad_c,
                                DevScalars* __restrict__ dsc, SysDesc* __restrict__ desc) {
  const int k = threadIdx.x;
  if (k < nb) rad_c[k] = 0.0;
  if (k == 0) {
    dsc->time = t;
    dsc->switched = 0;
    desc->h = dt;
  }
}

// ------------------------------------------------- kick + jump + drift
// Growing bodies (k < gpre with growth[3 k + 2] > 0) take their mass at the
// step start here, with k_growth's arithmetic: every block evaluates it for its
// momentum sum, and the owner of the body stores the mass and changeover radius
// (no block reads mu of a growing body, so the store races with nothing).
__global__ __launch_bounds__(kBlock) void k_kick_jump_drift(
    int n, int nb, double mu0, double h, DragConst dc, int gas_on, double* __restrict__ x,
    double* __restrict__ u, const double* __restrict__ ag, double* __restrict__ x0s,
    double* __restrict__ u0s, double* __restrict__ mu, double* __restrict__ rcrit,
    const double* __restrict__ r_p, const double* __restrict__ rho_p,
    FlagSource* __restrict__ fpack, DevScalars* __restrict__ dsc,
    const double* __restrict__ bigsnap, int gpre, const double* __restrict__ growth,
    const double* __restrict__ mu_init, const double* __restrict__ rcrit_init) {
  __shared__ double sh[6 * kBlock];
  const double hh = 0.5 * h;
  const double tg = gpre > 0 ? (double)dsc->step * h : 0.0;
  // massive-body momentum before (drag frame) and after the half kick (jump);
  // big bodies feel no drag, so their kicked velocity is u + hh * ag.
  // (from the step-start snapshot: the blocks that own massive bodies overwrite
  // u while other blocks are still reading)
  double v[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll 4
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    double m;
    if (k < gpre && growth[3 * k + 2] > 0.0) m = grown_mass(growth, k, tg);
    else m = mu[k];
    double ux = bigsnap[3 * nb + k], uy = bigsnap[4 * nb + k], uz = bigsnap[5 * nb + k];
    v[0] += m * ux;
    v[1] += m * uy;
    v[2] += m * uz;
    v[3] += m * (ux + hh * (bigsnap[6 * nb + k] + 0.0));
    v[4] += m * (uy + hh * (bigsnap[7 * nb + k] + 0.0));
    v[5] += m * (uz + hh * (bigsnap[8 * nb + k] + 0.0));
  }
  mxd::block_sum_waves<kBlock, 6>(v, sh);
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  double px = x[t], py = x[n + t], pz = x[2 * n + t];
  double vx = u[t], vy = u[n + t], vz = u[2 * n + t];
  double adx = 0.0, ady = 0.0, adz = 0.0;
  if (t >= nb && gas_on) {
    int j = t - nb;
    mxd::gas_drag(dc, px, py, vx + v[0] / mu0, vy + v[1] / mu0, vz + v[2] / mu0, r_p[j],
                  rho_p[j], adx, ady, adz);
  }
  vx += hh * (ag[t] + adx);
  vy += hh * (ag[n + t] + ady);
  vz += hh * (ag[2 * n + t] + adz);
  px += hh * v[3] / mu0;
  py += hh * v[4] / mu0;
  pz += hh * v[5] / mu0;
  x0s[t] = px; x0s[n + t] = py; x0s[2 * n + t] = pz;
  u0s[t] = vx; u0s[n + t] = vy; u0s[2 * n + t] = vz;
  double qx = px, qy = py, qz = pz, wx = vx, wy = vy, wz = vz;
  if (!mxd::kepler_drift(mu0, h, qx, qy, qz, wx, wy, wz)) atomicOr(&dsc->err, MXE_NOCONV);
  x[t] = qx; x[n + t] = qy; x[2 * n + t] = qz;
  u[t] = wx; u[n + t] = wy; u[2 * n + t] = wz;
  if (t < nb) {
    double rc;
    if (t < gpre && growth[3 * t + 2] > 0.0) {
      const double m = grown_mass(growth, t, tg);
      rc = rcrit_init[t] * cbrt(m / mu_init[t]);
      mu[t] = m;
      rcrit[t] = rc;
    } else {
      rc = rcrit[t];
    }
    FlagSource f;
    f.x0 = px; f.y0 = py; f.z0 = pz; f.u0x = vx; f.u0y = vy; f.u0z = vz;
    f.dx = qx - px; f.dy = qy - py; f.dz = qz - pz;  // displacement over the drift
    f.u1x = wx; f.u1y = wy; f.u1z = wz;
    f.rc = rc;
    f.pad0 = f.pad1 = f.pad2 = 0.0;
    fpack[t] = f;
  }
}

// ------------------------------------------------------------ jump + pack
// x += (h/2) P / mu0 with P over the massive bodies (after the encounter
// integrator); records P for the drag of the closing kick and packs the
// massive bodies for the force sum.  rc2 is floored at 1e-300 so that a body's
// own entry falls in the K = 0 branch.
__global__ __launch_bounds__(kBlock) void k_jump_pack(int n, int nb, double mu0, double hh,
                                                      double* __restrict__ x,
                                                      const double* __restrict__ u,
                                                      const double* __restrict__ mu,
                                                      const double* __restrict__ rcrit,
                                                      KickSource* __restrict__ kpack,
                                                      DevScalars* __restrict__ dsc, int jump) {
  __shared__ double sh[3 * kBlock];
  double v[3] = {0, 0, 0};
#pragma unroll 4
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    double m = mu[k];
    v[0] += m * u[k];
    v[1] += m * u[n + k];
    v[2] += m * u[2 * n + k];
  }
  mxd::block_sum_waves<kBlock, 3>(v, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    dsc->P[0] = v[0];
    dsc->P[1] = v[1];
    dsc->P[2] = v[2];
  }
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  double px = x[t], py = x[n + t], pz = x[2 * n + t];
  if (jump) {
    px += hh * v[0] / mu0;
    py += hh * v[1] / mu0;
    pz += hh * v[2] / mu0;
    x[t] = px; x[n + t] = py; x[2 * n + t] = pz;
  }
  if (t < nb) {
    KickSource k;
    double rc = rcrit[t];
    k.x = px; k.y = py; k.z = pz;
    k.mu = mu[t];
    k.rc2 = fmax(rc * rc, 1e-300);
    k.rc = rc;
    k.pad0 = k.pad1 = 0.0;
    kpack[t] = k;
  }
}

// ------------------------------------------------------------- force + kick
// Each lane holds one target t; the wave walks sources [s0, s1) of its split
// with scalar loads.  Fast branch (s2 >= rc2, K = 1): mu * y^3 with y the
// corrected hardware rsqrt.  Changeover branch (rare, divergent): the quintic K.
// With split > 1 the per-split partial sums go to `part` and a second kernel adds
// them in split order, so the result does not depend on block scheduling and no
// device-wide fence is needed inside the force kernel.
__device__ __forceinline__ void finish_body(int t, int n, int nb, double mu0, double hh,
                                            const DragConst& dc, int gas_on, int kick,
                                            double ax, double ay, double az,
                                            const double* __restrict__ x,
                                            double* __restrict__ u, double* __restrict__ ag,
                                            const double* __restrict__ r_p,
                                            const double* __restrict__ rho_p,
                                            const double* P, int32_t* err,
                                            double* __restrict__ bigsnap) {
  ag[t] = ax; ag[n + t] = ay; ag[2 * n + t] = az;
  double vx = u[t], vy = u[n + t], vz = u[2 * n + t];
  if (!kick) {
    if (t < nb) {
      bigsnap[t] = x[t]; bigsnap[nb + t] = x[n + t]; bigsnap[2 * nb + t] = x[2 * n + t];
      bigsnap[3 * nb + t] = vx; bigsnap[4 * nb + t] = vy; bigsnap[5 * nb + t] = vz;
      bigsnap[6 * nb + t] = ax; bigsnap[7 * nb + t] = ay; bigsnap[8 * nb + t] = az;
    }
    return;
  }
  double adx = 0.0, ady = 0.0, adz = 0.0;
  if (t >= nb && gas_on) {
    int j = t - nb;
    mxd::gas_drag(dc, x[t], x[n + t], vx + P[0] / mu0, vy + P[1] / mu0, vz + P[2] / mu0,
                  r_p[j], rho_p[j], adx, ady, adz);
  }
  vx += hh * (ax + adx);
  vy += hh * (ay + ady);
  vz += hh * (az + adz);
  u[t] = vx; u[n + t] = vy; u[2 * n + t] = vz;
  double chk = vx + vy + vz + x[t] + x[n + t] + x[2 * n + t];
  if (!isfinite(chk)) atomicOr(err, MXE_NONFINITE);
  if (t < nb) {
    bigsnap[t] = x[t]; bigsnap[nb + t] = x[n + t]; bigsnap[2 * nb + t] = x[2 * n + t];
    bigsnap[3 * nb + t] = vx; bigsnap[4 * nb + t] = vy; bigsnap[5 * nb + t] = vz;
    bigsnap[6 * nb + t] = ax; bigsnap[7 * nb + t] = ay; bigsnap[8 * nb + t] = az;
  }
}

// Wide layout (few massive bodies): 256 targets per block, every wave walks
// all sources, and the body is finished in the same kernel.
__global__ __launch_bounds__(kBlock) void k_force_kick(
    int n, int nb, double mu0, double hh, DragConst dc, int gas_on, int kick,
    const double* __restrict__ x, double* __restrict__ u, double* __restrict__ ag,
    const KickSource* __restrict__ kpack, const double* __restrict__ r_p,
    const double* __restrict__ rho_p, DevScalars* __restrict__ dsc,
    double* __restrict__ bigsnap) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int tt = t < n ? t : n - 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (kick) {
      dsc->step += 1;
      dsc->n_pairs[0] = 0;  // the encounter list of this step has been planned
    }
    dsc->plan_ready[0] = 0;  // the in-kernel plan of the next step starts unpublished
  }
  const double xt = x[tt], yt = x[n + tt], zt = x[2 * n + tt];
  double rct = 0.0, rc2t = 0.0;
  if (tt < nb) {
    rct = kpack[tt].rc;
    rc2t = rct * rct;
  }
  double ax, ay, az;
  mxd::force_sum(kpack, 0, nb, xt, yt, zt, rc2t, rct, ax, ay, az);
  double P[3] = {dsc->P[0], dsc->P[1], dsc->P[2]};
  if (t < n) finish_body(t, n, nb, mu0, hh, dc, gas_on, kick, ax, ay, az, x, u, ag, r_p, rho_p, P, &dsc->err, bigsnap);
}

// Symmetric layout of the massive-massive forces (Newton's third law, the
// triangular form of the direct-force routine).  The massive bodies are cut into
// 64-body tiles; one wave takes one tile pair (I, J) with J = (I + d) mod nT,
// d = 0 .. nT/2 (every unordered pair once; d = 0 is the diagonal tile).
// Pass 1: lanes hold the bodies i of I and walk the 64 sources j of J, read with
// wave-uniform (scalar) loads one group of four ahead; they accumulate
// mu_j K/r^3 (x_j - x_i) and store w_ij = mu_i K/r^3 in LDS, 16 sources at a
// time.  Pass 2 after each 16 sources: lane (g, l) sums w_ij (x_i - x_j) for
// source j = l of the chunk over the 16 targets i of group g, and the four
// groups are added across lanes ((g0 + g1) + (g2 + g3)), so the reaction costs
// no second inverse square root.  Diagonal tiles take pass 1 only, self pairs
// excluded.  Rows of 3 x 64 partial sums go to `out` at [I][J] (forces on the
// bodies of I from J) and [J][I]; the finish kernel adds the rows of each tile
// in ascending source tile.  The record array is padded to whole tiles with
// massless bodies far away from everything (see pad_kick_sources), so the loops
// have no bounds.  Each workgroup is one independent wave (no block barrier);
// the 4,004-body kick gives about two waves per SIMD.
constexpr int kSymT = 64;     // bodies per tile
constexpr int kSymC = 16;     // sources per pass-2 chunk
constexpr int kSymS = 65;     // LDS row stride of the weights (odd: no bank conflicts)
constexpr int kSymWaves = 1;  // independent waves per block

struct SymSrc {
  double x, y, z, mu;
};

struct SymLds {                 // one wave's LDS
  double tx[kSymT], ty[kSymT], tz[kSymT];   // positions of the tile I bodies
  double W[kSymC * kSymS];                  // w_ij of one chunk, [j][i]
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ SymSrc sym_src(const KickSource* __restrict__ S, int j) {
  return SymSrc{S[j].x, S[j].y, S[j].z, S[j].mu};
}

// tile pair of work unit u (units nT x (nT/2 + 1)); skip marks the duplicate
// pairs of d = nT/2 for even nT
__device__ __forceinline__ void sym_unit(int u, int nT, int& I, int& J, bool& skip) {
  const int d = u / nT;
  I = u - d * nT;
  J = I + d;
  if (J >= nT) J -= nT;
  skip = 2 * d == nT && 2 * I >= nT;
}

__global__ __launch_bounds__(64 * kSymWaves) void k_force_sym(int nb, int nT, int nunits,
                                                               const KickSource* __restrict__ kp,
                                                               double* __restrict__ out) {
  __shared__ SymLds lds[kSymWaves];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int u = blockIdx.x * kSymWaves + wv;
  if (u >= nunits) return;
  int I, J;
  bool skip;
  sym_unit(u, nT, I, J, skip);
  if (skip) return;
  I = __builtin_amdgcn_readfirstlane(I);
  J = __builtin_amdgcn_readfirstlane(J);
  SymLds& L = lds[wv];
  const int nI = min(kSymT, nb - I * kSymT), nJ = min(kSymT, nb - J * kSymT);
  const KickSource& tk = kp[I * kSymT + lane];
  const double xi = tk.x, yi = tk.y, zi = tk.z, mui = tk.mu, rci = tk.rc, rc2i = rci * rci;
  // wave-uniform bound >= max(rc2) over both tiles: pairs below it take the
  // exact changeover test
  const uint32_t hi = mxd::wave_max_hi(fmax(rc2i, kp[J * kSymT + lane].rc2));
  const double bound = __longlong_as_double((long long)(((uint64_t)hi << 32) | 0xffffffffull));
  L.tx[lane] = xi;
  L.ty[lane] = yi;
  L.tz[lane] = zi;
  double k15, k1875;
  mxd::vgpr_constants(k15, k1875);
  wave_sync();
  const bool diag = I == J;
  const KickSource* __restrict__ S = kp + J * kSymT;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  SymSrc A0 = sym_src(S, 0), A1 = sym_src(S, 1), A2 = sym_src(S, 2), A3 = sym_src(S, 3);
#pragma unroll 1
  for (int j = 0; j < kSymT; j += 4) {
    const int jn = j + 4 < kSymT ? j + 4 : j;
    const SymSrc N0 = sym_src(S, jn), N1 = sym_src(S, jn + 1), N2 = sym_src(S, jn + 2),
                 N3 = sym_src(S, jn + 3);
    const SymSrc Sx[4] = {A0, A1, A2, A3};
    double dx[4], dy[4], dz[4], s2[4], w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      dx[q] = Sx[q].x - xi;
      dy[q] = Sx[q].y - yi;
      dz[q] = Sx[q].z - zi;
      s2[q] = fma(dz[q], dz[q], fma(dy[q], dy[q], dx[q] * dx[q]));
      w[q] = mxd::fast_weight(1.0, s2[q], k15, k1875);
    }
    const uint64_t near = __builtin_amdgcn_ballot_w64(s2[0] < bound) |
                          __builtin_amdgcn_ballot_w64(s2[1] < bound) |
                          __builtin_amdgcn_ballot_w64(s2[2] < bound) |
                          __builtin_amdgcn_ballot_w64(s2[3] < bound);
    if (__builtin_expect(near != 0, 0)) {
      // a self pair (s2 = 0) always lands here
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double rc2 = fmax(S[j + q].rc2, rc2i);
        if (s2[q] < rc2) w[q] = mxd::changeover_weight_slow(s2[q], fmax(S[j + q].rc, rci), rc2);
        if (diag && j + q == lane) w[q] = 0.0;
      }
    }
    const int jw = j & (kSymC - 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double t = Sx[q].mu * w[q];
      a0 = fma(t, dx[q], a0);
      a1 = fma(t, dy[q], a1);
      a2 = fma(t, dz[q], a2);
      L.W[(jw + q) * kSymS + lane] = mui * w[q];
    }
    A0 = N0;
    A1 = N1;
    A2 = N2;
    A3 = N3;
    if (jw + 4 == kSymC && !diag) {
      const int j0 = j + 4 - kSymC;
      wave_sync();
      const int g = lane / kSymC, jl = lane % kSymC;
      const double xj = S[j0 + jl].x, yj = S[j0 + jl].y, zj = S[j0 + jl].z;
      double r0 = 0.0, r1 = 0.0, r2 = 0.0;
#pragma unroll 8
      for (int k = 0; k < kSymC; ++k) {
        const int i = g * kSymC + k;
        const double ww = L.W[jl * kSymS + i];
        r0 = fma(ww, L.tx[i] - xj, r0);
        r1 = fma(ww, L.ty[i] - yj, r1);
        r2 = fma(ww, L.tz[i] - zj, r2);
      }
#pragma unroll
      for (int off = kSymC; off < 64; off <<= 1) {
        r0 += __shfl_xor(r0, off);
        r1 += __shfl_xor(r1, off);
        r2 += __shfl_xor(r2, off);
      }
      if (lane < kSymC && j0 + jl < nJ) {
        double* row = out + ((size_t)J * nT + I) * 3 * kSymT;  // forces on J from I
        row[j0 + jl] = r0;
        row[kSymT + j0 + jl] = r1;
        row[2 * kSymT + j0 + jl] = r2;
      }
      wave_sync();
    }
  }
  if (lane < nI) {
    double* row = out + ((size_t)I * nT + J) * 3 * kSymT;  // forces on I from J
    row[lane] = a0;
    row[kSymT + lane] = a1;
    row[2 * kSymT + lane] = a2;
  }
}

// Padding records of the last tile: massless, far apart from each other and
// from every body, so that they add exactly zero to every sum.
__global__ void k_pad_kick_sources(int nb, int ntot, KickSource* __restrict__ kp) {
  const int t = nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntot) return;
  KickSource k;
  k.x = -1e20 * (double)(1 + (t & (kSymT - 1)));
  k.y = k.z = 0.0;
  k.mu = 0.0;
  k.rc2 = 1e-300;
  k.rc = 0.0;
  k.pad0 = k.pad1 = 0.0;
  kp[t] = k;
}

// Finish.  Massive bodies (blocks < nT, one per tile): 16 slices of the source
// tiles, thread q * 64 + l sums slice q for body l of the tile, then the slices
// are added in order (fixed order: the result does not depend on scheduling).
// Massless bodies (blocks >= nT): the split partials in split order.  Then drag
// and the half kick.
constexpr int kFinSlices = 16;

__global__ __launch_bounds__(64 * kFinSlices) void k_force_finish_sym(
    int n, int nb, int nT, int split, double mu0, double hh, DragConst dc, int gas_on,
    int kick, const double* __restrict__ x, double* __restrict__ u, double* __restrict__ ag,
    const double* __restrict__ r_p, const double* __restrict__ rho_p,
    const double* __restrict__ sym, const double* __restrict__ part,
    DevScalars* __restrict__ dsc, double* __restrict__ bigsnap) {
  __shared__ double sl[kFinSlices][3][kSymT];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (kick) {
      dsc->step += 1;
      dsc->n_pairs[0] = 0;  // the encounter list of this step has been planned
    }
    dsc->plan_ready[0] = 0;  // the in-kernel plan of the next step starts unpublished
  }
  double P[3] = {dsc->P[0], dsc->P[1], dsc->P[2]};
  if ((int)blockIdx.x < nT) {
    const int I = blockIdx.x;
    const int q = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int Ja = (q * nT) / kFinSlices, Jb = ((q + 1) * nT) / kFinSlices;
    const double* row = sym + (size_t)I * nT * 3 * kSymT + l;
    double bx = 0.0, by = 0.0, bz = 0.0;
#pragma unroll 4
    for (int J = Ja; J < Jb; ++J) {
      bx += row[(size_t)J * 3 * kSymT];
      by += row[(size_t)J * 3 * kSymT + kSymT];
      bz += row[(size_t)J * 3 * kSymT + 2 * kSymT];
    }
    sl[q][0][l] = bx;
    sl[q][1][l] = by;
    sl[q][2][l] = bz;
    __syncthreads();
    const int t = I * kSymT + l;
    if (q != 0 || t >= nb) return;
    double a[3];
    for (int c = 0; c < 3; ++c) {
      double s = sl[0][c][l];
      for (int k = 1; k < kFinSlices; ++k) s += sl[k][c][l];
      a[c] = s;
    }
    finish_body(t, n, nb, mu0, hh, dc, gas_on, kick, a[0], a[1], a[2], x, u, ag, r_p, rho_p, P,
                &dsc->err, bigsnap);
    return;
  }
  const int t = nb + ((int)blockIdx.x - nT) * (64 * kFinSlices) + threadIdx.x;
  if (t >= n) return;
  double bx = 0.0, by = 0.0, bz = 0.0;
#pragma unroll 8
  for (int q = 0; q < split; ++q) {
    size_t base = (size_t)q * 3 * n;
    bx += part[base + t];
    by += part[base + n + t];
    bz += part[base + 2 * n + t];
  }
  finish_body(t, n, nb, mu0, hh, dc, gas_on, kick, bx, by, bz, x, u, ag, r_p, rho_p, P, &dsc->err, bigsnap);
}

// split layout for massless targets only (bodies first .. n - 1)
__global__ __launch_bounds__(kBlock) void k_force_split_small(
    int n, int nb, int first, int split, const double* __restrict__ x,
    const KickSource* __restrict__ kpack, double* __restrict__ part) {
  const int tile = blockIdx.x / split;
  const int sp = blockIdx.x - tile * split;
  const int t = first + tile * kBlock + threadIdx.x;
  const int tt = t < n ? t : n - 1;
  const double xt = x[tt], yt = x[n + tt], zt = x[2 * n + tt];
  const int per = (nb + split - 1) / split;
  const int s0 = sp * per;
  const int s1 = min(nb, s0 + per);
  double ax, ay, az;
  mxd::force_sum(kpack, s0, s1, xt, yt, zt, 0.0, 0.0, ax, ay, az);
  if (t < n) {
    size_t base = (size_t)sp * 3 * n;
    part[base + t] = ax;
    part[base + n + t] = ay;
    part[base + 2 * n + t] = az;
  }
}

// stateless gravity (single-kernel entry): packs then sums, no kick
__global__ void k_pack_plain(int n, int nb, const double* __restrict__ x,
                             const double* __restrict__ mu, const double* __restrict__ rcrit,
                             KickSource* __restrict__ kp) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb) return;
  double rc = rcrit[t];
  KickSource k;
  k.x = x[t]; k.y = x[n + t]; k.z = x[2 * n + t];
  k.mu = mu[t];
  k.rc2 = fmax(rc * rc, 1e-300);
  k.rc = rc;
  k.pad0 = k.pad1 = 0.0;
  kp[t] = k;
}

__global__ __launch_bounds__(kBlock) void k_gravity_plain(int n, int nb,
                                                          const double* __restrict__ x,
                                                          const KickSource* __restrict__ kp,
                                                          double* __restrict__ a) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int tt = t < n ? t : n - 1;
  double rct = tt < nb ? kp[tt].rc : 0.0;
  double ax, ay, az;
  mxd::force_sum(kp, 0, nb, x[tt], x[n + tt], x[2 * n + tt], rct * rct, rct, ax, ay, az);
  if (t < n) { a[t] = ax; a[n + t] = ay; a[2 * n + t] = az; }
}

__global__ __launch_bounds__(kBlock) void k_drag_plain(int n, int nb, double mu0, DragConst dc,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ u,
                                                       const double* __restrict__ mu,
                                                       const double* __restrict__ r_p,
                                                       const double* __restrict__ rho_p,
                                                       double* __restrict__ a) {
  __shared__ double sh[3 * kBlock];
  double v[3] = {0, 0, 0};
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    v[0] += mu[k] * u[k];
    v[1] += mu[k] * u[n + k];
    v[2] += mu[k] * u[2 * n + k];
  }
  mxd::block_sum<kBlock, 3>(v, sh);
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  double ax = 0.0, ay = 0.0, az = 0.0;
  if (t >= nb) {
    int j = t - nb;
    mxd::gas_drag(dc, x[t], x[n + t], u[t] + v[0] / mu0, u[n + t] + v[1] / mu0,
                  u[2 * n + t] + v[2] / mu0, r_p[j], rho_p[j], ax, ay, az);
  }
  a[t] = ax; a[n + t] = ay; a[2 * n + t] = az;
}

__global__ __launch_bounds__(kBlock) void k_kepler_plain(int n, double mu0, double h,
                                                         const double* __restrict__ x0,
                                                         const double* __restrict__ u0,
                                                         double* __restrict__ x1,
                                                         double* __restrict__ u1,
                                                         int32_t* __restrict__ err) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  double px = x0[t], py = x0[n + t], pz = x0[2 * n + t];
  double vx = u0[t], vy = u0[n + t], vz = u0[2 * n + t];
  if (!mxd::kepler_drift(mu0, h, px, py, pz, vx, vy, vz)) atomicOr(err, MXE_NOCONV);
  x1[t] = px; x1[n + t] = py; x1[2 * n + t] = pz;
  u1[t] = vx; u1[n + t] = vy; u1[2 * n + t] = vz;
}

int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }

}  // namespace

namespace mxk {

// Source split of the force kernel: with at least 128 massive bodies the force
// runs in the split layout, with enough blocks to give every SIMD about four
// waves (256 CUs x 4 SIMDs) and at least 32 sources per split; 1 selects the
// wide layout.
int force_split(int n, int nb) {
  if (nb < 128) return 1;
  int tiles = blocks_for(n);
  int split = (1024 + tiles - 1) / tiles;
  int maxs = nb / 32;
  if (split > maxs) split = maxs;
  if (split > 64) split = 64;
  if (split < 1) split = 1;
  return split;
}

hipError_t launch_growth(mx_system* s) {
  if (!s->has_growth || s->nb == 0) return hipSuccess;
  return mxlaunch(s, k_growth, dim3((s->nb + 255) / 256), dim3(256), s->nb, s->p.dt,
                  s->growth, s->mu_init, s->rcrit_init, s->mu, s->rcrit, s->dsc);
}

hipError_t launch_physics_reset(mx_system* s, double t) {
  if (!s->has_phys) return hipSuccess;
  return mxlaunch(s, k_physics_reset, dim3(1), dim3(64), s->nb, t, s->p.dt, s->rad_c, s->dsc,
                  s->desc);
}

hipError_t launch_physics(mx_system* s, int masses_only, double t) {
  if (!s->has_phys) return hipSuccess;
  return mxlaunch(s, k_physics, dim3(1), dim3(64), s->n, s->nb, s->p.G, s->mu0,
                  make_drag_const(s->p), s->phys, s->mu_init, s->rcrit_init, s->mu, s->rcrit, s->x,
                  s->u, s->bigsnap, s->radius, s->rad_c, s->gaps, s->dsc, s->desc, s->a_switch,
                  s->a_min, masses_only, t);
}

hipError_t launch_kick_jump_drift(mx_system* s) {
  DragConst dc = make_drag_const(s->p);
  return mxlaunch(s, k_kick_jump_drift, dim3(blocks_for(s->n)), dim3(kBlock), s->n,
                  s->nb, s->mu0, s->p.dt, dc, s->p.gas_on, s->x, s->u, s->ag, s->x0, s->u0,
                  s->mu, s->rcrit, s->r_p, s->rho_p, s->fpack, s->dsc, s->bigsnap,
                  s->has_growth ? s->growth_prefix : 0, s->growth, s->mu_init, s->rcrit_init);
}

hipError_t launch_jump_pack(mx_system* s) {
  return mxlaunch(s, k_jump_pack, dim3(blocks_for(s->n)), dim3(kBlock), s->n, s->nb,
                  s->mu0, 0.5 * s->p.dt, s->x, s->u, s->mu, s->rcrit, s->kpack, s->dsc, 1);
}

hipError_t launch_pack_only(mx_system* s) {
  return mxlaunch(s, k_jump_pack, dim3(blocks_for(s->n)), dim3(kBlock), s->n, s->nb,
                  s->mu0, 0.0, s->x, s->u, s->mu, s->rcrit, s->kpack, s->dsc, 0);
}

hipError_t launch_force_kick(mx_system* s, int kick) {
  DragConst dc = make_drag_const(s->p);
  const double hh = 0.5 * s->p.dt;
  if (!s->use_sym)
    return mxlaunch(s, k_force_kick, dim3(blocks_for(s->n)), dim3(kBlock), s->n, s->nb, s->mu0,
                    hh, dc, s->p.gas_on, kick, s->x, s->u, s->ag, s->kpack, s->r_p, s->rho_p,
                    s->dsc, s->bigsnap);
  // massive-massive block by symmetric tile pairs, massless targets by the split
  const int nT = (s->nb + kSymT - 1) / kSymT;
  const int nunits = nT * (nT / 2 + 1);
  hipError_t e = mxlaunch(s, k_force_sym, dim3((nunits + kSymWaves - 1) / kSymWaves),
                          dim3(64 * kSymWaves), s->nb, nT, nunits, s->kpack, s->sympart);
  if (e != hipSuccess) return e;
  if (s->ns > 0) {
    e = mxlaunch(s, k_force_split_small, dim3(blocks_for(s->ns) * s->split), dim3(kBlock), s->n,
                 s->nb, s->nb, s->split, s->x, s->kpack, s->part);
    if (e != hipSuccess) return e;
  }
  return mxlaunch(s, k_force_finish_sym,
                  dim3(nT + (s->ns + 64 * kFinSlices - 1) / (64 * kFinSlices)),
                  dim3(64 * kFinSlices), s->n, s->nb, nT, s->split, s->mu0, hh, dc, s->p.gas_on,
                  kick, s->x, s->u, s->ag, s->r_p, s->rho_p, s->sympart, s->part, s->dsc,
                  s->bigsnap);
}

// Padding records [nb, kick_source_count(nb)) written once at initialisation.
int kick_source_count(int nb) { return ((nb + kSymT - 1) / kSymT) * kSymT; }

hipError_t pad_kick_sources(int nb, KickSource* kp, hipStream_t st) {
  const int ntot = kick_source_count(nb);
  if (ntot == nb) return hipSuccess;
  hipLaunchKernelGGL(k_pad_kick_sources, dim3(1), dim3(kSymT), 0, st, nb, ntot, kp);
  return hipGetLastError();
}

hipError_t gravity(int n, int nb, const double* x, const double* mu, const double* rcrit,
                   double* a, hipStream_t st) {
  KickSource* kp = nullptr;
  hipError_t e = hipMalloc((void**)&kp, sizeof(KickSource) * (nb > 0 ? nb : 1));
  if (e != hipSuccess) return e;
  if (nb > 0)
    hipLaunchKernelGGL(k_pack_plain, dim3((nb + 255) / 256), dim3(256), 0, st, n, nb, x, mu,
                       rcrit, kp);
  hipLaunchKernelGGL(k_gravity_plain, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, nb, x, kp, a);
  e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFree(kp);
  return e != hipSuccess ? e : e2;
}

hipError_t gas_drag(const mx_params* p, int n, int nb, const double* x, const double* u,
                    const double* mu, const double* r_p, const double* rho_p, double* a,
                    hipStream_t st) {
  DragConst dc = make_drag_const(*p);
  hipLaunchKernelGGL(k_drag_plain, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, nb, p->G * p->m0,
                     dc, x, u, mu, r_p, rho_p, a);
  return hipGetLastError();
}

hipError_t kepler(int n, double mu0, double h, const double* x0, const double* u0, double* x1,
                  double* u1, int32_t* err, hipStream_t st) {
  hipLaunchKernelGGL(k_kepler_plain, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, mu0, h, x0, u0,
                     x1, u1, err);
  return hipGetLastError();
}

}  // namespace mxk
