// Internal layout of an mx_system and the host-side launchers of its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <hip/hip_ext.h>
#include <math.h>
#include <stdint.h>

#include "../../include/mx.h"

// Latched device failure bits (OR-ed by kernels into mx_system::d_err).
enum : int32_t {
  MXE_NOCONV = 1,      // Kepler iteration did not converge
  MXE_BS = 2,          // Bulirsch-Stoer halving limit
  MXE_PAIRS = 4,       // more flagged pairs than the list holds
  MXE_SUBSYS = 8,      // a subsystem larger than the encounter integrator holds
  MXE_NONFINITE = 16,  // non-finite state after a step
  MXE_ADJOINT = 32,    // a subsystem beyond what the adjoint handles
  MXE_PLANWAIT = 64,   // a block of the encounter integrator gave up waiting for the plan
};

// Systems with at most this many massive bodies use the fused small-B kernels.
constexpr int kSmallBig = 64;

// Encounter-integrator capacity (members and pairs of one subsystem).
constexpr int kBsMaxMembers = 16;
constexpr int kBsMaxPairs = 48;
constexpr int kBsColumns = 8;   // substep sequence n = 2, 4, ..., 16
constexpr int kBsMaxSched = 64; // accepted steps of one subsystem kept for the adjoint

// Packed source records read with scalar (wave-uniform) loads.
struct __align__(64) KickSource {   // one massive body at kick time
  double x, y, z, mu, rc2, rc, pad0, pad1;
};
struct __align__(128) FlagSource {  // one massive body over a drift
  double x0, y0, z0, u0x, u0y, u0z;   // pre-drift state
  double dx, dy, dz;                  // displacement x1 - x0 over the drift
  double u1x, u1y, u1z;               // post-drift velocity
  double rc, pad0, pad1, pad2;
};

// Per 64-body chunk of the culled encounter test (massive-only systems, bodies in
// the order flag_perm): range of the bodies' distances from the star at the step
// start, the largest reach |Delta|_inf + (4/27) h (|u0|_inf + |u1|_inf) over the
// drift, the largest changeover radius.
struct ChunkBound {
  double rmin, rmax, reach, rc;
};

struct Subsystem {                  // one Bulirsch-Stoer subsystem
  int32_t m, keep_from, np;
  int32_t jm;  // general plan: the massless body a subsystem was built for (else 0)
  int32_t mem[kBsMaxMembers];
  int32_t pl[kBsMaxPairs][2];
};

// Device scalars of a system (one allocation).
// Per-step flags and counters come in three copies indexed by the step phase:
// consecutive steps of a joined sequence use alternating (two-step joins) or
// rotating (joint launches, which run the encounter integrator of step q beside
// the opening of step q + 1) copies, so that no launch clears or appends to a
// copy that another part of the same launch still reads.  Outside joined
// launches the phase is 0.
struct DevScalars {
  int64_t step;          // step counter (t = step * dt)
  int32_t n_pairs[3];    // pairs flagged so far in the step of each phase (append counters)
  int32_t n_sub;         // subsystems of the current step
  int32_t err;           // latched failure bits
  int32_t n_pairs_last;  // flagged pairs of the last completed step
  double P[3];           // massive-body momentum sum mu*u after the last jump
  unsigned long long bs_flop;        // cumulative model FP64 ops of the encounter integrator
  unsigned long long pairs_flagged;  // cumulative flagged pairs
  int32_t plan_ready[3];  // set when the in-kernel general plan of the step is written
  int32_t bn_valid[3];    // BigNext[phase] holds the step boundary's massive bodies
  int32_t bs_done[3];     // joint launches: encounter-integrator blocks finished
  int32_t n_jsub[3];      // joint launches: subsystem records appended for the step
  double time;           // time at the start of the next step (time-dependent physics)
  int32_t switched;      // the step switch has happened
  int32_t pad_phys;
  int32_t joint_runs;    // joint launches since the host last looked
  int32_t joint_slow;    // of which the tiles waited for the integrator
};

// Append counter of the flagged list for step phase w (0 outside joined launches).
__host__ __device__ inline int32_t* pair_counter(DevScalars* d, int w) { return &d->n_pairs[w]; }

namespace mxd {
// Gas-disk constants of a parameter set in the units of the drag formula.
struct DragConst {
  double mu0, sigma1_unit, gamma, r_c, inv_rc, r_in, h_over_r, vg_fac, kexp, mfp_coef;
  double rc_norm;  // (1/r_c)^(2-gamma), the normalisation of the taper at 1 AU
  double rho_fac;  // 1 / (sqrt(2 pi) H/r): midplane density = Sigma / R * rho_fac
  double re_fac;   // 6 / (sqrt(8/pi) mfp_coef): Re = re_fac r_p dv rho_g / c_s
  // disk model beyond the constant aspect ratio (ext != 0)
  double cs2_1au;   // c_s^2 at 1 AU from the temperature (0: c_s = h_over_r v_K)
  double beta;      // temperature slope
  double eta;       // fixed eta
  double eta6_fac;  // (gamma + beta/2 + 3/2) / (2 gamma_C), or 0 for the fixed eta
  double dg_fac;    // disk gravity per unit Sigma: 2 pi G S(gamma), or 2 pi G r_in / R
                    // per unit Sigma / R for gamma = 1; 0 = off
  const double* gaps;  // [gap_n][4] centre R, half width, density factor, open (device)
  int gap_n;
  int ext, dg_edge;
};

// S(gamma) of the disk-gravity series of Eq. 10 through its closed form for a
// power-law disk, -Gamma((1+g)/2) Gamma(1-g/2) / (Gamma(g/2) Gamma((3-g)/2)),
// valid for 0 < g < 2.
inline double dg_series_closed(double g) {
  return -std::tgamma(0.5 * (1.0 + g)) * std::tgamma(1.0 - 0.5 * g) /
         (std::tgamma(0.5 * g) * std::tgamma(0.5 * (3.0 - g)));
}

// Drag constants of a parameter set (host side).
inline DragConst make_drag_const(const mx_params& p) {
  DragConst c;
  const double kTwoPi = 6.283185307179586;
  c.cs2_1au = p.temp_1au > 0.0 ? p.cs2_per_k * p.temp_1au : 0.0;
  c.beta = p.temp_beta;
  c.eta = p.eta;
  c.eta6_fac = p.eta_mode ? (p.gamma + 0.5 * p.temp_beta + 1.5) / (2.0 * 1.4) : 0.0;
  c.dg_edge = p.dg_mode && p.gamma == 1.0;
  c.dg_fac = !p.dg_mode ? 0.0 : (c.dg_edge ? kTwoPi * p.G * p.r_in
                                          : kTwoPi * p.G * dg_series_closed(p.gamma));
  c.ext = (c.cs2_1au > 0.0 || p.eta_mode || p.dg_mode) ? 1 : 0;
  c.gaps = nullptr;
  c.gap_n = 0;
  c.mu0 = p.G * p.m0;
  c.sigma1_unit = p.sigma1 * (p.rho_unit / p.au_cm);
  c.gamma = p.gamma;
  c.r_c = p.r_c;
  c.inv_rc = p.r_c > 0.0 ? 1.0 / p.r_c : 0.0;
  c.r_in = p.r_in;
  c.h_over_r = p.h_over_r;
  c.vg_fac = sqrt(1.0 - 2.0 * p.eta);
  c.kexp = p.kdrag_exp;
  c.mfp_coef = p.mfp_coef;
  c.rc_norm = p.r_c > 0.0 ? pow(1.0 / p.r_c, 2.0 - p.gamma) : 0.0;
  c.rho_fac = 1.0 / (2.5066282746310002 * p.h_over_r);
  c.re_fac = 6.0 / (1.5957691216057308 * p.mfp_coef);
  return c;
}
}  // namespace mxd

// The massive bodies at a joined step boundary (closing step n, opening step
// n + 1), precomputed when the encounter integrator of step n leaves them
// unchanged (by that integrator, or by the launch that opened step n); the
// kernel that closes step n then reads them instead of computing them.
struct BigNext {
  double P[3], J[3], vpre[3], Ppre[3], Ppost[3], pad;
  KickSource src[kSmallBig];
  double bst[12][kSmallBig];
  double brc[kSmallBig];
};

// Joint launches: the subsystem of one flagged massless body j, recorded by the
// launch that flags it (its massive partners as a bit mask, its pre-drift state),
// so that the encounter integrator of the next launch starts from one record.
struct JointSub {
  uint64_t mask;  // massive partners, bit i for massive body i
  int32_t j, pad;
  double x[3], v[3];
  double rp, rhop;  // radius and density of the body (gas drag)
};

// Device view of one system for the kernels that step one or many systems per
// launch (fused small-B step, planner, encounter integrator).  All pointers are
// device pointers into the system's own allocations; the state is SoA [3][n].
struct SysDesc {
  double *x, *u, *ag, *x0, *u0;
  const double *mu, *rcrit;         // [nb]
  const double *r_p, *rho_p;        // [n - nb]
  double *bigsnap, *bigmid;         // [9][nb], [3][6][nb] (by step phase)
  double* bigpre;                   // [3][6][nb]: pre-drift x, u of the massive bodies (by phase)
  BigNext* bignext;                 // [3] (by step phase)
  int32_t* pairs;                   // [lists][cap_pairs][2]: flagged list (joint launches: by phase)
  JointSub* jsub;                   // [3][cap_subs] (by step phase), single systems with n_big <= 64
  int64_t* keys;                    // planner scratch [2 * cap_pairs]
  int32_t* plan_idx;                // planner scratch [2 * cap_pairs]
  int32_t* uf;                      // [2 * nb] union-find scratch
  Subsystem* subs;                  // [cap_subs]
  DevScalars* dsc;
  // accepted Bulirsch-Stoer steps of each subsystem of the step, for the adjoint
  // (null when not recorded): bs_sched[(b * kBsMaxSched + q) * 2 + {0,1}] = (H,
  // accepted column) of the q-th accepted step of subsystem b; bs_nsched[b] count
  double* bs_sched;
  int32_t* bs_nsched;
  mxd::DragConst dc;
  double mu0, h, bs_tol;
  int32_t n, nb, cap_pairs, cap_subs, gas_on;
  // 1: the fused step keeps the pre-drift state of every body in x0, u0 (the
  // adjoint records it); 0: only of the massive and the flagged bodies, the
  // ones the encounter integrator starts from
  int32_t keep_x0;
};

// Global-memory view of a device pointer.  Pointers read from a descriptor
// table are generic, and accesses through them compile to flat instructions
// (which also hold the LDS counter); through this view they compile to global
// loads and stores.
template <class T>
using gmem = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gmem<T> gbl(T* p) {
  return (gmem<T>)p;
}

// A tile of consecutive bodies of one system for the fused small-B kernels.
struct Tile {
  int32_t sys, first;
};

// Kernel timing of one kernel group (eager launches only, never under
// capture): the next kernel launched while armed records `start` at its start,
// which is then cleared; every kernel launched while armed records `stop` at
// its end.
struct LaunchTiming {
  bool armed;
  hipEvent_t start, stop;
};

// Time-dependent physics of one massive body (the mx_planet fields).
struct PlanetPhys {
  double M0, Mc, tau_c, Mf, tau_g, R_I, da1, tau1, da2, tau2, gap_C;
};

struct mx_system {
  mx_params p;
  int n, nb, ns;
  double mu0;
  hipStream_t stream;
  bool own_stream;
  // state, [3][n] SoA
  double *x, *u, *ag, *x0, *u0;
  // massive bodies
  double *mu, *rcrit, *mu_init, *rcrit_init, *growth;  // growth: [nb][3] (G*M0, G*Mc, tau)
  int has_growth;
  int growth_prefix;  // 1 + the largest index of a growing body (0: none)
  // time-dependent physics (mx_set_planet_physics): per-body parameters, radius,
  // radius at the onset of the runaway, gap records [nb][4]
  PlanetPhys* phys;
  double *radius, *rad_c, *gaps;
  int has_phys, any_gap;
  double a_switch, a_min;
  // body removal: status [n] (0, -2, -3), radial direction at the previous check
  // [n] (-1, +1, 0), counter of flagged bodies, momentum scratch [3]
  int32_t* stat;
  int8_t* rsign;
  int32_t* ejcount;
  double* rm_P;
  // snapshots of the massive bodies, so that a kernel whose every block reads
  // them never sees them half-updated by the block that owns them:
  //   bigsnap [9][nb]: x, u, a at the step start (written at the end of a step)
  //   bigmid  [3][6][nb]: x, u after drift and encounter integration (fused path,
  //           by step phase)
  //   bigpre  [3][6][nb]: x, u before the drift (joint launches, by step phase)
  double *bigsnap, *bigmid, *bigpre;
  BigNext* bignext;  // [3]: precomputed massive bodies of a joined step boundary
  // massless bodies
  double *r_p, *rho_p;  // rho_p in Msun/AU^3
  // packed sources
  KickSource* kpack;
  FlagSource* fpack;
  int32_t* flag_perm;     // [nb] body order of the culled encounter test (massive-only systems), or null
  ChunkBound* flag_bounds;  // [ceil(nb / 64)] per-chunk bounds of the culled encounter test
  // force partials: split sums of the massless targets, symmetric tile-pair rows
  // of the massive-massive block (n_big >= 128)
  double* part;
  double* sympart;
  int split;
  int use_sym;
  // encounters
  int32_t* pairs;      // [3][cap][2] (lists by step phase in joint launches)
  Tile* tiles64;       // 64-body tiles of the joint launch
  int32_t n_tiles64;
  JointSub* jsub;      // [3][cap_subs] subsystem records of joint launches (0 < n_big <= 64)
  int32_t last_list;   // phase of the list of the last completed step
  int32_t* pairs_tmp;  // [4*cap] int32 = [2*cap] int64 sort keys of the planner
  int32_t* plan_idx;   // [2*cap] index lists of the planner
  int32_t cap_pairs;
  Subsystem* subs;
  int32_t cap_subs;
  int32_t* uf;         // [nb] union-find scratch
  DevScalars* dsc;
  // energy scratch
  double* red;
  int red_blocks;
  // graph of one step
  hipGraphExec_t graph;
  bool graph_ok;
  bool no_joint;  // steps of a call are never joint (the adjoint records per-step tapes)
  // joint launches switched off for a while: in a system whose massive bodies
  // meet often, the tiles wait for the integrator in most steps and two launches
  // per step are faster
  bool joint_off;
  int64_t joint_retry_at;  // host step from which joint launches are tried again
  int launch_mode;  // MX_LAUNCH_EAGER or MX_LAUNCH_GRAPH
  LaunchTiming tev;
  hipEvent_t* tev_pool;  // events of mx_step_timed, kept between calls
  int32_t tev_pool_n;
  // one-entry device view and the tile table of the fused small-B kernels
  SysDesc* desc;
  Tile* tiles;
  int32_t n_tiles;
  bool owned;  // owned by a batch or an adjoint: mx_destroy leaves it alone
  int64_t host_step;
};

// Launch on a stream with optional kernel timing (see LaunchTiming).
template <typename... KArgs, typename... Args>
inline hipError_t mxlaunch_on(hipStream_t st, LaunchTiming* tm, void (*k)(KArgs...), dim3 grid,
                              dim3 block, Args... args) {
  if (tm && tm->armed) {
    hipExtLaunchKernelGGL(k, grid, block, 0, st, tm->start, tm->stop, 0,
                          static_cast<KArgs>(args)...);
    tm->start = nullptr;
  } else {
    k<<<grid, block, 0, st>>>(static_cast<KArgs>(args)...);
  }
  return hipGetLastError();
}

// Launch on the system's stream with the system's kernel timing.
template <typename... KArgs, typename... Args>
inline hipError_t mxlaunch(mx_system* s, void (*k)(KArgs...), dim3 grid, dim3 block,
                           Args... args) {
  return mxlaunch_on(s->stream, &s->tev, k, grid, block, args...);
}

// ---- launchers (kernels_*.hip)
namespace mxk {
hipError_t launch_growth(mx_system* s);
hipError_t launch_kick_jump_drift(mx_system* s);
hipError_t launch_flag(mx_system* s);
hipError_t launch_jump_pack(mx_system* s);
hipError_t launch_force_kick(mx_system* s, int kick);
hipError_t launch_pack_only(mx_system* s);
hipError_t launch_energy(mx_system* s, double* out7);  // device [7] out
hipError_t launch_h2dh(mx_system* s, const double* v_h);
hipError_t launch_dh2h(mx_system* s, double* v_h);
hipError_t launch_init_bodies(mx_system* s, const double* x_h, const double* v_h);
hipError_t launch_reset_scalars(mx_system* s, int64_t step);
hipError_t launch_physics(mx_system* s, int masses_only, double t);
hipError_t launch_physics_reset(mx_system* s, double t);
hipError_t launch_check_removal(mx_system* s, double r_cen);
hipError_t compact_bodies(mx_system* s, int32_t* n_new, int32_t* map_dev);
// fused small-B kernels over a tile table (n_big <= kSmallBig in every system);
// blk bodies per tile (64, 128, 256 or 512), tpb consecutive tiles per block
// joint != 0: the first launch of a joint sequence (single system, blk 256)
hipError_t launch_step_a_tiles(hipStream_t st, LaunchTiming* tm, const SysDesc* desc,
                               const Tile* tiles, int n_tiles, int blk, int tpb, int par,
                               int joint = 0);
hipError_t launch_step_b_tiles(hipStream_t st, LaunchTiming* tm, const SysDesc* desc,
                               const Tile* tiles, int n_tiles, int blk, int tpb, int kick,
                               int par);
// k_step_b (with kick) of one step joined with k_step_a of the next.  par: the
// step parity (0 outside joined sequences): selects the bigmid buffer and the
// append counter of the flagged list; the joined kernel reads parity par and
// writes par ^ 1.
hipError_t launch_step_ba_tiles(hipStream_t st, LaunchTiming* tm, const SysDesc* desc,
                                const Tile* tiles, int n_tiles, int blk, int tpb, int par);
// planner (one block per system) and encounter integrator (bps blocks per system;
// plan != 0: the integrator plans its subsystems itself, systems of n_big <= 64)
hipError_t launch_bs_sys(hipStream_t st, LaunchTiming* tm, const SysDesc* desc, int n_sys,
                         int bps, int plan, int par, int lst, int clr);
// encounter integrator of step q (phase ph, nbs one-wave blocks per system) beside
// the closing of step q and the opening of step q + 1 over a table of 64-body tiles
hipError_t launch_step_joint(hipStream_t st, LaunchTiming* tm, const SysDesc* desc,
                             const Tile* tiles64, int n_tiles64, int nbs, int n_sys, int ph);

// stateless single-kernel launchers
hipError_t gravity(int n, int nb, const double* x, const double* mu, const double* rcrit,
                   double* a, hipStream_t st);
hipError_t gas_drag(const mx_params* p, int n, int nb, const double* x, const double* u,
                    const double* mu, const double* r_p, const double* rho_p, double* a,
                    hipStream_t st);
hipError_t kepler(int n, double mu0, double h, const double* x0, const double* u0, double* x1,
                  double* u1, int32_t* err, hipStream_t st);
hipError_t flag_pairs(int n, int nb, const double* rcrit, const double* x0, const double* u0,
                      const double* x1, const double* u1, double h, int32_t* pairs,
                      int32_t* pairs_tmp, int32_t cap, DevScalars* dsc, hipStream_t st);
hipError_t flag_pairs_enqueue(int n, int nb, const double* rcrit, const double* x0,
                              const double* u0, const double* x1, const double* u1, double h,
                              int32_t* pairs, int32_t* pairs_tmp, int32_t cap, DevScalars* dsc,
                              FlagSource* fp, hipStream_t st);
}  // namespace mxk
