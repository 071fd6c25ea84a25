// Host side of the C ABI declared in include/mx.h.
//
// A system owns all of its device memory (allocated once at init, freed at
// destroy; nothing is allocated per step).  One hybrid step is the kernel
// sequence
//   [growth] -> kick_jump_drift -> flag -> plan -> BS -> jump_pack -> force_kick
// on the system's stream (with n_big <= 64 the fused small-B kernels replace
// kick_jump_drift + flag and jump_pack + force_kick).  Steps are launched kernel
// by kernel, or, in graph mode, captured once into a HIP graph that is replayed
// for every step.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>

#include <algorithm>
#include <mutex>
#include <vector>

#include "mx_internal.h"

namespace mxk {
int force_split(int n, int nb);
int kick_source_count(int nb);
hipError_t pad_kick_sources(int nb, KickSource* kp, hipStream_t st);
}

namespace {

thread_local std::string g_err;

mx_status fail(mx_status st, const char* msg) {
  g_err = msg;
  return st;
}

mx_status hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return MX_EHIP;
}

#define HIPCHK(expr, where)                      \
  do {                                           \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) return hip_fail(_e, where); \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, sizeof(T) * count);
}

hipError_t copy_in(void* dst, const void* src, size_t bytes, int is_dev, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  return hipMemcpyAsync(dst, src, bytes, is_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        st);
}

hipError_t copy_out(void* dst, const void* src, size_t bytes, int is_dev, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  return hipMemcpyAsync(dst, src, bytes, is_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        st);
}

constexpr int kTileBlk = 256;   // bodies per tile of a single system's fused kernels
constexpr int kBsBlocks = 512;  // encounter-integrator blocks of a single system
constexpr int kJointBs = 128;   // integrator blocks of a single system's joint launch

SysDesc make_desc(const mx_system* s) {
  SysDesc d;
  std::memset((void*)&d, 0, sizeof(d));
  d.x = s->x;
  d.u = s->u;
  d.ag = s->ag;
  d.x0 = s->x0;
  d.u0 = s->u0;
  d.mu = s->mu;
  d.rcrit = s->rcrit;
  d.r_p = s->r_p;
  d.rho_p = s->rho_p;
  d.bigsnap = s->bigsnap;
  d.bigmid = s->bigmid;
  d.bigpre = s->bigpre;
  d.bignext = s->bignext;
  d.pairs = s->pairs;
  d.jsub = s->jsub;
  d.keys = reinterpret_cast<int64_t*>(s->pairs_tmp);
  d.plan_idx = s->plan_idx;
  d.uf = s->uf;
  d.subs = s->subs;
  d.dsc = s->dsc;
  d.dc = mxd::make_drag_const(s->p);
  if (s->has_phys && s->any_gap) {
    d.dc.gaps = s->gaps;
    d.dc.gap_n = s->nb;
    d.dc.ext = 1;
  }
  d.mu0 = s->mu0;
  d.h = s->p.dt;
  d.bs_tol = s->p.bs_tol;
  d.n = s->n;
  d.nb = s->nb;
  d.cap_pairs = s->cap_pairs;
  d.cap_subs = s->cap_subs;
  d.gas_on = s->p.gas_on;
  return d;
}

// tiles of blk consecutive bodies of system `sys` (n bodies), appended to out
void append_tiles(std::vector<Tile>& out, int sys, int n, int blk) {
  for (int f = 0; f < n; f += blk) out.push_back(Tile{sys, f});
}

void free_system(mx_system* s) {
  if (!s) return;
  if (s->graph_ok) (void)hipGraphExecDestroy(s->graph);
  for (int32_t k = 0; k < s->tev_pool_n; ++k) (void)hipEventDestroy(s->tev_pool[k]);
  delete[] s->tev_pool;
  void* ptrs[] = {s->x, s->u, s->ag, s->x0, s->u0, s->mu, s->rcrit, s->mu_init, s->rcrit_init,
                  s->growth, s->r_p, s->rho_p, s->bigsnap, s->bigmid, s->bigpre, s->bignext, s->kpack,
                  s->fpack, s->flag_perm, s->flag_bounds, s->part,
                  s->sympart,
                  s->pairs, s->jsub, s->tiles64, s->pairs_tmp, s->plan_idx, s->subs, s->uf, s->dsc, s->red,
                  s->desc, s->tiles, s->phys, s->radius, s->rad_c, s->gaps, s->stat,
                  s->rsign, s->ejcount, s->rm_P};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete s;
}

// kernel group k of one step (MX_K_* order); the fused small-B path runs its
// flagging inside the first kernel and its jump inside the last.  par: the step
// parity inside a joined sequence (0 otherwise).
hipError_t launch_group(mx_system* s, int k, int par = 0) {
  const bool small = s->nb <= kSmallBig;
  switch (k) {
    case MX_K_GROWTH:  // n_big > 64: the masses grow inside the next group's kernel
      return s->has_phys ? mxk::launch_physics(s, 0, 0.0)
                         : small ? mxk::launch_growth(s) : hipSuccess;
    case MX_K_KICK_JUMP_DRIFT:
      return small ? mxk::launch_step_a_tiles(s->stream, &s->tev, s->desc, s->tiles, s->n_tiles,
                                              kTileBlk, 1, par)
                   : mxk::launch_kick_jump_drift(s);
    case MX_K_FLAG: return small ? hipSuccess : mxk::launch_flag(s);
    case MX_K_PLAN:  // the encounter integrator plans its subsystems itself
      return hipSuccess;
    case MX_K_BS:
      return s->nb > 0 ? mxk::launch_bs_sys(s->stream, &s->tev, s->desc, 1, kBsBlocks, 1, par, 0,
                                            par ^ 1)
                       : hipSuccess;
    case MX_K_JUMP_PACK: return small ? hipSuccess : mxk::launch_jump_pack(s);
    default:
      return small ? mxk::launch_step_b_tiles(s->stream, &s->tev, s->desc, s->tiles, s->n_tiles,
                                              kTileBlk, 1, 1, par)
                   : mxk::launch_force_kick(s, 1);
  }
}

hipError_t enqueue_step(mx_system* s) {
  s->last_list = 0;
  for (int k = 0; k < MX_NUM_KERNELS; ++k) {
    hipError_t e = launch_group(s, k);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// n steps launched eagerly.  On the fused path without growth the closing kernel
// of a step and the opening kernel of the next one run as one launch
// (k_step_ba), the same operations per body.  visit(k, q) runs before the launch
// of group k of step q (the joined launch is visited as the closing group of its
// first step) and after(k, q) right after it.
// whether a call of n steps joins the closing and opening kernels of its steps
bool joinable(const mx_system* s, int32_t n) {
  return n >= 2 && s->nb <= kSmallBig && !s->has_growth && !s->has_phys;
}

// whether a call of n steps runs as a joint sequence: the first step opened by
// k_step_a, then one launch per step that integrates its encounters beside the
// closing of that step and the opening of the next (k_step_joint), the last
// step's encounters and closing as usual
bool joint_ok(const mx_system* s, int32_t n) {
  return joinable(s, n) && s->nb > 0 && s->n < (1 << 26) && !s->no_joint &&
         (!s->joint_off || s->host_step >= s->joint_retry_at);
}

// n >= 2 steps as a joint sequence; visit/after as for enqueue_steps, the joint
// launch visited as MX_K_STEP_JOINT of the step whose encounters it integrates
template <class Visit, class After>
hipError_t enqueue_joint(mx_system* s, int32_t n, Visit visit, After after) {
  hipError_t e;
  visit(MX_K_KICK_JUMP_DRIFT, 0);
  e = mxk::launch_step_a_tiles(s->stream, &s->tev, s->desc, s->tiles, s->n_tiles, kTileBlk, 1, 0,
                               1);
  after(MX_K_KICK_JUMP_DRIFT, 0);
  if (e != hipSuccess) return e;
  for (int32_t q = 0; q < n - 1; ++q) {
    visit(MX_K_STEP_JOINT, q);
    e = mxk::launch_step_joint(s->stream, &s->tev, s->desc, s->tiles64, s->n_tiles64, kJointBs, 1,
                               q % 3);
    after(MX_K_STEP_JOINT, q);
    if (e != hipSuccess) return e;
  }
  const int pf = (n - 1) % 3;  // phase of the last step
  visit(MX_K_BS, n - 1);
  e = mxk::launch_bs_sys(s->stream, &s->tev, s->desc, 1, kBsBlocks, 1, pf, pf, -1);
  after(MX_K_BS, n - 1);
  if (e != hipSuccess) return e;
  visit(MX_K_FORCE_KICK, n - 1);
  e = mxk::launch_step_b_tiles(s->stream, &s->tev, s->desc, s->tiles, s->n_tiles, kTileBlk, 1, 1,
                               pf);
  after(MX_K_FORCE_KICK, n - 1);
  s->last_list = pf;
  return e;
}

template <class Visit, class After>
hipError_t enqueue_steps(mx_system* s, int32_t n, bool join, Visit visit, After after) {
  join = join && joinable(s, n);
  s->last_list = 0;
  for (int32_t q = 0; q < n; ++q) {
    const int par = join ? (q & 1) : 0;  // step parity (buffers alternate between joined steps)
    for (int k = 0; k < MX_NUM_KERNELS; ++k) {
      if (join && q > 0 && (k == MX_K_GROWTH || k == MX_K_KICK_JUMP_DRIFT)) continue;
      visit(k, q);
      hipError_t e;
      if (join && q < n - 1 && k == MX_K_FORCE_KICK)
        e = mxk::launch_step_ba_tiles(s->stream, &s->tev, s->desc, s->tiles, s->n_tiles,
                                      kTileBlk, 1, par);
      else
        e = launch_group(s, k, par);
      after(k, q);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// FSAL gravity at the current positions (no kick)
hipError_t refresh_accel(mx_system* s) {
  hipError_t e;
  if ((e = mxk::launch_pack_only(s)) != hipSuccess) return e;
  return mxk::launch_force_kick(s, 0);
}

// Joint launches whose tiles had to wait for the integrator (a pair of massive
// bodies in an encounter) take longer than two launches; when more than a fifth
// of the last 32 or more did, joint launches stop for the next 4,096 steps (both
// forms compute the same bits).
constexpr int kJointWindow = 32;
constexpr int64_t kJointPause = 4096;

mx_status read_err(mx_system* s) {
  HIPCHK(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
  DevScalars d;
  HIPCHK(hipMemcpy(&d, s->dsc, sizeof(DevScalars), hipMemcpyDeviceToHost), "read scalars");
  const int32_t err = d.err;
  if (d.joint_runs >= kJointWindow) {
    if (d.joint_slow * 5 > d.joint_runs) {
      s->joint_off = true;
      s->joint_retry_at = s->host_step + kJointPause;
    } else {
      s->joint_off = false;
    }
    int32_t zero2[2] = {0, 0};
    HIPCHK(hipMemcpy(&s->dsc->joint_runs, zero2, sizeof(zero2), hipMemcpyHostToDevice),
           "clear joint counts");
  }
  if (err) {
    int32_t zero = 0;
    HIPCHK(hipMemcpy(&s->dsc->err, &zero, sizeof(int32_t), hipMemcpyHostToDevice), "clear err");
    if (err & MXE_NONFINITE) return fail(MX_ENONFINITE, "non-finite state after a step");
    if (err & MXE_NOCONV) return fail(MX_ENOCONV, "Kepler iteration did not converge");
    if (err & MXE_BS) return fail(MX_EBS, "Bulirsch-Stoer step-halving limit reached");
    if (err & (MXE_PAIRS | MXE_SUBSYS)) return fail(MX_ECAPACITY, "encounter capacity exceeded");
    if (err & MXE_ADJOINT)
      return fail(MX_ECAPACITY, "an encounter subsystem exceeds what the adjoint handles "
                                "(more than 4 members or 64 accepted steps)");
    if (err & MXE_PLANWAIT)
      return fail(MX_EHIP, "the encounter integrator's wait for its plan expired");
  }
  return MX_OK;
}

mx_status check_params(const mx_params* p) {
  if (!p) return fail(MX_EINVAL, "params is NULL");
  if (p->n_big < 0 || p->n_small < 0 || (int64_t)p->n_big + p->n_small <= 0)
    return fail(MX_EINVAL, "need n_big >= 0, n_small >= 0 and at least one body");
  if ((int64_t)p->n_big + p->n_small > (1 << 28)) return fail(MX_EINVAL, "too many bodies");
  if (!(p->G > 0.0) || !(p->m0 > 0.0)) return fail(MX_EINVAL, "G and m0 must be positive");
  if (!(p->dt == p->dt) || p->dt == 0.0) return fail(MX_EINVAL, "dt must be finite and non-zero");
  if (!(p->bs_tol > 0.0)) return fail(MX_EINVAL, "bs_tol must be positive");
  if (!(p->rcrit_hill >= 0.0)) return fail(MX_EINVAL, "rcrit_hill must be >= 0");
  if (p->gas_on && !(p->h_over_r > 0.0 && p->rho_unit > 0.0 && p->au_cm > 0.0 &&
                     p->mfp_coef > 0.0 && p->eta < 0.5))
    return fail(MX_EINVAL, "gas parameters out of range");
  if (!(p->temp_1au >= 0.0) || (p->temp_1au > 0.0 && !(p->cs2_per_k > 0.0)) ||
      (p->eta_mode != 0 && p->eta_mode != 1) || (p->dg_mode != 0 && p->dg_mode != 1) ||
      (p->dg_mode && p->gamma != 1.0 && !(p->gamma > 0.0 && p->gamma < 2.0)))
    return fail(MX_EINVAL, "disk parameters out of range (temp_1au >= 0 with cs2_per_k > 0, "
                           "eta_mode and dg_mode 0 or 1, disk gravity needs 0 < gamma < 2)");
  return MX_OK;
}

}  // namespace

extern "C" {

const char* mx_last_error(void) { return g_err.c_str(); }

mx_status mx_init_system(const mx_params* p, const double* x_h, const double* v_h,
                         const double* m_big, const double* r_p, const double* rho_p,
                         const double* growth, int is_device_ptr, void* hip_stream,
                         mx_system** out) {
  if (!out) return fail(MX_EINVAL, "out is NULL");
  *out = nullptr;
  mx_status st = check_params(p);
  if (st != MX_OK) return st;
  if (!x_h || !v_h || (p->n_big > 0 && !m_big))
    return fail(MX_EINVAL, "x_h, v_h and m_big are required");
  if (p->gas_on && p->n_small > 0 && (!r_p || !rho_p))
    return fail(MX_EINVAL, "r_p and rho_p are required when gas_on");
  if (!is_device_ptr) {
    for (int k = 0; k < p->n_big; ++k)
      if (!(m_big[k] > 0.0)) return fail(MX_EINVAL, "big-body masses must be positive");
  }
  mx_system* s = new mx_system();
  std::memset((void*)s, 0, sizeof(mx_system));
  s->p = *p;
  s->nb = p->n_big;
  s->ns = p->n_small;
  s->n = s->nb + s->ns;
  s->mu0 = p->G * p->m0;
  s->stream = (hipStream_t)hip_stream;
  const size_t n3 = 3 * (size_t)s->n;
  const int nb = s->nb;
  s->use_sym = mxk::force_split(s->n, nb) > 1;  // many massive bodies: symmetric tile pairs
  s->split = s->ns > 0 ? mxk::force_split(s->ns, nb) : 1;
  s->cap_pairs = 1 << 16;
  s->cap_subs = 4096;
  s->red_blocks = 256;
  s->has_growth = growth != nullptr && nb > 0;
  hipError_t e = hipSuccess;
#define ALLOC(ptr, cnt)                                          \
  if (e == hipSuccess) e = dalloc(&(ptr), (size_t)(cnt));
  ALLOC(s->x, n3) ALLOC(s->u, n3) ALLOC(s->ag, n3) ALLOC(s->x0, n3) ALLOC(s->u0, n3)
  ALLOC(s->mu, nb) ALLOC(s->rcrit, nb) ALLOC(s->mu_init, nb) ALLOC(s->rcrit_init, nb)
  ALLOC(s->growth, 3 * (size_t)nb) ALLOC(s->r_p, s->ns) ALLOC(s->rho_p, s->ns)
  ALLOC(s->bigsnap, 9 * (size_t)nb) ALLOC(s->bigmid, 18 * (size_t)nb)
  ALLOC(s->bigpre, 18 * (size_t)nb) ALLOC(s->bignext, 3)
  ALLOC(s->kpack, mxk::kick_source_count(nb)) ALLOC(s->fpack, nb)
  ALLOC(s->part, s->use_sym && s->ns > 0 ? (size_t)s->split * n3 : 1)
  {
    const size_t nT = (size_t)(nb + 63) / 64;
    ALLOC(s->sympart, s->use_sym ? nT * nT * 3 * 64 : 1)
  }
  ALLOC(s->pairs, 6 * (size_t)s->cap_pairs) ALLOC(s->pairs_tmp, 4 * (size_t)s->cap_pairs)
  ALLOC(s->plan_idx, 2 * (size_t)s->cap_pairs)
  ALLOC(s->subs, s->cap_subs) ALLOC(s->uf, 2 * (size_t)nb) ALLOC(s->dsc, 1) ALLOC(s->red, s->red_blocks)
  ALLOC(s->jsub, nb > 0 && nb <= kSmallBig ? 3 * (size_t)s->cap_subs : 1)
  s->n_tiles = (s->n + kTileBlk - 1) / kTileBlk;
  s->n_tiles64 = (s->n + 63) / 64;
  ALLOC(s->desc, 1) ALLOC(s->tiles, s->n_tiles)
  ALLOC(s->tiles64, nb > 0 && nb <= kSmallBig ? s->n_tiles64 : 1)
#undef ALLOC
  if (e != hipSuccess) {
    free_system(s);
    return fail(MX_ENOMEM, "device allocation failed");
  }
  double* vh_tmp = nullptr;
  hipStream_t sm = s->stream;
#define STEP(expr, where)                                    \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) {                                  \
      if (vh_tmp) (void)hipFree(vh_tmp);                           \
      mx_status _r = hip_fail(_e, where);                    \
      free_system(s);                                        \
      return _r;                                             \
    }                                                        \
  } while (0)
  {
    SysDesc d = make_desc(s);
    std::vector<Tile> tl;
    append_tiles(tl, 0, s->n, kTileBlk);
    STEP(hipMemcpy(s->desc, &d, sizeof(SysDesc), hipMemcpyHostToDevice), "copy descriptor");
    STEP(hipMemcpy(s->tiles, tl.data(), sizeof(Tile) * tl.size(), hipMemcpyHostToDevice),
         "copy tiles");
    if (nb > 0 && nb <= kSmallBig) {
      std::vector<Tile> t64;
      append_tiles(t64, 0, s->n, 64);
      STEP(hipMemcpy(s->tiles64, t64.data(), sizeof(Tile) * t64.size(), hipMemcpyHostToDevice),
           "copy tiles");
    }
  }
  STEP(dalloc(&vh_tmp, n3), "alloc v_h");
  STEP(hipMemsetAsync(s->dsc, 0, sizeof(DevScalars), sm), "memset");
  STEP(hipMemsetAsync(s->ag, 0, sizeof(double) * n3, sm), "memset");
  STEP(mxk::pad_kick_sources(nb, s->kpack, sm), "pad sources");
  STEP(copy_in(s->x, x_h, sizeof(double) * n3, is_device_ptr, sm), "copy x");
  STEP(copy_in(vh_tmp, v_h, sizeof(double) * n3, is_device_ptr, sm), "copy v");
  STEP(copy_in(s->mu_init, m_big, sizeof(double) * nb, is_device_ptr, sm), "copy m");
  if (s->has_growth) STEP(copy_in(s->growth, growth, sizeof(double) * 3 * nb, is_device_ptr, sm), "copy growth");
  if (s->ns > 0 && r_p) STEP(copy_in(s->r_p, r_p, sizeof(double) * s->ns, is_device_ptr, sm), "copy r_p");
  if (s->ns > 0 && rho_p) STEP(copy_in(s->rho_p, rho_p, sizeof(double) * s->ns, is_device_ptr, sm), "copy rho_p");
  STEP(mxk::launch_init_bodies(s, s->x, vh_tmp), "init kernels");
  STEP(mxk::launch_h2dh(s, vh_tmp), "h2dh");
  STEP(refresh_accel(s), "initial force");
  STEP(hipStreamSynchronize(sm), "sync");
  (void)hipFree(vh_tmp);
  vh_tmp = nullptr;
  if (s->nb > kSmallBig && s->ns == 0) {
    // order of the culled encounter test: increasing heliocentric distance at init
    std::vector<double> xh(n3);
    STEP(hipMemcpy(xh.data(), s->x, sizeof(double) * n3, hipMemcpyDeviceToHost), "read x");
    std::vector<double> r(nb);
    for (int k = 0; k < nb; ++k)
      r[k] = xh[k] * xh[k] + xh[s->n + k] * xh[s->n + k] + xh[2 * s->n + k] * xh[2 * s->n + k];
    std::vector<int32_t> perm(nb);
    for (int k = 0; k < nb; ++k) perm[k] = k;
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return r[a] < r[b]; });
    STEP(dalloc(&s->flag_perm, nb), "alloc order");
    STEP(dalloc(&s->flag_bounds, (nb + 63) / 64), "alloc chunk bounds");
    STEP(hipMemcpy(s->flag_perm, perm.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice),
         "copy order");
  }
  if (s->has_growth) {  // bodies [0, growth_prefix) hold every growing body
    std::vector<double> gh(3 * (size_t)nb);
    STEP(hipMemcpy(gh.data(), s->growth, sizeof(double) * gh.size(), hipMemcpyDeviceToHost),
         "read growth");
    for (int k = 0; k < nb; ++k)
      if (gh[3 * k + 2] > 0.0) s->growth_prefix = k + 1;
  }
#undef STEP
  if (is_device_ptr && nb > 0) {
    // validate the masses now that they are on the device
    double* hm = new double[nb];
    hipError_t e2 = hipMemcpy(hm, s->mu, sizeof(double) * nb, hipMemcpyDeviceToHost);
    bool bad = false;
    for (int k = 0; k < nb && e2 == hipSuccess; ++k) bad |= !(hm[k] > 0.0);
    delete[] hm;
    if (e2 != hipSuccess || bad) {
      free_system(s);
      return fail(MX_EINVAL, "big-body masses must be positive");
    }
  }
  st = read_err(s);
  if (st != MX_OK) {
    free_system(s);
    return st;
  }
  *out = s;
  return MX_OK;
}

mx_status mx_step(mx_system* s, int32_t n_steps) {
  if (!s || n_steps < 0) return fail(MX_EINVAL, "bad system or step count");
  if (n_steps == 0) return MX_OK;
  const bool use_graph = s->launch_mode == MX_LAUNCH_GRAPH && s->stream != nullptr;
  if (use_graph && !s->graph_ok) {
    hipGraph_t g;
    HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t e = enqueue_step(s);
    hipError_t e2 = hipStreamEndCapture(s->stream, &g);
    if (e != hipSuccess) return hip_fail(e, "capture step");
    if (e2 != hipSuccess) return hip_fail(e2, "end capture");
    e = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    s->graph_ok = true;
  }
  if (use_graph) {
    s->last_list = 0;  // one step per graph
    for (int32_t k = 0; k < n_steps; ++k)
      HIPCHK(hipGraphLaunch(s->graph, s->stream), "graph launch");
  } else if (joint_ok(s, n_steps)) {
    HIPCHK(enqueue_joint(s, n_steps, [](int, int) {}, [](int, int) {}), "step launch");
  } else {
    HIPCHK(enqueue_steps(s, n_steps, true, [](int, int) {}, [](int, int) {}), "step launch");
  }
  s->host_step += n_steps;
  return MX_OK;
}

mx_status mx_set_launch_mode(mx_system* s, int32_t mode) {
  if (!s || (mode != MX_LAUNCH_EAGER && mode != MX_LAUNCH_GRAPH))
    return fail(MX_EINVAL, "bad system or launch mode");
  if (mode == MX_LAUNCH_GRAPH && s->stream == nullptr)
    return fail(MX_EINVAL, "graph launches need a non-default stream");
  s->launch_mode = mode;
  return MX_OK;
}

mx_status mx_step_profiled(mx_system* s, int32_t n_steps, double* kernel_ms) {
  if (!s || n_steps < 0 || !kernel_ms) return fail(MX_EINVAL, "bad argument");
  const int K = MX_NUM_KERNELS;
  hipEvent_t ev[K + 1];
  for (int k = 0; k <= K; ++k) HIPCHK(hipEventCreate(&ev[k]), "event create");
  for (int k = 0; k < K; ++k) kernel_ms[k] = 0.0;
  hipError_t e = hipSuccess;
  s->last_list = 0;
  for (int32_t q = 0; q < n_steps && e == hipSuccess; ++q) {
    e = hipEventRecord(ev[0], s->stream);
    for (int k = 0; k < K && e == hipSuccess; ++k) {
      e = launch_group(s, k);
      if (e == hipSuccess) e = hipEventRecord(ev[k + 1], s->stream);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[K]);
    for (int k = 0; k < K && e == hipSuccess; ++k) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      kernel_ms[k] += ms;
    }
  }
  for (int k = 0; k <= K; ++k) (void)hipEventDestroy(ev[k]);
  if (e != hipSuccess) return hip_fail(e, "profiled step");
  s->host_step += n_steps;
  return read_err(s);
}

mx_status mx_step_timed(mx_system* s, int32_t n_steps, int32_t group, int32_t stride,
                        float* kernel_ms, int32_t* n_launched) {
  if (!s || n_steps < 0 || group < 0 || group > MX_K_STEP_JOINT || stride < 1 || !kernel_ms ||
      !n_launched)
    return fail(MX_EINVAL, "bad argument");
  *n_launched = 0;
  if (n_steps == 0) return MX_OK;
  if (n_steps > (1 << 24)) return fail(MX_EINVAL, "too many timed steps in one call");
  hipError_t e = hipSuccess;
  const int32_t n_timed = (n_steps - 1) / stride + 1;  // steps 0, stride, 2 stride, ...
  if (s->tev_pool_n < 2 * n_timed) {  // grow the event pool (kept for later calls)
    hipEvent_t* pool = new hipEvent_t[2 * (size_t)n_timed];
    int32_t k = 0;
    for (; k < s->tev_pool_n; ++k) pool[k] = s->tev_pool[k];
    for (; k < 2 * n_timed && e == hipSuccess; ++k) e = hipEventCreate(&pool[k]);
    if (e != hipSuccess) --k;  // pool[k] was not created
    delete[] s->tev_pool;
    s->tev_pool = pool;
    s->tev_pool_n = k;
    if (e != hipSuccess) return hip_fail(e, "event create");
  }
  hipEvent_t* ev = s->tev_pool;
  std::vector<char> used(n_steps, 0);
  // the joined launch spans two steps: it is used unless the timed group is one
  // of the two kernels it joins
  const bool join = group != MX_K_KICK_JUMP_DRIFT && group != MX_K_FORCE_KICK;
  const bool joins = joinable(s, n_steps);
  // the group launched as kernel k of step q (the joined launch stands at the
  // closing group of every step but the last)
  auto timed = [&](int k, int q) {
    if (q % stride != 0) return false;
    if (group == MX_K_STEP_JOINED) return joins && k == MX_K_FORCE_KICK && q < n_steps - 1;
    return k == group;
  };
  auto visit = [&](int k, int q) {
    if (timed(k, q)) {
      s->tev.armed = true;
      s->tev.start = ev[2 * (q / stride)];
      s->tev.stop = ev[2 * (q / stride) + 1];
    }
  };
  auto after = [&](int k, int q) {
    if (timed(k, q)) {
      used[q] = s->tev.start == nullptr;  // the start event went to a kernel
      s->tev.armed = false;
      s->tev.start = s->tev.stop = nullptr;
    }
  };
  // the joint launch is timed in the joint sequence mx_step runs; every other
  // group in the sequence of separate (or two-step joined) launches
  if (group == MX_K_STEP_JOINT && joint_ok(s, n_steps))
    e = enqueue_joint(s, n_steps, visit, after);
  else
    e = enqueue_steps(s, n_steps, join, visit, after);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  int32_t nl = 0;
  for (int32_t q = 0; q < n_steps; ++q) {
    float ms = 0.f;
    if (e == hipSuccess && used[q]) {
      e = hipEventElapsedTime(&ms, ev[2 * (q / stride)], ev[2 * (q / stride) + 1]);
      ++nl;
    }
    kernel_ms[q] = ms;
  }
  if (e != hipSuccess) return hip_fail(e, "timed step");
  *n_launched = nl;
  s->host_step += n_steps;
  return read_err(s);
}

mx_status mx_get_counters(mx_system* s, uint64_t* bs_flop, uint64_t* pairs_flagged) {
  if (!s || !bs_flop || !pairs_flagged) return fail(MX_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  DevScalars d;
  HIPCHK(hipMemcpy(&d, s->dsc, sizeof(DevScalars), hipMemcpyDeviceToHost), "read scalars");
  *bs_flop = d.bs_flop;
  *pairs_flagged = d.pairs_flagged;
  return MX_OK;
}

mx_status mx_sync(mx_system* s) {
  if (!s) return fail(MX_EINVAL, "system is NULL");
  return read_err(s);
}

mx_status mx_energy(mx_system* s, double* E, double L[3]) {
  if (!s || !E || !L) return fail(MX_EINVAL, "NULL argument");
  double* out = nullptr;
  HIPCHK(hipMalloc((void**)&out, 4 * sizeof(double)), "alloc");
  hipError_t e = mxk::launch_energy(s, out);
  double h[4] = {0, 0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(out);
  if (e != hipSuccess) return hip_fail(e, "energy");
  *E = h[0];
  L[0] = h[1];
  L[1] = h[2];
  L[2] = h[3];
  return read_err(s);
}

mx_status mx_encounters(mx_system* s, int32_t* pairs, int32_t cap, int32_t* n_out) {
  if (!s || !n_out || cap < 0 || (cap > 0 && !pairs)) return fail(MX_EINVAL, "bad argument");
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  DevScalars d;
  HIPCHK(hipMemcpy(&d, s->dsc, sizeof(DevScalars), hipMemcpyDeviceToHost), "read scalars");
  *n_out = d.n_pairs_last;
  // the planner may leave the list in append order: order it by (i, j) here
  const int all = d.n_pairs_last < s->cap_pairs ? d.n_pairs_last : s->cap_pairs;
  const int m = all < cap ? all : cap;
  if (m > 0) {
    std::vector<int32_t> buf(2 * (size_t)all);
    HIPCHK(hipMemcpy(buf.data(), s->pairs + (size_t)s->last_list * 2 * s->cap_pairs,
                     sizeof(int32_t) * 2 * all, hipMemcpyDeviceToHost),
           "copy pairs");
    std::vector<int64_t> key(all);
    for (int q = 0; q < all; ++q)
      key[q] = ((int64_t)buf[2 * q] << 32) | (uint32_t)buf[2 * q + 1];
    std::sort(key.begin(), key.end());
    for (int q = 0; q < m; ++q) {
      pairs[2 * q] = (int32_t)(key[q] >> 32);
      pairs[2 * q + 1] = (int32_t)(key[q] & 0xffffffff);
    }
  }
  return MX_OK;
}

mx_status mx_get_state(mx_system* s, double* x_h, double* v_h, int is_device_ptr) {
  if (!s || !x_h || !v_h) return fail(MX_EINVAL, "NULL argument");
  size_t bytes = sizeof(double) * 3 * (size_t)s->n;
  double* vt = nullptr;
  HIPCHK(hipMalloc((void**)&vt, bytes), "alloc");
  hipError_t e = mxk::launch_dh2h(s, vt);
  if (e == hipSuccess) e = copy_out(x_h, s->x, bytes, is_device_ptr, s->stream);
  if (e == hipSuccess) e = copy_out(v_h, vt, bytes, is_device_ptr, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(vt);
  if (e != hipSuccess) return hip_fail(e, "get_state");
  return MX_OK;
}

static mx_status set_common(mx_system* s, int64_t step_index) {
  if (s->has_phys) {
    // restart: the clock at step_index * dt with the initial step, R_c forgotten,
    // the masses of the step before in force
    HIPCHK(mxk::launch_reset_scalars(s, step_index), "reset");
    HIPCHK(mxk::launch_physics_reset(s, (double)step_index * s->p.dt), "physics reset");
    if (step_index > 0)
      HIPCHK(mxk::launch_physics(s, 1, (double)(step_index - 1) * s->p.dt), "masses");
    else {
      HIPCHK(hipMemcpyAsync(s->mu, s->mu_init, sizeof(double) * s->nb, hipMemcpyDeviceToDevice, s->stream), "mu");
      HIPCHK(hipMemcpyAsync(s->rcrit, s->rcrit_init, sizeof(double) * s->nb, hipMemcpyDeviceToDevice, s->stream), "rcrit");
    }
  } else if (s->has_growth) {
    // the masses of the step before step_index were the ones in force
    int64_t prev = step_index > 0 ? step_index - 1 : 0;
    HIPCHK(mxk::launch_reset_scalars(s, prev), "reset");
    if (step_index > 0) HIPCHK(mxk::launch_growth(s), "growth");
    else {
      HIPCHK(hipMemcpyAsync(s->mu, s->mu_init, sizeof(double) * s->nb, hipMemcpyDeviceToDevice, s->stream), "mu");
      HIPCHK(hipMemcpyAsync(s->rcrit, s->rcrit_init, sizeof(double) * s->nb, hipMemcpyDeviceToDevice, s->stream), "rcrit");
    }
  }
  HIPCHK(mxk::launch_reset_scalars(s, step_index), "reset");
  HIPCHK(refresh_accel(s), "force");
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  s->host_step = step_index;
  return MX_OK;
}

mx_status mx_set_state(mx_system* s, const double* x_h, const double* v_h, int is_device_ptr,
                       int64_t step_index) {
  if (!s || !x_h || !v_h || step_index < 0) return fail(MX_EINVAL, "bad argument");
  size_t bytes = sizeof(double) * 3 * (size_t)s->n;
  double* vt = nullptr;
  HIPCHK(hipMalloc((void**)&vt, bytes), "alloc");
  hipError_t e = copy_in(s->x, x_h, bytes, is_device_ptr, s->stream);
  if (e == hipSuccess) e = copy_in(vt, v_h, bytes, is_device_ptr, s->stream);
  if (e == hipSuccess) e = mxk::launch_h2dh(s, vt);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(vt);
  if (e != hipSuccess) return hip_fail(e, "set_state");
  return set_common(s, step_index);
}

mx_status mx_get_state_dh(mx_system* s, double* x, double* u, int is_device_ptr) {
  if (!s || !x || !u) return fail(MX_EINVAL, "NULL argument");
  size_t bytes = sizeof(double) * 3 * (size_t)s->n;
  HIPCHK(copy_out(x, s->x, bytes, is_device_ptr, s->stream), "copy x");
  HIPCHK(copy_out(u, s->u, bytes, is_device_ptr, s->stream), "copy u");
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  return MX_OK;
}

mx_status mx_set_state_dh(mx_system* s, const double* x, const double* u, int is_device_ptr,
                          int64_t step_index) {
  if (!s || !x || !u || step_index < 0) return fail(MX_EINVAL, "bad argument");
  size_t bytes = sizeof(double) * 3 * (size_t)s->n;
  HIPCHK(copy_in(s->x, x, bytes, is_device_ptr, s->stream), "copy x");
  HIPCHK(copy_in(s->u, u, bytes, is_device_ptr, s->stream), "copy u");
  return set_common(s, step_index);
}

mx_status mx_get_accel(mx_system* s, double* a, int is_device_ptr) {
  if (!s || !a) return fail(MX_EINVAL, "NULL argument");
  HIPCHK(copy_out(a, s->ag, sizeof(double) * 3 * (size_t)s->n, is_device_ptr, s->stream), "copy a");
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  return MX_OK;
}

mx_status mx_get_masses(mx_system* s, double* mu, double* rcrit) {
  if (!s || (s->nb > 0 && (!mu || !rcrit))) return fail(MX_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  if (s->nb > 0) {
    HIPCHK(hipMemcpy(mu, s->mu, sizeof(double) * s->nb, hipMemcpyDeviceToHost), "copy mu");
    HIPCHK(hipMemcpy(rcrit, s->rcrit, sizeof(double) * s->nb, hipMemcpyDeviceToHost), "copy rcrit");
  }
  return MX_OK;
}

mx_status mx_get_step_index(mx_system* s, int64_t* step_index) {
  if (!s || !step_index) return fail(MX_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  DevScalars d;
  HIPCHK(hipMemcpy(&d, s->dsc, sizeof(DevScalars), hipMemcpyDeviceToHost), "read scalars");
  *step_index = d.step;
  return MX_OK;
}

mx_status mx_set_planet_physics(mx_system* s, const mx_planet* planets, double a_switch,
                                double a_min) {
  if (!s || !planets) return fail(MX_EINVAL, "NULL argument");
  if (s->owned) return fail(MX_EINVAL, "planet physics is for a system of its own");
  if (s->nb <= 0 || s->nb > kSmallBig)
    return fail(MX_EINVAL, "planet physics needs 1 <= n_big <= 64");
  if (a_switch > 0.0 && !(a_min > 0.0)) return fail(MX_EINVAL, "the step switch needs a_min > 0");
  static_assert(sizeof(mx_planet) == sizeof(PlanetPhys), "planet record layout");
  const int nb = s->nb;
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  if (!s->phys) {
    HIPCHK(dalloc(&s->phys, nb), "alloc");
    HIPCHK(dalloc(&s->radius, nb), "alloc");
    HIPCHK(dalloc(&s->rad_c, nb), "alloc");
    HIPCHK(dalloc(&s->gaps, 4 * (size_t)nb), "alloc");
  }
  s->any_gap = 0;
  for (int k = 0; k < nb; ++k) s->any_gap |= planets[k].gap_C > 0.0 && planets[k].tau_g > 0.0;
  HIPCHK(hipMemcpy(s->phys, planets, sizeof(PlanetPhys) * nb, hipMemcpyHostToDevice), "copy");
  HIPCHK(hipMemset(s->radius, 0, sizeof(double) * nb), "clear");
  HIPCHK(hipMemset(s->gaps, 0, sizeof(double) * 4 * nb), "clear");
  s->has_phys = 1;
  s->has_growth = 0;
  s->a_switch = a_switch;
  s->a_min = a_min;
  SysDesc d = make_desc(s);
  HIPCHK(hipMemcpy(s->desc, &d, sizeof(SysDesc), hipMemcpyHostToDevice), "descriptor");
  DevScalars hd;
  HIPCHK(hipMemcpy(&hd, s->dsc, sizeof(hd), hipMemcpyDeviceToHost), "read scalars");
  HIPCHK(mxk::launch_physics_reset(s, (double)hd.step * s->p.dt), "physics reset");
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  if (s->graph_ok) {
    (void)hipGraphExecDestroy(s->graph);
    s->graph_ok = false;
  }
  return MX_OK;
}

mx_status mx_get_planet_radii(mx_system* s, double* radius) {
  if (!s || !radius) return fail(MX_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  if (!s->has_phys || s->nb == 0) {
    for (int k = 0; k < s->nb; ++k) radius[k] = 0.0;
    return MX_OK;
  }
  HIPCHK(hipMemcpy(radius, s->radius, sizeof(double) * s->nb, hipMemcpyDeviceToHost), "copy");
  return MX_OK;
}

mx_status mx_get_time(mx_system* s, double* t, double* h) {
  if (!s || !t || !h) return fail(MX_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  DevScalars hd;
  HIPCHK(hipMemcpy(&hd, s->dsc, sizeof(hd), hipMemcpyDeviceToHost), "read scalars");
  SysDesc d;
  HIPCHK(hipMemcpy(&d, s->desc, sizeof(d), hipMemcpyDeviceToHost), "read descriptor");
  *t = s->has_phys ? hd.time : (double)hd.step * s->p.dt;
  *h = d.h;
  return MX_OK;
}

mx_status mx_check_removal(mx_system* s, double r_cen, int32_t* ejcount) {
  if (!s || !ejcount) return fail(MX_EINVAL, "NULL argument");
  if (s->owned) return fail(MX_EINVAL, "body removal is for a system of its own");
  if (!(r_cen >= 0.0)) return fail(MX_EINVAL, "r_cen must be >= 0");
  if (!s->stat) {
    HIPCHK(dalloc(&s->stat, s->n), "alloc");
    HIPCHK(dalloc(&s->rsign, s->n), "alloc");
    HIPCHK(dalloc(&s->ejcount, 1), "alloc");
    HIPCHK(dalloc(&s->rm_P, 3), "alloc");
    HIPCHK(hipMemsetAsync(s->stat, 0, sizeof(int32_t) * s->n, s->stream), "clear");
    HIPCHK(hipMemsetAsync(s->rsign, 0, (size_t)s->n, s->stream), "clear");
    HIPCHK(hipMemsetAsync(s->ejcount, 0, sizeof(int32_t), s->stream), "clear");
  }
  HIPCHK(mxk::launch_check_removal(s, r_cen), "check removal");
  HIPCHK(hipMemcpyAsync(ejcount, s->ejcount, sizeof(int32_t), hipMemcpyDeviceToHost, s->stream),
         "copy");
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  return MX_OK;
}

mx_status mx_compact(mx_system* s, int32_t* n_removed, int32_t* index_map) {
  if (!s || !n_removed) return fail(MX_EINVAL, "NULL argument");
  if (s->owned) return fail(MX_EINVAL, "body removal is for a system of its own");
  const int n = s->n;
  *n_removed = 0;
  if (!s->stat) {
    if (index_map)
      for (int t = 0; t < n; ++t) index_map[t] = t;
    return MX_OK;
  }
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  int32_t* map = nullptr;
  HIPCHK(dalloc(&map, n), "alloc");
  int32_t m = n;
  hipError_t e = mxk::compact_bodies(s, &m, map);
  if (e == hipSuccess && index_map)
    e = hipMemcpy(index_map, map, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
  (void)hipFree(map);
  if (e != hipSuccess) return hip_fail(e, "compact");
  if (m == n) return MX_OK;
  // the survivors with the new stride: counts, tiles and descriptor follow; the
  // flagged massive bodies stay, so the count of flagged bodies is theirs
  s->n = m;
  s->ns = m - s->nb;
  s->p.n_small = s->ns;
  std::vector<Tile> tl;
  append_tiles(tl, 0, s->n, kTileBlk);
  s->n_tiles = (int32_t)tl.size();
  SysDesc d = make_desc(s);
  HIPCHK(hipMemcpy(s->desc, &d, sizeof(SysDesc), hipMemcpyHostToDevice), "descriptor");
  HIPCHK(hipMemcpy(s->tiles, tl.data(), sizeof(Tile) * tl.size(), hipMemcpyHostToDevice), "tiles");
  if (s->nb > 0 && s->nb <= kSmallBig) {
    std::vector<Tile> t64;
    append_tiles(t64, 0, s->n, 64);
    s->n_tiles64 = (int32_t)t64.size();
    HIPCHK(hipMemcpy(s->tiles64, t64.data(), sizeof(Tile) * t64.size(), hipMemcpyHostToDevice),
           "tiles");
  }
  std::vector<int32_t> st(s->nb > 0 ? s->nb : 1);
  int32_t flagged = 0;
  if (s->nb > 0) {
    HIPCHK(hipMemcpy(st.data(), s->stat, sizeof(int32_t) * s->nb, hipMemcpyDeviceToHost), "status");
    for (int k = 0; k < s->nb; ++k) flagged += st[k] < 0;
  }
  HIPCHK(hipMemcpy(s->ejcount, &flagged, sizeof(int32_t), hipMemcpyHostToDevice), "count");
  if (s->graph_ok) {
    (void)hipGraphExecDestroy(s->graph);
    s->graph_ok = false;
  }
  *n_removed = n - m;
  return MX_OK;
}

mx_status mx_get_status(mx_system* s, int32_t* stat) {
  if (!s || !stat) return fail(MX_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(s->stream), "sync");
  if (!s->stat) {
    for (int t = 0; t < s->n; ++t) stat[t] = 0;
    return MX_OK;
  }
  HIPCHK(hipMemcpy(stat, s->stat, sizeof(int32_t) * s->n, hipMemcpyDeviceToHost), "copy");
  return MX_OK;
}

mx_status mx_get_counts(mx_system* s, int32_t* n_big, int32_t* n_small) {
  if (!s || !n_big || !n_small) return fail(MX_EINVAL, "NULL argument");
  *n_big = s->nb;
  *n_small = s->ns;
  return MX_OK;
}

void mx_destroy(mx_system* s) {
  if (!s || s->owned) return;
  (void)hipStreamSynchronize(s->stream);
  free_system(s);
}

// ------------------------------------------------ single-kernel entry points
mx_status mx_gravity(int32_t n, int32_t n_big, const double* x, const double* mu,
                     const double* rcrit, double* a, void* hip_stream) {
  if (n <= 0 || n_big < 0 || n_big > n || !x || !a || (n_big > 0 && (!mu || !rcrit)))
    return fail(MX_EINVAL, "bad argument");
  HIPCHK(mxk::gravity(n, n_big, x, mu, rcrit, a, (hipStream_t)hip_stream), "gravity");
  return MX_OK;
}

mx_status mx_gas_drag(const mx_params* p, int32_t n, int32_t n_big, const double* x,
                      const double* u, const double* mu, const double* r_p,
                      const double* rho_p, double* a, void* hip_stream) {
  if (!p || n <= 0 || n_big < 0 || n_big > n || !x || !u || !a ||
      (n > n_big && (!r_p || !rho_p)) || (n_big > 0 && !mu))
    return fail(MX_EINVAL, "bad argument");
  HIPCHK(mxk::gas_drag(p, n, n_big, x, u, mu, r_p, rho_p, a, (hipStream_t)hip_stream), "drag");
  return MX_OK;
}

mx_status mx_kepler_drift(int32_t n, double mu0, double h, const double* x0, const double* u0,
                          double* x1, double* u1, void* hip_stream) {
  if (n <= 0 || !(mu0 > 0.0) || !x0 || !u0 || !x1 || !u1) return fail(MX_EINVAL, "bad argument");
  hipStream_t st = (hipStream_t)hip_stream;
  int32_t* err = nullptr;
  HIPCHK(hipMalloc((void**)&err, sizeof(int32_t)), "alloc");
  HIPCHK(hipMemsetAsync(err, 0, sizeof(int32_t), st), "memset");
  HIPCHK(mxk::kepler(n, mu0, h, x0, u0, x1, u1, err, st), "kepler");
  int32_t herr = 0;
  HIPCHK(hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipStreamSynchronize(st), "sync");
  (void)hipFree(err);
  if (herr) return fail(MX_ENOCONV, "Kepler iteration did not converge");
  return MX_OK;
}

mx_status mx_flag_pairs(int32_t n, int32_t n_big, const double* rcrit, const double* x0,
                        const double* u0, const double* x1, const double* u1, double h,
                        int32_t* pairs, int32_t cap, int32_t* n_out, void* hip_stream) {
  if (n <= 0 || n_big < 0 || n_big > n || !x0 || !u0 || !x1 || !u1 || !n_out || cap <= 0 ||
      !pairs || (n_big > 0 && !rcrit) || (cap & (cap - 1)) != 0)
    return fail(MX_EINVAL, "bad argument (cap must be a power of two)");
  hipStream_t st = (hipStream_t)hip_stream;
  DevScalars* dsc = nullptr;
  int32_t* tmp = nullptr;
  HIPCHK(hipMalloc((void**)&dsc, sizeof(DevScalars)), "alloc");
  HIPCHK(hipMalloc((void**)&tmp, 4 * sizeof(int32_t) * (size_t)cap), "alloc");
  HIPCHK(hipMemsetAsync(dsc, 0, sizeof(DevScalars), st), "memset");
  HIPCHK(mxk::flag_pairs(n, n_big, rcrit, x0, u0, x1, u1, h, pairs, tmp, cap, dsc, st), "flag");
  DevScalars hd;
  HIPCHK(hipMemcpyAsync(&hd, dsc, sizeof(hd), hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipStreamSynchronize(st), "sync");
  (void)hipFree(dsc);
  (void)hipFree(tmp);
  *n_out = hd.n_pairs_last;
  if (hd.err) return fail(MX_ECAPACITY, "more flagged pairs than cap");
  return MX_OK;
}

}  // extern "C"

// ------------------------------------------- allocation-free encounter test
// A file-scope device array serves as the scratch of mx_flag_pairs_noalloc: the
// DevScalars block (counters, cleared by a kernel at every call), the packed
// source records of up to kNoAllocMaxBig massive bodies and the sort keys of up
// to kNoAllocMaxPairs pairs.  Every device holds its own copy, at its own
// address, which is looked up once per device; host code never passes the
// array's name itself to a kernel.
namespace {
constexpr int32_t kNoAllocMaxBig = 4096;
constexpr int32_t kNoAllocMaxPairs = 1 << 16;
constexpr size_t kScrDsc = 256;
constexpr size_t kScrFp = sizeof(FlagSource) * (size_t)kNoAllocMaxBig;
constexpr size_t kScrKeys = 2 * sizeof(int64_t) * (size_t)kNoAllocMaxPairs;
constexpr size_t kScrBytes = kScrDsc + kScrFp + kScrKeys;  // 1.5 MiB
static_assert(sizeof(DevScalars) <= kScrDsc, "scratch header too small");
static_assert(sizeof(DevScalars) % 4 == 0 && sizeof(DevScalars) / 4 <= 64,
              "the header is cleared by one 64-lane wave, a word per lane");
static_assert(kScrDsc % alignof(FlagSource) == 0, "record alignment");
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScrBytes];

namespace {
std::mutex g_scr_mu;
void* g_scr_ptr[kMaxDevices];

// Device address of this device's scratch array (the current device).
hipError_t scratch_address(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scr_mu);
  if (!g_scr_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scr_ptr[dev] = p;
  }
  *out = (unsigned char*)g_scr_ptr[dev];
  return hipSuccess;
}

__global__ void k_zero_words(uint32_t* __restrict__ p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}
}  // namespace

extern "C" {

mx_status mx_flag_pairs_noalloc(int32_t n, int32_t n_big, const double* rcrit, const double* x0,
                                const double* u0, const double* x1, const double* u1, double h,
                                int32_t* pairs, int32_t cap, int32_t* n_out, void* hip_stream) {
  if (n <= 0 || n_big < 0 || n_big > n || !x0 || !u0 || !x1 || !u1 || !n_out || cap <= 0 ||
      !pairs || (n_big > 0 && !rcrit) || (cap & (cap - 1)) != 0)
    return fail(MX_EINVAL, "bad argument (cap must be a power of two)");
  if (n_big > kNoAllocMaxBig || cap > kNoAllocMaxPairs)
    return fail(MX_ECAPACITY, "mx_flag_pairs_noalloc: n_big above 4096 or cap above 65536");
  hipStream_t st = (hipStream_t)hip_stream;
  unsigned char* scr = nullptr;
  HIPCHK(scratch_address(&scr), "scratch address");
  DevScalars* dsc = (DevScalars*)scr;
  FlagSource* fp = (FlagSource*)(scr + kScrDsc);
  int32_t* keys = (int32_t*)(scr + kScrDsc + kScrFp);
  const int words = (int)(sizeof(DevScalars) / sizeof(uint32_t));
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, (uint32_t*)dsc, words);
  HIPCHK(hipGetLastError(), "clear");
  HIPCHK(mxk::flag_pairs_enqueue(n, n_big, rcrit, x0, u0, x1, u1, h, pairs, keys, cap, dsc, fp,
                                 st),
         "flag");
  DevScalars hd;
  HIPCHK(hipMemcpyAsync(&hd, dsc, sizeof(hd), hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipStreamSynchronize(st), "sync");
  *n_out = hd.n_pairs_last;
  if (hd.err) return fail(MX_ECAPACITY, "more flagged pairs than cap");
  return MX_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
struct mx_batch {
  int32_t n_sys;
  mx_system** sys;
  hipStream_t stream;
  SysDesc* desc;    // device [n_sys]
  Tile* tiles;      // device, room for the finest tiling (64 bodies per tile)
  int32_t tiles_cap;
  int32_t n_tiles;
  int32_t blk, tpb, bps;
  int32_t launch_mode, graph_steps;
  hipGraphExec_t graph;
  bool graph_ok;
  LaunchTiming tev;
};

namespace {

bool valid_config(int blk, int tpb, int bps) {
  return (blk == 64 || blk == 128 || blk == 256 || blk == 512) && tpb >= 1 && tpb <= 64 &&
         bps >= 1 && bps <= 1024;
}

// tile table of the current blk: systems in order, tiles of each system in order
hipError_t upload_tiles(mx_batch* b) {
  std::vector<Tile> tl;
  for (int k = 0; k < b->n_sys; ++k) append_tiles(tl, k, b->sys[k]->n, b->blk);
  if ((int64_t)tl.size() > b->tiles_cap) return hipErrorInvalidValue;
  b->n_tiles = (int32_t)tl.size();
  return hipMemcpy(b->tiles, tl.data(), sizeof(Tile) * tl.size(), hipMemcpyHostToDevice);
}

// n batch steps; between two steps the closing and opening kernels are one launch
// (k_step_ba), the same operations per body
hipError_t enqueue_batch_steps(mx_batch* b, int32_t n) {
  hipError_t e = hipSuccess;
  // (joint launches, the integrator beside the tiles, measured slower here: the
  // integrator's registers and LDS hold the ensemble's many tiles to one wave per
  // SIMD)
  for (int k = 0; k < b->n_sys; ++k) b->sys[k]->last_list = 0;
  for (int32_t q = 0; q < n && e == hipSuccess; ++q) {
    const int par = q & 1;  // step parity (buffers alternate between joined steps)
    if (q == 0)
      e = mxk::launch_step_a_tiles(b->stream, &b->tev, b->desc, b->tiles, b->n_tiles, b->blk,
                                   b->tpb, 0);
    if (e == hipSuccess)
      e = mxk::launch_bs_sys(b->stream, &b->tev, b->desc, b->n_sys, b->bps, 1, par, 0, par ^ 1);
    if (e != hipSuccess) break;
    if (q < n - 1)
      e = mxk::launch_step_ba_tiles(b->stream, &b->tev, b->desc, b->tiles, b->n_tiles, b->blk,
                                    b->tpb, par);
    else
      e = mxk::launch_step_b_tiles(b->stream, &b->tev, b->desc, b->tiles, b->n_tiles, b->blk,
                                   b->tpb, 1, par);
  }
  return e;
}

void drop_graph(mx_batch* b) {
  if (b->graph_ok) (void)hipGraphExecDestroy(b->graph);
  b->graph_ok = false;
}

void free_batch(mx_batch* b) {
  if (!b) return;
  drop_graph(b);
  if (b->sys) {
    for (int k = 0; k < b->n_sys; ++k)
      if (b->sys[k]) {
        b->sys[k]->owned = false;
        mx_destroy(b->sys[k]);
      }
    delete[] b->sys;
  }
  if (b->desc) (void)hipFree(b->desc);
  if (b->tiles) (void)hipFree(b->tiles);
  delete b;
}

void advance_host_steps(mx_batch* b, int32_t n) {
  for (int k = 0; k < b->n_sys; ++k) b->sys[k]->host_step += n;
}

}  // namespace

extern "C" {

mx_status mx_init_batch(int32_t n_sys, const mx_params* params, const int64_t* offsets,
                        const double* x_h, const double* v_h, const double* m_big,
                        const double* r_p, const double* rho_p, int is_device_ptr,
                        void* hip_stream, mx_batch** out) {
  if (!out) return fail(MX_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_sys <= 0 || !params || !offsets || !x_h || !v_h)
    return fail(MX_EINVAL, "need n_sys > 0, params, offsets, x_h and v_h");
  if (offsets[0] != 0) return fail(MX_EINVAL, "offsets[0] must be 0");
  int64_t nbig_total = 0, nsmall_total = 0;
  bool any_gas = false;
  for (int k = 0; k < n_sys; ++k) {
    mx_status st = check_params(&params[k]);
    if (st != MX_OK) return st;
    if (params[k].n_big > kSmallBig)
      return fail(MX_EINVAL, "batched systems need n_big <= 64");
    if (offsets[k + 1] - offsets[k] != (int64_t)params[k].n_big + params[k].n_small)
      return fail(MX_EINVAL, "offsets[k+1] - offsets[k] must equal n_big + n_small of system k");
    nbig_total += params[k].n_big;
    nsmall_total += params[k].n_small;
    any_gas |= params[k].gas_on && params[k].n_small > 0;
  }
  if (nbig_total > 0 && !m_big) return fail(MX_EINVAL, "m_big is required");
  if (any_gas && (!r_p || !rho_p)) return fail(MX_EINVAL, "r_p and rho_p are required with gas");
  const int64_t N = offsets[n_sys];
  mx_batch* b = new mx_batch();
  std::memset((void*)b, 0, sizeof(mx_batch));
  b->n_sys = n_sys;
  b->stream = (hipStream_t)hip_stream;
  b->blk = kTileBlk;
  b->tpb = 1;
  b->bps = 32;
  b->graph_steps = 1;
  b->sys = new mx_system*[n_sys]();
  // each system from its columns of the concatenated SoA arrays
  int64_t boff = 0, soff = 0;
  std::vector<double> hx, hv;
  double *dx = nullptr, *dv = nullptr;
  for (int k = 0; k < n_sys; ++k) {
    const int64_t off = offsets[k], nk = offsets[k + 1] - offsets[k];
    const double *xs, *vs;
    hipError_t e = hipSuccess;
    if (is_device_ptr) {
      if (dx) (void)hipFree(dx);
      if (dv) (void)hipFree(dv);
      dx = dv = nullptr;
      if ((e = dalloc(&dx, 3 * nk)) == hipSuccess && (e = dalloc(&dv, 3 * nk)) == hipSuccess &&
          (e = hipMemcpy2DAsync(dx, nk * 8, x_h + off, N * 8, nk * 8, 3,
                                hipMemcpyDeviceToDevice, b->stream)) == hipSuccess)
        e = hipMemcpy2DAsync(dv, nk * 8, v_h + off, N * 8, nk * 8, 3, hipMemcpyDeviceToDevice,
                             b->stream);
      xs = dx;
      vs = dv;
    } else {
      hx.resize(3 * nk);
      hv.resize(3 * nk);
      for (int c = 0; c < 3; ++c)
        for (int64_t i = 0; i < nk; ++i) {
          hx[c * nk + i] = x_h[c * N + off + i];
          hv[c * nk + i] = v_h[c * N + off + i];
        }
      xs = hx.data();
      vs = hv.data();
    }
    mx_status st = MX_OK;
    if (e != hipSuccess) {
      st = hip_fail(e, "gather system state");
    } else {
      const bool gas = params[k].gas_on && params[k].n_small > 0;
      st = mx_init_system(&params[k], xs, vs, nbig_total ? m_big + boff : nullptr,
                          gas ? r_p + soff : nullptr, gas ? rho_p + soff : nullptr, nullptr,
                          is_device_ptr, hip_stream, &b->sys[k]);
    }
    if (st != MX_OK) {
      std::string msg = "system " + std::to_string(k) + ": " + g_err;
      if (dx) (void)hipFree(dx);
      if (dv) (void)hipFree(dv);
      free_batch(b);
      g_err = msg;
      return st;
    }
    b->sys[k]->owned = true;
    boff += params[k].n_big;
    soff += params[k].n_small;
  }
  if (dx) (void)hipFree(dx);
  if (dv) (void)hipFree(dv);
  // descriptor and tile tables
  std::vector<SysDesc> d(n_sys);
  int64_t max_tiles = 0;
  for (int k = 0; k < n_sys; ++k) {
    d[k] = make_desc(b->sys[k]);
    max_tiles += (b->sys[k]->n + 63) / 64;
  }
  hipError_t e = dalloc(&b->desc, n_sys);
  if (e == hipSuccess) e = dalloc(&b->tiles, max_tiles);
  if (e == hipSuccess)
    e = hipMemcpy(b->desc, d.data(), sizeof(SysDesc) * n_sys, hipMemcpyHostToDevice);
  b->tiles_cap = (int32_t)max_tiles;
  if (e == hipSuccess) e = upload_tiles(b);

  if (e != hipSuccess) {
    free_batch(b);
    return hip_fail(e, "batch tables");
  }
  *out = b;
  return MX_OK;
}

mx_status mx_batch_set_config(mx_batch* b, int32_t blk, int32_t tiles_per_block,
                              int32_t bs_blocks) {
  if (!b || !valid_config(blk, tiles_per_block, bs_blocks))
    return fail(MX_EINVAL, "bad batch or config (blk in {64,128,256,512}, 1 <= tpb <= 64, "
                           "1 <= bs_blocks <= 1024)");
  HIPCHK(hipStreamSynchronize(b->stream), "sync");
  const bool retile = blk != b->blk;
  b->blk = blk;
  b->tpb = tiles_per_block;
  b->bps = bs_blocks;
  if (retile) HIPCHK(upload_tiles(b), "tile table");
  drop_graph(b);
  return MX_OK;
}

mx_status mx_batch_get_config(mx_batch* b, int32_t* cfg) {
  if (!b || !cfg) return fail(MX_EINVAL, "NULL argument");
  cfg[0] = b->blk;
  cfg[1] = b->tpb;
  cfg[2] = b->bps;
  return MX_OK;
}

mx_status mx_batch_set_launch_mode(mx_batch* b, int32_t mode, int32_t steps_per_graph) {
  if (!b || (mode != MX_LAUNCH_EAGER && mode != MX_LAUNCH_GRAPH) || steps_per_graph < 1 ||
      steps_per_graph > 1000)
    return fail(MX_EINVAL, "bad batch, launch mode or steps per graph (1..1000)");
  if (mode == MX_LAUNCH_GRAPH && b->stream == nullptr)
    return fail(MX_EINVAL, "graph launches need a non-default stream");
  if (steps_per_graph != b->graph_steps) drop_graph(b);
  b->launch_mode = mode;
  b->graph_steps = steps_per_graph;
  return MX_OK;
}

mx_status mx_step_batch(mx_batch* b, int32_t n_steps) {
  if (!b || n_steps < 0) return fail(MX_EINVAL, "bad batch or step count");
  int32_t done = 0;
  if (b->launch_mode == MX_LAUNCH_GRAPH && n_steps >= b->graph_steps) {
    if (!b->graph_ok) {
      hipGraph_t g;
      HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
      hipError_t e = hipSuccess;
      e = enqueue_batch_steps(b, b->graph_steps);
      hipError_t e2 = hipStreamEndCapture(b->stream, &g);
      if (e != hipSuccess) return hip_fail(e, "capture batch step");
      if (e2 != hipSuccess) return hip_fail(e2, "end capture");
      e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail(e, "graph instantiate");
      b->graph_ok = true;
    }
    for (; done + b->graph_steps <= n_steps; done += b->graph_steps)
      HIPCHK(hipGraphLaunch(b->graph, b->stream), "graph launch");
    for (int k = 0; k < b->n_sys; ++k) b->sys[k]->last_list = 0;
  }
  if (done < n_steps) HIPCHK(enqueue_batch_steps(b, n_steps - done), "batch step launch");
  advance_host_steps(b, n_steps);
  return MX_OK;
}

mx_status mx_batch_autotune(mx_batch* b, int32_t steps_per_candidate, int32_t* steps_taken,
                            int32_t* cfg_out, float* best_ms) {
  if (!b || steps_per_candidate < 1 || !steps_taken || !cfg_out || !best_ms)
    return fail(MX_EINVAL, "bad argument");
  *steps_taken = 0;
  hipEvent_t ev[4];
  for (int k = 0; k < 4; ++k) HIPCHK(hipEventCreate(&ev[k]), "event");
  const int saved_mode = b->launch_mode;
  b->launch_mode = MX_LAUNCH_EAGER;
  int32_t taken = 0;
  // `steps_per_candidate` real steps of the batch under one configuration, with
  // events around the body kernels (the tile shape's) and around the encounter
  // integrator (its width's) of every step: each knob is judged by the kernels
  // it shapes, so the encounters of the moment, which set the integrator's time,
  // do not decide the tile shape
  auto trial = [&](int blk, int tpb, int bps, float* body_ms, float* bs_ms) -> mx_status {
    mx_status st = mx_batch_set_config(b, blk, tpb, bps);
    if (st != MX_OK) return st;
    float tb = 0.f, ts = 0.f;
    const int n = steps_per_candidate;
    for (int q = 0; q < n; ++q) {
      const int par = q & 1;
      float m0 = 0.f, m1 = 0.f, m2 = 0.f;
      HIPCHK(hipEventRecord(ev[0], b->stream), "record");
      if (q == 0)
        HIPCHK(mxk::launch_step_a_tiles(b->stream, &b->tev, b->desc, b->tiles, b->n_tiles,
                                        b->blk, b->tpb, 0),
               "trial step");
      HIPCHK(hipEventRecord(ev[1], b->stream), "record");
      HIPCHK(mxk::launch_bs_sys(b->stream, &b->tev, b->desc, b->n_sys, b->bps, 1, par, 0, par ^ 1),
             "trial step");
      HIPCHK(hipEventRecord(ev[2], b->stream), "record");
      if (q < n - 1)
        HIPCHK(mxk::launch_step_ba_tiles(b->stream, &b->tev, b->desc, b->tiles, b->n_tiles,
                                         b->blk, b->tpb, par),
               "trial step");
      else
        HIPCHK(mxk::launch_step_b_tiles(b->stream, &b->tev, b->desc, b->tiles, b->n_tiles,
                                        b->blk, b->tpb, 1, par),
               "trial step");
      HIPCHK(hipEventRecord(ev[3], b->stream), "record");
      HIPCHK(hipEventSynchronize(ev[3]), "sync");
      HIPCHK(hipEventElapsedTime(&m0, ev[0], ev[1]), "elapsed");
      HIPCHK(hipEventElapsedTime(&m1, ev[1], ev[2]), "elapsed");
      HIPCHK(hipEventElapsedTime(&m2, ev[2], ev[3]), "elapsed");
      tb += m0 + m2;
      ts += m1;
    }
    for (int k = 0; k < b->n_sys; ++k) b->sys[k]->last_list = 0;
    advance_host_steps(b, n);
    taken += n;
    *body_ms = tb;
    *bs_ms = ts;
    return MX_OK;
  };
  mx_status st = MX_OK;
  float best_body = 3.0e38f;
  int bb = b->blk, bt = b->tpb, bs = b->bps;
  // tile shape of the body kernels first, then the encounter-integrator width
  const int blks[] = {64, 128, 256, 512};
  const int tpbs[] = {1, 2, 4, 8};
  // widths of the encounter integrator, tried twice in mirrored order (its time
  // varies with the encounters of the moment; the sums compare like with like)
  const int bpss[] = {8, 16, 32, 64};
  constexpr int nbps = sizeof(bpss) / sizeof(bpss[0]);
  float tb = 0.f, ts = 0.f;
  if (st == MX_OK) st = trial(bb, bt, bs, &tb, &ts);  // warm-up of the current configuration
  for (int blk : blks)
    for (int tpb : tpbs) {
      if (st != MX_OK) break;
      st = trial(blk, tpb, bs, &tb, &ts);
      if (st == MX_OK && tb < best_body) {
        best_body = tb;
        bb = blk;
        bt = tpb;
      }
    }
  float sum[nbps] = {};
  for (int pass = 0; pass < 2; ++pass)
    for (int q = 0; q < nbps; ++q) {
      if (st != MX_OK) break;
      const int k = pass == 0 ? q : nbps - 1 - q;
      st = trial(bb, bt, bpss[k], &tb, &ts);
      sum[k] += ts;
    }
  float best = 0.f;
  if (st == MX_OK) {
    int kb = 0;
    for (int k = 1; k < nbps; ++k)
      if (sum[k] < sum[kb]) kb = k;
    bs = bpss[kb];
    best = best_body + 0.5f * sum[kb];
  }
  for (int k = 0; k < 4; ++k) (void)hipEventDestroy(ev[k]);
  b->launch_mode = saved_mode;
  *steps_taken = taken;
  if (st != MX_OK) return st;
  st = mx_batch_set_config(b, bb, bt, bs);
  if (st != MX_OK) return st;
  cfg_out[0] = bb;
  cfg_out[1] = bt;
  cfg_out[2] = bs;
  *best_ms = best / steps_per_candidate;
  for (int k = 0; k < b->n_sys; ++k) {
    st = read_err(b->sys[k]);
    if (st != MX_OK) return st;
  }
  return MX_OK;
}

mx_status mx_batch_sync(mx_batch* b) {
  if (!b) return fail(MX_EINVAL, "batch is NULL");
  HIPCHK(hipStreamSynchronize(b->stream), "sync");
  for (int k = 0; k < b->n_sys; ++k) {
    mx_status st = read_err(b->sys[k]);
    if (st != MX_OK) {
      g_err = "system " + std::to_string(k) + ": " + g_err;
      return st;
    }
  }
  return MX_OK;
}

mx_status mx_batch_system(mx_batch* b, int32_t k, mx_system** view) {
  if (!b || !view || k < 0 || k >= b->n_sys) return fail(MX_EINVAL, "bad batch or index");
  *view = b->sys[k];
  return MX_OK;
}

void mx_destroy_batch(mx_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  free_batch(b);
}

}  // extern "C"

// ------------------------------------------------------------------ adjoint
namespace mxk {
hipError_t adj_kick(hipStream_t st, int n, int nb, double mu0, double hh,
                    const mxd::DragConst& dc, int gas_on, const double* x, const double* up,
                    const double* mu, const double* rcrit, const double* r_p,
                    const double* rho_p, double* lx, double* lu, double* lmu, double* part,
                    double* tot, double jump_coef);
hipError_t adj_momentum(hipStream_t st, int n, int nb, const double* a, double coef,
                        const double* mu, const double* uref, double* lu, double* lmu,
                        double* part, double* tot);
hipError_t adj_drift(hipStream_t st, int n, int nb, double mu0, double h, const double* x0,
                     const double* u0, const double* mu, const double* rcrit,
                     const Subsystem* subs, const int32_t* n_sub, const double* sched,
                     const int32_t* nsched, int32_t* kept, double* contrib, double* lx,
                     double* lu, double* lmu, int32_t* err);
hipError_t adj_h2dh(hipStream_t st, int n, int nb, double G, double m0, const double* m_big,
                    const double* v_h, const double* lu, const double* lmu, double* gm,
                    double* gv, double* part, double* tot);
hipError_t adj_copy(hipStream_t st, double* const* ptr, const int64_t* len, int count,
                    double* packed, int unpack);
hipError_t adj_record(hipStream_t st, double* const* ptr, const int64_t* len, int count,
                      double* packed, const Subsystem* subs, const DevScalars* dsc,
                      const double* sched, const int32_t* nsched, Subsystem* dsubs,
                      int32_t* n_sub_out, double* dsched, int32_t* dnsched);
}  // namespace mxk

// A differentiable run.  Per step of the segment being reversed, the record
// ("tape") keeps the pre-drift state x0, u0, the velocities after drift and
// encounters, the subsystem table, its size and the accepted Bulirsch-Stoer
// steps; the positions after the step are those of the next saved state.
struct mx_adjoint {
  mx_system* s;
  int32_t n_steps, every, n_ckpt;
  size_t blk;        // doubles of one saved state: x, u, ag [3][n], bigsnap [9][nb]
  double* ckpt;      // [n_ckpt][blk]: states at steps 0, every, 2 every, ...
  double* seg;       // [every][blk]: step-start states of the segment being reversed
  double* fin;       // [blk]: state after the last step
  double* tape;      // [every][9 n]: x0, u0, u after drift/encounters
  Subsystem* tsubs;  // [every][cap_subs]
  int32_t* tnsub;    // [every]
  double* tsched;    // [every][cap_subs][kBsMaxSched][2]
  int32_t* tnsched;  // [every][cap_subs]
  double *lx, *lu, *lmu;  // adjoints of x, u [3][n] and of mu [n_big]
  double* part;      // wave partials
  double* tot;       // reduced partials, then the reductions' block counter
  double* sched;     // [cap_subs][kBsMaxSched][2] written by the forward integrator
  int32_t* nsched;   // [cap_subs]
  double* contrib;   // [cap_subs][28]
  int32_t* kept;     // [n]
  double *m_big, *v_h0;   // start masses [n_big] and heliocentric velocities [3][n]
  double *gm, *gv;        // gradient scratch [n_big], [3][n]
  bool forward_done;
};

namespace {

void free_adjoint(mx_adjoint* a) {
  if (!a) return;
  if (a->s) {
    a->s->owned = false;
    mx_destroy(a->s);
  }
  void* ptrs[] = {a->ckpt, a->seg, a->fin, a->tape, a->tsubs, a->tnsub, a->tsched, a->tnsched,
                  a->lx, a->lu, a->lmu, a->part, a->tot, a->sched, a->nsched, a->contrib,
                  a->kept, a->m_big, a->v_h0, a->gm, a->gv};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete a;
}

// pack (x, u, ag, bigsnap) of the system into dst, or unpack src into it
hipError_t state_copy(mx_adjoint* a, double* buf, int unpack) {
  mx_system* s = a->s;
  const int64_t n3 = 3 * (int64_t)s->n;
  double* ptr[4] = {s->x, s->u, s->ag, s->bigsnap};
  int64_t len[4] = {n3, n3, n3, 9 * (int64_t)s->nb};
  return mxk::adj_copy(s->stream, ptr, len, 4, buf, unpack);
}

hipError_t restore_state(mx_adjoint* a, const double* src, int64_t step) {
  hipError_t e = state_copy(a, const_cast<double*>(src), 1);
  if (e == hipSuccess) e = mxk::launch_reset_scalars(a->s, step);
  return e;
}

// one step from the current state, recording slot q of the tape
hipError_t recorded_step(mx_adjoint* a, int q) {
  mx_system* s = a->s;
  const int64_t n3 = 3 * (int64_t)s->n;
  double* tp = a->tape + (size_t)q * 3 * n3;
  hipError_t e = hipSuccess;
  for (int k = 0; k < MX_NUM_KERNELS && e == hipSuccess; ++k) {
    if (k == MX_K_JUMP_PACK) {
      // after drift and encounters: x0, u0 (pre-drift), u, and the subsystems
      double* ptr[3] = {s->x0, s->u0, s->u};
      int64_t len[3] = {n3, n3, n3};
      e = mxk::adj_record(s->stream, ptr, len, 3, tp, s->subs, s->dsc, a->sched, a->nsched,
                          a->tsubs + (size_t)q * s->cap_subs, a->tnsub + q,
                          a->tsched + (size_t)q * s->cap_subs * kBsMaxSched * 2,
                          a->tnsched + (size_t)q * s->cap_subs);
    }
    if (e == hipSuccess) e = launch_group(s, k);
  }
  return e;
}

// adjoint of the step recorded in slot q, whose start state is `start` and end
// state `end` (saved states: the positions come first)
hipError_t reverse_step(mx_adjoint* a, int q, const double* start, const double* end) {
  mx_system* s = a->s;
  const int n = s->n, nb = s->nb;
  const double h = s->p.dt, hh = 0.5 * h, mu0 = s->mu0;
  const mxd::DragConst dc = mxd::make_drag_const(s->p);
  const size_t n3 = 3 * (size_t)n;
  const double* tp = a->tape + (size_t)q * 3 * n3;
  const double *x0 = tp, *u0 = tp + n3, *ud = tp + 2 * n3, *xe = end;
  hipError_t e;
  // closing half kick at the final positions, with the jump before it
  e = mxk::adj_kick(s->stream, n, nb, mu0, hh, dc, s->p.gas_on, xe, ud, s->mu, s->rcrit, s->r_p,
                    s->rho_p, a->lx, a->lu, a->lmu, a->part, a->tot, hh / mu0);
  if (e != hipSuccess) return e;
  // Kepler drift / encounter integration from the pre-drift state (x0, u0)
  e = mxk::adj_drift(s->stream, n, nb, mu0, h, x0, u0, s->mu, s->rcrit,
                     a->tsubs + (size_t)q * s->cap_subs, a->tnsub + q,
                     a->tsched + (size_t)q * s->cap_subs * kBsMaxSched * 2,
                     a->tnsched + (size_t)q * s->cap_subs, a->kept, a->contrib, a->lx, a->lu,
                     a->lmu, &s->dsc->err);
  if (e != hipSuccess) return e;
  // first jump: x0 = x_a + hh P(u0) / mu0
  e = mxk::adj_momentum(s->stream, n, nb, a->lx, hh / mu0, s->mu, u0, a->lu, a->lmu, a->part,
                        a->tot);
  if (e != hipSuccess) return e;
  // opening half kick at the step-start state
  return mxk::adj_kick(s->stream, n, nb, mu0, hh, dc, s->p.gas_on, start, start + n3, s->mu,
                       s->rcrit, s->r_p, s->rho_p, a->lx, a->lu, a->lmu, a->part, a->tot, 0.0);
}

}  // namespace

extern "C" {

mx_status mx_adjoint_create(const mx_params* p, const double* x_h, const double* v_h,
                            const double* m_big, const double* r_p, const double* rho_p,
                            const double* rcrit, int32_t n_steps, int32_t checkpoint_every,
                            int is_device_ptr, void* hip_stream, mx_adjoint** out) {
  if (!out) return fail(MX_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p || n_steps < 1 || checkpoint_every < 1)
    return fail(MX_EINVAL, "need params, n_steps >= 1 and checkpoint_every >= 1");
  if (p->n_big > kSmallBig) return fail(MX_EINVAL, "the adjoint needs n_big <= 64");
  if (p->temp_1au > 0.0 || p->eta_mode || p->dg_mode)
    return fail(MX_EINVAL, "the adjoint supports the constant aspect-ratio disk with fixed "
                           "eta and no disk gravity");
  if (hip_stream == nullptr) return fail(MX_EINVAL, "the adjoint needs a non-default stream");
  mx_adjoint* a = new mx_adjoint();
  std::memset((void*)a, 0, sizeof(mx_adjoint));
  mx_status st = mx_init_system(p, x_h, v_h, m_big, r_p, rho_p, nullptr, is_device_ptr,
                                hip_stream, &a->s);
  if (st != MX_OK) {
    delete a;
    return st;
  }
  mx_system* s = a->s;
  s->owned = true;
  s->no_joint = true;
  const int n = s->n, nb = s->nb;
  const size_t n3 = 3 * (size_t)n;
  a->n_steps = n_steps;
  a->every = checkpoint_every < n_steps ? checkpoint_every : n_steps;
  a->n_ckpt = (n_steps + a->every - 1) / a->every;
  a->blk = 3 * n3 + 9 * (size_t)nb;
  const size_t nwaves = 4 * (size_t)((n + 255) / 256);
  hipError_t e = hipSuccess;
#define ALLOC(ptr, cnt) \
  if (e == hipSuccess) e = dalloc(&(ptr), (size_t)(cnt));
  const size_t cs = (size_t)s->cap_subs;
  ALLOC(a->ckpt, a->n_ckpt * a->blk) ALLOC(a->seg, a->every * a->blk) ALLOC(a->fin, a->blk)
  ALLOC(a->tape, a->every * 3 * n3) ALLOC(a->tsubs, a->every * cs) ALLOC(a->tnsub, a->every)
  ALLOC(a->tsched, a->every * cs * kBsMaxSched * 2) ALLOC(a->tnsched, a->every * cs)
  ALLOC(a->lx, n3) ALLOC(a->lu, n3) ALLOC(a->lmu, nb)
  ALLOC(a->part, nwaves * (4 * (size_t)kSmallBig + 6)) ALLOC(a->tot, 4 * (size_t)kSmallBig + 7)
  ALLOC(a->sched, (size_t)s->cap_subs * kBsMaxSched * 2) ALLOC(a->nsched, s->cap_subs)
  ALLOC(a->contrib, (size_t)s->cap_subs * 28) ALLOC(a->kept, n) ALLOC(a->m_big, nb)
  ALLOC(a->v_h0, n3) ALLOC(a->gm, nb) ALLOC(a->gv, n3)
#undef ALLOC
  if (e == hipSuccess) e = hipMemsetAsync(a->kept, 0, sizeof(int32_t) * n, s->stream);
  // the sums, then the block counter of the reductions (left at zero by each)
  if (e == hipSuccess)
    e = hipMemsetAsync(a->tot, 0, sizeof(double) * (4 * kSmallBig + 7), s->stream);
  if (e == hipSuccess && nb > 0)
    e = copy_in(a->m_big, m_big, sizeof(double) * nb, is_device_ptr, s->stream);
  if (e == hipSuccess) e = copy_in(a->v_h0, v_h, sizeof(double) * n3, is_device_ptr, s->stream);
  if (e == hipSuccess && rcrit && nb > 0) {
    // changeover radii given by the caller (held fixed, as under differentiation)
    e = copy_in(s->rcrit, rcrit, sizeof(double) * nb, is_device_ptr, s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->rcrit_init, s->rcrit, sizeof(double) * nb, hipMemcpyDeviceToDevice,
                         s->stream);
    if (e == hipSuccess) e = refresh_accel(s);
  }
  if (e == hipSuccess) {
    SysDesc d = make_desc(s);
    d.bs_sched = a->sched;
    d.keep_x0 = 1;
    d.bs_nsched = a->nsched;
    e = hipMemcpy(s->desc, &d, sizeof(SysDesc), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = state_copy(a, a->ckpt, 0);  // the start state
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    free_adjoint(a);
    return hip_fail(e, "adjoint set-up");
  }
  st = read_err(s);
  if (st != MX_OK) {
    free_adjoint(a);
    return st;
  }
  *out = a;
  return MX_OK;
}

mx_status mx_adjoint_forward(mx_adjoint* a, double* x_h, double* v_h, int is_device_ptr) {
  if (!a || !x_h || !v_h) return fail(MX_EINVAL, "NULL argument");
  mx_system* s = a->s;
  HIPCHK(restore_state(a, a->ckpt, 0), "restore start");
  // each segment between checkpoints is one call of joined steps (the closing
  // kernel of a step and the opening kernel of the next as one launch: the same
  // operations per body as single steps, so the same states bit for bit)
  for (int32_t c = 0; c < a->n_ckpt; ++c) {
    const int32_t j0 = c * a->every;
    const int32_t j1 = j0 + a->every < a->n_steps ? j0 + a->every : a->n_steps;
    if (c > 0) HIPCHK(state_copy(a, a->ckpt + (size_t)c * a->blk, 0), "checkpoint");
    HIPCHK(enqueue_steps(s, j1 - j0, true, [](int, int) {}, [](int, int) {}), "steps");
  }
  HIPCHK(state_copy(a, a->fin, 0), "final state");
  s->host_step = a->n_steps;
  mx_status st = read_err(s);
  if (st != MX_OK) return st;
  st = mx_get_state(s, x_h, v_h, is_device_ptr);
  if (st == MX_OK) a->forward_done = true;
  return st;
}

mx_status mx_adjoint_backward(mx_adjoint* a, const double* gx, const double* gv, double* g_m,
                              double* g_x, double* g_v, int is_device_ptr) {
  if (!a || !gx || !gv || !g_x || !g_v || (a->s->nb > 0 && !g_m))
    return fail(MX_EINVAL, "NULL argument");
  if (!a->forward_done) return fail(MX_EINVAL, "call mx_adjoint_forward first");
  mx_system* s = a->s;
  const int n = s->n, nb = s->nb;
  const size_t n3 = 3 * (size_t)n;
  hipStream_t st = s->stream;
  HIPCHK(copy_in(a->lx, gx, n3 * 8, is_device_ptr, st), "copy gx");
  HIPCHK(copy_in(a->lu, gv, n3 * 8, is_device_ptr, st), "copy gv");
  if (nb > 0) HIPCHK(hipMemsetAsync(a->lmu, 0, sizeof(double) * nb, st), "zero lmu");
  // final heliocentric velocities v = u + P / mu0
  HIPCHK(mxk::adj_momentum(st, n, nb, a->lu, 1.0 / s->mu0, s->mu, a->fin + n3, a->lu, a->lmu,
                           a->part, a->tot),
         "final velocities");
  for (int c = a->n_ckpt - 1; c >= 0; --c) {
    const int32_t j0 = c * a->every;
    const int32_t j1 = j0 + a->every < a->n_steps ? j0 + a->every : a->n_steps;
    // forward over the segment, recording every step
    HIPCHK(restore_state(a, a->ckpt + (size_t)c * a->blk, j0), "restore checkpoint");
    for (int32_t j = j0; j < j1; ++j) {
      HIPCHK(state_copy(a, a->seg + (size_t)(j - j0) * a->blk, 0), "segment state");
      HIPCHK(recorded_step(a, j - j0), "recorded step");
    }
    // and back; the state after the segment's last step is the next checkpoint (the
    // recording reproduces the forward run bit for bit) or the final state
    const double* after = c + 1 < a->n_ckpt ? a->ckpt + (size_t)(c + 1) * a->blk : a->fin;
    for (int32_t j = j1 - 1; j >= j0; --j) {
      const double* end = j + 1 < j1 ? a->seg + (size_t)(j + 1 - j0) * a->blk : after;
      HIPCHK(reverse_step(a, j - j0, a->seg + (size_t)(j - j0) * a->blk, end), "adjoint step");
    }
  }
  hipError_t e = mxk::adj_h2dh(st, n, nb, s->p.G, s->p.m0, a->m_big, a->v_h0, a->lu, a->lmu,
                               a->gm, a->gv, a->part, a->tot);
  if (e == hipSuccess) e = copy_out(g_x, a->lx, n3 * 8, is_device_ptr, st);
  if (e == hipSuccess) e = copy_out(g_v, a->gv, n3 * 8, is_device_ptr, st);
  if (e == hipSuccess && nb > 0) e = copy_out(g_m, a->gm, sizeof(double) * nb, is_device_ptr, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "adjoint output");
  // leave the system at its final state
  HIPCHK(restore_state(a, a->fin, a->n_steps), "restore final");
  return read_err(s);
}

mx_status mx_adjoint_system(mx_adjoint* a, mx_system** view) {
  if (!a || !view) return fail(MX_EINVAL, "NULL argument");
  *view = a->s;
  return MX_OK;
}

void mx_destroy_adjoint(mx_adjoint* a) {
  if (!a) return;
  (void)hipStreamSynchronize(a->s->stream);
  free_adjoint(a);
}

}  // extern "C"
