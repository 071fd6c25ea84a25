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

#include <vector>

#include "mx_internal.h"

namespace mxk {
int force_split(int n, int nb);
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

void free_system(mx_system* s) {
  if (!s) return;
  if (s->graph_ok) (void)hipGraphExecDestroy(s->graph);
  for (int32_t k = 0; k < s->tev_pool_n; ++k) (void)hipEventDestroy(s->tev_pool[k]);
  delete[] s->tev_pool;
  void* ptrs[] = {s->x, s->u, s->ag, s->x0, s->u0, s->mu, s->rcrit, s->mu_init, s->rcrit_init,
                  s->growth, s->r_p, s->rho_p, s->bigsnap, s->bigmid, s->kpack, s->fpack, s->part,
                  s->pairs, s->pairs_tmp, s->plan_idx, s->subs, s->uf, s->dsc, s->red};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete s;
}

// kernel group k of one step (MX_K_* order); the fused small-B path runs its
// flagging inside the first kernel and its jump inside the last
hipError_t launch_group(mx_system* s, int k) {
  const bool small = s->nb <= kSmallBig;
  switch (k) {
    case MX_K_GROWTH: return mxk::launch_growth(s);
    case MX_K_KICK_JUMP_DRIFT:
      return small ? mxk::launch_step_a_small(s) : mxk::launch_kick_jump_drift(s);
    case MX_K_FLAG: return small ? hipSuccess : mxk::launch_flag(s);
    case MX_K_PLAN: return mxk::launch_plan(s);
    case MX_K_BS: return mxk::launch_bs(s);
    case MX_K_JUMP_PACK: return small ? hipSuccess : mxk::launch_jump_pack(s);
    default: return small ? mxk::launch_step_b_small(s, 1) : mxk::launch_force_kick(s, 1);
  }
}

hipError_t enqueue_step(mx_system* s) {
  for (int k = 0; k < MX_NUM_KERNELS; ++k) {
    hipError_t e = launch_group(s, k);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// FSAL gravity at the current positions (no kick)
hipError_t refresh_accel(mx_system* s) {
  hipError_t e;
  if ((e = mxk::launch_pack_only(s)) != hipSuccess) return e;
  return mxk::launch_force_kick(s, 0);
}

mx_status read_err(mx_system* s) {
  int32_t err = 0;
  HIPCHK(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
  HIPCHK(hipMemcpy(&err, &s->dsc->err, sizeof(int32_t), hipMemcpyDeviceToHost), "read err");
  if (err) {
    int32_t zero = 0;
    HIPCHK(hipMemcpy(&s->dsc->err, &zero, sizeof(int32_t), hipMemcpyHostToDevice), "clear err");
    if (err & MXE_NONFINITE) return fail(MX_ENONFINITE, "non-finite state after a step");
    if (err & MXE_NOCONV) return fail(MX_ENOCONV, "Kepler iteration did not converge");
    if (err & MXE_BS) return fail(MX_EBS, "Bulirsch-Stoer step-halving limit reached");
    if (err & (MXE_PAIRS | MXE_SUBSYS)) return fail(MX_ECAPACITY, "encounter capacity exceeded");
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
  s->split = mxk::force_split(s->n, nb);
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
  ALLOC(s->bigsnap, 9 * (size_t)nb) ALLOC(s->bigmid, 6 * (size_t)nb)
  ALLOC(s->kpack, nb) ALLOC(s->fpack, nb)
  ALLOC(s->part, s->split > 1 ? (size_t)s->split * n3 : 1)
  ALLOC(s->pairs, 2 * (size_t)s->cap_pairs) ALLOC(s->pairs_tmp, 4 * (size_t)s->cap_pairs)
  ALLOC(s->plan_idx, 2 * (size_t)s->cap_pairs)
  ALLOC(s->subs, s->cap_subs) ALLOC(s->uf, 2 * (size_t)nb) ALLOC(s->dsc, 1) ALLOC(s->red, s->red_blocks)
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
  STEP(dalloc(&vh_tmp, n3), "alloc v_h");
  STEP(hipMemsetAsync(s->dsc, 0, sizeof(DevScalars), sm), "memset");
  STEP(hipMemsetAsync(s->ag, 0, sizeof(double) * n3, sm), "memset");
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
  for (int32_t k = 0; k < n_steps; ++k) {
    if (use_graph) HIPCHK(hipGraphLaunch(s->graph, s->stream), "graph launch");
    else HIPCHK(enqueue_step(s), "step launch");
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

mx_status mx_step_timed(mx_system* s, int32_t n_steps, int32_t group, float* kernel_ms,
                        int32_t* n_launched) {
  if (!s || n_steps < 0 || group < 0 || group >= MX_NUM_KERNELS || !kernel_ms || !n_launched)
    return fail(MX_EINVAL, "bad argument");
  *n_launched = 0;
  if (n_steps == 0) return MX_OK;
  if (n_steps > (1 << 24)) return fail(MX_EINVAL, "too many timed steps in one call");
  hipError_t e = hipSuccess;
  if (s->tev_pool_n < 2 * n_steps) {  // grow the event pool (kept for later calls)
    hipEvent_t* pool = new hipEvent_t[2 * (size_t)n_steps];
    int32_t k = 0;
    for (; k < s->tev_pool_n; ++k) pool[k] = s->tev_pool[k];
    for (; k < 2 * n_steps && e == hipSuccess; ++k) e = hipEventCreate(&pool[k]);
    if (e != hipSuccess) --k;  // pool[k] was not created
    delete[] s->tev_pool;
    s->tev_pool = pool;
    s->tev_pool_n = k;
    if (e != hipSuccess) return hip_fail(e, "event create");
  }
  hipEvent_t* ev = s->tev_pool;
  std::vector<char> used(n_steps, 0);
  for (int32_t q = 0; q < n_steps && e == hipSuccess; ++q) {
    for (int k = 0; k < MX_NUM_KERNELS && e == hipSuccess; ++k) {
      if (k == group) {
        s->tev_armed = true;
        s->tev_start = ev[2 * q];
        s->tev_stop = ev[2 * q + 1];
      }
      e = launch_group(s, k);
      if (k == group) {
        used[q] = s->tev_start == nullptr;  // the start event went to a kernel
        s->tev_armed = false;
        s->tev_start = s->tev_stop = nullptr;
      }
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  int32_t nl = 0;
  for (int32_t q = 0; q < n_steps; ++q) {
    float ms = 0.f;
    if (e == hipSuccess && used[q]) {
      e = hipEventElapsedTime(&ms, ev[2 * q], ev[2 * q + 1]);
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
  int m = d.n_pairs_last < cap ? d.n_pairs_last : cap;
  if (m > s->cap_pairs) m = s->cap_pairs;
  if (m > 0) HIPCHK(hipMemcpy(pairs, s->pairs, sizeof(int32_t) * 2 * m, hipMemcpyDeviceToHost), "copy pairs");
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
  if (s->has_growth) {
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

void mx_destroy(mx_system* s) {
  if (!s) return;
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
