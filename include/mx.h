/*
 * mx -- MI355X (gfx950) hybrid symplectic step: C ABI.
 *
 * One hybrid step of the Mercury+ integrator (Mercury-Arxes, Sect. 2): a
 * changeover-weighted kick of every body by the massive ("big") bodies, the
 * gas-drag acceleration of the massless bodies (Sect. 3.1, Eqs. 1-7), a jump by
 * the massive-body momentum, a Kepler drift of every body in democratic-
 * heliocentric coordinates, close-encounter flagging of big/any pairs (the
 * mce_snif region of Sect. 2.1.2) and a Bulirsch-Stoer hand-off of the flagged
 * subsystems ("BS for conservative forces", Sect. 2.1).
 *
 * Conventions (every entry point):
 *  - Units: AU, day, solar mass; G is given in mx_params.
 *  - Bodies: n = n_big + n_small non-star bodies, big bodies first.  The star is
 *    not an array element.  Vectors are structure-of-arrays double[3][n]
 *    (x coordinates of all bodies, then y, then z).
 *  - Pointers marked "host or device" follow is_device_ptr: 0 = host memory,
 *    1 = device memory on the current HIP device.  Inputs are copied; the library
 *    never keeps a caller pointer after the call returns.
 *  - Work is queued on the stream given at init (a hipStream_t; NULL = the null
 *    stream, which disables graph replay).  Calls that return host values
 *    synchronise that stream.
 *  - Every call returns an mx_status.  MX_EINVAL and MX_ECAPACITY leave the
 *    system unchanged.  Device-side failures (MX_ENOCONV, MX_EBS, MX_ENONFINITE,
 *    MX_ECAPACITY of a step) are latched on the device and reported by the next
 *    synchronising call.  mx_last_error() gives a thread-local message.
 */
#ifndef MX_H
#define MX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mx_system mx_system; /* opaque; owned by the library */
typedef struct mx_batch mx_batch;   /* opaque; many independent systems stepped together */
typedef struct mx_adjoint mx_adjoint; /* opaque; a differentiable run of one system */

typedef enum {
  MX_OK = 0,
  MX_EINVAL = -1,      /* bad argument (sizes, NULL where required, non-positive mass) */
  MX_ENOMEM = -2,      /* device or host allocation failed */
  MX_EHIP = -3,        /* a HIP runtime call failed */
  MX_ENOCONV = -4,     /* Kepler iteration cap reached */
  MX_EBS = -5,         /* Bulirsch-Stoer step-halving limit reached */
  MX_ENONFINITE = -6,  /* non-finite position or velocity after a step */
  MX_ECAPACITY = -7    /* encounter list or subsystem table overflow */
} mx_status;

/* Physical and numerical parameters, all double precision unless stated.
 * Gas-disk fields follow Sect. 3.1: Sigma(R) = sigma1 (R/1AU)^-gamma, tapered by
 * exp[(1/r_c)^(2-gamma) - (R/r_c)^(2-gamma)] when r_c > 0 (Eq. 1 normalised to
 * sigma1 at 1 AU), zero inside r_in; scale height h = (H/r) R; sub-Keplerian
 * gas speed v_k sqrt(1 - 2 eta) (Eq. 5); drag coefficient of Eq. 7 with its
 * first bracket raised to kdrag_exp (printed as -2). */
typedef struct {
  double G;           /* AU^3 Msun^-1 day^-2 */
  double m0;          /* stellar mass, Msun */
  double dt;          /* step, day (may be negative) */
  double rcrit_hill;  /* changeover radius in Hill radii */
  double bs_tol;      /* Bulirsch-Stoer relative tolerance */
  int32_t n_big;      /* massive bodies (>= 0) */
  int32_t n_small;    /* massless bodies (>= 0) */
  int32_t gas_on;     /* 1: gas drag on the massless bodies */
  int32_t pad;
  double sigma1;      /* gas surface density at 1 AU, g cm^-2 */
  double gamma;       /* surface-density slope */
  double r_c;         /* taper radius, AU; 0 = none */
  double r_in;        /* inner edge, AU */
  double h_over_r;    /* aspect ratio */
  double eta;         /* sub-Keplerian parameter */
  double kdrag_exp;   /* exponent of the first bracket of Eq. 7 */
  double rho_unit;    /* Msun AU^-3 per g cm^-3 */
  double au_cm;       /* cm per AU */
  double mfp_coef;    /* mean free path lambda[AU] = mfp_coef / rho_gas[Msun AU^-3] */
  /* Further disk physics of Sect. 3.1 (all off when zero): */
  double temp_1au;    /* midplane temperature at 1 AU, K (Eq. 2); 0 = c_s = h_over_r v_K */
  double temp_beta;   /* slope beta of T = temp_1au (R / 1 AU)^-beta */
  double cs2_per_k;   /* isothermal c_s^2 per kelvin, AU^2 day^-2 K^-1 (k_B / mu m_H) */
  int32_t eta_mode;   /* 1: eta(R) of Eq. 6 (gamma_C = 7/5) instead of the fixed eta */
  int32_t dg_mode;    /* 1: disk gravity of Eqs. 10-12 on the massless bodies, as the
                         signed radial acceleration (positive away from the star):
                         2 pi G Sigma S(gamma) for gamma != 1 (0 < gamma < 2), and
                         2 pi G Sigma r_in / R for gamma = 1 */
} mx_params;

/* ---------------------------------------------------------------- system */

/* Create a system from heliocentric states (Sect. 2: the DH transform of
 * mco_h2dh).  x_h, v_h: [3][n] host or device.  m_big: [n_big] masses (Msun, each
 * > 0) host or device.  r_p, rho_p: [n_small] radius (AU) and density (g cm^-3) of
 * each massless body, host or device; required when gas_on.  growth: NULL, or
 * [n_big][3] = (M0, Mc [Msun], tau_c [day]) per big body, the core-growth law of
 * Eq. 13 applied at each step start (tau_c <= 0: fixed mass), host or device.
 * hip_stream: hipStream_t used for all work.  The changeover radius of big body k
 * is rcrit_hill * a_k (m_k / 3 m0)^(1/3), a_k its osculating semi-major axis
 * (|x_k| if unbound).  On success *out owns all device memory of the system. */
mx_status mx_init_system(const mx_params* p, const double* x_h, const double* v_h,
                         const double* m_big, const double* r_p, const double* rho_p,
                         const double* growth, int is_device_ptr, void* hip_stream,
                         mx_system** out);

/* Queue n_steps hybrid steps (Sect. 2; kick listing of Sect. 2.1.2, direct force
 * of Sect. 2.1.3).  Asynchronous; device failures surface at the next sync.
 * Kernels are launched one by one (MX_LAUNCH_EAGER, the default) or as one
 * captured HIP graph per step (MX_LAUNCH_GRAPH); both run the same kernels on
 * the same data and give bitwise identical states. */
mx_status mx_step(mx_system* s, int32_t n_steps);

enum { MX_LAUNCH_EAGER = 0, MX_LAUNCH_GRAPH = 1 };

/* Select how mx_step launches a step (see above).  The graph is captured on the
 * first graph-mode step and kept until destroy. */
mx_status mx_set_launch_mode(mx_system* s, int32_t mode);

/* Kernels of one step, in launch order (indices into kernel_ms below). */
enum {
  MX_K_GROWTH = 0,          /* core-growth mass schedule (no-op without growth) */
  MX_K_KICK_JUMP_DRIFT = 1, /* half kick + gas drag + jump + Kepler drift (with n_big <= 64
                               also the close-encounter flagging) */
  MX_K_FLAG = 2,            /* close-encounter flagging (empty with n_big <= 64) */
  MX_K_PLAN = 3,            /* empty: the encounter integrator sorts the list and plans its
                               subsystems itself */
  MX_K_BS = 4,              /* subsystem plan + Bulirsch-Stoer integration of the subsystems */
  MX_K_JUMP_PACK = 5,       /* second jump, source packing (empty with n_big <= 64: the jump
                               is done by the force kernel) */
  MX_K_FORCE_KICK = 6,      /* changeover-weighted gravity + gas drag + half kick */
  MX_NUM_KERNELS = 7,
  MX_K_STEP_JOINED = 7,     /* mx_step_timed only: the single launch that closes one step and
                               opens the next between the steps of a call (n_big <= 64 without
                               time-dependent masses); never launched in the last step */
  MX_K_STEP_JOINT = 8       /* mx_step_timed only: the launch that integrates the encounters of
                               one step beside the closing of that step and the opening of the
                               next, between the steps of a call (single systems with
                               0 < n_big <= 64 without time-dependent masses: what mx_step
                               launches there); never launched in the last step */
};

/* Same as mx_step, launched without the graph and with a HIP event around each
 * kernel group on the system stream; kernel_ms[MX_NUM_KERNELS] (host) receives the
 * summed event time of each group over the n_steps.  Synchronises every step. */
mx_status mx_step_profiled(mx_system* s, int32_t n_steps, double* kernel_ms);

/* Runs n_steps steps with eager launches (no graph) and times one kernel group
 * (an MX_K_* value, MX_K_STEP_JOINED or MX_K_STEP_JOINT) with HIP events bound to its
 * kernels' own
 * start and end, in
 * every stride-th step (steps 0, stride, 2 stride, ...; stride >= 1, else
 * MX_EINVAL): kernel_ms[q] (host, [n_steps]) is the time from the start of the
 * group's first kernel to the end of its last in step q, 0 where step q was not
 * timed or the group launched nothing; *n_launched counts the timed steps where
 * it launched.  An event recorded between two kernels delays the second, so a
 * stride above 1 keeps the other steps' launches as mx_step issues them.
 * Synchronises. */
mx_status mx_step_timed(mx_system* s, int32_t n_steps, int32_t group, int32_t stride,
                        float* kernel_ms, int32_t* n_launched);

/* Cumulative work counters of the system since init: FP64 operations of the
 * encounter integrator (a model count per force evaluation and extrapolation
 * entry, FMA = 2) and encounter pairs flagged.  Host pointers.  Synchronises. */
mx_status mx_get_counters(mx_system* s, uint64_t* bs_flop, uint64_t* pairs_flagged);

/* Wait for queued work and report any latched device failure (clears it). */
mx_status mx_sync(mx_system* s);

/* Energy with the potential over massive bodies only (the mxx_en change of
 * Sect. 2.1.3) and total angular momentum.  E: Msun AU^2 day^-2; L: Msun AU^2
 * day^-1 (host pointers).  Synchronises. */
mx_status mx_energy(mx_system* s, double* E, double L[3]);

/* Flagged pairs of the last step, sorted by (i, j), i < n_big, i < j < n
 * (the ice/jce list of Sect. 2.1.2).  pairs: host [cap][2]; *n_out receives the
 * total count (may exceed cap).  Synchronises. */
mx_status mx_encounters(mx_system* s, int32_t* pairs, int32_t cap, int32_t* n_out);

/* Heliocentric state (mco_dh2h) / its replacement.  set_state also recomputes
 * the stored end-of-step gravity and sets the step counter to step_index. */
mx_status mx_get_state(mx_system* s, double* x_h, double* v_h, int is_device_ptr);
mx_status mx_set_state(mx_system* s, const double* x_h, const double* v_h, int is_device_ptr,
                       int64_t step_index);

/* Democratic-heliocentric state (positions, barycentric velocities), exact copy. */
mx_status mx_get_state_dh(mx_system* s, double* x, double* u, int is_device_ptr);
mx_status mx_set_state_dh(mx_system* s, const double* x, const double* u, int is_device_ptr,
                          int64_t step_index);

/* Stored changeover-weighted gravity [3][n] (reused by the next half kick). */
mx_status mx_get_accel(mx_system* s, double* a, int is_device_ptr);

/* Current mu = G m and rcrit of the big bodies, host [n_big] each.  Synchronises. */
mx_status mx_get_masses(mx_system* s, double* mu, double* rcrit);

/* Steps taken so far (the step counter). */
mx_status mx_get_step_index(mx_system* s, int64_t* step_index);

/* Time-dependent physics of one massive body (Sects. 3.2-3.3, 3.1 gaps): masses
 * in Msun, times in days, lengths in AU. */
typedef struct {
  double M0, Mc, tau_c; /* core growth, Eq. 13 (tau_c <= 0: fixed mass, no later phase) */
  double Mf, tau_g;     /* runaway gas accretion for t >= tau_c, Eq. 15 (tau_g <= 0: Mc) */
  double R_I;           /* radius after the collapse, Eq. 16 (Delta R = R_c - R_I) */
  double da1, tau1;     /* linear migration, Eq. 17 (tau1 <= 0: none) */
  double da2, tau2;     /* second migration phase, Eq. 18 (tau2 <= 0: none) */
  double gap_C;         /* gap half width in Hill radii, Eq. 8 (the paper's C = 4; 0: no gap) */
} mx_planet;

/* Install the time-dependent physics of the massive bodies (n_big <= 64, a single
 * system; replaces a growth schedule given at init).  planets: host [n_big].  At the
 * start of each step, at its time t, held through the step:
 *  - mass of Eq. 13 for t < tau_c, then of Eq. 15 (or Mc), and rcrit scaled by the
 *    cube root of the mass (Hill radius);
 *  - radius of Eq. 14 (k1 = 1, k2 = 1/4, c_s of the disk at the body's cylindrical
 *    distance, R_H = r (m / 3 m0)^(1/3) at its distance r), from tau_c on Eq. 16
 *    with R_c the Eq. 14 radius at the first step of the runaway;
 *  - migration: a change of the velocity along the heliocentric velocity by
 *    Eq. 17 for t < tau1 and by Eq. 18 after (a_p the osculating semi-major axis,
 *    v_k = sqrt(G (m0 + m) / a_p), Delta t the step);
 *  - gap (after tau_c, with tau_g > 0 and gap_C > 0): massless bodies strictly
 *    within gap_C R_H of the body's cylindrical distance see the drag density times
 *    exp(-(t - tau_c)/tau_g) (Eqs. 8-9; the highest-index gap wins);
 *  - step switch (Sect. 3.6; a_switch > 0): once a migrating body's a_p <= a_switch
 *    the step becomes 1/25 of the orbital period at a_min, from that step on.
 * The time advances by the step actually taken.  mx_set_state / mx_set_state_dh
 * restart the clock at step_index * dt with the initial step and forget R_c.
 * MX_EINVAL for n_big > 64, n_big = 0 or a_switch > 0 without a_min > 0.
 * Synchronises. */
mx_status mx_set_planet_physics(mx_system* s, const mx_planet* planets, double a_switch,
                                double a_min);

/* Radii of the massive bodies from the last step (0 before any step with physics),
 * host [n_big]; the time at the start of the next step and the current step size,
 * host scalars.  Synchronise. */
mx_status mx_get_planet_radii(mx_system* s, double* radius);
mx_status mx_get_time(mx_system* s, double* t, double* h);

/* Body removal (single systems).  mx_check_removal flags, among the bodies not yet
 * flagged: the ejection criterion of Sect. 3.5, e >= 1 of the osculating orbit
 * about the star (gm = G(m0 + m) for massive bodies, G m0 for massless ones;
 * heliocentric state) -> status -3; with r_cen > 0 the central-body encounters
 * (the mce_cent routine of Sect. 4.1, whose test the paper does not print): the
 * distance from the star <= r_cen, or a pericentre passage since the previous
 * check (radial velocity inward then, outward or zero now) on an orbit of
 * perihelion distance q = |h|^2 / (gm (1 + e)) <= r_cen -> status -2.  A flagged
 * massive body keeps its place with zero mass and zero changeover radius, its
 * growth, migration and gap switched off (the force stored for the next half kick
 * still has it).  *ejcount (host) receives the number of bodies with status < 0,
 * the workshare count of Sect. 2.1.2.  Synchronises. */
mx_status mx_check_removal(mx_system* s, double r_cen, int32_t* ejcount);

/* Removes the flagged massless bodies (stable: the others keep their order) on the
 * device; massive bodies keep their places.  *n_removed (host) the number removed;
 * index_map: host [n before the call] receiving each body's new index or -1, or
 * NULL.  The system then has fewer massless bodies (mx_get_counts); the state and
 * stored force of the survivors are unchanged.  Synchronises. */
mx_status mx_compact(mx_system* s, int32_t* n_removed, int32_t* index_map);

/* Status of every body (0, -2, -3), host [n]; current body counts.  Synchronise. */
mx_status mx_get_status(mx_system* s, int32_t* stat);
mx_status mx_get_counts(mx_system* s, int32_t* n_big, int32_t* n_small);

void mx_destroy(mx_system* s);
const char* mx_last_error(void);

/* ---------------------------------------------------------------- batches
 * Many independent systems stepped together: every launch of a step covers all
 * systems (the fused small-B kernels walk one table of body tiles of all the
 * systems, the planner runs one block per system, the encounter integrator a
 * grid of bs_blocks x n_sys).  Each system computes exactly what mx_step computes
 * for it alone, with bitwise identical results whatever the configuration.
 * Every system needs n_big <= 64; growth schedules are not supported here. */

/* params: host [n_sys] (n_big, n_small of each); offsets: host [n_sys + 1] body
 * offsets, offsets[0] = 0, offsets[k+1] - offsets[k] = n_big + n_small of system
 * k.  x_h, v_h: concatenated SoA [3][N], N = offsets[n_sys], system k in columns
 * offsets[k] .. offsets[k+1] (big bodies first), heliocentric.  m_big: the
 * systems' n_big masses one after the other; r_p, rho_p: the systems' massless
 * bodies one after the other (NULL allowed when no system has gas).  Host or
 * device pointers per is_device_ptr, read during the call only.  Systems share
 * hip_stream.  Each system is initialised as mx_init_system would. */
mx_status mx_init_batch(int32_t n_sys, const mx_params* params, const int64_t* offsets,
                        const double* x_h, const double* v_h, const double* m_big,
                        const double* r_p, const double* rho_p, int is_device_ptr,
                        void* hip_stream, mx_batch** out);

/* Queue n_steps steps of every system.  Eager launches, or in graph mode one
 * captured HIP graph of steps_per_graph whole steps replayed as often as it fits
 * (the rest eagerly).  Asynchronous. */
mx_status mx_step_batch(mx_batch* b, int32_t n_steps);
mx_status mx_batch_set_launch_mode(mx_batch* b, int32_t mode, int32_t steps_per_graph);

/* Launch shape: blk bodies per tile (64, 128, 256 or 512), tiles_per_block
 * consecutive tiles per workgroup (1..64; the massive bodies of a system are
 * advanced once per workgroup and system), bs_blocks encounter-integrator
 * workgroups per system (1..1024).  cfg (host [3]) receives the same triple. */
mx_status mx_batch_set_config(mx_batch* b, int32_t blk, int32_t tiles_per_block,
                              int32_t bs_blocks);
mx_status mx_batch_get_config(mx_batch* b, int32_t* cfg);

/* Autotuner: runs real steps of the batch (steps_per_candidate per candidate;
 * every candidate gives the same results) with HIP events around each step's
 * kernels: the tile shapes are judged by the time of the body kernels, then the
 * encounter-integrator widths 8..64 by the integrator's time (each width tried
 * twice, in mirrored order, and judged by the sum), and the fastest of each is
 * kept.  *steps_taken (host) is the number of steps it advanced; cfg_out (host
 * [3]) the chosen triple; *best_ms the kernel time per step of the choice.
 * Synchronises and reports device failures. */
mx_status mx_batch_autotune(mx_batch* b, int32_t steps_per_candidate, int32_t* steps_taken,
                            int32_t* cfg_out, float* best_ms);

/* Wait for queued work; reports the first system with a latched failure. */
mx_status mx_batch_sync(mx_batch* b);

/* Borrowed view of system k for the per-system calls (energy, encounters, state,
 * step index, and mx_step to advance that system alone).  Owned by the batch:
 * mx_destroy on it does nothing. */
mx_status mx_batch_system(mx_batch* b, int32_t k, mx_system** view);

void mx_destroy_batch(mx_batch* b);

/* ---------------------------------------------------------------- adjoint
 * Reverse-mode derivative of a run of n_steps hybrid steps of one system
 * (n_big <= 64, no growth schedule) with respect to the massive-body masses and
 * the initial heliocentric state of every body.  The run is the map of mx_step;
 * its adjoint takes every sub-step back in reverse order: the half kicks (the
 * changeover-weighted gravity of Sect. 2.1.3 and its mass dependence, the gas
 * drag of Sect. 3.1 with its regime held at the value), the jumps by the
 * massive-body momentum, the Kepler drift (derivative through the solved time
 * equation) and the Bulirsch-Stoer integration of encounter subsystems of up to
 * four members (derivative of the map along the accepted step sizes and
 * columns of the forward run).  The changeover radii are constants of the map.
 * The forward run keeps its state every checkpoint_every steps; the reverse pass
 * recomputes each segment forward from its checkpoint.  Storage: about
 * (n_steps / checkpoint_every + checkpoint_every) x 72 n bytes on the device. */

/* As mx_init_system (no growth); rcrit: changeover radii [n_big] to use instead
 * of the Hill-radius rule (host or device per is_device_ptr), or NULL.  hip_stream
 * must not be the default stream. */
mx_status mx_adjoint_create(const mx_params* p, const double* x_h, const double* v_h,
                            const double* m_big, const double* r_p, const double* rho_p,
                            const double* rcrit, int32_t n_steps, int32_t checkpoint_every,
                            int is_device_ptr, void* hip_stream, mx_adjoint** out);

/* Runs the n_steps from the initial state (again at every call); x_h, v_h
 * ([3][n], host or device) receive the final heliocentric state.  Synchronises. */
mx_status mx_adjoint_forward(mx_adjoint* a, double* x_h, double* v_h, int is_device_ptr);

/* Given gx, gv = dL/d(final x_h, v_h) ([3][n]), writes g_m = dL/dm ([n_big],
 * masses in Msun) and g_x, g_v = dL/d(initial x_h, v_h) ([3][n]).  Needs a
 * completed mx_adjoint_forward; leaves the system at the final state.  Reports
 * MX_ECAPACITY when an encounter subsystem had more than four members or more
 * than 64 accepted Bulirsch-Stoer steps.  Synchronises. */
mx_status mx_adjoint_backward(mx_adjoint* a, const double* gx, const double* gv, double* g_m,
                              double* g_x, double* g_v, int is_device_ptr);

/* Borrowed view of the system being differentiated (masses, radii, energy). */
mx_status mx_adjoint_system(mx_adjoint* a, mx_system** view);

void mx_destroy_adjoint(mx_adjoint* a);

/* -------------------------------------------- single-kernel entry points
 * Stateless launches of one kernel of the step on device pointers, queued on
 * hip_stream.  They exist so that each kernel can be checked on its own. */

/* Changeover-weighted gravity (Sect. 2.1.3): a[t] = sum_{s<n_big, s!=t} mu_s K /r^3
 * (x_s - x_t), rc = max(rcrit_s, rcrit_t) (rcrit_t = 0 for t >= n_big).
 * x, a: device [3][n]; mu, rcrit: device [n_big]. */
mx_status mx_gravity(int32_t n, int32_t n_big, const double* x, const double* mu,
                     const double* rcrit, double* a, void* hip_stream);

/* Gas acceleration (Sect. 3.1: drag of Eqs. 1-7, and with dg_mode the disk gravity of
 * Eqs. 10-12) on bodies t >= n_big; a[t] = 0 for big bodies.
 * u: barycentric velocities; mu: device [n_big] (for the heliocentric shift);
 * r_p: AU; rho_p: Msun AU^-3.  All device pointers. */
mx_status mx_gas_drag(const mx_params* p, int32_t n, int32_t n_big, const double* x,
                      const double* u, const double* mu, const double* r_p,
                      const double* rho_p, double* a, void* hip_stream);

/* Kepler drift of n bodies about mu0 over h (universal variables).
 * x0, u0, x1, u1: device [3][n]; x1/u1 may alias x0/u0.  Reports MX_ENOCONV. */
mx_status mx_kepler_drift(int32_t n, double mu0, double h, const double* x0,
                          const double* u0, double* x1, double* u1, void* hip_stream);

/* Encounter flagging: pairs (i < n_big, i < j < n) whose minimum separation over
 * [0, h] (cubic Hermite interpolant of the relative motion) is <= max(rcrit).
 * pairs: device [cap][2], sorted by (i, j) on return; *n_out (host) total count.
 * Synchronises hip_stream. */
mx_status mx_flag_pairs(int32_t n, int32_t n_big, const double* rcrit, const double* x0,
                        const double* u0, const double* x1, const double* u1, double h,
                        int32_t* pairs, int32_t cap, int32_t* n_out, void* hip_stream);

/* For callers that cannot allocate (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): mx_flag_pairs with the same arguments, results
 * and errors, whose scratch (counters, packed records of the massive bodies, sort
 * keys) is a fixed device array of about 1.5 MiB that the library holds on each
 * device it runs on until the process ends; it calls no hipMalloc, hipFree or
 * allocating library routine.  Limits: n_big <= 4096 and cap <= 65536, else
 * MX_ECAPACITY.  The array keeps the last call's contents and is cleared where
 * needed at each call; calls that overlap on one device (other streams or
 * threads) share it and race.  Synchronises hip_stream. */
mx_status mx_flag_pairs_noalloc(int32_t n, int32_t n_big, const double* rcrit, const double* x0,
                                const double* u0, const double* x1, const double* u1, double h,
                                int32_t* pairs, int32_t cap, int32_t* n_out, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
