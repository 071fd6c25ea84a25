/*
 * CPU oracle of the hybrid symplectic step (TEST INFRASTRUCTURE ONLY).
 *
 * Plain, slow, double-precision C written from the paper's description of the
 * Mercury+ hybrid integrator and the Arxes gas-drag model.  It exists to check the
 * HIP path: only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header or constant table with the
 * HIP library, and it is never called by the product path.
 *
 * Coordinates: democratic-heliocentric (heliocentric positions x, barycentric
 * velocities u).  Arrays are structure-of-arrays [3][n] with the n non-star bodies,
 * massive ("big") bodies first.  Masses are held as mu = G*m.
 */
#ifndef ORACLE_H
#define ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double G, m0, dt, rcrit_hill, bs_tol;
  int32_t n_big, n_small, gas_on, pad;
  double sigma1, gamma, r_c, r_in, h_over_r, eta;
  double kdrag_exp, rho_unit, au_cm, mfp_coef;
  /* Sect. 3.1 extensions: midplane temperature T = temp_1au (R/1 AU)^-temp_beta
   * (Eq. 2; temp_1au = 0 keeps c_s = h_over_r v_k), isothermal c_s^2 = cs2_per_k T;
   * eta_mode 1: eta(R) of Eq. 6 instead of the fixed eta; dg_mode 1: disk gravity
   * (Eqs. 10-12) on the massless bodies.                                      */
  double temp_1au, temp_beta, cs2_per_k;
  int32_t eta_mode, dg_mode;
} or_params;

typedef struct or_sys or_sys;

/* Time-dependent physics of one massive body (Sects. 3.1-3.3): growth, radius,
 * migration and its gap.  Masses in Msun, times in days, lengths in AU. */
typedef struct {
  double M0, Mc, tau_c; /* core growth, Eq. 13 (tau_c <= 0: fixed mass, no later phase) */
  double Mf, tau_g;     /* runaway gas accretion after tau_c, Eq. 15 (tau_g <= 0: held at Mc) */
  double R_I;           /* radius reached by the collapse of Eq. 16 */
  double da1, tau1;     /* first migration phase, Eq. 17 (tau1 <= 0: none) */
  double da2, tau2;     /* second migration phase, Eq. 18 (tau2 <= 0: none) */
  double gap_C;         /* gap width in Hill radii, Eq. 8 (0: no gap) */
} or_planet;

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2, OR_ENOCONV = -4, OR_EBS = -5 };

/* --- whole-system API -------------------------------------------------- */
or_sys* or_create(const or_params* p, const double* x_h, const double* v_h,
                  const double* m_big, const double* r_p, const double* rho_p,
                  const double* growth /* [n_big][3] or NULL */, int* status);
void or_destroy(or_sys* s);
int or_step(or_sys* s, int n_steps);
void or_energy(const or_sys* s, double* E, double L[3]);
int or_encounters(const or_sys* s, int32_t* pairs, int cap);
void or_get_state(const or_sys* s, double* x_h, double* v_h);
void or_get_dh(const or_sys* s, double* x, double* u);
void or_set_dh(or_sys* s, const double* x, const double* u, long step_index);
void or_get_accel(const or_sys* s, double* a);  /* FSAL gravity (changeover-weighted) */
void or_get_mu(const or_sys* s, double* mu, double* rcrit);
void or_set_rcrit(or_sys* s, const double* rcrit);
long or_step_index(const or_sys* s);
double or_last_pair_dmin2(const or_sys* s, int i, int j, double* rc2);
int or_threads(void);
int or_set_physics(or_sys* s, const or_planet* pl, double a_switch, double a_min);
void or_get_radii(const or_sys* s, double* radius);
double or_time(const or_sys* s);
double or_step_size(const or_sys* s);
void or_set_xu(or_sys* s, const double* x, const double* u);
void or_get_gaps(const or_sys* s, double* g);
or_sys* or_clone(const or_sys* s);
int or_check_removal(or_sys* s, double r_cen);
int or_compact(or_sys* s, int32_t* index_map);
void or_get_status(const or_sys* s, int32_t* stat);
int or_n_bodies(const or_sys* s);

/* --- component functions (pins and kernel-level parity) --------------- */
double or_changeover(double s, double rc);
void or_gravity(int n, int n_big, const double* x, const double* mu, const double* rcrit,
                double* a);
void or_drag(const or_params* p, int n, int n_big, const double* x, const double* u,
             const double* mu, const double* r_p, const double* rho_p, double* a);
double or_drag_cd(double re, double ma, double kexp);
void or_drag_gaps(const or_params* p, int n, int n_big, const double* x, const double* u,
                  const double* mu, const double* r_p, const double* rho_p,
                  const double* gaps /* [n_big][3] R, half width, factor, or NULL */,
                  const int* gap_on /* [n_big] */, double* a);
double or_gas_sigma(const or_params* p, double R);
double or_dg_series(double gamma);
double or_disk_gravity(const or_params* p, double R);
int or_drift(double mu0, const double x0[3], const double v0[3], double h, double x1[3],
             double v1[3]);
double or_pair_dmin2(const double r0[3], const double w0[3], const double r1[3],
                     const double w1[3], double h);
int or_flag(int n, int n_big, const double* rcrit, const double* x0, const double* u0,
            const double* x1, const double* u1, double h, int32_t* pairs, int cap,
            int* n_pairs);
int or_bs(int m, const double* mu_m, const double* rcrit_m, int np, const int32_t* pl,
          double mu0, double h, double tol, double* xs, double* vs);
void or_x2el(double gm, const double x[3], const double v[3], double el[6]);

#ifdef __cplusplus
}
#endif
#endif
