// Set-up, frame changes and diagnostics of a system (gfx950).
//
//   k_init_big   : mu = G m, changeover radius rcrit_hill * a (m / 3 m0)^(1/3)
//                  from the osculating semi-major axis (|x| when unbound),
//                  growth parameters to mu units
//   k_init_small : particle densities to Msun / AU^3
//   k_h2dh       : heliocentric -> democratic heliocentric velocities
//                  (u = v - sum m v / (m0 + sum m)), the mco_h2dh transform
//   k_dh2h       : back again (v = u + P / m0), the mco_dh2h transform
//   k_energy_*   : energy with the potential over massive bodies only (the mxx_en
//                  change of Sect. 2.1.3) and angular momentum, with fixed-order
//                  two-level reductions
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "mx_internal.h"

namespace {

constexpr int kBlock = 256;

__global__ void k_init_big(int n, int nb, double G, double mu0, double hill,
                           const double* __restrict__ xh, const double* __restrict__ vh,
                           const double* __restrict__ m, const double* __restrict__ growth_in,
                           int has_growth, double* __restrict__ mu, double* __restrict__ mu_init,
                           double* __restrict__ rcrit, double* __restrict__ rcrit_init,
                           double* __restrict__ growth, int32_t* __restrict__ uf) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  double muk = G * m[k];
  double x = xh[k], y = xh[n + k], z = xh[2 * n + k];
  double vx = vh[k], vy = vh[n + k], vz = vh[2 * n + k];
  double r = sqrt(x * x + y * y + z * z);
  double v2 = vx * vx + vy * vy + vz * vz;
  double gm = mu0 + muk;
  double a = 1.0 / (2.0 / r - v2 / gm);
  if (!(a > 0.0) || !isfinite(a)) a = r;
  double rc = hill * a * cbrt(muk / (3.0 * mu0));
  mu[k] = muk;
  mu_init[k] = muk;
  rcrit[k] = rc;
  rcrit_init[k] = rc;
  if (has_growth) {
    growth[3 * k] = G * growth_in[3 * k];
    growth[3 * k + 1] = G * growth_in[3 * k + 1];
    growth[3 * k + 2] = growth_in[3 * k + 2];
  }
  uf[k] = k;
  uf[nb + k] = 0;
}

__global__ void k_init_small(int ns, double rho_unit, double* __restrict__ rho_p) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < ns) rho_p[j] *= rho_unit;
}

__global__ __launch_bounds__(kBlock) void k_h2dh(int n, int nb, double mu0,
                                                 const double* __restrict__ mu,
                                                 const double* __restrict__ vh,
                                                 double* __restrict__ u) {
  __shared__ double sh[4 * kBlock];
  double v[4] = {0, 0, 0, 0};
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    v[0] += mu[k] * vh[k];
    v[1] += mu[k] * vh[n + k];
    v[2] += mu[k] * vh[2 * n + k];
    v[3] += mu[k];
  }
  mxd::block_sum<kBlock, 4>(v, sh);
  double mt = mu0 + v[3];
  int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  u[t] = vh[t] - v[0] / mt;
  u[n + t] = vh[n + t] - v[1] / mt;
  u[2 * n + t] = vh[2 * n + t] - v[2] / mt;
}

__global__ __launch_bounds__(kBlock) void k_dh2h(int n, int nb, double mu0,
                                                 const double* __restrict__ mu,
                                                 const double* __restrict__ u,
                                                 double* __restrict__ vh) {
  __shared__ double sh[3 * kBlock];
  double v[3] = {0, 0, 0};
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    v[0] += mu[k] * u[k];
    v[1] += mu[k] * u[n + k];
    v[2] += mu[k] * u[2 * n + k];
  }
  mxd::block_sum<kBlock, 3>(v, sh);
  int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  vh[t] = u[t] + v[0] / mu0;
  vh[n + t] = u[n + t] + v[1] / mu0;
  vh[2 * n + t] = u[2 * n + t] + v[2] / mu0;
}

// pair potential: block b takes rows i = b, b + G, ...; partial sum per block
__global__ __launch_bounds__(kBlock) void k_energy_pairs(int n, int nb,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ mu,
                                                         double* __restrict__ red) {
  __shared__ double sh[kBlock];
  double pe[1] = {0.0};
  for (int i = blockIdx.x; i < nb; i += gridDim.x) {
    double xi = x[i], yi = x[n + i], zi = x[2 * n + i], mi = mu[i];
    for (int j = i + 1 + threadIdx.x; j < nb; j += kBlock) {
      double dx = x[j] - xi, dy = x[n + j] - yi, dz = x[2 * n + j] - zi;
      pe[0] -= mi * mu[j] / sqrt(dx * dx + dy * dy + dz * dz);
    }
  }
  mxd::block_sum<kBlock, 1>(pe, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = pe[0];
}

__global__ __launch_bounds__(kBlock) void k_energy_final(int n, int nb, int nred, double mu0,
                                                         double G, const double* __restrict__ x,
                                                         const double* __restrict__ u,
                                                         const double* __restrict__ mu,
                                                         const double* __restrict__ red,
                                                         double* __restrict__ out) {
  __shared__ double sh[8 * kBlock];
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nred; b += kBlock) v[0] += red[b];
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    double m = mu[k];
    double xk = x[k], yk = x[n + k], zk = x[2 * n + k];
    double ux = u[k], uy = u[n + k], uz = u[2 * n + k];
    v[1] += 0.5 * m * (ux * ux + uy * uy + uz * uz) - mu0 * m / sqrt(xk * xk + yk * yk + zk * zk);
    v[2] += m * (yk * uz - zk * uy);
    v[3] += m * (zk * ux - xk * uz);
    v[4] += m * (xk * uy - yk * ux);
    v[5] += m * ux;
    v[6] += m * uy;
    v[7] += m * uz;
  }
  mxd::block_sum<kBlock, 8>(v, sh);
  if (threadIdx.x == 0) {
    double ke_p = (v[5] * v[5] + v[6] * v[6] + v[7] * v[7]) / (2.0 * mu0);
    out[0] = (v[0] + v[1] + ke_p) / G;
    out[1] = v[2] / G;
    out[2] = v[3] / G;
    out[3] = v[4] / G;
  }
}

__global__ void k_reset(DevScalars* dsc, int64_t step) {
  dsc->step = step;
  dsc->n_pairs = 0;
  dsc->n_pairs_alt = 0;
  dsc->n_sub = 0;
  dsc->plan_ready = 0;
  dsc->P[0] = dsc->P[1] = dsc->P[2] = 0.0;
}

int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }

}  // namespace

namespace mxk {

hipError_t launch_init_bodies(mx_system* s, const double* x_h_dev, const double* v_h_dev) {
  // expects: s->x holds x_h; v_h_dev holds heliocentric velocities; s->mu holds the
  // raw masses (Msun) until converted here; s->growth holds raw growth if any
  if (s->nb > 0)
    hipLaunchKernelGGL(k_init_big, dim3((s->nb + 255) / 256), dim3(256), 0, s->stream, s->n,
                       s->nb, s->p.G, s->mu0, s->p.rcrit_hill, x_h_dev, v_h_dev, s->mu_init,
                       s->growth, s->has_growth, s->mu, s->mu_init, s->rcrit, s->rcrit_init,
                       s->growth, s->uf);
  if (s->ns > 0)
    hipLaunchKernelGGL(k_init_small, dim3((s->ns + 255) / 256), dim3(256), 0, s->stream, s->ns,
                       s->p.rho_unit, s->rho_p);
  return hipGetLastError();
}

hipError_t launch_h2dh(mx_system* s, const double* v_h) {
  hipLaunchKernelGGL(k_h2dh, dim3(blocks_for(s->n)), dim3(kBlock), 0, s->stream, s->n, s->nb,
                     s->mu0, s->mu, v_h, s->u);
  return hipGetLastError();
}

hipError_t launch_dh2h(mx_system* s, double* v_h) {
  hipLaunchKernelGGL(k_dh2h, dim3(blocks_for(s->n)), dim3(kBlock), 0, s->stream, s->n, s->nb,
                     s->mu0, s->mu, s->u, v_h);
  return hipGetLastError();
}

hipError_t launch_energy(mx_system* s, double* out) {
  if (s->nb > 1)
    hipLaunchKernelGGL(k_energy_pairs, dim3(s->red_blocks), dim3(kBlock), 0, s->stream, s->n,
                       s->nb, s->x, s->mu, s->red);
  int nred = s->nb > 1 ? s->red_blocks : 0;
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, s->stream, s->n, s->nb, nred,
                     s->mu0, s->p.G, s->x, s->u, s->mu, s->red, out);
  return hipGetLastError();
}

hipError_t launch_reset_scalars(mx_system* s, int64_t step) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, s->stream, s->dsc, step);
  return hipGetLastError();
}

}  // namespace mxk
