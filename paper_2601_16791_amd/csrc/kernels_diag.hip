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
  for (int r = 0; r < 3; ++r) {
    dsc->n_pairs[r] = 0;
    dsc->plan_ready[r] = 0;
    dsc->bs_done[r] = 0;
    dsc->n_jsub[r] = 0;
  }
  dsc->n_sub = 0;
  dsc->P[0] = dsc->P[1] = dsc->P[2] = 0.0;
}

// ------------------------------------------------------------ body removal
// Massive-body momentum P = sum mu u in index order (one thread), for the
// heliocentric velocities of the removal test.
__global__ void k_removal_momentum(int n, int nb, const double* __restrict__ mu,
                                   const double* __restrict__ u, double* __restrict__ P) {
  double p0 = 0.0, p1 = 0.0, p2 = 0.0;
  for (int k = 0; k < nb; ++k) {
    p0 += mu[k] * u[k];
    p1 += mu[k] * u[n + k];
    p2 += mu[k] * u[2 * n + k];
  }
  P[0] = p0;
  P[1] = p1;
  P[2] = p2;
}

// Ejection (e >= 1, Sect. 3.5) and central-body encounter test of every body not
// yet flagged; a flagged massive body loses its mass, changeover radius, growth,
// migration and gap.
__global__ __launch_bounds__(kBlock) void k_check_removal(
    int n, int nb, double mu0, double r_cen, const double* __restrict__ x,
    const double* __restrict__ u, const double* __restrict__ P, double* __restrict__ mu,
    double* __restrict__ rcrit, double* __restrict__ growth, PlanetPhys* __restrict__ phys,
    int32_t* __restrict__ stat, int8_t* __restrict__ rsign, int32_t* __restrict__ ejcount) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n || stat[t] < 0) return;
  const double px = x[t], py = x[n + t], pz = x[2 * n + t];
  const double vx = u[t] + P[0] / mu0, vy = u[n + t] + P[1] / mu0, vz = u[2 * n + t] + P[2] / mu0;
  const double gm = mu0 + (t < nb ? mu[t] : 0.0);
  const double r = sqrt(px * px + py * py + pz * pz);
  // specific angular momentum and the Laplace-Runge-Lenz vector / gm
  const double hx = py * vz - pz * vy, hy = pz * vx - px * vz, hz = px * vy - py * vx;
  const double ex = (vy * hz - vz * hy) / gm - px / r;
  const double ey = (vz * hx - vx * hz) / gm - py / r;
  const double ez = (vx * hy - vy * hx) / gm - pz / r;
  const double e = sqrt(ex * ex + ey * ey + ez * ez);
  const double q = (hx * hx + hy * hy + hz * hz) / (gm * (1.0 + e));
  const double rdot = px * vx + py * vy + pz * vz;
  int st = 0;
  if (e >= 1.0) st = -3;
  else if (r_cen > 0.0 && (r <= r_cen || (rsign[t] < 0 && rdot >= 0.0 && q <= r_cen))) st = -2;
  rsign[t] = rdot < 0.0 ? -1 : 1;
  if (st < 0) {
    stat[t] = st;
    atomicAdd(ejcount, 1);
    if (t < nb) {
      mu[t] = 0.0;
      rcrit[t] = 0.0;
      if (growth) growth[3 * t + 2] = 0.0;
      if (phys) phys[t] = PlanetPhys{};
    }
  }
}

// Stable compaction of the flagged massless bodies: survivors per block, an
// exclusive scan of the block counts (one thread, in order), then each block's
// scan in LDS gives every survivor its new index.
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(kScanBlock) void k_keep_count(int n, int nb,
                                                           const int32_t* __restrict__ stat,
                                                           int32_t* __restrict__ counts) {
  __shared__ int32_t sh[kScanBlock / 64];
  const int t = blockIdx.x * kScanBlock + threadIdx.x;
  const bool keep = t < n && (t < nb || stat[t] >= 0);
  const uint64_t b = __builtin_amdgcn_ballot_w64(keep);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = __popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t c = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) c += sh[w];
    counts[blockIdx.x] = c;
  }
}

__global__ void k_keep_offsets(int nblk, int32_t* __restrict__ counts, int32_t* __restrict__ total) {
  int32_t run = 0;
  for (int b = 0; b < nblk; ++b) {
    const int32_t c = counts[b];
    counts[b] = run;
    run += c;
  }
  *total = run;
}

__global__ __launch_bounds__(kScanBlock) void k_keep_map(int n, int nb,
                                                         const int32_t* __restrict__ stat,
                                                         const int32_t* __restrict__ offsets,
                                                         int32_t* __restrict__ map) {
  __shared__ int32_t sh[kScanBlock / 64];
  const int t = blockIdx.x * kScanBlock + threadIdx.x;
  const bool keep = t < n && (t < nb || stat[t] >= 0);
  const uint64_t b = __builtin_amdgcn_ballot_w64(keep);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = __popcll(b);
  __syncthreads();
  int32_t base = offsets[blockIdx.x];
  for (int k = 0; k < w; ++k) base += sh[k];
  const int32_t below = __popcll(b & ((1ull << lane) - 1ull));
  if (t < n) map[t] = keep ? base + below : -1;
}

// dst[c * m + map[t]] = src[c * n + t] for the survivors, c < rows
__global__ __launch_bounds__(kBlock) void k_gather_rows(int n, int m, int rows, int first,
                                                        const int32_t* __restrict__ map,
                                                        const double* __restrict__ src,
                                                        double* __restrict__ dst) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t < first || t >= n) return;
  const int j = map[t];
  if (j < 0) return;
  for (int c = 0; c < rows; ++c) dst[(size_t)c * m + (j - first)] = src[(size_t)c * n + (t - first)];
}

__global__ __launch_bounds__(kBlock) void k_gather_status(int n, const int32_t* __restrict__ map,
                                                          const int32_t* __restrict__ st,
                                                          const int8_t* __restrict__ rs,
                                                          int32_t* __restrict__ st2,
                                                          int8_t* __restrict__ rs2) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const int j = map[t];
  if (j < 0) return;
  st2[j] = st[t];
  rs2[j] = rs[t];
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

hipError_t launch_check_removal(mx_system* s, double r_cen) {
  hipLaunchKernelGGL(k_removal_momentum, dim3(1), dim3(1), 0, s->stream, s->n, s->nb, s->mu, s->u,
                     s->rm_P);
  hipLaunchKernelGGL(k_check_removal, dim3(blocks_for(s->n)), dim3(kBlock), 0, s->stream, s->n,
                     s->nb, s->mu0, r_cen, s->x, s->u, s->rm_P, s->mu, s->rcrit,
                     s->has_growth ? s->growth : nullptr, s->has_phys ? s->phys : nullptr, s->stat,
                     s->rsign, s->ejcount);
  return hipGetLastError();
}

// Compacts x, u, ag, r_p, rho_p, status and radial directions of the system into
// the survivors (new stride *n_new); map_dev: device [n] receives the index map.
// Temporary buffers are allocated and freed here (not a step of the integrator).
hipError_t compact_bodies(mx_system* s, int32_t* n_new, int32_t* map_dev) {
  const int n = s->n, nb = s->nb;
  const int nblk = (n + kScanBlock - 1) / kScanBlock;
  int32_t* counts = nullptr;
  hipError_t e = hipMalloc((void**)&counts, sizeof(int32_t) * (nblk + 1));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_keep_count, dim3(nblk), dim3(kScanBlock), 0, s->stream, n, nb, s->stat,
                     counts);
  hipLaunchKernelGGL(k_keep_offsets, dim3(1), dim3(1), 0, s->stream, nblk, counts, counts + nblk);
  hipLaunchKernelGGL(k_keep_map, dim3(nblk), dim3(kScanBlock), 0, s->stream, n, nb, s->stat,
                     counts, map_dev);
  int32_t m = n;
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(&m, counts + nblk, sizeof(int32_t), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(counts);
  if (e != hipSuccess) return e;
  *n_new = m;
  if (m == n) return hipSuccess;
  double* tmp = nullptr;
  const size_t rows = 9 * (size_t)m + 2 * (size_t)(m - nb);
  e = hipMalloc((void**)&tmp, sizeof(double) * (rows > 0 ? rows : 1));
  int32_t* st2 = nullptr;
  int8_t* rs2 = nullptr;
  if (e == hipSuccess) e = hipMalloc((void**)&st2, sizeof(int32_t) * m);
  if (e == hipSuccess) e = hipMalloc((void**)&rs2, (size_t)m);
  if (e == hipSuccess) {
    const dim3 g(blocks_for(n)), b(kBlock);
    hipLaunchKernelGGL(k_gather_rows, g, b, 0, s->stream, n, m, 3, 0, map_dev, s->x, tmp);
    hipLaunchKernelGGL(k_gather_rows, g, b, 0, s->stream, n, m, 3, 0, map_dev, s->u, tmp + 3 * (size_t)m);
    hipLaunchKernelGGL(k_gather_rows, g, b, 0, s->stream, n, m, 3, 0, map_dev, s->ag, tmp + 6 * (size_t)m);
    if (n > nb) {
      // the massless bodies' properties are indexed from nb: shift map and arrays
      hipLaunchKernelGGL(k_gather_rows, dim3(blocks_for(n)), b, 0, s->stream, n, m - nb, 1, nb,
                         map_dev, s->r_p, tmp + 9 * (size_t)m);
      hipLaunchKernelGGL(k_gather_rows, dim3(blocks_for(n)), b, 0, s->stream, n, m - nb, 1, nb,
                         map_dev, s->rho_p, tmp + 9 * (size_t)m + (m - nb));
    }
    hipLaunchKernelGGL(k_gather_status, g, b, 0, s->stream, n, map_dev, s->stat, s->rsign, st2, rs2);
    e = hipGetLastError();
  }
  const size_t v3 = sizeof(double) * 3 * (size_t)m;
  if (e == hipSuccess) e = hipMemcpyAsync(s->x, tmp, v3, hipMemcpyDeviceToDevice, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s->u, tmp + 3 * (size_t)m, v3, hipMemcpyDeviceToDevice, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s->ag, tmp + 6 * (size_t)m, v3, hipMemcpyDeviceToDevice, s->stream);
  if (e == hipSuccess && m > nb) {
    e = hipMemcpyAsync(s->r_p, tmp + 9 * (size_t)m, sizeof(double) * (m - nb), hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->rho_p, tmp + 9 * (size_t)m + (m - nb), sizeof(double) * (m - nb),
                         hipMemcpyDeviceToDevice, s->stream);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(s->stat, st2, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s->rsign, rs2, (size_t)m, hipMemcpyDeviceToDevice, s->stream);
  hipError_t e2 = hipStreamSynchronize(s->stream);
  if (tmp) (void)hipFree(tmp);
  if (st2) (void)hipFree(st2);
  if (rs2) (void)hipFree(rs2);
  return e != hipSuccess ? e : e2;
}

hipError_t launch_reset_scalars(mx_system* s, int64_t step) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, s->stream, s->dsc, step);
  return hipGetLastError();
}

}  // namespace mxk
