// Close encounters of the hybrid step (gfx950): flagging, planning and the
// Bulirsch-Stoer hand-off.
//
//   k_flag       : every unordered pair {big i, body j > i}; a conservative bound
//                  on the relative motion rejects far pairs with ~30 FP64 ops, the
//                  rest get the Hermite minimum-separation test; flagged pairs are
//                  appended with an integer atomic (the mce_snif critical region of
//                  Sect. 2.1.2 becomes a ticket counter)
//   k_sort_pairs : one block, bitonic sort of the list by (i, j): deterministic
//                  order whatever the append order was
//   k_plan       : one block; connected big-big components and one subsystem per
//                  flagged massless body with copies of the big components it
//                  touches
//   k_bs         : one wave per subsystem; the eight Stoermer sequences of a BS
//                  step run in eight lanes at once, the Aitken-Neville table is
//                  built across lanes, and the first accepted column is taken, the
//                  same column a sequential integrator would stop at.  Pair forces
//                  inside a subsystem are owner-computed in one lane (no atomics,
//                  the fo_hkce critical region of Sect. 2.1.2 disappears).
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "mx_internal.h"

namespace {

constexpr int kBlock = 256;

// ------------------------------------------------------------------ flag
__global__ __launch_bounds__(kBlock) void k_flag(
    int n, int nb, int split, double h, const double* __restrict__ x0s,
    const double* __restrict__ u0s, const double* __restrict__ x1s,
    const double* __restrict__ u1s, const FlagSource* __restrict__ fp,
    int32_t* __restrict__ pairs, int32_t cap, int32_t* __restrict__ counter,
    int32_t* __restrict__ err) {
  const int tile = blockIdx.x / split;
  const int sp = blockIdx.x - tile * split;
  const int j = tile * kBlock + threadIdx.x;
  const int jj = j < n ? j : n - 1;
  const double ax0 = x0s[jj], ay0 = x0s[n + jj], az0 = x0s[2 * n + jj];
  const double bx0 = u0s[jj], by0 = u0s[n + jj], bz0 = u0s[2 * n + jj];
  const double ax1 = x1s[jj], ay1 = x1s[n + jj], az1 = x1s[2 * n + jj];
  const double bx1 = u1s[jj], by1 = u1s[n + jj], bz1 = u1s[2 * n + jj];
  const double djx = ax1 - ax0, djy = ay1 - ay0, djz = az1 - az0;
  const double rcj = jj < nb ? fp[jj].rc : 0.0;
  const int per = (nb + split - 1) / split;
  const int s0 = sp * per;
  int s1 = min(nb, s0 + per);
  // no lane of this block pairs with a source index >= its own
  const int jmax = min(n - 1, tile * kBlock + kBlock - 1);
  s1 = min(s1, jmax);
  const double k427 = (4.0 / 27.0) * fabs(h);
  for (int i = s0; i < s1; ++i) {
    const FlagSource S = fp[i];
    double r0x = ax0 - S.x0, r0y = ay0 - S.y0, r0z = az0 - S.z0;
    double w0x = bx0 - S.u0x, w0y = by0 - S.u0y, w0z = bz0 - S.u0z;
    double w1x = bx1 - S.u1x, w1y = by1 - S.u1y, w1z = bz1 - S.u1z;
    double ddx = djx - S.dx, ddy = djy - S.dy, ddz = djz - S.dz;
    double m0 = fma(r0z, r0z, fma(r0y, r0y, r0x * r0x));
    double nd = fmax(fmax(fabs(ddx), fabs(ddy)), fabs(ddz));
    double nw = fmax(fmax(fabs(w0x), fabs(w0y)), fabs(w0z)) +
                fmax(fmax(fabs(w1x), fabs(w1y)), fabs(w1z));
    double rc = fmax(S.rc, rcj);
    // |r(tau) - r0| <= |Delta| + (4/27) h (|w0| + |w1|) for the cubic Hermite on [0,1]
    double bound = rc + 1.7320508075688773 * fma(k427, nw, nd) * (1.0 + 1e-12);
    bool cand = (i < j) && (j < n) && (m0 <= bound * bound * (1.0 + 1e-12));
    if (__builtin_expect(cand, 0)) {
      double r1x = ax1 - x1s[i], r1y = ay1 - x1s[n + i], r1z = az1 - x1s[2 * n + i];
      double q0x = ax0 - x0s[i], q0y = ay0 - x0s[n + i], q0z = az0 - x0s[2 * n + i];
      double dmin = mxd::hermite_dmin2(q0x, q0y, q0z, w0x, w0y, w0z, r1x, r1y, r1z, w1x, w1y,
                                       w1z, h);
      if (dmin <= rc * rc) {
        int idx = atomicAdd(counter, 1);
        if (idx < cap) {
          pairs[2 * idx] = i;
          pairs[2 * idx + 1] = j;
        } else {
          atomicOr(err, MXE_PAIRS);
        }
      }
    }
  }
}

// Bitonic sort of up to `cap` 64-bit keys with one block (global memory).
__device__ void block_bitonic(int64_t* key, int p2) {
  for (int k = 2; k <= p2; k <<= 1) {
    for (int jx = k >> 1; jx > 0; jx >>= 1) {
      for (int i = threadIdx.x; i < p2; i += blockDim.x) {
        int ixj = i ^ jx;
        if (ixj > i) {
          bool up = (i & k) == 0;
          int64_t a = key[i], b = key[ixj];
          if ((a > b) == up) {
            key[i] = b;
            key[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

__device__ int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

__global__ __launch_bounds__(1024) void k_sort_pairs(int32_t* __restrict__ pairs,
                                                     int64_t* __restrict__ keys, int32_t cap,
                                                     const int32_t* __restrict__ counter) {
  int np = min(*counter, cap);
  if (np <= 1) return;
  int p2 = next_pow2(np);
  for (int q = threadIdx.x; q < p2; q += blockDim.x)
    keys[q] = q < np ? (((int64_t)pairs[2 * q]) << 32) | (uint32_t)pairs[2 * q + 1] : INT64_MAX;
  __syncthreads();
  block_bitonic(keys, p2);
  for (int q = threadIdx.x; q < np; q += blockDim.x) {
    pairs[2 * q] = (int32_t)(keys[q] >> 32);
    pairs[2 * q + 1] = (int32_t)(keys[q] & 0xffffffff);
  }
}

// ------------------------------------------------------------------ plan
__device__ int uf_find(int32_t* par, int a) {
  while (par[a] != a) a = par[a];
  return a;
}

__device__ int index_in(const int32_t* v, int m, int b) {
  for (int k = 0; k < m; ++k)
    if (v[k] == b) return k;
  return -1;
}

__device__ void insert_sorted(int32_t* v, int& m, int b) {
  int k = m;
  while (k > 0 && v[k - 1] > b) {
    v[k] = v[k - 1];
    --k;
  }
  v[k] = b;
  ++m;
}

// uf: [2*nb]; par = uf[0..nb) (self at rest), flag = uf[nb..2nb) (0 at rest).
// keys: scratch of cap int64 (the small-pair list, sorted by (j, i)).
__global__ __launch_bounds__(1024) void k_plan(int nb, const int32_t* __restrict__ pairs,
                                               int32_t cap, int64_t* __restrict__ keys,
                                               int32_t* __restrict__ uf,
                                               Subsystem* __restrict__ subs, int32_t cap_subs,
                                               DevScalars* __restrict__ dsc) {
  const int np = min(dsc->n_pairs, cap);
  if (np == 0) return;
  // small-body pairs keyed by (j, i)
  __shared__ int nsmall;
  if (threadIdx.x == 0) {
    int c = 0;
    for (int q = 0; q < np; ++q)
      if (pairs[2 * q + 1] >= nb) keys[c++] = (((int64_t)pairs[2 * q + 1]) << 32) | (uint32_t)pairs[2 * q];
    nsmall = c;
  }
  __syncthreads();
  int ns = nsmall;
  if (ns > 1) {
    int p2 = next_pow2(ns);
    for (int q = ns + threadIdx.x; q < p2; q += blockDim.x) keys[q] = INT64_MAX;
    __syncthreads();
    block_bitonic(keys, p2);
  }
  if (threadIdx.x != 0) return;
  int32_t* par = uf;
  int32_t* inbig = uf + nb;
  // union of big-big pairs (root = smallest index)
  int nbb = 0;
  for (int q = 0; q < np; ++q) {
    int i = pairs[2 * q], j = pairs[2 * q + 1];
    if (j >= nb) continue;
    ++nbb;
    int ri = uf_find(par, i), rj = uf_find(par, j);
    if (ri != rj) {
      if (ri < rj) par[rj] = ri;
      else par[ri] = rj;
    }
    inbig[i] = 1;
    inbig[j] = 1;
  }
  int nsub = 0;
  // big components, ordered by their smallest member: walk the pair list's
  // bodies in ascending order (a body of a big-big pair is its own or a
  // later root's member)
  for (int q = 0; q < np && nbb > 0; ++q) {
    int i = pairs[2 * q], j = pairs[2 * q + 1];
    if (j >= nb) continue;
    int r = uf_find(par, i);
    if (inbig[r] != 1) continue;  // component already emitted (marked 2)
    Subsystem S;
    S.m = 0;
    S.keep_from = 0;
    S.np = 0;
    S.pad = 0;
    bool over = false;
    for (int q2 = 0; q2 < np; ++q2) {
      int a = pairs[2 * q2], b = pairs[2 * q2 + 1];
      if (b >= nb || uf_find(par, a) != r) continue;
      if (index_in(S.mem, S.m, a) < 0) {
        if (S.m >= kBsMaxMembers) { over = true; break; }
        insert_sorted(S.mem, S.m, a);
      }
      if (index_in(S.mem, S.m, b) < 0) {
        if (S.m >= kBsMaxMembers) { over = true; break; }
        insert_sorted(S.mem, S.m, b);
      }
    }
    for (int q2 = 0; q2 < np && !over; ++q2) {
      int a = pairs[2 * q2], b = pairs[2 * q2 + 1];
      if (b >= nb || uf_find(par, a) != r) continue;
      if (S.np >= kBsMaxPairs) { over = true; break; }
      S.pl[S.np][0] = index_in(S.mem, S.m, a);
      S.pl[S.np][1] = index_in(S.mem, S.m, b);
      ++S.np;
    }
    inbig[r] = 2;
    if (over || nsub >= cap_subs) {
      atomicOr(&dsc->err, MXE_SUBSYS);
      continue;
    }
    subs[nsub++] = S;
  }
  // one subsystem per flagged massless body, ascending
  for (int q = 0; q < ns; ++q) {
    int j = (int)(keys[q] >> 32);
    if (q > 0 && (int)(keys[q - 1] >> 32) == j) continue;
    Subsystem S;
    S.m = 0;
    S.np = 0;
    S.pad = 0;
    bool over = false;
    for (int q2 = q; q2 < ns && (int)(keys[q2] >> 32) == j && !over; ++q2) {
      int i = (int)(keys[q2] & 0xffffffff);
      if (inbig[i]) {
        int r = uf_find(par, i);
        for (int q3 = 0; q3 < np && !over; ++q3) {
          int a = pairs[2 * q3], b = pairs[2 * q3 + 1];
          if (b >= nb || uf_find(par, a) != r) continue;
          if (index_in(S.mem, S.m, a) < 0) {
            if (S.m >= kBsMaxMembers - 1) { over = true; break; }
            insert_sorted(S.mem, S.m, a);
          }
          if (index_in(S.mem, S.m, b) < 0) {
            if (S.m >= kBsMaxMembers - 1) { over = true; break; }
            insert_sorted(S.mem, S.m, b);
          }
        }
      } else if (index_in(S.mem, S.m, i) < 0) {
        if (S.m >= kBsMaxMembers - 1) { over = true; break; }
        insert_sorted(S.mem, S.m, i);
      }
    }
    int nbig_mem = S.m;
    if (!over) {
      S.mem[S.m++] = j;
      S.keep_from = nbig_mem;
      for (int q2 = 0; q2 < np && !over; ++q2) {
        int a = pairs[2 * q2], b = pairs[2 * q2 + 1];
        if (b < nb) {
          int la = index_in(S.mem, nbig_mem, a), lb = index_in(S.mem, nbig_mem, b);
          if (la >= 0 && lb >= 0) {
            if (S.np >= kBsMaxPairs) { over = true; break; }
            S.pl[S.np][0] = la;
            S.pl[S.np][1] = lb;
            ++S.np;
          }
        } else if (b == j) {
          if (S.np >= kBsMaxPairs) { over = true; break; }
          S.pl[S.np][0] = index_in(S.mem, nbig_mem, a);
          S.pl[S.np][1] = nbig_mem;
          ++S.np;
        }
      }
    }
    if (over || nsub >= cap_subs) {
      atomicOr(&dsc->err, MXE_SUBSYS);
      continue;
    }
    subs[nsub++] = S;
  }
  // restore the union-find scratch
  for (int q = 0; q < np; ++q) {
    int i = pairs[2 * q], j = pairs[2 * q + 1];
    par[i] = i;
    inbig[i] = 0;
    if (j < nb) {
      par[j] = j;
      inbig[j] = 0;
    }
  }
  dsc->n_sub = nsub;
}

// ------------------------------------------------------------------ BS
// Plain IEEE evaluation (no contraction) so that the integrator is the same
// sequence of operations as its definition.
#pragma clang fp contract(off)

constexpr int kM = kBsMaxMembers;
constexpr int kC = kBsColumns;

__device__ double bs_k(double s2, double rc) {
  double rc2 = rc * rc;
  if (s2 >= rc2) return 1.0;
  if (s2 <= 0.01 * rc2) return 0.0;
  double s = sqrt(s2);
  double q = (s - 0.1 * rc) / (0.9 * rc);
  double q2 = q * q, q3 = q * q2, q4 = q2 * q2, q5 = q2 * q3;
  return 10.0 * q3 - 15.0 * q4 + 6.0 * q5;
}

// star (mu0) plus the complementary (1-K) part of every flagged pair
__device__ void bs_force(int m, int np, const int32_t (*pl)[2], const double* mum,
                         const double* rcm, double mu0, const double* xs, double* as) {
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
    int a = pl[q][0], b = pl[q][1];
    double d0 = xs[3 * b] - xs[3 * a];
    double d1 = xs[3 * b + 1] - xs[3 * a + 1];
    double d2 = xs[3 * b + 2] - xs[3 * a + 2];
    double s2 = d0 * d0 + d1 * d1 + d2 * d2;
    double rc = rcm[a] > rcm[b] ? rcm[a] : rcm[b];
    double w = s2 > 0.0 ? (1.0 / (s2 * sqrt(s2))) * (1.0 - bs_k(s2, rc)) : 0.0;
    as[3 * a] += mum[b] * w * d0;
    as[3 * a + 1] += mum[b] * w * d1;
    as[3 * a + 2] += mum[b] * w * d2;
    as[3 * b] -= mum[a] * w * d0;
    as[3 * b + 1] -= mum[a] * w * d1;
    as[3 * b + 2] -= mum[a] * w * d2;
  }
}

__global__ __launch_bounds__(64) void k_bs(int n, int nb, double mu0, double h, double tol,
                                           const double* __restrict__ x0s,
                                           const double* __restrict__ u0s,
                                           double* __restrict__ x, double* __restrict__ u,
                                           const double* __restrict__ mu,
                                           const double* __restrict__ rcrit,
                                           const Subsystem* __restrict__ subs,
                                           DevScalars* __restrict__ dsc) {
  __shared__ Subsystem S;
  __shared__ double xs[3 * kM], vs[3 * kM], mum[kM], rcm[kM], scal[2 * kM];
  __shared__ double res[kC][6 * kM];
  __shared__ double wk[kC][3][3 * kM];
  __shared__ double errk[kC];
  const int lane = threadIdx.x;
  const int nsub = dsc->n_sub;
  for (int b = blockIdx.x; b < nsub; b += gridDim.x) {
    __syncthreads();
    if (lane == 0) S = subs[b];
    __syncthreads();
    const int m = S.m, np = S.np;
    const int nn = 3 * m;
    for (int e = lane; e < nn; e += 64) {
      int k = e / 3, c = e - 3 * (e / 3);
      int body = S.mem[k];
      xs[e] = x0s[(size_t)c * n + body];
      vs[e] = u0s[(size_t)c * n + body];
    }
    for (int k = lane; k < m; k += 64) {
      int body = S.mem[k];
      mum[k] = body < nb ? mu[body] : 0.0;
      rcm[k] = body < nb ? rcrit[body] : 0.0;
    }
    __syncthreads();
    double done = 0.0, H = h;
    int fails = 0;
    bool failed = false;
    while (fabs(h - done) > 1e-14 * fabs(h)) {
      double rem = h - done;
      if (fabs(H) > fabs(rem)) H = rem;
      for (int k = lane; k < m; k += 64) {
        const double* p = xs + 3 * k;
        const double* q = vs + 3 * k;
        scal[k] = 1.0 / (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        scal[m + k] = 1.0 / (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
      }
      // the Stoermer (velocity-Verlet) sequences n = 2, 4, ..., 16 in lanes 0..7
      if (lane < kC) {
        const int ns = 2 * (lane + 1);
        const double dt = H / ns;
        double* pos = wk[lane][0];
        double* d = wk[lane][1];
        double* acc = wk[lane][2];
        for (int i = 0; i < nn; ++i) pos[i] = xs[i];
        bs_force(m, np, S.pl, mum, rcm, mu0, pos, acc);
        for (int i = 0; i < nn; ++i) {
          d[i] = dt * (vs[i] + 0.5 * dt * acc[i]);
          pos[i] += d[i];
        }
        for (int k = 1; k < ns; ++k) {
          bs_force(m, np, S.pl, mum, rcm, mu0, pos, acc);
          for (int i = 0; i < nn; ++i) {
            d[i] += dt * dt * acc[i];
            pos[i] += d[i];
          }
        }
        bs_force(m, np, S.pl, mum, rcm, mu0, pos, acc);
        for (int i = 0; i < nn; ++i) {
          res[lane][i] = pos[i];
          res[lane][nn + i] = d[i] / dt + 0.5 * dt * acc[i];
        }
      }
      if (lane < kC) errk[lane] = 0.0;
      __syncthreads();
      // Aitken-Neville extrapolation in (H/n)^2, one table per element, and the
      // per-column error max(dx^2 xscal, dv^2 vscal)
      double diag[2][kC];
      double lerr[kC];
      for (int k = 0; k < kC; ++k) lerr[k] = 0.0;
      for (int slot = 0; slot < 2; ++slot) {
        int e = lane + 64 * slot;
        for (int k = 0; k < kC; ++k) diag[slot][k] = 0.0;
        if (e >= 2 * nn) continue;
        double sc = e < nn ? scal[e / 3] : scal[m + (e - nn) / 3];
        double T[kC], P[kC];
        for (int k = 0; k < kC; ++k) {
          T[0] = res[k][e];
          for (int jx = 1; jx <= k; ++jx) {
            double ratio = (double)(2 * (k + 1)) / (double)(2 * (k - jx + 1));
            double den = ratio * ratio - 1.0;
            T[jx] = T[jx - 1] + (T[jx - 1] - P[jx - 1]) / den;
          }
          diag[slot][k] = T[k];
          if (k >= 1) {
            double ex = T[k] - T[k - 1];
            double v = ex * ex * sc;
            if (v > lerr[k]) lerr[k] = v;
          }
          for (int jx = 0; jx <= k; ++jx) P[jx] = T[jx];
        }
      }
      // wave-wide maximum of each column's error
      for (int k = 1; k < kC; ++k) {
        double v = lerr[k];
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
        lerr[k] = v;
      }
      int accepted = -1;
      for (int k = 1; k < kC; ++k)
        if (accepted < 0 && lerr[k] <= tol * tol) accepted = k;
      __syncthreads();
      if (accepted >= 0) {
        for (int slot = 0; slot < 2; ++slot) {
          int e = lane + 64 * slot;
          if (e >= 2 * nn) continue;
          double val = diag[slot][0];
#pragma unroll
          for (int k = 1; k < kC; ++k)
            if (k == accepted) val = diag[slot][k];
          if (e < nn) xs[e] = val;
          else vs[e - nn] = val;
        }
        done += H;
        fails = 0;
        if (accepted <= 4) H = 2.0 * H;
      } else {
        H = 0.5 * H;
        if (++fails > 30) {
          failed = true;
          break;
        }
      }
      __syncthreads();
    }
    if (failed) {
      if (lane == 0) atomicOr(&dsc->err, MXE_BS);
      continue;
    }
    for (int e = lane; e < nn; e += 64) {
      int k = e / 3, c = e - 3 * (e / 3);
      if (k < S.keep_from) continue;
      int body = S.mem[k];
      x[(size_t)c * n + body] = xs[e];
      u[(size_t)c * n + body] = vs[e];
    }
  }
}
#pragma clang fp contract(on)

}  // namespace

namespace mxk {

int force_split(int n, int nb);

hipError_t launch_flag(mx_system* s) {
  int tiles = (s->n + kBlock - 1) / kBlock;
  int split = force_split(s->n, s->nb);
  if (s->nb > 0)
    hipLaunchKernelGGL(k_flag, dim3(tiles * split), dim3(kBlock), 0, s->stream, s->n, s->nb, split,
                       s->p.dt, s->x0, s->u0, s->x, s->u, s->fpack, s->pairs, s->cap_pairs,
                       &s->dsc->n_pairs, &s->dsc->err);
  return hipGetLastError();
}

hipError_t launch_bs(mx_system* s) {
  if (s->nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_pairs, dim3(1), dim3(1024), 0, s->stream, s->pairs,
                     (int64_t*)s->pairs_tmp, s->cap_pairs, &s->dsc->n_pairs);
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, s->stream, s->nb, s->pairs, s->cap_pairs,
                     (int64_t*)s->pairs_tmp, s->uf, s->subs, s->cap_subs, s->dsc);
  hipLaunchKernelGGL(k_bs, dim3(512), dim3(64), 0, s->stream, s->n, s->nb, s->mu0, s->p.dt,
                     s->p.bs_tol, s->x0, s->u0, s->x, s->u, s->mu, s->rcrit, s->subs, s->dsc);
  return hipGetLastError();
}

// flag + sort for the stateless entry; fpack built from the given states
__global__ void k_fpack_plain(int n, int nb, const double* __restrict__ rcrit,
                              const double* __restrict__ x0, const double* __restrict__ u0,
                              const double* __restrict__ x1, const double* __restrict__ u1,
                              FlagSource* __restrict__ fp) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb) return;
  FlagSource f;
  f.x0 = x0[t]; f.y0 = x0[n + t]; f.z0 = x0[2 * n + t];
  f.u0x = u0[t]; f.u0y = u0[n + t]; f.u0z = u0[2 * n + t];
  f.dx = x1[t] - x0[t]; f.dy = x1[n + t] - x0[n + t]; f.dz = x1[2 * n + t] - x0[2 * n + t];
  f.u1x = u1[t]; f.u1y = u1[n + t]; f.u1z = u1[2 * n + t];
  f.rc = rcrit[t];
  f.pad0 = f.pad1 = f.pad2 = 0.0;
  fp[t] = f;
}

hipError_t flag_pairs(int n, int nb, const double* rcrit, const double* x0, const double* u0,
                      const double* x1, const double* u1, double h, int32_t* pairs,
                      int32_t* pairs_tmp, int32_t cap, int32_t* counter, hipStream_t st) {
  if (nb == 0) return hipSuccess;
  FlagSource* fp = nullptr;
  hipError_t e = hipMalloc((void**)&fp, sizeof(FlagSource) * nb);
  if (e != hipSuccess) return e;
  int32_t* err = counter + 1;
  hipLaunchKernelGGL(k_fpack_plain, dim3((nb + 255) / 256), dim3(256), 0, st, n, nb, rcrit, x0, u0,
                     x1, u1, fp);
  int tiles = (n + kBlock - 1) / kBlock;
  int split = force_split(n, nb);
  hipLaunchKernelGGL(k_flag, dim3(tiles * split), dim3(kBlock), 0, st, n, nb, split, h, x0, u0, x1,
                     u1, fp, pairs, cap, counter, err);
  hipLaunchKernelGGL(k_sort_pairs, dim3(1), dim3(1024), 0, st, pairs, (int64_t*)pairs_tmp, cap,
                     counter);
  e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFree(fp);
  return e != hipSuccess ? e : e2;
}

}  // namespace mxk
