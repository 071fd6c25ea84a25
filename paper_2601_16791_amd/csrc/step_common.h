// Per-body and massive-body pieces of the fused step (systems of at most 64
// massive bodies), shared by the step kernels and by the encounter integrator,
// which precomputes the massive bodies of a joined step boundary: one
// definition, so every caller performs the same operations.
#pragma once
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "force_sum.h"
#include "mx_internal.h"

namespace mxs {

using mxd::DragConst;

// half kick (with drag for massless bodies, in the frame shifted by Ppre/mu0),
// jump by Ppost/mu0, Kepler drift.  On entry (p, v, a) is the step-start state;
// on exit (p, v) is the pre-drift state and (q, w) the post-drift state.  site:
// the gas at p when already evaluated, else null.
__device__ __forceinline__ bool advance_body(int t, int nb, double mu0, double h,
                                             const DragConst& dc, int gas_on, double rp,
                                             double rhop, const double* vpre,
                                             const double* jpost, double (&p)[3], double (&v)[3],
                                             const double (&a)[3], double (&q)[3],
                                             double (&w)[3],
                                             const mxd::GasSite* site = nullptr) {
  // vpre = Ppre / mu0 (frame velocity of the drag), jpost = (h/2) Ppost / mu0 (jump);
  // rp, rhop: radius and density of a massless body (unused for massive ones)
  const double hh = 0.5 * h;
  double ad[3] = {0.0, 0.0, 0.0};
  if (t >= nb && gas_on) {
    if (site)
      mxd::gas_drag_at(dc, *site, v[0] + vpre[0], v[1] + vpre[1], v[2] + vpre[2], rp, rhop,
                       ad[0], ad[1], ad[2]);
    else
      mxd::gas_drag(dc, p[0], p[1], v[0] + vpre[0], v[1] + vpre[1], v[2] + vpre[2], rp, rhop,
                    ad[0], ad[1], ad[2]);
  }
  for (int c = 0; c < 3; ++c) {
    v[c] += hh * (a[c] + ad[c]);
    p[c] += jpost[c];
    q[c] = p[c];
    w[c] = v[c];
  }
  return mxd::kepler_drift(mu0, h, q[0], q[1], q[2], w[0], w[1], w[2]);
}

// Momentum terms of the massive bodies for the opening half of a step: lane
// k < nb of the first wave holds massive body k (velocity v, acceleration a,
// mass m); the sums of m v and m (v + h/2 a) go to sh[0..5] by the fixed lane
// reduction (the same bits in every block).  Called by the whole first wave.
__device__ __forceinline__ void big_sums_a(const SysDesc& D, int lane, double* sh,
                                           const double (&v)[3], const double (&a)[3],
                                           double m) {
  const int nb = D.nb;
  const double hh = 0.5 * D.h;
  double t[6];
  for (int c = 0; c < 3; ++c) {
    t[c] = lane < nb ? m * v[c] : 0.0;
    t[3 + c] = lane < nb ? m * (v[c] + hh * a[c]) : 0.0;
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) t[c] = mxd::wave_sum_fixed(t[c]);
  if (lane == 0)
    for (int c = 0; c < 6; ++c) sh[c] = t[c];
}

// Ppre = P_pre / mu0 and Ppost = (h/2) P_post / mu0 from the sums in sh.
__device__ __forceinline__ void big_frame_a(const SysDesc& D, const double* sh,
                                            double (&Ppre)[3], double (&Ppost)[3]) {
  const double hh = 0.5 * D.h;
  for (int c = 0; c < 3; ++c) {
    Ppre[c] = sh[c] / D.mu0;
    Ppost[c] = hh * sh[3 + c] / D.mu0;
  }
}

// Half kick, jump and drift of massive body k (identical arithmetic in every
// block), kept in LDS: bst rows x0 (3) u0 (3) x1 (3) u1 (3), brc its changeover
// radius rc.  `first` latches a failure once per system.
__device__ __forceinline__ void big_advance_a(const SysDesc& D, bool first, int k,
                                              double (*bst)[kSmallBig], double* brc,
                                              double (&p)[3], double (&v)[3],
                                              const double (&a)[3], double rc,
                                              const double (&Ppre)[3], const double (&Ppost)[3]) {
  const int nb = D.nb;
  double q[3], w[3];
  bool ok = advance_body(k, nb, D.mu0, D.h, D.dc, D.gas_on, 0.0, 0.0, Ppre, Ppost, p, v, a, q, w);
  if (!ok && first) atomicOr(&D.dsc->err, MXE_NOCONV);
  for (int c = 0; c < 3; ++c) {
    bst[c][k] = p[c];
    bst[3 + c][k] = v[c];
    bst[6 + c][k] = q[c];
    bst[9 + c][k] = w[c];
  }
  brc[k] = rc;
}

// Closing part of a step for one body, from its state after the encounter
// integrator: jump by J, changeover-weighted gravity of the massive bodies in
// src (rct: the body's own changeover radius, 0 when massless) and, with kick,
// the gas drag (massless bodies, frame velocity vpre) and the half kick.
// pos: in before the jump, out after it; acc: out, the gravity.
__device__ __forceinline__ void close_body(int t, int nb, const KickSource* src, double rct,
                                           const double (&J)[3], const double (&vpre)[3],
                                           double hh, const DragConst& dc, int gas_on, double rp,
                                           double rhop, bool kick, double (&pos)[3],
                                           double (&vel)[3], double (&acc)[3]) {
  const double px = pos[0] + J[0], py = pos[1] + J[1], pz = pos[2] + J[2];
  const double rc2t = rct * rct;
  double k15, k1875;
  mxd::vgpr_constants(k15, k1875);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
  for (int s = 0; s < nb; ++s) {
    const KickSource S = src[s];
    double dx = S.x - px, dy = S.y - py, dz = S.z - pz;
    double s2 = fma(dz, dz, fma(dy, dy, dx * dx));
    double rc2 = fmax(S.rc2, rc2t);
    double wgt = mxd::fast_weight(S.mu, s2, k15, k1875);
    if (s2 < rc2) wgt = S.mu * mxd::changeover_weight_slow(s2, fmax(S.rc, rct), rc2);
    a0 = fma(wgt, dx, a0);
    a1 = fma(wgt, dy, a1);
    a2 = fma(wgt, dz, a2);
  }
  pos[0] = px;
  pos[1] = py;
  pos[2] = pz;
  acc[0] = a0;
  acc[1] = a1;
  acc[2] = a2;
  if (!kick) return;
  double adx = 0.0, ady = 0.0, adz = 0.0;
  if (t >= nb && gas_on)
    mxd::gas_drag(dc, px, py, vel[0] + vpre[0], vel[1] + vpre[1], vel[2] + vpre[2], rp, rhop,
                  adx, ady, adz);
  vel[0] += hh * (a0 + adx);
  vel[1] += hh * (a1 + ady);
  vel[2] += hh * (a2 + adz);
}

// The massive bodies' part of a joined step boundary for one block: from their
// state after the encounter integrator of step n, close step n (momentum sum,
// jump J, frame vpre, the sources in src, gravity, half kick), then open step
// n + 1 (momentum sums, frame Ppre / Ppost, half kick, jump and drift into bst,
// brc).  Every thread of the block calls it (it holds block barriers); lane k <
// nb of the first wave enters with massive body k: bpos, bvel after the
// encounter integrator, its mass bm and changeover radius brc_t.  P, J, vpre,
// Ppre, Ppost come out in every thread.  `latch` reports failures of the
// massive bodies (once per system).
__device__ __forceinline__ void big_boundary(const SysDesc& D, bool latch, double* sh,
                                             KickSource* src, double (*bst)[kSmallBig],
                                             double* brc, double (&bpos)[3], double (&bvel)[3],
                                             double bm, double brc_t, double (&P)[3],
                                             double (&J)[3], double (&vpre)[3],
                                             double (&Ppre)[3], double (&Ppost)[3]) {
  const int tid = threadIdx.x, nb = D.nb;
  const bool w0 = tid < 64;
  const double hh = 0.5 * D.h, mu0 = D.mu0;
  __syncthreads();  // the previous user of the LDS copies is done
  // step n: momentum after the encounter integrator (as k_step_b)
  if (w0) {
    double Q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) Q[c] = mxd::wave_sum_fixed(tid < nb ? bm * bvel[c] : 0.0);
    if (tid == 0)
      for (int c = 0; c < 3; ++c) sh[c] = Q[c];
  }
  __syncthreads();
  for (int c = 0; c < 3; ++c) {
    P[c] = sh[c];
    J[c] = hh * P[c] / mu0;
    vpre[c] = P[c] / mu0;
  }
  if (tid < nb) {
    KickSource k;
    k.x = bpos[0] + J[0];
    k.y = bpos[1] + J[1];
    k.z = bpos[2] + J[2];
    k.mu = bm;
    k.rc2 = fmax(brc_t * brc_t, 1e-300);
    k.rc = brc_t;
    k.pad0 = k.pad1 = 0.0;
    src[tid] = k;
  }
  __syncthreads();
  // step n closed for the massive bodies; the momentum terms of step n + 1
  double bacc[3];
  if (w0) {
    if (tid < nb) {
      close_body(tid, nb, src, src[tid].rc, J, vpre, hh, D.dc, D.gas_on, 0.0, 0.0, true, bpos,
                 bvel, bacc);
      if (latch && !isfinite(bvel[0] + bvel[1] + bvel[2] + bpos[0] + bpos[1] + bpos[2]))
        atomicOr(&D.dsc->err, MXE_NONFINITE);
    }
    big_sums_a(D, tid, sh, bvel, bacc, bm);
  }
  __syncthreads();
  big_frame_a(D, sh, Ppre, Ppost);
  // step n + 1 opened for the massive bodies
  if (tid < nb) big_advance_a(D, latch, tid, bst, brc, bpos, bvel, bacc, brc_t, Ppre, Ppost);
}

// Encounter test of body t (pre-drift p, v; post-drift q, w) against every
// massive body i < t held in LDS (same bound and exact Hermite test as the
// general flag kernel): the bound marks candidates in a bit mask (nb <= 64), then
// the lanes of the wave take their candidates one at a time together, so a wave
// with candidates against different massive bodies runs the Hermite test once
// per round rather than once per body.  Flagged pairs are appended to list lst
// with the append counter of step phase par; the pre-drift state is stored
// where the encounter integrator starts from it.  rec: a flagged massless body
// also appends its subsystem record for the joint launch (phase par; rp, rhop its
// radius and density).  Returns whether the body flagged a pair.
__device__ __forceinline__ void joint_record(const SysDesc& D, int par, int t, uint64_t mask,
                                             const double (&p)[3], const double (&v)[3], double rp,
                                             double rhop) {
  const int idx = atomicAdd(&D.dsc->n_jsub[par], 1);
  if (idx >= D.cap_subs) {
    atomicOr(&D.dsc->err, MXE_SUBSYS);
    return;
  }
  JointSub* R = D.jsub + (size_t)par * D.cap_subs + idx;
  R->mask = mask;
  R->j = t;
  R->pad = 0;
  for (int c = 0; c < 3; ++c) {
    R->x[c] = p[c];
    R->v[c] = v[c];
  }
  R->rp = rp;
  R->rhop = rhop;
}

__device__ __forceinline__ bool flag_body(const SysDesc& D, int par, int lst, int t, int n, int nb,
                                          double h, const double (*bst)[kSmallBig],
                                          const double* brc, const double (&p)[3],
                                          const double (&v)[3], const double (&q)[3],
                                          const double (&w)[3], bool rec = false, double rp = 0.0,
                                          double rhop = 0.0) {
  const double rct = t < nb ? brc[t] : 0.0;
  const int imax = t < nb ? t : nb;
  const double k427 = (4.0 / 27.0) * fabs(h);
  uint64_t cmask = 0;
#pragma unroll 4
  for (int i = 0; i < imax; ++i) {
    double r0[3], w0[3], w1[3], dd[3];
    for (int c = 0; c < 3; ++c) {
      r0[c] = p[c] - bst[c][i];
      w0[c] = v[c] - bst[3 + c][i];
      w1[c] = w[c] - bst[9 + c][i];
      dd[c] = (q[c] - p[c]) - (bst[6 + c][i] - bst[c][i]);
    }
    double m0 = fma(r0[2], r0[2], fma(r0[1], r0[1], r0[0] * r0[0]));
    double nd = fmax(fmax(fabs(dd[0]), fabs(dd[1])), fabs(dd[2]));
    double nw = fmax(fmax(fabs(w0[0]), fabs(w0[1])), fabs(w0[2])) +
                fmax(fmax(fabs(w1[0]), fabs(w1[1])), fabs(w1[2]));
    double rc = fmax(brc[i], rct);
    double bound = rc + 1.7320508075688773 * fma(k427, nw, nd) * (1.0 + 1e-12);
    if (__builtin_expect(m0 <= bound * bound * (1.0 + 1e-12), 0)) cmask |= 1ull << i;
  }
  uint64_t hmask = 0;
  while (cmask != 0) {
    const int i = __builtin_ctzll(cmask);
    cmask &= cmask - 1;
    double r0[3], w0[3], w1[3], r1[3];
    for (int c = 0; c < 3; ++c) {
      r0[c] = p[c] - bst[c][i];
      w0[c] = v[c] - bst[3 + c][i];
      w1[c] = w[c] - bst[9 + c][i];
      r1[c] = q[c] - bst[6 + c][i];
    }
    const double rc = fmax(brc[i], rct);
    double dmin = mxd::hermite_dmin2(r0[0], r0[1], r0[2], w0[0], w0[1], w0[2], r1[0], r1[1],
                                     r1[2], w1[0], w1[1], w1[2], h);
    if (dmin <= rc * rc) hmask |= 1ull << i;
  }
  // the body's pairs are appended together, in increasing i: the list holds each
  // body's partners as one ordered run
  const bool hit = hmask != 0;
  if (rec && hit && t >= nb) joint_record(D, par, t, hmask, p, v, rp, rhop);
  if (hit) {
    const auto list = gbl(D.pairs) + (size_t)lst * 2 * D.cap_pairs;
    int idx = atomicAdd(pair_counter(D.dsc, par), __popcll(hmask));
    for (; hmask != 0; hmask &= hmask - 1, ++idx) {
      if (idx < D.cap_pairs) {
        list[2 * idx] = __builtin_ctzll(hmask);
        list[2 * idx + 1] = t;
      } else {
        atomicOr(&D.dsc->err, MXE_PAIRS);
      }
    }
  }
  // pre-drift state: the encounter integrator starts its subsystems from it
  if (hit || t < nb || D.keep_x0) {
    for (int c = 0; c < 3; ++c) {
      gbl(D.x0)[c * n + t] = p[c];
      gbl(D.u0)[c * n + t] = v[c];
    }
  }
  return hit;
}

// Launches that open step q in a joint sequence (the next launch integrates the
// encounters of step q beside opening step q + 1): the block of the massive
// bodies (bodies 0 .. nb - 1, lane k of the first wave holding massive body k
// with its state q, w after the drift, its mass bm and changeover radius brc_t)
// prepares the boundary that closes step q, when no flagged pair of step q joins
// two massive bodies (the encounter integrator then leaves them as they are),
// with big_boundary's arithmetic: BigNext[ph] and bn_valid[ph] = 1, or
// bn_valid[ph] = 0 when such a pair exists.  Every thread of the block calls it.
__device__ __forceinline__ void prepare_boundary(const SysDesc& D, int ph, bool any_bb,
                                                 double* sh, KickSource* src,
                                                 double (*bst)[kSmallBig], double* brc,
                                                 const double (&q)[3], const double (&w)[3],
                                                 double bm, double brc_t) {
  const int tid = threadIdx.x, nb = D.nb;
  if (any_bb) {
    if (tid == 0) D.dsc->bn_valid[ph] = 0;
    return;
  }
  double bpos[3] = {q[0], q[1], q[2]}, bvel[3] = {w[0], w[1], w[2]};
  double P[3], J[3], vpre[3], Ppre[3], Ppost[3];
  big_boundary(D, true, sh, src, bst, brc, bpos, bvel, bm, brc_t, P, J, vpre, Ppre, Ppost);
  __syncthreads();
  BigNext* N = D.bignext + ph;
  if (tid == 0) {
    for (int c = 0; c < 3; ++c) {
      N->P[c] = P[c];
      N->J[c] = J[c];
      N->vpre[c] = vpre[c];
      N->Ppre[c] = Ppre[c];
      N->Ppost[c] = Ppost[c];
    }
  }
  for (int i = tid; i < 8 * nb; i += blockDim.x)
    reinterpret_cast<double*>(N->src)[i] = reinterpret_cast<const double*>(src)[i];
  for (int i = tid; i < 12 * nb; i += blockDim.x) N->bst[i / nb][i % nb] = bst[i / nb][i % nb];
  for (int i = tid; i < nb; i += blockDim.x) N->brc[i] = brc[i];
  if (tid == 0) D.dsc->bn_valid[ph] = 1;
}

}  // namespace mxs
