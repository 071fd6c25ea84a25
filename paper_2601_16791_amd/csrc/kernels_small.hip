// Fused step kernels for systems with few massive bodies (n_big <= 64), the
// embryo-disk regime: massless planetesimals that feel a handful of embryos.
// Both kernels walk a table of tiles (system, first body), so one launch steps
// one system or a whole batch of independent systems with the same code.
//
//   k_step_a : the block first advances the massive bodies of the tile's system
//              itself (half kick, jump, Kepler drift: the same few bodies in every
//              block, with identical arithmetic) and keeps them in LDS; then each
//              thread takes one body through drag, half kick, jump and drift and
//              tests it against the massive bodies for close encounters (Hermite
//              minimum separation) with the sources read from LDS.
//   k_step_b : jump by the massive-body momentum after the encounter integrator,
//              changeover-weighted gravity from the massive bodies held in LDS,
//              gas drag and the closing half kick.
//
// Between the two runs the Bulirsch-Stoer kernel, which plans its subsystems
// itself.  Three launches per step instead of six, and no packed-source round
// trip through HBM.
// A block takes tpb consecutive tiles (persistent over them) and redoes the
// massive-body phase only when the system changes.  Per body the arithmetic does
// not depend on the tile shape: the block sums run over at most 64 massive bodies,
// one per thread, with the same pairing for every block size >= 64.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "force_sum.h"
#include "mx_internal.h"
#include "step_common.h"

namespace {

using mxd::DragConst;
using namespace mxs;

// Massive bodies of system D for a block: half kick, jump and drift of every
// massive body (identical arithmetic in every block), kept in LDS.  Thread
// tid < nb enters with massive body tid (p, v, a, mass m) already loaded from the
// step-start snapshot.  Returns the momentum terms through Ppre and Ppost.
template <int BLK>
__device__ __forceinline__ void big_phase_a(const SysDesc& D, bool first, double* sh,
                                            double (*bst)[kSmallBig], double* brc,
                                            double (&p)[3], double (&v)[3], const double (&a)[3],
                                            double m, double rc, double (&Ppre)[3],
                                            double (&Ppost)[3]) {
  const int tid = threadIdx.x;
  if (tid < 64) big_sums_a(D, tid, sh, v, a, m);
  __syncthreads();
  big_frame_a(D, sh, Ppre, Ppost);
  if (tid < D.nb) big_advance_a(D, first, tid, bst, brc, p, v, a, rc, Ppre, Ppost);
}

// First half of the fused step over a tile table: per tile, drag + half kick +
// jump + Kepler drift of its bodies and the encounter test against the massive
// bodies.  A block takes `tpb` consecutive tiles and redoes the massive-body
// phase only when the system changes.
// kJoint: the first launch of a joint sequence (single system): the massive
// bodies' pre-drift state also goes to bigpre[par], and the block of the massive
// bodies prepares the boundary that closes this step (prepare_boundary).
template <int BLK, bool kJoint>
__global__ __launch_bounds__(BLK) void k_step_a(const SysDesc* __restrict__ desc,
                                                const Tile* __restrict__ tiles, int n_tiles,
                                                int tpb, int par) {
  __shared__ double sh[8];
  __shared__ double bst[12][kSmallBig];  // x0 (3) u0 (3) x1 (3) u1 (3) of the big bodies
  __shared__ double brc[kSmallBig];
  __shared__ KickSource jsrc[kJoint ? kSmallBig : 1];
  const int tid = threadIdx.x;
  const int t_lo = blockIdx.x * tpb;
  const int t_hi = min(n_tiles, t_lo + tpb);
  int cur = -1;
  double Ppre[3], Ppost[3];
  for (int ti = t_lo; ti < t_hi; ++ti) {
    const Tile tl = tiles[ti];
    const SysDesc& D = desc[tl.sys];
    const int n = D.n, nb = D.nb;
    const double h = D.h;
    const int t = tl.first + tid;
    const bool fresh = tl.sys != cur;  // block-uniform
    // the massive bodies (step-start snapshot: the owner tile overwrites x, u of
    // the massive bodies while other blocks may still be reading) are requested
    // first, then the body's own state: the massive-body phase waits only for the
    // former, and the latter arrives while it runs
    double bp[3], bv[3], ba[3], bm = 0.0, brc_t = 0.0;
    if (fresh && tid < nb) {
      const auto bigsnap = gbl(D.bigsnap);
      bm = gbl(D.mu)[tid];
      brc_t = gbl(D.rcrit)[tid];
      for (int c = 0; c < 3; ++c) {
        bp[c] = bigsnap[c * nb + tid];
        bv[c] = bigsnap[(3 + c) * nb + tid];
        ba[c] = bigsnap[(6 + c) * nb + tid];
      }
    }
    double p[3], v[3], q[3], w[3], a[3], rp = 0.0, rhop = 0.0;
    if (t < n && t >= nb) {
      for (int c = 0; c < 3; ++c) {
        p[c] = gbl(D.x)[c * n + t];
        v[c] = gbl(D.u)[c * n + t];
        a[c] = gbl(D.ag)[c * n + t];
      }
      if (D.gas_on) {
        rp = gbl(D.r_p)[t - nb];
        rhop = gbl(D.rho_p)[t - nb];
      }
    }
    if (fresh) {
      __syncthreads();  // the previous tile is done with the LDS copies
      big_phase_a<BLK>(D, tl.first == 0, sh, bst, brc, bp, bv, ba, bm, brc_t, Ppre, Ppost);
      __syncthreads();
      cur = tl.sys;
    }
    bool hit = false;
    if (t < n) {
      if (t < nb) {
        for (int c = 0; c < 3; ++c) {
          p[c] = bst[c][t];
          v[c] = bst[3 + c][t];
          q[c] = bst[6 + c][t];
          w[c] = bst[9 + c][t];
        }
        const auto bigmid = gbl(D.bigmid) + (size_t)par * 6 * nb;
        for (int c = 0; c < 3; ++c) {
          bigmid[c * nb + t] = q[c];
          bigmid[(3 + c) * nb + t] = w[c];
        }
        if (kJoint) {
          const auto bigpre = gbl(D.bigpre) + (size_t)par * 6 * nb;
          for (int c = 0; c < 3; ++c) {
            bigpre[c * nb + t] = p[c];
            bigpre[(3 + c) * nb + t] = v[c];
          }
        }
      } else {
        if (!advance_body(t, nb, D.mu0, h, D.dc, D.gas_on, rp, rhop, Ppre, Ppost, p, v, a, q, w))
          atomicOr(&D.dsc->err, MXE_NOCONV);
      }
      for (int c = 0; c < 3; ++c) {
        gbl(D.x)[c * n + t] = q[c];
        gbl(D.u)[c * n + t] = w[c];
      }
      hit = flag_body(D, par, kJoint ? par : 0, t, n, nb, h, bst, brc, p, v, q, w, kJoint, rp,
                      rhop);
    }
    if (kJoint && tl.first == 0) {  // block-uniform: the block of the massive bodies
      const bool any_bb = __syncthreads_or(t < nb && hit);
      prepare_boundary(D, par, any_bb, sh, jsrc, bst, brc, q, w, bm, brc_t);
    }
  }
}

// Second half of the fused step over a tile table: jump by the massive-body
// momentum after the encounter integrator, changeover-weighted gravity from the
// massive bodies held in LDS, gas drag and (kick != 0) the closing half kick.
template <int BLK>
__global__ __launch_bounds__(BLK) void k_step_b(const SysDesc* __restrict__ desc,
                                                const Tile* __restrict__ tiles, int n_tiles,
                                                int tpb, int kick, int par) {
  __shared__ double sh[4];
  __shared__ KickSource src[kSmallBig];
  const int tid = threadIdx.x;
  const int t_lo = blockIdx.x * tpb;
  const int t_hi = min(n_tiles, t_lo + tpb);
  int cur = -1;
  double P[3], J[3], vpre[3];
  for (int ti = t_lo; ti < t_hi; ++ti) {
    const Tile tl = tiles[ti];
    const SysDesc& D = desc[tl.sys];
    const int n = D.n, nb = D.nb;
    const double hh = 0.5 * D.h, mu0 = D.mu0;
    const int t = tl.first + tid;
    const auto x = gbl(D.x);
    const auto u = gbl(D.u);
    const auto ag = gbl(D.ag);
    const bool fresh = tl.sys != cur;  // block-uniform
    // massive bodies after drift and encounters from their snapshot (the owner
    // tile overwrites x, u of the massive bodies while other blocks may read),
    // requested before the body's own state
    double bx = 0.0, by = 0.0, bz = 0.0, bm = 0.0, brc = 0.0;
    double Q[3] = {0.0, 0.0, 0.0};
    if (fresh && tid < nb) {
      const auto bigmid = gbl(D.bigmid) + (size_t)par * 6 * nb;
      bx = bigmid[tid];
      by = bigmid[nb + tid];
      bz = bigmid[2 * nb + tid];
      bm = gbl(D.mu)[tid];
      brc = gbl(D.rcrit)[tid];
      for (int c = 0; c < 3; ++c) Q[c] = bigmid[(3 + c) * nb + tid];
    }
    double x0 = 0.0, x1 = 0.0, x2 = 0.0, vx = 0.0, vy = 0.0, vz = 0.0, rp = 0.0, rhop = 0.0;
    if (t < n) {
      x0 = x[t];
      x1 = x[n + t];
      x2 = x[2 * n + t];
      if (kick) {
        vx = u[t];
        vy = u[n + t];
        vz = u[2 * n + t];
        if (t >= nb && D.gas_on) {
          rp = gbl(D.r_p)[t - nb];
          rhop = gbl(D.rho_p)[t - nb];
        }
      }
    }
    if (fresh) {
      __syncthreads();  // the previous tile is done with the LDS sources
      // the first wave sums the momentum by the fixed lane reduction (the same
      // bits in every block)
      if (tid < 64) {
#pragma unroll
        for (int c = 0; c < 3; ++c) Q[c] = mxd::wave_sum_fixed(bm * Q[c]);
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
        k.x = bx + J[0];
        k.y = by + J[1];
        k.z = bz + J[2];
        k.mu = bm;
        k.rc2 = fmax(brc * brc, 1e-300);
        k.rc = brc;
        k.pad0 = k.pad1 = 0.0;
        src[tid] = k;
      }
      __syncthreads();
      cur = tl.sys;
    }
    if (tl.first == 0 && tid == 0) {
      D.dsc->P[0] = P[0];
      D.dsc->P[1] = P[1];
      D.dsc->P[2] = P[2];
      if (kick) {
        D.dsc->step += 1;
        for (int r = 0; r < 3; ++r) {  // the encounter lists of the call have been planned
          D.dsc->n_pairs[r] = 0;
          D.dsc->plan_ready[r] = 0;
          D.dsc->bs_done[r] = 0;
          D.dsc->n_jsub[r] = 0;
        }
      }
    }
    if (t >= n) continue;
    double pos[3] = {x0, x1, x2}, vel[3] = {vx, vy, vz}, acc[3];
    close_body(t, nb, src, t < nb ? src[t].rc : 0.0, J, vpre, hh, D.dc, D.gas_on, rp, rhop,
               kick != 0, pos, vel, acc);
    const double px = pos[0], py = pos[1], pz = pos[2];
    const double a0 = acc[0], a1 = acc[1], a2 = acc[2];
    x[t] = px;
    x[n + t] = py;
    x[2 * n + t] = pz;
    ag[t] = a0;
    ag[n + t] = a1;
    ag[2 * n + t] = a2;
    if (!kick) continue;
    vx = vel[0];
    vy = vel[1];
    vz = vel[2];
    u[t] = vx;
    u[n + t] = vy;
    u[2 * n + t] = vz;
    if (!isfinite(vx + vy + vz + px + py + pz)) atomicOr(&D.dsc->err, MXE_NONFINITE);
    if (t < nb) {
      const auto bigsnap = gbl(D.bigsnap);
      bigsnap[t] = px; bigsnap[nb + t] = py; bigsnap[2 * nb + t] = pz;
      bigsnap[3 * nb + t] = vx; bigsnap[4 * nb + t] = vy; bigsnap[5 * nb + t] = vz;
      bigsnap[6 * nb + t] = a0; bigsnap[7 * nb + t] = a1; bigsnap[8 * nb + t] = a2;
    }
  }
}

// Two steps joined at their boundary: the closing part of step n (as k_step_b,
// with kick) and the opening part of step n + 1 (as k_step_a) in one pass over
// the tiles, the body's state staying in registers in between.  Each block
// closes step n for the massive bodies itself, from their state after the
// encounter integrator (the same arithmetic as the owner tile of k_step_b, in
// every block), then advances them as k_step_a does; every body sees exactly the
// operations of k_step_b followed by k_step_a.  What only those kernels store in
// between (positions after the jump, accelerations, the massive-body snapshot)
// is not stored.  Step n's massive bodies are read from bigmid buffer par (every
// block reads them), step n + 1's are written to buffer par ^ 1, and its flagged
// pairs are counted by the append counter of parity par ^ 1: no block overwrites
// what another may still read.  (A variant that gave the massive bodies a wave
// of their own measured slower: at this kernel's register use a CU holds only
// one five-wave block.)
template <int BLK>
__global__ __launch_bounds__(BLK) void k_step_ba(const SysDesc* __restrict__ desc,
                                                 const Tile* __restrict__ tiles, int n_tiles,
                                                 int tpb, int par) {
  __shared__ double sh[8];
  __shared__ KickSource src[kSmallBig];
  __shared__ double bst[12][kSmallBig];
  __shared__ double brc[kSmallBig];
  const int tid = threadIdx.x;
  const int t_lo = blockIdx.x * tpb;
  const int t_hi = min(n_tiles, t_lo + tpb);
  int cur = -1;
  double J[3], vpre[3], Ppre[3], Ppost[3];
  // the massive body of this lane of the first wave (lane < nb) for a fresh tile
  double bpos[3], bvel[3], bm = 0.0, brc_t = 0.0;
  for (int ti = t_lo; ti < t_hi; ++ti) {
    const Tile tl = tiles[ti];
    const SysDesc& D = desc[tl.sys];
    const int n = D.n, nb = D.nb;
    const double h = D.h, hh = 0.5 * D.h, mu0 = D.mu0;
    const int t = tl.first + tid;
    const bool mine = t < n;
    const bool fresh = tl.sys != cur;  // block-uniform
    // massive bodies after the encounter integrator, then the body's own state
    if (fresh && tid < nb) {
      const auto bigmid = gbl(D.bigmid) + (size_t)par * 6 * nb;
      for (int c = 0; c < 3; ++c) {
        bpos[c] = bigmid[c * nb + tid];
        bvel[c] = bigmid[(3 + c) * nb + tid];
      }
      bm = gbl(D.mu)[tid];
      brc_t = gbl(D.rcrit)[tid];
    }
    double p[3], v[3], a[3], q[3], w[3], rp = 0.0, rhop = 0.0;
    if (mine && t >= nb) {
      for (int c = 0; c < 3; ++c) {
        p[c] = gbl(D.x)[c * n + t];
        v[c] = gbl(D.u)[c * n + t];
      }
      if (D.gas_on) {
        rp = gbl(D.r_p)[t - nb];
        rhop = gbl(D.rho_p)[t - nb];
      }
    }
    if (fresh) {
      double P[3];
      // the encounter integrator of step n may have prepared the massive bodies
      // of this boundary (when it left them unchanged): they are copied into LDS
      // while the flag that says so is read, and computed here otherwise
      const BigNext* N = D.bignext + par;
      const int pre = nb > 0 ? D.dsc->bn_valid[par] : 0;
      __syncthreads();  // the previous tile is done with the LDS copies
      if (nb > 0) {
        for (int i = tid; i < 8 * nb; i += BLK)
          reinterpret_cast<double*>(src)[i] = reinterpret_cast<const double*>(N->src)[i];
        for (int i = tid; i < 12 * nb; i += BLK) bst[i / nb][i % nb] = N->bst[i / nb][i % nb];
        for (int i = tid; i < nb; i += BLK) brc[i] = N->brc[i];
      }
      if (pre) {
        for (int c = 0; c < 3; ++c) {
          P[c] = N->P[c];
          J[c] = N->J[c];
          vpre[c] = N->vpre[c];
          Ppre[c] = N->Ppre[c];
          Ppost[c] = N->Ppost[c];
        }
        __syncthreads();
      } else {
        big_boundary(D, tl.first == 0, sh, src, bst, brc, bpos, bvel, bm, brc_t, P, J, vpre, Ppre,
                     Ppost);
      }
      if (tl.first == 0 && tid == 0) {
        D.dsc->P[0] = P[0];
        D.dsc->P[1] = P[1];
        D.dsc->P[2] = P[2];
        D.dsc->step += 1;
        D.dsc->plan_ready[par] = 0;
      }
      cur = tl.sys;
    }
    // step n closed and step n + 1 opened for the body
    if (mine && t >= nb) {
      close_body(t, nb, src, 0.0, J, vpre, hh, D.dc, D.gas_on, rp, rhop, true, p, v, a);
      if (!isfinite(v[0] + v[1] + v[2] + p[0] + p[1] + p[2]))
        atomicOr(&D.dsc->err, MXE_NONFINITE);
      if (!advance_body(t, nb, mu0, h, D.dc, D.gas_on, rp, rhop, Ppre, Ppost, p, v, a, q, w))
        atomicOr(&D.dsc->err, MXE_NOCONV);
    }
    __syncthreads();  // the massive bodies of step n + 1 are in LDS
    if (mine) {
      if (t < nb) {
        for (int c = 0; c < 3; ++c) {
          p[c] = bst[c][t];
          v[c] = bst[3 + c][t];
          q[c] = bst[6 + c][t];
          w[c] = bst[9 + c][t];
        }
        // step n + 1's massive bodies go to the other bigmid buffer
        const auto bigmid = gbl(D.bigmid) + (size_t)(par ^ 1) * 6 * nb;
        for (int c = 0; c < 3; ++c) {
          bigmid[c * nb + t] = q[c];
          bigmid[(3 + c) * nb + t] = w[c];
        }
      }
      for (int c = 0; c < 3; ++c) {
        gbl(D.x)[c * n + t] = q[c];
        gbl(D.u)[c * n + t] = w[c];
      }
      flag_body(D, par ^ 1, 0, t, n, nb, h, bst, brc, p, v, q, w);
    }
  }
}

}  // namespace

namespace mxk {

hipError_t launch_step_a_tiles(hipStream_t st, LaunchTiming* tm, const SysDesc* desc,
                               const Tile* tiles, int n_tiles, int blk, int tpb, int par,
                               int joint) {
  if (n_tiles <= 0) return hipSuccess;
  const dim3 grid((n_tiles + tpb - 1) / tpb);
  if (joint)
    return blk == 256 ? mxlaunch_on(st, tm, k_step_a<256, true>, grid, dim3(256), desc, tiles,
                                    n_tiles, tpb, par)
                      : hipErrorInvalidValue;
  switch (blk) {
    case 64: return mxlaunch_on(st, tm, k_step_a<64, false>, grid, dim3(64), desc, tiles, n_tiles, tpb, par);
    case 128: return mxlaunch_on(st, tm, k_step_a<128, false>, grid, dim3(128), desc, tiles, n_tiles, tpb, par);
    case 256: return mxlaunch_on(st, tm, k_step_a<256, false>, grid, dim3(256), desc, tiles, n_tiles, tpb, par);
    case 512: return mxlaunch_on(st, tm, k_step_a<512, false>, grid, dim3(512), desc, tiles, n_tiles, tpb, par);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step_ba_tiles(hipStream_t st, LaunchTiming* tm, const SysDesc* desc,
                                const Tile* tiles, int n_tiles, int blk, int tpb, int par) {
  if (n_tiles <= 0) return hipSuccess;
  const dim3 grid((n_tiles + tpb - 1) / tpb);
  switch (blk) {
    case 64:
      return mxlaunch_on(st, tm, k_step_ba<64>, grid, dim3(64), desc, tiles, n_tiles, tpb, par);
    case 128:
      return mxlaunch_on(st, tm, k_step_ba<128>, grid, dim3(128), desc, tiles, n_tiles, tpb, par);
    case 256:
      return mxlaunch_on(st, tm, k_step_ba<256>, grid, dim3(256), desc, tiles, n_tiles, tpb, par);
    case 512:
      return mxlaunch_on(st, tm, k_step_ba<512>, grid, dim3(512), desc, tiles, n_tiles, tpb, par);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step_b_tiles(hipStream_t st, LaunchTiming* tm, const SysDesc* desc,
                               const Tile* tiles, int n_tiles, int blk, int tpb, int kick,
                               int par) {
  if (n_tiles <= 0) return hipSuccess;
  const dim3 grid((n_tiles + tpb - 1) / tpb);
  switch (blk) {
    case 64:
      return mxlaunch_on(st, tm, k_step_b<64>, grid, dim3(64), desc, tiles, n_tiles, tpb, kick, par);
    case 128:
      return mxlaunch_on(st, tm, k_step_b<128>, grid, dim3(128), desc, tiles, n_tiles, tpb, kick, par);
    case 256:
      return mxlaunch_on(st, tm, k_step_b<256>, grid, dim3(256), desc, tiles, n_tiles, tpb, kick, par);
    case 512:
      return mxlaunch_on(st, tm, k_step_b<512>, grid, dim3(512), desc, tiles, n_tiles, tpb, kick, par);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mxk
