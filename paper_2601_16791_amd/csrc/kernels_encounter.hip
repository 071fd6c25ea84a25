// Close encounters of the hybrid step (gfx950): flagging, planning and the
// Bulirsch-Stoer hand-off.
//
//   k_flag       : every unordered pair {big i, body j > i}; a conservative bound
//                  on the relative motion rejects far pairs with ~30 FP64 ops, the
//                  rest get the Hermite minimum-separation test; flagged pairs are
//                  appended with an integer atomic (the mce_snif critical region of
//                  Sect. 2.1.2 becomes a ticket counter)
//   k_plan       : one block: bitonic sort of the list by (i, j) (deterministic
//                  order whatever the append order was), connected big-big
//                  components, and one subsystem per flagged massless body with
//                  copies of the big components it touches; ordered compactions
//                  by block-wide prefix sums, one massless subsystem per thread
//   k_bs         : one wave per subsystem; the eight Stoermer sequences of a BS
//                  step run in eight lanes at once, the Aitken-Neville table is
//                  built across lanes, and the first accepted column is taken, the
//                  same column a sequential integrator would stop at.  Pair forces
//                  inside a subsystem are owner-computed in one lane (no atomics,
//                  the fo_hkce critical region of Sect. 2.1.2 disappears).  For
//                  systems of at most 64 massive bodies the blocks plan the
//                  subsystems themselves first (see FastPlan), without k_plan.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "mx_internal.h"
#include "step_common.h"

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
  FlagSource S;
  if (s0 < s1) S = fp[s0];
  for (int i = s0; i < s1; ++i) {
    const FlagSource N = fp[i + 1 < s1 ? i + 1 : i];  // requested ahead of use
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
    S = N;
  }
}

// ------------------------------------------------------- flag, culled form
// Systems of massive bodies only (n_big > 64, no massless body): the bodies are
// taken in an order of increasing heliocentric distance fixed at init (`perm`)
// and cut into 64-body chunks.  k_chunk_bounds gives every chunk the range of its
// bodies' distances at the step start, the largest reach
// R = |Delta|_inf + (4/27) h (|u0|_inf + |u1|_inf) and the largest changeover
// radius (ChunkBound; a separate launch: taking the bodies in this order in the
// drift kernel scatters its accesses and costs more than the launch).  A wave takes a pair of chunks (S <= T;
// every unordered pair of bodies once): every pair's separation at the step
// start is at least the radial gap
// of the chunks (| |a| - |b| | <= |a - b|), and every pair's cheap bound is at
// most rc_max + sqrt(3) (R_T + R_S), because the relative displacement and
// velocities are differences of the bodies' own.  A unit whose gap exceeds that
// (with a margin for rounding) has no candidate and stops.  The order is only a
// heuristic: a stale order makes the bound weaker, never wrong.  A chunk pair
// that is not rejected is tested by four waves, each with a quarter of chunk S
// (so the surviving work spreads over the chip).  The cheap bound
// and the Hermite minimum are symmetric in the two bodies (the relative
// quantities only change sign), so each pair is tested with the chunk roles as
// they come and appended as (smaller index, larger index).
__device__ __forceinline__ double wave_min_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

__global__ __launch_bounds__(64) void k_chunk_bounds(int nb, double h,
                                                     const int32_t* __restrict__ perm,
                                                     const FlagSource* __restrict__ fp,
                                                     ChunkBound* __restrict__ cb) {
  const int lane = threadIdx.x, p = blockIdx.x * 64 + lane;
  const bool v = p < nb;
  const FlagSource& F = fp[v ? perm[p] : perm[0]];
  const double k427 = (4.0 / 27.0) * fabs(h);
  const double r = sqrt(fma(F.z0, F.z0, fma(F.y0, F.y0, F.x0 * F.x0)));
  const double reach = fmax(fmax(fabs(F.dx), fabs(F.dy)), fabs(F.dz)) +
                       k427 * (fmax(fmax(fabs(F.u0x), fabs(F.u0y)), fabs(F.u0z)) +
                               fmax(fmax(fabs(F.u1x), fabs(F.u1y)), fabs(F.u1z)));
  const double inf = __builtin_inf();
  const double rmin = wave_min_d(v ? r : inf), rmax = wave_max_d(v ? r : -inf);
  const double R = wave_max_d(v ? reach : 0.0), rc = wave_max_d(v ? F.rc : 0.0);
  if (lane == 0) cb[blockIdx.x] = ChunkBound{rmin, rmax, R, rc};
}

constexpr int kCullPart = 16;  // sources of chunk S per wave: four waves per chunk pair

struct FlagRec {  // the fields of a source record the cheap bound uses
  double x0, y0, z0, u0x, u0y, u0z, dx, dy, dz, u1x, u1y, u1z, rc;
};
__device__ __forceinline__ FlagRec flag_rec(const FlagSource& f) {
  return FlagRec{f.x0, f.y0, f.z0, f.u0x, f.u0y, f.u0z, f.dx, f.dy, f.dz, f.u1x, f.u1y, f.u1z, f.rc};
}

__global__ __launch_bounds__(64) void k_flag_cull(
    int nb, double h, const int32_t* __restrict__ perm, const ChunkBound* __restrict__ cb,
    const double* __restrict__ x0s, const double* __restrict__ u0s,
    const double* __restrict__ x1s, const double* __restrict__ u1s,
    const FlagSource* __restrict__ fp, int32_t* __restrict__ pairs, int32_t cap,
    int32_t* __restrict__ counter, int32_t* __restrict__ err) {
  __shared__ FlagSource ls[kCullPart];
  const int lane = threadIdx.x;
  const int u = blockIdx.x / (64 / kCullPart);            // chunk pair
  const int q0 = (blockIdx.x % (64 / kCullPart)) * kCullPart;  // first source of this part
  // unit u -> chunks (T, S), S <= T, units in order of T
  int T = (int)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
  while (T * (T + 1) / 2 > u) --T;
  while ((T + 1) * (T + 2) / 2 <= u) ++T;
  const int S = u - T * (T + 1) / 2;
  const ChunkBound bT = cb[T], bS = cb[S];
  const double gap = fmax(0.0, fmax(bS.rmin - bT.rmax, bT.rmin - bS.rmax));
  const double B = fmax(bT.rc, bS.rc) + 1.7320508075688773 * (bT.reach + bS.reach) * (1.0 + 1e-12);
  if (gap > B * (1.0 + 1e-9)) return;  // no pair of the unit is a candidate
  const int n = nb;  // the arrays' stride: no massless body
  const double k427 = (4.0 / 27.0) * fabs(h);
  // this part's source records into LDS (one round trip), this lane's target of chunk T
  const int q1 = min(q0 + kCullPart, nb - S * 64);
  if (q0 >= q1) return;
  {
    constexpr int kW = sizeof(FlagSource) / sizeof(double);
    double* dst = reinterpret_cast<double*>(ls);
    for (int e = lane; e < (q1 - q0) * kW; e += 64)
      dst[e] = reinterpret_cast<const double*>(fp + perm[S * 64 + q0 + e / kW])[e % kW];
  }
  const int pt = T * 64 + lane;
  const bool tv = pt < nb;
  const int jb = tv ? perm[pt] : perm[0];
  const double ax0 = x0s[jb], ay0 = x0s[n + jb], az0 = x0s[2 * n + jb];
  const double bx0 = u0s[jb], by0 = u0s[n + jb], bz0 = u0s[2 * n + jb];
  const double bx1 = u1s[jb], by1 = u1s[n + jb], bz1 = u1s[2 * n + jb];
  const double djx = x1s[jb] - ax0, djy = x1s[n + jb] - ay0, djz = x1s[2 * n + jb] - az0;
  const double rcj = fp[jb].rc;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint64_t mask = 0;  // bit q - q0: source q of chunk S is a candidate
  FlagRec Sr = flag_rec(ls[0]);
  for (int q = q0; q < q1; ++q) {
    const FlagRec N = flag_rec(ls[(q + 1 < q1 ? q + 1 : q) - q0]);  // read while this one is tested
    const double r0x = ax0 - Sr.x0, r0y = ay0 - Sr.y0, r0z = az0 - Sr.z0;
    const double w0x = bx0 - Sr.u0x, w0y = by0 - Sr.u0y, w0z = bz0 - Sr.u0z;
    const double w1x = bx1 - Sr.u1x, w1y = by1 - Sr.u1y, w1z = bz1 - Sr.u1z;
    const double ddx = djx - Sr.dx, ddy = djy - Sr.dy, ddz = djz - Sr.dz;
    const double m0 = fma(r0z, r0z, fma(r0y, r0y, r0x * r0x));
    const double nd = fmax(fmax(fabs(ddx), fabs(ddy)), fabs(ddz));
    const double nw = fmax(fmax(fabs(w0x), fabs(w0y)), fabs(w0z)) +
                      fmax(fmax(fabs(w1x), fabs(w1y)), fabs(w1z));
    const double rc = fmax(Sr.rc, rcj);
    // |r(tau) - r0| <= |Delta| + (4/27) h (|w0| + |w1|) for the cubic Hermite on [0,1]
    const double bound = rc + 1.7320508075688773 * fma(k427, nw, nd) * (1.0 + 1e-12);
    // each unordered pair once: the whole square off the diagonal, below it on it
    const bool own = tv & ((T > S) | (q < lane));
    const bool cand = own & (m0 <= bound * bound * (1.0 + 1e-12));
    mask |= (uint64_t)cand << (q - q0);
    Sr = N;
  }
  while (mask != 0) {
    const int q = q0 + __builtin_ctzll(mask);
    mask &= mask - 1;
    const int i = perm[S * 64 + q];
    const FlagSource& Si = fp[i];
    const double w0x = bx0 - Si.u0x, w0y = by0 - Si.u0y, w0z = bz0 - Si.u0z;
    const double w1x = bx1 - Si.u1x, w1y = by1 - Si.u1y, w1z = bz1 - Si.u1z;
    const double r1x = x1s[jb] - x1s[i], r1y = x1s[n + jb] - x1s[n + i],
                 r1z = x1s[2 * n + jb] - x1s[2 * n + i];
    const double q0x = ax0 - x0s[i], q0y = ay0 - x0s[n + i], q0z = az0 - x0s[2 * n + i];
    const double dmin = mxd::hermite_dmin2(q0x, q0y, q0z, w0x, w0y, w0z, r1x, r1y, r1z, w1x, w1y,
                                           w1z, h);
    const double rc = fmax(Si.rc, rcj);
    if (dmin <= rc * rc) {
      const int idx = atomicAdd(counter, 1);
      if (idx < cap) {
        pairs[2 * idx] = min(i, jb);
        pairs[2 * idx + 1] = max(i, jb);
      } else {
        atomicOr(err, MXE_PAIRS);
      }
    }
  }
}

// Bitonic sort of p2 (a power of two) 64-bit keys with the first T threads of a
// block; `key` may point to LDS or to global memory.
__device__ void block_bitonic(int64_t* key, int p2, int T) {
  for (int k = 2; k <= p2; k <<= 1) {
    for (int jx = k >> 1; jx > 0; jx >>= 1) {
      for (int i = threadIdx.x; i < p2; i += T) {
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

// Ordered compaction over q in [0, m): emit(position, q) for every q with pred(q),
// positions in increasing q.  Each thread scans a contiguous chunk; chunk counts
// are prefix-summed in LDS (Hillis-Steele) over the first T threads of the block.
// Returns the total (the same in every thread).
template <class Pred, class Emit>
__device__ int block_compact(int m, Pred pred, Emit emit, int* scan, int T) {
  const int tid = threadIdx.x;
  const int per = (m + T - 1) / T;
  const int b = min(m, tid * per), e = min(m, b + per);
  int c = 0;
  for (int q = b; q < e; ++q) c += pred(q) ? 1 : 0;
  scan[tid] = c;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    int v = tid >= off ? scan[tid - off] : 0;
    __syncthreads();
    scan[tid] += v;
    __syncthreads();
  }
  int pos = scan[tid] - c;
  for (int q = b; q < e; ++q)
    if (pred(q)) emit(pos++, q);
  int total = scan[T - 1];
  __syncthreads();
  return total;
}

__device__ __forceinline__ int key_hi(int64_t k) { return (int)(k >> 32); }
__device__ __forceinline__ int key_lo(int64_t k) { return (int)(k & 0xffffffff); }
__device__ __forceinline__ int64_t make_key(int a, int b) {
  return (((int64_t)a) << 32) | (uint32_t)b;
}

__device__ int uf_find(const int32_t* par, int a) {
  while (par[a] != a) a = par[a];
  return a;
}

__device__ int index_in(const int32_t* v, int m, int b) {
  for (int k = 0; k < m; ++k)
    if (v[k] == b) return k;
  return -1;
}

__device__ bool insert_sorted(int32_t* v, int& m, int cap, int b) {
  if (index_in(v, m, b) >= 0) return true;
  if (m >= cap) return false;
  int k = m;
  while (k > 0 && v[k - 1] > b) {
    v[k] = v[k - 1];
    --k;
  }
  v[k] = b;
  ++m;
  return true;
}

// ---- single-wave planner for short lists of massless encounters
// Sort of np distinct keys in[0, np) into out by rank: the rank of a key is the
// number of smaller keys, counted against every key read as a wave-uniform LDS
// broadcast, 32 reads in flight per round.  in[np, np rounded up to 32) must
// hold key_max (never smaller than a key), so every round is whole; np <= 256.
// One wave; its LDS accesses complete in order.
__device__ __forceinline__ int64_t key_max(int64_t) { return INT64_MAX; }
__device__ __forceinline__ uint32_t key_max(uint32_t) { return 0xffffffffu; }

template <class K>
__device__ __forceinline__ void wave_rank_sort(const K* in, K* out, int np) {
  const int lane = threadIdx.x & 63;
  const int nr = (np + 63) >> 6;  // key slots in use per lane
  const int np32 = (np + 31) & ~31;
  K key[4];
  int rank[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = 64 * r + lane;
    key[r] = e < np ? in[e] : key_max(K());
    rank[r] = 0;
  }
  for (int f = 0; f < np32; f += 32) {
    K kk[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) kk[q] = in[f + q];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (r < nr) {
        int c = 0;
#pragma unroll
        for (int q = 0; q < 32; ++q) c += kk[q] < key[r];
        rank[r] += c;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (64 * r + lane < np) out[rank[r]] = key[r];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// key_max into in[np, np rounded up to 32): the padding wave_rank_sort reads
template <class K>
__device__ __forceinline__ void pad_keys(K* in, int np) {
  const int lane = threadIdx.x & 63;
  const int e = np + lane;
  if (e < ((np + 31) & ~31)) in[e] = key_max(K());
}

constexpr int kPlanThreads = 256;
constexpr int kPlanLds = 2048;   // pairs handled in LDS; larger lists use global scratch

// General plan (any list): sort by (i, j), big-big components by union-find,
// one subsystem per flagged massless body.  K, S: 64-bit key arrays of at least
// next_pow2(np) entries; BB, GS: index arrays of np entries (LDS or global
// scratch); scan: T ints of LDS.  Run by the first T threads of the block (the
// block's other threads, if any, have exited).  write_back: the list itself is
// left sorted (else only the subsystem table is written).
__device__ void plan_general(int nb, gmem<int32_t> gpairs, int np, int64_t* K, int64_t* S,
                             int32_t* BB, int32_t* GS, int32_t* __restrict__ uf,
                             Subsystem* __restrict__ subs, int32_t cap_subs,
                             DevScalars* __restrict__ dsc, int sort_only, int* scan,
                             int* s_nbig_sub, int T, bool write_back) {
  const int tid = threadIdx.x;
  // 1. sort by (i, j)
  int p2 = next_pow2(np);
  for (int q = tid; q < p2; q += T)
    K[q] = q < np ? make_key(gpairs[2 * q], gpairs[2 * q + 1]) : INT64_MAX;
  __syncthreads();
  if (np > 1) block_bitonic(K, p2, T);
  if (write_back) {
    for (int q = tid; q < np; q += T) {
      gpairs[2 * q] = key_hi(K[q]);
      gpairs[2 * q + 1] = key_lo(K[q]);
    }
  }
  if (sort_only) return;
  // 2. big-big pairs (in (i, j) order) and massless pairs keyed (j, i)
  const int nbb = block_compact(
      np, [&](int q) { return key_lo(K[q]) < nb; }, [&](int pos, int q) { BB[pos] = q; }, scan, T);
  const int ns = block_compact(
      np, [&](int q) { return key_lo(K[q]) >= nb; },
      [&](int pos, int q) { S[pos] = make_key(key_lo(K[q]), key_hi(K[q])); }, scan, T);
  int p2s = next_pow2(ns > 0 ? ns : 1);
  for (int q = ns + tid; q < p2s; q += T) S[q] = INT64_MAX;
  __syncthreads();
  if (ns > 1) block_bitonic(S, p2s, T);
  // 3. one group per flagged massless body
  const int ng = block_compact(
      ns, [&](int q) { return q == 0 || key_hi(S[q]) != key_hi(S[q - 1]); },
      [&](int pos, int q) { GS[pos] = q; }, scan, T);
  int32_t* par = uf;
  int32_t* inbig = uf + nb;
  // 4. components of the big-big graph and their subsystems (one thread; the
  //    big-big list is short)
  if (tid == 0) {
    for (int b = 0; b < nbb; ++b) {
      int64_t k = K[BB[b]];
      int i = key_hi(k), j = key_lo(k);
      int ri = uf_find(par, i), rj = uf_find(par, j);
      if (ri != rj) {
        if (ri < rj) par[rj] = ri;
        else par[ri] = rj;
      }
      inbig[i] = 1;
      inbig[j] = 1;
    }
    int nsub = 0;
    for (int b = 0; b < nbb; ++b) {
      int i = key_hi(K[BB[b]]);
      int r = uf_find(par, i);
      if (inbig[r] != 1) continue;  // component already emitted (root marked 2)
      if (nsub >= cap_subs) {
        inbig[r] = 2;
        atomicOr(&dsc->err, MXE_SUBSYS);
        continue;
      }
      Subsystem& sub = subs[nsub];  // built in place (no private copy)
      sub.m = 0;
      sub.keep_from = 0;
      sub.np = 0;
      sub.jm = 0;
      bool ok = true;
      for (int c = 0; c < nbb && ok; ++c) {
        int64_t k = K[BB[c]];
        if (uf_find(par, key_hi(k)) != r) continue;
        ok = insert_sorted(sub.mem, sub.m, kBsMaxMembers, key_hi(k)) &&
             insert_sorted(sub.mem, sub.m, kBsMaxMembers, key_lo(k));
      }
      for (int c = 0; c < nbb && ok; ++c) {
        int64_t k = K[BB[c]];
        if (uf_find(par, key_hi(k)) != r) continue;
        if (sub.np >= kBsMaxPairs) { ok = false; break; }
        sub.pl[sub.np][0] = index_in(sub.mem, sub.m, key_hi(k));
        sub.pl[sub.np][1] = index_in(sub.mem, sub.m, key_lo(k));
        ++sub.np;
      }
      inbig[r] = 2;
      if (!ok) {
        atomicOr(&dsc->err, MXE_SUBSYS);
        continue;
      }
      ++nsub;
    }
    *s_nbig_sub = nsub;
  }
  __syncthreads();
  const int nbig_sub = *s_nbig_sub;
  // 5. massless subsystems, one group per thread
  for (int g = tid; g < ng; g += T) {
    const int q0 = GS[g];
    const int q1 = g + 1 < ng ? GS[g + 1] : ns;
    const int j = key_hi(S[q0]);
    const int slot = nbig_sub + g;
    if (slot >= cap_subs) {
      atomicOr(&dsc->err, MXE_SUBSYS);
      continue;
    }
    Subsystem& sub = subs[slot];  // built in place (no private copy)
    sub.m = 0;
    sub.np = 0;
    sub.jm = j;
    bool ok = true;
    for (int q = q0; q < q1 && ok; ++q) {
      int i = key_lo(S[q]);
      if (inbig[i]) {
        int r = uf_find(par, i);
        for (int c = 0; c < nbb && ok; ++c) {
          int64_t k = K[BB[c]];
          if (uf_find(par, key_hi(k)) != r) continue;
          ok = insert_sorted(sub.mem, sub.m, kBsMaxMembers - 1, key_hi(k)) &&
               insert_sorted(sub.mem, sub.m, kBsMaxMembers - 1, key_lo(k));
        }
      } else {
        ok = insert_sorted(sub.mem, sub.m, kBsMaxMembers - 1, i);
      }
    }
    const int nbm = sub.m;
    if (ok) {
      sub.mem[sub.m++] = j;
      sub.keep_from = nbm;
      // big-big pairs among the members, then the pairs naming j, both in (i, j) order
      for (int c = 0; c < nbb && ok; ++c) {
        int64_t k = K[BB[c]];
        int la = index_in(sub.mem, nbm, key_hi(k)), lb = index_in(sub.mem, nbm, key_lo(k));
        if (la < 0 || lb < 0) continue;
        if (sub.np >= kBsMaxPairs) { ok = false; break; }
        sub.pl[sub.np][0] = la;
        sub.pl[sub.np][1] = lb;
        ++sub.np;
      }
      for (int q = q0; q < q1 && ok; ++q) {
        if (sub.np >= kBsMaxPairs) { ok = false; break; }
        sub.pl[sub.np][0] = index_in(sub.mem, nbm, key_lo(S[q]));
        sub.pl[sub.np][1] = nbm;
        ++sub.np;
      }
    }
    if (!ok) {
      atomicOr(&dsc->err, MXE_SUBSYS);
      sub.m = 0;  // an empty subsystem keeps the table dense; the integrator skips it
      sub.np = 0;
      sub.keep_from = 0;
    }
  }
  __syncthreads();
  // 6. restore the union-find scratch
  for (int b = tid; b < nbb; b += T) {
    int64_t k = K[BB[b]];
    par[key_hi(k)] = key_hi(k);
    par[key_lo(k)] = key_lo(k);
    inbig[key_hi(k)] = 0;
    inbig[key_lo(k)] = 0;
  }
  if (tid == 0) dsc->n_sub = min(nbig_sub + ng, cap_subs);
}

// ---- single-wave general planner for short lists (np <= kPlanShort, any pairs)
// The same table as plan_general, with every list held in lanes: the sorted
// pairs (one per lane), the big-big pairs, the union-find over the bodies they
// name (node k in lane k, root = smallest body index as in plan_general), the
// members and pair list of the subsystem being built (lane k = entry k).  The
// sequential parts run as wave-uniform loops over register data, so no step
// waits on a memory round trip; each record is stored with one write per lane.
constexpr int kPlanShort = 32;

struct ShortPlanLds {
  int64_t a[64], b[64];  // sort input (padded to whole rounds) and output
};

__device__ __forceinline__ int lane_of(uint64_t m) { return m ? __builtin_ctzll(m) : -1; }

// members held one per lane (lane < m), ascending; insert b unless present
__device__ __forceinline__ bool wave_insert_sorted(int& memv, int& m, int cap, int b) {
  const int lane = threadIdx.x & 63;
  const bool in = lane < m;
  if (__builtin_amdgcn_ballot_w64(in && memv == b) != 0) return true;
  if (m >= cap) return false;
  const int pos = __popcll(__builtin_amdgcn_ballot_w64(in && memv < b));
  const int up = __shfl_up(memv, 1);
  if (lane == pos) memv = b;
  else if (lane > pos && lane <= m) memv = up;
  ++m;
  return true;
}

__device__ void plan_short(int nb, gmem<int32_t> gpairs, int np, gmem<Subsystem> subs,
                           int32_t cap_subs, DevScalars* __restrict__ dsc, int sort_only,
                           ShortPlanLds& L) {
  const int lane = threadIdx.x & 63;
  // 1. sort by (i, j)
  const int64_t key_in = lane < np ? make_key(gpairs[2 * lane], gpairs[2 * lane + 1]) : INT64_MAX;
  L.a[lane] = key_in;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  wave_rank_sort(L.a, L.b, np);
  const int64_t K = lane < np ? L.b[lane] : INT64_MAX;
  const int ki = key_hi(K), kj = key_lo(K);
  if (lane < np) {
    gpairs[2 * lane] = ki;
    gpairs[2 * lane + 1] = kj;
  }
  if (sort_only) return;
  const uint64_t lt = (1ull << lane) - 1ull;
  // 2. big-big pairs in (i, j) order (lane b = pair b); massless pairs keyed (j, i)
  const bool isbb = lane < np && kj < nb;
  const uint64_t bbm = __builtin_amdgcn_ballot_w64(isbb);
  const int nbb = __popcll(bbm);
  const bool isms = lane < np && !isbb;
  const uint64_t msm = __builtin_amdgcn_ballot_w64(isms);
  const int ns = __popcll(msm);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (isbb) L.a[__popcll(bbm & lt)] = K;
  if (isms) L.b[__popcll(msm & lt)] = make_key(kj, ki);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int bi = lane < nbb ? key_hi(L.a[lane]) : -1;
  const int bj = lane < nbb ? key_lo(L.a[lane]) : -1;
  // massless pairs sorted by (j, i)
  const int64_t skey = lane < ns ? L.b[lane] : INT64_MAX;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  L.a[lane] = skey;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  wave_rank_sort(L.a, L.b, ns);
  const int64_t sk = lane < ns ? L.b[lane] : INT64_MAX;
  const int sj = key_hi(sk), si = key_lo(sk);
  // 3. union-find over the bodies of the big-big pairs (node k = lane k)
  int nodeb = -1, nodep = lane;
  int nn = 0;
  for (int b = 0; b < nbb; ++b) {
    const int e[2] = {__builtin_amdgcn_readlane(bi, b), __builtin_amdgcn_readlane(bj, b)};
    int r[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      int k = lane_of(__builtin_amdgcn_ballot_w64(lane < nn && nodeb == e[t]));
      if (k < 0) {
        k = nn++;
        if (lane == k) nodeb = e[t];
      }
      int x = k;
      for (;;) {
        const int px = __builtin_amdgcn_readlane(nodep, x);
        if (px == x) break;
        x = px;
      }
      r[t] = x;
    }
    if (r[0] != r[1]) {
      const int b0 = __builtin_amdgcn_readlane(nodeb, r[0]);
      const int b1 = __builtin_amdgcn_readlane(nodeb, r[1]);
      if (b0 < b1) {
        if (lane == r[1]) nodep = r[0];
      } else {
        if (lane == r[0]) nodep = r[1];
      }
    }
  }
  // root node of every big-big pair and of every node (lane-parallel finds)
  int ncomp = lane;
  for (;;) {
    const int p = __shfl(nodep, ncomp);
    if (__builtin_amdgcn_ballot_w64(p != ncomp) == 0) break;
    ncomp = p;
  }
  int broot = -1;  // root node of big-big pair `lane`
  for (int k = 0; k < nn; ++k) {
    const int nbk = __builtin_amdgcn_readlane(nodeb, k), nck = __builtin_amdgcn_readlane(ncomp, k);
    if (lane < nbb && bi == nbk) broot = nck;
  }
  // 4. one subsystem per component, in order of its first pair
  int nsub = 0;
  uint64_t emitted = 0;
  for (int b = 0; b < nbb; ++b) {
    const int r = __builtin_amdgcn_readlane(broot, b);
    if ((emitted >> r) & 1ull) continue;
    emitted |= 1ull << r;
    if (nsub >= cap_subs) {
      if (lane == 0) atomicOr(&dsc->err, MXE_SUBSYS);
      continue;
    }
    const bool inc = lane < nbb && broot == r;
    const uint64_t incm = __builtin_amdgcn_ballot_w64(inc);
    int memv = 0, m = 0;
    bool ok = true;
    for (uint64_t q = incm; q != 0 && ok; q &= q - 1) {
      const int c = __builtin_ctzll(q);
      ok = wave_insert_sorted(memv, m, kBsMaxMembers, __builtin_amdgcn_readlane(bi, c)) &&
           wave_insert_sorted(memv, m, kBsMaxMembers, __builtin_amdgcn_readlane(bj, c));
    }
    const int npl = __popcll(incm);
    if (ok && npl > kBsMaxPairs) ok = false;
    if (!ok) {
      if (lane == 0) atomicOr(&dsc->err, MXE_SUBSYS);
      continue;
    }
    const auto R = subs + nsub;
    if (lane == 0) {
      R->m = m;
      R->keep_from = 0;
      R->np = npl;
      R->jm = 0;
    }
    if (lane < m) R->mem[lane] = memv;
    // member indices of each pair's ends (uniform loop over the members)
    int la = -1, lb = -1;
    for (int k = 0; k < m; ++k) {
      const int mk = __builtin_amdgcn_readlane(memv, k);
      if (bi == mk) la = k;
      if (bj == mk) lb = k;
    }
    if (inc) {
      const int slot = __popcll(incm & lt);
      R->pl[slot][0] = la;
      R->pl[slot][1] = lb;
    }
    ++nsub;
  }
  const int nbig_sub = nsub;
  // 5. one subsystem per flagged massless body, groups of equal j in order of j
  const int sjp = __shfl_up(sj, 1);
  const bool gstart = lane < ns && (lane == 0 || sjp != sj);
  const uint64_t gsm = __builtin_amdgcn_ballot_w64(gstart);
  const int ng = __popcll(gsm);
  int g = 0;
  for (uint64_t q = gsm; q != 0; q &= q - 1, ++g) {
    const int q0 = __builtin_ctzll(q);
    const uint64_t rest = q & (q - 1);
    const int q1 = rest ? __builtin_ctzll(rest) : ns;
    const int j = __builtin_amdgcn_readlane(sj, q0);
    const int slot = nbig_sub + g;
    if (slot >= cap_subs) {
      if (lane == 0) atomicOr(&dsc->err, MXE_SUBSYS);
      continue;
    }
    int memv = 0, m = 0;
    bool ok = true;
    for (int e = q0; e < q1 && ok; ++e) {
      const int i = __builtin_amdgcn_readlane(si, e);
      const int k = lane_of(__builtin_amdgcn_ballot_w64(lane < nn && nodeb == i));
      if (k >= 0) {
        const int r = __builtin_amdgcn_readlane(ncomp, k);
        const uint64_t incm = __builtin_amdgcn_ballot_w64(lane < nbb && broot == r);
        for (uint64_t c2 = incm; c2 != 0 && ok; c2 &= c2 - 1) {
          const int c = __builtin_ctzll(c2);
          ok = wave_insert_sorted(memv, m, kBsMaxMembers - 1, __builtin_amdgcn_readlane(bi, c)) &&
               wave_insert_sorted(memv, m, kBsMaxMembers - 1, __builtin_amdgcn_readlane(bj, c));
        }
      } else {
        ok = wave_insert_sorted(memv, m, kBsMaxMembers - 1, i);
      }
    }
    const auto R = subs + slot;
    int npl = 0;
    if (ok) {
      const int nbm = m;
      if (lane == nbm) memv = j;
      m = nbm + 1;
      // big-big pairs among the members, then the pairs naming j, both in (i, j) order
      int la = -1, lb = -1;
      for (int k = 0; k < nbm; ++k) {
        const int mk = __builtin_amdgcn_readlane(memv, k);
        if (bi == mk) la = k;
        if (bj == mk) lb = k;
      }
      const bool inbb = lane < nbb && la >= 0 && lb >= 0;
      const uint64_t inbbm = __builtin_amdgcn_ballot_w64(inbb);
      const int nbbp = __popcll(inbbm);
      npl = nbbp + (q1 - q0);
      if (npl > kBsMaxPairs) {
        ok = false;
      } else {
        if (inbb) {
          const int sl = __popcll(inbbm & lt);
          R->pl[sl][0] = la;
          R->pl[sl][1] = lb;
        }
        int li = -1;
        for (int k = 0; k < nbm; ++k)
          if (__builtin_amdgcn_readlane(memv, k) == si) li = k;
        if (lane >= q0 && lane < q1) {
          R->pl[nbbp + lane - q0][0] = li;
          R->pl[nbbp + lane - q0][1] = nbm;
        }
        if (lane < m) R->mem[lane] = memv;
        if (lane == 0) {
          R->m = m;
          R->keep_from = nbm;
          R->np = npl;
          R->jm = 0;
        }
      }
    }
    if (!ok && lane == 0) {
      atomicOr(&dsc->err, MXE_SUBSYS);
      R->m = 0;  // an empty subsystem keeps the table dense; the integrator skips it
      R->np = 0;
      R->keep_from = 0;
      R->jm = 0;
    }
  }
  if (lane == 0) dsc->n_sub = min(nbig_sub + ng, cap_subs);
}

// Sort of the flagged list by (i, j) and the subsystem plan, in one block.
//   - big-big pairs join big bodies (union-find, root = smallest index); every
//     component of two or more bodies is one subsystem (all members kept);
//   - each flagged massless body j is one subsystem: copies of the components
//     of the big bodies flagged with j, plus j (only j kept).
// gkeys: [2*cap] int64 global scratch; gidx: [2*cap] int32 global scratch.
// uf: [2*nb] with par[b] = b and inbig[b] = 0 at rest (restored on exit).
__device__ __forceinline__ void plan_block(int n, int nb, int32_t* __restrict__ pairs, int32_t cap,
                                           int64_t* __restrict__ gkeys,
                                           int32_t* __restrict__ gidx, int32_t* __restrict__ uf,
                                           Subsystem* __restrict__ subs, int32_t cap_subs,
                                           DevScalars* __restrict__ dsc, int sort_only) {
  const auto gpairs = gbl(pairs);
  const auto gsubs = gbl(subs);
  __shared__ int64_t lk[kPlanLds];
  __shared__ int64_t ls[kPlanLds];
  __shared__ int32_t lbb[kPlanLds];
  __shared__ int32_t lgs[kPlanLds];
  __shared__ int scan[kPlanThreads];
  __shared__ int s_nbig_sub;
  const int np = min(dsc->n_pairs[0], cap);
  if (threadIdx.x == 0) {
    dsc->n_pairs_last = dsc->n_pairs[0];
    if (!sort_only) dsc->pairs_flagged += (unsigned long long)dsc->n_pairs[0];
  }
  if (np == 0) {
    if (threadIdx.x == 0 && !sort_only) dsc->n_sub = 0;
    return;
  }
  // Short lists without big-big pairs (the common case): one wave sorts in
  // registers and writes each flagged massless body's subsystem directly; the
  // result is the same table as the general path below.
  {
    bool bb = false;
    if (np <= 256)
      for (int q = threadIdx.x; q < np; q += blockDim.x) bb |= gpairs[2 * q + 1] < nb;
    const bool any_bb = __syncthreads_or(bb);
    if (np <= 256 && !any_bb) {
      if (threadIdx.x >= 64) return;
      const int lane = threadIdx.x;
      int32_t* lj = reinterpret_cast<int32_t*>(lk);  // [256] j of the (j, i)-sorted list
      int32_t* li = lj + 256;                          // [256] i
      if (!sort_only && nb <= 64 && n > 0 && n < (1 << 26)) {
        // Only the grouping by massless body is needed here: one sort of 32-bit
        // keys (j, i).  The list in memory stays in append order; the host puts
        // it in (i, j) order when it is read.
        uint32_t* ka = reinterpret_cast<uint32_t*>(ls);
        uint32_t* kb = ka + 256;
        for (int e = lane; e < np; e += 64)
          ka[e] = ((uint32_t)gpairs[2 * e + 1] << 6) | (uint32_t)gpairs[2 * e];
        pad_keys(ka, np);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        wave_rank_sort(ka, kb, np);
        for (int e = lane; e < np; e += 64) {
          lj[e] = (int32_t)(kb[e] >> 6);
          li[e] = (int32_t)(kb[e] & 63u);
        }
      } else {
        for (int e = lane; e < np; e += 64) ls[e] = make_key(gpairs[2 * e], gpairs[2 * e + 1]);
        pad_keys(ls, np);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        wave_rank_sort(ls, lk, np);  // (i, j) order
        for (int e = lane; e < np; e += 64) {
          gpairs[2 * e] = key_hi(lk[e]);
          gpairs[2 * e + 1] = key_lo(lk[e]);
        }
        if (sort_only) return;
        // regroup by massless body j: keys (j, i)
        for (int e = lane; e < np; e += 64) lk[256 + e] = make_key(key_lo(lk[e]), key_hi(lk[e]));
        pad_keys(lk + 256, np);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        wave_rank_sort(lk + 256, ls, np);
        for (int e = lane; e < np; e += 64) {
          lj[e] = key_hi(ls[e]);
          li[e] = key_lo(ls[e]);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // group starts, numbered in list order
      int base = 0;
      for (int r = 0; r < (np + 63) / 64; ++r) {
        const int e = 64 * r + lane;
        const bool start = e < np && (e == 0 || lj[e] != lj[e - 1]);
        const uint64_t bal = __ballot(start);
        const int g = base + __popcll(bal & ((1ull << lane) - 1ull));
        base += __popcll(bal);
        if (!start) continue;
        int k = 1;
        while (e + k < np && lj[e + k] == lj[e]) ++k;
        const int j = lj[e];
        const auto S = gsubs + g;
        if (g >= cap_subs) {
          atomicOr(&dsc->err, MXE_SUBSYS);
          continue;
        }
        if (k + 1 > kBsMaxMembers || k > kBsMaxPairs) {
          atomicOr(&dsc->err, MXE_SUBSYS);
          S->m = 0;  // an empty subsystem keeps the table dense; the integrator skips it
          S->np = 0;
          S->keep_from = 0;
          S->jm = 0;
          continue;
        }
        S->m = k + 1;
        S->keep_from = k;
        S->np = k;
        S->jm = 0;
        for (int q = 0; q < k; ++q) {
          S->mem[q] = li[e + q];
          S->pl[q][0] = q;
          S->pl[q][1] = k;
        }
        S->mem[k] = j;
      }
      if (lane == 0) dsc->n_sub = min(base, cap_subs);
      return;
    }
  }
  if (np <= kPlanShort) {
    if (threadIdx.x >= 64) return;
    plan_short(nb, gpairs, np, gsubs, cap_subs, dsc, sort_only,
               *reinterpret_cast<ShortPlanLds*>(lk));
    return;
  }
  const bool small_list = np <= kPlanLds;
  int64_t* K = small_list ? lk : gkeys;
  int64_t* S = small_list ? ls : gkeys + cap;
  int32_t* BB = small_list ? lbb : gidx;
  int32_t* GS = small_list ? lgs : gidx + cap;
  plan_general(nb, gpairs, np, K, S, BB, GS, uf, subs, cap_subs, dsc, sort_only, scan, &s_nbig_sub,
               blockDim.x, true);
}

__global__ __launch_bounds__(kPlanThreads) void k_plan(
    int nb, int32_t* __restrict__ pairs, int32_t cap, int64_t* __restrict__ gkeys,
    int32_t* __restrict__ gidx, int32_t* __restrict__ uf, Subsystem* __restrict__ subs,
    int32_t cap_subs, DevScalars* __restrict__ dsc, int sort_only) {
  plan_block(0, nb, pairs, cap, gkeys, gidx, uf, subs, cap_subs, dsc, sort_only);
}

// ------------------------------------------------------------------ BS
constexpr int kM = kBsMaxMembers;
constexpr int kC = kBsColumns;

// 1 / ((n_k / n_{k-j})^2 - 1) for the substep counts n_k = 2 (k + 1): the
// Aitken-Neville weights of polynomial extrapolation in (H/n)^2.
__constant__ double kNevilleInv[kC][kC] = {
    {0, 0, 0, 0, 0, 0, 0, 0},
    {0, 1.0 / 3.0, 0, 0, 0, 0, 0, 0},
    {0, 1.0 / (9.0 / 4.0 - 1.0), 1.0 / 8.0, 0, 0, 0, 0, 0},
    {0, 1.0 / (16.0 / 9.0 - 1.0), 1.0 / (16.0 / 4.0 - 1.0), 1.0 / 15.0, 0, 0, 0, 0},
    {0, 1.0 / (25.0 / 16.0 - 1.0), 1.0 / (25.0 / 9.0 - 1.0), 1.0 / (25.0 / 4.0 - 1.0), 1.0 / 24.0,
     0, 0, 0},
    {0, 1.0 / (36.0 / 25.0 - 1.0), 1.0 / (36.0 / 16.0 - 1.0), 1.0 / (36.0 / 9.0 - 1.0),
     1.0 / (36.0 / 4.0 - 1.0), 1.0 / 35.0, 0, 0},
    {0, 1.0 / (49.0 / 36.0 - 1.0), 1.0 / (49.0 / 25.0 - 1.0), 1.0 / (49.0 / 16.0 - 1.0),
     1.0 / (49.0 / 9.0 - 1.0), 1.0 / (49.0 / 4.0 - 1.0), 1.0 / 48.0, 0},
    {0, 1.0 / (64.0 / 49.0 - 1.0), 1.0 / (64.0 / 36.0 - 1.0), 1.0 / (64.0 / 25.0 - 1.0),
     1.0 / (64.0 / 16.0 - 1.0), 1.0 / (64.0 / 9.0 - 1.0), 1.0 / (64.0 / 4.0 - 1.0), 1.0 / 63.0}};

// star (mu0) plus the complementary (1-K) part of every flagged pair; inverse
// cubes from the corrected hardware rsqrt
__device__ void bs_force(int m, int np, const int32_t (*pl)[2], const double* mum,
                         const double* rcm, double mu0, const double* xs, double* as) {
  for (int k = 0; k < m; ++k) {
    const double* p = xs + 3 * k;
    double r2 = fma(p[2], p[2], fma(p[1], p[1], p[0] * p[0]));
    double y = mxd::rsqrt_full(r2);
    double f = -mu0 * (y * y * y);
    as[3 * k] = f * p[0];
    as[3 * k + 1] = f * p[1];
    as[3 * k + 2] = f * p[2];
  }
  for (int q = 0; q < np; ++q) {
    int a = pl[q][0], b = pl[q][1];
    double d0 = xs[3 * b] - xs[3 * a];
    double d1 = xs[3 * b + 1] - xs[3 * a + 1];
    double d2 = xs[3 * b + 2] - xs[3 * a + 2];
    double s2 = fma(d2, d2, fma(d1, d1, d0 * d0));
    double rc = fmax(rcm[a], rcm[b]);
    double rc2 = rc * rc;
    double w = 0.0;
    if (s2 < rc2 && s2 > 0.0) {
      double y = mxd::rsqrt_full(s2);
      double y3 = y * y * y;
      if (s2 <= 0.01 * rc2) {
        w = y3;
      } else {
        double q1 = (s2 * y - 0.1 * rc) / (0.9 * rc);
        double q2 = q1 * q1, q3 = q1 * q2;
        double K = q3 * fma(q1, fma(q1, 6.0, -15.0), 10.0);
        w = y3 * (1.0 - K);
      }
    }
    double wa = mum[b] * w, wb = mum[a] * w;
    as[3 * a] = fma(wa, d0, as[3 * a]);
    as[3 * a + 1] = fma(wa, d1, as[3 * a + 1]);
    as[3 * a + 2] = fma(wa, d2, as[3 * a + 2]);
    as[3 * b] = fma(-wb, d0, as[3 * b]);
    as[3 * b + 1] = fma(-wb, d1, as[3 * b + 1]);
    as[3 * b + 2] = fma(-wb, d2, as[3 * b + 2]);
  }
}

// One Stoermer (velocity-Verlet) sequence of ns = 2 (col + 1) substeps over H
// from (xs, vs); end positions and velocities go to out[0..nn) and out[nn..2nn).
__device__ void stoermer_seq(int col, double H, int m, int np, const int32_t (*pl)[2],
                             const double* mum, const double* rcm, double mu0, const double* xs,
                             const double* vs, double* pos, double* d, double* acc, double* out) {
  const int nn = 3 * m;
  const int ns = 2 * (col + 1);
  const double dt = H / ns;
  for (int i = 0; i < nn; ++i) pos[i] = xs[i];
  bs_force(m, np, pl, mum, rcm, mu0, pos, acc);
  for (int i = 0; i < nn; ++i) {
    d[i] = dt * (vs[i] + 0.5 * dt * acc[i]);
    pos[i] += d[i];
  }
  for (int k = 1; k < ns; ++k) {
    bs_force(m, np, pl, mum, rcm, mu0, pos, acc);
    for (int i = 0; i < nn; ++i) {
      d[i] += dt * dt * acc[i];
      pos[i] += d[i];
    }
  }
  bs_force(m, np, pl, mum, rcm, mu0, pos, acc);
  for (int i = 0; i < nn; ++i) {
    out[i] = pos[i];
    out[nn + i] = d[i] / dt + 0.5 * dt * acc[i];
  }
}

constexpr int kRound = 4;

// Rows K0..K0+3 of the Aitken-Neville table for this lane's two elements (all
// indices compile-time, so the table stays in registers), with the per-row
// error max(dx^2 xscal, dv^2 vscal) of the lane.
template <int K0>
__device__ __forceinline__ void neville_round(int lane, int nn, int m, const double (*res)[6 * kM],
                                              const double* scal, double (&prev)[2][kC],
                                              double (&diag)[2][kC], double (&lerr)[kRound]) {
#pragma unroll
  for (int kk = 0; kk < kRound; ++kk) lerr[kk] = 0.0;
#pragma unroll
  for (int slot = 0; slot < 2; ++slot) {
    const int e = lane + 64 * slot;
    if (e >= 2 * nn) continue;
    const double sc = e < nn ? scal[e / 3] : scal[m + (e - nn) / 3];
#pragma unroll
    for (int kk = 0; kk < kRound; ++kk) {
      const int k = K0 + kk;
      double T[kC];
      T[0] = res[k][e];
#pragma unroll
      for (int jx = 1; jx < kC; ++jx)
        if (jx <= k) T[jx] = fma(T[jx - 1] - prev[slot][jx - 1], kNevilleInv[k][jx], T[jx - 1]);
#pragma unroll
      for (int jx = 0; jx < kC; ++jx)
        if (jx == k) diag[slot][jx] = T[jx];
      if (k >= 1) {
        double ex = T[k] - T[k - 1];
        lerr[kk] = fmax(lerr[kk], ex * ex * sc);
      }
#pragma unroll
      for (int jx = 0; jx < kC; ++jx)
        if (jx <= k) prev[slot][jx] = T[jx];
    }
  }
}

// Register-resident variant for subsystems of M <= 4 members: positions,
// increments and accelerations stay in VGPRs; the flagged pairs are a bit mask
// over the M (M-1) / 2 possible pairs, walked at compile time.  The pair weight
// is formed without branches (the lanes of a wave sit at different step sizes
// and would otherwise run every branch in turn): inside 0.1 rc the full y^3,
// in the changeover zone y^3 (1 - K) with q = (s - 0.1 rc) / (0.9 rc) taken as
// a product with the reciprocal of 0.9 rc, zero outside rc.
template <int M>
struct PairConst {
  double rc2[M * (M - 1) / 2 > 0 ? M * (M - 1) / 2 : 1];
  double rc01[M * (M - 1) / 2 > 0 ? M * (M - 1) / 2 : 1];   // 0.1 rc
  double inv09[M * (M - 1) / 2 > 0 ? M * (M - 1) / 2 : 1];  // 1 / (0.9 rc)
};

template <int M>
__device__ __forceinline__ void pair_consts(const double (&rc)[M], PairConst<M>& pc) {
  int bit = 0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
#pragma unroll
    for (int b = a + 1; b < M; ++b, ++bit) {
      const double rcp = fmax(rc[a], rc[b]);
      pc.rc2[bit] = rcp * rcp;
      pc.rc01[bit] = 0.1 * rcp;
      pc.inv09[bit] = 1.0 / (0.9 * rcp);
    }
  }
}

// LM: the last member is massless, so it exerts no force (its reaction terms
// are zero and are skipped: the other members' sums are unchanged bit for bit).
template <int M, bool LM = false>
__device__ __forceinline__ void force_reg(uint32_t pmask, const double (&mu)[M],
                                          const PairConst<M>& pc, double mu0,
                                          const double (&pos)[3 * M], double (&acc)[3 * M]) {
#pragma unroll
  for (int k = 0; k < M; ++k) {
    double r2 = fma(pos[3 * k + 2], pos[3 * k + 2],
                    fma(pos[3 * k + 1], pos[3 * k + 1], pos[3 * k] * pos[3 * k]));
    double y = mxd::rsqrt_full(r2);
    double f = -mu0 * (y * y * y);
    acc[3 * k] = f * pos[3 * k];
    acc[3 * k + 1] = f * pos[3 * k + 1];
    acc[3 * k + 2] = f * pos[3 * k + 2];
  }
  // every possible pair, unflagged ones with weight zero: one basic block, so
  // the independent chains of the members and pairs interleave
  int bit = 0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
#pragma unroll
    for (int b = a + 1; b < M; ++b, ++bit) {
      double d0 = pos[3 * b] - pos[3 * a];
      double d1 = pos[3 * b + 1] - pos[3 * a + 1];
      double d2 = pos[3 * b + 2] - pos[3 * a + 2];
      double s2 = fma(d2, d2, fma(d1, d1, d0 * d0));
      const double rc2 = pc.rc2[bit];
      double y = mxd::rsqrt_full(s2);
      double y3 = y * y * y;
      double q1 = (s2 * y - pc.rc01[bit]) * pc.inv09[bit];
      double q2 = q1 * q1, q3 = q1 * q2;
      double K = q3 * fma(q1, fma(q1, 6.0, -15.0), 10.0);
      double wz = s2 <= 0.01 * rc2 ? y3 : y3 * (1.0 - K);
      const bool on = ((pmask >> bit) & 1u) && s2 < rc2 && s2 > 0.0;
      double w = on ? wz : 0.0;
      const double wb = mu[a] * w;
      if (!(LM && b == M - 1)) {
        const double wa = mu[b] * w;
        acc[3 * a] = fma(wa, d0, acc[3 * a]);
        acc[3 * a + 1] = fma(wa, d1, acc[3 * a + 1]);
        acc[3 * a + 2] = fma(wa, d2, acc[3 * a + 2]);
      }
      acc[3 * b] = fma(-wb, d0, acc[3 * b]);
      acc[3 * b + 1] = fma(-wb, d1, acc[3 * b + 1]);
      acc[3 * b + 2] = fma(-wb, d2, acc[3 * b + 2]);
    }
  }
}

template <int M>
__device__ void stoermer_reg(int col, double H, uint32_t pmask, const double* mum,
                             const double* rcm, double mu0, const double* xs, const double* vs,
                             double* out) {
  constexpr int NN = 3 * M;
  double mu[M], rc[M], pos[NN], d[NN], acc[NN];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    mu[k] = mum[k];
    rc[k] = rcm[k];
  }
  PairConst<M> pc;
  pair_consts<M>(rc, pc);
#pragma unroll
  for (int i = 0; i < NN; ++i) pos[i] = xs[i];
  const int ns = 2 * (col + 1);
  const double dt = H / ns;
  force_reg<M>(pmask, mu, pc, mu0, pos, acc);
#pragma unroll
  for (int i = 0; i < NN; ++i) {
    d[i] = dt * (vs[i] + 0.5 * dt * acc[i]);
    pos[i] += d[i];
  }
  const double dt2 = dt * dt;
  for (int k = 1; k < ns; ++k) {
    force_reg<M>(pmask, mu, pc, mu0, pos, acc);
#pragma unroll
    for (int i = 0; i < NN; ++i) {
      d[i] = fma(dt2, acc[i], d[i]);
      pos[i] += d[i];
    }
  }
  force_reg<M>(pmask, mu, pc, mu0, pos, acc);
#pragma unroll
  for (int i = 0; i < NN; ++i) {
    out[i] = pos[i];
    out[NN + i] = d[i] / dt + 0.5 * dt * acc[i];
  }
}

// pair (a, b), a < b, of an M-member subsystem -> bit of the pair mask
__device__ __forceinline__ int pair_bit(int a, int b, int m) {
  return a * (2 * m - a - 1) / 2 + (b - a - 1);
}

__device__ __forceinline__ void run_column(int col, double H, int m, int np,
                                           const int32_t (*pl)[2], uint32_t pmask,
                                           const double* mum, const double* rcm, double mu0,
                                           const double* xs, const double* vs, double* wk0,
                                           double* wk1, double* wk2, double* out) {
  switch (m) {
    case 2: stoermer_reg<2>(col, H, pmask, mum, rcm, mu0, xs, vs, out); break;
    case 3: stoermer_reg<3>(col, H, pmask, mum, rcm, mu0, xs, vs, out); break;
    case 4: stoermer_reg<4>(col, H, pmask, mum, rcm, mu0, xs, vs, out); break;
    default: stoermer_seq(col, H, m, np, pl, mum, rcm, mu0, xs, vs, wk0, wk1, wk2, out);
  }
}

// Rows K0 .. K1-1 of the Aitken-Neville tables of one candidate group: lane j
// of the group holds elements j, j + 8, ...; prev/dg carry the previous row and
// the diagonal across calls, lerr[k] the lane's error of row k.
template <int M, int K0, int K1>
__device__ __forceinline__ void neville_rows(int cand, int j, const double* scal,
                                             const double (*resS)[kC][6 * 4],
                                             double (&prev)[(6 * M + 7) / 8][kC],
                                             double (&dg)[(6 * M + 7) / 8][kC], double (&lerr)[kC]) {
  constexpr int NN = 3 * M, E = 2 * NN, EPL = (E + 7) / 8;
#pragma unroll
  for (int s = 0; s < EPL; ++s) {
    const int e = j + 8 * s;
    if (e >= E) continue;
    const double sc = e < NN ? scal[e / 3] : scal[M + (e - NN) / 3];
#pragma unroll
    for (int k = K0; k < K1; ++k) {
      double T[kC];
      T[0] = resS[cand][k][e];
#pragma unroll
      for (int jx = 1; jx < kC; ++jx)
        if (jx <= k) T[jx] = fma(T[jx - 1] - prev[s][jx - 1], kNevilleInv[k][jx], T[jx - 1]);
      dg[s][k] = T[k];
      if (k >= 1) {
        const double ex = T[k] - T[k - 1];
        lerr[k] = fmax(lerr[k], ex * ex * sc);
      }
#pragma unroll
      for (int jx = 0; jx < kC; ++jx)
        if (jx <= k) prev[s][jx] = T[jx];
    }
  }
}

// Lane exchange within rows of the wave by DPP (VALU moves, no LDS round trip):
// quad_perm [1,0,3,2] (0xB1) and [2,3,0,1] (0x4E) swap within quads, row_half_mirror
// (0x141) maps lane i of each group of eight to lane 7 - i.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// maximum over the 8 lanes of each group (every lane receives it)
__device__ __forceinline__ double group8_max(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  return fmax(v, dpp_f64<0x141>(v));
}

// first row k in [K0, K1) whose error, reduced over the 8 lanes of the group,
// is within tolerance (-1 if none)
template <int K0, int K1>
__device__ __forceinline__ int first_ok(const double (&lerr)[kC], double tol2) {
  int acc = -1;
#pragma unroll
  for (int k = K0; k < K1; ++k) {
    const double v = group8_max(lerr[k]);
    if (acc < 0 && k >= 1 && v <= tol2) acc = k;
  }
  return acc;
}

// Subsystems of M <= 4 members: each round evaluates eight step sizes at once,
// H, H/2, ..., H/128 (lanes 8c .. 8c + 7 run the eight substep sequences of
// step size H / 2^c), and takes the largest one the sequential control would
// accept: candidate c is the step the sequential integrator tries after c
// consecutive failures of the larger ones, from the same state with the same
// scales, so the accepted steps, their columns and the results are those of
// the sequential loop, bit for bit, while a run of failures costs one round.
// The sequences stop after 8 and after 12 substeps for a look at columns 0..3
// and 4..5: when step size H is accepted there (the usual case) the longer
// sequences are not finished.  Returns the number of accepted steps, or -1
// when more than 30 consecutive failures occurred.
template <int M, bool LM>
__device__ __forceinline__ int bs_small(int lane, int b, double h, double tol2, uint32_t pmask, int np,
                        const double* mum, const double* rcm, double mu0, double* xs,
                        double* vs, double* scal, double (*resS)[kC][6 * 4],
                        const SysDesc& D, DevScalars* __restrict__ dsc) {
  constexpr int NN = 3 * M, E = 2 * NN;
  constexpr int EPL = (E + 7) / 8;  // table elements per lane of a candidate group
  const int cand = lane >> 3, j = lane & 7;
  double mu[M], rc[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    mu[k] = mum[k];
    rc[k] = rcm[k];
  }
  PairConst<M> pc;
  pair_consts<M>(rc, pc);
  // model count per sequential attempt: sequences of columns 0..3, 0..5 (the
  // two looks) or 0..7, 3 per extrapolation-table entry (FMA = 2)
  unsigned long long f_look0 = 0, f_look1 = 0, f_look2 = 0;
  for (int c = 0; c < kC; ++c) {
    const unsigned long long fc = (unsigned long long)(2 * (c + 1) + 1) * (24 * M + 25 * np) +
                                  (unsigned long long)3 * c * 6 * M;
    f_look2 += fc;
    if (c < 6) f_look1 += fc;
    if (c < 4) f_look0 += fc;
  }
  double done = 0.0, H = h;
  int fails = 0, nsched = 0;
  while (fabs(h - done) > 1e-14 * fabs(h)) {
    const double rem = h - done;
    if (fabs(H) > fabs(rem)) H = rem;
    if (lane < M) {
      const double* p = xs + 3 * lane;
      const double* q = vs + 3 * lane;
      scal[lane] = 1.0 / (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
      scal[M + lane] = 1.0 / (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    }
    // H / 2^cand: repeated halving is exact, so is the scaling by 2^-cand
    const double Hc = H * __longlong_as_double((long long)(1023 - cand) << 52);
    // Stoermer sequence of n = 2 (j + 1) substeps (the same operations as
    // stoermer_reg up to the velocity, formed with the reciprocal of the
    // substep), split after substeps 8 and 12
    const int ns = 2 * (j + 1);
    const double dt = Hc / ns, dt2 = dt * dt, idt = 1.0 / dt, hdt = 0.5 * dt;
    double pos[NN], d[NN], acc[NN];
#pragma unroll
    for (int i = 0; i < NN; ++i) pos[i] = xs[i];
    force_reg<M, LM>(pmask, mu, pc, mu0, pos, acc);
#pragma unroll
    for (int i = 0; i < NN; ++i) {
      d[i] = dt * (vs[i] + hdt * acc[i]);
      pos[i] += d[i];
    }
    // substeps k0 .. min(ns, k1) - 1, then the column's entry when it ends by k1
    auto advance = [&](int k0, int k1) {
      const int ke = ns < k1 ? ns : k1;
      for (int k = k0; k < ke; ++k) {
        force_reg<M, LM>(pmask, mu, pc, mu0, pos, acc);
#pragma unroll
        for (int i = 0; i < NN; ++i) {
          d[i] = fma(dt2, acc[i], d[i]);
          pos[i] += d[i];
        }
      }
      if (ns > k0 && ns <= k1) {
        force_reg<M, LM>(pmask, mu, pc, mu0, pos, acc);
#pragma unroll
        for (int i = 0; i < NN; ++i) {
          resS[cand][j][i] = pos[i];
          resS[cand][j][NN + i] = fma(d[i], idt, hdt * acc[i]);
        }
      }
    };
    advance(1, 8);
    __syncthreads();
    double lerr[kC], prev[EPL][kC], dg[EPL][kC];
#pragma unroll
    for (int k = 0; k < kC; ++k) lerr[k] = 0.0;
#pragma unroll
    for (int s = 0; s < EPL; ++s)
#pragma unroll
      for (int k = 0; k < kC; ++k) prev[s][k] = dg[s][k] = 0.0;
    neville_rows<M, 0, 4>(cand, j, scal, resS, prev, dg, lerr);
    int okc = first_ok<0, 4>(lerr, tol2);
    int look = 0;  // 0, 1: accepted by candidate 0 at the first or second look
    int chosen = -1, accepted = -1;
    bool failed = false;
    if ((__builtin_amdgcn_ballot_w64(lane == 0 && okc >= 0) & 1ull) != 0) {
      chosen = 0;
      accepted = __shfl(okc, 0);
    } else {
      advance(8, 12);
      __syncthreads();
      neville_rows<M, 4, 6>(cand, j, scal, resS, prev, dg, lerr);
      const int ok2 = first_ok<4, 6>(lerr, tol2);  // all lanes: the reduction crosses lanes
      if (okc < 0) okc = ok2;
      look = 1;
      if ((__builtin_amdgcn_ballot_w64(lane == 0 && okc >= 0) & 1ull) != 0) {
        chosen = 0;
        accepted = __shfl(okc, 0);
      } else {
        advance(12, 16);
        __syncthreads();
        neville_rows<M, 6, kC>(cand, j, scal, resS, prev, dg, lerr);
        const int ok3 = first_ok<6, kC>(lerr, tol2);
        if (okc < 0) okc = ok3;
        look = 2;
        // the sequential control: candidates in order, failures counted
        const uint64_t okm = __builtin_amdgcn_ballot_w64(j == 0 && okc >= 0);
        for (int c = 0; c < 8; ++c) {
          if ((okm >> (8 * c)) & 1ull) {
            chosen = c;
            break;
          }
          if (++fails > 30) {
            failed = true;
            break;
          }
        }
        if (chosen >= 0) accepted = __shfl(okc, 8 * chosen);
      }
    }
    if (lane == 0) {
      const unsigned long long f =
          look == 0 ? f_look0
          : look == 1 ? f_look1
                      : f_look2 * (unsigned long long)(chosen >= 0 ? chosen + 1 : 8);
      atomicAdd(&dsc->bs_flop, f);
    }
    __syncthreads();
    if (failed) return -1;
    if (chosen < 0) {
      H = H * 0.00390625;  // eight halvings
      continue;
    }
    if (cand == chosen) {
#pragma unroll
      for (int s = 0; s < EPL; ++s) {
        const int e = j + 8 * s;
        if (e >= E) continue;
        double val = dg[s][1];
#pragma unroll
        for (int k = 2; k < kC; ++k)
          if (k == accepted) val = dg[s][k];
        if (e < NN) xs[e] = val;
        else vs[e - NN] = val;
      }
    }
    const double Hs = H * __longlong_as_double((long long)(1023 - chosen) << 52);
    if (D.bs_sched && lane == 0) {
      if (nsched < kBsMaxSched) {
        D.bs_sched[((size_t)b * kBsMaxSched + nsched) * 2] = Hs;
        D.bs_sched[((size_t)b * kBsMaxSched + nsched) * 2 + 1] = (double)accepted;
      } else {
        atomicOr(&dsc->err, MXE_ADJOINT);
      }
    }
    ++nsched;
    done += Hs;
    fails = 0;
    H = accepted <= 4 ? 2.0 * Hs : Hs;
    __syncthreads();
  }
  return nsched;
}

// Columns are evaluated in two rounds (n = 2..8, then n = 10..16, four lanes
// each): most steps are accepted in the first round, and the table rows do not
// depend on later rows, so the accepted column is the one a sequential
// integrator would stop at.
// In-kernel plan (plan != 0): the blocks of a system plan their subsystems
// themselves, so the step needs no planning launch.  In systems of at most 64
// massive bodies a list of at most 256 pairs none of which joins two massive
// bodies (the common case) is planned by every block at once: one wave
// rank-sorts the 32-bit keys (j, i) in LDS and numbers the groups of equal j,
// which is the table the planning kernel builds (one subsystem per flagged
// massless body in order of j, its partners in order of i).  Block 0 also
// writes that table and the list counters for the readers after the step.  Any
// other list (and every list of a system with more massive bodies) takes the
// general plan in block 0 -- the single-wave planner for short lists -- while
// the other blocks of the system wait for its flag; the wait is bounded, and an
// expired wait latches an error.  The step's closing kernel clears the flag.
struct FastPlan {
  uint32_t ka[256], kb[256];  // keys (j << 6) | i in append order, then sorted
  int32_t gs[257];            // first sorted entry of each group, then the list length
};
constexpr int kPlanWaitMax = 1 << 22;  // polls of the plan flag (each after a short sleep)

// Joint launches: step q closed and step q + 1 opened for massless body j (the
// joined step kernel's operations) by the integrator's whole wave, with the
// boundary prepared for phase par (jsrc, jbst, jbrc, and jsc = J, vpre, Ppre,
// Ppost, in LDS), from its state after the integrator (xj, vj in LDS) or, when
// its subsystem was not integrated, after the drift (null: read from x, u); jr:
// its radius and density (LDS), or null (read here).  Lane s takes the gravity
// terms and the encounter test of massive body s; the terms are added in order
// of s and everything else runs on the same values in every lane, so each
// quantity is the per-body code's (close_body, advance_body, flag_body), bit
// for bit, with a shorter chain.  Step q + 1's pairs go to phase nx.
__device__ __forceinline__ void joint_member(const SysDesc& D, int j, const double* xj,
                                             const double* vj, int par, int nx,
                                             const KickSource* jsrc,
                                             const double (*jbst)[kSmallBig], const double* jbrc,
                                             const double* jsc, const double* jr) {
  const int n = D.n, nb = D.nb;
  if (j < nb || j >= n) return;  // wave-uniform
  const int lane = threadIdx.x & 63;
  const double h = D.h, hh = 0.5 * D.h, mu0 = D.mu0;
  const double rct = 0.0;  // a massless body has no changeover radius of its own
  double p[3], v[3], a[3], q[3], w[3], J[3], vpre[3], Ppre[3], Ppost[3];
  for (int c = 0; c < 3; ++c) {
    p[c] = xj ? xj[c] : gbl(D.x)[(size_t)c * n + j];
    v[c] = vj ? vj[c] : gbl(D.u)[(size_t)c * n + j];
    J[c] = jsc[c];
    vpre[c] = jsc[3 + c];
    Ppre[c] = jsc[6 + c];
    Ppost[c] = jsc[9 + c];
  }
  const double rp = !D.gas_on ? 0.0 : jr ? jr[0] : gbl(D.r_p)[j - nb];
  const double rhop = !D.gas_on ? 0.0 : jr ? jr[1] : gbl(D.rho_p)[j - nb];
  // step q closed: jump, gravity, drag, half kick (the gas where the body is
  // closed is also where it is opened)
  const double px = p[0] + J[0], py = p[1] + J[1], pz = p[2] + J[2];
  mxd::GasSite site;
  {
    const double rc2t = rct * rct;
    double k15, k1875;
    mxd::vgpr_constants(k15, k1875);
    double wgt = 0.0, dx = 0.0, dy = 0.0, dz = 0.0;
    if (lane < nb) {
      const KickSource S = jsrc[lane];
      dx = S.x - px;
      dy = S.y - py;
      dz = S.z - pz;
      double s2 = fma(dz, dz, fma(dy, dy, dx * dx));
      double rc2 = fmax(S.rc2, rc2t);
      wgt = mxd::fast_weight(S.mu, s2, k15, k1875);
      if (s2 < rc2) wgt = S.mu * mxd::changeover_weight_slow(s2, fmax(S.rc, rct), rc2);
    }
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int s = 0; s < nb; ++s) {
      const double ws = __shfl(wgt, s);
      a0 = fma(ws, __shfl(dx, s), a0);
      a1 = fma(ws, __shfl(dy, s), a1);
      a2 = fma(ws, __shfl(dz, s), a2);
    }
    double adx = 0.0, ady = 0.0, adz = 0.0;
    if (D.gas_on) {
      site = mxd::gas_site(D.dc, px, py);
      mxd::gas_drag_at(D.dc, site, v[0] + vpre[0], v[1] + vpre[1], v[2] + vpre[2], rp, rhop, adx,
                       ady, adz);
    }
    v[0] += hh * (a0 + adx);
    v[1] += hh * (a1 + ady);
    v[2] += hh * (a2 + adz);
    p[0] = px;
    p[1] = py;
    p[2] = pz;
    a[0] = a0;
    a[1] = a1;
    a[2] = a2;
  }
  const bool fin = isfinite(v[0] + v[1] + v[2] + p[0] + p[1] + p[2]);
  // step q + 1 opened: drag, half kick, jump, drift
  const bool conv = mxs::advance_body(j, nb, mu0, h, D.dc, D.gas_on, rp, rhop, Ppre, Ppost, p, v,
                                      a, q, w, &site);
  // encounter test of step q + 1 against massive body `lane`
  bool hit = false;
  if (lane < nb) {
    const int i = lane;
    const double k427 = (4.0 / 27.0) * fabs(h);
    double r0[3], w0[3], w1[3], dd[3];
    for (int c = 0; c < 3; ++c) {
      r0[c] = p[c] - jbst[c][i];
      w0[c] = v[c] - jbst[3 + c][i];
      w1[c] = w[c] - jbst[9 + c][i];
      dd[c] = (q[c] - p[c]) - (jbst[6 + c][i] - jbst[c][i]);
    }
    double m0 = fma(r0[2], r0[2], fma(r0[1], r0[1], r0[0] * r0[0]));
    double nd = fmax(fmax(fabs(dd[0]), fabs(dd[1])), fabs(dd[2]));
    double nw = fmax(fmax(fabs(w0[0]), fabs(w0[1])), fabs(w0[2])) +
                fmax(fmax(fabs(w1[0]), fabs(w1[1])), fabs(w1[2]));
    double rc = fmax(jbrc[i], rct);
    double bound = rc + 1.7320508075688773 * fma(k427, nw, nd) * (1.0 + 1e-12);
    if (m0 <= bound * bound * (1.0 + 1e-12)) {
      double r1[3];
      for (int c = 0; c < 3; ++c) r1[c] = q[c] - jbst[6 + c][i];
      double dmin = mxd::hermite_dmin2(r0[0], r0[1], r0[2], w0[0], w0[1], w0[2], r1[0], r1[1],
                                       r1[2], w1[0], w1[1], w1[2], h);
      hit = dmin <= rc * rc;
    }
  }
  const uint64_t hits = __ballot(hit);
  if (lane == 0) {
    if (!fin) atomicOr(&D.dsc->err, MXE_NONFINITE);
    if (!conv) atomicOr(&D.dsc->err, MXE_NOCONV);
    for (int c = 0; c < 3; ++c) {
      gbl(D.x)[(size_t)c * n + j] = q[c];
      gbl(D.u)[(size_t)c * n + j] = w[c];
    }
    // the body's pairs appended together, in increasing i (as flag_body), and
    // its subsystem record; both slots are taken before either is written
    uint64_t hmask = hits;
    if (hmask != 0) {
      const auto list = gbl(D.pairs) + (size_t)nx * 2 * D.cap_pairs;
      int idx = atomicAdd(pair_counter(D.dsc, nx), __popcll(hmask));
      const int ridx = atomicAdd(&D.dsc->n_jsub[nx], 1);
      if (ridx < D.cap_subs) {
        JointSub* R = D.jsub + (size_t)nx * D.cap_subs + ridx;
        R->mask = hits;
        R->j = j;
        R->pad = 0;
        for (int c = 0; c < 3; ++c) {
          R->x[c] = p[c];
          R->v[c] = v[c];
        }
        R->rp = rp;
        R->rhop = rhop;
      } else {
        atomicOr(&D.dsc->err, MXE_SUBSYS);
      }
      for (; hmask != 0; hmask &= hmask - 1, ++idx) {
        if (idx < D.cap_pairs) {
          list[2 * idx] = __builtin_ctzll(hmask);
          list[2 * idx + 1] = j;
        } else {
          atomicOr(&D.dsc->err, MXE_PAIRS);
        }
      }
    }
    if (hits != 0 || D.keep_x0) {
      for (int c = 0; c < 3; ++c) {
        gbl(D.x0)[(size_t)c * n + j] = p[c];
        gbl(D.u0)[(size_t)c * n + j] = v[c];
      }
    }
  }
}

// One block (one wave) of a system's encounter integrator: block bx of nbx.
// par: the step phase (append counter, plan flag, bigmid and BigNext copies),
// lst: the flagged list read, clr: the append counter cleared for the next step
// (-1: none).  kJoint: the integrator runs inside a joint launch beside the
// closing of step q and the opening of step q + 1 (phase nx); the massive
// members start from bigpre[par], and with jfast (bn_valid[par]: the boundary of
// step q was prepared, no flagged pair joins two massive bodies, so every
// subsystem is one massless body and the massive bodies it met, the massless
// body last) the subsystems are the records the flagging launch appended (one
// per flagged massless body, with its pre-drift state), and the wave closes and
// opens its massless member itself with the prepared boundary (jsrc, jbst, jbrc,
// jsc: LDS of the launch; jr: LDS for the member's radius and density, read with
// the subsystem's state).  Without jfast the list is planned as in k_bs and left
// in append order.  Returns jfast.
template <bool kJoint>
__device__ __forceinline__ bool bs_body(const SysDesc& D, const int bx, const int nbx, int plan,
                                        int par, int nx, int lst, int clr, KickSource* jsrc,
                                        double (*jbst)[kSmallBig], double* jbrc, double* jsc,
                                        double* jr) {
  const int n = D.n, nb = D.nb;
  const double mu0 = D.mu0, h = D.h, tol = D.bs_tol;
  const auto x0s = gbl(D.x0);
  const auto u0s = gbl(D.u0);
  const auto x = gbl(D.x);
  const auto u = gbl(D.u);
  const auto mu = gbl(D.mu);
  const auto rcrit = gbl(D.rcrit);
  const auto subs = gbl(D.subs);
  DevScalars* __restrict__ dsc = D.dsc;
  const auto bigmid = gbl(D.bigmid) + (size_t)par * 6 * nb;
  if (nb == 0) return false;
  // joint launches: whether the boundary was prepared
  const bool jfast = kJoint && dsc->bn_valid[par] != 0;
  __shared__ Subsystem S;
  __shared__ double xs[3 * kM], vs[3 * kM], mum[kM], rcm[kM], scal[2 * kM];
  // the tables of larger subsystems and the speculative rounds of subsystems of
  // at most four members (never both for one subsystem), the general planner's
  // scan (before any integration) and the boundary a block without subsystems
  // prepares share their LDS
  union BsTables {
    struct {
      double res[kC][6 * kM];
      double wk[kC][3][3 * kM];
    } big;
    double resS[8][kC][6 * 4];
    int scan[64];
    struct {
      double sh[8];
      KickSource src[kSmallBig];
      double bst[12][kSmallBig];
      double brc[kSmallBig];
    } prep;
  };
  __shared__ BsTables U;
  auto& res = U.big.res;
  auto& wk = U.big.wk;
  auto& resS = U.resS;
  __shared__ FastPlan F;
  __shared__ int s_nbig, s_nsub;
  int* s_scan = U.scan;
  // joint launches: the massive bodies' pre-drift state [6][nb], masses [nb] and
  // changeover radii [nb]
  __shared__ double jstage[kJoint ? 8 * kSmallBig : 1];
  const int lane = threadIdx.x;
  const double tol2 = tol * tol;
  int nsub = 0;
  bool fast = false;
  bool bigs_kept = true;  // false: no subsystem of this step changes a massive body
  // the block's first record (joint launches)
  uint64_t r0mask = 0;
  int r0j = 0;
  double r0x[3] = {0.0, 0.0, 0.0}, r0v[3] = {0.0, 0.0, 0.0}, r0rp = 0.0, r0rh = 0.0;
  // joint launches: requested at once, before the mode is known (every address is
  // valid either way): the counts, the block's first record (used only if it
  // exists), the massive bodies' state, masses and radii, and the prepared
  // boundary
  int nrec = 0, n_pairs = 0;
  double sv[kJoint ? 6 : 1], bsrc[kJoint ? 8 : 1], bbst[kJoint ? 12 : 1];
  double muv = 0.0, rcv = 0.0, bbrc = 0.0, bsc = 0.0;
  if constexpr (kJoint) {
    const BigNext* N = D.bignext + par;
    const auto bpre = gbl(D.bigpre) + (size_t)par * 6 * nb;
    const JointSub* R0 = D.jsub + (size_t)par * D.cap_subs + bx;
    nrec = dsc->n_jsub[par];
    n_pairs = *pair_counter(dsc, par);
    r0mask = R0->mask;
    r0j = R0->j;
    for (int c = 0; c < 3; ++c) {
      r0x[c] = R0->x[c];
      r0v[c] = R0->v[c];
    }
    r0rp = R0->rp;
    r0rh = R0->rhop;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      const int e = lane + 64 * r;
      sv[r] = e < 6 * nb ? bpre[e] : 0.0;
    }
    muv = lane < nb ? mu[lane] : 0.0;
    rcv = lane < nb ? rcrit[lane] : 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = lane + 64 * r;
      bsrc[r] = e < 8 * nb ? reinterpret_cast<const double*>(N->src)[e] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 12; ++r) bbst[r] = lane < nb ? N->bst[r][lane] : 0.0;
    bbrc = lane < nb ? N->brc[lane] : 0.0;
    bsc = lane < 12 ? reinterpret_cast<const double*>(N)[3 + lane] : 0.0;
  }
  if (!plan) {
    nsub = dsc->n_sub;
  } else if (kJoint && jfast) {
    // one subsystem per record appended by the launch that flagged the step's
    // pairs (the massless body, its massive partners, its pre-drift state); the
    // subsystem table is not written (only the adjoint reads it, and it never
    // runs joint launches)
    nsub = min(nrec, D.cap_subs);
    if (bx == 0 && lane == 0) {
      dsc->n_pairs_last = n_pairs;
      dsc->pairs_flagged += (unsigned long long)n_pairs;
      dsc->n_sub = nsub;
    }
    if (bx >= nsub) return jfast;
    bigs_kept = false;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      const int e = lane + 64 * r;
      if (e < 6 * nb) jstage[e] = sv[r];
    }
    if (lane < nb) {
      jstage[6 * nb + lane] = muv;
      jstage[7 * nb + lane] = rcv;
    }
    // the prepared boundary: the massless members are closed and opened with it
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = lane + 64 * r;
      if (e < 8 * nb) reinterpret_cast<double*>(jsrc)[e] = bsrc[r];
    }
#pragma unroll
    for (int r = 0; r < 12; ++r)
      if (lane < nb) jbst[r][lane] = bbst[r];
    if (lane < nb) jbrc[lane] = bbrc;
    if (lane < 12) jsc[lane] = bsc;
  } else {
    const bool b0 = bx == 0;
    const int cap_pairs = D.cap_pairs, cap_subs = D.cap_subs;
    const bool ordered = D.bs_sched != nullptr;
    const auto gpairs = gbl(D.pairs) + (size_t)lst * 2 * cap_pairs;
    // the first 256 entries of the list are requested with its length (entries
    // past the length are not used)
    int32_t pre_i[4], pre_j[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = 64 * r + lane;
      pre_i[r] = e < cap_pairs ? gpairs[2 * e] : 0;
      pre_j[r] = e < cap_pairs ? gpairs[2 * e + 1] : 0;
    }
    const int n_pairs = *pair_counter(dsc, par);
    // the next step's append counter when the closing and opening kernels of
    // two steps are joined; nothing reads or appends to it while this kernel runs
    if (clr >= 0 && b0 && lane == 0) *pair_counter(dsc, clr) = 0;
    const int np = min(n_pairs, cap_pairs);
    if (b0 && lane == 0) {
      dsc->n_pairs_last = n_pairs;
      dsc->pairs_flagged += (unsigned long long)n_pairs;
      if (np == 0) dsc->n_sub = 0;
    }
    // a system never has more subsystems than flagged pairs: blocks past the
    // pair count have nothing to integrate (the last block may still prepare
    // the next step boundary's massive bodies)
    if (bx >= np && (kJoint || bx != nbx - 1)) return jfast;
    bigs_kept = np > 0;
    if (np > 0) {
      fast = np <= 256 && nb <= 64 && n < (1 << 26);
      if (fast) {
        bool bb = false;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = 64 * r + lane;
          if (e < np) {
            bb |= pre_j[r] < nb;
            F.ka[e] = ((uint32_t)pre_j[r] << 6) | (uint32_t)pre_i[r];
          }
        }
        fast = __builtin_amdgcn_ballot_w64(bb) == 0;
      }
      if (fast) {
        bigs_kept = false;  // massless subsystems keep only their massless member
        // The fused step appends each body's pairs as one run in increasing i, so
        // the runs of equal j are the subsystems.  Their numbering only decides
        // which block integrates which subsystem, except for the tape the adjoint
        // records (bs_sched set): that needs the table in order of j, so the list
        // is sorted first.
        if (ordered) {
          pad_keys(F.ka, np);
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          wave_rank_sort(F.ka, F.kb, np);
        } else {
          for (int e = lane; e < np; e += 64) F.kb[e] = F.ka[e];
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
        }
        // group starts, numbered in list order
        int base = 0;
        for (int r = 0; r < (np + 63) / 64; ++r) {
          const int e = 64 * r + lane;
          const bool start = e < np && (e == 0 || (F.kb[e] >> 6) != (F.kb[e - 1] >> 6));
          const uint64_t bal = __ballot(start);
          const int g = base + __popcll(bal & ((1ull << lane) - 1ull));
          base += __popcll(bal);
          if (start) F.gs[g] = e;
        }
        if (lane == 0) F.gs[base] = np;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        nsub = min(base, cap_subs);
        if (b0) {
          // the table for the readers after the step (same records as the
          // planning kernel writes)
          for (int g = lane; g < base; g += 64) {
            if (g >= cap_subs) {
              atomicOr(&dsc->err, MXE_SUBSYS);
              continue;
            }
            const int e0 = F.gs[g], k = F.gs[g + 1] - e0;
            const auto R = subs + g;
            R->jm = 0;
            if (k + 1 > kBsMaxMembers || k > kBsMaxPairs) {
              atomicOr(&dsc->err, MXE_SUBSYS);
              R->m = 0;
              R->np = 0;
              R->keep_from = 0;
              continue;
            }
            R->m = k + 1;
            R->keep_from = k;
            R->np = k;
            for (int q = 0; q < k; ++q) {
              R->mem[q] = (int32_t)(F.kb[e0 + q] & 63u);
              R->pl[q][0] = q;
              R->pl[q][1] = k;
            }
            R->mem[k] = (int32_t)(F.kb[e0] >> 6);
          }
          if (lane == 0) dsc->n_sub = nsub;
        }
      } else {
        if (b0) {
          static_assert(sizeof(FastPlan) >= sizeof(ShortPlanLds), "short plan scratch");
          if (np <= kPlanShort)
            plan_short(nb, gpairs, np, subs, cap_subs, dsc, 0,
                       *reinterpret_cast<ShortPlanLds*>(&F));
          else
            plan_general(nb, gpairs, np, D.keys, D.keys + cap_pairs, D.plan_idx,
                         D.plan_idx + cap_pairs, D.uf, D.subs, cap_subs, dsc, 0, s_scan, &s_nbig,
                         64, !kJoint);
          __syncthreads();
          if (lane == 0) {
            s_nsub = dsc->n_sub;
            __hip_atomic_store(&dsc->plan_ready[par], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          }
        } else if (lane == 0) {
          // relaxed polls (an acquiring load would invalidate this CU's caches on
          // every poll), then one acquire fence once the flag is seen
          int it = 0;
          while (__hip_atomic_load(&dsc->plan_ready[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            __builtin_amdgcn_s_sleep(8);
            if (++it >= kPlanWaitMax) break;
          }
          if (it >= kPlanWaitMax) {
            atomicOr(&dsc->err, MXE_PLANWAIT);
            s_nsub = 0;
          } else {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_nsub = __hip_atomic_load(&dsc->n_sub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
        __syncthreads();
        nsub = s_nsub;
      }
    }
  }
  // The system's last block, when it has no subsystem and the subsystems leave
  // the massive bodies as they are, prepares the massive bodies of the joined
  // step boundary that follows (the same arithmetic as the joined step kernel,
  // which then copies them instead of computing them in every block).
  if constexpr (!kJoint) {
  if (plan && bx == nbx - 1) {
    if (!bigs_kept && nsub < nbx && nb <= kSmallBig) {
      double* b_sh = U.prep.sh;
      KickSource* b_src = U.prep.src;
      auto& b_bst = U.prep.bst;
      double* b_brc = U.prep.brc;
      double bpos[3], bvel[3], bm = 0.0, brc_t = 0.0, P[3], J[3], vpre[3], Ppre[3], Ppost[3];
      if (lane < nb) {
        for (int c = 0; c < 3; ++c) {
          bpos[c] = bigmid[c * nb + lane];
          bvel[c] = bigmid[(3 + c) * nb + lane];
        }
        bm = mu[lane];
        brc_t = rcrit[lane];
      }
      mxs::big_boundary(D, true, b_sh, b_src, b_bst, b_brc, bpos, bvel, bm, brc_t, P, J, vpre,
                        Ppre, Ppost);
      __syncthreads();
      BigNext* N = D.bignext + par;
      if (lane == 0) {
        for (int c = 0; c < 3; ++c) {
          N->P[c] = P[c];
          N->J[c] = J[c];
          N->vpre[c] = vpre[c];
          N->Ppre[c] = Ppre[c];
          N->Ppost[c] = Ppost[c];
        }
      }
      for (int i = lane; i < 8 * nb; i += 64)
        reinterpret_cast<double*>(N->src)[i] = reinterpret_cast<const double*>(b_src)[i];
      for (int i = lane; i < 12 * nb; i += 64) N->bst[i / nb][i % nb] = b_bst[i / nb][i % nb];
      for (int i = lane; i < nb; i += 64) N->brc[i] = b_brc[i];
      if (lane == 0) dsc->bn_valid[par] = 1;
    } else if (lane == 0) {
      dsc->bn_valid[par] = 0;
    }
  }
  }
  for (int b = bx; b < nsub; b += nbx) {
    __syncthreads();
    if (kJoint && jfast) {
      // subsystem b from its record: the massive partners in increasing index,
      // then the massless body, with its state, radius and density (the other
      // members' state from bigpre)
      uint64_t mask = r0mask;
      int jj = r0j;
      double rx[3] = {r0x[0], r0x[1], r0x[2]}, rv[3] = {r0v[0], r0v[1], r0v[2]};
      double rrp = r0rp, rrh = r0rh;
      if (b != bx) {
        const JointSub* R = D.jsub + (size_t)par * D.cap_subs + b;
        mask = R->mask;
        jj = R->j;
        for (int c = 0; c < 3; ++c) {
          rx[c] = R->x[c];
          rv[c] = R->v[c];
        }
        rrp = R->rp;
        rrh = R->rhop;
      }
      const int k = __popcll(mask);
      const bool fits = k + 1 <= kBsMaxMembers && k <= kBsMaxPairs;
      if (lane == 0) {
        S.m = fits ? k + 1 : 0;
        S.keep_from = fits ? k : 0;
        S.np = fits ? k : 0;
        S.jm = jj;
        if (fits) S.mem[k] = jj;
      }
      if (fits && ((mask >> lane) & 1ull)) {
        const int pos = __popcll(mask & ((1ull << lane) - 1ull));
        S.mem[pos] = lane;
        S.pl[pos][0] = pos;
        S.pl[pos][1] = k;
      }
      if (fits && lane < 6) {
        if (lane < 3) xs[3 * k + lane] = rx[lane];
        else vs[3 * k + lane - 3] = rv[lane - 3];
      }
      if (lane == 6) jr[0] = rrp;
      if (lane == 7) jr[1] = rrh;
    } else if (fast) {
      // subsystem b from the sorted keys in LDS
      const int e0 = F.gs[b], k = F.gs[b + 1] - e0;
      const bool fits = k + 1 <= kBsMaxMembers && k <= kBsMaxPairs;
      if (lane == 0) {
        S.m = fits ? k + 1 : 0;
        S.keep_from = fits ? k : 0;
        S.np = fits ? k : 0;
        S.jm = 0;
        if (fits) S.mem[k] = (int32_t)(F.kb[e0] >> 6);
      }
      if (fits && lane < k) {
        S.mem[lane] = (int32_t)(F.kb[e0 + lane] & 63u);
        S.pl[lane][0] = lane;
        S.pl[lane][1] = k;
      }
    } else {
      const auto src = reinterpret_cast<gmem<const int32_t>>(subs + b);
      int32_t* dst = reinterpret_cast<int32_t*>(&S);
      for (int i = lane; i < (int)(sizeof(Subsystem) / 4); i += 64) dst[i] = src[i];
    }
    __syncthreads();
    const int m = S.m, np = S.np;
    const int nn = 3 * m;
    if (m == 0) {  // a subsystem dropped for capacity (error already latched)
      if (kJoint && jfast)
        joint_member(D, S.jm, nullptr, nullptr, par, nx, jsrc, jbst, jbrc, jsc, nullptr);
      continue;
    }
    for (int e = lane; e < nn; e += 64) {
      int k = e / 3, c = e - 3 * (e / 3);
      int body = S.mem[k];
      if (kJoint && jfast) {  // massive members staged in LDS, the massless one from its record
        if (body < nb) {
          xs[e] = jstage[c * nb + body];
          vs[e] = jstage[(3 + c) * nb + body];
        }
        continue;
      }
      if (kJoint && body < nb) {
        const auto bigpre = gbl(D.bigpre) + (size_t)par * 6 * nb;
        xs[e] = bigpre[c * nb + body];
        vs[e] = bigpre[(3 + c) * nb + body];
      } else {
        xs[e] = x0s[(size_t)c * n + body];
        vs[e] = u0s[(size_t)c * n + body];
      }
    }
    for (int k = lane; k < m; k += 64) {
      int body = S.mem[k];
      if (kJoint && jfast) {
        mum[k] = body < nb ? jstage[6 * nb + body] : 0.0;
        rcm[k] = body < nb ? jstage[7 * nb + body] : 0.0;
      } else {
        mum[k] = body < nb ? mu[body] : 0.0;
        rcm[k] = body < nb ? rcrit[body] : 0.0;
      }
    }
    uint32_t pmask = 0;
    if (m <= 4)
      for (int q = 0; q < np; ++q) pmask |= 1u << pair_bit(S.pl[q][0], S.pl[q][1], m);
    __syncthreads();
    double done = 0.0, H = h;
    int fails = 0, nsched = 0;
    bool failed = false;
    if (m <= 4) {
      // a massless last member (the usual subsystem: massive bodies and the
      // planetesimal they met) takes the variant without its reaction terms
      const bool lm = mum[m - 1] == 0.0;
#define MX_BS_SMALL(MM, LMV) bs_small<MM, LMV>(lane, b, h, tol2, pmask, np, mum, rcm, mu0, xs, vs, scal, resS, D, dsc)
      if (m == 2) nsched = lm ? MX_BS_SMALL(2, true) : MX_BS_SMALL(2, false);
      else if (m == 3) nsched = lm ? MX_BS_SMALL(3, true) : MX_BS_SMALL(3, false);
      else nsched = lm ? MX_BS_SMALL(4, true) : MX_BS_SMALL(4, false);
#undef MX_BS_SMALL
      failed = nsched < 0;
      done = h;  // the loop below is for larger subsystems
    }
    while (fabs(h - done) > 1e-14 * fabs(h)) {
      double rem = h - done;
      if (fabs(H) > fabs(rem)) H = rem;
      for (int k = lane; k < m; k += 64) {
        const double* p = xs + 3 * k;
        const double* q = vs + 3 * k;
        scal[k] = 1.0 / (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        scal[m + k] = 1.0 / (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
      }
      // per element (two per lane): the previous table row and the diagonal
      double prev[2][kC], diag[2][kC];
      int accepted = -1;
      // all eight columns run at once in lanes 0..7: a step costs the longest
      // sequence (n = 16) instead of n = 8 followed by n = 16, which is what the
      // slowest subsystem of a launch pays; the accepted column is still the
      // first one within tolerance
      const bool wide = true;
#pragma unroll
      for (int r = 0; r < kC / kRound; ++r) {
        if (accepted < 0) {
          const int k0 = r * kRound;
          int c_lo = 0, c_hi = 0;  // columns evaluated in this round
          if (r == 0 && wide) {
            c_lo = 0;
            c_hi = kC;
            if (lane < kC)
              run_column(lane, H, m, np, S.pl, pmask, mum, rcm, mu0, xs, vs, wk[lane][0],
                         wk[lane][1], wk[lane][2], res[lane]);
          } else if (!(r == 1 && wide)) {
            c_lo = k0;
            c_hi = k0 + kRound;
            if (lane < kRound)
              run_column(k0 + lane, H, m, np, S.pl, pmask, mum, rcm, mu0, xs, vs, wk[lane][0],
                         wk[lane][1], wk[lane][2], res[k0 + lane]);
          }
          if (lane == 0) {
            // model count: per force evaluation 24 ops per member (star term and
            // position update) and 25 per flagged pair; 3 per extrapolation entry
            unsigned long long f = 0;
            for (int c = c_lo; c < c_hi; ++c)
              f += (unsigned long long)(2 * (c + 1) + 1) * (24 * m + 25 * np);
            for (int k = k0; k < k0 + kRound; ++k) f += (unsigned long long)3 * k * 6 * m;
            atomicAdd(&dsc->bs_flop, f);
          }
          __syncthreads();
          double lerr[kRound];
          if (r == 0) neville_round<0>(lane, nn, m, res, scal, prev, diag, lerr);
          else neville_round<kRound>(lane, nn, m, res, scal, prev, diag, lerr);
#pragma unroll
          for (int kk = 0; kk < kRound; ++kk) {
            double v = lerr[kk];
            for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
            const int k = k0 + kk;
            if (accepted < 0 && k >= 1 && v <= tol2) accepted = k;
          }
          __syncthreads();
        }
      }
      if (accepted >= 0) {
        for (int slot = 0; slot < 2; ++slot) {
          const int e = lane + 64 * slot;
          if (e >= 2 * nn) continue;
          double val = diag[slot][1];
#pragma unroll
          for (int k = 2; k < kC; ++k)
            if (k == accepted) val = diag[slot][k];
          if (e < nn) xs[e] = val;
          else vs[e - nn] = val;
        }
        if (D.bs_sched && lane == 0) {
          if (nsched < kBsMaxSched) {
            D.bs_sched[((size_t)b * kBsMaxSched + nsched) * 2] = H;
            D.bs_sched[((size_t)b * kBsMaxSched + nsched) * 2 + 1] = (double)accepted;
          } else {
            atomicOr(&dsc->err, MXE_ADJOINT);
          }
        }
        ++nsched;
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
    if (D.bs_sched && lane == 0) D.bs_nsched[b] = failed ? 0 : nsched;
    if (failed) {
      if (lane == 0) atomicOr(&dsc->err, MXE_BS);
      if (kJoint && jfast) joint_member(D, S.mem[m - 1], nullptr, nullptr, par, nx, jsrc, jbst,
                                        jbrc, jsc, jr);
      continue;
    }
    if (kJoint && jfast) {  // the member's closing and opening replace the write-back
      joint_member(D, S.mem[m - 1], xs + 3 * (m - 1), vs + 3 * (m - 1), par, nx, jsrc, jbst,
                   jbrc, jsc, jr);
      continue;
    }
    for (int e = lane; e < nn; e += 64) {
      int k = e / 3, c = e - 3 * (e / 3);
      if (k < S.keep_from) continue;
      int body = S.mem[k];
      x[(size_t)c * n + body] = xs[e];
      u[(size_t)c * n + body] = vs[e];
      if (body < nb) {
        bigmid[(size_t)c * nb + body] = xs[e];
        bigmid[(size_t)(3 + c) * nb + body] = vs[e];
      }
    }
  }
  return jfast;
}

__global__ __launch_bounds__(64) void k_bs(const SysDesc* __restrict__ desc, int plan, int par,
                                           int lst, int clr) {
  bs_body<false>(desc[blockIdx.y], blockIdx.x, gridDim.x, plan, par, 0, lst, clr, nullptr,
                 nullptr, nullptr, nullptr, nullptr);
}

// One launch per step of a joint sequence (systems with 0 < n_big <= 64 and no
// core growth: a single system, or every member of a batch): blocks 0 ..
// nbs * n_sys - 1 run the encounter integrator of step q (phase ph; nbs one-wave
// blocks per system, system-major), the following blocks (one BLK-body tile of
// the tile table each) close step q and open step q + 1 (phase nx) for their
// bodies with exactly the joined step kernel's operations.  The integrator's registers set the launch
// to one wave per SIMD; with one-wave blocks an integrator block holds one SIMD
// of a CU, not the whole CU, while it runs.  The two parts depend on each other only
// through the bodies the integrator moves, and the launch that opened step q
// prepared what the closing needs when no flagged pair of step q joins two
// massive bodies (prepare_boundary: the massive bodies are then left as they
// are; jfast, read by every block from the same final value): the tile blocks
// then skip the flagged bodies, whose closing and opening the integrator's wave
// does after their subsystem, and nothing waits.
// Otherwise the tile blocks wait for every integrator block (a count released
// at agent scope; the integrator's blocks have the lower indices, so they are
// dispatched first and the wait ends) and then close every body as the joined
// kernel does, from the massive bodies the integrator left.  What step q + 1
// appends goes to the copies of phase nx, which nothing in this launch reads, the
// massive members start from bigpre (the tile of the massive bodies rewrites
// x0, u0), and the tile of the massive bodies clears the copies of step q - 1 and
// prepares the next boundary.
template <int BLK>
__global__ __launch_bounds__(BLK) void k_step_joint(const SysDesc* __restrict__ desc,
                                                    const Tile* __restrict__ tiles, int nbs,
                                                    int n_sys, int ph) {
  using namespace mxs;
  const int nbs_all = nbs * n_sys;
  const Tile tl = (int)blockIdx.x < nbs_all ? Tile{(int)blockIdx.x / nbs, 0}
                                            : tiles[blockIdx.x - nbs_all];
  const SysDesc& D = desc[tl.sys];
  __shared__ double sh[8];
  __shared__ KickSource src[kSmallBig];
  __shared__ double bst[12][kSmallBig];
  __shared__ double brc[kSmallBig];
  __shared__ uint32_t fl[BLK / 32];  // the tile's bodies the integrator closes
  __shared__ double jsc[12], jr[2];  // integrator blocks: J, vpre, Ppre, Ppost; rp, rho_p
  const int nx = ph == 2 ? 0 : ph + 1;
  const int tid = threadIdx.x;
  const int n = D.n, nb = D.nb;
  const double h = D.h, hh = 0.5 * D.h, mu0 = D.mu0;
  DevScalars* __restrict__ dsc = D.dsc;
  if ((int)blockIdx.x < nbs_all) {
    if (tid >= 64) return;  // one wave per integrator block
    // the integrator's chain sets the launch time: its wave takes the issue
    // slots first when a tile wave shares its SIMD
    __builtin_amdgcn_s_setprio(3);
    const bool jfast =
        bs_body<true>(D, (int)blockIdx.x % nbs, nbs, 1, ph, nx, ph, -1, src, bst, brc, jsc, jr);
    if (!jfast) {
      __syncthreads();  // the wave's stores precede the release
      if (tid == 0)
        __hip_atomic_fetch_add(&dsc->bs_done[ph], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  const bool jfast = dsc->bn_valid[ph] != 0;
  const int t = tl.first + tid;
  const bool owner = tl.first == 0;  // block-uniform: the tile of the massive bodies
  if (!jfast) {
    if (tid == 0) {
      int it = 0;
      while (__hip_atomic_load(&dsc->bs_done[ph], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
             nbs) {
        __builtin_amdgcn_s_sleep(8);
        if (++it >= kPlanWaitMax) break;
      }
      if (it >= kPlanWaitMax) atomicOr(&dsc->err, MXE_PLANWAIT);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
  }
  double bpos[3], bvel[3], bm = 0.0, brc_t = 0.0;
  if (tid < nb) {
    bm = gbl(D.mu)[tid];
    brc_t = gbl(D.rcrit)[tid];
    if (!jfast) {
      const auto bigmid = gbl(D.bigmid) + (size_t)ph * 6 * nb;
      for (int c = 0; c < 3; ++c) {
        bpos[c] = bigmid[c * nb + tid];
        bvel[c] = bigmid[(3 + c) * nb + tid];
      }
    }
  }
  double p[3], v[3], a[3], q[3], w[3], rp = 0.0, rhop = 0.0;
  if (t < n && t >= nb) {
    for (int c = 0; c < 3; ++c) {
      p[c] = gbl(D.x)[c * n + t];
      v[c] = gbl(D.u)[c * n + t];
    }
    if (D.gas_on) {
      rp = gbl(D.r_p)[t - nb];
      rhop = gbl(D.rho_p)[t - nb];
    }
  }
  double P[3], J[3], vpre[3], Ppre[3], Ppost[3];
  if (jfast) {
    const BigNext* N = D.bignext + ph;
    if (tid < BLK / 32) fl[tid] = 0u;
    for (int i = tid; i < 8 * nb; i += BLK)
      reinterpret_cast<double*>(src)[i] = reinterpret_cast<const double*>(N->src)[i];
    for (int i = tid; i < 12 * nb; i += BLK) bst[i / nb][i % nb] = N->bst[i / nb][i % nb];
    for (int i = tid; i < nb; i += BLK) brc[i] = N->brc[i];
    for (int c = 0; c < 3; ++c) {
      P[c] = N->P[c];
      J[c] = N->J[c];
      vpre[c] = N->vpre[c];
      Ppre[c] = N->Ppre[c];
      Ppost[c] = N->Ppost[c];
    }
    __syncthreads();
    // the bodies with a subsystem record: the integrator closes and opens them
    const int nrec = min(dsc->n_jsub[ph], D.cap_subs);
    const JointSub* recs = D.jsub + (size_t)ph * D.cap_subs;
    for (int e = tid; e < nrec; e += BLK) {
      const int j = recs[e].j - tl.first;
      if (j >= 0 && j < BLK) atomicOr(&fl[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
  } else {
    big_boundary(D, owner, sh, src, bst, brc, bpos, bvel, bm, brc_t, P, J, vpre, Ppre, Ppost);
  }
  if (owner && tid == 0) {
    dsc->P[0] = P[0];
    dsc->P[1] = P[1];
    dsc->P[2] = P[2];
    dsc->step += 1;
    dsc->joint_runs += 1;
    if (!jfast) dsc->joint_slow += 1;
    const int r = nx == 2 ? 0 : nx + 1;  // step q - 1: nothing in this launch reads its copies
    dsc->n_pairs[r] = 0;
    dsc->plan_ready[r] = 0;
    dsc->bs_done[r] = 0;
    dsc->n_jsub[r] = 0;
  }
  const bool skip = jfast && ((fl[tid >> 5] >> (tid & 31)) & 1u);
  const bool mine = t < n && !skip;
  // step q closed and step q + 1 opened for the body
  if (mine && t >= nb) {
    close_body(t, nb, src, 0.0, J, vpre, hh, D.dc, D.gas_on, rp, rhop, true, p, v, a);
    if (!isfinite(v[0] + v[1] + v[2] + p[0] + p[1] + p[2])) atomicOr(&dsc->err, MXE_NONFINITE);
    if (!advance_body(t, nb, mu0, h, D.dc, D.gas_on, rp, rhop, Ppre, Ppost, p, v, a, q, w))
      atomicOr(&dsc->err, MXE_NOCONV);
  }
  __syncthreads();  // the massive bodies of step q + 1 are in LDS
  bool hit = false;
  if (mine) {
    if (t < nb) {
      for (int c = 0; c < 3; ++c) {
        p[c] = bst[c][t];
        v[c] = bst[3 + c][t];
        q[c] = bst[6 + c][t];
        w[c] = bst[9 + c][t];
      }
      const auto bigmid = gbl(D.bigmid) + (size_t)nx * 6 * nb;
      const auto bigpre = gbl(D.bigpre) + (size_t)nx * 6 * nb;
      for (int c = 0; c < 3; ++c) {
        bigmid[c * nb + t] = q[c];
        bigmid[(3 + c) * nb + t] = w[c];
        bigpre[c * nb + t] = p[c];
        bigpre[(3 + c) * nb + t] = v[c];
      }
    }
    for (int c = 0; c < 3; ++c) {
      gbl(D.x)[c * n + t] = q[c];
      gbl(D.u)[c * n + t] = w[c];
    }
    hit = flag_body(D, nx, nx, t, n, nb, h, bst, brc, p, v, q, w, true, rp, rhop);
  }
  if (owner) {
    const bool any_bb = __syncthreads_or(t < nb && hit);
    prepare_boundary(D, nx, any_bb, sh, src, bst, brc, q, w, bm, brc_t);
  }
}

}  // namespace

namespace mxk {

// Source split of the flag kernel: 256 targets per block, enough blocks for
// about four waves per SIMD, at least 32 sources per split.
int flag_split(int n, int nb) {
  int tiles = (n + kBlock - 1) / kBlock;
  int split = (1024 + tiles - 1) / tiles;
  int maxs = nb / 32;
  if (split > maxs) split = maxs;
  if (split > 64) split = 64;
  if (split < 1) split = 1;
  return split;
}

hipError_t launch_flag(mx_system* s) {
  if (s->flag_perm && s->nb > 0) {
    const int nC = (s->nb + 63) / 64;
    hipError_t e = mxlaunch(s, k_chunk_bounds, dim3(nC), dim3(64), s->nb, s->p.dt,
                            s->flag_perm, s->fpack, s->flag_bounds);
    if (e != hipSuccess) return e;
    return mxlaunch(s, k_flag_cull, dim3(nC * (nC + 1) / 2 * (64 / kCullPart)), dim3(64), s->nb,
                    s->p.dt, s->flag_perm, s->flag_bounds, s->x0, s->u0, s->x, s->u, s->fpack,
                    s->pairs, s->cap_pairs, &s->dsc->n_pairs[0], &s->dsc->err);
  }
  int tiles = (s->n + kBlock - 1) / kBlock;
  int split = flag_split(s->n, s->nb);
  if (s->nb == 0) return hipSuccess;
  return mxlaunch(s, k_flag, dim3(tiles * split), dim3(kBlock), s->n, s->nb, split, s->p.dt,
                  s->x0, s->u0, s->x, s->u, s->fpack, s->pairs, s->cap_pairs, &s->dsc->n_pairs[0],
                  &s->dsc->err);
}

hipError_t launch_bs_sys(hipStream_t st, LaunchTiming* tm, const SysDesc* desc, int n_sys,
                         int bps, int plan, int par, int lst, int clr) {
  if (n_sys <= 0 || bps <= 0) return hipSuccess;
  return mxlaunch_on(st, tm, k_bs, dim3(bps, n_sys), dim3(64), desc, plan, par, lst, clr);
}

hipError_t launch_step_joint(hipStream_t st, LaunchTiming* tm, const SysDesc* desc,
                             const Tile* tiles64, int n_tiles64, int nbs, int n_sys, int ph) {
  if (n_tiles64 <= 0 || nbs <= 0 || n_sys <= 0 || ph < 0 || ph > 2) return hipErrorInvalidValue;
  return mxlaunch_on(st, tm, k_step_joint<64>, dim3(nbs * n_sys + n_tiles64), dim3(64), desc,
                     tiles64, nbs, n_sys, ph);
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

// Queues the stateless encounter test on caller buffers: source packing into fp
// ([nb] records), flagging into pairs, and the (i, j) sort of the list with
// pairs_tmp (2 cap int64) as keys; dsc must start zeroed.  No allocation, no
// synchronisation.
hipError_t flag_pairs_enqueue(int n, int nb, const double* rcrit, const double* x0,
                              const double* u0, const double* x1, const double* u1, double h,
                              int32_t* pairs, int32_t* pairs_tmp, int32_t cap, DevScalars* dsc,
                              FlagSource* fp, hipStream_t st) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fpack_plain, dim3((nb + 255) / 256), dim3(256), 0, st, n, nb, rcrit, x0, u0,
                     x1, u1, fp);
  int tiles = (n + kBlock - 1) / kBlock;
  int split = flag_split(n, nb);
  hipLaunchKernelGGL(k_flag, dim3(tiles * split), dim3(kBlock), 0, st, n, nb, split, h, x0, u0, x1,
                     u1, fp, pairs, cap, &dsc->n_pairs[0], &dsc->err);
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, st, nb, pairs, cap,
                     (int64_t*)pairs_tmp, nullptr, nullptr, nullptr, 0, dsc, 1);
  return hipGetLastError();
}

hipError_t flag_pairs(int n, int nb, const double* rcrit, const double* x0, const double* u0,
                      const double* x1, const double* u1, double h, int32_t* pairs,
                      int32_t* pairs_tmp, int32_t cap, DevScalars* dsc, hipStream_t st) {
  if (nb == 0) return hipSuccess;
  FlagSource* fp = nullptr;
  hipError_t e = hipMalloc((void**)&fp, sizeof(FlagSource) * nb);
  if (e != hipSuccess) return e;
  e = flag_pairs_enqueue(n, nb, rcrit, x0, u0, x1, u1, h, pairs, pairs_tmp, cap, dsc, fp, st);
  hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFree(fp);
  return e != hipSuccess ? e : e2;
}

}  // namespace mxk
