// sfhk_kernels.hpp -- device data layout and the propagation kernels of the SFHK hot path
// (gfx950): single-job, multi-job and batched (graph-replayed) forms, FP64 and FP32-mixed.
// Included by sfhk.hip (the host runtime behind include/sfhk.h), in one translation unit.
//
// Layout in HBM (per job):
//   trajectories are ordered by birth step (stable) and padded to tiles of 64 lanes; tile t holds
//   sorted trajectories 64t..64t+63, so tiles are ordered longest first;
//   state y[43][n_pad] (SoA, FP64): q(3) p(3) M(6 columns of Q(3) P(3)) S; aux[5][n_pad]:
//   C_prev (re, im), w (re, im), branch sign; n0[n_pad], death[n_pad] (int32);
//   one exact accumulator per step for Re F and one for Im F (sfhk_exact_sum.hpp: 68 64-bit
//   words each, zero when the job is created), and two more per step for the dipole velocity:
//   each tile adds, per step, the sum of its lanes' integrands with integer atomics.
// The accumulated totals are exact and do not depend on the order of the additions, so the dipole
// is bitwise reproducible for a given input however the tiles are scheduled, chunked or batched.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/sfhk.h"
#include "sfhk_device.hpp"
#include "sfhk_device_f32.hpp"
#include "sfhk_exact_sum.hpp"

using namespace sfhk;

namespace {

constexpr int kTile = 64;           // trajectories per tile = lanes per wave
constexpr int kNY = 43;

// ------------------------------------------------------------------------------------------------
// device-side job description
// ------------------------------------------------------------------------------------------------
struct GtoConst {
  int l, n_prim;
  double A[SFHK_MAX_PRIM];   // 1 / (4 (gamma + alpha_j))
  double B[SFHK_MAX_PRIM];   // alpha_j gamma / (gamma + alpha_j)
  double D[SFHK_MAX_PRIM];   // alpha_j / (gamma + alpha_j)
  double N[SFHK_MAX_PRIM];   // c_j (gamma + alpha_j)^(-5/2) (l = 0) or ^(-7/2) (l = 1)
  double G2[SFHK_MAX_PRIM];  // 2 (gamma + alpha_j)
  double Va[SFHK_MAX_PRIM];  // dipole velocity: alpha_j
  double Vg[SFHK_MAX_PRIM];  // dipole velocity: 2 gamma (gamma + alpha_j)
  double two_gamma, ip;
  double Amin, Bmin, cut_hi;  // all-primitives-skipped bound (see overlap_all_skipped)
  int vel;                    // also evaluate the dipole-velocity element (App. C.2)
};

struct JobDev {
  int kind;
  PotParams pot;
  GtoConst gto;
  double gamma, inv4g, kay2, cut;
  double r64sq;  // mixed precision: steps that start at r^2 < r64sq run in FP64
  double t_a, h, h2, h6;
  int n_steps;
  int n_tiles;
  long long n_pad;
  const double* e_half;
  double* y;
  double* aux;
  int* n0;
  int* death;
  int* tile_n0;
  int* tile_next;
  int* tile_last;
  long long* acc;      // [n_steps + 1][2][kExactWords]: exact sums of Re F, Im F per step
  long long* acc_v;    // the same for the dipole velocity (nullptr: not accumulated)
  int pw_mask;        // partial-wave filter (0: every step counts), see pw_keep
  double pw_r2;       // its radius, squared
  unsigned long long* counters;  // steps_evaluated, kay_removed, nonfinite_removed, steps_fp64,
                                 // GTO primitives evaluated, integrands evaluated
  // regrouping of live trajectories (compact_every > 0; see k_propagate_rg)
  int compact_every;  // boundary interval in steps (0: off)
  long long* perm;    // [n_pad] slot -> caller's trajectory index (-1: padding); nullptr: identity
};

// values that are the same in every lane of the wave (per-tile bookkeeping): kept in scalar
// registers so the step loop's control runs on the scalar unit
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uniform_i64(long long v) {
  const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)(unsigned long long)v);
  const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// ------------------------------------------------------------------------------------------------
// wave-level sum (butterfly: every lane ends with the same, order-independent-by-symmetry value)
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ------------------------------------------------------------------------------------------------
// dipole element <psi0|z|p,q,gamma> over GTOs (App. C.1, overall constant 1). Tolerance-level
// arithmetic: it does not feed back into the trajectory.
// ------------------------------------------------------------------------------------------------
// Every primitive is skipped when p^2 A_j + q^2 B_j > cut for all j. Since A_j >= A_min and
// B_j >= B_min, p^2 A_min + q^2 B_min > cut (1 + 1e-12) implies it; the margin covers rounding.
__device__ __forceinline__ bool overlap_all_skipped(double amin, double bmin, double cut_hi,
                                                    double p2, double q2) {
  return SFHK_FMA(p2, amin, q2 * bmin) > cut_hi;
}

// sin and cos of x for the dipole integrand (held to the oracle at a relative tolerance, not bit
// for bit). Reduction x = n pi/2 + r with the two-part constant pi/2 = C1 + C2 and fused
// multiply-adds (|r| <= pi/4, error about |n| 2e-33), Taylor polynomials in r^2 to degree 13 (sin)
// and 14 (cos), truncation below 3e-14, then the quadrant. Accurate for |x| < 2^52; beyond that,
// and for a NaN or an infinity, both are NaN. The integrand's arguments, phi - D_j p.q, stay far
// below: an evaluated primitive has p^2 A_j + q^2 B_j <= overlap_cut, so
// |p.q| <= overlap_cut / sqrt(A_min B_min), and the phase phi = S - Ip t is an action of order
// 10^4 at most.
struct InvFactorials14 {
  double v[15];
  constexpr InvFactorials14() : v() {
    double f = 1.0;
    for (int n = 0; n < 15; ++n) {
      if (n > 0) f *= (double)n;  // n! is exact in binary64 for n <= 18
      v[n] = 1.0 / f;
    }
  }
};
constexpr InvFactorials14 kInvFact14{};

__device__ __forceinline__ void sincos_integrand(double x, double* sp, double* cp) {
  constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
  constexpr double kC1 = 0x1.921fb54442d18p+0;   // pi/2 rounded to binary64
  constexpr double kC2 = 0x1.1a62633145c07p-54;  // pi/2 - kC1 rounded
  const double n = rint(x * kTwoOverPi);
  double r = SFHK_FMA(-n, kC1, x);
  r = SFHK_FMA(-n, kC2, r);
  const double r2 = r * r;
  // sin r = r (1 - r^2/3! + r^4/5! - ...), cos r = 1 - r^2/2! + r^4/4! - ...
  double ps = kInvFact14.v[13];
#pragma unroll
  for (int k = 11; k >= 3; k -= 2) ps = fma3(ps, r2, (k % 4 == 1) ? kInvFact14.v[k] : -kInvFact14.v[k]);
  const double sr = SFHK_FMA(ps * r2, r, r);
  double pc = -kInvFact14.v[14];
#pragma unroll
  for (int k = 12; k >= 4; k -= 2) pc = fma3(pc, r2, (k % 4 == 0) ? kInvFact14.v[k] : -kInvFact14.v[k]);
  pc = SFHK_FMA(pc, r2, -0.5);  // -1/2!: an inline constant
  const double cr = SFHK_FMA(pc, r2, 1.0);
  const int q = (int)(n - 4.0 * floor(0.25 * n));  // n mod 4, exact for |n| < 2^53
  double s = (q & 1) ? cr : sr;
  double c = (q & 1) ? sr : cr;
  s = (q & 2) ? -s : s;
  c = ((q + 1) & 2) ? -c : c;
  const bool ok = fabs(x) < 0x1p52;  // beyond, and for NaN or infinity: NaN
  *sp = ok ? s : __builtin_nan("");
  *cp = ok ? c : __builtin_nan("");
}

// The dipole element O = <psi0|z|p,q,gamma> (App. C.1) and, when G.vel is set, the
// dipole-velocity element Ov = <psi0|k_z|p,q,gamma> (App. C.2) in the same scale. With
// a = 2 gamma q_z + i p_z (so p_z - 2 i gamma q_z = -i a) and E_j the primitive's exponential:
//   s-wave: O = a sum_j N_j E_j,                   Ov = -2 i a sum_j alpha_j N_j E_j
//   p-wave: O = sum_j N_j E_j (a^2 + 2 (g + a_j)),  Ov = 2 i sum_j N_j E_j (2 g (g + a_j) - a_j a^2)
// (the printed velocity forms times 2 and 4 i gamma, the ratio of the two elements' written-out
// constants, so that the real part taken by "+ c.c." is the same for both forms). Both come out
// times the phase e^{i phi}, which enters each primitive's angle: E_j e^{i phi} =
// N_j e^{Re_j} e^{i (phi - D_j p.q)}, one sincos per primitive and none for the phase alone.
struct Elements {
  cplx o, ov;
};

// the GTO constants seen through the constant address space: with a wave-uniform pointer their
// reads are scalar loads
typedef const __attribute__((address_space(4))) GtoConst& gto_cref;
typedef const __attribute__((address_space(4))) GtoConst* gto_cptr;

template <typename GREF>
__device__ __forceinline__ Elements overlap(GREF G, double cut, const double* q,
                                            const double* p, double p2, double q2, double phi,
                                            unsigned int& n_eval) {
  double pq = SFHK_FMA(p[2], q[2], SFHK_FMA(p[1], q[1], p[0] * q[0]));
  cplx a = {G.two_gamma * q[2], p[2]};
  cplx sum = {0.0, 0.0}, sumv = {0.0, 0.0};
  cplx a2 = cmul(a, a);
  for (int j = 0; j < G.n_prim; ++j) {
    double re = -SFHK_FMA(p2, G.A[j], q2 * G.B[j]);
    if (re >= -cut) {
      ++n_eval;
      double im = SFHK_FMA(-pq, G.D[j], phi);
      double e = exp_cw_nonpos(re) * G.N[j];
      double s, c;
      sincos_integrand(im, &s, &c);
      cplx E = {e * c, e * s};
      if (G.l == 0) {
        sum.re += E.re;
        sum.im += E.im;
        if (G.vel) {
          sumv.re += G.Va[j] * E.re;
          sumv.im += G.Va[j] * E.im;
        }
      } else {
        cplx b = {a2.re + G.G2[j], a2.im};
        cplx t = cmul(E, b);
        sum.re += t.re;
        sum.im += t.im;
        if (G.vel) {
          cplx bv = {G.Vg[j] - G.Va[j] * a2.re, -(G.Va[j] * a2.im)};
          cplx tv = cmul(E, bv);
          sumv.re += tv.re;
          sumv.im += tv.im;
        }
      }
    }
  }
  Elements r;
  if (G.l == 0) {
    r.o = cmul(a, sum);
    const cplx t = cmul(a, sumv);
    r.ov = {2.0 * t.im, -2.0 * t.re};  // -2 i t
  } else {
    r.o = sum;
    r.ov = {-2.0 * sumv.im, 2.0 * sumv.re};  // 2 i sumv
  }
  return r;
}

// The integrands f = w C O e^{i (S - Ip t_n)} and fv = w C Ov e^{i (S - Ip t_n)} of one lane
// (0 when every primitive is skipped). Kept out of line: it runs only for lanes near the ground
// state, and inlined, the constants and temporaries of its exp and sincos would occupy registers
// for the whole step loop.
struct Contrib {
  double re, im, vre, vim;
  unsigned int n_eval;
};

__device__ __noinline__ Contrib contribution(const GtoConst* Gv, double cut, double qx,
                                             double qy, double qz, double px, double py, double pz,
                                             double p2, double q2, double S, double tn, double wcr,
                                             double wci) {
  // every lane passes the same constants: read through a uniform pointer in the constant address
  // space they are scalar loads, instead of a vector load and a wait per primitive
  const gto_cptr __restrict__ G = (gto_cptr)uniform_i64((long long)Gv);
  const double q[3] = {qx, qy, qz}, p[3] = {px, py, pz};
  unsigned int n_eval = 0;
  const double phi = S - G->ip * tn;
  const Elements el = overlap<gto_cref>(*G, cut, q, p, p2, q2, phi, n_eval);
  const cplx w = {wcr, wci};
  const cplx f = cmul(w, el.o);
  Contrib r = {f.re, f.im, 0.0, 0.0, n_eval};
  if (G->vel) {
    const cplx fv = cmul(w, el.ov);
    r.vre = fv.re;
    r.vim = fv.im;
  }
  return r;
}

// ------------------------------------------------------------------------------------------------
// propagation, FP64: one wave per tile, one trajectory per lane
// ------------------------------------------------------------------------------------------------
// The dipole integrand is deferred. At a given step few lanes of a wave are near the ground state,
// and evaluated in place their integrand would cost the whole wave. Instead each such lane appends
// (q, p, S, w C, n) to a per-wave LDS queue; when the queue cannot take the next step's entries,
// and at the end of the launch, the wave evaluates up to 64 of them at once, one per lane. A
// step's entries are consecutive lanes in lane order; a segmented scan over the wave (run_sum)
// sums each run and its last lane adds the sum to the step's exact accumulators. The scan's
// additions depend only on positions within the run, and the entries of one step never straddle
// two evaluations, so a run's sum does not depend on where it lies in the queue, nor on how the
// propagation is split into launches or batched; the accumulators' totals do not depend on the
// order of the additions. The wave is the whole workgroup, so the queue needs no cross-wave
// synchronisation.
constexpr int kQueue = kTile;

struct WorkItem {
  int job, tile;
};

struct QueueEntry {
  double2 a, b, c, d, e;  // (qx, qy) (qz, px) (py, pz) (S, Re wC) (Im wC, n)
};
struct IntegrandQueue {
  QueueEntry e[kQueue];
};

typedef __attribute__((address_space(4))) const double* const_dptr;  // scalar (uniform) loads

// position of this lane among the set bits of the wave mask m
__device__ __forceinline__ int lanes_below(unsigned long long m) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned int)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned int)m, 0u));
}

__device__ __forceinline__ void queue_push(IntegrandQueue& Q, int idx, double qx, double qy,
                                           double qz, double px, double py, double pz, double S,
                                           cplx wC, int n) {
  QueueEntry& x = Q.e[idx];
  x.a = make_double2(qx, qy);
  x.b = make_double2(qz, px);
  x.c = make_double2(py, pz);
  x.d = make_double2(S, wC.re);
  x.e = make_double2(wC.im, (double)n);
}

// Partial-wave filter (Sec. III.A): near the core the angular momentum l = |q x p| is nearly
// conserved, and each step there is labelled by the band [k - 1/2, k + 1/2) that holds l (s, p,
// d, ... for k = 0, 1, 2, ...; bit 7 for l >= 13/2). A step's terms count when r^2 < pw_r2 and the
// band's bit is set, or, beyond the radius, when bit 8 is set. r^2 and l^2 are formed by one fixed
// sequence and compared with the squared edges, so the decision is reproducible bit for bit.
__device__ __forceinline__ bool pw_keep(int pw_mask, double pw_r2, double qx, double qy, double qz,
                                        double px, double py, double pz) {
  const double r2 = SFHK_FMA(qz, qz, SFHK_FMA(qy, qy, qx * qx));
  if (!(r2 < pw_r2)) return (pw_mask >> 8) & 1;
  const double cx = SFHK_FMA(qy, pz, -(qz * py));
  const double cy = SFHK_FMA(qz, px, -(qx * pz));
  const double cz = SFHK_FMA(qx, py, -(qy * px));
  const double l2 = SFHK_FMA(cz, cz, SFHK_FMA(cy, cy, cx * cx));
  int k = 0;
  while (k < 7 && !(l2 < (k + 0.5) * (k + 0.5))) ++k;
  return (pw_mask >> k) & 1;
}

// sum over the run of equal keys that ends at this lane, for runs of consecutive lanes (run_start
// = first lane of this lane's run): a Hillis-Steele scan whose additions depend only on positions
// relative to the run's start, so a run's total does not depend on where the run lies in the wave
__device__ __forceinline__ double run_sum(double x, int lane, int run_start) {
#pragma unroll
  for (int off = 1; off < kQueue; off <<= 1) {
    const double y = __shfl_up(x, off, 64);
    if (lane - off >= run_start) x += y;
  }
  return x;
}

// global-memory view of an accumulator: its atomics then count only as vector-memory operations, so
// waiting for LDS results does not wait for them
typedef __attribute__((address_space(1))) unsigned long long* acc_gptr;

// adds one value to an exact accumulator (sfhk_exact_sum.hpp) with integer atomics
__device__ __forceinline__ void acc_add(long long* __restrict__ a, double v) {
  const sfhk_exact::Slices sl = sfhk_exact::slices_of(v);
  const acc_gptr w = (acc_gptr)a;
  if (sl.flag) {
    __hip_atomic_fetch_or(w + sfhk_exact::kExactFlag, (unsigned long long)sl.flag, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  if (sl.n == 0) return;
  __hip_atomic_fetch_add(w + sl.bin, (unsigned long long)sl.s[0], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_add(w + sl.bin + 1, (unsigned long long)sl.s[1], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  if (sl.n == 3)
    __hip_atomic_fetch_add(w + sl.bin + 2, (unsigned long long)sl.s[2], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// adds (re, im) to step n's pair of accumulators
__device__ __forceinline__ void acc_add_step(long long* __restrict__ acc, long long n, double re,
                                             double im) {
  long long* a = acc + n * (2 * sfhk_exact::kExactWords);
  acc_add(a, re);
  acc_add(a + sfhk_exact::kExactWords, im);
}

// the job's values the queue evaluation needs, read once per tile: the accumulators' atomics could
// alias the descriptor as far as the compiler knows, and re-reading it after them would wait for
// them to complete
struct QueueCtx {
  const GtoConst* gto;
  long long* acc;
  long long* acc_v;
  double cut, t_a, h, pw_r2;
  int pw_mask;
};

__device__ __forceinline__ QueueCtx queue_ctx(const JobDev& J) {
  QueueCtx c;
  c.gto = &J.gto;
  c.acc = J.acc;
  c.acc_v = J.acc_v;
  c.cut = J.cut;
  c.t_a = J.t_a;
  c.h = J.h;
  c.pw_r2 = J.pw_r2;
  c.pw_mask = J.pw_mask;
  return c;
}

// Orders a wave's accesses to its own LDS queue: the LDS requests of one wave complete in issue
// order, so a wave needs no barrier with the other waves of its workgroup, only that neither the
// compiler nor the wait counters move an access across this point. ONE_WAVE: the workgroup is this
// wave, and the workgroup barrier serves.
template <bool ONE_WAVE>
__device__ __forceinline__ void queue_sync() {
  if (ONE_WAVE) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS accesses have completed
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// evaluates the qn queued entries (one per lane) and adds their per-step sums to the job's
// accumulators; returns this lane's count of evaluated primitives. A step's entries are
// consecutive lanes (a run); the last lane of the run adds the run's sum.
template <bool ONE_WAVE = true>
__device__ __forceinline__ unsigned int queue_eval(IntegrandQueue& Q, int qn, int lane,
                                                   const QueueCtx& J) {
  queue_sync<ONE_WAVE>();
  unsigned int n_eval = 0;
  Contrib cb = {0.0, 0.0, 0.0, 0.0, 0u};
  double ns = -1.0;
  if (lane < qn) {
    const QueueEntry x = Q.e[lane];
    const double qx = x.a.x, qy = x.a.y, qz = x.b.x, px = x.b.y, py = x.c.x, pz = x.c.y;
    const double p2 = SFHK_FMA(pz, pz, SFHK_FMA(py, py, px * px));
    const double q2 = SFHK_FMA(qz, qz, SFHK_FMA(qy, qy, qx * qx));
    ns = x.e.y;
    if (!J.pw_mask || pw_keep(J.pw_mask, J.pw_r2, qx, qy, qz, px, py, pz))
      cb = contribution(J.gto, J.cut, qx, qy, qz, px, py, pz, p2, q2, x.d.x, J.t_a + x.e.y * J.h,
                        x.d.y, x.e.x);
    n_eval = cb.n_eval;
  }
  // runs of equal steps: starts as a wave mask, this lane's run start, and whether it ends one
  const double prev = __shfl_up(ns, 1, 64);
  const unsigned long long starts =
      __builtin_amdgcn_ballot_w64(lane < qn && (lane == 0 || prev != ns));
  const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
  const int rs = 63 - __clzll(starts & upto);
  const bool last = lane < qn && (lane == qn - 1 || ((starts >> (lane + 1)) & 1ull));
  const double sr = run_sum(cb.re, lane, rs), si = run_sum(cb.im, lane, rs);
  if (last) acc_add_step(J.acc, (long long)ns, sr, si);
  if (J.acc_v) {
    const double vr = run_sum(cb.vre, lane, rs), vi = run_sum(cb.vim, lane, rs);
    if (last) acc_add_step(J.acc_v, (long long)ns, vr, vi);
  }
  queue_sync<ONE_WAVE>();
  return n_eval;
}

// ------------------------------------------------------------------------------------------------
// regrouping of live trajectories within a workgroup (FP64, one job)
// ------------------------------------------------------------------------------------------------
// Trajectories removed by the Kay test leave their lanes idle until the tile ends. A job created
// with regroup_every = E > 0 runs its tiles kRgWaves at a time: one workgroup of kRgWaves waves
// takes kRgWaves consecutive tiles that share their first birth step, the waves propagate their
// tiles independently up to the next multiple of E, and there the workgroup moves the group's
// live trajectories to the group's first slots (a stable partition: live slots in slot order,
// then the removed ones) so that ceil(live / 64) tiles continue and the waves of the others end.
// A trajectory's arithmetic does not depend on its lane, and the grouping after a boundary
// depends only on the removal steps, so results are reproducible bit for bit and do not depend on
// how propagation is split into launches (the boundaries are fixed steps of the grid). Only the
// per-step sums of a wave's queued integrands change with the grouping, at rounding level. No
// workgroup waits for another. Groups whose tiles do not share a first birth step run as
// kRgWaves independent tiles.
constexpr int kRgWaves = 4;

// moves the records of the group's slots so that slot i receives the record of slot src[i]
// (state, auxiliary values, birth and removal steps, caller index); every thread of the
// workgroup takes one slot, rows in blocks of kRgRows between barriers so that every read of a
// row precedes every write of it
constexpr int kRgRows = 8;

__device__ __forceinline__ void rg_move(const JobDev& J, long long base, int i, const int* src) {
  const long long np = J.n_pad;
  const long long from = base + src[i], to = base + i;
  for (int r0 = 0; r0 < kNY; r0 += kRgRows) {
    double v[kRgRows];
#pragma unroll
    for (int r = 0; r < kRgRows; ++r)
      if (r0 + r < kNY) v[r] = J.y[(r0 + r) * np + from];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRgRows; ++r)
      if (r0 + r < kNY) J.y[(r0 + r) * np + to] = v[r];
  }
  double a[5];
#pragma unroll
  for (int r = 0; r < 5; ++r) a[r] = J.aux[r * np + from];
  const int n0 = J.n0[from], death = J.death[from];
  const long long pm = J.perm[from];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 5; ++r) J.aux[r * np + to] = a[r];
  J.n0[to] = n0;
  J.death[to] = death;
  J.perm[to] = pm;
}

// The boundary at step nb of the group whose first tile is t0, called by the nw waves still in the
// workgroup (the tiles of the waves that have ended hold removed trajectories only) once every
// tile's state is stored: regroups the live trajectories into the first tiles and sets the tiles'
// progress. Returns the number of tiles that continue.
__device__ int rg_boundary(const JobDev& J, int t0, int nb, int nw, int* src, int* cnt) {
  const int i = threadIdx.x;
  const int w = uniform_i32(i >> 6);
  const long long base = (long long)t0 * kTile;
  const bool live = J.death[base + i] == -1;  // not removed (or not yet born)
  const unsigned long long m = __builtin_amdgcn_ballot_w64(live);
  if ((i & (kTile - 1)) == 0) cnt[w] = __popcll(m);
  __syncthreads();
  int before = 0, L = 0;
  for (int k = 0; k < nw; ++k) {
    before += k < w ? cnt[k] : 0;
    L += cnt[k];
  }
  const int live_before = before + lanes_below(m);
  const int dest = live ? live_before : L + (i - live_before);
  // whether any slot moves: per wave, then over the waves present (cnt[kRgWaves + k])
  const bool mv = __builtin_amdgcn_ballot_w64(dest != i) != 0ull;
  if ((i & (kTile - 1)) == 0) cnt[kRgWaves + w] = mv ? 1 : 0;
  __syncthreads();
  int moved = 0;
  for (int k = 0; k < nw; ++k) moved |= cnt[kRgWaves + k];
  if (moved) {
    src[dest] = i;
    __syncthreads();
    rg_move(J, base, i, src);
  }
  const int keep = (L + kTile - 1) / kTile;
  if ((i & (kTile - 1)) == 0) {
    if (w < keep) {
      J.tile_next[t0 + w] = nb;
      J.tile_last[t0 + w] = nb - 1;
    } else {
      J.tile_next[t0 + w] = J.n_steps + 1;
    }
  }
  __syncthreads();  // the moved records and the tiles' progress, before the next interval
  return keep;
}

// Regrouping state of a wave of a k_propagate_rg workgroup (see there): the next boundary step
// (INT_MAX: none), the interval, the group's first tile, the waves still in the workgroup, this
// wave's index, and the workgroup's LDS for the boundary.
struct RgWave {
  int nb, E, t0, nw, w;
  int* src;
  int* cnt;
};

// A removed lane's steps from the interval that began at `first_step` (its steps evaluated in
// [max(first_step, n0), removal step or last]) when it entered the interval as not removed.
__device__ __forceinline__ int lane_evals(int death_in, int death, int n0l, int first_step,
                                          int last) {
  if (death_in != -1) return 0;
  const int first = max(first_step, n0l);
  const int lastn = death >= 0 ? death : last;
  return max(0, lastn - first + 1);
}

// Propagates tile `tile` over steps n_begin..n_stop (n_begin <= n_stop <= n_steps; wave-uniform)
// and stores its state; returns the tile's next step, n_steps + 1 once every lane is removed or the
// grid's end is reached. KIND >= 0: the potential kind is a compile-time constant (its dispatch
// folds away); -1: read from the job descriptor at run time. ONE_WAVE: the workgroup is this wave.
// RG: the wave belongs to a regrouping workgroup (rg): at each boundary step inside the range the
// workgroup regroups its trajectories and the lanes continue with the trajectories then in their
// slots; returns -1 if the wave's tile was retired there (the wave must end).
template <int KIND, bool ONE_WAVE = true, bool RG = false>
__device__ __forceinline__ int run_tile_to(const JobDev& J, const int tile, const int n_begin,
                                           const int n_stop, IntegrandQueue& Q,
                                           RgWave* rg = nullptr) {
  const int lane = threadIdx.x & (kTile - 1);
  const int N = J.n_steps;
  const long long np = J.n_pad;
  const long long s = (long long)tile * kTile + lane;

  Traj T;
  const double* y = J.y;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T.q[i] = y[i * np + s];
    T.p[i] = y[(3 + i) * np + s];
  }
#pragma unroll
  for (int c = 0; c < 36; ++c) T.M[c] = y[(6 + c) * np + s];
  T.S = y[42 * np + s];
  cplx cprev = {J.aux[s], J.aux[np + s]};
  cplx w = {J.aux[2 * np + s], J.aux[3 * np + s]};
  double sgn = J.aux[4 * np + s];
  int n0l = J.n0[s];
  int death_in = J.death[s];
  int death = death_in;
  bool alive = death_in == -1;

  const const_dptr eh = (const_dptr)J.e_half;
  const PotParams P = J.pot;
  const int kind = KIND >= 0 ? KIND : J.kind;
  const double gamma = J.gamma, inv4g = J.inv4g, kay2 = J.kay2;
  const double h = J.h, h2 = J.h2, h6 = J.h6;
  const QueueCtx QC = queue_ctx(J);
  const double amin = J.gto.Amin, bmin = J.gto.Bmin, cut_hi = J.gto.cut_hi;

  int qn = 0;  // queued integrands (wave-uniform)
  unsigned int kay = 0, nonfin = 0, prims = 0;
  int ents = 0;  // queued integrand entries evaluated (wave-uniform)
  int evals = 0;           // RG: steps evaluated by this lane's trajectories of earlier intervals
  int first_step = n_begin;  // RG: the first step of the current interval
  int n = n_begin;
  double ea = eh[2 * n];
  for (; n <= n_stop; ++n) {
    if constexpr (RG) {
      if (n == rg->nb) {  // boundary: regroup with the other waves of the workgroup
        if (qn > 0) {
          ents += qn;
          prims += queue_eval<ONE_WAVE>(Q, qn, lane, QC);
          qn = 0;
        }
        // the arrays' addresses through volatile reads: computed here, not held in registers for
        // the whole step loop
        double* const yw = *(double* const volatile*)&J.y;
        double* const ax = *(double* const volatile*)&J.aux;
        int* const dt = *(int* const volatile*)&J.death;
        const int* const nz = *(int* const volatile*)&J.n0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          yw[i * np + s] = T.q[i];
          yw[(3 + i) * np + s] = T.p[i];
        }
#pragma unroll
        for (int c = 0; c < 36; ++c) yw[(6 + c) * np + s] = T.M[c];
        yw[42 * np + s] = T.S;
        ax[s] = cprev.re;
        ax[np + s] = cprev.im;
        ax[4 * np + s] = sgn;
        dt[s] = death;
        evals += lane_evals(death_in, death, n0l, first_step, n - 1);
        __syncthreads();  // every tile's state is stored
        rg->nw = rg_boundary(J, rg->t0, n, rg->nw, rg->src, rg->cnt);
        if (rg->w >= rg->nw) {  // this wave's tile is retired: count and end
          double ev = wave_sum((double)evals), ka = wave_sum((double)kay);
          double nf = wave_sum((double)nonfin), pr = wave_sum((double)prims);
          if (lane == 0) {
            atomicAdd(&J.counters[0], (unsigned long long)ev);
            atomicAdd(&J.counters[1], (unsigned long long)ka);
            atomicAdd(&J.counters[2], (unsigned long long)nf);
            atomicAdd(&J.counters[4], (unsigned long long)pr);
            atomicAdd(&J.counters[5], (unsigned long long)ents);
          }
          return -1;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          T.q[i] = yw[i * np + s];
          T.p[i] = yw[(3 + i) * np + s];
        }
#pragma unroll
        for (int c = 0; c < 36; ++c) T.M[c] = yw[(6 + c) * np + s];
        T.S = yw[42 * np + s];
        cprev = {ax[s], ax[np + s]};
        w = {ax[2 * np + s], ax[3 * np + s]};
        sgn = ax[4 * np + s];
        n0l = nz[s];
        death_in = dt[s];
        death = death_in;
        alive = death_in == -1;
        first_step = n;
        ea = eh[2 * n];
        rg->nb += rg->E;
      }
    }
    bool contrib = false;
    cplx C = {0.0, 0.0};
    if (alive && n >= n0l) {
      cplx d = hk_det(T.M, gamma, inv4g);
      double a2 = d.re * d.re;
      a2 = SFHK_FMA(d.im, d.im, a2);
      bool finite = isfinite(T.q[0]) && isfinite(T.q[1]) && isfinite(T.q[2]) &&
                    isfinite(T.p[0]) && isfinite(T.p[1]) && isfinite(T.p[2]) && isfinite(T.S);
      if (!(a2 <= kay2) || !finite) {  // Kay removal (or a non-finite state) from step n on
        alive = false;
        death = n;
        if (!finite || isnan(a2))
          ++nonfin;
        else
          ++kay;
      } else {
        cplx c = hk_sqrt(d, a2);
        double dot = SFHK_FMA(c.im, cprev.im, c.re * cprev.re);
        if (sgn * dot < 0.0) sgn = -sgn;
        C = {sgn * c.re, sgn * c.im};
        cprev = C;
        contrib = true;
      }
    }
    // dipole element: costly only for lanes near the ground state
    // |p|^2 and |q|^2 of the state at t_n: the skip bound below and the RK4's first stage use them
    const double p2 = norm2(T.p[0], T.p[1], T.p[2]);
    const double q2 = norm2(T.q[0], T.q[1], T.q[2]);
    const bool need = contrib && !overlap_all_skipped(amin, bmin, cut_hi, p2, q2);
    const unsigned long long m = __builtin_amdgcn_ballot_w64(need);
    if (m) {
      const int k = __popcll(m);
      if (qn + k > kQueue) {
        ents += qn;
        prims += queue_eval<ONE_WAVE>(Q, qn, lane, QC);
        qn = 0;
      }
      if (need)
        queue_push(Q, qn + lanes_below(m), T.q[0], T.q[1], T.q[2], T.p[0], T.p[1], T.p[2], T.S,
                   cmul(w, C), n);
      qn += k;
    }
    if (n < N) {
      const double eb = eh[2 * n + 1], ec = eh[2 * n + 2];
      if (alive && n >= n0l) rk4_step(kind, P, T, q2, p2, ea, eb, ec, h, h2, h6);
      ea = ec;
    }
    if (!__any(alive)) {  // every lane removed: the rest of the tile's row stays zero
      if constexpr (RG) {
        if (rg->nb <= n_stop) {  // idle to the next boundary, where the workgroup regroups
          n = rg->nb - 1;
          continue;
        }
      }
      ++n;
      break;
    }
  }
  if (qn > 0) {
    ents += qn;
    prims += queue_eval<ONE_WAVE>(Q, qn, lane, QC);
  }
  // n is now one past the last step processed
  double* yw = J.y;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    yw[i * np + s] = T.q[i];
    yw[(3 + i) * np + s] = T.p[i];
  }
#pragma unroll
  for (int c = 0; c < 36; ++c) yw[(6 + c) * np + s] = T.M[c];
  yw[42 * np + s] = T.S;
  J.aux[s] = cprev.re;
  J.aux[np + s] = cprev.im;
  J.aux[4 * np + s] = sgn;
  J.death[s] = death;
  const bool finished = !__any(alive) || n > N;
  const int next = finished ? N + 1 : n;
  if (lane == 0) {
    J.tile_next[tile] = next;
    J.tile_last[tile] = n - 1;
  }
  // steps evaluated by this lane in this call: from max(n_begin, n0) to its removal step or the
  // last step processed
  evals += lane_evals(death_in, death, n0l, first_step, n - 1);
  double ev = wave_sum((double)evals), ka = wave_sum((double)kay), nf = wave_sum((double)nonfin);
  double pr = wave_sum((double)prims);
  if (lane == 0) {
    atomicAdd(&J.counters[0], (unsigned long long)ev);
    atomicAdd(&J.counters[1], (unsigned long long)ka);
    atomicAdd(&J.counters[2], (unsigned long long)nf);
    atomicAdd(&J.counters[4], (unsigned long long)pr);
    atomicAdd(&J.counters[5], (unsigned long long)ents);
  }
  return next;
}

// one launch's share of a tile: max_steps steps (max_steps <= 0: to the end of the grid)
template <int KIND, bool ONE_WAVE = true>
__device__ __forceinline__ void run_tile(const JobDev& J, const int tile, const int max_steps,
                                         IntegrandQueue& Q) {
  const int n_begin = uniform_i32(J.tile_next[tile]);
  const int N = J.n_steps;
  if (n_begin > N) return;
  const int n_stop = (max_steps > 0) ? min(N, n_begin + max_steps - 1) : N;
  run_tile_to<KIND, ONE_WAVE>(J, tile, n_begin, n_stop, Q);
}

#ifndef SFHK_PROPAGATE_WAVES_PER_EU
#define SFHK_PROPAGATE_WAVES_PER_EU 2
#endif
template <int KIND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(SFHK_PROPAGATE_WAVES_PER_EU)))
void k_propagate_fp64(
    const JobDev* __restrict__ jobs, const WorkItem* __restrict__ work, int max_steps) {
  __shared__ IntegrandQueue Q;
  const WorkItem wi = work[blockIdx.x];
  run_tile<KIND>(jobs[wi.job], wi.tile, max_steps, Q);
}

// ------------------------------------------------------------------------------------------------
// propagation, mixed precision: q, p, M carried and integrated in FP32 away from the nucleus; the
// action, the HK square root and branch, the dipole integrand and the reduction in FP64; a lane
// whose step starts at r < r_fp64 takes the FP64 step on its exactly promoted state and rounds the
// result back to FP32. The precision decision is per lane, so a trajectory's result does not
// depend on the other trajectories of its wave.
// ------------------------------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ void run_tile_mixed(const JobDev& J, const int tile, const int max_steps,
                                               IntegrandQueue& Q) {
  const int lane = threadIdx.x;
  const int n_begin = uniform_i32(J.tile_next[tile]);
  const int N = J.n_steps;
  if (n_begin > N) return;
  const int n_stop = (max_steps > 0) ? min(N, n_begin + max_steps - 1) : N;
  const long long np = J.n_pad;
  const long long s = (long long)tile * kTile + lane;

  TrajF T;
  const double* y = J.y;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T.q[i] = (float)y[i * np + s];
    T.p[i] = (float)y[(3 + i) * np + s];
  }
#pragma unroll
  for (int c = 0; c < 36; ++c) T.M[c] = (float)y[(6 + c) * np + s];
  T.S = y[42 * np + s];
  cplx cprev = {J.aux[s], J.aux[np + s]};
  const cplx w = {J.aux[2 * np + s], J.aux[3 * np + s]};
  double sgn = J.aux[4 * np + s];
  const int n0l = J.n0[s];
  const int death_in = J.death[s];
  int death = death_in;
  bool alive = death_in == -1;

  const const_dptr eh = (const_dptr)J.e_half;
  const PotParams P = J.pot;
  const PotParamsF PF = {(float)P.z_inf, (float)P.z_in, (float)P.soft2, (float)P.omega_ho,
                         (float)P.inv_rscr};
  const int kind = KIND >= 0 ? KIND : J.kind;
  const double kay2 = J.kay2;
  const double h = J.h, h2 = J.h2, h6 = J.h6;
  const QueueCtx QC = queue_ctx(J);
  const float hf = (float)h, h2f = (float)h2, h6f = (float)h6;
  const float gammaf = (float)J.gamma, inv4gf = (float)J.inv4g;
  const float aminf = (float)J.gto.Amin, bminf = (float)J.gto.Bmin;
  const float cut_lo = (float)(J.cut * (1.0 + 1e-5));  // FP32 bound: margin for FP32 rounding
  const float r64sq = (float)J.r64sq;

  int qn = 0;  // queued integrands (wave-uniform)
  unsigned int kay = 0, nonfin = 0, prims = 0, steps64 = 0;
  int ents = 0;  // queued integrand entries evaluated (wave-uniform)
  int n = n_begin;
  double ea = eh[2 * n];
  for (; n <= n_stop; ++n) {
    bool contrib = false;
    cplx C = {0.0, 0.0};
    if (alive && n >= n0l) {
      cplx d = hk_det_f32(T.M, gammaf, inv4gf);
      double a2 = d.re * d.re;
      a2 = SFHK_FMA(d.im, d.im, a2);
      bool finite = isfinite(T.q[0]) && isfinite(T.q[1]) && isfinite(T.q[2]) &&
                    isfinite(T.p[0]) && isfinite(T.p[1]) && isfinite(T.p[2]) && isfinite(T.S);
      if (!(a2 <= kay2) || !finite) {
        alive = false;
        death = n;
        if (!finite || isnan(a2))
          ++nonfin;
        else
          ++kay;
      } else {
        cplx c = hk_sqrt(d, a2);
        double dot = SFHK_FMA(c.im, cprev.im, c.re * cprev.re);
        if (sgn * dot < 0.0) sgn = -sgn;
        C = {sgn * c.re, sgn * c.im};
        cprev = C;
        contrib = true;
      }
    }
    const float p2f = __builtin_fmaf(T.p[2], T.p[2], __builtin_fmaf(T.p[1], T.p[1], T.p[0] * T.p[0]));
    const float q2f = __builtin_fmaf(T.q[2], T.q[2], __builtin_fmaf(T.q[1], T.q[1], T.q[0] * T.q[0]));
    const bool need = contrib && !(__builtin_fmaf(p2f, aminf, q2f * bminf) > cut_lo);
    const unsigned long long m = __builtin_amdgcn_ballot_w64(need);
    if (m) {
      const int k = __popcll(m);
      if (qn + k > kQueue) {
        ents += qn;
        prims += queue_eval(Q, qn, lane, QC);
        qn = 0;
      }
      if (need)
        queue_push(Q, qn + lanes_below(m), T.q[0], T.q[1], T.q[2], T.p[0], T.p[1], T.p[2], T.S,
                   cmul(w, C), n);
      qn += k;
    }
    if (n < N) {
      const double eb = eh[2 * n + 1], ec = eh[2 * n + 2];
      if (alive && n >= n0l) {
        if (q2f < r64sq) {  // near the nucleus: the FP64 step on the promoted state
          Traj D;
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            D.q[i] = T.q[i];
            D.p[i] = T.p[i];
          }
#pragma unroll
          for (int c = 0; c < 36; ++c) D.M[c] = T.M[c];
          D.S = T.S;
          rk4_step(kind, P, D, ea, eb, ec, h, h2, h6);
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            T.q[i] = (float)D.q[i];
            T.p[i] = (float)D.p[i];
          }
#pragma unroll
          for (int c = 0; c < 36; ++c) T.M[c] = (float)D.M[c];
          T.S = D.S;
          ++steps64;
        } else {
          rk4_step_f32(kind, PF, T, (float)ea, (float)eb, (float)ec, hf, h2f, h6f, h6);
        }
      }
      ea = ec;
    }
    if (!__any(alive)) {
      ++n;
      break;
    }
  }
  if (qn > 0) {
    ents += qn;
    prims += queue_eval(Q, qn, lane, QC);
  }
  double* yw = J.y;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    yw[i * np + s] = T.q[i];
    yw[(3 + i) * np + s] = T.p[i];
  }
#pragma unroll
  for (int c = 0; c < 36; ++c) yw[(6 + c) * np + s] = T.M[c];
  yw[42 * np + s] = T.S;
  J.aux[s] = cprev.re;
  J.aux[np + s] = cprev.im;
  J.aux[4 * np + s] = sgn;
  J.death[s] = death;
  const bool finished = !__any(alive) || n > N;
  if (lane == 0) {
    J.tile_next[tile] = finished ? N + 1 : n;
    J.tile_last[tile] = n - 1;
  }
  int evals = 0;
  if (death_in == -1) {
    const int first = max(n_begin, n0l);
    const int lastn = death >= 0 ? death : n - 1;
    evals = max(0, lastn - first + 1);
  }
  double ev = wave_sum((double)evals), ka = wave_sum((double)kay), nf = wave_sum((double)nonfin);
  double pr = wave_sum((double)prims), s64 = wave_sum((double)steps64);
  if (lane == 0) {
    atomicAdd(&J.counters[0], (unsigned long long)ev);
    atomicAdd(&J.counters[1], (unsigned long long)ka);
    atomicAdd(&J.counters[2], (unsigned long long)nf);
    atomicAdd(&J.counters[3], (unsigned long long)s64);
    atomicAdd(&J.counters[4], (unsigned long long)pr);
    atomicAdd(&J.counters[5], (unsigned long long)ents);
  }
}

// Three waves per SIMD (168 VGPRs): the FP32 step's dependency chains leave the VALU idle at two
// waves, and the register allocation this forces moves 160-272 B per lane to scratch, mostly
// around the rarely taken FP64 step (screened workload 366 -> 326 ms; four waves: 360 ms).
#ifndef SFHK_MIXED_WAVES_PER_EU
#define SFHK_MIXED_WAVES_PER_EU 3
#endif
template <int KIND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(SFHK_MIXED_WAVES_PER_EU)))
void k_propagate_mixed(const JobDev* __restrict__ jobs, const WorkItem* __restrict__ work, int max_steps) {
  __shared__ IntegrandQueue Q;
  const WorkItem wi = work[blockIdx.x];
  run_tile_mixed<KIND>(jobs[wi.job], wi.tile, max_steps, Q);
}

// ------------------------------------------------------------------------------------------------
// persistent form (batched, graph-captured launches): a fixed number of single-wave workgroups pop
// tiles from a longest-first work list through one atomic counter per precision segment. The
// segment sizes live in device memory so the host can rewrite the job table between graph
// replays without capturing again.
// ------------------------------------------------------------------------------------------------
constexpr int kKinds = 4;              // potential kinds
constexpr int kSegs = 2 * kKinds;       // work-list segments: precision * kKinds + kind

struct BatchDev {
  int n_items[kSegs];        // per segment
  int offset[kSegs];         // first work item of the segment
  unsigned int next[kSegs];  // queue heads, zeroed at the start of every replay
};

__global__ void k_batch_reset(BatchDev* __restrict__ B) {
  if (threadIdx.x < kSegs) B->next[threadIdx.x] = 0u;
}

// one tile per call: inlined into the queue loop, the tile loop's register allocation degrades.
// The LDS queue is declared here, not passed in, so its accesses stay LDS instructions.
template <int PREC, int KIND>
__device__ __noinline__ void tile_call(const JobDev* J, int tile, int max_steps) {
  __shared__ IntegrandQueue Q;
  if (PREC == 0)
    run_tile<KIND>(*J, tile, max_steps, Q);
  else
    run_tile_mixed<KIND>(*J, tile, max_steps, Q);
}

template <int PREC, int KIND>
__device__ __forceinline__ void queue_loop(const JobDev* __restrict__ jobs, const WorkItem* __restrict__ work,
                                           BatchDev* __restrict__ B, int max_steps) {
  constexpr int seg = PREC * kKinds + KIND;
  const int n_items = B->n_items[seg];
  const WorkItem* sw = work + B->offset[seg];
  for (;;) {
    unsigned int it = 0;
    if (threadIdx.x == 0) it = atomicAdd(&B->next[seg], 1u);
    it = __shfl(it, 0, 64);
    if (it >= (unsigned int)n_items) break;  // every wave of the grid reaches this exit
    const WorkItem wi = sw[it];
    tile_call<PREC, KIND>(jobs + wi.job, wi.tile, max_steps);
  }
}

template <int KIND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(SFHK_PROPAGATE_WAVES_PER_EU)))
void k_queue_fp64(const JobDev* __restrict__ jobs, const WorkItem* __restrict__ work,
                  BatchDev* __restrict__ B, int max_steps) {
  queue_loop<0, KIND>(jobs, work, B, max_steps);
}

template <int KIND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(SFHK_MIXED_WAVES_PER_EU)))
void k_queue_mixed(const JobDev* __restrict__ jobs, const WorkItem* __restrict__ work,
                   BatchDev* __restrict__ B, int max_steps) {
  queue_loop<1, KIND>(jobs, work, B, max_steps);
}

// hardware-dispatch alternative for graph replays: one workgroup per work item of capacity;
// workgroups past the segment's current size exit at once
template <int KIND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(SFHK_PROPAGATE_WAVES_PER_EU)))
void k_grid_fp64(const JobDev* __restrict__ jobs, const WorkItem* __restrict__ work,
                 const BatchDev* __restrict__ B, int max_steps) {
  __shared__ IntegrandQueue Q;
  constexpr int seg = KIND;
  if ((int)blockIdx.x >= B->n_items[seg]) return;
  const WorkItem wi = work[B->offset[seg] + blockIdx.x];
  run_tile<KIND>(jobs[wi.job], wi.tile, max_steps, Q);
}

template <int KIND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(SFHK_MIXED_WAVES_PER_EU)))
void k_grid_mixed(const JobDev* __restrict__ jobs, const WorkItem* __restrict__ work,
                  const BatchDev* __restrict__ B, int max_steps) {
  __shared__ IntegrandQueue Q;
  constexpr int seg = kKinds + KIND;
  if ((int)blockIdx.x >= B->n_items[seg]) return;
  const WorkItem wi = work[B->offset[seg] + blockIdx.x];
  run_tile_mixed<KIND>(jobs[wi.job], wi.tile, max_steps, Q);
}

template <int KIND>
__global__ __launch_bounds__(kRgWaves * kTile) __attribute__((amdgpu_waves_per_eu(SFHK_PROPAGATE_WAVES_PER_EU)))
void k_propagate_rg(const JobDev* __restrict__ jobs, const WorkItem* __restrict__ work, int n_items,
                    int max_steps) {
  __shared__ IntegrandQueue Q[kRgWaves];
  __shared__ int src[kRgWaves * kTile];
  __shared__ int cnt[2 * kRgWaves];
  __shared__ int next[kRgWaves];
  __shared__ int group;  // the first tile of a group, else -1
  const int w = uniform_i32((int)threadIdx.x >> 6);
  const int lane = threadIdx.x & (kTile - 1);
  const long long k0 = (long long)blockIdx.x * kRgWaves;
  const long long k = k0 + w;
  const WorkItem wi = work[k < n_items ? k : k0];
  const JobDev& J = jobs[wi.job];
  const int N = J.n_steps;
  if (threadIdx.x == 0) {
    int g = k0 + kRgWaves <= n_items && J.compact_every > 0 ? work[k0].tile : -1;
    for (int u = 1; u < kRgWaves && g >= 0; ++u) {
      const WorkItem x = work[k0 + u];
      if (x.job != work[k0].job || x.tile != g + u || J.tile_n0[g + u] != J.tile_n0[g]) g = -1;
    }
    group = g;
  }
  if (lane == 0) next[w] = k < n_items ? J.tile_next[wi.tile] : N + 1;
  __syncthreads();
  const int t0 = uniform_i32(group);
  RgWave rg{INT_MAX, J.compact_every, t0, kRgWaves, w, src, cnt};
  int n;
  if (t0 >= 0) {  // a group: its running tiles share their next step
    n = N + 1;
    for (int u = 0; u < kRgWaves; ++u) n = min(n, next[u]);
    n = uniform_i32(n);
    if (n > N) return;  // the whole workgroup
    // the first boundary at or after n: a launch that starts on a boundary step regroups there
    // first, as a launch running through that step does at the top of its iteration
    rg.nb = (n + rg.E - 1) / rg.E * rg.E;
  } else {        // four independent tiles
    n = uniform_i32(next[w]);
    if (k >= n_items || n > N) return;
  }
  const int stop = max_steps > 0 ? min(N, n + max_steps - 1) : N;
  run_tile_to<KIND, false, true>(J, t0 >= 0 ? t0 + w : wi.tile, n, stop, Q[w], &rg);
}

}  // namespace
