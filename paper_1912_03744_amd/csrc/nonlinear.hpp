// nonlinear.hpp -- device side of the paper's method with temperature-dependent material
// laws: the simple (Picard) iteration of each Peaceman-Rachford half step
// (Sec. 3, eq. 12 and eq. 14) with the max-norm stop of eq. 13, step halving
// when an iteration does not stop within its limit (end of Sec. 3), the
// pulsed source of Sec. 2 (eq. 2-4) and the time loop of Sec. 4 (step size
// from the source's phase, periodic-regime stop).
//
// With laws that depend on T every line matrix changes with every iterate,
// so nothing is factored ahead of time: each iteration assembles the
// coefficients of its lines from the current iterate and solves them.  The
// whole time loop runs in one persistent cooperative launch (every
// workgroup resident, NW waves each):
//
//   * a workgroup takes one row of the r half step at a time (all its NW
//     waves on the row), a wave one column of the z half step (or the whole
//     workgroup, for columns longer than 16 cells per lane), stages the
//     line's iterate, current layer and explicit part in LDS, assembles the
//     tridiagonal row of every cell and solves the line by a partition
//     method computed on the fly: each lane eliminates a chunk of
//     consecutive cells (Thomas with two spike columns), the chunk-end
//     unknowns form a reduced tridiagonal system of one row per lane, solved
//     by parallel cyclic reduction over wavefront shuffles (and, across the
//     waves of a workgroup, through LDS), then the lane substitutes back;
//   * fields that other workgroups read are written and read through
//     device-coherent buffer accesses, so no workgroup has to write back
//     its L2 at a barrier, and the grid-wide barrier has two levels (groups
//     of workgroups, then the group leaders);
//   * the largest change |T^{s+1} - T^s| of each line is folded into one
//     device word per iteration by an atomic max (non-negative doubles order
//     like their bit patterns); after a grid-wide barrier every wave reads the
//     same word and takes the same decision (stop, iterate again, or give up
//     and halve the step);
//   * the explicit part of a half step (Lambda_z of T for eq. 12, Lambda_r of
//     T-bar plus the source for eq. 14) does not change over the iteration:
//     the first iteration computes it and keeps it in a field buffer;
//   * one lane of workgroup 0 runs the step control between attempts (time,
//     step size, counters, which buffer holds T), then a barrier publishes it.
//
// Every grid-wide wait is bounded: a wave that waits too long raises an abort
// flag that makes every other wave leave at its next wait, and the run
// reports the failure instead of hanging.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

// The step control must take the same decisions as a plain FP64 program
// evaluating the same expressions: no fused multiply-adds in this file.
#pragma clang fp contract(off)

namespace adi {
namespace nl {

constexpr int ITER_CAP = 64;   // largest iteration limit per half step
constexpr int MAX_M = 48;      // cells per lane: lines of up to 64 * 48 = 3072 cells
constexpr int MIN_M = 3;       // a chunk has a first, an interior and a last cell
constexpr long long SPIN_LIMIT = 1LL << 25;  // default bound of a grid-wide wait (about a second)
constexpr unsigned BAR_GROUPS = 8;           // first level of the grid barrier
constexpr int NW = 4;                        // waves per workgroup

// Temperature laws per region (0 cooler .. 4 terminal): cubic polynomials
// c0 + c1 T + c2 T^2 + c3 T^3 of the conductivity lambda, the volumetric heat
// capacity rho c_V and the source amplitude chi I^2 / S_C (eq. 1-2).
struct Laws {
  double lam[5][4], cap[5][4], src[5][4];
};

// Normalised periodic source p(t) (eq. 2): kind 0 constant 1, 1 rectangular
// pulse train (eq. 3), 2 erf-smoothed switching (eq. 4).
struct Pulse {
  int kind;
  double tper, tsrc, ttrs, xi, zeta;
};

enum RunStatus {
  RUNNING = 0,
  END_TIME = 1,      // t reached t_end
  END_PERIODIC = 2,  // the periodic-regime stop fired
  END_STEPS = 3,     // the step cap was reached
  END_SINGLE = 4,    // single-attempt mode finished its attempt
  FAIL_TAU = -1,     // halving took the step below tau_min
  FAIL_WAIT = -2     // a grid-wide wait ran out
};

// Device-resident state of a run.
struct Ctl {
  double t, t_end, tau, min_margin;
  double last_chg[2];          // change norm that decided each half of the last attempt
  long long steps, rejected, solves_r, solves_z, max_steps;
  int cur;                     // buffer holding T
  int status;
  int ends_period;             // the current step ends on a period start
  int last_it[2];              // solves of each half of the last attempt (-1 failed, 0 not run)
  int accepted;                // the last attempt was accepted
  unsigned bar_count, bar_gen;
  int abort;
  int pad;
  struct {
    unsigned count, gen;
    unsigned pad[30];   // one 128-byte line per group
  } bar_sub[8];
  // [attempt parity][half][iteration]: bits of the largest change
  unsigned long long chg[2][2][ITER_CAP];
  unsigned long long pchg;     // periodic-check change
};

struct Args {
  Params P;
  Geom g;
  Laws L;
  Pulse pulse;
  double* F[4];     // field buffers; F[cur] holds T
  double* E;        // explicit part of the current half step
  double* prev;     // field at the last period start (periodic stop)
  Ctl* ctl;
  double* log;      // per accepted step (t_before, tau, solves_r, solves_z), or null
  long long log_cap;
  double eps, tau_min, ptol, div_trs, div_src, guard;
  int iter_max;
  int single;       // one attempt at the given tau, no step rule
  int attempts;     // attempts in this launch
  int Mr, Gr, Mz, Gz;   // chunking: r lines over NW waves, z lines over wz waves
  int wz;               // waves per z line: 1 or NW
  long long spin_limit; // polls of a grid-wide wait before the run is aborted
};

// Device-scope accesses: coherent across XCDs without fences (see the
// coherence notes before grid_sync).  Field data goes through buffer loads and
// stores with the device-scope coherence bit (sc1), which the compiler
// schedules like ordinary memory operations; the step state and the
// barrier words through device-scope relaxed atomics.
constexpr int DEVICE_SCOPE = 0x10;     // cache policy: sc1
constexpr int RSRC_WORD3 = 0x00020000; // raw buffer, 32-bit data format (gfx9)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const double* p) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, 0, 0x7fffffff, RSRC_WORD3);
}
__device__ __forceinline__ double ldc(__amdgpu_buffer_rsrc_t r, long i) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(i * 8), 0, DEVICE_SCOPE));
}
__device__ __forceinline__ void stc(__amdgpu_buffer_rsrc_t r, long i, double v) {
  using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, (int)(i * 8), 0, DEVICE_SCOPE);
}
template <class T>
__device__ __forceinline__ T ald(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void ast(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------- physics --

__device__ __forceinline__ double law(const double* c, double T) { return c[0] + T * (c[1] + T * (c[2] + T * c[3])); }

// Sum over periods n >= 0 of the switch-on minus the switch-off term; periods
// that start after t contribute exactly 0 to eq. 3 and only the far erf tail to
// eq. 4, so the sum stops one period after the one containing t.
__device__ double pulse_at(const Pulse& p, double t) {
  if (p.kind == 0) return 1.0;
  const long last = (long)floor(t / p.tper) + 1;
  double s = 0.0;
  for (long n = 0; n <= last; ++n) {
    const double on = t - n * p.tper;          // time since the n-th switch-on
    const double off = t - n * p.tper - p.tsrc;  // since the n-th switch-off
    if (p.kind == 1)
      s += (on >= 0.0 ? 1.0 : 0.0) - (off >= 0.0 ? 1.0 : 0.0);
    else
      s += 0.5 * (erf(p.xi * (p.zeta * on / p.ttrs - 1.0)) - erf(p.xi * (p.zeta * off / p.ttrs - 1.0)));
  }
  return s;
}

__device__ __forceinline__ int region_at(const Geom& g, int i, int j) { return region_of(g.bet[j], g.kap[i]); }

// Operator of one direction at an active cell with the laws evaluated on a
// field F (eq. 10 for r, eq. 11 for z, balance form): Lambda T = lo T[-1] +
// up T[+1] + cc T + b, where cc = -(lo + up + films) and b the films'
// ambient part.  Fm, Fc, Fp: F at the previous, this and the next cell along
// the direction (ignored where no such cell couples).
struct Op {
  double lo, up, cc, b;
};

__device__ Op op_r(const Args& a, const Laws& L, int i, int j, int m, double Fm, double Fc, double Fp) {
  const Params& P = a.P;
  const Geom& g = a.g;
  Op o{0.0, 0.0, 0.0, 0.0};
  const double vol = g.rc[i] * g.dr[i];
  const double kc = law(L.lam[m], Fc);
  if (i > 0) {
    const int mw = region_at(g, i - 1, j);
    if (mw == MASKED) {
      const double f = g.rf[i] * film(g.dr[i], kc, P.h[3]);
      o.cc -= f / vol;
      o.b += f * P.tinf[3] / vol;
    } else {
      const double Tf = 0.5 * (Fm + Fc);
      o.lo = g.rf[i] * series2(g.dr[i - 1], law(L.lam[mw], Tf), g.dr[i], law(L.lam[m], Tf)) / vol;
      o.cc -= o.lo;
    }
  }
  const int me = i < P.nr - 1 ? region_at(g, i + 1, j) : MASKED;
  if (i == P.nr - 1 || me == MASKED) {
    const int cls = i == P.nr - 1 ? 1 : 3;
    const double f = g.rf[i + 1] * film(g.dr[i], kc, P.h[cls]);
    o.cc -= f / vol;
    o.b += f * P.tinf[cls] / vol;
  } else {
    const double Tf = 0.5 * (Fc + Fp);
    o.up = g.rf[i + 1] * series2(g.dr[i], law(L.lam[m], Tf), g.dr[i + 1], law(L.lam[me], Tf)) / vol;
    o.cc -= o.up;
  }
  return o;
}

__device__ Op op_z(const Args& a, const Laws& L, int i, int j, int m, double Fm, double Fc, double Fp) {
  const Params& P = a.P;
  const Geom& g = a.g;
  Op o{0.0, 0.0, 0.0, 0.0};
  const double dz = g.dz[j];
  const double kc = law(L.lam[m], Fc);
  const int ms = j > 0 ? region_at(g, i, j - 1) : MASKED;
  if (j == 0 || ms == MASKED) {
    const int cls = j == 0 ? 0 : 3;
    const double f = film(dz, kc, P.h[cls]);
    o.cc -= f / dz;
    o.b += f * P.tinf[cls] / dz;
  } else {
    const double Tf = 0.5 * (Fm + Fc);
    o.lo = series2(g.dz[j - 1], law(L.lam[ms], Tf), dz, law(L.lam[m], Tf)) / dz;
    o.cc -= o.lo;
  }
  const int mn = j < P.nz - 1 ? region_at(g, i, j + 1) : MASKED;
  if (j == P.nz - 1 || mn == MASKED) {
    const int cls = j == P.nz - 1 ? 2 : 3;
    const double f = film(dz, kc, P.h[cls]);
    o.cc -= f / dz;
    o.b += f * P.tinf[cls] / dz;
  } else {
    const double Tf = 0.5 * (Fc + Fp);
    o.up = series2(dz, law(L.lam[m], Tf), g.dz[j + 1], law(L.lam[mn], Tf)) / dz;
    o.cc -= o.up;
  }
  return o;
}

// Explicit part of a half step at cell (i, j) of field F (laws on F):
// dir 0 (eq. 12): Lambda_z[F]; dir 1 (eq. 14): Lambda_r[F] + X(F).
template <int dir>
__device__ double explicit_part(const Args& a, const Laws& L, int i, int j, const double* F, double pval) {
  const int nr = a.P.nr, nz = a.P.nz;
  const int m = region_at(a.g, i, j);
  if (m == MASKED) return 0.0;
  const long c = (long)j * nr + i;
  const __amdgpu_buffer_rsrc_t Fr = rsrc(F);
  const double Fc = ldc(Fr, c);
  if constexpr (dir == 0) {
    const double Fm = j > 0 ? ldc(Fr, c - nr) : 0.0, Fp = j < nz - 1 ? ldc(Fr, c + nr) : 0.0;
    const Op o = op_z(a, L, i, j, m, Fm, Fc, Fp);
    return o.cc * Fc + o.b + o.lo * Fm + o.up * Fp;
  } else {
    const double Fm = i > 0 ? ldc(Fr, c - 1) : 0.0, Fp = i < nr - 1 ? ldc(Fr, c + 1) : 0.0;
    const Op o = op_r(a, L, i, j, m, Fm, Fc, Fp);
    return o.cc * Fc + o.b + o.lo * Fm + o.up * Fp + law(L.src[m], Fc) * pval;
  }
}

// ------------------------------------------------- coherence and sync --
//
// Workgroups on different XCDs share the field buffers, and each XCD has its
// own L2.  A device-scope release fence would write back a whole L2, and
// every workgroup would issue one per barrier; instead every access to the
// shared buffers (the field buffers, the explicit part, the periodic
// reference, the published step state) is a device-scope relaxed atomic
// load or store, which is coherent across XCDs by itself, and the barrier
// only has to order each wave's accesses before its arrival: a wave-scope
// wait for its own outstanding memory operations (the workgroup barrier's
// release), then a device-scope atomic arrival.

// Order the lanes of one wave around LDS exchanges.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Grid-wide barrier over every workgroup of the launch, in two levels: the
// workgroups of each of 8 groups (by index) count on their group's word, the
// last of a group counts on the top word, and the last group releases every
// group's generation word, which its workgroups poll.  Returns false when
// the run was aborted: some wave polled more than `limit` times.  gen: this
// workgroup's count of passed barriers.
__device__ bool grid_sync(Ctl* c, unsigned nblocks, unsigned& gen, long long limit) {
  __syncthreads();  // every wave's device-scope accesses have completed
  __shared__ int ok_s;
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned g0 = gen;
    const unsigned ngroups = nblocks < BAR_GROUPS ? nblocks : BAR_GROUPS;
    const unsigned grp = blockIdx.x % ngroups;
    const unsigned members = (nblocks - grp + ngroups - 1) / ngroups;
    if (atomicAdd(&c->bar_sub[grp].count, 1u) == members - 1) {
      ast(&c->bar_sub[grp].count, 0u);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (atomicAdd(&c->bar_count, 1u) == ngroups - 1) {
        ast(&c->bar_count, 0u);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        for (unsigned q = 0; q < ngroups; ++q) ast(&c->bar_sub[q].gen, g0 + 1);
      }
    }
    long long spins = 0;
    while (ald(&c->bar_sub[grp].gen) == g0) {
      if (ald(&c->abort)) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      if (++spins > limit) {
        ast(&c->abort, 1);
        ok = 0;
        break;
      }
    }
    gen = g0 + 1;
    ok_s = ok;
  }
  __syncthreads();
  return ok_s != 0;
}

__device__ __forceinline__ unsigned long long as_bits(double x) { return (unsigned long long)__double_as_longlong(x); }
__device__ __forceinline__ double from_bits(unsigned long long b) { return __longlong_as_double((long long)b); }

// Largest of two values, NaN winning (a NaN change must never pass the stop
// rule).
__device__ __forceinline__ double nan_max(double x, double y) { return (x > y || x != x) ? x : y; }

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = nan_max(v, __shfl_xor(v, o));
  return v;
}

// -------------------------------------------------------- line solver --

// Solve one line of a half step with NWL waves (1 or NW): dir 0, row
// `line`, the line system of eq. 12 (iterate Ts, current layer Tc = T);
// dir 1, column `line`, that of eq. 14 (Tc = T-bar).  The rows are assembled
// on the fly from the staged iterate, current layer and explicit part (E,
// computed here on the first iteration); the line is solved by a partition
// method: lane k of the line's 64 NWL lanes eliminates chunk k of M
// consecutive cells by Thomas with two spike columns (responses to the
// chunk's first and last unknowns), the chunk-end unknowns form a reduced
// tridiagonal system of one row per lane, solved by parallel cyclic
// reduction (wavefront shuffles inside a wave, LDS across the waves of the
// line), then each lane substitutes back.  Writes the new iterate to out and
// returns the largest |x - Ts| over the line's active cells (the same value
// in every lane of the line).
//
// LDS (per line): ts[L + 2] (iterate with a zero cell before and after),
// tc[L] (current layer, then the eliminated right-hand side y', then the
// solution), ev[L] (explicit part, then the eliminated spike v'), cp[L]
// (eliminated super-diagonal c'), L = 64 NWL M, plus for NWL > 1 an
// exchange space of 4 x 64 NWL doubles.
template <int dir, int NWL>
__device__ double solve_line(const Args& a, const Laws& laws, int line, const double* Ts, const double* Tc, double* E,
                             double* out, bool first, double ta, double pval, double* lds) {
  const int nr = a.P.nr;
  const int n = dir == 0 ? a.P.nr : a.P.nz;
  const int M = dir == 0 ? a.Mr : a.Mz;
  const int G = dir == 0 ? a.Gr : a.Gz;
  constexpr int NL = 64 * NWL;                          // lanes of the line
  const int L = NL * M;
  double* ts = lds;
  double* tc = ts + L + 2;
  double* ev = tc + L;
  double* cp = ev + L;
  double* xch = cp + L;                                 // NWL > 1: 4 x NL exchange
  const int lane = NWL == 1 ? (threadIdx.x & 63) : (int)threadIdx.x;
  auto sync = [&]() {
    if constexpr (NWL == 1) wave_sync();
    else __syncthreads();
  };
  auto addr = [&](int e) -> long { return dir == 0 ? (long)line * nr + e : (long)e * nr + line; };
  const __amdgpu_buffer_rsrc_t Tsr = rsrc(Ts), Tcr = rsrc(Tc), Er = rsrc(E), Or = rsrc(out);
  // stage the line (lane-contiguous: coalesced along rows)
#pragma unroll 4
  for (int e = lane; e < L; e += NL) {
    double vs = 0.0, vc = 0.0, ve = 0.0;
    if (e < n) {
      const long c = addr(e);
      vs = ldc(Tsr, c);
      vc = ldc(Tcr, c);
      if (first) {
        if constexpr (dir == 0) ve = explicit_part<0>(a, laws, e, line, Tc, pval);
        else ve = explicit_part<1>(a, laws, line, e, Tc, pval);
        stc(Er, c, ve);
      } else {
        ve = ldc(Er, c);
      }
    }
    ts[e + 1] = vs;
    tc[e] = vc;
    ev[e] = ve;
  }
  if (lane == 0) {
    ts[0] = 0.0;
    ts[L + 1] = 0.0;
  }
  sync();

  // row p of the line: a x[p-1] + b x[p] + c x[p+1] = d; identity for cells
  // outside the domain and past the line's end
  auto row = [&](int p, double& ra, double& rb, double& rc, double& rd) {
    ra = 0.0; rb = 1.0; rc = 0.0; rd = 0.0;
    if (p >= n) return;
    const int i = dir == 0 ? p : line, j = dir == 0 ? line : p;
    const int m = region_at(a.g, i, j);
    if (m == MASKED) return;
    const double s = ts[p + 1];
    Op o;
    if constexpr (dir == 0) o = op_r(a, laws, i, j, m, ts[p], s, ts[p + 2]);
    else o = op_z(a, laws, i, j, m, ts[p], s, ts[p + 2]);
    // eq. 12: rho c_V and the source at the iterate; eq. 14: rho c_V at T-bar
    const double C = law(laws.cap[m], dir == 0 ? s : tc[p]) / ta;
    ra = -o.lo;
    rb = C - o.cc;
    rc = -o.up;
    rd = C * tc[p] + ev[p];
    if constexpr (dir == 0) rd += law(laws.src[m], s) * pval;
    rd += o.b;
  };

  // chunk of this lane: cells k M .. k M + M - 1.  One pass over the chunk:
  // the first and last rows are kept, the interior rows 1 .. M-2 are
  // eliminated by Thomas with the first unknown's column (v') on the right;
  // the last interior row's super-diagonal goes to the last unknown's column
  // (w')
  const int p0 = lane * M;
  const int pl = p0 + M - 1;
  double a0 = 0.0, b0 = 1.0, c0 = 0.0, d0 = 0.0;   // first row
  double aL = 0.0, bL = 1.0, cL = 0.0, dL = 0.0;   // last row
  double cprev = 0.0, yprev = 0.0, vprev = 0.0, wlast = 0.0;
#pragma unroll 1
  for (int t = 0; t < M; ++t) {
    const int p = p0 + t;
    double ra, rb, rc, rd;
    row(p, ra, rb, rc, rd);
    if (t == 0) {
      a0 = ra; b0 = rb; c0 = rc; d0 = rd;
    } else if (t == M - 1) {
      aL = ra; bL = rb; cL = rc; dL = rd;
    } else {
      const double inv = 1.0 / (rb - ra * cprev);
      const double y = (rd - ra * yprev) * inv;
      const double v = (t == 1 ? -ra : -ra * vprev) * inv;
      double cq = rc * inv;
      if (t == M - 2) {
        wlast = -cq;
        cq = 0.0;
      }
      tc[p] = y;
      ev[p] = v;
      cp[p] = cq;
      cprev = cq;
      yprev = y;
      vprev = v;
    }
  }
  // responses of the first interior cell to the chunk's data (y1), first
  // unknown (v1) and last unknown (w1)
  const int pi = p0 + M - 2;
  double y1 = tc[pi], v1 = ev[pi], w1 = wlast;
#pragma unroll 1
  for (int t = M - 3; t >= 1; --t) {
    const int p = p0 + t;
    const double cq = cp[p];
    y1 = tc[p] - cq * y1;
    v1 = ev[p] - cq * v1;
    w1 = -cq * w1;
  }
  const double yl = tc[pi], vl = ev[pi], wl = wlast;
  // reduced rows: first cell s, last cell e of chunk k
  //   a0 x_e(k-1) + (b0 + c0 v1) x_s + c0 w1 x_e = d0 - c0 y1
  //   aL vl x_s + (bL + aL wl) x_e + cL x_s(k+1) = dL - aL yl
  const double BS = b0 + c0 * v1;
  const double qA = a0 / BS, qC = c0 * w1 / BS, qR = (d0 - c0 * y1) / BS;
  const double AE = aL * vl, BE = bL + aL * wl, RE = dL - aL * yl;
  // the next chunk's first-row terms (lane k + 1)
  double nA, nC, nR;
  {
    const double sA = __shfl_down(qA, 1), sC = __shfl_down(qC, 1), sR = __shfl_down(qR, 1);
    nA = sA;
    nC = sC;
    nR = sR;
    if constexpr (NWL > 1) {
      xch[lane] = qA;
      xch[NL + lane] = qC;
      xch[2 * NL + lane] = qR;
      __syncthreads();
      if ((lane & 63) == 63 && lane + 1 < NL) {
        nA = xch[lane + 1];
        nC = xch[NL + lane + 1];
        nR = xch[2 * NL + lane + 1];
      }
      __syncthreads();
    }
  }
  // eliminate every x_s: one row per lane in the chunk-end unknowns x_e
  double al = -AE * qA;
  double be = BE - AE * qC - cL * nA;
  double ga = -cL * nC;
  double de = RE - AE * qR - cL * nR;
  // parallel cyclic reduction: strides below 64 by shuffles inside the wave
  // (every lane takes part in every shuffle), larger strides through LDS
#pragma unroll 1
  for (int s = 1; s < G && s < 64; s <<= 1) {
    const int wl_ = lane & 63;
    const bool hasm = lane >= s, hasp = lane + s < G;
    const double am = __shfl_up(al, s), bm = __shfl_up(be, s), gm = __shfl_up(ga, s), dm = __shfl_up(de, s);
    const double ap = __shfl_down(al, s), bp = __shfl_down(be, s), gp = __shfl_down(ga, s), dp = __shfl_down(de, s);
    // across the wave boundary (NWL > 1) the partner sits in another wave:
    // its values come from LDS below
    double Am = am, Bm = bm, Gm = gm, Dm = dm, Ap = ap, Bp = bp, Gp = gp, Dp = dp;
    if constexpr (NWL > 1) {
      xch[lane] = al;
      xch[NL + lane] = be;
      xch[2 * NL + lane] = ga;
      xch[3 * NL + lane] = de;
      __syncthreads();
      if (hasm && wl_ < s) {
        Am = xch[lane - s]; Bm = xch[NL + lane - s]; Gm = xch[2 * NL + lane - s]; Dm = xch[3 * NL + lane - s];
      }
      if (hasp && wl_ + s >= 64) {
        Ap = xch[lane + s]; Bp = xch[NL + lane + s]; Gp = xch[2 * NL + lane + s]; Dp = xch[3 * NL + lane + s];
      }
      __syncthreads();
    }
    const double k1 = hasm ? al / Bm : 0.0;
    const double k2 = hasp ? ga / Bp : 0.0;
    const double nal = hasm ? -Am * k1 : 0.0;
    const double nga = hasp ? -Gp * k2 : 0.0;
    const double nbe = be - (hasm ? Gm * k1 : 0.0) - (hasp ? Ap * k2 : 0.0);
    const double nde = de - (hasm ? Dm * k1 : 0.0) - (hasp ? Dp * k2 : 0.0);
    al = nal;
    be = nbe;
    ga = nga;
    de = nde;
  }
  if constexpr (NWL > 1) {
#pragma unroll 1
    for (int s = 64; s < G; s <<= 1) {
      const bool hasm = lane >= s, hasp = lane + s < G;
      xch[lane] = al;
      xch[NL + lane] = be;
      xch[2 * NL + lane] = ga;
      xch[3 * NL + lane] = de;
      __syncthreads();
      const double Am = hasm ? xch[lane - s] : 0.0, Bm = hasm ? xch[NL + lane - s] : 1.0;
      const double Gm = hasm ? xch[2 * NL + lane - s] : 0.0, Dm = hasm ? xch[3 * NL + lane - s] : 0.0;
      const double Ap = hasp ? xch[lane + s] : 0.0, Bp = hasp ? xch[NL + lane + s] : 1.0;
      const double Gp = hasp ? xch[2 * NL + lane + s] : 0.0, Dp = hasp ? xch[3 * NL + lane + s] : 0.0;
      __syncthreads();
      const double k1 = hasm ? al / Bm : 0.0;
      const double k2 = hasp ? ga / Bp : 0.0;
      const double nal = hasm ? -Am * k1 : 0.0;
      const double nga = hasp ? -Gp * k2 : 0.0;
      const double nbe = be - (hasm ? Gm * k1 : 0.0) - (hasp ? Ap * k2 : 0.0);
      const double nde = de - (hasm ? Dm * k1 : 0.0) - (hasp ? Dp * k2 : 0.0);
      al = nal;
      be = nbe;
      ga = nga;
      de = nde;
    }
  }
  const double xe = lane < G ? de / be : 0.0;
  // the previous chunk's last unknown (lane k - 1)
  double xe_prev;
  {
    const double up = __shfl_up(xe, 1);  // every lane takes part in the shuffle
    xe_prev = (lane & 63) > 0 ? up : 0.0;
    if constexpr (NWL > 1) {
      xch[lane] = xe;
      __syncthreads();
      if ((lane & 63) == 0 && lane > 0) xe_prev = xch[lane - 1];
      __syncthreads();
    }
  }
  const double xs = qR - qA * xe_prev - qC * xe;
  // back substitution into the chunk; largest change over active cells
  // (identity rows outside the domain keep 0, and the iterate is 0 there:
  // they never change)
  double dmax = 0.0;
  if (pl < n) dmax = fabs(xe - ts[pl + 1]);
  tc[pl] = xe;
  double x = xe;
#pragma unroll 1
  for (int t = M - 2; t >= 1; --t) {
    const int p = p0 + t;
    x = t == M - 2 ? tc[p] + ev[p] * xs + wl * xe : tc[p] + ev[p] * xs - cp[p] * x;
    if (p < n) dmax = nan_max(dmax, fabs(x - ts[p + 1]));
    tc[p] = x;
  }
  if (p0 < n) dmax = nan_max(dmax, fabs(xs - ts[p0 + 1]));
  tc[p0] = xs;
  sync();
#pragma unroll 4
  for (int e = lane; e < n; e += NL) stc(Or, addr(e), tc[e]);
  dmax = wave_max(dmax);
  if constexpr (NWL > 1) {
    if ((lane & 63) == 0) xch[lane >> 6] = dmax;
    __syncthreads();
    for (int q = 0; q < NWL; ++q) dmax = nan_max(dmax, xch[q]);
    __syncthreads();
  } else {
    sync();
  }
  return dmax;
}

// ------------------------------------------------------- step control --

// Inside a transition of the source: the first t_trs after a switch-on or a
// switch-off.
__device__ bool in_transition(const Pulse& p, double t) {
  const double ph = t - floor(t / p.tper) * p.tper;
  return ph < p.ttrs || (ph >= p.tsrc && ph < p.tsrc + p.ttrs);
}

// First switch point or transition end later than t + guard, over the period
// of t and the next one.
__device__ double next_switch(const Pulse& p, double t, double guard) {
  const double n0 = floor(t / p.tper);
  double best = INFINITY;
  for (int k = 0; k < 2; ++k) {
    const double base = (n0 + k) * p.tper;
    const double cand[4] = {base, base + p.ttrs, base + p.tsrc, base + p.tsrc + p.ttrs};
    for (int q = 0; q < 4; ++q)
      if (cand[q] > t + guard && cand[q] < best) best = cand[q];
  }
  return best;
}

// Size of the next step from time t (the rule of Sec. 4: t_trs/div_trs in a
// transition, t_src/div_src elsewhere, never across a switch point or
// transition end, never past t_end), or the end of the run (status).
__device__ void begin_step(const Args& a, double t, long long steps, long long max_steps, double t_end,
                           double& tau_out, int& ends_out, int& status) {
  if (steps >= max_steps) {
    status = END_STEPS;
    return;
  }
  if (!(t_end - t > a.guard)) {
    status = END_TIME;
    return;
  }
  const Pulse& p = a.pulse;
  double tau = (p.kind != 0 && in_transition(p, t + a.guard)) ? p.ttrs / a.div_trs : p.tsrc / a.div_src;
  int ends = 0;
  if (p.kind != 0) {
    const double b = next_switch(p, t, a.guard);
    if (b - t <= tau) {
      tau = b - t;
      const double k = floor(b / p.tper + 0.5);
      ends = fabs(b - k * p.tper) <= a.guard;
    }
  }
  if (t_end - t < tau) {
    tau = t_end - t;
    ends = 0;
  }
  tau_out = tau;
  ends_out = ends;
}

__device__ void note_margin(Ctl* c, double chg, double bound) {
  const double mg = fabs(chg - bound) / bound;
  if (mg < c->min_margin) c->min_margin = mg;
}

// ------------------------------------------------------------- kernel --

// Dynamic LDS of a workgroup (doubles): an r line over the whole workgroup
// (4 staged arrays of 64 NW Mr cells, 2 halo cells, 4 x 64 NW exchange), z
// lines one wave each (NW slices of 4 x 64 Mz + 2) or over the whole
// workgroup.
__host__ __device__ inline size_t nl_lds_doubles(int Mr, int Mz, int wz) {
  const size_t r = 4 * (size_t)(64 * NW) * Mr + 2 + 4 * (size_t)(64 * NW);
  const size_t z = wz == 1 ? (size_t)NW * (4 * 64 * (size_t)Mz + 2)
                           : 4 * (size_t)(64 * NW) * Mz + 2 + 4 * (size_t)(64 * NW);
  return r > z ? r : z;
}

// The two buffer indices (of 0..3) other than x and y (the two lowest other
// than x when x == y).
__device__ __forceinline__ void other_two(int x, int y, int& u, int& v) {
  u = -1;
  v = -1;
  for (int q = 0; q < 4; ++q)
    if (q != x && q != y) {
      if (u < 0) u = q;
      else if (v < 0) v = q;
    }
}

// Step state every workgroup reads at the start of an attempt, published by
// workgroup 0 with device-scope stores.
__device__ __forceinline__ void publish(Ctl* c, double t, double tau, int cur, long long steps, long long rej,
                                        int ends, int status) {
  ast(&c->t, t);
  ast(&c->tau, tau);
  ast(&c->cur, cur);
  ast(&c->steps, steps);
  ast(&c->rejected, rej);
  ast(&c->ends_period, ends);
  ast(&c->status, status);
}

__global__ void __launch_bounds__(64 * NW) k_nl_run(Args a) {
  HIP_DYNAMIC_SHARED(double, lds_all)
  __shared__ Laws laws;
  for (int q = threadIdx.x; q < 60; q += blockDim.x) (&laws.lam[0][0])[q] = (&a.L.lam[0][0])[q];
  __syncthreads();
  Ctl* c = a.ctl;
  const unsigned nb = gridDim.x;
  const int wv = threadIdx.x >> 6;
  const int w = blockIdx.x * NW + wv;             // this wave
  const int nw = (int)nb * NW;                    // waves in the grid
  // LDS: an r line uses the workgroup's whole space; z lines one slice per
  // wave when a wave takes a line alone
  double* lds_z = a.wz == 1 ? lds_all + (size_t)wv * (4 * 64 * a.Mz + 2) : lds_all;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  unsigned gen = 0;
  if (threadIdx.x == 0) gen = ald(&c->bar_sub[0].gen);
  for (int att = 0; att < a.attempts; ++att) {
    if (ald(&c->status) != RUNNING) break;
    const long long steps0 = ald(&c->steps), rej0 = ald(&c->rejected);
    const long long par = (steps0 + rej0) & 1;
    const double t = ald(&c->t), tau = ald(&c->tau), ta = 0.5 * tau;
    const int cur = ald(&c->cur);
    const bool ends_period = ald(&c->ends_period) != 0;  // this step lands on a period start
    const double pval = pulse_at(a.pulse, t + 0.5 * tau);
    // half step 1 (eq. 12): lines along r, iterate from T
    int in = cur, A0, A1, bar = -1, it_r = -1, it_z = 0;
    other_two(cur, cur, A0, A1);
    double chg_r = 0.0, chg_z = 0.0;
    for (int s = 0; s < a.iter_max; ++s) {
      const int o = (s & 1) ? A1 : A0;
      double lmax = 0.0;
      for (int j = blockIdx.x; j < a.P.nz; j += nb)
        lmax = nan_max(lmax, solve_line<0, NW>(a, laws, j, a.F[in], a.F[cur], a.E, a.F[o], s == 0, ta, pval, lds_all));
      if (threadIdx.x == 0 && !(lmax <= 0.0)) atomicMax(&c->chg[par][0][s], as_bits(lmax));
      if (!grid_sync(c, nb, gen, a.spin_limit)) return;
      chg_r = from_bits(ald(&c->chg[par][0][s]));
      in = o;
      if (chg_r < a.eps) {
        bar = o;
        it_r = s + 1;
        break;
      }
    }
    if (bar >= 0) {
      // half step 2 (eq. 14): lines along z, iterate from T-bar; T stays
      // untouched so that a failed attempt can restart from it
      int B0, B1;
      other_two(cur, bar, B0, B1);
      in = bar;
      it_z = -1;
      for (int s = 0; s < a.iter_max; ++s) {
        const int o = (s & 1) ? B1 : B0;
        double lmax = 0.0;
        if (a.wz == 1) {
          for (int i = w; i < a.P.nr; i += nw)
            lmax = nan_max(lmax, solve_line<1, 1>(a, laws, i, a.F[in], a.F[bar], a.E, a.F[o], s == 0, ta, pval, lds_z));
          if ((threadIdx.x & 63) == 0 && !(lmax <= 0.0)) atomicMax(&c->chg[par][1][s], as_bits(lmax));
        } else {
          for (int i = blockIdx.x; i < a.P.nr; i += nb)
            lmax = nan_max(lmax, solve_line<1, NW>(a, laws, i, a.F[in], a.F[bar], a.E, a.F[o], s == 0, ta, pval,
                                                   lds_all));
          if (threadIdx.x == 0 && !(lmax <= 0.0)) atomicMax(&c->chg[par][1][s], as_bits(lmax));
        }
        if (!grid_sync(c, nb, gen, a.spin_limit)) return;
        chg_z = from_bits(ald(&c->chg[par][1][s]));
        in = o;
        if (chg_z < a.eps) {
          it_z = s + 1;
          break;
        }
      }
    }
    const bool ok = bar >= 0 && it_z > 0;
    // step control (one lane).  The fields only this lane reads (counters,
    // margins, the log, the last attempt's record) are plain; the next
    // attempt's change words are cleared here: every wave read them before
    // the barrier that ended that attempt's last iteration
    if (lead) {
      for (int h = 0; h < 2; ++h)
        for (int s = 0; s < ITER_CAP; ++s) ast(&c->chg[par ^ 1][h][s], 0ull);
      c->last_it[0] = it_r;
      c->last_it[1] = it_z;
      c->last_chg[0] = chg_r;
      c->last_chg[1] = chg_z;
      note_margin(c, chg_r, a.eps);
      if (bar >= 0) note_margin(c, chg_z, a.eps);
      c->accepted = ok;
      double nt = t, ntau = tau;
      int ncur = cur, nends = ends_period, status = RUNNING;
      long long nsteps = steps0, nrej = rej0;
      if (ok) {
        if (a.log && steps0 < a.log_cap) {
          double* r = a.log + 4 * steps0;
          r[0] = t;
          r[1] = tau;
          r[2] = it_r;
          r[3] = it_z;
        }
        nt = t + tau;
        nsteps += 1;
        c->solves_r += it_r;
        c->solves_z += it_z;
        ncur = in;
        ast(&c->pchg, 0ull);
      } else {
        nrej += 1;
      }
      if (a.single) {
        status = END_SINGLE;
      } else if (!ok) {
        ntau = 0.5 * tau;
        nends = 0;
        if (ntau < a.tau_min) status = FAIL_TAU;
      } else if (!(ends_period && a.ptol > 0.0)) {
        begin_step(a, nt, nsteps, c->max_steps, c->t_end, ntau, nends, status);
      }
      publish(c, nt, ntau, ncur, nsteps, nrej, nends, status);
    }
    if (!grid_sync(c, nb, gen, a.spin_limit)) return;
    // periodic regime: at a period start, compare T with the field of the
    // previous period start
    if (ok && !a.single && ends_period && a.ptol > 0.0) {
      const long n = (long)a.P.nr * a.P.nz;
      const __amdgpu_buffer_rsrc_t Tr = rsrc(a.F[ald(&c->cur)]), Pr = rsrc(a.prev);
      double lmax = 0.0;
      for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)nb * blockDim.x) {
        const double v = ldc(Tr, e);
        if (region_at(a.g, (int)(e % a.P.nr), (int)(e / a.P.nr)) != MASKED) lmax = nan_max(lmax, fabs(v - ldc(Pr, e)));
        stc(Pr, e, v);
      }
      lmax = wave_max(lmax);
      if ((threadIdx.x & 63) == 0 && !(lmax <= 0.0)) atomicMax(&c->pchg, as_bits(lmax));
      if (!grid_sync(c, nb, gen, a.spin_limit)) return;
      if (lead) {
        const double d = from_bits(ald(&c->pchg));
        note_margin(c, d, a.ptol);
        double nt = ald(&c->t), ntau = ald(&c->tau);
        int nends = 0, status = RUNNING;
        const long long nsteps = ald(&c->steps);
        if (d < a.ptol) status = END_PERIODIC;
        else begin_step(a, nt, nsteps, c->max_steps, c->t_end, ntau, nends, status);
        publish(c, nt, ntau, ald(&c->cur), nsteps, ald(&c->rejected), nends, status);
      }
      if (!grid_sync(c, nb, gen, a.spin_limit)) return;
    }
  }
}

// Set up the first step of a run (one lane).
__global__ void k_nl_begin(Args a) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    Ctl* c = a.ctl;
    double tau = c->tau;
    int ends = 0, status = RUNNING;
    begin_step(a, c->t, c->steps, c->max_steps, c->t_end, tau, ends, status);
    publish(c, c->t, tau, c->cur, c->steps, c->rejected, ends, status);
  }
}

__global__ void k_nl_copy(const double* __restrict__ src, double* __restrict__ dst, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) dst[e] = src[e];
}

}  // namespace nl
}  // namespace adi
