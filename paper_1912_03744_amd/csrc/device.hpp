// device.hpp -- device-side building blocks of the ADI solver for gfx950.
//
// Method (Ayriyan & Busa, arXiv 1912.03744): the axisymmetric heat equation
// (Sec. 2, eq. 1) with piecewise-constant coefficients on the L-shaped
// layered domain of Fig. 1, discretised on the cell-centred grid of eq. 7
// with the conservative operators of eq. 10-11 (balance form, harmonic face
// conductivity) and advanced by Peaceman-Rachford half steps (eq. 8-9) or by
// the locally one-dimensional backward-Euler splitting.  Each half step is a
// set of independent tridiagonal line systems, solved here instead of by the
// paper's sequential Thomas recurrence (end of Sec. 3) by a partition method
// that maps one line onto many GPU lanes:
//
//   * a line of n cells is cut into G chunks of M consecutive cells (G*M >= n,
//     extra cells are identity rows);
//   * every lane eliminates the interior rows of its chunk with precomputed
//     Thomas factors, which expresses the interior through the chunk's first
//     and last unknowns via two precomputed "spike" vectors;
//   * the 2G chunk-end unknowns satisfy a tridiagonal "reduced" system whose
//     Thomas recurrences are first-order linear recurrences over the chunks;
//     they are evaluated by recursive doubling (Kogge-Stone) with wavefront
//     shuffles inside a wave and a carry pass through LDS across waves;
//   * back substitution into the interior.
//
// With constant coefficients every line of a class (an r-row band or a
// z-column class) has the same matrix, so all factors -- interior pivots,
// spikes, reduced-system factors and the products the doubling steps need --
// are computed once per (time step, materials) by assemble_class() and the
// sweeps read only the right-hand side.  Each sweep also produces the
// right-hand side of the following half step, using the same-direction
// operator on the freshly solved line, so no halo rows are read.

#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adi {

constexpr uint8_t MASKED = 255;

// ------------------------------------------------------------ descriptors --

// Problem parameters of one instance as the device sees them.
struct Params {
  double r0, r1, r2, rmax, z0, zmax, ztop;
  double h[4], tinf[4];
  double k[5], rhoc[5], q[5];
  double ta;      // implicit weight: tau/2 (PR) or tau (LOD-BE)
  double theta;   // 1 (PR): explicit other-direction terms present; 0 (LOD-BE)
  int nr, nz;
};

// Geometry arrays of one instance (device pointers).
struct Geom {
  double *rf, *zf;   // faces, nr+1 / nz+1
  double *rc, *zc;   // centres
  double *dr, *dz;   // widths
  uint8_t *kap;      // column class per r position (0..3, by r_c against r0/r1/r2)
  uint8_t *bet;      // band per z position (0: z<z0, 1: z0<=z<zmax, 2: terminal)
};

// Per-position fields of a line-class table, chunk-interleaved: the value for
// chunk k, offset t lives at [field][t*G + k].
enum PosField {
  P_W = 0,   // inverse interior pivot
  P_QA,      // sub-diagonal times inverse pivot
  P_CP,      // eliminated super-diagonal
  P_SP,      // spike: response of the interior to the chunk's first unknown
  P_SR,      // spike: response to the chunk's last unknown
  P_OD,      // output operator: diagonal
  P_OL,      //   lower neighbour
  P_OU,      //   upper neighbour
  P_OC,      //   constant
  P_NFIELDS
};

constexpr int MAX_LEV = 6;  // log2(64): chunks per wave

// Per-chunk fields.
enum ChkField {
  C_CS = 0,  // super-diagonal of the chunk's first row
  C_AE,      // sub-diagonal of the chunk's last row
  C_W0, C_Q0, C_C0,   // reduced-system Thomas factors of row 2k
  C_W1, C_Q1, C_C1,   // ... of row 2k+1
  C_CPREV,   // C of row 2k-1
  C_BPRE,    // prefix product of the forward coefficients within the wave
  C_ESUF,    // suffix product of the backward coefficients within the wave
  C_KSF,     // MAX_LEV forward doubling coefficients
  C_KSB = C_KSF + MAX_LEV,  // MAX_LEV backward doubling coefficients
  C_NFIELDS = C_KSB + MAX_LEV
};

// One line class in one direction.
struct LineTab {
  const double* pos;   // [P_NFIELDS][G*M]
  const double* chk;   // [C_NFIELDS][G]
  int n, G, M;         // line length, chunks, cells per chunk
  int skip_lo, skip_hi;  // positions [skip_lo, skip_hi) are outside the domain
};

// Arguments of one sweep (one direction of one instance).
struct SweepArgs {
  const double* din;      // right-hand side of this half step
  double* dout;           // right-hand side of the next half step
  double* xout;           // solution of this half step, or null
  const LineTab* tabs;    // line-class tables of this direction
  const uint8_t* line_class;  // class of every line
  const uint8_t* pos_xclass;  // class of the crossing line at every position
  const double* xc;       // [xclass][line] constant of the other direction, or null
  long line_stride, pos_stride;
  int nlines, ngroups;
};

// ---------------------------------------------------------------- regions --

__device__ __forceinline__ int column_class(const Params& P, double rc) {
  return rc < P.r0 ? 0 : (rc < P.r1 ? 1 : (rc < P.r2 ? 2 : 3));
}
__device__ __forceinline__ int row_band(const Params& P, double zc) {
  return zc >= P.zmax ? 2 : (zc >= P.z0 ? 1 : 0);
}
// Region of a cell from its row band and column class: the centre rule
// z >= zmax -> terminal; r < r0 -> cooler; z >= z0 -> outside; else by r.
__device__ __forceinline__ int region_of(int band, int cls) {
  if (band == 2) return 4;
  if (cls == 0) return 0;
  if (band == 1) return MASKED;
  return cls;
}

// Grid of eq. 7 for one axis: faces, centres, widths.  Uniform grids use the
// exact expressions length*i/n and (i+0.5)*length/n.
__device__ __forceinline__ void axis_point(int i, int n, double length, const double* faces_in,
                                           double* f, double* c, double* d) {
  double f0, f1, cc;
  if (faces_in) {
    f0 = faces_in[i];
    f1 = faces_in[i + 1];
    cc = 0.5 * (f0 + f1);
  } else {
    f0 = length * i / n;
    f1 = length * (i + 1) / n;
    cc = (i + 0.5) * length / n;
  }
  f[i] = f0;
  if (i == n - 1) f[n] = f1;
  c[i] = cc;
  d[i] = f1 - f0;
}

// Fill the geometry arrays; called by one workgroup (any size).
__device__ void build_geometry(const Params& P, const double* rfaces_in, const double* zfaces_in,
                               const Geom& g) {
  for (int i = threadIdx.x; i < P.nr; i += blockDim.x) {
    axis_point(i, P.nr, P.rmax, rfaces_in, g.rf, g.rc, g.dr);
    g.kap[i] = (uint8_t)column_class(P, g.rc[i]);
  }
  for (int j = threadIdx.x; j < P.nz; j += blockDim.x) {
    axis_point(j, P.nz, P.ztop, zfaces_in, g.zf, g.zc, g.dz);
    g.bet[j] = (uint8_t)row_band(P, g.zc[j]);
  }
}

// ------------------------------------------------------------- assembly --

// Half-cell conductance in series with a film h (h = 0: none, h = inf: the
// face is held at t_inf).
__device__ __forceinline__ double film(double d, double k, double h) {
  if (h == 0.0) return 0.0;
  if (__builtin_isinf(h)) return 2.0 * k / d;
  return 1.0 / (d / (2.0 * k) + 1.0 / h);
}
__device__ __forceinline__ double series2(double da, double ka, double db, double kb) {
  return 1.0 / (da / (2.0 * ka) + db / (2.0 * kb));
}

// Row p of the line matrix of one class plus the output operator, the
// boundary-flow weights and the boundary constant of this direction.
struct RowCoef {
  double a, b, c;          // matrix: a x[p-1] + b x[p] + c x[p+1]
  double od, ol, ou, oc;   // output operator
  double bw, bt;           // boundary flow weight and its T_inf part
  double bconst;           // boundary constant b of this direction's operator
};

// dir 0: r line in band `cls` at position i; dir 1: z line of column class
// `cls` at position j.  Balance form of eq. 10 (r) or eq. 11 (z).
__device__ RowCoef row_coef(const Params& P, const Geom& g, int dir, int cls, int p) {
  RowCoef R = {0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int n = dir == 0 ? P.nr : P.nz;
  if (p >= n) return R;  // padding: identity row
  auto reg = [&](int q) {
    return dir == 0 ? region_of(cls, g.kap[q]) : region_of(g.bet[q], cls);
  };
  const int m = reg(p);
  if (m == MASKED) return R;
  const double kc = P.k[m];
  const double C = P.rhoc[m] / P.ta;
  double lo = 0.0, up = 0.0, diag = 0.0, bconst = 0.0, bw = 0.0, bt = 0.0;
  if (dir == 0) {
    const double vol = g.rc[p] * g.dr[p];
    // west face at rf[p]
    if (p > 0) {
      const int mw = reg(p - 1);
      if (mw == MASKED) {
        const double gg = g.rf[p] * film(g.dr[p], kc, P.h[3]);
        diag -= gg / vol; bconst += gg * P.tinf[3] / vol; bw += gg; bt += gg * P.tinf[3];
      } else {
        const double w = g.rf[p] * series2(g.dr[p - 1], P.k[mw], g.dr[p], kc) / vol;
        lo = w; diag -= w;
      }
    }  // p == 0: the axis carries no flux
    // east face at rf[p+1]
    const int me = p + 1 < n ? reg(p + 1) : MASKED;
    if (p == n - 1 || me == MASKED) {
      const int bc = p == n - 1 ? 1 : 3;
      const double gg = g.rf[p + 1] * film(g.dr[p], kc, P.h[bc]);
      diag -= gg / vol; bconst += gg * P.tinf[bc] / vol; bw += gg; bt += gg * P.tinf[bc];
    } else {
      const double w = g.rf[p + 1] * series2(g.dr[p], kc, g.dr[p + 1], P.k[me]) / vol;
      up = w; diag -= w;
    }
  } else {
    const double vol = g.dz[p];
    const int ms = p > 0 ? reg(p - 1) : MASKED;
    if (p == 0 || ms == MASKED) {
      const int bc = p == 0 ? 0 : 3;
      const double gg = film(g.dz[p], kc, P.h[bc]);
      diag -= gg / vol; bconst += gg * P.tinf[bc] / vol; bw += gg; bt += gg * P.tinf[bc];
    } else {
      const double w = series2(g.dz[p - 1], P.k[ms], g.dz[p], kc) / vol;
      lo = w; diag -= w;
    }
    const int mn = p + 1 < n ? reg(p + 1) : MASKED;
    if (p == n - 1 || mn == MASKED) {
      const int bc = p == n - 1 ? 2 : 3;
      const double gg = film(g.dz[p], kc, P.h[bc]);
      diag -= gg / vol; bconst += gg * P.tinf[bc] / vol; bw += gg; bt += gg * P.tinf[bc];
    } else {
      const double w = series2(g.dz[p], kc, g.dz[p + 1], P.k[mn]) / vol;
      up = w; diag -= w;
    }
  }
  R.a = -lo;
  R.b = C - diag;
  R.c = -up;
  // The next half step's right-hand side: (C/ta) x + theta (A x) + ...
  R.od = C + P.theta * diag;
  R.ol = P.theta * lo;
  R.ou = P.theta * up;
  // r sweep output: theta (b_r + Q) (+ b_z from the crossing table);
  // z sweep output: theta b_z + Q (+ b_r from the crossing table).
  R.oc = dir == 0 ? P.theta * (bconst + P.q[m]) : P.theta * bconst + P.q[m];
  R.bw = bw;
  R.bt = bt;
  R.bconst = bconst;
  return R;
}

// Work area of assemble_class, in doubles.
__host__ __device__ constexpr long assemble_work(int G, int M) { return 3L * G * M + 12L * G; }

// Build the table of one line class.  Must be called by a whole workgroup.
//  pos: [P_NFIELDS][G*M], chk: [C_NFIELDS][G], eng: [2][n] boundary-flow
//  weights, xc: [n] boundary constants of this direction (the other
//  direction's sweeps add them), work: assemble_work(G, M) doubles.
__device__ void assemble_class(const Params& P, const Geom& g, int dir, int cls, int G, int M,
                               int CPW, double* pos, double* chk, double* eng, double* xc,
                               double* work) {
  const int n = dir == 0 ? P.nr : P.nz;
  const int GM = G * M;
  double* A = work;
  double* B = work + GM;
  double* Cc = work + 2 * GM;
  double* rlo = work + 3 * GM;          // 2G each
  double* rdi = rlo + 2 * G;
  double* rup = rdi + 2 * G;
  double* rW = rup + 2 * G;
  double* rQ = rW + 2 * G;
  double* rC = rQ + 2 * G;

  // Phase 1: matrix rows and output operator at every position.
  for (int p = threadIdx.x; p < GM; p += blockDim.x) {
    const RowCoef R = row_coef(P, g, dir, cls, p);
    A[p] = R.a; B[p] = R.b; Cc[p] = R.c;
    const int ix = (p % M) * G + p / M;
    pos[P_OD * GM + ix] = R.od;
    pos[P_OL * GM + ix] = R.ol;
    pos[P_OU * GM + ix] = R.ou;
    pos[P_OC * GM + ix] = R.oc;
    if (p < n) {
      eng[p] = R.bw;
      eng[n + p] = R.bt;
      xc[p] = R.bconst;
    }
  }
  __syncthreads();

  // Phase 2: per chunk, Thomas factors of the interior rows 1..M-2, the two
  // spikes, and the chunk's two rows of the reduced system.
  for (int k = threadIdx.x; k < G; k += blockDim.x) {
    const int s = k * M;
    auto at = [&](int f, int t) -> double& { return pos[f * GM + t * G + k]; };
    at(P_W, 0) = at(P_QA, 0) = at(P_CP, 0) = at(P_SP, 0) = at(P_SR, 0) = 0.0;
    at(P_W, M - 1) = at(P_QA, M - 1) = at(P_CP, M - 1) = at(P_SP, M - 1) = at(P_SR, M - 1) = 0.0;
    double cprev = 0.0, sp = 0.0;
    for (int t = 1; t <= M - 2; ++t) {
      const double a = t > 1 ? A[s + t] : 0.0;
      const double w = 1.0 / (B[s + t] - a * cprev);
      const double cp = t < M - 2 ? Cc[s + t] * w : 0.0;
      at(P_W, t) = w;
      at(P_QA, t) = a * w;
      at(P_CP, t) = cp;
      // forward pass of the first spike: right-hand side a_1 e_1
      sp = t == 1 ? A[s + 1] * w : -(a * w) * sp;
      at(P_SP, t) = sp;
      cprev = cp;
    }
    // backward passes of both spikes
    double spn = 0.0, srn = 0.0;
    for (int t = M - 2; t >= 1; --t) {
      const double cp = at(P_CP, t);
      spn = at(P_SP, t) - cp * spn;
      srn = (t == M - 2 ? Cc[s + M - 2] * at(P_W, t) : 0.0) - cp * srn;
      at(P_SP, t) = spn;
      at(P_SR, t) = srn;
    }
    const double P1 = at(P_SP, 1), R1 = at(P_SR, 1);
    const double Pl = at(P_SP, M - 2), Rl = at(P_SR, M - 2);
    const int e = s + M - 1;
    rlo[2 * k] = A[s];
    rdi[2 * k] = B[s] - Cc[s] * P1;
    rup[2 * k] = -Cc[s] * R1;
    rlo[2 * k + 1] = -A[e] * Pl;
    rdi[2 * k + 1] = B[e] - A[e] * Rl;
    rup[2 * k + 1] = Cc[e];
    chk[C_CS * G + k] = Cc[s];
    chk[C_AE * G + k] = A[e];
  }
  __syncthreads();

  // Phase 3: Thomas factors of the reduced system (2G rows, sequential).
  if (threadIdx.x == 0) {
    double cprev = 0.0;
    for (int l = 0; l < 2 * G; ++l) {
      const double lo = l > 0 ? rlo[l] : 0.0;
      const double w = 1.0 / (rdi[l] - lo * cprev);
      rW[l] = w;
      rQ[l] = lo * w;
      rC[l] = l < 2 * G - 1 ? rup[l] * w : 0.0;
      cprev = rC[l];
    }
  }
  __syncthreads();

  // Phase 4: per-chunk factors and the products used by recursive doubling.
  for (int k = threadIdx.x; k < G; k += blockDim.x) {
    chk[C_W0 * G + k] = rW[2 * k];
    chk[C_Q0 * G + k] = rQ[2 * k];
    chk[C_C0 * G + k] = rC[2 * k];
    chk[C_W1 * G + k] = rW[2 * k + 1];
    chk[C_Q1 * G + k] = rQ[2 * k + 1];
    chk[C_C1 * G + k] = rC[2 * k + 1];
    chk[C_CPREV * G + k] = k > 0 ? rC[2 * k - 1] : 0.0;
    auto Bf = [&](int t) { return rQ[2 * t + 1] * rQ[2 * t]; };
    auto Eb = [&](int t) { return rC[2 * t] * rC[2 * t + 1]; };
    const int ws = (k / CPW) * CPW, we = ws + CPW - 1;
    double pre = 1.0;
    for (int t = ws; t <= k; ++t) pre *= Bf(t);
    double suf = 1.0;
    for (int t = k; t <= we; ++t) suf *= Eb(t);
    chk[C_BPRE * G + k] = pre;
    chk[C_ESUF * G + k] = suf;
    for (int lev = 0; lev < MAX_LEV; ++lev) {
      const int d = 1 << lev;
      double f = 0.0, b = 0.0;
      if (k - d >= ws) {
        f = 1.0;
        for (int t = k - d + 1; t <= k; ++t) f *= Bf(t);
      }
      if (k + d <= we) {
        b = 1.0;
        for (int t = k; t <= k + d - 1; ++t) b *= Eb(t);
      }
      chk[(C_KSF + lev) * G + k] = f;
      chk[(C_KSB + lev) * G + k] = b;
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------ line solve --

// Solve the lines of one line group: LPW lines side by side in each wave,
// each line spread over CPW = 64/LPW chunks per wave and WPL waves.  `lds`
// holds LPW*WPL doubles for this group.  `valid` is false for groups past the
// end (they still take part in the barriers).
template <int MM, int LPW, int WPL>
__device__ __forceinline__ void solve_group(const SweepArgs& a, int group, double* lds, bool valid,
                                            int wave_in_group) {
  constexpr int CPW = 64 / LPW;
  constexpr int LEV = __builtin_ctz(CPW);
  const int lane = threadIdx.x & 63;
  const int li = lane % LPW;
  const int ci = lane / LPW;
  const int wv = wave_in_group;
  const int k = wv * CPW + ci;
  const int L = group * LPW + li;
  const bool act = valid && L < a.nlines;
  const int cls = act ? a.line_class[L] : a.line_class[0];
  const LineTab tb = a.tabs[cls];
  const int M = tb.M, G = tb.G, GM = G * M;
  const double* __restrict__ pos = tb.pos;
  const double* __restrict__ chk = tb.chk;
  const long base = (long)(act ? L : 0) * a.line_stride;

  double v[MM];
#pragma unroll
  for (int t = 0; t < MM; ++t) {
    v[t] = 0.0;
    if (t < M) {
      const int p = k * M + t;
      const bool ok = act && p < tb.n && (p < tb.skip_lo || p >= tb.skip_hi);
      if (ok) v[t] = a.din[base + (long)p * a.pos_stride];
    }
  }
  const double ds = v[0];
  double de = 0.0;
#pragma unroll
  for (int t = 0; t < MM; ++t)
    if (t == M - 1) de = v[t];

  // interior forward elimination and back substitution (rows 1..M-2)
  double run = 0.0;
#pragma unroll
  for (int t = 1; t < MM - 1; ++t) {
    if (t <= M - 2) {
      const int ix = t * G + k;
      run = v[t] * pos[P_W * GM + ix] - pos[P_QA * GM + ix] * run;
      v[t] = run;
    }
  }
  run = 0.0;
#pragma unroll
  for (int t = MM - 2; t >= 1; --t) {
    if (t <= M - 2) {
      run = v[t] - pos[P_CP * GM + t * G + k] * run;
      v[t] = run;
    }
  }
  double zl = 0.0;
#pragma unroll
  for (int t = 1; t < MM; ++t)
    if (t == M - 2) zl = v[t];
  const double g0 = ds - chk[C_CS * G + k] * v[1 < MM ? 1 : 0];
  const double g1 = de - chk[C_AE * G + k] * zl;

  // reduced system, forward recurrence F_k = A_k + B_k F_{k-1}
  const double W0 = chk[C_W0 * G + k], Q0 = chk[C_Q0 * G + k], C0 = chk[C_C0 * G + k];
  const double W1 = chk[C_W1 * G + k], Q1 = chk[C_Q1 * G + k], C1 = chk[C_C1 * G + k];
  const double g0w = g0 * W0;
  double F = g1 * W1 - Q1 * g0w;
#pragma unroll
  for (int lev = 0; lev < LEV; ++lev) {
    const int d = 1 << lev;
    const double o = __shfl_up(F, d * LPW, 64);
    if (ci >= d) F += chk[(C_KSF + lev) * G + k] * o;
  }
  double Fin = 0.0;
  if constexpr (WPL > 1) {
    if (ci == CPW - 1) lds[li * WPL + wv] = F;
    __syncthreads();
    double cin = 0.0;
    for (int w = 0; w < wv; ++w) cin = lds[li * WPL + w] + chk[C_BPRE * G + w * CPW + CPW - 1] * cin;
    F += chk[C_BPRE * G + k] * cin;
    Fin = cin;
    __syncthreads();
  }
  double Fprev = __shfl_up(F, LPW, 64);
  if (ci == 0) Fprev = Fin;

  // backward recurrence U_k = H_k + E_k U_{k+1}
  const double f0 = g0w - Q0 * Fprev;
  double U = f0 - C0 * F;
#pragma unroll
  for (int lev = 0; lev < LEV; ++lev) {
    const int d = 1 << lev;
    const double o = __shfl_down(U, d * LPW, 64);
    if (ci + d < CPW) U += chk[(C_KSB + lev) * G + k] * o;
  }
  double Uin = 0.0;
  if constexpr (WPL > 1) {
    if (ci == 0) lds[li * WPL + wv] = U;
    __syncthreads();
    double cin = 0.0;
    for (int w = WPL - 1; w > wv; --w) cin = lds[li * WPL + w] + chk[C_ESUF * G + w * CPW] * cin;
    U += chk[C_ESUF * G + k] * cin;
    Uin = cin;
    __syncthreads();
  }
  double Unext = __shfl_down(U, LPW, 64);
  if (ci == CPW - 1) Unext = Uin;

  const double xs = U;                                   // first unknown of the chunk
  const double xe = F - C1 * Unext;                      // last unknown
  const double xm1 = Fprev - chk[C_CPREV * G + k] * U;   // last unknown of chunk k-1
  const double xp1 = Unext;                              // first unknown of chunk k+1

  // interior back substitution
  v[0] = xs;
#pragma unroll
  for (int t = 1; t < MM; ++t) {
    if (t <= M - 2) {
      const int ix = t * G + k;
      v[t] = v[t] - pos[P_SP * GM + ix] * xs - pos[P_SR * GM + ix] * xe;
    } else if (t == M - 1) {
      v[t] = xe;
    }
  }

  // outputs: solution (optional) and the next half step's right-hand side
  double xprev = xm1;
#pragma unroll
  for (int t = 0; t < MM; ++t) {
    if (t < M) {
      const int p = k * M + t;
      const bool ok = act && p < tb.n && (p < tb.skip_lo || p >= tb.skip_hi);
      const double xt = v[t];
      const double xn = (t + 1 < MM && t + 1 < M) ? v[t + 1 < MM ? t + 1 : t] : xp1;
      const int ix = t * G + k;
      double o = pos[P_OD * GM + ix] * xt + pos[P_OL * GM + ix] * xprev +
                 pos[P_OU * GM + ix] * xn + pos[P_OC * GM + ix];
      if (ok) {
        const long addr = base + (long)p * a.pos_stride;
        if (a.xc) o += a.xc[(long)a.pos_xclass[p] * a.nlines + L];
        a.dout[addr] = o;
        if (a.xout) a.xout[addr] = xt;
      }
      xprev = xt;
    }
  }
}

}  // namespace adi
