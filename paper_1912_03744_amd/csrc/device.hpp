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

// Keep the scheduler from hoisting the factor-table loads of later steps of
// an unrolled recurrence (which would exhaust registers); loads of the
// current step still overlap with the arithmetic of the previous one.
#define ADI_STEP_FENCE()                                  \
  do {                                                    \
    if constexpr (M * R > ADI_FENCE_CELLS) __builtin_amdgcn_sched_barrier(0); \
  } while (0)
#ifndef ADI_FENCE_CELLS
#define ADI_FENCE_CELLS 12  // short chunks keep all their table loads in flight
#endif

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
  P_OK,      // (1 + theta) rho c / tau_a: with the solve's own right-hand
             // side d, od x + ol x[-1] + ou x[+1] + oc = P_OK x - theta d + oc
  P_NFIELDS
};

// Per-chunk fields: the chunk's two rows of the reduced system.
enum ChkField {
  C_CS = 0,  // super-diagonal of the chunk's first row
  C_AE,      // sub-diagonal of the chunk's last row
  C_W0, C_Q0, C_C0,   // reduced-system Thomas factors of row 2k
  C_W1, C_Q1, C_C1,   // ... of row 2k+1
  C_CPREV,   // C of row 2k-1 (the previous chunk's last row)
  C_NFIELDS
};

// Table layout.  Plain: field f of position ix (= t*G + k) at f*GM + ix, of
// chunk k at f*G + k.  Paired (the tables of the strip-layout sweeps): the
// fields those kernels load together are stored as interleaved pairs, so
// that one 16-byte load per lane fetches both: (w, qa), (cp, sp), (oc, ok)
// of the positions and (cs, ae), (W0, Q0), (C0, W1), (Q1, C1) of the chunks;
// the other fields stay plain arrays.
__host__ __device__ constexpr bool pos_paired(int f) {
  return f == P_W || f == P_QA || f == P_CP || f == P_SP || f == P_OC || f == P_OK;
}
__host__ __device__ constexpr long pos_at(int f, long GM, long ix, bool paired) {
  return paired && pos_paired(f) ? (long)(f & ~1) * GM + 2 * ix + (f & 1) : (long)f * GM + ix;
}
__host__ __device__ constexpr long chk_at(int f, long G, long k, bool paired) {
  return paired && f < C_CPREV ? (long)(f & ~1) * G + 2 * k + (f & 1) : (long)f * G + k;
}
static_assert(P_QA == P_W + 1 && (P_W & 1) == 0 && P_SP == P_CP + 1 && (P_CP & 1) == 0 &&
              P_OK == P_OC + 1 && (P_OC & 1) == 0, "paired position fields");
static_assert(C_AE == C_CS + 1 && C_CS == 0 && C_Q0 == C_W0 + 1 && C_W0 == 2 && C_W1 == C_C0 + 1 &&
              C_C0 == 4 && C_C1 == C_Q1 + 1 && C_Q1 == 6 && C_CPREV == 8, "paired chunk fields");

// One line class in one direction.
struct LineTab {
  const double* pos;   // [P_NFIELDS][G*M]
  const double* chk;   // [C_NFIELDS][G]
  int n, G, M;         // line length, chunks, cells per chunk
  int skip_lo, skip_hi;  // positions [skip_lo, skip_hi) are outside the domain
};

constexpr int MAX_CLS = 4;

// Arguments of one sweep (one direction of one instance).  The lines of a
// class form one contiguous index range [cls_l0[c], cls_l1[c]); line groups
// never straddle two classes, so every group reads one set of tables: class c
// owns groups [cls_g0[c], cls_g0[c+1]).
struct SweepArgs {
  const double* din;      // right-hand side of this half step
  double* dout;           // right-hand side of the next half step
  double* xout;           // solution of this half step, or null
  const LineTab* tabs;    // line-class tables of this direction
  const uint8_t* pos_xclass;  // class of the crossing line at every position
  const double* xc;       // [xclass][line] constant of the other direction, or null
  long line_stride, pos_stride;
  int nlines, ncls, ngroups;
  int cls_l0[MAX_CLS], cls_l1[MAX_CLS], cls_g0[MAX_CLS + 1];
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

// Fill the geometry arrays; called by one workgroup (any size).  ranges
// (17 ints, any memory) receives, per direction (0: rows by band, 1: columns
// by class) and class, the index range [first, last+1) of its lines; a class
// with no lines gets [0, 0).  ranges[16] is set non-zero if a class is not
// one contiguous run (centres are monotone, so it never is).
__device__ void build_geometry(const Params& P, const double* rfaces_in, const double* zfaces_in,
                               const Geom& g, int* ranges) {
  for (int q = threadIdx.x; q < 17; q += blockDim.x) ranges[q] = 0;
  for (int i = threadIdx.x; i < P.nr; i += blockDim.x) {
    axis_point(i, P.nr, P.rmax, rfaces_in, g.rf, g.rc, g.dr);
    g.kap[i] = (uint8_t)column_class(P, g.rc[i]);
  }
  for (int j = threadIdx.x; j < P.nz; j += blockDim.x) {
    axis_point(j, P.nz, P.ztop, zfaces_in, g.zf, g.zc, g.dz);
    g.bet[j] = (uint8_t)row_band(P, g.zc[j]);
  }
  __shared__ int cnt[2 * MAX_CLS];
  for (int q = threadIdx.x; q < 2 * MAX_CLS; q += blockDim.x) cnt[q] = 0;
  __syncthreads();
  // run boundaries: where the class changes along each axis
  for (int dir = 0; dir < 2; ++dir) {
    const uint8_t* cl = dir == 0 ? g.bet : g.kap;
    const int n = dir == 0 ? P.nz : P.nr;
    int* rg = ranges + dir * MAX_CLS * 2;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
      const int c = cl[q];
      atomicAdd(&cnt[dir * MAX_CLS + c], 1);
      if (q == 0 || cl[q - 1] != c) rg[2 * c] = q;
      if (q == n - 1 || cl[q + 1] != c) rg[2 * c + 1] = q + 1;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int q = 0; q < 2 * MAX_CLS; ++q)
      if (cnt[q] != ranges[2 * q + 1] - ranges[2 * q]) ranges[16] = 1;
  __syncthreads();
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
  double ok;               // (1 + theta) C: diagonal of the output operator written against d
  double bw, bt;           // boundary flow weight and its T_inf part
  double bconst;           // boundary constant b of this direction's operator
};

// dir 0: r line in band `cls` at position i; dir 1: z line of column class
// `cls` at position j.  Balance form of eq. 10 (r) or eq. 11 (z).
__device__ RowCoef row_coef(const Params& P, const Geom& g, int dir, int cls, int p) {
  RowCoef R = {0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
  // od = (1 + theta) C - theta b, ol = -theta a, ou = -theta c
  R.ok = (1.0 + P.theta) * C;
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
                               double* pos, double* chk, double* eng, double* xc, double* work,
                               bool paired) {
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
    pos[pos_at(P_OD, GM, ix, paired)] = R.od;
    pos[pos_at(P_OL, GM, ix, paired)] = R.ol;
    pos[pos_at(P_OU, GM, ix, paired)] = R.ou;
    pos[pos_at(P_OC, GM, ix, paired)] = R.oc;
    pos[pos_at(P_OK, GM, ix, paired)] = R.ok;
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
    auto at = [&](int f, int t) -> double& { return pos[pos_at(f, GM, (long)t * G + k, paired)]; };
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
    chk[chk_at(C_CS, G, k, paired)] = Cc[s];
    chk[chk_at(C_AE, G, k, paired)] = A[e];
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

  // Phase 4: per-chunk factors of the reduced system.
  for (int k = threadIdx.x; k < G; k += blockDim.x) {
    chk[chk_at(C_W0, G, k, paired)] = rW[2 * k];
    chk[chk_at(C_Q0, G, k, paired)] = rQ[2 * k];
    chk[chk_at(C_C0, G, k, paired)] = rC[2 * k];
    chk[chk_at(C_W1, G, k, paired)] = rW[2 * k + 1];
    chk[chk_at(C_Q1, G, k, paired)] = rQ[2 * k + 1];
    chk[chk_at(C_C1, G, k, paired)] = rC[2 * k + 1];
    chk[chk_at(C_CPREV, G, k, paired)] = k > 0 ? rC[2 * k - 1] : 0.0;
  }
  __syncthreads();
}

// ------------------------------------------------------------ line solve --

// Bit t set iff position p0 + t of a chunk is a real cell (below n) outside
// the skipped run [skip_lo, skip_hi).
__device__ __forceinline__ unsigned long long chunk_live_mask(int p0, int M, int n, int skip_lo,
                                                              int skip_hi) {
  auto below = [](int c) -> unsigned long long {  // bits [0, c)
    return c <= 0 ? 0ull : (c >= 64 ? ~0ull : ((1ull << c) - 1ull));
  };
  const int m = M < n - p0 ? M : n - p0;
  return below(m) & ~(below(skip_hi - p0) & ~below(skip_lo - p0));
}

// ---- scans of affine maps over the chunks of a line slot ----
//
// A line slot is CPW consecutive lanes (CPW a power of two from 4 to 64),
// lane ci of the slot holding chunk ci.  Forward: x_k = A_k + B_k x_{k-1},
// lane ci ends with the composition over chunks 0..ci.  Backward: x_k = H_k +
// E_k x_{k+1}, lane ci ends with the composition over chunks ci..CPW-1.
// Steps inside rows of 16 lanes are DPP row shifts (lanes without a source
// in the slot combine with the identity map); across rows the forward scan
// uses DPP row broadcasts and the backward scan reads the row totals with
// readlane.

template <int CTRL>
__device__ __forceinline__ double dpp_row(double old, double src) {
  const long long o = __double_as_longlong(old), v = __double_as_longlong(src);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(v >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The same row shift with 0 in lanes without a source (DPP bound control),
// so no identity value has to be placed in the destination first.
template <int CTRL>
__device__ __forceinline__ double dpp_row0(double src) {
  const long long v = __double_as_longlong(src);
  const int lo = __builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// DPP broadcast across rows (row_bcast:15 / row_bcast:31), writing only the
// rows in ROWS; other lanes keep `old`.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_bcast(double old, double src) {
  const long long o = __double_as_longlong(old), v = __double_as_longlong(src);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)v, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(v >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double read_lane(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, l);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The R values of a lane belong to R lines; lines r < NA compose with the
// multiplier BA, the others with BB (lines of two classes in one block).
template <int CPW, int D, int R, int NA>
__device__ __forceinline__ void fwd_step(double (&F)[R], double& BA, double& BB, int ci) {
  if constexpr (D < CPW && D < 16) {
    double BoA = dpp_row<0x110 + D>(1.0, BA);
    double BoB = NA < R ? dpp_row<0x110 + D>(1.0, BB) : 1.0;
    double Ao[R];
#pragma unroll
    for (int r = 0; r < R; ++r) Ao[r] = dpp_row0<0x110 + D>(F[r]);
    if constexpr (CPW < 16) {  // slot starts inside a row
      if (ci < D) {
        BoA = BoB = 1.0;
#pragma unroll
        for (int r = 0; r < R; ++r) Ao[r] = 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) F[r] += (r < NA ? BA : BB) * Ao[r];
    BA *= BoA;
    if constexpr (NA < R) BB *= BoB;
  }
}

template <int CPW, int D, int R, int NA>
__device__ __forceinline__ void bwd_step(double (&U)[R], double& EA, double& EB, int ci) {
  if constexpr (D < CPW && D < 16) {
    double EoA = dpp_row<0x100 + D>(1.0, EA);
    double EoB = NA < R ? dpp_row<0x100 + D>(1.0, EB) : 1.0;
    double Uo[R];
#pragma unroll
    for (int r = 0; r < R; ++r) Uo[r] = dpp_row0<0x100 + D>(U[r]);
    if constexpr (CPW < 16) {  // slot ends inside a row
      if (ci + D >= CPW) {
        EoA = EoB = 1.0;
#pragma unroll
        for (int r = 0; r < R; ++r) Uo[r] = 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) U[r] += (r < NA ? EA : EB) * Uo[r];
    EA *= EoA;
    if constexpr (NA < R) EB *= EoB;
  }
}

template <int CPW, int R, int NA = R>
__device__ __forceinline__ void slot_scan_fwd(double (&F)[R], double& BA, double& BB) {
  static_assert(CPW >= 4 && CPW <= 64 && (CPW & (CPW - 1)) == 0, "slot width");
  static_assert(NA >= 1 && NA <= R, "split");
  const int ci = (threadIdx.x & 63) & (CPW - 1);
  fwd_step<CPW, 1, R, NA>(F, BA, BB, ci);
  fwd_step<CPW, 2, R, NA>(F, BA, BB, ci);
  fwd_step<CPW, 4, R, NA>(F, BA, BB, ci);
  fwd_step<CPW, 8, R, NA>(F, BA, BB, ci);
  if constexpr (CPW >= 32) {
    // rows 1 and 3 take the totals of rows 0 and 2 (lanes 15 and 47)
    const double BoA = dpp_bcast<0x142, 0xa>(1.0, BA);
    const double BoB = NA < R ? dpp_bcast<0x142, 0xa>(1.0, BB) : 1.0;
#pragma unroll
    for (int r = 0; r < R; ++r) F[r] += (r < NA ? BA : BB) * dpp_bcast<0x142, 0xa>(0.0, F[r]);
    BA *= BoA;
    if constexpr (NA < R) BB *= BoB;
  }
  if constexpr (CPW == 64) {
    // rows 2 and 3 take the total of rows 0..1 (lane 31)
    const double BoA = dpp_bcast<0x143, 0xc>(1.0, BA);
    const double BoB = NA < R ? dpp_bcast<0x143, 0xc>(1.0, BB) : 1.0;
#pragma unroll
    for (int r = 0; r < R; ++r) F[r] += (r < NA ? BA : BB) * dpp_bcast<0x143, 0xc>(0.0, F[r]);
    BA *= BoA;
    if constexpr (NA < R) BB *= BoB;
  }
}

template <int CPW, int R, int NA = R>
__device__ __forceinline__ void slot_scan_bwd(double (&U)[R], double& EA, double& EB) {
  static_assert(CPW >= 4 && CPW <= 64 && (CPW & (CPW - 1)) == 0, "slot width");
  static_assert(NA >= 1 && NA <= R, "split");
  const int lane = threadIdx.x & 63;
  const int ci = lane & (CPW - 1);
  bwd_step<CPW, 1, R, NA>(U, EA, EB, ci);
  bwd_step<CPW, 2, R, NA>(U, EA, EB, ci);
  bwd_step<CPW, 4, R, NA>(U, EA, EB, ci);
  bwd_step<CPW, 8, R, NA>(U, EA, EB, ci);
  if constexpr (CPW >= 32) {
    // rows compose the totals of the rows after them inside their slot
    // (totals sit at the first lane of each row)
    const int row = lane >> 4;
    double cU[R], cEA = 1.0, cEB = 1.0;
#pragma unroll
    for (int r = 0; r < R; ++r) cU[r] = 0.0;
#pragma unroll
    for (int q = 3; q >= 1; --q) {
      const double tEA = read_lane(EA, 16 * q);
      const double tEB = NA < R ? read_lane(EB, 16 * q) : 1.0;
      double tU[R];
#pragma unroll
      for (int r = 0; r < R; ++r) tU[r] = read_lane(U[r], 16 * q);
      // row `row` takes row q if q is after it within the same slot
      const bool take = q > row && (q * 16) / CPW == (row * 16) / CPW;
      if (take) {
#pragma unroll
        for (int r = 0; r < R; ++r) cU[r] = tU[r] + (r < NA ? tEA : tEB) * cU[r];
        cEA *= tEA;
        if constexpr (NA < R) cEB *= tEB;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) U[r] += (r < NA ? EA : EB) * cU[r];
    EA *= cEA;
    if constexpr (NA < R) EB *= cEB;
  }
}

// One multiplier for all R lines.
template <int CPW, int R>
__device__ __forceinline__ void slot_scan_fwd(double (&F)[R], double& B) {
  slot_scan_fwd<CPW, R, R>(F, B, B);
}
template <int CPW, int R>
__device__ __forceinline__ void slot_scan_bwd(double (&U)[R], double& E) {
  slot_scan_bwd<CPW, R, R>(U, E, E);
}

// Solve one line group.  The group has LPW lane slots per wave (each slot
// CPW = 64/LPW consecutive lanes) owning R consecutive lines; every line is
// spread over CPW chunks per wave and WPL waves, M cells per chunk.  A lane
// therefore holds an R x M block: the same chunk of R lines, so each
// factor-table value it loads serves R lines.  All sizes are compile-time,
// so every loop unrolls without branches.  The reduced system is solved by
// recursive doubling on affine maps (x_k = A + B x_{k-2^s}) over the slot's
// lanes with DPP row operations (slot_scan_fwd / slot_scan_bwd), with a
// carry through LDS when a line spans several waves.
// `lds` holds WPL*LPW*(R+1) doubles for this group; groups past the end
// (valid = false) still take part in the barriers.
// CONTIG: positions of a line are adjacent in memory (pos_stride == 1, r
// lines); the chunk is then moved with 16-byte accesses where it lies inside
// the line.  Otherwise lines are adjacent (line_stride == 1, z lines).
template <int M, int LPW, int WPL, int R, bool CONTIG>
__device__ __forceinline__ void solve_group(const SweepArgs& a, int group, double* lds, bool valid,
                                            int wv) {
  static_assert(M >= 3, "chunks need an interior row");
  constexpr int CPW = 64 / LPW;
  constexpr int G = CPW * WPL;
  constexpr int GM = G * M;
  const int lane = threadIdx.x & 63;
  const int li = lane / CPW;  // line slot: CPW consecutive lanes
  const int ci = lane % CPW;  // chunk within the wave's part of the line
  const int k = wv * CPW + ci;

  // class of the group (uniform across the group)
  int c = 0;
  while (c + 1 < a.ncls && group >= a.cls_g0[c + 1]) ++c;
  const int Lfirst = a.cls_l0[c] + (group - a.cls_g0[c]) * (LPW * R) + li * R;
  const int Lend = valid ? a.cls_l1[c] : 0;
  const LineTab tb = a.tabs[c];
  const double* __restrict__ pos = tb.pos + k;  // plain tables (pos_at, chk_at)
  const double* __restrict__ chk = tb.chk + k;
  const int p0 = k * M;

  // Addresses: a uniform base (scalar registers) plus one 32-bit byte offset
  // per lane; the per-step and per-line increments are uniform too.
  const long ls8 = a.line_stride * 8, ps8 = a.pos_stride * 8;
  const unsigned lane_off = (unsigned)((long)Lfirst * ls8 + (long)p0 * ps8);
  const char* __restrict__ din = (const char*)a.din;
  // bit t set: chunk offset t is a real cell inside the domain
  const unsigned long long live = chunk_live_mask(p0, M, tb.n, tb.skip_lo, tb.skip_hi);
  // cells of the chunk that lie inside the line (readable even if masked)
  const int inl = tb.n - p0;
  const bool pairs_ok = CONTIG && (M % 2 == 0) && ((a.line_stride & 1) == 0);

  double v[R][M];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool act = Lfirst + r < Lend;
    const char* rowp = din + (long)r * ls8;  // uniform
    if (pairs_ok) {
#pragma unroll
      for (int t = 0; t < M; t += 2) {
        double2 q = make_double2(0.0, 0.0);
        if (act && t + 1 < inl) q = *(const double2*)(rowp + lane_off + t * 8);
        else if (act && t < inl) q.x = *(const double*)(rowp + lane_off + t * 8);
        v[r][t] = ((live >> t) & 1ull) ? q.x : 0.0;
        v[r][t + 1] = ((live >> (t + 1)) & 1ull) ? q.y : 0.0;
      }
    } else {
#pragma unroll
      for (int t = 0; t < M; ++t) {
        const bool ok = act && ((live >> t) & 1ull);
        v[r][t] = ok ? *(const double*)(rowp + (long)t * ps8 + lane_off) : 0.0;
      }
    }
  }

  // interior forward elimination and back substitution (rows 1..M-2)
  double run[R];
#pragma unroll
  for (int r = 0; r < R; ++r) run[r] = 0.0;
#pragma unroll
  for (int t = 1; t <= M - 2; ++t) {
    ADI_STEP_FENCE();
    const double w = pos[P_W * GM + t * G], qa = pos[P_QA * GM + t * G];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      run[r] = v[r][t] * w - qa * run[r];
      v[r][t] = run[r];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) run[r] = 0.0;
#pragma unroll
  for (int t = M - 2; t >= 1; --t) {
    ADI_STEP_FENCE();
    const double cp = pos[P_CP * GM + t * G];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      run[r] = v[r][t] - cp * run[r];
      v[r][t] = run[r];
    }
  }

  // reduced system: forward recurrence F_k = A_k + B_k F_{k-1}
  const double cs = chk[C_CS * G], ae = chk[C_AE * G];
  const double W0 = chk[C_W0 * G], Q0 = chk[C_Q0 * G], C0 = chk[C_C0 * G];
  const double W1 = chk[C_W1 * G], Q1 = chk[C_Q1 * G], C1 = chk[C_C1 * G];
  const double cprev = chk[C_CPREV * G];
  double g0w[R], F[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    g0w[r] = (v[r][0] - cs * v[r][1]) * W0;
    F[r] = (v[r][M - 1] - ae * v[r][M - 2]) * W1 - Q1 * g0w[r];
  }
  double B = Q1 * Q0;
  slot_scan_fwd<CPW, R>(F, B);
  double Fin[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Fin[r] = 0.0;
  if constexpr (WPL > 1) {
    double* slot = lds + (wv * LPW + li) * (R + 1);
    if (ci == CPW - 1) {
#pragma unroll
      for (int r = 0; r < R; ++r) slot[r] = F[r];
      slot[R] = B;
    }
    __syncthreads();
    for (int w = 0; w < wv; ++w) {
      const double* o = lds + (w * LPW + li) * (R + 1);
#pragma unroll
      for (int r = 0; r < R; ++r) Fin[r] = o[r] + o[R] * Fin[r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) F[r] += B * Fin[r];
    __syncthreads();
  }
  double Fprev[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    Fprev[r] = __shfl_up(F[r], 1, 64);
    if (ci == 0) Fprev[r] = Fin[r];
  }

  // backward recurrence U_k = H_k + E_k U_{k+1}
  double U[R];
#pragma unroll
  for (int r = 0; r < R; ++r) U[r] = g0w[r] - Q0 * Fprev[r] - C0 * F[r];
  double E = C0 * C1;
  slot_scan_bwd<CPW, R>(U, E);
  double Uin[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Uin[r] = 0.0;
  if constexpr (WPL > 1) {
    double* slot = lds + (wv * LPW + li) * (R + 1);
    if (ci == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) slot[r] = U[r];
      slot[R] = E;
    }
    __syncthreads();
    for (int w = WPL - 1; w > wv; --w) {
      const double* o = lds + (w * LPW + li) * (R + 1);
#pragma unroll
      for (int r = 0; r < R; ++r) Uin[r] = o[r] + o[R] * Uin[r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) U[r] += E * Uin[r];
    __syncthreads();
  }

  // chunk ends and their outer neighbours; interior back substitution
  double xm1[R], xp1[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double un = __shfl_down(U[r], 1, 64);
    if (ci == CPW - 1) un = Uin[r];
    const double xs = U[r];
    const double xe = F[r] - C1 * un;
    xm1[r] = Fprev[r] - cprev * U[r];
    xp1[r] = un;
    v[r][0] = xs;
    v[r][M - 1] = xe;
    F[r] = xs;
    U[r] = xe;
  }
#pragma unroll
  for (int t = 1; t <= M - 2; ++t) {
    ADI_STEP_FENCE();
    const double sp = pos[P_SP * GM + t * G], sr = pos[P_SR * GM + t * G];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r][t] = v[r][t] - sp * F[r] - sr * U[r];
  }

  // outputs: the next half step's right-hand side (and the solution)
  double o[R][M];
#pragma unroll
  for (int t = 0; t < M; ++t) {
    ADI_STEP_FENCE();
    const double od = pos[P_OD * GM + t * G], ol = pos[P_OL * GM + t * G];
    const double ou = pos[P_OU * GM + t * G], oc = pos[P_OC * GM + t * G];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double xl = t > 0 ? v[r][t > 0 ? t - 1 : 0] : xm1[r];
      const double xr = t < M - 1 ? v[r][t < M - 1 ? t + 1 : t] : xp1[r];
      o[r][t] = od * v[r][t] + ol * xl + ou * xr + oc;
      if (a.xc && ((live >> t) & 1ull) && Lfirst + r < Lend)
        o[r][t] += a.xc[(long)a.pos_xclass[p0 + t] * a.nlines + Lfirst + r];
    }
  }
  char* __restrict__ dout = (char*)a.dout;
  char* __restrict__ xout = (char*)a.xout;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool act = Lfirst + r < Lend;
    const long roff = (long)r * ls8;  // uniform
    if (pairs_ok) {
      // cells outside the domain hold 0 in every buffer and come out as 0,
      // so whole pairs inside the line can be stored
#pragma unroll
      for (int t = 0; t < M; t += 2) {
        if (act && t + 1 < inl) {
          *(double2*)(dout + roff + lane_off + t * 8) = make_double2(o[r][t], o[r][t + 1]);
          if (xout) *(double2*)(xout + roff + lane_off + t * 8) = make_double2(v[r][t], v[r][t + 1]);
        } else if (act && t < inl && ((live >> t) & 1ull)) {
          *(double*)(dout + roff + lane_off + t * 8) = o[r][t];
          if (xout) *(double*)(xout + roff + lane_off + t * 8) = v[r][t];
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < M; ++t) {
        if (act && ((live >> t) & 1ull)) {
          const long uoff = roff + (long)t * ps8;
          *(double*)(dout + uoff + lane_off) = o[r][t];
          if (xout) *(double*)(xout + uoff + lane_off) = v[r][t];
        }
      }
    }
  }
}

// ------------------------------------------------------ lane-block solver --

// Loads through a pointer the compiler knows to be global memory.
typedef const __attribute__((address_space(1))) double* gptr;

// The factor-table values one lane needs for its chunk k of a line class:
// interior factors (rows 1..M-2), output scale and constant (all rows),
// reduced-system factors of the chunk.  Loaded once, right behind the
// data loads.
template <int M>
struct LaneTab {
  double w[M], qa[M], cp[M], sp[M], sr[M];
  double ok[M], oc[M];
  double cs, ae, W0, Q0, C0, W1, Q1, C1;
};

// pos/chk: the class tables (uniform across the workgroup), k: the lane's
// chunk, G chunks.  Every load is a uniform base plus a lane offset.  PAIRS:
// paired tables, each pair of fields in one 16-byte load (the single
// problem's strip sweeps, whose table loads cost per instruction); else
// plain tables, one value per load (the batch kernels, which the paired
// layout costs registers and occupancy).
template <int M, int G, bool PAIRS>
__device__ __forceinline__ void load_lanetab(LaneTab<M>& L, const double* pos_, const double* chk_, int k) {
  constexpr int GM = G * M;
  const gptr pos = (gptr)pos_;
  const gptr chk = (gptr)chk_;
  if constexpr (PAIRS) {
    static_assert(G % 2 == 0, "paired fields need 16-byte aligned field arrays");
    // half the load instructions (the sweeps' table loads cost per instruction)
    auto pair = [](const double* p) { return *(const double2*)p; };  // 16-byte aligned
#pragma unroll
    for (int t = 1; t <= M - 2; ++t) {
      const double2 wq = pair(pos_ + pos_at(P_W, GM, t * G + k, true));
      const double2 cs = pair(pos_ + pos_at(P_CP, GM, t * G + k, true));
      L.w[t] = wq.x; L.qa[t] = wq.y;
      L.cp[t] = cs.x; L.sp[t] = cs.y;
      L.sr[t] = pos[pos_at(P_SR, GM, t * G + k, true)];
    }
#pragma unroll
    for (int t = 0; t < M; ++t) {
      const double2 ck = pair(pos_ + pos_at(P_OC, GM, t * G + k, true));
      L.oc[t] = ck.x; L.ok[t] = ck.y;
    }
    const double2 c0 = pair(chk_ + chk_at(C_CS, G, k, true)), c1 = pair(chk_ + chk_at(C_W0, G, k, true));
    const double2 c2 = pair(chk_ + chk_at(C_C0, G, k, true)), c3 = pair(chk_ + chk_at(C_Q1, G, k, true));
    L.cs = c0.x; L.ae = c0.y;
    L.W0 = c1.x; L.Q0 = c1.y;
    L.C0 = c2.x; L.W1 = c2.y;
    L.Q1 = c3.x; L.C1 = c3.y;
  } else {
    // plain tables, one value per load
#pragma unroll
    for (int t = 1; t <= M - 2; ++t) {
      L.w[t] = pos[P_W * GM + t * G + k];
      L.qa[t] = pos[P_QA * GM + t * G + k];
      L.cp[t] = pos[P_CP * GM + t * G + k];
      L.sp[t] = pos[P_SP * GM + t * G + k];
      L.sr[t] = pos[P_SR * GM + t * G + k];
    }
#pragma unroll
    for (int t = 0; t < M; ++t) {
      L.ok[t] = pos[P_OK * GM + t * G + k];
      L.oc[t] = pos[P_OC * GM + t * G + k];
    }
    L.cs = chk[C_CS * G + k]; L.ae = chk[C_AE * G + k];
    L.W0 = chk[C_W0 * G + k]; L.Q0 = chk[C_Q0 * G + k]; L.C0 = chk[C_C0 * G + k];
    L.W1 = chk[C_W1 * G + k]; L.Q1 = chk[C_Q1 * G + k]; L.C1 = chk[C_C1 * G + k];
  }
}

// Solve a block of R lines in place.  Lane k = 64*wave + lane holds chunk
// k (M cells) of each of the R lines in v[R][M]; the NW waves of the
// workgroup hold the G = 64*NW chunks of the lines.  With CPW < 64 (one
// wave), each slot of CPW consecutive lanes holds its own R lines of CPW
// chunks.  Lines r < NA have the
// factors LA, the others LB (a block whose lines span two classes; NA = R:
// one class, LB unused).  Same partition method as solve_group (interior
// elimination with the class's precomputed factors, reduced system by
// recursive doubling over the chunks, back substitution), with data and
// factors already in registers.  Cells outside the domain and past the
// line's end are identity rows carrying exactly 0 in every right-hand side,
// so they solve to 0 without masking.  `lds` holds 2*NW*(R+2) doubles.
// Every lane of the workgroup must call this (it contains barriers when
// NW > 1).
template <int M, int NW, int R, int NA, int CPW = 64>
__device__ __forceinline__ void solve_lanes(double (*v)[M], const LaneTab<M>& LA, const LaneTab<M>& LB,
                                            double* lds) {
  static_assert(M >= 3, "chunks need an interior row");
  static_assert(NA >= 1 && NA <= R, "split");
  static_assert(NW == 1 || CPW == 64, "lines narrower than a wave stay inside it");
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int ci = lane & (CPW - 1);  // chunk within the lane's slot of CPW lanes
#define ADI_TAB(r) ((r) < NA ? LA : LB)

  // interior forward elimination and back substitution (rows 1..M-2)
  double run[R];
#pragma unroll
  for (int r = 0; r < R; ++r) run[r] = 0.0;
#pragma unroll
  for (int t = 1; t <= M - 2; ++t)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      run[r] = v[r][t] * ADI_TAB(r).w[t] - ADI_TAB(r).qa[t] * run[r];
      v[r][t] = run[r];
    }
#pragma unroll
  for (int r = 0; r < R; ++r) run[r] = 0.0;
#pragma unroll
  for (int t = M - 2; t >= 1; --t)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      run[r] = v[r][t] - ADI_TAB(r).cp[t] * run[r];
      v[r][t] = run[r];
    }

  // reduced system, forward recurrence over the chunks
  double g0w[R], F[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const LaneTab<M>& L = ADI_TAB(r);
    g0w[r] = (v[r][0] - L.cs * v[r][1]) * L.W0;
    F[r] = (v[r][M - 1] - L.ae * v[r][M - 2]) * L.W1 - L.Q1 * g0w[r];
  }
  double BA = LA.Q1 * LA.Q0, BB = LB.Q1 * LB.Q0;
  slot_scan_fwd<CPW, R, NA>(F, BA, BB);
  double Fin[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Fin[r] = 0.0;
  if constexpr (NW > 1) {
    double* slots = lds;  // forward totals of the waves
    if (lane == 63) {
#pragma unroll
      for (int r = 0; r < R; ++r) slots[wv * (R + 2) + r] = F[r];
      slots[wv * (R + 2) + R] = BA;
      slots[wv * (R + 2) + R + 1] = BB;
    }
    __syncthreads();
    for (int w = 0; w < wv; ++w) {
      const double* q = slots + w * (R + 2);
#pragma unroll
      for (int r = 0; r < R; ++r) Fin[r] = q[r] + q[r < NA ? R : R + 1] * Fin[r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) F[r] += (r < NA ? BA : BB) * Fin[r];
  }
  double Fprev[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    Fprev[r] = __shfl_up(F[r], 1, 64);
    if (ci == 0) Fprev[r] = Fin[r];
  }

  // backward recurrence
  double U[R];
#pragma unroll
  for (int r = 0; r < R; ++r) U[r] = g0w[r] - ADI_TAB(r).Q0 * Fprev[r] - ADI_TAB(r).C0 * F[r];
  double EA = LA.C0 * LA.C1, EB = LB.C0 * LB.C1;
  slot_scan_bwd<CPW, R, NA>(U, EA, EB);
  double Uin[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Uin[r] = 0.0;
  if constexpr (NW > 1) {
    double* slots = lds + NW * (R + 2);  // backward totals (separate: no barrier between phases)
    if (lane == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) slots[wv * (R + 2) + r] = U[r];
      slots[wv * (R + 2) + R] = EA;
      slots[wv * (R + 2) + R + 1] = EB;
    }
    __syncthreads();
    for (int w = NW - 1; w > wv; --w) {
      const double* q = slots + w * (R + 2);
#pragma unroll
      for (int r = 0; r < R; ++r) Uin[r] = q[r] + q[r < NA ? R : R + 1] * Uin[r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) U[r] += (r < NA ? EA : EB) * Uin[r];
  }

  // chunk ends, interior back substitution
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double un = __shfl_down(U[r], 1, 64);
    if (ci == CPW - 1) un = Uin[r];
    const double xs = U[r];
    const double xe = F[r] - ADI_TAB(r).C1 * un;
    v[r][0] = xs;
    v[r][M - 1] = xe;
    F[r] = xs;
    U[r] = xe;
  }
#pragma unroll
  for (int t = 1; t <= M - 2; ++t)
#pragma unroll
    for (int r = 0; r < R; ++r) v[r][t] = v[r][t] - ADI_TAB(r).sp[t] * F[r] - ADI_TAB(r).sr[t] * U[r];
#undef ADI_TAB
}

// The next half step's right-hand side of line r of a block at chunk
// offset t, from the solution x and the right-hand side d the line was
// solved with: with a x[-1] + b x + c x[+1] = d the output operator
// od x + ol x[-1] + ou x[+1] + oc (eq. 8-9: the explicit half of the
// same direction) equals ok x - theta d + oc, so no neighbour is needed.
// Outside the domain ok = oc = 0 and x = d = 0, so the result is 0.
__device__ __forceinline__ double next_rhs(double ok, double oc, double theta, double x, double d) {
  return fma(ok, x, fma(-theta, d, oc));
}

}  // namespace adi
