// resident.hpp -- the whole time loop of a small grid in one workgroup, with
// the carried right-hand side resident in LDS.
//
// For grids whose field fits in LDS (the single layout of Fig. 1 at 64 x 160
// is 80 KB) launching two sweeps per step costs more than the sweeps
// themselves.  Here one workgroup of 1024 lanes keeps the right-hand side in
// LDS for every step of a run.  Each half step solves its lines by the
// partition method (the decomposition of the streaming sweeps, mapped the
// other way round): a line per lane, 64 lines per wave, and the cells of a
// line cut into L chunks of M cells, one chunk per wave, so that a lane keeps
// its chunk in registers from the load to the store.
//   A. every lane eliminates the interior rows of its chunk with the class's
//      precomputed factors (interior unknowns in terms of the chunk's first
//      and last unknowns, through two precomputed spike vectors) and writes
//      its chunk's two rows of the reduced system;
//   B. the reduced system of each line (2L unknowns, the chunk ends) is
//      solved by two waves per 64 lines, one eliminating from the first row
//      and one from the last, meeting in the middle (the two-ended form of
//      the Thomas recurrence);
//   C. every lane substitutes the chunk ends into its interior and writes
//      the next half step's right-hand side in place: with a x[-1] + b x +
//      c x[+1] = d, the explicit operator of the same direction (eq. 10-11)
//      plus the source and boundary constants equals ok x - theta d + oc, so
//      no neighbour is read.
// Every line of a class (an r band or a z column class) has the same matrix,
// so all factors are computed once per launch into LDS.  Per cell and half
// step a lane reads its right-hand side and six factors and writes the
// result, each once.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace adi {

constexpr int RES_THREADS = 1024;
constexpr int RES_WAVES = RES_THREADS / 64;
constexpr int RES_MMAX = 16;  // cells per chunk held in registers
constexpr int RP_NFIELDS_ = 7, RQ_NFIELDS_ = 2, RR_NFIELDS_ = 4;  // table fields (the enums below)

// Partition of one direction: nl lines of n cells in g groups of up to 64
// lines, each line in L chunks of M cells (L*M >= n; cells past n are
// identity rows).
struct ResShape {
  int nl, n, g, L, M;
  int ps, qs, rs;  // per-class strides of the position, chunk and reduced-row tables
};

// Per-class table stride (unpadded: padding the strides apart in the LDS
// banks measured no faster).
__host__ __device__ inline int res_cstride(long x) { return (int)x; }

__host__ __device__ inline ResShape res_shape(int nl, int n) {
  ResShape s;
  s.nl = nl;
  s.n = n;
  s.g = (nl + 63) / 64;
  int L = RES_WAVES / (s.g > 0 ? s.g : 1);
  if (L > n / 2) L = n / 2;  // at least two cells per chunk
  if (L < 1) L = 1;
  s.L = L;
  s.M = (n + L - 1) / L;
  s.ps = res_cstride((long)RP_NFIELDS_ * L * s.M);
  s.qs = res_cstride((long)RQ_NFIELDS_ * L);
  s.rs = res_cstride((long)RR_NFIELDS_ * 2 * L);
  return s;
}

// Per-position factors of a class, [field][L*M]: l (interior forward
// elimination), g (interior back substitution, scaled by the pivots), K1..K3
// (the output scale folded with the interior solution and the two spikes),
// oc, ok.
enum ResPosField { RP_L = 0, RP_G, RP_K1, RP_K2, RP_K3, RP_OC, RP_OK, RP_NFIELDS };
static_assert(RP_NFIELDS == RP_NFIELDS_, "position fields");
// Per chunk: c_0 / u_1 and a_{M-1} / u_{M-2} (the reduced right-hand sides).
enum ResChunkField { RQ_CW = 0, RQ_AW, RQ_NFIELDS };
static_assert(RQ_NFIELDS == RQ_NFIELDS_, "chunk fields");
// Per reduced row, [field][2L]: sub- and super-diagonal, inverse pivots of
// the two-ended elimination, back-substitution factors.
enum ResRedField { RR_A = 0, RR_C, RR_INV, RR_CF, RR_NFIELDS };
static_assert(RR_NFIELDS == RR_NFIELDS_, "reduced-row fields");
// Set-up work area per position: a, b, c, ok, oc.
enum ResWorkField { RW_A = 0, RW_B, RW_C, RW_OK, RW_OC, RW_NFIELDS };

struct ResLayout {
  ResShape s[2];                 // 0: r lines (nz lines of nr cells), 1: z lines
  int ldd;                       // row stride of the right-hand side (odd: no bank conflicts in the r sweeps)
  long work[2], wred[2];         // set-up work areas (in region 0, which then holds the right-hand side)
  long tp[2], tq[2], tr[2];      // factor tables
  long red, xch, cls, total;     // reduced systems, middle exchange, class bytes; doubles in all
};

__host__ __device__ inline ResLayout res_layout(int nr, int nz) {
  ResLayout y;
  y.s[0] = res_shape(nz, nr);
  y.s[1] = res_shape(nr, nz);
  y.ldd = nr | 1;
  const int ncls[2] = {3, 4};
  long o = 0;
  for (int d = 0; d < 2; ++d) {
    y.work[d] = o;
    o += (long)RW_NFIELDS * ncls[d] * y.s[d].L * y.s[d].M;
    y.wred[d] = o;
    o += 3L * ncls[d] * 2 * y.s[d].L;
  }
  o = o > (long)nz * y.ldd ? o : (long)nz * y.ldd;
  long red = 0, xch = 0;
  for (int d = 0; d < 2; ++d) {
    const long LM = (long)y.s[d].L * y.s[d].M;
    y.tp[d] = o;
    o += (long)y.s[d].ps * ncls[d];
    y.tq[d] = o;
    o += (long)y.s[d].qs * ncls[d];
    y.tr[d] = o;
    o += (long)y.s[d].rs * ncls[d];
    const long r = 2L * y.s[d].L * 64 * y.s[d].g, x = 2L * 64 * y.s[d].g;
    red = red > r ? red : r;
    xch = xch > x ? xch : x;
  }
  y.red = o;
  o += red;
  y.xch = o;
  o += xch;
  y.cls = o;
  o += (nr + nz + 7) / 8;
  y.total = o;
  return y;
}

// LDS doubles the kernel needs.
__host__ __device__ inline long resident_lds_doubles(int nr, int nz) { return res_layout(nr, nz).total; }

// Whether the partition suits the kernel (the LDS size is the caller's
// check): at least 3 cells per line, at most RES_MMAX cells per chunk and two
// waves per group of lines.
__host__ __device__ inline bool resident_shape_ok(int nr, int nz) {
  if (nr < 3 || nz < 3) return false;
  const ResLayout y = res_layout(nr, nz);
  for (int d = 0; d < 2; ++d)
    if (y.s[d].M > RES_MMAX || 2 * y.s[d].g > RES_WAVES) return false;
  return true;
}

struct ResArgs {
  Params P;
  Geom g;
  double* rhs;          // carried right-hand side of the next r sweep (rows layout), read and written
  double* T;            // the field after the last step (written when write_T)
  const double* xcr;    // [band][nr] ambient constants the z sweep's output adds (null: none)
  const double* xcz;    // [column class][nz] ambient constants the r sweep's output adds (null: none)
  int nsteps;
  int write_T;
};

// Set-up of chunk k of one class (one lane): interior Thomas factors,
// spikes, the chunk's two reduced rows and the folded output factors.  W:
// the class's work arrays (RW fields, L*M each), tp / tq: its tables, wr: its
// reduced rows (lower, diagonal, upper; 2L each).
__device__ inline void res_chunk_setup(const double* W, double* tp, double* tq, double* wr, int L, int M, int k) {
  const long LM = (long)L * M;
  const int p0 = k * M;
  const double* A = W + RW_A * LM + p0;
  const double* B = W + RW_B * LM + p0;
  const double* C = W + RW_C * LM + p0;
  const double* OK = W + RW_OK * LM + p0;
  double* TL = tp + RP_L * LM + p0;
  double* TG = tp + RP_G * LM + p0;
  double* K1 = tp + RP_K1 * LM + p0;
  double* K2 = tp + RP_K2 * LM + p0;
  double* K3 = tp + RP_K3 * LM + p0;
  for (int q = 0; q < M; ++q) {
    tp[RP_OC * LM + p0 + q] = W[RW_OC * LM + p0 + q];
    tp[RP_OK * LM + p0 + q] = OK[q];
    TL[q] = TG[q] = K1[q] = K2[q] = K3[q] = 0.0;
  }
  double lo0, di0, up0, lo1, di1, up1, cw = 0.0, aw = 0.0;
  if (M >= 3) {
    // interior rows 1..M-2: unit-lower LU, 1/u kept in K1 for now
    double u = B[1];
    K1[1] = 1.0 / u;
    for (int q = 2; q <= M - 2; ++q) {
      const double l = A[q] / u;
      u = B[q] - l * C[q - 1];
      TL[q] = l;
      K1[q] = 1.0 / u;
    }
    for (int q = 1; q <= M - 3; ++q) TG[q] = C[q] * K1[q + 1];
    // spikes: s = T_I^{-1} (a_1 e_1) in K2, t = T_I^{-1} (c_{M-2} e_{M-2}) in K3
    double zs = A[1];
    K2[1] = zs;
    for (int q = 2; q <= M - 2; ++q) {
      zs = -TL[q] * zs;
      K2[q] = zs;
    }
    K2[M - 2] = K2[M - 2] * K1[M - 2];
    for (int q = M - 3; q >= 1; --q) K2[q] = (K2[q] - C[q] * K2[q + 1]) * K1[q];
    K3[M - 2] = C[M - 2] * K1[M - 2];
    for (int q = M - 3; q >= 1; --q) K3[q] = -C[q] * K3[q + 1] * K1[q];
    // the chunk's first and last rows with the interior substituted
    lo0 = A[0];
    di0 = B[0] - C[0] * K2[1];
    up0 = -C[0] * K3[1];
    lo1 = -A[M - 1] * K2[M - 2];
    di1 = B[M - 1] - A[M - 1] * K3[M - 2];
    up1 = C[M - 1];
    cw = C[0] * K1[1];
    aw = A[M - 1] * K1[M - 2];
    for (int q = 1; q <= M - 2; ++q) {
      K1[q] = OK[q] * K1[q];
      K2[q] = OK[q] * K2[q];
      K3[q] = OK[q] * K3[q];
    }
  } else {
    lo0 = A[0];
    di0 = B[0];
    up0 = C[0];
    lo1 = A[1];
    di1 = B[1];
    up1 = C[1];
  }
  // chunk ends: x_0 = F, x_{M-1} = X
  K2[0] = -OK[0];
  K3[M - 1] = -OK[M - 1];
  tq[RQ_CW * L + k] = cw;
  tq[RQ_AW * L + k] = aw;
  const int L2 = 2 * L;
  wr[2 * k] = lo0;
  wr[L2 + 2 * k] = di0;
  wr[2 * L2 + 2 * k] = up0;
  wr[2 * k + 1] = lo1;
  wr[L2 + 2 * k + 1] = di1;
  wr[2 * L2 + 2 * k + 1] = up1;
}

// Two-ended factorisation of one class's reduced system (2L rows): side 0
// rows 0..L-1 from the first row, side 1 rows 2L-1..L+1 from the last.
__device__ inline void res_reduced_factor(const double* wr, double* tr, int L, int side) {
  const int L2 = 2 * L, m = L;
  const double* lo = wr;
  const double* di = wr + L2;
  const double* up = wr + 2 * L2;
  double* RA = tr + RR_A * L2;
  double* RC = tr + RR_C * L2;
  double* RI = tr + RR_INV * L2;
  double* RF = tr + RR_CF * L2;
  double prev = 0.0;
  if (side == 0) {
    for (int i = 0; i < m; ++i) {
      RI[i] = 1.0 / (di[i] - lo[i] * prev);
      RA[i] = lo[i];
      RC[i] = up[i];
      RF[i] = up[i] * RI[i];
      prev = RF[i];
    }
    RA[m] = lo[m];
    RC[m] = up[m];
  } else {
    for (int i = L2 - 1; i > m; --i) {
      RI[i] = 1.0 / (di[i] - up[i] * prev);
      RA[i] = lo[i];
      RC[i] = up[i];
      RF[i] = lo[i] * RI[i];
      prev = RF[i];
    }
  }
}

// Factor loads run at most four cells ahead of their use (a measured gain:
// hoisting all of a chunk's loads queues them behind each other in LDS).
#define RES_FENCE(q)                                        \
  do {                                                      \
    if ((q) % 4 == 3) __builtin_amdgcn_sched_barrier(0);    \
  } while (0)

// LDS pointers (address space 3, so that a separately compiled sweep
// still addresses LDS directly).
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

// One half step in direction DIR, M cells per chunk, over the right-hand
// side in LDS.  lcls: class of each line; xcls: crossing class of each
// position, for the ambient constants xc ([crossing class][nl], from the
// other direction; null: none).  T: the solution is stored too (the last
// step's z sweep).  Every lane of the workgroup calls this.
// Each instance is compiled as a function of its own: inlined into the time
// loop, the loop-invariant address arithmetic of every instance would be
// hoisted out of it and exhaust the registers.
template <int DIR, int M, bool LAST>
__device__ __attribute__((noinline)) void res_sweep(
    const ResShape S, const int ldd, lds_f64* __restrict__ D, lds_f64* __restrict__ red, lds_f64* __restrict__ xch,
    const lds_f64* __restrict__ tpos, const lds_f64* __restrict__ tchk, const lds_f64* __restrict__ tred,
    const lds_u8* __restrict__ lcls, const lds_u8* __restrict__ xcls, const double* __restrict__ xc, double theta,
    double* __restrict__ T) {
  const int nl = S.nl, n = S.n, L = S.L, L2 = 2 * L;
  const long LM = (long)L * M;
  const long NLP = 64L * S.g;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  // ---- A: interior elimination and the reduced right-hand sides
  const bool inA = w < S.g * L;
  const int grp = inA ? w / L : 0, k = inA ? w % L : 0;
  const int ln = grp * 64 + lane;
  const bool act = inA && ln < nl;
  const int lnc = act ? ln : nl - 1;  // lanes past the last line load a real line and store nothing
  const int cls = lcls[lnc];
  const lds_f64* tp = tpos + (long)cls * S.ps + (long)k * M;
  const lds_f64* tq = tchk + (long)cls * S.qs;
  const long lbase = DIR == 0 ? (long)lnc * ldd : (long)lnc;
  const long pst = DIR == 0 ? 1 : ldd;
  const int p0 = k * M;
  double v[M], dd[M];
  if (inA) {
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const int p = p0 + q < n ? p0 + q : n - 1;
      const double x = D[lbase + p * pst];
      dd[q] = p0 + q < n ? x : 0.0;
      v[q] = 0.0;
    }
    if constexpr (M >= 3) {
      // interior forward elimination (rows 1..M-2), then back substitution
      // scaled by the pivots
      double z = dd[1];
      v[1] = z;
#pragma unroll
      for (int q = 2; q <= M - 2; ++q) {
        z = dd[q] - tp[RP_L * LM + q] * z;
        v[q] = z;
        RES_FENCE(q);
      }
#pragma unroll
      for (int q = M - 3; q >= 1; --q) {
        v[q] = v[q] - tp[RP_G * LM + q] * v[q + 1];
        RES_FENCE(q);
      }
    }
    if (act) {
      red[(2 * k) * NLP + ln] = M >= 3 ? dd[0] - tq[RQ_CW * L + k] * v[1] : dd[0];
      red[(2 * k + 1) * NLP + ln] = M >= 3 ? dd[M - 1] - tq[RQ_AW * L + k] * v[M > 2 ? M - 2 : 0] : dd[M - 1];
    }
    if constexpr (!LAST) {
      // everything of the output but the chunk-end terms, kept in v: the
      // right-hand side is not needed after this
#pragma unroll
      for (int q = 0; q < M; ++q) {
        v[q] = tp[RP_K1 * LM + q] * v[q] + tp[RP_OC * LM + q] - theta * dd[q];
        RES_FENCE(q);
      }
      if (xc) {
#pragma unroll
        for (int q = 0; q < M; ++q) v[q] += xc[(long)xcls[p0 + q < n ? p0 + q : n - 1] * nl + lnc];
      }
    }
  }
  __syncthreads();
  // ---- B: the reduced systems, two waves per group of 64 lines, rows
  // loaded four at a time ahead of their recurrence steps
  const bool inB = w < 2 * S.g;
  const int side = w & 1;
  const int bl = (w >> 1) * 64 + lane;
  const bool bact = inB && bl < nl;
  const lds_f64* tr = tred + (long)(bact ? lcls[bl] : 0) * S.rs;
  const lds_f64* RA = tr + RR_A * L2;
  const lds_f64* RC = tr + RR_C * L2;
  const lds_f64* RI = tr + RR_INV * L2;
  const lds_f64* RF = tr + RR_CF * L2;
  const int m = L;
  if (bact) {
    double h = 0.0;
    if (side == 0) {
      for (int i0 = 0; i0 < m; i0 += 4) {
        double r[4], c4[4], iv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + u < m ? i0 + u : m - 1;
          r[u] = red[i * NLP + bl];
          c4[u] = RA[i];
          iv[u] = RI[i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + u < m) {
            h = (r[u] - c4[u] * h) * iv[u];
            red[(i0 + u) * NLP + bl] = h;
          }
      }
      xch[bl] = red[m * NLP + bl] - RA[m] * h;
    } else {
      for (int i0 = L2 - 1; i0 > m; i0 -= 4) {
        double r[4], c4[4], iv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 - u > m ? i0 - u : m + 1;
          r[u] = red[i * NLP + bl];
          c4[u] = RC[i];
          iv[u] = RI[i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 - u > m) {
            h = (r[u] - c4[u] * h) * iv[u];
            red[(i0 - u) * NLP + bl] = h;
          }
      }
      xch[NLP + bl] = RC[m] * h;
    }
  }
  __syncthreads();
  if (bact) {
    const double xm = (xch[bl] - xch[NLP + bl]) * RI[m];
    double x = xm;
    if (side == 0) {
      red[m * NLP + bl] = xm;
      for (int i0 = m - 1; i0 >= 0; i0 -= 4) {
        double r[4], f4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 - u >= 0 ? i0 - u : 0;
          r[u] = red[i * NLP + bl];
          f4[u] = RF[i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 - u >= 0) {
            x = r[u] - f4[u] * x;
            red[(i0 - u) * NLP + bl] = x;
          }
      }
    } else {
      for (int i0 = m + 1; i0 < L2; i0 += 4) {
        double r[4], f4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + u < L2 ? i0 + u : L2 - 1;
          r[u] = red[i * NLP + bl];
          f4[u] = RF[i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + u < L2) {
            x = r[u] - f4[u] * x;
            red[(i0 + u) * NLP + bl] = x;
          }
      }
    }
  }
  __syncthreads();
  // ---- C: substitution and the next right-hand side, in place
  if (act) {
    const double F = red[(2 * k) * NLP + ln];
    const double X = red[(2 * k + 1) * NLP + ln];
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const int p = p0 + q;
      if constexpr (LAST) {
        // the last step also stores the solution: ok x, then x
        const double okx = tp[RP_K1 * LM + q] * v[q] - tp[RP_K2 * LM + q] * F - tp[RP_K3 * LM + q] * X;
        double o = okx + tp[RP_OC * LM + q] - theta * dd[q];
        if (xc) o += xc[(long)xcls[p < n ? p : n - 1] * nl + ln];
        if (p < n) {
          D[lbase + p * pst] = o;
          const double ok = tp[RP_OK * LM + q];
          T[DIR == 0 ? (long)ln * n + p : (long)p * nl + ln] = ok != 0.0 ? okx / ok : 0.0;
        }
      } else {
        const double o = v[q] - tp[RP_K2 * LM + q] * F - tp[RP_K3 * LM + q] * X;
        if (p < n) D[lbase + p * pst] = o;
      }
      RES_FENCE(q);
    }
  }
  __syncthreads();
}

#undef RES_FENCE

// The half step of direction DIR at the direction's chunk size.
template <int DIR>
__device__ __forceinline__ void res_half_step(const ResLayout& Y, double* lds, const uint8_t* lcls,
                                              const uint8_t* xcls, const double* xc, double theta, double* T) {
  lds_f64* D = (lds_f64*)lds;
  lds_f64* red = (lds_f64*)(lds + Y.red);
  lds_f64* xch = (lds_f64*)(lds + Y.xch);
  const lds_f64* tp = (const lds_f64*)(lds + Y.tp[DIR]);
  const lds_f64* tq = (const lds_f64*)(lds + Y.tq[DIR]);
  const lds_f64* tr = (const lds_f64*)(lds + Y.tr[DIR]);
  const lds_u8* lc = (const lds_u8*)lcls;
  const lds_u8* xk = (const lds_u8*)xcls;
  const ResShape S = Y.s[DIR];
#define ADI_RES_CASE(MM)                                                                        \
  case MM:                                                                                      \
    if (DIR == 1 && T)                                                                          \
      res_sweep<DIR, MM, DIR == 1>(S, Y.ldd, D, red, xch, tp, tq, tr, lc, xk, xc, theta, T);    \
    else                                                                                        \
      res_sweep<DIR, MM, false>(S, Y.ldd, D, red, xch, tp, tq, tr, lc, xk, xc, theta, T);       \
    break;
  switch (S.M) {
    ADI_RES_CASE(2) ADI_RES_CASE(3) ADI_RES_CASE(4) ADI_RES_CASE(5) ADI_RES_CASE(6) ADI_RES_CASE(7)
    ADI_RES_CASE(8) ADI_RES_CASE(9) ADI_RES_CASE(10) ADI_RES_CASE(11) ADI_RES_CASE(12) ADI_RES_CASE(13)
    ADI_RES_CASE(14) ADI_RES_CASE(15) ADI_RES_CASE(16)
    default: break;
  }
#undef ADI_RES_CASE
}

// The time loop: nsteps steps of (r sweep, z sweep) from the carried
// right-hand side rhs, which it leaves carried again; T receives the field
// after the last step when write_T is set.  One workgroup of RES_THREADS
// lanes; needs resident_shape_ok(nr, nz) and resident_lds_doubles(nr, nz)
// doubles of dynamic LDS.
__global__ void __launch_bounds__(RES_THREADS) k_resident(ResArgs a) {
  HIP_DYNAMIC_SHARED(double, lds)
  const int nr = a.P.nr, nz = a.P.nz;
  const ResLayout Y = res_layout(nr, nz);
  const int t = threadIdx.x, nt = blockDim.x;
  uint8_t* kap = (uint8_t*)(lds + Y.cls);
  uint8_t* bet = kap + nr;
  for (int i = t; i < nr; i += nt) kap[i] = a.g.kap[i];
  for (int j = t; j < nz; j += nt) bet[j] = a.g.bet[j];
  // row coefficients of every class and position (cells past the line are
  // identity rows)
  const int ncls[2] = {3, 4};
  for (int d = 0; d < 2; ++d) {
    const long LM = (long)Y.s[d].L * Y.s[d].M;
    for (long q = t; q < ncls[d] * LM; q += nt) {
      const int c = (int)(q / LM), p = (int)(q % LM);
      const RowCoef R = row_coef(a.P, a.g, d, c, p);
      double* W = lds + Y.work[d] + (long)c * RW_NFIELDS * LM;
      W[RW_A * LM + p] = R.a;
      W[RW_B * LM + p] = R.b;
      W[RW_C * LM + p] = R.c;
      W[RW_OK * LM + p] = R.ok;
      W[RW_OC * LM + p] = R.oc;
    }
  }
  __syncthreads();
  // chunk factors: one lane per (direction, class, chunk)
  for (int q = t; q < 3 * Y.s[0].L + 4 * Y.s[1].L; q += nt) {
    const int d = q < 3 * Y.s[0].L ? 0 : 1;
    const int r = d == 0 ? q : q - 3 * Y.s[0].L;
    const int L = Y.s[d].L, M = Y.s[d].M, c = r / L, k = r % L;
    const long LM = (long)L * M;
    res_chunk_setup(lds + Y.work[d] + (long)c * RW_NFIELDS * LM, lds + Y.tp[d] + (long)c * Y.s[d].ps,
                    lds + Y.tq[d] + (long)c * Y.s[d].qs, lds + Y.wred[d] + (long)c * 3 * 2 * L, L, M, k);
  }
  __syncthreads();
  // reduced-system factors: one lane per (direction, class, side), then the
  // middle pivots
  if (t < 14) {
    const int d = t < 6 ? 0 : 1;
    const int c = (d == 0 ? t : t - 6) >> 1;
    const int L = Y.s[d].L;
    res_reduced_factor(lds + Y.wred[d] + (long)c * 3 * 2 * L, lds + Y.tr[d] + (long)c * Y.s[d].rs, L,
                       t & 1);
  }
  __syncthreads();
  if (t < 7) {
    const int d = t < 3 ? 0 : 1, c = d == 0 ? t : t - 3;
    const int L = Y.s[d].L, L2 = 2 * L, m = L;
    const double* wr = lds + Y.wred[d] + (long)c * 3 * L2;
    double* tr = lds + Y.tr[d] + (long)c * Y.s[d].rs;
    double piv = wr[L2 + m] - wr[m] * tr[RR_CF * L2 + m - 1];
    if (m + 1 < L2) piv -= wr[2 * L2 + m] * tr[RR_CF * L2 + m + 1];
    tr[RR_INV * L2 + m] = 1.0 / piv;
  }
  __syncthreads();
  double* D = lds;
  for (long e = t; e < (long)nr * nz; e += nt) D[(e / nr) * Y.ldd + e % nr] = a.rhs[e];
  __syncthreads();
  for (int s = 0; s < a.nsteps; ++s) {
    const bool last = s == a.nsteps - 1;
    // the r sweep's output adds the z constants, the z sweep's the r ones
    res_half_step<0>(Y, lds, bet, kap, a.xcz, a.P.theta, nullptr);
    res_half_step<1>(Y, lds, kap, bet, a.xcr, a.P.theta, last && a.write_T ? a.T : nullptr);
  }
  for (long e = t; e < (long)nr * nz; e += nt) a.rhs[e] = D[(e / nr) * Y.ldd + e % nr];
}

}  // namespace adi
