// strip.hpp -- sweeps over right-hand sides stored in strips of 4 columns.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace adi {

// Workgroups are dealt to the 8 XCDs round-robin by block index; remap so
// that each XCD gets one contiguous range of line groups, which keeps
// neighbouring lines (sharing cache lines in the strided direction) in one
// L2.  A bijection on [0, nblocks).
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  constexpr int NX = 8;
  const int q = nblocks / NX, rem = nblocks % NX;
  const int x = b % NX, slot = b / NX;
  return x * q + (x < rem ? x : rem) + slot;
}

// ----------------------------------------------------- strip layout ----
//
// Alternative storage of the carried right-hand sides for coalesced sweeps
// in both directions: the columns are grouped in strips of 4, each strip is
// one contiguous array of rows of 4 doubles (element (j, i) at
// (i/4)*strip + 4*j + i%4, with strip = 16*ceil(nz/4) doubles: 4*ceil(nz/4)
// rows).  A z sweep then
// reads and writes one contiguous block per strip; an r sweep over 4
// consecutive rows touches one whole 128-byte tile per strip.  Both kernels
// stage their block through LDS with fully coalesced copies, and each lane
// solves the same chunk of 4 lines, so every table value it loads serves
// 4 lines.

struct StripArgs {
  const double* din;        // right-hand side of this half step (strip layout)
  double* dout;             // right-hand side of the next half step (strip layout)
  double* xout;             // solution in the plain layout (nz rows of nr), or null
  LineTab tabs[MAX_CLS];    // line-class tables of this direction
  const double* xc;         // [crossing class][line] constants of the other direction, or null
  long strip;               // doubles per strip
  int nr, nz;
  int nlines;               // lines of this direction
  int nblocks;              // strips (z sweep) or row groups (r sweep)
  int line_end[3];          // class of line l: number of q with l >= line_end[q]
  int pos_end[3];           // crossing class of position p: number of q with p >= pos_end[q]
  int nxcls;                // crossing classes
  int nmix;                 // blocks whose 4 lines are not all of one class ...
  int mix[4];               // ... solved one line per workgroup by nblocks + 4*m + line
};

__device__ __forceinline__ int class_at(const int* ends, int x) {
  return (x >= ends[0]) + (x >= ends[1]) + (x >= ends[2]);
}

// Which block and which of its lines a workgroup takes: b < nblocks is block
// b with all its lines (lc = -1) unless the block is mixed (then nothing);
// b >= nblocks is line lc of mixed block mix[(b - nblocks) / 4].
__device__ __forceinline__ bool strip_work(const StripArgs& a, int b, int* blk, int* lc) {
  if (b < a.nblocks) {
    for (int m = 0; m < a.nmix; ++m)
      if (a.mix[m] == b) return false;
    *blk = b;
    *lc = -1;
    return true;
  }
  *blk = a.mix[(b - a.nblocks) >> 2];
  *lc = (b - a.nblocks) & 3;
  return true;
}

// Crossing constants of the block's lines: xcv[c][r] for crossing class c
// and line line0 + r (uniform across the workgroup).
template <int R>
__device__ __forceinline__ void load_crossing(const StripArgs& a, int line0, int nact, double (*xcv)[R]) {
#pragma unroll
  for (int c = 0; c < MAX_CLS; ++c)
#pragma unroll
    for (int r = 0; r < R; ++r)
      xcv[c][r] = (c < a.nxcls && r < nact) ? a.xc[(long)c * a.nlines + line0 + r] : 0.0;
}

template <int M, int R>
__device__ __forceinline__ void add_crossing(const StripArgs& a, double (*o)[M], const double (*xcv)[R],
                                             unsigned long long live, int p0) {
#pragma unroll
  for (int t = 0; t < M; ++t) {
    if (!((live >> t) & 1ull)) continue;
    const int c = class_at(a.pos_end, p0 + t);
#pragma unroll
    for (int r = 0; r < R; ++r)
      o[r][t] += c == 0 ? xcv[0][r] : (c == 1 ? xcv[1][r] : (c == 2 ? xcv[2][r] : xcv[3][r]));
  }
}

// z sweep: workgroup per strip (4 adjacent columns), lane k holds rows
// [kM, kM+M) of the strip's columns.
template <int M, int NW>
__global__ void __launch_bounds__(64 * NW) k_sweep_zs(StripArgs a) {
  constexpr int NT = 64 * NW;
  constexpr int CH = 4 * M;  // LDS doubles per chunk
  // The staged strip takes exactly 64*NW*4*M doubles (80 KB for a 2560-row
  // strip), so that two workgroups fit in one compute unit's LDS; the
  // solver's carries live in the same buffer while the data sit in
  // registers.
  __shared__ __align__(16) double buf[NT * CH];
  double* carry = buf;
  static_assert(NT * CH >= NW * 5, "carry slots");
  int s, lc;
  if (!strip_work(a, xcd_block(blockIdx.x, gridDim.x), &s, &lc)) return;
  const int tid = threadIdx.x;
  const int c0 = 4 * s;
  const int nact = min(4, a.nr - c0);
  if (lc >= nact) return;
  const int line0 = lc < 0 ? c0 : c0 + lc;
  const LineTab& tb = a.tabs[class_at(a.line_end, line0)];
  const int p0 = tid * M;
  LaneTab<M> L;
  load_lanetab<M, NT>(L, tb.pos + tid, tb.chk + tid);
  const unsigned long long live = chunk_live_mask(p0, M, a.nz, tb.skip_lo, tb.skip_hi);

  const double2* __restrict__ src = (const double2*)(a.din + (long)s * a.strip);
#pragma unroll
  for (int u = 0; u < 2 * M; ++u) {
    const int q = tid + u * NT;  // row q/2, column pair q%2
    const int j = q >> 1;
    double2 x = make_double2(0.0, 0.0);
    if (j < a.nz) x = src[q];
    const int kk = j / M, t = j - kk * M;
    *(double2*)&buf[kk * CH + t * 4 + (q & 1) * 2] = x;
  }
  __syncthreads();
  if (lc < 0) {
    double v[4][M], o[4][M];
#pragma unroll
    for (int t = 0; t < M; ++t) {
      const double2 lo = *(const double2*)&buf[tid * CH + t * 4];
      const double2 hi = *(const double2*)&buf[tid * CH + t * 4 + 2];
      v[0][t] = lo.x; v[1][t] = lo.y; v[2][t] = hi.x; v[3][t] = hi.y;
    }
    __syncthreads();  // buf is reused for the outputs
    solve_lanes<M, NW, 4>(v, o, L, live, carry);
    if (a.xc) {
      double xcv[MAX_CLS][4];
      load_crossing<4>(a, line0, nact, xcv);
      add_crossing<M, 4>(a, o, xcv, live, p0);
    }
#pragma unroll
    for (int t = 0; t < M; ++t) {
      *(double2*)&buf[tid * CH + t * 4] = make_double2(o[0][t], nact > 1 ? o[1][t] : 0.0);
      *(double2*)&buf[tid * CH + t * 4 + 2] = make_double2(nact > 2 ? o[2][t] : 0.0, nact > 3 ? o[3][t] : 0.0);
    }
    __syncthreads();
    double2* __restrict__ dst = (double2*)(a.dout + (long)s * a.strip);
#pragma unroll
    for (int u = 0; u < 2 * M; ++u) {
      const int q = tid + u * NT;
      const int j = q >> 1;
      if (j < a.nz) {
        const int kk = j / M, t = j - kk * M;
        dst[q] = *(const double2*)&buf[kk * CH + t * 4 + (q & 1) * 2];
      }
    }
    if (a.xout) {
#pragma unroll
      for (int t = 0; t < M; ++t)
        if (p0 + t < a.nz)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (c < nact) a.xout[(long)(p0 + t) * a.nr + c0 + c] = v[c][t];
    }
  } else {
    // one line of a mixed strip: column lc with its own class
    double v[1][M], o[1][M];
#pragma unroll
    for (int t = 0; t < M; ++t) v[0][t] = buf[tid * CH + t * 4 + lc];
    __syncthreads();  // the carries overwrite buf
    solve_lanes<M, NW, 1>(v, o, L, live, carry);
    if (a.xc) {
      double xcv[MAX_CLS][1];
      load_crossing<1>(a, line0, 1, xcv);
      add_crossing<M, 1>(a, o, xcv, live, p0);
    }
    double* __restrict__ dst = a.dout + (long)s * a.strip + lc;
#pragma unroll
    for (int t = 0; t < M; ++t)
      if (p0 + t < a.nz) {
        dst[4L * (p0 + t)] = o[0][t];
        if (a.xout) a.xout[(long)(p0 + t) * a.nr + line0] = v[0][t];
      }
  }
}

// r sweep: workgroup per group of 4 consecutive rows, lane k holds columns
// [4k, 4k+4) of the rows: exactly tile k of the row group.
template <int NW>
__global__ void __launch_bounds__(64 * NW) k_sweep_rs(StripArgs a) {
  constexpr int M = 4;
  constexpr int NT = 64 * NW;
  constexpr int CH = 18;  // a 16-double tile + 2 pad
  __shared__ __align__(16) double buf[NT * CH];
  __shared__ double carry[NW * 5];
  int J, lc;
  if (!strip_work(a, xcd_block(blockIdx.x, gridDim.x), &J, &lc)) return;
  const int tid = threadIdx.x;
  const int j0 = 4 * J;
  const int nact = min(4, a.nz - j0);
  if (lc >= nact) return;
  const int line0 = lc < 0 ? j0 : j0 + lc;
  const LineTab& tb = a.tabs[class_at(a.line_end, line0)];
  const int p0 = tid * M;
  LaneTab<M> L;
  load_lanetab<M, NT>(L, tb.pos + tid, tb.chk + tid);
  const unsigned long long live = chunk_live_mask(p0, M, a.nr, tb.skip_lo, tb.skip_hi);
  const int nstrips = (a.nr + 3) >> 2;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int q = tid + u * NT;  // tile q/8, piece q%8
    const int st = q >> 3;
    double2 x = make_double2(0.0, 0.0);
    if (st < nstrips) x = *(const double2*)(a.din + (long)st * a.strip + (long)j0 * 4 + (q & 7) * 2);
    *(double2*)&buf[st * CH + (q & 7) * 2] = x;
  }
  __syncthreads();
  if (lc < 0) {
    double v[4][M], o[4][M];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double2 lo = *(const double2*)&buf[tid * CH + r * 4];
      const double2 hi = *(const double2*)&buf[tid * CH + r * 4 + 2];
      v[r][0] = lo.x; v[r][1] = lo.y; v[r][2] = hi.x; v[r][3] = hi.y;
    }
    __syncthreads();
    solve_lanes<M, NW, 4>(v, o, L, live, carry);
    if (a.xc) {
      double xcv[MAX_CLS][4];
      load_crossing<4>(a, line0, nact, xcv);
      add_crossing<M, 4>(a, o, xcv, live, p0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool on = r < nact;
      *(double2*)&buf[tid * CH + r * 4] = make_double2(on ? o[r][0] : 0.0, on ? o[r][1] : 0.0);
      *(double2*)&buf[tid * CH + r * 4 + 2] = make_double2(on ? o[r][2] : 0.0, on ? o[r][3] : 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = tid + u * NT;
      const int st = q >> 3;
      if (st < nstrips)
        *(double2*)(a.dout + (long)st * a.strip + (long)j0 * 4 + (q & 7) * 2) =
            *(const double2*)&buf[st * CH + (q & 7) * 2];
    }
    if (a.xout) {
      const int i0 = 4 * tid;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (r < nact)
#pragma unroll
          for (int t = 0; t < M; ++t)
            if (i0 + t < a.nr) a.xout[(long)(j0 + r) * a.nr + i0 + t] = v[r][t];
    }
  } else {
    // one row of a mixed row group
    double v[1][M], o[1][M];
#pragma unroll
    for (int t = 0; t < M; ++t) v[0][t] = buf[tid * CH + lc * 4 + t];
    solve_lanes<M, NW, 1>(v, o, L, live, carry);
    if (a.xc) {
      double xcv[MAX_CLS][1];
      load_crossing<1>(a, line0, 1, xcv);
      add_crossing<M, 1>(a, o, xcv, live, p0);
    }
    if (tid < nstrips) {
      double* __restrict__ d = a.dout + (long)tid * a.strip + (long)line0 * 4;
      *(double2*)d = make_double2(o[0][0], o[0][1]);
      *(double2*)(d + 2) = make_double2(o[0][2], o[0][3]);
      if (a.xout) {
        const int i0 = 4 * tid;
#pragma unroll
        for (int t = 0; t < M; ++t)
          if (i0 + t < a.nr) a.xout[(long)line0 * a.nr + i0 + t] = v[0][t];
      }
    }
  }
}

}  // namespace adi
