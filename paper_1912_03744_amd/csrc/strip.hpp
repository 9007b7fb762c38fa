// strip.hpp -- sweeps over right-hand sides stored in strips of 4 columns.
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

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
  int line_end[3];          // class of line l: number of q with l >= line_end[q]
  int pos_end[3];           // crossing class of position p: number of q with p >= pos_end[q]
  int nxcls;                // crossing classes
  int nblocks;              // row groups (r sweep)
  int nmix;                 // r sweep: row groups whose rows are not all of one band ...
  int mix[4];               // ... solved one row per workgroup by nblocks + 4*m + row
};

// ---- host side: launch arguments shared by the library and its tests ----

// Cumulative class ends along one axis (dir 0: rows by band, 1: columns by
// class) from the class ranges of build_geometry: the class of index x is the
// number of q with x >= ends[q].
__host__ __device__ inline void strip_class_ends(const int* ranges, int dir, int ncls, int* ends) {
  int e = 0;
  for (int c = 0; c < 3; ++c) {
    if (c < ncls) {
      const int* rg = ranges + (dir * MAX_CLS + c) * 2;
      if (rg[1] > rg[0]) e = rg[1];
      ends[c] = c < ncls - 1 ? e : INT32_MAX;
    } else {
      ends[c] = INT32_MAX;
    }
  }
}

// Fill the class fields of a sweep's arguments and return its grid size.
// dir 0 (r sweep): lines are rows (band classes), positions columns; row
// groups straddling a band boundary get one workgroup per row.  dir 1 (z
// sweep): lines are columns, positions rows; one workgroup per strip.
inline int strip_setup(StripArgs& a, const int* ranges, int dir, int nlines, int ncls_lines, int ncls_pos) {
  strip_class_ends(ranges, dir == 0 ? 0 : 1, ncls_lines, a.line_end);
  strip_class_ends(ranges, dir == 0 ? 1 : 0, ncls_pos, a.pos_end);
  a.nxcls = ncls_pos;
  a.nlines = nlines;
  a.nblocks = (nlines + 3) / 4;
  a.nmix = 0;
  if (dir == 0)
    for (int q = 0; q < 3; ++q) {
      const int e = a.line_end[q];
      if (e <= 0 || e >= nlines || e % 4 == 0) continue;
      bool seen = false;
      for (int m = 0; m < a.nmix; ++m) seen = seen || a.mix[m] == e / 4;
      if (!seen) a.mix[a.nmix++] = e / 4;
    }
  for (int m = a.nmix; m < 4; ++m) a.mix[m] = -1;
  return a.nblocks + 4 * a.nmix;
}

// r sweep work of a workgroup: b < nblocks is row group b with all its rows
// (lc = -1) unless the group is mixed (then nothing); b >= nblocks is row lc
// of mixed group mix[(b - nblocks) / 4].
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

// Orders LDS accesses among the lanes of one wave (no workgroup barrier):
// staging copies are per wave, so waves proceed independently until the
// solver's carries.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int class_at(const int* ends, int x) {
  return (x >= ends[0]) + (x >= ends[1]) + (x >= ends[2]);
}

// Add the crossing constants of the other direction to the outputs of the
// lines in `mask`: for line line0 + r at position p, xc[class of p][line]
// (uniform across the workgroup), at positions inside the domain.
template <int M>
__device__ __forceinline__ void add_crossing(const StripArgs& a, double (*o)[M], int line0, unsigned mask,
                                             int n, int p0) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (!((mask >> r) & 1u)) continue;
    double xcv[MAX_CLS];
#pragma unroll
    for (int c = 0; c < MAX_CLS; ++c) xcv[c] = c < a.nxcls ? a.xc[(long)c * a.nlines + line0 + r] : 0.0;
    const LineTab& tb = a.tabs[class_at(a.line_end, line0 + r)];
    const unsigned long long live = chunk_live_mask(p0, M, n, tb.skip_lo, tb.skip_hi);
#pragma unroll
    for (int t = 0; t < M; ++t) {
      const int c = class_at(a.pos_end, p0 + t);
      if ((live >> t) & 1ull) o[r][t] += c == 0 ? xcv[0] : (c == 1 ? xcv[1] : (c == 2 ? xcv[2] : xcv[3]));
    }
  }
}

// Solve the 4 lines of a block and hand each line's outputs to `emit`
// (v: solution, o: next right-hand side, mask of the lines to take).  Lines
// of one class are solved together; a block whose lines span several classes
// (classes grow with the line index) is solved once per class, each pass
// refetching the block's right-hand side with `fetch`.  L: the tables of the
// first class, already loaded; later passes reload it.
template <int M, int NW, class Fetch, class Emit>
__device__ __forceinline__ void solve_block(const StripArgs& a, double (*v)[M], int line0, int nact, int n, int tid,
                                            double* carry, LaneTab<M>& L, Fetch fetch, Emit emit) {
  const int p0 = tid * M;
  const int c_lo = class_at(a.line_end, line0), c_hi = class_at(a.line_end, line0 + nact - 1);
  auto lines_of = [&](int c) {
    unsigned mine = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (r < nact && class_at(a.line_end, line0 + r) == c) mine |= 1u << r;
    return mine;
  };
  for (int c = c_lo; c <= c_hi; ++c) {
    const LineTab& tb = a.tabs[c];
    if (c > c_lo) {
      load_lanetab<M, 64 * NW>(L, tb.pos, tb.chk, tid);  // L held the first class
      fetch(v);
    }
    double o[4][M];
    solve_lanes<M, NW, 4>(v, o, L, chunk_live_mask(p0, M, n, tb.skip_lo, tb.skip_hi), carry);
    emit(v, o, lines_of(c));
  }
}

// Each lane reads and writes only its own chunk's LDS slots between the
// staging copies, which each wave does for its own chunks.
// The z-sweep work on strip s by lanes tid = 0 .. 64*NW-1 (a workgroup, or
// one wave when NW = 1), staging through buf (64*NW*4*M doubles) and
// carrying through `carry` (2*NW*5 doubles).
template <int M, int NW>
__device__ __forceinline__ void strip_z_body(const StripArgs& a, int s, int tid, double* buf, double* carry) {
  constexpr int NT = 64 * NW;
  constexpr int CH = 4 * M;  // LDS doubles per chunk (rows of 4, no padding)
  const int c0 = 4 * s;
  const int nact = min(4, a.nr - c0);
  const int p0 = tid * M;
  // factor tables of the first class ahead of the data
  LaneTab<M> L0;
  {
    const LineTab& tb = a.tabs[class_at(a.line_end, c0)];
    load_lanetab<M, NT>(L0, tb.pos, tb.chk, tid);
  }
  // each wave stages the 64*M rows of its own 64 chunks (contiguous in the
  // strip) through its own LDS region
  const int lane = tid & 63, wrow0 = (tid >> 6) * 64 * M;
  double* wbuf = buf + (tid >> 6) * 64 * CH;
  const double2* __restrict__ src = (const double2*)(a.din + (long)s * a.strip) + 2 * wrow0;
  // with 4*M doubles per chunk, local row jl sits at 4*jl in the wave's
  // region, as in the strip: the copy is contiguous
#pragma unroll
  for (int u = 0; u < 2 * M; ++u) {
    const int q = lane + u * 64;  // local row q/2, column pair q%2
    double2 x = make_double2(0.0, 0.0);
    if (wrow0 + (q >> 1) < a.nz) x = src[q];
    *(double2*)&wbuf[2 * q] = x;
  }
  wave_sync();
  double* mine_slots = buf + tid * CH;
  auto fetch = [&](double (*v)[M]) {
#pragma unroll
    for (int t = 0; t < M; ++t) {
      const double2 lo = *(const double2*)&mine_slots[t * 4];
      const double2 hi = *(const double2*)&mine_slots[t * 4 + 2];
      v[0][t] = lo.x; v[1][t] = lo.y; v[2][t] = hi.x; v[3][t] = hi.y;
    }
  };
  auto emit = [&](double (*v)[M], double (*o)[M], unsigned mask) {
    if (a.xc) add_crossing<M>(a, o, c0, mask, a.nz, p0);
    if (mask == 0xfu) {
#pragma unroll
      for (int t = 0; t < M; ++t) {
        *(double2*)&mine_slots[t * 4] = make_double2(o[0][t], o[1][t]);
        *(double2*)&mine_slots[t * 4 + 2] = make_double2(o[2][t], o[3][t]);
      }
    } else {
#pragma unroll
      for (int t = 0; t < M; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if ((mask >> r) & 1u) mine_slots[t * 4 + r] = o[r][t];
    }
    if (a.xout)
#pragma unroll
      for (int t = 0; t < M; ++t)
        if (p0 + t < a.nz)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if ((mask >> c) & 1u) a.xout[(long)(p0 + t) * a.nr + c0 + c] = v[c][t];
  };
  double v[4][M];
  fetch(v);
  // columns past the grid's edge hold 0
#pragma unroll
  for (int t = 0; t < M; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (r >= nact) mine_slots[t * 4 + r] = 0.0;
  solve_block<M, NW>(a, v, c0, nact, a.nz, tid, carry, L0, fetch, emit);
  wave_sync();
  double2* __restrict__ dst = (double2*)(a.dout + (long)s * a.strip) + 2 * wrow0;
#pragma unroll
  for (int u = 0; u < 2 * M; ++u) {
    const int q = lane + u * 64;
    if (wrow0 + (q >> 1) < a.nz) dst[q] = *(const double2*)&wbuf[2 * q];
  }
}

// z sweep: workgroup per strip (4 adjacent columns), lane k holds rows
// [kM, kM+M) of the strip's columns.
template <int M, int NW>
__global__ void __launch_bounds__(64 * NW) k_sweep_zs(StripArgs a) {
  __shared__ __align__(16) double buf[64 * NW * 4 * M];
  __shared__ double carry[2 * NW * 5];
  strip_z_body<M, NW>(a, xcd_block(blockIdx.x, gridDim.x), threadIdx.x, buf, carry);
}

// The r-sweep work on row group J by lanes tid = 0 .. 64*NW-1, solving the
// rows of each band present in one pass per band (used by the batch, where
// a workgroup holds no extra rows to hand out), staging through buf
// (64*NW*18 doubles).
template <int NW>
__device__ __forceinline__ void strip_r_body(const StripArgs& a, int J, int tid, double* buf, double* carry) {
  constexpr int M = 4;
  constexpr int NT = 64 * NW;
  constexpr int CH = 18;  // a 16-double tile + 2 pad
  const int j0 = 4 * J;
  const int nact = min(4, a.nz - j0);
  const int p0 = tid * M;
  LaneTab<M> L0;
  {
    const LineTab& tb = a.tabs[class_at(a.line_end, j0)];
    load_lanetab<M, NT>(L0, tb.pos, tb.chk, tid);
  }
  const int nstrips = (a.nr + 3) >> 2;
  const int lane = tid & 63, wst0 = (tid >> 6) * 64;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int q = lane + u * 64;  // local tile q/8, piece q%8
    const int st = wst0 + (q >> 3);
    double2 x = make_double2(0.0, 0.0);
    if (st < nstrips) x = *(const double2*)(a.din + (long)st * a.strip + (long)j0 * 4 + (q & 7) * 2);
    *(double2*)&buf[st * CH + (q & 7) * 2] = x;
  }
  wave_sync();
  double* mine_slots = buf + tid * CH;
  auto fetch = [&](double (*v)[M]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double2 lo = *(const double2*)&mine_slots[r * 4];
      const double2 hi = *(const double2*)&mine_slots[r * 4 + 2];
      v[r][0] = lo.x; v[r][1] = lo.y; v[r][2] = hi.x; v[r][3] = hi.y;
    }
  };
  auto emit = [&](double (*v)[M], double (*o)[M], unsigned mask) {
    if (a.xc) add_crossing<M>(a, o, j0, mask, a.nr, p0);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if ((mask >> r) & 1u) {
        *(double2*)&mine_slots[r * 4] = make_double2(o[r][0], o[r][1]);
        *(double2*)&mine_slots[r * 4 + 2] = make_double2(o[r][2], o[r][3]);
      }
    if (a.xout) {
      const int i0 = 4 * tid;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if ((mask >> r) & 1u)
#pragma unroll
          for (int t = 0; t < M; ++t)
            if (i0 + t < a.nr) a.xout[(long)(j0 + r) * a.nr + i0 + t] = v[r][t];
    }
  };
  double v[4][M];
  fetch(v);
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (r >= nact) {
      *(double2*)&mine_slots[r * 4] = make_double2(0.0, 0.0);
      *(double2*)&mine_slots[r * 4 + 2] = make_double2(0.0, 0.0);
    }
  solve_block<M, NW>(a, v, j0, nact, a.nr, tid, carry, L0, fetch, emit);
  wave_sync();
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int q = lane + u * 64;
    const int st = wst0 + (q >> 3);
    if (st < nstrips)
      *(double2*)(a.dout + (long)st * a.strip + (long)j0 * 4 + (q & 7) * 2) =
          *(const double2*)&buf[st * CH + (q & 7) * 2];
  }
}

// r sweep: workgroup per group of 4 consecutive rows, lane k holds columns
// [4k, 4k+4) of the rows: exactly tile k of the row group, in its own LDS
// slots.  Row groups that straddle a band boundary are solved one row per
// workgroup (extra workgroups of the same launch).
template <int NW>
__global__ void __launch_bounds__(64 * NW) k_sweep_rs(StripArgs a) {
  constexpr int M = 4;
  constexpr int NT = 64 * NW;
  constexpr int CH = 18;  // a 16-double tile + 2 pad
  __shared__ __align__(16) double buf[NT * CH];
  __shared__ double carry[2 * NW * 5];
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
  load_lanetab<M, NT>(L, tb.pos, tb.chk, tid);
  const unsigned long long live = chunk_live_mask(p0, M, a.nr, tb.skip_lo, tb.skip_hi);
  const int nstrips = (a.nr + 3) >> 2;
  // each wave stages the 64 tiles of its own chunks through its own LDS region
  const int lane = tid & 63, wst0 = (tid >> 6) * 64;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int q = lane + u * 64;  // local tile q/8, piece q%8
    const int st = wst0 + (q >> 3);
    double2 x = make_double2(0.0, 0.0);
    if (st < nstrips) x = *(const double2*)(a.din + (long)st * a.strip + (long)j0 * 4 + (q & 7) * 2);
    *(double2*)&buf[st * CH + (q & 7) * 2] = x;
  }
  wave_sync();
  double* mine_slots = buf + tid * CH;
  if (lc < 0) {
    double v[4][M], o[4][M];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double2 lo = *(const double2*)&mine_slots[r * 4];
      const double2 hi = *(const double2*)&mine_slots[r * 4 + 2];
      v[r][0] = lo.x; v[r][1] = lo.y; v[r][2] = hi.x; v[r][3] = hi.y;
    }
    solve_lanes<M, NW, 4>(v, o, L, live, carry);
    const unsigned mask = nact == 4 ? 0xfu : (1u << nact) - 1u;
    if (a.xc) add_crossing<M>(a, o, j0, mask, a.nr, p0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool on = r < nact;
      *(double2*)&mine_slots[r * 4] = make_double2(on ? o[r][0] : 0.0, on ? o[r][1] : 0.0);
      *(double2*)&mine_slots[r * 4 + 2] = make_double2(on ? o[r][2] : 0.0, on ? o[r][3] : 0.0);
    }
    wave_sync();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = lane + u * 64;
      const int st = wst0 + (q >> 3);
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
    for (int t = 0; t < M; ++t) v[0][t] = mine_slots[lc * 4 + t];
    solve_lanes<M, NW, 1>(v, o, L, live, carry);
    if (a.xc) {
      double o4[4][M];
#pragma unroll
      for (int t = 0; t < M; ++t) o4[0][t] = o[0][t], o4[1][t] = o4[2][t] = o4[3][t] = 0.0;
      add_crossing<M>(a, o4, line0, 1u, a.nr, p0);
#pragma unroll
      for (int t = 0; t < M; ++t) o[0][t] = o4[0][t];
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
