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
// (i/4)*strip + 4*j + i%4, with strip = strip_stride(nz) doubles: at least
// 4*ceil(nz/4) rows).  A z sweep then
// reads and writes one contiguous block per strip; an r sweep over 4
// consecutive rows touches one whole 128-byte tile per strip.  Both kernels
// stage their block through LDS with fully coalesced copies, and each lane
// solves the same chunk of 4 lines, so every table value it loads serves
// 4 lines.

// Doubles per strip: 4*ceil(nz/4) rows of 4 plus 1 KB, so that the tiles
// an r sweep reads from consecutive strips (one strip apart) do not all fall
// on the same memory channels when the rows alone span a power of two.
// Padding rows hold 0 and are never read by a sweep.
__host__ __device__ inline long strip_stride(int nz) { return 16L * ((nz + 3) / 4) + 128; }

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
  int nblocks;              // row groups (r sweep) or strips (z sweep)
  int nmix;                 // r sweep: row groups whose rows are not all of one band, solved
  int mix[4];               //   one row per workgroup by nblocks + 4*m + row (mix[m]: group);
                            // z sweep: extra workgroups nblocks + m, one per further class
                            //   of a strip solved class by class (mix[m] = 4 * strip + class)
  double theta;             // weight of the solved right-hand side in the next one (1 PR, 0 LOD-BE)
};

// LDS doubles of a workgroup's reduced-system carries (NW waves).
__host__ __device__ constexpr int strip_carry(int NW) { return 2 * NW * 6; }

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

__host__ __device__ inline int class_at(const int* ends, int x) {
  return (x >= ends[0]) + (x >= ends[1]) + (x >= ends[2]);
}

// Lines r < nact of a block of 4 starting at line0 whose class is c.
__host__ __device__ inline unsigned block_lines_of(const StripArgs& a, int line0, int nact, int c) {
  unsigned m = 0;
  for (int r = 0; r < 4; ++r)
    if (r < nact && class_at(a.line_end, line0 + r) == c) m |= 1u << r;
  return m;
}

// A z strip (columns c0 .. c0+nact-1) whose columns split 3|1 or 1|3 between
// two consecutive classes: solved in one pass with both classes' tables.
__host__ __device__ inline bool strip_split(const StripArgs& a, int c0, int nact) {
  const int c_lo = class_at(a.line_end, c0), c_hi = class_at(a.line_end, c0 + nact - 1);
  const unsigned m = block_lines_of(a, c0, nact, c_lo);
  const int na = (m & 1u) + ((m >> 1) & 1u) + ((m >> 2) & 1u) + ((m >> 3) & 1u);
  return c_hi == c_lo + 1 && na != 2;
}

// Fill the class fields of a sweep's arguments and return its grid size.
// dir 0 (r sweep): lines are rows (band classes), positions columns; row
// groups straddling a band boundary get one workgroup per row.  dir 1 (z
// sweep): lines are columns, positions rows; one workgroup per strip.
// theta: 1 for Peaceman-Rachford, 0 for LOD backward Euler.
inline int strip_setup(StripArgs& a, const int* ranges, int dir, int nlines, int ncls_lines, int ncls_pos,
                       double theta) {
  a.theta = theta;
  strip_class_ends(ranges, dir == 0 ? 0 : 1, ncls_lines, a.line_end);
  strip_class_ends(ranges, dir == 0 ? 1 : 0, ncls_pos, a.pos_end);
  a.nxcls = ncls_pos;
  a.nlines = nlines;
  a.nblocks = (nlines + 3) / 4;
  a.nmix = 0;
  if (dir == 0) {
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
  // z sweep: every class boundary inside a strip that is not solved in one
  // pass adds a workgroup for the class starting there
  for (int q = 0; q < 3; ++q) {
    const int e = a.line_end[q];
    if (e <= 0 || e >= nlines || e % 4 == 0) continue;
    const int s = e / 4, c0 = 4 * s, nact = nlines - c0 < 4 ? nlines - c0 : 4;
    const int w = 4 * s + class_at(a.line_end, e);
    bool seen = false;  // boundaries of empty classes coincide
    for (int m = 0; m < a.nmix; ++m) seen = seen || a.mix[m] == w;
    if (!seen && !strip_split(a, c0, nact)) a.mix[a.nmix++] = w;
  }
  for (int m = a.nmix; m < 4; ++m) a.mix[m] = -1;
  return a.nblocks + a.nmix;
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

// Add the crossing constants of the other direction to the outputs of the
// block slots in `mask`: for line l at position p, xc[class of p][l]
// (uniform across the workgroup), at positions inside the domain.  Slot r
// holds line line0 + r, or line0 + 3 - r when `rev` is set.
template <int M>
__device__ __forceinline__ void add_crossing(const StripArgs& a, double (*o)[M], int line0, unsigned mask,
                                             int n, int p0, bool rev = false) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (!((mask >> r) & 1u)) continue;
    const int line = line0 + (rev ? 3 - r : r);
    double xcv[MAX_CLS];
#pragma unroll
    for (int c = 0; c < MAX_CLS; ++c) xcv[c] = c < a.nxcls ? a.xc[(long)c * a.nlines + line] : 0.0;
    const LineTab& tb = a.tabs[class_at(a.line_end, line)];
    const unsigned long long live = chunk_live_mask(p0, M, n, tb.skip_lo, tb.skip_hi);
#pragma unroll
    for (int t = 0; t < M; ++t) {
      const int c = class_at(a.pos_end, p0 + t);
      if ((live >> t) & 1ull) o[r][t] += c == 0 ? xcv[0] : (c == 1 ? xcv[1] : (c == 2 ? xcv[2] : xcv[3]));
    }
  }
}

// The next right-hand side of the lines of a block in `mask`, in place
// (v: solution on entry, the outputs on return), from the right-hand sides
// d the block was solved with: lines r < NA have the tables LA, the others
// LB.  `rhs(r, t)` returns d of line r at chunk offset t.
template <int M, int NA, class Rhs>
__device__ __forceinline__ void block_outputs(const StripArgs& a, double (*v)[M], const LaneTab<M>& LA,
                                              const LaneTab<M>& LB, unsigned mask, Rhs rhs) {
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if ((mask >> r) & 1u) {
      const LaneTab<M>& L = r < NA ? LA : LB;
#pragma unroll
      for (int t = 0; t < M; ++t) v[r][t] = next_rhs(L.ok[t], L.oc[t], a.theta, v[r][t], rhs(r, t));
    }
}

// z-sweep building blocks.  Lane tid of a strip's workgroup owns chunk tid:
// rows [tid*M, tid*M+M) of the strip's 4 columns, staged by its wave (each
// wave copies the 64*M rows of its own 64 chunks, contiguous in the strip,
// through its own LDS region) into its own LDS slots (4*M doubles, laid out
// as in the strip).  Each lane reads and writes only its own slots between
// the staging copies.

template <int M>
__device__ __forceinline__ void stage_z(const StripArgs& a, int s, int tid, double* buf) {
  const int lane = tid & 63, wrow0 = (tid >> 6) * 64 * M;
  double* wbuf = buf + (tid >> 6) * 64 * 4 * M;
  const double2* __restrict__ src = (const double2*)(a.din + (long)s * a.strip) + 2 * wrow0;
#pragma unroll
  for (int u = 0; u < 2 * M; ++u) {
    const int q = lane + u * 64;  // local row q/2, column pair q%2
    double2 x = make_double2(0.0, 0.0);
    if (wrow0 + (q >> 1) < a.nz) x = src[q];
    *(double2*)&wbuf[2 * q] = x;
  }
}

// Store the wave's rows back: whole rows, or only the columns in colmask.
template <int M>
__device__ __forceinline__ void store_z(const StripArgs& a, int s, int tid, const double* buf, unsigned colmask) {
  const int lane = tid & 63, wrow0 = (tid >> 6) * 64 * M;
  const double* wbuf = buf + (tid >> 6) * 64 * 4 * M;
  double2* __restrict__ dst = (double2*)(a.dout + (long)s * a.strip) + 2 * wrow0;
  if (colmask == 0xfu) {
#pragma unroll
    for (int u = 0; u < 2 * M; ++u) {
      const int q = lane + u * 64;
      if (wrow0 + (q >> 1) < a.nz) dst[q] = *(const double2*)&wbuf[2 * q];
    }
  } else {
    double* __restrict__ d1 = (double*)dst;
    for (int u = 0; u < 2 * M; ++u) {
      const int q = lane + u * 64, c = 2 * (q & 1);
      if (wrow0 + (q >> 1) < a.nz) {
        if ((colmask >> c) & 1u) d1[2 * q] = wbuf[2 * q];
        if ((colmask >> (c + 1)) & 1u) d1[2 * q + 1] = wbuf[2 * q + 1];
      }
    }
  }
}

// Solve the strip's columns with slots r < NA on LA, the rest on LB, and put
// the next right-hand side of the slots in `mask` into the lane's LDS
// slots (and the solution into xout).  Slot r holds column c0 + r, or
// c0 + 3 - r when `rv` is set (NA < 4 only).
template <int M, int NW, int NA>
__device__ __forceinline__ void z_pass(const StripArgs& a, int c0, int tid, double* mine_slots, const LaneTab<M>& LA,
                                       const LaneTab<M>& LB, double* carry, bool rv, unsigned mask) {
  const bool rev = NA < 4 && rv;
  const int p0 = tid * M;
  auto col = [&](int r) { return rev ? 3 - r : r; };
  double v[4][M];
#pragma unroll
  for (int t = 0; t < M; ++t) {
    const double2 lo = *(const double2*)&mine_slots[t * 4];
    const double2 hi = *(const double2*)&mine_slots[t * 4 + 2];
    if (rev) {
      v[0][t] = hi.y; v[1][t] = hi.x; v[2][t] = lo.y; v[3][t] = lo.x;
    } else {
      v[0][t] = lo.x; v[1][t] = lo.y; v[2][t] = hi.x; v[3][t] = hi.y;
    }
  }
  solve_lanes<M, NW, 4, NA>(v, LA, LB, carry);
  if (a.xout)
#pragma unroll
    for (int t = 0; t < M; ++t)
      if (p0 + t < a.nz)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if ((mask >> r) & 1u) a.xout[(long)(p0 + t) * a.nr + c0 + col(r)] = v[r][t];
  block_outputs<M, NA>(a, v, LA, LB, mask, [&](int r, int t) { return mine_slots[t * 4 + col(r)]; });
  if (a.xc) add_crossing<M>(a, v, c0, mask, a.nz, p0, rev);
  if (mask == 0xfu && !rev) {
#pragma unroll
    for (int t = 0; t < M; ++t) {
      *(double2*)&mine_slots[t * 4] = make_double2(v[0][t], v[1][t]);
      *(double2*)&mine_slots[t * 4 + 2] = make_double2(v[2][t], v[3][t]);
    }
  } else {
#pragma unroll
    for (int t = 0; t < M; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if ((mask >> r) & 1u) mine_slots[t * 4 + col(r)] = v[r][t];
  }
}

// Columns past the grid's edge hold 0 in the lane's slots.
template <int M>
__device__ __forceinline__ void zero_past_edge(double* mine_slots, int nact) {
#pragma unroll
  for (int t = 0; t < M; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (r >= nact) mine_slots[t * 4 + r] = 0.0;
}

// The z-sweep work on strip s by lanes tid = 0 .. 64*NW-1 (a workgroup, or
// one wave when NW = 1), staging through buf (64*NW*4*M doubles) and
// carrying through `carry` (strip_carry(NW) doubles), one pass per class
// of the strip's columns (used by the batch).
template <int M, int NW>
__device__ __forceinline__ void strip_z_body(const StripArgs& a, int s, int tid, double* buf, double* carry) {
  constexpr int NT = 64 * NW;
  const int c0 = 4 * s;
  const int nact = min(4, a.nr - c0);
  const int c_lo = class_at(a.line_end, c0), c_hi = class_at(a.line_end, c0 + nact - 1);
  stage_z<M>(a, s, tid, buf);
  wave_sync();
  double* mine_slots = buf + tid * 4 * M;
  zero_past_edge<M>(mine_slots, nact);
  for (int c = c_lo; c <= c_hi; ++c) {
    LaneTab<M> L;  // behind the data loads; live for one pass only
    load_lanetab<M, NT, false>(L, a.tabs[c].pos, a.tabs[c].chk, tid);
    z_pass<M, NW, 4>(a, c0, tid, mine_slots, L, L, carry, false, block_lines_of(a, c0, nact, c));
  }
  wave_sync();
  store_z<M>(a, s, tid, buf, 0xfu);
}

// z sweep: workgroup per strip (4 adjacent columns), lane k holds rows
// [kM, kM+M) of the strip's columns.  A strip of one class, or split 3|1 or
// 1|3 between two classes (both classes' tables, slots 0..2 on the first,
// columns in reverse order for 1|3), is solved in one pass; in any other
// strip spanning several classes this workgroup solves the first class and
// extra workgroups (nblocks + m) one further class each, every one storing
// only its own columns.
template <int M, int NW>
__global__ void __launch_bounds__(64 * NW) k_sweep_zs(StripArgs a) {
  constexpr int NT = 64 * NW;
  __shared__ __align__(16) double buf[NT * 4 * M];
  __shared__ double carry[strip_carry(NW)];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x;
  const int s = b < a.nblocks ? b : a.mix[b - a.nblocks] >> 2;
  const int c0 = 4 * s;
  const int nact = min(4, a.nr - c0);
  const int c_lo = class_at(a.line_end, c0), c_hi = class_at(a.line_end, c0 + nact - 1);
  const unsigned all = nact == 4 ? 0xfu : (1u << nact) - 1u;
  const bool split = c_hi == c_lo + 1 && strip_split(a, c0, nact);
  const bool rev = split && block_lines_of(a, c0, nact, c_lo) == 1u;
  // this workgroup's class (one-class passes) and its columns
  const int c = b < a.nblocks ? c_lo : a.mix[b - a.nblocks] & 3;
  const unsigned mine = c_lo == c_hi ? all : block_lines_of(a, c0, nact, c);
  // data loads first: waiting for them then does not wait for the tables
  stage_z<M>(a, s, tid, buf);
  LaneTab<M> LA, LB;
  {
    const int ca = rev ? c_hi : c;
    load_lanetab<M, NT, true>(LA, a.tabs[ca].pos, a.tabs[ca].chk, tid);
    if (split) load_lanetab<M, NT, true>(LB, a.tabs[rev ? c_lo : c_hi].pos, a.tabs[rev ? c_lo : c_hi].chk, tid);
  }
  wave_sync();
  double* mine_slots = buf + tid * 4 * M;
  zero_past_edge<M>(mine_slots, nact);
  if (split) {
    // slot mask of the active columns
    const unsigned m = rev ? ((all & 1u) << 3) | ((all & 2u) << 1) | ((all & 4u) >> 1) | ((all & 8u) >> 3) : all;
    z_pass<M, NW, 3>(a, c0, tid, mine_slots, LA, LB, carry, rev, m);
  } else {
    z_pass<M, NW, 4>(a, c0, tid, mine_slots, LA, LA, carry, false, mine);
  }
  wave_sync();
  store_z<M>(a, s, tid, buf, split || c_lo == c_hi ? 0xfu : mine);
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
  const int c_lo = class_at(a.line_end, j0), c_hi = class_at(a.line_end, j0 + nact - 1);
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
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (r >= nact) {
      *(double2*)&mine_slots[r * 4] = make_double2(0.0, 0.0);
      *(double2*)&mine_slots[r * 4 + 2] = make_double2(0.0, 0.0);
    }
  auto rhs = [&](int r, int t) { return mine_slots[r * 4 + t]; };
  for (int c = c_lo; c <= c_hi; ++c) {
    LaneTab<M> L;  // behind the data loads; live for one pass only
    load_lanetab<M, NT, false>(L, a.tabs[c].pos, a.tabs[c].chk, tid);
    const unsigned mask = block_lines_of(a, j0, nact, c);
    double v[4][M];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double2 lo = *(const double2*)&mine_slots[r * 4];
      const double2 hi = *(const double2*)&mine_slots[r * 4 + 2];
      v[r][0] = lo.x; v[r][1] = lo.y; v[r][2] = hi.x; v[r][3] = hi.y;
    }
    solve_lanes<M, NW, 4, 4>(v, L, L, carry);
    if (a.xout) {
      const int i0 = 4 * tid;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if ((mask >> r) & 1u)
#pragma unroll
          for (int t = 0; t < M; ++t)
            if (i0 + t < a.nr) a.xout[(long)(j0 + r) * a.nr + i0 + t] = v[r][t];
    }
    block_outputs<M, 4>(a, v, L, L, mask, rhs);
    if (a.xc) add_crossing<M>(a, v, j0, mask, a.nr, p0);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if ((mask >> r) & 1u) {
        *(double2*)&mine_slots[r * 4] = make_double2(v[r][0], v[r][1]);
        *(double2*)&mine_slots[r * 4 + 2] = make_double2(v[r][2], v[r][3]);
      }
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
}

// The r-sweep work of one wave on 64/CPW consecutive row groups J0, J0+1,
// ... (lines of up to 4*CPW cells): lane slot g = lane / CPW holds row
// group J0 + g, lane ci = lane % CPW of the slot holds tile ci of it, in its
// own LDS slots (buf: 64*18 doubles).  Rows of each band present are solved
// in one pass per band (each slot emits only its rows of that band).  Used
// by the batched sweep launches, where lines are short and the solution of
// an r half step is not written out.
template <int CPW>
__device__ __forceinline__ void strip_r_slots(const StripArgs& a, int J0, double* buf, double* carry) {
  constexpr int M = 4;
  constexpr int CH = 18;  // a 16-double tile + 2 pad
  constexpr int S = 64 / CPW;
  const int lane = threadIdx.x & 63;
  const int g = lane / CPW, ci = lane % CPW;
  const int nrg = (a.nz + 3) >> 2, nstrips = (a.nr + 3) >> 2;
  const int j0 = 4 * (J0 + g);  // first row of the lane's row group
  const int nact = max(0, min(4, a.nz - j0));
  const int row_lo = 4 * J0, row_hi = min(4 * (J0 + S), a.nz) - 1;
  const int c_lo = class_at(a.line_end, row_lo), c_hi = class_at(a.line_end, row_hi);
  // data: tile t = q/8 of the wave (slot t / CPW, tile t % CPW), piece q%8
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int q = lane + u * 64;
    const int t = q >> 3, tg = t / CPW, tk = t % CPW;
    double2 x = make_double2(0.0, 0.0);
    if (tk < nstrips && J0 + tg < nrg)
      x = *(const double2*)(a.din + (long)tk * a.strip + (long)(J0 + tg) * 16 + (q & 7) * 2);
    *(double2*)&buf[t * CH + (q & 7) * 2] = x;
  }
  wave_sync();
  double* mine_slots = buf + lane * CH;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (r >= nact) {
      *(double2*)&mine_slots[r * 4] = make_double2(0.0, 0.0);
      *(double2*)&mine_slots[r * 4 + 2] = make_double2(0.0, 0.0);
    }
  for (int c = c_lo; c <= c_hi; ++c) {
    LaneTab<M> L;  // behind the data loads; live for one pass only
    load_lanetab<M, 64, false>(L, a.tabs[c].pos, a.tabs[c].chk, ci);
    const unsigned mask = block_lines_of(a, j0, nact, c);
    double v[4][M];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double2 lo = *(const double2*)&mine_slots[r * 4];
      const double2 hi = *(const double2*)&mine_slots[r * 4 + 2];
      v[r][0] = lo.x; v[r][1] = lo.y; v[r][2] = hi.x; v[r][3] = hi.y;
    }
    solve_lanes<M, 1, 4, 4, CPW>(v, L, L, carry);
    block_outputs<M, 4>(a, v, L, L, mask, [&](int r, int t) { return mine_slots[r * 4 + t]; });
    if (a.xc) add_crossing<M>(a, v, j0, mask, a.nr, ci * M);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if ((mask >> r) & 1u) {
        *(double2*)&mine_slots[r * 4] = make_double2(v[r][0], v[r][1]);
        *(double2*)&mine_slots[r * 4 + 2] = make_double2(v[r][2], v[r][3]);
      }
  }
  wave_sync();
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int q = lane + u * 64;
    const int t = q >> 3, tg = t / CPW, tk = t % CPW;
    if (tk < nstrips && J0 + tg < nrg)
      *(double2*)(a.dout + (long)tk * a.strip + (long)(J0 + tg) * 16 + (q & 7) * 2) =
          *(const double2*)&buf[t * CH + (q & 7) * 2];
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
  __shared__ double carry[strip_carry(NW)];
  int J, lc;
  if (!strip_work(a, xcd_block(blockIdx.x, gridDim.x), &J, &lc)) return;
  const int tid = threadIdx.x;
  const int j0 = 4 * J;
  const int nact = min(4, a.nz - j0);
  if (lc >= nact) return;
  const int line0 = lc < 0 ? j0 : j0 + lc;
  const LineTab& tb = a.tabs[class_at(a.line_end, line0)];
  const int p0 = tid * M;
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
  LaneTab<M> L;  // behind the data loads
  load_lanetab<M, NT, true>(L, tb.pos, tb.chk, tid);
  wave_sync();
  double* mine_slots = buf + tid * CH;
  if (lc < 0) {
    double v[4][M];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double2 lo = *(const double2*)&mine_slots[r * 4];
      const double2 hi = *(const double2*)&mine_slots[r * 4 + 2];
      v[r][0] = lo.x; v[r][1] = lo.y; v[r][2] = hi.x; v[r][3] = hi.y;
    }
    solve_lanes<M, NW, 4, 4>(v, L, L, carry);
    const unsigned mask = nact == 4 ? 0xfu : (1u << nact) - 1u;
    if (a.xout) {
      const int i0 = 4 * tid;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (r < nact)
#pragma unroll
          for (int t = 0; t < M; ++t)
            if (i0 + t < a.nr) a.xout[(long)(j0 + r) * a.nr + i0 + t] = v[r][t];
    }
    block_outputs<M, 4>(a, v, L, L, mask, [&](int r, int t) { return mine_slots[r * 4 + t]; });
    if (a.xc) add_crossing<M>(a, v, j0, mask, a.nr, p0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool on = r < nact;  // rows past the grid's edge hold 0
      *(double2*)&mine_slots[r * 4] = make_double2(on ? v[r][0] : 0.0, on ? v[r][1] : 0.0);
      *(double2*)&mine_slots[r * 4 + 2] = make_double2(on ? v[r][2] : 0.0, on ? v[r][3] : 0.0);
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
  } else {
    // one row of a mixed row group
    double v[4][M];
#pragma unroll
    for (int t = 0; t < M; ++t) v[0][t] = mine_slots[lc * 4 + t];
    solve_lanes<M, NW, 1, 1>(v, L, L, carry);
    if (a.xout && tid < nstrips) {
      const int i0 = 4 * tid;
#pragma unroll
      for (int t = 0; t < M; ++t)
        if (i0 + t < a.nr) a.xout[(long)line0 * a.nr + i0 + t] = v[0][t];
    }
    block_outputs<M, 4>(a, v, L, L, 1u, [&](int, int t) { return mine_slots[lc * 4 + t]; });
    if (a.xc) add_crossing<M>(a, v, line0, 1u, a.nr, p0);
    if (tid < nstrips) {
      double* __restrict__ d = a.dout + (long)tid * a.strip + (long)line0 * 4;
      *(double2*)d = make_double2(v[0][0], v[0][1]);
      *(double2*)(d + 2) = make_double2(v[0][2], v[0][3]);
    }
  }
}

}  // namespace adi
