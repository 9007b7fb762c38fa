// batch.hpp -- ragged batch: instance descriptors, scratch layout and the
// persistent kernel on the strip-layout line solver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "strip.hpp"

namespace adi {

// Compiled line shapes of the batch kernel (one wave per line group):
// r lines use 4 lines x 16 chunks per wave, z lines 2 lines x 32 chunks.
constexpr int kBR_LPW = 4, kBR_G = 16;
constexpr int kBZ_LPW = 2, kBZ_G = 32;
constexpr int kBR_M[4] = {4, 6, 8, 12};   // r lines up to 64, 96, 128, 192 cells
constexpr int kBZ_M[4] = {5, 8, 10, 15};  // z lines up to 160, 256, 320, 480 cells
constexpr int kMaxNr = 192, kMaxNz = 480;

struct BatchInst {
  Params P;
  long toff;   // offset of the instance's field in the arena (doubles)
  int rs, zs;  // shape index of its r and z lines (rows-layout kernels)
  int zss;     // shape index of its z lines for the strip-layout kernel
  double T0;   // uniform initial temperature
};

// Byte offsets inside one workgroup's scratch area.
struct BatchLayout {
  long dA, dB, geo, kap, bet, ranges, rtabs, rpos, rchk, reng, rxc, ztabs, zpos, zchk, zeng, zxc, work;
  long stride;
};

struct BatchArgs {
  const BatchInst* inst;
  const int* order;
  int ninst;
  int* queue;
  double* T;
  double* prof;
  int nsnap, npts, snap_every;
  int nsteps;
  char* scratch;
  BatchLayout lay;
};

__device__ __forceinline__ void skip_range(int dir, int cls, const int* ranges, int n, int* lo, int* hi) {
  // masked cells of an r line in band 1: columns of classes 1..3, i.e. from
  // the end of column class 0; of a z line of class >= 1: rows of band 1
  *lo = *hi = n;
  if (dir == 0 && cls == 1) {
    const int i0 = ranges[(1 * MAX_CLS + 0) * 2 + 1];
    if (i0 < n) { *lo = i0; *hi = n; }
  } else if (dir == 1 && cls >= 1) {
    const int a = ranges[(0 * MAX_CLS + 1) * 2], b = ranges[(0 * MAX_CLS + 1) * 2 + 1];
    if (b > a) { *lo = a; *hi = b; }
  }
}

// Strip-layout batch kernel: one wave per block of 4 lines.  r lines: 64
// chunks of 4 cells (up to 256 cells); z lines: 64 chunks of kBSZ_M[zss]
// cells (up to 192, 256, 320, 512 rows).
constexpr int kBSR_M = 4;
constexpr int kBSZ_M[4] = {3, 4, 5, 8};
constexpr int kBS_G = 64;

__host__ __device__ inline int batch_strip_zshape(int nz) {
  for (int s = 0; s < 4; ++s)
    if (kBS_G * kBSZ_M[s] >= nz) return s;
  return -1;
}

// Doubles of one right-hand side of an nr x nz instance in the strip layout.
__host__ __device__ inline long batch_strip_doubles(int nr, int nz) {
  return (long)((nr + 3) / 4) * 16L * ((nz + 3) / 4);
}

// The persistent batch kernel on the strip-layout line solver.  Each
// workgroup pops the next instance from the queue, builds its geometry and
// line-class tables in its scratch, writes the first right-hand side (strip
// layout, exact zeros outside the domain) and runs the time loop: every wave
// takes whole blocks of 4 lines (r row groups, then z strips) and solves
// them alone (DPP scans inside the wave, no workgroup barrier inside a
// sweep); the workgroup synchronises between sweeps.
template <int NW>
__global__ void __launch_bounds__(64 * NW) k_batch_s(BatchArgs a) {
  __shared__ __align__(16) double lbuf[NW][64 * 4 * 8];  // per wave: a z strip or 64 r tiles
  __shared__ double lcarry[NW][strip_carry(1)];          // unused: one wave per line
  __shared__ LineTab s_tabs[2][MAX_CLS];
  __shared__ StripArgs s_args[2];  // r sweep, z sweep
  __shared__ int s_next;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* ws = a.scratch + (long)blockIdx.x * a.lay.stride;
  const BatchLayout& Ly = a.lay;
  double* dA = (double*)(ws + Ly.dA);
  double* dB = (double*)(ws + Ly.dB);
  int* ranges = (int*)(ws + Ly.ranges);
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(a.queue, 1);
    __syncthreads();
    const int q = s_next;
    __syncthreads();
    if (q >= a.ninst) break;  // every wave of the workgroup leaves together
    const int idx = a.order[q];
    const BatchInst I = a.inst[idx];
    const Params& P = I.P;
    const int nr = P.nr, nz = P.nz;
    const int Mz = kBSZ_M[I.zss];

    Geom g;
    double* gd = (double*)(ws + Ly.geo);
    g.rf = gd; g.rc = gd + (kMaxNr + 1); g.dr = gd + 2 * (kMaxNr + 1);
    g.zf = gd + 3 * (kMaxNr + 1); g.zc = g.zf + (kMaxNz + 1); g.dz = g.zf + 2 * (kMaxNz + 1);
    g.kap = (uint8_t*)(ws + Ly.kap);
    g.bet = (uint8_t*)(ws + Ly.bet);
    build_geometry(P, nullptr, nullptr, g, ranges);

    double* rpos = (double*)(ws + Ly.rpos);
    double* rchk = (double*)(ws + Ly.rchk);
    double* reng = (double*)(ws + Ly.reng);
    double* rxc = (double*)(ws + Ly.rxc);
    double* zpos = (double*)(ws + Ly.zpos);
    double* zchk = (double*)(ws + Ly.zchk);
    double* zeng = (double*)(ws + Ly.zeng);
    double* zxc = (double*)(ws + Ly.zxc);
    double* work = (double*)(ws + Ly.work);
    const long rGM = (long)kBS_G * kBSR_M, zGM = (long)kBS_G * Mz;
    for (int c = 0; c < 3; ++c)
      assemble_class(P, g, 0, c, kBS_G, kBSR_M, rpos + c * P_NFIELDS * rGM, rchk + c * C_NFIELDS * kBS_G,
                     reng + c * 2 * nr, rxc + c * nr, work);
    for (int c = 0; c < 4; ++c)
      assemble_class(P, g, 1, c, kBS_G, Mz, zpos + c * P_NFIELDS * zGM, zchk + c * C_NFIELDS * kBS_G,
                     zeng + c * 2 * nz, zxc + c * nz, work);
    if (threadIdx.x == 0) {
      for (int c = 0; c < MAX_CLS; ++c) {
        LineTab t;
        const int cr = c < 3 ? c : 0;
        t.pos = rpos + cr * P_NFIELDS * rGM;
        t.chk = rchk + cr * C_NFIELDS * kBS_G;
        t.n = nr; t.G = kBS_G; t.M = kBSR_M;
        skip_range(0, cr, ranges, nr, &t.skip_lo, &t.skip_hi);
        s_tabs[0][c] = t;
        t.pos = zpos + c * P_NFIELDS * zGM;
        t.chk = zchk + c * C_NFIELDS * kBS_G;
        t.n = nz; t.G = kBS_G; t.M = Mz;
        skip_range(1, c, ranges, nz, &t.skip_lo, &t.skip_hi);
        s_tabs[1][c] = t;
      }
    }
    __syncthreads();

    // sweep arguments, in LDS (uniform across the workgroup; read on use)
    if (threadIdx.x == 0) {
      bool ambient = false;
      for (int c = 0; c < 4; ++c) ambient = ambient || P.tinf[c] != 0.0;
      StripArgs& ar = s_args[0];
      StripArgs& az = s_args[1];
      ar.strip = az.strip = 16L * ((nz + 3) / 4);
      ar.nr = az.nr = nr;
      ar.nz = az.nz = nz;
      for (int c = 0; c < MAX_CLS; ++c) {
        ar.tabs[c] = s_tabs[0][c];
        az.tabs[c] = s_tabs[1][c];
      }
      ar.xc = ambient ? zxc : nullptr;  // the r sweep adds b_z, the z sweep b_r
      az.xc = ambient ? rxc : nullptr;
      ar.nlines = nz;
      az.nlines = nr;
      strip_class_ends(ranges, 0, 3, ar.line_end);
      strip_class_ends(ranges, 1, 4, ar.pos_end);
      ar.nxcls = 4;
      strip_class_ends(ranges, 1, 4, az.line_end);
      strip_class_ends(ranges, 0, 3, az.pos_end);
      az.nxcls = 3;
      ar.nblocks = az.nblocks = 0;
      ar.nmix = az.nmix = 0;
      ar.theta = az.theta = P.theta;
      ar.din = dA; ar.dout = dB; ar.xout = nullptr;
      az.din = dB; az.dout = dA; az.xout = nullptr;
    }
    const long sstrip = 16L * ((nz + 3) / 4);

    // right-hand side of the first r half step from the uniform field T0
    const long nbuf = batch_strip_doubles(nr, nz);
    for (long e = threadIdx.x; e < nbuf; e += blockDim.x) {
      const long s = e / sstrip, rem = e - s * sstrip;
      const int j = (int)(rem >> 2), i = (int)(4 * s + (rem & 3));
      double o = 0.0;
      if (i < nr && j < nz) {
        const int kap = g.kap[i], bet = g.bet[j];
        if (region_of(bet, kap) != MASKED) {
          const double* pz = zpos + kap * P_NFIELDS * zGM;
          const long ix = (long)(j % Mz) * kBS_G + j / Mz;
          o = (pz[P_OD * zGM + ix] + pz[P_OL * zGM + ix] * (j > 0) + pz[P_OU * zGM + ix] * (j < nz - 1)) * I.T0 +
              pz[P_OC * zGM + ix] + rxc[bet * nr + i];
        }
      }
      dA[e] = o;
    }
    __syncthreads();

    double* Ti = a.T + I.toff;
    const int nrg = (nz + 3) / 4, nstrips = (nr + 3) / 4;
    int snap = 0;
    for (int st = 1; st <= a.nsteps; ++st) {
      const bool take = a.snap_every > 0 && st % a.snap_every == 0 && snap < a.nsnap;
      for (int J = wave; J < nrg; J += NW) strip_r_body<1>(s_args[0], J, lane, lbuf[wave], lcarry[wave]);
      if (threadIdx.x == 0) s_args[1].xout = (take || st == a.nsteps) ? Ti : nullptr;
      __syncthreads();
      for (int s = wave; s < nstrips; s += NW) {
        switch (I.zss) {
          case 0: strip_z_body<kBSZ_M[0], 1>(s_args[1], s, lane, lbuf[wave], lcarry[wave]); break;
          case 1: strip_z_body<kBSZ_M[1], 1>(s_args[1], s, lane, lbuf[wave], lcarry[wave]); break;
          case 2: strip_z_body<kBSZ_M[2], 1>(s_args[1], s, lane, lbuf[wave], lcarry[wave]); break;
          default: strip_z_body<kBSZ_M[3], 1>(s_args[1], s, lane, lbuf[wave], lcarry[wave]); break;
        }
      }
      __syncthreads();
      if (take) {
        // outer terminal-face profile from the top row
        const double* row = Ti + (long)(nz - 1) * nr;
        for (int kk = threadIdx.x; kk < a.npts; kk += blockDim.x) {
          const double r = (kk + 0.5) * P.rmax / a.npts;
          double o;
          if (r <= g.rc[0]) o = row[0];
          else if (r >= g.rc[nr - 1]) o = row[nr - 1];
          else {
            int lo = 0, hi = nr - 1;
            while (hi - lo > 1) {
              const int mid = (lo + hi) >> 1;
              if (g.rc[mid] <= r) lo = mid; else hi = mid;
            }
            o = row[lo] + (row[lo + 1] - row[lo]) * (r - g.rc[lo]) / (g.rc[lo + 1] - g.rc[lo]);
          }
          a.prof[((long)idx * a.nsnap + snap) * a.npts + kk] = o;
        }
        ++snap;
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

}  // namespace adi
